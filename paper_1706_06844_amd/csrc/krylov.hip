// Flexible GMRES building blocks (the Krylov solver of paper Sec. 4.3 and Sec. 5): fused
// Gram-Schmidt passes with deterministic FP64 reductions, the Givens update of the Hessenberg
// least-squares problem, and the solution update x += Z y.
//
// The basis V is stored unnormalised: column k holds a multiple of v_k and vscale[k] turns it into
// v_k.  This saves the separate normalisation pass; every consumer applies the scale.
//
// Orthogonalisation is classical Gram-Schmidt with a second pass only when the first one removed
// more than the fraction 1 - keep_min of the squared norm (the criterion of Daniel, Gragg, Kaufman
// and Stewart, 1976, who take 1/2).  keep_min is set per basis storage: 1e-6 for an FP64 basis (a
// single pass then loses at most about 1e3 rounding units of orthogonality); 1/10 for FP32 restart
// cycles (FP32 or BF16 basis), whose stored columns are orthonormal only to their storage rounding,
// so that the second pass pays off only when the first cancels most of w.  A direction whose norm after orthogonalisation falls below brk_tol times the
// projected column is a breakdown (the Krylov space is invariant to the basis' precision): 1e-14
// for FP64 storage, 1e-6 for FP32 and 4e-3 for BF16, a few units of the storage rounding.
//
// Reductions: every thread accumulates a fixed strided subset, a fixed tree combines the block's
// values, each block writes its partials, and a one-workgroup kernel combines the partials in block
// order.  The result does not depend on scheduling, so runs are bitwise
// reproducible for a given launch shape.
#include "common.h"
#include "fft.h"  // static_for

namespace fde {

constexpr int kCgsBlock = 256;
constexpr int kCgsWaves = kCgsBlock / 64;
constexpr int kCgsMaxGrid = 512;
constexpr int kFinBlock = 1024;  // finalize: one workgroup
constexpr int kFinLds = 6144;    // doubles of partials staged at a time (48 KB; >= one row of kCgsMaxGrid)

int cgs_grid(size_t N) {
  const size_t pairs = (N + 1) / 2;
  size_t g = (pairs + (size_t)kCgsBlock * 4 - 1) / ((size_t)kCgsBlock * 4);
  if (g < 1) g = 1;
  if (g > kCgsMaxGrid) g = kCgsMaxGrid;
  return (int)g;
}
size_t cgs_partials_len(size_t) { return (size_t)(kMaxRestart + 2) * kCgsMaxGrid; }
size_t basis_ld(size_t N) { return (N + 63) / 64 * 64; }

// Sum over the wavefront in a fixed order; the result is valid in lane 0.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Givens update after column j of the Hessenberg matrix is known (single thread).
__device__ void givens_step(GmresState* st, int j, double nrm) {
  constexpr int K = kMaxRestart;
  double col[kMaxRestart + 1];
  for (int i = 0; i <= j; ++i) col[i] = st->h1[i] + (st->reorth ? st->h2[i] : 0.0);
  col[j + 1] = nrm;
  for (int i = 0; i < j; ++i) {
    const double c = st->cs[i], s = st->sn[i];
    const double a = c * col[i] + s * col[i + 1];
    col[i + 1] = -s * col[i] + c * col[i + 1];
    col[i] = a;
  }
  const double r = hypot(col[j], col[j + 1]);
  double c = 1.0, s = 0.0;
  if (r > 0.0) {
    c = col[j] / r;
    s = col[j + 1] / r;
  }
  st->cs[j] = c;
  st->sn[j] = s;
  col[j] = r;
  st->g[j + 1] = -s * st->g[j];
  st->g[j] = c * st->g[j];
  for (int i = 0; i <= j; ++i) st->Rm[j * K + i] = col[i];
  const double est = fabs(st->g[j + 1]);
  st->est = est;
  st->iters += 1;
  st->nused = j + 1;
  st->nreorth += st->reorth;
  if (st->reorth) st->reorth_mask |= 1u << j;
  st->vscale[j + 1] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  // breakdown: the new direction vanished relative to the column (the Krylov space is invariant)
  const bool breakdown = !(nrm > st->brk_tol * r);
  if (est <= st->atol || st->iters >= st->maxit || breakdown || j + 1 >= st->restart) st->done = 1;
}

constexpr int kFusedMaxGrid = 32;  // passes with at most this many workgroups finalise themselves

// LDS of the combination of a pass's partials: the solver state, the combined rows, and a staging
// buffer of PL partials.
template <int PL>
struct FinLds {
  GmresState ls;
  double fin[kMaxRestart + 2];
  double pl[PL];
};

template <int PL>
__device__ void finalize_block(int kind, int nv, int G, const double* partials, GmresState* gst, FinLds<PL>& F);

// Runs of VEC consecutive entries per thread: 16-byte loads of the basis columns (FP64: 2 entries,
// FP32: 4, BF16: 8) and the matching entries of the work vector w (FP64 or FP32).  Basis entries
// are used as `reg` (FP64, or FP32 for FP32 and BF16 storage).
template <typename TB>
struct BasisT {
  using reg = TB;
};
template <>
struct BasisT<bf16_t> {
  using reg = float;
};

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T* p, typename BasisT<T>::reg (&v)[VEC]) {
  if constexpr (std::is_same<T, double>::value) {
    static_assert(VEC == 2, "FP64 runs are 2 entries");
    const double2 a = *reinterpret_cast<const double2*>(p);
    v[0] = a.x;
    v[1] = a.y;
  } else if constexpr (std::is_same<T, float>::value) {
    static_assert(VEC == 4 || VEC == 8, "FP32 runs are 4 or 8 entries");
#pragma unroll
    for (int q = 0; q < VEC / 4; ++q) {
      const float4 a = *reinterpret_cast<const float4*>(p + 4 * q);
      v[4 * q] = a.x;
      v[4 * q + 1] = a.y;
      v[4 * q + 2] = a.z;
      v[4 * q + 3] = a.w;
    }
  } else {
    static_assert(std::is_same<T, double>::value || std::is_same<T, float>::value, "FP64 or FP32 runs");
  }
}
// A run of basis entries as loaded (16 bytes: 2 FP64, 4 FP32 or 8 BF16 entries), unpacked entry by
// entry where it is used, so that the loads of all columns are issued before any result is needed.
template <typename TB>
struct RawT;
template <>
struct RawT<double> {
  using type = double2;
};
template <>
struct RawT<float> {
  using type = float4;
};
template <>
struct RawT<bf16_t> {
  using type = uint4;  // 8 entries
};
template <typename TB>
__device__ __forceinline__ typename RawT<TB>::type load_raw(const TB* p) {
  return *reinterpret_cast<const typename RawT<TB>::type*>(p);
}
template <typename TB>
__device__ __forceinline__ typename RawT<TB>::type zero_raw() {
  return typename RawT<TB>::type{};
}
template <typename TB, int E>
__device__ __forceinline__ typename BasisT<TB>::reg raw_elem(const typename RawT<TB>::type& r) {
  if constexpr (std::is_same<TB, double>::value) return E == 0 ? r.x : r.y;
  else if constexpr (std::is_same<TB, float>::value) return E == 0 ? r.x : E == 1 ? r.y : E == 2 ? r.z : r.w;
  else {
    const unsigned u = E < 2 ? r.x : E < 4 ? r.y : E < 6 ? r.z : r.w;
    return __uint_as_float((E & 1) ? (u & 0xffff0000u) : (u << 16));
  }
}
// zero the entries of a run at positions >= nin (the padding past N)
template <typename TB>
__device__ __forceinline__ void raw_mask(typename RawT<TB>::type& r, int nin) {
  if constexpr (std::is_same<TB, double>::value) {
    if (nin < 2) r.y = 0.0;
  } else if constexpr (std::is_same<TB, float>::value) {
    if (nin < 2) r.y = 0.f;
    if (nin < 3) r.z = 0.f;
    if (nin < 4) r.w = 0.f;
  } else {
    unsigned* u = &r.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (nin <= 2 * q) u[q] = 0u;
      else if (nin == 2 * q + 1) u[q] &= 0xffffu;
    }
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec(T* p, const T (&v)[VEC]) {
  if constexpr (std::is_same<T, double>::value) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  } else {
#pragma unroll
    for (int q = 0; q < VEC / 4; ++q)
      *reinterpret_cast<float4*>(p + 4 * q) = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  }
}
// FP32 to BF16, rounded to nearest even (NaN and infinity stay what they are).
__device__ __forceinline__ unsigned bf16_bits(float f) {
  const unsigned u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ void store_bf16x8(bf16_t* p, const float (&v)[8]) {
  *reinterpret_cast<uint4*>(p) =
      make_uint4(bf16_bits(v[0]) | (bf16_bits(v[1]) << 16), bf16_bits(v[2]) | (bf16_bits(v[3]) << 16),
                 bf16_bits(v[4]) | (bf16_bits(v[5]) << 16), bf16_bits(v[6]) | (bf16_bits(v[7]) << 16));
}

// One pass over the basis (products, sums and coefficients in FP64).  TW is the storage of the work
// vector w (FP64 or FP32), TB that of the basis: the same type, w then being a basis column, or BF16
// with an FP32 w, the final pass then also writing the BF16 rounding of w into the basis column
// `vout` (INIT and RESNORM too).  Each thread handles runs of VEC consecutive entries; the basis
// columns and w are padded to a multiple of VEC, so the last run is readable and its entries past N
// are masked to zero (and written back as zero).  `src` (FP64) is copied into w by INIT, and by
// RESNORM when given: the norm is then taken of the FP64 values.  FUSED: the last workgroup to
// finish (counted on the state's ticket) combines the partials itself, which saves small problems a
// launch per pass.
template <typename TB, typename TW, int MAXV, bool FUSED>
__global__ __launch_bounds__(kCgsBlock) void cgs_kernel(int kind, int N, int nv, const TB* __restrict__ V,
                                                        size_t ldv, TW* __restrict__ w, TB* __restrict__ vout,
                                                        const double* __restrict__ src, GmresState* st,
                                                        double* __restrict__ partials, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(V);
  FDE_ZSHIFT(w);
  FDE_ZSHIFT(vout);
  FDE_ZSHIFT(src);
  FDE_ZSHIFT(st);
  FDE_ZSHIFT(partials);
  if (st->idle) return;
  constexpr bool kSplit = std::is_same<TB, bf16_t>::value;
  constexpr int VEC = kSplit ? 8 : 16 / (int)sizeof(TW);  // 16-byte loads of the basis
  using RB = typename BasisT<TB>::reg;
  if (kind == CGS_DOTS || kind == CGS_UPDATE_DOTS || kind == CGS_UPDATE_NORM) {
    if (st->done) return;
    if (kind == CGS_UPDATE_DOTS && !st->reorth) return;
  }
  __shared__ double hc[MAXV];
  __shared__ double red[kCgsWaves][MAXV + 1];
  // coefficients of the unnormalised columns for the update passes
  if (threadIdx.x < MAXV) {
    double c = 0.0;
    if ((int)threadIdx.x < nv) {
      if (kind == CGS_UPDATE_DOTS) c = st->h1[threadIdx.x] * st->vscale[threadIdx.x];
      if (kind == CGS_UPDATE_NORM) c = (st->reorth ? st->h2[threadIdx.x] : st->h1[threadIdx.x]) * st->vscale[threadIdx.x];
    }
    hc[threadIdx.x] = c;
  }
  __syncthreads();
  const bool dots = (kind == CGS_DOTS || kind == CGS_UPDATE_DOTS);
  const bool upd = (kind == CGS_UPDATE_DOTS || kind == CGS_UPDATE_NORM);
  const bool norm = (kind != CGS_UPDATE_DOTS);
  const bool copy = (kind == CGS_INIT) || (kind == CGS_RESNORM && src);
  double acc[MAXV];
#pragma unroll
  for (int k = 0; k < MAXV; ++k) acc[k] = 0.0;
  double nacc = 0.0;
  const int P = (N + VEC - 1) / VEC;
  const int stride = gridDim.x * kCgsBlock;
  for (int i = blockIdx.x * kCgsBlock + threadIdx.x; i < P; i += stride) {
    const int p = VEC * i;
    const int nin = min(VEC, N - p);
    TW wv[VEC];
    if (copy) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const double b = e < nin ? src[p + e] : 0.0;
        wv[e] = (TW)b;
        nacc += b * b;
      }
      store_vec(w + p, wv);
      if constexpr (kSplit) store_bf16x8(vout + p, wv);
      continue;
    }
    load_vec<TW, VEC>(w + p, wv);
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      if (e >= nin) wv[e] = TW(0);
    if (kind == CGS_RESNORM) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) nacc += (double)wv[e] * (double)wv[e];
      continue;
    }
    // basis entries: FP64 and FP32 runs unpacked at load; BF16 runs kept packed until used (with
    // the unpacking next to the loads the compiler waits for each load before issuing the next)
    RB vu[kSplit ? 1 : MAXV][VEC];
    typename RawT<TB>::type vk[kSplit ? MAXV : 1];
    if constexpr (kSplit) {
#pragma unroll
      for (int k = 0; k < MAXV; ++k) vk[k] = (k < nv) ? load_raw(V + (size_t)k * ldv + p) : zero_raw<TB>();
      if (nin < VEC) {
#pragma unroll
        for (int k = 0; k < MAXV; ++k) raw_mask<TB>(vk[k], nin);
      }
    } else {
#pragma unroll
      for (int k = 0; k < MAXV; ++k) {
        if (k < nv) {
          load_vec<TB, VEC>(V + (size_t)k * ldv + p, vu[k]);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) vu[k][e] = RB(0);
        }
      }
      if (nin < VEC) {
#pragma unroll
        for (int k = 0; k < MAXV; ++k)
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            if (e >= nin) vu[k][e] = RB(0);
      }
    }
    auto basis = [&](int k, auto ec) -> RB {
      constexpr int e = decltype(ec)::value;
      if constexpr (kSplit) return raw_elem<TB, e>(vk[k]);
      else return vu[k][e];
    };
    if (upd) {
      double wd[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) wd[e] = wv[e];
#pragma unroll
      for (int k = 0; k < MAXV; ++k)
        if (k < nv) {
          static_for<0, VEC>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            wd[e] -= hc[k] * (double)basis(k, ec);
          });
        }
#pragma unroll
      for (int e = 0; e < VEC; ++e) wv[e] = (TW)wd[e];
      store_vec(w + p, wv);
      if constexpr (kSplit) {
        if (kind == CGS_UPDATE_NORM) store_bf16x8(vout + p, wv);
      }
    }
    if (dots) {
#pragma unroll
      for (int k = 0; k < MAXV; ++k)
        if (k < nv) {
          static_for<0, VEC>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            acc[k] += (double)basis(k, ec) * (double)wv[e];
          });
        }
    }
    if (norm) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) nacc += (double)wv[e] * (double)wv[e];
    }
  }
  // rows of this pass: the nv dot products (DOTS, UPDATE_DOTS), then the squared norm (DOTS,
  // UPDATE_NORM, INIT, RESNORM)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nd = dots ? nv : 0;
  const int nres = nd + (norm ? 1 : 0);
  if (dots) {
#pragma unroll
    for (int k = 0; k < MAXV; ++k)
      if (k < nv) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[wid][k] = s;
      }
  }
  if (norm) {
    const double s = wave_sum(nacc);
    if (lane == 0) red[wid][nd] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < nres) {
    double s = 0.0;
    for (int q = 0; q < kCgsWaves; ++q) s += red[q][threadIdx.x];
    partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
  if constexpr (FUSED) {
    __shared__ int last;
    __threadfence();  // this workgroup's partials are visible before its ticket
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&st->ticket, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();  // and the other workgroups' partials are seen after it
    if (threadIdx.x == 0) atomicExch(&st->ticket, 0u);
    __shared__ FinLds<kFusedMaxGrid * (kMaxRestart + 2)> F;
    finalize_block(kind, nv, (int)gridDim.x, partials, st, F);
  }
}

// Combination of a pass's partials and the state update, run by one whole workgroup.  The state is
// copied into LDS by the workgroup (one round of independent loads), updated there by one thread,
// and copied back: the update's many small dependent accesses then stay on chip instead of paying a
// device-memory round trip each.  `partials` is read through volatile loads (the fused path reads
// what other workgroups of the same launch wrote).
template <int PL>
__device__ void finalize_block(int kind, int nv, int G, const double* partials, GmresState* gst, FinLds<PL>& F) {
  constexpr int kWords = sizeof(GmresState) / 4;
  static_assert(sizeof(GmresState) % 4 == 0, "state is copied as 32-bit words");
  GmresState& ls = F.ls;
  double* fin = F.fin;
  double* pl = F.pl;
  const volatile double* vp = partials;
  {
    const unsigned* src = reinterpret_cast<const unsigned*>(gst);
    unsigned* dst = reinterpret_cast<unsigned*>(&ls);
    for (int k = threadIdx.x; k < kWords; k += blockDim.x) dst[k] = src[k];
  }
  __syncthreads();
  // nothing to combine for an idle slot of a batched group, after convergence, or for a second pass
  // that was not taken (decided from the state before any partial is read)
  if (ls.idle) return;
  if (kind == CGS_DOTS || kind == CGS_UPDATE_DOTS || kind == CGS_UPDATE_NORM) {
    if (ls.done) return;
    if (kind == CGS_UPDATE_DOTS && !ls.reorth) return;
  }
  if (threadIdx.x == 0) ls.ticket = 0;
  const bool dots = (kind == CGS_DOTS || kind == CGS_UPDATE_DOTS);
  const bool norm = (kind != CGS_UPDATE_DOTS);
  const int nres = (dots ? nv : 0) + (norm ? 1 : 0);
  // the partials are fetched in rounds of independent loads (as many rows as fit the LDS buffer,
  // usually all of them), then summed from LDS in block order
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int rows = PL / G;
  for (int r0 = 0; r0 < nres; r0 += rows) {
    const int nr = min(rows, nres - r0);
    for (int e = threadIdx.x; e < nr * G; e += blockDim.x) pl[e] = vp[(size_t)r0 * G + e];
    __syncthreads();
    for (int r = wid; r < nr; r += nw) {
      double v = 0.0;
      for (int b = lane; b < G; b += 64) v += pl[r * G + b];
      v = wave_sum(v);
      if (lane == 0) fin[r0 + r] = v;
    }
    __syncthreads();
  }
  GmresState* st = &ls;
  if (threadIdx.x == 0) {
    if (kind == CGS_DOTS) {
      double hh = 0.0;
      for (int k = 0; k < nv; ++k) {
        const double h = fin[k] * st->vscale[k];
        st->h1[k] = h;
        hh += h * h;
      }
      // After one projection ||w - V h||^2 = ||w||^2 - ||h||^2 (orthonormal V).  A second pass is
      // needed when the projection removed more than the fraction 1 - keep_min of ||w||^2 (the
      // classical criterion takes keep_min = 1/2, a norm ratio below 1/sqrt 2).
      const double ww = fin[nv];
      st->reorth = st->orth == 1 ? 1 : st->orth == 0 ? 0 : (ww - hh < st->keep_min * ww ? 1 : 0);
    } else if (kind == CGS_UPDATE_DOTS) {
      for (int k = 0; k < nv; ++k) st->h2[k] = fin[k] * st->vscale[k];
    } else if (kind == CGS_UPDATE_NORM) {
      givens_step(st, nv - 1, sqrt(fin[0]));
    } else if (kind == CGS_INIT) {
      const double bn = sqrt(fin[0]);
      st->bnorm = bn;
      st->atol = st->rtol * bn;
      st->resnorm = bn;
      st->est = bn;
      st->g[0] = bn;
      st->vscale[0] = bn > 0.0 ? 1.0 / bn : 0.0;
      st->iters = 0;
      st->nreorth = 0;
      st->reorth_mask = 0;
      st->nused = 0;
      st->conv = (bn == 0.0);
      st->done = (bn == 0.0);
    } else if (kind == CGS_RESNORM) {
      const double rn = sqrt(fin[0]);
      st->resnorm = rn;
      st->conv = (rn <= st->atol);
      st->g[0] = rn;
      st->vscale[0] = rn > 0.0 ? 1.0 / rn : 0.0;
      st->nused = 0;
      st->reorth_mask = 0;
      st->done = (st->conv || st->iters >= st->maxit) ? 1 : 0;
    }
  }
  __syncthreads();
  {
    const unsigned* src = reinterpret_cast<const unsigned*>(&ls);
    unsigned* dst = reinterpret_cast<unsigned*>(gst);
    for (int k = threadIdx.x; k < kWords; k += blockDim.x) dst[k] = src[k];
  }
}

// Combines the G per-block partials of a pass in block order and updates the solver state: a
// launch of its own for wide passes, where one counter hit by every workgroup of the grid (the
// last-workgroup ticket of the fused form) would serialise at the memory side.
__global__ __launch_bounds__(kFinBlock) void cgs_finalize_kernel(int kind, int nv, int G,
                                                                 const double* __restrict__ partials,
                                                                 GmresState* gst, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(partials);
  FDE_ZSHIFT(gst);
  __shared__ FinLds<kFinLds> F;
  finalize_block(kind, nv, G, partials, gst, F);
}

// Grid of a pass: wide passes (many columns) stream best with one workgroup per CU, narrow ones with
// two; `cap` is the size-dependent maximum (cgs_grid).
int cgs_pass_grid(int nv, int cap) {
  int g = cap < 1 ? 1 : (cap > kCgsMaxGrid ? kCgsMaxGrid : cap);
  if (nv > 8 && g > kCgsMaxGrid / 2) g = kCgsMaxGrid / 2;
  return g;
}

template <typename TB, typename TW>
hipError_t launch_cgs_pass(int kind, size_t N, int nv, TB* V, size_t ldv, TW* w, TB* vout, const double* src,
                           GmresState* st, double* partials, int cap, hipStream_t s) {
  constexpr bool split = std::is_same<TB, bf16_t>::value;
  constexpr int VEC = split ? 8 : 16 / (int)sizeof(TW);
  if (nv > kMaxRestart + 1 || N > (size_t)0x7ffffffe || cap < 1) return hipErrorInvalidValue;
  if (ldv % VEC || (reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(w)) % 16) return hipErrorInvalidValue;
  if (kind == CGS_INIT && !src) return hipErrorInvalidValue;
  // the BF16 column is written by the passes that finish a vector
  const bool writes = kind == CGS_UPDATE_NORM || kind == CGS_INIT || (kind == CGS_RESNORM && src);
  if (split && writes && (!vout || reinterpret_cast<uintptr_t>(vout) % 16)) return hipErrorInvalidValue;
  const int n = (int)N;
  const int grid = cgs_pass_grid(nv, cap);
  const bool fused = grid <= kFusedMaxGrid;
#define L_(M)                                                                                              \
  if (fused)                                                                                               \
    hipLaunchKernelGGL((cgs_kernel<TB, TW, M, true>), dim3(grid, 1, batch_nz()), dim3(kCgsBlock), 0, s, kind, n, nv, \
                       V, ldv, w, vout, src, st, partials, batch_ztab());                                   \
  else                                                                                                     \
    hipLaunchKernelGGL((cgs_kernel<TB, TW, M, false>), dim3(grid, 1, batch_nz()), dim3(kCgsBlock), 0, s, kind, n, nv, \
                       V, ldv, w, vout, src, st, partials, batch_ztab())
  if (nv <= 4) { L_(4); }
  else if (nv <= 8) { L_(8); }
  else if (nv <= 12) { L_(12); }
  else if (nv <= 16) { L_(16); }
  else if (nv <= 24) { L_(24); }
  else { L_(kMaxRestart + 1); }
#undef L_
  return hipGetLastError();
}
template hipError_t launch_cgs_pass<double, double>(int, size_t, int, double*, size_t, double*, double*,
                                                    const double*, GmresState*, double*, int, hipStream_t);
template hipError_t launch_cgs_pass<float, float>(int, size_t, int, float*, size_t, float*, float*, const double*,
                                                  GmresState*, double*, int, hipStream_t);
template hipError_t launch_cgs_pass<bf16_t, float>(int, size_t, int, bf16_t*, size_t, float*, bf16_t*,
                                                   const double*, GmresState*, double*, int, hipStream_t);

bool cgs_fused(int nv, int cap) { return cgs_pass_grid(nv, cap) <= kFusedMaxGrid; }

hipError_t launch_cgs_finalize(int kind, int nv, double* partials, GmresState* st, int cap, hipStream_t s) {
  if (nv > kMaxRestart + 1 || cap < 1) return hipErrorInvalidValue;
  if (cgs_fused(nv, cap)) return hipErrorInvalidValue;  // the pass has combined its partials itself
  hipLaunchKernelGGL(cgs_finalize_kernel, dim3(1, 1, batch_nz()), dim3(kFinBlock), 0, s, kind, nv, cgs_pass_grid(nv, cap),
                     partials, st, batch_ztab());
  return hipGetLastError();
}

// x = (first ? 0 : x) + Z y, with y solving the nused x nused triangular system R y = g.
template <typename Tz>
__global__ __launch_bounds__(256) void update_x_kernel(size_t N, const Tz* __restrict__ Z, size_t ldz,
                                                       double* __restrict__ x, int first, GmresState* st,
                                                       const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(Z);
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(st);
  if (st->idle) return;
  __shared__ double y[kMaxRestart];
  __shared__ int m_s;
  if (threadIdx.x == 0) {
    const int m = st->nused;
    for (int i = m - 1; i >= 0; --i) {
      double v = st->g[i];
      for (int k = i + 1; k < m; ++k) v -= st->Rm[k * kMaxRestart + i] * y[k];
      const double d = st->Rm[i * kMaxRestart + i];
      y[i] = d != 0.0 ? v / d : 0.0;
    }
    m_s = m;
    if (blockIdx.x == 0)
      for (int i = 0; i < m; ++i) st->y[i] = y[i];
  }
  __syncthreads();
  const int m = m_s;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += stride) {
    double a = first ? 0.0 : x[p];
    for (int i = 0; i < m; ++i) a += y[i] * (double)Z[(size_t)i * ldz + p];
    x[p] = a;
  }
}

template <typename Tz>
hipError_t launch_update_x(size_t N, const Tz* Z, size_t ldz, double* x, int first, GmresState* st,
                           hipStream_t s) {
  size_t g = (N + 256 * 4 - 1) / (256 * 4);
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  hipLaunchKernelGGL((update_x_kernel<Tz>), dim3((int)g, 1, batch_nz()), dim3(256), 0, s, N, Z, ldz, x, first, st,
                     batch_ztab());
  return hipGetLastError();
}
template hipError_t launch_update_x<double>(size_t, const double*, size_t, double*, int, GmresState*,
                                            hipStream_t);
template hipError_t launch_update_x<float>(size_t, const float*, size_t, double*, int, GmresState*,
                                           hipStream_t);

}  // namespace fde
