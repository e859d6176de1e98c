// Multigrid kernels (paper Sec. 4): damped-Jacobi smoothing, full-weighting restriction, bilinear
// prolongation, coarse-level construction, and a single-workgroup V-cycle for the small levels.
//
// Grid transfer: P = T(p) U with p = (1 + cos t1)(1 + cos t2) (Sec. 4.1, Lemma lemapp): coarse point
// J (0-based) sits on fine point 2J+1, and P spreads it with weights 1, 1/2, 1/4 (bilinear
// interpolation).  Restriction is R = P^T / 4, the 9-point full-weighting stencil
// [1 2 1; 2 4 2; 1 2 1] / 16.  Coarse geometric levels rediscretise the operator with h doubled and
// the coefficient fields injected at the coarse points (Sec. 4.2).
#include "common.h"
#include "fft.h"  // static_for

namespace fde {

constexpr int kBlock = 256;

// p[i] where ok, else 0, with the load itself unconditional (index 0, which must be valid, where
// !ok).  A load under a per-lane branch whose other side writes 0 into the same register is waited
// for where the branches join, so a run of such loads would be issued one at a time.
template <typename T, typename I>
__device__ __forceinline__ T load_or_zero(const T* __restrict__ p, I i, bool ok) {
  const T v = p[ok ? i : I(0)];
  return ok ? v : T(0);
}

static inline int grid_for(size_t n, int per_block = kBlock) {
  size_t g = (n + per_block - 1) / per_block;
  if (g > 65535 * 16) g = 65535 * 16;
  return (int)(g == 0 ? 1 : g);
}

// ---- pre-smoothing from a zero initial guess: x = dinv .* b (one Jacobi step with x0 = 0) ------
template <typename R, typename Tin>
__global__ void presmooth_kernel(int N, const Tin* __restrict__ b, const double* __restrict__ bscale,
                                 const R* __restrict__ dinv, R* __restrict__ x, R* __restrict__ bcopy,
                                 const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(b);
  FDE_ZSHIFT(bscale);
  FDE_ZSHIFT(dinv);
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(bcopy);
  FDE_ZSHIFT(skip);
  if (load_flag(skip)) return;
  const double s = bscale ? *bscale : 1.0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
    const R bv = (R)(s * (double)b[p]);
    if (bcopy) bcopy[p] = bv;
    x[p] = dinv[p] * bv;
  }
}

// Runs of 4 entries per thread with 16-byte accesses (an FP64 run takes two), all arrays 16-byte
// aligned; the tail of N mod 4 elementwise.  Same arithmetic as presmooth_kernel.
template <typename T>
__device__ __forceinline__ void load4(const T* p, T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 c = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = c.x;
    v[3] = c.y;
  }
}
template <typename T>
__device__ __forceinline__ void store4(T* p, const T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
  }
}
template <typename R, typename Tin>
__global__ void presmooth4_kernel(int N, const Tin* __restrict__ b, const double* __restrict__ bscale,
                                  const R* __restrict__ dinv, R* __restrict__ x, R* __restrict__ bcopy,
                                  const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(b);
  FDE_ZSHIFT(bscale);
  FDE_ZSHIFT(dinv);
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(bcopy);
  FDE_ZSHIFT(skip);
  if (load_flag(skip)) return;
  const double s = bscale ? *bscale : 1.0;
  const int N4 = N >> 2;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < N4; q += gridDim.x * blockDim.x) {
    Tin bb[4];
    R d4[4], v[4], xo[4];
    load4(b + 4 * q, bb);
    load4(dinv + 4 * q, d4);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (R)(s * (double)bb[k]);
    if (bcopy) store4(bcopy + 4 * q, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) xo[k] = d4[k] * v[k];
    store4(x + 4 * q, xo);
  }
  if (blockIdx.x == 0 && (int)threadIdx.x < N - 4 * N4) {
    const int p = 4 * N4 + threadIdx.x;
    const R bv = (R)(s * (double)b[p]);
    if (bcopy) bcopy[p] = bv;
    x[p] = dinv[p] * bv;
  }
}

template <typename R, typename Tin>
hipError_t launch_presmooth(int N, const Tin* b, const double* bscale, const R* dinv, R* x, R* bcopy,
                            const int* skip, hipStream_t st) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(dinv) |
                      reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(bcopy);
  if (a % 16 == 0) {
    hipLaunchKernelGGL((presmooth4_kernel<R, Tin>), dim3(grid_for((size_t)(N + 3) / 4), 1, batch_nz()), dim3(kBlock), 0,
                       st, N, b, bscale, dinv, x, bcopy, skip, batch_ztab());
    return hipGetLastError();
  }
  hipLaunchKernelGGL((presmooth_kernel<R, Tin>), dim3(grid_for(N), 1, batch_nz()), dim3(kBlock), 0, st, N, b, bscale,
                     dinv, x, bcopy, skip, batch_ztab());
  return hipGetLastError();
}

// ---- restriction rc = P^T r / 4 ---------------------------------------------------------------
// With xc given, also the coarse level's first Jacobi sweep from zero: xc = dinv_c .* rc (the same
// product the pre-smoothing kernel forms, fused to save a launch).
// One coarse row J per blockIdx.y; coarse point (J, I) sits at fine (2J + o2, 2I + o1), o = n mod 2,
// and reads the 3 x 3 fine block around it (on an even side the block of J = 0 starts outside the
// grid, where the field is zero).

// Full weighting at fine centre (fy, fx): [1 2 1; 2 4 2; 1 2 1] / 16, entries at index -1 zero (the
// block never passes the last row or column).
template <typename R>
__device__ __forceinline__ R full_weight(const R* f, int n1, int fy, int fx) {
  auto F = [&](int y, int x) -> R { return (y >= 0 && x >= 0) ? f[(size_t)y * n1 + x] : R(0); };
  const R a0 = F(fy - 1, fx - 1) + 2 * F(fy - 1, fx) + F(fy - 1, fx + 1);
  const R a1 = F(fy, fx - 1) + 2 * F(fy, fx) + F(fy, fx + 1);
  const R a2 = F(fy + 1, fx - 1) + 2 * F(fy + 1, fx) + F(fy + 1, fx + 1);
  return (a0 + 2 * a1 + a2) * R(0.0625);
}
template <typename R>
__global__ void restrict_kernel(int n1, int n2, const R* __restrict__ r, R* __restrict__ rc,
                                const R* __restrict__ dinv_c, R* __restrict__ xc, const int* __restrict__ skip,
                                const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(r);
  FDE_ZSHIFT(rc);
  FDE_ZSHIFT(dinv_c);
  FDE_ZSHIFT(xc);
  FDE_ZSHIFT(skip);
  const int skipv = load_flag(skip);  // waited for after the loads below are issued
  const int k1 = n1 >> 1;
  const int J = blockIdx.y;
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= k1) return;
  const size_t q = (size_t)J * k1 + I;
  R v;
  if (n1 & n2 & 1) {
    // odd sides: the block lies inside the grid
    const R* r0 = r + (size_t)(2 * J) * n1 + 2 * I + 1;
    const R* r1 = r0 + n1;
    const R* r2 = r1 + n1;
    const R a0 = r0[-1] + 2 * r0[0] + r0[1];
    const R a1 = r1[-1] + 2 * r1[0] + r1[1];
    const R a2 = r2[-1] + 2 * r2[0] + r2[1];
    v = (a0 + 2 * a1 + a2) * R(0.0625);
  } else {
    v = full_weight(r, n1, 2 * J + (n2 & 1), 2 * I + (n1 & 1));
  }
  const R dc = xc ? dinv_c[q] : R(0);
  if (skipv) return;
  rc[q] = v;
  if (xc) xc[q] = dc * v;
}

template <typename R>
hipError_t launch_restrict(int n1, int n2, const R* r, R* rc, const R* dinv_c, R* xc, const int* skip,
                           hipStream_t st) {
  if (xc && !dinv_c) return hipErrorInvalidValue;
  const int k1 = n1 >> 1, k2 = n2 >> 1;
  if (k1 < 1 || k2 < 1) return hipErrorInvalidValue;
  if (k2 > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((restrict_kernel<R>), dim3(ceil_div(k1, kBlock), k2, batch_nz()), dim3(kBlock), 0, st, n1, n2, r,
                     rc, dinv_c, xc, skip, batch_ztab());
  return hipGetLastError();
}

// ---- prolongation and correction x += P e -----------------------------------------------------
// Coarse neighbours of fine index f (0-based) on a side of n points (k = n >> 1 coarse points): with
// g = f + 1 - n mod 2 (so that coarse J sits at g = 2J + 1), odd g = 2c+1 -> (c, 1); even g = 2c ->
// (c-1, 1/2), (c, 1/2), dropping indices outside [0, k).  (Used by the one-workgroup V-cycle.)
__device__ __forceinline__ void coarse_nbrs(int f, int n, int* c, float* w, int* cnt) {
  const int k = n >> 1;
  f += 1 - (n & 1);
  if (f & 1) {
    c[0] = (f - 1) >> 1;
    w[0] = 1.0f;
    *cnt = 1;
  } else {
    int m = 0;
    const int h = f >> 1;
    if (h - 1 >= 0) {
      c[m] = h - 1;
      w[m++] = 0.5f;
    }
    if (h < k) {
      c[m] = h;
      w[m++] = 0.5f;
    }
    *cnt = m;
  }
}

// Fine index f (0-based) takes (e[(g-1)>>1] + e[g>>1]) / 2 from its coarse neighbours, g = f + 1 -
// n mod 2, entries outside [0, k) being zero: an odd g = 2c+1 gets e[c] (both indices equal), an
// even g = 2c the mean of e[c-1] and e[c].  One fine row per blockIdx.y, so the row weights are
// uniform per workgroup.
template <typename R>
__global__ void prolong_kernel(int n1, int n2, const R* __restrict__ e, R* __restrict__ x,
                               const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(e);
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(skip);
  const int skipv = load_flag(skip);  // waited for after the loads below are issued
  const int k1 = n1 >> 1, k2 = n2 >> 1;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1) return;
  const int gy = j + 1 - (n2 & 1), gx = i + 1 - (n1 & 1);
  const int ya = (gy - 1) >> 1, yb = gy >> 1;  // coarse rows (equal for odd gy)
  const int xa = (gx - 1) >> 1, xb = gx >> 1;
  auto E = [&](int cy, int cx) -> R {
    return (cy >= 0 && cy < k2 && cx >= 0 && cx < k1) ? e[(size_t)cy * k1 + cx] : R(0);
  };
  const R v = R(0.25) * ((E(ya, xa) + E(ya, xb)) + (E(yb, xa) + E(yb, xb)));
  const R xv = x[(size_t)j * n1 + i];
  if (skipv) return;
  x[(size_t)j * n1 + i] = xv + v;
}

template <typename R>
hipError_t launch_prolong(int n1, int n2, const R* e, R* x, const int* skip, hipStream_t st) {
  if (n1 < 3 || n2 < 3) return hipErrorInvalidValue;
  if (n2 > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((prolong_kernel<R>), dim3(ceil_div(n1, kBlock), n2, batch_nz()), dim3(kBlock), 0, st, n1, n2, e, x,
                     skip, batch_ztab());
  return hipGetLastError();
}

// ---- elementwise helpers ----------------------------------------------------------------------
template <typename Tout, typename Tin>
__global__ void convert_kernel(size_t N, const Tin* __restrict__ in, Tout* __restrict__ out, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(in);
  FDE_ZSHIFT(out);
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < N; p += (size_t)gridDim.x * blockDim.x)
    out[p] = (Tout)in[p];
}
template <typename Tout, typename Tin>
hipError_t launch_convert(size_t N, const Tin* in, Tout* out, hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<Tout, Tin>), dim3(grid_for(N), 1, batch_nz()), dim3(kBlock), 0, st, N, in, out,
                     batch_ztab());
  return hipGetLastError();
}

template <typename R>
__global__ void fill_kernel(size_t N, R* __restrict__ out, R v, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(out);
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < N; p += (size_t)gridDim.x * blockDim.x)
    out[p] = v;
}
template <typename R>
hipError_t launch_fill(size_t N, R* out, R v, hipStream_t st) {
  hipLaunchKernelGGL((fill_kernel<R>), dim3(grid_for(N), 1, batch_nz()), dim3(kBlock), 0, st, N, out, v, batch_ztab());
  return hipGetLastError();
}

template <typename R>
__global__ void interleave_kernel(size_t N, const double* __restrict__ a, const double* __restrict__ b,
                                  R* __restrict__ out) {
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < N; p += (size_t)gridDim.x * blockDim.x) {
    out[2 * p] = (R)a[p];
    out[2 * p + 1] = (R)b[p];
  }
}
template <typename R>
hipError_t launch_interleave(size_t N, const double* a, const double* b, R* out, hipStream_t st) {
  hipLaunchKernelGGL((interleave_kernel<R>), dim3(grid_for(N)), dim3(kBlock), 0, st, N, a, b, out);
  return hipGetLastError();
}

template <typename R>
__global__ void inject_pairs_kernel(int n1, int n2, const R* __restrict__ in, R* __restrict__ out) {
  const int k1 = n1 >> 1, k2 = n2 >> 1;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < k1 * k2; q += gridDim.x * blockDim.x) {
    const int J = q / k1, I = q - J * k1;
    const size_t f = (size_t)(2 * J + (n2 & 1)) * n1 + (2 * I + (n1 & 1));
    out[2 * q] = in[2 * f];
    out[2 * q + 1] = in[2 * f + 1];
  }
}
template <typename R>
hipError_t launch_inject_pairs(int n1, int n2, const R* in, R* out, hipStream_t st) {
  const int Kc = (n1 >> 1) * (n2 >> 1);
  hipLaunchKernelGGL((inject_pairs_kernel<R>), dim3(grid_for(Kc)), dim3(kBlock), 0, st, n1, n2, in, out);
  return hipGetLastError();
}

// diag(A) = 1 - sx w1^a (d+ + d-) - sy w1^b (e+ + e-): T has w_1 on its diagonal (eq. (AN)).
template <typename R>
__global__ void diag_kernel(int N, const R* __restrict__ dpm, const R* __restrict__ epm, double sxw1,
                            double syw1, double omega, R* __restrict__ dinv, double* __restrict__ dout) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
    const double d = 1.0 - sxw1 * ((double)dpm[2 * p] + (double)dpm[2 * p + 1]) -
                     syw1 * ((double)epm[2 * p] + (double)epm[2 * p + 1]);
    if (dinv) dinv[p] = (R)(omega / d);
    if (dout) dout[p] = d;
  }
}
template <typename R>
hipError_t launch_diag(int N, const R* dpm, const R* epm, double sxw1, double syw1, double omega, R* dinv,
                       double* diag_out, hipStream_t st) {
  hipLaunchKernelGGL((diag_kernel<R>), dim3(grid_for(N)), dim3(kBlock), 0, st, N, dpm, epm, sxw1, syw1,
                     omega, dinv, diag_out);
  return hipGetLastError();
}

__global__ void scan_fields_kernel(size_t N, const double* f0, const double* f1, const double* f2,
                                   const double* f3, int nf, int* flags) {
  int neg = 0, bad = 0;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < N; p += (size_t)gridDim.x * blockDim.x) {
    const double* fs[4] = {f0, f1, f2, f3};
    for (int k = 0; k < nf; ++k) {
      const double v = fs[k][p];
      if (!(v == v) || v == __builtin_inf() || v == -__builtin_inf()) bad = 1;
      else if (v < 0.0) neg = 1;
    }
  }
  if (neg) atomicOr(&flags[0], 1);
  if (bad) atomicOr(&flags[1], 1);
}
hipError_t launch_scan_fields(size_t N, const double* const* f, int nf, int* flags, hipStream_t st) {
  const double* g[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < nf && k < 4; ++k) g[k] = f[k];
  hipLaunchKernelGGL(scan_fields_kernel, dim3(grid_for(N)), dim3(kBlock), 0, st, N, g[0], g[1], g[2], g[3],
                     nf, flags);
  return hipGetLastError();
}

// ---- direct (dense Toeplitz sum) operator on small levels -------------------------------------
// l(j,i) = d+ sum_k swx[i-k+1] X[j][k] + d- sum_k swx[k-i+1] X[j][k]
//        + e+ sum_k swy[j-k+1] X[k][i] + e- sum_k swy[k-j+1] X[k][i]   (only indices >= 0)
// l = (tau/2 L x)(j, i) on a small level held in LDS.  wx, wy: the scaled weights zero-extended,
// w[n + m] = s w_m for 0 <= m <= n and 0 below (2n + 2 entries), so that every sum runs over the
// whole row or column without bounds (fixed trip counts the compiler can pipeline).
template <typename R>
__device__ __forceinline__ R direct_l(int n1, int n2, int j, int i, const R* X, const R* wx,
                                      const R* wy, const R* __restrict__ dpm,
                                      const R* __restrict__ epm) {
  R lx = 0, rx = 0, ly = 0, ry = 0;
  const R* row = X + j * n1;
  const R* wl = wx + n1 + i + 1;  // wl[-k] = s w_{i-k+1}
  const R* wr = wx + n1 - i + 1;  // wr[k]  = s w_{k-i+1}
#pragma unroll 4
  for (int k = 0; k < n1; ++k) {
    const R v = row[k];
    lx += wl[-k] * v;
    rx += wr[k] * v;
  }
  const R* vl = wy + n2 + j + 1;
  const R* vr = wy + n2 - j + 1;
#pragma unroll 4
  for (int k = 0; k < n2; ++k) {
    const R v = X[k * n1 + i];
    ly += vl[-k] * v;
    ry += vr[k] * v;
  }
  const int p = j * n1 + i;
  return dpm[2 * p] * lx + dpm[2 * p + 1] * rx + epm[2 * p] * ly + epm[2 * p + 1] * ry;
}

// Fills the zero-extended weight table w[0, 2n + 2) from sw[0..n] (see direct_l).
template <typename R>
__device__ __forceinline__ void fill_wext(R* w, const R* __restrict__ sw, int n, int tid, int nt) {
  for (int m = tid; m < 2 * n + 2; m += nt) w[m] = (m >= n && m - n <= n) ? sw[m - n] : R(0);
}

// ---- tiled operator kernels of the direct (dense-Toeplitz) levels, fused with the transfers -------
// A workgroup owns a tile of output points and stages in LDS what its Toeplitz sums read: the tile's
// rows over the whole row length and its columns over the whole column length (as x, or as the
// prolongated-and-corrected x + P e), plus the zero-extended weight tables.  Two fusions of the
// V-cycle's transfer steps (Sec. 4.1, Lemma lemapp) follow:
//   * residual + restriction: the residual b - A x of a 15 x 15 fine block, then the 9-point
//     full weighting P^T r / 4 onto the 7 x 7 coarse points whose stencils the block covers (coarse
//     J, I <-> fine 2J+1, 2I+1), and the coarse level's first Jacobi sweep from zero; the residual
//     never leaves LDS (blocks overlap by one fine row and column);
//   * prolongation + Jacobi: x_new = x + P e formed while staging, then one damped-Jacobi sweep
//     x_new + dinv (b - A x_new) on a 16 x 16 tile, written to a second buffer (neighbouring tiles
//     still read x).
// These levels are small (at most 255 points per side), so a kernel's time is mostly the latency of
// its global loads: every thread issues all of its loads (the skip flag included) in one round
// before it waits for any of them.
constexpr int kTileJ = 16;            // Jacobi tile side (fine points)
constexpr int kTileRC = 7;            // restriction tile side (coarse points)
constexpr int kTileRF = 2 * kTileRC + 1;  // fine rows and columns it covers
constexpr int kTileThreads = 256;
constexpr int kTileMaxN = 255;        // largest side of a tiled level (one staged row per thread)
constexpr int kTileCS = kTileJ / 2 + 1;   // coarse rows (columns) under the 16 fine rows of a tile

template <typename R>
struct Pair {
  R a, b;
};
template <typename R>
__device__ __forceinline__ Pair<R> load_pair(const R* p) {
  using R2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
  const R2 v = *reinterpret_cast<const R2*>(p);
  return {v.x, v.y};
}

// Entry m of the zero-extended weight table (w[n + k] = sw[k] for 0 <= k <= n, 0 below).
template <typename R>
__device__ __forceinline__ R wext_value(const R* __restrict__ sw, int n, int m) {
  return load_or_zero(sw, m - n, m >= n && m - n <= n && m < 2 * n + 2);
}

// tau/2 (L x)(j, i) from the staged row xrow (whole length n1), the staged column xcol (stride nc)
// and the point's coefficient pairs.
template <typename R>
__device__ __forceinline__ R tile_l(int n1, int n2, int j, int i, const R* xrow, const R* xcol, int nc, const R* wx,
                                    const R* wy, Pair<R> d, Pair<R> e) {
  R lx = 0, rx = 0, ly = 0, ry = 0;
  const R* wl = wx + n1 + i + 1;  // wl[-k] = swx[i-k+1]
  const R* wr = wx + n1 - i + 1;  // wr[k]  = swx[k-i+1]
#pragma unroll 4
  for (int k = 0; k < n1; ++k) {
    const R v = xrow[k];
    lx += wl[-k] * v;
    rx += wr[k] * v;
  }
  const R* vl = wy + n2 + j + 1;
  const R* vr = wy + n2 - j + 1;
#pragma unroll 4
  for (int k = 0; k < n2; ++k) {
    const R v = xcol[k * nc];
    ly += vl[-k] * v;
    ry += vr[k] * v;
  }
  return d.a * lx + d.b * rx + e.a * ly + e.b * ry;
}

template <typename R>
__host__ __device__ constexpr size_t tile_rr_lds(int n1, int n2) {
  return ((size_t)kTileRF * n1 + (size_t)n2 * kTileRF + 2 * n1 + 2 + 2 * n2 + 2 + kTileRF * kTileRF) * sizeof(R);
}
template <typename R>
__host__ __device__ constexpr size_t tile_j_lds(int n1, int n2) {
  return ((size_t)kTileJ * n1 + (size_t)n2 * kTileJ + 2 * n1 + 2 + 2 * n2 + 2 +
          (size_t)kTileCS * ((n1 - 1) / 2) + (size_t)((n2 - 1) / 2) * kTileCS) *
         sizeof(R);
}

// Staged values of a tile: its NR rows at column tid of each, and its NC columns (column tid % NC,
// rows tid / NC + u * (256 / NC)), loaded into registers in one round.
template <typename R, int NR, int NC>
struct TileLoads {
  static constexpr int KSTEP = kTileThreads / NC;
  static constexpr int NU = (kTileMaxN + KSTEP - 1) / KSTEP;
  R xrv[NR], xcv[NU], wxv[2], wyv[2];
  __device__ __forceinline__ void load(int n1, int n2, const R* __restrict__ x, int r0, int c0,
                                       const R* __restrict__ swx, const R* __restrict__ swy) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < NR; ++r) xrv[r] = load_or_zero(x, (size_t)(r0 + r) * n1 + tid, tid < n1 && r0 + r < n2);
    const int cc = tid % NC, i = c0 + cc;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int k = tid / NC + u * KSTEP;
      xcv[u] = load_or_zero(x, (size_t)k * n1 + i, tid < KSTEP * NC && k < n2 && i < n1);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      wxv[q] = wext_value(swx, n1, tid + q * kTileThreads);
      wyv[q] = wext_value(swy, n2, tid + q * kTileThreads);
    }
  }
  __device__ __forceinline__ void store_weights(int n1, int n2, R* wx, R* wy) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int m = tid + q * kTileThreads;
      if (m < 2 * n1 + 2) wx[m] = wxv[q];
      if (m < 2 * n2 + 2) wy[m] = wyv[q];
    }
  }
  // stage x (+ f(row, col) when given) into xr[NR][n1] and xc[n2][NC]
  template <class F>
  __device__ __forceinline__ void store_x(int n1, int n2, int r0, int c0, R* xr, R* xc, F&& add) const {
    const int tid = threadIdx.x;
    if (tid < n1) {
#pragma unroll
      for (int r = 0; r < NR; ++r) xr[r * n1 + tid] = (r0 + r < n2) ? xrv[r] + add(r0 + r, tid) : R(0);
    }
    const int cc = tid % NC, i = c0 + cc;
    if (tid < KSTEP * NC) {
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int k = tid / NC + u * KSTEP;
        if (k < n2) xc[k * NC + cc] = i < n1 ? xcv[u] + add(k, i) : R(0);
      }
    }
  }
};

template <typename R>
__global__ __launch_bounds__(kTileThreads) void tile_resid_restrict_kernel(
    int n1, int n2, const R* __restrict__ x, const R* __restrict__ b, const R* __restrict__ dpm,
    const R* __restrict__ epm, const R* __restrict__ swx, const R* __restrict__ swy, R* __restrict__ bc,
    const R* __restrict__ dinv_c, R* __restrict__ xcout, const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(b);
  FDE_ZSHIFT(dpm);
  FDE_ZSHIFT(epm);
  FDE_ZSHIFT(swx);
  FDE_ZSHIFT(swy);
  FDE_ZSHIFT(bc);
  FDE_ZSHIFT(dinv_c);
  FDE_ZSHIFT(xcout);
  FDE_ZSHIFT(skip);
  extern __shared__ unsigned char smem_raw[];
  R* xr = reinterpret_cast<R*>(smem_raw);  // kTileRF x n1
  R* xc = xr + kTileRF * n1;               // n2 x kTileRF
  R* wx = xc + n2 * kTileRF;
  R* wy = wx + 2 * n1 + 2;
  R* rt = wy + 2 * n2 + 2;                 // kTileRF x kTileRF residual block
  const int tid = threadIdx.x;
  const int k1 = (n1 - 1) / 2, k2 = (n2 - 1) / 2;
  const int I0 = blockIdx.x * kTileRC, J0 = blockIdx.y * kTileRC;
  const int r0 = 2 * J0, c0 = 2 * I0;
  // one round of loads: skip flag, staged rows and columns, weights, this thread's point and coarse point
  const int skipv = load_flag(skip);
  TileLoads<R, kTileRF, kTileRF> ld;
  ld.load(n1, n2, x, r0, c0, swx, swy);
  const int rr = tid / kTileRF, cc = tid - rr * kTileRF;
  const int j = r0 + rr, i = c0 + cc;
  const bool own = tid < kTileRF * kTileRF && j < n2 && i < n1;
  // every load unconditional (index 0 for threads without a point), the values selected afterwards
  const size_t p = own ? (size_t)j * n1 + i : 0;
  Pair<R> dpv = load_pair(dpm + 2 * p);
  Pair<R> epv = load_pair(epm + 2 * p);
  const R bv = load_or_zero(b, p, own);
  if (!own) dpv = epv = Pair<R>{0, 0};
  const int JJ = tid / kTileRC, II = tid - JJ * kTileRC;
  const int J = J0 + JJ, I = I0 + II;
  const bool cown = tid < kTileRC * kTileRC && J < k2 && I < k1;
  const size_t q = cown ? (size_t)J * k1 + I : 0;
  const R dcv = xcout ? load_or_zero(dinv_c, q, cown) : R(0);
  if (skipv) return;
  ld.store_weights(n1, n2, wx, wy);
  ld.store_x(n1, n2, r0, c0, xr, xc, [](int, int) { return R(0); });
  __syncthreads();
  if (tid < kTileRF * kTileRF) {
    R r = R(0);
    if (own) r = bv - xr[rr * n1 + i] + tile_l(n1, n2, j, i, xr + rr * n1, xc + cc, kTileRF, wx, wy, dpv, epv);
    rt[tid] = r;
  }
  __syncthreads();
  if (cown) {
    const R* q0 = rt + (2 * JJ) * kTileRF + 2 * II + 1;
    const R* q1 = q0 + kTileRF;
    const R* q2 = q1 + kTileRF;
    const R a0 = q0[-1] + 2 * q0[0] + q0[1];
    const R a1 = q1[-1] + 2 * q1[0] + q1[1];
    const R a2 = q2[-1] + 2 * q2[0] + q2[1];
    const R v = (a0 + 2 * a1 + a2) * R(0.0625);
    bc[q] = v;
    if (xcout) xcout[q] = dcv * v;
  }
}

template <typename R, bool PRO>
__global__ __launch_bounds__(kTileThreads) void tile_jacobi_kernel(
    int n1, int n2, const R* __restrict__ x, const R* __restrict__ e, const R* __restrict__ b,
    const R* __restrict__ dpm, const R* __restrict__ epm, const R* __restrict__ dinv, const R* __restrict__ swx,
    const R* __restrict__ swy, R* __restrict__ xout, const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(e);
  FDE_ZSHIFT(b);
  FDE_ZSHIFT(dpm);
  FDE_ZSHIFT(epm);
  FDE_ZSHIFT(dinv);
  FDE_ZSHIFT(swx);
  FDE_ZSHIFT(swy);
  FDE_ZSHIFT(xout);
  FDE_ZSHIFT(skip);
  extern __shared__ unsigned char smem_raw[];
  const int k1 = (n1 - 1) / 2, k2 = (n2 - 1) / 2;
  R* xr = reinterpret_cast<R*>(smem_raw);  // kTileJ x n1
  R* xc = xr + kTileJ * n1;                // n2 x kTileJ
  R* wx = xc + n2 * kTileJ;
  R* wy = wx + 2 * n1 + 2;
  R* er = wy + 2 * n2 + 2;                 // coarse rows cr0 .. cr0 + kTileCS - 1 (all k1 columns)
  R* ec = er + kTileCS * k1;               // coarse columns cc0 .. cc0 + kTileCS - 1 (all k2 rows)
  const int tid = threadIdx.x;
  const int r0 = blockIdx.y * kTileJ, c0 = blockIdx.x * kTileJ;
  const int cr0 = (r0 >> 1) - 1, cc0 = (c0 >> 1) - 1;  // first coarse row/column under the tile
  // one round of loads
  const int skipv = load_flag(skip);
  TileLoads<R, kTileJ, kTileJ> ld;
  ld.load(n1, n2, x, r0, c0, swx, swy);
  const int rr = tid / kTileJ, cc = tid - rr * kTileJ;
  const int j = r0 + rr, i = c0 + cc;
  const bool own = j < n2 && i < n1;
  const size_t p = own ? (size_t)j * n1 + i : 0;
  const Pair<R> dpv = own ? load_pair(dpm + 2 * p) : Pair<R>{0, 0};
  const Pair<R> epv = own ? load_pair(epm + 2 * p) : Pair<R>{0, 0};
  const R bv = own ? b[p] : R(0);
  const R dv = own ? dinv[p] : R(0);
  constexpr int NE = PRO ? (kTileCS * ((kTileMaxN - 1) / 2) + kTileThreads - 1) / kTileThreads : 1;
  R erv[NE], ecv[NE];
  if constexpr (PRO) {
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int qr = tid + t * kTileThreads;
      const int cr = qr / k1, ci = qr - cr * k1, y = cr0 + cr;
      erv[t] = (qr < kTileCS * k1 && y >= 0 && y < k2) ? e[(size_t)y * k1 + ci] : R(0);
      const int ck = qr / kTileCS, cj = qr - ck * kTileCS, xcol = cc0 + cj;
      ecv[t] = (qr < k2 * kTileCS && xcol >= 0 && xcol < k1) ? e[(size_t)ck * k1 + xcol] : R(0);
    }
  }
  if (skipv) return;
  ld.store_weights(n1, n2, wx, wy);
  if constexpr (PRO) {
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int qr = tid + t * kTileThreads;
      if (qr < kTileCS * k1) er[qr] = erv[t];
      if (qr < k2 * kTileCS) ec[qr] = ecv[t];
    }
    __syncthreads();
    // (P e)(j, i): a quarter of the sum of the up to four coarse neighbours, read from the row strip
    // (staged rows) or the column strip (staged columns)
    auto pe_row = [&](int jj, int ii) -> R {
      const int ya = ((jj - 1) >> 1) - cr0, yb = (jj >> 1) - cr0, xa = (ii - 1) >> 1, xb = ii >> 1;
      const R a = xa >= 0 ? er[ya * k1 + xa] + er[yb * k1 + xa] : R(0);
      const R c = xb < k1 ? er[ya * k1 + xb] + er[yb * k1 + xb] : R(0);
      return R(0.25) * (a + c);
    };
    auto pe_col = [&](int jj, int ii) -> R {
      const int ya = (jj - 1) >> 1, yb = jj >> 1, xa = ((ii - 1) >> 1) - cc0, xb = (ii >> 1) - cc0;
      const R a = ya >= 0 ? ec[ya * kTileCS + xa] + ec[ya * kTileCS + xb] : R(0);
      const R c = yb < k2 ? ec[yb * kTileCS + xa] + ec[yb * kTileCS + xb] : R(0);
      return R(0.25) * (a + c);
    };
    if (tid < n1) {
#pragma unroll
      for (int r = 0; r < kTileJ; ++r)
        xr[r * n1 + tid] = (r0 + r < n2) ? ld.xrv[r] + pe_row(r0 + r, tid) : R(0);
    }
    {
      constexpr int KS = TileLoads<R, kTileJ, kTileJ>::KSTEP, NU = TileLoads<R, kTileJ, kTileJ>::NU;
      const int ci = c0 + tid % kTileJ;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int k = tid / kTileJ + u * KS;
        if (k < n2) xc[k * kTileJ + tid % kTileJ] = ci < n1 ? ld.xcv[u] + pe_col(k, ci) : R(0);
      }
    }
  } else {
    ld.store_x(n1, n2, r0, c0, xr, xc, [](int, int) { return R(0); });
  }
  __syncthreads();
  if (!own) return;
  const R xv = xr[rr * n1 + i];
  const R l = tile_l(n1, n2, j, i, xr + rr * n1, xc + cc, kTileJ, wx, wy, dpv, epv);
  xout[p] = xv + dv * (bv - xv + l);
}

template <typename R>
bool tile_lds_fits(int n1, int n2) {
  return n1 <= kTileMaxN && n2 <= kTileMaxN && tile_rr_lds<R>(n1, n2) <= 160 * 1024 &&
         tile_j_lds<R>(n1, n2) <= 160 * 1024;
}

template <typename R>
hipError_t launch_tile_resid_restrict(int n1, int n2, const R* x, const R* b, const R* dpm, const R* epm,
                                      const R* swx, const R* swy, R* bc, const R* dinv_c, R* xc, const int* skip,
                                      hipStream_t st) {
  const int k1 = (n1 - 1) / 2, k2 = (n2 - 1) / 2;
  // (fine blocks laid out for odd sides: coarse J at fine 2J + 1)
  if (!(n1 & n2 & 1) || k1 < 1 || k2 < 1 || (xc && !dinv_c) || !tile_lds_fits<R>(n1, n2))
    return hipErrorInvalidValue;
  const size_t bytes = tile_rr_lds<R>(n1, n2);
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_resid_restrict_kernel<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((tile_resid_restrict_kernel<R>), dim3(ceil_div(k1, kTileRC), ceil_div(k2, kTileRC), batch_nz()),
                     dim3(kTileThreads), bytes, st, n1, n2, x, b, dpm, epm, swx, swy, bc, dinv_c, xc, skip,
                     batch_ztab());
  return hipGetLastError();
}

template <typename R, bool PRO>
static hipError_t launch_tile_jacobi_t(int n1, int n2, const R* x, const R* e, const R* b, const R* dpm,
                                       const R* epm, const R* dinv, const R* swx, const R* swy, R* xout,
                                       const int* skip, size_t bytes, hipStream_t st) {
  if (bytes > 65536) {
    hipError_t er = hipFuncSetAttribute(reinterpret_cast<const void*>(&tile_jacobi_kernel<R, PRO>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (er != hipSuccess) return er;
  }
  hipLaunchKernelGGL((tile_jacobi_kernel<R, PRO>), dim3(ceil_div(n1, kTileJ), ceil_div(n2, kTileJ), batch_nz()),
                     dim3(kTileThreads), bytes, st, n1, n2, x, e, b, dpm, epm, dinv, swx, swy, xout, skip,
                     batch_ztab());
  return hipGetLastError();
}

template <typename R>
hipError_t launch_tile_jacobi(int n1, int n2, const R* x, const R* e, const R* b, const R* dpm, const R* epm,
                              const R* dinv, const R* swx, const R* swy, R* xout, const int* skip, hipStream_t st) {
  if (!(n1 & n2 & 1) || n1 < 3 || n2 < 3 || x == xout || !tile_lds_fits<R>(n1, n2)) return hipErrorInvalidValue;
  const size_t bytes = tile_j_lds<R>(n1, n2);
  if (e) return launch_tile_jacobi_t<R, true>(n1, n2, x, e, b, dpm, epm, dinv, swx, swy, xout, skip, bytes, st);
  return launch_tile_jacobi_t<R, false>(n1, n2, x, e, b, dpm, epm, dinv, swx, swy, xout, skip, bytes, st);
}

template <typename R>
struct CoarseLds {
  R* B[kMaxCoarseLevels];
  R* X[kMaxCoarseLevels];
  R* T;
  R* swx[kMaxCoarseLevels];
  R* swy[kMaxCoarseLevels];
  R* dpm[kMaxCoarseLevels];
  R* epm[kMaxCoarseLevels];
  R* dinv[kMaxCoarseLevels];
  double* inv;
};

// LDS of the one-workgroup V-cycle: per level b, x, the weights and the coefficient fields
// (d+-, e+- pairs and omega/diag), one scratch field, and the FP64 coarsest inverse.
template <typename R>
__host__ __device__ size_t coarse_lds_elems(const CoarseView<R>& cv) {
  size_t n = 0, mx = 0;
  for (int l = 0; l < cv.nlev; ++l) {
    const size_t N = (size_t)cv.n1[l] * cv.n2[l];
    n += 2 * N + (2 * cv.n1[l] + 2) + (2 * cv.n2[l] + 2) + 5 * N;
    if (N > mx) mx = N;
  }
  n += mx;
  n += (sizeof(double) / sizeof(R)) + 1;  // alignment slack for the FP64 inverse
  return n;
}
template <typename R>
size_t coarse_lds_bytes(const CoarseView<R>& cv) {
  const int l = cv.nlev - 1;
  const size_t Nc = (size_t)cv.n1[l] * cv.n2[l];
  return coarse_lds_elems(cv) * sizeof(R) + Nc * Nc * sizeof(double);
}

constexpr int kCoarseMaxN = 1024;  // points per level of the one-workgroup V-cycle (31^2 = 961)
constexpr int kCoarseInvPer = 16;  // entries of the coarsest inverse per thread (128^2 / 1024)

// The level loops of the one-workgroup V-cycle run over compile-time level indices (NL levels), so
// that the per-level pointers stay in registers instead of a private array in scratch memory.
template <typename R, int NL>
__device__ CoarseLds<R> coarse_carve(const CoarseView<R>& cv, R* base) {
  CoarseLds<R> s;
  R* q = base;
  int mx = 0;
  static_for<0, NL>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    const int N = cv.n1[l] * cv.n2[l];
    s.B[l] = q;
    q += N;
    s.X[l] = q;
    q += N;
    s.swx[l] = q;  // zero-extended tables (direct_l)
    q += 2 * cv.n1[l] + 2;
    s.swy[l] = q;
    q += 2 * cv.n2[l] + 2;
    s.dpm[l] = q;
    q += 2 * N;
    s.epm[l] = q;
    q += 2 * N;
    s.dinv[l] = q;
    q += N;
    if (N > mx) mx = N;
  });
  s.T = q;
  q += mx;
  uintptr_t a = reinterpret_cast<uintptr_t>(q);
  a = (a + sizeof(double) - 1) & ~(uintptr_t)(sizeof(double) - 1);
  s.inv = reinterpret_cast<double*>(a);
  return s;
}

// One Jacobi step on level L: X <- X + dinv (B - X + l(X)), through the scratch T.
template <typename R, int L>
__device__ void coarse_jacobi(const CoarseView<R>& cv, const CoarseLds<R>& s) {
  const int n1 = cv.n1[L], n2 = cv.n2[L], N = n1 * n2;
  for (int p = threadIdx.x; p < N; p += blockDim.x) {
    const int j = p / n1, i = p - j * n1;
    const R xv = s.X[L][p];
    const R lv = direct_l(n1, n2, j, i, s.X[L], s.swx[L], s.swy[L], s.dpm[L], s.epm[L]);
    s.T[p] = xv + s.dinv[L][p] * (s.B[L][p] - xv + lv);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < N; p += blockDim.x) s.X[L][p] = s.T[p];
  __syncthreads();
}

template <typename R, int NL>
__global__ __launch_bounds__(1024) void coarse_vcycle_kernel(CoarseView<R> cv, const R* __restrict__ b_in,
                                                             R* __restrict__ x_out,
                                                             const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(b_in);
  FDE_ZSHIFT(x_out);
  FDE_ZSHIFT(skip);
  if (zoff) {
    static_for<0, NL>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      FDE_ZSHIFT(cv.dpm[l]);
      FDE_ZSHIFT(cv.epm[l]);
      FDE_ZSHIFT(cv.dinv[l]);
      FDE_ZSHIFT(cv.swx[l]);
      FDE_ZSHIFT(cv.swy[l]);
    });
    FDE_ZSHIFT(cv.inv);
  }
  extern __shared__ unsigned char smem_raw[];
  R* base = reinterpret_cast<R*>(smem_raw);
  const CoarseLds<R> s = coarse_carve<R, NL>(cv, base);
  const int tid = threadIdx.x, nt = blockDim.x;
  constexpr int last = NL - 1;
  // Everything the cycle reads is copied into LDS once.  All loads (the skip flag included) are
  // issued before the first of them is waited for: one round of memory latency instead of one per
  // array.  Per thread: at most 2 pair entries and 1 entry of each level field (levels of at most
  // kCoarseMaxN points), 1 weight-table entry, kCoarseInvPer entries of the FP64 inverse.
  const int skipv = load_flag(skip);
  R gd[NL][2], ge[NL][2], gi[NL], gwx[NL], gwy[NL];
  static_for<0, NL>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    const int N = cv.n1[l] * cv.n2[l];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int k = tid + u * nt;
      gd[l][u] = k < 2 * N ? cv.dpm[l][k] : R(0);
      ge[l][u] = k < 2 * N ? cv.epm[l][k] : R(0);
    }
    gi[l] = tid < N ? cv.dinv[l][tid] : R(0);
    gwx[l] = wext_value(cv.swx[l], cv.n1[l], tid);
    gwy[l] = wext_value(cv.swy[l], cv.n2[l], tid);
  });
  const int Nc = cv.n1[last] * cv.n2[last];
  double ginv[kCoarseInvPer];
#pragma unroll
  for (int u = 0; u < kCoarseInvPer; ++u) {
    const int k = tid + u * nt;
    ginv[u] = k < Nc * Nc ? cv.inv[k] : 0.0;
  }
  const int N0 = cv.n1[0] * cv.n2[0];
  const R gb = tid < N0 ? b_in[tid] : R(0);
  if (skipv) return;
  static_for<0, NL>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    const int N = cv.n1[l] * cv.n2[l];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int k = tid + u * nt;
      if (k < 2 * N) {
        s.dpm[l][k] = gd[l][u];
        s.epm[l][k] = ge[l][u];
      }
    }
    if (tid < N) s.dinv[l][tid] = gi[l];
    if (tid < 2 * cv.n1[l] + 2) s.swx[l][tid] = gwx[l];
    if (tid < 2 * cv.n2[l] + 2) s.swy[l][tid] = gwy[l];
  });
#pragma unroll
  for (int u = 0; u < kCoarseInvPer; ++u) {
    const int k = tid + u * nt;
    if (k < Nc * Nc) s.inv[k] = ginv[u];
  }
  if (tid < N0) s.B[0][tid] = gb;
  __syncthreads();
  // descend: pre-smooth, residual, restrict
  static_for<0, last>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    const int n1 = cv.n1[l], n2 = cv.n2[l], N = n1 * n2;
    for (int p = tid; p < N; p += nt) s.X[l][p] = cv.nu_pre > 0 ? s.dinv[l][p] * s.B[l][p] : R(0);
    __syncthreads();
    for (int it = 1; it < cv.nu_pre; ++it) coarse_jacobi<R, l>(cv, s);
    for (int p = tid; p < N; p += nt) {
      const int j = p / n1, i = p - j * n1;
      const R xv = s.X[l][p];
      s.T[p] = s.B[l][p] - xv + direct_l(n1, n2, j, i, s.X[l], s.swx[l], s.swy[l], s.dpm[l], s.epm[l]);
    }
    __syncthreads();
    const int k1 = n1 >> 1, k2 = n2 >> 1;
    for (int q = tid; q < k1 * k2; q += nt) {
      const int J = q / k1, I = q - J * k1;
      s.B[l + 1][q] = full_weight(s.T, n1, 2 * J + (n2 & 1), 2 * I + (n1 & 1));
    }
    __syncthreads();
  });
  // coarsest: X = inv B (FP64 inverse from Gauss-Jordan elimination with partial pivoting)
  {
    const int Nc = cv.n1[last] * cv.n2[last];
    for (int p = tid; p < Nc; p += nt) {
      double acc = 0.0;
      const double* row = s.inv + (size_t)p * Nc;
      for (int q = 0; q < Nc; ++q) acc += row[q] * (double)s.B[last][q];
      s.X[last][p] = (R)acc;
    }
    __syncthreads();
  }
  // ascend: prolongate, correct, post-smooth
  static_for<0, last>([&](auto kc) {
    constexpr int l = last - 1 - decltype(kc)::value;
    const int n1 = cv.n1[l], n2 = cv.n2[l], N = n1 * n2;
    const int k1 = n1 >> 1;
    const R* E = s.X[l + 1];
    for (int p = tid; p < N; p += nt) {
      const int j = p / n1, i = p - j * n1;
      int cy[2], cx[2], ny, nx;
      float wy[2], wx[2];
      coarse_nbrs(j, n2, cy, wy, &ny);
      coarse_nbrs(i, n1, cx, wx, &nx);
      R v = 0;
      for (int a = 0; a < ny; ++a) {
        R t = 0;
        for (int c = 0; c < nx; ++c) t += (R)wx[c] * E[cy[a] * k1 + cx[c]];
        v += (R)wy[a] * t;
      }
      s.X[l][p] += v;
    }
    __syncthreads();
    for (int it = 0; it < cv.nu_post; ++it) coarse_jacobi<R, l>(cv, s);
  });
  {
    const int N0 = cv.n1[0] * cv.n2[0];
    for (int p = tid; p < N0; p += nt) x_out[p] = s.X[0][p];
  }
}

template <typename R, int NL>
static hipError_t launch_coarse_vcycle_n(const CoarseView<R>& cv, const R* b, R* x, const int* skip, size_t bytes,
                                         hipStream_t st) {
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&coarse_vcycle_kernel<R, NL>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((coarse_vcycle_kernel<R, NL>), dim3(1, 1, batch_nz()), dim3(1024), bytes, st, cv, b, x, skip,
                     batch_ztab());
  return hipGetLastError();
}

template <typename R>
hipError_t launch_coarse_vcycle(const CoarseView<R>& cv, const R* b, R* x, const int* skip, hipStream_t st) {
  const size_t bytes = coarse_lds_bytes(cv);
  if (bytes > 160 * 1024 || !cv.inv) return hipErrorInvalidValue;
  // the single-round load phase holds at most kCoarseMaxN points per level and kCoarseInvPer * 1024
  // entries of the inverse per thread
  for (int l = 0; l < cv.nlev; ++l)
    if (cv.n1[l] * cv.n2[l] > kCoarseMaxN || 2 * cv.n1[l] + 2 > 1024 || 2 * cv.n2[l] + 2 > 1024)
      return hipErrorInvalidValue;
  {
    const int Nc = cv.n1[cv.nlev - 1] * cv.n2[cv.nlev - 1];
    if (Nc * Nc > kCoarseInvPer * 1024) return hipErrorInvalidValue;
  }
  switch (cv.nlev) {
    case 1:
      return launch_coarse_vcycle_n<R, 1>(cv, b, x, skip, bytes, st);
    case 2:
      return launch_coarse_vcycle_n<R, 2>(cv, b, x, skip, bytes, st);
    case 3:
      return launch_coarse_vcycle_n<R, 3>(cv, b, x, skip, bytes, st);
    case 4:
      return launch_coarse_vcycle_n<R, 4>(cv, b, x, skip, bytes, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R>
__global__ void direct_apply_kernel(CoarseView<R> cv, int l, const R* __restrict__ x, R* __restrict__ out,
                                    int mode, const R* __restrict__ b) {
  extern __shared__ unsigned char smem_raw[];
  R* X = reinterpret_cast<R*>(smem_raw);
  const int n1 = cv.n1[l], n2 = cv.n2[l], N = n1 * n2;
  R* swx = X + N;
  R* swy = swx + 2 * n1 + 2;
  for (int p = threadIdx.x; p < N; p += blockDim.x) X[p] = x[p];
  fill_wext(swx, cv.swx[l], n1, threadIdx.x, blockDim.x);
  fill_wext(swy, cv.swy[l], n2, threadIdx.x, blockDim.x);
  __syncthreads();
  for (int p = threadIdx.x; p < N; p += blockDim.x) {
    const int j = p / n1, i = p - j * n1;
    const R lv = direct_l(n1, n2, j, i, X, swx, swy, cv.dpm[l], cv.epm[l]);
    const R xv = X[p];
    R v;
    if (mode == EP_APPLY) v = xv - lv;
    else if (mode == EP_RESID) v = b[p] - xv + lv;
    else if (mode == EP_JACOBI) v = xv + cv.dinv[l][p] * (b[p] - xv + lv);
    else v = lv;
    out[p] = v;
  }
}
template <typename R>
hipError_t launch_direct_apply(const CoarseView<R>& cv, int level, const R* x, R* out, int mode, const R* b,
                               hipStream_t st) {
  const size_t N = (size_t)cv.n1[level] * cv.n2[level];
  const size_t bytes = (N + 2 * cv.n1[level] + 2 * cv.n2[level] + 4) * sizeof(R);
  hipLaunchKernelGGL((direct_apply_kernel<R>), dim3(1), dim3(1024), bytes, st, cv, level, x, out, mode, b);
  return hipGetLastError();
}

// ---- coarsest matrix: assembly and in-place Gauss-Jordan inversion with partial pivoting --------
constexpr int kMaxCoarseN = 128;  // unknowns on the coarsest grid

template <typename R>
__global__ __launch_bounds__(1024) void coarse_invert_kernel(CoarseView<R> cv, const double* __restrict__ dense,
                                                             double* __restrict__ inv, int* __restrict__ status) {
  extern __shared__ unsigned char smem_raw[];
  const int l = cv.nlev - 1;
  const int n1 = cv.n1[l], n2 = cv.n2[l], n = n1 * n2;
  double* A = reinterpret_cast<double*>(smem_raw);
  __shared__ int perm[kMaxCoarseN];
  __shared__ double fcol[kMaxCoarseN];
  __shared__ int piv_row;
  __shared__ int singular;
  const R* dpm = cv.dpm[l];
  const R* epm = cv.epm[l];
  const R* swx = cv.swx[l];
  const R* swy = cv.swy[l];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    if (dense) {
      A[e] = dense[e];
      continue;
    }
    const int p = e / n, q = e - p * n;
    const int j = p / n1, i = p - j * n1, jq = q / n1, iq = q - jq * n1;
    double a = (p == q) ? 1.0 : 0.0;
    if (j == jq) {
      if (i - iq + 1 >= 0) a -= (double)dpm[2 * p] * (double)swx[i - iq + 1];
      if (iq - i + 1 >= 0) a -= (double)dpm[2 * p + 1] * (double)swx[iq - i + 1];
    }
    if (i == iq) {
      if (j - jq + 1 >= 0) a -= (double)epm[2 * p] * (double)swy[j - jq + 1];
      if (jq - j + 1 >= 0) a -= (double)epm[2 * p + 1] * (double)swy[jq - j + 1];
    }
    A[e] = a;
  }
  if (threadIdx.x == 0) singular = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      int pr = k;
      double best = fabs(A[k * n + k]);
      for (int i = k + 1; i < n; ++i) {
        const double v = fabs(A[i * n + k]);
        if (v > best) {
          best = v;
          pr = i;
        }
      }
      if (best == 0.0) singular = 1;
      piv_row = pr;
      perm[k] = pr;
    }
    __syncthreads();
    if (singular) break;
    const int pr = piv_row;
    if (pr != k)
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const double t = A[k * n + c];
        A[k * n + c] = A[pr * n + c];
        A[pr * n + c] = t;
      }
    __syncthreads();
    const double pv = A[k * n + k];
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) A[k * n + c] = (c == k ? 1.0 : A[k * n + c]) / pv;
    for (int i = threadIdx.x; i < n; i += blockDim.x) fcol[i] = A[i * n + k];
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e / n, c = e - i * n;
      if (i == k) continue;
      // the pivot column of row i becomes -f / pv, the corresponding entry of the inverse
      A[e] = (c == k ? 0.0 : A[e]) - fcol[i] * A[k * n + c];
    }
    __syncthreads();
  }
  if (!singular) {
    for (int k = n - 1; k >= 0; --k) {
      const int pr = perm[k];
      if (pr != k)
        for (int r = threadIdx.x; r < n; r += blockDim.x) {
          const double t = A[r * n + k];
          A[r * n + k] = A[r * n + pr];
          A[r * n + pr] = t;
        }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) inv[e] = A[e];
  }
  if (threadIdx.x == 0) *status = singular;
}

template <typename R>
hipError_t launch_coarse_invert(const CoarseView<R>& cv, const double* dense, double* inv, int* status,
                                hipStream_t st) {
  const int l = cv.nlev - 1;
  const int n = cv.n1[l] * cv.n2[l];
  if (n > kMaxCoarseN) return hipErrorInvalidValue;
  const size_t bytes = (size_t)n * n * sizeof(double);
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&coarse_invert_kernel<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((coarse_invert_kernel<R>), dim3(1), dim3(1024), bytes, st, cv, dense, inv, status);
  return hipGetLastError();
}

template <typename R>
__global__ void coarse_solve_kernel(int Nc, const double* __restrict__ inv, const R* __restrict__ b,
                                    R* __restrict__ x, const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(inv);
  FDE_ZSHIFT(b);
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(skip);
  if (skip && *skip) return;
  for (int p = threadIdx.x; p < Nc; p += blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < Nc; ++q) acc += inv[(size_t)p * Nc + q] * (double)b[q];
    x[p] = (R)acc;
  }
}
template <typename R>
hipError_t launch_coarse_solve(int Nc, const double* inv, const R* b, R* x, const int* skip, hipStream_t st) {
  hipLaunchKernelGGL((coarse_solve_kernel<R>), dim3(1, 1, batch_nz()), dim3(256), 0, st, Nc, inv, b, x, skip,
                     batch_ztab());
  return hipGetLastError();
}

// ---- x += z (FP64 x, z in the preconditioner precision) ---------------------------------------
template <typename R>
__global__ void add_to_kernel(size_t N, const R* __restrict__ z, double* __restrict__ x) {
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < N; p += (size_t)gridDim.x * blockDim.x)
    x[p] += (double)z[p];
}
template <typename R>
hipError_t launch_add_to(size_t N, const R* z, double* x, hipStream_t st) {
  hipLaunchKernelGGL((add_to_kernel<R>), dim3(grid_for(N)), dim3(kBlock), 0, st, N, z, x);
  return hipGetLastError();
}
template hipError_t launch_add_to<float>(size_t, const float*, double*, hipStream_t);
template hipError_t launch_add_to<double>(size_t, const double*, double*, hipStream_t);

// ---- explicit instantiations ------------------------------------------------------------------
#define FDE_INST_R(R)                                                                                   \
  template hipError_t launch_restrict<R>(int, int, const R*, R*, const R*, R*, const int*, hipStream_t); \
  template hipError_t launch_prolong<R>(int, int, const R*, R*, const int*, hipStream_t);              \
  template hipError_t launch_fill<R>(size_t, R*, R, hipStream_t);                                      \
  template hipError_t launch_interleave<R>(size_t, const double*, const double*, R*, hipStream_t);     \
  template hipError_t launch_tile_resid_restrict<R>(int, int, const R*, const R*, const R*, const R*,    \
                                                    const R*, const R*, R*, const R*, R*, const int*,     \
                                                    hipStream_t);                                         \
  template bool tile_lds_fits<R>(int, int);                                                            \
  template hipError_t launch_tile_jacobi<R>(int, int, const R*, const R*, const R*, const R*, const R*,  \
                                            const R*, const R*, const R*, R*, const int*, hipStream_t);   \
  template hipError_t launch_inject_pairs<R>(int, int, const R*, R*, hipStream_t);                     \
  template hipError_t launch_diag<R>(int, const R*, const R*, double, double, double, R*, double*,      \
                                     hipStream_t);                                                      \
  template hipError_t launch_coarse_vcycle<R>(const CoarseView<R>&, const R*, R*, const int*,           \
                                              hipStream_t);                                             \
  template size_t coarse_lds_bytes<R>(const CoarseView<R>&);                                            \
  template hipError_t launch_direct_apply<R>(const CoarseView<R>&, int, const R*, R*, int, const R*,    \
                                             hipStream_t);                                              \
  template hipError_t launch_coarse_invert<R>(const CoarseView<R>&, const double*, double*, int*, hipStream_t); \
  template hipError_t launch_coarse_solve<R>(int, const double*, const R*, R*, const int*, hipStream_t);
FDE_INST_R(double)
FDE_INST_R(float)
template hipError_t launch_presmooth<double, double>(int, const double*, const double*, const double*,
                                                     double*, double*, const int*, hipStream_t);
template hipError_t launch_presmooth<float, double>(int, const double*, const double*, const float*, float*,
                                                    float*, const int*, hipStream_t);
template hipError_t launch_presmooth<float, float>(int, const float*, const double*, const float*, float*,
                                                   float*, const int*, hipStream_t);
template hipError_t launch_convert<float, double>(size_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<double, float>(size_t, const float*, double*, hipStream_t);
template hipError_t launch_convert<double, double>(size_t, const double*, double*, hipStream_t);
template hipError_t launch_convert<float, float>(size_t, const float*, float*, hipStream_t);

}  // namespace fde
