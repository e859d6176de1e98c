// Toeplitz operator application on the GPU: A x = x - tau/2 L x with
//   tau/2 L x = D+ .* (X sxT^T) + D- .* (X sxT) + E+ .* (syT X) + E- .* (syT^T X)   (fields, x fastest)
// where T = [w_{i-j+1}] is the lower-Hessenberg Toeplitz matrix of the WSGD weights (eq. (AN) up to
// sign), sx = tau/(2 hx^alpha), sy = tau/(2 hy^beta) (the r and s of eq. (system)), following the
// Kronecker form of eq. (AxAy).
//
// Both directions use the circulant embedding of length L = 2(n+1): T v is the first n entries of
// C v_pad with C the circulant whose first column is c = [t_0 .. t_{n-1}, 0 .. 0, t_{-1}], t_m =
// w_{m+1}.  With lam = DFT(c):  T v = IDFT(lam .* DFT(v))  and  T^T v = IDFT(conj(lam) .* DFT(v)).
// Two real vectors a, b share every transform: with z = a + i b and Z = DFT(z),
//   IDFT(lam .* Z) = T a + i T b   and   IDFT(conj(lam) .* Z) = T^T a + i T^T b,
// because T and T^T are real.  So one forward and two inverse transforms give all four products.
//
// Kernels:
//   toep_y_kernel : column strips of 2*S columns per workgroup (S transform slots interleaved
//                   across lanes so that each load instruction covers 2*S adjacent columns);
//                   writes ay = E+ .* (syT X) + E- .* (syT^T X).
//   toep_x_kernel : two rows per workgroup; adds the x part and applies the epilogue.
#include <cmath>
#include <complex>
#include <vector>

#include "common.h"
#include "fft.h"
#include "toep_dev.h"

namespace fde {

// Epilogue at one point, MODE fixed at compile time.  l = x part + y part of tau/2 L x.
template <int MODE, typename R, typename Tin>
__device__ __forceinline__ R epilogue_value(R l, Tin xv, R bv, R dv, double srcv, double tau) {
  if constexpr (MODE == EP_LOUT) return l;
  else if constexpr (MODE == EP_APPLY) return (R)xv - l;
  else if constexpr (MODE == EP_RESID) return bv - (R)xv + l;
  else if constexpr (MODE == EP_JACOBI) return (R)xv + dv * (bv - (R)xv + l);
  else return (R)xv + l + (R)(tau * srcv);  // EP_RHS
}

template <typename R, typename Tin, int L, int MODE, bool ZB>
__global__ __launch_bounds__((XCfg<R, L>::THREADS), FDE_XW) void toep_x_kernel(
    int n1, int n2, const Tin* x, const R* __restrict__ dpm, const R* __restrict__ mu,
    const R* __restrict__ twtab, const R* __restrict__ ay, const R* __restrict__ b,
    const R* __restrict__ dinv, SrcTerms src, double tau, R* out, const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN_IF(ZB);
  // batched launches: every per-instance pointer (the source terms of EP_RHS are never batched)
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(dpm);
  FDE_ZSHIFT(mu);
  FDE_ZSHIFT(twtab);
  FDE_ZSHIFT(ay);
  FDE_ZSHIFT(b);
  FDE_ZSHIFT(dinv);
  FDE_ZSHIFT(out);
  FDE_ZSHIFT(skip);
  const int skipv = load_flag(skip);  // waited for after the row loads are issued
  using P = XPlan<R, L>;
  constexpr int E = P::E, T = P::T, S = XCfg<R, L>::S;
  constexpr int SLOT = lds_exchange(L) + 2 * L;
  __shared__ R lds_all[S * SLOT];
  const int slot = threadIdx.x / T;
  const int t = threadIdx.x - slot * T;
  R* lds = lds_all + slot * SLOT;
  R* zs = lds + lds_exchange(L);
  Twiddles<R, L, P> tw;
  tw.load(twtab, t);
  const int rowA = 2 * (blockIdx.x * S + slot);
  const bool hasA = rowA < n2;
  const bool hasB = rowA + 1 < n2;
  // per-row base pointers (uniform when a workgroup holds one row pair); in-row offsets are 32-bit.
  // The x rows of a missing row point at row 0, so that their (unused) loads stay in bounds.
  const size_t oA = (size_t)rowA * n1, oB = oA + n1;
  auto U = [&](auto* ptr) { return S == 1 ? uniform_ptr(ptr) : ptr; };
  const Tin* xa = U(x + (hasA ? oA : 0));
  const Tin* xb = U(x + (hasB ? oB : 0));
  const R* dA = U(dpm + 2 * oA);
  const R* dB = U(dpm + 2 * oB);
  // n1 <= L/2: a row occupies registers m < E/2; the rest is the zero padding of the embedding, and
  // of the results only those registers are needed
  constexpr int EH = E / 2;
  R zr[E], zi[E];
  static_for<0, E>([&](auto m) {
    const int i = t + T * m;
    if constexpr (decltype(m)::value < EH) {
      if constexpr (sizeof(R) == 8) {
        zr[m] = (R)load_or_zero(xa, i, hasA & (i < n1));
        zi[m] = (R)load_or_zero(xb, i, hasB & (i < n1));
      } else {  // the FP32 passes issued these together already (measured 1 us faster this way)
        zr[m] = (hasA && i < n1) ? (R)xa[i] : R(0);
        zi[m] = (hasB && i < n1) ? (R)xb[i] : R(0);
      }
    } else {
      zr[m] = R(0);
      zi[m] = R(0);
    }
  });
  using R2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
  constexpr bool PF = XCfg<R, L>::PREFETCH && MODE != EP_RHS;
  if constexpr (XCfg<R, L>::PREFETCH_EPI && MODE != EP_RHS) {
    R dmA[EH], dmB[EH];
    R pr[E], pi[E];
    if constexpr (PF) {
      R lr[E], li[E];
      static_for<0, E>([&](auto m) {
        const int k = t + T * m;
        lr[m] = mu[2 * k];
        li[m] = mu[2 * k + 1];
      });
      if (skipv) return;
      fft<L, -1, true>(zr, zi, lds, tw, t);
      symbol_both_regs<L, P>(zr, zi, zs, lr, li, t);
      R2 dA2[EH], dB2[EH];
      static_for<0, EH>([&](auto m) {
        const int i = t + T * m;
        dA2[m] = R2{};
        dB2[m] = R2{};
        if (hasA && i < n1) dA2[m] = *reinterpret_cast<const R2*>(dA + 2 * i);
        if (hasB && i < n1) dB2[m] = *reinterpret_cast<const R2*>(dB + 2 * i);
      });
      fft<L, +1>(zr, zi, lds, tw, t);  // real part: T xa, imaginary part: T xb
      unstash<L, P>(pr, pi, zs, t);
      static_for<0, EH>([&](auto m) {
        const int i = t + T * m;
        zs[i] = dA2[m].x * zr[m];
        zs[L + i] = dB2[m].x * zi[m];
        dmA[m] = dA2[m].y;
        dmB[m] = dB2[m].y;
      });
    } else {
      if (skipv) return;
      fft<L, -1, true>(zr, zi, lds, tw, t);
      symbol_both<L, P>(zr, zi, zs, mu, t);
      fft<L, +1>(zr, zi, lds, tw, t);  // real part: T xa, imaginary part: T xb
      unstash<L, P>(pr, pi, zs, t);
      chunked_for<EH, kEpiGroup>([&](auto m) {
        const int i = t + T * m;
        R2 a{}, c{};
        if (hasA && i < n1) a = *reinterpret_cast<const R2*>(dA + 2 * i);
        if (hasB && i < n1) c = *reinterpret_cast<const R2*>(dB + 2 * i);
        zs[i] = a.x * zr[m];
        zs[L + i] = c.x * zi[m];
        dmA[m] = a.y;
        dmB[m] = c.y;
      });
    }
    // the epilogue's operands of both rows, loaded before the second inverse transform
    constexpr bool NX = MODE != EP_LOUT, NB = MODE == EP_RESID || MODE == EP_JACOBI, ND = MODE == EP_JACOBI;
    Tin xv[2][EH];
    R ayv[2][EH], bv[2][EH], dv[2][EH];
    const size_t oR[2] = {oA, oB};
    const bool hasR[2] = {hasA, hasB};
    static_for<0, 2>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const size_t o = oR[r];
      static_for<0, EH>([&](auto m) {
        const int i = t + T * m;
        const bool ok = hasR[r] && i < n1;
        xv[r][m] = Tin(0);
        ayv[r][m] = bv[r][m] = dv[r][m] = R(0);
        if (ok) {
          if constexpr (NX) xv[r][m] = x[o + i];
          if (ay) ayv[r][m] = ay[o + i];
          if constexpr (NB) bv[r][m] = b[o + i];
          if constexpr (ND) dv[r][m] = dinv[o + i];
        }
      });
    });
    fft<L, +1>(pr, pi, lds, tw, t);  // real part: T^T xa, imaginary part: T^T xb
    static_for<0, EH>([&](auto m) {
      const int i = t + T * m;
      if (hasA && i < n1) {
        const R l = zs[i] + dmA[m] * pr[m] + ayv[0][m];
        out[oA + i] = epilogue_value<MODE, R, Tin>(l, xv[0][m], bv[0][m], dv[0][m], 0.0, tau);
        if (hasB) {
          const R l2 = zs[L + i] + dmB[m] * pi[m] + ayv[1][m];
          out[oB + i] = epilogue_value<MODE, R, Tin>(l2, xv[1][m], bv[1][m], dv[1][m], 0.0, tau);
        }
      }
    });
    return;
  }
  if (skipv) return;
  fft<L, -1, true>(zr, zi, lds, tw, t);
  symbol_both<L, P>(zr, zi, zs, mu, t);
  fft<L, +1>(zr, zi, lds, tw, t);  // real part: T xa, imaginary part: T xb
  R pr[E], pi[E];
  unstash<L, P>(pr, pi, zs, t);
  R dmA[EH], dmB[EH];
  chunked_for<EH, kEpiGroup>([&](auto m) {
    const int i = t + T * m;
    R2 a{}, c{};
    if (hasA && i < n1) a = *reinterpret_cast<const R2*>(dA + 2 * i);
    if (hasB && i < n1) c = *reinterpret_cast<const R2*>(dB + 2 * i);
    zs[i] = a.x * zr[m];
    zs[L + i] = c.x * zi[m];
    dmA[m] = a.y;
    dmB[m] = c.y;
  });
  fft<L, +1>(pr, pi, lds, tw, t);  // real part: T^T xa, imaginary part: T^T xb
  const R* ayA = ay ? U(ay + oA) : nullptr;
  const R* ayB = ay ? U(ay + oB) : nullptr;
  const R* bA = b ? U(b + oA) : nullptr;
  const R* bB = b ? U(b + oB) : nullptr;
  const R* diA = dinv ? U(dinv + oA) : nullptr;
  const R* diB = dinv ? U(dinv + oB) : nullptr;
  R* outA = U(out + oA);
  R* outB = U(out + oB);
  auto finish = [&](const Tin* xr, R dm, const R* ayr, const R* br, const R* dir, R* outr, size_t o,
                    R lpart, R rpart, int i) {
    R l = lpart + dm * rpart;
    if (ayr) l += ayr[i];
    R bv = R(0), dv = R(0);
    double sv = 0.0;
    Tin xv = Tin(0);
    if constexpr (MODE != EP_LOUT) xv = xr[i];
    if constexpr (MODE == EP_RESID || MODE == EP_JACOBI) bv = br[i];
    if constexpr (MODE == EP_JACOBI) dv = dir[i];
    if constexpr (MODE == EP_RHS) {
      for (int k = 0; k < src.n; ++k) sv += src.phi[k] * src.S[k][o + i];
    }
    outr[i] = epilogue_value<MODE, R, Tin>(l, xv, bv, dv, sv, tau);
  };
  chunked_for<EH, kEpiGroup>([&](auto m) {
    const int i = t + T * m;
    if (hasA && i < n1) {
      finish(xa, dmA[m], ayA, bA, diA, outA, oA, zs[i], pr[m], i);
      if (hasB) finish(xb, dmB[m], ayB, bB, diB, outB, oB, zs[L + i], pi[m], i);
    }
  });
}

// ay = e+ (T a) + e- (T^T a) for the column pair (c0, c0 + 1): the first products wait in zs, the
// second in (pr, pi).
template <int L, int EH, int T, typename R, int E>
__device__ __forceinline__ void y_store(int n1, int n2, int c0, bool v0, bool v1, int t, const R* zs,
                                        const R (&em0)[EH], const R (&em1)[EH], const R (&pr)[E],
                                        const R (&pi)[E], R* __restrict__ ay) {
  chunked_for<EH, kEpiGroup>([&](auto m) {
    const int row = t + T * m;
    if (row < n2) {
      const unsigned p = (unsigned)row * (unsigned)n1 + (unsigned)c0;
      if (v0) ay[p] = zs[row] + em0[m] * pr[m];
      if (v1) ay[p + 1] = zs[L + row] + em1[m] * pi[m];
    }
  });
}

template <typename R, typename Tin, int L, bool ZB>
__global__ __launch_bounds__((YCfg<R, L>::THREADS), FDE_YW) void toep_y_kernel(
    int n1, int n2, const Tin* __restrict__ x, const R* __restrict__ epm, const R* __restrict__ mu,
    const R* __restrict__ twtab, R* __restrict__ ay, int nstrips, const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN_IF(ZB);
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(epm);
  FDE_ZSHIFT(mu);
  FDE_ZSHIFT(twtab);
  FDE_ZSHIFT(ay);
  FDE_ZSHIFT(skip);
  const int skipv = load_flag(skip);  // waited for after the column loads are issued
  using P = YPlan<R, L>;
  constexpr int E = P::E, T = P::T, S = YCfg<R, L>::S;
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous range of strips so
  // that neighbouring strips (which share cache lines) meet in the same L2.
  const int per = gridDim.x / 8;
  const int strip = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (strip >= nstrips) return;
  constexpr int SLOT = lds_exchange(L) + 2 * L;
  __shared__ R lds_all[S * SLOT];
  const int slot = threadIdx.x % S;
  const int t = threadIdx.x / S;
  R* lds = lds_all + slot * SLOT;
  R* zs = lds + lds_exchange(L);
  Twiddles<R, L, P> tw;
  tw.load(twtab, t);
  const int c0 = strip * 2 * S + 2 * slot;
  const bool v0 = c0 < n1, v1 = c0 + 1 < n1;
  // n2 <= L/2: a column occupies registers m < E/2 (the rest is the zero padding of the embedding),
  // and of the results only those registers are needed
  constexpr int EH = E / 2;
  R zr[E], zi[E];
  // element offsets fit in 32 bits (n1 * n2 < 2^23); the base pointers are kernel arguments
  static_for<0, E>([&](auto m) {
    const int row = t + T * m;
    const unsigned p = (unsigned)row * (unsigned)n1 + (unsigned)c0;
    if constexpr (decltype(m)::value < EH) {
      zr[m] = (R)load_or_zero(x, p, (row < n2) & v0);
      zi[m] = (R)load_or_zero(x, p + 1u, (row < n2) & v1);
    } else {
      zr[m] = R(0);
      zi[m] = R(0);
    }
  });
  using R2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
  R em0[EH], em1[EH];
  if constexpr (YCfg<R, L>::PREFETCH) {
    R lr[E], li[E];
    static_for<0, E>([&](auto m) {
      const int k = t + T * m;
      lr[m] = mu[2 * k];
      li[m] = mu[2 * k + 1];
    });
    if (skipv) return;
    fft<L, -1, true>(zr, zi, lds, tw, t);
    symbol_both_regs<L, P>(zr, zi, zs, lr, li, t);
    R2 e0[EH], e1[EH];
    static_for<0, EH>([&](auto m) {
      const int row = t + T * m;
      const unsigned p = (unsigned)row * (unsigned)n1 + (unsigned)c0;
      e0[m] = R2{};
      e1[m] = R2{};
      if (row < n2 && v0) e0[m] = *reinterpret_cast<const R2*>(epm + 2 * p);
      if (row < n2 && v1) e1[m] = *reinterpret_cast<const R2*>(epm + 2 * p + 2);
    });
    fft<L, +1>(zr, zi, lds, tw, t);  // T a + i T b along the columns
    R pr[E], pi[E];
    unstash<L, P>(pr, pi, zs, t);
    static_for<0, EH>([&](auto m) {
      const int row = t + T * m;
      zs[row] = e0[m].x * zr[m];
      zs[L + row] = e1[m].x * zi[m];
      em0[m] = e0[m].y;
      em1[m] = e1[m].y;
    });
    fft<L, +1>(pr, pi, lds, tw, t);  // T^T a + i T^T b
    y_store<L, EH, T>(n1, n2, c0, v0, v1, t, zs, em0, em1, pr, pi, ay);
    return;
  }
  if (skipv) return;
  fft<L, -1, true>(zr, zi, lds, tw, t);
  symbol_both<L, P>(zr, zi, zs, mu, t);
  fft<L, +1>(zr, zi, lds, tw, t);  // T a + i T b along the columns
  R pr[E], pi[E];
  unstash<L, P>(pr, pi, zs, t);
  // (e+, e-) of both columns in one read: e+ weights the first product now, e- waits in registers
  chunked_for<EH, kEpiGroup>([&](auto m) {
    const int row = t + T * m;
    const unsigned p = (unsigned)row * (unsigned)n1 + (unsigned)c0;
    R2 e0{}, e1{};
    if (row < n2 && v0) e0 = *reinterpret_cast<const R2*>(epm + 2 * p);
    if (row < n2 && v1) e1 = *reinterpret_cast<const R2*>(epm + 2 * p + 2);
    zs[row] = e0.x * zr[m];
    zs[L + row] = e1.x * zi[m];
    em0[m] = e0.y;
    em1[m] = e1.y;
  });
  fft<L, +1>(pr, pi, lds, tw, t);  // T^T a + i T^T b
  y_store<L, EH, T>(n1, n2, c0, v0, v1, t, zs, em0, em1, pr, pi, ay);
}

template <typename R, typename Tin, int L>
static hipError_t launch_y(const OpView<R>& op, const Tin* x, R* ay, const int* skip, hipStream_t st) {
  constexpr int S = YCfg<R, L>::S;
  const int nstrips = ceil_div(op.n1, 2 * S);
  const int grid = 8 * ceil_div(nstrips, 8);
  // batched launches (grid z over a slot table) run their own instantiation; the plain one carries
  // no table lookup
  if (batch_ztab())
    hipLaunchKernelGGL((toep_y_kernel<R, Tin, L, true>), dim3(grid, 1, batch_nz()), dim3(YCfg<R, L>::THREADS), 0, st,
                       op.n1, op.n2, x, op.epm, op.mu_y, op.tw_y, ay, nstrips, skip, batch_ztab());
  else
    hipLaunchKernelGGL((toep_y_kernel<R, Tin, L, false>), dim3(grid, 1, 1), dim3(YCfg<R, L>::THREADS), 0, st, op.n1,
                       op.n2, x, op.epm, op.mu_y, op.tw_y, ay, nstrips, skip, nullptr);
  return hipGetLastError();
}

template <typename R, typename Tin, int L, int MODE>
static hipError_t launch_x_mode(const OpView<R>& op, const Tin* x, const R* ay, R* out, const R* b,
                                const SrcTerms& src, double tau, const int* skip, hipStream_t st) {
  const int grid = ceil_div(op.n2, 2 * XCfg<R, L>::S);
  if (batch_ztab()) {
    // the epilogues of a restart cycle (the right-hand side is assembled per instance)
    if constexpr (MODE == EP_APPLY || MODE == EP_RESID || MODE == EP_JACOBI)
      hipLaunchKernelGGL((toep_x_kernel<R, Tin, L, MODE, true>), dim3(grid, 1, batch_nz()), dim3((XCfg<R, L>::THREADS)),
                         0, st, op.n1, op.n2, x, op.dpm, op.mu_x, op.tw_x, ay, b, op.dinv, src, tau, out, skip,
                         batch_ztab());
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((toep_x_kernel<R, Tin, L, MODE, false>), dim3(grid, 1, 1), dim3((XCfg<R, L>::THREADS)), 0, st,
                       op.n1, op.n2, x, op.dpm, op.mu_x, op.tw_x, ay, b, op.dinv, src, tau, out, skip, nullptr);
  }
  return hipGetLastError();
}

// The (precision, input, epilogue) combinations the solver uses.
template <typename R, typename Tin>
struct ModeSet {
  static constexpr bool ok(int m) {
    if (sizeof(R) == 8 && sizeof(Tin) == 8) return true;
    if (sizeof(R) == 8) return m == EP_APPLY;
    return m == EP_APPLY || m == EP_RESID || m == EP_JACOBI;
  }
};

template <typename R, typename Tin, int L>
static hipError_t launch_x(const OpView<R>& op, const Tin* x, const R* ay, R* out, int mode,
                           const R* b, const SrcTerms& src, double tau, const int* skip,
                           hipStream_t st) {
  switch (mode) {
#define M_(MM)                                                                                   \
  case MM:                                                                                       \
    if constexpr (ModeSet<R, Tin>::ok(MM))                                                       \
      return launch_x_mode<R, Tin, L, MM>(op, x, ay, out, b, src, tau, skip, st);                \
    else                                                                                         \
      return hipErrorInvalidValue;
    M_(EP_APPLY) M_(EP_RESID) M_(EP_JACOBI) M_(EP_RHS) M_(EP_LOUT)
#undef M_
    default:
      return hipErrorInvalidValue;
  }
}


bool fft_length_supported(int L) {
  switch (L) {
#define C_(LL) case LL:
    FDE_L_CASES(C_)
#undef C_
    return true;
    default:
      return false;
  }
}

template <typename R, typename Tin>
hipError_t launch_op_y(const OpView<R>& op, const Tin* x, R* ay, const int* skip, hipStream_t st) {
  if (!x || !ay || !op.epm || !op.mu_y || !op.tw_y || op.L2 != fft_len(op.n2)) return hipErrorInvalidValue;
  switch (op.L2) {
#define C_(LL) \
  case LL:     \
    return launch_y<R, Tin, LL>(op, x, ay, skip, st);
    FDE_L_CASES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R, typename Tin>
hipError_t launch_op_x(const OpView<R>& op, const Tin* x, const R* ay, R* out, int mode, const R* b,
                       const SrcTerms* src, double tau, const int* skip, hipStream_t st) {
  if (!x || !out || !op.dpm || !op.mu_x || !op.tw_x || op.L1 != fft_len(op.n1)) return hipErrorInvalidValue;
  if ((mode == EP_RESID || mode == EP_JACOBI) && !b) return hipErrorInvalidValue;
  if (mode == EP_JACOBI && !op.dinv) return hipErrorInvalidValue;
  SrcTerms s{};
  if (src) s = *src;
  switch (op.L1) {
#define C_(LL) \
  case LL:     \
    return launch_x<R, Tin, LL>(op, x, ay, out, mode, b, s, tau, skip, st);
    FDE_L_CASES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R, typename Tin>
hipError_t launch_operator(const OpView<R>& op, const Tin* x, R* ay, R* out, int mode, const R* b,
                           const SrcTerms* src, double tau, const int* skip, hipStream_t st) {
  hipError_t e = launch_op_y<R, Tin>(op, x, ay, skip, st);
  if (e != hipSuccess) return e;
  return launch_op_x<R, Tin>(op, x, ay, out, mode, b, src, tau, skip, st);
}

#define FDE_INST_OP(R, Tin)                                                                          \
  template hipError_t launch_op_y<R, Tin>(const OpView<R>&, const Tin*, R*, const int*, hipStream_t); \
  template hipError_t launch_op_x<R, Tin>(const OpView<R>&, const Tin*, const R*, R*, int, const R*, \
                                          const SrcTerms*, double, const int*, hipStream_t);
FDE_INST_OP(double, double)
FDE_INST_OP(double, float)
FDE_INST_OP(float, float)

template hipError_t launch_operator<double, double>(const OpView<double>&, const double*, double*,
                                                    double*, int, const double*, const SrcTerms*,
                                                    double, const int*, hipStream_t);
template hipError_t launch_operator<double, float>(const OpView<double>&, const float*, double*,
                                                   double*, int, const double*, const SrcTerms*,
                                                   double, const int*, hipStream_t);
template hipError_t launch_operator<float, float>(const OpView<float>&, const float*, float*, float*,
                                                  int, const float*, const SrcTerms*, double,
                                                  const int*, hipStream_t);

// ---- direct operator for small levels ------------------------------------------------------------
// One workgroup per output row j, one thread per column i (n1 <= blockDim):
//   row part:    sum_k swx[i-k+1] x[j][k] (left) and sum_k swx[k-i+1] x[j][k] (right), x[j][:] in LDS;
//   column part: sum_k swy[j-k+1] x[k][i] and sum_k swy[k-j+1] x[k][i], rows k read coalesced (the
//                whole field is cache resident at these sizes).
// The weight tables are stored zero-extended (w[m] for m >= 0, 0 for m < 0) so every term is
// branch-free.  swx, swy: sx*w_k and sy*w_k, k = 0..n.
template <typename R, typename Tin, int MODE>
__global__ __launch_bounds__(512) void direct_op_kernel(int n1, int n2, const Tin* __restrict__ x,
                                                        const R* __restrict__ dpm, const R* __restrict__ epm,
                                                        const R* __restrict__ swx, const R* __restrict__ swy,
                                                        const R* __restrict__ b, const R* __restrict__ dinv,
                                                        SrcTerms src, double tau, R* __restrict__ out,
                                                        const int* __restrict__ skip, const long long* __restrict__ ztab) {
  FDE_ZBEGIN;
  FDE_ZSHIFT(x);
  FDE_ZSHIFT(dpm);
  FDE_ZSHIFT(epm);
  FDE_ZSHIFT(swx);
  FDE_ZSHIFT(swy);
  FDE_ZSHIFT(b);
  FDE_ZSHIFT(dinv);
  FDE_ZSHIFT(out);
  FDE_ZSHIFT(skip);
  if (skip && *skip) return;
  extern __shared__ unsigned char smem_raw[];
  R* xr = reinterpret_cast<R*>(smem_raw);  // n1
  R* wx = xr + n1;                          // 2 n1 + 2: wx[n1 + m] = swx[m] (m >= 0), 0 below
  R* wy = wx + 2 * n1 + 2;                  // 2 n2 + 2
  const int j = blockIdx.x;
  const int i = threadIdx.x;
  const Tin* xrow = x + (size_t)j * n1;
  for (int k = threadIdx.x; k < n1; k += blockDim.x) xr[k] = (R)xrow[k];
  for (int m = threadIdx.x; m < 2 * n1 + 2; m += blockDim.x) wx[m] = m >= n1 && m - n1 <= n1 ? swx[m - n1] : R(0);
  for (int m = threadIdx.x; m < 2 * n2 + 2; m += blockDim.x) wy[m] = m >= n2 && m - n2 <= n2 ? swy[m - n2] : R(0);
  __syncthreads();
  if (i >= n1) return;
  R lx = 0, rx = 0, ly = 0, ry = 0;
  const R* wl = wx + n1 + i + 1;  // wl[-k] = swx[i-k+1]
  const R* wr = wx + n1 - i + 1;  // wr[k]  = swx[k-i+1]
#pragma unroll 4
  for (int k = 0; k < n1; ++k) {
    const R v = xr[k];
    lx += wl[-k] * v;
    rx += wr[k] * v;
  }
  const R* vl = wy + n2 + j + 1;
  const R* vr = wy + n2 - j + 1;
  const Tin* xc = x + i;
  // column values are independent loads: fetch 16 at a time so their latencies overlap
  constexpr int CH = 16;
  int k0 = 0;
  for (; k0 + CH <= n2; k0 += CH) {
    R v[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = (R)xc[(size_t)(k0 + c) * n1];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      ly += vl[-(k0 + c)] * v[c];
      ry += vr[k0 + c] * v[c];
    }
  }
  for (int k = k0; k < n2; ++k) {
    const R v = (R)xc[(size_t)k * n1];
    ly += vl[-k] * v;
    ry += vr[k] * v;
  }
  const size_t p = (size_t)j * n1 + i;
  const R l = dpm[2 * p] * lx + dpm[2 * p + 1] * rx + epm[2 * p] * ly + epm[2 * p + 1] * ry;
  R bv = R(0), dv = R(0);
  double sv = 0.0;
  if constexpr (MODE == EP_RESID || MODE == EP_JACOBI) bv = b[p];
  if constexpr (MODE == EP_JACOBI) dv = dinv[p];
  if constexpr (MODE == EP_RHS) {
    for (int k = 0; k < src.n; ++k) sv += src.phi[k] * src.S[k][p];
  }
  out[p] = epilogue_value<MODE, R, Tin>(l, xr[i], bv, dv, sv, tau);
}

template <typename R, typename Tin>
hipError_t launch_direct_op(int n1, int n2, const Tin* x, const R* dpm, const R* epm, const R* swx, const R* swy,
                            R* out, int mode, const R* b, const R* dinv, const SrcTerms* src, double tau,
                            const int* skip, hipStream_t st) {
  if (n1 > 512 || n1 < 1 || n2 < 1 || !x || !dpm || !epm || !swx || !swy || !out) return hipErrorInvalidValue;
  if ((mode == EP_RESID || mode == EP_JACOBI) && !b) return hipErrorInvalidValue;
  if (mode == EP_JACOBI && !dinv) return hipErrorInvalidValue;
  SrcTerms s{};
  if (src) s = *src;
  const int threads = ((n1 + 63) / 64) * 64;
  const size_t bytes = (size_t)(n1 + 2 * n1 + 2 + 2 * n2 + 2) * sizeof(R);
  switch (mode) {
#define M_(MM)                                                                                                  \
  case MM:                                                                                                      \
    if constexpr (ModeSet<R, Tin>::ok(MM)) {                                                                    \
      hipLaunchKernelGGL((direct_op_kernel<R, Tin, MM>), dim3(n2, 1, batch_nz()), dim3(threads), bytes, st, n1, n2, \
                         x, dpm, epm, swx, swy, b, dinv, s, tau, out, skip, batch_ztab());                      \
      return hipGetLastError();                                                                                 \
    } else {                                                                                                    \
      return hipErrorInvalidValue;                                                                              \
    }
    M_(EP_APPLY) M_(EP_RESID) M_(EP_JACOBI) M_(EP_RHS) M_(EP_LOUT)
#undef M_
    default:
      return hipErrorInvalidValue;
  }
}
template hipError_t launch_direct_op<double, double>(int, int, const double*, const double*, const double*,
                                                     const double*, const double*, double*, int, const double*,
                                                     const double*, const SrcTerms*, double, const int*,
                                                     hipStream_t);
template hipError_t launch_direct_op<double, float>(int, int, const float*, const double*, const double*,
                                                    const double*, const double*, double*, int, const double*,
                                                    const double*, const SrcTerms*, double, const int*,
                                                    hipStream_t);
template hipError_t launch_direct_op<float, float>(int, int, const float*, const float*, const float*,
                                                   const float*, const float*, float*, int, const float*,
                                                   const float*, const SrcTerms*, double, const int*, hipStream_t);

// ---- host side: twiddle tables and symbols ---------------------------------------------------
int fft_twiddle_count(int L, int) { return L; }

// exp(-2 pi i k / M) accurate to the last bit via long double
static void unit_root(long long k, long long M, double* re, double* im) {
  const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)M;
  *re = (double)cosl(a);
  *im = (double)sinl(a);
}

// The twiddle table of every transform plan of length L: exp(-2 pi i k/L), k < L/2.
void fft_twiddles(int L, int, double* out, int* count) {
  for (int k = 0; k < L / 2; ++k) unit_root(k, L, &out[2 * k], &out[2 * k + 1]);
  if (count) *count = L;
}

// In-place radix-2 DFT (forward, sign -1) of length L (power of two), host side.
static void host_fft(std::vector<std::complex<double>>& a) {
  const int n = (int)a.size();
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < len / 2; ++k) {
        double wr, wi;
        unit_root(k, len, &wr, &wi);
        const std::complex<double> w(wr, wi);
        const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

void toeplitz_symbol(const double* w, int n, int L, double scale, double* out) {
  std::vector<std::complex<double>> c(L, 0.0);
  for (int m = 0; m < n; ++m) c[m] = w[m + 1];  // t_m = w_{m+1}, m = 0..n-1
  c[L - 1] = w[0];                              // t_{-1} = w_0
  host_fft(c);
  const double f = scale / L;  // the inverse transforms are unnormalised
  for (int k = 0; k < L; ++k) {
    out[2 * k] = f * c[k].real();
    out[2 * k + 1] = f * c[k].imag();
  }
}

}  // namespace fde
