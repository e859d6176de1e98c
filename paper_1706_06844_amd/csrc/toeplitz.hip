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

namespace fde {

// (zr, zi) <- lam .* Z  and  (pr, pi) <- conj(lam) .* Z, lam the scaled symbol.
template <int L, typename R>
__device__ __forceinline__ void symbol_multiply(Reg<R, L>& zr, Reg<R, L>& zi, Reg<R, L>& pr,
                                                Reg<R, L>& pi,
                                                const R* __restrict__ lam, int t) {
  constexpr int E = PlanFor<R, L>::E, T = PlanFor<R, L>::T;
  static_for<0, E>([&](auto m) {
    const int k = t + T * m;
    const R lr = lam[2 * k], li = lam[2 * k + 1];
    const R a = zr[m], b = zi[m];
    zr[m] = lr * a - li * b;
    zi[m] = lr * b + li * a;
    pr[m] = lr * a + li * b;
    pi[m] = lr * b - li * a;
  });
}

template <typename R, typename Tin>
__device__ __forceinline__ void epilogue_point(size_t p, R lx, const Tin* x, const R* __restrict__ ay,
                                               const R* __restrict__ b, const R* __restrict__ dinv,
                                               int mode, const SrcTerms& src, double tau, R* out) {
  R l = lx;
  if (ay) l += ay[p];
  R v;
  if (mode == EP_LOUT) {
    v = l;
  } else {
    const R xv = (R)x[p];
    if (mode == EP_APPLY) {
      v = xv - l;
    } else if (mode == EP_RESID) {
      v = b[p] - xv + l;
    } else if (mode == EP_JACOBI) {
      v = xv + dinv[p] * (b[p] - xv + l);
    } else {  // EP_RHS
      double s = 0.0;
      for (int k = 0; k < src.n; ++k) s += src.phi[k] * src.S[k][p];
      v = xv + l + (R)(tau * s);
    }
  }
  out[p] = v;
}

template <typename R, typename Tin, int L>
__global__ __launch_bounds__((PlanFor<R, L>::T), 2) void toep_x_kernel(
    int n1, int n2, const Tin* x, const R* __restrict__ dpm, const R* __restrict__ mu,
    const R* __restrict__ tw, const R* __restrict__ ay, const R* __restrict__ b,
    const R* __restrict__ dinv, int mode, SrcTerms src, double tau, R* out,
    const int* __restrict__ skip) {
  if (skip && *skip) return;
  using P = PlanFor<R, L>;
  constexpr int E = P::E, T = P::T;
  __shared__ R lds[lds_len(L)];
  const int t = threadIdx.x;
  const int rowA = 2 * blockIdx.x;
  const int rowB = rowA + 1;
  const bool hasB = rowB < n2;
  const Tin* xa = x + (size_t)rowA * n1;
  const Tin* xb = x + (size_t)rowB * n1;
  R zr[E], zi[E], pr[E], pi[E];
  static_for<0, E>([&](auto m) {
    const int i = t + T * m;
    zr[m] = i < n1 ? (R)xa[i] : R(0);
    zi[m] = (hasB && i < n1) ? (R)xb[i] : R(0);
  });
  fft<L, -1>(zr, zi, lds, tw, t);
  symbol_multiply<L>(zr, zi, pr, pi, mu, t);
  fft<L, +1>(zr, zi, lds, tw, t);  // real part: T xa, imaginary part: T xb
  static_for<0, E>([&](auto m) {
    const int i = t + T * m;
    const size_t pa = (size_t)rowA * n1 + i, pb = (size_t)rowB * n1 + i;
    zr[m] = i < n1 ? dpm[2 * pa] * zr[m] : R(0);
    zi[m] = (hasB && i < n1) ? dpm[2 * pb] * zi[m] : R(0);
  });
  fft<L, +1>(pr, pi, lds, tw, t);  // real part: T^T xa, imaginary part: T^T xb
  static_for<0, E>([&](auto m) {
    const int i = t + T * m;
    if (i < n1) {
      const size_t pa = (size_t)rowA * n1 + i;
      epilogue_point<R, Tin>(pa, zr[m] + dpm[2 * pa + 1] * pr[m], x, ay, b, dinv, mode, src, tau, out);
      if (hasB) {
        const size_t pb = (size_t)rowB * n1 + i;
        epilogue_point<R, Tin>(pb, zi[m] + dpm[2 * pb + 1] * pi[m], x, ay, b, dinv, mode, src, tau, out);
      }
    }
  });
}

// Slots (transforms) per workgroup of the column pass.
template <typename R, int L>
struct YCfg {
  static constexpr int S0 = sizeof(R) == 8 ? 2 : 4;
  static constexpr int S = PlanFor<R, L>::T * S0 <= 512 ? S0 : (PlanFor<R, L>::T >= 512 ? 1 : 512 / PlanFor<R, L>::T);
  static constexpr int THREADS = PlanFor<R, L>::T * S;
};

template <typename R, typename Tin, int L>
__global__ __launch_bounds__((YCfg<R, L>::THREADS), 2) void toep_y_kernel(
    int n1, int n2, const Tin* __restrict__ x, const R* __restrict__ epm, const R* __restrict__ mu,
    const R* __restrict__ tw, R* __restrict__ ay, int nstrips, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using P = PlanFor<R, L>;
  constexpr int E = P::E, T = P::T, S = YCfg<R, L>::S;
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous range of strips so
  // that neighbouring strips (which share cache lines) meet in the same L2.
  const int per = gridDim.x / 8;
  const int strip = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (strip >= nstrips) return;
  __shared__ R lds_all[S * lds_len(L)];
  const int slot = threadIdx.x % S;
  const int t = threadIdx.x / S;
  R* lds = lds_all + slot * lds_len(L);
  const int c0 = strip * 2 * S + 2 * slot;
  const bool v0 = c0 < n1, v1 = c0 + 1 < n1;
  R zr[E], zi[E], pr[E], pi[E];
  static_for<0, E>([&](auto m) {
    const int row = t + T * m;
    const size_t p = (size_t)row * n1 + c0;
    zr[m] = (row < n2 && v0) ? (R)x[p] : R(0);
    zi[m] = (row < n2 && v1) ? (R)x[p + 1] : R(0);
  });
  fft<L, -1>(zr, zi, lds, tw, t);
  symbol_multiply<L>(zr, zi, pr, pi, mu, t);
  fft<L, +1>(zr, zi, lds, tw, t);  // T a + i T b along the columns
  static_for<0, E>([&](auto m) {
    const int row = t + T * m;
    const size_t p = (size_t)row * n1 + c0;
    zr[m] = (row < n2 && v0) ? epm[2 * p] * zr[m] : R(0);
    zi[m] = (row < n2 && v1) ? epm[2 * p + 2] * zi[m] : R(0);
  });
  fft<L, +1>(pr, pi, lds, tw, t);  // T^T a + i T^T b
  static_for<0, E>([&](auto m) {
    const int row = t + T * m;
    if (row < n2) {
      const size_t p = (size_t)row * n1 + c0;
      if (v0) ay[p] = zr[m] + epm[2 * p + 1] * pr[m];
      if (v1) ay[p + 1] = zi[m] + epm[2 * p + 3] * pi[m];
    }
  });
}

template <typename R, typename Tin, int L>
static hipError_t launch_y(const OpView<R>& op, const Tin* x, R* ay, const int* skip, hipStream_t st) {
  constexpr int S = YCfg<R, L>::S;
  const int nstrips = ceil_div(op.n1, 2 * S);
  const int grid = 8 * ceil_div(nstrips, 8);
  hipLaunchKernelGGL((toep_y_kernel<R, Tin, L>), dim3(grid), dim3(YCfg<R, L>::THREADS), 0, st, op.n1,
                     op.n2, x, op.epm, op.mu_y, op.tw_y, ay, nstrips, skip);
  return hipGetLastError();
}

template <typename R, typename Tin, int L>
static hipError_t launch_x(const OpView<R>& op, const Tin* x, const R* ay, R* out, int mode,
                           const R* b, const SrcTerms& src, double tau, const int* skip,
                           hipStream_t st) {
  const int grid = ceil_div(op.n2, 2);
  hipLaunchKernelGGL((toep_x_kernel<R, Tin, L>), dim3(grid), dim3((PlanFor<R, L>::T)), 0, st, op.n1, op.n2, x,
                     op.dpm, op.mu_x, op.tw_x, ay, b, op.dinv, mode, src, tau, out, skip);
  return hipGetLastError();
}

#define FDE_L_CASES(MACRO) \
  MACRO(16) MACRO(32) MACRO(64) MACRO(128) MACRO(256) MACRO(512) MACRO(1024) MACRO(2048) MACRO(4096)

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

// ---- host side: twiddle tables and symbols ---------------------------------------------------
struct RtPlan {
  int E, T, nst;
  int radix[16], ns[16];
};
static RtPlan rt_plan(int L, int emax) {
  RtPlan p{};
  p.E = L >= 64 * emax ? emax : (L >= 128 ? L / 64 : 2);
  p.T = L / p.E;
  int logL = 0, logE = 0;
  while ((1 << logL) < L) ++logL;
  while ((1 << logE) < p.E) ++logE;
  p.nst = (logL + logE - 1) / logE;
  int ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    p.radix[s] = (s < p.nst - 1 || logL % logE == 0) ? p.E : (1 << (logL % logE));
    p.ns[s] = ns;
    ns *= p.radix[s];
  }
  return p;
}

int fft_twiddle_count(int L, int elem_bytes) {
  RtPlan p = rt_plan(L, elem_bytes == 8 ? 8 : 16);
  int c = 0;
  for (int s = 1; s < p.nst; ++s) c += p.ns[s] * (p.radix[s] - 1);
  return 2 * c;
}

// exp(-2 pi i k / M) accurate to the last bit via long double
static void unit_root(long long k, long long M, double* re, double* im) {
  const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)M;
  *re = (double)cosl(a);
  *im = (double)sinl(a);
}

void fft_twiddles(int L, int elem_bytes, double* out, int* count) {
  RtPlan p = rt_plan(L, elem_bytes == 8 ? 8 : 16);
  int o = 0;
  for (int s = 1; s < p.nst; ++s) {
    const int R = p.radix[s], NS = p.ns[s];
    for (int j = 0; j < NS; ++j)
      for (int r = 1; r < R; ++r) {
        unit_root((long long)r * j, (long long)NS * R, &out[o], &out[o + 1]);
        o += 2;
      }
  }
  if (count) *count = o;
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
