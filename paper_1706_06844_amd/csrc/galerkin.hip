// Galerkin coarse operators (paper Sec. 4.2, the variant built as A_l = R A_{l-1} P with R = P^T/4)
// applied in factored form, never assembled (the paper notes that the explicit Galerkin matrices of
// this problem are too expensive to form).
//
// With the composite bilinear interpolation P^ = P^_y (x) P^_x from level l to the fine grid -- hat
// functions of half-width H = 2^l around the coarse points c_I = H(I+1) - 1 (0-based) --
//   A_l x = 4^-l [ (M_y (x) M_x) x - tau/2 P^T L_0 P^ x ],      M = P^T P^ (tridiagonal),
// and the x part of tau/2 P^T L_0 P^ x at the coarse point (J, I) is
//   sum_i hat_I(i) sum_{D=-1,0,1} ( c+_D[J,i] (T u_{J+D})[i] + c-_D[J,i] (T^T u_{J+D})[i] ),
//   u_J' = P^_x x[J', :]              (coarse row J' interpolated to the fine x grid),
//   c+-_D[J, i] = sum_j hat_J(j) hat_{J+D}(j) d+-[j, i]     (coarse rows x fine columns),
// with T the fine-grid Toeplitz factor scaled by tau/(2 h_x^alpha).  The y part is the same with e+-,
// the y factor and columns.  Because hat_J hat_{J+D} vanishes for |D| > 1, only three neighbouring
// coarse rows meet; c_{-1}[J] = c_{+1}[J-1], so c_0 and c_{+1} are stored.
//
// One application: gal_row_kernel (one fine-length transform pair per pair of coarse rows) writes
// V[J'][i] = ((T u_J')[i], (T^T u_J')[i]); gal_col_kernel does the same over coarse columns into W;
// gal_combine_kernel forms the sums above, the mass term and the epilogue.
#include <cmath>
#include <vector>

#include "common.h"
#include "fft.h"
#include "toep_dev.h"

namespace fde {

// Value at fine index i of the coarse vector x (stride `stride`, nl entries) interpolated with the
// composite hats of half-width H = 2^logH.  Coarse point I sits at fine index H(I+1) - 1; outside
// the coarse range the vector is zero (homogeneous Dirichlet data).
template <typename R>
__device__ __forceinline__ R interp(const R* x, int stride, int nl, int i, int logH) {
  const int q = i + 1;
  const int I0 = (q >> logH) - 1;
  const int r = q & ((1 << logH) - 1);
  const R f = (R)r / (R)(1 << logH);  // exact: H is a power of two
  const R a = I0 >= 0 ? x[(size_t)I0 * stride] : R(0);
  const R b = (r != 0 && I0 + 1 < nl) ? x[(size_t)(I0 + 1) * stride] : R(0);
  return (R(1) - f) * a + f * b;
}

template <typename R>
__device__ __forceinline__ void store_pair(R* p, R a, R b) {
  if constexpr (sizeof(R) == 4) *reinterpret_cast<float2*>(p) = make_float2(a, b);
  else *reinterpret_cast<double2*>(p) = make_double2(a, b);
}

// Pairs of coarse rows, interpolated to the fine x grid, through the Toeplitz factor and its
// transpose: V[J'][i] = ((T u_J')[i], (T^T u_J')[i]), fine length n0.
template <typename R, int L>
__global__ __launch_bounds__((XCfg<R, L>::THREADS), FDE_XW) void gal_row_kernel(
    int n0, int nl, int nrows, int logH, const R* __restrict__ x, const R* __restrict__ mu,
    const R* __restrict__ twtab, R* __restrict__ V, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using P = PlanFor<R, L>;
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
  const bool hasA = rowA < nrows, hasB = rowA + 1 < nrows;
  const R* xa = x + (size_t)rowA * nl;
  const R* xb = xa + nl;
  R zr[E], zi[E];
  static_for<0, E>([&](auto m) {
    const int i = t + T * m;
    zr[m] = (hasA && i < n0) ? interp(xa, 1, nl, i, logH) : R(0);
    zi[m] = (hasB && i < n0) ? interp(xb, 1, nl, i, logH) : R(0);
  });
  fft<L, -1>(zr, zi, lds, tw, t);
  symbol_both<L, P>(zr, zi, zs, mu, t);
  fft<L, +1>(zr, zi, lds, tw, t);  // T u_A + i T u_B
  R pr[E], pi[E];
  unstash<L, P>(pr, pi, zs, t);
  static_for<0, E>([&](auto m) {  // the first products wait in LDS during the second transform
    const int i = t + T * m;
    zs[i] = zr[m];
    zs[L + i] = zi[m];
  });
  fft<L, +1>(pr, pi, lds, tw, t);  // T^T u_A + i T^T u_B
  static_for<0, E>([&](auto m) {
    const int i = t + T * m;
    if (i < n0) {
      if (hasA) store_pair(V + 2 * ((size_t)rowA * n0 + i), zs[i], pr[m]);
      if (hasB) store_pair(V + 2 * ((size_t)(rowA + 1) * n0 + i), zs[L + i], pi[m]);
    }
  });
}

// Pairs of coarse columns, interpolated to the fine y grid, through the y factor and its transpose:
// W[j][I'] = ((T w_I')[j], (T^T w_I')[j]), fine length n0 in y, nlx coarse columns.
template <typename R, int L>
__global__ __launch_bounds__((YCfg<R, L>::THREADS), FDE_YW) void gal_col_kernel(
    int n0, int nly, int nlx, int logH, const R* __restrict__ x, const R* __restrict__ mu,
    const R* __restrict__ twtab, R* __restrict__ W, int nstrips, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using P = PlanFor<R, L>;
  constexpr int E = P::E, T = P::T, S = YCfg<R, L>::S;
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
  const bool v0 = c0 < nlx, v1 = c0 + 1 < nlx;
  R zr[E], zi[E];
  static_for<0, E>([&](auto m) {
    const int j = t + T * m;
    zr[m] = (j < n0 && v0) ? interp(x + c0, nlx, nly, j, logH) : R(0);
    zi[m] = (j < n0 && v1) ? interp(x + c0 + 1, nlx, nly, j, logH) : R(0);
  });
  fft<L, -1>(zr, zi, lds, tw, t);
  symbol_both<L, P>(zr, zi, zs, mu, t);
  fft<L, +1>(zr, zi, lds, tw, t);
  R pr[E], pi[E];
  unstash<L, P>(pr, pi, zs, t);
  static_for<0, E>([&](auto m) {
    const int j = t + T * m;
    zs[j] = zr[m];
    zs[L + j] = zi[m];
  });
  fft<L, +1>(pr, pi, lds, tw, t);
  static_for<0, E>([&](auto m) {
    const int j = t + T * m;
    if (j < n0) {
      if (v0) store_pair(W + 2 * ((size_t)j * nlx + c0), zs[j], pr[m]);
      if (v1) store_pair(W + 2 * ((size_t)j * nlx + c0 + 1), zs[L + j], pi[m]);
    }
  });
}

// The sums of the factored form, the mass term and the epilogue, one workgroup per coarse row J.
// Phase 1 collapses the three row couplings at every fine x point into LDS; phase 2 weights them with
// the hat of each coarse column and adds the y part, which it reads along fine rows j of the hat of J.
template <typename R, int MODE>
__global__ __launch_bounds__(512) void gal_combine_kernel(GalView<R> g, const R* __restrict__ x,
                                                          const R* __restrict__ b, R* __restrict__ out,
                                                          const int* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ unsigned char smem_raw[];
  R* gx = reinterpret_cast<R*>(smem_raw);
  const int J = blockIdx.x;
  const int n0x = g.n0x, nlx = g.nlx, nly = g.nly, H = 1 << g.logH;
  for (int i = threadIdx.x; i < n0x; i += blockDim.x) {
    const size_t o = (size_t)J * n0x + i;
    R acc = g.cx0[2 * o] * g.V[2 * o] + g.cx0[2 * o + 1] * g.V[2 * o + 1];
    if (J > 0) {
      const size_t om = o - n0x;
      acc += g.cx1[2 * om] * g.V[2 * om] + g.cx1[2 * om + 1] * g.V[2 * om + 1];
    }
    if (J + 1 < nly) {
      const size_t op = o + n0x;
      acc += g.cx1[2 * o] * g.V[2 * op] + g.cx1[2 * o + 1] * g.V[2 * op + 1];
    }
    gx[i] = acc;
  }
  __syncthreads();
  const R rH = R(1) / R(H);
  const int cJ = H * (J + 1) - 1;
  for (int I = threadIdx.x; I < nlx; I += blockDim.x) {
    const int cI = H * (I + 1) - 1;
    R X = gx[cI];
    for (int d = 1; d < H; ++d) X += (R(1) - R(d) * rH) * (gx[cI - d] + gx[cI + d]);
    R Y = R(0);
    for (int d = -H + 1; d < H; ++d) {
      const R w = R(1) - R(d < 0 ? -d : d) * rH;
      const size_t o = (size_t)(cJ + d) * nlx + I;
      R acc = g.ey0[2 * o] * g.W[2 * o] + g.ey0[2 * o + 1] * g.W[2 * o + 1];
      if (I > 0) acc += g.ey1[2 * (o - 1)] * g.W[2 * (o - 1)] + g.ey1[2 * (o - 1) + 1] * g.W[2 * (o - 1) + 1];
      if (I + 1 < nlx) acc += g.ey1[2 * o] * g.W[2 * (o + 1)] + g.ey1[2 * o + 1] * g.W[2 * (o + 1) + 1];
      Y += w * acc;
    }
    auto mrow = [&](int JJ) {
      const R* xr = x + (size_t)JJ * nlx;
      R v = R(g.m0x) * xr[I];
      if (I > 0) v += R(g.m1x) * xr[I - 1];
      if (I + 1 < nlx) v += R(g.m1x) * xr[I + 1];
      return v;
    };
    R mass = R(g.m0y) * mrow(J);
    if (J > 0) mass += R(g.m1y) * mrow(J - 1);
    if (J + 1 < nly) mass += R(g.m1y) * mrow(J + 1);
    const R ax = R(g.scale) * (mass - X - Y);
    const size_t p = (size_t)J * nlx + I;
    if constexpr (MODE == EP_APPLY) out[p] = ax;
    else if constexpr (MODE == EP_RESID) out[p] = b[p] - ax;
    else out[p] = x[p] + g.dinv[p] * (b[p] - ax);  // EP_JACOBI
  }
}

// ---- setup -------------------------------------------------------------------------------------
// c+-_0[J][i] and c+-_1[J][i] from the fine FP64 pairs (d+, d-); accumulated in FP64.
template <typename R>
__global__ void gal_cx_kernel(int n0x, int nly, int logH, const double* __restrict__ dpm, R* __restrict__ cx0,
                              R* __restrict__ cx1) {
  const int H = 1 << logH;
  const size_t total = (size_t)nly * n0x;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
    const int J = (int)(q / n0x), i = (int)(q - (size_t)J * n0x);
    const int cJ = H * (J + 1) - 1;
    double a0p = 0, a0m = 0, a1p = 0, a1m = 0;
    for (int d = -H + 1; d < H; ++d) {
      const double w = 1.0 - std::fabs((double)d) / H;
      const size_t f = (size_t)(cJ + d) * n0x + i;
      const double vp = dpm[2 * f], vm = dpm[2 * f + 1];
      a0p += w * w * vp;
      a0m += w * w * vm;
      if (d > 0 && J + 1 < nly) {
        const double w1 = (double)d / H;  // hat of coarse row J+1 at the same fine row
        a1p += w * w1 * vp;
        a1m += w * w1 * vm;
      }
    }
    cx0[2 * q] = (R)a0p;
    cx0[2 * q + 1] = (R)a0m;
    cx1[2 * q] = (R)a1p;
    cx1[2 * q + 1] = (R)a1m;
  }
}

// e+-_0[j][I] and e+-_1[j][I] from the fine FP64 pairs (e+, e-).
template <typename R>
__global__ void gal_ey_kernel(int n0x, int n0y, int nlx, int logH, const double* __restrict__ epm,
                              R* __restrict__ ey0, R* __restrict__ ey1) {
  const int H = 1 << logH;
  const size_t total = (size_t)n0y * nlx;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(q / nlx), I = (int)(q - (size_t)j * nlx);
    const int cI = H * (I + 1) - 1;
    double a0p = 0, a0m = 0, a1p = 0, a1m = 0;
    for (int d = -H + 1; d < H; ++d) {
      const double w = 1.0 - std::fabs((double)d) / H;
      const size_t f = (size_t)j * n0x + (cI + d);
      const double vp = epm[2 * f], vm = epm[2 * f + 1];
      a0p += w * w * vp;
      a0m += w * w * vm;
      if (d > 0 && I + 1 < nlx) {
        const double w1 = (double)d / H;
        a1p += w * w1 * vp;
        a1m += w * w1 * vm;
      }
    }
    ey0[2 * q] = (R)a0p;
    ey0[2 * q + 1] = (R)a0m;
    ey1[2 * q] = (R)a1p;
    ey1[2 * q + 1] = (R)a1m;
  }
}

// Diagonal of A_l.  q[k*(2H-1) + d + H - 1] = ((T hat)[d], (T^T hat)[d]) for k = 0, 1 and
// |d| < H: the factor applied to one hat, seen from the hat's own support (the same for every
// coarse point, since every hat lies inside the grid).
template <typename R>
__global__ void gal_diag_kernel(GalView<R> g, const double* __restrict__ qx, const double* __restrict__ qy,
                                double omega, R* __restrict__ dinv, double* __restrict__ dout) {
  const int H = 1 << g.logH, K = 2 * H - 1;
  const size_t total = (size_t)g.nly * g.nlx;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < total; p += (size_t)gridDim.x * blockDim.x) {
    const int J = (int)(p / g.nlx), I = (int)(p - (size_t)J * g.nlx);
    const int cI = H * (I + 1) - 1, cJ = H * (J + 1) - 1;
    double X = 0, Y = 0;
    for (int d = -H + 1; d < H; ++d) {
      const double w = 1.0 - std::fabs((double)d) / H;
      const size_t ox = (size_t)J * g.n0x + (cI + d);
      X += w * ((double)g.cx0[2 * ox] * qx[d + H - 1] + (double)g.cx0[2 * ox + 1] * qx[K + d + H - 1]);
      const size_t oy = (size_t)(cJ + d) * g.nlx + I;
      Y += w * ((double)g.ey0[2 * oy] * qy[d + H - 1] + (double)g.ey0[2 * oy + 1] * qy[K + d + H - 1]);
    }
    const double dg = g.scale * (g.m0x * g.m0y - X - Y);
    if (dinv) dinv[p] = (R)(omega / dg);
    if (dout) dout[p] = dg;
  }
}

// Dense matrix of A_l (the coarsest level), entry (p, q) with p = (J, I), q = (J', I'), in FP64.
// Qx[k][I'][i] = (T hat_I')[i] (k = 0) and (T^T hat_I')[i] (k = 1) for all fine i; Qy likewise.
template <typename R>
__global__ void gal_dense_kernel(GalView<R> g, const double* __restrict__ Qx, const double* __restrict__ Qy,
                                 double* __restrict__ A) {
  const int H = 1 << g.logH;
  const int n = g.nlx * g.nly;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int p = e / n, q = e - p * n;
    const int J = p / g.nlx, I = p - J * g.nlx, Jq = q / g.nlx, Iq = q - Jq * g.nlx;
    const int cI = H * (I + 1) - 1, cJ = H * (J + 1) - 1;
    double X = 0, Y = 0;
    const int D = Jq - J, Dp = Iq - I;
    if (D >= -1 && D <= 1) {
      const R* c = (D == 0) ? g.cx0 + (size_t)J * g.n0x * 2
                            : (D == 1 ? g.cx1 + (size_t)J * g.n0x * 2 : g.cx1 + (size_t)(J - 1) * g.n0x * 2);
      const double* qp = Qx + (size_t)Iq * g.n0x;
      const double* qm = Qx + ((size_t)g.nlx + Iq) * g.n0x;
      for (int d = -H + 1; d < H; ++d) {
        const double w = 1.0 - std::fabs((double)d) / H;
        const int i = cI + d;
        X += w * ((double)c[2 * i] * qp[i] + (double)c[2 * i + 1] * qm[i]);
      }
    }
    if (Dp >= -1 && Dp <= 1) {
      const int Ie = (Dp == -1) ? I - 1 : I;
      const R* e0 = (Dp == 0) ? g.ey0 : g.ey1;
      const double* qp = Qy + (size_t)Jq * g.n0y;
      const double* qm = Qy + ((size_t)g.nly + Jq) * g.n0y;
      for (int d = -H + 1; d < H; ++d) {
        const double w = 1.0 - std::fabs((double)d) / H;
        const int j = cJ + d;
        const size_t o = (size_t)j * g.nlx + Ie;
        Y += w * ((double)e0[2 * o] * qp[j] + (double)e0[2 * o + 1] * qm[j]);
      }
    }
    const double mx = (I == Iq) ? g.m0x : ((Dp == 1 || Dp == -1) ? g.m1x : 0.0);
    const double my = (J == Jq) ? g.m0y : ((D == 1 || D == -1) ? g.m1y : 0.0);
    A[e] = g.scale * (mx * my - X - Y);
  }
}

// ---- launchers ---------------------------------------------------------------------------------
template <typename R>
static bool gal_view_ok(const GalView<R>& g) {
  return g.cx0 && g.cx1 && g.ey0 && g.ey1 && g.nlx > 0 && g.nly > 0 && g.logH >= 1 &&
         g.n0x == (1 << g.logH) * (g.nlx + 1) - 1 && g.n0y == (1 << g.logH) * (g.nly + 1) - 1;
}

template <typename R, int L>
static hipError_t launch_gal_row_L(const GalView<R>& g, const R* x, const int* skip, hipStream_t st) {
  constexpr int S = XCfg<R, L>::S;
  const int grid = ceil_div(g.nly, 2 * S);
  hipLaunchKernelGGL((gal_row_kernel<R, L>), dim3(grid), dim3((XCfg<R, L>::THREADS)), 0, st, g.n0x, g.nlx, g.nly,
                     g.logH, x, g.mu_x, g.tw_x, g.V, skip);
  return hipGetLastError();
}

template <typename R, int L>
static hipError_t launch_gal_col_L(const GalView<R>& g, const R* x, const int* skip, hipStream_t st) {
  constexpr int S = YCfg<R, L>::S;
  const int nstrips = ceil_div(g.nlx, 2 * S);
  const int grid = 8 * ceil_div(nstrips, 8);
  hipLaunchKernelGGL((gal_col_kernel<R, L>), dim3(grid), dim3((YCfg<R, L>::THREADS)), 0, st, g.n0y, g.nly, g.nlx,
                     g.logH, x, g.mu_y, g.tw_y, g.W, nstrips, skip);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_gal_apply(const GalView<R>& g, const R* x, R* out, int mode, const R* b, const int* skip,
                            hipStream_t st) {
  if (!gal_view_ok(g) || !x || !out || !g.V || !g.W || !g.mu_x || !g.mu_y || !g.tw_x || !g.tw_y)
    return hipErrorInvalidValue;
  if (g.L0x != 2 * (g.n0x + 1) || g.L0y != 2 * (g.n0y + 1)) return hipErrorInvalidValue;
  if ((mode == EP_RESID || mode == EP_JACOBI) && !b) return hipErrorInvalidValue;
  if (mode == EP_JACOBI && (!g.dinv || out == x)) return hipErrorInvalidValue;
  if (mode != EP_APPLY && mode != EP_RESID && mode != EP_JACOBI) return hipErrorInvalidValue;
  hipError_t e = hipErrorInvalidValue;
  switch (g.L0x) {
#define C_(LL)                                    \
  case LL:                                        \
    e = launch_gal_row_L<R, LL>(g, x, skip, st); \
    break;
    FDE_L_CASES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (g.L0y) {
#define C_(LL)                                    \
  case LL:                                        \
    e = launch_gal_col_L<R, LL>(g, x, skip, st); \
    break;
    FDE_L_CASES(C_)
#undef C_
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)g.n0x * sizeof(R);
  if (mode == EP_APPLY)
    hipLaunchKernelGGL((gal_combine_kernel<R, EP_APPLY>), dim3(g.nly), dim3(512), lds, st, g, x, b, out, skip);
  else if (mode == EP_RESID)
    hipLaunchKernelGGL((gal_combine_kernel<R, EP_RESID>), dim3(g.nly), dim3(512), lds, st, g, x, b, out, skip);
  else
    hipLaunchKernelGGL((gal_combine_kernel<R, EP_JACOBI>), dim3(g.nly), dim3(512), lds, st, g, x, b, out, skip);
  return hipGetLastError();
}

static int grid_of(size_t n) {
  size_t gsz = (n + 255) / 256;
  if (gsz > 8192) gsz = 8192;
  return (int)(gsz ? gsz : 1);
}

template <typename R>
hipError_t launch_gal_setup(GalView<R>& g, const double* dpm, const double* epm, hipStream_t st) {
  if (!gal_view_ok(g) || !dpm || !epm) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gal_cx_kernel<R>), dim3(grid_of((size_t)g.nly * g.n0x)), dim3(256), 0, st, g.n0x, g.nly,
                     g.logH, dpm, const_cast<R*>(g.cx0), const_cast<R*>(g.cx1));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((gal_ey_kernel<R>), dim3(grid_of((size_t)g.n0y * g.nlx)), dim3(256), 0, st, g.n0x, g.n0y,
                     g.nlx, g.logH, epm, const_cast<R*>(g.ey0), const_cast<R*>(g.ey1));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_gal_diag(const GalView<R>& g, const double* qx, const double* qy, double omega, R* dinv,
                           double* dout, hipStream_t st) {
  if (!gal_view_ok(g) || !qx || !qy || (!dinv && !dout)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gal_diag_kernel<R>), dim3(grid_of((size_t)g.nly * g.nlx)), dim3(256), 0, st, g, qx, qy, omega,
                     dinv, dout);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_gal_dense(const GalView<R>& g, const double* Qx, const double* Qy, double* A, hipStream_t st) {
  if (!gal_view_ok(g) || !Qx || !Qy || !A) return hipErrorInvalidValue;
  const size_t n = (size_t)g.nlx * g.nly;
  hipLaunchKernelGGL((gal_dense_kernel<R>), dim3(grid_of(n * n)), dim3(256), 0, st, g, Qx, Qy, A);
  return hipGetLastError();
}

#define FDE_INST_GAL(R)                                                                                        \
  template hipError_t launch_gal_apply<R>(const GalView<R>&, const R*, R*, int, const R*, const int*,          \
                                          hipStream_t);                                                        \
  template hipError_t launch_gal_setup<R>(GalView<R>&, const double*, const double*, hipStream_t);             \
  template hipError_t launch_gal_diag<R>(const GalView<R>&, const double*, const double*, double, R*, double*, \
                                         hipStream_t);                                                         \
  template hipError_t launch_gal_dense<R>(const GalView<R>&, const double*, const double*, double*, hipStream_t);
FDE_INST_GAL(double)
FDE_INST_GAL(float)

}  // namespace fde
