// Device helpers shared by the Toeplitz operator kernels (toeplitz.hip) and the Galerkin
// coarse-operator kernels (galerkin.hip): symbol products, uniform pointers, launch shapes.
#pragma once
#include "common.h"
#include "fft.h"

// Minimum waves per SIMD the operator kernels are compiled for (register budget 256 at 2).
#ifndef FDE_XW
#define FDE_XW 2
#endif
#ifndef FDE_YW
#define FDE_YW 2
#endif

// Transform lengths the launchers instantiate.
#ifndef FDE_L_CASES
#define FDE_L_CASES(MACRO) \
  MACRO(16) MACRO(32) MACRO(64) MACRO(128) MACRO(256) MACRO(512) MACRO(1024) MACRO(2048) MACRO(4096)
#endif

namespace fde {

// Only one spectrum is live in registers at a time; the second product waits in LDS:
//   pass 1: (zr, zi) <- lam .* Z, inverse -> (T a, T b)
//   pass 2: (pr, pi) <- conj(lam) .* Z, inverse -> (T^T a, T^T b)
// Both symbol products from one read of the symbol: Z = (zr, zi) becomes lam * Z in registers and
// conj(lam) * Z goes to zs (real parts zs[0, L), imaginary parts zs[L, 2L)), each thread at its own
// positions t + T*m, so no barrier is needed before it reads them back.  Between the two inverse
// transforms the partial results of the first take the second product's place in zs.
template <int L, typename P, typename R>
__device__ __forceinline__ void symbol_both(R (&zr)[P::E], R (&zi)[P::E], R* zs, const R* __restrict__ lam,
                                            int t) {
  constexpr int E = P::E, T = P::T;
  static_for<0, E>([&](auto m) {
    const int k = t + T * m;
    const R lr = lam[2 * k], li = lam[2 * k + 1];
    const R a = zr[m], b = zi[m];
    zr[m] = lr * a - li * b;
    zi[m] = lr * b + li * a;
    zs[k] = lr * a + li * b;
    zs[L + k] = lr * b - li * a;
  });
}

// The same products from symbol values already in registers (lr, li at positions t + T*m), for
// kernels that load the symbol ahead of the forward transform.
template <int L, typename P, typename R>
__device__ __forceinline__ void symbol_both_regs(R (&zr)[P::E], R (&zi)[P::E], R* zs, const R (&lr)[P::E],
                                                 const R (&li)[P::E], int t) {
  constexpr int E = P::E, T = P::T;
  static_for<0, E>([&](auto m) {
    const int k = t + T * m;
    const R a = zr[m], b = zi[m];
    zr[m] = lr[m] * a - li[m] * b;
    zi[m] = lr[m] * b + li[m] * a;
    zs[k] = lr[m] * a + li[m] * b;
    zs[L + k] = lr[m] * b - li[m] * a;
  });
}

template <int L, typename P, typename R>
__device__ __forceinline__ void unstash(R (&pr)[P::E], R (&pi)[P::E], const R* zs, int t) {
  constexpr int E = P::E, T = P::T;
  static_for<0, E>([&](auto m) {
    pr[m] = zs[t + T * m];
    pi[m] = zs[L + t + T * m];
  });
}

// p[i] where ok, else 0, with the load itself unconditional (index 0, which must be valid, where
// !ok).  Written as (a && b) ? p[i] : 0, the load went under a per-lane branch on a and was waited
// for before the branch closed, so the run of loads at the start of a pass went out one at a time.
// The index passes through an empty asm statement, so the compiler cannot move the load under a
// branch again; callers combine their conditions with & rather than &&.
template <typename T, typename I>
__device__ __forceinline__ T load_or_zero(const T* __restrict__ p, I i, bool ok) {
  I j = ok ? i : I(0);
  __asm__("" : "+v"(j));
  const T v = p[j];
  return ok ? v : T(0);
}

// A pointer that is the same for the whole wavefront, kept in scalar registers: loads then use a
// scalar base plus a 32-bit per-lane offset instead of one 64-bit address per element.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}

// Runs f(m) for m = 0..E-1 in groups of G, with scheduling barriers between groups so that the
// compiler does not hoist every group's global loads at once (which would exhaust registers).
template <int E, int G0, class F>
__device__ __forceinline__ void chunked_for(F&& f) {
  constexpr int G = G0 < E ? G0 : E;
  static_for<0, E / G>([&](auto gc) {
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, G>([&](auto mc) { f(ic<decltype(gc)::value * G + decltype(mc)::value>{}); });
  });
  __builtin_amdgcn_sched_barrier(0);
}
#ifndef FDE_EPI_GROUP
#define FDE_EPI_GROUP 16
#endif
constexpr int kEpiGroup = FDE_EPI_GROUP;

// Elements per thread of the row pass: at most 8 (more threads per transform and fewer registers
// per thread than the column pass's plan; the row pass's six streams need the resident waves).
#ifndef FDE_EMAX_X
#define FDE_EMAX_X 8
#endif
template <typename R, int L>
using XPlan = Plan<L, (emax_for(sizeof(R), L) < FDE_EMAX_X ? emax_for(sizeof(R), L) : FDE_EMAX_X)>;
template <typename R, int L>
using YPlan = PlanFor<R, L>;

// Loads issued one transform ahead.  The transforms of a pass are separated by LDS barriers, so a
// load placed next to its use waits out its whole latency with every wave of the workgroup.
// Row passes (toep_x_kernel): the operands of the epilogue (x, ay, b, 1/diag) are loaded before the
// last inverse transform, for L >= FDE_X_PREFETCH_EPI_L; where a workgroup fills a CU's LDS (one
// workgroup per CU, 2 waves per SIMD, so up to 256 registers cost no occupancy) the symbol is also
// loaded before the forward transform and the (d+, d-) pairs before the first inverse one.
// Measured at 2047^2 on gfx950 (kernel trace of one CN step): FP64 row pass at L = 4096 85.3 ->
// 61.3 us, FP32 row passes 41.5 -> 34.0 us (L = 4096) and 16.1 -> 12.8 us (L = 2048), with the
// same register occupancy; at L = 512 the FP64 Jacobi pass would lose a wave per SIMD, so the
// threshold stays at 1024.  Results are unchanged (same arithmetic in the same order).
#ifndef FDE_X_PREFETCH
#define FDE_X_PREFETCH 1
#endif
#ifndef FDE_X_PREFETCH_EPI
#define FDE_X_PREFETCH_EPI 1
#endif
#ifndef FDE_X_PREFETCH_EPI_L
#define FDE_X_PREFETCH_EPI_L 1024
#endif
// FP32 row passes keep their occupancy with the epilogue's loads ahead down to L = 256.
#ifndef FDE_X_PREFETCH_EPI_L32
#define FDE_X_PREFETCH_EPI_L32 256
#endif
// Row pairs (transforms) per workgroup of the row pass: short transforms share a wavefront.
template <typename R, int L>
struct XCfg {
  static constexpr int S = XPlan<R, L>::T >= 64 ? 1 : 64 / XPlan<R, L>::T;
  static constexpr int THREADS = XPlan<R, L>::T * S;
  static constexpr int LDS_BYTES = S * (lds_exchange(L) + 2 * L) * (int)sizeof(R);
  static constexpr bool PREFETCH = FDE_X_PREFETCH && LDS_BYTES > 80 * 1024;
  static constexpr bool PREFETCH_EPI =
      PREFETCH || (FDE_X_PREFETCH_EPI && L >= (sizeof(R) == 4 ? FDE_X_PREFETCH_EPI_L32 : FDE_X_PREFETCH_EPI_L));
};

#ifndef FDE_Y_THREADS
#define FDE_Y_THREADS 512
#endif
#ifndef FDE_Y_COLS_PER_SLOT_L
#define FDE_Y_COLS_PER_SLOT_L 1024
#endif
// Slots (transforms, two columns each) per workgroup of the column pass: adjacent columns make the
// row reads of a workgroup contiguous, but too many slots leave CUs idle on the shorter levels.
// Measured on gfx950: L/1024 slots (at least a full wavefront, at most 512 threads) is best for
// L = 1024..4096.
// Column passes (toep_y_kernel) whose workgroup fills a CU's LDS load the symbol before the forward
// transform and the (e+, e-) pairs before the first inverse one.  FP64 only: at L = 4096 it took the
// FP64 pass from 96.0 to 92.4 us, while the FP32 pass went from 48.9 to 49.6 us.
#ifndef FDE_Y_PREFETCH
#define FDE_Y_PREFETCH 1
#endif
template <typename R, int L>
struct YCfg {
  static constexpr int T_ = YPlan<R, L>::T;
  static constexpr int SW = L / FDE_Y_COLS_PER_SLOT_L > 1 ? L / FDE_Y_COLS_PER_SLOT_L : 1;
  static constexpr int S0 = SW > 64 / T_ ? SW : 64 / T_;
  static constexpr int S = T_ * S0 <= FDE_Y_THREADS ? S0 : (T_ >= FDE_Y_THREADS ? 1 : FDE_Y_THREADS / T_);
  static constexpr int THREADS = YPlan<R, L>::T * S;
  static constexpr int LDS_BYTES = S * (lds_exchange(L) + 2 * L) * (int)sizeof(R);
  static constexpr bool PREFETCH = FDE_Y_PREFETCH && LDS_BYTES > 80 * 1024 && sizeof(R) == 8;
};

}  // namespace fde
