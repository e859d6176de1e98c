// Register-resident Stockham FFT for one power-of-two length L per group of T = L/E threads.
//
// Used by the Toeplitz operator kernels: a Toeplitz matrix-vector product is a linear convolution,
// computed through a circulant embedding of power-of-two length L >= 2n-1, so n <= L/2 and the upper
// half of every input is zero padding (the O(N log N) product the
// paper relies on, Sec. 1 and the Toeplitz-like structure of Sec. 2).
//
// Data layout between stages: thread t holds element t + T*m in register m (natural order), m < E.
// A stage of radix R with NS = product of the previous radices performs E/R butterflies per thread;
// butterfly b = t + T*q reads elements b + r*(L/R) (= registers q + r*(E/R)), multiplies element r by
// exp(sign 2 pi i r (b mod NS) / (NS R)), does a radix-R DFT, and writes element r of its output to
// position (b / NS) * NS * R + (b mod NS) + r * NS.  After the last stage (NS * R = L) that position
// is again t + T*m, so the result stays in registers in natural order; earlier stages exchange data
// through LDS.  Twiddles: a thread needs w^r, r = 1..R-1, with w = exp(sign 2 pi i (b mod NS)/(NS R));
// it loads the single base value w of each stage once per kernel from the table of exp(-2 pi i k/L),
// k < L/2 (entry k = (b mod NS) L/(NS R), the same table for every plan), and forms the powers with a
// product tree of depth <= 4.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace fde {

template <int V>
using ic = std::integral_constant<int, V>;

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

// cos and sin of 2 pi k / 16, k = 0..15.
constexpr double kCos16[16] = {1.0,
                               0.92387953251128675613,
                               0.70710678118654752440,
                               0.38268343236508977173,
                               0.0,
                               -0.38268343236508977173,
                               -0.70710678118654752440,
                               -0.92387953251128675613,
                               -1.0,
                               -0.92387953251128675613,
                               -0.70710678118654752440,
                               -0.38268343236508977173,
                               0.0,
                               0.38268343236508977173,
                               0.70710678118654752440,
                               0.92387953251128675613};
constexpr double kSin16[16] = {0.0,
                               0.38268343236508977173,
                               0.70710678118654752440,
                               0.92387953251128675613,
                               1.0,
                               0.92387953251128675613,
                               0.70710678118654752440,
                               0.38268343236508977173,
                               0.0,
                               -0.38268343236508977173,
                               -0.70710678118654752440,
                               -0.92387953251128675613,
                               -1.0,
                               -0.92387953251128675613,
                               -0.70710678118654752440,
                               -0.38268343236508977173};

// (re, im) *= exp(SIGN * 2 pi i * K / N) for compile-time K and N (N divides 16).
template <int K, int N, int SIGN, typename R>
__device__ __forceinline__ void rot(R& re, R& im) {
  constexpr int k = ((K % N) + N) % N;
  constexpr int k16 = k * (16 / N);
  if constexpr (k16 == 0) {
  } else if constexpr (k16 == 8) {
    re = -re;
    im = -im;
  } else if constexpr ((k16 == 4 && SIGN > 0) || (k16 == 12 && SIGN < 0)) {  // times +i
    R t = re;
    re = -im;
    im = t;
  } else if constexpr ((k16 == 4 && SIGN < 0) || (k16 == 12 && SIGN > 0)) {  // times -i
    R t = re;
    re = im;
    im = -t;
  } else {
    constexpr R c = (R)kCos16[k16];
    constexpr R s = (R)(SIGN > 0 ? kSin16[k16] : -kSin16[k16]);
    R t = re * c - im * s;
    im = re * s + im * c;
    re = t;
  }
}

// In-place DFT of N points held in registers, natural order in and out, sign SIGN.
template <int N, int SIGN, typename R>
__device__ __forceinline__ void dft(R (&re)[N], R (&im)[N]) {
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    R ar = re[0], ai = im[0];
    re[0] = ar + re[1];
    im[0] = ai + im[1];
    re[1] = ar - re[1];
    im[1] = ai - im[1];
  } else if constexpr (N == 4) {
    R t0r = re[0] + re[2], t0i = im[0] + im[2];
    R t1r = re[0] - re[2], t1i = im[0] - im[2];
    R t2r = re[1] + re[3], t2i = im[1] + im[3];
    R t3r = re[1] - re[3], t3i = im[1] - im[3];
    rot<1, 4, SIGN>(t3r, t3i);
    re[0] = t0r + t2r;
    im[0] = t0i + t2i;
    re[2] = t0r - t2r;
    im[2] = t0i - t2i;
    re[1] = t1r + t3r;
    im[1] = t1i + t3i;
    re[3] = t1r - t3r;
    im[3] = t1i - t3i;
  } else {
    // N = N1 * N2 with N1 = 4: input n = N2*n1 + n2, output k = k1 + N1*k2.
    constexpr int N1 = 4, N2 = N / 4;
    R yr[N2][N1], yi[N2][N1];
    static_for<0, N2>([&](auto n2) {
      R ar[N1], ai[N1];
      static_for<0, N1>([&](auto n1) {
        ar[n1] = re[N2 * n1 + n2];
        ai[n1] = im[N2 * n1 + n2];
      });
      dft<N1, SIGN>(ar, ai);
      static_for<0, N1>([&](auto k1) {
        rot<decltype(n2)::value * decltype(k1)::value, N, SIGN>(ar[k1], ai[k1]);
        yr[n2][k1] = ar[k1];
        yi[n2][k1] = ai[k1];
      });
    });
    static_for<0, N1>([&](auto k1) {
      R br[N2], bi[N2];
      static_for<0, N2>([&](auto n2) {
        br[n2] = yr[n2][k1];
        bi[n2] = yi[n2][k1];
      });
      dft<N2, SIGN>(br, bi);
      static_for<0, N2>([&](auto k2) {
        re[k1 + N1 * k2] = br[k2];
        im[k1 + N1 * k2] = bi[k2];
      });
    });
  }
}

// DFT of N points whose upper half is zero (re, im [N/2, N) are not read): the zero-padded input of
// a circulant embedding.  Same decomposition as dft, with the first radix-4 layer reduced to its two
// nonzero inputs: [a0, a1, 0, 0] -> [a0 + a1, a0 + W a1, a0 - a1, a0 - W a1], W = rotation by 1/4.
template <int N, int SIGN, typename R>
__device__ __forceinline__ void dft_half(R (&re)[N], R (&im)[N]) {
  auto dft4h = [](R& r0, R& i0, R& r1, R& i1, R& r2, R& i2, R& r3, R& i3) {
    const R ar = r0, ai = i0, br = r1, bi = i1;
    R wr = br, wi = bi;
    rot<1, 4, SIGN>(wr, wi);
    r0 = ar + br;
    i0 = ai + bi;
    r2 = ar - br;
    i2 = ai - bi;
    r1 = ar + wr;
    i1 = ai + wi;
    r3 = ar - wr;
    i3 = ai - wi;
  };
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    re[1] = re[0];
    im[1] = im[0];
  } else if constexpr (N == 4) {
    dft4h(re[0], im[0], re[1], im[1], re[2], im[2], re[3], im[3]);
  } else {
    constexpr int N1 = 4, N2 = N / 4;
    R yr[N2][N1], yi[N2][N1];
    static_for<0, N2>([&](auto n2) {
      R ar[N1], ai[N1];
      ar[0] = re[n2];
      ai[0] = im[n2];
      ar[1] = re[N2 + n2];
      ai[1] = im[N2 + n2];
      dft4h(ar[0], ai[0], ar[1], ai[1], ar[2], ai[2], ar[3], ai[3]);
      static_for<0, N1>([&](auto k1) {
        rot<decltype(n2)::value * decltype(k1)::value, N, SIGN>(ar[k1], ai[k1]);
        yr[n2][k1] = ar[k1];
        yi[n2][k1] = ai[k1];
      });
    });
    static_for<0, N1>([&](auto k1) {
      R br[N2], bi[N2];
      static_for<0, N2>([&](auto n2) {
        br[n2] = yr[n2][k1];
        bi[n2] = yi[n2][k1];
      });
      dft<N2, SIGN>(br, bi);
      static_for<0, N2>([&](auto k2) {
        re[k1 + N1 * k2] = br[k2];
        im[k1 + N1 * k2] = bi[k2];
      });
    });
  }
}

// LDS index padding: one spare slot every 2^FDE_LPAD_SHIFT elements spreads the strided stage writes
// over the banks.  Measured on gfx950 (SQ_LDS_BANK_CONFLICT): one slot in 32 halves the conflict
// cycles of the FP32 row pass against one in 16 and takes 1-3 % off the FP64 passes; the transforms
// are not bound by LDS conflicts (the FP32 passes' times moved by 1 %).
#ifndef FDE_LPAD_SHIFT
#define FDE_LPAD_SHIFT 5
#endif
__device__ __forceinline__ int lpad(int i) { return i + (i >> FDE_LPAD_SHIFT); }
__host__ __device__ constexpr int lds_len(int L) { return L + (L >> FDE_LPAD_SHIFT) + 1; }
// Exchange of a stage: real and imaginary parts together (one barrier pair per stage) or one after
// the other through a single buffer (half the LDS, two barrier pairs).
#ifndef FDE_EXCH_SPLIT
#define FDE_EXCH_SPLIT 0
#endif
// LDS reals one transform's exchange needs.
__host__ __device__ constexpr int lds_exchange(int L) { return FDE_EXCH_SPLIT ? lds_len(L) : 2 * lds_len(L); }

// Radix plan: E elements per thread, stages of radix E except a smaller last one.
__host__ __device__ constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// EMAX: elements per thread for long transforms (register budget: 16 for FP32, 8 for FP64).
template <int L, int EMAX = 16>
struct Plan {
  static constexpr int E = L >= 2 * EMAX ? EMAX : L / 2;
  static constexpr int T = L / E;
  static constexpr int LOGE = ilog2(E);
  static constexpr int LOGL = ilog2(L);
  static constexpr int NSTAGES = (LOGL + LOGE - 1) / LOGE;
  __host__ __device__ static constexpr int radix(int s) {
    return (s < NSTAGES - 1 || LOGL % LOGE == 0) ? E : (1 << (LOGL % LOGE));
  }
  __host__ __device__ static constexpr int ns(int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= radix(i);
    return v;
  }
  // complex base-twiddle entries of stage s (stage 0 has none)
  __host__ __device__ static constexpr int tw_count(int s) { return s == 0 ? 0 : ns(s); }
  __host__ __device__ static constexpr int tw_offset(int s) {
    int o = 0;
    for (int i = 0; i < s; ++i) o += tw_count(i);
    return o;
  }
  __host__ __device__ static constexpr int tw_total() { return tw_offset(NSTAGES); }
};

#ifndef FDE_EMAX_F32
#define FDE_EMAX_F32 16
#endif
#ifndef FDE_EMAX_F64
#define FDE_EMAX_F64 8
#endif
#ifndef FDE_EMAX_F32_SHORT
#define FDE_EMAX_F32_SHORT 8
#endif
#ifndef FDE_SHORT_L
#define FDE_SHORT_L 2048
#endif
#ifndef FDE_EMAX_F32_TINY
#define FDE_EMAX_F32_TINY 4
#endif
#ifndef FDE_TINY_L
#define FDE_TINY_L 1024
#endif
// Elements per thread for a length-L transform with elements of `bytes` bytes.  Measured on gfx950:
// FP32 transforms of length 4096 run fastest with 16 elements (three radix-16 stages), length 2048
// with 8 and length 1024 and below with 4 (more threads per transform, more waves resident on the
// smaller grids); FP64 with 8.
__host__ __device__ constexpr int emax_for(int bytes, int L) {
  return bytes == 8 ? FDE_EMAX_F64
                    : (L <= FDE_TINY_L ? FDE_EMAX_F32_TINY : (L <= FDE_SHORT_L ? FDE_EMAX_F32_SHORT : FDE_EMAX_F32));
}
template <typename R, int L>
using PlanFor = Plan<L, emax_for(sizeof(R), L)>;

// One Stockham stage of plan P.  `rr`/`ri` hold the thread's E elements (natural positions t + T*m).
// Every stage but the last has one butterfly per thread (radix E), computed in place; its outputs
// are exchanged through `lds` (lds_exchange(L) reals) and read back at positions t + T*m.  The last
// stage (possibly of smaller radix, several butterflies per thread) writes each butterfly's outputs
// over its own inputs, which are exactly positions t + T*m.
// ZH: the transform's input is zero from element L/2 on; the first stage (one butterfly per thread
// over elements t + T r, so inputs r >= R/2 are those zeros) then skips them.
template <int L, int S, int SIGN, typename R, typename P, bool ZH = false>
__device__ __forceinline__ void fft_stage(R (&rr)[P::E], R (&ri)[P::E], R* lds, const R* bw, int t) {
  constexpr int E = P::E, T = P::T;
  constexpr int RADIX = P::radix(S);
  constexpr int NS = P::ns(S);
  constexpr int BPT = E / RADIX;
  constexpr bool LAST = (S == P::NSTAGES - 1);
  static_assert(LAST || BPT == 1, "only the last stage may use a smaller radix");
  static_for<0, BPT>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    R vr[RADIX], vi[RADIX];
    static_for<0, RADIX>([&](auto rc) {
      vr[rc] = rr[q + rc * BPT];
      vi[rc] = ri[q + rc * BPT];
    });
    if constexpr (NS > 1) {
      // base twiddle of butterfly q (preloaded), powers by a product tree
      R pr_[RADIX], pi_[RADIX];
      pr_[1] = bw[2 * q];
      pi_[1] = (SIGN > 0) ? -bw[2 * q + 1] : bw[2 * q + 1];
      static_for<2, RADIX>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        constexpr int a = (r & (r - 1)) == 0 ? r / 2 : (1 << (31 - __builtin_clz(r)));
        constexpr int c = r - a;
        pr_[r] = pr_[a] * pr_[c] - pi_[a] * pi_[c];
        pi_[r] = pr_[a] * pi_[c] + pi_[a] * pr_[c];
      });
      static_for<1, RADIX>([&](auto rc) {
        const R c = pr_[rc], s = pi_[rc];
        const R a = vr[rc] * c - vi[rc] * s;
        vi[rc] = vr[rc] * s + vi[rc] * c;
        vr[rc] = a;
      });
    }
    if constexpr (ZH && S == 0 && BPT == 1 && NS == 1) dft_half<RADIX, SIGN>(vr, vi);
    else dft<RADIX, SIGN>(vr, vi);
    static_for<0, RADIX>([&](auto rc) {
      rr[q + rc * BPT] = vr[rc];
      ri[q + rc * BPT] = vi[rc];
    });
  });
  if constexpr (!LAST) {
    // output r of this thread's butterfly b = t goes to (b / NS) * NS * RADIX + (b mod NS) + r * NS;
    // real parts in lds[0 .. lds_len), imaginary parts in lds[lds_len .. 2 lds_len)
    const int base = (t / NS) * NS * RADIX + (t & (NS - 1));
    if constexpr (FDE_EXCH_SPLIT) {
      static_for<0, RADIX>([&](auto rc) { lds[lpad(base + rc * NS)] = rr[rc]; });
      __syncthreads();
      static_for<0, E>([&](auto m) { rr[m] = lds[lpad(t + T * m)]; });
      __syncthreads();
      static_for<0, RADIX>([&](auto rc) { lds[lpad(base + rc * NS)] = ri[rc]; });
      __syncthreads();
      static_for<0, E>([&](auto m) { ri[m] = lds[lpad(t + T * m)]; });
      __syncthreads();
    } else {
      R* lre = lds;
      R* lim = lds + lds_len(L);
      static_for<0, RADIX>([&](auto rc) {
        lre[lpad(base + rc * NS)] = rr[rc];
        lim[lpad(base + rc * NS)] = ri[rc];
      });
      __syncthreads();
      static_for<0, E>([&](auto m) {
        rr[m] = lre[lpad(t + T * m)];
        ri[m] = lim[lpad(t + T * m)];
      });
      __syncthreads();
    }
  }
}

// Base twiddles of every stage for this thread: bw[s][2q], bw[s][2q+1] = exp(-2 pi i j/(NS R)),
// j = (t + T q) mod NS, loaded once per kernel from the table of exp(-2 pi i k/L), k < L/2.
template <typename R, int L, typename P_ = PlanFor<R, L>>
struct Twiddles {
  using P = P_;
  static constexpr int NST = P::NSTAGES > 1 ? P::NSTAGES : 2;
  static constexpr int BPTMAX = P::E / P::radix(P::NSTAGES - 1);
  R w[NST][2 * BPTMAX];
  __device__ __forceinline__ void load(const R* __restrict__ tab, int t) {
    static_for<1, P::NSTAGES>([&](auto sc) {
      constexpr int S = decltype(sc)::value;
      constexpr int NS = P::ns(S);
      constexpr int BPT = P::E / P::radix(S);
      constexpr int STEP = L / (NS * P::radix(S));
      static_for<0, BPT>([&](auto qc) {
        const int j = (t + P::T * decltype(qc)::value) & (NS - 1);
        w[S][2 * qc] = tab[2 * j * STEP];
        w[S][2 * qc + 1] = tab[2 * j * STEP + 1];
      });
    });
  }
};

// Full length-L DFT (SIGN = -1 forward, +1 unnormalised inverse) of the thread group's data.
// Every thread of the workgroup must call this (it contains barriers) even if its group is idle.
// ZH: elements L/2 .. L-1 of the input are zero (their registers are not read).
template <int L, int SIGN, bool ZH = false, typename R, typename P>
__device__ __forceinline__ void fft(R (&rr)[P::E], R (&ri)[P::E], R* lds, const Twiddles<R, L, P>& tw, int t_in) {
  // An opaque copy of the thread index: without it the compiler computes the LDS addresses of all
  // transforms of a kernel once and keeps them live throughout, which exhausts the registers.
  int t = t_in;
  __asm__ volatile("" : "+v"(t));
  static_for<0, P::NSTAGES>([&](auto s) {
    constexpr int S = decltype(s)::value;
    fft_stage<L, S, SIGN, R, P, ZH>(rr, ri, lds, tw.w[S < Twiddles<R, L, P>::NST ? S : 0], t);
  });
}

}  // namespace fde
