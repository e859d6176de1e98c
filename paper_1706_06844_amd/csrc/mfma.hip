// Toeplitz operator passes as BF16 matrix products on the MFMA units (FP32 accumulation), for the
// large FP32 levels of the V-cycle.
//
// The x part of tau/2 L x is a product of the field with dense Toeplitz matrices,
//   P1 = X B1, B1[k][i] = sx w_{i-k+1}   (= X T^T, multiplied by d+),
//   P2 = X B2, B2[k][i] = sx w_{k-i+1}   (= X T,   multiplied by d-),
// and the y part the same with the transposed field: (T X)^T = X^T B1 etc. with sy and e+-.  So one
// kernel serves both directions: the A operand is the field read along rows (x) or along columns (y),
// the B operand a Toeplitz tile.  Because B1 vanishes below its first subdiagonal and B2 above its
// first superdiagonal, each output tile needs P1 only for k <= i + 1 and P2 only for k >= i - 1: one
// full product's worth of work for both.
//
// Toeplitz tiles: the B fragment of a 32x32x16 MFMA for the output columns [n0, n0+32) and the
// reduction slice [k0, k0+16) depends only on o = n0 - k0.  All of them are precomputed once per
// level in the MFMA lane order (16 bytes per lane), so a B fragment is one coalesced load that stays
// in L2.
//
// A workgroup computes a 64x64 output tile with four wavefronts that split the active reduction
// range (split-K); the partial products meet in LDS, where the epilogue also reads them back in
// coalesced order.
#include <cstdint>
#include <cstring>
#include <vector>

#include "common.h"

namespace fde {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

constexpr int kMT = 64;     // output tile
constexpr int kKS = 16;     // reduction slice of one MFMA
constexpr int kLdsStride = kMT + 1;

// Output (m, n) of a direction maps to the field point: x: row m, column n; y: row n, column m.
template <int DIR>
__device__ __forceinline__ size_t field_index(int m, int n, int n1) {
  return DIR == 0 ? (size_t)m * n1 + n : (size_t)n * n1 + m;
}

// x[i] where ok, else 0, with the load itself unconditional (index 0 where !ok, always in bounds): a
// load under a branch is waited for before the branch closes, which serialises a run of such loads.
template <typename I>
__device__ __forceinline__ float ldg_or_zero(const float* __restrict__ x, I i, bool ok) {
  const float f = x[ok ? i : I(0)];
  return ok ? f : 0.f;
}

// A fragment: rows m0 + lane%32 of the direction's A operand, reduction indices k0 + 8*(lane/32) + v.
template <int DIR>
__device__ __forceinline__ bf16x8 load_a(const float* __restrict__ x, int n1, int M, int K, int m, int k) {
  bf16x8 a;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int kk = k + v;
    const bool ok = m < M && kk < K;
    const float f = ldg_or_zero(x, DIR == 0 ? (size_t)m * n1 + kk : (size_t)kk * n1 + m, ok);
    a[v] = (__bf16)f;
  }
  return a;
}

// A operand through LDS: each wave stages the A fragments of kChunk consecutive slices of its range
// with loads that run along the field's rows (four 64-byte row segments per instruction in the x
// direction, 64 consecutive floats in the y direction, instead of 32 rows per instruction), converts
// them to BF16 once and stores them in fragment order; the MFMA loop then reads each fragment with
// one 16-byte LDS load.  The values and the order of the products are those of the direct loads.
// Bit d of FDE_MFMA_LDS stages direction d.  Measured at 2047^2 on gfx950 (kernel trace): x pass
// 177 us direct, 102 us staged; y pass 79 us direct (its direct loads already read 128-byte rows),
// 85 us staged.
#ifndef FDE_MFMA_LDS
#define FDE_MFMA_LDS 1
#endif
constexpr int kChunk = 4;

// The A values of slice [k0, k0 + 16), rows [m0, m0 + 64), as this lane loads them: y direction, lane
// = row m and v[kk] = A[m][k0 + kk] (each instruction reads 64 consecutive floats); x direction, lane =
// (kk, r4) and v[q] = A[r4 + 4q][k0 + kk] (each instruction reads four 16-float row segments).  Offsets
// are 32-bit (at most 2048^2 points), so every load is the uniform base plus one offset register.
template <int DIR>
__device__ __forceinline__ void load_slice(const float* __restrict__ x, int n1, int M, int K, int m0, int k0,
                                           int lane, float (&v)[kKS]) {
  if constexpr (DIR == 1) {
    const int m = m0 + lane;
#pragma unroll
    for (int kk = 0; kk < kKS; ++kk)
      v[kk] = ldg_or_zero(x, (unsigned)(k0 + kk) * (unsigned)n1 + (unsigned)m, m < M && k0 + kk < K);
  } else {
    const int kk = lane & 15, r4 = lane >> 4;
#pragma unroll
    for (int q = 0; q < kKS; ++q) {
      const int m = m0 + r4 + 4 * q;
      v[q] = ldg_or_zero(x, (unsigned)m * (unsigned)n1 + (unsigned)(k0 + kk), m < M && k0 + kk < K);
    }
  }
}

// Those values in BF16 into st in fragment order: fragment i (rows 32 i .. 32 i + 31), lane L = row
// + 32 * (k / 8), value k mod 8.
template <int DIR>
__device__ __forceinline__ void store_slice(const float (&v)[kKS], int lane, bf16x8* st) {
  if constexpr (DIR == 1) {
    bf16x8 lo, hi;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      lo[q] = (__bf16)v[q];
      hi[q] = (__bf16)v[8 + q];
    }
    const int i = lane >> 5, l0 = lane & 31;
    st[i * 64 + l0] = lo;
    st[i * 64 + l0 + 32] = hi;
  } else {
    const int kk = lane & 15, r4 = lane >> 4;
    __bf16* s16 = reinterpret_cast<__bf16*>(st);
#pragma unroll
    for (int q = 0; q < kKS; ++q) {
      const int ml = r4 + 4 * q;
      const int i = ml >> 5, L = (ml & 31) + 32 * (kk >> 3);
      s16[(i * 64 + L) * 8 + (kk & 7)] = (__bf16)v[q];
    }
  }
}

// DIR 0: x pass with the mode epilogue (out = epilogue(l + ay)); DIR 1: y pass, ay = l.
// M x N outputs, reduction length K; cpm = (c+, c-) pairs of the direction (d+- or e+-).
template <int DIR, int MODE>
__global__ __launch_bounds__(256, 2) void mfma_toep_kernel(int n1, int n2, const float* __restrict__ x,
                                                           const bf16x8* __restrict__ bt1,
                                                           const bf16x8* __restrict__ bt2, int omin,
                                                           const float* __restrict__ cpm, const float* ay,
                                                           const float* __restrict__ b,
                                                           const float* __restrict__ dinv, float* out,
                                                           const int* __restrict__ skip) {
  if (skip && *skip) return;
  // the partial tiles of the epilogue; the staged A fragments use the same memory before it
  __shared__ __attribute__((aligned(16))) float part[4][kMT * kLdsStride];
  const int M = DIR == 0 ? n2 : n1, N = DIR == 0 ? n1 : n2, K = N;
  const int tiles_n = (N + kMT - 1) / kMT;
  const int m0 = (blockIdx.x / tiles_n) * kMT, n0 = (blockIdx.x % tiles_n) * kMT;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int KS = (K + kKS - 1) / kKS;
  // active slices: P1 for k0 <= n0 + 64, P2 for k0 + 15 >= n0 - 1
  const int e1 = min(KS - 1, (n0 + kMT) / kKS);
  const int s2 = max(0, n0 / kKS - 1);
  const int U1 = e1 + 1, U = U1 + (KS - s2);
  const int ub = (w * U) / 4, ue = ((w + 1) * U) / 4;
  floatx16 acc[2][2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[p][i][j] = floatx16{};
  const int lm = lane & 31, lk = 8 * (lane >> 5);
  auto k_of = [&](int u) { return (u >= U1 ? s2 + (u - U1) : u) * kKS; };
  // the B fragments of slice u (output columns n0 .. n0 + 31 and n0 + 32 .. n0 + 63)
  auto load_b = [&](int u, bf16x8& b0, bf16x8& b1) {
    const int k0 = k_of(u);
    const bf16x8* bt = u >= U1 ? bt2 : bt1;
    b0 = bt[(size_t)((n0 - k0 - omin) / kKS) * 64 + lane];
    b1 = bt[(size_t)((n0 + 32 - k0 - omin) / kKS) * 64 + lane];
  };
  auto slice = [&](int u, const bf16x8& a0, const bf16x8& a1, const bf16x8& b0, const bf16x8& b1) {
    const bool second = u >= U1;
    if (!second) {
      acc[0][0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0][0], 0, 0, 0);
      acc[0][0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][0][1], 0, 0, 0);
      acc[0][1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[0][1][0], 0, 0, 0);
      acc[0][1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[0][1][1], 0, 0, 0);
    } else {
      acc[1][0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[1][0][0], 0, 0, 0);
      acc[1][0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[1][0][1], 0, 0, 0);
      acc[1][1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][1][0], 0, 0, 0);
      acc[1][1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1][1], 0, 0, 0);
    }
  };
  if constexpr ((FDE_MFMA_LDS >> DIR) & 1) {
    // every wave runs the same number of chunks (the ranges differ by at most one slice), so the
    // workgroup barriers around the staging are uniform; slices past a wave's range load slice U - 1
    // (always a valid slice) and skip their products
    const int span = (U + 3) / 4;
    const int nchunks = (span + kChunk - 1) / kChunk;
    bf16x8* st = reinterpret_cast<bf16x8*>(&part[0][0]) + w * (kChunk * 2 * 64);
    for (int c = 0; c < nchunks; ++c) {
      const int u0 = ub + c * kChunk;
      float va[kChunk][kKS];
#pragma unroll
      for (int j = 0; j < kChunk; ++j) load_slice<DIR>(x, n1, M, K, m0, k_of(min(u0 + j, U - 1)), lane, va[j]);
#pragma unroll
      for (int j = 0; j < kChunk; ++j) store_slice<DIR>(va[j], lane, st + j * 128);
      // the B fragments (L2-resident tables) arrive while the workgroup meets at the barrier
      bf16x8 bq[kChunk][2];
#pragma unroll
      for (int j = 0; j < kChunk; ++j) load_b(min(u0 + j, U - 1), bq[j][0], bq[j][1]);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kChunk; ++j)
        if (u0 + j < ue) slice(u0 + j, st[j * 128 + lane], st[j * 128 + 64 + lane], bq[j][0], bq[j][1]);
      __syncthreads();
    }
  } else {
    for (int u = ub; u < ue; ++u) {
      const int k0 = k_of(u);
      bf16x8 b0, b1;
      load_b(u, b0, b1);
      slice(u, load_a<DIR>(x, n1, M, K, m0 + lm, k0 + lk), load_a<DIR>(x, n1, M, K, m0 + 32 + lm, k0 + lk), b0, b1);
    }
  }
  // reduce the four partial tiles of each product through LDS; element (m, n) of the tile sits at
  // [row][col] = [m][n] (x) or [n][m] (y), so the epilogue reads along field rows
  float p1[16], p2[16];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int mr = 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int nr = 32 * j + lm;
          const int row = DIR == 0 ? mr : nr, col = DIR == 0 ? nr : mr;
          part[w][row * kLdsStride + col] = acc[p][i][j][r];
        }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int row = e >> 6, col = e & 63;
      const int o = row * kLdsStride + col;
      const float s = part[0][o] + part[1][o] + part[2][o] + part[3][o];
      if (p == 0) p1[q] = s;
      else p2[q] = s;
    }
    __syncthreads();
  }
  const int r0 = DIR == 0 ? m0 : n0, c0 = DIR == 0 ? n0 : m0;  // tile origin in field rows/columns
  // every operand load first (unconditional, clamped to index 0 outside the field), then the stores
  // (field indices fit 32 bits: the MFMA levels have at most 2048^2 points)
  float res[16];
  unsigned fq[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int fr = r0 + (e >> 6), fc = c0 + (e & 63);
    fq[q] = (fr < n2 && fc < n1) ? (unsigned)fr * (unsigned)n1 + (unsigned)fc : 0xffffffffu;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const unsigned f = fq[q] == 0xffffffffu ? 0u : fq[q];
    const float l = cpm[2 * f] * p1[q] + cpm[2 * f + 1] * p2[q];
    if constexpr (DIR == 1) {
      res[q] = l;
    } else {
      const float lt = l + ay[f];
      const float xv = x[f];
      if constexpr (MODE == EP_APPLY) res[q] = xv - lt;
      else if constexpr (MODE == EP_RESID) res[q] = b[f] - xv + lt;
      else res[q] = xv + dinv[f] * (b[f] - xv + lt);
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (fq[q] != 0xffffffffu) out[fq[q]] = res[q];
}

// ---- host side ----------------------------------------------------------------------------------
static uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}

int mfma_table_entries(int n) {
  const int pad = (n + kKS - 1) / kKS * kKS;
  const int padn = (n + kMT - 1) / kMT * kMT;
  return (padn + pad) / kKS + 2;
}
int mfma_table_omin(int n) { return -((n + kKS - 1) / kKS * kKS); }

// Tables for one direction: t1 for B1 = s w_{n-k+1}, t2 for B2 = s w_{k-n+1}; each entry is one B
// fragment (64 lanes x 8 values) for o = n0 - k0 = omin + 16 e.  w: weights w_0..w_n (n = size).
void mfma_tables(const double* w, int n, double s, uint16_t* t1, uint16_t* t2) {
  const int E = mfma_table_entries(n), omin = mfma_table_omin(n);
  auto wt = [&](long m) -> float { return (m >= 0 && m <= n) ? (float)(s * w[m]) : 0.f; };
  for (int e = 0; e < E; ++e) {
    const long o = omin + (long)kKS * e;
    for (int l = 0; l < 64; ++l)
      for (int v = 0; v < 8; ++v) {
        const long kr = 8 * (l >> 5) + v, nr = l & 31;
        t1[((size_t)e * 64 + l) * 8 + v] = to_bf16(wt(o + nr - kr + 1));
        t2[((size_t)e * 64 + l) * 8 + v] = to_bf16(wt(kr - nr - o + 1));
      }
  }
}

template <int DIR, int MODE>
static void launch_one(const MfmaView& v, const float* x, const float* cpm, const float* ay, const float* b,
                       const float* dinv, float* out, const int* skip, hipStream_t st) {
  const int M = DIR == 0 ? v.n2 : v.n1, N = DIR == 0 ? v.n1 : v.n2;
  const int grid = ((M + kMT - 1) / kMT) * ((N + kMT - 1) / kMT);
  const bf16x8* t1 = reinterpret_cast<const bf16x8*>(DIR == 0 ? v.tx1 : v.ty1);
  const bf16x8* t2 = reinterpret_cast<const bf16x8*>(DIR == 0 ? v.tx2 : v.ty2);
  const int omin = mfma_table_omin(N);
  hipLaunchKernelGGL((mfma_toep_kernel<DIR, MODE>), dim3(grid), dim3(256), 0, st, v.n1, v.n2, x, t1, t2, omin,
                     cpm, ay, b, dinv, out, skip);
}

hipError_t launch_mfma_op(const MfmaView& v, const float* dpm, const float* epm, const float* x, float* ay,
                          float* out, int mode, const float* b, const float* dinv, const int* skip, hipStream_t st) {
  if (!v.tx1 || !v.tx2 || !v.ty1 || !v.ty2 || !dpm || !epm || !x || !ay || !out || v.n1 < 1 || v.n2 < 1)
    return hipErrorInvalidValue;
  if (out == x || out == ay || ay == x) return hipErrorInvalidValue;  // no pass updates in place
  if ((mode == EP_RESID || mode == EP_JACOBI) && !b) return hipErrorInvalidValue;
  if (mode == EP_JACOBI && !dinv) return hipErrorInvalidValue;
  launch_one<1, EP_APPLY>(v, x, epm, nullptr, nullptr, nullptr, ay, skip, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == EP_APPLY) launch_one<0, EP_APPLY>(v, x, dpm, ay, b, dinv, out, skip, st);
  else if (mode == EP_RESID) launch_one<0, EP_RESID>(v, x, dpm, ay, b, dinv, out, skip, st);
  else if (mode == EP_JACOBI) launch_one<0, EP_JACOBI>(v, x, dpm, ay, b, dinv, out, skip, st);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fde
