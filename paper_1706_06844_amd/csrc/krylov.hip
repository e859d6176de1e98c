// Flexible GMRES building blocks (the Krylov solver of paper Sec. 4.3 and Sec. 5): fused
// Gram-Schmidt passes with deterministic FP64 reductions, the Givens update of the Hessenberg
// least-squares problem, and the solution update x += Z y.
//
// The basis V is stored unnormalised: column k holds a multiple of v_k and vscale[k] turns it into
// v_k.  This saves the separate normalisation pass; every consumer applies the scale.
//
// Reductions: every thread accumulates a fixed strided subset, a fixed tree combines the block's
// values, each block writes its partials, and the last block to finish (ticket counter) combines
// the partials in block order.  The result does not depend on scheduling, so runs are bitwise
// reproducible for a given launch shape.
#include "common.h"

namespace fde {

constexpr int kCgsBlock = 256;
constexpr int kCgsMaxGrid = 512;

int cgs_grid(size_t N) {
  size_t g = (N + (size_t)kCgsBlock * 8 - 1) / ((size_t)kCgsBlock * 8);
  if (g < 1) g = 1;
  if (g > kCgsMaxGrid) g = kCgsMaxGrid;
  return (int)g;
}
size_t cgs_partials_len(size_t) { return (size_t)(kMaxRestart + 1) * kCgsMaxGrid; }

// Sum of v over the block in a fixed order; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// Givens update after column j of the Hessenberg matrix is known (single thread).
__device__ void givens_step(GmresState* st, int j, double nrm) {
  constexpr int K = kMaxRestart;
  double col[kMaxRestart + 1];
  for (int i = 0; i <= j; ++i) col[i] = st->h1[i] + (st->cgs2 ? st->h2[i] : 0.0);
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
  st->vscale[j + 1] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  // breakdown: the new direction vanished relative to the column (the Krylov space is invariant)
  const bool breakdown = !(nrm > 1e-14 * r);
  if (est <= st->atol || st->iters >= st->maxit || breakdown || j + 1 >= st->restart) st->done = 1;
}

template <int MAXV>
__global__ __launch_bounds__(kCgsBlock) void cgs_kernel(int kind, size_t N, int nv, const double* __restrict__ V,
                                                        size_t ldv, double* __restrict__ w,
                                                        const double* __restrict__ src, GmresState* st,
                                                        double* __restrict__ partials) {
  if ((kind == CGS_DOTS || kind == CGS_UPDATE_DOTS || kind == CGS_UPDATE_NORM) && st->done) return;
  __shared__ double hc[MAXV];
  __shared__ double red[16];
  __shared__ int is_last;
  // coefficients of the unnormalised columns for the update passes
  if (threadIdx.x < MAXV) {
    double c = 0.0;
    if ((int)threadIdx.x < nv) {
      if (kind == CGS_UPDATE_DOTS) c = st->h1[threadIdx.x] * st->vscale[threadIdx.x];
      if (kind == CGS_UPDATE_NORM) c = (st->cgs2 ? st->h2[threadIdx.x] : st->h1[threadIdx.x]) * st->vscale[threadIdx.x];
    }
    hc[threadIdx.x] = c;
  }
  __syncthreads();
  const bool dots = (kind == CGS_DOTS || kind == CGS_UPDATE_DOTS);
  const bool upd = (kind == CGS_UPDATE_DOTS || kind == CGS_UPDATE_NORM);
  double acc[MAXV];
#pragma unroll
  for (int k = 0; k < MAXV; ++k) acc[k] = 0.0;
  double nacc = 0.0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += stride) {
    if (kind == CGS_INIT) {
      const double b = src[p];
      w[p] = b;
      nacc += b * b;
      continue;
    }
    if (kind == CGS_RESNORM) {
      const double r = w[p];
      nacc += r * r;
      continue;
    }
    double wv = w[p];
    double vk[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) vk[k] = (k < nv) ? V[(size_t)k * ldv + p] : 0.0;
    if (upd) {
#pragma unroll
      for (int k = 0; k < MAXV; ++k)
        if (k < nv) wv -= hc[k] * vk[k];
      w[p] = wv;
    }
    if (dots) {
#pragma unroll
      for (int k = 0; k < MAXV; ++k)
        if (k < nv) acc[k] += vk[k] * wv;
    } else {
      nacc += wv * wv;
    }
  }
  // block reductions -> partials[k * gridDim.x + blockIdx.x]
  const int G = gridDim.x;
  if (dots) {
    for (int k = 0; k < nv; ++k) {
      const double s = block_sum(acc[k], red);
      if (threadIdx.x == 0) partials[(size_t)k * G + blockIdx.x] = s;
    }
  } else {
    const double s = block_sum(nacc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int t = atomicAdd(&st->ticket[0], 1u);
    is_last = (t == (unsigned int)G - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const volatile double* vp = partials;
  const int nres = dots ? nv : 1;
  for (int k = 0; k < nres; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < G; b += blockDim.x) v += vp[(size_t)k * G + b];
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) {
      if (kind == CGS_DOTS) st->h1[k] = s * st->vscale[k];
      else if (kind == CGS_UPDATE_DOTS) st->h2[k] = s * st->vscale[k];
      else red[15] = s;
    }
  }
  if (threadIdx.x == 0) {
    st->ticket[0] = 0;
    if (kind == CGS_UPDATE_NORM) {
      givens_step(st, nv - 1, sqrt(red[15]));
    } else if (kind == CGS_INIT) {
      const double bn = sqrt(red[15]);
      st->bnorm = bn;
      st->atol = st->rtol * bn;
      st->resnorm = bn;
      st->est = bn;
      st->g[0] = bn;
      st->vscale[0] = bn > 0.0 ? 1.0 / bn : 0.0;
      st->iters = 0;
      st->nused = 0;
      st->conv = (bn == 0.0);
      st->done = (bn == 0.0);
    } else if (kind == CGS_RESNORM) {
      const double rn = sqrt(red[15]);
      st->resnorm = rn;
      st->conv = (rn <= st->atol);
      st->g[0] = rn;
      st->vscale[0] = rn > 0.0 ? 1.0 / rn : 0.0;
      st->nused = 0;
      st->done = (st->conv || st->iters >= st->maxit) ? 1 : 0;
    }
  }
}

hipError_t launch_cgs_pass(int kind, size_t N, int nv, double* V, size_t ldv, double* w, const double* src,
                           GmresState* st, double* partials, int grid, hipStream_t s) {
  if (nv > kMaxRestart + 1) return hipErrorInvalidValue;
#define L_(M)                                                                                            \
  hipLaunchKernelGGL((cgs_kernel<M>), dim3(grid), dim3(kCgsBlock), 0, s, kind, N, nv, V, ldv, w, src, st, \
                     partials)
  if (nv <= 4) L_(4);
  else if (nv <= 8) L_(8);
  else if (nv <= 16) L_(16);
  else if (nv <= 24) L_(24);
  else L_(kMaxRestart + 1);
#undef L_
  return hipGetLastError();
}

// x = (first ? 0 : x) + Z y, with y solving the nused x nused triangular system R y = g.
template <typename Tz>
__global__ __launch_bounds__(256) void update_x_kernel(size_t N, const Tz* __restrict__ Z, size_t ldz,
                                                       double* __restrict__ x, int first, GmresState* st) {
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
  hipLaunchKernelGGL((update_x_kernel<Tz>), dim3((int)g), dim3(256), 0, s, N, Z, ldz, x, first, st);
  return hipGetLastError();
}
template hipError_t launch_update_x<double>(size_t, const double*, size_t, double*, int, GmresState*,
                                            hipStream_t);
template hipError_t launch_update_x<float>(size_t, const float*, size_t, double*, int, GmresState*,
                                           hipStream_t);

}  // namespace fde
