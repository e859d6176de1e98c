// The system operator of eq. (system), y = (I - tau/2 L) x with L of eq. (AxAy), without a solver
// handle and without allocating device memory: for callers that cannot call hipMalloc (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// Everything beyond the caller's inputs and outputs -- the WSGD weights (eq. (gk), eq. (w)), the
// FFT twiddle tables, the symbols of both circulant embeddings, the interleaved coefficient pairs
// and the intermediate column-pass field -- lives in one file-scope device array of fixed size,
// `scratch`, which every GPU the library runs on holds until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for the symbol): the first
// call on a device looks up that device's address of the array with hipGetSymbolAddress and keeps
// it, and every kernel argument is derived from that address.
//
// The operator passes are the ones fde_apply runs for the FP64 system operator (toeplitz.hip); only
// the set-up of their tables differs: here the weights, twiddles and symbols are computed on the
// device (the symbol as a direct DFT of the circulant embedding's n + 1 non-zeros, with exact
// integer reduction of the angle), instead of on the host and uploaded.
#include <cmath>
#include <mutex>

#include "../../include/fde.h"
#include "common.h"
#include "engine.h"

namespace fde {
namespace {

constexpr int kNaMaxN = FDE_NOALLOC_MAX_N;  // largest n1, n2
constexpr int kNaMaxL = 2 * (kNaMaxN + 1);  // largest transform length
constexpr size_t kNaMaxField = (size_t)kNaMaxN * kNaMaxN;
// layout of the scratch array, in doubles (every part starts on a 256-byte boundary)
constexpr size_t align32(size_t v) { return (v + 31) / 32 * 32; }
constexpr size_t kOffAy = 0;
constexpr size_t kOffDpm = kOffAy + align32(kNaMaxField);
constexpr size_t kOffEpm = kOffDpm + align32(2 * kNaMaxField);
constexpr size_t kOffLamX = kOffEpm + align32(2 * kNaMaxField);
constexpr size_t kOffLamY = kOffLamX + align32(2 * (size_t)kNaMaxL);
constexpr size_t kOffTwX = kOffLamY + align32(2 * (size_t)kNaMaxL);
constexpr size_t kOffTwY = kOffTwX + align32((size_t)kNaMaxL);
constexpr size_t kOffWa = kOffTwY + align32((size_t)kNaMaxL);
constexpr size_t kOffWb = kOffWa + align32((size_t)kNaMaxN + 2);
constexpr size_t kScratchDoubles = kOffWb + align32((size_t)kNaMaxN + 2);
}  // namespace

// The library-owned buffer of the entry point (external linkage, so that the runtime registers it
// under a stable name for hipGetSymbolAddress).
__device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Per-device address of `scratch`, looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

// WSGD weights w_0..w_K of order g (eq. (w)) from the Grunwald coefficients g_k = g_{k-1}(k-1-g)/k
// (eq. (gk)); one thread per direction.
__global__ void na_weights_kernel(double ga, int Ka, double* wa, double gb, int Kb, double* wb) {
  if (threadIdx.x > 1 || blockIdx.x != 0) return;
  const double g = threadIdx.x == 0 ? ga : gb;
  const int K = threadIdx.x == 0 ? Ka : Kb;
  double* w = threadIdx.x == 0 ? wa : wb;
  double gprev = 1.0;
  w[0] = 0.5 * g;
  for (int k = 1; k <= K; ++k) {
    const double gk = gprev * ((double)(k - 1) - g) / (double)k;
    w[k] = 0.5 * g * gk + (1.0 - 0.5 * g) * gprev;
    gprev = gk;
  }
}

// exp(-2 pi i k / L), k < L/2, interleaved (the table every transform plan of length L reads).
__global__ void na_twiddles_kernel(int L, double* tw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L / 2) return;
  double s, c;
  sincospi(-2.0 * (double)k / (double)L, &s, &c);
  tw[2 * k] = c;
  tw[2 * k + 1] = s;
}

// Symbol of one direction: out[k] = (scale / L) DFT(c)[k], c = [t_0 .. t_{n-1}, 0 .. 0, t_{-1}],
// t_m = w_{m+1}: a direct sum over the n + 1 non-zeros, the angle index k m reduced mod L exactly.
__global__ void na_symbol_kernel(const double* __restrict__ w, int n, int L, double scale, double* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  double re = 0.0, im = 0.0;
  for (int m = 0; m < n; ++m) {
    const int idx = (int)(((long long)k * m) % L);
    double s, c;
    sincospi(-2.0 * (double)idx / (double)L, &s, &c);
    re += w[m + 1] * c;
    im += w[m + 1] * s;
  }
  {
    const int idx = (int)(((long long)k * (L - 1)) % L);
    double s, c;
    sincospi(-2.0 * (double)idx / (double)L, &s, &c);
    re += w[0] * c;
    im += w[0] * s;
  }
  const double f = scale / (double)L;
  out[2 * k] = f * re;
  out[2 * k + 1] = f * im;
}

int fail(int code, const char* msg) {
  set_global_error(msg);
  return code;
}

}  // namespace
}  // namespace fde

using namespace fde;

extern "C" int fde_apply_noalloc(const fde_problem* p, const double* dp, const double* dm, const double* ep,
                                 const double* em, const double* x, double* y, void* stream) {
  if (!p) return fail(FDE_EINVAL, "problem is NULL");
  if (!dp || !dm || !ep || !em || !x || !y) return fail(FDE_EINVAL, "a field pointer is NULL");
  if (x == y) return fail(FDE_EINVAL, "y may not alias x");
  if (!(p->alpha > 1.0 && p->alpha < 2.0) || !(p->beta > 1.0 && p->beta < 2.0))
    return fail(FDE_EINVAL, "alpha and beta must lie in (1,2)");
  if (!is_mg_side(p->n1) || !is_mg_side(p->n2) || p->n1 < 7 || p->n2 < 7)
    return fail(FDE_EINVAL, "n1 and n2 must be 2^l - 1 or 2^l with l >= 3");
  if (p->n1 > kNaMaxN || p->n2 > kNaMaxN)
    return fail(FDE_EINVAL, "fde_apply_noalloc: n1 and n2 are limited to FDE_NOALLOC_MAX_N (1023); "
                            "use a handle (fde_setup, fde_apply) for larger grids");
  if (!(p->b1 > p->a1) || !(p->b2 > p->a2)) return fail(FDE_EINVAL, "domain needs a < b");
  if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(FDE_EINVAL, "tau must be positive and finite");
  double* base = nullptr;
  hipError_t e = scratch_ptr(&base);
  if (e != hipSuccess) return fail(FDE_EDEVICE, hipGetErrorString(e));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int n1 = p->n1, n2 = p->n2, L1 = fft_len(n1), L2 = fft_len(n2);
  const size_t N = (size_t)n1 * n2;
  const double hx = (p->b1 - p->a1) / (n1 + 1), hy = (p->b2 - p->a2) / (n2 + 1);
  const double sx = p->tau / (2.0 * std::pow(hx, p->alpha)), sy = p->tau / (2.0 * std::pow(hy, p->beta));
  double* wa = base + kOffWa;
  double* wb = base + kOffWb;
  double* lam_x = base + kOffLamX;
  double* lam_y = base + kOffLamY;
  double* tw_x = base + kOffTwX;
  double* tw_y = base + kOffTwY;
  double* dpm = base + kOffDpm;
  double* epm = base + kOffEpm;
  double* ay = base + kOffAy;
  hipLaunchKernelGGL(na_weights_kernel, dim3(1), dim3(64), 0, st, p->alpha, n1 + 1, wa, p->beta, n2 + 1, wb);
  hipLaunchKernelGGL(na_twiddles_kernel, dim3(ceil_div(L1 / 2, 256)), dim3(256), 0, st, L1, tw_x);
  hipLaunchKernelGGL(na_twiddles_kernel, dim3(ceil_div(L2 / 2, 256)), dim3(256), 0, st, L2, tw_y);
  hipLaunchKernelGGL(na_symbol_kernel, dim3(ceil_div(L1, 256)), dim3(256), 0, st, wa, n1, L1, sx, lam_x);
  hipLaunchKernelGGL(na_symbol_kernel, dim3(ceil_div(L2, 256)), dim3(256), 0, st, wb, n2, L2, sy, lam_y);
  if ((e = hipGetLastError()) != hipSuccess) return fail(FDE_EDEVICE, hipGetErrorString(e));
  if ((e = launch_interleave<double>(N, dp, dm, dpm, st)) != hipSuccess) return fail(FDE_EDEVICE, hipGetErrorString(e));
  if ((e = launch_interleave<double>(N, ep, em, epm, st)) != hipSuccess) return fail(FDE_EDEVICE, hipGetErrorString(e));
  OpView<double> op{};
  op.n1 = n1;
  op.n2 = n2;
  op.L1 = L1;
  op.L2 = L2;
  op.dpm = dpm;
  op.epm = epm;
  op.mu_x = lam_x;
  op.mu_y = lam_y;
  op.tw_x = tw_x;
  op.tw_y = tw_y;
  e = launch_operator<double, double>(op, x, ay, y, EP_APPLY, nullptr, nullptr, 0.0, nullptr, st);
  if (e != hipSuccess) return fail(FDE_EDEVICE, hipGetErrorString(e));
  return FDE_OK;
}
