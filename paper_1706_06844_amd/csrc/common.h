// Internal declarations shared by the libfde sources (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace fde {

// Epilogue of an operator application.  With l = tau/2 * L x (both directions):
//   APPLY  : out = x - l                         (A x, A = I - tau/2 L)
//   RESID  : out = b - x + l                     (b - A x)
//   JACOBI : out = x + dinv * (b - x + l)        (damped Jacobi, dinv = omega / diag(A))
//   RHS    : out = x + l + tau * sum_k phi_k S_k (explicit CN half step plus source)
//   LOUT   : out = l
enum Mode : int { EP_APPLY = 0, EP_RESID = 1, EP_JACOBI = 2, EP_RHS = 3, EP_LOUT = 4 };

constexpr int kMaxSrc = 4;
struct SrcTerms {
  int n;
  double phi[kMaxSrc];
  const double* S[kMaxSrc];
};

// Device view of one operator level in precision R.
template <typename R>
struct OpView {
  int n1, n2;
  int L1, L2;
  const R* dpm;   // [n2][n1][2] = (d+, d-)
  const R* epm;   // [n2][n1][2] = (e+, e-)
  const R* dinv;  // [n2][n1] = omega / diag(A)
  const R* mu_x;  // [L1][2] symbol of the x products (scale and 1/L folded in)
  const R* mu_y;  // [L2][2]
  const R* tw_x;  // FFT twiddles for L1
  const R* tw_y;  // FFT twiddles for L2
  const R* swx;   // direct levels: sx * w_k, k = 0..n1
  const R* swy;   // direct levels: sy * w_k, k = 0..n2
  int direct;     // 1: apply with the direct dense-Toeplitz kernel instead of the FFT passes
};

// ---- launchers (toeplitz.hip) ------------------------------------------------------------------
// y-pass into ay, then x-pass with the epilogue.  x may alias out for EP_JACOBI.
template <typename R, typename Tin>
hipError_t launch_operator(const OpView<R>& op, const Tin* x, R* ay, R* out, int mode, const R* b,
                           const SrcTerms* src, double tau, const int* skip, hipStream_t st);

// The two passes separately: ay = y part; out = epilogue(x part + ay).
template <typename R, typename Tin>
hipError_t launch_op_y(const OpView<R>& op, const Tin* x, R* ay, const int* skip, hipStream_t st);
template <typename R, typename Tin>
hipError_t launch_op_x(const OpView<R>& op, const Tin* x, const R* ay, R* out, int mode, const R* b,
                       const SrcTerms* src, double tau, const int* skip, hipStream_t st);

// Direct dense-Toeplitz operator for small levels (n1 <= 512): one launch for both directions and
// the epilogue; swx/swy are sx*w_k, sy*w_k for k = 0..n.
template <typename R, typename Tin>
hipError_t launch_direct_op(int n1, int n2, const Tin* x, const R* dpm, const R* epm, const R* swx, const R* swy,
                            R* out, int mode, const R* b, const R* dinv, const SrcTerms* src, double tau,
                            const int* skip, hipStream_t st);

bool fft_length_supported(int L);
// FFT twiddle table for length L, shared by every transform plan and element size: exp(-2 pi i k/L),
// k < L/2, interleaved complex, computed in extended precision; count = 2 * entries = L.
void fft_twiddles(int L, int elem_bytes, double* out, int* count);
int fft_twiddle_count(int L, int elem_bytes);
// Symbol of one direction: out[k] = scale * lam[k] / L, lam = DFT of the circulant embedding of
// T = [w_{i-j+1}] (n x n, L = 2(n+1)).  out: 2L doubles (interleaved complex).
void toeplitz_symbol(const double* w, int n, int L, double scale, double* out);

// ---- multigrid kernels (mg.hip) ----------------------------------------------------------------
template <typename R, typename Tin>
hipError_t launch_presmooth(int N, const Tin* b, const double* bscale, const R* dinv, R* x, R* bcopy,
                            const int* skip, hipStream_t st);
template <typename R>
hipError_t launch_restrict(int n1, int n2, const R* r, R* rc, const R* dinv_c, R* xc, const int* skip,
                           hipStream_t st);
template <typename R>
hipError_t launch_prolong(int n1, int n2, const R* e, R* x, const int* skip, hipStream_t st);
// Direct (dense-Toeplitz) levels, tiled with LDS-staged rows and columns:
// residual b - A x fused with the full-weighting restriction rc = P^T r / 4 (and, with xc given,
// the coarse level's first Jacobi sweep from zero, xc = dinv_c .* rc); the residual stays on chip.
template <typename R>
hipError_t launch_tile_resid_restrict(int n1, int n2, const R* x, const R* b, const R* dpm, const R* epm,
                                      const R* swx, const R* swy, R* rc, const R* dinv_c, R* xc, const int* skip,
                                      hipStream_t st);
// True if both tiled kernels' LDS staging fits a workgroup for an n1 x n2 level.
template <typename R>
bool tile_lds_fits(int n1, int n2);
// One damped-Jacobi sweep xout = xn + dinv (b - A xn) with xn = x + P e (prolongation and
// correction fused into the staging; e = NULL: xn = x).  xout may not alias x.
template <typename R>
hipError_t launch_tile_jacobi(int n1, int n2, const R* x, const R* e, const R* b, const R* dpm, const R* epm,
                              const R* dinv, const R* swx, const R* swy, R* xout, const int* skip, hipStream_t st);
template <typename Tout, typename Tin>
hipError_t launch_convert(size_t N, const Tin* in, Tout* out, hipStream_t st);
template <typename R>
hipError_t launch_fill(size_t N, R* out, R v, hipStream_t st);
// Interleave two FP64 fields into (a, b) pairs of type R, scaled by s.
template <typename R>
hipError_t launch_interleave(size_t N, const double* a, const double* b, R* out, hipStream_t st);
// Injection of a pair field to the coarse grid: out[J][I] = in[2J+1][2I+1].
template <typename R>
hipError_t launch_inject_pairs(int n1, int n2, const R* in, R* out, hipStream_t st);
// dinv = omega / (1 - sx (d+ + d-) w1a - sy (e+ + e-) w1b)
template <typename R>
hipError_t launch_diag(int N, const R* dpm, const R* epm, double sxw1, double syw1, double omega,
                       R* dinv, double* diag_out, hipStream_t st);
// Validation scan: flags[0] |= negative, flags[1] |= non-finite.
hipError_t launch_scan_fields(size_t N, const double* const* f, int nf, int* flags, hipStream_t st);

// Direct (dense Toeplitz sum) coarse levels, one workgroup runs the whole V-cycle below `lc`.
constexpr int kMaxCoarseLevels = 4;
template <typename R>
struct CoarseView {
  int nlev;                         // levels handled (the last is solved exactly)
  int n1[kMaxCoarseLevels], n2[kMaxCoarseLevels];
  const R* dpm[kMaxCoarseLevels];
  const R* epm[kMaxCoarseLevels];
  const R* dinv[kMaxCoarseLevels];
  const R* swx[kMaxCoarseLevels];   // scaled weights sx * w_k, k = 0..n1
  const R* swy[kMaxCoarseLevels];
  const double* inv;                // FP64 inverse of the coarsest matrix (row-major Nc x Nc)
  int nu_pre, nu_post;
};
template <typename R>
hipError_t launch_coarse_vcycle(const CoarseView<R>& cv, const R* b, R* x, const int* skip,
                                hipStream_t st);
template <typename R>
size_t coarse_lds_bytes(const CoarseView<R>& cv);
// Direct apply of a coarse level (test hook): out = A x via dense Toeplitz sums.
template <typename R>
hipError_t launch_direct_apply(const CoarseView<R>& cv, int level, const R* x, R* out, int mode,
                               const R* b, hipStream_t st);
// Assemble the dense coarsest matrix from the coarsest level and invert it in place (FP64).
// With `dense` given (row-major FP64, the coarsest level's matrix), that matrix is inverted instead.
template <typename R>
hipError_t launch_coarse_invert(const CoarseView<R>& cv, const double* dense, double* inv, int* status,
                                hipStream_t st);
// x = inv * b for the coarsest level (test hook)
template <typename R>
hipError_t launch_coarse_solve(int Nc, const double* inv, const R* b, R* x, const int* skip, hipStream_t st);

// x += z elementwise (x FP64, z in precision R).
template <typename R>
hipError_t launch_add_to(size_t N, const R* z, double* x, hipStream_t st);

// ---- Galerkin coarse operators (galerkin.hip) ----------------------------------------------------
// Level l of the Galerkin hierarchy in factored form: coarse grid nlx x nly, fine grid n0x x n0y,
// H = 2^logH.  cx0/cx1: [nly][n0x] pairs (c+_D, c-_D) for D = 0, 1; ey0/ey1: [n0y][nlx] pairs.
// V: [nly][n0x] pairs and W: [n0y][nlx] pairs of transform results (scratch shared by the levels).
template <typename R>
struct GalView {
  int n0x, n0y, nlx, nly, logH;
  int L0x, L0y;
  const R* cx0;
  const R* cx1;
  const R* ey0;
  const R* ey1;
  const R* mu_x;  // fine-grid symbols and twiddles in precision R
  const R* mu_y;
  const R* tw_x;
  const R* tw_y;
  const R* dinv;
  R* V;
  R* W;
  double m0x, m1x, m0y, m1y;  // mass (P^T P) stencils per direction
  double scale;               // 4^-l
};
// out = A_l x (EP_APPLY), b - A_l x (EP_RESID) or x + dinv (b - A_l x) (EP_JACOBI, out != x).
template <typename R>
hipError_t launch_gal_apply(const GalView<R>& g, const R* x, R* out, int mode, const R* b, const int* skip,
                            hipStream_t st);
// cx0/cx1/ey0/ey1 from the fine FP64 coefficient pairs (the pointers in g are written).
template <typename R>
hipError_t launch_gal_setup(GalView<R>& g, const double* dpm, const double* epm, hipStream_t st);
// Diagonal: dinv = omega / diag and/or dout = diag; qx, qy: [2][2H-1] factor-times-hat tables.
template <typename R>
hipError_t launch_gal_diag(const GalView<R>& g, const double* qx, const double* qy, double omega, R* dinv,
                           double* dout, hipStream_t st);
// Dense FP64 matrix of the level (row-major, (nlx*nly)^2); Qx: [2][nlx][n0x], Qy: [2][nly][n0y].
template <typename R>
hipError_t launch_gal_dense(const GalView<R>& g, const double* Qx, const double* Qy, double* A, hipStream_t st);

// ---- BF16 MFMA operator passes (mfma.hip) ----------------------------------------------------------
// Precomputed Toeplitz B fragments of one level: tx1/tx2 for the x factors (length n1, scale sx),
// ty1/ty2 for the y factors; each mfma_table_entries(n) * 64 * 8 BF16 values.
struct MfmaView {
  int n1, n2;
  const uint16_t* tx1;
  const uint16_t* tx2;
  const uint16_t* ty1;
  const uint16_t* ty2;
};
int mfma_table_entries(int n);
int mfma_table_omin(int n);
void mfma_tables(const double* w, int n, double s, uint16_t* t1, uint16_t* t2);
// ay = y part (BF16 products, FP32 accumulation), then out = epilogue(x part + ay); out != x.
hipError_t launch_mfma_op(const MfmaView& v, const float* dpm, const float* epm, const float* x, float* ay,
                          float* out, int mode, const float* b, const float* dinv, const int* skip, hipStream_t st);

// ---- Krylov kernels (krylov.hip) ---------------------------------------------------------------
constexpr int kMaxRestart = 32;
// Device-resident state of one flexible GMRES solve.  The first block of fields is copied to the
// host to decide about restarts.
struct GmresState {
  int done;       // 1: stop issuing Arnoldi steps in this cycle (converged, cycle full, breakdown)
  int iters;      // Arnoldi steps so far in this solve
  int nused;      // Arnoldi steps in the current cycle
  int conv;       // 1: the FP64 true residual met the tolerance
  int nreorth;    // Arnoldi steps in this solve that took a second Gram-Schmidt pass
  unsigned reorth_mask;  // bit j: step j of the current cycle took the second pass
  double resnorm; // last true residual norm
  double est;     // last Givens residual estimate
  double bnorm;
  double atol;    // rtol * ||b||
  // configuration
  double rtol;
  int maxit, restart;
  int orth;       // Gram-Schmidt policy: 0 one pass, 1 always two passes, 2 second pass when needed
  int reorth;     // 1: the current Arnoldi step takes the second pass
  unsigned ticket;  // workgroups of a small pass that have written their partials
  int idle;         // 1: a slot of a batched group without a solve in flight: the cycle's kernels skip it
  double keep_min;  // policy 2: second pass when the first leaves less than this fraction of ||w||^2
  double brk_tol;   // breakdown: the new direction's norm below brk_tol times its column's
  double g[kMaxRestart + 1], cs[kMaxRestart], sn[kMaxRestart];
  double Rm[kMaxRestart * kMaxRestart];  // column j in Rm[j*kMaxRestart + i], i <= j
  double h1[kMaxRestart + 1], h2[kMaxRestart + 1];
  double vscale[kMaxRestart + 1];
  double y[kMaxRestart];
};

// Passes of one Arnoldi step: DOTS (h1 = V^T w and ||w||^2, decides the second pass), UPDATE_DOTS
// (second pass only: w -= V h1, h2 = V^T w), UPDATE_NORM (w -= V h, h = h2 or h1, then ||w|| and the
// Givens update); INIT (w = src, ||src||) and RESNORM (||w||, or w = src and ||src|| when src is
// given) start a solve and a cycle.
enum CgsKind : int { CGS_DOTS = 0, CGS_UPDATE_DOTS = 1, CGS_UPDATE_NORM = 2, CGS_INIT = 3, CGS_RESNORM = 4 };
// BF16 storage of a Krylov basis entry (the upper half of the FP32 bit pattern).
struct bf16_t {
  uint16_t bits;
};
// One fused pass over the basis V[0..nv) (storage TB: FP64, FP32 or BF16; column stride ldv a
// multiple of the run length, 16 bytes of basis entries; columns 16-byte aligned) and the work vector
// w (storage TW: FP64 or FP32, 16-byte aligned, readable and writable up to N rounded up to a run);
// src is FP64.  With TB = TW, w is itself a basis column and vout is unused; with BF16 storage the
// passes that finish a vector (UPDATE_NORM, INIT, RESNORM with src) also write its BF16 rounding
// to the basis column vout.  Streams the pass and writes per-workgroup partials; `cap` bounds the
// grid (cgs_grid(N)).
template <typename TB, typename TW>
hipError_t launch_cgs_pass(int kind, size_t N, int nv, TB* V, size_t ldv, TW* w, TB* vout, const double* src,
                           GmresState* st, double* partials, int cap, hipStream_t s);
// Combines the partials of the preceding pass (same kind, nv, cap) and updates the solver state.
// Not needed (and not launched) when cgs_fused(nv, cap): the pass then finalises itself.
hipError_t launch_cgs_finalize(int kind, int nv, double* partials, GmresState* st, int cap, hipStream_t s);
bool cgs_fused(int nv, int cap);
int cgs_grid(size_t N);
size_t cgs_partials_len(size_t N);
// Column stride of the Krylov basis for N unknowns (multiple of 64 doubles).
size_t basis_ld(size_t N);
template <typename Tz>
hipError_t launch_update_x(size_t N, const Tz* Z, size_t ldz, double* x, int first,
                           GmresState* st, hipStream_t s);

// ---- small helpers -----------------------------------------------------------------------------
inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }
// ---- batched launches ---------------------------------------------------------------------------
// Instances of one shape whose device buffers are laid out identically (equal slots of one region)
// can be advanced by one launch: the grid's z dimension runs over a table of byte offsets, and every
// kernel of the solve shifts each of its pointer arguments by its entry ztab[blockIdx.z] (the offset
// of an instance's slot from the slot whose pointers the launch carries).  An entry kZSkip makes the
// workgroups of that z exit at once (padding up to the launch's fixed z extent).  The launchers read
// the current batch from this thread's context (1 instance, no table outside a batched section).
constexpr long long kZSkip = (long long)0x8000000000000000ull;
struct BatchCtx {
  int nz = 1;
  const long long* ztab = nullptr;
};
inline thread_local BatchCtx g_batch;
inline int batch_nz() { return g_batch.nz; }
inline const long long* batch_ztab() { return g_batch.ztab; }
// Sets the batch for the lifetime of the object (restores the previous one).
struct BatchScope {
  BatchCtx saved;
  BatchScope(int nz, const long long* ztab) : saved(g_batch) { g_batch = BatchCtx{nz, ztab}; }
  ~BatchScope() { g_batch = saved; }
};
template <typename T>
__device__ __forceinline__ T* zshift(T* p, long long zoff) {
  return (p && zoff) ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + (uintptr_t)zoff) : p;
}
// The first statement of a batched kernel: this workgroup's slot offset (a uniform scalar load of
// the table, none outside a batch), or exit for a padding entry.
#define FDE_ZBEGIN                                                  \
  const long long zoff = ztab ? ztab[blockIdx.z] : 0ll;             \
  if (zoff == kZSkip) return
#define FDE_ZSHIFT(p) (p = zshift(p, zoff))
// The same for kernels instantiated with and without batching (ZB a template parameter): without,
// the table lookup and every shift fold away.
#define FDE_ZBEGIN_IF(ZB)                                \
  const long long zoff = (ZB) ? ztab[blockIdx.z] : 0ll;  \
  if ((ZB) && zoff == kZSkip) return

// Reads a device flag (the skip flag of speculatively issued Arnoldi steps) with a vector load: the
// index is an opaque zero in a vector register, so that waiting for the flag does not also wait for
// the kernel's scalar argument loads, and a kernel can issue its other loads before it needs the flag.
__device__ const int kZeroFlag = 0;
__device__ __forceinline__ int load_flag(const int* p) {
  int z = 0;
  __asm__ volatile("" : "+v"(z));
  const int* q = p ? p : &kZeroFlag;
  return q[z];
}

inline bool is_pow2m1(int n) { return n >= 1 && ((n + 1) & n) == 0; }
inline bool is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }
// Grid sides the multigrid takes: n = 2^l - 1 or n = 2^l.  The down-sampling of Sec. 4.1 keeps
// k = (n - n mod 2) / 2 = n >> 1 coarse points, coarse index J at fine index 2J + (n mod 2)
// (0-based): the odd fine points of an odd grid, the even ones of an even grid.
inline bool is_mg_side(int n) { return is_pow2m1(n) || is_pow2(n); }
// Length of the circulant embedding of an n x n Toeplitz matrix with offsets -1..n-1: the smallest
// power of two >= 2n - 1 (2(n + 1) for n = 2^l - 1, 2n for n = 2^l).
inline int fft_len(int n) {
  int L = 2;
  while (L < 2 * n - 1) L <<= 1;
  return L;
}

}  // namespace fde
