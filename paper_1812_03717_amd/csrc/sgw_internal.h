// Internal declarations shared by the translation units of libsgw.so.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/sgw.h"

namespace sgw {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
sgw_status fail(sgw_status code, const std::string &msg);

#define SGW_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::sgw::fail(SGW_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SGW_CHECK(cond, msg)                                               \
  do {                                                                     \
    if (!(cond)) return ::sgw::fail(SGW_ERR_INVALID_ARG, (msg));           \
  } while (0)

// ---------------------------------------------------------------------------
// kernel identifiers for timing statistics
// ---------------------------------------------------------------------------
enum KernelId {
  K_STICKS_INV = 0,
  K_PLANES,
  K_STICKS_FWD,
  K_PROJ_DOT,
  K_PROJ_APPLY,
  K_RHS,
  K_INIT,
  K_LANCZOS,
  K_TRIDIAG,
  K_COMBINE,
  K_RESIDUAL,
  K_PERMUTE,
  K_NL_DOT,
  K_NL_APPLY,
  K_CHI_DOT,
  K_DIELECTRIC,
  K_BLK_PRODUCT,
  K_COUNT
};
const char *kernel_name(int id);

struct KernelStat {
  int64_t launches = 0;
  double ms = 0, bytes = 0, flops = 0;
};

struct PendingTiming {
  int kid;
  hipEvent_t start, stop;
  double bytes, flops;
};

}  // namespace sgw

struct sgw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  unsigned profile_mask = 0;        // bit k: time launches of kernel k
  int fft_planes = 0;               // plane-pass kernel of H.x (SGW_FFT_*), the context's setting
  int fft_active = 0;               // the same for the solve in progress (0: fft_planes)
  sgw::KernelStat stats[sgw::K_COUNT];
  std::vector<sgw::PendingTiming> pending;
  std::vector<hipEvent_t> event_pool;
  // pinned host staging (status polls, small uploads)
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  // autotuned options per system class (grid / n_pw / n_occ / n_omega)
  std::map<std::string, sgw_opts> tuned;
  // rocBLAS handle of the block solver (created on its first use, bound to `stream`)
  void *blas = nullptr;
};

// Device-resident index maps of one Hamiltonian.  "internal" order is
// stick-major: plane waves grouped by (m0, m1) column along axis 2.
struct sgw_ham {
  sgw_ctx *ctx = nullptr;           // creating context (not used after it is destroyed)
  int device = 0;
  int n[3] = {0, 0, 0};
  int n_pw = 0;
  int n_stick = 0;
  int m0_lo = 0, n_row = 0;         // rows (axis 0) holding sticks: m0 in [m0_lo, m0_lo + n_row)
  int m1_lo = 0, m1_hi = -1;        // m1 range of all sticks
  int m2_lo = 0, m2_hi = -1;        // m2 range of all plane waves
  double kvec[3];
  double recip[3][3];
  std::vector<int32_t> miller;      // host copy, caller order
  int box_lo[3], box_dim[3];        // Miller lookup box (caller indices)
  // device arrays
  int32_t *d_i2u = nullptr;         // [n_pw] internal -> caller index
  int32_t *d_u2i = nullptr;         // [n_pw] caller -> internal index
  int32_t *d_stick_off = nullptr;   // [n_stick + 1]
  int4 *d_rows = nullptr;           // [n_row] {first stick, m1_lo, m1_hi, 0} of row m0 = m0_lo + t
  int32_t *d_stick_ij = nullptr;    // [n_stick] (i0 << 16) | i1: the stick's grid column
  int32_t *d_pw_stick = nullptr;    // [n_pw] internal -> stick
  int32_t *d_pw_z = nullptr;        // [n_pw] internal -> i2
  int32_t *d_miller_int = nullptr;  // [n_pw][3] internal order
  double *d_kin = nullptr;          // [n_pw] internal order, 0.5|k+G|^2
  double *d_vt = nullptr;           // [N2][N0][N1] potential, plane-major
  float *d_vt32 = nullptr;          // the same in FP32
  int32_t *d_box = nullptr;         // [box volume] -> caller index or -1
  double2 *d_tw = nullptr;          // twiddles: 3 tables of N_d entries exp(-2 pi i t / N_d)
  float2 *d_tw32 = nullptr;         // the same in FP32
  int tw_off[3];
  // separable non-local pseudopotential sum_p |beta_p> E_p <beta_p| (n_proj = 0: none)
  int n_proj = 0;
  double2 *d_beta = nullptr;        // [n_proj][n_pw] internal order
  double *d_ekb = nullptr;          // [n_proj] E_p (Ha)
};

namespace sgw {

// Describes where vector a of a batch lives: base + a*ld, or, with a slot list,
// base + list[a]*slot_stride (+ kidx[list[a]]*ld when kidx is given).  With a block table (a
// pooled Krylov basis), vector k of slot s is row k mod 2^bshift of block btab[s][k >> bshift],
// each block 2^bshift rows of ld values from base.
struct VecSrc {
  const double2 *base;
  long ld;
  const int32_t *list;
  const int32_t *kidx;
  long slot_stride;
  const int32_t *btab = nullptr;
  int nbmax = 0, bshift = 0;
  __host__ __device__ inline const double2 *ptr(int a) const {
    if (!list) return base + (long)a * ld;
    int s = list[a];
    if (btab) {
      const int k = kidx[s];
      const long row = ((long)btab[s * nbmax + (k >> bshift)] << bshift) + (k & ((1 << bshift) - 1));
      return base + row * ld;
    }
    return base + (long)s * slot_stride + (kidx ? (long)kidx[s] * ld : 0L);
  }
};

inline VecSrc listed(const double2 *p, long ld, const int32_t *list) { return VecSrc{p, ld, list, nullptr, ld}; }

inline VecSrc contiguous(const double2 *p, long ld) { return VecSrc{p, ld, nullptr, nullptr, 0}; }

// Timing helpers (no-ops when profiling is off).
void timing_begin(sgw_ctx *ctx, int kid, double bytes, double flops, PendingTiming *out);
void timing_end(sgw_ctx *ctx, PendingTiming *t);
sgw_status timing_collect(sgw_ctx *ctx);
// pinned host staging of at least `bytes` in ctx->pinned
sgw_status ensure_pinned(sgw_ctx *ctx, size_t bytes);
// waits for the context's stream, then collects kernel timings
sgw_status sync(sgw_ctx *ctx);

// H.x over a batch (internal order): y = T.x + F V F^-1 x (+ V_NL x).  `tbuf` holds
// hx_tbuf_bytes(h, n_vec) bytes: the stick buffer (n_vec * N2 * n_stick complex entries,
// complex128, or complex64 when fp32), which also takes the non-local overlaps once the stick
// passes are done.  fp32: the potential term F V F^-1 x runs in FP32 (x rounded to FP32, FP32
// transforms and potential); the kinetic and non-local terms and y stay FP64.  x and y must not
// overlap.
sgw_status hx_batch(sgw_ctx *ctx, const sgw_ham *h, int n_vec, VecSrc x, double2 *y, long ldy, void *tbuf,
                    bool fp32 = false);
bool hx_grid_supported(int n);
// the plane-pass kernel (SGW_FFT_LINE / PAIR / LDS) that H.x of `h` uses under ctx's setting
int hx_plane_kernel(const sgw_ctx *ctx, const sgw_ham *h, bool fp32);
// the solve in progress uses plane kernel `v` (0: the context's setting) while the scope lives
struct FftScope {
  sgw_ctx *ctx;
  int saved;
  FftScope(sgw_ctx *c, int v) : ctx(c), saved(c->fft_active) { c->fft_active = v; }
  ~FftScope() { ctx->fft_active = saved; }
  FftScope(const FftScope &) = delete;
  FftScope &operator=(const FftScope &) = delete;
};

// Projector pieces (internal order, FP64 MFMA).  The overlaps are produced as
// partial sums over plane-wave chunks: cp[chunk][a][i] for chunk < n_chunks,
// a < n_vec (leading dimension `rows` >= n_vec), i < n_occ.
constexpr int kProjChunks = 64;
// plane waves per overlap chunk: chunk c holds plane waves [c * kProjChunkLen, (c + 1) * kProjChunkLen)
constexpr int kProjChunkLen = 256;
// worker streams of a batch solve
constexpr int kMaxWorkers = 16;
// number of chunks for n_pw plane waves; *kc receives the chunk length
int proj_chunks(int n_pw, int *kc);
// cp[chunk][a][i] = sum_{g in chunk} conj(psi[i][g]) x_a[g], then cp[0][a][i] = the sum over all
// chunks (in chunk order): on return chunk 0 holds the complete overlaps
// (kid: the timing slot the launches are charged to)
sgw_status proj_dot(sgw_ctx *ctx, int n_pw, int n_occ, const double2 *psi, int n_vec, VecSrc x,
                    double2 *cp, long rows, int kid = K_PROJ_DOT);
// with c = cp[0]:  mode 0: y_a = x_a - psi^T c_a ; mode 1: y_a += alpha psi^T c_a
// (mode 0 may run in place, y_a == x_a); row_scale (n_occ values, may be NULL) multiplies c_a[i]
// by row_scale[i] first
sgw_status proj_apply(sgw_ctx *ctx, int n_pw, int n_occ, const double2 *psi, int n_vec, VecSrc x,
                      const double2 *cp, long rows, double2 *y, long ldy, double alpha, int mode,
                      const double *row_scale = nullptr, int kid = K_PROJ_APPLY);
// bytes of H.x scratch (`tbuf` of hx_batch) for n_vec vectors of h
inline size_t hx_tbuf_bytes(const sgw_ham *h, long n_vec) {
  int kc;
  const size_t sticks = 16ul * (size_t)n_vec * h->n[2] * h->n_stick;
  const size_t nl = h->n_proj > 0 ? 16ul * (size_t)n_vec * proj_chunks(h->n_pw, &kc) * h->n_proj : 0;
  return std::max(sticks, nl);
}
// Split-BF16 projector (FP32-level accuracy on the BF16 matrix cores, FP32 accumulation): `split`
// holds proj_split_bytes(n_pw, n_occ) bytes (256-byte aligned), written by proj_split from psi
// (internal order); proj_dot_bf16 / proj_apply_bf16 then take the place of proj_dot / proj_apply
// (same cp layout and modes).
size_t proj_split_bytes(int n_pw, int n_occ);
sgw_status proj_split(sgw_ctx *ctx, int n_pw, int n_occ, const double2 *psi, void *split);
sgw_status proj_dot_bf16(sgw_ctx *ctx, int n_pw, int n_occ, const void *split, int n_vec, VecSrc x, double2 *cp,
                         long rows);
sgw_status proj_apply_bf16(sgw_ctx *ctx, int n_pw, int n_occ, const void *split, int n_vec, VecSrc x,
                           const double2 *cp, double2 *y, long ldy, double alpha, int mode);
// y_a = x_a
sgw_status permute_copy(sgw_ctx *ctx, int n_pw, int n_vec, VecSrc x, double2 *y, long ldy);
// out[a][g] = in[a][perm[g]] (gather) or out[a][perm[g]] = in[a][g] (scatter)
sgw_status permute(sgw_ctx *ctx, int n_pw, int n_vec, const double2 *in, long ldin, double2 *out,
                   long ldout, const int32_t *perm, int scatter, double scale = 1.0);

// Block solver (SGW_SOLVER_BLOCK): one block Krylov space per band over its perturbations.
constexpr int kBlockMaxPert = 32;                        // perturbations per band (block size)
constexpr double kBlockBudget = 144.0 * (1ull << 30);   // workspace the band chunks are sized for
size_t block_workspace_bytes(const sgw_ham *h_kq, int n_occ, int n_band, int n_pert, int n_omega,
                             const sgw_opts &o);
sgw_status block_solve(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq, const sgw_ham *h_k,
                       int n_band, const sgw_c128 *psi_v, const double *eps_v, int n_pert, const int32_t *dv_miller,
                       int n_omega, const double *omega, double eta, double tol, const sgw_opts &o, void *workspace,
                       size_t workspace_bytes, sgw_c128 *dpsi, sgw_solve_info *info);
// releases the context's rocBLAS handle
void blas_release(sgw_ctx *ctx);

}  // namespace sgw
