// Device-side state of the slot-based multishift solver (passed by value to kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sgw_internal.h"

namespace sgw {

constexpr int kMaxOcc = 256;  // occupied states held in LDS by the per-vector kernels
// ||(1 - P_occ) s|| below this fraction of ||s|| counts as a zero right-hand side
// mixed precision: default of sgw_opts.mixed_switch (a slot's Krylov steps apply the potential in
// FP32 once the largest estimated relative residual of its shifts is below mixed_switch * tol)
constexpr double kMixedSwitch = 1e4;
constexpr double kZeroRhsRel = 1e-13;

enum SlotStatus {
  SLOT_FREE = -1,
  SLOT_RUNNING = 0,
  SLOT_CONVERGED = 1,
  SLOT_MAXITER = 2,
  SLOT_BREAKDOWN = 3,
  SLOT_NONFINITE = 4,
  SLOT_ZERO_RHS = 5
};

struct SolverState {
  int npw, n_occ, n_omega, n_pert, kmax;
  long slot_stride;          // (kmax + 1) * npw
  const double2 *psi;        // [n_occ][npw] occupied states, internal order
  double2 *basis;            // [slots][kmax + 1][npw], or a pool of blocks of 2^bshift vectors
  const int32_t *btab = nullptr;  // pooled basis: [slots][nbmax] block of each 2^bshift Krylov vectors
  int nbmax = 0, bshift = 0;
  double2 *bvec;             // [slots][npw] right-hand sides
  double *alpha_t;           // [slots][kmax] Lanczos diagonal
  double *beta;              // [slots][kmax + 1]; beta[0] = ||b||
  double2 *rho;              // [slots][n_omega] last LU pivot per shift
  double *res;               // [slots][n_omega] estimated relative residual
  double *maxres;            // [slots] largest estimated relative residual over the shifts
  int32_t *conv;             // [slots][n_omega] Krylov dimension at which the estimate met tol_int, or -1
  int32_t *pair;             // [slots] pair index v * n_pert + p
  int32_t *kcur;             // [slots] completed steps
  int32_t *status;           // [slots] SlotStatus
  double *eps;               // [slots] band energy of the slot's pair
  const double *eps_band;    // [n_band]
  const double *omega;       // [n_omega]
  double eta;
  const double *eta_j = nullptr;  // [n_omega] per-shift imaginary parts, or NULL: eta for all
  double alpha;              // coefficient of P_occ
  double tol_int;            // stop when every estimated residual is below this
};

// Krylov vector k of a slot, in the stored basis or through the block table of the pool
__device__ __forceinline__ double2 *basis_vec(const SolverState &S, int slot, int k) {
  if (S.btab) {
    const long row = ((long)S.btab[slot * S.nbmax + (k >> S.bshift)] << S.bshift) + (k & ((1 << S.bshift) - 1));
    return S.basis + row * S.npw;
  }
  return S.basis + (long)slot * S.slot_stride + (long)k * S.npw;
}

sgw_status rhs_source(sgw_ctx *ctx, const sgw_ham *h_kq, const sgw_ham *h_k, int n_vec, const int32_t *pairs,
                      int n_pert, const int32_t *dvm, const double2 *psi_v, long ld_psi, double2 *s, long lds);
// b = -proj (proj = (1 - P_occ) src), ||src|| for the zero test, v_0 = b / ||b||
sgw_status slot_init(sgw_ctx *ctx, const SolverState &S, int n_fill, const double2 *src, const double2 *proj,
                     const int32_t *fill_slots, const int32_t *fill_pairs);
// Y[a] must hold (H + alpha P_occ) v_k of slot list[a]
sgw_status lanczos_step(sgw_ctx *ctx, const SolverState &S, int n_active, const int32_t *list, const double2 *Y);
// FOM coefficients of each shift at its own Krylov dimension; order[f][rank] = the pair's shifts by
// (dimension, index)
sgw_status tridiag(sgw_ctx *ctx, const SolverState &S, const int32_t *flist, int nf, double2 *ycoef, double2 *cp,
                   int32_t *order);
// (est_kavg: mean Krylov dimension of the pairs, est_kshift: of their shifts; timing statistics only)
sgw_status combine(sgw_ctx *ctx, const SolverState &S, const int32_t *flist, int nf, const double2 *ycoef,
                   const int32_t *order, double2 *X, double est_kavg, double est_kshift);
// AX must hold (H + alpha P_occ) X; cp[0] the overlaps of X (as proj_dot leaves them); u2i maps
// caller to internal plane-wave indices (dpsi is written in the caller's order)
sgw_status residual(sgw_ctx *ctx, const SolverState &S, const int32_t *flist, int nf, const double2 *X,
                    const double2 *AX, const double2 *cp, long rows, const int32_t *u2i, double2 *dpsi,
                    sgw_solve_info *info, double tol, int *n_bad);
// out[a][g] = 1 if g == cols[a] else 0, for a < n_col (device cols, caller's plane-wave order)
sgw_status unit_columns(sgw_ctx *ctx, int npw, int n_col, const int32_t *cols, double2 *out);
// plane-major copies of the potential, FP64 and FP32
sgw_status transpose_potential(sgw_ctx *ctx, const double *v, double *vt, float *vt32, const int n[3]);

}  // namespace sgw
