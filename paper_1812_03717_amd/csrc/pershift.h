// Per-shift preconditioned solves (BiCGStab with right preconditioning), the
// learned diagonal model, and their host drivers.
#pragma once

#include "sgw_internal.h"
#include "solver_state.h"

namespace sgw {

// ---- small MLP: 5 features -> 64 -> 64 -> 4 (tanh) ----
constexpr int kMlpIn = 5, kMlpHid = 64, kMlpOut = 4;
constexpr int kMlpW1 = 0;                               // [kMlpHid][kMlpIn]
constexpr int kMlpB1 = kMlpW1 + kMlpHid * kMlpIn;       // [kMlpHid]
constexpr int kMlpW2 = kMlpB1 + kMlpHid;                // [kMlpHid][kMlpHid]
constexpr int kMlpB2 = kMlpW2 + kMlpHid * kMlpHid;      // [kMlpHid]
constexpr int kMlpW3 = kMlpB2 + kMlpHid;                // [kMlpOut][kMlpHid]
constexpr int kMlpB3 = kMlpW3 + kMlpOut * kMlpHid;      // [kMlpOut]
constexpr int kMlpParams = kMlpB3 + kMlpOut;            // 4804

}  // namespace sgw

struct sgw_mlp {
  sgw_ctx *ctx = nullptr;
  int device = 0;
  float *w = nullptr;        // device FP32 master weights [kMlpParams]
  uint16_t *wb = nullptr;    // device BF16 copy used for inference
  float *m1 = nullptr, *m2 = nullptr;  // Adam moments
  float *grad = nullptr;     // [kMlpParams]
  float *gpart = nullptr;    // per-block gradient partials
  int gpart_blocks = 0;
  float *loss = nullptr;     // [1 + blocks]
  int64_t step = 0;
};

namespace sgw {

// features of plane wave G for band energy eps and shift z = omega + i eta (Hartree):
// {T_G/10, eps/10, omega, 100 eta, (T_G - eps - omega)/10}; outputs are scaled by 1/(T_G + 1)
__host__ __device__ inline void mlp_features(double t, double eps, double om, double eta, float *f) {
  f[0] = (float)(t * 0.1);
  f[1] = (float)(eps * 0.1);
  f[2] = (float)om;
  f[3] = (float)(eta * 100.0);
  f[4] = (float)((t - eps - om) * 0.1);
}

// Device state of the per-shift slots: scalars [slots], vectors [slots][npw]
// (internal plane-wave order).
struct PsState {
  int npw, n_occ, max_iter;
  double tol;                 // recurrence stopping threshold (relative)
  double tol_final;           // target of the true FP64 residual
  int32_t *status, *iters, *out_index, *pair;
  double *eps, *zr, *zi, *bnorm, *rnorm;
  double2 *rho_prev, *rho_cur, *alph, *omg;
  double2 *b, *x, *r, *rh, *p, *v, *s, *ph, *sh, *m;
  // optional snapshot of (r_k, x_k) at iteration hist_iter, caller order [out_index][npw]
  int hist_iter;
  double2 *hist_r, *hist_x;
  const int32_t *i2u;
};

enum PsStatus { PS_RUNNING = 0, PS_CONVERGED = 1, PS_MAXITER = 2, PS_BREAKDOWN = 3, PS_NONFINITE = 4, PS_ZERO = 5 };
enum PcMode { PC_NONE = 0, PC_TETER = 1, PC_LEARNED = 2 };

// launchers (pershift.hip)
// slot parameters of system sys[a] (index (v*n_pert + p)*n_omega + j) into slot list[a]
sgw_status ps_setup(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const int32_t *sys,
                    const double *eps_band, const double *omega, double eta, const double *eta_j, int n_pert,
                    int n_omega);
// x of slot list[a] from dpsi[out_index] (caller order)
sgw_status ps_load_x(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *dpsi);
sgw_status ps_rhs(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *src,
                  const double2 *proj);
sgw_status ps_precond(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double *kin, int mode,
                      const sgw_mlp *mlp, int guess);
sgw_status ps_start(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y, int has_x0);
sgw_status ps_k1(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list);
sgw_status ps_k2(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y);
sgw_status ps_k3(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y);
sgw_status ps_final(sgw_ctx *ctx, const PsState &S, int n, const int32_t *list, const double2 *Y,
                    const double2 *cp, long rows, double2 *dpsi, sgw_solve_info *info, int *n_bad,
                    int extra_flags);

// Host driver: per-shift solves of the systems in `systems` (all when empty).
struct PsProblem {
  const sgw_ham *h_kq, *h_k;
  int n_occ;
  const double2 *psi_occ_kq;  // caller order
  int n_band;
  const double2 *psi_v;
  const double *eps_v;        // host
  int n_pert;
  const int32_t *dv_miller;   // host
  int n_omega;
  const double *omega;        // host
  double eta, tol;
};
size_t ps_workspace_bytes(const sgw_ham *h, int n_occ, int n_band, int n_pert, int n_omega, const sgw_opts &o,
                          int n_systems);
// warm: start from x = dpsi (caller order) instead of the guess of o.guess
sgw_status ps_solve(sgw_ctx *ctx, const PsProblem &P, const sgw_opts &o, const std::vector<int32_t> &systems,
                    bool warm, void *workspace, size_t workspace_bytes, double2 *dpsi, sgw_solve_info *info,
                    int *n_bad_out);

// MLP launchers (mlp.hip)
sgw_status mlp_upload_bf16(sgw_ctx *ctx, sgw_mlp *m);

}  // namespace sgw
