/*
 * sgw.h - C ABI of the MI355X Sternheimer library (libsgw.so).
 *
 * The library solves the linear Sternheimer equations of the SternheimerGW
 * method (Schlipf, Lambert, Zibouche, Giustino; Sec. 2.3, Eqs. 6-8):
 *
 *     (H_{k+q} - eps_v - z_j + alpha * P_occ) dpsi_{v,p}(z_j) = -(1 - P_occ) dV_p psi_v
 *
 * for many occupied bands v, perturbations dV_p(r) = exp(i (q + G_p).r) and
 * complex frequencies z_j = omega_j + i*eta.  All frequencies of one (v, p)
 * share one Krylov space (Sec. 2.2: shifted systems span the same Krylov
 * subspace).  H is applied in plane waves: kinetic diagonal 0.5|k+G|^2 plus the
 * local potential multiplied on the real-space grid through 3D FFTs (Sec. 2.1).
 *
 * Conventions
 *  - Hartree atomic units, lengths in bohr.
 *  - sgw_c128 is two doubles (re, im): the layout of one complex128 element.
 *  - Plane-wave vectors are indexed in the caller's order: the order of the
 *    Miller list given to sgw_ham_create.  G_m = m0*b0 + m1*b1 + m2*b2.
 *  - Real-space grids are [N0][N1][N2] with the last index fastest; grid point
 *    j sits at r_j = sum_d (j_d/N_d) a_d.  The local-potential operator is the
 *    grid-defined one: its plane-wave matrix element between m and m' is the
 *    discrete Fourier coefficient of V(r_j) at (m - m') mod N (aliasing included).
 *  - "device" arrays are device memory of the context's device (for example
 *    torch CUDA tensors); "host" arrays are ordinary host memory.  The library
 *    never frees or retains caller memory beyond a call.
 *  - Every call enqueues its GPU work on the context's stream.  sternheimer_solve
 *    and sgw_apply_h return after their GPU work has completed (the solver
 *    schedules work from the host and waits on the stream).
 *  - Errors: a negative status and a message from sgw_last_error(); the library
 *    never aborts or throws across this boundary.  Argument errors are found
 *    before any GPU work is enqueued.
 *  - One context per host thread and stream; calls on one context must not overlap.
 */
#ifndef SGW_H
#define SGW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } sgw_c128;

typedef enum {
  SGW_OK = 0,
  SGW_NOT_CONVERGED = 1,      /* finished; at least one solve missed tol (see info flags) */
  SGW_ERR_INVALID_ARG = -1,
  SGW_ERR_HIP = -2,           /* a HIP runtime call failed */
  SGW_ERR_WORKSPACE = -3,     /* workspace missing or too small */
  SGW_ERR_UNSUPPORTED = -4    /* valid request this build does not implement (e.g. grid size) */
} sgw_status;

/* per-solve flags (sgw_solve_info.flags, bitwise) */
enum {
  SGW_FLAG_CONVERGED = 1,     /* true FP64 relative residual <= tol */
  SGW_FLAG_MAXITER = 2,       /* Krylov space reached max_iter before the estimate met tol */
  SGW_FLAG_BREAKDOWN = 4,     /* invariant Krylov subspace found (solution exact in it) */
  SGW_FLAG_NONFINITE = 8,     /* NaN or Inf met in the recurrence or the result */
  SGW_FLAG_ZERO_RHS = 16      /* right-hand side zero to working precision, i.e.
                                 ||(1 - P_occ) s|| <= 1e-13 ||s||: dpsi = 0, relres = 0 */
};

enum { SGW_FP64 = 0 };        /* precision modes */

typedef struct sgw_ctx sgw_ctx;
typedef struct sgw_ham sgw_ham;

/* Last error message of the calling thread ("" if none). Never NULL. */
const char *sgw_last_error(void);

/* Library version string. */
const char *sgw_version(void);

/*
 * Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  The stream is borrowed.
 */
sgw_status sgw_ctx_create(int device, void *hip_stream, sgw_ctx **out);
sgw_status sgw_ctx_destroy(sgw_ctx *ctx);

/*
 * Kernel timing: for the kernels named in `kernels` (comma-separated names as
 * in sgw_kernel_stats, "all", or NULL/"" for none) the context records HIP
 * events around every launch on its stream and accumulates, per kernel, the
 * launch count, total duration and the algorithmic bytes and flops those
 * launches were charged with.  Unknown names: SGW_ERR_INVALID_ARG.
 */
sgw_status sgw_ctx_set_profiling(sgw_ctx *ctx, const char *kernels);
/* Clears all accumulated kernel statistics. */
sgw_status sgw_ctx_reset_stats(sgw_ctx *ctx);
/*
 * Statistics of kernel `name` ("hx_sticks_inv", "hx_planes", "hx_sticks_fwd",
 * "proj_dot", "lanczos_step", "combine", "residual", ...).  Outputs may be NULL.
 * Durations are summed over launches, in milliseconds.
 */
sgw_status sgw_kernel_stats(sgw_ctx *ctx, const char *name, int64_t *launches, double *total_ms,
                            double *alg_bytes, double *alg_flops);

/*
 * Hamiltonian at one Bloch vector (Sec. 2.1, Eq. 1): the plane-wave basis and
 * the local potential on the FFT grid.
 */
typedef struct {
  int32_t grid[3];          /* N0, N1, N2; each in {16, 24, 32, 48, 64, 72} */
  double recip[3][3];       /* rows b_i of the reciprocal lattice, bohr^-1 */
  double kvec[3];           /* Cartesian Bloch vector, bohr^-1 */
  int32_t n_pw;             /* number of plane waves */
  const int32_t *miller;    /* host [n_pw][3]; distinct; 2*max|m_d| + 1 <= N_d required */
  const double *v_loc;      /* device [N0][N1][N2], Ha; read during sgw_ham_create only */
} sgw_ham_desc;

/*
 * Builds the index maps (sticks along axis 2, permutation to the internal
 * stick-major order, lookup box of the Miller set) and a plane-major copy of
 * the potential on the device.  The descriptor's arrays may be released after
 * the call returns.
 */
sgw_status sgw_ham_create(sgw_ctx *ctx, const sgw_ham_desc *desc, sgw_ham **out);
sgw_status sgw_ham_destroy(sgw_ham *ham);
/* Number of plane waves of a Hamiltonian. */
int32_t sgw_ham_npw(const sgw_ham *ham);

/*
 * y = H x for n_vec vectors (Sec. 2.1): y_G = 0.5|k+G|^2 x_G + [F V F^-1 x]_G
 * with F^-1 x (r_j) = sum_G x_G exp(i G.r_j) and F f (G) = (1/N) sum_j f_j exp(-i G.r_j).
 * x, y: device [n_vec][n_pw] in the caller's order; may not alias.
 */
sgw_status sgw_apply_h(sgw_ctx *ctx, const sgw_ham *ham, int n_vec, const sgw_c128 *x, sgw_c128 *y);

/*
 * Occupied-manifold projector (Sec. 2.3, Eqs. 7-8), applied to n_vec vectors:
 *   mode 0:  y = x - Psi (Psi^H x)          (the conduction projector 1 - P_occ)
 *   mode 1:  y = y + alpha * Psi (Psi^H x)   (the + alpha P_occ term of the operator)
 * psi: device [n_occ][n_pw] (rows are orthonormal occupied states), x, y: device
 * [n_vec][n_pw], caller's order.  x and y may not alias.
 */
sgw_status sgw_apply_projector(sgw_ctx *ctx, const sgw_ham *ham, int n_occ, const sgw_c128 *psi,
                               int n_vec, const sgw_c128 *x, sgw_c128 *y, double alpha, int mode);

/*
 * Right-hand sides (Sec. 2.3, Eq. 8, with a minus sign):
 *   b_{v,p} = -(1 - P_occ) [exp(i (q+G_p).r) psi_v]
 * where the product moves the coefficient of G (basis at k) to G + G_p (basis at
 * k+q): s(G'') = psi_v(G'' - G_p) if G'' - G_p is in the basis at k, else 0.
 * psi_v: device [n_band][n_pw_k]; psi_occ_kq: device [n_occ][n_pw_kq];
 * dv_miller: host [n_pert][3]; b: device [n_band][n_pert][n_pw_kq].
 */
sgw_status sgw_build_rhs(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                         const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, int n_pert,
                         const int32_t *dv_miller, sgw_c128 *b);

typedef struct {
  int32_t precision;        /* SGW_FP64 (only mode of this build) */
  int32_t max_iter;         /* Krylov dimension limit per (v,p); <= 0 -> 600 */
  double alpha_pv;          /* coefficient of P_occ in the operator, Ha; <= 0 -> 1.0 */
  double tol_safety;        /* the recurrence stops when every shift's estimated residual
                               is below tol*tol_safety; <= 0 -> 0.5 */
  int32_t slots;            /* (v,p) pairs iterated concurrently; <= 0 -> automatic */
  int32_t finalize_batch;   /* pairs per finalisation batch; <= 0 -> automatic */
  int32_t steps_per_sync;   /* Krylov steps between host polls; <= 0 -> 8 */
  int32_t reserved;
} sgw_opts;

/* Fills *opts with the defaults. */
sgw_status sgw_opts_default(sgw_opts *opts);

typedef struct {
  int32_t iters;            /* Krylov dimension used (matrix-vector products of the seed) */
  int32_t flags;            /* SGW_FLAG_* */
  double relres;            /* true FP64 ||b - A_z x|| / ||b||, A_z applied afresh to x */
  double occ_leak;          /* ||Psi^H x|| / ||x|| (0 for x = 0) */
} sgw_solve_info;

/*
 * Device workspace needed by sternheimer_solve for these sizes and options.
 */
sgw_status sternheimer_workspace_size(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, int n_band,
                                      int n_pert, int n_omega, const sgw_opts *opts, size_t *bytes);

/*
 * The Sternheimer solves (Sec. 2.3, Eqs. 6-8; shifts sharing one Krylov space,
 * Sec. 2.2).  For every band v < n_band, perturbation p < n_pert and frequency
 * j < n_omega:
 *
 *   (H_{k+q} - eps_v[v] - z_j + alpha P_occ) dpsi[v][p][j] = b_{v,p}   (b as in sgw_build_rhs)
 *
 * with z_j = omega[j] + i*eta (eta != 0; the sign selects the time ordering).
 *
 * h_kq        Hamiltonian at k+q (its basis is the solution's basis)
 * psi_occ_kq  device [n_occ][n_pw_kq], orthonormal occupied states at k+q
 * h_k         Hamiltonian at k (only its basis is used: the Miller set of psi_v)
 * psi_v       device [n_band][n_pw_k], the unperturbed states
 * eps_v       host [n_band], their energies (Ha)
 * dv_miller   host [n_pert][3], Miller indices of G_p; q = k_kq - k
 * omega       host [n_omega] (Ha)
 * tol         target true relative residual (FP64), > 0
 * workspace   device, >= sternheimer_workspace_size bytes, 256-byte aligned
 * dpsi        device out [n_band][n_pert][n_omega][n_pw_kq]
 * info        device out [n_band][n_pert][n_omega]
 * Returns SGW_OK when every solve converged, SGW_NOT_CONVERGED when some did
 * not (their best iterate and flags are still written), or an error.
 */
sgw_status sternheimer_solve(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                             const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, const double *eps_v,
                             int n_pert, const int32_t *dv_miller, int n_omega, const double *omega,
                             double eta, double tol, const sgw_opts *opts, void *workspace,
                             size_t workspace_bytes, sgw_c128 *dpsi, sgw_solve_info *info);

#ifdef __cplusplus
}
#endif
#endif /* SGW_H */
