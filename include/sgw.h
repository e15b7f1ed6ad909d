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
  SGW_ERR_UNSUPPORTED = -4    /* valid request the library does not implement (e.g. grid size) */
} sgw_status;

/* per-solve flags (sgw_solve_info.flags, bitwise) */
enum {
  SGW_FLAG_CONVERGED = 1,     /* true FP64 relative residual <= tol */
  SGW_FLAG_MAXITER = 2,       /* Krylov space reached max_iter before the estimate met tol */
  SGW_FLAG_BREAKDOWN = 4,     /* invariant Krylov subspace found (solution exact in it) */
  SGW_FLAG_NONFINITE = 8,     /* NaN or Inf met in the recurrence or the result */
  SGW_FLAG_ZERO_RHS = 16,     /* right-hand side zero to working precision, i.e.
                                 ||(1 - P_occ) s|| <= 1e-13 ||s||: dpsi = 0, relres = 0 */
  SGW_FLAG_PER_SHIFT = 32     /* finished by the per-shift solver: iters counts its
                                 BiCGStab iterations (two operator applications each) */
};

/* precision modes */
enum {
  SGW_FP64 = 0,               /* complex128 throughout */
  SGW_MIXED = 1               /* a (v,p) pair's Krylov steps apply the potential term of H.x in
                                 complex64 (FP32 transforms and V) and the occupied projector as a
                                 split-BF16 contraction (SGW_PROJ_SPLIT_BF16) once the estimated
                                 residuals of all its shifts are below mixed_switch * tol (matvec
                                 errors made late enter the solutions weighted by the shrinking step
                                 coefficients); the recurrences, basis and residuals stay FP64, and
                                 every shift whose true FP64 residual is still above tol is then
                                 refined by FP64 per-shift solves from its multishift iterate */
};

/* sgw_apply_projector: with this bit in `mode` the contraction runs on the BF16 matrix cores: every
   FP64 value is split into three BF16 terms (h = bf16(v), m = bf16(v - h), l = bf16(v - h - m)),
   each real product keeps the six largest term products, accumulated in FP32 (FP32-level accuracy,
   the terms dropped are below 2^-24 relative) */
enum { SGW_PROJ_SPLIT_BF16 = 16 };

/* solver (sgw_opts.solver) */
enum {
  SGW_SOLVER_MULTISHIFT = 0,  /* all shifts of one (v,p) share one Krylov space (Sec. 2.2) */
  SGW_SOLVER_PER_SHIFT = 1,   /* every (v,p,z) its own preconditioned BiCGStab solve */
  SGW_SOLVER_TAIL = 2,        /* multishift up to Krylov dimension tail_iter, then the shifts
                                 still above tol continue per shift, warm-started from the
                                 multishift iterate */
  SGW_SOLVER_BLOCK = 3        /* all perturbations and shifts of one band v share one block Krylov
                                 space (block Lanczos over the n_pert right-hand sides, FOM
                                 solutions per shift; Secs. 2.2-2.3): FP64 only, no preconditioner
                                 or guess; more than 32 perturbations are split into ceil(n_pert/32)
                                 blocks of near-equal size, solved one after another; max_iter
                                 limits the block steps, info.iters reports them; slots > 0 caps
                                 the bands iterated together (default: as many as a 144 GiB
                                 workspace holds, all bands if it can); solves whose estimate met
                                 the threshold while the true residual missed tol are refined per
                                 shift, as after the plain multishift solver; a band whose block
                                 loses rank (linearly dependent or zero right-hand sides, or a
                                 block space that stops growing in some direction) keeps the steps
                                 before it, and its solutions that miss tol are refined the same
                                 way */
};
/* diagonal preconditioner of the per-shift solves (sgw_opts.precond) */
enum { SGW_PC_NONE = 0, SGW_PC_TETER = 1, SGW_PC_LEARNED = 2 };
/* initial guess of the per-shift solves (sgw_opts.guess); TAIL always warm-starts */
enum { SGW_GUESS_ZERO = 0, SGW_GUESS_LEARNED = 1 };
/*
 * Kernel of the plane pass of the FP64 H.x (sgw_opts.fft_planes, sgw_ctx_set_fft_planes): the
 * 2D inverse FFT of a plane, the potential and the 2D forward FFT (Sec. 2.1).
 *   SGW_FFT_AUTO  the built-in choice: LINE where it applies, else TRI, else PAIR, else LDS
 *   SGW_FFT_LINE  one thread per row or column, the whole line in registers: lines of at most 48
 *                 points whose sticks lie in the central half of the plane (|m| < N/4)
 *   SGW_FFT_PAIR  two threads per line, split by real-space parity: lines of at most 72 points in
 *                 the central half
 *   SGW_FFT_LDS   the whole plane in LDS, radix stages exchanged through it: every grid
 *   SGW_FFT_TRI   three threads per line, split by the real-space index mod 3: lines of 24, 48 or
 *                 72 points in the central half
 * A kernel that does not apply to a grid falls back to the built-in choice; the FP32 potential
 * path of SGW_MIXED always takes the built-in choice (PAIR has no FP32 form).  All give H.x to
 * rounding.
 */
enum { SGW_FFT_AUTO = 0, SGW_FFT_LINE = 1, SGW_FFT_PAIR = 2, SGW_FFT_LDS = 3, SGW_FFT_TRI = 4 };

typedef struct sgw_ctx sgw_ctx;
typedef struct sgw_ham sgw_ham;
typedef struct sgw_mlp sgw_mlp;

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
/*
 * Plane-pass kernel of this context's H.x (SGW_FFT_*): used by sgw_apply_h and by solves whose
 * sgw_opts.fft_planes is SGW_FFT_AUTO.  Default SGW_FFT_AUTO.  Other values: SGW_ERR_INVALID_ARG.
 */
sgw_status sgw_ctx_set_fft_planes(sgw_ctx *ctx, int fft_planes);
/*
 * The plane-pass kernel (SGW_FFT_LINE, SGW_FFT_PAIR or SGW_FFT_LDS) that H.x of `ham` runs under the
 * context's setting, for `precision` SGW_FP64 or SGW_MIXED (the FP32 potential path); *out.
 */
sgw_status sgw_plane_kernel(sgw_ctx *ctx, const sgw_ham *ham, int precision, int32_t *out);
/* Clears all accumulated kernel statistics. */
sgw_status sgw_ctx_reset_stats(sgw_ctx *ctx);
/*
 * Statistics of kernel `name` ("hx_sticks_inv", "hx_planes", "hx_sticks_fwd",
 * "proj_dot", "lanczos_step", "combine", "residual", "nl_dot", "nl_apply", "blk_product" (the block
 * solver's final batched products X = V Y, (AV) Y, (psi^H V) Y, one rocBLAS launch each), ...).
 * Outputs may be NULL.
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
 * Non-local part of the pseudopotential, represented in reciprocal space (Sec. 2.1, the text after
 * Eq. 1), in the fully separable form V_NL = sum_p |beta_p> E_p <beta_p|: every later H.x of `ham`
 * (sgw_apply_h, the solves, the Green's function columns) adds
 *     [V_NL x]_G = sum_p E_p beta_p(G) sum_G' conj(beta_p(G')) x_G'
 * as two FP64 matrix-core contractions (in every precision mode).  A Hermitian coupling matrix
 * between the projectors of an atom reduces to this form by diagonalising it.
 *   n_proj  number of projectors, 0 <= n_proj <= 4096 (above: SGW_ERR_UNSUPPORTED); 0 removes the term
 *   beta    device [n_proj][n_pw] complex128, rows in the caller's plane-wave order; copied into
 *           memory the Hamiltonian owns before the call returns
 *   e_kb    host [n_proj] energies E_p in Ha, finite
 * Replaces any earlier projectors.  The call waits for the context's stream first; it must not run
 * while another stream or thread uses `ham`.  Set it before sizing workspaces (the H.x scratch of a
 * solve holds the projector overlaps).  NULL arguments, negative n_proj or non-finite energies:
 * SGW_ERR_INVALID_ARG.
 */
sgw_status sgw_ham_set_nonlocal(sgw_ctx *ctx, sgw_ham *ham, int n_proj, const sgw_c128 *beta, const double *e_kb);
/* Number of non-local projectors of a Hamiltonian (0: none). */
int32_t sgw_ham_nproj(const sgw_ham *ham);

/*
 * y = H x for n_vec vectors (Sec. 2.1): y_G = 0.5|k+G|^2 x_G + [F V F^-1 x]_G (+ [V_NL x]_G when
 * the Hamiltonian has non-local projectors, sgw_ham_set_nonlocal)
 * with F^-1 x (r_j) = sum_G x_G exp(i G.r_j) and F f (G) = (1/N) sum_j f_j exp(-i G.r_j).
 * x, y: device [n_vec][n_pw] in the caller's order; may not alias.
 * precision SGW_FP64, or SGW_MIXED: the potential term in FP32 (x rounded to
 * complex64, FP32 transforms and V(r)), the kinetic term and y in FP64.
 */
sgw_status sgw_apply_h(sgw_ctx *ctx, const sgw_ham *ham, int n_vec, const sgw_c128 *x, sgw_c128 *y,
                       int precision);

/*
 * sgw_apply_h without device allocation, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * result as sgw_apply_h, bit for bit.  Its scratch (x and y in the library's internal plane-wave
 * order and the stick buffer between the FFT passes) lives in one fixed 64 MiB device array per GPU,
 * held until the process ends: n_vec * (32 n_pw + 16 max(N2 n_sticks, n_chunks n_proj)) bytes, with
 * n_chunks = ceil(n_pw / 256) (each part rounded up to 256), must fit, about 170 vectors of the
 * 16-atom cell (48^3 grid) or 45 of the 64-atom cell (72^3);
 * larger calls return SGW_ERR_WORKSPACE before any GPU work.  No scratch value has to start at zero:
 * every kernel writes each scratch element before reading it.  Every call on one GPU shares that GPU's
 * array, so calls that overlap on one GPU (other contexts, streams or host threads) race; calls on one
 * context are serial (each returns after its GPU work has completed).  Kernel timing
 * (sgw_ctx_set_profiling) does not record these calls.
 */
sgw_status sgw_apply_h_noalloc(sgw_ctx *ctx, const sgw_ham *ham, int n_vec, const sgw_c128 *x, sgw_c128 *y,
                               int precision);

/*
 * Density response to the plane-wave perturbations (Sec. 2.3, Eq. 5), from the linear variations
 * that two sternheimer_solve calls return: dpsi_plus at the shifts z_j = omega_j + i eta and
 * dpsi_minus at -z_j (omega -> -omega_j, eta -> -eta), both [n_band][n_pert][n_omega][n_pw_kq]
 * device arrays in the layout sternheimer_solve writes.  With the same h_kq, psi_occ_kq, h_k, psi_v
 * and dv_miller as those solves:
 *     chi[j][g][h] (+)= weight * (2 / Omega) * sum_v < exp(i (q+G_g) . r) u_v | dpsi_{v,h}(z_j) + dpsi_{v,h}(-z_j) >
 * i.e. the Fourier component q + G_g of 2 sum_v u_v^* (du_v(z) + du_v(-z)) per unit cell (Omega
 * from h_kq's reciprocal lattice; 2: spin), the response at q + G_g to the unit perturbation
 * exp(i (q+G_h) . r).  The bra is taken as (1 - P_occ) exp(i (q+G) . r) u_v (the variations have no
 * occupied component).  weight: the Brillouin-zone weight of the k point (1 / N_k for a uniform
 * grid); accumulate = 0 overwrites chi, 1 adds to it (a sum over k points).
 *   chi  device [n_omega][n_pert][n_pert] complex128, out (or in/out)
 * Allocates its scratch (the right-hand sides of all bands, n_band * n_pert * n_pw_kq complex, and
 * the band's overlap partials); returns after the GPU work.  NULL arrays, negative sizes or a
 * non-finite weight: SGW_ERR_INVALID_ARG.
 */
sgw_status sgw_density_response(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                                const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, int n_pert,
                                const int32_t *dv_miller, int n_omega, const sgw_c128 *dpsi_plus,
                                const sgw_c128 *dpsi_minus, double weight, int accumulate, sgw_c128 *chi);

/*
 * Coulomb potential of the wave vectors q + G_p (Hartree units; q = k of h_kq minus k of h_k,
 * G_p = dv_miller[p] on h_kq's reciprocal lattice): 4 pi / |q+G|^2, or with r_cut > 0 the spherical
 * truncation (Sec. 2.6, Eq. 12) 4 pi / |q+G|^2 (1 - cos(|q+G| r_cut)), 2 pi r_cut^2 at q + G = 0.
 *   v  host [n_pert] out
 * q + G = 0 with r_cut <= 0: SGW_ERR_INVALID_ARG.
 */
sgw_status sgw_coulomb(const sgw_ham *h_kq, const sgw_ham *h_k, int n_pert, const int32_t *dv_miller, double r_cut,
                       double *v);

/*
 * Dielectric matrix, its inverse and the correlation part of the screened interaction per frequency
 * (Sec. 2.3, Eq. 4; Sec. 2.4, Eq. 9), from chi of sgw_density_response and v of sgw_coulomb:
 *     eps_{gh}   = delta_{gh} - chi_{gh} v_h          (the perturbing charge's potential on the columns)
 *     W_bar_{gh} = v_g (eps^{-1}_{gh} - delta_{gh})   (rows), off-diagonal elements zero in the row and
 *                                                      column of a q + G = 0 (Sec. 2.4)
 * (together W_bar = W - v with W = v (1 - chi v)^{-1}).  eps^{-1} by Gauss-Jordan elimination with
 * partial pivoting in FP64, one workgroup per frequency.
 *   chi                 device [n_omega][n_pert][n_pert] in
 *   eps, eps_inv, wbar  device [n_omega][n_pert][n_pert] out; any may be NULL
 * n_pert above 64: SGW_ERR_UNSUPPORTED.  Errors of sgw_coulomb are passed on.
 */
sgw_status sgw_screened_coulomb(sgw_ctx *ctx, const sgw_ham *h_kq, const sgw_ham *h_k, int n_pert,
                                const int32_t *dv_miller, double r_cut, int n_omega, const sgw_c128 *chi,
                                sgw_c128 *eps, sgw_c128 *eps_inv, sgw_c128 *wbar);

/*
 * Occupied-manifold projector (Sec. 2.3, Eqs. 7-8), applied to n_vec vectors:
 *   mode 0:  y = x - Psi (Psi^H x)          (the conduction projector 1 - P_occ)
 *   mode 1:  y = y + alpha * Psi (Psi^H x)   (the + alpha P_occ term of the operator)
 * psi: device [n_occ][n_pw] (rows are orthonormal occupied states), x, y: device
 * [n_vec][n_pw], caller's order.  x and y may not alias.  n_occ above 256: SGW_ERR_UNSUPPORTED.
 * mode | SGW_PROJ_SPLIT_BF16: the same with the split-BF16 contraction (FP32-level accuracy).
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
 * n_occ above 256: SGW_ERR_UNSUPPORTED.
 */
sgw_status sgw_build_rhs(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                         const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, int n_pert,
                         const int32_t *dv_miller, sgw_c128 *b);

typedef struct {
  int32_t precision;        /* SGW_FP64 or SGW_MIXED (not with the per-shift solver) */
  int32_t max_iter;         /* Krylov dimension limit per (v,p); <= 0 -> 600 */
  double alpha_pv;          /* coefficient of P_occ in the operator, Ha; <= 0 -> 1.0 */
  double tol_safety;        /* the recurrence stops when every shift's estimated residual
                               is below tol*tol_safety; <= 0 -> 0.5 */
  int32_t slots;            /* (v,p) pairs iterated concurrently; <= 0 -> automatic (as many as
                               a 144 GiB workspace holds, at most all pairs); block solver: the
                               most bands per chunk */
  int32_t finalize_batch;   /* pairs per finalisation batch; <= 0 -> automatic */
  int32_t steps_per_sync;   /* Krylov steps between host polls; <= 0 -> 8 */
  int32_t solver;           /* SGW_SOLVER_* (default MULTISHIFT) */
  int32_t precond;          /* SGW_PC_* for per-shift solves (default NONE): the per-shift solver
                               and the per-shift phases of TAIL and MIXED; a preconditioner or a
                               non-zero initial guess breaks the shared Krylov space, so a plain
                               FP64 multishift solve accepts only NONE / ZERO */
  int32_t guess;            /* SGW_GUESS_* for per-shift solves (default ZERO) */
  int32_t tail_iter;        /* TAIL: multishift Krylov dimension cap; <= 0 -> 160 */
  int32_t ps_max_iter;      /* per-shift BiCGStab iteration limit; <= 0 -> 2000 */
  int32_t ps_slots;         /* per-shift systems iterated concurrently; <= 0 -> automatic */
  const sgw_mlp *mlp;       /* model for PC_LEARNED / GUESS_LEARNED (same device), else NULL */
  sgw_c128 *hist_r;         /* optional device out [n_band][n_pert][n_omega][n_pw_kq]: per-shift
                               residual r_k after hist_iter iterations (caller's order); left
                               untouched for solves that finished earlier */
  sgw_c128 *hist_x;         /* optional device out, same shape: the iterate x_k with r_k */
  int32_t hist_iter;        /* iteration of the snapshot (> 0 with hist_r, hist_x) */
  double mixed_switch;      /* SGW_MIXED: a pair's steps use FP32 potential matvecs once all its
                               shifts' estimated residuals are below mixed_switch * tol; <= 0 -> 1e4 */
  int32_t graph;            /* 1: the multishift solver captures the Krylov steps between two
                               polls in a HIP graph and replays it (re-captured when the number
                               of active slots changes; ignored while kernel timing is on and
                               on the legacy default stream, which cannot be captured) */
  int32_t fft_planes;       /* plane-pass kernel of the FP64 H.x (SGW_FFT_*); SGW_FFT_AUTO: the
                               context's setting (sgw_ctx_set_fft_planes) */
  int32_t basis_blocks;     /* Krylov bases of the multishift slots.  0: each slot holds max_iter + 1
                               vectors when the workspace budget allows one slot per (v,p) pair;
                               otherwise 4x the slots draw their vectors from a pool of the same
                               memory in blocks of 32 as they grow, a pair being admitted only when
                               the pool can carry the admitted pairs to their expected Krylov
                               dimension.  > 0: a pool of this many blocks (at least (max_iter + 1)
                               / 32 rounded up), admitting whenever blocks for a pair's first steps
                               are free.  A pair that cannot grow waits; when no running pair can
                               grow, the least advanced one is restarted later.  Results do not
                               change. */
  const double *shift_imag; /* optional host [n_omega]: shift j is omega[j] + i shift_imag[j] (each
                               finite) instead of omega[j] + i eta, e.g. frequencies on the
                               imaginary axis; NULL: eta for every shift.  The shifts still share
                               one Krylov space (any complex shift of the Hermitian operator does) */
} sgw_opts;

/* Fills *opts with the defaults. */
sgw_status sgw_opts_default(sgw_opts *opts);

typedef struct {
  int32_t iters;            /* Krylov dimension at which this shift's residual estimate met the
                               stopping threshold (the pair's full dimension if it never did) */
  int32_t flags;            /* SGW_FLAG_* */
  double relres;            /* true FP64 ||b - A_z x|| / ||b||, A_z applied afresh to x */
  double occ_leak;          /* ||Psi^H x|| / ||x|| (0 for x = 0) */
} sgw_solve_info;

/*
 * Device workspace needed by sternheimer_solve for these sizes and options.  Multishift: the slots
 * that a 144 GiB budget holds (opts.slots overrides).  Block solver: one chunk of bands, as many as
 * the 144 GiB budget holds (opts.slots caps them), each band holding its basis and its products AV
 * for max_iter + 1 block steps (2 x 16 (max_iter + 1) min(n_pert, 32) n_pw bytes) beside the
 * per-shift block recurrences and one run of final products; a larger workspace given to the solve
 * is used for larger chunks.
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
 * not (their best iterate and flags are still written), or an error;
 * SGW_ERR_UNSUPPORTED for n_occ > 256 or a k+q basis above 16384 plane waves.
 */
sgw_status sternheimer_solve(sgw_ctx *ctx, const sgw_ham *h_kq, int n_occ, const sgw_c128 *psi_occ_kq,
                             const sgw_ham *h_k, int n_band, const sgw_c128 *psi_v, const double *eps_v,
                             int n_pert, const int32_t *dv_miller, int n_omega, const double *omega,
                             double eta, double tol, const sgw_opts *opts, void *workspace,
                             size_t workspace_bytes, sgw_c128 *dpsi, sgw_solve_info *info);

/*
 * Pair elements of the Green's function for the correlation self-energy (Sec. 2.4, Eq. 10; Sec. 2.2):
 *     m[n][j][g][h] = < t_{n,g} | (z_j - H)^{-1} | t_{n,h} >,   t_{n,g} = exp(-i (q+G_g) . r) u_n,
 * z_j = z_re[j] + i z_im[j], q = k of h_k minus k of h_kmq, G_g = g_miller[g] on h_kmq's reciprocal
 * lattice.  On the imaginary axis z_j = mu + i w'_j (mu: the chemical potential, in the gap); on the
 * real axis z_j = w'_j + i eta_j with the sign of eta_j chosen by the caller for the time ordering
 * (positive above mu, negative below).  All z_j of one (n, h) share one Krylov space (the multishift
 * solver with per-shift imaginary parts, no occupied projector, zero band energy: the solve of
 * (H - z_j) x = -t_{n,h}); the bra is a plane-wave contraction on the FP64 matrix cores.
 *   psi_n    device [n_band][n_pw of h_k] states u_n at k (caller's order)
 *   g_miller host [n_g][3]; z_re, z_im host [n_freq] (finite)
 *   opts     solver options (NULL: defaults; its shift_imag is replaced by z_im)
 *   m_out    device [n_band][n_freq][n_g][n_g] out;  info  device [n_band][n_g][n_freq] or NULL
 *   workspace device, >= sgw_green_pair_workspace_size bytes (same sizes and opts), 256-byte aligned:
 *            the solver's workspace, the solutions (n_band n_g n_freq vectors of h_kmq's basis), the
 *            right-hand sides and the overlaps; nothing is allocated
 * Returns the solve's status (SGW_NOT_CONVERGED when a solve missed tol; m_out is still written),
 * SGW_ERR_WORKSPACE for a missing, short or misaligned workspace.
 */
sgw_status sgw_green_pair_workspace_size(sgw_ctx *ctx, const sgw_ham *h_kmq, int n_band, int n_g, int n_freq,
                                         const sgw_opts *opts, size_t *bytes);
sgw_status sgw_green_pair_elements(sgw_ctx *ctx, const sgw_ham *h_kmq, const sgw_ham *h_k, int n_band,
                                   const sgw_c128 *psi_n, int n_g, const int32_t *g_miller, int n_freq,
                                   const double *z_re, const double *z_im, double tol, const sgw_opts *opts,
                                   void *workspace, size_t workspace_bytes, sgw_c128 *m_out,
                                   sgw_solve_info *info);

/*
 * Diagonal correlation self-energy (Sec. 2.4, Eq. 10):
 *     sigma[n][k] = (alpha / (2 pi volume)) sum_j weights[j] sum_{g,h} wbar[w_index[k][j]][g][h] m_elem[n][j][g][h]
 * alpha = alpha_re + i alpha_im: -1 for the convolution along the imaginary axis (frequencies i w'_j,
 * W_bar at i (w'_j - w_k)), i along the real axis (W_bar at w'_j - w_k).  m_elem: the pair elements at
 * the integration frequencies (sgw_green_pair_elements), weighted by weights[j]; W_bar
 * (sgw_screened_coulomb) at the needed differences through w_index (host [n_out][n_freq], values
 * < n_w).  volume: the unit cell's, bohr^3.
 *   m_elem device [n_band][n_freq][n_g][n_g]; wbar device [n_w][n_g][n_g]; sigma device [n_band][n_out]
 */
sgw_status sgw_sigma_c(sgw_ctx *ctx, int n_band, int n_g, int n_freq, const sgw_c128 *m_elem, const double *weights,
                       int n_w, const sgw_c128 *wbar, int n_out, const int32_t *w_index, double volume,
                       double alpha_re, double alpha_im, sgw_c128 *sigma);

/*
 * Rational approximation of f at the points z by the adaptive Antoulas-Anderson algorithm (Sec. 2.7):
 * support points are added where the approximant is worst, the barycentric weights are the right
 * singular vector of the smallest singular value of the Loewner matrix of the other points (one-sided
 * Jacobi SVD), until max |f - r| <= tol max |f| or max_terms (at most n - 1) support points;
 *     r(x) = sum_s w_s f_s / (x - z_s) / sum_s w_s / (x - z_s).
 * Host arrays: z, f [n] in (distinct, finite); z_sup, f_sup, w_sup [max_terms] out; *n_sup out.
 * Runs in the calling thread (a few small SVDs); no GPU work.
 */
sgw_status sgw_aaa_fit(int n, const sgw_c128 *z, const sgw_c128 *f, double tol, int max_terms, int *n_sup,
                       sgw_c128 *z_sup, sgw_c128 *f_sup, sgw_c128 *w_sup);

/*
 * N-point Pade interpolant of f at the points z in continued-fraction form (the continuation Sec. 2.7
 * compares with AAA; Vidberg-Serene recursion):
 *     C(x) = a_0 / (1 + a_1 (x - z_0) / (1 + a_2 (x - z_1) / (1 + ...))),  C(z_i) = f_i.
 * sgw_pade_fit: a host [n] out; SGW_ERR_INVALID_ARG for repeated or non-finite points or a breakdown
 * (a zero intermediate value).  sgw_pade_eval: C at the host points x [n_x] into out [n_x], by the
 * three-term recursion of the numerators and denominators.  Host only.
 */
sgw_status sgw_pade_fit(int n, const sgw_c128 *z, const sgw_c128 *f, sgw_c128 *a);
sgw_status sgw_pade_eval(int n, const sgw_c128 *z, const sgw_c128 *a, int n_x, const sgw_c128 *x, sgw_c128 *out);

/*
 * Spectral function of each state (Sec. 2.8, Eq. 16) on real frequencies from its continued
 * self-energy: Sigma^c(w + i broad) = r_n(w + i broad) of the state's AAA approximant and
 *     A_n(w) = -Im Sigma^c(w) / (pi |w - eps_n - Sigma^c(w) - delta_n|^2),
 * delta_n = Sigma^x_n - V^xc_n (the static part, given).
 *   n_sup host [n_band]; z_sup, f_sup, w_sup host [n_band][n_sup_max]; omega host [n_omega];
 *   eps_n, delta host [n_band]; sigma device [n_band][n_omega] out (or NULL); a device [n_band][n_omega]
 *   out (or NULL)
 */
sgw_status sgw_spectral_function(sgw_ctx *ctx, int n_band, int n_sup_max, const int32_t *n_sup,
                                 const sgw_c128 *z_sup, const sgw_c128 *f_sup, const sgw_c128 *w_sup, int n_omega,
                                 const double *omega, double broad, const double *eps_n, const double *delta,
                                 sgw_c128 *sigma, double *a);

/*
 * Linearised quasiparticle energy (Sec. 2.8, Eq. 17) from a state's approximant r:
 * eps_qp = eps_n + Z (Re r(eps_n) + delta), Z = 1 / (1 - Re r'(eps_n)).  Host only.
 */
sgw_status sgw_quasiparticle(int n_sup, const sgw_c128 *z_sup, const sgw_c128 *f_sup, const sgw_c128 *w_sup,
                             double eps_n, double delta, double *eps_qp, double *z_factor);

/*
 * Green's function columns (Sec. 2.2, Eqs. 2-3): for every column index c < n_col and frequency
 * j < n_omega, the solution of
 *
 *   (H_k - z_j) G_{.G'}(z_j) = -e_{G'},   G' = cols[c],   z_j = omega[j] + i*eta,
 *
 * i.e. column G' of G(z_j) = (z_j - H_k)^{-1}, with all frequencies sharing one Krylov space, as in
 * sternheimer_solve (the same solver, options and flags; no occupied projector, no band energy).
 * The paper takes the complex frequency on the side that satisfies the time ordering: here the
 * caller chooses the sign of eta (eta > 0 above the chemical potential, eta < 0 below), one call
 * per side.  With opts.solver = SGW_SOLVER_BLOCK the columns share one block Krylov space (the
 * operator is the same for all of them): blocks of at most 32 columns, info.iters in block steps.
 * h_k         the Hamiltonian (its basis is the columns' and the solution's basis)
 * cols        host [n_col], plane-wave indices G' in the caller's order, 0 <= cols[c] < n_pw
 * omega       host [n_omega] (Ha); eta != 0; tol > 0 as in sternheimer_solve
 * workspace   device, >= sgw_green_workspace_size bytes, 256-byte aligned
 * g           device out [n_col][n_omega][n_pw]
 * info        device out [n_col][n_omega] (relres = ||-e_{G'} - (H - z) x|| since ||e_{G'}|| = 1)
 * Returns SGW_OK, SGW_NOT_CONVERGED (some solve missed tol; flags tell which) or an error.
 */
sgw_status sgw_green_workspace_size(sgw_ctx *ctx, const sgw_ham *h_k, int n_col, int n_omega,
                                    const sgw_opts *opts, size_t *bytes);
sgw_status sgw_green_solve(sgw_ctx *ctx, const sgw_ham *h_k, int n_col, const int32_t *cols, int n_omega,
                           const double *omega, double eta, double tol, const sgw_opts *opts, void *workspace,
                           size_t workspace_bytes, sgw_c128 *g, sgw_solve_info *info);

/*
 * Batches of independent systems (each a Sternheimer problem of Sec. 2.3,
 * Eqs. 6-8, with its own Hamiltonians, bands, perturbations and frequencies).
 * The arguments of one sternheimer_solve call, plus per-system options and outputs.
 */
typedef struct {
  const sgw_ham *h_kq;
  const sgw_ham *h_k;
  int32_t n_occ, n_band, n_pert, n_omega;
  const sgw_c128 *psi_occ_kq;   /* device [n_occ][n_pw_kq] */
  const sgw_c128 *psi_v;        /* device [n_band][n_pw_k] */
  const double *eps_v;          /* host [n_band] */
  const int32_t *dv_miller;     /* host [n_pert][3] */
  const double *omega;          /* host [n_omega] */
  double eta, tol;
  sgw_opts opts;                /* per-system options (for example from sgw_autotune) */
  sgw_c128 *dpsi;               /* device out [n_band][n_pert][n_omega][n_pw_kq] */
  sgw_solve_info *info;         /* device out [n_band][n_pert][n_omega] */
  int32_t status;               /* out: this system's sgw_status */
  int32_t worker;               /* out: worker stream that solved it */
  double ms;                    /* out: wall time of its solve on that worker */
} sgw_problem;

/*
 * Workspace for sternheimer_solve_batch with n_workers workers: n_workers equal
 * parts, each large enough for every system with its slot count fitted to a
 * per-worker share of the default memory budget, and (n_workers > 1) at least
 * the single-solve workspace of every system that fills the GPU by itself (at
 * least 128 band x perturbation pairs of at least 4,096 plane waves).
 */
sgw_status sternheimer_batch_workspace_size(sgw_ctx *ctx, int n_sys, const sgw_problem *problems, int n_workers,
                                            size_t *bytes);
/*
 * Solves every system of the batch.  n_workers (1..16) worker streams of the
 * context's device, each driven by its own host thread, take systems from one
 * queue in order of decreasing predicted cost and solve them exactly as
 * sternheimer_solve would (results are identical), each in its own part of the
 * workspace; a multishift system's slot count is lowered to fit that part.
 * Small systems thereby share the GPU.  With n_workers > 1, the systems that
 * fill the GPU by themselves (see above) run first, one at a time over the whole
 * workspace with the options of a single solve (a share would cut their slots).
 * The workers start after the work already
 * enqueued on the context's stream; the call returns when all systems are done.
 * Returns the first error (problems[i].status tells which), else SGW_NOT_CONVERGED
 * if any system did not converge, else SGW_OK.  Kernel timing statistics of the
 * workers are added to the context's.
 */
sgw_status sternheimer_solve_batch(sgw_ctx *ctx, int n_sys, sgw_problem *problems, int n_workers, void *workspace,
                                   size_t workspace_bytes);
/*
 * Autotuner for the multishift solver: times the candidate settings of
 * steps_per_sync (4, 8, 16) and graph (0, 1) on a sample of the problem (its two
 * highest bands, up to eight perturbations, all frequencies; allocates the sample's
 * buffers) and writes problem->opts with the fastest of them to *best.  Results
 * are cached in the context per class (the grid, and n_pw, n_occ and n_omega each
 * to within a factor sqrt(2)); a cached class
 * returns at once with *tune_ms = 0.  tune_ms (may be NULL): wall time spent.
 */
sgw_status sgw_autotune(sgw_ctx *ctx, const sgw_problem *problem, sgw_opts *best, double *tune_ms);

/*
 * Learned diagonal preconditioner and initial guess for the per-shift solves
 * (not part of the paper; its solves replace the sum over empty states, Sec. 2.3,
 * and any preconditioner leaves their solution unchanged).  A 3-layer perceptron,
 * 5 -> 64 -> 64 -> 4 with tanh, evaluated per plane wave G of a system with band
 * energy eps and shift z = omega + i*eta (Ha), on the features
 *     f = (T/10, eps/10, omega, 100*eta, (T - eps - omega)/10),  T = 0.5|k+G|^2.
 * With outputs o and s = 1/(T + 1): preconditioner m_G = s (o0 + i o1), guess
 * x0_G = s (o2 + i o3) b_G.
 *
 * Parameters: FP32, sgw_mlp_num_params() of them, in this order (row-major):
 *     W1[64][5], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].
 * Inference inside the solver uses a BF16 rounding of the weights with FP32
 * arithmetic; sgw_mlp_forward / _grad / _train_step use the FP32 weights.
 *
 * Training rows: feat [n_rows][5] and target [n_rows][8] = (u_m, w_m, u_g, w_g) as
 * complex (re, im) pairs; the loss is the mean over rows of
 *     |m u_m - w_m|^2 + |g u_g - w_g|^2,   m = s (o0 + i o1), g = s (o2 + i o3).
 * feat, target, out, grad_out and loss_out are device arrays (FP32).
 */
int32_t sgw_mlp_num_params(void);
/* init_w: host [num_params] or NULL for a seeded Glorot-uniform start with m = g = s. */
sgw_status sgw_mlp_create(sgw_ctx *ctx, const float *init_w, uint64_t seed, sgw_mlp **out);
sgw_status sgw_mlp_destroy(sgw_mlp *mlp);
/* host copies of the FP32 master weights */
sgw_status sgw_mlp_get_weights(const sgw_mlp *mlp, float *w);
sgw_status sgw_mlp_set_weights(sgw_mlp *mlp, const float *w);
/* out [n_rows][4]: the raw outputs o */
sgw_status sgw_mlp_forward(sgw_ctx *ctx, const sgw_mlp *mlp, int n_rows, const float *feat, float *out);
/* grad_out [num_params]: d loss / d w; loss_out [1] (may be NULL).  Deterministic. */
sgw_status sgw_mlp_grad(sgw_ctx *ctx, const sgw_mlp *mlp, int n_rows, const float *feat, const float *target,
                        float *grad_out, float *loss_out);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr on the loss of these rows.
   loss_out: host [1] (may be NULL), the loss before the step. */
sgw_status sgw_mlp_train_step(sgw_ctx *ctx, sgw_mlp *mlp, int n_rows, const float *feat, const float *target,
                              float lr, float *loss_out);
/*
 * Column statistics of the operator A0 = H + alpha P_occ (the shifted operator of
 * Sec. 2.3, Eq. 6, without -eps_v - z): for every plane wave G (caller's order)
 *     diag[G] = (A0)_GG,   off2[G] = sum_{G' != G} |(A0)_G'G|^2.
 * Computed by applying A0 to unit vectors in batches.  psi: device [n_occ][n_pw];
 * diag, off2: device [n_pw].  Allocates a temporary device buffer.
 */
sgw_status sgw_operator_columns(sgw_ctx *ctx, const sgw_ham *ham, int n_occ, const sgw_c128 *psi, double alpha,
                                double *diag, double *off2);
/*
 * Training rows from residual histories (device [n_vec][n_pw], caller's order):
 * r are residuals of per-shift solves (snapshots, sternheimer_solve hist_r), b the
 * right-hand sides; eps, omega: host [n_vec] band energies and frequencies (Ha).
 * With D_G = diag[G] - eps - (omega + i eta) and c_G = off2[G], each sampled plane
 * wave u = stride*t (t < P = ceil(n_pw/stride)) of vector a gives rows 2(aP+t)
 * and 2(aP+t)+1:
 *     (u_m, w_m, u_g, w_g) = (D r, r, D b, b) / norms   and   (sqrt(c) r, 0, sqrt(c) b, 0) / norms
 * (norms: ||r|| for the first pair, ||b|| for the second, over the sampled plane
 * waves).  Summed over a vector's rows the loss is the diagonal approximate-
 * inverse objective  sum_G |r_G|^2 (|1 - D_G m_G|^2 + c_G |m_G|^2) / ||r||^2:
 * the residual left after one step x += m (.) r, with the off-diagonal part of A
 * counted by its column norm.  feat: device [2 n_vec P][5], target [2 n_vec P][8].
 */
sgw_status sgw_mlp_rows(sgw_ctx *ctx, const sgw_ham *ham, const double *diag, const double *off2, int n_vec,
                        const double *eps, const double *omega, double eta, const sgw_c128 *r, const sgw_c128 *b,
                        int stride, float *feat, float *target);

/*
 * Test hook of the per-shift solves' diagonal preconditioner and initial guess (not part of the
 * paper: any diagonal preconditioner or guess leaves the solution of Sec. 2.3, Eqs. 6-8, unchanged).
 * For n_vec systems with right-hand sides b (device [n_vec][n_pw], caller's order), band energies
 * eps and frequencies omega (host [n_vec], Ha) and eta, writes the values the per-shift solver uses,
 * computed by the same kernel:
 *   m   device out [n_vec][n_pw]: SGW_PC_NONE 1; SGW_PC_TETER K(T_G / E_ref) (Teter, Payne, Allan,
 *       Phys. Rev. B 40, 12255 (1989)) with E_ref = sum_G T_G |b_G|^2 / sum_G |b_G|^2, T_G = 0.5|k+G|^2;
 *       SGW_PC_LEARNED s (o0 + i o1) from the BF16 rounding of mlp's weights, FP32 arithmetic;
 *   x0  device out [n_vec][n_pw]: 0 for SGW_GUESS_ZERO, s (o2 + i o3) b_G for SGW_GUESS_LEARNED.
 * mlp may be NULL unless the learned model is asked for.  Allocates temporary device buffers and
 * returns after the GPU work has completed.
 */
sgw_status sgw_precond_values(sgw_ctx *ctx, const sgw_ham *ham, int precond, int guess, const sgw_mlp *mlp,
                              int n_vec, const double *eps, const double *omega, double eta, const sgw_c128 *b,
                              sgw_c128 *m, sgw_c128 *x0);

#ifdef __cplusplus
}
#endif
#endif /* SGW_H */
