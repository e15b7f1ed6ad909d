"""Plain CPU FP64 oracle for the linear Sternheimer solves of the SternheimerGW method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link this module; only the test suite, the
smoke check and the benchmark's CPU-baseline leg do.  It shares no code with
the HIP path.

What it computes (Hartree units; every function cites the passage it follows):

* the plane-wave Hamiltonian at one Bloch vector as a dense matrix
  (Sec. 2.1, Eq. 1 and the text after it: kinetic part diagonal in
  reciprocal space, local potential applied on the real-space grid, and the
  separable non-local part of the pseudopotential in reciprocal space);
* the driving term of the density response, projected off the occupied
  manifold (Sec. 2.3, Eq. 8), with the sign reading documented in ``rhs``;
* the Coulomb-response operator with the occupied projector (Sec. 2.3, Eq. 7)
  and the Sternheimer equation it enters (Sec. 2.3, Eq. 6);
* the exact solution of every shifted system, by two direct routes: an LU
  solve of the shifted operator, and the sum over all unoccupied eigenstates
  that the Sternheimer approach avoids (Sec. 1 and Sec. 2.2);
* the relative residual and the condition number used for the error budget;
* the Green's function columns (Sec. 2.2, Eqs. 2-3): (H_k - z) G_{.G'}(z) = -e_{G'},
  by the sum over all eigenstates that the linear equation replaces;
* the density response to the plane-wave perturbations (Sec. 2.3, Eq. 5), by the
  sum over empty states and from given linear variations, the dielectric matrix
  (Eq. 4), the correlation part of the screened interaction (Sec. 2.4, Eq. 9) and
  the (optionally truncated) Coulomb potential (Sec. 2.6, Eq. 12);
* the diagonal correlation self-energy on the imaginary or the real axis (Sec. 2.4,
  Eq. 10), the AAA and Pade rational continuations (Sec. 2.7), the spectral function
  and the linearised quasiparticle energy (Sec. 2.8, Eqs. 16-17).

The Krylov method itself is not reproduced: the iterative solver reaches
(up to rounding) the exact solution of each shifted system, and that solution
has the plain definition written out here.

Readings of the paper taken here:

* The energy in the shifted operator is the unperturbed eigenvalue of band v
  at k (Eq. 6 writes the band energy at k+q; the two coincide at q = 0).
* The right-hand side carries a minus sign, b = -(1 - P_occ) dV psi_v.
* The coefficient alpha of the occupied projector is a free parameter; the
  solution does not depend on it because b is orthogonal to the occupied space.
* Complex frequencies are z_j = omega_j + i*eta; the operator solved is
  H - eps_v - z_j + alpha * P_occ.
* The local potential is defined by its grid samples; its matrix element
  between plane waves m and m' is the discrete Fourier coefficient at the
  cyclic difference (m - m') mod N (grid-defined operator, aliasing included).
* The density response chi_{GG'} is the response to the unit perturbation
  exp(i (q+G') . r); the Coulomb factor that Eq. 4 leaves implicit is the
  potential v(q+G') of the perturbing charge, so eps_{GG'} = delta_{GG'} -
  chi_{GG'} v(q+G'), and Eq. 9 puts v(q+G) on the rows of W_bar (together they
  give W_bar = W - v with W = v (1 - chi v)^{-1}).  The +/- in Eq. 5 are the
  variations at the complex frequencies z and -z.
* Eq. 10 on the imaginary axis (alpha = -1): Sigma(i w) = -(1/2pi) sum_j w_j
  G(mu + i w'_j) W_bar(i (w'_j - w)) with the chemical potential mu in the
  gap; its diagonal element in state n is the sum over the W_bar plane waves of
  W_bar_{GG'} <t_G| G |t_G'> / Omega, t_G = exp(-i (q+G) . r) u_n.  The
  renormalisation of Eq. 17 is read as Z = 1 / (1 - Re dSigma/dw).
* The non-local part of the pseudopotential is taken in the fully separable
  form sum_p |beta_p> E_p <beta_p| with real E_p (any Hermitian coupling matrix
  between the projectors of an atom reduces to it by diagonalisation); the
  projector coefficients beta_p(G) are inputs.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# ---------------------------------------------------------------------------
# Hamiltonian (Sec. 2.1)
# ---------------------------------------------------------------------------

def kinetic(miller: np.ndarray, B: np.ndarray, kvec) -> np.ndarray:
    """Kinetic energy 0.5 |k + G|^2 of each plane wave (Sec. 2.1, Eq. 1)."""
    kg = np.asarray(miller, float) @ np.asarray(B, float) + np.asarray(kvec, float)
    return 0.5 * np.einsum("gd,gd->g", kg, kg)


def potential_coefficients(v_grid: np.ndarray) -> np.ndarray:
    """Discrete Fourier coefficients V~[m] = (1/N) sum_j V(r_j) exp(-i G_m . r_j).

    Sec. 2.1: the local potential is applied in real space; for plane waves
    sampled on the grid this is multiplication by V(r_j), whose plane-wave
    matrix element is V~ at the cyclic index difference.
    """
    return np.fft.fftn(np.asarray(v_grid, float)) / v_grid.size


def nonlocal_matrix(beta: np.ndarray, e_kb, rows=None) -> np.ndarray:
    """Separable non-local pseudopotential between plane waves (Sec. 2.1, the text after Eq. 1: the
    non-local part is represented in reciprocal space):
    V_NL[i, j] = sum_p E_p beta_p(G_i) conj(beta_p(G_j)), for the rows i in `rows` (all if None)."""
    b = np.asarray(beta, complex)
    br = b if rows is None else b[:, np.asarray(rows, np.int64)]
    return (br.T * np.asarray(e_kb, float)[None, :]) @ b.conj()


def hamiltonian(miller: np.ndarray, B: np.ndarray, kvec, v_grid: np.ndarray, nl=None) -> np.ndarray:
    """Dense plane-wave Hamiltonian H[i, j] = T_i delta_ij + V~[(m_i - m_j) mod N] (+ V_NL[i, j] when
    nl = (beta, e_kb) is given)."""
    vq = potential_coefficients(v_grid)
    n0, n1, n2 = v_grid.shape
    m = np.asarray(miller, np.int64)
    h = vq[(m[:, None, 0] - m[None, :, 0]) % n0,
           (m[:, None, 1] - m[None, :, 1]) % n1,
           (m[:, None, 2] - m[None, :, 2]) % n2]
    h[np.diag_indices_from(h)] += kinetic(miller, B, kvec)
    if nl is not None:
        h += nonlocal_matrix(nl[0], nl[1])
    return h


def hamiltonian_rows(miller: np.ndarray, B: np.ndarray, kvec, v_grid: np.ndarray, rows, nl=None) -> np.ndarray:
    """Rows `rows` of the dense plane-wave Hamiltonian, by the same definition as `hamiltonian`:
    H[i, j] = T_i delta_ij + V~[(m_i - m_j) mod N] (+ V_NL[i, j]) (for bases too large to hold H
    whole)."""
    vq = potential_coefficients(v_grid)
    n0, n1, n2 = v_grid.shape
    m = np.asarray(miller, np.int64)
    r = np.asarray(rows, np.int64)
    h = vq[(m[r, None, 0] - m[None, :, 0]) % n0,
           (m[r, None, 1] - m[None, :, 1]) % n1,
           (m[r, None, 2] - m[None, :, 2]) % n2]
    h[np.arange(len(r)), r] += kinetic(miller, B, kvec)[r]
    if nl is not None:
        h += nonlocal_matrix(nl[0], nl[1], rows=r)
    return h


def eigh(h: np.ndarray):
    """All eigenpairs of the Hermitian matrix (LAPACK divide and conquer)."""
    return sla.eigh(h, driver="evd")


# ---------------------------------------------------------------------------
# right-hand side (Sec. 2.3, Eq. 8)
# ---------------------------------------------------------------------------

def shifted_source(psi_v: np.ndarray, miller_k: np.ndarray, miller_kq: np.ndarray,
                   m_p) -> np.ndarray:
    """Plane-wave coefficients at k+q of exp(i (q + G_p) . r) times psi_v.

    Multiplying the Bloch state at k by the plane wave moves the coefficient of
    G to G + G_p on the k+q basis: s(G'') = psi_v(G'' - G_p), zero when
    G'' - G_p lies outside the basis sphere at k.
    """
    index_k = {tuple(int(c) for c in m): i for i, m in enumerate(np.asarray(miller_k))}
    m_p = np.asarray(m_p, np.int64)
    s = np.zeros(len(miller_kq), complex)
    for g, m in enumerate(np.asarray(miller_kq, np.int64)):
        i = index_k.get(tuple(int(c) for c in (m - m_p)))
        if i is not None:
            s[g] = psi_v[i]
    return s


def apply_occupied_projector(psi_occ: np.ndarray, x: np.ndarray) -> np.ndarray:
    """P_occ x = sum_n psi_n <psi_n | x>; ``psi_occ`` rows are the occupied states."""
    return psi_occ.T @ (psi_occ.conj() @ x)


def rhs(psi_v, miller_k, miller_kq, m_p, psi_occ_kq) -> np.ndarray:
    """b = -(1 - P_occ) dV_p psi_v on the k+q basis (Sec. 2.3, Eq. 8; sign per module docstring)."""
    s = shifted_source(psi_v, miller_k, miller_kq, m_p)
    return -(s - apply_occupied_projector(psi_occ_kq, s))


# ---------------------------------------------------------------------------
# shifted operator and its solution (Sec. 2.3, Eqs. 6-7)
# ---------------------------------------------------------------------------

def coulomb_operator(h_kq: np.ndarray, psi_occ_kq: np.ndarray, eps_v: float, alpha: float):
    """A0 = H_{k+q} - eps_v + alpha * P_occ (Eq. 7 with the band energy moved into the shift)."""
    a0 = h_kq - eps_v * np.eye(h_kq.shape[0]) + alpha * (psi_occ_kq.T @ psi_occ_kq.conj())
    return a0


def solve_lu(a0: np.ndarray, b: np.ndarray, z: complex) -> np.ndarray:
    """x = (A0 - z)^{-1} b by LU with partial pivoting (Eq. 6 solved directly)."""
    return sla.solve(a0 - z * np.eye(a0.shape[0]), b)


def solve_spectral(evals: np.ndarray, evecs: np.ndarray, n_occ: int, eps_v: float,
                   b: np.ndarray, zs) -> np.ndarray:
    """x(z) = sum over unoccupied c of u_c <u_c|b> / (eps_c - eps_v - z).

    This is the sum over empty states that the Sternheimer approach replaces
    (Sec. 1; Sec. 2.2).  ``evecs`` columns are eigenvectors of H_{k+q} in
    ascending order; the lowest ``n_occ`` are occupied.  Returns [len(zs)][n_pw].
    """
    uc = evecs[:, n_occ:]
    coef = uc.conj().T @ b
    zs = np.atleast_1d(np.asarray(zs, complex))
    den = evals[None, n_occ:] - eps_v - zs[:, None]
    return (coef[None, :] / den) @ uc.T


def relative_residual(a0: np.ndarray, x: np.ndarray, b: np.ndarray, z: complex) -> float:
    """||b - (A0 - z) x|| / ||b||, zero for a zero right-hand side with x = 0."""
    nb = np.linalg.norm(b)
    r = b - (a0 @ x - z * x)
    if nb == 0.0:
        return float(np.linalg.norm(r))
    return float(np.linalg.norm(r) / nb)


def condition_number(evals: np.ndarray, n_occ: int, eps_v: float, z: complex) -> float:
    """kappa of (H - eps_v - z) on the unoccupied space, from the exact spectrum."""
    lam = np.abs(evals[n_occ:] - eps_v - z)
    return float(lam.max() / lam.min())


# ---------------------------------------------------------------------------
# Green's function (Sec. 2.2, Eqs. 2-3)
# ---------------------------------------------------------------------------

def green_columns_spectral(evals: np.ndarray, evecs: np.ndarray, cols, zs) -> np.ndarray:
    """Columns G' = cols of G(z) = (z - H)^{-1}, the solution of (H - z) G_{.G'} = -e_{G'}, as the sum
    over all eigenstates n of u_n(G) conj(u_n(G')) / (z - eps_n).  Returns [len(cols)][len(zs)][n_pw]."""
    cols = np.asarray(cols, np.int64)
    zs = np.atleast_1d(np.asarray(zs, complex))
    w = evecs[cols, :].conj()                              # [col][n] conj(u_n(G'))
    coef = w[:, None, :] / (zs[None, :, None] - evals[None, None, :])   # [col][z][n]
    out = coef.reshape(-1, evals.size) @ evecs.T           # sum over n of u_n(G) coef[col][z][n]
    return out.reshape(len(cols), len(zs), evecs.shape[0])


def green_column_lu(h: np.ndarray, col: int, z: complex) -> np.ndarray:
    """One column of G(z) by LU: solve (H - z) x = -e_col directly (Eq. 2)."""
    e = np.zeros(h.shape[0], complex)
    e[col] = -1.0
    return sla.solve(h - z * np.eye(h.shape[0]), e)


def green_condition_number(evals: np.ndarray, z: complex) -> float:
    """kappa of H - z over the whole spectrum (no occupied projection in Eq. 3)."""
    lam = np.abs(evals - z)
    return float(lam.max() / lam.min())


# ---------------------------------------------------------------------------
# density response, dielectric matrix and screened interaction (Sec. 2.3, Eqs. 4-5; Sec. 2.4,
# Eq. 9; Sec. 2.6, Eq. 12)
# ---------------------------------------------------------------------------

def cell_volume(B: np.ndarray) -> float:
    """Unit-cell volume Omega = (2 pi)^3 / |det B| from the reciprocal lattice rows."""
    return float((2.0 * np.pi) ** 3 / abs(np.linalg.det(np.asarray(B, float))))


def coulomb(qg: np.ndarray, r_cut: float = 0.0) -> np.ndarray:
    """Coulomb potential of each wave vector q + G (Cartesian rows, Hartree units): 4 pi / |q+G|^2, or
    with the spherical truncation at r_cut > 0 (Sec. 2.6, Eq. 12) 4 pi / |q+G|^2 (1 - cos(|q+G| r_cut)),
    whose value at q + G = 0 is its limit 2 pi r_cut^2."""
    k = np.sqrt(np.einsum("gd,gd->g", np.asarray(qg, float), np.asarray(qg, float)))
    if r_cut <= 0.0:
        return 4.0 * np.pi / k ** 2
    out = np.empty_like(k)
    z = k == 0.0
    out[~z] = 4.0 * np.pi / k[~z] ** 2 * (1.0 - np.cos(k[~z] * r_cut))
    out[z] = 2.0 * np.pi * r_cut ** 2
    return out


def pair_matrix_elements(evecs_c: np.ndarray, psi_v: np.ndarray, miller_k, miller_kq, m_ps) -> np.ndarray:
    """M[p][c] = <u_c | exp(i (q + G_p) . r) u_v> for the k+q states in the columns of evecs_c."""
    return np.array([evecs_c.conj().T @ shifted_source(psi_v, miller_k, miller_kq, m_p) for m_p in m_ps])


def density_response_spectral(evals: np.ndarray, evecs: np.ndarray, n_occ: int, psi_k: np.ndarray,
                              eps_k: np.ndarray, miller_k, miller_kq, m_ps, zs, volume: float) -> np.ndarray:
    """Density response chi[z][G][G'] to the unit perturbations exp(i (q + G') . r), at the wave vectors
    q + G of the same set, by the sum over all empty states c at k+q that the Sternheimer route
    replaces (Sec. 2.3, Eq. 5 with each linear variation written as that sum):

        chi_{GG'}(z) = (2 / Omega) sum_v sum_c conj(M_cv(G)) M_cv(G') [1/(z - d_cv) - 1/(z + d_cv)],

    d_cv = eps_c - eps_v, M_cv(G) = <u_c | exp(i (q+G) . r) u_v>; the factor 2 is the spin degeneracy
    and the two terms are the variations at +z and -z.  psi_k rows: the occupied states at k (bands
    v = 0 .. len(psi_k) - 1 with energies eps_k).  Returns [len(zs)][n_G][n_G]."""
    zs = np.atleast_1d(np.asarray(zs, complex))
    uc = evecs[:, n_occ:]
    chi = np.zeros((len(zs), len(m_ps), len(m_ps)), complex)
    for v in range(psi_k.shape[0]):
        m = pair_matrix_elements(uc, psi_k[v], miller_k, miller_kq, m_ps)      # [G][c]
        d = evals[n_occ:] - eps_k[v]
        for j, z in enumerate(zs):
            w = 1.0 / (z - d) - 1.0 / (z + d)
            chi[j] += (m.conj() * w[None, :]) @ m.T
    return 2.0 / volume * chi


def density_response_from_solutions(psi_k: np.ndarray, miller_k, miller_kq, m_ps, psi_occ_kq: np.ndarray,
                                    dpsi_plus: np.ndarray, dpsi_minus: np.ndarray, volume: float) -> np.ndarray:
    """The same response from the linear variations themselves (Sec. 2.3, Eq. 5): the Fourier component
    q + G of 2 sum_v u_v^* (du_v(z) + du_v(-z)) per unit cell, which on the plane-wave bases is

        chi_{GG'}(z) = (2 / Omega) sum_v < (1 - P_occ) exp(i (q+G) . r) u_v | du_{v,G'}(z) + du_{v,G'}(-z) >

    (the variations have no occupied component).  dpsi_plus / dpsi_minus: [n_band][n_G'][n_z][n_pw_kq],
    the solutions at z and at -z.  Returns [n_z][n_G][n_G']."""
    nb, npert, nz, _ = dpsi_plus.shape
    chi = np.zeros((nz, npert, npert), complex)
    for v in range(nb):
        s = np.array([-rhs(psi_k[v], miller_k, miller_kq, m_p, psi_occ_kq) for m_p in m_ps])   # [G][pw]
        x = dpsi_plus[v] + dpsi_minus[v]                                                      # [G'][z][pw]
        chi += np.einsum("gp,hzp->zgh", s.conj(), x)
    return 2.0 / volume * chi


def dielectric(chi: np.ndarray, v: np.ndarray) -> np.ndarray:
    """eps_{GG'} = delta_{GG'} - chi_{GG'} v(q + G') (Sec. 2.3, Eq. 4, with the Coulomb factor of the
    perturbing potential restored on the columns)."""
    n = chi.shape[-1]
    return np.eye(n) - chi * np.asarray(v, float)[None, :]


def screened_correlation(eps: np.ndarray, v: np.ndarray, zero_rows=()) -> np.ndarray:
    """W_bar_{GG'} = v(q + G) (eps^{-1}_{GG'} - delta_{GG'}) (Sec. 2.4, Eq. 9); for the rows and columns
    listed in zero_rows (q + G = 0) the off-diagonal elements are set to zero."""
    n = eps.shape[-1]
    w = np.asarray(v, float)[:, None] * (np.linalg.inv(eps) - np.eye(n))
    for g in zero_rows:
        keep = w[..., g, g].copy()
        w[..., g, :] = 0.0
        w[..., :, g] = 0.0
        w[..., g, g] = keep
    return w


# ---------------------------------------------------------------------------
# correlation self-energy on the imaginary axis, analytic continuation and spectral function
# (Sec. 2.4, Eq. 10; Sec. 2.7; Sec. 2.8, Eqs. 15-17)
# ---------------------------------------------------------------------------

def green_pair_elements_spectral(evals: np.ndarray, evecs: np.ndarray, psi_n: np.ndarray, miller_k, miller_kmq,
                                 m_gs, zs) -> np.ndarray:
    """M[z][G][G'] = < t_G | G(z) | t_G' > with t_G = exp(-i (q+G) . r) u_n on the k-q basis and the
    Green's function G(z) = (z - H_{k-q})^{-1} = sum_m u_m u_m^H / (z - eps_m) over all eigenstates
    (Sec. 2.2): the pair of plane-wave factors that the real-space product G(r,r') W_bar(r,r') of Eq. 10
    puts around G in a diagonal matrix element.  ``evecs`` columns: eigenvectors of H_{k-q}."""
    zs = np.atleast_1d(np.asarray(zs, complex))
    t = np.array([shifted_source(psi_n, miller_k, miller_kmq, -np.asarray(m, np.int64)) for m in m_gs])   # [G][pw]
    c = evecs.conj().T @ t.T                                     # c[m][G] = <u_m | t_G>
    out = np.empty((len(zs), len(m_gs), len(m_gs)), complex)
    for j, z in enumerate(zs):
        out[j] = (c.conj().T * (1.0 / (z - evals))[None, :]) @ c
    return out


def green_pair_elements_lu(h: np.ndarray, psi_n: np.ndarray, miller_k, miller_kmq, m_gs, z) -> np.ndarray:
    """The same for one z by LU: x_G' = (z - H)^{-1} t_G' directly, then < t_G | x_G' >."""
    t = np.array([shifted_source(psi_n, miller_k, miller_kmq, -np.asarray(m, np.int64)) for m in m_gs])
    x = sla.solve(z * np.eye(h.shape[0]) - h, t.T)
    return t.conj() @ x


def sigma_c(m_elem: np.ndarray, wbar_at: np.ndarray, weights, volume: float, alpha: complex) -> np.ndarray:
    """Diagonal matrix element of the correlation self-energy (Sec. 2.4, Eq. 10): alpha / (2 pi Omega)
    sum_j w_j sum_{G,G'} W_bar_{GG'}(w'_j - w_k) M_{GG'}(z_j), with alpha = -1 along the imaginary axis and
    alpha = i along the real axis.  Shapes as in sigma_c_imag."""
    w = np.asarray(weights, float)
    return alpha * np.einsum("j,kjgh,jgh->k", w, wbar_at, m_elem) / (2.0 * np.pi * volume)


def sigma_c_imag(m_elem: np.ndarray, wbar_at: np.ndarray, weights, volume: float) -> np.ndarray:
    """Diagonal matrix element of the correlation self-energy on the imaginary axis (Sec. 2.4, Eq. 10 with
    alpha = -1): Sigma(i w_k) = -(1 / (2 pi Omega)) sum_j w_j sum_{G,G'} W_bar_{GG'}(i (w'_j - w_k)) M_{GG'}(mu + i w'_j),
    the real-space product of G and W_bar written on the plane waves of both.
    m_elem: [n_w'][G][G'] (green_pair_elements at the integration frequencies), wbar_at: [n_k][n_w'][G][G']
    (W_bar at each difference), weights: [n_w'].  Returns [n_k]."""
    w = np.asarray(weights, float)
    return -np.einsum("j,kjgh,jgh->k", w, wbar_at, m_elem) / (2.0 * np.pi * volume)


def aaa(zs, fs, tol: float = 1e-13, mmax: int = 100):
    """Rational approximation by the adaptive Antoulas-Anderson algorithm (Sec. 2.7; Nakatsukasa, Sete and
    Trefethen 2018): support points are added greedily where the current approximant is worst, the
    barycentric weights are the right singular vector of the smallest singular value of the Loewner
    matrix of the other points, until max |f - r| <= tol * max |f|.  Returns (z_sup, f_sup, w_sup) of
    r(z) = sum_s w_s f_s / (z - z_s) / sum_s w_s / (z - z_s)."""
    z = np.asarray(zs, complex)
    f = np.asarray(fs, complex)
    rest = np.ones(len(z), bool)
    r = np.full(len(z), f.mean())
    sup = []
    w = np.zeros(0, complex)
    for _ in range(min(mmax, len(z) - 1)):
        err = np.where(rest, np.abs(f - r), -1.0)
        j = int(np.argmax(err))
        sup.append(j)
        rest[j] = False
        zs_, fs_ = z[sup], f[sup]
        c = 1.0 / (z[rest][:, None] - zs_[None, :])
        a = (f[rest][:, None] - fs_[None, :]) * c
        w = np.linalg.svd(a)[2][-1].conj()
        r = f.copy()
        r[rest] = (c @ (w * fs_)) / (c @ w)
        if np.abs(f - r).max() <= tol * np.abs(f).max():
            break
    return z[sup], f[sup], w


def aaa_eval(z_sup, f_sup, w_sup, zs) -> np.ndarray:
    """r(z) of an aaa() approximant (the support values at the support points)."""
    zs = np.atleast_1d(np.asarray(zs, complex))
    out = np.empty(len(zs), complex)
    for i, z in enumerate(zs):
        d = z - z_sup
        hit = d == 0
        if hit.any():
            out[i] = f_sup[np.argmax(hit)]
        else:
            out[i] = np.sum(w_sup * f_sup / d) / np.sum(w_sup / d)
    return out


def pade_coefficients(zs, fs) -> np.ndarray:
    """Coefficients a_p of the N-point Pade interpolant in continued-fraction form (Sec. 2.7 compares it
    with AAA; Vidberg and Serene 1977): g_1(z_i) = f_i, g_p(z_i) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_i)) /
    ((z_i - z_{p-1}) g_{p-1}(z_i)) for i >= p, a_p = g_p(z_p)."""
    z = np.asarray(zs, complex)
    g = np.array(fs, complex)
    a = np.empty(len(z), complex)
    a[0] = g[0]
    for p in range(1, len(z)):
        g[p:] = (g[p - 1] - g[p:]) / ((z[p:] - z[p - 1]) * g[p:])
        a[p] = g[p]
    return a


def pade_eval(zs, a, x) -> np.ndarray:
    """C(x) = a_1 / (1 + a_2 (x - z_1) / (1 + a_3 (x - z_2) / (1 + ...))), by the three-term recursion
    A_{n+1} = A_n + (x - z_n) a_{n+1} A_{n-1} (the same for B), C = A_N / B_N."""
    z = np.asarray(zs, complex)
    x = np.atleast_1d(np.asarray(x, complex))
    a_prev, a_cur = np.zeros_like(x), np.full_like(x, a[0])
    b_prev, b_cur = np.ones_like(x), np.ones_like(x)
    for n in range(1, len(a)):
        t = (x - z[n - 1]) * a[n]
        a_prev, a_cur = a_cur, a_cur + t * a_prev
        b_prev, b_cur = b_cur, b_cur + t * b_prev
    return a_cur / b_cur


def spectral_function(omega, sigma, eps_n: float, delta: float) -> np.ndarray:
    """A(w) = -Im Sigma^c(w) / (pi |w - eps_n - Sigma^c(w) - delta|^2) (Sec. 2.8, Eq. 16; delta = Sigma^x -
    V^xc, the static part of Sigma^xc - V^xc, given)."""
    s = np.asarray(sigma, complex)
    return -s.imag / (np.pi * np.abs(np.asarray(omega, float) - eps_n - s - delta) ** 2)


def quasiparticle(eps_n: float, sigma_at_eps: complex, dsigma_at_eps: complex, delta: float):
    """Linearised quasiparticle energy (Sec. 2.8, Eq. 17): eps + Z (Re Sigma^c(eps) + delta) with the
    renormalisation Z = 1 / (1 - Re dSigma^c/dw at eps).  Returns (eps_qp, Z)."""
    z = 1.0 / (1.0 - np.real(dsigma_at_eps))
    return eps_n + z * (np.real(sigma_at_eps) + delta), z
