"""Seeded synthetic crystals: lattices, plane-wave spheres, local potentials, non-local projectors.

This module only *generates inputs*. It holds none of the Sternheimer method's
arithmetic (no operator application, no projector, no solver). Both the HIP
library's tests/benchmarks and the CPU oracle draw their inputs from here.

Conventions (Hartree atomic units throughout, lengths in bohr):

* Direct lattice ``A``: rows are the primitive vectors a_i.
* Reciprocal lattice ``B = 2*pi*inv(A).T``: rows b_i, so a_i . b_j = 2*pi*delta_ij.
* A reciprocal vector is G_m = m @ B for integer Miller indices m.
* Plane-wave basis at Bloch vector k (the expansion of the Kohn-Sham reference
  system, paper Sec. 2.1, Eq. 1): all m with 0.5*|k + G_m|^2 <= E_cut.
* Grid point j = (j0, j1, j2) sits at r_j = sum_d (j_d / N_d) a_d, so
  G_m . r_j = 2*pi * sum_d m_d j_d / N_d.  Arrays on the grid are C-ordered
  ``[N0][N1][N2]`` (last index fastest).
"""
from __future__ import annotations

import numpy as np

HA_EV = 27.211386245988  # 1 Hartree in eV (CODATA 2018)


# ----------------------------------------------------------------------------
# lattices
# ----------------------------------------------------------------------------

def fcc_primitive(a: float):
    """Diamond structure in the fcc primitive cell: lattice rows and 2 atoms (Cartesian)."""
    A = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    tau = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
    return A, tau


def conventional_cubic(a: float):
    """Diamond structure in the conventional cubic cell: 8 atoms."""
    A = a * np.eye(3)
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    frac = np.concatenate([fcc, fcc + 0.25])
    return A, frac @ A


def supercell(A: np.ndarray, tau: np.ndarray, n: tuple[int, int, int]):
    """n0 x n1 x n2 supercell of (A, tau)."""
    n = tuple(int(x) for x in n)
    shifts = np.array([[i, j, k] for i in range(n[0]) for j in range(n[1]) for k in range(n[2])], float)
    As = np.diag(np.array(n, float)) @ A
    taus = (tau[None, :, :] + (shifts @ A)[:, None, :]).reshape(-1, 3)
    return As, taus


def reciprocal(A: np.ndarray) -> np.ndarray:
    return 2.0 * np.pi * np.linalg.inv(A).T


# ----------------------------------------------------------------------------
# plane-wave sphere
# ----------------------------------------------------------------------------

def g_sphere(B: np.ndarray, kvec: np.ndarray, ecut: float) -> np.ndarray:
    """Miller indices of the plane-wave sphere 0.5|k+G|^2 <= ecut, in canonical order.

    Canonical order: ascending kinetic energy, ties (one shell) broken by
    (m0, m1, m2) ascending.  Kinetic energies are compared on a 1e-9 Ha
    quantum so that members of one shell sort by Miller index and not by
    rounding noise.
    """
    kvec = np.asarray(kvec, float)
    # bound on |m_d|: |G.a_d| = 2*pi*|m_d| and |G| <= sqrt(2 ecut) + |k|
    A = 2.0 * np.pi * np.linalg.inv(B).T
    gmax = np.sqrt(2.0 * ecut) + np.linalg.norm(kvec)
    mbound = [int(np.ceil(gmax * np.linalg.norm(A[d]) / (2 * np.pi))) + 1 for d in range(3)]
    r = [np.arange(-mb, mb + 1) for mb in mbound]
    m = np.stack(np.meshgrid(*r, indexing="ij"), -1).reshape(-1, 3)
    ek = 0.5 * ((m @ B + kvec) ** 2).sum(1)
    sel = ek <= ecut
    m, ek = m[sel], ek[sel]
    q = np.round(ek * 1e9).astype(np.int64)
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], q))
    return np.ascontiguousarray(m[order].astype(np.int32))


def kinetic_energies(miller: np.ndarray, B: np.ndarray, kvec) -> np.ndarray:
    return 0.5 * ((miller @ B + np.asarray(kvec, float)) ** 2).sum(1)


# ----------------------------------------------------------------------------
# local potential on the FFT grid
# ----------------------------------------------------------------------------

def _grid_miller(n: int) -> np.ndarray:
    """Signed frequency index of each grid position along one axis (numpy fftfreq order)."""
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def gaussian_potential(A: np.ndarray, tau: np.ndarray, grid, amp: float = 0.5,
                       sigma: float = 1.5, noise: float = 0.05, seed: int = 0) -> np.ndarray:
    """Empirical local pseudopotential sampled on the grid, with seeded noise.

    V(G_m) = -amp * exp(-|G_m|^2 / (2 sigma^2)) * (1/N_at) sum_tau exp(-i G_m . tau)
    for every grid frequency |m_d| < N_d/2 (the Nyquist planes are zeroed so the
    potential is real), V0(r_j) = sum_m V(G_m) exp(i G_m . r_j), then each grid
    sample is scaled by (1 + noise * u_j) with u_j ~ U[-1, 1] i.i.d. from
    ``numpy.random.default_rng(seed)``.  The real-space noise breaks the point
    symmetry of the crystal so that the occupied/unoccupied boundary is not
    degenerate.
    """
    grid = tuple(int(n) for n in grid)
    B = reciprocal(A)
    ms = [_grid_miller(n) for n in grid]
    m = np.stack(np.meshgrid(*ms, indexing="ij"), -1)  # [N0,N1,N2,3]
    G = m @ B
    g2 = (G ** 2).sum(-1)
    form = -amp * np.exp(-g2 / (2.0 * sigma ** 2))
    phase = np.exp(-1j * np.einsum("xyzd,ad->xyza", G, tau))
    sfac = phase.mean(-1)
    vg = form * sfac
    nyq = np.zeros(grid, bool)
    for d, n in enumerate(grid):
        if n % 2 == 0:
            sl = [slice(None)] * 3
            sl[d] = n // 2
            nyq[tuple(sl)] = True
    vg[nyq] = 0.0
    ntot = grid[0] * grid[1] * grid[2]
    v0 = np.fft.ifftn(vg) * ntot
    assert np.abs(v0.imag).max() <= 1e-10 * max(1.0, np.abs(v0.real).max())
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=grid)
    return np.ascontiguousarray(v0.real * (1.0 + noise * u))


def kb_projectors(miller: np.ndarray, B: np.ndarray, kvec, A: np.ndarray, tau: np.ndarray, r_c: float = 1.2,
                  e_s: float = 0.6, e_p: float = -0.25, channels: str = "sp"):
    """Synthetic separable (Kleinman-Bylander) non-local pseudopotential: projectors and energies.

    For each atom a and channel (s: l = 0; p: l = 1, three real harmonics x, y, z), with
    K = k + G_m and the Gaussian radial form exp(-|K|^2 r_c^2 / 2):

        beta_{a,s}(G)   = N_s / sqrt(Omega) * exp(-|K|^2 r_c^2 / 2) * exp(-i K . tau_a)
        beta_{a,p_d}(G) = N_p / sqrt(Omega) * (K_d r_c) * exp(-|K|^2 r_c^2 / 2) * exp(-i K . tau_a)

    with N_s^2 = 8 pi^(3/2) r_c^3 and N_p^2 = 16 pi^(3/2) r_c^3, so that each projector has unit norm
    in the complete-basis limit.  The operator they define is V_NL = sum_i |beta_i> E_i <beta_i|
    (E_i = e_s or e_p), whose plane-wave matrix element between G and G' is
    sum_i E_i beta_i(G) conj(beta_i(G')): the phase exp(-i (G - G') . tau_a) is the one the local
    potential's structure factor carries.  Real pseudopotential files are not used; these stand in
    for them with the same structure (one radial form per channel, atom-centred phases).

    Returns (beta [n_proj][n_pw] complex128 in the order of ``miller``, e_kb [n_proj] float64),
    projectors ordered by atom, then channel (s, p_x, p_y, p_z).
    """
    A = np.asarray(A, float)
    omega = abs(np.linalg.det(A))
    K = np.asarray(miller, float) @ np.asarray(B, float) + np.asarray(kvec, float)
    radial = np.exp(-0.5 * (K * K).sum(1) * r_c * r_c) / np.sqrt(omega)
    n_s = np.sqrt(8.0 * np.pi ** 1.5 * r_c ** 3)
    n_p = np.sqrt(16.0 * np.pi ** 1.5 * r_c ** 3)
    beta, ekb = [], []
    for t in np.asarray(tau, float):
        ph = radial * np.exp(-1j * (K @ t))
        if "s" in channels:
            beta.append(n_s * ph)
            ekb.append(e_s)
        if "p" in channels:
            for d in range(3):
                beta.append(n_p * r_c * K[:, d] * ph)
                ekb.append(e_p)
    return np.ascontiguousarray(np.array(beta, np.complex128)), np.array(ekb, float)


def seeded_q(B: np.ndarray, seed: int) -> np.ndarray:
    """One seeded q: uniform fractional coordinates in [0,1)^3 of the reciprocal cell."""
    rng = np.random.default_rng(seed + 7919)
    return rng.uniform(0.0, 1.0, size=3) @ B


def perturbations(B: np.ndarray, qvec, n_pert: int) -> np.ndarray:
    """Miller indices of the n_pert shortest non-zero q+G, in canonical order.

    The perturbation is the plane wave dV_p(r) = exp(i (q + G_p) . r) with unit
    amplitude (the driving field of the dielectric response, paper Sec. 2.3).
    """
    qvec = np.asarray(qvec, float)
    # enlarge the search sphere until it holds enough vectors
    ecut = 1.0
    while True:
        m = g_sphere(B, qvec, ecut)
        ek = kinetic_energies(m, B, qvec)
        keep = ek > 1e-12
        if keep.sum() >= n_pert + 64:
            return np.ascontiguousarray(m[keep][:n_pert])
        ecut *= 2.0


def frequencies_ev(lo: float, hi: float, n: int) -> np.ndarray:
    return np.linspace(lo, hi, n)
