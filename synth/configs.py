"""The synthetic Sternheimer workloads, seeded and fully determined.

Each workload is a diamond-structure crystal with the Gaussian empirical local
pseudopotential of ``crystal.gaussian_potential`` (a = 10.26 bohr), the Bloch
vector k = Gamma, and a set of (band, frequency, perturbation) solves:

=========  ==========================  =====  ======  ====  =====  ===========================  =====  ======
name       cell                        atoms  E_cut   grid  n_occ  omega (eV) / eta (eV)        perts  tol
=========  ==========================  =====  ======  ====  =====  ===========================  =====  ======
si2        fcc primitive               2      8.157   16^3  4      linspace(0,20,8) / 0.1       4, q=0 1e-10
si16       fcc 2x2x2                   16     11.46   48^3  32     linspace(0,40,64) / 0.05     50     1e-8
si64       conventional cubic 2x2x2    64     11.46   72^3  128    linspace(0,40,100) / 0.05    20     1e-8
=========  ==========================  =====  ======  ====  =====  ===========================  =====  ======

``small(...)`` builds reduced cells of the same recipe for tests.  Seeds are
``1000*config + system``; when the occupied/unoccupied gap at k or k+q is
below 1e-3 Ha the seed is bumped by one (the bump is recorded in
``Problem.seed``).
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

from . import crystal as cx
from .ground_state import _gpu_present, lowest_states

A_LAT = 10.26
MIN_GAP_HA = 1e-3


@dataclasses.dataclass
class Problem:
    name: str
    A: np.ndarray
    B: np.ndarray
    tau: np.ndarray
    grid: tuple
    ecut: float
    kvec: np.ndarray
    qvec: np.ndarray
    miller_k: np.ndarray        # [n_pw_k][3] int32, canonical order
    miller_kq: np.ndarray       # [n_pw_kq][3]
    v_grid: np.ndarray          # [N0][N1][N2] float64, Ha
    n_occ: int
    n_band: int
    eps_k: np.ndarray           # [n_occ+1] lowest energies at k (Ha)
    psi_k: np.ndarray           # [n_occ][n_pw_k] occupied states at k
    eps_kq: np.ndarray          # [n_occ+1] at k+q
    psi_kq: np.ndarray          # [n_occ][n_pw_kq] occupied states at k+q
    omega: np.ndarray           # [n_omega] real frequencies (Ha)
    eta: float                  # imaginary part of every shift (Ha)
    dv_miller: np.ndarray       # [n_pert][3] int32, perturbation G_p
    tol: float
    seed: int
    # separable non-local pseudopotential (None: local potential only): projectors at k and k+q
    # ([n_proj][n_pw], rows in the order of miller_k / miller_kq) and their energies [n_proj] (Ha)
    beta_k: np.ndarray = None
    beta_kq: np.ndarray = None
    e_kb: np.ndarray = None

    @property
    def kqvec(self):
        return self.kvec + self.qvec

    @property
    def n_pw_k(self):
        return int(self.miller_k.shape[0])

    @property
    def n_pw_kq(self):
        return int(self.miller_kq.shape[0])

    @property
    def n_pert(self):
        return int(self.dv_miller.shape[0])

    @property
    def n_omega(self):
        return int(self.omega.shape[0])

    @property
    def psi_v(self):
        return self.psi_k[: self.n_band]

    @property
    def eps_v(self):
        return self.eps_k[: self.n_band]

    @property
    def n_proj(self):
        return 0 if self.e_kb is None else int(self.e_kb.shape[0])

    @property
    def n_solves(self):
        return self.n_band * self.n_pert * self.n_omega

    def gap(self):
        return min(self.eps_k[self.n_occ] - self.eps_k[self.n_occ - 1],
                   self.eps_kq[self.n_occ] - self.eps_kq[self.n_occ - 1])


def make_problem(name, A, tau, grid, ecut, n_occ, omega_ev, eta_ev, n_pert, tol, seed,
                 q_zero=False, n_band=None, noise=0.05, max_bumps=20, occ_window=0, min_gap=MIN_GAP_HA,
                 nonlocal_pp=False, gpu_min_pw=None):
    """occ_window > 0: when the states n_occ - 1 and n_occ are (near-)degenerate, take the band count
    within n_occ +- occ_window closest to n_occ that has a gap >= MIN_GAP_HA at k and k+q.
    nonlocal_pp: add the synthetic s and p projectors of ``crystal.kb_projectors`` on every atom to the
    Hamiltonian whose eigenstates are the reference states.  gpu_min_pw: see ``lowest_states``."""
    B = cx.reciprocal(A)
    kvec = np.zeros(3)
    target = n_occ
    for bump in range(max_bumps):
        s = seed + bump
        qvec = np.zeros(3) if q_zero else cx.seeded_q(B, s)
        v = cx.gaussian_potential(A, tau, grid, noise=noise, seed=s)
        mk = cx.g_sphere(B, kvec, ecut)
        mkq = mk if q_zero else cx.g_sphere(B, kvec + qvec, ecut)
        nl_k = cx.kb_projectors(mk, B, kvec, A, tau) if nonlocal_pp else None
        nl_kq = (nl_k if q_zero else cx.kb_projectors(mkq, B, kvec + qvec, A, tau)) if nonlocal_pp else None
        n_states = target + occ_window + 1
        ek, pk = lowest_states(mk, B, kvec, v, n_states, nl_k, gpu_min_pw=gpu_min_pw)
        if q_zero:
            ekq, pkq = ek, pk
        else:
            ekq, pkq = lowest_states(mkq, B, kvec + qvec, v, n_states, nl_kq, gpu_min_pw=gpu_min_pw)
        cands = sorted(range(max(1, target - occ_window), target + occ_window + 1), key=lambda n: (abs(n - target), n))
        ok = [n for n in cands if min(ek[n] - ek[n - 1], ekq[n] - ekq[n - 1]) >= min_gap]
        if ok:
            n_occ = ok[0]
            break
    else:  # pragma: no cover
        raise RuntimeError(f"{name}: no seed with a gap >= {min_gap} Ha")
    pert = cx.perturbations(B, qvec, n_pert)
    return Problem(
        name=name, A=A, B=B, tau=tau, grid=tuple(int(g) for g in grid), ecut=float(ecut),
        kvec=kvec, qvec=qvec, miller_k=mk, miller_kq=mkq, v_grid=v, n_occ=n_occ,
        n_band=n_occ if n_band is None else n_band,
        eps_k=ek, psi_k=np.ascontiguousarray(pk[:n_occ]),
        eps_kq=ekq, psi_kq=np.ascontiguousarray(pkq[:n_occ]),
        omega=np.asarray(omega_ev, float) / cx.HA_EV, eta=float(eta_ev) / cx.HA_EV,
        dv_miller=np.ascontiguousarray(pert.astype(np.int32)), tol=float(tol), seed=s,
        beta_k=None if nl_k is None else nl_k[0], beta_kq=None if nl_kq is None else nl_kq[0],
        e_kb=None if nl_k is None else nl_k[1])


@functools.lru_cache(maxsize=None)
def si2():
    """2-atom fcc cell, 307 PW, 16^3 grid, 4 bands x 8 omegas x 4 perts (q = 0)."""
    A, tau = cx.fcc_primitive(A_LAT)
    return make_problem("si2", A, tau, (16, 16, 16), 8.157, 4, cx.frequencies_ev(0, 20, 8), 0.1,
                        4, 1e-10, 1000, q_zero=True)


@functools.lru_cache(maxsize=None)
def si16():
    """16-atom fcc 2x2x2 supercell, 4015 PW, 48^3, 32 bands x 64 omegas x 50 perts."""
    A, tau = cx.supercell(*cx.fcc_primitive(A_LAT), (2, 2, 2))
    return make_problem("si16", A, tau, (48, 48, 48), 11.46, 32, cx.frequencies_ev(0, 40, 64), 0.05,
                        50, 1e-8, 2000)


@functools.lru_cache(maxsize=None)
def si64():
    """64-atom conventional 2x2x2 cell, 15967 PW, 72^3, ~128 bands x 100 omegas x 20 perts.  Its levels
    near state 128 are a quasi-continuum (spacing ~5e-4 Ha): the nearest band count within +-6 whose
    gap at k and k+q is at least 3e-4 Ha is occupied."""
    A, tau = cx.supercell(*cx.conventional_cubic(A_LAT), (2, 2, 2))
    return make_problem("si64", A, tau, (72, 72, 72), 11.46, 128, cx.frequencies_ev(0, 40, 100), 0.05,
                        20, 1e-8, 4000, occ_window=6, min_gap=3e-4)


@functools.lru_cache(maxsize=None)
def si64nl():
    """si64 with the synthetic non-local s and p projectors on every atom (256 projectors)."""
    A, tau = cx.supercell(*cx.conventional_cubic(A_LAT), (2, 2, 2))
    return make_problem("si64nl", A, tau, (72, 72, 72), 11.46, 128, cx.frequencies_ev(0, 40, 100), 0.05,
                        20, 1e-8, 4000, occ_window=6, min_gap=3e-4, nonlocal_pp=True)


@functools.lru_cache(maxsize=None)
def small(cells=(1, 1, 1), grid=None, ecut=11.46, n_occ=None, n_omega=8, n_pert=3,
          eta_ev=0.1, omega_hi_ev=20.0, q_zero=False, seed=9000, tol=1e-12, n_band=None, nonlocal_pp=False):
    """Reduced fcc n0 x n1 x n2 cells of the same recipe (grid 24 n_d unless given)."""
    A, tau = cx.supercell(*cx.fcc_primitive(A_LAT), cells)
    if grid is None:
        grid = tuple(24 * c for c in cells)
    if n_occ is None:
        n_occ = 2 * len(tau)
    return make_problem(f"small{cells}", A, tau, grid, ecut, n_occ,
                        cx.frequencies_ev(0, omega_hi_ev, n_omega), eta_ev, n_pert, tol, seed,
                        q_zero=q_zero, n_band=n_band, nonlocal_pp=nonlocal_pp)


@functools.lru_cache(maxsize=None)
def held_out(name, seed):
    """Cells for evaluating the learned preconditioner, with seeds of their own: "fcc222" (16 atoms,
    48^3), "fcc233" (36 atoms, 48 x 72 x 72) or "conv222" (the 64-atom conventional cell, 72^3);
    E_cut 11.46 Ha, all ~2*atoms bands occupied (the nearest count within +-6 with a gap >= 3e-4 Ha),
    64 omega in [0, 40] eV, eta 0.05 eV, 4 perturbations at a seeded q, tol 1e-8."""
    if name == "conv222":
        A, tau = cx.supercell(*cx.conventional_cubic(A_LAT), (2, 2, 2))
        grid = (72, 72, 72)
    else:
        cells = {"fcc222": (2, 2, 2), "fcc233": (2, 3, 3)}[name]
        A, tau = cx.supercell(*cx.fcc_primitive(A_LAT), cells)
        grid = tuple(24 * c for c in cells)
    return make_problem(f"{name}_s{seed}", A, tau, grid, 11.46, 2 * len(tau), cx.frequencies_ev(0, 40, 64), 0.05,
                        4, 1e-8, seed, occ_window=6, min_gap=3e-4, gpu_min_pw=5000)


CONFIGS = {"si2": si2, "si16": si16, "si64": si64, "si64nl": si64nl}


def _batch_cells(i, seed0, cells_max, n_omega_range, n_pert_range):
    rng = np.random.default_rng([seed0 + i, 1])
    cells = tuple(int(c) for c in rng.integers(1, cells_max + 1, 3))
    n_omega = int(rng.integers(n_omega_range[0], n_omega_range[1] + 1))
    n_pert = int(rng.integers(n_pert_range[0], n_pert_range[1] + 1))
    return cells, n_omega, n_pert


def _batch_system(args):
    i, seed0, ecut, cells_max, n_omega_range, n_pert_range, tol, threads, gpu_min_pw, min_gap = args
    from threadpoolctl import threadpool_limits
    cells, n_omega, n_pert = _batch_cells(i, seed0, cells_max, n_omega_range, n_pert_range)
    A, tau = cx.supercell(*cx.fcc_primitive(A_LAT), cells)
    with threadpool_limits(threads):
        return make_problem(f"batch{i}{cells}", A, tau, tuple(24 * c for c in cells), ecut, 2 * len(tau),
                            cx.frequencies_ev(0, 40, n_omega), 0.05, n_pert, tol, seed0 + i, occ_window=6,
                            gpu_min_pw=gpu_min_pw, min_gap=min_gap)


def batch(n_sys=200, seed0=3000, ecut=4.0, cells_max=3, n_omega_range=(16, 128), n_pert_range=(4, 16), tol=1e-8,
          workers=8, gpu_min_pw=None, min_gap=MIN_GAP_HA):
    """Independent systems of uneven size: fcc n0 x n1 x n2 cells (n_d uniform in 1..cells_max, 2-54
    atoms), grid 24 n_d per axis, all 2*atoms occupied bands, n_omega and n_pert uniform in their
    ranges, frequencies linspace(0, 40 eV), eta 0.05 eV, one seeded q each; system i has seed seed0 + i.
    Where states 2*atoms - 1 and 2*atoms are degenerate the nearest band count (within +-6) with a gap
    is occupied instead.
    Generated in `workers` processes (dense eigensolver per system on the CPU).  With gpu_min_pw set
    and a GPU present, the systems whose basis at k has at least that many plane waves are generated
    in this process with the eigensolver on the GPU (while the pool does the others).  min_gap: the
    smallest gap at the occupation edge (see make_problem)."""
    big = set()
    if gpu_min_pw is not None and _gpu_present():
        for i in range(n_sys):
            cells, _, _ = _batch_cells(i, seed0, cells_max, n_omega_range, n_pert_range)
            A, _ = cx.supercell(*cx.fcc_primitive(A_LAT), cells)
            if cx.g_sphere(cx.reciprocal(A), np.zeros(3), ecut).shape[0] >= gpu_min_pw:
                big.add(i)
    no_gpu = 1 << 62
    args = [(i, seed0, ecut, cells_max, n_omega_range, n_pert_range, tol, 2, gpu_min_pw if i in big else no_gpu,
             min_gap) for i in range(n_sys)]
    if workers <= 1:
        return [_batch_system(a) for a in args]
    import concurrent.futures as cf
    import multiprocessing as mp
    out = [None] * n_sys
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(_batch_system, a): a[0] for a in args if a[0] not in big}
        for i in sorted(big):
            out[i] = _batch_system(args[i])
        for f in cf.as_completed(futs):
            out[futs[f]] = f.result()
    return out
