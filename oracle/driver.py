"""Batch driver of the oracle: exact solutions for a list of (band, perturbation) pairs.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Uses only the routines
of ``sternheimer_oracle``; the spectral route needs one full diagonalisation of
H_{k+q}, after which every (band, perturbation, frequency) solve is a pair of
matrix-vector products (Sec. 1: the sum over unoccupied states).
"""
from __future__ import annotations

import numpy as np

from . import sternheimer_oracle as so


def spectral_setup(miller_kq, B, kqvec, v_grid):
    """Dense H_{k+q} and its full eigendecomposition."""
    h = so.hamiltonian(miller_kq, B, kqvec, v_grid)
    w, u = so.eigh(h)
    return h, w, u


def solve_pairs(setup, n_occ, psi_v, eps_v, miller_k, miller_kq, dv_miller, psi_occ_kq,
                omega, eta, pairs):
    """Exact Delta psi for each (v, p) in ``pairs`` and every omega.

    Returns (x [len(pairs)][n_omega][n_pw_kq], b [len(pairs)][n_pw_kq]).
    """
    _, w, u = setup
    zs = np.asarray(omega, float) + 1j * float(eta)
    xs, bs = [], []
    for v, p in pairs:
        b = so.rhs(psi_v[v], miller_k, miller_kq, dv_miller[p], psi_occ_kq)
        xs.append(so.solve_spectral(w, u, n_occ, float(eps_v[v]), b, zs))
        bs.append(b)
    return np.array(xs), np.array(bs)
