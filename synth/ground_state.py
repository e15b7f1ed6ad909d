"""Kohn-Sham reference states of the synthetic crystals (an input, not the method).

In the paper the occupied states, their energies and the Hamiltonian
parameters come from a preceding Kohn-Sham DFT run (paper Sec. 2.1); the
Sternheimer solves take them as given.  Here a dense diagonalisation of the
synthetic plane-wave Hamiltonian plays that role.  It exists only to produce
inputs for the solver; nothing in the solver or its checks calls it.

The Hamiltonian it diagonalises is the grid-defined operator: kinetic term
0.5|k+G|^2 on the diagonal plus the cyclic convolution with the discrete
Fourier coefficients of the sampled potential V(r_j).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .crystal import kinetic_energies


def _potential_matrix(miller: np.ndarray, v_grid: np.ndarray) -> np.ndarray:
    grid = v_grid.shape
    vq = np.fft.fftn(v_grid) / v_grid.size          # coefficient of exp(+i G_m . r)
    m = miller.astype(np.int64)
    d0 = (m[:, None, 0] - m[None, :, 0]) % grid[0]
    d1 = (m[:, None, 1] - m[None, :, 1]) % grid[1]
    d2 = (m[:, None, 2] - m[None, :, 2]) % grid[2]
    return vq[d0, d1, d2]


def lowest_states(miller: np.ndarray, B: np.ndarray, kvec, v_grid: np.ndarray, n_states: int):
    """Lowest ``n_states`` eigenpairs of the plane-wave Hamiltonian.

    Returns (energies [n_states] in Ha ascending, states [n_states][n_pw] complex128,
    coefficient rows in the order of ``miller``).  Each state's phase is fixed so
    that its largest-magnitude coefficient (first one on ties) is real positive.
    """
    h = _potential_matrix(miller, v_grid)
    h[np.diag_indices_from(h)] += kinetic_energies(miller, B, kvec)
    h = 0.5 * (h + h.conj().T)
    n_states = min(n_states, h.shape[0])
    w, u = sla.eigh(h, subset_by_index=[0, n_states - 1], driver="evr")
    u = u.T.copy()
    piv = np.argmax(np.abs(u), axis=1)
    ph = u[np.arange(u.shape[0]), piv]
    u *= (np.abs(ph) / ph)[:, None]
    return w, np.ascontiguousarray(u)
