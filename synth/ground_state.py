"""Kohn-Sham reference states of the synthetic crystals (an input, not the method).

In the paper the occupied states, their energies and the Hamiltonian
parameters come from a preceding Kohn-Sham DFT run (paper Sec. 2.1); the
Sternheimer solves take them as given.  Here a dense diagonalisation of the
synthetic plane-wave Hamiltonian plays that role.  It exists only to produce
inputs for the solver; nothing in the solver or its checks calls it.

The Hamiltonian it diagonalises is the grid-defined operator: kinetic term
0.5|k+G|^2 on the diagonal plus the cyclic convolution with the discrete
Fourier coefficients of the sampled potential V(r_j), plus, when given, the
separable non-local term sum_i E_i beta_i beta_i^H.
"""
from __future__ import annotations

import hashlib
import os

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


# above this many plane waves the dense eigensolver runs on the GPU when one is present
GPU_EIGH_MIN_PW = 8000


def _lowest_states_gpu(miller, B, kvec, v_grid, n_states, nl=None):
    """The same Hamiltonian and eigenpairs with torch.linalg.eigh on the GPU (rocSOLVER): for the
    64-atom cell the CPU eigensolver takes over a quarter of an hour.  Input generation only."""
    import torch
    dev = torch.device("cuda")
    grid = v_grid.shape
    vq = torch.from_numpy(np.fft.fftn(v_grid) / v_grid.size).to(dev)
    m = torch.from_numpy(miller.astype(np.int64)).to(dev)
    n = m.shape[0]
    h = torch.empty((n, n), dtype=torch.complex128, device=dev)
    for r0 in range(0, n, 2048):  # rows in blocks to bound the index tensors
        mr = m[r0:r0 + 2048]
        d = [(mr[:, None, a] - m[None, :, a]) % grid[a] for a in range(3)]
        h[r0:r0 + 2048] = vq[d[0], d[1], d[2]]
    h.diagonal().add_(torch.from_numpy(kinetic_energies(miller, B, kvec)).to(dev))
    if nl is not None:
        beta = torch.from_numpy(np.asarray(nl[0], np.complex128)).to(dev)
        e = torch.from_numpy(np.asarray(nl[1], np.float64)).to(dev).to(torch.complex128)
        h += (beta.T * e[None, :]) @ beta.conj()
        del beta
    h = 0.5 * (h + h.conj().T)
    import sys
    import time
    t0 = time.time()
    print(f"[synth] dense eigh of {n} plane waves on the GPU", file=sys.stderr, flush=True)
    w, u = torch.linalg.eigh(h)
    torch.cuda.synchronize()
    print(f"[synth] eigh done in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    w = w[:n_states].cpu().numpy()
    u = u[:, :n_states].T.contiguous().cpu().numpy()
    del h
    torch.cuda.empty_cache()
    return w, u


def _cache_path(miller, B, kvec, v_grid, n_states, nl=None):
    """File of a cached eigensystem under $SYNTH_EIGH_CACHE (unset: no cache), keyed by the inputs."""
    root = os.environ.get("SYNTH_EIGH_CACHE")
    if not root:
        return None
    h = hashlib.sha256()
    for a in (np.asarray(miller, np.int64), np.asarray(B, float), np.asarray(kvec, float), np.asarray(v_grid, float)):
        h.update(np.ascontiguousarray(a).tobytes())
    if nl is not None:
        h.update(np.ascontiguousarray(np.asarray(nl[0], np.complex128)).tobytes())
        h.update(np.ascontiguousarray(np.asarray(nl[1], np.float64)).tobytes())
    h.update(str(n_states).encode())
    return os.path.join(root, f"eigh_{h.hexdigest()[:24]}.npz")


def lowest_states(miller: np.ndarray, B: np.ndarray, kvec, v_grid: np.ndarray, n_states: int, nl=None,
                  gpu_min_pw=None):
    """Lowest ``n_states`` eigenpairs of the plane-wave Hamiltonian.

    Returns (energies [n_states] in Ha ascending, states [n_states][n_pw] complex128,
    coefficient rows in the order of ``miller``).  Each state's phase is fixed so
    that its largest-magnitude coefficient (first one on ties) is real positive.
    With $SYNTH_EIGH_CACHE set, the result is stored there and later calls with the same
    inputs load it instead of diagonalising again (e.g. profiler runs that should not
    trace the eigensolver).  ``nl`` = (beta [n_proj][n_pw], e_kb [n_proj]) adds the separable
    non-local term.  ``gpu_min_pw``: basis size from which the eigensolver runs on the GPU when one
    is present (None: GPU_EIGH_MIN_PW).
    """
    n_states = min(n_states, miller.shape[0])
    path = _cache_path(miller, B, kvec, v_grid, n_states, nl)
    if path and os.path.exists(path):
        with np.load(path) as d:
            return d["w"], d["u"]
    if miller.shape[0] >= (GPU_EIGH_MIN_PW if gpu_min_pw is None else gpu_min_pw) and _gpu_present():
        w, u = _lowest_states_gpu(miller, B, kvec, v_grid, n_states, nl)
    else:
        h = _potential_matrix(miller, v_grid)
        h[np.diag_indices_from(h)] += kinetic_energies(miller, B, kvec)
        if nl is not None:
            beta, e = np.asarray(nl[0], np.complex128), np.asarray(nl[1], float)
            h += (beta.T * e[None, :]) @ beta.conj()
        h = 0.5 * (h + h.conj().T)
        w, u = sla.eigh(h, subset_by_index=[0, n_states - 1], driver="evr")
        u = u.T.copy()
    piv = np.argmax(np.abs(u), axis=1)
    ph = u[np.arange(u.shape[0]), piv]
    u *= (np.abs(ph) / ph)[:, None]
    u = np.ascontiguousarray(u)
    if path:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp.npz"
        np.savez(tmp, w=w, u=u)
        os.replace(tmp, path)  # readers see a whole file or none
    return w, u


def _gpu_present() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except ImportError:  # pragma: no cover
        return False
