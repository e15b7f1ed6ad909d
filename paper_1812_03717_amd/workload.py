"""Marshal one Sternheimer problem (plain arrays) onto the device through the binding.

``problem`` is any object with the attributes grid, B (reciprocal rows), kvec,
qvec, miller_k, miller_kq, v_grid, psi_k, psi_kq, n_band, eps_k, omega, eta,
dv_miller (numpy arrays, Hartree units).  Nothing here computes: arrays are
copied to device tensors and handed to the library.
"""
from __future__ import annotations

import numpy as np

from . import sgw


class DeviceProblem:
    def __init__(self, ctx, problem):
        import torch
        dev = ctx.device
        p = problem
        self.problem = p
        self.v = torch.from_numpy(np.ascontiguousarray(p.v_grid, np.float64)).to(dev)
        self.h_k = sgw.sgw_ham_create(ctx, p.grid, p.B, p.kvec, p.miller_k, self.v)
        same = np.array_equal(p.miller_k, p.miller_kq) and np.allclose(p.qvec, 0.0)
        self.h_kq = self.h_k if same else sgw.sgw_ham_create(ctx, p.grid, p.B, np.asarray(p.kvec) + np.asarray(p.qvec),
                                                              p.miller_kq, self.v)
        if getattr(p, "e_kb", None) is not None:  # separable non-local pseudopotential at k and k+q
            self.h_k.set_nonlocal(torch.from_numpy(np.ascontiguousarray(p.beta_k)).to(dev), p.e_kb)
            if self.h_kq is not self.h_k:
                self.h_kq.set_nonlocal(torch.from_numpy(np.ascontiguousarray(p.beta_kq)).to(dev), p.e_kb)
        self.psi_v = torch.from_numpy(np.ascontiguousarray(p.psi_k[: p.n_band])).to(dev)
        self.psi_occ_kq = torch.from_numpy(np.ascontiguousarray(p.psi_kq)).to(dev)
        self.eps_v = np.ascontiguousarray(p.eps_k[: p.n_band])
        self.ctx = ctx

    def solve(self, tol=None, opts=None, workspace=None, bands=None, perts=None, omega=None, dpsi=None, info=None):
        import torch
        p = self.problem
        psi_v, eps_v = self.psi_v, self.eps_v
        if bands is not None:
            psi_v = psi_v[list(bands)].contiguous()
            eps_v = eps_v[list(bands)]
        dvm = p.dv_miller if perts is None else p.dv_miller[list(perts)]
        om = p.omega if omega is None else np.asarray(omega, np.float64)
        return sgw.sternheimer_solve(self.ctx, self.h_kq, self.psi_occ_kq, self.h_k, psi_v, eps_v, dvm, om, p.eta,
                                     p.tol if tol is None else tol, opts=opts, workspace=workspace, dpsi=dpsi,
                                     info=info)
