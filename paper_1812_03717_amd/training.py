"""Training loop of the learned preconditioner / initial guess (host-side orchestration).

Rows come from the method's own per-shift solves: residual snapshots r_k after
k BiCGStab iterations (taken by the solver), the right-hand sides b (r_0 for a
zero start) and the column statistics of H + alpha P_occ.  The loss those rows
define is the residual left by one preconditioned step, in the diagonal
approximate-inverse form (see sgw_mlp_rows).  Row building, gradients and the
Adam update run in the library's kernels (sgw_operator_columns, sgw_mlp_rows,
sgw_mlp_train_step); this module only selects systems, allocates device
buffers and loops.
"""
from __future__ import annotations

import numpy as np

from . import sgw


def collect_rows(ctx, dev, bands, perts, omega, hist_iters=(3, 10, 30), stride=1, precond=sgw.PC_TETER,
                 alpha=1.0, workspace=None):
    """Rows (feat, target) from per-shift residual histories of one DeviceProblem over bands x perts x omega."""
    import torch
    p = dev.problem
    bands = list(bands)
    perts = list(perts)
    om = np.asarray(omega, np.float64)
    psi_v = dev.psi_v[bands].contiguous()
    eps_v = dev.eps_v[bands]
    dvm = np.asarray(p.dv_miller)[perts]
    nb, npt, nw, npw = len(bands), len(perts), len(om), dev.h_kq.n_pw
    n_vec = nb * npt * nw
    diag, off2 = sgw.sgw_operator_columns(ctx, dev.h_kq, dev.psi_occ_kq, alpha)
    b = sgw.sgw_build_rhs(ctx, dev.h_kq, dev.psi_occ_kq, dev.h_k, psi_v, dvm)
    bb = b[:, :, None, :].expand(nb, npt, nw, npw).contiguous().view(n_vec, npw)
    eps_rows = np.repeat(eps_v, npt * nw)
    om_rows = np.tile(om, nb * npt)
    # r_0 = b (zero start), then snapshots after k iterations
    snaps = [bb]
    for k in hist_iters:
        hr = torch.zeros((nb, npt, nw, npw), dtype=torch.complex128, device=ctx.device)
        hx = torch.zeros_like(hr)
        opts = sgw.sgw_opts_default(solver=sgw.SOLVER_PER_SHIFT, precond=precond, alpha_pv=alpha, hist_r=hr,
                                    hist_x=hx, hist_iter=int(k), ps_max_iter=int(k))
        st, _, _ = sgw.sternheimer_solve(ctx, dev.h_kq, dev.psi_occ_kq, dev.h_k, psi_v, eps_v, dvm, om, p.eta,
                                         1e-14, opts=opts, workspace=workspace)
        if st < 0:
            raise sgw.SgwError(st, sgw.load_library().sgw_last_error().decode())
        snaps.append(hr.view(n_vec, npw))
    feats, tgts = [], []
    for r in snaps:
        f, t = sgw.sgw_mlp_rows(ctx, dev.h_kq, diag, off2, eps_rows, om_rows, p.eta, r, bb, stride=stride)
        feats.append(f)
        tgts.append(t)
    return torch.cat(feats), torch.cat(tgts)


def train(ctx, mlp, feat, target, steps=400, lr=2e-3, batch=8192, seed=0, log_every=0):
    """Adam on random minibatches; returns the per-step losses (before each step)."""
    import torch
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    n = int(feat.shape[0])
    losses = []
    for s in range(steps):
        if n > batch:
            idx = torch.randint(0, n, (batch,), generator=g).to(ctx.device)
            f, t = feat[idx].contiguous(), target[idx].contiguous()
        else:
            f, t = feat, target
        losses.append(sgw.sgw_mlp_train_step(ctx, mlp, f, t, lr))
        if log_every and s % log_every == 0:
            print(f"train step {s} loss {losses[-1]:.5f}", flush=True)
    return losses
