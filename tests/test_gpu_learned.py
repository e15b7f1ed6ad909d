"""GPU: what the trained model gains.  The model is trained on the GPU by the
library's kernels from residual histories of per-shift solves on small cells,
then used as the preconditioner of per-shift solves on held-out cells (other
seeds and sizes), against the Teter diagonal (the fallback) on the same
systems.  Every solve is decided by its true FP64 residual."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests.libutil import ensure_library
    ensure_library()
    from paper_1812_03717_amd import sgw
    c = sgw.sgw_ctx_create(0)
    yield c
    torch.cuda.synchronize()


def _train_problems():
    kw = dict(n_omega=16, n_pert=6, eta_ev=0.05, omega_hi_ev=40.0)
    return [synth.small((1, 1, 1), seed=9501, **kw), synth.small((1, 1, 1), seed=9502, **kw),
            synth.small((1, 1, 2), seed=9503, **kw)]


@pytest.fixture(scope="module")
def trained(ctx):
    from paper_1812_03717_amd import sgw, training
    from paper_1812_03717_amd.workload import DeviceProblem
    ws = sgw.Workspace(ctx)
    feats, tgts = [], []
    for p in _train_problems():
        d = DeviceProblem(ctx, p)
        f, t = training.collect_rows(ctx, d, range(p.n_band), range(p.n_pert), p.omega, workspace=ws)
        feats.append(f)
        tgts.append(t)
    feat, tgt = torch.cat(feats), torch.cat(tgts)
    mlp = sgw.sgw_mlp_create(ctx, seed=1)
    losses = training.train(ctx, mlp, feat, tgt, steps=1500, lr=2e-3, batch=32768)
    print("rows", feat.shape[0], "loss", losses[0], "->", np.mean(losses[-20:]), flush=True)
    yield mlp, losses, ws
    mlp.close()


def test_training_lowers_the_objective(trained):
    _, losses, _ = trained
    assert np.mean(losses[-20:]) < 0.2 * losses[0]


@pytest.mark.parametrize("held_out", ["fcc112_s9701", "fcc122_s9702"])
def test_learned_beats_teter_on_held_out(ctx, trained, held_out):
    from paper_1812_03717_amd import sgw
    from paper_1812_03717_amd.workload import DeviceProblem
    mlp, _, ws = trained
    cells, seed = {"fcc112_s9701": ((1, 1, 2), 9701), "fcc122_s9702": ((1, 2, 2), 9702)}[held_out]
    p = synth.small(cells, n_omega=16, n_pert=3, eta_ev=0.05, omega_hi_ev=40.0, seed=seed, tol=1e-8)
    d = DeviceProblem(ctx, p)
    bands = [p.n_occ // 2, p.n_occ - 1]
    res = {}
    for name, kw in {"none": dict(precond=sgw.PC_NONE), "teter": dict(precond=sgw.PC_TETER),
                     "learned": dict(precond=sgw.PC_LEARNED, mlp=mlp)}.items():
        opts = sgw.sgw_opts_default(solver=sgw.SOLVER_PER_SHIFT, **kw)
        st, _, info = d.solve(tol=1e-8, opts=opts, workspace=ws, bands=bands)
        inf = sgw.info_to_numpy(info)
        conv = (inf["flags"] & sgw.FLAG_CONVERGED) != 0
        res[name] = (int(inf["iters"].sum()), float(conv.mean()))
    st, _, info = d.solve(tol=1e-8, workspace=ws, bands=bands)
    ms = sgw.info_to_numpy(info)
    print(held_out, "per-shift BiCGStab iterations (sum, converged fraction):", res,
          "| multishift Krylov dimension sum", int(ms["iters"].sum()), flush=True)
    assert res["learned"][1] >= res["teter"][1]
    assert res["learned"][0] <= 0.95 * res["teter"][0]
