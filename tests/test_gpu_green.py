"""GPU parity of the Green's function columns (Sec. 2.2, Eqs. 2-3): (H_k - z) G_{.G'}(z) = -e_{G'}
with all frequencies sharing one Krylov space, through sgw_green_solve, against the oracle's sum
over all eigenstates, G(z) = (z - H)^{-1}.

Bar: 1e-8 relative error per column and frequency, with the solver tolerance set from the
condition number of H - z over the whole spectrum (tol_eff = 1e-8 / (2 kappa), not below 2e-13,
where FP64 residuals of these near-resonant shifts bottom out); both signs of eta (the two sides of
the time ordering), |eta| = 0.1 eV, and frequencies through the occupied and low empty levels.
"""
from synth import crystal as cx
import numpy as np
import pytest

import oracle.sternheimer_oracle as so
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


CASES = {
    # 2-atom cell, 307 plane waves, 16^3 grid (the whole-plane LDS kernels)
    "si2": (lambda: synth.si2(), [0, 1, 7, 150, 306], 12),
    # 16-atom cell, 4015 plane waves, 48^3 grid (the whole-line kernels)
    "si16": (lambda: synth.si16(), [0, 33, 2000, 4014], 8),
}


@pytest.mark.parametrize("solver", ["multishift", "block"])
@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("side", [1.0, -1.0], ids=["eta+", "eta-"])
def test_green_columns_match_oracle(ctx, name, side, solver):
    from paper_1812_03717_amd import sgw
    from paper_1812_03717_amd.workload import DeviceProblem
    make, cols, n_om = CASES[name]
    p = make()
    d = DeviceProblem(ctx, p)
    h = so.hamiltonian(p.miller_k, p.B, p.kvec, p.v_grid)
    w, u = so.eigh(h)
    # frequencies from below the lowest level to above the first empty ones, eta of either sign
    omega = np.linspace(w[0] - 0.2, w[p.n_occ] + 0.5, n_om)
    eta = side * 0.1 / cx.HA_EV
    zs = omega + 1j * eta
    kap = max(so.green_condition_number(w, z) for z in zs)
    tol = max(2e-13, min(1e-10, 1e-8 / (2.0 * kap)))
    kw = {"solver": sgw.SOLVER_BLOCK} if solver == "block" else {}
    st, g, info = sgw.sgw_green_solve(ctx, d.h_k, cols, omega, eta, tol,
                                      opts=sgw.sgw_opts_default(max_iter=3000, **kw))
    inf = sgw.info_to_numpy(info, (len(cols), n_om))
    print(f"{name} {solver} eta {eta:+.2e}: kappa {kap:.2e}, tol {tol:.1e}, status {st}, iters "
          f"{inf['iters'].min()}..{inf['iters'].max()}, max relres {inf['relres'].max():.2e}", flush=True)
    assert st == sgw.SGW_OK, sgw.load_library().sgw_last_error()
    assert np.all(inf["flags"] & sgw.FLAG_CONVERGED) and inf["relres"].max() <= tol
    ref = so.green_columns_spectral(w, u, cols, zs)
    got = g.cpu().numpy()
    worst = 0.0
    for c in range(len(cols)):
        for j in range(n_om):
            err = np.linalg.norm(got[c, j] - ref[c, j]) / np.linalg.norm(ref[c, j])
            worst = max(worst, err)
            assert err <= 1e-8, (cols[c], j, err)
    print(f"{name} eta {eta:+.2e}: max rel err vs oracle {worst:.2e}", flush=True)


def test_green_argument_errors(ctx):
    from paper_1812_03717_amd import sgw
    from paper_1812_03717_amd.workload import DeviceProblem
    p = synth.si2()
    d = DeviceProblem(ctx, p)
    with pytest.raises(sgw.SgwError):
        sgw.sgw_green_solve(ctx, d.h_k, [0, p.n_pw_k], [0.1], 0.01, 1e-8)   # column outside the basis
    with pytest.raises(sgw.SgwError):
        sgw.sgw_green_solve(ctx, d.h_k, [0], [0.1], 0.0, 1e-8)              # eta = 0
    st, g, info = sgw.sgw_green_solve(ctx, d.h_k, [], [0.1], 0.01, 1e-8)   # nothing to do
    assert st == sgw.SGW_OK and g.numel() == 0
