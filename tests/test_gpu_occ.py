"""GPU parity of the occupied projector across occupied counts (Sec. 2.3, Eqs. 7-8), and a whole
solve with more occupied states than one pass of the overlap kernel takes.

The overlap kernel takes up to four 16-state occupied tiles per pass, so n_occ above 64 runs
several passes, and the apply kernel holds 16 * n_occ coefficients per vector tile in LDS: the
counts below cover one partial tile (17), whole passes (48, 64), one state past a pass (65), the
two-pass count of the 64-atom cell (128), a ragged multi-pass count (200) and the limit (256).
Bar: 1e-12 relative to the largest entry (complex128; only the summation order differs).
"""
import numpy as np
import pytest

import oracle.sternheimer_oracle as so
import synth
from synth import configs
from synth import crystal as cx

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


@pytest.fixture(scope="module")
def basis(ctx):
    """The 16-atom cell's basis at a seeded q (4014 plane waves, 48^3 grid)."""
    from paper_1812_03717_amd import sgw
    A, tau = cx.supercell(*cx.fcc_primitive(configs.A_LAT), (2, 2, 2))
    B = cx.reciprocal(A)
    q = cx.seeded_q(B, 31)
    grid = (48, 48, 48)
    v = cx.gaussian_potential(A, tau, grid, noise=0.05, seed=31)
    miller = cx.g_sphere(B, q, 11.46)
    vt = torch.from_numpy(np.ascontiguousarray(v, np.float64)).to(ctx.device)
    ham = sgw.sgw_ham_create(ctx, grid, B, q, miller, vt)
    return ham, miller.shape[0], vt


@pytest.mark.parametrize("n_occ", [17, 48, 64, 65, 128, 200, 256])
def test_apply_projector_occupied_counts(ctx, basis, n_occ):
    from paper_1812_03717_amd import sgw
    ham, n, _ = basis
    rng = np.random.default_rng(n_occ)
    psi = np.linalg.qr(rng.standard_normal((n, n_occ)) + 1j * rng.standard_normal((n, n_occ)))[0].T.copy()
    n_vec = 37  # a ragged vector count (the kernels tile vectors by 16)
    x = rng.standard_normal((n_vec, n)) + 1j * rng.standard_normal((n_vec, n))
    d_psi = torch.from_numpy(psi).to(ctx.device)
    xt = torch.from_numpy(x).to(ctx.device)
    y0 = sgw.sgw_apply_projector(ctx, ham, d_psi, xt, mode=0).cpu().numpy()
    px = np.array([so.apply_occupied_projector(psi, xi) for xi in x])
    ref0 = x - px
    e0 = np.abs(y0 - ref0).max() / np.abs(ref0).max()
    base = rng.standard_normal((n_vec, n)) + 1j * rng.standard_normal((n_vec, n))
    y1 = sgw.sgw_apply_projector(ctx, ham, d_psi, xt, alpha=1.7, mode=1,
                                 y=torch.from_numpy(base.copy()).to(ctx.device)).cpu().numpy()
    ref1 = base + 1.7 * px
    e1 = np.abs(y1 - ref1).max() / np.abs(ref1).max()
    print(f"n_occ {n_occ}: mode 0 rel err {e0:.2e}, mode 1 rel err {e1:.2e}", flush=True)
    assert e0 <= 1e-12 and e1 <= 1e-12
    # the (1 - P_occ) output is orthogonal to the occupied states
    assert np.abs(psi.conj() @ y0.T).max() <= 1e-12 * np.abs(y0).max() * np.sqrt(n)


@pytest.mark.parametrize("n_occ", [17, 64, 65, 128, 256])
def test_apply_projector_split_bf16(ctx, basis, n_occ):
    """The split-BF16 contraction (the FP32 phase of mixed-precision solves): three BF16 terms per
    value and the six largest term products leave under 2^-24 relative per product, and FP32
    accumulation over 256-plane-wave chunks (overlaps) and n_occ states (apply) adds rounding of the
    same order; bar 2e-6 of the largest projected entry (about 30 FP32 unit roundoffs), and above
    1e-12 (it is not the FP64 path)."""
    from paper_1812_03717_amd import sgw
    ham, n, _ = basis
    rng = np.random.default_rng(1000 + n_occ)
    psi = np.linalg.qr(rng.standard_normal((n, n_occ)) + 1j * rng.standard_normal((n, n_occ)))[0].T.copy()
    n_vec = 37
    x = rng.standard_normal((n_vec, n)) + 1j * rng.standard_normal((n_vec, n))
    d_psi = torch.from_numpy(psi).to(ctx.device)
    xt = torch.from_numpy(x).to(ctx.device)
    px = np.array([so.apply_occupied_projector(psi, xi) for xi in x])
    y0 = sgw.sgw_apply_projector(ctx, ham, d_psi, xt, mode=0 | sgw.PROJ_SPLIT_BF16).cpu().numpy()
    e0 = np.abs(y0 - (x - px)).max() / np.abs(px).max()
    base = rng.standard_normal((n_vec, n)) + 1j * rng.standard_normal((n_vec, n))
    y1 = sgw.sgw_apply_projector(ctx, ham, d_psi, xt, alpha=1.7, mode=1 | sgw.PROJ_SPLIT_BF16,
                                 y=torch.from_numpy(base.copy()).to(ctx.device)).cpu().numpy()
    e1 = np.abs(y1 - (base + 1.7 * px)).max() / np.abs(1.7 * px).max()
    print(f"n_occ {n_occ} split BF16: mode 0 rel err {e0:.2e}, mode 1 rel err {e1:.2e}", flush=True)
    assert 1e-12 < e0 <= 2e-6 and 1e-12 < e1 <= 2e-6


def test_projector_rejects_too_many_states(ctx, basis):
    from paper_1812_03717_amd import sgw
    ham, n, _ = basis
    many = torch.zeros((257, n), dtype=torch.complex128, device=ctx.device)
    x = torch.zeros((2, n), dtype=torch.complex128, device=ctx.device)
    with pytest.raises(sgw.SgwError) as e:
        sgw.sgw_apply_projector(ctx, ham, many, x, mode=0)
    assert e.value.code == sgw.SGW_ERR_UNSUPPORTED


def _problem_128():
    """fcc 2x2x2 cell (16 atoms) on a 48^3 grid at E_cut 6 Ha (~1500 plane waves) with about its lowest
    128 states occupied: four times the 16-atom cell's valence count, so the projector runs its
    multi-pass path inside the solver.  The levels there are dense, so the band count is the one within
    +-12 of 128 closest to it with a gap of at least 1e-3 Ha at k and k+q."""
    A, tau = cx.supercell(*cx.fcc_primitive(configs.A_LAT), (2, 2, 2))
    return configs.make_problem("fcc222_occ128", A, tau, (48, 48, 48), 6.0, 128, cx.frequencies_ev(0, 40, 6), 0.05,
                                3, 1e-12, 9800, occ_window=12)


def test_solve_occ128_matches_lu(ctx):
    """Whole solves with ~128 occupied states (two overlap passes per Krylov step): the top and a middle
    band, three perturbations, six frequencies in [0, 40] eV, against the oracle's LU route at the bar
    of the other solve tests (tol_eff = 1e-8 / (2 kappa), relative error 1e-8 per solve)."""
    from paper_1812_03717_amd import sgw
    from paper_1812_03717_amd.workload import DeviceProblem
    p = _problem_128()
    assert p.n_occ > 64
    d = DeviceProblem(ctx, p)
    h = so.hamiltonian(p.miller_kq, p.B, p.kvec + p.qvec, p.v_grid)
    w = np.linalg.eigvalsh(h)
    bands = [p.n_occ - 1, 64]
    kap = max(so.condition_number(w, p.n_occ, p.eps_k[v], om + 1j * p.eta) for v in bands for om in p.omega)
    tol = min(1e-10, 1e-8 / (2.0 * kap))
    st, dpsi, info = d.solve(tol=tol, bands=bands, opts=sgw.sgw_opts_default(max_iter=3000))
    inf = sgw.info_to_numpy(info, (len(bands), p.n_pert, p.n_omega))
    print(f"occ128: {p.n_pw_kq} PW, kappa {kap:.3e}, tol {tol:.2e}, status {st}, iters "
          f"{inf['iters'].min()}..{inf['iters'].max()}, max relres {inf['relres'].max():.2e}", flush=True)
    assert st == sgw.SGW_OK, sgw.load_library().sgw_last_error()
    assert np.all(inf["flags"] & sgw.FLAG_CONVERGED)
    assert inf["occ_leak"].max() <= 1e-10
    x = dpsi.cpu().numpy()
    worst = 0.0
    for bi, v in enumerate(bands):
        a0 = so.coulomb_operator(h, p.psi_kq, p.eps_k[v], 1.0)
        for q in range(p.n_pert):
            b = so.rhs(p.psi_k[v], p.miller_k, p.miller_kq, p.dv_miller[q], p.psi_kq)
            for j, om in enumerate(p.omega):
                ref = so.solve_lu(a0, b, om + 1j * p.eta)
                err = np.linalg.norm(x[bi, q, j] - ref) / np.linalg.norm(ref)
                worst = max(worst, err)
                assert err <= 1e-8, (v, q, j, err)
    print(f"occ128: max rel err vs LU {worst:.2e}", flush=True)
