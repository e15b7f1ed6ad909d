"""Pins of the CPU oracle against facts that do not come from the oracle itself.

The paper prints no worked example for the Sternheimer path (its numerical
results are band gaps of the full GW pipeline and figures that are not part
of the text), so the oracle is pinned by:

* closed forms: free electrons (V = const), where H is diagonal and every
  solve has an analytic value that fixes the sign of the right-hand side, the
  direction of the perturbation's index shift and the kinetic factor 1/2;
* brute force: the plane-wave Hamiltonian applied through explicit
  real-space sums with Cartesian G.r phases (no FFT, no Miller index
  arithmetic), and the shifted source evaluated in real space;
* an independent high-precision solve (mpmath, 40 digits) on a tiny basis;
* two independent direct routes (LU vs the sum over unoccupied states);
* invariants: Hermiticity, P_occ x = 0, residual, alpha-independence,
  linearity, reciprocity of the resolvent.

Each pin is a ``check_*`` function so that ``test_planted_mistakes`` can plant
a plausible mistake into the oracle and confirm that some pin catches it.
"""
import numpy as np
import pytest

import oracle.sternheimer_oracle as so
from synth import crystal as cx

A_LAT = 10.26


def _tiny(ecut=2.1, grid=(8, 8, 8), seed=5, kvec=(0.0, 0.0, 0.0)):
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    miller = cx.g_sphere(B, np.asarray(kvec), ecut)
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 0.5, size=grid)       # no symmetry at all
    return A, B, miller, v


def _realspace_apply_h(A, B, miller, kvec, v, x):
    """y = T x + F V F^-1 x with explicit exponentials of Cartesian G.r (no FFT)."""
    grid = v.shape
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    r = (j / np.array(grid, float)) @ A                       # Cartesian grid points
    G = miller.astype(float) @ B                              # Cartesian G (no k: periodic part)
    phase = np.exp(1j * (r @ G.T))                            # [Nr][Npw]
    psi_r = phase @ x
    f = v.reshape(-1) * psi_r
    y_loc = phase.conj().T @ f / v.size
    kg = G + np.asarray(kvec, float)
    return 0.5 * (kg * kg).sum(1) * x + y_loc


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------

def check_kinetic_closed_form():
    # simple cubic cell of side a: G_(1,0,0) = (2 pi / a, 0, 0)
    A = A_LAT * np.eye(3)
    B = cx.reciprocal(A)
    m = np.array([[1, 0, 0], [0, -2, 0], [1, 1, 1]])
    k = np.array([0.1, 0.0, -0.2])
    g = 2 * np.pi / A_LAT
    expect = 0.5 * np.array([(g + 0.1) ** 2 + 0.04, 0.01 + 4 * g * g + 0.04,
                             (g + 0.1) ** 2 + g * g + (g - 0.2) ** 2])
    assert np.allclose(so.kinetic(m, B, k), expect, rtol=1e-14, atol=0)


def check_hamiltonian_bruteforce(kvec=(0.03, -0.02, 0.05)):
    A, B, miller, v = _tiny(kvec=kvec)
    h = so.hamiltonian(miller, B, kvec, v)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(len(miller)) + 1j * rng.standard_normal(len(miller))
    y_ref = _realspace_apply_h(A, B, miller, kvec, v, x)
    err = np.linalg.norm(h @ x - y_ref) / np.linalg.norm(y_ref)
    assert err <= 1e-13, err
    assert np.abs(h - h.conj().T).max() <= 1e-14 * np.abs(h).max()
    # the row-restricted form (sampled outputs at bases too large for H) against the same sums
    rows = np.array([0, 3, len(miller) // 2, len(miller) - 1])
    hr = so.hamiltonian_rows(miller, B, kvec, v, rows)
    err_r = np.abs(hr @ x - y_ref[rows]).max() / np.abs(y_ref).max()
    assert err_r <= 1e-13, err_r


def check_shifted_source_realspace():
    """s(G'') is the k+q coefficient of exp(i(q+G_p).r) psi(r), evaluated on an alias-free grid."""
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    k = np.array([0.0, 0.0, 0.0])
    q = np.array([0.05, 0.11, -0.07])
    mk = cx.g_sphere(B, k, 2.1)
    mkq = cx.g_sphere(B, k + q, 2.1)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(len(mk)) + 1j * rng.standard_normal(len(mk))
    m_p = np.array([1, -1, 0])
    n = 16                                            # > 2*(max|m| + |m_p|) + 1: no aliasing
    grid = (n, n, n)
    j = np.stack(np.meshgrid(*[np.arange(g) for g in grid], indexing="ij"), -1).reshape(-1, 3)
    r = (j / n) @ A
    u_k = np.exp(1j * (r @ (mk.astype(float) @ B).T)) @ psi          # periodic part at k
    g_p = m_p.astype(float) @ B
    prod = np.exp(1j * (r @ g_p)) * u_k                              # periodic part at k+q
    coef = np.exp(-1j * (r @ (mkq.astype(float) @ B).T)).T @ prod / r.shape[0]
    inside = np.array([any((mm - m_p == mk).all(1)) for mm in mkq])
    s = so.shifted_source(psi, mk, mkq, m_p)
    assert np.allclose(s[inside], coef[inside], rtol=0, atol=1e-12 * np.abs(psi).max())
    assert np.all(s[~inside] == 0)


def check_free_electron_closed_form():
    """V = V0: H diagonal; Delta psi has one non-zero coefficient, -1 / (0.5|k+q+G_p|^2 - z)."""
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    k = np.zeros(3)
    q = 0.1 * B[0]
    v0 = -0.7
    grid = (10, 10, 10)
    v = np.full(grid, v0)
    mk = cx.g_sphere(B, k, 2.1)
    mkq = cx.g_sphere(B, k + q, 2.1)
    h_k = so.hamiltonian(mk, B, k, v)
    h_kq = so.hamiltonian(mkq, B, k + q, v)
    # the lowest state at k and at k+q is G = 0 (first in canonical order)
    assert (mk[0] == 0).all() and (mkq[0] == 0).all()
    psi_k = np.zeros((1, len(mk)), complex); psi_k[0, 0] = 1.0
    psi_kq = np.zeros((1, len(mkq)), complex); psi_kq[0, 0] = 1.0
    eps_v = h_k[0, 0].real
    assert abs(eps_v - v0) < 1e-15
    zs = np.array([0.0 + 0.01j, 0.3 + 0.05j, -0.2 + 0.002j])
    w, u = np.linalg.eigh(h_kq)
    for m_p in ([1, 0, 0], [0, -1, 1], [1, 1, 1]):
        m_p = np.array(m_p)
        gidx = int(np.nonzero((mkq == m_p).all(1))[0][0])
        b = so.rhs(psi_k[0], mk, mkq, m_p, psi_kq)
        e = np.zeros(len(mkq), complex); e[gidx] = -1.0
        assert np.array_equal(b, e)
        ekin = 0.5 * np.sum((k + q + m_p @ B) ** 2)
        for z in zs:
            expect = np.zeros(len(mkq), complex)
            expect[gidx] = -1.0 / (ekin - z)
            for x in (so.solve_lu(so.coulomb_operator(h_kq, psi_kq, eps_v, 1.0), b, z),
                      so.solve_spectral(w, u, 1, eps_v, b, [z])[0]):
                assert np.allclose(x, expect, rtol=0, atol=1e-14 / abs(ekin - z))
    # G_p = 0 drives the occupied state only: zero right-hand side
    assert np.abs(so.rhs(psi_k[0], mk, mkq, np.zeros(3, int), psi_kq)).max() == 0.0


def _small_problem(q=(0.04, -0.03, 0.09), n_occ=4, seed=11, ecut=2.1):
    A, B, mk, v = _tiny(seed=seed, ecut=ecut)
    k = np.zeros(3)
    q = np.asarray(q, float)
    mkq = cx.g_sphere(B, k + q, ecut)
    h_k = so.hamiltonian(mk, B, k, v)
    h_kq = so.hamiltonian(mkq, B, k + q, v)
    wk, uk = np.linalg.eigh(h_k)
    wq, uq = np.linalg.eigh(h_kq)
    return dict(B=B, mk=mk, mkq=mkq, v=v, h_kq=h_kq, wk=wk, uk=uk, wq=wq, uq=uq, n_occ=n_occ,
                psi_k=uk[:, :n_occ].T.copy(), psi_kq=uq[:, :n_occ].T.copy())


def check_mpmath_tiny():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    P = _small_problem()
    n_occ, psi_kq = P["n_occ"], P["psi_kq"]
    v, p = 1, np.array([1, 0, -1])
    b = so.rhs(P["psi_k"][v], P["mk"], P["mkq"], p, psi_kq)
    eps_v = P["wk"][v]
    z = 0.25 + 0.004j
    a0 = so.coulomb_operator(P["h_kq"], psi_kq, eps_v, 1.0)
    n = a0.shape[0]
    M = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            M[i, j] = mpmath.mpc(complex(a0[i, j])) - (z if i == j else 0)
    rhs_mp = mpmath.matrix([mpmath.mpc(complex(c)) for c in b])
    x_mp = mpmath.lu_solve(M, rhs_mp)
    x_hp = np.array([complex(x_mp[i]) for i in range(n)])
    kappa = so.condition_number(P["wq"], n_occ, eps_v, z)
    for x in (so.solve_lu(a0, b, z),
              so.solve_spectral(P["wq"], P["uq"], n_occ, eps_v, b, [z])[0]):
        err = np.linalg.norm(x - x_hp) / np.linalg.norm(x_hp)
        assert err <= 1e-14 * kappa + 1e-15, (err, kappa)


def check_routes_and_invariants():
    P = _small_problem()
    n_occ, psi_kq = P["n_occ"], P["psi_kq"]
    zs = np.array([0.0 + 0.003j, 0.4 + 0.003j, 1.1 + 0.02j, -0.3 + 0.01j])
    for v in range(n_occ):
        eps_v = P["wk"][v]
        for p in ([1, 0, 0], [0, 1, -1], [-1, -1, -1]):
            b = so.rhs(P["psi_k"][v], P["mk"], P["mkq"], np.array(p), psi_kq)
            xs_s = so.solve_spectral(P["wq"], P["uq"], n_occ, eps_v, b, zs)
            for z, x_s in zip(zs, xs_s):
                kappa = so.condition_number(P["wq"], n_occ, eps_v, z)
                a1 = so.coulomb_operator(P["h_kq"], psi_kq, eps_v, 1.0)
                x_l = so.solve_lu(a1, b, z)
                nx = np.linalg.norm(x_l)
                assert np.linalg.norm(x_l - x_s) <= 1e-13 * kappa * nx
                # P_occ x = 0
                assert np.linalg.norm(psi_kq.conj() @ x_l) <= 1e-13 * kappa * nx
                # residual of the direct solve
                assert so.relative_residual(a1, x_l, b, z) <= 1e-13
                # independence of the projector coefficient
                for alpha in (0.5, 5.0):
                    x_a = so.solve_lu(so.coulomb_operator(P["h_kq"], psi_kq, eps_v, alpha), b, z)
                    assert np.linalg.norm(x_a - x_l) <= 1e-13 * kappa * nx


def check_linearity_and_reciprocity():
    P = _small_problem()
    n_occ, psi_kq = P["n_occ"], P["psi_kq"]
    eps_v = P["wk"][2]
    a0 = so.coulomb_operator(P["h_kq"], psi_kq, eps_v, 1.0)
    b1 = so.rhs(P["psi_k"][2], P["mk"], P["mkq"], np.array([1, 0, 0]), psi_kq)
    b2 = so.rhs(P["psi_k"][3], P["mk"], P["mkq"], np.array([0, 1, 1]), psi_kq)
    c = 0.3 - 1.7j
    z = 0.37 + 0.01j
    x1, x2 = so.solve_lu(a0, b1, z), so.solve_lu(a0, b2, z)
    x12 = so.solve_lu(a0, b1 + c * b2, z)
    assert np.linalg.norm(x12 - x1 - c * x2) <= 1e-12 * np.linalg.norm(x12)
    # (A - conj z)^{-1} is the adjoint of (A - z)^{-1} for Hermitian A
    lhs = np.vdot(b2, so.solve_lu(a0, b1, np.conj(z)))
    rhs = np.vdot(so.solve_lu(a0, b2, z), b1)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def check_generator_ground_state():
    """The generator's occupied states are eigenstates of the oracle's Hamiltonian."""
    import synth
    p = synth.si2()
    h = so.hamiltonian(p.miller_k, p.B, p.kvec, p.v_grid)
    hn = np.abs(h).max()
    res = h @ p.psi_k.T - p.psi_k.T * p.eps_k[None, : p.n_occ]
    assert np.abs(res).max() <= 1e-11 * hn
    assert np.abs(p.psi_k.conj() @ p.psi_k.T - np.eye(p.n_occ)).max() <= 1e-12
    w = np.linalg.eigvalsh(h)
    assert np.allclose(w[: p.n_occ + 1], p.eps_k, rtol=0, atol=1e-11 * hn)
    assert p.gap() >= 1e-3


def check_relative_residual_closed_form():
    """Free electrons (V = V0): A0 - z is diagonal with entries 0.5|k+q+G|^2 + V0 - eps_v - z (+ alpha on
    the occupied G = 0).  The exact solution has residual 0; moving one coefficient by delta leaves the
    residual -(d_g - z) delta e_g, so relres = |d_g - z| |delta| / ||b|| exactly; b = 0 with x = 0 gives 0.
    The diagonal entries are written out from the kinetic closed form, not taken from the oracle."""
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    q = 0.1 * B[0]
    v0, alpha = -0.7, 1.3
    grid = (10, 10, 10)
    mk = cx.g_sphere(B, np.zeros(3), 2.1)
    mkq = cx.g_sphere(B, q, 2.1)
    h_kq = so.hamiltonian(mkq, B, q, np.full(grid, v0))
    psi_kq = np.zeros((1, len(mkq)), complex); psi_kq[0, 0] = 1.0
    psi_k = np.zeros(len(mk), complex); psi_k[0] = 1.0
    eps_v = v0
    a0 = so.coulomb_operator(h_kq, psi_kq, eps_v, alpha)
    m_p = np.array([0, -1, 1])
    scale = 3.5                                        # ||b|| = 3.5, so a missing division shows
    b = scale * so.rhs(psi_k, mk, mkq, m_p, psi_kq)
    g = int(np.nonzero((mkq == m_p).all(1))[0][0])
    kq = q + mkq.astype(float) @ B
    d = 0.5 * (kq * kq).sum(1) + v0 - eps_v
    d[0] += alpha                                      # G = 0 is the occupied state at k+q
    for z in (0.0 + 0.01j, 0.45 - 0.02j, -0.3 + 0.2j):
        x = np.zeros(len(mkq), complex)
        x[g] = -scale / (d[g] - z)                     # b = -scale e_g
        assert so.relative_residual(a0, x, b, z) <= 1e-15
        for h, delta in ((g, 0.02 - 0.01j), (0, 0.3j), (len(mkq) - 1, -0.05)):
            xp = x.copy()
            xp[h] += delta
            expect = abs(d[h] - z) * abs(delta) / scale
            got = so.relative_residual(a0, xp, b, z)
            assert abs(got - expect) <= 1e-13 * expect, (h, got, expect)
    zero = np.zeros(len(mkq), complex)
    assert so.relative_residual(a0, zero, zero, 0.2 + 0.01j) == 0.0


def check_condition_number_svd():
    """kappa of H - eps_v - z on the unoccupied space against the singular values of the operator
    restricted to that space, Q^H (H - eps_v - z) Q with Q an orthonormal basis of the complement of
    the occupied states (from a QR of the residual of random vectors, not from the eigenvectors),
    computed by LAPACK's SVD; z complex, eps_v an occupied level and omega near it, where counting
    the occupied levels would change kappa by orders of magnitude."""
    P = _small_problem()
    n_occ, psi_kq, h = P["n_occ"], P["psi_kq"], P["h_kq"]
    n = h.shape[0]
    rng = np.random.default_rng(7)
    r = rng.standard_normal((n, n - n_occ)) + 1j * rng.standard_normal((n, n - n_occ))
    r -= psi_kq.T @ (psi_kq.conj() @ r)                # off the occupied span
    qc = np.linalg.qr(r)[0]
    for v in (0, n_occ - 1):
        eps_v = P["wk"][v]
        for z in (0.0 + 0.002j, 0.3 + 0.05j, -0.2 + 0.01j, 1.5 + 0.1j):
            m = qc.conj().T @ (h - (eps_v + z) * np.eye(n)) @ qc
            s = np.linalg.svd(m, compute_uv=False)
            expect = s.max() / s.min()
            got = so.condition_number(P["wq"], n_occ, eps_v, z)
            assert abs(got - expect) <= 1e-9 * expect, (v, z, got, expect)


def check_green_free_electron():
    """V = V0: H diagonal, so G_{GG'}(z) = delta_{GG'} / (z - 0.5|k+G|^2 - V0) (Eqs. 2-3 with the kinetic
    closed form); both the spectral sum and the LU route must give it, and the Green's kappa counts
    every level (the lowest one near z makes it large)."""
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    k = np.array([0.02, -0.01, 0.03])
    v0 = -0.4
    m = cx.g_sphere(B, k, 2.1)
    h = so.hamiltonian(m, B, k, np.full((10, 10, 10), v0))
    w, u = np.linalg.eigh(h)
    kg = m.astype(float) @ B + k
    t = 0.5 * (kg * kg).sum(1) + v0
    cols = [0, 3, len(m) - 1]
    zs = np.array([v0 + 0.001 + 0.002j, 0.7 - 0.01j, 2.5 + 0.3j])
    gs = so.green_columns_spectral(w, u, cols, zs)
    for ci, c in enumerate(cols):
        for zi, z in enumerate(zs):
            expect = np.zeros(len(m), complex)
            expect[c] = 1.0 / (z - t[c])
            assert np.allclose(gs[ci, zi], expect, rtol=0, atol=1e-13 * abs(expect[c]))
            assert np.allclose(so.green_column_lu(h, c, z), expect, rtol=0, atol=1e-13 * abs(expect[c]))
    kap = so.green_condition_number(w, zs[0])
    assert abs(kap - np.abs(t - zs[0]).max() / np.abs(t - zs[0]).min()) <= 1e-12 * kap


def check_green_routes_and_symmetry():
    """Random local potential: spectral sum vs LU (two independent routes), the symmetry
    G(z)^H = G(conj z) of a Hermitian H, and the first terms of the large-|z| expansion
    G(z) = 1/z + H/z^2 + O(|z|^-3)."""
    A, B, m, v = _tiny()
    h = so.hamiltonian(m, B, np.zeros(3), v)
    w, u = np.linalg.eigh(h)
    n = len(m)
    cols = list(range(n))
    for z in (0.3 + 0.004j, -0.8 + 0.02j, 1.9 - 0.05j):
        g = so.green_columns_spectral(w, u, cols, [z])[:, 0, :].T       # [G][G']
        kap = so.green_condition_number(w, z)
        for c in (0, n // 2, n - 1):
            x = so.green_column_lu(h, c, z)
            assert np.linalg.norm(g[:, c] - x) <= 1e-13 * kap * np.linalg.norm(x)
        gc = so.green_columns_spectral(w, u, cols, [np.conj(z)])[:, 0, :].T
        assert np.abs(g.conj().T - gc).max() <= 1e-12 * kap * np.abs(g).max()
    z = 5e3 + 2e3j
    g = so.green_columns_spectral(w, u, cols, [z])[:, 0, :].T
    approx = np.eye(n) / z + h / z ** 2
    assert np.abs(g - approx).max() <= 5 * np.abs(h @ h).max() / abs(z) ** 3


def _nl_cell(ecut=2.5):
    """fcc primitive cell with a basis whose Miller indices stay within |m| <= 3: on a 16-point grid
    no difference m_i - m_j aliases, so the grid-defined local potential is exactly the Fourier series
    of the continuous one."""
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    k = np.array([0.031, -0.017, 0.052])
    miller = cx.g_sphere(B, k, ecut)
    assert np.abs(miller).max() <= 3 and len(miller) >= 20
    return A, tau, B, k, miller, (16, 16, 16)


def check_nonlocal_translation():
    """Moving every atom by the same vector d multiplies the local potential's coefficients by
    exp(-i G.d) and every projector by exp(-i (k+G).d), so the Hamiltonian must transform as
    H(tau + d) = U H(tau) U^H with U = diag(exp(-i (k+G).d)).  This fixes the relative phase
    convention of the non-local and local parts (a conjugated or transposed V_NL breaks it)."""
    A, tau, B, k, miller, grid = _nl_cell()
    d = np.array([0.37, -1.21, 0.58])
    hs = []
    for t in (tau, tau + d):
        v = cx.gaussian_potential(A, t, grid, noise=0.0)
        nl = cx.kb_projectors(miller, B, k, A, t, e_s=0.6, e_p=-0.45)
        hs.append(so.hamiltonian(miller, B, k, v, nl=nl))
    u = np.exp(-1j * ((miller @ B + k) @ d))
    h1 = (u[:, None] * hs[0]) * u.conj()[None, :]
    assert np.abs(hs[1] - h1).max() <= 1e-12 * np.abs(hs[0]).max()
    # the non-local part is not negligible here
    assert np.abs(so.nonlocal_matrix(*nl)).max() >= 0.05 * np.abs(hs[0]).max()
    # sampled rows by the same definition
    rows = np.array([0, 5, len(miller) - 1])
    hr = so.hamiltonian_rows(miller, B, k, v, rows, nl=nl)
    assert np.abs(hr - hs[1][rows]).max() <= 1e-14 * np.abs(hs[1]).max()


def check_nonlocal_secular():
    """Free electrons plus one projector: the eigenvalues of T + E beta beta^H away from the kinetic
    levels are the roots of the secular equation E sum_G |beta_G|^2 / (lambda - T_G) = 1, and there is
    one such root between consecutive distinct levels (rank-one update of a diagonal matrix)."""
    A, tau, B, k, miller, grid = _nl_cell()
    beta, _ = cx.kb_projectors(miller, B, k, A, tau[1:] + np.array([0.2, 0.1, -0.3]), channels="s")
    e = 0.7
    h = so.hamiltonian(miller, B, k, np.zeros(grid), nl=(beta, np.array([e])))
    lam = np.linalg.eigvalsh(h)
    t = 0.5 * ((miller @ B + k) ** 2).sum(1)      # kinetic closed form, written out here
    w2 = np.abs(beta[0]) ** 2
    far = [x for x in lam if np.abs(x - t).min() > 1e-3]
    assert len(far) >= 5
    for x in far:
        f = e * np.sum(w2 / (x - t))
        assert abs(f - 1.0) <= 1e-7, (x, f)
    # interlacing: the largest root lies above max T (E > 0) and every level moved up
    assert lam.max() > t.max() and np.all(np.sort(lam) >= np.sort(t) - 1e-12)


M_PS = np.array([[1, 0, 0], [0, -1, 1], [1, 1, 0], [0, 0, -1]])


def check_density_response_free_electron():
    """V = V0: the states are single plane waves, M_cv(G) = 1 exactly when G_c = G_v + G, so chi is
    diagonal with chi_GG(z) = (2/Omega) sum_v [G_v + G empty at k+q] (1/(z - d) - 1/(z + d)),
    d = 0.5|k+q+G_v+G|^2 - 0.5|k+G_v|^2 (V0 cancels), written out here from the kinetic closed form;
    then eps and W_bar are diagonal too: W_bar_GG = v_G (1 / (1 - chi_GG v_G) - 1)."""
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    k = np.array([0.013, -0.021, 0.008])
    q = np.array([0.071, 0.032, -0.045])
    mk, mkq = cx.g_sphere(B, k, 2.5), cx.g_sphere(B, k + q, 2.5)
    grid, v0, n_occ = (12, 12, 12), -0.4, 5
    tk = 0.5 * ((mk @ B + k) ** 2).sum(1)
    tq = 0.5 * ((mkq @ B + k + q) ** 2).sum(1)
    occ_k = np.argsort(tk)[:n_occ]
    occ_q = set(int(i) for i in np.argsort(tq)[:n_occ])
    psi_k = np.zeros((n_occ, len(mk)), complex)
    psi_k[np.arange(n_occ), occ_k] = 1.0
    w, u = so.eigh(so.hamiltonian(mkq, B, k + q, np.full(grid, v0)))
    omega = so.cell_volume(B)
    assert abs(omega - abs(np.linalg.det(A))) <= 1e-12 * omega
    zs = np.array([0.3 + 0.01j, -0.7 + 0.02j, 0.05j])
    chi = so.density_response_spectral(w, u, n_occ, psi_k, tk[occ_k] + v0, mk, mkq, M_PS, zs, omega)
    index_q = {tuple(m): i for i, m in enumerate(mkq)}
    ref = np.zeros((len(zs), len(M_PS)), complex)
    for gi, mp in enumerate(M_PS):
        for vi in occ_k:
            c = index_q.get(tuple(mk[vi] + mp))
            if c is None or c in occ_q:
                continue
            d = tq[c] - tk[vi]
            ref[:, gi] += 1.0 / (zs - d) - 1.0 / (zs + d)
    ref *= 2.0 / omega
    assert np.abs(ref).min() > 0
    for j in range(len(zs)):
        assert np.allclose(chi[j], np.diag(ref[j]), rtol=0, atol=1e-12 * np.abs(ref).max())
    qg = (M_PS + 0.0) @ B + q
    vq = 4.0 * np.pi / (qg ** 2).sum(1)
    wb = so.screened_correlation(so.dielectric(chi, so.coulomb(qg)), so.coulomb(qg))
    for j in range(len(zs)):
        expect = vq * (1.0 / (1.0 - ref[j] * vq) - 1.0)
        assert np.allclose(wb[j], np.diag(expect), rtol=1e-12, atol=1e-13 * np.abs(expect).max())


def check_density_response_routes():
    """chi by the sum over empty states against chi from LU solutions at z and -z (independent
    routes), its symmetries chi(-z) = chi(z) and chi(z)^H = chi(conj z), its sign at z = 0 (Hermitian,
    negative semidefinite), and W_bar = v (eps^-1 - 1) against W - v with W = (1 - v chi)^{-1} v, the
    other factor order."""
    P = _small_problem()
    n_occ, psi_kq = P["n_occ"], P["psi_kq"]
    omega = so.cell_volume(P["B"])
    zs = np.array([0.3 + 0.004j, -1.1 + 0.01j])
    chi = so.density_response_spectral(P["wq"], P["uq"], n_occ, P["psi_k"], P["wk"], P["mk"], P["mkq"], M_PS,
                                       zs, omega)
    dp = np.zeros((n_occ, len(M_PS), len(zs), len(P["mkq"])), complex)
    dm = np.zeros_like(dp)
    for v in range(n_occ):
        a0 = so.coulomb_operator(P["h_kq"], psi_kq, P["wk"][v], 1.0)
        for gi, mp in enumerate(M_PS):
            b = so.rhs(P["psi_k"][v], P["mk"], P["mkq"], mp, psi_kq)
            for j, z in enumerate(zs):
                dp[v, gi, j] = so.solve_lu(a0, b, z)
                dm[v, gi, j] = so.solve_lu(a0, b, -z)
    chi2 = so.density_response_from_solutions(P["psi_k"], P["mk"], P["mkq"], M_PS, psi_kq, dp, dm, omega)
    assert np.abs(chi2 - chi).max() <= 1e-10 * np.abs(chi).max()
    chi_m = so.density_response_spectral(P["wq"], P["uq"], n_occ, P["psi_k"], P["wk"], P["mk"], P["mkq"], M_PS,
                                         -zs, omega)
    assert np.abs(chi_m - chi).max() <= 1e-12 * np.abs(chi).max()
    chi_c = so.density_response_spectral(P["wq"], P["uq"], n_occ, P["psi_k"], P["wk"], P["mk"], P["mkq"], M_PS,
                                         np.conj(zs), omega)
    assert np.abs(np.conj(np.swapaxes(chi, 1, 2)) - chi_c).max() <= 1e-12 * np.abs(chi).max()
    # static response at q = 0 (every empty level above every occupied one): Hermitian, <= 0
    P0 = _small_problem(q=(0.0, 0.0, 0.0))
    assert P0["wq"][n_occ] - P0["wk"][n_occ - 1] > 1e-3
    chi0 = so.density_response_spectral(P0["wq"], P0["uq"], n_occ, P0["psi_k"], P0["wk"], P0["mk"], P0["mkq"],
                                        M_PS, [0.0], omega)[0]
    assert np.abs(chi0 - chi0.conj().T).max() <= 1e-13 * np.abs(chi0).max()
    ev = np.linalg.eigvalsh(chi0)
    assert ev.max() <= 1e-13 * np.abs(ev).max() and ev.min() < 0
    qg = (M_PS + 0.0) @ P["B"] + np.array([0.04, -0.03, 0.09])
    v = so.coulomb(qg)
    wb = so.screened_correlation(so.dielectric(chi, v), v)
    n = len(M_PS)
    for j in range(len(zs)):
        w_full = np.linalg.solve(np.eye(n) - v[:, None] * chi[j], np.diag(v))
        assert np.abs(wb[j] - (w_full - np.diag(v))).max() <= 1e-12 * np.abs(w_full).max()
    # the rule for q + G = 0 (Sec. 2.4): that row's and column's off-diagonal elements are zero
    wz = so.screened_correlation(so.dielectric(chi, v), v, zero_rows=[1])
    off = ~np.eye(n, dtype=bool)
    assert np.all(wz[:, 1, off[1]] == 0) and np.all(wz[:, off[:, 1], 1] == 0)
    keep = np.ones((n, n), bool)
    keep[1, :] = keep[:, 1] = False
    keep[1, 1] = True
    assert np.array_equal(wz[:, keep], wb[:, keep])


def check_coulomb_truncation():
    """Bare: 4 pi / |q|^2 at |q|^2 = 0.25; spherical truncation: its series 2 pi R^2 (1 - (qR)^2 / 12)
    at small q and 2 pi R^2 at q = 0, the bare value times (1 - cos qR) elsewhere with cos qR = -1 at
    qR = pi (twice the bare value)."""
    v = so.coulomb(np.array([[0.3, 0.0, 0.4]]))
    assert abs(v[0] - 16.0 * np.pi) <= 1e-13 * v[0]
    r = 7.5
    q = np.array([[1e-3, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, np.pi / r, 0.0]])
    vt = so.coulomb(q, r_cut=r)
    assert abs(vt[0] - 2 * np.pi * r * r * (1 - (1e-3 * r) ** 2 / 12)) <= 1e-9 * vt[0]
    assert vt[1] == 2 * np.pi * r * r
    assert abs(vt[2] - 2.0 * 4.0 * np.pi / (np.pi / r) ** 2) <= 1e-12 * vt[2]


def check_green_pair_free_electron():
    """V = V0 and a plane-wave state u_n = e_{G_n}: t_G = exp(-i(q+G).r) u_n is the plane wave G_n - G at
    k-q, so <t_G| (z - H)^{-1} |t_G'> = delta_GG' / (z - 0.5|k-q+G_n-G|^2 - V0); with a diagonal
    W_bar_GG(i nu) = c_G / (nu^2 + a^2) the self-energy of Eq. 10 is the explicit sum
    -(1/(2 pi Omega)) sum_j w_j sum_G c_G / ((w'_j - w)^2 + a^2) / (mu + i w'_j - e_G), written out here."""
    A, tau = cx.fcc_primitive(A_LAT)
    B = cx.reciprocal(A)
    k = np.array([0.011, -0.007, 0.019])
    q = np.array([0.052, -0.031, 0.044])
    mk, mkmq = cx.g_sphere(B, k, 2.5), cx.g_sphere(B, k - q, 2.5)
    grid, v0 = (12, 12, 12), -0.3
    w, u = so.eigh(so.hamiltonian(mkmq, B, k - q, np.full(grid, v0)))
    n_idx = 3
    psi = np.zeros(len(mk), complex)
    psi[n_idx] = 1.0
    zs = np.array([0.1 + 0.05j, 0.1 + 0.4j, 0.1 - 0.3j])
    mel = so.green_pair_elements_spectral(w, u, psi, mk, mkmq, M_PS, zs)
    index = {tuple(m): i for i, m in enumerate(mkmq)}
    e = []
    for mp in M_PS:
        g = index[tuple(mk[n_idx] - mp)]
        kg = (mkmq[g] + 0.0) @ B + (k - q)
        e.append(0.5 * kg @ kg + v0)
    e = np.array(e)
    for j, z in enumerate(zs):
        assert np.allclose(mel[j], np.diag(1.0 / (z - e)), rtol=0, atol=1e-13 * np.abs(1.0 / (z - e)).max())
    mu, a = 0.1, 0.7
    c = np.array([0.9, 0.5, 1.3, 0.2])
    wp = np.linspace(-3.0, 3.0, 41)
    wq = np.full(wp.size, wp[1] - wp[0])
    wout = np.array([0.0, 0.45, -1.2])
    m_int = so.green_pair_elements_spectral(w, u, psi, mk, mkmq, M_PS, mu + 1j * wp)
    wbar_at = np.zeros((len(wout), len(wp), 4, 4), complex)
    for kk, wo in enumerate(wout):
        for j, x in enumerate(wp):
            wbar_at[kk, j] = np.diag(c / ((x - wo) ** 2 + a * a))
    omega = so.cell_volume(B)
    sig = so.sigma_c_imag(m_int, wbar_at, wq, omega)
    for kk, wo in enumerate(wout):
        ref = -sum(wq[j] * np.sum(c / ((wp[j] - wo) ** 2 + a * a) / (mu + 1j * wp[j] - e))
                   for j in range(len(wp))) / (2 * np.pi * omega)
        assert abs(sig[kk] - ref) <= 1e-13 * abs(ref), (sig[kk], ref)


def check_green_pair_routes():
    """<t_G| G(z) |t_G'> by the sum over all eigenstates against LU solves, on the small random problem
    (k - q basis from q -> -q), and G(z)^H = G(conj z)."""
    P = _small_problem()
    h = P["h_kq"]
    zs = [0.2 + 0.05j, -0.4 + 0.3j]
    mel = so.green_pair_elements_spectral(P["wq"], P["uq"], P["psi_k"][1], P["mk"], P["mkq"], M_PS, zs)
    for j, z in enumerate(zs):
        ref = so.green_pair_elements_lu(h, P["psi_k"][1], P["mk"], P["mkq"], M_PS, z)
        assert np.abs(mel[j] - ref).max() <= 1e-11 * np.abs(ref).max()
    melc = so.green_pair_elements_spectral(P["wq"], P["uq"], P["psi_k"][1], P["mk"], P["mkq"], M_PS, np.conj(zs))
    assert np.abs(np.conj(np.swapaxes(mel, 1, 2)) - melc).max() <= 1e-12 * np.abs(mel).max()
    # Eq. 10's contraction is the quadratic form sum_m (c_m^H W c_m) / (z - eps_m) of the pair amplitudes
    # c_m(G) = <u_m | t_G> for a Hermitian (complex) W_bar
    rng = np.random.default_rng(8)
    x = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    wb = x + x.conj().T
    t = np.array([so.shifted_source(P["psi_k"][1], P["mk"], P["mkq"], -mp) for mp in M_PS])
    c = P["uq"].conj().T @ t.T                                # [m][G]
    vol = so.cell_volume(P["B"])
    for j, z in enumerate(zs):
        quad = np.einsum("mg,gh,mh->m", c.conj(), wb, c)
        ref = -np.sum(quad / (z - P["wq"])) / (2 * np.pi * vol)
        sig = so.sigma_c_imag(mel[j:j + 1], wb[None, None], [1.0], vol)[0]
        assert abs(sig - ref) <= 1e-12 * abs(ref)


def check_aaa_rational():
    """A rational function with four poles below the real axis, sampled on the imaginary axis, is
    reproduced by AAA on the real axis (its continuation) to 1e-8, with at most a few more support
    points than its degree; constants come back exactly."""
    p = np.array([0.3 - 0.05j, -0.8 - 0.1j, 1.5 - 0.2j, 2.2 - 0.08j])
    a = np.array([0.4, 1.1, -0.6, 0.3])
    f = lambda z: np.sum(a[None, :] / (np.asarray(z, complex)[:, None] - p[None, :]), axis=1)
    zi = 1j * np.linspace(0.02, 4.0, 60)
    zs, fs, ws = so.aaa(zi, f(zi), tol=1e-13)
    assert len(zs) <= 8
    zr = np.linspace(-2.0, 3.0, 101) + 0.01j
    err = np.abs(so.aaa_eval(zs, fs, ws, zr) - f(zr)).max() / np.abs(f(zr)).max()
    assert err <= 1e-8, err
    zc, fc, wc = so.aaa(zi, np.full(zi.size, 2.5 - 1j))
    assert np.allclose(so.aaa_eval(zc, fc, wc, zr), 2.5 - 1j, rtol=1e-14, atol=0)


def check_spectral_and_quasiparticle():
    """A constant Sigma = s_r + i s_i (s_i < 0) gives a Lorentzian of unit weight centred at
    eps + s_r + delta; a linear Sigma(w) = s0 + s1 (w - eps) gives the root of w - eps - Sigma(w) - delta
    = 0, eps + (s0 + delta) / (1 - s1), as the linearised quasiparticle energy, with Z = 1 / (1 - s1)."""
    eps, delta, sr, si = 0.2, -0.05, 0.13, -0.02
    w = np.linspace(-40.0, 40.0, 800001)
    a = so.spectral_function(w, np.full(w.size, sr + 1j * si), eps, delta)
    assert abs(np.trapezoid(a, w) - 1.0) <= 2e-3
    assert abs(w[np.argmax(a)] - (eps + sr + delta)) <= 1e-4
    s0, s1 = 0.07 - 0.01j, -0.35
    eq, z = so.quasiparticle(eps, s0, s1, delta)
    assert abs(eq - (eps + (s0.real + delta) / (1 - s1))) <= 1e-15 and abs(z - 1 / (1 - s1)) <= 1e-15
    assert abs(eq - eps - (s0.real + s1 * (eq - eps)) - delta) <= 1e-15


def check_sigma_plasmon_pole():
    """Eq. 10 for one state and one plane wave with a plasmon-pole W_bar(nu) = A [1/(nu - Om + i eta) -
    1/(nu + Om - i eta)] and the time-ordered G(w') = 1/(w' - eps + i eta sgn(eps - mu)): closing the
    contour gives Sigma(w) = A / (w - eps - Om + 2 i eta) for an empty state and A / (w - eps + Om - 2 i eta)
    for an occupied one; along the imaginary axis (alpha = -1, G(mu + i w'), W_bar(i nu) = A [1/(i nu - Om) -
    1/(i nu + Om)]) the same poles give Sigma(mu + i w) = A / (mu + i w - eps -+ Om).  The oracle's sums on
    a fine uniform grid (trapezoid, exponentially accurate for these analytic integrands; 1/w'^3 tails)
    must match to 1e-6."""
    amp, om, eta, mu = 0.7, 0.9, 0.1, 0.0
    h, lim = 0.005, 200.0
    wp = np.arange(-lim, lim + h / 2, h)
    wq = np.full(len(wp), h)
    for eps in (0.5, -0.4):
        s = 1.0 if eps > mu else -1.0
        g_real = (1.0 / (wp - eps + 1j * eta * s))[:, None, None]
        g_imag = (1.0 / (mu + 1j * wp - eps))[:, None, None]
        for w in (-0.3, 0.2, 1.1):
            nu = wp - w
            wb = amp * (1.0 / (nu - om + 1j * eta) - 1.0 / (nu + om - 1j * eta))
            sig = so.sigma_c(g_real, wb[None, :, None, None], wq, 1.0, 1j)[0]
            ref = amp / (w - eps - s * om + 2j * s * eta)
            assert abs(sig - ref) <= 1e-6 * abs(ref), (eps, w, sig, ref)
            wi = amp * (1.0 / (1j * nu - om) - 1.0 / (1j * nu + om))
            ref_i = amp / (mu + 1j * w - eps - s * om)
            for sig_i in (so.sigma_c(g_imag, wi[None, :, None, None], wq, 1.0, -1.0)[0],
                          so.sigma_c_imag(g_imag, wi[None, :, None, None], wq, 1.0)[0]):
                assert abs(sig_i - ref_i) <= 1e-6 * abs(ref_i), (eps, w, sig_i, ref_i)


def check_pade():
    """The N-point Pade interpolant: it reproduces the samples, recovers a type-(1, 1) function
    exactly from 7 points and a 3-pole function from 13, and its three-term evaluation equals the
    nested continued fraction a_1 / (1 + a_2 (x - z_1) / (1 + ...)) written out from the inside."""
    pole = 0.4 - 0.1j
    f = lambda x: (2.0 * x + 1.0) / (x - pole)
    z = 1j * np.linspace(0.1, 3.0, 7)
    a = so.pade_coefficients(z, f(z))
    x = np.linspace(-2.0, 2.0, 17) + 0.05j
    assert np.abs(so.pade_eval(z, a, z) - f(z)).max() <= 1e-13 * np.abs(f(z)).max()
    assert np.abs(so.pade_eval(z, a, x) - f(x)).max() <= 1e-11 * np.abs(f(x)).max()

    def rat(q):
        poles = np.array([0.3 - 0.05j, -0.8 - 0.1j, 1.5 - 0.2j])
        res = np.array([0.4, 1.1, -0.6])
        return np.sum(res[None, :] / (np.asarray(q, complex)[:, None] - poles[None, :]), axis=1)

    z = 1j * np.linspace(0.05, 3.0, 13)
    a = so.pade_coefficients(z, rat(z))
    assert np.abs(so.pade_eval(z, a, x) - rat(x)).max() <= 1e-9 * np.abs(rat(x)).max()
    z4 = np.array([0.5j, 1.0j, 1.7j, 2.2j])
    f4 = np.array([1 + 1j, 0.5 - 0.2j, 0.1 + 0.3j, -0.4j])
    a = so.pade_coefficients(z4, f4)
    for xv in (0.3 + 0.2j, -1.0 + 0.05j):
        v = 1.0 + 0j
        for n in range(len(a) - 1, 0, -1):
            v = 1.0 + a[n] * (xv - z4[n - 1]) / v
        assert abs(a[0] / v - so.pade_eval(z4, a, [xv])[0]) <= 1e-14


PINS = [check_kinetic_closed_form, check_hamiltonian_bruteforce, check_shifted_source_realspace,
        check_free_electron_closed_form, check_mpmath_tiny, check_routes_and_invariants,
        check_linearity_and_reciprocity, check_relative_residual_closed_form, check_condition_number_svd,
        check_green_free_electron, check_green_routes_and_symmetry, check_nonlocal_translation,
        check_nonlocal_secular, check_density_response_free_electron, check_density_response_routes,
        check_coulomb_truncation, check_green_pair_free_electron, check_green_pair_routes, check_aaa_rational,
        check_spectral_and_quasiparticle, check_sigma_plasmon_pole, check_pade]


@pytest.mark.parametrize("pin", PINS + [check_generator_ground_state], ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def _run_all_pins():
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    return failed


_orig_rhs = so.rhs
_orig_shift = so.shifted_source
_orig_kin = so.kinetic
_orig_coef = so.potential_coefficients
_orig_op = so.coulomb_operator
_orig_spec = so.solve_spectral
_orig_relres = so.relative_residual
_orig_green = so.green_columns_spectral
_orig_green_lu = so.green_column_lu
_orig_kappa = so.condition_number


def _mut_transposed_potential(miller, B, kvec, v_grid, nl=None):
    h = _orig_ham(miller, B, kvec, v_grid, nl=nl)
    return h.T.copy()


_orig_ham = so.hamiltonian
_orig_rows = so.hamiltonian_rows


def _mut_rows_index_swap(miller, B, kvec, v_grid, rows, nl=None):
    # V~ at m_j - m_i instead of m_i - m_j
    return _orig_ham(miller, B, kvec, v_grid, nl=nl).T[np.asarray(rows)].copy()


_orig_nl = so.nonlocal_matrix
_orig_chi = so.density_response_spectral
_orig_chi_sol = so.density_response_from_solutions
_orig_eps = so.dielectric
_orig_wbar = so.screened_correlation
_orig_coul = so.coulomb
_orig_gpe = so.green_pair_elements_spectral
_orig_sig = so.sigma_c_imag
_orig_sigma = so.sigma_c
_orig_pade = so.pade_coefficients
_orig_pade_eval = so.pade_eval
_orig_aaa = so.aaa
_orig_spec_fn = so.spectral_function
_orig_qp = so.quasiparticle


def _chi_one_term(w, u, n, pk, ek, mk, mkq, mps, zs, vol):
    # only the variation at +z
    zs = np.atleast_1d(np.asarray(zs, complex))
    out = np.zeros((len(zs), len(mps), len(mps)), complex)
    for v in range(pk.shape[0]):
        m = so.pair_matrix_elements(u[:, n:], pk[v], mk, mkq, mps)
        d = w[n:] - ek[v]
        for j, z in enumerate(zs):
            out[j] += (m.conj() * (1.0 / (z - d))[None, :]) @ m.T
    return 2.0 / vol * out


def _chi_conj_pairs(w, u, n, pk, ek, mk, mkq, mps, zs, vol):
    # conj on the perturbation's element instead of the density component's
    zs = np.atleast_1d(np.asarray(zs, complex))
    out = np.zeros((len(zs), len(mps), len(mps)), complex)
    for v in range(pk.shape[0]):
        m = so.pair_matrix_elements(u[:, n:], pk[v], mk, mkq, mps)
        d = w[n:] - ek[v]
        for j, z in enumerate(zs):
            out[j] += (m * (1.0 / (z - d) - 1.0 / (z + d))[None, :]) @ m.conj().T
    return 2.0 / vol * out

MUTATIONS = {
    "rhs_sign": ("rhs", lambda *a: -_orig_rhs(*a)),
    "rhs_no_projection": ("rhs", lambda psi_v, mk, mkq, mp, po: -_orig_shift(psi_v, mk, mkq, mp)),
    "shift_direction": ("shifted_source", lambda psi, mk, mkq, mp: _orig_shift(psi, mk, mkq, -np.asarray(mp))),
    "kinetic_no_half": ("kinetic", lambda m, B, k: 2.0 * _orig_kin(m, B, k)),
    "kinetic_drops_k": ("kinetic", lambda m, B, k: _orig_kin(m, B, 0.0 * np.asarray(k))),
    "potential_conjugated": ("potential_coefficients", lambda v: np.conj(_orig_coef(v))),
    "hamiltonian_transposed": ("hamiltonian", _mut_transposed_potential),
    "hamiltonian_rows_index_swap": ("hamiltonian_rows", _mut_rows_index_swap),
    "operator_shift_sign": ("coulomb_operator", lambda h, po, e, a: _orig_op(h, po, -e, a)),
    "spectral_off_by_one": ("solve_spectral", lambda w, u, n, e, b, z: _orig_spec(w, u, n + 1, e, b, z)),
    "spectral_conj_shift": ("solve_spectral", lambda w, u, n, e, b, z: _orig_spec(w, u, n, e, b, np.conj(z))),
    "relres_returns_zero": ("relative_residual", lambda a0, x, b, z: 0.0),
    "relres_no_division": ("relative_residual",
                           lambda a0, x, b, z: float(np.linalg.norm(b - (a0 @ x - z * x)))),
    "relres_shift_sign": ("relative_residual", lambda a0, x, b, z: _orig_relres(a0, x, b, -z)),
    "kappa_includes_occ": ("condition_number", lambda w, n, e, z: _orig_kappa(w, 0, e, z)),
    "kappa_drops_eta": ("condition_number", lambda w, n, e, z: _orig_kappa(w, n, e, complex(z).real + 1e-300j)),
    "kappa_inverted": ("condition_number", lambda w, n, e, z: 1.0 / _orig_kappa(w, n, e, z)),
    "green_sign": ("green_columns_spectral", lambda w, u, c, z: -_orig_green(w, u, c, z)),
    "green_conj_shift": ("green_columns_spectral", lambda w, u, c, z: _orig_green(w, u, c, np.conj(z))),
    "green_no_conj": ("green_columns_spectral",
                      lambda w, u, c, z: np.einsum("gn,cn,zn->czg", u, u[np.asarray(c), :],
                                                   1.0 / (np.atleast_1d(np.asarray(z, complex))[:, None] - w[None, :]))),
    "green_lu_rhs_sign": ("green_column_lu", lambda h, c, z: -_orig_green_lu(h, c, z)),
    "chi_sign": ("density_response_spectral", lambda *a: -_orig_chi(*a)),
    "chi_no_spin": ("density_response_spectral", lambda *a: 0.5 * _orig_chi(*a)),
    "chi_one_frequency": ("density_response_spectral", _chi_one_term),
    "chi_conj_pairs": ("density_response_spectral", _chi_conj_pairs),
    "chi_no_volume": ("density_response_spectral", lambda *a: _orig_chi(*a) * a[-1]),
    "chi_solutions_plus_only": ("density_response_from_solutions",
                                lambda pk, mk, mkq, mps, po, dp, dm, vol:
                                _orig_chi_sol(pk, mk, mkq, mps, po, dp, 0 * dm, vol)),
    "chi_solutions_sign": ("density_response_from_solutions", lambda *a: -_orig_chi_sol(*a)),
    "eps_rows": ("dielectric", lambda chi, v: np.eye(chi.shape[-1]) - chi * np.asarray(v)[:, None]),
    "eps_no_coulomb": ("dielectric", lambda chi, v: np.eye(chi.shape[-1]) - chi),
    "wbar_columns": ("screened_correlation",
                     lambda eps, v, zero_rows=(): np.asarray(v)[None, :] *
                     (np.linalg.inv(eps) - np.eye(eps.shape[-1]))),
    "coulomb_no_4pi": ("coulomb", lambda qg, r_cut=0.0: _orig_coul(qg, r_cut) / (4 * np.pi)),
    "coulomb_trunc_limit": ("coulomb", lambda qg, r_cut=0.0: np.where(
        np.einsum("gd,gd->g", np.asarray(qg, float), np.asarray(qg, float)) == 0, np.pi * r_cut ** 2,
        _orig_coul(qg, r_cut))),
    "green_pair_resolvent_sign": ("green_pair_elements_spectral", lambda *a: -_orig_gpe(*a)),
    "green_pair_transposed": ("green_pair_elements_spectral",
                              lambda *a: np.swapaxes(_orig_gpe(*a), 1, 2)),
    "sigma_sign": ("sigma_c_imag", lambda *a: -_orig_sig(*a)),
    "sigma_no_volume": ("sigma_c_imag", lambda m, w, q, vol: _orig_sig(m, w, q, 1.0)),
    "sigma_w_transposed": ("sigma_c_imag", lambda m, w, q, vol: _orig_sig(m, np.swapaxes(w, 2, 3), q, vol)),
    "sigma_alpha_conjugated": ("sigma_c", lambda m, w, q, vol, a: _orig_sigma(m, w, q, vol, np.conj(a))),
    "sigma_alpha_dropped": ("sigma_c", lambda m, w, q, vol, a: _orig_sigma(m, w, q, vol, 1.0)),
    "sigma_no_2pi": ("sigma_c", lambda m, w, q, vol, a: 2 * np.pi * _orig_sigma(m, w, q, vol, a)),
    "pade_coefficients_conjugated": ("pade_coefficients", lambda z, f: np.conj(_orig_pade(z, f))),
    "pade_eval_wrong_node": ("pade_eval", lambda z, a, x: _orig_pade_eval(np.roll(np.asarray(z), -1), a, x)),
    "aaa_unconjugated_weights": ("aaa", lambda zs, fs, tol=1e-13, mmax=100: (lambda r: (r[0], r[1], np.conj(r[2])))(
        _orig_aaa(zs, fs, tol, mmax))),
    "spectral_sign": ("spectral_function", lambda *a: -_orig_spec_fn(*a)),
    "qp_z_not_inverted": ("quasiparticle", lambda e, s, ds, d: (e + (1 - np.real(ds)) * (np.real(s) + d),
                                                                 1 - np.real(ds))),
    "nl_conjugated": ("nonlocal_matrix", lambda b, e, rows=None: np.conj(_orig_nl(b, e, rows))),
    "nl_energy_dropped": ("nonlocal_matrix", lambda b, e, rows=None: _orig_nl(b, np.ones_like(e), rows)),
    "nl_energy_sign": ("nonlocal_matrix", lambda b, e, rows=None: _orig_nl(b, -np.asarray(e), rows)),
    "nl_energy_squared": ("nonlocal_matrix",
                          lambda b, e, rows=None: _orig_nl(b, np.asarray(e) ** 2, rows)),
    "nl_rows_conjugated": ("nonlocal_matrix",
                           lambda b, e, rows=None: (_orig_nl(b, e, rows) if rows is None
                                                    else np.conj(_orig_nl(b, e, rows)))),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes(name, monkeypatch):
    """Plant one plausible mistake in the oracle (on the CPU): at least one pin must fail."""
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(so, attr, fn)
    failed = _run_all_pins()
    assert failed, f"no pin caught the planted mistake {name}"
