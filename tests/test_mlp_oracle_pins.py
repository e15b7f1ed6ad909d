"""Pins of the FP64 model reference (oracle.mlp_oracle) against closed forms,
special cases and finite differences, plus planted mistakes each pin must catch."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as mo


def _random_case(seed=3, n=7):
    rng = np.random.default_rng(seed)
    w = 0.3 * rng.standard_normal(mo.N_PARAMS)
    t = rng.uniform(0.0, 12.0, n)
    feat = mo.features(t, rng.uniform(-1, 0.5, n), rng.uniform(0, 1.5, n), 0.0018)
    target = rng.standard_normal((n, 8))
    return w, feat, target


def check_fd_gradient():
    """Backpropagated gradient == central finite differences of the loss (FP64, h = 1e-6)."""
    w, feat, target = _random_case()
    g = mo.grad(w, feat, target)
    h = 1e-6
    fd = np.empty_like(w)
    for i in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[i] = (mo.loss(wp, feat, target) - mo.loss(wm, feat, target)) / (2 * h)
    err = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    assert err < 1e-7, err


def check_output_bias_closed_form():
    """All weights zero, b3 = (2, 0, 0, 2): o = b3, so m = 2s and g = 2is.  At T = 1 (s = 1/2),
    u_m = 3, w_m = 1 gives |3 - 1|^2 = 4; u_g = 1, w_g = i gives 0: the loss is 4."""
    p = {name: np.zeros(shape) for name, shape in mo.SIZES}
    p["b3"] = np.array([2.0, 0.0, 0.0, 2.0])
    w = mo.pack(p)
    feat = mo.features(np.array([1.0]), 0.3, 0.2, 0.001)
    target = np.array([[3.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 1.0]])
    assert abs(mo.loss(w, feat, target) - 4.0) < 1e-14
    m, g = mo.model_outputs(w, feat)
    assert abs(m[0] - 1.0) < 1e-15 and abs(g[0] - 1j) < 1e-15


def check_layer_orientation():
    """One path through distinct units: feature 2 -> hidden-1 unit 3 -> hidden-2 unit 1 -> output 2,
    so o2 = 1.5 tanh(tanh(0.7 omega) - 0.25) and every other output is 0."""
    p = {name: np.zeros(shape) for name, shape in mo.SIZES}
    p["W1"][3, 2] = 0.7
    p["W2"][1, 3] = 1.0
    p["b2"][1] = -0.25
    p["W3"][2, 1] = 1.5
    w = mo.pack(p)
    omega = 0.9
    feat = mo.features(np.array([5.0]), 0.1, omega, 0.001)
    o, _ = mo.forward(w, feat)
    expect = 1.5 * math.tanh(math.tanh(0.7 * omega) - 0.25)
    assert abs(o[0, 2] - expect) < 1e-15
    assert np.all(o[0, [0, 1, 3]] == 0.0)
    _, g = mo.model_outputs(w, feat)
    assert abs(g[0] - expect / 6.0) < 1e-15  # s = 1/(T+1) = 1/6


def check_features():
    f = mo.features(np.array([10.0]), 20.0, 0.5, 0.01)[0]
    assert np.allclose(f, [1.0, 2.0, 0.5, 1.0, -1.05], rtol=0, atol=1e-15)


def check_teter():
    """K(0) = 1, K(1) = 65/81, K(x) ~ 1/(2x) for large x, decreasing on [0, 20]."""
    assert mo.teter(0.0) == 1.0
    assert abs(mo.teter(1.0) - 65.0 / 81.0) < 1e-15
    x = 1e4
    assert abs(2 * x * mo.teter(x) - 1.0) < 1e-3
    k = mo.teter(np.linspace(0, 20, 401))
    assert np.all(np.diff(k) < 0)


def check_teter_diagonal():
    """A right-hand side on one plane wave has E_ref = T_G there, so K = K(1) = 65/81 at that G; for
    equal weights E_ref is the mean kinetic energy; the weights are |b|^2, not |b|."""
    kin = np.array([0.5, 2.0, 4.0, 9.5])
    b = np.array([0, 0, 3 - 4j, 0])
    assert abs(mo.teter_diagonal(kin, b)[2] - 65.0 / 81.0) < 1e-15
    ones = np.ones(4, complex)
    assert np.allclose(mo.teter_diagonal(kin, ones), mo.teter(kin / kin.mean()), rtol=1e-15, atol=0)
    b2 = np.array([1.0, 2.0, 0.0, 0.0])       # E_ref = (0.5 + 4 * 2) / 5 = 1.7
    assert np.allclose(mo.teter_diagonal(kin, b2), mo.teter(kin / 1.7), rtol=1e-15, atol=0)


def check_bf16_round():
    """BF16 keeps 8 significant bits: exact values stay, halfway cases go to the even neighbour."""
    x = np.array([1.0, -2.5, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7 + 2 ** -9, 3.0e-5], np.float32)
    r = mo.bf16_round(x)
    assert r[0] == 1.0 and r[1] == -2.5
    assert r[2] == 1.0                        # tie: 1 (even) rather than 1 + 2^-7
    assert r[3] == 1 + 2 ** -6                # tie: 1 + 2^-6 (even) rather than 1 + 2^-7
    assert r[4] == 1 + 2 ** -7                # below the midpoint to 1 + 2^-6
    assert abs(r[5] - 3.0e-5) <= 2 ** -9 * 3.0e-5


def check_operator_columns():
    """2x2 Hermitian [[1, 2+i], [2-i, 3]]: diagonal (1, 3), off-diagonal column norms (5, 5);
    and the column sums add up to the Frobenius norm of a random matrix."""
    d, off2 = mo.operator_columns(np.array([[1.0, 2 + 1j], [2 - 1j, 3.0]]))
    assert np.allclose(d, [1, 3], atol=0) and np.allclose(off2, [5, 5], atol=1e-14)
    rng = np.random.default_rng(4)
    a = rng.standard_normal((9, 9)) + 1j * rng.standard_normal((9, 9))
    a = a + a.conj().T
    d, off2 = mo.operator_columns(a)
    assert abs(np.sum(d ** 2 + off2) - np.linalg.norm(a) ** 2) < 1e-12 * np.linalg.norm(a) ** 2


def check_rows_give_spai_objective():
    """The model loss over one vector's rows equals the diagonal approximate-inverse objective
    of the model's m on that residual (plus the same objective of g on b), divided by the row count;
    and conj(d)/(|d|^2 + c) minimises the objective (perturbations only raise it)."""
    rng = np.random.default_rng(6)
    npw = 40
    kin = rng.uniform(0, 12, npw)
    diag = kin - 0.5 + rng.uniform(-0.1, 0.1, npw)
    off2 = rng.uniform(0.5, 2.0, npw)
    eps, om, eta = np.array([-0.3]), np.array([0.8]), 0.002
    r = rng.standard_normal((1, npw)) + 1j * rng.standard_normal((1, npw))
    b = rng.standard_normal((1, npw)) + 1j * rng.standard_normal((1, npw))
    feat, target = mo.rows(kin, diag, off2, eps, om, eta, r, b)
    w = 0.3 * rng.standard_normal(mo.N_PARAMS)
    m, g = mo.model_outputs(w, feat[0::2])
    d = diag - eps[0] - (om[0] + 1j * eta)
    expect = (mo.spai_objective(m, d, off2, r[0]) + mo.spai_objective(g, d, off2, b[0])) / feat.shape[0]
    assert abs(mo.loss(w, feat, target) - expect) < 1e-12 * expect
    # stationary point: both m* + dm and m* - dm raise the objective (a wide shift, eta = 0.5)
    d = diag - eps[0] - (om[0] + 0.5j)
    mstar = mo.spai_optimum(d, off2)
    f0 = mo.spai_objective(mstar, d, off2, r[0])
    for k in range(5):
        dm = 1e-3 * (rng.standard_normal(npw) + 1j * rng.standard_normal(npw))
        assert mo.spai_objective(mstar + dm, d, off2, r[0]) > f0
        assert mo.spai_objective(mstar - dm, d, off2, r[0]) > f0


PINS = [check_fd_gradient, check_output_bias_closed_form, check_layer_orientation, check_features, check_teter,
        check_operator_columns, check_rows_give_spai_objective, check_teter_diagonal, check_bf16_round]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


_orig = {name: getattr(mo, name) for name in ("grad", "loss", "forward", "features", "teter", "scale", "rows",
                                              "spai_optimum", "operator_columns", "teter_diagonal", "bf16_round")}


def _rows_conj_d(kin, diag, off2, eps, omega, eta, r, b, stride=1):
    # D with the wrong sign of the shift's imaginary part
    return _orig["rows"](kin, diag, off2, eps, omega, -eta, r, b, stride)


def _grad_imag_sign(w, feat, target):
    # the d/d o_b terms with the wrong sign: equivalent to conjugating the model's imaginary part
    t = np.asarray(target, np.float64).copy()
    t[:, [1, 3, 5, 7]] *= -1.0
    return _orig["grad"](w, feat, t)


def _forward_transposed(w, feat):
    p = mo.unpack(w)
    x = np.asarray(feat, np.float64)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"] + p["b2"])
    o = h2 @ p["W3"].T + p["b3"]
    return o, (x, h1, h2)


MUTATIONS = {
    "grad_imag_sign": ("grad", _grad_imag_sign),
    "grad_no_mean": ("grad", lambda w, f, t: _orig["grad"](w, f, t) * f.shape[0]),
    "loss_no_scale": ("scale", lambda feat: np.ones(np.asarray(feat).shape[0])),
    "hidden_transposed": ("forward", _forward_transposed),
    "feature_sign": ("features", lambda t, e, o, eta: _orig["features"](t, e, o, eta) * np.array([1, 1, 1, 1, -1])),
    "teter_no_quartic": ("teter", lambda x: np.ones_like(np.asarray(x, np.float64))),
    "rows_shift_sign": ("rows", _rows_conj_d),
    "spai_no_conj": ("spai_optimum", lambda d, c: d / (np.abs(d) ** 2 + c)),
    "columns_keep_diag": ("operator_columns", lambda a: (np.diag(a).real.copy(), np.sum(np.abs(a) ** 2, axis=0))),
    "teter_eref_abs_weights": ("teter_diagonal", lambda kin, b: mo.teter(
        np.asarray(kin) / (np.sum(np.asarray(kin) * np.abs(b)) / np.sum(np.abs(b))))),
    "bf16_truncates": ("bf16_round", lambda w: (np.ascontiguousarray(np.asarray(w, np.float32)).view(np.uint32)
                                                & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(mo, attr, fn)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught the planted mistake {name}"
