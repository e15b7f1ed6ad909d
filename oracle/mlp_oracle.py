"""FP64 reference of the learned diagonal preconditioner / initial-guess model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product may import or call this
module; only the test suite, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP path.

The paper has no learned component: its Sternheimer solves (Sec. 2.3, Eqs. 6-8)
are what the model accelerates, and a diagonal preconditioner or an initial
guess leaves their exact solution unchanged.  What is defined here is the
model the library trains and evaluates, written out plainly:

* features of plane wave G for band energy eps and shift z = omega + i*eta,
  with T = 0.5|k+G|^2 (Hartree):  f = (T/10, eps/10, omega, 100*eta, (T-eps-omega)/10);
* a perceptron 5 -> 64 -> 64 -> 4, tanh on the two hidden layers, linear output o;
* with s = 1/(T+1): preconditioner m = s (o0 + i o1), guess factor g = s (o2 + i o3);
* loss over rows with complex pairs (u_m, w_m), (u_g, w_g):
      L = (1/n) sum_rows |m u_m - w_m|^2 + |g u_g - w_g|^2.

Parameter vector order (row-major blocks): W1[64][5], b1[64], W2[64][64],
b2[64], W3[4][64], b3[4].

The gradient is by explicit backpropagation (chain rule through each layer);
it is pinned by central finite differences of ``loss`` in the tests.

Also here: the Teter-Payne-Allan diagonal, K(x) = P(x) / (P(x) + 16 x^4) with
P(x) = 27 + 18x + 12x^2 + 8x^3 (Phys. Rev. B 40, 12255 (1989)).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 5, 64, 4
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(w):
    """Parameter vector -> dict of FP64 arrays, in the documented order."""
    w = np.asarray(w, np.float64)
    assert w.shape == (N_PARAMS,)
    out, off = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = w[off:off + n].reshape(shape)
        off += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SIZES])


def features(t, eps, omega, eta):
    """Feature rows for kinetic energies t (array), scalars or arrays eps, omega, eta (Ha)."""
    t = np.asarray(t, np.float64)
    eps = np.broadcast_to(np.asarray(eps, np.float64), t.shape)
    omega = np.broadcast_to(np.asarray(omega, np.float64), t.shape)
    eta = np.broadcast_to(np.asarray(eta, np.float64), t.shape)
    return np.stack([t / 10.0, eps / 10.0, omega, 100.0 * eta, (t - eps - omega) / 10.0], axis=-1)


def forward(w, feat):
    """Raw outputs o [n][4] and the hidden activations."""
    p = unpack(w)
    x = np.asarray(feat, np.float64)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    o = h2 @ p["W3"].T + p["b3"]
    return o, (x, h1, h2)


def scale(feat):
    """s = 1/(T+1), with T recovered from the first feature."""
    return 1.0 / (10.0 * np.asarray(feat, np.float64)[:, 0] + 1.0)


def model_outputs(w, feat):
    """(m, g): complex preconditioner and guess factor per row."""
    o, _ = forward(w, feat)
    s = scale(feat)
    return s * (o[:, 0] + 1j * o[:, 1]), s * (o[:, 2] + 1j * o[:, 3])


def _pairs(target):
    t = np.asarray(target, np.float64)
    um = t[:, 0] + 1j * t[:, 1]
    wm = t[:, 2] + 1j * t[:, 3]
    ug = t[:, 4] + 1j * t[:, 5]
    wg = t[:, 6] + 1j * t[:, 7]
    return um, wm, ug, wg


def loss(w, feat, target):
    m, g = model_outputs(w, feat)
    um, wm, ug, wg = _pairs(target)
    n = m.shape[0]
    return float((np.sum(np.abs(m * um - wm) ** 2) + np.sum(np.abs(g * ug - wg) ** 2)) / n)


def grad(w, feat, target):
    """d loss / d w by backpropagation, FP64."""
    p = unpack(w)
    o, (x, h1, h2) = forward(w, feat)
    s = scale(feat)
    um, wm, ug, wg = _pairs(target)
    n = o.shape[0]
    # e = s (o_a + i o_b) u - w;  |e|^2 = Re(e)^2 + Im(e)^2
    # d|e|^2 / d o_a = 2 Re(conj(e) s u),  d|e|^2 / d o_b = 2 Re(conj(e) i s u) = -2 Im(conj(e) s u)
    d_o = np.zeros_like(o)
    for k, (u, tw) in enumerate(((um, wm), (ug, wg))):
        e = s * (o[:, 2 * k] + 1j * o[:, 2 * k + 1]) * u - tw
        c = np.conj(e) * s * u
        d_o[:, 2 * k] = 2.0 * c.real / n
        d_o[:, 2 * k + 1] = -2.0 * c.imag / n
    g = {}
    g["W3"] = d_o.T @ h2
    g["b3"] = d_o.sum(axis=0)
    d_z2 = (d_o @ p["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = d_z2.T @ h1
    g["b2"] = d_z2.sum(axis=0)
    d_z1 = (d_z2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d_z1.T @ x
    g["b1"] = d_z1.sum(axis=0)
    return pack(g)


def teter(x):
    """Teter-Payne-Allan diagonal K(x); x = T_G / E_ref >= 0."""
    x = np.asarray(x, np.float64)
    p = 27.0 + 18.0 * x + 12.0 * x ** 2 + 8.0 * x ** 3
    return p / (p + 16.0 * x ** 4)


def teter_diagonal(kin, b):
    """The per-shift Teter diagonal for right-hand side b: K(T_G / E_ref) with the kinetic energy
    of b as the reference, E_ref = sum_G T_G |b_G|^2 / sum_G |b_G|^2 (1 for b = 0)."""
    kin = np.asarray(kin, np.float64)
    w = np.abs(np.asarray(b)) ** 2
    eref = float(np.sum(kin * w) / np.sum(w)) if np.sum(w) > 0 else 1.0
    return teter(kin / eref)


def bf16_round(w):
    """FP32 weights rounded to the nearest BF16 value (ties to even), as FP64: the weights the
    solver's inference uses."""
    u = np.ascontiguousarray(np.asarray(w, np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def operator_columns(a0):
    """Column statistics of a dense operator: (Re diag, squared off-diagonal column norms)."""
    a0 = np.asarray(a0)
    d = np.diag(a0)
    off2 = np.sum(np.abs(a0) ** 2, axis=0) - np.abs(d) ** 2
    return d.real.copy(), off2


def rows(kin, diag, off2, eps, omega, eta, r, b, stride=1):
    """Training rows in FP64, same layout as the library's row builder.

    For vector a (band energy eps[a], shift omega[a] + i eta) and sampled plane
    wave u = stride * t: row 2t holds (D r, r, D b, b), row 2t + 1 holds
    (sqrt(c) r, 0, sqrt(c) b, 0), with D = diag - eps - z, c = off2, the r pair
    divided by ||r|| and the b pair by ||b|| (norms over the sampled plane waves).
    kin, diag, off2: [n_pw] in the vectors' order.
    """
    r = np.asarray(r)
    b = np.asarray(b)
    n_vec, npw = r.shape
    idx = np.arange(0, npw, stride)
    feats, tgts = [], []
    for a in range(n_vec):
        ra, ba = r[a, idx], b[a, idx]
        nr, nb = np.linalg.norm(ra), np.linalg.norm(ba)
        sr = 1.0 / nr if nr > 0 else 0.0
        sb = 1.0 / nb if nb > 0 else 0.0
        d = diag[idx] - eps[a] - (omega[a] + 1j * eta)
        c = np.sqrt(np.maximum(off2[idx], 0.0))
        f = features(kin[idx], eps[a], omega[a], eta)
        t = np.zeros((2 * idx.size, 8))
        p1 = [d * ra * sr, ra * sr, d * ba * sb, ba * sb]
        p2 = [c * ra * sr, 0 * ra, c * ba * sb, 0 * ba]
        for k in range(4):
            t[0::2, 2 * k], t[0::2, 2 * k + 1] = p1[k].real, p1[k].imag
            t[1::2, 2 * k], t[1::2, 2 * k + 1] = p2[k].real, p2[k].imag
        feats.append(np.repeat(f, 2, axis=0))
        tgts.append(t)
    return np.concatenate(feats), np.concatenate(tgts)


def spai_objective(m, d, c, r):
    """sum_G |r_G|^2 (|1 - d_G m_G|^2 + c_G |m_G|^2) / ||r||^2 for one residual r."""
    w = np.abs(r) ** 2
    return float(np.sum(w * (np.abs(1.0 - d * m) ** 2 + c * np.abs(m) ** 2)) / np.sum(w))


def spai_optimum(d, c):
    """Minimiser of |1 - d m|^2 + c |m|^2 over complex m: conj(d) / (|d|^2 + c)."""
    return np.conj(d) / (np.abs(d) ** 2 + c)
