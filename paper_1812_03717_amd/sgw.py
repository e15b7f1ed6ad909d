"""Thin ctypes binding of libsgw.so (argument marshalling only).

Every function keeps the name of the C entry point it wraps.  Device arrays
are torch tensors on the context's device (complex128 for plane-wave vectors,
float64 for the potential); all GPU work runs in the library's HIP kernels.
There is no fallback: if the library is missing or no GPU is present, the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgw.so")

SGW_OK, SGW_NOT_CONVERGED = 0, 1
SGW_ERR_INVALID_ARG, SGW_ERR_HIP, SGW_ERR_WORKSPACE, SGW_ERR_UNSUPPORTED = -1, -2, -3, -4
FLAG_CONVERGED, FLAG_MAXITER, FLAG_BREAKDOWN, FLAG_NONFINITE, FLAG_ZERO_RHS = 1, 2, 4, 8, 16
FLAG_PER_SHIFT = 32
SOLVER_MULTISHIFT, SOLVER_PER_SHIFT, SOLVER_TAIL, SOLVER_BLOCK = 0, 1, 2, 3
FP64, MIXED = 0, 1
PC_NONE, PC_TETER, PC_LEARNED = 0, 1, 2
GUESS_ZERO, GUESS_LEARNED = 0, 1
FFT_AUTO, FFT_LINE, FFT_PAIR, FFT_LDS, FFT_TRI = 0, 1, 2, 3, 4
PROJ_SPLIT_BF16 = 16  # sgw_apply_projector mode bit: split-BF16 contraction

INFO_DTYPE = np.dtype([("iters", "<i4"), ("flags", "<i4"), ("relres", "<f8"), ("occ_leak", "<f8")])

EXPORTED = [
    "sgw_last_error", "sgw_version", "sgw_ctx_create", "sgw_ctx_destroy", "sgw_ctx_set_profiling",
    "sgw_ctx_set_fft_planes", "sgw_plane_kernel",
    "sgw_ctx_reset_stats", "sgw_kernel_stats", "sgw_ham_create", "sgw_ham_destroy", "sgw_ham_npw",
    "sgw_apply_h", "sgw_apply_projector", "sgw_build_rhs", "sgw_opts_default",
    "sternheimer_workspace_size", "sternheimer_solve", "sgw_mlp_num_params", "sgw_mlp_create",
    "sgw_mlp_destroy", "sgw_mlp_get_weights", "sgw_mlp_set_weights", "sgw_mlp_forward", "sgw_mlp_grad",
    "sgw_mlp_train_step", "sgw_operator_columns", "sgw_mlp_rows", "sternheimer_batch_workspace_size",
    "sternheimer_solve_batch", "sgw_autotune", "sgw_precond_values", "sgw_apply_h_noalloc",
    "sgw_green_workspace_size", "sgw_green_solve", "sgw_ham_set_nonlocal", "sgw_ham_nproj",
    "sgw_density_response", "sgw_coulomb", "sgw_screened_coulomb", "sgw_green_pair_workspace_size",
    "sgw_green_pair_elements", "sgw_sigma_c", "sgw_aaa_fit", "sgw_spectral_function", "sgw_quasiparticle",
    "sgw_pade_fit", "sgw_pade_eval",
]


class SgwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sgw error {code}: {msg}")
        self.code = code


class sgw_ham_desc(C.Structure):
    _fields_ = [("grid", C.c_int32 * 3), ("recip", (C.c_double * 3) * 3), ("kvec", C.c_double * 3),
                ("n_pw", C.c_int32), ("miller", C.POINTER(C.c_int32)), ("v_loc", C.c_void_p)]


class sgw_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_iter", C.c_int32), ("alpha_pv", C.c_double),
                ("tol_safety", C.c_double), ("slots", C.c_int32), ("finalize_batch", C.c_int32),
                ("steps_per_sync", C.c_int32), ("solver", C.c_int32), ("precond", C.c_int32),
                ("guess", C.c_int32), ("tail_iter", C.c_int32), ("ps_max_iter", C.c_int32),
                ("ps_slots", C.c_int32), ("mlp", C.c_void_p), ("hist_r", C.c_void_p), ("hist_x", C.c_void_p),
                ("hist_iter", C.c_int32), ("mixed_switch", C.c_double), ("graph", C.c_int32),
                ("fft_planes", C.c_int32), ("basis_blocks", C.c_int32),
                ("shift_imag", C.POINTER(C.c_double))]


class sgw_problem(C.Structure):
    _fields_ = [("h_kq", C.c_void_p), ("h_k", C.c_void_p), ("n_occ", C.c_int32), ("n_band", C.c_int32),
                ("n_pert", C.c_int32), ("n_omega", C.c_int32), ("psi_occ_kq", C.c_void_p), ("psi_v", C.c_void_p),
                ("eps_v", C.POINTER(C.c_double)), ("dv_miller", C.POINTER(C.c_int32)),
                ("omega", C.POINTER(C.c_double)), ("eta", C.c_double), ("tol", C.c_double), ("opts", sgw_opts),
                ("dpsi", C.c_void_p), ("info", C.c_void_p), ("status", C.c_int32), ("worker", C.c_int32),
                ("ms", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsgw.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run `python -m paper_1812_03717_amd.build`")
    lib = C.CDLL(path)
    vp, i32, dbl, sz = C.c_void_p, C.c_int32, C.c_double, C.c_size_t
    lib.sgw_last_error.restype = C.c_char_p
    lib.sgw_version.restype = C.c_char_p
    sig = {
        "sgw_ctx_create": [C.c_int, vp, C.POINTER(vp)],
        "sgw_ctx_destroy": [vp],
        "sgw_ctx_set_profiling": [vp, C.c_char_p],
        "sgw_ctx_set_fft_planes": [vp, C.c_int],
        "sgw_plane_kernel": [vp, vp, C.c_int, C.POINTER(i32)],
        "sgw_ctx_reset_stats": [vp],
        "sgw_kernel_stats": [vp, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)],
        "sgw_ham_create": [vp, C.POINTER(sgw_ham_desc), C.POINTER(vp)],
        "sgw_ham_destroy": [vp],
        "sgw_apply_h": [vp, vp, C.c_int, vp, vp, C.c_int],
        "sgw_apply_h_noalloc": [vp, vp, C.c_int, vp, vp, C.c_int],
        "sgw_apply_projector": [vp, vp, C.c_int, vp, C.c_int, vp, vp, dbl, C.c_int],
        "sgw_build_rhs": [vp, vp, C.c_int, vp, vp, C.c_int, vp, C.c_int, C.POINTER(i32), vp],
        "sgw_density_response": [vp, vp, C.c_int, vp, vp, C.c_int, vp, C.c_int, C.POINTER(i32), C.c_int, vp, vp,
                                 dbl, C.c_int, vp],
        "sgw_coulomb": [vp, vp, C.c_int, C.POINTER(i32), dbl, C.POINTER(dbl)],
        "sgw_screened_coulomb": [vp, vp, vp, C.c_int, C.POINTER(i32), dbl, C.c_int, vp, vp, vp, vp],
        "sgw_green_pair_workspace_size": [vp, vp, C.c_int, C.c_int, C.c_int, C.POINTER(sgw_opts), C.POINTER(sz)],
        "sgw_green_pair_elements": [vp, vp, vp, C.c_int, vp, C.c_int, C.POINTER(i32), C.c_int, C.POINTER(dbl),
                                    C.POINTER(dbl), dbl, C.POINTER(sgw_opts), vp, sz, vp, vp],
        "sgw_sigma_c": [vp, C.c_int, C.c_int, C.c_int, vp, C.POINTER(dbl), C.c_int, vp, C.c_int, C.POINTER(i32), dbl,
                        dbl, dbl, vp],
        "sgw_aaa_fit": [C.c_int, vp, vp, dbl, C.c_int, C.POINTER(C.c_int), vp, vp, vp],
        "sgw_spectral_function": [vp, C.c_int, C.c_int, C.POINTER(i32), vp, vp, vp, C.c_int, C.POINTER(dbl), dbl,
                                  C.POINTER(dbl), C.POINTER(dbl), vp, vp],
        "sgw_quasiparticle": [C.c_int, vp, vp, vp, dbl, dbl, C.POINTER(dbl), C.POINTER(dbl)],
        "sgw_pade_fit": [C.c_int, vp, vp, vp],
        "sgw_pade_eval": [C.c_int, vp, vp, C.c_int, vp, vp],
        "sgw_opts_default": [C.POINTER(sgw_opts)],
        "sternheimer_workspace_size": [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(sgw_opts),
                                       C.POINTER(sz)],
        "sternheimer_solve": [vp, vp, C.c_int, vp, vp, C.c_int, vp, C.POINTER(dbl), C.c_int, C.POINTER(i32),
                              C.c_int, C.POINTER(dbl), dbl, dbl, C.POINTER(sgw_opts), vp, sz, vp, vp],
        "sgw_green_workspace_size": [vp, vp, C.c_int, C.c_int, C.POINTER(sgw_opts), C.POINTER(sz)],
        "sgw_green_solve": [vp, vp, C.c_int, C.POINTER(i32), C.c_int, C.POINTER(dbl), dbl, dbl, C.POINTER(sgw_opts),
                            vp, sz, vp, vp],
        "sgw_mlp_create": [vp, C.POINTER(C.c_float), C.c_uint64, C.POINTER(vp)],
        "sgw_mlp_destroy": [vp],
        "sgw_mlp_get_weights": [vp, C.POINTER(C.c_float)],
        "sgw_mlp_set_weights": [vp, C.POINTER(C.c_float)],
        "sgw_mlp_forward": [vp, vp, C.c_int, vp, vp],
        "sgw_mlp_grad": [vp, vp, C.c_int, vp, vp, vp, vp],
        "sgw_mlp_train_step": [vp, vp, C.c_int, vp, vp, C.c_float, C.POINTER(C.c_float)],
        "sgw_operator_columns": [vp, vp, C.c_int, vp, dbl, vp, vp],
        "sternheimer_batch_workspace_size": [vp, C.c_int, C.POINTER(sgw_problem), C.c_int, C.POINTER(sz)],
        "sternheimer_solve_batch": [vp, C.c_int, C.POINTER(sgw_problem), C.c_int, vp, sz],
        "sgw_autotune": [vp, C.POINTER(sgw_problem), C.POINTER(sgw_opts), C.POINTER(dbl)],
        "sgw_mlp_rows": [vp, vp, vp, vp, C.c_int, C.POINTER(dbl), C.POINTER(dbl), dbl, vp, vp, C.c_int, vp, vp],
        "sgw_precond_values": [vp, vp, C.c_int, C.c_int, vp, C.c_int, C.POINTER(dbl), C.POINTER(dbl), dbl, vp, vp,
                               vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.sgw_ham_npw.argtypes = [vp]
    lib.sgw_ham_npw.restype = C.c_int32
    lib.sgw_ham_nproj.argtypes = [vp]
    lib.sgw_ham_nproj.restype = C.c_int32
    lib.sgw_ham_set_nonlocal.argtypes = [vp, vp, C.c_int, vp, C.POINTER(C.c_double)]
    lib.sgw_ham_set_nonlocal.restype = C.c_int
    lib.sgw_mlp_num_params.argtypes = []
    lib.sgw_mlp_num_params.restype = C.c_int32
    _lib = lib
    return lib


def _check(code):
    if code < 0:
        raise SgwError(code, load_library().sgw_last_error().decode())
    return code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _require(t, dtype, device, shape=None, name="array"):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

class sgw_ctx_create:
    """Context on ``device`` enqueuing on ``stream`` (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib.sgw_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load_library().sgw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, kernels):
        """kernels: comma-separated kernel names, "all", or None."""
        _check(load_library().sgw_ctx_set_profiling(self.handle, kernels.encode() if kernels else None))

    def set_fft_planes(self, kernel):
        """Plane-pass kernel of H.x: FFT_AUTO, FFT_LINE, FFT_PAIR or FFT_LDS."""
        _check(load_library().sgw_ctx_set_fft_planes(self.handle, int(kernel)))

    def plane_kernel(self, ham, precision=0):
        """The plane-pass kernel H.x of `ham` runs under this context's setting (FFT_LINE/PAIR/LDS)."""
        out = C.c_int32()
        _check(load_library().sgw_plane_kernel(self.handle, ham.handle if hasattr(ham, "handle") else ham,
                                               int(precision), C.byref(out)))
        return out.value

    def reset_stats(self):
        _check(load_library().sgw_ctx_reset_stats(self.handle))

    def kernel_stats(self, name: str):
        n, ms, b, f = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        _check(load_library().sgw_kernel_stats(self.handle, name.encode(), C.byref(n), C.byref(ms), C.byref(b),
                                               C.byref(f)))
        return {"launches": n.value, "ms": ms.value, "bytes": b.value, "flops": f.value}


class sgw_ham_create:
    """Hamiltonian at one Bloch vector: grid, reciprocal rows, k, Miller list (host), V(r) (device float64)."""

    def __init__(self, ctx: sgw_ctx_create, grid, recip, kvec, miller, v_loc):
        lib = load_library()
        _require(v_loc, __import__("torch").float64, ctx.device, tuple(grid), "v_loc")
        self.ctx = ctx
        self.miller = np.ascontiguousarray(np.asarray(miller, np.int32))
        d = sgw_ham_desc()
        for a in range(3):
            d.grid[a] = int(grid[a])
            d.kvec[a] = float(kvec[a])
            for b in range(3):
                d.recip[a][b] = float(recip[a][b])
        d.n_pw = int(self.miller.shape[0])
        d.miller = self.miller.ctypes.data_as(C.POINTER(C.c_int32))
        d.v_loc = C.c_void_p(v_loc.data_ptr())
        h = C.c_void_p()
        _check(lib.sgw_ham_create(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h
        self.n_pw = d.n_pw
        self.grid = tuple(int(g) for g in grid)

    def set_nonlocal(self, beta, e_kb):
        """Separable non-local pseudopotential: beta device complex128 [n_proj][n_pw] (caller order),
        e_kb host energies [n_proj] (Ha); beta=None removes it."""
        sgw_ham_set_nonlocal(self.ctx, self, beta, e_kb)

    @property
    def n_proj(self):
        return int(load_library().sgw_ham_nproj(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            load_library().sgw_ham_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------

def sgw_ham_set_nonlocal(ctx, ham, beta, e_kb):
    import torch
    if beta is None:
        _check(load_library().sgw_ham_set_nonlocal(ctx.handle, ham.handle, 0, None, None))
        return
    _require(beta, torch.complex128, ctx.device, (beta.shape[0], ham.n_pw), "beta")
    e = np.ascontiguousarray(np.asarray(e_kb, np.float64))
    if e.shape != (beta.shape[0],):
        raise ValueError(f"e_kb has shape {e.shape}, expected ({beta.shape[0]},)")
    _check(load_library().sgw_ham_set_nonlocal(ctx.handle, ham.handle, int(beta.shape[0]), _ptr(beta),
                                               e.ctypes.data_as(C.POINTER(C.c_double))))


def sgw_apply_h(ctx, ham, x, precision=0):
    import torch
    _require(x, torch.complex128, ctx.device, (x.shape[0], ham.n_pw), "x")
    y = torch.empty_like(x)
    _check(load_library().sgw_apply_h(ctx.handle, ham.handle, int(x.shape[0]), _ptr(x), _ptr(y), int(precision)))
    return y


def sgw_apply_h_noalloc(ctx, ham, x, y, precision=0):
    """y = H x through the allocation-free entry point (y: a caller-allocated tensor like x)."""
    import torch
    _require(x, torch.complex128, ctx.device, (x.shape[0], ham.n_pw), "x")
    _require(y, torch.complex128, ctx.device, tuple(x.shape), "y")
    _check(load_library().sgw_apply_h_noalloc(ctx.handle, ham.handle, int(x.shape[0]), _ptr(x), _ptr(y),
                                              int(precision)))
    return y


def sgw_apply_projector(ctx, ham, psi, x, alpha=1.0, mode=0, y=None):
    import torch
    _require(x, torch.complex128, ctx.device, (x.shape[0], ham.n_pw), "x")
    _require(psi, torch.complex128, ctx.device, (psi.shape[0], ham.n_pw), "psi")
    if y is None:
        y = torch.zeros_like(x)
    _check(load_library().sgw_apply_projector(ctx.handle, ham.handle, int(psi.shape[0]), _ptr(psi),
                                              int(x.shape[0]), _ptr(x), _ptr(y), float(alpha), int(mode)))
    return y


def sgw_build_rhs(ctx, h_kq, psi_occ_kq, h_k, psi_v, dv_miller):
    import torch
    _require(psi_v, torch.complex128, ctx.device, (psi_v.shape[0], h_k.n_pw), "psi_v")
    _require(psi_occ_kq, torch.complex128, ctx.device, (psi_occ_kq.shape[0], h_kq.n_pw), "psi_occ_kq")
    dvm = np.ascontiguousarray(np.asarray(dv_miller, np.int32).reshape(-1, 3))
    n_band, n_pert = int(psi_v.shape[0]), int(dvm.shape[0])
    b = torch.empty((n_band, n_pert, h_kq.n_pw), dtype=torch.complex128, device=ctx.device)
    _check(load_library().sgw_build_rhs(ctx.handle, h_kq.handle, int(psi_occ_kq.shape[0]), _ptr(psi_occ_kq),
                                        h_k.handle, n_band, _ptr(psi_v), n_pert,
                                        dvm.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(b)))
    return b


def sgw_density_response(ctx, h_kq, psi_occ_kq, h_k, psi_v, dv_miller, dpsi_plus, dpsi_minus, weight=1.0,
                         chi=None, accumulate=False):
    """chi[j][g][h] (+)= weight * (2/Omega) sum_v <exp(i(q+G_g).r) u_v | dpsi_{v,h}(z_j) + dpsi_{v,h}(-z_j)>;
    dpsi_plus / dpsi_minus: [n_band][n_pert][n_omega][n_pw_kq] from solves at z and -z."""
    import torch
    dvm = np.ascontiguousarray(np.asarray(dv_miller, np.int32).reshape(-1, 3))
    n_band, n_pert = int(psi_v.shape[0]), int(dvm.shape[0])
    n_omega = int(dpsi_plus.shape[2])
    shape = (n_band, n_pert, n_omega, h_kq.n_pw)
    _require(psi_v, torch.complex128, ctx.device, (n_band, h_k.n_pw), "psi_v")
    _require(psi_occ_kq, torch.complex128, ctx.device, (psi_occ_kq.shape[0], h_kq.n_pw), "psi_occ_kq")
    _require(dpsi_plus, torch.complex128, ctx.device, shape, "dpsi_plus")
    _require(dpsi_minus, torch.complex128, ctx.device, shape, "dpsi_minus")
    if chi is None:
        chi = torch.empty((n_omega, n_pert, n_pert), dtype=torch.complex128, device=ctx.device)
        accumulate = False
    _require(chi, torch.complex128, ctx.device, (n_omega, n_pert, n_pert), "chi")
    _check(load_library().sgw_density_response(ctx.handle, h_kq.handle, int(psi_occ_kq.shape[0]), _ptr(psi_occ_kq),
                                               h_k.handle, n_band, _ptr(psi_v), n_pert,
                                               dvm.ctypes.data_as(C.POINTER(C.c_int32)), n_omega, _ptr(dpsi_plus),
                                               _ptr(dpsi_minus), float(weight), int(bool(accumulate)), _ptr(chi)))
    return chi


def sgw_coulomb(h_kq, h_k, dv_miller, r_cut=0.0):
    """v(q + G_p) (host float64 [n_pert]), bare or spherically truncated at r_cut."""
    dvm = np.ascontiguousarray(np.asarray(dv_miller, np.int32).reshape(-1, 3))
    v = np.zeros(dvm.shape[0], np.float64)
    _check(load_library().sgw_coulomb(h_kq.handle, h_k.handle, int(dvm.shape[0]),
                                      dvm.ctypes.data_as(C.POINTER(C.c_int32)), float(r_cut),
                                      v.ctypes.data_as(C.POINTER(C.c_double))))
    return v


def sgw_screened_coulomb(ctx, h_kq, h_k, dv_miller, chi, r_cut=0.0):
    """(eps, eps_inv, wbar), each [n_omega][n_pert][n_pert] on the device, from chi."""
    import torch
    dvm = np.ascontiguousarray(np.asarray(dv_miller, np.int32).reshape(-1, 3))
    n_pert = int(dvm.shape[0])
    n_omega = int(chi.shape[0])
    _require(chi, torch.complex128, ctx.device, (n_omega, n_pert, n_pert), "chi")
    eps, inv, wbar = (torch.empty_like(chi) for _ in range(3))
    _check(load_library().sgw_screened_coulomb(ctx.handle, h_kq.handle, h_k.handle, n_pert,
                                               dvm.ctypes.data_as(C.POINTER(C.c_int32)), float(r_cut), n_omega,
                                               _ptr(chi), _ptr(eps), _ptr(inv), _ptr(wbar)))
    return eps, inv, wbar


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def sgw_green_pair_elements(ctx, h_kmq, h_k, psi_n, g_miller, z, tol, opts=None, workspace=None):
    """(status, m [n_band][n_freq][n_g][n_g], info): <t_g| (z_j - H)^{-1} |t_h>, t_g = exp(-i(q+G_g).r) u_n, at the
    complex frequencies z (e.g. mu + 1j * w' on the imaginary axis)."""
    import torch
    _require(psi_n, torch.complex128, ctx.device, (psi_n.shape[0], h_k.n_pw), "psi_n")
    g = np.ascontiguousarray(np.asarray(g_miller, np.int32).reshape(-1, 3))
    zz = np.atleast_1d(np.asarray(z, np.complex128))
    zr, zi = np.ascontiguousarray(zz.real), np.ascontiguousarray(zz.imag)
    n_band, n_g, n_freq = int(psi_n.shape[0]), int(g.shape[0]), int(zz.shape[0])
    lib = load_library()
    o = C.byref(opts) if opts is not None else None
    n = C.c_size_t()
    _check(lib.sgw_green_pair_workspace_size(ctx.handle, h_kmq.handle, n_band, n_g, n_freq, o, C.byref(n)))
    ws = (workspace or Workspace(ctx)).get(int(n.value))
    m = torch.empty((n_band, n_freq, n_g, n_g), dtype=torch.complex128, device=ctx.device)
    info = torch.empty(n_band * n_g * n_freq * INFO_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    st = _check(lib.sgw_green_pair_elements(ctx.handle, h_kmq.handle, h_k.handle, n_band, _ptr(psi_n), n_g,
                                            g.ctypes.data_as(C.POINTER(C.c_int32)), n_freq, _dptr(zr), _dptr(zi),
                                            float(tol), o, _ptr(ws), C.c_size_t(ws.numel()), _ptr(m), _ptr(info)))
    return st, m, info


def sgw_sigma_c(ctx, m_elem, weights, wbar, w_index, volume, alpha=-1.0):
    """sigma [n_band][n_out] on the device; w_index host int [n_out][n_freq] into wbar's frequencies;
    alpha = -1 (imaginary axis) or 1j (real axis)."""
    import torch
    n_band, n_freq, n_g = int(m_elem.shape[0]), int(m_elem.shape[1]), int(m_elem.shape[2])
    _require(m_elem, torch.complex128, ctx.device, (n_band, n_freq, n_g, n_g), "m_elem")
    _require(wbar, torch.complex128, ctx.device, (wbar.shape[0], n_g, n_g), "wbar")
    idx = np.ascontiguousarray(np.asarray(w_index, np.int32))
    wq = np.ascontiguousarray(np.asarray(weights, np.float64))
    if idx.ndim != 2 or idx.shape[1] != n_freq or wq.shape != (n_freq,):
        raise ValueError("w_index must be [n_out][n_freq] and weights [n_freq]")
    a = complex(alpha)
    sigma = torch.empty((n_band, idx.shape[0]), dtype=torch.complex128, device=ctx.device)
    _check(load_library().sgw_sigma_c(ctx.handle, n_band, n_g, n_freq, _ptr(m_elem), _dptr(wq), int(wbar.shape[0]),
                                      _ptr(wbar), int(idx.shape[0]), idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                      float(volume), a.real, a.imag, _ptr(sigma)))
    return sigma


def sgw_aaa_fit(z, f, tol=1e-13, max_terms=100):
    """(z_sup, f_sup, w_sup) numpy complex arrays of the AAA approximant (host computation)."""
    z = np.ascontiguousarray(np.asarray(z, np.complex128))
    f = np.ascontiguousarray(np.asarray(f, np.complex128))
    mt = int(min(max_terms, len(z) - 1))
    zs, fs, ws = (np.zeros(max(mt, 1), np.complex128) for _ in range(3))
    n = C.c_int()
    _check(load_library().sgw_aaa_fit(len(z), z.ctypes.data_as(C.c_void_p), f.ctypes.data_as(C.c_void_p),
                                      float(tol), mt, C.byref(n), zs.ctypes.data_as(C.c_void_p),
                                      fs.ctypes.data_as(C.c_void_p), ws.ctypes.data_as(C.c_void_p)))
    return zs[:n.value].copy(), fs[:n.value].copy(), ws[:n.value].copy()


def sgw_pade_fit(z, f):
    """Continued-fraction coefficients a (numpy complex) of the Pade interpolant of f at z (host)."""
    z = np.ascontiguousarray(np.asarray(z, np.complex128))
    f = np.ascontiguousarray(np.asarray(f, np.complex128))
    a = np.zeros(len(z), np.complex128)
    _check(load_library().sgw_pade_fit(len(z), z.ctypes.data_as(C.c_void_p), f.ctypes.data_as(C.c_void_p),
                                       a.ctypes.data_as(C.c_void_p)))
    return a


def sgw_pade_eval(z, a, x):
    z = np.ascontiguousarray(np.asarray(z, np.complex128))
    a = np.ascontiguousarray(np.asarray(a, np.complex128))
    x = np.ascontiguousarray(np.atleast_1d(np.asarray(x, np.complex128)))
    out = np.zeros(len(x), np.complex128)
    _check(load_library().sgw_pade_eval(len(z), z.ctypes.data_as(C.c_void_p), a.ctypes.data_as(C.c_void_p), len(x),
                                        x.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p)))
    return out


def sgw_spectral_function(ctx, fits, omega, broad, eps_n, delta):
    """(sigma [n_band][n_omega], a [n_band][n_omega]) device tensors from per-state AAA fits."""
    import torch
    n_band = len(fits)
    nmax = max(len(f[0]) for f in fits)
    zs, fs, ws = (np.zeros((n_band, nmax), np.complex128) for _ in range(3))
    ns = np.zeros(n_band, np.int32)
    for i, (a, b, c) in enumerate(fits):
        ns[i] = len(a)
        zs[i, :len(a)], fs[i, :len(a)], ws[i, :len(a)] = a, b, c
    om = np.ascontiguousarray(np.asarray(omega, np.float64))
    e = np.ascontiguousarray(np.asarray(eps_n, np.float64))
    d = np.ascontiguousarray(np.asarray(delta, np.float64))
    sigma = torch.empty((n_band, len(om)), dtype=torch.complex128, device=ctx.device)
    a = torch.empty((n_band, len(om)), dtype=torch.float64, device=ctx.device)
    _check(load_library().sgw_spectral_function(ctx.handle, n_band, nmax, ns.ctypes.data_as(C.POINTER(C.c_int32)),
                                                zs.ctypes.data_as(C.c_void_p), fs.ctypes.data_as(C.c_void_p),
                                                ws.ctypes.data_as(C.c_void_p), len(om), _dptr(om), float(broad),
                                                _dptr(e), _dptr(d), _ptr(sigma), _ptr(a)))
    return sigma, a


def sgw_quasiparticle(fit, eps_n, delta):
    zs, fs, ws = (np.ascontiguousarray(x, np.complex128) for x in fit)
    e, z = C.c_double(), C.c_double()
    _check(load_library().sgw_quasiparticle(len(zs), zs.ctypes.data_as(C.c_void_p), fs.ctypes.data_as(C.c_void_p),
                                            ws.ctypes.data_as(C.c_void_p), float(eps_n), float(delta), C.byref(e),
                                            C.byref(z)))
    return e.value, z.value


def sgw_opts_default(**overrides):
    """Default options with overrides; mlp takes an sgw_mlp_create, hist_r / hist_x device tensors."""
    o = sgw_opts()
    _check(load_library().sgw_opts_default(C.byref(o)))
    for k, v in overrides.items():
        if k == "mlp" and v is not None and hasattr(v, "handle"):
            v = v.handle.value
        elif k in ("hist_r", "hist_x") and v is not None and hasattr(v, "data_ptr"):
            v = v.data_ptr()
        elif k == "shift_imag" and v is not None:
            arr = np.ascontiguousarray(np.asarray(v, np.float64))
            o._shift_imag = arr  # keeps the host array alive with the options
            v = arr.ctypes.data_as(C.POINTER(C.c_double))
        setattr(o, k, v)
    return o


def sternheimer_workspace_size(ctx, h_kq, n_occ, n_band, n_pert, n_omega, opts=None):
    o = opts if opts is not None else sgw_opts_default()
    n = C.c_size_t()
    _check(load_library().sternheimer_workspace_size(ctx.handle, h_kq.handle, n_occ, n_band, n_pert, n_omega,
                                                     C.byref(o), C.byref(n)))
    return int(n.value)


class Workspace:
    """Caller-owned device workspace (a torch uint8 tensor), reused across calls."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.buf = None

    def get(self, nbytes):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.ctx.device)
        return self.buf


def sternheimer_solve(ctx, h_kq, psi_occ_kq, h_k, psi_v, eps_v, dv_miller, omega, eta, tol, opts=None,
                      workspace=None, dpsi=None, info=None):
    """Returns (status, dpsi [n_band][n_pert][n_omega][n_pw_kq] complex128 tensor, info device uint8 tensor)."""
    import torch
    _require(psi_v, torch.complex128, ctx.device, (psi_v.shape[0], h_k.n_pw), "psi_v")
    _require(psi_occ_kq, torch.complex128, ctx.device, (psi_occ_kq.shape[0], h_kq.n_pw), "psi_occ_kq")
    eps = np.ascontiguousarray(np.asarray(eps_v, np.float64))
    om = np.ascontiguousarray(np.asarray(omega, np.float64))
    dvm = np.ascontiguousarray(np.asarray(dv_miller, np.int32).reshape(-1, 3))
    n_band, n_pert, n_omega, n_occ = int(psi_v.shape[0]), int(dvm.shape[0]), int(om.shape[0]), int(psi_occ_kq.shape[0])
    if eps.shape != (n_band,):
        raise ValueError("eps_v must have one energy per band")
    o = opts if opts is not None else sgw_opts_default()
    nbytes = sternheimer_workspace_size(ctx, h_kq, n_occ, n_band, n_pert, n_omega, o)
    ws = (workspace or Workspace(ctx)).get(nbytes)
    if dpsi is None:
        dpsi = torch.empty((n_band, n_pert, n_omega, h_kq.n_pw), dtype=torch.complex128, device=ctx.device)
    if info is None:
        info = torch.empty(n_band * n_pert * n_omega * INFO_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    st = _check(load_library().sternheimer_solve(
        ctx.handle, h_kq.handle, n_occ, _ptr(psi_occ_kq), h_k.handle, n_band, _ptr(psi_v),
        eps.ctypes.data_as(C.POINTER(C.c_double)), n_pert, dvm.ctypes.data_as(C.POINTER(C.c_int32)), n_omega,
        om.ctypes.data_as(C.POINTER(C.c_double)), float(eta), float(tol), C.byref(o), _ptr(ws),
        C.c_size_t(ws.numel()), _ptr(dpsi), _ptr(info)))
    return st, dpsi, info


def sgw_green_solve(ctx, h_k, cols, omega, eta, tol, opts=None, workspace=None, g=None, info=None):
    """Green's function columns: returns (status, G [n_col][n_omega][n_pw] complex128, info uint8 tensor)."""
    import torch
    cl = np.ascontiguousarray(np.asarray(cols, np.int32).reshape(-1))
    om = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(-1))
    n_col, n_omega = int(cl.shape[0]), int(om.shape[0])
    o = opts if opts is not None else sgw_opts_default()
    n = C.c_size_t()
    _check(load_library().sgw_green_workspace_size(ctx.handle, h_k.handle, n_col, n_omega, C.byref(o), C.byref(n)))
    ws = (workspace or Workspace(ctx)).get(int(n.value))
    if g is None:
        g = torch.empty((n_col, n_omega, h_k.n_pw), dtype=torch.complex128, device=ctx.device)
    if info is None:
        info = torch.empty(n_col * n_omega * INFO_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    st = _check(load_library().sgw_green_solve(
        ctx.handle, h_k.handle, n_col, cl.ctypes.data_as(C.POINTER(C.c_int32)), n_omega,
        om.ctypes.data_as(C.POINTER(C.c_double)), float(eta), float(tol), C.byref(o), _ptr(ws),
        C.c_size_t(ws.numel()), _ptr(g), _ptr(info)))
    return st, g, info


class Batch:
    """A batch of systems for sternheimer_solve_batch: add() marshals one problem (keeping its host
    arrays and output tensors alive); solve() runs them all."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.items = []

    def add(self, h_kq, psi_occ_kq, h_k, psi_v, eps_v, dv_miller, omega, eta, tol, opts=None, dpsi=None):
        """dpsi: optional caller-owned output tensor [n_band][n_pert][n_omega][n_pw_kq] (else allocated)."""
        import torch
        _require(psi_v, torch.complex128, self.ctx.device, (psi_v.shape[0], h_k.n_pw), "psi_v")
        _require(psi_occ_kq, torch.complex128, self.ctx.device, (psi_occ_kq.shape[0], h_kq.n_pw), "psi_occ_kq")
        eps = np.ascontiguousarray(np.asarray(eps_v, np.float64))
        om = np.ascontiguousarray(np.asarray(omega, np.float64))
        dvm = np.ascontiguousarray(np.asarray(dv_miller, np.int32).reshape(-1, 3))
        n_band, n_pert, n_omega = int(psi_v.shape[0]), int(dvm.shape[0]), int(om.shape[0])
        if dpsi is None:
            dpsi = torch.empty((n_band, n_pert, n_omega, h_kq.n_pw), dtype=torch.complex128, device=self.ctx.device)
        else:
            _require(dpsi, torch.complex128, self.ctx.device, (n_band, n_pert, n_omega, h_kq.n_pw), "dpsi")
        info = torch.empty(n_band * n_pert * n_omega * INFO_DTYPE.itemsize, dtype=torch.uint8, device=self.ctx.device)
        p = sgw_problem()
        p.h_kq, p.h_k = h_kq.handle.value, h_k.handle.value
        p.n_occ, p.n_band, p.n_pert, p.n_omega = int(psi_occ_kq.shape[0]), n_band, n_pert, n_omega
        p.psi_occ_kq, p.psi_v = psi_occ_kq.data_ptr(), psi_v.data_ptr()
        p.eps_v = eps.ctypes.data_as(C.POINTER(C.c_double))
        p.dv_miller = dvm.ctypes.data_as(C.POINTER(C.c_int32))
        p.omega = om.ctypes.data_as(C.POINTER(C.c_double))
        p.eta, p.tol = float(eta), float(tol)
        p.opts = opts if opts is not None else sgw_opts_default()
        p.dpsi, p.info = dpsi.data_ptr(), info.data_ptr()
        self.items.append(dict(problem=p, keep=(eps, om, dvm, psi_v, psi_occ_kq, h_kq, h_k), dpsi=dpsi, info=info,
                               shape=(n_band, n_pert, n_omega)))
        return len(self.items) - 1

    def _array(self):
        arr = (sgw_problem * len(self.items))()
        for i, it in enumerate(self.items):
            arr[i] = it["problem"]
        return arr

    def autotune(self, index):
        """sgw_autotune on one problem; stores the tuned options in it and returns the time spent (ms)."""
        best = sgw_opts()
        ms = C.c_double()
        p = self.items[index]["problem"]
        _check(load_library().sgw_autotune(self.ctx.handle, C.byref(p), C.byref(best), C.byref(ms)))
        p.opts = best
        return ms.value

    def workspace_size(self, n_workers):
        arr = self._array()
        n = C.c_size_t()
        _check(load_library().sternheimer_batch_workspace_size(self.ctx.handle, len(self.items), arr, n_workers,
                                                              C.byref(n)))
        return int(n.value)

    def solve(self, n_workers=4, workspace=None):
        """Returns the batch status; per-system status / worker / ms are stored in self.items."""
        arr = self._array()
        nbytes = self.workspace_size(n_workers)
        ws = (workspace or Workspace(self.ctx)).get(nbytes)
        st = _check(load_library().sternheimer_solve_batch(self.ctx.handle, len(self.items), arr, n_workers,
                                                          _ptr(ws), C.c_size_t(ws.numel())))
        for i, it in enumerate(self.items):
            it["status"], it["worker"], it["ms"] = arr[i].status, arr[i].worker, arr[i].ms
        return st


def info_to_numpy(info, shape=None):
    """Device info bytes -> structured numpy array (fields iters, flags, relres, occ_leak)."""
    a = info.cpu().numpy().view(INFO_DTYPE)
    return a.reshape(shape) if shape is not None else a


# ---------------------------------------------------------------------------
# learned preconditioner / initial guess
# ---------------------------------------------------------------------------

def sgw_mlp_num_params():
    return int(load_library().sgw_mlp_num_params())


class sgw_mlp_create:
    """The 5-64-64-4 model; init_w: host float32 [num_params] or None (seeded start)."""

    def __init__(self, ctx: sgw_ctx_create, init_w=None, seed: int = 0):
        lib = load_library()
        self.ctx = ctx
        h = C.c_void_p()
        w = None
        if init_w is not None:
            w = np.ascontiguousarray(np.asarray(init_w, np.float32))
            if w.shape != (sgw_mlp_num_params(),):
                raise ValueError("init_w has the wrong size")
        _check(lib.sgw_mlp_create(ctx.handle, w.ctypes.data_as(C.POINTER(C.c_float)) if w is not None else None,
                                  C.c_uint64(seed), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load_library().sgw_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self):
        w = np.empty(sgw_mlp_num_params(), np.float32)
        _check(load_library().sgw_mlp_get_weights(self.handle, w.ctypes.data_as(C.POINTER(C.c_float))))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(np.asarray(w, np.float32))
        if w.shape != (sgw_mlp_num_params(),):
            raise ValueError("weights have the wrong size")
        _check(load_library().sgw_mlp_set_weights(self.handle, w.ctypes.data_as(C.POINTER(C.c_float))))


def sgw_mlp_forward(ctx, mlp, feat):
    import torch
    _require(feat, torch.float32, ctx.device, (feat.shape[0], 5), "feat")
    out = torch.empty((feat.shape[0], 4), dtype=torch.float32, device=ctx.device)
    _check(load_library().sgw_mlp_forward(ctx.handle, mlp.handle, int(feat.shape[0]), _ptr(feat), _ptr(out)))
    return out


def sgw_mlp_grad(ctx, mlp, feat, target):
    """Returns (grad [num_params] device float32, loss [1] device float32)."""
    import torch
    n = int(feat.shape[0])
    _require(feat, torch.float32, ctx.device, (n, 5), "feat")
    _require(target, torch.float32, ctx.device, (n, 8), "target")
    g = torch.empty(sgw_mlp_num_params(), dtype=torch.float32, device=ctx.device)
    loss = torch.empty(1, dtype=torch.float32, device=ctx.device)
    _check(load_library().sgw_mlp_grad(ctx.handle, mlp.handle, n, _ptr(feat), _ptr(target), _ptr(g), _ptr(loss)))
    return g, loss


def sgw_mlp_train_step(ctx, mlp, feat, target, lr):
    """One Adam step; returns the loss before the step."""
    import torch
    n = int(feat.shape[0])
    _require(feat, torch.float32, ctx.device, (n, 5), "feat")
    _require(target, torch.float32, ctx.device, (n, 8), "target")
    loss = C.c_float()
    _check(load_library().sgw_mlp_train_step(ctx.handle, mlp.handle, n, _ptr(feat), _ptr(target), C.c_float(lr),
                                             C.byref(loss)))
    return float(loss.value)


def sgw_operator_columns(ctx, ham, psi, alpha=1.0):
    """(diag, off2): device float64 [n_pw] column statistics of H + alpha P_occ (caller's order)."""
    import torch
    _require(psi, torch.complex128, ctx.device, (psi.shape[0], ham.n_pw), "psi")
    diag = torch.empty(ham.n_pw, dtype=torch.float64, device=ctx.device)
    off2 = torch.empty_like(diag)
    _check(load_library().sgw_operator_columns(ctx.handle, ham.handle, int(psi.shape[0]), _ptr(psi), float(alpha),
                                               _ptr(diag), _ptr(off2)))
    return diag, off2


def sgw_mlp_rows(ctx, ham, diag, off2, eps, omega, eta, r, b, stride=1):
    """Training rows (feat [2 n_vec P][5], target [2 n_vec P][8]) from residuals r and right-hand sides b."""
    import torch
    n_vec = int(r.shape[0])
    _require(r, torch.complex128, ctx.device, (n_vec, ham.n_pw), "r")
    _require(b, torch.complex128, ctx.device, (n_vec, ham.n_pw), "b")
    _require(diag, torch.float64, ctx.device, (ham.n_pw,), "diag")
    _require(off2, torch.float64, ctx.device, (ham.n_pw,), "off2")
    e = np.ascontiguousarray(np.asarray(eps, np.float64).reshape(n_vec))
    om = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(n_vec))
    per = (ham.n_pw + stride - 1) // stride
    feat = torch.empty((2 * n_vec * per, 5), dtype=torch.float32, device=ctx.device)
    tgt = torch.empty((2 * n_vec * per, 8), dtype=torch.float32, device=ctx.device)
    _check(load_library().sgw_mlp_rows(ctx.handle, ham.handle, _ptr(diag), _ptr(off2), n_vec,
                                       e.ctypes.data_as(C.POINTER(C.c_double)),
                                       om.ctypes.data_as(C.POINTER(C.c_double)), float(eta), _ptr(r), _ptr(b),
                                       int(stride), _ptr(feat), _ptr(tgt)))
    return feat, tgt


def sgw_precond_values(ctx, ham, precond, b, eps, omega, eta, guess=0, mlp=None):
    """(m, x0): device complex128 [n_vec][n_pw], the per-shift solver's diagonal preconditioner and
    initial guess for right-hand sides b (caller's order), band energies eps and frequencies omega."""
    import torch
    n_vec = int(b.shape[0])
    _require(b, torch.complex128, ctx.device, (n_vec, ham.n_pw), "b")
    e = np.ascontiguousarray(np.asarray(eps, np.float64).reshape(n_vec))
    om = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(n_vec))
    m = torch.empty_like(b)
    x0 = torch.empty_like(b)
    _check(load_library().sgw_precond_values(ctx.handle, ham.handle, int(precond), int(guess),
                                             mlp.handle if mlp is not None else C.c_void_p(0), n_vec,
                                             e.ctypes.data_as(C.POINTER(C.c_double)),
                                             om.ctypes.data_as(C.POINTER(C.c_double)), float(eta), _ptr(b),
                                             _ptr(m), _ptr(x0)))
    return m, x0
