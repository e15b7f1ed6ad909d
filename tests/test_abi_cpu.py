"""Host-only checks of the C ABI: the library loads and exports every declared symbol,
and host-side argument validation answers without a GPU."""
import ctypes as C
import os
import re

from paper_1812_03717_amd import sgw
from tests.libutil import ensure_library

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sgw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:sgw|sternheimer)_\w+)\s*\(", src)))


def test_header_declares_the_binding_names():
    decl = declared_functions()
    assert set(decl) == set(sgw.EXPORTED), (set(decl) ^ set(sgw.EXPORTED))


def test_library_exports_every_declared_symbol():
    lib = ensure_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_side_calls():
    lib = ensure_library()
    assert b"gfx950" in lib.sgw_version()
    o = sgw.sgw_opts()
    assert lib.sgw_opts_default(C.byref(o)) == 0
    assert o.max_iter == 600 and o.alpha_pv == 1.0 and o.precision == 0
    # NULL arguments are rejected with a message, never a crash
    assert lib.sgw_opts_default(None) == sgw.SGW_ERR_INVALID_ARG
    assert b"NULL" in lib.sgw_last_error()
    n = C.c_size_t()
    assert lib.sternheimer_workspace_size(None, None, 1, 1, 1, 1, None, C.byref(n)) == sgw.SGW_ERR_INVALID_ARG
    assert lib.sgw_ctx_create(0, None, None) == sgw.SGW_ERR_INVALID_ARG
    assert lib.sgw_ham_create(None, None, None) == sgw.SGW_ERR_INVALID_ARG
    assert lib.sgw_apply_h(None, None, 1, None, None, 0) == sgw.SGW_ERR_INVALID_ARG
    assert lib.sgw_kernel_stats(None, b"hx_planes", None, None, None, None) == sgw.SGW_ERR_INVALID_ARG
    st = lib.sternheimer_solve(None, None, 0, None, None, 0, None, None, 0, None, 0, None, 0.1, 1e-8, None, None,
                               0, None, None)
    assert st == sgw.SGW_ERR_INVALID_ARG


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, from the C compiler."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{ROOT}/include/sgw.h"', 'int main(void) {',
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


def test_struct_layouts_match_the_binding(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes and field offsets."""
    import ctypes as C
    for cls, struct in ((sgw.sgw_opts, "sgw_opts"), (sgw.sgw_problem, "sgw_problem"),
                        (sgw.sgw_ham_desc, "sgw_ham_desc")):
        names = [f[0] for f in cls._fields_]
        size, offs = _c_layout(tmp_path, struct, names)
        assert C.sizeof(cls) == size, struct
        assert [getattr(cls, n).offset for n in names] == offs, struct
    size, offs = _c_layout(tmp_path, "sgw_solve_info", list(sgw.INFO_DTYPE.names))
    assert sgw.INFO_DTYPE.itemsize == size
    assert [sgw.INFO_DTYPE.fields[n][1] for n in sgw.INFO_DTYPE.names] == offs


def test_enum_values_match_the_binding(tmp_path):
    """Every status, flag, solver, precision, preconditioner, guess and plane-kernel constant of the
    binding has the value the header gives it (from the C compiler)."""
    import subprocess
    pairs = {"SGW_OK": sgw.SGW_OK, "SGW_NOT_CONVERGED": sgw.SGW_NOT_CONVERGED,
             "SGW_ERR_INVALID_ARG": sgw.SGW_ERR_INVALID_ARG, "SGW_ERR_HIP": sgw.SGW_ERR_HIP,
             "SGW_ERR_WORKSPACE": sgw.SGW_ERR_WORKSPACE, "SGW_ERR_UNSUPPORTED": sgw.SGW_ERR_UNSUPPORTED,
             "SGW_PROJ_SPLIT_BF16": sgw.PROJ_SPLIT_BF16}
    for names in (("FLAG", ("CONVERGED", "MAXITER", "BREAKDOWN", "NONFINITE", "ZERO_RHS", "PER_SHIFT")),
                  ("SOLVER", ("MULTISHIFT", "PER_SHIFT", "TAIL", "BLOCK")),
                  ("PC", ("NONE", "TETER", "LEARNED")), ("GUESS", ("ZERO", "LEARNED")),
                  ("FFT", ("AUTO", "LINE", "PAIR", "LDS", "TRI"))):
        for n in names[1]:
            pairs[f"SGW_{names[0]}_{n}"] = getattr(sgw, f"{names[0]}_{n}")
    pairs["SGW_FP64"], pairs["SGW_MIXED"] = sgw.FP64, sgw.MIXED
    keys = sorted(pairs)
    src = tmp_path / "enums.c"
    lines = ['#include <stdio.h>', f'#include "{ROOT}/include/sgw.h"', 'int main(void) {']
    lines += [f'  printf("%d\\n", (int){k});' for k in keys]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "enums"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert dict(zip(keys, got)) == {k: pairs[k] for k in keys}
