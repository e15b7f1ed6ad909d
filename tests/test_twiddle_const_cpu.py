"""Host check of the compile-time twiddle table used by the whole-line plane kernel.

The table cos(2 pi k / N), 0 <= k <= N/4, is computed by the C++ compiler in
double-double arithmetic; here it is compiled on the host (the same clang the
device code uses, else g++) and compared with cosines evaluated in 60-digit
decimal arithmetic (Taylor series, pi from Machin's formula) and rounded once
to double.  Every entry must be the correctly rounded value; cos(pi/2) must be
exactly 0.
"""
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIZES = (16, 24, 32, 48, 64, 72)

PROGRAM = r"""
#include <cstdio>
#include "twiddle_const.h"
template <int N> void dump() {
  constexpr sgw::ctw::QuarterCos<N> q{};
  for (int k = 0; k <= N / 4; ++k) std::printf("%d %d %a\n", N, k, q.v[k]);
}
int main() { BODY return 0; }
"""


def _compiler():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++"), shutil.which("g++")):
        if c and os.path.exists(c):
            return c
    pytest.skip("no host C++ compiler")


def _pi():
    # Machin: pi = 16 atan(1/5) - 4 atan(1/239)
    def atan_inv(x):
        x = Decimal(x)
        s, t, n, k = Decimal(0), 1 / x, 1, 0
        while True:
            term = t / n
            if term == 0 or abs(term) < Decimal(10) ** -(getcontext().prec + 2):
                break
            s += term if k % 2 == 0 else -term
            t /= x * x
            n += 2
            k += 1
        return s
    return 16 * atan_inv(5) - 4 * atan_inv(239)


def _cos(x):
    s, term, j = Decimal(1), Decimal(1), 1
    while True:
        term = -term * x * x / ((2 * j - 1) * (2 * j))
        if abs(term) < Decimal(10) ** -(getcontext().prec + 2):
            return s
        s += term
        j += 1


def test_quarter_cos_table_is_correctly_rounded(tmp_path):
    getcontext().prec = 60
    pi = _pi()
    src = tmp_path / "tw.cpp"
    src.write_text(PROGRAM.replace("BODY", " ".join(f"dump<{n}>();" for n in SIZES)))
    exe = tmp_path / "tw"
    r = subprocess.run([_compiler(), "-std=c++17", "-O1", f"-I{ROOT}/paper_1812_03717_amd/csrc", str(src), "-o",
                        str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line.strip():
            continue
        n, k, v = line.split()
        n, k, v = int(n), int(k), float.fromhex(v)
        ref = _cos(2 * pi * k / n)
        if 4 * k == n:
            assert v == 0.0, (n, k, v)
        else:
            assert v == float(ref), (n, k, v, float(ref))
        seen += 1
    assert seen == sum(n // 4 + 1 for n in SIZES)
