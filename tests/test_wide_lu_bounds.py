"""Bounds of the large-mechanism LU's index arithmetic, checked on the CPU.

`tests/wide_lu_bounds.c` replays the workgroup kernel's left-looking blocked
LU and its triangular solves (their loops, bounds and guards, thread by
thread, with the waves' register arrays as arrays per thread) with every LDS
and HBM buffer allocated on its own at exactly the kernel's size, built with
AddressSanitizer. It is run for every state size of the workgroup kernel
(65..256), so every tail panel width appears, including 1 (n = 1 mod 12) and
a full last panel (n = 0 mod 12), and every count of row slots per lane (2, 3
and 4). The matrices include pivots taken from the last row at every step, a
singular last column and a zero pivot in the middle, whose multipliers must
not reach later columns. The integrator's form of the call, where the LU
receives J and forms g I - J as it first reads each column, is run as well. Uninitialised buffers and the padding rows hold
NaN, so any use of them shows in the factors. The replica's factors and
pivots must equal the oracle's in every bit, which shows that it follows the
kernel's arithmetic; its solutions must match the oracle's to rounding.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wide_lu_bounds.c")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("wlb")
    out = str(d / "wide_lu_bounds")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off"] + san
                          + ["-o", out, SRC, "-lm"])
    return out, str(d)


def _read(path):
    raw = open(path, "rb").read()
    off, out = 0, []
    while off < len(raw):
        n, ld, info = np.frombuffer(raw, dtype=np.int32, count=3, offset=off)
        off += 12
        A = np.frombuffer(raw, dtype=np.float64, count=n * n, offset=off).reshape(n, n)
        off += 8 * n * n
        F = np.frombuffer(raw, dtype=np.float64, count=n * n, offset=off).reshape(n, n)
        off += 8 * n * n
        piv = np.frombuffer(raw, dtype=np.int32, count=n, offset=off)
        off += 4 * n
        x = np.frombuffer(raw, dtype=np.float64, count=n, offset=off)
        off += 8 * n
        out.append((int(n), int(ld), int(info), A, F, piv, x))
    return out


# every size of the workgroup kernel on random matrices; the other patterns on
# windows of sizes that hold every tail width, and the largest sizes
CASES = [(0, 65, 256, 0), (0, 65, 256, 1)] + [(pattern, 140, 163, 0) for pattern in (1, 2, 3, 4)] + [
    (1, 233, 256, 0), (4, 233, 256, 0), (1, 140, 163, 1), (3, 140, 163, 1)]


@pytest.mark.parametrize("pattern,n_lo,n_hi,form", CASES)
def test_wide_lu_in_bounds(exe, pattern, n_lo, n_hi, form):
    path, d = exe
    out = os.path.join(d, "r_%d_%d_%d.bin" % (pattern, n_lo, form))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23")
    r = subprocess.run([path, out, str(n_lo), str(n_hi), str(pattern), str(form)], env=env, capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    res = _read(out)
    assert [n for n, *_ in res] == list(range(n_lo, n_hi + 1))
    tails = set()
    for n, ld, info, A, F, piv, x in res:
        tails.add((n - 1) % 12 + 1)
        LU, piv_o, info_o = O.lu(A)
        assert info == info_o, n
        assert np.array_equal(piv, piv_o), n
        assert np.array_equal(F, LU), n          # same operations in the same order
        if pattern == 1 and not form:
            assert (piv[:-1] == n - 1).all(), n
        if pattern == 2:
            assert (piv == np.arange(n)).all(), n
        if info == 0:
            xo = O.lu_solve(LU, piv_o, np.arange(n, dtype=float) + 1)
            assert np.max(np.abs(x - xo)) <= 1e-12 * np.max(np.abs(xo)), n
        elif pattern == 3 and not form:
            assert info == n, n
        else:
            assert pattern == 4 and info == n // 2 + 1, n
    assert tails == set(range(1, 13))   # every tail panel width, 1 and full included
