"""The exact build's reciprocal and square root (refinement steps without the
general sequences' operand scaling, the general operation outside 2^-767 ..
2^1000) agree bit for bit with the GPU's IEEE division and square root and
with the host's, over every exponent, both ends of the fast range, zeros,
infinities, NaNs and subnormals."""
import ctypes
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "hip", "libmathcheck.so")


def operands():
    rng = np.random.default_rng(1803)
    n = 1 << 20
    raw = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True).view(np.float64)
    wide = np.exp2(rng.uniform(-800.0, 1010.0, n)) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    phys = np.exp2(rng.uniform(-40.0, 40.0, n))
    sp = [0.0, -0.0, np.inf, -np.inf, np.nan, 5e-324, 2.2250738585072014e-308, 2.0 ** -767, 2.0 ** 1000,
          1.0, 9.81]
    edges = []
    for v in sp + [float(2.0 ** e) for e in range(-1074, 1024)]:
        for w in (v, -v):
            edges += [w, np.nextafter(w, 0.0), np.nextafter(w, np.inf)]
    return np.ascontiguousarray(np.concatenate([raw, wide, phys, np.array(edges)]))


@pytest.mark.gpu
def test_reciprocal_and_root_bitwise():
    print("case: exact reciprocal and square root, bitwise", flush=True)
    if not os.path.exists(LIB):
        raise RuntimeError("tests/hip/libmathcheck.so is not built: run __graft_entry__.build()")
    L = ctypes.CDLL(LIB)
    L.math_check.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]
    L.math_check.restype = ctypes.c_int
    x = operands()
    counts = (ctypes.c_longlong * 4)()
    rc = L.math_check(x.ctypes.data_as(ctypes.c_void_p), x.size, counts)
    assert rc == 0, rc
    assert list(counts) == [0, 0, 0, 0], list(counts)
