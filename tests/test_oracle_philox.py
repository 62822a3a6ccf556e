"""Pins for the oracle's Philox4x32-10 and its uniform-draw stream.

* Against an independent implementation: rocRAND's Philox4x32-10 engine,
  evaluated on the host through a small helper built here.
* Statistical: byte and bit uniformity of the 32-bit draws.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats as sst

import oracle

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_ref.cpp")


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("ref") / "ref.so")
    subprocess.check_call([hipcc, "-O1", "-fPIC", "-shared", "--offload-arch=gfx950", HELPER, "-o", out])
    L = ctypes.CDLL(out)
    L.ref_philox.argtypes = [ctypes.c_void_p] * 3
    return L


def _ref(L, ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    L.ref_philox(c, k, o)
    return tuple(o)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(11)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF], [0xFFFFFFFF] * 2)]
    for _ in range(3000):
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        ctr[1] &= (1 << 30) - 1          # the reference's offset argument is 64-bit
        cases.append((ctr, [int(x) for x in rng.integers(0, 2 ** 32, 2)]))
    for ctr, key in cases:
        assert oracle.philox(ctr, key) == _ref(rocrand_ref, ctr, key), (ctr, key)


def test_uniform_is_uniform():
    # 32-bit draws over many (t, chain, node): byte histogram and bit balance.
    seed = 7828
    vals = np.array([oracle.uniform(seed, t, c, i, tag)
                     for t in range(40) for c in range(5) for i in range(50) for tag in (0, 2)],
                    dtype=np.uint64)
    for shift in (24, 16, 0):
        hist = np.bincount(((vals >> np.uint64(shift)) & np.uint64(0xFF)).astype(np.int64), minlength=256)
        assert sst.chisquare(hist).pvalue > 1e-4
    bits = ((vals[:, None] >> np.arange(32, dtype=np.uint64)[None, :]) & np.uint64(1)).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * np.sqrt(0.25 / vals.size))


def test_uniform_streams_distinct():
    # perturbation and selection draws of the same (t, chain, node) differ
    same = sum(oracle.uniform(1, t, 0, i, 0) == oracle.uniform(1, t, 0, i, 2)
               for t in range(20) for i in range(20))
    assert same == 0
