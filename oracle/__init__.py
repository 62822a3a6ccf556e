"""CPU oracle for the PBN steady-state hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library (``paper_1508_07828_amd``) and never imports it.

Layers:
  * ``sim.c``      plain C simulator (Philox4x32-10 stream, parser, transitions,
                   state-of-interest indicators), built into ``liboracle.so``;
  * ``stats``      the paper's formulas (Gelman-Rubin, two-state M/N, Skart-P);
  * ``drivers``    Alg. 3 (GR), Alg. 4 (parallel two-state), Alg. 5 (parallel
                   Skart) over oracle chains, and the one-chain Alg. 1
                   (sequential two-state) and Alg. 2 (sequential Skart);
  * ``exact``      brute-force 2^n transition matrix and stationary distribution.

The Skart procedures (Alg. 2, Alg. 5) follow a stated reading where the paper
defers to the published Skart method, whose constants it does not give: they
are pinned by hand-worked cases, the textbook t-interval special case and CI
coverage of exact stationary probabilities, but their parity against the
published Skart itself is unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile sim.c with gcc (plain -O2, no fast-math, no FP contraction)."""
    src = os.path.join(_HERE, "sim.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-ffp-contract=off", "-fno-fast-math", src, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.orc_parse.restype = vp
        L.orc_parse.argtypes = [ctypes.c_char_p]
        L.orc_free.argtypes = [vp]
        L.orc_error.restype = ctypes.c_char_p
        L.orc_n.argtypes = [vp]
        L.orc_p_thr.argtypes = [vp]
        L.orc_p_thr.restype = u32
        L.orc_nfun.argtypes = [vp]
        L.orc_node_thresholds.argtypes = [vp, i32, vp]
        L.orc_philox.argtypes = [vp, vp, vp]
        L.orc_uniform.argtypes = [u64, u32, u32, u32, u32]
        L.orc_uniform.restype = u32
        L.orc_init.argtypes = [vp, u64, u32, u32, vp]
        L.orc_run.argtypes = [vp, u64, u32, u32, vp, u64, u64, u32, vp, vp, vp, vp, i32]
        L.orc_run.restype = i32
        L.orc_step_one.argtypes = [vp, u64, u32, u32, vp, vp, vp]
        L.orc_sample_next.argtypes = [vp, u64, u32, vp, u32, u32, vp]
        L.orc_sample_next.restype = i32
        _lib = L
    return _lib


def philox(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return tuple(int(v) for v in o)


def uniform(seed: int, t: int, chain: int, node: int, tag: int) -> int:
    return int(lib().orc_uniform(seed, t, chain, node, tag))


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class Net:
    """A parsed network (oracle side)."""

    def __init__(self, text: str):
        h = lib().orc_parse(text.encode())
        if not h:
            raise ValueError("oracle parse error: " + lib().orc_error().decode())
        self._h = h
        self.n = int(lib().orc_n(h))
        self.p_thr = int(lib().orc_p_thr(h))

    def thresholds(self, i: int) -> List[int]:
        buf = (ctypes.c_uint32 * 64)()
        l = lib().orc_node_thresholds(self._h, i, buf)
        return [int(buf[j]) for j in range(l)]

    def step_one(self, seed: int, t: int, chain: int, s: np.ndarray):
        """One transition from state s (uint8[n]); returns (s_next, gamma)."""
        s = np.ascontiguousarray(s, dtype=np.uint8)
        nx = np.zeros(self.n, np.uint8)
        g = np.zeros(self.n, np.uint8)
        lib().orc_step_one(self._h, seed, t, chain, s.ctypes.data, nx.ctypes.data, g.ctypes.data)
        return nx, g

    def sample_next(self, seed: int, chain: int, s: np.ndarray, t0: int, count: int) -> np.ndarray:
        """Next-state indices of `count` transitions out of s (t = t0..t0+count-1)."""
        s = np.ascontiguousarray(s, dtype=np.uint8)
        out = np.zeros(count, np.uint32)
        if lib().orc_sample_next(self._h, seed, chain, s.ctypes.data, t0, count, out.ctypes.data):
            raise ValueError("n too large")
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None


def _props_csr(patterns):
    offs = [0]
    nodes: List[int] = []
    vals: List[int] = []
    for pat in patterns:
        for a, b in pat:
            nodes.append(int(a))
            vals.append(int(b))
        offs.append(len(nodes))
    return (np.asarray(offs, np.int32), np.asarray(nodes if nodes else [0], np.int32),
            np.asarray(vals if vals else [0], np.uint8))


class Chains:
    """omega oracle chains with their recorded indicator streams.

    Position l (1-based) of a chain is the state after transition l*thin - 1
    (0-based transitions; thin = 1: after transition l-1; the initial state
    s(0) is not recorded).  ``bits[q][c][l-1]`` is the indicator of property q
    at position l of chain c.
    """

    def __init__(self, net: Net, omega: int, seed: int, patterns, chain0: int = 0,
                 threads: int | None = None, thin: int = 1):
        self.net = net
        self.omega = int(omega)
        self.seed = int(seed)
        self.chain0 = int(chain0)
        self.thin = int(thin)
        self.patterns = [tuple(p) for p in patterns]
        self.threads = threads or default_threads()
        self.states = np.zeros((self.omega, net.n), np.uint8)
        lib().orc_init(net._h, self.seed, self.chain0, self.omega, self.states.ctypes.data)
        self.length = 0
        self.transitions = 0
        self._cap = 0
        self._bits = np.zeros((len(self.patterns), self.omega, 0), np.uint8)
        self._csr = _props_csr(self.patterns)

    @property
    def bits(self) -> np.ndarray:
        return self._bits[:, :, : self.length]

    def extend(self, k: int) -> None:
        k = int(k)
        if k <= 0:
            return
        need = self.length + k
        if need > self._cap:
            cap = max(need, 2 * self._cap, 256)
            nb = np.zeros((len(self.patterns), self.omega, cap), np.uint8)
            nb[:, :, : self.length] = self._bits[:, :, : self.length]
            self._bits, self._cap = nb, cap
        steps = k * self.thin
        out = np.zeros((len(self.patterns), self.omega, steps), np.uint8)
        offs, nodes, vals = self._csr
        rc = lib().orc_run(self.net._h, self.seed, self.chain0, self.omega, self.states.ctypes.data,
                           self.transitions, steps, len(self.patterns), offs.ctypes.data, nodes.ctypes.data,
                           vals.ctypes.data, out.ctypes.data if len(self.patterns) else None,
                           self.threads)
        if rc != 0:
            raise RuntimeError(lib().orc_error().decode())
        # every thin-th state is a recorded position
        self._bits[:, :, self.length: need] = out[:, :, self.thin - 1:: self.thin]
        self.length = need
        self.transitions += steps

    def extend_to(self, length: int) -> None:
        if length > self.length:
            self.extend(length - self.length)
