"""Python binding of libpbnssa (steady-state analysis of PBNs on MI355X).

Argument marshalling only: every step of the method runs in the HIP library
(``libpbnssa.so``, built in-tree by ``build.py``).  PyTorch provides the device
buffers (uint8 tensors) and the HIP stream handles.  There is no CPU fallback:
if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbnssa.so")

PBN_OK, PBN_EINVAL, PBN_EFORMAT, PBN_ENOMEM, PBN_EDEVICE, PBN_ENOTCONV, PBN_ELIMIT = range(7)
TWO_STATE, SKART, SEQ_TWO_STATE, SEQ_SKART = 0, 1, 2, 3
MAX_PROPS = 8

EXPORTS = (
    "pbn_load", "pbn_free", "pbn_net_get_info", "pbn_net_thresholds", "pbn_sim_bytes", "pbn_sim_create",
    "pbn_sim_free", "pbn_sim_reset", "run_chains", "psrf", "pbn_window_counts", "pbn_batch_sums",
    "pbn_sim_read_state", "pbn_sim_read_bits", "pbn_sim_position", "pbn_sim_sync", "estimate_prob",
    "pbn_batch_run", "pbn_batch_estimate", "pbn_server_create", "pbn_server_free", "pbn_server_submit",
    "pbn_server_step", "pbn_server_poll", "pbn_server_memory", "pbn_normal_quantile", "pbn_t_quantile",
    "pbn_last_error", "pbn_profile_enable", "pbn_profile_read", "pbn_profile_reset", "pbn_set_kernel", "pbn_set_split", "pbn_set_split_polls",
    "pbn_autotune", "pbn_autotune_reset", "pbn_skart_batch_stats", "run_chains_noalloc", "pbn_load_file",
    "pbn_sim_set_kernel", "pbn_sim_set_split", "pbn_server_configure",
    "pbn_server_lane_stats",
)


class PbnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("pbnssa error {}: {}".format(code, msg))
        self.code = code


class Pattern(ctypes.Structure):
    _fields_ = [("nterms", ctypes.c_uint32), ("node", ctypes.POINTER(ctypes.c_uint32)),
                ("val", ctypes.POINTER(ctypes.c_uint8))]


class Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("psi0", ctypes.c_uint64), ("psrf_max", ctypes.c_double),
                ("eps", ctypes.c_double), ("max_len", ctypes.c_uint64), ("thin", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("prob", ctypes.c_double), ("ci_lo", ctypes.c_double), ("ci_hi", ctypes.c_double),
                ("rhat", ctypes.c_double), ("psi_gr", ctypes.c_uint64), ("psi", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("N", ctypes.c_uint64), ("M", ctypes.c_uint64),
                ("kappa", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("chain_len", ctypes.c_uint64),
                ("status", ctypes.c_int), ("reserved", ctypes.c_int), ("sample_size", ctypes.c_uint64),
                ("rounds", ctypes.c_uint64)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class NetInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("W", ctypes.c_uint32), ("nfun", ctypes.c_uint32),
                ("p_thr", ctypes.c_uint32), ("max_k", ctypes.c_uint32), ("max_l", ctypes.c_uint32),
                ("blob_bytes", ctypes.c_uint64), ("density", ctypes.c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("kernel_ms", ctypes.c_double), ("chain_steps", ctypes.c_double),
                ("node_updates", ctypes.c_double), ("alg_ops", ctypes.c_double), ("philox_evals", ctypes.c_double),
                ("split_launches", ctypes.c_uint64), ("split_fallbacks", ctypes.c_uint64)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Counts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("T1", "T2", "n00", "n01", "n10", "n11")]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slice_us", ctypes.c_double), ("ahead_us", ctypes.c_double), ("long_lane_us", ctypes.c_double),
                ("long_slice_us", ctypes.c_double), ("long_quarters", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class SkartStats(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("ci_lo", ctypes.c_double), ("ci_hi", ctypes.c_double),
                ("H", ctypes.c_double), ("vn_C", ctypes.c_double), ("vn_limit", ctypes.c_double),
                ("vn_passes", ctypes.c_int), ("reserved", ctypes.c_int)]


_lib = None


def lib():
    """Load libpbnssa.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpbnssa.so not built: run paper_1508_07828_amd/build.py")
    # torch first: its HIP runtime is then the one the library binds to (same
    # soname).  Loaded the other way round, torch would bring a second HIP
    # runtime into the process, whose device memory and streams the library's
    # runtime does not know, and the library's first HIP call fails.
    _torch()
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32, dbl, sz = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_size_t)
    sig = {
        "pbn_load": (i32, [ctypes.c_char_p, sz, ctypes.POINTER(vp)]),
        "pbn_load_file": (i32, [ctypes.c_char_p, ctypes.POINTER(vp)]),
        "pbn_sim_set_kernel": (i32, [vp, i32, u32]),
        "pbn_sim_set_split": (i32, [vp, i32]),
        "pbn_free": (None, [vp]),
        "pbn_net_get_info": (i32, [vp, ctypes.POINTER(NetInfo)]),
        "pbn_net_thresholds": (i32, [vp, u32, vp, u32]),
        "pbn_sim_bytes": (sz, [vp, u32, u32, u64]),
        "pbn_sim_create": (i32, [vp, u32, u64, u32, u64, vp, sz, vp, ctypes.POINTER(vp)]),
        "pbn_sim_free": (None, [vp]),
        "pbn_sim_reset": (i32, [vp, ctypes.POINTER(Pattern), u32]),
        "run_chains": (i32, [vp, u64, u64, u32]),
        "run_chains_noalloc": (i32, [vp, u64, u64, u32]),
        "psrf": (i32, [vp, u32, u64, ctypes.POINTER(dbl)]),
        "pbn_window_counts": (i32, [vp, u32, u64, u64, ctypes.POINTER(Counts)]),
        "pbn_batch_sums": (i32, [vp, u32, u64, u64, u64, vp]),
        "pbn_sim_read_state": (i32, [vp, vp]),
        "pbn_sim_read_bits": (i32, [vp, u32, u64, u64, vp]),
        "pbn_sim_position": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "pbn_sim_sync": (i32, [vp]),
        "estimate_prob": (i32, [vp, ctypes.POINTER(Pattern), u32, dbl, dbl, ctypes.POINTER(Opts),
                                ctypes.POINTER(Result)]),
        "pbn_batch_run": (i32, [vp, u32, vp, vp]),
        "pbn_batch_estimate": (i32, [vp, u32, ctypes.POINTER(Pattern), vp, vp, vp, vp, ctypes.POINTER(Opts),
                                     vp, ctypes.POINTER(Result)]),
        "pbn_server_create": (i32, [vp, sz, vp, ctypes.POINTER(vp)]),
        "pbn_server_free": (None, [vp]),
        "pbn_server_submit": (i32, [vp, vp, u32, u64, ctypes.POINTER(Pattern), u32, dbl, dbl,
                                    ctypes.POINTER(Opts), u64, ctypes.POINTER(u64)]),
        "pbn_server_step": (i32, [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "pbn_server_poll": (i32, [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(Result)]),
        "pbn_server_configure": (i32, [vp, ctypes.POINTER(ServerOpts)]),
        "pbn_server_lane_stats": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "pbn_server_memory": (i32, [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]),
        "pbn_normal_quantile": (dbl, [dbl]),
        "pbn_t_quantile": (dbl, [dbl, dbl]),
        "pbn_last_error": (ctypes.c_char_p, []),
        "pbn_profile_enable": (i32, [i32]),
        "pbn_profile_read": (i32, [ctypes.POINTER(Profile)]),
        "pbn_profile_reset": (i32, []),
        "pbn_set_kernel": (i32, [i32, u32]),
        "pbn_set_split": (i32, [u32]),
        "pbn_set_split_polls": (i32, [u32]),
        "pbn_autotune": (i32, [vp, ctypes.POINTER(TuneRow), u32, ctypes.POINTER(u32)]),
        "pbn_autotune_reset": (i32, []),
        "pbn_skart_batch_stats": (i32, [vp, u32, u64, u64, dbl, ctypes.POINTER(SkartStats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != PBN_OK:
        raise PbnError(rc, lib().pbn_last_error().decode())


def normal_quantile(p: float) -> float:
    return float(lib().pbn_normal_quantile(p))


def t_quantile(p: float, nu: float) -> float:
    return float(lib().pbn_t_quantile(p, nu))


def skart_batch_stats(bsum, kappa: int, confidence: float) -> Dict:
    """Skart statistics of integer batch sums bsum[omega][m] (host call)."""
    b = np.ascontiguousarray(bsum, dtype=np.int32)
    if b.ndim != 2:
        raise ValueError("bsum must be [omega][m]")
    out = SkartStats()
    _check(lib().pbn_skart_batch_stats(b.ctypes.data, b.shape[0], b.shape[1], int(kappa), float(confidence),
                                       ctypes.byref(out)))
    d = {k: getattr(out, k) for k, _ in out._fields_ if k != "reserved"}
    d["vn_passes"] = bool(d["vn_passes"])
    return d


def set_kernel(mode: str = "auto", waves: int = 0) -> None:
    """Trajectory-kernel choice: "auto", "lane" (lane per chain) or "bitsliced"."""
    _check(lib().pbn_set_kernel({"auto": 0, "lane": 1, "bitsliced": 2}[mode], waves))


def set_split(parts: int = 0) -> None:
    """Node-split form: 0 automatic, 1 never, P >= 2 forced P parts per 64-chain group."""
    _check(lib().pbn_set_split(parts))


def set_split_polls(polls: int = 0) -> None:
    """Counter polls before a node-split block gives up (0 = default; tests of the failure path)."""
    _check(lib().pbn_set_split_polls(polls))


class TuneRow(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("waves_throughput", ctypes.c_uint32),
                ("waves_latency", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("node_updates_per_s", ctypes.c_double), ("transition_us", ctypes.c_double)]


def autotune(stream=None) -> List[Dict]:
    """Measure the bit-sliced kernel's shapes per network size and use them from now on."""
    rows = (TuneRow * 16)()
    count = ctypes.c_uint32()
    _check(lib().pbn_autotune(_stream_handle(stream), rows, 16, ctypes.byref(count)))
    return [{f: getattr(rows[i], f) for f, _ in TuneRow._fields_ if f != "reserved"} for i in range(count.value)]


def autotune_reset() -> None:
    """Back to the built-in shape rule."""
    _check(lib().pbn_autotune_reset())


def profile_enable(on: bool = True) -> None:
    _check(lib().pbn_profile_enable(1 if on else 0))


def profile_reset() -> None:
    _check(lib().pbn_profile_reset())


def profile_read() -> Dict:
    """Totals of the event-timed trajectory-kernel launches since the last reset."""
    p = Profile()
    _check(lib().pbn_profile_read(ctypes.byref(p)))
    return p.as_dict()


# ------------------------------------------------------------ patterns

class _Patterns:
    """Keeps the ctypes arrays of a list of conjunction patterns alive."""

    def __init__(self, patterns: Sequence[Sequence[Tuple[int, int]]]):
        self.keep = []
        self.arr = (Pattern * max(1, len(patterns)))()
        for q, pat in enumerate(patterns):
            nodes = (ctypes.c_uint32 * max(1, len(pat)))(*[int(a) for a, _ in pat])
            vals = (ctypes.c_uint8 * max(1, len(pat)))(*[int(b) for _, b in pat])
            self.keep += [nodes, vals]
            self.arr[q] = Pattern(len(pat), ctypes.cast(nodes, ctypes.POINTER(ctypes.c_uint32)),
                                  ctypes.cast(vals, ctypes.POINTER(ctypes.c_uint8)))
        self.count = len(patterns)


def make_opts(method: str = "two_state", psi0: int = 256, psrf_max: float = 1.1, eps: float = 1e-10,
              max_len: int = 0, thin: int = 1) -> Opts:
    code = {"two_state": TWO_STATE, "skart": SKART, "sequential": SEQ_TWO_STATE,
            "sequential_skart": SEQ_SKART}[method]
    return Opts(code, psi0, psrf_max, eps, max_len, thin, 0)


# ------------------------------------------------------------ objects

class Network:
    """A parsed and compiled network (host memory)."""

    def __init__(self, text: str = None, path: str = None):
        h = ctypes.c_void_p()
        if path is not None:
            _check(lib().pbn_load_file(os.fsencode(path), ctypes.byref(h)))
        else:
            b = text.encode()
            _check(lib().pbn_load(b, len(b), ctypes.byref(h)))
        self._h = h
        info = NetInfo()
        _check(lib().pbn_net_get_info(h, ctypes.byref(info)))
        self.info = info
        self.n = info.n
        self.W = info.W

    def thresholds(self, node: int) -> List[int]:
        buf = (ctypes.c_uint32 * 64)()
        l = lib().pbn_net_thresholds(self._h, node, buf, 64)
        return [int(buf[j]) for j in range(l)]

    def sim_bytes(self, omega: int, max_props: int, max_len: int) -> int:
        return int(lib().pbn_sim_bytes(self._h, omega, max_props, max_len))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pbn_free(h)
            self._h = None


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Simulation:
    """omega chains of one network, held in a device buffer owned by a torch tensor."""

    def __init__(self, net: Network, omega: int, seed: int, max_props: int = 1, max_len: int = 1 << 16,
                 device: str = "cuda", stream=None):
        torch = _torch()
        self.net = net
        self.omega = int(omega)
        self.max_props = int(max_props)
        self.max_len = int(max_len)
        nbytes = net.sim_bytes(self.omega, self.max_props, self.max_len)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        _check(lib().pbn_sim_create(net._h, self.omega, int(seed), self.max_props, self.max_len,
                                    self.buffer.data_ptr(), nbytes, self.stream, ctypes.byref(h)))
        self._h = h
        self.nprops = 0

    def reset(self, patterns: Sequence[Sequence[Tuple[int, int]]]) -> None:
        P = _Patterns(patterns)
        _check(lib().pbn_sim_reset(self._h, P.arr, P.count))
        self.nprops = P.count

    def run(self, steps: int, burn_in: int = 0, thin: int = 1) -> None:
        _check(lib().run_chains(self._h, burn_in, steps, thin))

    def set_kernel(self, mode: str = "global", waves: int = 0) -> None:
        """This simulation's kernel choice ("global": the process-wide one)."""
        code = {"global": -1, "auto": 0, "lane": 1, "bitsliced": 2}[mode]
        _check(lib().pbn_sim_set_kernel(self._h, code, waves))

    def set_split(self, parts: int = -1) -> None:
        """This simulation's node-split parts (-1: the process-wide setting)."""
        _check(lib().pbn_sim_set_split(self._h, parts))

    def run_noalloc(self, steps: int, burn_in: int = 0, thin: int = 1) -> None:
        """run_chains_noalloc: the same extension, with no allocation."""
        _check(lib().run_chains_noalloc(self._h, burn_in, steps, thin))

    def sync(self) -> None:
        _check(lib().pbn_sim_sync(self._h))

    def psrf(self, prop: int, psi: int) -> float:
        r = ctypes.c_double()
        _check(lib().psrf(self._h, prop, psi, ctypes.byref(r)))
        return r.value

    def window_counts(self, prop: int, lo: int, hi: int) -> Dict[str, int]:
        c = Counts()
        _check(lib().pbn_window_counts(self._h, prop, lo, hi, ctypes.byref(c)))
        return {k: int(getattr(c, k)) for k, _ in Counts._fields_}

    def batch_sums(self, prop: int, base: int, kappa: int, m: int) -> np.ndarray:
        out = np.zeros(self.omega * m, np.int32)
        _check(lib().pbn_batch_sums(self._h, prop, base, kappa, m, out.ctypes.data))
        return out.reshape(self.omega, m)

    def read_state(self) -> np.ndarray:
        """Chain states unpacked to uint8 [omega][n]."""
        W, n = self.net.W, self.net.n
        out = np.zeros(self.omega * W, np.uint32)
        _check(lib().pbn_sim_read_state(self._h, out.ctypes.data))
        words = out.reshape(self.omega, W)
        bits = (words[:, :, None] >> np.arange(32, dtype=np.uint32)[None, None, :]) & 1
        return bits.reshape(self.omega, W * 32)[:, :n].astype(np.uint8)

    def read_bits(self, prop: int, pos0: int, npos: int) -> np.ndarray:
        out = np.zeros(self.omega * npos, np.uint8)
        _check(lib().pbn_sim_read_bits(self._h, prop, pos0, npos, out.ctypes.data))
        return out.reshape(self.omega, npos)

    def position(self) -> Tuple[int, int]:
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pbn_sim_position(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def estimate(self, patterns, r: float, confidence: float = 0.95, **opts) -> List[Dict]:
        P = _Patterns(patterns)
        o = make_opts(**opts)
        res = (Result * P.count)()
        _check(lib().estimate_prob(self._h, P.arr, P.count, r, confidence, ctypes.byref(o), res))
        self.nprops = P.count
        return [res[q].as_dict() for q in range(P.count)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pbn_sim_free(h)
            self._h = None


def batch_run(sims: Sequence[Simulation], steps: Sequence[int], stream=None) -> None:
    arr = (ctypes.c_void_p * len(sims))(*[s._h.value for s in sims])
    st = (ctypes.c_uint64 * len(sims))(*[int(x) for x in steps])
    _check(lib().pbn_batch_run(arr, len(sims), st, _stream_handle(stream)))


def batch_estimate(sims: Sequence[Simulation], patterns: Sequence[Sequence], r: Sequence[float],
                   confidence: Sequence[float], stream=None, **opts) -> List[List[Dict]]:
    count = len(sims)
    flat = [p for ps_ in patterns for p in ps_]
    P = _Patterns(flat)
    nprops = (ctypes.c_uint32 * count)(*[len(p) for p in patterns])
    offs, acc = [], 0
    for p in patterns:
        offs.append(acc)
        acc += len(p)
    off = (ctypes.c_uint32 * count)(*offs)
    rr = (ctypes.c_double * count)(*r)
    cc = (ctypes.c_double * count)(*confidence)
    arr = (ctypes.c_void_p * count)(*[s._h.value for s in sims])
    o = make_opts(**opts)
    res = (Result * max(1, len(flat)))()
    _check(lib().pbn_batch_estimate(arr, count, P.arr, nprops, off, rr, cc, ctypes.byref(o),
                                    _stream_handle(stream), res))
    out = []
    for i, p in enumerate(patterns):
        out.append([res[offs[i] + q].as_dict() for q in range(len(p))])
    for s, p in zip(sims, patterns):
        s.nprops = len(p)
    return out


class Server:
    """Continuous-batching server over a device arena (torch uint8 tensor)."""

    def __init__(self, arena_bytes: int, device: str = "cuda", stream=None):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().pbn_server_create(self.arena.data_ptr(), int(arena_bytes), _stream_handle(stream),
                                       ctypes.byref(h)))
        self._h = h
        self._nprops = {}

    def submit(self, net: Network, omega: int, seed: int, patterns, r: float, confidence: float = 0.95,
               max_len: int = 1 << 16, **opts) -> int:
        P = _Patterns(patterns)
        o = make_opts(**opts)
        rid = ctypes.c_uint64()
        _check(lib().pbn_server_submit(self._h, net._h, omega, seed, P.arr, P.count, r, confidence,
                                       ctypes.byref(o), max_len, ctypes.byref(rid)))
        self._nprops[rid.value] = P.count
        return int(rid.value)

    def configure(self, slice_us: float = 0.0, ahead_us: float = 0.0, long_lane_us: float = 0.0,
                  long_slice_us: float = 0.0, long_quarters: int = 0) -> None:
        """Round scheduling (see pbn_server_configure; 0 keeps a default)."""
        o = ServerOpts(float(slice_us), float(ahead_us), float(long_lane_us), float(long_slice_us),
                       int(long_quarters), 0)
        _check(lib().pbn_server_configure(self._h, ctypes.byref(o)))

    def lane_stats(self) -> Tuple[int, int]:
        """(requests moved to the long lane, rounds it began)."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pbn_server_lane_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def step(self) -> Tuple[int, int, int]:
        a, w, d = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().pbn_server_step(self._h, ctypes.byref(a), ctypes.byref(w), ctypes.byref(d)))
        return a.value, w.value, d.value

    def poll(self, rid: int) -> Optional[List[Dict]]:
        n = self._nprops[rid]
        res = (Result * n)()
        ready = ctypes.c_int()
        _check(lib().pbn_server_poll(self._h, rid, ctypes.byref(ready), res))
        if not ready.value:
            return None
        return [res[q].as_dict() for q in range(n)]

    def memory(self) -> Tuple[int, int]:
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().pbn_server_memory(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pbn_server_free(h)
            self._h = None
