"""Host-side checks of the HIP library that need no GPU.

* The shared library loads and exports every function include/pbnssa.h declares.
* Its network compiler agrees with the oracle's parser: same thresholds, same
  rejections (both written independently from the canonical format).
* Its quantiles are bit-identical to the oracle's (both evaluate AS 241 and the
  Cornish-Fisher series in the same order), so sample sizes decided from them
  agree exactly.
"""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1508_07828_amd as pkg
import pbnsynth as ps
from oracle import stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1508_07828_amd import build
        build.build()


def test_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "pbnssa.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", hdr)) - {"sizeof", "if", "for", "while"}
    names = {n for n in names if n.startswith("pbn_") or n.startswith("run_chains") or n in ("psrf", "estimate_prob")}
    assert len(names) >= 25
    L = pkg.lib()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(pkg.EXPORTS) <= names


def _nets():
    yield ps.to_text(ps.tiny().net)
    yield ps.to_text(ps.medium().net)
    for s in range(4):
        yield ps.to_text(ps.small_network(s, 9, l_max=4, k_max=7))


def test_thresholds_match_oracle():
    for text in _nets():
        a, b = pkg.Network(text), oracle.Net(text)
        assert a.n == b.n and a.info.p_thr == b.p_thr
        for i in range(a.n):
            assert a.thresholds(i) == b.thresholds(i)


def test_density_and_sizes():
    job = ps.medium()
    net = pkg.Network(ps.to_text(job.net))
    assert abs(net.info.density - job.net.density()) < 1e-12
    assert net.info.nfun == job.net.n_functions()
    assert net.W == (job.net.n + 31) // 32
    assert net.sim_bytes(256, 1, 1 << 12) > 256 * net.W * 4


@pytest.mark.parametrize("bad", [
    "PBN 2 0.5\nN 0 1\nF 1.0 1 0 2\nN 1 1\nF 0.9 1 0 1\n",
    "PBN 2 0.5\nN 0 1\nF 1.0 2 1 1 6\nN 1 1\nF 1.0 1 0 1\n",
    "PBN 2 0.5\nN 0 1\nF 1.0 1 2 2\nN 1 1\nF 1.0 1 0 1\n",
    "PBN 2 1.5\nN 0 1\nF 1.0 1 1 2\nN 1 1\nF 1.0 1 0 1\n",
    "PBN 2 0.5\nN 0 1\nF 1.0 1 1 1f\nN 1 1\nF 1.0 1 0 1\n",
    "PBN 2 0.5\nN 1 1\nF 1.0 1 1 2\nN 0 1\nF 1.0 1 0 1\n",
    "PBN 2 0.5\nN 0 1\nF 1.0 1 1 2\n",
    "",
])
def test_rejects_like_oracle(bad):
    with pytest.raises(pkg.PbnError):
        pkg.Network(bad)
    with pytest.raises(ValueError):
        oracle.Net(bad)


def _nudged(rng, text):
    """The network text with one to three numbers moved a little (ids and counts
    by small steps or past the 16-bit range, probabilities by zero, halving,
    doubling or 1e-13 relative)."""
    t = text.split(" ")
    for _ in range(rng.randint(1, 3)):
        i = rng.randrange(len(t))
        w = t[i].strip()
        try:
            t[i] = t[i].replace(w, str(int(w) + rng.choice([-1, 1, -2, 2, 15, -15, 65536])))
        except ValueError:
            try:
                t[i] = t[i].replace(w, repr(float(w) * rng.choice([0.0, 0.5, 2.0, 1 + 1e-13, 1 - 1e-13])))
            except ValueError:
                pass
    return " ".join(t)


def test_parser_agrees_with_oracle_on_nudged_networks():
    """1500 networks with a few numbers nudged: the library accepts exactly
    what the oracle's parser accepts, and compiles the same thresholds."""
    import random
    rng = random.Random(1508)
    base = [ps.to_text(ps.tiny().net), ps.to_text(ps.small_network(3, 40, l_max=4, k_max=6, p=0.05)),
            ps.to_text(ps.random_network(np.random.default_rng(100), 33, (1, 4), (1, 6), 0.01))]
    accepted = 0
    for _ in range(1500):
        text = _nudged(rng, rng.choice(base))
        try:
            a = pkg.Network(text)
        except pkg.PbnError:
            a = None
        try:
            b = oracle.Net(text)
        except ValueError:
            b = None
        assert (a is None) == (b is None), text
        if a is not None:
            accepted += 1
            assert a.n == b.n and a.info.p_thr == b.p_thr
            for i in range(a.n):
                assert a.thresholds(i) == b.thresholds(i)
    assert 200 < accepted < 1400


def test_limits():
    big_k = "PBN 20 0.5\n" + "".join(
        "N {} 1\nF 1.0 17 {} 0\n".format(i, " ".join(str(v) for v in range(17))) for i in range(20))
    with pytest.raises(pkg.PbnError) as e:
        pkg.Network(big_k)
    assert e.value.code == pkg.PBN_ELIMIT


def test_sim_bytes_limits():
    """Simulation sizes beyond the stated limits report 0 bytes instead of a
    size whose arithmetic wrapped around."""
    net = pkg.Network(ps.to_text(ps.tiny().net))
    assert net.sim_bytes(8, 1, 1 << 16) > 0
    assert net.sim_bytes(1 << 24, 8, 0xFFFFFFFF) > 0
    assert net.sim_bytes((1 << 24) + 1, 1, 1024) == 0
    assert net.sim_bytes(8, 9, 1024) == 0
    assert net.sim_bytes(8, 1, 1 << 32) == 0
    assert net.sim_bytes(8, 1, (1 << 64) - 1) == 0


def test_quantiles_bit_identical():
    rng = np.random.default_rng(3)
    ps_ = list(rng.uniform(1e-12, 1 - 1e-12, 2000)) + [0.975, 0.995, 0.8, 0.5, 1e-300, 0.025]
    for p in ps_:
        assert pkg.normal_quantile(p) == stats.normal_quantile(p)
    for nu in (100, 1279, 5000, 8191):
        for p in (0.975, 0.995, 0.9, 0.025):
            assert pkg.t_quantile(p, nu) == stats.t_quantile(p, nu)


def _skart_cases():
    rng = np.random.default_rng(21)
    for omega, m, K in ((64, 20, 16), (3, 200, 1), (500, 3, 1000), (1500, 1, 77), (7, 90, 1 << 20),
                        (8192, 1, 3), (2, 640, 8), (1, 1279, 1), (101, 1, 1 << 16)):
        walk = np.cumsum(rng.normal(size=(omega, m)), axis=1)
        q = 1.0 / (1.0 + np.exp(-walk / 3.0 - rng.normal()))
        yield rng.binomial(K, q), K
    yield np.full((40, 5), 3), 7                         # all equal
    b = np.full((40, 5), 3)
    b[7, 2] = 4
    yield b, 7                                           # one batch off
    yield np.tile([0, 1], (3, 100)), 1                   # alternating 0-1 batches
    # batch means a few observations apart at a huge batch size: Q2 is tiny
    # beside S1^2, a cancellation that only exact sums survive
    b = np.full((1280, 1), (1 << 28) + 3, dtype=np.int64)
    b[::7] += 1
    b[::11] -= 2
    yield b, 1 << 29
    # at the observation limit itself (batch size x batches = 2^40)
    yield rng.integers((1 << 31) - 64, 1 << 31, size=(256, 2)), 1 << 31
    for _ in range(40):                                  # small random sets near the t interval's size
        omega = int(rng.integers(1, 50))
        m = int(rng.integers(1, 40))
        if omega * m < 101:
            m = 101 // omega + 1
        K = int(rng.integers(1, 5000))
        yield rng.integers(0, K + 1, size=(omega, m)), K


def test_skart_stats_bit_identical():
    """The library's Skart statistics equal the oracle's bit for bit: both take
    every sum over the batches exactly, so no decision (randomness test, H > H*)
    can depend on a summation order.  For each set, an H* placed at H and at its
    neighbouring doubles decides the same way on both sides."""
    for b, K in _skart_cases():
        got = pkg.skart_batch_stats(b, K, 0.95)
        mu, lo, hi = stats.adjusted_ci(b, K, 0.05)
        H = max(mu - lo, hi - mu)
        assert (got["mu"], got["ci_lo"], got["ci_hi"], got["H"]) == (mu, lo, hi, H), (b.shape, K)
        assert got["vn_passes"] == stats.von_neumann_passes(b), (b.shape, K)
        for h_star in (H, np.nextafter(H, 0.0), np.nextafter(H, 1.0), H * (1 + 1e-12), H * (1 - 1e-12)):
            assert (got["H"] > h_star) == (H > h_star)


def test_skart_stats_rejects():
    b = np.ones((2, 60), dtype=np.int32)
    for args in ((b, 0, 0.95), (b, 1, 1.0), (b[:, :50], 1, 0.95), (b * 3, 2, 0.95), (-b, 1, 0.95)):
        with pytest.raises(pkg.PbnError) as e:
            pkg.skart_batch_stats(*args)
        assert e.value.code == pkg.PBN_EINVAL
    with pytest.raises(pkg.PbnError) as e:
        pkg.skart_batch_stats(b, 1 << 34, 0.95)
    assert e.value.code == pkg.PBN_ELIMIT


def test_load_file(tmp_path):
    """Loading from a file gives the network loading its text gives; an
    unreadable path is PBN_EINVAL."""
    text = ps.to_text(ps.medium().net)
    f = tmp_path / "medium.pbn"
    f.write_text(text)
    a, b = pkg.Network(text), pkg.Network(path=str(f))
    assert (a.n, a.W, a.info.nfun, a.info.p_thr, a.info.blob_bytes) == (b.n, b.W, b.info.nfun, b.info.p_thr,
                                                                        b.info.blob_bytes)
    for i in range(a.n):
        assert a.thresholds(i) == b.thresholds(i)
    with pytest.raises(pkg.PbnError) as e:
        pkg.Network(path=str(tmp_path / "missing.pbn"))
    assert e.value.code == pkg.PBN_EINVAL
