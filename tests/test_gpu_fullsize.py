"""GPU parity at the workloads' full sizes: the HIP library against the oracle.

* The large network (n = 2000) over 2000 transitions on 256 of its 8192 chains,
  in the launch shapes the solves use (node-split parts chosen automatically)
  and in the 16-wave shape.
* The large configuration solved end to end: 8192 chains, five 4-node state
  sets, Gelman-Rubin to R < 1.05, then the parallel Skart procedure (Sec. 4.3)
  at H* = 0.005, every result equal to the oracle's.
* The parallel Skart procedure with at least 1280 chains, where every chain
  holds one batch (no lag pairs, the randomness test passes at once), and with
  a cap reached while the batches grow.
* Integers bit-exact, floating point within 1e-12 relative (the Skart
  statistics are bit-equal: both sides take them from exact integer sums).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1508_07828_amd as pkg
import pbnsynth as ps
from oracle import drivers

pytestmark = pytest.mark.gpu

INT_KEYS = ("status", "psi_gr", "psi", "n", "N", "M", "kappa", "batches", "chain_len")
FP_KEYS = ("prob", "rhat", "ci_lo", "ci_hi")


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def assert_same_result(got, want, tag="", exact_fp=()):
    for k in INT_KEYS:
        assert got[k] == want[k], (tag, k, got[k], want[k])
    for k in FP_KEYS:
        a, b = got[k], want[k]
        if np.isnan(a) and np.isnan(b):
            continue
        if k in exact_fp:
            assert a == b, (tag, k, a, b)
        else:
            assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (tag, k, a, b)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.lib()
    yield
    pkg.set_kernel("auto", 0)
    pkg.set_split(0)


LARGE_STEPS = 2000
LARGE_GROUPS = (0, 2048, 4032, 8128)          # four 64-chain groups: 256 chains


@pytest.fixture(scope="module")
def large_oracle():
    job = ps.large()
    text = ps.to_text(job.net)
    onet = oracle.Net(text)
    out = {}
    for c0 in LARGE_GROUPS:
        say("oracle: large chains {}..{} x {} transitions".format(c0, c0 + 63, LARGE_STEPS))
        ch = oracle.Chains(onet, 64, job.seed, job.patterns, chain0=c0)
        init = ch.states.copy()
        ch.extend(LARGE_STEPS)
        out[c0] = (init, ch.states.copy(), ch.bits.copy())
    return job, text, out


@pytest.mark.parametrize("shape", ["auto", "bs16"])
def test_large_long_trajectories(large_oracle, shape):
    """8192 chains of the 2000-node network over 2000 transitions: states and
    the five state sets' indicators of 256 chains equal the oracle's.  'auto'
    runs the shapes of the large solve (128 groups on 256 CUs: node-split
    parts); 'bs16' one 16-wave block per group."""
    job, text, want = large_oracle
    if shape == "bs16":
        pkg.set_kernel("bitsliced", 16)
        pkg.set_split(1)
    pkg.profile_reset()
    pkg.profile_enable(True)
    try:
        say("large trajectories: 8192 chains x {} transitions, shape {}".format(LARGE_STEPS, shape))
        sim = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=5, max_len=LARGE_STEPS + 64)
        sim.reset(job.patterns)
        init = sim.read_state()
        sim.run(LARGE_STEPS // 2)
        sim.run(LARGE_STEPS - LARGE_STEPS // 2)
        st = sim.read_state()
        bits = [sim.read_bits(q, 0, LARGE_STEPS) for q in range(5)]
        prof = pkg.profile_read()
    finally:
        pkg.profile_enable(False)
        pkg.set_kernel("auto", 0)
        pkg.set_split(0)
    for c0, (w_init, w_st, w_bits) in want.items():
        assert np.array_equal(init[c0:c0 + 64], w_init), c0
        assert np.array_equal(st[c0:c0 + 64], w_st), c0
        for q in range(5):
            assert np.array_equal(bits[q][c0:c0 + 64], w_bits[q]), (c0, q)
    assert sim.position() == (LARGE_STEPS, LARGE_STEPS)
    if shape == "auto":
        assert prof["split_launches"] > 0, prof
    else:
        assert prof["split_launches"] == 0, prof


@pytest.mark.parametrize("target_n,chains", [(803, 65536), (2000, 32768)])
def test_owned_throughput_shapes(target_n, chains):
    """A plain run with more chains than the chip holds in latency shapes
    takes the throughput shapes of a launch that owns the CUs (8 waves per
    block at n = 803, 12 at n = 2000): states and indicators of three sampled
    64-chain groups equal the oracle's after 200 transitions."""
    jobs = ps.batched(512)
    job = min(jobs, key=lambda j: abs(j.net.n - target_n)) if target_n != 2000 else ps.large()
    text = ps.to_text(job.net)
    pats = job.patterns[:1]
    steps = 200
    say("owned throughput shape: n={} chains={} x {} transitions".format(job.net.n, chains, steps))
    sim = pkg.Simulation(pkg.Network(text), chains, job.seed, max_props=1, max_len=steps + 64)
    sim.reset(pats)
    sim.run(steps // 2)
    sim.run(steps - steps // 2)
    st = sim.read_state()
    bits = sim.read_bits(0, 0, steps)
    onet = oracle.Net(text)
    for c0 in (0, chains // 2 + 64, chains - 64):
        ch = oracle.Chains(onet, 64, job.seed, pats, chain0=c0)
        ch.extend(steps)
        assert np.array_equal(st[c0:c0 + 64], ch.states), c0
        assert np.array_equal(bits[c0:c0 + 64], ch.bits[0]), c0


def test_large_config_end_to_end():
    """The large configuration as the benchmark solves it (automatic shapes,
    node-split parts), against the oracle's Alg. 3 then Alg. 5 for each state
    set on one shared set of 8192 oracle chains (each set's result equals its
    solo run, since the chains do not depend on which sets are recorded)."""
    job = ps.large()
    text = ps.to_text(job.net)
    say("large end to end: GPU, 8192 chains, five state sets, Skart-P")
    pkg.profile_reset()
    pkg.profile_enable(True)
    try:
        sim = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=5, max_len=1 << 15)
        got = sim.estimate(job.patterns, job.r, job.confidence, method="skart", psrf_max=job.psrf_max)
        prof = pkg.profile_read()
    finally:
        pkg.profile_enable(False)
    assert prof["split_launches"] > 0, prof
    ch = oracle.Chains(oracle.Net(text), job.chains, job.seed, job.patterns)
    for q in range(5):
        say("large end to end: oracle state set {}".format(q))
        want = drivers.estimate_ci_in_parallel(ch, q, 256, job.psrf_max, job.r, job.confidence, 1 << 15)
        assert want["status"] == 0
        assert_same_result(got[q], want, ("large", q), exact_fp=("prob", "ci_lo", "ci_hi"))
    # the chains grew to the longest requirement: a Gelman-Rubin window
    # (2 psi positions) or a Skart batch set
    assert sim.position()[0] == max(max(2 * g["psi_gr"], g["chain_len"]) for g in got)


@pytest.mark.parametrize("omega", [1280, 2048, 1500])
def test_skart_one_batch_per_chain(omega):
    """omega >= 1280: eta0 = omega, one batch per chain, the randomness test
    has no within-chain pairs and passes at once, and the CI has no lag-1
    term; the batch size grows until H <= H*.  A rare state set (skewness
    beyond 4: batches of 16) beside a common one."""
    job = ps.medium()
    text = ps.to_text(job.net)
    net = job.net
    pats = [job.patterns[0], ((0, 1),), ((1, 0), (2, 1))]
    say("skart one batch per chain: medium network, omega {}".format(omega))
    sim = pkg.Simulation(pkg.Network(text), omega, 17 + omega, max_props=3, max_len=1 << 14)
    got = sim.estimate(pats, 0.004, 0.95, method="skart", psrf_max=1.1)
    want = drivers.solve(text, omega, 17 + omega, pats, 0.004, 0.95, 1.1, method="skart", cap=1 << 14)
    for q in range(3):
        assert want[q]["status"] == 0 and want[q]["batches"] == omega
        assert_same_result(got[q], want[q], (omega, q), exact_fp=("prob", "ci_lo", "ci_hi"))
    assert any(w["kappa"] > 1 for w in want)
    del net


def test_skart_cap_while_batches_grow():
    """A cap reached in the CI stage: both sides report the batch size and
    count they had grown to, and not converged."""
    job = ps.medium()
    text = ps.to_text(job.net)
    say("skart cap in the CI stage")
    sim = pkg.Simulation(pkg.Network(text), 64, 5, max_props=1, max_len=1 << 14)
    got = sim.estimate(job.patterns, 0.0005, 0.95, method="skart", psrf_max=1.1, max_len=3000)
    want = drivers.solve(text, 64, 5, job.patterns, 0.0005, 0.95, 1.1, method="skart", cap=3000)
    assert want[0]["status"] == drivers.NOT_CONVERGED and want[0]["kappa"] > 0
    assert_same_result(got[0], want[0], "cap")


BATCH_CAP = 1 << 17
ORACLE_BUDGET = 3e9                   # node-updates the sampled oracle solves may take in all


def test_batched_full_workload_sampled():
    """The 512-network batched workload in one call, as the benchmark runs it;
    eight networks' results equal the oracle's solo solves: the two smallest,
    two near the median size and the four largest whose solves fit the
    oracle's budget (the choice uses the GPU's chain lengths, the expected
    values come from the oracle alone)."""
    jobs = ps.batched(512)
    say("batched full workload: 512 networks on the GPU")
    nets = [pkg.Network(ps.to_text(j.net)) for j in jobs]
    sims = [pkg.Simulation(nt, j.chains, j.seed, max_props=1, max_len=BATCH_CAP) for nt, j in zip(nets, jobs)]
    got = pkg.batch_estimate(sims, [j.patterns for j in jobs], [j.r for j in jobs],
                             [j.confidence for j in jobs], psrf_max=1.1)
    assert all(g[0]["status"] == 0 for g in got)
    cost = [j.net.n * j.chains * g[0]["chain_len"] for j, g in zip(jobs, got)]
    by_n = sorted(range(len(jobs)), key=lambda b: jobs[b].net.n)
    pick = by_n[:2] + by_n[len(by_n) // 2: len(by_n) // 2 + 2]
    spent = sum(cost[b] for b in pick)
    for b in reversed(by_n):
        if len(pick) == 8:
            break
        if b not in pick and spent + cost[b] <= ORACLE_BUDGET:
            pick.append(b)
            spent += cost[b]
    assert len(pick) == 8 and max(jobs[b].net.n for b in pick) > 1500
    for b in pick:
        j = jobs[b]
        say("oracle: batched[{}] n={} chains={} chain_len={}".format(b, j.net.n, j.chains, got[b][0]["chain_len"]))
        want = drivers.solve(ps.to_text(j.net), j.chains, j.seed, j.patterns, j.r, j.confidence, 1.1,
                             cap=BATCH_CAP)
        assert_same_result(got[b][0], want[0], j.name)
