"""The allocation-free entry point (run_chains_noalloc) against run_chains.

Each call of run_chains_noalloc must leave a simulation exactly as run_chains
leaves its twin (same network, chains and seed): chain states and recorded
indicator bits bit-exact.  Two calls in a row on one device, the second with
a smaller input (fewer chains, fewer steps), check that the shared launch
table carries nothing from one call into the next.  Both kernels (bit-sliced
and lane-per-chain) are covered, and the oracle confirms the chains.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1508_07828_amd as pkg
import pbnsynth as ps

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.lib()
    yield


def _twins(text, omega, seed, pats, max_len=2048):
    net = pkg.Network(text)
    a = pkg.Simulation(net, omega, seed, max_props=len(pats), max_len=max_len)
    b = pkg.Simulation(net, omega, seed, max_props=len(pats), max_len=max_len)
    a.reset(pats)
    b.reset(pats)
    return a, b


def _same(a, b, nprops):
    assert np.array_equal(a.read_state(), b.read_state())
    assert a.position() == b.position()
    L = a.position()[0]
    for q in range(nprops):
        assert np.array_equal(a.read_bits(q, 0, L), b.read_bits(q, 0, L)), q


@pytest.mark.parametrize("case", ["bitsliced", "lane"])
def test_noalloc_equals_run_chains(case):
    if case == "bitsliced":
        net = ps.random_network(np.random.default_rng(4), 300, (1, 4), (1, 6), 0.004)
        pats = [((7, 1), (299, 0)), ((3, 0),)]
        big, small = 1000, 130
    else:
        net = ps.small_network(5, 37, l_max=4, k_max=7, p=0.05)          # k = 7: lane-per-chain
        pats = [((0, 1), (5, 0))]
        big, small = 700, 70
    text = ps.to_text(net)
    # first call: many chains, burn-in and thinning
    say("noalloc {}: first call, {} chains".format(case, big))
    a, b = _twins(text, big, 11, pats)
    a.run(150, burn_in=7, thin=2)
    b.run_noalloc(150, burn_in=7, thin=2)
    _same(a, b, len(pats))
    # second call on another simulation with fewer chains and fewer steps
    say("noalloc {}: second call, {} chains".format(case, small))
    c, d = _twins(text, small, 12, pats)
    c.run(41)
    d.run_noalloc(41)
    _same(c, d, len(pats))
    ch = oracle.Chains(oracle.Net(text), small, 12, pats)
    ch.extend(41)
    assert np.array_equal(d.read_state(), ch.states)
    for q in range(len(pats)):
        assert np.array_equal(d.read_bits(q, 0, 41), ch.bits[q])
    # and the first simulation continues from where it stood
    a.run(33)
    b.run_noalloc(33)
    _same(a, b, len(pats))


@pytest.mark.parametrize("target_n", [803, 1100])
def test_noalloc_one_network_shapes(target_n):
    """More chains than the chip holds in latency shapes: both calls take the
    throughput shapes of one network alone on the chip (8 waves per block at
    n = 803, 12 beyond 1000 nodes) and leave identical chains, the second call
    smaller than the first."""
    jobs = ps.batched(512)
    job = min(jobs, key=lambda j: abs(j.net.n - target_n))
    text = ps.to_text(job.net)
    pats = job.patterns[:1]
    for omega, steps in ((32768, 24), (28672, 9)):
        say("noalloc one-network shape: n={} chains={} steps={}".format(job.net.n, omega, steps))
        a, b = _twins(text, omega, job.seed, pats, max_len=64)
        a.run(steps)
        b.run_noalloc(steps)
        _same(a, b, 1)


def test_noalloc_limits():
    net = pkg.Network(ps.to_text(ps.tiny().net))
    sim = pkg.Simulation(net, (1 << 18) + 1, 1, max_props=1, max_len=64)
    sim.reset([((0, 1),)])
    with pytest.raises(pkg.PbnError) as e:
        sim.run_noalloc(1)
    assert e.value.code == pkg.PBN_ELIMIT
    with pytest.raises(pkg.PbnError) as e:
        sim.run_noalloc(1000)                          # beyond the bit-stream capacity
    assert e.value.code == pkg.PBN_ELIMIT
    # at the limit itself the call runs and matches run_chains
    a, b = _twins(ps.to_text(ps.tiny().net), 1 << 18, 3, [((0, 1),)], max_len=64)
    a.run(5)
    b.run_noalloc(5)
    _same(a, b, 1)
