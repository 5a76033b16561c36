"""Pins for event delivery and the epoch spike exchange (Sec. II connection
tuples and minimum-delay epochs; Sec. IV-A exchange)."""
import numpy as np

import oracle
from tests import models
from workloads import gen


def _run(m, K, n):
    s = oracle.Sim(m, epoch_steps=K)
    tr = s.run(n, probes=oracle.cell_cv_begin(m)[:-1])
    return tr, s.spikes(), s.state()


def test_epoch_length_invariance_bitwise():
    """Any epoch length K <= min delay gives bitwise identical results."""
    m = models.identical_ring(6, kick_cells=(0, 3), n_steps=1200)
    m2 = gen.config2(n_cells=6, kick_all=False)
    for mm in (m, m2):
        ref = _run(mm, 200, 1200)
        for K in (1, 37, 100):
            got = _run(mm, K, 1200)
            assert np.array_equal(ref[0], got[0])
            for a, b in zip(ref[1], got[1]):
                assert np.array_equal(a, b)


def test_identical_ring_spike_steps_arithmetic_progression():
    """A ring of identical cells kicked at cell 0: each hop costs the delay
    plus one and the same spike latency."""
    n, D = 5, 200
    m = models.identical_ring(n, delay=D, n_steps=1300)
    s = oracle.Sim(m)
    s.run(1300)
    gid, st, _ = s.spikes()
    assert list(gid) == list(range(n)) + [0]
    hops = np.diff(st)
    assert np.all(hops == hops[0])
    assert hops[0] > D


def test_delay_shifts_target_spike_exactly():
    """Lengthening one connection by k steps delays the target spike by k."""
    base = None
    for extra in (0, 7, 31):
        m = models.chain(2, [200 + extra], n_steps=600)
        s = oracle.Sim(m)
        s.run(600)
        gid, st, _ = s.spikes()
        t1 = st[gid == 1]
        assert len(t1) == 1
        if base is None:
            base = t1[0]
        assert t1[0] - base == extra


def test_zero_weight_connection_delivers_nothing():
    m = models.chain(2, [200], w=0.0, n_steps=600)
    s = oracle.Sim(m)
    s.run(600)
    gid, _, _ = s.spikes()
    assert list(gid) == [0]


def test_event_brute_force_delivery_on_tiny_network():
    """Spikes of a small random network, replayed by brute force over all
    (spike, connection) pairs, reproduce the synaptic conductances exactly."""
    m = gen.config5(n_cells=6, n_in=4, n_steps=1200)
    # strong kicks on every cell's background synapse so the network spikes
    bg = np.array([np.nonzero(m["syn_cell"] == c)[0][-1] for c in range(6)], np.uint32)
    m["ev_syn"] = np.concatenate([m["ev_syn"], np.repeat(bg, 3)])
    m["ev_step"] = np.concatenate([m["ev_step"], np.tile([0, 410, 820], 6)])
    m["ev_w"] = np.concatenate([m["ev_w"], np.full(18, 0.3)])
    m["con_w"][:] = 0.05
    s = oracle.Sim(m)
    s.run(1200)
    gid, st, _ = s.spikes()
    assert len(gid) > 3
    # brute force: conductance of every synapse at the end of the run
    g = np.zeros(len(m["syn_cell"]))
    decay = np.exp(-gen.DT / m["syn_tau"])
    events = [(int(st[i]) + int(m["con_delay"][c]), int(m["con_syn"][c]), float(m["con_w"][c]))
              for i in range(len(gid)) for c in range(len(m["con_src"])) if m["con_src"][c] == gid[i]]
    events += [(int(a), int(b), float(w)) for a, b, w in zip(m["ev_step"], m["ev_syn"], m["ev_w"])]
    ok = 0
    for sidx in range(len(g)):
        val = 0.0
        for stp, sy, w in events:
            if sy == sidx and stp < 1200:
                val += 1000 * w * decay[sidx] ** (1200 - stp)
        ref = s.state()["g"][sidx]
        assert abs(val - ref) <= 1e-11 * max(1.0, abs(ref))
        ok += val > 0
    assert ok > 0
