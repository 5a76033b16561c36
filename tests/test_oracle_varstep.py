"""Pins for the oracle's variable time step (Sec. II: the step is shortened
so that every event falls at the beginning of a step; steps otherwise end on
the grid k dt): with every time on the step grid it is the fixed-step scheme
exactly; an uneven step sequence decays a passive cell by the product of its
steps' factors; an event arrives exactly at its time; a spike's events
arrive at its interpolated crossing time plus the delay; the epoch length
does not change the run."""
import numpy as np
import pytest

import oracle
from tests import models
from workloads import gen

DT = gen.DT


def test_on_grid_times_reproduce_the_fixed_step():
    """External events at grid times k dt and no network (a spike's events
    arrive at its interpolated time, not on the grid): the variable-step run
    takes exactly the fixed step's steps, of length dt, and gives its
    voltages bit for bit and its spikes (the crossing times interpolated
    from the same voltages, k dt + dt f against (k + f) dt)."""
    n = 4000
    m = gen.config3(cells=[321, 2047, 4095, 7, 11], n_steps=n)
    assert len(m["con_src"]) == 0
    fixed = oracle.Sim(m)
    fixed.run(n)
    var = oracle.Sim(gen.timed(m)).set_varstep()
    var.advance_to(n)
    assert var.grid_point == n and var.varstep_steps == 5 * n
    assert np.array_equal(fixed.state()["V"], var.state()["V"])
    gf, _, tf = fixed.spikes()
    gv, stv, tv = var.spikes()
    of, ov = np.lexsort((tf, gf)), np.lexsort((tv, gv))
    assert len(gf) >= 3 and np.array_equal(gf[of], gv[ov]) and np.all(stv == -1)
    assert np.max(np.abs(tf[of] - tv[ov])) <= 1e-12


def _passive_cell_with_idle_events(times):
    """All-passive tree (uniform V, so no axial current) with a synapse that
    receives zero-weight events at the given times: they only cut steps."""
    d = models.bare_cell(gen.full_binary_parents(2), [4] * 7, np.linspace(100, 250, 7),
                         np.linspace(1, 3, 7), soma_mech=gen.MECH_PAS)
    d.syn.append((2, 1, 2.0, 0.0))
    d.ext = [(0, 0, 0.0) for _ in times]
    m = gen.assemble([d], n_steps=0)
    return gen.timed(m, ev_t=np.asarray(times, np.float64))


def test_uneven_steps_decay_a_passive_cell_exactly():
    """With the explicit membrane current each step of length h multiplies
    V - e by (1 - h/tau) (tau = 1 ms): over the variable step sequence cut at
    off-grid event times, V(T) - e = (V0 - e) prod(1 - h_k/tau)."""
    times = [0.0113, 0.0499, 0.0499, 0.31, 0.3125, 0.375, 1.70001]
    K = 80  # 2 ms
    m = _passive_cell_with_idle_events(times)
    s = oracle.Sim(m).set_varstep(epoch_steps=1000)
    v0 = -40.0
    s.set_voltage(np.full(s.ncv, v0))
    s.advance_to(K)
    # the steps: the grid intervals, each cut at the distinct event times
    # inside it (0.3125 and 0.375 are grid points: no cut)
    hs = []
    for k in range(K):
        a, b = k * DT, (k + 1) * DT
        cuts = sorted({x for x in times if a < x < b})
        pts = [a] + cuts + [b]
        hs += [DT] if not cuts else [pts[j + 1] - pts[j] for j in range(len(pts) - 1)]
    assert s.varstep_steps == len(hs) == K + 5
    ref = gen.PAS_E + (v0 - gen.PAS_E) * np.prod(1.0 - np.array(hs) / 1.0)
    assert np.max(np.abs(s.state()["V"] - ref)) < 1e-12


def test_event_lands_at_its_exact_time():
    """An expsyn event at an off-grid time t0: after it g = w exp(-(t - t0)/tau)
    (the steps between decay by exp(-h/tau)); delivered at the next grid
    point instead, it would be larger by exp(delta/tau)."""
    t0, w, T = 0.3371, 0.02, 3.0
    d = models.bare_cell([-1], [10], [200.0], [2.0], soma_mech=gen.MECH_PAS)
    d.syn.append((0, 4, 2.0, 0.0))
    d.ext = [(0, 0, w)]
    m = gen.timed(gen.assemble([d], n_steps=0), ev_t=[t0])
    s = oracle.Sim(m).set_varstep(epoch_steps=1000)
    s.advance_to(int(round(T / DT)))
    g = s.state()["g"][0]
    ref = 1000.0 * w * np.exp(-(T - t0) / 2.0)
    assert abs(g - ref) <= 1e-12 * ref
    grid = np.ceil(t0 / DT) * DT
    assert abs(1000.0 * w * np.exp(-(T - grid) / 2.0) - ref) > 1e-4 * ref


def test_spike_events_arrive_at_interpolated_time_plus_delay():
    """Cell 0 (hh soma) kicked at an off-grid time fires at its interpolated
    crossing time t_s; cell 1 hears it on a synapse with delay 5.0123 ms, so
    afterwards that synapse's g = w exp(-(t - t_s - d)/tau)."""
    d0 = models.bare_cell([-1], [8], [200.0], [2.0])
    d0.syn.append((-1, 0, 2.0, 0.0))
    d0.ext = [(0, 0, 0.05)]
    d1 = models.bare_cell([-1], [8], [200.0], [2.0])
    d1.syn.append((0, 3, 1.5, 0.0))
    w, delay = 0.001, 5.0123
    d1.in_conn = [(0, 0, 200, w)]
    m = gen.timed(gen.assemble([d0, d1], n_steps=0), con_delay_ms=[delay], ev_t=[0.4567])
    s = oracle.Sim(m).set_varstep()
    T = 12.0
    s.advance_to(int(round(T / DT)))
    gid, _, ts = s.spikes()
    assert list(gid) == [0]
    t_s = ts[0]
    assert 0.4567 < t_s < 5.0 and abs(t_s / DT - round(t_s / DT)) > 1e-3  # off the grid
    g = s.state()["g"][1]
    ref = 1000.0 * w * np.exp(-(T - t_s - delay) / 1.5)
    assert abs(g - ref) <= 1e-12 * ref


def test_epoch_length_invariance():
    """Any epoch no longer than the minimum delay gives the same run, bit for
    bit (epochs end on the grid, and the exchange only decides when spikes
    become events, never when they act)."""
    m = gen.config2_timed(n_cells=6, t_ms=30.0)
    runs = []
    for K in (200, 100, 37, 1):
        s = oracle.Sim(m).set_varstep(epoch_steps=K)
        s.advance_to(1200)
        runs.append((s.state()["V"], s.spikes()))
    assert len(runs[0][1][0]) >= 6
    key = lambda sp: sorted(zip(sp[0].tolist(), sp[2].tolist()))
    for V, sp in runs[1:]:
        assert np.array_equal(V, runs[0][0])
        assert key(sp) == key(runs[0][1])


def test_rejects_clamps_and_long_epochs():
    m = gen.timed(models.single_compartment(amp_uA_cm2=5.0, T_ms=5.0))
    with pytest.raises(ValueError):
        oracle.Sim(m).set_varstep()
    m = gen.config2_timed(n_cells=3, t_ms=10.0)
    with pytest.raises(ValueError):
        oracle.Sim(m).set_varstep(epoch_steps=240)  # 6 ms > the shortest delay
