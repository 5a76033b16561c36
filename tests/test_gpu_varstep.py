"""The variable time step on the GPU (Sec. II: a step is shortened so that
every event falls at the beginning of a step; each cell keeps its own time)
against the oracle's variable step, on the same seeded models: voltages at
several grid points within 1e-8 mV, the same spikes (gid) at the same
interpolated times within 1e-9 ms, and the same number of steps taken."""
import numpy as np
import pytest

import oracle
from tests import models
from workloads import gen

pytestmark = pytest.mark.gpu
TOL = 1e-8    # mV
TTOL = 1e-9   # ms


def _gpu(m, chunks, **kw):
    from paper_1901_07454_amd import arbmi
    sim = arbmi.Simulation(m, **kw)
    assert sim.timed
    Vs, at = [], 0
    for k in chunks:
        sim.step(k - at)
        at = k
        Vs.append(sim.voltages_host())
    sp = sim.spikes()
    n = sim.step_count()
    info = sim.info
    sim.close()
    return Vs, sp, n, info


def _oracle(m, chunks, epoch_steps=None):
    s = oracle.Sim(m).set_varstep(epoch_steps)
    Vs = []
    for k in chunks:
        s.advance_to(k)
        Vs.append(s.state()["V"])
    return Vs, s.spikes(), s.varstep_steps


def _sorted_spikes(g, t):
    g = np.asarray(g).astype(np.int64)
    o = np.lexsort((t, g))
    return g[o], np.asarray(t)[o]


def _compare(m, chunks, **kw):
    Vg, sp, ng, info = _gpu(m, chunks, **kw)
    Vo, (go, so, to), no = _oracle(m, chunks)
    err = max(float(np.max(np.abs(a - b))) for a, b in zip(Vg, Vo))
    assert np.all(sp["step"] == -1) and np.all(so == -1)
    gg, tg = _sorted_spikes(sp["gid"], sp["t_ms"])
    og, ot = _sorted_spikes(go, to)
    terr = float(np.max(np.abs(tg - ot))) if len(tg) and len(tg) == len(ot) else 0.0
    print(f"max|dV| {err:.3e} mV, spikes {len(gg)} (oracle {len(og)}), max|dt_spike| {terr:.3e} ms, "
          f"steps {ng} (oracle {no}), shape T={info['block_threads']} S={info['reg_slots']}", flush=True)
    assert err <= TOL
    assert np.array_equal(gg, og)
    assert terr <= TTOL
    assert ng == no
    return len(gg), ng


def test_on_grid_times_take_the_fixed_steps():
    """External events on the step grid and no network: the variable step
    takes exactly the fixed step's steps (one per grid interval and cell) and
    reproduces the fixed-step kernel's voltages bit for bit (the same code
    runs a step of dt), and the oracle's within tolerance."""
    from paper_1901_07454_amd import arbmi
    ncv = np.array([1 + gen.cell_c3(i, 1.0).n_cv.sum() for i in range(64)])
    cells = [int(c) for c in np.argsort(ncv)[[0, 20, 40, 60]]]
    n = 2000
    m = gen.config3(cells=cells, n_steps=n)
    assert len(m["con_src"]) == 0
    tm = gen.timed(m)
    nsp, ng = _compare(tm, [700, n])
    assert ng == len(cells) * n
    var = arbmi.Simulation(tm)
    var.step(n)
    fixed = arbmi.Simulation(m, coef_mode=3, cells_per_pack=1, block_threads=var.info["block_threads"])
    fixed.step(n)
    assert fixed.info["reg_slots"] == var.info["reg_slots"]
    assert np.array_equal(fixed.voltages_host(), var.voltages_host())
    fixed.close()
    var.close()


@pytest.mark.parametrize("T", [64, 128, 256])
def test_ring_with_off_grid_events_matches_oracle(T):
    """16 cells of the timed ring (delays U(5, 5.5) ms, kicks at U(0, 1) ms,
    Poisson input at continuous times), 1600 steps (40 ms, several epochs
    with launches that end inside an epoch): every cell's voltages at three
    grid points, its spikes and the step count, for each workgroup size
    (two register slots per thread at 64 threads, one above)."""
    m = gen.config2_timed(n_cells=16, t_ms=40.0)
    nsp, ng = _compare(m, [333, 1000, 1600], block_threads=T)
    assert nsp >= 16 and ng > 16 * 1600


@pytest.mark.parametrize("T", [64, 256])
def test_shallow_cells_take_shortened_steps(T):
    """A soma-only cell and a one-branch cell, each alone in its pack, with
    synaptic events at off-grid times: the shortened steps' refactoring and
    the tree passes at their smallest (no tree round for the soma, one for
    the branch), voltages, spikes and step counts against the oracle."""
    cells = [models.bare_cell([], [], [], [], soma_mech=gen.MECH_HH | gen.MECH_PAS),
             models.bare_cell([-1], [5], [150.0], [1.3])]
    for d in cells:
        d.syn.append((-1, 0, 2.0, 0.0))
    m = gen.assemble(cells, n_steps=0)
    times = [[0.0131, 0.5006, 2.71, 2.7125, 9.9], [0.0249, 1.0001, 3.333, 7.5]]
    ws = [[0.06, 0.02, 0.05, 0.05, 0.08], [0.09, 0.01, 0.07, 0.04]]
    m["ev_syn"] = np.array([c for c in range(2) for _ in times[c]], np.uint32)
    m["ev_step"] = np.zeros(len(m["ev_syn"]), np.int64)
    m["ev_w"] = np.array([w for c in range(2) for w in ws[c]], np.float64)
    tm = gen.timed(m, ev_t=np.array([t for c in range(2) for t in times[c]], np.float64))
    nsp, ng = _compare(tm, [150, 500], block_threads=T, cells_per_pack=1)
    assert nsp >= 2 and ng > 2 * 500


def test_uneven_steps_decay_a_passive_cell_exactly():
    """The closed form the oracle is pinned to, on the GPU: zero-weight
    events at off-grid times only cut steps; each step of length h scales
    V - e by (1 - h/tau)."""
    from paper_1901_07454_amd import arbmi
    times = [0.0113, 0.0499, 0.0499, 0.31, 0.3125, 0.375, 1.70001]
    d = models.bare_cell(gen.full_binary_parents(2), [4] * 7, np.linspace(100, 250, 7), np.linspace(1, 3, 7),
                         soma_mech=gen.MECH_PAS)
    d.syn.append((2, 1, 2.0, 0.0))
    d.ext = [(0, 0, 0.0) for _ in times]
    m = gen.timed(gen.assemble([d], n_steps=0), ev_t=np.asarray(times))
    m["v_init"] = -40.0
    K = 80
    sim = arbmi.Simulation(m)
    sim.step(K)
    V = sim.voltages_host()
    steps = sim.step_count()
    sim.close()
    hs = []
    for k in range(K):
        a, b = k * gen.DT, (k + 1) * gen.DT
        cuts = sorted({x for x in times if a < x < b})
        pts = [a] + cuts + [b]
        hs += [gen.DT] if not cuts else [pts[j + 1] - pts[j] for j in range(len(pts) - 1)]
    ref = gen.PAS_E + (-40.0 - gen.PAS_E) * np.prod(1.0 - np.array(hs) / 1.0)
    assert steps == len(hs) == K + 5
    assert np.max(np.abs(V - ref)) < 1e-11


def test_epoch_length_and_graph_replay_do_not_change_the_run():
    """Epochs of K, 100, 37 and 1 grid steps, and whole epochs replayed from a
    captured HIP graph, give the same voltages and spikes bit for bit (the
    exchange only decides when spikes become events, never when they act)."""
    from paper_1901_07454_amd import arbmi
    m = gen.config2_timed(n_cells=6, t_ms=30.0)
    runs = []
    for kw in ({}, {"epoch_steps": 100}, {"epoch_steps": 37}, {"epoch_steps": 1},
               {"flags": arbmi.ARB_FLAG_GRAPH}, {"flags": arbmi.ARB_FLAG_GRAPH, "epoch_steps": 50}):
        Vs, sp, n, _ = _gpu(m, [600, 1200], **kw)
        runs.append((Vs, sp, n))
    Vo, (go, _, to), no = _oracle(m, [600, 1200])
    assert np.max(np.abs(runs[0][0][1] - Vo[1])) <= TOL
    assert len(runs[0][1]) >= 6
    for Vs, sp, n in runs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(Vs, runs[0][0]))
        assert np.array_equal(np.sort(sp, order=["t_ms", "gid"]), np.sort(runs[0][1], order=["t_ms", "gid"]))
        assert n == runs[0][2] == no


def test_full_size_timed_ring_sampled_cells():
    """The timed ring at full size (8192 cells, 4000 steps, 100 ms) in the
    benchmark's launch configuration (whole epochs replayed from a graph):
    sampled cells against the oracle on their light cones (every ring delay
    is at least 5 ms = 200 steps, so within 4000 steps only the 20 ring
    predecessors can reach a cell)."""
    from paper_1901_07454_amd import arbmi
    n = 4000
    m = gen.config2_timed(t_ms=n * gen.DT)
    cv0 = oracle.cell_cv_begin(m)
    sim = arbmi.Simulation(m, flags=arbmi.ARB_FLAG_GRAPH)
    sim.step(n)
    V = sim.voltages_host()
    sp = sim.spikes()
    steps = sim.step_count()
    info = sim.info
    sim.close()
    del m
    print("timed ring info", info, "spikes", len(sp), "steps", steps, flush=True)
    assert steps > 8192 * n
    for c in (0, 4097, 8191):
        chain = gen.ring_light_cone(8192, c, n)
        sub = gen.config2_timed(cells=chain, t_ms=n * gen.DT)
        s = oracle.Sim(sub).set_varstep()
        s.advance_to(n)
        c0 = oracle.cell_cv_begin(sub)
        err = float(np.max(np.abs(V[cv0[c]:cv0[c + 1]] - s.state()["V"][c0[-2]:c0[-1]])))
        g, _, t = s.spikes()
        mine = np.sort(sp["t_ms"][sp["gid"] == c])
        ref = np.sort(t[g == len(chain) - 1])
        print(f"cell {c}: max|dV| = {err:.3e}, spikes {len(mine)}", flush=True)
        assert err <= TOL
        assert len(mine) == len(ref) and (len(ref) == 0 or np.max(np.abs(mine - ref)) <= TTOL)
