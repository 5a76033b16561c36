"""Full-size parity in the benchmark's launch configuration, on sampled
outputs the CPU oracle can compute one cell (or one light cone) at a time."""
import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu
TOL = 1e-8


def _gpu(m, n, probes, **kw):
    from paper_1901_07454_amd import arbmi
    sim = arbmi.Simulation(m, **kw)
    sim.set_probes(probes, n)
    sim.step(n)
    tr = sim.trace(n)
    V = sim.voltages_host()
    sp = sim.spikes()
    info = sim.info
    sim.close()
    return tr, V, sp, info


def test_config3_full_size_sampled_cells():
    """4096 uneven cells, 8000 steps (200 ms); no network, so every cell is
    independent and each sampled cell runs alone in the oracle."""
    from paper_1901_07454_amd import arbmi
    m = gen.config3()
    cv0 = oracle.cell_cv_begin(m)
    ncv = np.diff(cv0)
    samples = sorted({0, 1, 2047, 4095, int(np.argmax(ncv)), int(np.argmin(ncv))})
    tr, V, sp, info = _gpu(m, 8000, cv0[samples], flags=arbmi.ARB_FLAG_AUTOTUNE)
    print("config 3 info", info, flush=True)
    for k, c in enumerate(samples):
        sub = gen.config3(cells=[c])
        s = oracle.Sim(sub)
        rtr = s.run(8000, probes=[0])[0]
        err = max(np.max(np.abs(tr[k] - rtr)), np.max(np.abs(V[cv0[c]:cv0[c + 1]] - s.state()["V"])))
        g, st, _ = s.spikes()
        mine = sorted(int(x) for x in sp["step"][sp["gid"] == c])
        print(f"cell {c} ({ncv[c]} CVs): max|dV| = {err:.3e}, spikes {len(mine)}", flush=True)
        assert err <= TOL
        assert mine == sorted(int(x) for x in st)


def test_config3_register_layout_largest_and_smallest_cells():
    """The register layout at 256 threads x 3 slots on the uneven workload's
    four largest cells (their packs read hh conductances from HBM) and four
    small ones, 2000 steps, each cell against the oracle."""
    from paper_1901_07454_amd import arbmi
    ncv = np.array([1 + gen.cell_c3(i, 1.0).n_cv.sum() for i in range(4096)])
    order = np.argsort(-ncv)
    cells = sorted([int(c) for c in order[:4]] + [int(c) for c in order[-2:]] + [0, 2047])
    n = 2000
    m = gen.config3(cells=cells, n_steps=n)
    cv0 = oracle.cell_cv_begin(m)
    tr, V, sp, info = _gpu(m, n, cv0[:-1], block_threads=256, coef_mode=3)
    print("info", info, flush=True)
    assert info["coef_mode"] == 3 and info["syn_hbm"] == 1
    for k, c in enumerate(cells):
        s = oracle.Sim(gen.config3(cells=[c], n_steps=n))
        rtr = s.run(n, probes=[0])[0]
        err = max(np.max(np.abs(tr[k] - rtr)), np.max(np.abs(V[cv0[k]:cv0[k + 1]] - s.state()["V"])))
        g, st, _ = s.spikes()
        mine = sorted(int(x) for x in sp["step"][sp["gid"] == k])
        print(f"cell {c} ({ncv[c]} CVs): max|dV| = {err:.3e}, spikes {len(mine)}", flush=True)
        assert err <= TOL
        assert mine == sorted(int(x) for x in st)


def _c5_cell_alone(args):
    """Oracle run of cell i of the 65536-cell network alone for n steps, its
    network input replaced by the events its sources' given spikes deliver
    before step n (each connection has its own synapse, so the conductance
    sums are the network run's); returns (spike steps, soma trace, final V)."""
    i, n, spikes, want = args
    import numpy as np

    import oracle
    from workloads import gen
    d = gen.cell_c5(i, 65536, t_ms=20.0)
    d.ext = [e for e in d.ext if e[1] < n]
    for (src, ls, delay, w) in d.in_conn:
        for t in spikes.get(int(src), ()):
            if t + delay < n:
                d.ext.append((ls, int(t + delay), w))
    d.in_conn = []
    s = oracle.Sim(gen.assemble([d], gids=[i], n_steps=n))
    tr = s.run(n, probes=[0])[0] if want else (s.run(n), None)[1]
    _, st, _ = s.spikes()
    return [int(x) for x in st], tr, (s.state()["V"] if want else None)


def _c5_light_cone(m, c, n, pool):
    """Cell c of the 65536-cell network over n = 800 steps, exactly, from
    oracle runs of single cells: with delays of at least 200 steps, c's
    dynamics to step 800 depend on its sources' spikes before 600, theirs on
    their sources' spikes before 400, and those on spikes before 200, which
    come from background input alone (no network event arrives before step
    200).  A cell without any input event before its horizon cannot spike
    and is not run."""
    src_of = {}
    order = np.argsort(m["con_dst"], kind="stable")
    bounds = np.searchsorted(m["con_dst"][order], np.arange(len(m["cell_n_branch"]) + 1))

    def sources(j):
        if j not in src_of:
            src_of[j] = [int(x) for x in m["con_src"][order[bounds[j]:bounds[j + 1]]]]
        return src_of[j]

    ev_cell = m["syn_cell"][m["ev_syn"]]
    first_bg = np.full(len(m["cell_n_branch"]), np.iinfo(np.int64).max)
    np.minimum.at(first_bg, ev_cell, m["ev_step"])
    s1 = sorted(set(sources(c)))
    s2 = sorted({x for j in s1 for x in sources(j)})
    s3 = sorted({x for j in s2 for x in sources(j)})
    spikes = {}
    # level 3: spikes before step 200 (background only)
    run3 = [j for j in s3 if first_bg[j] < 200]
    for j, (st, _, _) in zip(run3, pool.map(_c5_cell_alone, [(j, 200, {}, False) for j in run3])):
        spikes[j] = st
    # level 2 (to step 400), level 1 (to step 600)
    for level, horizon in ((s2, 400), (s1, 600)):
        prev = dict(spikes)
        run = [j for j in level if first_bg[j] < horizon or any(
            t + 200 <= horizon for x in sources(j) for t in prev.get(x, ()))]
        res = pool.map(_c5_cell_alone, [(j, horizon, {x: prev[x] for x in sources(j) if x in prev}, False)
                                        for j in run])
        spikes = dict(prev)
        for j, (st, _, _) in zip(run, res):
            spikes[j] = st
    print(f"cell {c}: light cone {len(s1)} / {len(s2)} / {len(s3)} cells, "
          f"{sum(len(v) for v in spikes.values())} spikes", flush=True)
    return _c5_cell_alone((c, n, {x: spikes[x] for x in sources(c) if x in spikes}, True))


@pytest.fixture(scope="module")
def _c5_oracle():
    """The network, its sampled cells and the oracle's results for them
    through their light cones (_c5_light_cone), computed once."""
    import multiprocessing as mp
    import os
    n = 800
    m = gen.config5(n_steps=n)
    cv0 = oracle.cell_cv_begin(m)
    samples = [0, 65535]
    with mp.get_context("spawn").Pool(max(1, min(16, os.cpu_count() or 1))) as pool:
        ref = [_c5_light_cone(m, c, n, pool) for c in samples]
    return m, cv0, samples, ref


@pytest.mark.parametrize("T,S", [(128, 2), (64, 3)])
def test_config5_full_size_light_cone(_c5_oracle, T, S):
    """65536 cells x 1497 CVs, 800 steps (20 ms), in the two launch shapes
    the benchmark's autotuner chooses between for this network
    (reg_step_kernel<128, 2, 8> and <64, 3, 8>, one cell per workgroup):
    sampled cells against the oracle through their light cones."""
    m, cv0, samples, ref = _c5_oracle
    tr, V, sp, info = _gpu(m, 800, cv0[samples], block_threads=T, coef_mode=3, cells_per_pack=1)
    print("config 5 info", info, "spikes", len(sp), flush=True)
    assert (info["block_threads"], info["coef_mode"], info["reg_slots"], info["reg_len"]) == (T, 3, S, 8)
    assert info["n_packs"] == 65536
    for k, c in enumerate(samples):
        st, rtr, rV = ref[k]
        err = max(np.max(np.abs(tr[k] - rtr)), np.max(np.abs(V[cv0[c]:cv0[c + 1]] - rV)))
        mine = sorted(int(x) for x in sp["step"][sp["gid"] == c])
        print(f"cell {c}: max|dV| = {err:.3e}, spikes {mine}", flush=True)
        assert err <= TOL
        assert mine == sorted(st)


def test_config4_full_size_adjoint_sampled_cells():
    """256 cells x 200 CVs, 2000 steps, checkpoints every 100: gradients of
    the trace MSE for sampled cells against the oracle's discrete adjoint."""
    import torch

    from paper_1901_07454_amd import grad
    n = 2000
    m0 = gen.config4(n_steps=n)
    mh = gen.config4(hidden=True, n_steps=n)
    th0 = gen.config4_theta(m0)
    gs = grad.GradSim(m0)
    # target traces from the hidden parameters, computed on the GPU forward
    # and checked against the oracle for the sampled cells below
    sim_t = grad.GradSim(mh)
    tgt = grad.soma_trace(torch.tensor(gen.config4_theta(mh), device="cuda"), sim_t, n, 100).detach()
    sim_t.close()
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    tr = grad.soma_trace(theta, gs, n, 100)
    loss = torch.mean((tr - tgt) ** 2)
    loss.backward()
    g = theta.grad.cpu().numpy()
    tr = tr.detach().cpu().numpy()
    tgt = tgt.cpu().numpy()
    C = tr.shape[0]
    for c in (0, 77, 255):
        ref_t = oracle.Sim(gen.config4(cells=[c], hidden=True, n_steps=n)).run(n, probes=[0])[0]
        assert np.max(np.abs(tgt[c] - ref_t)) <= TOL
        s = oracle.Sim(gen.config4(cells=[c], n_steps=n))
        dl = (2.0 * (tr[c] - tgt[c]) / (C * n))[None, :]
        otr, og = s.adjoint(n, dl)
        assert np.max(np.abs(otr[0] - tr[c])) <= TOL
        rel = np.abs(g[c] - og) / np.maximum(np.abs(og), 1e-3 * np.abs(og).max())
        print(f"cell {c}: max rel grad err {rel.max():.3e}", flush=True)
        assert rel.max() <= 1e-7
    gs.close()


def test_config6_full_size_light_cone():
    """The synapse-dominated ring at full size (8192 cells x ~130 CVs x 10,000
    expsyn, 82M synapses), 400 steps, autotuned shape: a sampled cell's inputs
    within 400 steps come from its own kick and its ring predecessor."""
    from paper_1901_07454_amd import arbmi
    n = 400
    m = gen.config6(n_steps=n)
    cv0 = oracle.cell_cv_begin(m)
    samples = [0, 4097, 8191]
    tr, V, sp, info = _gpu(m, n, cv0[samples], flags=arbmi.ARB_FLAG_AUTOTUNE)
    print("config 6 info", info, "spikes", len(sp), flush=True)
    del m
    for k, c in enumerate(samples):
        chain = gen.ring_light_cone(8192, c, n)
        sub = gen.config6(n_cells=8192, cells=chain, n_steps=n)
        s = oracle.Sim(sub)
        c0 = oracle.cell_cv_begin(sub)
        rtr = s.run(n, probes=[c0[-2]])[0]
        err = max(np.max(np.abs(tr[k] - rtr)), np.max(np.abs(V[cv0[c]:cv0[c + 1]] - s.state()["V"][c0[-2]:c0[-1]])))
        g, st, _ = s.spikes()
        mine = sorted(int(x) for x in sp["step"][sp["gid"] == c])
        print(f"cell {c}: max|dV| = {err:.3e}", flush=True)
        assert err <= TOL
        assert mine == sorted(int(x) for x, gg in zip(st, g) if gg == len(chain) - 1)


def _c7_reduced_source(s: int) -> gen.CellDesc:
    """Source cell s of the 10k-connectivity model without its network input
    and without the synapses that only network input reaches: before the
    first volley arrives (step 800) its voltages, hence its first spike, are
    those of the full cell (idle synapses add exactly zero current)."""
    d = gen.cell_c7(s, 8192, n_steps=900)
    d.syn_arr = tuple(np.asarray(x)[:1] for x in d.syn_arr)
    d.in_conn_arr = None
    return d


def test_config7_full_size_first_volley():
    """The 10k-connectivity model at full size (8192 cells x ~130 CVs,
    82M synapses and connections, delay 800 steps, 50 Hz drive), 900 steps,
    autotuned shape: a sampled cell receives the first volley (its ~5,900
    distinct sources' spikes after the drive at step 0) at steps 811-825,
    while it fires after the second drive; the oracle runs it with every
    source reduced as above."""
    from paper_1901_07454_amd import arbmi
    n = 900
    m = gen.config7(n_steps=n)
    cv0 = oracle.cell_cv_begin(m)
    samples = [0, 5003, 8191]
    tr, V, sp, info = _gpu(m, n, cv0[samples], flags=arbmi.ARB_FLAG_AUTOTUNE)
    print("config 7 info", info, "spikes", len(sp), flush=True)
    del m
    assert len(sp) == 2 * 8192  # every cell fires once per drive
    for k, c in enumerate(samples):
        tgt = gen.cell_c7(c, 8192, n_steps=n)
        srcs = sorted(set(int(x) for x in tgt.in_conn_arr[0]))
        sub = gen.assemble([tgt] + [_c7_reduced_source(x) for x in srcs], gids=[c] + srcs, n_steps=n)
        assert len(sub["con_src"]) == 10000
        s = oracle.Sim(sub)
        c0 = oracle.cell_cv_begin(sub)
        rtr = s.run(n, probes=[0])[0]
        err = max(np.max(np.abs(tr[k] - rtr)), np.max(np.abs(V[cv0[c]:cv0[c + 1]] - s.state()["V"][:c0[1]])))
        g, st, _ = s.spikes()
        mine = sorted(int(x) for x in sp["step"][sp["gid"] == c])
        print(f"cell {c}: {len(srcs)} sources, max|dV| = {err:.3e}, spikes {mine}", flush=True)
        assert err <= TOL
        assert mine == sorted(int(x) for x in st[g == 0])


def _region0(m, c):
    """Index of cell c's first region (its soma) in the flat region order."""
    return int(c + np.sum(m["cell_n_branch"][:c]))


def test_config5_subset_forward_adjoint():
    """Forward + adjoint of the 1024-cell subset of the 65536-cell network
    (1497 CVs per cell, network input as fixed seeded events, background
    kept), 800 steps (20 ms), checkpoints every 100, in the benchmark's launch
    shape for this network (128 threads, register layout, one cell per
    workgroup).  Loss: mean squared distance of every soma trace from -65 mV.
    Sampled cells' gradients against the oracle's discrete adjoint, and
    central finite differences of the GPU forward on a few parameters."""
    import torch

    from paper_1901_07454_amd import arbmi
    from tests.test_gpu_adjoint import model_theta
    n, k = 800, 100
    m = gen.config5_subset(n_steps=n)
    th = model_theta(m)
    sim = arbmi.Simulation(m, flags=arbmi.ARB_FLAG_GRADIENTS, block_threads=128, coef_mode=3, cells_per_pack=1)
    info = sim.info
    print("config 5 subset gradient sim", info, flush=True)
    assert (info["block_threads"], info["coef_mode"], info["reg_slots"], info["reg_len"]) == (128, 3, 2, 8)
    assert info["n_packs"] == 1024
    state0 = sim.get_state()
    C = info["n_cells"]

    def forward(theta):
        sim.set_state(state0)
        sim.set_params(theta)
        tr = torch.empty(C, n, dtype=torch.float64, device="cuda")
        arbmi.arb_grad_forward(sim.h, n, k, tr)
        return tr

    tr = forward(th)
    dl = 2.0 * (tr + 65.0) / tr.numel()
    out = torch.empty(th.size, dtype=torch.float64, device="cuda")
    arbmi.arb_grad_backward(sim.h, dl.contiguous(), out)
    g = out.cpu().numpy().reshape(-1, 3)
    trh, dlh = tr.cpu().numpy(), dl.cpu().numpy()
    for c in (0, 511, 1023):
        sub = gen.config5_subset(cells=[c], n_steps=n)
        r0, r1 = _region0(m, c), _region0(m, c + 1)
        s = oracle.Sim(sub)
        s.set_params(th[r0:r1])
        otr, og = s.adjoint(n, dlh[c][None, :])
        err = np.max(np.abs(otr[0] - trh[c]))
        den = np.maximum(np.abs(og), 1e-3 * np.max(np.abs(og), axis=0, keepdims=True))
        rel = np.abs(g[r0:r1] - og) / den
        print(f"cell {c}: max|dV| = {err:.3e}, max rel grad err {rel.max():.3e}", flush=True)
        assert err <= TOL
        assert rel.max() <= 1e-7
    # central differences (relative step 1e-5) of the loss; a parameter of
    # cell c moves only cell c's terms, so only those are summed (the other
    # cells' terms would add nothing but rounding)
    h = 1e-5
    for (c, r, q) in ((0, 0, 0), (0, 0, 1), (0, 40, 2), (511, 1, 2)):
        j = _region0(m, c) + r
        vals = []
        for sgn in (1, -1):
            t = th.copy()
            t[j, q] *= 1 + sgn * h
            trp = forward(t)[c].cpu().numpy()
            vals.append(float(np.sum((trp + 65.0) ** 2)) / (C * n))
        fd = (vals[0] - vals[1]) / (2 * h * th[j, q])
        rel = abs(g[j, q] - fd) / max(abs(fd), 1e-30)
        print(f"FD cell {c} region {r} param {q}: adjoint {g[j, q]:.6e} fd {fd:.6e} rel {rel:.2e}", flush=True)
        assert rel <= 1e-5
    sim.close()
