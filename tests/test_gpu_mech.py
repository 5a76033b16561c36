"""Generated density mechanisms on the GPU (the description language's
mechanisms compiled into the register-resident kernel) against the oracle's
hand-written ones: voltages within 1e-8 mV, identical spike steps; and the
generated Hodgkin-Huxley mechanism reproducing the hand-written built-in
one."""
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


@pytest.mark.parametrize("kw", [{}, {"block_threads": 128}, {"cells_per_pack": 4}, {"flags": 4}])
def test_ring_with_generated_mechanisms_matches_oracle(kw):
    """8 ring cells with hcn on the soma, kdr on every dendritic branch and
    hh_dsl on branch 0, kicked every 10 ms, 2000 steps: soma traces, final
    voltages and spike steps, in several launch shapes (one cell per
    workgroup and four, graph replay)."""
    n = 2000
    m = gen.config2_mech(n_cells=8, n_steps=n)
    cv0 = oracle.cell_cv_begin(m)
    tr, V, sp, info = _gpu(m, n, cv0[:-1], **kw)
    s = oracle.Sim(m)
    rtr = s.run(n, probes=cv0[:-1])
    err = max(np.max(np.abs(tr - rtr)), np.max(np.abs(V - s.state()["V"])))
    g, st, _ = s.spikes()
    print(f"{kw}: max|dV| {err:.3e} mV, spikes {len(sp)} (oracle {len(g)}), shape {info['block_threads']}",
          flush=True)
    assert info["coef_mode"] == 3
    assert err <= TOL
    assert sorted(zip(sp["step"].tolist(), sp["gid"].tolist())) == sorted(zip(st.tolist(), g.tolist()))
    assert len(g) >= 8


def test_generated_hh_reproduces_the_built_in_hh():
    """Two ring cells: built-in hh on the soma, and the same densities as the
    generated hh_dsl mechanism on a soma without built-in mechanisms.  The
    two runs agree to rounding (the generated current adds the leak
    explicitly, the built-in one folds it into the step coefficients)."""
    n = 2000
    m = gen.config2_mech(n_cells=2, n_steps=n)
    m["densities"] = []
    twin = dict(m)
    for k in ("soma_mech",):
        twin[k] = np.asarray(m[k]).copy()
    twin["soma_mech"] = twin["soma_mech"] & ~np.uint32(gen.MECH_HH)
    twin = gen.with_densities(twin, [(c, -1, "hh_dsl", {"gnabar": float(m["soma_gna"][c]),
                                                       "gkbar": float(m["soma_gk"][c]),
                                                       "gl": float(m["soma_gl"][c])}) for c in range(2)])
    cv0 = oracle.cell_cv_begin(m)
    tr_a, V_a, sp_a, _ = _gpu(m, n, cv0[:-1], coef_mode=3)
    tr_b, V_b, sp_b, _ = _gpu(twin, n, cv0[:-1])
    err = max(np.max(np.abs(tr_a - tr_b)), np.max(np.abs(V_a - V_b)))
    print(f"built-in vs generated hh: max|dV| {err:.3e} mV, spikes {len(sp_a)}", flush=True)
    assert err <= 1e-9
    assert sp_a["step"].tolist() == sp_b["step"].tolist() and len(sp_a) >= 2


def _uneven_with_mechanisms(n):
    """Fourteen Yule-tree cells of the uneven workload (56-548 CVs, hh on a
    quarter of the branches, 10 Hz Poisson input), with hcn on every soma
    and kdr on every other branch, each instance with its own parameters
    drawn from a seeded generator."""
    cells = [3, 4, 5, 8, 11, 15, 20, 23, 33, 34, 35, 38, 0, 12]
    m = gen.config3(cells=cells, n_steps=n)
    rng = np.random.default_rng(1901)
    dens = []
    for c in range(len(cells)):
        dens.append((c, -1, "hcn", {"gbar": float(rng.uniform(1e-4, 5e-4)), "vhalf": float(rng.uniform(-80, -65))}))
        for b in range(0, int(m["cell_n_branch"][c]), 2):
            dens.append((c, b, "kdr", {"gbar": float(rng.uniform(1e-3, 4e-3))}))
    return gen.with_densities(m, dens)


@pytest.mark.parametrize("T", [64, 128, 256])
def test_generated_mechanisms_on_uneven_trees_match_oracle(T):
    """Generated mechanisms in packs of several irregular trees (the
    general tree rounds, not the binary ones), with per-instance
    parameters: 1600 steps, soma traces, final voltages and spike steps
    against the oracle."""
    n = 1600
    m = _uneven_with_mechanisms(n)
    cv0 = oracle.cell_cv_begin(m)
    tr, V, sp, info = _gpu(m, n, cv0[:-1], block_threads=T, coef_mode=3)
    s = oracle.Sim(m)
    assert s.ngen > 1000
    rtr = s.run(n, probes=cv0[:-1])
    err = max(np.max(np.abs(tr - rtr)), np.max(np.abs(V - s.state()["V"])))
    g, st, _ = s.spikes()
    print(f"T={T}: max|dV| {err:.3e} mV, spikes {len(sp)} (oracle {len(g)}), packs {info['n_packs']}", flush=True)
    assert info["coef_mode"] == 3 and info["n_packs"] < len(cv0) - 1
    assert err <= TOL
    assert sorted(zip(sp["step"].tolist(), sp["gid"].tolist())) == sorted(zip(st.tolist(), g.tolist()))
    assert len(g) >= 5


def test_instance_counts():
    """arb_get_mechanism_instances on three ring cells: one instance per CV
    and density entry whose region the CV covers, a branch's region being
    covered by its 8 CVs and by its parent's node CV, which holds its first
    half-segment: hcn (soma) 1 per cell, hh_dsl (branch 0) 9, kdr (127
    branches) 1143; the total is the oracle's."""
    from paper_1901_07454_amd import arbmi
    m = gen.config2_mech(n_cells=3, n_steps=10)
    sim = arbmi.Simulation(m)
    counts = sim.mechanism_instances()
    sim.close()
    assert counts == {"hcn": 3, "hh_dsl": 3 * 9, "kdr": 3 * 127 * 9}
    assert sum(counts.values()) == oracle.Sim(m).ngen
