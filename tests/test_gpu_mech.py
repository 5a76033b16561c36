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
