"""Pins for discretisation, assembly and units (eq. 2a, implicit-Euler system):
exact passive decay, the sealed-end cable closed form, charge conservation."""
import numpy as np

import oracle
from tests import models
from workloads import gen


def test_uniform_passive_decay_exact():
    """All-passive tree with uniform V: the Laplacian vanishes, so with the
    explicit membrane current V^n - e = (V^0 - e)(1 - dt/tau)^n, tau = cm/g
    (1 uF/cm^2 / 0.001 S/cm^2 = 1 ms)."""
    d = models.bare_cell(gen.full_binary_parents(2), [5] * 7, np.linspace(100, 250, 7),
                         np.linspace(1, 3, 7), soma_mech=gen.MECH_PAS)
    m = gen.assemble([d], n_steps=200)
    s = oracle.Sim(m)
    v0 = -40.0
    s.set_voltage(np.full(s.ncv, v0))
    tr = s.run(200, probes=[0, 3, s.ncv - 1])
    n = np.arange(1, 201)
    ref = gen.PAS_E + (v0 - gen.PAS_E) * (1 - gen.DT / 1.0) ** n
    assert np.max(np.abs(tr - ref[None, :])) < 1e-11


def _cable_error(n_cv):
    m = models.sealed_cable(n_cv)
    s = oracle.Sim(m)
    s.run(m["n_steps"])
    V = s.state()["V"]
    L, dm, Ra, g, I = 1000.0, 2.0, 100.0, 1e-3, 0.1e-9
    lam = np.sqrt(dm * 1e-4 / (4 * Ra * g))          # cm
    ra = 4 * Ra / (np.pi * (dm * 1e-4) ** 2)         # ohm / cm
    h = L / n_cv
    x = np.concatenate([[0.0], h * np.arange(1, n_cv + 1)]) * 1e-4  # cm
    Lc = L * 1e-4
    ref = 1e3 * I * ra * lam * np.cosh((Lc - x) / lam) / np.sinh(Lc / lam)  # mV
    return np.max(np.abs((V - gen.PAS_E) - ref)) / ref[0], (V[0] - gen.PAS_E), ref[0]


def test_sealed_end_cable_closed_form_second_order():
    """Steady state of a sealed-end cable driven at x=0 converges to
    V(x) - e = I r_a lambda cosh((L-x)/lambda)/sinh(L/lambda) at O(h^2)."""
    e1, v1, r1 = _cable_error(50)
    e2, v2, r2 = _cable_error(100)
    assert e2 < 2e-3
    assert 3.0 < e1 / e2 < 5.0
    assert v1 > 0 and abs(r1 - 7.12) < 0.05  # ~71 MOhm input resistance x 0.1 nA


def test_charge_conservation_random_tree():
    """sum_i c_i V_i^{n+1} = sum_i c_i V_i^n - dt sum_i I_i: the axial terms
    cancel pairwise for any tree."""
    m = gen.config3(n_cells=3)
    m["ev_step"] = m["ev_step"] + 10_000  # no events in the tested steps
    s = oracle.Sim(m)
    info = s.cv_info()
    rng = np.random.default_rng(0)
    for k in range(3):
        s.set_voltage(rng.uniform(-80, 20, s.ncv))
        V0 = s.state()["V"]
        I = s.membrane_current()
        s.run(1)
        V1 = s.state()["V"]
        for c in range(3):
            cb = oracle.cell_cv_begin(m)
            sl = slice(cb[c], cb[c + 1])
            lhs = np.sum(info["cap"][sl] * V1[sl])
            rhs = np.sum(info["cap"][sl] * V0[sl]) - gen.DT * np.sum(I[sl])
            assert abs(lhs - rhs) <= 1e-12 * np.sum(info["cap"][sl] * np.abs(V0[sl]))


def test_cv_counts_and_areas():
    """CV count = 1 + sum n_cv; total membrane area = soma + lateral areas."""
    m = gen.config1()
    s = oracle.Sim(m)
    assert s.ncv == 129
    info = s.cv_info()
    lat = np.sum(np.pi * m["br_diam"] * m["br_length"])
    assert abs(info["area"].sum() - (500.0 + lat)) < 1e-9 * lat
