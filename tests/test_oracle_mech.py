"""Pins for the mechanisms (hh, expsyn) and the operator-split state update:
textbook HH values, HH repetitive firing, convergence to an independent ODE
integration, and the exact exponential synapse decay."""
import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from tests import models
from workloads import gen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hh_textbook.json")))


def test_hh_resting_gates_textbook():
    r = oracle.hh_rates(GOLD["v_rest_mV"])
    tol = GOLD["abs_tol_gates"]
    assert abs(r[0] / (r[0] + r[1]) - GOLD["m_inf_rest"]) < tol
    assert abs(r[2] / (r[2] + r[3]) - GOLD["h_inf_rest"]) < tol
    assert abs(r[4] / (r[4] + r[5]) - GOLD["n_inf_rest"]) < tol


def test_hh_rates_removable_singularities():
    assert oracle.hh_rates(-40.0)[0] == pytest.approx(GOLD["alpha_m_at_minus40"], rel=1e-14)
    assert oracle.hh_rates(-55.0)[4] == pytest.approx(GOLD["alpha_n_at_minus55"], rel=1e-14)
    # continuity across the singular points
    for v0, k in ((-40.0, 0), (-55.0, 4)):
        a = oracle.hh_rates(v0 - 1e-7)[k]
        b = oracle.hh_rates(v0 + 1e-7)[k]
        assert abs(a - b) < 1e-7


def test_hh_rate_derivatives_match_differences():
    def fd(v, h=1e-3):  # fourth-order central stencil
        f = oracle.hh_rates
        return (-f(v + 2 * h) + 8 * f(v + h) - 8 * f(v - h) + f(v - 2 * h)) / (12 * h)
    for v in list(np.linspace(-90, 40, 27) + 0.123) + [-40.0, -55.0, -40.0 + 3e-4, -55.0 - 2e-4]:
        assert np.allclose(oracle.hh_rates_dv(v), fd(v), rtol=1e-8, atol=1e-12)


def _spikes_single(amp, T=300.0):
    m = models.single_compartment(amp_uA_cm2=amp, T_ms=T)
    s = oracle.Sim(m)
    tr = s.run(m["n_steps"], probes=[0])
    return s.spikes()[2], tr[0]


def test_hh_repetitive_firing_rate_textbook():
    rf = GOLD["repetitive_firing"]
    t, v = _spikes_single(rf["current_uA_per_cm2"])
    assert len(t) >= 10
    rate = 1000.0 / np.mean(np.diff(t[-5:]))
    lo, hi = rf["rate_hz_range"]
    assert lo < rate < hi
    plo, phi = GOLD["spike_peak_mV_range"]
    assert plo < v.max() < phi


def test_hh_single_spike_below_repetitive_threshold():
    t, _ = _spikes_single(GOLD["single_spike_only_current_uA_per_cm2"])
    assert len(t) == 1


def _hh_rhs(t, y, I_uA_cm2):
    """Textbook HH membrane (per unit area): C dV/dt = I - I_ion."""
    V, m, h, n = y
    x = -(V + 40) / 10
    am = x / np.expm1(x) if abs(x) > 1e-12 else 1.0
    bm = 4 * np.exp(-(V + 65) / 18)
    ah = 0.07 * np.exp(-(V + 65) / 20)
    bh = 1 / (1 + np.exp(-(V + 35) / 10))
    x = -(V + 55) / 10
    an = 0.1 * (x / np.expm1(x) if abs(x) > 1e-12 else 1.0)
    bn = 0.125 * np.exp(-(V + 65) / 80)
    Iion = 120 * m ** 3 * h * (V - 50) + 36 * n ** 4 * (V + 77) + 0.3 * (V + 54.3)  # uA/cm^2 with mS/cm^2
    return [(I_uA_cm2 - Iion) / 1.0, am * (1 - m) - bm * m, ah * (1 - h) - bh * h, an * (1 - n) - bn * n]


def test_single_compartment_first_order_convergence():
    """Operator splitting + implicit Euler + exponential gate update is first
    order in dt: errors against a tight Radau solution halve with dt."""
    T, I = 10.0, 10.0
    r = oracle.hh_rates(-65.0)
    y0 = [-65.0, r[0] / (r[0] + r[1]), r[2] / (r[2] + r[3]), r[4] / (r[4] + r[5])]
    errs, tsp = [], []
    for dt in (0.025, 0.0125, 0.00625):
        m = models.single_compartment(amp_uA_cm2=I, T_ms=T, dt=dt)
        s = oracle.Sim(m)
        tr = s.run(m["n_steps"], probes=[0])[0]
        t = dt * np.arange(1, m["n_steps"] + 1)
        sol = solve_ivp(_hh_rhs, (0, T), y0, method="Radau", rtol=1e-11, atol=1e-11,
                        t_eval=t, args=(I,))
        errs.append(np.max(np.abs(tr - sol.y[0])))
        tsp.append(s.spikes()[2][0])
    assert errs[0] < 10.0  # mV, the largest error sits on the spike upstroke
    assert 1.8 < errs[0] / errs[1] < 2.2
    assert 1.8 < errs[1] / errs[2] < 2.2
    # spike time converges at first order too (differences halve)
    d1, d2 = tsp[1] - tsp[0], tsp[2] - tsp[1]
    assert d1 > 0 and 1.6 < d1 / d2 < 2.4


def test_expsyn_exact_exponential_decay():
    """A single event of weight w at step s0: g(t) = 1000 w exp(-(t - t0)/tau)."""
    d = models.bare_cell([-1], [4], [150.0], [2.0])
    d.syn.append((0, 2, 3.0, 0.0))
    d.ext.append((0, 5, 0.002))
    m = gen.assemble([d], n_steps=400)
    s = oracle.Sim(m)
    s.run(5)
    assert s.state()["g"][0] == 0.0
    for n in range(1, 300):
        s.run(1)
        ref = 1000 * 0.002 * np.exp(-n * gen.DT / 3.0)
        assert abs(s.state()["g"][0] - ref) <= 1e-13 * 2.0 + 1e-12 * ref
