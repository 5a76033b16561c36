"""Small hand-built models for the pin and parity tests (descriptions only)."""
import numpy as np

from workloads import gen


def bare_cell(parents, n_cv, length, diam, soma_mech=gen.MECH_HH, dend_mech=gen.MECH_PAS):
    d = gen.CellDesc()
    d.parents = np.asarray(parents, np.int32)
    nb = len(d.parents)
    d.n_cv = np.asarray(n_cv, np.int32).reshape(nb)
    d.length = np.asarray(length, float).reshape(nb)
    d.diam = np.asarray(diam, float).reshape(nb)
    gen._dend_pas(d)
    d.mech[:] = dend_mech
    if soma_mech & gen.MECH_HH:
        gen._soma_hh(d)
        d.soma_mech = soma_mech
        if soma_mech & gen.MECH_PAS:
            d.soma_g = (gen.HH_DEF[0], gen.HH_DEF[1], gen.HH_DEF[2], gen.PAS_G, gen.PAS_E)
    else:
        d.soma_mech = soma_mech
        d.soma_g = (0.0, 0.0, 0.0, gen.PAS_G if soma_mech & gen.MECH_PAS else 0.0, gen.PAS_E)
    return d


def single_compartment(area=1000.0, amp_uA_cm2=0.0, T_ms=100.0, dt=gen.DT):
    d = bare_cell([], [], [], [])
    n = int(round(T_ms / dt))
    if amp_uA_cm2:
        d.clamps.append((-1, 0, 0, n, amp_uA_cm2 * area * 1e-5))
    m = gen.assemble([d], n_steps=n, dt=dt)
    m["soma_area"][:] = area
    return m


def sealed_cable(n_cv, L=1000.0, diam=2.0, amp_nA=0.1, T_ms=200.0, dt=0.1):
    """Unbranched passive cable on a vanishing soma, current injected at x=0."""
    d = bare_cell([-1], [n_cv], [L], [diam], soma_mech=0)
    n = int(round(T_ms / dt))
    d.clamps.append((-1, 0, 0, n, amp_nA))
    m = gen.assemble([d], n_steps=n, dt=dt)
    m["soma_area"][:] = 1e-9
    return m


def identical_ring(n_cells, delay=200, w=0.05, kick_cells=(0,), n_steps=4000, proto=0):
    """Ring of copies of one config-2 cell; only `kick_cells` get the step-0 kick."""
    base = gen.cell_c2(proto, n_cells)
    cells = []
    for i in range(n_cells):
        d = gen.CellDesc()
        for f in ("parents", "n_cv", "length", "diam", "mech", "gna", "gk", "gl", "gpas", "epas",
                  "soma_mech", "soma_g"):
            setattr(d, f, getattr(base, f))
        d.syn = list(base.syn)
        d.in_conn = [((i - 1) % n_cells, 0, delay, w)]
        d.ext = [(0, 0, 0.05)] if i in kick_cells else []
        cells.append(d)
    return gen.assemble(cells, n_steps=n_steps)


def chain(n_cells, delays, w=0.05, n_steps=2000, cfg_cells=None):
    """Open chain 0 -> 1 -> ... with the given per-link delays; cell 0 kicked."""
    ids = cfg_cells if cfg_cells is not None else list(range(n_cells))
    cells = []
    for k, i in enumerate(ids):
        d = gen.cell_c2(i, 1 << 20, kick_all=False)
        d.in_conn = [(k - 1, 0, int(delays[k - 1]), w)] if k > 0 else []
        d.ext = [(0, 0, 0.05)] if k == 0 else []
        cells.append(d)
    return gen.assemble(cells, n_steps=n_steps)


def mixed_pull_chunks(n_steps=4000, seed=11):
    """Targets whose incoming connections, in rank order (synapse, then
    source), make chunks of 64 of three kinds within one epoch of 800 steps
    (all delays 800): gids 0-95 and 98-105 are sources kicked every 850 steps
    (even gids from step 100, odd from step 400), so each has at most one
    spike per epoch; gids 96 and 97 fire every ~366 steps under a clamp, two
    or three spikes per epoch.  Each of the two targets (106, 107) hears every
    kicked source once and each clamped source 16 times, on synapse 0 (plus a
    few kicked sources on synapse 1): its first 64 connections carry at most
    one event each, the next 64 mix kicked and clamped sources, and the last
    ones are a ragged chunk of kicked sources, whose events share their steps
    with the first chunk's."""
    rng = np.random.default_rng(seed)
    kicked = list(range(96)) + list(range(98, 106))
    cells = []
    for g in range(106):
        d = bare_cell([], [], [], [])
        if g in (96, 97):
            d.clamps.append((-1, 0, 0, n_steps, 0.2))
        else:
            d.syn.append((-1, 0, 2.0, 0.0))
            d.ext = [(0, s, 0.05) for s in range(100 if g % 2 == 0 else 400, n_steps, 850)]
        cells.append(d)
    for _ in range(2):
        d = bare_cell([], [], [], [])
        d.syn.append((-1, 0, 2.0, 0.0))
        d.syn.append((-1, 0, 5.0, -70.0))
        d.in_conn = [(s, 0, 800, float(rng.uniform(1e-4, 5e-4))) for s in kicked]
        d.in_conn += [(s, 0, 800, float(rng.uniform(1e-4, 5e-4))) for s in (96, 97) for _ in range(16)]
        d.in_conn += [(s, 1, 800, float(rng.uniform(1e-4, 5e-4))) for s in kicked[:5]]
        cells.append(d)
    return gen.assemble(cells, n_steps=n_steps)


def longest_epochs(n_steps=33000):
    """Soma-only cells whose shortest delay (20,000 steps) exceeds the
    longest network epoch (16,384 steps), with events due at the last step
    of epoch 1 (step 32767) and the first step of epoch 2 (32768): cell 0,
    kicked at step 0, fires at step 7 and reaches cell 1 (delay 20,000) and
    cell 2 (delay 32,760); cell 3, kicked at step 12,761, fires at 12,768 and
    reaches cell 4 (delay 20,000).  Each event makes its target fire."""
    cells = []
    for _ in range(5):
        d = bare_cell([], [], [], [])
        d.syn.append((-1, 0, 2.0, 0.0))
        cells.append(d)
    cells[0].ext = [(0, 0, 0.05)]
    cells[3].ext = [(0, 12761, 0.05)]
    cells[1].in_conn = [(0, 0, 20000, 0.05)]
    cells[2].in_conn = [(0, 0, 32760, 0.05)]
    cells[4].in_conn = [(3, 0, 20000, 0.05)]
    return gen.assemble(cells, n_steps=n_steps)
