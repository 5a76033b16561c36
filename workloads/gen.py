"""Seeded synthetic workloads for the multi-compartment cell stepper.

This module only draws random model descriptions: morphologies (branch
topology, lengths, diameters), mechanism placement and densities, synapse
placement, network connections, external input events and current clamps.
It holds none of the method's arithmetic (no discretisation, no currents, no
solves); both the CPU oracle and the GPU library consume its output and do all
of that themselves, independently.

A model is a dict of flat numpy column arrays:

cells      cell_branch_begin i64, cell_n_branch i32, soma_area f64,
           soma_mech u32, soma_gna/soma_gk/soma_gl/soma_gpas/soma_epas f64,
           cm f64 (uF/cm^2), Ra f64 (ohm cm)
branches   br_parent i32 (-1 = soma), br_n_cv i32, br_length f64 (um),
           br_diam f64 (um), br_mech u32, br_gna/br_gk/br_gl/br_gpas f64
           (S/cm^2), br_epas f64 (mV)
synapses   syn_cell i32, syn_branch i32 (-1 = soma), syn_cv i32 (0-based CV
           along the branch, proximal first), syn_tau f64 (ms), syn_e f64 (mV)
conns      con_src u32, con_dst u32, con_syn u32 (global synapse index),
           con_delay i32 (steps), con_w f64 (uS)
events     ev_syn u32, ev_step i64, ev_w f64 (uS)
iclamps    ic_cell i32, ic_branch i32, ic_cv i32, ic_on i64, ic_off i64
           (active for step_on <= n < step_off), ic_amp f64 (nA, positive
           depolarises)
scalars    dt (ms), threshold (mV), v_init (mV), n_steps

Every cell draws from its own generator, SeedSequence(entropy, spawn_key=(i,)),
so any subset of cells can be regenerated alone and identically (used to build
the light-cone sub-models the full-size parity checks run on the CPU).

Units and constants follow the textbook Hodgkin-Huxley squid-axon values,
with passive and synapse values chosen where the paper gives none: hh gNa
0.12, gK 0.036, gL 0.0003 S/cm^2; pas 0.001 S/cm^2 at -65 mV; expsyn
reversal 0 mV.
"""
from __future__ import annotations

import math

import numpy as np

MECH_HH = 1
MECH_PAS = 2

SEED_BASE = 1901_07454
DT = 0.025
THRESHOLD = -10.0
V_INIT = -65.0
CM = 1.0
RA = 100.0
SOMA_AREA = 500.0
HH_DEF = (0.12, 0.036, 0.0003)
PAS_G = 0.001
PAS_E = -65.0


def cell_rng(cfg: int, i: int) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED_BASE + int(cfg), spawn_key=(int(i),))
    return np.random.Generator(np.random.PCG64(ss))


def steps_of(t_ms, dt=DT):
    """Map times (ms) to the step grid (ceil), as the Poisson inputs do."""
    return np.ceil(np.asarray(t_ms) / dt - 1e-9).astype(np.int64)


# ----------------------------------------------------------------------------
# topology helpers (parents listed in topological order, -1 = soma)

def full_binary_parents(depth: int) -> np.ndarray:
    n = 2 ** (depth + 1) - 1
    p = np.empty(n, np.int32)
    p[0] = -1
    for b in range(1, n):
        p[b] = (b - 1) // 2
    return p


def yule_parents(rng: np.random.Generator, n_branch_min: int) -> np.ndarray:
    """Yule tree: start with one root branch, split a uniformly chosen leaf
    into two children until at least n_branch_min branches exist."""
    parents = [-1]
    leaves = [0]
    while len(parents) < n_branch_min:
        k = int(rng.integers(len(leaves)))
        b = leaves[k]
        c1, c2 = len(parents), len(parents) + 1
        parents += [b, b]
        leaves[k] = c1
        leaves.append(c2)
    return np.asarray(parents, np.int32)


def spread(total: int, parts: int, rng: np.random.Generator) -> np.ndarray:
    """Split `total` CVs as evenly as possible over `parts` branches."""
    base = total // parts
    out = np.full(parts, base, np.int32)
    extra = total - base * parts
    if extra:
        out[rng.choice(parts, size=extra, replace=False)] += 1
    return out


# ----------------------------------------------------------------------------
# per-cell description

class CellDesc:
    __slots__ = ("parents", "n_cv", "length", "diam", "mech", "gna", "gk", "gl",
                 "gpas", "epas", "soma_mech", "soma_g", "syn", "syn_arr", "in_conn",
                 "in_conn_arr", "ext", "clamps")

    def __init__(self):
        self.syn = []       # (branch, cv, tau, e)
        self.syn_arr = None  # or the same four columns as arrays (many synapses)
        self.in_conn = []   # (src gid, local syn, delay_steps, w)
        self.in_conn_arr = None  # or the same four columns as arrays (many connections)
        self.ext = []       # (local syn, step, w)
        self.clamps = []    # (branch, cv, on, off, amp)


def _geometry(d: CellDesc, rng, n_cv):
    nb = len(d.parents)
    d.n_cv = np.asarray(n_cv, np.int32)
    d.length = rng.uniform(100.0, 300.0, nb)
    d.diam = rng.uniform(1.0, 3.0, nb)


def _dend_pas(d: CellDesc):
    nb = len(d.parents)
    d.mech = np.full(nb, MECH_PAS, np.uint32)
    d.gna = np.zeros(nb)
    d.gk = np.zeros(nb)
    d.gl = np.zeros(nb)
    d.gpas = np.full(nb, PAS_G)
    d.epas = np.full(nb, PAS_E)


def _soma_hh(d: CellDesc):
    d.soma_mech = MECH_HH
    d.soma_g = (HH_DEF[0], HH_DEF[1], HH_DEF[2], 0.0, PAS_E)


def _random_cv(rng, d: CellDesc):
    b = int(rng.integers(len(d.parents)))
    return b, int(rng.integers(int(d.n_cv[b])))


def _poisson_steps(rng, rate_hz, t_ms, dt=DT):
    n = rng.poisson(rate_hz * t_ms * 1e-3)
    return np.sort(steps_of(rng.uniform(0.0, t_ms, n), dt))


def cell_c1(i: int) -> CellDesc:
    rng = cell_rng(1, i)
    d = CellDesc()
    d.parents = np.full(4, -1, np.int32)
    _geometry(d, rng, [32] * 4)
    _dend_pas(d)
    _soma_hh(d)
    d.syn.append((-1, 0, 2.0, 0.0))
    t = np.sort(rng.uniform(0.0, 100.0, 10))
    for s in steps_of(t):
        d.ext.append((0, int(s), 0.01))
    return d


def cell_c2(i: int, n_cells: int, kick_all: bool = True) -> CellDesc:
    rng = cell_rng(2, i)
    d = CellDesc()
    d.parents = full_binary_parents(6)
    _geometry(d, rng, [8] * len(d.parents))
    _dend_pas(d)
    _soma_hh(d)
    d.syn.append((-1, 0, 2.0, 0.0))
    for _ in range(9):
        b, k = _random_cv(rng, d)
        d.syn.append((b, k, 2.0, 0.0))
    d.in_conn.append(((i - 1) % n_cells, 0, 200, 0.05))
    if kick_all or i == 0:
        d.ext.append((0, 0, 0.05))
    return d


def cell_c3(i: int, t_ms: float = 200.0) -> CellDesc:
    rng = cell_rng(3, i)
    d = CellDesc()
    n = int(round(math.exp(rng.uniform(math.log(50.0), math.log(5000.0)))))
    nb_min = -(-(n - 1) // 8)
    d.parents = yule_parents(rng, nb_min)
    nb = len(d.parents)
    _geometry(d, rng, spread(n - 1, nb, rng))
    _dend_pas(d)
    hh = rng.uniform(size=nb) < 0.25
    d.mech[hh] = MECH_HH
    d.gna[hh], d.gk[hh], d.gl[hh] = HH_DEF
    d.gpas[hh] = 0.0
    _soma_hh(d)
    for s in range(20):
        b, k = _random_cv(rng, d)
        d.syn.append((b, k, 2.0, 0.0))
        for st in _poisson_steps(rng, 10.0, t_ms):
            d.ext.append((s, int(st), 0.01))
    return d


C4_COUNTS = [16] * 4 + [15] * 9


def cell_c4(i: int, hidden: bool) -> CellDesc:
    """Adjoint workload cell. `hidden` selects the target parameters;
    otherwise the perturbed starting point theta_0 is returned."""
    rng = cell_rng(4, i)
    d = CellDesc()
    d.parents = yule_parents(rng, 13)
    nb = len(d.parents)
    _geometry(d, rng, rng.permutation(np.asarray(C4_COUNTS, np.int32)))
    nr = nb + 1
    th = np.stack([rng.uniform(0.08, 0.16, nr), rng.uniform(0.024, 0.048, nr),
                   rng.uniform(2e-4, 4e-4, nr)], axis=1)
    pert = rng.uniform(0.8, 1.2, (nr, 3))
    if not hidden:
        th = th * pert
    d.soma_mech = MECH_HH | MECH_PAS
    d.soma_g = (th[0, 0], th[0, 1], 0.0, th[0, 2], PAS_E)
    d.mech = np.full(nb, MECH_HH | MECH_PAS, np.uint32)
    d.gna, d.gk, d.gpas = th[1:, 0].copy(), th[1:, 1].copy(), th[1:, 2].copy()
    d.gl = np.zeros(nb)
    d.epas = np.full(nb, PAS_E)
    d.clamps.append((-1, 0, 200, 2000, 0.2))
    return d


def cell_c5(i: int, n_cells: int, n_in: int = 100, t_ms: float = 200.0,
            w_bg: float = 0.05) -> CellDesc:
    rng = cell_rng(5, i)
    d = CellDesc()
    d.parents = yule_parents(rng, 187)
    nb = len(d.parents)
    _geometry(d, rng, [8] * nb)
    _dend_pas(d)
    _soma_hh(d)
    n_in = min(n_in, n_cells - 1)
    src = rng.choice(n_cells - 1, size=n_in, replace=False)
    src = np.where(src >= i, src + 1, src)
    delays = np.rint(rng.uniform(5.0, 10.0, n_in) / DT).astype(np.int64)
    bs = rng.integers(nb, size=n_in)
    ks = rng.integers(d.n_cv[bs])
    d.syn = list(zip(bs.tolist(), ks.tolist(), [2.0] * n_in, [0.0] * n_in))
    d.in_conn = list(zip(src.tolist(), range(n_in), delays.tolist(), [0.01] * n_in))
    d.syn.append((-1, 0, 2.0, 0.0))
    for st in _poisson_steps(rng, 5.0, t_ms):
        d.ext.append((n_in, int(st), w_bg))
    return d


def cell_c6(i: int, n_cells: int, n_syn: int = 10000, kick_all: bool = True) -> CellDesc:
    """The synapse-dominated ring: random trees of 90-170 CVs (mean 130),
    hh soma, pas dendrites, n_syn expsyn at random CVs of which only synapse 0
    (on the soma) receives the ring connection from cell i - 1."""
    rng = cell_rng(6, i)
    d = CellDesc()
    n = int(rng.integers(90, 171))
    d.parents = yule_parents(rng, -(-(n - 1) // 8))
    nb = len(d.parents)
    _geometry(d, rng, spread(n - 1, nb, rng))
    _dend_pas(d)
    _soma_hh(d)
    bs = rng.integers(nb, size=n_syn - 1)
    ks = rng.integers(d.n_cv[bs])
    d.syn_arr = (np.concatenate([[-1], bs]), np.concatenate([[0], ks]),
                 np.full(n_syn, 2.0), np.zeros(n_syn))
    d.in_conn.append(((i - 1) % n_cells, 0, 200, 0.05))
    if kick_all or i == 0:
        d.ext.append((0, 0, 0.05))
    return d


def cell_c7(i: int, n_cells: int, n_syn: int = 10000, min_delay_ms: float = 20.0,
            w_net: float = 2e-6, rate_hz: float = 50.0, n_steps: int = 4000) -> CellDesc:
    """The 10k-connectivity model: the cells of the synapse-dominated ring
    (same morphologies and synapse placement), every synapse wired from a
    uniformly drawn other cell with the minimum delay and a small excitatory
    weight, and a periodic drive on synapse 0 that makes all cells fire
    together at `rate_hz`."""
    d = cell_c6(i, n_cells, n_syn, kick_all=False)
    d.in_conn = []
    d.ext = []
    rng = cell_rng(7, i)
    src = rng.integers(n_cells - 1, size=n_syn) if n_cells > 1 else np.zeros(0, np.int64)
    src = np.where(src >= i, src + 1, src)
    k = len(src)
    d.in_conn_arr = (src, np.arange(k), np.full(k, int(round(min_delay_ms / DT))), np.full(k, w_net))
    period = int(round(1000.0 / rate_hz / DT))
    for st in range(0, max(int(n_steps), 1), period):
        d.ext.append((0, st, 0.05))
    return d


# ----------------------------------------------------------------------------
# assembly of a model from cell descriptions

def assemble(cells: list[CellDesc], gids=None, n_steps: int = 0,
             dt: float = DT, remote_sources: bool = False) -> dict:
    """Flatten per-cell descriptions into the column model.  `gids` are the
    global ids the cells had in the full network; connections whose source is
    not among them are dropped (used for light-cone sub-models), unless
    remote_sources, which keeps every source gid as it is (the cells are then
    gids 0 .. n-1, one rank of a larger network)."""
    if gids is None:
        gids = list(range(len(cells)))
    remap = {int(g): k for k, g in enumerate(gids)}
    C = len(cells)
    nbs = np.array([len(c.parents) for c in cells], np.int64)
    bb = np.zeros(C, np.int64)
    bb[1:] = np.cumsum(nbs)[:-1]
    cat = lambda f, dt_: np.concatenate([np.asarray(getattr(c, f), dt_) for c in cells]) if C else np.zeros(0, dt_)
    m = dict(
        cell_branch_begin=bb, cell_n_branch=nbs.astype(np.int32),
        soma_area=np.full(C, SOMA_AREA), soma_mech=np.array([c.soma_mech for c in cells], np.uint32),
        soma_gna=np.array([c.soma_g[0] for c in cells]), soma_gk=np.array([c.soma_g[1] for c in cells]),
        soma_gl=np.array([c.soma_g[2] for c in cells]), soma_gpas=np.array([c.soma_g[3] for c in cells]),
        soma_epas=np.array([c.soma_g[4] for c in cells]),
        cm=np.full(C, CM), Ra=np.full(C, RA),
        br_parent=cat("parents", np.int32), br_n_cv=cat("n_cv", np.int32),
        br_length=cat("length", np.float64), br_diam=cat("diam", np.float64),
        br_mech=cat("mech", np.uint32), br_gna=cat("gna", np.float64), br_gk=cat("gk", np.float64),
        br_gl=cat("gl", np.float64), br_gpas=cat("gpas", np.float64), br_epas=cat("epas", np.float64),
    )
    cols = []
    for c in cells:
        if c.syn_arr is not None:
            cols.append(tuple(np.asarray(x) for x in c.syn_arr))
        else:
            cols.append(tuple(np.array([s[j] for s in c.syn]) for j in range(4)))
    nsyn = np.array([len(x[0]) for x in cols], np.int64)
    sb = np.zeros(C + 1, np.int64)
    sb[1:] = np.cumsum(nsyn)
    colcat = lambda j, dt_: np.concatenate([x[j].astype(dt_) for x in cols]) if C else np.zeros(0, dt_)
    m["syn_cell"] = np.repeat(np.arange(C, dtype=np.int32), nsyn)
    m["syn_branch"] = colcat(0, np.int32)
    m["syn_cv"] = colcat(1, np.int32)
    m["syn_tau"] = colcat(2, np.float64)
    m["syn_e"] = colcat(3, np.float64)
    con = [(remap[src], ci, int(sb[ci]) + ls, dl, w)
           for ci, c in enumerate(cells) for (src, ls, dl, w) in c.in_conn if int(src) in remap]
    ccols = [np.array([x[j] for x in con], t) for j, t in
             enumerate((np.uint32, np.uint32, np.uint32, np.int32, np.float64))]
    if any(c.in_conn_arr is not None for c in cells):
        # vectorised connection columns (many connections per cell)
        lut = np.full(int(max(gids)) + 1 if len(gids) else 1, -1, np.int64)
        lut[np.asarray(gids, np.int64)] = np.arange(len(gids))
        parts = [ccols]
        for ci, c in enumerate(cells):
            if c.in_conn_arr is None:
                continue
            src, ls, dl, w = (np.asarray(x) for x in c.in_conn_arr)
            src = src.astype(np.int64)
            if remote_sources:
                parts.append([src.astype(np.uint32), np.full(len(src), ci, np.uint32),
                              (sb[ci] + ls).astype(np.uint32), dl.astype(np.int32), w.astype(np.float64)])
                continue
            ok = src < len(lut)
            ok[ok] = lut[src[ok]] >= 0
            parts.append([lut[src[ok]].astype(np.uint32), np.full(int(ok.sum()), ci, np.uint32),
                          (sb[ci] + ls[ok]).astype(np.uint32), dl[ok].astype(np.int32), w[ok].astype(np.float64)])
        ccols = [np.concatenate([p_[j] for p_ in parts]) for j in range(5)]
    m["con_src"], m["con_dst"], m["con_syn"], m["con_delay"], m["con_w"] = ccols
    # a connection's or event's synapse is local to its cell: one index past
    # the cell's synapses would silently name another cell's synapse
    bad = [ci for ci, c in enumerate(cells)
           if any(not 0 <= int(x[1]) < nsyn[ci] for x in c.in_conn)
           or any(not 0 <= int(x[0]) < nsyn[ci] for x in c.ext)
           or (c.in_conn_arr is not None and len(c.in_conn_arr[1])
               and not (0 <= np.min(c.in_conn_arr[1]) and np.max(c.in_conn_arr[1]) < nsyn[ci]))]
    if bad:
        raise ValueError(f"cell {bad[0]}: connection or event synapse out of the cell's range")
    ev = [(int(sb[ci]) + ls, st, w) for ci, c in enumerate(cells) for (ls, st, w) in c.ext]
    m["ev_syn"] = np.array([x[0] for x in ev], np.uint32)
    m["ev_step"] = np.array([x[1] for x in ev], np.int64)
    m["ev_w"] = np.array([x[2] for x in ev], np.float64)
    ic = [(ci,) + tuple(x) for ci, c in enumerate(cells) for x in c.clamps]
    m["ic_cell"] = np.array([x[0] for x in ic], np.int32)
    m["ic_branch"] = np.array([x[1] for x in ic], np.int32)
    m["ic_cv"] = np.array([x[2] for x in ic], np.int32)
    m["ic_on"] = np.array([x[3] for x in ic], np.int64)
    m["ic_off"] = np.array([x[4] for x in ic], np.int64)
    m["ic_amp"] = np.array([x[5] for x in ic], np.float64)
    m["dt"], m["threshold"], m["v_init"], m["n_steps"] = dt, THRESHOLD, V_INIT, int(n_steps)
    m["gids"] = np.asarray(gids, np.int64)
    return m


def n_cvs(m: dict) -> np.ndarray:
    """CVs per cell: one soma CV plus the branch CV counts (a count, not a
    discretisation)."""
    out = np.ones(len(m["cell_n_branch"]), np.int64)
    np.add.at(out, np.repeat(np.arange(len(out)), m["cell_n_branch"]), m["br_n_cv"])
    return out


# ----------------------------------------------------------------------------
# the five workloads (and scaled-down variants used by tests)

def config1() -> dict:
    return assemble([cell_c1(0)], n_steps=4000)


def config2(n_cells: int = 8192, cells=None, kick_all: bool = True, n_steps: int = 4000) -> dict:
    ids = range(n_cells) if cells is None else cells
    return assemble([cell_c2(i, n_cells, kick_all) for i in ids], gids=list(ids), n_steps=n_steps)


def config3(n_cells: int = 4096, cells=None, n_steps: int = 8000) -> dict:
    ids = range(n_cells) if cells is None else cells
    t_ms = n_steps * DT
    return assemble([cell_c3(i, t_ms) for i in ids], gids=list(ids), n_steps=n_steps)


def config4(n_cells: int = 256, hidden: bool = False, cells=None, n_steps: int = 2000) -> dict:
    ids = range(n_cells) if cells is None else cells
    return assemble([cell_c4(i, hidden) for i in ids], gids=list(ids), n_steps=n_steps)


def config4_theta(m: dict) -> np.ndarray:
    """Per-region (soma, branches...) [gNa, gK, g_pas] of a config-4 model,
    shape [cells, 14, 3]."""
    C = len(m["cell_n_branch"])
    nb = int(m["cell_n_branch"][0])
    th = np.empty((C, nb + 1, 3))
    th[:, 0, 0], th[:, 0, 1], th[:, 0, 2] = m["soma_gna"], m["soma_gk"], m["soma_gpas"]
    th[:, 1:, 0] = m["br_gna"].reshape(C, nb)
    th[:, 1:, 1] = m["br_gk"].reshape(C, nb)
    th[:, 1:, 2] = m["br_gpas"].reshape(C, nb)
    return th


def config5(n_cells: int = 65536, cells=None, n_in: int = 100, n_steps: int = 8000) -> dict:
    ids = range(n_cells) if cells is None else cells
    t_ms = n_steps * DT
    return assemble([cell_c5(i, n_cells, n_in, t_ms) for i in ids], gids=list(ids), n_steps=n_steps)


def cell_c5_fixed_inputs(i: int, n_cells: int = 65536, t_ms: float = 20.0, src_rate_hz: float = 5.0) -> CellDesc:
    """Cell i of the 65536-cell network with its network input replaced by
    fixed input events (the gradient workload treats input events as fixed):
    each incoming connection delivers a seeded Poisson spike train of rate
    src_rate_hz standing for its source, delayed by the connection's delay
    and with its weight; the background input is unchanged."""
    d = cell_c5(i, n_cells, t_ms=t_ms)
    ss = np.random.SeedSequence(SEED_BASE + 5, spawn_key=(int(i), 1))
    rng = np.random.Generator(np.random.PCG64(ss))
    end = int(steps_of(t_ms))
    for (_, ls, delay, w) in d.in_conn:
        for st in _poisson_steps(rng, src_rate_hz, t_ms):
            if int(st) + int(delay) < end:
                d.ext.append((int(ls), int(st) + int(delay), float(w)))
    d.in_conn = []
    return d


def config5_subset(n_cells: int = 1024, cells=None, n_steps: int = 800) -> dict:
    """The first n_cells cells of the 65536-cell network as a gradient
    workload: morphologies, synapses and background as in the network, the
    network input as fixed seeded events (cell_c5_fixed_inputs)."""
    ids = range(n_cells) if cells is None else cells
    t_ms = n_steps * DT
    return assemble([cell_c5_fixed_inputs(i, 65536, t_ms) for i in ids], gids=list(ids), n_steps=n_steps)


def config6(n_cells: int = 8192, cells=None, kick_all: bool = True, n_steps: int = 4000,
            n_syn: int = 10000) -> dict:
    ids = range(n_cells) if cells is None else cells
    return assemble([cell_c6(i, n_cells, n_syn, kick_all) for i in ids], gids=list(ids), n_steps=n_steps)


def config7(n_cells: int = 8192, cells=None, n_steps: int = 4000, n_syn: int = 10000,
            min_delay_ms: float = 20.0, w_net: float = 2e-6) -> dict:
    ids = range(n_cells) if cells is None else cells
    return assemble([cell_c7(i, n_cells, n_syn, min_delay_ms, w_net, n_steps=n_steps) for i in ids],
                    gids=list(ids), n_steps=n_steps)


def config7_dry_run(n_cells: int = 8192, ranks: int = 1, n_steps: int = 4000, n_syn: int = 10000,
                    min_delay_ms: float = 20.0, w_net: float = 2e-6) -> dict:
    """One rank's share of the 10k-connectivity model on `ranks` identical
    ranks (the dry run of Sec. V-E): the cells of config 7, every synapse
    wired from a uniformly drawn other gid of all ranks' ranks x n_cells
    cells (source gids kept as they are).  Run with dry_run_ranks = ranks, a
    remote gid g fires as local cell g mod n_cells does."""
    cells = []
    for i in range(n_cells):
        d = cell_c7(i, n_cells, n_syn, min_delay_ms, w_net, n_steps=n_steps)
        src = _dry_run_sources(i, n_cells, ranks, n_syn)
        k = len(src)
        d.in_conn_arr = (src, np.arange(k), np.full(k, int(round(min_delay_ms / DT))), np.full(k, w_net))
        cells.append(d)
    return assemble(cells, n_steps=n_steps, remote_sources=True)


def _dry_run_sources(i: int, n_cells: int, ranks: int, n_syn: int) -> np.ndarray:
    ss = np.random.SeedSequence(SEED_BASE + 7, spawn_key=(int(i), 2))
    rng = np.random.Generator(np.random.PCG64(ss))
    n_src = int(ranks) * int(n_cells)
    src = rng.integers(n_src - 1, size=n_syn) if n_src > 1 else np.zeros(0, np.int64)
    return np.where(src >= i, src + 1, src)


def config7_dry_run_sources(n_cells: int, ranks: int, n_syn: int = 10000) -> np.ndarray:
    """The con_src column of config7_dry_run(n_cells, ranks, ..., n_syn) (the
    connections of cell 0, then cell 1, ... each in synapse order), drawn
    alone: the same model at another rank count differs only in it."""
    return np.concatenate([_dry_run_sources(i, n_cells, ranks, n_syn) for i in range(n_cells)]).astype(np.uint32)


def timed(m: dict, con_delay_ms=None, ev_t=None) -> dict:
    """A model for the variable time step: continuous connection delays
    (con_delay_ms, ms) and event times (ev_t, ms), by default the step-grid
    ones (delay_steps x dt, step x dt)."""
    out = dict(m)
    out["con_delay_ms"] = (np.asarray(con_delay_ms, np.float64) if con_delay_ms is not None
                           else m["con_delay"].astype(np.float64) * m["dt"])
    out["ev_t"] = np.asarray(ev_t, np.float64) if ev_t is not None else m["ev_step"].astype(np.float64) * m["dt"]
    return out


def config2_timed(n_cells: int = 8192, cells=None, t_ms: float = 100.0) -> dict:
    """The 8192-cell ring for the variable time step: the cells of config 2,
    ring delays U(5, 5.5) ms and kicks at U(0, 1) ms (off the step grid), and
    Poisson input at 10 Hz on each dendritic synapse (w 0.01 uS) at
    continuous times."""
    ids = list(range(n_cells)) if cells is None else list(cells)
    m = config2(n_cells=n_cells, cells=ids, n_steps=int(round(t_ms / DT)))
    delay, ev_syn, ev_t, ev_w = [], [], [], []
    syn0 = np.concatenate([[0], np.cumsum(np.bincount(m["syn_cell"], minlength=len(ids)))])
    for k, i in enumerate(ids):
        ss = np.random.SeedSequence(SEED_BASE + 2, spawn_key=(int(i), 3))
        rng = np.random.Generator(np.random.PCG64(ss))
        delay.append(rng.uniform(5.0, 5.5))
        ev_syn.append(syn0[k])
        ev_t.append(rng.uniform(0.0, 1.0))
        ev_w.append(0.05)
        for q in range(int(syn0[k]) + 1, int(syn0[k + 1])):
            times = np.sort(rng.uniform(0.0, t_ms, rng.poisson(10.0 * t_ms * 1e-3)))
            ev_syn.extend([q] * len(times))
            ev_t.extend(times.tolist())
            ev_w.extend([0.01] * len(times))
    # connection j ends on the cell ids[j'] whose ring predecessor fired; the
    # delay drawn for that destination cell
    dst_pos = {int(g): k for k, g in enumerate(ids)}
    d_ms = np.array([delay[dst_pos[int(m["gids"][int(dc)])]] for dc in m["con_dst"]], np.float64)
    m["ev_syn"] = np.array(ev_syn, np.uint32)
    m["ev_step"] = np.zeros(len(ev_syn), np.int64)
    m["ev_w"] = np.array(ev_w, np.float64)
    return timed(m, con_delay_ms=d_ms, ev_t=np.array(ev_t, np.float64))


def with_densities(m: dict, dens) -> dict:
    """The model with generated density mechanisms: (cell, branch, mechanism
    name, {parameter: value}) entries, branch -1 = the soma."""
    out = dict(m)
    out["densities"] = [(int(c), int(b), str(n), dict(p or {})) for c, b, n, p in dens]
    return out


def config2_mech(n_cells: int = 8, n_steps: int = 2000, cells=None) -> dict:
    """The ring's cells with the generated mechanisms on them: hcn on the soma
    (gbar 3e-4 S/cm^2), kdr on every dendritic branch (gbar 2e-3), and
    hh_dsl on branch 0 (gnabar 0.04, gkbar 0.012, no leak); every cell is
    kicked again on its soma synapse every 10 ms (w 0.05 uS), so that it
    keeps firing.  `cells` picks a subset of the n_cells ring's cells."""
    m = config2(n_cells=n_cells, cells=cells, n_steps=n_steps)
    nc = len(m["cell_n_branch"])
    syn0 = np.concatenate([[0], np.cumsum(np.bincount(m["syn_cell"], minlength=nc))])[:-1]
    kick = np.arange(400, n_steps, 400, dtype=np.int64)
    m["ev_syn"] = np.concatenate([m["ev_syn"], np.repeat(syn0.astype(np.uint32), len(kick))])
    m["ev_step"] = np.concatenate([m["ev_step"], np.tile(kick, nc)])
    m["ev_w"] = np.concatenate([m["ev_w"], np.full(nc * len(kick), 0.05)])
    dens = []
    for c in range(nc):
        dens.append((c, -1, "hcn", {"gbar": 3e-4}))
        for b in range(int(m["cell_n_branch"][c])):
            dens.append((c, b, "kdr", {"gbar": 2e-3}))
        dens.append((c, 0, "hh_dsl", {"gnabar": 0.04, "gkbar": 0.012, "gl": 0.0}))
    return with_densities(m, dens)


def ring_light_cone(n_cells: int, target: int, n_steps: int, delay: int = 200) -> list[int]:
    """Cells of the config-2 ring whose spikes can reach `target` within
    n_steps: a spike of cell target-j needs at least j*(delay+1) steps."""
    hops = n_steps // (delay + 1) + 1
    return [(target - j) % n_cells for j in range(min(hops, n_cells - 1), -1, -1)]
