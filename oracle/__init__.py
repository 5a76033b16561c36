"""CPU oracle for the multi-compartment cell stepper -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps `oracle.c` (plain scalar FP64 C, built with
`-O2 -ffp-contract=off`, no fast-math) through ctypes.  It shares no code with
the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# A build of the same source to load instead (the sanitizer test's
# instrumented build); unset, the in-tree library above.
LIB_OVERRIDE = os.environ.get("ORACLE_LIB_OVERRIDE")

_lib = None


def build(threads: bool = False) -> str:
    """Compile the oracle shared library in-tree."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if LIB_OVERRIDE:
            L = C.CDLL(LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB):
                build()
            L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_build.restype = P
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [P, C.c_int64, P, C.c_int64, P]
        L.orc_free.argtypes = [P]
        L.orc_ncv.restype = C.c_int64
        L.orc_ncv.argtypes = [P]
        L.orc_step.restype = C.c_int64
        L.orc_step.argtypes = [P]
        L.orc_nspikes.restype = C.c_int64
        L.orc_nspikes.argtypes = [P]
        L.orc_spikes.argtypes = [P, P, P, P]
        L.orc_get_state.argtypes = [P, P, P, P, P, P]
        L.orc_set_voltage.argtypes = [P, P]
        L.orc_set_gates.argtypes = [P, P, P, P]
        L.orc_cv_info.argtypes = [P, P, P, P, P]
        L.orc_membrane_current.argtypes = [P, C.c_int64, P]
        L.orc_set_params.argtypes = [P, P]
        L.orc_set_varstep.restype = C.c_int
        L.orc_set_varstep.argtypes = [P, P, C.c_int64, P, P, P, C.c_int64]
        L.orc_advance_to.restype = C.c_int
        L.orc_advance_to.argtypes = [P, C.c_int64]
        L.orc_varstep_steps.restype = C.c_int64
        L.orc_varstep_steps.argtypes = [P]
        L.orc_varstep_grid.restype = C.c_int64
        L.orc_varstep_grid.argtypes = [P]
        L.orc_adjoint.restype = C.c_int
        L.orc_adjoint.argtypes = [P, C.c_int64, P, P, P]
        L.orc_hines_solve.argtypes = [C.c_int64, P, P, P, P]
        L.orc_hh_rates.argtypes = [C.c_double, P]
        L.orc_hh_rates_dv.argtypes = [C.c_double, P]
        L.orc_set_densities.restype = C.c_int
        L.orc_set_densities.argtypes = [P, C.c_int64, P, P, P, P, P]
        L.orc_gen_states.restype = C.c_int
        L.orc_gen_states.argtypes = [P, P]
        L.orc_gen_count.restype = C.c_int64
        L.orc_gen_count.argtypes = [P]
        L.orc_gen_defaults.restype = C.c_int
        L.orc_gen_defaults.argtypes = [C.c_int32, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def hines_solve(parent, d, u, b):
    """Solve the symmetric parent-ordered system (diag d, off-diagonal u[i]
    between i and parent[i]); returns x."""
    parent = _c(parent, np.int64)
    d = _c(d, np.float64).copy()
    u = _c(u, np.float64)
    x = _c(b, np.float64).copy()
    lib().orc_hines_solve(len(x), _p(parent), _p(d), _p(u), _p(x))
    return x


def hh_rates(v: float) -> np.ndarray:
    r = np.zeros(6)
    lib().orc_hh_rates(float(v), _p(r))
    return r


def hh_rates_dv(v: float) -> np.ndarray:
    r = np.zeros(6)
    lib().orc_hh_rates_dv(float(v), _p(r))
    return r


# The further density mechanisms the oracle implements (oracle.c, each
# written out from its definition): its number and its parameters in order.
MECHANISMS = {"kdr": (0, ("gbar", "ek")), "hcn": (1, ("gbar", "eh", "vhalf")),
              "hh_dsl": (2, ("gnabar", "gkbar", "gl", "ena", "ek", "el"))}


class Sim:
    """Oracle simulation of a column model (see workloads.gen)."""

    def __init__(self, m: dict, epoch_steps: int | None = None):
        L = lib()
        if epoch_steps is None:
            epoch_steps = int(m["con_delay"].min()) if len(m["con_delay"]) else 1 << 30
        self.K = int(epoch_steps)
        self.m = m
        keep = []

        def a(name, dt):
            x = _c(m[name], dt)
            keep.append(x)
            return _p(x)

        i32, i64, u32, f64 = np.int32, np.int64, np.uint32, np.float64
        args = [C.c_int32(len(m["cell_n_branch"])),
                a("cell_branch_begin", i64), a("cell_n_branch", i32), a("soma_area", f64),
                a("soma_mech", u32), a("soma_gna", f64), a("soma_gk", f64), a("soma_gl", f64),
                a("soma_gpas", f64), a("soma_epas", f64), a("cm", f64), a("Ra", f64),
                a("br_parent", i32), a("br_n_cv", i32), a("br_length", f64), a("br_diam", f64),
                a("br_mech", u32), a("br_gna", f64), a("br_gk", f64), a("br_gl", f64),
                a("br_gpas", f64), a("br_epas", f64),
                C.c_int64(len(m["syn_cell"])), a("syn_cell", i32), a("syn_branch", i32),
                a("syn_cv", i32), a("syn_tau", f64), a("syn_e", f64),
                C.c_int64(len(m["con_src"])), a("con_src", u32), a("con_syn", u32),
                a("con_delay", i32), a("con_w", f64),
                C.c_int64(len(m["ev_syn"])), a("ev_syn", u32), a("ev_step", i64), a("ev_w", f64),
                C.c_int64(len(m["ic_cell"])), a("ic_cell", i32), a("ic_branch", i32),
                a("ic_cv", i32), a("ic_on", i64), a("ic_off", i64), a("ic_amp", f64),
                C.c_double(m["dt"]), C.c_double(m["threshold"]), C.c_double(m["v_init"]),
                C.c_int32(min(self.K, 1 << 30))]
        self.h = C.c_void_p(L.orc_build(*args))
        self.ncv = int(L.orc_ncv(self.h))
        self.nsyn = len(m["syn_cell"])
        dens = m.get("densities") or []
        if dens:  # (cell, branch, mechanism name, {parameter: value})
            n = len(dens)
            cell, branch, mech, npar = (np.zeros(n, np.int32) for _ in range(4))
            prm = np.zeros((n, 8))
            for k, (c, b, name, pv) in enumerate(dens):
                if name not in MECHANISMS:
                    raise ValueError(f"the oracle has no mechanism {name}")
                mid, names = MECHANISMS[name]
                cell[k], branch[k], mech[k] = c, b, mid
                dflt = np.zeros(8)
                npar[k] = L.orc_gen_defaults(mid, _p(dflt))
                prm[k] = dflt
                for pn, v in (pv or {}).items():
                    prm[k, names.index(pn)] = float(v)
            rc = L.orc_set_densities(self.h, n, _p(cell), _p(branch), _p(mech), _p(npar), _p(prm))
            if rc != 0:
                raise ValueError("bad density entry")
        self.ngen = int(L.orc_gen_count(self.h))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    @property
    def step(self) -> int:
        return int(lib().orc_step(self.h))

    def run(self, n_steps: int, probes=None) -> np.ndarray | None:
        if probes is None or len(probes) == 0:
            lib().orc_run(self.h, int(n_steps), None, 0, None)
            return None
        pr = _c(probes, np.int64)
        tr = np.zeros((len(pr), int(n_steps)))
        lib().orc_run(self.h, int(n_steps), _p(pr), len(pr), _p(tr))
        return tr

    def spikes(self):
        n = int(lib().orc_nspikes(self.h))
        gid = np.zeros(n, np.uint32)
        st = np.zeros(n, np.int64)
        t = np.zeros(n)
        if n:
            lib().orc_spikes(self.h, _p(gid), _p(st), _p(t))
        return gid, st, t

    def state(self):
        V, mm, hh, nn = (np.zeros(self.ncv) for _ in range(4))
        g = np.zeros(max(self.nsyn, 1))
        lib().orc_get_state(self.h, _p(V), _p(mm), _p(hh), _p(nn), _p(g))
        return dict(V=V, m=mm, h=hh, n=nn, g=g[: self.nsyn])

    # variable time step (models with continuous times: con_delay_ms, ev_t)
    def set_varstep(self, epoch_steps: int | None = None):
        """Switch to the variable-step mode with the model's continuous
        delays (con_delay_ms) and event times (ev_t); epochs of epoch_steps
        grid steps (default: the most within the minimum delay, or 1000
        without connections)."""
        m = self.m
        d = _c(m["con_delay_ms"], np.float64)
        if epoch_steps is None:
            epoch_steps = 1000
            if len(d):
                epoch_steps = int(np.floor(float(d.min()) / float(m["dt"])))
                while (epoch_steps + 1) * float(m["dt"]) <= float(d.min()):
                    epoch_steps += 1
                while epoch_steps > 1 and epoch_steps * float(m["dt"]) > float(d.min()):
                    epoch_steps -= 1
        syn, t, w = _c(m["ev_syn"], np.uint32), _c(m["ev_t"], np.float64), _c(m["ev_w"], np.float64)
        self._keep_vs = (d, syn, t, w)
        rc = lib().orc_set_varstep(self.h, _p(d), len(syn), _p(syn), _p(t), _p(w), int(epoch_steps))
        if rc != 0:
            raise ValueError("the variable-step mode takes no current clamps, and epochs of at most the "
                             "minimum delay")
        return self

    def advance_to(self, k_end: int):
        """Every cell to grid point k_end (time k_end dt)."""
        lib().orc_advance_to(self.h, int(k_end))

    @property
    def varstep_steps(self) -> int:
        return int(lib().orc_varstep_steps(self.h))

    @property
    def grid_point(self) -> int:
        return int(lib().orc_varstep_grid(self.h))

    def gen_states(self) -> np.ndarray:
        """States of the further mechanisms' instances, [instance][4]."""
        st = np.zeros(max(self.ngen, 1) * 4)
        lib().orc_gen_states(self.h, _p(st))
        return st[: self.ngen * 4].reshape(self.ngen, 4)

    def set_voltage(self, V):
        V = _c(V, np.float64)
        assert V.shape == (self.ncv,)
        lib().orc_set_voltage(self.h, _p(V))

    def set_gates(self, mm, hh, nn):
        mm, hh, nn = (_c(x, np.float64) for x in (mm, hh, nn))
        lib().orc_set_gates(self.h, _p(mm), _p(hh), _p(nn))

    def cv_info(self):
        par = np.zeros(self.ncv, np.int64)
        cap, sig, area = np.zeros(self.ncv), np.zeros(self.ncv), np.zeros(self.ncv)
        lib().orc_cv_info(self.h, _p(par), _p(cap), _p(sig), _p(area))
        return dict(parent=par, cap=cap, sig=sig, area=area)

    def membrane_current(self, n_step: int | None = None):
        I = np.zeros(self.ncv)
        lib().orc_membrane_current(self.h, self.step if n_step is None else int(n_step), _p(I))
        return I

    def set_params(self, theta):
        th = _c(theta, np.float64).reshape(-1)
        lib().orc_set_params(self.h, _p(th))

    def adjoint(self, n_steps: int, dL_dtrace):
        """Run n_steps forward (recording the trajectory), then the discrete
        adjoint.  Returns (trace [cells, n_steps], grad [regions, 3])."""
        ncell = len(self.m["cell_n_branch"])
        nreg = ncell + int(np.sum(self.m["cell_n_branch"]))
        dl = _c(dL_dtrace, np.float64).reshape(ncell, int(n_steps))
        grad = np.zeros((nreg, 3))
        tr = np.zeros((ncell, int(n_steps)))
        rc = lib().orc_adjoint(self.h, int(n_steps), _p(dl), _p(grad), _p(tr))
        if rc == -3:
            raise ValueError("the oracle adjoint does not cover the further density mechanisms")
        if rc != 0:
            raise MemoryError("oracle adjoint: out of memory")
        return tr, grad


def cell_cv_begin(m: dict) -> np.ndarray:
    """User CV numbering: per cell, the soma CV then each branch's CVs
    proximal to distal, branches in the order given."""
    n = np.ones(len(m["cell_n_branch"]), np.int64)
    np.add.at(n, np.repeat(np.arange(len(n)), m["cell_n_branch"]), m["br_n_cv"])
    out = np.zeros(len(n) + 1, np.int64)
    out[1:] = np.cumsum(n)
    return out
