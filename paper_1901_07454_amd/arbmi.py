"""Python binding of the C ABI in include/arbmi.h (argument marshalling only).

Every function here forwards to the HIP library `libarbmi.so`; nothing of the
method runs in Python.  If the library has not been built this module raises
on use: there is no CPU fallback.

Device memory for a sim comes from PyTorch's caching allocator (passed in as
the ABI's allocator callbacks) and work goes on PyTorch's current stream
unless another stream is given.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libarbmi.so")

ARB_OK, ARB_EINVAL, ARB_ENOMEM, ARB_EHIP, ARB_ESTATE, ARB_EOVERFLOW = 0, -1, -2, -3, -4, -5
ARB_MECH_HH, ARB_MECH_PAS = 1, 2
ARB_FLAG_TIME_KERNELS = 1
ARB_FLAG_GRADIENTS = 2
ARB_FLAG_GRAPH = 4
ARB_FLAG_AUTOTUNE = 8

# numpy mirrors of the ABI structs (natural C alignment)
BRANCH = np.dtype([("parent", "<i4"), ("n_cv", "<i4"), ("length_um", "<f8"), ("diam_um", "<f8"),
                   ("mech", "<u4"), ("reserved", "<u4"), ("gbar_na", "<f8"), ("gbar_k", "<f8"),
                   ("gl_hh", "<f8"), ("g_pas", "<f8"), ("e_pas", "<f8")], align=True)
CELL = np.dtype([("branch_begin", "<i8"), ("n_branch", "<i4"), ("soma_mech", "<u4"),
                 ("soma_area_um2", "<f8"), ("soma_gbar_na", "<f8"), ("soma_gbar_k", "<f8"),
                 ("soma_gl_hh", "<f8"), ("soma_g_pas", "<f8"), ("soma_e_pas", "<f8"),
                 ("cm_uF_cm2", "<f8"), ("Ra_ohm_cm", "<f8")], align=True)
SYNAPSE = np.dtype([("cell", "<i4"), ("branch", "<i4"), ("cv", "<i4"), ("reserved", "<i4"),
                    ("tau_ms", "<f8"), ("e_rev_mV", "<f8")], align=True)
CONNECTION = np.dtype([("src", "<u4"), ("dst", "<u4"), ("syn", "<u4"), ("delay_steps", "<i4"),
                       ("w_uS", "<f8")], align=True)
EVENT = np.dtype([("syn", "<u4"), ("reserved", "<i4"), ("step", "<i8"), ("w_uS", "<f8")], align=True)
ICLAMP = np.dtype([("cell", "<i4"), ("branch", "<i4"), ("cv", "<i4"), ("reserved", "<i4"),
                   ("step_on", "<i8"), ("step_off", "<i8"), ("amp_nA", "<f8")], align=True)
SPIKE = np.dtype([("gid", "<u4"), ("reserved", "<i4"), ("step", "<i8"), ("t_ms", "<f8")], align=True)

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class arb_params(C.Structure):
    _fields_ = [("dt_ms", C.c_double), ("threshold_mV", C.c_double), ("v_init_mV", C.c_double),
                ("epoch_steps", C.c_int32), ("flags", C.c_int32), ("hip_stream", C.c_void_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("spike_capacity", C.c_int64), ("event_capacity", C.c_int64),
                ("block_threads", C.c_int32), ("coef_mode", C.c_int32),
                ("cells_per_pack", C.c_int32), ("dry_run_ranks", C.c_int32), ("reserved0", C.c_int32),
                ("densities", C.c_void_p), ("n_densities", C.c_int64)]


class arb_density(C.Structure):
    _fields_ = [("cell", C.c_int32), ("branch", C.c_int32), ("mech", C.c_int32), ("n_param", C.c_int32),
                ("param", C.c_double * 8)]


class arb_mech_info(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("n_params", C.c_int32), ("n_states", C.c_int32),
                ("param_names", (C.c_char * 16) * 8), ("defaults", C.c_double * 8)]


class arb_info(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_packs", C.c_int32), ("n_cv", C.c_int64),
                ("n_slots", C.c_int64), ("n_hh", C.c_int64), ("n_syn", C.c_int64),
                ("n_conn", C.c_int64), ("step", C.c_int64), ("epoch_steps", C.c_int32),
                ("block_threads", C.c_int32), ("coef_mode", C.c_int32), ("lds_bytes", C.c_int32),
                ("device_bytes", C.c_int64), ("bytes_per_step", C.c_int64),
                ("reg_slots", C.c_int32), ("reg_len", C.c_int32), ("syn_hbm", C.c_int32),
                ("n_classes", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["arb_build_cells", "arb_step", "arb_get_voltages", "arb_get_spikes", "arb_set_probes",
           "arb_get_trace", "arb_set_params", "arb_grad_forward", "arb_grad_backward",
           "arb_get_state", "arb_set_state", "arb_get_info", "arb_get_kernel_time", "arb_sync",
           "arb_free", "arb_last_error", "arb_plan_layout", "arb_get_voltages_noalloc", "arb_build_cells_timed",
           "arb_get_step_count", "arb_mechanism_count", "arb_mechanism_info", "arb_get_mechanism_instances"]

_lib = None


class ArbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"arbmi error {code}: {msg}")
        self.code = code


def load():
    """Load libarbmi.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing")
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "arb_build_cells": [P, I32, P, I64, P, I64, P, I64, P, I64, P, I32, C.POINTER(arb_params), C.POINTER(P)],
            "arb_build_cells_timed": [P, I32, P, I64, P, I64, P, P, I64, P, P, I64, C.POINTER(arb_params),
                                      C.POINTER(P)],
            "arb_get_step_count": [P, C.POINTER(I64)],
            "arb_mechanism_count": [],
            "arb_mechanism_info": [I32, C.POINTER(arb_mech_info)],
            "arb_get_mechanism_instances": [P, C.POINTER(I64), I32],
            "arb_step": [P, I64],
            "arb_get_voltages": [P, P, I64, C.c_int],
            "arb_get_voltages_noalloc": [P, P, I64],
            "arb_get_spikes": [P, P, I64, C.POINTER(I64)],
            "arb_set_probes": [P, P, I32, I64],
            "arb_get_trace": [P, P, I64, C.c_int, C.POINTER(I64)],
            "arb_set_params": [P, P, I64],
            "arb_grad_forward": [P, I64, I32, P],
            "arb_grad_backward": [P, P, P],
            "arb_get_state": [P, P, I64, C.POINTER(I64)],
            "arb_set_state": [P, P, I64],
            "arb_get_info": [P, C.POINTER(arb_info)],
            "arb_get_kernel_time": [P, C.POINTER(C.c_double), C.POINTER(I64)],
            "arb_sync": [P],
            "arb_free": [P],
            "arb_last_error": [],
            "arb_plan_layout": [P, I32, P, I64, P, I64, P, I64, P, I64, P, I32, C.POINTER(arb_params),
                                C.POINTER(arb_info)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.arb_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def arb_last_error() -> str:
    return load().arb_last_error().decode()


def _check(rc):
    if rc != ARB_OK:
        raise ArbError(rc, arb_last_error())
    return rc


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# the ABI calls, one to one

def arb_build_cells(cells, branches, syn, conn, ev, stim, params: arb_params):
    L = load()
    out = C.c_void_p()
    arrs = [np.ascontiguousarray(x, dtype=d) for x, d in
            ((cells, CELL), (branches, BRANCH), (syn, SYNAPSE), (conn, CONNECTION), (ev, EVENT), (stim, ICLAMP))]
    c, b, s, k, e, i = arrs
    _check(L.arb_build_cells(_ptr(c), len(c), _ptr(b), len(b), _ptr(s), len(s), _ptr(k), len(k), _ptr(e), len(e),
                             _ptr(i), len(i), C.byref(params), C.byref(out)))
    return out


def arb_build_cells_timed(cells, branches, syn, conn, delay_ms, ev, t_ms, params: arb_params):
    L = load()
    out = C.c_void_p()
    arrs = [np.ascontiguousarray(x, dtype=d) for x, d in
            ((cells, CELL), (branches, BRANCH), (syn, SYNAPSE), (conn, CONNECTION), (ev, EVENT))]
    c, b, s, k, e = arrs
    dm = np.ascontiguousarray(delay_ms, dtype=np.float64)
    tm = np.ascontiguousarray(t_ms, dtype=np.float64)
    if len(dm) != len(k) or len(tm) != len(e):
        raise ValueError("one delay per connection and one time per event")
    _check(L.arb_build_cells_timed(_ptr(c), len(c), _ptr(b), len(b), _ptr(s), len(s), _ptr(k), _ptr(dm), len(k),
                                   _ptr(e), _ptr(tm), len(e), C.byref(params), C.byref(out)))
    return out


def mechanism_catalogue() -> list[dict]:
    """The generated mechanisms: name, parameter names and defaults, state
    count, in id order."""
    L = load()
    out = []
    for i in range(L.arb_mechanism_count()):
        info = arb_mech_info()
        _check(L.arb_mechanism_info(i, C.byref(info)))
        names = [info.param_names[k].value.decode() for k in range(info.n_params)]
        out.append({"id": i, "name": info.name.decode(), "params": names,
                    "defaults": [info.defaults[k] for k in range(info.n_params)], "n_states": info.n_states})
    return out


def density_structs(dens) -> np.ndarray | None:
    """(cell, branch, mechanism name, {parameter: value}) tuples as the ABI's
    arb_density entries (branch -1 = the soma)."""
    if not dens:
        return None
    cat = {m["name"]: m for m in mechanism_catalogue()}
    arr = (arb_density * len(dens))()
    for k, (cell, branch, name, prm) in enumerate(dens):
        if name not in cat:
            raise ValueError(f"unknown mechanism {name}")
        m = cat[name]
        arr[k].cell, arr[k].branch, arr[k].mech = int(cell), int(branch), m["id"]
        vals = list(m["defaults"])
        for pn, v in (prm or {}).items():
            if pn not in m["params"]:
                raise ValueError(f"{name} has no parameter {pn}")
            vals[m["params"].index(pn)] = float(v)
        arr[k].n_param = len(vals)
        for j, v in enumerate(vals):
            arr[k].param[j] = v
    return arr


def arb_get_step_count(sim) -> int:
    n = C.c_int64()
    _check(load().arb_get_step_count(sim, C.byref(n)))
    return n.value


def arb_plan_layout(cells, branches, syn, conn, ev, stim, params: arb_params) -> dict:
    L = load()
    info = arb_info()
    arrs = [np.ascontiguousarray(x, dtype=d) for x, d in
            ((cells, CELL), (branches, BRANCH), (syn, SYNAPSE), (conn, CONNECTION), (ev, EVENT), (stim, ICLAMP))]
    c, b, s, k, e, i = arrs
    _check(L.arb_plan_layout(_ptr(c), len(c), _ptr(b), len(b), _ptr(s), len(s), _ptr(k), len(k), _ptr(e), len(e),
                             _ptr(i), len(i), C.byref(params), C.byref(info)))
    return info.as_dict()


def arb_step(sim, n_steps: int):
    _check(load().arb_step(sim, int(n_steps)))


def arb_get_voltages(sim, dst, on_device: bool):
    _check(load().arb_get_voltages(sim, _ptr(dst), int(dst.numel() if hasattr(dst, "numel") else dst.size),
                                   1 if on_device else 0))


def arb_get_voltages_noalloc(sim, dst):
    _check(load().arb_get_voltages_noalloc(sim, _ptr(dst), int(dst.size)))


def arb_get_spikes(sim, cap: int):
    out = np.zeros(max(int(cap), 1), SPIKE)
    n = C.c_int64()
    _check(load().arb_get_spikes(sim, _ptr(out), int(cap), C.byref(n)))
    return out[: n.value]


def arb_set_probes(sim, cv, max_steps: int):
    cv = np.ascontiguousarray(cv, dtype=np.int64)
    _check(load().arb_set_probes(sim, _ptr(cv), len(cv), int(max_steps)))


def arb_get_trace(sim, dst, cap: int, on_device: bool) -> int:
    n = C.c_int64()
    _check(load().arb_get_trace(sim, _ptr(dst), int(cap), 1 if on_device else 0, C.byref(n)))
    return n.value


def arb_set_params(sim, theta):
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    _check(load().arb_set_params(sim, _ptr(th), len(th)))


def arb_grad_forward(sim, n_steps: int, ckpt_every: int, trace_dev):
    _check(load().arb_grad_forward(sim, int(n_steps), int(ckpt_every), _ptr(trace_dev)))


def arb_grad_backward(sim, dL_dtrace_dev, dL_dtheta_dev):
    _check(load().arb_grad_backward(sim, _ptr(dL_dtrace_dev), _ptr(dL_dtheta_dev)))


def arb_get_state(sim) -> bytes:
    L = load()
    n = C.c_int64()
    _check(L.arb_get_state(sim, None, 0, C.byref(n)))
    buf = np.zeros(n.value, np.uint8)
    _check(L.arb_get_state(sim, _ptr(buf), n.value, C.byref(n)))
    return buf


def arb_set_state(sim, blob):
    blob = np.ascontiguousarray(blob, dtype=np.uint8)
    _check(load().arb_set_state(sim, _ptr(blob), len(blob)))


def arb_get_info(sim) -> dict:
    info = arb_info()
    _check(load().arb_get_info(sim, C.byref(info)))
    return info.as_dict()


def arb_get_kernel_time(sim):
    ms, n = C.c_double(), C.c_int64()
    _check(load().arb_get_kernel_time(sim, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def arb_sync(sim):
    _check(load().arb_sync(sim))


def arb_free(sim):
    _check(load().arb_free(sim))


# ---------------------------------------------------------------------------
# marshalling of a column model (workloads.gen layout) into the ABI structs

def model_structs(m: dict):
    nc = len(m["cell_n_branch"])
    cells = np.zeros(nc, CELL)
    cells["branch_begin"] = m["cell_branch_begin"]
    cells["n_branch"] = m["cell_n_branch"]
    cells["soma_mech"] = m["soma_mech"]
    cells["soma_area_um2"] = m["soma_area"]
    cells["soma_gbar_na"] = m["soma_gna"]
    cells["soma_gbar_k"] = m["soma_gk"]
    cells["soma_gl_hh"] = m["soma_gl"]
    cells["soma_g_pas"] = m["soma_gpas"]
    cells["soma_e_pas"] = m["soma_epas"]
    cells["cm_uF_cm2"] = m["cm"]
    cells["Ra_ohm_cm"] = m["Ra"]
    br = np.zeros(len(m["br_parent"]), BRANCH)
    for f, g in (("parent", "br_parent"), ("n_cv", "br_n_cv"), ("length_um", "br_length"),
                 ("diam_um", "br_diam"), ("mech", "br_mech"), ("gbar_na", "br_gna"), ("gbar_k", "br_gk"),
                 ("gl_hh", "br_gl"), ("g_pas", "br_gpas"), ("e_pas", "br_epas")):
        br[f] = m[g]
    syn = np.zeros(len(m["syn_cell"]), SYNAPSE)
    syn["cell"], syn["branch"], syn["cv"] = m["syn_cell"], m["syn_branch"], m["syn_cv"]
    syn["tau_ms"], syn["e_rev_mV"] = m["syn_tau"], m["syn_e"]
    con = np.zeros(len(m["con_src"]), CONNECTION)
    con["src"], con["dst"], con["syn"] = m["con_src"], m["con_dst"], m["con_syn"]
    con["delay_steps"], con["w_uS"] = m["con_delay"], m["con_w"]
    ev = np.zeros(len(m["ev_syn"]), EVENT)
    ev["syn"], ev["step"], ev["w_uS"] = m["ev_syn"], m["ev_step"], m["ev_w"]
    ic = np.zeros(len(m["ic_cell"]), ICLAMP)
    ic["cell"], ic["branch"], ic["cv"] = m["ic_cell"], m["ic_branch"], m["ic_cv"]
    ic["step_on"], ic["step_off"], ic["amp_nA"] = m["ic_on"], m["ic_off"], m["ic_amp"]
    return cells, br, syn, con, ev, ic


class Simulation:
    """A sim built from a column model, with device memory from torch."""

    def __init__(self, m: dict, epoch_steps: int = 0, block_threads: int = 0, coef_mode: int = 0,
                 cells_per_pack: int = 0, flags: int = 0, spike_capacity: int = 0, event_capacity: int = 0, stream=None,
                 use_torch_allocator: bool = True, dry_run_ranks: int = 0, timed: bool | None = None):
        """timed: build for the variable time step (arb_build_cells_timed) with
        the model's continuous delays and event times (con_delay_ms, ev_t);
        None = when the model has them."""
        import torch
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p = arb_params()
        p.dt_ms, p.threshold_mV, p.v_init_mV = m["dt"], m["threshold"], m["v_init"]
        p.epoch_steps, p.flags = int(epoch_steps), int(flags)
        p.hip_stream = C.c_void_p(self.stream.cuda_stream)
        p.spike_capacity, p.event_capacity = int(spike_capacity), int(event_capacity)
        p.block_threads, p.coef_mode = int(block_threads), int(coef_mode)
        p.cells_per_pack = int(cells_per_pack)
        p.dry_run_ranks = int(dry_run_ranks)
        self._dens = density_structs(m.get("densities"))
        if self._dens is not None:
            p.densities = C.cast(self._dens, C.c_void_p)
            p.n_densities = len(self._dens)
        if use_torch_allocator:
            dev = self.stream.device
            st = self.stream

            def _alloc(n, ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(int(n), dev, st)
                except Exception:  # out of memory -> NULL -> ARB_ENOMEM
                    return None

            def _free(ptr, ctx):
                torch.cuda.caching_allocator_delete(ptr)

            self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
            p.alloc, p.free = self._cb
        self.params = p
        self.m = m
        if timed is None:
            timed = "con_delay_ms" in m and "ev_t" in m
        self.timed = bool(timed)
        cells, br, syn, con, ev, ic = model_structs(m)
        if self.timed:
            if len(ic):
                raise ValueError("the variable time step takes no current clamps")
            self.h = arb_build_cells_timed(cells, br, syn, con, m["con_delay_ms"], ev, m["ev_t"], p)
        else:
            self.h = arb_build_cells(cells, br, syn, con, ev, ic, p)
        self.info = arb_get_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            arb_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        arb_step(self.h, n)

    def voltages(self):
        out = self._torch.empty(self.info["n_cv"], dtype=self._torch.float64, device=self.stream.device)
        arb_get_voltages(self.h, out, True)
        return out

    def voltages_host(self):
        out = np.zeros(self.info["n_cv"])
        arb_get_voltages(self.h, out, False)
        return out

    def spikes(self, cap: int | None = None):
        return arb_get_spikes(self.h, cap if cap is not None else max(1 << 16, 64 * self.info["n_cells"]))

    def set_probes(self, cv, max_steps: int):
        self.n_probe = len(cv)
        arb_set_probes(self.h, cv, max_steps)

    def trace(self, cap: int):
        out = np.zeros((self.n_probe, cap))
        n = arb_get_trace(self.h, out, cap, False)
        return out[:, :n]

    def set_params(self, theta):
        arb_set_params(self.h, theta)

    def get_state(self):
        return arb_get_state(self.h)

    def set_state(self, blob):
        arb_set_state(self.h, blob)

    def kernel_time(self):
        return arb_get_kernel_time(self.h)

    def sync(self):
        arb_sync(self.h)

    def step_count(self) -> int:
        return arb_get_step_count(self.h)

    def mechanism_instances(self) -> dict:
        """Instances of each generated mechanism in the sim, by name."""
        cat = mechanism_catalogue()
        counts = (C.c_int64 * max(len(cat), 1))()
        _check(load().arb_get_mechanism_instances(self.h, counts, len(cat)))
        return {m["name"]: int(counts[m["id"]]) for m in cat}

    def refresh_info(self):
        self.info = arb_get_info(self.h)
        return self.info
