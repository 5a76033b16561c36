"""The C ABI library loads, exports every declared symbol, its structs match
the binding's layouts, and host-side validation rejects bad models (no GPU
needed: validation runs before any device call)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1901_07454_amd import arbmi
from tests import models
from workloads import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "arbmi.h")


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_library_exports_every_declared_symbol():
    lib = arbmi.load()
    declared = set(re.findall(r"\b(arb_[a-z_]+)\s*\(", open(HDR).read()))
    assert declared >= {"arb_build_cells", "arb_step", "arb_get_voltages", "arb_get_spikes"}
    for name in declared:
        assert hasattr(lib, name), name
    assert set(arbmi.EXPORTS) == declared


def test_struct_layouts_match_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "arbmi.h"\n'
                    '#define S(t) printf(#t " %zu\\n", sizeof(t));\n'
                    '#define O(t,f) printf(#t "." #f " %zu\\n", offsetof(t,f));\n'
                    "int main(void){S(arb_branch)S(arb_cell)S(arb_synapse)S(arb_connection)S(arb_event)"
                    "S(arb_iclamp)S(arb_spike)S(arb_params)S(arb_info)"
                    "O(arb_branch,gbar_na)O(arb_cell,soma_area_um2)O(arb_params,hip_stream)"
                    "O(arb_params,spike_capacity)O(arb_params,coef_mode)O(arb_info,bytes_per_step)O(arb_info,reg_len)O(arb_info,syn_hbm)return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                              check=True).stdout.split("\n") if line)
    got = {k: int(v) for k, v in got.items()}
    assert got["arb_branch"] == arbmi.BRANCH.itemsize
    assert got["arb_cell"] == arbmi.CELL.itemsize
    assert got["arb_synapse"] == arbmi.SYNAPSE.itemsize
    assert got["arb_connection"] == arbmi.CONNECTION.itemsize
    assert got["arb_event"] == arbmi.EVENT.itemsize
    assert got["arb_iclamp"] == arbmi.ICLAMP.itemsize
    assert got["arb_spike"] == arbmi.SPIKE.itemsize
    assert got["arb_params"] == ctypes.sizeof(arbmi.arb_params)
    assert got["arb_info"] == ctypes.sizeof(arbmi.arb_info)
    assert got["arb_branch.gbar_na"] == arbmi.BRANCH.fields["gbar_na"][1]
    assert got["arb_cell.soma_area_um2"] == arbmi.CELL.fields["soma_area_um2"][1]
    assert got["arb_params.hip_stream"] == arbmi.arb_params.hip_stream.offset
    assert got["arb_params.spike_capacity"] == arbmi.arb_params.spike_capacity.offset
    assert got["arb_params.coef_mode"] == arbmi.arb_params.coef_mode.offset
    assert got["arb_info.bytes_per_step"] == arbmi.arb_info.bytes_per_step.offset
    assert got["arb_info.reg_len"] == arbmi.arb_info.reg_len.offset
    assert got["arb_info.syn_hbm"] == arbmi.arb_info.syn_hbm.offset


def _params(**kw):
    p = arbmi.arb_params()
    p.dt_ms, p.threshold_mV, p.v_init_mV = 0.025, -10.0, -65.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _build(m, **kw):
    return arbmi.arb_build_cells(*arbmi.model_structs(m), _params(**kw))


def _expect_einval(m, text, **kw):
    with pytest.raises(arbmi.ArbError) as e:
        _build(m, **kw)
    assert e.value.code == arbmi.ARB_EINVAL, str(e.value)
    assert text in str(e.value)


def _ring():
    return gen.config2(n_cells=3, n_steps=10)


def test_rejects_bad_parent():
    m = _ring()
    m["br_parent"] = m["br_parent"].copy()
    m["br_parent"][5] = 9
    _expect_einval(m, "parent")


def test_rejects_zero_cvs_and_bad_geometry():
    m = _ring()
    m["br_n_cv"] = m["br_n_cv"].copy()
    m["br_n_cv"][3] = 0
    _expect_einval(m, "n_cv")
    m = _ring()
    m["br_diam"] = m["br_diam"].copy()
    m["br_diam"][0] = 0.0
    _expect_einval(m, "diameter")
    m = _ring()
    m["soma_area"] = m["soma_area"].copy()
    m["soma_area"][1] = -1.0
    _expect_einval(m, "soma area")
    m = _ring()
    m["br_gpas"] = m["br_gpas"].copy()
    m["br_gpas"][2] = np.nan
    _expect_einval(m, "not finite")


def test_rejects_bad_synapses_and_connections():
    m = _ring()
    m["syn_cv"] = m["syn_cv"].copy()
    m["syn_cv"][4] = 99
    _expect_einval(m, "synapse 4")
    m = _ring()
    m["con_delay"] = m["con_delay"].copy()
    m["con_delay"][0] = 0
    _expect_einval(m, "delay_steps")
    m = _ring()
    m["con_syn"] = m["con_syn"].copy()
    m["con_syn"][0] = 10  # a synapse of cell 1, but connection 0 ends on cell 0
    _expect_einval(m, "destination")
    m = _ring()
    m["ev_syn"] = m["ev_syn"].copy()
    m["ev_syn"][0] = 10_000
    _expect_einval(m, "event 0")
    m = _ring()
    m["ic_cell"], m["ic_branch"], m["ic_cv"] = np.array([0], np.int32), np.array([-1], np.int32), np.array([1], np.int32)
    m["ic_on"], m["ic_off"], m["ic_amp"] = np.array([0]), np.array([5]), np.array([0.1])
    _expect_einval(m, "clamp 0")


def test_rejects_epoch_longer_than_min_delay():
    _expect_einval(_ring(), "minimum delay", epoch_steps=201)


def test_rejects_bad_launch_parameters():
    _expect_einval(_ring(), "block_threads", block_threads=96)
    _expect_einval(_ring(), "coef_mode", coef_mode=4)


def test_dry_run_sources_and_limits():
    """Dry-run mode accepts connection sources among ranks x cells gids
    only, and at most 2^20 ranks."""
    m = gen.config7_dry_run(n_cells=6, ranks=4, n_steps=10, n_syn=20)
    assert int(m["con_src"].max()) >= 6
    assert _plan(m, dry_run_ranks=4)["n_conn"] == 120
    with pytest.raises(arbmi.ArbError) as e:
        _plan(m)  # sources beyond the cells without a dry run
    assert e.value.code == arbmi.ARB_EINVAL and "connection" in str(e.value)
    with pytest.raises(arbmi.ArbError) as e:
        _plan(m, dry_run_ranks=(1 << 20) + 1)
    assert "dry_run_ranks" in str(e.value)


def test_gradient_layouts():
    """Sims built for gradients take the register layout when its packs also
    fit the adjoint kernel; a cell whose synapses would have to stay in HBM
    (the adjoint reads them from LDS) falls back to streamed coefficients, or
    is refused when the register layout was asked for."""
    G = arbmi.ARB_FLAG_GRADIENTS
    assert _plan(gen.config4(n_cells=4, n_steps=100), flags=G)["coef_mode"] == 3
    assert _plan(gen.config2(n_cells=4, n_steps=100), flags=G)["coef_mode"] == 3
    m = gen.config6(n_cells=4, n_steps=100, n_syn=2000)
    assert _plan(m)["syn_hbm"] == 1
    assert _plan(m, flags=G)["coef_mode"] == 2
    with pytest.raises(arbmi.ArbError) as e:
        _plan(m, flags=G, coef_mode=3)
    assert e.value.code == arbmi.ARB_EINVAL


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device error path")
def test_valid_model_without_device_reports_hip_error():
    with pytest.raises(arbmi.ArbError) as e:
        _build(_ring())
    assert e.value.code == arbmi.ARB_EHIP


def test_null_sim_handles_are_rejected():
    lib = arbmi.load()
    assert lib.arb_step(None, 1) == arbmi.ARB_EINVAL
    assert lib.arb_free(None) == arbmi.ARB_OK
    n = ctypes.c_int64()
    assert lib.arb_get_spikes(None, None, 0, ctypes.byref(n)) == arbmi.ARB_EINVAL


def test_rejects_lds_resident_coefficients_for_a_huge_cell():
    big = [i for i in range(40) if 1 + gen.cell_c3(i, 10.0).n_cv.sum() > 4000][:1]
    m = gen.config3(cells=big, n_steps=10)
    _expect_einval(m, "LDS", coef_mode=1)


def _plan(m, **kw):
    return arbmi.arb_plan_layout(*arbmi.model_structs(m), _params(**kw))


@pytest.mark.parametrize("mode,T", [(0, 0), (1, 64), (2, 128), (2, 256), (3, 64), (3, 128), (3, 256)])
def test_plan_layout_invariants_ring(mode, T):
    m = gen.config2(n_cells=40, n_steps=10)
    info = _plan(m, coef_mode=mode, block_threads=T)
    assert info["n_cv"] == 40 * 1017
    assert info["n_slots"] >= info["n_cv"]
    assert info["lds_bytes"] <= 160 * 1024 - 256
    if mode in (0, 3):
        assert info["coef_mode"] == 3
        # every branch gets reg_len rows: the 8-CV branches of the full
        # binary trees fill theirs, each 1-CV soma leaves 7 spare
        assert info["reg_len"] == 8
        assert info["n_slots"] == info["n_cv"] + 40 * 7


@pytest.mark.parametrize("mode,T", [(0, 0), (2, 64), (2, 256), (3, 128), (3, 256)])
def test_plan_layout_invariants_uneven_and_networks(mode, T):
    for m in (gen.config3(n_cells=30, n_steps=10), gen.config5(n_cells=20, n_in=6, n_steps=10),
              gen.config4(n_cells=9, n_steps=10), gen.config1()):
        try:
            info = _plan(m, coef_mode=mode, block_threads=T)
        except arbmi.ArbError as e:
            # an explicit register layout may not hold every cell, in its
            # registers or in LDS
            assert mode == 3 and e.code == arbmi.ARB_EINVAL and ("register" in str(e) or "LDS" in str(e))
            continue
        assert info["n_cv"] == int(gen.n_cvs(m).sum())
        assert info["lds_bytes"] <= 160 * 1024 - 256


def test_plan_register_layout_holds_the_largest_uneven_cells():
    """The 4096 uneven cells in the register layout at 256 threads x 3 slots:
    the largest (up to 4990 CVs) exceed LDS with their hh conductances there,
    so their packs keep those in HBM (reported as syn_hbm), and every pack
    fits the device's LDS."""
    m = gen.config3(n_steps=10)
    info = _plan(m, coef_mode=3, block_threads=256)
    assert info["coef_mode"] == 3 and info["reg_slots"] == 3 and info["reg_len"] == 8
    assert info["syn_hbm"] == 1
    assert info["lds_bytes"] <= 160 * 1024 - 256
    assert info["n_cv"] == int(gen.n_cvs(m).sum())
    small = gen.config3(cells=[0, 1, 2], n_steps=10)
    assert _plan(small, coef_mode=3, block_threads=256)["syn_hbm"] == 0


def test_plan_cuts_long_branches_into_register_segments():
    m = gen.config1()  # 32-CV branches do not fit 16 registers
    assert _plan(m)["coef_mode"] == 2  # the default keeps the streamed layout for them
    info = _plan(m, coef_mode=3)  # on request: chains of four 8-CV segments
    assert info["coef_mode"] == 3 and info["reg_len"] == 8
    assert info["n_slots"] == 8 * (1 + 4 * 4)  # soma + 16 segments, 8 rows each


def test_plan_register_layout_for_full_ring_packs_four_cells():
    m = gen.config2(n_cells=64, n_steps=10)
    info = _plan(m, coef_mode=3, block_threads=256)
    assert info["n_packs"] == 16  # 4 cells of 128 branch tasks fill 256 threads x 2 slots


def test_plan_network_epochs_at_most_16384_steps():
    """A network's epoch is its minimum delay, at most 16,384 steps (the event
    pull keeps one LDS counter per step of the epoch)."""
    cells = [models.bare_cell([], [], [], []) for _ in range(2)]
    for k, d in enumerate(cells):
        d.syn.append((-1, 0, 2.0, 0.0))
        d.in_conn.append((1 - k, 0, 20000, 0.01))
    m = gen.assemble(cells, n_steps=10)
    assert _plan(m)["epoch_steps"] == 16384
    cells[0].in_conn[0] = (1, 0, 300, 0.01)
    assert _plan(gen.assemble(cells, n_steps=10))["epoch_steps"] == 300


def test_plan_cells_with_many_inputs_get_a_pack_each():
    """Packs of several cells hold at most 4096 incoming connections; a cell
    with more takes a pack of its own."""
    m = gen.config7(n_cells=8, n_syn=5000, n_steps=10)
    assert _plan(m, coef_mode=3, block_threads=128)["n_packs"] == 8
    m = gen.config7(n_cells=8, n_syn=500, n_steps=10)
    assert _plan(m, coef_mode=3, block_threads=128)["n_packs"] < 8


def test_plan_segments_are_balanced_chains():
    """A 100-CV branch in the register layout: ceil(100 / 8) = 13 segments of
    7 or 8 CVs (nearly equal), each given 8 register rows, plus the soma."""
    m = gen.assemble([models.bare_cell([-1], [100], [900.0], [2.0])], n_steps=10)
    info = _plan(m, coef_mode=3, block_threads=64)
    assert info["coef_mode"] == 3 and info["reg_len"] == 8
    assert info["n_cv"] == 101 and info["n_slots"] == 8 * (1 + 13)
    assert _plan(m)["coef_mode"] == 2  # not chosen by default for such branches


def _build_timed(m, **kw):
    cells, br, syn, con, ev, _ = arbmi.model_structs(m)
    return arbmi.arb_build_cells_timed(cells, br, syn, con, m["con_delay_ms"], ev, m["ev_t"], _params(**kw))


def _expect_timed_einval(m, text, **kw):
    with pytest.raises(arbmi.ArbError) as e:
        _build_timed(m, **kw)
    assert e.value.code == arbmi.ARB_EINVAL, str(e.value)
    assert text in str(e.value)


def test_timed_build_validation():
    """The variable-step build checks its continuous inputs and refuses
    what it does not run: delays below dt, event times out of range,
    gradients, the dry run, current clamps (the timed call takes none) and an
    epoch longer than the shortest delay (K dt <= min delay, in grid steps)."""
    m = gen.config2_timed(n_cells=3, t_ms=5.0)
    bad = dict(m, con_delay_ms=m["con_delay_ms"].copy())
    bad["con_delay_ms"][1] = 0.01
    _expect_timed_einval(bad, "delay_ms")
    bad = dict(m, ev_t=m["ev_t"].copy())
    bad["ev_t"][0] = -1e-9
    _expect_timed_einval(bad, "time out of range")
    bad["ev_t"][0] = float("nan")
    _expect_timed_einval(bad, "time out of range")
    _expect_timed_einval(m, "gradients", flags=arbmi.ARB_FLAG_GRADIENTS)
    _expect_timed_einval(m, "dry-run", dry_run_ranks=2)
    # epochs of at most K grid steps, K dt <= the shortest delay
    K = int(np.floor(m["con_delay_ms"].min() / gen.DT))
    while (K + 1) * gen.DT <= m["con_delay_ms"].min():
        K += 1
    _expect_timed_einval(m, "minimum delay", epoch_steps=K + 1)
    with pytest.raises(ValueError):
        arbmi.arb_build_cells_timed(*arbmi.model_structs(m)[:4], m["con_delay_ms"][:1], arbmi.model_structs(m)[4],
                                    m["ev_t"], _params())


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device error path")
def test_timed_build_valid_model_reaches_the_device_step():
    """A valid timed model passes validation and lowering (one cell per
    workgroup, register layout) and fails only for want of a device."""
    with pytest.raises(arbmi.ArbError) as e:
        _build_timed(gen.config2_timed(n_cells=3, t_ms=5.0))
    assert e.value.code == arbmi.ARB_EHIP
    with pytest.raises(arbmi.ArbError) as e:  # block_threads honoured
        _build_timed(gen.config2_timed(n_cells=3, t_ms=5.0), block_threads=128)
    assert e.value.code == arbmi.ARB_EHIP


def test_density_validation():
    """Generated density mechanisms: entries are checked (cell, branch,
    mechanism, parameter count, finite values), and refused with gradients,
    the variable time step and layouts other than the register-resident one."""
    m = gen.config2_mech(n_cells=2, n_steps=10)

    def expect(mm, text, **kw):
        with pytest.raises(arbmi.ArbError) as e:
            _build(mm, **kw)
        assert e.value.code == arbmi.ARB_EINVAL and text in str(e.value), str(e.value)

    def bad(**change):
        d = arbmi.density_structs(m["densities"][:1])
        for k, v in change.items():
            setattr(d[0], k, v)
        return d

    def build_with(d, **kw):
        p = _params(**kw)
        p.densities = ctypes.cast(d, ctypes.c_void_p)
        p.n_densities = len(d)
        return arbmi.arb_build_cells(*arbmi.model_structs(m), p)

    for change, text in (({"cell": 5}, "out of range"), ({"branch": 999}, "out of range"),
                         ({"mech": 99}, "unknown mechanism"), ({"n_param": 9}, "parameters")):
        with pytest.raises(arbmi.ArbError) as e:
            build_with(bad(**change))
        assert text in str(e.value), str(e.value)
    d = bad()
    d[0].param[0] = float("nan")
    with pytest.raises(arbmi.ArbError) as e:
        build_with(d)
    assert "not finite" in str(e.value)
    for kw, text in (({"flags": arbmi.ARB_FLAG_GRADIENTS}, "gradients"), ({"coef_mode": 1}, "register layout")):
        with pytest.raises(arbmi.ArbError) as e:
            build_with(arbmi.density_structs(m["densities"]), **kw)
        assert text in str(e.value), str(e.value)
