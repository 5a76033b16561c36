"""Benchmark: CV-updates/s of the multi-compartment cell stepper on one MI355X.

A "step" is one time step dt of every cell: event delivery, hh/pas/expsyn
currents, implicit-Euler assembly, Hines solve, state update, threshold
detection, and (every epoch) the spike exchange.  The default workload is the
8192-cell ring (random-geometry depth-6 binary trees, 1017 CVs per cell,
8,331,264 CVs, hh soma, passive dendrites, 10 expsyn per cell, ring delay
5 ms, dt 0.025 ms), timed over 4000 steps (100 ms of model time) after a
warm-up epoch.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `--config 3|4|5|1` selects the other workloads,
`--config 6` the synapse-dominated ring (10,000 expsyn per cell) and
`--config 7` the 10k-connectivity model.  `--varstep` runs the ring with the
variable time step (Sec. II: steps shortened at event times): off-grid ring
delays U(5, 5.5) ms, kicks at U(0, 1) ms and 10 Hz Poisson input on every
dendritic synapse at continuous times; its rate counts n_cv CV-updates per
grid step (the shortened steps taken on top are reported beside it).
`--mech` runs the ring's cells with generated density mechanisms (Sec.
III-C): hcn on every soma, kdr on every dendritic branch, the generated hh on
branch 0, each soma kicked every 10 ms.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64

# Algorithmic FP64 operations per step (a transcendental or a division counts
# as one): a CV's assembly (alpha V + R), elimination and substitution with
# the step-invariant factorisation take 7; an hh instance's current (14), six
# rates (26) and three gate updates (21) take 61; an expsyn's current and
# decay take 4.
FLOPS_PER_CV, FLOPS_PER_HH, FLOPS_PER_SYN = 7, 61, 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_model(cfg: int, n_cells: int | None, ranks: int = 1):
    from workloads import gen
    if cfg == 1:
        return gen.config1(), "1 cell, 129 CVs (hh soma + 4x32 pas), 1 expsyn, 10 input events"
    if cfg == 2:
        n = n_cells or 8192
        return gen.config2(n_cells=n), (f"{n}-cell ring, depth-6 binary trees x 8 CVs/branch (1017 CVs/cell), "
                                        "hh soma, pas dendrites, 10 expsyn/cell, delay 5 ms")
    if cfg == 3:
        n = n_cells or 4096
        return gen.config3(n_cells=n), (f"{n} uneven Yule-tree cells, CVs log-uniform in [50, 5000], "
                                        "hh soma + 25% hh branches, 20 expsyn/cell, 10 Hz Poisson input")
    if cfg == 5:
        n = n_cells or 65536
        return gen.config5(n_cells=n), (f"{n} Yule-tree cells x 1497 CVs, 100 random incoming connections "
                                        "(delay 5-10 ms) + 5 Hz background per cell")
    if cfg == 4:
        n = n_cells or 256
        return gen.config4(n_cells=n), f"{n} cells x 200 CVs, hh+pas everywhere, soma clamp 0.2 nA"
    if cfg == 6:
        n = n_cells or 8192
        return gen.config6(n_cells=n), (f"{n}-cell synapse-dominated ring, random trees of 90-170 CVs (mean 130), "
                                        "hh soma, pas dendrites, 10,000 expsyn/cell (one on the ring), delay 5 ms")
    if cfg == 7 and ranks > 1:
        n = n_cells or 8192
        return gen.config7_dry_run(n_cells=n, ranks=ranks), (
            f"dry run of the 10k-connectivity model: one rank of {n} cells (the cells of config 6) in {ranks} "
            f"identical ranks, every synapse wired from a random gid of all {ranks * n} cells (delay 20 ms), "
            "remote spikes as proxies of the local cells, all cells driven to fire together at 50 Hz")
    if cfg == 7:
        n = n_cells or 8192
        return gen.config7(n_cells=n), (f"{n}-cell 10k-connectivity model: the cells of config 6, every synapse "
                                        "wired from a random other cell (delay 20 ms), all cells driven to fire "
                                        "together at 50 Hz")
    raise SystemExit(f"unknown config {cfg}")


def copy_bandwidth_gbps(torch) -> float:
    """Device-to-device copy rate of a 2 GiB buffer (read + write bytes)."""
    n = 1 << 28
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del a, b
    return 2 * 8 * n * reps / dt / 1e9


def _oracle_chunk(args):
    cfg, cells, steps = args
    import oracle
    from workloads import gen
    if cfg == "2t":  # the timed ring, the oracle's variable step
        m = gen.config2_timed(cells=cells, t_ms=VARSTEP_T_MS)
        s = oracle.Sim(m).set_varstep()
        t0 = time.perf_counter()
        s.advance_to(steps)
        dt = time.perf_counter() - t0
        return int(gen.n_cvs(m).sum()) * steps, dt
    if cfg == "2m":
        m = gen.config2_mech(n_cells=8192, cells=cells, n_steps=steps + 1)
    elif cfg == 2:
        m = gen.config2(n_cells=8192, cells=cells)
    elif cfg == 3:
        m = gen.config3(cells=cells)
    elif cfg == 5:
        m = gen.config5(n_cells=65536, cells=cells)
    elif cfg == 4:
        m = gen.config4(cells=cells)
    elif cfg == 6:
        m = gen.config6(n_cells=8192, cells=cells)
    elif cfg == 7:
        m = gen.config7(n_cells=8192, cells=cells)
    else:
        m = gen.config1()
    s = oracle.Sim(m)
    t0 = time.perf_counter()
    s.run(steps)
    dt = time.perf_counter() - t0
    return int(gen.n_cvs(m).sum()) * steps, dt


def host_cpu():
    """Host cores this process may use, the machine's count and the CPU model."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return usable, os.cpu_count() or 1, model


# Host cores one GPU's share of the box provides: the CPU oracle's process
# pool never exceeds it.
HOST_CORES_PER_GPU = 16

# The oracle's workload per configuration: (cells, steps) of the parallel leg
# (the whole model where its rate allows a run of about 10-30 s) and of the
# single-thread leg.
CPU_LEGS = {1: ((1, 4000), (1, 4000)), 2: ((8192, 4000), (64, 4000)), 3: ((4096, 8000), (16, 8000)),
            4: ((256, 2000), (64, 2000)), 5: ((65536, 800), (16, 800)), 6: ((8192, 800), (16, 800)),
            7: ((8192, 800), (16, 800)), "2t": ((8192, 4000), (64, 4000)), "2m": ((8192, 800), (16, 800))}
CPU_BASE_CELLS = {1: 1, 2: 8192, 3: 4096, 4: 256, 5: 65536, 6: 8192, 7: 8192, "2t": 8192, "2m": 8192}
# model time of the timed ring's inputs (the benchmark's steps and warm-up fit)
VARSTEP_T_MS = 200.0


def cpu_baseline(cfg):
    """The CPU oracle as it stands (single-threaded C, built -O2 without
    fast-math), timed twice on the same workload as the GPU: on every usable
    host core (up to one GPU's share), as independent processes over disjoint
    contiguous chunks of the cells, and on one core.  Only the stepping loop
    is timed; the rate is CV-updates / stepping time (summed over processes
    for the parallel leg)."""
    import multiprocessing as mp

    import oracle
    oracle.build() if not os.path.exists(oracle.LIB) else None
    usable, nproc, model = host_cpu()
    workers = max(1, min(HOST_CORES_PER_GPU, usable))
    (n_cells, steps), (n1, steps1) = CPU_LEGS[cfg]
    base = CPU_BASE_CELLS[cfg]
    if cfg == 1:
        chunks = [(1, [0], steps) for _ in range(workers)]
    else:
        per = (n_cells + workers - 1) // workers
        chunks = [(cfg, list(range(w * per, min(n_cells, (w + 1) * per))), steps) for w in range(workers)
                  if w * per < n_cells]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(chunks)) as pool:
        res = pool.map(_oracle_chunk, chunks)
    wall = time.perf_counter() - t0
    rate = sum(u / t for u, t in res)
    cpu_s = sum(t for _, t in res)
    u1, t1 = _oracle_chunk((cfg, list(range(min(n1, base))), steps1))
    whole = "the whole model" if n_cells >= base else f"cells 0-{n_cells - 1} of {base}"
    return {"value": rate, "unit": "CV-updates/s", "cores": len(chunks), "kind": "oracle",
            "single_thread": {"value": u1 / t1, "unit": "CV-updates/s", "cells": min(n1, base), "steps": steps1},
            "nproc": nproc, "usable_cores": usable, "cpu_model": model,
            "sample": (f"{whole} x {steps} steps, split into {len(chunks)} contiguous cell chunks run as "
                       f"independent processes (connections between chunks dropped), stepping time only; "
                       f"{cpu_s:.1f} s CPU, {wall:.1f} s wall; pool capped at {HOST_CORES_PER_GPU} cores, "
                       f"one GPU's share of the host")}


def kernel_name(info: dict, timed: bool = False, generated: bool = False) -> str:
    if timed:
        return f"var_step_kernel<{info['block_threads']}, {info['reg_slots']}, {info['reg_len']}>"
    if generated:  # the variant with generated mechanisms (state in LDS, no recording)
        return f"reg_step_kernel<{info['block_threads']}, {info['reg_slots']}, {info['reg_len']}, false, false, true>"
    if info["coef_mode"] == 3:
        return (f"reg_step_kernel<{info['block_threads']}, {info['reg_slots']}, {info['reg_len']}, "
                f"{'true' if info['syn_hbm'] else 'false'}>")
    return f"step_kernel<{info['block_threads']}, {'true' if info['coef_mode'] == 1 else 'false'}>"


def measured_traffic(path: str, cfg: int, kernel: str, steps_per_launch: float):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, if it was taken on this kernel variant with the kernel
    sources unchanged since; else None.  The summary holds a fixed part per
    launch (loading and storing the packs' state) and a part per step, fitted
    from launches of two lengths, so any launch length gets a figure."""
    try:
        rec = json.load(open(path))[f"config{cfg}"]
        if _sources_sha(rec["kernel_sources"]) != rec["kernel_sha256"] or rec["kernel"] != kernel:
            return None
        return rec["fixed_bytes_per_launch"] + rec["bytes_per_step"] * steps_per_launch
    except Exception:
        return None


# The sources a step kernel's traffic depends on (a recorded figure holds
# while their hash is unchanged).
CSRC = "paper_1901_07454_amd/csrc/"
KERNEL_SOURCES = {
    "reg": [CSRC + f for f in ("reg_kernels.hip", "reg_solve.hpp", "kernel_common.hpp", "layout.hpp",
                               "kernels.hpp", "fastexp.hpp", "gen/mechanisms.hpp", "gen/mechanisms_desc.hpp")],
    "var": [CSRC + f for f in ("var_kernels.hip", "var_kernels.hpp", "reg_solve.hpp", "kernel_common.hpp",
                               "layout.hpp", "kernels.hpp", "fastexp.hpp")],
}


def _sources_sha(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def _counter_rows(path: str):
    import csv
    return list(csv.DictReader(open(path)))


def fit_traffic(run_dir: str, key: str, kernel: str, family: str, out_path: str) -> dict:
    """Fit the HBM traffic of one workload's step kernels from rocprofv3
    counter runs of the benchmark at two epoch lengths.  run_dir holds, per
    epoch length K, `fetch_K<K>/` and `write_K<K>/` (the `--pmc FETCH_SIZE`
    and `--pmc WRITE_SIZE` runs, csv output) and `bench_K<K>.json` (the
    benchmark's line, for the number of epochs run).  Per epoch, the step
    kernels' dispatches (every launch class) are summed; the counters are
    scaled by what they read for the benchmark's 2 GiB device copy (FETCH_SIZE
    and WRITE_SIZE in KiB per dispatch against 2 GiB read and written);
    bytes per epoch = fixed + per_step K is solved from the two lengths.  The
    record is written into out_path (JSON) under `key`."""
    import glob
    pts, scales = {}, {"FETCH_SIZE": [], "WRITE_SIZE": []}
    for bj in sorted(glob.glob(os.path.join(run_dir, "bench_K*.json"))):
        K = int(re.search(r"bench_K(\d+)\.json", bj).group(1))
        line = json.loads([ln for ln in open(bj).read().splitlines() if ln.startswith("{")][-1])
        epochs = (line["steps"] + line["warmup"]) // K
        kib = {}
        for ctr, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
            rows = _counter_rows(glob.glob(os.path.join(run_dir, f"{sub}_K{K}", "**", "*counter_collection.csv"),
                                           recursive=True)[0])
            step = sum(float(r["Counter_Value"]) for r in rows
                       if r["Counter_Name"] == ctr and "step_kernel" in r["Kernel_Name"])
            copies = sorted((float(r["Counter_Value"]) for r in rows
                             if r["Counter_Name"] == ctr and "copyBuffer" in r["Kernel_Name"]), reverse=True)[:10]
            scales[ctr].append(2097152.0 / float(np.median(copies)))
            kib[ctr] = step / epochs
        pts[K] = kib
    (k1, p1), (k2, p2) = sorted(pts.items())[:2]
    sf, sw = float(np.median(scales["FETCH_SIZE"])), float(np.median(scales["WRITE_SIZE"]))
    b1 = 1024.0 * (p1["FETCH_SIZE"] * sf + p1["WRITE_SIZE"] * sw)
    b2 = 1024.0 * (p2["FETCH_SIZE"] * sf + p2["WRITE_SIZE"] * sw)
    per_step = (b2 - b1) / (k2 - k1)
    rec = {"kernel": kernel, "epoch_lengths": [k1, k2],
           "fetch_kib_per_epoch": [p1["FETCH_SIZE"], p2["FETCH_SIZE"]],
           "write_kib_per_epoch": [p1["WRITE_SIZE"], p2["WRITE_SIZE"]],
           "fetch_scale": sf, "write_scale": sw,
           "fixed_bytes_per_launch": b1 - per_step * k1, "bytes_per_step": per_step,
           "kernel_sources": KERNEL_SOURCES[family], "kernel_sha256": _sources_sha(KERNEL_SOURCES[family])}
    try:
        allrec = json.load(open(out_path))
    except Exception:
        allrec = {}
    allrec[key] = rec
    with open(out_path, "w") as f:
        json.dump(allrec, f, indent=1, sort_keys=True)
        f.write("\n")
    return rec


def grad_ratio(torch, reps: int = 3, subset: bool = False):
    """Wall time of the forward+adjoint gradient (checkpoints every 100 steps,
    through the autograd wrapper) over the wall time of the plain forward of
    the same model on the same GPU, built as the plain benchmark builds it
    (autotuned launch shape, no gradient flag).  Config 4 (256 cells x 200
    CVs, 2000 steps, loss: soma traces against zero), or with subset the
    1024-cell subset of the 65536-cell network (800 steps, network input as
    fixed events, loss: soma traces against -65 mV)."""
    from paper_1901_07454_amd import arbmi, grad
    from workloads import gen
    k = 100
    if subset:
        n_steps = 800
        m0 = gen.config5_subset(n_steps=n_steps)
        regions = grad_regions(m0)
        workload = ("1024-cell subset of the 65536-cell network: 1497 CVs per cell, network input as fixed "
                    "events, 800 steps (20 ms), checkpoint every 100")
        v_target = -65.0
    else:
        n_steps = 2000
        m0 = gen.config4(n_steps=n_steps)
        regions = gen.config4_theta(m0)
        workload = "config 4: 256 cells x 200 CVs, hh+pas, 2000 steps, checkpoint every 100"
        v_target = 0.0
    plain = arbmi.Simulation(m0, flags=arbmi.ARB_FLAG_AUTOTUNE)
    plain_state0 = plain.get_state()
    gs = grad.GradSim(m0, flags=arbmi.ARB_FLAG_AUTOTUNE)
    theta = torch.tensor(regions, dtype=torch.float64, device="cuda", requires_grad=True)
    target = torch.full((gs.n_cells, n_steps), v_target, dtype=torch.float64, device="cuda")

    def fwd():
        plain.set_state(plain_state0)
        plain.step(n_steps)
        plain.sync()

    def fwd_adj():
        th = theta.detach().clone().requires_grad_(True)
        tr = grad.soma_trace(th, gs, n_steps, k)
        loss = torch.mean((tr - target) ** 2)
        loss.backward()
        torch.cuda.synchronize()
        return th.grad

    fwd()
    fwd_adj()
    t_f, t_fa = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fwd()
        t_f.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        fwd_adj()
        t_fa.append(time.perf_counter() - t0)
    kp, kg = kernel_name(plain.info), kernel_name(gs.sim.info)
    gs.close()
    plain.close()
    f, fa = min(t_f), min(t_fa)
    return {"workload": workload,
            "fwd_ms": f * 1e3, "fwd_adj_ms": fa * 1e3, "ratio": fa / f, "target_ratio": 4.0,
            "fwd_kernel": kp, "grad_sim_kernel": kg,
            "note": "fwd: the plain benchmark's sim (autotuned, no gradient flag); fwd_adj: the gradient sim"}


def grad_regions(m: dict):
    """Per-region (soma, then branches, per cell) [gNa, gK, g_pas] of a model,
    flat [regions, 3]."""
    out = []
    b = 0
    for c, nb in enumerate(m["cell_n_branch"]):
        out.append((m["soma_gna"][c], m["soma_gk"][c], m["soma_gpas"][c]))
        for q in range(int(nb)):
            out.append((m["br_gna"][b + q], m["br_gk"][b + q], m["br_gpas"][b + q]))
        b += int(nb)
    return np.array(out, dtype=np.float64)


def dry_run_sweep(m: dict, ranks_list, K: int, epochs: int = 3):
    """The 10k-connectivity model's rank of cells at each rank count (only
    the connection sources change): wall time per epoch of direct launches
    after a warm-up epoch, the step kernel's share from HIP events, and the
    rest (spike collection, the source index over ranks x cells gids, the
    event pull, launch gaps) per epoch."""
    import torch

    from paper_1901_07454_amd import arbmi
    from workloads import gen
    n = len(m["cell_n_branch"])
    n_syn = len(m["con_src"]) // n
    rows = []
    for r in ranks_list:
        mm = dict(m)
        mm["con_src"] = gen.config7_dry_run_sources(n, r, n_syn)
        sim = arbmi.Simulation(mm, flags=arbmi.ARB_FLAG_TIME_KERNELS | arbmi.ARB_FLAG_AUTOTUNE, dry_run_ranks=r)
        sim.step(K)
        sim.sync()
        sim.kernel_time()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(epochs * K)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms, _ = sim.kernel_time()
        sim.sync()
        sp = len(sim.spikes())
        info = sim.info
        sim.close()
        rows.append({"ranks": r, "source_gids": r * n, "cv_updates_per_s": info["n_cv"] * epochs * K / wall,
                     "ms_per_epoch": wall * 1e3 / epochs, "step_kernel_ms_per_epoch": kms / epochs,
                     "exchange_and_gaps_ms_per_epoch": (wall * 1e3 - kms) / epochs,
                     "local_spikes": sp, "indexed_spikes_per_epoch": sp * r / (epochs + 1)})
        log(f"dry run, {r} ranks: {rows[-1]}")
    return {"model": "config 7 rank of %d cells, 10,000 synapses each, sources among ranks x cells gids" % n,
            "epoch_steps": K, "epochs_timed": epochs, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--cells", type=int, default=None)
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--coef-mode", type=int, default=0)
    ap.add_argument("--cells-per-pack", type=int, default=0)
    ap.add_argument("--epoch-steps", type=int, default=0, help="0 = the minimum delay (or 1000 without a network)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch every epoch's kernels directly")
    ap.add_argument("--dry-run-ranks", default="1",
                    help="config 7: emulate this many identical ranks (proxy spikes, Sec. V-E dry run); a comma "
                         "list sweeps them, the first giving the headline line")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.txt"))
    ap.add_argument("--fit-traffic", metavar="RUN_DIR", default=None,
                    help="fit the step kernels' HBM traffic from counter runs in RUN_DIR (see fit_traffic) "
                         "into --traffic-json for --config (or --varstep), then exit")
    ap.add_argument("--kernel", default=None, help="with --fit-traffic: the kernel the runs launched")
    ap.add_argument("--varstep", action="store_true",
                    help="the ring (config 2) with the variable time step: steps cut at off-grid event times")
    ap.add_argument("--mech", action="store_true",
                    help="the ring's cells (config 2) with generated density mechanisms (hcn, kdr, generated hh)")
    args = ap.parse_args()
    if (args.varstep or args.mech) and args.config != 2:
        raise SystemExit("--varstep and --mech run the ring: use them with --config 2")
    if args.varstep and args.mech:
        raise SystemExit("the variable time step does not run generated mechanisms")
    leg = "2t" if args.varstep else "2m" if args.mech else args.config
    if args.fit_traffic:
        key = f"config{leg}"
        rec = fit_traffic(args.fit_traffic, key, args.kernel, "var" if args.varstep else "reg", args.traffic_json)
        print(json.dumps({key: rec}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        raise SystemExit(2)

    import torch

    from paper_1901_07454_amd import arbmi
    from workloads import gen

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    sweep = [int(x) for x in str(args.dry_run_ranks).split(",")]
    args.dry_run_ranks = sweep[0]
    if args.varstep:
        n = args.cells or 8192
        m = gen.config2_timed(n_cells=n, t_ms=VARSTEP_T_MS)
        desc = (f"{n}-cell ring with the variable time step: depth-6 binary trees x 8 CVs/branch (1017 CVs/cell), "
                "hh soma, pas dendrites, 10 expsyn/cell, ring delays U(5, 5.5) ms, kicks at U(0, 1) ms, 10 Hz "
                "Poisson input per dendritic synapse at continuous times")
    elif args.mech:
        n = args.cells or 8192
        # kicks every 400 steps through the warm-up and the timed steps (both
        # rounded up to whole epochs of at most 200 steps)
        m = gen.config2_mech(n_cells=n, n_steps=args.warmup + args.steps + 400)
        desc = (f"{n}-cell ring with generated mechanisms: depth-6 binary trees x 8 CVs/branch (1017 CVs/cell), "
                "built-in hh soma, pas dendrites, 10 expsyn/cell, delay 5 ms; generated hcn on the soma, kdr on "
                "every branch, hh on branch 0; every soma kicked each 10 ms")
    else:
        m, desc = make_model(args.config, args.cells, args.dry_run_ranks)
    log(f"model built in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    # whole epochs (exchange and step kernels) replay from a captured HIP graph
    flags = arbmi.ARB_FLAG_TIME_KERNELS | (0 if args.no_graph else arbmi.ARB_FLAG_GRAPH)
    if not (args.block_threads or args.coef_mode or args.cells_per_pack or args.varstep):
        flags |= arbmi.ARB_FLAG_AUTOTUNE
    sim = arbmi.Simulation(m, flags=flags, block_threads=args.block_threads, epoch_steps=args.epoch_steps,
                           dry_run_ranks=args.dry_run_ranks if args.config == 7 else 0,
                           coef_mode=args.coef_mode, cells_per_pack=args.cells_per_pack)
    info = sim.info
    log(f"sim built in {time.perf_counter() - t0:.1f} s: {info}")
    n_cv = info["n_cv"]

    # whole epochs only, so that every timed step pays its share of the
    # spike exchange (index, pull and collect run once per epoch), after at
    # least one warm-up epoch
    K = info["epoch_steps"]
    warmup = max(1, -(-args.warmup // K)) * K
    steps = max(1, -(-args.steps // K)) * K
    if args.varstep and (warmup + steps) * float(m["dt"]) > VARSTEP_T_MS:
        raise SystemExit(f"--varstep: at most {VARSTEP_T_MS} ms of input (warm-up plus timed steps)")
    sim.step(warmup)
    sim.sync()
    sim.kernel_time()  # discard warm-up launches
    taken0 = sim.step_count()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, nlaunch = sim.kernel_time()
    sim.sync()
    spikes = sim.spikes()
    taken = sim.step_count() - taken0  # steps of all cells, shortened ones included
    log(f"timed {steps} steps in {wall:.4f} s, {nlaunch} step-kernel launches, {kms:.2f} ms in them, "
        f"{len(spikes)} spikes")

    value = n_cv * steps / wall
    steps_per_launch = steps / max(nlaunch, 1)
    avg_launch_s = kms / 1e3 / max(nlaunch, 1)
    flops_per_step = FLOPS_PER_CV * n_cv + FLOPS_PER_HH * info["n_hh"] + FLOPS_PER_SYN * info["n_syn"]
    gen_instances = {}
    if args.mech:  # each generated instance's operations, counted from its description
        from paper_1901_07454_amd import mechgen
        ops = {m_.name: mechgen.op_count(m_) for m_ in mechgen.load_catalogue()}
        gen_instances = sim.mechanism_instances()
        flops_per_step += sum(ops[k] * v for k, v in gen_instances.items())
    # steps taken per grid step of every cell (1 with the fixed step)
    taken_ratio = taken / (steps * info["n_cells"])
    tflops = flops_per_step * taken_ratio * steps_per_launch / avg_launch_s / 1e12
    model_gbps = info["bytes_per_step"] * steps_per_launch / avg_launch_s / 1e9
    kernel = kernel_name(info, args.varstep, args.mech)
    traffic = measured_traffic(args.traffic_json, leg, kernel, steps_per_launch)
    traffic_gbps = None if traffic is None else traffic / avg_launch_s / 1e9
    copy_gbps = copy_bandwidth_gbps(torch)
    # The bound: the resource the kernel comes closest to.  The fused kernel
    # keeps voltages, states and coefficients on chip for a whole epoch, so on
    # the CV-dominated workloads its measured HBM traffic is a small fraction
    # of the peak and FP64 issue is the nearer roofline (the kernel itself is
    # bound by the latency of the solve's dependency chains); synapse-heavy
    # workloads stream their synapse state and sit on HBM.
    alu_frac = tflops / FP64_PEAK_TFLOPS
    hbm_frac = None if traffic_gbps is None else traffic_gbps / HBM_PEAK_GBPS
    if hbm_frac is not None and hbm_frac > alu_frac:
        roof = {"bound": "hbm", "achieved": traffic_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": hbm_frac, "traffic": traffic,
                "basis": "measured FETCH_SIZE + WRITE_SIZE bytes per launch / average launch time"}
        if hbm_frac > 1.0:
            roof["note"] = ("FETCH_SIZE and WRITE_SIZE count the L2's traffic to the fabric, hits in the "
                            "256 MB last-level cache included, so their rate can pass the HBM peak")
    else:
        roof = {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": alu_frac, "traffic": traffic,
                "basis": ("algorithmic FP64 operations per launch (7 per CV, 61 per hh instance, 4 per "
                          "synapse" + (", each generated mechanism instance the count of its description"
                                       if args.mech else "") +
                          ", per step taken) / average launch time; peak = MI355X vector FP64")}
    roof.update({
        "kernel": kernel, "steps_per_launch": steps_per_launch, "avg_launch_ms": avg_launch_s * 1e3,
        "launches": nlaunch, "kernel_ms_total": kms,
        "traffic_GBps": traffic_gbps, "traffic_frac_of_hbm_peak": hbm_frac,
        "fp64": {"achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": alu_frac,
                 "flops_per_step": flops_per_step},
        "byte_model": {"bytes_per_step": info["bytes_per_step"], "GBps": model_gbps,
                       "ratio_to_hbm_peak": model_gbps / HBM_PEAK_GBPS,
                       "note": ("per-step SoA byte model (44 B/CV, 56 B/hh, 20 B/synapse) over the launch time; "
                                "not a roofline fraction: one launch keeps the state on chip for a whole "
                                "epoch, so it moves far fewer bytes than the model counts")},
        "measured_copy_GBps": copy_gbps,
    })
    out = {
        "metric": "CV-updates/s per GPU (fwd FP64)",
        "value": value,
        "unit": "CV-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("variable step: " if args.varstep else "generated mechanisms: " if args.mech
                                else f"config {args.config}: ") + desc,
                   "cells": info["n_cells"], "cvs": n_cv,
                   "dt_ms": float(m["dt"]), "epoch_steps": K,
                   "block_threads": info["block_threads"], "coef_mode": info["coef_mode"],
                   "packs": info["n_packs"], "lds_bytes": info["lds_bytes"], "launch_classes": info["n_classes"],
                   "graph": not args.no_graph, "spikes": int(len(spikes)),
                   **({"steps_taken": int(taken), "steps_taken_per_grid_step": taken_ratio} if args.varstep else {}),
                   **({"dry_run_ranks": args.dry_run_ranks} if args.config == 7 and args.dry_run_ranks > 1 else {}),
                   **({"mechanism_instances": gen_instances} if args.mech else {})},
        "roofline": roof,
    }
    if info["n_syn"] > 0:
        out["synapse_updates_per_s"] = info["n_syn"] * steps / wall
    sim.close()
    if args.config == 7 and len(sweep) > 1:
        out["dry_run"] = dry_run_sweep(m, sweep, K)
    if not args.no_grad:
        out["grad"] = grad_ratio(torch)
        if args.config == 5:
            out["grad_subset"] = grad_ratio(torch, subset=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(leg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
