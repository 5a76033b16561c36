"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle, built from its source with both sanitizers, runs every
kind of workload (networks, external events, clamps, the adjoint, the
standalone solve and rate routines) in a child process; the library's host
lowering, built with g++ and both sanitizers beside a small driver
(tests/lowering_check.cpp), lowers several workloads under every launch
layout and runs the state-blob checks of arb_set_state on valid and
corrupted blobs.  Any sanitizer report aborts the child and fails the test."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1901_07454_amd import arbmi
from workloads import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


ASAN, UBSAN = _runtime("libasan.so"), _runtime("libubsan.so")
pytestmark = pytest.mark.skipif(not (ASAN and UBSAN), reason="gcc sanitizer runtimes not installed")

ORACLE_RUN = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle
from workloads import gen
from tests import models

def run(m, n, **kw):
    s = oracle.Sim(m, **kw)
    tr = s.run(n, probes=np.arange(min(s.ncv, 40)))
    assert np.all(np.isfinite(tr))
    s.spikes()
    s.state()
    return s

run(gen.config1(), 400)
run(gen.config2(n_cells=3, n_steps=400), 400)
run(gen.config2(n_cells=3, n_steps=400), 400, epoch_steps=37)
run(gen.config3(cells=[0, 321], n_steps=300), 300)
run(gen.config5(n_cells=65536, cells=[0, 1, 2], n_steps=300), 300)
m4 = gen.config4(n_cells=2, n_steps=200)
s = oracle.Sim(m4)
s.set_params(gen.config4_theta(m4).reshape(-1, 3))
tr, g = s.adjoint(200, np.ones((2, 200)) * 1e-3)
assert np.all(np.isfinite(g))
for k in (1, 2, 7, 30):
    models_rng = np.random.default_rng(k)
    par = np.array([-1] + [int(models_rng.integers(0, i)) for i in range(1, k)], np.int64)
    d = 4.0 + models_rng.random(k)
    u = -models_rng.random(k)
    b = models_rng.random(k)
    x = oracle.hines_solve(par, d, u, b)
    assert np.all(np.isfinite(x))
for v in (-100.0, -40.0, -55.0, 0.0, 30.0):
    oracle.hh_rates(v)
    oracle.hh_rates_dv(v)
print("SANITIZE-OK")
'''


def test_oracle_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", *SAN, "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    script = tmp_path / "run.py"
    script.write_text(ORACLE_RUN)
    env = dict(os.environ, LD_PRELOAD=f"{ASAN} {UBSAN}", ASAN_OPTIONS="detect_leaks=0",
               ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, str(script), ROOT], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "SANITIZE-OK" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]


def _write_model(path, m):
    arrs = arbmi.model_structs(m)
    with open(path, "wb") as f:
        f.write(np.array([len(a) for a in arrs], np.int64).tobytes())
        for a in arrs:
            f.write(np.ascontiguousarray(a).tobytes())


def test_host_lowering_under_sanitizers(tmp_path):
    exe = tmp_path / "lowering_check"
    subprocess.run(["g++", "-std=c++17", *SAN, "-o", str(exe), os.path.join(ROOT, "tests", "lowering_check.cpp"),
                    os.path.join(ROOT, "paper_1901_07454_amd", "csrc", "lower.cpp")], check=True)
    workloads = {
        "config1": gen.config1(),
        "ring": gen.config2(n_cells=6, n_steps=100),
        "uneven": gen.config3(cells=[0, 1, 321, 1040], n_steps=100),
        "clamp": gen.config4(n_cells=3, n_steps=100),
        "network": gen.config5(n_cells=65536, cells=list(range(8)), n_steps=100),
        "synapse_heavy": gen.config6(n_cells=3, n_steps=100, n_syn=1500),
    }
    for name, m in workloads.items():
        path = tmp_path / f"{name}.bin"
        _write_model(path, m)
        r = subprocess.run([str(exe), str(path)], capture_output=True, text=True, timeout=600,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
        print(name, r.stdout.strip().splitlines()[-1] if r.stdout.strip() else "", flush=True)
        assert r.returncode == 0, name + "\n" + r.stdout[-3000:] + r.stderr[-4000:]
