"""The register-resident kernel's e^x / e^x - 1 core (fastexp.hpp), built for
the host from the same source (every product-sum is an explicit fma, so host
and device round alike), against numpy's exp and expm1."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def fastexp(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("fastexp") / "fastexp_check")
    subprocess.run(["hipcc", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "fastexp_check.cpp")],
                   check=True, capture_output=True, timeout=600)

    def run(xs):
        out = subprocess.run([exe], input="\n".join(float(x).hex() for x in xs), capture_output=True,
                             text=True, check=True, timeout=120).stdout.split()
        v = np.array([float.fromhex(t) for t in out]).reshape(-1, 3)
        assert np.array_equal(v[:, 0], np.asarray(xs, float))
        return v[:, 1], v[:, 2]
    return run


def _ulp(got, ref):
    return np.where(ref == 0, np.abs(got - ref), np.abs(got - ref) / np.spacing(np.abs(ref)))


def test_exp_and_expm1_within_two_ulp(fastexp):
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.uniform(-20, 20, 20000), rng.uniform(-1e-4, 1e-4, 3000),
                         rng.uniform(-0.35, 0.35, 5000), rng.uniform(-700, 700, 2000)])
    e, em = fastexp(xs)
    assert _ulp(e, np.exp(xs)).max() <= 2
    assert _ulp(em, np.expm1(xs)).max() <= 3


def test_special_points(fastexp):
    xs = np.array([0.0, -0.0, 1e-300, -1e-300, np.log(2) / 2, -np.log(2) / 2, np.log(2), 1.0, -1.0])
    e, em = fastexp(xs)
    assert e[0] == 1.0 and em[0] == 0.0 and e[1] == 1.0
    assert em[2] == 1e-300 and em[3] == -1e-300        # e^x - 1 = x below the rounding of x
    assert _ulp(e[4:], np.exp(xs[4:])).max() <= 1
    assert _ulp(em[4:], np.expm1(xs[4:])).max() <= 2
