"""The kernels' float64 math routines (fp64_math.hpp: exp by Cody-Waite reduction, log1p on
[0, 1] by the atanh series, softplus from the two), compiled for the host with hipcc and
checked against mpmath's values at 30 digits (an independent arbitrary-precision
implementation): relative error of exp within 2 x 2^-52 on [-700, 700], of log1p within
2 x 2^-52 on [0, 1], of softplus within 3 x 2^-52 on [-40, 40]; exp(0) = 1, log1p(0) = 0,
softplus(0) = log 2 to rounding.  The device build runs the same operation sequence (explicit
fma, correctly rounded division)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_10042_amd", "csrc")

PROG = r"""
#include <math.h>
#include <stdio.h>
#include "fp64_math.hpp"
int main() {
    double x;
    while (scanf("%la", &x) == 1)   // each routine only on its documented range
        printf("%a %a %a\n", fabs(x) <= 700.0 ? cse::exp_cw(x) : NAN,
               (x >= 0.0 && x <= 1.0) ? cse::log1p_unit(x) : NAN, fabs(x) <= 700.0 ? cse::softplus_fast(x) : NAN);
    return 0;
}
"""


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("fp64math")
    src, exe = os.path.join(d, "prog.cpp"), os.path.join(d, "prog")
    with open(src, "w") as f:
        f.write(PROG)
    subprocess.run([hipcc, "-O2", "-std=c++17", "-I", CSRC, src, "-o", exe], check=True, capture_output=True)

    def call(xs):
        inp = "".join(float(x).hex() + "\n" for x in xs)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
        return np.array([[float.fromhex(v) for v in line.split()] for line in out if line.strip()])

    return call


def _worst(got, ref_fn, xs):
    mp.mp.dps = 30
    return max(float(abs((mp.mpf(g) - ref_fn(mp.mpf(x))) / ref_fn(mp.mpf(x)))) / 2.0**-52 for g, x in zip(got, xs))


def test_exp(run):
    xs = np.concatenate([np.linspace(-700.0, 700.0, 2801), np.linspace(-1.0, 1.0, 401),
                         np.random.default_rng(0).uniform(-40.0, 0.0, 1000)])
    w = _worst(run(xs)[:, 0], mp.exp, xs)
    print(f"exp worst {w:.2f} x 2^-52")
    assert w <= 2.0


def test_log1p_unit(run):
    xs = np.unique(np.concatenate([np.linspace(0.0, 1.0, 2001)[1:], np.geomspace(1e-300, 1.0, 1200)]))
    w = _worst(run(xs)[:, 1], mp.log1p, xs)
    print(f"log1p worst {w:.2f} x 2^-52")
    assert w <= 2.0


def test_softplus(run):
    xs = np.concatenate([np.linspace(-40.0, 40.0, 4001), np.random.default_rng(1).normal(0.0, 3.0, 1000)])
    w = _worst(run(xs)[:, 2], lambda x: mp.log1p(mp.exp(x)), xs)
    print(f"softplus worst {w:.2f} x 2^-52")
    assert w <= 3.0


def test_special_values(run):
    r = run([0.0, -0.0])
    assert np.all(r[:, 0] == 1.0) and np.all(r[:, 1] == 0.0)
    assert abs(r[0, 2] - np.log(2.0)) <= 2.0**-53
