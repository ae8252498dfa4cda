"""Host check of the coarsest-level dense inverse (csrc/dense.h), built with g++ alone.

The inverse runs inside an OpenMP loop over the coarsest level's components, so it
reports a singular block by its return value (the setup then fails with
KNP_E_NUMERIC after the loop) instead of throwing.  Checked: a well-conditioned
matrix and a nearly singular one that still has digits (condition ~1e10, like the
intracellular potential blocks that only the membrane mass keeps invertible) are
inverted; an exactly singular matrix, one singular up to rounding, a zero matrix and
one holding a NaN are refused.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2403_04491_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "dense.h"
int main() {
    int n;
    while (std::scanf("%d", &n) == 1) {
        std::vector<double> a(size_t(n) * n);
        for (auto &v : a) std::scanf("%lf", &v);
        const bool ok = knp::invert_dense(n, a);
        std::printf("%d", ok ? 1 : 0);
        if (ok)
            for (double v : a) std::printf(" %.17g", v);
        std::printf("\n");
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("dense")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([gxx, "-O2", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)], check=True)
    return str(exe)


def _run(exe, mats):
    text = "".join(f"{m.shape[0]} " + " ".join(repr(float(v)) for v in m.ravel()) + "\n" for m in mats)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.splitlines()
    res = []
    for line, m in zip(out, mats):
        f = line.split()
        res.append(None if f[0] == "0" else np.array([float(x) for x in f[1:]]).reshape(m.shape))
    return res


def test_dense_inverse_and_singular_blocks(driver):
    rng = np.random.Generator(np.random.PCG64(5))
    n = 40
    good = rng.standard_normal((n, n)) + n * np.eye(n)
    # 1D Laplacian with Neumann ends (singular) plus a 1e-10 shift: condition ~1e10
    lap = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    lap[0, 0] = lap[-1, -1] = 1.0
    near_ok = lap + 1e-10 * np.eye(n)
    singular = good.copy()
    singular[7] = singular[3]
    rank_def = rng.standard_normal((n, 5)) @ rng.standard_normal((5, n))
    nan = good.copy()
    nan[2, 2] = np.nan
    zero = np.zeros((3, 3))
    inv_good, inv_near, r_sing, r_rank, r_nan, r_zero = _run(
        driver, [good, near_ok, singular, rank_def, nan, zero])
    assert np.abs(inv_good @ good - np.eye(n)).max() < 1e-12
    assert inv_near is not None
    assert np.abs(inv_near - np.linalg.inv(near_ok)).max() <= 1e-4 * np.abs(np.linalg.inv(near_ok)).max()
    assert r_sing is None
    assert r_rank is None
    assert r_nan is None
    assert r_zero is None
