"""The library's positive-argument power (csrc/powd.h, used by every kernel
for the equation of state, Eq. pressure, and its inverse), built for the
host with g++ and compared with the C library's pow over seeded arguments:
the model's range (p / p_ref and R_d rho theta / p_ref within 1e-3..1e3,
exponents C_p / C_v and C_v / C_p for gases with C_p / C_v in 1.2..1.45),
a wider range, and exact cases (squares of powers of two, 1^y)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path_factory.mktemp("powd") / "powd")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(ROOT, "tests", "native", "powd_driver.cpp"),
                    "-o", exe], check=True, capture_output=True, timeout=120)
    return exe


def _run(exe, *args):
    out = subprocess.run([exe] + [str(a) for a in args], check=True, capture_output=True, text=True,
                         timeout=120).stdout.split()
    return float(out[0]), float(out[3])


def test_power_in_the_model_range(driver):
    worst, exact = _run(driver, -3, 3, 1.2, 1.45, 2000000)
    assert worst < 2.5e-15, worst
    assert exact < 2e-15, exact


def test_power_over_a_wide_range(driver):
    # the error grows with |y ln x| (the rounding of the product): 27 at the far end
    worst, _ = _run(driver, -6, 8, 1.0, 1.7, 2000000)
    assert worst < 8e-15, worst
