"""The solver's complementary error function and exponential
(paper_2108_07031_amd/csrc/qlskum_erfc.h), built for the host with hipcc and
checked against 40-digit mpmath: erfc in FP64 within 1e-15 relative on
[-30, 30]; in FP32 within 1e-6 relative for |y| <= 3 (the range of
S = u_e sqrt(beta) up to Mach ~3.5), a bound set by the FP32 rounding of y^2
inside exp(-y^2), 2 y^2 x 6e-8 -- the same size as the effect of rounding the
argument y itself to FP32.  The exponential within 2.5e-16 relative over its
whole normal range, exact at 0, 0 and inf past the ends, NaN kept."""
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def erfc_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("erfc") / "erfc_check")
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-x", "hip", os.path.join(ROOT, "tests", "erfc_check.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def test_erfc_accuracy(erfc_exe):
    ys = np.concatenate([np.linspace(-6, 6, 2401), np.linspace(-1e-3, 1e-3, 41),
                         np.linspace(-1.001, 1.001, 801), [np.nextafter(1.0, 2.0), -np.nextafter(1.0, 2.0)],
                         [-30.0, -10.0, 8.0, 10.0, 20.0, 26.0, 0.0]])
    out = subprocess.run([erfc_exe], input="\n".join(repr(float(v)) for v in ys),
                         capture_output=True, text=True, check=True).stdout.split()
    vals = np.array(out, dtype=float).reshape(-1, 2)
    mp.mp.dps = 40
    ex64 = np.array([float(mp.erfc(mp.mpf(float(v)))) for v in ys])
    ex32 = np.array([float(mp.erfc(mp.mpf(float(np.float32(v))))) for v in ys])
    tiny = 1e-300
    r64 = np.abs(vals[:, 0] - ex64) / np.maximum(np.abs(ex64), tiny)
    assert r64.max() <= 1e-15, r64.max()
    m = np.abs(ys) <= 3
    r32 = np.abs(vals[m, 1] - ex32[m]) / np.abs(ex32[m])
    assert r32.max() <= 1e-6, r32.max()


def test_exp_accuracy(erfc_exe):
    xs = np.concatenate([np.linspace(-745, 709, 20001), np.linspace(-2, 2, 4001),
                         np.linspace(-1e-3, 1e-3, 41), [0.0, 1e-300, -1e-300, 709.7, -708.3]])
    out = subprocess.run([erfc_exe, "exp"], input="\n".join(repr(float(v)) for v in xs),
                         capture_output=True, text=True, check=True).stdout.split()
    vals = np.array(out, dtype=float)
    mp.mp.dps = 40
    ex = np.array([float(mp.exp(mp.mpf(float(v)))) for v in xs])
    normal = ex >= 2.2250738585072014e-308
    rel = np.abs(vals[normal] - ex[normal]) / ex[normal]
    assert rel.max() <= 2.5e-16, rel.max()
    assert vals[xs == 0.0][0] == 1.0
    edge = subprocess.run([erfc_exe, "exp"], input="-746\n-1e14\n710\n1e14\nnan\n",
                          capture_output=True, text=True, check=True).stdout.split()
    e = np.array(edge, dtype=float)
    assert e[0] == 0.0 and e[1] == 0.0 and np.isposinf(e[2]) and np.isposinf(e[3])
    assert np.isnan(e[4])
