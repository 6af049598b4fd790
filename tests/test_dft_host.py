"""The step kernel's register-resident DFTs (csrc/cmath.h, dft<R, DIR>), built for the host
with hipcc and checked against numpy's FFT: every radix the FFT plans use, R = 2 .. 32,
forward (kernel exp(-2 pi i jk/R), Section 2.1) and inverse (conjugate kernel, unnormalised)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2504_10118_amd", "csrc")


@pytest.fixture(scope="module")
def dft_output(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("dft") / "dft_check")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "dft_host_check.hip"), "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    vals = {}
    for line in out.splitlines():
        kind, R, D, j, re, im = line.split()
        vals.setdefault((kind, int(R), int(D)), {})[int(j)] = complex(float(re), float(im))
    return vals


@pytest.mark.parametrize("R", [2, 4, 8, 16, 32])
@pytest.mark.parametrize("direction", [1, -1])
def test_register_dft_matches_numpy(dft_output, R, direction):
    x = np.array([dft_output[("in", R, direction)][j] for j in range(R)])
    y = np.array([dft_output[("out", R, direction)][j] for j in range(R)])
    ref = np.fft.fft(x) if direction > 0 else np.fft.ifft(x) * R
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    assert err < 2e-6 * np.log2(R) + 1e-7, (R, direction, err)


def test_wrong_sign_would_fail(dft_output):
    """The comparison tells the two directions apart (the inverse is not the forward)."""
    x = np.array([dft_output[("in", 32, -1)][j] for j in range(32)])
    y = np.array([dft_output[("out", 32, -1)][j] for j in range(32)])
    assert np.max(np.abs(y - np.fft.fft(x))) > 0.1 * np.max(np.abs(y))
