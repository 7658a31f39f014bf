"""The C-ABI from plain C: paper_1609_09833_amd/examples/abp_c_client.c is
compiled with gcc against include/abp.h and libabp.so (CPU), and on a GPU its
printed results are checked against the oracle."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1609_09833_amd")
SRC = os.path.join(PKG, "examples", "abp_c_client.c")


def _build(tmp_path):
    exe = tmp_path / "abp_c_client"
    lib = os.path.join(PKG, "libabp.so")
    if not os.path.exists(lib):
        pytest.skip("libabp.so not built")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", SRC, "-L", PKG, "-labp", f"-Wl,-rpath,{PKG}", "-L", "/opt/rocm/lib",
                    "-lamdhip64", "-lm", "-o", str(exe)], check=True)
    return exe


def test_c_client_compiles_and_links(tmp_path):
    exe = _build(tmp_path)
    assert exe.exists()


@pytest.mark.gpu
def test_c_client_matches_oracle(tmp_path):
    import oracle
    from paper_1609_09833_amd import workloads as W
    exe = _build(tmp_path)
    hills_bin = tmp_path / "hills.bin"
    r = subprocess.run([str(exe), "1500", "64", "9", str(hills_bin)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rows = np.array([[float(x) for x in l.split()] for l in r.stdout.splitlines() if not l.startswith("#")])
    raw = np.fromfile(hills_bin, dtype=np.float64)
    cen, hts = raw[:3000].reshape(2, 1500), raw[3000:]
    spec = W.BiasSpec(ndim=2, periodic=(1, 1), lo=(-np.pi, -np.pi), hi=(np.pi, np.pi), width=(0.3, 0.3),
                      grid_n=(128, 128))
    q = rows[:, :2].T.copy()
    Vo, dVo, sV, sG = oracle.bias_eval(spec, cen, hts, q)
    assert np.all(np.abs(rows[:, 2] - Vo) <= 1e-5 * np.maximum(np.abs(Vo), sV))
    assert np.all(np.abs(rows[:, 3:5].T - dVo) <= 1e-5 * (np.abs(dVo) + sG))
    # the grid value is the Hermite interpolant of the oracle's grid
    H = oracle.grid_all(spec, cen, hts)
    hq, _, _ = oracle.grid_eval(spec, H, q)
    assert np.all(np.abs(rows[:, 5] - hq) <= 1e-9 * (np.abs(hq) + sV))
