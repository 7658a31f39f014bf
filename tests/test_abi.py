"""CPU checks of the C-ABI boundary: the library is built, loads, exports every
function include/abp.h declares, lays out its structures as the Python
binding does, and rejects bad arguments on the host before touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abp.h")
LIB = os.path.join(ROOT, "paper_1609_09833_amd", "libabp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:abp_status|int64_t|const char\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libabp.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("abp_create", "abp_destroy", "bias_deposit", "bias_eval", "cv_compute", "bias_force",
                     "abp_sync", "abp_reserve", "abp_commit"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for n in declared_functions():
        assert hasattr(lib, n)


def test_struct_layout_matches_binding(tmp_path):
    """Compile the header with gcc and compare sizes/offsets with the ctypes mirrors."""
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "abp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(abp_bias_desc), offsetof(abp_bias_desc, capacity),
         offsetof(abp_bias_desc, grid_n), offsetof(abp_bias_desc, kT), offsetof(abp_bias_desc, quantize),
         offsetof(abp_bias_desc, wt_dT));
  printf("%zu %zu %zu\\n", sizeof(abp_cv_desc), offsetof(abp_cv_desc, list_off), offsetof(abp_cv_desc, ref_z));
  printf("%zu %zu %zu\\n", sizeof(abp_walkers), offsetof(abp_walkers, x), offsetof(abp_walkers, fz));
  printf("%zu %zu %zu %zu\\n", sizeof(abp_server_desc), offsetof(abp_server_desc, max_pending),
         offsetof(abp_server_desc, cv_kind), offsetof(abp_server_desc, eval_mode));
  printf("%zu %zu\\n", sizeof(abp_server_stats), offsetof(abp_server_stats, wall_seconds));
  printf("%d\\n", ABP_SERVER_BYTES_PER_ATOM);
  printf("%zu %zu %zu %zu %zu\\n", sizeof(abp_server_result), offsetof(abp_server_result, walker),
         offsetof(abp_server_result, t_submit), offsetof(abp_server_result, V), offsetof(abp_server_result, dVds));
  printf("%zu %zu %zu\\n", sizeof(abp_server_batch), offsetof(abp_server_batch, requests),
         offsetof(abp_server_batch, admitted));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    vals = [list(map(int, l.split())) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines()]
    # the binding's mirrors (the binding imports torch, which is available here)
    from paper_1609_09833_amd import abp
    assert vals[0] == [C.sizeof(abp.BiasDesc), abp.BiasDesc.capacity.offset, abp.BiasDesc.grid_n.offset,
                       abp.BiasDesc.kT.offset, abp.BiasDesc.quantize.offset, abp.BiasDesc.wt_dT.offset]
    assert vals[1] == [C.sizeof(abp.CvDesc), abp.CvDesc.list_off.offset, abp.CvDesc.ref_z.offset]
    assert vals[2] == [C.sizeof(abp.WalkersDesc), abp.WalkersDesc.x.offset, abp.WalkersDesc.fz.offset]
    assert vals[3] == [C.sizeof(abp.ServerDesc), abp.ServerDesc.max_pending.offset, abp.ServerDesc.cv_kind.offset,
                       abp.ServerDesc.eval_mode.offset]
    assert vals[4] == [C.sizeof(abp.ServerStats), abp.ServerStats.wall_seconds.offset]
    assert vals[5] == [abp.ABP_SERVER_BYTES_PER_ATOM]
    R, B = abp.SERVER_RESULT, abp.SERVER_BATCH
    assert vals[6] == [R.itemsize, R.fields["walker"][1], R.fields["t_submit"][1], R.fields["V"][1],
                       R.fields["dVds"][1]]
    assert vals[7] == [B.itemsize, B.fields["requests"][1], B.fields["admitted"][1]]


def test_host_side_validation_without_gpu(lib):
    lib.abp_create.restype = C.c_int32
    lib.abp_create.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    lib.abp_last_error.restype = C.c_char_p
    lib.abp_status_str.restype = C.c_char_p
    lib.abp_status_str.argtypes = [C.c_int32]
    out = C.c_void_p()
    assert lib.abp_create(None, 0, C.byref(out)) == 1          # ABP_E_INVAL: NULL descriptor
    assert b"NULL" in lib.abp_last_error()
    from paper_1609_09833_amd import abp
    from paper_1609_09833_amd import workloads as W
    spec = W.BiasSpec(ndim=4, periodic=(1,), lo=(0.0,), hi=(1.0,), width=(0.1,))
    d = abp.make_desc(W.BiasSpec(ndim=2, periodic=(1, 1), lo=(0, 0), hi=(1, 1), width=(0.1, -1.0)), 10)
    assert lib.abp_create(C.byref(d), 0, C.byref(out)) == 1      # negative width
    assert b"width" in lib.abp_last_error()
    d = abp.make_desc(W.BiasSpec(ndim=2, periodic=(1, 1), lo=(0, 0), hi=(1, 1), width=(0.1, 0.1),
                                 kernel=1, p=0), 10)
    assert lib.abp_create(C.byref(d), 0, C.byref(out)) == 1      # compact needs p >= 1
    d = abp.make_desc(W.BiasSpec(ndim=1, periodic=(1,), lo=(0,), hi=(1,), width=(0.1,)), 0)
    assert lib.abp_create(C.byref(d), 0, C.byref(out)) == 1      # zero capacity
    d = abp.make_desc(W.BiasSpec(ndim=1, periodic=(1,), lo=(0,), hi=(1,), width=(0.1,), transform=1, b=1.5), 5)
    assert lib.abp_create(C.byref(d), 0, C.byref(out)) == 1      # mABP needs 0 < b < 1
    d = abp.make_desc(W.BiasSpec(ndim=2, periodic=(1, 0), lo=(0, 2.0), hi=(1, 2.0), width=(0.1, 0.1)), 5)
    assert lib.abp_create(C.byref(d), 0, C.byref(out)) == 1      # every axis needs hi > lo
    assert b"hi > lo" in lib.abp_last_error()
    del spec
    for code, name in enumerate([b"ABP_OK", b"ABP_E_INVAL", b"ABP_E_NOMEM", b"ABP_E_CAPACITY", b"ABP_E_DEVICE",
                                 b"ABP_E_INDEX", b"ABP_E_NONFINITE", b"ABP_E_BUSY"]):
        assert lib.abp_status_str(code) == name


def test_null_context_calls_fail_cleanly(lib):
    lib.bias_eval.restype = C.c_int32
    lib.bias_eval.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_void_p, C.c_void_p]
    assert lib.bias_eval(None, 0, 0, 10, 0, None, -1, None, None, None) == 1
    lib.abp_num_hills.restype = C.c_int64
    lib.abp_num_hills.argtypes = [C.c_void_p]
    assert lib.abp_num_hills(None) == -1
    lib.abp_destroy.restype = C.c_int32
    lib.abp_destroy.argtypes = [C.c_void_p]
    assert lib.abp_destroy(None) == 0


def test_product_path_does_not_touch_the_oracle():
    """The GPU binding and sources never import, load or name the oracle."""
    pkg = os.path.join(ROOT, "paper_1609_09833_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and "abp_oracle" not in text, f


def test_serving_driver_positions_match_the_engine_model():
    """The load generator's CV-atom positions are the synthetic engine's,
    x0 + amplitude * u(walker, step, atom, coordinate), bit for bit."""
    import numpy as np
    from paper_1609_09833_amd import workloads as W
    from paper_1609_09833_amd.examples import serve_driver as D
    rng = np.random.default_rng(3)
    n_atoms = [50, 7, 120]
    atoms = [np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32) for n, k in zip(n_atoms, (9, 4, 30))]
    base_full = [rng.uniform(0, 6, (3, n)).astype(np.float32) for n in n_atoms]

    class E(D.Engines):
        def __init__(self):
            self.n_cv = np.array([a.size for a in atoms], dtype=np.int32)
            self.atoms = np.concatenate(atoms)
            self.base = np.concatenate([b[:, a].ravel() for b, a in zip(base_full, atoms)]).astype(np.float32)
            self.base_off = np.zeros(3, dtype=np.int64)
            self.base_off[1:] = np.cumsum(3 * self.n_cv.astype(np.int64))[:-1]

    walker = np.array([2, 0, 1, 2, 0], dtype=np.int32)
    step = np.array([1, 5, 9, 2, 4_000_000_000], dtype=np.int64)
    amp = 2.0 ** -7
    pos, off = E().positions(walker, step, amp, threads=3)
    for i, (w, t) in enumerate(zip(walker, step)):
        b = base_full[w]
        x, y, z = W.engine_positions(b[0], b[1], b[2], int(w), int(t), atoms[w], amp)
        k = atoms[w].size
        want = np.concatenate([x[atoms[w]], y[atoms[w]], z[atoms[w]]])
        assert np.array_equal(pos[off[i]:off[i] + 3 * k], want), i
