"""The coefficients of the FP64 hill-term exponential (kExp2Poly in the
device header) are those the generator script computes, and the polynomial
meets its error bound: 2^r on [-1/2, 1/2] within 1e-17 relative in exact
(long double) arithmetic, and within 2 units of the last place when evaluated
by Horner's rule in FP64 with fused multiply-adds emulated in long double."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_09833_amd", "csrc")


def _generator():
    spec = importlib.util.spec_from_file_location("exp2_poly", os.path.join(CSRC, "exp2_poly.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _header_coefficients():
    text = open(os.path.join(CSRC, "abp_device.h")).read()
    m = re.search(r"kExp2Poly\[(\d+)\]\s*=\s*\{([^}]*)\}", text)
    assert m, "kExp2Poly not found"
    vals = [float(v) for v in m.group(2).replace("\n", " ").split(",") if v.strip()]
    assert len(vals) == int(m.group(1))
    return vals


def test_header_matches_generator():
    gen = _generator()
    want = [float(c) for c in gen.coefficients()]
    assert _header_coefficients() == want


def test_interpolant_error_bound():
    gen = _generator()
    assert gen.max_rel_error(gen.coefficients()) < 1e-17
    # the leading coefficients are those of the Taylor series of exp(r ln 2)
    c = _header_coefficients()
    ln2 = np.log(np.longdouble(2))
    assert c[0] == 1.0
    assert abs(c[1] / float(ln2) - 1) < 1e-15
    assert abs(c[2] / float(ln2 ** 2 / 2) - 1) < 1e-12


def test_fp64_horner_within_two_ulp():
    c = np.array(_header_coefficients(), dtype=np.longdouble)
    r = np.linspace(-0.5, 0.5, 20001)
    rl = r.astype(np.longdouble)
    p = np.full(r.shape, c[-1], dtype=np.longdouble)
    for ck in c[-2::-1]:
        p = (p * rl + ck).astype(np.float64).astype(np.longdouble)     # one rounding per fused step
    exact = np.exp2(rl)
    err = np.abs(p - exact) / exact
    assert float(err.max()) < 2 * 2.0 ** -53
