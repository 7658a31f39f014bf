"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle's C source, plants one plausible mistake (a
dropped term, a wrong sign, a wrong index, a transposed operand), builds the
copy, and runs the pin suite against it in a subprocess. The pins pass on the
real oracle (test_oracle_pins.py); here every mutant must make them fail.
Everything runs on the CPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "abp_oracle.c")

MUTANTS = {
    "gauss_width_factor": ("exp(-(delta * delta) / (2.0 * sigma * sigma))", "exp(-(delta * delta) / (sigma * sigma))"),
    "gauss_deriv_sign": ("*deriv = -(delta / (sigma * sigma)) * k;", "*deriv = (delta / (sigma * sigma)) * k;"),
    "compact_drop_ep": ("double S = exp((double)p) * exp(-(double)p / one_minus);", "double S = exp(-(double)p / one_minus);"),
    "compact_deriv_factor": ("*deriv = -2.0 * p * delta", "*deriv = -1.0 * p * delta"),
    "wrap_floor": ("return delta - period * nearbyint(delta / period);", "return delta - period * floor(delta / period);"),
    "grad_product_index": ("if (j != i) g *= val[j];", "if (j == i) g *= val[j];"),
    "centers_transposed": ("double ck = centers[(int64_t)i * nh + k];",
                           "double ck = centers[(int64_t)k * d + i];"),
    "snap_truncates": ("double t = floor((x - B->lo[axis]) / node_spacing(B, axis) + 0.5);",
                       "double t = floor((x - B->lo[axis]) / node_spacing(B, axis));"),
    "quantised_hills_not_snapped": ("if (B->quantize) ck = orc_snap(B, i, ck);", "(void)0;"),
    "quantised_stride": ("stride *= (int64_t)B->grid_n[i];", "stride *= (int64_t)B->grid_n[0];"),
    "quantised_query_not_snapped": ("x[i] = B->quantize ? orc_snap(B, i, s[i]) : s[i];", "x[i] = s[i];"),
    "mabp_grad_drop_b": ("dV[i] = c * b * kT * dh[i] / den;", "dV[i] = c * kT * dh[i] / den;"),
    "mabp_value_factor": ("log1p(c * (1.0 - b) * h)", "log1p(c * b * h)"),
    "hermite_basis_term": ("phi[0][1] = t3 - 2 * t2 + t;", "phi[0][1] = t3 - 2 * t2;"),
    "hermite_deriv_scale": ("dphi[i][c][mi] * scale / dx[i]", "dphi[i][c][mi] * scale"),
    "grid_coord_spacing": ("(double)j * (B->hi[axis] - B->lo[axis]) / (double)(n - 1);",
                           "(double)j * (B->hi[axis] - B->lo[axis]) / (double)n;"),
    "grid_stride": ("stride *= B->grid_n[i];", "stride *= B->grid_n[0];"),
    "torsion_grad_sign": ("grad4[3 + c] = (lb2 / nn1 + r1 / (nn1 * lb2))", "grad4[3 + c] = (lb2 / nn1 - r1 / (nn1 * lb2))"),
    "com_mass_swap": ("grad_a[3 * j + c] = ma[j] / MA * u[c];", "grad_a[3 * j + c] = ma[j] / MB * u[c];"),
    "rmsd_offset": ("sqrt(acc / (double)n + 0.01)", "sqrt(acc / (double)n + 0.1)"),
    "force_sign": ("fx[g] += -dV[a] * grad[a][slot][3 * r + 0];", "fx[g] += dV[a] * grad[a][slot][3 * r + 0];"),
    "condition_sum_heights": ("nsum_add(&AH, fabs(w * K));", "nsum_add(&AH, fabs(w));"),
    "condition_sum_gradient": ("nsum_add(&AG[i], fabs(g));", "nsum_add(&AG[i], fabs(w * K));"),
    "neumaier_drop": ("if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;", "if (fabs(a->s) >= fabs(x)) a->c += 0.0;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutated = src.replace(old, new)
    csrc = tmp_path / "abp_oracle.c"
    csrc.write_text(mutated)
    (tmp_path / "abp_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "abp_oracle.h")).read())
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(csrc), "-lm"],
                   check=True)
    env = dict(os.environ, ABP_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
