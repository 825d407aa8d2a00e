"""The oracle pins catch plausible mistakes (CPU only).

Each case plants one mistake in a temporary copy of the oracle source (a
dropped term, a wrong sign, a wrong index or parameter), builds it, and runs
a selection of the pins against it: at least one pin must fail.  The
committed oracle is never modified.
"""
from __future__ import annotations

import importlib.util
import os
import subprocess

import pytest

from tests import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "zpo.c")

# (name, text in zpo.c, replacement)
MUTANTS = [
    ("drop_second_derivative_term", "16 * r * r * D[2] - 4 * D[1]", "16 * r * r * D[2]"),
    ("wrong_sign_first_derivative", "g[1] = J >= 1 ? -4 * r * D[1] : 0;", "g[1] = J >= 1 ? 4 * r * D[1] : 0;"),
    ("third_derivative_coefficient", "+ 48 * r * D[2]", "+ 24 * r * D[2]"),
    ("missing_parity_sign", "quad sgn = (K % 2) ? -1 : 1;", "quad sgn = 1;"),
    ("recurrence_coefficient", "quad t2 = 2 * (A - 1) * (B - 1) * c;", "quad t2 = 2 * (A - 1) * B * c;"),
    ("jacobi_argument", "quad x = 1 - 2 * r * r;", "quad x = 1 - r * r;"),
    ("derivative_chain_beta", "jacobi_chain(Kmax - j, alpha + j, j, x,", "jacobi_chain(Kmax - j, alpha + j, 0, x,"),
    ("pochhammer_offset", "pochhammer(alpha + K + 1, j)", "pochhammer(alpha + K, j)"),
    ("leibniz_binomial", "acc += binom_q(j, i) * w[i] * g[j - i];", "acc += w[i] * g[j - i];"),
    ("seed_p1", "quad xm = (x - 1) / 2, xp = (x + 1) / 2, sum = 0;", "quad xm = (x - 1) / 2, xp = (x + 1) / 3, sum = 0;"),
    ("sin_cos_swap", "quad f = mm < 0 ? sn : cs;", "quad f = mm < 0 ? cs : sn;"),
    ("dtheta_sign", "-(quad)a * R * sn", "(quad)a * R * sn"),
]

PINS = [
    pins.test_golden_low_order_polynomials,
    pins.test_golden_center_values,
    pins.test_exact_rational_small_n,
    pins.test_parity_negative_r,
    pins.test_zernike_radial_ode,
    pins.test_basis_angular_factor_vs_mpmath,
]


def _mutant_module(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique/present: {old!r}"
    csrc = tmp_path / f"{name}.c"
    csrc.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", str(csrc), "-lquadmath", "-lm", "-o", str(so)],
                   check=True)
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}", os.path.join(ROOT, "oracle", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._SO = str(so)
    mod._lib = None
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    mod = _mutant_module(tmp_path, name, old, new)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
