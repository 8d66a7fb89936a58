"""The pins of the error estimates detect plausible mistakes.

Each case copies the oracle's C source, plants one mistake (a wrong index or
factor in an estimate), builds the copy with the oracle's own compiler flags
and runs the corresponding pin against it: the pin must fail.  The planted
copies live in a temporary directory; the oracle itself is untouched.
"""
import os
import subprocess

import pytest

from tests import test_oracle_error_estimates as E

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "bdf_oracle.c")

MUTATIONS = [
    # error constant of the accepted step: xi_q in place of xi_{q+1}
    ("cerr_xi_index", "*Cerr = 1.0 / (l[1] * xi[q + 1]);", "*Cerr = 1.0 / (l[1] * xi[q]);",
     [E.check_local_error_constant_from_exact_history,
      E.check_local_error_estimate_in_a_running_integration]),
    # order q-1 estimate: factorial and harmonic number off by one
    ("lower_factorial", "orc_factorial(q - 1) / orc_harmonic(q - 1)",
     "orc_factorial(q) / orc_harmonic(q - 1)", [E.check_lower_order_estimate]),
    ("lower_harmonic", "orc_factorial(q - 1) / orc_harmonic(q - 1)",
     "orc_factorial(q - 1) / orc_harmonic(q)", [E.check_lower_order_estimate]),
    # order q+1 estimate: harmonic number and leading factor off by one
    ("higher_harmonic", "((q + 2) * orc_harmonic(q + 1))", "((q + 2) * orc_harmonic(q))",
     [E.check_higher_order_estimate]),
    ("higher_factor", "((q + 2) * orc_harmonic(q + 1))", "((q + 1) * orc_harmonic(q + 1))",
     [E.check_higher_order_estimate]),
    # initial step: the safety factor 0.5 dropped; the interval bound 0.1 changed
    ("initial_half", "double h0 = 0.5 * hnew;", "double h0 = hnew;", [E.check_initial_step]),
    ("initial_bound", "double hub = 0.1 * tdist;", "double hub = 0.2 * tdist;",
     [E.check_initial_step]),
]


def _build_variant(tmp_path, name, old, new):
    with open(SRC) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"{name}: the text to change must occur once"
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", str(so), str(c), "-lm"], check=True)
    return str(so)


@pytest.mark.parametrize("name,old,new,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_detected(oracle, tmp_path, name, old, new, checks):
    path = _build_variant(tmp_path, name, old, new)
    with oracle.use_library(path):
        for check in checks:
            with pytest.raises(AssertionError):
                check(oracle)
    # the unmodified oracle passes the same checks
    for check in checks:
        check(oracle)
