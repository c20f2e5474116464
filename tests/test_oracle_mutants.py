"""The pins catch plausible mistakes: each test plants one mistake in a copy
of the oracle's C source (compiled into a temporary directory, on the CPU) and
checks that the hand-derived worked examples reject the planted copy while
they accept the oracle itself.

Planted mistakes (each a one-line change of the evaluation step):
  uniform_average     the epoch average weights every iterate by 1 instead of
                      its step size (Algorithm 1);
  omega_not_squared   KKT_omega weighs the residuals by omega and 1/omega
                      instead of omega^2 and 1/omega^2 (eq. (kkt));
  inverted_candidate  the restart candidate is the iterate with the larger
                      KKT_omega (Section 3.4);
  kkt0_old_weight     after a restart KKT_0 keeps the value computed with the
                      old primal weight instead of being recomputed with the
                      new one (Algorithm 1 with the Section 2.2 update).
"""
import os
import subprocess

import pytest

import oracle
from tests.test_oracle_pins import check_evaluation_golden

SRC = os.path.join(os.path.dirname(oracle.__file__), "pdlp_oracle.c")

MUTANTS = {
    "uniform_average": [("sum_eta += eta;", "sum_eta += 1.0;"),
                        ("xs[j] += eta * x[j];", "xs[j] += x[j];"),
                        ("ys[i] += eta * y[i];", "ys[i] += y[i];")],
    "omega_not_squared": [("double w = power == 1 ? omega : omega * omega;", "double w = omega;")],
    "inverted_candidate": [("int cand_avg = !(kc_cur < kc_avg - 1e-12 * kc_avg);",
                            "int cand_avg = (kc_cur < kc_avg - 1e-12 * kc_avg);")],
    "kkt0_old_weight": [("kkt0 = o.restart_metric == 1 ? kc : kkt_omega(cand_avg ? ea.scaled : ec.scaled, omega, "
                         "o.kkt_omega_power);", "kkt0 = kc;")],
}


def _build_mutant(tmp_path, name):
    text = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert text.count(old) == 1, f"mutation site not found: {old}"
        text = text.replace(old, new)
    src = tmp_path / f"{name}.c"
    lib = tmp_path / f"lib{name}.so"
    src.write_text(text)
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
                           "-D_POSIX_C_SOURCE=200809L", "-I", os.path.dirname(SRC), "-o", str(lib), str(src),
                           "-lm"])
    return str(lib)


@pytest.fixture
def swap(monkeypatch):
    def use(path):
        oracle.lib()
        monkeypatch.setattr(oracle, "_LIB", path)
        monkeypatch.setattr(oracle, "_lib", None)
        monkeypatch.setattr(oracle, "build", lambda force=False: path)
        lib = oracle.lib()
        assert lib._name == path
        return oracle
    return use


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_worked_examples_reject_planted_mistake(tmp_path, swap, name):
    mutant = swap(_build_mutant(tmp_path, name))
    failures = 0
    for case in ("A", "B"):
        try:
            check_evaluation_golden(mutant, case)
        except AssertionError:
            failures += 1
    assert failures >= 1, f"the planted mistake '{name}' passes every worked example"


def test_worked_examples_accept_the_oracle(orc):
    for case in ("A", "B"):
        check_evaluation_golden(orc, case)
