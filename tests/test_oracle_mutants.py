"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of oracle.c (a wrong power, sign,
index, cutoff, image or rounding rule), builds it into a temporary library,
points the oracle front end at it and runs the pins: at least one must fail.
Everything here runs on the CPU."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import pytest

from oracle import oracle as O
import tests.test_oracle_pins as P

SRC = os.path.join(os.path.dirname(O.__file__), "oracle.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("power of s in p", "sk *= s;", "sk *= s * s;"),
    ("sign of p", "1.0 / (se * sqrt(se)) - poly5(poly, s)", "1.0 / (se * sqrt(se)) + poly5(poly, s)"),
    ("softening on r", "double se = s + eps;", "double se = s + sqrt(eps);"),
    ("Plummer exponent", "1.0 / (se * sqrt(se))", "1.0 / (se * se)"),
    ("cutoff not strict", "if (s < r2) {", "if (s <= r2) {"),
    ("source mass index", "double w = m[j] * f;", "double w = m[i] * f;"),
    ("image threshold", "if (d[k] > 0.5 * L[k])", "if (d[k] > L[k])"),
    ("separation sign", "double d[3] = {x[j] - pi[0], y[j] - pi[1], z[j] - pi[2]};",
     "double d[3] = {pi[0] - x[j], pi[1] - y[j], pi[2] - z[j]};"),
    ("cell rounding", "double t = floor(x * inv);", "double t = floor(x * inv + 0.5);"),
    ("unstable scatter", "for (int64_t i = 0; i < n; ++i)\n        perm[count[id[i]]++] = (int32_t)i;",
     "for (int64_t i = n - 1; i >= 0; --i)\n        perm[count[id[i]]++] = (int32_t)i;"),
    ("passive not strict", "if (lo < skin || hi < skin)", "if (lo <= skin || hi <= skin)"),
    ("kick before stream", "V[d][i] += dt * a[d * n + i];", "V[d][i] += 0.5 * dt * a[d * n + i];"),
    ("abs sum without |d|", "double mag = fabs(w) * sqrt(s);", "double mag = fabs(w);"),
    ("tie band too wide", "const double band = r2 * ldexp(1.0, -18);",
     "const double band = r2 * ldexp(1.0, -8);"),
]

PINS = [
    lambda: [P.test_newtonian_limit(r, (0.3, -0.4, 0.866)) for r in (0.01, 1.0)],
    lambda: [P.test_plummer_term_is_gradient_of_plummer_potential(r) for r in (0.3, 1.0)],
    lambda: [P.test_short_range_is_newton_minus_paper_grid_force(r) for r in (0.5, 1.5, 2.5)],
    P.test_cutoff_strict_and_zero_beyond,
    P.test_minimum_image,
    P.test_lattice_symmetry_and_shell_counts,
    P.test_newton_third_law_and_translation,
    P.test_passive_skin_rule,
    P.test_bin_matches_library_stable_sort,
    P.test_bin_exact_cell_edges,
    P.test_sks_free_streaming_and_reversibility,
    P.test_sks_one_step_closed_form,
    lambda: [P.test_abs_sum_two_particles_closed_form(r, mj) for r, mj in ((0.5, 2.0), (2.9, 4.0))],
    P.test_abs_sum_three_particles_closed_form,
    lambda: [P.test_tie_band_membership(s) for s in (-1.0, 1.0)],
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _build(src_text, path):
    c = path + ".c"
    with open(c, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c99", "-shared",
                           "-fPIC", "-o", path, c, "-lm"])


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(workdir, name, orig, bad):
    text = open(SRC).read()
    assert text.count(orig) == 1, "mutation anchor not found: %s" % name
    lib_path = os.path.join(workdir, "mut_%d.so" % MUTANTS.index((name, orig, bad)))
    _build(text.replace(orig, bad), lib_path)
    saved_lib, saved_path = O._lib, O._LIB
    try:
        O._lib = None
        O._LIB = lib_path
        O._load()
        caught = []
        for pin in PINS:
            try:
                pin()
            except (AssertionError, ValueError):
                caught.append(pin)
        assert caught, "no pin caught the planted mistake: %s" % name
    finally:
        O._lib, O._LIB = saved_lib, saved_path


def test_unmutated_copy_passes_all_pins(workdir):
    """Control: the same harness on an unmodified copy catches nothing."""
    lib_path = os.path.join(workdir, "control.so")
    _build(open(SRC).read(), lib_path)
    saved_lib, saved_path = O._lib, O._LIB
    try:
        O._lib = None
        O._LIB = lib_path
        O._load()
        for pin in PINS:
            pin()
    finally:
        O._lib, O._LIB = saved_lib, saved_path
