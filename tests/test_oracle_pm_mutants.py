"""The PM and step pins must catch plausible mistakes in the PM oracle.

Each case plants one mistake in a copy of the PM oracle's source (a dropped
factor, a wrong coefficient, sign, weight or time step), loads it as a fresh
module, points the pin module at it and runs the pins: at least one must
fail.  CPU only."""
import importlib.util

import pytest

from oracle import pm
import tests.test_oracle_pm_pins as P

SRC = pm.__file__

MUTANTS = [
    ("no filter", "out = out * sc ** ns", "out = out * 1.0"),
    ("filter power", "out = out * sc ** ns", "out = out * sc ** (ns - 1)"),
    ("gaussian width", "np.exp(-k2 * sd * sd / 4.0)", "np.exp(-k2 * sd * sd / 2.0)"),
    ("sigma in length units", "sd = sigma * d", "sd = sigma"),
    ("G6 second weight", "(5.0 / 64.0) * np.cos(2 * kc * d)", "(5.0 / 32.0) * np.cos(2 * kc * d)"),
    ("G6 constant", "s = s - 2835.0 / 1024.0", "s = s - 2836.0 / 1024.0"),
    ("G6 normalisation", "(45.0 / 128.0) * d * d / s", "(45.0 / 64.0) * d * d / s"),
    ("lanczos second term", "- (1.0 / 6.0) * np.sin(2.0 * kc * d)", "- (1.0 / 3.0) * np.sin(2.0 * kc * d)"),
    ("gradient sign", "np.fft.irfftn(-sl_derivative", "np.fft.irfftn(sl_derivative"),
    ("no 4 pi", "phi_k = 4.0 * np.pi * green6", "phi_k = 1.0 * green6"),
    ("CIC weights swapped", "wx = f[:, 0] if cx else 1.0 - f[:, 0]\n        ix = i1[:, 0] if cx else i0[:, 0]\n        for cy in (0, 1):\n            wy = f[:, 1] if cy else 1.0 - f[:, 1]\n            iy = i1[:, 1] if cy else i0[:, 1]\n            for cz in (0, 1):\n                wz = f[:, 2] if cz else 1.0 - f[:, 2]\n                iz = i1[:, 2] if cz else i0[:, 2]\n                out",
     "wx = 1.0 - f[:, 0] if cx else f[:, 0]\n        ix = i1[:, 0] if cx else i0[:, 0]\n        for cy in (0, 1):\n            wy = f[:, 1] if cy else 1.0 - f[:, 1]\n            iy = i1[:, 1] if cy else i0[:, 1]\n            for cz in (0, 1):\n                wz = f[:, 2] if cz else 1.0 - f[:, 2]\n                iz = i1[:, 2] if cz else i0[:, 2]\n                out"),
    ("density not per volume", "return rho / d ** 3", "return rho"),
    ("subcycle length", "tau = dt / nsub", "tau = dt"),
    ("stale long-range force", "    a_lr = pm_accel(pos, m, ng, L, sigma, ns)\n    vel = vel + 0.5 * dt * a_lr\n    return",
     "    vel = vel + 0.5 * dt * a_lr\n    return"),
    ("full first kick", "vel = vel + 0.5 * dt * a_lr\n    tau", "vel = vel + dt * a_lr\n    tau"),
]

PINS = [
    P.test_green6_sixth_order_along_an_axis,
    P.test_super_lanczos_fourth_order,
    P.test_filter_limits,
    P.test_grid_unit_scaling,
    P.test_cic_identities,
    P.test_newton_third_law_and_no_self_force,
    lambda: [P.test_test_pair_reproduces_fitform(r) for r in (1.0, 3.0)],
    P.test_ksk_free_particle_and_reversibility,
    P.test_ksk_second_order_against_fine_leapfrog,
]


def _load_mutant(name, old, new):
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) >= 1, "mutation site not found: %s" % name
    mod_name = "pm_mutant_%d" % abs(hash(name))
    spec = importlib.util.spec_from_loader(mod_name, loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__file__ = SRC
    exec(compile(src.replace(old, new, 1), SRC, "exec"), mod.__dict__)
    return mod


def test_unmutated_passes():
    for pin in PINS:
        pin()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(monkeypatch, name, old, new):
    mod = _load_mutant(name, old, new)
    monkeypatch.setattr(P, "pm", mod)
    caught = False
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            caught = True
            break
    assert caught, "no pin catches: %s" % name
