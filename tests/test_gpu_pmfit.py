"""The polynomial of Eq. (force) regenerated from the library's own PM
(Sec. 2.4 test pairs): GPU samples and fit against the FP64 oracle's, and
the force split closed by it."""
import numpy as np
import pytest
import torch

from oracle import pmfit as OF
from paper_1410_2805_amd import gridfit
from paper_1410_2805_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    from paper_1410_2805_amd import sr as S
    return S


@pytest.fixture(scope="module")
def ctx(sr):
    c = sr.Context(0)
    yield c
    c.close()


def test_samples_and_fit_match_oracle(sr, ctx):
    from paper_1410_2805_amd import pmfit
    sets = W.pm_test_pairs(12, 2048, 64.0, 3.0, 17)
    r, f = pmfit.measure(ctx, 64, sets)
    r0, f0 = OF.radial_samples(sets, 64)
    assert np.array_equal(r, r0)
    rms = np.sqrt((f0 ** 2).mean())
    assert np.all(np.abs(f - f0) <= 1e-5 * rms + 1e-4 * np.abs(f0))
    c, c0 = pmfit.fit(r, f), OF.fit(r0, f0)
    s = np.linspace(0.0, 9.0, 200)
    pg = sum(c[k] * s ** k for k in range(6))
    po = OF.p_of_s(c0, s)
    assert np.abs(pg - po).max() <= 1e-4 * np.abs(po).max()


def test_regenerated_polynomial_closes_the_force_split(sr, ctx):
    """SR (with the polynomial) + PM for orientation-averaged pairs must give
    the softened Newtonian force.  With the polynomial measured from this PM
    the mean residual per separation bin is at the level of the bin's
    scatter, and smaller than with the printed-fit polynomial."""
    from paper_1410_2805_amd import pmfit
    # many sources: the average over source positions inside a grid cell
    # dominates the uncertainty of a bin mean
    c_pm, _ = pmfit.poly_from_pm(ctx, ng=64, nsrc=256, ntest=512, seed=17)
    c_fit = gridfit.poly_coeffs()
    sets = W.pm_test_pairs(256, 512, 64.0, 2.95, 99, r_lo=0.3)
    pmh = sr.PM(ctx, 64, 64.0)
    eps = 1e-6
    box = sr.Box.make(64.0)
    errs = {}
    try:
        for name, c in (("pm", c_pm), ("printed fit", c_fit)):
            rr, rel = [], []
            for s in sets:
                t = [torch.from_numpy(np.ascontiguousarray(s.pos[:, d])).cuda() for d in range(3)]
                m = torch.from_numpy(s.m).cuda()
                a_lr = pmh.force(*t, m)
                a_sr = sr.sr_force(ctx, *t, m, box, 3.0, 3.0, eps, c)[:3]
                ctx.sync()
                a = (torch.stack(a_lr, 1) + torch.stack(a_sr, 1)).double().cpu().numpy()[1:]
                f = -np.einsum("ij,ij->i", a, s.u)
                newton = s.r / (s.r ** 2 + eps) ** 1.5
                rr.append(s.r)
                rel.append(f / newton - 1.0)
            rr, rel = np.concatenate(rr), np.concatenate(rel)
            bins = []
            for lo in np.arange(0.3, 2.95, 0.25):
                sel = (rr >= lo) & (rr < lo + 0.25)
                bins.append((rel[sel].mean(), rel[sel].std() / np.sqrt(sel.sum())))
            errs[name] = bins
        worst_pm = max(abs(m) for m, _ in errs["pm"])
        worst_fit = max(abs(m) for m, _ in errs["printed fit"])
        print("worst bin-mean closure error: PM-derived %.4f, printed fit %.4f"
              % (worst_pm, worst_fit))
        for m, se in errs["pm"]:
            assert abs(m) <= 4 * se + 1e-3
        assert worst_pm < worst_fit
    finally:
        pmh.close()
