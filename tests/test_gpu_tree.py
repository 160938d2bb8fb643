"""RCB-tree short-range variant (Sec. 2.4 RCB tree, Sec. 3.1 trees per bin):
the leaves against the FP64 RCB oracle (exact partition), the forces against
the FP64 force oracle, and agreement with the chaining-mesh pass."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import rcb
from paper_1410_2805_amd import gridfit
from paper_1410_2805_amd import workloads as W
from tests.parity import accel_np, check_accel, to_dev

pytestmark = pytest.mark.gpu

R_MAX, EPS = 3.0, 0.1


@pytest.fixture(scope="module")
def sr():
    from paper_1410_2805_amd import sr as S
    return S


@pytest.fixture(scope="module")
def ctx(sr):
    c = sr.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def poly():
    return gridfit.poly_coeffs()


def _cases():
    out = []
    c = W.nfw_share(20000, 24.0, 3, periodic=True, halo_cap=6000)
    c.m = np.random.default_rng(3).uniform(0.5, 2.0, c.n).astype(np.float32)
    out.append(("clustered periodic, mixed masses", c))
    out.append(("open with skin", W.nfw_share(12000, 21.0, 4, skin=3.0)))
    out.append(("uniform", W.uniform(8000, 18.0, 5)))
    return out


def _sets_from_leaf_of(leaf_of, nleaves):
    groups = [[] for _ in range(nleaves)]
    for i, l in enumerate(leaf_of):
        groups[l].append(i)
    assert all(groups), "empty leaf"
    return sorted(tuple(g) for g in groups)


@pytest.mark.parametrize("leaf_max", [1, 16, 128, 10 ** 6])
def test_leaves_match_oracle(sr, ctx, leaf_max):
    for name, p in _cases():
        t = to_dev(p)
        box = sr.Box.make(p.L, periodic=p.periodic, skin=p.skin)
        leaf_of, nleaves = sr.sr_tree_leaves(ctx, t["x"], t["y"], t["z"], t["m"], box, 3.0,
                                             leaf_max)
        got = _sets_from_leaf_of(leaf_of.cpu().numpy(), nleaves)
        want = sorted(tuple(sorted(int(i) for i in l))
                      for l in rcb.leaves(p.x, p.y, p.z, p.m, p.L, 3.0, leaf_max))
        assert got == want, "%s leaf_max=%d: %d vs %d leaves" % (name, leaf_max, len(got),
                                                                len(want))


@pytest.mark.parametrize("leaf_max", [1, 16, 128])
def test_tree_force_matches_oracle(sr, ctx, poly, leaf_max):
    for name, p in _cases():
        t = to_dev(p)
        box = sr.Box.make(p.L, periodic=p.periodic, skin=p.skin)
        ax, ay, az, mom = sr.sr_force_tree(ctx, t["x"], t["y"], t["z"], t["m"], box, 3.0, R_MAX,
                                           EPS, poly, leaf_max=leaf_max, momentum=True)
        ctx.sync()
        a = accel_np(ax, ay, az)
        ref = O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64),
                      periodic=p.periodic, skin=p.skin)
        check_accel(a, ref, "tree %s leaf_max=%d" % (name, leaf_max))
        want = (p.m.astype(np.float64)[:, None] * a).sum(0)
        assert np.allclose(mom.cpu().numpy(), want, rtol=0, atol=1e-9 * (np.abs(a).sum() + 1))
        # deterministic
        b = sr.sr_force_tree(ctx, t["x"], t["y"], t["z"], t["m"], box, 3.0, R_MAX, EPS, poly,
                             leaf_max=leaf_max)
        ctx.sync()
        assert np.array_equal(accel_np(*b[:3]), a)


def test_tree_and_chaining_mesh_agree(sr, ctx, poly):
    """Both passes sum the same pairs: within float32 rounding of each other
    on a 64^3 Zel'dovich box (the paper's accuracy cross-check)."""
    p = W.zeldovich(64, 64.0, 7, rms=1.5)
    t = to_dev(p)
    box = sr.Box.make(p.L)
    a_tree = accel_np(*sr.sr_force_tree(ctx, t["x"], t["y"], t["z"], t["m"], box, 3.0, R_MAX, EPS,
                                        poly, leaf_max=64)[:3])
    a_mesh = accel_np(*sr.sr_force(ctx, t["x"], t["y"], t["z"], t["m"], box, 3.0, R_MAX, EPS,
                                   poly)[:3])
    ctx.sync()
    err = np.linalg.norm(a_tree - a_mesh, axis=1)
    nrm = np.linalg.norm(a_mesh, axis=1)
    assert np.sqrt((err ** 2).sum() / (nrm ** 2).sum()) < 2e-6
    tg = np.sort(np.random.default_rng(1).choice(p.n, 1024, replace=False))
    ref = O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64), targets=tg)
    check_accel(a_tree[tg], ref, "tree zeldovich64")


def test_tree_empty_and_bad_arguments(sr, ctx, poly):
    e = torch.zeros(0, dtype=torch.float32, device="cuda:0")
    ax, ay, az, _ = sr.sr_force_tree(ctx, e, e, e, e, sr.Box.make(12.0), 3.0, R_MAX, EPS, poly)
    ctx.sync()
    assert ax.numel() == 0
    p = W.uniform(500, 12.0, 2)
    t = to_dev(p)
    for lm in (0, 2 ** 21):
        with pytest.raises(sr.SRError):
            sr.sr_force_tree(ctx, t["x"], t["y"], t["z"], t["m"], sr.Box.make(12.0), 3.0, R_MAX,
                             EPS, poly, leaf_max=lm)


@pytest.mark.slow
def test_tree_zeldovich128_sampled(sr, ctx, poly):
    """The full 128^3 Zel'dovich box through the tree pass, sampled targets."""
    p = W.config("zeldovich128")
    t = to_dev(p)
    a = accel_np(*sr.sr_force_tree(ctx, t["x"], t["y"], t["z"], t["m"], sr.Box.make(p.L), 3.0,
                                   R_MAX, EPS, poly, leaf_max=128)[:3])
    ctx.sync()
    tg = np.sort(np.random.default_rng(77).choice(p.n, 2048, replace=False))
    ref = O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64), targets=tg)
    check_accel(a[tg], ref, "tree zeldovich128")


@pytest.mark.slow
def test_tree_nfw256_sampled(sr, ctx, poly):
    """The 256^3 clustered open share through the tree pass (leaf 128),
    targets half from the densest cells, where the trees are deep."""
    p = W.config("nfw256")
    t = to_dev(p)
    box = sr.Box.make(p.L, periodic=False, skin=p.skin)
    a = accel_np(*sr.sr_force_tree(ctx, t["x"], t["y"], t["z"], t["m"], box, 3.0, R_MAX, EPS,
                                   poly, leaf_max=128)[:3])
    ctx.sync()
    rng = np.random.default_rng(78)
    _, _, cid = O.bin(p.x, p.y, p.z, 256.0, 3.0)
    counts = np.bincount(cid)
    dense = np.nonzero(counts[cid] >= np.sort(counts)[-50])[0]
    tg = np.unique(np.concatenate([rng.choice(p.n, 128, replace=False),
                                   rng.choice(dense, 128, replace=False)]))
    ref = O.force(p.x, p.y, p.z, p.m, p.L, R_MAX, EPS, poly.astype(np.float64), periodic=False,
                  skin=p.skin, targets=tg)
    check_accel(a[tg], ref, "tree nfw256")
