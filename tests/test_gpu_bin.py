"""sr_bin on the GPU against the oracle's stable counting sort: bit-exact
cell_offsets and perm."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
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


def _bin_both(sr, ctx, x, y, z, L, cell, periodic=True):
    dev = "cuda:0"
    tx, ty, tz = (torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(dev)
                  for v in (x, y, z))
    box = sr.Box.make(L, periodic=periodic)
    off, perm = sr.sr_bin(ctx, tx, ty, tz, box, cell)
    ctx.sync()
    o_off, o_perm, _ = O.bin(x, y, z, L, cell)
    return off.cpu().numpy(), perm.cpu().numpy(), o_off, o_perm


def _assert_same(off, perm, o_off, o_perm):
    assert off.shape == o_off.shape and np.array_equal(off, o_off)
    assert perm.shape == o_perm.shape and np.array_equal(perm, o_perm)


def test_uniform_32k(sr, ctx):
    p = W.config("uniform32")
    _assert_same(*_bin_both(sr, ctx, p.x, p.y, p.z, 32.0, 3.0))


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 129, 500, 1000, 1024, 1025, 3000, 40896, 40897, 70000])
def test_one_cell_sizes(sr, ctx, n):
    """Every particle in one cell: exercises the register, LDS and
    multi-run merge paths of the per-cell sort (a whole-block sort in LDS up
    to 40896 particles, runs merged through global memory beyond)."""
    rng = np.random.default_rng(n)
    x = (rng.random(n) * 2.9).astype(np.float32)
    y = (3.0 + rng.random(n) * 2.9).astype(np.float32)
    z = (rng.random(n) * 2.9).astype(np.float32)
    _assert_same(*_bin_both(sr, ctx, x, y, z, 12.0, 3.0))


def test_mixed_cell_sizes(sr, ctx):
    """Cells of 0..5000 particles side by side, random input order."""
    rng = np.random.default_rng(9)
    sizes = [0, 1, 5, 64, 65, 200, 1024, 1025, 2047, 4097, 5000]
    pts = []
    for k, s in enumerate(sizes):
        c = np.array([k % 5, (k // 5) % 5, k // 25], dtype=np.float64) * 3.0
        pts.append(c + rng.random((s, 3)) * 2.999)
    pos = np.concatenate(pts)
    pos = pos[rng.permutation(pos.shape[0])].astype(np.float32)
    _assert_same(*_bin_both(sr, ctx, pos[:, 0], pos[:, 1], pos[:, 2], 15.0, 3.0))


def test_large_cells_side_by_side(sr, ctx):
    """Several cells of 1025..50000 particles in one box, random input order:
    large cells sorted by different blocks, in LDS and through global memory."""
    rng = np.random.default_rng(11)
    sizes = [1025, 12000, 40896, 40897, 25000, 2049, 50000, 20480, 20481]
    pts = []
    for k, s in enumerate(sizes):
        c = np.array([k % 4, (k // 4) % 4, k // 16], dtype=np.float64) * 3.0
        pts.append(c + rng.random((s, 3)) * 2.999)
    pos = np.concatenate(pts)
    pos = pos[rng.permutation(pos.shape[0])].astype(np.float32)
    _assert_same(*_bin_both(sr, ctx, pos[:, 0], pos[:, 1], pos[:, 2], 12.0, 3.0))


def test_cell_edges_and_top(sr, ctx):
    f32 = np.float32
    xs = []
    for k in range(8):
        xs += [f32(4 * k), np.nextafter(f32(4 * k), f32(0)) if k else f32(0)]
    xs += [np.nextafter(f32(32.0), f32(0))] * 3
    x = np.array(xs, dtype=np.float32)
    y = x[::-1].copy()
    z = np.roll(x, 3)
    _assert_same(*_bin_both(sr, ctx, x, y, z, 32.0, 4.0))
    # non-integer cell width: L = 10, n_c = 3
    rng = np.random.default_rng(1)
    v = (rng.random((5000, 3)) * 10).astype(np.float32)
    v[v >= 10] = 0
    _assert_same(*_bin_both(sr, ctx, v[:, 0], v[:, 1], v[:, 2], 10.0, 3.0))


def test_out_of_range_reported(sr, ctx):
    x = np.array([1.0, 5.0, 32.0], dtype=np.float32)
    y = np.ones(3, np.float32)
    dev = "cuda:0"
    t = [torch.from_numpy(v).to(dev) for v in (x, y, y)]
    sr.sr_bin(ctx, *t, sr.Box.make(32.0), 4.0)
    with pytest.raises(sr.SRError) as e:
        ctx.sync()
    assert e.value.code == sr.SR_ERANGE
    t[0][2] = float("nan")
    sr.sr_bin(ctx, *t, sr.Box.make(32.0), 4.0)
    with pytest.raises(sr.SRError):
        ctx.sync()
    ctx.sync()  # status cleared


def test_zeldovich_128(sr, ctx):
    p = W.config("zeldovich128")
    _assert_same(*_bin_both(sr, ctx, p.x, p.y, p.z, 128.0, 3.0))


def test_nfw_256(sr, ctx):
    """The 256^3 clustered share (radix path: 2^22 particles or more)."""
    p = W.config("nfw256")
    off, perm, o_off, o_perm = _bin_both(sr, ctx, p.x, p.y, p.z, 256.0, 3.0, periodic=False)
    _assert_same(off, perm, o_off, o_perm)
    assert np.diff(off).max() > 1025  # cells of more than 1024 particles


@pytest.mark.parametrize("case", ["uniform", "one_cell", "cell_order", "two_cells"])
def test_radix_path(sr, ctx, case):
    """Passes of at least 2^22 particles bin by a stable radix sort of the
    cell ids (three 8-bit passes for 10^6 cells): bit-exact against the
    oracle's counting sort with a ragged count (2^22 + 123), many empty
    cells, every particle in one cell, input already in cell order, and two
    cells of interleaved particles (every digit pass sees one or two
    digits)."""
    n = (1 << 22) + 123
    L = 300.0
    rng = np.random.default_rng(len(case))
    if case == "one_cell":
        v = rng.random((n, 3)) * 2.9
    elif case == "two_cells":
        v = rng.random((n, 3)) * 2.9
        v[1::2, 0] += 3.0 * 77
    else:
        v = np.minimum(rng.random((n, 3)) * L, np.float32(299.99))
    x, y, z = (np.ascontiguousarray(v[:, k], dtype=np.float32) for k in range(3))
    if case == "cell_order":
        _, o_perm, _ = O.bin(x, y, z, L, 3.0)
        x, y, z = x[o_perm], y[o_perm], z[o_perm]
    print("case:", case, n, flush=True)
    _assert_same(*_bin_both(sr, ctx, x, y, z, L, 3.0))


def test_permute_keeps_cell_order(sr, ctx):
    """sr_permute re-orders attributes by sr_bin's permutation (4-, 8- and
    16-byte elements against numpy's fancy indexing); binning the re-ordered
    particles again gives the same offsets and the identity permutation."""
    rng = np.random.default_rng(21)
    n = 50_000
    x, y, z = (rng.random(n, dtype=np.float32) * np.float32(29.9) for _ in range(3))
    dev = "cuda:0"
    tx, ty, tz = (torch.from_numpy(v).to(dev) for v in (x, y, z))
    box = sr.Box.make(30.0)
    off, perm = sr.sr_bin(ctx, tx, ty, tz, box, 3.0)
    ids = torch.arange(n, dtype=torch.int32, device=dev) * 7
    d64 = torch.from_numpy(rng.random(n)).to(dev)
    c128 = torch.from_numpy(rng.random(n) + 1j * rng.random(n)).to(dev)
    outs = [sr.sr_permute(ctx, perm, t) for t in (tx, ty, tz, ids, d64, c128)]
    ctx.sync()
    p = perm.cpu().numpy()
    for t, o in zip((tx, ty, tz, ids, d64, c128), outs):
        assert np.array_equal(o.cpu().numpy(), t.cpu().numpy()[p])
    off2, perm2 = sr.sr_bin(ctx, outs[0], outs[1], outs[2], box, 3.0)
    ctx.sync()
    assert np.array_equal(off2.cpu().numpy(), off.cpu().numpy())
    assert np.array_equal(perm2.cpu().numpy(), np.arange(n, dtype=np.int32))


def test_permute_errors(sr, ctx):
    dev = "cuda:0"
    a = torch.arange(8, dtype=torch.float32, device=dev)
    bad = torch.tensor([0, 1, 2, 3, 4, 5, 6, 8], dtype=torch.int32, device=dev)
    out = sr.sr_permute(ctx, bad, a)
    with pytest.raises(sr.SRError) as e:
        ctx.sync()
    assert e.value.code == sr.SR_ERANGE
    assert out[7].item() == 0.0 and out[:7].cpu().tolist() == list(range(7))
    ctx.sync()  # status cleared
    perm = torch.arange(8, dtype=torch.int32, device=dev)
    with pytest.raises(sr.SRError):
        sr.sr_permute(ctx, perm, a, out=a)  # in place is refused
    with pytest.raises(sr.SRError):
        sr.sr_permute(ctx, perm, torch.zeros(8, dtype=torch.int16, device=dev))  # 2-byte elements


def test_invalid_args(sr, ctx):
    t = torch.zeros(4, device="cuda:0")
    with pytest.raises(sr.SRError):
        sr.sr_bin(ctx, t, t, t, sr.Box.make(32.0), -1.0)
    with pytest.raises(sr.SRError):
        sr.sr_bin(ctx, t, t, t, sr.Box.make(float(np.float64(1) / 3)), 0.1)
