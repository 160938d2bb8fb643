"""CPU-side checks of the C ABI: the library loads, exports every entry
point the header declares, and its host-only geometry calls behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    inc = os.path.join(ROOT, "include")
    txt = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc))
                  if f.endswith(".h"))
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1410_2805_amd import sr
    lib = ctypes.CDLL(sr.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(sr.exported_symbols()) <= set(names)


def test_grid_dims_and_scratch():
    from paper_1410_2805_amd import sr
    dims, nc = sr.sr_grid_dims(sr.Box.make(128.0), 3.0)
    assert dims == (42, 42, 42) and nc == 42 ** 3
    dims, nc = sr.sr_grid_dims(sr.Box.make((32.0, 64.0, 9.0)), 3.0)
    assert dims == (10, 21, 3) and nc == 630
    with pytest.raises(sr.SRError):
        sr.sr_grid_dims(sr.Box.make(2.0), 3.0)
    with pytest.raises(sr.SRError):
        sr.sr_grid_dims(sr.Box.make(10.0), 0.0)
    b1 = sr.sr_scratch_bytes(sr.Box.make(128.0), 3.0, 2 ** 21, True)
    b0 = sr.sr_scratch_bytes(sr.Box.make(128.0), 3.0, 2 ** 21, False)
    # up to 2^22 particles a force pass may cut long chunks into sub-items:
    # partial sums of 7 x 16 B per particle
    assert b1 > b0 + 7 * 16 * 2 ** 21
    assert b0 > 2 ** 21 * 8
    # the multilevel step adds target counts, levels, mask and cell counts
    b2 = sr.sr_scratch_bytes(sr.Box.make(128.0), 3.0, 2 ** 21, 2)
    assert b2 > b1 + 2 * 2 ** 21
    # beyond 2^22 particles only the masked passes of the multilevel step do
    big0 = sr.sr_scratch_bytes(sr.Box.make(256.0), 3.0, 2 ** 23, False)
    big1 = sr.sr_scratch_bytes(sr.Box.make(256.0), 3.0, 2 ** 23, True)
    big2 = sr.sr_scratch_bytes(sr.Box.make(256.0), 3.0, 2 ** 23, 2)
    assert big0 < big1 < big0 + 48 * 2 ** 23
    assert big2 > big1 + 7 * 16 * 2 ** 23
    # box sides are bounded so that tile padding (at 1e6) stays beyond every cutoff
    assert sr.sr_scratch_bytes(sr.Box.make((131072.0, 12.0, 12.0)), 3.0, 1000, True) > 0
    with pytest.raises(sr.SRError):
        sr.sr_scratch_bytes(sr.Box.make((131073.0, 12.0, 12.0)), 3.0, 1000, True)


def test_quanta_fixed_point_rounding():
    """The pair loop rounds a tile's kept count n (0..256) up to a multiple
    of the slice quantum q = 4 S (S = 1..16) with a 16-bit fixed-point
    reciprocal r = ceil(2^16 / q): ((n + q - 1) r) >> 16 = ceil(n / q) over
    every q up to 64 (quanta_of in sr_pair.h)."""
    for q in range(1, 65):
        r = (65536 + q - 1) // q
        for n in range(0, 257):
            assert ((n + q - 1) * r) >> 16 == -(-n // q), (n, q)


def test_null_context_is_rejected():
    from paper_1410_2805_amd import sr
    assert sr.lib.sr_sync(None) == sr.SR_EINVAL
    assert sr.lib.sr_ctx_destroy(None) == sr.SR_EINVAL
    assert sr.lib.sr_bin(None, None, None, None, 0, None, 3.0, None, None) == sr.SR_EINVAL


def test_lane_group_fixed_point_division():
    """lane // ln from a 16-bit fixed-point reciprocal, for every lane of a
    wavefront and every lane-group length (lane_group in sr_pair.h)."""
    for ln in range(1, 65):
        r = (65536 + ln - 1) // ln
        for lane in range(64):
            assert (lane * r) >> 16 == lane // ln, (lane, ln)


def test_cell_decode_division_constants():
    """Cell decoding divides by nc[0] nc[1] and nc[0] with multiply-shift
    constants (div_const in sr_internal.h): s = ceil(log2 d), m =
    floor(2^(31+s) / d) + 1 must fit 32 bits and give floor(n / d) for all
    0 <= n < 2^31."""
    import numpy as np
    rng = np.random.default_rng(5)
    divisors = list(range(1, 5000)) + [2 ** k for k in range(31)] + \
        [2 ** k + 1 for k in range(1, 31)] + [2 ** k - 1 for k in range(2, 31)] + \
        [int(v) for v in rng.integers(1, 2 ** 31 - 1, 2000)]
    for d in divisors:
        s = 0
        while (1 << s) < d:
            s += 1
        m = (1 << (31 + s)) // d + 1
        assert m < 2 ** 32, d
        ns = [0, 1, d - 1, d, d + 1, 2 ** 31 - 1, 2 ** 31 - 2, (2 ** 31 - 1) // d * d,
              (2 ** 31 - 1) // d * d - 1] + [int(v) for v in rng.integers(0, 2 ** 31, 64)]
        for n in ns:
            if 0 <= n < 2 ** 31:
                assert (n * m) >> (31 + s) == n // d, (n, d)


def test_ordered_key_preserves_float_order():
    """The target box is reduced on int32 keys b ^ ((b >> 31) & 0x7fffffff) of
    the float bits b (ordered_key in sr_pair.h): integer order must be float
    order over finite floats of both signs, and the map its own inverse."""
    import numpy as np
    rng = np.random.default_rng(11)
    f = np.concatenate([rng.uniform(-300.0, 300.0, 20000), rng.normal(0.0, 1e-3, 5000),
                        [0.0, -0.0, 1e-45, -1e-45, 131072.0, -131072.0, 3.4e38, -3.4e38]])
    f = f.astype(np.float32)
    b = f.view(np.int32)
    key = b ^ ((b >> 31) & np.int32(0x7fffffff))
    order = np.argsort(f, kind="stable")
    fs, ks = f[order], key[order]
    # wherever the floats increase the keys increase (only -0 and +0 tie
    # as floats; their keys are -1 and 0)
    strict = np.diff(fs) > 0
    assert np.all(np.diff(ks.astype(np.int64))[strict] > 0)
    back = key ^ ((key >> 31) & np.int32(0x7fffffff))
    assert np.array_equal(back, b)
