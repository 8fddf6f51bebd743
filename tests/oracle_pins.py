"""Pins of the oracle to facts outside the oracle itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
when the oracle disagrees with what mathematics or an independent library
routine fixes.  ``test_oracle_pins.py`` runs them on the real oracle and
``test_oracle_mutants.py`` runs them on deliberately broken copies of it, to
show that a plausible mistake anywhere in the oracle fails at least one pin.

What pins what:
  * mean / m2 / std: a textbook worked example (golden file), exact rational
    arithmetic with ``fractions`` and the ``statistics`` module, closed forms
    of constant and integer-ramp cubes, the merge identity of two halves, and
    numpy's extended-real mean and std for boxes holding +-Inf.
  * min / max / NaN count: numpy's nanmin / nanmax / isnan, signed zeros by
    bit pattern, all-NaN, single voxel, NaN payloads.
  * histogram: closed forms (integer ramp with power-of-two bin width;
    unit-width bins equal numpy.floor), hand-derived edge and subnormal cases,
    an exact-rational model of IEEE-754 binary32 rounding applied to the bin
    rule, numpy.histogram as a loose cross-check, and the counting invariants.
"""
from __future__ import annotations

import math
import os
import statistics
from fractions import Fraction

import warnings

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def f32(x) -> np.float32:
    return np.float32(x)


def bits_f32(u: int) -> np.float32:
    return np.array([u], dtype=np.uint32).view(np.float32)[0]


def signbit(x) -> bool:
    return bool(np.signbit(np.float32(x)))


# ------------------------------------------------------------------ moments
def pin_textbook(o):
    vals, want = None, {}
    with open(os.path.join(GOLDEN, "textbook_std.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split(":", 1)
            if k == "values":
                vals = np.array([float(t) for t in v.split()], dtype=np.float32)
            else:
                want[k] = float(v)
    s = o.stats(vals)
    assert s.n_valid == len(vals) and s.n_nan == 0
    assert s.mean == want["mean"], s.mean
    assert s.m2 == want["m2"], s.m2
    assert s.std == want["std"], s.std


def _exact(vals):
    fr = [Fraction(float(v)) for v in vals if not math.isnan(v)]
    mean = statistics.mean(fr)                 # exact on Fractions
    pvar = statistics.pvariance(fr)            # exact on Fractions
    return fr, mean, pvar * len(fr), pvar


def pin_exact_rational(o):
    rng = np.random.default_rng(1)
    shapes = [(1, 1, 1), (2, 1, 1), (3, 2, 1), (7, 5, 3), (17, 13, 11), (64, 9, 2)]
    for i, (nx, ny, nz) in enumerate(shapes):
        a = (rng.standard_normal((nz, ny, nx)) * 10 ** rng.uniform(-3, 3)
             + rng.uniform(-100, 100)).astype(np.float32)
        if a.size > 4:
            a.reshape(-1)[rng.random(a.size) < 0.1] = np.nan
        fr, mean, m2, pvar = _exact(a.reshape(-1))
        s = o.stats(a)
        assert s.n_valid == len(fr) and s.n_nan == a.size - len(fr)
        mabs = float(sum(abs(x) for x in fr) / len(fr))
        assert abs(s.mean - float(mean)) <= 1e-15 * mabs + 1e-300, (i, s.mean, float(mean))
        assert abs(s.mean_abs - mabs) <= 1e-15 * mabs
        if m2 == 0:
            assert s.m2 == 0.0
        else:
            assert abs(s.m2 - float(m2)) <= 1e-13 * float(m2), (i, s.m2, float(m2))
            assert abs(s.std - math.sqrt(pvar)) <= 1e-14 * math.sqrt(pvar)


def pin_closed_forms(o):
    for c in (0.0, -3.25, 1e4, 123456.0, 3e-30):
        a = np.full((5, 6, 7), c, dtype=np.float32)
        s = o.stats(a)
        assert s.mean == float(np.float32(c)) and s.m2 == 0.0 and s.std == 0.0
    # integer ramp a + b*i, exactly representable in float32
    for (a0, b, n) in ((-3.0, 0.5, 100_000), (1000.0, 1.0, 4097), (0.0, -2.0, 12345)):
        v = (a0 + b * np.arange(n, dtype=np.float64)).astype(np.float32)
        assert np.all(v.astype(np.float64) == a0 + b * np.arange(n))
        s = o.stats(v)
        mean = a0 + b * (n - 1) / 2
        var = b * b * (n * n - 1) / 12
        assert abs(s.mean - mean) <= 1e-15 * max(abs(mean), 1.0)
        assert abs(s.m2 / n - var) <= 1e-13 * var
        assert s.min == min(v[0], v[-1]) and s.max == max(v[0], v[-1])


def pin_merge(o):
    rng = np.random.default_rng(2)
    a = (rng.standard_normal((40, 30, 20)) * 3 + 7).astype(np.float32)
    a[rng.random(a.shape) < 0.05] = np.nan
    whole = o.stats(a)
    A, B = o.stats(a[:13]), o.stats(a[13:])
    n = A.n_valid + B.n_valid
    d = B.mean - A.mean
    mean = A.mean + d * B.n_valid / n
    m2 = A.m2 + B.m2 + d * d * A.n_valid * B.n_valid / n   # Chan et al. pairwise
    assert whole.n_valid == n
    assert abs(whole.mean - mean) <= 1e-13 * abs(mean)
    assert abs(whole.m2 - m2) <= 1e-12 * m2


def pin_infinite_moments(o):
    """Moments with +-Inf among the valid voxels, over the extended reals:
    numpy's float64 mean and population std of the valid voxels (IEEE
    arithmetic on infinities, an independent routine) fix them, and the
    finite voxels around them must not disturb the reading.  The infinite
    voxels are still ordinary values for the extrema and counts."""
    import warnings
    cases = [
        ([1.0, np.inf, 2.0], np.inf),
        ([np.inf], np.inf),
        ([np.inf, np.inf, np.nan], np.inf),
        ([-np.inf, 1.0, np.nan, -5.0], -np.inf),
        ([np.inf, -np.inf], None),
        ([3.0, np.nan, -np.inf, 2.5, np.inf, 1e30], None),
    ]
    for vals, want_mean in cases:
        a = np.array(vals, dtype=np.float32)
        v = a[~np.isnan(a)].astype(np.float64)
        with np.errstate(invalid="ignore"), warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            np_mean, np_std = float(np.mean(v)), float(np.std(v))
            np_mabs = float(np.mean(np.abs(v)))
        s = o.stats(a)
        if want_mean is None:
            assert math.isnan(np_mean) and math.isnan(s.mean), (vals, s.mean)
        else:
            assert np_mean == want_mean and s.mean == want_mean, (vals, s.mean, np_mean)
        assert math.isnan(np_std) and math.isnan(s.std) and math.isnan(s.m2), (vals, s.std)
        assert s.mean_abs == np_mabs == np.inf, (vals, s.mean_abs)
        assert s.n_valid == v.size and s.n_nan == a.size - v.size
        assert s.min == v.min() and s.max == v.max()
    # a large finite cube with one +Inf: +Inf mean; without it, finite again
    rng = np.random.default_rng(12)
    b = rng.standard_normal(10_000).astype(np.float32)
    fin = o.stats(b)
    b[4321] = np.inf
    s = o.stats(b)
    assert s.mean == np.inf and math.isnan(s.std) and s.max == np.inf
    assert math.isfinite(fin.mean) and math.isfinite(fin.std)
    # streamed in pieces, with the infinity in the second piece only
    pieces = lambda: iter((b[:5000], b[5000:]))
    t = o.stats_pieces(pieces)
    assert t.mean == np.inf and math.isnan(t.std) and t.n_valid == b.size


def pin_slabs(o):
    """Slabs swept on several threads and added in slab order: counts and
    extrema equal numpy's over the whole cube exactly, and the moments equal
    exact rational arithmetic (``fractions``) to double rounding, including
    a first slab with no valid voxel, signed zeros at the far end, and a sum
    whose value survives only in the compensation of one slab (2^60 and
    many ones, cancelled by -2^60 in the next slab)."""
    rng = np.random.default_rng(21)
    a = (rng.standard_normal((23, 9, 11)) * 2.5 + 4.0).astype(np.float32)
    a[rng.random(a.shape) < 0.04] = np.nan
    a[:3] = np.nan                       # the first slab holds no valid voxel
    a[-1, 0, :4] = [-0.0, 0.0, -0.0, 0.0]
    cuts = [0, 3, 4, 11, 17, 23]
    slabs = [(lambda z0=z0, z1=z1: iter((a[z0:z1],))) for z0, z1 in zip(cuts, cuts[1:])]
    s = o.stats_slabs(slabs, 3)
    v = a[~np.isnan(a)].astype(np.float64)
    assert s.n_total == a.size and s.n_valid == v.size and s.n_nan == a.size - v.size
    assert s.min == np.nanmin(a) and s.max == np.nanmax(a)
    fr = [Fraction(float(x)) for x in v]
    mean = sum(fr) / len(fr)
    m2 = sum((x - mean) ** 2 for x in fr)
    assert abs(s.mean - float(mean)) <= 1e-15 * abs(float(mean))
    assert abs(s.m2 - float(m2)) <= 1e-13 * float(m2)
    one = o.stats(a)
    assert (one.n_valid, one.min, one.max) == (s.n_valid, s.min, s.max)
    # a sum carried by one slab's compensation term
    big = np.float32(2.0 ** 60)
    b = np.ones(4001, dtype=np.float32)
    b[0], b[2000] = big, -big
    t = o.stats_slabs([lambda: iter((b[:2000],)), lambda: iter((b[2000:],))], 2)
    want = Fraction(3999, 4001)          # 3999 ones over 4001 valid voxels
    assert abs(t.mean - float(want)) <= 1e-15, t.mean
    # +Inf in the middle slab only: the extended-real reading survives the adds
    c = rng.standard_normal(300).astype(np.float32)
    c[150] = np.inf
    u = o.stats_slabs([lambda: iter((c[:100],)), lambda: iter((c[100:200],)),
                       lambda: iter((c[200:],))], 2)
    assert u.mean == np.inf and math.isnan(u.std) and u.max == np.inf


# ------------------------------------------------------------ extrema / NaN
def pin_extrema_nan(o):
    rng = np.random.default_rng(3)
    for trial in range(6):
        a = (rng.standard_normal(5000) * 10 ** trial).astype(np.float32)
        a[rng.random(a.size) < 0.2] = np.nan
        if trial == 5:
            a[17], a[99] = np.inf, -np.inf
        s = o.stats(a)
        assert s.n_nan == int(np.isnan(a).sum())
        assert s.n_valid == int((~np.isnan(a)).sum())
        assert s.n_total == a.size
        assert s.min == np.nanmin(a) and s.max == np.nanmax(a)
    # signed zeros: -0 orders before +0
    for arr in ([0.0, -0.0], [-0.0, 0.0], [0.0, np.nan, -0.0, 0.0]):
        s = o.stats(np.array(arr, dtype=np.float32))
        assert s.min == 0.0 and signbit(s.min) and not signbit(s.max), arr
    s = o.stats(np.array([0.0, 0.0], dtype=np.float32))
    assert not signbit(s.min)
    s = o.stats(np.array([-0.0, -0.0], dtype=np.float32))
    assert signbit(s.max)
    # all blank, single voxel, NaN payloads (quiet, signalling, negative)
    s = o.stats(np.full(10, np.nan, dtype=np.float32))
    assert s.n_valid == 0 and s.n_nan == 10 and math.isnan(s.min) and math.isnan(s.mean)
    s = o.stats(np.array([2.5], dtype=np.float32))
    assert (s.min, s.max, s.mean, s.m2, s.std) == (2.5, 2.5, 2.5, 0.0, 0.0)
    weird = np.array([bits_f32(0x7F800001), bits_f32(0xFFC00000), bits_f32(0x7FFFFFFF),
                      f32(1.0), f32(-2.0)], dtype=np.float32)
    s = o.stats(weird)
    assert s.n_nan == 3 and s.n_valid == 2 and s.min == -2.0 and s.max == 1.0


def pin_strided(o):
    rng = np.random.default_rng(4)
    big = rng.standard_normal((12, 21, 37)).astype(np.float32)
    big[rng.random(big.shape) < 0.03] = np.nan
    for sl in [np.s_[2:9, 3:17, 5:30], np.s_[:, 1:2, :], np.s_[4:5, :, 1:36],
               np.s_[0:12, 0:21, 7:8]]:
        view = big[sl]
        dense = np.ascontiguousarray(view)
        sv, sd = o.stats(view), o.stats(dense)
        assert sv == sd or (math.isnan(sv.mean) and math.isnan(sd.mean))
        flat = dense.reshape(-1)
        assert sv.n_nan == int(np.isnan(flat).sum())
        assert sv.min == np.nanmin(flat) and sv.max == np.nanmax(flat)
        assert o.hist(view, -1.0, 1.5, 10).tolist() == o.hist(dense, -1.0, 1.5, 10).tolist()
    # piecewise streaming over z slabs equals the one-shot result
    whole = o.stats(big)
    pieces = lambda: (big[z0:z0 + 5] for z0 in range(0, 12, 5))
    assert o.stats_pieces(pieces) == whole
    h = o.hist(big, -2.0, 2.0, 33)
    assert o.hist_pieces(pieces, -2.0, 2.0, 33).tolist() == h.tolist()


# ------------------------------------------------------------------ histogram
def pin_hist_ramp(o):
    # 0..N-1 over [0, N] with N = nbins * 2^k: width 2^k exactly, every bin 2^k
    for nbins, k in ((256, 0), (256, 3), (1024, 2), (7, 4), (4096, 1)):
        n = nbins << k
        v = np.arange(n, dtype=np.float32)
        c = o.hist(v, 0.0, float(n), nbins)
        assert np.all(c[:nbins] == (1 << k)), (nbins, k)
        assert c[nbins:].tolist() == [0, 0, 0]
        # the top edge itself lands in the last bin (closed range)
        c2 = o.hist(np.append(v, np.float32(n)), 0.0, float(n), nbins)
        assert c2[nbins - 1] == (1 << k) + 1


def pin_hist_unit_scale(o):
    # lo = 0, hi = nbins: scale is exactly 1, so the bin is numpy.floor(x)
    rng = np.random.default_rng(5)
    for nbins in (1, 10, 256, 1000):
        x = (rng.random(20000) * nbins).astype(np.float32)
        x = np.append(x, np.float32(nbins))
        want = np.minimum(np.floor(x).astype(np.int64), nbins - 1)
        c = o.hist(x, 0.0, float(nbins), nbins)
        assert c[:nbins].tolist() == np.bincount(want, minlength=nbins).tolist()


def pin_hist_edges(o):
    lo, hi, nb = f32(-1.5), f32(2.5), 8     # scale = 8 / 4 = 2 exactly
    ninf, pinf = np.float32(-np.inf), np.float32(np.inf)
    cases = [  # value, expected slot (0..7 bins, 8 below, 9 above, 10 NaN)
        (lo, 0), (hi, 7), (np.nextafter(hi, pinf), 9), (np.nextafter(lo, ninf), 8),
        (np.nextafter(hi, ninf), 7), (f32(np.nan), 10), (pinf, 9), (ninf, 8),
        (f32(-1.0), 1), (f32(-0.0), 3), (f32(0.0), 3), (f32(0.5), 4), (f32(2.0), 7),
        # x - lo is itself rounded: 0.5 - 2^-25 minus -1.5 rounds up to 2.0
        # (bin 4), and 2 - 2^-23 minus -1.5 ties to even at 3.5 (bin 7); values
        # a few ulps lower stay in the bin below.
        (f32(0.49999997), 4), (f32(0.4999999), 3), (f32(1.9999999), 7), (f32(1.9999996), 6),
        (bits_f32(0xFFC00000), 10),
    ]
    for v, slot in cases:
        c = o.hist(np.array([v], dtype=np.float32), lo, hi, nb)
        assert c.sum() == 1 and c[slot] == 1, (v, slot, c.tolist())
    # degenerate range hi == lo: x == lo is bin 0, the rest below or above
    c = o.hist(np.array([3.0, 3.0, 2.0, 4.0, np.nan], dtype=np.float32), 3.0, 3.0, 5)
    assert c.tolist() == [2, 0, 0, 0, 0, 1, 1, 1]
    c = o.hist(np.array([-0.0, 0.0], dtype=np.float32), -0.0, 0.0, 4)
    assert c.tolist() == [2, 0, 0, 0, 0, 0, 0]


def pin_hist_subnormal(o):
    # lo = 0, hi = 2^-119, 256 bins: scale = 2^127 exactly.  Subnormal inputs
    # must keep their value (no flush to zero): 2^-127 -> bin 1, 2^-126 -> 2.
    lo, hi, nb = f32(0.0), np.float32(2.0 ** -119), 256
    assert o.hist_scale(lo, hi, nb) == 2.0 ** 127
    cases = [(2.0 ** -149, 0), (2.0 ** -127, 1), (3 * 2.0 ** -128, 1), (2.0 ** -126, 2),
             (2.0 ** -120, 128), (2.0 ** -119, 255)]
    for v, b in cases:
        c = o.hist(np.array([v], dtype=np.float32), lo, hi, nb)
        assert c[b] == 1, (v, b)


def _round_f32(q: Fraction) -> Fraction:
    """Round an exact rational to IEEE-754 binary32, nearest-even, with
    gradual underflow (an independent model of the hardware rounding)."""
    if q == 0:
        return Fraction(0)
    sgn = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)                      # subnormals share the bottom exponent
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * ulp
    if r >= Fraction(2) ** 128:
        return Fraction(sgn) * Fraction(10) ** 60   # overflow marker (not used)
    return sgn * r


def pin_hist_rounding_model(o):
    """The bin of every in-range x is min(nbins-1, floor(fl(fl(x - lo) * s)))
    with s = fl(nbins / fl(hi - lo)): checked against exact rationals rounded
    by an IEEE binary32 model, on ranges whose scale is not a power of two."""
    rng = np.random.default_rng(6)
    for lo, hi, nb in ((0.1, 1.7, 7), (-3.3, 12.9, 1000), (1e4 - 0.007, 1.1e4, 4096),
                       (-5.25, 47.5, 256)):
        lo, hi = f32(lo), f32(hi)
        w = _round_f32(Fraction(float(hi)) - Fraction(float(lo)))
        s = _round_f32(Fraction(nb) / w)
        assert Fraction(float(o.hist_scale(lo, hi, nb))) == s
        x = (lo + (hi - lo) * rng.random(3000)).astype(np.float32)
        # plus values next to every bin edge, where rounding decides
        edges = (lo.astype(np.float64) + np.arange(nb + 1) * (float(hi) - float(lo)) / nb)
        near = np.concatenate([np.nextafter(edges.astype(np.float32), np.float32(-np.inf)),
                               edges.astype(np.float32),
                               np.nextafter(edges.astype(np.float32), np.float32(np.inf))])
        x = np.concatenate([x, near[(near >= lo) & (near <= hi)]]).astype(np.float32)
        want = np.zeros(nb, dtype=np.int64)
        for v in x:
            u = _round_f32(_round_f32(Fraction(float(v)) - Fraction(float(lo))) * s)
            b = min(nb - 1, math.floor(u))
            want[b] += 1
        c = o.hist(x, lo, hi, nb)
        assert c[:nb].tolist() == want.tolist(), (float(lo), float(hi), nb)
        assert c[nb:].tolist() == [0, 0, 0]


def pin_hist_numpy(o):
    """numpy.histogram bins by float64 edges, so it may differ from the FP32
    rule only for values within a few float32 ulps of an edge."""
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(200_000) * 3).astype(np.float32)
    lo, hi, nb = f32(-7.0), f32(9.5), 1024
    c = o.hist(x, lo, hi, nb)
    ref, edges = np.histogram(x[(x >= lo) & (x <= hi)].astype(np.float64), bins=nb,
                              range=(float(lo), float(hi)))
    moved = int(np.abs(c[:nb].astype(np.int64) - ref).sum()) // 2
    xd = x.astype(np.float64)
    idx = np.clip(np.searchsorted(edges, xd), 1, nb)
    gap = np.minimum(np.abs(xd - edges[idx - 1]), np.abs(xd - edges[idx]))
    near = int((gap <= 4 * np.abs(np.spacing(x)).astype(np.float64) + 4 * np.spacing(np.float32(hi - lo))).sum())
    assert moved <= near, (moved, near)
    assert c[nb] == int((x < lo).sum()) and c[nb + 1] == int((x > hi).sum())


def pin_hist_invariants(o):
    import synth
    a = synth.make_numpy(synth.WORKLOADS["tiny"], synth.BASE_SEED)
    s = o.stats(a)
    c = o.hist(a, s.min, s.max, 256)
    assert int(c.sum()) == a.size
    assert c[256] == 0 and c[257] == 0 and c[258] == s.n_nan
    assert c[0] >= 1 and c[255] >= 1
    assert s.min <= s.mean <= s.max


def pin_hist_validation(o):
    bad = [(np.nan, 1.0, 10), (0.0, np.nan, 10), (2.0, 1.0, 10), (-np.inf, 1.0, 10),
           (0.0, np.inf, 10), (-3e38, 3e38, 10), (0.0, 1.0, 0), (0.0, 1.0, 65537),
           (0.0, 1e-45, 256)]
    for lo, hi, nb in bad:
        try:
            o.hist_scale(f32(lo), f32(hi), nb)
        except ValueError:
            continue
        raise AssertionError(f"accepted invalid range {(lo, hi, nb)}")
    assert o.hist_scale(f32(0.0), f32(1.0), 65536) == 65536.0
    assert o.hist_scale(f32(1.0), f32(1.0), 3) == 0.0


# --------------------------------------------------------------- selection
def pin_select(o):
    rng = np.random.default_rng(8)
    for n in (1, 2, 3, 10, 1001):
        a = (rng.standard_normal(n) * 50).astype(np.float32)
        if n > 3:
            a[rng.random(n) < 0.1] = np.nan
        valid = np.sort(a[~np.isnan(a)])          # numpy's sort as the reference
        for k in sorted({0, len(valid) // 2, len(valid) - 1}):
            assert o.select(a, k) == valid[k], (n, k)
        med = np.median(valid.astype(np.float64))  # numpy's median as the reference
        assert o.median(a) == med, (n, o.median(a), med)
    # integer ramp: the median is (N-1)/2 exactly, select(k) = k
    v = np.arange(1000, dtype=np.float32)[::-1].copy()
    assert o.median(v) == 499.5 and o.select(v, 0) == 0.0 and o.select(v, 999) == 999.0
    # signed zeros: -0 before +0; infinities are values; NaN is skipped
    a = np.array([0.0, -0.0, np.nan, np.inf, -np.inf, 0.0], dtype=np.float32)
    got = [o.select(a, k) for k in range(5)]
    assert got[0] == -np.inf and got[4] == np.inf
    assert signbit(got[1]) and not signbit(got[2]) and not signbit(got[3])
    for bad in (5, 100):
        try:
            o.select(a, bad)
        except ValueError:
            continue
        raise AssertionError("accepted an out-of-range rank")


def pin_quantiles(o):
    """Quantiles against closed forms (a shuffled integer ramp, where every
    interpolated level is exact), numpy's own quantile (linear method, to a
    few ulps, as it rounds its interpolation differently), the extremes and
    median from other oracle routines, and the readings for infinities."""
    rng = np.random.default_rng(31)
    # ramp 0..N-1 shuffled, with NaNs put between: quantile(q) = q * (N - 1)
    N = 1001
    ramp = rng.permutation(np.arange(N, dtype=np.float32))
    a = np.full(N + 40, np.nan, dtype=np.float32)
    keep = np.sort(rng.choice(N + 40, N, replace=False))
    a[keep] = ramp
    qs = [0.0, 0.001, 0.25, 0.5, 0.3337, 0.75, 0.999, 1.0]
    got = o.quantiles(a, qs)
    for q, g in zip(qs, got):
        assert g == q * (N - 1), (q, g)
    # a ramp of step 2 with offset: a + 2h
    b = (np.arange(200, dtype=np.float32) * 2 + 7)[::-1].copy()
    assert list(o.quantiles(b, [0.5, 0.25, 0.0625])) == [7 + 2 * 99.5, 7 + 2 * 49.75, 7 + 2 * 12.4375]
    # random values: numpy's linear quantile, the extremes and the median
    for n in (1, 2, 5, 1000):
        v = (rng.standard_normal(n) * 30).astype(np.float32)
        v[rng.random(n) < 0.1] = np.nan
        valid = v[~np.isnan(v)].astype(np.float64)
        if valid.size == 0:
            continue
        lv = [0.0, 0.1, 0.5, 0.9, 1.0]
        got = o.quantiles(v, lv)
        want = np.quantile(valid, lv)
        assert np.allclose(got, want, rtol=1e-14, atol=1e-12), (n, got, want)
        st = o.stats(v)
        assert got[0] == st.min and got[-1] == st.max
        assert got[2] == o.median(v)
        assert all(got[i] <= got[i + 1] for i in range(len(got) - 1))
    # infinities: an infinite end point is the result; -Inf to +Inf is NaN
    w = np.array([-np.inf, 1.0, 2.0, np.nan, np.inf], dtype=np.float32)
    r = o.quantiles(w, [0.0, 1 / 6, 0.5, 5 / 6, 1.0])
    assert r[0] == -np.inf and r[1] == -np.inf and r[2] == 1.5 and r[3] == np.inf
    assert r[4] == np.inf
    assert np.isnan(o.quantiles(np.array([-np.inf, np.inf], np.float32), [0.5])[0])
    # repeated values: no interpolation between equal neighbours
    assert list(o.quantiles(np.array([9, 3, 3, 9, 3], np.float32), [0.25, 0.375, 0.625])) == \
        [3.0, 3.0, 6.0]
    # signed zeros order -0 before +0
    z = o.quantiles(np.array([0.0, -0.0, -0.0], np.float32), [0.0, 1.0])
    assert signbit(z[0]) and not signbit(z[1])
    # errors: a level outside [0, 1] or NaN, and no valid voxel
    for bad_q, arr in (([1.5], a), ([-0.1], a), ([np.nan], a), ([0.5], np.full(4, np.nan, np.float32))):
        try:
            o.quantiles(arr, bad_q)
        except ValueError:
            continue
        raise AssertionError(f"accepted {bad_q}")


def pin_project(o):
    """Projections along z against numpy reductions over axis 0, exact sums
    (math.fsum) and the -0 < +0 order, plus consistency with the global
    statistics."""
    import math
    rng = np.random.default_rng(21)
    a = (rng.standard_normal((13, 7, 11)) * 3).astype(np.float32)
    a[rng.random(a.shape) < 0.2] = np.nan
    a[:, 2, 3] = np.nan                       # an all-blank pixel
    mip, mom0, nv = o.project(a)
    assert mip.shape == (7, 11) and mom0.shape == (7, 11) and nv.shape == (7, 11)
    want_nv = np.count_nonzero(~np.isnan(a), axis=0)
    assert np.array_equal(nv, want_nv)
    with np.errstate(invalid="ignore"), warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        want_mip = np.nanmax(a, axis=0)
    assert np.array_equal(np.isnan(mip), want_nv == 0)
    assert np.array_equal(mip[want_nv > 0], want_mip[want_nv > 0])
    for y in range(7):
        for x in range(11):
            col = a[:, y, x]
            col = col[~np.isnan(col)]
            if col.size == 0:
                assert math.isnan(mom0[y, x])
            else:
                assert mom0[y, x] == math.fsum(col.astype(np.float64)), (y, x)
    st = o.stats(a)
    assert int(nv.sum()) == st.n_valid
    assert np.nanmax(mip) == st.max
    assert abs(np.nansum(mom0) - st.mean * st.n_valid) <= 1e-12 * st.mean_abs * st.n_valid
    # the channel axis is z: a cube constant along y and x but not along z
    r = np.broadcast_to(np.arange(5, dtype=np.float32)[:, None, None], (5, 3, 4)).copy()
    mip, mom0, nv = o.project(r)
    assert (mip == 4.0).all() and (mom0 == 10.0).all() and (nv == 5).all()
    # signed zeros: +0 is the larger; a lone -0 stays -0
    z = np.array([[[-0.0, 0.0, -0.0]], [[0.0, -0.0, -0.0]]], dtype=np.float32)
    mip, _, _ = o.project(z)
    assert [signbit(v) for v in mip[0]] == [False, False, True]
    # infinities: the sum over the extended reals
    w = np.array([[[1.0, np.inf, -np.inf, np.inf]], [[2.0, 5.0, 3.0, -np.inf]],
                  [[np.nan, 1.0, -1.0, 7.0]]], dtype=np.float32)
    mip, mom0, nv = o.project(w)
    assert mom0[0, 0] == 3.0 and mom0[0, 1] == np.inf and mom0[0, 2] == -np.inf
    assert math.isnan(mom0[0, 3]) and mip[0, 3] == np.inf and mip[0, 2] == 3.0
    assert list(nv[0]) == [2, 3, 3, 3]
    # a strided view equals its contiguous copy
    big = (rng.standard_normal((9, 12, 15))).astype(np.float32)
    view = big[1:8, 2:11, 3:14]
    for u, v in zip(o.project(view), o.project(np.ascontiguousarray(view))):
        assert np.array_equal(u, v, equal_nan=True)


ALL_PINS = [pin_textbook, pin_exact_rational, pin_closed_forms, pin_merge, pin_infinite_moments,
            pin_slabs,
            pin_extrema_nan, pin_strided, pin_hist_ramp, pin_hist_unit_scale,
            pin_hist_edges, pin_hist_subnormal, pin_hist_rounding_model, pin_hist_numpy,
            pin_hist_invariants, pin_hist_validation, pin_select, pin_quantiles,
            pin_project]
