"""Properties of the oracle over random shapes, NaN rates and value scales
(CPU, hypothesis).  These hold for any input and are fixed by the
definitions, not by the oracle's code: conservation of counts, the
[min, max] range invariants, the ordering of extrema and mean, agreement of
a streamed cube with the same cube at once, and the consistency of
selection and projection with the statistics."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

SETTINGS = settings(max_examples=60, deadline=None,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def cubes(draw):
    nz = draw(st.integers(1, 6))
    ny = draw(st.integers(1, 9))
    nx = draw(st.integers(1, 23))
    seed = draw(st.integers(0, 2**31 - 1))
    nan_frac = draw(st.sampled_from([0.0, 0.05, 0.5, 1.0]))
    scale = draw(st.sampled_from([1e-3, 1.0, 1e3]))
    offset = draw(st.sampled_from([0.0, -7.0, 1e4]))
    rng = np.random.default_rng(seed)
    a = (offset + scale * rng.standard_normal((nz, ny, nx))).astype(np.float32)
    if draw(st.booleans()):
        a = np.round(a)  # ties and repeated values
    a[rng.random(a.shape) < nan_frac] = np.nan
    return a


@SETTINGS
@given(a=cubes(), nbins=st.integers(1, 300))
def test_counts_conserved_and_range_invariants(a, nbins):
    s = oracle.stats(a)
    assert s.n_valid + s.n_nan == a.size
    if s.n_valid == 0:
        assert math.isnan(s.min) and math.isnan(s.max) and math.isnan(s.mean)
        return
    assert s.min <= s.mean <= s.max or math.isclose(s.mean, s.min) or math.isclose(s.mean, s.max)
    assert s.std >= 0.0
    if s.max == s.min:
        assert s.std == 0.0
    c = oracle.hist(a, s.min, s.max, nbins)
    assert int(c.sum()) == a.size
    assert int(c[nbins]) == 0 and int(c[nbins + 1]) == 0          # nothing outside [min, max]
    assert int(c[nbins + 2]) == s.n_nan
    assert c[0] >= 1 and c[nbins - 1] >= 1 or (s.max == s.min and c[0] == s.n_valid)
    # a range that excludes everything
    below = oracle.hist(a, s.max + abs(s.max) + 1.0, s.max + abs(s.max) + 2.0, nbins)
    assert int(below[nbins]) == s.n_valid and int(below[:nbins].sum()) == 0


@SETTINGS
@given(a=cubes(), cut=st.integers(1, 5))
def test_streaming_equals_one_shot(a, cut):
    """A cube streamed in pieces along z gives the statistics and counts of
    the whole (within rounding for the moments, exactly for the rest)."""
    k = min(cut, a.shape[0])
    pieces = lambda: iter([a[:k], a[k:]] if k < a.shape[0] else [a])  # noqa: E731
    whole = oracle.stats(a)
    part = oracle.stats_pieces(pieces)
    assert (part.n_valid, part.n_nan) == (whole.n_valid, whole.n_nan)
    if whole.n_valid:
        assert part.min == whole.min and part.max == whole.max
        assert math.isclose(part.mean, whole.mean, rel_tol=1e-12, abs_tol=1e-12 * whole.mean_abs)
        assert math.isclose(part.std, whole.std, rel_tol=1e-10, abs_tol=1e-12 * whole.mean_abs)
        lo, hi = whole.min, whole.max
        assert np.array_equal(oracle.hist_pieces(pieces, lo, hi, 17), oracle.hist(a, lo, hi, 17))


@SETTINGS
@given(a=cubes())
def test_selection_and_projection_agree_with_stats(a):
    s = oracle.stats(a)
    mip, mom0, nv = oracle.project(a)
    assert int(nv.sum()) == s.n_valid
    if s.n_valid == 0:
        assert np.isnan(mip).all() and np.isnan(mom0).all()
        with pytest.raises(ValueError):
            oracle.median(a)
        return
    assert oracle.select(a, 0) == s.min and oracle.select(a, s.n_valid - 1) == s.max
    assert np.nanmax(mip) == s.max
    total = float(np.nansum(mom0))
    assert math.isclose(total, s.mean * s.n_valid, rel_tol=1e-9,
                        abs_tol=1e-9 * s.mean_abs * s.n_valid)
    m = oracle.median(a)
    assert s.min <= m <= s.max
    # quantiles: the extremes at 0 and 1, the median at 1/2 (to rounding:
    # the median averages, the quantile interpolates), monotone in the level
    levels = [0.0, 0.1, 0.5, 0.9, 1.0]
    qv = oracle.quantiles(a, levels)
    assert qv[0] == s.min and qv[-1] == s.max
    assert math.isclose(qv[2], m, rel_tol=1e-15, abs_tol=1e-300)
    assert all(qv[i] <= qv[i + 1] for i in range(len(qv) - 1))
    # the median splits the valid voxels: at most half lie strictly below it
    # and at most half strictly above it
    v = a[~np.isnan(a)]
    assert np.count_nonzero(v < m) <= s.n_valid // 2
    assert np.count_nonzero(v > m) <= s.n_valid // 2
