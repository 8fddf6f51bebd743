"""Randomized GPU parity (hypothesis, derandomized so every run checks the
same cases): random shapes, strided sub-boxes, offsets that break 16-byte
alignment, NaN rates, value scales, ranges and bin counts.  Statistics,
two-pass, fused and histogram-only against the oracle; selection,
quantiles at random levels and the projection maps too."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests.parity import assert_counts_match, assert_stats_match, same_f32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow,
                                           HealthCheck.function_scoped_fixture])


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    cs.cube_set_launch(0, 0, 0, 0)
    cs.cube_set_accum_mode(cs.CUBE_ACCUM_FP64MERGE)
    return cs


@st.composite
def boxes(draw):
    """(device view, host copy of the view)."""
    nz, ny, nx = draw(st.integers(1, 40)), draw(st.integers(1, 70)), draw(st.integers(1, 300))
    pz, py, px = draw(st.integers(0, 3)), draw(st.integers(0, 5)), draw(st.integers(0, 7))
    seed = draw(st.integers(0, 2**31 - 1))
    nan_frac = draw(st.sampled_from([0.0, 0.01, 0.3, 1.0]))
    scale = draw(st.sampled_from([1e-2, 1.0, 1e3]))
    offset = draw(st.sampled_from([0.0, 3.0, -1e4]))
    rng = np.random.default_rng(seed)
    full = (offset + scale * rng.standard_normal((nz + pz, ny + py, nx + px))).astype(np.float32)
    full[rng.random(full.shape) < nan_frac] = np.nan
    dev = torch.from_numpy(full).cuda()
    return dev[pz:, py:, px:], full[pz:, py:, px:]


@SETTINGS
@given(box=boxes(), nbins=st.integers(1, 2048), frac=st.floats(0.0, 0.5))
def test_random_boxes(cs, box, nbins, frac):
    t, host = box
    ref = oracle.stats(host)
    assert_stats_match(cs.stats(t), ref, "stats")
    st2, c2 = cs.stats_hist_minmax(t, nbins)
    assert_stats_match(st2, ref, "two-pass")
    if ref.n_valid == 0:
        assert c2[:nbins + 2].sum() == 0 and c2[nbins + 2] == ref.n_total
        return
    assert_counts_match(c2, oracle.hist(host, ref.min, ref.max, nbins), "two-pass counts")
    # a given range covering part of the data (below / above both used)
    w = ref.max - ref.min
    lo = float(np.float32(ref.min + frac * w))
    hi = float(np.float32(ref.max - frac * w))
    if hi < lo:
        lo, hi = hi, lo
    try:
        want = oracle.hist(host, lo, hi, nbins)
    except ValueError:           # a range too narrow for nbins bins in FP32
        with pytest.raises(cs.CubeError):
            cs.hist(t, lo, hi, nbins)
        return
    st3, c3 = cs.stats_hist(t, lo, hi, nbins)
    assert_stats_match(st3, ref, "fused")
    assert_counts_match(c3, want, "fused counts")
    assert_counts_match(cs.hist(t, lo, hi, nbins), want, "hist counts")


@settings(max_examples=15, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(box=boxes(), q=st.floats(0.0, 1.0),
       levels=st.lists(st.floats(0.0, 1.0), min_size=1, max_size=64))
def test_random_select_and_project(cs, box, q, levels):
    t, host = box
    ref = oracle.stats(host)
    if ref.n_valid:
        k = min(ref.n_valid - 1, int(q * ref.n_valid))
        assert same_f32(cs.select(t, k), oracle.select(host, k))
        assert cs.median(t)[0] == oracle.median(host)
        got, nv = cs.quantiles(t, levels)
        want = oracle.quantiles(host, levels)
        assert nv == ref.n_valid
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (levels, got, want)
    mip, mom0, nv = (g.cpu().numpy() for g in cs.project(t))
    rmip, rmom0, rnv = oracle.project(host)
    assert np.array_equal(nv.view(np.uint32), rnv)
    assert np.array_equal(mip.view(np.uint32), rmip.view(np.uint32))
    scale = np.nansum(np.abs(host.astype(np.float64)), axis=0)
    ok = (np.isnan(mom0) & np.isnan(rmom0)) | (np.abs(mom0 - rmom0) <= 1e-12 * scale)
    assert ok.all()
