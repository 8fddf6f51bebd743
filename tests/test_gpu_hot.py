"""The hot-bin histogram form (GPU) against the oracle: every block keeps the
bin of its first in-range voxel out of LDS and counts it as its in-range
total minus the other bins, so the counts must stay bit-exact whatever the
hot bin is -- the modal bin, a rare bin, the rounding slot at x == hi, or
none (a block starting on blank or out-of-range voxels)."""
import numpy as np
import pytest

import oracle
from tests.parity import assert_counts_match, assert_stats_match

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    cs.cube_set_launch(0, 0, 0, 0)
    prev = cs.cube_set_hist_mode(cs.CUBE_HIST_HOT)
    yield cs
    cs.cube_set_hist_mode(prev)
    cs.cube_set_launch(0, 0, 0, 0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(cs, t, host, nbins, what, lo=None, hi=None):
    ref = oracle.stats(host)
    if ref.n_valid and not (np.isfinite(ref.min) and np.isfinite(ref.max)):
        # an infinite extremum: no [min, max] histogram (CUBE_EINVAL by contract)
        with pytest.raises(cs.CubeError):
            cs.stats_hist_minmax(t, nbins)
    else:
        st2, c2 = cs.stats_hist_minmax(t, nbins)
        assert_stats_match(st2, ref, what + " minmax-stats")
        if ref.n_valid:
            assert_counts_match(c2, oracle.hist(host, ref.min, ref.max, nbins), what + " minmax")
    if lo is None:
        if not ref.n_valid:
            return
        lo, hi = ref.min, ref.max
    want = oracle.hist(host, lo, hi, nbins)
    st3, c3 = cs.stats_hist(t, lo, hi, nbins)
    assert_stats_match(st3, ref, what + " fused-stats")
    assert_counts_match(c3, want, what + " fused")
    assert_counts_match(cs.hist(t, lo, hi, nbins), want, what + " hist")


def test_tiny_workload(cs):
    import synth
    t = synth.cube_tensor(synth.WORKLOADS["tiny"], synth.BASE_SEED, device="cuda")
    host = t.cpu().numpy()
    ref = oracle.stats(host)
    for nb in (1, 7, 256, 4096):
        check(cs, t, host, nb, f"tiny-{nb}")
    check(cs, t, host, 256, "tiny-2sigma", float(np.float32(ref.mean - 2 * ref.std)),
          float(np.float32(ref.mean + 2 * ref.std)))


@pytest.mark.parametrize("launch", [(256, 1, 1, 4), (256, 37, 2, 2), (1024, 300, 8, 4),
                                    (512, 2000, 32, 4)])
def test_launch_shapes(cs, launch):
    """From one block to thousands (each with its own hot bin), with 1 to 32
    LDS copies."""
    import synth
    r = synth.WORKLOADS["tiny"].scaled(301, 67, 53)
    t = synth.cube_tensor(r, 777, device="cuda")
    host = t.cpu().numpy()
    cs.cube_set_launch(*launch)
    try:
        check(cs, t, host, 512, f"launch{launch}")
    finally:
        cs.cube_set_launch(0, 0, 0, 0)


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (1_000_003, 1, 1), (63, 65, 64)])
def test_ragged_shapes(cs, shape):
    import synth
    nx, ny, nz = shape
    r = synth.WORKLOADS["tiny"].scaled(nx, ny, nz)
    t = synth.cube_tensor(r, 4321 + nx, device="cuda")
    check(cs, t, t.cpu().numpy(), 128, f"shape{shape}")


def test_strided_view(cs):
    import synth
    r = synth.WORKLOADS["tiny"].scaled(256, 64, 64)
    big = synth.cube_tensor(r, 4242, device="cuda")
    box = np.s_[3:40, 5:60, 7:200]
    check(cs, big[box], big.cpu().numpy()[box], 64, "strided")


def test_skewed_and_degenerate(cs):
    rng = np.random.default_rng(5)
    n = 2_000_003
    cases = {
        # nearly everything in one bin (the precision-stress shape)
        "skewed": (1e4 + rng.standard_normal(n) * 1e-3).astype(np.float32),
        # a constant cube: one bin, and hi == lo
        "constant": np.full(n, 3.25, np.float32),
        # blocks that start on blank voxels: no hot bin there
        "blank-runs": np.where((np.arange(n) // 40_000) % 2 == 0, np.nan,
                               rng.standard_normal(n)).astype(np.float32),
        # the hot bin is the rounding slot floor(u) == nbins (x == hi)
        "at-hi": np.concatenate([np.full(n // 2, 2.0, np.float32),
                                 rng.uniform(0, 2, n - n // 2).astype(np.float32)]),
        "with-inf": np.concatenate([[np.inf, -np.inf, np.nan], rng.standard_normal(n)]
                                   ).astype(np.float32),
    }
    for name, a in cases.items():
        t = _dev(a)
        rng_ = (-1.0, 2.0) if name == "with-inf" else (None, None)
        check(cs, t, a, 256, name, *rng_)
        check(cs, t, a, 4096, name + "-4096", *rng_)
    a = cases["at-hi"]
    check(cs, _dev(a), a, 100, "at-hi-range", 0.0, 2.0)
    # ranges that leave most voxels below or above, and NaN payloads
    a = cases["skewed"]
    check(cs, _dev(a), a, 64, "above", 9999.0, 9999.5)
    check(cs, _dev(a), a, 64, "below", 10000.5, 10001.0)
    p = np.array([0x7F800001, 0xFFC00000, 0x3F800000, 0x40000000] * 5000, np.uint32).view(np.float32)
    check(cs, _dev(p), p, 16, "nan-payloads")


def test_hot_equals_plain_bit_for_bit(cs):
    """Counts and statistics bytes of the two forms are identical."""
    import synth
    t = synth.cube_tensor(synth.WORKLOADS["tiny"].scaled(512, 256, 33), 99, device="cuda")
    st = cs.stats(t)
    got = {}
    for mode in (cs.CUBE_HIST_PLAIN, cs.CUBE_HIST_HOT):
        cs.cube_set_hist_mode(mode)
        got[mode] = cs.stats_hist(t, st.min, st.max, 1024)
    cs.cube_set_hist_mode(cs.CUBE_HIST_HOT)
    (sa, ca), (sb, cb) = got[cs.CUBE_HIST_PLAIN], got[cs.CUBE_HIST_HOT]
    assert np.array_equal(ca, cb)
    assert (sa.n_valid, sa.min, sa.max, sa.mean, sa.std) == (sb.n_valid, sb.min, sb.max, sb.mean,
                                                             sb.std)
