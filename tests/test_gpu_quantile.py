"""Quantiles (GPU) against the oracle: many levels at once, levels whose
ranks fall in more than eight leading key buckets (several refinement
reads), special values, strided and misaligned boxes, and the errors."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    return cs


def same(got, want):
    """Bit-equal FP64 arrays (NaN equal to NaN)."""
    got, want = np.asarray(got), np.asarray(want)
    return got.shape == want.shape and np.array_equal(got.view(np.uint64), want.view(np.uint64))


LEVELS64 = np.concatenate([[0.0, 1.0, 0.5, 0.25, 0.75, 1e-9, 1 - 1e-9],
                           np.random.default_rng(3).random(57)])


def test_tiny_workload_64_levels(cs):
    import synth
    t = synth.cube_tensor(synth.WORKLOADS["tiny"], synth.BASE_SEED, device="cuda")
    host = t.cpu().numpy()
    got, n = cs.quantiles(t, LEVELS64)
    assert n == oracle.stats(host).n_valid
    assert same(got, oracle.quantiles(host, LEVELS64))
    st = cs.stats(t)
    assert got[0] == st.min and got[1] == st.max


def test_many_leading_buckets(cs):
    """Values spread over 2^-60 .. 2^60 of both signs: the 64 levels' ranks
    fall in dozens of distinct top-12-bit key buckets, so the call takes the
    12 + 8 + 6 + 6-bit passes (four reads of the box)."""
    rng = np.random.default_rng(17)
    n = 300_000
    a = (np.exp2(rng.uniform(-60, 60, n)) * rng.choice([-1, 1], n)).astype(np.float32)
    a[rng.random(n) < 0.02] = np.nan
    t = torch.from_numpy(a.reshape(30, 100, 100)).cuda()
    levels = np.linspace(0, 1, 64)
    got, nv = cs.quantiles(t, levels)
    assert nv == int((~np.isnan(a)).sum())
    assert same(got, oracle.quantiles(a, levels))
    assert cs.cube_last_quantile_reads() == 4


@pytest.mark.parametrize("groups", [1, 8, 9, 64])
def test_bucket_count_boundary(cs, groups):
    """Clusters [2^e, 1.1 * 2^e) of 1000 voxels each (e = 0..59 positive,
    then negative ones) lie in top key buckets of their own, and one level
    falls inside each sorted cluster: up to 8 buckets take the 12 + 12 +
    8-bit passes, more the 12 + 8 + 6 + 6-bit ones."""
    rng = np.random.default_rng(groups)
    per = 1000
    parts = []
    for g in range(groups):
        sign = 1.0 if g < 60 else -1.0
        parts.append(sign * 2.0 ** (g % 60) * (1 + 0.1 * rng.random(per)))
    a = np.concatenate(parts).astype(np.float32)
    rng.shuffle(a)
    n = a.size
    levels = [(g * per + per // 2 + 0.37) / (n - 1) for g in range(groups)]
    t = torch.from_numpy(a.reshape(groups, 1, per)).cuda()
    got, nv = cs.quantiles(t, levels)
    assert nv == n
    assert same(got, oracle.quantiles(a, levels))
    assert cs.cube_last_quantile_reads() == (3 if groups <= 8 else 4)


def test_many_ranks_in_few_buckets(cs):
    """64 levels (up to 128 ranks) inside 4 top key buckets: more than 96
    ranks take the 12 + 8 + 6 + 6-bit passes although few buckets are hit;
    ties make some ranks share a key."""
    rng = np.random.default_rng(41)
    parts = [2.0 ** e * (1 + 0.1 * rng.random(50_000)) for e in (0, 3, 7, 11)]
    a = np.concatenate(parts).astype(np.float32)
    a[::97] = a[5]                                 # a run of equal keys
    rng.shuffle(a)
    levels = np.sort(rng.random(64))
    t = torch.from_numpy(a.reshape(4, 500, 100)).cuda()
    got, nv = cs.quantiles(t, levels)
    assert nv == a.size
    assert same(got, oracle.quantiles(a, levels))
    assert cs.cube_last_quantile_reads() == 4


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 2), (3, 1, 1), (7, 5, 301), (64, 64, 128),
                                   (1, 1, 3_000_001)])
def test_shapes(cs, shape):
    rng = np.random.default_rng(sum(shape))
    a = (rng.standard_normal(shape) * 10).astype(np.float32)
    a[rng.random(shape) < 0.1] = np.nan
    t = torch.from_numpy(a).cuda()
    lv = [0.0, 0.3, 0.5, 0.999, 1.0]
    if np.isnan(a).all():
        with pytest.raises(cs.CubeError):
            cs.quantiles(t, lv)
        return
    assert same(cs.quantiles(t, lv)[0], oracle.quantiles(a, lv))


def test_special_values_and_ties(cs):
    a = np.array([0.0, -0.0, np.nan, np.inf, -np.inf, 0.0, 3.5, -1e-45, 1e-45, np.nan,
                  3.5, 3.5, -2.0, 7.0], dtype=np.float32)
    t = torch.from_numpy(a).cuda()
    lv = np.linspace(0, 1, 23)
    assert same(cs.quantiles(t, lv)[0], oracle.quantiles(a, lv))
    # -Inf to +Inf gives NaN; equal neighbours give the value itself
    b = torch.tensor([-np.inf, np.inf, np.nan], dtype=torch.float32, device="cuda")
    assert np.isnan(cs.quantiles(b, [0.5])[0][0])
    r = torch.round(torch.randn(1000, device="cuda") * 2)
    lv = np.linspace(0, 1, 64)
    assert same(cs.quantiles(r, lv)[0], oracle.quantiles(r.cpu().numpy(), lv))


def test_strided_and_misaligned(cs):
    rng = np.random.default_rng(5)
    full = rng.standard_normal((40, 70, 333)).astype(np.float32)
    full[rng.random(full.shape) < 0.05] = np.nan
    dev = torch.from_numpy(full).cuda()
    for sl in (np.s_[3:, 1:, 1:], np.s_[:, 5:60, 7:300], np.s_[10:11, 2:3, 3:]):
        lv = LEVELS64[:20]
        got, _ = cs.quantiles(dev[sl], lv)
        assert same(got, oracle.quantiles(full[sl], lv)), sl


def test_agrees_with_select_and_median(cs):
    import synth
    r = synth.WORKLOADS["tiny"].scaled(129, 65, 33)
    t = synth.cube_tensor(r, 9, device="cuda")
    n = cs.stats(t).n_valid
    q = np.array([0.0, 0.5, 1.0, 17 / (n - 1)])
    got, _ = cs.quantiles(t, q)
    assert got[0] == cs.select(t, 0) and got[2] == cs.select(t, n - 1)
    assert got[3] == cs.select(t, 17) or abs(got[3] - cs.select(t, 17)) <= 1e-6 * abs(got[3])
    assert abs(got[1] - cs.median(t)[0]) <= 1e-15 * abs(got[1])


def test_errors(cs):
    t = torch.randn(100, device="cuda")
    for bad in ([], [1.5], [-0.01], [float("nan")], [0.5] * 65):
        with pytest.raises(cs.CubeError):
            cs.quantiles(t, bad)
    with pytest.raises(cs.CubeError):
        cs.quantiles(torch.full((1, 5, 5), float("nan"), device="cuda"), [0.5])
    with pytest.raises(cs.CubeError):
        cs.quantiles(torch.zeros((0, 3, 3), device="cuda"), [0.5])
    # 64 levels are accepted
    assert cs.quantiles(t, [0.5] * 64)[0].shape == (64,)
