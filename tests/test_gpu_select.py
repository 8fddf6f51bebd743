"""Exact selection and median (GPU) against the oracle."""
import math

import numpy as np
import pytest

import oracle
from tests.parity import same_f32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    return cs


def test_select_and_median_tiny(cs):
    import synth
    t = synth.cube_tensor(synth.WORKLOADS["tiny"], synth.BASE_SEED, device="cuda")
    host = t.cpu().numpy()
    ref = oracle.stats(host)
    n = ref.n_valid
    for k in (0, 1, n // 3, n // 2, n - 2, n - 1):
        assert same_f32(cs.select(t, k), oracle.select(host, k)), k
    m, nv = cs.median(t)
    assert nv == n and m == oracle.median(host)
    with pytest.raises(cs.CubeError):
        cs.select(t, n)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 1), (1001, 3, 1), (257, 129, 33)])
def test_median_shapes(cs, shape):
    import synth
    r = synth.WORKLOADS["tiny"].scaled(*shape)
    t = synth.cube_tensor(r, 55, device="cuda")
    host = t.cpu().numpy()
    if oracle.stats(host).n_valid == 0:
        with pytest.raises(cs.CubeError):
            cs.median(t)
        return
    m, _ = cs.median(t)
    assert m == oracle.median(host)


def test_select_special_values(cs):
    a = np.array([0.0, -0.0, np.nan, np.inf, -np.inf, 0.0, 3.5, -1e-45, 1e-45, np.nan],
                 dtype=np.float32)
    t = torch.from_numpy(a).cuda()
    n = int((~np.isnan(a)).sum())
    for k in range(n):
        assert same_f32(cs.select(t, k), oracle.select(a, k)), k
    assert cs.median(t)[0] == oracle.median(a)
    with pytest.raises(cs.CubeError):
        cs.median(torch.full((10,), float("nan"), device="cuda"))


def test_median_strided_and_ties(cs):
    import synth
    big = synth.cube_tensor(synth.WORKLOADS["tiny"].scaled(200, 50, 20), 8, device="cuda")
    view = big[2:17, 3:44, 5:190]
    host = big.cpu().numpy()[2:17, 3:44, 5:190]
    assert cs.median(view)[0] == oracle.median(host)
    # many ties: a cube of a few distinct values
    a = np.repeat(np.array([1.0, 2.0, 2.0, 3.0], np.float32), 12345)
    t = torch.from_numpy(a).cuda()
    assert cs.median(t)[0] == 2.0
    assert cs.select(t, 0) == 1.0 and cs.select(t, a.size - 1) == 3.0


def test_median_even_count_upper_middle(cs):
    """The upper middle of an even count found three ways: the same key
    again, the next key of the last histogram, and the extra pass for the
    smallest key above the lower middle."""
    one_up = np.nextafter(np.float32(1.0), np.float32(2.0))
    cases = [
        np.repeat(np.array([1.0, 1.0, 1.0, 3.0], np.float32), 1000),     # same key
        np.repeat(np.array([1.0, one_up], np.float32), 3000),             # same histogram
        np.repeat(np.array([1.0, 2.0], np.float32), 5000),                # extra pass
        np.array([-0.0, 0.0], np.float32),                                # -0 then +0
        np.array([np.nan, 5.0, np.nan, -7.5, 1e30, -1e-40], np.float32),  # blanks, subnormal
    ]
    for a in cases:
        t = torch.from_numpy(a).cuda()
        m, nv = cs.median(t)
        assert nv == int((~np.isnan(a)).sum())
        assert m == oracle.median(a), (a[:8], m, oracle.median(a))


def test_select_candidate_paths(cs):
    """The third pass reads the candidates the second copied out (a small
    first-pass bucket), the whole cube when the bucket is too large to copy,
    and the whole cube again when one block's region overflowed."""
    rng = np.random.default_rng(17)
    # a bucket of 2^25 equal voxels: larger than every candidate region together
    many = np.full(1 << 25, 1.5, np.float32)
    many[::7] = rng.standard_normal(many[::7].size).astype(np.float32)
    # 10M equal voxels at the front: about 10M in the bucket (fits in total)
    # but about 39K of them in each of the first blocks (more than a region)
    skew = rng.standard_normal(20_000_000).astype(np.float32)
    skew[:10_000_000] = 0.25
    # small buckets everywhere: the candidate path
    spread = (rng.standard_normal(5_000_003) * 100).astype(np.float32)
    spread[rng.random(spread.size) < 0.01] = np.nan
    for a in (many, skew, spread):
        t = torch.from_numpy(a).cuda()
        n = int((~np.isnan(a)).sum())
        for k in (0, n // 3, (n - 1) // 2, n - 1):
            assert same_f32(cs.select(t, k), oracle.select(a, k)), (a.size, k)
        m, nv = cs.median(t)
        assert nv == n and m == oracle.median(a), a.size
