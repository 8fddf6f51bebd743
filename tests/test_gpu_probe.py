"""The read probe (GPU): it must read every voxel of the box exactly where
the fused pass reads it.  Each case plants voxels that carry a mantissa bit
no other voxel has, at the places a scan gets wrong first (the first and last
voxel, a misaligned head, a ragged tail, tile and segment boundaries), so
that a skipped voxel loses its bit from the OR."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    cs.cube_set_launch(0, 0, 0, 0)
    return cs


def planted(shape, seed, nan_frac=0.01):
    """1.0 everywhere, some NaNs (bit 22 of the mantissa), and voxels with one
    of mantissa bits 0..21 each at chosen flat positions of the full array."""
    rng = np.random.default_rng(seed)
    a = np.ones(shape, dtype=np.float32)
    a[rng.random(shape) < nan_frac] = np.nan
    n = a.size
    picks = [0, 1, 2, 3, n - 1, n - 2, n - 3, n // 2]
    for tile in (256 * 4 * 4, 1024 * 4 * 4, 1024 * 4 * 4 * 2):
        picks += [tile - 1, tile, tile + 1]
    picks += list(rng.integers(0, n, 22))
    picks = [p for p in dict.fromkeys(picks) if 0 <= p < n][:22]
    bits = a.view(np.uint32).reshape(-1)
    for b, p in enumerate(picks):
        bits[p] = np.uint32(0x3f800000 | (1 << b))
    return a


def or_of(a):
    return int(np.bitwise_or.reduce(np.ascontiguousarray(a).view(np.uint32).reshape(-1)))


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 7), (3, 5, 301), (33, 17, 301),
                                   (64, 256, 1024), (5, 3, (1 << 22) + 5)])
@pytest.mark.parametrize("nbins", [1, 1024, 40000])
def test_probe_dense(cs, shape, nbins):
    a = planted(shape, seed=sum(shape) + nbins)
    t = torch.from_numpy(a).cuda()
    assert cs.read_probe(t, nbins) == or_of(a)


@pytest.mark.parametrize("off", [(0, 0, 1), (1, 2, 3), (2, 0, 2)])
def test_probe_strided_and_misaligned(cs, off):
    """Sub-boxes whose rows start off 16-byte boundaries and sit at pitches
    wider than their rows; the voxels outside the box carry a bit of their
    own (bit 21 is kept for them) that must not appear."""
    pz, py, px = off
    full = planted((40 + pz, 70 + py, 777 + px), seed=7 + px)
    bits = full.view(np.uint32)
    outside = np.ones(full.shape, bool)
    outside[pz:, py:, px:] = False
    bits[outside] = np.uint32(0x3f800000 | (1 << 21))
    view = full[pz:, py:, px:]
    inside = view.view(np.uint32)
    inside[inside == np.uint32(0x3f800000 | (1 << 21))] = np.uint32(0x3f800000)
    t = torch.from_numpy(full).cuda()[pz:, py:, px:]
    got = cs.read_probe(t, 1024)
    assert got == or_of(view)
    assert got & (1 << 21) == 0


def test_probe_empty_and_errors(cs):
    t = torch.zeros((0, 4, 4), dtype=torch.float32, device="cuda")
    assert cs.read_probe(t, 16) == 0                    # nothing launched, word stays 0
    x = torch.ones((2, 2, 2), dtype=torch.float32, device="cuda")
    ptr, d = cs.box_of(x)
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    with pytest.raises(cs.CubeError):
        cs.cube_read_probe(ptr, d, 0, out.data_ptr())
    with pytest.raises(cs.CubeError):
        cs.cube_read_probe(ptr, d, 16, 0)
    with pytest.raises(cs.CubeError):
        cs.cube_read_probe(ptr, d, 16, out.data_ptr() + 2)
