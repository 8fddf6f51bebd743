"""Projections along the channel axis (GPU) against the oracle.

mip and nvalid must be bit-exact; mom0 is an FP64 sum on both sides and must
agree within 1e-12 of the column's sum of |x| (the GPU adds in channel order,
the oracle compensates; both are far below that bound).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MOM0_TOL = 1e-12


@pytest.fixture(scope="module")
def cs():
    import paper_1111_6661_amd as cs
    assert torch.cuda.is_available()
    cs.load()
    return cs


def compare(got, host, what):
    mip, mom0, nv = (g.cpu().numpy() for g in got)
    rmip, rmom0, rnv = oracle.project(host)
    assert np.array_equal(nv.view(np.uint32), rnv), what
    assert np.array_equal(mip.view(np.uint32), rmip.view(np.uint32)), what
    with np.errstate(invalid="ignore"):  # Inf - Inf where both maps hold the same Inf
        scale = np.nansum(np.abs(host.astype(np.float64)), axis=0).reshape(rmom0.shape)
        close = np.abs(mom0 - rmom0) <= MOM0_TOL * scale
    both_nan = np.isnan(mom0) & np.isnan(rmom0)
    inf_equal = np.isinf(rmom0) & (mom0 == rmom0)
    ok = both_nan | inf_equal | close
    assert ok.all(), (what, np.argwhere(~ok)[:5])


def cube_of(shape, seed, nan_frac=0.02):
    import synth
    nz, ny, nx = shape
    r = synth.WORKLOADS["tiny"].scaled(nx, ny, nz)
    return synth.cube_tensor(r, seed, device="cuda")


# Shapes (z, y, x) that reach every launch form: the whole-image quad path
# with 4, 8 and 16 quads per lane, with and without a general-kernel tail and
# channel slices; the row-wise kernel with quads and single pixels.
@pytest.mark.parametrize("shape", [(128, 64, 64), (37, 41, 203), (5, 3, 4), (1, 1, 1),
                                   (2000, 8, 16), (700, 5, 33), (64, 256, 256),
                                   (50, 33, 260), (512, 16, 64), (8, 1024, 2048),
                                   (4, 2049, 2048)])
def test_project_shapes(cs, shape):
    t = cube_of(shape, 7 + shape[0])
    compare(cs.project(t), t.cpu().numpy(), f"shape {shape}")


def test_project_strided_views(cs):
    big = cube_of((90, 70, 120), 3)
    for sl in [(slice(3, 80), slice(2, 60), slice(5, 117)),     # unaligned x start
               (slice(0, 90), slice(0, 70), slice(4, 116)),     # aligned, strided rows
               (slice(10, 11), slice(0, 70), slice(0, 120)),    # one channel
               (slice(0, 90), slice(7, 8), slice(0, 120))]:     # one row
        v = big[sl]
        compare(cs.project(v), big.cpu().numpy()[sl], f"view {sl}")


def test_project_special_values(cs):
    a = np.zeros((6, 2, 8), np.float32)
    a[:, 0, 0] = np.nan                                        # blank pixel
    a[:, 0, 1] = [-0.0, 0.0, -0.0, np.nan, -0.0, -0.0]         # +0 wins
    a[:, 0, 2] = -0.0                                          # stays -0
    a[:, 0, 3] = [1.0, np.inf, 2.0, 3.0, 4.0, 5.0]             # +inf
    a[:, 0, 4] = [1.0, np.inf, -np.inf, 3.0, 4.0, 5.0]         # NaN sum
    a[:, 0, 5] = [-np.inf, -1.0, np.nan, np.nan, np.nan, np.nan]
    a[:, 1, :] = np.float32(1e-45)                             # subnormals
    a[2, 1, 3] = np.float32(-3e38)
    a[3, 1, 3] = np.float32(3e38)
    t = torch.from_numpy(a).cuda()
    compare(cs.project(t), a, "special values")


def test_project_empty_and_errors(cs):
    t = torch.zeros((0, 4, 4), device="cuda")
    mip, mom0, nv = cs.project(t)
    assert torch.isnan(mip).all() and torch.isnan(mom0).all() and (nv == 0).all()
    t = cube_of((8, 4, 4), 1)
    ptr, d = cs.box_of(t)
    with pytest.raises(cs.CubeError):
        cs.cube_project(ptr, d)                                 # no output
    host = np.zeros(16, np.float32)
    with pytest.raises(cs.CubeError):
        cs.cube_project(ptr, d, mip=host.ctypes.data)           # host output
    # too small: the last 15 elements of a fresh 1 GiB allocation (empty the
    # cache first so that the allocation is exactly that size)
    torch.cuda.empty_cache()
    big = torch.zeros(1 << 28, dtype=torch.int32, device="cuda")
    with pytest.raises(cs.CubeError):
        cs.cube_project(ptr, d, nvalid=big[-15:].data_ptr())
    cs.cube_project(ptr, d, nvalid=big[-16:].data_ptr())
    del big
    m = torch.zeros(40, dtype=torch.float64, device="cuda")
    with pytest.raises(cs.CubeError):                           # misaligned mom0
        cs.cube_project(ptr, d, mom0=m.data_ptr() + 4)


def test_project_full_brick_sampled(cs):
    """The 16 GiB brick in the benchmark's launch: pixels sampled against the
    oracle one column at a time, and the maps' totals against the stats."""
    import synth
    r = synth.WORKLOADS["brick16g"]
    t = synth.cube_tensor(r, synth.BASE_SEED + 1, device="cuda")
    mip, mom0, nv = cs.project(t)
    torch.cuda.synchronize()
    st = cs.stats(t)
    assert int(nv.to(torch.int64).sum()) == st.n_valid
    assert float(torch.nan_to_num(mip, nan=-np.inf).max()) == st.max
    rng = np.random.default_rng(5)
    ys = rng.integers(0, r.ny, 256)
    xs = rng.integers(0, r.nx, 256)
    ys[:2] = [0, r.ny - 1]
    xs[:2] = [0, r.nx - 1]
    iy = torch.from_numpy(ys).cuda()
    ix = torch.from_numpy(xs).cuda()
    cols = t[:, iy, ix].cpu().numpy()                            # [z, 256]
    host = np.ascontiguousarray(cols.reshape(r.nz, 1, 256))
    rmip, rmom0, rnv = oracle.project(host)
    g_mip = mip[iy, ix].cpu().numpy()
    g_mom0 = mom0[iy, ix].cpu().numpy()
    g_nv = nv[iy, ix].cpu().numpy().view(np.uint32)
    assert np.array_equal(g_nv, rnv[0])
    assert np.array_equal(g_mip.view(np.uint32), rmip[0].view(np.uint32))
    scale = np.nansum(np.abs(cols.astype(np.float64)), axis=0)
    both_nan = np.isnan(g_mom0) & np.isnan(rmom0[0])
    assert (both_nan | (np.abs(g_mom0 - rmom0[0]) <= MOM0_TOL * scale)).all()
    del t
    torch.cuda.empty_cache()
