"""The synthetic-cube recipe (CPU): deterministic, with the stated blanking."""
import numpy as np

import synth


def test_numpy_generator_deterministic_and_blanked():
    r = synth.WORKLOADS["tiny"]
    a = synth.make_numpy(r, synth.BASE_SEED)
    b = synth.make_numpy(r, synth.BASE_SEED)
    assert a.shape == (128, 64, 64) and a.dtype == np.float32
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert abs(np.isnan(a).mean() - 0.01) < 0.002
    c = synth.make_numpy(r, synth.BASE_SEED + 1)
    assert not np.array_equal(np.nan_to_num(a), np.nan_to_num(c))
    # sources lift the maximum well above the noise
    assert np.nanmax(a) > 5.0


def test_channel_and_pixel_blanking():
    r = synth.WORKLOADS["brick16g"].scaled(64, 48, 200)
    r = synth.Recipe(**{**r.__dict__, "p_pixel_nan": 0.05, "chan_nan_frac": 0.05})
    a = synth.make_numpy(r, 7)
    d = synth.draw(r, 7)
    assert sum(b - a0 for a0, b in d.chan_ranges) == 10
    for lo, hi in d.chan_ranges:
        assert np.isnan(a[lo:hi]).all()
    pix = np.isnan(a).all(axis=0)
    assert 0.01 < pix.mean() < 0.12


def test_tile_lists_cover_every_footprint():
    r = synth.Recipe(70, 40, 90, n_sources=50)
    d = synth.draw(r, 3)
    tx, ty, tz = d.tiles
    assert len(d.tile_start) == tx * ty * tz + 1
    for s in range(r.n_sources):
        cx, cy, cz, _ = d.src[s]
        x, y, z = int(min(r.nx - 1, cx)), int(min(r.ny - 1, cy)), int(min(r.nz - 1, cz))
        t = x // synth.TILE + tx * (y // synth.TILE + ty * (z // synth.TILE))
        assert s in d.src_idx[d.tile_start[t]:d.tile_start[t + 1]]


def test_batch_and_serve_shapes():
    items = synth.batch_item_recipes()
    assert len(items) == 64
    assert all(32 <= it.nx <= 512 and 32 <= it.ny <= 512 and 32 <= it.nz <= 256 for it in items)
    total = sum(a * b * c for a, b, c in synth.SERVE_SHAPES) * 4 / 2**30
    assert 195 < total < 205
