"""Comparison rules between the GPU library and the oracle.

Integer results (counts, n_valid, n_nan) and extrema are compared exactly
(extrema by bit pattern, so -0 and +0 differ).  Mean and std are compared
with a relative tolerance of 1e-6: std relative to the oracle's std (exactly
0 when the oracle's is 0); mean relative to max(|mean|, MEAN_FLOOR *
mean_abs).  The floor reflects the conditioning of a sum: any FP32
per-element evaluation carries an absolute mean error of order
u * mean(|x - K|) (u = 2^-24), independent of how close the mean is to zero,
so for a mean much smaller than the data's magnitude the error is measured
against that magnitude (a normwise relative error, Higham's summation bound).
"""
from __future__ import annotations

import math

import numpy as np

REL_TOL = 1e-6
MEAN_FLOOR = 0.1


def f32_bits(x: float) -> int:
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def same_f32(a: float, b: float) -> bool:
    if math.isnan(a) and math.isnan(b):
        return True
    return f32_bits(a) == f32_bits(b)


def mean_scale(ref) -> float:
    return max(abs(ref.mean), MEAN_FLOOR * ref.mean_abs)


def mean_ok(m: float, ref) -> bool:
    return abs(m - ref.mean) <= REL_TOL * mean_scale(ref)


def std_ok(s: float, ref) -> bool:
    if ref.std == 0.0:
        return s == 0.0
    return abs(s - ref.std) <= REL_TOL * ref.std


# Partial moments are FP32 (deviations d = x - K and their squares), so they
# are meaningful only while d^2 stays a normal FP32 number: deviations between
# about 2^-60 and 2^60.  Outside that range only the exact results (counts,
# extrema) are compared.
FP32_MOMENT_RANGE = (2.0 ** -60, 2.0 ** 60)


def moments_in_fp32_range(ref) -> bool:
    spread = max(abs(ref.max - ref.mean), abs(ref.mean - ref.min))
    return ref.std == 0.0 or (FP32_MOMENT_RANGE[0] <= ref.std and
                              spread <= FP32_MOMENT_RANGE[1])


def assert_stats_match(got, ref, what: str = "", tol_mul: float = 1.0):
    assert got.n_total == ref.n_total, (what, got.n_total, ref.n_total)
    assert got.n_valid == ref.n_valid, (what, got.n_valid, ref.n_valid)
    assert got.n_nan == ref.n_nan, (what, got.n_nan, ref.n_nan)
    assert same_f32(got.min, ref.min), (what, "min", got.min, ref.min)
    assert same_f32(got.max, ref.max), (what, "max", got.max, ref.max)
    if ref.n_valid == 0:
        assert math.isnan(got.mean) and math.isnan(got.std), what
        return
    if not (math.isfinite(ref.mean) and math.isfinite(ref.std)):
        assert not (math.isfinite(got.mean) and math.isfinite(got.std)), (what, got, ref)
        return
    if not moments_in_fp32_range(ref):
        return
    scale = mean_scale(ref)
    assert abs(got.mean - ref.mean) <= tol_mul * REL_TOL * scale, \
        (what, "mean", got.mean, ref.mean, abs(got.mean - ref.mean) / max(scale, 1e-300))
    if ref.std == 0.0:
        assert got.std == 0.0, (what, "std", got.std)
    else:
        assert abs(got.std - ref.std) <= tol_mul * REL_TOL * ref.std, \
            (what, "std", got.std, ref.std, abs(got.std - ref.std) / ref.std)


def rel_err(got, ref):
    """(mean error, std error) in the units of the tolerance rule above."""
    scale = mean_scale(ref)
    em = abs(got.mean - ref.mean) / scale if scale else 0.0
    es = abs(got.std - ref.std) / ref.std if ref.std else abs(got.std)
    return em, es


def assert_counts_match(got: np.ndarray, ref: np.ndarray, what: str = ""):
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    if not np.array_equal(got, ref):
        diff = np.nonzero(got != ref)[0]
        raise AssertionError(f"{what}: {len(diff)} slots differ, first {diff[:8].tolist()}: "
                             f"got {got[diff[:8]].tolist()} want {ref[diff[:8]].tolist()}")
