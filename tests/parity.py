"""Comparison rules between the GPU library and the oracle.

Integer results (counts, n_valid, n_nan) and extrema are compared exactly
(extrema by bit pattern, so -0 and +0 differ).  Moments that are not finite
(a box holding +-Inf: an infinite or NaN mean, a NaN std, over the extended
reals) are compared exactly too: the same infinity, or NaN against NaN.

Finite std: |s - s_ref| <= 1e-6 * s_ref (exactly 0 when s_ref is 0).

Finite mean, with a = mean_abs_ref (the mean of |x| over the valid voxels)
and n = n_valid:

  * the rule for every box: |m - m_ref| <= 1e-6 * max(|m_ref|, 1e-3 * a).
    Above the cut |m_ref| >= 1e-3 * a this is 1e-6 relative; below it the
    error is judged against 1e-3 * a (stricter than falling back to 1e-6 * a
    there).  Boxes of at least 2^20 voxels are held to this rule alone.
  * smaller boxes may in addition carry the rounding of the FP32 deviations
    d = x - K (K the wavefront's pivot) and of their FP32 chunk sums, which no
    compensation after the fact removes: under the model of independent
    rounding errors of mean zero (Higham & Mary, probabilistic rounding error
    analysis) each voxel adds an error of standard deviation below
    u * rms(d) * sqrt(CHUNK / 2) (u = 2^-24; the k-th add of a chunk rounds a
    partial sum of about sqrt(k) * rms(d)), so the mean of n voxels carries
    at most u * rms(d) * sqrt(CHUNK / (2 n)).  With rms(d) <= 2 a (x and K
    drawn from the same noise: rms(d) = sqrt(2) std, about 1.8 a) and RHO
    standard deviations of margin the allowance is
    RHO * u * sqrt(2 * CHUNK / n) * a, about 1.2e-7 * a at 250 voxels and
    1.9e-9 * a just under 2^20.

The plain relative error of the mean is always reported (``rel_err``).
"""
from __future__ import annotations

import math

import numpy as np

REL_TOL = 1e-6
C8_CUT = 1e-3          # |mean| / mean_abs below which the mean is judged against the data scale
LARGE_BOX = 1 << 20    # boxes held to the 1e-6 / 1e-3 rule alone
U32 = 2.0 ** -24       # unit roundoff of binary32
CHUNK = 32             # voxels a lane sums in plain FP32 before a compensated fold
RHO = 4.0              # standard deviations of margin of the rounding allowance


def f32_bits(x: float) -> int:
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def same_f32(a: float, b: float) -> bool:
    if math.isnan(a) and math.isnan(b):
        return True
    return f32_bits(a) == f32_bits(b)


def same_value(a: float, b: float) -> bool:
    """Equal, or both NaN (for moments that are not finite)."""
    return (math.isnan(a) and math.isnan(b)) or a == b


def mean_tol(ref) -> float:
    """Absolute tolerance of a finite mean (see the module docstring)."""
    a = ref.mean_abs
    tol = REL_TOL * max(abs(ref.mean), C8_CUT * a)
    if ref.n_valid < LARGE_BOX:
        tol = max(tol, RHO * U32 * math.sqrt(2.0 * CHUNK / ref.n_valid) * a)
    return tol


def mean_ok(m: float, ref) -> bool:
    if not math.isfinite(ref.mean):
        return same_value(m, ref.mean)
    return abs(m - ref.mean) <= mean_tol(ref)


def std_ok(s: float, ref) -> bool:
    if not math.isfinite(ref.std):
        return same_value(s, ref.std)
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
        # infinities among the valid voxels: the extended-real reading, exactly
        assert same_value(got.mean, ref.mean), (what, "mean", got.mean, ref.mean)
        assert same_value(got.std, ref.std), (what, "std", got.std, ref.std)
        assert same_value(got.m2, ref.m2), (what, "m2", got.m2, ref.m2)
        return
    if not moments_in_fp32_range(ref):
        return
    tol = mean_tol(ref)
    assert abs(got.mean - ref.mean) <= tol_mul * tol, \
        (what, "mean", got.mean, ref.mean, "error/tolerance", abs(got.mean - ref.mean) / tol)
    if ref.std == 0.0:
        assert got.std == 0.0, (what, "std", got.std)
    else:
        assert abs(got.std - ref.std) <= tol_mul * REL_TOL * ref.std, \
            (what, "std", got.std, ref.std, abs(got.std - ref.std) / ref.std)


def rel_err(got, ref):
    """(plain relative error of the mean, relative error of the std)."""
    em = abs(got.mean - ref.mean) / abs(ref.mean) if ref.mean else abs(got.mean)
    es = abs(got.std - ref.std) / ref.std if ref.std else abs(got.std)
    return em, es


def assert_counts_match(got: np.ndarray, ref: np.ndarray, what: str = ""):
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    if not np.array_equal(got, ref):
        diff = np.nonzero(got != ref)[0]
        raise AssertionError(f"{what}: {len(diff)} slots differ, first {diff[:8].tolist()}: "
                             f"got {got[diff[:8]].tolist()} want {ref[diff[:8]].tolist()}")
