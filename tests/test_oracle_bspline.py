"""Pins for the oracle's cubic B-spline (the abstract: spline interpolation of
both images at the mesh nodes).  Checked against closed forms, finite
differences and scipy's independent cubic-spline evaluator."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import bspline


def test_kernel_values_and_partition_of_unity():
    assert bspline.beta(0.0) == pytest.approx(2.0 / 3.0, abs=0)
    assert bspline.beta(1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert bspline.beta(-1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert bspline.beta(2.0) == 0.0 and bspline.beta(-2.5) == 0.0
    x = np.random.default_rng(1).uniform(-5, 5, 1000)
    n = np.floor(x)[:, None] + np.arange(-1, 3)[None, :]
    assert np.abs(bspline.beta(x[:, None] - n).sum(1) - 1).max() < 1e-14
    assert np.abs(bspline.dbeta(x[:, None] - n).sum(1)).max() < 1e-14
    # linear reproduction: sum_n n beta(x - n) = x
    assert np.abs((n * bspline.beta(x[:, None] - n)).sum(1) - x).max() < 1e-13


def test_derivatives_match_finite_differences():
    t = np.random.default_rng(2).uniform(-2.2, 2.2, 500)
    h = 1e-6
    fd1 = (bspline.beta(t + h) - bspline.beta(t - h)) / (2 * h)
    fd2 = (bspline.dbeta(t + h) - bspline.dbeta(t - h)) / (2 * h)
    assert np.abs(fd1 - bspline.dbeta(t)).max() < 1e-8
    assert np.abs(fd2 - bspline.ddbeta(t)).max() < 1e-6


def test_fold_is_half_sample_symmetric():
    N = 5
    got = bspline.fold(np.arange(-12, 17), N)
    ext = np.concatenate([np.arange(N), np.arange(N)[::-1]])   # period 2N
    want = ext[np.mod(np.arange(-12, 17), 2 * N)]
    assert np.array_equal(got, want)
    assert bspline.fold(-1, N) == 0 and bspline.fold(N, N) == N - 1


@pytest.mark.parametrize("shape", [(1, 7), (2, 3), (17, 31), (40, 9)])
def test_interpolates_samples(shape):
    img = np.random.default_rng(3).random(shape)
    c = bspline.prefilter(img)
    ii, jj = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    assert np.abs(bspline.evaluate(c, jj, ii)[0] - img).max() < 1e-12


def test_reproduces_quadratics_away_from_borders():
    H, W = 70, 80
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    f = lambda x, y: 0.3 + 0.01 * x - 0.02 * y + 1e-3 * x * x - 2e-3 * x * y + 5e-4 * y * y
    c = bspline.prefilter(f(jj.astype(float), ii.astype(float)))
    rng = np.random.default_rng(4)
    x = rng.uniform(24, W - 1 - 24, 300)
    y = rng.uniform(24, H - 1 - 24, 300)
    v, gx, gy, hxx, hxy, hyy = bspline.evaluate(c, x, y, order=2)
    assert np.abs(v - f(x, y)).max() < 1e-12
    assert np.abs(gx - (0.01 + 2e-3 * x - 2e-3 * y)).max() < 1e-12
    assert np.abs(gy - (-0.02 - 2e-3 * x + 1e-3 * y)).max() < 1e-12
    assert np.abs(hxx - 2e-3).max() < 1e-12
    assert np.abs(hxy + 2e-3).max() < 1e-12
    assert np.abs(hyy - 1e-3).max() < 1e-12


def test_matches_scipy_reflect_spline_everywhere():
    """scipy's order-3 spline with mode 'reflect' is the same half-sample
    symmetric interpolant; it is computed by independent code."""
    rng = np.random.default_rng(5)
    img = rng.random((21, 34))
    c = bspline.prefilter(img)
    x = rng.uniform(-4, 38, 2000)
    y = rng.uniform(-4, 25, 2000)
    ref = ndi.map_coordinates(img, [y, x], order=3, mode="reflect")
    assert np.abs(bspline.evaluate(c, x, y)[0] - ref).max() < 1e-12


def test_gradient_and_hessian_match_finite_differences():
    rng = np.random.default_rng(6)
    c = bspline.prefilter(rng.random((16, 16)))
    x = rng.uniform(1, 14, 100)
    y = rng.uniform(1, 14, 100)
    h = 1e-5
    v, gx, gy, hxx, hxy, hyy = bspline.evaluate(c, x, y, order=2)
    vxp, gxp, gyp = bspline.evaluate(c, x + h, y)
    vxm, gxm, gym = bspline.evaluate(c, x - h, y)
    vyp, gxq, gyq = bspline.evaluate(c, x, y + h)
    vym, gxr, gyr = bspline.evaluate(c, x, y - h)
    assert np.abs((vxp - vxm) / (2 * h) - gx).max() < 1e-8
    assert np.abs((vyp - vym) / (2 * h) - gy).max() < 1e-8
    assert np.abs((gxp - gxm) / (2 * h) - hxx).max() < 1e-6
    assert np.abs((gyq - gyr) / (2 * h) - hyy).max() < 1e-6
    assert np.abs((gyp - gym) / (2 * h) - hxy).max() < 1e-6


def test_prefilter_is_self_adjoint():
    rng = np.random.default_rng(7)
    a, b = rng.random((13, 19)), rng.random((13, 19))
    assert abs(np.sum(bspline.prefilter(a) * b) - np.sum(a * bspline.prefilter(b))) < 1e-12
