"""Cubic B-spline interpolation in FP64 (the abstract: both images are sampled
with spline interpolation).

Conventions (a reading; the paper only names "spline interpolation"):

* Sample ``s[i][j]`` (row ``i``, column ``j``) sits at spline coordinate
  ``(x, y) = (j, i)``.
* Boundary: half-sample symmetric extension ``... c b a | a b c ...``, i.e.
  index ``n`` folds with period ``2N``: ``n < 0 -> -n - 1``, ``n >= N -> 2N - 1 - n``.
* Kernel: the centred cubic B-spline ``beta``; the interpolant is
  ``s(x, y) = sum_{m,n} c[m][n] beta(x - n) beta(y - m)``.
* The coefficients ``c`` solve ``B c = s`` along each axis, where ``B`` is the
  tridiagonal matrix with 4/6 on the diagonal (5/6 in its first and last
  entries, from the mirrored neighbour) and 1/6 off it.
"""
from __future__ import annotations

import numpy as np


def beta(t):
    """Centred cubic B-spline: 2/3 - t^2 + |t|^3/2 on |t|<1, (2-|t|)^3/6 on 1<=|t|<2."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                    np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def dbeta(t):
    """First derivative of ``beta``."""
    t = np.asarray(t, dtype=np.float64)
    a = np.abs(t)
    return np.where(a < 1.0, -2.0 * t + 1.5 * t * a,
                    np.where(a < 2.0, -0.5 * np.sign(t) * (2.0 - a) ** 2, 0.0))


def ddbeta(t):
    """Second derivative of ``beta``."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(a < 1.0, -2.0 + 3.0 * a, np.where(a < 2.0, 2.0 - a, 0.0))


def fold(n, size: int):
    """Half-sample symmetric index folding with period ``2 * size``."""
    m = np.mod(np.asarray(n, dtype=np.int64), 2 * size)
    return np.where(m >= size, 2 * size - 1 - m, m)


def prefilter_1d(s: np.ndarray, axis: int) -> np.ndarray:
    """Solve ``B c = s`` along ``axis`` with the Thomas algorithm (FP64)."""
    s = np.moveaxis(np.asarray(s, dtype=np.float64), axis, 0).copy()
    N = s.shape[0]
    if N == 1:
        return np.moveaxis(s, 0, axis)
    diag = np.full(N, 4.0 / 6.0)
    diag[0] = diag[-1] = 5.0 / 6.0
    off = 1.0 / 6.0
    # forward elimination
    cp = np.empty(N)
    d = s
    cp[0] = off / diag[0]
    d[0] = d[0] / diag[0]
    for k in range(1, N):
        den = diag[k] - off * cp[k - 1]
        cp[k] = off / den
        d[k] = (d[k] - off * d[k - 1]) / den
    # back substitution
    for k in range(N - 2, -1, -1):
        d[k] = d[k] - cp[k] * d[k + 1]
    return np.moveaxis(d, 0, axis)


def prefilter(img: np.ndarray) -> np.ndarray:
    """2-D interpolation coefficients: rows first, then columns."""
    return prefilter_1d(prefilter_1d(img, axis=1), axis=0)


def evaluate(c: np.ndarray, x, y, order: int = 1):
    """Spline value, gradient and (``order == 2``) Hessian at spline coordinates.

    Returns ``(val, gx, gy)`` or ``(val, gx, gy, hxx, hxy, hyy)``; the sums run
    over the 4x4 taps ``n = floor(x)-1 .. floor(x)+2``, ``m = floor(y)-1 .. floor(y)+2``.
    """
    c = np.asarray(c, dtype=np.float64)
    H, W = c.shape
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    fx = np.floor(x).astype(np.int64)
    fy = np.floor(y).astype(np.int64)
    val = np.zeros(x.shape)
    gx = np.zeros(x.shape)
    gy = np.zeros(x.shape)
    if order >= 2:
        hxx = np.zeros(x.shape)
        hxy = np.zeros(x.shape)
        hyy = np.zeros(x.shape)
    for dm in range(-1, 3):
        m = fy + dm
        by, dby, ddby = beta(y - m), dbeta(y - m), ddbeta(y - m)
        rows = fold(m, H)
        for dn in range(-1, 3):
            n = fx + dn
            bx, dbx, ddbx = beta(x - n), dbeta(x - n), ddbeta(x - n)
            cv = c[rows, fold(n, W)]
            val += cv * bx * by
            gx += cv * dbx * by
            gy += cv * bx * dby
            if order >= 2:
                hxx += cv * ddbx * by
                hxy += cv * dbx * dby
                hyy += cv * bx * ddby
    if order >= 2:
        return val, gx, gy, hxx, hxy, hyy
    return val, gx, gy


def tap_weights(c_shape, x, y):
    """The 16 tap indices and weights of each point, for adjoint scatters.

    Returns ``(rows, cols, wv, wx, wy)`` each ``[npts][16]``: ``wv`` are the
    value weights ``beta(x-n) beta(y-m)``, ``wx`` and ``wy`` the gradient weights.
    """
    H, W = c_shape
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    fx = np.floor(x).astype(np.int64)
    fy = np.floor(y).astype(np.int64)
    rows, cols, wv, wx, wy = [], [], [], [], []
    for dm in range(-1, 3):
        m = fy + dm
        for dn in range(-1, 3):
            n = fx + dn
            rows.append(fold(m, H))
            cols.append(fold(n, W))
            wv.append(beta(x - n) * beta(y - m))
            wx.append(dbeta(x - n) * beta(y - m))
            wy.append(beta(x - n) * dbeta(y - m))
    return tuple(np.stack(a, axis=-1) for a in (rows, cols, wv, wx, wy))
