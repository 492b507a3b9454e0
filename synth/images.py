"""Seeded synthetic image pairs standing in for the paper's brain-CT slices.

The paper's examples (Section 3.2, Example 1; Section 3.3, Example 2 and
Table 1) use brain-CT images that are not available, so every workload here is
synthetic: a template made of Gaussian blobs plus a flat disk, and a reference
that is the same analytic template evaluated at positions displaced by a
smooth sine-series field.  Nothing in this module performs any step of the
registration method; it only produces the method's inputs (Algorithm 1,
"Inputs").

Recipe (all draws from one ``numpy.random.default_rng(seed)`` in this order):

1. ``n_blobs`` blob centres ``cx ~ U[0, W)``, ``cy ~ U[0, H)``, widths
   ``sigma ~ U[4, 16]`` px and amplitudes ``amp ~ U[0.2, 1]``.
2. Sine-series amplitudes ``a_x`` then ``a_y``, each 4x4 from ``U[-A, A]``.

Pixel ``(row i, col j)`` has its centre at ``(j + 1/2, i + 1/2)``.  A blob is
``amp * exp(-|x - c|^2 / (2 sigma^2))`` inside radius ``6 sigma`` and exactly 0
outside it (the cut-off keeps generation cheap at 2048^2; the jump there is
below 2e-8 * amp).  The disk adds 0.5 where the distance to the image centre
is at most 30 px.  The displacement is
``d_c(x, y) = s_c * sum_{p,q=1..4} a_c[p,q] sin(p pi x / W) sin(q pi y / H)``
with ``s_c = min(1, A / max_pixels |unscaled d_c|)``, and the reference is
``Re(x) = F(x + d(x))`` evaluated analytically.  The 12-bit variant clips both
images to [0, 1] and rounds to multiples of 1/4095.
"""
from __future__ import annotations

import numpy as np

BLOB_CUTOFF_SIGMAS = 6.0
DISK_RADIUS = 30.0
DISK_VALUE = 0.5


def blob_count(height: int, width: int, per_128sq: float = 8.0) -> int:
    """Blob count scaled with the image area: 8 blobs per 128x128 pixels."""
    return int(round(per_128sq * height * width / (128.0 * 128.0)))


def draw_params(rng: np.random.Generator, height: int, width: int,
                amplitude: float, n_blobs: int | None = None) -> dict:
    """Draw blob and sine-series parameters in the fixed order of the recipe."""
    nb = blob_count(height, width) if n_blobs is None else int(n_blobs)
    cx = rng.uniform(0.0, width, nb)
    cy = rng.uniform(0.0, height, nb)
    sigma = rng.uniform(4.0, 16.0, nb)
    amp = rng.uniform(0.2, 1.0, nb)
    ax = rng.uniform(-amplitude, amplitude, (4, 4))
    ay = rng.uniform(-amplitude, amplitude, (4, 4))
    return dict(cx=cx, cy=cy, sigma=sigma, amp=amp, ax=ax, ay=ay,
                amplitude=float(amplitude), height=int(height), width=int(width))


def _sine_field(a: np.ndarray, X: np.ndarray, Y: np.ndarray, width: int,
                height: int) -> np.ndarray:
    d = np.zeros_like(X)
    for p in range(1, 5):
        sx = np.sin(p * np.pi * X / width)
        for q in range(1, 5):
            d += a[p - 1, q - 1] * sx * np.sin(q * np.pi * Y / height)
    return d


def displacement(params: dict) -> tuple[np.ndarray, np.ndarray]:
    """The scaled sine-series displacement at every pixel centre (float64)."""
    H, W = params["height"], params["width"]
    X, Y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    out = []
    for a in (params["ax"], params["ay"]):
        d = _sine_field(a, X, Y, W, H)
        peak = float(np.max(np.abs(d))) if d.size else 0.0
        scale = 1.0 if peak == 0.0 else min(1.0, params["amplitude"] / peak)
        out.append(d * scale)
    return out[0], out[1]


def _render(params: dict, PX: np.ndarray, PY: np.ndarray,
            box_pad: float) -> np.ndarray:
    """Evaluate the analytic template at positions (PX, PY) laid on the pixel grid.

    ``PX[i, j]`` lies within ``box_pad`` of the pixel centre ``(j+1/2, i+1/2)``,
    which bounds the pixel window each blob can reach.
    """
    H, W = params["height"], params["width"]
    img = np.zeros((H, W), dtype=np.float64)
    for cx, cy, s, a in zip(params["cx"], params["cy"], params["sigma"], params["amp"]):
        rad = BLOB_CUTOFF_SIGMAS * s
        j0 = max(0, int(np.floor(cx - rad - box_pad)) - 1)
        j1 = min(W, int(np.ceil(cx + rad + box_pad)) + 1)
        i0 = max(0, int(np.floor(cy - rad - box_pad)) - 1)
        i1 = min(H, int(np.ceil(cy + rad + box_pad)) + 1)
        if j0 >= j1 or i0 >= i1:
            continue
        dx = PX[i0:i1, j0:j1] - cx
        dy = PY[i0:i1, j0:j1] - cy
        r2 = dx * dx + dy * dy
        val = a * np.exp(-r2 / (2.0 * s * s))
        val[r2 > rad * rad] = 0.0
        img[i0:i1, j0:j1] += val
    mx, my = W / 2.0, H / 2.0
    img += DISK_VALUE * (((PX - mx) ** 2 + (PY - my) ** 2) <= DISK_RADIUS ** 2)
    return img


def quantise_12bit(img: np.ndarray) -> np.ndarray:
    return np.round(np.clip(img, 0.0, 1.0) * 4095.0) / 4095.0


def make_images(params: dict, quantise: bool = False):
    """Return ``(Te, Re)`` as float32 ``[H][W]`` arrays."""
    H, W = params["height"], params["width"]
    X, Y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    te = _render(params, X, Y, 0.0)
    dx, dy = displacement(params)
    re = _render(params, X + dx, Y + dy, params["amplitude"] + 1.0)
    if quantise:
        te, re = quantise_12bit(te), quantise_12bit(re)
    return te.astype(np.float32), re.astype(np.float32)


def textured_translation_pair(height: int, width: int, shift, seed: int,
                              n_blobs: int = 32, border: int = 24):
    """A textured template with a zero border and its exact translate.

    Blobs have ``sigma ~ U[6, 10]`` and centres kept ``border + 3 sigma`` away
    from the edges; no disk.  ``Re(x) = F(x + shift)``.  Used to check that the
    method recovers a pure translation.
    """
    rng = np.random.default_rng(seed)
    sig = rng.uniform(6.0, 10.0, n_blobs)
    lo = border + 3.0 * sig
    cx = lo + rng.uniform(0.0, 1.0, n_blobs) * (width - 2 * lo)
    cy = lo + rng.uniform(0.0, 1.0, n_blobs) * (height - 2 * lo)
    amp = rng.uniform(0.2, 1.0, n_blobs)
    X, Y = np.meshgrid(np.arange(width) + 0.5, np.arange(height) + 0.5)

    def F(PX, PY):
        img = np.zeros((height, width))
        for a, x0, y0, s in zip(amp, cx, cy, sig):
            img += a * np.exp(-((PX - x0) ** 2 + (PY - y0) ** 2) / (2 * s * s))
        return img

    te = F(X, Y)
    re = F(X + shift[0], Y + shift[1])
    return te.astype(np.float32), re.astype(np.float32)
