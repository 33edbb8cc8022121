"""Seeded image column: procedurally drawn glyphs, shifted and noised.

Ten glyph classes are drawn here from plain geometric strokes (ring, bar, Z,
X, plus, square, triangle, L, three bars, T) on a 28x28 canvas.  Each image
picks a class label uniformly from 0..9, shifts the class template by an
integer offset in [-2, 2] on each axis (zero fill), adds N(0, 20^2) noise,
rounds and clips to [0, 255].  Consecutive groups of four images form one grid
row of the image table.

The network's initial weights are also drawn here (He-uniform bounds), because
every random number the method consumes is an input to it.
"""
from __future__ import annotations

import numpy as np

GLYPH_SIZE = 28
_OFF = 4.0  # glyph strokes live in a 20x20 box placed at (4, 4)

_SEGMENTS = {
    1: [((10, 2), (10, 18))],
    2: [((3, 3), (17, 3)), ((17, 3), (3, 17)), ((3, 17), (17, 17))],
    3: [((3, 3), (17, 17)), ((17, 3), (3, 17))],
    4: [((10, 2), (10, 18)), ((2, 10), (18, 10))],
    5: [((3, 3), (17, 3)), ((17, 3), (17, 17)), ((17, 17), (3, 17)), ((3, 17), (3, 3))],
    6: [((10, 2), (18, 17)), ((18, 17), (2, 17)), ((2, 17), (10, 2))],
    7: [((4, 2), (4, 17)), ((4, 17), (16, 17))],
    8: [((3, 4), (17, 4)), ((3, 10), (17, 10)), ((3, 16), (17, 16))],
    9: [((2, 3), (18, 3)), ((10, 3), (10, 18))],
}


def _seg_dist(px, py, a, b):
    ax, ay = a[0] + _OFF, a[1] + _OFF
    bx, by = b[0] + _OFF, b[1] + _OFF
    dx, dy = bx - ax, by - ay
    t = np.clip(((px - ax) * dx + (py - ay) * dy) / (dx * dx + dy * dy), 0.0, 1.0)
    return np.hypot(px - (ax + t * dx), py - (ay + t * dy))


def glyph_templates() -> np.ndarray:
    """float64 [10, 28, 28] templates with intensities in [0, 255]."""
    yy, xx = np.mgrid[0:GLYPH_SIZE, 0:GLYPH_SIZE].astype(np.float64)
    out = np.zeros((10, GLYPH_SIZE, GLYPH_SIZE))
    for c in range(10):
        if c == 0:
            d = np.abs(np.hypot(xx - (10 + _OFF), yy - (10 + _OFF)) - 7.0)
        else:
            d = np.min(np.stack([_seg_dist(xx, yy, a, b) for a, b in _SEGMENTS[c]]), axis=0)
        out[c] = 255.0 * np.clip(1.6 - d, 0.0, 1.0)
    return out


def _shifted(templates):
    """[10, 5, 5, 28, 28]: template shifted by (dy, dx) in [-2, 2] with zero fill."""
    n = GLYPH_SIZE
    out = np.zeros((10, 5, 5, n, n))
    for iy, dy in enumerate(range(-2, 3)):
        for ix, dx in enumerate(range(-2, 3)):
            ys, yd = (slice(0, n - dy), slice(dy, n)) if dy >= 0 else (slice(-dy, n), slice(0, n + dy))
            xs, xd = (slice(0, n - dx), slice(dx, n)) if dx >= 0 else (slice(-dx, n), slice(0, n + dx))
            out[:, iy, ix, yd, xd] = templates[:, ys, xs]
    return out


def image_column(n_images=120_000, cells_per_row=4, n_buckets=100, noise_sigma=20.0, seed=None):
    """Return a dict with ``images`` u8[n,28,28], hidden ``label`` i8[n],
    ``grid_row`` i32[n] (image i belongs to grid row i // cells_per_row) and
    ``bucket`` i32[n] (grid row mod n_buckets)."""
    from . import SEED_IMAGES, stream_seed, uniform_int, normal_f32
    if seed is None:
        seed = SEED_IMAGES
    s = lambda c: stream_seed(seed, c)
    label = uniform_int(s(0), n_images, 0, 9, np.int64)
    dy = uniform_int(s(1), n_images, 0, 4, np.int64)
    dx = uniform_int(s(2), n_images, 0, 4, np.int64)
    shifted = _shifted(glyph_templates())
    base = shifted[label, dy, dx]  # [n, 28, 28]
    noise = normal_f32(s(3), s(4), n_images * GLYPH_SIZE * GLYPH_SIZE).reshape(base.shape)
    img = np.clip(np.rint(base + noise_sigma * noise.astype(np.float64)), 0, 255).astype(np.uint8)
    row = (np.arange(n_images, dtype=np.int64) // cells_per_row).astype(np.int32)
    return {
        "images": img,
        "label": label.astype(np.int8),
        "grid_row": row,
        "bucket": (row % n_buckets).astype(np.int32),
    }


# Network shapes (NHWC activations; weights [Cout][ky][kx][Cin]; fc1 input in (y, x, c) order).
CNN_SHAPES = {
    "conv1_w": (32, 3, 3, 1), "conv1_b": (32,),
    "conv2_w": (64, 3, 3, 32), "conv2_b": (64,),
    "fc1_w": (128, 12 * 12 * 64), "fc1_b": (128,),
    "fc2_w": (10, 128), "fc2_b": (10,),
}


def cnn_init(seed=0x7D0D0C00):
    """Float32 initial parameters: weights U(-b, b) with b = sqrt(6 / fan_in)
    (sqrt(3 / fan_in) for the output layer), biases zero."""
    from . import stream_seed, uniform01_f32
    params = {}
    for i, (name, shape) in enumerate(CNN_SHAPES.items()):
        if name.endswith("_b"):
            params[name] = np.zeros(shape, dtype=np.float32)
            continue
        fan_in = int(np.prod(shape[1:]))
        bound = np.sqrt((3.0 if name == "fc2_w" else 6.0) / fan_in)
        u = uniform01_f32(stream_seed(seed, i), int(np.prod(shape)))
        params[name] = ((2.0 * u - 1.0) * bound).astype(np.float32).reshape(shape)
    return params
