"""Seeded synthetic inputs for the fast-HOG hot path.

This module only draws random inputs; it holds none of the method's
arithmetic (no gradients, bins, integrals or scores), so both the HIP path
and the CPU oracle can be fed from it without sharing any computation.

Images stand in for the paper's inputs (800x600 colour frames and 352x288
video frames for vehicle detection, Sec. 1 and Sec. 4); the paper names no
public dataset and ships none. Each channel is, independently,

    128 + noise + sum_{k<4} A_k sin(2 pi f_k (x cos t_k + y sin t_k) + p_k)

rounded to nearest and clipped to 0..255, with x the column and y the row.
For each channel the draws happen in this order: the four gratings, each
as (A ~ U[16,64], f ~ U[1/96, 1/6] cycles/px, t ~ U[0, pi), p ~ U[0, 2 pi)),
then i.i.d. noise ~ U[-32, 32] per pixel. Clipping leaves flat saturated
patches, so zero-gradient pixels occur in realistic numbers.
"""
from __future__ import annotations

import numpy as np

# Seeds of the standard workloads.
SEED_IMAGE_BASE = 1000       # image of workload i uses 1000 + i
SEED_BATCH_BASE = 4000       # batched image j uses 4000 + j
SEED_TEMPLATE_BASE = 9000    # templates of workload i use 9000 + i
SEED_SERVING = 5000


def synth_image(width: int, height: int, channels: int, seed: int) -> np.ndarray:
    """uint8 image of shape (height, width, channels), channels interleaved."""
    if width < 1 or height < 1 or channels < 1:
        raise ValueError("image dimensions must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.arange(width, dtype=np.float64)[None, :]
    y = np.arange(height, dtype=np.float64)[:, None]
    out = np.empty((height, width, channels), dtype=np.uint8)
    for ch in range(channels):
        acc = np.full((height, width), 128.0)
        for _ in range(4):
            amp = rng.uniform(16.0, 64.0)
            freq = rng.uniform(1.0 / 96.0, 1.0 / 6.0)
            theta = rng.uniform(0.0, np.pi)
            phase = rng.uniform(0.0, 2.0 * np.pi)
            acc += amp * np.sin(2.0 * np.pi * freq * (x * np.cos(theta) + y * np.sin(theta)) + phase)
        acc += rng.uniform(-32.0, 32.0, size=(height, width))
        out[:, :, ch] = np.clip(np.rint(acc), 0, 255).astype(np.uint8)
    return out


def synth_templates(k: int, dim: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """K linear templates: weights N(0,1) as float32 of shape (k, dim), bias 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((k, dim), dtype=np.float32)
    b = np.zeros((k,), dtype=np.float32)
    return w, b


def synth_bin_map(width: int, height: int, n_bins: int, seed: int,
                  empty_frac: float = 0.1) -> np.ndarray:
    """A random bin map (uint8, height x width) with values in 0..n_bins-1 and
    about `empty_frac` of the entries set to 255 (no bin). Used to drive the
    integral and window stages directly, independent of any image."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.integers(0, n_bins, size=(height, width), dtype=np.uint8)
    if empty_frac > 0:
        m[rng.random((height, width)) < empty_frac] = 255
    return m
