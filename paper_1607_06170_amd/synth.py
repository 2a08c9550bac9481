"""Seeded synthetic inputs and workload shapes.

This module holds numbers and random draws only -- none of the method's
arithmetic -- so that the tests can feed the same inputs to the library and to
the oracle.  The paper's own workload (GATE responses, the Eplus-260 scanner,
Derenzo and point-source data) is not available; these shapes stand in for a
small-animal / primate PET ring and are described next to each constant.
"""
from __future__ import annotations

import numpy as np

# 2D single ring: 16 blocks x 8 LYSO crystals of 2 mm pitch and 15 mm depth,
# front faces 65 mm from the centre, 64 x 64 image of 1 mm voxels.  The block
# size and the 65 mm radius fix the gap between blocks (about 9.7 mm at the
# front corners).
CFG_2D = dict(n_blocks=16, n_ct=8, n_cz=1, n_brings=1, pitch_t=2.0, pitch_z=2.0, depth=15.0, r_face=65.0,
              gap_z=0.0, mu=0.087, phi0=0.0, nx=64, ny=64, nz=1, dx=1.0, dy=1.0, dz=1.0,
              n_rows=61, n_sub=4, step_deg=1.0, threshold=1e-6)

# The same crystals with a 0.5 mm gap between neighbouring blocks' front
# corners: faces 41.4756 mm from the centre.  A 44 x 44 image fits inside.
# Here photons cross into the neighbouring block (two-block penetration).
CFG_2D_NARROW = dict(CFG_2D, r_face=8.25 / np.tan(np.pi / 16), nx=44, ny=44)

# 3D: 32 blocks per ring of 12 x 12 crystals (2 x 2 x 15 mm), 4 block rings
# (48 crystal rings, no axial gap), faces 130 mm from the axis; 128 x 128 x 96
# image of 1 mm voxels.  Tables: 61 x 61 angle rows x 4 x 4 sub-positions x
# 5 x 5 neighbours.
CFG_3D = dict(n_blocks=32, n_ct=12, n_cz=12, n_brings=4, pitch_t=2.0, pitch_z=2.0, depth=15.0, r_face=130.0,
              gap_z=0.0, mu=0.087, phi0=0.0, nx=128, ny=128, nz=96, dx=1.0, dy=1.0, dz=1.0,
              n_rows=61, n_sub=4, step_deg=1.0, threshold=0.0)


# A small 3D scanner for element-by-element checks: 12 blocks of 4 x 4
# crystals (2 mm, 10 mm deep), 2 block rings (8 crystal rings), faces 16 mm
# from the axis (1.1 mm half-gap, so photons cross into the next block);
# 10 x 10 x 6 image of 1 mm voxels; tables cover 0-90 degrees.
CFG_3D_SMALL = dict(n_blocks=12, n_ct=4, n_cz=4, n_brings=2, pitch_t=2.0, pitch_z=2.0, depth=10.0, r_face=16.0,
                    gap_z=0.0, mu=0.087, phi0=0.0, nx=10, ny=10, nz=6, dx=1.0, dy=1.0, dz=1.0,
                    n_rows=91, n_sub=4, step_deg=1.0, threshold=0.0)


def phantom_uniform(cfg: dict, seed: int = 1, batch: int = 1) -> np.ndarray:
    """Uniform [0, 1) random image(s), float64, shape [batch, n_voxels]."""
    rng = np.random.default_rng(seed)
    n = cfg["nx"] * cfg["ny"] * cfg.get("nz", 1)
    return rng.random((batch, n))


def phantom_blobs(cfg: dict, seed: int = 2, n_blobs: int = 20) -> np.ndarray:
    """Uniform cylinder (r <= 55 mm, |z| <= 48 mm, value 1) plus n_blobs
    isotropic Gaussian blobs: centres uniform in r <= 45, |z| <= 40, sigma
    uniform in [2, 10] mm, amplitude uniform in [1, 4].  Shape [n_voxels]."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg.get("nz", 1)
    x = (np.arange(nx) - 0.5 * (nx - 1)) * cfg["dx"]
    y = (np.arange(ny) - 0.5 * (ny - 1)) * cfg["dy"]
    z = (np.arange(nz) - 0.5 * (nz - 1)) * cfg.get("dz", 1.0)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    img = ((X ** 2 + Y ** 2 <= 55.0 ** 2) & (np.abs(Z) <= 48.0)).astype(np.float64)
    for _ in range(n_blobs):
        r = 45.0 * np.sqrt(rng.random())
        th = 2 * np.pi * rng.random()
        cz = rng.uniform(-40.0, 40.0)
        s = rng.uniform(2.0, 10.0)
        amp = rng.uniform(1.0, 4.0)
        cx, cy = r * np.cos(th), r * np.sin(th)
        img += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) / (2 * s * s))
    return img.reshape(-1)


def random_table(shape, seed: int = 5, scale: float = 0.3) -> np.ndarray:
    """A seeded table of non-negative entries (for gradient and FD checks)."""
    rng = np.random.default_rng(seed)
    return scale * rng.random(shape)


def poisson_counts(mean: np.ndarray, seed: int = 200) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.poisson(mean).astype(np.float64)


def sample_events(weights: np.ndarray, n_true: int, n_randoms: int, seed: int = 300) -> np.ndarray:
    """Bin indices of list-mode events: n_true drawn with probability
    proportional to ``weights`` (an expected-count sinogram), n_randoms uniform
    over the bins with positive weight, then shuffled.  int64 [n_events]."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64).reshape(-1)
    p = w / w.sum()
    trues = rng.choice(w.size, size=n_true, p=p)
    valid = np.nonzero(w > 0)[0]
    rnd = valid[rng.integers(0, valid.size, size=n_randoms)]
    ev = np.concatenate([trues, rnd])
    rng.shuffle(ev)
    return ev.astype(np.int64)


def bin_to_pair(bins: np.ndarray, n: int):
    """Crystal pair (i < j) of canonical bin indices (inverse of the
    ordering of unordered pairs by (min, max)); a pure index map."""
    bins = np.asarray(bins, dtype=np.int64)
    # row i starts at i*n - i*(i+1)/2
    starts = np.array([i * n - i * (i + 1) // 2 for i in range(n)], dtype=np.int64)
    i = np.searchsorted(starts, bins, side="right") - 1
    j = bins - starts[i] + i + 1
    return i.astype(np.int32), j.astype(np.int32)
