"""Seeded synthetic frames that stand in for the paper's rendered test set.

The paper evaluates on 1080p path-traced frames with noise-free guide images
(albedo, normals, depth, ambient occlusion) and 1 spp noisy indirect lighting
(Sec. 4.1, "Dataset"). That data set is not available, so these generators
build frames with the same shapes, channel types and noise character:

* guides: piecewise-planar depth over seeded Voronoi regions, the plane
  normals, an ambient-occlusion-like blurred random field in [0, 1], and (for
  the RGB configuration) piecewise-constant albedo;
* clean shading: a sum of three seeded clamped-cosine lobes over the normals,
  times the AO field (Lambertian-like, albedo-free, Sec. 3 Eqs. 2-3);
* noisy input: clean x i.i.d. Exponential(1) per pixel and channel, which has
  mean 1 like a 1 spp estimator; optionally a 10% firefly mask multiplies by
  a Pareto(alpha = 1.5) factor.

This module contains no part of the regression method: it only draws inputs.
It is shared by the oracle's tests, the GPU parity tests and the benchmark.
All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter
from scipy.spatial import cKDTree

__all__ = ["make_frame", "make_config", "CONFIGS", "small_integer_frame", "random_frame"]


def _pixel_centres(h: int, w: int):
    u = (np.arange(w, dtype=np.float64) + 0.5) / w
    v = (np.arange(h, dtype=np.float64) + 0.5) / h
    return np.meshgrid(u, v)  # (h, w) each


def _voronoi_labels(rng, n_cells: int, uu, vv):
    seeds = rng.uniform(0.0, 1.0, size=(n_cells, 2))
    tree = cKDTree(seeds)
    pts = np.stack([uu.ravel(), vv.ravel()], axis=1)
    _, lab = tree.query(pts)
    return seeds, lab.reshape(uu.shape)


def _unit_hemisphere(rng, n: int):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[:, 2] = np.abs(d[:, 2])
    return d


def make_frame(h: int, w: int, seed: int, *, rgb: bool, fireflies: bool,
               n_regions: int = 6, n_albedo_cells: int = 40, ao_sigma: float = 8.0):
    """Build one synthetic frame.

    Returns a dict of float32 arrays: ``noisy`` [C,H,W], ``guides`` [Q,H,W],
    ``clean`` [C,H,W], plus ``guide_names``. With ``rgb`` the guides are
    albedo RGB, nx, ny, nz, depth, AO (Q = 8) and C = 3; otherwise AO, depth,
    nx, ny (Q = 4) and C = 1. The implicit constant guide is not included.
    """
    rng = np.random.default_rng(seed)
    uu, vv = _pixel_centres(h, w)

    # Piecewise-planar depth over Voronoi regions, with the plane normals.
    seeds, lab = _voronoi_labels(rng, n_regions, uu, vv)
    z0 = rng.uniform(2.0, 9.0, size=n_regions)
    gxy = rng.uniform(-3.0, 3.0, size=(n_regions, 2))
    depth = z0[lab] + gxy[lab, 0] * (uu - seeds[lab, 0]) + gxy[lab, 1] * (vv - seeds[lab, 1])
    depth = np.clip(depth, 1.0, 10.0)
    nrm = np.concatenate([-gxy, np.ones((n_regions, 1))], axis=1)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    normals = nrm[lab]  # (h, w, 3)

    # Ambient-occlusion-like field: blurred white noise rescaled to [0, 1].
    ao = gaussian_filter(rng.standard_normal((h, w)), sigma=ao_sigma, mode="reflect")
    ao = (ao - ao.min()) / max(ao.max() - ao.min(), 1e-12)

    # Clean Lambertian-like shading: three clamped cosine lobes, times AO.
    dirs = _unit_hemisphere(rng, 3)
    wts = rng.uniform(0.5, 1.5, size=3)
    shade = np.zeros((h, w))
    for j in range(3):
        shade += wts[j] * np.maximum(0.0, normals @ dirs[j])
    clean1 = ao * shade

    if rgb:
        tints = rng.uniform(0.5, 1.5, size=3)
        clean = tints[:, None, None] * clean1[None]
        noise = rng.exponential(1.0, size=(3, h, w))
        noisy = clean * noise
        if fireflies:
            mask = rng.random((h, w)) < 0.10
            boost = 1.0 + rng.pareto(1.5, size=(h, w))
            noisy = noisy * np.where(mask, boost, 1.0)[None]
        _, alab = _voronoi_labels(rng, n_albedo_cells, uu, vv)
        alb = rng.uniform(0.05, 0.95, size=(n_albedo_cells, 3))[alab]  # (h, w, 3)
        guides = np.stack([alb[..., 0], alb[..., 1], alb[..., 2],
                           normals[..., 0], normals[..., 1], normals[..., 2],
                           depth, ao])
        names = ["albedo_r", "albedo_g", "albedo_b", "nx", "ny", "nz", "depth", "ao"]
    else:
        clean = clean1[None]
        noisy = clean * rng.exponential(1.0, size=(1, h, w))
        if fireflies:
            mask = rng.random((h, w)) < 0.10
            noisy = noisy * np.where(mask, 1.0 + rng.pareto(1.5, size=(h, w)), 1.0)[None]
        guides = np.stack([ao, depth, normals[..., 0], normals[..., 1]])
        names = ["ao", "depth", "nx", "ny"]

    return {
        "noisy": np.ascontiguousarray(noisy, dtype=np.float32),
        "guides": np.ascontiguousarray(guides, dtype=np.float32),
        "clean": np.ascontiguousarray(clean, dtype=np.float32),
        "guide_names": names,
    }


# The two workload configurations of the regression path:
#  0: one 256x256 frame, one channel, 4 guides + constant (a 5x5 system);
#  1: one 1920x1080 RGB frame with fireflies, 8 guides + constant.
CONFIGS = {
    0: dict(h=256, w=256, seed=0, rgb=False, fireflies=False, radius=8, eps=1e-3),
    1: dict(h=1080, w=1920, seed=1, rgb=True, fireflies=True, radius=8, eps=1e-3),
}


def make_config(i: int, seed: int | None = None, h: int | None = None, w: int | None = None):
    """Frame for workload configuration ``i`` (optionally resized or reseeded)."""
    c = dict(CONFIGS[i])
    fr = make_frame(h or c["h"], w or c["w"], c["seed"] if seed is None else seed,
                    rgb=c["rgb"], fireflies=c["fireflies"])
    fr["radius"] = c["radius"]
    fr["eps"] = c["eps"]
    return fr


def small_integer_frame(h: int, w: int, q: int, c: int, seed: int,
                        gmax: int = 7, ymax: int = 15):
    """Guides in {0..gmax} and noisy values in {0..ymax}, as float32.

    Window sums of products of such values stay below 2**24 for windows of a
    few hundred pixels, so they are exact in float32 arithmetic.
    """
    rng = np.random.default_rng(seed)
    g = rng.integers(0, gmax + 1, size=(q, h, w)).astype(np.float32)
    y = rng.integers(0, ymax + 1, size=(c, h, w)).astype(np.float32)
    return {"noisy": y, "guides": g}


def random_frame(h: int, w: int, q: int, c: int, seed: int, *, smooth: float = 0.0,
                 offset: float = 0.0):
    """Generic random guides / noisy input with optional smoothing and offset."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((q, h, w))
    if smooth > 0:
        g = np.stack([gaussian_filter(gi, smooth, mode="reflect") for gi in g])
        g /= max(np.abs(g).max(), 1e-12)
    g = g + offset
    y = rng.exponential(1.0, size=(c, h, w)) * (1.0 + 0.5 * np.abs(g[:1]))
    return {"noisy": y.astype(np.float32), "guides": g.astype(np.float32)}


def make_training_batch(n: int = 8, crop: int = 256, seed: int = 3, frame_h: int = 512,
                        frame_w: int = 512, samples: int = 256, frame_seed0: int = 100):
    """The FLNR training workload: ``n`` random crop x crop windows, one from
    each of ``n`` frames in the style of configuration 1 (frame seeds
    frame_seed0, frame_seed0 + 1, ..., default 100, 101, ..., generated at
    frame_h x frame_w), each with a target that is the
    mean of ``samples`` independent Exponential(1) noise draws times the clean
    shading. That mean is drawn directly from its distribution,
    Gamma(samples, 1 / samples). Returns a list of dicts with ``guides``
    [8,crop,crop], ``noisy`` and ``target`` [3,crop,crop] (float32)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        fr = make_frame(frame_h, frame_w, frame_seed0 + k, rgb=True, fireflies=True)
        y0 = int(rng.integers(0, frame_h - crop + 1))
        x0 = int(rng.integers(0, frame_w - crop + 1))
        sl = (slice(None), slice(y0, y0 + crop), slice(x0, x0 + crop))
        clean = fr["clean"][sl]
        target = clean * rng.gamma(samples, 1.0 / samples, size=clean.shape)
        out.append({"guides": np.ascontiguousarray(fr["guides"][sl]),
                    "noisy": np.ascontiguousarray(fr["noisy"][sl]),
                    "target": np.ascontiguousarray(target, dtype=np.float32)})
    return out
