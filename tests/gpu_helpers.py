"""Shared helpers for the GPU parity tests (comparison metrics and scene sizes)."""
from __future__ import annotations

import math

import numpy as np

# parity bar: per-pixel relative error <= 1e-4; at most 0.1 % of pixels may differ
# through branch flips, and those must stay within 3 sigma of the Monte Carlo noise
REL_TOL = 1e-4
FLIP_FRACTION = 1e-3
FLIP_SIGMAS = 3.0
# pixels sampled at random for the full-size checks (the oracle traces only those): enough that
# the raw flipped fraction resolves FLIP_FRACTION (at most 20 of them)
NPIX_SAMPLED = 20000


def compare_images(gpu: np.ndarray, ref: dict, spp: int, label: str = ""):
    """Element-wise comparison of a GPU image with the oracle's mean/variance images.

    The relative error uses a floor of 1e-6 of the image maximum so that pixels holding
    only round-off sized radiance do not dominate.  Returns a stats dict."""
    o = ref["mean"]
    g = np.asarray(gpu, np.float64)
    floor = 1e-6 * max(float(np.abs(o).max()), 1e-30)
    rel = np.abs(g - o) / np.maximum(np.abs(o), floor)
    bad = rel > REL_TOL
    se = np.sqrt(np.maximum(ref["var"], 0.0) / spp)
    within = np.abs(g - o) <= FLIP_SIGMAS * se + floor
    stats = {
        "label": label,
        "n_pixels": int(o.size),
        "n_flipped": int(bad.sum()),
        "flip_fraction": float(bad.mean()),
        "max_rel_unflipped": float(rel[~bad].max()) if (~bad).any() else 0.0,
        "flipped_outside_3sigma": int((bad & ~within).sum()),
        "mean_abs_diff": float(np.abs(g - o).mean()),
        "image_mean": float(o.mean()),
    }
    return stats


def assert_parity(stats: dict):
    msg = str(stats)
    assert stats["flip_fraction"] <= FLIP_FRACTION, msg
    assert stats["flipped_outside_3sigma"] == 0, msg
    assert stats["max_rel_unflipped"] <= REL_TOL, msg


def compare_paths(gpu_paths: np.ndarray, ref_paths: np.ndarray):
    g = np.asarray(gpu_paths, np.float64).ravel()
    o = np.asarray(ref_paths, np.float64).ravel()
    floor = 1e-6 * max(float(np.abs(o).max()), 1e-30)
    rel = np.abs(g - o) / np.maximum(np.abs(o), floor)
    return {"n_paths": int(o.size), "paths_over_tol": int((rel > REL_TOL).sum()),
            "path_flip_fraction": float((rel > REL_TOL).mean()),
            "max_rel_path": float(rel.max())}


def se_of(ref, spp):
    return np.sqrt(np.maximum(ref["var"], 0) / spp)


def fmt(stats: dict) -> str:
    return " ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}" for k, v in stats.items())


def isclose_rel(a, b, rel):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


__all__ = ["compare_images", "assert_parity", "compare_paths", "fmt", "math"]


def compare_sampled(gpu_vals, ref: dict, spp: int, label: str = ""):
    """Sampled-pixel comparison: gpu_vals and ref['mean'/'var'] are 1-D over the samples."""
    o = np.asarray(ref["mean"], np.float64)
    g = np.asarray(gpu_vals, np.float64)
    floor = 1e-6 * max(float(np.abs(o).max()), 1e-30)
    rel = np.abs(g - o) / np.maximum(np.abs(o), floor)
    bad = rel > REL_TOL
    se = np.sqrt(np.maximum(ref["var"], 0.0) / spp)
    within = np.abs(g - o) <= FLIP_SIGMAS * se + floor
    return {"label": label, "n_pixels": int(o.size), "n_flipped": int(bad.sum()),
            "flip_fraction": float(bad.mean()),
            "max_rel_unflipped": float(rel[~bad].max()) if (~bad).any() else 0.0,
            "flipped_outside_3sigma": int((bad & ~within).sum()), "image_mean": float(o.mean())}


def assert_sampled_parity(stats: dict):
    """The same bar as assert_parity on a sample of the pixels: the raw fraction of sampled
    pixels above the relative tolerance is at most FLIP_FRACTION (no allowance for the
    sampling), each within FLIP_SIGMAS standard errors."""
    msg = str(stats)
    assert stats["flip_fraction"] <= FLIP_FRACTION, msg
    assert stats["flipped_outside_3sigma"] == 0, msg
    assert stats["max_rel_unflipped"] <= REL_TOL, msg
