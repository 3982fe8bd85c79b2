"""Comparison helpers shared by the GPU parity tests."""
import numpy as np

# Image parity bar: per pixel, the largest channel error relative to the
# reference (floored at 1e-4 of the reference image mean) must be <= 1e-4 on
# at least 99.9 % of pixels, and its mean over pixels <= 1e-3.
PIX_TOL = 1e-4
PIX_FRAC = 0.999
MEAN_TOL = 1e-3


def rel_errors(gpu, ref):
    g = np.asarray(gpu, np.float64).reshape(-1, 3)
    c = np.asarray(ref, np.float64).reshape(-1, 3)
    floor = 1e-4 * max(float(np.abs(c).mean()), 1e-30)
    return (np.abs(g - c) / np.maximum(np.abs(c), floor)).max(axis=1)


def assert_image_parity(gpu, ref, what=""):
    rel = rel_errors(gpu, ref)
    frac = float((rel <= PIX_TOL).mean())
    mean = float(rel.mean())
    assert frac >= PIX_FRAC and mean <= MEAN_TOL, \
        f"{what}: {frac * 100:.3f}% of pixels within {PIX_TOL}, mean rel {mean:.3g}, worst {rel.max():.3g}"
    return frac, mean


def assert_grids_equal(gpu: dict, ref: dict, what=""):
    assert gpu["ids"].shape == ref["ids"].shape, f"{what}: {len(gpu['ids'])} vs {len(ref['ids'])} tets"
    for k in ["ids", "nbr", "verts", "sigma", "majorant"]:
        a, b = gpu[k], ref[k]
        if k in ("sigma", "majorant"):
            eq = a.view(np.uint32) == b.view(np.uint32)
        else:
            eq = a == b
        assert eq.all(), f"{what}: {k} differs at {np.argwhere(~eq)[:5].tolist()} of {a.shape}"
