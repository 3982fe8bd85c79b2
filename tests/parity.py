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


def assert_faces_equal(g, ref: dict, what=""):
    """The face data the walk reads -- orientation codes and plane offsets of
    the 48-byte and (when the grid has them) the compact records -- equal the
    oracle's, and each layout's links equal the exported neighbour table."""
    nbr = g.export(fields=("nbr",))["nbr"]
    for layout in (48, 32):
        try:
            f = g.export_faces(layout)
        except Exception as e:  # no compact records (loose majorants)
            assert layout == 32 and getattr(e, "status", None) == -1, e
            continue
        assert np.array_equal(f["codes"], ref["codes"]), f"{what}: face codes differ ({layout}-byte records)"
        assert np.array_equal(f["offsets"], ref["offsets"]), f"{what}: plane offsets differ ({layout}-byte records)"
        want = nbr if layout == 48 else np.where(nbr == 0xFFFFFFFF, (1 << 27) - 1, nbr >> 2).astype(np.uint32)
        assert np.array_equal(f["links"], want), f"{what}: links of the {layout}-byte records"
