"""Pins of the oracle's density models inside a tet (an extension of the
paper's one density value per tet): linear interpolation between trilinear
vertex samples with the largest vertex value as majorant, and voxel lookup
against the largest voxel of the tet's box.  Checked against scipy's
trilinear interpolation, brute-force box maxima, the exact reduction to the
plain tracer for a constant volume, closed-form transmittance of an
absorber, and the regular-grid tracer (no GPU)."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st
from scipy import ndimage

import oracle
import synthetic

S = 1 << 20
TINY = synthetic.scene("tiny")


def uniform_grid(density, n, depth):
    b = dict(want_mode=1, uniform_depth=depth, max_depth=depth, density_scale=1.0, max_tets=1 << 20)
    return oracle.leb_build(np.ascontiguousarray(density, np.float32), n, TINY["camera"], b)


def adaptive_grid(density, n):
    b = dict(want_mode=0, uniform_depth=0, max_depth=13, majorant_mode=0, variation_tau=0.2, target_px=1.0,
             density_scale=1.0, max_tets=1 << 20)
    return oracle.leb_build(np.ascontiguousarray(density, np.float32), n, TINY["camera"], b)


def trilinear_scipy(density, n, pts_world):
    """Clamp-to-edge trilinear interpolation of voxel-centre samples."""
    vol = np.asarray(density, np.float64).reshape(n, n, n)  # [z, y, x]
    c = pts_world * n - 0.5
    return ndimage.map_coordinates(vol, [c[:, 2], c[:, 1], c[:, 0]], order=1, mode="nearest")


def eval_linear(coef, x):
    """sigma(x) in FP32 in the evaluation order of the tracer."""
    c = coef.astype(np.float32)
    x = x.astype(np.float32)
    return ((c[:, 0] + c[:, 1] * x[:, 0]) + c[:, 2] * x[:, 1]) + c[:, 3] * x[:, 2]


@pytest.fixture(scope="module")
def rough():
    rng = np.random.default_rng(12)
    n = 16
    d = (synthetic.blobs(4, n) * 3.0 + rng.uniform(0.0, 0.5, n ** 3)).astype(np.float32)
    return d, n


def test_linear_vertex_values(rough):
    d, n = rough
    g = adaptive_grid(d, n)
    scale = 1.75
    g.set_density_model(1, d, n, scale)
    m = g.export_density_model()
    verts = g.export()["verts"].astype(np.float64) / S  # (T, 4, 3) world
    T = len(verts)
    rho = scale * trilinear_scipy(d, n, verts.reshape(-1, 3)).reshape(T, 4)
    # the majorant is the largest vertex value
    np.testing.assert_allclose(m["majorant"], rho.max(axis=1), rtol=2e-7, atol=1e-7)
    # the affine function takes the vertex values at the vertices
    c = m["coef"].astype(np.float64)
    at_v = c[:, None, 0] + np.einsum("ta,tja->tj", c[:, 1:], verts)
    mag = np.abs(c[:, None, 0]) + np.einsum("ta,tja->tj", np.abs(c[:, 1:]), np.abs(verts)) + np.abs(rho)
    assert np.all(np.abs(at_v - rho) <= 4e-7 * mag + 1e-7)
    assert T > 1000


def test_linear_interior_points(rough):
    """Inside each tet the extinction is the barycentric blend of the
    vertex values, and never above the majorant (up to FP32 rounding)."""
    d, n = rough
    g = adaptive_grid(d, n)
    g.set_density_model(1, d, n, 1.0)
    m = g.export_density_model()
    verts = g.export()["verts"].astype(np.float64) / S
    T = len(verts)
    rho = trilinear_scipy(d, n, verts.reshape(-1, 3)).reshape(T, 4)
    rng = np.random.default_rng(3)
    lam = rng.dirichlet(np.ones(4), size=T)
    x = np.einsum("tj,tja->ta", lam, verts)
    s32 = eval_linear(m["coef"], x).astype(np.float64)
    blend = np.einsum("tj,tj->t", lam, rho)
    scale_mag = np.abs(m["coef"][:, 0]) + np.abs(m["coef"][:, 1:]).sum(axis=1) + 1.0
    assert np.all(np.abs(s32 - blend) <= 1e-6 * scale_mag)
    assert np.all(s32 <= m["majorant"] + 1e-6 * scale_mag)


def test_voxel_majorant_brute_force(rough):
    d, n = rough
    g = adaptive_grid(d, n)
    scale = 2.5
    g.set_density_model(2, d, n, scale)
    m = g.export_density_model()
    assert m["coef"] is None
    vol = d.reshape(n, n, n)
    vs = S // n
    verts = g.export()["verts"]
    ref = np.empty(len(verts), np.float32)
    for t, v in enumerate(verts):
        lo, hi = v.min(axis=0) // vs, -(-v.max(axis=0) // vs)
        ref[t] = np.float32(np.float64(np.float32(scale)) * np.float64(vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].max()))
    assert np.array_equal(m["majorant"], ref)


@pytest.mark.parametrize("model,trans", [(1, 0), (1, 1), (1, 2), (2, 1), (2, 2)])
def test_constant_volume_is_the_plain_tracer(model, trans):
    """A constant volume: every model gives the tet's own value everywhere,
    so the image and event counts are exactly the plain tracer's."""
    n = 8
    d = np.full(n ** 3, 1.5, np.float32)
    b = dict(want_mode=1, uniform_depth=5, max_depth=5, density_scale=2.0, max_tets=1 << 20)
    g = oracle.leb_build(d, n, TINY["camera"], b)
    cam = dict(TINY["camera"], width=20, height=20)
    r = dict(TINY["render"], transmittance=trans)
    a, sa = g.render(cam, TINY["medium"], TINY["light"], 4, 5, r, threads=4)
    g.set_density_model(model, d, n, 2.0)
    bimg, sb = g.render(cam, TINY["medium"], TINY["light"], 4, 5, r, threads=4)
    assert np.array_equal(a, bimg)
    assert sa == sb and sb["null_collisions"] == 0
    g.set_density_model(0)
    c, _ = g.render(cam, TINY["medium"], TINY["light"], 4, 5, r, threads=4)
    assert np.array_equal(a, c)


def footprint_rays(cam, k):
    """Unit directions through a k x k sub-grid of every pixel (same
    pinhole model as the tracer), shape (H, W, k, k, 3)."""
    W, H = cam["width"], cam["height"]
    pos = np.array(cam["pos"], np.float64)
    f = np.array(cam["look_at"], np.float64) - pos
    f /= np.linalg.norm(f)
    r = np.cross(f, cam["up"])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    ty = math.tan(math.radians(cam["fov_y_deg"]) / 2)
    tx = ty * W / H
    sub = (np.arange(k) + 0.5) / k
    px = np.arange(W)[None, :, None, None] + sub[None, None, None, :]
    py = np.arange(H)[:, None, None, None] + sub[None, None, :, None]
    xs = (2 * px / W - 1) * tx
    ys = (1 - 2 * py / H) * ty
    dirs = f + xs[..., None] * r + ys[..., None] * u
    return pos, dirs / np.linalg.norm(dirs, axis=-1, keepdims=True)


def optical_depth_z(pos, dirs, fz, planes):
    """Integral of fz(z) along each ray through the unit cube, exactly for
    fz linear between the given z planes (midpoint rule per piece)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (0.0 - pos) / dirs
        t1 = (1.0 - pos) / dirs
    tmin = np.maximum(np.nanmax(np.minimum(t0, t1), axis=-1), 0.0)
    tmax = np.nanmin(np.maximum(t0, t1), axis=-1)
    hit = tmax > tmin
    dz = dirs[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tp = (np.asarray(planes)[None, :] - pos[2]) / dz.reshape(-1, 1)
    tp = tp.reshape(dz.shape + (len(planes),))
    tp = np.clip(np.nan_to_num(tp, nan=0.0, posinf=0.0, neginf=0.0), tmin[..., None], tmax[..., None])
    ts = np.sort(np.concatenate([tmin[..., None], tp, tmax[..., None]], axis=-1), axis=-1)
    mid = 0.5 * (ts[..., 1:] + ts[..., :-1])
    z = pos[2] + mid * dz[..., None]
    od = (np.diff(ts, axis=-1) * fz(z)).sum(axis=-1)
    return np.where(hit, od, 0.0)


@pytest.mark.parametrize("model", [1, 2])
def test_absorber_closed_form(model):
    """Pure absorber whose voxels grow linearly with z: a camera sample
    escapes with probability exp(-optical depth), the depth integrated
    exactly along the ray for the model's extinction (linear: the clamped
    linear profile, exact on a grid whose tets never straddle its kinks at
    z = 1/2n and 1 - 1/2n; voxel: the staircase of the voxel values)."""
    n, a, b, scale = 8, 0.2, 3.0, 1.5
    zc = (np.arange(n) + 0.5) / n
    d = np.broadcast_to((a + b * zc)[:, None, None], (n, n, n)).astype(np.float32).reshape(-1)
    # linear: tets inside cubes of side 1/16; voxel: cubes of side 1/4, two
    # voxel layers each, so that lookups below the majorant happen
    g = uniform_grid(d, n, 12 if model == 1 else 6)
    g.set_density_model(model, d, n, scale)
    env = np.array([0.3, 0.4, 0.5])
    light = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[0.0, 0.0, 0.0], env_radiance=env.tolist())
    W = H = 12
    cam = dict(pos=[0.45, 0.5, -1.1], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=45.0, width=W, height=H)
    spp = 256
    img, st = g.render(cam, dict(albedo=0.0, g=0.0), light, spp, 17,
                       dict(max_bounces=1, transmittance=2, max_steps_per_path=1 << 20), threads=8)
    assert st["null_collisions"] > 0
    pos, dirs = footprint_rays(cam, 12)
    if model == 1:
        def fz(z):
            return scale * (a + b * np.clip(z, 0.5 / n, 1 - 0.5 / n))
        planes = [0.5 / n, 1 - 0.5 / n]
    else:
        def fz(z):
            return scale * (a + b * (np.clip(np.floor(z * n), 0, n - 1) + 0.5) / n)
        planes = list(np.arange(1, n) / n)
    p = np.exp(-optical_depth_z(pos, dirs, fz, planes)).mean(axis=(2, 3))  # (H, W)
    expect = p[..., None] * env
    var = (p * (1 - p))[..., None] * env ** 2
    z = np.abs(img - expect) / np.sqrt(var / spp + 1e-12)
    assert z.max() < 5.5, z.max()


def seed_stats(render, seeds):
    imgs = np.stack([render(s) for s in seeds])
    return imgs.mean(axis=0), imgs.var(axis=0, ddof=1)


def mean_sq_z(a, b, k):
    (ma, va), (mb, vb) = a, b
    z2 = (ma - mb) ** 2 / ((va + vb) / k + 1e-12)
    return float(z2.mean())


def test_voxel_model_matches_the_regular_grid():
    """Voxel lookup against tet majorants estimates the same image as the
    regular-grid (DDA) tracer over the voxels; the one-value-per-tet grid
    does not."""
    n = 16
    d = (synthetic.blobs(6, n) * 4.0).astype(np.float32)
    scale = 2.0
    b = dict(want_mode=1, uniform_depth=6, max_depth=6, density_scale=scale, max_tets=1 << 20)
    g = oracle.leb_build(d, n, TINY["camera"], b)
    cam = dict(TINY["camera"], width=14, height=14)
    med, light = TINY["medium"], TINY["light"]
    r = dict(max_bounces=6, transmittance=2, max_steps_per_path=1 << 20)
    seeds, spp = list(range(100, 108)), 24
    plain = seed_stats(lambda s: g.render(cam, med, light, spp, s, r, threads=8)[0], seeds)
    g.set_density_model(2, d, n, scale)
    vox = seed_stats(lambda s: g.render(cam, med, light, spp, s, r, threads=8)[0], seeds)
    dda = seed_stats(lambda s: oracle.dda_render(d, n, scale, cam, med, light, spp, s + 1000, r, threads=8)[0], seeds)
    k = len(seeds)
    assert mean_sq_z(vox, dda, k) < 2.0
    assert mean_sq_z(plain, dda, k) > 4.0  # the test tells the two media apart


def test_linear_model_light_estimators_agree():
    """The analytic light transmittance of the linear model (trapezoid per
    segment) and the ratio- and delta-tracking estimators estimate the same
    image."""
    n = 16
    d = (synthetic.blobs(8, n) * 5.0).astype(np.float32)
    g = uniform_grid(d, n, 6)
    g.set_density_model(1, d, n, 1.5)
    cam = dict(TINY["camera"], width=14, height=14)
    med, light = TINY["medium"], TINY["light"]
    seeds, spp = list(range(8)), 24
    res = {}
    for tr in (0, 1, 2):
        r = dict(max_bounces=4, transmittance=tr, max_steps_per_path=1 << 20)
        res[tr] = seed_stats(lambda s: g.render(cam, med, light, spp, s, r, threads=8)[0], seeds)
    assert mean_sq_z(res[0], res[1], len(seeds)) < 2.0
    assert mean_sq_z(res[0], res[2], len(seeds)) < 2.0


def test_density_model_input_checks():
    n = 8
    d = np.ones(n ** 3, np.float32)
    g = uniform_grid(d, n, 3)
    with pytest.raises(oracle.OracleError):
        g.set_density_model(3, d, n, 1.0)
    with pytest.raises(oracle.OracleError):
        g.set_density_model(1, np.ones(6 ** 3, np.float32), 6, 1.0)  # n not a power of two
    bad = d.copy()
    bad[9] = -1.0
    with pytest.raises(oracle.OracleError):
        g.set_density_model(1, bad, n, 1.0)
    with pytest.raises(oracle.OracleError):  # no model set
        g.export_density_model()
    g.set_density_model(2, d, n, 1.0)
    with pytest.raises(oracle.OracleError):  # voxel lookups: no analytic light transmittance
        g.render(TINY["camera"], TINY["medium"], TINY["light"], 1, 1, dict(TINY["render"], transmittance=0))



@settings(max_examples=25, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31 - 1), logn=st.integers(1, 3), depth=st.integers(0, 8),
       scale=st.floats(0.25, 4.0))
def test_model_bounds_random_volumes(seed, logn, depth, scale):
    """For random volumes (including constant and zero regions) and grid
    depths: the linear model never exceeds its majorant inside a tet (FP32
    evaluation, tolerance of its rounding) and reproduces the vertex values;
    the voxel model's majorant is the largest voxel value any interior point
    of the tet can look up."""
    n = 2 ** logn
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.0, 5.0, n ** 3).astype(np.float32)
    d[rng.random(n ** 3) < 0.3] = 0.0
    g = uniform_grid(d, n, depth)
    verts = g.export()["verts"].astype(np.float64) / S
    T = len(verts)
    g.set_density_model(1, d, n, scale)
    m = g.export_density_model()
    lam = rng.dirichlet(np.ones(4), size=T)
    x = np.einsum("tj,tja->ta", lam, verts)
    s32 = eval_linear(m["coef"], x).astype(np.float64)
    mag = np.abs(m["coef"][:, 0]) + np.abs(m["coef"][:, 1:]).sum(axis=1) + 1.0
    assert np.all(s32 <= m["majorant"] + 1e-6 * mag)
    rho = scale * trilinear_scipy(d, n, verts.reshape(-1, 3)).reshape(T, 4)
    np.testing.assert_allclose(m["majorant"], rho.max(axis=1), rtol=2e-7, atol=1e-6)
    g.set_density_model(2, d, n, scale)
    m2 = g.export_density_model()
    vol = d.reshape(n, n, n)
    idx = np.clip(np.floor(x * n).astype(np.int64), 0, n - 1)
    looked = np.float32(scale) * vol[idx[:, 2], idx[:, 1], idx[:, 0]]
    assert np.all(looked <= m2["majorant"])
