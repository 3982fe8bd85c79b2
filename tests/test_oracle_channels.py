"""Pins of the oracle's extra channels (the paper's implementation carries
e.g. temperature, albedo and phase-function parameters per tet): per-tet
means against brute force, reductions to the plain tracer, and the emission
of a pure absorber against its closed form (no GPU)."""
import math

import numpy as np
import pytest

import oracle
import synthetic

S = 1 << 20
TINY = synthetic.scene("tiny")


def uniform_grid(density, n, depth):
    b = dict(want_mode=1, uniform_depth=depth, max_depth=depth, density_scale=1.0, max_tets=1 << 20)
    return oracle.leb_build(np.ascontiguousarray(density, np.float32), n, TINY["camera"], b)


def box_mean_brute(verts, ch, n):
    """Mean of the voxels overlapping the open bounding box of each tet, by
    direct summation (voxel index ranges from the lattice box)."""
    vs = S // n
    grid = ch.reshape(n, n, n).astype(np.float64)  # [z, y, x]
    out = np.empty(len(verts))
    for t, v in enumerate(verts):
        lo, hi = v.min(axis=0), v.max(axis=0)
        r0 = lo // vs
        r1 = -(-hi // vs)
        out[t] = grid[r0[2]:r1[2], r0[1]:r1[1], r0[0]:r1[0]].mean()
    return out


def test_channel_means_against_brute_force():
    rng = np.random.default_rng(5)
    n = 16
    g = uniform_grid(np.ones(n ** 3), n, 7)
    temp = rng.uniform(0.0, 4.0, n ** 3).astype(np.float32)
    alb = rng.uniform(0.0, 1.0, n ** 3).astype(np.float32)
    gg = rng.uniform(-0.9, 0.9, n ** 3).astype(np.float32)
    g.set_channels(n, temperature=temp, albedo=alb, g=gg)
    ch = g.export_channels()
    verts = g.export()["verts"]
    for name, src in (("temperature", temp), ("albedo", alb), ("g", gg)):
        ref = box_mean_brute(verts, src, n)
        np.testing.assert_allclose(ch[name], ref, rtol=2e-7, atol=1e-7, err_msg=name)
    # absent channels are absent
    g.set_channels(n, albedo=alb)
    ch = g.export_channels()
    assert ch["temperature"] is None and ch["g"] is None and ch["albedo"] is not None


def test_channel_input_checks():
    n = 8
    g = uniform_grid(np.ones(n ** 3), n, 3)
    bad = np.full(n ** 3, 0.5, np.float32)
    bad[3] = 1.5
    with pytest.raises(oracle.OracleError):
        g.set_channels(n, albedo=bad)
    bad[3] = 1.0
    with pytest.raises(oracle.OracleError):
        g.set_channels(n, g=bad)
    bad[3] = -0.25
    with pytest.raises(oracle.OracleError):
        g.set_channels(n, temperature=bad)
    # channels requested on a grid without them
    with pytest.raises(oracle.OracleError):
        g.render(TINY["camera"], TINY["medium"], TINY["light"], 1, 1, dict(TINY["render"], channels=1))


@pytest.mark.parametrize("alb,gv", [(0.9, 0.3), (0.55, -0.5), (1.0, 0.8)])
def test_constant_channels_are_the_plain_tracer(alb, gv):
    """Constant albedo and g channels (and zero temperature) give exactly
    the image of the plain tracer whose medium has those values: the
    per-tet values replace the medium's at the throughput, the light
    estimate and the phase sample, and nothing else changes."""
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]()
    g = oracle.leb_build(d, sc["n"], sc["camera"], sc["build"])
    n = 8
    g.set_channels(n, temperature=np.zeros(n ** 3, np.float32), albedo=np.full(n ** 3, alb, np.float32),
                   g=np.full(n ** 3, gv, np.float32))
    ch = g.export_channels()
    assert (ch["albedo"] == np.float32(alb)).all() and (ch["g"] == np.float32(gv)).all()
    cam = dict(sc["camera"], width=24, height=24)
    med_plain = dict(albedo=alb, g=gv)
    a, sa = g.render(cam, med_plain, sc["light"], 8, 77, sc["render"], threads=4)
    b, sb = g.render(cam, dict(albedo=0.3, g=0.0), sc["light"], 8, 77,
                     dict(sc["render"], channels=1, emission=[2.0, 1.0, 0.5]), threads=4)
    assert np.array_equal(a, b)
    assert sa == sb


def test_emitting_absorber_closed_form():
    """Pure absorber (albedo channel 0) of uniform extinction s and uniform
    temperature T: a camera ray through the cube over length l sees
    T e (1 - exp(-s l)) + env exp(-s l) (the emission estimator scores
    T e at the single real collision, else the ray leaves to the
    environment); misses see env."""
    n, s, T = 8, 2.5, 3.0
    em = np.array([0.8, 0.5, 0.2])
    env = np.array([0.3, 0.4, 0.5])
    g = uniform_grid(np.full(n ** 3, s), n, 6)
    g.set_channels(n, temperature=np.full(n ** 3, T, np.float32), albedo=np.zeros(n ** 3, np.float32))
    light = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[5.0, 5.0, 5.0], env_radiance=env.tolist())
    W = H = 16
    cam = dict(pos=[0.4, 0.55, -1.3], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=50.0, width=W, height=H)
    spp = 256
    img, st = g.render(cam, dict(albedo=0.5, g=0.2), light, spp, 9,
                       dict(max_bounces=4, transmittance=0, channels=1, emission=em.tolist()), threads=8)
    # ray lengths inside the cube through pixel centres are not the sampled
    # rays (jittered), so compare per pixel against the expectation over the
    # pixel footprint, integrated on a 16 x 16 sub-grid
    pos = np.array(cam["pos"], np.float64)
    f = np.array(cam["look_at"], np.float64) - pos
    f /= np.linalg.norm(f)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    ty = math.tan(math.radians(cam["fov_y_deg"]) / 2)
    tx = ty * W / H
    k = 16
    sub = (np.arange(k) + 0.5) / k
    worst = 0.0
    for py in range(H):
        for px in range(W):
            xs = (2 * ((px + sub[None, :]) / W) - 1) * tx
            ys = (1 - 2 * ((py + sub[:, None]) / H)) * ty
            dirs = f[None, None, :] + xs[..., None] * r[None, None, :] + ys[..., None] * u[None, None, :]
            dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
            with np.errstate(divide="ignore", invalid="ignore"):
                t0 = (0.0 - pos) / dirs
                t1 = (1.0 - pos) / dirs
            tmin = np.nanmax(np.minimum(t0, t1), axis=-1)
            tmax = np.nanmin(np.maximum(t0, t1), axis=-1)
            length = np.clip(tmax - np.maximum(tmin, 0.0), 0.0, None)
            p = 1.0 - np.exp(-s * length)
            pbar = p.mean()  # a sample scores T e with probability pbar, else env
            expect = pbar * (T * em) + (1 - pbar) * env
            var = pbar * (1 - pbar) * (T * em - env) ** 2
            z = np.abs(img[py, px] - expect) / np.sqrt(var / spp + 1e-10)
            worst = max(worst, float(z.max()))
    assert worst < 5.5, worst
    assert st["real_collisions"] > 0
