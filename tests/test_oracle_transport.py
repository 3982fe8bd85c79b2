"""Pins of the oracle's path tracer (paper: Algorithm 1 and "Path Tracing
within Tetrahedral Grids") against closed forms, invariants and special
cases (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import synthetic

S = 1 << 20
NOSUN = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[0.0, 0.0, 0.0], env_radiance=[1.0, 1.0, 1.0])
PENCIL = dict(pos=[0.5, 0.5, -1.0], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=0.01, width=1, height=1)


def homogeneous_grid(sigma, depth=6, n=8):
    d = np.full(n ** 3, sigma, np.float32)
    b = dict(want_mode=1, uniform_depth=depth, max_depth=depth, density_scale=1.0, max_tets=1 << 20)
    return oracle.leb_build(d, n, PENCIL, b)


# ---------------------------------------------------------------- RNG
def test_philox_known_answers():
    """Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) known-answer values
    published with the Random123 reference implementation."""
    assert [hex(x) for x in oracle.philox([0, 0, 0, 0], [0, 0])] == \
        ["0x6627e8d5", "0xe169c58d", "0xbc57ac4c", "0x9b00dbd8"]
    assert [hex(x) for x in oracle.philox([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)] == \
        ["0x408f276d", "0x41c83b0e", "0xa20bc7c6", "0x6d5451fd"]
    assert [hex(x) for x in oracle.philox([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                                          [0xA4093822, 0x299F31D0])] == \
        ["0xd16cfe09", "0x94fdcceb", "0x5001e420", "0x24126ea1"]


def test_uniforms_are_uniform_and_keyed():
    u = np.array([oracle.uniform(7, p, s, 0, 1, j) for p in range(50) for s in range(20) for j in range(10)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert ((u >= 0) & (u < 1)).all()
    # (u * 2^24) is an integer: 24-bit uniforms
    assert np.array_equal(u * 2 ** 24, np.floor(u * 2 ** 24))
    # a different stream / bounce / draw gives a different number
    a = oracle.uniform(7, 3, 4, 0, 1, 0)
    assert a != oracle.uniform(7, 3, 4, 0, 2, 0) and a != oracle.uniform(7, 3, 4, 1, 1, 0)
    assert a != oracle.uniform(7, 3, 4, 0, 1, 1) and a != oracle.uniform(8, 3, 4, 0, 1, 0)


# ---------------------------------------------------------------- elementary functions
def test_elementary_functions_closed_forms():
    """The oracle's -ln(1-u), e^-x and (cos, sin)(2 pi u) at arguments whose
    values are known in closed form (FP64 library functions rounded once)."""
    assert oracle.neglog1m(0.0) == 0.0
    # 1 - u = 2^-k exactly: -ln(2^-k) = k ln 2
    for k in (1, 2, 8, 24):
        u = 1.0 - 2.0 ** -k
        assert oracle.neglog1m(u) == np.float32(k * math.log(2.0))
    assert oracle.neglog1m(0.5) == np.float32(math.log(2.0))
    assert oracle.expneg(0.0) == 1.0 and oracle.expneg(200.0) == 0.0
    for k in (1, 3, 10):
        # e^-(k ln 2) = 2^-k up to the rounding of k ln 2 to FP32
        x = np.float32(k * math.log(2.0))
        assert oracle.expneg(float(x)) == pytest.approx(2.0 ** -k, rel=2e-7)
    assert oracle.sincos2pi(0.0) == (1.0, 0.0)
    c, s = oracle.sincos2pi(0.125)
    assert c == np.float32(math.sqrt(0.5)) and s == np.float32(math.sqrt(0.5))
    c, s = oracle.sincos2pi(1.0 / 12.0)
    assert c == np.float32(math.sqrt(3.0) / 2.0) and s == pytest.approx(0.5, abs=6e-8)
    # -ln(1-u) of a uniform is Exp(1): mean 1 and variance 1 over a fine lattice of u
    u = np.arange(0, 1 << 24, 97) / float(1 << 24)
    t = np.array([oracle.neglog1m(float(x)) for x in u[::64]])
    assert t.mean() == pytest.approx(1.0, abs=0.02) and t.var() == pytest.approx(1.0, abs=0.08)


# ---------------------------------------------------------------- phase function
@pytest.mark.parametrize("g", [-0.7, -0.2, 0.0, 0.3, 0.6, 0.9])
def test_hg_density_and_sampling(g):
    """HG: integrates to 1 over the sphere, mean cosine g, and the sampling
    routine is the inverse of its cumulative distribution."""
    pdf = lambda mu: oracle.hg_eval(g, mu)
    tot = 2 * math.pi * integrate.quad(pdf, -1, 1, epsabs=1e-10, limit=200)[0]
    assert tot == pytest.approx(1.0, abs=2e-6)
    mean = 2 * math.pi * integrate.quad(lambda m: m * pdf(m), -1, 1, limit=200)[0]
    assert mean == pytest.approx(g, abs=2e-6)
    for u in [0.05, 0.3, 0.5, 0.77, 0.95]:
        mu = oracle.hg_sample_mu(g, u)
        cdf = 2 * math.pi * integrate.quad(pdf, -1, mu, limit=200)[0]
        assert cdf == pytest.approx(u, abs=2e-5)
    if g == 0.0:
        assert oracle.hg_eval(0.0, 0.3) == pytest.approx(1 / (4 * math.pi), rel=1e-7)


def test_hg_direction_geometry():
    rng = np.random.default_rng(3)
    for _ in range(200):
        d = rng.normal(size=3)
        d = (d / np.linalg.norm(d)).astype(np.float32)
        g = float(rng.uniform(-0.9, 0.9))
        u1, u2 = np.float32(rng.random()), np.float32(rng.random())
        o = oracle.hg_direction(d, g, u1, u2)
        assert np.linalg.norm(o) == pytest.approx(1.0, abs=1e-6)
        assert float(np.dot(o, d)) == pytest.approx(oracle.hg_sample_mu(g, u1), abs=2e-6)


# ---------------------------------------------------------------- camera
def test_camera_ray_closed_form():
    cam = dict(pos=[0.1, 0.2, -2.0], look_at=[0.4, 0.6, 0.5], up=[0, 1, 0], fov_y_deg=50.0, width=40, height=30)
    f = np.array(cam["look_at"]) - np.array(cam["pos"])
    f /= np.linalg.norm(f)
    r = np.cross(f, cam["up"])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    ty = math.tan(math.radians(25.0))
    tx = ty * 40 / 30
    for px, py, u0, u1 in [(0, 0, 0.0, 0.0), (39, 29, 1.0, 1.0), (20, 15, 0.0, 0.0), (7, 11, 0.25, 0.75)]:
        o, d = oracle.camera_ray(cam, px, py, u0, u1)
        sx = (2 * (px + u0) / 40 - 1) * tx
        sy = (1 - 2 * (py + u1) / 30) * ty
        e = f + sx * r + sy * u
        e /= np.linalg.norm(e)
        assert np.allclose(d, e, atol=2e-7)
        assert np.allclose(o, cam["pos"])


# ---------------------------------------------------------------- transport
def test_homogeneous_transmittance():
    """Pure absorber (albedo 0), environment 1: the pixel is the probability
    of crossing the unit cube without a collision, exp(-sigma L), L = 1."""
    for sigma in [0.5, 2.0]:
        g = homogeneous_grid(sigma)
        img, st = g.render(PENCIL, dict(albedo=0.0, g=0.0), NOSUN, spp=40000, seed=5, render=dict(max_bounces=1))
        p = math.exp(-sigma)
        sd = math.sqrt(p * (1 - p) / 40000)
        assert abs(float(img[0, 0, 0]) - p) < 5 * sd


def test_white_furnace_is_exact():
    """Albedo 1, environment 1, no sun: every path returns exactly 1 whatever
    the medium, so every pixel is exactly 1."""
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]()
    g = oracle.leb_build(d, 64, sc["camera"], dict(sc["build"], uniform_depth=8))
    cam = dict(sc["camera"], width=16, height=16)
    img, st = g.render(cam, dict(albedo=1.0, g=0.4), NOSUN, spp=4, seed=1, render=dict(max_bounces=1 << 30))
    assert st["real_collisions"] > 500 and st["truncated"] == 0
    assert (img == 1.0).all()


def _dist_to_boundary(x, w):
    t = np.inf
    for a in range(3):
        if w[a] > 0:
            t = min(t, (1 - x[a]) / w[a])
        elif w[a] < 0:
            t = min(t, -x[a] / w[a])
    return t


def test_single_scattering_against_quadrature():
    """max_bounces = 1, homogeneous cube: the expected pixel is the 1-D
    integral of sigma e^{-sigma s} albedo p_HG(mu) E e^{-sigma l_sun(s)}."""
    sigma, albedo, gg = 2.0, 0.8, 0.5
    w = np.array([0.3, 0.8, -0.5])
    w /= np.linalg.norm(w)
    light = dict(sun_dir=w.tolist(), sun_irradiance=[1.0, 1.0, 1.0], env_radiance=[0.0, 0.0, 0.0])
    g = homogeneous_grid(sigma)
    mu = float(np.float32(w[2]))
    ph = oracle.hg_eval(gg, mu)

    def f(s):
        x = np.array([0.5, 0.5, s])
        return sigma * math.exp(-sigma * s) * albedo * ph * math.exp(-sigma * _dist_to_boundary(x, w))

    expect = integrate.quad(f, 0, 1, limit=200)[0]
    vals = []
    for seed in range(16):
        img, _ = g.render(PENCIL, dict(albedo=albedo, g=gg), light, spp=4000, seed=100 + seed,
                          render=dict(max_bounces=1))
        vals.append(float(img[0, 0, 0]))
    vals = np.array(vals)
    assert abs(vals.mean() - expect) < 5 * vals.std(ddof=1) / math.sqrt(len(vals)) + 1e-6


def _image_means(render_fn, seeds):
    return np.array([float(render_fn(s).mean()) for s in seeds])


def test_transmittance_estimators_and_majorants_agree():
    """Analytic, ratio-tracking and delta-tracking light transmittance, and
    free flights against tight or loose majorants (null collisions), all
    estimate the same image."""
    sc = synthetic.scene("blobs_adaptive")
    d = sc["density_fn"]()
    cam = dict(sc["camera"], width=12, height=10)
    res = {}
    for maj in [0, 1]:
        g = oracle.leb_build(d, 32, sc["camera"], dict(sc["build"], majorant_mode=maj, variation_tau=0.6))
        for mode in ([0, 1, 2] if maj == 1 else [0]):
            fn = lambda s: g.render(cam, sc["medium"], sc["light"], spp=64, seed=s,
                                    render=dict(max_bounces=6, transmittance=mode))[0]
            res[(maj, mode)] = _image_means(fn, range(12))
    ref = res[(0, 0)]
    for k, v in res.items():
        se = math.sqrt(ref.var(ddof=1) / len(ref) + v.var(ddof=1) / len(v))
        assert abs(v.mean() - ref.mean()) < 5 * se + 1e-7, k


def test_tets_of_voxels_match_dda():
    """At uniform depth 3 log2(n) every tet is a Kuhn tet of one voxel, so its
    extinction is that voxel's exactly and the tet tracer and the voxel (DDA)
    tracer estimate the same image."""
    n = 8
    d = synthetic.blobs(4, n)
    cam = dict(pos=[0.3, 0.6, -1.5], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=40.0, width=10, height=10)
    g = oracle.leb_build(d, n, cam, dict(want_mode=1, uniform_depth=9, max_depth=9, max_tets=1 << 20))
    e = g.export()
    c = e["verts"].astype(np.int64).sum(1) // 4  # centroid (floor), never on a voxel face
    vox = c // (S // n)
    assert np.array_equal(e["sigma"], d[vox[:, 0] + n * (vox[:, 1] + n * vox[:, 2])])
    med = dict(albedo=0.9, g=0.3)
    light = synthetic.LIGHT_DEFAULT
    tet = _image_means(lambda s: g.render(cam, med, light, 64, s, dict(max_bounces=8))[0], range(10))
    dda = _image_means(lambda s: oracle.dda_render(d, n, 1.0, cam, med, light, 64, s, dict(max_bounces=8))[0],
                       range(10))
    se = math.sqrt(tet.var(ddof=1) / 10 + dda.var(ddof=1) / 10)
    assert abs(tet.mean() - dda.mean()) < 5 * se


def test_walk_visits_the_tets_the_segment_crosses():
    """Walk vs brute force: the midpoint of every segment piece lies in the
    tet the walk reports for it."""
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]()
    g = oracle.leb_build(d, 64, sc["camera"], dict(sc["build"], want_mode=2, max_depth=12, rand_seed=8,
                                                   rand_thresh=40000))
    e = g.export()
    V = e["verts"].astype(np.float64) / S
    T = np.stack([V[:, 1] - V[:, 0], V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]], axis=2)
    Tinv = np.linalg.inv(T)
    rng = np.random.default_rng(2)
    pieces = 0
    for _ in range(20):
        o = rng.uniform(0.1, 0.9, 3).astype(np.float32)
        dd = rng.normal(size=3)
        dd = (dd / np.linalg.norm(dd)).astype(np.float32)
        start = int(g.locate(o[None])[0])
        tets, faces, tex = g.walk(o, dd, start)
        assert faces[-1] >= 0 and len(tets) < 100000
        t0 = 0.0
        for t, te in zip(tets, tex):
            if te - t0 > 1e-5:
                m = o.astype(np.float64) + 0.5 * (t0 + te) * dd
                lam = Tinv[t] @ (m - V[t, 0])
                assert lam.min() > -1e-6 and lam.sum() < 1 + 1e-6
                pieces += 1
            t0 = te
        # the walk ends on the cube boundary
        end = o.astype(np.float64) + tex[-1] * dd
        assert np.isclose(end, 0, atol=1e-5).any() or np.isclose(end, 1, atol=1e-5).any()
    assert pieces > 200


def test_cost_linear_in_spp_and_sample_offset():
    """Cost scales linearly with the number of samples (paper, Results);
    samples [0,a) + [a,b) equal samples [0,b)."""
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]()
    g = oracle.leb_build(d, 64, sc["camera"], sc["build"])
    cam = dict(sc["camera"], width=16, height=16)
    a, sa = g.render(cam, sc["medium"], sc["light"], 8, 3, dict(max_bounces=8))
    b, sb = g.render(cam, sc["medium"], sc["light"], 8, 3, dict(max_bounces=8, sample_offset=8))
    c, sc_ = g.render(cam, sc["medium"], sc["light"], 16, 3, dict(max_bounces=8))
    assert np.allclose((a + b) / 2, c, rtol=1e-6, atol=1e-7)
    assert sa["tet_steps"] + sb["tet_steps"] == sc_["tet_steps"]
    assert 1.7 < sc_["tet_steps"] / sa["tet_steps"] < 2.3


def test_render_argument_errors():
    g = homogeneous_grid(1.0, depth=3)
    with pytest.raises(oracle.OracleError):
        g.render(PENCIL, dict(albedo=0.5, g=1.0), NOSUN, 1, 0)
    with pytest.raises(oracle.OracleError):
        g.render(PENCIL, dict(albedo=0.5, g=0.0), NOSUN, 0, 0)
    with pytest.raises(oracle.OracleError):
        g.render(PENCIL, dict(albedo=0.5, g=0.0), NOSUN, 1, 0, pixels=np.array([5], np.int32))
