"""Pins of the oracle's radiance-cache transport (an addition of this
project, not in the paper): training records of untruncated paths and the
render truncated at a vertex where the cache's estimate stands in for the
rest of the path.  No GPU."""
import numpy as np
import pytest
from scipy import stats

import oracle
import synthetic

NP = oracle.N_PARAMS
FURNACE = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[0.0, 0.0, 0.0], env_radiance=[1.0, 1.0, 1.0])


@pytest.fixture(scope="module")
def tiny():
    sc = synthetic.scene("tiny")
    g = oracle.leb_build(sc["density_fn"](), 64, sc["camera"], sc["build"])
    cam = dict(sc["camera"], width=24, height=20)
    return sc, g, cam


def constant_cache(c):
    """Every weight zero, output bias c: the network returns c exactly."""
    P = np.zeros(NP)
    P[-3:] = c
    return P


def rand_params(seed):
    return np.random.default_rng(seed).normal(0, 0.2, NP)


def test_train_pixel_is_uniform():
    npix = 37 * 23
    pix = np.array([oracle.train_pixel(5, j, npix) for j in range(40000)])
    assert pix.min() >= 0 and pix.max() < npix
    counts = np.bincount(pix, minlength=npix)
    assert stats.chisquare(counts).pvalue > 1e-4


def test_furnace_targets_are_exact(tiny):
    """Albedo 1/2, environment 1, no sun: the path's radiance is 2^-K after
    K real vertices and the throughput reaching vertex k is 2^-(k-1), so
    the target at vertex k is exactly 2^-(K-k+1)."""
    sc, g, cam = tiny
    r = g.nrc_collect(cam, dict(albedo=0.5, g=0.3), FURNACE, frame_seed=3, n_paths=3000, max_vertices=8,
                      render=dict(max_bounces=1 << 20))
    assert len(r["tag"]) > 1000
    j, k = r["tag"] // 16, r["tag"] % 16 + 1
    nv = np.bincount(j, minlength=3000)
    full = nv[j] < 8  # the path's last vertex is recorded: K = its count
    K = nv[j]
    assert full.sum() > 500
    expect = 2.0 ** -(K - k + 1)
    assert np.array_equal(r["target"][full], np.repeat(expect[full, None], 3, 1).astype(np.float32))
    assert np.array_equal(r["path_L"][nv == 0], np.ones(((nv == 0).sum(), 3), np.float32))


def test_records_follow_plain_paths(tiny):
    """A training path's radiance is the plain estimator's sample `j` of its
    pixel, and its first record sits on that path (the camera ray's first
    real collision, in the cell holding it)."""
    sc, g, cam = tiny
    r = g.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=9, n_paths=300, max_vertices=4,
                      render=dict(max_bounces=8))
    for j in range(0, 300, 7):
        img, _ = g.render(cam, sc["medium"], sc["light"], 1, 9, dict(max_bounces=8, sample_offset=j),
                          pixels=np.array([r["path_pixel"][j]]))
        assert np.array_equal(img[0], r["path_L"][j])
    first = r["tag"] % 16 == 0
    sig = g.export()["sigma"]
    cells = g.locate(r["pos"][first])
    ok = cells >= 0
    assert ok.mean() > 0.95
    assert np.array_equal(sig[cells[ok]], r["sigma"][first][ok])
    # records of vertex 1: target = path radiance (throughput 1, nothing gathered before)
    j1 = r["tag"][first] // 16
    assert np.array_equal(r["target"][first], r["path_L"][j1])


def test_truncation_beyond_max_bounces_is_the_plain_render(tiny):
    sc, g, cam = tiny
    ro = dict(max_bounces=3)
    a, _ = g.render(cam, sc["medium"], sc["light"], 4, 2, ro)
    b, _ = g.nrc_render(cam, sc["medium"], sc["light"], 4, 2, rand_params(1), ro, truncate_bounce=4)
    assert np.array_equal(a, b)


def test_zero_cache_without_environment_is_single_scattering(tiny):
    """No environment light: with a cache that returns 0 the render
    truncated at vertex 2 keeps only the light estimate of vertex 1, which is
    the plain render with one bounce (bit for bit)."""
    sc, g, cam = tiny
    light = dict(sc["light"], env_radiance=[0.0, 0.0, 0.0])
    a, _ = g.render(cam, sc["medium"], light, 4, 5, dict(max_bounces=1))
    b, st = g.nrc_render(cam, sc["medium"], light, 4, 5, constant_cache(0.0), dict(max_bounces=32),
                         truncate_bounce=2)
    assert a.max() > 0 and np.array_equal(a, b)


@pytest.mark.parametrize("bf16", [False, True])
def test_exact_cache_in_the_furnace(tiny, bf16):
    """Albedo 1, environment 1, no sun: the radiance leaving any vertex per
    unit throughput is exactly 1, so a cache returning 1 makes every pixel
    exactly 1."""
    sc, g, cam = tiny
    img, st = g.nrc_render(cam, dict(albedo=1.0, g=0.5), FURNACE, 4, 7, constant_cache(1.0),
                           dict(max_bounces=1 << 20), truncate_bounce=2, bf16=bf16)
    assert st["real_collisions"] > 200
    assert (img == 1.0).all()


def test_cache_estimate_is_the_clamped_network(tiny):
    P = rand_params(3)
    rng = np.random.default_rng(4)
    for _ in range(5):
        p, d = rng.random(3).astype(np.float32), rng.normal(size=3).astype(np.float32)
        s = np.float32(rng.random() * 10)
        y = oracle.mlp_forward(P, oracle.nrc_encode(p[None], d[None], [s], 10.0), bf16=True)[0]
        assert np.array_equal(oracle.nrc_eval_point(P, p, d, s, 10.0), np.maximum(y.astype(np.float32), 0))


# ---- the cache with extra channels (temperature, albedo, phase parameter per tet)

def channel_grid(sc, n=8, seed=0, temperature=None, albedo=None, g=None):
    """A fresh grid of the tiny scene carrying the given n^3 channels."""
    gr = oracle.leb_build(sc["density_fn"](), 64, sc["camera"], sc["build"])
    gr.set_channels(n, temperature=temperature, albedo=albedo, g=g)
    return gr


def random_channels(n, seed):
    rng = np.random.default_rng(seed)
    return dict(temperature=rng.uniform(0.0, 3.0, n ** 3).astype(np.float32),
                albedo=rng.uniform(0.3, 1.0, n ** 3).astype(np.float32),
                g=rng.uniform(-0.7, 0.8, n ** 3).astype(np.float32))


def test_constant_channels_with_cache_are_the_plain_cache_path(tiny):
    """Constant albedo and g channels and zero temperature: training records
    and the truncated render are those of the medium with these values, bit
    for bit (the channels replace the medium's values and add nothing)."""
    sc, _, cam = tiny
    n = 8
    g = channel_grid(sc, n, temperature=np.zeros(n ** 3, np.float32), albedo=np.full(n ** 3, 0.8, np.float32),
                     g=np.full(n ** 3, -0.4, np.float32))
    med = dict(albedo=0.8, g=-0.4)
    ch = dict(max_bounces=8, channels=1, emission=[1.5, 1.0, 0.5])
    a = g.nrc_collect(cam, med, sc["light"], frame_seed=4, n_paths=500, max_vertices=4, render=dict(max_bounces=8))
    b = g.nrc_collect(cam, dict(albedo=0.2, g=0.6), sc["light"], frame_seed=4, n_paths=500, max_vertices=4,
                      render=ch)
    assert len(a["tag"]) > 200
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    P = rand_params(6)
    x, _ = g.nrc_render(cam, med, sc["light"], 4, 3, P, dict(max_bounces=8), truncate_bounce=2)
    y, _ = g.nrc_render(cam, dict(albedo=0.2, g=0.6), sc["light"], 4, 3, P, ch, truncate_bounce=2)
    assert x.max() > 0 and np.array_equal(x, y)


def test_emitting_furnace_targets_are_exact(tiny):
    """Albedo channel 1/2, temperature 1, emission 1, no other light: each
    real vertex k emits 2^-k (its throughput 2^-(k-1) times the absorbed
    half), so a path of K vertices has radiance 1 - 2^-K and the target at
    vertex k -- recorded before its own emission -- is exactly
    1 - 2^-(K-k+1)."""
    sc, _, cam = tiny
    n = 4
    g = channel_grid(sc, n, temperature=np.ones(n ** 3, np.float32), albedo=np.full(n ** 3, 0.5, np.float32))
    dark = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[0.0, 0.0, 0.0], env_radiance=[0.0, 0.0, 0.0])
    r = g.nrc_collect(cam, dict(albedo=0.9, g=0.3), dark, frame_seed=3, n_paths=3000, max_vertices=8,
                      render=dict(max_bounces=1 << 20, channels=1, emission=[1.0, 1.0, 1.0]))
    j, k = r["tag"] // 16, r["tag"] % 16 + 1
    nv = np.bincount(j, minlength=3000)
    full = nv[j] < 8
    K = nv[j]
    assert full.sum() > 500
    expect = 1.0 - 2.0 ** -(K - k + 1)
    assert np.array_equal(r["target"][full], np.repeat(expect[full, None], 3, 1).astype(np.float32))
    done = (nv > 0) & (nv < 8)
    assert np.array_equal(r["path_L"][done], np.repeat((1.0 - 2.0 ** -nv[done])[:, None], 3, 1).astype(np.float32))
    assert (r["path_L"][nv == 0] == 0).all()


def test_cache_stands_for_the_vertex_emission(tiny):
    """Same emitting furnace, one sample per pixel, a cache returning 1/4
    and truncation at vertex 2: a sample scores 0 (no vertex), 1/2 (vertex
    1's emission, no vertex 2) or 1/2 + 1/4 x 1/2 (vertex 2's throughput
    times the cache, without vertex 2's own emission)."""
    sc, _, cam = tiny
    n = 4
    g = channel_grid(sc, n, temperature=np.ones(n ** 3, np.float32), albedo=np.full(n ** 3, 0.5, np.float32))
    dark = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[0.0, 0.0, 0.0], env_radiance=[0.0, 0.0, 0.0])
    img, st = g.nrc_render(cam, dict(albedo=0.9, g=0.3), dark, 1, 8, constant_cache(0.25),
                           dict(max_bounces=1 << 20, channels=1, emission=[1.0, 1.0, 1.0]), truncate_bounce=2)
    v = img.reshape(-1, 3)
    assert (v == v[:, :1]).all()
    vals, counts = np.unique(v[:, 0], return_counts=True)
    assert set(vals.tolist()) == {0.0, 0.5, 0.625}, vals
    assert counts.min() >= 20


def test_records_and_truncation_with_varying_channels(tiny):
    """Channels that vary per tet: a training path's radiance is the plain
    channel estimator's sample j of its pixel, its first target that
    radiance, and truncation past the last bounce is the plain channel
    render."""
    sc, _, cam = tiny
    n = 8
    g = channel_grid(sc, n, **random_channels(n, 9))
    ro = dict(max_bounces=6, channels=1, emission=[0.6, 0.3, 0.1])
    r = g.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=13, n_paths=300, max_vertices=4, render=ro)
    for j in range(0, 300, 11):
        img, _ = g.render(cam, sc["medium"], sc["light"], 1, 13, dict(ro, sample_offset=j),
                          pixels=np.array([r["path_pixel"][j]]))
        assert np.array_equal(img[0], r["path_L"][j])
    first = r["tag"] % 16 == 0
    assert np.array_equal(r["target"][first], r["path_L"][r["tag"][first] // 16])
    a, _ = g.render(cam, sc["medium"], sc["light"], 4, 2, dict(ro, max_bounces=3))
    b, _ = g.nrc_render(cam, sc["medium"], sc["light"], 4, 2, rand_params(1), dict(ro, max_bounces=3),
                        truncate_bounce=4)
    assert a.max() > 0 and np.array_equal(a, b)
    # channels asked of a grid without them
    _, plain, _ = tiny
    with pytest.raises(oracle.OracleError):
        plain.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=1, n_paths=10, max_vertices=2, render=ro)


# ---- the cache on grids with a density model inside the tets

def test_model_records_carry_the_point_extinction(tiny):
    """On a grid with a density model the cache's extinction input at a
    vertex is the model's at the vertex: for voxel lookups the density
    scale times the voxel floor(x n) holding the record's point (a value
    read straight from the volume), for the linear model the tet's plane at
    the point."""
    sc, _, cam = tiny
    d = sc["density_fn"]()
    n = 64
    g = oracle.leb_build(d, n, sc["camera"], sc["build"])
    scale = 1.75
    g.set_density_model(2, d, n, scale)
    r = g.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=5, n_paths=800, max_vertices=4,
                      render=dict(max_bounces=8, transmittance=2))
    assert len(r["tag"]) > 300
    idx = np.clip(np.floor(r["pos"] * np.float32(n)).astype(np.int64), 0, n - 1)
    vox = d[idx[:, 0] + n * (idx[:, 1] + n * idx[:, 2])]
    assert np.array_equal(r["sigma"], (np.float32(scale) * vox).astype(np.float32))
    # the cell's own value is another number: the records do not carry it
    cells = g.locate(r["pos"])
    assert (r["sigma"] != g.export()["sigma"][cells]).mean() > 0.5

    g.set_density_model(1, d, n, scale)
    r = g.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=5, n_paths=800, max_vertices=4,
                      render=dict(max_bounces=8))
    coef = g.export_density_model()["coef"]
    cells = g.locate(r["pos"])
    ok = cells >= 0
    c = coef[cells[ok]]
    p = r["pos"][ok]
    plane = ((c[:, 0] + c[:, 1] * p[:, 0]) + c[:, 2] * p[:, 1]) + c[:, 3] * p[:, 2]
    assert ok.mean() > 0.99 and (plane == r["sigma"][ok]).mean() > 0.99


def test_uniform_linear_model_with_cache_is_the_plain_grid(tiny):
    """A uniform volume: the linear model is the constant, its majorant the
    tet's value, so the model grid's records and truncated render equal the
    plain grid's bit for bit."""
    sc, _, cam = tiny
    n = 16
    d = np.full(n ** 3, 6.0, np.float32)
    b = dict(want_mode=1, uniform_depth=9, max_depth=9, density_scale=1.0, max_tets=1 << 20)
    plain = oracle.leb_build(d, n, sc["camera"], b)
    mod = oracle.leb_build(d, n, sc["camera"], b)
    mod.set_density_model(1, d, n, 1.0)
    ro = dict(max_bounces=8)
    a = plain.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=2, n_paths=400, max_vertices=4, render=ro)
    m = mod.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=2, n_paths=400, max_vertices=4, render=ro)
    assert len(a["tag"]) > 200
    for k in a:
        assert np.array_equal(a[k], m[k]), k
    P = rand_params(8)
    x, _ = plain.nrc_render(cam, sc["medium"], sc["light"], 4, 6, P, ro, truncate_bounce=2)
    y, _ = mod.nrc_render(cam, sc["medium"], sc["light"], 4, 6, P, ro, truncate_bounce=2)
    assert x.max() > 0 and np.array_equal(x, y)


def test_model_truncation_beyond_max_bounces_is_the_plain_model_render(tiny):
    sc, _, cam = tiny
    d = sc["density_fn"]()
    g = oracle.leb_build(d, 64, sc["camera"], sc["build"])
    g.set_density_model(2, d, 64, 1.0)
    ro = dict(max_bounces=3, transmittance=1)
    a, _ = g.render(cam, sc["medium"], sc["light"], 4, 2, ro)
    b, _ = g.nrc_render(cam, sc["medium"], sc["light"], 4, 2, rand_params(2), ro, truncate_bounce=4)
    assert a.max() > 0 and np.array_equal(a, b)
    with pytest.raises(oracle.OracleError):  # voxel lookups: no analytic light transmittance
        g.nrc_collect(cam, sc["medium"], sc["light"], frame_seed=1, n_paths=10, max_vertices=2,
                      render=dict(max_bounces=3, transmittance=0))
