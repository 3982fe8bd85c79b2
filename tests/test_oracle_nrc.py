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
