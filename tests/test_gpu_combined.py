"""GPU: the extensions together -- extra channels and density models with
the radiance cache, and both in batches -- through the C ABI against the
oracle on the same seeded inputs.

The cache at a vertex stands for all radiance from the vertex on, its own
emission included (records are taken before it), and its extinction input
there is the density model's at the vertex.  Batches follow the same paths
as single renders, so their images differ from single renders only in the
order FP32 sample values are summed per pixel (relative 1e-5), and their
tet-step counts are equal."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from parity import assert_image_parity, rel_errors

pytestmark = pytest.mark.gpu
NP = oracle.N_PARAMS
EMISSION = [1.2, 0.7, 0.3]
TINY = synthetic.scene("tiny")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tv():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    import paper_2506_11510_amd as tv
    tv.lib()
    return tv


def grids(tv, channels=None, model=0, scale=1.0):
    """GPU and oracle grids of the tiny scene, with channels (n, seed) and a
    density model (on the scene's own volume)."""
    import torch
    d = TINY["density_fn"]()
    g = tv.leb_build(torch.from_numpy(d).cuda(), 64, TINY["camera"], build=TINY["build"])
    o = oracle.leb_build(d, 64, TINY["camera"], TINY["build"])
    if channels:
        ch = synthetic.channels(channels[1], channels[0])
        g.set_channels(channels[0], **ch)
        o.set_channels(channels[0], **ch)
    if model:
        g.set_density_model(model, torch.from_numpy(d).cuda(), 64, scale)
        o.set_density_model(model, d, 64, scale)
    return g, o


def records_match(r, ro, what):
    say(f"  {what}: {len(r['tag'])} records vs {len(ro['tag'])}")
    assert len(r["tag"]) > 1000
    common, ia, ib = np.intersect1d(r["tag"], ro["tag"], return_indices=True)
    assert len(common) >= 0.99 * len(ro["tag"])
    same = np.ones(len(common), bool)
    for k in ("pos", "dir", "sigma", "target"):
        a, b = r[k][ia].reshape(len(common), -1), ro[k][ib].reshape(len(common), -1)
        same &= (a.view(np.uint32) == b.view(np.uint32)).all(axis=1)
    say(f"  {same.mean() * 100:.3f}% of common records bit-exact")
    assert same.mean() >= 0.99
    assert np.array_equal(np.sort(r["tag"]), r["tag"])


def constant_cache(tv, c, truncate=2):
    P = np.zeros(NP, np.float32)
    P[-3:] = c
    n = tv.Nrc(dict(sigma_ref=10.0, truncate_bounce=truncate))
    n.load(P)
    return n, P.astype(np.float64)


# (render options, channels (n, seed), model, scale) of each extension case
CASES = {
    "channels": (dict(channels=1, emission=EMISSION), (16, 3), 0, 1.0),
    "linear model": (dict(), None, 1, 1.3),
    "voxel model": (dict(transmittance=2), None, 2, 0.8),
    "channels + linear model": (dict(channels=1, emission=EMISSION, transmittance=1), (32, 4), 1, 1.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_collect_with_extensions_matches_oracle(tv, case):
    say(f"case cache collect with {case}")
    ro_ext, ch, model, scale = CASES[case]
    g, o = grids(tv, ch, model, scale)
    cam = dict(TINY["camera"], width=48, height=40)
    n = tv.Nrc(dict(train_paths=3000, train_vertices=4, sigma_ref=10.0))
    ro = dict(max_bounces=8, **ro_ext)
    r = n.collect(g, cam, TINY["medium"], TINY["light"], 17, ro)
    ref = o.nrc_collect(cam, TINY["medium"], TINY["light"], 17, 3000, 4, ro, threads=8)
    records_match(r, ref, case)


@pytest.mark.parametrize("case", list(CASES))
def test_truncated_render_with_extensions_matches_oracle(tv, case):
    """A constant cache is exact on both sides: the truncated render meets
    the plain image bar."""
    say(f"case cache render with {case}")
    ro_ext, ch, model, scale = CASES[case]
    g, o = grids(tv, ch, model, scale)
    cam = dict(TINY["camera"], width=40, height=36)
    n, P = constant_cache(tv, [0.4, 0.3, 0.2])
    ro = dict(TINY["render"], max_bounces=8, **ro_ext)
    img, st = tv.render(g, cam, TINY["medium"], TINY["light"], 8, 23, dict(ro, nrc=n))
    ref, _ = o.nrc_render(cam, TINY["medium"], TINY["light"], 8, 23, P, ro, truncate_bounce=2, sigma_ref=10.0,
                          bf16=True, threads=8)
    assert st["cache_queries"] > 0
    assert_image_parity(img.cpu().numpy(), ref, f"cache with {case}")


def test_random_cache_with_channels_and_model(tv):
    """A random network on the channel + model grid: the cache term within
    the BF16 tolerance of the radiance-cache tests, per pixel 2^-6."""
    say("case random cache with channels + linear model")
    ro_ext, ch, model, scale = CASES["channels + linear model"]
    g, o = grids(tv, ch, model, scale)
    cam = dict(TINY["camera"], width=40, height=36)
    rng = np.random.default_rng(31)
    P = np.zeros(NP, np.float32)
    dims = [76, 64, 64, 64, 64, 3]
    off = 0
    for layer in range(5):
        fi, fo = dims[layer], dims[layer + 1]
        P[off:off + fo * fi] = rng.normal(0, 0.5 * np.sqrt(2.0 / fi), fo * fi)
        P[off + fo * fi:off + fo * fi + fo] = rng.normal(0, 0.1, fo)
        off += fo * fi + fo
    n = tv.Nrc(dict(sigma_ref=10.0, truncate_bounce=2))
    n.load(P)
    ro = dict(TINY["render"], max_bounces=8, **ro_ext)
    img, _ = tv.render(g, cam, TINY["medium"], TINY["light"], 8, 24, dict(ro, nrc=n))
    ref, _ = o.nrc_render(cam, TINY["medium"], TINY["light"], 8, 24, P.astype(np.float64), ro, truncate_bounce=2,
                          sigma_ref=10.0, bf16=True, threads=8)
    rel = rel_errors(img.cpu().numpy(), ref)
    say(f"  per-pixel: max {rel.max():.3g}, mean {rel.mean():.3g}, {(rel <= 1e-4).mean() * 100:.2f}% within 1e-4")
    assert rel.max() <= 2 ** -6 and (rel <= 1e-4).mean() >= 0.5


def test_training_inside_the_render_with_channels_and_model(tv):
    """nrc_train on the channel + model grid: the records and weights equal
    those of a separate training frame with the render's training key."""
    say("case cache training inside the render, channels + model")
    ro_ext, ch, model, scale = CASES["channels + linear model"]
    g, _ = grids(tv, ch, model, scale)
    cam = dict(TINY["camera"], width=48, height=40)
    ro = dict(TINY["render"], max_bounces=8, **ro_ext)
    a = tv.Nrc(dict(sigma_ref=10.0, train_paths=4000))
    b = tv.Nrc(dict(sigma_ref=10.0, train_paths=4000))
    P = a.export()
    b.load(P)
    a.load(P)
    seed = 78
    _, st = tv.render(g, cam, TINY["medium"], TINY["light"], 8, seed, dict(ro, nrc=a, nrc_train=1))
    sf = b.train_frame(g, cam, TINY["medium"], TINY["light"], seed ^ 0x6A09E667F3BCC909, ro)
    say(f"  records {st['cache_records']} vs {sf['records']}")
    assert st["cache_records"] == sf["records"] > 1000
    assert st["cache_loss"] == sf["loss"]
    assert np.array_equal(a.export(), b.export())


def sum_order_close(img, ref, what, tol=1e-5):
    a = np.asarray(img, np.float64).reshape(-1, 3)
    b = np.asarray(ref, np.float64).reshape(-1, 3)
    floor = 1e-4 * max(float(np.abs(b).mean()), 1e-30)
    rel = (np.abs(a - b) / np.maximum(np.abs(b), floor)).max()
    say(f"  {what}: worst relative difference {rel:.3g}")
    assert rel <= tol, f"{what}: {rel:.3g}"


@pytest.fixture(scope="module")
def batch_scenes(tv):
    """Scenes on grids with channels (one also with the linear model), and
    scenes on grids with a model or none, for batches with and without the
    channels option."""
    gc, oc = grids(tv, (16, 5))
    gcm, ocm = grids(tv, (32, 6), 1, 1.1)
    gm1, om1 = grids(tv, None, 1, 1.4)
    gm2, om2 = grids(tv, None, 2, 0.9)
    gp, op = grids(tv)
    t = TINY
    cams = [dict(t["camera"], width=40, height=32), dict(t["camera"], pos=[1.6, 0.7, 0.2], width=37, height=23),
            dict(t["camera"], width=1, height=1), dict(t["camera"], pos=[0.5, 1.8, 0.5], up=[0, 0, 1], width=24,
                                                       height=24)]
    media = [t["medium"], dict(albedo=0.7, g=-0.4), dict(albedo=0.95, g=0.6), t["medium"]]
    light2 = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[1.0, 2.0, 3.0], env_radiance=[0.1, 0.1, 0.1])
    lights = [t["light"], light2, t["light"], light2]
    return {
        "channels": dict(grids=[gc, gcm, gc, gcm], ograds=[oc, ocm, oc, ocm], cams=cams, media=media, lights=lights,
                         spp=[8, 5, 3, 6], seeds=[31, 32, 33, 34],
                         ro=dict(max_bounces=8, transmittance=1, channels=1, emission=EMISSION)),
        "models": dict(grids=[gm1, gm2, gp, gm2], ograds=[om1, om2, op, om2], cams=cams, media=media, lights=lights,
                       spp=[8, 5, 3, 6], seeds=[41, 42, 43, 44], ro=dict(max_bounces=8, transmittance=2)),
    }


@pytest.mark.parametrize("kind", ["channels", "models"])
def test_batch_with_extensions_matches_single_renders(tv, batch_scenes, kind):
    say(f"case batch with {kind} vs single renders")
    S = batch_scenes[kind]
    outs, st = tv.render_batch(S["grids"], S["cams"], S["media"], S["lights"], S["spp"], S["seeds"], S["ro"])
    total = 0
    for i in range(len(outs)):
        ref, sti = tv.render(S["grids"][i], S["cams"][i], S["media"][i], S["lights"][i], S["spp"][i], S["seeds"][i],
                             S["ro"])
        total += sti["tet_steps"]
        sum_order_close(outs[i].cpu().numpy(), ref.cpu().numpy(), f"{kind} scene {i}")
    assert st["tet_steps"] == total
    # and two scenes against the oracle
    for i in (0, 1):
        ref, _ = S["ograds"][i].render(S["cams"][i], S["media"][i], S["lights"][i], S["spp"][i], S["seeds"][i],
                                       S["ro"], threads=8)
        assert_image_parity(outs[i].cpu().numpy(), ref, f"{kind} batch scene {i} vs oracle")


@pytest.mark.parametrize("kind", ["channels", "models"])
def test_batch_graph_with_extensions_replays(tv, batch_scenes, kind):
    say(f"case batch graph with {kind}")
    import torch
    S = batch_scenes[kind]
    b = tv.Batch(S["grids"], S["cams"], S["media"], S["lights"], S["spp"], S["ro"])
    for rep, base in enumerate([100, 200, 100]):
        seeds = [base + k for k in range(len(S["grids"]))]
        st = b.render(seeds)
        got = [x.cpu().numpy().copy() for x in b.outs]
        ref, sr = tv.render_batch(S["grids"], S["cams"], S["media"], S["lights"], S["spp"], seeds, S["ro"])
        torch.cuda.synchronize()
        assert st["tet_steps"] == sr["tet_steps"]
        for i in range(len(got)):
            sum_order_close(got[i], ref[i].cpu().numpy(), f"replay {rep} scene {i}")
