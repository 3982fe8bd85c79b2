"""GPU parity of the extra per-tet channels (temperature -> emission, per-tet
albedo and phase parameter g) against the oracle: per-tet values bit-exact,
images within the pixel bar, the constant-channel reduction exact, and the
argument errors."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from parity import assert_image_parity

pytestmark = pytest.mark.gpu

EMISSION = [1.5, 0.9, 0.4]


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


def both_grids(tv, name, ch_n, ch_seed):
    import torch
    sc = synthetic.scene(name)
    d = sc["density_fn"]()
    g = tv.leb_build(torch.from_numpy(d).cuda(), sc["n"], sc["camera"], build=sc["build"])
    o = oracle.leb_build(d, sc["n"], sc["camera"], sc["build"])
    ch = synthetic.channels(ch_seed, ch_n)
    g.set_channels(ch_n, **ch)
    o.set_channels(ch_n, **ch)
    return sc, g, o


@pytest.mark.parametrize("name,ch_n", [("tiny", 32), ("blobs_adaptive", 64)])
def test_channel_values_bitexact(tv, name, ch_n):
    say(f"case channels {name}: per-tet values, {ch_n}^3 channel grids")
    sc, g, o = both_grids(tv, name, ch_n, 11)
    a, b = g.export_channels(), o.export_channels()
    for k in ("temperature", "albedo", "g"):
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k


@pytest.mark.parametrize("name,layout", [("tiny", 32), ("tiny", 48), ("blobs_adaptive", 0)])
def test_channels_render_parity(tv, name, layout):
    say(f"case channels {name}: render, {layout}-byte records")
    import torch
    sc, g, o = both_grids(tv, name, 32, 21)
    r = dict(sc["render"], channels=1, emission=EMISSION, record_layout=layout)
    cam = sc["camera"]
    spp = 16
    img, st = tv.render(g, cam, sc["medium"], sc["light"], spp, 4321, r)
    torch.cuda.synchronize()
    ref, rst = o.render(cam, sc["medium"], sc["light"], spp, 4321, r, threads=8)
    assert_image_parity(img.cpu().numpy(), ref, f"channels {name}")
    assert st["real_collisions"] > 0
    # the channels matter: the plain image differs
    plain, _ = tv.render(g, cam, sc["medium"], sc["light"], spp, 4321, dict(sc["render"], record_layout=layout))
    assert not np.allclose(plain.cpu().numpy(), img.cpu().numpy(), rtol=1e-3)


def test_constant_channels_are_the_plain_tracer(tv):
    say("case channels: constant channels = plain tracer")
    import torch
    sc = synthetic.scene("tiny")
    g = tv.leb_build(torch.from_numpy(sc["density_fn"]()).cuda(), sc["n"], sc["camera"], build=sc["build"])
    n = 16
    g.set_channels(n, temperature=np.zeros(n ** 3, np.float32), albedo=np.full(n ** 3, 0.55, np.float32),
                   g=np.full(n ** 3, -0.5, np.float32))
    # bit for bit with the lanes' own light walks (pixels written once)...
    own = dict(sc["render"], max_steps_per_path=1 << 20)
    a, _ = tv.render(g, sc["camera"], dict(albedo=0.55, g=-0.5), sc["light"], 8, 99, own)
    b, _ = tv.render(g, sc["camera"], dict(albedo=0.9, g=0.3), sc["light"], 8, 99,
                     dict(own, channels=1, emission=EMISSION))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # ...and with queued light rays, whose terms reach the pixels in any
    # order: the same steps, the image up to FP32 summation order
    a, sa = tv.render(g, sc["camera"], dict(albedo=0.55, g=-0.5), sc["light"], 8, 99, sc["render"])
    b, sb = tv.render(g, sc["camera"], dict(albedo=0.9, g=0.3), sc["light"], 8, 99,
                      dict(sc["render"], channels=1, emission=EMISSION))
    assert sa["tet_steps"] == sb["tet_steps"] and sa["light_rays_queued"] == sb["light_rays_queued"] > 0
    x, y = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
    assert (np.abs(x - y) / np.maximum(np.abs(x), 1e-4 * np.abs(x).mean())).max() <= 1e-5


def test_channel_errors(tv):
    say("case channels: errors")
    import torch
    sc = synthetic.scene("tiny")
    g = tv.leb_build(torch.from_numpy(sc["density_fn"]()).cuda(), sc["n"], sc["camera"], build=sc["build"])
    r = dict(sc["render"], channels=1, emission=EMISSION)
    with pytest.raises(tv.TetError) as e:  # no channels yet
        tv.render(g, sc["camera"], sc["medium"], sc["light"], 1, 1, r)
    assert e.value.status == -1
    n = 8
    good = np.full(n ** 3, 0.5, np.float32)
    g.set_channels(n, albedo=good)
    for k, v in (("albedo", 1.25), ("g", -1.0), ("temperature", float("nan"))):
        bad = good.copy()
        bad[7] = v
        with pytest.raises(tv.TetError) as e:
            g.set_channels(n, **{k: bad})
        assert e.value.status == -5
    # the failed calls left the grid's channels as they were
    assert np.all(g.export_channels()["albedo"] == np.float32(0.5))
    with pytest.raises(tv.TetError):  # negative emission
        tv.render(g, sc["camera"], sc["medium"], sc["light"], 1, 1, dict(r, emission=[1.0, -1.0, 0.0]))
    bare = tv.leb_build(torch.from_numpy(sc["density_fn"]()).cuda(), sc["n"], sc["camera"], build=sc["build"])
    with pytest.raises(tv.TetError) as e:  # a batch whose grids do not all carry channels
        tv.render_batch([g, bare], [sc["camera"]] * 2, [sc["medium"]] * 2, [sc["light"]] * 2, [1, 1], [1, 2], r)
    assert e.value.status == -1


@pytest.mark.timeout(900)
def test_cloud_full_size_channels(tv):
    """The benchmark frame (256^3 cloud, 7 M tets, 1024^2, 32 spp, 32
    bounces) with 256^3 temperature, albedo and g channels: per-tet values
    bit-exact, image on a strided pixel subset the oracle renders."""
    import torch
    sc = synthetic.scene("cloud")
    d = sc["density_fn"]()
    ch = synthetic.channels(7, 256)
    say("case channels cloud: gpu build")
    g = tv.leb_build(torch.from_numpy(d).cuda(), 256, sc["camera"], build=sc["build"])
    g.set_channels(256, **{k: torch.from_numpy(v).cuda() for k, v in ch.items()})
    say("case channels cloud: oracle build", g.info())
    o = oracle.leb_build(d, 256, sc["camera"], sc["build"])
    o.set_channels(256, **ch)
    a, b = g.export_channels(), o.export_channels()
    for k in ("temperature", "albedo", "g"):
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k
    r = dict(sc["render"], channels=1, emission=[0.6, 0.35, 0.15])
    say("case channels cloud: gpu render")
    img, st = tv.render(g, sc["camera"], sc["medium"], sc["light"], 32, 2026, r)
    img = img.cpu().numpy().reshape(-1, 3)
    say("case channels cloud: oracle subset", st)
    pix = np.arange(0, 1024 * 1024, 61, dtype=np.int32)  # 17,190 pixels
    ref, _ = o.render(sc["camera"], sc["medium"], sc["light"], 32, 2026, r, pixels=pix, threads=8)
    assert_image_parity(img[pix], ref, "cloud channels subset")


@pytest.mark.parametrize("seed", [0, 1])
def test_channel_values_random(tv, seed):
    """Random channel grids at resolutions other than the density's (values
    at the range ends, exact ties): per-tet means bit-exact."""
    say(f"case channels random seed {seed}")
    import torch
    rng = np.random.default_rng(500 + seed)
    sc = synthetic.scene(["tiny", "blobs_adaptive"][seed])
    d = sc["density_fn"]()
    g = tv.leb_build(torch.from_numpy(d).cuda(), sc["n"], sc["camera"], build=sc["build"])
    o = oracle.leb_build(d, sc["n"], sc["camera"], sc["build"])
    n = [8, 128][seed]
    t = np.round(rng.uniform(0.0, 10.0, n ** 3), 2).astype(np.float32)
    a = rng.choice(np.array([0.0, 0.25, 1.0], np.float32), n ** 3)
    gg = rng.uniform(-0.99, 0.99, n ** 3).astype(np.float32)
    ch = dict(temperature=t, albedo=a, g=gg)
    g.set_channels(n, **ch)
    o.set_channels(n, **ch)
    x, y = g.export_channels(), o.export_channels()
    for k in ch:
        assert np.array_equal(x[k].view(np.uint32), y[k].view(np.uint32)), k
