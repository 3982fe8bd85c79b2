"""GPU parity of the density models inside a tet (linear between trilinear
vertex samples; voxel lookup against the tet's box maximum) against the
oracle: per-tet majorants and coefficients bit-exact, images within the
pixel bar for every light estimator and both record layouts, the exact
reduction to the plain tracer for a constant volume, the benchmark frame on
a strided pixel subset, and the argument errors."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from parity import assert_image_parity

pytestmark = pytest.mark.gpu


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


def both(tv, name, model, scale):
    import torch
    sc = synthetic.scene(name)
    d = sc["density_fn"]()
    n = sc["n"]
    g = tv.leb_build(torch.from_numpy(d).cuda(), n, sc["camera"], build=sc["build"])
    o = oracle.leb_build(d, n, sc["camera"], sc["build"])
    g.set_density_model(model, torch.from_numpy(d).cuda(), n, scale)
    o.set_density_model(model, d, n, scale)
    return sc, d, g, o


@pytest.mark.parametrize("name", ["tiny", "blobs_adaptive"])
@pytest.mark.parametrize("model", [1, 2])
def test_model_values_bitexact(tv, name, model):
    say(f"case density model {model} {name}: per-tet values")
    _, _, g, o = both(tv, name, model, 1.25)
    a, b = g.export_density_model(), o.export_density_model()
    assert np.array_equal(a["majorant"].view(np.uint32), b["majorant"].view(np.uint32))
    if model == 1:
        assert np.array_equal(a["coef"].view(np.uint32), b["coef"].view(np.uint32))
    else:
        assert a["coef"] is None


@pytest.mark.parametrize("name,model,trans,layout", [
    ("tiny", 1, 0, 32), ("tiny", 1, 1, 48), ("tiny", 1, 2, 32), ("tiny", 2, 1, 32), ("tiny", 2, 2, 48),
    ("blobs_adaptive", 1, 0, 0), ("blobs_adaptive", 2, 2, 0)])
def test_model_render_parity(tv, name, model, trans, layout):
    say(f"case density model {model} {name}: render, transmittance {trans}, layout {layout}")
    import torch
    sc, _, g, o = both(tv, name, model, 1.0)
    r = dict(sc["render"], transmittance=trans, record_layout=layout)
    img, st = tv.render(g, sc["camera"], sc["medium"], sc["light"], 16, 777, r)
    torch.cuda.synchronize()
    ref, rst = o.render(sc["camera"], sc["medium"], sc["light"], 16, 777, r, threads=8)
    assert_image_parity(img.cpu().numpy(), ref, f"model {model} {name}")
    assert st["null_collisions"] > 0 and rst["null_collisions"] > 0
    rel = abs(st["null_collisions"] - rst["null_collisions"]) / rst["null_collisions"]
    assert rel < 1e-3, (st, rst)


@pytest.mark.parametrize("model,trans", [(1, 0), (2, 2)])
def test_constant_volume_is_the_plain_tracer(tv, model, trans):
    say(f"case density model {model}: constant volume = plain tracer")
    import torch
    n = 16
    d = np.full(n ** 3, 1.5, np.float32)
    sc = synthetic.scene("tiny")
    b = dict(sc["build"], uniform_depth=6, max_depth=6, density_scale=2.0)
    g = tv.leb_build(torch.from_numpy(d).cuda(), n, sc["camera"], build=b)
    # the lanes' own light walks on both sides (the model's renders never
    # queue light rays), so the pixels are written once, bit for bit
    r = dict(sc["render"], transmittance=trans, max_steps_per_path=1 << 20)
    a, sa = tv.render(g, sc["camera"], sc["medium"], sc["light"], 8, 5, r)
    a = a.clone()
    g.set_density_model(model, d, n, 2.0)
    m, sm = tv.render(g, sc["camera"], sc["medium"], sc["light"], 8, 5, r)
    torch.cuda.synchronize()
    assert torch.equal(a, m)
    assert sm["null_collisions"] == 0 and sm["tet_steps"] == sa["tet_steps"]


@pytest.fixture(scope="module")
def cloud_grids(tv):
    import torch
    sc = synthetic.scene("cloud")
    d = sc["density_fn"]()
    say("case density model cloud: gpu build")
    g = tv.leb_build(torch.from_numpy(d).cuda(), 256, sc["camera"], build=sc["build"])
    say("case density model cloud: oracle build", g.info())
    o = oracle.leb_build(d, 256, sc["camera"], sc["build"])
    return sc, d, g, o


@pytest.mark.timeout(900)
@pytest.mark.parametrize("model,trans", [(1, 0), (2, 1)])
def test_cloud_full_size(tv, cloud_grids, model, trans):
    """The benchmark frame (256^3 cloud, 7 M tets, 1024^2, 32 spp, 32
    bounces) with each model: per-tet values bit-exact, image on a strided
    pixel subset the oracle renders."""
    import torch
    sc, d, g, o = cloud_grids
    scale = sc["build"]["density_scale"]
    g.set_density_model(model, torch.from_numpy(d).cuda(), 256, scale)
    o.set_density_model(model, d, 256, scale)
    a, b = g.export_density_model(), o.export_density_model()
    assert np.array_equal(a["majorant"].view(np.uint32), b["majorant"].view(np.uint32))
    if model == 1:
        assert np.array_equal(a["coef"].view(np.uint32), b["coef"].view(np.uint32))
    r = dict(sc["render"], transmittance=trans)
    say(f"case density model {model} cloud: gpu render")
    img, st = tv.render(g, sc["camera"], sc["medium"], sc["light"], 32, 2025, r)
    img = img.cpu().numpy().reshape(-1, 3)
    say(f"case density model {model} cloud: oracle subset", st)
    pix = np.arange(0, 1024 * 1024, 61, dtype=np.int32)  # 17,190 pixels
    ref, rst = o.render(sc["camera"], sc["medium"], sc["light"], 32, 2025, r, pixels=pix, threads=8)
    assert_image_parity(img[pix], ref, f"cloud model {model} subset")


def test_model_errors(tv):
    say("case density model: errors")
    import torch
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]()
    g = tv.leb_build(torch.from_numpy(d).cuda(), sc["n"], sc["camera"], build=sc["build"])
    with pytest.raises(tv.TetError) as e:  # no model yet
        g.export_density_model()
    assert e.value.status == -1
    with pytest.raises(tv.TetError) as e:
        g.set_density_model(3, d, sc["n"], 1.0)
    assert e.value.status == -1
    g.set_density_model(2, d, sc["n"], 1.0)
    before = g.export_density_model()["majorant"].copy()
    bad = d.copy()
    bad[100] = -0.5
    with pytest.raises(tv.TetError) as e:
        g.set_density_model(1, bad, sc["n"], 1.0)
    assert e.value.status == -5
    assert np.array_equal(g.export_density_model()["majorant"], before)  # unchanged
    r = dict(sc["render"], transmittance=0)
    with pytest.raises(tv.TetError) as e:  # voxel lookups: no analytic light transmittance
        tv.render(g, sc["camera"], sc["medium"], sc["light"], 1, 1, r)
    assert e.value.status == -1
    with pytest.raises(tv.TetError) as e:  # in batches too
        tv.render_batch([g], [sc["camera"]], [sc["medium"]], [sc["light"]], [1], [1], r)
    assert e.value.status == -1
    g.set_density_model(0)
    with pytest.raises(tv.TetError):
        g.export_density_model()
    tv.render(g, sc["camera"], sc["medium"], sc["light"], 1, 1, r)  # the plain tracer again


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_model_values_random_volumes(tv, seed):
    """Random volumes (zeros, exact ties, a constant block) on uniform and
    adaptive grids: majorants and coefficients bit-exact for both models."""
    say(f"case density model random volume seed {seed}")
    import torch
    rng = np.random.default_rng(300 + seed)
    n = [8, 16, 32][seed]
    d = np.round(rng.uniform(0.0, 6.0, n ** 3), 1).astype(np.float32)
    d[rng.random(n ** 3) < 0.3] = 0.0
    d.reshape(n, n, n)[: n // 2, : n // 2, : n // 2] = 2.5
    sc = synthetic.scene("blobs_adaptive")
    b = dict(sc["build"], max_depth=[9, 12, 14][seed], variation_tau=0.2)
    if seed == 0:
        b = dict(b, want_mode=1, uniform_depth=9, max_depth=9)
    g = tv.leb_build(torch.from_numpy(d).cuda(), n, sc["camera"], build=b)
    o = oracle.leb_build(d, n, sc["camera"], b)
    for model in (1, 2):
        scale = [0.5, 1.75, 3.0][seed]
        g.set_density_model(model, d, n, scale)
        o.set_density_model(model, d, n, scale)
        a, r = g.export_density_model(), o.export_density_model()
        assert np.array_equal(a["majorant"].view(np.uint32), r["majorant"].view(np.uint32)), model
        if model == 1:
            assert np.array_equal(a["coef"].view(np.uint32), r["coef"].view(np.uint32))
