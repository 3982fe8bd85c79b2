"""GPU: batched rendering of several scenes in one persistent launch, and
the same batch replayed as a captured HIP graph frame.  A scene's samples
follow the same paths as in a single render (same Philox streams), so the
images differ from single renders only by the order in which FP32 sample
values are summed per pixel: relative 1e-5 at these sample counts.  Every
scene is also checked against the oracle at the image bar."""
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


def sum_order_close(img, ref, what, tol=1e-5):
    a = np.asarray(img, np.float64).reshape(-1, 3)
    b = np.asarray(ref, np.float64).reshape(-1, 3)
    floor = 1e-4 * max(float(np.abs(b).mean()), 1e-30)
    rel = (np.abs(a - b) / np.maximum(np.abs(b), floor)).max()
    say(f"  {what}: worst relative difference {rel:.3g}")
    assert rel <= tol, f"{what}: {rel:.3g}"


@pytest.fixture(scope="module")
def scenes(tv):
    """Six scenes on two grids: varied cameras, ragged sizes, spp, media,
    lights and seeds."""
    import torch
    t = synthetic.scene("tiny")
    a = synthetic.scene("blobs_adaptive")
    da, db = t["density_fn"](), a["density_fn"]()
    g1 = tv.leb_build(torch.from_numpy(da).cuda(), 64, t["camera"], build=t["build"])
    g2 = tv.leb_build(torch.from_numpy(db).cuda(), 32, a["camera"], build=a["build"])
    o1 = oracle.leb_build(da, 64, t["camera"], t["build"])
    o2 = oracle.leb_build(db, 32, a["camera"], a["build"])
    cams = [dict(t["camera"], width=40, height=32),
            dict(t["camera"], pos=[1.6, 0.7, 0.2], width=37, height=23),
            dict(a["camera"]),
            dict(t["camera"], width=1, height=1),
            dict(a["camera"], pos=[-0.5, 0.4, 0.6], width=64, height=48),
            dict(t["camera"], pos=[0.5, 1.8, 0.5], up=[0, 0, 1], width=24, height=24)]
    grids = [g1, g1, g2, g1, g2, g1]
    ograds = [o1, o1, o2, o1, o2, o1]
    media = [t["medium"], dict(albedo=0.7, g=-0.4), a["medium"], t["medium"], dict(albedo=0.95, g=0.6), t["medium"]]
    light2 = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[1.0, 2.0, 3.0], env_radiance=[0.1, 0.1, 0.1])
    lights = [t["light"], light2, a["light"], t["light"], light2, t["light"]]
    spp = [8, 5, 8, 3, 4, 16]
    seeds = [11, 12, 13, 14, 15, 16]
    return dict(grids=grids, ograds=ograds, cams=cams, media=media, lights=lights, spp=spp, seeds=seeds)


RO = dict(max_bounces=8)


def test_batch_matches_single_renders(tv, scenes):
    say("case batch vs single renders")
    S = scenes
    outs, st = tv.render_batch(S["grids"], S["cams"], S["media"], S["lights"], S["spp"], S["seeds"], RO)
    assert st["tet_steps"] > 0
    total = 0
    for i in range(len(outs)):
        ref, sti = tv.render(S["grids"][i], S["cams"][i], S["media"][i], S["lights"][i], S["spp"][i], S["seeds"][i],
                             RO)
        total += sti["tet_steps"]
        sum_order_close(outs[i].cpu().numpy(), ref.cpu().numpy(), f"scene {i}")
    assert st["tet_steps"] == total  # the same paths, step for step


@pytest.mark.parametrize("i", range(6))
def test_batch_matches_oracle(tv, scenes, i):
    say(f"case batch vs oracle, scene {i}")
    S = scenes
    outs, _ = tv.render_batch(S["grids"], S["cams"], S["media"], S["lights"], S["spp"], S["seeds"], RO)
    ref, _ = S["ograds"][i].render(S["cams"][i], S["media"][i], S["lights"][i], S["spp"][i], S["seeds"][i], RO,
                                   threads=8)
    assert_image_parity(outs[i].cpu().numpy(), ref, f"batch scene {i}")


def test_graph_replays_match_eager_batches(tv, scenes):
    """The captured frame, replayed with new seeds and with eager renders
    and synchronisations in between, equals the eager batch every time."""
    say("case batch graph replays")
    import torch
    S = scenes
    b = tv.Batch(S["grids"], S["cams"], S["media"], S["lights"], S["spp"], RO)
    for rep, base in enumerate([100, 200, 100, 300]):
        seeds = [base + k for k in range(len(S["grids"]))]
        st = b.render(seeds)
        got = [o.cpu().numpy().copy() for o in b.outs]
        ref, sr = tv.render_batch(S["grids"], S["cams"], S["media"], S["lights"], S["spp"], seeds, RO)
        torch.cuda.synchronize()
        assert st["tet_steps"] == sr["tet_steps"]
        for i in range(len(got)):
            sum_order_close(got[i], ref[i].cpu().numpy(), f"replay {rep} scene {i}")


def test_c3_batch_is_faster_than_sequential(tv):
    """Sixteen small scenes of the batch generator: one graph frame takes
    less time than the sixteen renders one after another."""
    say("case batch C3 speed")
    import time

    import torch
    sb = synthetic.scene_batch(16)
    grids = [tv.leb_build(torch.from_numpy(s["density_fn"]()).cuda(), s["n"], s["camera"], build=s["build"])
             for s in sb]
    args = ([s["camera"] for s in sb], [s["medium"] for s in sb], [s["light"] for s in sb],
            [s["render"]["spp"] for s in sb])
    ro = dict(max_bounces=16)
    b = tv.Batch(grids, *args, ro)
    seeds = [s["seed"] for s in sb]
    b.render(seeds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.render(seeds)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / 3
    for i, s in enumerate(sb):
        tv.render(grids[i], s["camera"], s["medium"], s["light"], s["render"]["spp"], s["seed"], ro)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        for i, s in enumerate(sb):
            tv.render(grids[i], s["camera"], s["medium"], s["light"], s["render"]["spp"], s["seed"], ro)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / 3
    say(f"  16 scenes: graph frame {t_batch * 1e3:.2f} ms, sequential {t_seq * 1e3:.2f} ms")
    assert t_batch < t_seq


def test_autotune_picks_valid_options_and_caches_them(tv, scenes, tmp_path):
    """The autotuner returns options from its candidate sets, stores them
    under the workload key, returns the stored ones on a second call, and the
    tuned options render the image the defaults render (summation order
    aside)."""
    say("case autotune")
    import json
    S = scenes
    g, cam, med, light = S["grids"][0], dict(S["cams"][0], width=128, height=96), S["media"][0], S["lights"][0]
    path = str(tmp_path / "tune.json")
    opts, ms = tv.autotune(g, cam, med, light, RO, probe_spp=4, cache_path=path)
    say(f"  tuned {opts}, {ms:.3f} ms")
    assert opts["waves_per_simd"] in (4, 5, 6) and opts["event_wait"] in (16, 32, 48)
    assert opts["batch_items"] in (32, 64, 128) and opts["block_size"] in (128, 256)
    assert opts["record_layout"] in (32, 48) and opts["samples_per_item"] == 1 and ms > 0
    stored = json.load(open(path))
    assert len(stored) == 1 and list(stored.values())[0]["waves_per_simd"] == opts["waves_per_simd"]
    opts2, ms2 = tv.autotune(g, cam, med, light, RO, probe_spp=4, cache_path=path)
    assert opts2 == opts and ms2 == pytest.approx(ms, abs=1e-4)
    a, _ = tv.render(g, cam, med, light, 8, 5, opts)
    b, _ = tv.render(g, cam, med, light, 8, 5, RO)
    sum_order_close(a.cpu().numpy(), b.cpu().numpy(), "tuned vs default options")
