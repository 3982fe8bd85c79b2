"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Grids bit-exact (ids, neighbour links, vertices,
extinction, majorant); images per the pixel bar in parity.py."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from parity import assert_faces_equal, assert_grids_equal, assert_image_parity

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


def gpu_build(tv, d, n, camera, build):
    import torch
    dt = torch.from_numpy(np.ascontiguousarray(d)).cuda()
    return tv.leb_build(dt, n, camera, build=build)


TINY = synthetic.scene("tiny")


@pytest.fixture(scope="module")
def tiny_density():
    return TINY["density_fn"]()


@pytest.mark.parametrize("depth", [0, 1, 2, 5, 9])
def test_build_uniform_bitexact(tv, tiny_density, depth):
    say(f"case build uniform depth {depth}")
    b = dict(TINY["build"], uniform_depth=depth)
    g = gpu_build(tv, tiny_density, 64, TINY["camera"], b)
    o = oracle.leb_build(tiny_density, 64, TINY["camera"], b)
    e = o.export()
    assert_grids_equal(g.export(), e, f"uniform {depth}")
    assert_faces_equal(g, e, f"uniform {depth}")
    assert g.info()["max_depth"] == depth


@pytest.mark.parametrize("seed,depth,thresh", [(0, 14, 40000), (1, 16, 30000), (2, 12, 60000), (3, 17, 22000)])
def test_build_random_adaptive_bitexact(tv, tiny_density, seed, depth, thresh):
    say(f"case build random seed {seed} depth {depth}")
    b = dict(TINY["build"], want_mode=2, max_depth=depth, rand_seed=seed, rand_thresh=thresh)
    g = gpu_build(tv, tiny_density, 64, TINY["camera"], b)
    o = oracle.leb_build(tiny_density, 64, TINY["camera"], b)
    e = o.export()
    assert_grids_equal(g.export(), e, f"random {seed}")
    assert_faces_equal(g, e, f"random {seed}")


@pytest.mark.parametrize("maj,tau,tgt", [(1, 0.3, 2.0), (0, 0.1, 1.0), (1, 0.6, 0.5)])
def test_build_criteria_bitexact(tv, maj, tau, tgt):
    sc = synthetic.scene("blobs_adaptive")
    d = sc["density_fn"]()
    b = dict(sc["build"], majorant_mode=maj, variation_tau=tau, target_px=tgt)
    say(f"case build criteria maj {maj} tau {tau} target {tgt}")
    g = gpu_build(tv, d, 32, sc["camera"], b)
    o = oracle.leb_build(d, 32, sc["camera"], b)
    e = o.export()
    assert_grids_equal(g.export(), e, "criteria")
    assert_faces_equal(g, e, "criteria")  # loose majorants (maj 1): 48-byte records only


RANDOM_706K = dict(want_mode=2, max_depth=17, rand_seed=3, rand_thresh=22000)  # 706,206 tets


@pytest.mark.parametrize("max_tets", [706206, 1 << 22])
def test_build_phases_bitexact(tv, tiny_density, max_tets):
    """The build's three kinds of rounds meet: with max_tets at the final
    size the rounds in one cooperative launch stop at half of it and the
    compacting, then appending (tail) rounds finish the grid; with a large
    max_tets the cooperative launch builds it all.  Both bit-exact, and one
    tet fewer is a capacity error."""
    say(f"case build phases max_tets {max_tets}")
    b = dict(TINY["build"], **RANDOM_706K)
    o = oracle.leb_build(tiny_density, 64, TINY["camera"], b)
    g = gpu_build(tv, tiny_density, 64, TINY["camera"], dict(b, max_tets=max_tets))
    assert g.info()["num_tets"] == 706206
    assert_grids_equal(g.export(), o.export(), f"phases {max_tets}")
    if max_tets == 706206:
        with pytest.raises(tv.TetError) as e:
            gpu_build(tv, tiny_density, 64, TINY["camera"], dict(b, max_tets=706205))
        assert e.value.status == -3


@pytest.mark.parametrize("b", [dict(uniform_depth=9), dict(want_mode=2, max_depth=16, rand_seed=1, rand_thresh=30000)])
def test_build_host_rounds_option(tv, tiny_density, b):
    """host_rounds = 1 drives every round from the host (no cooperative
    launch): the same grid as the default build and the oracle's."""
    say(f"case build host_rounds {b}")
    bb = dict(TINY["build"], **b)
    g = gpu_build(tv, tiny_density, 64, TINY["camera"], dict(bb, host_rounds=1))
    o = oracle.leb_build(tiny_density, 64, TINY["camera"], bb)
    assert_grids_equal(g.export(), o.export(), f"host rounds {b}")
    assert_grids_equal(gpu_build(tv, tiny_density, 64, TINY["camera"], bb).export(), o.export(), "default")


def test_build_host_rounds_only(tv, tiny_density):
    """max_tets below 12 leaves no room for the cooperative rounds, so every
    round runs from the host (the path of devices without cooperative
    launch): the 6 roots bit-exact, and depth 1 (12 tets) a capacity error."""
    say("case build host rounds only")
    b = dict(TINY["build"], uniform_depth=0, max_tets=6)
    g = gpu_build(tv, tiny_density, 64, TINY["camera"], b)
    o = oracle.leb_build(tiny_density, 64, TINY["camera"], b)
    assert_grids_equal(g.export(), o.export(), "host rounds depth 0")
    with pytest.raises(tv.TetError) as e:
        gpu_build(tv, tiny_density, 64, TINY["camera"], dict(TINY["build"], uniform_depth=1, max_tets=11))
    assert e.value.status == -3


def test_locate_matches_oracle(tv, tiny_density):
    say("case locate")
    b = dict(TINY["build"], want_mode=2, max_depth=15, rand_seed=7, rand_thresh=40000)
    g = gpu_build(tv, tiny_density, 64, TINY["camera"], b)
    o = oracle.leb_build(tiny_density, 64, TINY["camera"], b)
    rng = np.random.default_rng(0)
    pts = rng.random((20000, 3)).astype(np.float32)
    # points on lattice planes, edges and corners, and on the cube boundary
    q = (rng.integers(0, 65, (4000, 3)) / 64.0).astype(np.float32)
    pts = np.concatenate([pts, q, np.float32([[0, 0, 0], [1, 1, 1], [0.5, 0.5, 0.5], [1, 0, 0.25]])])
    assert np.array_equal(g.locate(pts), o.locate(pts))


def render_both(tv, g, o, sc, cam, spp, seed, ropts):
    import torch
    img, st = tv.render(g, cam, sc["medium"], sc["light"], spp, seed, ropts)
    torch.cuda.synchronize()
    ref, rst = o.render(cam, sc["medium"], sc["light"], spp, seed, ropts, threads=8)
    return img.cpu().numpy(), st, ref, rst


QUEUED, OWN = (1 << 31) - 1, 1 << 20  # step guards: light rays queued and sorted / walked by their lanes


@pytest.mark.parametrize("layout,waves,guard", [(32, 8, QUEUED), (48, 8, OWN), (32, 5, OWN), (48, 4, QUEUED)])
def test_render_tiny_parity(tv, tiny_density, layout, waves, guard):
    say(f"case render tiny 64x64 16spp, {layout}-byte records, {waves} waves, step guard {guard}")
    sc = TINY
    g = gpu_build(tv, tiny_density, 64, sc["camera"], sc["build"])
    o = oracle.leb_build(tiny_density, 64, sc["camera"], sc["build"])
    r = dict(sc["render"], record_layout=layout, waves_per_simd=waves, max_steps_per_path=guard)
    img, st, ref, rst = render_both(tv, g, o, sc, sc["camera"], 16, 1234, r)
    assert_image_parity(img, ref, "tiny")
    assert st["real_collisions"] > 0 and st["escapes"] > 0
    # identical paths take identical numbers of steps (up to rare last-ulp
    # differences of transcendental functions)
    assert abs(st["tet_steps"] - rst["tet_steps"]) <= 1e-4 * rst["tet_steps"]


@pytest.mark.parametrize("mode,per_item", [(0, 0), (1, 0), (2, 0), (0, 3)])
def test_render_modes_parity(tv, mode, per_item):
    """Loose majorants (null collisions), ratio / delta light transmittance,
    and work items of a few samples accumulated with atomics."""
    sc = synthetic.scene("blobs_adaptive")
    d = sc["density_fn"]()
    say(f"case render modes transmittance {mode} per_item {per_item}")
    g = gpu_build(tv, d, 32, sc["camera"], sc["build"])
    o = oracle.leb_build(d, 32, sc["camera"], sc["build"])
    r = dict(sc["render"], transmittance=mode, samples_per_item=per_item)
    img, st, ref, rst = render_both(tv, g, o, sc, sc["camera"], 8, 99, r)
    assert_image_parity(img, ref, f"mode {mode}")
    if mode == 0:
        assert st["null_collisions"] > 0


@pytest.mark.parametrize("dense", [False, True])
def test_queued_light_rays_equal_lane_walks(tv, dense):
    """Light rays queued and walked after the pass in the order of where
    they start give the paths, steps and collisions of the lanes' own light
    walks, and the image up to the order of FP32 sums per pixel (relative
    1e-5); both against the oracle.  The dense case (thick, bright medium,
    many bounces) has more light rays than the queue holds: the rest are
    walked by their lanes."""
    sc = synthetic.scene("blobs_adaptive")
    d = sc["density_fn"]() * (30.0 if dense else 1.0)
    med = dict(albedo=0.99, g=0.5) if dense else sc["medium"]
    say(f"case queued light rays, dense {dense}")
    g = gpu_build(tv, d, 32, sc["camera"], sc["build"])
    o = oracle.leb_build(d, 32, sc["camera"], sc["build"])
    cam = dict(sc["camera"], width=48, height=40)
    base = dict(sc["render"], max_bounces=64 if dense else 8)
    out = {}
    for guard in (QUEUED, OWN):
        img, st = tv.render(g, cam, med, sc["light"], 8, 31, dict(base, max_steps_per_path=guard))
        out[guard] = (img.cpu().numpy().astype(np.float64), st)
    (a, sa), (b, sb) = out[QUEUED], out[OWN]
    say(f"  queued {sa['light_rays_queued']} of {sa['real_collisions']} light rays")
    for k in ("tet_steps", "real_collisions", "null_collisions", "escapes", "truncated"):
        assert sa[k] == sb[k], k
    assert sb["light_rays_queued"] == 0 and sa["light_rays_queued"] > 0
    if dense:
        assert sa["light_rays_queued"] < sa["real_collisions"]
    else:
        assert sa["light_rays_queued"] == sa["real_collisions"]
    floor = 1e-4 * np.abs(b).mean()
    assert (np.abs(a - b) / np.maximum(np.abs(b), floor)).max() <= 1e-5
    ref, rst = o.render(cam, med, sc["light"], 8, 31, dict(base, max_steps_per_path=QUEUED), threads=8)
    assert_image_parity(a.reshape(-1, 3), ref, f"queued light rays, dense {dense}")
    assert abs(sa["tet_steps"] - rst["tet_steps"]) <= 1e-4 * rst["tet_steps"]


def test_render_ragged_sizes_and_offsets(tv, tiny_density):
    """Image sizes that do not fill the 8x8 tiles, 1 spp, sample offsets."""
    sc = TINY
    g = gpu_build(tv, tiny_density, 64, sc["camera"], dict(sc["build"], uniform_depth=7))
    o = oracle.leb_build(tiny_density, 64, sc["camera"], dict(sc["build"], uniform_depth=7))
    for w, h, spp, off in [(1, 1, 1, 0), (13, 7, 3, 5), (70, 9, 2, 0)]:
        say(f"case render ragged {w}x{h} spp {spp} offset {off}")
        cam = dict(sc["camera"], width=w, height=h)
        img, st, ref, rst = render_both(tv, g, o, sc, cam, spp, 7, dict(sc["render"], sample_offset=off))
        assert_image_parity(img, ref, f"{w}x{h}")


@pytest.mark.parametrize("spp,off,per_item", [(48, 0, 0), (70, 3, 8)])
def test_render_multi_pass(tv, tiny_density, spp, off, per_item):
    """A render whose entry records do not fit one pass (at most 2^25 per
    pass: 32 samples of a 1024^2 image): the passes' samples add up in the
    image exactly as one pass would (strided subset against the oracle)."""
    sc = TINY
    say(f"case render multi-pass 1024x1024 spp {spp} offset {off} per item {per_item}")
    g = gpu_build(tv, tiny_density, 64, sc["camera"], sc["build"])
    o = oracle.leb_build(tiny_density, 64, sc["camera"], sc["build"])
    cam = dict(sc["camera"], width=1024, height=1024)
    r = dict(sc["render"], sample_offset=off, samples_per_item=per_item)
    img, st = tv.render(g, cam, sc["medium"], sc["light"], spp, 77, r)
    pix = np.arange(0, 1024 * 1024, 257, dtype=np.int32)
    ref, rst = o.render(cam, sc["medium"], sc["light"], spp, 77, r, pixels=pix, threads=8)
    assert_image_parity(img.cpu().numpy().reshape(-1, 3)[pix], ref, f"multi-pass spp {spp}")
    # counters of all passes: the subset's steps scale to the whole image
    assert abs(st["tet_steps"] / (1024 * 1024) - rst["tet_steps"] / len(pix)) < 0.02 * rst["tet_steps"] / len(pix)


def test_render_edge_cases(tv, tiny_density):
    """Edge cases of the walk: the camera inside the grid (rays start in a
    tet instead of entering through the boundary), a light exactly along an
    axis and along a face diagonal (light rays with zero denominators for
    most face planes), and an empty volume (6 tets, the environment and the
    sun through clear space)."""
    import torch
    sc = TINY
    g = gpu_build(tv, tiny_density, 64, sc["camera"], dict(sc["build"], uniform_depth=8))
    o = oracle.leb_build(tiny_density, 64, sc["camera"], dict(sc["build"], uniform_depth=8))
    inside = dict(pos=[0.5, 0.47, 0.41], look_at=[0.9, 0.6, 0.8], up=[0, 1, 0], fov_y_deg=70.0, width=40, height=36)
    for what, cam, light in [
            ("camera inside", inside, sc["light"]),
            ("sun along +y", sc["camera"], dict(sc["light"], sun_dir=[0.0, 1.0, 0.0])),
            ("sun along -x", inside, dict(sc["light"], sun_dir=[-1.0, 0.0, 0.0])),
            ("sun along a face diagonal", sc["camera"],
             dict(sc["light"], sun_dir=[float(np.float32(0.5 ** 0.5)), 0.0, float(np.float32(0.5 ** 0.5))]))]:
        cam = dict(cam, width=40, height=36)
        for mode in (0, 1):
            say(f"case edge: {what}, light transmittance {mode}")
            r = dict(sc["render"], transmittance=mode)
            img, st = tv.render(g, cam, sc["medium"], light, 8, 31, r)
            ref, rst = o.render(cam, sc["medium"], light, 8, 31, r, threads=8)
            assert_image_parity(img.cpu().numpy(), ref, what)
            assert st["truncated"] == 0 and st["real_collisions"] > 0
    say("case edge: empty volume")
    z = np.zeros(64 ** 3, np.float32)
    ge = gpu_build(tv, z, 64, sc["camera"], dict(sc["build"], want_mode=0, variation_tau=0.2, max_depth=20))
    assert ge.num_tets == 6
    img, st = tv.render(ge, sc["camera"], sc["medium"], sc["light"], 4, 3, sc["render"])
    env = np.float32(sc["light"]["env_radiance"])
    assert np.array_equal(img.cpu().numpy().reshape(-1, 3), np.broadcast_to(env, (64 * 64, 3)))
    assert st["real_collisions"] == 0 and st["null_collisions"] == 0


def test_dda_parity(tv):
    import torch
    say("case dda")
    n = 32
    d = synthetic.blobs(5, n)
    cam = dict(pos=[0.3, 0.6, -1.5], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=40.0, width=40, height=32)
    med = dict(albedo=0.9, g=0.3)
    ropt = dict(max_bounces=8)
    img, st = tv.dda_render(torch.from_numpy(d).cuda(), n, 1.5, cam, med, synthetic.LIGHT_DEFAULT, 8, 5, ropt)
    ref, rst = oracle.dda_render(d, n, 1.5, cam, med, synthetic.LIGHT_DEFAULT, 8, 5, ropt, threads=8)
    assert_image_parity(img.cpu().numpy(), ref, "dda")


def test_build_errors(tv, tiny_density):
    import torch
    say("case build errors")
    with pytest.raises(tv.TetError) as e:
        gpu_build(tv, tiny_density, 64, TINY["camera"], dict(TINY["build"], max_tets=1000))
    assert e.value.status == -3
    bad = tiny_density.copy()
    bad[77] = np.nan
    with pytest.raises(tv.TetError) as e:
        gpu_build(tv, bad, 64, TINY["camera"], TINY["build"])
    assert e.value.status == -5
    bad[77] = -2.0
    with pytest.raises(tv.TetError) as e:
        gpu_build(tv, bad, 64, TINY["camera"], TINY["build"])
    assert e.value.status == -5
    # host-side density gives the same grid as a device one
    g1 = tv.leb_build(tiny_density, 64, TINY["camera"], build=TINY["build"])
    g2 = gpu_build(tv, tiny_density, 64, TINY["camera"], TINY["build"])
    assert np.array_equal(g1.export()["nbr"], g2.export()["nbr"])


@pytest.mark.timeout(900)
def test_cloud_full_size(tv):
    """The benchmark workload: 256^3 fBm cloud, adaptive grid at 1 px,
    1024^2, 32 spp, 32 bounces, in the benchmark's launch configuration.
    Grid bit-exact against the oracle's; image checked on a strided subset of
    17,190 pixels the oracle renders."""
    import torch
    sc = synthetic.scene("cloud")
    d = sc["density_fn"]()
    say("case cloud full size: gpu build")
    g = gpu_build(tv, d, 256, sc["camera"], sc["build"])
    say("case cloud full size: oracle build", g.info())
    o = oracle.leb_build(d, 256, sc["camera"], sc["build"])
    say("case cloud full size: compare grids")
    e = o.export()
    assert_grids_equal(g.export(), e, "cloud")
    assert_faces_equal(g, e, "cloud")
    del e
    say("case cloud full size: gpu render")
    # the launch bench.py times (one sample per work item, chunk sums added
    # atomically, compact records, 5 waves per SIMD)
    launch = dict(samples_per_item=1, batch_items=64, record_layout=32, waves_per_simd=5, event_wait=48)
    img, st = tv.render(g, sc["camera"], sc["medium"], sc["light"], 32, 2024, dict(sc["render"], **launch))
    img = img.cpu().numpy().reshape(-1, 3)
    say("case cloud full size: oracle subset", st)
    pix = np.arange(0, 1024 * 1024, 61, dtype=np.int32)  # 17,190 pixels
    ref, rst = o.render(sc["camera"], sc["medium"], sc["light"], 32, 2024, sc["render"], pixels=pix, threads=8)
    assert_image_parity(img[pix], ref, "cloud subset")
