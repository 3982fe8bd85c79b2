"""GPU: leb_update, the rebuild of a grid for a moving camera seeded from
its previous tree (the real-time pre-visualisation use of the paper's
"Results"; the camera criterion of "Subdivision Criteria" is what makes
the grid follow the camera).  The grid after an update must be the grid a
scratch leb_build makes with the same arguments, bit for bit (ids,
neighbour links, vertices, extinction, majorant), at every camera of
scripted paths -- turns, dollies in and out, a camera inside the volume,
one looking away -- and against the oracle's build on the small scenes."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from parity import assert_grids_equal, assert_image_parity

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


def device_grids_equal(a, b, what):
    """Bit equality of two device grids, compared on the device."""
    import torch
    fa = a.export(device=True)
    fb = b.export(device=True)
    assert fa["ids"].shape == fb["ids"].shape, f"{what}: {fa['ids'].shape[0]} vs {fb['ids'].shape[0]} tets"
    for k in ("ids", "nbr", "verts", "sigma", "majorant"):
        x, y = fa[k], fb[k]
        if k in ("sigma", "majorant"):
            x, y = x.view(torch.int32), y.view(torch.int32)
        assert torch.equal(x, y), f"{what}: {k} differs"


def path(cam, moves):
    """Cameras of a scripted path: (degrees, dolly) steps from `cam`."""
    out = [cam]
    for deg, dolly in moves:
        out.append(synthetic.camera_path(out[-1], 2, deg, dolly)[1])
    return out


SMALL_MOVES = [(4.0, 0.0), (4.0, 0.0), (0.0, 0.2), (0.0, 0.3), (25.0, 0.0), (0.0, -0.6), (90.0, 0.0),
               (0.0, -0.5), (180.0, 0.0), (3.0, 0.1)]


@pytest.mark.parametrize("scene", ["blobs_adaptive", "plume_tiny"])
def test_update_along_a_path_matches_scratch_and_oracle(tv, scene):
    import torch
    if scene == "plume_tiny":
        sc = synthetic.scene("plume_small")
        d = synthetic.plume(2, 64)
        n = 64
        sc["build"] = dict(sc["build"], max_depth=22)
    else:
        sc = synthetic.scene(scene)
        d = sc["density_fn"]()
        n = sc["n"]
    cam0 = dict(sc["camera"], width=160, height=120)
    dev = torch.from_numpy(d).cuda()
    g = tv.leb_build(dev, n, cam0, build=sc["build"])
    for i, cam in enumerate(path(cam0, SMALL_MOVES)):
        say(f"case update {scene} frame {i} pos {np.round(cam['pos'], 3).tolist()}")
        g.update(dev, n, cam, build=sc["build"])
        ref = tv.leb_build(dev, n, cam, build=sc["build"])
        device_grids_equal(g, ref, f"{scene} frame {i}")
        if i % 3 == 0:
            o = oracle.leb_build(d, n, cam, sc["build"])
            assert_grids_equal(g.export(), o.export(), f"{scene} frame {i} vs oracle")
        say(f"  {g.num_tets} tets, {g.info()['rounds']} rounds")


def test_update_camera_inside_and_looking_away(tv):
    import torch
    sc = synthetic.scene("blobs_adaptive")
    d = sc["density_fn"]()
    dev = torch.from_numpy(d).cuda()
    cams = [sc["camera"],
            dict(sc["camera"], pos=[0.5, 0.52, 0.45], look_at=[0.9, 0.5, 0.8]),   # inside the volume
            dict(sc["camera"], pos=[0.5, 0.5, -3.0], look_at=[0.5, 0.5, -4.0]),   # looking away: 6 roots
            dict(sc["camera"], pos=[0.45, 0.6, -0.2], look_at=[0.5, 0.5, 0.5]),
            sc["camera"]]
    g = tv.leb_build(dev, sc["n"], cams[0], build=sc["build"])
    for i, cam in enumerate(cams):
        say(f"case update inside/away {i}")
        g.update(dev, sc["n"], cam, build=sc["build"])
        o = oracle.leb_build(d, sc["n"], cam, sc["build"])
        assert_grids_equal(g.export(), o.export(), f"camera {i}")
    assert tv.leb_build(dev, sc["n"], cams[2], build=sc["build"]).num_tets == 6


def test_update_other_options_density_and_sparse(tv):
    """The previous tree is only a seed: updates that change the variation
    threshold, the depth cap, the want mode, the density itself, or read
    bricks all give the scratch build's grid."""
    import torch
    sc = synthetic.scene("blobs_adaptive")
    d = sc["density_fn"]()
    n = sc["n"]
    dev = torch.from_numpy(d).cuda()
    other = torch.from_numpy(synthetic.blobs(11, n)).cuda()
    g = tv.leb_build(dev, n, sc["camera"], build=sc["build"])
    steps = [("tau 0.1", dev, dict(sc["build"], variation_tau=0.1)),
             ("max depth 11", dev, dict(sc["build"], max_depth=11)),
             ("uniform depth 7", dev, dict(sc["build"], want_mode=1, uniform_depth=7)),
             ("random marks", dev, dict(sc["build"], want_mode=2, max_depth=14, rand_seed=3, rand_thresh=30000)),
             ("other density", other, sc["build"]),
             ("loose majorants", dev, dict(sc["build"], majorant_mode=1)),
             ("back", dev, sc["build"]),
             ("same again", dev, sc["build"]),
             # the variation criterion does not change with the volume's scale:
             # the same tree, with the new extinction
             ("density scale 2.5", dev, dict(sc["build"], density_scale=2.5)),
             ("volume doubled", dev * 2.0, sc["build"])]
    for what, vol, b in steps:
        say(f"case update {what}")
        g.update(vol, n, sc["camera"], build=b)
        device_grids_equal(g, tv.leb_build(vol, n, sc["camera"], build=b), what)
        if what in ("same again", "density scale 2.5", "volume doubled"):
            assert g.info()["rounds"] == 0, f"{what}: the tree should stand"
    # sparse: the bricks of the volume, shuffled
    nb = n // 8
    v = dev.view(nb, 8, nb, 8, nb, 8).permute(0, 2, 4, 1, 3, 5).reshape(nb ** 3, 512)
    pick = torch.nonzero(v.ne(0).any(dim=1)).flatten()
    pick = pick[torch.randperm(pick.numel(), generator=torch.Generator().manual_seed(1)).cuda()]
    vals = v.index_select(0, pick).contiguous()
    coords = torch.stack([pick % nb, (pick // nb) % nb, pick // (nb * nb)], dim=1).to(torch.int32).contiguous()
    for i, cam in enumerate(path(sc["camera"], [(10.0, 0.1), (-20.0, 0.0)])):
        say(f"case update sparse {i}")
        g.update_sparse(coords, vals, n, cam, build=sc["build"])
        device_grids_equal(g, tv.leb_build(dev, n, cam, build=sc["build"]), f"sparse {i}")


def test_update_errors_leave_the_grid_unchanged_and_drop_channels(tv):
    import torch
    sc = synthetic.scene("blobs_adaptive")
    d = sc["density_fn"]()
    n = sc["n"]
    dev = torch.from_numpy(d).cuda()
    g = tv.leb_build(dev, n, sc["camera"], build=sc["build"])
    before = g.export()
    far = synthetic.camera_path(sc["camera"], 2, 0.0, 0.5)[1]
    with pytest.raises(tv.TetError) as e:
        g.update(dev, n, far, build=dict(sc["build"], max_tets=1000))
    assert e.value.status == -3
    bad = d.copy()
    bad[5] = np.nan
    with pytest.raises(tv.TetError) as e:
        g.update(bad, n, far, build=sc["build"])
    assert e.value.status == -5
    assert_grids_equal(g.export(), before, "after failed updates")
    # channels are per tet: an update drops them
    g.set_channels(n, temperature=torch.ones(n ** 3, device="cuda"))
    g.update(dev, n, far, build=sc["build"])
    with pytest.raises(tv.TetError):
        g.export_channels()
    # the updated grid renders as the scratch grid does (the lanes' own light
    # walks: pixels written once, bit for bit)
    ref = tv.leb_build(dev, n, far, build=sc["build"])
    own = dict(sc["render"], max_steps_per_path=1 << 20)
    a, _ = tv.render(g, far, sc["medium"], sc["light"], 4, 5, own)
    b, _ = tv.render(ref, far, sc["medium"], sc["light"], 4, 5, own)
    assert torch.equal(a, b)
    import ctypes
    from paper_2506_11510_amd import _abi
    cam = _abi.make_camera(far)
    ds = tv.density_struct(dev, n, 1.0)
    assert tv.lib().leb_update(None, ctypes.byref(ds), ctypes.byref(cam), 1.0, None, None) == -1


@pytest.mark.timeout(600)
def test_update_cloud_orbit_full_size(tv):
    """The benchmark's cloud (256^3, 7 M tets) along a camera path of small
    steps (2 degrees and 1 % dolly a frame, as a real-time camera moves):
    every update equals the scratch build on the device; the first and the
    last frame also against the oracle (its image on a strided subset)."""
    import torch
    sc = synthetic.scene("cloud")
    d = sc["density_fn"]()
    dev = torch.from_numpy(d).cuda()
    cams = synthetic.camera_path(sc["camera"], 9, 2.0, 0.01)
    g = tv.leb_build(dev, 256, cams[0], build=sc["build"])
    for i, cam in enumerate(cams[1:], 1):
        g.update(dev, 256, cam, build=sc["build"])
        ref = tv.leb_build(dev, 256, cam, build=sc["build"])
        say(f"case cloud orbit frame {i}: {g.num_tets} tets, update {g.info()['ms']:.2f} ms "
            f"({g.info()['rounds']} rounds), scratch {ref.info()['ms']:.2f} ms")
        device_grids_equal(g, ref, f"cloud frame {i}")
        del ref
    o = oracle.leb_build(d, 256, cams[-1], sc["build"])
    assert_grids_equal(g.export(), o.export(), "cloud last frame vs oracle")
    cam = dict(cams[-1], width=256, height=256)
    img, _ = tv.render(g, cam, sc["medium"], sc["light"], 8, 44, sc["render"])
    pix = np.arange(0, 256 * 256, 7, dtype=np.int32)
    ref, _ = o.render(cam, sc["medium"], sc["light"], 8, 44, sc["render"], pixels=pix, threads=8)
    assert_image_parity(img.cpu().numpy().reshape(-1, 3)[pix], ref, "cloud orbit image")
