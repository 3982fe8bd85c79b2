"""GPU build from a sparse volume (8^3 bricks, zero elsewhere): grids bit
for bit those of the dense build of the volume the bricks describe (and of
the oracle's build of it), for host and device bricks in any order, with
empty bricks listed, no bricks at all, one brick; and the argument
errors."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from parity import assert_grids_equal

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


def cut(d, keep):
    thr = np.quantile(d, 1.0 - keep)
    return np.where(d > thr, d - thr, 0.0).astype(np.float32)


def sparse_build(tv, d, n, cam, build, device, keep_empty=0, seed=0):
    import torch
    coords, values = synthetic.bricks(d, n, keep_empty=keep_empty, seed=seed)
    if device:
        coords, values = torch.from_numpy(coords).cuda(), torch.from_numpy(values).cuda()
    return tv.leb_build_sparse(coords, values, n, cam, build=build), len(coords)


@pytest.mark.parametrize("name,keep,device,empty", [("tiny", 0.3, True, 0), ("tiny", 0.05, False, 7),
                                                    ("blobs_adaptive", 0.2, True, 3), ("blobs_adaptive", 1.0, False, 0)])
def test_sparse_build_bitexact(tv, name, keep, device, empty):
    say(f"case sparse build {name} keep {keep} device {device} empty {empty}")
    import torch
    sc = synthetic.scene(name)
    n = sc["n"]
    d = cut(sc["density_fn"](), keep) if keep < 1.0 else sc["density_fn"]()
    g, nbr = sparse_build(tv, d, n, sc["camera"], sc["build"], device, empty, seed=3)
    dense = tv.leb_build(torch.from_numpy(d).cuda(), n, sc["camera"], build=sc["build"])
    assert_grids_equal(g.export(), dense.export(), f"sparse vs dense {name}")
    o = oracle.leb_build(oracle.densify(*synthetic.bricks(d, n, keep_empty=empty, seed=3), n), n, sc["camera"],
                         sc["build"])
    assert_grids_equal(g.export(), o.export(), f"sparse vs oracle {name}")
    assert nbr <= (n // 8) ** 3


def test_sparse_adaptive_criteria(tv):
    """The paper's criteria on a cut cloud: density variation and camera,
    loose majorants (max over the box reads the sparse levels)."""
    say("case sparse build cloud 64^3 criteria")
    import torch
    n = 64
    d = synthetic.cloud(5, n)
    sc = synthetic.scene("blobs_adaptive")
    b = dict(sc["build"], max_depth=18, majorant_mode=1, variation_tau=0.25, target_px=1.0)
    cam = dict(sc["camera"], width=256, height=256)
    g, _ = sparse_build(tv, d, n, cam, b, True, 11, seed=5)
    dense = tv.leb_build(torch.from_numpy(d).cuda(), n, cam, build=b)
    o = oracle.leb_build(d, n, cam, b)
    assert_grids_equal(g.export(), dense.export(), "sparse cloud vs dense")
    assert_grids_equal(g.export(), o.export(), "sparse cloud vs oracle")
    assert g.num_tets > 10000


@pytest.mark.timeout(600)
def test_sparse_cloud_full_size(tv):
    """The benchmark volume (256^3 cloud, 20 % occupancy) from its bricks:
    the 7 M-tet grid equals the dense build's."""
    say("case sparse build cloud 256^3")
    import torch
    sc = synthetic.scene("cloud")
    d = sc["density_fn"]()
    g, nbr = sparse_build(tv, d, 256, sc["camera"], sc["build"], True, 0, seed=1)
    dense = tv.leb_build(torch.from_numpy(d).cuda(), 256, sc["camera"], build=sc["build"])
    a, b = g.export(), dense.export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    say("bricks", nbr, "of", 32 ** 3, g.info())


def test_sparse_edge_cases(tv):
    say("case sparse build edge cases")
    import torch
    sc = synthetic.scene("tiny")
    cam = sc["camera"]
    b = dict(sc["build"], uniform_depth=4, max_depth=4)
    # no bricks: the all-zero volume
    e = np.zeros((0, 3), np.int32), np.zeros((0, 512), np.float32)
    g = tv.leb_build_sparse(*e, 16, cam, build=b)
    z = tv.leb_build(torch.zeros(16 ** 3, device="cuda"), 16, cam, build=b)
    assert_grids_equal(g.export(), z.export(), "empty")
    assert (g.export()["sigma"] == 0).all()
    # n = 8: one brick is the whole volume
    v = np.random.default_rng(2).uniform(0, 3, 512).astype(np.float32)
    g = tv.leb_build_sparse(np.zeros((1, 3), np.int32), v[None], 8, cam, build=b)
    z = tv.leb_build(torch.from_numpy(v).cuda(), 8, cam, build=b)
    assert_grids_equal(g.export(), z.export(), "one brick")
    # errors: duplicate, out of range, negative value, n below a brick
    c = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    vals = np.ones((2, 512), np.float32)
    with pytest.raises(tv.TetError) as ex:
        tv.leb_build_sparse(np.array([[1, 1, 0], [1, 1, 0]], np.int32), vals, 16, cam, build=b)
    assert ex.value.status == -1
    with pytest.raises(tv.TetError) as ex:
        tv.leb_build_sparse(np.array([[0, 0, 0], [2, 0, 0]], np.int32), vals, 16, cam, build=b)
    assert ex.value.status == -1
    bad = vals.copy()
    bad[1, 17] = -1.0
    with pytest.raises(tv.TetError) as ex:
        tv.leb_build_sparse(c, bad, 16, cam, build=b)
    assert ex.value.status == -5
    with pytest.raises(tv.TetError) as ex:
        tv.leb_build_sparse(np.zeros((0, 3), np.int32), np.zeros((0, 512), np.float32), 4, cam, build=b)
    assert ex.value.status == -1


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_sparse_random_bricks(tv, seed):
    """Random brick subsets of random volumes (some bricks all zero, values
    with exact ties), the paper's criteria: sparse and dense builds agree bit
    for bit."""
    say(f"case sparse random bricks seed {seed}")
    import torch
    rng = np.random.default_rng(100 + seed)
    n = [16, 32, 64, 32][seed]
    nb = n // 8
    keep = rng.random(nb ** 3) < [0.1, 0.3, 0.6, 1.0][seed]
    vals = np.round(rng.uniform(0.0, 8.0, (nb ** 3, 512)), 1).astype(np.float32)
    vals[rng.random(nb ** 3) < 0.2] = 0.0
    pick = np.flatnonzero(keep)
    coords = np.stack([pick % nb, (pick // nb) % nb, pick // (nb * nb)], axis=1).astype(np.int32)
    values = vals[pick]
    d = oracle.densify(coords, values, n)
    sc = synthetic.scene("blobs_adaptive")
    b = dict(sc["build"], max_depth=14, variation_tau=[0.1, 0.3, 0.5, 0.2][seed], majorant_mode=seed % 2)
    order = rng.permutation(len(coords))
    g = tv.leb_build_sparse(torch.from_numpy(coords[order]).cuda(), torch.from_numpy(values[order]).cuda(), n,
                            sc["camera"], build=b)
    dense = tv.leb_build(torch.from_numpy(d).cuda(), n, sc["camera"], build=b)
    assert_grids_equal(g.export(), dense.export(), f"random bricks {seed}")
