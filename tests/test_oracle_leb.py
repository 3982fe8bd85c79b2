"""Pins of the oracle's grid construction against what the paper and the
mathematics fix (no GPU).  Paper: "Grid Construction" (control cube of 24
tets, Maubach bisection, conforming propagation, subdivision criteria) and
"Path Tracing within Tetrahedral Grids" (<= 4 neighbours, 18 orientations)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synthetic

S = 1 << 20
TINY = synthetic.scene("tiny")


@pytest.fixture(scope="module")
def dens64():
    return TINY["density_fn"]()


def build(d, n=64, **b):
    return oracle.leb_build(d, n, TINY["camera"], dict(TINY["build"], **b))


def edges(V):
    return [(i, j) for i in range(4) for j in range(i + 1, 4)]


def test_uniform_counts(dens64):
    """Every bisection doubles: 6 * 2^d tets at uniform depth d."""
    for d in range(0, 10):
        g = build(dens64, uniform_depth=d)
        assert g.num_tets == 6 * 2 ** d
        assert g.max_depth == d


def test_depth2_is_the_papers_24_halfedge_tets(dens64):
    """The paper's control cube: 24 tets, one per half-edge of the cube, made
    of the half-edge's two vertices, the centre of the face carrying it and
    the cube centre.  They are exactly depth 2 of the 6 Kuhn roots."""
    e = build(dens64, uniform_depth=2).export()
    got = {frozenset(map(tuple, v)) for v in e["verts"].tolist()}
    corners = list(itertools.product([0, S], repeat=3))
    centre = (S // 2,) * 3
    want = set()
    for a, b in itertools.combinations(corners, 2):
        diff = [x != y for x, y in zip(a, b)]
        if sum(diff) != 1:
            continue  # not a cube edge
        ax = diff.index(True)
        for other in range(3):
            if other == ax:
                continue
            # the two faces carrying this edge: fixed coordinate `other`
            fc = [S // 2] * 3
            fc[other] = a[other]
            want.add(frozenset([a, b, tuple(fc), centre]))
    assert len(want) == 24
    assert got == want


def test_refinement_edge_is_unique_longest(dens64):
    """Maubach's tagged rule picks (x0, x_k), k = 3 - d mod 3; on these grids
    that is the unique longest edge at every depth ("longest edge
    bisection")."""
    for d in range(0, 10):
        e = build(dens64, uniform_depth=d).export()
        V = e["verts"].astype(np.int64)
        k = 3 - d % 3
        L = {(i, j): ((V[:, i] - V[:, j]) ** 2).sum(1) for i, j in edges(V)}
        ref = L[(0, k)]
        for key, val in L.items():
            if key != (0, k):
                assert (ref > val).all()


def test_eighteen_face_orientations_and_outwardness(dens64):
    """The grid produces exactly 18 face orientations; each stored normal is
    outward (away from the opposite vertex) and orthogonal to the face."""
    e = build(dens64, uniform_depth=9).export()
    assert np.unique(e["codes"]).size == 18
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, -1, 0], [1, 0, 1], [1, 0, -1], [0, 1, 1],
                     [0, 1, -1]])
    V = e["verts"].astype(np.int64)
    for f in range(4):
        n = dirs[e["codes"][:, f] >> 1] * np.where(e["codes"][:, f] & 1, -1, 1)[:, None]
        others = [j for j in range(4) if j != f]
        for j in others:
            assert ((n * V[:, j]).sum(1) == e["offsets"][:, f]).all()
        assert ((n * V[:, f]).sum(1) < e["offsets"][:, f]).all()


def volumes(V):
    V = V.astype(np.int64)
    a, b, c = V[:, 1] - V[:, 0], V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]
    det = np.einsum("ij,ij->i", a.astype(float), np.cross(b.astype(float), c.astype(float)))
    return np.abs(det) / 6.0


def test_volumes_sum_to_cube(dens64):
    for b in [dict(uniform_depth=9), dict(want_mode=2, max_depth=16, rand_seed=3, rand_thresh=30000)]:
        e = build(dens64, **b).export()
        vol = volumes(e["verts"])
        assert vol.sum() == pytest.approx(float(S) ** 3, rel=1e-12)
        # each bisection halves the volume: vol = S^3 / 6 / 2^depth
        depth = np.array([int(i).bit_length() - 4 for i in e["ids"]])
        assert np.allclose(vol, float(S) ** 3 / 6 / 2.0 ** depth)


def brute_neighbours(e):
    """O(N^2)-free but definition-level face matching with Python dicts."""
    faces = {}
    V = e["verts"]
    for t in range(len(V)):
        for f in range(4):
            key = frozenset(tuple(V[t, j]) for j in range(4) if j != f)
            faces.setdefault(key, []).append((t, f))
    return faces


@pytest.mark.parametrize("b", [dict(uniform_depth=6), dict(want_mode=2, max_depth=12, rand_seed=11, rand_thresh=45000),
                               dict(want_mode=2, max_depth=14, rand_seed=5, rand_thresh=20000)])
def test_conforming_and_reciprocal(dens64, b):
    """Conforming: every interior face is shared by exactly 2 tets, every
    other face lies on the cube boundary; exactly one neighbour per face and
    nbr[nbr[i][f]][bf] == i (paper: exactly 4 neighbours, fewer at the
    boundary)."""
    e = build(dens64, **b).export()
    faces = brute_neighbours(e)
    nbr = e["nbr"]
    for key, owners in faces.items():
        assert len(owners) <= 2
        if len(owners) == 1:
            t, f = owners[0]
            pts = np.array(list(key))
            assert any((pts[:, a] == pts[0, a]).all() and pts[0, a] in (0, S) for a in range(3))
            assert nbr[t, f] == 0xFFFFFFFF
        else:
            (t, f), (u, g) = owners
            assert nbr[t, f] == (u << 2) | g
            assert nbr[u, g] == (t << 2) | f
    inner = nbr != 0xFFFFFFFF
    j = (nbr[inner] >> 2).astype(np.int64)
    bf = (nbr[inner] & 3).astype(np.int64)
    ti = np.nonzero(inner)[0]
    assert (nbr[j, bf] >> 2 == ti).all()


def test_order_independence(dens64):
    """The propagation rule is deterministic: the final grid does not depend
    on the order in which wanted tets are refined."""
    base = build(dens64, want_mode=2, max_depth=14, rand_seed=21, rand_thresh=40000).export()["ids"]
    for sh in [1, 2, 3]:
        e = build(dens64, want_mode=2, max_depth=14, rand_seed=21, rand_thresh=40000, shuffle_seed=sh).export()
        assert np.array_equal(e["ids"], base)


def test_minimal_and_no_leaf_wanted(dens64):
    """The result is want-free and locally minimal: merging any pair of leaf
    siblings back into their parent would either leave a wanted tet or break
    conformity (a vertex of the mesh on one of the parent's edge
    midpoints)."""
    b = dict(TINY["build"], want_mode=2, max_depth=13, rand_seed=9, rand_thresh=35000)
    e = oracle.leb_build(dens64, 64, TINY["camera"], b).export()
    ids = e["ids"]
    depth = np.array([int(i).bit_length() - 4 for i in ids], np.int32)
    w = oracle.want(dens64, 64, TINY["camera"], b, e["verts"], depth, ids)
    assert not w.any()
    V = e["verts"].astype(np.int64)
    vcount = {}
    for t in range(len(V)):
        for j in range(4):
            vcount[tuple(V[t, j])] = vcount.get(tuple(V[t, j]), 0) + 1
    pos = {int(i): t for t, i in enumerate(ids)}
    pairs = []
    for t, i in enumerate(ids):
        i = int(i)
        if i % 2 == 0 and (i + 1) in pos:
            pairs.append((t, pos[i + 1], i // 2, int(depth[t]) - 1))
    assert len(pairs) > 10
    parents, zs = [], []
    for t, u, par, pd in pairs:
        k = 3 - pd % 3
        # the first child is the parent with x_k replaced by z; the second
        # child is (x1..x_k, z, ...), so its slot k-1 holds x_k
        Vp = V[t].copy()
        zs.append(tuple(V[t, k]))
        Vp[k] = V[u, k - 1]
        parents.append(Vp)
    parents = np.array(parents)
    pw = oracle.want(dens64, 64, TINY["camera"], b, parents.astype(np.int32),
                     np.array([p[3] for p in pairs], np.int32), np.array([p[2] for p in pairs], np.uint64))
    for Vp, z, w_par in zip(parents, zs, pw):
        # does a vertex of the mesh, other than z held by the two children,
        # sit on an edge midpoint of the parent?
        hanging = False
        for a in range(4):
            for c in range(a + 1, 4):
                m = Vp[a] + Vp[c]
                if (m % 2).any():
                    continue
                m = tuple(m // 2)
                cnt = vcount.get(m, 0) - (2 if m == z else 0)
                hanging |= cnt > 0
        assert w_par or hanging


def test_edge_valence_at_most_8(dens64):
    e = build(dens64, want_mode=2, max_depth=15, rand_seed=2, rand_thresh=40000).export()
    cnt = {}
    V = e["verts"]
    for t in range(len(V)):
        for a in range(4):
            for c in range(a + 1, 4):
                key = frozenset([tuple(V[t, a]), tuple(V[t, c])])
                cnt[key] = cnt.get(key, 0) + 1
    assert max(cnt.values()) <= 8


def test_box_stats_against_brute_force():
    """D(T) statistics: min/max exactly those of the voxels overlapping the
    open box; the FP64 sum within the bound of summation error of the exact
    rational sum; count = number of voxels."""
    rng = np.random.default_rng(0)
    n = 16
    d = (rng.random(n ** 3) * rng.integers(0, 2, n ** 3)).astype(np.float32)
    G = d.reshape(n, n, n)  # [k][j][i]
    vs = S // n
    for _ in range(200):
        lv = int(rng.integers(0, 5))
        cell = S >> lv
        lo = [int(rng.integers(0, 1 << lv)) * cell for _ in range(3)]
        ext = [cell // int(rng.choice([1, 2])) for _ in range(3)]
        hi = [l + e for l, e in zip(lo, ext)]
        hi = [min(h, S) for h in hi]
        mn, mx, s, c = oracle.box_stats(d, n, lo, hi)
        r0 = [l // vs for l in lo]
        r1 = [-(-h // vs) for h in hi]
        sub = G[r0[2]:r1[2], r0[1]:r1[1], r0[0]:r1[0]]
        assert mn == sub.min() and mx == sub.max()
        assert c == sub.size
        exact = sum(Fraction(float(x)) for x in sub.ravel())
        assert abs(Fraction(s) - exact) <= Fraction(sub.size * 2.0 ** -52) * (abs(exact) + 1)


def test_point_location_against_brute_force(dens64):
    """Point location equals the tet whose closed set strictly contains the
    point (barycentric test over all tets), for points away from faces."""
    g = build(dens64, want_mode=2, max_depth=11, rand_seed=4, rand_thresh=40000)
    e = g.export()
    V = e["verts"].astype(np.float64) / S
    rng = np.random.default_rng(1)
    pts = rng.random((300, 3)).astype(np.float32)
    got = g.locate(pts)
    T = np.stack([V[:, 1] - V[:, 0], V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]], axis=2)  # (n,3,3)
    Tinv = np.linalg.inv(T)
    checked = 0
    for p, gi in zip(pts.astype(np.float64), got):
        lam = np.einsum("nij,nj->ni", Tinv, p[None] - V[:, 0])
        lam4 = np.concatenate([1 - lam.sum(1, keepdims=True), lam], axis=1)
        inside = (lam4 > 1e-9).all(1)
        if inside.sum() == 1:
            assert gi == np.nonzero(inside)[0][0]
            checked += 1
    assert checked > 250


def test_camera_criterion_closed_forms(dens64):
    """Camera test: a tet behind the camera is never wanted; a tet's split
    flips exactly when its projected size l * k_px / z crosses target_px."""
    cam = dict(pos=[0.5, 0.5, -3.0], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=90.0, width=100, height=100)
    b = dict(want_mode=0, max_depth=40, variation_tau=-1.0, target_px=1.0, density_scale=1.0, max_tets=1 << 20)
    d = np.ones(8 ** 3, np.float32)
    d[0] = 2.0  # mean > 0 and variation > -1 everywhere
    # a depth-0 root: longest edge = sqrt(3); centroid distance known
    e = oracle.leb_build(d, 8, cam, dict(b, want_mode=1, uniform_depth=0)).export()
    verts, ids = e["verts"], e["ids"]
    depth = np.zeros(len(ids), np.int32)
    c = verts.astype(np.float64).mean(1) / S
    z = np.linalg.norm(c - np.array(cam["pos"]), axis=1)
    l = math.sqrt(3.0)
    assert (z > l).all()  # camera outside every tet's bounding sphere
    kpx = 50.0 / math.tan(math.radians(45.0))
    proj = l * kpx / z
    for tgt in [proj.min() * 0.999, proj.max() * 1.001]:
        w = oracle.want(d, 8, cam, dict(b, target_px=float(tgt)), verts, depth, ids)
        assert np.array_equal(w, proj > tgt)
    # same tets with the camera looking away: behind it, never wanted
    away = dict(cam, look_at=[0.5, 0.5, -4.0])
    w = oracle.want(d, 8, away, dict(b, target_px=1e-6), verts, depth, ids)
    assert not w.any()


def test_capacity_and_bad_input(dens64):
    assert oracle.leb_build_status(dens64, 64, TINY["camera"], dict(TINY["build"], max_tets=1000)) == -3
    bad = dens64.copy()
    bad[5] = np.nan
    assert oracle.leb_build_status(bad, 64, TINY["camera"], TINY["build"]) == -5
    bad[5] = -1.0
    assert oracle.leb_build_status(bad, 64, TINY["camera"], TINY["build"]) == -5
    assert oracle.leb_build_status(dens64[:1000], 10, TINY["camera"], TINY["build"]) == -1


# ---------------------------------------------------------------- criteria and per-tet medium
# A camera for which the camera criterion holds for every tet of the cube: far
# enough that the whole cube sits inside the frustum, and a target size no tet
# falls below, so want = (depth < max depth) and the density variation alone.
WIDE = dict(pos=[0.5, 0.5, -3.0], look_at=[0.5, 0.5, 0.5], up=[0, 1, 0], fov_y_deg=60.0, width=64, height=64)


def open_box_voxels(G, v):
    """The voxels of G ([k][j][i], n^3) overlapping the open bounding box of
    the tet with lattice vertices v (4 x 3): voxel i spans [i, i+1) * S/n on
    each axis and overlaps (lo, hi) iff i S/n < hi and (i+1) S/n > lo."""
    n = G.shape[0]
    vs = S // n
    idx = np.arange(n)
    sel = []
    for a in range(3):
        lo, hi = int(v[:, a].min()), int(v[:, a].max())
        sel.append(np.flatnonzero((idx * vs < hi) & ((idx + 1) * vs > lo)))
    return G[np.ix_(sel[2], sel[1], sel[0])]


def test_variation_predicate_on_hand_built_volumes():
    """Density variation (Subdivision Criteria): a tet is split iff max D -
    min D > tau * mean D with mean D > 0.  Roots span the whole cube, so D is
    the whole volume: half the voxels 0.5 and half 1.5 give mean 1 and
    max - min = 1 exactly, which puts tau = 1 on the boundary (strict >)."""
    n = 8
    e = oracle.leb_build(np.ones(n ** 3, np.float32), n, WIDE, dict(want_mode=1, uniform_depth=0, max_tets=64)).export()
    verts, ids = e["verts"], e["ids"]
    depth = np.zeros(len(ids), np.int32)
    b = dict(want_mode=0, max_depth=30, target_px=1e-6, density_scale=1.0, max_tets=1 << 20)

    def w(d, tau):
        return oracle.want(d, n, WIDE, dict(b, variation_tau=tau), verts, depth, ids)

    half = np.where(np.arange(n ** 3) % 2 == 0, 0.5, 1.5).astype(np.float32)
    assert w(half, 1.0 - 2.0 ** -40).all()
    assert not w(half, 1.0).any()  # equal is not "varies above"
    assert not w(half, 1.0 + 2.0 ** -40).any()
    assert w(half, 0.0).all() and w(half, -1.0).all()
    # constant volume: max - min = 0, so only a negative tau splits
    const = np.full(n ** 3, 3.0, np.float32)
    assert not w(const, 0.0).any() and w(const, -1e-9).all()
    # an empty volume (mean 0) is never split, whatever tau
    zero = np.zeros(n ** 3, np.float32)
    assert not w(zero, -1.0).any() and not w(zero, 0.0).any()
    # one hot voxel of value 512 among zeros: mean 1, max - min = 512
    hot = zero.copy()
    hot[137] = 512.0
    assert w(hot, 511.999).all() and not w(hot, 512.0).any()
    # the same predicate with max depth reached: never split
    assert not oracle.want(half, n, WIDE, dict(b, variation_tau=0.0, max_depth=0), verts, depth, ids).any()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_variation_predicate_against_brute_force(seed):
    """Every tet of uniform grids at depths 0-10 on integer-valued volumes
    (sums exact in any order): the oracle's split decision equals max - min >
    tau * mean over the voxels of the tet's open bounding box, mean > 0."""
    rng = np.random.default_rng(seed)
    n = 16
    d = (rng.integers(0, 8, n ** 3) * (rng.random(n ** 3) < 0.6)).astype(np.float32)
    d[: n * n * 3] = 0.0  # a slab of empty voxels: mean-0 boxes
    G = d.reshape(n, n, n)
    b = dict(want_mode=0, max_depth=40, target_px=1e-6, density_scale=1.0, max_tets=1 << 20)
    checked = 0
    for depth in range(0, 11):
        e = oracle.leb_build(d, n, WIDE, dict(want_mode=1, uniform_depth=depth, max_tets=1 << 16)).export()
        verts, ids = e["verts"], e["ids"]
        dep = np.full(len(ids), depth, np.int32)
        stats = [(float(B.max()) - float(B.min()), float(B.sum()) / B.size)
                 for B in (open_box_voxels(G, v) for v in verts)]
        for tau in (0.0, 0.5, 1.0, 2.5):
            got = oracle.want(d, n, WIDE, dict(b, variation_tau=tau), verts, dep, ids)
            want = np.array([m > 0 and r > tau * m for r, m in stats])
            assert np.array_equal(got, want), f"depth {depth} tau {tau}: {np.flatnonzero(got != want)[:5]}"
            checked += len(ids)
    assert checked > 20000


@pytest.mark.parametrize("n,scale", [(8, 1.0), (16, 0.37), (16, 2.5)])
def test_sigma_and_loose_majorant_at_coarse_depths(n, scale):
    """One density value per tet (Volumetric Path Tracing): sigma = scale *
    mean of D(T), and in loose mode the majorant = scale * max of D(T), over
    the voxels of the tet's open bounding box, at depths from the roots to
    voxel size and one level below, rounded once to FP32 (up to 2000 tets a
    depth)."""
    rng = np.random.default_rng(n + int(scale * 100))
    d = (rng.integers(0, 16, n ** 3) * (rng.random(n ** 3) < 0.7)).astype(np.float32)
    G = d.reshape(n, n, n)
    vox = 3 * int(math.log2(n))
    for depth in sorted(set(range(0, vox, 2)) | {vox - 1, vox, vox + 1}):
        b = dict(want_mode=1, uniform_depth=depth, density_scale=scale, majorant_mode=1, max_tets=1 << 20)
        e = oracle.leb_build(d, n, WIDE, b).export()
        pick = rng.permutation(len(e["ids"]))[:2000]
        e = {k: e[k][pick] for k in ("verts", "sigma", "majorant")}
        boxes = [open_box_voxels(G, v) for v in e["verts"]]
        sc = np.float64(np.float32(scale))  # the scale is an FP32 parameter
        sig = np.array([np.float32(sc * (float(B.sum()) / B.size)) for B in boxes], np.float32)
        maj = np.array([np.float32(sc * float(B.max())) for B in boxes], np.float32)
        assert np.array_equal(e["sigma"].view(np.uint32), sig.view(np.uint32)), f"sigma at depth {depth}"
        assert np.array_equal(e["majorant"].view(np.uint32), maj.view(np.uint32)), f"majorant at depth {depth}"
        assert (e["sigma"] <= e["majorant"]).all()
        tight = oracle.leb_build(d, n, WIDE, dict(b, majorant_mode=0)).export()
        assert np.array_equal(tight["majorant"][pick].view(np.uint32), sig.view(np.uint32))


def test_sigma_of_real_valued_volume_within_rounding():
    """The same definition on a real-valued volume: sigma within FP32
    rounding of the exact box mean (the FP64 sum's order is the oracle's
    own), and the loose majorant exact."""
    rng = np.random.default_rng(5)
    n = 16
    d = (rng.random(n ** 3) * 7.0 * (rng.random(n ** 3) < 0.5)).astype(np.float32)
    G = d.reshape(n, n, n)
    for depth in (1, 4, 7, 11):
        e = oracle.leb_build(d, n, WIDE, dict(want_mode=1, uniform_depth=depth, density_scale=1.0,
                                              majorant_mode=1, max_tets=1 << 20)).export()
        for v, s, m in zip(e["verts"], e["sigma"], e["majorant"]):
            B = open_box_voxels(G, v)
            exact = float(sum(Fraction(float(x)) for x in B.ravel()) / B.size)
            assert abs(float(s) - exact) <= 2 ** -23 * abs(exact) + 1e-30
            assert m == B.max()
