"""Pins of the sparse-volume input (the paper builds from OpenVDB data):
the oracle's densify (the plain definition: zero outside the listed 8^3
bricks) against direct voxel reads of the brick list and a round trip
through the brick generator (no GPU)."""
import numpy as np

import oracle
import synthetic


def cut(n, seed, keep=0.3):
    d = synthetic.blobs(seed, n).astype(np.float32)
    thr = np.quantile(d, 1.0 - keep)
    return np.where(d > thr, d - thr, 0.0).astype(np.float32)


def test_densify_reads_each_voxel_from_its_brick():
    n = 32
    rng = np.random.default_rng(4)
    nb = n // 8
    pick = rng.choice(nb ** 3, size=20, replace=False)
    coords = np.stack([pick % nb, (pick // nb) % nb, pick // (nb * nb)], axis=1).astype(np.int32)
    values = rng.uniform(0.5, 2.0, (20, 512)).astype(np.float32)
    d = oracle.densify(coords, values, n)
    owner = {tuple(c): b for b, c in enumerate(coords)}
    for _ in range(2000):
        x, y, z = rng.integers(0, n, 3)
        b = owner.get((x // 8, y // 8, z // 8))
        want = 0.0 if b is None else values[b][(x % 8) + 8 * (y % 8) + 64 * (z % 8)]
        assert d[x + n * (y + n * z)] == np.float32(want)
    assert np.count_nonzero(d) == 20 * 512


def test_bricks_round_trip():
    n = 64
    d = cut(n, 2)
    coords, values = synthetic.bricks(d, n, keep_empty=5, seed=9)
    assert coords.shape[1] == 3 and values.shape[1] == 512
    assert len(np.unique(coords, axis=0)) == len(coords)
    assert np.array_equal(oracle.densify(coords, values, n), d)
    # only bricks holding a nonzero voxel, plus the requested empty ones
    nz = (values != 0).any(axis=1)
    assert (~nz).sum() == 5
    assert nz.sum() < (n // 8) ** 3
