"""Writes plume1024.json: the oracle's grid and image of the production-scale
smoke plume (1024^3 curl-advected fBm, ~5 % occupancy, sigma_t max 50;
adaptive LEB at a 1-pixel target, tau 0.2, depth <= 30; 1024^2, 64 bounces,
albedo 0.95, HG g 0.6 -- the paper's production-scale workload, "Results"),
for the GPU test that compares the device build with it.

Only the input generator (synthetic/) and the oracle (oracle/) run here.
The oracle's recursive build of the 85.7 M-tet grid takes ~7 minutes and
~55 GB of host memory, too long for the GPU test itself, so the test checks
the device grid against these SHA-256 digests (bit-exact: ids, neighbour
links, vertices, extinction, majorant) and its 32-spp image against the
oracle's render of a strided pixel subset stored here.

Usage: python tests/golden/make_plume1024.py  (from the repository root)
"""
import base64
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synthetic  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plume1024.json")
SEED, SPP, STRIDE = 9, 32, 256


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    sc = synthetic.scene("plume")
    t0 = time.time()
    d = sc["density_fn"]()
    print(f"density {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    g = oracle.leb_build(d, sc["n"], sc["camera"], sc["build"])
    t_build = time.time() - t0
    print(f"oracle build {t_build:.1f} s, {g.num_tets} tets", flush=True)
    rec = {"what": "oracle grid and image of the 1024^3 plume scene (synthetic.scene('plume'))",
           "density_sha256": sha(d), "num_tets": g.num_tets, "max_depth": g.max_depth,
           "oracle_build_s": round(t_build, 1)}
    del d
    e = g.export()
    for k in ("ids", "nbr", "verts", "sigma", "majorant"):
        rec[f"{k}_sha256"] = sha(e[k])
    del e
    pix = np.arange(0, sc["camera"]["width"] * sc["camera"]["height"], STRIDE, dtype=np.int32)
    t0 = time.time()
    img, st = g.render(sc["camera"], sc["medium"], sc["light"], SPP, SEED, sc["render"], pixels=pix,
                       threads=os.cpu_count() or 1)
    print(f"oracle render of {len(pix)} pixels {time.time() - t0:.1f} s", flush=True)
    rec["render"] = {"spp": SPP, "seed": SEED, "pixel_stride": STRIDE, "pixels": int(len(pix)),
                     "tet_steps": int(st["tet_steps"]), "real_collisions": int(st["real_collisions"]),
                     "rgb_f32_le_base64": base64.b64encode(img.astype("<f4").tobytes()).decode()}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
