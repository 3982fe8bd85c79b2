"""GPU: calls on different threads and streams at the same time.  The
library's device-memory cache hands a freed block only to the thread that
freed it (a call may free scratch whose kernels are still queued on its own
stream), so a build on one thread and stream running while another thread
renders on another stream must give exactly the grid and image each gives
alone: grids bit for bit, images up to the order in which FP32 sample values
are summed per pixel."""
import sys
import threading

import numpy as np
import pytest

import synthetic

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


def grid_arrays(g):
    e = g.export()
    return {k: e[k].copy() for k in ("ids", "nbr", "verts", "sigma", "majorant")}


def test_build_and_render_on_two_threads(tv):
    import torch
    sc = synthetic.scene("blobs_adaptive")
    d = torch.from_numpy(sc["density_fn"]()).cuda()
    cams = [dict(sc["camera"], width=256, height=256),
            dict(sc["camera"], pos=[1.4, 0.6, -0.3], width=256, height=256)]
    torch.cuda.synchronize()
    # each call alone
    ref_grids, ref_imgs = [], []
    for cam in cams:
        g = tv.leb_build(d, sc["n"], cam, build=sc["build"])
        ref_grids.append(grid_arrays(g))
        img, _ = tv.render(g, cam, sc["medium"], sc["light"], 16, 5, sc["render"])
        ref_imgs.append(img.cpu().numpy())
    # renders of one grid while another thread builds the other camera's grid,
    # both directions, several times (freed blocks are reused)
    sA, sB = torch.cuda.Stream(), torch.cuda.Stream()
    g0 = tv.leb_build(d, sc["n"], cams[0], build=sc["build"])
    for rep in range(4):
        k = rep % 2
        box = {}

        def build():
            with torch.cuda.stream(sB):
                box["g"] = tv.leb_build(d, sc["n"], cams[1 - k], build=sc["build"])
                torch.cuda.current_stream().synchronize()

        th = threading.Thread(target=build)
        th.start()
        with torch.cuda.stream(sA):
            img, _ = tv.render(g0, cams[k], sc["medium"], sc["light"], 16, 5, sc["render"])
            torch.cuda.current_stream().synchronize()
        th.join()
        say(f"case concurrent build + render, repetition {rep}")
        got = img.cpu().numpy().astype(np.float64)
        want = ref_imgs[k].astype(np.float64)
        rel = np.abs(got - want).max() / np.abs(want).max()
        assert rel <= 1e-5, f"repetition {rep}: image differs by {rel:.3g}"
        other = grid_arrays(box["g"])
        for key, a in ref_grids[1 - k].items():
            b = other[key]
            eq = (a.view(np.uint32) == b.view(np.uint32)) if key in ("sigma", "majorant") else (a == b)
            assert eq.all(), f"repetition {rep}: {key} of the concurrent build differs"
        g0 = box["g"]
