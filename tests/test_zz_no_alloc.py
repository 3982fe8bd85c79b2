"""tet_render_noalloc: the render for callers that cannot allocate device
memory.  Called through the C ABI, its images must match tet_render's on
the same grid, camera and seed (the parity bar), call after call on the
shared fixed scratch -- the second call smaller than the first, then calls
that need several passes and the largest image the scratch holds -- and it
must refuse what it cannot do before launching anything."""
import ctypes
import sys

import pytest

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


def noalloc(tv, g, cam, sc, spp, seed, ropts, out):
    """One call of tet_render_noalloc through ctypes; returns its status."""
    from paper_2506_11510_amd import _abi
    import torch
    c = _abi.make_camera(cam)
    rc = tv.lib().tet_render_noalloc(g.handle, ctypes.byref(c), ctypes.byref(_abi.make_medium(sc["medium"])),
                                     ctypes.byref(_abi.make_light(sc["light"])), int(spp), int(seed),
                                     ctypes.byref(_abi.make_render_opts(ropts)), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc


def test_noalloc_matches_render(tv):
    import torch
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]()
    g = tv.leb_build(torch.from_numpy(d).cuda(), 64, sc["camera"], build=sc["build"])
    cases = [  # (width, height, spp, seed, options): large, then smaller, then several passes
        (96, 80, 12, 5, dict(sc["render"])),
        (24, 20, 3, 6, dict(sc["render"], transmittance=1)),
        (1024, 1024, 5, 7, dict(sc["render"], samples_per_item=1)),
        (2048, 1024, 2, 9, dict(sc["render"])),  # the largest image: one sample per pixel fills the array
        (33, 17, 4, 8, dict(sc["render"], record_layout=48)),
    ]
    for w, h, spp, seed, r in cases:
        say(f"case noalloc {w}x{h} spp {spp} seed {seed}")
        cam = dict(sc["camera"], width=w, height=h)
        out = torch.full((h, w, 3), -1.0, dtype=torch.float32, device="cuda")
        assert noalloc(tv, g, cam, sc, spp, seed, r, out) == 0, tv.lib().tet_last_error()
        ref, _ = tv.render(g, cam, sc["medium"], sc["light"], spp, seed, r)
        assert_image_parity(out.cpu().numpy(), ref.cpu().numpy(), f"noalloc {w}x{h}")
        assert float(out.min()) >= 0.0


def test_noalloc_refusals(tv):
    import torch
    from paper_2506_11510_amd import _abi
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]()
    g = tv.leb_build(torch.from_numpy(d).cuda(), 64, dict(sc["camera"]), build=dict(sc["build"], uniform_depth=4))
    # one sample of every pixel must fit the fixed scratch: 2048^2 does not
    cam = dict(sc["camera"], width=2048, height=2048)
    out = torch.empty((1, 1, 3), dtype=torch.float32, device="cuda")
    say("case noalloc refusals")
    assert noalloc(tv, g, cam, sc, 1, 1, sc["render"], out) == _abi.TET_ERR_CAPACITY
    assert b"fixed scratch" in tv.lib().tet_last_error()
    # a NULL output and a radiance cache are refused before any launch
    c = _abi.make_camera(dict(sc["camera"], width=8, height=8))
    rc = tv.lib().tet_render_noalloc(g.handle, ctypes.byref(c), ctypes.byref(_abi.make_medium(sc["medium"])),
                                     ctypes.byref(_abi.make_light(sc["light"])), 1, 1, None, None, None)
    assert rc == _abi.TET_ERR_INVALID_ARG
    n = tv.Nrc(dict(sigma_ref=10.0))
    r = _abi.make_render_opts(dict(sc["render"]))
    r.nrc = n.handle
    out = torch.empty((8, 8, 3), dtype=torch.float32, device="cuda")
    rc = tv.lib().tet_render_noalloc(g.handle, ctypes.byref(c), ctypes.byref(_abi.make_medium(sc["medium"])),
                                     ctypes.byref(_abi.make_light(sc["light"])), 1, 1, ctypes.byref(r),
                                     ctypes.c_void_p(out.data_ptr()), None)
    assert rc == _abi.TET_ERR_UNSUPPORTED
    assert tv.lib().tet_render_noalloc(None, ctypes.byref(c), ctypes.byref(_abi.make_medium(sc["medium"])),
                                       ctypes.byref(_abi.make_light(sc["light"])), 1, 1, None,
                                       ctypes.c_void_p(out.data_ptr()), None) == _abi.TET_ERR_INVALID_ARG
