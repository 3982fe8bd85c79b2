"""The tracer's device elementary functions against their definitions.

Free-path sampling (-ln(1 - u)), transmittance (e^-x), the scattered
direction's azimuth (cos, sin of 2 pi u) and the Henyey-Greenstein density
and inverse CDF (Algorithm 1's free-path and phase-function sampling) are,
by definition, the exact functions.  The device evaluates each in FP64 and
rounds once to FP32, so it must return the correctly rounded value -- the
FP64 definition rounded to FP32 -- except where the exact value sits within
~1e-16 of a rounding midpoint.  The HG formulas use only IEEE operations,
so they must agree bit for bit with the same FP64 formula here.
"""
import math
import sys

import numpy as np
import pytest

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


def ulps(a, b):
    """Distance in FP32 units in the last place (same-sign finite values)."""
    ia = a.astype(np.float32).view(np.int32).astype(np.int64)
    ib = b.astype(np.float32).view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


def assert_correctly_rounded(got, exact64, what, max_miss=1e-6):
    ref = exact64.astype(np.float32)
    d = ulps(got, ref)
    miss = float((d != 0).mean())
    say(f"  {what}: {len(got)} values, {miss * 100:.5f}% not correctly rounded, max {d.max()} ulp")
    assert d.max() <= 1, what
    assert miss <= max_miss, what


# uniforms are multiples of 2^-24 in [0, 1)
U = np.concatenate([np.arange(0, 1 << 24, 13), np.arange(0, 4096), (1 << 24) - np.arange(1, 4097)]) / float(1 << 24)
U = np.unique(U).astype(np.float32)


def test_neglog1m(tv):
    say("case device -ln(1 - u)")
    got = tv.eval_functions("neglog1m", U)
    exact = -np.log1p(-U.astype(np.float64))
    assert got[U == 0.0][0] == 0.0
    assert_correctly_rounded(got, exact, "-ln(1 - u)")


def test_expneg(tv):
    say("case device e^-x")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(0, 110, 1 << 20), rng.uniform(0, 1e-3, 1 << 16), rng.uniform(100, 106, 1 << 16),
                        [0.0, 1e-30, 0.3465, 87.0, 103.9, 104.0, 1e4]]).astype(np.float32)
    got = tv.eval_functions("expneg", x)
    exact = np.exp(-x.astype(np.float64))
    assert got[x == 0.0][0] == 1.0 and got[x >= 104.0].max() == 0.0
    assert_correctly_rounded(got, exact, "e^-x")


def test_sincos2pi(tv):
    say("case device (cos, sin)(2 pi u)")
    rng = np.random.default_rng(2)
    u = np.concatenate([U, rng.random(1 << 18).astype(np.float32)])
    got = tv.eval_functions("sincos2pi", u)
    a = 2.0 * math.pi * u.astype(np.float64)
    c, s = np.cos(a), np.sin(a)
    # at u = k/4 the device reduces exactly and returns an exact 0 where the
    # FP64 argument 2 pi u, itself rounded, gives a value of order 1e-16
    for k, (ce, se) in enumerate([(1, 0), (0, 1), (-1, 0), (0, -1)]):
        i = np.flatnonzero(u == np.float32(k / 4))
        if len(i):
            assert got[i[0], 0] == ce and got[i[0], 1] == se
    keep = (np.abs(c) > 1e-12) & (np.abs(s) > 1e-12)
    assert_correctly_rounded(got[keep, 0], c[keep], "cos 2 pi u")
    assert_correctly_rounded(got[keep, 1], s[keep], "sin 2 pi u")


def test_hg_functions_bitexact(tv):
    say("case device HG density and inverse CDF")
    rng = np.random.default_rng(3)
    n = 1 << 18
    g = np.concatenate([rng.uniform(-0.99, 0.99, n), np.full(4096, 0.3), np.full(4096, 5e-4),
                        np.full(4096, -0.9)]).astype(np.float32)
    a = np.concatenate([rng.uniform(-1, 1, n), np.linspace(-1, 1, 4096), np.linspace(-1, 1, 4096),
                        np.linspace(-1, 1, 4096)]).astype(np.float32)
    gd, md = g.astype(np.float64), a.astype(np.float64)
    g2 = gd * gd
    den = (1.0 + g2) - (2.0 * gd) * md
    pdf = ((1.0 - g2) / (((4.0 * math.pi) * den) * np.sqrt(den))).astype(np.float32)
    got = tv.eval_functions("hg_pdf", a, g)
    assert np.array_equal(got.view(np.uint32), pdf.view(np.uint32))
    u = ((a + 1.0) * 0.5).astype(np.float32)
    ud = u.astype(np.float64)
    sv = (1.0 - g2) / ((1.0 - gd) + (2.0 * gd) * ud)
    mu = np.where(np.abs(gd) < 1e-3, 2.0 * ud - 1.0, ((1.0 + g2) - sv * sv) / (2.0 * gd))
    mu = np.clip(mu, -1.0, 1.0).astype(np.float32)
    got = tv.eval_functions("hg_mu", u, g)
    assert np.array_equal(got.view(np.uint32), mu.view(np.uint32))
    # the inverse CDF inverts the CDF of the density: E[mu] = g
    for gv in (0.3, -0.6, 0.9):
        uu = ((np.arange(1 << 16) + 0.5) / (1 << 16)).astype(np.float32)
        m = tv.eval_functions("hg_mu", uu, np.float32(gv)).astype(np.float64)
        assert abs(m.mean() - gv) < 2e-4


def test_bad_arguments(tv):
    import ctypes
    lib = tv.lib()
    out = np.empty(4, np.float32)
    x = np.zeros(4, np.float32)
    assert lib.tet_eval_functions(7, 4, x.ctypes.data, None, out.ctypes.data, 0, None) == -1
    assert lib.tet_eval_functions(3, 4, x.ctypes.data, None, out.ctypes.data, 0, None) == -1
    assert lib.tet_eval_functions(0, -1, x.ctypes.data, None, out.ctypes.data, 0, None) == -1
    assert lib.tet_eval_functions(0, 0, None, None, None, 0, ctypes.c_void_p()) == 0
