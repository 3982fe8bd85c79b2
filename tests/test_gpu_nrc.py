"""GPU parity of the radiance cache (an addition to the paper's method):
the HIP path through the C ABI against the CPU oracle on the same seeded
inputs.

Tolerances.  The GPU network rounds every matrix-product operand to
bfloat16 and accumulates in FP32; the oracle's BF16-operand mode rounds the
same operands and sums exactly.  The two differ (a) by FP32 accumulation
(~1e-6 relative) and (b) where an operand lies within that distance of a
bfloat16 rounding boundary, so that the two sides round it one bfloat16
unit (2^-8 relative) apart; the features add a third such source, the GPU's
FP32 sine/cosine (error < 5e-7) against FP64.  A flip moves the outputs by
at most the flipped value's share times 2^-8, so: all outputs within
2^-6 of the output scale, and nearly all (where nothing flipped) within
1e-4 of it.  Networks whose every operand is exactly representable leave
no rounding to disagree on: there the GPU must match bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from parity import assert_image_parity, rel_errors

pytestmark = pytest.mark.gpu
NP = oracle.N_PARAMS


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


TINY = synthetic.scene("tiny")


@pytest.fixture(scope="module")
def tiny(tv):
    import torch
    d = TINY["density_fn"]()
    g = tv.leb_build(torch.from_numpy(d).cuda(), 64, TINY["camera"], build=TINY["build"])
    o = oracle.leb_build(d, 64, TINY["camera"], TINY["build"])
    return g, o


def rand_params(seed, scale=1.0):
    """He-like random weights and small random biases."""
    rng = np.random.default_rng(seed)
    P = np.zeros(NP, np.float32)
    dims = [76, 64, 64, 64, 64, 3]
    o = 0
    for l in range(5):
        fi, fo = dims[l], dims[l + 1]
        P[o:o + fo * fi] = rng.normal(0, scale * np.sqrt(2.0 / fi), fo * fi)
        P[o + fo * fi:o + fo * fi + fo] = rng.normal(0, 0.1, fo)
        o += fo * fi + fo
    return P


def sparse_int_params(seed):
    """Weights in {-1, 0, 1} (few per row) and integer biases: every
    operand, activation and error of the network is a small integer."""
    rng = np.random.default_rng(seed)
    P = np.zeros(NP, np.float32)
    dims = [76, 64, 64, 64, 64, 3]
    o = 0
    for l in range(5):
        fi, fo = dims[l], dims[l + 1]
        W = np.zeros((fo, fi), np.float32)
        nnz = 8 if l == 0 else 2
        for r in range(fo):
            W[r, rng.choice(fi, nnz, replace=False)] = rng.choice([-1.0, 1.0], nnz)
        P[o:o + fo * fi] = W.ravel()
        P[o + fo * fi:o + fo * fi + fo] = rng.integers(-2, 3, fo)
        o += fo * fi + fo
    return P


def rand_points(seed, n, sigma_max=20.0):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    s = (rng.random(n) * sigma_max).astype(np.float32)
    s[::7] = 0.0
    return pos, d, s


def out_errors(y, ref):
    y = np.asarray(y, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = float(np.sqrt((ref ** 2).mean()))
    return np.abs(y - ref) / scale


def assert_bf16_parity(y, ref, what):
    e = out_errors(y, ref)
    near = float((e <= 1e-4).mean())
    say(f"  {what}: max {e.max():.3g} x scale, {near * 100:.2f}% within 1e-4")
    assert e.max() <= 2 ** -6, f"{what}: max error {e.max():.3g} of the output scale"
    assert near >= 0.95, f"{what}: only {near * 100:.2f}% within 1e-4 of the scale"


def test_params_roundtrip(tv):
    say("case nrc export/import")
    n = tv.Nrc(dict(seed=3))
    p0 = n.export()
    assert p0.shape == (NP,) and np.isfinite(p0).all()
    # He-uniform init: |w| <= sqrt(6 / fan_in), biases zero
    assert np.abs(p0[:4864]).max() <= np.sqrt(6 / 76) and (p0[4864:4928] == 0).all()
    P = rand_params(1)
    n.load(P)
    assert np.array_equal(n.export(), P)
    assert n.info()["adam_steps"] == 0


@pytest.mark.parametrize("count", [1, 64, 200, 4097])
def test_exact_on_representable_network(tv, count):
    """Integer network, 0/1 features, integer output gradients: outputs and
    gradients bit-exact (checks the fragment layouts, the unit
    permutation between layers and the transposed backward weights)."""
    say(f"case nrc exact integer network, {count} samples")
    P = sparse_int_params(7)
    rng = np.random.default_rng(count)
    x = rng.integers(0, 2, (count, 76)).astype(np.float32)
    dy = rng.integers(-1, 2, (count, 3)).astype(np.float32)
    n = tv.Nrc(dict(sigma_ref=1.0))
    n.load(P)
    y, g = n.forward_backward(x, dy)
    yo, go = oracle.mlp_backward(P.astype(np.float64), x.astype(np.float64), dy.astype(np.float64), bf16=True)
    assert np.abs(yo).max() > 4
    assert np.array_equal(y.cpu().numpy().astype(np.float64), yo)
    gg = g.cpu().numpy().astype(np.float64)
    bad = np.flatnonzero(gg != go)
    assert bad.size == 0, f"{bad.size} gradients differ, first at {bad[:8].tolist()}"


def test_infer_matches_oracle(tv):
    say("case nrc infer vs oracle")
    P = rand_params(2)
    n = tv.Nrc(dict(sigma_ref=20.0))
    n.load(P)
    pos, d, s = rand_points(3, 3000)
    y = n.infer(pos, d, s).cpu().numpy()
    x = oracle.nrc_encode(pos, d, s, 20.0).astype(np.float64)
    yo = oracle.mlp_forward(P.astype(np.float64), x, bf16=True)
    assert_bf16_parity(y, yo, "infer")


def test_forward_backward_matches_oracle(tv):
    say("case nrc forward/backward vs oracle")
    P = rand_params(4)
    pos, d, s = rand_points(5, 1000)
    x = oracle.nrc_encode(pos, d, s, 20.0)
    dy = np.random.default_rng(6).normal(size=(1000, 3)).astype(np.float32)
    n = tv.Nrc(dict(sigma_ref=20.0))
    n.load(P)
    y, g = n.forward_backward(x, dy)
    yo, go = oracle.mlp_backward(P.astype(np.float64), x.astype(np.float64), dy.astype(np.float64), bf16=True)
    assert_bf16_parity(y.cpu().numpy(), yo, "forward")
    gg = g.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    e = np.abs(gg - go) / np.sqrt((go ** 2).mean())
    say(f"  gradients: normwise {rel:.3g}, max {e.max():.3g} x rms, {(e <= 1e-3).mean() * 100:.2f}% within 1e-3")
    assert rel <= 2 ** -6
    assert (e <= 1e-3).mean() >= 0.95


def test_adam_steps_match_oracle(tv):
    """Two Adam steps on one batch: the loss, and every update where the
    gradient is clearly nonzero (the first step moves each parameter by
    lr * sign(g), so near-zero gradients, whose sign the BF16 rounding may
    flip, are left out)."""
    say("case nrc adam vs oracle")
    P = rand_params(8, scale=0.5)
    pos, d, s = rand_points(9, 2048)
    t = np.abs(np.random.default_rng(10).normal(0.5, 0.3, (2048, 3))).astype(np.float32)
    n = tv.Nrc(dict(sigma_ref=20.0, lr=1e-3))
    n.load(P)
    x = oracle.nrc_encode(pos, d, s, 20.0).astype(np.float64)
    Po = P.astype(np.float64)
    m = np.zeros(NP)
    v = np.zeros(NP)
    prev = P.astype(np.float64)
    for step in (1, 2):
        loss = n.train_batch(pos, d, s, t)
        yo = oracle.mlp_forward(prev, x, bf16=True)
        loss_o, dyo = oracle.nrc_loss_grad(yo, t.astype(np.float64))
        _, go = oracle.mlp_backward(prev, x, dyo, bf16=True)
        Po = prev.copy()
        oracle.adam_step(Po, go, m, v, step, lr=1e-3, beta1=0.9, beta2=0.99, eps=1e-8)
        cur = n.export().astype(np.float64)
        say(f"  step {step}: loss {loss:.6g} vs {loss_o:.6g}")
        assert loss == pytest.approx(loss_o, rel=2 ** -6)
        sig = np.abs(go) > 0.05 * np.sqrt((go ** 2).mean())
        du, duo = cur - prev, Po - prev
        err = np.abs(du - duo)[sig]
        say(f"  step {step}: {sig.sum()} clear gradients, worst update error {err.max():.3g} (lr 1e-3)")
        assert err.max() <= 1e-4 * 1e-3 + 2e-4 * np.abs(duo[sig]).max()
        assert n.info()["adam_steps"] == step
        prev = cur


def test_collect_matches_oracle(tv, tiny):
    """Training records: same paths (Philox streams), so records match the
    oracle's bit for bit except on the rare path whose FP32 decisions
    differ."""
    say("case nrc collect vs oracle")
    g, o = tiny
    cam = dict(TINY["camera"], width=48, height=40)
    n = tv.Nrc(dict(train_paths=3000, train_vertices=4, sigma_ref=10.0))
    ro = dict(max_bounces=8)
    r = n.collect(g, cam, TINY["medium"], TINY["light"], 11, ro)
    ro_ = o.nrc_collect(cam, TINY["medium"], TINY["light"], 11, 3000, 4, ro, threads=8)
    say(f"  {len(r['tag'])} records vs {len(ro_['tag'])}")
    assert len(r["tag"]) > 1000
    common, ia, ib = np.intersect1d(r["tag"], ro_["tag"], return_indices=True)
    assert len(common) >= 0.99 * len(ro_["tag"])
    same = np.ones(len(common), bool)
    for k in ("pos", "dir", "sigma", "target"):
        a, b = r[k][ia].reshape(len(common), -1), ro_[k][ib].reshape(len(common), -1)
        same &= (a.view(np.uint32) == b.view(np.uint32)).all(axis=1)
    say(f"  {same.mean() * 100:.3f}% of common records bit-exact")
    assert same.mean() >= 0.99
    assert np.array_equal(np.sort(r["tag"]), r["tag"])  # (path, vertex) order


def test_truncated_render_constant_cache_parity(tv, tiny):
    """A cache returning a constant (all weights 0, output bias c) is exact
    on both sides, so the truncated render meets the plain image bar."""
    say("case nrc truncated render, constant cache")
    g, o = tiny
    cam = dict(TINY["camera"], width=40, height=36)
    P = np.zeros(NP, np.float32)
    P[-3:] = [0.5, 0.25, 0.125]
    n = tv.Nrc(dict(sigma_ref=10.0, truncate_bounce=2))
    n.load(P)
    ro = dict(TINY["render"], max_bounces=8)
    img, st = tv.render(g, cam, TINY["medium"], TINY["light"], 8, 21, dict(ro, nrc=n))
    ref, _ = o.nrc_render(cam, TINY["medium"], TINY["light"], 8, 21, P.astype(np.float64), ro, truncate_bounce=2,
                          sigma_ref=10.0, bf16=True, threads=8)
    assert st["cache_ms"] > 0
    assert_image_parity(img.cpu().numpy(), ref, "constant cache")


def test_truncated_render_random_cache(tv, tiny):
    """Random network: the cache term carries the BF16 tolerance, the rest
    of the estimate the plain bar; per pixel within 2^-6 relative."""
    say("case nrc truncated render, random cache")
    g, o = tiny
    cam = dict(TINY["camera"], width=40, height=36)
    P = rand_params(12, scale=0.5)
    n = tv.Nrc(dict(sigma_ref=10.0, truncate_bounce=2))
    n.load(P)
    ro = dict(TINY["render"], max_bounces=8)
    img, st = tv.render(g, cam, TINY["medium"], TINY["light"], 8, 22, dict(ro, nrc=n))
    ref, _ = o.nrc_render(cam, TINY["medium"], TINY["light"], 8, 22, P.astype(np.float64), ro, truncate_bounce=2,
                          sigma_ref=10.0, bf16=True, threads=8)
    rel = rel_errors(img.cpu().numpy(), ref)
    say(f"  per-pixel: max {rel.max():.3g}, mean {rel.mean():.3g}, {(rel <= 1e-4).mean() * 100:.2f}% within 1e-4")
    assert rel.max() <= 2 ** -6 and (rel <= 1e-4).mean() >= 0.5


def test_furnace_with_exact_cache_is_one(tv, tiny):
    say("case nrc furnace")
    g, _ = tiny
    cam = dict(TINY["camera"], width=32, height=32)
    P = np.zeros(NP, np.float32)
    P[-3:] = 1.0
    n = tv.Nrc(dict(sigma_ref=10.0))
    n.load(P)
    light = dict(sun_dir=[0.0, 1.0, 0.0], sun_irradiance=[0.0, 0.0, 0.0], env_radiance=[1.0, 1.0, 1.0])
    img, st = tv.render(g, cam, dict(albedo=1.0, g=0.5), light, 8, 3, dict(max_bounces=1 << 20, nrc=n))
    assert st["real_collisions"] > 1000
    assert (img.cpu().numpy() == 1.0).all()


def test_trained_cache_lowers_error(tv):
    """Online training pays: on a thick, bright medium the render truncated
    at vertex 2 with a trained cache is closer to a converged plain render
    than the plain render at the same samples per pixel, at fewer tet steps,
    and much closer than with the untrained cache."""
    say("case nrc gain")
    import torch
    sc = synthetic.scene("tiny")
    d = sc["density_fn"]() * 2.0
    g = tv.leb_build(torch.from_numpy(d).cuda(), 64, sc["camera"], build=sc["build"])
    cam = dict(sc["camera"], width=64, height=64)
    med = dict(albedo=0.95, g=0.3)
    light = sc["light"]
    ro = dict(max_bounces=64)
    ref, _ = tv.render(g, cam, med, light, 4096, 100, ro)
    ref = ref.cpu().numpy().astype(np.float64)
    rmse = lambda img: float(np.sqrt(((img.cpu().numpy() - ref) ** 2).mean()))
    n = tv.Nrc(dict(train_paths=8192, train_steps=4, lr=3e-3))
    plain, sp = tv.render(g, cam, med, light, 4, 7, ro)
    n.train_frame(g, cam, med, light, 1, ro)  # first frame sets sigma_ref; reset to the untrained weights
    n.load(tv.Nrc(dict(seed=n.info()["seed"])).export())
    untrained, _ = tv.render(g, cam, med, light, 4, 7, dict(ro, nrc=n))
    losses = []
    for f in range(200):
        losses.append(n.train_frame(g, cam, med, light, 1000 + f, ro)["loss"])
    trained, st = tv.render(g, cam, med, light, 4, 7, dict(ro, nrc=n))
    e_p, e_u, e_t = rmse(plain), rmse(untrained), rmse(trained)
    say(f"  rmse plain {e_p:.4g} ({sp['tet_steps']} steps), untrained {e_u:.4g}, trained {e_t:.4g} "
        f"({st['tet_steps']} steps); loss {np.mean(losses[:10]):.4g} -> {np.mean(losses[-10:]):.4g}")
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])
    assert e_t < e_p and e_t < 0.5 * e_u
    assert st["tet_steps"] < sp["tet_steps"]


def test_training_inside_the_render_launch(tv, tiny):
    """nrc_train: the render also traces the frame's training paths (key =
    seed XOR 0x6A09E667F3BCC909) and then trains.  The image is the one the
    pre-call weights give, and the weights after it are those a separate
    training frame with that key gives, bit for bit (same paths, same
    records, same batches)."""
    say("case nrc training inside the render launch")
    g, _ = tiny
    cam = dict(TINY["camera"], width=48, height=40)
    ro = dict(TINY["render"], max_bounces=8)
    P = rand_params(13, scale=0.5)
    a = tv.Nrc(dict(sigma_ref=10.0, train_paths=4000))
    b = tv.Nrc(dict(sigma_ref=10.0, train_paths=4000))
    a.load(P)
    b.load(P)
    seed = 77
    img_plain, _ = tv.render(g, cam, TINY["medium"], TINY["light"], 8, seed, dict(ro, nrc=a))
    img, st = tv.render(g, cam, TINY["medium"], TINY["light"], 8, seed, dict(ro, nrc=a, nrc_train=1))
    sf = b.train_frame(g, cam, TINY["medium"], TINY["light"], seed ^ 0x6A09E667F3BCC909, ro)
    say(f"  records {st['cache_records']} vs {sf['records']}, loss {st['cache_loss']:.5g} vs {sf['loss']:.5g}")
    assert st["cache_records"] == sf["records"] > 1000
    assert st["cache_loss"] == sf["loss"]
    assert np.array_equal(a.export(), b.export())
    assert a.info()["adam_steps"] == b.info()["adam_steps"] == 4
    x, y = img.cpu().numpy().astype(np.float64), img_plain.cpu().numpy().astype(np.float64)
    assert np.abs(x - y).max() <= 1e-5 * max(np.abs(y).max(), 1e-30)


def test_weight_average_matches_oracle(tv):
    """Queries use the bias-corrected average of the weights after each Adam
    step (ema 0.9 here); it equals the oracle's average of the exported
    master weights to FP32 rounding."""
    say("case nrc weight average")
    P = rand_params(15, scale=0.5)
    pos, d, s = rand_points(16, 1024)
    t = np.abs(np.random.default_rng(17).normal(0.5, 0.3, (1024, 3))).astype(np.float32)
    n = tv.Nrc(dict(sigma_ref=20.0, ema=0.9))
    n.load(P)
    assert np.array_equal(n.export_inference(), P)  # before any step: the weights themselves
    ema = np.zeros(NP)
    for step in range(1, 4):
        n.train_batch(pos, d, s, t)
        want = oracle.ema_step(ema, n.export().astype(np.float64), 0.9, step)
        got = n.export_inference().astype(np.float64)
        err = np.abs(got - want).max() / np.abs(want).max()
        say(f"  step {step}: worst relative difference {err:.3g}")
        assert err <= 1e-6
    # the queries use these weights
    y = n.infer(pos[:256], d[:256], s[:256]).cpu().numpy()
    x = oracle.nrc_encode(pos[:256], d[:256], s[:256], 20.0).astype(np.float64)
    assert_bf16_parity(y, oracle.mlp_forward(n.export_inference().astype(np.float64), x, bf16=True), "averaged infer")
