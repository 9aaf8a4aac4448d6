"""GPU parity of the learned-sampling kernels with the float64 reference.

Features, targets and probabilities are compared value by value.  The MLP
forward and gradient kernels are compared with the plain float64 network
(``mlp.forward`` / ``mlp.grad`` with ``emulate=False``) evaluated on the same
BF16-rounded weights and inputs (the kernels' operands by definition); no
kernel-side rounding point is copied into the reference.  The tolerance of
every output element is a first-order error bound propagated through the
network from two unit roundoffs only: BF16 (2^-8, for the matrix-core
operands the kernels round: h1, dZ2, dZ1) and FP32 (2^-24, for every sum of n
terms, bounded by gamma_n = n u / (1 - n u) times the sum of magnitudes, in
any order).  A ReLU whose input lies within its own error bound of 0 may
switch either way and is bounded by the full magnitude.  Beside that
worst-case bound, each output block as a whole must stay within 2^-6 (four
BF16 steps) of the plain network in norm: independent roundings do not add
up coherently, while a missing or wrong term would move a block further.
The reference rounded where the kernels round (``emulate=True``) is printed
as a diagnostic only.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1801_00338_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1801_00338_amd import api, learned
    api.lib()
    oracle.build(force=False)
    return torch, api, learned


def _graph(name):
    if name == "er":
        return (2_000, 3_000) + gen.WORKLOADS["er_2k_3k_20k"].edges()
    return (3_000, 15_000) + gen.chung_lu(3_000, 15_000, 150_000, 2.1, 2.3, 2000, seed=7)


U32 = 2.0 ** -24      # FP32 unit roundoff
UB = 2.0 ** -8        # BF16 unit roundoff (8-bit significand, round to nearest)


def _gam(n):
    return n * U32 / (1 - n * U32)


def _plain_params(p):
    """The parameters as the kernels use them: BF16 W1, W2, w3; FP32 biases."""
    W1, b1, W2, b2, w3, b3 = mlp.unpack(np.asarray(p, np.float64))
    return mlp.pack(mlp.bf16(W1), mlp.f32(b1), mlp.bf16(W2), mlp.f32(b2), mlp.bf16(w3),
                    float(mlp.f32(b3)))


def _forward_bound(c, pr):
    """Per-row bound of |y_kernel - y| with the plain cache c (emulate=False).

    z1 = x W1 + b1 is a sum of 9 FP32 terms; h1 = bf16(relu(z1)); z2 a sum of
    65 terms; y = h2 w3 + b3 a sum of 65 terms.  Returns the intermediate
    bounds too (e1 on z1, d1 on h1, e2 on z2 and h2, ey on y).
    """
    W1, b1, W2, b2, w3, b3 = mlp.unpack(pr)
    ax, aW1, aW2, aw3 = np.abs(c["x"]), np.abs(W1), np.abs(W2), np.abs(w3)
    e1 = _gam(9) * (ax @ aW1 + np.abs(b1))
    d1 = e1 + UB * (c["h1"] + e1)
    H1 = c["h1"] + d1
    e2 = d1 @ aW2 + _gam(65) * (H1 @ aW2 + np.abs(b2))
    H2 = c["h2"] + e2
    ey = e2 @ aw3 + _gam(65) * (H2 @ aw3 + abs(b3))
    return dict(e1=e1, d1=d1, H1=H1, e2=e2, H2=H2, ey=ey)


def _grad_bound(c, pr, fb, err, rows):
    """Per-parameter bound of |grad_kernel - grad| (plain back-propagation).

    dy = 2 err / rows (FP32 products); db3, dw3, db2, dW2, db1, dW1 are sums
    over the rows (gamma_{rows + 16}); dZ2 and dZ1 are rounded to BF16 before
    the products dW2 = H1^T dZ2, dH1 = dZ2 W2^T (64 terms) and dW1 = X^T dZ1.
    """
    W1, b1, W2, b2, w3, b3 = mlp.unpack(pr)
    aW2, aw3 = np.abs(W2), np.abs(w3)
    gR = _gam(rows + 16)
    aerr = np.abs(err)
    Eerr = fb["ey"] + U32 * (aerr + fb["ey"])
    Edy = 2.0 / rows * (Eerr + 4 * U32 * (aerr + Eerr))
    Dy = 2.0 / rows * aerr + Edy
    h2, z2, h1, z1 = c["h2"], c["z2"], c["h1"], c["z1"]
    e2, e1 = fb["e2"], fb["e1"]
    out = {}
    out["b3"] = np.atleast_1d(Edy.sum() + gR * Dy.sum())
    out["w3"] = e2.T @ Dy + h2.T @ Edy + _gam(rows + 17) * (fb["H2"].T @ Dy)
    dz2 = (z2 > 0) * np.outer(2.0 * err / rows, w3)
    maybe2 = np.abs(z2) <= e2
    E_dz2 = np.where(maybe2, np.outer(Dy, aw3) * (1 + U32),
                     np.where(z2 > 0, np.outer(Edy, aw3) + U32 * np.outer(Dy, aw3), 0.0))
    DZ2 = np.abs(dz2) + E_dz2
    out["b2"] = E_dz2.sum(axis=0) + gR * DZ2.sum(axis=0)
    E_dz2m = E_dz2 + UB * DZ2
    DZ2m = np.abs(dz2) + E_dz2m
    out["W2"] = fb["d1"].T @ DZ2m + h1.T @ E_dz2m + gR * (fb["H1"].T @ DZ2m)
    dh1 = dz2 @ W2.T
    E_dh1 = E_dz2m @ aW2.T + _gam(64) * (DZ2m @ aW2.T)
    DH1 = np.abs(dh1) + E_dh1
    dz1 = (z1 > 0) * dh1
    maybe1 = np.abs(z1) <= e1
    E_dz1 = np.where(maybe1, DH1, np.where(z1 > 0, E_dh1, 0.0))
    DZ1 = np.abs(dz1) + E_dz1
    out["b1"] = E_dz1.sum(axis=0) + gR * DZ1.sum(axis=0)
    E_dz1m = E_dz1 + UB * DZ1
    DZ1m = np.abs(dz1) + E_dz1m
    ax = np.abs(c["x"])
    out["W1"] = ax.T @ E_dz1m + gR * (ax.T @ DZ1m)
    E_loss = np.sum(2 * aerr * Eerr + Eerr ** 2) + _gam(rows + 17) * np.sum((aerr + Eerr) ** 2)
    return out, E_loss


def _bits(torch, t):
    return t.cpu().numpy().view(np.uint16)


def _params(seed):
    p = gen.mlp_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    p[mlp.P_B1:mlp.P_W2] = rng.normal(0, 0.1, 64)
    p[mlp.P_B2:mlp.P_W3] = rng.normal(0, 0.1, 64)
    p[mlp.P_B3] = 0.3
    return p.astype(np.float32)


@pytest.mark.parametrize("name", ["er", "cl"])
def test_features(env, name):
    torch, api, learned = env
    nl, nr, l, r = _graph(name)
    print(f"features {name}", flush=True)
    g = api.Graph(nl, nr, l, r)
    got = _bits(torch, learned.features(g))
    want = mlp.features(nl, nr, l, r)
    assert got.shape == want.shape
    # Both sides round the float64 value to FP32 and then to BF16; a last-bit
    # difference in log1p can move that decision by one BF16 step, rarely.
    diff = np.abs(got.astype(np.int32) - want.astype(np.int32))
    assert diff.max() <= 1
    assert np.count_nonzero(diff) <= max(2, got.size // 10_000)


def test_targets_and_probs(env):
    torch, api, learned = env
    cnt = np.array([0, 1, 2, 5, 1000, 123456789, 2**40 + 17, 2**62], np.uint64)
    dc = torch.from_numpy(cnt.view(np.int64)).cuda()
    t = learned.targets(dc).cpu().numpy().astype(np.float64)
    ref = mlp.targets(cnt)
    assert np.all(np.abs(t - ref) <= np.spacing(np.abs(ref).astype(np.float32)))
    y = np.random.default_rng(3).normal(0.5, 0.4, 10_001).astype(np.float32)
    for fl in (1e-9, 0.05, 1.0):
        p, mean = learned.probs(torch.from_numpy(y).cuda(), fl)
        pr, mr = mlp.probs_from_predictions(y.astype(np.float64), fl)
        assert math.isclose(float(mean.item()), mr, rel_tol=1e-12)
        assert np.allclose(p.cpu().numpy(), pr, rtol=1e-13, atol=0)
        assert np.all(p.cpu().numpy() > 0)
    # no positive prediction: uniform probabilities, never a zero
    yneg = -np.abs(y) - 0.01
    p, mean = learned.probs(torch.from_numpy(yneg.astype(np.float32)).cuda(), 0.05)
    assert float(mean.item()) == 0.0 and np.all(p.cpu().numpy() == 1.0)


@pytest.mark.parametrize("rows", [1, 17, 1_000, 18_000])
def test_forward(env, rows):
    torch, api, learned = env
    nl, nr, l, r = _graph("cl")
    x = mlp.features(nl, nr, l, r)[:rows]
    p = _params(1)
    print(f"forward rows={rows}", flush=True)
    net = learned.Mlp(p)
    y = net.forward(torch.from_numpy(x.view(np.int16)).cuda()).cpu().numpy().astype(np.float64)
    pr = _plain_params(p)
    want, c = mlp.forward(pr, mlp.bf16_value(x), emulate=False)
    fb = _forward_bound(c, pr)
    dev = np.abs(y - want)
    assert np.all(dev <= fb["ey"]), (dev - fb["ey"]).max()
    # the bound is not vacuous: it is a few BF16 steps of the output scale
    assert np.all(fb["ey"] <= 2.0 ** -4 * (np.abs(c["h2"]) @ np.abs(mlp.unpack(pr)[4]) + 1))
    # and the typical scale: independent roundings of relative size <= 2^-8
    # do not add up coherently, so the output as a whole stays within a few
    # BF16 steps (a wrong term would not)
    assert np.linalg.norm(dev) <= 2.0 ** -6 * np.linalg.norm(want) + 1e-6
    # diagnostic only: distance to the reference rounded where the kernels round
    emu, _ = mlp.forward(p, x, emulate=True)
    print(f"max |y - plain| {dev.max():.3g} (bound {fb['ey'].max():.3g}); "
          f"max |y - emulated| {np.abs(y - emu).max():.3g}", flush=True)


def _blocks(g):
    W1, b1, W2, b2, w3, b3 = mlp.unpack(g)
    return dict(W1=W1, b1=b1, W2=W2, b2=b2, w3=w3, b3=np.atleast_1d(b3))


@pytest.mark.parametrize("rows,use_idx", [(1, False), (1_000, False), (3_001, True),
                                          (70_000, True)])
def test_grad(env, rows, use_idx):
    torch, api, learned = env
    nl, nr, l, r = _graph("cl")
    x = mlp.features(nl, nr, l, r)
    cl, cr = oracle.per_vertex(nl, nr, l, r)
    tgt = mlp.targets(np.concatenate([cl, cr])).astype(np.float32)
    n = x.shape[0]
    if use_idx:
        idx = np.random.default_rng(rows).integers(0, n, rows).astype(np.uint32)
    else:
        idx = np.arange(rows, dtype=np.uint32)
    p = _params(2)
    print(f"grad rows={rows} idx={use_idx}", flush=True)
    net = learned.Mlp(p)
    dx = torch.from_numpy(x.view(np.int16)).cuda()
    dt = torch.from_numpy(tgt).cuda()
    di = torch.from_numpy(idx.view(np.int32)).cuda() if use_idx else None
    g1, l1 = net.grad(dx, dt, di, rows=rows)
    g1 = g1.cpu().numpy().astype(np.float64)
    loss = float(l1.item())
    g2, _ = net.grad(dx, dt, di, rows=rows)
    assert np.array_equal(g1, g2.cpu().numpy())          # fixed reduction order
    pr = _plain_params(p)
    xs = mlp.bf16_value(x[idx])
    ts = tgt[idx].astype(np.float64)
    want, sse = mlp.grad(pr, xs, ts, emulate=False)
    y, c = mlp.forward(pr, xs, emulate=False)
    fb = _forward_bound(c, pr)
    bound, e_loss = _grad_bound(c, pr, fb, y - ts, rows)
    assert abs(loss - sse) <= e_loss + 1e-30, (loss, sse, e_loss)
    got_b, want_b = _blocks(g1), _blocks(want)
    for k in want_b:
        dev = np.abs(got_b[k] - want_b[k]).ravel()
        bnd = np.asarray(bound[k], np.float64).ravel()
        assert np.all(dev <= bnd), (k, float((dev - bnd).max()))
        # typical scale: independent BF16 roundings do not add up coherently,
        # so each block as a whole stays within a few BF16 steps of the plain
        # gradient (a missing or wrong term would not)
        assert np.linalg.norm(got_b[k] - want_b[k]) <= 2.0 ** -6 * np.linalg.norm(want_b[k]) \
            + 1e-7, k
    # diagnostic only: distance to the reference rounded where the kernels round
    emu, _ = mlp.grad(p, x[idx], ts, emulate=True)
    print("grad max |g - plain| / bound:",
          {k: round(float(np.max(np.abs(got_b[k] - want_b[k]).ravel()
                                 / np.maximum(np.asarray(bound[k]).ravel(), 1e-300))), 3)
           for k in want_b},
          "max |g - emulated|", float(np.abs(g1 - emu).max()), flush=True)


def test_adam_step(env):
    torch, api, learned = env
    p = _params(3)
    net = learned.Mlp(p)
    rng = np.random.default_rng(4)
    g = rng.normal(0, 1e-2, mlp.P_N).astype(np.float32)
    m1 = np.zeros(mlp.P_N); m2 = np.zeros(mlp.P_N); pp = p.astype(np.float64)
    for step in (1, 2, 3):
        net.grad_buf.copy_(torch.from_numpy(g))
        net.adam(lr=1e-3)
        pp, m1, m2 = mlp.adam(pp, m1, m2, g.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, step)
        got = net.params.cpu().numpy().astype(np.float64)
        assert np.allclose(got, pp, rtol=0, atol=2e-6 + 1e-6 * np.abs(pp).max())
        assert np.array_equal(_bits(torch, net.wbf16), mlp.bf16_bits(got.astype(np.float32)))
        g = (g * 0.5 + rng.normal(0, 1e-3, mlp.P_N)).astype(np.float32)


def test_errors(env):
    torch, api, learned = env
    from paper_1801_00338_amd._lib import BfcError
    net = learned.Mlp(_params(5))
    x = torch.zeros((16, 8), dtype=torch.int16, device="cuda")
    t = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(BfcError):
        net.grad(x, t, rows=0)
    with pytest.raises(BfcError):
        net.adam(lr=0.0)
    with pytest.raises(BfcError):
        learned.probs(torch.zeros(0, dtype=torch.float32, device="cuda"))
    for bad in (0.0, -0.5, float("nan"), float("inf")):
        with pytest.raises(BfcError):
            learned.probs(torch.ones(8, dtype=torch.float32, device="cuda"), bad)


def test_learned_sampling_beats_uniform(env):
    """Train on small graphs, then compare closed-form single-draw variances on a held-out one.

    The held-out graph is drawn from the same generator with a different seed.
    The learned probabilities must cut the variance of one VSamp draw well
    below uniform sampling's, the weighted sampler must stay seed-exact with
    the oracle, and its mean over many seeds must sit within a few standard
    errors of the exact count.
    """
    torch, api, learned = env
    train = gen.training_graphs(4, 20_000, 200_000, seed=5)
    x, t = learned.training_set(train)
    net = learned.Mlp.init(7)
    th = t.cpu().numpy().astype(np.float64)
    mse = lambda: float(np.mean((net.forward(x).cpu().numpy() - th) ** 2))
    before = mse()
    losses = net.train(x, t, steps=600, batch=8192, lr=3e-3, seed=1, log_every=50)
    after = mse()
    print(f"mse before {before:.4g} after {after:.4g}; batch losses",
          [round(v, 4) for v in losses], flush=True)
    assert after < 0.1 * before

    nl, nr = 6_000, 24_000
    l, r = gen.chung_lu(nl, nr, 120_000, 2.1, 2.3, 1500, seed=(5 << 32) | 99)
    g = api.Graph(nl, nr, l, r)
    probs = learned.learned_probs(g, net, floor_frac=0.05)
    p_host = probs.cpu().numpy()
    cl, cr = oracle.per_vertex(nl, nr, l, r)
    cnt = np.concatenate([cl, cr])
    B = int(cnt.sum() // 4)
    v_uni = mlp.single_draw_variance(cnt, None, exact=False)
    v_lrn = mlp.single_draw_variance(cnt, mlp.vsamp_weights(p_host), exact=False)
    print(f"B={B} var1 uniform={v_uni:.4g} learned={v_lrn:.4g} "
          f"k(1%,95%) uniform={mlp.draws_for(math.sqrt(v_uni), B)} "
          f"learned={mlp.draws_for(math.sqrt(v_lrn), B)}", flush=True)
    assert v_lrn < 0.25 * v_uni

    # seed-exact with the oracle on the learned probabilities
    ids, c, est = g.vsamp(500, 42, probs=probs)
    ids2, c2, est2 = oracle.vsamp(nl, nr, l, r, 500, 42, probs=p_host)
    assert np.array_equal(ids, ids2) and np.array_equal(c, c2) and est == est2

    # unbiased: the mean over seeds is within 4 standard errors of B
    k, trials = 200, 100
    ests = np.array([g.vsamp(k, 1000 + s, probs=probs)[2] for s in range(trials)])
    se = math.sqrt(v_lrn / k / trials)
    assert abs(ests.mean() - B) <= 4 * se + 1e-9 * B
