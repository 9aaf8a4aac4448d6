"""GPU parity of the learned-sampling kernels with the float64 reference.

Features, targets and probabilities are compared value by value; the MLP
forward and gradient against the reference run with the kernels' rounding
points (BF16 weights, features, hidden layer 1, dZ2 and dZ1).  What is left
is FP32 accumulation order inside the matrix-core products and the rare BF16
rounding decision that an FP32 difference moves across a rounding boundary;
each tolerance below is derived from those two sources.
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
    for fl in (0.0, 0.05, 1.0):
        p, mean = learned.probs(torch.from_numpy(y).cuda(), fl)
        pr, mr = mlp.probs_from_predictions(y.astype(np.float64), fl)
        assert math.isclose(float(mean.item()), mr, rel_tol=1e-12)
        assert np.allclose(p.cpu().numpy(), pr, rtol=1e-13, atol=0)


@pytest.mark.parametrize("rows", [1, 17, 1_000, 18_000])
def test_forward(env, rows):
    torch, api, learned = env
    nl, nr, l, r = _graph("cl")
    x = mlp.features(nl, nr, l, r)[:rows]
    p = _params(1)
    print(f"forward rows={rows}", flush=True)
    net = learned.Mlp(p)
    y = net.forward(torch.from_numpy(x.view(np.int16)).cuda()).cpu().numpy().astype(np.float64)
    want, c = mlp.forward(p, x, emulate=True)
    # a BF16 rounding of h1 moved by one step (2^-8 relative) on every entry
    # changes y by at most 2^-8 |h1| |W2| |w3|; FP32 sums add ~2^-20 relative
    bound = 2.0 ** -8 * (np.abs(c["h1"]) @ np.abs(c["W2"]) @ np.abs(c["w3"]))
    bound += 1e-5 * (1 + np.abs(want))
    assert np.all(np.abs(y - want) <= bound)
    # and nearly every row is far tighter than that
    assert np.mean(np.abs(y - want) <= 1e-5 * (1 + np.abs(want))) >= 0.99


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
    want, sse = mlp.grad(p, x[idx], tgt[idx].astype(np.float64), emulate=True)
    assert math.isclose(loss, sse, rel_tol=1e-4, abs_tol=1e-6)
    # Every BF16 operand moved by one step would change a block by at most
    # 2^-8 of its norm (twice for the two rounded operands of a product).
    for k, (a, b) in {k: (_blocks(g1)[k], _blocks(want)[k]) for k in _blocks(want)}.items():
        scale = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 2.0 ** -7 * scale + 1e-7, k


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
