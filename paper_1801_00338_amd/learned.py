"""Learned importance sampling for VSamp, driven through the C ABI.

A small network (8 -> 64 -> 64 -> 1, ReLU, BF16 weights with FP32 master copy
and FP32 accumulation on the matrix cores) predicts log1p(B_v) / 8 from eight
cheap per-vertex features.  Its predictions set the probabilities of the
weighted vertex sampler (the paper's VSamp, Alg. 4, with the single-draw term
B_v / (4 q_v) of a Hansen-Hurwitz estimator), mixed with a floor of a fraction
of the mean prediction so that no vertex has probability zero.  The network
only decides which vertices are counted; every count is exact, so the
estimate is unbiased whatever the network predicts.

Every step runs in the library's kernels: features (bfc_features), targets
from the exact per-vertex counts (bfc_per_vertex, bfc_mlp_targets), the
gradient (bfc_mlp_grad), Adam (bfc_adam_step), inference (bfc_mlp_forward),
probabilities (bfc_probs_from_predictions) and the sampler (bfc_vsamp).
Random inputs (initial weights, mini-batch order) come from ``gen``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import gen
from ._lib import check, lib
from .api import Graph, _bytes, _stream

NFEAT = 8


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def param_count() -> int:
    return int(lib().bfc_mlp_param_count())


def features(graph: Graph, stream=None) -> torch.Tensor:
    """(n_left + n_right, 8) BF16 features (int16 storage), rows by global id."""
    n = graph.n_left + graph.n_right
    x = torch.empty((max(n, 1), NFEAT), dtype=torch.int16, device=graph.device)
    check(lib().bfc_features(C.byref(graph.g), _p(x), _stream(stream)), "features")
    return x[:n]


def vertex_counts(graph: Graph, stream=None) -> torch.Tensor:
    """Exact per-vertex butterfly counts, L ids then R ids, on the device (int64 storage)."""
    n = graph.n_left + graph.n_right
    cnt = torch.zeros(max(n, 1) + 1, dtype=torch.int64, device=graph.device)
    cl = cnt[:graph.n_left] if graph.n_left else None
    cr = cnt[graph.n_left:graph.n_left + graph.n_right] if graph.n_right else None
    graph.local_async(cl, cr, None, stream=stream)
    return cnt[:n]


def targets(counts: torch.Tensor, stream=None) -> torch.Tensor:
    """log1p(B_v) / 8 (float32) from per-vertex counts (uint64 in int64 storage)."""
    t = torch.empty(max(counts.numel(), 1), dtype=torch.float32, device=counts.device)
    check(lib().bfc_mlp_targets(_p(counts), counts.numel(), _p(t), _stream(stream)), "targets")
    return t[:counts.numel()]


class Mlp:
    """Parameters (FP32 master, BF16 copy) and Adam state of the network, on one device."""

    def __init__(self, params, device="cuda"):
        self.device = torch.device(device)
        n = param_count()
        p = torch.as_tensor(np.ascontiguousarray(params, dtype=np.float32))
        if p.numel() != n:
            raise ValueError(f"expected {n} parameters, got {p.numel()}")
        self.params = p.to(self.device)
        self.m1 = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.m2 = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.grad_buf = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.wbf16 = torch.empty(n, dtype=torch.int16, device=self.device)
        self.step = 0
        self._ws = None
        check(lib().bfc_mlp_bf16(_p(self.params), _p(self.wbf16), _stream()), "bf16 copy")

    @classmethod
    def init(cls, seed: int, device="cuda") -> "Mlp":
        return cls(gen.mlp_init(seed), device)

    # -------------------------------------------------------------- kernels
    def forward(self, x: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        rows = x.shape[0]
        y = out if out is not None else torch.empty(max(rows, 1), dtype=torch.float32,
                                                    device=self.device)
        check(lib().bfc_mlp_forward(_p(x), rows, _p(self.params), _p(self.wbf16), _p(y),
                                    _stream(stream)), "mlp forward")
        return y[:rows]

    def grad(self, x: torch.Tensor, target: torch.Tensor, idx=None, rows=None, stream=None):
        """Gradient of the mean squared error of the batch into self.grad_buf (async)."""
        if rows is None:
            rows = idx.numel() if idx is not None else x.shape[0]
        sz = C.c_size_t()
        check(lib().bfc_mlp_grad_ws_size(rows, C.byref(sz)), "grad ws size")
        if self._ws is None or self._ws.numel() < sz.value:
            self._ws = _bytes(sz.value, self.device)
        check(lib().bfc_mlp_grad(_p(x), _p(target), _p(idx), rows, _p(self.params),
                                 _p(self.wbf16), _p(self.grad_buf), _p(self.loss_buf),
                                 _p(self._ws), self._ws.numel(), _stream(stream)), "mlp grad")
        return self.grad_buf, self.loss_buf

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        check(lib().bfc_adam_step(_p(self.params), _p(self.m1), _p(self.m2), _p(self.grad_buf),
                                  _p(self.wbf16), C.c_float(lr), C.c_float(beta1),
                                  C.c_float(beta2), C.c_float(eps), self.step, _stream(stream)),
              "adam")

    # -------------------------------------------------------------- training
    @staticmethod
    def batch_orders(n: int, steps: int, batch: int, seed: int, device="cuda"):
        """The seeded per-epoch row orders that ``train`` walks, on the device."""
        batch = min(batch, n)
        per_epoch = max(1, n // batch)
        epochs = (steps + per_epoch - 1) // per_epoch
        return [torch.from_numpy(gen.batch_order(seed, n, e).view(np.int32)).to(device)
                for e in range(epochs)]

    def train(self, x: torch.Tensor, target: torch.Tensor, steps: int, batch: int = 65536,
              lr: float = 1e-3, seed: int = 0, log_every: int = 0, orders=None):
        """Adam on mini-batches drawn without replacement per epoch (seeded order).

        ``orders`` (from ``batch_orders``) may be prepared beforehand.
        Returns the mean squared errors read back every ``log_every`` steps
        (none if 0); reading them synchronises the stream.
        """
        n = x.shape[0]
        batch = min(batch, n)
        per_epoch = max(1, n // batch)
        if orders is None:
            orders = self.batch_orders(n, steps, batch, seed, self.device)
        losses = []
        for s in range(steps):
            e, b = divmod(s, per_epoch)
            idx = orders[e][b * batch:(b + 1) * batch]
            self.grad(x, target, idx)
            self.adam(lr)
            if log_every and (s + 1) % log_every == 0:
                losses.append(float(self.loss_buf.item()) / batch)
        return losses

    def state(self) -> np.ndarray:
        return self.params.cpu().numpy().copy()


def probs(y: torch.Tensor, floor_frac: float = 0.05, stream=None):
    """Sampling probabilities max(expm1(8 y), floor_frac * mean) (float64) and the mean."""
    n = y.numel()
    sz = C.c_size_t()
    check(lib().bfc_probs_ws_size(C.byref(sz)), "probs ws size")
    ws = _bytes(sz.value, y.device)
    p = torch.empty(max(n, 1), dtype=torch.float64, device=y.device)
    mean = torch.zeros(1, dtype=torch.float64, device=y.device)
    check(lib().bfc_probs_from_predictions(_p(y), n, C.c_double(floor_frac), _p(p), _p(mean),
                                           _p(ws), ws.numel(), _stream(stream)), "probs")
    return p[:n], mean


def learned_probs(graph: Graph, mlp: Mlp, floor_frac: float = 0.05, stream=None):
    """Features -> inference -> probabilities for every vertex of ``graph``."""
    x = features(graph, stream)
    y = mlp.forward(x, stream=stream)
    return probs(y, floor_frac, stream)[0]


def training_set(graphs, device="cuda"):
    """Features and targets of several graphs, concatenated on the device.

    ``graphs`` holds (nl, nr, l, r) tuples; targets come from the exact
    per-vertex counts of each graph.
    """
    xs, ts = [], []
    for nl, nr, l, r in graphs:
        g = Graph(nl, nr, l, r, device=device)
        xs.append(features(g))
        ts.append(targets(vertex_counts(g)))
        torch.cuda.synchronize(g.device)
        del g
    return torch.cat(xs), torch.cat(ts)
