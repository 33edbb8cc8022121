"""Learning from label proportions (the paper's LLP and Label-DP use cases):
a linear classifier trained only through a relaxed GROUP BY bag, label
COUNT(*) query against released per-bag label counts.

Everything numeric runs in libtdp: the exact per-(bag, label) counts
(tdp_groupby_agg), their dense release with caller-drawn noise
(tdp_count_table), the soft bag counts with the loss fused into their
final writes, and their backward (tdp_llp_bag_count[_bwd]), Adam
(tdp_adam_step_multi) and the exact swap at inference (tdp_llp_predict).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .query import GroupbyQuery, Key, check_flags


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def released_counts(bag_id: torch.Tensor, label: torch.Tensor, n_bags: int, n_classes: int,
                    noise: torch.Tensor | None = None) -> torch.Tensor:
    """The bags' label counts as the data owner releases them: the exact
    SELECT bag, label, COUNT(*) GROUP BY bag, label as a dense float32
    [n_bags * n_classes] table, each cell plus its noise draw when given."""
    lib = L.load()
    dev = bag_id.device
    q = GroupbyQuery(bag_id.numel(), [Key(bag_id, 0, n_bags), Key(label, 0, n_classes)])
    q.launch()
    out = torch.empty(n_bags * n_classes, dtype=torch.float32, device=dev)
    L.check("tdp_count_table", lib.tdp_count_table(_p(q.key0), _p(q.key1), _p(q.count), _p(q.n_groups), 0, n_bags, 0,
                                                   n_classes, _p(noise), _p(out), _p(q.status),
                                                   L.stream_handle(dev)))
    check_flags(q.status, "tdp_count_table")
    return out


class LinearLLP:
    """softmax(W x + b) over C classes, W [C][F] and b [C] float32 on the GPU."""

    def __init__(self, W: torch.Tensor, b: torch.Tensor):
        self.lib = L.load()
        self.W, self.b = W.contiguous(), b.contiguous()
        self.C, self.F = W.shape
        dev = W.device
        self.dev = dev
        f32 = dict(dtype=torch.float32, device=dev)
        self.gW, self.gb = torch.zeros_like(self.W), torch.zeros_like(self.b)
        self.mW, self.vW = torch.zeros_like(self.W), torch.zeros_like(self.W)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.ws = L.workspace(self.lib.tdp_llp_workspace_size(self.C), dev)
        self.loss = torch.empty(1, **f32)
        self.step_count = 0
        # pointers of the tensors every step passes (they live as long as the model)
        self._pW, self._pb, self._pws, self._ploss = _p(self.W), _p(self.b), _p(self.ws), _p(self.loss)
        self._pgW, self._pgb = _p(self.gW), _p(self.gb)
        self._adam = (L.AdamTensor * 2)(L.AdamTensor(self._pW, self._pgW, _p(self.mW), _p(self.vW), None, self.W.numel()),
                                        L.AdamTensor(self._pb, self._pgb, _p(self.mb), _p(self.vb), None, self.b.numel()))

    def _s(self):
        return L.stream_handle(self.dev)

    def bag_counts(self, X: torch.Tensor, bag: int, S: torch.Tensor | None = None, T: torch.Tensor | None = None,
                   dS: torch.Tensor | None = None) -> torch.Tensor:
        """Soft counts S [n_bags * C]; with T also the loss (self.loss) and dS."""
        n = X.shape[0]
        S = torch.empty(((n + bag - 1) // bag) * self.C, dtype=torch.float32, device=self.dev) if S is None else S
        L.check("tdp_llp_bag_count", self.lib.tdp_llp_bag_count(
            _p(X), n, self.F, _p(self.W), _p(self.b), self.C, bag, _p(S), _p(T), _p(self.loss) if T is not None else None,
            _p(dS), _p(self.ws), self.ws.numel(), self._s()))
        return S

    def bag_counts_bwd(self, X: torch.Tensor, bag: int, dS: torch.Tensor):
        L.check("tdp_llp_bag_count_bwd",
                self.lib.tdp_llp_bag_count_bwd(_p(X), X.shape[0], self.F, _p(self.W), _p(self.b), self.C, bag, _p(dS),
                                               _p(self.gW), _p(self.gb), _p(self.ws), self.ws.numel(), self._s()))
        return self.gW, self.gb

    def step(self, X: torch.Tensor, T: torch.Tensor, bag: int, lr: float):
        """One training step on whole bags: soft counts, mean squared error
        against the released counts T, backward, Adam."""
        n = X.shape[0]
        nb = (n + bag - 1) // bag
        if getattr(self, "_nb", None) != nb:
            self._nb = nb
            self._S = torch.empty(nb * self.C, dtype=torch.float32, device=self.dev)
            self._dS = torch.empty_like(self._S)
            self._pS, self._pdS = _p(self._S), _p(self._dS)
        lib, sh, pX = self.lib, self._s(), _p(X)
        L.check("tdp_llp_bag_count", lib.tdp_llp_bag_count(
            pX, n, self.F, self._pW, self._pb, self.C, bag, self._pS, _p(T), self._ploss, self._pdS, self._pws,
            self.ws.numel(), sh))
        L.check("tdp_llp_bag_count_bwd", lib.tdp_llp_bag_count_bwd(
            pX, n, self.F, self._pW, self._pb, self.C, bag, self._pdS, self._pgW, self._pgb, self._pws, self.ws.numel(),
            sh))
        self.step_count += 1
        L.check("tdp_adam_step_multi", lib.tdp_adam_step_multi(self._adam, 2, lr, 0.9, 0.999, 1e-8, self.step_count, sh))
        return self.loss

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        """The exact swap at inference: argmax labels (int8)."""
        out = torch.empty(X.shape[0], dtype=torch.int8, device=self.dev)
        L.check("tdp_llp_predict", self.lib.tdp_llp_predict(_p(X), X.shape[0], self.F, _p(self.W), _p(self.b), self.C,
                                                            _p(out), self._s()))
        return out


def train(X: torch.Tensor, y: torch.Tensor, bag: int, noise: torch.Tensor | None = None, epochs: int = 30,
          batch: int = 4096, lr: float = 0.05) -> LinearLLP:
    """Train a zero-initialised binary linear classifier from bag label
    counts only: consecutive bags of `bag` rows of X [n][F] (n a multiple of
    bag), counts released with `noise` (or exactly), mini-batches of whole
    bags, fixed order."""
    n, F = X.shape
    nb = n // bag
    bag_id = L.segment_ids(n, bag, X.device)
    T = released_counts(bag_id, y, nb, 2, noise)
    m = LinearLLP(torch.zeros(2, F, dtype=torch.float32, device=X.device),
                  torch.zeros(2, dtype=torch.float32, device=X.device))
    rows = max(batch, bag)
    for _ in range(epochs):
        for r0 in range(0, n, rows):
            m.step(X[r0:r0 + rows], T[(r0 // bag) * 2:((r0 + rows) // bag) * 2], bag, lr)
    return m
