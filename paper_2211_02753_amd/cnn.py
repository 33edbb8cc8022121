"""The learned label column: a small CNN over an image column, trained only
through aggregate answers (Section 3's grid-of-images query, Sections 4 and
5.5).  Every layer, gradient and optimizer step runs in libtdp's kernels;
this module owns the device buffers and the order of the calls.

Architecture (the paper leaves it open): conv3x3 1->32 + ReLU, conv3x3
32->64 + ReLU, 2x2 max pool, fc 9216->128 + ReLU, fc 128->10, softmax.  The
soft label of an image is the expectation sum_k k p_k; the soft SUM of the
label column per grid row is a soft group-by of those expectations; the
exact swap at inference takes argmax labels into the exact group-by.
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import soft

SHAPES = {
    "conv1_w": (32, 3, 3, 1), "conv1_b": (32,),
    "conv2_w": (64, 3, 3, 32), "conv2_b": (64,),
    "fc1_w": (128, 12 * 12 * 64), "fc1_b": (128,),
    "fc2_w": (10, 128), "fc2_b": (10,),
}
N_CLASSES = 10


def _p(t):
    return L.ptr(t)


class DigitCNN:
    """Parameters (float32 masters + bf16 copies), Adam state, and activation
    buffers for up to ``max_batch`` images."""

    def __init__(self, params: dict, device="cuda:0", max_batch: int = 1024):
        self.lib = L.load()
        self.dev = torch.device(device)
        self.max_batch = max_batch
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.p = {k: torch.as_tensor(v, dtype=torch.float32).to(self.dev).contiguous() for k, v in params.items()}
        self.g = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.wb = {k: torch.empty(v.shape, dtype=torch.int16, device=self.dev) for k, v in self.p.items()
                   if k.endswith("_w")}
        for k in self.wb:
            self._chk("tdp_f32_to_bf16", self.lib.tdp_f32_to_bf16(_p(self.p[k]), self.p[k].numel(), _p(self.wb[k]),
                                                                   self._s()))
        self.step_count = 0
        B = max_batch
        bf = dict(dtype=torch.int16, device=self.dev)
        self.x0 = torch.empty((B, 28, 28, 1), **bf)
        self.a1 = torch.empty((B, 26, 26, 32), **bf)
        self.a2 = torch.empty((B, 24, 24, 64), **bf)
        self.p2 = torch.empty((B, 12, 12, 64), **bf)
        self.a3 = torch.empty((B, 128), **bf)
        self.a3f = torch.empty((B, 128), **f32)  # float32 accumulator of the split-K fc1
        self.logits = torch.empty((B, N_CLASSES), **f32)
        self.prob = torch.empty((B, N_CLASSES), **f32)
        self.e = torch.empty(B, **f32)
        # gradient buffers
        self.dlog = torch.empty((B, N_CLASSES), **bf)
        self.dz3 = torch.empty((B, 128), **bf)
        self.dp2 = torch.empty((B, 12, 12, 64), **bf)
        self.dz2 = torch.empty((B, 24, 24, 64), **bf)
        self.dz1 = torch.empty((B, 26, 26, 32), **bf)

    def _s(self):
        return L.stream_handle(self.dev)

    @staticmethod
    def _chk(fn, rc):
        L.check(fn, rc)

    # ------------------------------------------------------------ forward
    def forward(self, img: torch.Tensor):
        """img uint8 [B, 28, 28] -> (p [B, 10], e [B]) views of internal buffers."""
        B = img.shape[0]
        assert B <= self.max_batch and img.dtype == torch.uint8 and img.is_contiguous()
        lib, s, w = self.lib, self._s(), self.wb
        self._chk("tdp_image_to_bf16", lib.tdp_image_to_bf16(_p(img), img.numel(), _p(self.x0), s))
        self._chk("conv1", lib.tdp_conv3x3_fwd_bf16(_p(self.x0), _p(w["conv1_w"]), _p(self.p["conv1_b"]), B, 28, 28, 1,
                                                    32, 1, _p(self.a1), s))
        self._chk("conv2", lib.tdp_conv3x3_fwd_bf16(_p(self.a1), _p(w["conv2_w"]), _p(self.p["conv2_b"]), B, 26, 26,
                                                    32, 64, 1, _p(self.a2), s))
        self._chk("pool", lib.tdp_maxpool2_fwd_bf16(_p(self.a2), B, 24, 24, 64, _p(self.p2), s))
        self._chk("fc1", lib.tdp_linear_fwd_bf16(_p(self.p2), _p(w["fc1_w"]), _p(self.p["fc1_b"]), B, 128, 9216, 1,
                                                 _p(self.a3), _p(self.a3f), s))
        self._chk("fc2", lib.tdp_linear_fwd_bf16(_p(self.a3), _p(w["fc2_w"]), _p(self.p["fc2_b"]), B, N_CLASSES, 128,
                                                 0, None, _p(self.logits), s))
        self._chk("softmax", lib.tdp_softmax_expect_fwd(_p(self.logits), B, N_CLASSES, _p(self.prob), _p(self.e), s))
        self.B = B
        return self.prob[:B], self.e[:B]

    # ----------------------------------------------------------- backward
    def backward(self, dE: torch.Tensor):
        """dL/de [B] (gradient of the expected labels, float32) -> parameter gradients in self.g."""
        dE = dE.contiguous()  # a copy must outlive the asynchronous call
        self._chk("softmax_expect_bwd", self.lib.tdp_softmax_expect_bwd(_p(self.prob), _p(dE), self.B,
                                                                        N_CLASSES, None, _p(self.dlog), self._s()))
        self._backward_from_logits()

    def backward_probs(self, dP: torch.Tensor):
        """dL/dp [B, 10] (gradient of the class probabilities) -> parameter gradients in self.g."""
        dP = dP.contiguous()  # a copy must outlive the asynchronous call
        self._chk("softmax_bwd", self.lib.tdp_softmax_bwd(_p(self.prob), _p(dP), self.B, N_CLASSES, None,
                                                          _p(self.dlog), self._s()))
        self._backward_from_logits()

    def _backward_from_logits(self):
        B = self.B
        lib, s, w, g = self.lib, self._s(), self.wb, self.g
        self._chk("fc2_w", lib.tdp_linear_wgrad_bf16(_p(self.a3), _p(self.dlog), B, N_CLASSES, 128, _p(g["fc2_w"]),
                                                     _p(g["fc2_b"]), s))
        self._chk("fc2_x", lib.tdp_linear_dgrad_bf16(_p(self.dlog), _p(w["fc2_w"]), _p(self.a3), B, N_CLASSES, 128,
                                                     _p(self.dz3), s))
        self._chk("fc1_w", lib.tdp_linear_wgrad_bf16(_p(self.p2), _p(self.dz3), B, 128, 9216, _p(g["fc1_w"]),
                                                     _p(g["fc1_b"]), s))
        self._chk("fc1_x", lib.tdp_linear_dgrad_bf16(_p(self.dz3), _p(w["fc1_w"]), None, B, 128, 9216, _p(self.dp2), s))
        self._chk("pool_bwd", lib.tdp_maxpool2_bwd_bf16(_p(self.a2), _p(self.dp2), B, 24, 24, 64, 1, _p(self.dz2), s))
        self._chk("conv2_w", lib.tdp_conv3x3_wgrad_bf16(_p(self.a1), _p(self.dz2), B, 26, 26, 32, 64, _p(g["conv2_w"]),
                                                        _p(g["conv2_b"]), s))
        self._chk("conv2_x", lib.tdp_conv3x3_dgrad_bf16(_p(self.dz2), _p(w["conv2_w"]), _p(self.a1), B, 26, 26, 32, 64,
                                                        _p(self.dz1), s))
        self._chk("conv1_w", lib.tdp_conv3x3_wgrad_bf16(_p(self.x0), _p(self.dz1), B, 28, 28, 1, 32, _p(g["conv1_w"]),
                                                        _p(g["conv1_b"]), s))

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        """One Adam step of every parameter tensor, in one launch."""
        self.step_count += 1
        keys = list(self.p)
        arr = (L.AdamTensor * len(keys))()
        for i, k in enumerate(keys):
            arr[i] = L.AdamTensor(_p(self.p[k]), _p(self.g[k]), _p(self.m[k]), _p(self.v[k]), _p(self.wb.get(k)),
                                  self.p[k].numel())
        self._chk("adam", self.lib.tdp_adam_step_multi(arr, len(keys), lr, b1, b2, eps, self.step_count, self._s()))

    def predict_labels(self, img: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Exact swap at inference: argmax labels (int8) for a batch of images."""
        p, _ = self.forward(img)
        B = img.shape[0]
        out = torch.empty(B, dtype=torch.int8, device=self.dev) if out is None else out
        self._chk("argmax", self.lib.tdp_argmax_rows(_p(p), B, N_CLASSES, _p(out), self._s()))
        return out

    def label_column(self, images: torch.Tensor) -> torch.Tensor:
        """Argmax labels for a whole image column, batch by batch."""
        n = images.shape[0]
        out = torch.empty(n, dtype=torch.int8, device=self.dev)
        for a in range(0, n, self.max_batch):
            b = min(n, a + self.max_batch)
            self.predict_labels(images[a:b], out[a:b])
        return out

    def state_dict(self):
        return {k: v.detach().cpu().clone() for k, v in self.p.items()}


class GridQueryTrainer:
    """Trains the CNN through a trainable query over the grid rows (the loop
    of Section 3, with Adam).

    mode "count": SELECT grid_row, label, COUNT(*) GROUP BY grid_row, label
        on the probability-encoded label column (the soft COUNT per class,
        Section 4; the shape of the paper's own grid query), against the
        exact engine's counts [R, 10].
    mode "sum": SELECT grid_row, SUM(label) GROUP BY grid_row with the
        expected label as the soft value, against the exact row sums [R].
    Either way the loss is the mean squared error over the answer cells."""

    def __init__(self, model: DigitCNN, cells_per_row: int = 4, lr: float = 5e-4, mode: str = "count"):
        assert mode in ("count", "sum")
        self.model = model
        self.cpr = cells_per_row
        self.lr = lr
        self.mode = mode
        dev = model.dev
        B = model.max_batch
        K = N_CLASSES if mode == "count" else 1
        self.K = K
        self.rows_max = B // cells_per_row
        self.g = L.segment_ids(B, cells_per_row, dev)
        self.ws = soft.new_soft_workspace(dev)
        self.S = torch.empty(self.rows_max * K, dtype=torch.float32, device=dev)
        self.dS = torch.empty(self.rows_max * K, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.dV = torch.empty(B * K, dtype=torch.float32, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)

    def step(self, img: torch.Tensor, target: torch.Tensor):
        """One step on R grid rows: img [R*cpr, 28, 28] uint8; target [R, 10]
        counts (mode "count") or [R] sums (mode "sum"), float32."""
        m, lib = self.model, self.model.lib
        R = target.shape[0]
        n = R * self.cpr
        K = self.K
        s = m._s()
        p, e = m.forward(img)
        v = p if K > 1 else e
        L.check("soft_groupby", lib.tdp_soft_groupby(_p(self.g), None, _p(v), n, K, R, _p(self.S), _p(self.status),
                                                     _p(self.ws), self.ws.numel(), s))
        target = target.contiguous()  # a copy must outlive the asynchronous call
        L.check("mse", lib.tdp_mse_loss(_p(self.S), _p(target), R * K, _p(self.loss), _p(self.dS), s))
        L.check("soft_groupby_bwd", lib.tdp_soft_groupby_bwd(_p(self.g), None, _p(v), _p(self.dS), n, K, R, None,
                                                             _p(self.dV), s))
        if K > 1:
            m.backward_probs(self.dV[:n * K].view(n, K))
        else:
            m.backward(self.dV[:n])
        m.adam_step(lr=self.lr)
        return self.loss
