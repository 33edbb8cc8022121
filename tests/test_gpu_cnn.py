"""Parity of the classifier layers (bf16 MFMA, float32 accumulation) with
the float64 oracle, and training of the learned label column through the
soft aggregate.

Layer tolerances: the oracle gets exactly the bf16 operands the GPU used
(products of two bf16 values are exact in float32), so the only differences
are float32 accumulation order and, for bf16 outputs, the final rounding:
|gpu - ref| <= 2^-8 |ref| + 1e-4 * max|ref| for bf16 outputs, and normwise
relative 1e-5 for float32 outputs (weight gradients, logits)."""
import numpy as np
import pytest
import torch

import oracle
import tdp_datagen as gen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def lib():
    from paper_2211_02753_amd import _lib
    return _lib.load()


def s():
    from paper_2211_02753_amd import _lib
    return _lib.stream_handle(torch.device(DEV))


def P(t):
    from paper_2211_02753_amd import _lib
    return _lib.ptr(t)


def chk(rc):
    from paper_2211_02753_amd import _lib
    _lib.check("cnn call", rc)


def to_bf16_dev(a):
    """float array -> (device bf16 tensor, float32 values it holds)."""
    r = oracle.bf16_round(np.asarray(a, np.float32))
    u = (r.view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(u.view(np.int16).copy()).to(DEV), r


def from_bf16(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


def f32_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def close_bf16(got, ref):
    ref = np.asarray(ref, np.float64)
    err = np.abs(np.asarray(got, np.float64) - ref)
    bound = 2.0 ** -8 * np.abs(ref) + 1e-4 * max(np.max(np.abs(ref)), 1e-30)
    assert np.all(err <= bound), float(np.max(err - bound))


def normwise(got, ref):
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(np.asarray(got, np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def test_image_to_bf16_all_pixel_values():
    img = torch.arange(256, dtype=torch.int32).to(torch.uint8).to(DEV)
    out = torch.empty(256, dtype=torch.int16, device=DEV)
    chk(lib().tdp_image_to_bf16(P(img), 256, P(out), s()))
    want = oracle.bf16_round(np.arange(256, dtype=np.float32) / np.float32(255.0))
    assert np.array_equal(from_bf16(out), want)


@pytest.mark.parametrize("B,H,W,Cin,Cout", [(3, 28, 28, 1, 32), (2, 26, 26, 32, 64), (1, 7, 9, 8, 5), (2, 5, 6, 3, 70),
                                             (64, 28, 28, 1, 32), (64, 26, 26, 32, 64)])  # training-batch shapes last
def test_conv_fwd_dgrad_wgrad(B, H, W, Cin, Cout):
    rng = np.random.default_rng(B * 100 + Cin)
    xd, x = to_bf16_dev(rng.standard_normal((B, H, W, Cin)))
    wd, w = to_bf16_dev(rng.standard_normal((Cout, 3, 3, Cin)) * 0.2)
    bias = rng.standard_normal(Cout).astype(np.float32)
    y = torch.empty((B, H - 2, W - 2, Cout), dtype=torch.int16, device=DEV)
    print("conv", B, H, W, Cin, Cout, flush=True)
    chk(lib().tdp_conv3x3_fwd_bf16(P(xd), P(wd), P(f32_dev(bias)), B, H, W, Cin, Cout, 1, P(y), s()))
    close_bf16(from_bf16(y), oracle.conv3x3_fwd(x, w, bias, relu=True))
    # input gradient, masked by a ReLU'd activation
    dyd, dy = to_bf16_dev(rng.standard_normal((B, H - 2, W - 2, Cout)))
    maskd, mask = to_bf16_dev(np.maximum(rng.standard_normal((B, H, W, Cin)), 0))
    dx = torch.empty((B, H, W, Cin), dtype=torch.int16, device=DEV)
    chk(lib().tdp_conv3x3_dgrad_bf16(P(dyd), P(wd), P(maskd), B, H, W, Cin, Cout, P(dx), s()))
    close_bf16(from_bf16(dx), oracle.conv3x3_dgrad(dy, w, H, W) * (mask > 0))
    # weight and bias gradients
    dw = torch.empty((Cout, 3, 3, Cin), dtype=torch.float32, device=DEV)
    db = torch.empty(Cout, dtype=torch.float32, device=DEV)
    chk(lib().tdp_conv3x3_wgrad_bf16(P(xd), P(dyd), B, H, W, Cin, Cout, P(dw), P(db), s()))
    rdw, rdb = oracle.conv3x3_wgrad(x, dy)
    assert normwise(dw.cpu().numpy(), rdw) <= 1e-5
    assert normwise(db.cpu().numpy(), rdb) <= 1e-5


@pytest.mark.parametrize("M,N,K", [(5, 128, 9216), (64, 10, 128), (130, 70, 40), (1, 1, 8),
                                   (1024, 128, 9216), (1024, 10, 128)])  # fc1 and fc2 at the training batch
def test_linear_fwd_dgrad_wgrad(M, N, K):
    rng = np.random.default_rng(M * 7 + N)
    xd, x = to_bf16_dev(rng.standard_normal((M, K)))
    wd, w = to_bf16_dev(rng.standard_normal((N, K)) / np.sqrt(K))
    bias = rng.standard_normal(N).astype(np.float32)
    yb = torch.empty((M, N), dtype=torch.int16, device=DEV)
    yf = torch.empty((M, N), dtype=torch.float32, device=DEV)
    print("linear", M, N, K, flush=True)
    chk(lib().tdp_linear_fwd_bf16(P(xd), P(wd), P(f32_dev(bias)), M, N, K, 1, P(yb), None, s()))
    chk(lib().tdp_linear_fwd_bf16(P(xd), P(wd), P(f32_dev(bias)), M, N, K, 0, None, P(yf), s()))
    ref = oracle.linear_fwd(x, w, bias, relu=False)
    close_bf16(from_bf16(yb), np.maximum(ref, 0))
    assert normwise(yf.cpu().numpy(), ref) <= 1e-5
    # both outputs: the split-K form (float32 accumulator, then bias + ReLU)
    yb2 = torch.empty((M, N), dtype=torch.int16, device=DEV)
    yf2 = torch.full((M, N), float("nan"), dtype=torch.float32, device=DEV)
    chk(lib().tdp_linear_fwd_bf16(P(xd), P(wd), P(f32_dev(bias)), M, N, K, 1, P(yb2), P(yf2), s()))
    assert normwise(yf2.cpu().numpy(), np.maximum(ref, 0)) <= 1e-5
    close_bf16(from_bf16(yb2), np.maximum(ref, 0))
    dyd, dy = to_bf16_dev(rng.standard_normal((M, N)))
    maskd, mask = to_bf16_dev(np.maximum(rng.standard_normal((M, K)), 0))
    dx = torch.empty((M, K), dtype=torch.int16, device=DEV)
    chk(lib().tdp_linear_dgrad_bf16(P(dyd), P(wd), P(maskd), M, N, K, P(dx), s()))
    rdx, rdw, rdb = oracle.linear_bwd(x, w, dy)
    close_bf16(from_bf16(dx), rdx * (mask > 0))
    dw = torch.empty((N, K), dtype=torch.float32, device=DEV)
    db = torch.empty(N, dtype=torch.float32, device=DEV)
    chk(lib().tdp_linear_wgrad_bf16(P(xd), P(dyd), M, N, K, P(dw), P(db), s()))
    assert normwise(dw.cpu().numpy(), rdw) <= 1e-5
    assert normwise(db.cpu().numpy(), rdb) <= 1e-5


@pytest.mark.parametrize("C", [64, 12])  # eight channels per thread, and the one-channel path
def test_maxpool_fwd_bwd_bit_exact(C):
    rng = np.random.default_rng(3 + C)
    raw = np.maximum(rng.standard_normal((3, 24, 24, C)), 0)  # ReLU output: many zero ties
    xd, x = to_bf16_dev(raw)
    y = torch.empty((3, 12, 12, C), dtype=torch.int16, device=DEV)
    chk(lib().tdp_maxpool2_fwd_bf16(P(xd), 3, 24, 24, C, P(y), s()))
    assert np.array_equal(from_bf16(y), oracle.maxpool2_fwd(x).astype(np.float32))
    dyd, dy = to_bf16_dev(rng.standard_normal((3, 12, 12, C)))
    dx = torch.empty((3, 24, 24, C), dtype=torch.int16, device=DEV)
    chk(lib().tdp_maxpool2_bwd_bf16(P(xd), P(dyd), 3, 24, 24, C, 0, P(dx), s()))
    assert np.array_equal(from_bf16(dx), oracle.maxpool2_bwd(x, dy).astype(np.float32))
    chk(lib().tdp_maxpool2_bwd_bf16(P(xd), P(dyd), 3, 24, 24, C, 1, P(dx), s()))
    assert np.array_equal(from_bf16(dx), (oracle.maxpool2_bwd(x, dy) * (x > 0)).astype(np.float32))


def test_softmax_expectation_head_and_argmax():
    rng = np.random.default_rng(4)
    M = 1000
    z = (rng.standard_normal((M, 10)) * 3).astype(np.float32)
    z[0] = 0  # all ties: argmax picks class 0
    p = torch.empty((M, 10), dtype=torch.float32, device=DEV)
    e = torch.empty(M, dtype=torch.float32, device=DEV)
    chk(lib().tdp_softmax_expect_fwd(P(f32_dev(z)), M, 10, P(p), P(e), s()))
    rp, re = oracle.softmax_expect(z)
    assert normwise(p.cpu().numpy(), rp) <= 1e-5 and normwise(e.cpu().numpy(), re) <= 1e-5
    dE = rng.standard_normal(M).astype(np.float32)
    dz = torch.empty((M, 10), dtype=torch.float32, device=DEV)
    chk(lib().tdp_softmax_expect_bwd(P(p), P(f32_dev(dE)), M, 10, P(dz), None, s()))
    pg = p.cpu().numpy().astype(np.float64)
    assert normwise(dz.cpu().numpy(), oracle.softmax_expect_bwd(pg, dE.astype(np.float64))) <= 1e-5
    dP = rng.standard_normal((M, 10)).astype(np.float32)
    chk(lib().tdp_softmax_bwd(P(p), P(f32_dev(dP)), M, 10, P(dz), None, s()))
    assert normwise(dz.cpu().numpy(), oracle.softmax_bwd(pg, dP.astype(np.float64))) <= 1e-5
    lab = torch.empty(M, dtype=torch.int8, device=DEV)
    chk(lib().tdp_argmax_rows(P(p), M, 10, P(lab), s()))
    assert np.array_equal(lab.cpu().numpy(), oracle.argmax(p.cpu().numpy()))


def test_adam_matches_oracle():
    rng = np.random.default_rng(5)
    n = 10001
    p0 = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m0 = (rng.standard_normal(n) * 0.1).astype(np.float32)
    v0 = (rng.random(n) * 0.1).astype(np.float32)
    pd, md, vd = f32_dev(p0), f32_dev(m0), f32_dev(v0)
    pb = torch.empty(n, dtype=torch.int16, device=DEV)
    chk(lib().tdp_adam_step(P(pd), P(f32_dev(g)), P(md), P(vd), n, 1e-3, 0.9, 0.999, 1e-8, 7, P(pb), s()))
    # the kernel's hyperparameters are float32 values: give the oracle the same ones
    f = lambda c: float(np.float32(c))
    rp, rm, rv = oracle.adam(p0, g, m0, v0, f(1e-3), f(0.9), f(0.999), f(1e-8), 7)
    # float32 update: within a few float32 ulps of the parameter plus 1e-5 of the step size
    err = np.abs(pd.cpu().numpy().astype(np.float64) - rp)
    assert np.all(err <= 2.0 ** -22 * np.abs(rp) + 1e-5 * np.max(np.abs(rp - p0)))
    assert normwise(md.cpu().numpy(), rm) <= 1e-6 and normwise(vd.cpu().numpy(), rv) <= 1e-6
    assert np.array_equal(from_bf16(pb), oracle.bf16_round(pd.cpu().numpy()))


def test_adam_multi_matches_single_tensor_calls():
    """One launch over several tensors (ragged sizes, with and without bf16
    copies) gives exactly what one call per tensor gives."""
    from paper_2211_02753_amd import _lib as L
    rng = np.random.default_rng(9)
    sizes = [1, 31, 10001, 4096, 300_000]
    def state():
        out = []
        for k, n in enumerate(sizes):
            out.append([f32_dev(rng.standard_normal(n).astype(np.float32)) for _ in range(2)] +
                       [f32_dev((rng.random(n) * 0.1).astype(np.float32)) for _ in range(2)] +
                       [torch.empty(n, dtype=torch.int16, device=DEV) if k % 2 == 0 else None])
        return out
    a = state()
    b = [[t.clone() if t is not None else None for t in ts] for ts in a]
    for p_, g_, m_, v_, pb in a:
        chk(lib().tdp_adam_step(P(p_), P(g_), P(m_), P(v_), p_.numel(), 1e-3, 0.9, 0.999, 1e-8, 3, P(pb), s()))
    arr = (L.AdamTensor * len(b))()
    for i, (p_, g_, m_, v_, pb) in enumerate(b):
        arr[i] = L.AdamTensor(P(p_), P(g_), P(m_), P(v_), P(pb), p_.numel())
    chk(lib().tdp_adam_step_multi(arr, len(b), 1e-3, 0.9, 0.999, 1e-8, 3, s()))
    torch.cuda.synchronize()
    for ta, tb in zip(a, b):
        for x, y in zip(ta, tb):
            if x is not None:
                assert torch.equal(x, y)
    assert lib().tdp_adam_step_multi(arr, 17, 1e-3, 0.9, 0.999, 1e-8, 3, s()) == L.TDP_EINVAL


def test_network_forward_backward_against_layerwise_oracle():
    """One forward and backward of the whole network on 8 images; each layer
    is checked against the oracle fed with the GPU's own bf16 input to it."""
    from paper_2211_02753_amd.cnn import DigitCNN
    col = gen.image_column(n_images=8)
    model = DigitCNN(gen.cnn_init(), device=DEV, max_batch=8)
    img = torch.from_numpy(col["images"]).to(DEV)
    p, e = model.forward(img)
    torch.cuda.synchronize()
    wb = {k: from_bf16(v) for k, v in model.wb.items()}
    pr = {k: v.cpu().numpy() for k, v in model.p.items()}
    x0 = from_bf16(model.x0[:8])
    a1 = from_bf16(model.a1[:8])
    close_bf16(a1, oracle.conv3x3_fwd(x0, wb["conv1_w"], pr["conv1_b"], True))
    a2 = from_bf16(model.a2[:8])
    close_bf16(a2, oracle.conv3x3_fwd(a1, wb["conv2_w"], pr["conv2_b"], True))
    p2 = from_bf16(model.p2[:8])
    assert np.array_equal(p2, oracle.maxpool2_fwd(a2).astype(np.float32))
    a3 = from_bf16(model.a3[:8])
    close_bf16(a3, oracle.linear_fwd(p2.reshape(8, -1), wb["fc1_w"], pr["fc1_b"], True))
    logits = model.logits[:8].cpu().numpy()
    assert normwise(logits, oracle.linear_fwd(a3, wb["fc2_w"], pr["fc2_b"], False)) <= 1e-5
    rp, re = oracle.softmax_expect(logits)
    assert normwise(p.cpu().numpy(), rp) <= 1e-5 and normwise(e.cpu().numpy(), re) <= 1e-5
    dE = np.linspace(-1, 1, 8).astype(np.float32)
    model.backward(f32_dev(dE))
    torch.cuda.synchronize()
    dlog = from_bf16(model.dlog[:8])
    close_bf16(dlog, oracle.softmax_expect_bwd(p.cpu().numpy().astype(np.float64), dE.astype(np.float64)))
    rdx, rdw, rdb = oracle.linear_bwd(a3, wb["fc2_w"], dlog)
    assert normwise(model.g["fc2_w"].cpu().numpy(), rdw) <= 1e-5
    dz3 = from_bf16(model.dz3[:8])
    close_bf16(dz3, rdx * (a3 > 0))
    rdx, rdw, rdb = oracle.linear_bwd(p2.reshape(8, -1), wb["fc1_w"], dz3)
    assert normwise(model.g["fc1_w"].cpu().numpy(), rdw) <= 1e-5
    assert normwise(model.g["fc1_b"].cpu().numpy(), rdb) <= 1e-5
    dp2 = from_bf16(model.dp2[:8]).reshape(8, -1)
    close_bf16(dp2, rdx)
    dz2 = from_bf16(model.dz2[:8])
    assert np.array_equal(dz2, (oracle.maxpool2_bwd(a2, dp2.reshape(8, 12, 12, 64)) * (a2 > 0)).astype(np.float32))
    rdw, rdb = oracle.conv3x3_wgrad(a1, dz2)
    assert normwise(model.g["conv2_w"].cpu().numpy(), rdw) <= 1e-5
    dz1 = from_bf16(model.dz1[:8])
    close_bf16(dz1, oracle.conv3x3_dgrad(dz2, wb["conv2_w"], 26, 26) * (a1 > 0))
    rdw, rdb = oracle.conv3x3_wgrad(x0, dz1)
    assert normwise(model.g["conv1_w"].cpu().numpy(), rdw) <= 1e-5
    assert normwise(model.g["conv1_b"].cpu().numpy(), rdb) <= 1e-5
