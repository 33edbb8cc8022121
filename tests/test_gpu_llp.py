"""Learning from label proportions (Section 5.3) and its Label-DP release
(Section 5.4) on the GPU: the soft bag counts, their backward and the exact
swap against the oracle, the released count table bit-exact, and training
through the relaxed query on a synthetic tabular stand-in."""
import numpy as np
import pytest
import torch

import oracle
import tdp_datagen as gen
from paper_2211_02753_amd import _lib as L
from paper_2211_02753_amd import llp

pytestmark = pytest.mark.gpu
DEV = "cuda"


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _case(n, F, C, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, F)).astype(np.float32)
    W = (rng.standard_normal((C, F)) * 0.7).astype(np.float32)
    b = (rng.standard_normal(C) * 0.3).astype(np.float32)
    return X, W, b


@pytest.mark.parametrize("n,F,C,bag", [(5, 8, 2, 1), (100_003, 8, 2, 1), (100_003, 8, 2, 8), (100_003, 5, 3, 64),
                                       (100_003, 8, 2, 512), (1_000_000, 16, 4, 128), (70_001, 7, 2, 4096)])
def test_llp_bag_count_forward_and_backward(n, F, C, bag):
    X, W, b = _case(n, F, C, n + bag)
    m = llp.LinearLLP(t(W), t(b))
    print(f"llp bag counts n={n} F={F} C={C} bag={bag}", flush=True)
    S = m.bag_counts(t(X), bag).cpu().numpy().astype(np.float64).reshape(-1, C)
    want = oracle.llp_forward(X, W.astype(np.float64), b.astype(np.float64), bag)
    assert np.max(np.abs(S - want)) <= 1e-5 * np.max(np.abs(want))
    # the loss fused into the forward's writes: mean squared error against T and its gradient
    T = (want + np.random.default_rng(2).standard_normal(want.shape)).astype(np.float32)
    dSl = torch.empty(want.size, dtype=torch.float32, device=DEV)
    m.bag_counts(t(X), bag, None, t(T.reshape(-1)), dSl)
    wl, wdS = oracle.mse(want.reshape(-1), T.reshape(-1).astype(np.float64))
    assert abs(m.loss.item() - wl) <= 1e-5 * wl + 2e-5 * np.max(np.abs(want)) * np.sqrt(wl)
    gdS = dSl.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gdS - wdS)) <= 1e-5 * np.max(np.abs(wdS)) + 2e-5 * np.max(np.abs(want)) / want.size
    dS = np.random.default_rng(1).standard_normal(want.shape).astype(np.float32)
    gW, gb = m.bag_counts_bwd(t(X), bag, t(dS.reshape(-1)))
    wdW, wdb = oracle.llp_backward(X, W.astype(np.float64), b.astype(np.float64), bag, dS.astype(np.float64))
    # tolerance scale of the mixed-sign sums: sum over rows of |dz| |x| and |dz|
    p = oracle.llp_forward(X, W.astype(np.float64), b.astype(np.float64), 1)
    dp = np.repeat(dS.astype(np.float64), bag, axis=0)[:n]
    dz = np.abs(p * (dp - (p * dp).sum(1, keepdims=True)))
    bW = dz.T @ np.abs(X.astype(np.float64))
    bb = dz.sum(0)
    assert np.all(np.abs(gW.cpu().numpy() - wdW) <= 1e-5 * bW + 1e-30)
    assert np.all(np.abs(gb.cpu().numpy() - wdb) <= 1e-5 * bb + 1e-30)


def test_llp_predict_is_the_exact_argmax_and_count_table():
    X, W, b = _case(200_003, 8, 3, 5)
    m = llp.LinearLLP(t(W), t(b))
    got = m.predict(t(X)).cpu().numpy()
    assert np.array_equal(got, oracle.llp_predict(X, W.astype(np.float64), b.astype(np.float64)))
    # released counts: exact COUNT per (bag, label), dense, plus noise
    n, bagsz = 200_003, 64
    lab = got
    bag_id = (np.arange(n) // bagsz).astype(np.int32)
    nb = int(bag_id[-1]) + 1
    noise = gen.laplace_f32(gen.stream_seed(gen.SEED_LLP, 50), nb * 3, 10.0)
    rel = llp.released_counts(t(bag_id), t(lab), nb, 3, t(noise)).cpu().numpy()
    q = oracle.query(n, keys=[(bag_id, 0), (lab, 0)])
    counts = np.zeros(nb * 3, np.int64)
    counts[q["k0"] * 3 + q["k1"]] = q["count"]
    assert np.array_equal(rel.view(np.uint32), oracle.noisy_counts(counts, noise).view(np.uint32))
    plain = llp.released_counts(t(bag_id), t(lab), nb, 3).cpu().numpy()
    assert np.array_equal(plain, counts.astype(np.float32))


def _train(Xtr, ytr, bag, noise_scale, seed=1):
    nb = Xtr.shape[0] // bag
    noise = None
    if noise_scale:
        noise = t(gen.laplace_f32(gen.stream_seed(gen.SEED_LLP, 1000 + bag + seed), nb * 2, noise_scale))
    return llp.train(t(Xtr), t(ytr), bag, noise)


def test_llp_and_label_dp_training_through_the_count_query():
    """Train the classifier only through the relaxed GROUP BY bag, label
    COUNT(*) against the released counts, then judge it on held-out rows
    through the exact swap (argmax labels)."""
    X, y = gen.tabular_income(49_152)
    Xtr, ytr, Xte, yte = X[:32768], y[:32768], X[32768:], y[32768:]
    err = {}
    for bag in (1, 8, 64, 512):
        for eps in (None, 0.1):
            m = _train(Xtr, ytr, bag, 1.0 / eps if eps else 0.0)
            pred = m.predict(t(Xte)).cpu().numpy()
            err[(bag, eps)] = float(np.mean(pred != yte))
    print("held-out error by bag size (LLP; LLP with Laplace counts, eps 0.1):", flush=True)
    for bag in (1, 8, 64, 512):
        print(f"  bag {bag:4d}: {err[(bag, None)]:.4f}  {err[(bag, 0.1)]:.4f}", flush=True)
    majority = float(np.mean(yte != 0))
    # every trained classifier beats the label-free guess by far
    assert all(e < majority - 0.05 for e in err.values()), (err, majority)
    # small bags train about as well as per-row labels; large bags dilute the signal
    assert abs(err[(8, None)] - err[(1, None)]) <= 0.02
    assert abs(err[(64, None)] - err[(1, None)]) <= 0.02
    assert err[(512, None)] > err[(8, None)]
