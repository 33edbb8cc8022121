"""The learned label column end to end: the CNN is trained on the GPU only
through aggregate answers computed by the exact engine — the COUNT per
(grid row, label), the shape of the paper's grouped count query, or the
config's literal SUM(label) per grid row — then the exact swap (argmax
labels into the exact group-by) answers SUM(label) per grid row.  The exact
query over the true labels judges it, and the trained network must beat the
same method without it: the label-free estimate (every row predicts the mean
training sum) and the untrained network."""
import numpy as np
import pytest
import torch

import tdp_datagen as gen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_learned_label_column_gain():
    from paper_2211_02753_amd import _lib as L
    from paper_2211_02753_amd import query as Q
    from paper_2211_02753_amd.cnn import DigitCNN, GridQueryTrainer

    n_rows, cpr, n_train_rows = 30_000, 4, 25_000
    col = gen.image_column(n_images=n_rows * cpr)
    images = torch.from_numpy(col["images"]).to(DEV)
    labels = torch.from_numpy(col["label"]).to(DEV)
    grid_row = torch.from_numpy(col["grid_row"]).to(DEV)
    bucket = torch.from_numpy(col["bucket"]).to(DEV)

    def row_sums(label_col):
        r = Q.GroupbyQuery(n_rows * cpr, keys=[Q.Key(grid_row, 0, n_rows)], expr=L.EXPR_COL, a=Q.Operand(label_col))()
        out = torch.zeros(n_rows, dtype=torch.int64, device=DEV)
        out[r["k0"]] = r["sum"]
        return out

    def bucket_sums(label_col):
        r = Q.GroupbyQuery(n_rows * cpr, keys=[Q.Key(bucket, 0, 100)], expr=L.EXPR_COL, a=Q.Operand(label_col))()
        return r["sum"].clone()

    truth_rows = row_sums(labels)           # the exact engine on the hidden labels: targets and judge
    truth_buckets = bucket_sums(labels)
    # training answers: COUNT(*) per (grid row, label) from the exact engine
    r = Q.GroupbyQuery(n_rows * cpr, keys=[Q.Key(grid_row, 0, n_rows), Q.Key(labels, 0, 10)], expr=L.EXPR_NONE)()
    counts = torch.zeros((n_rows, 10), dtype=torch.float32, device=DEV)
    counts[r["k0"], r["k1"]] = r["count"].to(torch.float32)
    target = truth_rows.to(torch.float32)

    model = DigitCNN(gen.cnn_init(), device=DEV, max_batch=1024)
    untrained = model.label_column(images)
    test = slice(n_train_rows, n_rows)

    def row_err(pred_labels):
        return (row_sums(pred_labels)[test] - truth_rows[test]).abs().double().mean().item()

    err_untrained = row_err(untrained)
    mean_sum = target[:n_train_rows].mean().item()
    err_label_free = (truth_rows[test].double() - mean_sum).abs().mean().item()

    trainer = GridQueryTrainer(model, cells_per_row=cpr, lr=5e-4, mode="count")
    rows_per_batch = 64
    order = np.random.default_rng(0).permutation(n_train_rows // rows_per_batch)
    for epoch in range(2):
        for bi in order:
            r0 = int(bi) * rows_per_batch
            img = images[r0 * cpr:(r0 + rows_per_batch) * cpr]
            loss = trainer.step(img, counts[r0:r0 + rows_per_batch])
        print("epoch", epoch, "loss", float(loss.item()), flush=True)
    assert float(counts[:n_train_rows].sum().item()) == n_train_rows * cpr

    pred = model.label_column(images)
    err_trained = row_err(pred)
    img_acc = (pred[n_train_rows * cpr:] == labels[n_train_rows * cpr:]).double().mean().item()
    row_exact = (row_sums(pred)[test] == truth_rows[test]).double().mean().item()
    bucket_err = ((bucket_sums(pred) - truth_buckets).abs().double() / truth_buckets.double()).mean().item()
    print(f"row |err| trained {err_trained:.3f} untrained {err_untrained:.3f} label-free {err_label_free:.3f}; "
          f"held-out image accuracy {img_acc:.4f}; row exact {row_exact:.4f}; bucket rel err {bucket_err:.5f}", flush=True)
    assert err_trained < err_label_free and err_trained < err_untrained
    assert img_acc > 0.9


def test_learned_label_column_sum_supervision():
    """Training only through SUM(label) per grid row (the soft SUM of the
    expected labels): the relaxed answer, the expected label sums of the
    held-out rows, must beat the label-free estimate and the untrained
    network; the exact swap's accuracy is reported (a sum pins the mean of
    each image's class distribution, not its mode)."""
    from paper_2211_02753_amd import _lib as L
    from paper_2211_02753_amd import query as Q
    from paper_2211_02753_amd.cnn import DigitCNN, GridQueryTrainer

    n_rows, cpr, n_train_rows = 30_000, 4, 25_000
    col = gen.image_column(n_images=n_rows * cpr)
    images = torch.from_numpy(col["images"]).to(DEV)
    labels = torch.from_numpy(col["label"]).to(DEV)
    grid_row = torch.from_numpy(col["grid_row"]).to(DEV)
    r = Q.GroupbyQuery(n_rows * cpr, keys=[Q.Key(grid_row, 0, n_rows)], expr=L.EXPR_COL, a=Q.Operand(labels))()
    truth = torch.zeros(n_rows, dtype=torch.int64, device=DEV)
    truth[r["k0"]] = r["sum"]
    target = truth.to(torch.float32)
    model = DigitCNN(gen.cnn_init(), device=DEV, max_batch=1024)
    test_img = images[n_train_rows * cpr:]

    def soft_row_err():
        es = []
        for a in range(0, test_img.shape[0], 1024):
            _, e = model.forward(test_img[a:a + 1024])
            es.append(e[:min(1024, test_img.shape[0] - a)].double().clone())
        rows = torch.cat(es).view(-1, cpr).sum(1)
        return (rows - truth[n_train_rows:].double()).abs().mean().item()

    err_untrained = soft_row_err()
    err_label_free = (truth[n_train_rows:].double() - target[:n_train_rows].mean().item()).abs().mean().item()
    trainer = GridQueryTrainer(model, cells_per_row=cpr, lr=5e-4, mode="sum")
    rows_per_batch = 64
    order = np.random.default_rng(1).permutation(n_train_rows // rows_per_batch)
    for epoch in range(2):
        for bi in order:
            r0 = int(bi) * rows_per_batch
            loss = trainer.step(images[r0 * cpr:(r0 + rows_per_batch) * cpr], target[r0:r0 + rows_per_batch])
        print("sum supervision epoch", epoch, "loss", float(loss.item()), flush=True)
    err_soft = soft_row_err()
    pred = model.label_column(images)
    img_acc = (pred[n_train_rows * cpr:] == labels[n_train_rows * cpr:]).double().mean().item()
    r = Q.GroupbyQuery(n_rows * cpr, keys=[Q.Key(grid_row, 0, n_rows)], expr=L.EXPR_COL, a=Q.Operand(pred))()
    swap = torch.zeros(n_rows, dtype=torch.int64, device=DEV)
    swap[r["k0"]] = r["sum"]
    err_swap = (swap[n_train_rows:] - truth[n_train_rows:]).abs().double().mean().item()
    print(f"SUM supervision: soft row |err| {err_soft:.3f} (untrained {err_untrained:.3f}, label-free "
          f"{err_label_free:.3f}); exact swap row |err| {err_swap:.3f}, held-out image accuracy {img_acc:.4f}", flush=True)
    assert err_soft < err_label_free and err_soft < err_untrained
