"""Writes mn_full_digest.json: the exact answer of the many-to-many join
aggregate over its full workload (two 20M-row tables with Zipf(0.8) keys over
2M values, SUM(l.payload * r.payload) and COUNT(*) GROUP BY l.gkey over 1M
groups), computed by the oracle's per-group enumeration of every joined pair
(about 1.2e11 pairs, never the pre-aggregated form), split over processes by
group range.  Stored: the SHA-256 of the canonical table (gkey, sum, count as
little-endian int64 triples, groups with COUNT > 0 in key order), its size and
totals, and the top-100 rows by (SUM desc, gkey asc).

Run: python tests/golden/make_mn_digest.py [workers]   (calls only oracle/ and
the shared input generator; several minutes of CPU time)."""
import hashlib
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import tdp_datagen as gen  # noqa: E402

N_GROUPS = 1_000_000
_MO = None


def _init():
    global _MO
    l, r = gen.mn_join_tables()
    _MO = oracle.MNGroupOracle(l["key"], l["gkey"], l["payload"], r["key"], r["payload"])


def _range(bounds):
    a, b = bounds
    out = np.zeros((b - a, 2), np.int64)
    for g in range(a, b):
        out[g - a] = _MO.group(g)
    return a, out


def table_digest(k0, sums, counts):
    """SHA-256 of the canonical (gkey, sum, count) int64 triples."""
    t = np.stack([np.asarray(k0, np.int64), np.asarray(sums, np.int64), np.asarray(counts, np.int64)], axis=1)
    return hashlib.sha256(np.ascontiguousarray(t).astype("<i8").tobytes()).hexdigest()


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    step = 5000
    chunks = [(a, min(a + step, N_GROUPS)) for a in range(0, N_GROUPS, step)]
    res = np.zeros((N_GROUPS, 2), np.int64)
    with mp.get_context("fork").Pool(workers, initializer=_init) as pool:
        for i, (a, part) in enumerate(pool.imap_unordered(_range, chunks)):
            res[a:a + len(part)] = part
            if i % 20 == 0:
                print(f"{i + 1}/{len(chunks)} ranges", flush=True)
    keep = np.nonzero(res[:, 1] > 0)[0]
    k0, sums, counts = keep.astype(np.int64), res[keep, 0], res[keep, 1]
    top = oracle.topk(k0, sums, 100)
    out = {
        "workload": "many-to-many join: 20M x 20M rows, keys Zipf(0.8) over 2M values, GROUP BY l.gkey (1M groups)",
        "source": "oracle per-group enumeration of every joined pair (orc_mn_group)",
        "groups": int(len(keep)),
        "count_total": int(counts.sum()),
        "sum_total_mod_2_64": int(sums.astype(np.uint64).sum(dtype=np.uint64)),
        "sha256": table_digest(k0, sums, counts),
        "top100": [[int(k0[i]), int(sums[i]), int(counts[i])] for i in top],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mn_full_digest.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["groups"], out["count_total"], out["sha256"])


if __name__ == "__main__":
    main()
