// CPU oracle for the tensor-program relational operators, their relaxed
// (differentiable) versions and the small image classifier.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
// statement of what every operator computes.  Only the test suite, the smoke
// check and the benchmark's CPU-baseline leg load it.  It shares no code,
// header, table or helper with the GPU library and includes nothing from it.
//
// Paper: "The Tensor Data Platform: Towards an AI-centric Database System"
// (arXiv 2211.02753).  Section references below are to that paper.  Where
// the paper is silent (it never defines a join, a hash table or a sort; it
// defers operator internals to its TQP citation in Section 2), the oracle
// takes standard SQL semantics, and the reading is named in the comment.
//
// Conventions: integers are widened to int64 before comparison or
// arithmetic; SUM is computed in uint64 so that it wraps modulo 2^64 without
// undefined behaviour, and an __int128 shadow sum reports groups that wrapped.
// Floating point is float64 throughout, on float32 (or bfloat16-valued float32)
// inputs.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

enum { O_I8 = 1, O_I32 = 2, O_I64 = 3, O_F32 = 4 };
enum { O_LT = 0, O_LE = 1, O_GT = 2, O_GE = 3, O_EQ = 4, O_NE = 5 };
enum { O_EXPR_COL = 0, O_EXPR_MUL = 1, O_EXPR_MUL_CONST_SUB = 2, O_EXPR_NONE = 3 };

int64_t read_int(const void* col, int dtype, int64_t i) {
    switch (dtype) {
        case O_I8: return (int64_t)((const int8_t*)col)[i];
        case O_I32: return (int64_t)((const int32_t*)col)[i];
        case O_I64: return ((const int64_t*)col)[i];
        default: return 0;
    }
}

bool compare(int64_t a, int cmp, int64_t b) {
    switch (cmp) {
        case O_LT: return a < b;
        case O_LE: return a <= b;
        case O_GT: return a > b;
        case O_GE: return a >= b;
        case O_EQ: return a == b;
        case O_NE: return a != b;
    }
    return false;
}

struct Acc {
    uint64_t sum = 0;      // wraps modulo 2^64
    int64_t count = 0;
    __int128 wide = 0;     // exact sum, to report wrap
};

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Exact operators
// ---------------------------------------------------------------------------

// WHERE col <cmp> literal (Section 2 query processor; the filter of the
// Section 5.2 document query).  Candidates are rows 0..n-1, or the rows
// listed in sel (ascending) when sel is not null.  Survivors are written
// in candidate order, i.e. ascending row ids.  Returns their number.
int64_t orc_filter(const void* col, int dtype, int64_t n, int cmp, int64_t lit,
                   const int32_t* sel, int64_t n_sel, int32_t* out) {
    int64_t m = 0;
    int64_t n_cand = sel ? n_sel : n;
    for (int64_t j = 0; j < n_cand; ++j) {
        int64_t row = sel ? (int64_t)sel[j] : j;
        if (compare(read_int(col, dtype, row), cmp, lit)) out[m++] = (int32_t)row;
    }
    return m;
}

// The same WHERE on a float32 column: x op lit with the literal rounded to
// float32 first (the comparison a float32 engine makes).
int64_t orc_filter_f32(const float* col, int64_t n, int cmp, double lit, const int32_t* sel, int64_t n_sel,
                       int32_t* out) {
    const double l = (double)(float)lit;
    int64_t m = 0;
    int64_t n_cand = sel ? n_sel : n;
    for (int64_t j = 0; j < n_cand; ++j) {
        int64_t row = sel ? (int64_t)sel[j] : j;
        const double x = (double)col[row];
        bool keep = false;
        switch (cmp) {
            case O_LT: keep = x < l; break;
            case O_LE: keep = x <= l; break;
            case O_GT: keep = x > l; break;
            case O_GE: keep = x >= l; break;
            case O_EQ: keep = x == l; break;
            case O_NE: keep = x != l; break;
        }
        if (keep) out[m++] = (int32_t)row;
    }
    return m;
}

// Inner equi-join probe.key = build.key (standard SQL semantics; the paper
// gives none).  Every (probe row, build row) pair with equal keys is one
// output row; duplicates on both sides give their cross product.  Probe
// candidates are all rows or those in psel.  Pairs are written in probe
// candidate order, then ascending build row, up to cap; the return value is
// the total number of pairs.  Steps: sort build rows by (key, row), then for
// each probe row take the equal range.
int64_t orc_join_pairs(const int32_t* bkey, int64_t nb, const int32_t* pkey, int64_t np,
                       const int32_t* psel, int64_t n_psel, int64_t cap,
                       int32_t* out_probe, int32_t* out_build) {
    std::vector<std::pair<int32_t, int32_t>> b((size_t)nb);
    for (int64_t j = 0; j < nb; ++j) b[(size_t)j] = {bkey[j], (int32_t)j};
    std::sort(b.begin(), b.end());
    int64_t total = 0;
    int64_t n_cand = psel ? n_psel : np;
    for (int64_t c = 0; c < n_cand; ++c) {
        int32_t i = psel ? psel[c] : (int32_t)c;
        auto lo = std::lower_bound(b.begin(), b.end(), std::make_pair(pkey[i], INT32_MIN));
        for (auto it = lo; it != b.end() && it->first == pkey[i]; ++it) {
            if (total < cap) {
                out_probe[total] = i;
                out_build[total] = it->second;
            }
            ++total;
        }
    }
    return total;
}

// SELECT k0[, k1], SUM(e), COUNT(*), AVG(e) FROM fact [JOIN dim ON fk = pk]
// WHERE pred GROUP BY k0[, k1]   (Section 2 and the Section 3 grouped
// COUNT example; AVG as in the Section 5.2 document query).
//
// Steps, in order: take the candidate rows (all fact rows, or sel_in);
// filter them on pred (if pred_col is given);
// join every surviving fact row with every dim row of equal key (if fk is
// given); for each joined pair read the group keys and evaluate e from the
// fact (side 0) or dim (side 1) column; group the pairs by key tuple.
//   e = a            (expr 0)
//   e = a * b        (expr 1)
//   e = a * (K - b)  (expr 2)
//   none             (expr 3: only COUNT is meaningful, SUM is 0)
// SUM wraps modulo 2^64; AVG = (double)SUM / (double)COUNT with one rounding
// each.  Groups come out in ascending (signed) key order, only those with
// COUNT > 0.  wrapped[g] is 1 where the exact sum left the int64 range.
// Returns the number of groups (outputs are written up to cap groups).
int64_t orc_query(int64_t n_fact, const int32_t* sel_in, int64_t n_sel_in,
                  const void* pred_col, int pred_dtype, int pred_cmp, int64_t pred_lit,
                  const int32_t* fk, const int32_t* pk, int64_t n_dim,
                  int n_keys, const void* k0, int k0_dtype, int k0_side,
                  const void* k1, int k1_dtype, int k1_side,
                  int expr, const void* a, int a_dtype, int a_side,
                  const void* b, int b_dtype, int b_side, int64_t K,
                  int64_t cap, int64_t* out_k0, int64_t* out_k1, int64_t* out_sum,
                  int64_t* out_count, double* out_avg, int32_t* out_wrapped) {
    // 1. filter (the candidates are every fact row, or the ascending list
    // sel_in left by earlier conjuncts of the WHERE clause)
    std::vector<int32_t> sel((size_t)(sel_in ? n_sel_in : n_fact));
    int64_t n_sel = (int64_t)sel.size();
    if (pred_col) {
        n_sel = orc_filter(pred_col, pred_dtype, n_fact, pred_cmp, pred_lit, sel_in, n_sel_in, sel.data());
    } else {
        for (int64_t i = 0; i < n_sel; ++i) sel[(size_t)i] = sel_in ? sel_in[i] : (int32_t)i;
    }
    sel.resize((size_t)n_sel);
    // 2. join
    std::vector<int32_t> pf, pd;
    if (fk) {
        int64_t total = orc_join_pairs(pk, n_dim, fk, n_fact, sel.data(), n_sel, 0, nullptr, nullptr);
        pf.resize((size_t)total);
        pd.resize((size_t)total);
        orc_join_pairs(pk, n_dim, fk, n_fact, sel.data(), n_sel, total, pf.data(), pd.data());
    } else {
        pf = sel;
        pd.assign(sel.size(), -1);
    }
    // 3. group
    std::map<std::pair<int64_t, int64_t>, Acc> groups;
    for (size_t p = 0; p < pf.size(); ++p) {
        int64_t row[2] = {pf[p], pd[p]};
        int64_t key0 = read_int(k0, k0_dtype, row[k0_side]);
        int64_t key1 = n_keys > 1 ? read_int(k1, k1_dtype, row[k1_side]) : 0;
        int64_t e = 0;
        if (expr == O_EXPR_COL) {
            e = read_int(a, a_dtype, row[a_side]);
        } else if (expr == O_EXPR_MUL) {
            e = (int64_t)((uint64_t)read_int(a, a_dtype, row[a_side]) *
                          (uint64_t)read_int(b, b_dtype, row[b_side]));
        } else if (expr == O_EXPR_MUL_CONST_SUB) {
            uint64_t kb = (uint64_t)K - (uint64_t)read_int(b, b_dtype, row[b_side]);
            e = (int64_t)((uint64_t)read_int(a, a_dtype, row[a_side]) * kb);
        }
        Acc& g = groups[{key0, key1}];
        g.sum += (uint64_t)e;
        g.count += 1;
        g.wide += (__int128)e;
    }
    int64_t m = 0;
    for (auto& kv : groups) {
        if (m < cap) {
            out_k0[m] = kv.first.first;
            if (out_k1) out_k1[m] = kv.first.second;
            int64_t s = (int64_t)kv.second.sum;
            out_sum[m] = s;
            out_count[m] = kv.second.count;
            out_avg[m] = (double)s / (double)kv.second.count;
            out_wrapped[m] = (kv.second.wide != (__int128)s) ? 1 : 0;
        }
        ++m;
    }
    return m;
}

// One group of the many-to-many join aggregate, by enumeration of its pairs:
// SUM over pairs (l, r) with l.gkey = g and l.key = r.key of
// l.payload * r.payload (mod 2^64), and the number of such pairs.
// The right side must be given sorted by key (rkey ascending, rpay aligned),
// which is how the caller prepares it once for many groups.
void orc_mn_group(int64_t g, const int32_t* lkey, const int32_t* lgkey, const int64_t* lpay,
                  int64_t nl, const int32_t* rkey_sorted, const int64_t* rpay_sorted, int64_t nr,
                  int64_t* out_sum, int64_t* out_count) {
    uint64_t s = 0;
    int64_t c = 0;
    for (int64_t i = 0; i < nl; ++i) {
        if (lgkey[i] != g) continue;
        const int32_t* lo = std::lower_bound(rkey_sorted, rkey_sorted + nr, lkey[i]);
        for (const int32_t* p = lo; p != rkey_sorted + nr && *p == lkey[i]; ++p) {
            s += (uint64_t)lpay[i] * (uint64_t)rpay_sorted[p - rkey_sorted];
            ++c;
        }
    }
    *out_sum = (int64_t)s;
    *out_count = c;
}

// Exact top-k of a group table: the k groups of largest SUM, ties broken by
// ascending key.  Writes group indices in rank order; returns min(k, n).
int64_t orc_topk(const int64_t* keys, const int64_t* sums, int64_t n, int64_t k, int64_t* out_idx) {
    std::vector<int64_t> idx((size_t)n);
    for (int64_t i = 0; i < n; ++i) idx[(size_t)i] = i;
    std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
        if (sums[x] != sums[y]) return sums[x] > sums[y];
        return keys[x] < keys[y];
    });
    int64_t m = std::min(n, k);
    for (int64_t i = 0; i < m; ++i) out_idx[i] = idx[(size_t)i];
    return m;
}

// ---------------------------------------------------------------------------
// Relaxed operators (Section 4: a logistic function stands in for the step
// of a comparison; grouped soft aggregation uses only + and *).
// ---------------------------------------------------------------------------

static double logistic(double z) {
    if (z >= 0) return 1.0 / (1.0 + std::exp(-z));
    double e = std::exp(z);
    return e / (1.0 + e);
}

// w_i = sigma((c - x_i) / tau): the logistic relaxation of x_i < c.
void orc_soft_filter(const float* x, int64_t n, double c, double tau, double* w) {
    for (int64_t i = 0; i < n; ++i) w[i] = logistic((c - (double)x[i]) / tau);
}

// Backward of the soft filter given dL/dw: dL/dx_i = -dw_i w_i (1 - w_i) / tau
// and dL/dc = sum_i dw_i w_i (1 - w_i) / tau.  With z_i = (c - x_i) / tau,
// dw_i/dtau = -w_i (1 - w_i) z_i / tau, so dL/dtau = -sum_i dw_i w_i (1 - w_i) z_i / tau
// (the temperature as a learnable parameter).  dx and dtau may be null.
void orc_soft_filter_bwd(const float* x, int64_t n, double c, double tau, const double* dw,
                         double* dx, double* dc, double* dtau) {
    double acc = 0.0, acc_tau = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double z = (c - (double)x[i]) / tau;
        double w = logistic(z);
        double t = dw[i] * w * (1.0 - w) / tau;
        if (dx) dx[i] = -t;
        acc += t;
        acc_tau -= t * z;
    }
    *dc = acc;
    if (dtau) *dtau = acc_tau;
}

// Soft WHERE clause of J conjuncts with a grouped SUM: the relaxed form of
//   SELECT g, SUM(v) FROM t WHERE x_1 op_1 c_1 AND ... AND x_J op_J c_J GROUP BY g
// that a trainable query runs (Section 4: a logistic function in place of
// each comparison's step, the conjunction as the product of its terms, and
// the grouped sum using only + and *).  Conjunct j is
//   sigma_j(i) = sigma(z_ij),  z_ij = s_j (c_j - x_ij) / tau_j,
// with s_j = +1 for "<" and "<=" (x below c) and -1 for ">" and ">=".  Then
//   w_i = prod_j sigma_j(i),   S[g] = sum over rows with gid_i = g of w_i v_i
// (v = 1 when null: the soft COUNT).  x is row-major by conjunct: x[j * n + i].
void orc_soft_where(const double* x, const int* s, const double* c, const double* tau, int J, const double* v,
                    const int64_t* gid, int64_t n, int64_t G, double* S) {
    for (int64_t k = 0; k < G; ++k) S[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double w = 1.0;
        for (int j = 0; j < J; ++j) w *= logistic(s[j] * (c[j] - x[(int64_t)j * n + i]) / tau[j]);
        S[gid[i]] += w * (v ? v[i] : 1.0);
    }
}

// Its backward from dS[G].  With d_i = dS[gid_i] v_i and
// dw_i/dc_j = w_i (1 - sigma_j(i)) s_j / tau_j,
// dw_i/dtau_j = -w_i (1 - sigma_j(i)) z_ij / tau_j:
//   dc[j] = sum_i d_i w_i (1 - sigma_j(i)) s_j / tau_j
//   dtau[j] = -sum_i d_i w_i (1 - sigma_j(i)) z_ij / tau_j
//   dv[i] = dS[gid_i] w_i            (dv and dtau may be null)
void orc_soft_where_bwd(const double* x, const int* s, const double* c, const double* tau, int J, const double* v,
                        const int64_t* gid, int64_t n, const double* dS, double* dc, double* dtau, double* dv) {
    for (int j = 0; j < J; ++j) {
        dc[j] = 0.0;
        if (dtau) dtau[j] = 0.0;
    }
    std::vector<double> z((size_t)J), sg((size_t)J);
    for (int64_t i = 0; i < n; ++i) {
        double w = 1.0;
        for (int j = 0; j < J; ++j) {
            z[(size_t)j] = s[j] * (c[j] - x[(int64_t)j * n + i]) / tau[j];
            sg[(size_t)j] = logistic(z[(size_t)j]);
            w *= sg[(size_t)j];
        }
        const double vi = v ? v[i] : 1.0;
        const double d = dS[gid[i]] * vi;
        if (dv) dv[i] = dS[gid[i]] * w;
        for (int j = 0; j < J; ++j) {
            // 1 - sigma(z) = sigma(-z), taken from the logistic itself
            const double t = d * w * logistic(-z[(size_t)j]) / tau[j];
            dc[j] += t * s[j];
            if (dtau) dtau[j] -= t * z[(size_t)j];
        }
    }
}

// S[g, k] = sum over rows i with g_i = g of w_i * v[i, k] (w = 1 when null).
// Rows are visited in order.  Empty groups are 0.
void orc_soft_groupby(const int32_t* g, const double* w, const double* v, int64_t n, int K, int G,
                      double* S) {
    for (int64_t j = 0; j < (int64_t)G * K; ++j) S[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double wi = w ? w[i] : 1.0;
        for (int k = 0; k < K; ++k) S[(int64_t)g[i] * K + k] += wi * v[i * K + k];
    }
}

// Backward of the soft group-by: dv[i, k] = dS[g_i, k] w_i and
// dw_i = sum_k dS[g_i, k] v[i, k].  Either output may be null.
void orc_soft_groupby_bwd(const int32_t* g, const double* w, const double* v, const double* dS,
                          int64_t n, int K, double* dw, double* dv) {
    for (int64_t i = 0; i < n; ++i) {
        double wi = w ? w[i] : 1.0;
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            double d = dS[(int64_t)g[i] * K + k];
            if (dv) dv[i * K + k] = d * wi;
            acc += d * v[i * K + k];
        }
        if (dw) dw[i] = acc;
    }
}

// Soft COUNT grouped by two probability-encoded attributes.  Section 4
// counts on probability-encoded data with additions and multiplications
// only; the grid-of-images query of Sections 3 and 5.5 groups COUNT(*) by
// two predicted attributes (digit and size), each a probability vector per
// tile.  A tile contributes to the (a, b) cell the probability that it has
// value a in the first attribute and b in the second, p[i][a] q[i][b] (the
// two classifiers are independent given the tile), so
//   S[g][a][b] = sum over the rows i of segment g of p[i][a] * q[i][b].
// Segment g holds rows seg[g] .. seg[g+1]-1 (the tiles of one image);
// seg == null is one segment of all n rows.  q == null means q = 1 with
// K2 = 1, the soft COUNT per class of p alone.  Segments with
// seg[g] > seg[g+1] or outside [0, n] are left 0.
void orc_soft_pe_groupby(const int64_t* seg, int G, const double* p, int K1, const double* q, int K2, int64_t n,
                         double* S) {
    const int64_t cells = (int64_t)K1 * K2;
    for (int64_t j = 0; j < (int64_t)G * cells; ++j) S[j] = 0.0;
    for (int g = 0; g < G; ++g) {
        const int64_t lo = seg ? seg[g] : 0, hi = seg ? seg[g + 1] : n;
        if (lo < 0 || hi > n || hi < lo) continue;
        for (int64_t i = lo; i < hi; ++i)
            for (int a = 0; a < K1; ++a)
                for (int b = 0; b < K2; ++b)
                    S[g * cells + a * K2 + b] += p[i * K1 + a] * (q ? q[i * K2 + b] : 1.0);
    }
}

// Backward of the grouped soft COUNT from dS[G][K1][K2], for row i of
// segment g:  dp[i][a] = sum_b dS[g][a][b] q[i][b]  and
// dq[i][b] = sum_a dS[g][a][b] p[i][a].  Rows outside every segment get 0.
void orc_soft_pe_groupby_bwd(const int64_t* seg, int G, const double* p, int K1, const double* q, int K2, int64_t n,
                             const double* dS, double* dp, double* dq) {
    const int64_t cells = (int64_t)K1 * K2;
    if (dp)
        for (int64_t j = 0; j < n * K1; ++j) dp[j] = 0.0;
    if (dq)
        for (int64_t j = 0; j < n * K2; ++j) dq[j] = 0.0;
    for (int g = 0; g < G; ++g) {
        const int64_t lo = seg ? seg[g] : 0, hi = seg ? seg[g + 1] : n;
        if (lo < 0 || hi > n || hi < lo) continue;
        for (int64_t i = lo; i < hi; ++i)
            for (int a = 0; a < K1; ++a)
                for (int b = 0; b < K2; ++b) {
                    const double d = dS[g * cells + a * K2 + b];
                    if (dp) dp[i * K1 + a] += d * (q ? q[i * K2 + b] : 1.0);
                    if (dq) dq[i * K2 + b] += d * p[i * K1 + a];
                }
    }
}

// Learning from label proportions (Section 5.3): a linear classifier
// table-valued function labels every row of a bag, and a grouped COUNT per
// (bag, class) is the query answer the training compares with the bags'
// released label counts.  Relaxed (Section 4), the classifier outputs the
// class probabilities p_i = softmax(W x_i + b) and the COUNT of class c in
// bag j is the soft count
//   S[j][c] = sum over the rows i of bag j of p_i[c].
// Bags are consecutive runs of `bag` rows (the last one may be shorter).
// X is row-major [n][F], W is [C][F], S is [n_bags][C].
static void llp_probs(const float* x, const double* W, const double* b, int F, int C, double* p) {
    double zmax = -1e300;
    for (int c = 0; c < C; ++c) {
        double z = b[c];
        for (int f = 0; f < F; ++f) z += W[c * F + f] * (double)x[f];
        p[c] = z;
        zmax = std::max(zmax, z);
    }
    double sum = 0.0;
    for (int c = 0; c < C; ++c) {
        p[c] = std::exp(p[c] - zmax);
        sum += p[c];
    }
    for (int c = 0; c < C; ++c) p[c] /= sum;
}

void orc_llp_forward(const float* X, int64_t n, int F, const double* W, const double* b, int C, int64_t bag,
                     double* S) {
    const int64_t n_bags = (n + bag - 1) / bag;
    for (int64_t j = 0; j < n_bags * C; ++j) S[j] = 0.0;
    std::vector<double> p((size_t)C);
    for (int64_t i = 0; i < n; ++i) {
        llp_probs(X + i * F, W, b, F, C, p.data());
        for (int c = 0; c < C; ++c) S[(i / bag) * C + c] += p[(size_t)c];
    }
}

// Its backward from dS[n_bags][C]: with dp_i = dS[bag of i] and the softmax
// Jacobian, dz_i[c] = p_i[c] (dp_i[c] - sum_k p_i[k] dp_i[k]); then
// dW[c][f] = sum_i dz_i[c] x_i[f] and db[c] = sum_i dz_i[c].
void orc_llp_backward(const float* X, int64_t n, int F, const double* W, const double* b, int C, int64_t bag,
                      const double* dS, double* dW, double* db) {
    for (int j = 0; j < C * F; ++j) dW[j] = 0.0;
    for (int c = 0; c < C; ++c) db[c] = 0.0;
    std::vector<double> p((size_t)C);
    for (int64_t i = 0; i < n; ++i) {
        llp_probs(X + i * F, W, b, F, C, p.data());
        const double* dp = dS + (i / bag) * C;
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += p[(size_t)c] * dp[c];
        for (int c = 0; c < C; ++c) {
            const double dz = p[(size_t)c] * (dp[c] - s);
            db[c] += dz;
            for (int f = 0; f < F; ++f) dW[c * F + f] += dz * (double)X[i * F + f];
        }
    }
}

// The exact swap at inference: the classifier's label is the class of the
// largest logit (ties to the smallest class).  The logit is accumulated in
// float64 as z = b, then z = fma(W[c][f], x[f], z) for f = 0, 1, ... (one
// rounding per term), so that an integer decision made from it is the same
// on any machine that follows the same steps.
void orc_llp_predict(const float* X, int64_t n, int F, const double* W, const double* b, int C, int8_t* out) {
    for (int64_t i = 0; i < n; ++i) {
        int best = 0;
        double bz = 0.0;
        for (int c = 0; c < C; ++c) {
            double z = b[c];
            for (int f = 0; f < F; ++f) z = std::fma(W[c * F + f], (double)X[i * F + f], z);
            if (c == 0 || z > bz) {
                best = c;
                bz = z;
            }
        }
        out[i] = (int8_t)best;
    }
}

// Mean squared error over G groups (the training loop of Section 3 takes
// the mean of squared differences): L = (1/G) sum (S - T)^2,
// dL/dS = 2 (S - T) / G.
double orc_mse(const double* S, const double* T, int64_t G, double* dS) {
    double L = 0.0;
    for (int64_t j = 0; j < G; ++j) {
        double d = S[j] - T[j];
        L += d * d;
        if (dS) dS[j] = 2.0 * d / (double)G;
    }
    return L / (double)G;
}

// ---------------------------------------------------------------------------
// Image classifier layers (the classifier inside the table-valued function of
// Section 3; its architecture is not given by the paper).  Activations are
// NHWC, weights [Cout][3][3][Cin], valid padding, stride 1.  Inputs are float
// arrays whose values the caller has already rounded to bfloat16 where the
// GPU computes in bfloat16; all sums are float64.
// ---------------------------------------------------------------------------

// float -> bfloat16 -> float with round-to-nearest-even; NaN stays NaN
// (quiet), infinities stay infinities.
void orc_bf16_round(const float* in, float* out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        uint32_t u;
        std::memcpy(&u, &in[i], 4);
        uint32_t r;
        if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0) {
            r = (u | 0x00400000u) & 0xFFFF0000u;
        } else {
            uint32_t lsb = (u >> 16) & 1u;
            r = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
        }
        std::memcpy(&out[i], &r, 4);
    }
}

// y[b, oy, ox, co] = bias[co] + sum_{ky, kx, ci} x[b, oy+ky, ox+kx, ci] w[co, ky, kx, ci]
// (then max(0, .) when relu).  Output is (H-2) x (W-2).
void orc_conv3x3_fwd(const float* x, const float* w, const float* bias, int B, int H, int W, int Cin,
                     int Cout, int relu, double* y) {
    int Ho = H - 2, Wo = W - 2;
    for (int b = 0; b < B; ++b)
        for (int oy = 0; oy < Ho; ++oy)
            for (int ox = 0; ox < Wo; ++ox)
                for (int co = 0; co < Cout; ++co) {
                    double acc = bias ? (double)bias[co] : 0.0;
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            for (int ci = 0; ci < Cin; ++ci)
                                acc += (double)x[(((int64_t)b * H + oy + ky) * W + ox + kx) * Cin + ci] *
                                       (double)w[((co * 3 + ky) * 3 + kx) * Cin + ci];
                    if (relu && acc < 0.0) acc = 0.0;
                    y[(((int64_t)b * Ho + oy) * Wo + ox) * Cout + co] = acc;
                }
}

// Gradient of the convolution with respect to its input:
// dx[b, iy, ix, ci] = sum over (oy, ox, ky, kx) with oy+ky = iy, ox+kx = ix of
// dy[b, oy, ox, co] w[co, ky, kx, ci].
void orc_conv3x3_dgrad(const float* dy, const float* w, int B, int H, int W, int Cin, int Cout,
                       double* dx) {
    int Ho = H - 2, Wo = W - 2;
    for (int64_t j = 0; j < (int64_t)B * H * W * Cin; ++j) dx[j] = 0.0;
    for (int b = 0; b < B; ++b)
        for (int oy = 0; oy < Ho; ++oy)
            for (int ox = 0; ox < Wo; ++ox)
                for (int co = 0; co < Cout; ++co) {
                    double d = dy[(((int64_t)b * Ho + oy) * Wo + ox) * Cout + co];
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            for (int ci = 0; ci < Cin; ++ci)
                                dx[(((int64_t)b * H + oy + ky) * W + ox + kx) * Cin + ci] +=
                                    d * (double)w[((co * 3 + ky) * 3 + kx) * Cin + ci];
                }
}

// Gradient with respect to the weights and bias:
// dw[co, ky, kx, ci] = sum_{b, oy, ox} dy[b, oy, ox, co] x[b, oy+ky, ox+kx, ci];
// db[co] = sum_{b, oy, ox} dy[b, oy, ox, co].
void orc_conv3x3_wgrad(const float* x, const float* dy, int B, int H, int W, int Cin, int Cout,
                       double* dw, double* db) {
    int Ho = H - 2, Wo = W - 2;
    for (int j = 0; j < Cout * 9 * Cin; ++j) dw[j] = 0.0;
    for (int j = 0; j < Cout; ++j) db[j] = 0.0;
    for (int b = 0; b < B; ++b)
        for (int oy = 0; oy < Ho; ++oy)
            for (int ox = 0; ox < Wo; ++ox)
                for (int co = 0; co < Cout; ++co) {
                    double d = dy[(((int64_t)b * Ho + oy) * Wo + ox) * Cout + co];
                    db[co] += d;
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            for (int ci = 0; ci < Cin; ++ci)
                                dw[((co * 3 + ky) * 3 + kx) * Cin + ci] +=
                                    d * (double)x[(((int64_t)b * H + oy + ky) * W + ox + kx) * Cin + ci];
                }
}

// 2x2 max pooling, stride 2 (H, W even).  The gradient goes to the first
// maximum of each window in (dy, dx) row-major order.
void orc_maxpool2_fwd(const float* x, int B, int H, int W, int C, double* y) {
    int Ho = H / 2, Wo = W / 2;
    for (int b = 0; b < B; ++b)
        for (int oy = 0; oy < Ho; ++oy)
            for (int ox = 0; ox < Wo; ++ox)
                for (int c = 0; c < C; ++c) {
                    double m = -INFINITY;
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx)
                            m = std::max(m, (double)x[(((int64_t)b * H + 2 * oy + dy) * W + 2 * ox + dx) * C + c]);
                    y[(((int64_t)b * Ho + oy) * Wo + ox) * C + c] = m;
                }
}

void orc_maxpool2_bwd(const float* x, const float* dy, int B, int H, int W, int C, double* dx) {
    int Ho = H / 2, Wo = W / 2;
    for (int64_t j = 0; j < (int64_t)B * H * W * C; ++j) dx[j] = 0.0;
    for (int b = 0; b < B; ++b)
        for (int oy = 0; oy < Ho; ++oy)
            for (int ox = 0; ox < Wo; ++ox)
                for (int c = 0; c < C; ++c) {
                    int64_t best = -1;
                    double m = -INFINITY;
                    for (int ddy = 0; ddy < 2; ++ddy)
                        for (int ddx = 0; ddx < 2; ++ddx) {
                            int64_t at = (((int64_t)b * H + 2 * oy + ddy) * W + 2 * ox + ddx) * C + c;
                            if (best < 0 || (double)x[at] > m) {
                                m = x[at];
                                best = at;
                            }
                        }
                    dx[best] += dy[(((int64_t)b * Ho + oy) * Wo + ox) * C + c];
                }
}

// Fully connected layer: y[m, n] = b[n] + sum_k x[m, k] w[n, k] (relu optional).
void orc_linear_fwd(const float* x, const float* w, const float* bias, int M, int N, int K, int relu,
                    double* y) {
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < N; ++n) {
            double acc = bias ? (double)bias[n] : 0.0;
            for (int k = 0; k < K; ++k) acc += (double)x[(int64_t)m * K + k] * (double)w[(int64_t)n * K + k];
            if (relu && acc < 0.0) acc = 0.0;
            y[(int64_t)m * N + n] = acc;
        }
}

// dx[m, k] = sum_n dy[m, n] w[n, k]; dw[n, k] = sum_m dy[m, n] x[m, k];
// db[n] = sum_m dy[m, n].  Any output may be null.
void orc_linear_bwd(const float* x, const float* w, const float* dy, int M, int N, int K, double* dx,
                    double* dw, double* db) {
    if (dx)
        for (int m = 0; m < M; ++m)
            for (int k = 0; k < K; ++k) {
                double acc = 0.0;
                for (int n = 0; n < N; ++n) acc += (double)dy[(int64_t)m * N + n] * (double)w[(int64_t)n * K + k];
                dx[(int64_t)m * K + k] = acc;
            }
    if (dw)
        for (int n = 0; n < N; ++n)
            for (int k = 0; k < K; ++k) {
                double acc = 0.0;
                for (int m = 0; m < M; ++m) acc += (double)dy[(int64_t)m * N + n] * (double)x[(int64_t)m * K + k];
                dw[(int64_t)n * K + k] = acc;
            }
    if (db)
        for (int n = 0; n < N; ++n) {
            double acc = 0.0;
            for (int m = 0; m < M; ++m) acc += dy[(int64_t)m * N + n];
            db[n] = acc;
        }
}

// Softmax over K classes as the smooth stand-in for argmax (Section 4), and
// the expected label E = sum_k k p_k, which a soft SUM of the label column
// over probability-encoded rows reduces to (only + and *).
void orc_softmax_expect(const float* logits, int M, int K, double* p, double* e) {
    for (int m = 0; m < M; ++m) {
        double mx = -INFINITY;
        for (int k = 0; k < K; ++k) mx = std::max(mx, (double)logits[(int64_t)m * K + k]);
        double z = 0.0;
        for (int k = 0; k < K; ++k) z += std::exp((double)logits[(int64_t)m * K + k] - mx);
        double ev = 0.0;
        for (int k = 0; k < K; ++k) {
            double pk = std::exp((double)logits[(int64_t)m * K + k] - mx) / z;
            p[(int64_t)m * K + k] = pk;
            ev += (double)k * pk;
        }
        if (e) e[m] = ev;
    }
}

// Backward of E with respect to the logits: dz_k = dE p_k (k - E).
void orc_softmax_expect_bwd(const double* p, const double* dE, int M, int K, double* dz) {
    for (int m = 0; m < M; ++m) {
        double ev = 0.0;
        for (int k = 0; k < K; ++k) ev += (double)k * p[(int64_t)m * K + k];
        for (int k = 0; k < K; ++k)
            dz[(int64_t)m * K + k] = dE[m] * p[(int64_t)m * K + k] * ((double)k - ev);
    }
}

// Backward of p = softmax(z) for a general upstream gradient dP:
// dz_k = p_k (dP_k - sum_j p_j dP_j).
void orc_softmax_bwd(const double* p, const double* dP, int M, int K, double* dz) {
    for (int m = 0; m < M; ++m) {
        double dot = 0.0;
        for (int k = 0; k < K; ++k) dot += p[(int64_t)m * K + k] * dP[(int64_t)m * K + k];
        for (int k = 0; k < K; ++k)
            dz[(int64_t)m * K + k] = p[(int64_t)m * K + k] * (dP[(int64_t)m * K + k] - dot);
    }
}

// Index of the largest probability per row; ties go to the smallest index.
void orc_argmax(const float* p, int M, int K, int8_t* out) {
    for (int m = 0; m < M; ++m) {
        int best = 0;
        for (int k = 1; k < K; ++k)
            if (p[(int64_t)m * K + k] > p[(int64_t)m * K + best]) best = k;
        out[m] = (int8_t)best;
    }
}

// One Adam step (Kingma & Ba), as used by the Section 3 training loop:
// m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; mhat = m / (1-b1^t);
// vhat = v / (1-b2^t); p = p - lr mhat / (sqrt(vhat) + eps).
void orc_adam(const float* p, const float* g, const float* m, const float* v, int64_t n, double lr,
              double b1, double b2, double eps, int step, double* p_out, double* m_out, double* v_out) {
    double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        double mi = b1 * (double)m[i] + (1.0 - b1) * (double)g[i];
        double vi = b2 * (double)v[i] + (1.0 - b2) * (double)g[i] * (double)g[i];
        m_out[i] = mi;
        v_out[i] = vi;
        p_out[i] = (double)p[i] - lr * (mi / c1) / (std::sqrt(vi / c2) + eps);
    }
}

}  // extern "C"
