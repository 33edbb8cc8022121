/*
 * tdp.h: C ABI of the MI355X (gfx950) relational-operator library.
 *
 * Relational operators run as tensor programs over columnar data, after
 * "The Tensor Data Platform: Towards an AI-centric Database System"
 * (arXiv 2211.02753): every column is a tensor (Section 2, storage model),
 * queries are filters, joins and grouped aggregates (Section 2, query
 * processor; Section 3, GROUP BY ... COUNT(*)), and trainable queries replace
 * the comparison step and the grouped count by differentiable relaxations
 * (Section 4).  The small image classifier stands in for a missing label
 * column (Sections 3 and 5.5).
 *
 * Conventions shared by every call:
 *   - All data pointers are DEVICE pointers on the current HIP device unless
 *     stated otherwise.  Inputs are read only.  Outputs must not alias inputs.
 *   - The caller owns every buffer: outputs and workspace.  The library never
 *     allocates or frees device memory and keeps no mutable global state,
 *     except the static scratch array of tdp_filter_noalloc.
 *   - Workspace is sized by the matching *_workspace_size call and must be
 *     256-byte aligned.  Its contents on entry are ignored.
 *   - Every call is asynchronous on `stream`.  Counts (number of output rows,
 *     number of groups) are written to device int64 scalars; the caller
 *     synchronises when it needs them on the host.
 *   - A call returns a status (TDP_OK or a negative TDP_E* code) after
 *     validating its arguments on the host and launching its kernels;
 *     argument errors return before any launch.  Conditions that only the
 *     device can see (a group key outside its declared domain, a duplicate
 *     key in a build side declared unique) are OR-ed as TDP_FLAG_* bits into
 *     the caller's device int32 `d_status` word, which each call clears
 *     first; read it after synchronising.  Outputs are unspecified when a
 *     flag is set.
 *   - No C++ exception crosses this interface.
 *   - Calls on different streams with different workspaces may run
 *     concurrently; two calls that share a workspace must be ordered.
 */
#ifndef TDP_H
#define TDP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    TDP_OK = 0,
    TDP_EINVAL = -1,       /* null pointer, negative size, bad enum, unsupported combination of arguments */
    TDP_ECAPACITY = -2,    /* an output buffer is too small for the guaranteed bound (see tdp_last_needed) */
    TDP_EWORKSPACE = -3,   /* workspace smaller than *_workspace_size (see tdp_last_needed) */
    TDP_EUNSUPPORTED = -4, /* dtype / operator combination this library does not implement */
    TDP_EDEVICE = -5       /* a HIP runtime call failed (see tdp_last_error) */
};

/* Device-side condition bits written to d_status. */
enum {
    TDP_FLAG_KEY_DOMAIN = 1,   /* a group key fell outside [key_lo, key_lo + key_card) */
    TDP_FLAG_DUP_BUILD = 2,    /* a build key repeated although build_unique was set */
    TDP_FLAG_GROUP_RANGE = 4,  /* a soft group id fell outside [0, G) */
    TDP_FLAG_TABLE_FULL = 8,   /* a hash table ran out of slots (cannot happen at the sized load) */
    TDP_FLAG_SPIN = 16,        /* an inter-workgroup wait exceeded its bound; results are invalid */
    TDP_FLAG_BAD_PARAM = 32    /* a device-side parameter (a temperature) was not positive and finite */
};

/* Human-readable text of a status code (static storage). */
const char* tdp_status_string(int status);
/* Text of the last error raised on the calling host thread ("" if none). */
const char* tdp_last_error(void);
/* After a call on this host thread returned TDP_ECAPACITY or TDP_EWORKSPACE:
 * the size it needed (output elements, or workspace bytes).  0 after any
 * other failure. */
int64_t tdp_last_needed(void);

/* Measurement hook (not part of any operator): select one stage whose
 * launches are bracketed by HIP events on their own stream, then read the
 * summed event time.  tdp_stage_timer(stage) clears the record and selects
 * the stage (TDP_STAGE_NONE turns it off); tdp_stage_time writes the total
 * milliseconds and the number of launches timed since (at most 256; later
 * launches run untimed).  Host-side state of the calling process, not
 * thread-safe; events are created on the device current at the first call. */
enum { TDP_STAGE_NONE = 0, TDP_STAGE_RP_SCATTER = 1, TDP_STAGE_RP_PROBE = 2, TDP_STAGE_FUSED_PROBE = 3 };
int tdp_stage_timer(int stage);
int tdp_stage_time(double* total_ms, int64_t* launches);

/* ------------------------------------------------------------- columns */
enum { TDP_I8 = 1, TDP_I32 = 2, TDP_I64 = 3, TDP_F32 = 4 };
enum { TDP_LT = 0, TDP_LE = 1, TDP_GT = 2, TDP_GE = 3, TDP_EQ = 4, TDP_NE = 5 };
enum { TDP_SIDE_PROBE = 0, TDP_SIDE_BUILD = 1 };

/* One column of a table: a 1-d tensor (Section 2, storage model).  Integer
 * columns are widened to int64 before any comparison or arithmetic. */
typedef struct tdp_col {
    const void* data; /* device pointer to n values of `dtype` */
    int32_t dtype;    /* TDP_I8, TDP_I32 or TDP_I64 (TDP_F32 only where stated) */
    int32_t side;     /* TDP_SIDE_PROBE or TDP_SIDE_BUILD, where a call joins two tables */
    int64_t n;        /* number of rows */
} tdp_col;

/* -------------------------------------------------------------- filter */
/* WHERE col <cmp> literal (Section 2 query processor; the timestamp filter of
 * the Section 5.2 document query).
 *
 * Candidates are rows 0..col->n-1, or the rows listed in sel_in[0..n_sel_in)
 * when sel_in is not NULL (this chains a conjunction of predicates; sel_in
 * must then hold valid row ids).  The comparison is signed after widening
 * both sides to int64.  Surviving row ids are written to rows_out in
 * candidate order (stable compaction), so with sel_in == NULL they are
 * ascending.  *d_n_out (device int64) receives their number.
 *
 * cap is the capacity of rows_out and must be at least the number of
 * candidates (the only bound known before the scan); else TDP_ECAPACITY.
 * Candidates are limited to 2^31 - 1 rows.  Workspace:
 * tdp_filter_workspace_size(number of candidates). */
size_t tdp_filter_workspace_size(int64_t n_candidates);
int tdp_filter(const tdp_col* col, int32_t cmp, int64_t literal, const int32_t* sel_in, int64_t n_sel_in,
               int32_t* rows_out, int64_t cap, int64_t* d_n_out, int32_t* d_status, void* ws, size_t ws_bytes,
               hipStream_t stream);

/* Allocation-free variant of tdp_filter, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, semantics and errors as
 * tdp_filter, without the workspace: the tile states and ticket live in a
 * static device array of the library (about 1 MiB per GPU, held until the
 * process ends), which the call clears with a kernel before use.  Candidates
 * are limited to tdp_filter_noalloc_max_candidates() (2^31 - 1); more return
 * TDP_EINVAL.  Every call on one GPU shares that GPU's array, so calls that
 * overlap in time on one GPU (different streams, or host threads) race and
 * must be ordered by the caller.  The call allocates and frees nothing. */
int64_t tdp_filter_noalloc_max_candidates(void);
int tdp_filter_noalloc(const tdp_col* col, int32_t cmp, int64_t literal, const int32_t* sel_in, int64_t n_sel_in,
                       int32_t* rows_out, int64_t cap, int64_t* d_n_out, int32_t* d_status, hipStream_t stream);

/* ------------------------------------------------------------ hash join */
/* Inner equi-join probe.key = build.key (standard SQL semantics: the paper
 * defers relational operator details to its TQP citation in Section 2).
 * Duplicate keys on both sides give their cross product.  The build side is
 * inserted into an open-addressing hash table held in the workspace; the
 * probe side streams through it. */
typedef struct tdp_join_desc {
    const int32_t* build_key; /* device, n_build values */
    int64_t n_build;
    const int32_t* probe_key; /* device, n_probe values */
    int64_t n_probe;
    const int32_t* probe_sel; /* optional device list of probe rows to join (NULL = all) */
    int64_t n_probe_sel;
    int32_t build_unique;     /* 1: the caller asserts build keys are distinct (a primary key);
                                 a repeat raises TDP_FLAG_DUP_BUILD */
    int32_t load_pct;         /* table load bound in percent, 10..90 (0 = 50) */
    int64_t max_distinct;     /* upper bound on the distinct build keys, sizes the table (0 = n_build;
                                 values above n_build are taken as n_build).  A build side with more
                                 distinct keys than the table holds raises TDP_FLAG_TABLE_FULL. */
} tdp_join_desc;

enum { TDP_JOIN_PAIRS = 0, TDP_JOIN_COUNT = 1 };

/* mode TDP_JOIN_PAIRS writes matching (probe_row, build_row) pairs to
 * out_probe[i], out_build[i] for i < min(total, cap) in UNSPECIFIED order
 * (compare after sorting by (probe_row, build_row)); if total > cap which
 * pairs were written is unspecified.  Both modes write the total number of
 * pairs to *d_n_out.  Workspace: tdp_hash_join_workspace_size(d). */
size_t tdp_hash_join_workspace_size(const tdp_join_desc* d);
int tdp_hash_join(const tdp_join_desc* d, int32_t mode, int32_t* out_probe, int32_t* out_build, int64_t cap,
                  int64_t* d_n_out, int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------- group-by/agg */
/* One conjunct of a WHERE clause beyond the descriptor's first predicate:
 * probe-side `col <cmp> literal`.  Integer columns (I8, I32, I64) compare
 * signed with `literal` after widening to int64; float32 columns (TDP_F32)
 * compare in float32 with (float)literal_f (an EQ / NE on floats is the
 * bitwise-equal comparison of IEEE values: NaN fails "==" and passes "!="). */
typedef struct tdp_pred {
    tdp_col col;
    int32_t cmp;       /* TDP_LT ... TDP_NE */
    int32_t reserved;  /* 0 */
    int64_t literal;   /* integer columns */
    double literal_f;  /* float32 columns */
} tdp_pred;

enum { TDP_MAX_MORE_PREDS = 3 };

/* Value expression of SUM / AVG, evaluated per joined row in int64 with
 * wrap-around modulo 2^64:  */
enum {
    TDP_EXPR_COL = 0,           /* a                       */
    TDP_EXPR_MUL = 1,           /* a * b                   */
    TDP_EXPR_MUL_CONST_SUB = 2, /* a * (k - b)             */
    TDP_EXPR_NONE = 3           /* no value: COUNT(*) only; sums are 0 */
};

/* SELECT key0[, key1], SUM(e), COUNT(*), AVG(e)
 *   FROM probe [JOIN build ON probe.key = build.key]
 *   WHERE pred GROUP BY key0[, key1] [ORDER BY SUM(e) DESC, keys ASC LIMIT topk]
 * (Section 2 query processor; Section 3 grouped COUNT(*); AVG as in the
 * Section 5.2 query.)
 *
 * The WHERE clause is the conjunction of the optional first predicate (an
 * integer probe-side column compared with pred_literal) and up to
 * TDP_MAX_MORE_PREDS further conjuncts more_preds[0..n_more_preds) (integer
 * or float32 columns; the array is read on the host during the call); sel
 * (optional) restricts the probe rows first.  Group keys and value
 * operands are integer columns from either side (tdp_col.side).  A group key
 * must lie in its declared domain [key_lo, key_lo + key_card), the caller's
 * statistics of that column (TDP_FLAG_KEY_DOMAIN otherwise); the product of
 * the domains is at most 2^27.
 *
 * With a join whose build side is not unique, group keys must come from the
 * probe side and the expression must be linear in build-side values
 * (COL of either side, MUL / MUL_CONST_SUB with a on the probe side and b on
 * the build side); the build side is then pre-aggregated per key
 * (count and sum of b), which is exact modulo 2^64 by distributivity.  Other
 * combinations return TDP_EUNSUPPORTED.
 *
 * Output: only groups with COUNT > 0, in ascending (key0, key1) order, or the
 * topk groups ranked by SUM descending then keys ascending.  AVG is
 * (double)SUM / (double)COUNT, each conversion and the division rounded to
 * nearest even.  *d_n_groups receives the number of groups written. */
typedef struct tdp_groupby_desc {
    int64_t n_rows;           /* probe-side row count */
    int32_t has_pred;
    int32_t pred_cmp;         /* TDP_LT ... TDP_NE */
    int64_t pred_literal;
    tdp_col pred;             /* probe-side column */
    const int32_t* sel;       /* optional device list of probe rows (NULL = all) */
    int64_t n_sel;
    const tdp_join_desc* join;/* NULL = no join (probe_key, n_probe of the descriptor are ignored:
                                 the probe key column is join->probe_key over n_rows) */
    int32_t n_keys;           /* 1 or 2 */
    int32_t expr;             /* TDP_EXPR_* */
    tdp_col key[2];
    int64_t key_lo[2];
    int64_t key_card[2];
    tdp_col a, b;             /* value operands */
    int64_t k;                /* constant of TDP_EXPR_MUL_CONST_SUB */
    int32_t topk;             /* 0 = every group */
    int32_t strategy;         /* probe strategy hint: TDP_PROBE_AUTO, _DIRECT, _STAGED or _PARTITIONED */
    const tdp_pred* more_preds;/* further conjuncts of the WHERE clause (host array, may be NULL) */
    int32_t n_more_preds;     /* 0 .. TDP_MAX_MORE_PREDS */
    int32_t reserved;         /* 0 */
} tdp_groupby_desc;

/* Execution strategy hint; results are identical under every strategy.
 * DIRECT: one fused kernel reads, filters, probes and aggregates each row in
 * row order.  STAGED (keys-only joins without a selection vector, fewer than
 * 65535 groups, tables of at least 65536 slots): rows are first partitioned by
 * table region into (key, group, value) records, then each region is probed
 * with its table slice resident in one XCD's L2.  PARTITIONED (keys-only
 * joins without a selection vector, at most 2^(pbits-1) - 1 groups where
 * 2^pbits is the partition count, 64 .. 1024, chosen from the build size and
 * the group count): both sides are partitioned by the top bits of the key's
 * hash, every probe row becomes one 8-byte (group | tag, value) record in its
 * partition (a value outside int32 is re-read from its column at the match),
 * and each partition's records stream through an LDS table of its build keys.
 * AUTO: the partitioned probe for keys-only joins it accepts with at least
 * 2^18 build keys and 2^22 probe rows; otherwise the fused kernel, except
 * that dense group tables beyond LDS (more than 2048 groups, at most 2^20)
 * over at least 2^20 rows with probe-side group keys and no selection vector
 * aggregate through group-range partitions reduced in LDS; DIRECT turns both
 * off. */
enum { TDP_PROBE_AUTO = 0, TDP_PROBE_DIRECT = 1, TDP_PROBE_STAGED = 2, TDP_PROBE_PARTITIONED = 3 };

typedef struct tdp_groupby_out {
    int64_t cap;              /* capacity of the arrays below, in groups */
    int64_t* d_n_groups;      /* device int64 */
    int64_t* key0;            /* device [cap] */
    int64_t* key1;            /* device [cap], may be NULL when n_keys == 1 */
    int64_t* sum;             /* device [cap] */
    int64_t* count;           /* device [cap] */
    double* avg;              /* device [cap] */
} tdp_groupby_out;

/* cap must be at least min(product of key domains, topk if set).
 * Workspace: tdp_groupby_workspace_size(d). */
size_t tdp_groupby_workspace_size(const tdp_groupby_desc* d);
int tdp_groupby_agg(const tdp_groupby_desc* d, const tdp_groupby_out* o, int32_t* d_status, void* ws,
                    size_t ws_bytes, hipStream_t stream);

/* The same query in two calls that share one workspace: tdp_groupby_build
 * clears *d_status, resets the workspace's accumulators and builds the
 * join's hash table (when there is a join); tdp_groupby_probe then streams
 * the probe side, OR-ing its flags into *d_status, and leaves the
 * accumulators reset.  A probe needs a build on the same workspace before
 * it; one build may serve several probes with the same descriptor (the
 * build side must stay unchanged in between). */
int tdp_groupby_build(const tdp_groupby_desc* d, int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream);
int tdp_groupby_probe(const tdp_groupby_desc* d, const tdp_groupby_out* o, int32_t* d_status, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------ relaxed (soft) operators */
/* Soft filter (Section 4: a logistic function relaxes the step of a
 * comparison): w[i] = 1 / (1 + exp(-(c - x[i]) / tau)), which tends to
 * 1[x[i] < c] as tau -> 0.  c is a device float scalar (a learnable
 * threshold); tau > 0 is a host float, else TDP_EINVAL. */
int tdp_soft_filter(const float* x, int64_t n, const float* d_c, float tau, float* w, hipStream_t stream);

/* Workspace of the soft calls that reduce across workgroups: size
 * tdp_soft_workspace_size(), prepared ONCE by tdp_soft_workspace_init.
 * Every soft call returns the workspace to its prepared state when its last
 * workgroup finishes, so calls need no clearing launch; calls that share a
 * workspace must be ordered (same stream).  In these calls *d_status is
 * overwritten with the call's flags. */
size_t tdp_soft_workspace_size(void);
int tdp_soft_workspace_init(void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward of the soft filter from dL/dw: dx[i] = -dw[i] w[i] (1 - w[i]) / tau
 * (dx may be NULL) and *d_dc = sum_i dw[i] w[i] (1 - w[i]) / tau (device
 * float, overwritten).  When d_dtau is not NULL it receives the gradient in
 * the temperature, with z[i] = (c - x[i]) / tau:
 * *d_dtau = -sum_i dw[i] w[i] (1 - w[i]) z[i] / tau.  w is recomputed, not read. */
int tdp_soft_filter_bwd(const float* x, int64_t n, const float* d_c, float tau, const float* dw, float* dx,
                        float* d_dc, float* d_dtau, void* ws, size_t ws_bytes, hipStream_t stream);

/* Soft grouped aggregation (Section 4, the grouped generalisation of the
 * soft count on probability-encoded data, using only + and *):
 * S[g][k] = sum over rows i with g[i] = g of w[i] * v[i][k], for K value
 * columns stored row-major v[n][K]; w == NULL means w = 1 (a plain soft SUM;
 * with v the class probabilities it is the soft COUNT per class).  Empty
 * groups give 0.  1 <= K <= 16, 1 <= G <= 65536.  A group id outside [0, G)
 * raises TDP_FLAG_GROUP_RANGE and the row is dropped. */
int tdp_soft_groupby(const int32_t* g, const float* w, const float* v, int64_t n, int32_t K, int32_t G, float* S,
                     int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward of the soft grouped aggregation from dS[G][K]:
 * dv[i][k] = dS[g[i]][k] * w[i] and dw[i] = sum_k dS[g[i]][k] * v[i][k].
 * Either output may be NULL; w == NULL means w = 1. */
int tdp_soft_groupby_bwd(const int32_t* g, const float* w, const float* v, const float* dS, int64_t n, int32_t K,
                         int32_t G, float* dw, float* dv, hipStream_t stream);

/* Fused soft filter + soft group-by SUM(v), the pair a trainable query runs:
 * S[g] = sum_{i: g[i] = g} sigma((c - x[i]) / tau) v[i].  w is never stored.
 * When T is not NULL the call also evaluates the training loss of the
 * Section 3 loop, the mean squared error over the G groups,
 * *d_loss = (1/G) sum_g (S[g] - T[g])^2, and writes dS[g] = 2 (S[g] - T[g]) / G
 * (d_loss and dS must then be non-NULL). */
int tdp_soft_filter_groupby(const float* x, const float* v, const int32_t* g, int64_t n, const float* d_c, float tau,
                            int32_t G, float* S, const float* T, float* d_loss, float* dS, int32_t* d_status,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward of the fused pair from dS[G], recomputing the mask:
 * dv[i] = dS[g[i]] w[i];  *d_dc = sum_i dS[g[i]] v[i] w[i] (1 - w[i]) / tau;
 * dx[i] = -dS[g[i]] v[i] w[i] (1 - w[i]) / tau when dx is not NULL;
 * *d_dtau = -sum_i dS[g[i]] v[i] w[i] (1 - w[i]) z[i] / tau, z[i] = (c - x[i]) / tau,
 * when d_dtau is not NULL (the temperature as a learnable parameter). */
int tdp_soft_filter_groupby_bwd(const float* x, const float* v, const int32_t* g, int64_t n, const float* d_c,
                                float tau, int32_t G, const float* dS, float* dv, float* dx, float* d_dc,
                                float* d_dtau, void* ws, size_t ws_bytes, hipStream_t stream);

/* Soft COUNT grouped by two probability-encoded attributes.  Section 4
 * counts on probability-encoded data with + and * only; the grid-of-images
 * query (Sections 3 and 5.5) groups COUNT(*) by two predicted attributes
 * (digit and size) of each tile:
 *   S[g][a][b] = sum over the rows i of segment g of p[i][a] * q[i][b].
 * Segment g is rows seg[g] .. seg[g+1]-1 (a table-valued function emits the
 * tiles of one image together); seg == NULL is one segment of all n rows and
 * requires G == 1.  Segments may leave rows out; a segment outside [0, n] or
 * with seg[g+1] < seg[g] raises TDP_FLAG_GROUP_RANGE and gives zeros.
 * p is float32 [n][K1], q float32 [n][K2] (row-major); q == NULL means q = 1
 * and requires K2 == 1 (the soft COUNT per class of p).  1 <= K1, K2 <= 16,
 * K1 * K2 <= 64.  seg is a device int64 array of G + 1 entries; S is
 * float32 [G][K1][K2], overwritten.  Products and sums run in float64 inside
 * a segment; without segments the per-workgroup sums are added in a fixed
 * order.  Uses the soft workspace (tdp_soft_workspace_size). */
int tdp_soft_pe_groupby(const int64_t* seg, int32_t G, const float* p, int32_t K1, const float* q, int32_t K2,
                        int64_t n, float* S, int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward of the grouped soft COUNT from dS[G][K1][K2], for each row i of
 * segment g:  dp[i][a] = sum_b dS[g][a][b] q[i][b]  and
 * dq[i][b] = sum_a dS[g][a][b] p[i][a]  (float32, sums in b or a order).
 * Either output may be NULL; dq requires q.  Segments must not overlap; rows
 * outside every valid segment are not written. */
int tdp_soft_pe_groupby_bwd(const int64_t* seg, int32_t G, const float* p, int32_t K1, const float* q, int32_t K2,
                            int64_t n, const float* dS, float* dp, float* dq, hipStream_t stream);

/* The trainable form of a tdp_groupby_desc query (Section 4: a flag at
 * compilation makes a query trainable by relaxing its operators; the exact
 * operators come back at inference).  The same descriptor that
 * tdp_groupby_agg runs exactly is run relaxed:
 *   - each conjunct j of the WHERE clause (the first predicate when
 *     has_pred, then more_preds in order; J <= 4 in all) becomes
 *     sigma(z_j), z_j = s_j (c[j] - x_j) / tau[j], with x_j the column value
 *     as float32 (integers converted), s_j = +1 for TDP_LT / TDP_LE and -1
 *     for TDP_GT / TDP_GE (EQ / NE have no relaxation: TDP_EUNSUPPORTED);
 *     the literals are replaced by the learnable thresholds d_c[J] (device
 *     float32) and d_tau[J] (device float32) are the temperatures, each
 *     positive and finite (otherwise the forward raises TDP_FLAG_BAD_PARAM
 *     and its results are invalid; both stay on the device, so a training
 *     loop that updates them never waits for the host);
 *   - the conjunction is the product w = prod_j sigma(z_j);
 *   - the grouped aggregate is S[gid] = sum of w * e over the rows of the
 *     group, with e = a as float32 for TDP_EXPR_COL (I8, I32, I64 or F32 a)
 *     and e = 1 for TDP_EXPR_NONE (the soft COUNT); gid is the dense group
 *     id of the key domains, (key0 - key_lo0) * key_card1 + (key1 - key_lo1),
 *     and S (float32 [G], G = product of the key domains <= 65536) covers
 *     every group, empty ones 0.  A key outside its domain raises
 *     TDP_FLAG_KEY_DOMAIN and the row is dropped.
 * Joins, selection vectors, other expressions and topk: TDP_EUNSUPPORTED.
 * When T is not NULL the call also evaluates the training loss,
 * *d_loss = (1/G) sum (S - T)^2, and dS = 2 (S - T) / G.  Uses the soft
 * workspace (tdp_soft_workspace_size); *d_status is overwritten. */
int tdp_soft_query(const tdp_groupby_desc* d, const float* d_c, const float* d_tau, float* S, const float* T,
                   float* d_loss, float* dS, int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward of tdp_soft_query from dS[G], recomputing every sigma (d_c and
 * d_tau as in the forward, device float32 [J]): with d_i = dS[gid_i] e_i,
 *   d_dc[j] = sum_i d_i w_i (1 - sigma(z_ij)) s_j / tau[j]        (device float32 [J], overwritten)
 *   d_dtau[j] = -sum_i d_i w_i (1 - sigma(z_ij)) z_ij / tau[j]    (device float32 [J], may be NULL)
 *   de[i] = dS[gid_i] w_i, the gradient in the value column       (device float32 [n_rows], may be NULL;
 *                                                                   rows outside a key domain get 0) */
int tdp_soft_query_bwd(const tdp_groupby_desc* d, const float* d_c, const float* d_tau, const float* dS, float* d_dc,
                       float* d_dtau, float* de, void* ws, size_t ws_bytes, hipStream_t stream);

/* Mean squared error over G values (the Section 3 training loop's loss):
 * *d_loss = (1/G) sum (S - T)^2 and dS = 2 (S - T) / G (dS may be NULL). */
int tdp_mse_loss(const float* S, const float* T, int32_t G, float* d_loss, float* dS, hipStream_t stream);

/* ------------------------------- learning from label proportions (LLP) */
/* Section 5.3: a linear classifier (a table-valued function) labels every
 * row of a bag and a GROUP BY bag, label COUNT(*) query, relaxed, is trained
 * against the bags' released label counts; Section 5.4 releases those counts
 * through the Laplace mechanism (Label-DP).  The classifier's class
 * probabilities are p_i = softmax(W x_i + b), and the soft COUNT of class c
 * in bag j is
 *   S[j][c] = sum over the rows i of bag j of p_i[c],
 * with bags the consecutive runs of `bag` rows (a power of two, 1 .. 2^20;
 * the last bag may be short).  X is float32 row-major [n][F] (16-byte
 * aligned), 1 <= F <= 16; W is float32 [C][F], b [C], 2 <= C <= 4; S is
 * float32 [ceil(n / bag)][C], overwritten.  Each bag's sum is formed in
 * float64 in a fixed order inside one wave.  When T (the released counts,
 * float32 [n_bags][C]) is not NULL the call also evaluates the training
 * loss over the n_bags * C cells, *d_loss = mean (S - T)^2, and writes
 * dS = 2 (S - T) / (n_bags * C) (d_loss, dS and the workspace
 * tdp_llp_workspace_size(C) are then required; otherwise ws may be NULL). */
int tdp_llp_bag_count(const float* X, int64_t n, int32_t F, const float* W, const float* b, int32_t C, int64_t bag,
                      float* S, const float* T, float* d_loss, float* dS, void* ws, size_t ws_bytes,
                      hipStream_t stream);

/* Backward of tdp_llp_bag_count from dS [n_bags][C], recomputing p: with
 * dp_i = dS[bag of i] and dz_i[c] = p_i[c] (dp_i[c] - sum_k p_i[k] dp_i[k]),
 * dW[c][f] = sum_i dz_i[c] x_i[f] and db[c] = sum_i dz_i[c] (float32,
 * overwritten; summed in a fixed order through float64 per-workgroup
 * partials).  Workspace: tdp_llp_workspace_size(C). */
size_t tdp_llp_workspace_size(int32_t C);
int tdp_llp_bag_count_bwd(const float* X, int64_t n, int32_t F, const float* W, const float* b, int32_t C,
                          int64_t bag, const float* dS, float* dW, float* db, void* ws, size_t ws_bytes,
                          hipStream_t stream);

/* The exact swap at inference (Section 4): out[i] = argmax_c (W x_i + b)[c],
 * ties to the smallest class.  Each logit is accumulated in float64 as b[c]
 * followed by one fused multiply-add per feature in feature order. */
int tdp_llp_predict(const float* X, int64_t n, int32_t F, const float* W, const float* b, int32_t C, int8_t* out,
                    hipStream_t stream);

/* A grouped COUNT answer (the groups of tdp_groupby_agg: keys key0[, key1]
 * and count, *d_n_groups of them) as a dense float32 table
 * out[(key0 - lo0) * card1 + (key1 - lo1)], empty cells 0; with noise (a
 * float32 [card0 * card1] array of draws the caller makes, e.g. Laplace with
 * scale 1 / epsilon for the Section 5.4 Label-DP release) every cell is
 * count + noise, rounded once to float32.  key1 == NULL requires card1 == 1.
 * A key outside its table raises TDP_FLAG_KEY_DOMAIN in *d_status (OR-ed;
 * not cleared). */
int tdp_count_table(const int64_t* key0, const int64_t* key1, const int64_t* count, const int64_t* d_n_groups,
                    int64_t lo0, int64_t card0, int64_t lo1, int64_t card1, const float* noise, float* out,
                    int32_t* d_status, hipStream_t stream);

/* out[i] = i / width for i < n (int32): the bag of each row when bags are
 * consecutive runs of `width` rows, or the grid row of each image cell. */
int tdp_segment_ids(int64_t n, int64_t width, int32_t* out, hipStream_t stream);

/* ------------------------------------- dictionary-encoded string columns */
/* Section 2 (storage and encodings): a string column is stored through an
 * order-preserving dictionary, itself a 2-d byte tensor with one string per
 * row.  Here a string column is a zero-padded byte matrix [n][L] with L a
 * multiple of 4 in 4..32 (strings hold no zero bytes; 4-byte aligned);
 * strings order byte by byte, a prefix first.  The dictionary is the sorted
 * list of the distinct strings, [d][L]; a string's code is its position in
 * it (int32), so codes compare exactly as the strings do and serve as keys
 * of tdp_filter, tdp_hash_join and tdp_groupby_agg (key domain [0, d)).
 *
 * tdp_dict_build: the dictionary of a column and the column's codes, in one
 * asynchronous call.  max_distinct bounds the distinct strings (0 = n): dict
 * must hold that many rows; more distinct strings raise TDP_FLAG_TABLE_FULL
 * (outputs then unspecified).  *d_n_dict (device int64) receives d.
 * Workspace: tdp_dict_build_workspace_size(n, max_distinct) bytes, 256-byte
 * aligned (TDP_EINVAL otherwise). */
size_t tdp_dict_build_workspace_size(int64_t n, int64_t max_distinct);
int tdp_dict_build(const uint8_t* strs, int64_t n, int32_t L, int64_t max_distinct, uint8_t* dict, int64_t* d_n_dict,
                   int32_t* codes, int32_t* d_status, void* ws, size_t ws_bytes, hipStream_t stream);
/* For each string of strs [n][L]: pos = the number of dictionary entries
 * below it (its code when it is present) and found = 1 when it is present
 * (found may be NULL).  n_dict is the dictionary size on the host.  Used to
 * encode another column against a dictionary (absent strings have found 0)
 * and to turn a comparison with a string literal into one with a code. */
int tdp_dict_lookup(const uint8_t* dict, int64_t n_dict, int32_t L, const uint8_t* strs, int64_t n, int32_t* pos,
                    int8_t* found, hipStream_t stream);
/* out[i] = dict[codes[i]] (rows of L bytes); a code outside [0, n_dict)
 * gives a zero row and raises TDP_FLAG_KEY_DOMAIN (OR-ed into *d_status). */
int tdp_dict_decode(const int32_t* codes, int64_t n, const uint8_t* dict, int64_t n_dict, int32_t L, uint8_t* out,
                    int32_t* d_status, hipStream_t stream);

/* --------------------------------------------- learned label column (CNN) */
/* The classifier inside the table-valued function that fills a missing
 * label column from an image column (Section 3's grid-of-images example;
 * trained through the soft aggregation in Sections 4 and 5.5).  The paper
 * does not give its architecture.  Layers follow: NHWC activations, weights
 * [Cout][3][3][Cin] for 3x3 valid convolutions (stride 1), [N][K] for fully
 * connected layers.  bf16 tensors are uint16_t bit patterns; products run on
 * bf16 MFMA with float32 accumulation; every float32 -> bf16 conversion
 * rounds to nearest even (NaN stays NaN).  All pointers are device pointers
 * and calls are asynchronous on `stream`. */

/* out[i] = bf16(img[i] / 255) for uint8 pixels. */
int tdp_image_to_bf16(const uint8_t* img, int64_t n, uint16_t* out, hipStream_t stream);
/* out[i] = bf16(in[i]). */
int tdp_f32_to_bf16(const float* in, int64_t n, uint16_t* out, hipStream_t stream);

/* y[b,oy,ox,co] = act(bias[co] + sum_{ky,kx,ci} x[b,oy+ky,ox+kx,ci] w[co][ky][kx][ci]),
 * x [B][H][W][Cin], y [B][H-2][W-2][Cout]; act = ReLU when relu != 0; bias
 * (float32) may be NULL.  x and w 16-byte aligned. */
int tdp_conv3x3_fwd_bf16(const uint16_t* x, const uint16_t* w, const float* bias, int B, int H, int W, int Cin,
                         int Cout, int relu, uint16_t* y, hipStream_t stream);
/* Input gradient dx[b,iy,ix,ci] = sum dy[b,iy-ky,ix-kx,co] w[co][ky][kx][ci], then
 * zeroed where mask_act <= 0 when mask_act (the layer input after its ReLU,
 * [B][H][W][Cin]) is given.  dy [B][H-2][W-2][Cout], 16-byte aligned. */
int tdp_conv3x3_dgrad_bf16(const uint16_t* dy, const uint16_t* w, const uint16_t* mask_act, int B, int H, int W,
                           int Cin, int Cout, uint16_t* dx, hipStream_t stream);
/* Weight and bias gradients: dw[co][ky][kx][ci] = sum_{b,oy,ox} dy[b,oy,ox,co] x[b,oy+ky,ox+kx,ci]
 * and db[co] = sum dy[...,co] (float32, overwritten; db may be NULL).  x and dy 16-byte
 * aligned.  Partial sums over pixel ranges are added with float32 atomics, so the
 * summation order (and the last bits) may vary between calls. */
int tdp_conv3x3_wgrad_bf16(const uint16_t* x, const uint16_t* dy, int B, int H, int W, int Cin, int Cout, float* dw,
                           float* db, hipStream_t stream);

/* y[m,n] = act(bias[n] + sum_k x[m,k] w[n,k]); x [M][K], w [N][K]; output
 * bf16 (y_bf16) or float32 (y_f32).  When both are given, y_f32 receives the
 * float32 output and y_bf16 its bf16 rounding, and the product runs split over K
 * (partial sums added into y_f32 with float32 atomics, then bias and activation):
 * the form for layers whose M x N is too small to fill the GPU; the summation
 * order may then vary between calls. */
int tdp_linear_fwd_bf16(const uint16_t* x, const uint16_t* w, const float* bias, int M, int N, int K, int relu,
                        uint16_t* y_bf16, float* y_f32, hipStream_t stream);
/* dx[m,k] = sum_n dy[m,n] w[n,k], zeroed where mask_act[m,k] <= 0 when given. */
int tdp_linear_dgrad_bf16(const uint16_t* dy, const uint16_t* w, const uint16_t* mask_act, int M, int N, int K,
                          uint16_t* dx, hipStream_t stream);
/* dw[n,k] = sum_m dy[m,n] x[m,k]; db[n] = sum_m dy[m,n] (float32, overwritten; db may be NULL).
 * x and dy 16-byte aligned; float32 atomics as for the convolution. */
int tdp_linear_wgrad_bf16(const uint16_t* x, const uint16_t* dy, int M, int N, int K, float* dw, float* db,
                          hipStream_t stream);

/* 2x2 max pooling, stride 2 (H, W even), x [B][H][W][C] -> y [B][H/2][W/2][C]. */
int tdp_maxpool2_fwd_bf16(const uint16_t* x, int B, int H, int W, int C, uint16_t* y, hipStream_t stream);
/* Its gradient: dy of each window goes to the window's first maximum in
 * row-major order; with relu_mask != 0 it is also zeroed where x <= 0 (the
 * ReLU in front of the pooling). */
int tdp_maxpool2_bwd_bf16(const uint16_t* x, const uint16_t* dy, int B, int H, int W, int C, int relu_mask,
                          uint16_t* dx, hipStream_t stream);

/* Section 4's smooth stand-in for argmax: p = softmax(logits) per row
 * [M][K] (K <= 64), and e[m] = sum_k k p[m,k] (the expected label, which a
 * soft SUM over the probability-encoded label reduces to; e may be NULL). */
int tdp_softmax_expect_fwd(const float* logits, int M, int K, float* p, float* e, hipStream_t stream);
/* dlogits[m,k] = dE[m] p[m,k] (k - e[m]) (float32 and/or bf16 output). */
int tdp_softmax_expect_bwd(const float* p, const float* dE, int M, int K, float* dlogits, uint16_t* dlogits_bf16,
                           hipStream_t stream);
/* General softmax backward from dL/dp (the soft COUNT per class of a
 * probability-encoded column feeds it): dlogits[m,k] = p[m,k] (dP[m,k] -
 * sum_j p[m,j] dP[m,j]) (float32 and/or bf16 output). */
int tdp_softmax_bwd(const float* p, const float* dP, int M, int K, float* dlogits, uint16_t* dlogits_bf16,
                    hipStream_t stream);
/* The exact swap at inference (Section 4): out[m] = argmax_k p[m,k], ties to the smallest k. */
int tdp_argmax_rows(const float* p, int M, int K, int8_t* out, hipStream_t stream);

/* One Adam step (the optimizer of the Section 3 training loop) on float32
 * parameters, in place: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps); p_bf16 (may be
 * NULL) receives bf16(p). */
int tdp_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                  int step, uint16_t* p_bf16, hipStream_t stream);

/* The same step for up to 16 tensors in one launch (a model's parameters):
 * each entry names its parameters p, gradient g, moments m and v, length n
 * and optional bf16 copy p_bf16, as in tdp_adam_step; the array is read on
 * the host during the call.  Results are identical to one tdp_adam_step per
 * tensor. */
typedef struct {
    float* p;
    const float* g;
    float* m;
    float* v;
    uint16_t* p_bf16;
    int64_t n;
} tdp_adam_tensor;
int tdp_adam_step_multi(const tdp_adam_tensor* tensors, int32_t count, float lr, float b1, float b2, float eps,
                        int step, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TDP_H */
