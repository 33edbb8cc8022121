// Open-addressing hash table over int32 keys, held in caller workspace.
//
// Layout (`cap` a power of two, linear probing that wraps inside aligned
// blocks of kTableBlock slots, so that one block is a self-contained table a
// workgroup can build in LDS):
//   keys[cap + 1]   int32, kEmpty marks a free slot.  The key value kEmpty
//                   itself is kept in the extra slot `cap` (keys[cap] = 1 when
//                   present), so every int32 key is representable.
//   rowid[cap + 1]  build row of the key (unique build sides).
//   rec[cap + 1]    pre-aggregated (many-to-many) sides instead of keys: one
//                   16-byte record per slot holding the key, the number of
//                   build rows with it and the sum of a build-side value over
//                   them (mod 2^64), so a probe that finds its key has the
//                   aggregate in the same line.
//   head[cap + 1]   first build row of the key's chain, next[n_build] the
//                   following ones (pair enumeration).
#pragma once

#include "common.hpp"

namespace tdp {

constexpr int32_t kEmpty = INT32_MIN;
constexpr uint32_t kTableBlock = 4096;      // slots per probing block

enum TableKind { TABLE_KEYS = 0, TABLE_ROWID = 1, TABLE_AGG = 2, TABLE_LIST = 3 };

struct alignas(16) AggRec {
    int32_t key;              // kEmpty when free (in slot cap: 1 when the key kEmpty is present)
    uint32_t cnt;             // build rows with the key (n_build < 2^31)
    unsigned long long sum;   // sum of the build operand over them, mod 2^64
};

struct HashView {
    int32_t* keys = nullptr;            // key, row-id and list tables
    int32_t* rowid = nullptr;
    AggRec* rec = nullptr;              // aggregate tables
    int32_t with_sum = 0;
    int32_t* head = nullptr;
    int32_t* next = nullptr;
    uint32_t mask = 0;   // cap - 1
    uint32_t bmask = 0;  // slots per probing block - 1
};

// Next slot of a linear probe: wraps inside the aligned block.
__device__ __forceinline__ uint32_t ht_next(uint32_t s, uint32_t bmask) { return (s & ~bmask) | ((s + 1) & bmask); }

// Table capacity for n keys at a load bound of load_pct percent.  n is the
// number of distinct keys the table must hold (at most the build rows).
inline uint32_t table_cap(int64_t n, int load_pct) {
    if (load_pct <= 0) load_pct = 50;
    load_pct = std::max(10, std::min(90, load_pct));
    int64_t need = std::max<int64_t>(16, (n * 100 + load_pct - 1) / load_pct);
    uint64_t cap = 16;
    while ((int64_t)cap < need) cap <<= 1;
    return (uint32_t)cap;
}

// Distinct keys the table of a join must hold: the caller's bound, at most
// the build rows.
inline int64_t distinct_bound(const tdp_join_desc* j) {
    return j->max_distinct > 0 && j->max_distinct < j->n_build ? j->max_distinct : j->n_build;
}

// Carve the table of `kind` out of the workspace (base may be null to size it).
inline HashView table_alloc(WsAlloc& wa, TableKind kind, int64_t n_build, uint32_t cap, bool with_sum) {
    HashView t;
    t.mask = cap - 1;
    t.bmask = std::min(cap, kTableBlock) - 1;
    if (kind == TABLE_AGG) {
        t.rec = wa.take<AggRec>((size_t)cap + 1);
        t.with_sum = with_sum;
        return t;
    }
    t.keys = wa.take<int32_t>((size_t)cap + 1);
    if (kind == TABLE_ROWID) t.rowid = wa.take<int32_t>((size_t)cap + 1);
    if (kind == TABLE_LIST) {
        t.head = wa.take<int32_t>((size_t)cap + 1);
        t.next = wa.take<int32_t>((size_t)std::max<int64_t>(n_build, 1));
    }
    return t;
}

// Slot of `key` after inserting it (kEmpty goes to slot cap).  `fresh` tells
// whether this call created the entry.  Returns -1 if the table is full.
__device__ __forceinline__ int64_t ht_insert(const HashView& t, int32_t key, bool& fresh) {
    if (key == kEmpty) {
        fresh = atomicExch(&t.keys[t.mask + 1], 1) == 0;
        return (int64_t)t.mask + 1;
    }
    uint32_t h = hash32((uint32_t)key) & t.mask;
    for (uint32_t probe = 0; probe <= t.bmask; ++probe) {
        int32_t prev = atomicCAS(&t.keys[h], kEmpty, key);
        if (prev == kEmpty) {
            fresh = true;
            return h;
        }
        if (prev == key) {
            fresh = false;
            return h;
        }
        h = ht_next(h, t.bmask);
    }
    fresh = false;
    return -1;
}

// Aggregate tables: slot of `key` after inserting it (kEmpty goes to slot
// cap), or -1 when its block is full; then add a count and a sum to it.
__device__ __forceinline__ int64_t agg_insert(const HashView& t, int32_t key) {
    if (key == kEmpty) {
        atomicExch(&t.rec[t.mask + 1].key, 1);
        return (int64_t)t.mask + 1;
    }
    uint32_t h = hash32((uint32_t)key) & t.mask;
    for (uint32_t probe = 0; probe <= t.bmask; ++probe) {
        const int32_t prev = atomicCAS(&t.rec[h].key, kEmpty, key);
        if (prev == kEmpty || prev == key) return h;
        h = ht_next(h, t.bmask);
    }
    return -1;
}

__device__ __forceinline__ void agg_add(const HashView& t, int64_t slot, uint32_t c, unsigned long long v) {
    atomicAdd(&t.rec[slot].cnt, c);
    if (t.with_sum) atomicAdd(&t.rec[slot].sum, v);
}

// Slot holding `key`, or -1.  The table must be complete (built by an
// earlier kernel).
__device__ __forceinline__ int64_t ht_find(const int32_t* __restrict__ keys, uint32_t mask, uint32_t bmask,
                                           int32_t key) {
    if (key == kEmpty) return keys[(int64_t)mask + 1] ? (int64_t)mask + 1 : -1;
    uint32_t h = hash32((uint32_t)key) & mask;
    for (uint32_t probe = 0; probe <= bmask; ++probe) {
        int32_t k = keys[h];
        if (k == key) return h;
        if (k == kEmpty) return -1;
        h = ht_next(h, bmask);
    }
    return -1;
}

// Scratch of the LDS build: rows are bucketed by build group (a run of
// consecutive probing blocks: 2 blocks of keys or of keys + row ids, 1 block
// of keys + counts + sums, at most 64 KiB of LDS) with a counting sort
// (per-workgroup histograms, their scan, a scatter), then one workgroup per
// group builds its blocks in LDS and writes them out whole.  Coarser groups
// keep fewer scatter runs open per workgroup, so more scattered writes
// combine in L2; larger ones cost LDS occupancy (measured: 2 blocks of keys
// beat 1, 4 and 8 on the 15M-key build).
inline uint32_t build_group_slots(TableKind kind, uint32_t cap) {
    const uint32_t most = kind == TABLE_AGG ? kTableBlock : 2 * kTableBlock;
    return cap < most ? cap : most;
}

// A bucketed build row of an aggregate table with a sum: key and value in
// one 16-byte record, so the scatter writes each row with one aligned store
// (separate 4- and 8-byte arrays left most written lines partial).
struct alignas(16) AggIn {
    int32_t key;
    uint32_t pad;  // 1 marks a padding record (the last unit of a scatter region), skipped by the builds
    unsigned long long val;
};

// Aggregate build sides with a sum and at most kAggUnitMaxBlk build groups
// are bucketed in whole 64-byte units of kAggUnit records (each workgroup's
// run of a group rounded up to a unit and padded).
constexpr int kAggUnit = 4;
constexpr uint32_t kAggUnitMaxBlk = 1024;
constexpr int kAggSub = 4096;            // rows the unit scatter orders at once (four per thread)
constexpr int kAggScatThreads = 1024;    // threads of the unit scatter (one group per thread)

struct BuildScratch {
    bool lds = false;
    int nw = 0;             // histogram workgroups
    int threads = 0;        // threads of a histogram / scatter workgroup (512 or 1024)
    int64_t chunk = 0;      // build rows per histogram workgroup
    uint32_t nblk = 0;      // build groups
    uint32_t gslots = 0;    // table slots per build group (a power of two, >= kTableBlock)
    int gshift = 0;         // log2(gslots)
    uint32_t* mat = nullptr;   // [nw][nblk] counts, then offsets
    uint32_t* base = nullptr;  // [nblk + 1] first bucketed row of each group
    int32_t* skeys = nullptr;  // [n_build] keys in block order
    int32_t* srows = nullptr;  // [n_build] their build rows (row-id tables)
    AggIn* srec = nullptr;     // [n_build] keys and build values (aggregate tables with a sum), instead of skeys
    uint32_t* xseg = nullptr;  // [nblk + 1] aggregate tables: first extra segment of each group
    int64_t max_xseg = 0;      // bound on the extra segments (launch size of the merge)
    bool units = false;        // srec bucketed in whole units (padding records included)
};

// Rows of a group the LDS build takes in its one workgroup; an aggregate
// group with more rows (a skewed key) gets extra workgroups that aggregate
// kBuildSegRows rows each in LDS and merge them into the table.
constexpr uint32_t kBuildSegRows = 16384;

inline BuildScratch build_scratch_alloc(WsAlloc& wa, TableKind kind, int64_t n_build, uint32_t cap, bool with_sum) {
    BuildScratch b;
    if (kind == TABLE_LIST || cap < kTableBlock) return b;
    b.gslots = build_group_slots(kind, cap);
    const uint32_t nblk = cap / b.gslots;
    b.lds = n_build >= 65536 && nblk >= 1 && nblk <= 8192;
    if (!b.lds) return b;
    b.nblk = nblk;
    while ((1u << b.gshift) < b.gslots) ++b.gshift;
    // Measured on the 15M-key build and the skewed 20M-row aggregate build:
    // keys and row ids scatter fastest from 128 workgroups of 1024 threads
    // (fewer open runs per L2); aggregate sides, whose hot keys make the
    // per-group counters contend, from 256 workgroups of 512 threads.
    const bool agg = kind == TABLE_AGG;
    b.threads = agg ? 512 : 1024;
    b.nw = (int)std::min<int64_t>(agg ? 256 : 128, ceil_div(n_build, 16384));
    b.chunk = ceil_div(ceil_div(n_build, b.nw), 4) * 4;  // a multiple of 4 (16-byte key loads)
    b.units = kind == TABLE_AGG && with_sum && nblk <= kAggUnitMaxBlk;
    if (b.units) {
        // the unit scatter's workgroups take whole sub-chunks
        b.threads = 512;  // of the histogram
        b.chunk = ceil_div(ceil_div(n_build, b.nw), (int64_t)kAggSub) * kAggSub;
    }
    b.nw = (int)ceil_div(n_build, b.chunk);
    b.mat = wa.take<uint32_t>((size_t)b.nw * nblk);
    b.base = wa.take<uint32_t>((size_t)nblk + 1);
    const int64_t n_srec = n_build + (b.units ? (int64_t)(kAggUnit - 1) * nblk * b.nw : 0);
    if (kind == TABLE_AGG && with_sum)
        b.srec = wa.take<AggIn>((size_t)n_srec);
    else
        b.skeys = wa.take<int32_t>((size_t)n_build);
    if (kind == TABLE_ROWID) b.srows = wa.take<int32_t>((size_t)n_build);
    if (kind == TABLE_AGG) {
        b.xseg = wa.take<uint32_t>((size_t)nblk + 1);
        b.max_xseg = ceil_div(n_srec, (int64_t)kBuildSegRows);
    }
    return b;
}

// Host: reset every slot (and zero *d_status and *d_counter when given).
int table_clear(const HashView& t, int32_t* d_status, unsigned long long* d_counter, hipStream_t s);

// Host: insert n build rows into a cleared table (with an LDS build, only
// the extra slot `cap` needs clearing).  b_vals (optional, dtype b_dt) feeds
// the sums of a TABLE_AGG built with_sum.
int table_build(const HashView& t, const BuildScratch& bs, TableKind kind, const int32_t* build_key, int64_t n_build,
                bool unique, const void* b_vals, int b_dt, int32_t* d_status, hipStream_t s);

}  // namespace tdp
