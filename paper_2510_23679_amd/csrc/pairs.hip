// Best hits and bidirectional best hits for many genome pairs on gfx950.
//
// For a genome pair (A, B) the similarity of Eq. jaccard_k needs, for every
// gene pair, m = sum over shared k-mers of min(mult_a, mult_b); the sum of
// maxima over the union is then n_a + n_b - m (max + min = x + y per k-mer).
// The path never forms the |A| x |B| matrix, in HBM or in LDS:
//  1. k_join_fused: both genomes' inverted indexes are sorted by code and split into the
//     same leading-letter bucket ranges.  A work-group takes one range ("item"), stages
//     the target side in LDS and finds the partners of every query entry through the
//     bucket directory.  Per batch of query entries it counts the records each
//     accumulation tile (2^s rows of one direction) gets, reserves a run of each tile's
//     region (sized by the plan) with one atomic, and writes, per shared (k-mer, gene a,
//     gene b), a record (row in tile, column, both counts) for each requested direction.
//     Runs land in a tile's region in any order; the tile pass does not depend on it.
//  2. Back-up, gated on an overflow flag: a reservation past its region's end stops the
//     one-pass join; then k_join (count pass) counts per (item, tile), a scan of the tile
//     totals gives every tile its exact range, k_join (write pass) writes the records
//     there, and the regions are refitted to those counts for the next launch.  With no
//     overflow these kernels exit at once.  PDP_PARAM_TWO_PASS runs the two passes alone.
//  3. k_tile_ranges: each tile's record range for the tile pass.
//  4. k_tile_count: one work-group per tile sums the tile's records into m per
//     (row, column) in an LDS hash table, finds each row's maximum of
//     J = m/d by exact cross-multiplication, and counts the columns that reach
//     it, keeping the first few per row (ties kept; a row without shared
//     k-mers has no best hit), following Eq. best_hit and the per-row work of
//     Alg. 2.  A tile with more records than the table holds goes in groups of
//     rows, and a row alone past it is summed densely.  The slab copy orders
//     each row's hits by column; k_tile_write recomputes tiles with a row of
//     more ties (sorted in LDS, or densely) and writes them in column order.
//  5. k_bbh: each best hit (a, b) is kept when a is among b's best hits
//     (Eq. bidirectional_best_hit, the cross-check of Alg. 3).
// With PDP_PARAM_COLMAX a task asking for both directions writes records for its
// a-rows only; b's best hits are the rows at each column's maximum (Alg. 3): the AB
// tiles raise a 64-bit key per column that orders the values of m/d exactly, list every
// pair that reaches its column's running maximum, and the pairs still at the final
// maximum become b's best hits.
// Every output is written in a canonical order, so results do not depend on
// scheduling.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace pdp {

constexpr uint32_t kJoinThreads = 256;
constexpr uint32_t kJoinUnroll = 4;   // query entries a join thread loads at once (64-bit codes)
constexpr uint32_t kJoinUnrollP = 4;  // the same with packed keys
static_assert(kTilePer * (kTileThreads / kWave) <= kWave, "tile head counts are scanned by one wave");

// LDS of one join item: the task descriptor, the item's slice of both bucket
// directories, one counter per tile of the task, and one sub-range of the
// target side (codes and genes; the write pass also stages the counts).
struct JoinLdsBase {
    DevTask task;
    uint32_t adir[kJoinDirCap + 1];
    uint32_t bdir[kJoinDirCap + 1];
    uint32_t tcount[kJoinTileCap];  // count pass: records per tile; write pass: next slot per tile
    uint32_t scan[kJoinThreads / kWave + 1];
    uint32_t found;
    uint32_t next;
};
struct JoinLdsCount : JoinLdsBase {
    uint64_t bcode[kJoinLdsCap];
    uint32_t bgene[kJoinLdsCap];
};
struct JoinLdsWrite : JoinLdsCount {
    uint16_t bcnt[kJoinLdsCapP];  // multiplicities are at most PDP_MAX_WINDOWS
};
static_assert(sizeof(uint32_t) * kJoinLdsCap >= sizeof(uint16_t) * kJoinLdsCapP, "bucket table fits the gene stage");
static_assert(sizeof(uint64_t) * kJoinLdsCap >= sizeof(uint32_t) * kJoinLdsCapP, "packed keys reuse the code stage");
template <bool WRITE>
using JoinLds = typename std::conditional<WRITE, JoinLdsWrite, JoinLdsCount>::type;
__device__ __forceinline__ uint16_t *bcnt_of(JoinLdsWrite &L) { return L.bcnt; }
__device__ __forceinline__ uint16_t *bcnt_of(JoinLdsCount &) { return nullptr; }

// Index of the last task whose chunk_base <= chunk, found by the whole work-group with a
// 256-way search (one memory round trip per level: two levels cover 65536 tasks).
__device__ __forceinline__ uint32_t find_task_coop(const DevTask *tasks, uint32_t n_tasks, uint32_t chunk,
                                                   uint32_t *found) {
    uint32_t lo = 0, hi = n_tasks;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + blockDim.x - 1) / blockDim.x;
        if (threadIdx.x == 0) *found = 0;
        __syncthreads();
        const uint32_t idx = lo + threadIdx.x * step;
        if (idx < hi && tasks[idx].chunk_base <= chunk) atomicMax(found, threadIdx.x);
        __syncthreads();
        const uint32_t t = *found;
        __syncthreads();
        lo = lo + t * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Query entries [a0, a1) of genome a against the target entries staged from b0 on
// (bc/bg/bn, indexed relative to b0).  The partners of a query code lie in its
// leading-letter bucket, whose target range the directory slice bdir gives (index
// bucket - bl); a binary search inside that bucket finds the first equal code.
// WRITE = false adds the records each tile will receive to tcount; WRITE = true
// takes slots from the tcount cursors and writes the records.  No barriers.
template <bool WRITE, typename CN>
__device__ __forceinline__ void join_range(const DevTask &T, uint32_t a0, uint32_t a1, uint32_t b0, uint32_t nbe,
                                           const uint64_t *bc, const uint32_t *bg, const CN *bn,
                                           const uint32_t *bdir, uint32_t bl, uint32_t *tcount, uint2 *recs,
                                           uint64_t rec_cap) {
    const uint32_t k = T.a.k, lead = T.a.lead, bits = T.a.bits;
    const bool ab = T.flags & 1u, ba = T.flags & 2u;
    const uint32_t s0 = T.tile_shift[0], s1 = T.tile_shift[1], t1 = T.tiles_n[0];
    constexpr uint32_t U = kJoinUnroll;
    // each thread takes U query entries per round, strided by the work-group size; their
    // code, gene and count are loaded together up front so the global latencies overlap
    for (uint32_t base = a0; base < a1; base += U * kJoinThreads) {
        uint64_t code[U];
        uint32_t gene[U], cnt[U];
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            const uint32_t i = base + q * kJoinThreads + threadIdx.x;
            const bool v = i < a1;
            code[q] = v ? T.a.ix_code[i] : ~0ull;
            gene[q] = v ? T.a.ix_gene[i] : 0u;
            cnt[q] = v && WRITE ? T.a.ix_cnt[i] : 0u;
        }
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            if (base + q * kJoinThreads + threadIdx.x >= a1) continue;
            const uint64_t c = code[q];
            const uint32_t u = bucket_of(c, k, lead, bits) - bl;
            const uint32_t end = min(bdir[u + 1] - b0, nbe);  // the bucket lies inside the staged range
            uint32_t lo = min(bdir[u] - b0, end);
            uint32_t hi = end;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (bc[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            uint32_t m = 0;
            while (lo + m < end && bc[lo + m] == c) ++m;
            if (!m) continue;
            const uint32_t ag = gene[q];
            if (!WRITE) {
                if (ab) atomicAdd(&tcount[ag >> s0], m);
                if (ba)
                    for (uint32_t t = 0; t < m; ++t) atomicAdd(&tcount[t1 + (bg[lo + t] >> s1)], 1u);
            } else {
                const uint32_t an = cnt[q];
                if (ab) {
                    const uint32_t p = atomicAdd(&tcount[ag >> s0], m);
                    const uint32_t rl = (ag & ((1u << s0) - 1u)) << 24;
                    for (uint32_t t = 0; t < m; ++t)
                        if (p + t < rec_cap)
                            recs[p + t] = make_uint2(rl | bg[lo + t], an | (static_cast<uint32_t>(bn[lo + t]) << 16));
                }
                if (ba) {
                    for (uint32_t t = 0; t < m; ++t) {
                        const uint32_t g = bg[lo + t];
                        const uint32_t p = atomicAdd(&tcount[t1 + (g >> s1)], 1u);
                        if (p < rec_cap)
                            recs[p] = make_uint2(((g & ((1u << s1) - 1u)) << 24) | ag,
                                                 static_cast<uint32_t>(bn[lo + t]) | (an << 16));
                    }
                }
            }
        }
    }
}

// Packed form of the join, used when both dictionaries carry 32-bit (tail, gene) keys:
// entries are compared by the tail (the code without its leading letters, which the
// bucket fixes), so an entry moves 4 bytes (8 in the write pass, with its count) instead
// of 16, and twice as many target entries fit the LDS stage.  A query entry's bucket
// comes from the staged query directory (the last bucket starting at or before it).
struct JoinRoundP {
    uint32_t key[kJoinUnrollP], cnt[kJoinUnrollP];
};

template <bool WRITE>
__device__ __forceinline__ void join_load_p(const DevDict &A, uint32_t base, uint32_t a1, JoinRoundP &r) {
#pragma unroll
    for (uint32_t q = 0; q < kJoinUnrollP; ++q) {
        const uint32_t i = base + q * kJoinThreads + threadIdx.x;
        const bool v = i < a1;
        r.key[q] = v ? A.ix_key[i] : 0u;
        r.cnt[q] = v && WRITE ? A.ix_cnt[i] : 0u;
    }
}

template <bool WRITE, typename CN>
__device__ __forceinline__ void join_round_p(const DevTask &T, const JoinRoundP &r, uint32_t base, uint32_t a0,
                                             uint32_t a1, const uint16_t *abk, uint32_t jlo, uint32_t jhi,
                                             const uint32_t *adir, uint32_t b0,
                                             uint32_t nbe, const uint32_t *bk, const CN *bn,
                                             const uint32_t *bdir, uint32_t *tcount, uint2 *recs, uint64_t rec_cap) {
    const bool ab = T.flags & 1u, ba = T.flags & 2u;
    const uint32_t s0 = T.tile_shift[0], s1 = T.tile_shift[1], t1 = T.tiles_n[0];
    const uint32_t sha = T.a.key_shift, shb = T.b.key_shift;
    const uint32_t mska = (1u << sha) - 1u, mskb = (1u << shb) - 1u;
#pragma unroll
    for (uint32_t q = 0; q < kJoinUnrollP; ++q) {
        const uint32_t i = base + q * kJoinThreads + threadIdx.x;
        if (i >= a1) continue;
        const uint32_t ag = r.key[q] & mska, tail = r.key[q] >> sha;
        // bucket of entry i: from the sub-range's table, else the last directory slot in
        // [jlo, jhi) with adir <= i
        uint32_t lo = jlo, hi = jhi;
        if (abk) {
            lo = abk[i - a0];
        } else {
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (adir[mid] <= i) lo = mid;
                else hi = mid;
            }
        }
        const uint32_t end = min(bdir[lo + 1] - b0, nbe);
        uint32_t p = min(bdir[lo] - b0, end), h = end;
        while (p < h) {
            const uint32_t mid = (p + h) >> 1;
            if ((bk[mid] >> shb) < tail) p = mid + 1;
            else h = mid;
        }
        uint32_t m = 0;
        while (p + m < end && (bk[p + m] >> shb) == tail) ++m;
        if (!m) continue;
        if (!WRITE) {
            if (ab) atomicAdd(&tcount[ag >> s0], m);
            if (ba)
                for (uint32_t t = 0; t < m; ++t) atomicAdd(&tcount[t1 + ((bk[p + t] & mskb) >> s1)], 1u);
        } else {
            const uint32_t an = r.cnt[q];
            if (ab) {
                const uint32_t o = atomicAdd(&tcount[ag >> s0], m);
                const uint32_t rl = (ag & ((1u << s0) - 1u)) << 24;
                for (uint32_t t = 0; t < m; ++t)
                    if (o + t < rec_cap)
                        recs[o + t] = make_uint2(rl | (bk[p + t] & mskb), an | (static_cast<uint32_t>(bn[p + t]) << 16));
            }
            if (ba) {
                for (uint32_t t = 0; t < m; ++t) {
                    const uint32_t g = bk[p + t] & mskb;
                    const uint32_t o = atomicAdd(&tcount[t1 + (g >> s1)], 1u);
                    if (o < rec_cap)
                        recs[o] = make_uint2(((g & ((1u << s1) - 1u)) << 24) | ag, static_cast<uint32_t>(bn[p + t]) | (an << 16));
                }
            }
        }
    }
}

template <bool WRITE, typename CN>
__device__ __forceinline__ void join_range_p(const DevTask &T, JoinRoundP &r, bool loaded, uint32_t a0, uint32_t a1,
                                             const uint16_t *abk, uint32_t jlo, uint32_t jhi, const uint32_t *adir,
                                             uint32_t b0,
                                             uint32_t nbe, const uint32_t *bk, const CN *bn,
                                             const uint32_t *bdir, uint32_t *tcount, uint2 *recs, uint64_t rec_cap) {
    for (uint32_t base = a0; base < a1; base += kJoinUnrollP * kJoinThreads) {
        if (!loaded || base != a0) join_load_p<WRITE>(T.a, base, a1, r);
        join_round_p<WRITE>(T, r, base, a0, a1, abk, jlo, jhi, adir, b0, nbe, bk, bn, bdir, tcount, recs, rec_cap);
    }
}

// One join item: up to T.subs consecutive sub-ranges of T.bpw leading-letter buckets of
// one task.  The count pass stores the item's column of the task's (tile, item) count
// matrix and adds its total to *total; the write pass seeds its tile cursors from the
// scanned matrix and writes the records.  Ends with a barrier so the LDS can take the
// next item.
template <bool WRITE>
__device__ __forceinline__ void join_chunk(uint32_t chunk, const DevTask *__restrict__ tasks, uint32_t n_tasks,
                                           uint32_t *__restrict__ cells, uint32_t *__restrict__ tile_tot,
                                           const uint32_t *__restrict__ tile_off, unsigned long long *__restrict__ total,
                                           uint2 *__restrict__ recs, uint64_t rec_cap, JoinLds<WRITE> &L) {
    const uint32_t task = find_task_coop(tasks, n_tasks, chunk, &L.found);
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&tasks[task]);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&L.task);
        for (uint32_t i = threadIdx.x; i < sizeof(DevTask) / 4; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const DevTask &T = L.task;
    const uint32_t c = chunk - T.chunk_base;
    const uint32_t nb = T.a.n_buckets;
    const uint32_t span = T.bpw * T.subs;
    const uint32_t bl = c * span;
    const uint32_t bh = min(nb, bl + span);
    const uint32_t ntiles = T.tiles_n[0] + T.tiles_n[1];
    const bool packed = T.a.key_shift && T.b.key_shift;
    {  // directory slices: all loads of a thread issued before the LDS stores
        constexpr uint32_t kIters = (kJoinDirCap + 1 + kJoinThreads - 1) / kJoinThreads;
        uint32_t da[kIters], db[kIters];
#pragma unroll
        for (uint32_t it = 0; it < kIters; ++it) {
            const uint32_t i = threadIdx.x + it * kJoinThreads;
            da[it] = i <= bh - bl ? T.a.ix_dir[bl + i] : 0u;
            db[it] = i <= bh - bl ? T.b.ix_dir[bl + i] : 0u;
        }
#pragma unroll
        for (uint32_t it = 0; it < kIters; ++it) {
            const uint32_t i = threadIdx.x + it * kJoinThreads;
            if (i <= bh - bl) {
                L.adir[i] = da[it];
                L.bdir[i] = db[it];
            }
        }
    }
    // write pass: the item takes a run of each tile's range for its records, one atomic on the
    // tile's remaining count per tile it feeds; the cursors start at the runs
    const uint64_t crow = T.cell_base + static_cast<uint64_t>(c) * ntiles;
    for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
        uint32_t cur = 0;
        if (WRITE) {
            const uint32_t v = cells[crow + t], gt = T.tile_base[0] + t;
            if (v) cur = tile_off[gt] + atomicSub(&tile_tot[gt], v) - v;
        }
        L.tcount[t] = cur;
    }
    __syncthreads();
    for (uint32_t s0 = bl; s0 < bh; s0 += T.bpw) {
        const uint32_t s1 = min(bh, s0 + T.bpw);
        const uint32_t a0 = L.adir[s0 - bl], a1 = L.adir[s1 - bl];
        const uint32_t b0 = L.bdir[s0 - bl], b1 = L.bdir[s1 - bl];
        if (a0 == a1 || b0 == b1) continue;  // uniform across the work-group
        const uint32_t nbe = b1 - b0;
        if (packed) {
            JoinRoundP r;
            uint32_t *bkey = reinterpret_cast<uint32_t *>(L.bcode);  // packed keys take the code stage
            // the query entries' buckets, when they fit, in a table over the unused gene stage
            uint16_t *abk = a1 - a0 <= kJoinLdsCapP ? reinterpret_cast<uint16_t *>(L.bgene) : nullptr;
            if (nbe <= kJoinLdsCapP) {
                join_load_p<WRITE>(T.a, a0, a1, r);  // in flight while the target side is staged
                {
                    constexpr uint32_t kIters = kJoinLdsCapP / kJoinThreads;
                    uint32_t kv[kIters], cv[kIters];
#pragma unroll
                    for (uint32_t it = 0; it < kIters; ++it) {
                        const uint32_t i = threadIdx.x + it * kJoinThreads;
                        kv[it] = i < nbe ? T.b.ix_key[b0 + i] : 0u;
                        cv[it] = WRITE && i < nbe ? T.b.ix_cnt[b0 + i] : 0u;
                    }
#pragma unroll
                    for (uint32_t it = 0; it < kIters; ++it) {
                        const uint32_t i = threadIdx.x + it * kJoinThreads;
                        if (i < nbe) {
                            bkey[i] = kv[it];
                            if constexpr (WRITE) L.bcnt[i] = static_cast<uint16_t>(cv[it]);
                        }
                    }
                }
                if (abk)
                    for (uint32_t u = s0 - bl + threadIdx.x; u < s1 - bl; u += kJoinThreads)
                        for (uint32_t i = L.adir[u]; i < L.adir[u + 1]; ++i) abk[i - a0] = static_cast<uint16_t>(u);
                __syncthreads();
                join_range_p<WRITE>(T, r, true, a0, a1, abk, s0 - bl, s1 - bl, L.adir, b0, nbe, bkey,
                                    WRITE ? bcnt_of(L) : nullptr, L.bdir, L.tcount, recs, rec_cap);
                __syncthreads();
            } else {
                join_range_p<WRITE>(T, r, false, a0, a1, nullptr, s0 - bl, s1 - bl, L.adir, b0, nbe, T.b.ix_key + b0,
                                    T.b.ix_cnt + b0, L.bdir, L.tcount, recs, rec_cap);
            }
            continue;
        }
        if (nbe <= kJoinLdsCap) {
            for (uint32_t i = threadIdx.x; i < nbe; i += kJoinThreads) {
                L.bcode[i] = T.b.ix_code[b0 + i];
                L.bgene[i] = T.b.ix_gene[b0 + i];
                if constexpr (WRITE) L.bcnt[i] = T.b.ix_cnt[b0 + i];
            }
            __syncthreads();
            if constexpr (WRITE)
                join_range<true>(T, a0, a1, b0, nbe, L.bcode, L.bgene, L.bcnt, L.bdir, bl, L.tcount, recs, rec_cap);
            else
                join_range<false>(T, a0, a1, b0, nbe, L.bcode, L.bgene, static_cast<const uint16_t *>(nullptr), L.bdir,
                                  bl, L.tcount, recs, rec_cap);
            __syncthreads();  // the staged arrays take the next sub-range
        } else {
            join_range<WRITE>(T, a0, a1, b0, nbe, T.b.ix_code + b0, T.b.ix_gene + b0, T.b.ix_cnt + b0, L.bdir, bl,
                              L.tcount, recs, rec_cap);
        }
    }
    if (!WRITE) {
        __syncthreads();
        uint32_t mine = 0;
        for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
            const uint32_t v = L.tcount[t];
            cells[crow + t] = v;
            if (v) atomicAdd(&tile_tot[T.tile_base[0] + t], v);
            mine += v;
        }
        uint32_t sum;
        (void)block_exclusive_scan<kJoinThreads>(mine, L.scan, &sum);
        if (threadIdx.x == 0 && sum) atomicAdd(total, static_cast<unsigned long long>(sum));
    }
    __syncthreads();
}

__global__ void k_pairs_init(pdp_status *st, uint32_t *counters, uint32_t *tile_tot, uint32_t *fill, uint32_t n_tiles) {
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        st->code = 0;
        st->flags = 0;
        st->needed = 0;
        st->where = ~0ull;
    }
    if (i0 < 16) counters[i0] = 0;
    for (uint32_t t = i0; t < n_tiles; t += gridDim.x * blockDim.x) {
        tile_tot[t] = 0;
        fill[t] = 0;
    }
}

// The write pass stops when the records do not fit; the count pass's total is then the
// capacity needed.
__device__ __forceinline__ bool join_overflow(const unsigned long long *total, uint64_t rec_cap, pdp_status *st) {
    const unsigned long long n = *total;
    if (n <= rec_cap) return false;
    if (blockIdx.x == 0 && threadIdx.x == 0) raise_status(st, PDP_E_CAPACITY, n, 0);
    return true;
}

template <bool WRITE>
__global__ __launch_bounds__(kJoinThreads) void k_join(const DevTask *__restrict__ tasks, uint32_t n_tasks,
                                                       uint32_t *__restrict__ cells, uint32_t *__restrict__ tile_tot,
                                                       const uint32_t *__restrict__ tile_off,
                                                       unsigned long long *__restrict__ total,
                                                       uint2 *__restrict__ recs, uint64_t rec_cap, pdp_status *st,
                                                       const uint32_t *__restrict__ gate) {
    __shared__ JoinLds<WRITE> L;
    if (gate && *gate == 0u) return;  // backing up the one-pass join, which did not overflow
    if (!WRITE && gate && blockIdx.x == 0 && threadIdx.x == 0) st->flags |= PDP_STATUS_TWO_PASS;
    if (WRITE && join_overflow(total, rec_cap, st)) return;
    join_chunk<WRITE>(blockIdx.x, tasks, n_tasks, cells, tile_tot, tile_off, total, recs, rec_cap, L);
}

// Persistent form: a fixed grid claims join items kClaimJoin at a time from a counter
// (one atomic per claim, not per item) until none are left.
constexpr uint32_t kClaim = 8;
constexpr uint32_t kClaimJoin = 2;

template <bool WRITE>
__global__ __launch_bounds__(kJoinThreads) void k_join_persistent(const DevTask *__restrict__ tasks, uint32_t n_tasks,
                                                                  uint32_t total_chunks, uint32_t *__restrict__ cells,
                                                                  uint32_t *__restrict__ tile_tot,
                                                                  const uint32_t *__restrict__ tile_off,
                                                                  unsigned long long *__restrict__ total,
                                                                  uint2 *__restrict__ recs, uint64_t rec_cap,
                                                                  pdp_status *st, uint32_t *__restrict__ next,
                                                                  const uint32_t *__restrict__ gate) {
    __shared__ JoinLds<WRITE> L;
    if (gate && *gate == 0u) return;  // backing up the one-pass join, which did not overflow
    if (!WRITE && gate && blockIdx.x == 0 && threadIdx.x == 0) st->flags |= PDP_STATUS_TWO_PASS;
    if (WRITE && join_overflow(total, rec_cap, st)) return;
    for (;;) {
        if (threadIdx.x == 0) L.next = atomicAdd(next, kClaimJoin);
        __syncthreads();
        const uint32_t first = L.next;
        __syncthreads();
        if (first >= total_chunks) break;
        const uint32_t last = min(total_chunks, first + kClaimJoin);
        for (uint32_t chunk = first; chunk < last; ++chunk)
            join_chunk<WRITE>(chunk, tasks, n_tasks, cells, tile_tot, tile_off, total, recs, rec_cap, L);
    }
}

// ------------------------------------------------------------------ one-pass join
// The one-pass join searches every query entry once.  Each batch of query entries
// (kFuseUnroll per thread) is searched against the staged target side.  The records the
// batch produces are counted per tile in LDS.  Every tile the batch feeds then reserves a
// run of its record region, with one atomic on the tile's fill count.  Finally the
// records are written into those runs from LDS cursors.  The plan sizes every tile's
// region from the dictionary sizes.  A reservation that passes its region's end sets the
// fallback flag and stops the item; the count pass, the scan and the write pass then
// lay out every record again (when the flag is clear they exit at once).
constexpr uint32_t kFuseUnroll = 4;
// The LDS of a work-group sets how many fit a CU (the join waits on memory, so more work-groups
// hide more of it): the target side's multiplicities are not staged but read from the index when
// a record is written (their cache lines were just read by the staging of the keys), and items
// span at most 512 buckets; about 17 KiB, nine work-groups per CU.
struct JoinLdsFused {
    DevTask task;
    uint32_t adir[kJoinDirCap + 1];
    uint32_t bdir[kJoinDirCap + 1];
    // staged target codes, or kJoinLdsCapP packed keys; the last word pairs are spare: the
    // packed search reads up to two keys past the end of a run
    uint64_t bcode[kJoinLdsCap + 2];
    uint32_t bgene[kJoinLdsCap];  // staged target genes (64-bit codes)
    uint32_t found, next, drop;
};
// followed in dynamic LDS by two words per tile of the task: the batch's record count and
// the write cursor

// A batch of query entries: packed key or 64-bit code (one of the two arrays is used), gene
// and multiplicity.
struct FusedBatch {
    uint64_t code[kFuseUnroll];
    uint32_t key[kFuseUnroll];
    uint32_t clo[kFuseUnroll];  // low word of the code, packed keys with query buckets from codes
    uint32_t ag[kFuseUnroll], an[kFuseUnroll];
};

// Query buckets from codes.  Within an item (fewer than kJoinDirCap buckets from its first, bl) a
// packed query entry's bucket follows from the low 32 bits of its code, with no directory
// search.  Amino acids (base-20 buckets): the last three leading letters, whole in the low word
// when the tail takes at most 17 bits, give the bucket mod 8000.  Nucleotides (2-bit letters,
// base-4 buckets): the low 9 bits of the bucket, there when the tail takes at most 23 bits.
// Otherwise (kQbSearch) each entry's bucket is searched in the item's directory.  (Filling a
// table of the query entries' buckets from the directory, one thread per bucket, cost the join
// 4% more: the fill waits for the longest bucket of each wave.)
constexpr uint32_t kQbSearch = 0, kQbAmino = 1, kQbNucleotide = 2;
static_assert(kJoinDirCap <= 512, "an item's buckets are told apart by 9 bits (nucleotides), mod 8000 (amino acids)");
__device__ __forceinline__ uint32_t query_bucket_mode(const DevDict &A) {
    const uint32_t tb = A.bits * (A.k - A.lead);
    if (A.bits == 5) return tb <= 17 ? kQbAmino : kQbSearch;
    return tb <= 23 ? kQbNucleotide : kQbSearch;
}
// The item-relative bucket of a query entry whose code's low word is clo (tb tail bits).
__device__ __forceinline__ uint32_t query_bucket(uint32_t mode, uint32_t clo, uint32_t tb, uint32_t bl) {
    const uint32_t x = clo >> tb;  // leading letters, the last one lowest
    if (mode == kQbAmino) {
        const uint32_t m = (x & 31u) + ((x >> 5) & 31u) * 20u + ((x >> 10) & 31u) * 400u;  // bucket mod 8000
        const uint32_t c = bl % 8000u;
        return m >= c ? m - c : m + 8000u - c;
    }
    return (x - bl) & 511u;
}

template <bool PACKED>
__device__ __forceinline__ void fused_load(const DevDict &A, uint32_t base, uint32_t a1, uint32_t qmode, FusedBatch &r) {
#pragma unroll
    for (uint32_t q = 0; q < kFuseUnroll; ++q) {
        const uint32_t i = base + q * kJoinThreads + threadIdx.x;
        const bool v = i < a1;
        if constexpr (PACKED) {
            r.key[q] = v ? load_global(A.ix_key + i) : 0u;
            r.clo[q] = v ? load_global(reinterpret_cast<const uint32_t *>(A.ix_code + i)) : 0u;
            r.ag[q] = 0u;
        } else {
            r.code[q] = v ? load_global(A.ix_code + i) : ~0ull;
            r.ag[q] = v ? load_global(A.ix_gene + i) : 0u;
        }
        r.an[q] = v ? load_global(A.ix_cnt + i) : 0u;
    }
}

// Query entries [a0, a1) against the target entries from b0 on (nbe of them): packed keys bk
// or codes bc with genes bg, counts bn (the index's own array), all indexed relative to b0; bdir is the item's slice
// of the target directory (index bucket - bl), adir the query's.  Packed: qmode says how a query
// entry's bucket is found (query_bucket_mode), qtb is the query's tail bits.  STAGED: the packed
// keys bk are in LDS, with two readable words past the last one.  Returns false, uniformly, when
// a region overflowed.
template <bool PACKED, bool STAGED, typename CN>
__device__ __forceinline__ bool fused_range(const DevTask &T, FusedBatch &r, bool loaded, uint32_t a0, uint32_t a1,
                                            uint32_t qmode, uint32_t qtb, uint32_t jlo, uint32_t jhi, const uint32_t *adir,
                                            uint32_t bl, uint32_t b0, uint32_t nbe, const uint64_t *bc,
                                            const uint32_t *bk, const uint32_t *bg, const CN *bn, const uint32_t *bdir,
                                            uint32_t *tcount, uint32_t *tcur, uint32_t *drop,
                                            uint32_t *__restrict__ fill, const DevTile *__restrict__ tiles,
                                            uint32_t *__restrict__ fallback, uint2 *__restrict__ recs) {
    constexpr uint32_t U = kFuseUnroll;
    const bool ab = T.flags & 1u, ba = T.flags & 2u;
    const uint32_t s0 = T.tile_shift[0], s1 = T.tile_shift[1], t1 = T.tiles_n[0];
    const uint32_t ntiles = T.tiles_n[0] + T.tiles_n[1];
    const uint32_t sha = T.a.key_shift, shb = T.b.key_shift;
    const uint32_t mska = (1u << sha) - 1u, mskb = (1u << shb) - 1u;
    auto gene_at = [&](uint32_t j) -> uint32_t {
        if constexpr (PACKED) return bk[j] & mskb;
        else return bg[j];
    };
    for (uint32_t base = a0; base < a1; base += U * kJoinThreads) {
        if (!loaded || base != a0) fused_load<PACKED>(T.a, base, a1, qmode, r);
        uint32_t p[U], m[U];
        // search: the first target entry of the query's k-mer inside its bucket, and the run length
        // (packed keys compare their 32-bit tails, codes their 64 bits)
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            const uint32_t i = base + q * kJoinThreads + threadIdx.x;
            p[q] = 0;
            m[q] = 0;
            if (i >= a1) continue;
            if constexpr (PACKED) {
                const uint32_t key = r.key[q];
                r.ag[q] = key & mska;
                const uint32_t want = key >> sha;
                uint32_t u;
                if (qmode != kQbSearch) {
                    u = query_bucket(qmode, r.clo[q], qtb, bl);
                } else {  // the last directory slot in [jlo, jhi) with adir <= i
                    uint32_t lo = jlo, hi = jhi;
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (adir[mid] <= i) lo = mid;
                        else hi = mid;
                    }
                    u = lo;
                }
                const uint32_t end = min(bdir[u + 1] - b0, nbe);
                uint32_t lo = min(bdir[u] - b0, end), n = 0;
                if constexpr (STAGED) {
                    // target keys with the query's tail lie in [wlo, whi], whatever their gene
                    const uint32_t wlo = want << shb, whi = wlo | mskb;
                    // halving without an early exit: the first key >= wlo stays in [lo, lo + len]
                    // (positions as byte offsets: one shift-and-add forms a probe's address)
                    const char *bkb = reinterpret_cast<const char *>(bk);
                    uint32_t len = end - lo, lob = lo * 4u;
                    while (len > 1) {
                        const uint32_t half = len >> 1, pb = lob + half * 4u;
                        lob = *reinterpret_cast<const uint32_t *>(bkb + pb) < wlo ? pb : lob;
                        len -= half;
                    }
                    lo = lob >> 2;
                    // it is lo or lo + 1; the equal run mostly holds 0 or 1 keys, so three keys
                    // are read at once (those at or past end are not used)
                    const uint32_t k0 = bk[lo], k1 = bk[lo + 1], k2 = bk[lo + 2];
                    const bool step = len && k0 < wlo;
                    lo += step;
                    const uint32_t c0 = step ? k1 : k0, c1 = step ? k2 : k1;
                    if (lo < end && c0 <= whi) {
                        n = 1;
                        if (lo + 1 < end && c1 <= whi) {
                            n = 2;
                            while (lo + n < end && bk[lo + n] <= whi) ++n;
                        }
                    }
                } else {
                    uint32_t hi = end;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if ((bk[mid] >> shb) < want) lo = mid + 1;
                        else hi = mid;
                    }
                    while (lo + n < end && (bk[lo + n] >> shb) == want) ++n;
                }
                p[q] = lo;
                m[q] = n;
            } else {
                const uint64_t want = r.code[q];
                const uint32_t u = bucket_of(want, T.a.k, T.a.lead, T.a.bits) - bl;
                const uint32_t end = min(bdir[u + 1] - b0, nbe);
                uint32_t lo = min(bdir[u] - b0, end), hi = end;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (bc[mid] < want) lo = mid + 1;
                    else hi = mid;
                }
                uint32_t n = 0;
                while (lo + n < end && bc[lo + n] == want) ++n;
                p[q] = lo;
                m[q] = n;
            }
        }
        // count the batch's records per tile
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            if (!m[q]) continue;
            if (ab) atomicAdd(&tcount[r.ag[q] >> s0], m[q]);
            if (ba)
                for (uint32_t t = 0; t < m[q]; ++t) atomicAdd(&tcount[t1 + (gene_at(p[q] + t) >> s1)], 1u);
        }
        __syncthreads();
        // reserve a run of each fed tile's region; a run past the region's end stops the item
        for (uint32_t t = threadIdx.x; t < ntiles; t += kJoinThreads) {
            const uint32_t c = tcount[t];
            if (!c) continue;
            const uint32_t gt = T.tile_base[0] + t;
            const uint32_t at = atomicAdd(&fill[gt], c);
            const uint32_t rbase = tiles[gt].rbase, rcap = tiles[gt].rcap;
            if (static_cast<uint64_t>(at) + c > rcap) *drop = 1u;
            tcur[t] = rbase + at;
            tcount[t] = 0;
        }
        __syncthreads();
        if (*drop) {
            if (threadIdx.x == 0) atomicOr(fallback, 1u);
            return false;
        }
        // write the records into the runs: every reservation of the batch fitted its region, so
        // each record lands inside its tile's region, and the regions lie inside the capacity
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            if (!m[q]) continue;
            const uint32_t a = r.ag[q], na = r.an[q];
            if (ab) {
                const uint32_t o = atomicAdd(&tcur[a >> s0], m[q]);
                const uint32_t rl = (a & ((1u << s0) - 1u)) << 24;
                for (uint32_t t = 0; t < m[q]; ++t)
                    recs[o + t] = make_uint2(rl | gene_at(p[q] + t), na | (load_global(bn + p[q] + t) << 16));
            }
            if (ba) {
                for (uint32_t t = 0; t < m[q]; ++t) {
                    const uint32_t g = gene_at(p[q] + t);
                    const uint32_t o = atomicAdd(&tcur[t1 + (g >> s1)], 1u);
                    recs[o] = make_uint2(((g & ((1u << s1) - 1u)) << 24) | a, load_global(bn + p[q] + t) | (na << 16));
                }
            }
        }
    }
    return true;
}

// Target keys [b0, b0 + nbe) of a packed dictionary into LDS, in
// ITERS rounds of the work-group with every load issued before the first store.
template <uint32_t ITERS>
__device__ __forceinline__ void stage_packed(const DevDict &B, uint32_t b0, uint32_t nbe, uint32_t *bkey) {
    uint32_t kv[ITERS];
#pragma unroll
    for (uint32_t it = 0; it < ITERS; ++it) {
        const uint32_t i = threadIdx.x + it * kJoinThreads;
        kv[it] = i < nbe ? load_global(B.ix_key + b0 + i) : 0u;
    }
#pragma unroll
    for (uint32_t it = 0; it < ITERS; ++it) {
        const uint32_t i = threadIdx.x + it * kJoinThreads;
        if (i < nbe) bkey[i] = kv[it];
    }
}

// One item of the one-pass join (the same bucket ranges and sub-ranges as the two-pass
// join).  Ends with a barrier so the LDS can take the next item.
__device__ __forceinline__ void fused_chunk(uint32_t chunk, const DevTask *__restrict__ tasks,
                                            const DevItem *__restrict__ items, uint32_t *__restrict__ fill,
                                            const DevTile *__restrict__ tiles, uint32_t *__restrict__ fallback,
                                            uint2 *__restrict__ recs, JoinLdsFused &L,
                                            uint32_t *tcount, uint32_t *tcur, uint32_t join_tiles) {
    // set-up in one round of loads: the item (same address for every thread), then the task's
    // words and both directory slices together
    const DevItem it = items[chunk];
    {
        constexpr uint32_t kTaskWords = sizeof(DevTask) / 4;
        constexpr uint32_t kIters = (kJoinDirCap + 1 + kJoinThreads - 1) / kJoinThreads;
        static_assert(kTaskWords <= kJoinThreads, "one task word per thread");
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&tasks[it.task]);
        const uint32_t tw = threadIdx.x < kTaskWords ? src[threadIdx.x] : 0u;
        uint32_t da[kIters], db[kIters];
#pragma unroll
        for (uint32_t k = 0; k < kIters; ++k) {
            const uint32_t i = threadIdx.x + k * kJoinThreads;
            da[k] = i <= it.n_buckets ? load_global(it.adir + i) : 0u;
            db[k] = i <= it.n_buckets ? load_global(it.bdir + i) : 0u;
        }
        for (uint32_t t = threadIdx.x; t < join_tiles; t += kJoinThreads) tcount[t] = 0;
        // an item that starts after another one overflowed has nothing left to do
        if (threadIdx.x == 0) L.drop = __hip_atomic_load(fallback, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        if (threadIdx.x < kTaskWords) reinterpret_cast<uint32_t *>(&L.task)[threadIdx.x] = tw;
#pragma unroll
        for (uint32_t k = 0; k < kIters; ++k) {
            const uint32_t i = threadIdx.x + k * kJoinThreads;
            if (i <= it.n_buckets) {
                L.adir[i] = da[k];
                L.bdir[i] = db[k];
            }
        }
    }
    __syncthreads();
    const DevTask &T = L.task;
    const uint32_t bl = it.bl;
    const uint32_t bh = bl + it.n_buckets;
    const bool packed = T.a.key_shift && T.b.key_shift;
    // the same in every lane: scalar registers (as values read from LDS they would take vector ones)
    const uint32_t qmode = __builtin_amdgcn_readfirstlane(packed ? query_bucket_mode(T.a) : kQbSearch);
    const uint32_t qtb = __builtin_amdgcn_readfirstlane(T.a.bits * (T.a.k - T.a.lead));
    const bool skip = L.drop != 0;
    for (uint32_t s0 = bl; s0 < bh && !skip; s0 += T.bpw) {
        const uint32_t s1 = min(bh, s0 + T.bpw);
        const uint32_t a0 = L.adir[s0 - bl], a1 = L.adir[s1 - bl];
        const uint32_t b0 = L.bdir[s0 - bl], b1 = L.bdir[s1 - bl];
        if (a0 == a1 || b0 == b1) continue;  // uniform across the work-group
        const uint32_t nbe = b1 - b0;
        FusedBatch r;
        bool ok;
        if (packed) {
            uint32_t *bkey = reinterpret_cast<uint32_t *>(L.bcode);  // packed keys take the code stage
            if (nbe <= kJoinLdsCapP) {
                fused_load<true>(T.a, a0, a1, qmode, r);  // in flight while the target side is staged
                // a typical sub-range stages at most half the stage: half the unrolled iterations
                if (nbe <= kJoinLdsCapP / 2)
                    stage_packed<kJoinLdsCapP / 2 / kJoinThreads>(T.b, b0, nbe, bkey);
                else
                    stage_packed<kJoinLdsCapP / kJoinThreads>(T.b, b0, nbe, bkey);
                __syncthreads();
                ok = fused_range<true, true>(T, r, true, a0, a1, qmode, qtb, s0 - bl, s1 - bl, L.adir, bl, b0, nbe,
                                             nullptr, bkey, nullptr, T.b.ix_cnt + b0, L.bdir, tcount, tcur, &L.drop,
                                             fill, tiles, fallback, recs);
                __syncthreads();  // the staged arrays take the next sub-range
            } else {
                ok = fused_range<true, false>(T, r, false, a0, a1, qmode, qtb, s0 - bl, s1 - bl, L.adir, bl, b0, nbe,
                                              nullptr, T.b.ix_key + b0, nullptr, T.b.ix_cnt + b0, L.bdir, tcount, tcur,
                                              &L.drop, fill, tiles, fallback, recs);
            }
        } else if (nbe <= kJoinLdsCap) {
            for (uint32_t i = threadIdx.x; i < nbe; i += kJoinThreads) {
                L.bcode[i] = T.b.ix_code[b0 + i];
                L.bgene[i] = T.b.ix_gene[b0 + i];
            }
            __syncthreads();
            ok = fused_range<false, false>(T, r, false, a0, a1, kQbSearch, qtb, s0 - bl, s1 - bl, L.adir, bl, b0, nbe,
                                           L.bcode, nullptr, L.bgene, T.b.ix_cnt + b0, L.bdir, tcount, tcur, &L.drop,
                                           fill, tiles, fallback, recs);
            __syncthreads();
        } else {
            ok = fused_range<false, false>(T, r, false, a0, a1, kQbSearch, qtb, s0 - bl, s1 - bl, L.adir, bl, b0, nbe,
                                           T.b.ix_code + b0, nullptr, T.b.ix_gene + b0, T.b.ix_cnt + b0, L.bdir,
                                           tcount, tcur, &L.drop, fill, tiles, fallback, recs);
        }
        if (!ok) break;  // uniform: every thread read the same drop flag after a barrier
    }
    __syncthreads();
}

// Work-groups of a launch go to the XCDs in turn (work-group b to XCD b mod 8); item b' below gives
// XCD x a contiguous run of items.  The plan orders items by leading-letter bucket range across
// tasks, so an XCD works on one stretch of every genome's index at a time and its L2 serves
// the same slices to all the genome pairs that read them.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t n) {
    const uint32_t q = n / kXcds, r = n % kXcds, x = b % kXcds;
    return x * q + min(x, r) + b / kXcds;  // a bijection of [0, n)
}

__global__ __launch_bounds__(kJoinThreads) void k_join_fused(const DevTask *__restrict__ tasks,
                                                             const DevItem *__restrict__ items,
                                                             uint32_t *__restrict__ fill,
                                                             const DevTile *__restrict__ tiles,
                                                             uint32_t *__restrict__ fallback,
                                                             uint2 *__restrict__ recs,
                                                             uint32_t join_tiles) {
    __shared__ JoinLdsFused L;
    extern __shared__ uint32_t join_dyn[];
    fused_chunk(xcd_item(blockIdx.x, gridDim.x), tasks, items, fill, tiles, fallback, recs, L, join_dyn,
                join_dyn + join_tiles, join_tiles);
}

// Persistent form: XCD x (work-groups b with b mod 8 = x) claims, from a counter of its own, the
// items a one-per-item launch would run on it, in the same order, so the L2 reuse of the bucket
// ranges survives; once its own counter is spent it helps the other XCDs' in turn.  Every
// work-group ends after all eight counters are spent, whatever the grid size.
__global__ __launch_bounds__(kJoinThreads, 6) void k_join_fused_persistent(
    const DevTask *__restrict__ tasks, const DevItem *__restrict__ items, uint32_t total_chunks,
    uint32_t *__restrict__ fill, const DevTile *__restrict__ tiles, uint32_t *__restrict__ fallback,
    uint2 *__restrict__ recs, uint32_t join_tiles, uint32_t *__restrict__ next) {
    __shared__ JoinLdsFused L;
    extern __shared__ uint32_t join_dyn[];
    const uint32_t home = blockIdx.x % kXcds;
    for (uint32_t s = 0; s < kXcds; ++s) {
        const uint32_t x = (home + s) % kXcds;
        const uint32_t own = x < total_chunks ? (total_chunks - x + kXcds - 1) / kXcds : 0u;  // v = x + 8 j < total
        for (;;) {
            if (threadIdx.x == 0) L.next = atomicAdd(&next[x], kClaimJoin);
            __syncthreads();
            const uint32_t first = L.next;
            __syncthreads();
            if (first >= own) break;
            const uint32_t last = min(own, first + kClaimJoin);
            for (uint32_t j = first; j < last; ++j)
                fused_chunk(xcd_item(x + kXcds * j, total_chunks), tasks, items, fill, tiles, fallback, recs, L,
                            join_dyn, join_dyn + join_tiles, join_tiles);
        }
    }
}

// Each tile's record range for the tile kernels: its region's filled part after the
// one-pass join, its scanned range after the two-pass join.  When the two passes backed up
// the one-pass join (and the records fitted the capacity), the regions are refitted to this
// launch's exact counts: tile t's region starts at off_t + floor(slack * off_t / total), with
// off_t its scanned offset and slack the capacity left over, so every region holds its count
// and the regions still fill the capacity.  The next launch of the plan on the same
// dictionaries then fits in one pass.
__global__ void k_tile_ranges(DevTile *__restrict__ tiles, uint32_t n_tiles, const uint32_t *__restrict__ tile_off,
                              const uint32_t *__restrict__ fill, const uint32_t *__restrict__ fallback,
                              uint64_t rec_cap, uint2 *__restrict__ rng) {
    const bool two = fill == nullptr || *fallback != 0u;
    const uint64_t total = tile_off[n_tiles];
    const bool refit = fill != nullptr && two && total <= rec_cap && total > 0;
    const uint64_t slack = refit ? rec_cap - total : 0;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += gridDim.x * blockDim.x) {
        if (two) {
            const uint32_t o0 = tile_off[t], o1 = tile_off[t + 1];
            rng[t] = make_uint2(o0, o1);
            if (refit) {
                const uint64_t r0 = o0 + slack * o0 / total, r1 = o1 + slack * o1 / total;
                tiles[t].rbase = static_cast<uint32_t>(r0);
                tiles[t].rcap = static_cast<uint32_t>(r1 - r0);
            }
        } else {
            const uint32_t b = tiles[t].rbase;
            rng[t] = make_uint2(b, b + min(fill[t], tiles[t].rcap));
        }
    }
}

__device__ __forceinline__ bool j_greater(uint32_t m1, uint32_t d1, uint32_t m2, uint32_t d2) {
    return static_cast<uint64_t>(m1) * d2 > static_cast<uint64_t>(m2) * d1;
}
__device__ __forceinline__ bool j_equal(uint32_t m1, uint32_t d1, uint32_t m2, uint32_t d2) {
    return static_cast<uint64_t>(m1) * d2 == static_cast<uint64_t>(m2) * d1;
}

__device__ __forceinline__ uint32_t rec_min(uint32_t y) { return min(y & 0xFFFFu, y >> 16); }

// Candidate filters on one (row, column) pair: nr / nc windows of the two genes (their
// lengths are windows + k - 1: a pair with a shared k-mer has windows on both sides),
// sr / sc the occurrences of the shared k-mers in the row / column gene.  Eq.
// length_threshold: each length at least theta times the other; Eq. directional_jaccard:
// sr / nr and sc / nc at least tau.  Exact 64-bit products; a zero denominator is "off".
__device__ __forceinline__ bool candidate(const DevTask &T, uint32_t nr, uint32_t nc, uint32_t sr, uint32_t sc) {
    if (T.theta_d) {
        const uint64_t lr = nr + T.a.k - 1, lc = nc + T.a.k - 1;
        if (lr * T.theta_d < uint64_t(T.theta_n) * lc || lc * T.theta_d < uint64_t(T.theta_n) * lr) return false;
    }
    if (T.tau_d) {
        if (uint64_t(sr) * T.tau_d < uint64_t(T.tau_n) * nr || uint64_t(sc) * T.tau_d < uint64_t(T.tau_n) * nc)
            return false;
    }
    return true;
}

// Static LDS of a tile work-group.
struct TileLds {
    uint32_t rowlen[kTileMaxRows];    // distinct columns per row (sorted path)
    uint32_t rowfirst[kTileMaxRows];  // first distinct (row, column) of the row
    uint32_t nr[kTileMaxRows];        // window counts of the tile's rows
    uint32_t rowcnt[kTileMaxRows];    // records per row (hashed path, when the tile overflows the table)
    uint32_t ties[kTileMaxRows];      // columns at the row maximum (hashed path)
    unsigned long long best[kTileMaxRows];  // row maximum as (m << 32) | d (hashed path)
    uint32_t rank[kTilePer * (kTileThreads / kWave) + 1];
    uint32_t flag;
    uint32_t next;
    uint32_t cand_n, cand_base;  // column candidates of a row group (column maxima)
};

// Column maxima: the scratch of the tasks with kTaskColmax.
struct ColWs {
    unsigned long long *key;  // per best-hit row (a BA row): the running maximum key of its column
    uint4 *cands;             // pairs that reached their column's running maximum: (BA row, a, m, d)
    uint32_t *count;
    uint64_t cap;
};

// Key of J = m/d that orders values exactly: the bits of the correctly rounded double m / d.
// Distinct values differ by at least 1/(d1 d2) > 2^-34 (d < 2^17), far more than the rounding
// error (2^-53 relative, values at most 1), so their quotients keep their order; equal values
// round alike; positive doubles order as their bit patterns.  (An integer key floor(m 2^42 / d)
// orders them too, but its 64-bit division is a long instruction sequence per pair.)
__device__ __forceinline__ unsigned long long colmax_key(uint32_t m, uint32_t d) {
    return static_cast<unsigned long long>(__double_as_longlong(static_cast<double>(m) / static_cast<double>(d)));
}

// Raises the column's running maximum by the pair's key; true when the pair is at or above
// the maximum so far (the final maximum is never below it, so no final best hit is missed).
__device__ __forceinline__ bool colmax_raise(const ColWs &cw, uint32_t ba_row, uint32_t m, uint32_t d) {
    const unsigned long long k = colmax_key(m, d);
    return k >= atomicMax(&cw.key[ba_row], k);
}

// Best hits of one row, given its candidates one lane-chunk at a time in ascending
// column order: cand(e, &c, &m, &d) yields the column, the sum of minima and the sum of
// maxima of candidate e < n.  Pass 1 finds the exact maximum of m/d, pass 2 emits every column at the
// maximum (ballot + prefix for positions).  WRITE = false puts the first kSlab ties in
// the row's slab and the count in bh_ptr; WRITE = true writes all ties from the row's
// scanned offset.  Every lane of the wave calls it.
template <bool WRITE, typename Cand>
__device__ __forceinline__ void emit_row(uint32_t grow, uint32_t n, Cand cand,
                                         uint32_t *bh_ptr, uint4 *slab, uint32_t *bh_col, uint32_t *bh_num,
                                         uint32_t *bh_den, uint64_t bh_cap, uint32_t *flag) {
    const uint32_t lane = lane_id();
    uint32_t bm = 0, bd = 1;
    for (uint32_t e = lane; e < n; e += kWave) {
        uint32_t c, m, d;
        cand(e, &c, &m, &d);
        if (m && j_greater(m, d, bm, bd)) {
            bm = m;
            bd = d;
        }
    }
#pragma unroll
    for (uint32_t o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t om = __shfl_xor(bm, o, kWave), od = __shfl_xor(bd, o, kWave);
        if (j_greater(om, od, bm, bd)) {
            bm = om;
            bd = od;
        }
    }
    uint32_t pos = WRITE ? bh_ptr[grow] : 0u;
    if (bm) {
        for (uint32_t e0 = 0; e0 < n; e0 += kWave) {
            const uint32_t e = e0 + lane;
            uint32_t c = 0, m = 0, d = 0;
            bool tie = false;
            if (e < n) {
                cand(e, &c, &m, &d);
                tie = m && j_equal(m, d, bm, bd);
            }
            const uint64_t mask = __ballot(tie);
            const uint32_t p = pos + mask_below(mask);
            if (tie) {
                if (WRITE) {
                    if (p < bh_cap) {
                        bh_col[p] = c;
                        bh_num[p] = m;
                        bh_den[p] = d;
                    }
                } else if (p < kSlab) {
                    slab[static_cast<uint64_t>(grow) * kSlab + p] = make_uint4(c, m, d, 0);
                }
            }
            pos += static_cast<uint32_t>(__popcll(mask));
        }
    }
    if (!WRITE && lane == 0) {
        bh_ptr[grow] = pos;
        if (pos > kSlab) *flag = 1;
    }
}

// Sorted path: the tile's n <= kTileCap records sit in LDS as 64-bit keys (row 8 bits,
// column 24 bits, the two counts 32 bits); after the sort every (row, column) is one run.
// Each thread keeps its kTilePer keys (strided by the work-group size) in registers,
// ranks the run heads with one ballot scan, then the key array is reused for the
// distinct columns and their sums.
template <bool WRITE>
__device__ __forceinline__ void tile_sorted(const DevTile &tl, const DevTask &T, const uint2 *recs, uint64_t rb,
                                            uint32_t n, uint32_t *bh_ptr, uint4 *slab, uint32_t *bh_col,
                                            uint32_t *bh_num, uint32_t *bh_den, uint64_t bh_cap, uint32_t *lds,
                                            TileLds &S) {
    const DevDict &R = tl.dir == 0 ? T.a : T.b;
    const DevDict &C = tl.dir == 0 ? T.b : T.a;
    uint64_t *keys = reinterpret_cast<uint64_t *>(lds);
    for (uint32_t r = threadIdx.x; r < tl.nrows; r += kTileThreads) S.rowlen[r] = 0;
    for (uint32_t i = threadIdx.x; i < n; i += kTileThreads) {
        const uint2 r = recs[rb + i];
        keys[i] = (static_cast<uint64_t>(r.x) << 32) | r.y;
    }
    __syncthreads();
    wg_network_sort(n, [&](uint32_t lo, uint32_t hi) {
        const uint64_t x = keys[lo], y = keys[hi];
        if (x > y) {
            keys[lo] = y;
            keys[hi] = x;
        }
    });
    const uint32_t w = threadIdx.x / kWave;
    constexpr uint32_t NW = kTileThreads / kWave;
    uint64_t kr[kTilePer];
    uint32_t below[kTilePer];
    uint32_t head = 0, rstart = 0;
#pragma unroll
    for (uint32_t j = 0; j < kTilePer; ++j) {
        const uint32_t i = j * kTileThreads + threadIdx.x;
        const bool valid = i < n;
        const uint64_t x = valid ? keys[i] : 0;
        const uint64_t xp = valid && i ? keys[i - 1] : 0;
        const bool h = valid && (i == 0 || (x >> 32) != (xp >> 32));
        const bool rs = valid && (i == 0 || (x >> 56) != (xp >> 56));
        const uint64_t mask = __ballot(h);
        kr[j] = x;
        below[j] = mask_below(mask);
        head |= static_cast<uint32_t>(h) << j;
        rstart |= static_cast<uint32_t>(rs) << j;
        if (lane_id() == 0) S.rank[j * NW + w] = static_cast<uint32_t>(__popcll(mask));
    }
    __syncthreads();
    if (threadIdx.x < kWave) {  // exclusive scan of the kTilePer x NW head counts, chunk-major
        const uint32_t x = threadIdx.x < kTilePer * NW ? S.rank[threadIdx.x] : 0u;
        const uint32_t incl = wave_inclusive_sum(x);
        if (threadIdx.x < kTilePer * NW) S.rank[threadIdx.x] = incl - x;
        if (threadIdx.x == kWave - 1) S.rank[kTilePer * NW] = incl;
    }
    __syncthreads();
    const uint32_t u = S.rank[kTilePer * NW];  // distinct (row, column)
    uint32_t *ucol = lds;                      // (row << 24) | column, per distinct pair
    uint32_t *msum = lds + kTileCap;           // sum of minima, per distinct pair
    uint32_t *ssum = lds + 2 * kTileCap;       // with filters: both sums of counts (16 bits each)
    const bool filt = T.theta_d || T.tau_d;
    for (uint32_t r = threadIdx.x; r < u; r += kTileThreads) {
        msum[r] = 0;
        if (filt) ssum[r] = 0;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kTilePer; ++j) {
        const uint32_t i = j * kTileThreads + threadIdx.x;
        if (i >= n) continue;
        const bool h = (head >> j) & 1u;
        const uint32_t r = S.rank[j * NW + w] + below[j] + (h ? 0u : ~0u);  // rank of the run head
        const uint32_t row = static_cast<uint32_t>(kr[j] >> 56);
        if (h) {
            ucol[r] = static_cast<uint32_t>(kr[j] >> 32);
            atomicAdd(&S.rowlen[row], 1u);
            if ((rstart >> j) & 1u) S.rowfirst[row] = r;
        }
        const uint32_t y = static_cast<uint32_t>(kr[j]);
        atomicAdd(&msum[r], rec_min(y));
        if (filt) atomicAdd(&ssum[r], y);  // each half stays below 2^16: no carry
    }
    __syncthreads();
    // window counts in one round trip for the whole tile: the column's joins its sum
    // (both at most 16 bits), the rows' go to S.nr
    for (uint32_t r = threadIdx.x; r < u; r += kTileThreads) {
        const uint32_t c = ucol[r] & 0xFFFFFFu;
        msum[r] |= (c < C.n_genes ? load_global(C.nwin + c) : 0u) << 16;  // a column past the genome is never a row's
    }
    for (uint32_t rl = threadIdx.x; rl < tl.nrows; rl += kTileThreads) S.nr[rl] = load_global(R.nwin + tl.row0 + rl);
    __syncthreads();
    for (uint32_t rl = w; rl < tl.nrows; rl += NW) {
        const uint32_t len = S.rowlen[rl];
        const uint32_t beg = len ? S.rowfirst[rl] : 0u;
        const uint32_t nr = S.nr[rl];
        emit_row<WRITE>(T.row_base[tl.dir] + tl.row0 + rl, len,
                        [&](uint32_t e, uint32_t *c, uint32_t *m, uint32_t *d) {
                            const uint32_t v = msum[beg + e];
                            *c = ucol[beg + e] & 0xFFFFFFu;
                            *m = v & 0xFFFFu;
                            *d = nr + (v >> 16) - *m;
                            if (filt) {
                                const uint32_t sv = ssum[beg + e];
                                if (!candidate(T, nr, v >> 16, sv & 0xFFFFu, sv >> 16)) *m = 0;  // not a candidate
                            }
                        },
                        bh_ptr, slab, bh_col, bh_num, bh_den, bh_cap, &S.flag);
    }
}

// Dense path for rows [rlo, rhi) of a tile whose records overflow LDS otherwise: the
// column genome's window counts (16 bits each) stay in LDS, and groups of rows are
// summed into 16-bit LDS accumulators (two per word) with a touched-word bitmap; each
// group rescans the tile's records.  With candidate filters two more accumulators per
// row hold the occurrence sums of each gene.  Rows visit only their touched words.
template <bool WRITE, bool CM = false>
__device__ __forceinline__ void tile_dense(const DevTile &tl, const DevTask &T, const uint2 *recs, uint64_t rb,
                                           uint32_t n, uint32_t rlo, uint32_t rhi, uint32_t lds_words,
                                           uint32_t *bh_ptr, uint4 *slab,
                                           uint32_t *bh_col, uint32_t *bh_num, uint32_t *bh_den, uint64_t bh_cap,
                                           uint32_t *lds, TileLds &S, const ColWs *cmx) {
    const bool colmax = CM && !WRITE && cmx && (T.flags & kTaskColmax) && tl.dir == 0;
    const DevDict &R = tl.dir == 0 ? T.a : T.b;
    const DevDict &C = tl.dir == 0 ? T.b : T.a;
    const bool filt = T.theta_d || T.tau_d;
    const uint32_t ncols = C.n_genes;
    const uint32_t W = (ncols + 1) >> 1;  // accumulator words per row and sum
    const uint32_t WB = (W + 31) >> 5;    // bitmap words per row
    const uint32_t NA = filt ? 3 : 1;     // sums per column: minima (+ row and column occurrences)
    const uint32_t cw_words = (W + 3) & ~3u;
    uint16_t *cw = reinterpret_cast<uint16_t *>(lds);
    for (uint32_t c = threadIdx.x; c < ncols; c += kTileThreads) cw[c] = static_cast<uint16_t>(load_global(C.nwin + c));
    uint32_t *acc_base = lds + cw_words;
    const uint32_t G = (lds_words - cw_words) / (NA * W + WB);  // rows per pass, at least 1 by plan
    const uint32_t wave = threadIdx.x / kWave;
    for (uint32_t g0 = rlo; g0 < rhi; g0 += G) {
        const uint32_t gn = min(G, rhi - g0);
        uint32_t *acc = acc_base;              // [gn][W] minima
        uint32_t *asr = acc_base + gn * W;     // [gn][W] row occurrences (filters)
        uint32_t *asc = asr + gn * W;          // [gn][W] column occurrences (filters)
        uint32_t *bits = acc_base + NA * gn * W;
        const uint32_t words = gn * (NA * W + WB);
        for (uint32_t i = threadIdx.x; i < words; i += kTileThreads) acc[i] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += kTileThreads) {
            const uint2 r = recs[rb + i];
            const uint32_t rr = (r.x >> 24) - g0;
            const uint32_t c = r.x & 0xFFFFFFu, wd = c >> 1;
            if (rr >= gn || c >= ncols) continue;
            const uint32_t sh = (c & 1u) << 4;
            const uint32_t old = atomicAdd(&acc[rr * W + wd], rec_min(r.y) << sh);
            if (filt) {
                atomicAdd(&asr[rr * W + wd], (r.y & 0xFFFFu) << sh);
                atomicAdd(&asc[rr * W + wd], (r.y >> 16) << sh);
            }
            if (old == 0) atomicOr(&bits[rr * WB + (wd >> 5)], 1u << (wd & 31u));
        }
        __syncthreads();
        for (uint32_t rr = wave; rr < gn; rr += kTileThreads / kWave) {
            const uint32_t row = tl.row0 + g0 + rr;
            const uint32_t *arow = acc + rr * W;
            const uint32_t *srow = asr + rr * W;
            const uint32_t *crow = asc + rr * W;
            const uint32_t *brow = bits + rr * WB;
            // candidates: the touched words of the row, two columns each, in ascending order;
            // a lane walks one bitmap word, so lane chunks of 64 words stay in column order
            const uint32_t lane = lane_id();
            const uint32_t grow = T.row_base[tl.dir] + row;
            const uint32_t nr = load_global(R.nwin + row);
            // sum of minima of column 2*wd + h, or 0 when the pair is filtered out
            auto mval = [&](uint32_t wd, uint32_t h) -> uint32_t {
                const uint32_t sh = h << 4;
                const uint32_t m = (arow[wd] >> sh) & 0xFFFFu;
                if (!m || !filt) return m;
                return candidate(T, nr, cw[2 * wd + h], (srow[wd] >> sh) & 0xFFFFu, (crow[wd] >> sh) & 0xFFFFu) ? m
                                                                                                                : 0u;
            };
            uint32_t bm = 0, bd = 1;
            for (uint32_t bw = lane; bw < WB; bw += kWave) {
                for (uint32_t msk = brow[bw]; msk;) {
                    const uint32_t wd = (bw << 5) + (__ffs(msk) - 1);
                    msk &= msk - 1;
#pragma unroll
                    for (uint32_t h = 0; h < 2; ++h) {
                        const uint32_t m = mval(wd, h);
                        if (!m) continue;
                        const uint32_t d = nr + cw[2 * wd + h] - m;
                        if (j_greater(m, d, bm, bd)) {
                            bm = m;
                            bd = d;
                        }
                        // column maxima (rows past the hash table are rare: one global slot each)
                        if (colmax && colmax_raise(*cmx, T.row_base[1] + 2 * wd + h, m, d)) {
                            const uint32_t idx = atomicAdd(cmx->count, 1u);
                            if (idx < cmx->cap) cmx->cands[idx] = make_uint4(T.row_base[1] + 2 * wd + h, row, m, d);
                        }
                    }
                }
            }
#pragma unroll
            for (uint32_t o = kWave / 2; o > 0; o >>= 1) {
                const uint32_t om = __shfl_xor(bm, o, kWave), od = __shfl_xor(bd, o, kWave);
                if (j_greater(om, od, bm, bd)) {
                    bm = om;
                    bd = od;
                }
            }
            uint32_t pos = WRITE ? bh_ptr[grow] : 0u;
            if (bm) {
                for (uint32_t b0 = 0; b0 < WB; b0 += kWave) {
                    const uint32_t bw = b0 + lane;
                    const uint32_t mask = bw < WB ? brow[bw] : 0u;
                    uint32_t cnt = 0;
                    for (uint32_t msk = mask; msk;) {
                        const uint32_t wd = (bw << 5) + (__ffs(msk) - 1);
                        msk &= msk - 1;
#pragma unroll
                        for (uint32_t h = 0; h < 2; ++h) {
                            const uint32_t m = mval(wd, h);
                            if (m && j_equal(m, nr + cw[2 * wd + h] - m, bm, bd)) ++cnt;
                        }
                    }
                    const uint32_t incl = wave_inclusive_sum(cnt);
                    const uint32_t total = __shfl(incl, kWave - 1, kWave);
                    uint32_t p = pos + incl - cnt;
                    for (uint32_t msk = cnt ? mask : 0u; msk;) {
                        const uint32_t wd = (bw << 5) + (__ffs(msk) - 1);
                        msk &= msk - 1;
#pragma unroll
                        for (uint32_t h = 0; h < 2; ++h) {
                            const uint32_t mm = mval(wd, h);
                            if (!mm) continue;
                            const uint32_t c = 2 * wd + h;
                            const uint32_t d = nr + cw[c] - mm;
                            if (!j_equal(mm, d, bm, bd)) continue;
                            if (WRITE) {
                                if (p < bh_cap) {
                                    bh_col[p] = c;
                                    bh_num[p] = mm;
                                    bh_den[p] = d;
                                }
                            } else if (p < kSlab) {
                                slab[static_cast<uint64_t>(grow) * kSlab + p] = make_uint4(c, mm, d, 0);
                            }
                            ++p;
                        }
                    }
                    pos += total;
                }
            }
            if (!WRITE && lane == 0) {
                bh_ptr[grow] = pos;
                if (pos > kSlab) S.flag = 1;
            }
        }
        __syncthreads();
    }
}

// Hashed path of the first tile launch, for rows [g0, g1) of a tile (filter: skip the
// tile's records of other rows): the sums of minima per (row, column) collect in an LDS
// open-addressing table of kHashSlots (key = record field + 1, so 0 marks a free slot)
// holding at most kHashMax distinct pairs.  Then one thread per slot: the column's
// window count is gathered (one round trip for the whole table), d = n_row + n_col - m,
// and the row maximum of m/d is kept as (m, d) by an exact compare-and-swap loop
// (64-bit cross-multiplication).  A second sweep counts the columns at the maximum
// (ties) and puts the first kSlab of them, unordered, in the row's slab; the slab copy
// orders them by column.
template <bool CM>
__device__ __forceinline__ void tile_hashed(const DevTile &tl, const DevTask &T, const uint2 *recs, uint64_t rb,
                                            uint32_t n, uint32_t g0, uint32_t g1, bool filter, uint32_t *bh_ptr,
                                            uint4 *slab, uint32_t *lds, TileLds &S, const ColWs &cmx) {
    const bool colmax = CM && (T.flags & kTaskColmax) && tl.dir == 0;
    const DevDict &R = tl.dir == 0 ? T.a : T.b;
    const DevDict &C = tl.dir == 0 ? T.b : T.a;
    const bool filt = T.theta_d || T.tau_d;
    uint32_t *hk = lds;
    uint32_t *hv = lds + kHashSlots;
    uint32_t *hs = lds + 2 * kHashSlots;  // with filters: occurrences of the row and column genes (16 bits each)
    uint4 *z = reinterpret_cast<uint4 *>(lds);
    for (uint32_t i = threadIdx.x; i < (filt ? 3 : 2) * kHashSlots / 4; i += kTileThreads) z[i] = make_uint4(0, 0, 0, 0);
    for (uint32_t rl = g0 + threadIdx.x; rl < g1; rl += kTileThreads) {
        S.best[rl] = 0;
        S.ties[rl] = 0;
        S.nr[rl] = load_global(R.nwin + tl.row0 + rl);
    }
    __syncthreads();
    const uint32_t ncols = C.n_genes;
    constexpr uint32_t kRB = 4;  // records a thread loads per round, all before its inserts
    for (uint32_t base = 0; base < n; base += kRB * kTileThreads) {
        uint2 rr[kRB];
#pragma unroll
        for (uint32_t q = 0; q < kRB; ++q) {
            const uint32_t i = base + q * kTileThreads + threadIdx.x;
            rr[q] = i < n ? recs[rb + i] : make_uint2(0xFFFFFFFFu, 0u);
        }
#pragma unroll
        for (uint32_t q = 0; q < kRB; ++q) {
            const uint2 r = rr[q];
            if (base + q * kTileThreads + threadIdx.x >= n) continue;
            // rows and columns are checked, so no record can address past the tile's rows or
            // the column genome's window counts
            if ((r.x >> 24) - g0 >= g1 - g0 || (r.x & 0xFFFFFFu) >= ncols) continue;
            const uint32_t key = r.x + 1;  // columns stay below 2^24 - 1, so no wrap to 0
            uint32_t h = (key * 2654435761u) >> (32 - kHashBits);
            for (;;) {  // ends: at most kHashMax < kHashSlots keys are distinct
                const uint32_t prev = atomicCAS(&hk[h], 0u, key);
                if (prev == 0u || prev == key) break;
                h = (h + 1) & (kHashSlots - 1);
            }
            atomicAdd(&hv[h], rec_min(r.y));
            if (filt) atomicAdd(&hs[h], r.y);  // each half stays below 2^16: no carry
        }
    }
    __syncthreads();
    constexpr uint32_t kSlotsPer = kHashSlots / kTileThreads;
    static_assert(kSlotsPer <= 32, "a thread's column candidates fit one mask word");
    uint32_t ncw[kSlotsPer];  // the column window counts of a thread's slots, gathered together
    uint32_t app = 0;         // column maxima: this thread's slots at their column's running maximum
#pragma unroll
    for (uint32_t q = 0; q < kSlotsPer; ++q) {
        const uint32_t key = hk[q * kTileThreads + threadIdx.x];
        ncw[q] = key ? load_global(C.nwin + ((key - 1) & 0xFFFFFFu)) : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < kSlotsPer; ++q) {
        const uint32_t sl = q * kTileThreads + threadIdx.x;
        const uint32_t key = hk[sl];
        if (!key) continue;
        const uint32_t rl = (key - 1) >> 24;
        uint32_t m = hv[sl];  // at most PDP_MAX_WINDOWS
        const uint32_t nc = ncw[q];
        if (filt && !candidate(T, S.nr[rl], nc, hs[sl] & 0xFFFFu, hs[sl] >> 16)) m = 0;  // not a candidate
        hv[sl] = m | (nc << 16);
        if (!m) continue;
        const uint32_t d = S.nr[rl] + nc - m;
        if (colmax && colmax_raise(cmx, T.row_base[1] + ((key - 1) & 0xFFFFFFu), m, d)) app |= 1u << q;
        const unsigned long long want = (static_cast<unsigned long long>(m) << 32) | d;
        unsigned long long cur = S.best[rl];
        for (;;) {
            const uint32_t om = static_cast<uint32_t>(cur >> 32), od = static_cast<uint32_t>(cur);
            if (om && !j_greater(m, d, om, od)) break;
            const unsigned long long prev = atomicCAS(&S.best[rl], cur, want);
            if (prev == cur) break;
            cur = prev;
        }
    }
    __syncthreads();
    if (colmax) {  // uniform per tile: the row group's candidates go out with one global atomic
        if (threadIdx.x == 0) S.cand_n = 0;
        __syncthreads();
        const uint32_t mine = __popc(app);
        uint32_t off = mine ? atomicAdd(&S.cand_n, mine) : 0u;
        __syncthreads();
        if (threadIdx.x == 0 && S.cand_n) S.cand_base = atomicAdd(cmx.count, S.cand_n);
        __syncthreads();
#pragma unroll
        for (uint32_t q = 0; q < kSlotsPer; ++q) {
            if (!((app >> q) & 1u)) continue;
            const uint32_t sl = q * kTileThreads + threadIdx.x;
            const uint32_t key = hk[sl], v = hv[sl];
            const uint32_t rl = (key - 1) >> 24, m = v & 0xFFFFu;
            const uint64_t idx = uint64_t(S.cand_base) + off++;
            if (idx < cmx.cap)
                cmx.cands[idx] = make_uint4(T.row_base[1] + ((key - 1) & 0xFFFFFFu), tl.row0 + rl, m, S.nr[rl] + (v >> 16) - m);
        }
    }
    const uint32_t rbase = T.row_base[tl.dir] + tl.row0;
    for (uint32_t sl = threadIdx.x; sl < kHashSlots; sl += kTileThreads) {
        const uint32_t key = hk[sl];
        if (!key) continue;
        const uint32_t rl = (key - 1) >> 24, c = (key - 1) & 0xFFFFFFu;
        const uint32_t v = hv[sl];
        const uint32_t m = v & 0xFFFFu, d = S.nr[rl] + (v >> 16) - m;
        if (!m) continue;  // filtered out
        const unsigned long long b = S.best[rl];
        if (!j_equal(m, d, static_cast<uint32_t>(b >> 32), static_cast<uint32_t>(b))) continue;
        const uint32_t t = atomicAdd(&S.ties[rl], 1u);
        if (t < kSlab) slab[static_cast<uint64_t>(rbase + rl) * kSlab + t] = make_uint4(c, m, d, 0);
    }
    __syncthreads();
    for (uint32_t rl = g0 + threadIdx.x; rl < g1; rl += kTileThreads) {
        const uint32_t cnt = S.ties[rl];
        bh_ptr[rbase + rl] = cnt;
        if (cnt > kSlab) S.flag = 1;
    }
    __syncthreads();  // the table takes the next row group
}

// One tile: its records are tile_rng[tile] (its region's filled part, or its range of the
// scanned tile totals, clamped to the record capacity, so a capacity overflow reads no further).  The first
// launch (WRITE = false) hashes the tile, or, past kHashMax records, groups of whole rows
// that fit the table (a row alone beyond it is summed densely); ties go to per-row slabs
// and counts to bh_ptr, and a tile with a row of more than kSlab ties is listed for the
// second launch (WRITE = true), which recomputes it by sorting (or densely) and writes
// its rows straight into the CSR output in column order.
template <bool WRITE, bool CM = false>
__device__ __forceinline__ void tile_process(uint32_t tile_id, const DevTask *__restrict__ tasks,
                                             const DevTile *__restrict__ tiles, const uint2 *__restrict__ tile_rng,
                                             const uint2 *__restrict__ recs, uint64_t rec_cap,
                                             const unsigned long long *__restrict__ total, uint32_t lds_words,
                                             uint32_t *__restrict__ bh_ptr, uint4 *__restrict__ slab,
                                             uint32_t *__restrict__ bh_col, uint32_t *__restrict__ bh_num,
                                             uint32_t *__restrict__ bh_den, uint64_t bh_cap, uint32_t *overflow_tiles,
                                             uint32_t *overflow_count, uint32_t *lds, TileLds &S, const ColWs &cmx) {
    const DevTile tl = tiles[tile_id];
    const DevTask &T = tasks[tl.task];
    // when the join's records overflowed the scratch its write pass wrote none: every tile is
    // empty then (the status already asks for a larger capacity)
    const uint2 rg = tile_rng[tile_id];
    const uint64_t c0 = rg.x, c1 = rg.y;
    const uint64_t rb = min(c0, rec_cap);
    const uint64_t re = *total > rec_cap ? rb : max(rb, min(c1, rec_cap));
    const uint32_t n = static_cast<uint32_t>(re - rb);
    if (threadIdx.x == 0) S.flag = 0;
    __syncthreads();
    if (WRITE) {
        if (n <= kTileCap)
            tile_sorted<true>(tl, T, recs, rb, n, bh_ptr, slab, bh_col, bh_num, bh_den, bh_cap, lds, S);
        else
            tile_dense<true>(tl, T, recs, rb, n, 0, tl.nrows, lds_words, bh_ptr, slab, bh_col, bh_num, bh_den, bh_cap,
                             lds, S, nullptr);
    } else if (n <= kHashMax) {
        tile_hashed<CM>(tl, T, recs, rb, n, 0, tl.nrows, false, bh_ptr, slab, lds, S, cmx);
    } else {
        for (uint32_t rl = threadIdx.x; rl < tl.nrows; rl += kTileThreads) S.rowcnt[rl] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += kTileThreads) atomicAdd(&S.rowcnt[recs[rb + i].x >> 24], 1u);
        __syncthreads();
        // every thread walks the same counts, so the group loop is uniform
        for (uint32_t g0 = 0; g0 < tl.nrows;) {
            if (S.rowcnt[g0] > kHashMax) {
                tile_dense<false, CM>(tl, T, recs, rb, n, g0, g0 + 1, lds_words, bh_ptr, slab, nullptr, nullptr, nullptr,
                                      0, lds, S, &cmx);
                ++g0;
                continue;
            }
            uint32_t g1 = g0, sum = 0;
            while (g1 < tl.nrows && sum + S.rowcnt[g1] <= kHashMax) sum += S.rowcnt[g1++];
            tile_hashed<CM>(tl, T, recs, rb, n, g0, g1, true, bh_ptr, slab, lds, S, cmx);
            g0 = g1;
        }
    }
    __syncthreads();
    if (!WRITE && threadIdx.x == 0 && S.flag) overflow_tiles[atomicAdd(overflow_count, 1u)] = tile_id;
    __syncthreads();
}

// CM: the plan has column-maximum tasks (a separate instance, so the default carries none of it).
template <bool CM>
__global__ __launch_bounds__(kTileThreads) void k_tile_count(const DevTask *__restrict__ tasks,
                                                             const DevTile *__restrict__ tiles,
                                                             const uint2 *__restrict__ tile_rng,
                                                             const uint2 *__restrict__ recs, uint64_t rec_cap,
                                                             const unsigned long long *__restrict__ total,
                                                             uint32_t lds_words, uint32_t *__restrict__ bh_ptr,
                                                             uint4 *__restrict__ slab, uint32_t *overflow_tiles,
                                                             uint32_t *overflow_count, ColWs cmx) {
    extern __shared__ uint32_t lds[];
    __shared__ TileLds S;
    tile_process<false, CM>(blockIdx.x, tasks, tiles, tile_rng, recs, rec_cap, total, lds_words, bh_ptr, slab, nullptr,
                            nullptr, nullptr, 0, overflow_tiles, overflow_count, lds, S, cmx);
}

// Persistent form: a fixed grid pulls tiles from a counter until none are left.
template <bool CM>
__global__ __launch_bounds__(kTileThreads) void k_tile_count_persistent(
    const DevTask *__restrict__ tasks, const DevTile *__restrict__ tiles, uint32_t total_tiles,
    const uint2 *__restrict__ tile_rng, const uint2 *__restrict__ recs, uint64_t rec_cap,
    const unsigned long long *__restrict__ total, uint32_t lds_words, uint32_t *__restrict__ bh_ptr,
    uint4 *__restrict__ slab, uint32_t *overflow_tiles, uint32_t *overflow_count, uint32_t *__restrict__ next, ColWs cmx) {
    extern __shared__ uint32_t lds[];
    __shared__ TileLds S;
    for (;;) {
        if (threadIdx.x == 0) S.next = atomicAdd(next, kClaim);
        __syncthreads();
        const uint32_t first = S.next;
        __syncthreads();
        if (first >= total_tiles) break;
        const uint32_t last = min(total_tiles, first + kClaim);
        for (uint32_t t = first; t < last; ++t)
            tile_process<false, CM>(t, tasks, tiles, tile_rng, recs, rec_cap, total, lds_words, bh_ptr, slab, nullptr,
                                    nullptr, nullptr, 0, overflow_tiles, overflow_count, lds, S, cmx);
    }
}

// Rows with more ties than the slab holds: their tiles again, written to the CSR output.
__global__ __launch_bounds__(kTileThreads) void k_tile_write(const DevTask *__restrict__ tasks,
                                                             const DevTile *__restrict__ tiles,
                                                             const uint2 *__restrict__ tile_rng,
                                                             const uint2 *__restrict__ recs, uint64_t rec_cap,
                                                             const unsigned long long *__restrict__ total,
                                                             uint32_t lds_words, uint32_t *__restrict__ bh_ptr,
                                                             uint32_t *__restrict__ bh_col, uint32_t *__restrict__ bh_num,
                                                             uint32_t *__restrict__ bh_den, uint64_t bh_cap,
                                                             const uint32_t *__restrict__ overflow_tiles,
                                                             const uint32_t *__restrict__ overflow_count) {
    extern __shared__ uint32_t lds[];
    __shared__ TileLds S;
    const uint32_t n = *overflow_count;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x)
        tile_process<true>(overflow_tiles[i], tasks, tiles, tile_rng, recs, rec_cap, total, lds_words, bh_ptr, nullptr, bh_col,
                           bh_num, bh_den, bh_cap, nullptr, nullptr, lds, S, ColWs{});
}

// One thread per best-hit row: the slab entries of a row with at most kSlab ties go to the CSR output.
__global__ __launch_bounds__(256) void k_slab_copy(uint32_t bh_rows, const uint32_t *__restrict__ bh_ptr,
                                                   const uint4 *__restrict__ slab, uint32_t *__restrict__ bh_col,
                                                   uint32_t *__restrict__ bh_num, uint32_t *__restrict__ bh_den,
                                                   uint64_t bh_cap, pdp_status *st) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0 && bh_ptr[bh_rows] > bh_cap) raise_status(st, PDP_E_CAPACITY, bh_ptr[bh_rows], 1);
    if (r >= bh_rows) return;
    const uint32_t p = bh_ptr[r], n = bh_ptr[r + 1] - p;
    if (n > kSlab) return;
    uint4 e[kSlab];
#pragma unroll
    for (uint32_t i = 0; i < kSlab; ++i) e[i] = i < n ? slab[static_cast<uint64_t>(r) * kSlab + i] : make_uint4(~0u, 0, 0, 0);
    // the first tile launch leaves a row's ties in any order: insertion sort by column
#pragma unroll
    for (uint32_t i = 1; i < kSlab; ++i)
#pragma unroll
        for (uint32_t j = i; j > 0; --j)
            if (e[j - 1].x > e[j].x) {
                const uint4 t = e[j - 1];
                e[j - 1] = e[j];
                e[j] = t;
            }
#pragma unroll
    for (uint32_t i = 0; i < kSlab; ++i) {
        if (i >= n || p + i >= bh_cap) continue;
        bh_col[p + i] = e[i].x;
        bh_num[p + i] = e[i].y;
        bh_den[p + i] = e[i].z;
    }
}

// Column maxima, after the AB tiles: every listed pair still at its column's final maximum
// is a best hit of the column's gene (Alg. 3's test S[l,k] = max_r S[r,k]).  The count goes
// to the BA row's bh_ptr and the first kSlab hits to its slab, as the tiles do for AB rows.
__global__ __launch_bounds__(256) void k_colmax_rows(ColWs cmx, uint32_t *__restrict__ bh_ptr, uint4 *__restrict__ slab,
                                                     pdp_status *st) {
    const uint32_t n = *cmx.count;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n > cmx.cap) raise_status(st, PDP_E_CAPACITY, n, 0);
    const uint64_t lim = min(static_cast<uint64_t>(n), cmx.cap);
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < lim; i += gridDim.x * 256ull) {
        const uint4 c = cmx.cands[i];
        if (colmax_key(c.z, c.w) != cmx.key[c.x]) continue;
        const uint32_t t = atomicAdd(&bh_ptr[c.x], 1u);
        if (t < kSlab) slab[static_cast<uint64_t>(c.x) * kSlab + t] = make_uint4(c.y, c.z, c.w, 0);
    }
}

// After the scan: hits of BA rows with more than kSlab of them go straight to the CSR (in
// any order; k_colmax_sort orders those rows), slots taken from a per-row cursor.
__global__ __launch_bounds__(256) void k_colmax_big(ColWs cmx, uint32_t *__restrict__ cursor,
                                                    const uint32_t *__restrict__ bh_ptr, uint32_t *__restrict__ bh_col,
                                                    uint32_t *__restrict__ bh_num, uint32_t *__restrict__ bh_den,
                                                    uint64_t bh_cap) {
    const uint64_t lim = min(static_cast<uint64_t>(*cmx.count), cmx.cap);
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < lim; i += gridDim.x * 256ull) {
        const uint4 c = cmx.cands[i];
        if (colmax_key(c.z, c.w) != cmx.key[c.x]) continue;
        const uint32_t p = bh_ptr[c.x];
        if (bh_ptr[c.x + 1] - p <= kSlab) continue;
        const uint64_t pos = uint64_t(p) + atomicAdd(&cursor[c.x], 1u);
        if (pos < bh_cap) {
            bh_col[pos] = c.y;
            bh_num[pos] = c.z;
            bh_den[pos] = c.w;
        }
    }
}

// One thread per row that k_colmax_big filled: insertion sort of its hits by column.
__global__ __launch_bounds__(256) void k_colmax_sort(uint32_t bh_rows, const uint32_t *__restrict__ cursor,
                                                     const uint32_t *__restrict__ bh_ptr, uint32_t *__restrict__ bh_col,
                                                     uint32_t *__restrict__ bh_num, uint32_t *__restrict__ bh_den,
                                                     uint64_t bh_cap) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= bh_rows || !cursor[r]) return;
    const uint64_t p0 = bh_ptr[r], p1 = min(static_cast<uint64_t>(bh_ptr[r + 1]), bh_cap);
    for (uint64_t x = p0 + 1; x < p1; ++x) {
        const uint32_t c = bh_col[x], m = bh_num[x], d = bh_den[x];
        uint64_t y = x;
        while (y > p0 && bh_col[y - 1] > c) {
            bh_col[y] = bh_col[y - 1];
            bh_num[y] = bh_num[y - 1];
            bh_den[y] = bh_den[y - 1];
            --y;
        }
        bh_col[y] = c;
        bh_num[y] = m;
        bh_den[y] = d;
    }
}

// BBH of one row: keep each best hit (a, b) whose reverse row contains a.  Every read stays
// inside the best-hit arrays' capacity (bh_cap) and a column b outside the reverse rows
// (ncols) is skipped, so a corrupt or overflowed input cannot send the walk out of bounds;
// the callers stop before this when the best-hit output overflowed.
template <bool WRITE>
__device__ __forceinline__ void bbh_row(uint32_t a, uint32_t grow, uint32_t rab, uint32_t ba_base, uint32_t ncols,
                                        const uint32_t *ab_ptr, const uint32_t *ab_col, const uint32_t *ab_num,
                                        const uint32_t *ab_den, uint64_t ab_cap, const uint32_t *ba_ptr,
                                        const uint32_t *ba_col, uint64_t ba_cap, uint32_t *out_ptr, uint32_t *out_a,
                                        uint32_t *out_b, uint32_t *out_num, uint32_t *out_den, uint64_t cap) {
    uint32_t pos = WRITE ? out_ptr[grow] : 0u;
    const uint64_t pend = min(static_cast<uint64_t>(ab_ptr[rab + 1]), ab_cap);
    for (uint64_t p = ab_ptr[rab]; p < pend; ++p) {
        const uint32_t b = ab_col[p];
        if (b >= ncols) continue;
        const uint32_t rba = ba_base + b;
        bool found = false;
        const uint64_t qend = min(static_cast<uint64_t>(ba_ptr[rba + 1]), ba_cap);
        for (uint64_t q = ba_ptr[rba]; q < qend; ++q) {
            const uint32_t x = ba_col[q];
            if (x >= a) {
                found = x == a;
                break;
            }
        }
        if (found) {
            if (WRITE && pos < cap) {
                out_a[pos] = a;
                out_b[pos] = b;
                out_num[pos] = ab_num[p];
                out_den[pos] = ab_den[p];
            }
            ++pos;
        }
    }
    if (!WRITE) out_ptr[grow] = pos;
}

// The task table is stored in processing order (largest tasks first); order[]
// lists it in the caller's order, in which BBH row bases increase.
__device__ __forceinline__ uint32_t find_bbh_task(const DevTask *tasks, const uint32_t *order, uint32_t n_tasks,
                                                  uint32_t row) {
    uint32_t lo = 0, hi = n_tasks - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (tasks[order[mid]].bbh_row_base <= row) lo = mid;
        else hi = mid - 1;
    }
    return order[lo];
}

// BBH of a plan: one thread per BBH row.  When an earlier kernel of the launch raised an
// error (record or best-hit capacity, the best-hit entries then being incomplete), no row
// is walked: the count pass writes zeros and the write pass writes nothing.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_bbh(const DevTask *__restrict__ tasks, const uint32_t *__restrict__ order,
                                             uint32_t n_tasks, uint32_t bbh_rows, uint32_t bh_rows,
                                             const uint32_t *__restrict__ bh_ptr, const uint32_t *__restrict__ bh_col,
                                             const uint32_t *__restrict__ bh_num, const uint32_t *__restrict__ bh_den,
                                             uint64_t bh_cap, uint32_t *__restrict__ out_ptr, uint32_t *__restrict__ out_a,
                                             uint32_t *__restrict__ out_b, uint32_t *__restrict__ out_num,
                                             uint32_t *__restrict__ out_den, uint64_t cap, pdp_status *st) {
    const uint32_t grow = blockIdx.x * blockDim.x + threadIdx.x;
    if (grow >= bbh_rows) return;
    if (st->code != 0 || bh_ptr[bh_rows] > bh_cap) {
        if (!WRITE) out_ptr[grow] = 0;
        return;
    }
    if (WRITE && grow == 0 && out_ptr[bbh_rows] > cap) raise_status(st, PDP_E_CAPACITY, out_ptr[bbh_rows], 2);
    const DevTask &T = tasks[find_bbh_task(tasks, order, n_tasks, grow)];
    const uint32_t a = grow - T.bbh_row_base;  // a gene of the caller's a
    const bool sw = T.flags & kTaskSwapped;    // the caller's a is the task's b
    const uint32_t ab_base = T.row_base[sw ? 1 : 0], ba_base = T.row_base[sw ? 0 : 1];
    bbh_row<WRITE>(a, grow, ab_base + a, ba_base, sw ? T.a.n_genes : T.b.n_genes, bh_ptr, bh_col, bh_num, bh_den, bh_cap,
                   bh_ptr, bh_col, bh_cap, out_ptr, out_a, out_b, out_num, out_den, cap);
}

// pdp_bbh: the two best-hit outputs are the caller's.  A total past an output's capacity
// (an overflowed best-hit call) is PDP_E_CAPACITY (where = 1), a column past the reverse
// output's rows PDP_E_INVAL (where = the row); either way nothing is walked.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_bbh_pair(uint32_t rows, const uint32_t *__restrict__ ab_ptr,
                                                  const uint32_t *__restrict__ ab_col, const uint32_t *__restrict__ ab_num,
                                                  const uint32_t *__restrict__ ab_den, uint64_t ab_cap,
                                                  const uint32_t *__restrict__ ba_ptr, const uint32_t *__restrict__ ba_col,
                                                  uint32_t ba_rows, uint64_t ba_cap, uint32_t *__restrict__ out_ptr,
                                                  uint32_t *__restrict__ out_a, uint32_t *__restrict__ out_b,
                                                  uint32_t *__restrict__ out_num, uint32_t *__restrict__ out_den,
                                                  uint64_t cap, pdp_status *st) {
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= rows) return;
    const uint32_t ab_tot = ab_ptr[rows], ba_tot = ba_ptr[ba_rows];
    if (ab_tot > ab_cap || ba_tot > ba_cap) {
        if (a == 0 && !WRITE) raise_status(st, PDP_E_CAPACITY, ab_tot > ab_cap ? ab_tot : ba_tot, 1);
        if (!WRITE) out_ptr[a] = 0;
        return;
    }
    if (WRITE && a == 0 && out_ptr[rows] > cap) raise_status(st, PDP_E_CAPACITY, out_ptr[rows], 2);
    // a column index past the reverse output's rows cannot name a best hit there
    for (uint32_t p = ab_ptr[a]; p < ab_ptr[a + 1]; ++p) {
        if (ab_col[p] >= ba_rows) {
            if (!WRITE) {
                raise_status(st, PDP_E_INVAL, 0, a);
                out_ptr[a] = 0;
            }
            return;
        }
    }
    bbh_row<WRITE>(a, a, a, 0, ba_rows, ab_ptr, ab_col, ab_num, ab_den, ab_cap, ba_ptr, ba_col, ba_cap, out_ptr, out_a,
                   out_b, out_num, out_den, cap);
}

// ------------------------------------------------------------------ long genes
// Rows of the tasks that name a dictionary bound for long genes, whose multiplicities and sums
// of minima may pass 16 bits.  One work-group computes a row on its own, as Eq. jaccard_k
// reads: for every k-mer of the row gene's multiplicity vector it finds the k-mer in the column
// genome's index (its leading-letter bucket, then a binary search on the code) and adds
// min(count in the row gene, count in the column gene) to that column gene's 32-bit LDS sum;
// with the filters the occurrence sums of both genes are kept the same way.  The column genes
// are taken kLongCols at a time in ascending order: a first sweep finds the row's maximum of
// m/d (Eq. best_hit, exact 64-bit cross-multiplication), a second one emits the columns at the
// maximum in column order.  WRITE = false puts the first kSlab ties in the row's slab and the
// count in bh_ptr, as the tiles do; WRITE = true writes the rows with more than kSlab ties
// straight into the CSR output after the scan.
constexpr uint32_t kLongThreads = 256;
constexpr uint32_t kLongGrid = 4096;   // work-groups at most; each takes rows in turn

template <bool WRITE>
__global__ __launch_bounds__(kLongThreads) void k_long_rows(const DevTask *__restrict__ tasks,
                                                            const DevLongSeg *__restrict__ segs, uint32_t n_segs,
                                                            uint32_t n_rows, uint32_t *__restrict__ bh_ptr,
                                                            uint4 *__restrict__ slab, uint32_t *__restrict__ bh_col,
                                                            uint32_t *__restrict__ bh_num, uint32_t *__restrict__ bh_den,
                                                            uint64_t bh_cap) {
    // dynamic LDS: the sums of minima per column gene of the block, and with filters the
    // occurrences in the row gene and in the column gene of the shared k-mers (kLongCols each)
    extern __shared__ uint32_t long_lds[];
    uint32_t *acc = long_lds;
    uint32_t *asr = long_lds + kLongCols;
    uint32_t *asc = long_lds + 2 * kLongCols;
    __shared__ uint32_t red[2 * (kLongThreads / kWave)];
    constexpr uint32_t NW = kLongThreads / kWave;
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    for (uint32_t lr = blockIdx.x; lr < n_rows; lr += gridDim.x) {
        uint32_t lo = 0, hi = n_segs;  // the last segment whose first row is <= lr (segments are non-empty)
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (segs[mid].first <= lr) lo = mid;
            else hi = mid;
        }
        const DevLongSeg sg = segs[lo];
        const DevTask &T = tasks[sg.task];
        const DevDict &R = sg.dir == 0 ? T.a : T.b;
        const DevDict &C = sg.dir == 0 ? T.b : T.a;
        const uint32_t row = lr - sg.first;
        const uint32_t grow = T.row_base[sg.dir] + row;
        const uint32_t pos0 = WRITE ? bh_ptr[grow] : 0u;
        if (WRITE && bh_ptr[grow + 1] - pos0 <= kSlab) continue;  // the slab copy placed this row
        const bool filt = T.theta_d || T.tau_d;
        const uint32_t nr = load_global(R.nwin + row);
        const uint32_t e0 = load_global(R.mv_ptr + row), e1 = load_global(R.mv_ptr + row + 1);
        const uint32_t ncols = C.n_genes;
        const uint32_t nblk = (ncols + kLongCols - 1) / kLongCols;
        // sums of column genes [c0, c0 + cn) into acc / asr / asc
        auto accumulate = [&](uint32_t c0, uint32_t cn) {
            for (uint32_t i = tid; i < cn; i += kLongThreads) {
                acc[i] = 0;
                if (filt) {
                    asr[i] = 0;
                    asc[i] = 0;
                }
            }
            __syncthreads();
            for (uint32_t e = e0 + tid; e < e1; e += kLongThreads) {
                const uint64_t code = load_global(R.mv_code + e);
                const uint32_t cr = load_global(R.mv_cnt + e);
                const uint32_t b = bucket_of(code, C.k, C.lead, C.bits);
                if (b >= C.n_buckets) continue;  // not a k-mer of the alphabet: in no index
                const uint32_t end = load_global(C.ix_dir + b + 1);
                uint32_t l = load_global(C.ix_dir + b), h = end;  // first entry of the code: entries ascend by (code, gene)
                while (l < h) {
                    const uint32_t mid = (l + h) >> 1;
                    if (load_global(C.ix_code + mid) < code) l = mid + 1;
                    else h = mid;
                }
                for (uint32_t i = l; i < end && load_global(C.ix_code + i) == code; ++i) {
                    const uint32_t g = load_global(C.ix_gene + i) - c0;  // genes below c0 wrap past cn
                    if (g >= cn) continue;
                    const uint32_t cc = load_global(C.ix_cnt + i);
                    atomicAdd(&acc[g], min(cr, cc));
                    if (filt) {
                        atomicAdd(&asr[g], cr);
                        atomicAdd(&asc[g], cc);
                    }
                }
            }
            __syncthreads();
        };
        // (m, d) of column c0 + i of the block, m = 0 when the pair shares nothing or is filtered out
        auto value = [&](uint32_t c0, uint32_t i, uint32_t *m, uint32_t *d) {
            *m = acc[i];
            *d = 0;
            if (!*m) return;
            const uint32_t nc = load_global(C.nwin + c0 + i);
            if (filt && !candidate(T, nr, nc, asr[i], asc[i])) {
                *m = 0;
                return;
            }
            *d = nr + nc - *m;  // below 2^32: both window counts are at most PDP_MAX_WINDOWS_LONG
        };
        uint32_t bm = 0, bd = 1;
        for (uint32_t blk = 0; blk < nblk; ++blk) {
            const uint32_t c0 = blk * kLongCols, cn = min(kLongCols, ncols - c0);
            accumulate(c0, cn);
            for (uint32_t i = tid; i < cn; i += kLongThreads) {
                uint32_t m, d;
                value(c0, i, &m, &d);
                if (m && j_greater(m, d, bm, bd)) {
                    bm = m;
                    bd = d;
                }
            }
            __syncthreads();  // the next block clears the sums
        }
#pragma unroll
        for (uint32_t o = kWave / 2; o > 0; o >>= 1) {
            const uint32_t om = __shfl_xor(bm, o, kWave), od = __shfl_xor(bd, o, kWave);
            if (j_greater(om, od, bm, bd)) {
                bm = om;
                bd = od;
            }
        }
        if (lane == 0) {
            red[w] = bm;
            red[NW + w] = bd;
        }
        __syncthreads();
        bm = 0;
        bd = 1;
        for (uint32_t v = 0; v < NW; ++v)
            if (j_greater(red[v], red[NW + v], bm, bd)) {
                bm = red[v];
                bd = red[NW + v];
            }
        __syncthreads();
        uint32_t pos = 0;  // ties so far, in column order
        if (bm) {
            for (uint32_t blk = 0; blk < nblk; ++blk) {
                const uint32_t c0 = blk * kLongCols, cn = min(kLongCols, ncols - c0);
                if (nblk > 1) accumulate(c0, cn);  // a single block still holds its sums
                // wave w takes a contiguous quarter of the block's columns: it counts its ties,
                // then, after one barrier, emits them from its offset in column order
                const uint32_t q = (cn + NW - 1) / NW, lo = min(cn, w * q), hi = min(cn, lo + q);
                uint32_t mine = 0;
                for (uint32_t i0 = lo; i0 < hi; i0 += kWave) {
                    const uint32_t i = i0 + lane;
                    uint32_t m = 0, d = 0;
                    if (i < hi) value(c0, i, &m, &d);
                    mine += static_cast<uint32_t>(__popcll(__ballot(m && j_equal(m, d, bm, bd))));
                }
                if (lane == 0) red[w] = mine;
                __syncthreads();
                uint32_t at = pos, total = 0;
                for (uint32_t v = 0; v < NW; ++v) {
                    if (v < w) at += red[v];
                    total += red[v];
                }
                for (uint32_t i0 = lo; i0 < hi; i0 += kWave) {
                    const uint32_t i = i0 + lane;
                    uint32_t m = 0, d = 0;
                    if (i < hi) value(c0, i, &m, &d);
                    const bool tie = m && j_equal(m, d, bm, bd);
                    const uint64_t mask = __ballot(tie);
                    const uint32_t p = at + mask_below(mask);
                    if (tie) {
                        if (WRITE) {
                            const uint64_t dst = uint64_t(pos0) + p;
                            if (dst < bh_cap) {
                                bh_col[dst] = c0 + i;
                                bh_num[dst] = m;
                                bh_den[dst] = d;
                            }
                        } else if (p < kSlab) {
                            slab[static_cast<uint64_t>(grow) * kSlab + p] = make_uint4(c0 + i, m, d, 0);
                        }
                    }
                    at += static_cast<uint32_t>(__popcll(mask));
                }
                pos += total;
                __syncthreads();  // the next block clears the sums and the counts
            }
        }
        if (!WRITE && tid == 0) bh_ptr[grow] = pos;
    }
}

// ------------------------------------------------------------------ host

static uint32_t device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    return cus > 0 ? static_cast<uint32_t>(cus) : 1u;
}

uint32_t persistent_join_grid() {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_join_persistent<true>, kJoinThreads, 0) != hipSuccess || per < 1)
        per = 1;
    return device_cus() * static_cast<uint32_t>(per);
}

uint32_t persistent_fused_grid(uint32_t join_tiles) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_join_fused_persistent, kJoinThreads, 8 * join_tiles) !=
            hipSuccess ||
        per < 1)
        per = 1;
    return device_cus() * static_cast<uint32_t>(per);
}

uint32_t persistent_tile_grid(uint32_t tile_lds) {
    int per = 0;
    int per_cm = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tile_count_persistent<false>, kTileThreads, tile_lds) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cm, k_tile_count_persistent<true>, kTileThreads, tile_lds) !=
            hipSuccess)
        per = 1;
    per = std::min(per, per_cm);  // one grid size for both instances
    if (per < 1) per = 1;
    return device_cus() * static_cast<uint32_t>(per);
}

// Tiles above 64 KiB of dynamic LDS need the kernels' limit raised (gfx950 has 160 KiB per work-group).
hipError_t allow_tile_lds(uint32_t tile_lds) {
    if (tile_lds <= 64 * 1024) return hipSuccess;
    const int v = static_cast<int>(tile_lds);
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_count<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, v));
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_count<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, v));
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_count_persistent<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, v));
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_count_persistent<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, v));
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_write), hipFuncAttributeMaxDynamicSharedMemorySize, v));
    return hipSuccess;
}

static uint64_t pair_partials(const PlanShape &p) {
    return std::max({scan_partials(p.total_tiles), scan_partials(p.bh_rows), scan_partials(p.bbh_rows)});
}

uint64_t pair_ws_bytes(const PlanShape &p) {
    const uint64_t A = 256;
    uint64_t s = 0;
    s += align_up(sizeof(DevTask) * std::max<uint64_t>(p.n_tasks, 1), A);
    s += align_up(sizeof(DevTile) * std::max<uint64_t>(p.total_tiles, 1), A);
    s += align_up(sizeof(DevItem) * std::max<uint64_t>(p.total_chunks, 1), A);
    s += align_up(4 * std::max<uint64_t>(p.n_tasks, 1), A);
    s += align_up(8 * std::max<uint64_t>(p.rec_cap, 1), A);
    s += align_up(64, A);
    s += align_up(4 * (uint64_t(p.total_cells) + 1), A);
    s += align_up(4 * (uint64_t(p.total_tiles) + 1), A);  // records per tile (join), consumed by the write pass
    s += align_up(4 * (uint64_t(p.total_tiles) + 1), A);  // scanned: each tile's first record
    s += align_up(4 * (uint64_t(p.total_tiles) + 1), A);  // one-pass join: records reserved per region
    s += align_up(8 * (uint64_t(p.total_tiles) + 1), A);  // record range of each tile
    s += align_up(16 * kSlab * (uint64_t(p.bh_rows) + 1), A);
    s += align_up(4 * (uint64_t(p.total_tiles) + 1), A);
    s += align_up(4 * pair_partials(p), A);
    const uint64_t colrows = p.colmax ? uint64_t(p.bh_rows) + 1 : 1;
    s += align_up(8 * colrows, A);                                  // column keys
    s += align_up(4 * colrows, A);                                  // big-row cursors
    s += align_up(16 * std::max<uint64_t>(p.colmax ? p.cand_cap : 0, 1), A);  // candidates
    s += align_up(sizeof(DevLongSeg) * std::max<uint64_t>(p.n_long_segs, 1), A);
    return s;
}

PairWs pair_ws_carve(void *ws, const PlanShape &p) {
    const uint64_t A = 256;
    char *q = static_cast<char *>(ws);
    auto take = [&](uint64_t bytes) {
        char *r = q;
        q += align_up(bytes, A);
        return r;
    };
    PairWs w;
    w.tasks = reinterpret_cast<DevTask *>(take(sizeof(DevTask) * std::max<uint64_t>(p.n_tasks, 1)));
    w.tiles = reinterpret_cast<DevTile *>(take(sizeof(DevTile) * std::max<uint64_t>(p.total_tiles, 1)));
    w.items = reinterpret_cast<DevItem *>(take(sizeof(DevItem) * std::max<uint64_t>(p.total_chunks, 1)));
    w.order = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(p.n_tasks, 1)));
    w.recs = reinterpret_cast<uint2 *>(take(8 * std::max<uint64_t>(p.rec_cap, 1)));
    w.counters = reinterpret_cast<unsigned long long *>(take(64));
    w.overflow_count = reinterpret_cast<uint32_t *>(w.counters) + 2;
    w.next_join = reinterpret_cast<uint32_t *>(w.counters) + 3;
    w.next_tile = reinterpret_cast<uint32_t *>(w.counters) + 4;
    w.next_join_write = reinterpret_cast<uint32_t *>(w.counters) + 5;
    w.cells = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_cells) + 1)));
    w.tile_tot = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_tiles) + 1)));
    w.tile_off = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_tiles) + 1)));
    w.fill = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_tiles) + 1)));
    w.tile_rng = reinterpret_cast<uint2 *>(take(8 * (uint64_t(p.total_tiles) + 1)));
    w.fallback = reinterpret_cast<uint32_t *>(w.counters) + 7;
    w.next_fused = reinterpret_cast<uint32_t *>(w.counters) + 8;
    w.slab = reinterpret_cast<uint4 *>(take(16 * kSlab * (uint64_t(p.bh_rows) + 1)));
    w.overflow_tiles = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_tiles) + 1)));
    w.partials = reinterpret_cast<uint32_t *>(take(4 * pair_partials(p)));
    const uint64_t colrows = p.colmax ? uint64_t(p.bh_rows) + 1 : 1;
    w.colkey = reinterpret_cast<unsigned long long *>(take(8 * colrows));
    w.colcursor = reinterpret_cast<uint32_t *>(take(4 * colrows));
    w.cands = reinterpret_cast<uint4 *>(take(16 * std::max<uint64_t>(p.colmax ? p.cand_cap : 0, 1)));
    w.cand_count = reinterpret_cast<uint32_t *>(w.counters) + 6;
    w.long_segs = reinterpret_cast<DevLongSeg *>(take(sizeof(DevLongSeg) * std::max<uint64_t>(p.n_long_segs, 1)));
    return w;
}

hipError_t launch_pairs(const PlanShape &p, const PairWs &w, pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *st,
                        hipStream_t s, const KernelTimer *timer) {
    auto mark = [&](int32_t kernel, bool begin) -> hipError_t {
        if (!timer || timer->kernel != kernel) return hipSuccess;
        return hipEventRecord(begin ? timer->start : timer->stop, s);
    };
    const uint32_t lds_words = p.tile_lds / 4;
    PDP_TRY(mark(PDP_KERNEL_ALL, true));
    // status and counters (record total (64 bits), overflow tiles, next join item (count
    // pass), next tile, next join item (write pass), column candidates) in one launch
    hipLaunchKernelGGL(k_pairs_init, dim3(std::max<uint32_t>(1, std::min<uint32_t>(1024, (p.total_tiles + 255) / 256))),
                       dim3(256), 0, s, st, reinterpret_cast<uint32_t *>(w.counters), w.tile_tot, w.fill, p.total_tiles);
    PDP_TRY(hipGetLastError());
    const ColWs cmx{w.colkey, w.cands, w.cand_count, p.colmax ? p.cand_cap : 0};
    if (p.colmax) {  // BA rows are counted by atomics; column keys and cursors start at zero
        PDP_TRY(launch_fill_u32(bh->ptr, uint64_t(p.bh_rows) + 1, 0u, s));
        PDP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(w.colkey), 2 * (uint64_t(p.bh_rows) + 1), 0u, s));
        PDP_TRY(launch_fill_u32(w.colcursor, uint64_t(p.bh_rows) + 1, 0u, s));
    }
    // the join: the one-pass kernel (PDP_KERNEL_JOIN), then its back-up, the two-pass join gated on
    // the fallback flag (PDP_KERNEL_JOIN_BACKUP); with PDP_PARAM_TWO_PASS the two passes are the join
    if (p.total_chunks) {
        const bool pers = p.join_grid != 0;
        const uint32_t *gate = nullptr;
        bool two_pers = pers;
        dim3 g2 = pers ? dim3(std::min(p.join_grid, (p.total_chunks + kClaimJoin - 1) / kClaimJoin)) : dim3(p.total_chunks);
        if (p.fused) {
            const uint32_t dyn = 8 * p.join_tiles;
            PDP_TRY(mark(PDP_KERNEL_JOIN, true));
            if (pers)
                hipLaunchKernelGGL(k_join_fused_persistent,
                                   dim3(std::min(p.join_grid, (p.total_chunks + kClaimJoin - 1) / kClaimJoin)),
                                   dim3(kJoinThreads), dyn, s, w.tasks, w.items, p.total_chunks, w.fill, w.tiles,
                                   w.fallback, w.recs, p.join_tiles, w.next_fused);
            else
                hipLaunchKernelGGL(k_join_fused, dim3(p.total_chunks), dim3(kJoinThreads), dyn, s, w.tasks, w.items,
                                   w.fill, w.tiles, w.fallback, w.recs, p.join_tiles);
            PDP_TRY(hipGetLastError());
            PDP_TRY(mark(PDP_KERNEL_JOIN, false));
            PDP_TRY(mark(PDP_KERNEL_JOIN_BACKUP, true));
            // the back-up is persistent and gated: a few empty work-groups when no region overflowed
            gate = w.fallback;
            two_pers = true;
            g2 = dim3(std::max<uint32_t>(1, std::min(p.fallback_grid, (p.total_chunks + kClaimJoin - 1) / kClaimJoin)));
        } else {
            PDP_TRY(mark(PDP_KERNEL_JOIN, true));
        }
        if (two_pers)
            hipLaunchKernelGGL(k_join_persistent<false>, g2, dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, p.total_chunks,
                               w.cells, w.tile_tot, w.tile_off, w.counters, w.recs, p.rec_cap, st, w.next_join, gate);
        else
            hipLaunchKernelGGL(k_join<false>, g2, dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, w.cells, w.tile_tot,
                               w.tile_off, w.counters, w.recs, p.rec_cap, st, gate);
        PDP_TRY(hipGetLastError());
        PDP_TRY(mark(PDP_KERNEL_BUCKET, true));
        PDP_TRY(launch_scan(w.tile_tot, w.tile_off, p.total_tiles, w.partials, s));
        PDP_TRY(mark(PDP_KERNEL_BUCKET, false));
        if (two_pers)
            hipLaunchKernelGGL(k_join_persistent<true>, g2, dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, p.total_chunks,
                               w.cells, w.tile_tot, w.tile_off, w.counters, w.recs, p.rec_cap, st, w.next_join_write, gate);
        else
            hipLaunchKernelGGL(k_join<true>, g2, dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, w.cells, w.tile_tot,
                               w.tile_off, w.counters, w.recs, p.rec_cap, st, gate);
        PDP_TRY(hipGetLastError());
        if (!p.fused) {
            PDP_TRY(mark(PDP_KERNEL_JOIN, false));
            PDP_TRY(mark(PDP_KERNEL_JOIN_BACKUP, true));
        }
    } else {  // no join items (every task on the long-gene path): empty intervals for the join timers
        PDP_TRY(mark(PDP_KERNEL_JOIN, true));
        PDP_TRY(mark(PDP_KERNEL_JOIN, false));
        PDP_TRY(mark(PDP_KERNEL_BUCKET, true));
        PDP_TRY(mark(PDP_KERNEL_BUCKET, false));
        PDP_TRY(mark(PDP_KERNEL_JOIN_BACKUP, true));
        PDP_TRY(launch_fill_u32(w.tile_off, uint64_t(p.total_tiles) + 1, 0u, s));
    }
    if (p.total_tiles) {
        hipLaunchKernelGGL(k_tile_ranges, dim3(std::min<uint32_t>(1024, (p.total_tiles + 255) / 256)), dim3(256), 0, s,
                           w.tiles, p.total_tiles, w.tile_off, p.fused && p.total_chunks ? w.fill : nullptr, w.fallback,
                           p.rec_cap, w.tile_rng);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(mark(PDP_KERNEL_JOIN_BACKUP, false));
    PDP_TRY(mark(PDP_KERNEL_TILE_COUNT, true));
    if (p.total_tiles && p.tile_grid) {
        const dim3 g(std::min(p.tile_grid, (p.total_tiles + kClaim - 1) / kClaim));
        if (p.colmax)
            hipLaunchKernelGGL(k_tile_count_persistent<true>, g, dim3(kTileThreads), p.tile_lds, s, w.tasks, w.tiles,
                               p.total_tiles, w.tile_rng, w.recs, p.rec_cap, w.counters, lds_words, bh->ptr, w.slab,
                               w.overflow_tiles, w.overflow_count, w.next_tile, cmx);
        else
            hipLaunchKernelGGL(k_tile_count_persistent<false>, g, dim3(kTileThreads), p.tile_lds, s, w.tasks, w.tiles,
                               p.total_tiles, w.tile_rng, w.recs, p.rec_cap, w.counters, lds_words, bh->ptr, w.slab,
                               w.overflow_tiles, w.overflow_count, w.next_tile, cmx);
        PDP_TRY(hipGetLastError());
    } else if (p.total_tiles) {
        if (p.colmax)
            hipLaunchKernelGGL(k_tile_count<true>, dim3(p.total_tiles), dim3(kTileThreads), p.tile_lds, s, w.tasks,
                               w.tiles, w.tile_rng, w.recs, p.rec_cap, w.counters, lds_words, bh->ptr, w.slab,
                               w.overflow_tiles, w.overflow_count, cmx);
        else
            hipLaunchKernelGGL(k_tile_count<false>, dim3(p.total_tiles), dim3(kTileThreads), p.tile_lds, s, w.tasks,
                               w.tiles, w.tile_rng, w.recs, p.rec_cap, w.counters, lds_words, bh->ptr, w.slab,
                               w.overflow_tiles, w.overflow_count, cmx);
        PDP_TRY(hipGetLastError());
    }
    const uint32_t col_grid = std::max<uint32_t>(1, std::min<uint32_t>(2048, static_cast<uint32_t>((p.cand_cap + 255) / 256)));
    if (p.colmax) {
        hipLaunchKernelGGL(k_colmax_rows, dim3(col_grid), dim3(256), 0, s, cmx, bh->ptr, w.slab, st);
        PDP_TRY(hipGetLastError());
    }
    const dim3 long_grid(std::min(p.long_rows, kLongGrid));
    if (p.long_rows) {
        hipLaunchKernelGGL(k_long_rows<false>, long_grid, dim3(kLongThreads), p.long_lds, s, w.tasks, w.long_segs, p.n_long_segs,
                           p.long_rows, bh->ptr, w.slab, nullptr, nullptr, nullptr, 0);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(mark(PDP_KERNEL_TILE_COUNT, false));
    PDP_TRY(launch_scan(bh->ptr, bh->ptr, p.bh_rows, w.partials, s));
    PDP_TRY(mark(PDP_KERNEL_TILE_WRITE, true));
    if (p.bh_rows) {
        hipLaunchKernelGGL(k_slab_copy, dim3((p.bh_rows + 255) / 256), dim3(256), 0, s, p.bh_rows, bh->ptr, w.slab,
                           bh->col, bh->num, bh->den, bh->capacity, st);
        PDP_TRY(hipGetLastError());
    }
    if (p.total_tiles) {
        const uint32_t g = p.total_tiles < 256 ? p.total_tiles : 256;
        hipLaunchKernelGGL(k_tile_write, dim3(g), dim3(kTileThreads), p.tile_lds, s, w.tasks, w.tiles, w.tile_rng, w.recs,
                           p.rec_cap, w.counters, lds_words, bh->ptr, bh->col, bh->num, bh->den, bh->capacity, w.overflow_tiles,
                           w.overflow_count);
        PDP_TRY(hipGetLastError());
    }
    if (p.long_rows) {
        hipLaunchKernelGGL(k_long_rows<true>, long_grid, dim3(kLongThreads), p.long_lds, s, w.tasks, w.long_segs, p.n_long_segs,
                           p.long_rows, bh->ptr, nullptr, bh->col, bh->num, bh->den, bh->capacity);
        PDP_TRY(hipGetLastError());
    }
    if (p.colmax && p.bh_rows) {
        hipLaunchKernelGGL(k_colmax_big, dim3(col_grid), dim3(256), 0, s, cmx, w.colcursor, bh->ptr, bh->col, bh->num,
                           bh->den, bh->capacity);
        PDP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_colmax_sort, dim3((p.bh_rows + 255) / 256), dim3(256), 0, s, p.bh_rows, w.colcursor, bh->ptr,
                           bh->col, bh->num, bh->den, bh->capacity);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(mark(PDP_KERNEL_TILE_WRITE, false));
    PDP_TRY(mark(PDP_KERNEL_BBH, true));
    if (p.bbh_rows && bbh) {
        const uint32_t g = (p.bbh_rows + 255) / 256;
        hipLaunchKernelGGL(k_bbh<false>, dim3(g), dim3(256), 0, s, w.tasks, w.order, p.n_tasks, p.bbh_rows, p.bh_rows,
                           bh->ptr, bh->col, bh->num, bh->den, bh->capacity, bbh->ptr, bbh->a, bbh->b, bbh->num, bbh->den,
                           bbh->capacity, st);
        PDP_TRY(hipGetLastError());
        PDP_TRY(launch_scan(bbh->ptr, bbh->ptr, p.bbh_rows, w.partials, s));
        hipLaunchKernelGGL(k_bbh<true>, dim3(g), dim3(256), 0, s, w.tasks, w.order, p.n_tasks, p.bbh_rows, p.bh_rows,
                           bh->ptr, bh->col, bh->num, bh->den, bh->capacity, bbh->ptr, bbh->a, bbh->b, bbh->num, bbh->den,
                           bbh->capacity, st);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(mark(PDP_KERNEL_BBH, false));
    PDP_TRY(mark(PDP_KERNEL_ALL, false));
    return hipSuccess;
}


hipError_t launch_bbh_standalone(const pdp_bh_out *ab, const pdp_bh_out *ba, pdp_bbh_out *out, pdp_status *st,
                                 uint32_t *partials, hipStream_t s) {
    PDP_TRY(launch_status_init(st, s));
    const uint32_t rows = ab->n_rows;
    if (rows) {
        const uint32_t g = (rows + 255) / 256;
        hipLaunchKernelGGL(k_bbh_pair<false>, dim3(g), dim3(256), 0, s, rows, ab->ptr, ab->col, ab->num, ab->den,
                           ab->capacity, ba->ptr, ba->col, ba->n_rows, ba->capacity, out->ptr, out->a, out->b, out->num,
                           out->den, out->capacity, st);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(launch_scan(out->ptr, out->ptr, rows, partials, s));
    if (rows) {
        const uint32_t g = (rows + 255) / 256;
        hipLaunchKernelGGL(k_bbh_pair<true>, dim3(g), dim3(256), 0, s, rows, ab->ptr, ab->col, ab->num, ab->den,
                           ab->capacity, ba->ptr, ba->col, ba->n_rows, ba->capacity, out->ptr, out->a, out->b, out->num,
                           out->den, out->capacity, st);
        PDP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace pdp
