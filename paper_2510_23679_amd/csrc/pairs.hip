// Best hits and bidirectional best hits for many genome pairs on gfx950.
//
// For a genome pair (A, B) the similarity of Eq. jaccard_k needs, for every
// gene pair, m = sum over shared k-mers of min(mult_a, mult_b); the sum of
// maxima over the union is then n_a + n_b - m (max + min = x + y per k-mer).
// The path never forms the |A| x |B| matrix in HBM:
//  1. k_join: both genomes' inverted indexes are sorted by code and split into
//     the same leading-residue bucket ranges; one work-group joins one range
//     (target side staged in LDS) and emits an incidence (a, b, min count) per
//     shared (k-mer, gene a, gene b).  Reads are sequential in both indexes.
//  2. k_inc_bucket: incidences are grouped by accumulation tile (T rows of the
//     query genome) with a counting sort; each pair contributes to the tiles
//     of both directions.
//  3. k_tile: one work-group per tile accumulates m for its T rows against all
//     columns in LDS (two 16-bit sums per 32-bit word), then one wave per row
//     finds the row maximum of J = m/d by exact cross-multiplication and
//     counts or writes every column that reaches it (ties kept, ascending
//     column order; an all-zero row has no best hit), following Eq. best_hit
//     and the per-row work of Alg. 2.
//  4. k_bbh: each best hit (a, b) is kept when a is among b's best hits
//     (Eq. bidirectional_best_hit, the cross-check of Alg. 3).
// Counts, scans and writes keep every output in a canonical order, so results
// do not depend on scheduling.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace pdp {

constexpr uint32_t kJoinThreads = 256;
constexpr uint32_t kBucketGroups = 1024;

// LDS of one join item: the task descriptor, the item's slice of both bucket
// directories, and one sub-range of both sides' codes (the count pass needs no more;
// the write pass also stages the target side's genes and counts).
struct JoinLdsBase {
    DevTask task;
    uint32_t adir[kJoinDirCap + 1];
    uint32_t bdir[kJoinDirCap + 1];
    uint32_t scan[kJoinThreads / kWave + 1];
    uint32_t found;
    uint32_t next;
};
struct JoinLdsCount : JoinLdsBase {
    uint64_t bcode[kJoinLdsCap];
    uint64_t acode[kJoinLdsCap];
};
struct JoinLdsWrite : JoinLdsBase {
    uint64_t bcode[kJoinLdsCap];
    uint64_t acode[kJoinLdsCap];
    uint32_t bgene[kJoinLdsCap];
    uint32_t bcnt[kJoinLdsCap];
};
template <bool WRITE>
using JoinLds = typename std::conditional<WRITE, JoinLdsWrite, JoinLdsCount>::type;

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

// Query entries [a0, a1) of genome a (codes ac, indexed from a0) against the target
// entries of the same bucket range (bc/bg/bn, nbe entries sorted by code): a binary
// search per query entry.  WRITE = false returns the number of incidences; WRITE = true
// writes them from out_base on in a fixed order (blocks of kJoinThreads query entries,
// thread order within a block), so positions need no atomics.  Contains barriers.
template <bool WRITE>
__device__ __forceinline__ uint32_t join_range(const DevTask &T, uint32_t task, uint32_t a0, uint32_t a1,
                                               const uint64_t *ac, const uint64_t *bc, const uint32_t *bg,
                                               const uint32_t *bn, uint32_t nbe, uint4 *inc, uint64_t out_base,
                                               uint64_t inc_cap, uint32_t *scan_tmp) {
    uint32_t done = 0;
    for (uint32_t base = a0; base < a1; base += kJoinThreads) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < a1;
        const uint64_t code = valid ? ac[i - a0] : 0;
        uint32_t lo = 0, hi = valid ? nbe : 0;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (bc[mid] < code) lo = mid + 1;
            else hi = mid;
        }
        uint32_t m = 0;
        if (valid)
            while (lo + m < nbe && bc[lo + m] == code) ++m;
        uint32_t total;
        const uint32_t before = block_exclusive_scan<kJoinThreads>(m, scan_tmp, &total);
        if (WRITE && m) {
            const uint32_t ag = T.a.ix_gene[i], an = T.a.ix_cnt[i];
            const uint64_t slot = out_base + done + before;
            for (uint32_t t = 0; t < m; ++t) {
                if (slot + t < inc_cap) inc[slot + t] = make_uint4(task, ag, bg[lo + t], min(an, bn[lo + t]));
            }
        }
        done += total;
    }
    return done;
}

// One join item: up to T.subs consecutive sub-ranges of T.bpw leading-residue buckets of
// one task.  Pass WRITE = false stores the item's incidence count in chunk_cnt[chunk];
// WRITE = true writes the incidences from the scanned offset chunk_cnt[chunk] on.  The
// task descriptor and the directory slice arrive in one round trip, then each sub-range
// stages both sides in LDS when they fit.  Ends with a barrier so the LDS can take the
// next item.
template <bool WRITE>
__device__ __forceinline__ void join_chunk(uint32_t chunk, const DevTask *__restrict__ tasks, uint32_t n_tasks,
                                           uint32_t *__restrict__ chunk_cnt, uint4 *__restrict__ inc, uint64_t inc_cap,
                                           JoinLds<WRITE> &L) {
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
    for (uint32_t i = threadIdx.x; i <= bh - bl; i += blockDim.x) {
        L.adir[i] = T.a.ix_dir[bl + i];
        L.bdir[i] = T.b.ix_dir[bl + i];
    }
    uint64_t out = WRITE ? chunk_cnt[chunk] : 0;
    __syncthreads();
    uint32_t n = 0;
    for (uint32_t s0 = bl; s0 < bh; s0 += T.bpw) {
        const uint32_t s1 = min(bh, s0 + T.bpw);
        const uint32_t a0 = L.adir[s0 - bl], a1 = L.adir[s1 - bl];
        const uint32_t b0 = L.bdir[s0 - bl], b1 = L.bdir[s1 - bl];
        if (a0 == a1 || b0 == b1) continue;  // uniform across the work-group
        const uint32_t nbe = b1 - b0, nae = a1 - a0;
        uint32_t got;
        if (nbe <= kJoinLdsCap && nae <= kJoinLdsCap) {
            for (uint32_t i = threadIdx.x; i < nbe; i += kJoinThreads) {
                L.bcode[i] = T.b.ix_code[b0 + i];
                if constexpr (WRITE) {
                    L.bgene[i] = T.b.ix_gene[b0 + i];
                    L.bcnt[i] = T.b.ix_cnt[b0 + i];
                }
            }
            for (uint32_t i = threadIdx.x; i < nae; i += kJoinThreads) L.acode[i] = T.a.ix_code[a0 + i];
            __syncthreads();
            if constexpr (WRITE)
                got = join_range<true>(T, task, a0, a1, L.acode, L.bcode, L.bgene, L.bcnt, nbe, inc, out, inc_cap,
                                       L.scan);
            else
                got = join_range<false>(T, task, a0, a1, L.acode, L.bcode, nullptr, nullptr, nbe, inc, out, inc_cap,
                                        L.scan);
        } else {
            got = join_range<WRITE>(T, task, a0, a1, T.a.ix_code + a0, T.b.ix_code + b0, T.b.ix_gene + b0,
                                    T.b.ix_cnt + b0, nbe, inc, out, inc_cap, L.scan);
        }
        n += got;
        out += got;
        __syncthreads();  // the staged arrays take the next sub-range
    }
    if (!WRITE && threadIdx.x == 0) chunk_cnt[chunk] = n;
    __syncthreads();
}

template <bool WRITE>
__global__ __launch_bounds__(kJoinThreads) void k_join(const DevTask *__restrict__ tasks, uint32_t n_tasks,
                                                       uint32_t *__restrict__ chunk_cnt, uint4 *__restrict__ inc,
                                                       uint64_t inc_cap) {
    __shared__ JoinLds<WRITE> L;
    join_chunk<WRITE>(blockIdx.x, tasks, n_tasks, chunk_cnt, inc, inc_cap, L);
}

// Persistent form: a fixed grid claims join items kClaim at a time from a counter
// (one atomic per claim, not per item) until none are left.
constexpr uint32_t kClaim = 8;
constexpr uint32_t kClaimJoin = 2;

template <bool WRITE>
__global__ __launch_bounds__(kJoinThreads) void k_join_persistent(const DevTask *__restrict__ tasks, uint32_t n_tasks,
                                                                  uint32_t total_chunks, uint32_t *__restrict__ chunk_cnt,
                                                                  uint4 *__restrict__ inc, uint64_t inc_cap,
                                                                  uint32_t *__restrict__ next) {
    __shared__ JoinLds<WRITE> L;
    for (;;) {
        if (threadIdx.x == 0) L.next = atomicAdd(next, kClaimJoin);
        __syncthreads();
        const uint32_t first = L.next;
        __syncthreads();
        if (first >= total_chunks) break;
        const uint32_t last = min(total_chunks, first + kClaimJoin);
        for (uint32_t chunk = first; chunk < last; ++chunk)
            join_chunk<WRITE>(chunk, tasks, n_tasks, chunk_cnt, inc, inc_cap, L);
    }
}

template <bool SCATTER>
__global__ __launch_bounds__(256) void k_inc_bucket(const DevTask *__restrict__ tasks, const uint4 *__restrict__ inc,
                                                    const uint32_t *__restrict__ inc_total, uint64_t inc_cap,
                                                    uint32_t *__restrict__ tile_cnt, const uint32_t *__restrict__ tile_off,
                                                    uint32_t *__restrict__ tile_fill, uint2 *__restrict__ recs,
                                                    pdp_status *st) {
    const uint64_t total = *inc_total;
    if (!SCATTER && blockIdx.x == 0 && threadIdx.x == 0 && total > inc_cap) raise_status(st, PDP_E_CAPACITY, total, 0);
    const uint64_t n = total < inc_cap ? total : inc_cap;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint4 r = inc[i];
        const DevTask &T = tasks[r.x];
#pragma unroll
        for (uint32_t d = 0; d < 2; ++d) {
            if (!(T.flags & (1u << d))) continue;
            const uint32_t row = d == 0 ? r.y : r.z;
            const uint32_t col = d == 0 ? r.z : r.y;
            const uint32_t tr = T.tile_rows[d];
            const uint32_t q = row / tr;
            const uint32_t tile = T.tile_base[d] + q;
            if (!SCATTER) {
                atomicAdd(&tile_cnt[tile], 1u);
            } else {
                const uint32_t pos = tile_off[tile] + atomicAdd(&tile_fill[tile], 1u);
                recs[pos] = make_uint2(((row - q * tr) << 24) | col, r.w);
            }
        }
    }
}

__device__ __forceinline__ bool j_greater(uint32_t m1, uint32_t d1, uint32_t m2, uint32_t d2) {
    return static_cast<uint64_t>(m1) * d2 > static_cast<uint64_t>(m2) * d1;
}
__device__ __forceinline__ bool j_equal(uint32_t m1, uint32_t d1, uint32_t m2, uint32_t d2) {
    return static_cast<uint64_t>(m1) * d2 == static_cast<uint64_t>(m2) * d1;
}

// One accumulation tile: T rows of one direction of one task against every
// column of the other genome.  LDS holds the sums of minima (two 16-bit sums
// per 32-bit word) and a bitmap with one bit per word that has been touched,
// so a row's maximum and ties cost time in proportion to its touched columns.
// One wave per row: pass 1 finds the exact maximum of m/d (64-bit
// cross-multiplication); pass 2 emits every column at the maximum in
// ascending order (lanes own ascending, disjoint column ranges; a wave prefix
// sum gives positions).  In the first launch (WRITE = false) the ties go to a
// per-row slab of kSlab entries and the row's count to cnt[row]; a row with
// more ties marks its tile, and the second launch (WRITE = true) recomputes
// only the marked tiles and writes their rows straight into the CSR output.
template <bool WRITE>
__device__ __forceinline__ void tile_process(uint32_t tile_id, const DevTask *__restrict__ tasks,
                                             const DevTile *__restrict__ tiles, const uint32_t *__restrict__ tile_off,
                                             const uint2 *__restrict__ recs, uint32_t *__restrict__ bh_ptr,
                                             uint4 *__restrict__ slab, uint32_t *__restrict__ bh_col,
                                             uint32_t *__restrict__ bh_num, uint32_t *__restrict__ bh_den,
                                             uint64_t bh_cap, uint32_t *overflow_tiles, uint32_t *overflow_count,
                                             uint32_t *lds, uint32_t *s_flag) {
    const DevTile tl = tiles[tile_id];
    const DevTask &T = tasks[tl.task];
    const DevDict &R = tl.dir == 0 ? T.a : T.b;
    const DevDict &C = tl.dir == 0 ? T.b : T.a;
    const uint32_t ncols = C.n_genes;
    const uint32_t W = (ncols + 1) >> 1;   // accumulator words per row
    const uint32_t WB = (W + 31) >> 5;     // bitmap words per row
    uint32_t *acc = lds;
    uint32_t *bits = lds + tl.nrows * W;
    const uint32_t words = tl.nrows * (W + WB);
    uint4 *lds4 = reinterpret_cast<uint4 *>(lds);
    for (uint32_t i = threadIdx.x; i < (words + 3) / 4; i += kTileThreads) lds4[i] = make_uint4(0, 0, 0, 0);
    // window counts of the column genome, 16 bits each (at most PDP_MAX_WINDOWS)
    uint16_t *cw = reinterpret_cast<uint16_t *>(lds + ((words + 3) & ~3u));
    for (uint32_t c = threadIdx.x; c < ncols; c += kTileThreads) cw[c] = static_cast<uint16_t>(C.nwin[c]);
    if (threadIdx.x == 0) *s_flag = 0;
    __syncthreads();
    const uint32_t r0 = tile_off[tile_id], r1 = tile_off[tile_id + 1];
    for (uint32_t i = r0 + threadIdx.x; i < r1; i += kTileThreads) {
        const uint2 r = recs[i];
        const uint32_t rl = r.x >> 24, c = r.x & 0xFFFFFFu, w = c >> 1;
        const uint32_t old = atomicAdd(&acc[rl * W + w], r.y << ((c & 1u) << 4));
        if (old == 0) atomicOr(&bits[rl * WB + (w >> 5)], 1u << (w & 31u));
    }
    __syncthreads();
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    for (uint32_t rl = wave; rl < tl.nrows; rl += kTileThreads / kWave) {
        const uint32_t row = tl.row0 + rl;
        const uint32_t grow = T.row_base[tl.dir] + row;
        const uint32_t nr = R.nwin[row];
        const uint32_t *arow = acc + rl * W;
        const uint32_t *brow = bits + rl * WB;
        uint32_t bm = 0, bd = 1;
        for (uint32_t bw = lane; bw < WB; bw += kWave) {
            uint32_t m = brow[bw];
            while (m) {
                const uint32_t w = (bw << 5) + (__ffs(m) - 1);
                m &= m - 1;
                const uint32_t v = arow[w];
                const uint32_t m0 = v & 0xFFFFu, m1 = v >> 16;
                if (m0) {
                    const uint32_t d = nr + cw[2 * w] - m0;
                    if (j_greater(m0, d, bm, bd)) { bm = m0; bd = d; }
                }
                if (m1) {
                    const uint32_t d = nr + cw[2 * w + 1] - m1;
                    if (j_greater(m1, d, bm, bd)) { bm = m1; bd = d; }
                }
            }
        }
#pragma unroll
        for (uint32_t o = kWave / 2; o > 0; o >>= 1) {
            const uint32_t om = __shfl_xor(bm, o, kWave), od = __shfl_xor(bd, o, kWave);
            if (j_greater(om, od, bm, bd)) { bm = om; bd = od; }
        }
        uint32_t pos = WRITE ? bh_ptr[grow] : 0u;
        if (bm) {
            for (uint32_t b0 = 0; b0 < WB; b0 += kWave) {
                const uint32_t bw = b0 + lane;
                const uint32_t mask = bw < WB ? brow[bw] : 0u;
                uint32_t cnt = 0;
                for (uint32_t m = mask; m;) {
                    const uint32_t w = (bw << 5) + (__ffs(m) - 1);
                    m &= m - 1;
                    const uint32_t v = arow[w];
                    const uint32_t m0 = v & 0xFFFFu, m1 = v >> 16;
                    if (m0 && j_equal(m0, nr + cw[2 * w] - m0, bm, bd)) ++cnt;
                    if (m1 && j_equal(m1, nr + cw[2 * w + 1] - m1, bm, bd)) ++cnt;
                }
                const uint32_t incl = wave_inclusive_sum(cnt);
                const uint32_t total = __shfl(incl, kWave - 1, kWave);
                uint32_t p = pos + incl - cnt;
                for (uint32_t m = cnt ? mask : 0u; m;) {
                    const uint32_t w = (bw << 5) + (__ffs(m) - 1);
                    m &= m - 1;
                    const uint32_t v = arow[w];
#pragma unroll
                    for (uint32_t h = 0; h < 2; ++h) {
                        const uint32_t mm = h ? v >> 16 : v & 0xFFFFu;
                        if (!mm) continue;
                        const uint32_t c = 2 * w + h;
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
            if (pos > kSlab) *s_flag = 1;
        }
    }
    __syncthreads();
    if (!WRITE && threadIdx.x == 0 && *s_flag) overflow_tiles[atomicAdd(overflow_count, 1u)] = tile_id;
    __syncthreads();
}

__global__ __launch_bounds__(kTileThreads) void k_tile_count(const DevTask *__restrict__ tasks,
                                                             const DevTile *__restrict__ tiles,
                                                             const uint32_t *__restrict__ tile_off,
                                                             const uint2 *__restrict__ recs, uint32_t *__restrict__ bh_ptr,
                                                             uint4 *__restrict__ slab, uint32_t *overflow_tiles,
                                                             uint32_t *overflow_count) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_flag;
    tile_process<false>(blockIdx.x, tasks, tiles, tile_off, recs, bh_ptr, slab, nullptr, nullptr, nullptr, 0,
                        overflow_tiles, overflow_count, lds, &s_flag);
}

// Persistent form: a fixed grid pulls tiles from a counter until none are left.
__global__ __launch_bounds__(kTileThreads) void k_tile_count_persistent(
    const DevTask *__restrict__ tasks, const DevTile *__restrict__ tiles, uint32_t total_tiles,
    const uint32_t *__restrict__ tile_off, const uint2 *__restrict__ recs, uint32_t *__restrict__ bh_ptr,
    uint4 *__restrict__ slab, uint32_t *overflow_tiles, uint32_t *overflow_count, uint32_t *__restrict__ next) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_flag, s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(next, kClaim);
        __syncthreads();
        const uint32_t first = s_next;
        __syncthreads();
        if (first >= total_tiles) break;
        const uint32_t last = min(total_tiles, first + kClaim);
        for (uint32_t t = first; t < last; ++t)
            tile_process<false>(t, tasks, tiles, tile_off, recs, bh_ptr, slab, nullptr, nullptr, nullptr, 0,
                                overflow_tiles, overflow_count, lds, &s_flag);
    }
}

// Rows with more ties than the slab holds: their tiles again, written to the CSR output.
__global__ __launch_bounds__(kTileThreads) void k_tile_write(const DevTask *__restrict__ tasks,
                                                             const DevTile *__restrict__ tiles,
                                                             const uint32_t *__restrict__ tile_off,
                                                             const uint2 *__restrict__ recs, uint32_t *__restrict__ bh_ptr,
                                                             uint32_t *__restrict__ bh_col, uint32_t *__restrict__ bh_num,
                                                             uint32_t *__restrict__ bh_den, uint64_t bh_cap,
                                                             const uint32_t *__restrict__ overflow_tiles,
                                                             const uint32_t *__restrict__ overflow_count) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_flag;
    const uint32_t n = *overflow_count;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x)
        tile_process<true>(overflow_tiles[i], tasks, tiles, tile_off, recs, bh_ptr, nullptr, bh_col, bh_num, bh_den,
                           bh_cap, nullptr, nullptr, lds, &s_flag);
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
    for (uint32_t i = 0; i < n; ++i) {
        if (p + i >= bh_cap) break;
        const uint4 e = slab[static_cast<uint64_t>(r) * kSlab + i];
        bh_col[p + i] = e.x;
        bh_num[p + i] = e.y;
        bh_den[p + i] = e.z;
    }
}

// BBH of one row: keep each best hit (a, b) whose reverse row contains a.
template <bool WRITE>
__device__ __forceinline__ void bbh_row(uint32_t a, uint32_t grow, uint32_t rab, uint32_t ba_base, const uint32_t *ab_ptr,
                                        const uint32_t *ab_col, const uint32_t *ab_num, const uint32_t *ab_den,
                                        const uint32_t *ba_ptr, const uint32_t *ba_col, uint32_t *out_ptr, uint32_t *out_a,
                                        uint32_t *out_b, uint32_t *out_num, uint32_t *out_den, uint64_t cap) {
    uint32_t pos = WRITE ? out_ptr[grow] : 0u;
    for (uint32_t p = ab_ptr[rab]; p < ab_ptr[rab + 1]; ++p) {
        const uint32_t b = ab_col[p];
        const uint32_t rba = ba_base + b;
        bool found = false;
        for (uint32_t q = ba_ptr[rba]; q < ba_ptr[rba + 1]; ++q) {
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

template <bool WRITE>
__global__ __launch_bounds__(256) void k_bbh(const DevTask *__restrict__ tasks, const uint32_t *__restrict__ order,
                                             uint32_t n_tasks, uint32_t bbh_rows,
                                             const uint32_t *__restrict__ bh_ptr, const uint32_t *__restrict__ bh_col,
                                             const uint32_t *__restrict__ bh_num, const uint32_t *__restrict__ bh_den,
                                             uint32_t *__restrict__ out_ptr, uint32_t *__restrict__ out_a,
                                             uint32_t *__restrict__ out_b, uint32_t *__restrict__ out_num,
                                             uint32_t *__restrict__ out_den, uint64_t cap, pdp_status *st) {
    const uint32_t grow = blockIdx.x * blockDim.x + threadIdx.x;
    if (WRITE && grow == 0 && out_ptr[bbh_rows] > cap) raise_status(st, PDP_E_CAPACITY, out_ptr[bbh_rows], 2);
    if (grow >= bbh_rows) return;
    const DevTask &T = tasks[find_bbh_task(tasks, order, n_tasks, grow)];
    const uint32_t a = grow - T.bbh_row_base;
    bbh_row<WRITE>(a, grow, T.row_base[0] + a, T.row_base[1], bh_ptr, bh_col, bh_num, bh_den, bh_ptr, bh_col, out_ptr,
                   out_a, out_b, out_num, out_den, cap);
}

template <bool WRITE>
__global__ __launch_bounds__(256) void k_bbh_pair(uint32_t rows, const uint32_t *__restrict__ ab_ptr,
                                                  const uint32_t *__restrict__ ab_col, const uint32_t *__restrict__ ab_num,
                                                  const uint32_t *__restrict__ ab_den, const uint32_t *__restrict__ ba_ptr,
                                                  const uint32_t *__restrict__ ba_col, uint32_t ba_rows,
                                                  uint32_t *__restrict__ out_ptr, uint32_t *__restrict__ out_a,
                                                  uint32_t *__restrict__ out_b, uint32_t *__restrict__ out_num,
                                                  uint32_t *__restrict__ out_den, uint64_t cap, pdp_status *st) {
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (WRITE && a == 0 && out_ptr[rows] > cap) raise_status(st, PDP_E_CAPACITY, out_ptr[rows], 2);
    if (a >= rows) return;
    // a column index past the reverse output's rows cannot name a best hit there
    for (uint32_t p = ab_ptr[a]; p < ab_ptr[a + 1]; ++p) {
        if (ab_col[p] >= ba_rows) {
            raise_status(st, PDP_E_INVAL, 0, a);
            if (!WRITE) out_ptr[a] = 0;
            return;
        }
    }
    bbh_row<WRITE>(a, a, a, 0, ab_ptr, ab_col, ab_num, ab_den, ba_ptr, ba_col, out_ptr, out_a, out_b, out_num, out_den, cap);
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

uint32_t persistent_tile_grid(uint32_t tile_lds) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tile_count_persistent, kTileThreads, tile_lds) != hipSuccess ||
        per < 1)
        per = 1;
    return device_cus() * static_cast<uint32_t>(per);
}

// Tiles above 64 KiB of dynamic LDS need the kernels' limit raised (gfx950 has 160 KiB per work-group).
hipError_t allow_tile_lds(uint32_t tile_lds) {
    if (tile_lds <= 64 * 1024) return hipSuccess;
    const int v = static_cast<int>(tile_lds);
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_count), hipFuncAttributeMaxDynamicSharedMemorySize, v));
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_count_persistent),
                                hipFuncAttributeMaxDynamicSharedMemorySize, v));
    PDP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_write), hipFuncAttributeMaxDynamicSharedMemorySize, v));
    return hipSuccess;
}

uint64_t pair_ws_bytes(const PlanShape &p) {
    const uint64_t A = 256;
    uint64_t s = 0;
    s += align_up(sizeof(DevTask) * std::max<uint64_t>(p.n_tasks, 1), A);
    s += align_up(sizeof(DevTile) * std::max<uint64_t>(p.total_tiles, 1), A);
    s += align_up(4 * std::max<uint64_t>(p.n_tasks, 1), A);
    s += align_up(16 * std::max<uint64_t>(p.inc_cap, 1), A);
    s += align_up(32, A);
    s += align_up(4 * (uint64_t(p.total_chunks) + 1), A);
    s += align_up(4 * (uint64_t(p.total_tiles) + 1), A);
    s += align_up(4 * (uint64_t(p.total_tiles) + 1), A);
    s += align_up(8 * 2 * std::max<uint64_t>(p.inc_cap, 1), A);
    s += align_up(16 * kSlab * (uint64_t(p.bh_rows) + 1), A);
    s += align_up(4 * (uint64_t(p.total_tiles) + 1), A);
    const uint64_t np = std::max({scan_partials(p.total_tiles), scan_partials(p.bh_rows), scan_partials(p.bbh_rows),
                                  scan_partials(p.total_chunks)});
    s += align_up(4 * np, A);
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
    w.order = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(p.n_tasks, 1)));
    w.inc = reinterpret_cast<uint4 *>(take(16 * std::max<uint64_t>(p.inc_cap, 1)));
    w.counters = reinterpret_cast<unsigned long long *>(take(32));
    w.overflow_count = reinterpret_cast<uint32_t *>(w.counters) + 2;
    w.next_join = reinterpret_cast<uint32_t *>(w.counters) + 3;
    w.next_tile = reinterpret_cast<uint32_t *>(w.counters) + 4;
    w.next_join_write = reinterpret_cast<uint32_t *>(w.counters) + 5;
    w.chunk_cnt = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_chunks) + 1)));
    w.tile_cnt = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_tiles) + 1)));
    w.tile_fill = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_tiles) + 1)));
    w.recs = reinterpret_cast<uint2 *>(take(8 * 2 * std::max<uint64_t>(p.inc_cap, 1)));
    w.slab = reinterpret_cast<uint4 *>(take(16 * kSlab * (uint64_t(p.bh_rows) + 1)));
    w.overflow_tiles = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(p.total_tiles) + 1)));
    const uint64_t np = std::max({scan_partials(p.total_tiles), scan_partials(p.bh_rows), scan_partials(p.bbh_rows),
                                  scan_partials(p.total_chunks)});
    w.partials = reinterpret_cast<uint32_t *>(take(4 * np));
    return w;
}

hipError_t launch_pairs(const PlanShape &p, const PairWs &w, pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *st,
                        hipStream_t s, const KernelTimer *timer) {
    auto mark = [&](int32_t kernel, bool begin) -> hipError_t {
        if (!timer || timer->kernel != kernel) return hipSuccess;
        return hipEventRecord(begin ? timer->start : timer->stop, s);
    };
    PDP_TRY(mark(PDP_KERNEL_ALL, true));
    PDP_TRY(launch_status_init(st, s));
    // counters: (unused), overflow tiles, next join item (count pass), next tile, next join item (write pass)
    PDP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(w.counters), 8, 0u, s));
    PDP_TRY(launch_fill_u32(w.tile_cnt, uint64_t(p.total_tiles) + 1, 0u, s));
    PDP_TRY(launch_fill_u32(w.tile_fill, uint64_t(p.total_tiles) + 1, 0u, s));
    const uint32_t *inc_total = w.chunk_cnt + p.total_chunks;  // after the scan: all incidences
    PDP_TRY(mark(PDP_KERNEL_JOIN, true));
    if (p.total_chunks && p.join_grid) {
        const dim3 g(std::min(p.join_grid, (p.total_chunks + kClaimJoin - 1) / kClaimJoin));
        hipLaunchKernelGGL(k_join_persistent<false>, g, dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, p.total_chunks,
                           w.chunk_cnt, w.inc, p.inc_cap, w.next_join);
        PDP_TRY(hipGetLastError());
        PDP_TRY(launch_scan(w.chunk_cnt, w.chunk_cnt, p.total_chunks, w.partials, s));
        hipLaunchKernelGGL(k_join_persistent<true>, g, dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, p.total_chunks,
                           w.chunk_cnt, w.inc, p.inc_cap, w.next_join_write);
        PDP_TRY(hipGetLastError());
    } else if (p.total_chunks) {
        hipLaunchKernelGGL(k_join<false>, dim3(p.total_chunks), dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, w.chunk_cnt,
                           w.inc, p.inc_cap);
        PDP_TRY(hipGetLastError());
        PDP_TRY(launch_scan(w.chunk_cnt, w.chunk_cnt, p.total_chunks, w.partials, s));
        hipLaunchKernelGGL(k_join<true>, dim3(p.total_chunks), dim3(kJoinThreads), 0, s, w.tasks, p.n_tasks, w.chunk_cnt,
                           w.inc, p.inc_cap);
        PDP_TRY(hipGetLastError());
    } else {
        PDP_TRY(launch_fill_u32(w.chunk_cnt, 1, 0u, s));
    }
    PDP_TRY(mark(PDP_KERNEL_JOIN, false));
    PDP_TRY(mark(PDP_KERNEL_BUCKET, true));
    hipLaunchKernelGGL(k_inc_bucket<false>, dim3(kBucketGroups), dim3(256), 0, s, w.tasks, w.inc, inc_total, p.inc_cap,
                       w.tile_cnt, w.tile_cnt, w.tile_fill, w.recs, st);
    PDP_TRY(hipGetLastError());
    PDP_TRY(launch_scan(w.tile_cnt, w.tile_cnt, p.total_tiles, w.partials, s));
    hipLaunchKernelGGL(k_inc_bucket<true>, dim3(kBucketGroups), dim3(256), 0, s, w.tasks, w.inc, inc_total, p.inc_cap,
                       w.tile_cnt, w.tile_cnt, w.tile_fill, w.recs, st);
    PDP_TRY(hipGetLastError());
    PDP_TRY(mark(PDP_KERNEL_BUCKET, false));
    PDP_TRY(mark(PDP_KERNEL_TILE_COUNT, true));
    if (p.total_tiles && p.tile_grid) {
        hipLaunchKernelGGL(k_tile_count_persistent, dim3(std::min(p.tile_grid, (p.total_tiles + kClaim - 1) / kClaim)),
                           dim3(kTileThreads),
                           p.tile_lds, s, w.tasks, w.tiles, p.total_tiles, w.tile_cnt, w.recs, bh->ptr, w.slab,
                           w.overflow_tiles, w.overflow_count, w.next_tile);
        PDP_TRY(hipGetLastError());
    } else if (p.total_tiles) {
        hipLaunchKernelGGL(k_tile_count, dim3(p.total_tiles), dim3(kTileThreads), p.tile_lds, s, w.tasks, w.tiles,
                           w.tile_cnt, w.recs, bh->ptr, w.slab, w.overflow_tiles, w.overflow_count);
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
        hipLaunchKernelGGL(k_tile_write, dim3(g), dim3(kTileThreads), p.tile_lds, s, w.tasks, w.tiles, w.tile_cnt,
                           w.recs, bh->ptr, bh->col, bh->num, bh->den, bh->capacity, w.overflow_tiles,
                           w.overflow_count);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(mark(PDP_KERNEL_TILE_WRITE, false));
    PDP_TRY(mark(PDP_KERNEL_BBH, true));
    if (p.bbh_rows && bbh) {
        const uint32_t g = (p.bbh_rows + 255) / 256;
        hipLaunchKernelGGL(k_bbh<false>, dim3(g), dim3(256), 0, s, w.tasks, w.order, p.n_tasks, p.bbh_rows, bh->ptr, bh->col,
                           bh->num, bh->den, bbh->ptr, bbh->a, bbh->b, bbh->num, bbh->den, bbh->capacity, st);
        PDP_TRY(hipGetLastError());
        PDP_TRY(launch_scan(bbh->ptr, bbh->ptr, p.bbh_rows, w.partials, s));
        hipLaunchKernelGGL(k_bbh<true>, dim3(g), dim3(256), 0, s, w.tasks, w.order, p.n_tasks, p.bbh_rows, bh->ptr, bh->col,
                           bh->num, bh->den, bbh->ptr, bbh->a, bbh->b, bbh->num, bbh->den, bbh->capacity, st);
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
        hipLaunchKernelGGL(k_bbh_pair<false>, dim3(g), dim3(256), 0, s, rows, ab->ptr, ab->col, ab->num, ab->den, ba->ptr,
                           ba->col, ba->n_rows, out->ptr, out->a, out->b, out->num, out->den, out->capacity, st);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(launch_scan(out->ptr, out->ptr, rows, partials, s));
    if (rows) {
        const uint32_t g = (rows + 255) / 256;
        hipLaunchKernelGGL(k_bbh_pair<true>, dim3(g), dim3(256), 0, s, rows, ab->ptr, ab->col, ab->num, ab->den, ba->ptr,
                           ba->col, ba->n_rows, out->ptr, out->a, out->b, out->num, out->den, out->capacity, st);
        PDP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace pdp
