// k-mer dictionary build for one or many genomes on gfx950, in one set of launches.
//
// 1. k_mv_wave: one wave per gene encodes every window g[p..p+k-1] into a
//    code of 5 bits per amino acid or 2 per nucleotide (a lane's windows are
//    consecutive, so each code is the previous one shifted by one letter),
//    sorts the codes in registers (a bitonic network of
//    kMvWaveCap keys, eight per lane, lanes exchanging by shuffles) and
//    run-length encodes them into the gene's multiplicity vector (Multiplicity
//    vector building phase, Alg. 1: group equal identifiers, count, ascending
//    order).  Longer genes are queued by size for k_mv_mid (one work-group
//    per gene, 8, 16 or 32 codes per thread sorted in registers, exchanges
//    across waves through LDS) and, past kMvSortCap windows, for k_mv_long
//    (codes sorted in global memory).
// 2. A scan of the distinct-k-mer counts of all genes gives the CSR offsets,
//    and k_mv_compact packs the vectors (and notes each entry's gene).
// 3. The inverted index (all entries ordered by k-mer code, ties by gene) is a
//    two-level partition: the leading-letter buckets are grouped into coarse
//    bins of 2^s buckets (s per genome, ~500 entries per bin); k_ix_hist
//    counts bins per block of entries in LDS and adds them to the bin totals
//    (one global atomic per block and bin), a scan gives every bin its output
//    range, k_ix_place hands each block a run of every bin's range (again one
//    atomic per block and bin) and drops its entries there by LDS rank, and
//    k_ix_sort_bin sorts each bin by (code, gene) in LDS (a counting sort by
//    bucket and the next one or two letters, which leaves about one entry per
//    slot, then a sort inside each slot) and writes the bin's part of the
//    bucket directory.
// Genes and buckets of all genomes of a call are numbered consecutively; a
// work-group finds its genome by binary search over the per-genome bases.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace pdp {

constexpr uint32_t kMvThreads = 256;
static_assert(kMvSortCap == kMvThreads * 32, "the largest k_mv_mid class sorts 32 codes per thread");
constexpr uint32_t kIxBatch = 8;  // index entries a thread loads per round in the histogram and placement
constexpr uint32_t kDescPerLaunch = 16;

struct DescChunk {
    uint32_t first, count;
    DevBuild d[kDescPerLaunch];
};
static_assert(sizeof(DescChunk) <= 4096, "descriptor chunks travel as kernel arguments");

// Copies descriptors passed by value into the workspace table (kernel
// arguments are captured at launch, so the host copy may go away at once).
__global__ void k_put_desc(DevBuild *table, DescChunk c) {
    const uint32_t i = threadIdx.x;
    if (i < c.count) table[c.first + i] = c.d[i];
}

__device__ __forceinline__ uint32_t find_genome_by_gene(const DevBuild *t, uint32_t n, uint32_t gene) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (t[mid].gene_base <= gene) lo = mid;
        else hi = mid - 1;
    }
    // genomes without genes share a base with the next one; take the last with genes
    return lo;
}


// Set-up of a build in one launch: every genome's status cleared and the CSR of a genome
// without genes written (nothing else writes it), the build's counters and the bin totals
// zeroed.
__global__ void k_build_init(const DevBuild *table, uint32_t n, uint32_t *counters, uint32_t *bintot,
                             uint32_t total_bins) {
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    for (uint32_t t = i0; t < n; t += stride) {
        pdp_status *st = table[t].status;
        st->code = 0;
        st->flags = 0;
        st->needed = 0;
        st->where = ~0ull;
        if (table[t].n_genes == 0) table[t].mv_ptr[0] = 0;
    }
    if (i0 < 4) counters[i0] = 0;
    for (uint32_t b = i0; b < total_bins; b += stride) bintot[b] = 0;
}

// Orders LDS writes of a wave before its later LDS reads (a wave runs in lock step,
// so no work-group barrier is needed).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value of x in lane (this lane ^ lj), lj a power of two below kWave, without an LDS
// round trip where the lane pattern allows: DPP moves for 1 and 2 (quad permutations) and 8
// (rotation by 8 inside each row of 16 lanes), ds_swizzle in bit-mask mode (lanes of a half
// wave, no address operand) for 4 and 16, ds_bpermute for 32.  Every lane of the wave must
// be active.
__device__ __forceinline__ uint32_t xor_lanes32(uint32_t x, uint32_t lj) {
    const int v = static_cast<int>(x);
    switch (lj) {
        case 1: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false));
        case 2: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false));
        case 8: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false));
        case 4: return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(v, 0x101F));
        case 16: return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(v, 0x401F));
        default: return __shfl_xor(x, lj, kWave);
    }
}
// 32-bit keys only: with 64-bit keys, and in the work-group sort (whose distance is not a
// compile-time constant), the variants raised register use enough to cost occupancy.
template <typename K>
__device__ __forceinline__ K xor_lanes(K x, uint32_t lj) {
    if constexpr (sizeof(K) == 4) return xor_lanes32(x, lj);
    else return __shfl_xor(x, lj, kWave);
}

// Ascending bitonic sort of kWave * E keys, E per lane in blocked order (lane l holds
// elements l*E .. l*E+E-1): comparators inside a lane swap registers, the others pair
// lanes by a shuffle and keep the minimum or maximum.
template <uint32_t E, typename K>
__device__ __forceinline__ void wave_bitonic_sort(K (&key)[E]) {
    constexpr uint32_t N = kWave * E;
    const uint32_t l = lane_id();
#pragma unroll
    for (uint32_t size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (uint32_t j = size >> 1; j > 0; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (uint32_t e = 0; e < E; ++e) {
                    if (e & j) continue;
                    const bool asc = ((l * E + e) & size) == 0;
                    const K a = key[e], b = key[e | j];
                    const bool sw = asc ? a > b : a < b;
                    key[e] = sw ? b : a;
                    key[e | j] = sw ? a : b;
                }
            } else {
                const uint32_t lj = j / E;
                const bool lower = (l & lj) == 0;
#pragma unroll
                for (uint32_t e = 0; e < E; ++e) {
                    const K o = xor_lanes(key[e], lj);
                    const bool keep_min = lower == (((l * E + e) & size) == 0);
                    const K mn = o < key[e] ? o : key[e], mx = o < key[e] ? key[e] : o;
                    key[e] = keep_min ? mn : mx;
                }
            }
        }
    }
}

// Checks a gene's offsets and window count; on failure records the status and an empty
// vector and returns false.
__device__ __forceinline__ bool gene_ok(const DevBuild &B, uint32_t g, uint32_t G, uint32_t *dcnt, uint64_t *o,
                                        uint64_t *len, uint32_t *nw) {
    *o = B.off[g];
    const uint64_t e = B.off[g + 1];
    if (e < *o || e > B.n_residues) {
        if (lane_id() == 0) {
            raise_status(B.status, PDP_E_INVAL, 0, g);
            B.nwin[g] = 0;
            dcnt[G] = 0;
        }
        return false;
    }
    *len = e - *o;
    const uint64_t nw64 = *len >= B.k ? *len - B.k + 1 : 0;
    if (nw64 > B.max_windows) {
        if (lane_id() == 0) {
            raise_status(B.status, PDP_E_LIMIT, nw64, g);
            B.nwin[g] = 0;
            dcnt[G] = 0;
        }
        return false;
    }
    *nw = static_cast<uint32_t>(nw64);
    return true;
}

// Amino-acid k-mers of 7 letters take 35 bits as 5-bit codes but only 31 as base-20 values
// (20^7 < 2^31), and both order k-mers alike (letter by letter, first letter most
// significant).  For such genomes the multiplicity-vector sorts run on 32-bit base-20 keys, and
// each distinct key is turned back into its 5-bit code when the vector is written.
__device__ __forceinline__ bool base20_keys(const DevBuild &B) { return B.bits == 5u && B.k == 7u; }
constexpr uint32_t kPow20_6 = 64000000u;  // 20^(7-1): the weight of a 7-mer's first letter

__device__ __forceinline__ uint64_t base20_to_code(uint32_t v, uint32_t k) {
    uint64_t c = 0;
    for (uint32_t i = 0; i < k; ++i) {  // digits from the last letter on
        const uint32_t q = v / 20u;
        c |= static_cast<uint64_t>(v - q * 20u) << (5u * i);
        v = q;
    }
    return c;
}

// The keys of windows p0 .. p0+E-1 (those below nw; the rest sort last) from the gene's symbols:
// 5-bit codes, or base-20 values when B20; each window's key is the previous one shifted by one
// letter, so the first k-1 letters are read once.
template <uint32_t E, typename K, bool B20>
__device__ __forceinline__ void window_keys(const uint8_t *sym, uint32_t p0, uint32_t nw, uint32_t k, uint32_t bits,
                                            K (&key)[E]) {
    if constexpr (B20) {
        uint32_t c = 0;  // base-20 value of the k-1 letters after the window's first
        if (p0 < nw)
            for (uint32_t j = 0; j + 1 < k; ++j) c = c * 20u + sym[p0 + j];
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
            const uint32_t p = p0 + e;
            uint32_t full = ~0u;
            if (p < nw) {
                full = c * 20u + sym[p + k - 1];
                c = full - sym[p] * kPow20_6;
            }
            key[e] = static_cast<K>(full);
        }
    } else {
        const uint64_t mask = (1ull << (bits * k)) - 1ull;  // bits * k <= 62
        uint64_t c = 0;
        if (p0 < nw)
            for (uint32_t j = 0; j + 1 < k; ++j) c = (c << bits) | sym[p0 + j];
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
            const uint32_t p = p0 + e;
            if (p < nw) c = ((c << bits) | sym[p + k - 1]) & mask;
            key[e] = p < nw ? static_cast<K>(c) : static_cast<K>(~0ull);  // past the windows: sorts last
        }
    }
}

template <bool B20, typename K>
__device__ __forceinline__ uint64_t key_code(K key, uint32_t k) {
    if constexpr (B20) return base20_to_code(static_cast<uint32_t>(key), k);
    else return static_cast<uint64_t>(key);
}

constexpr uint32_t kMvWaveEMax = 16;
constexpr uint32_t kMvWaveCap = kWave * kMvWaveEMax;  // windows a wave sorts in registers
constexpr uint32_t kMvWaves = kMvThreads / kWave;

// One gene's multiplicity vector by one wave: codes E per lane in registers, sorted by the
// wave's bitonic network (E = 4, 8 or 16: the smallest that holds the gene), then run
// heads ranked by a wave scan; head positions in LDS give the run lengths.  sym holds the
// gene's residue symbols, hp kWave*E+1 slots.
// K: the key type, 32 bits when the codes fit (bits * k <= 32), halving the shuffles.
// B20: base-20 keys (base20_keys).
template <uint32_t E, typename K, bool B20 = false>
__device__ __forceinline__ void mv_wave_gene(const DevBuild &B, const uint8_t *sym, uint16_t *hp, uint64_t o,
                                             uint32_t nw, uint32_t *cnt_out) {
    const uint32_t lane = lane_id();
    const uint32_t k = B.k;
    K key[E];
    // the lane's windows p0 .. p0+E-1 are consecutive
    window_keys<E, K, B20>(sym, lane * E, nw, k, B.bits, key);
    wave_bitonic_sort<E, K>(key);
    const K before = __shfl_up(key[E - 1], 1, kWave);
    uint32_t hmask = 0, nh = 0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
        const uint32_t i = lane * E + e;
        const K prev = e ? key[e - 1] : before;
        const bool h = i < nw && (i == 0 || key[e] != prev);
        hmask |= static_cast<uint32_t>(h) << e;
        nh += h;
    }
    const uint32_t incl = wave_inclusive_sum(nh);
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    uint32_t r = incl - nh;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e)
        if ((hmask >> e) & 1u) hp[r++] = static_cast<uint16_t>(lane * E + e);
    if (lane == 0) hp[total] = static_cast<uint16_t>(nw);
    wave_lds_sync();
    uint64_t *slot_code = B.slot_code + o;
    uint32_t *slot_cnt = B.slot_cnt + o;
    r = incl - nh;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
        if (!((hmask >> e) & 1u)) continue;
        store_global(slot_code + r, key_code<B20>(key[e], k));
        store_global(slot_cnt + r, static_cast<uint32_t>(hp[r + 1]) - hp[r]);
        ++r;
    }
    *cnt_out = total;
}

// Longer genes go to lists by size: counters[0] / long_list past kMvSortCap windows,
// counters[c] / mid_list + (c - 1) * stride for k_mv_mid<8 << (c - 1)>, c = 1, 2, 3.
// NARROW: every genome of the build sorts 32-bit keys (5-bit codes of at most 32 bits, or
// base-20 values): a separate instance without the 64-bit path, which needs fewer registers.
template <bool NARROW>
__global__ __launch_bounds__(kMvThreads) void k_mv_wave(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                        uint32_t total_genes, uint32_t *__restrict__ dcnt,
                                                        uint64_t *__restrict__ mid_list, uint64_t *__restrict__ long_list,
                                                        uint32_t stride, uint32_t *__restrict__ counters) {
    __shared__ uint8_t sym_all[kMvWaves][kMvWaveCap + kKMaxAll];
    __shared__ uint16_t hp_all[kMvWaves][kMvWaveCap + 1];
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t G = blockIdx.x * kMvWaves + w;
    if (G >= total_genes) return;
    const uint32_t t = find_genome_by_gene(table, n_genomes, G);
    const DevBuild &B = table[t];
    const uint32_t g = G - B.gene_base;
    uint64_t o, len;
    uint32_t nw;
    if (!gene_ok(B, g, G, dcnt, &o, &len, &nw)) return;
    if (lane == 0) B.nwin[g] = nw;
    if (nw > kMvWaveCap) {
        if (lane == 0) {
            const uint64_t item = (static_cast<uint64_t>(t) << 32) | g;
            const uint32_t c = nw > kMvSortCap ? 0u : (nw <= kMvThreads * 8 ? 1u : (nw <= kMvThreads * 16 ? 2u : 3u));
            if (c == 0) long_list[atomicAdd(&counters[0], 1u)] = item;
            else mid_list[(c - 1) * stride + atomicAdd(&counters[c], 1u)] = item;
        }
        return;
    }
    uint8_t *sym = sym_all[w];
    // rounds of 4 residues per lane, the 4 loads issued before any is used
    for (uint32_t base = 0; base < len; base += 4 * kWave) {
        uint32_t res[4];
#pragma unroll
        for (uint32_t it = 0; it < 4; ++it) {
            const uint32_t p = base + lane + it * kWave;
            res[it] = p < len ? load_global(B.res + o + p) : 'A';
        }
#pragma unroll
        for (uint32_t it = 0; it < 4; ++it) {
            const uint32_t p = base + lane + it * kWave;
            if (p >= len) continue;
            uint32_t x = sym_in(res[it], B.bits);
            if (x == kInvalidSym) {
                raise_status(B.status, PDP_E_ALPHABET, 0, o + p);
                x = 0;
            }
            sym[p] = static_cast<uint8_t>(x);
        }
    }
    wave_lds_sync();
    uint32_t total;
    if (B.bits * B.k <= 32) {  // uniform per wave
        if (nw <= kWave * 4) mv_wave_gene<4, uint32_t>(B, sym, hp_all[w], o, nw, &total);
        else if (nw <= kWave * 8) mv_wave_gene<8, uint32_t>(B, sym, hp_all[w], o, nw, &total);
        else mv_wave_gene<16, uint32_t>(B, sym, hp_all[w], o, nw, &total);
    } else if (base20_keys(B)) {
        if (nw <= kWave * 4) mv_wave_gene<4, uint32_t, true>(B, sym, hp_all[w], o, nw, &total);
        else if (nw <= kWave * 8) mv_wave_gene<8, uint32_t, true>(B, sym, hp_all[w], o, nw, &total);
        else mv_wave_gene<16, uint32_t, true>(B, sym, hp_all[w], o, nw, &total);
    } else {
        if constexpr (!NARROW) {
            if (nw <= kWave * 4) mv_wave_gene<4, uint64_t>(B, sym, hp_all[w], o, nw, &total);
            else if (nw <= kWave * 8) mv_wave_gene<8, uint64_t>(B, sym, hp_all[w], o, nw, &total);
            else mv_wave_gene<16, uint64_t>(B, sym, hp_all[w], o, nw, &total);
        }
    }
    if (lane == 0) dcnt[G] = total;
}

// Ascending bitonic sort of kMvThreads * E keys by one work-group, E per thread in blocked
// order (thread t holds elements t*E .. t*E+E-1): comparators inside a thread swap
// registers, those inside a wave pair lanes by shuffles, and only those across waves go
// through LDS (xch: kMvThreads * E keys), so a stage costs a barrier only when its stride
// spans waves.  Contains barriers; every thread of the work-group must call it.
template <uint32_t E, typename K>
__device__ __forceinline__ void block_bitonic_sort(K (&key)[E], K *xch) {
    constexpr uint32_t N = kMvThreads * E;
    const uint32_t t = threadIdx.x;
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t j = size >> 1; j >= kWave * E; j >>= 1) {  // partner in another wave
            const uint32_t lj = j / E;
#pragma unroll
            for (uint32_t e = 0; e < E; ++e) xch[e * kMvThreads + t] = key[e];
            __syncthreads();
            const bool lower = (t & lj) == 0;
#pragma unroll
            for (uint32_t e = 0; e < E; ++e) {
                const K o = xch[e * kMvThreads + (t ^ lj)];
                const bool keep_min = lower == (((t * E + e) & size) == 0);
                const K mn = o < key[e] ? o : key[e], mx = o < key[e] ? key[e] : o;
                key[e] = keep_min ? mn : mx;
            }
            __syncthreads();
        }
        for (uint32_t j = min(size >> 1, kWave * E / 2); j >= E; j >>= 1) {  // partner lane in this wave
            const uint32_t lj = j / E;
            const bool lower = (t & lj) == 0;
#pragma unroll
            for (uint32_t e = 0; e < E; ++e) {
                const K o = __shfl_xor(key[e], lj, kWave);
                const bool keep_min = lower == (((t * E + e) & size) == 0);
                const K mn = o < key[e] ? o : key[e], mx = o < key[e] ? key[e] : o;
                key[e] = keep_min ? mn : mx;
            }
        }
#pragma unroll
        for (uint32_t j = E / 2; j > 0; j >>= 1) {  // partner in this thread's registers
            if (j >= size) continue;
#pragma unroll
            for (uint32_t e = 0; e < E; ++e) {
                if (e & j) continue;
                const bool asc = ((t * E + e) & size) == 0;
                const K a = key[e], b = key[e | j];
                const bool sw = asc ? a > b : a < b;
                key[e] = sw ? b : a;
                key[e | j] = sw ? a : b;
            }
        }
    }
}

// Genes queued by k_mv_wave with more windows than a wave sorts, up to kMvThreads * E: one
// work-group per gene.  The gene's symbols go to LDS, every thread encodes E consecutive
// windows (one new letter per window), the work-group sorts the codes in registers, and
// run heads ranked by a work-group scan give the multiplicity vector.  The symbols, the
// sort's exchange area and the head positions share one LDS array.
// One gene of k_mv_mid: len letters at offset o, nw <= kMvThreads * E windows; K as in the wave kernel.
template <uint32_t E, typename K, bool B20 = false>
__device__ __forceinline__ void mid_gene(const DevBuild &B, uint32_t G, uint64_t o, uint32_t len, uint32_t nw,
                                         uint64_t *xch64, K *s_last, uint32_t *tmp, uint32_t *__restrict__ dcnt) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint32_t k = B.k, bits = B.bits;
    uint8_t *sym = reinterpret_cast<uint8_t *>(xch64);
    uint16_t *hp = reinterpret_cast<uint16_t *>(xch64);
    K *xch = reinterpret_cast<K *>(xch64);
    for (uint32_t base = 0; base < len; base += 4 * kMvThreads) {  // 4 loads in flight per thread
        uint32_t res[4];
#pragma unroll
        for (uint32_t it = 0; it < 4; ++it) {
            const uint32_t p = base + it * kMvThreads + tid;
            res[it] = p < len ? load_global(B.res + o + p) : 'A';
        }
#pragma unroll
        for (uint32_t it = 0; it < 4; ++it) {
            const uint32_t p = base + it * kMvThreads + tid;
            if (p >= len) continue;
            uint32_t x = sym_in(res[it], bits);
            if (x == kInvalidSym) {
                raise_status(B.status, PDP_E_ALPHABET, 0, o + p);
                x = 0;
            }
            sym[p] = static_cast<uint8_t>(x);
        }
    }
    __syncthreads();
    K key[E];
    window_keys<E, K, B20>(sym, tid * E, nw, k, bits, key);
    __syncthreads();  // the symbols are read before the sort overwrites them
    block_bitonic_sort<E, K>(key, xch);
    if (lane == kWave - 1) s_last[w] = key[E - 1];
    K before = __shfl_up(key[E - 1], 1, kWave);
    __syncthreads();
    if (lane == 0 && w > 0) before = s_last[w - 1];
    uint32_t hmask = 0, nh = 0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
        const uint32_t i = tid * E + e;
        const K prev = e ? key[e - 1] : before;
        const bool h = i < nw && (i == 0 || key[e] != prev);
        hmask |= static_cast<uint32_t>(h) << e;
        nh += h;
    }
    uint32_t total;
    const uint32_t r0 = block_exclusive_scan<kMvThreads>(nh, tmp, &total);
    uint32_t r = r0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e)
        if ((hmask >> e) & 1u) hp[r++] = static_cast<uint16_t>(tid * E + e);
    if (tid == 0) hp[total] = static_cast<uint16_t>(nw);
    __syncthreads();
    uint64_t *slot_code = B.slot_code + o;
    uint32_t *slot_cnt = B.slot_cnt + o;
    r = r0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
        if (!((hmask >> e) & 1u)) continue;
        store_global(slot_code + r, key_code<B20>(key[e], k));
        store_global(slot_cnt + r, static_cast<uint32_t>(hp[r + 1]) - hp[r]);
        ++r;
    }
    if (tid == 0) dcnt[G] = total;
    __syncthreads();  // LDS takes the next gene
}

template <uint32_t E, bool NARROW>
__global__ __launch_bounds__(kMvThreads) void k_mv_mid(const DevBuild *__restrict__ table, uint32_t *__restrict__ dcnt,
                                                       const uint64_t *__restrict__ list,
                                                       const uint32_t *__restrict__ count) {
    constexpr uint32_t N = kMvThreads * E;
    static_assert(N + kKMaxAll <= 8 * N && N + 1 <= 4 * N && N <= 65535, "symbols and u16 head positions fit");
    __shared__ uint64_t xch[N];
    __shared__ uint64_t s_last[kMvWaves];
    __shared__ uint32_t tmp[kMvWaves + 1];
    const uint32_t n_items = *count;
    for (uint32_t li = blockIdx.x; li < n_items; li += gridDim.x) {
        const uint64_t item = list[li];
        const DevBuild &B = table[item >> 32];
        const uint32_t g = static_cast<uint32_t>(item);
        const uint64_t o = B.off[g];
        const uint32_t len = static_cast<uint32_t>(B.off[g + 1] - o);
        const uint32_t nw = len - B.k + 1;  // k_mv_wave queued this gene for nw <= kMvThreads * E
        if (B.bits * B.k <= 32) {  // uniform per work-group
            mid_gene<E, uint32_t>(B, B.gene_base + g, o, len, nw, xch, reinterpret_cast<uint32_t *>(s_last), tmp, dcnt);
        } else if (base20_keys(B)) {
            mid_gene<E, uint32_t, true>(B, B.gene_base + g, o, len, nw, xch, reinterpret_cast<uint32_t *>(s_last), tmp,
                                        dcnt);
        } else {
            if constexpr (!NARROW) mid_gene<E, uint64_t>(B, B.gene_base + g, o, len, nw, xch, s_last, tmp, dcnt);
        }
    }
}

// Genes with more windows than fit in LDS: same steps, codes sorted in global memory.
__global__ __launch_bounds__(kMvThreads) void k_mv_long(const DevBuild *__restrict__ table, uint32_t *__restrict__ dcnt,
                                                        const uint64_t *__restrict__ long_list,
                                                        const uint32_t *__restrict__ counters) {
    __shared__ uint32_t tmp[kMvThreads / kWave + 1];
    const uint32_t n_long = counters[0];
    const uint32_t tid = threadIdx.x;
    for (uint32_t li = blockIdx.x; li < n_long; li += gridDim.x) {
        const uint64_t item = long_list[li];
        const DevBuild &B = table[item >> 32];
        const uint32_t g = static_cast<uint32_t>(item);
        const uint32_t k = B.k;
        const uint64_t o = B.off[g];
        const uint32_t nw = static_cast<uint32_t>(B.off[g + 1] - o - k + 1);
        uint64_t *w = B.long_tmp + o;
        for (uint64_t p = tid; p < nw + k - 1; p += kMvThreads)
            if (sym_in(B.res[o + p], B.bits) == kInvalidSym) raise_status(B.status, PDP_E_ALPHABET, 0, o + p);
        for (uint32_t p = tid; p < nw; p += kMvThreads) {
            uint64_t c = 0;
            for (uint32_t j = 0; j < k; ++j) {
                uint32_t s = sym_in(B.res[o + p + j], B.bits);
                c = (c << B.bits) | (s == kInvalidSym ? 0u : s);
            }
            w[p] = c;
        }
        __syncthreads();
        wg_network_sort(nw, [&](uint32_t lo, uint32_t hi) {
            const uint64_t a = w[lo], b = w[hi];
            if (b < a) {
                w[lo] = b;
                w[hi] = a;
            }
        });
        uint32_t base = 0;
        for (uint32_t c0 = 0; c0 < nw; c0 += kMvThreads) {
            const uint32_t i = c0 + tid;
            const bool head = i < nw && (i == 0 || w[i] != w[i - 1]);
            uint32_t total;
            const uint32_t r = block_exclusive_scan<kMvThreads>(head ? 1u : 0u, tmp, &total);
            if (head) {
                const uint64_t c = w[i];
                uint32_t end = i + 1;
                while (end < nw && w[end] == c) ++end;
                B.slot_code[o + base + r] = c;
                B.slot_cnt[o + base + r] = end - i;
            }
            base += total;
        }
        if (tid == 0) dcnt[B.gene_base + g] = base;
        __syncthreads();
    }
}

// One wave per gene: CSR offset of the gene, its vector moved into place, and the
// gene of every entry noted for the index.
__global__ __launch_bounds__(kWave) void k_mv_compact(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                      const uint32_t *__restrict__ gptr, uint32_t *__restrict__ ent_gene) {
    __shared__ uint32_t s_t;
    const uint32_t G = blockIdx.x;
    if (threadIdx.x == 0) s_t = find_genome_by_gene(table, n_genomes, G);
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t g = G - B.gene_base;
    const uint64_t o = B.off[g];
    const uint32_t base = gptr[B.gene_base];
    const uint32_t p = gptr[G] - base;
    const uint32_t d = gptr[G + 1] - gptr[G];
    if (threadIdx.x == 0) {
        B.mv_ptr[g] = p;
        if (g + 1 == B.n_genes) B.mv_ptr[g + 1] = p + d;
    }
    for (uint32_t e = threadIdx.x; e < d; e += kWave) {
        store_global(B.mv_code + p + e, load_global(B.slot_code + o + e));
        store_global(B.mv_cnt + p + e, load_global(B.slot_cnt + o + e));
        ent_gene[gptr[G] + e] = g;
    }
}


__device__ __forceinline__ uint32_t find_genome_by_block(const DevBuild *t, uint32_t n, uint32_t blk) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (t[mid].blk_base <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t find_genome_by_bin(const DevBuild *t, uint32_t n, uint32_t bin) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (t[mid].bin_base <= bin) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Entries [j*kIxBlock, ...) of genome t: genome-local range, clipped to the genome's entry count.
__device__ __forceinline__ void block_range(const DevBuild &B, const uint32_t *gptr, uint32_t j, uint32_t *e0,
                                            uint32_t *e1, uint32_t *gbase) {
    const uint32_t base = gptr[B.gene_base];
    const uint32_t E = gptr[B.gene_base + B.n_genes] - base;
    *gbase = base;
    *e0 = min(E, j * kIxBlock);
    *e1 = min(E, (j + 1) * kIxBlock);
}

// One work-group per block of entries: coarse-bin histogram in LDS, added to the genome's
// bin totals with one global atomic per non-empty bin.
__global__ __launch_bounds__(256) void k_ix_hist(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                 const uint32_t *__restrict__ gptr, uint32_t *__restrict__ bintot) {
    extern __shared__ uint32_t h[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) s_t = find_genome_by_block(table, n_genomes, blockIdx.x);
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t j = blockIdx.x - B.blk_base;
    for (uint32_t i = threadIdx.x; i < B.nh; i += blockDim.x) h[i] = 0;
    __syncthreads();
    uint32_t e0, e1, gbase;
    block_range(B, gptr, j, &e0, &e1, &gbase);
    // rounds of kIxBatch entries per thread: the loads of a round are issued before its atomics
    for (uint32_t base = e0; base < e1; base += kIxBatch * 256) {
        uint64_t c[kIxBatch];
#pragma unroll
        for (uint32_t q = 0; q < kIxBatch; ++q) {
            const uint32_t e = base + q * 256 + threadIdx.x;
            c[q] = e < e1 ? load_global(B.mv_code + e) : 0ull;
        }
#pragma unroll
        for (uint32_t q = 0; q < kIxBatch; ++q)
            if (base + q * 256 + threadIdx.x < e1) atomicAdd(&h[bucket_of(c[q], B.k, B.lead, B.bits) >> B.hshift], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < B.nh; i += blockDim.x)
        if (h[i]) atomicAdd(&bintot[B.bin_base + i], h[i]);
}

__device__ __forceinline__ uint64_t rec_code(const uint4 &r) { return (static_cast<uint64_t>(r.y) << 32) | r.x; }
__device__ __forceinline__ uint32_t rec_gene(const uint4 &r) { return r.z; }
__device__ __forceinline__ uint32_t rec_cnt(const uint4 &r) { return r.w; }
__device__ __forceinline__ uint64_t rec_code(const uint2 &r) { return r.x; }
__device__ __forceinline__ uint32_t rec_gene(const uint2 &r) { return r.y & 0xFFFFu; }
__device__ __forceinline__ uint32_t rec_cnt(const uint2 &r) { return r.y >> 16; }
// An index record in the form a bin sort keeps in LDS: uint4 = (code low, code high, gene,
// count), or, when every genome of the build has 32-bit keys (codes of at most 32 bits, or
// base-20 values: base20_keys) and at most 65536 genes, uint2 = (key, gene | count << 16):
// half the LDS, more work-groups per CU.  A base-20 key orders records as the code does.
__device__ __forceinline__ uint32_t code_to_base20(uint64_t c, uint32_t k) {
    uint32_t v = 0;
    for (uint32_t i = 0; i < k; ++i) v = v * 20u + static_cast<uint32_t>((c >> (5u * (k - 1u - i))) & 31u);
    return v;
}
__device__ __forceinline__ void to_rec(const DevBuild &, const uint4 &v, uint4 *r) { *r = v; }
__device__ __forceinline__ void to_rec(const DevBuild &B, const uint4 &v, uint2 *r) {
    const uint32_t key = base20_keys(B) ? code_to_base20((static_cast<uint64_t>(v.y) << 32) | v.x, B.k) : v.x;
    *r = make_uint2(key, v.z | (v.w << 16));
}
// The 5-bit code of a record.
__device__ __forceinline__ uint64_t rec_code5(const DevBuild &, const uint4 &r) { return rec_code(r); }
__device__ __forceinline__ uint64_t rec_code5(const DevBuild &B, const uint2 &r) {
    return base20_keys(B) ? base20_to_code(r.x, B.k) : static_cast<uint64_t>(r.x);
}

constexpr uint32_t kIxPlaceThreads = 1024;  // a placement work-group: its block of entries in registers, 16 per thread
constexpr uint32_t kIxPerThread = kIxBlock / kIxPlaceThreads;  // entries a placement thread keeps
static_assert(kIxPerThread % kIxBatch == 0, "placement rounds divide the entries of a thread");

// Same blocks: each entry goes to its bin's range.  The block counts its entries per bin in
// LDS (every entry's rank among the block's entries of its bin comes back from the LDS
// atomic), takes a run of each bin's range with one global atomic on the bin's remaining
// count (binoff holds the scanned totals; the runs of a bin are handed out from its end),
// and writes each entry at its run start plus its rank, in the record form R the bin sort
// keeps (8 bytes when the build allows it, so the scattered stores and the sort's loads move
// half the bytes).  The order inside a bin depends on scheduling; k_ix_sort_bin sorts every
// bin completely.
template <typename R>
__global__ __launch_bounds__(kIxPlaceThreads) void k_ix_place(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                  const uint32_t *__restrict__ gptr, const uint32_t *__restrict__ binoff,
                                                  uint32_t *__restrict__ bintot, const uint32_t *__restrict__ ent_gene) {
    extern __shared__ uint32_t cur[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) s_t = find_genome_by_block(table, n_genomes, blockIdx.x);
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t j = blockIdx.x - B.blk_base;
    for (uint32_t i = threadIdx.x; i < B.nh; i += blockDim.x) cur[i] = 0;
    __syncthreads();
    uint32_t e0, e1, gbase;
    block_range(B, gptr, j, &e0, &e1, &gbase);
    uint64_t c[kIxPerThread];
    uint32_t rank[kIxPerThread];
#pragma unroll
    for (uint32_t q = 0; q < kIxPerThread; ++q) {
        const uint32_t e = e0 + q * kIxPlaceThreads + threadIdx.x;
        c[q] = e < e1 ? load_global(B.mv_code + e) : 0ull;
    }
#pragma unroll
    for (uint32_t q = 0; q < kIxPerThread; ++q)
        if (e0 + q * kIxPlaceThreads + threadIdx.x < e1) rank[q] = atomicAdd(&cur[bucket_of(c[q], B.k, B.lead, B.bits) >> B.hshift], 1u);
    __syncthreads();
    const uint32_t gstart = binoff[B.bin_base];  // the genome's first entry in the scanned order
    for (uint32_t i = threadIdx.x; i < B.nh; i += blockDim.x) {
        const uint32_t n = cur[i];
        if (n) cur[i] = binoff[B.bin_base + i] - gstart + atomicSub(&bintot[B.bin_base + i], n) - n;
    }
    __syncthreads();
    for (uint32_t q0 = 0; q0 < kIxPerThread; q0 += kIxBatch) {
        uint32_t gn[kIxBatch], ct[kIxBatch];
#pragma unroll
        for (uint32_t q = 0; q < kIxBatch; ++q) {
            const uint32_t e = e0 + (q0 + q) * kIxPlaceThreads + threadIdx.x;
            const bool v = e < e1;
            gn[q] = v ? ent_gene[gbase + e] : 0u;
            ct[q] = v ? load_global(B.mv_cnt + e) : 0u;
        }
#pragma unroll
        for (uint32_t q = 0; q < kIxBatch; ++q) {
            if (e0 + (q0 + q) * kIxPlaceThreads + threadIdx.x >= e1) continue;
            const uint64_t code = c[q0 + q];
            const uint32_t pos = cur[bucket_of(code, B.k, B.lead, B.bits) >> B.hshift] + rank[q0 + q];
            // one record per entry: a single scattered store instead of three
            R r;
            to_rec(B, make_uint4(static_cast<uint32_t>(code), static_cast<uint32_t>(code >> 32), gn[q], ct[q]), &r);
            if constexpr (sizeof(R) == 8)  // as one 64-bit word, through a global (not flat) store
                store_global(reinterpret_cast<uint64_t *>(B.ix_tmp) + pos, (static_cast<uint64_t>(r.y) << 32) | r.x);
            else
                reinterpret_cast<R *>(B.ix_tmp)[pos] = r;
        }
    }
}

__device__ __forceinline__ bool entry_less(uint64_t ca, uint32_t ga, uint64_t cb, uint32_t gb) {
    return ca < cb || (ca == cb && ga < gb);
}

template <typename CP, typename GP>
__device__ void sort_entries(CP code, GP gene, GP cnt, uint32_t n) {
    wg_network_sort(n, [&](uint32_t lo, uint32_t hi) {
        const uint64_t cl = code[lo], ch = code[hi];
        const uint32_t gl = gene[lo], gh = gene[hi];
        if (entry_less(ch, gh, cl, gl)) {
            code[lo] = ch;
            code[hi] = cl;
            gene[lo] = gh;
            gene[hi] = gl;
            const uint32_t t = cnt[lo];
            cnt[lo] = cnt[hi];
            cnt[hi] = t;
        }
    });
}

// Directory entries of buckets [b0, b1) from a bin sorted by code: the first entry of
// each bucket, found by binary search on the bucket of the codes.
template <typename CP>
__device__ void bin_directory(const DevBuild &B, CP code, uint32_t n, uint32_t lo, uint32_t b0, uint32_t b1) {
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
        uint32_t l = 0, r = n;
        while (l < r) {
            const uint32_t mid = (l + r) >> 1;
            if (bucket_of(code[mid], B.k, B.lead, B.bits) < b) l = mid + 1;
            else r = mid;
        }
        B.ix_dir[b] = lo + l;
    }
}

// Packed join key of an index entry: the code's trailing letters (the leading ones are
// the bucket) above the gene.
__device__ __forceinline__ uint32_t entry_key(const DevBuild &B, uint64_t code, uint32_t gene) {
    const uint32_t tb = B.bits * (B.k - B.lead);
    const uint64_t tail = tb ? code & ((1ull << tb) - 1) : 0ull;
    return static_cast<uint32_t>(tail << B.key_shift) | gene;
}

template <typename R>
__device__ __forceinline__ void put_entry(const DevBuild &B, uint32_t pos, const R &v) {
    const uint64_t c = rec_code5(B, v);
    const uint32_t g = rec_gene(v);
    store_global(B.ix_code + pos, c);
    store_global(B.ix_gene + pos, g);
    store_global(B.ix_cnt + pos, rec_cnt(v));
    if (B.key_shift) store_global(B.ix_key + pos, entry_key(B, c, g));
}
template <typename R>
__device__ __forceinline__ bool rec_less(const R &a, const R &b) {
    return entry_less(rec_code(a), rec_gene(a), rec_code(b), rec_gene(b));
}

// Work-group sort of index records (code, gene, count) in LDS by (code, gene).
template <typename R>
__device__ __forceinline__ void sort_recs(R *r, uint32_t n) {
    wg_network_sort(n, [&](uint32_t lo, uint32_t hi) {
        const R a = r[lo], b = r[hi];
        if (rec_less(b, a)) {
            r[lo] = b;
            r[hi] = a;
        }
    });
}

constexpr uint32_t kIxSmallBucket = 16;   // slots up to this size are sorted by one thread
constexpr uint32_t kIxBigList = 64;       // larger slots a bin sorts one by one with the work-group
constexpr uint32_t kIxPer = kIxBinSlots / 256;  // counting-sort slots per thread

// Counting-sort slot of a code inside the bin starting at bucket b0: the bucket, then the
// next xb bits of the code (whole letters), so slots ascend like codes.
__device__ __forceinline__ uint32_t bin_slot(const DevBuild &B, uint64_t code, uint32_t b0) {
    const uint32_t b = bucket_of(code, B.k, B.lead, B.bits) - b0;
    if (!B.xb) return b;
    const uint32_t sh = B.bits * (B.k - B.lead) - B.xb;
    return (b << B.xb) | (static_cast<uint32_t>(code >> sh) & ((1u << B.xb) - 1u));
}
// The same from a record: a base-20 key of a 7-mer gives its bucket (first 4 letters) and next
// letter directly.
__device__ __forceinline__ uint32_t rec_slot(const DevBuild &B, const uint4 &r, uint32_t b0) {
    return bin_slot(B, rec_code(r), b0);
}
__device__ __forceinline__ uint32_t rec_slot(const DevBuild &B, const uint2 &r, uint32_t b0) {
    if (!base20_keys(B)) return bin_slot(B, r.x, b0);
    const uint32_t b = r.x / 8000u - b0;  // 20^3: the last three letters
    return B.xb ? (b << B.xb) | ((r.x / 400u) % 20u) : b;
}

// One work-group per coarse bin: its entries ordered by (code, gene) and the bin's part of
// the bucket directory.  Usual case (the bin fits LDS and its slots fit kIxBinSlots): a
// counting sort by slot (LDS histogram, scan, scatter), whose offsets at the first slot of
// every bucket are the directory, then every slot sorted on its own, by one thread
// (insertion sort) or, if large, by the work-group.  Otherwise the whole bin is sorted in
// LDS, or in place in global memory when it does not fit.
template <typename R>
__global__ __launch_bounds__(256) void k_ix_sort_bin(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                     const uint32_t *__restrict__ off) {
    __shared__ R s_rec[kIxBinLds];
    __shared__ uint32_t s_bstart[kIxBinSlots + 1];
    __shared__ uint32_t s_big[kIxBigList];
    __shared__ uint32_t s_tmp[256 / kWave + 1];
    __shared__ uint32_t s_t, s_nbig;
    if (threadIdx.x == 0) {
        s_t = find_genome_by_bin(table, n_genomes, blockIdx.x);
        s_nbig = 0;
    }
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t h = blockIdx.x - B.bin_base;
    const uint32_t base = off[B.bin_base];
    const uint32_t lo = off[B.bin_base + h] - base;
    const uint32_t hi = off[B.bin_base + h + 1] - base;  // for the last bin: the next genome's start
    const uint32_t n = hi - lo;
    const uint32_t b0 = h << B.hshift;
    const uint32_t b1 = min(B.nb, (h + 1) << B.hshift);
    const uint32_t nbb = b1 - b0;
    const uint32_t nslot = nbb << B.xb;
    const R *tmp = reinterpret_cast<const R *>(B.ix_tmp);  // the placement wrote R records
    if (n <= kIxBinLds && nslot <= kIxBinSlots) {
        for (uint32_t i = threadIdx.x; i <= nslot; i += 256) s_bstart[i] = 0;
        __syncthreads();
        R r[kIxPer];
        uint32_t slot[kIxPer], bk[kIxPer];
#pragma unroll
        for (uint32_t q = 0; q < kIxPer; ++q) {  // every load issued before the first atomic
            const uint32_t i = q * 256 + threadIdx.x;
            if constexpr (sizeof(R) == 8) {  // one 64-bit word, through a global (not flat) load
                const uint64_t w = i < n ? load_global(reinterpret_cast<const uint64_t *>(tmp) + lo + i) : 0ull;
                r[q] = R{static_cast<uint32_t>(w), static_cast<uint32_t>(w >> 32)};
            } else {
                r[q] = i < n ? tmp[lo + i] : R{};
            }
        }
#pragma unroll
        for (uint32_t q = 0; q < kIxPer; ++q) {
            const uint32_t i = q * 256 + threadIdx.x;
            if (i < n) {
                bk[q] = rec_slot(B, r[q], b0);
                slot[q] = atomicAdd(&s_bstart[bk[q]], 1u);
            }
        }
        __syncthreads();
        // exclusive scan of the slot sizes; thread t owns slots [kIxPer*t, kIxPer*t + kIxPer)
        uint32_t c[kIxPer], sum = 0;
#pragma unroll
        for (uint32_t q = 0; q < kIxPer; ++q) {
            const uint32_t b = threadIdx.x * kIxPer + q;
            c[q] = b < nslot ? s_bstart[b] : 0u;
            sum += c[q];
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan<256>(sum, s_tmp, &total);
#pragma unroll
        for (uint32_t q = 0; q < kIxPer; ++q) {
            const uint32_t b = threadIdx.x * kIxPer + q;
            if (b < nslot) s_bstart[b] = run;
            run += c[q];
        }
        if (threadIdx.x == 0) s_bstart[nslot] = n;
        __syncthreads();
#pragma unroll
        for (uint32_t q = 0; q < kIxPer; ++q) {
            const uint32_t i = q * 256 + threadIdx.x;
            if (i < n) s_rec[s_bstart[bk[q]] + slot[q]] = r[q];
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < nbb; b += 256) store_global(B.ix_dir + b0 + b, lo + s_bstart[b << B.xb]);
        for (uint32_t b = threadIdx.x; b < nslot; b += 256) {
            const uint32_t st = s_bstart[b], size = s_bstart[b + 1] - st;
            if (size <= kIxSmallBucket) {
                for (uint32_t x = st + 1; x < st + size; ++x) {
                    const R v = s_rec[x];
                    uint32_t y = x;
                    while (y > st && rec_less(v, s_rec[y - 1])) {
                        s_rec[y] = s_rec[y - 1];
                        --y;
                    }
                    s_rec[y] = v;
                }
            } else {
                const uint32_t idx = atomicAdd(&s_nbig, 1u);
                if (idx < kIxBigList) s_big[idx] = b;
            }
        }
        __syncthreads();
        const uint32_t nbig = s_nbig;
        if (nbig > kIxBigList) {
            sort_recs(s_rec, n);
        } else {
            for (uint32_t j = 0; j < nbig; ++j) {  // uniform loop
                const uint32_t b = s_big[j];
                sort_recs(s_rec + s_bstart[b], s_bstart[b + 1] - s_bstart[b]);
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += 256) put_entry(B, lo + i, s_rec[i]);
    } else if (n <= kIxBinLds) {
        for (uint32_t i = threadIdx.x; i < n; i += 256) s_rec[i] = tmp[lo + i];
        __syncthreads();
        sort_recs(s_rec, n);
        for (uint32_t i = threadIdx.x; i < n; i += 256) put_entry(B, lo + i, s_rec[i]);
        __syncthreads();
        bin_directory(B, B.ix_code + lo, n, lo, b0, b1);
    } else {
        for (uint32_t i = threadIdx.x; i < n; i += 256) {
            const R v = tmp[lo + i];
            B.ix_code[lo + i] = rec_code5(B, v);
            B.ix_gene[lo + i] = rec_gene(v);
            B.ix_cnt[lo + i] = rec_cnt(v);
        }
        __syncthreads();
        sort_entries(B.ix_code + lo, B.ix_gene + lo, B.ix_cnt + lo, n);
        if (B.key_shift)
            for (uint32_t i = threadIdx.x; i < n; i += 256) B.ix_key[lo + i] = entry_key(B, B.ix_code[lo + i], B.ix_gene[lo + i]);
        bin_directory(B, B.ix_code + lo, n, lo, b0, b1);
    }
    if (h + 1 == B.nh && threadIdx.x == 0) B.ix_dir[B.nb] = hi;
}

// ------------------------------------------------------------------ host

// Coarse-bin shift: bins of 2^s buckets holding about kIxBinTarget entries on average.
static uint32_t bin_shift(uint32_t nb, uint64_t cap) {
    uint32_t s = 0;
    while ((uint64_t(nb) >> (s + 1)) > 0 && (cap << (s + 1)) <= uint64_t(nb) * kIxBinTarget) ++s;
    while ((uint64_t(nb) >> s) > kIxMaxBins) ++s;  // keep the LDS histogram bounded
    return s;
}

// Bin shift s and sub-slot bits xb of one genome: a bin's counting sort goes by bucket and,
// where the slots still fit kIxBinSlots, the next letter (amino acids, 5 bits) or two
// (nucleotides, 4 bits), so that a slot holds about one entry.  (Smaller bins to make room
// for the sub-slots cost more in the histogram and placement than they save.)
struct BinPlan {
    uint32_t s, xb;
};
static BinPlan bin_plan(uint32_t nb, uint64_t cap, uint32_t k, uint32_t alphabet) {
    const AlphaSpec a = alpha_spec(alphabet);
    const uint32_t s = bin_shift(nb, cap);
    const uint32_t rest = k - lead_letters(k, alphabet);
    uint32_t xb = a.bits * std::min<uint32_t>(rest, a.bits == 2 ? 2u : 1u);
    while (xb && (1ull << (s + xb)) > kIxBinSlots) xb -= a.bits;
    return {s, xb};
}

static BuildShape shape_of(const pdp_genome *g, const pdp_dict *const *d, uint32_t n) {
    BuildShape s{};
    s.n_genomes = n;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t cap = g[i].n_residues + 1;
        const uint32_t nb = d[i]->n_buckets;
        const uint32_t sh = bin_plan(nb, cap, d[i]->k, d[i]->alphabet).s;
        const uint64_t nh = (uint64_t(nb) + (1ull << sh) - 1) >> sh;
        const uint64_t nblk = (cap + kIxBlock - 1) / kIxBlock;
        s.total_genes += g[i].n_genes;
        s.total_residues += cap;
        s.total_blocks += nblk;
        s.total_bins += nh;
        s.max_nh = std::max<uint64_t>(s.max_nh, nh);
    }
    return s;
}

uint64_t build_ws_bytes(const BuildShape &s) {
    const uint64_t A = 256;
    uint64_t b = 0;
    b += align_up(sizeof(DevBuild) * std::max<uint64_t>(s.n_genomes, 1), A);
    b += align_up(8 * s.total_residues, A);             // slot_code
    b += align_up(4 * s.total_residues, A);             // slot_cnt
    b += align_up(8 * s.total_residues, A);             // long_tmp
    b += align_up(4 * s.total_residues, A);             // ent_gene
    b += align_up(16 * s.total_residues, A);            // ix_tmp
    b += align_up(4 * (s.total_genes + 1), A);          // dcnt / gptr
    b += align_up(4 * (s.total_bins + 1), A);           // bin totals
    b += align_up(4 * (s.total_bins + 1), A);           // scanned bin offsets
    b += align_up(8 * (s.total_genes + 1), A);          // long_list
    b += align_up(3 * 8 * (s.total_genes + 1), A);      // mid_list: three size classes
    b += align_up(4 * 4, A);                            // counters
    const uint64_t np = std::max<uint64_t>(scan_partials(s.total_genes), scan_partials(s.total_bins));
    b += align_up(4 * np, A);
    return b;
}

BuildShape build_shape(const pdp_genome *g, const pdp_dict *const *d, uint32_t n) { return shape_of(g, d, n); }

BuildShape single_build_shape(uint32_t n_genes, uint64_t n_residues, uint32_t k, uint32_t alphabet) {
    pdp_genome g{};
    g.n_genes = n_genes;
    g.n_residues = n_residues;
    pdp_dict d{};
    d.k = k;
    d.alphabet = alphabet;
    d.n_buckets = n_buckets_for(k, alphabet);
    const pdp_dict *dp = &d;
    return shape_of(&g, &dp, 1);
}

hipError_t launch_dict_build_many(const pdp_genome *g, pdp_dict *const *d, uint32_t n, void *ws, hipStream_t s) {
    const BuildShape sh = shape_of(g, d, n);
    const uint64_t A = 256;
    char *p = static_cast<char *>(ws);
    auto take = [&](uint64_t bytes) {
        char *q = p;
        p += align_up(bytes, A);
        return q;
    };
    DevBuild *table = reinterpret_cast<DevBuild *>(take(sizeof(DevBuild) * std::max<uint64_t>(n, 1)));
    uint64_t *slot_code = reinterpret_cast<uint64_t *>(take(8 * sh.total_residues));
    uint32_t *slot_cnt = reinterpret_cast<uint32_t *>(take(4 * sh.total_residues));
    uint64_t *long_tmp = reinterpret_cast<uint64_t *>(take(8 * sh.total_residues));
    uint32_t *ent_gene = reinterpret_cast<uint32_t *>(take(4 * sh.total_residues));
    uint4 *ix_tmp = reinterpret_cast<uint4 *>(take(16 * sh.total_residues));
    uint32_t *dcnt = reinterpret_cast<uint32_t *>(take(4 * (sh.total_genes + 1)));
    uint32_t *bintot = reinterpret_cast<uint32_t *>(take(4 * (sh.total_bins + 1)));
    uint32_t *binoff = reinterpret_cast<uint32_t *>(take(4 * (sh.total_bins + 1)));
    uint64_t *long_list = reinterpret_cast<uint64_t *>(take(8 * (sh.total_genes + 1)));
    uint64_t *mid_list = reinterpret_cast<uint64_t *>(take(3 * 8 * (sh.total_genes + 1)));
    const uint32_t stride = static_cast<uint32_t>(sh.total_genes + 1);
    uint32_t *counters = reinterpret_cast<uint32_t *>(take(4 * 4));
    const uint64_t np = std::max<uint64_t>(scan_partials(sh.total_genes), scan_partials(sh.total_bins));
    uint32_t *partials = reinterpret_cast<uint32_t *>(take(4 * np));

    // descriptors, passed by value to a tiny kernel in chunks
    uint64_t gene_base = 0, res_base = 0, blk_base = 0, bin_base = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += kDescPerLaunch) {
        DescChunk ch{};
        ch.first = c0;
        ch.count = std::min<uint32_t>(kDescPerLaunch, n - c0);
        for (uint32_t j = 0; j < ch.count; ++j) {
            const pdp_genome &G = g[c0 + j];
            const pdp_dict &D = *d[c0 + j];
            DevBuild &B = ch.d[j];
            const uint64_t cap = G.n_residues + 1;
            B.res = G.residues;
            B.off = G.gene_off;
            B.n_residues = G.n_residues;
            B.n_genes = G.n_genes;
            B.k = D.k;
            B.nb = D.n_buckets;
            B.lead = D.lead;
            B.bits = alpha_spec(D.alphabet).bits;
            const BinPlan bp = bin_plan(D.n_buckets, cap, D.k, D.alphabet);
            B.hshift = bp.s;
            B.xb = bp.xb;
            B.nh = static_cast<uint32_t>((uint64_t(D.n_buckets) + (1ull << B.hshift) - 1) >> B.hshift);
            B.nblk = static_cast<uint32_t>((cap + kIxBlock - 1) / kIxBlock);
            B.gene_base = static_cast<uint32_t>(gene_base);
            B.blk_base = static_cast<uint32_t>(blk_base);
            B.bin_base = static_cast<uint32_t>(bin_base);
            B.nwin = D.nwin;
            B.mv_ptr = D.mv_ptr;
            B.mv_code = D.mv_code;
            B.mv_cnt = D.mv_cnt;
            B.ix_dir = D.ix_dir;
            B.ix_code = D.ix_code;
            B.ix_gene = D.ix_gene;
            B.ix_cnt = D.ix_cnt;
            B.ix_key = D.ix_key;
            B.key_shift = D.key_shift;
            B.max_windows = (D.flags & PDP_DICT_LONG_GENES) ? PDP_MAX_WINDOWS_LONG : PDP_MAX_WINDOWS;
            B.status = D.status;
            B.slot_code = slot_code + res_base;
            B.slot_cnt = slot_cnt + res_base;
            B.long_tmp = long_tmp + res_base;
            B.ix_tmp = ix_tmp + res_base;
            gene_base += G.n_genes;
            res_base += cap;
            blk_base += B.nblk;
            bin_base += B.nh;
        }
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(kDescPerLaunch), 0, s, table, ch);
        PDP_TRY(hipGetLastError());
    }
    const uint32_t tg = static_cast<uint32_t>(sh.total_genes);
    const uint32_t hist_lds = static_cast<uint32_t>(4 * sh.max_nh);
    const uint64_t init_items = std::max<uint64_t>(std::max<uint64_t>(n, sh.total_bins), 4);
    hipLaunchKernelGGL(k_build_init, dim3(static_cast<uint32_t>(std::min<uint64_t>((init_items + 255) / 256, 1024))),
                       dim3(256), 0, s, table, n, counters, bintot, static_cast<uint32_t>(sh.total_bins));
    PDP_TRY(hipGetLastError());
    if (tg > 0) {
        bool narrow = true;
        for (uint32_t i = 0; i < n; ++i)
            narrow &= alpha_spec(d[i]->alphabet).bits * d[i]->k <= 32 || (d[i]->alphabet == PDP_ALPHA_AMINO && d[i]->k == 7);
        if (narrow)
            hipLaunchKernelGGL(k_mv_wave<true>, dim3((tg + kMvWaves - 1) / kMvWaves), dim3(kMvThreads), 0, s, table, n,
                               tg, dcnt, mid_list, long_list, stride, counters);
        else
            hipLaunchKernelGGL(k_mv_wave<false>, dim3((tg + kMvWaves - 1) / kMvWaves), dim3(kMvThreads), 0, s, table, n,
                               tg, dcnt, mid_list, long_list, stride, counters);
        PDP_TRY(hipGetLastError());
        // a fixed grid per size class; work-groups past the class's gene count exit at once; the
        // larger classes hold fewer genes and fewer work-groups fit a CU: smaller grids
        const uint32_t mid_groups = tg < 2048 ? tg : 2048;
        if (narrow) {
            hipLaunchKernelGGL((k_mv_mid<8, true>), dim3(mid_groups), dim3(kMvThreads), 0, s, table, dcnt, mid_list,
                               counters + 1);
            PDP_TRY(hipGetLastError());
            hipLaunchKernelGGL((k_mv_mid<16, true>), dim3(std::min(mid_groups, 1024u)), dim3(kMvThreads), 0, s, table,
                               dcnt, mid_list + stride, counters + 2);
            PDP_TRY(hipGetLastError());
            hipLaunchKernelGGL((k_mv_mid<32, true>), dim3(std::min(mid_groups, 512u)), dim3(kMvThreads), 0, s, table,
                               dcnt, mid_list + 2 * stride, counters + 3);
        } else {
            hipLaunchKernelGGL((k_mv_mid<8, false>), dim3(mid_groups), dim3(kMvThreads), 0, s, table, dcnt, mid_list,
                               counters + 1);
            PDP_TRY(hipGetLastError());
            hipLaunchKernelGGL((k_mv_mid<16, false>), dim3(std::min(mid_groups, 1024u)), dim3(kMvThreads), 0, s, table,
                               dcnt, mid_list + stride, counters + 2);
            PDP_TRY(hipGetLastError());
            hipLaunchKernelGGL((k_mv_mid<32, false>), dim3(std::min(mid_groups, 512u)), dim3(kMvThreads), 0, s, table,
                               dcnt, mid_list + 2 * stride, counters + 3);
        }
        PDP_TRY(hipGetLastError());
        const uint32_t long_groups = tg < 64 ? tg : 64;
        hipLaunchKernelGGL(k_mv_long, dim3(long_groups), dim3(kMvThreads), 0, s, table, dcnt, long_list, counters);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(launch_scan(dcnt, dcnt, tg, partials, s));  // in place: dcnt becomes the global offsets
    if (tg > 0) {
        hipLaunchKernelGGL(k_mv_compact, dim3(tg), dim3(kWave), 0, s, table, n, dcnt, ent_gene);
        PDP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ix_hist, dim3(static_cast<uint32_t>(sh.total_blocks)), dim3(256), hist_lds, s, table, n, dcnt,
                       bintot);
    PDP_TRY(hipGetLastError());
    PDP_TRY(launch_scan(bintot, binoff, sh.total_bins, partials, s));  // every bin's range
    // bins placed and sorted as 8-byte records when every key fits 32 bits, every gene index 16
    // bits and every multiplicity 16 bits (no long-gene dictionary)
    bool narrow_rec = true;
    for (uint32_t i = 0; i < n; ++i)
        narrow_rec &= (alpha_spec(d[i]->alphabet).bits * d[i]->k <= 32 || (d[i]->alphabet == PDP_ALPHA_AMINO && d[i]->k == 7)) &&
                      g[i].n_genes <= 65536 && !(d[i]->flags & PDP_DICT_LONG_GENES);
    if (narrow_rec)
        hipLaunchKernelGGL(k_ix_place<uint2>, dim3(static_cast<uint32_t>(sh.total_blocks)), dim3(kIxPlaceThreads), hist_lds,
                           s, table, n, dcnt, binoff, bintot, ent_gene);
    else
        hipLaunchKernelGGL(k_ix_place<uint4>, dim3(static_cast<uint32_t>(sh.total_blocks)), dim3(kIxPlaceThreads), hist_lds,
                           s, table, n, dcnt, binoff, bintot, ent_gene);
    PDP_TRY(hipGetLastError());
    if (narrow_rec)
        hipLaunchKernelGGL(k_ix_sort_bin<uint2>, dim3(static_cast<uint32_t>(sh.total_bins)), dim3(256), 0, s, table, n,
                           binoff);
    else
        hipLaunchKernelGGL(k_ix_sort_bin<uint4>, dim3(static_cast<uint32_t>(sh.total_bins)), dim3(256), 0, s, table, n,
                           binoff);
    PDP_TRY(hipGetLastError());
    return hipSuccess;
}

}  // namespace pdp
