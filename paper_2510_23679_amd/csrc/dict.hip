// k-mer dictionary build for one or many genomes on gfx950, in one set of launches.
//
// 1. k_mv_local: one work-group per gene encodes every window g[p..p+k-1]
//    into a 5-bit-per-residue code, sorts the codes in LDS and run-length
//    encodes them into the gene's multiplicity vector (Multiplicity vector
//    building phase, Alg. 1: group equal identifiers, count, ascending order).
//    Genes with more than kMvSortCap windows are queued for k_mv_long, which
//    does the same with the codes in global memory.
// 2. A scan of the distinct-k-mer counts of all genes gives the CSR offsets,
//    and k_mv_compact packs the vectors (and notes each entry's gene).
// 3. The inverted index (all entries ordered by k-mer code, ties by gene) is a
//    two-level partition with no global atomics: the leading-residue buckets
//    are grouped into coarse bins of 2^s buckets (s per genome, ~1K entries
//    per bin); k_ix_hist counts bins per block of entries in LDS, a scan gives
//    every (bin, block) its output range, k_ix_place drops the entries there
//    (LDS cursors), and k_ix_sort_bin sorts each bin by (code, gene) in LDS
//    and writes the bin's part of the bucket directory.
// Genes and buckets of all genomes of a call are numbered consecutively; a
// work-group finds its genome by binary search over the per-genome bases.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace pdp {

constexpr uint32_t kMvThreads = 256;
constexpr uint32_t kMvPer = kMvSortCap / kMvThreads;
constexpr uint32_t kDescPerLaunch = 8;

struct DescChunk {
    uint32_t first, count;
    DevBuild d[kDescPerLaunch];
};

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


__global__ void k_build_init(const DevBuild *table, uint32_t n) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    pdp_status *st = table[t].status;
    st->code = 0;
    st->reserved = 0;
    st->needed = 0;
    st->where = ~0ull;
}

__global__ __launch_bounds__(kMvThreads) void k_mv_local(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                         uint32_t *__restrict__ dcnt, uint64_t *__restrict__ long_list,
                                                         uint32_t *__restrict__ counters) {
    __shared__ uint64_t keys[kMvSortCap];
    __shared__ uint8_t sym[kMvSortCap + PDP_K_MAX];
    __shared__ uint32_t tmp[kMvThreads / kWave + 1];
    __shared__ uint32_t s_t;
    const uint32_t G = blockIdx.x;  // global gene
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_t = find_genome_by_gene(table, n_genomes, G);
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t g = G - B.gene_base;
    const uint32_t k = B.k;
    const uint64_t o = B.off[g];
    const uint64_t e = B.off[g + 1];
    if (e < o || e > B.n_residues) {
        if (tid == 0) {
            raise_status(B.status, PDP_E_INVAL, 0, g);
            B.nwin[g] = 0;
            dcnt[G] = 0;
        }
        return;
    }
    const uint64_t len = e - o;
    const uint64_t nw64 = len >= k ? len - k + 1 : 0;
    if (nw64 > PDP_MAX_WINDOWS) {
        if (tid == 0) {
            raise_status(B.status, PDP_E_LIMIT, nw64, g);
            B.nwin[g] = 0;
            dcnt[G] = 0;
        }
        return;
    }
    const uint32_t nw = static_cast<uint32_t>(nw64);
    const bool in_lds = nw <= kMvSortCap;
    const uint8_t *res = B.res;
    for (uint64_t p = tid; p < len; p += kMvThreads) {
        uint32_t s = kSym.v[res[o + p]];
        if (s == kInvalidSym) {
            raise_status(B.status, PDP_E_ALPHABET, 0, o + p);
            s = 0;
        }
        if (in_lds) sym[p] = static_cast<uint8_t>(s);
    }
    if (tid == 0) B.nwin[g] = nw;
    if (!in_lds) {
        if (tid == 0) long_list[atomicAdd(&counters[0], 1u)] = (static_cast<uint64_t>(s_t) << 32) | g;
        return;
    }
    __syncthreads();
    for (uint32_t p = tid; p < nw; p += kMvThreads) {
        uint64_t c = 0;
        for (uint32_t j = 0; j < k; ++j) c = (c << 5) | sym[p + j];
        keys[p] = c;
    }
    __syncthreads();
    wg_network_sort(nw, [&](uint32_t lo, uint32_t hi) {
        const uint64_t a = keys[lo], b = keys[hi];
        if (b < a) {
            keys[lo] = b;
            keys[hi] = a;
        }
    });
    // run-length encoding; each thread owns kMvPer consecutive sorted codes
    const uint32_t i0 = tid * kMvPer;
    uint32_t heads = 0;
#pragma unroll
    for (uint32_t j = 0; j < kMvPer; ++j) {
        const uint32_t i = i0 + j;
        if (i < nw && (i == 0 || keys[i] != keys[i - 1])) ++heads;
    }
    uint32_t total;
    uint32_t rank = block_exclusive_scan<kMvThreads>(heads, tmp, &total);
    uint64_t *slot_code = B.slot_code + o;
    uint32_t *slot_cnt = B.slot_cnt + o;
#pragma unroll
    for (uint32_t j = 0; j < kMvPer; ++j) {
        const uint32_t i = i0 + j;
        if (i < nw && (i == 0 || keys[i] != keys[i - 1])) {
            const uint64_t c = keys[i];
            uint32_t end = i + 1;
            while (end < nw && keys[end] == c) ++end;
            slot_code[rank] = c;
            slot_cnt[rank] = end - i;
            ++rank;
        }
    }
    if (tid == 0) dcnt[G] = total;
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
        for (uint32_t p = tid; p < nw; p += kMvThreads) {
            uint64_t c = 0;
            for (uint32_t j = 0; j < k; ++j) {
                uint32_t s = kSym.v[B.res[o + p + j]];
                c = (c << 5) | (s == kInvalidSym ? 0u : s);
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
        B.mv_code[p + e] = B.slot_code[o + e];
        B.mv_cnt[p + e] = B.slot_cnt[o + e];
        ent_gene[gptr[G] + e] = g;
    }
}

// Per genome: empty CSR of a genome without genes.
__global__ void k_mv_empty(const DevBuild *table, uint32_t n) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && table[t].n_genes == 0) table[t].mv_ptr[0] = 0;
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

// One work-group per block of entries: coarse-bin histogram in LDS, written bin-major.
__global__ __launch_bounds__(256) void k_ix_hist(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                 const uint32_t *__restrict__ gptr, uint32_t *__restrict__ hist) {
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
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x)
        atomicAdd(&h[bucket_of(B.mv_code[e], B.k, B.lead) >> B.hshift], 1u);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < B.nh; i += blockDim.x) hist[B.hist_base + i * B.nblk + j] = h[i];
}

// Same blocks: each entry goes to its bin's range (scanned histogram), position by LDS cursor.
__global__ __launch_bounds__(256) void k_ix_place(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                  const uint32_t *__restrict__ gptr, const uint32_t *__restrict__ off,
                                                  const uint32_t *__restrict__ ent_gene) {
    extern __shared__ uint32_t cur[];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) s_t = find_genome_by_block(table, n_genomes, blockIdx.x);
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t j = blockIdx.x - B.blk_base;
    const uint32_t gbase_off = off[B.hist_base];  // the genome's first entry in the scanned order
    for (uint32_t i = threadIdx.x; i < B.nh; i += blockDim.x) cur[i] = off[B.hist_base + i * B.nblk + j] - gbase_off;
    __syncthreads();
    uint32_t e0, e1, gbase;
    block_range(B, gptr, j, &e0, &e1, &gbase);
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const uint64_t c = B.mv_code[e];
        const uint32_t pos = atomicAdd(&cur[bucket_of(c, B.k, B.lead) >> B.hshift], 1u);
        // one 16-byte record per entry: a single scattered store instead of three
        B.ix_tmp[pos] = make_uint4(static_cast<uint32_t>(c), static_cast<uint32_t>(c >> 32), ent_gene[gbase + e],
                                   B.mv_cnt[e]);
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
            if (bucket_of(code[mid], B.k, B.lead) < b) l = mid + 1;
            else r = mid;
        }
        B.ix_dir[b] = lo + l;
    }
}

// One work-group per coarse bin: its entries sorted by (code, gene), in LDS when they fit
// (else in place in global memory), then the bin's buckets in the directory.
__global__ __launch_bounds__(256) void k_ix_sort_bin(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                     const uint32_t *__restrict__ off) {
    __shared__ uint64_t s_code[kIxBinLds];
    __shared__ uint32_t s_gene[kIxBinLds];
    __shared__ uint32_t s_cnt[kIxBinLds];
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) s_t = find_genome_by_bin(table, n_genomes, blockIdx.x);
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t h = blockIdx.x - B.bin_base;
    const uint32_t base = off[B.hist_base];
    const uint32_t lo = off[B.hist_base + h * B.nblk] - base;
    const uint32_t hi = off[B.hist_base + (h + 1) * B.nblk] - base;  // for the last bin: the next genome's start
    const uint32_t n = hi - lo;
    const uint32_t b0 = h << B.hshift;
    const uint32_t b1 = min(B.nb, (h + 1) << B.hshift);
    if (n <= kIxBinLds) {
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint4 r = B.ix_tmp[lo + i];
            s_code[i] = (static_cast<uint64_t>(r.y) << 32) | r.x;
            s_gene[i] = r.z;
            s_cnt[i] = r.w;
        }
        __syncthreads();
        sort_entries(s_code, s_gene, s_cnt, n);
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            B.ix_code[lo + i] = s_code[i];
            B.ix_gene[lo + i] = s_gene[i];
            B.ix_cnt[lo + i] = s_cnt[i];
        }
        bin_directory(B, s_code, n, lo, b0, b1);
    } else {
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint4 r = B.ix_tmp[lo + i];
            B.ix_code[lo + i] = (static_cast<uint64_t>(r.y) << 32) | r.x;
            B.ix_gene[lo + i] = r.z;
            B.ix_cnt[lo + i] = r.w;
        }
        __syncthreads();
        sort_entries(B.ix_code + lo, B.ix_gene + lo, B.ix_cnt + lo, n);
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

static BuildShape shape_of(const pdp_genome *g, const pdp_dict *const *d, uint32_t n) {
    BuildShape s{};
    s.n_genomes = n;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t cap = g[i].n_residues + 1;
        const uint32_t nb = d[i]->n_buckets;
        const uint32_t sh = bin_shift(nb, cap);
        const uint64_t nh = (uint64_t(nb) + (1ull << sh) - 1) >> sh;
        const uint64_t nblk = (cap + kIxBlock - 1) / kIxBlock;
        s.total_genes += g[i].n_genes;
        s.total_residues += cap;
        s.total_blocks += nblk;
        s.total_bins += nh;
        s.total_hist += nh * nblk;
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
    b += align_up(4 * (s.total_hist + 1), A);           // hist / off
    b += align_up(8 * (s.total_genes + 1), A);          // long_list
    b += align_up(4 * 4, A);                            // counters
    const uint64_t np = std::max<uint64_t>(scan_partials(s.total_genes), scan_partials(s.total_hist));
    b += align_up(4 * np, A);
    return b;
}

BuildShape build_shape(const pdp_genome *g, const pdp_dict *const *d, uint32_t n) { return shape_of(g, d, n); }

BuildShape single_build_shape(uint32_t n_genes, uint64_t n_residues, uint32_t k) {
    pdp_genome g{};
    g.n_genes = n_genes;
    g.n_residues = n_residues;
    pdp_dict d{};
    d.k = k;
    d.n_buckets = n_buckets_for(k);
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
    uint32_t *hist = reinterpret_cast<uint32_t *>(take(4 * (sh.total_hist + 1)));
    uint64_t *long_list = reinterpret_cast<uint64_t *>(take(8 * (sh.total_genes + 1)));
    uint32_t *counters = reinterpret_cast<uint32_t *>(take(4 * 4));
    const uint64_t np = std::max<uint64_t>(scan_partials(sh.total_genes), scan_partials(sh.total_hist));
    uint32_t *partials = reinterpret_cast<uint32_t *>(take(4 * np));

    // descriptors, passed by value to a tiny kernel in chunks
    uint64_t gene_base = 0, res_base = 0, blk_base = 0, bin_base = 0, hist_base = 0;
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
            B.lead = lead_residues(D.k);
            B.hshift = bin_shift(D.n_buckets, cap);
            B.nh = static_cast<uint32_t>((uint64_t(D.n_buckets) + (1ull << B.hshift) - 1) >> B.hshift);
            B.nblk = static_cast<uint32_t>((cap + kIxBlock - 1) / kIxBlock);
            B.gene_base = static_cast<uint32_t>(gene_base);
            B.blk_base = static_cast<uint32_t>(blk_base);
            B.bin_base = static_cast<uint32_t>(bin_base);
            B.hist_base = static_cast<uint32_t>(hist_base);
            B.nwin = D.nwin;
            B.mv_ptr = D.mv_ptr;
            B.mv_code = D.mv_code;
            B.mv_cnt = D.mv_cnt;
            B.ix_dir = D.ix_dir;
            B.ix_code = D.ix_code;
            B.ix_gene = D.ix_gene;
            B.ix_cnt = D.ix_cnt;
            B.status = D.status;
            B.slot_code = slot_code + res_base;
            B.slot_cnt = slot_cnt + res_base;
            B.long_tmp = long_tmp + res_base;
            B.ix_tmp = ix_tmp + res_base;
            gene_base += G.n_genes;
            res_base += cap;
            blk_base += B.nblk;
            bin_base += B.nh;
            hist_base += uint64_t(B.nh) * B.nblk;
        }
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(kDescPerLaunch), 0, s, table, ch);
        PDP_TRY(hipGetLastError());
    }
    const uint32_t tg = static_cast<uint32_t>(sh.total_genes);
    const uint32_t gblocks = (n + 255) / 256;
    const uint32_t hist_lds = static_cast<uint32_t>(4 * sh.max_nh);
    hipLaunchKernelGGL(k_build_init, dim3(gblocks), dim3(256), 0, s, table, n);
    PDP_TRY(hipGetLastError());
    PDP_TRY(launch_fill_u32(counters, 4, 0u, s));
    if (tg > 0) {
        hipLaunchKernelGGL(k_mv_local, dim3(tg), dim3(kMvThreads), 0, s, table, n, dcnt, long_list, counters);
        PDP_TRY(hipGetLastError());
        const uint32_t long_groups = tg < 64 ? tg : 64;
        hipLaunchKernelGGL(k_mv_long, dim3(long_groups), dim3(kMvThreads), 0, s, table, dcnt, long_list, counters);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(launch_scan(dcnt, dcnt, tg, partials, s));  // in place: dcnt becomes the global offsets
    hipLaunchKernelGGL(k_mv_empty, dim3(gblocks), dim3(256), 0, s, table, n);
    PDP_TRY(hipGetLastError());
    if (tg > 0) {
        hipLaunchKernelGGL(k_mv_compact, dim3(tg), dim3(kWave), 0, s, table, n, dcnt, ent_gene);
        PDP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ix_hist, dim3(static_cast<uint32_t>(sh.total_blocks)), dim3(256), hist_lds, s, table, n, dcnt,
                       hist);
    PDP_TRY(hipGetLastError());
    PDP_TRY(launch_scan(hist, hist, sh.total_hist, partials, s));  // in place: every (bin, block) range
    hipLaunchKernelGGL(k_ix_place, dim3(static_cast<uint32_t>(sh.total_blocks)), dim3(256), hist_lds, s, table, n, dcnt,
                       hist, ent_gene);
    PDP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_ix_sort_bin, dim3(static_cast<uint32_t>(sh.total_bins)), dim3(256), 0, s, table, n, hist);
    PDP_TRY(hipGetLastError());
    return hipSuccess;
}

}  // namespace pdp
