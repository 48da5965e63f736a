// k-mer dictionary build for one or many genomes on gfx950, in one set of launches.
//
// 1. k_mv_local: one work-group per gene encodes every window g[p..p+k-1]
//    into a 5-bit-per-residue code, sorts the codes in LDS and run-length
//    encodes them into the gene's multiplicity vector (Multiplicity vector
//    building phase, Alg. 1: group equal identifiers, count, ascending order).
//    Genes with more than kMvSortCap windows are queued for k_mv_long, which
//    does the same with the codes in global memory.
// 2. A scan of the distinct-k-mer counts of all genes gives the CSR offsets,
//    and k_mv_compact packs the vectors while counting index entries per
//    leading-residue bucket.
// 3. A scan of the bucket counts gives every index directory; k_ix_scatter
//    places each (code, gene, count) entry in its bucket and the bucket sorts
//    order each bucket by (code, gene).  The result is each genome's inverted
//    index: all entries ordered by k-mer code, ties by gene.
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

__device__ __forceinline__ uint32_t find_genome_by_bucket(const DevBuild *t, uint32_t n, uint32_t b) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (t[mid].bucket_base <= b) lo = mid;
        else hi = mid - 1;
    }
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

// One wave per gene: CSR offset of the gene, its vector moved into place, bucket sizes counted.
__global__ __launch_bounds__(kWave) void k_mv_compact(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                      const uint32_t *__restrict__ gptr, uint32_t *__restrict__ bcount) {
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
    const uint32_t k = B.k, lead = B.lead;
    for (uint32_t e = threadIdx.x; e < d; e += kWave) {
        const uint64_t c = B.slot_code[o + e];
        B.mv_code[p + e] = c;
        B.mv_cnt[p + e] = B.slot_cnt[o + e];
        atomicAdd(&bcount[B.bucket_base + bucket_of(c, k, lead)], 1u);
    }
}

// Per genome: empty CSR of a genome without genes.
__global__ void k_mv_empty(const DevBuild *table, uint32_t n) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && table[t].n_genes == 0) table[t].mv_ptr[0] = 0;
}

// Every bucket of every genome: its directory entry (offset inside its genome).
__global__ void k_dir_write(const DevBuild *__restrict__ table, uint32_t n_genomes, uint32_t total_buckets,
                            const uint32_t *__restrict__ gdir) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= total_buckets) return;
    const DevBuild &B = table[find_genome_by_bucket(table, n_genomes, b)];
    const uint32_t lb = b - B.bucket_base;
    const uint32_t base = gdir[B.bucket_base];
    B.ix_dir[lb] = gdir[b] - base;
    if (lb + 1 == B.nb) B.ix_dir[lb + 1] = gdir[b + 1] - base;
}

// One wave per gene: drop each entry into its bucket (order inside a bucket is fixed later).
__global__ __launch_bounds__(kWave) void k_ix_scatter(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                      uint32_t *__restrict__ bfill) {
    __shared__ uint32_t s_t;
    const uint32_t G = blockIdx.x;
    if (threadIdx.x == 0) s_t = find_genome_by_gene(table, n_genomes, G);
    __syncthreads();
    const DevBuild &B = table[s_t];
    const uint32_t g = G - B.gene_base;
    const uint32_t p = B.mv_ptr[g];
    const uint32_t d = B.mv_ptr[g + 1] - p;
    const uint32_t k = B.k, lead = B.lead;
    for (uint32_t e = threadIdx.x; e < d; e += kWave) {
        const uint64_t c = B.mv_code[p + e];
        const uint32_t b = bucket_of(c, k, lead);
        const uint32_t pos = B.ix_dir[b] + atomicAdd(&bfill[B.bucket_base + b], 1u);
        B.ix_code[pos] = c;
        B.ix_gene[pos] = g;
        B.ix_cnt[pos] = B.mv_cnt[p + e];
    }
}

__device__ __forceinline__ bool entry_less(uint64_t ca, uint32_t ga, uint64_t cb, uint32_t gb) {
    return ca < cb || (ca == cb && ga < gb);
}

// One thread per bucket: insertion sort of small buckets; large ones are queued.
__global__ __launch_bounds__(256) void k_ix_sort_small(const DevBuild *__restrict__ table, uint32_t n_genomes,
                                                       uint32_t total_buckets, uint64_t *__restrict__ big_list,
                                                       uint32_t *__restrict__ counters) {
    const uint32_t gb = blockIdx.x * blockDim.x + threadIdx.x;
    if (gb >= total_buckets) return;
    const uint32_t t = find_genome_by_bucket(table, n_genomes, gb);
    const DevBuild &B = table[t];
    const uint32_t b = gb - B.bucket_base;
    const uint32_t lo = B.ix_dir[b], hi = B.ix_dir[b + 1];
    const uint32_t n = hi - lo;
    if (n < 2) return;
    if (n > kBucketSmall) {
        big_list[atomicAdd(&counters[1], 1u)] = (static_cast<uint64_t>(t) << 32) | b;
        return;
    }
    uint64_t *code = B.ix_code;
    uint32_t *gene = B.ix_gene, *cnt = B.ix_cnt;
    for (uint32_t i = lo + 1; i < hi; ++i) {
        const uint64_t c = code[i];
        const uint32_t gg = gene[i], m = cnt[i];
        uint32_t j = i;
        while (j > lo && entry_less(c, gg, code[j - 1], gene[j - 1])) {
            code[j] = code[j - 1];
            gene[j] = gene[j - 1];
            cnt[j] = cnt[j - 1];
            --j;
        }
        code[j] = c;
        gene[j] = gg;
        cnt[j] = m;
    }
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

constexpr uint32_t kBigLds = 2048;

// One work-group per large bucket: sorted in LDS when it fits, else in place in global memory.
__global__ __launch_bounds__(256) void k_ix_sort_big(const DevBuild *__restrict__ table, const uint64_t *__restrict__ big_list,
                                                     const uint32_t *__restrict__ counters) {
    __shared__ uint64_t s_code[kBigLds];
    __shared__ uint32_t s_gene[kBigLds];
    __shared__ uint32_t s_cnt[kBigLds];
    const uint32_t n_big = counters[1];
    for (uint32_t bi = blockIdx.x; bi < n_big; bi += gridDim.x) {
        const uint64_t item = big_list[bi];
        const DevBuild &B = table[item >> 32];
        const uint32_t b = static_cast<uint32_t>(item);
        const uint32_t lo = B.ix_dir[b], n = B.ix_dir[b + 1] - lo;
        if (n <= kBigLds) {
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                s_code[i] = B.ix_code[lo + i];
                s_gene[i] = B.ix_gene[lo + i];
                s_cnt[i] = B.ix_cnt[lo + i];
            }
            __syncthreads();
            sort_entries(s_code, s_gene, s_cnt, n);
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                B.ix_code[lo + i] = s_code[i];
                B.ix_gene[lo + i] = s_gene[i];
                B.ix_cnt[lo + i] = s_cnt[i];
            }
        } else {
            sort_entries(B.ix_code + lo, B.ix_gene + lo, B.ix_cnt + lo, n);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host

static BuildShape shape_of(const pdp_genome *g, const pdp_dict *const *d, uint32_t n) {
    BuildShape s{};
    s.n_genomes = n;
    for (uint32_t i = 0; i < n; ++i) {
        s.total_genes += g[i].n_genes;
        s.total_buckets += d[i]->n_buckets;
        s.total_residues += g[i].n_residues + 1;
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
    b += align_up(4 * (s.total_genes + 1), A);          // dcnt / gptr
    b += align_up(4 * (s.total_buckets + 1), A);        // bcount / gdir
    b += align_up(8 * (s.total_genes + 1), A);          // long_list
    b += align_up(8 * (s.total_buckets + 1), A);        // big_list
    b += align_up(4 * 4, A);                            // counters
    const uint64_t np = std::max<uint64_t>(scan_partials(s.total_genes), scan_partials(s.total_buckets));
    b += align_up(4 * np, A);
    return b;
}

BuildShape build_shape(const pdp_genome *g, const pdp_dict *const *d, uint32_t n) { return shape_of(g, d, n); }

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
    uint32_t *dcnt = reinterpret_cast<uint32_t *>(take(4 * (sh.total_genes + 1)));
    uint32_t *bcount = reinterpret_cast<uint32_t *>(take(4 * (sh.total_buckets + 1)));
    uint64_t *long_list = reinterpret_cast<uint64_t *>(take(8 * (sh.total_genes + 1)));
    uint64_t *big_list = reinterpret_cast<uint64_t *>(take(8 * (sh.total_buckets + 1)));
    uint32_t *counters = reinterpret_cast<uint32_t *>(take(4 * 4));
    const uint64_t np = std::max<uint64_t>(scan_partials(sh.total_genes), scan_partials(sh.total_buckets));
    uint32_t *partials = reinterpret_cast<uint32_t *>(take(4 * np));

    // descriptors, passed by value to a tiny kernel in chunks
    uint64_t gene_base = 0, bucket_base = 0, res_base = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += kDescPerLaunch) {
        DescChunk ch{};
        ch.first = c0;
        ch.count = std::min<uint32_t>(kDescPerLaunch, n - c0);
        for (uint32_t j = 0; j < ch.count; ++j) {
            const pdp_genome &G = g[c0 + j];
            const pdp_dict &D = *d[c0 + j];
            DevBuild &B = ch.d[j];
            B.res = G.residues;
            B.off = G.gene_off;
            B.n_residues = G.n_residues;
            B.n_genes = G.n_genes;
            B.k = D.k;
            B.nb = D.n_buckets;
            B.lead = lead_residues(D.k);
            B.gene_base = static_cast<uint32_t>(gene_base);
            B.bucket_base = static_cast<uint32_t>(bucket_base);
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
            gene_base += G.n_genes;
            bucket_base += D.n_buckets;
            res_base += G.n_residues + 1;
        }
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(kDescPerLaunch), 0, s, table, ch);
        PDP_TRY(hipGetLastError());
    }
    const uint32_t tg = static_cast<uint32_t>(sh.total_genes);
    const uint32_t tb = static_cast<uint32_t>(sh.total_buckets);
    const uint32_t gblocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_build_init, dim3(gblocks), dim3(256), 0, s, table, n);
    PDP_TRY(hipGetLastError());
    PDP_TRY(launch_fill_u32(counters, 4, 0u, s));
    PDP_TRY(launch_fill_u32(bcount, uint64_t(tb) + 1, 0u, s));
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
        hipLaunchKernelGGL(k_mv_compact, dim3(tg), dim3(kWave), 0, s, table, n, dcnt, bcount);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(launch_scan(bcount, bcount, tb, partials, s));  // in place: bcount becomes the directories
    hipLaunchKernelGGL(k_dir_write, dim3((tb + 255) / 256), dim3(256), 0, s, table, n, tb, bcount);
    PDP_TRY(hipGetLastError());
    PDP_TRY(launch_fill_u32(bcount, tb, 0u, s));
    if (tg > 0) {
        hipLaunchKernelGGL(k_ix_scatter, dim3(tg), dim3(kWave), 0, s, table, n, bcount);
        PDP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_ix_sort_small, dim3((tb + 255) / 256), dim3(256), 0, s, table, n, tb, big_list, counters);
        PDP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_ix_sort_big, dim3(256), dim3(256), 0, s, table, big_list, counters);
        PDP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace pdp
