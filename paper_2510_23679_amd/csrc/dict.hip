// k-mer dictionary build for one genome on gfx950.
//
// 1. k_mv_local: one work-group per gene encodes every window g[p..p+k-1]
//    into a 5-bit-per-residue code, sorts the codes in LDS and run-length
//    encodes them into the gene's multiplicity vector (Multiplicity vector
//    building phase, Alg. 1: group equal identifiers, count, ascending order).
//    Genes with more than kMvSortCap windows are queued for k_mv_long, which
//    does the same with the codes in global memory.
// 2. A scan of the distinct-k-mer counts gives the CSR offsets, and
//    k_mv_compact packs the vectors while counting index entries per
//    leading-residue bucket.
// 3. A scan of the bucket counts gives the index directory; k_ix_scatter
//    places every (code, gene, count) entry in its bucket and the bucket sorts
//    order each bucket by (code, gene).  The result is the genome's inverted
//    index: all entries ordered by k-mer code, ties by gene.
#include "common.hpp"
#include "internal.hpp"

namespace pdp {

constexpr uint32_t kMvThreads = 256;
constexpr uint32_t kMvPer = kMvSortCap / kMvThreads;

__global__ __launch_bounds__(kMvThreads) void k_mv_local(const uint8_t *__restrict__ res, const uint64_t *__restrict__ off,
                                                         uint64_t n_residues, uint32_t k, uint32_t *__restrict__ nwin,
                                                         uint64_t *__restrict__ slot_code, uint32_t *__restrict__ slot_cnt,
                                                         uint32_t *__restrict__ dcnt, uint32_t *__restrict__ long_list,
                                                         uint32_t *__restrict__ counters, pdp_status *st) {
    __shared__ uint64_t keys[kMvSortCap];
    __shared__ uint8_t sym[kMvSortCap + PDP_K_MAX];
    __shared__ uint32_t tmp[kMvThreads / kWave + 1];
    const uint32_t g = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint64_t o = off[g];
    const uint64_t e = off[g + 1];
    if (e < o || e > n_residues) {
        if (tid == 0) {
            raise_status(st, PDP_E_INVAL, 0, g);
            nwin[g] = 0;
            dcnt[g] = 0;
        }
        return;
    }
    const uint64_t len = e - o;
    const uint64_t nw64 = len >= k ? len - k + 1 : 0;
    if (nw64 > PDP_MAX_WINDOWS) {
        if (tid == 0) {
            raise_status(st, PDP_E_LIMIT, nw64, g);
            nwin[g] = 0;
            dcnt[g] = 0;
        }
        return;
    }
    const uint32_t nw = static_cast<uint32_t>(nw64);
    const bool in_lds = nw <= kMvSortCap;
    for (uint64_t p = tid; p < len; p += kMvThreads) {
        uint32_t s = kSym.v[res[o + p]];
        if (s == kInvalidSym) {
            raise_status(st, PDP_E_ALPHABET, 0, o + p);
            s = 0;
        }
        if (in_lds) sym[p] = static_cast<uint8_t>(s);
    }
    if (tid == 0) nwin[g] = nw;
    if (!in_lds) {
        if (tid == 0) long_list[atomicAdd(&counters[0], 1u)] = g;
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
#pragma unroll
    for (uint32_t j = 0; j < kMvPer; ++j) {
        const uint32_t i = i0 + j;
        if (i < nw && (i == 0 || keys[i] != keys[i - 1])) {
            const uint64_t c = keys[i];
            uint32_t end = i + 1;
            while (end < nw && keys[end] == c) ++end;
            slot_code[o + rank] = c;
            slot_cnt[o + rank] = end - i;
            ++rank;
        }
    }
    if (tid == 0) dcnt[g] = total;
}

// Genes with more windows than fit in LDS: same steps, codes sorted in global memory.
__global__ __launch_bounds__(kMvThreads) void k_mv_long(const uint8_t *__restrict__ res, const uint64_t *__restrict__ off,
                                                        uint32_t k, uint64_t *tmp_codes, uint64_t *__restrict__ slot_code,
                                                        uint32_t *__restrict__ slot_cnt, uint32_t *__restrict__ dcnt,
                                                        const uint32_t *__restrict__ long_list,
                                                        const uint32_t *__restrict__ counters) {
    __shared__ uint32_t tmp[kMvThreads / kWave + 1];
    const uint32_t n_long = counters[0];
    const uint32_t tid = threadIdx.x;
    for (uint32_t li = blockIdx.x; li < n_long; li += gridDim.x) {
        const uint32_t g = long_list[li];
        const uint64_t o = off[g];
        const uint32_t nw = static_cast<uint32_t>(off[g + 1] - o - k + 1);
        uint64_t *w = tmp_codes + o;
        for (uint32_t p = tid; p < nw; p += kMvThreads) {
            uint64_t c = 0;
            for (uint32_t j = 0; j < k; ++j) {
                uint32_t s = kSym.v[res[o + p + j]];
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
                slot_code[o + base + r] = c;
                slot_cnt[o + base + r] = end - i;
            }
            base += total;
        }
        if (tid == 0) dcnt[g] = base;
        __syncthreads();
    }
}

// One wave per gene: move the vector to its CSR place and count bucket sizes.
__global__ __launch_bounds__(kWave) void k_mv_compact(const uint64_t *__restrict__ off, const uint64_t *__restrict__ slot_code,
                                                      const uint32_t *__restrict__ slot_cnt, const uint32_t *__restrict__ mv_ptr,
                                                      uint64_t *__restrict__ mv_code, uint32_t *__restrict__ mv_cnt,
                                                      uint32_t *__restrict__ bcount, uint32_t k, uint32_t lead) {
    const uint32_t g = blockIdx.x;
    const uint64_t o = off[g];
    const uint32_t p = mv_ptr[g];
    const uint32_t d = mv_ptr[g + 1] - p;
    for (uint32_t e = threadIdx.x; e < d; e += kWave) {
        const uint64_t c = slot_code[o + e];
        mv_code[p + e] = c;
        mv_cnt[p + e] = slot_cnt[o + e];
        atomicAdd(&bcount[bucket_of(c, k, lead)], 1u);
    }
}

// One wave per gene: drop each entry into its bucket (order inside a bucket is fixed later).
__global__ __launch_bounds__(kWave) void k_ix_scatter(const uint32_t *__restrict__ mv_ptr, const uint64_t *__restrict__ mv_code,
                                                      const uint32_t *__restrict__ mv_cnt, const uint32_t *__restrict__ ix_dir,
                                                      uint32_t *__restrict__ bfill, uint64_t *__restrict__ ix_code,
                                                      uint32_t *__restrict__ ix_gene, uint32_t *__restrict__ ix_cnt, uint32_t k,
                                                      uint32_t lead) {
    const uint32_t g = blockIdx.x;
    const uint32_t p = mv_ptr[g];
    const uint32_t d = mv_ptr[g + 1] - p;
    for (uint32_t e = threadIdx.x; e < d; e += kWave) {
        const uint64_t c = mv_code[p + e];
        const uint32_t b = bucket_of(c, k, lead);
        const uint32_t pos = ix_dir[b] + atomicAdd(&bfill[b], 1u);
        ix_code[pos] = c;
        ix_gene[pos] = g;
        ix_cnt[pos] = mv_cnt[p + e];
    }
}

__device__ __forceinline__ bool entry_less(uint64_t ca, uint32_t ga, uint64_t cb, uint32_t gb) {
    return ca < cb || (ca == cb && ga < gb);
}

// One thread per bucket: insertion sort of small buckets; large ones are queued.
__global__ __launch_bounds__(256) void k_ix_sort_small(uint32_t nb, const uint32_t *__restrict__ ix_dir, uint64_t *ix_code,
                                                       uint32_t *ix_gene, uint32_t *ix_cnt, uint32_t *__restrict__ big_list,
                                                       uint32_t *__restrict__ counters) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const uint32_t lo = ix_dir[b], hi = ix_dir[b + 1];
    const uint32_t n = hi - lo;
    if (n < 2) return;
    if (n > kBucketSmall) {
        big_list[atomicAdd(&counters[1], 1u)] = b;
        return;
    }
    for (uint32_t i = lo + 1; i < hi; ++i) {
        const uint64_t c = ix_code[i];
        const uint32_t gg = ix_gene[i], m = ix_cnt[i];
        uint32_t j = i;
        while (j > lo && entry_less(c, gg, ix_code[j - 1], ix_gene[j - 1])) {
            ix_code[j] = ix_code[j - 1];
            ix_gene[j] = ix_gene[j - 1];
            ix_cnt[j] = ix_cnt[j - 1];
            --j;
        }
        ix_code[j] = c;
        ix_gene[j] = gg;
        ix_cnt[j] = m;
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
__global__ __launch_bounds__(256) void k_ix_sort_big(const uint32_t *__restrict__ ix_dir, uint64_t *ix_code, uint32_t *ix_gene,
                                                     uint32_t *ix_cnt, const uint32_t *__restrict__ big_list,
                                                     const uint32_t *__restrict__ counters) {
    __shared__ uint64_t s_code[kBigLds];
    __shared__ uint32_t s_gene[kBigLds];
    __shared__ uint32_t s_cnt[kBigLds];
    const uint32_t n_big = counters[1];
    for (uint32_t bi = blockIdx.x; bi < n_big; bi += gridDim.x) {
        const uint32_t b = big_list[bi];
        const uint32_t lo = ix_dir[b], n = ix_dir[b + 1] - lo;
        if (n <= kBigLds) {
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                s_code[i] = ix_code[lo + i];
                s_gene[i] = ix_gene[lo + i];
                s_cnt[i] = ix_cnt[lo + i];
            }
            __syncthreads();
            sort_entries(s_code, s_gene, s_cnt, n);
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                ix_code[lo + i] = s_code[i];
                ix_gene[lo + i] = s_gene[i];
                ix_cnt[lo + i] = s_cnt[i];
            }
        } else {
            sort_entries(ix_code + lo, ix_gene + lo, ix_cnt + lo, n);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host

uint64_t dict_ws_bytes(uint32_t n_genes, uint64_t n_residues, uint32_t k) {
    const uint64_t nb = n_buckets_for(k);
    const uint64_t A = 256;
    uint64_t s = 0;
    s += align_up(8 * (n_residues + 1), A);      // slot_code
    s += align_up(4 * (n_residues + 1), A);      // slot_cnt
    s += align_up(8 * (n_residues + 1), A);      // long_tmp
    s += align_up(4 * (uint64_t(n_genes) + 1), A);  // dcnt
    s += align_up(4 * (nb + 1), A);              // bcount
    s += align_up(4 * (uint64_t(n_genes) + 1), A);  // long_list
    s += align_up(4 * (nb + 1), A);              // big_list
    s += align_up(4 * 4, A);                     // counters
    const uint64_t np = std::max<uint64_t>(scan_partials(n_genes), scan_partials(nb));
    s += align_up(4 * np, A);
    return s;
}

DictBuildWs dict_ws_carve(void *ws, uint32_t n_genes, uint64_t n_residues, uint32_t k) {
    const uint64_t nb = n_buckets_for(k);
    const uint64_t A = 256;
    char *p = static_cast<char *>(ws);
    DictBuildWs w;
    auto take = [&](uint64_t bytes) {
        char *q = p;
        p += align_up(bytes, A);
        return q;
    };
    w.slot_code = reinterpret_cast<uint64_t *>(take(8 * (n_residues + 1)));
    w.slot_cnt = reinterpret_cast<uint32_t *>(take(4 * (n_residues + 1)));
    w.long_tmp = reinterpret_cast<uint64_t *>(take(8 * (n_residues + 1)));
    w.dcnt = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(n_genes) + 1)));
    w.bcount = reinterpret_cast<uint32_t *>(take(4 * (nb + 1)));
    w.long_list = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(n_genes) + 1)));
    w.big_list = reinterpret_cast<uint32_t *>(take(4 * (nb + 1)));
    w.counters = reinterpret_cast<uint32_t *>(take(4 * 4));
    const uint64_t np = std::max<uint64_t>(scan_partials(n_genes), scan_partials(nb));
    w.partials = reinterpret_cast<uint32_t *>(take(4 * np));
    return w;
}

#define PDP_TRY(x)                              \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

hipError_t launch_dict_build(const pdp_genome *g, pdp_dict *d, const DictBuildWs &w, hipStream_t s) {
    const uint32_t n = g->n_genes;
    const uint32_t k = d->k;
    const uint32_t nb = d->n_buckets;
    const uint32_t lead = lead_residues(k);
    PDP_TRY(launch_status_init(d->status, s));
    PDP_TRY(launch_fill_u32(w.counters, 4, 0u, s));
    PDP_TRY(launch_fill_u32(w.bcount, uint64_t(nb) + 1, 0u, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_mv_local, dim3(n), dim3(kMvThreads), 0, s, g->residues, g->gene_off, g->n_residues, k, d->nwin,
                           w.slot_code, w.slot_cnt, w.dcnt, w.long_list, w.counters, d->status);
        PDP_TRY(hipGetLastError());
        const uint32_t long_groups = n < 64 ? n : 64;
        hipLaunchKernelGGL(k_mv_long, dim3(long_groups), dim3(kMvThreads), 0, s, g->residues, g->gene_off, k, w.long_tmp,
                           w.slot_code, w.slot_cnt, w.dcnt, w.long_list, w.counters);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(launch_scan(w.dcnt, d->mv_ptr, n, w.partials, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_mv_compact, dim3(n), dim3(kWave), 0, s, g->gene_off, w.slot_code, w.slot_cnt, d->mv_ptr,
                           d->mv_code, d->mv_cnt, w.bcount, k, lead);
        PDP_TRY(hipGetLastError());
    }
    PDP_TRY(launch_scan(w.bcount, d->ix_dir, nb, w.partials, s));
    PDP_TRY(launch_fill_u32(w.bcount, nb, 0u, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_ix_scatter, dim3(n), dim3(kWave), 0, s, d->mv_ptr, d->mv_code, d->mv_cnt, d->ix_dir, w.bcount,
                           d->ix_code, d->ix_gene, d->ix_cnt, k, lead);
        PDP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_ix_sort_small, dim3((nb + 255) / 256), dim3(256), 0, s, nb, d->ix_dir, d->ix_code, d->ix_gene,
                           d->ix_cnt, w.big_list, w.counters);
        PDP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_ix_sort_big, dim3(64), dim3(256), 0, s, d->ix_dir, d->ix_code, d->ix_gene, d->ix_cnt,
                           w.big_list, w.counters);
        PDP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace pdp
