// Gene families from the bidirectional best hits (phase (c) of the pipeline): the BBH
// pairs of every genome pair of a plan are the edges of one network over all genes of all
// genomes, and a family is a connected component of it.  The paper names no refinement of
// the network, so none is applied.
//
// Lock-free union-find on the label array itself: every node starts as its own root; an
// edge hooks the larger of its two roots under the smaller with a compare-and-swap, and
// finding a root follows parent links, halving the path on the way.  A link only ever
// points to a smaller node, so every walk and every retry ends, and the root left in each
// component is its smallest node, which becomes every member's label.
#include "common.hpp"
#include "internal.hpp"

namespace pdp {

__device__ __forceinline__ uint32_t cc_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x; links on the way are shortened to their grandparents (still ancestors).
__device__ __forceinline__ uint32_t cc_find(uint32_t *parent, uint32_t x) {
    for (;;) {
        const uint32_t p = cc_load(&parent[x]);
        if (p == x) return x;
        const uint32_t gp = cc_load(&parent[p]);
        if (gp != p) atomicMin(&parent[x], gp);
        x = gp;
    }
}

__device__ __forceinline__ void cc_union(uint32_t *parent, uint32_t u, uint32_t v) {
    for (;;) {
        u = cc_find(parent, u);
        v = cc_find(parent, v);
        if (u == v) return;
        const uint32_t hi = u > v ? u : v, lo = u > v ? v : u;
        if (atomicCAS(&parent[hi], hi, lo) == hi) return;
        // hi was hooked by another edge meanwhile: its new root is smaller, try again
    }
}

__global__ __launch_bounds__(256) void k_cc_init(uint32_t *parent, uint32_t n) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) parent[v] = v;
}

// Caller-order index of the task owning BBH row `row` (BBH row bases ascend in caller order).
__device__ __forceinline__ uint32_t bbh_caller_task(const DevTask *tasks, const uint32_t *order, uint32_t n_tasks,
                                                    uint32_t row) {
    uint32_t lo = 0, hi = n_tasks - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (tasks[order[mid]].bbh_row_base <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One thread per BBH row: every pair of the row joins its two genes' families.
__global__ __launch_bounds__(256) void k_cc_hook(const DevTask *__restrict__ tasks, const uint32_t *__restrict__ order,
                                                 uint32_t n_tasks, uint32_t bbh_rows, const uint32_t *__restrict__ ptr,
                                                 const uint32_t *__restrict__ pa, const uint32_t *__restrict__ pb,
                                                 uint64_t cap, const uint32_t *__restrict__ node_a,
                                                 const uint32_t *__restrict__ node_b, uint32_t n_nodes,
                                                 uint32_t *parent, pdp_status *st) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= bbh_rows) return;
    const uint32_t ct = bbh_caller_task(tasks, order, n_tasks, r);
    const uint64_t base_a = node_a[ct], base_b = node_b[ct];
    const uint32_t p1 = ptr[r + 1] < cap ? ptr[r + 1] : static_cast<uint32_t>(cap);
    for (uint32_t p = ptr[r]; p < p1; ++p) {
        const uint64_t u = base_a + pa[p], v = base_b + pb[p];
        if (u >= n_nodes || v >= n_nodes) {
            raise_status(st, PDP_E_INVAL, u > v ? u : v, r);
            continue;
        }
        cc_union(parent, static_cast<uint32_t>(u), static_cast<uint32_t>(v));
    }
}

// After every union: each node's label is its root.
__global__ __launch_bounds__(256) void k_cc_flatten(uint32_t *parent, uint32_t n) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        const uint32_t r = cc_find(parent, v);
        parent[v] = r;
    }
}

hipError_t launch_families(const PlanShape &p, const PairWs &w, const pdp_bbh_out *bbh, const uint32_t *node_a,
                           const uint32_t *node_b, uint32_t n_nodes, uint32_t *labels, pdp_status *st, hipStream_t s) {
    PDP_TRY(launch_status_init(st, s));
    if (n_nodes) {
        hipLaunchKernelGGL(k_cc_init, dim3((n_nodes + 255) / 256), dim3(256), 0, s, labels, n_nodes);
        PDP_TRY(hipGetLastError());
    }
    if (p.bbh_rows && n_nodes) {
        hipLaunchKernelGGL(k_cc_hook, dim3((p.bbh_rows + 255) / 256), dim3(256), 0, s, w.tasks, w.order, p.n_tasks,
                           p.bbh_rows, bbh->ptr, bbh->a, bbh->b, bbh->capacity, node_a, node_b, n_nodes, labels, st);
        PDP_TRY(hipGetLastError());
    }
    if (n_nodes) {
        hipLaunchKernelGGL(k_cc_flatten, dim3((n_nodes + 255) / 256), dim3(256), 0, s, labels, n_nodes);
        PDP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace pdp
