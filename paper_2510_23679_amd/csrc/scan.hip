// Utility kernels: fills, status initialisation and a device-wide exclusive scan.
#include "common.hpp"
#include "internal.hpp"

namespace pdp {

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_status_init(pdp_status *st) {
    st->code = 0;
    st->flags = 0;
    st->needed = 0;
    st->where = ~0ull;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_status_init(pdp_status *st, hipStream_t s) {
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError();
}

// ----------------------------------------------------------------- scan
// Three phases: per-group sums, a scan of the sums by one group, and a
// per-group scan that adds the group's offset (up to kScanFuseGroups groups the
// second phase folds into the third).  A group covers kScanItems
// consecutive values (16 per thread, blocked).
constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPer = kScanItems / kScanThreads;

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *in, uint64_t n, uint32_t *partials) {
    __shared__ uint32_t tmp[kScanThreads / kWave + 1];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanItems + threadIdx.x * kScanPer;
    uint32_t s = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j)
        if (base + j < n) s += in[base + j];
    uint32_t total;
    block_exclusive_scan<kScanThreads>(s, tmp, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t *partials, uint32_t nb) {
    __shared__ uint32_t tmp[kScanThreads / kWave + 1];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? partials[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<kScanThreads>(v, tmp, &total);
        if (i < nb) partials[i] = carry + ex;
        carry += total;
    }
}

// FUSED: partials holds the groups' plain sums (no k_scan_top), and every group adds up
// those of the groups before it itself, so a scan of up to kScanFuseGroups groups takes
// two launches instead of three.
template <bool FUSED>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint32_t *in, uint32_t *out, uint64_t n,
                                                              const uint32_t *partials, uint32_t nb) {
    __shared__ uint32_t tmp[kScanThreads / kWave + 1];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanItems + threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j) {
        v[j] = base + j < n ? in[base + j] : 0u;
        s += v[j];
    }
    uint32_t before = 0;
    if (FUSED) {
        uint32_t mine = 0;
        for (uint32_t g = threadIdx.x; g < blockIdx.x; g += kScanThreads) mine += partials[g];
        uint32_t all;
        (void)block_exclusive_scan<kScanThreads>(mine, tmp, &all);
        before = all;
    } else if (nb > 1) {
        before = partials[blockIdx.x];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan<kScanThreads>(s, tmp, &total) + before;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
        // the last thread of the last group ends on the grand total
        out[n] = run;
    }
}

constexpr uint32_t kScanFuseGroups = 1024;  // up to here each group sums the earlier group totals itself

hipError_t launch_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *partials, hipStream_t s) {
    const uint32_t nb = static_cast<uint32_t>((n + kScanItems - 1) / kScanItems);
    if (nb == 0) return launch_fill_u32(out, 1, 0u, s);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply<false>, dim3(1), dim3(kScanThreads), 0, s, in, out, n, partials, nb);
    } else if (nb <= kScanFuseGroups) {
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, partials);
        hipLaunchKernelGGL(k_scan_apply<true>, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, partials, nb);
    } else {
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, partials);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, partials, nb);
        hipLaunchKernelGGL(k_scan_apply<false>, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, partials, nb);
    }
    return hipGetLastError();
}

}  // namespace pdp
