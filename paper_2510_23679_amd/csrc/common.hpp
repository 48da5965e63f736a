// Device helpers shared by the gfx950 kernels of the best-hit library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdp.h"

namespace pdp {

constexpr uint32_t kWave = 64;
constexpr uint32_t kInvalidSym = 0xFFu;

// Residue letter -> 5-bit symbol (A=0 ... Y=19 in the order ACDEFGHIKLMNPQRSTVWY), kInvalidSym
// otherwise.  The 26 upper-case letters' symbols sit 5 bits each in three 64-bit constants
// (12 letters per word, 31 = not an amino acid), so the mapping is register arithmetic and
// no memory load.
constexpr uint64_t sym_word(int w) {
    const char letters[] = "ACDEFGHIKLMNPQRSTVWY";
    uint64_t word = 0;
    for (int j = 0; j < 12; ++j) {
        const int letter = 12 * w + j;  // 0 = 'A'
        uint64_t s = 31;
        for (int i = 0; i < 20; ++i)
            if (letters[i] - 'A' == letter) s = static_cast<uint64_t>(i);
        word |= s << (5 * j);
    }
    return word;
}
constexpr uint64_t kSymWord0 = sym_word(0), kSymWord1 = sym_word(1), kSymWord2 = sym_word(2);
static_assert((kSymWord0 & 31) == 0 && ((kSymWord0 >> 5) & 31) == 31 && ((kSymWord0 >> 10) & 31) == 1,
              "A -> 0, B -> none, C -> 1");
static_assert((kSymWord2 & 31) == 19 && ((kSymWord2 >> 5) & 31) == 31, "Y -> 19, Z -> none");

__device__ __forceinline__ uint32_t sym_of(uint32_t byte) {
    const uint32_t i = byte - 'A';
    if (i >= 26u) return kInvalidSym;
    const uint64_t word = i < 12u ? kSymWord0 : (i < 24u ? kSymWord1 : kSymWord2);
    const uint32_t s = static_cast<uint32_t>(word >> (5u * (i % 12u))) & 31u;
    return s == 31u ? kInvalidSym : s;
}

// Nucleotide letter -> 2-bit symbol (A=0, C=1, G=2, T=3), kInvalidSym otherwise: a mask of
// the four letters among the 26 and their symbols 2 bits each at the letter's index.
constexpr uint32_t kNtMask = (1u << ('A' - 'A')) | (1u << ('C' - 'A')) | (1u << ('G' - 'A')) | (1u << ('T' - 'A'));
constexpr uint64_t kNtWord = (1ull << (2 * ('C' - 'A'))) | (2ull << (2 * ('G' - 'A'))) | (3ull << (2 * ('T' - 'A')));

__device__ __forceinline__ uint32_t sym_nt(uint32_t byte) {
    const uint32_t i = byte - 'A';
    if (i >= 26u || !((kNtMask >> i) & 1u)) return kInvalidSym;
    return static_cast<uint32_t>(kNtWord >> (2u * i)) & 3u;
}

// Symbol of a letter in a dictionary whose symbols are `bits` wide (5: amino acids, 2: nucleotides).
__device__ __forceinline__ uint32_t sym_in(uint32_t byte, uint32_t bits) { return bits == 2u ? sym_nt(byte) : sym_of(byte); }

// Leading-letter bucket of a k-mer code: for nucleotides the leading 2*lead bits (the code
// is the k-mer's base-4 value), for amino acids the first `lead` residues read as a base-20
// number.
__device__ __forceinline__ uint32_t bucket_of(uint64_t code, uint32_t k, uint32_t lead, uint32_t bits) {
    if (bits == 2u) return static_cast<uint32_t>(code >> (2u * (k - lead)));
    uint32_t b = 0;
    for (uint32_t i = 0; i < lead; ++i) b = b * 20u + static_cast<uint32_t>((code >> (5u * (k - 1u - i))) & 31u);
    return b;
}

// Loads and stores issued as global (not flat) accesses, for pointers read out of memory (a
// table in LDS or device memory) whose address space the compiler cannot infer: a flat access
// also waits on the LDS counter, so it serialises with the kernel's LDS traffic.  Only for
// pointers into device memory.
template <typename T>
__device__ __forceinline__ T load_global(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ void store_global(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of mask in lanes below this lane.
__device__ __forceinline__ uint32_t mask_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (uint32_t d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// Reserves n slots per lane from a global 64-bit counter with one atomic per wave;
// returns this lane's first slot.  Every lane of the wave must call it.
__device__ __forceinline__ unsigned long long wave_reserve(uint32_t n, unsigned long long *counter) {
    const uint32_t incl = wave_inclusive_sum(n);
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    unsigned long long base = 0;
    if (lane_id() == kWave - 1 && total) base = atomicAdd(counter, static_cast<unsigned long long>(total));
    base = __shfl(base, kWave - 1, kWave);
    return base + (incl - n);
}

// Exclusive scan over a work-group of NT threads; tmp needs NT/64 + 1 words of LDS.
// Returns this thread's exclusive prefix; *total receives the sum.  Contains barriers.
template <uint32_t NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *tmp, uint32_t *total) {
    constexpr uint32_t NW = NT / kWave;
    const uint32_t lane = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t incl = wave_inclusive_sum(x);
    if (lane == kWave - 1) tmp[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t i = 0; i < NW; ++i) {
            uint32_t t = tmp[i];
            tmp[i] = run;
            run += t;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    const uint32_t r = tmp[w] + incl - x;
    *total = tmp[NW];
    __syncthreads();
    return r;
}

// Comparator network sort of n items by one work-group, ascending, for any n.
// It is the bitonic network in its "flip" form: every comparator (lo, hi) with
// lo < hi leaves the smaller item at lo, so the missing items past n act as +inf
// and comparators that reach past n are skipped.  cmpswap(lo, hi) orders one
// pair; the items may live in LDS or in global memory (the barriers order both
// within the work-group).
template <typename CmpSwap>
__device__ void wg_network_sort(uint32_t n, CmpSwap cmpswap) {
    if (n < 2) return;
    uint32_t p2 = 1;
    while (p2 < n) p2 <<= 1;
    const uint32_t half_n = p2 >> 1;  // comparators per step
    for (uint32_t size = 2; size <= p2; size <<= 1) {
        const uint32_t half = size >> 1;
        const uint32_t lh = 31u - __builtin_clz(half);
        for (uint32_t i = threadIdx.x; i < half_n; i += blockDim.x) {
            const uint32_t blk = i >> lh, pos = i & (half - 1u);
            const uint32_t lo = blk * size + pos;
            const uint32_t hi = blk * size + size - 1u - pos;
            if (hi < n) cmpswap(lo, hi);
        }
        __syncthreads();
        for (uint32_t stride = half >> 1; stride > 0; stride >>= 1) {
            const uint32_t ls = 31u - __builtin_clz(stride);
            for (uint32_t i = threadIdx.x; i < half_n; i += blockDim.x) {
                const uint32_t blk = i >> ls, pos = i & (stride - 1u);
                const uint32_t lo = blk * 2u * stride + pos;
                const uint32_t hi = lo + stride;
                if (hi < n) cmpswap(lo, hi);
            }
            __syncthreads();
        }
    }
}

// Status reporting from device code: the first error code wins.
__device__ __forceinline__ void raise_status(pdp_status *st, int32_t code, uint64_t needed, uint64_t where) {
    atomicCAS(&st->code, 0, code);
    if (needed) atomicMax(reinterpret_cast<unsigned long long *>(&st->needed), static_cast<unsigned long long>(needed));
    if (where != ~0ull) atomicMin(reinterpret_cast<unsigned long long *>(&st->where), static_cast<unsigned long long>(where));
}

}  // namespace pdp
