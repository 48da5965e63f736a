// Host/device declarations shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdp.h"

namespace pdp {

// Returns a failing hipError_t from the enclosing launcher.
#define PDP_TRY(x)                              \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// ---------------------------------------------------------------- sizes
constexpr uint32_t kScanItems = 4096;        // elements per scan work-group (256 threads x 16)
constexpr uint32_t kMvSortCap = 8192;        // windows a gene may have to be sorted in LDS
constexpr uint32_t kKMaxAll = PDP_K_MAX_NT > PDP_K_MAX ? PDP_K_MAX_NT : PDP_K_MAX;  // k bound over alphabets
constexpr uint32_t kIxBlock = 16384;         // index entries per histogram block
constexpr uint32_t kIxBinTarget = 512;       // average index entries per coarse bin
constexpr uint32_t kIxBinLds = 1024;         // coarse bins up to this size are sorted in LDS
constexpr uint32_t kIxBinSlots = 2048;       // counting-sort slots of a bin (buckets x sub-slots)
constexpr uint32_t kIxMaxBins = 8192;        // coarse bins per genome at most (LDS histogram)
constexpr uint32_t kJoinLdsCap = 1024;       // target index entries staged in LDS per join sub-range
constexpr uint32_t kJoinLdsCapP = 2048;      // the same for dictionaries with packed 32-bit keys
constexpr uint32_t kJoinDirCap = 512;        // leading-letter buckets per join item (sub-ranges x buckets)
constexpr uint32_t kJoinTileCap = 1024;      // accumulation tiles per task (one LDS counter each in the join)
constexpr uint32_t kTileMaxRows = 256;       // rows per accumulation tile (8-bit row field of a record)
constexpr uint32_t kDefaultTileShift = 6;    // 64 rows per tile unless tuned
constexpr uint32_t kTileThreads = 256;
constexpr uint32_t kTileCap = 4096;          // records a tile sorts in LDS (8 bytes each)
constexpr uint32_t kTilePer = kTileCap / kTileThreads;
constexpr uint32_t kHashBits = 12;           // LDS hash table of a tile: 2^12 slots, 8 bytes each
constexpr uint32_t kHashSlots = 1u << kHashBits;
constexpr uint32_t kHashMax = kHashSlots * 3 / 4;  // records one table pass takes (load factor <= 3/4)
constexpr uint32_t kDefaultLdsBudget = 8 * kTileCap;
constexpr uint32_t kMaxTileLds = 160 * 1024 - 4096;  // gfx950 LDS per work-group, less the static part
constexpr uint32_t kSlab = 4;                // best hits per row kept by the first tile pass
constexpr uint32_t kLongCols = 4096;         // long-gene path: column genes per LDS block (one word per sum)

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Per alphabet: bits of a letter's symbol, letters, leading letters of an index bucket
// (amino acids: 20^4 = 160000 buckets; nucleotides: 4^9 = 262144, so that a bucket of a
// genome holds a few entries either way), largest k.
struct AlphaSpec {
    uint32_t bits, sigma, lead_max, k_max;
};
inline bool alpha_known(uint32_t a) { return a == PDP_ALPHA_AMINO || a == PDP_ALPHA_NUCLEOTIDE; }
inline AlphaSpec alpha_spec(uint32_t a) {
    return a == PDP_ALPHA_NUCLEOTIDE ? AlphaSpec{2, 4, 9, PDP_K_MAX_NT} : AlphaSpec{5, 20, 4, PDP_K_MAX};
}
inline uint32_t lead_letters(uint32_t k, uint32_t a) {
    const uint32_t m = alpha_spec(a).lead_max;
    return k < m ? k : m;
}
inline uint32_t n_buckets_for(uint32_t k, uint32_t a) {
    uint32_t nb = 1;
    for (uint32_t i = 0; i < lead_letters(k, a); ++i) nb *= alpha_spec(a).sigma;
    return nb;
}
// Gene bits of a dictionary's packed index keys, 0 when tail and gene do not fit 32 bits.
inline uint32_t key_shift_for(uint32_t n_genes, uint32_t k, uint32_t a) {
    uint32_t gb = 1;
    while (gb < 32 && (1ull << gb) < n_genes) ++gb;
    return alpha_spec(a).bits * (k - lead_letters(k, a)) + gb <= 32 ? gb : 0;
}
inline uint32_t scan_partials(uint64_t n) { return static_cast<uint32_t>((n + kScanItems - 1) / kScanItems) + 1; }

// --------------------------------------------------------- device tables
struct DevDict {
    const uint64_t *ix_code;
    const uint32_t *ix_gene;
    const uint32_t *ix_cnt;
    const uint32_t *ix_dir;
    const uint32_t *nwin;
    const uint32_t *ix_key;  // packed (tail, gene) keys when key_shift > 0
    const uint32_t *mv_ptr;  // multiplicity vectors (the long-gene path walks a row gene's)
    const uint64_t *mv_code;
    const uint32_t *mv_cnt;
    uint32_t n_genes;
    uint32_t n_buckets;
    uint32_t k;
    uint32_t key_shift;
    uint32_t bits;  // symbol bits per letter: 5 (amino acids) or 2 (nucleotides)
    uint32_t lead;  // leading letters of a bucket
};

// DevTask.flags: PDP_TASK_AB / PDP_TASK_BA select the join's record directions; a task whose
// BA best hits come from the column maxima of its AB tiles has kTaskColmax instead of BA.
constexpr uint32_t kTaskColmax = 8u;
// DevTask.flags: a and b hold the caller's b and a (the smaller genome queries the join); the
// directions (flags, tile fields, row bases) are the task's own, BBH rows keep the caller's a.
constexpr uint32_t kTaskSwapped = 16u;

struct DevTask {
    DevDict a, b;
    uint32_t flags;
    uint32_t bpw;           // buckets per join sub-range
    uint32_t subs;          // sub-ranges per join item
    uint32_t chunk_base;    // first join item of the task
    uint32_t n_chunks;      // join items of the task
    uint32_t tile_shift[2]; // rows per tile = 2^tile_shift, direction 0 (a rows) and 1 (b rows)
    uint32_t tiles_n[2];    // tiles per direction (0 when the direction is not requested)
    uint32_t tile_base[2];  // first tile of each direction
    uint32_t row_base[2];   // first best-hit row of each direction (UINT32_MAX: none)
    uint32_t bbh_row_base;  // first BBH row (UINT32_MAX: none)
    uint32_t cell_base;     // first cell of the task's (item, tile) record counts (item-major)
    uint32_t theta_n, theta_d, tau_n, tau_d;  // candidate filters (zero denominator: off)
};

// A join item of the one-pass join, laid out by the plan: its task, its buckets' slices of
// both genomes' directories (from its first bucket), and how many buckets it covers.
struct DevItem {
    const uint32_t *adir;
    const uint32_t *bdir;
    uint32_t task;
    uint32_t n_buckets;
    uint32_t bl;  // first bucket
    uint32_t reserved;
};

// The rows of one direction of a task on the long-gene path: rows first .. first + n_rows of
// the plan's long-row numbering are the task's row genes 0 .. n_rows - 1 in direction dir.
struct DevLongSeg {
    uint32_t task;
    uint32_t dir;
    uint32_t first;
    uint32_t n_rows;
};

struct DevTile {
    uint32_t task;
    uint32_t dir;
    uint32_t row0;
    uint32_t nrows;
    uint32_t rbase;  // the tile's record region in the one-pass join: records rbase .. rbase + rcap
    uint32_t rcap;
};

// ------------------------------------------------------------- launchers
// All return hipError_t of the launch.
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_status_init(pdp_status *st, hipStream_t s);
// Exclusive scan of n values: out[0..n] with out[n] = total.  out may equal in
// (then in needs n+1 slots).  partials: scan_partials(n) words of scratch.
hipError_t launch_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *partials, hipStream_t s);

// One genome of a dictionary build: input, outputs and its slices of the
// workspace.  Genes and buckets of all genomes of a build are numbered
// consecutively from gene_base / bucket_base.
struct DevBuild {
    const uint8_t *res;
    const uint64_t *off;
    uint64_t n_residues;
    uint32_t n_genes, k, nb, lead, gene_base;
    uint32_t hshift, nh, nblk;            // coarse bins of 2^hshift buckets; entry blocks for the histogram
    uint32_t xb;                          // sub-slot bits per bucket of a bin's counting sort (next letters)
    uint32_t blk_base, bin_base;          // first block and bin of the genome
    uint32_t *nwin, *mv_ptr;
    uint64_t *mv_code;
    uint32_t *mv_cnt, *ix_dir;
    uint64_t *ix_code;
    uint32_t *ix_gene, *ix_cnt;
    uint32_t *ix_key;     // packed keys, written when key_shift > 0
    uint32_t key_shift;
    uint32_t bits;        // symbol bits per letter: 5 (amino acids) or 2 (nucleotides)
    uint32_t max_windows; // PDP_MAX_WINDOWS, or PDP_MAX_WINDOWS_LONG for a long-gene dictionary
    pdp_status *status;
    uint64_t *slot_code;  // per gene g: sorted distinct codes at offset gene_off[g]
    uint32_t *slot_cnt;
    uint64_t *long_tmp;   // windows of genes too long for LDS
    uint4 *ix_tmp;        // index entries placed by coarse bin, before the bin sort
};
struct BuildShape {
    uint64_t n_genomes, total_genes, total_residues, total_blocks, total_bins, max_nh;
};
BuildShape build_shape(const pdp_genome *g, const pdp_dict *const *d, uint32_t n);
BuildShape single_build_shape(uint32_t n_genes, uint64_t n_residues, uint32_t k, uint32_t alphabet);
uint64_t build_ws_bytes(const BuildShape &s);
hipError_t launch_dict_build_many(const pdp_genome *g, pdp_dict *const *d, uint32_t n, void *ws, hipStream_t s);

struct PairWs {
    DevTask *tasks;
    DevTile *tiles;
    DevItem *items;               // one per join item (the one-pass join)
    uint2 *recs;                  // records grouped by tile: ((row in tile << 24) | column, min count)
    unsigned long long *counters; // [0] records counted by the join
    uint32_t *cells;              // (item, tile) record counts of the join's count pass, item-major
    uint32_t *tile_tot;           // records per tile, counted by the join (the write pass consumes them)
    uint32_t *tile_off;           // scanned tile totals: tile t's records start at tile_off[t]; + 1
    uint32_t *fill;               // one-pass join: records reserved in each tile's region
    uint2 *tile_rng;              // records of each tile, [x, y), for the tile kernels
    uint32_t *fallback;           // counters word 7: a region overflowed, the two-pass join redoes the records
    uint32_t *next_fused;         // counters words 8..15: next item of each XCD in the persistent one-pass join
    uint4 *slab;                  // kSlab (column, m, d, -) per best-hit row
    uint32_t *overflow_tiles;     // tiles holding a row with more than kSlab ties
    uint32_t *overflow_count;     // counters word 2
    uint32_t *next_join;          // counters word 3: next item of the persistent join
    uint32_t *next_tile;          // counters word 4: next tile of the persistent tile pass
    uint32_t *next_join_write;    // counters word 5: next item of the persistent join's write pass
    uint32_t *order;              // task table indices in the caller's order
    uint32_t *partials;
    // column maxima (kTaskColmax): per best-hit row the running maximum key of its column,
    // a cursor for rows with more than kSlab ties, and the candidate list with its count
    unsigned long long *colkey;
    uint32_t *colcursor;
    uint4 *cands;
    uint32_t *cand_count;         // counters word 6
    DevLongSeg *long_segs;        // long-gene path, by first row
};

struct PlanShape {
    uint32_t n_tasks, total_chunks, total_tiles, total_cells, bh_rows, bbh_rows, tile_lds;
    uint64_t rec_cap;               // records the scratch holds
    uint32_t join_grid, tile_grid;  // persistent grids (0: one work-group per item)
    uint32_t colmax;                // some task takes its BA best hits from column maxima
    uint32_t fused;                 // one-pass join into per-tile regions (else count pass + write pass)
    uint32_t join_tiles;            // most tiles of one task: LDS counters of the one-pass join
    uint32_t fallback_grid;         // work-groups of the two-pass join when it backs up the one-pass join
    uint64_t cand_cap;              // column candidates the scratch holds (colmax: rec_cap)
    uint32_t n_long_segs;           // long-gene path: segments and rows
    uint32_t long_rows;
    uint32_t long_lds;              // long-gene path: LDS bytes of a work-group (one or three sums per column)
};
// Records the message that pdp_last_error() returns on this thread; returns code.
int32_t api_fail(int32_t code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Work-groups of the persistent kernels that fit the current device at once.
uint32_t persistent_join_grid();
// Moves a plan's pointers from dictionary `from` to dictionary `to`, bound with the same sizes
// elsewhere (so a plan made before a dictionary's memory is placed serves it afterwards).
// PDP_E_INVAL when the two differ in anything but their addresses.
int32_t plan_rebind(pdp_plan *plan, const pdp_dict *from, const pdp_dict *to);
uint32_t persistent_fused_grid(uint32_t join_tiles);
uint32_t persistent_tile_grid(uint32_t tile_lds);
hipError_t allow_tile_lds(uint32_t tile_lds);
uint64_t pair_ws_bytes(const PlanShape &p);
PairWs pair_ws_carve(void *ws, const PlanShape &p);
// Optional events recorded around one kernel of a launch (kernel < 0: none).
struct KernelTimer {
    int32_t kernel;
    hipEvent_t start, stop;
};
hipError_t launch_pairs(const PlanShape &p, const PairWs &w, pdp_bh_out *bh, pdp_bbh_out *bbh,
                        pdp_status *st, hipStream_t s, const KernelTimer *timer);
// Families (connected components of the BBH network) into labels[n_nodes].
hipError_t launch_families(const PlanShape &p, const PairWs &w, const pdp_bbh_out *bbh, const uint32_t *node_a,
                           const uint32_t *node_b, uint32_t n_nodes, uint32_t *labels, pdp_status *st, hipStream_t s);
hipError_t launch_bbh_standalone(const pdp_bh_out *ab, const pdp_bh_out *ba, pdp_bbh_out *out,
                                 pdp_status *st, uint32_t *partials, hipStream_t s);

}  // namespace pdp
