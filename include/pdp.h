/*
 * pdp.h -- C-ABI of the MI355X (gfx950) best-hit library for PanDelos-plus.
 *
 * The library computes, for pairs of genomes, the generalised Jaccard
 * similarity of every gene pair (Eq. jaccard_k), each gene's best hits in the
 * other genome with ties kept (Eq. best_hit, the jagged array of Alg. 2) and
 * the bidirectional best hits (Eq. bidirectional_best_hit, Alg. 3).  The
 * problem statement it follows is the paper's Basic notions section: a
 * genome is an ordered list of genes, a gene is a string over a nucleotide
 * or an amino-acid alphabet (both are supported), and k is chosen by phase
 * (a) (Eq. k_length).
 *
 * Conventions shared by every entry point
 *  - Device buffers are allocated and owned by the caller.  The library never
 *    frees caller memory and keeps no caller pointer after a call returns;
 *    a pdp_plan keeps copies of the dictionary descriptors it was created
 *    from, so those dictionaries must stay alive while the plan is used.
 *  - "device" below means memory of the current HIP device; "host" means
 *    ordinary process memory.
 *  - Calls that take a stream only enqueue work on it (the stream is a
 *    hipStream_t passed as void*, NULL = the default stream) and return after
 *    synchronous validation.  Conditions found while the kernels run go to a
 *    caller-provided device pdp_status, to be read after the stream has
 *    synchronised.
 *  - Return codes: PDP_OK (0) or a negative PDP_E_* code.  No C++ exception
 *    crosses this boundary.  pdp_last_error() gives a message for the last
 *    failing call on the calling thread.
 *  - Integer results are exact; nothing on the path uses floating point.
 */
#ifndef PDP_H
#define PDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDP_ABI_VERSION 6u

/* The two alphabets of the Basic notions section.  A dictionary's alphabet
 * fixes how a letter becomes a symbol, the symbol width of a k-mer code and
 * the largest k. */
enum pdp_alphabet {
    PDP_ALPHA_AMINO = 0,      /* ACDEFGHIKLMNPQRSTVWY -> 0..19, 5 bits per letter */
    PDP_ALPHA_NUCLEOTIDE = 1  /* ACGT -> 0..3, 2 bits per letter */
};
/* Largest k per alphabet: codes of k letters fit in 60 (amino acids) or 62
 * (nucleotides) bits, below the all-ones value the kernels use as padding. */
#define PDP_K_MAX 12u
#define PDP_K_MAX_NT 31u
/* A gene may have at most this many k-mer windows (|g| - k + 1) unless its
 * dictionary is bound with PDP_DICT_LONG_GENES; longer genes are rejected with
 * PDP_E_LIMIT in the device status.  Every multiplicity and every sum of
 * minima then fits in 16 bits, which the default pair path relies on. */
#define PDP_MAX_WINDOWS 65535u
/* pdp_dict_bind flags.  PDP_DICT_LONG_GENES: genes may have up to
 * PDP_MAX_WINDOWS_LONG windows.  Multiplicities and sums of minima (Eq.
 * kmer_multiplicity, Eq. jaccard_k) are then carried in 32 bits: every task
 * that names such a dictionary takes the long-gene path, which computes each
 * best-hit row on its own from the row gene's multiplicity vector and the
 * other genome's index (no shared-k-mer records, no column maxima).  It gives
 * the same results as the default path, more slowly; set the flag only for
 * genomes that hold such a gene. */
#define PDP_DICT_LONG_GENES 1u
#define PDP_MAX_WINDOWS_LONG 2147483647u
/* A genome may hold at most this many genes (column indices are 24-bit). */
#define PDP_MAX_GENES 16777215u

enum pdp_code {
    PDP_OK = 0,
    PDP_E_INVAL = -1,     /* null pointer, inconsistent sizes, k differs inside a pair */
    PDP_E_KRANGE = -2,    /* k == 0 or k above the alphabet's largest (PDP_K_MAX, PDP_K_MAX_NT) */
    PDP_E_WORKSPACE = -3, /* workspace or arena smaller than the size functions require */
    PDP_E_CAPACITY = -4,  /* device: an output or scratch array was too small; needed holds the size */
    PDP_E_ALPHABET = -5,  /* device: a letter outside the dictionary's alphabet; where holds its offset.
                             host: an unknown pdp_alphabet value */
    PDP_E_HIP = -6,       /* a HIP runtime call failed */
    PDP_E_BUDGET = -7,    /* serving: a request cannot fit the admission budget */
    PDP_E_LIMIT = -8,     /* a size beyond PDP_MAX_WINDOWS(_LONG) / PDP_MAX_GENES / 2^32 entries */
    PDP_E_UNIMPL = -9
};

/* Device-side status, written by the kernels of one call.  code is the first
 * error raised (0 if none); needed is the size that would have fitted
 * (PDP_E_CAPACITY, the largest over the arrays that overflowed) or the
 * offending size (PDP_E_LIMIT); where is the smallest residue offset
 * (PDP_E_ALPHABET), the gene index (PDP_E_LIMIT, PDP_E_INVAL) or, for
 * PDP_E_CAPACITY, the first array that overflowed in pipeline order
 * (0: shared-k-mer records, 1: best-hit entries, 2: BBH pairs); else
 * UINT64_MAX.  On any error the call's outputs are unspecified.  flags
 * reports how a call ran, not an error: PDP_STATUS_TWO_PASS. */
typedef struct pdp_status {
    int32_t code;
    uint32_t flags;
    uint64_t needed;
    uint64_t where;
} pdp_status;

/* pdp_status.flags: a tile's record region of the one-pass join overflowed, and
 * the two-pass join laid out the records instead (see PDP_PARAM_TWO_PASS). */
#define PDP_STATUS_TWO_PASS 1u

uint32_t pdp_abi_version(void);
const char *pdp_strerror(int32_t code);
const char *pdp_last_error(void);

/* ------------------------------------------------------------- phase (a) */

/* Eq. k_length: k = log_|alphabet| (total), computed in integers.  mode 0
 * rounds up (smallest k with alphabet^k >= total), mode 1 rounds down (largest
 * k with alphabet^k <= total); k is at least 1.  The paper sums the sizes of
 * the genomes; this library's callers pass the total number of residues.
 * Host only.  Errors: PDP_E_INVAL (alphabet < 2, k_out NULL, bad mode). */
int32_t pdp_k_rule(uint64_t total, uint32_t alphabet, int32_t mode, uint32_t *k_out);

/* ------------------------------------------------- k-mer dictionary build */

/* One genome on the device: gene i is residues[gene_off[i] .. gene_off[i+1]),
 * ASCII upper-case letters of the dictionary's alphabet.  gene_off has n_genes+1 entries, gene_off[0] = 0,
 * non-decreasing, gene_off[n_genes] == n_residues (host copy of the last
 * offset, which the library trusts for sizing). */
typedef struct pdp_genome {
    const uint8_t *residues;   /* device, n_residues bytes */
    const uint64_t *gene_off;  /* device, n_genes + 1 */
    uint32_t n_genes;
    uint32_t reserved;
    uint64_t n_residues;
} pdp_genome;

/* The k-mer dictionary of one genome: the multiplicity vector of every gene
 * (Multiplicity vector building phase, Alg. 1) and an inverted index from
 * k-mer to (gene, multiplicity).  A k-mer's code packs its letters, first
 * letter most significant: amino acids 5 bits each with A=0, C=1, ..., Y=19
 * in the order ACDEFGHIKLMNPQRSTVWY; nucleotides 2 bits each with A=0, C=1,
 * G=2, T=3 (the code is then the base-4 value of the k-mer).  Either way codes
 * sort like the k-mer strings.  The index is split into buckets by the
 * leading `lead` letters: min(k, 4) amino acids (20^lead buckets, the leading
 * letters read as a base-20 number) or min(k, 9) nucleotides (4^lead buckets,
 * the leading 2*lead bits of the code).
 * All arrays are device memory carved by pdp_dict_bind from one arena.
 * The host fields are set by pdp_dict_bind and must not be changed. */
typedef struct pdp_dict {
    uint32_t n_genes;
    uint32_t k;
    uint64_t capacity;    /* entries every per-entry array can hold (>= total windows) */
    uint32_t n_buckets;   /* index directory size: 20^lead or 4^lead leading-letter buckets */
    uint32_t key_shift;   /* gene bits of ix_key; 0: this dictionary has no packed keys */
    uint32_t alphabet;    /* pdp_alphabet */
    uint32_t lead;        /* leading letters that name a k-mer's bucket */
    uint32_t flags;       /* PDP_DICT_* given to pdp_dict_bind */
    uint32_t reserved;
    uint32_t *nwin;       /* [n_genes] windows per gene, max(0, |g|-k+1) */
    uint32_t *mv_ptr;     /* [n_genes+1] CSR offsets; mv_ptr[n_genes] = entries E */
    uint64_t *mv_code;    /* [capacity] codes, strictly ascending inside a gene */
    uint32_t *mv_cnt;     /* [capacity] multiplicity of each code in its gene */
    uint32_t *ix_dir;     /* [n_buckets+1] first index entry of each bucket */
    uint64_t *ix_code;    /* [capacity] all entries ordered by (code, gene) */
    uint32_t *ix_gene;    /* [capacity] gene of each index entry */
    uint32_t *ix_cnt;     /* [capacity] multiplicity of the code in that gene */
    uint32_t *ix_key;     /* [capacity] when key_shift > 0: (tail << key_shift) | gene per index
                             entry, where tail is the code without its leading `lead` letters
                             (those are the entry's bucket) and key_shift is the bit length of
                             n_genes - 1 (at least 1); packed when bits*(k - lead) + key_shift
                             <= 32 (bits = 5 or 2 per letter).  Within a bucket the keys ascend
                             like (code, gene). */
    pdp_status *status;   /* device status of the last pdp_dict_build */
} pdp_dict;

/* Bytes of the device arena that pdp_dict_bind carves, and of the scratch
 * workspace that pdp_dict_build needs, for a genome of n_genes genes and
 * n_residues letters over the given pdp_alphabet.  Host only.  Errors:
 * PDP_E_ALPHABET (unknown alphabet), PDP_E_KRANGE, PDP_E_LIMIT
 * (n_genes > PDP_MAX_GENES or n_residues >= 2^32), PDP_E_INVAL. */
int32_t pdp_dict_size(uint32_t n_genes, uint64_t n_residues, uint32_t k, uint32_t alphabet,
                      uint64_t *arena_bytes, uint64_t *ws_bytes);

/* Points the arrays of *out into a caller-allocated device arena (256-byte
 * aligned, at least pdp_dict_size's arena_bytes).  flags: 0 or
 * PDP_DICT_LONG_GENES.  Enqueues nothing.  Errors: PDP_E_INVAL (also unknown
 * flags), PDP_E_WORKSPACE (arena too small), as pdp_dict_size. */
int32_t pdp_dict_bind(void *arena, uint64_t arena_bytes, uint32_t n_genes, uint64_t n_residues,
                      uint32_t k, uint32_t alphabet, uint32_t flags, pdp_dict *out);

/* Builds the dictionary of genome g into d (bound with the same n_genes,
 * n_residues, k and alphabet).  ws is device scratch of pdp_dict_size's ws_bytes.
 * Gene i keeps index i.  Device errors (in d->status): PDP_E_ALPHABET,
 * PDP_E_LIMIT (a gene with more than PDP_MAX_WINDOWS windows, or
 * PDP_MAX_WINDOWS_LONG with PDP_DICT_LONG_GENES; where = the gene).
 * Errors: PDP_E_INVAL (sizes differ from the bind), PDP_E_WORKSPACE, PDP_E_HIP. */
int32_t pdp_dict_build(const pdp_genome *g, pdp_dict *d, void *ws, uint64_t ws_bytes, void *stream);

/* Builds n dictionaries in one set of launches (the kernels number the genes
 * and buckets of all genomes consecutively), so the launch count does not grow
 * with n.  genomes[i] goes into *dicts[i]; each dictionary keeps its own k and
 * status.  Enqueues only kernels (the per-genome descriptors travel as kernel
 * arguments), so it can be captured in a HIP graph.  ws: device scratch of
 * pdp_dict_build_many_ws_size bytes.  Errors as pdp_dict_build, plus
 * PDP_E_LIMIT when the genes or buckets of all genomes pass 2^32 - 1. */
int32_t pdp_dict_build_many_ws_size(const pdp_genome *genomes, pdp_dict *const *dicts, uint32_t n,
                                    uint64_t *ws_bytes);
int32_t pdp_dict_build_many(const pdp_genome *genomes, pdp_dict *const *dicts, uint32_t n, void *ws,
                            uint64_t ws_bytes, void *stream);

/* ------------------------------------------------------- best hits, BBH */

/* Best hits in CSR form (the jagged array A_ij of Alg. 2): row r's hits are
 * col[ptr[r] .. ptr[r+1]) in ascending column order; num is the sum of minima
 * and den the sum of maxima of Eq. jaccard_k for that gene pair, so J =
 * num/den exactly.  A row is empty exactly when its gene shares no k-mer with
 * the other genome (a best hit needs a maximum above zero).  All device. */
typedef struct pdp_bh_out {
    uint32_t n_rows;      /* rows the ptr array covers */
    uint32_t reserved;
    uint64_t capacity;    /* entries col/num/den can hold */
    uint32_t *ptr;        /* [n_rows+1] */
    uint32_t *col;        /* [capacity] */
    uint32_t *num;        /* [capacity] */
    uint32_t *den;        /* [capacity] */
} pdp_bh_out;

/* Bidirectional best hits (Eq. bidirectional_best_hit): pairs (a[i], b[i])
 * in ascending (a, b) order with their num/den; ptr is a CSR over the genes
 * of the first genome (pairs of gene a are ptr[a] .. ptr[a+1]).  All device. */
typedef struct pdp_bbh_out {
    uint32_t n_rows;
    uint32_t reserved;
    uint64_t capacity;
    uint32_t *ptr;        /* [n_rows+1] */
    uint32_t *a;          /* [capacity] */
    uint32_t *b;          /* [capacity] */
    uint32_t *num;        /* [capacity] */
    uint32_t *den;        /* [capacity] */
} pdp_bbh_out;

/* Tuning knobs; zero means "choose automatically". */
typedef struct pdp_params {
    uint64_t inc_capacity;   /* shared-k-mer records the scratch can hold, below 2^32: one per shared
                                (k-mer, gene a, gene b) and requested direction (0: from the dictionary sizes) */
    uint32_t tile_rows;      /* query genes per accumulation tile, 1..256, rounded down to a power of two
                                (0: 64; raised when a task would have more than 1024 tiles) */
    uint32_t join_entries;   /* index entries of the larger genome per join sub-range (1..1024) */
    uint32_t lds_budget;     /* LDS bytes of a tile work-group, at most 156 KiB (0 and anything below
                                32 KiB: 32 KiB, the sorted path's 4096 records); more lets a tile whose
                                records overflow the sort sum more rows per dense pass */
    uint32_t flags;          /* PDP_PARAM_* */
    /* Candidate filters; a zero denominator switches a filter off (the default).
     * Eq. length_threshold: genes a, b are compared only if |a| >= theta |b| and
     * |b| >= theta |a| (theta = theta_num / theta_den <= 1; lengths in residues).
     * Eq. directional_jaccard: only if p(a -> b) >= tau and p(b -> a) >= tau,
     * where p(a -> b) = occurrences in a of the k-mers a shares with b, over
     * |a| - k + 1.  A pair that fails is no best-hit candidate; a row without
     * candidates has no best hit.  Both tests are exact integer comparisons. */
    uint32_t theta_num, theta_den;
    uint32_t tau_num, tau_den;
} pdp_params;
/* The join and the first tile pass run as persistent kernels: a grid sized to
 * the device pulls work items from a counter (largest tasks first) instead of
 * one work-group per item. */
#define PDP_PARAM_PERSISTENT 1u
/* Column maxima (Alg. 3: a gene of the second genome takes as best hits the
 * rows at the maximum of its column of S): for a task that asks for both
 * directions, the best hits of one genome's genes come from the column maxima
 * of the similarities computed for the other's (the genome with fewer k-mer
 * entries, the join's query side), so the join emits shared-k-mer records for
 * one direction only.  Results are identical to the default.  The column
 * candidates share the record capacity (PDP_E_CAPACITY with where = 0). */
#define PDP_PARAM_COLMAX 2u
/* The shared-k-mer join in two passes (count, then write) instead of one.  By
 * default one pass searches every query entry once and writes each record into
 * its tile's region, whose size the plan derives from the record capacity; when
 * a region overflows, the two passes run after it and lay the records out
 * exactly, and the regions in the workspace are refitted to that launch's
 * record counts (with the spare capacity spread in proportion), so the next
 * launch on the same dictionaries fits in one pass.  pdp_plan_upload restores
 * the estimated regions.  Results are identical either way. */
#define PDP_PARAM_TWO_PASS 4u

/* One unit of work: genomes a and b (same k and alphabet).  flags select the outputs. */
#define PDP_TASK_AB 1u   /* best hits of a's genes in b */
#define PDP_TASK_BA 2u   /* best hits of b's genes in a */
#define PDP_TASK_BBH 4u  /* bidirectional best hits of (a, b); needs AB and BA */
typedef struct pdp_task {
    const pdp_dict *a;
    const pdp_dict *b;
    uint32_t flags;
    uint32_t reserved;
} pdp_task;

/* A plan: the host-side schedule of many tasks (join work-groups,
 * accumulation tiles, output row ranges) computed once from host-known sizes,
 * plus the workspace layout.  Opaque; host memory owned by the library. */
typedef struct pdp_plan pdp_plan;

typedef struct pdp_plan_info {
    uint64_t ws_bytes;        /* device workspace pdp_plan_run needs */
    uint64_t inc_capacity;    /* shared-k-mer records the workspace holds */
    uint32_t bh_rows;         /* rows of the combined best-hit output */
    uint32_t bbh_rows;        /* rows of the combined BBH output */
    uint32_t n_tasks;
    uint32_t join_groups;     /* join items (bucket ranges) per run */
    uint32_t tiles;           /* accumulation tiles per run */
    uint32_t tile_lds;        /* LDS bytes per accumulation tile */
    uint32_t long_rows;       /* best-hit rows of the tasks that take the long-gene path */
    uint32_t reserved;
} pdp_plan_info;

/* Builds a plan for n_tasks tasks.  Best-hit rows of the combined output are
 * laid out task by task: first a's genes (if AB), then b's genes (if BA); BBH
 * rows are a's genes of every task with PDP_TASK_BBH, task by task.  Inside a
 * task the join searches the entries of the genome with fewer k-mer entries
 * (by dictionary capacity) in the other's index, whichever the caller named
 * first; the outputs keep the caller's orientation.
 * pdp_plan_rows gives each task's first row in both outputs.  A task that
 * names a dictionary bound with PDP_DICT_LONG_GENES has no join items and no
 * tiles: its rows take the long-gene path (and PDP_PARAM_COLMAX does not apply
 * to it), with the same output layout.  Host only.
 * Errors: PDP_E_INVAL (null, k or alphabet mismatch, BBH without AB|BA), PDP_E_LIMIT. */
int32_t pdp_plan_create(const pdp_task *tasks, uint32_t n_tasks, const pdp_params *params, pdp_plan **out);
int32_t pdp_plan_info_get(const pdp_plan *plan, pdp_plan_info *info);
/* For task t: first row of its AB rows, of its BA rows (in bh), and of its BBH
 * rows (in bbh); UINT32_MAX where the task has no such output. */
int32_t pdp_plan_rows(const pdp_plan *plan, uint32_t t, uint32_t *ab_row, uint32_t *ba_row, uint32_t *bbh_row);
void pdp_plan_destroy(pdp_plan *plan);

/* Copies the plan's device tables into ws (once per workspace, or after the
 * workspace was overwritten).  Enqueues host-to-device copies on stream. */
int32_t pdp_plan_upload(const pdp_plan *plan, void *ws, uint64_t ws_bytes, void *stream);

/* Enqueues the whole best-hit path for every task of the plan: shared-k-mer
 * join, LDS accumulation of the sums of minima, best hits with ties, BBH.
 * Enqueues only kernels (no allocation, no host copies, no memset), so it can
 * be captured in a HIP graph.  bh must cover info.bh_rows rows, bbh
 * info.bbh_rows rows (bbh may be NULL if no task asks for BBH).  status is
 * device memory.  Device errors: PDP_E_CAPACITY (needed = required
 * records, best-hit entries or BBH pairs; retry with more).  status.flags
 * reports PDP_STATUS_TWO_PASS when the join's record regions overflowed and
 * the two-pass join ran; the launch then also refits the regions held in ws
 * (see PDP_PARAM_TWO_PASS), so a launch writes the plan's tile table in ws.
 * Errors: PDP_E_INVAL, PDP_E_WORKSPACE, PDP_E_HIP. */
int32_t pdp_plan_launch(const pdp_plan *plan, pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *status,
                        void *ws, uint64_t ws_bytes, void *stream);

/* Kernels of a plan launch, for pdp_plan_timer_start. */
#define PDP_KERNEL_JOIN 0        /* shared-k-mer join: the one-pass kernel (with PDP_PARAM_TWO_PASS: count
                                    pass, scan of the counts, write pass) */
#define PDP_KERNEL_BUCKET 1      /* the scan of the per-tile record totals alone */
#define PDP_KERNEL_TILE_COUNT 2  /* per tile: sort and sum of records, row maxima, tie counts */
#define PDP_KERNEL_TILE_WRITE 3  /* best-hit output (slab copy, rows with many ties) */
#define PDP_KERNEL_BBH 4         /* BBH count and write passes together */
#define PDP_KERNEL_ALL 5         /* the whole launch */
#define PDP_KERNEL_JOIN_BACKUP 6 /* the two-pass join gated behind the one-pass join (empty unless a
                                    region overflowed) and the tiles' record ranges */

/* Gene families from the BBH of a launched plan (phase (c): families are
 * extracted from the network the bidirectional best hits form; the paper
 * specifies no refinement, so a family here is a connected component of that
 * network, over all genes of all genomes).  Node ids are global gene ids
 * chosen by the caller: node_a[t] / node_b[t] (device, one per task in the
 * caller's task order) are the ids of gene 0 of task t's genomes a and b, so
 * gene g of a is node node_a[t] + g.  labels (device, n_nodes) receives, for
 * every node, the smallest node id of its family (a node without BBH pairs is
 * its own family).  bbh must hold the BBH output of the plan's last launch; ws
 * is that launch's workspace (its task tables are read).  Enqueues kernels only.
 * Device errors: PDP_E_INVAL (a pair names a node >= n_nodes; where = BBH row).
 * Errors: PDP_E_INVAL, PDP_E_WORKSPACE, PDP_E_HIP. */
int32_t pdp_plan_families(const pdp_plan *plan, const pdp_bbh_out *bbh, const uint32_t *node_a,
                          const uint32_t *node_b, uint32_t n_nodes, uint32_t *labels, pdp_status *status,
                          void *ws, uint64_t ws_bytes, void *stream);

/* Measurement hook: from now on every pdp_plan_launch of this plan records a
 * pair of HIP events (owned by the plan) on its stream around the given
 * kernel, for at most max_launches launches.  pdp_plan_timer_read waits for
 * the recorded events and returns the summed milliseconds and the number of
 * timed launches; pdp_plan_timer_stop releases the events.  Host only apart
 * from the event records.  Errors: PDP_E_INVAL, PDP_E_HIP. */
int32_t pdp_plan_timer_start(pdp_plan *plan, int32_t kernel, uint32_t max_launches);
int32_t pdp_plan_timer_read(pdp_plan *plan, double *total_ms, uint32_t *launches);
int32_t pdp_plan_timer_stop(pdp_plan *plan);

/* Upload + launch. */
int32_t pdp_plan_run(const pdp_plan *plan, pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *status,
                     void *ws, uint64_t ws_bytes, void *stream);

/* ----------------------------------------------- batching: graphs, tuning */

/* HIP graphs of library work (many instances and genome pairs replayed as one
 * launch): pdp_capture_begin starts capturing everything enqueued on stream
 * (thread-local capture mode; not the NULL stream), pdp_capture_end stops and
 * instantiates it, pdp_graph_launch replays it on any stream.  Capture only
 * calls that enqueue kernels (pdp_dict_build_many, pdp_plan_launch): upload
 * plans before capturing.  A graph refers to the workspaces and outputs it was
 * captured with; they must stay allocated while it is used.
 * Errors: PDP_E_INVAL, PDP_E_HIP. */
typedef struct pdp_graph pdp_graph;
int32_t pdp_capture_begin(void *stream);
int32_t pdp_capture_end(void *stream, pdp_graph **out);
int32_t pdp_graph_launch(pdp_graph *graph, void *stream);
void pdp_graph_destroy(pdp_graph *graph);

/* Autotuner for tile shapes and work splits: each candidate pdp_params is
 * planned for the given tasks, run once to warm up and then reps times between
 * two HIP events; the fastest candidate whose runs end with a clean status is
 * returned.  candidates NULL: a built-in grid of tile heights (32, 64, 128
 * rows), join sub-range sizes (256, 512, 768, 1024 entries), persistent on/off and
 * column maxima on/off (PDP_PARAM_COLMAX).  bh/bbh/status as
 * for pdp_plan_launch (their rows do not depend on the parameters); ws of
 * pdp_autotune_ws_size bytes.  Synchronises the stream.
 * Errors: PDP_E_INVAL, PDP_E_HIP, PDP_E_LIMIT (no candidate ran cleanly). */
typedef struct pdp_tune_result {
    pdp_params best;
    double best_ms;   /* average milliseconds per launch of the best candidate */
    double first_ms;  /* the same for the first candidate that ran */
    uint32_t tried;   /* candidates that ran cleanly */
    uint32_t reserved;
} pdp_tune_result;
int32_t pdp_autotune_ws_size(const pdp_task *tasks, uint32_t n_tasks, const pdp_params *candidates,
                             uint32_t n_candidates, uint64_t *ws_bytes);
int32_t pdp_autotune(const pdp_task *tasks, uint32_t n_tasks, const pdp_params *candidates, uint32_t n_candidates,
                     uint32_t reps, pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *status, void *ws,
                     uint64_t ws_bytes, void *stream, pdp_tune_result *result);

/* ----------------------------------------------------------------- serving */

/* A request loop: genomes arrive one at a time and each is compared (best
 * hits both ways and BBH, Eqs. best_hit and bidirectional_best_hit) with every
 * resident genome, whose dictionaries stay on the device.  A worker thread
 * admits waiting requests in arrival order whenever a slot (one HIP stream) is
 * free and the request's device footprint (its genome, dictionary, scratch and
 * outputs) fits the budget, carved from the caller's arena; admitted requests
 * run concurrently on their slots, and a finished request's slot and memory
 * pass at once to the next waiting one.  Results are copied to host memory
 * owned by the server.  A request's results do not depend on which other
 * requests share the device. */
typedef struct pdp_server pdp_server;

typedef struct pdp_server_config {
    uint64_t budget_bytes;  /* device bytes for requests in flight (at most arena_bytes) */
    uint32_t slots;         /* requests in flight at most, 1..64 */
    uint32_t k;             /* k of every resident and request */
    uint32_t alphabet;      /* pdp_alphabet of every resident and request */
    uint32_t reserved;
    pdp_params params;      /* pair-path parameters (inc_capacity is managed per request) */
} pdp_server_config;

/* A finished request.  Times are microseconds since pdp_server_create. */
typedef struct pdp_request_done {
    uint64_t tag;
    int32_t code;        /* PDP_OK, or the request's error (PDP_E_BUDGET: never fits the budget) */
    uint32_t n_genes;
    uint32_t attempts;   /* runs, more than 1 after a capacity error grew its buffers */
    uint32_t flags;      /* pdp_status.flags of its last run (PDP_STATUS_TWO_PASS) */
    double submit_us, admit_us, done_us;
    uint64_t bh_entries, bbh_pairs;
    /* Device time of the request's last run, in milliseconds between HIP events on its slot's
     * stream: the copy of its genome to the device, its dictionary build, the plan launch
     * against every resident (join, tiles, best hits, BBH), and the copies of its results to
     * host memory (both steps: statuses and row pointers, then the used entries; the worker's
     * turnaround between the two is not included). */
    float h2d_ms, build_ms, pairs_ms, d2h_ms;
} pdp_request_done;

/* A finished request's results (host memory owned by the server, valid until
 * pdp_server_release).  Task r is (request, resident r): its rows start at
 * ab_row[r] (request genes in resident r) and ba_row[r] (resident r's genes
 * in the request) of the best-hit CSR, and at bbh_row[r] of the BBH CSR. */
typedef struct pdp_request_result {
    int32_t code;
    uint32_t n_residents;
    pdp_status status;
    uint32_t bh_rows, bbh_rows;
    const uint32_t *ab_row, *ba_row, *bbh_row;                 /* [n_residents] */
    const uint32_t *bh_ptr, *bh_col, *bh_num, *bh_den;         /* CSR */
    const uint32_t *bbh_ptr, *bbh_a, *bbh_b, *bbh_num, *bbh_den;
} pdp_request_result;

typedef struct pdp_server_stats {
    uint64_t admitted, completed, retries, pending;
    uint64_t budget_bytes, used_bytes, peak_used_bytes;
    uint32_t inflight, peak_inflight;
} pdp_server_stats;

/* residents: dictionaries built with cfg->k and cfg->alphabet, borrowed until pdp_server_destroy.
 * arena: caller device memory (256-byte aligned) of which budget_bytes are used.
 * Errors: PDP_E_INVAL, PDP_E_WORKSPACE, PDP_E_HIP. */
int32_t pdp_server_create(const pdp_server_config *cfg, const pdp_dict *const *residents, uint32_t n_residents,
                          void *arena, uint64_t arena_bytes, pdp_server **out);
/* Queues one genome (host arrays, copied before return); tag must be unused.
 * A genome with a gene past PDP_MAX_WINDOWS windows gets a dictionary bound
 * with PDP_DICT_LONG_GENES, so its pairs take the long-gene path. */
int32_t pdp_server_submit(pdp_server *server, const uint8_t *residues, const uint64_t *gene_off, uint32_t n_genes,
                          uint64_t tag);
/* Up to max finished requests not yet reported, oldest first; waits up to
 * wait_us for one if none is ready.  Returns PDP_E_HIP after a device error. */
int32_t pdp_server_poll(pdp_server *server, pdp_request_done *done, uint32_t max, uint32_t *n_done, uint32_t wait_us);
int32_t pdp_server_fetch(pdp_server *server, uint64_t tag, pdp_request_result *out);
int32_t pdp_server_release(pdp_server *server, uint64_t tag);
int32_t pdp_server_stats_get(pdp_server *server, pdp_server_stats *out);
/* Waits for requests in flight, then frees the server (not the arena). */
void pdp_server_destroy(pdp_server *server);

/* Convenience form of one task: best hits of every gene of q in t (Eq.
 * best_hit, Alg. 2); out->n_rows must equal q->n_genes.  The workspace size
 * comes from pdp_bh_ws_size.  The plan tables are uploaded and the stream is
 * synchronised once before the kernels are enqueued, so this call is not for
 * graph capture (use a plan for that). */
int32_t pdp_bh_ws_size(const pdp_dict *q, const pdp_dict *t, const pdp_params *params, uint64_t *ws_bytes);
int32_t pdp_bh(const pdp_dict *q, const pdp_dict *t, const pdp_params *params, pdp_bh_out *out,
               pdp_status *status, void *ws, uint64_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, hosts that forbid hipMalloc): pdp_bh with its scratch in a
 * fixed device array of the library instead of a caller workspace.  Arguments,
 * results and device errors as pdp_bh.  The array holds PDP_NOALLOC_SCRATCH_BYTES
 * on every device the library runs on, from the library's load to the end of the
 * process; a genome pair whose pdp_bh_ws_size exceeds it is rejected with
 * PDP_E_WORKSPACE before anything is enqueued.  The call allocates no device
 * memory.  All calls on one device share that device's array: calls that overlap
 * on one device (concurrent streams or threads) race and give undefined results;
 * calls one after another are independent of each other.  Synchronises the
 * stream once, as pdp_bh does.
 * Errors: PDP_E_INVAL, PDP_E_WORKSPACE, PDP_E_LIMIT, PDP_E_HIP, as pdp_bh. */
#define PDP_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t pdp_bh_noalloc(const pdp_dict *q, const pdp_dict *t, const pdp_params *params, pdp_bh_out *out,
                       pdp_status *status, void *stream);

/* BBH from two best-hit outputs (Alg. 3's cross-check of A_ij against A_ji):
 * ab has one row per gene of genome i, ba one row per gene of genome j.
 * out->n_rows must equal ab->n_rows.  Device errors: PDP_E_CAPACITY.
 * ws: device scratch of pdp_bbh_ws_size bytes. */
int32_t pdp_bbh_ws_size(uint32_t n_rows, uint64_t *ws_bytes);
int32_t pdp_bbh(const pdp_bh_out *ab, const pdp_bh_out *ba, pdp_bbh_out *out, pdp_status *status,
                void *ws, uint64_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PDP_H */
