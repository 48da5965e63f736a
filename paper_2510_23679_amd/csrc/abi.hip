// C-ABI entry points: argument validation, planning, workspace layout and
// error reporting around the gfx950 kernels.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace pdp;

namespace {

thread_local char g_last_error[512] = "";

int32_t fail(int32_t code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t fail(int32_t code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

int32_t hip_fail(hipError_t e, const char *what) {
    return fail(PDP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int32_t ok() {
    g_last_error[0] = '\0';
    return PDP_OK;
}

}  // namespace

int32_t pdp::api_fail(int32_t code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

struct pdp_plan {
    std::vector<DevTask> tasks;
    std::vector<DevTile> tiles;
    std::vector<DevItem> items;
    std::vector<DevLongSeg> long_segs;  // long-gene path: row segments by first row
    std::vector<uint32_t> ab_row, ba_row, bbh_row;
    std::vector<uint32_t> order;  // order[t]: position of caller task t in the task table
    PlanShape shape;
    uint64_t ws_bytes;
    bool persistent = false;
    mutable bool device_ready = false;  // persistent grids and LDS limit set up on the device
    mutable uint32_t join_grid = 0, tile_grid = 0, fallback_grid = 0;
    // measurement hook: event pairs owned by the plan, one per timed launch
    mutable int32_t timer_kernel = -1;
    mutable uint32_t timer_used = 0;
    mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> timer_events;

    void timer_release() const {
        for (auto &e : timer_events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        timer_events.clear();
        timer_kernel = -1;
        timer_used = 0;
    }
    ~pdp_plan() { timer_release(); }
};

extern "C" {

uint32_t pdp_abi_version(void) { return PDP_ABI_VERSION; }

const char *pdp_strerror(int32_t code) {
    switch (code) {
    case PDP_OK: return "ok";
    case PDP_E_INVAL: return "invalid argument";
    case PDP_E_KRANGE: return "k out of range for the alphabet (amino acids 1..12, nucleotides 1..31)";
    case PDP_E_WORKSPACE: return "workspace or arena too small";
    case PDP_E_CAPACITY: return "output or scratch capacity too small";
    case PDP_E_ALPHABET: return "letter outside the dictionary's alphabet, or unknown alphabet";
    case PDP_E_HIP: return "HIP runtime error";
    case PDP_E_BUDGET: return "request exceeds the admission budget";
    case PDP_E_LIMIT: return "size beyond a documented limit";
    case PDP_E_UNIMPL: return "not implemented";
    default: return "unknown error";
    }
}

const char *pdp_last_error(void) { return g_last_error; }

int32_t pdp_k_rule(uint64_t total, uint32_t alphabet, int32_t mode, uint32_t *k_out) {
    if (!k_out || alphabet < 2 || (mode != 0 && mode != 1)) return fail(PDP_E_INVAL, "pdp_k_rule: bad argument");
    // Powers are compared in 128-bit integers so no power near 2^64 overflows.
    unsigned __int128 p = 1;
    uint32_t k = 0;
    if (mode == 0) {
        while (p < total) {
            p *= alphabet;
            ++k;
        }
    } else {
        while (p * alphabet <= total) {
            p *= alphabet;
            ++k;
        }
    }
    *k_out = k < 1 ? 1 : k;
    return ok();
}

// ------------------------------------------------------------ dictionary

static int32_t dict_check(uint32_t n_genes, uint64_t n_residues, uint32_t k, uint32_t alphabet) {
    if (!alpha_known(alphabet)) return fail(PDP_E_ALPHABET, "unknown alphabet %u", alphabet);
    const uint32_t kmax = alpha_spec(alphabet).k_max;
    if (k == 0 || k > kmax) return fail(PDP_E_KRANGE, "k = %u outside 1..%u for this alphabet", k, kmax);
    if (n_genes > PDP_MAX_GENES) return fail(PDP_E_LIMIT, "%u genes exceed %u", n_genes, PDP_MAX_GENES);
    if (n_residues >= (1ull << 32)) return fail(PDP_E_LIMIT, "%llu residues exceed 2^32 - 1", (unsigned long long)n_residues);
    return PDP_OK;
}

static uint64_t dict_arena_bytes(uint32_t n_genes, uint64_t n_residues, uint32_t k, uint32_t alphabet) {
    const uint64_t A = 256, cap = n_residues + 1, nb = n_buckets_for(k, alphabet);
    uint64_t s = 0;
    s += align_up(4 * (uint64_t(n_genes) + 1), A);  // nwin
    s += align_up(4 * (uint64_t(n_genes) + 1), A);  // mv_ptr
    s += align_up(8 * cap, A);                      // mv_code
    s += align_up(4 * cap, A);                      // mv_cnt
    s += align_up(4 * (nb + 1), A);                 // ix_dir
    s += align_up(8 * cap, A);                      // ix_code
    s += align_up(4 * cap, A);                      // ix_gene
    s += align_up(4 * cap, A);                      // ix_cnt
    s += align_up(4 * cap, A);                      // ix_key
    s += align_up(sizeof(pdp_status), A);           // status
    return s;
}

int32_t pdp_dict_size(uint32_t n_genes, uint64_t n_residues, uint32_t k, uint32_t alphabet, uint64_t *arena_bytes,
                      uint64_t *ws_bytes) {
    int32_t rc = dict_check(n_genes, n_residues, k, alphabet);
    if (rc) return rc;
    if (arena_bytes) *arena_bytes = dict_arena_bytes(n_genes, n_residues, k, alphabet);
    if (ws_bytes) {
        *ws_bytes = build_ws_bytes(single_build_shape(n_genes, n_residues, k, alphabet));
    }
    return ok();
}

int32_t pdp_dict_bind(void *arena, uint64_t arena_bytes, uint32_t n_genes, uint64_t n_residues, uint32_t k,
                      uint32_t alphabet, uint32_t flags, pdp_dict *out) {
    if (!arena || !out) return fail(PDP_E_INVAL, "pdp_dict_bind: null pointer");
    if (flags & ~PDP_DICT_LONG_GENES) return fail(PDP_E_INVAL, "pdp_dict_bind: unknown flags 0x%x", flags);
    if (reinterpret_cast<uintptr_t>(arena) % 256) return fail(PDP_E_INVAL, "pdp_dict_bind: arena not 256-byte aligned");
    int32_t rc = dict_check(n_genes, n_residues, k, alphabet);
    if (rc) return rc;
    const uint64_t need = dict_arena_bytes(n_genes, n_residues, k, alphabet);
    if (arena_bytes < need) return fail(PDP_E_WORKSPACE, "arena %llu < %llu bytes", (unsigned long long)arena_bytes, (unsigned long long)need);
    const uint64_t A = 256, cap = n_residues + 1, nb = n_buckets_for(k, alphabet);
    char *p = static_cast<char *>(arena);
    auto take = [&](uint64_t bytes) {
        char *q = p;
        p += align_up(bytes, A);
        return q;
    };
    pdp_dict d;
    std::memset(&d, 0, sizeof(d));
    d.n_genes = n_genes;
    d.k = k;
    d.capacity = cap;
    d.n_buckets = static_cast<uint32_t>(nb);
    d.nwin = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(n_genes) + 1)));
    d.mv_ptr = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(n_genes) + 1)));
    d.mv_code = reinterpret_cast<uint64_t *>(take(8 * cap));
    d.mv_cnt = reinterpret_cast<uint32_t *>(take(4 * cap));
    d.ix_dir = reinterpret_cast<uint32_t *>(take(4 * (nb + 1)));
    d.ix_code = reinterpret_cast<uint64_t *>(take(8 * cap));
    d.ix_gene = reinterpret_cast<uint32_t *>(take(4 * cap));
    d.ix_cnt = reinterpret_cast<uint32_t *>(take(4 * cap));
    d.ix_key = reinterpret_cast<uint32_t *>(take(4 * cap));
    d.key_shift = key_shift_for(n_genes, k, alphabet);
    d.alphabet = alphabet;
    d.lead = lead_letters(k, alphabet);
    d.flags = flags;
    d.status = reinterpret_cast<pdp_status *>(take(sizeof(pdp_status)));
    *out = d;
    return ok();
}

static int32_t build_check(const pdp_genome *genomes, pdp_dict *const *dicts, uint32_t n) {
    if (n == 0 || !genomes || !dicts) return fail(PDP_E_INVAL, "dictionary build: no genomes");
    uint64_t genes = 0, buckets = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const pdp_genome *g = &genomes[i];
        const pdp_dict *d = dicts[i];
        if (!d) return fail(PDP_E_INVAL, "dictionary %u is null", i);
        if (!g->gene_off || (g->n_residues && !g->residues)) return fail(PDP_E_INVAL, "genome %u: null arrays", i);
        int32_t rc = dict_check(g->n_genes, g->n_residues, d->k, d->alphabet);
        if (!rc && (d->lead != lead_letters(d->k, d->alphabet) || d->n_buckets != n_buckets_for(d->k, d->alphabet) ||
                    (d->flags & ~PDP_DICT_LONG_GENES)))
            rc = fail(PDP_E_INVAL, "dictionary %u: fields changed since pdp_dict_bind", i);
        if (rc) return rc;
        if (g->n_genes != d->n_genes || g->n_residues + 1 > d->capacity)
            return fail(PDP_E_INVAL, "genome %u (%u genes, %llu residues) does not match its dictionary (%u genes, capacity %llu)",
                        i, g->n_genes, (unsigned long long)g->n_residues, d->n_genes, (unsigned long long)d->capacity);
        genes += g->n_genes;
        buckets += d->n_buckets;
    }
    if (genes >= UINT32_MAX || buckets >= UINT32_MAX) return fail(PDP_E_LIMIT, "build too large for 32-bit indices");
    return PDP_OK;
}

int32_t pdp_dict_build_many_ws_size(const pdp_genome *genomes, pdp_dict *const *dicts, uint32_t n, uint64_t *ws_bytes) {
    if (!ws_bytes) return fail(PDP_E_INVAL, "pdp_dict_build_many_ws_size: null output");
    int32_t rc = build_check(genomes, dicts, n);
    if (rc) return rc;
    *ws_bytes = build_ws_bytes(build_shape(genomes, dicts, n));
    return ok();
}

int32_t pdp_dict_build_many(const pdp_genome *genomes, pdp_dict *const *dicts, uint32_t n, void *ws, uint64_t ws_bytes,
                            void *stream) {
    if (!ws) return fail(PDP_E_INVAL, "dictionary build: null workspace");
    int32_t rc = build_check(genomes, dicts, n);
    if (rc) return rc;
    const uint64_t need = build_ws_bytes(build_shape(genomes, dicts, n));
    if (ws_bytes < need) return fail(PDP_E_WORKSPACE, "workspace %llu < %llu bytes", (unsigned long long)ws_bytes, (unsigned long long)need);
    hipError_t e = launch_dict_build_many(genomes, dicts, n, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dictionary build");
    return ok();
}

int32_t pdp_dict_build(const pdp_genome *g, pdp_dict *d, void *ws, uint64_t ws_bytes, void *stream) {
    if (!g || !d) return fail(PDP_E_INVAL, "pdp_dict_build: null pointer");
    return pdp_dict_build_many(g, &d, 1, ws, ws_bytes, stream);
}

// ------------------------------------------------------------------ plans

static DevDict dev_dict(const pdp_dict *d) {
    DevDict x;
    x.ix_code = d->ix_code;
    x.ix_gene = d->ix_gene;
    x.ix_cnt = d->ix_cnt;
    x.ix_dir = d->ix_dir;
    x.nwin = d->nwin;
    x.ix_key = d->ix_key;
    x.mv_ptr = d->mv_ptr;
    x.mv_code = d->mv_code;
    x.mv_cnt = d->mv_cnt;
    x.n_genes = d->n_genes;
    x.n_buckets = d->n_buckets;
    x.k = d->k;
    x.key_shift = d->key_shift;
    x.bits = alpha_spec(d->alphabet).bits;
    x.lead = d->lead;
    return x;
}

int32_t pdp_plan_create(const pdp_task *tasks, uint32_t n_tasks, const pdp_params *params, pdp_plan **out) {
    if (!out || (n_tasks && !tasks)) return fail(PDP_E_INVAL, "pdp_plan_create: null pointer");
    *out = nullptr;
    if (n_tasks == 0) return fail(PDP_E_INVAL, "pdp_plan_create: no tasks");
    pdp_params prm;
    std::memset(&prm, 0, sizeof(prm));
    if (params) prm = *params;
    const uint32_t lds_budget = prm.lds_budget ? prm.lds_budget : kDefaultLdsBudget;
    const uint32_t join_entries = prm.join_entries ? prm.join_entries : kJoinLdsCap / 2;  // ~2x headroom to the stage
    if (lds_budget > kMaxTileLds) return fail(PDP_E_INVAL, "lds_budget above %u bytes", kMaxTileLds);
    if (join_entries > kJoinLdsCap) return fail(PDP_E_INVAL, "join_entries above %u", kJoinLdsCap);
    if (prm.tile_rows > kTileMaxRows) return fail(PDP_E_INVAL, "tile_rows above %u", kTileMaxRows);
    if (prm.inc_capacity > UINT32_MAX) return fail(PDP_E_LIMIT, "record capacity above 2^32 - 1");
    uint32_t base_shift = kDefaultTileShift;  // tile rows: the largest power of two <= tile_rows
    if (prm.tile_rows)
        for (base_shift = 0; (2u << base_shift) <= prm.tile_rows; ++base_shift) {
        }
    if (prm.flags & ~(PDP_PARAM_PERSISTENT | PDP_PARAM_COLMAX | PDP_PARAM_TWO_PASS))
        return fail(PDP_E_INVAL, "unknown parameter flags 0x%x", prm.flags);
    bool any_colmax = false;
    if (prm.theta_den && prm.theta_num > prm.theta_den) return fail(PDP_E_INVAL, "theta above 1");
    const bool filt = prm.theta_den || prm.tau_den;

    pdp_plan *P = new (std::nothrow) pdp_plan();
    if (!P) return fail(PDP_E_INVAL, "out of host memory");
    auto bail = [&](int32_t rc) {
        delete P;
        return rc;
    };
    // Pass 1, in the caller's order: validation, output row layout, tile height per direction.
    uint64_t bh_rows = 0, bbh_rows = 0, rec_est = 0;
    // the sorted and hashed tile paths keep 8 bytes per record (12 with the filters' sums)
    uint32_t tile_lds = std::max<uint32_t>(lds_budget, (filt ? 12 : 8) * kTileCap);
    std::vector<DevTask> caller(n_tasks);
    std::vector<uint64_t> cost(n_tasks);
    std::vector<uint8_t> is_long(n_tasks, 0);  // the task takes the long-gene path
    for (uint32_t t = 0; t < n_tasks; ++t) {
        const pdp_task &tk = tasks[t];
        if (!tk.a || !tk.b) return bail(fail(PDP_E_INVAL, "task %u: null dictionary", t));
        if (tk.a->k != tk.b->k || tk.a->alphabet != tk.b->alphabet || tk.a->lead != tk.b->lead ||
            tk.a->n_buckets != tk.b->n_buckets)
            return bail(fail(PDP_E_INVAL, "task %u: dictionaries built with different k or alphabet (k %u/%u, alphabet %u/%u)",
                             t, tk.a->k, tk.b->k, tk.a->alphabet, tk.b->alphabet));
        uint32_t flags = tk.flags & (PDP_TASK_AB | PDP_TASK_BA | PDP_TASK_BBH);
        if (flags & PDP_TASK_BBH) flags |= PDP_TASK_AB | PDP_TASK_BA;
        if (!flags) return bail(fail(PDP_E_INVAL, "task %u: no output selected", t));
        DevTask &d = caller[t];
        std::memset(&d, 0, sizeof(d));
        const bool long_task = ((tk.a->flags | tk.b->flags) & PDP_DICT_LONG_GENES) != 0;
        is_long[t] = long_task ? 1 : 0;
        // The join searches every entry of its query genome (the task's a) in the other one, so
        // the smaller genome (by entry capacity) takes that side: the task then holds the caller's
        // genomes swapped, with its directions swapped alike (kTaskSwapped); output rows keep the
        // caller's layout.
        const bool swap = !long_task && tk.b->capacity < tk.a->capacity;
        const pdp_dict *qa = swap ? tk.b : tk.a, *qb = swap ? tk.a : tk.b;
        const uint32_t dflags = swap ? (flags & PDP_TASK_BBH) | ((flags & PDP_TASK_AB) ? PDP_TASK_BA : 0u) |
                                           ((flags & PDP_TASK_BA) ? PDP_TASK_AB : 0u)
                                     : flags;
        d.a = dev_dict(qa);
        d.b = dev_dict(qb);
        // column maxima: b's best hits from the AB tiles' columns, records for one direction
        const bool colmax =
            !long_task && (prm.flags & PDP_PARAM_COLMAX) && (flags & PDP_TASK_AB) && (flags & PDP_TASK_BA);
        any_colmax |= colmax;
        d.flags = (colmax ? (dflags & ~PDP_TASK_BA) | kTaskColmax : dflags) | (swap ? kTaskSwapped : 0u);
        d.theta_n = prm.theta_num;
        d.theta_d = prm.theta_den;
        d.tau_n = prm.tau_num;
        d.tau_d = prm.tau_den;
        const uint32_t nb = tk.a->n_buckets;
        const uint64_t e_max = std::max<uint64_t>(std::max(tk.a->capacity, tk.b->capacity), 1);
        // sub-ranges of bpw buckets hold ~join_entries entries of the larger genome; an item
        // takes as many sub-ranges as its directory slice (kJoinDirCap buckets) allows
        // packed keys take half the LDS per staged entry: twice the entries per sub-range
        const bool packed = tk.a->key_shift && tk.b->key_shift;
        uint64_t bpw = uint64_t(join_entries) * (packed ? kJoinLdsCapP / kJoinLdsCap : 1) * nb / e_max;
        bpw = std::min<uint64_t>(std::max<uint64_t>(bpw, 1), std::min<uint64_t>(nb, kJoinDirCap));
        const uint64_t subs = std::max<uint64_t>(1, kJoinDirCap / bpw);
        d.bpw = static_cast<uint32_t>(bpw);
        d.subs = static_cast<uint32_t>(subs);
        d.n_chunks = long_task ? 0u : static_cast<uint32_t>((nb + bpw * subs - 1) / (bpw * subs));
        // output rows in the caller's orientation: a's genes (AB), then b's (BA)
        uint32_t orow[2] = {UINT32_MAX, UINT32_MAX};
        for (uint32_t odir = 0; odir < 2; ++odir) {
            if (!(flags & (1u << odir))) continue;
            orow[odir] = static_cast<uint32_t>(bh_rows);
            bh_rows += (odir == 0 ? tk.a : tk.b)->n_genes;
        }
        uint32_t ndirs = 0;
        for (uint32_t dir = 0; dir < 2; ++dir) {  // the task's own directions from here on
            d.row_base[dir] = orow[swap ? 1 - dir : dir];
            d.tile_shift[dir] = base_shift;
            d.tiles_n[dir] = 0;
            if (!(dflags & (1u << dir))) continue;
            if ((dir == 1 && colmax) || long_task) continue;  // rows in the output, no tiles and no records of their own
            ++ndirs;
            const pdp_dict *R = dir == 0 ? qa : qb;
            const pdp_dict *C = dir == 0 ? qb : qa;
            // a tile whose records overflow the LDS sort is summed densely: the column genome's
            // window counts (16 bits each) and at least one row of packed 16-bit sums plus its
            // touched-word bitmap must fit
            const uint64_t W = (uint64_t(C->n_genes) + 1) / 2;
            const uint64_t dense = 4 * (((W + 3) & ~3ull) + (filt ? 3 : 1) * W + (W + 31) / 32);
            if (dense > kMaxTileLds)
                return bail(fail(PDP_E_LIMIT, "task %u: %u target genes do not fit an LDS tile", t, C->n_genes));
            tile_lds = std::max<uint32_t>(tile_lds, static_cast<uint32_t>(dense));
            // a tile's (row, column) sums share one LDS hash table, and a row meets more
            // columns by chance the more k-mers it has: unless the caller fixed the height,
            // rows of long genes (over 512 letters on average, e.g. nucleotide genes) go 32
            // to a tile instead of 64
            if (!prm.tile_rows && R->n_genes && R->capacity / R->n_genes > 512) d.tile_shift[dir] = kDefaultTileShift - 1;
            d.tiles_n[dir] = static_cast<uint32_t>((uint64_t(R->n_genes) + (1u << d.tile_shift[dir]) - 1) >>
                                                   d.tile_shift[dir]);
        }
        // the join keeps one LDS counter per tile of the task: taller tiles when there are too many
        while (d.tiles_n[0] + d.tiles_n[1] > kJoinTileCap) {
            const bool can0 = d.tiles_n[0] && d.tile_shift[0] < 8, can1 = d.tiles_n[1] && d.tile_shift[1] < 8;
            if (!can0 && !can1)
                return bail(fail(PDP_E_LIMIT, "task %u: too many genes for %u tiles of %u rows", t, kJoinTileCap,
                                 kTileMaxRows));
            const uint32_t dir = can0 && (!can1 || d.tiles_n[0] >= d.tiles_n[1]) ? 0 : 1;
            ++d.tile_shift[dir];
            const uint32_t nrows = dir == 0 ? qa->n_genes : qb->n_genes;
            d.tiles_n[dir] = static_cast<uint32_t>((uint64_t(nrows) + (1u << d.tile_shift[dir]) - 1) >> d.tile_shift[dir]);
        }
        d.bbh_row_base = static_cast<uint32_t>(bbh_rows);
        if (flags & PDP_TASK_BBH) bbh_rows += tk.a->n_genes;
        // divergent homologs share a fraction of their k-mers: an eighth of the entries per
        // direction covers the family workloads with room; more needs a capacity retry
        rec_est += ndirs * ((tk.a->capacity + tk.b->capacity) / 8 + 4096);
        cost[t] = tk.a->capacity + tk.b->capacity;
        P->ab_row.push_back(orow[0]);
        P->ba_row.push_back(orow[1]);
        P->bbh_row.push_back((flags & PDP_TASK_BBH) ? d.bbh_row_base : UINT32_MAX);
        if (bh_rows >= UINT32_MAX) return bail(fail(PDP_E_LIMIT, "plan too large for 32-bit indices"));
    }
    // Pass 2, largest tasks first: join items and tiles are numbered in this order, so work-groups
    // (and the persistent kernels' counters) take the long items early.
    // each tile's expected records, the estimate rec_est sums: a region of the one-pass join each
    std::vector<uint64_t> tile_est;
    {
        uint64_t n_items = 0, n_tiles = 0;
        for (const DevTask &d : caller) {
            n_items += d.n_chunks;
            n_tiles += uint64_t(d.tiles_n[0]) + d.tiles_n[1];
        }
        P->tiles.reserve(n_tiles);
        tile_est.reserve(n_tiles);
    }
    uint32_t join_tiles = 1;
    std::vector<uint32_t> by_cost(n_tasks);
    for (uint32_t t = 0; t < n_tasks; ++t) by_cost[t] = t;
    std::stable_sort(by_cost.begin(), by_cost.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
    P->order.assign(n_tasks, 0);
    uint64_t chunks = 0, cells = 0, long_rows = 0;
    for (uint32_t i = 0; i < n_tasks; ++i) {
        const uint32_t t = by_cost[i];
        P->order[t] = i;
        DevTask d = caller[t];
        d.chunk_base = static_cast<uint32_t>(chunks);
        chunks += d.n_chunks;
        d.cell_base = static_cast<uint32_t>(cells);
        uint32_t tile_local = 0;
        const uint64_t dir_est = (tasks[t].a->capacity + tasks[t].b->capacity) / 8 + 4096;
        for (uint32_t dir = 0; dir < 2; ++dir) {
            d.tile_base[dir] = static_cast<uint32_t>(P->tiles.size());
            if (!(d.flags & (1u << dir))) continue;
            if (is_long[t]) {  // the long-gene path: a row segment instead of tiles
                const uint32_t nrows = dir == 0 ? d.a.n_genes : d.b.n_genes;
                if (nrows) P->long_segs.push_back(DevLongSeg{i, dir, static_cast<uint32_t>(long_rows), nrows});
                long_rows += nrows;
                continue;
            }
            const uint32_t nrows = dir == 0 ? d.a.n_genes : d.b.n_genes;
            const uint32_t T = 1u << d.tile_shift[dir];
            for (uint32_t r0 = 0; r0 < nrows; r0 += T, ++tile_local) {
                DevTile tl;
                tl.task = i;
                tl.dir = dir;
                tl.row0 = r0;
                tl.nrows = std::min<uint32_t>(T, nrows - r0);
                tl.rbase = 0;
                tl.rcap = 0;
                P->tiles.push_back(tl);
                // the direction's estimate split by rows (a direction without genes expects none)
                tile_est.push_back(nrows ? dir_est * tl.nrows / nrows : 0);
            }
        }
        join_tiles = std::max(join_tiles, tile_local);
        cells += uint64_t(tile_local) * d.n_chunks;
        if (cells >= UINT32_MAX) return bail(fail(PDP_E_LIMIT, "plan too large for 32-bit record counts"));
        P->tasks.push_back(d);
        if (chunks > UINT32_MAX || P->tiles.size() >= UINT32_MAX)
            return bail(fail(PDP_E_LIMIT, "plan too large for 32-bit indices"));
    }
    {  // the one-pass join's items: each task's bucket ranges of bpw * subs buckets, ordered by range
       // across tasks (a range's first bucket as a fraction of its task's buckets, in kSteps steps),
       // tasks in processing order within a step, so that the items in flight read the same stretch
       // of each genome's index (see the join kernel's XCD mapping).  A counting sort, generating
       // every item once in its place.
        constexpr uint32_t kSteps = 4096;
        auto step_of = [](uint64_t bl, uint64_t mult) {
            const uint64_t x = static_cast<uint64_t>((static_cast<unsigned __int128>(bl) * mult) >> 32);
            return static_cast<uint32_t>(std::min<uint64_t>(x, kSteps - 1));
        };
        std::vector<uint32_t> start(kSteps + 1, 0);
        std::vector<uint64_t> mult(P->tasks.size());
        for (size_t i = 0; i < P->tasks.size(); ++i) {
            const DevTask &d = P->tasks[i];
            mult[i] = (static_cast<uint64_t>(kSteps) << 32) / std::max<uint32_t>(d.a.n_buckets, 1);
            const uint64_t span = uint64_t(d.bpw) * d.subs;
            for (uint32_t c = 0; c < d.n_chunks; ++c) ++start[step_of(c * span, mult[i]) + 1];
        }
        for (uint32_t b = 0; b < kSteps; ++b) start[b + 1] += start[b];
        P->items.resize(chunks);
        for (size_t i = 0; i < P->tasks.size(); ++i) {
            const DevTask &d = P->tasks[i];
            const uint64_t span = uint64_t(d.bpw) * d.subs;
            for (uint32_t c = 0; c < d.n_chunks; ++c) {
                const uint64_t bl = c * span;
                DevItem &it = P->items[start[step_of(bl, mult[i])]++];
                it.adir = d.a.ix_dir + bl;
                it.bdir = d.b.ix_dir + bl;
                it.task = static_cast<uint32_t>(i);
                it.n_buckets = static_cast<uint32_t>(std::min<uint64_t>(d.a.n_buckets - bl, span));
                it.bl = static_cast<uint32_t>(bl);
                it.reserved = 0;
            }
        }
    }
    P->shape.n_tasks = n_tasks;
    P->shape.total_chunks = static_cast<uint32_t>(chunks);
    P->shape.total_tiles = static_cast<uint32_t>(P->tiles.size());
    P->shape.total_cells = static_cast<uint32_t>(cells);
    P->shape.bh_rows = static_cast<uint32_t>(bh_rows);
    P->shape.bbh_rows = static_cast<uint32_t>(bbh_rows);
    P->shape.tile_lds = static_cast<uint32_t>(align_up(tile_lds, 16));
    P->shape.rec_cap = prm.inc_capacity ? prm.inc_capacity : std::min<uint64_t>(rec_est, UINT32_MAX);
    P->shape.fused = (prm.flags & PDP_PARAM_TWO_PASS) ? 0u : 1u;
    P->shape.join_tiles = join_tiles;
    P->shape.fallback_grid = 0;
    {  // regions of the one-pass join: the record capacity split in proportion to the estimates
        unsigned __int128 est_sum = 0;
        for (uint64_t e : tile_est) est_sum += e;
        uint64_t at = 0;
        for (size_t ti = 0; ti < P->tiles.size(); ++ti) {
            const uint64_t cap = est_sum ? static_cast<uint64_t>(
                                               static_cast<unsigned __int128>(P->shape.rec_cap) * tile_est[ti] / est_sum)
                                         : 0;
            P->tiles[ti].rbase = static_cast<uint32_t>(at);
            P->tiles[ti].rcap = static_cast<uint32_t>(cap);
            at += cap;
        }
    }
    P->shape.join_grid = 0;
    P->shape.tile_grid = 0;
    P->shape.colmax = any_colmax ? 1u : 0u;
    P->shape.cand_cap = any_colmax ? P->shape.rec_cap : 0;
    P->shape.n_long_segs = static_cast<uint32_t>(P->long_segs.size());
    P->shape.long_rows = static_cast<uint32_t>(long_rows);  // at most the best-hit rows, below 2^32
    P->shape.long_lds = (filt ? 3u : 1u) * kLongCols * 4u;
    P->persistent = (prm.flags & PDP_PARAM_PERSISTENT) != 0;
    P->ws_bytes = pair_ws_bytes(P->shape);
    *out = P;
    return ok();
}

}  // extern "C"

namespace pdp {
int32_t plan_rebind(pdp_plan *P, const pdp_dict *from, const pdp_dict *to) {
    if (!P || !from || !to) return PDP_E_INVAL;
    if (from->n_genes != to->n_genes || from->capacity != to->capacity || from->k != to->k ||
        from->alphabet != to->alphabet || from->n_buckets != to->n_buckets || from->key_shift != to->key_shift ||
        from->flags != to->flags || (from->ix_key == nullptr) != (to->ix_key == nullptr))
        return PDP_E_INVAL;
    const DevDict nd = dev_dict(to);
    const uint32_t *lo = from->ix_dir, *hi = from->ix_dir + from->n_buckets + 1;
    auto move = [&](const uint32_t *p) { return p >= lo && p < hi ? to->ix_dir + (p - lo) : p; };
    for (DevTask &t : P->tasks) {
        if (t.a.ix_dir == from->ix_dir) t.a = nd;
        if (t.b.ix_dir == from->ix_dir) t.b = nd;
    }
    for (DevItem &it : P->items) {
        it.adir = move(it.adir);
        it.bdir = move(it.bdir);
    }
    return PDP_OK;
}
}  // namespace pdp

extern "C" {

int32_t pdp_plan_info_get(const pdp_plan *plan, pdp_plan_info *info) {
    if (!plan || !info) return fail(PDP_E_INVAL, "pdp_plan_info_get: null pointer");
    info->ws_bytes = plan->ws_bytes;
    info->inc_capacity = plan->shape.rec_cap;
    info->bh_rows = plan->shape.bh_rows;
    info->bbh_rows = plan->shape.bbh_rows;
    info->n_tasks = plan->shape.n_tasks;
    info->join_groups = plan->shape.total_chunks;
    info->tiles = plan->shape.total_tiles;
    info->tile_lds = plan->shape.tile_lds;
    info->long_rows = plan->shape.long_rows;
    info->reserved = 0;
    return ok();
}

int32_t pdp_plan_rows(const pdp_plan *plan, uint32_t t, uint32_t *ab_row, uint32_t *ba_row, uint32_t *bbh_row) {
    if (!plan) return fail(PDP_E_INVAL, "pdp_plan_rows: null plan");
    if (t >= plan->shape.n_tasks) return fail(PDP_E_INVAL, "task %u out of range", t);
    if (ab_row) *ab_row = plan->ab_row[t];
    if (ba_row) *ba_row = plan->ba_row[t];
    if (bbh_row) *bbh_row = plan->bbh_row[t];
    return ok();
}

void pdp_plan_destroy(pdp_plan *plan) { delete plan; }

int32_t pdp_plan_upload(const pdp_plan *plan, void *ws, uint64_t ws_bytes, void *stream) {
    if (!plan || !ws) return fail(PDP_E_INVAL, "pdp_plan_upload: null pointer");
    if (ws_bytes < plan->ws_bytes) return fail(PDP_E_WORKSPACE, "workspace %llu < %llu bytes", (unsigned long long)ws_bytes, (unsigned long long)plan->ws_bytes);
    PairWs w = pair_ws_carve(ws, plan->shape);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(w.tasks, plan->tasks.data(), sizeof(DevTask) * plan->tasks.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "pdp_plan_upload");
    e = hipMemcpyAsync(w.order, plan->order.data(), sizeof(uint32_t) * plan->order.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "pdp_plan_upload");
    if (!plan->items.empty()) {
        e = hipMemcpyAsync(w.items, plan->items.data(), sizeof(DevItem) * plan->items.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "pdp_plan_upload");
    }
    if (!plan->tiles.empty()) {
        e = hipMemcpyAsync(w.tiles, plan->tiles.data(), sizeof(DevTile) * plan->tiles.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "pdp_plan_upload");
    }
    if (!plan->long_segs.empty()) {
        e = hipMemcpyAsync(w.long_segs, plan->long_segs.data(), sizeof(DevLongSeg) * plan->long_segs.size(),
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "pdp_plan_upload");
    }
    return ok();
}

static int32_t check_outputs(const pdp_plan *plan, const pdp_bh_out *bh, const pdp_bbh_out *bbh, const pdp_status *st) {
    if (!bh || !st) return fail(PDP_E_INVAL, "null output or status");
    if (bh->n_rows != plan->shape.bh_rows || !bh->ptr || (bh->capacity && (!bh->col || !bh->num || !bh->den)))
        return fail(PDP_E_INVAL, "best-hit output: %u rows given, plan has %u", bh->n_rows, plan->shape.bh_rows);
    if (plan->shape.bbh_rows) {
        if (!bbh) return fail(PDP_E_INVAL, "plan has BBH rows but no BBH output was given");
        if (bbh->n_rows != plan->shape.bbh_rows || !bbh->ptr || (bbh->capacity && (!bbh->a || !bbh->b || !bbh->num || !bbh->den)))
            return fail(PDP_E_INVAL, "BBH output: %u rows given, plan has %u", bbh->n_rows, plan->shape.bbh_rows);
    }
    return PDP_OK;
}

int32_t pdp_plan_launch(const pdp_plan *plan, pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *status, void *ws,
                        uint64_t ws_bytes, void *stream) {
    if (!plan || !ws) return fail(PDP_E_INVAL, "pdp_plan_launch: null pointer");
    int32_t rc = check_outputs(plan, bh, bbh, status);
    if (rc) return rc;
    if (ws_bytes < plan->ws_bytes) return fail(PDP_E_WORKSPACE, "workspace %llu < %llu bytes", (unsigned long long)ws_bytes, (unsigned long long)plan->ws_bytes);
    PairWs w = pair_ws_carve(ws, plan->shape);
    PlanShape shape = plan->shape;
    if (!plan->device_ready) {
        hipError_t e = allow_tile_lds(plan->shape.tile_lds);
        if (e != hipSuccess) return hip_fail(e, "pdp_plan_launch");
        if (plan->persistent) {
            plan->join_grid = plan->shape.fused ? persistent_fused_grid(plan->shape.join_tiles) : persistent_join_grid();
            plan->tile_grid = persistent_tile_grid(plan->shape.tile_lds);
        }
        if (plan->shape.fused) plan->fallback_grid = persistent_join_grid();
        plan->device_ready = true;
    }
    shape.join_grid = plan->join_grid;
    shape.tile_grid = plan->tile_grid;
    shape.fallback_grid = plan->fallback_grid;
    KernelTimer timer{-1, nullptr, nullptr};
    if (plan->timer_kernel >= 0 && plan->timer_used < plan->timer_events.size()) {
        timer.kernel = plan->timer_kernel;
        timer.start = plan->timer_events[plan->timer_used].first;
        timer.stop = plan->timer_events[plan->timer_used].second;
        plan->timer_used++;
    }
    hipError_t e = launch_pairs(shape, w, bh, plan->shape.bbh_rows ? bbh : nullptr, status,
                                static_cast<hipStream_t>(stream), timer.kernel >= 0 ? &timer : nullptr);
    if (e != hipSuccess) return hip_fail(e, "pdp_plan_launch");
    return ok();
}

int32_t pdp_plan_families(const pdp_plan *plan, const pdp_bbh_out *bbh, const uint32_t *node_a, const uint32_t *node_b,
                          uint32_t n_nodes, uint32_t *labels, pdp_status *status, void *ws, uint64_t ws_bytes,
                          void *stream) {
    if (!plan || !bbh || !ws || !status || (n_nodes && (!labels || !node_a || !node_b)))
        return fail(PDP_E_INVAL, "pdp_plan_families: null pointer");
    if (bbh->n_rows != plan->shape.bbh_rows || !bbh->ptr || (bbh->capacity && (!bbh->a || !bbh->b)))
        return fail(PDP_E_INVAL, "pdp_plan_families: BBH output has %u rows, plan has %u", bbh->n_rows,
                    plan->shape.bbh_rows);
    if (ws_bytes < plan->ws_bytes) return fail(PDP_E_WORKSPACE, "workspace %llu < %llu bytes", (unsigned long long)ws_bytes, (unsigned long long)plan->ws_bytes);
    PairWs w = pair_ws_carve(ws, plan->shape);
    hipError_t e = launch_families(plan->shape, w, bbh, node_a, node_b, n_nodes, labels, status,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pdp_plan_families");
    return ok();
}

int32_t pdp_plan_timer_start(pdp_plan *plan, int32_t kernel, uint32_t max_launches) {
    if (!plan || kernel < PDP_KERNEL_JOIN || kernel > PDP_KERNEL_JOIN_BACKUP || max_launches == 0)
        return fail(PDP_E_INVAL, "pdp_plan_timer_start: bad argument");
    plan->timer_release();
    for (uint32_t i = 0; i < max_launches; ++i) {
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return hip_fail(e, "pdp_plan_timer_start");
        e = hipEventCreate(&b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            return hip_fail(e, "pdp_plan_timer_start");
        }
        plan->timer_events.emplace_back(a, b);
    }
    plan->timer_kernel = kernel;
    plan->timer_used = 0;
    return ok();
}

int32_t pdp_plan_timer_read(pdp_plan *plan, double *total_ms, uint32_t *launches) {
    if (!plan || !total_ms || !launches) return fail(PDP_E_INVAL, "pdp_plan_timer_read: null pointer");
    double sum = 0;
    for (uint32_t i = 0; i < plan->timer_used; ++i) {
        hipError_t e = hipEventSynchronize(plan->timer_events[i].second);
        if (e != hipSuccess) return hip_fail(e, "pdp_plan_timer_read");
        float ms = 0;
        e = hipEventElapsedTime(&ms, plan->timer_events[i].first, plan->timer_events[i].second);
        if (e != hipSuccess) return hip_fail(e, "pdp_plan_timer_read");
        sum += ms;
    }
    *total_ms = sum;
    *launches = plan->timer_used;
    return ok();
}

int32_t pdp_plan_timer_stop(pdp_plan *plan) {
    if (!plan) return fail(PDP_E_INVAL, "pdp_plan_timer_stop: null plan");
    plan->timer_release();
    return ok();
}

int32_t pdp_plan_run(const pdp_plan *plan, pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *status, void *ws, uint64_t ws_bytes,
                     void *stream) {
    int32_t rc = pdp_plan_upload(plan, ws, ws_bytes, stream);
    if (rc) return rc;
    return pdp_plan_launch(plan, bh, bbh, status, ws, ws_bytes, stream);
}

// ------------------------------------------------------- single-task forms

int32_t pdp_bh_ws_size(const pdp_dict *q, const pdp_dict *t, const pdp_params *params, uint64_t *ws_bytes) {
    if (!ws_bytes) return fail(PDP_E_INVAL, "pdp_bh_ws_size: null output");
    pdp_task task = {q, t, PDP_TASK_AB, 0};
    pdp_plan *P = nullptr;
    int32_t rc = pdp_plan_create(&task, 1, params, &P);
    if (rc) return rc;
    *ws_bytes = P->ws_bytes;
    delete P;
    return ok();
}

int32_t pdp_bh(const pdp_dict *q, const pdp_dict *t, const pdp_params *params, pdp_bh_out *out, pdp_status *status, void *ws,
               uint64_t ws_bytes, void *stream) {
    pdp_task task = {q, t, PDP_TASK_AB, 0};
    pdp_plan *P = nullptr;
    int32_t rc = pdp_plan_create(&task, 1, params, &P);
    if (rc) return rc;
    rc = pdp_plan_upload(P, ws, ws_bytes, stream);
    if (!rc) {
        // the plan's host tables must outlive the copy
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) rc = hip_fail(e, "pdp_bh");
    }
    if (!rc) rc = pdp_plan_launch(P, out, nullptr, status, ws, ws_bytes, stream);
    delete P;
    return rc;
}

int32_t pdp_bbh_ws_size(uint32_t n_rows, uint64_t *ws_bytes) {
    if (!ws_bytes) return fail(PDP_E_INVAL, "pdp_bbh_ws_size: null output");
    *ws_bytes = align_up(4ull * scan_partials(n_rows), 256);
    return ok();
}

int32_t pdp_bbh(const pdp_bh_out *ab, const pdp_bh_out *ba, pdp_bbh_out *out, pdp_status *status, void *ws, uint64_t ws_bytes,
                void *stream) {
    if (!ab || !ba || !out || !status || !ws) return fail(PDP_E_INVAL, "pdp_bbh: null pointer");
    if (out->n_rows != ab->n_rows) return fail(PDP_E_INVAL, "pdp_bbh: output has %u rows, input %u", out->n_rows, ab->n_rows);
    if (!ab->ptr || !ba->ptr || !out->ptr) return fail(PDP_E_INVAL, "pdp_bbh: null row pointers");
    uint64_t need = 0;
    pdp_bbh_ws_size(ab->n_rows, &need);
    if (ws_bytes < need) return fail(PDP_E_WORKSPACE, "workspace %llu < %llu bytes", (unsigned long long)ws_bytes, (unsigned long long)need);
    hipError_t e = launch_bbh_standalone(ab, ba, out, status, static_cast<uint32_t *>(ws), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pdp_bbh");
    return ok();
}

}  // extern "C"
