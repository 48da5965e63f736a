// Serving runtime: genomes arrive one by one and each is compared against a
// set of resident genomes whose dictionaries stay on the device.
//
// A worker thread owns the device side.  Requests wait in arrival order; the
// head request is admitted when a slot (one HIP stream) is free and its whole
// device footprint fits the budget, carved first-fit from a caller-provided
// arena.  An admitted request runs, on its own stream: copy of its residues to
// the device, dictionary build, one plan of |residents| tasks (best hits both
// ways + BBH against every resident), and the copy of every result and the
// status back to a pinned host buffer of the request's own (from a pool; the
// results stay there, and fetch returns views, until the request is released),
// closed by an event.  Requests admitted
// while others run overlap with them on the device (continuous batching); a
// finished slot and its memory go to the next waiting request at once.  Every
// request's arithmetic depends only on its own inputs and the residents, so
// its results are the same alone or in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

using namespace pdp;

namespace {

// First-fit allocator over [0, size) in 256-byte granules, with coalescing.
class Arena {
public:
    explicit Arena(uint64_t size) : size_(size) {
        if (size) free_[0] = size;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = align_up(std::max<uint64_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes;
                const uint64_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align_up(std::max<uint64_t>(bytes, 1), 256);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }

private:
    uint64_t size_, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

double now_us(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

struct Pinned {
    void *p = nullptr;
    uint64_t bytes = 0;
    bool ensure(uint64_t n) {
        if (n <= bytes) return true;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) return false;
        bytes = n;
        return true;
    }
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};

}  // namespace

struct ServeRequest {
    uint64_t tag;
    std::vector<uint8_t> res;
    std::vector<uint64_t> off;
    uint32_t n_genes = 0;
    uint64_t n_res = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int32_t code = PDP_OK;
    uint32_t attempts = 0;
    uint64_t inc_cap = 0, bh_cap = 0, bbh_cap = 0;
    uint32_t dict_flags = 0;  // PDP_DICT_LONG_GENES when a gene passes PDP_MAX_WINDOWS windows
    float h2d_ms = 0, build_ms = 0, pairs_ms = 0, d2h_ms = 0;  // device time of the last run
    // admission: the provisional plan and the footprint it gives are made once per run of the
    // request and kept while it waits for memory (cleared when a capacity retry grows it)
    bool planned = false;
    uint64_t foot_bytes = 0, foot_plan_ws = 0;
    // device side while in flight
    uint64_t dev_off = 0, dev_bytes = 0;
    pdp_dict dict{};
    pdp_plan *plan = nullptr;
    pdp_bh_out bh{};
    pdp_bbh_out bbh{};
    pdp_status *status = nullptr;
    // results, host: the arrays stay in the pinned buffer they were copied to (one of the
    // server's pool, held until the request is released)
    pdp_status hstatus{};
    std::unique_ptr<Pinned> out;
    std::vector<uint32_t> ab_row, ba_row, bbh_row;
    uint32_t bh_rows = 0, bbh_rows = 0;
    uint64_t nbh = 0, nbb = 0;
    const uint32_t *bh_ptr = nullptr, *bh_col = nullptr, *bh_num = nullptr, *bh_den = nullptr;
    const uint32_t *bbh_ptr = nullptr, *bbh_a = nullptr, *bbh_b = nullptr, *bbh_num = nullptr, *bbh_den = nullptr;
};

// A request on a slot ends in two steps: `head` completes when its statuses and both row-pointer
// arrays are on the host; the worker then reads the totals and enqueues copies of the used
// entries only (tail_queued), which `done` closes.
// Timing events of a run on a slot's stream: before the genome's copy, after it, after the
// dictionary build, after the plan launch, after the first result copies; before and after the
// second.
enum { kEvStart, kEvH2d, kEvBuild, kEvPairs, kEvHead, kEvTail0, kEvTail1, kEvCount };
struct ServeSlot {
    hipStream_t stream = nullptr;
    hipEvent_t head = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t ev[kEvCount] = {};
    bool tail_queued = false;
    ServeRequest *req = nullptr;
    Pinned pin;
};

struct pdp_server {
    pdp_server_config cfg{};
    int device = 0;
    std::vector<pdp_dict> residents;
    char *arena_base = nullptr;
    std::unique_ptr<Arena> arena;
    std::vector<ServeSlot> slots;
    std::deque<ServeRequest *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<ServeRequest>> all;
    std::deque<uint64_t> finished;  // tags, completion order, not yet polled
    std::vector<std::unique_ptr<Pinned>> pins;  // pinned result buffers not held by a request
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    int32_t fatal = PDP_OK;
    std::chrono::steady_clock::time_point t0;
    uint64_t admitted = 0, completed = 0, retries = 0, peak_used = 0;
    uint32_t peak_inflight = 0;
};

namespace {

// A pinned buffer of at least n bytes from the pool (the smallest that fits, else one grown).
std::unique_ptr<Pinned> take_pin(pdp_server *S, uint64_t n) {
    size_t best = S->pins.size();
    for (size_t i = 0; i < S->pins.size(); ++i)
        if (S->pins[i]->bytes >= n && (best == S->pins.size() || S->pins[i]->bytes < S->pins[best]->bytes)) best = i;
    if (best == S->pins.size() && !S->pins.empty()) best = 0;  // grow one
    std::unique_ptr<Pinned> p;
    if (best < S->pins.size()) {
        p = std::move(S->pins[best]);
        S->pins.erase(S->pins.begin() + static_cast<std::ptrdiff_t>(best));
    } else {
        p = std::make_unique<Pinned>();
    }
    if (!p->ensure(n)) return nullptr;
    return p;
}

void give_pin(pdp_server *S, std::unique_ptr<Pinned> &p) {
    if (p) S->pins.push_back(std::move(p));
}

uint64_t footprint(pdp_server *S, ServeRequest *r, uint64_t *plan_ws) {
    uint64_t arena = 0, bws = 0;
    if (pdp_dict_size(r->n_genes, r->n_res, S->cfg.k, S->cfg.alphabet, &arena, &bws) != PDP_OK) return 0;
    pdp_plan_info info;
    pdp_plan_info_get(r->plan, &info);
    *plan_ws = info.ws_bytes;
    const uint64_t A = 256;
    uint64_t b = 0;
    b += align_up(r->n_res + 1, A) + align_up(8 * (uint64_t(r->n_genes) + 1), A);  // genome
    b += align_up(arena, A);                                                         // dictionary
    b += align_up(std::max(bws, info.ws_bytes), A);                                  // build, then plan scratch
    b += align_up(4 * (uint64_t(info.bh_rows) + 1), A) + 3 * align_up(4 * std::max<uint64_t>(r->bh_cap, 1), A);
    b += align_up(4 * (uint64_t(info.bbh_rows) + 1), A) + 4 * align_up(4 * std::max<uint64_t>(r->bbh_cap, 1), A);
    b += A;  // status
    return b;
}

// Creates the request's plan from its (not yet built) dictionary descriptor.
int32_t make_plan(pdp_server *S, ServeRequest *r) {
    if (r->plan) pdp_plan_destroy(r->plan);
    r->plan = nullptr;
    std::vector<pdp_task> tasks(S->residents.size());
    for (size_t i = 0; i < tasks.size(); ++i) tasks[i] = {&r->dict, &S->residents[i], PDP_TASK_BBH, 0};
    pdp_params p = S->cfg.params;
    p.inc_capacity = r->inc_cap;
    return pdp_plan_create(tasks.data(), static_cast<uint32_t>(tasks.size()), &p, &r->plan);
}

// The provisional plan of a request and the device footprint it gives: the descriptor is bound
// to a placeholder address (planning reads only its sizes); launch_request moves the plan's
// pointers once the memory is placed.  Both are kept while the request waits for memory.  Reads
// only the request and the server's fixed configuration, so any thread may call it for a request
// it owns.
int32_t prepare_plan(pdp_server *S, ServeRequest *r) {
    uint64_t dict_bytes = 0, build_ws = 0;
    int32_t rc = pdp_dict_size(r->n_genes, r->n_res, S->cfg.k, S->cfg.alphabet, &dict_bytes, &build_ws);
    if (rc == PDP_OK)
        rc = pdp_dict_bind(reinterpret_cast<void *>(uintptr_t(256)), dict_bytes, r->n_genes, r->n_res, S->cfg.k,
                           S->cfg.alphabet, r->dict_flags, &r->dict);
    if (rc == PDP_OK) rc = make_plan(S, r);
    if (rc == PDP_OK) r->foot_bytes = footprint(S, r, &r->foot_plan_ws);
    r->planned = rc == PDP_OK;
    return rc;
}

// Everything a request enqueues on its slot's stream.
int32_t launch_request(pdp_server *S, ServeSlot &slot, ServeRequest *r, uint64_t plan_ws) {
    hipStream_t s = slot.stream;
    char *base = S->arena_base + r->dev_off;
    const uint64_t A = 256;
    auto take = [&](uint64_t bytes) {
        char *q = base;
        base += align_up(bytes, A);
        return q;
    };
    uint8_t *res = reinterpret_cast<uint8_t *>(take(r->n_res + 1));
    uint64_t *off = reinterpret_cast<uint64_t *>(take(8 * (uint64_t(r->n_genes) + 1)));
    uint64_t arena = 0, bws = 0;
    pdp_dict_size(r->n_genes, r->n_res, S->cfg.k, S->cfg.alphabet, &arena, &bws);
    void *dict_mem = take(arena);
    void *scratch = take(std::max(bws, plan_ws));
    const uint64_t scratch_bytes = std::max(bws, plan_ws);
    pdp_plan_info info;
    pdp_plan_info_get(r->plan, &info);
    r->bh.n_rows = info.bh_rows;
    r->bh.capacity = r->bh_cap;
    r->bh.ptr = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(info.bh_rows) + 1)));
    r->bh.col = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(r->bh_cap, 1)));
    r->bh.num = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(r->bh_cap, 1)));
    r->bh.den = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(r->bh_cap, 1)));
    r->bbh.n_rows = info.bbh_rows;
    r->bbh.capacity = r->bbh_cap;
    r->bbh.ptr = reinterpret_cast<uint32_t *>(take(4 * (uint64_t(info.bbh_rows) + 1)));
    r->bbh.a = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(r->bbh_cap, 1)));
    r->bbh.b = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(r->bbh_cap, 1)));
    r->bbh.num = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(r->bbh_cap, 1)));
    r->bbh.den = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(r->bbh_cap, 1)));
    r->status = reinterpret_cast<pdp_status *>(take(sizeof(pdp_status)));
    // The dictionary now lives in this allocation: the admission plan, made with the
    // descriptor bound to a placeholder address, moves its pointers here.
    const pdp_dict placeholder = r->dict;
    int32_t rc = pdp_dict_bind(dict_mem, arena, r->n_genes, r->n_res, S->cfg.k, S->cfg.alphabet, r->dict_flags, &r->dict);
    if (rc) return rc;
    rc = r->plan ? plan_rebind(r->plan, &placeholder, &r->dict) : make_plan(S, r);
    if (rc) return rc;
    // host input -> pinned staging -> device; pinned output staging sized for the results
    const uint64_t in_bytes = r->n_res + 8 * (uint64_t(r->n_genes) + 1);
    const uint64_t out_bytes = 2 * sizeof(pdp_status) + 4 * (uint64_t(info.bh_rows) + 1 + 3 * r->bh_cap) +
                               4 * (uint64_t(info.bbh_rows) + 1 + 4 * r->bbh_cap);
    if (!slot.pin.ensure(in_bytes + 64)) return PDP_E_HIP;
    give_pin(S, r->out);  // a retried request gives back its earlier buffer
    r->out = take_pin(S, out_bytes + 64);
    if (!r->out) return PDP_E_HIP;
    if (hipEventRecord(slot.ev[kEvStart], s) != hipSuccess) return PDP_E_HIP;
    std::memcpy(slot.pin.p, r->res.data(), r->n_res);
    std::memcpy(static_cast<char *>(slot.pin.p) + r->n_res, r->off.data(), 8 * (uint64_t(r->n_genes) + 1));
    if (hipMemcpyAsync(res, slot.pin.p, r->n_res, hipMemcpyHostToDevice, s) != hipSuccess) return PDP_E_HIP;
    if (hipMemcpyAsync(off, static_cast<char *>(slot.pin.p) + r->n_res, 8 * (uint64_t(r->n_genes) + 1),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return PDP_E_HIP;
    if (hipEventRecord(slot.ev[kEvH2d], s) != hipSuccess) return PDP_E_HIP;
    pdp_genome g{res, off, r->n_genes, 0, r->n_res};
    rc = pdp_dict_build(&g, &r->dict, scratch, scratch_bytes, s);
    if (rc) return rc;
    if (hipEventRecord(slot.ev[kEvBuild], s) != hipSuccess) return PDP_E_HIP;
    rc = pdp_plan_upload(r->plan, scratch, scratch_bytes, s);
    if (rc) return rc;
    rc = pdp_plan_launch(r->plan, &r->bh, &r->bbh, r->status, scratch, scratch_bytes, s);
    if (rc) return rc;
    if (hipEventRecord(slot.ev[kEvPairs], s) != hipSuccess) return PDP_E_HIP;
    // first step of the results: both statuses and both row-pointer arrays, to the request's own
    // pinned buffer (the entries follow once their totals are known, copy_tail)
    char *h = static_cast<char *>(r->out->p);
    auto d2h = [&](const void *src, uint64_t bytes) {
        if (hipMemcpyAsync(h, src, bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return false;
        h += bytes;
        return true;
    };
    bool ok = d2h(r->status, sizeof(pdp_status)) && d2h(r->dict.status, sizeof(pdp_status)) &&
              d2h(r->bh.ptr, 4 * (uint64_t(info.bh_rows) + 1)) && d2h(r->bbh.ptr, 4 * (uint64_t(info.bbh_rows) + 1));
    if (!ok) return PDP_E_HIP;
    if (hipEventRecord(slot.ev[kEvHead], s) != hipSuccess || hipEventRecord(slot.head, s) != hipSuccess)
        return PDP_E_HIP;
    slot.tail_queued = false;
    return PDP_OK;
}

// Layout of a request's pinned results: statuses, best-hit row pointers, BBH row pointers, then
// the used entries of each array (bh col, num, den; BBH a, b, num, den).
struct HostLayout {
    const char *base;
    uint64_t bh_rows, bbh_rows;
    const pdp_status *status() const { return reinterpret_cast<const pdp_status *>(base); }
    const pdp_status *dict_status() const { return reinterpret_cast<const pdp_status *>(base) + 1; }
    const uint32_t *bh_ptr() const { return reinterpret_cast<const uint32_t *>(base + 2 * sizeof(pdp_status)); }
    const uint32_t *bbh_ptr() const { return bh_ptr() + bh_rows + 1; }
    const uint32_t *entries() const { return bbh_ptr() + bbh_rows + 1; }
};

// Second step: the used entries, sized by the totals the first step brought back (a total is
// at most its capacity once the status is clean), then `done`.
int32_t copy_tail(ServeSlot &slot, ServeRequest *r) {
    pdp_plan_info info;
    pdp_plan_info_get(r->plan, &info);
    const HostLayout L{static_cast<const char *>(r->out->p), info.bh_rows, info.bbh_rows};
    const uint64_t nbh = std::min<uint64_t>(L.bh_ptr()[info.bh_rows], r->bh_cap);
    const uint64_t nbb = std::min<uint64_t>(L.bbh_ptr()[info.bbh_rows], r->bbh_cap);
    char *h = const_cast<char *>(reinterpret_cast<const char *>(L.entries()));
    hipStream_t s = slot.stream;
    if (hipEventRecord(slot.ev[kEvTail0], s) != hipSuccess) return PDP_E_HIP;
    auto d2h = [&](const void *src, uint64_t bytes) {
        if (bytes && hipMemcpyAsync(h, src, bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return false;
        h += bytes;
        return true;
    };
    const bool ok = d2h(r->bh.col, 4 * nbh) && d2h(r->bh.num, 4 * nbh) && d2h(r->bh.den, 4 * nbh) &&
                    d2h(r->bbh.a, 4 * nbb) && d2h(r->bbh.b, 4 * nbb) && d2h(r->bbh.num, 4 * nbb) &&
                    d2h(r->bbh.den, 4 * nbb);
    if (!ok) return PDP_E_HIP;
    if (hipEventRecord(slot.ev[kEvTail1], s) != hipSuccess || hipEventRecord(slot.done, s) != hipSuccess)
        return PDP_E_HIP;
    slot.tail_queued = true;
    return PDP_OK;
}

// After the first step: 0 when the run is clean (its entries are to be copied), 1 when the request
// is done with an error, 2 when a capacity error grew its buffers and it runs again.
int head_check(pdp_server *S, ServeRequest *r) {
    const pdp_status st = *reinterpret_cast<const pdp_status *>(r->out->p);
    const pdp_status dst = *(reinterpret_cast<const pdp_status *>(r->out->p) + 1);
    if (dst.code != PDP_OK) {
        r->hstatus = dst;
        r->code = dst.code;
        return 1;
    }
    if (st.code == PDP_E_CAPACITY && r->attempts < 4) {
        // grow the array that overflowed and run the request again
        const uint64_t grow = st.needed + st.needed / 4 + 1024;
        if (st.where == 0) r->inc_cap = grow;
        else if (st.where == 1) r->bh_cap = grow;
        else r->bbh_cap = grow;
        S->retries++;
        r->planned = false;  // the capacities changed: plan and footprint are made again
        give_pin(S, r->out);
        return 2;
    }
    r->hstatus = st;
    r->code = st.code;
    return st.code != PDP_OK ? 1 : 0;
}

float event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : 0.0f;
}

// After the second step: the run's device times, and views of the arrays in the pinned buffer,
// laid out as the copies wrote them.
void collect(pdp_server *S, const ServeSlot &slot, ServeRequest *r) {
    r->h2d_ms = event_ms(slot.ev[kEvStart], slot.ev[kEvH2d]);
    r->build_ms = event_ms(slot.ev[kEvH2d], slot.ev[kEvBuild]);
    r->pairs_ms = event_ms(slot.ev[kEvBuild], slot.ev[kEvPairs]);
    r->d2h_ms = event_ms(slot.ev[kEvPairs], slot.ev[kEvHead]) + event_ms(slot.ev[kEvTail0], slot.ev[kEvTail1]);
    pdp_plan_info info;
    pdp_plan_info_get(r->plan, &info);
    const HostLayout L{static_cast<const char *>(r->out->p), info.bh_rows, info.bbh_rows};
    r->bh_rows = info.bh_rows;
    r->bbh_rows = info.bbh_rows;
    r->bh_ptr = L.bh_ptr();
    r->bbh_ptr = L.bbh_ptr();
    r->nbh = r->bh_ptr[info.bh_rows];
    r->nbb = r->bbh_ptr[info.bbh_rows];
    const uint32_t *e = L.entries();
    r->bh_col = e;
    r->bh_num = e + r->nbh;
    r->bh_den = e + 2 * r->nbh;
    e += 3 * r->nbh;
    r->bbh_a = e;
    r->bbh_b = e + r->nbb;
    r->bbh_num = e + 2 * r->nbb;
    r->bbh_den = e + 3 * r->nbb;
    const uint32_t nt = static_cast<uint32_t>(S->residents.size());
    r->ab_row.resize(nt);
    r->ba_row.resize(nt);
    r->bbh_row.resize(nt);
    for (uint32_t t = 0; t < nt; ++t) pdp_plan_rows(r->plan, t, &r->ab_row[t], &r->ba_row[t], &r->bbh_row[t]);
}

void finish(pdp_server *S, ServeRequest *r) {
    r->t_done = now_us(S->t0);
    r->res.clear();
    r->res.shrink_to_fit();
    r->off.clear();
    r->off.shrink_to_fit();
    if (r->plan) pdp_plan_destroy(r->plan);
    r->plan = nullptr;
    S->finished.push_back(r->tag);
    S->completed++;
}

void worker_loop(pdp_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop) {
        bool progress = false;
        // advance and retire slots: a clean first step gets its entries copied; a finished second
        // step, or a first step with an error, frees the slot and the request's memory
        for (ServeSlot &slot : S->slots) {
            if (!slot.req) continue;
            const hipError_t q = hipEventQuery(slot.tail_queued ? slot.done : slot.head);
            if (q == hipErrorNotReady) continue;
            ServeRequest *r = slot.req;
            progress = true;
            bool done = true;
            if (q != hipSuccess) {
                r->code = PDP_E_HIP;
                S->fatal = PDP_E_HIP;
            } else if (!slot.tail_queued) {
                const int h = head_check(S, r);
                if (h == 0) {
                    if (copy_tail(slot, r) == PDP_OK) continue;  // the slot keeps the request until `done`
                    (void)hipStreamSynchronize(slot.stream);
                    r->code = PDP_E_HIP;
                    S->fatal = PDP_E_HIP;
                }
                done = h != 2;
            } else {
                collect(S, slot, r);
            }
            S->arena->release(r->dev_off, r->dev_bytes);
            slot.req = nullptr;
            slot.tail_queued = false;
            if (done) finish(S, r);
            else S->pending.push_front(r);  // retried ahead of newer requests
        }
        // admit waiting requests in arrival order
        while (!S->pending.empty()) {
            ServeSlot *free_slot = nullptr;
            for (ServeSlot &slot : S->slots)
                if (!slot.req) {
                    free_slot = &slot;
                    break;
                }
            if (!free_slot) break;
            ServeRequest *r = S->pending.front();
            // normally planned by pdp_server_submit; again here after a capacity retry
            int32_t rc = r->planned ? PDP_OK : prepare_plan(S, r);
            const uint64_t bytes = r->foot_bytes, plan_ws = r->foot_plan_ws;
            if (rc != PDP_OK || bytes == 0 || bytes > S->arena->size()) {
                S->pending.pop_front();
                r->code = rc != PDP_OK ? rc : PDP_E_BUDGET;
                finish(S, r);
                progress = true;
                continue;
            }
            uint64_t off = 0;
            if (!S->arena->alloc(bytes, &off)) break;  // wait for memory to free up
            S->pending.pop_front();
            r->dev_off = off;
            r->dev_bytes = bytes;
            // a run starts only now that its memory is placed: waiting for memory is no attempt
            r->attempts++;
            if (r->attempts == 1) r->t_admit = now_us(S->t0);
            rc = launch_request(S, *free_slot, r, plan_ws);
            if (rc != PDP_OK) {
                (void)hipStreamSynchronize(free_slot->stream);
                S->arena->release(off, bytes);
                r->code = rc;
                finish(S, r);
            } else {
                free_slot->req = r;
                S->admitted++;
            }
            progress = true;
            S->peak_used = std::max(S->peak_used, S->arena->used());
            uint32_t inflight = 0;
            for (ServeSlot &slot : S->slots) inflight += slot.req != nullptr;
            S->peak_inflight = std::max(S->peak_inflight, inflight);
        }
        if (progress) {
            S->cv.notify_all();
            continue;
        }
        bool busy = false;
        for (ServeSlot &slot : S->slots) busy = busy || slot.req != nullptr;
        // poll completions quickly while work is in flight; sleep until a submit otherwise
        if (busy) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            S->cv.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace

extern "C" {

int32_t pdp_server_create(const pdp_server_config *cfg, const pdp_dict *const *residents, uint32_t n_residents,
                          void *arena, uint64_t arena_bytes, pdp_server **out) {
    if (!cfg || !out || !arena || (n_residents && !residents)) return api_fail(PDP_E_INVAL, "pdp_server_create: null argument");
    *out = nullptr;
    if (n_residents == 0) return api_fail(PDP_E_INVAL, "pdp_server_create: no resident genomes");
    if (cfg->slots == 0 || cfg->slots > 64) return api_fail(PDP_E_INVAL, "pdp_server_create: slots must be 1..64");
    if (cfg->budget_bytes > arena_bytes) return api_fail(PDP_E_WORKSPACE, "budget larger than the arena");
    if (reinterpret_cast<uintptr_t>(arena) % 256) return api_fail(PDP_E_INVAL, "arena not 256-byte aligned");
    for (uint32_t i = 0; i < n_residents; ++i) {
        if (!residents[i] || residents[i]->k != cfg->k || residents[i]->alphabet != cfg->alphabet)
            return api_fail(PDP_E_INVAL, "resident %u: missing or built with another k or alphabet", i);
    }
    auto S = std::make_unique<pdp_server>();
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess) return api_fail(PDP_E_HIP, "hipGetDevice");
    for (uint32_t i = 0; i < n_residents; ++i) S->residents.push_back(*residents[i]);
    S->arena_base = static_cast<char *>(arena);
    S->arena = std::make_unique<Arena>(cfg->budget_bytes);
    S->slots.resize(cfg->slots);
    for (ServeSlot &slot : S->slots) {
        if (hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&slot.head, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&slot.done, hipEventDisableTiming) != hipSuccess)
            return api_fail(PDP_E_HIP, "pdp_server_create: stream or event creation failed");
        for (hipEvent_t &e : slot.ev)
            if (hipEventCreate(&e) != hipSuccess) return api_fail(PDP_E_HIP, "pdp_server_create: event creation failed");
    }
    S->t0 = std::chrono::steady_clock::now();
    pdp_server *raw = S.release();
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return PDP_OK;
}

int32_t pdp_server_submit(pdp_server *S, const uint8_t *residues, const uint64_t *gene_off, uint32_t n_genes,
                          uint64_t tag) {
    if (!S || !gene_off || (!residues && gene_off[n_genes])) return api_fail(PDP_E_INVAL, "pdp_server_submit: null argument");
    const double t_in = now_us(S->t0);  // the request's latency counts from here, planning included
    if (gene_off[0] != 0) return api_fail(PDP_E_INVAL, "pdp_server_submit: gene_off[0] must be 0");
    uint64_t longest = 0;
    for (uint32_t i = 0; i < n_genes; ++i) {
        if (gene_off[i + 1] < gene_off[i]) return api_fail(PDP_E_INVAL, "pdp_server_submit: offsets decrease at gene %u", i);
        longest = std::max<uint64_t>(longest, gene_off[i + 1] - gene_off[i]);
    }
    auto r = std::make_unique<ServeRequest>();
    // a gene past the 16-bit window limit puts the request's pairs on the long-gene path
    if (longest >= S->cfg.k && longest - S->cfg.k + 1 > PDP_MAX_WINDOWS) r->dict_flags = PDP_DICT_LONG_GENES;
    r->tag = tag;
    r->n_genes = n_genes;
    r->n_res = gene_off[n_genes];
    if (r->n_res >= (1ull << 32) || n_genes > PDP_MAX_GENES) return api_fail(PDP_E_LIMIT, "pdp_server_submit: genome too large");
    r->res.assign(residues, residues + r->n_res);
    r->off.assign(gene_off, gene_off + n_genes + 1);
    // starting capacities; a capacity error grows them and runs the request again
    uint64_t resident_entries = 0, resident_genes = 0;
    for (const pdp_dict &d : S->residents) {
        resident_entries += d.capacity;
        resident_genes += d.n_genes;
    }
    // records: half the entries of every pair with records for both directions, a quarter with
    // column maxima (records for the request's rows only).  Arrivals share many k-mers with the
    // residents (their genes come from resident families), and the one-pass join falls back to two
    // passes when one tile's share of the capacity overflows, so the capacity is generous.
    const uint64_t entries = resident_entries + S->residents.size() * (r->n_res + 1);
    r->inc_cap = (S->cfg.params.flags & PDP_PARAM_COLMAX ? entries / 4 : entries / 2) + 65536;
    const uint64_t rows = uint64_t(n_genes) * S->residents.size() + resident_genes;
    r->bh_cap = rows + rows / 4 + 4096;
    r->bbh_cap = uint64_t(n_genes) * S->residents.size() * 3 / 4 + 4096;
    // planning here, in the caller's thread, keeps it off the worker's loop (the worker plans
    // again only when this fails, to report the error, or after a capacity retry)
    (void)prepare_plan(S, r.get());
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->all.count(tag)) {
        if (r->plan) pdp_plan_destroy(r->plan);
        return api_fail(PDP_E_INVAL, "pdp_server_submit: tag already in use");
    }
    r->t_submit = t_in;
    S->pending.push_back(r.get());
    S->all[tag] = std::move(r);
    S->cv.notify_all();
    return PDP_OK;
}

int32_t pdp_server_poll(pdp_server *S, pdp_request_done *done, uint32_t max, uint32_t *n_done, uint32_t wait_us) {
    if (!S || !n_done || (max && !done)) return api_fail(PDP_E_INVAL, "pdp_server_poll: null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->finished.empty() && wait_us)
        S->cv.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !S->finished.empty(); });
    uint32_t n = 0;
    while (n < max && !S->finished.empty()) {
        const uint64_t tag = S->finished.front();
        S->finished.pop_front();
        ServeRequest *r = S->all[tag].get();
        pdp_request_done &d = done[n++];
        std::memset(&d, 0, sizeof(d));
        d.tag = tag;
        d.code = r->code;
        d.n_genes = r->n_genes;
        d.attempts = r->attempts;
        d.flags = r->hstatus.flags;
        d.submit_us = r->t_submit;
        d.admit_us = r->t_admit;
        d.done_us = r->t_done;
        d.bh_entries = r->code == PDP_OK ? r->nbh : 0;
        d.bbh_pairs = r->code == PDP_OK ? r->nbb : 0;
        d.h2d_ms = r->h2d_ms;
        d.build_ms = r->build_ms;
        d.pairs_ms = r->pairs_ms;
        d.d2h_ms = r->d2h_ms;
    }
    *n_done = n;
    return S->fatal;
}

int32_t pdp_server_fetch(pdp_server *S, uint64_t tag, pdp_request_result *out) {
    if (!S || !out) return api_fail(PDP_E_INVAL, "pdp_server_fetch: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(tag);
    if (it == S->all.end() || it->second->t_done == 0) return api_fail(PDP_E_INVAL, "pdp_server_fetch: unknown or unfinished tag");
    ServeRequest *r = it->second.get();
    std::memset(out, 0, sizeof(*out));
    out->code = r->code;
    out->status = r->hstatus;
    out->n_residents = static_cast<uint32_t>(S->residents.size());
    if (r->code != PDP_OK) return PDP_OK;
    out->bh_rows = r->bh_rows;
    out->bbh_rows = r->bbh_rows;
    out->ab_row = r->ab_row.data();
    out->ba_row = r->ba_row.data();
    out->bbh_row = r->bbh_row.data();
    out->bh_ptr = r->bh_ptr;
    out->bh_col = r->bh_col;
    out->bh_num = r->bh_num;
    out->bh_den = r->bh_den;
    out->bbh_ptr = r->bbh_ptr;
    out->bbh_a = r->bbh_a;
    out->bbh_b = r->bbh_b;
    out->bbh_num = r->bbh_num;
    out->bbh_den = r->bbh_den;
    return PDP_OK;
}

int32_t pdp_server_release(pdp_server *S, uint64_t tag) {
    if (!S) return api_fail(PDP_E_INVAL, "pdp_server_release: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(tag);
    if (it == S->all.end() || it->second->t_done == 0) return api_fail(PDP_E_INVAL, "pdp_server_release: unknown or unfinished tag");
    give_pin(S, it->second->out);  // its pinned result buffer goes back to the pool
    S->all.erase(it);
    return PDP_OK;
}

int32_t pdp_server_stats_get(pdp_server *S, pdp_server_stats *out) {
    if (!S || !out) return api_fail(PDP_E_INVAL, "pdp_server_stats_get: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof(*out));
    out->admitted = S->admitted;
    out->completed = S->completed;
    out->retries = S->retries;
    out->pending = S->pending.size();
    out->budget_bytes = S->arena->size();
    out->used_bytes = S->arena->used();
    out->peak_used_bytes = S->peak_used;
    out->peak_inflight = S->peak_inflight;
    for (const ServeSlot &slot : S->slots) out->inflight += slot.req != nullptr;
    return PDP_OK;
}

void pdp_server_destroy(pdp_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (ServeSlot &slot : S->slots) {
        if (slot.stream) (void)hipStreamSynchronize(slot.stream);
        if (slot.req && slot.req->plan) pdp_plan_destroy(slot.req->plan);
        for (hipEvent_t e : slot.ev)
            if (e) (void)hipEventDestroy(e);
        if (slot.head) (void)hipEventDestroy(slot.head);
        if (slot.done) (void)hipEventDestroy(slot.done);
        if (slot.stream) (void)hipStreamDestroy(slot.stream);
    }
    for (auto &kv : S->all)
        if (kv.second->plan) pdp_plan_destroy(kv.second->plan);
    delete S;
}

}  // extern "C"
