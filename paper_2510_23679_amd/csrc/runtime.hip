// Host runtime around the kernels: HIP-graph capture of enqueued library work
// and an autotuner that picks tile shapes and work splits by timing them.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"

using namespace pdp;

namespace {

int32_t rt_fail(int32_t code, const char *msg) { return pdp::api_fail(code, "%s", msg); }

}  // namespace

struct pdp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int32_t pdp_capture_begin(void *stream) {
    if (!stream) return rt_fail(PDP_E_INVAL, "capture needs a stream other than the NULL stream");
    hipError_t e = hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal);
    return e == hipSuccess ? PDP_OK : rt_fail(PDP_E_HIP, hipGetErrorString(e));
}

int32_t pdp_capture_end(void *stream, pdp_graph **out) {
    if (!stream || !out) return rt_fail(PDP_E_INVAL, "pdp_capture_end: null argument");
    *out = nullptr;
    pdp_graph *g = new pdp_graph();
    hipError_t e = hipStreamEndCapture(static_cast<hipStream_t>(stream), &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return rt_fail(PDP_E_HIP, hipGetErrorString(e));
    }
    *out = g;
    return PDP_OK;
}

int32_t pdp_graph_launch(pdp_graph *g, void *stream) {
    if (!g || !g->exec) return rt_fail(PDP_E_INVAL, "pdp_graph_launch: no graph");
    hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PDP_OK : rt_fail(PDP_E_HIP, hipGetErrorString(e));
}

void pdp_graph_destroy(pdp_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

// ------------------------------------------------------------- autotuner

// Tile height x join sub-range size x persistent kernels x column maxima: the best tile height
// follows the records per row (denser at small k), column maxima pay off when the join dominates.
static std::vector<pdp_params> default_candidates() {
    std::vector<pdp_params> c;
    const uint32_t rows[] = {32, 64, 128};
    const uint32_t join[] = {256, 512, 768, 1024};
    for (uint32_t colmax = 0; colmax < 2; ++colmax)
        for (uint32_t persistent = 0; persistent < 2; ++persistent)
            for (uint32_t r : rows)
                for (uint32_t j : join) {
                    pdp_params p;
                    std::memset(&p, 0, sizeof(p));
                    p.tile_rows = r;
                    p.join_entries = j;
                    p.flags = (persistent ? PDP_PARAM_PERSISTENT : 0) | (colmax ? PDP_PARAM_COLMAX : 0);
                    c.push_back(p);
                }
    return c;
}

int32_t pdp_autotune_ws_size(const pdp_task *tasks, uint32_t n_tasks, const pdp_params *cands, uint32_t n_cands,
                             uint64_t *ws_bytes) {
    if (!ws_bytes) return rt_fail(PDP_E_INVAL, "pdp_autotune_ws_size: null output");
    std::vector<pdp_params> c = cands ? std::vector<pdp_params>(cands, cands + n_cands) : default_candidates();
    uint64_t need = 0;
    for (const pdp_params &p : c) {
        pdp_plan *P = nullptr;
        if (pdp_plan_create(tasks, n_tasks, &p, &P) != PDP_OK) continue;  // a candidate that does not fit is skipped
        pdp_plan_info info;
        pdp_plan_info_get(P, &info);
        need = std::max<uint64_t>(need, info.ws_bytes);
        pdp_plan_destroy(P);
    }
    if (need == 0) return rt_fail(PDP_E_LIMIT, "no candidate fits these tasks");
    *ws_bytes = need;
    return PDP_OK;
}

int32_t pdp_autotune(const pdp_task *tasks, uint32_t n_tasks, const pdp_params *cands, uint32_t n_cands, uint32_t reps,
                     pdp_bh_out *bh, pdp_bbh_out *bbh, pdp_status *status, void *ws, uint64_t ws_bytes, void *stream,
                     pdp_tune_result *out) {
    if (!out || !status || !ws) return rt_fail(PDP_E_INVAL, "pdp_autotune: null argument");
    if (reps == 0) reps = 1;
    std::vector<pdp_params> c = cands ? std::vector<pdp_params>(cands, cands + n_cands) : default_candidates();
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return rt_fail(PDP_E_HIP, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return rt_fail(PDP_E_HIP, "hipEventCreate");
    }
    std::memset(out, 0, sizeof(*out));
    double best = -1;
    int32_t rc = PDP_OK;
    for (size_t i = 0; i < c.size(); ++i) {
        pdp_plan *P = nullptr;
        if (pdp_plan_create(tasks, n_tasks, &c[i], &P) != PDP_OK) continue;
        pdp_plan_info info;
        pdp_plan_info_get(P, &info);
        bool ok = info.ws_bytes <= ws_bytes && pdp_plan_upload(P, ws, ws_bytes, stream) == PDP_OK &&
                  pdp_plan_launch(P, bh, bbh, status, ws, ws_bytes, stream) == PDP_OK;  // warm-up
        float ms = 0;
        if (ok) {
            ok = hipEventRecord(e0, s) == hipSuccess;
            for (uint32_t r = 0; ok && r < reps; ++r) ok = pdp_plan_launch(P, bh, bbh, status, ws, ws_bytes, stream) == PDP_OK;
            ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        }
        pdp_status st;
        std::memset(&st, 0, sizeof(st));
        if (ok) ok = hipMemcpy(&st, status, sizeof(st), hipMemcpyDeviceToHost) == hipSuccess && st.code == PDP_OK;
        pdp_plan_destroy(P);
        if (!ok) continue;
        const double avg = ms / reps;
        if (out->tried == 0) out->first_ms = avg;
        out->tried++;
        if (best < 0 || avg < best) {
            best = avg;
            out->best = c[i];
            out->best_ms = avg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (out->tried == 0) rc = rt_fail(PDP_E_LIMIT, "no candidate ran cleanly (capacity or workspace too small)");
    return rc;
}

}  // extern "C"
