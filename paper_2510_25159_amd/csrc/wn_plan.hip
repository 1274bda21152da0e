// Plans: preallocated batched queries captured into a HIP graph, with an
// autotuner over workgroup tiling and queue policy.
#include "wn_host_internal.h"

#include <algorithm>
#include <new>
#include <vector>

using namespace wn;

struct wn_plan {
    const wn_faces* faces = nullptr;
    wn_points pts{};
    wn_query_opts q{};
    Scratch sc{};
    double* out_w = nullptr;
    uint8_t* out_lab = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
};

namespace {

void drop_graph(wn_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

wn_status capture(wn_plan* p) {
    drop_graph(p);
    const wn_points pts = p->pts;
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_status(e);
    const wn_status st = query_core(p->faces, &pts, p->out_w, p->out_lab, &p->q, &p->sc, p->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap, &g);
    if (st != WN_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_status(e);
    p->graph = g;
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    return hip_status(e);
}

}  // namespace

extern "C" {

wn_status wn_plan_create(const wn_faces* h, const wn_points* pts, double* out_w, uint8_t* out_lab,
                         const wn_query_opts* qo, void* stream, wn_plan** out) {
    if (!h || !pts || !out || !out_w || !out_lab) return WN_E_INVALID;
    if (pts->num_points < 1 || pts->num_points >= 0x7fffffffll || !pts->u || !pts->v || pts->stride < 1 ||
        !pts->face_point_offsets)
        return WN_E_INVALID;
    *out = nullptr;
    wn_query_opts q;
    wn_default_query_opts(&q);
    if (qo) q = *qo;
    if (q.profile || q.stats || q.depth_log) return WN_E_INVALID;
    const int sched = q.schedule >= 0 ? q.schedule : h->schedule;
    if (sched == WN_SCHED_PLAIN) return WN_E_UNSUPPORTED;
    wn_plan* p = new (std::nothrow) wn_plan();
    if (!p) return WN_E_NOMEM;
    p->faces = h;
    p->pts = *pts;
    p->pts.face_point_offsets_host = nullptr;
    p->q = q;
    p->out_w = out_w;
    p->out_lab = out_lab;
    const bool binned = sched == WN_SCHED_BINNED;
    int64_t cap = q.near_capacity > 0 ? q.near_capacity : 8 * pts->num_points + 65536;
    cap = std::min<int64_t>(cap, (int64_t)1 << 34);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = scratch_alloc(h, pts->num_points, cap, binned, binned, out_w, out_lab, h->rule, p->sc, st, false);
    if (e == hipSuccess) e = hipStreamCreate(&p->cap);
    if (e != hipSuccess) {
        wn_plan_destroy(p);
        return hip_status(e);
    }
    const wn_status s2 = capture(p);
    if (s2 != WN_OK) {
        wn_plan_destroy(p);
        return s2;
    }
    *out = p;
    return WN_OK;
}

wn_status wn_plan_launch(wn_plan* p, void* stream) {
    if (!p || !p->exec) return WN_E_INVALID;
    return hip_status(hipGraphLaunch(p->exec, (hipStream_t)stream));
}

wn_status wn_plan_autotune(wn_plan* p, int32_t reps, void* stream, double* report) {
    if (!p || reps < 1 || reps > 1000) return WN_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const wn_points pts = p->pts;
    constexpr int kQ = 5;
    const int qpws[kQ] = {64, 128, 256, 512, 1024};
    const int pols[2] = {1, 2};
    double best = 1e300;
    int bq = 256, bp = 1, k = 0;
    wn_status ws = WN_OK;
    for (int i = 0; i < kQ && e == hipSuccess && ws == WN_OK; ++i)
        for (int j = 0; j < 2 && e == hipSuccess && ws == WN_OK; ++j, ++k) {
            wn_query_opts q = p->q;
            q.queries_per_wg = qpws[i];
            q.queue_policy = pols[j];
            ws = query_core(p->faces, &pts, p->out_w, p->out_lab, &q, &p->sc, st);  // warm
            e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && ws == WN_OK; ++r)
                ws = query_core(p->faces, &pts, p->out_w, p->out_lab, &q, &p->sc, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const double avg = (double)ms / reps;
            if (report) report[k] = avg;
            if (avg < best) {
                best = avg;
                bq = qpws[i];
                bp = pols[j];
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ws != WN_OK) return ws;
    if (e != hipSuccess) return hip_status(e);
    p->q.queries_per_wg = bq;
    p->q.queue_policy = bp;
    if (report) {
        report[2 * kQ] = bq;
        report[2 * kQ + 1] = bp;
    }
    return capture(p);
}

void wn_plan_destroy(wn_plan* p) {
    if (!p) return;
    drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->sc.base) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->sc.base);
    }
    delete p;
}

}  // extern "C"
