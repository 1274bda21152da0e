// Host-side internals shared by the library's host sources.
#pragma once

#include "../../include/wn.h"
#include "wn_internal.h"

#include <vector>

struct wn_faces {
    int device = 0;
    void* dmem = nullptr;
    int64_t dbytes = 0;
    wn::Segs sg{};
    wn::FaceTab ft_plan{};   // planar faces, largest first
    wn::FaceTab ft_per{};    // periodic faces, largest first
    wn::FaceTab ft_tree{};   // planar faces with a chain of >= kTreeAutoSegs segments (automatic hierarchy)
    wn::FaceTab ft_flat{};   // the other planar faces
    wn::PerTab pt{};
    wn::PathTree tree{};     // path hierarchy of the planar faces
    int32_t num_faces = 0, num_loops = 0, num_segments = 0;
    int32_t num_planar = 0, num_periodic = 0;
    int32_t max_spf = 0, max_depth = 0;
    double eps = 1e-10, eps2 = 1e-20;
    int precision = WN_PREC_FP64, rule = WN_RULE_NONZERO, schedule = WN_SCHED_BATCHED;
    int cu_count = 0;
    int bpc_far[2][3] = {{1, 1, 1}, {1, 1, 1}};  // resident workgroups per CU, k_far batched: [FP64, MIXED][64/128/256 points per workgroup]
    int bpc_farq[5] = {1, 1, 1, 1, 1}, bpc_far_tree = 1, bpc_far_wtree = 1, bpc_far_per = 1, bpc_redo_per = 1,
        bpc_near = 1;
    int bpc_near_cp = 1;
    std::vector<int32_t> h_seg_begin;
    std::vector<int32_t> h_dom;
    std::vector<int32_t> per_pos;  // position of each periodic face in ft_per.order
    std::vector<int32_t> h_ord_plan;  // ft_plan.order on the host
    std::vector<int32_t> h_ord_flat;  // ft_flat.order on the host
    std::vector<int32_t> h_ord_tree;  // ft_tree.order on the host
    std::vector<wn::PUnit> h_units;   // periodic units (torus pairs included) on the host
    std::vector<wn::PFace> h_pface;   // [F] periodic face records on the host (planar: zero)
    // side stream of the overlapped far/near passes (default priority); null
    // without WN_FLAG_OVERLAP or when it could not be created
    hipStream_t side = nullptr;
};

struct wn_profile {
    std::vector<hipEvent_t> ev;  // 2 per slot
    std::vector<int> kind;
    int used = 0;
};


struct wn_predictor {
    int device = 0;
    int cu_count = 256;
    float* d_master = nullptr;  // [P] FP32 master parameters
    float* d_m = nullptr;       // [P] AdamW first moment
    float* d_v = nullptr;       // [P] AdamW second moment
    float* d_wbf = nullptr;     // [P] BF16-rounded parameters used by the kernels
    float* d_norm = nullptr;    // [32] feature means, standard deviations
    uint16_t* d_w16 = nullptr;  // [kMlpFragSlots] W1, W2 as BF16 in matrix-core fragment order
    void* dmem = nullptr;
    int step = 0;
};

namespace wn {

// Per-call device scratch of the batched schedules.
struct Scratch {
    void* base = nullptr;
    int32_t* item_offs = nullptr;
    int2* item_map = nullptr;
    uint32_t* counters = nullptr;
    int64_t max_items = 0;
    NearQueue nq{};
    Out out{};
    const unsigned long long* near_lo = nullptr;  // set by an overlapped far pass: the final near pass starts here
    hipEvent_t near_join = nullptr;               // ... and waits for this (the side stream's near passes)
    uint32_t* perm = nullptr;  // spatial order of the periodic faces' points (periodic face sets)
    // binned schedule
    uint2* qs2 = nullptr;
    double2* sh2 = nullptr;
    uint8_t* bins = nullptr;
    uint32_t* wg_hist = nullptr;
    uint8_t* depth = nullptr;
    double* w_tmp = nullptr;
    uint8_t* lab_tmp = nullptr;
};

// Allocate (stream-ordered) scratch for N points; outputs the caller did
// not provide are allocated too.  binned adds the binning buffers.
// order: also hold a spatial order of the points (always held for periodic
// face sets; the path hierarchy's wave walk needs it for planar faces).
hipError_t scratch_alloc(const wn_faces* h, int64_t N, int64_t cap, bool binned, bool depth, double* out_w,
                         uint8_t* out_lab, int rule, Scratch& sc, hipStream_t st, bool stream_ordered,
                         bool order = false);
void scratch_free(Scratch& sc, hipStream_t st);

// Item build + persistent far passes (planar, periodic) filling sc.nq.  With
// host_offs (the host copy of the points' face offsets) the planar flat pass
// may overlap near passes on h->side and leave sc.near_lo for the final one.
// host_offs: the host offsets when the far/near overlap may run; counts_host:
// the host offsets whenever the caller gave them (the hierarchy reads the
// per-face point counts from them); stats: the query's work counters
// (WN_STAT_PERIODIC_PAIRS), or null.
hipError_t far_passes(const wn_faces* h, const Points& pts, int qpw, int policy, bool mixed, int tree, Scratch& sc,
                      wn_profile* prof, hipStream_t st, const int64_t* host_offs = nullptr,
                      const int64_t* counts_host = nullptr, unsigned long long* stats = nullptr);
// Near pass over nq; entry_depth optional.
hipError_t near_pass(const wn_faces* h, const Points& pts, NearQueue nq, Out out, unsigned long long* stats,
                     uint8_t* entry_depth, wn_profile* prof, hipStream_t st, unsigned long long* cursor,
                     bool cp_bound = false);

// Chunk cursor i (0..3) of a query's near passes, in the scratch counters
// (zeroed by the query's first item build).
inline unsigned long long* near_cursor(const Scratch& sc, int i) {
    return reinterpret_cast<unsigned long long*>(sc.counters + 24) + i;
}
int binning_grid(const wn_faces* h);

wn_status hip_status(hipError_t e);
wn_status query_core(const wn_faces* h, const wn_points* p, double* out_w, uint8_t* out_lab, const wn_query_opts* q,
                     Scratch* preset, void* stream);

}  // namespace wn
