// A batched query that allocates nothing: its scratch (work items, counters,
// near queue, spatial order of the points of periodic faces and of the faces
// the path hierarchy walks) lives in one file-scope
// device array of kNoAllocScratchBytes, laid out afresh by every call.
//
// The array's name is a host-side stand-in in host code, not a device
// address: the address is taken once per device with hipGetSymbolAddress (with
// that device current) and only that pointer is handed to kernels.  Every
// call on a device shares the device's array: calls that overlap on one
// device race (one stream per device at a time).  Nothing in the array has to
// start at zero: the item build kernel of each call resets the counters it
// uses, and the queue is written before it is read.
#include "wn_host_internal.h"

#include <mutex>

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev (resolved once per device).
hipError_t scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        const hipError_t er = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return e;
        if (er != hipSuccess) return er;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

using namespace wn;

extern "C" {

int64_t wn_query_noalloc_scratch_bytes(void) { return (int64_t)kNoAllocScratchBytes; }

wn_status wn_query_noalloc(const wn_faces* h, const wn_points* p, double* out_w, uint8_t* out_lab,
                           const wn_query_opts* qo, void* stream) {
    if (!h || !p || !out_w || !out_lab) return WN_E_INVALID;
    wn_query_opts q;
    wn_default_query_opts(&q);
    if (qo) q = *qo;
    const int sched = q.schedule >= 0 ? q.schedule : h->schedule;
    if (sched != WN_SCHED_BATCHED) return WN_E_UNSUPPORTED;
    const int64_t N = p->num_points;
    if (N < 0 || N > WN_NOALLOC_MAX_POINTS || h->num_faces > WN_NOALLOC_MAX_FACES) return WN_E_INVALID;
    if (N == 0) return WN_OK;
    const int32_t F = h->num_faces;
    const bool periodic = h->num_periodic > 0;
    const bool ordered = periodic || q.path_hierarchy != 0;
    // layout: item offsets, item map, counters, spatial order, then the near
    // queue (entries, and their copy shifts for periodic face sets) in the rest
    Scratch sc;
    sc.max_items = N / 64 + F + 1;
    const size_t o_io = 0;
    const size_t o_im = o_io + align256(((size_t)F + 1) * 4);
    const size_t o_ct = o_im + align256((size_t)sc.max_items * 8);
    const size_t o_pm = o_ct + 256;
    const size_t o_nq = o_pm + (ordered ? align256((size_t)N * 4) : 0);
    if (o_nq >= kNoAllocScratchBytes) return WN_E_INVALID;
    const size_t per_entry = periodic ? 8 + 16 : 8;
    int64_t cap = (int64_t)((kNoAllocScratchBytes - o_nq - 256) / per_entry);
    if (q.near_capacity > 0 && q.near_capacity < cap) cap = q.near_capacity;
    if (cap < 65536) return WN_E_INVALID;  // a queue this small would send most near pairs to the in-line redo
    const size_t o_sh = o_nq + align256((size_t)cap * 8);
    void* base = nullptr;
    hipError_t e = scratch_address(h->device, &base);
    if (e != hipSuccess) return hip_status(e);
    char* b = (char*)base;
    sc.base = nullptr;  // not owned
    sc.item_offs = (int32_t*)(b + o_io);
    sc.item_map = (int2*)(b + o_im);
    sc.counters = (uint32_t*)(b + o_ct);
    sc.perm = ordered ? (uint32_t*)(b + o_pm) : nullptr;
    sc.nq = NearQueue{(uint2*)(b + o_nq), periodic ? (double2*)(b + o_sh) : nullptr,
                      (unsigned long long*)(sc.counters + 2), (uint64_t)cap};
    q.near_capacity = cap;
    return query_core(h, p, out_w, out_lab, &q, &sc, stream);
}

}  // extern "C"
