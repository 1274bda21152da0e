// Drivers of the applications of Sec. 5.4 on the query pipeline:
//  - tessellation of trimmed surfaces (Sec. 5.4.3): the cell centres of a
//    uniform grid over each face's parameter rectangle are classified, so
//    that the cells (or the triangles built on them) outside the trimmed
//    region can be dropped;
//  - multiple patches (Sec. 5.4.1): a point sampled on a base surface is
//    inside when it lies inside any trimmed face that references the
//    surface; the points of a surface are gathered once per face that
//    references it (face-major, so each face's copy is one contiguous range
//    of the query), queried together, and the labels reduced per point.
// Both are HBM-bound gathers and scatters around one query launch.
#include "wn_host_internal.h"

#include <math.h>

#include <vector>

namespace wn {
namespace {

constexpr int kPatchWG = 256;

struct GridDev {
    double u0, v0, du, dv;
    int32_t nu, nv;
};

// First index i in [0, n) with offs[i + 1] > e (offs non-decreasing, e < offs[n]).
__device__ __forceinline__ int32_t owner(const int64_t* offs, int32_t n, int64_t e) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Sample k of the grids: face f = owner(k), row-major (i fastest) inside the
// face; u = u0 + (i + 1/2) du and v = v0 + (j + 1/2) dv with the product and
// the sum rounded separately (contraction into a fused multiply-add is off
// here), so a caller can rebuild the same coordinates.
__global__ __launch_bounds__(kPatchWG) void k_grid_samples(const GridDev* grids, const int64_t* offs, int32_t F,
                                                           int64_t total, double* u, double* v) {
#pragma clang fp contract(off)
    for (int64_t k = blockIdx.x * (int64_t)kPatchWG + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * kPatchWG) {
        const int32_t f = owner(offs, F, k);
        const GridDev g = grids[f];
        const int64_t r = k - offs[f];
        const int64_t j = r / g.nu, i = r - j * g.nu;
        u[k] = g.u0 + ((double)i + 0.5) * g.du;  // not contracted into an fma (pragma above)
        v[k] = g.v0 + ((double)j + 0.5) * g.dv;
    }
}

// Face-major copies of the surfaces' points: entry e of face f's range is
// point src_begin[f] + (e - dst_offs[f]).
__global__ __launch_bounds__(kPatchWG) void k_gather_points(const double* pu, const double* pv, int64_t stride,
                                                            const int64_t* src_begin, const int64_t* dst_offs,
                                                            int32_t F, int64_t total, double* u, double* v) {
    for (int64_t e = blockIdx.x * (int64_t)kPatchWG + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kPatchWG) {
        const int32_t f = owner(dst_offs, F, e);
        const int64_t s = src_begin[f] + (e - dst_offs[f]);
        u[e] = pu[s * stride];
        v[e] = pv[s * stride];
    }
}

// Label of point p of surface s from the labels of its copies: inside if any
// face labels it inside, else on-boundary if any face does, else invalid if
// its coordinates are invalid, else outside.  face_out (optional): the first
// face of the surface's list that labels it inside, or -1.
__global__ __launch_bounds__(kPatchWG) void k_reduce_surfaces(const int64_t* surf_offs, int32_t S,
                                                              const int32_t* sf_offs, const int32_t* sf_faces,
                                                              const int64_t* dst_offs, const uint8_t* lab_copy,
                                                              int64_t N, uint8_t* lab_out, int32_t* face_out) {
    for (int64_t p = blockIdx.x * (int64_t)kPatchWG + threadIdx.x; p < N; p += (int64_t)gridDim.x * kPatchWG) {
        const int32_t s = owner(surf_offs, S, p);
        const int64_t r = p - surf_offs[s];
        bool in = false, onb = false, bad = false;
        int32_t first = -1;
        for (int32_t k = sf_offs[s]; k < sf_offs[s + 1]; ++k) {
            const int32_t f = sf_faces[k];
            const uint8_t l = lab_copy[dst_offs[f] + r];
            if (l == WN_INSIDE && !in) {
                in = true;
                first = f;
            }
            onb |= l == WN_ON_BOUNDARY;
            bad |= l == WN_INVALID_POINT;
        }
        if (lab_out) lab_out[p] = in ? WN_INSIDE : (onb ? WN_ON_BOUNDARY : (bad ? WN_INVALID_POINT : WN_OUTSIDE));
        if (face_out) face_out[p] = first;
    }
}

int64_t patch_grid(const wn_faces* h, int64_t n) {
    const int64_t want = (n + kPatchWG - 1) / kPatchWG;
    const int64_t cap = (int64_t)(h->cu_count > 0 ? h->cu_count : 256) * 16;
    return want < 1 ? 1 : (want < cap ? want : cap);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace wn

using namespace wn;

extern "C" wn_status wn_classify_grid(const wn_faces* h, const wn_grid* grids, double* out_u, double* out_v,
                                      double* out_winding, uint8_t* out_inside, const wn_query_opts* q,
                                      void* stream) {
    if (!h || !grids) return WN_E_INVALID;
    const int32_t F = h->num_faces;
    if (F <= 0) return WN_E_INVALID;
    std::vector<int64_t> offs((size_t)F + 1, 0);
    std::vector<GridDev> g((size_t)F);
    for (int32_t f = 0; f < F; ++f) {
        const wn_grid& G = grids[f];
        if (G.nu < 0 || G.nv < 0 || !isfinite(G.u0) || !isfinite(G.v0) || !isfinite(G.du) || !isfinite(G.dv) ||
            !(G.du > 0.0) || !(G.dv > 0.0))
            return WN_E_INVALID;
        const int64_t n = (int64_t)G.nu * (int64_t)G.nv;
        offs[f + 1] = offs[f] + n;
        if (offs[f + 1] >= 0x7fffffffll) return WN_E_INVALID;
        g[f] = GridDev{G.u0, G.v0, G.du, G.dv, G.nu > 0 ? G.nu : 1, G.nv};
    }
    const int64_t N = offs[F];
    if (N == 0) return WN_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool own_uv = !out_u || !out_v;
    const size_t o_g = 0, o_o = align256(sizeof(GridDev) * F);
    const size_t o_u = o_o + align256(8 * ((size_t)F + 1));
    const size_t o_v = o_u + (own_uv ? align256(8 * (size_t)N) : 0);
    const size_t total = o_v + (own_uv ? align256(8 * (size_t)N) : 0);
    char* base = nullptr;
    hipError_t e = hipMallocAsync((void**)&base, total, st);
    if (e != hipSuccess) return WN_E_NOMEM;
    GridDev* d_g = (GridDev*)(base + o_g);
    int64_t* d_o = (int64_t*)(base + o_o);
    double* u = own_uv ? (double*)(base + o_u) : out_u;
    double* v = own_uv ? (double*)(base + o_v) : out_v;
    // the host tables are uploaded before the call returns
    e = hipMemcpyAsync(d_g, g.data(), sizeof(GridDev) * F, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_o, offs.data(), 8 * ((size_t)F + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_grid_samples, dim3((unsigned)patch_grid(h, N)), dim3(kPatchWG), 0, st, d_g, d_o, F, N,
                           u, v);
        e = hipGetLastError();
    }
    wn_status s = hip_status(e);
    if (s == WN_OK) {
        const wn_points p{N, u, v, 1, d_o, offs.data()};
        s = query_core(h, &p, out_winding, out_inside, q, nullptr, stream);
    }
    (void)hipFreeAsync(base, st);
    return s;
}

extern "C" wn_status wn_classify_surfaces(const wn_faces* h, int32_t num_surfaces,
                                          const int32_t* surface_face_offsets, const int32_t* surface_faces,
                                          const wn_points* points, uint8_t* out_inside, int32_t* out_face,
                                          const wn_query_opts* q, void* stream) {
    if (!h || !points || num_surfaces <= 0 || !surface_face_offsets || !surface_faces) return WN_E_INVALID;
    const int32_t F = h->num_faces, S = num_surfaces;
    const int64_t N = points->num_points;
    const int64_t* so = points->face_point_offsets_host;
    if (!so || !points->face_point_offsets || N < 0 || points->stride < 1) return WN_E_INVALID;
    if (N > 0 && (!points->u || !points->v)) return WN_E_INVALID;
    if (so[0] != 0 || so[S] != N) return WN_E_INVALID;
    for (int32_t s = 0; s < S; ++s)
        if (so[s + 1] < so[s]) return WN_E_INVALID;
    if (surface_face_offsets[0] != 0) return WN_E_INVALID;
    std::vector<int32_t> surf_of((size_t)F, -1);
    for (int32_t s = 0; s < S; ++s) {
        if (surface_face_offsets[s + 1] < surface_face_offsets[s]) return WN_E_INVALID;
        for (int32_t k = surface_face_offsets[s]; k < surface_face_offsets[s + 1]; ++k) {
            const int32_t f = surface_faces[k];
            if (f < 0 || f >= F || surf_of[f] != -1) return WN_E_INVALID;  // a face references one surface
            surf_of[f] = s;
        }
    }
    if (N == 0) return WN_OK;
    // face f's copy: the points of its surface (none for an unreferenced face)
    std::vector<int64_t> dst((size_t)F + 1, 0), src((size_t)F, 0);
    for (int32_t f = 0; f < F; ++f) {
        const int32_t s = surf_of[f];
        const int64_t n = s < 0 ? 0 : so[s + 1] - so[s];
        src[f] = s < 0 ? 0 : so[s];
        dst[f + 1] = dst[f] + n;
        if (dst[f + 1] >= 0x7fffffffll) return WN_E_INVALID;
    }
    const int64_t M = dst[F];
    const int32_t K = surface_face_offsets[S];
    hipStream_t st = (hipStream_t)stream;
    const size_t o_dst = 0, o_src = align256(8 * ((size_t)F + 1));
    const size_t o_sfo = o_src + align256(8 * (size_t)F);
    const size_t o_sff = o_sfo + align256(4 * ((size_t)S + 1));
    const size_t o_u = o_sff + align256(4 * (size_t)(K > 0 ? K : 1));
    const size_t o_v = o_u + align256(8 * (size_t)M);
    const size_t o_l = o_v + align256(8 * (size_t)M);
    const size_t total = o_l + align256((size_t)M);
    char* base = nullptr;
    hipError_t e = hipMallocAsync((void**)&base, total, st);
    if (e != hipSuccess) return WN_E_NOMEM;
    int64_t* d_dst = (int64_t*)(base + o_dst);
    int64_t* d_src = (int64_t*)(base + o_src);
    int32_t* d_sfo = (int32_t*)(base + o_sfo);
    int32_t* d_sff = (int32_t*)(base + o_sff);
    double* u = (double*)(base + o_u);
    double* v = (double*)(base + o_v);
    uint8_t* lab = (uint8_t*)(base + o_l);
    // the host tables are uploaded before the call returns
    e = hipMemcpyAsync(d_dst, dst.data(), 8 * ((size_t)F + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_src, src.data(), 8 * (size_t)F, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_sfo, surface_face_offsets, 4 * ((size_t)S + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && K > 0) e = hipMemcpyAsync(d_sff, surface_faces, 4 * (size_t)K, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && M > 0) {
        hipLaunchKernelGGL(k_gather_points, dim3((unsigned)patch_grid(h, M)), dim3(kPatchWG), 0, st, points->u,
                           points->v, points->stride, d_src, d_dst, F, M, u, v);
        e = hipGetLastError();
    }
    wn_status s = hip_status(e);
    if (s == WN_OK && M > 0) {
        // The host offsets go only to the plain schedule: for the batched one
        // they would turn on the overlap of near and far passes, which is
        // slower on surface sets (little near work against the far work:
        // 6.1 ms in series against 6.5 ms overlapped on 128 surfaces).
        const bool plain = ((q && q->schedule >= 0) ? q->schedule : h->schedule) == WN_SCHED_PLAIN;
        const wn_points p{M, u, v, 1, d_dst, plain ? dst.data() : nullptr};
        s = query_core(h, &p, nullptr, lab, q, nullptr, stream);
    }
    if (s == WN_OK && (out_inside || out_face)) {
        hipLaunchKernelGGL(k_reduce_surfaces, dim3((unsigned)patch_grid(h, N)), dim3(kPatchWG), 0, st,
                           points->face_point_offsets, S, d_sfo, d_sff, d_dst, lab, N, out_inside, out_face);
        s = hip_status(hipGetLastError());
    }
    (void)hipFreeAsync(base, st);
    return s;
}
