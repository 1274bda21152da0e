// Host side of the winding-number library: validation, per-segment bounds,
// device packing and query scheduling behind the C ABI of include/wn.h.
#include "wn_host_internal.h"
#include "wn_learn.h"
#include "wn_topology.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <new>
#include <numeric>
#include <vector>

using namespace wn;

namespace wn {
wn_status hip_status(hipError_t e) {
    if (e == hipSuccess) return WN_OK;
    if (e == hipErrorOutOfMemory) return WN_E_NOMEM;
    return WN_E_DEVICE;
}
}  // namespace wn

namespace {

// Records an event pair around one launch when a profile with room is given.
struct ProfScope {
    wn_profile* p;
    int slot = -1;
    hipStream_t st;
    ProfScope(wn_profile* prof, int k, hipStream_t s) : p(prof), st(s) {
        if (p && p->used < (int)p->kind.size()) {
            slot = p->used++;
            p->kind[slot] = k;
            (void)hipEventRecord(p->ev[2 * slot], st);
        }
    }
    ~ProfScope() {
        if (slot >= 0) (void)hipEventRecord(p->ev[2 * slot + 1], st);
    }
};

constexpr int kBinom[kCoef][kCoef] = {{1, 0, 0, 0, 0, 0}, {1, 1, 0, 0, 0, 0},  {1, 2, 1, 0, 0, 0},
                                      {1, 3, 3, 1, 0, 0}, {1, 4, 6, 4, 1, 0}, {1, 5, 10, 10, 5, 1}};

bool finite_small(double x) { return isfinite(x) && fabs(x) < kCoordLimit; }


// Lemma 1 / App. A.1 bound for one segment (no validation).
double segment_bound(const double* u, const double* v, const double* w, int n) {
    double maxd = 0.0;  // max_i |P_i - P_{i-1}|
    for (int i = 1; i <= n; ++i) maxd = std::max(maxd, hypot(u[i] - u[i - 1], v[i] - v[i - 1]));
    if (!w) return n * maxd;
    double wmin = w[0], wmax = w[0];
    for (int i = 1; i <= n; ++i) {
        wmin = std::min(wmin, w[i]);
        wmax = std::max(wmax, w[i]);
    }
    bool unit = true;
    for (int i = 0; i <= n; ++i) unit = unit && (w[i] == 1.0);
    if (unit) return n * maxd;
    double diam = 0.0;  // max_{i,j} |P_i - P_j|
    for (int i = 0; i <= n; ++i)
        for (int j = i + 1; j <= n; ++j) diam = std::max(diam, hypot(u[i] - u[j], v[i] - v[j]));
    const double r = wmax / wmin;
    const double b1 = n * r * diam;
    const double b2 = n * r * r * maxd;
    // a few ulps of slack for the rounding of the products above
    return std::min(b1, b2) * (1.0 + 8.0 * 2.220446049250313e-16);
}

}  // namespace

extern "C" {

const char* wn_status_string(wn_status s) {
    switch (s) {
        case WN_OK: return "ok";
        case WN_E_INVALID: return "invalid argument or descriptor";
        case WN_E_NOMEM: return "out of memory";
        case WN_E_DEVICE: return "HIP device error";
        case WN_E_TOPOLOGY: return "periodic loops violate the pairing proposition";
        case WN_E_DEPTH: return "recursion depth bound exceeds the stack cap";
        case WN_E_UNSUPPORTED: return "unsupported option combination";
    }
    return "unknown status";
}

void wn_default_options(wn_options* opt) {
    if (!opt) return;
    opt->eps = 1e-10;
    opt->precision = WN_PREC_FP64;
    opt->rule = WN_RULE_NONZERO;
    opt->schedule = WN_SCHED_BATCHED;
    opt->stack_cap = kDepthCap;
    opt->flags = 0;
}

void wn_default_query_opts(wn_query_opts* q) {
    if (!q) return;
    memset(q, 0, sizeof(*q));
    q->schedule = -1;
    q->precision = -1;
    q->rule = -1;
}

wn_status wn_segment_bound(const double* cp_u, const double* cp_v, const double* cp_w, int32_t degree,
                           double* out_B) {
    if (!cp_u || !cp_v || !out_B || degree < 1 || degree > kMaxDeg) return WN_E_INVALID;
    for (int i = 0; i <= degree; ++i) {
        if (!finite_small(cp_u[i]) || !finite_small(cp_v[i])) return WN_E_INVALID;
        if (cp_w && !(cp_w[i] > 0.0 && isfinite(cp_w[i]))) return WN_E_INVALID;
    }
    *out_B = segment_bound(cp_u, cp_v, cp_w, degree);
    return WN_OK;
}

wn_status wn_create_faces(const wn_faces_desc* d, const wn_options* opt_in, void* stream, wn_faces** out) {
    if (!d || !out) return WN_E_INVALID;
    *out = nullptr;
    wn_options opt;
    wn_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!(opt.eps >= 1e-15 && opt.eps <= 1e-2)) return WN_E_INVALID;
    if (opt.stack_cap < 1 || opt.stack_cap > kDepthCap) return WN_E_INVALID;
    if (opt.precision < 0 || opt.precision > WN_PREC_MIXED) return WN_E_INVALID;
    if (opt.rule < 0 || opt.rule > WN_RULE_POSITIVE) return WN_E_INVALID;
    if (opt.schedule < 0 || opt.schedule > WN_SCHED_BINNED) return WN_E_INVALID;
    if (opt.flags & ~(int32_t)(WN_FLAG_HOST_PAIRING | WN_FLAG_OVERLAP)) return WN_E_INVALID;
    const int32_t F = d->num_faces, L = d->num_loops, S = d->num_segments;
    if (F < 0 || L < 0 || S < 0) return WN_E_INVALID;
    if (!d->face_loop_offsets || !d->loop_seg_offsets || !d->seg_cp_offsets) return WN_E_INVALID;
    if (S > 0 && (!d->cp_u || !d->cp_v)) return WN_E_INVALID;
    // CSR structure
    if (d->face_loop_offsets[0] != 0 || d->face_loop_offsets[F] != L) return WN_E_INVALID;
    for (int32_t f = 0; f < F; ++f)
        if (d->face_loop_offsets[f + 1] < d->face_loop_offsets[f]) return WN_E_INVALID;
    if (d->loop_seg_offsets[0] != 0 || d->loop_seg_offsets[L] != S) return WN_E_INVALID;
    for (int32_t l = 0; l < L; ++l)
        if (d->loop_seg_offsets[l + 1] < d->loop_seg_offsets[l]) return WN_E_INVALID;
    if (d->seg_cp_offsets[0] != 0 || d->seg_cp_offsets[S] != d->num_cps) return WN_E_INVALID;
    for (int32_t s = 0; s < S; ++s) {
        const int64_t n = d->seg_cp_offsets[s + 1] - d->seg_cp_offsets[s] - 1;
        if (n < 1 || n > kMaxDeg) return WN_E_INVALID;
    }
    for (int64_t i = 0; i < d->num_cps; ++i) {
        if (!finite_small(d->cp_u[i]) || !finite_small(d->cp_v[i])) return WN_E_INVALID;
        if (d->cp_w && !(d->cp_w[i] > 0.0 && isfinite(d->cp_w[i]) && d->cp_w[i] < 1e100)) return WN_E_INVALID;
    }
    std::vector<int32_t> dom((size_t)F, WN_DOMAIN_PLANE);
    int32_t nper = 0;
    for (int32_t f = 0; f < F; ++f) {
        dom[f] = d->face_domain ? d->face_domain[f] : WN_DOMAIN_PLANE;
        if (dom[f] < WN_DOMAIN_PLANE || dom[f] > WN_DOMAIN_CONE_U) return WN_E_INVALID;
        if (dom[f] != WN_DOMAIN_PLANE) {
            if (!d->face_period) return WN_E_INVALID;
            const double Tu = d->face_period[2 * f], Tv = d->face_period[2 * f + 1];
            if (!(Tu > 0.0 && Tu < 1e6) || (dom[f] == WN_DOMAIN_TORUS && !(Tv > 0.0 && Tv < 1e6))) return WN_E_INVALID;
            ++nper;
        }
    }

    wn_faces* h = new (std::nothrow) wn_faces();
    if (!h) return WN_E_NOMEM;
    h->num_faces = F;
    h->num_loops = L;
    h->num_segments = S;
    h->num_periodic = nper;
    h->num_planar = F - nper;
    h->eps = opt.eps;
    h->eps2 = opt.eps * opt.eps;
    h->precision = opt.precision;
    h->rule = opt.rule;
    h->schedule = opt.schedule;
    h->h_dom = dom;

    // per face: segment range, scale of the rounding margin
    h->h_seg_begin.resize((size_t)F + 1);
    std::vector<double> face_scale((size_t)F, 0.0);
    for (int32_t f = 0; f <= F; ++f) h->h_seg_begin[f] = d->loop_seg_offsets[d->face_loop_offsets[f]];
    for (int32_t f = 0; f < F; ++f) {
        const int32_t a = h->h_seg_begin[f], b = h->h_seg_begin[f + 1];
        h->max_spf = std::max(h->max_spf, b - a);
        double m = 0.0;
        for (int64_t i = d->seg_cp_offsets[a]; i < d->seg_cp_offsets[b]; ++i)
            m = std::max(m, std::max(fabs(d->cp_u[i]), fabs(d->cp_v[i])));
        face_scale[f] = m;
    }

    // per segment host arrays
    std::vector<double> p0x(S), p0y(S), pnx(S), pny(S), hb2(S), Bv(S), eta(S);
    std::vector<double> coef((size_t)S * kCoef * 4, 0.0);
    std::vector<uint8_t> deg(S), rat(S), segper(S, 0);
    std::vector<double> box((size_t)S * 4);
    std::vector<float> wrange((size_t)S * 2);
    int32_t maxd = 0;
    for (int32_t f = 0; f < F; ++f) {
        const double e = 8.0 * 1.1102230246251565e-16 * (1.0 + face_scale[f]);
        for (int32_t s = h->h_seg_begin[f]; s < h->h_seg_begin[f + 1]; ++s) {
            const int64_t c0 = d->seg_cp_offsets[s];
            const int n = (int)(d->seg_cp_offsets[s + 1] - c0 - 1);
            const double* u = d->cp_u + c0;
            const double* v = d->cp_v + c0;
            const double* w = d->cp_w ? d->cp_w + c0 : nullptr;
            bool is_rat = false;
            if (w)
                for (int i = 0; i <= n; ++i) is_rat = is_rat || (w[i] != 1.0);
            const double B = segment_bound(u, v, is_rat ? w : nullptr, n);
            // Termination lemma: depth <= ceil(log2(B/eps)) + 2 (+1 for the rounding margins)
            const int D = B > 0.0 ? (int)ceil(log2(B / opt.eps)) + 3 : 1;
            maxd = std::max(maxd, D);
            p0x[s] = u[0];
            p0y[s] = v[0];
            pnx[s] = u[n];
            pny[s] = v[n];
            Bv[s] = B;
            eta[s] = e;
            const double Be = B * (1.0 + kAxisInflate) + e;
            hb2[s] = 0.5 * Be * Be;
            deg[s] = (uint8_t)n;
            rat[s] = is_rat ? 1 : 0;
            segper[s] = dom[f] != WN_DOMAIN_PLANE ? 1 : 0;
            double* bx = &box[4 * (size_t)s];
            bx[0] = bx[1] = u[0];
            bx[2] = bx[3] = v[0];
            float wl = 1.f, wh = 1.f;
            if (is_rat) wl = wh = (float)w[0];
            for (int i = 0; i <= n; ++i) {
                bx[0] = std::min(bx[0], u[i]);
                bx[1] = std::max(bx[1], u[i]);
                bx[2] = std::min(bx[2], v[i]);
                bx[3] = std::max(bx[3], v[i]);
                if (is_rat) {
                    wl = std::min(wl, (float)w[i]);
                    wh = std::max(wh, (float)w[i]);
                }
            }
            wrange[2 * (size_t)s] = wl;
            wrange[2 * (size_t)s + 1] = wh;
            for (int i = 0; i <= n; ++i) {  // slot i: C(n,i) w_i (P_i, 1); slots above n stay zero
                const double wi = is_rat ? w[i] : 1.0;
                const double c = (double)kBinom[n][i] * wi;
                double* slot = &coef[((size_t)s * kCoef + i) * 4];
                slot[0] = c * u[i];
                slot[1] = c * v[i];
                slot[2] = c;
                slot[3] = 0.0;
            }
            // the near pass's per-segment data in the slots' fourth components
            const double pads[kCoef] = {B, e, u[0], v[0], u[n], v[n]};
            for (int j = 0; j < kCoef; ++j) coef[((size_t)s * kCoef + j) * 4 + 3] = pads[j];
        }
    }
    std::vector<uint8_t> join(S, 0);
    for (int32_t s = 1; s < S; ++s) join[s] = (p0x[s] == pnx[s - 1] && p0y[s] == pny[s - 1]) ? 1 : 0;

    // path hierarchy of the planar faces: per chain of joined segments, a
    // balanced binary tree of subpaths in preorder.  An inner node's axis is
    // the sum of its segments' inflated axes, inflated once more, so that its
    // ellipse contains every descendant's (triangle inequality) with a margin
    // for the rounding of the tests.
    std::vector<TNode> tree;
    std::vector<int32_t> tree_begin((size_t)F + 1, 0);
    {
        std::function<double(int32_t, int32_t, bool)> build = [&](int32_t lo, int32_t hi, bool root) -> double {
            const size_t at = tree.size();
            tree.push_back(TNode{});
            double axis;
            if (hi - lo == 1) {
                axis = Bv[lo] * (1.0 + kAxisInflate) + eta[lo];
                tree[at].hb2 = hb2[lo];
                tree[at].seg = lo;
            } else {
                const int32_t mid = lo + (hi - lo) / 2;
                axis = build(lo, mid, false) + build(mid, hi, false);
                const double a = axis * (1.0 + kAxisInflate);
                tree[at].hb2 = 0.5 * a * a;
                tree[at].seg = -1;
            }
            tree[at].sx = p0x[lo];
            tree[at].sy = p0y[lo];
            tree[at].ex = pnx[hi - 1];
            tree[at].ey = pny[hi - 1];
            tree[at].skip = (int32_t)tree.size() | (root ? kTreeRoot : 0);
            return axis;
        };
        for (int32_t f = 0; f < F; ++f) {
            tree_begin[f] = (int32_t)tree.size();
            if (dom[f] != WN_DOMAIN_PLANE) continue;
            const int32_t a = h->h_seg_begin[f], b = h->h_seg_begin[f + 1];
            for (int32_t c0 = a; c0 < b;) {
                int32_t c1 = c0 + 1;
                while (c1 < b && join[c1]) ++c1;
                (void)build(c0, c1, true);
                c0 = c1;
            }
        }
        tree_begin[F] = (int32_t)tree.size();
        if (tree.size() > (size_t)INT32_MAX / 2) {
            delete h;
            return WN_E_INVALID;
        }
    }
    // LDS chunks: consecutive whole chains of a face, at most kTreeChunk nodes
    // (a longer chain is a chunk of its own)
    std::vector<int2> tchunk;
    std::vector<int32_t> tchunk_begin((size_t)F + 1, 0);
    for (int32_t f = 0; f < F; ++f) {
        tchunk_begin[f] = (int32_t)tchunk.size();
        int32_t lo = tree_begin[f];
        for (int32_t r = tree_begin[f]; r < tree_begin[f + 1]; r = tree[r].skip & ~kTreeRoot) {
            const int32_t end = tree[r].skip & ~kTreeRoot;  // the chain rooted at r is [r, end)
            if (end - lo > kTreeChunk && r > lo) {
                tchunk.push_back(make_int2(lo, r));
                lo = r;
            }
        }
        if (tree_begin[f + 1] > lo) tchunk.push_back(make_int2(lo, tree_begin[f + 1]));
    }
    tchunk_begin[F] = (int32_t)tchunk.size();
    h->max_depth = maxd;
    if (maxd > opt.stack_cap) {
        delete h;
        return WN_E_DEPTH;
    }
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
        delete h;
        return WN_E_DEVICE;
    }
    // resident workgroups per CU of the persistent kernels (queried once, so
    // that a captured query issues no host queries)
    for (int m = 0; m < 2; ++m) {
        h->bpc_far[m][0] = far_blocks_per_cu(false, m == 1, 64);
        h->bpc_far[m][1] = far_blocks_per_cu(false, m == 1, 128);
        h->bpc_far[m][2] = far_blocks_per_cu(false, m == 1, 256);
    }
    h->bpc_far_tree = far_tree_blocks_per_cu();
    h->bpc_far_wtree = far_wtree_blocks_per_cu();
    for (int qpl = 2; qpl <= 4; ++qpl) h->bpc_farq[qpl] = farq_blocks_per_cu(qpl);
    h->bpc_far_per = far_periodic_blocks_per_cu(kPerQueue);
    h->bpc_redo_per = far_periodic_blocks_per_cu(kPerRedo);
    h->bpc_near = near_blocks_per_cu();
    h->bpc_near_cp = near_cp_blocks_per_cu();

    // faces ordered by segment count (largest first) for the work queues (the
    // periodic faces are ordered again by their copies once these are known)
    std::vector<int32_t> ord_plan, ord_per;
    for (int32_t f = 0; f < F; ++f) (dom[f] == WN_DOMAIN_PLANE ? ord_plan : ord_per).push_back(f);
    auto by_size = [&](int32_t a, int32_t b) {
        return (h->h_seg_begin[a + 1] - h->h_seg_begin[a]) > (h->h_seg_begin[b + 1] - h->h_seg_begin[b]);
    };
    std::stable_sort(ord_plan.begin(), ord_plan.end(), by_size);
    h->h_ord_plan = ord_plan;
    // automatic hierarchy: faces with a chain of at least kTreeAutoSegs segments
    // take the tree walk, the others the flat scan
    std::vector<int32_t> ord_tree, ord_flat;
    for (int32_t f : ord_plan) {
        int32_t longest = 0;
        for (int32_t r = tree_begin[f]; r < tree_begin[f + 1]; r = tree[r].skip & ~kTreeRoot)
            longest = std::max(longest, ((tree[r].skip & ~kTreeRoot) - r + 1) / 2);  // 2m - 1 nodes
        (longest >= kTreeAutoSegs ? ord_tree : ord_flat).push_back(f);
    }
    h->h_ord_flat = ord_flat;
    h->h_ord_tree = ord_tree;
    std::stable_sort(ord_per.begin(), ord_per.end(), by_size);
    h->per_pos.assign((size_t)F, 0);
    for (size_t r = 0; r < ord_per.size(); ++r) h->per_pos[ord_per[r]] = (int32_t)r;

    // one device allocation, 256-byte aligned sub-buffers
    struct Part {
        const void* src;
        size_t bytes;
        size_t off;
    };
    std::vector<Part> parts;
    size_t total = 0;
    auto add = [&](const void* src, size_t bytes) -> size_t {
        const size_t off = total;
        parts.push_back({src, bytes, off});
        total += (bytes + 255) & ~(size_t)255;
        return off;
    };
    const size_t o_p0x = add(p0x.data(), S * 8), o_p0y = add(p0y.data(), S * 8);
    const size_t o_pnx = add(pnx.data(), S * 8), o_pny = add(pny.data(), S * 8);
    const size_t o_hb2 = add(hb2.data(), S * 8), o_B = add(Bv.data(), S * 8), o_eta = add(eta.data(), S * 8);
    const size_t o_coef = add(coef.data(), coef.size() * 8);
    const size_t o_deg = add(deg.data(), S), o_rat = add(rat.data(), S), o_sper = add(segper.data(), S);
    const size_t o_box = add(box.data(), box.size() * 8), o_wr = add(wrange.data(), wrange.size() * 4);
    const size_t o_join = add(join.data(), S);
    const size_t o_tree = add(tree.data(), tree.size() * sizeof(TNode));
    const size_t o_tbeg = add(tree_begin.data(), tree_begin.size() * 4);
    const size_t o_tch = add(tchunk.data(), tchunk.size() * sizeof(int2));
    const size_t o_tchb = add(tchunk_begin.data(), tchunk_begin.size() * 4);
    const size_t o_sb = add(h->h_seg_begin.data(), ((size_t)F + 1) * 4);
    const size_t o_op = add(ord_plan.data(), ord_plan.size() * 4), o_oq = add(ord_per.data(), ord_per.size() * 4);
    const size_t o_ot = add(ord_tree.data(), ord_tree.size() * 4), o_of = add(ord_flat.data(), ord_flat.size() * 4);
    // periodic tables (filled after the lift)
    const size_t o_ploop = add(nullptr, nper ? (size_t)L * sizeof(PLoop) : 0);
    const size_t o_pface = add(nullptr, nper ? (size_t)F * sizeof(PFace) : 0);
    const size_t o_punit = add(nullptr, nper ? (size_t)(2 * L + 1) * sizeof(PUnit) : 0);
    const size_t o_frec = add(nullptr, nper ? (size_t)S * sizeof(FarRec) : 0);
    if (total == 0) total = 256;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMalloc(&h->dmem, total);
    if (e != hipSuccess) {
        delete h;
        return hip_status(e);
    }
    h->dbytes = (int64_t)total;
    char* base = (char*)h->dmem;
    for (const Part& p : parts) {
        if (p.bytes == 0 || !p.src) continue;
        e = hipMemcpyAsync(base + p.off, p.src, p.bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    auto fail = [&](wn_status code) {
        (void)hipFree(h->dmem);
        delete h;
        return code;
    };
    if (e != hipSuccess) return fail(hip_status(e));
    h->sg.p0x = (const double*)(base + o_p0x);
    h->sg.p0y = (const double*)(base + o_p0y);
    h->sg.pnx = (const double*)(base + o_pnx);
    h->sg.pny = (const double*)(base + o_pny);
    h->sg.hb2 = (const double*)(base + o_hb2);
    h->sg.B = (const double*)(base + o_B);
    h->sg.eta = (const double*)(base + o_eta);
    h->sg.coef = (const double*)(base + o_coef);
    h->sg.deg = (const uint8_t*)(base + o_deg);
    h->sg.rat = (const uint8_t*)(base + o_rat);
    h->sg.box = (const double*)(base + o_box);
    h->sg.wrange = (const float*)(base + o_wr);
    h->sg.join = (const uint8_t*)(base + o_join);
    h->sg.frec = nper ? (const FarRec*)(base + o_frec) : nullptr;
    h->tree = PathTree{(const TNode*)(base + o_tree), (const int32_t*)(base + o_tbeg), (const int2*)(base + o_tch),
                       (const int32_t*)(base + o_tchb)};
    const int32_t* d_sb = (const int32_t*)(base + o_sb);
    h->ft_plan = FaceTab{d_sb, (const int32_t*)(base + o_op), (int32_t)ord_plan.size()};
    h->ft_tree = FaceTab{d_sb, (const int32_t*)(base + o_ot), (int32_t)ord_tree.size()};
    h->ft_flat = FaceTab{d_sb, (const int32_t*)(base + o_of), (int32_t)ord_flat.size()};
    h->ft_per = FaceTab{d_sb, (const int32_t*)(base + o_oq), (int32_t)ord_per.size()};
    h->pt.seg_periodic = (const uint8_t*)(base + o_sper);

    if (nper > 0) {
        // ---- covering-space lift on the GPU (k_lift), read back for the topology
        std::vector<int32_t> lift_loops, loop_face((size_t)L, 0);
        for (int32_t f = 0; f < F; ++f)
            for (int32_t l = d->face_loop_offsets[f]; l < d->face_loop_offsets[f + 1]; ++l) {
                loop_face[l] = f;
                if (dom[f] != WN_DOMAIN_PLANE) lift_loops.push_back(l);
            }
        std::vector<double> per2((size_t)2 * F, 0.0);
        for (int32_t f = 0; f < F; ++f)
            if (dom[f] != WN_DOMAIN_PLANE) {
                per2[2 * f] = d->face_period[2 * f];
                per2[2 * f + 1] = d->face_period[2 * f + 1];
            }
        size_t tt = 0;
        auto tk = [&](size_t bytes) {
            const size_t off = tt;
            tt += (bytes + 255) & ~(size_t)255;
            return off;
        };
        const size_t t_loops = tk(lift_loops.size() * 4), t_lf = tk((size_t)L * 4), t_dom = tk((size_t)F * 4);
        const size_t t_per = tk((size_t)F * 16), t_ls = tk(((size_t)L + 1) * 4), t_sc = tk(((size_t)S + 1) * 8);
        const size_t t_cu = tk((size_t)d->num_cps * 8), t_cv = tk((size_t)d->num_cps * 8);
        const size_t t_off = tk((size_t)S * 16);
        void* tmp = nullptr;
        e = hipMalloc(&tmp, tt ? tt : 256);
        if (e != hipSuccess) return fail(hip_status(e));
        char* tb = (char*)tmp;
        const std::pair<size_t, std::pair<const void*, size_t>> ups[] = {
            {t_loops, {lift_loops.data(), lift_loops.size() * 4}},
            {t_lf, {loop_face.data(), (size_t)L * 4}},
            {t_dom, {dom.data(), (size_t)F * 4}},
            {t_per, {per2.data(), (size_t)F * 16}},
            {t_ls, {d->loop_seg_offsets, ((size_t)L + 1) * 4}},
            {t_sc, {d->seg_cp_offsets, ((size_t)S + 1) * 8}},
            {t_cu, {d->cp_u, (size_t)d->num_cps * 8}},
            {t_cv, {d->cp_v, (size_t)d->num_cps * 8}},
        };
        for (const auto& u : ups)
            if (e == hipSuccess && u.second.second)
                e = hipMemcpyAsync(tb + u.first, u.second.first, u.second.second, hipMemcpyHostToDevice, st);
        PLoop* d_ploop = (PLoop*)(base + o_ploop);
        LiftArgs la{(const int32_t*)(tb + t_loops), (int32_t)lift_loops.size(), (const int32_t*)(tb + t_lf),
                    (const int32_t*)(tb + t_dom), (const double*)(tb + t_per), (const int32_t*)(tb + t_ls),
                    (const int64_t*)(tb + t_sc), (const double*)(tb + t_cu), (const double*)(tb + t_cv),
                    (double*)(tb + t_off), d_ploop};
        if (e == hipSuccess) e = hipMemsetAsync(d_ploop, 0, (size_t)L * sizeof(PLoop), st);
        if (e == hipSuccess) e = launch_lift(la, h->sg, st);
        std::vector<PLoop> ploop((size_t)L);
        std::vector<double> seg_off((size_t)2 * S, 0.0);
        if (e == hipSuccess) e = hipMemcpyAsync(ploop.data(), d_ploop, (size_t)L * sizeof(PLoop), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(seg_off.data(), tb + t_off, (size_t)S * 16, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(tmp);
        if (e != hipSuccess) return fail(hip_status(e));

        // ---- loop classes, homology checks, pairing (host)
        std::vector<HostSeg> hsegs((size_t)S);
        for (int32_t f = 0; f < F; ++f) {
            if (dom[f] == WN_DOMAIN_PLANE) continue;
            for (int32_t s = h->h_seg_begin[f]; s < h->h_seg_begin[f + 1]; ++s) {
                const int64_t c0 = d->seg_cp_offsets[s];
                HostSeg& g = hsegs[s];
                g.n = deg[s];
                g.B = Bv[s];
                for (int i = 0; i <= g.n; ++i) {
                    g.x[i] = d->cp_u[c0 + i] + seg_off[2 * s];
                    g.y[i] = d->cp_v[c0 + i] + seg_off[2 * s + 1];
                    g.w[i] = (rat[s] && d->cp_w) ? d->cp_w[c0 + i] : 1.0;
                }
            }
        }
        // rounding margin for the magnitudes met by translated copies
        auto face_margin = [&](int32_t f, double t1x, double t1y) {
            double reach = fabs(t1x) + fabs(t1y) + 2.0 * (d->face_period[2 * f] + d->face_period[2 * f + 1]);
            for (int32_t l = d->face_loop_offsets[f]; l < d->face_loop_offsets[f + 1]; ++l)
                reach = std::max(reach, 3.0 * ploop[l].lv + 4.0 * (fabs(ploop[l].bb[0]) + fabs(ploop[l].bb[1]) +
                                                                   fabs(ploop[l].bb[2]) + fabs(ploop[l].bb[3])));
            return 8.0 * 1.1102230246251565e-16 * (1.0 + face_scale[f] + reach);
        };
        // loop classes and homology (host), torus pairing (GPU by default)
        std::vector<TorusSetup> tsu((size_t)F);
        for (int32_t f = 0; f < F; ++f) {
            if (dom[f] == WN_DOMAIN_PLANE) continue;
            if (torus_setup(dom[f], d->face_period[2 * f], d->face_period[2 * f + 1], d->face_loop_offsets[f],
                            d->face_loop_offsets[f + 1], ploop, tsu[f]) != 0)
                return fail(WN_E_TOPOLOGY);
        }
        std::vector<int2> choice;
        std::vector<int32_t> choice_at((size_t)F, -1);
        if (!(opt.flags & WN_FLAG_HOST_PAIRING)) {
            std::vector<PairJob> jobs;
            std::vector<int32_t> lists;
            for (int32_t f = 0; f < F; ++f) {
                const TorusSetup& t = tsu[f];
                if (dom[f] != WN_DOMAIN_TORUS || t.A.empty() || t.B.size() > 64) continue;  // (larger: host)
                PairJob J{};
                J.a0 = (int32_t)lists.size();
                J.na = (int32_t)t.A.size();
                lists.insert(lists.end(), t.A.begin(), t.A.end());
                J.b0 = (int32_t)lists.size();
                J.nb = (int32_t)t.B.size();
                lists.insert(lists.end(), t.B.begin(), t.B.end());
                J.out0 = (int32_t)choice.size();
                J.t1x = t.t1x;
                J.t1y = t.t1y;
                J.nx = t.nx;
                J.ny = t.ny;
                J.Delta = t.Delta;
                J.eta = face_margin(f, t.t1x, t.t1y);
                choice_at[f] = J.out0;
                choice.resize(choice.size() + t.A.size(), make_int2(-1, 0));
                jobs.push_back(J);
            }
            if (!jobs.empty()) {
                const size_t b_jobs = ((jobs.size() * sizeof(PairJob)) + 255) & ~(size_t)255;
                const size_t b_lists = ((lists.size() * 4) + 255) & ~(size_t)255;
                void* ptmp = nullptr;
                e = hipMalloc(&ptmp, b_jobs + b_lists + choice.size() * sizeof(int2));
                if (e != hipSuccess) return fail(hip_status(e));
                char* pb = (char*)ptmp;
                e = hipMemcpyAsync(pb, jobs.data(), jobs.size() * sizeof(PairJob), hipMemcpyHostToDevice, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(pb + b_jobs, lists.data(), lists.size() * 4, hipMemcpyHostToDevice, st);
                if (e == hipSuccess)
                    e = launch_pair_torus(h->sg, d_ploop, (const PairJob*)pb, (int)jobs.size(),
                                          (const int32_t*)(pb + b_jobs), (int2*)(pb + b_jobs + b_lists), h->eps2, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(choice.data(), pb + b_jobs + b_lists, choice.size() * sizeof(int2),
                                       hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                (void)hipFree(ptmp);
                if (e != hipSuccess) return fail(hip_status(e));
            }
        }
        std::vector<PUnit> units;
        std::vector<PFace> pface((size_t)F);
        for (int32_t f = 0; f < F; ++f) {
            if (dom[f] == WN_DOMAIN_PLANE) continue;
            const int2* ch = choice_at[f] >= 0 ? choice.data() + choice_at[f] : nullptr;
            if (build_periodic_face(dom[f], d->face_period[2 * f], d->face_period[2 * f + 1], d->face_loop_offsets[f],
                                    d->face_loop_offsets[f + 1], hsegs, ploop, &tsu[f], ch, units, pface[f]) != 0)
                return fail(WN_E_TOPOLOGY);
            const double em = face_margin(f, pface[f].t1x, pface[f].t1y);
            for (int32_t s = h->h_seg_begin[f]; s < h->h_seg_begin[f + 1]; ++s) {
                eta[s] = em;
                const double Be = Bv[s] * (1.0 + kAxisInflate) + em;
                hb2[s] = 0.5 * Be * Be;
            }
        }
        if (units.size() > (size_t)(2 * L + 1)) return fail(WN_E_TOPOLOGY);
        // Work-queue order of the periodic faces: most (segment, copy) pairs
        // per query first, so that the cheap faces' items fill the end of the
        // persistent pass.  A unit's copy windows span its extent over the
        // period (or family spacing) plus the windows' widening by one copy on
        // each side; the estimate only orders the faces.
        {
            auto ext_pairs = [&](int32_t l) {
                const PLoop& Lp = ploop[l];
                const double copies = Lp.lv > 0.0 ? (Lp.xi_hi - Lp.xi_lo) / Lp.lv + 3.0 : 1.0;
                return copies * (double)(Lp.s1 - Lp.s0);
            };
            std::vector<double> cost((size_t)F, 0.0);
            for (int32_t f = 0; f < F; ++f) {
                if (dom[f] == WN_DOMAIN_PLANE) continue;
                const PFace& pf = pface[f];
                for (int32_t u = pf.u0; u < pf.u1; ++u) {
                    const PUnit& U = units[u];
                    if (U.kind == kUnitExtended) {
                        cost[f] += ext_pairs(U.la);
                    } else if (U.kind == kUnitContractible) {
                        const PLoop& Lp = ploop[U.la];
                        double c = (Lp.bb[1] - Lp.bb[0]) / pf.Tu + 3.0;
                        if (pf.dom == WN_DOMAIN_TORUS) c *= (Lp.bb[3] - Lp.bb[2]) / pf.Tv + 3.0;
                        cost[f] += c * (double)(Lp.s1 - Lp.s0);
                    } else {
                        const double fam = pf.Delta > 0.0 ? (U.eta_hi - U.eta_lo) / pf.Delta + 3.0 : 1.0;
                        cost[f] += fam * (ext_pairs(U.la) + ext_pairs(U.lb));
                    }
                }
            }
            std::stable_sort(ord_per.begin(), ord_per.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
            for (size_t r = 0; r < ord_per.size(); ++r) h->per_pos[ord_per[r]] = (int32_t)r;
            e = hipMemcpyAsync(base + o_oq, ord_per.data(), ord_per.size() * 4, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return fail(hip_status(e));
        }
        // far-test records: the lifted end points (the lift's own additions,
        // repeated with its offsets) and the final hb2
        std::vector<FarRec> frec((size_t)S);
        for (int32_t f = 0; f < F; ++f) {
            if (dom[f] == WN_DOMAIN_PLANE) continue;
            for (int32_t s = h->h_seg_begin[f]; s < h->h_seg_begin[f + 1]; ++s) {
                const int64_t c0 = d->seg_cp_offsets[s], c1 = d->seg_cp_offsets[s + 1] - 1;
                FarRec& r = frec[s];
                r.p0x = d->cp_u[c0] + seg_off[2 * s];
                r.p0y = d->cp_v[c0] + seg_off[2 * s + 1];
                r.pnx = d->cp_u[c1] + seg_off[2 * s];
                r.pny = d->cp_v[c1] + seg_off[2 * s + 1];
                r.hb2 = hb2[s];
            }
        }
        e = hipMemcpyAsync(base + o_frec, frec.data(), (size_t)S * sizeof(FarRec), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return fail(hip_status(e));
        e = hipMemcpyAsync(base + o_eta, eta.data(), (size_t)S * 8, hipMemcpyHostToDevice, st);
        // ... and the near pass's copy of eta in each coefficient record (the
        // records themselves were lifted on the device)
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(base + o_coef + (kPadEta * 4 + 3) * 8, kCoef * 4 * 8, eta.data(), 8, 8, (size_t)S,
                                 hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(base + o_hb2, hb2.data(), (size_t)S * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !units.empty())
            e = hipMemcpyAsync(base + o_punit, units.data(), units.size() * sizeof(PUnit), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(base + o_pface, pface.data(), (size_t)F * sizeof(PFace), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(hip_status(e));
        h->h_units = units;
        h->h_pface = pface;
        h->pt.loop = d_ploop;
        h->pt.unit = (const PUnit*)(base + o_punit);
        h->pt.face = (const PFace*)(base + o_pface);
    }
    // side stream of the overlapped passes (none: no overlap)
    if ((opt.flags & WN_FLAG_OVERLAP) && hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
        h->side = nullptr;
        (void)hipGetLastError();
    }
    *out = h;
    return WN_OK;
}

wn_status wn_torus_pairs(const wn_faces* h, int32_t face, int32_t cap, int32_t* alpha, int32_t* beta, double* shift,
                         int32_t* count) {
    if (!h || !count || face < 0 || face >= h->num_faces || cap < 0) return WN_E_INVALID;
    if (cap > 0 && (!alpha || !beta || !shift)) return WN_E_INVALID;
    *count = 0;
    if (h->h_pface.empty() || h->h_dom[face] == WN_DOMAIN_PLANE) return WN_OK;
    const PFace& pf = h->h_pface[face];
    int32_t k = 0;
    for (int u = pf.u0; u < pf.u1; ++u) {
        const PUnit& U = h->h_units[u];
        if (U.kind != kUnitPair) continue;
        if (k < cap) {
            alpha[k] = U.la;
            beta[k] = U.lb;
            shift[2 * k] = U.pshx;
            shift[2 * k + 1] = U.pshy;
        }
        ++k;
    }
    *count = k;
    return WN_OK;
}

void wn_destroy_faces(wn_faces* h) {
    if (!h) return;
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->dmem) (void)hipFree(h->dmem);
    delete h;
}

wn_status wn_get_faces_info(const wn_faces* h, wn_faces_info* info) {
    if (!h || !info) return WN_E_INVALID;
    info->num_faces = h->num_faces;
    info->num_loops = h->num_loops;
    info->num_segments = h->num_segments;
    info->num_periodic_faces = h->num_periodic;
    info->max_segments_per_face = h->max_spf;
    info->max_depth_bound = h->max_depth;
    info->device_bytes = h->dbytes;
    return WN_OK;
}

wn_status wn_profile_create(int32_t capacity, wn_profile** out) {
    if (!out || capacity < 1 || capacity > (1 << 20)) return WN_E_INVALID;
    *out = nullptr;
    wn_profile* p = new (std::nothrow) wn_profile();
    if (!p) return WN_E_NOMEM;
    p->ev.resize((size_t)capacity * 2, nullptr);
    p->kind.resize((size_t)capacity, 0);
    for (auto& e : p->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            wn_profile_destroy(p);
            return WN_E_DEVICE;
        }
    }
    *out = p;
    return WN_OK;
}

wn_status wn_profile_collect(wn_profile* p, int64_t* launches, double* total_ms) {
    if (!p || !launches || !total_ms) return WN_E_INVALID;
    for (int k = 0; k < WN_KERNEL_KINDS; ++k) {
        launches[k] = 0;
        total_ms[k] = 0.0;
    }
    wn_status st = WN_OK;
    for (int i = 0; i < p->used; ++i) {
        if (hipEventSynchronize(p->ev[2 * i + 1]) != hipSuccess) {
            st = WN_E_DEVICE;
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess) {
            st = WN_E_DEVICE;
            continue;
        }
        const int k = p->kind[i];
        launches[k] += 1;
        total_ms[k] += ms;
    }
    p->used = 0;
    return st;
}

void wn_profile_destroy(wn_profile* p) {
    if (!p) return;
    for (auto& e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

static int pick_qpw(int64_t n, int cu) {
    // enough workgroups to cover every CU a few times before using 4 query
    // groups per workgroup (segment split over waves otherwise), two queries
    // per lane beyond that, and four once there are 16 items per CU (the
    // four-query kernel runs 3 workgroups per CU: with fewer items its last
    // round leaves CUs idle)
    if (n >= (int64_t)cu * 1024 * 16) return 1024;
    if (n >= (int64_t)cu * 512 * 4) return 512;
    if (n >= (int64_t)cu * 256 * 4) return 256;
    if (n >= (int64_t)cu * 128 * 4) return 128;
    return 64;
}

}  // extern "C"

namespace wn {

// The query pipeline.  With `preset` scratch (a plan) nothing is allocated or
// synchronised, so the call can be captured into a graph.
wn_status query_core(const wn_faces* h, const wn_points* p, double* out_w, uint8_t* out_lab, const wn_query_opts* qo,
                     Scratch* preset, void* stream) {
    if (!h || !p) return WN_E_INVALID;
    wn_query_opts q;
    wn_default_query_opts(&q);
    if (qo) q = *qo;
    const int sched = q.schedule >= 0 ? q.schedule : h->schedule;
    const int prec = q.precision >= 0 ? q.precision : h->precision;
    const int rule = q.rule >= 0 ? q.rule : h->rule;
    if (sched > WN_SCHED_BINNED || prec > WN_PREC_MIXED || rule > WN_RULE_POSITIVE) return WN_E_INVALID;
    if (q.queries_per_wg != 0 && q.queries_per_wg != 64 && q.queries_per_wg != 128 && q.queries_per_wg != 256 &&
        q.queries_per_wg != 512 && q.queries_per_wg != 768 && q.queries_per_wg != 1024)
        return WN_E_INVALID;
    if (q.queue_policy < 0 || q.queue_policy > 2 || q.near_capacity < 0) return WN_E_INVALID;
    if (q.depth_log && sched != WN_SCHED_PLAIN) return WN_E_UNSUPPORTED;
    const int64_t N = p->num_points;
    const int32_t F = h->num_faces;
    if (N < 0 || N >= 0x7fffffffll) return WN_E_INVALID;
    if (N == 0) return WN_OK;
    if (!p->u || !p->v || p->stride < 1 || !p->face_point_offsets) return WN_E_INVALID;
    if (F == 0) return WN_E_INVALID;
    if (p->face_point_offsets_host) {
        const int64_t* o = p->face_point_offsets_host;
        if (o[0] != 0 || o[F] != N) return WN_E_INVALID;
        for (int32_t f = 0; f < F; ++f)
            if (o[f + 1] < o[f]) return WN_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    const Points pts{p->u, p->v, p->stride, p->face_point_offsets, N};
    const int qpw = q.queries_per_wg ? q.queries_per_wg : pick_qpw(N, h->cu_count);
    const bool periodic = h->num_periodic > 0;
    hipError_t e = hipSuccess;

    const bool plain = sched == WN_SCHED_PLAIN;
    const bool binned = sched == WN_SCHED_BINNED && q.bin_source != WN_BIN_NONE &&
                        !((q.bin_source == WN_BIN_PREDICTOR || q.bin_source == WN_BIN_PREDICTOR_VALU) && !q.predictor);
    if (q.bin_source < 0 || q.bin_source > WN_BIN_PREDICTOR_VALU) return WN_E_INVALID;
    if (q.path_hierarchy < 0 || q.path_hierarchy > 2) return WN_E_INVALID;
    if (q.bound != WN_BOUND_GLOBAL && q.bound != WN_BOUND_SUBDIVIDED) return WN_E_INVALID;
    const bool cp = q.bound == WN_BOUND_SUBDIVIDED;
    int64_t cap = q.near_capacity > 0 ? q.near_capacity : 8 * N + 65536;
    cap = std::min<int64_t>(cap, (int64_t)1 << 34);
    if (plain) cap = 0;  // periodic faces of the plain schedule recurse in line
    Scratch sc;
    if (preset) {
        if (plain || (binned && (!preset->qs2 || (q.bin_source == WN_BIN_MEASURED && !preset->depth))))
            return WN_E_UNSUPPORTED;
        sc = *preset;
        sc.out = Out{out_w, out_lab, nullptr, 0, rule};
    } else {
        e = scratch_alloc(h, N, cap, binned, binned && q.bin_source == WN_BIN_MEASURED, out_w, out_lab, rule, sc,
                          st, true, q.path_hierarchy != 0);
        if (e != hipSuccess) return hip_status(e);
    }

    if (plain) {
        const int64_t* ho = p->face_point_offsets_host;
        const Out pout{sc.out.w, sc.out.lab, q.depth_log, h->max_spf, rule};
        const int qg = qpw > 256 ? 256 : qpw;  // in-line recursion: one query per lane
        if (!ho) {
            // Device offsets only (nothing is read back): the faces' tiles come
            // from item tables built on the device, one in-line launch per
            // domain kind.  The periodic pass and the finalize of every point
            // run first; the planar in-line pass then writes its final values
            // over whatever that finalize left on planar points.
            if (h->num_periodic > 0) {
                ProfScope ps(q.profile, WN_KERNEL_FAR_PERIODIC, st);
                e = launch_build_items(h->ft_per, pts, 256, sc.item_offs, sc.item_map, sc.max_items, sc.counters,
                                       true, st);
                if (e == hipSuccess) e = launch_spatial_order(h->ft_per, pts, sc.perm, st);
                if (e == hipSuccess)
                    e = launch_far_periodic(kPerInline, h->sg, h->ft_per, pts, sc.item_offs, sc.item_map, nullptr,
                                            sc.max_items, sc.nq, sc.out, h->eps2, h->pt, sc.perm, st);
                if (e == hipSuccess) e = launch_finalize(pts, sc.out, 0, N, -1, st);
            }
            if (e == hipSuccess && h->num_planar > 0) {
                ProfScope ps(q.profile, WN_KERNEL_FAR, st);
                e = launch_build_items(h->ft_plan, pts, qg, sc.item_offs, sc.item_map, sc.max_items, sc.counters,
                                       true, st);
                if (e == hipSuccess)
                    e = launch_far(true, prec == WN_PREC_MIXED, qg, h->sg, h->ft_plan, pts, sc.item_offs,
                                   sc.item_map, nullptr, -1, sc.max_items, NearQueue{}, pout, h->eps2, st);
            }
            if (!preset) scratch_free(sc, st);
            return hip_status(e);
        }
        bool zero_near = true;
        for (int32_t f = 0; f < F && e == hipSuccess; ++f) {
            const int64_t nf = ho[f + 1] - ho[f];
            if (nf == 0) continue;
            ProfScope ps(q.profile, WN_KERNEL_FAR, st);
            if (h->h_dom[f] == WN_DOMAIN_PLANE) {
                e = launch_far(true, prec == WN_PREC_MIXED, qg, h->sg, h->ft_plan, pts, nullptr, nullptr, nullptr, f,
                               (nf + qg - 1) / qg, NearQueue{}, pout, h->eps2, st);
            } else {
                // one-face item table, in-line recursion (queue capacity 0), finalize of its range
                const FaceTab one{h->ft_per.seg_begin, h->ft_per.order + h->per_pos[f], 1};
                e = launch_build_items(one, pts, 256, sc.item_offs, sc.item_map, sc.max_items, sc.counters, zero_near,
                                       st);
                zero_near = false;
                if (e == hipSuccess) e = launch_spatial_order(one, pts, sc.perm, st);
                if (e == hipSuccess)
                    e = launch_far_periodic(kPerInline, h->sg, one, pts, sc.item_offs, sc.item_map, nullptr,
                                            (nf + 255) / 256, sc.nq, sc.out, h->eps2, h->pt, sc.perm, st);
                if (e == hipSuccess) e = launch_finalize(pts, sc.out, ho[f], ho[f + 1], -1, st);
            }
        }
        if (!preset) scratch_free(sc, st);
        return hip_status(e);
    }

    // batched / binned: persistent far launches, (binning), near pass, finalize, redo
    // the far/near overlap is for the plain batched FP64 query (not binned, not
    // captured into a plan, no work counters)
    sc.near_lo = nullptr;
    sc.near_join = nullptr;
    const int64_t* ovl =
        (!binned && !preset && !q.stats && !cp && prec == WN_PREC_FP64) ? p->face_point_offsets_host : nullptr;
    e = far_passes(h, pts, qpw, q.queue_policy, prec == WN_PREC_MIXED, q.path_hierarchy, sc, q.profile, st, ovl,
                   p->face_point_offsets_host, q.stats);
    NearQueue nq = sc.nq;
    if (e == hipSuccess && binned) {
        const wn_predictor* pr = q.predictor;
        if (q.bin_source == WN_BIN_MEASURED) {
            // first near pass into throw-away outputs, logging each entry's depth
            const Out tmp{sc.w_tmp, sc.lab_tmp, nullptr, 0, rule};
            e = near_pass(h, pts, sc.nq, tmp, nullptr, sc.depth, nullptr, st, near_cursor(sc, 1), cp);
        }
        if (e == hipSuccess) {
            ProfScope ps(q.profile, WN_KERNEL_BIN, st);
            // the MLP runs on the matrix cores (BF16 weights) unless the VALU
            // version is asked for
            const bool valu = q.bin_source == WN_BIN_PREDICTOR_VALU;
            const int mode = valu ? WN_BIN_PREDICTOR : q.bin_source;
            const uint16_t* w16 = (mode == WN_BIN_PREDICTOR && !valu && pr) ? pr->d_w16 : nullptr;
            e = launch_binning(h->sg, pts, sc.nq, h->pt.seg_periodic, h->eps, mode, pr ? pr->d_wbf : nullptr, w16,
                               pr ? pr->d_norm : nullptr, sc.depth, sc.bins, sc.wg_hist, binning_grid(h), sc.qs2,
                               sc.sh2, st);
        }
        nq.qs = sc.qs2;
        nq.shift = sc.sh2;
    }
    if (e == hipSuccess && sc.near_lo) {
        // the entries after the last overlapped phase, then join the side stream
        {
            ProfScope ps(q.profile, WN_KERNEL_NEAR, st);
            e = launch_near(h->sg, pts, nq, sc.out, h->eps2, (int64_t)h->cu_count * h->bpc_near, Stats{nullptr},
                            h->pt.seg_periodic, nullptr, st, sc.near_lo, nullptr, near_cursor(sc, 3));
        }
    } else if (e == hipSuccess) {
        e = near_pass(h, pts, nq, sc.out, q.stats, nullptr, q.profile, st, near_cursor(sc, 0), cp);
    }
    if (sc.near_join) {
        // join the side stream (errors included: the scratch is released on st)
        const hipError_t ej = hipStreamWaitEvent(st, sc.near_join, 0);
        if (ej != hipSuccess) (void)hipStreamSynchronize(h->side);
        if (e == hipSuccess) e = ej;
        (void)hipEventDestroy(sc.near_join);
        sc.near_join = nullptr;
    }
    if (e == hipSuccess && h->num_periodic > 0) {
        // periodic queries that lost a near pair: recomputed in line over the
        // periodic item table (still the last one built), before finalize
        ProfScope ps(q.profile, WN_KERNEL_REDO, st);
        const bool persistent = q.queue_policy != 2;
        const int64_t grid = persistent ? (int64_t)h->cu_count * h->bpc_redo_per : sc.max_items;
        e = launch_far_periodic(kPerRedo, h->sg, h->ft_per, pts, sc.item_offs, sc.item_map,
                                persistent ? sc.counters + 1 : nullptr, grid, sc.nq, sc.out, h->eps2, h->pt, sc.perm,
                                st);
    }
    if (e == hipSuccess) {
        ProfScope ps(q.profile, WN_KERNEL_FINALIZE, st);
        e = launch_finalize(pts, sc.out, 0, N, F, st);
    }
    if (e == hipSuccess && h->num_planar > 0) {
        ProfScope ps(q.profile, WN_KERNEL_REDO, st);
        e = launch_redo(h->sg, FaceTab{h->ft_plan.seg_begin, nullptr, F}, pts, sc.out, h->eps2, sc.nq,
                        (int64_t)h->cu_count * 8, st);
    }
    if (!preset) scratch_free(sc, st);
    return hip_status(e);
}

}  // namespace wn

extern "C" {

wn_status wn_query_ex(const wn_faces* h, const wn_points* p, double* out_w, uint8_t* out_lab,
                      const wn_query_opts* qo, void* stream) {
    return query_core(h, p, out_w, out_lab, qo, nullptr, stream);
}

}  // extern "C"

namespace wn {

hipError_t scratch_alloc(const wn_faces* h, int64_t N, int64_t cap, bool binned, bool depth, double* out_w,
                         uint8_t* out_lab, int rule, Scratch& sc, hipStream_t st, bool stream_ordered, bool order) {
    const bool periodic = h->num_periodic > 0;
    const bool ordered = periodic || order;
    const int32_t F = h->num_faces;
    sc.max_items = N / 64 + F + 1;
    size_t total = 0;
    auto take = [&](size_t bytes) {
        const size_t off = total;
        total += (bytes + 255) & ~(size_t)255;
        return off;
    };
    const int G = binning_grid(h);
    const size_t o_io = take(((size_t)F + 1) * 4), o_im = take((size_t)sc.max_items * 8), o_ct = take(128);
    const size_t o_nq = take((size_t)cap * 8), o_sh = take(periodic ? (size_t)cap * 16 : 0);
    const size_t o_w = out_w ? 0 : take((size_t)N * 8), o_l = out_lab ? 0 : take((size_t)N);
    const size_t o_q2 = take(binned ? (size_t)cap * 8 : 0), o_s2 = take(binned && periodic ? (size_t)cap * 16 : 0);
    const size_t o_bn = take(binned ? (size_t)cap : 0), o_wh = take(binned ? (size_t)G * 32 * 4 : 0);
    const size_t o_dp = take(depth ? (size_t)cap : 0), o_pm = take(ordered ? (size_t)N * 4 : 0);
    const size_t o_wt = take(depth ? (size_t)N * 8 : 0), o_lt = take(depth ? (size_t)N : 0);
    const hipError_t e = stream_ordered ? hipMallocAsync(&sc.base, total, st) : hipMalloc(&sc.base, total);
    if (e != hipSuccess) return e;
    char* b = (char*)sc.base;
    sc.item_offs = (int32_t*)(b + o_io);
    sc.item_map = (int2*)(b + o_im);
    sc.counters = (uint32_t*)(b + o_ct);
    sc.nq = NearQueue{(uint2*)(b + o_nq), periodic ? (double2*)(b + o_sh) : nullptr,
                      (unsigned long long*)(sc.counters + 2), (uint64_t)cap};
    sc.out = Out{out_w ? out_w : (double*)(b + o_w), out_lab ? out_lab : (uint8_t*)(b + o_l), nullptr, 0, rule};
    sc.perm = ordered ? (uint32_t*)(b + o_pm) : nullptr;
    if (binned) {
        sc.qs2 = (uint2*)(b + o_q2);
        sc.sh2 = periodic ? (double2*)(b + o_s2) : nullptr;
        sc.bins = (uint8_t*)(b + o_bn);
        sc.wg_hist = (uint32_t*)(b + o_wh);
    }
    if (depth) {
        sc.depth = (uint8_t*)(b + o_dp);
        sc.w_tmp = (double*)(b + o_wt);
        sc.lab_tmp = (uint8_t*)(b + o_lt);
    }
    return hipSuccess;
}

void scratch_free(Scratch& sc, hipStream_t st) {
    if (sc.base) (void)hipFreeAsync(sc.base, st);
    sc.base = nullptr;
}

int binning_grid(const wn_faces* h) { return std::min(1024, std::max(1, h->cu_count * 4)); }

// Far and near passes overlapped (batched FP64, planar flat scan).  The
// planar faces (rank order: largest first) are split into kOverlapPhases runs
// at the pair-count fractions kOverlapCut / 20: 45 %, 35 %, 10 % and 10 % of
// the pairs.  The last run's near pass has no far pass left to share the CUs
// with, so the last runs are small; the last far phase still has to be long
// enough to cover the previous run's near pass (on a batch of 2,000 faces,
// last runs of 3-5 % of the pairs were slower).  After the far pass over run
// k (on st) the queue's count is marked, and the near pass over run k's
// entries runs on the side stream while the far pass over run k + 1 runs on
// st.  The far phases after the first and the side near passes take half
// the persistent grid each, so that both are resident (a persistent kernel on
// the whole grid would hold every slot).  The last run's entries, and those
// of any later far pass, go to the final near pass on st (from sc.near_lo),
// which joins the side stream.  The near passes read disjoint queue ranges
// and the phases write disjoint queries, so the results are those of the
// serial passes.
constexpr int kOverlapPhases = 4;
constexpr int kOverlapCut[kOverlapPhases - 1] = {9, 16, 18};  // twentieths of the pairs

static hipError_t far_near_overlapped(const wn_faces* h, const FaceTab& ft, const std::vector<int32_t>& ord,
                                      const Points& pts, int qpl, int64_t grid, const int64_t* host_offs, Scratch& sc,
                                      wn_profile* prof, hipStream_t st) {
    const int Fp = (int)ord.size();
    auto pairs = [&](int r) {
        const int f = ord[r];
        const int64_t nq = std::max<int64_t>(0, host_offs[f + 1] - host_offs[f]);
        return (int64_t)(h->h_seg_begin[f + 1] - h->h_seg_begin[f]) * nq;
    };
    int64_t tot = 0;
    for (int r = 0; r < Fp; ++r) tot += pairs(r);
    int rk[kOverlapPhases + 1];
    rk[0] = 0;
    int64_t acc = 0;
    for (int k = 1, r = 0; k < kOverlapPhases; ++k) {
        while (r < Fp - 1 && acc * 20 < tot * kOverlapCut[k - 1]) acc += pairs(r++);
        rk[k] = r;
    }
    rk[kOverlapPhases] = Fp;
    unsigned long long* marks = reinterpret_cast<unsigned long long*>(sc.counters + 16);
    const int64_t side_grid = std::max<int64_t>(1, (int64_t)h->cu_count * h->bpc_near / 2);
    // events of this call only (queries on one handle from several threads
    // share the side stream, never an event)
    hipEvent_t fork = nullptr, join = nullptr;
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    for (int k = 0; k < kOverlapPhases && e == hipSuccess; ++k) {
        {
            ProfScope ps(prof, WN_KERNEL_FAR, st);
            e = launch_farq(qpl, h->sg, ft, pts, sc.item_offs, sc.item_map, sc.counters + 8 + k,
                            k == 0 ? grid : std::max<int64_t>(1, grid / 2), sc.nq, sc.out, h->eps2, st, rk[k],
                            rk[k + 1]);
        }
        if (k == kOverlapPhases - 1) break;
        if (e == hipSuccess) e = launch_queue_mark(sc.nq.count, marks + k, st);
        if (e == hipSuccess) e = hipEventRecord(fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->side, fork, 0);
        if (e == hipSuccess) {
            ProfScope ps(prof, WN_KERNEL_NEAR, h->side);
            e = launch_near(h->sg, pts, sc.nq, sc.out, h->eps2, side_grid, Stats{nullptr}, h->pt.seg_periodic,
                            nullptr, h->side, k == 0 ? nullptr : marks + k - 1, marks + k, near_cursor(sc, k));
        }
    }
    // The join is recorded whatever happened, so that the query stream always
    // waits for the side stream's work before the scratch is released; if
    // even that fails, the host waits for the side stream.
    if (join) {
        const hipError_t ej = hipEventRecord(join, h->side);
        if (ej == hipSuccess) {
            sc.near_join = join;
        } else {
            (void)hipStreamSynchronize(h->side);
            (void)hipEventDestroy(join);
        }
        if (e == hipSuccess) e = ej;
    }
    // a destroyed event's recorded work still completes, and waits already
    // enqueued on it still hold
    if (fork) (void)hipEventDestroy(fork);
    if (e == hipSuccess) sc.near_lo = marks + kOverlapPhases - 2;
    return e;
}

hipError_t far_passes(const wn_faces* h, const Points& pts, int qpw, int policy, bool mixed, int tree, Scratch& sc,
                      wn_profile* prof, hipStream_t st, const int64_t* host_offs, const int64_t* counts_host,
                      unsigned long long* stats) {
    hipError_t e = hipSuccess;
    bool zero_near = true;
    const bool persistent = policy != 2;
    // planar faces: the flat scan, the hierarchy walk, or each where it pays
    const FaceTab& flat_ft = tree == 2 ? h->ft_flat : h->ft_plan;
    const FaceTab& tree_ft = tree == 2 ? h->ft_tree : h->ft_plan;
    if (tree != 1 && flat_ft.num_faces > 0) {
        // 512 / 1024: two / four queries per lane (FP64); the mixed-precision
        // pass keeps one
        const int qpl = mixed || qpw <= 256 ? 1 : qpw / 256;
        const int qg = qpw > 256 && mixed ? 256 : qpw;
        {
            ProfScope ps(prof, WN_KERNEL_ITEMS, st);
            e = launch_build_items(flat_ft, pts, qg, sc.item_offs, sc.item_map, sc.max_items, sc.counters,
                                   zero_near, st);
            zero_near = false;
        }
        const int* bp = h->bpc_far[mixed ? 1 : 0];
        const int bpc = qpl > 1 ? h->bpc_farq[qpl] : (qg == 64 ? bp[0] : (qg == 128 ? bp[1] : bp[2]));
        const int64_t grid = persistent ? (int64_t)h->cu_count * bpc : sc.max_items;
        if (e == hipSuccess && qpl > 1 && persistent && host_offs && h->side && flat_ft.num_faces >= kOverlapPhases) {
            // (tree == 2: the hierarchy faces' entries go to the final near pass)
            e = far_near_overlapped(h, flat_ft, tree == 2 ? h->h_ord_flat : h->h_ord_plan, pts, qpl, grid,
                                    host_offs, sc, prof, st);
        } else if (e == hipSuccess) {
            ProfScope ps(prof, WN_KERNEL_FAR, st);
            if (qpl > 1)
                e = launch_farq(qpl, h->sg, flat_ft, pts, sc.item_offs, sc.item_map,
                                persistent ? sc.counters : nullptr, grid, sc.nq, sc.out, h->eps2, st);
            else
                e = launch_far(false, mixed, qg, h->sg, flat_ft, pts, sc.item_offs, sc.item_map,
                               persistent ? sc.counters : nullptr, -1, grid, sc.nq, sc.out, h->eps2, st);
        }
    }
    if (e == hipSuccess && tree != 0 && tree_ft.num_faces > 0) {
        // With a spatial order of the points (the query's scratch holds one),
        // faces of at most kOrderMaxPoints points take the walk shared by the
        // wave's spatially neighbouring queries, and the per-lane walk takes
        // the faces whose points keep the caller's order.  Each walk only runs
        // when a face of its kind may exist (both without host offsets).
        bool wave_walk = sc.perm != nullptr;
        bool big = true;
        if (wave_walk && counts_host) {
            bool small = false;
            big = false;
            for (const int32_t f : tree == 2 ? h->h_ord_tree : h->h_ord_plan) {
                const int64_t nf = counts_host[f + 1] - counts_host[f];
                big |= nf > kOrderMaxPoints;
                small |= nf > 0 && nf <= kOrderMaxPoints;
            }
            wave_walk = small;
        }
        if (wave_walk) {
            {
                ProfScope ps(prof, WN_KERNEL_ITEMS, st);
                e = launch_build_items(tree_ft, pts, kWave * kWtreeQPL * kWavesPerWG, sc.item_offs, sc.item_map,
                                       sc.max_items, sc.counters, zero_near, st);
                zero_near = false;
                if (e == hipSuccess) e = launch_spatial_order(tree_ft, pts, sc.perm, st);
            }
            if (e == hipSuccess) {
                const int64_t grid = persistent ? (int64_t)h->cu_count * h->bpc_far_wtree : sc.max_items;
                ProfScope ps(prof, WN_KERNEL_FAR, st);
                e = launch_far_wtree(h->tree, tree_ft, pts, sc.perm, sc.item_offs, sc.item_map,
                                     persistent ? sc.counters : nullptr, grid, sc.nq, sc.out, h->eps2, st);
            }
        }
        if (e == hipSuccess && (!wave_walk || big)) {
            {
                ProfScope ps(prof, WN_KERNEL_ITEMS, st);
                e = launch_build_items(tree_ft, pts, 256, sc.item_offs, sc.item_map, sc.max_items, sc.counters,
                                       zero_near, st);
                zero_near = false;
            }
            if (e == hipSuccess) {
                const int64_t grid = persistent ? (int64_t)h->cu_count * h->bpc_far_tree : sc.max_items;
                ProfScope ps(prof, WN_KERNEL_FAR, st);
                e = launch_far_tree(h->tree, tree_ft, pts, sc.item_offs, sc.item_map,
                                    persistent ? sc.counters : nullptr, grid, sc.nq, sc.out, h->eps2, st, wave_walk);
            }
        }
    }
    if (e == hipSuccess && h->num_periodic > 0) {
        {
            ProfScope ps(prof, WN_KERNEL_ITEMS, st);
            e = launch_build_items(h->ft_per, pts, 256, sc.item_offs, sc.item_map, sc.max_items, sc.counters,
                                   zero_near, st);
            zero_near = false;
            if (e == hipSuccess) e = launch_spatial_order(h->ft_per, pts, sc.perm, st);
        }
        if (e == hipSuccess) {
            const int64_t grid = persistent ? (int64_t)h->cu_count * h->bpc_far_per : sc.max_items;
            ProfScope ps(prof, WN_KERNEL_FAR_PERIODIC, st);
            e = launch_far_periodic(kPerQueue, h->sg, h->ft_per, pts, sc.item_offs, sc.item_map,
                                    persistent ? sc.counters : nullptr, grid, sc.nq, sc.out, h->eps2, h->pt, sc.perm,
                                    st, stats ? stats + WN_STAT_PERIODIC_PAIRS : nullptr);
        }
    }
    return e;
}

hipError_t near_pass(const wn_faces* h, const Points& pts, NearQueue nq, Out out, unsigned long long* stats,
                     uint8_t* entry_depth, wn_profile* prof, hipStream_t st, unsigned long long* cursor,
                     bool cp_bound) {
    ProfScope ps(prof, WN_KERNEL_NEAR, st);
    if (cp_bound)
        return launch_near_cp(h->sg, pts, nq, out, h->eps2, (int64_t)h->cu_count * h->bpc_near_cp, Stats{stats},
                              h->pt.seg_periodic, entry_depth, st, nullptr, nullptr, cursor);
    return launch_near(h->sg, pts, nq, out, h->eps2, (int64_t)h->cu_count * h->bpc_near, Stats{stats},
                       h->pt.seg_periodic, entry_depth, st, nullptr, nullptr, cursor);
}

}  // namespace wn

extern "C" {

wn_status wn_query(const wn_faces* h, const wn_points* p, double* out_w, uint8_t* out_lab, void* stream) {
    return wn_query_ex(h, p, out_w, out_lab, nullptr, stream);
}

}  // extern "C"
