// NURBS p-curves to (rational) Bezier segments by knot insertion (host only).
//
// A NURBS curve of degree p with clamped knots U and homogeneous control
// points H_i = (w_i x_i, w_i y_i, w_i) is a piecewise polynomial curve in
// homogeneous space.  Inserting a knot t into the span U_k <= t < U_{k+1}
// (Boehm's rule) keeps the curve and replaces H_{k-p+1..k-s} by the convex
// combinations a_i H_i + (1 - a_i) H_{i-1}, a_i = (t - U_i) / (U_{i+p} - U_i),
// s = current multiplicity of t.  Once every interior knot has multiplicity p,
// span j is a Bezier segment with control points H_{jp..jp+p} (the curve
// subdivides into Bezier segments, Sec. 3.1); projecting back gives the
// rational Bezier control points and weights.
#include "wn_host_internal.h"

#include <math.h>

#include <vector>

namespace {

struct H3 {
    double x, y, w;
};

bool finite_cp(double v) { return isfinite(v) && fabs(v) < wn::kCoordLimit; }

constexpr int kMaxNurbsCps = 16384;

}  // namespace

extern "C" wn_status wn_nurbs_to_bezier(int32_t degree, int32_t num_cps, const double* knots, const double* cp_u,
                                        const double* cp_v, const double* cp_w, int64_t out_cap, double* out_u,
                                        double* out_v, double* out_w, int32_t* out_segments) {
    const int p = degree;
    // each insertion rewrites the control polygon (O(num_cps)); longer curves
    // are to be split into several NURBS first
    if (p < 1 || p > wn::kMaxDeg || num_cps < p + 1 || num_cps > kMaxNurbsCps || !knots || !cp_u || !cp_v ||
        !out_segments)
        return WN_E_INVALID;
    const int n = num_cps;
    std::vector<double> U(knots, knots + n + p + 1);
    for (int i = 0; i < n + p + 1; ++i)
        if (!isfinite(U[i]) || (i > 0 && U[i] < U[i - 1])) return WN_E_INVALID;
    for (int i = 1; i <= p; ++i)
        if (U[i] != U[0] || U[n + p - i] != U[n + p]) return WN_E_INVALID;
    if (!(U[p] < U[n])) return WN_E_INVALID;
    // the end values appear exactly p + 1 times (more would leave basis
    // functions without support inside [U[p], U[n]])
    if (!(U[p + 1] > U[p]) || !(U[n - 1] < U[n])) return WN_E_INVALID;
    std::vector<H3> H((size_t)n);
    for (int i = 0; i < n; ++i) {
        const double w = cp_w ? cp_w[i] : 1.0;
        if (!finite_cp(cp_u[i]) || !finite_cp(cp_v[i]) || !(w > 0.0) || !isfinite(w)) return WN_E_INVALID;
        H[i] = H3{w * cp_u[i], w * cp_v[i], w};
    }
    // raise every interior knot to multiplicity p
    for (size_t k = (size_t)p + 1; k + (size_t)p + 1 < U.size();) {
        const double t = U[k];
        size_t e = k;  // [k, e): the run of knots equal to t
        while (e < U.size() && U[e] == t) ++e;
        if (U[e - 1] == U[U.size() - 1]) break;  // reached the clamped end
        int s = (int)(e - k);
        if (s > p) return WN_E_INVALID;  // a break in the curve: not one path
        while (s < p) {
            // span of t: U[kk] <= t < U[kk + 1] with kk = e - 1 (the last knot equal to t)
            const int kk = (int)e - 1;
            std::vector<H3> G(H.size() + 1);
            for (int i = 0; i <= kk - p; ++i) G[i] = H[i];
            for (int i = kk - p + 1; i <= kk - s; ++i) {
                const double a = (t - U[i]) / (U[i + p] - U[i]);
                G[i] = H3{a * H[i].x + (1.0 - a) * H[i - 1].x, a * H[i].y + (1.0 - a) * H[i - 1].y,
                          a * H[i].w + (1.0 - a) * H[i - 1].w};
            }
            for (int i = kk - s + 1; i <= (int)H.size(); ++i) G[i] = H[i - 1];
            H.swap(G);
            U.insert(U.begin() + e, t);
            ++e;
            ++s;
        }
        k = e;
    }
    if (((int64_t)H.size() - 1) % p != 0) return WN_E_INVALID;  // cannot happen for a validated knot vector
    const int64_t segs = ((int64_t)H.size() - 1) / p;
    *out_segments = (int32_t)segs;
    if (out_cap < segs * p + 1 || !out_u || !out_v || (cp_w && !out_w)) return WN_E_INVALID;
    for (size_t i = 0; i < (size_t)(segs * p + 1); ++i) {
        out_u[i] = H[i].x / H[i].w;
        out_v[i] = H[i].y / H[i].w;
        if (cp_w) out_w[i] = H[i].w;
    }
    return WN_OK;
}

extern "C" wn_status wn_create_faces_nurbs(const wn_nurbs_faces_desc* d, const wn_options* opt, void* stream,
                                           wn_faces** out) {
    if (!d || !out || d->num_faces < 0 || d->num_loops < 0 || d->num_curves < 0 || !d->face_loop_offsets ||
        !d->loop_curve_offsets || (d->num_curves > 0 && (!d->curve_degree || !d->curve_cp_offsets || !d->knots ||
                                                         !d->cp_u || !d->cp_v)))
        return WN_E_INVALID;
    const int32_t F = d->num_faces, L = d->num_loops, C = d->num_curves;
    if (d->face_loop_offsets[0] != 0 || d->face_loop_offsets[F] != L) return WN_E_INVALID;
    if (d->loop_curve_offsets[0] != 0 || d->loop_curve_offsets[L] != C) return WN_E_INVALID;
    for (int32_t l = 0; l < L; ++l)
        if (d->loop_curve_offsets[l + 1] < d->loop_curve_offsets[l]) return WN_E_INVALID;
    if (C > 0 && d->curve_cp_offsets[0] != 0) return WN_E_INVALID;
    if (d->num_cps < 0 || d->num_knots < 0 || (C > 0 && d->curve_cp_offsets[C] != d->num_cps)) return WN_E_INVALID;
    {  // every curve's control points and knots inside the arrays
        int64_t kt = 0;
        for (int32_t c = 0; c < C; ++c) {
            const int64_t c0 = d->curve_cp_offsets[c], c1 = d->curve_cp_offsets[c + 1];
            const int p = d->curve_degree[c];
            if (c1 < c0 || c1 > d->num_cps || p < 1 || p > wn::kMaxDeg) return WN_E_INVALID;
            kt += (c1 - c0) + p + 1;
            if (kt > d->num_knots) return WN_E_INVALID;
        }
        if (kt != d->num_knots) return WN_E_INVALID;
    }
    // split every curve; the segments of curve c follow those of curve c - 1
    std::vector<int32_t> curve_seg((size_t)C + 1, 0);
    std::vector<int64_t> seg_cp(1, 0);
    std::vector<double> u, v, w;
    const bool rational = d->cp_w != nullptr;
    int64_t kb = 0;
    for (int32_t c = 0; c < C; ++c) {
        const int p = d->curve_degree[c];
        const int64_t c0 = d->curve_cp_offsets[c], c1 = d->curve_cp_offsets[c + 1];
        const int64_t n = c1 - c0;
        if (n < p + 1 || n > kMaxNurbsCps || p < 1 || p > wn::kMaxDeg) return WN_E_INVALID;
        const int64_t cap = (n - p) * p + 1;  // at most n - p spans
        std::vector<double> ou((size_t)cap), ov((size_t)cap), ow(rational ? (size_t)cap : 0);
        int32_t k = 0;
        const wn_status st = wn_nurbs_to_bezier(p, (int32_t)n, d->knots + kb, d->cp_u + c0, d->cp_v + c0,
                                                rational ? d->cp_w + c0 : nullptr, cap, ou.data(), ov.data(),
                                                rational ? ow.data() : nullptr, &k);
        if (st != WN_OK) return st;
        kb += n + p + 1;
        for (int32_t sgi = 0; sgi < k; ++sgi) {
            for (int i = 0; i <= p; ++i) {
                const size_t at = (size_t)sgi * p + i;
                u.push_back(ou[at]);
                v.push_back(ov[at]);
                if (rational) w.push_back(ow[at]);
            }
            seg_cp.push_back((int64_t)u.size());
        }
        curve_seg[c + 1] = curve_seg[c] + k;
    }
    std::vector<int32_t> loop_seg((size_t)L + 1, 0);
    for (int32_t l = 0; l <= L; ++l) loop_seg[l] = curve_seg[d->loop_curve_offsets[l]];
    wn_faces_desc fd{};
    fd.num_faces = F;
    fd.num_loops = L;
    fd.num_segments = curve_seg[C];
    fd.num_cps = (int64_t)u.size();
    fd.face_loop_offsets = d->face_loop_offsets;
    fd.loop_seg_offsets = loop_seg.data();
    fd.seg_cp_offsets = seg_cp.data();
    fd.cp_u = u.data();
    fd.cp_v = v.data();
    fd.cp_w = rational ? w.data() : nullptr;
    fd.face_domain = d->face_domain;
    fd.face_period = d->face_period;
    return wn_create_faces(&fd, opt, stream, out);
}
