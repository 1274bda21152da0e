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
    const int64_t segs = ((int64_t)H.size() - 1) / p;
    *out_segments = (int32_t)segs;
    if (out_cap < segs * p + 1 || !out_u || !out_v || (cp_w && !out_w)) return WN_E_INVALID;
    for (size_t i = 0; i < H.size(); ++i) {
        out_u[i] = H[i].x / H[i].w;
        out_v[i] = H[i].y / H[i].w;
        if (cp_w) out_w[i] = H[i].w;
    }
    return WN_OK;
}
