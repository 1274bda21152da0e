// Device helpers shared by the planar and periodic kernels (gfx950).
#pragma once

#include "wn_internal.h"

#include <math.h>

namespace wn {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr uint8_t kRedo = 4;  // label placeholder: query must be recomputed in line

// Element i of a read-only table at a wave-uniform index: read through the
// constant address space, so that the compiler uses a scalar load into SGPRs
// instead of broadcasting the value into VGPRs.  Only for data that no kernel
// of the same launch writes.  (The host pass only parses device code.)
template <class T>
__device__ __forceinline__ T kload(const T* p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) T*)p)[i];
#else
    return p[i];
#endif
}

// ---------------------------------------------------------------------------
// angle accumulator
// ---------------------------------------------------------------------------
struct Turn {
    double zr, zi;
    int K;
};

__device__ __forceinline__ int sign_bit(double x) { return (int)((unsigned)__double2hiint(x) >> 31); }

__device__ __forceinline__ void turn_mul(Turn& t, double wr, double wi) {
    const double nr = fma(t.zr, wr, -(t.zi * wi));
    const double ni = fma(t.zr, wi, t.zi * wr);
    const int sz = sign_bit(t.zi), sw = sign_bit(wi), sn = sign_bit(ni);
    t.K += (sz == sw) ? (sn - sz) : 0;
    t.zr = nr;
    t.zi = ni;
}

// Rescale z by a power of two (exact) so that products of a few factors can
// neither overflow nor underflow.
__device__ __forceinline__ void turn_norm(Turn& t) {
    int e;
    (void)frexp(fmax(fabs(t.zr), fabs(t.zi)), &e);
    t.zr = ldexp(t.zr, -e);
    t.zi = ldexp(t.zi, -e);
}

// Maclaurin coefficients of arctan: arctan(t) = t + t s sum_k c_k s^k with
// s = t^2, c_k = (-1)^(k+1) / (2k + 3).  Read from memory (scalar loads) at
// each use, so that loops calling arg_of() do not hold the table in vector
// registers.
static __device__ double g_atan_series[21] = {
    -1.0 / 3,  1.0 / 5,  -1.0 / 7,  1.0 / 9,  -1.0 / 11, 1.0 / 13, -1.0 / 15,
    1.0 / 17,  -1.0 / 19, 1.0 / 21, -1.0 / 23, 1.0 / 25, -1.0 / 27, 1.0 / 29,
    -1.0 / 31, 1.0 / 33, -1.0 / 35, 1.0 / 37, -1.0 / 39, 1.0 / 41, -1.0 / 43};

// arg(x + iy) in [-pi, pi] (atan2(y, x), signed zeros of y respected).
// Octant reduction: with n = min(|x|,|y|), d = max(|x|,|y|), arctan(n/d) is
// taken directly when n/d <= tan(pi/8), else as pi/4 + arctan((n-d)/(n+d));
// either way |t| <= tan(pi/8), s <= 0.1716, and the series above cut after
// s^20 leaves a truncation error below 1e-18 relative.
__device__ __forceinline__ double arg_of(double x, double y) {
    const double ax = fabs(x), ay = fabs(y);
    const bool swap = ay > ax;
    const double n = swap ? ax : ay, d = swap ? ay : ax;
    if (!(d > 0.0)) return 0.0;
    const bool big = n > 0.41421356237309503 * d;
    const double num = big ? n - d : n, den = big ? n + d : d;
    double r = __builtin_amdgcn_rcp(den);  // two Newton steps to full precision
    r = fma(fma(-den, r, 1.0), r, r);
    r = fma(fma(-den, r, 1.0), r, r);
    const double t = num * r, s = t * t;
    const double* c = g_atan_series;
    asm volatile("" : "+s"(c));  // opaque: the table is loaded here, not folded or hoisted
    double g = c[20];
#pragma unroll
    for (int k = 19; k >= 0; --k) g = fma(g, s, c[k]);
    double a = fma(t * s, g, t);
    if (big) a += 0.78539816339744830962;  // pi/4
    if (swap) a = 1.57079632679489661923 - a;
    if (__double2hiint(x) < 0) a = 3.14159265358979323846 - a;
    return __double2hiint(y) < 0 ? -a : a;
}

__device__ __forceinline__ double turn_angle(const Turn& t) { return arg_of(t.zr, t.zi) + kTwoPi * (double)t.K; }

// ---------------------------------------------------------------------------
// ellipse test (Lemma 1 / sub-segment bound), square-root free
// ---------------------------------------------------------------------------
// Outside <=> R < 0 or ra rb > R^2 with R = hb2 - (ra + rb) / 2.  Both in one
// comparison: for R < 0 the right side R |R| = -R^2 is <= 0 <= ra rb, so the
// test holds unless ra rb = R^2 = 0 (the query on an end point, which the
// eps test reports as on-boundary first).
__device__ __forceinline__ bool outside_ellipse(double ra, double rb, double hb2) {
    const double R = fma(-0.5, ra + rb, hb2);
    return ra * rb > R * fabs(R);
}

__device__ __forceinline__ double half_axis2(double B, double eta, int k) {
    const double Bk = fma(ldexp(B, -k), 1.0 + kAxisInflate, eta);
    return 0.5 * Bk * Bk;
}

// ---------------------------------------------------------------------------
// Signed crossings with the ray {(x, 0): x > 0} from the query (points
// relative to the query).  For a polygon that avoids the query, the sum of
// the principal angles its edges subtend is 2 pi times the sum of these
// crossings.  Ties are broken by one symbolic displacement of the query,
// q + (-e^2, e) with e -> 0+: a vertex on the ray's line counts as below it,
// and a zero orientation takes the sign of the e and e^2 terms.  Every
// caller evaluates the same expressions on the same doubles, so the
// decisions agree wherever two edges share a vertex.
// ---------------------------------------------------------------------------
// a x b as every caller computes it.
__device__ __forceinline__ double cross_raw(double ax, double ay, double bx, double by) {
    return fma(ax, by, -(ay * bx));
}

// Sign of the displaced query's orientation of a -> b: that of a x b, and
// for an exact zero that of b_x - a_x, then of b_y - a_y (a == b: positive).
__device__ __forceinline__ bool cross_tie_neg(double ax, double ay, double bx, double by) {
    const bool dx = bx != ax;
    return (dx & (bx < ax)) | (!dx & (by < ay));
}
__device__ __forceinline__ bool cross_neg(double ax, double ay, double bx, double by) {
    const double o = cross_raw(ax, ay, bx, by);
    return (o < 0.0) | ((o == 0.0) & cross_tie_neg(ax, ay, bx, by));
}
// The same for a wave in uniform control flow: the tie is only evaluated
// when some lane has an exact zero (the empty asm keeps that a branch).
__device__ __forceinline__ bool cross_neg_wave(double ax, double ay, double bx, double by) {
    const double o = cross_raw(ax, ay, bx, by);
    bool neg = o < 0.0;
    if (__builtin_amdgcn_ballot_w64(o == 0.0) != 0ull) {
        asm volatile("");
        neg |= (o == 0.0) & cross_tie_neg(ax, ay, bx, by);
    }
    return neg;
}

// Crossing of an edge from a (a_low: a_y <= 0) to b (b_low: b_y <= 0) with
// orientation sign neg: +1 upward, -1 downward, else 0.
__device__ __forceinline__ int ray_cross_n(bool a_low, bool b_low, bool neg) {
    return (a_low & !b_low & !neg) ? 1 : ((!a_low & b_low & neg) ? -1 : 0);
}

__device__ __forceinline__ int ray_cross(double ax, double ay, double bx, double by) {
    return ray_cross_n(ay <= 0.0, by <= 0.0, cross_neg(ax, ay, bx, by));
}

// Wave forms for uniform control flow, on lane masks (LLVM predicate codes
// of __builtin_amdgcn_fcmp: the comparison's lane mask, written directly).
constexpr int kCmpOEQ = 1, kCmpOLT = 4, kCmpOLE = 5, kCmpULE = 13;

__device__ __forceinline__ uint64_t low_mask(double y) { return __builtin_amdgcn_fcmp(y, 0.0, kCmpOLE); }

// Lanes of m below this lane (this lane's rank among them).
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// N += ray_cross(a, b) for the lanes of `keep`, with a_lo / b_lo the masks
// of a_y <= 0 / b_y <= 0.  Only lanes whose edge changes side of the ray's
// line can cross; when no lane does, no orientation is computed.
__device__ __forceinline__ void ray_cross_mask(int& N, uint64_t a_lo, uint64_t b_lo, double ax, double ay, double bx,
                                               double by, uint64_t keep = ~0ull) {
    const uint64_t sm = (a_lo ^ b_lo) & keep;
    if (sm) {
        const double o = cross_raw(ax, ay, bx, by);
        uint64_t nm = __builtin_amdgcn_fcmp(o, 0.0, kCmpOLT);
        const uint64_t zm = __builtin_amdgcn_fcmp(o, 0.0, kCmpOEQ) & sm;
        if (zm) nm |= __builtin_amdgcn_ballot_w64(cross_tie_neg(ax, ay, bx, by)) & zm;
        const uint64_t up = sm & a_lo & ~nm, dn = sm & ~a_lo & nm;
        const int cu = __builtin_amdgcn_inverse_ballot_w64(up) ? 1 : 0;
        const int cd = __builtin_amdgcn_inverse_ballot_w64(dn) ? 1 : 0;
        N += cu - cd;
    }
}

// Lanes where !outside_ellipse(ra, rb, hb2).
__device__ __forceinline__ uint64_t near_mask(double ra, double rb, double hb2) {
    const double R = fma(-0.5, ra + rb, hb2);
    return __builtin_amdgcn_fcmp(ra * rb, R * fabs(R), kCmpULE);
}

// Angle factor (a . b, a x b) of the edge a -> b for the accumulator, with
// an exact zero cross product replaced by the signed zero of cross_neg, so
// that a query on the edge gets +-pi on the side that ray_cross assumes.
__device__ __forceinline__ void edge_factor(Turn& T, double ax, double ay, double bx, double by) {
    double o = cross_raw(ax, ay, bx, by);
    if (o == 0.0) o = cross_neg(ax, ay, bx, by) ? -0.0 : 0.0;
    turn_mul(T, fma(ax, bx, ay * by), o);
}

// Chord factor of a near pair whose integer rest comes from near_pair.
__device__ __forceinline__ void chord_factor(Turn& T, double ax, double ay, double bx, double by) {
    edge_factor(T, ax, ay, bx, by);
}

// Close a chain of edges that runs from c to e: the chain's angle sum is
// the principal angle from c to e plus 2 pi (its crossings + those of the
// closing edge e -> c).  The first term goes to the accumulator, the
// closing edge's crossing to N; the closing edge's orientation is the
// negation of c -> e's, so the two terms agree on ties.
__device__ __forceinline__ void close_chain(Turn& T, int& N, double cx, double cy, double ex, double ey) {
    edge_factor(T, cx, cy, ex, ey);
    N += ray_cross_n(ey <= 0.0, cy <= 0.0, !cross_neg(cx, cy, ex, ey));
    turn_norm(T);
}

// ---------------------------------------------------------------------------
// curve evaluation
// ---------------------------------------------------------------------------
struct Coef {
    double x[kCoef], y[kCoef], w[kCoef];
    int n;
    bool rat;
};

__device__ __forceinline__ void load_coef(const Segs& sg, int s, Coef& c) {
    const double4* cf = reinterpret_cast<const double4*>(sg.coef) + (size_t)s * kCoef;
#pragma unroll
    for (int j = 0; j < kCoef; ++j) {
        const double4 v = cf[j];
        c.x[j] = v.x;
        c.y[j] = v.y;
        c.w[j] = v.z;
    }
    c.n = sg.deg[s];
    c.rat = sg.rat[s] != 0;
}

// The coefficient record's fourth components carry the segment's near-pass
// data, so that a near pair gathers one contiguous 192-B record.
struct NearSeg {
    double B, eta, p0x, p0y, pnx, pny;
};
__device__ __forceinline__ void load_near_seg(const Segs& sg, int s, Coef& c, NearSeg& g) {
    const double4* cf = reinterpret_cast<const double4*>(sg.coef) + (size_t)s * kCoef;
    double pad[kCoef];
#pragma unroll
    for (int j = 0; j < kCoef; ++j) {
        const double4 v = cf[j];
        c.x[j] = v.x;
        c.y[j] = v.y;
        c.w[j] = v.z;
        pad[j] = v.w;
    }
    c.n = sg.deg[s];
    c.rat = sg.rat[s] != 0;
    g = NearSeg{pad[kPadB], pad[kPadEta], pad[kPadP0x], pad[kPadP0y], pad[kPadPnx], pad[kPadPny]};
}
__device__ __forceinline__ double2 seg_end_point(const Segs& sg, int s) {
    const double4* cf = reinterpret_cast<const double4*>(sg.coef) + (size_t)s * kCoef;
    return make_double2(cf[kPadPnx].w, cf[kPadPny].w);
}

// Reciprocal to full precision: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    return fma(fma(-d, r, 1.0), r, r);
}

// gamma(t) = sum_k C(n,k) w_k P_k t^k (1-t)^(n-k) / sum_k C(n,k) w_k t^k (1-t)^(n-k).
// Slot k holds the k-th term's coefficient (zero for k > n).  Dividing both
// sums by (1-t)^n leaves polynomials in u = t / (1-t), so one Horner pass
// over all kCoef slots serves every degree without a branch; polynomial
// segments carry w_k = 1 (denominator (1+u)^n).  With positive weights the
// absolute error stays a few units in the last place of the control points'
// size for any u (0 < t < 1).
__device__ __forceinline__ void bez_eval(const Coef& c, double t, double& X, double& Y) {
    const double u = t * recip(1.0 - t);
    double px = c.x[kCoef - 1], py = c.y[kCoef - 1], pw = c.w[kCoef - 1];
#pragma unroll
    for (int k = kCoef - 2; k >= 0; --k) {
        px = fma(px, u, c.x[k]);
        py = fma(py, u, c.y[k]);
        pw = fma(pw, u, c.w[k]);
    }
    const double r = recip(pw);
    X = px * r;
    Y = py * r;
}

// ---------------------------------------------------------------------------
// Deferred intervals live in an LDS ring of kNearSlots slots per lane
// (slot = level mod kNearSlots, 32 B: both end points).  Storing at a level
// evicts whatever the slot held, at any level of the same residue.
// ---------------------------------------------------------------------------
static_assert(kNearSlots == 4, "the eviction mask assumes four slots");
__device__ __forceinline__ uint64_t slot_evict_mask(int level) {
    return 0x1111111111111111ull << (level & (kNearSlots - 1));
}

// Left end of the interval deferred at level kk while the current interval
// (left end a) lies in its left sibling: (a rounded down to 2^-(kk-1)) + 2^-kk.
__device__ __forceinline__ double deferred_left(double a, int kk) {
    return ldexp(floor(ldexp(a, kk - 1)), 1 - kk) + ldexp(1.0, -kk);
}

// ---------------------------------------------------------------------------
// near pair: Alg. 1 with an explicit stack.  The root [0,1] is known to be
// inside its ellipse and not on the boundary.  Points are kept relative to
// the query; `stk` is this lane's slot 0 in LDS (slot stride kWave).
//
// Each step halves the current interval and tests both halves: a half that
// passes is a leaf (its chord's crossing is taken at once), a half that fails
// becomes the current interval, the right one deferred when both fail.  The
// tested nodes, splits and leaves are exactly Alg. 1's.
//
// The pair's angle is the sum of the leaves' chord angles.  It is returned
// as an integer N: angle = (chord angle of the segment, given to the
// accumulator by the caller through chord_factor or a chain) + 2 pi N, where
// N = sum over leaves of ray_cross - ray_cross(chord).  This is exact: the
// leaves' chords followed by the reversed segment chord form a closed
// polygon that avoids the query, whose angle sum is 2 pi times its crossings.
// Returns the deepest level reached; sets onb on an eps hit.
// ---------------------------------------------------------------------------
__device__ int near_pair(int& N, const Coef& c, double B, double eta, double pnx, double pny, double qx, double qy,
                         double ax, double ay, double ra, double bx, double by, double rb, double eps2,
                         double4* stk, bool& onb) {
    int n = -ray_cross(ax, ay, bx, by);
    double a = 0.0;  // current interval [a, a + 2^-k], exact dyadic
    int k = 0;
    uint64_t pend = 0, stored = 0;
    int maxk = 0;
    for (;;) {
        if (k >= kDepthCap) {
            onb = true;  // cannot happen for a validated eps (depth bound <= cap)
            return maxk;
        }
        const int k1 = k + 1;
        const double tm = a + ldexp(1.0, -k1);
        double mx, my;
        bez_eval(c, tm, mx, my);
        mx -= qx;
        my -= qy;
        const double rm = mx * mx + my * my;
        if (rm < eps2) {
            onb = true;
            return k1;
        }
        maxk = k1 > maxk ? k1 : maxk;
        const double hb = half_axis2(B, eta, k1);
        const bool lfar = outside_ellipse(ra, rm, hb);
        const bool rfar = outside_ellipse(rm, rb, hb);
        if (lfar) n += ray_cross(ax, ay, mx, my);
        if (rfar) n += ray_cross(mx, my, bx, by);
        if (!lfar) {  // continue left; defer the right half when it failed too
            if (!rfar) {
                stk[(k1 & (kNearSlots - 1)) * kWave] = make_double4(mx, my, bx, by);
                stored = (stored & ~slot_evict_mask(k1)) | (1ull << k1);
                pend |= 1ull << k1;
            }
            bx = mx;
            by = my;
            rb = rm;
            k = k1;
        } else if (!rfar) {  // continue right
            a = tm;
            ax = mx;
            ay = my;
            ra = rm;
            k = k1;
        } else {  // both halves are leaves: resume the deepest deferred interval
            if (pend == 0) {
                N += n;
                return maxk;
            }
            const int kk = 63 - __clzll(pend);
            const uint64_t kbit = 1ull << kk;
            pend &= ~kbit;
            a = deferred_left(a, kk);
            if (stored & kbit) {
                const double4 p = stk[(kk & (kNearSlots - 1)) * kWave];
                ax = p.x;
                ay = p.y;
                bx = p.z;
                by = p.w;
            } else {  // evicted: evaluate both ends again (same parameters, same values)
                bez_eval(c, a, ax, ay);
                ax -= qx;
                ay -= qy;
                const double te = a + ldexp(1.0, -kk);
                if (te == 1.0) {
                    bx = pnx;
                    by = pny;
                } else {
                    bez_eval(c, te, bx, by);
                }
                bx -= qx;
                by -= qy;
            }
            stored &= ~kbit;
            ra = ax * ax + ay * ay;
            rb = bx * bx + by * by;
            k = kk;
        }
    }
}

// Near pair with all segment data read from global memory (integer part only).
__device__ __forceinline__ int near_from_global(int& N, const Segs& sg, uint32_t s, double qx, double qy,
                                                double eps2, double4* stk, bool& onb) {
    Coef c;
    NearSeg g;
    load_near_seg(sg, s, c, g);
    const double ax = g.p0x - qx, ay = g.p0y - qy;
    const double bx = g.pnx - qx, by = g.pny - qy;
    return near_pair(N, c, g.B, g.eta, g.pnx, g.pny, qx, qy, ax, ay, ax * ax + ay * ay, bx, by, bx * bx + by * by,
                     eps2, stk, onb);
}

__device__ __forceinline__ uint8_t classify(double omega, int rule) {
    if (rule == 1) return omega > 0.5 ? 1 : 0;
    return fabs(omega) > 0.5 ? 1 : 0;
}

}  // namespace wn
