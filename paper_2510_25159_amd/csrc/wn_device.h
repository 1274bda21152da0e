// Device helpers shared by the planar and periodic kernels (gfx950).
#pragma once

#include "wn_internal.h"

#include <math.h>

namespace wn {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr uint8_t kRedo = 4;  // label placeholder: query must be recomputed in line

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
__device__ __forceinline__ bool outside_ellipse(double ra, double rb, double hb2) {
    const double R = fma(-0.5, ra + rb, hb2);
    return (R < 0.0) || (ra * rb > R * R);
}

__device__ __forceinline__ double half_axis2(double B, double eta, int k) {
    const double Bk = fma(ldexp(B, -k), 1.0 + kAxisInflate, eta);
    return 0.5 * Bk * Bk;
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

// gamma(t) = sum_i C(n,i) w_i P_i t^i (1-t)^(n-i) / sum_i C(n,i) w_i t^i (1-t)^(n-i).
// Slot j holds index i = n - j, so Horner in t runs j = 0..n with (1-t)^j.
__device__ __forceinline__ void bez_eval(const Coef& c, double t, double& X, double& Y) {
    const double s = 1.0 - t;
    double ax = c.x[0], ay = c.y[0], aw = c.w[0], sp = 1.0;
#pragma unroll
    for (int j = 1; j < kCoef; ++j) {
        if (j <= c.n) {
            sp *= s;
            ax = fma(ax, t, c.x[j] * sp);
            ay = fma(ay, t, c.y[j] * sp);
            aw = fma(aw, t, c.w[j] * sp);
        }
    }
    if (c.rat) {
        const double r = 1.0 / aw;
        X = ax * r;
        Y = ay * r;
    } else {
        X = ax;
        Y = ay;
    }
}

// ---------------------------------------------------------------------------
// near pair: Alg. 1 on an explicit stack.  The root [0,1] is known to be
// inside its ellipse and not on the boundary.  Points are kept relative to
// the query.  `stk` is this lane's slot 0 in LDS (slot stride kWave).
// Returns the deepest level reached; sets onb on an eps hit.
// ---------------------------------------------------------------------------
__device__ int near_pair(Turn& T, const Coef& c, double B, double eta, double pnx, double pny, double qx, double qy,
                         double ax, double ay, double ra, double bx, double by, double rb, double eps2,
                         double2* stk, bool& onb) {
    double a = 0.0;  // left end of the current node, exact dyadic
    int k = 0;       // level: node = [a, a + 2^-k]
    uint64_t pend = 0, stored = 0;
    int maxk = 0;
    bool inside = true;
    for (;;) {
        if (inside) {
            if (k >= kDepthCap) {
                onb = true;  // cannot happen for a validated eps (depth bound <= cap)
                return maxk;
            }
            const int k1 = k + 1;
            const int slot = k1 & (kStackSlots - 1);
            stk[slot * kWave] = make_double2(bx, by);
            if (k1 >= kStackSlots) stored &= ~(1ull << (k1 - kStackSlots));
            stored |= 1ull << k1;
            pend |= 1ull << k1;
            double mx, my;
            bez_eval(c, a + ldexp(1.0, -k1), mx, my);
            mx -= qx;
            my -= qy;
            const double rm = mx * mx + my * my;
            if (rm < eps2) {
                onb = true;
                return k1;
            }
            bx = mx;
            by = my;
            rb = rm;
            k = k1;
            maxk = k1 > maxk ? k1 : maxk;
        } else {
            turn_mul(T, ax * bx + ay * by, ax * by - ay * bx);
            if (pend == 0) return maxk;
            turn_norm(T);
            const int kk = 63 - __clzll(pend);
            pend &= ~(1ull << kk);
            a += ldexp(1.0, -k);
            ax = bx;
            ay = by;
            ra = rb;
            if (stored & (1ull << kk)) {
                const double2 p = stk[(kk & (kStackSlots - 1)) * kWave];
                bx = p.x;
                by = p.y;
            } else {
                const double t = a + ldexp(1.0, -kk);
                if (t == 1.0) {
                    bx = pnx;
                    by = pny;
                } else {
                    bez_eval(c, t, bx, by);
                }
                bx -= qx;
                by -= qy;
            }
            stored &= ~(1ull << kk);
            rb = bx * bx + by * by;
            k = kk;
        }
        inside = !outside_ellipse(ra, rb, half_axis2(B, eta, k));
    }
}

// Near pair with all segment data read from global memory.
__device__ __forceinline__ int near_from_global(Turn& T, const Segs& sg, uint32_t s, double qx, double qy,
                                                double eps2, double2* stk, bool& onb) {
    const double ax = sg.p0x[s] - qx, ay = sg.p0y[s] - qy;
    const double pnx = sg.pnx[s], pny = sg.pny[s];
    const double bx = pnx - qx, by = pny - qy;
    Coef c;
    load_coef(sg, s, c);
    return near_pair(T, c, sg.B[s], sg.eta[s], pnx, pny, qx, qy, ax, ay, ax * ax + ay * ay, bx, by, bx * bx + by * by,
                     eps2, stk, onb);
}

__device__ __forceinline__ uint8_t classify(double omega, int rule) {
    if (rule == 1) return omega > 0.5 ? 1 : 0;
    return fabs(omega) > 0.5 ? 1 : 0;
}

}  // namespace wn
