// Host-side topology of periodic faces (Sec. 4.5, App. B-C): loop classes,
// homology checks and the pairing of torus loops.  Runs once per face set in
// wn_create_faces, on the lift computed by k_lift.
//
// Torus reading: loops split into A (h = +h*), B (h = -h*), C (h = 0),
// h* normalised to h1 > 0 (or h1 = 0, h2 > 0).  |A| = |B| and gcd(h1, h2) = 1
// are required.  Lattice copies of a loop fall into families m in Z with
// translation t_m = m (-b T_u, a T_v), a h1 + b h2 = 1 (re-indexing of the
// families gamma_{r,s}).  Each alpha is paired with the copy beta + t_m, over
// unused beta in B, that lies nearest on alpha's left, "left of" being a
// positive extended winding number at a point of the candidate (App. C,
// ToLeft / PairLoop / PairLoops).
#include "wn_internal.h"
#include "wn_topology.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace wn {
namespace {

constexpr double kPi = 3.14159265358979323846;

// de Casteljau point evaluation in homogeneous coordinates (host).
void hseg_eval(const HostSeg& s, double t, double& X, double& Y) {
    double x[kCoef], y[kCoef], w[kCoef];
    for (int i = 0; i <= s.n; ++i) {
        x[i] = s.w[i] * s.x[i];
        y[i] = s.w[i] * s.y[i];
        w[i] = s.w[i];
    }
    for (int k = 1; k <= s.n; ++k)
        for (int i = 0; i <= s.n - k; ++i) {
            x[i] = (1 - t) * x[i] + t * x[i + 1];
            y[i] = (1 - t) * y[i] + t * y[i + 1];
            w[i] = (1 - t) * w[i] + t * w[i + 1];
        }
    X = x[0] / w[0];
    Y = y[0] / w[0];
}

// Alg. 1 (recursive) seen from (px, py); angle in radians.
double hseg_angle(const HostSeg& s, double px, double py, double a, double b, double Ax, double Ay, double Bx,
                  double By, int depth) {
    const double ax = Ax - px, ay = Ay - py, bx = Bx - px, by = By - py;
    const double d1 = hypot(ax, ay), d2 = hypot(bx, by);
    if (d1 + d2 > s.B * (b - a) * (1.0 + 1e-9) + 1e-13 || depth >= 50)
        return atan2(ax * by - ay * bx, ax * bx + ay * by);
    const double m = 0.5 * (a + b);
    double Mx, My;
    hseg_eval(s, m, Mx, My);
    return hseg_angle(s, px, py, a, m, Ax, Ay, Mx, My, depth + 1) + hseg_angle(s, px, py, m, b, Mx, My, Bx, By, depth + 1);
}

double loop_turns(const std::vector<HostSeg>& segs, const PLoop& L, double x, double y) {
    double acc = 0.0;
    for (int s = L.s0; s < L.s1; ++s) {
        const HostSeg& g = segs[s];
        acc += hseg_angle(g, x, y, 0.0, 1.0, g.x[0], g.y[0], g.x[g.n], g.y[g.n], 0);
    }
    return acc / (2 * kPi);
}

// Extended curve of L (Sec. 4.4) seen from (x, y), same windows as the kernels.
double host_extended(const std::vector<HostSeg>& segs, const PLoop& L, double x, double y) {
    const double xi = L.dx * (x - L.b0x) + L.dy * (y - L.b0y);
    const long klo = (long)floor((xi - L.xi_hi) / L.lv) - 1;
    const long khi = (long)ceil((xi - L.xi_lo) / L.lv) + 1;
    double acc = 0.0;
    for (long k = klo; k <= khi; ++k) acc += loop_turns(segs, L, x - (double)k * L.vx, y - (double)k * L.vy);
    const double ax = L.b0x + (double)klo * L.vx - x, ay = L.b0y + (double)klo * L.vy - y;
    const double bx = L.b0x + (double)(khi + 1) * L.vx - x, by = L.b0y + (double)(khi + 1) * L.vy - y;
    const double rb = atan2(-L.dx * ay + L.dy * ax, -L.dx * ax - L.dy * ay);
    const double rf = atan2(bx * L.dy - by * L.dx, bx * L.dx + by * L.dy);
    return acc + (rb + rf) / (2 * kPi);
}

void loop_point(const std::vector<HostSeg>& segs, const PLoop& L, double& x, double& y) {
    const HostSeg& g = segs[L.s0 + (L.s1 - L.s0) / 2];
    x = g.x[0];
    y = g.y[0];
}

// Mean height of the extended curve of a non-contractible loop over one
// copy: the integral of v du along the lifted loop (its segments sampled as
// polylines) over the copy's u extent.  Two extended curves that do not
// cross are ordered by it (their difference is the area between them).
double mean_height(const std::vector<HostSeg>& segs, const PLoop& L) {
    constexpr int kSamples = 64;
    double I = 0.0;
    for (int s = L.s0; s < L.s1; ++s) {
        const HostSeg& g = segs[s];
        double px = g.x[0], py = g.y[0];
        for (int k = 1; k <= kSamples; ++k) {
            double x, y;
            if (k == kSamples) {
                x = g.x[g.n];
                y = g.y[g.n];
            } else {
                hseg_eval(g, (double)k / kSamples, x, y);
            }
            I += 0.5 * (py + y) * (x - px);
            px = x;
            py = y;
        }
    }
    return I / L.vx;
}

// Punctured sphere / cone (Sec. 4.3: puncturing the singular points leaves
// the cylinder case).  On the cylinder each extended curve adds +1/2 on its
// left and -1/2 on its right, so from below all of them the winding number
// steps by +1 across a loop running in +u and by -1 across one running in -u:
// region k gets -S/2 + p_k, p_k the partial sums of sign(h_u) in height
// order.  The constant c = S/2 - min_k p_k maps the regions to {0, 1}; a
// spread of more than one unit is no valid face (returns 1).
int puncture_offset(const std::vector<HostSeg>& segs, const std::vector<PLoop>& loops, int l0, int l1,
                    double& c) {
    std::vector<std::pair<double, int>> hs;
    for (int l = l0; l < l1; ++l) {
        const PLoop& L = loops[l];
        if (L.s1 == L.s0 || L.h0 == 0) continue;
        hs.push_back({mean_height(segs, L), L.h0 > 0 ? 1 : -1});
    }
    std::sort(hs.begin(), hs.end());
    int p = 0, lo = 0, hi = 0;
    for (const auto& e : hs) {
        p += e.second;
        lo = std::min(lo, p);
        hi = std::max(hi, p);
    }
    if (hi - lo > 1) return 1;
    c = 0.5 * (double)p - (double)lo;
    return 0;
}

long gcd_l(long a, long b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        const long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// a * x + b * y = gcd(a, b), a, b >= 0
void bezout(long a, long b, long& x, long& y) {
    long x0 = 1, y0 = 0, x1 = 0, y1 = 1;
    while (b != 0) {
        const long q = a / b;
        long t = a - q * b;
        a = b;
        b = t;
        t = x0 - q * x1;
        x0 = x1;
        x1 = t;
        t = y0 - q * y1;
        y0 = y1;
        y1 = t;
    }
    x = x0;
    y = y0;
}

}  // namespace

int torus_setup(int dom, double Tu, double Tv, int l0, int l1, const std::vector<PLoop>& loops, TorusSetup& ts) {
    ts = TorusSetup{};
    // common homology of the non-contractible loops
    int hs0 = 0, hs1 = 0;
    for (int l = l0; l < l1; ++l) {
        const PLoop& L = loops[l];
        if (L.s1 == L.s0 || (L.h0 == 0 && L.h1 == 0)) continue;
        int g0 = L.h0, g1 = L.h1;
        if (g0 < 0 || (g0 == 0 && g1 < 0)) {
            g0 = -g0;
            g1 = -g1;
        }
        if (hs0 == 0 && hs1 == 0) {
            hs0 = g0;
            hs1 = g1;
        }
        if (g0 != hs0 || g1 != hs1) return 1;  // two different homology classes
    }
    ts.hs0 = hs0;
    ts.hs1 = hs1;
    if (dom != 2 || (hs0 == 0 && hs1 == 0)) return 0;
    if (gcd_l(hs0, hs1) != 1) return 1;
    for (int l = l0; l < l1; ++l) {
        const PLoop& L = loops[l];
        if (L.s1 == L.s0) continue;
        if (L.h0 == hs0 && L.h1 == hs1) ts.A.push_back(l);
        else if (L.h0 == -hs0 && L.h1 == -hs1) ts.B.push_back(l);
    }
    if (ts.A.size() != ts.B.size()) return 1;
    long ea, eb;
    bezout(labs(hs0), labs(hs1), ea, eb);
    if (hs0 < 0) ea = -ea;
    if (hs1 < 0) eb = -eb;
    ts.t1x = -(double)eb * Tu;
    ts.t1y = (double)ea * Tv;
    const double vx = hs0 * Tu, vy = hs1 * Tv;
    const double lv = hypot(vx, vy);
    ts.nx = -vy / lv;
    ts.ny = vx / lv;
    ts.Delta = Tu * Tv / lv;
    return 0;
}

int torus_pair_host(const std::vector<HostSeg>& segs, const std::vector<PLoop>& loops, const TorusSetup& ts,
                    std::vector<int2>& choice) {
    choice.assign(ts.A.size(), make_int2(-1, 0));
    std::vector<char> used(ts.B.size(), 0);
    for (size_t ia = 0; ia < ts.A.size(); ++ia) {
        const PLoop& La = loops[ts.A[ia]];
        int best = -1;
        long bms = 0;
        double bshx = 0.0, bshy = 0.0;
        for (size_t j = 0; j < ts.B.size(); ++j) {
            if (used[j]) continue;
            const PLoop& Lb = loops[ts.B[j]];
            double px, py;
            loop_point(segs, Lb, px, py);
            const double eta = ts.nx * (px - La.b0x) + ts.ny * (py - La.b0y);
            const long m0 = (long)floor(-eta / ts.Delta);
            bool found = false;
            long ms = 0;
            for (long m = m0 - 3; m <= m0 + 4 && !found; ++m) {
                if (host_extended(segs, La, px + (double)m * ts.t1x, py + (double)m * ts.t1y) > 0.0) {
                    ms = m;
                    found = true;
                }
            }
            if (!found) continue;
            const double shx = (double)ms * ts.t1x, shy = (double)ms * ts.t1y;
            if (best < 0) {
                best = (int)j;
                bms = ms;
                bshx = shx;
                bshy = shy;
            } else {
                // the candidate replaces the best when it lies on the best's
                // left (App. C.2, PairLoops): the beta copies face alpha with
                // their left sides, so it is then the nearer one
                if (host_extended(segs, loops[ts.B[best]], px + shx - bshx, py + shy - bshy) > 0.0) {
                    best = (int)j;
                    bms = ms;
                    bshx = shx;
                    bshy = shy;
                }
            }
        }
        if (best < 0) return 1;
        used[best] = 1;
        choice[ia] = make_int2(best, (int)bms);
    }
    return 0;
}

int build_periodic_face(int dom, double Tu, double Tv, int l0, int l1, const std::vector<HostSeg>& segs,
                        const std::vector<PLoop>& loops, const TorusSetup* ts, const int2* choice,
                        std::vector<PUnit>& units, PFace& pf) {
    pf = PFace{};
    pf.dom = dom;
    pf.Tu = Tu;
    pf.Tv = Tv;
    pf.u0 = (int)units.size();
    TorusSetup local;
    if (!ts) {
        if (torus_setup(dom, Tu, Tv, l0, l1, loops, local) != 0) return 1;
        ts = &local;
    }
    const int hs0 = ts->hs0;
    for (int l = l0; l < l1; ++l) {
        const PLoop& L = loops[l];
        if (L.s1 == L.s0) continue;
        if (L.h0 == 0 && L.h1 == 0) {
            PUnit U{};
            U.kind = kUnitContractible;
            U.la = l;
            units.push_back(U);
        } else if (u_periodic_only(dom)) {
            if (hs0 > 1) return 1;  // a simple loop on a cylinder has |h| <= 1
            PUnit U{};
            U.kind = kUnitExtended;
            U.la = l;
            units.push_back(U);
        }
    }
    if ((dom == 3 || dom == 4) && puncture_offset(segs, loops, l0, l1, pf.offset) != 0) return 1;
    if (dom == 2 && (ts->hs0 != 0 || ts->hs1 != 0)) {
        pf.t1x = ts->t1x;
        pf.t1y = ts->t1y;
        pf.nx = ts->nx;
        pf.ny = ts->ny;
        pf.Delta = ts->Delta;
        std::vector<int2> host_choice;
        if (!choice) {
            if (torus_pair_host(segs, loops, *ts, host_choice) != 0) return 1;
            choice = host_choice.data();
        }
        std::vector<char> used(ts->B.size(), 0);
        for (size_t ia = 0; ia < ts->A.size(); ++ia) {
            const int a = ts->A[ia];
            const PLoop& La = loops[a];
            const int best = choice[ia].x;
            if (best < 0 || best >= (int)ts->B.size() || used[best]) return 1;
            used[best] = 1;
            const double bshx = (double)choice[ia].y * ts->t1x, bshy = (double)choice[ia].y * ts->t1y;
            PUnit U{};
            U.kind = kUnitPair;
            U.la = a;
            U.lb = ts->B[best];
            U.pshx = bshx;
            U.pshy = bshy;
            double lo = INFINITY, hi = -INFINITY;
            for (int w = 0; w < 2; ++w) {
                const PLoop& L = loops[w == 0 ? a : ts->B[best]];
                const double sx = w == 0 ? 0.0 : bshx, sy = w == 0 ? 0.0 : bshy;
                for (int s = L.s0; s < L.s1; ++s) {
                    const HostSeg& g = segs[s];
                    for (int i = 0; i <= g.n; ++i) {
                        const double e = pf.nx * (g.x[i] + sx - La.b0x) + pf.ny * (g.y[i] + sy - La.b0y);
                        lo = std::min(lo, e);
                        hi = std::max(hi, e);
                    }
                }
            }
            U.eta_lo = lo;
            U.eta_hi = hi;
            units.push_back(U);
        }
    }
    pf.u1 = (int)units.size();
    return 0;
}

}  // namespace wn
