// Host-side periodic topology (loop classes, pairing) of the library.
#pragma once

#include "wn_internal.h"

#include <vector>

namespace wn {

// One lifted segment on the host (control points with their lattice offset).
struct HostSeg {
    int n;
    double x[kCoef], y[kCoef], w[kCoef];
    double B;
};

// Periodic face: the common homology h* of its non-contractible loops (two
// classes are a topology violation); for a torus (dom 2) also the lists A
// (h = +h*) and B (h = -h*), the family step t_1 and the left normal /
// spacing of the families (Sec. 4.5).  Returns 1 on a topology violation
// (two homology classes; on a torus gcd(h1, h2) != 1 or |A| != |B|).
struct TorusSetup {
    int hs0 = 0, hs1 = 0;
    std::vector<int> A, B;
    double t1x = 0.0, t1y = 0.0, nx = 0.0, ny = 0.0, Delta = 0.0;
};
int torus_setup(int dom, double Tu, double Tv, int l0, int l1, const std::vector<PLoop>& loops, TorusSetup& ts);

// Pairing on the host (App. C: ToLeft, PairLoop, PairLoops): for each alpha
// in A, in order, choice[i] = (index j into B, family m of the shift m t_1).
// Returns 1 when some alpha finds no beta on its left.
int torus_pair_host(const std::vector<HostSeg>& segs, const std::vector<PLoop>& loops, const TorusSetup& ts,
                    std::vector<int2>& choice);

// Classify the loops [l0, l1) of one periodic face, check the homology
// conditions of Sec. 4.5 and append its units (extended curves, contractible
// loops, torus pairs).  ts / choice: the face's torus setup and pairing when
// already computed (the pairing may come from the GPU), else NULL (computed
// here, on the host).  Returns 0, or 1 on a topology violation.
int build_periodic_face(int dom, double Tu, double Tv, int l0, int l1, const std::vector<HostSeg>& segs,
                        const std::vector<PLoop>& loops, const TorusSetup* ts, const int2* choice,
                        std::vector<PUnit>& units, PFace& pf);

}  // namespace wn
