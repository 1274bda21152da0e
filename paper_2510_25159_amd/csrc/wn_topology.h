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

// Classify the loops [l0, l1) of one periodic face, check the homology
// conditions of Sec. 4.5 and append its units (extended curves, contractible
// loops, torus pairs).  Returns 0, or 1 on a topology violation.
int build_periodic_face(int dom, double Tu, double Tv, int l0, int l1, const std::vector<HostSeg>& segs,
                        const std::vector<PLoop>& loops, std::vector<PUnit>& units, PFace& pf);

}  // namespace wn
