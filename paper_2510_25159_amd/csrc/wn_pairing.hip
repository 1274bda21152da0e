// Torus pairing on the GPU (Sec. 4.5, App. C: ToLeft, PairLoop, PairLoops),
// run once per face set at creation, after the covering-space lift.
//
// One wave per torus face.  Each loop alpha of A, in order, takes the unused
// loop beta of B whose copy beta + m t_1 lies nearest on alpha's left:
//   - the probe point p of beta is the first control point of its middle
//     segment (lifted); the copy of beta in family m is "left of" alpha when
//     the extended winding number of alpha (Sec. 4.4) at p + m t_1 is
//     positive, and the first such m in a window of eight families around
//     the one that p's normal offset predicts is taken;
//   - a candidate replaces the best so far when it lies on the best's left
//     (the extended winding number of the best's copy at the candidate's
//     probe point is positive): the beta copies face alpha with their left
//     sides, so it is then the nearer one.
// The sequential choice over A is the wave's control flow; each extended
// winding number spreads its (copy, segment) pairs over the lanes: a pair's
// angle is its chord's principal angle plus 2 pi times Alg. 1's integer
// crossing correction (near_pair) when the query lies in the segment's root
// ellipse, and a wave sum adds them up.
#include "wn_device.h"

namespace wn {

// Angle (radians) of segment s (lifted) seen from (qx, qy), Alg. 1 with the
// axis inflation eta.
__device__ double seg_angle(const Segs& sg, int s, double qx, double qy, double eta, double eps2, double4* stk) {
    const double ax = sg.p0x[s] - qx, ay = sg.p0y[s] - qy;
    const double bx = sg.pnx[s] - qx, by = sg.pny[s] - qy;
    const double ra = fma(ax, ax, ay * ay), rb = fma(bx, bx, by * by);
    double th = arg_of(fma(ax, bx, ay * by), cross_raw(ax, ay, bx, by));
    const double Be = fma(sg.B[s], 1.0 + kAxisInflate, eta);
    if (!outside_ellipse(ra, rb, 0.5 * Be * Be)) {
        Coef c;
        load_coef(sg, s, c);
        int N = 0;
        bool onb = false;
        (void)near_pair(N, c, sg.B[s], eta, sg.pnx[s], sg.pny[s], qx, qy, ax, ay, ra, bx, by, rb, eps2, stk, onb);
        th += kTwoPi * (double)N;
    }
    return th;
}

// Extended winding number of loop L (Sec. 4.4) at (x, y), with the copy
// window of the query kernels: the lanes share the (copy, segment) pairs.
__device__ double pewn_wave(const Segs& sg, const PLoop& L, double x, double y, double eta, double eps2,
                            double4* stk, int lane) {
    const double xi = L.dx * (x - L.b0x) + L.dy * (y - L.b0y);
    const long klo = (long)floor((xi - L.xi_hi) / L.lv) - 1;
    const long khi = (long)ceil((xi - L.xi_lo) / L.lv) + 1;
    const int nseg = L.s1 - L.s0;
    const long total = (khi - klo + 1) * (long)nseg;
    double acc = 0.0;
    for (long i = lane; i < total; i += kWave) {
        const long k = klo + i / nseg;
        const int s = L.s0 + (int)(i % nseg);
        acc += seg_angle(sg, s, x - (double)k * L.vx, y - (double)k * L.vy, eta, eps2, stk);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    const double ax = L.b0x + (double)klo * L.vx - x, ay = L.b0y + (double)klo * L.vy - y;
    const double bx = L.b0x + (double)(khi + 1) * L.vx - x, by = L.b0y + (double)(khi + 1) * L.vy - y;
    // back ray: from direction -d to a; forward ray: from b to direction d
    const double rbk = arg_of(-L.dx * ax - L.dy * ay, -L.dx * ay + L.dy * ax);
    const double rfw = arg_of(bx * L.dx + by * L.dy, bx * L.dy - by * L.dx);
    return (acc + rbk + rfw) / kTwoPi;
}

__global__ __launch_bounds__(kWave) void k_pair_torus(Segs sg, const PLoop* loops, const PairJob* jobs,
                                                      const int32_t* lists, int2* out, double eps2) {
    __shared__ double4 s_stack[kNearSlots * kWave];
    const int lane = threadIdx.x;
    double4* stk = s_stack + lane;
    const PairJob J = jobs[blockIdx.x];
    uint64_t used = 0;  // nb <= 64 (checked on the host)
    for (int ia = 0; ia < J.na; ++ia) {
        const PLoop La = loops[lists[J.a0 + ia]];
        int best = -1, bms = 0;
        double bshx = 0.0, bshy = 0.0;
        for (int j = 0; j < J.nb; ++j) {
            if ((used >> j) & 1ull) continue;
            const PLoop Lb = loops[lists[J.b0 + j]];
            const int sm = Lb.s0 + (Lb.s1 - Lb.s0) / 2;  // probe: first control point of the middle segment
            const double px = sg.p0x[sm], py = sg.p0y[sm];
            const double eta = J.nx * (px - La.b0x) + J.ny * (py - La.b0y);
            const long m0 = (long)floor(-eta / J.Delta);
            bool found = false;
            long ms = 0;
            for (long m = m0 - 3; m <= m0 + 4 && !found; ++m) {
                if (pewn_wave(sg, La, px + (double)m * J.t1x, py + (double)m * J.t1y, J.eta, eps2, stk, lane) > 0.0) {
                    ms = m;
                    found = true;
                }
            }
            if (!found) continue;
            const double shx = (double)ms * J.t1x, shy = (double)ms * J.t1y;
            if (best < 0) {
                best = j;
                bms = (int)ms;
                bshx = shx;
                bshy = shy;
            } else {
                const PLoop Lbest = loops[lists[J.b0 + best]];
                if (pewn_wave(sg, Lbest, px + shx - bshx, py + shy - bshy, J.eta, eps2, stk, lane) > 0.0) {
                    best = j;
                    bms = (int)ms;
                    bshx = shx;
                    bshy = shy;
                }
            }
        }
        if (best >= 0) used |= 1ull << best;
        if (lane == 0) out[J.out0 + ia] = make_int2(best, bms);
    }
}

hipError_t launch_pair_torus(const Segs& sg, const PLoop* loops, const PairJob* jobs, int njobs, const int32_t* lists,
                             int2* out, double eps2, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_torus, dim3((unsigned)njobs), dim3(kWave), 0, st, sg, loops, jobs, lists, out, eps2);
    return hipGetLastError();
}

}  // namespace wn
