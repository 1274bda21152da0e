// Periodic domains on the GPU (gfx950): covering-space lift and the
// far-field pass over lifted loop copies (Sec. 4.3-4.5).
//
// Lift (Sec. 4.3): one lane per loop walks its segments and translates
// segment i by o_i = o_{i-1} + T * round((end_{i-1} - start_i) / T) on each
// periodic axis, so that the loop becomes a connected curve of the covering
// space; v = lifted end - start, homology h = round(v / T).
//
// Far field over copies: a query x of a periodic face sums
//   - extended curves (cylinder, Sec. 4.4): copies x - k v for k in the
//     query's own window [k_lo, k_hi] plus two rays along v outside it;
//   - contractible loops: lattice copies whose box (widened by one period)
//     holds x;
//   - torus pairs (eq. bandWN): families m in the query's window, each the
//     extended curves of alpha and of the paired beta copy, shifted by t_m.
// Each lane uses exactly its own windows (the truncation is part of the
// definition for loops with open joints); a wave walks the union of its
// lanes' windows and masks the lanes outside.  Segment data is read with
// wave-uniform addresses (broadcast through the scalar/vector caches).
#include "wn_device.h"

namespace wn {

__device__ __forceinline__ long iround_d(double x) { return (long)floor(x + 0.5); }

__global__ __launch_bounds__(256) void k_lift(LiftArgs a, Segs sg) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.nloops) return;
    const int l = a.loops[t];
    const int f = a.loop_face[l];
    const int dom = a.face_dom[f];
    const double Tu = a.face_per[2 * f], Tv = a.face_per[2 * f + 1];
    const bool perv = dom == 2;
    const int s0 = a.loop_seg[l], s1 = a.loop_seg[l + 1];
    double* p0x = const_cast<double*>(sg.p0x);
    double* p0y = const_cast<double*>(sg.p0y);
    double* pnx = const_cast<double*>(sg.pnx);
    double* pny = const_cast<double*>(sg.pny);
    double* coef = const_cast<double*>(sg.coef);
    double ox = 0.0, oy = 0.0, ex = 0.0, ey = 0.0;
    for (int s = s0; s < s1; ++s) {
        const int64_t c0 = a.seg_cp[s], c1 = a.seg_cp[s + 1] - 1;
        if (s > s0) {
            ox += Tu * (double)iround_d((ex - a.cpu[c0]) / Tu);
            if (perv) oy += Tv * (double)iround_d((ey - a.cpv[c0]) / Tv);
        }
        a.seg_off[2 * s] = ox;
        a.seg_off[2 * s + 1] = oy;
        ex = a.cpu[c1];
        ey = a.cpv[c1];
        p0x[s] = a.cpu[c0] + ox;
        p0y[s] = a.cpv[c0] + oy;
        pnx[s] = a.cpu[c1] + ox;
        pny[s] = a.cpv[c1] + oy;
        const int n = (int)(c1 - c0);
        double* box = const_cast<double*>(sg.box) + 4 * (size_t)s;
        box[0] = INFINITY;
        box[1] = -INFINITY;
        box[2] = INFINITY;
        box[3] = -INFINITY;
        for (int64_t c = c0; c <= c1; ++c) {
            box[0] = fmin(box[0], a.cpu[c] + ox);
            box[1] = fmax(box[1], a.cpu[c] + ox);
            box[2] = fmin(box[2], a.cpv[c] + oy);
            box[3] = fmax(box[3], a.cpv[c] + oy);
        }
        for (int j = 0; j <= n; ++j) {  // slot j: control point j
            double* slot = coef + ((size_t)s * kCoef + j) * 4;
            slot[0] = a.cpu[c0 + j] * slot[2] + ox * slot[2];
            slot[1] = a.cpv[c0 + j] * slot[2] + oy * slot[2];
        }
        double* rec = coef + (size_t)s * kCoef * 4;  // the near pass's copy of the lifted end points
        rec[kPadP0x * 4 + 3] = p0x[s];
        rec[kPadP0y * 4 + 3] = p0y[s];
        rec[kPadPnx * 4 + 3] = pnx[s];
        rec[kPadPny * 4 + 3] = pny[s];
    }
    PLoop L{};
    L.s0 = s0;
    L.s1 = s1;
    if (s1 > s0) {
        const int64_t cs = a.seg_cp[s0], ce = a.seg_cp[s1] - 1;
        L.b0x = a.cpu[cs];
        L.b0y = a.cpv[cs];
        L.vx = a.cpu[ce] + a.seg_off[2 * (s1 - 1)] - L.b0x;
        L.vy = a.cpv[ce] + a.seg_off[2 * (s1 - 1) + 1] - L.b0y;
        L.h0 = (int)iround_d(L.vx / Tu);
        L.h1 = perv ? (int)iround_d(L.vy / Tv) : 0;
        L.lv = hypot(L.vx, L.vy);
        if (L.lv > 0.0) {
            L.dx = L.vx / L.lv;
            L.dy = L.vy / L.lv;
        }
        L.bb[0] = L.bb[2] = INFINITY;
        L.bb[1] = L.bb[3] = -INFINITY;
        L.xi_lo = INFINITY;
        L.xi_hi = -INFINITY;
        for (int s = s0; s < s1; ++s) {
            const double o0 = a.seg_off[2 * s], o1 = a.seg_off[2 * s + 1];
            for (int64_t c = a.seg_cp[s]; c < a.seg_cp[s + 1]; ++c) {
                const double px = a.cpu[c] + o0, py = a.cpv[c] + o1;
                L.bb[0] = fmin(L.bb[0], px);
                L.bb[1] = fmax(L.bb[1], px);
                L.bb[2] = fmin(L.bb[2], py);
                L.bb[3] = fmax(L.bb[3], py);
                const double xi = L.dx * (px - L.b0x) + L.dy * (py - L.b0y);
                L.xi_lo = fmin(L.xi_lo, xi);
                L.xi_hi = fmax(L.xi_hi, xi);
            }
        }
    }
    a.out[l] = L;
}

hipError_t launch_lift(const LiftArgs& a, Segs sg_mut, hipStream_t st) {
    if (a.nloops <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lift, dim3((a.nloops + 255) / 256), dim3(256), 0, st, a, sg_mut);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// periodic far-field kernel: 4 waves per workgroup, each wave owns 64 queries
// ---------------------------------------------------------------------------
__device__ __forceinline__ long wave_min_l(long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ long wave_max_l(long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

struct PerLane {
    double qx, qy;
    int64_t qi;
    bool valid, onb, lost;
    Turn T;
    int xc;     // integer parts of near pairs recursed in line (2 pi units)
    int nfill;  // entries in the wave's near-pair buffer (wave-uniform)
    int cnt;    // pairs since the start (wave-uniform)
    uint32_t pairs;  // (segment, copy) pairs in this query's windows (work counter)
};

// Per-wave resources: near-pair staging buffers (queue variant) or the
// recursion stack (in-line variants).
struct PerWave {
    uint2* buf;
    double2* sbuf;
    NearQueue nq;
    double4* stk;
    double eps2;
    int lane;
};

// Append the wave's buffered near pairs (with their copy translation) to the
// queue with one atomic; lanes whose query lost a pair set P.lost.
__device__ void flush_near_per(const PerWave& W, PerLane& P) {
    const int nfill = P.nfill;
    P.nfill = 0;
    if (nfill == 0) return;
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (W.lane == 0) base = atomicAdd(W.nq.count, (unsigned long long)nfill);
    base = __shfl(base, 0);
    for (int e = W.lane; e < nfill; e += kWave) {
        if (base + (unsigned long long)e < W.nq.cap) {
            W.nq.qs[base + e] = W.buf[e];
            W.nq.shift[base + e] = W.sbuf[e];
        }
    }
    if (base + (unsigned long long)nfill > W.nq.cap) {
        for (int e = 0; e < nfill; ++e)
            if (base + (unsigned long long)e >= W.nq.cap && (int64_t)W.buf[e].x == P.qi) P.lost = true;
    }
    __builtin_amdgcn_wave_barrier();
}

// All segments of loop L seen from the query translated by -(shx, shy);
// lanes with act == false contribute nothing.  Each pair multiplies in its
// chord angle (periodic loops typically have open joints, so chains of
// bit-joined segments as in the planar pass would be one segment long); a
// near pair's integer rest comes from the near pass.
template <int MODE>
__device__ __forceinline__ void loop_copy(const Segs& sg, const PLoop& L, double shx, double shy, bool act,
                                          PerLane& P, const PerWave& W) {
    const double xq = P.qx - shx, yq = P.qy - shy;
    if (act && P.valid) P.pairs += (uint32_t)(L.s1 - L.s0);
    FarRec nx = kload(sg.frec, L.s0);
    for (int s = L.s0; s < L.s1; ++s) {
        const FarRec r = nx;  // loaded one segment ahead
        nx = kload(sg.frec, s + 1 < L.s1 ? s + 1 : s);
        const double ax = r.p0x - xq, ay = r.p0y - yq;
        const double bx = r.pnx - xq, by = r.pny - yq;
        const double ra = ax * ax + ay * ay, rb = bx * bx + by * by;
        const bool work = act && P.valid && !P.onb;
        if (work && (ra < W.eps2 || rb < W.eps2)) P.onb = true;
        const bool far = outside_ellipse(ra, rb, r.hb2);
        if (work && far) turn_mul(P.T, ax * bx + ay * by, ax * by - ay * bx);
        const bool need = work && !P.onb && !far;
        if (need) chord_factor(P.T, ax, ay, bx, by);  // the near pass adds the integer rest
        if constexpr (MODE == kPerQueue) {
            const uint64_t m = __ballot(need);
            if (m) {
                const int cntm = __popcll(m);
                if (P.nfill + cntm > kNearBuf) flush_near_per(W, P);
                const int rank = __popcll(m & ((1ull << W.lane) - 1ull));
                if (need) {
                    W.buf[P.nfill + rank] = make_uint2((uint32_t)P.qi, (uint32_t)s);
                    W.sbuf[P.nfill + rank] = make_double2(shx, shy);
                }
                P.nfill += cntm;
            }
        } else {
            if (need) (void)near_from_global(P.xc, sg, (uint32_t)s, xq, yq, W.eps2, W.stk, P.onb);
        }
        if ((++P.cnt & 3) == 0) turn_norm(P.T);
    }
}

// Extended curve of loop L (Sec. 4.4) seen from the query translated by -(sx, sy).
template <int MODE>
__device__ __forceinline__ void extended(const Segs& sg, const PLoop& L, double sx, double sy, bool act,
                                         PerLane& P, const PerWave& W) {
    const double xs = P.qx - sx, ys = P.qy - sy;
    const double xi = L.dx * (xs - L.b0x) + L.dy * (ys - L.b0y);
    const bool a = act && P.valid;
    const long klo = (long)floor((xi - L.xi_hi) / L.lv) - 1;
    const long khi = (long)ceil((xi - L.xi_lo) / L.lv) + 1;
    const long Klo = wave_min_l(a ? klo : LONG_MAX);
    const long Khi = wave_max_l(a ? khi : LONG_MIN);
    for (long k = Klo; k <= Khi; ++k) {
        const bool in = a && k >= klo && k <= khi;
        loop_copy<MODE>(sg, L, sx + (double)k * L.vx, sy + (double)k * L.vy, in, P, W);
    }
    if (a) {
        const double ax = L.b0x + (double)klo * L.vx - xs, ay = L.b0y + (double)klo * L.vy - ys;
        const double bx = L.b0x + (double)(khi + 1) * L.vx - xs, by = L.b0y + (double)(khi + 1) * L.vy - ys;
        // back ray: from direction -d to a; forward ray: from b to direction d
        turn_mul(P.T, -L.dx * ax - L.dy * ay, -L.dx * ay + L.dy * ax);
        turn_norm(P.T);
        turn_mul(P.T, bx * L.dx + by * L.dy, bx * L.dy - by * L.dx);
        turn_norm(P.T);
    }
}

// Shared memory of one variant: staging buffers or recursion stacks.
template <int MODE>
struct PerShared;
template <>
struct PerShared<kPerQueue> {
    uint2 nbuf[kWavesPerWG][kNearBuf];
    double2 nsh[kWavesPerWG][kNearBuf];
    int item;
};
template <>
struct PerShared<kPerInline> {
    double4 stack[kWavesPerWG * kNearSlots * kWave];
    int item;
};
template <>
struct PerShared<kPerRedo> : PerShared<kPerInline> {};

// Output (all variants): the far-field angle sum (radians, integer near
// parts included for the in-line variants) and label 0 / 2 (boundary) /
// 3 (invalid) / kRedo; k_finalize turns them into winding numbers.
template <int MODE>
__global__ __launch_bounds__(kWG) void k_far_periodic(Segs sg, FaceTab ft, Points pts, const int32_t* item_offs,
                                                      const int2* item_map, uint32_t* item_counter, NearQueue nq,
                                                      Out out, double eps2, PerTab pt,
                                                      const uint32_t* perm, unsigned long long* stat_pairs) {
    __shared__ PerShared<MODE> sh;
    if (MODE == kPerRedo && *nq.count <= nq.cap) return;  // the queue never overflowed: nothing was lost
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    PerWave W;
    if constexpr (MODE == kPerQueue) {
        W.buf = sh.nbuf[wave];
        W.sbuf = sh.nsh[wave];
        W.stk = nullptr;
    } else {
        W.buf = nullptr;
        W.sbuf = nullptr;
        W.stk = sh.stack + wave * kNearSlots * kWave + lane;
    }
    W.nq = nq;
    W.eps2 = eps2;
    W.lane = lane;
    const int total = kload(item_offs, ft.num_faces);
    for (int iter = 0;; ++iter) {
        int item;
        if (item_counter) {
            __syncthreads();
            if (tid == 0) sh.item = (int)atomicAdd(item_counter, 1u);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(sh.item);  // uniform: face data via scalar loads
        } else {
            if (iter > 0) break;
            item = blockIdx.x;
        }
        if (item >= total) break;
        const int2 mp = kload(item_map, item);
        const int f = mp.x, tile = mp.y;
        int64_t qb = kload(pts.offs, f), qe = kload(pts.offs, f + 1);
        qb = qb < 0 ? 0 : (qb > pts.n ? pts.n : qb);
        qe = qe < qb ? qb : (qe > pts.n ? pts.n : qe);
        PerLane P;
        // slot of the face's (spatially ordered) point list -> point index
        const int64_t slot = qb + (int64_t)tile * (kWave * kWavesPerWG) + wave * kWave + lane;
        bool active = slot < qe;
        P.qi = (perm && active) ? (int64_t)perm[slot] : slot;
        if constexpr (MODE == kPerRedo) {
            active = active && out.lab[P.qi] == kRedo;
            if (!__any(active)) continue;  // no __syncthreads below: waves may skip independently
        }
        P.qx = P.qy = 0.0;
        if (active) {
            P.qx = pts.u[P.qi * pts.stride];
            P.qy = pts.v[P.qi * pts.stride];
        }
        P.valid = active && fabs(P.qx) < kCoordLimit && fabs(P.qy) < kCoordLimit;
        if (!P.valid) P.qx = P.qy = 0.0;
        P.onb = false;
        P.lost = false;
        P.T = Turn{1.0, 0.0, 0};
        P.xc = 0;
        P.nfill = 0;
        P.cnt = 0;
        P.pairs = 0;
        const PFace pf = kload(pt.face, f);
        for (int u = pf.u0; u < pf.u1; ++u) {
            const PUnit U = kload(pt.unit, u);
            if (U.kind == kUnitExtended) {
                extended<MODE>(sg, kload(pt.loop, U.la), 0.0, 0.0, true, P, W);
            } else if (U.kind == kUnitContractible) {
                const PLoop L = kload(pt.loop, U.la);
                const long ilo = (long)ceil((P.qx - L.bb[1]) / pf.Tu) - 1;
                const long ihi = (long)floor((P.qx - L.bb[0]) / pf.Tu) + 1;
                long jlo = 0, jhi = 0;
                if (pf.dom == 2) {
                    jlo = (long)ceil((P.qy - L.bb[3]) / pf.Tv) - 1;
                    jhi = (long)floor((P.qy - L.bb[2]) / pf.Tv) + 1;
                }
                const long Ilo = wave_min_l(P.valid ? ilo : LONG_MAX), Ihi = wave_max_l(P.valid ? ihi : LONG_MIN);
                const long Jlo = wave_min_l(P.valid ? jlo : LONG_MAX), Jhi = wave_max_l(P.valid ? jhi : LONG_MIN);
                for (long i = Ilo; i <= Ihi; ++i)
                    for (long j = Jlo; j <= Jhi; ++j) {
                        const bool in = P.valid && i >= ilo && i <= ihi && j >= jlo && j <= jhi;
                        loop_copy<MODE>(sg, L, (double)i * pf.Tu, (double)j * pf.Tv, in, P, W);
                    }
            } else {
                const PLoop La = kload(pt.loop, U.la);
                const double eta = pf.nx * (P.qx - La.b0x) + pf.ny * (P.qy - La.b0y);
                const long mlo = (long)floor((eta - U.eta_hi) / pf.Delta) - 1;
                const long mhi = (long)ceil((eta - U.eta_lo) / pf.Delta) + 1;
                const long Mlo = wave_min_l(P.valid ? mlo : LONG_MAX), Mhi = wave_max_l(P.valid ? mhi : LONG_MIN);
                for (long m = Mlo; m <= Mhi; ++m) {
                    const bool in = P.valid && m >= mlo && m <= mhi;
                    const double tx = (double)m * pf.t1x, ty = (double)m * pf.t1y;
                    extended<MODE>(sg, La, tx, ty, in, P, W);
                    extended<MODE>(sg, kload(pt.loop, U.lb), tx + U.pshx, ty + U.pshy, in, P, W);
                }
            }
        }
        if constexpr (MODE == kPerQueue) flush_near_per(W, P);
        if (active) {
            out.w[P.qi] = turn_angle(P.T) + kTwoPi * ((double)P.xc + pf.offset);
            out.lab[P.qi] = !P.valid ? 3 : (P.onb ? 2 : (P.lost ? kRedo : 0));
        }
        if (stat_pairs) {  // work counter: one atomic per wave and item
            unsigned long long c = active ? (unsigned long long)P.pairs : 0ull;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
            if (lane == 0 && c) atomicAdd(stat_pairs, c);
        }
    }
}

// Spatial order of each periodic face's points: a counting sort by the
// Morton index of their 16 x 16 bin in the bounding box of the face's points
// (points with invalid coordinates go to bin 0).  perm[qb + r] is the r-th
// point of the face in that order, so a wave holds neighbouring points whose
// copy windows overlap and the wave's union of windows stays narrow.  The
// results do not depend on the order: a lane only accumulates the copies of
// its own window, in the same order.  One workgroup per face; faces with more
// than kOrderMaxPoints points get the identity.
constexpr int kOrderSide = 16, kOrderBins = kOrderSide * kOrderSide;
static_assert(kOrderBins == kWG, "one bin per thread");

__device__ __forceinline__ uint32_t morton8(uint32_t x, uint32_t y) {
    uint32_t z = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) z |= ((x >> b) & 1u) << (2 * b) | ((y >> b) & 1u) << (2 * b + 1);
    return z;
}

__global__ __launch_bounds__(kWG) void k_spatial_order(FaceTab ft, Points pts, uint32_t* perm) {
    __shared__ uint32_t s_cnt[kOrderBins];
    __shared__ double s_box[kWavesPerWG][4];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const int f = ft.order[blockIdx.x];
    int64_t qb = pts.offs[f], qe = pts.offs[f + 1];
    qb = qb < 0 ? 0 : (qb > pts.n ? pts.n : qb);
    qe = qe < qb ? qb : (qe > pts.n ? pts.n : qe);
    if (qe - qb > kOrderMaxPoints) {
        for (int64_t i = qb + tid; i < qe; i += kWG) perm[i] = (uint32_t)i;
        return;
    }
    auto ok = [](double x) { return fabs(x) < kCoordLimit; };  // false for NaN
    double b0 = INFINITY, b1 = -INFINITY, b2 = INFINITY, b3 = -INFINITY;
    for (int64_t i = qb + tid; i < qe; i += kWG) {
        const double u = pts.u[i * pts.stride], v = pts.v[i * pts.stride];
        if (ok(u) && ok(v)) {
            b0 = fmin(b0, u);
            b1 = fmax(b1, u);
            b2 = fmin(b2, v);
            b3 = fmax(b3, v);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        b0 = fmin(b0, __shfl_xor(b0, off));
        b1 = fmax(b1, __shfl_xor(b1, off));
        b2 = fmin(b2, __shfl_xor(b2, off));
        b3 = fmax(b3, __shfl_xor(b3, off));
    }
    if (lane == 0) {
        s_box[wave][0] = b0;
        s_box[wave][1] = b1;
        s_box[wave][2] = b2;
        s_box[wave][3] = b3;
    }
    s_cnt[tid] = 0;
    __syncthreads();
    for (int w = 0; w < kWavesPerWG; ++w) {
        b0 = fmin(b0, s_box[w][0]);
        b1 = fmax(b1, s_box[w][1]);
        b2 = fmin(b2, s_box[w][2]);
        b3 = fmax(b3, s_box[w][3]);
    }
    const double su = b1 > b0 ? kOrderSide / (b1 - b0) : 0.0, sv = b3 > b2 ? kOrderSide / (b3 - b2) : 0.0;
    auto bin_of = [&](int64_t i) -> uint32_t {
        const double u = pts.u[i * pts.stride], v = pts.v[i * pts.stride];
        if (!(ok(u) && ok(v))) return 0u;
        const int x = min(kOrderSide - 1, max(0, (int)((u - b0) * su)));
        const int y = min(kOrderSide - 1, max(0, (int)((v - b2) * sv)));
        return morton8((uint32_t)x, (uint32_t)y);
    };
    for (int64_t i = qb + tid; i < qe; i += kWG) atomicAdd(&s_cnt[bin_of(i)], 1u);
    __syncthreads();
    // exclusive scan of the 256 counts (Hillis-Steele on the inclusive sums)
    uint32_t c = s_cnt[tid];
    const uint32_t mine = c;
    for (int off = 1; off < kOrderBins; off <<= 1) {
        __syncthreads();
        const uint32_t o = tid >= off ? s_cnt[tid - off] : 0u;
        __syncthreads();
        c += o;
        s_cnt[tid] = c;
    }
    __syncthreads();
    s_cnt[tid] = c - mine;
    __syncthreads();
    for (int64_t i = qb + tid; i < qe; i += kWG) {
        const uint32_t r = atomicAdd(&s_cnt[bin_of(i)], 1u);
        perm[qb + r] = (uint32_t)i;
    }
}

hipError_t launch_spatial_order(const FaceTab& ft, const Points& pts, uint32_t* perm, hipStream_t st) {
    if (ft.num_faces <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spatial_order, dim3((unsigned)ft.num_faces), dim3(kWG), 0, st, ft, pts, perm);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_per(const Segs& sg, const FaceTab& ft, const Points& pts, const int32_t* item_offs,
                             const int2* item_map, uint32_t* item_counter, int64_t grid, NearQueue nq, Out out,
                             double eps2, PerTab pt, const uint32_t* perm, hipStream_t st,
                             unsigned long long* stat_pairs) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_far_periodic<MODE>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, ft, pts, item_offs, item_map,
                       item_counter, nq, out, eps2, pt, perm, stat_pairs);
    return hipGetLastError();
}

hipError_t launch_far_periodic(int mode, const Segs& sg, const FaceTab& ft, const Points& pts,
                               const int32_t* item_offs, const int2* item_map, uint32_t* item_counter, int64_t grid,
                               NearQueue nq, Out out, double eps2, PerTab pt, const uint32_t* perm, hipStream_t st,
                               unsigned long long* stat_pairs) {
    switch (mode) {
        case kPerQueue:
            return launch_per<kPerQueue>(sg, ft, pts, item_offs, item_map, item_counter, grid, nq, out, eps2, pt, perm,
                                   st, stat_pairs);
        case kPerInline:
            return launch_per<kPerInline>(sg, ft, pts, item_offs, item_map, item_counter, grid, nq, out, eps2, pt, perm,
                                   st, stat_pairs);
        case kPerRedo:
            return launch_per<kPerRedo>(sg, ft, pts, item_offs, item_map, item_counter, grid, nq, out, eps2, pt, perm,
                                   st, stat_pairs);
        default:
            return hipErrorInvalidValue;
    }
}

int far_periodic_blocks_per_cu(int mode) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (mode == kPerQueue)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_far_periodic<kPerQueue>, kWG, 0);
    else if (mode == kPerInline)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_far_periodic<kPerInline>, kWG, 0);
    else if (mode == kPerRedo)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_far_periodic<kPerRedo>, kWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace wn
