// Near pass with the subdivided control-point bound (a measured variant of
// Alg. 1; Sec. 4.2 and Table 1 contrast the ellipse bound with bounds taken
// from the control points of every sub-segment).
//
// A node [a, a + 2^-k] carries the control points of the curve restricted to
// it, in homogeneous coordinates relative to the query, (X_i, Y_i, W_i) =
// (w_i (P_i - q), w_i).  Splitting is de Casteljau's halving: the halves'
// control points are the first and the last entries of its levels, and its
// apex (their common point) is the midpoint.  A node's axis is the smaller of
// the global B 2^-k and the bound of Lemma 1 / App. A.1 computed from its own
// control points; both bound the sub-curve's length, so its ellipse still
// contains it, the recursion still sums the exact angle and omega does not
// change: only nodes the global bound would split can become leaves.
//
// The traversal is the near pass's (depth first, left first, both halves
// tested per step, the right one deferred when both fail; crossings on lane
// masks).  A deferred interval is kept as a level bit only: when it resumes,
// its control points are derived again by halving from the segment's, along
// the binary digits of its left end, and its end points are that piece's end
// control points (the same operations on the same values as when they were
// first formed as apexes, hence the same doubles), except t = 1, which is the
// segment's end point.  This costs O(n^2 k) per resumed interval, the price
// Table 1 puts on control-point bounds.
#include "wn_device.h"

namespace wn {

namespace {

constexpr double kBinomInv[kCoef][kCoef] = {
    {1.0, 0, 0, 0, 0, 0},
    {1.0, 1.0, 0, 0, 0, 0},
    {1.0, 0.5, 1.0, 0, 0, 0},
    {1.0, 1.0 / 3.0, 1.0 / 3.0, 1.0, 0, 0},
    {1.0, 0.25, 1.0 / 6.0, 0.25, 1.0, 0},
    {1.0, 0.2, 0.1, 0.1, 0.2, 1.0},
};

struct Piece {
    double X[kCoef], Y[kCoef], W[kCoef];
};

// The segment's control points relative to the query: the record holds
// C(n, j) w_j P_j in slot j; dividing by the binomial gives w_j P_j.
__device__ __forceinline__ void root_piece(const Segs& sg, uint32_t s, int n, double qx, double qy, Piece& P) {
    const double4* cf = reinterpret_cast<const double4*>(sg.coef) + (size_t)s * kCoef;
#pragma unroll
    for (int j = 0; j < kCoef; ++j) {
        const double4 v = cf[j];
        double inv = 0.0;
#pragma unroll
        for (int m = 1; m <= kMaxDeg; ++m) inv = n == m ? kBinomInv[m][j] : inv;
        const double w = v.z * inv;
        P.W[j] = w;
        P.X[j] = fma(-w, qx, v.x * inv);
        P.Y[j] = fma(-w, qy, v.y * inv);
    }
}

// Slot n of a piece's array (n varies per lane: selects, no dynamic index).
__device__ __forceinline__ double slot(const double (&v)[kCoef], int n) {
    double r = v[0];
#pragma unroll
    for (int j = 1; j < kCoef; ++j) r = j == n ? v[j] : r;
    return r;
}

// de Casteljau at 1/2 of degree n (slots above n untouched): L receives the
// left half, P the right half; returns the apex in L's slot n.
__device__ __forceinline__ void halve(Piece& P, Piece& L, int n) {
    L.X[0] = P.X[0];
    L.Y[0] = P.Y[0];
    L.W[0] = P.W[0];
#pragma unroll
    for (int r = 1; r <= kMaxDeg; ++r) {
#pragma unroll
        for (int i = 0; i + r <= kMaxDeg; ++i) {
            const bool upd = i + r <= n;
            P.X[i] = upd ? 0.5 * (P.X[i] + P.X[i + 1]) : P.X[i];
            P.Y[i] = upd ? 0.5 * (P.Y[i] + P.Y[i + 1]) : P.Y[i];
            P.W[i] = upd ? 0.5 * (P.W[i] + P.W[i + 1]) : P.W[i];
        }
        const bool keep = r <= n;
        L.X[r] = keep ? P.X[0] : L.X[r - 1];
        L.Y[r] = keep ? P.Y[0] : L.Y[r - 1];
        L.W[r] = keep ? P.W[0] : L.W[r - 1];
    }
}

// Lemma 1 / App. A.1 bound of a piece: n max |Q_i - Q_{i-1}| (polynomial) or
// min(n r max_{i,j} |Q_i - Q_j|, n r^2 max_i |Q_i - Q_{i-1}|), r the ratio of
// the largest to the smallest weight (rational); Q_i = (X_i, Y_i) / W_i.
__device__ __forceinline__ double piece_bound(const Piece& P, int n, bool rat) {
    double qx[kCoef], qy[kCoef];
    double wlo = P.W[0], whi = P.W[0];
#pragma unroll
    for (int i = 0; i < kCoef; ++i) {
        const double r = recip(i <= n ? P.W[i] : 1.0);
        qx[i] = P.X[i] * r;
        qy[i] = P.Y[i] * r;
        if (i > 0 && i <= n) {
            wlo = fmin(wlo, P.W[i]);
            whi = fmax(whi, P.W[i]);
        }
    }
    double leg2 = 0.0, diam2 = 0.0;
#pragma unroll
    for (int i = 1; i < kCoef; ++i) {
        const double dx = qx[i] - qx[i - 1], dy = qy[i] - qy[i - 1];
        if (i <= n) leg2 = fmax(leg2, fma(dx, dx, dy * dy));
    }
    if (rat) {
#pragma unroll
        for (int i = 0; i < kCoef; ++i)
#pragma unroll
            for (int j = i + 1; j < kCoef; ++j) {
                const double dx = qx[i] - qx[j], dy = qy[i] - qy[j];
                if (j <= n) diam2 = fmax(diam2, fma(dx, dx, dy * dy));
            }
    }
    const double nn = (double)n;
    if (!rat) return nn * sqrt(leg2);
    const double r = whi / wlo;
    return fmin(nn * r * sqrt(diam2), nn * r * r * sqrt(leg2));
}

struct CpCount {
    uint32_t split = 0, leaf = 0, maxk = 0;
    uint32_t trips = 0, busy = 0;  // loop trips of the wave (lane 0), trips holding a pair (every lane)
};

struct CpState {
    Piece P;
    double B, eta;
    double a, ax, ay, bx, by;
    uint64_t pend;
    int k, n, pmax, deg;
    bool rat;
    uint32_t seg;
};

// The piece of [a, a + 2^-k]: halvings from the segment's control points
// along the binary digits of a (digit j of a picks the half at level j).
__device__ __forceinline__ void derive_piece(CpState& st, const Segs& sg, double qx, double qy) {
    root_piece(sg, st.seg, st.deg, qx, qy, st.P);
    Piece L;
    double t = st.a;
    for (int j = 1; j <= st.k; ++j) {
        halve(st.P, L, st.deg);
        t *= 2.0;
        const bool right = t >= 1.0;
        t -= right ? 1.0 : 0.0;
        if (!right) st.P = L;
    }
}

template <bool COUNT>
__device__ __forceinline__ bool cp_step(CpState& st, double eps2, bool& onb, CpCount& nc, const Segs& sg,
                                        double qx, double qy, bool has) {
    const bool capped = has & (st.k >= kDepthCap);
    const int k1 = st.k + 1;
    const double tm = st.a + ldexp(1.0, -k1);
    Piece L;
    double mx = 0.0, my = 0.0, Bl = 0.0, Br = 0.0;
    if (has & !capped) {
        halve(st.P, L, st.deg);  // st.P: right half, L: left half
        const double r = recip(slot(L.W, st.deg));
        mx = slot(L.X, st.deg) * r;
        my = slot(L.Y, st.deg) * r;
        Bl = piece_bound(L, st.deg, st.rat);
        Br = piece_bound(st.P, st.deg, st.rat);
    }
    const double rm = fma(mx, mx, my * my);
    const double ra = fma(st.ax, st.ax, st.ay * st.ay);
    const double rb = fma(st.bx, st.bx, st.by * st.by);
    const bool hit = has & !capped & (rm < eps2);
    onb |= capped | hit;
    bool fin = capped | hit;
    const bool go = has & !capped & !hit;
    const double Bk = ldexp(st.B, -k1);
    const double El = fma(fmin(Bk, Bl), 1.0 + kAxisInflate, st.eta);
    const double Er = fma(fmin(Bk, Br), 1.0 + kAxisInflate, st.eta);
    const bool lfar = outside_ellipse(ra, rm, 0.5 * El * El);
    const bool rfar = outside_ellipse(rm, rb, 0.5 * Er * Er);
    {
        const uint64_t gm = __builtin_amdgcn_ballot_w64(go);
        const uint64_t am = low_mask(st.ay), mm = low_mask(my), bm = low_mask(st.by);
        ray_cross_mask(st.n, am, mm, st.ax, st.ay, mx, my, gm & __builtin_amdgcn_ballot_w64(lfar));
        ray_cross_mask(st.n, mm, bm, mx, my, st.bx, st.by, gm & __builtin_amdgcn_ballot_w64(rfar));
    }
    if (COUNT && go) {
        ++nc.split;
        nc.leaf += (lfar ? 1 : 0) + (rfar ? 1 : 0);
        nc.maxk = (uint32_t)k1 > nc.maxk ? (uint32_t)k1 : nc.maxk;
    }
    const bool both = go & !lfar & !rfar;
    const bool left = go & !lfar;
    const bool right = go & lfar & !rfar;
    const bool none = go & lfar & rfar;
    st.pend = both ? (st.pend | (1ull << k1)) : st.pend;
    st.pmax = (go & (k1 > st.pmax)) ? k1 : st.pmax;
    fin |= none & (st.pend == 0);
    const bool pop = none & (st.pend != 0);
    // continue left: the left half's control points; right: st.P already
#pragma unroll
    for (int i = 0; i < kCoef; ++i) {
        st.P.X[i] = left ? L.X[i] : st.P.X[i];
        st.P.Y[i] = left ? L.Y[i] : st.P.Y[i];
        st.P.W[i] = left ? L.W[i] : st.P.W[i];
    }
    st.ax = right ? mx : st.ax;
    st.ay = right ? my : st.ay;
    st.bx = left ? mx : st.bx;
    st.by = left ? my : st.by;
    st.a = right ? tm : st.a;
    st.k = (left | right) ? k1 : st.k;
    if (pop) {
        const int kk = 63 - __clzll(st.pend);
        st.pend &= ~(1ull << kk);
        st.a = deferred_left(st.a, kk);
        st.k = kk;
        derive_piece(st, sg, qx, qy);
        const double ra_ = recip(st.P.W[0]);
        st.ax = st.P.X[0] * ra_;
        st.ay = st.P.Y[0] * ra_;
        if (st.a + ldexp(1.0, -kk) == 1.0) {
            const double2 e = seg_end_point(sg, (int)st.seg);
            st.bx = e.x - qx;
            st.by = e.y - qy;
        } else {
            const double rb_ = recip(slot(st.P.W, st.deg));
            st.bx = slot(st.P.X, st.deg) * rb_;
            st.by = slot(st.P.Y, st.deg) * rb_;
        }
    }
    return fin;
}

template <bool COUNT>
__global__ __launch_bounds__(kWG) void k_near_cp(Segs sg, Points pts, NearQueue nq, Out out, double eps2,
                                                 Stats stats, const uint8_t* seg_per, uint8_t* entry_depth,
                                                 const unsigned long long* q_lo, const unsigned long long* q_hi,
                                                 unsigned long long* cursor) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    unsigned long long n = q_hi ? *q_hi : *nq.count;
    n = n < nq.cap ? n : nq.cap;
    unsigned long long base = q_lo ? *q_lo : 0ull;
    base = base < n ? base : n;
    const unsigned long long gw = (unsigned long long)blockIdx.x * kWavesPerWG + wave;
    unsigned long long next = 0, c_end = 0;
    bool more = true, shared_once = false;
    CpState st;
    bool onb = false, has = false;
    uint32_t q = 0;
    double qx = 0.0, qy = 0.0;
    unsigned long long cur = 0;
    CpCount nc;
    auto grab = [&]() {
        if (cursor) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(cursor, 512ull);
            c = __shfl(c, 0);
            next = base + c < n ? base + c : n;
            c_end = next + 512 < n ? next + 512 : n;
        } else if (!shared_once) {
            const unsigned long long nw = (unsigned long long)gridDim.x * kWavesPerWG;
            const unsigned long long per = (n - base + nw - 1) / nw;
            next = base + gw * per < n ? base + gw * per : n;
            c_end = next + per < n ? next + per : n;
            shared_once = true;
        } else {
            next = c_end = n;
        }
        more = next < c_end;
    };
    grab();
    for (;;) {
        const uint64_t idle = __ballot(!has);
        if (idle && more && (__popcll(idle) >= kRefillMin || idle == ~0ull)) {
            if (next >= c_end) grab();
            if (more) {
                const int rank = lanes_below(idle);
                if (!has && next + rank < c_end) {
                    const uint2 e = nq.qs[next + rank];
                    q = e.x;
                    cur = next + rank;
                    if ((int64_t)q < pts.n) {
                        qx = pts.u[(int64_t)q * pts.stride];
                        qy = pts.v[(int64_t)q * pts.stride];
                        if (nq.shift && seg_per[e.y]) {  // periodic copy: translate the query (App. C.1)
                            const double2 sh = nq.shift[next + rank];
                            qx -= sh.x;
                            qy -= sh.y;
                        }
                        Coef c;
                        NearSeg g;
                        load_near_seg(sg, e.y, c, g);
                        st.seg = e.y;
                        st.deg = c.n;
                        st.rat = c.rat;
                        st.B = g.B;
                        st.eta = g.eta;
                        st.ax = g.p0x - qx;
                        st.ay = g.p0y - qy;
                        st.bx = g.pnx - qx;
                        st.by = g.pny - qy;
                        st.n = -ray_cross(st.ax, st.ay, st.bx, st.by);
                        st.a = 0.0;
                        st.k = 0;
                        st.pend = 0;
                        st.pmax = 0;
                        root_piece(sg, e.y, st.deg, qx, qy, st.P);
                        onb = false;
                        has = true;
                    }
                }
                const unsigned long long took = (unsigned long long)__popcll(idle);
                next = next + took < c_end ? next + took : c_end;
            }
        }
        if (!__any(has)) {
            if (!more) break;
            continue;
        }
        if (COUNT) {
            nc.trips += lane == 0 ? 1u : 0u;
            nc.busy += has ? 1u : 0u;
        }
        if (cp_step<COUNT>(st, eps2, onb, nc, sg, qx, qy, has)) {
            if (onb) out.lab[q] = 2;
            else if (st.n != 0) unsafeAtomicAdd(&out.w[q], kTwoPi * (double)st.n);
            if (COUNT && entry_depth) entry_depth[cur] = (uint8_t)(st.pmax < 255 ? st.pmax : 255);
            has = false;
        }
    }
    if (COUNT && stats.c) {
        unsigned long long sp = nc.split, lf = nc.leaf, tr = nc.trips, bu = nc.busy;
        uint32_t mk = nc.maxk;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sp += __shfl_xor(sp, off);
            lf += __shfl_xor(lf, off);
            tr += __shfl_xor(tr, off);
            bu += __shfl_xor(bu, off);
            const uint32_t o = __shfl_xor(mk, off);
            mk = o > mk ? o : mk;
        }
        if (lane == 0) {
            atomicAdd(&stats.c[6], tr);
            atomicAdd(&stats.c[7], bu);
            if (gw == 0) atomicAdd(&stats.c[0], n);
            atomicAdd(&stats.c[1], sp);
            atomicAdd(&stats.c[2], lf);
            atomicMax(&stats.c[5], (unsigned long long)mk);
        }
    }
}

}  // namespace

int near_cp_blocks_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_near_cp<false>, kWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_near_cp(const Segs& sg, const Points& pts, NearQueue nq, Out out, double eps2, int64_t grid,
                          Stats stats, const uint8_t* seg_per, uint8_t* entry_depth, hipStream_t st,
                          const unsigned long long* q_lo, const unsigned long long* q_hi, unsigned long long* cursor) {
    if (grid <= 0) return hipSuccess;
    if (stats.c || entry_depth)
        hipLaunchKernelGGL(k_near_cp<true>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, pts, nq, out, eps2, stats,
                           seg_per, entry_depth, q_lo, q_hi, cursor);
    else
        hipLaunchKernelGGL(k_near_cp<false>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, pts, nq, out, eps2, stats,
                           seg_per, entry_depth, q_lo, q_hi, cursor);
    return hipGetLastError();
}

}  // namespace wn
