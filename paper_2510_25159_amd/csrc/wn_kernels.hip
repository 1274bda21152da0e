// HIP kernels (gfx950) of the winding-number containment library.
//
// Method (Alg. 1, Sec. 4.1-4.2): for every (query x, segment gamma) pair,
//   - if an evaluated curve point is within eps of x: on-boundary;
//   - else if x is outside the ellipse d(x, gamma(a)) + d(x, gamma(b)) <= B (b - a)
//     (Lemma 1, Eq. of the sub-segment bound): the sub-segment sweeps the
//     angle of its chord (Sec. 3.2 eqs. 2-3);
//   - else split at the midpoint and recurse.
// omega(x) = (sum of angles) / 2pi over all segments of the face (additivity,
// Sec. 3.2 eq. 1), rounded to a label (Sec. 4.1).
//
// gfx950 realisation.
//  * Far field: one lane per query, segments streamed through an LDS tile
//    (uniform-address LDS reads broadcast to the wave).  The ellipse test is
//    evaluated without square roots:  d1 + d2 > Bk  <=>  R < 0 or r1 r2 > R^2
//    with R = Bk^2/2 - (r1 + r2)/2, ri = di^2.
//  * Angle sums without an atan2 per pair.  For a closed polygon that avoids
//    x, the principal angles of its edges sum to 2 pi times its signed
//    crossings with the ray {x + (s, 0): s > 0}.  A chain of segments that
//    join bit for bit therefore sums to the angle from its start to its end
//    plus 2 pi (crossings of its chords and of the closing edge): a far pair
//    costs one crossing test, and a closed loop contributes an exact integer.
//    The few remaining angle factors (chain closures, periodic copies) go to
//    a complex accumulator z = prod (dot + i cross) with an integer K of
//    completed turns, sum(theta) = arg(z) + 2 pi K (sign rule on the
//    imaginary parts, see turn_mul): one atan2 per query.
//  * Near pairs: Alg. 1 with an explicit stack; each step halves the current
//    interval and tests both halves, so a pair costs one step per split
//    node.  The result is an integer correction N to the segment chord's
//    angle (leaves' crossings minus the chord's), added only when N != 0.
//    Deferred intervals sit in an LDS ring of kNearSlots slots per lane; one
//    whose slot was reused is evaluated again (same parameters => the same
//    values).
//  * Curve points: one Horner pass in u = t / (1 - t) over zero-padded
//    coefficient slots (no degree-dependent branch), then one reciprocal.
#include "wn_device.h"

namespace wn {

// Append this wave's buffered near pairs to the global queue with one atomic.
// Returns true for the lanes whose query lost a pair to a full queue (those
// queries are recomputed in line by k_redo).
__device__ __forceinline__ bool flush_near(const uint2* buf, int nfill, const NearQueue& nq, int lane, int64_t qi) {
    if (nfill == 0) return false;
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(nq.count, (unsigned long long)nfill);
    base = __shfl(base, 0);
    for (int e = lane; e < nfill; e += kWave)
        if (base + (unsigned long long)e < nq.cap) nq.qs[base + e] = buf[e];
    bool lost = false;
    if (base + (unsigned long long)nfill > nq.cap) {
        for (int e = 0; e < nfill; ++e)
            if (base + (unsigned long long)e >= nq.cap && (int64_t)buf[e].x == qi) lost = true;
    }
    __builtin_amdgcn_wave_barrier();
    return lost;
}


// ---------------------------------------------------------------------------
// work items: (face, tile of QPW queries), faces in descending segment count
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_build_items(FaceTab ft, Points pts, int qpw, int32_t* item_offs,
                                                      int2* item_map, int64_t map_cap, uint32_t* counters,
                                                      int zero_near) {
    __shared__ int64_t s_sum[1024];
    const int tid = threadIdx.x;
    const int F = ft.num_faces;
    const int chunk = (F + 1023) / 1024;
    const int r0 = min(F, tid * chunk), r1 = min(F, r0 + chunk);
    // [0] far item counter, [1] periodic redo item counter, [2..3] near-queue
    // count (64-bit), [8..15] item counters of the phases of an overlapped far
    // pass, [16..23] queue marks of those phases, [24..31] chunk cursors of up
    // to four near passes (64-bit).  The near count and the cursors are reset
    // by the first build of a query only.
    if (tid < 2 || (tid >= 8 && tid < 16)) counters[tid] = 0;
    if (zero_near && (tid == 2 || tid == 3 || (tid >= 24 && tid < 32))) counters[tid] = 0;
    auto tiles_of = [&](int r) -> int64_t {
        const int f = ft.order[r];
        int64_t qb = pts.offs[f], qe = pts.offs[f + 1];
        qb = qb < 0 ? 0 : (qb > pts.n ? pts.n : qb);
        qe = qe < qb ? qb : (qe > pts.n ? pts.n : qe);
        return (qe - qb + qpw - 1) / qpw;
    };
    int64_t local = 0;
    for (int r = r0; r < r1; ++r) local += tiles_of(r);
    s_sum[tid] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? s_sum[tid - off] : 0;
        __syncthreads();
        s_sum[tid] += v;
        __syncthreads();
    }
    int64_t base = s_sum[tid] - local;
    for (int r = r0; r < r1; ++r) {
        item_offs[r] = (int32_t)(base < map_cap ? base : map_cap);
        base += tiles_of(r);
    }
    const int64_t total = s_sum[1023] < map_cap ? s_sum[1023] : map_cap;
    if (tid == 1023) item_offs[F] = (int32_t)total;
    __syncthreads();
    // item i -> (face, tile): last r with item_offs[r] <= i
    for (int64_t i = tid; i < total; i += 1024) {
        int lo = 0, hi = F - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_offs[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        item_map[i] = make_int2(ft.order[lo], (int)(i - item_offs[lo]));
    }
}

// ---------------------------------------------------------------------------
// far-field kernel.  GQ query groups of 64 per workgroup, GS = 4 / GQ waves
// share one query group and split its segments.
//   INLINE: near pairs recursed in place; writes final omega and labels.
//   !INLINE: near pairs appended to the near queue (in place on overflow);
//            writes the angle sum and on-boundary flags for k_near/k_finalize.
// Item source: item_counter != nullptr -> persistent loop popping items;
// else item = blockIdx.x.  single_face >= 0 -> items are the tiles of that face.
// ---------------------------------------------------------------------------
template <bool INLINE, int GQ, bool MIXED>
__global__ __launch_bounds__(kWG) void k_far(Segs sg, FaceTab ft, Points pts, const int32_t* item_offs,
                                             const int2* item_map, uint32_t* item_counter, int32_t single_face,
                                             NearQueue nq, Out out, double eps2) {
    constexpr int GS = kWavesPerWG / GQ;
    constexpr int QPW = kWave * GQ;
    __shared__ double s_p0x[kSegChunk], s_p0y[kSegChunk], s_pnx[kSegChunk], s_pny[kSegChunk], s_hb2[kSegChunk];
    __shared__ uint8_t s_join[kSegChunk];
    __shared__ float s_bef[MIXED ? kSegChunk : 1];  // FP32 upper bound of the root ellipse's axis
    __shared__ double4 s_stack[INLINE ? kWavesPerWG * kNearSlots * kWave : 1];
    __shared__ double s_ang[kWavesPerWG][kWave];
    __shared__ int s_flag[kWavesPerWG][kWave];
    __shared__ uint2 s_nbuf[INLINE ? 1 : kWavesPerWG][INLINE ? 1 : kNearBufT];
    __shared__ int s_item;

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    const int gq = wave / GS, gs = wave % GS;
    double4* stk = INLINE ? s_stack + wave * kNearSlots * kWave + lane : s_stack;
    const int total = single_face >= 0 ? (int)gridDim.x : item_offs[ft.num_faces];

    for (int iter = 0;; ++iter) {
        int item;
        if (item_counter) {
            __syncthreads();
            if (tid == 0) s_item = (int)atomicAdd(item_counter, 1u);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);  // uniform: face data via scalar loads
        } else {
            if (iter > 0) break;
            item = blockIdx.x;
        }
        if (item >= total) break;
        int f, tile;
        if (single_face >= 0) {
            f = single_face;
            tile = item;
        } else {
            const int2 m = item_map[item];
            f = m.x;
            tile = m.y;
        }
        int64_t qb = pts.offs[f], qe = pts.offs[f + 1];
        qb = qb < 0 ? 0 : (qb > pts.n ? pts.n : qb);
        qe = qe < qb ? qb : (qe > pts.n ? pts.n : qe);
        const int64_t qi = qb + (int64_t)tile * QPW + gq * kWave + lane;
        const bool active = qi < qe;
        double qx = 0.0, qy = 0.0;
        if (active) {
            qx = pts.u[qi * pts.stride];
            qy = pts.v[qi * pts.stride];
        }
        const bool valid = active && fabs(qx) < kCoordLimit && fabs(qy) < kCoordLimit;
        if (!valid) qx = qy = 0.0;
        Turn T{1.0, 0.0, 0};
        int xc = 0;  // integer part of in-line near pairs (2 pi units)
        bool onb = false;
        const int s0 = ft.seg_begin[f], s1 = ft.seg_begin[f + 1];
        int nfill = 0;      // entries in this wave's near-pair buffer (wave-uniform)
        // a near pair of this lane's query did not fit in the queue (an int, not
        // a bool: lane masks updated inside divergent code cost scalar merges)
        int lost = 0;
        // Chains: runs of consecutive segments of this wave in which each
        // segment starts where the previous one ended (bit for bit).  A
        // chain's chord angles sum to the angle from its start to its end
        // plus 2 pi times the ray crossings of its chords and of the closing
        // edge, so a pair costs a crossing test instead of an angle factor;
        // near pairs keep their chord in the chain and get the integer rest
        // from the recursion.
        double csx = 0.0, csy = 0.0;             // start of the open chain, relative to the query
        double pbx = 0.0, pby = 0.0, prb = 0.0;  // end of the previous segment, relative
        bool pb_low = false;                     // pby <= 0 (below or on the ray's line)
        float pdf = 0.f;                         // |pb| in FP32 (precision MIXED)
        bool open = false;                       // wave-uniform
        const uint64_t vm = __builtin_amdgcn_ballot_w64(valid);
        double rmin = INFINITY;                  // smallest |b|^2 of the two-segment path
        for (int c0 = s0; c0 < s1; c0 += kSegChunk) {
            __syncthreads();
            const int sj = c0 + tid;
            if (sj < s1) {
                s_p0x[tid] = sg.p0x[sj];
                s_p0y[tid] = sg.p0y[sj];
                s_pnx[tid] = sg.pnx[sj];
                s_pny[tid] = sg.pny[sj];
                s_hb2[tid] = sg.hb2[sj];
                s_join[tid] = sg.join[sj];
                if constexpr (MIXED) s_bef[tid] = __double2float_ru(sqrt(2.0 * s_hb2[tid]));
            }
            __syncthreads();
            const int cn = min(kSegChunk, s1 - c0);
            // GS waves split the chunk into contiguous ranges
            const int jb = (cn * gs) / GS, je = (cn * (gs + 1)) / GS;
            for (int j0 = jb; j0 < je; j0 += kWave) {
                const int jn = __builtin_amdgcn_readfirstlane(min(kWave, je - j0));
                // bit i: segment j0 + i starts where segment j0 + i - 1 ended
                const uint64_t jm = __ballot(lane < jn && s_join[j0 + lane] != 0);
                int jj = 0;
                while (jj < jn) {
                    if (!(open & ((jm >> jj) & 1ull))) {  // a chain starts at segment j0 + jj
                        if (open) close_chain(T, xc, csx, csy, pbx, pby);
                        pbx = s_p0x[j0 + jj] - qx;
                        pby = s_p0y[j0 + jj] - qy;
                        prb = pbx * pbx + pby * pby;
                        onb |= valid & (prb < eps2);
                        pb_low = pby <= 0.0;
                        if constexpr (MIXED) pdf = sqrtf(fmaf((float)pbx, (float)pbx, (float)pby * (float)pby));
                        csx = pbx;
                        csy = pby;
                        open = true;
                    }
                    // the run jj .. re - 1 continues the chain without a break
                    const uint64_t brk = jj + 1 < 64 ? ~(jm >> (jj + 1)) : ~0ull;
                    const int re = min(jn, jj + 1 + (int)__builtin_ctzll(brk | (1ull << 63)));
                    if constexpr (!INLINE && !MIXED) {
                        // two segments per trip: their arithmetic is independent apart
                        // from the shared end point, which gives each wave two chains
                        // of dependent instructions to interleave.  Flags live as lane
                        // masks (SGPRs): a comparison writes its mask directly, and a
                        // pair's orientation is only computed when some lane's chord
                        // changes side of the ray's line.  End points closer than eps
                        // are collected in rmin and reported after the face.
                        auto append = [&](uint64_t m, int j) {
                            if (m) {
                                const int cntm = __popcll(m);
                                if (nfill + cntm > kNearBufT) {
                                    lost |= flush_near(s_nbuf[wave], nfill, nq, lane, qi) ? 1 : 0;
                                    nfill = 0;
                                }
                                if (__builtin_amdgcn_inverse_ballot_w64(m))
                                    s_nbuf[wave][nfill + lanes_below(m)] = make_uint2((uint32_t)qi, (uint32_t)(c0 + j));
                                nfill += cntm;
                            }
                        };
                        uint64_t am = __builtin_amdgcn_ballot_w64(pb_low);
                        for (; jj + 1 < re; jj += 2) {
                            const int j = j0 + jj;
                            const double bx0 = s_pnx[j] - qx, by0 = s_pny[j] - qy;
                            const double bx1 = s_pnx[j + 1] - qx, by1 = s_pny[j + 1] - qy;
                            const double rb0 = bx0 * bx0 + by0 * by0, rb1 = bx1 * bx1 + by1 * by1;
                            rmin = fmin(rmin, fmin(rb0, rb1));
                            const uint64_t b0m = low_mask(by0), b1m = low_mask(by1);
                            ray_cross_mask(xc, am, b0m, pbx, pby, bx0, by0);
                            ray_cross_mask(xc, b0m, b1m, bx0, by0, bx1, by1);
                            const uint64_t n0 = near_mask(prb, rb0, s_hb2[j]) & vm;
                            const uint64_t n1 = near_mask(rb0, rb1, s_hb2[j + 1]) & vm;
                            pbx = bx1;
                            pby = by1;
                            prb = rb1;
                            am = b1m;
                            append(n0, j);
                            append(n1, j + 1);
                        }
                        pb_low = __builtin_amdgcn_inverse_ballot_w64(am);
                    }
                    for (; jj < re; ++jj) {
                        const int j = j0 + jj;
                        const double cpx = s_pnx[j], cpy = s_pny[j], chb = s_hb2[j];
                        // a = the previous segment's end point (already tested against eps);
                        // flags combine with & and | (no short circuit, no branch)
                        const double ax = pbx, ay = pby, ra = prb;
                        const bool a_low = pb_low;
                        const double bx = cpx - qx, by = cpy - qy;
                        const double rb = bx * bx + by * by;
                        onb |= valid & (rb < eps2);
                        const bool b_low = by <= 0.0;
                        xc += ray_cross_n(a_low, b_low, cross_neg_wave(ax, ay, bx, by));  // = ray_cross(a, b)
                        pbx = bx;
                        pby = by;
                        prb = rb;
                        pb_low = b_low;
                        bool near;
                        if constexpr (MIXED) {
                            // FP32 admission: d1 + d2 beyond the axis by a relative 2^-20
                            // margin (far above the FP32 rounding of the two distances)
                            // proves the pair far; the FP64 test runs only when some lane
                            // is not admitted
                            const float bxf = (float)bx, byf = (float)by;
                            const float d2f = sqrtf(fmaf(bxf, bxf, byf * byf));
                            const bool admit = (pdf + d2f) * (1.0f - kMixedMargin) > s_bef[j] * (1.0f + kMixedMargin);
                            pdf = d2f;
                            near = false;
                            if (__ballot(!admit) != 0ull) near = !admit & !outside_ellipse(ra, rb, chb);
                        } else {
                            near = !outside_ellipse(ra, rb, chb);
                        }
                        bool need = valid & !onb & near;
                        int depth = 0;
                        if constexpr (!INLINE) {
                            const uint64_t m = __builtin_amdgcn_ballot_w64(need);
                            if (m) {
                                const int cntm = __popcll(m);
                                if (nfill + cntm > kNearBufT) {
                                    lost |= flush_near(s_nbuf[wave], nfill, nq, lane, qi) ? 1 : 0;
                                    nfill = 0;
                                }
                                const int rank = __popcll(m & ((1ull << lane) - 1ull));
                                if (need) {
                                    s_nbuf[wave][nfill + rank] = make_uint2((uint32_t)qi, (uint32_t)(c0 + j));
                                    need = false;
                                }
                                nfill += cntm;
                            }
                        }
                        if (INLINE && need) {
                            const int s = c0 + j;
                            Coef c;
                            load_coef(sg, s, c);
                            depth = near_pair(xc, c, sg.B[s], sg.eta[s], cpx, cpy, qx, qy, ax, ay, ra, bx, by, rb,
                                              eps2, stk, onb);
                        }
                        if (INLINE && out.depth && active)
                            out.depth[qi * (int64_t)out.depth_stride + (c0 + j - s0)] = (uint8_t)depth;
                    }
                }
            }
            if (GS > 1 && open) {  // this wave's next range is not adjacent
                close_chain(T, xc, csx, csy, pbx, pby);
                open = false;
            }
        }
        if (open) close_chain(T, xc, csx, csy, pbx, pby);
        onb |= valid & (rmin < eps2);
        if constexpr (!INLINE) lost |= flush_near(s_nbuf[wave], nfill, nq, lane, qi) ? 1 : 0;
        // combine the GS partial sums of each query group
        double ang = turn_angle(T) + kTwoPi * (double)xc;
        if constexpr (GS > 1) {
            s_ang[wave][lane] = ang;
            s_flag[wave][lane] = (onb ? 1 : 0) | (lost ? 2 : 0);
            __syncthreads();
            if (gs == 0) {
#pragma unroll
                for (int g = 1; g < GS; ++g) {
                    ang += s_ang[wave + g][lane];
                    onb = onb || (s_flag[wave + g][lane] & 1);
                    lost |= (s_flag[wave + g][lane] & 2) ? 1 : 0;
                }
            }
        }
        if (gs == 0 && active) {
            if constexpr (INLINE) {
                double w;
                uint8_t lab;
                if (!valid) {
                    w = __builtin_nan("");
                    lab = 3;
                } else if (onb) {
                    w = __builtin_nan("");
                    lab = 2;
                } else {
                    w = ang / kTwoPi;
                    lab = classify(w, out.rule);
                }
                if (out.w) out.w[qi] = w;
                if (out.lab) out.lab[qi] = lab;
            } else {
                out.w[qi] = ang;
                out.lab[qi] = !valid ? 3 : (onb ? 2 : (lost ? kRedo : 0));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Far-field kernel of the queued FP64 schedules with QPL queries per lane:
// each wave evaluates 64 QPL queries, so one LDS read of a segment feeds QPL
// pairs and every lane carries QPL independent dependency chains.  Same
// arithmetic and outputs as k_far<false, GQ, false>; flags live as lane
// masks (SGPRs) and the orientation of a pair is only computed when some
// lane's chord changes side of the ray's line.
// ---------------------------------------------------------------------------
// flush_near for QPL queries per lane (query q of the lane: qi0 + q kWave):
// bit q of lost is set when a pair of query q did not fit in the queue.
// Coordinates given to the inactive and invalid queries of the far passes
// that carry no validity masks (far beyond kCoordLimit, so that their
// squared distances overflow to +inf: outside every ellipse, within eps of no
// end point, crossing no chord).
constexpr double kAway = 1e300;

// A wave-uniform double held in scalar registers (lane 0's value).
__device__ __forceinline__ double uniform_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int QPL>
__device__ __forceinline__ void flush_near_q(const uint2* buf, int nfill, const NearQueue& nq, int lane, int64_t qi0,
                                             int& lost) {
    if (nfill == 0) return;
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(nq.count, (unsigned long long)nfill);
    base = __shfl(base, 0);
    for (int e = lane; e < nfill; e += kWave)
        if (base + (unsigned long long)e < nq.cap) nq.qs[base + e] = buf[e];
    if (base + (unsigned long long)nfill > nq.cap) {
        for (int e = 0; e < nfill; ++e) {
            if (base + (unsigned long long)e < nq.cap) continue;
            const int64_t x = (int64_t)buf[e].x;
#pragma unroll
            for (int q = 0; q < QPL; ++q) lost |= x == qi0 + (int64_t)q * kWave ? 1 << q : 0;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// occupancy target of k_farq: the register budget that keeps it (four
// queries per lane: 128 VGPRs, with two spilled, for 4 waves per SIMD; the
// near-pair buffers are sized so that four workgroups fit in LDS)
template <int QPL>
struct FarqWaves;
template <>
struct FarqWaves<2> {
    static constexpr int w = 5;
};
template <>
struct FarqWaves<3> {
    static constexpr int w = 4;
};
template <>
struct FarqWaves<4> {
    static constexpr int w = 4;
};

template <int QPL>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(FarqWaves<QPL>::w))) void k_farq(
    Segs sg, FaceTab ft, Points pts, const int32_t* item_offs, const int2* item_map, uint32_t* item_counter,
    NearQueue nq, Out out, double eps2, int rank_lo, int rank_hi) {
    constexpr int kQPL = QPL;
    constexpr int kQPWG2 = kWave * QPL * kWavesPerWG;  // queries per work item
    __shared__ double s_p0x[kSegChunk], s_p0y[kSegChunk], s_pnx[kSegChunk], s_pny[kSegChunk], s_hb2[kSegChunk];
    __shared__ uint8_t s_join[kSegChunk];
    __shared__ uint2 s_nbuf[kWavesPerWG][kNearBufQ];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    // items of the faces of rank [rank_lo, rank_hi)
    const int lo = item_offs[rank_lo], total = item_offs[rank_hi];
    for (int iter = 0;; ++iter) {
        int item;
        if (item_counter) {
            __syncthreads();
            if (tid == 0) s_item = lo + (int)atomicAdd(item_counter, 1u);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
        } else {
            if (iter > 0) break;
            item = lo + blockIdx.x;
        }
        if (item >= total) break;
        const int2 mp = item_map[item];
        const int f = mp.x, tile = mp.y;
        int64_t qb = pts.offs[f], qe = pts.offs[f + 1];
        qb = qb < 0 ? 0 : (qb > pts.n ? pts.n : qb);
        qe = qe < qb ? qb : (qe > pts.n ? pts.n : qe);
        // query q of this lane: qi0 + q kWave
        const int64_t qi0 = qb + (int64_t)tile * kQPWG2 + (int64_t)wave * kQPL * kWave + lane;
        double qx[kQPL], qy[kQPL];
        Turn T[kQPL];
        int xc[kQPL];
        int lost = 0;                    // bit q: a near pair of query q did not fit in the queue
        uint64_t em[kQPL], am[kQPL];     // eps hits, chain end below the ray's line
        double pbx[kQPL], pby[kQPL], prb[kQPL];
        double chx = 0.0, chy = 0.0;     // the open chain's start point (wave-uniform)
#pragma unroll
        for (int q = 0; q < kQPL; ++q) {
            const int64_t qi = qi0 + (int64_t)q * kWave;
            qx[q] = qy[q] = 0.0;
            if (qi < qe) {
                qx[q] = pts.u[qi * pts.stride];
                qy[q] = pts.v[qi * pts.stride];
            }
            // an inactive or invalid query sits at (kAway, kAway): no mask needed
            if (!(qi < qe && fabs(qx[q]) < kCoordLimit && fabs(qy[q]) < kCoordLimit)) qx[q] = qy[q] = kAway;
            T[q] = Turn{1.0, 0.0, 0};
            xc[q] = 0;
            em[q] = am[q] = 0;
            pbx[q] = pby[q] = prb[q] = 0.0;
        }
        const int s0 = ft.seg_begin[f], s1 = ft.seg_begin[f + 1];
        int nfill = 0;      // entries in this wave's near-pair buffer (wave-uniform)
        bool open = false;  // a chain is open (wave-uniform)
        for (int c0 = s0; c0 < s1; c0 += kSegChunk) {
            __syncthreads();
            const int sj = c0 + tid;
            if (sj < s1) {
                s_p0x[tid] = sg.p0x[sj];
                s_p0y[tid] = sg.p0y[sj];
                s_pnx[tid] = sg.pnx[sj];
                s_pny[tid] = sg.pny[sj];
                s_hb2[tid] = sg.hb2[sj];
                s_join[tid] = sg.join[sj];
            }
            __syncthreads();
            const int cn = min(kSegChunk, s1 - c0);
            for (int j0 = 0; j0 < cn; j0 += kWave) {
                const int jn = __builtin_amdgcn_readfirstlane(min(kWave, cn - j0));
                const uint64_t jm = __ballot(lane < jn && s_join[j0 + lane] != 0);
                int jj = 0;
                while (jj < jn) {
                    if (!(open & ((jm >> jj) & 1ull))) {  // a chain starts at segment j0 + jj
#pragma unroll
                        for (int q = 0; q < kQPL; ++q)
                            if (open) close_chain(T[q], xc[q], chx - qx[q], chy - qy[q], pbx[q], pby[q]);
                        chx = uniform_f64(s_p0x[j0 + jj]);
                        chy = uniform_f64(s_p0y[j0 + jj]);
#pragma unroll
                        for (int q = 0; q < kQPL; ++q) {
                            pbx[q] = chx - qx[q];
                            pby[q] = chy - qy[q];
                            prb[q] = pbx[q] * pbx[q] + pby[q] * pby[q];
                            em[q] |= __builtin_amdgcn_fcmp(prb[q], eps2, kCmpOLT);
                            am[q] = low_mask(pby[q]);
                        }
                        open = true;
                    }
                    // the run jj .. re - 1 continues the chain without a break
                    const uint64_t brk = jj + 1 < 64 ? ~(jm >> (jj + 1)) : ~0ull;
                    const int re = min(jn, jj + 1 + (int)__builtin_ctzll(brk | (1ull << 63)));
                    auto step = [&](int j, double px, double py, double hb) {
                        uint64_t nm[kQPL];
#pragma unroll
                        for (int q = 0; q < kQPL; ++q) {
                            const double bx = px - qx[q], by = py - qy[q];
                            const double rb = bx * bx + by * by;
                            em[q] |= __builtin_amdgcn_fcmp(rb, eps2, kCmpOLT);
                            const uint64_t bm = low_mask(by);
                            ray_cross_mask(xc[q], am[q], bm, pbx[q], pby[q], bx, by);
                            nm[q] = near_mask(prb[q], rb, hb);
                            pbx[q] = bx;
                            pby[q] = by;
                            prb[q] = rb;
                            am[q] = bm;
                        }
                        uint64_t any = 0;
#pragma unroll
                        for (int q = 0; q < kQPL; ++q) any |= nm[q];
                        if (any != 0ull) {
                            int cnt = 0;
#pragma unroll
                            for (int q = 0; q < kQPL; ++q) cnt += __popcll(nm[q]);
                            if (nfill + cnt > kNearBufQ) {
                                flush_near_q<kQPL>(s_nbuf[wave], nfill, nq, lane, qi0, lost);
                                nfill = 0;
                            }
                            const uint32_t seg = (uint32_t)(c0 + j);
#pragma unroll
                            for (int q = 0; q < kQPL; ++q) {
                                if (__builtin_amdgcn_inverse_ballot_w64(nm[q]))
                                    s_nbuf[wave][nfill + lanes_below(nm[q])] =
                                        make_uint2((uint32_t)(qi0 + (int64_t)q * kWave), seg);
                                nfill += __popcll(nm[q]);
                            }
                        }
                    };
                    for (; jj + 1 < re; jj += 2) {  // two segments per trip: no register copies between them
                        const int j = j0 + jj;
                        step(j, s_pnx[j], s_pny[j], s_hb2[j]);
                        step(j + 1, s_pnx[j + 1], s_pny[j + 1], s_hb2[j + 1]);
                    }
                    if (jj < re) {
                        const int j = j0 + jj++;
                        step(j, s_pnx[j], s_pny[j], s_hb2[j]);
                    }
                }
            }
        }
        flush_near_q<kQPL>(s_nbuf[wave], nfill, nq, lane, qi0, lost);
#pragma unroll
        for (int q = 0; q < kQPL; ++q) {
            if (open) close_chain(T[q], xc[q], chx - qx[q], chy - qy[q], pbx[q], pby[q]);
            const int64_t qi = qi0 + (int64_t)q * kWave;
            const bool valid = qx[q] != kAway;
            const bool onb = valid & __builtin_amdgcn_inverse_ballot_w64(em[q]);
            if (qi < qe) {
                out.w[qi] = turn_angle(T[q]) + kTwoPi * (double)xc[q];
                out.lab[qi] = !valid ? 3 : (onb ? 2 : (((lost >> q) & 1) ? kRedo : 0));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Far-field kernel over the path hierarchy (queued FP64 schedules): one query
// per lane, each lane walking its face's subpath trees in preorder with a
// skip index (no stack).  At a node the query either descends (inside the
// node's ellipse, inner node) or takes the node's chord: outside the ellipse
// the subpath and its chord form a closed curve that does not wind around
// the query, so in the chain identity the subpath's chord crossings equal the
// crossing of the node's chord.  A leaf inside its ellipse is a near pair
// (queued as in k_far).  A chain's root adds the chain's closing angle once.
// The near pairs are exactly the flat pass's: a leaf is only pruned under an
// ancestor whose (larger, inflated) ellipse the query is outside of.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_far_tree(PathTree tr, FaceTab ft, Points pts, const int32_t* item_offs,
                                                  const int2* item_map, uint32_t* item_counter, NearQueue nq,
                                                  Out out, double eps2, int skip_ordered) {
    __shared__ TNode s_node[kTreeChunk];  // the current chunk of whole chains
    __shared__ uint2 s_nbuf[kWavesPerWG][kNearBufT];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    const int total = item_offs[ft.num_faces];
    for (int iter = 0;; ++iter) {
        int item;
        if (item_counter) {
            __syncthreads();
            if (tid == 0) s_item = (int)atomicAdd(item_counter, 1u);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
        } else {
            if (iter > 0) break;
            item = blockIdx.x;
        }
        if (item >= total) break;
        const int2 mp = item_map[item];
        const int f = mp.x, tile = mp.y;
        int64_t qb = pts.offs[f], qe = pts.offs[f + 1];
        qb = qb < 0 ? 0 : (qb > pts.n ? pts.n : qb);
        qe = qe < qb ? qb : (qe > pts.n ? pts.n : qe);
        if (skip_ordered && qe - qb <= kOrderMaxPoints) continue;  // k_far_wtree's face
        const int64_t qi = qb + (int64_t)tile * (kWave * kWavesPerWG) + wave * kWave + lane;
        const bool active = qi < qe;
        double qx = 0.0, qy = 0.0;
        if (active) {
            qx = pts.u[qi * pts.stride];
            qy = pts.v[qi * pts.stride];
        }
        const bool valid = active && fabs(qx) < kCoordLimit && fabs(qy) < kCoordLimit;
        Turn T{1.0, 0.0, 0};
        int xc = 0, lost = 0;
        bool onb = false;
        int nfill = 0;  // entries in this wave's near-pair buffer (wave-uniform)
        // every chain's closing angle, once per query, in uniform control flow
        // (the roots follow each other through their skip indices)
        for (int r = kload(tr.begin, f), re_ = kload(tr.begin, f + 1); r < re_;) {
            const TNode rt = kload(tr.node, r);
            if (valid) close_chain(T, xc, rt.sx - qx, rt.sy - qy, rt.ex - qx, rt.ey - qy);
            r = rt.skip & ~kTreeRoot;
        }
        for (int k = tr.chunk_begin[f]; k < tr.chunk_begin[f + 1]; ++k) {
          const int2 ch = tr.chunk[k];
          const int lo = ch.x, ne = ch.y;
          __syncthreads();
          for (int i = tid; i < min(ne - lo, kTreeChunk); i += kWG) s_node[i] = tr.node[lo + i];
          __syncthreads();
          int n = valid ? lo : ne;
          for (;;) {
            const bool walk = n < ne;
            if (!__any(walk)) break;
            bool need = false;
            uint32_t seg = 0;
            if (walk) {
                const TNode nd = n - lo < kTreeChunk ? s_node[n - lo] : tr.node[n];
                const double ax = nd.sx - qx, ay = nd.sy - qy, bx = nd.ex - qx, by = nd.ey - qy;
                const double ra = ax * ax + ay * ay, rb = bx * bx + by * by;
                onb |= (ra < eps2) | (rb < eps2);
                const bool inside = !outside_ellipse(ra, rb, nd.hb2);
                const bool leaf = nd.seg >= 0;
                const bool take = !inside | leaf;  // the node's chord stands for its subpath
                ray_cross_mask(xc, low_mask(ay), low_mask(by), ax, ay, bx, by, __builtin_amdgcn_ballot_w64(take));
                need = take & leaf & inside & !onb;
                seg = (uint32_t)nd.seg;
                n = take ? (nd.skip & ~kTreeRoot) : n + 1;  // preorder: the left child follows its parent
            }
            const uint64_t m = __ballot(need);
            if (m) {
                const int cntm = __popcll(m);
                if (nfill + cntm > kNearBufT) {
                    lost |= flush_near(s_nbuf[wave], nfill, nq, lane, qi) ? 1 : 0;
                    nfill = 0;
                }
                if (need) s_nbuf[wave][nfill + lanes_below(m)] = make_uint2((uint32_t)qi, seg);
                nfill += cntm;
            }
          }
        }
        lost |= flush_near(s_nbuf[wave], nfill, nq, lane, qi) ? 1 : 0;
        if (active) {
            out.w[qi] = turn_angle(T) + kTwoPi * (double)xc;
            out.lab[qi] = !valid ? 3 : (onb ? 2 : (lost ? kRedo : 0));
        }
    }
}

// ---------------------------------------------------------------------------
// Far pass over the path hierarchy, one walk per wave.  The wave's 64 QPL
// queries are neighbours (the face's points in spatial order, through perm),
// and the wave visits the face's subpath trees in preorder in uniform control
// flow, one node per trip, read once from LDS for all lanes.  A query takes
// part in a node until it prunes an ancestor (skip_to: the node its walk
// resumes at).  At a node it takes the node's chord when outside the node's
// ellipse or at a leaf (the subpath and its chord bound no area around the
// query, so they cross its ray equally often), and an inner node it is
// outside of is pruned (skip_to = the node's skip index).  The wave goes down
// to the first child when some query is inside an inner node, else past the
// subtree.  Per query this is exactly k_far_tree's walk: the same chords, the
// same end points tested against eps, the same near pairs (a leaf inside its
// ellipse); only the reads and the control flow are shared.  Faces whose
// points keep the caller's order (more than kOrderMaxPoints) are skipped.
// ---------------------------------------------------------------------------
// flush_near for queries of arbitrary indices: bit q of lost is set when a
// pair of query qi[q] did not fit in the queue.
template <int QPL>
__device__ __forceinline__ void flush_near_list(const uint2* buf, int nfill, const NearQueue& nq, int lane,
                                                const int32_t (&qi)[QPL], int& lost) {
    if (nfill == 0) return;
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(nq.count, (unsigned long long)nfill);
    base = __shfl(base, 0);
    for (int e = lane; e < nfill; e += kWave)
        if (base + (unsigned long long)e < nq.cap) nq.qs[base + e] = buf[e];
    if (base + (unsigned long long)nfill > nq.cap) {
        for (int e = 0; e < nfill; ++e) {
            if (base + (unsigned long long)e < nq.cap) continue;
            const uint32_t x = buf[e].x;
#pragma unroll
            for (int q = 0; q < QPL; ++q) lost |= x == (uint32_t)qi[q] ? 1 << q : 0;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

template <int QPL>
__global__ __launch_bounds__(kWG) void k_far_wtree(PathTree tr, FaceTab ft, Points pts, const uint32_t* perm,
                                                   const int32_t* item_offs, const int2* item_map,
                                                   uint32_t* item_counter, NearQueue nq, Out out, double eps2) {
    constexpr int kQPWG = kWave * QPL * kWavesPerWG;  // queries per work item
    __shared__ TNode s_node[kTreeChunk];                // the current chunk of whole chains
    __shared__ uint2 s_nbuf[kWavesPerWG][kNearBufT];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    const int total = item_offs[ft.num_faces];
    for (int iter = 0;; ++iter) {
        int item;
        if (item_counter) {
            __syncthreads();
            if (tid == 0) s_item = (int)atomicAdd(item_counter, 1u);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
        } else {
            if (iter > 0) break;
            item = blockIdx.x;
        }
        if (item >= total) break;
        const int2 mp = item_map[item];
        const int f = mp.x, tile = mp.y;
        int64_t qb = pts.offs[f], qe = pts.offs[f + 1];
        qb = qb < 0 ? 0 : (qb > pts.n ? pts.n : qb);
        qe = qe < qb ? qb : (qe > pts.n ? pts.n : qe);
        if (qe - qb > kOrderMaxPoints) continue;  // k_far_tree's face (the same for the whole workgroup)
        int32_t qi[QPL];    // query index (-1: no query in this slot)
        double qx[QPL], qy[QPL];
        Turn T[QPL];
        int xc[QPL], skip_to[QPL];
        uint64_t em[QPL];   // lanes with an end point within eps
        int lost = 0;       // bit q: a near pair of query q did not fit in the queue
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            const int64_t slot = qb + (int64_t)tile * kQPWG + (int64_t)(wave * QPL + q) * kWave + lane;
            qi[q] = slot < qe ? (int32_t)perm[slot] : -1;
            qx[q] = qy[q] = 0.0;
            if (qi[q] >= 0) {
                qx[q] = pts.u[(int64_t)qi[q] * pts.stride];
                qy[q] = pts.v[(int64_t)qi[q] * pts.stride];
            }
            // an inactive or invalid query sits at (kAway, kAway): its squared
            // distances overflow to +inf, so it is outside every ellipse, within
            // eps of no end point and crosses no chord
            if (!(qi[q] >= 0 && fabs(qx[q]) < kCoordLimit && fabs(qy[q]) < kCoordLimit)) qx[q] = qy[q] = kAway;
            T[q] = Turn{1.0, 0.0, 0};
            xc[q] = 0;
            em[q] = 0;
        }
        int nfill = 0;  // entries in this wave's near-pair buffer (wave-uniform)
        // every chain's closing angle, once per query, in uniform control flow
        for (int r = kload(tr.begin, f), re_ = kload(tr.begin, f + 1); r < re_;) {
            const TNode rt = kload(tr.node, r);
#pragma unroll
            for (int q = 0; q < QPL; ++q)
                if (qx[q] != kAway) close_chain(T[q], xc[q], rt.sx - qx[q], rt.sy - qy[q], rt.ex - qx[q], rt.ey - qy[q]);
            r = rt.skip & ~kTreeRoot;
        }
        for (int k = tr.chunk_begin[f]; k < tr.chunk_begin[f + 1]; ++k) {
            const int2 ch = tr.chunk[k];
            const int lo = ch.x, ne = ch.y;
            __syncthreads();
            for (int i = tid; i < min(ne - lo, kTreeChunk); i += kWG) s_node[i] = tr.node[lo + i];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < QPL; ++q) skip_to[q] = lo;
            int i = lo;  // wave-uniform
            while (i < ne) {
                const TNode nd = i - lo < kTreeChunk ? s_node[i - lo] : kload(tr.node, i);
                const bool leaf = nd.seg >= 0;
                const int nskip = nd.skip & ~kTreeRoot;
                uint64_t nm[QPL];
                uint64_t stay = 0;
#pragma unroll
                for (int q = 0; q < QPL; ++q) {
                    const uint64_t am = __builtin_amdgcn_ballot_w64(skip_to[q] <= i);
                    const double ax = nd.sx - qx[q], ay = nd.sy - qy[q];
                    const double bx = nd.ex - qx[q], by = nd.ey - qy[q];
                    const double ra = fma(ax, ax, ay * ay), rb = fma(bx, bx, by * by);
                    em[q] |= (__builtin_amdgcn_fcmp(ra, eps2, kCmpOLT) | __builtin_amdgcn_fcmp(rb, eps2, kCmpOLT)) & am;
                    const uint64_t in = near_mask(ra, rb, nd.hb2);
                    const uint64_t take = leaf ? am : (am & ~in);
                    ray_cross_mask(xc[q], low_mask(ay), low_mask(by), ax, ay, bx, by, take);
                    nm[q] = leaf ? (am & in & ~em[q]) : 0ull;
                    if (!leaf) {
                        if (__builtin_amdgcn_inverse_ballot_w64(am & ~in)) skip_to[q] = nskip;
                        stay |= am & in;
                    }
                }
                if (leaf) {
                    int cnt = 0;
#pragma unroll
                    for (int q = 0; q < QPL; ++q) cnt += __popcll(nm[q]);
                    if (cnt > 0) {
                        if (nfill + cnt > kNearBufT) {
                            flush_near_list<QPL>(s_nbuf[wave], nfill, nq, lane, qi, lost);
                            nfill = 0;
                        }
#pragma unroll
                        for (int q = 0; q < QPL; ++q) {
                            if (__builtin_amdgcn_inverse_ballot_w64(nm[q]))
                                s_nbuf[wave][nfill + lanes_below(nm[q])] = make_uint2((uint32_t)qi[q], (uint32_t)nd.seg);
                            nfill += __popcll(nm[q]);
                        }
                    }
                }
                i = (!leaf && stay != 0ull) ? i + 1 : nskip;  // a leaf's skip index is i + 1
            }
        }
        flush_near_list<QPL>(s_nbuf[wave], nfill, nq, lane, qi, lost);
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            if (qi[q] < 0) continue;
            const bool valid = qx[q] != kAway;
            const bool onb = valid & __builtin_amdgcn_inverse_ballot_w64(em[q]);
            out.w[qi[q]] = turn_angle(T[q]) + kTwoPi * (double)xc[q];
            out.lab[qi[q]] = !valid ? 3 : (onb ? 2 : (((lost >> q) & 1) ? kRedo : 0));
        }
    }
}

// ---------------------------------------------------------------------------
// near pass.  Each wave owns a contiguous chunk of the queue and keeps all
// its lanes busy: a lane that finishes its pair takes the next pair of the
// chunk (wave-local counter, no global atomics).  One node of Alg. 1 per
// loop trip, so lanes with short and long recursions interleave.
// ---------------------------------------------------------------------------

// Near-pair state.  The current interval [a, a + 2^-k] is always one that
// failed its ellipse test (the root is queued for exactly that reason).
//
// Deferred intervals.  The traversal goes left first and defers the right
// half of a split whose halves both failed, so the deferred intervals form a
// stack whose levels increase from bottom to top, and the one to resume is
// always the top (the deepest).  An entry holds the deferred interval's two
// end points (32 B); its level is a bit of `pend`, its left end parameter
// follows from the current one (deferred_left).  The entries sit in an LDS
// ring of kNearSlots slots per lane, entry i in slot i mod kNearSlots, so a
// slot is only reused when more than kNearSlots intervals are pending: a push
// over a pending entry marks every entry below `lost` as overwritten, and such
// an entry's end points are evaluated again when it resumes (same parameters,
// same code, same values).
struct NodeState {
    Coef c;  // translated by -q: evaluates gamma(t) - q directly
    double B, eta;
    double a, ax, ay, bx, by;  // current interval: left end parameter, end points relative to q
    uint64_t pend;             // levels of the deferred intervals
    int k;
    int n;         // far children's ray crossings minus the segment chord's (see near_pair)
    int pmax;      // deepest level of this pair
    int sp;        // deferred intervals on the stack
    int lost;      // entries below this index were overwritten in the ring
    int mode;      // 0: split; 1, 2: evaluate the left, right end of a resumed overwritten interval
    uint32_t seg;  // segment (its end point is reloaded when a resumed interval ends at t = 1)
};

__device__ __forceinline__ void node_init(NodeState& st, const Segs& sg, uint32_t s, double qx, double qy) {
    NearSeg g;
    load_near_seg(sg, s, st.c, g);
    // sum_i C(n,i) w_i (P_i - q) B_i(t) / sum_i C(n,i) w_i B_i(t) = gamma(t) - q
#pragma unroll
    for (int j = 0; j < kCoef; ++j) {
        st.c.x[j] = fma(-st.c.w[j], qx, st.c.x[j]);
        st.c.y[j] = fma(-st.c.w[j], qy, st.c.y[j]);
    }
    st.B = g.B;
    st.eta = g.eta;
    st.seg = s;
    st.ax = g.p0x - qx;
    st.ay = g.p0y - qy;
    st.bx = g.pnx - qx;
    st.by = g.pny - qy;
    st.n = -ray_cross(st.ax, st.ay, st.bx, st.by);
    st.a = 0.0;
    st.k = 0;
    st.pend = 0;
    st.pmax = 0;
    st.sp = 0;
    st.lost = 0;
    st.mode = 0;
}

struct NodeCount {
    uint32_t split = 0, leaf = 0, reeval = 0, maxk = 0;
    uint64_t flops = 0;
    uint32_t trips = 0, busy = 0;  // loop trips of the wave (lane 0), trips holding a pair (every lane)
};

// One split of Alg. 1: the current interval is halved at its midpoint and
// BOTH halves are tested.  A half that passes is a leaf: its chord's ray
// crossing is taken at once (the sum does not depend on the order).  A half
// that fails becomes the current interval; when both fail, the right one is
// deferred.  When neither fails, the top deferred interval resumes (it failed
// its test when its parent was split).  Every step is therefore one curve
// evaluation: a pair costs as many steps as Alg. 1 has split nodes (plus two
// per resumed interval whose entry was overwritten), and the set of tested
// nodes, splits and leaves is exactly Alg. 1's.  State changes are selects;
// the memory accesses and the evaluation sit under branches.  `stk` is this
// lane's slot 0 (slot stride kWave).  Returns true when the pair is finished.
template <bool COUNT>
__device__ __forceinline__ bool node_step(NodeState& st, double eps2, double4* stk, bool& onb, NodeCount& nc,
                                          const Segs& sg, double qx, double qy, bool has) {
    // The step's one evaluation: the midpoint a + 2^-(k+1) for a split, or an
    // end point (a, then a + 2^-k) of a resumed overwritten interval.
    const bool sp = has & (st.mode == 0);
    const bool fl = has & (st.mode == 1), fr = has & (st.mode == 2);
    const bool capped = sp & (st.k >= kDepthCap);  // cannot happen for a validated eps
    const int k1 = st.k + 1;
    const double te = fl ? st.a : st.a + ldexp(1.0, fr ? -st.k : -k1);
    const bool at_end = fr & (te == 1.0);
    double mx = 0.0, my = 0.0;
    if ((sp & !capped) | fl | (fr & !at_end)) bez_eval(st.c, te, mx, my);
    if (at_end) {
        const double2 e = seg_end_point(sg, (int)st.seg);
        mx = e.x - qx;
        my = e.y - qy;
    }
    // squared distances of the end points (recomputed: cheaper than carrying them)
    const double rm = fma(mx, mx, my * my);
    const double ra = fma(st.ax, st.ax, st.ay * st.ay);
    const double rb = fma(st.bx, st.bx, st.by * st.by);
    if (COUNT) nc.reeval += (fl | fr) ? 1 : 0;
    st.mode = fl ? 2 : 0;
    // split
    const bool hit = sp & !capped & (rm < eps2);
    onb |= capped | hit;
    bool fin = capped | hit;
    const bool go = sp & !capped & !hit;
    // the two halves [a, m] and [m, b] at level k + 1
    const double hb = half_axis2(st.B, st.eta, k1);
    const bool lfar = outside_ellipse(ra, rm, hb);
    const bool rfar = outside_ellipse(rm, rb, hb);
    // n += ray_cross(a, m) for a far left half, ray_cross(m, b) for a far right
    // half, on lane masks: a half's orientation is only computed when some
    // lane's half changes side of the ray's line
    {
        const uint64_t gm = __builtin_amdgcn_ballot_w64(go);
        const uint64_t am = low_mask(st.ay), mm = low_mask(my), bm = low_mask(st.by);
        ray_cross_mask(st.n, am, mm, st.ax, st.ay, mx, my, gm & __builtin_amdgcn_ballot_w64(lfar));
        ray_cross_mask(st.n, mm, bm, mx, my, st.bx, st.by, gm & __builtin_amdgcn_ballot_w64(rfar));
    }
    if (COUNT && go) {
        ++nc.split;
        nc.flops += 6 * st.c.n + 15 + 11 * ((lfar ? 1 : 0) + (rfar ? 1 : 0));
        nc.leaf += (lfar ? 1 : 0) + (rfar ? 1 : 0);
        nc.maxk = (uint32_t)k1 > nc.maxk ? (uint32_t)k1 : nc.maxk;
    }
    const bool both = go & !lfar & !rfar;  // defer the right half, continue left
    const bool left = go & !lfar;          // continue with the left half
    const bool right = go & lfar & !rfar;  // continue with the right half
    const bool none = go & lfar & rfar;    // resume the top deferred interval
    // push the right half's end points
    if (both) stk[(st.sp & (kNearSlots - 1)) * kWave] = make_double4(mx, my, st.bx, st.by);
    const int lost_push = max(min(st.lost, st.sp), st.sp - (kNearSlots - 1));
    st.lost = both ? lost_push : st.lost;
    st.pend = both ? (st.pend | (1ull << k1)) : st.pend;
    st.sp += both ? 1 : 0;
    st.pmax = (go & (k1 > st.pmax)) ? k1 : st.pmax;
    fin |= none & (st.pend == 0);
    const bool pop = none & (st.pend != 0);
    const int kk = 63 - __clzll(st.pend | 1ull);
    const int top = st.sp - 1;
    const bool kept = top >= st.lost;
    double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
    if (pop & kept) p = stk[(top & (kNearSlots - 1)) * kWave];
    st.pend = pop ? (st.pend & ~(1ull << kk)) : st.pend;
    st.sp -= pop ? 1 : 0;
    st.mode = (pop & !kept) ? 1 : st.mode;
    st.a = right ? te : (pop ? deferred_left(st.a, kk) : st.a);
    st.k = (left | right) ? k1 : (pop ? kk : st.k);
    // end points of the next interval: m for a re-evaluated left end or when
    // continuing right (left end) / left (right end); the entry on a pop; else
    // unchanged (the cases exclude each other, so each field takes two selects)
    const bool take_a = fl | right, take_b = fr | left, pk = pop & kept;
    st.ax = take_a ? mx : (pk ? p.x : st.ax);
    st.ay = take_a ? my : (pk ? p.y : st.ay);
    st.bx = take_b ? mx : (pk ? p.z : st.bx);
    st.by = take_b ? my : (pk ? p.w : st.by);
    return fin;
}

// A wave-uniform 64-bit value made visibly uniform (scalar registers).
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

template <typename T_>
__device__ __forceinline__ T_ wave_sum(T_ v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Queue entries per chunk taken by a wave from the pass's cursor.
constexpr unsigned long long kNearChunk = 512;

template <bool COUNT>
__global__ __launch_bounds__(kWG) void k_near(
    Segs sg, Points pts, NearQueue nq, Out out, double eps2, Stats stats, const uint8_t* seg_per,
    uint8_t* entry_depth, const unsigned long long* q_lo, const unsigned long long* q_hi,
    unsigned long long* cursor) {
    __shared__ double4 s_stack[kWavesPerWG * kNearSlots * kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    double4* stk = s_stack + wave * kNearSlots * kWave + lane;
    // Queue entries [q_lo, q_hi) (defaults: 0 and the queue's count).  With a
    // cursor (zero at launch), a wave that runs dry takes the next chunk of
    // kNearChunk entries from it, so the pass ends when the work does rather
    // than when the slowest of equal shares does; without one, each wave takes
    // one equal share.
    unsigned long long n = q_hi ? *q_hi : *nq.count;
    n = n < nq.cap ? n : nq.cap;
    unsigned long long base = q_lo ? *q_lo : 0ull;
    base = base < n ? base : n;
    const unsigned long long gw = (unsigned long long)blockIdx.x * kWavesPerWG + wave;
    // wave-uniform chunk [next, c_end), kept in scalar registers
    unsigned long long next = 0, c_end = 0;
    bool more = true, shared_once = false;
    NodeState st;
    bool onb = false, has = false;
    uint32_t q = 0;
    double qx = 0.0, qy = 0.0;   // this lane's query (translated for periodic copies)
    unsigned long long cur = 0;  // queue index of this lane's pair
    NodeCount nc;
    // window of the next 64 queue entries, one per lane, loaded one refill ahead
    uint2 win = make_uint2(0xffffffffu, 0u);
    auto grab = [&]() {
        if (cursor) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(cursor, kNearChunk);
            c = uniform_u64(c);  // lane 0's
            next = uniform_u64(base + c < n ? base + c : n);
            c_end = uniform_u64(next + kNearChunk < n ? next + kNearChunk : n);
        } else if (!shared_once) {
            const unsigned long long nw = (unsigned long long)gridDim.x * kWavesPerWG;
            const unsigned long long per = (n - base + nw - 1) / nw;
            next = uniform_u64(base + gw * per < n ? base + gw * per : n);
            c_end = uniform_u64(next + per < n ? next + per : n);
            shared_once = true;
        } else {
            next = c_end = n;
        }
        more = next < c_end;
        if (next + lane < c_end) win = nq.qs[next + lane];
    };
    grab();
    for (;;) {
        const uint64_t idle = __ballot(!has);
        // refill idle lanes once kRefillMin of them are idle (each refill
        // waits for the gathers of the new pairs' data)
        if (idle && more && (__popcll(idle) >= kRefillMin || idle == ~0ull)) {
            if (next >= c_end) grab();
            if (more) {
                const int rank = lanes_below(idle);
                uint2 e;  // all lanes active here: entry next + rank comes from lane rank of the window
                e.x = (uint32_t)__shfl((int)win.x, rank);
                e.y = (uint32_t)__shfl((int)win.y, rank);
                if (!has && next + rank < c_end) {
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
                        node_init(st, sg, e.y, qx, qy);
                        onb = false;
                        has = true;
                    }
                }
                const unsigned long long took = (unsigned long long)__popcll(idle);
                next = uniform_u64(next + took < c_end ? next + took : c_end);
                if (next + lane < c_end) win = nq.qs[next + lane];
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
        if (node_step<COUNT>(st, eps2, stk, onb, nc, sg, qx, qy, has)) {
            // the pair's angle is its chord angle (already in the far pass's
            // sum) plus 2 pi n; most pairs have n = 0 and write nothing
            if (onb) out.lab[q] = 2;
            else if (st.n != 0) unsafeAtomicAdd(&out.w[q], kTwoPi * (double)st.n);
            if (COUNT && entry_depth) entry_depth[cur] = (uint8_t)(st.pmax < 255 ? st.pmax : 255);
            has = false;
        }
    }
    if (COUNT && stats.c) {
        const unsigned long long sp = wave_sum((unsigned long long)nc.split);
        const unsigned long long lf = wave_sum((unsigned long long)nc.leaf);
        const unsigned long long re = wave_sum((unsigned long long)nc.reeval);
        const unsigned long long fl = wave_sum((unsigned long long)nc.flops);
        const uint32_t mk = wave_max(nc.maxk);
        const unsigned long long tr = wave_sum((unsigned long long)nc.trips);
        const unsigned long long bu = wave_sum((unsigned long long)nc.busy);
        if (lane == 0) {
            atomicAdd(&stats.c[6], tr);
            atomicAdd(&stats.c[7], bu);
            if (gw == 0) atomicAdd(&stats.c[0], n);
            atomicAdd(&stats.c[1], sp);
            atomicAdd(&stats.c[2], lf);
            atomicAdd(&stats.c[3], re);
            atomicAdd(&stats.c[4], fl);
            atomicMax(&stats.c[5], (unsigned long long)mk);
        }
    }
}

__device__ __forceinline__ void redo_query(const Segs& sg, const FaceTab& ft, const Points& pts, const Out& out,
                                           double eps2, double4* stk, int64_t i) {
    // face of point i: last f with offs[f] <= i
    int lo = 0, hi = ft.num_faces - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pts.offs[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const double qx = pts.u[i * pts.stride], qy = pts.v[i * pts.stride];
    Turn T{1.0, 0.0, 0};
    int xc = 0;
    bool onb = false;
    int cnt = 0;
    for (int s = ft.seg_begin[lo]; s < ft.seg_begin[lo + 1] && !onb; ++s) {
        const double ax = sg.p0x[s] - qx, ay = sg.p0y[s] - qy;
        const double bx = sg.pnx[s] - qx, by = sg.pny[s] - qy;
        const double ra = ax * ax + ay * ay, rb = bx * bx + by * by;
        if (ra < eps2 || rb < eps2) {
            onb = true;
            break;
        }
        if (outside_ellipse(ra, rb, sg.hb2[s])) {
            turn_mul(T, ax * bx + ay * by, ax * by - ay * bx);
        } else {
            chord_factor(T, ax, ay, bx, by);
            (void)near_from_global(xc, sg, (uint32_t)s, qx, qy, eps2, stk, onb);
        }
        if ((++cnt & 3) == 0) turn_norm(T);
    }
    if (onb) {
        out.w[i] = __builtin_nan("");
        out.lab[i] = 2;
    } else {
        const double w = (turn_angle(T) + kTwoPi * (double)xc) / kTwoPi;
        out.w[i] = w;
        out.lab[i] = classify(w, out.rule);
    }
}


// Queries that lost a near pair to a full queue: recompute the whole query
// in line (one lane per query).  Runs after k_finalize and overwrites.  A
// queue that never overflowed lost nothing: then the kernel returns at once.
__global__ __launch_bounds__(kWG) void k_redo(Segs sg, FaceTab ft, Points pts, Out out, double eps2,
                                              const unsigned long long* near_count, uint64_t near_cap) {
    __shared__ double4 s_stack[kWavesPerWG * kNearSlots * kWave];
    if (*near_count <= near_cap) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    double4* stk = s_stack + wave * kNearSlots * kWave + lane;
    const int64_t n = min(pts.n, pts.offs[ft.num_faces]);
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        if (out.lab[i] == kRedo) redo_query(sg, ft, pts, out, eps2, stk, i);
}
// Points are [q0, q1), further bounded by offs[nf] when nf >= 0 (the live
// point count of a replayed graph).
__global__ __launch_bounds__(kWG) void k_finalize(Points pts, Out out, int64_t q0, int64_t q1, int32_t nf) {
    const int64_t i = q0 + (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= q1 || i >= pts.n) return;
    if (nf >= 0 && i >= pts.offs[nf]) return;
    const uint8_t f = out.lab[i];
    double w = out.w[i];
    uint8_t lab;
    if (f == kRedo) {
        return;  // recomputed by k_redo
    } else if (f == 3) {
        w = __builtin_nan("");
        lab = 3;
    } else if (f == 2) {
        w = __builtin_nan("");
        lab = 2;
    } else {
        w = w / kTwoPi;
        lab = classify(w, out.rule);
    }
    out.w[i] = w;
    out.lab[i] = lab;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_build_items(const FaceTab& ft, const Points& pts, int qpw, int32_t* item_offs, int2* item_map,
                              int64_t map_cap, uint32_t* counters, bool zero_near, hipStream_t st) {
    hipLaunchKernelGGL(k_build_items, dim3(1), dim3(1024), 0, st, ft, pts, qpw, item_offs, item_map, map_cap,
                       counters, zero_near ? 1 : 0);
    return hipGetLastError();
}

template <bool INLINE, bool MIXED>
static hipError_t launch_far_q(int qpw, dim3 grid, hipStream_t st, const Segs& sg, const FaceTab& ft,
                               const Points& pts, const int32_t* item_offs, const int2* item_map,
                               uint32_t* item_counter, int32_t single_face, NearQueue nq, Out out, double eps2) {
    switch (qpw) {
        case 64:
            hipLaunchKernelGGL((k_far<INLINE, 1, MIXED>), grid, dim3(kWG), 0, st, sg, ft, pts, item_offs, item_map,
                               item_counter, single_face, nq, out, eps2);
            break;
        case 128:
            hipLaunchKernelGGL((k_far<INLINE, 2, MIXED>), grid, dim3(kWG), 0, st, sg, ft, pts, item_offs, item_map,
                               item_counter, single_face, nq, out, eps2);
            break;
        default:
            hipLaunchKernelGGL((k_far<INLINE, 4, MIXED>), grid, dim3(kWG), 0, st, sg, ft, pts, item_offs, item_map,
                               item_counter, single_face, nq, out, eps2);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_far(bool inline_near, bool mixed, int qpw, const Segs& sg, const FaceTab& ft, const Points& pts,
                      const int32_t* item_offs, const int2* item_map, uint32_t* item_counter, int32_t single_face,
                      int64_t grid, NearQueue nq, Out out, double eps2, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    const dim3 g((unsigned)grid);
    if (inline_near)
        return mixed ? launch_far_q<true, true>(qpw, g, st, sg, ft, pts, item_offs, item_map, item_counter,
                                                single_face, nq, out, eps2)
                     : launch_far_q<true, false>(qpw, g, st, sg, ft, pts, item_offs, item_map, item_counter,
                                                 single_face, nq, out, eps2);
    return mixed ? launch_far_q<false, true>(qpw, g, st, sg, ft, pts, item_offs, item_map, item_counter, single_face,
                                             nq, out, eps2)
                 : launch_far_q<false, false>(qpw, g, st, sg, ft, pts, item_offs, item_map, item_counter,
                                              single_face, nq, out, eps2);
}

hipError_t launch_near(const Segs& sg, const Points& pts, NearQueue nq, Out out, double eps2, int64_t grid,
                       Stats stats, const uint8_t* seg_per, uint8_t* entry_depth, hipStream_t st,
                       const unsigned long long* q_lo, const unsigned long long* q_hi, unsigned long long* cursor) {
    if (grid <= 0) return hipSuccess;
    if (stats.c || entry_depth)
        hipLaunchKernelGGL(k_near<true>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, pts, nq, out, eps2, stats,
                           seg_per, entry_depth, q_lo, q_hi, cursor);
    else
        hipLaunchKernelGGL(k_near<false>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, pts, nq, out, eps2, stats,
                           seg_per, entry_depth, q_lo, q_hi, cursor);
    return hipGetLastError();
}

// The queue's entry count at this point of the stream (the end of one far
// phase's entries, the start of the next's).
__global__ void k_queue_mark(const unsigned long long* count, unsigned long long* mark) { *mark = *count; }

hipError_t launch_queue_mark(const unsigned long long* count, unsigned long long* mark, hipStream_t st) {
    hipLaunchKernelGGL(k_queue_mark, dim3(1), dim3(1), 0, st, count, mark);
    return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_split_pairs(const uint2* qs, int64_t n, int32_t* point, int32_t* segment) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
        const uint2 e = qs[i];
        point[i] = (int32_t)e.x;
        segment[i] = (int32_t)e.y;
    }
}

hipError_t launch_split_pairs(const uint2* qs, int64_t n, int32_t* point, int32_t* segment, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((n + kWG - 1) / kWG, 65536);
    hipLaunchKernelGGL(k_split_pairs, dim3((unsigned)g), dim3(kWG), 0, st, qs, n, point, segment);
    return hipGetLastError();
}

hipError_t launch_finalize(const Points& pts, Out out, int64_t q0, int64_t q1, int32_t nf, hipStream_t st) {
    if (q1 <= q0) return hipSuccess;
    const int64_t g = (q1 - q0 + kWG - 1) / kWG;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)g), dim3(kWG), 0, st, pts, out, q0, q1, nf);
    return hipGetLastError();
}

hipError_t launch_redo(const Segs& sg, const FaceTab& ft, const Points& pts, Out out, double eps2,
                       const NearQueue& nq, int64_t max_grid, hipStream_t st) {
    if (pts.n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((pts.n + kWG - 1) / kWG, std::max<int64_t>(1, max_grid));
    hipLaunchKernelGGL(k_redo, dim3((unsigned)g), dim3(kWG), 0, st, sg, ft, pts, out, eps2, nq.count, nq.cap);
    return hipGetLastError();
}

int near_blocks_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_near<false>, kWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

template <bool INLINE, bool MIXED>
static hipError_t far_occupancy(int* nb, int qpw) {
    return qpw == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_far<INLINE, 1, MIXED>, kWG, 0)
           : qpw == 128 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_far<INLINE, 2, MIXED>, kWG, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_far<INLINE, 4, MIXED>, kWG, 0);
}

hipError_t launch_farq(int qpl, const Segs& sg, const FaceTab& ft, const Points& pts, const int32_t* item_offs,
                       const int2* item_map, uint32_t* item_counter, int64_t grid, NearQueue nq, Out out, double eps2,
                       hipStream_t st, int rank_lo, int rank_hi) {
    if (rank_hi < 0) rank_hi = ft.num_faces;
    if (rank_lo < 0 || rank_lo > rank_hi || rank_hi > ft.num_faces) return hipErrorInvalidValue;
    if (grid <= 0) return hipSuccess;
    if (qpl == 2)
        hipLaunchKernelGGL(k_farq<2>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, ft, pts, item_offs, item_map,
                           item_counter, nq, out, eps2, rank_lo, rank_hi);
    else if (qpl == 3)
        hipLaunchKernelGGL(k_farq<3>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, ft, pts, item_offs, item_map,
                           item_counter, nq, out, eps2, rank_lo, rank_hi);
    else if (qpl == 4)
        hipLaunchKernelGGL(k_farq<4>, dim3((unsigned)grid), dim3(kWG), 0, st, sg, ft, pts, item_offs, item_map,
                           item_counter, nq, out, eps2, rank_lo, rank_hi);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int farq_blocks_per_cu(int qpl) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (qpl == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_farq<2>, kWG, 0);
    if (qpl == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_farq<3>, kWG, 0);
    if (qpl == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_farq<4>, kWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_far_tree(const PathTree& tr, const FaceTab& ft, const Points& pts, const int32_t* item_offs,
                           const int2* item_map, uint32_t* item_counter, int64_t grid, NearQueue nq, Out out,
                           double eps2, hipStream_t st, bool skip_ordered) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_far_tree, dim3((unsigned)grid), dim3(kWG), 0, st, tr, ft, pts, item_offs, item_map,
                       item_counter, nq, out, eps2, skip_ordered ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_far_wtree(const PathTree& tr, const FaceTab& ft, const Points& pts, const uint32_t* perm,
                            const int32_t* item_offs, const int2* item_map, uint32_t* item_counter, int64_t grid,
                            NearQueue nq, Out out, double eps2, hipStream_t st) {
    if (grid <= 0 || !perm) return grid <= 0 ? hipSuccess : hipErrorInvalidValue;
    hipLaunchKernelGGL(k_far_wtree<kWtreeQPL>, dim3((unsigned)grid), dim3(kWG), 0, st, tr, ft, pts, perm, item_offs,
                       item_map, item_counter, nq, out, eps2);
    return hipGetLastError();
}

int far_wtree_blocks_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_far_wtree<kWtreeQPL>, kWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

int far_tree_blocks_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_far_tree, kWG, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

int far_blocks_per_cu(bool inline_near, bool mixed, int qpw) {
    int nb = 0;
    hipError_t e;
    if (inline_near) e = mixed ? far_occupancy<true, true>(&nb, qpw) : far_occupancy<true, false>(&nb, qpw);
    else e = mixed ? far_occupancy<false, true>(&nb, qpw) : far_occupancy<false, false>(&nb, qpw);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace wn
