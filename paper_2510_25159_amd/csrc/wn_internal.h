// Internal layout shared by the host side (wn_host.hip) and the kernels
// (wn_kernels.hip) of the winding-number library.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wn {

constexpr int kMaxDeg = 5;
constexpr int kCoef = kMaxDeg + 1;  // coefficient slots per segment
// fourth components of a segment's coefficient slots
constexpr int kPadB = 0, kPadEta = 1, kPadP0x = 2, kPadP0y = 3, kPadPnx = 4, kPadPny = 5;
static_assert(kCoef == 6, "six padding doubles per segment record");
constexpr int kWave = 64;
constexpr int kWG = 256;            // threads per workgroup of the pair kernels
constexpr int kWavesPerWG = kWG / kWave;
constexpr int kNearSlots = 4;       // LDS ring slots per lane for deferred intervals (two end points each)
constexpr int kDepthCap = 52;       // dyadic parameters a + 2^-k stay exact in FP64
constexpr int kSegChunk = kWG;      // segments staged in LDS per chunk
// Per-wave LDS buffers of near pairs before one queue append (one atomic on
// the queue's count).  Appends to that single counter from every wave of the
// GPU contend: with 256-entry buffers the far pass of the batched planar set
// (154.5M near pairs) spent about half its time on them, so the planar far
// passes take larger buffers as far as their LDS budgets allow.
constexpr int kNearBuf = 256;    // periodic far pass (its entries carry a shift too)
constexpr int kNearBufQ = 896;   // k_farq (four queries per lane; four workgroups fit in LDS)
constexpr int kNearBufT = 480;   // k_far (queued), k_far_tree, k_far_wtree (4 workgroups of the
                                 // hierarchy passes, 24 KB of nodes each, fit in 160 KB of LDS)
constexpr int kRefillMin = 16;      // near pass: idle lanes of a wave before they take new pairs
constexpr float kMixedMargin = 0x1p-20f; // precision MIXED: relative FP32 admission margin
// Relative inflation of the ellipse axis: the far decision is taken only when
// it survives rounding (Lemma 1 boundary "<=" counts as inside, so inflating
// the bound only sends borderline pairs to the recursion).
constexpr double kAxisInflate = 9.094947017729282e-13;  // 2^-40
// Coordinates (control points at creation, queries at run time) must stay
// below this magnitude so that a few chord factors multiplied between two
// rescalings of the angle accumulator can neither overflow nor underflow.
constexpr double kCoordLimit = 1e15;

// Per-segment data.  Far-field arrays are structure-of-arrays (coalesced
// staging into LDS); the recursion coefficients of one segment are contiguous
// (each near-pair lane gathers a different segment).
// Far-test record of a periodic segment: lifted end points and the root
// ellipse's hb2, 64-B aligned so that one scalar load fetches it.
struct alignas(64) FarRec {
    double p0x, p0y, pnx, pny, hb2, pad[3];
};

struct Segs {
    const double* p0x;  // [S] curve start gamma(0)
    const double* p0y;
    const double* pnx;  // [S] curve end gamma(1)
    const double* pny;
    const double* hb2;  // [S] 0.5 * (B (1 + kAxisInflate) + eta)^2 : root ellipse test
    const double* B;    // [S] derivative bound (Lemma 1 / App. A.1)
    const double* eta;  // [S] absolute rounding margin of the ellipse axis
    const double* coef; // [S][kCoef][4]: slot j = (x, y, w, pad_j) of C(n, n-j) w_{n-j} P_{n-j};
                        // pad_j = B, eta, p0x, p0y, pnx, pny (kPad*) for the near pass
    const uint8_t* deg; // [S] degree 1..5
    const uint8_t* rat; // [S] 1 if any weight != 1
    const uint8_t* join;// [S] 1 when gamma(0) equals the previous segment's gamma(1) bit for bit
    const double* box;  // [S][4] control-point box umin, umax, vmin, vmax (lifted for periodic faces)
    const float* wrange;// [S][2] min, max weight
    const FarRec* frec; // [S] periodic segments' far-test records (face sets with periodic faces)
};

// Path hierarchy (Sec. 4.2): per chain of bit-joined segments
// of a planar face, a balanced binary tree of subpaths in preorder.  A node's
// ellipse has foci at the subpath's start and end and an axis bounding its
// length (sum of the segments' inflated bounds); a query outside it sees the
// whole subpath as its chord.  Leaves carry the segment's own root test.
struct TNode {
    double sx, sy, ex, ey;  // first segment's gamma(0), last segment's gamma(1)
    double hb2;             // 0.5 * axis^2 (leaves: the segment's hb2)
    int32_t skip;           // index of the node after this subtree; bit 31 set at a chain's root
    int32_t seg;            // segment of a leaf, -1 for an inner node
};
static_assert(sizeof(TNode) == 48, "one node per 48 B");
constexpr int32_t kTreeRoot = (int32_t)0x80000000u;

struct PathTree {
    const TNode* node;        // [nodes]
    const int32_t* begin;     // [F+1] nodes of face f are [begin[f], begin[f+1]) (empty for periodic faces)
    const int2* chunk;        // [chunks] node ranges of whole chains, at most kTreeChunk nodes unless one
                              // chain is longer (its nodes beyond kTreeChunk are read from memory)
    const int32_t* chunk_begin;  // [F+1] chunks of face f are [chunk_begin[f], chunk_begin[f+1])
};
constexpr int kTreeChunk = 512;  // nodes staged in LDS at a time (24 KB)
// Faces with more points keep the caller's order in the spatial ordering (one
// workgroup would take too long over them; large faces already fill several
// waves per copy).
constexpr int64_t kOrderMaxPoints = 65536;
constexpr int kTreeAutoSegs = 512;  // automatic hierarchy: faces with a chain at least this long

struct FaceTab {
    const int32_t* seg_begin;  // [F+1] segments of face f are [seg_begin[f], seg_begin[f+1])
    const int32_t* order;      // [F] faces sorted by segment count, descending
    int32_t num_faces;
};

struct Points {
    const double* u;
    const double* v;
    int64_t stride;
    const int64_t* offs;  // [F+1] device
    int64_t n;
};

struct NearQueue {
    uint2* qs;                     // [cap] (query index, segment index)
    double2* shift;                // [cap] translation of the segment copy (periodic faces), or nullptr
    unsigned long long* count;     // device counter (may exceed cap: overflow pairs are done in line)
    uint64_t cap;
};

// Periodic faces (Sec. 4.3-4.5).  Segments of periodic faces are stored
// lifted (translated by their lattice offsets) after creation.
struct PLoop {
    int32_t s0, s1;       // segments
    int32_t h0, h1;       // homology
    double vx, vy;        // lifted end - lifted start
    double dx, dy, lv;    // unit tangent of v, |v|
    double b0x, b0y;      // lifted start
    double xi_lo, xi_hi;  // tangent extent of lifted control points relative to b0
    double bb[4];         // lifted control-point box umin, umax, vmin, vmax
};

enum { kUnitExtended = 1, kUnitContractible = 2, kUnitPair = 3 };

struct PUnit {
    int32_t kind;
    int32_t la, lb;          // loop(s): extended curve / contractible loop / pair (alpha, beta)
    int32_t pad;
    double pshx, pshy;       // translation of the paired beta copy
    double eta_lo, eta_hi;   // normal extent of the pair relative to alpha's start
};

struct PFace {
    int32_t dom, u0, u1, pad;  // domain, units [u0, u1)
    double Tu, Tv;             // periods
    double t1x, t1y;           // family step t_1 (torus)
    double Delta, nx, ny;      // family spacing and left normal of h* (T_u, T_v) (torus)
    double offset;             // constant added to the winding number (punctured sphere / cone), turns
};

// Domains periodic in u only: the cylinder and the punctured sphere / cone.
inline __host__ __device__ bool u_periodic_only(int dom) { return dom == 1 || dom == 3 || dom == 4; }

struct PerTab {
    const PLoop* loop;   // [L]
    const PUnit* unit;   // [U]
    const PFace* face;   // [F]
    const uint8_t* seg_periodic;  // [S] 1 for segments of periodic faces
};

struct LiftArgs {
    const int32_t* loops;      // loop ids to lift
    int32_t nloops;
    const int32_t* loop_face;  // [L]
    const int32_t* face_dom;   // [F]
    const double* face_per;    // [2F]
    const int32_t* loop_seg;   // [L+1]
    const int64_t* seg_cp;     // [S+1]
    const double* cpu;         // raw control points
    const double* cpv;
    double* seg_off;           // [2S] out: lattice offset per segment
    PLoop* out;                // [L]
};

struct Stats {
    unsigned long long* c;  // device [8] or nullptr
};

struct Out {
    double* w;      // [N] omega (or angle accumulator in the batched path)
    uint8_t* lab;   // [N] label (or on-boundary flag in the batched path)
    uint8_t* depth; // optional depth log
    int32_t depth_stride;
    int32_t rule;
};

}  // namespace wn

// Kernel launchers (wn_kernels.hip).
namespace wn {
hipError_t launch_build_items(const FaceTab& ft, const Points& pts, int qpw, int32_t* item_offs, int2* item_map,
                              int64_t map_cap, uint32_t* counters, bool zero_near, hipStream_t st);
hipError_t launch_far(bool inline_near, bool mixed, int qpw, const Segs& sg, const FaceTab& ft, const Points& pts,
                      const int32_t* item_offs, const int2* item_map, uint32_t* item_counter, int32_t single_face,
                      int64_t grid, NearQueue nq, Out out, double eps2, hipStream_t st);
// Near pass over queue entries [*q_lo, *q_hi) (nullptr: 0 / the queue's count).
// Near pass over queue entries [q_lo, q_hi) (defaults: 0 and the queue's
// count).  cursor (nullable, zero at launch): waves take chunks of entries
// from it (dynamic balance); without it each wave takes one equal share.
hipError_t launch_near(const Segs& sg, const Points& pts, NearQueue nq, Out out, double eps2, int64_t grid,
                       Stats stats, const uint8_t* seg_per, uint8_t* entry_depth, hipStream_t st,
                       const unsigned long long* q_lo = nullptr, const unsigned long long* q_hi = nullptr,
                       unsigned long long* cursor = nullptr);
// The same pass with the subdivided control-point bound (WN_BOUND_SUBDIVIDED).
hipError_t launch_near_cp(const Segs& sg, const Points& pts, NearQueue nq, Out out, double eps2, int64_t grid,
                          Stats stats, const uint8_t* seg_per, uint8_t* entry_depth, hipStream_t st,
                          const unsigned long long* q_lo, const unsigned long long* q_hi, unsigned long long* cursor);
hipError_t launch_queue_mark(const unsigned long long* count, unsigned long long* mark, hipStream_t st);
// Queue entries [0, n) -> their query and segment indices (diagnostics).
hipError_t launch_split_pairs(const uint2* qs, int64_t n, int32_t* point, int32_t* segment, hipStream_t st);
hipError_t launch_finalize(const Points& pts, Out out, int64_t q0, int64_t q1, int32_t nf, hipStream_t st);
hipError_t launch_redo(const Segs& sg, const FaceTab& ft, const Points& pts, Out out, double eps2,
                       const NearQueue& nq, int64_t max_grid, hipStream_t st);
int far_blocks_per_cu(bool inline_near, bool mixed, int qpw);
// Queued FP64 far pass over the path hierarchy (items of 256 queries).
hipError_t launch_far_tree(const PathTree& tr, const FaceTab& ft, const Points& pts, const int32_t* item_offs,
                           const int2* item_map, uint32_t* item_counter, int64_t grid, NearQueue nq, Out out,
                           double eps2, hipStream_t st, bool skip_ordered = false);
int far_tree_blocks_per_cu();
// The same hierarchy walked once per wave over spatially ordered queries
// (perm, from launch_spatial_order), four queries per lane, items of 1024
// queries; faces with more than kOrderMaxPoints points are skipped (they keep
// the caller's order: launch_far_tree with skip_ordered takes them).
hipError_t launch_far_wtree(const PathTree& tr, const FaceTab& ft, const Points& pts, const uint32_t* perm,
                            const int32_t* item_offs, const int2* item_map, uint32_t* item_counter, int64_t grid,
                            NearQueue nq, Out out, double eps2, hipStream_t st);
int far_wtree_blocks_per_cu();
constexpr int kWtreeQPL = 4;
// Queued FP64 far pass with qpl (2, 3 or 4) queries per lane (items of 256 qpl
// queries), over the items of the faces of rank [rank_lo, rank_hi) of ft
// (rank_hi < 0: all faces).
hipError_t launch_farq(int qpl, const Segs& sg, const FaceTab& ft, const Points& pts, const int32_t* item_offs,
                       const int2* item_map, uint32_t* item_counter, int64_t grid, NearQueue nq, Out out, double eps2,
                       hipStream_t st, int rank_lo = 0, int rank_hi = -1);
int farq_blocks_per_cu(int qpl);
int near_blocks_per_cu();
int near_cp_blocks_per_cu();
hipError_t launch_lift(const LiftArgs& a, Segs sg_mut, hipStream_t st);

// One torus face for the pairing kernel: A = lists[a0 .. a0 + na), B =
// lists[b0 .. b0 + nb) (loop indices, nb <= 64), choices written to
// out[out0 .. out0 + na) as (index into B or -1, family m of the shift m t_1).
struct PairJob {
    int32_t a0, na, b0, nb, out0, pad;
    double t1x, t1y, nx, ny, Delta;
    double eta;  // axis inflation of the probes' ellipse tests
};
hipError_t launch_pair_torus(const Segs& sg, const PLoop* loops, const PairJob* jobs, int njobs, const int32_t* lists,
                             int2* out, double eps2, hipStream_t st);
// Periodic far pass variants: near pairs queued (overflow -> label kRedo),
// recursed in line, or recursed in line for the kRedo-labelled queries only.
// stat_pairs (optional): adds the (query, segment copy) pairs of the copy
// windows of the valid queries.
enum : int { kPerQueue = 0, kPerInline = 1, kPerRedo = 2 };
hipError_t launch_far_periodic(int mode, const Segs& sg, const FaceTab& ft, const Points& pts,
                               const int32_t* item_offs, const int2* item_map, uint32_t* item_counter, int64_t grid,
                               NearQueue nq, Out out, double eps2, PerTab pt, const uint32_t* perm, hipStream_t st,
                               unsigned long long* stat_pairs = nullptr);
// Spatial order of the points of every face of ft (one workgroup per face):
// perm[slot] = point index; perm == nullptr in launch_far_periodic = identity.
hipError_t launch_spatial_order(const FaceTab& ft, const Points& pts, uint32_t* perm, hipStream_t st);
int far_periodic_blocks_per_cu(int mode);
}  // namespace wn
