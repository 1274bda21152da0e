/* wn.h - batched generalized-winding-number containment queries on trimmed
 * surfaces, MI355X (gfx950).
 *
 * The problem (Sec. 4.1): given a query point x = (u, v) in the parameter
 * domain of a trimmed surface and the surface's trimming loops (p-curves,
 * Sec. 3.1) made of (rational) Bezier segments, decide whether x lies in the
 * trimmed region.  The library computes the generalized winding number
 * omega(x) = (1/2pi) * integral of d(theta) along the loops (Sec. 3.2) with the
 * recursive ellipse-bound algorithm (Alg. 1, Sec. 4.1-4.2), lifts loops of
 * periodic domains to the universal covering space (Sec. 4.3-4.5) and rounds
 * omega to inside/outside.
 *
 * Conventions
 *  - Every call returns a wn_status; WN_OK is 0.  No C++ exception crosses
 *    this interface.  Host-side validation errors are reported synchronously
 *    and leave outputs untouched.
 *  - "host" pointers are read during the call only; the caller keeps
 *    ownership.  "device" pointers are HIP device memory owned by the caller
 *    (for instance torch tensors); the library never frees them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Query work is enqueued on it and is asynchronous: outputs are valid once
 *    the stream reaches that point.  wn_create_faces synchronizes (it reads
 *    back the covering-space lift of periodic faces); so do the calls that
 *    say so below (the application drivers, which upload their tables once,
 *    and the diagnostics).  The queries themselves (wn_query, wn_query_ex,
 *    wn_query_noalloc, plan replays) never synchronize.
 *  - A wn_faces handle is immutable after creation: concurrent wn_query calls
 *    on different streams with the same handle are safe.  Each call allocates
 *    its own stream-ordered scratch memory.
 *  - With WN_FLAG_OVERLAP and host offsets (face_point_offsets_host), the
 *    batched FP64 schedule runs near passes of early face runs on a second
 *    stream that the handle owns (default priority), forked from `stream` and
 *    joined back to it
 *    before the call's work on `stream` ends, so ordering on `stream` holds as
 *    for any other call.  Concurrent calls on one handle share that stream:
 *    their side passes then run one after another, with the same results.
 */
#ifndef WN_H
#define WN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WN_OK = 0,
    WN_E_INVALID = 1,     /* malformed descriptor or argument                  */
    WN_E_NOMEM = 2,       /* device or host allocation failed                  */
    WN_E_DEVICE = 3,      /* a HIP call failed                                 */
    WN_E_TOPOLOGY = 4,    /* periodic loops violate the Proposition of Sec. 4.5 */
    WN_E_DEPTH = 5,       /* recursion depth bound exceeds the stack cap       */
    WN_E_UNSUPPORTED = 6  /* option combination not provided                   */
} wn_status;

/* Parameter domain of a face (Sec. 3.1, Sec. 4.3). */
typedef enum {
    WN_DOMAIN_PLANE = 0,      /* simply connected rectangle                  */
    WN_DOMAIN_CYLINDER_U = 1, /* periodic in u with period T_u (uni-periodic)  */
    WN_DOMAIN_TORUS = 2,      /* periodic in u and v (bi-periodic)             */
    /* Sphere- and cone-like: periodic in u with singular points (poles, apex)
     * at the ends of the v range.  The singular points are punctured, which
     * leaves the cylinder case (Sec. 4.3): loops that run around a pole are
     * non-contractible (h = (+-1, 0)) and no pole edge is given.  The face's
     * winding number is the cylinder's plus one constant c per face, chosen
     * so that every region between the non-contractible loops gets 0 or 1:
     * c = S/2 - m, S the sum of their h_u and m the least partial sum of
     * their h_u taken from the lowest loop up (a cap around one pole:
     * c = 1/2; a band: c = 0; both caps: c = 1).  A face whose regions would
     * span more than one unit is WN_E_TOPOLOGY. */
    WN_DOMAIN_SPHERE_U = 3,
    WN_DOMAIN_CONE_U = 4
} wn_domain;

/* Arithmetic of the root ellipse test of planar faces (Alg. 1; the
   recursion, the angle and crossing sums and periodic faces are always FP64).
   MIXED admits a pair as far when FP32 distances exceed the ellipse's axis by
   a relative 2^-20 margin, which certifies the FP64 decision, and falls back
   to the FP64 test otherwise: its results equal FP64's bit for bit. */
typedef enum {
    WN_PREC_FP64 = 0,  /* every step in FP64                                    */
    WN_PREC_MIXED = 1  /* FP32 certified far-field admission, FP64 fallback      */
} wn_precision;

/* Rounding of omega to a label (Sec. 4.1: "classify based on this value"). */
typedef enum {
    WN_RULE_NONZERO = 0,  /* inside iff |omega| > 1/2 */
    WN_RULE_POSITIVE = 1  /* inside iff omega > 1/2   */
} wn_rule;

/* How query work is scheduled on the GPU. */
typedef enum {
    WN_SCHED_PLAIN = 0,   /* one launch per face, near pairs recursed in line      */
    WN_SCHED_BATCHED = 1, /* one persistent work-queue launch over all faces;
                             near pairs compacted into a queue, recursed after    */
    WN_SCHED_BINNED = 2   /* BATCHED, near queue ordered by predicted depth        */
} wn_schedule;

/* Output labels written to out_inside. */
enum {
    WN_OUTSIDE = 0,
    WN_INSIDE = 1,
    WN_ON_BOUNDARY = 2, /* Alg. 1 met an evaluated curve point within eps     */
    WN_INVALID_POINT = 3 /* non-finite query coordinates                       */
};

/* Face descriptor: CSR faces -> loops -> segments -> control points.
 * All pointers are HOST pointers, copied during wn_create_faces. */
typedef struct {
    int32_t num_faces, num_loops, num_segments;
    int64_t num_cps;
    const int32_t* face_loop_offsets; /* [num_faces+1], loops of face f are [o[f], o[f+1])       */
    const int32_t* loop_seg_offsets;  /* [num_loops+1], segments of a loop, in path order         */
    const int64_t* seg_cp_offsets;    /* [num_segments+1], degree = count - 1, 1..5                */
    const double* cp_u;               /* [num_cps] control point u                                */
    const double* cp_v;               /* [num_cps] control point v                                */
    const double* cp_w;               /* [num_cps] weights > 0, or NULL for non-rational curves    */
    const int32_t* face_domain;       /* [num_faces] wn_domain, or NULL = all planar               */
    const double* face_period;        /* [2*num_faces] (T_u, T_v); read for periodic faces only    */
} wn_faces_desc;

typedef struct {
    double eps;        /* on-boundary tolerance of Alg. 1 (default 1e-10), in [1e-15, 1e-2] */
    int32_t precision; /* wn_precision (default WN_PREC_FP64)                              */
    int32_t rule;      /* wn_rule (default WN_RULE_NONZERO)                                 */
    int32_t schedule;  /* wn_schedule (default WN_SCHED_BATCHED)                            */
    int32_t stack_cap; /* largest accepted depth bound ceil(log2(B/eps))+3 (default 52, max 52) */
    int32_t flags;     /* WN_FLAG_* bits (default 0)                                         */
} wn_options;

/* wn_options.flags */
enum {
    /* Pair the loops of torus faces on the host instead of the GPU (the same
     * pairing rule, App. C; kept for comparison).  By default the pairing
     * runs on the GPU, one wave per torus face (faces with more than 64
     * loops in B always pair on the host). */
    WN_FLAG_HOST_PAIRING = 1,
    /* Let batched FP64 queries given host offsets run the near passes of
     * early face runs on a second stream beside the far pass of later runs
     * (see the conventions above).  Off by default: with the far pass's
     * queue appends batched, the far and near passes take about equal time
     * and both are instruction-bound, and the overlapped passes measured
     * slower than the passes in series on every workload here. */
    WN_FLAG_OVERLAP = 2
};

/* Query points, grouped by face: the points of face f are
 * [face_point_offsets[f], face_point_offsets[f+1]). */
typedef struct {
    int64_t num_points;
    const double* u;                       /* device, element i at u[i*stride]                 */
    const double* v;                       /* device, element i at v[i*stride]                 */
    int64_t stride;                        /* >= 1; 1 = separate arrays, 2 = interleaved (u,v) */
    const int64_t* face_point_offsets;     /* device [num_faces+1], non-decreasing, last = num_points */
    const int64_t* face_point_offsets_host;/* host copy of the same, or NULL (then the plain
                                              schedule builds its face tiles on the device
                                              and the batched one runs its passes in series) */
} wn_points;

typedef struct wn_faces wn_faces; /* opaque; owns all device copies */

/* Kernel timing: a pool of HIP event pairs recorded on the query stream
 * around each kernel the library launches (no allocation while recording). */
typedef struct wn_profile wn_profile;
enum {
    WN_KERNEL_ITEMS = 0,
    WN_KERNEL_FAR = 1,
    WN_KERNEL_NEAR = 2,
    WN_KERNEL_FINALIZE = 3,
    WN_KERNEL_REDO = 4,
    WN_KERNEL_FAR_PERIODIC = 5,
    WN_KERNEL_BIN = 6,
    WN_KERNEL_KINDS = 8
};

/* Learned depth predictor: an MLP 16 -> 64 -> 64 -> 1 (ReLU; BF16 weights,
 * FP32 accumulation; FP32 master weights for training) that predicts the
 * recursion depth Alg. 1 reaches on a near pair (root ellipse test failed)
 * from 16 features of the pair, used to order the near queue into
 * uniform-depth bins (WN_SCHED_BINNED).  Binning never changes results. */
typedef struct wn_predictor wn_predictor;
#define WN_MLP_IN 16
#define WN_MLP_HIDDEN 64
#define WN_MLP_PARAMS (WN_MLP_IN * WN_MLP_HIDDEN + WN_MLP_HIDDEN + WN_MLP_HIDDEN * WN_MLP_HIDDEN + WN_MLP_HIDDEN + WN_MLP_HIDDEN + 1)
/* Where WN_SCHED_BINNED takes the depth of each near pair from. */
enum {
    WN_BIN_PREDICTOR = 0, /* the MLP on the matrix cores: BF16 weights, inputs and hidden
                             activations, FP32 accumulation (v_mfma_f32_16x16x32_bf16);
                             falls back to WN_BIN_NONE without a predictor              */
    WN_BIN_HEURISTIC = 1, /* ceil(log2(B / max(eps, distance from the query to the chord))) */
    WN_BIN_MEASURED = 2,  /* depths measured by a first, discarded near pass (upper bound) */
    WN_BIN_NONE = 3,      /* no reordering (the unbinned queue) */
    WN_BIN_PREDICTOR_VALU = 4 /* the MLP as FP32 VALU dot products on BF16-rounded weights
                                 (the comparison version of WN_BIN_PREDICTOR)           */
};

/* Per-call overrides and diagnostics (all fields optional: 0/NULL = default). */
typedef struct {
    int32_t schedule;        /* -1 = the handle's default, else wn_schedule               */
    int32_t precision;       /* -1 = the handle's default, else wn_precision              */
    int32_t rule;            /* -1 = the handle's default, else wn_rule                   */
    int32_t queries_per_wg;  /* 0 = tuned; else 64, 128 or 256 queries per workgroup, or 512 /
                                768 / 1024 (two / three / four per lane: FP64 batched/binned
                                far pass; otherwise 256)                                   */
    int32_t queue_policy;    /* 0 = tuned, 1 = persistent workgroups popping an atomic work
                                queue, 2 = one workgroup per work item (batched schedules)  */
    int64_t near_capacity;   /* 0 = default (8 * num_points + 65536) near-queue entries    */
    uint8_t* depth_log;      /* device [num_points * max_segments_per_face] or NULL.  Entry
                                i * max_segments_per_face + j receives the deepest level Alg. 1
                                reached for point i against segment j of its face (0 = decided
                                at the whole segment).  Written by WN_SCHED_PLAIN only.     */
    wn_profile* profile;     /* NULL, or a profile that records kernel durations            */
    unsigned long long* stats; /* NULL, or device [WN_STATS_COUNT] counters the batched
                                  schedules ADD to (zero them first): see WN_STAT_*          */
    const wn_predictor* predictor; /* WN_SCHED_BINNED with WN_BIN_PREDICTOR                  */
    int32_t bin_source;      /* WN_BIN_* (WN_SCHED_BINNED only)                             */
    int32_t path_hierarchy;  /* 0 = every (point, segment) pair of a planar face is tested
                                (default); 1 = the path hierarchy of Sec. 4.2 prunes subpaths
                                whose ellipse bound excludes the point (batched and binned
                                schedules, FP64; the near pairs, hence the recursion, are
                                the same; points within eps of a vertex inside a pruned
                                subpath are classified instead of reported on-boundary);
                                2 = automatic: the hierarchy for faces with a chain of at
                                least 512 joined segments, the flat scan for the others   */
    int32_t bound;           /* WN_BOUND_GLOBAL (default): a node [a, b] of Alg. 1 has the
                                axis B (b - a) (Sec. 4.2); WN_BOUND_SUBDIVIDED: the smaller of
                                that and the Lemma 1 / App. A.1 bound of the node's own
                                control points (de Casteljau halving, the control-point bound
                                Table 1 contrasts): fewer or equal splits, the same omega.
                                Applies to the near pass of the batched and binned schedules
                                (in-line recursions keep the global bound)                  */
} wn_query_opts;

enum { WN_BOUND_GLOBAL = 0, WN_BOUND_SUBDIVIDED = 1 };

/* Work counters of the batched schedules (wn_query_opts.stats). */
enum {
    WN_STAT_NEAR_PAIRS = 0,   /* pairs whose root ellipse test failed (queued)           */
    WN_STAT_SPLITS = 1,       /* Alg. 1 nodes split (one midpoint evaluation each)       */
    WN_STAT_LEAVES = 2,       /* Alg. 1 leaves (one chord angle each)                    */
    WN_STAT_REEVALS = 3,      /* pending end points re-evaluated after an LDS slot reuse */
    WN_STAT_NEAR_FLOPS = 4,   /* algorithmic FP64 flops of the near pass (cost model:
                                 split 6n+15, leaf 11; n = segment degree)                */
    WN_STAT_MAX_DEPTH = 5,    /* deepest level reached (max, not sum)                    */
    WN_STAT_NEAR_STEPS = 6,   /* near pass: loop trips summed over its waves             */
    WN_STAT_NEAR_LANE_STEPS = 7, /* near pass: lanes holding a pair, summed over trips    */
    WN_STAT_PERIODIC_PAIRS = 8,  /* periodic far pass: (query, segment copy) pairs in the
                                    copy windows of the valid queries (Sec. 4.3-4.5)      */
    WN_STATS_COUNT = 9
};

/* Fill `opt` with the defaults listed above.  Never fails. */
void wn_default_options(wn_options* opt);
void wn_default_query_opts(wn_query_opts* q);

/* Validate `desc` (CSR monotone, degrees 1..5, finite coordinates with
 * |coordinate| < 1e30, weights > 0, periods > 0 for periodic faces), compute
 * each segment's derivative bound B (Lemma 1 and App. A.1; the minimum of the
 * two rational bounds), check the depth bound ceil(log2(B/eps))+3 against
 * opt->stack_cap (WN_E_DEPTH), pack structure-of-arrays device copies and, for
 * periodic faces, lift the loops to the covering space and pair them
 * (Sec. 4.3-4.5; WN_E_TOPOLOGY when the loops of a torus face cannot be split
 * into A, B, C with |A| = |B|).  `opt` may be NULL (defaults).  On success
 * *out owns the device data; release it with wn_destroy_faces.  Synchronizes
 * `stream`. */
wn_status wn_create_faces(const wn_faces_desc* desc, const wn_options* opt, void* stream, wn_faces** out);

/* The containment query of Sec. 4.1 (Alg. 1 per point-segment pair, with
 * the root ellipse test of Lemma 1 and the sub-segment bound of Sec. 4.2;
 * the periodic sums of Sec. 4.3-4.5 for periodic faces): omega and label for
 * every query point against the loops of its face (points grouped by face,
 * wn_points.face_point_offsets).  out_winding: device double [num_points]
 * (NaN for on-boundary and invalid points); out_inside: device uint8
 * [num_points], one of WN_OUTSIDE/INSIDE/ON_BOUNDARY/INVALID_POINT (inside
 * means |omega| > 1/2, or omega > 1/2 under WN_RULE_POSITIVE).  Either output
 * may be NULL.  Asynchronous on `stream`; per-call scratch is stream-ordered
 * (hipMallocAsync / hipFreeAsync on `stream`).  WN_E_INVALID for malformed
 * points or offsets (checked on the host when host offsets are given). */
wn_status wn_query(const wn_faces* faces, const wn_points* points, double* out_winding, uint8_t* out_inside,
                   void* stream);

/* wn_query (Sec. 4.1, Alg. 1) with per-call overrides of the handle's
 * schedule, precision and rule, work counters, profiling and the plain
 * schedule's depth log (`q` may be NULL: the handle's defaults). */
wn_status wn_query_ex(const wn_faces* faces, const wn_points* points, double* out_winding, uint8_t* out_inside,
                      const wn_query_opts* q, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): wn_query_ex
 * with the batched schedule, whose scratch (work items, counters, near queue,
 * spatial order of the points of periodic faces and, with path_hierarchy, of
 * planar faces) lives in a fixed device array of
 * wn_query_noalloc_scratch_bytes() bytes (64 MiB) that the library holds on
 * each device it runs on until the process ends.  No allocation of any kind
 * is made.  The near queue gets whatever the array has left; pairs that do
 * not fit are recomputed in line, so results equal wn_query_ex's.
 *   out_winding, out_inside  device outputs, both required (not NULL)
 *   limits                   num_points <= WN_NOALLOC_MAX_POINTS and the
 *                            handle's faces <= WN_NOALLOC_MAX_FACES, else
 *                            WN_E_INVALID; a schedule other than batched
 *                            (q->schedule or the handle's) gives
 *                            WN_E_UNSUPPORTED
 * Every call on a device shares that device's array (it keeps the last call's
 * contents, and nothing in it has to start at zero): calls that overlap in
 * time on one device race, so issue them on one stream per device.  The
 * device is the handle's.  Asynchronous on `stream`. */
#define WN_NOALLOC_MAX_POINTS (1 << 22)
#define WN_NOALLOC_MAX_FACES (1 << 18)
wn_status wn_query_noalloc(const wn_faces* faces, const wn_points* points, double* out_winding, uint8_t* out_inside,
                           const wn_query_opts* q, void* stream);
int64_t wn_query_noalloc_scratch_bytes(void);

/* Release a handle (waits for nothing: the caller must not destroy a handle
 * that queued work still uses).  NULL is ignored. */
void wn_destroy_faces(wn_faces* faces);

/* Static text for a status code. */
const char* wn_status_string(wn_status s);

/* Host-only helpers (no device access; usable without a GPU). */

/* Derivative bound B of one segment (Lemma 1, App. A.1): non-rational
 * n * max_i |P_i - P_{i-1}|; rational min(n (W/w) max_{i,j} |P_i - P_j|,
 * n (W/w)^2 max_i |P_i - P_{i-1}|).  cp_w may be NULL.  Returns WN_E_INVALID
 * for degree outside 1..5 or non-positive weights. */
wn_status wn_segment_bound(const double* cp_u, const double* cp_v, const double* cp_w, int32_t degree,
                           double* out_B);

/* NURBS p-curve to (rational) Bezier segments (Sec. 3.1: B-spline and NURBS
 * curves subdivide into Bezier segments): every interior knot is inserted
 * (Boehm's rule, in homogeneous coordinates) until its multiplicity equals
 * the degree; each knot span of nonzero length is then one segment.
 *   degree       1..5
 *   num_cps      degree + 1 <= n <= 16384; cp_u, cp_v [n]; cp_w [n] weights > 0 (finite),
 *                or NULL for a non-rational B-spline (out_w is then not written)
 *   knots        [n + degree + 1], non-decreasing and clamped: the first and the
 *                last value each repeated exactly degree + 1 times, U[degree] < U[n]
 *   out_cap      capacity of out_u, out_v (and out_w) in points
 *   out_u/v/w    segment i's control points are entries i*degree .. i*degree +
 *                degree (neighbours share their joint), so k segments fill
 *                k*degree + 1 points; the joints coincide with the curve's
 *                points at the knots
 *   out_segments number of segments k (also set when out_cap is too small,
 *                which returns WN_E_INVALID without writing the outputs)
 * Host-only, all pointers host.  WN_E_INVALID for malformed arguments. */
wn_status wn_nurbs_to_bezier(int32_t degree, int32_t num_cps, const double* knots, const double* cp_u,
                             const double* cp_v, const double* cp_w, int64_t out_cap, double* out_u, double* out_v,
                             double* out_w, int32_t* out_segments);

/* Applications of Sec. 5.4 on the same query pipeline. */

/* A uniform grid over a face's parameter rectangle: nu x nv cells of size
 * du x dv whose lower-left corner is (u0, v0). */
typedef struct {
    double u0, v0; /* lower-left corner (finite)                 */
    double du, dv; /* cell size (finite, > 0)                    */
    int32_t nu, nv; /* cells along u and along v (>= 0)           */
} wn_grid;

/* Tessellation driver (Sec. 5.4.3: the sample points of a uniform grid in
 * the parameter domain are classified so that the cells outside the trimmed
 * region can be removed, periodic faces included).  Classifies the cell
 * centres of grids[f] against face f for every face.
 *   grids        host [num_faces]; the total number of cells must be < 2^31 - 1
 *   samples      face by face, row-major inside a face (i along u fastest):
 *                cell (i, j) of face f is sample sum_{g<f} nu_g nv_g + j nu_f + i,
 *                at u = u0 + (i + 0.5) du, v = v0 + (j + 0.5) dv, the product and
 *                the sum each rounded once (no fused multiply-add)
 *   out_u, out_v device double [samples], receive the sample coordinates; if
 *                either is NULL the library stages them in its own memory
 *   out_winding, out_inside  device [samples], as in wn_query (either may be NULL)
 *   q            per-call overrides as in wn_query_ex (may be NULL)
 * Uploads the grid table and synchronizes `stream` once before launching
 * anything; the rest is asynchronous on `stream` (staging freed
 * stream-ordered).  WN_E_INVALID for malformed grids, WN_E_NOMEM when the
 * staging memory cannot be allocated, otherwise as wn_query_ex. */
wn_status wn_classify_grid(const wn_faces* faces, const wn_grid* grids, double* out_u, double* out_v,
                           double* out_winding, uint8_t* out_inside, const wn_query_opts* q, void* stream);

/* Multi-patch classification (Sec. 5.4.1: a point sampled on a base surface
 * is inside when it lies inside any trimmed face that references the
 * surface).  Surface s is referenced by the faces
 * surface_faces[surface_face_offsets[s] .. surface_face_offsets[s+1]) (host
 * arrays; each face belongs to at most one surface; faces of no surface are
 * not queried).  `points` holds the sample points grouped by SURFACE: its
 * offsets have num_surfaces + 1 entries and the host copy
 * (face_point_offsets_host) is required.
 *   out_inside   device uint8 [num_points] or NULL: WN_INSIDE if some face of
 *                the point's surface labels it inside, else WN_ON_BOUNDARY if
 *                some face does, else WN_INVALID_POINT for invalid coordinates,
 *                else WN_OUTSIDE (also for every point of a surface with no face)
 *   out_face     device int32 [num_points] or NULL: the first face in the
 *                surface's list that labels the point inside, or -1
 * The points are copied once per referencing face (face-major staging of
 * 17 bytes per copy; copies in total < 2^31 - 1) and queried in one call.
 * Uploads the tables and synchronizes `stream` once before launching
 * anything; the rest is asynchronous on `stream`.  WN_E_INVALID for
 * malformed tables, otherwise as wn_classify_grid. */
wn_status wn_classify_surfaces(const wn_faces* faces, int32_t num_surfaces, const int32_t* surface_face_offsets,
                               const int32_t* surface_faces, const wn_points* points, uint8_t* out_inside,
                               int32_t* out_face, const wn_query_opts* q, void* stream);

/* Faces whose loops are chains of NURBS p-curves (Sec. 3.1: B-Rep trimming
 * curves are NURBS; they subdivide into Bezier segments).  All pointers HOST.
 *   face_loop_offsets  [num_faces+1]  faces -> loops
 *   loop_curve_offsets [num_loops+1]  loops -> ordered curves
 *   curve_degree       [num_curves]   1..5
 *   curve_cp_offsets   [num_curves+1] curves -> control points (int64)
 *   knots              the curves' clamped knot vectors back to back: curve c
 *                      owns (cp count + degree + 1) entries, starting where
 *                      curve c-1's end
 *   cp_u, cp_v         control points; cp_w weights or NULL (non-rational)
 *   face_domain, face_period  as in wn_faces_desc */
typedef struct {
    int32_t num_faces;
    int32_t num_loops;
    int32_t num_curves;
    int64_t num_cps;    /* entries of cp_u, cp_v (and cp_w): must equal curve_cp_offsets[num_curves] */
    int64_t num_knots;  /* entries of knots: must equal the sum of (cp count + degree + 1) */
    const int32_t* face_loop_offsets;
    const int32_t* loop_curve_offsets;
    const int32_t* curve_degree;
    const int64_t* curve_cp_offsets;
    const double* knots;
    const double* cp_u;
    const double* cp_v;
    const double* cp_w;
    const int32_t* face_domain;
    const double* face_period;
} wn_nurbs_faces_desc;

/* wn_create_faces for NURBS loops: every curve is split into Bezier segments
 * by wn_nurbs_to_bezier (knot insertion), in order, and the segments replace
 * the curve in its loop; then as wn_create_faces.  WN_E_INVALID for
 * malformed tables or curves (the conditions of wn_nurbs_to_bezier). */
wn_status wn_create_faces_nurbs(const wn_nurbs_faces_desc* desc, const wn_options* opt, void* stream,
                                wn_faces** out);

/* Create a profile able to time `capacity` kernel launches (events are
 * created here, on the current device).  Timing a launch beyond the capacity
 * is skipped silently. */
wn_status wn_profile_create(int32_t capacity, wn_profile** out);
/* Wait for every recorded launch, then report per kernel kind (index
 * WN_KERNEL_*) the number of timed launches and their summed duration in
 * milliseconds (arrays of WN_KERNEL_KINDS entries, host).  Also resets the
 * profile for reuse. */
wn_status wn_profile_collect(wn_profile* p, int64_t* launches, double* total_ms);
void wn_profile_destroy(wn_profile* p);

/* Training options (0 = default in brackets) and report. */
typedef struct {
    int32_t epochs;       /* [8] passes over the samples                                   */
    int32_t batch;        /* [4096] samples per AdamW step                                 */
    float lr;             /* [2e-3] AdamW learning rate                                    */
    float weight_decay;   /* [1e-4] decoupled weight decay                                 */
    float huber_delta;    /* [1.0] Huber loss threshold                                    */
    float holdout;        /* [0.1] fraction of samples kept out of training for the report */
    int32_t seed;         /* shuffling seed                                                */
    int64_t max_samples;  /* [0 = all] cap on the near pairs used                          */
} wn_train_opts;

typedef struct {
    int64_t samples;        /* near pairs collected (root ellipse test failed)            */
    int64_t train_samples;
    int32_t steps;
    float final_train_loss; /* mean Huber loss of the last epoch                          */
    float holdout_mae;      /* mean |predicted - measured depth| on the holdout            */
    float baseline_mae;     /* same, predicting the training mean depth (no network)       */
    float heuristic_mae;    /* same, predicting the analytic heuristic                     */
    float mean_depth;       /* training mean depth                                         */
} wn_train_report;

/* Create a predictor with weights drawn from a seeded He-uniform
 * initialisation (host, deterministic) and uploaded to the current device. */
wn_status wn_predictor_create(int32_t seed, wn_predictor** out);
void wn_predictor_destroy(wn_predictor* p);

/* Collect every near pair of `points` against `faces` (batched far pass),
 * measure its depth with the near pass itself (labels), build the features,
 * standardise them, and train the MLP on the GPU (forward, backward, AdamW
 * kernels).  Synchronous.  `opts` and `report` may be NULL. */
wn_status wn_predictor_train(wn_predictor* p, const wn_faces* faces, const wn_points* points,
                             const wn_train_opts* opts, wn_train_report* report, void* stream);

/* FP32 master parameters (host [WN_MLP_PARAMS], layout W1[64][16], b1[64],
 * W2[64][64], b2[64], w3[64], b3) and the feature standardisation (host
 * [2 * WN_MLP_IN]: means then standard deviations).  set_* also refreshes
 * the BF16 copy. */
wn_status wn_predictor_get_params(const wn_predictor* p, float* params, float* feature_norm);
wn_status wn_predictor_set_params(wn_predictor* p, const float* params, const float* feature_norm);

/* Mean Huber loss and its gradient with respect to the FP32 master
 * parameters over n standardised feature rows (device [n][16]) and labels
 * (device [n]); forward in BF16-rounded weights as in inference.  Host
 * outputs; synchronous.  (Gradient checks.) */
wn_status wn_predictor_loss_grad(const wn_predictor* p, const float* features, const float* labels, int64_t n,
                                 float huber_delta, float* loss, float* grad, void* stream);

/* Predicted depth for n standardised feature rows (device in/out): FP32
 * VALU dot products on the BF16-rounded weights. */
wn_status wn_predictor_predict(const wn_predictor* p, const float* features, int64_t n, float* out, void* stream);

/* The same on the matrix cores: the inputs and the layer-1 activations are
 * rounded to BF16 on their way into v_mfma_f32_16x16x32_bf16 (weights stored
 * as BF16), accumulation in FP32; persistent waves of 64 rows per step.
 * features must be 16-byte aligned (WN_E_INVALID otherwise). */
wn_status wn_predictor_predict_mfma(const wn_predictor* p, const float* features, int64_t n, float* out,
                                    void* stream);

/* Raw (unstandardised) features of given (point, segment) pairs: pair k is
 * point pair_point[k] of `points` against segment pair_segment[k] (global
 * index, as lifted for periodic faces) -> device [n][16].  pair_point,
 * pair_segment: device int32 [n].  Features: query in the ellipse frame
 * (2, in units of B/2), semi-axes B/2 and sqrt((B/2)^2 - (L/2)^2), degree,
 * min/max weight, chord length L, distance to the control-point box, the two
 * end-point distances, (d1+d2)/B, log2(B/max(eps, box distance)), B, L/2, the
 * side of the chord. */
wn_status wn_pair_features(const wn_faces* faces, const wn_points* points, const int32_t* pair_point,
                           const int32_t* pair_segment, int64_t n, float* out, void* stream);

/* The near pairs of a query and the depth Alg. 1 reaches on each (Sec. 4.1,
 * Alg. 1; depth as in wn_query_opts.depth_log: the deepest tested level,
 * 0 = the whole segment).  Runs the batched FP64 far pass and the near pass
 * of the batched schedule, with its passes in series, and copies out the
 * near-pair queue: pair k is point pair_point[k] of `points` against global
 * segment pair_segment[k], whose depth is pair_depth[k].  The queue's order
 * follows the far pass's scheduling, not the points' order.
 *   capacity       entries the outputs hold (>= 0)
 *   pair_point, pair_segment  device int32 [capacity]; pair_depth device uint8
 *                  [capacity]; pair_shift device double [capacity][2] or NULL:
 *                  the translation subtracted from the point for a periodic
 *                  copy (zero for planar pairs)
 *   out_count      host: the number of near pairs (entries beyond capacity are
 *                  not written)
 *   bound          WN_BOUND_GLOBAL or WN_BOUND_SUBDIVIDED: the near pass's node
 *                  bound (wn_query_opts.bound)
 * Diagnostics and training data: allocates its scratch and synchronizes
 * `stream`.  WN_E_NOMEM when the near pairs exceed the internal queue
 * (8 N + 65536 entries, or capacity if larger). */
wn_status wn_near_pairs(const wn_faces* faces, const wn_points* points, int64_t capacity, int32_t* pair_point,
                        int32_t* pair_segment, uint8_t* pair_depth, double* pair_shift, int64_t* out_count,
                        int32_t bound, void* stream);

/* Plans: a preallocated batched query captured once into a HIP graph.  The
 * caller owns the point buffers (`points`: device u, v with stride, device
 * per-face offsets; points->num_points is the capacity) and the outputs
 * (device, capacity entries), which must outlive the plan.  Before each
 * launch the caller writes any number of points up to the capacity and their
 * per-face offsets (offsets[num_faces] = live count): the kernels read the
 * live count from the offsets.  The plan allocates its scratch once;
 * launching allocates nothing.  Launches that overlap on one plan race (they
 * share its scratch).  `q` selects the schedule (WN_SCHED_BATCHED or
 * WN_SCHED_BINNED) and tiling; q->profile, q->stats and q->depth_log must be
 * NULL.  The faces handle (and a predictor given in q) must outlive the plan. */
typedef struct wn_plan wn_plan;
wn_status wn_plan_create(const wn_faces* faces, const wn_points* points, double* out_winding, uint8_t* out_inside,
                         const wn_query_opts* q, void* stream, wn_plan** out);
/* Replay the captured graph on `stream` (asynchronous). */
wn_status wn_plan_launch(wn_plan* p, void* stream);
/* Autotuner: time every (points per workgroup in {64, 128, 256, 512, 1024})
 * x (queue policy in {persistent, one workgroup per item}) on the plan's
 * current buffers (`reps` runs each, HIP-event timed), keep the fastest and
 * re-capture the graph.  Synchronous.  report (host, nullable, 12 doubles):
 * average milliseconds in the order (64,p), (64,w), (128,p), (128,w),
 * (256,p), (256,w), (512,p), (512,w), (1024,p), (1024,w), then the chosen
 * points per workgroup and policy. */
wn_status wn_plan_autotune(wn_plan* p, int32_t reps, void* stream, double* report);
void wn_plan_destroy(wn_plan* p);

/* Summary of a created handle (host copy of sizes). */
typedef struct {
    int32_t num_faces, num_loops, num_segments;
    int32_t num_periodic_faces;
    int32_t max_segments_per_face;
    int32_t max_depth_bound;   /* largest ceil(log2(B/eps))+3 over segments */
    int64_t device_bytes;      /* device memory held by the handle */
} wn_faces_info;
wn_status wn_get_faces_info(const wn_faces* faces, wn_faces_info* info);

/* Pair table of torus face `face` (Sec. 4.5, App. C: each loop alpha of A
 * with the loop beta of B whose copy beta + shift lies nearest on alpha's
 * left).  Host-only read of the handle.  Writes up to `cap` pairs: alpha[i],
 * beta[i] (face-set loop indices) and shift[2i], shift[2i+1] (the copy's
 * translation); *count = the face's number of pairs (0 for a face without
 * torus pairs).  WN_E_INVALID for a bad face index or NULL pointers with
 * cap > 0. */
wn_status wn_torus_pairs(const wn_faces* faces, int32_t face, int32_t cap, int32_t* alpha, int32_t* beta,
                         double* shift, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* WN_H */
