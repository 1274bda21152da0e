/* CPU oracle for batched generalized-winding-number containment queries.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library; the product path (the
 * HIP library) neither links nor calls it, and the two share no source,
 * header, table or helper.  Plain C11 + pthreads, FP64 throughout (a long
 * double twin of the planar routine serves as a brute-force cross-check).
 *
 * What is computed, per query point x of face f:
 *   omega(x) = sum over the face's (lifted) segment copies of
 *              (1/2pi) * integral d(theta)                        (Sec. 3.2)
 * Planar faces: every loop, every segment (additivity, Sec. 3.2 eq. 1),
 * each segment by hull-bounded de Casteljau flattening (see the core file).
 * Periodic faces: the covering-space formulation of Sec. 4.3-4.5 (cylinder:
 * contractible copies + periodically extended curves, Eq. of Sec. 4.4;
 * torus: A/B/C split of the Proposition in Sec. 4.5 and band sums over
 * families of lifted copies, Eq. bandWN), written out in windowed form.
 *
 * near flag: 1 when the point is within `near_tol` of some curve (certified by
 * branch and bound on de Casteljau pieces) or when that could not be decided;
 * 0 when its distance to every curve (copy) is certified >= near_tol.
 *
 * Alg. 1 depth mirror (wn_oracle_alg1.inc): the recursion of Alg. 1 itself,
 * run per (query, segment) pair in FP64 to report the depth, split and leaf
 * counts the method reaches (pinned by exact rational arithmetic on small
 * curves and by the distance bounds of the termination argument).
 *
 * parity: the planar routine is pinned by closed forms, the long double
 * twin and quadrature; the periodic routine by closed-form straight bands on
 * cylinders and tori, lattice-translation, seam re-cutting and window
 * widening invariants.  parity unpinned: the pairing of wavy loops whose
 * normal ranges interleave (checked only through the 0/1 postcondition).
 */
#include <limits.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXDEG 5
#define ORC_MAXCP (ORC_MAXDEG + 1)
#define ORC_MAXDEPTH 64
#define ORC_PI 3.14159265358979323846264338327950288L

typedef struct {
    int32_t num_faces, num_loops, num_segments;
    int64_t num_cps;
    const int32_t* face_loop_offsets;
    const int32_t* loop_seg_offsets;
    const int64_t* seg_cp_offsets;
    const double *cp_u, *cp_v, *cp_w;
    const int32_t* face_domain;
    const double* face_period;
} orc_faces;

/* ---- FP64 instance ---------------------------------------------------- */
#define REAL double
#define SFX _d
#define R_SQRT sqrt
#define R_ATAN2 atan2
#define R_FABS fabs
#define R_EPS 1.1102230246251565e-16
#define R_DELTA 1e-12
#include "wn_oracle_core.inc"
#undef REAL
#undef SFX
#undef R_SQRT
#undef R_ATAN2
#undef R_FABS
#undef R_EPS
#undef R_DELTA

/* ---- long double instance (brute cross-check) ------------------------- */
#define REAL long double
#define SFX _ld
#define R_SQRT sqrtl
#define R_ATAN2 atan2l
#define R_FABS fabsl
#define R_EPS 5.42101086242752217e-20L
#define R_DELTA 1e-15L
#include "wn_oracle_core.inc"
#undef REAL
#undef SFX
#undef R_SQRT
#undef R_ATAN2
#undef R_FABS
#undef R_EPS
#undef R_DELTA

/* ------------------------------------------------------------------------
 * Certified distance test: is the distance from x to the segment below tol?
 * Branch and bound on de Casteljau pieces.  Lower bound of a piece: distance
 * from x to the axis-aligned box of its control points (the piece lies in the
 * hull, hence in the box).  Upper bound: distance to the piece's end points
 * (points of the curve).  Returns 1 (d < tol), 0 (d >= tol), or 2 (undecided).
 * ---------------------------------------------------------------------- */
static double box_dist(double x, double y, const double* px, const double* py, int m) {
    double lox = px[0], hix = px[0], loy = py[0], hiy = py[0];
    for (int i = 1; i < m; ++i) {
        lox = fmin(lox, px[i]); hix = fmax(hix, px[i]);
        loy = fmin(loy, py[i]); hiy = fmax(hiy, py[i]);
    }
    double dx = x < lox ? lox - x : (x > hix ? x - hix : 0.0);
    double dy = y < loy ? loy - y : (y > hiy ? y - hiy : 0.0);
    return sqrt(dx * dx + dy * dy);
}

static int segment_near(double x, double y, const double* cu, const double* cv, const double* cw, int n, double tol) {
    piece_d stack[2 * ORC_MAXDEPTH + 4];
    int sp = 0;
    piece_d root;
    root.n = n;
    root.depth = 0;
    for (int i = 0; i <= n; ++i) {
        double w = cw ? cw[i] : 1.0;
        root.W[i] = w; root.X[i] = w * cu[i]; root.Y[i] = w * cv[i];
    }
    {
        double px[ORC_MAXCP], py[ORC_MAXCP];
        project_d(&root, px, py);
        /* slack covers the rounding of the projection */
        if (box_dist(x, y, px, py, n + 1) >= tol * (1 + 1e-9) + 1e-15) return 0;
    }
    stack[sp++] = root;
    int undecided = 0;
    while (sp > 0) {
        piece_d p = stack[--sp];
        double px[ORC_MAXCP], py[ORC_MAXCP];
        project_d(&p, px, py);
        double up = fmin(hypot(px[0] - x, py[0] - y), hypot(px[n] - x, py[n] - y));
        if (up < tol * (1 - 1e-9)) return 1;
        double lo = box_dist(x, y, px, py, n + 1);
        if (lo >= tol * (1 + 1e-9) + 1e-15) continue;
        if (p.depth >= 60) { undecided = 1; continue; }
        piece_d l, r;
        split_half_d(&p, &l, &r);
        stack[sp++] = r;
        stack[sp++] = l;
    }
    return undecided ? 2 : 0;
}

/* ------------------------------------------------------------------------
 * Per-face evaluation.  Periodic domains are implemented in the periodic
 * section below; face_eval dispatches.
 * ---------------------------------------------------------------------- */
static int planar_near(const orc_faces* fc, int f, double x, double y, double tol) {
    int res = 0;
    int l0 = fc->face_loop_offsets[f], l1 = fc->face_loop_offsets[f + 1];
    for (int l = l0; l < l1; ++l) {
        for (int s = fc->loop_seg_offsets[l]; s < fc->loop_seg_offsets[l + 1]; ++s) {
            int64_t c0 = fc->seg_cp_offsets[s];
            int n = (int)(fc->seg_cp_offsets[s + 1] - c0) - 1;
            int r = segment_near(x, y, fc->cp_u + c0, fc->cp_v + c0, fc->cp_w ? fc->cp_w + c0 : NULL, n, tol);
            if (r == 1) return 1;
            if (r == 2) res = 1;
        }
    }
    return res;
}

#include "wn_oracle_periodic.inc"
#include "wn_oracle_alg1.inc"

/* ------------------------------------------------------------------------
 * Threaded driver
 * ---------------------------------------------------------------------- */
typedef struct {
    const orc_faces* fc;
    int64_t n;
    const int32_t* pf;
    const double *pu, *pv;
    double tol;
    int use_ld;
    double* out_w;
    int8_t* out_near;
    int64_t next;
    int status;
} job_t;

static void eval_point(job_t* J, int64_t i) {
    const orc_faces* fc = J->fc;
    int f = J->pf[i];
    double x = J->pu[i], y = J->pv[i];
    if (!(isfinite(x) && isfinite(y))) {
        J->out_w[i] = NAN;
        if (J->out_near) J->out_near[i] = 1;
        return;
    }
    int dom = fc->face_domain ? fc->face_domain[f] : 0;
    int near_flag = 0;
    double w;
    if (dom == 0) {
        if (J->use_ld) {
            w = (double)face_winding_planar_ld(fc, f, (long double)x, (long double)y, &near_flag);
        } else {
            w = face_winding_planar_d(fc, f, x, y, &near_flag);
        }
        if (J->out_near) J->out_near[i] = (int8_t)(planar_near(fc, f, x, y, J->tol) ? 1 : 0);
    } else {
        int st = periodic_eval(fc, f, x, y, J->tol, &w, J->out_near ? &J->out_near[i] : NULL);
        if (st != 0) J->status = st;
    }
    J->out_w[i] = w;
}

static void* worker(void* arg) {
    job_t* J = (job_t*)arg;
    const int64_t chunk = 64;
    for (;;) {
        int64_t s = __atomic_fetch_add(&J->next, chunk, __ATOMIC_RELAXED);
        if (s >= J->n) break;
        int64_t e = s + chunk < J->n ? s + chunk : J->n;
        for (int64_t i = s; i < e; ++i) eval_point(J, i);
    }
    return NULL;
}

/* Evaluate `num_points` queries; point i belongs to face point_face[i].
 * Returns 0 on success, a negative value on invalid input, or a periodic
 * topology error code (see wn_oracle_periodic.inc). */
int wno_query(int32_t num_faces, const int32_t* face_loop_offsets, int32_t num_loops,
              const int32_t* loop_seg_offsets, int32_t num_segments, const int64_t* seg_cp_offsets,
              const double* cp_u, const double* cp_v, const double* cp_w, const int32_t* face_domain,
              const double* face_period, int64_t num_points, const int32_t* point_face, const double* pu,
              const double* pv, double near_tol, int32_t nthreads, int32_t use_long_double, double* out_w,
              int8_t* out_near) {
    orc_faces fc = {num_faces, num_loops, num_segments, seg_cp_offsets[num_segments], face_loop_offsets,
                    loop_seg_offsets, seg_cp_offsets, cp_u, cp_v, cp_w, face_domain, face_period};
    for (int32_t s = 0; s < num_segments; ++s) {
        int64_t n = seg_cp_offsets[s + 1] - seg_cp_offsets[s] - 1;
        if (n < 1 || n > ORC_MAXDEG) return -1;
    }
    for (int64_t i = 0; i < num_points; ++i)
        if (point_face[i] < 0 || point_face[i] >= num_faces) return -2;
    int pst = periodic_prepare(&fc);
    if (pst != 0) {
        periodic_release(&fc);
        return pst;
    }
    job_t J = {&fc, num_points, point_face, pu, pv, near_tol, use_long_double, out_w, out_near, 0, 0};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&th[started], NULL, worker, &J) == 0) ++started;
    worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    periodic_release(&fc);
    return J.status;
}

/* Test knobs of the periodic formulation: widen every copy/family window by
 * `extra` on each side; pair each alpha with the unshifted beta instead of
 * its nearest left copy (negative control). */
void wno_set_periodic_options(int32_t extra, int32_t disable_pairing) {
    g_window_extra = extra < 0 ? 0 : extra;
    g_disable_pairing = disable_pairing != 0;
}

/* Winding of a single planar segment (radians / 2pi) seen from (x, y);
 * used by the tests for per-segment closed forms. */
double wno_segment_winding(const double* cu, const double* cv, const double* cw, int32_t degree, double x,
                           double y, int32_t use_long_double, int32_t* near) {
    int nr = 0;
    double r;
    if (use_long_double) {
        ksum_ld acc = {0, 0};
        segment_angle_ld((long double)x, (long double)y, cu, cv, cw, degree, &acc, &nr);
        r = (double)((acc.s + acc.c) / (2 * ORC_PI));
    } else {
        ksum_d acc = {0, 0};
        segment_angle_d(x, y, cu, cv, cw, degree, &acc, &nr);
        r = (acc.s + acc.c) / (2 * (double)ORC_PI);
    }
    if (near) *near = nr;
    return r;
}
