/*
 * FP64 reference ("oracle") for closest-hit ray traversal of a constrained
 * tetrahedral mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg are its only users; the library never links, loads or calls
 * it, and it shares no code, header or table with the library.
 *
 * It works on the user's uncompressed arrays:
 *   points  float32 [P][3]  (widened to double, which is exact)
 *   tets    int32   [T][4]  vertex ids
 *   nbrs    int32   [T][4]  tet across the face opposite vertex slot j, -1 = boundary
 *   cflag   uint8   [T][4]  1 = that face is scene geometry ("constrained")
 * No xor records, no reordering, an orthonormal ray frame, double precision.
 *
 * What is computed (paper, Sec. "Tetrahedron Traversal" and its subsections):
 *   - the ray frame: an orthonormal basis (b1, b2) of the plane orthogonal to
 *     the ray direction, built with Duff et al.'s branch-free construction (the
 *     method the paper cites for its basis); a vertex P projects to
 *     ((P-o).b1, (P-o).b2), so the ray is the 2-D origin;
 *   - point location: a straight-line walk from the centroid of a source tet to
 *     the query point (Sec. "Locating points in a tetrahedral mesh");
 *   - the exit face of the start tet: the face the ray line leaves through
 *     (smallest crossing parameter over the faces whose outward normal has a
 *     positive component along the direction); its vertices are kept in
 *     counter-clockwise order in the 2-D frame;
 *   - the walk: the fourth vertex of the next tet is fetched and projected,
 *     Algorithm 1 ("GetExitFace") picks which of the three kept vertices to
 *     replace, the neighbour across the remaining face is next; the walk stops
 *     at a constrained face (hit) or the mesh boundary (miss);
 *   - the hit: t along d as given and barycentric weights of the hit face.
 * Conventions that the paper leaves open (canonical triangle ids, tmax, error
 * codes, the start-face rule for secondary rays) are stated at each function.
 *
 * Per-ray result codes in out_tri: >= 0 triangle id, -1 miss, -3 invalid ray
 * or origin outside the mesh, -4 the mesh violated the face-connected chain
 * invariant during the walk.
 *
 * Degenerate rays.  In exact arithmetic every face the walk keeps contains the
 * ray: its projection holds the 2-D origin (all three edge determinants
 * det(q_i, q_i+1) of the counter-clockwise face are >= 0).  In floating point
 * this can only break where Algorithm 1 meets a zero determinant decided by
 * rounding: a mesh vertex lies on the ray (a ray through a vertex, or running
 * along a tet edge, whose endpoints both project onto the 2-D origin).  The
 * walk may then circle, or leave the ray altogether and end on a face the ray
 * never meets.  Both are detected -- a walk longer than T steps (a straight
 * line enters each tet at most once), or a kept face whose projection misses
 * the origin by more than rounding can explain (an edge determinant below
 * -1e-9 E (|q_i|_1 + |q_i+1|_1), E the extent of the mesh) -- and such a ray
 * takes the plain definition instead: the closest of all constrained
 * triangles it meets (Moller-Trumbore, inclusive edges), with steps = -1.
 *
 * Build: cc -O2 -ffp-contract=off -fPIC -shared walk.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

typedef struct { double x, y, z; } v3;

static v3 vsub(v3 a, v3 b) { v3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static v3 vadd(v3 a, v3 b) { v3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static v3 vscale(v3 a, double s) { v3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 vcross(v3 a, v3 b) {
    v3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}

typedef struct {
    int64_t np, nt, ntri;
    double extent;       /* largest side of the points' bounding box */
    const float* pts;
    const int32_t* tets;
    const int32_t* nbrs;
    const uint8_t* cflag;
    int32_t* face_tri;   /* [nt*4]: canonical triangle id of face (t, j) or -1 */
    int32_t* tri_tets;   /* [ntri*2]: the tets on the two sides (second may be -1) */
    int32_t* tri_verts;  /* [ntri*3]: vertex ids, ascending */
    char err[256];
} omesh;

static v3 point(const omesh* m, int32_t i) {
    v3 r = {(double)m->pts[3 * (int64_t)i], (double)m->pts[3 * (int64_t)i + 1],
            (double)m->pts[3 * (int64_t)i + 2]};
    return r;
}

/* ---- mesh set-up -------------------------------------------------------- */

/* Canonical triangle ids: walk the faces (t, j) in user order, t-major, and give
 * each constrained face a new id the first time it is seen; the same face seen
 * from the neighbouring tet gets the same id.  (The paper only says that the
 * neighbour field of a constrained face refers to a record holding the scene
 * triangle and the two adjacent tets.) */
void* oracle_mesh_new(const float* pts, int64_t np, const int32_t* tets,
                      const int32_t* nbrs, const uint8_t* cflag, int64_t nt,
                      char* err, int64_t errlen) {
    omesh* m = (omesh*)calloc(1, sizeof(omesh));
    if (!m) return NULL;
    m->np = np; m->nt = nt; m->pts = pts; m->tets = tets; m->nbrs = nbrs; m->cflag = cflag;
    for (int a = 0; a < 3; ++a) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t i = 0; i < np; ++i) {
            double c = (double)pts[3 * i + a];
            if (c < lo) lo = c;
            if (c > hi) hi = c;
        }
        if (np > 0 && hi - lo > m->extent) m->extent = hi - lo;
    }
    m->face_tri = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)(nt > 0 ? nt : 1));
    int64_t nflag = 0;
    for (int64_t k = 0; k < 4 * nt; ++k) { m->face_tri[k] = -1; nflag += cflag[k] != 0; }
    m->tri_tets = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(nflag + 1));
    m->tri_verts = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(nflag + 1));
    int64_t ntri = 0;
    for (int64_t t = 0; t < nt && !m->err[0]; ++t) {
        for (int j = 0; j < 4; ++j) {
            int64_t fj = 4 * t + j;
            if (!cflag[fj] || m->face_tri[fj] >= 0) continue;
            int32_t f[3]; int k = 0;
            for (int s = 0; s < 4; ++s) if (s != j) f[k++] = tets[4 * t + s];
            int32_t id = (int32_t)ntri++;
            m->face_tri[fj] = id;
            int32_t nb = nbrs[fj];
            m->tri_tets[2 * id] = (int32_t)t;
            m->tri_tets[2 * id + 1] = nb;
            /* ascending vertex ids */
            for (int a = 0; a < 3; ++a)
                for (int b = a + 1; b < 3; ++b)
                    if (f[b] < f[a]) { int32_t tmp = f[a]; f[a] = f[b]; f[b] = tmp; }
            memcpy(&m->tri_verts[3 * id], f, sizeof f);
            if (nb < 0) continue;
            /* the mirror slot: the vertex of nb that is not on the face */
            int mirror = -1, matches = 0;
            for (int s = 0; s < 4; ++s) {
                int32_t v = tets[4 * (int64_t)nb + s];
                if (v == f[0] || v == f[1] || v == f[2]) ++matches; else mirror = s;
            }
            if (matches != 3 || mirror < 0 || nbrs[4 * (int64_t)nb + mirror] != (int32_t)t ||
                !cflag[4 * (int64_t)nb + mirror]) {
                snprintf(m->err, sizeof m->err,
                         "face (%lld,%d) is not mirrored consistently by tet %d",
                         (long long)t, j, nb);
                break;
            }
            m->face_tri[4 * (int64_t)nb + mirror] = id;
        }
    }
    m->ntri = ntri;
    if (m->err[0]) {
        if (err && errlen > 0) { strncpy(err, m->err, (size_t)errlen - 1); err[errlen - 1] = 0; }
        free(m->face_tri); free(m->tri_tets); free(m->tri_verts); free(m);
        return NULL;
    }
    return m;
}

void oracle_mesh_free(void* h) {
    omesh* m = (omesh*)h;
    if (!m) return;
    free(m->face_tri); free(m->tri_tets); free(m->tri_verts); free(m);
}

int64_t oracle_mesh_ntri(void* h) { return ((omesh*)h)->ntri; }

/* Copy out the canonical tables: face_tri [T*4], tri_tets [ntri*2], tri_verts [ntri*3]. */
void oracle_mesh_tables(void* h, int32_t* face_tri, int32_t* tri_tets, int32_t* tri_verts) {
    omesh* m = (omesh*)h;
    if (face_tri) memcpy(face_tri, m->face_tri, sizeof(int32_t) * 4 * (size_t)m->nt);
    if (tri_tets) memcpy(tri_tets, m->tri_tets, sizeof(int32_t) * 2 * (size_t)m->ntri);
    if (tri_verts) memcpy(tri_verts, m->tri_verts, sizeof(int32_t) * 3 * (size_t)m->ntri);
}

/* ---- 2-D primitives ------------------------------------------------------ */

static double det2(const double a[2], const double b[2]) { return a[0] * b[1] - a[1] * b[0]; }

/* Algorithm 1 (exit face selection).  q[0..2] is the face the ray entered
 * through, counter-clockwise around the 2-D origin; q[3] the new vertex.
 * Returns the index (0..2) of the kept vertex that the exit face does not
 * contain, i.e. the slot the new vertex replaces. */
static int get_exit_face(const double q[4][2]) {
    if (det2(q[3], q[0]) < 0.0) {
        if (det2(q[3], q[2]) >= 0.0) return 1;
        return 0;
    }
    if (det2(q[3], q[1]) < 0.0) return 2;
    return 0;
}

/* Whether the kept face q[0..2] (counter-clockwise) misses the 2-D origin by
 * more than rounding can explain: the walk has left the ray (see the header). */
static int face_misses_ray(const double q[4][2], double extent) {
    for (int i = 0; i < 3; ++i) {
        const double* a = q[i];
        const double* b = q[(i + 1) % 3];
        double tol = 1e-9 * extent * (fabs(a[0]) + fabs(a[1]) + fabs(b[0]) + fabs(b[1]));
        if (det2(a, b) < -tol) return 1;
    }
    return 0;
}

int oracle_get_exit_face(const double* q8) {
    double q[4][2];
    for (int i = 0; i < 4; ++i) { q[i][0] = q8[2 * i]; q[i][1] = q8[2 * i + 1]; }
    return get_exit_face(q);
}

/* Duff et al.'s orthonormal basis for a unit vector n: the two tangents come
 * from one reciprocal and a sign, with no branch on the smallest component.
 * (b1, b2, n) is right-handed. */
static void onb(v3 n, v3* b1, v3* b2) {
    double sgn = n.z >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sgn + n.z);
    double b = n.x * n.y * a;
    b1->x = 1.0 + sgn * n.x * n.x * a; b1->y = sgn * b; b1->z = -sgn * n.x;
    b2->x = b; b2->y = sgn + n.y * n.y * a; b2->z = -n.y;
}

void oracle_onb(const double* n, double* b1, double* b2) {
    v3 nn = {n[0], n[1], n[2]}, u, v;
    onb(nn, &u, &v);
    b1[0] = u.x; b1[1] = u.y; b1[2] = u.z;
    b2[0] = v.x; b2[1] = v.y; b2[2] = v.z;
}

typedef struct { v3 o, d, b1, b2; double dd; } frame;

static void project(const frame* f, v3 p, double q[2]) {
    v3 r = vsub(p, f->o);
    q[0] = vdot(r, f->b1);
    q[1] = vdot(r, f->b2);
}

/* parameter along d (as given) of the orthogonal projection of p on the ray */
static double depth(const frame* f, v3 p) { return vdot(vsub(p, f->o), f->d) / f->dd; }

/* ---- 3-D helpers (start of a walk) --------------------------------------- */

/* Face opposite slot j of tet t, ordered so that (B-A) x (C-A) points out of the tet. */
static void outward_face(const omesh* m, int32_t t, int j, int32_t f[3], v3* nrm) {
    int k = 0;
    for (int s = 0; s < 4; ++s) if (s != j) f[k++] = m->tets[4 * (int64_t)t + s];
    v3 A = point(m, f[0]), B = point(m, f[1]), C = point(m, f[2]);
    v3 W = point(m, m->tets[4 * (int64_t)t + j]);
    v3 n = vcross(vsub(B, A), vsub(C, A));
    if (vdot(n, vsub(W, A)) > 0.0) {
        int32_t tmp = f[1]; f[1] = f[2]; f[2] = tmp;
        n = vscale(n, -1.0);
    }
    *nrm = n;
}

/* Slot of the face through which the line X + s*D leaves tet t (the smallest
 * crossing parameter among faces whose outward normal has n.D > 0) and that
 * parameter; -1 when no face is front-facing (D = 0). */
static int convex_exit(const omesh* m, int32_t t, v3 X, v3 D, double* s_out) {
    int best = -1;
    double bs = INFINITY;
    for (int j = 0; j < 4; ++j) {
        int32_t f[3]; v3 n;
        outward_face(m, t, j, f, &n);
        double nd = vdot(n, D);
        if (!(nd > 0.0)) continue;
        double s = vdot(n, vsub(point(m, f[0]), X)) / nd;
        if (s < bs) { bs = s; best = j; }
    }
    *s_out = bs;
    return best;
}

static v3 centroid(const omesh* m, int32_t t) {
    v3 c = {0, 0, 0};
    for (int s = 0; s < 4; ++s) c = vadd(c, point(m, m->tets[4 * (int64_t)t + s]));
    return vscale(c, 0.25);
}

/* Point location by a straight-line walk from the centroid S of the source tet
 * toward x: in each tet the segment leaves through the face found by
 * convex_exit; once that crossing lies at or beyond x (parameter >= 1) the
 * current tet contains x.  Returns the tet, -1 if the segment leaves the mesh
 * (x outside), -2 at the step cap.  Constrained faces are crossed like any
 * other face: location ignores scene geometry. */
static int32_t locate_one(const omesh* m, v3 x, int32_t src, int64_t cap) {
    int32_t t = src;
    v3 S = centroid(m, t);
    v3 D = vsub(x, S);
    for (int64_t it = 0; it < cap; ++it) {
        double s;
        int j = convex_exit(m, t, S, D, &s);
        if (j < 0 || s >= 1.0) return t;
        int32_t nb = m->nbrs[4 * (int64_t)t + j];
        if (nb < 0) return -1;
        t = nb;
    }
    return -2;
}

int oracle_locate(void* h, int64_t n, const float* xyz, int32_t source_tet, int32_t* out) {
    omesh* m = (omesh*)h;
    if (source_tet < 0 || source_tet >= m->nt) return -1;
    for (int64_t i = 0; i < n; ++i) {
        v3 x = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
        out[i] = locate_one(m, x, source_tet, 4 * m->nt + 4);
    }
    return 0;
}

/* ---- the definition: closest hit over all constrained triangles ---------- */

/* Moller-Trumbore with inclusive edges over every triangle; t in (0, tmax],
 * the start face excluded; ties within 1e-12 go to the lowest id.  Returns the
 * id or -1 and fills t, the weights of the 2nd and 3rd vertex (ascending ids),
 * and the tets in front of / behind the face along the ray. */
static int32_t closest_by_definition(const omesh* m, const frame* F, double tm, int32_t exclude,
                                     double* t_out, double bary[2], int32_t tets2[2]) {
    int32_t best = -1;
    double bt = INFINITY, bu = NAN, bv = NAN;
    for (int64_t f = 0; f < m->ntri; ++f) {
        if (f == exclude) continue;
        const int32_t* tv = &m->tri_verts[3 * f];
        v3 A = point(m, tv[0]), B = point(m, tv[1]), C = point(m, tv[2]);
        v3 e1 = vsub(B, A), e2 = vsub(C, A);
        v3 pv = vcross(F->d, e2);
        double det = vdot(e1, pv);
        if (det == 0.0) continue;
        v3 sv = vsub(F->o, A);
        double u = vdot(sv, pv) / det;
        v3 qv = vcross(sv, e1);
        double v = vdot(F->d, qv) / det;
        double t = vdot(e2, qv) / det;
        if (u < 0.0 || v < 0.0 || u + v > 1.0 || !(t > 0.0) || t > tm) continue;
        if (t < bt - 1e-12 || (fabs(t - bt) <= 1e-12 && f < best)) {
            if (t < bt) bt = t;
            best = (int32_t)f; bu = u; bv = v;
        }
    }
    tets2[0] = tets2[1] = -1;
    if (best >= 0) {
        /* the ray goes from the tet on one side of the face to the other */
        const int32_t* tv = &m->tri_verts[3 * (int64_t)best];
        v3 A = point(m, tv[0]);
        v3 nf = vcross(vsub(point(m, tv[1]), A), vsub(point(m, tv[2]), A));
        int32_t ta = m->tri_tets[2 * (int64_t)best], tb = m->tri_tets[2 * (int64_t)best + 1];
        int32_t w = -1;
        for (int s = 0; s < 4; ++s) {
            int32_t x = m->tets[4 * (int64_t)ta + s];
            if (x != tv[0] && x != tv[1] && x != tv[2]) w = x;
        }
        int ta_ahead = (vdot(nf, vsub(point(m, w), A)) > 0.0) == (vdot(nf, F->d) > 0.0);
        tets2[0] = ta_ahead ? tb : ta;
        tets2[1] = ta_ahead ? ta : tb;
    }
    *t_out = bt;
    bary[0] = bu;
    bary[1] = bv;
    return best;
}

/* ---- the walk ------------------------------------------------------------ */

/* Trace n rays.  Per ray i:
 *   orig, dir   float32 [n][3]; the hit point is orig + t*dir
 *   tmax        float32 [n] or NULL (= +inf); a hit counts when t <= tmax
 *   start_face  int32 [n] or NULL: >= 0 = the ray leaves from that constrained
 *               triangle and starts in the adjacent tet on the side dir points
 *               into (secondary rays; the start face itself is never reported)
 *   start_tet   int32 [n] or NULL: >= 0 = a tet known to contain the origin
 *   otherwise the origin is located from source_tet.
 *   early_out   1 = stop once every vertex of the face about to be crossed has
 *               a depth beyond tmax (the crossing point cannot be nearer than
 *               its nearest vertex, so this never changes a result)
 * Outputs: out_tri (id or code), out_t, out_bary [n][2] (weights of the 2nd and
 * 3rd vertex of the hit triangle in ascending vertex-id order), and optionally
 * out_tets [n][2] (tet on the ray's side of the hit face, tet beyond it),
 * out_steps (tets whose record the walk loaded after the start), out_start
 * (the start tet). */
int oracle_trace(void* h, int64_t n, const float* orig, const float* dir, const float* tmax,
                 const int32_t* start_face, const int32_t* start_tet, int32_t source_tet,
                 int early_out, int64_t max_steps,
                 int32_t* out_tri, double* out_t, double* out_bary,
                 int32_t* out_tets, int32_t* out_steps, int32_t* out_start) {
    omesh* m = (omesh*)h;
    if (source_tet < 0 || source_tet >= m->nt) return -1;
    if (max_steps <= 0) max_steps = m->nt + 4;
    for (int64_t i = 0; i < n; ++i) {
        frame F;
        F.o.x = orig[3 * i]; F.o.y = orig[3 * i + 1]; F.o.z = orig[3 * i + 2];
        F.d.x = dir[3 * i]; F.d.y = dir[3 * i + 1]; F.d.z = dir[3 * i + 2];
        double tm = tmax ? (double)tmax[i] : INFINITY;
        int32_t code = -1, cur = -1, nxt = -1, a[3] = {-1, -1, -1}, start = -1;
        int cons = 0, slot = -1;
        int64_t steps = 0;
        double q[4][2];
        double tt = NAN, bary[2] = {NAN, NAN};
        int32_t tets2[2] = {-1, -1};

        F.dd = vdot(F.d, F.d);
        double len = sqrt(F.dd);
        if (!(len > 0.0) || !isfinite(len) || !isfinite(F.o.x + F.o.y + F.o.z)) { code = -3; goto done; }
        onb(vscale(F.d, 1.0 / len), &F.b1, &F.b2);

        int32_t sf = start_face ? start_face[i] : -1;
        int32_t st = start_tet ? start_tet[i] : -1;
        if (sf >= 0) {
            if (sf >= m->ntri) { code = -3; goto done; }
            const int32_t* tv = &m->tri_verts[3 * (int64_t)sf];
            v3 A = point(m, tv[0]), B = point(m, tv[1]), C = point(m, tv[2]);
            v3 nf = vcross(vsub(B, A), vsub(C, A));
            double dn = vdot(nf, F.d);
            if (dn == 0.0) { code = -3; goto done; }
            /* the tet on the side the direction points into */
            int32_t ta = m->tri_tets[2 * (int64_t)sf], tb = m->tri_tets[2 * (int64_t)sf + 1];
            int32_t w = -1;
            for (int s = 0; s < 4; ++s) {
                int32_t v = m->tets[4 * (int64_t)ta + s];
                if (v != tv[0] && v != tv[1] && v != tv[2]) w = v;
            }
            double side = vdot(nf, vsub(point(m, w), A));
            start = ((side > 0.0) == (dn > 0.0)) ? ta : tb;
            cur = (start == ta) ? tb : ta;
            if (start < 0) { code = -1; goto done; }
            a[0] = tv[0]; a[1] = tv[1]; a[2] = tv[2];
            for (int k = 0; k < 3; ++k) project(&F, point(m, a[k]), q[k]);
            double o2 = (q[1][0] - q[0][0]) * (q[2][1] - q[0][1]) - (q[1][1] - q[0][1]) * (q[2][0] - q[0][0]);
            if (o2 < 0.0) {
                int32_t ti = a[1]; a[1] = a[2]; a[2] = ti;
                double t0 = q[1][0], t1 = q[1][1];
                q[1][0] = q[2][0]; q[1][1] = q[2][1]; q[2][0] = t0; q[2][1] = t1;
            }
            nxt = start; cons = 0;
        } else {
            if (st >= 0 && st < m->nt) start = st;
            else start = locate_one(m, F.o, source_tet, 4 * m->nt + 4);
            if (start < 0) { code = -3; goto done; }
            double s;
            int j = convex_exit(m, start, F.o, F.d, &s);
            if (j < 0) { code = -3; goto done; }
            v3 nrm;
            outward_face(m, start, j, a, &nrm);
            for (int k = 0; k < 3; ++k) project(&F, point(m, a[k]), q[k]);
            double o2 = (q[1][0] - q[0][0]) * (q[2][1] - q[0][1]) - (q[1][1] - q[0][1]) * (q[2][0] - q[0][0]);
            if (o2 < 0.0) {
                int32_t ti = a[1]; a[1] = a[2]; a[2] = ti;
                double t0 = q[1][0], t1 = q[1][1];
                q[1][0] = q[2][0]; q[1][1] = q[2][1]; q[2][0] = t0; q[2][1] = t1;
            }
            cur = start; slot = j;
            nxt = m->nbrs[4 * (int64_t)start + j];
            cons = m->cflag[4 * (int64_t)start + j] != 0;
        }

        for (;;) {
            if (cons) {  /* hit the face (a0, a1, a2) of tet cur */
                code = m->face_tri[4 * (int64_t)cur + slot];
                tets2[0] = cur; tets2[1] = nxt;
                break;
            }
            if (nxt < 0) { code = -1; break; }
            if (early_out && isfinite(tm)) {
                double d0 = depth(&F, point(m, a[0])), d1 = depth(&F, point(m, a[1])),
                       d2 = depth(&F, point(m, a[2]));
                double dmin = d0 < d1 ? d0 : d1;
                if (d2 < dmin) dmin = d2;
                if (dmin > tm) { code = -1; break; }
            }
            if (steps >= max_steps) {
                code = closest_by_definition(m, &F, tm, sf, &tt, bary, tets2);
                steps = -1;
                goto done;
            }
            ++steps;
            int32_t tet = nxt;
            /* the vertex of tet that is not on the face just crossed */
            int32_t id3 = -1; int matches = 0;
            for (int s = 0; s < 4; ++s) {
                int32_t v = m->tets[4 * (int64_t)tet + s];
                if (v == a[0] || v == a[1] || v == a[2]) ++matches; else id3 = v;
            }
            if (matches != 3) { code = -4; break; }
            project(&F, point(m, id3), q[3]);
            int e = get_exit_face(q);
            int32_t x = a[e];
            int j = -1;
            for (int s = 0; s < 4; ++s) if (m->tets[4 * (int64_t)tet + s] == x) j = s;
            cur = tet; slot = j;
            nxt = m->nbrs[4 * (int64_t)tet + j];
            cons = m->cflag[4 * (int64_t)tet + j] != 0;
            a[e] = id3; q[e][0] = q[3][0]; q[e][1] = q[3][1];
            if (face_misses_ray(q, m->extent)) {
                code = closest_by_definition(m, &F, tm, sf, &tt, bary, tets2);
                steps = -1;
                goto done;
            }
        }

        if (code >= 0) {
            v3 A0 = point(m, a[0]), A1 = point(m, a[1]), A2 = point(m, a[2]);
            /* the ray meets the face plane where the 2-D origin sits; the
             * projection along d is affine, so the 2-D barycentric weights of
             * the origin are the 3-D weights of the hit point */
            double l[3] = {det2(q[1], q[2]), det2(q[2], q[0]), det2(q[0], q[1])};
            double sum = l[0] + l[1] + l[2];
            v3 nf = vcross(vsub(A1, A0), vsub(A2, A0));
            tt = vdot(nf, vsub(A0, F.o)) / vdot(nf, F.d);
            if (tt > tm) {
                code = -1; tt = NAN; tets2[0] = tets2[1] = -1;
            } else {
                /* weights in ascending vertex-id order */
                int ord[3] = {0, 1, 2};
                for (int u = 0; u < 3; ++u)
                    for (int v = u + 1; v < 3; ++v)
                        if (a[ord[v]] < a[ord[u]]) { int tmp = ord[u]; ord[u] = ord[v]; ord[v] = tmp; }
                bary[0] = l[ord[1]] / sum;
                bary[1] = l[ord[2]] / sum;
            }
        }
    done:
        out_tri[i] = code;
        out_t[i] = code >= 0 ? tt : NAN;
        out_bary[2 * i] = code >= 0 ? bary[0] : NAN;
        out_bary[2 * i + 1] = code >= 0 ? bary[1] : NAN;
        if (out_tets) { out_tets[2 * i] = tets2[0]; out_tets[2 * i + 1] = tets2[1]; }
        if (out_steps) out_steps[i] = (int32_t)steps;
        if (out_start) out_start[i] = start;
    }
    return 0;
}
