/*
 * tetrt -- closest-hit ray traversal through a constrained tetrahedral mesh,
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Aman, Demirci, Gudukbay, "Compact Tetrahedralization-based
 * Acceleration Structure for Ray Tracing" (arXiv 2103.02309).  A scene is a
 * tetrahedral mesh whose faces include the scene triangles ("constrained"
 * faces).  A ray starts in the tet containing its origin, repeatedly finds the
 * face through which it leaves the current tet and steps to the neighbour
 * across it, and stops at the first constrained face (its closest hit) or at
 * the mesh boundary (a miss).
 *
 * Conventions shared by every call
 *   - Ids in and out are the caller's: point ids and tet ids index the arrays
 *     given to tetmesh_upload.  The library renumbers internally (space-filling
 *     curve order) and maps back.
 *   - Triangle ids are canonical: the faces (t, j) are visited t-major, j =
 *     0..3, in the caller's numbering, and every constrained face receives the
 *     next id the first time it is seen; the same face seen from its other tet
 *     shares the id.  tetmesh_tri_vertices maps an id to its vertices.
 *   - Device pointers are HIP device memory on the current device; host
 *     pointers are ordinary process memory.  The caller owns every buffer it
 *     passes.  No call allocates per ray batch.
 *   - Work is enqueued on the given HIP stream (NULL = the default stream) and
 *     returns without synchronising.  A handle is read-only after upload, so
 *     traces on different streams may run concurrently.
 *   - Return value: TM_OK, or a negative TM_ERR_* code; tm_last_error() then
 *     describes the first problem found (per calling thread).
 */
#ifndef TETRT_H
#define TETRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes returned by every call */
enum {
    TM_OK = 0,
    TM_ERR_ARG = -1,   /* bad argument (null pointer, size out of range, ...) */
    TM_ERR_MESH = -2,  /* the mesh failed validation */
    TM_ERR_OOM = -3,   /* a device or host allocation failed */
    TM_ERR_HIP = -4    /* a HIP runtime call or kernel launch failed */
};

/* per-ray codes written to tri[] by trace_closest instead of a triangle id */
enum {
    TM_RAY_MISS = -1,     /* no constrained face with t <= tmax, or the ray left the mesh */
    TM_RAY_STEP_CAP = -2, /* the walk reached the step cap (corrupt mesh or a cycle) */
    TM_RAY_INVALID = -3   /* zero or non-finite direction, or origin outside the mesh */
};

/* compact tet record layouts (paper, Sec. "Tetrahedral Mesh Representation") */
enum {
    TM_LAYOUT_TET20 = 0, /* xor of the four vertex ids + four neighbour fields
                            ordered by the id of the vertex they face (20 B/tet) */
    TM_LAYOUT_TET16 = 1, /* xor of the four vertex ids + three neighbour fields each
                            xored with the fourth; the walk decodes the next tet from
                            the previous one (16 B/tet) */
    TM_LAYOUT_TET32N = 2 /* not a layout of the paper: the four neighbour fields + the
                            xor-sum of each neighbour (32 B/tet), so a walk step loads
                            its record and its point together */
};

/* memory order of points and tets (paper, Sec. "Reordering tetrahedral mesh data") */
enum {
    TM_SFC_HILBERT = 0, /* points by position, tets by centroid, 3-D Hilbert key */
    TM_SFC_MORTON = 1,  /* same keys on the Morton (Z-order) curve */
    TM_SFC_NONE = 2     /* keep the caller's order */
};

typedef struct tm_mesh_s* tm_mesh;

/* Options for tetmesh_upload; pass NULL for the defaults (all fields 0 except
 * validate = 1). */
typedef struct {
    int32_t layout;    /* TM_LAYOUT_* */
    int32_t sfc;       /* TM_SFC_* */
    int32_t validate;  /* 1 = check the mesh before packing (recommended) */
    int32_t seed_grid; /* cells per axis of the point-location seed grid; 0 = automatic */
} tm_upload_opts;

/* Sizes of an uploaded mesh (tetmesh_info). */
typedef struct {
    int64_t n_tets;
    int64_t n_points;
    int64_t n_tris;      /* constrained triangles */
    int64_t hot_bytes;   /* bytes of the arrays the walk reads per step: tet records + points */
    int64_t cold_bytes;  /* every other device array of the handle */
    int32_t layout;
    int32_t sfc;
    int32_t seed_grid;
    int32_t reserved;
} tm_info;

/* Options for trace_closest; pass NULL for the defaults (all fields 0). */
typedef struct {
    int32_t max_steps;   /* walk step cap per ray (tets entered); 0 = 65536 */
    int32_t block;       /* threads per block: 64, 128 or 256 (0 = 256) */
    int32_t kernel;      /* 0 = automatic, 1 = one lane per ray, 2 = persistent lanes that
                            take further rays as theirs finish */
    int32_t refill;      /* persistent lanes: finished lanes per wavefront that trigger a
                            refill, 1..64 (0 = 16) */
    int32_t grid_cap;    /* persistent lanes: at most this many blocks (0 = enough blocks
                            to fill every compute unit) */
    int32_t xcds;        /* one lane per ray: number of accelerator dies (XCDs) that get one
                            contiguous range of blocks each; 0 or 1 = off (round-robin
                            placement, which balances the dies) */
    int32_t sort;        /* ray binning before the walk: 0 = automatic (on for batches of at
                            least 2^18 rays that carry tmax), 1 = off, 2 = on.  Inside each
                            chunk of consecutive rays, rays are grouped by quantised
                            direction, then by the low bits of the Morton index of their
                            origin's cell, and traced in that order; the outputs stay at
                            the caller's positions */
    int32_t sort_chunk_log2; /* rays per chunk = 2^this, 10..13 (0 = 12) */
    int32_t sort_cells_log2; /* origin cells per axis = 2^this, 1..7 (0 = 5) */
    int32_t sort_dirq;   /* direction bins per axis, 1..4 (0 = 4) */
    float eps;           /* precision variant, 0 = off.  When > 0 (one lane per ray only), a
                            walk step whose float32 exit-face determinants det(q3, q_i) are
                            within eps * (|q3|_1 + |q_i|_1) of zero recomputes the projections
                            and determinants in float64 from the float32 points, basis and
                            origin; the start tet's exit face is then also found in float64.
                            With the scene extent 1, eps >= 1e-6 covers float32 rounding */
    void* workspace;     /* device scratch for binning, or NULL: the handle then uses (and
                            grows) a workspace of its own, so binned traces on one handle
                            must not overlap in time unless each passes its own */
    int64_t workspace_bytes; /* size of workspace (tetmesh_trace_workspace gives the need) */
    int32_t* fp64_steps; /* device int32 [n_rays] or NULL: out: walk steps decided in float64
                            (0 when eps = 0) */
} tm_trace_opts;

/*
 * tetmesh_upload -- validate, reorder and pack a tetrahedral mesh, copy it to
 * the current HIP device and return a handle.
 *
 * Representation (paper, Sec. "Tetrahedral Mesh Representation"): the caller
 * gives the typical 32-byte form, four vertex ids and four neighbour ids per
 * tet, where neighbour j is the tet across the face opposite vertex j; plus a
 * flag per face marking scene geometry.  The library stores, per tet, the xor
 * of its four vertex ids and its four neighbour fields ordered by the id of the
 * vertex each one faces (the paper's Tet20).  A neighbour field is either a tet
 * id or, when its top bit is set, a reference to a constrained-face record
 * that holds the scene triangle and the two adjacent tets (paper, same
 * section); 0xFFFFFFFF marks the mesh boundary.  TM_LAYOUT_TET16 stores the
 * paper's 16-byte form instead.  Points and tets are reordered
 * along a 3-D space-filling curve (paper, Sec. "Reordering tetrahedral mesh
 * data").
 *
 *   points   host float32 [n_points][3]
 *   tets     host int32   [n_tets][4]  vertex ids in [0, n_points)
 *   nbrs     host int32   [n_tets][4]  tet across the face opposite vertex j; -1 = boundary
 *   cflag    host uint8   [n_tets][4]  nonzero = that face is a scene triangle; must be
 *                                      set on both sides of an interior face
 *   opts     host, nullable
 *   out      host; receives the handle (owns all device memory until tetmesh_free)
 * Limits: 1 <= n_tets <= 214,748,364 (134,217,727 with TM_LAYOUT_TET32N; records
 * are addressed by 32-bit byte offsets), 4 <= n_points <= 268,435,455, fewer
 * than 2^31 - 1 constrained triangles.  Inputs are copied; the caller may free them on return.
 * Errors: TM_ERR_ARG, TM_ERR_MESH (with validate = 1: vertex id out of range,
 * repeated vertex, zero volume, neighbour link not mutual, neighbours not
 * sharing the face, flag set on one side only -- the first offending tet is
 * named in tm_last_error), TM_ERR_OOM, TM_ERR_HIP.  Synchronous.
 */
int tetmesh_upload(const float* points, int64_t n_points, const int32_t* tets,
                   const int32_t* nbrs, const uint8_t* cflag, int64_t n_tets,
                   const tm_upload_opts* opts, tm_mesh* out);

/*
 * trace_closest -- closest constrained face along each ray.
 *
 * Per ray (paper, Sec. "Tetrahedron Traversal"): a 2-D basis orthogonal to the
 * direction, scaled so that its largest components are +-1 (subsection "Point
 * projection using specialized basis", Eq. 1-3), and the projected origin
 * (Sec. "GPU Implementation", Eq. 4-5); the exit face of the start tet; then
 * the walk: the fourth vertex id of the next tet from the xor field, its
 * projection, the exit face by Algorithm 1 and the next tet by the rank of the
 * exit vertex among the tet's vertex ids (Algorithms 4-5), until a constrained
 * face or the boundary.
 *
 *   m           handle from tetmesh_upload
 *   n_rays      0 <= n_rays < 2^31; 0 is a no-op
 *   d_orig      device float32 [n_rays][3]   ray origins
 *   d_dir       device float32 [n_rays][3]   directions (any nonzero length); hit = orig + t*dir
 *   d_tmax      device float32 [n_rays] or NULL (= +inf); a hit counts iff t <= tmax
 *   d_start_tet device int32 [n_rays] or NULL: >= 0 = a tet (caller id) known to contain
 *               the origin; otherwise the origin is located on the device from a seed
 *               grid by a straight-line walk (paper, Sec. "Locating points in a
 *               tetrahedral mesh")
 *   d_start_face device int32 [n_rays] or NULL: >= 0 = the ray leaves from this
 *               triangle and starts in the adjacent tet on the side dir points into
 *               (secondary rays, paper Sec. "Handling Common Ray-tracing
 *               Operations"); takes precedence over d_start_tet.  That triangle is
 *               never reported as the hit.
 *   d_tri       device int32 [n_rays]  out: triangle id, or TM_RAY_* code
 *   d_t         device float32 [n_rays] out: t of the hit (NaN when no hit)
 *   d_bary      device float32 [n_rays][2] out: barycentric weights of the hit
 *               triangle's 2nd and 3rd vertex in ascending caller vertex-id order
 *               (the 1st weight is 1 - sum); NaN when no hit
 *   d_hit_tets  device int32 [n_rays][2] or NULL: out: the tet on the ray's side of
 *               the hit face and the tet beyond it (-1 at the boundary), caller ids
 *   d_steps     device int32 [n_rays] or NULL: out: tets entered by the walk after
 *               its start tet (for start-face rays the start tet is counted)
 *   opts        host, nullable
 *   hip_stream  hipStream_t or NULL
 * Walk arithmetic is float32; t and the barycentric weights of the final face
 * are evaluated in float64.  Errors: TM_ERR_ARG, TM_ERR_HIP (launch failure).
 */
int trace_closest(tm_mesh m, int64_t n_rays, const float* d_orig, const float* d_dir,
                  const float* d_tmax, const int32_t* d_start_tet, const int32_t* d_start_face,
                  int32_t* d_tri, float* d_t, float* d_bary, int32_t* d_hit_tets,
                  int32_t* d_steps, const tm_trace_opts* opts, void* hip_stream);

/*
 * tetmesh_locate -- tet containing each point (paper, Sec. "Locating points in
 * a tetrahedral mesh": a straight-line walk from a source tet, here the seed
 * tet of the point's cell in a uniform grid over the mesh bounds).
 *   0 <= n < 2^31;  d_pts  device float32 [n][3];  d_tet  device int32 [n] out: caller tet id, -1 when
 *   the point is outside the mesh, -2 at the step cap.  A point on a shared face,
 *   edge or vertex gets one of the tets that contain it.
 */
int tetmesh_locate(tm_mesh m, int64_t n, const float* d_pts, int32_t* d_tet, void* hip_stream);

/* tetmesh_trace_workspace -- bytes of device workspace a trace_closest call with
 * these arguments needs (0 when it bins no rays).  d_tmax_present: the d_tmax
 * argument of that call (only tested for NULL).  *bytes host out. */
int tetmesh_trace_workspace(tm_mesh m, int64_t n_rays, const float* d_tmax_present,
                            const tm_trace_opts* opts, int64_t* bytes);

/* tetmesh_tri_vertices -- host: vertex ids (caller numbering, ascending) of
 * triangles.  tri host int32 [n]; out host int32 [n][3].  TM_ERR_ARG on an id
 * out of range. */
int tetmesh_tri_vertices(tm_mesh m, int64_t n, const int32_t* tri, int32_t* out);

/* tetmesh_info -- sizes of an uploaded mesh; out host. */
int tetmesh_info(tm_mesh m, tm_info* out);

/* tetmesh_free -- release the handle and its device memory (synchronises the
 * device first).  NULL is a no-op. */
int tetmesh_free(tm_mesh m);

/* tm_last_error -- description of the last error on the calling thread ("" if
 * none).  The string stays valid until the next call on that thread. */
const char* tm_last_error(void);

/* tetrt_sfc_keys -- host utility: space-filling-curve keys of integer points.
 * xyz host uint32 [n][3], each coordinate < 2^bits (1 <= bits <= 21);
 * curve TM_SFC_HILBERT or TM_SFC_MORTON; out host uint64 [n].  The Hilbert key
 * follows Skilling's transpose construction (Skilling, "Programming the Hilbert
 * curve", AIP Conf. Proc. 707, 2004). */
int tetrt_sfc_keys(int32_t curve, int32_t bits, int64_t n, const uint32_t* xyz, uint64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* TETRT_H */
