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
 *     passes.  No call allocates per ray batch.  A call on a mesh, batch or
 *     server needs the device it was created on to be current (TM_ERR_ARG
 *     otherwise).
 *   - Work is enqueued on the given HIP stream (NULL = the default stream) and
 *     returns without synchronising.  A handle is read-only after upload, so
 *     traces on different streams may run concurrently; traces that bin through
 *     the handle's own workspace are ordered one after another (a trace on
 *     another stream than the previous such trace waits for it on the device).
 *   - trace_closest, tetmesh_locate, tetmesh_bin_rays and the batch launches
 *     never allocate memory or wait for the device.
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
    TM_LAYOUT_TET32N = 2, /* not a layout of the paper: the four neighbour fields + the
                            xor-sum of each neighbour (32 B/tet), so a walk step loads
                            its record and its point together */
    TM_LAYOUT_TET32 = 3  /* the paper's Tet32 (Fig. 2): three vertex ids, the xor of all
                            four, and the four neighbour fields, N_j across V_j (32 B/tet);
                            the next tet is found by comparing the exit vertex with the
                            stored ids (Algorithms 2-3) */
};

/* memory order of points and tets (paper, Sec. "Reordering tetrahedral mesh data") */
enum {
    TM_SFC_HILBERT = 0, /* points by position, tets by centroid, 3-D Hilbert key */
    TM_SFC_MORTON = 1,  /* same keys on the Morton (Z-order) curve */
    TM_SFC_NONE = 2,    /* keep the caller's order */
    TM_SFC_HILBERT_REGIONS = 3 /* tets grouped by region first (tets that constrained faces
                            enclose together, which no walk leaves), regions in the
                            Hilbert order of their first tet, Hilbert order inside a
                            region; points as TM_SFC_HILBERT */
};

typedef struct tm_mesh_s* tm_mesh;

/* Options for tetmesh_upload; pass NULL for the defaults (all fields 0 except
 * validate = 1). */
typedef struct {
    int32_t layout;    /* TM_LAYOUT_* */
    int32_t sfc;       /* TM_SFC_* */
    int32_t validate;  /* 1 = check the mesh before packing (recommended) */
    int32_t seed_grid; /* cells per axis of the point-location seed grid; 0 = automatic */
    int64_t bin_rays;  /* rays the handle's own workspace serves (8 bytes each and about
                          400 KB), allocated here, once; 0 = none.  trace_closest uses it for
                          binning, the queue kernel and the precision variant's tie list
                          and two passes when the caller passes no workspace of its own.
                          0 <= bin_rays < 2^31 */
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
    int32_t n_regions;   /* TM_SFC_HILBERT_REGIONS: regions found at upload (else 0) */
} tm_info;

/* Options for trace_closest; pass NULL for the defaults (all fields 0). */
typedef struct {
    int32_t max_steps;   /* walk step cap per ray (tets entered); 0 = 65536 */
    int32_t block;       /* threads per block: 64, 128 or 256 (0 = automatic: 256 when the
                            rays are binned or in a caller's order, else 128) */
    int32_t kernel;      /* 0 = automatic, 1 = one lane per ray, 2 = persistent lanes that
                            take further rays as theirs finish, 3 = persistent waves that
                            drain a work queue: each wave takes chunks of queue_chunk rays
                            from a global counter per XCD (its own die's range first, then
                            the others'), stages their ids in LDS and refills its finished
                            lanes from them (needs a workspace, as binning does) */
    int32_t refill;      /* kernels 2 and 3: finished lanes per wavefront that trigger a
                            refill, 1..64 (0 = 16 for kernel 2, 64 for kernel 3) */
    int32_t grid_cap;    /* persistent lanes: at most this many blocks (0 = enough blocks
                            to fill every compute unit) */
    int32_t xcds;        /* one lane per ray: number of accelerator dies (XCDs, 8 on MI355X)
                            the blocks are renumbered for, so that consecutive blocks run
                            on one die and share its L2.  0 = automatic: the device's dies
                            for binned launches (or with order), off otherwise; 1 = off
                            (the dispatcher's round-robin placement) */
    int32_t sort;        /* ray binning before the walk: 0 = automatic (on for batches of at
                            least 2^18 rays that carry tmax), 1 = off, 2 = on.  Inside each
                            chunk of consecutive rays, rays are grouped by quantised
                            direction, then by the low bits of the Morton index of their
                            origin's cell, and traced in that order; the outputs stay at
                            the caller's positions */
    int32_t sort_chunk_log2; /* rays per chunk = 2^this, 10..13 (0 = 12) */
    int32_t sort_cells_log2; /* 0 (default): bins by direction only; 1..7: then by the
                                origin's cell in a grid of 2^this cells per axis */
    int32_t sort_dirq;   /* direction bins per axis, 1..4 (0 = 4) */
    int32_t xcd_blocks;  /* with xcds > 1: consecutive blocks per die (0 = one contiguous
                            range of the launch per die; > 0 = runs of this many blocks,
                            interleaved over the dies as they are dispatched) */
    float eps;           /* precision variant, 0 = off.  When > 0 (one lane per ray only), a
                            walk step whose float32 exit-face determinants det(q3, q_i) are
                            within eps * (|q3|_1 + |q_i|_1) of zero is decided in float64
                            along the ray as given (the sign of d . ((P3 - o) x (P_i - o))
                            from the float32 points, origin and direction); the start tet,
                            its exit face and the face's orientation are also found in
                            float64.  A ray whose float64 decision is an exact tie (a vertex
                            on the ray, a ray in a face's plane) takes the closest hit by
                            its definition (every constrained triangle tested in float64,
                            the lowest id among hits within 1e-12 of the nearest), found by
                            the whole grid for up to 16,384 ties per call when a workspace
                            holds the tie list, else (and past that) by the ray's wave; the
                            results are the same.  With the scene extent 1,
                            eps >= 1e-6 covers float32 rounding */
    void* workspace;     /* device scratch for binning, kernel 3's queue and the precision
                            variant's lists (tetmesh_trace_workspace gives the need), or
                            NULL: the handle's own
                            workspace (tm_upload_opts.bin_rays) is then used when it is large
                            enough.  A binned trace with neither: sort = 2 or kernel = 3 fails
                            (TM_ERR_ARG), sort = 0 traces the rays unbinned (the same
                            results) */
    int64_t workspace_bytes; /* size of workspace */
    int32_t* fp64_steps; /* device int32 [n_rays] or NULL: out: walk steps decided in float64
                            (0 when eps = 0) */
    const int32_t* order; /* device int32 [n_rays] or NULL: trace the rays in this order (lane j
                            takes ray order[j]; a permutation of 0..n_rays-1, e.g. from
                            tetmesh_bin_rays; entries out of range are skipped).  Replaces
                            the call's own binning (sort is then ignored) */
    int32_t queue_chunk; /* kernel 3: rays a wave takes from the queue at a time, a multiple
                            of 64 in [64, 4096] (0 = 64) */
    int32_t passes;      /* precision variant: 0 or 1 = one pass; 2 = two passes, a float32
                            walk that defers the rays meeting an unsure step to a list, then
                            the float64-capable walk of the listed rays only (same results;
                            needs a workspace, else one pass).  Measured slower than one pass
                            on the 12.6M-tet workload */
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
 * Limits: 1 <= n_tets <= 214,748,364 (134,217,727 with TM_LAYOUT_TET32N or _TET32: the
 * records and points stay below 4 GiB each), 4 <= n_points <= 357,913,941, fewer
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
 * trace_closest_noalloc -- trace_closest for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors as
 * trace_closest, except: opts->workspace must be NULL; a trace that bins its
 * rays (sort = 2, or the automatic rule) puts the binning permutation in a
 * fixed array of the library instead (4 bytes per ray, at most
 * TM_NOALLOC_MAX_BINNED_RAYS rays: more is TM_ERR_ARG), and the queue kernel's
 * counters (kernel = 3) and the precision variant's tie list (eps > 0) go to
 * 512 KiB beside that room.  The array exists once per device and lives until
 * the process ends (64 MiB + 512 KiB of device memory on every device the
 * library's kernels have run on); it is looked up, not allocated, on a
 * device's first call.  Every call on a device shares it, so calls that use it
 * (binning, kernel 3, eps > 0) and overlap in time on one device (other
 * streams, other threads) race and must be ordered by the caller.  Other
 * traces use no scratch at all.
 */
#define TM_NOALLOC_MAX_BINNED_RAYS (1 << 24)
int trace_closest_noalloc(tm_mesh m, int64_t n_rays, const float* d_orig, const float* d_dir,
                          const float* d_tmax, const int32_t* d_start_tet,
                          const int32_t* d_start_face, int32_t* d_tri, float* d_t, float* d_bary,
                          int32_t* d_hit_tets, int32_t* d_steps, const tm_trace_opts* opts,
                          void* hip_stream);

/*
 * tetmesh_locate -- tet containing each point (paper, Sec. "Locating points in
 * a tetrahedral mesh": a straight-line walk from a source tet, here the seed
 * tet of the point's cell in a uniform grid over the mesh bounds).
 *   0 <= n < 2^31;  d_pts  device float32 [n][3];  d_tet  device int32 [n] out: caller tet id, -1 when
 *   the point is outside the mesh, -2 at the step cap.  A point on a shared face,
 *   edge or vertex gets one of the tets that contain it.
 */
int tetmesh_locate(tm_mesh m, int64_t n, const float* d_pts, int32_t* d_tet, void* hip_stream);

/* tetmesh_bin_rays -- the ray order trace_closest's binning would use (the
 * sort option's chunked grouping by direction and origin cell, with
 * sort_chunk_log2, sort_cells_log2 and sort_dirq of opts), written to d_order
 * (device int32 [n_rays], caller-owned) for a later trace_closest with
 * opts->order.  Lets a caller bin once and trace several times, or time the
 * two kernels apart.  0 <= n_rays < 2^31.  Errors: TM_ERR_ARG, TM_ERR_HIP. */
int tetmesh_bin_rays(tm_mesh m, int64_t n_rays, const float* d_orig, const float* d_dir,
                     const tm_trace_opts* opts, int32_t* d_order, void* hip_stream);

/* tetmesh_trace_workspace -- bytes of device workspace a trace_closest call with
 * these arguments needs (0 when it needs none: no binning, kernel 1 or 2, eps = 0).  d_tmax_present: the d_tmax
 * argument of that call (only tested for NULL).  *bytes host out. */
int tetmesh_trace_workspace(tm_mesh m, int64_t n_rays, const float* d_tmax_present,
                            const tm_trace_opts* opts, int64_t* bytes);

/*
 * Batched traces over many meshes in one launch.
 *
 * A batch holds a table of jobs, each a mesh handle and its rays with the
 * arrays trace_closest takes.  One launch walks every ray of every job: the
 * blocks of the launch are split among the jobs in table order, each block
 * finds its job in the table, and the walk is that of trace_closest with one
 * lane per ray.  Small meshes thereby share the device with large ones without
 * a launch, and a host round trip, per mesh.  The results of a ray are those
 * that trace_closest gives it with the same max_steps.
 */
typedef struct {
    tm_mesh mesh;             /* uploaded on the batch's device; all jobs of a batch share
                                 one record layout; must outlive every launch of the job */
    int64_t n_rays;           /* 0 <= n_rays < 2^31 */
    const float* d_orig;      /* the arrays of trace_closest, same meaning, same rules */
    const float* d_dir;
    const float* d_tmax;      /* nullable */
    const int32_t* d_start_tet;  /* nullable */
    const int32_t* d_start_face; /* nullable */
    int32_t* d_tri;
    float* d_t;
    float* d_bary;
    int32_t* d_hit_tets;      /* nullable */
    int32_t* d_steps;         /* nullable */
} tm_job;

typedef struct tm_batch_s* tm_batch;

/* tm_batch_create -- a batch on the current HIP device for up to max_jobs jobs
 * (1..65536) of at most max_rays rays in total (0 <= max_rays < 2^40).  Allocates
 * the device job table, a pinned host staging copy of it, and the binning
 * workspace (4 bytes per ray), once.  out host.  Errors: TM_ERR_ARG,
 * TM_ERR_OOM, TM_ERR_HIP. */
int tm_batch_create(int32_t max_jobs, int64_t max_rays, tm_batch* out);

/* tm_batch_set -- replace the batch's jobs.  jobs host [n_jobs] (0 <= n_jobs <=
 * max_jobs), copied.  opts as for trace_closest, except: kernel 0, 1 or 3 (3:
 * persistent waves drain one queue of every job's rays, queue_chunk and refill
 * as for trace_closest; xcds = its number of per-XCD ranges, 0 = the device's
 * XCDs), eps > 0 (the precision variant, one pass) with kernel 0 or 1 only,
 * xcd_blocks, grid_cap, passes, workspace, fp64_steps and order are ignored, with kernel 1 xcds = 0 means round-robin placement (xcds > 1: one
 * contiguous range of the whole launch per XCD), and the binning chunk size is one for all jobs
 * (sort = 0 bins the jobs that carry tmax and have at least 2^18 rays).  The new table is copied to the device on
 * hip_stream, after the batch's previous table copy has left the staging
 * buffer; launches on that stream that follow see it.  A launch of the batch on
 * another stream must be ordered after this call's stream by the caller.
 * Errors: TM_ERR_ARG (the first offending job is named), TM_ERR_HIP. */
int tm_batch_set(tm_batch b, int32_t n_jobs, const tm_job* jobs, const tm_trace_opts* opts,
                 void* hip_stream);

/* tm_batch_launch -- enqueue the walk of every ray of every job on hip_stream:
 * at most three kernel launches (binning, the queue's counter reset with kernel
 * 3, walk), with no allocation, memory set, copy or synchronisation, so a
 * caller may capture it into a HIP graph.
 * Errors: TM_ERR_ARG, TM_ERR_HIP. */
int tm_batch_launch(tm_batch b, void* hip_stream);

/* tm_batch_graph_launch -- tm_batch_launch as a HIP graph owned by the batch.
 * The graph is captured on first use and again whenever tm_batch_set changed
 * the launch shape (blocks, chunks, block size); otherwise a replay costs one
 * graph launch.  Job contents may change between replays through tm_batch_set.
 * Errors: TM_ERR_ARG, TM_ERR_HIP. */
int tm_batch_graph_launch(tm_batch b, void* hip_stream);

/* tm_batch_tune -- autotuner: times tm_batch_launch on the current jobs for
 * each block size (64, 128, 256), binning setting (off; on with 2^11, 2^12,
 * 2^13 rays per chunk) and die placement (round-robin; one contiguous range of
 * blocks per XCD) of the one-lane-per-ray kernel, and for the queue kernel
 * each binning setting, rays per wave fetch (queue_chunk 64, 256, 1024) and
 * refill threshold (16, 64), reps timed launches each after one warm-up, with
 * HIP events on hip_stream, and keeps the fastest.  Overwrites the jobs' outputs
 * (with the same results).  Synchronous.  chosen host, nullable: receives the
 * options kept; ms host, nullable: their mean launch time in milliseconds.
 * Errors: TM_ERR_ARG, TM_ERR_HIP. */
int tm_batch_tune(tm_batch b, int32_t reps, void* hip_stream, tm_trace_opts* chosen, float* ms);

/* tm_batch_free -- release the batch (synchronises the device first).  NULL is
 * a no-op.  The meshes of its jobs are not freed. */
int tm_batch_free(tm_batch b);

/*
 * Serving: requests against resident meshes, batched continuously.
 *
 * A request renders one image of one mesh: a camera ray per pixel (pinhole,
 * as in the paper's renderer), and for shadow and ambient-occlusion requests
 * one more ray per pixel from the camera ray's hit (paper, Sec. "Handling
 * Common Ray-tracing Operations": secondary rays start from the hit face).
 * The server admits queued requests while their rays fit a preallocated ray
 * pool, generates rays on the device, and at each step traces the pending
 * phase of every admitted request in one batched launch (tm_batch), so work
 * of different requests and meshes shares the device.  Up to `ring` launches
 * are in flight; a step never waits for the device.  A server is driven by one
 * host thread.
 *
 * Results are written to the request's own device buffers, one entry per
 * pixel in tile order: 8x8 pixel tiles, tiles row-major over the image, pixels
 * row-major inside a tile (ray k is pixel (8 (tile % (W/8)) + k % 8,
 * 8 (tile / (W/8)) + (k % 64) / 8) with tile = k / 64).
 *   TM_REQ_PRIMARY: the camera ray's trace_closest results.
 *   TM_REQ_SHADOW:  the results of the ray from the hit point P towards the
 *                   light L (direction L - P, tmax 1): a triangle id = in
 *                   shadow, TM_RAY_MISS = lit; TM_RAY_INVALID where the camera
 *                   ray hit nothing.
 *   TM_REQ_AO:      the results of one cosine-weighted ray (tmax ao_tmax) about
 *                   the hit triangle's normal, on the side the camera ray came
 *                   from; TM_RAY_INVALID where the camera ray hit nothing.
 * A request's results depend on the request alone, not on what it was batched with.
 */
enum { TM_REQ_PRIMARY = 0, TM_REQ_SHADOW = 1, TM_REQ_AO = 2 };

typedef struct {
    int32_t mesh;        /* index into the meshes given to tm_server_create */
    int32_t kind;        /* TM_REQ_* */
    int32_t width;       /* image size, multiples of 8 in [8, 8192] */
    int32_t height;
    float eye[3];        /* camera position */
    float forward[3];    /* view direction, nonzero */
    float up[3];         /* up hint, not parallel to forward */
    float fov_h_deg;     /* horizontal field of view, in (0, 179] degrees */
    float light[3];      /* TM_REQ_SHADOW: point light */
    float ao_tmax;       /* TM_REQ_AO: ray length (> 0) */
    uint32_t seed;       /* TM_REQ_AO: random stream of the directions */
    int32_t* d_tri;      /* device out [width*height] (caller-owned until the request is done) */
    float* d_t;          /* device out [width*height] */
    float* d_bary;       /* device out [width*height][2], 8-byte aligned */
} tm_request;

typedef struct {
    int64_t max_rays;     /* ray pool slots (one per pixel of every admitted request),
                             1 <= max_rays <= 2^31 - 1; 48 bytes of device memory each */
    int32_t max_requests; /* admitted requests at once, 1..65536 (0 = 4096) */
    int32_t ring;         /* launches in flight, 1..8 (0 = 1) */
    int32_t block;        /* as tm_trace_opts */
    int32_t sort;
    int32_t max_steps;
    float eps;            /* the precision variant for every traced phase (0 = off) */
} tm_server_opts;

/* A finished request; times are host steady-clock nanoseconds. */
typedef struct {
    int64_t id;
    int64_t submit_ns;   /* tm_server_submit */
    int64_t admit_ns;    /* admitted to the pool */
    int64_t done_ns;     /* the step that saw its last launch complete */
    int64_t rays;        /* rays traced for it */
} tm_done;

typedef struct tm_server_s* tm_server;

/* tm_server_create -- meshes host [n_meshes] (1..65536 handles, one record
 * layout, current device; they must outlive the server); opts nullable.
 * Allocates the ray pool and the launch ring once.  Errors: TM_ERR_ARG,
 * TM_ERR_OOM, TM_ERR_HIP. */
int tm_server_create(const tm_mesh* meshes, int32_t n_meshes, const tm_server_opts* opts,
                     tm_server* out);

/* tm_server_submit -- queue a request (copied; FIFO admission); *id host out (ids
 * start at 1).  Host only, never blocks.  Errors: TM_ERR_ARG (a request that
 * could never fit the pool included). */
int tm_server_submit(tm_server s, const tm_request* req, int64_t* id);

/* tm_server_step -- retire completed launches, admit queued requests that fit,
 * and enqueue on hip_stream one launch of ray generation and one batched trace
 * of every pending phase.  Never waits for the device: with the ring full it
 * launches nothing.  *launched host out, nullable: rays launched.  Use one
 * stream for every step of a server.  Errors: TM_ERR_ARG, TM_ERR_HIP. */
int tm_server_step(tm_server s, void* hip_stream, int64_t* launched);

/* tm_server_poll -- move up to max finished requests to out (host [max]); *n
 * host out.  Their outputs are complete when they are reported. */
int tm_server_poll(tm_server s, tm_done* out, int32_t max, int32_t* n);

/* tm_server_drain -- step until every submitted request is finished, waiting
 * on the device between steps.  Errors as tm_server_step. */
int tm_server_drain(tm_server s, void* hip_stream);

/* tm_server_pending -- requests submitted and not yet reported by poll; host out. */
int tm_server_pending(tm_server s, int64_t* queued, int64_t* admitted, int64_t* finished);

/* tm_request_rays -- the rays a server generates for a request, written to
 * caller arrays (for checking results, or tracing them elsewhere).  m: the
 * request's mesh; req->mesh and the output pointers are ignored.
 *   phase 0: camera rays -> d_orig, d_dir [W*H][3], d_tmax (+inf), d_start_face (-1).
 *   phase 1 (shadow, AO): reads the camera rays in d_orig, d_dir and their
 *            trace_closest results d_tri, d_t [W*H], and overwrites d_orig, d_dir,
 *            d_tmax, d_start_face with the secondary rays (zero direction where
 *            d_tri < 0).
 * All device arrays, tile order as above.  Errors: TM_ERR_ARG, TM_ERR_HIP. */
int tm_request_rays(tm_mesh m, const tm_request* req, int32_t phase, float* d_orig, float* d_dir,
                    float* d_tmax, int32_t* d_start_face, const int32_t* d_tri, const float* d_t,
                    void* hip_stream);

/* tm_server_free -- release the server (synchronises the device first).  NULL
 * is a no-op. */
int tm_server_free(tm_server s);

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
