// Device-side view of an uploaded mesh and the kernel launchers.
#pragma once
#include <algorithm>
#include <cstdint>

#include <hip/hip_runtime_api.h>

namespace tetrt {

// Plain pointers into device memory owned by a tm_mesh handle; passed to the
// kernels by value.  Vector-typed arrays are stored as their scalar base type
// and reinterpreted in the kernels (int4 / int2, 16- or 8-byte aligned; points
// are plain x, y, z triples).
struct DevMesh {
    const int32_t* rec;       // [nt*5] Tet20 records (xor field, N0..N3),
                              // [nt*4] Tet16 records (xor field, NX0..NX2) or
                              // [nt*8] Tet32N records (N0..N3, neighbours' xor fields)
    const int32_t* n3;        // [nt]      Tet16 only: N3 of every tet (cold, for starts)
    const float* pts;         // [np*3]    x, y, z per point (12 bytes, no padding)
    const int32_t* tetv;      // [nt*4]    ascending vertex ids (int4 per tet)
    const int32_t* cfv;       // [ntri*4]  constrained-face vertices (int4)
    const int32_t* cft;       // [ntri*4]  constrained-face tets and their xor fields (int4)
    const int32_t* t_new2old; // [nt]
    const int32_t* t_old2new; // [nt]
    const int32_t* seed;      // [G^3]
    float lo[3];
    float inv_cell[3];
    int32_t G;
    int32_t nt;
    int32_t np;
    int32_t ntri;
    int32_t layout;           // TM_LAYOUT_*
};

struct RayArgs {
    const int32_t* perm;       // optional: lane j of the grid traces ray perm[j]
    const float* orig;
    const float* dir;
    const float* tmax;
    const int32_t* start_tet;
    const int32_t* start_face;
    int32_t* tri;
    float* t;
    float* bary;
    int32_t* hit_tets;
    int32_t* steps;
    int32_t* fp64_steps;       // optional: walk steps decided in float64, per ray
    int64_t n;
    int32_t max_steps;
};

// Work queue of the persistent-wave kernel: the ray order is cut into chunks of
// `chunk` rays, split into `xcds` contiguous ranges, one per accelerator die;
// each range has a counter (cursor[32 x], zero when the launch starts) from
// which the waves of that die take chunks, and a die whose range is exhausted
// takes chunks from the others' ranges.
struct Queue {
    uint32_t* cursor;       // [32 * xcds] counters, one per 128-byte line
    uint32_t n_chunks;      // chunks over all jobs
    uint32_t chunk;         // rays per chunk: 64, 128 or 256
    uint32_t xcds;          // ranges (1 = one shared range)
    int32_t refill;         // finished lanes of a wave that trigger a refill (1..64)
};
constexpr int64_t kQueueCursorBytes = 32 * 4 * 64;   // room for 64 dies

// Rays of the precision variant whose walk meets an exact float64 tie, listed by
// the walk so that their closest hits by definition (a scan of every constrained
// triangle) are found by the whole grid rather than by the one wave that met
// them.  Entries past `cap` are resolved by their wave as before.
struct TieList {
    uint32_t* count;            // [1] ties listed (zero when the walk starts); null = no list
    int32_t* ray;               // [cap] ray index
    int32_t* steps;             // [cap] walk steps before the tie
    int32_t* n64;               // [cap] steps decided in float64
    unsigned long long* tmin;   // [cap] bits of the nearest hit's t (a positive double); +inf: none
    int32_t* best;              // [cap] the lowest id hit within 1e-12 of it
    uint32_t cap;
};
constexpr uint32_t kTieCap = 16384;
// Bytes of a tie list of kTieCap entries (with its counter), 256-byte aligned parts.
int64_t tie_workspace_bytes();
// Carves a tie list out of `bytes` of device memory at p.
TieList tie_list_at(void* p);

struct LaunchCfg {
    int32_t block;          // threads per block (64, 128 or 256)
    int32_t kernel;         // 1 = one lane per ray, 2 = persistent lanes, 3 = persistent waves on a queue
    int32_t refill;         // persistent: finished lanes per wave that trigger a refill
    int32_t waves_per_simd; // persistent: resident waves per SIMD to launch for
    int32_t cus;            // compute units of the device
    int32_t grid_cap;       // persistent: at most this many blocks (0 = no cap)
    int32_t xcds;           // one lane per ray: XCDs the blocks are renumbered for (1 = off)
    int32_t xcd_blocks;     // consecutive blocks per XCD (0 = one contiguous range each)
    float eps;              // > 0: precision variant (one lane per ray)
    Queue queue;            // kernel 3
    struct Job* queue_job;  // kernel 3: device room for a one-entry job table
    uint32_t* defer_count;  // eps > 0, non-null: two passes (counter and list of deferred rays)
    int32_t* defer_list;    //   list: room for every ray
    TieList ties;           // eps > 0, one pass: count non-null = ties resolved by the grid
};

hipError_t launch_trace(const DevMesh& m, const RayArgs& r, const LaunchCfg& c, hipStream_t s);

// Ray binning inside chunks of 2^chunk_log2 consecutive rays: by direction
// quantised to dirq levels per axis, then (cells_log2 > 0) by the low bits of
// the Morton index of the origin's cell in a 2^cells_log2 grid over
// [lo, lo + G/inv).
struct SortCfg {
    int32_t chunk_log2;       // 10..13
    int32_t cells_log2;       // 0 (direction only) .. 7
    int32_t dirq;             // 1..4
    float lo[3];
    float inv[3];             // cells per unit length, per axis
};

int64_t sort_workspace_bytes(int64_t n);
// Workspace of the queue kernel in a single-mesh trace: its counters and a
// one-entry job table.
int64_t queue_workspace_bytes();

// One job of a batched launch: a mesh, its rays, and where its blocks and
// binning chunks start in the launch.  Lives in device memory.
struct Job {
    DevMesh m;
    RayArgs r;
    SortCfg sc;
    int64_t block0;           // first block of this job in the trace launch
    int64_t chunk0;           // first chunk of this job in the binning launch
    int64_t qchunk0;          // first chunk of this job in the persistent-wave queue
};

// One launch over all jobs (table in device memory, block0 ascending); jobs
// share the record layout.  Rays without tmax get +inf.  xcds > 1: the blocks
// are renumbered so that each XCD takes one contiguous range of them.  steps:
// some job has a step-count array (the kernel then keeps per-ray counts).
// eps > 0: the precision variant.
hipError_t launch_trace_batch(const Job* d_jobs, int32_t n_jobs, int64_t total_blocks, int32_t block,
                              int32_t layout, int32_t xcds, bool steps, float eps, hipStream_t s);
// The same walk by persistent waves draining the queue q over every job's rays
// (zeroes q's counters first, with a kernel of its own); `cus` sizes the grid.
hipError_t launch_trace_batch_queue(const Job* d_jobs, int32_t n_jobs, const Queue& q, int32_t layout,
                                    bool steps, int32_t cus, hipStream_t s);
// Binning of every job's rays (chunks of 2^chunk_log2; perm pointers in the table).
hipError_t launch_sort_batch(const Job* d_jobs, int32_t n_jobs, int64_t total_chunks,
                             int32_t chunk_log2, hipStream_t s);
// Fills the permutation (inside ws) that orders the rays by bin.
hipError_t launch_sort(const SortCfg& c, const float* orig, const float* dir, int64_t n, void* ws,
                       int32_t** perm_out, hipStream_t s);
hipError_t launch_locate(const DevMesh& m, int64_t n, const float* pts, int32_t* out,
                         int32_t max_steps, hipStream_t s);

// Ray generation for served requests.  The ray slots of a request are a range of
// a pool; phase 0 writes camera rays, phase 1 turns each slot's phase-0 ray and
// its hit (tri, t) into a shadow or ambient-occlusion ray in place.
struct RayPool {
    float* orig;       // [cap][3]
    float* dir;        // [cap][3]
    float* tmax;       // [cap]
    int32_t* sf;       // [cap] start face
    int32_t* tri;      // [cap] phase-0 results
    float* t;          // [cap]
    float* bary;       // [cap][2]
};

enum GenKind : int32_t { kGenCamera = 0, kGenShadow = 1, kGenAO = 2 };
constexpr int kGenBlock = 256;   // threads per block of the generation launch

struct GenEntry {
    int32_t kind;      // GenKind
    int32_t W, H;      // image size, multiples of 8; rays in 8x8 tiles, tiles row-major
    uint32_t seed;     // AO random stream
    int64_t block0;    // first block of this entry in the launch
    int64_t base;      // first pool slot
    float eye[3];
    float fwd[3];      // camera: unit forward, and right / up scaled by the half-extent
    float right[3];    //   of the image plane at distance 1
    float up[3];
    float light[3];    // shadow: light position
    float ao_tmax;
    const float* pts;  // mesh points (x, y, z) and constrained-face vertices (int4),
    const int32_t* cfv;//   for the normal of the hit triangle
};

hipError_t launch_gen(const GenEntry* d_gen, int32_t n, int64_t total_blocks, RayPool pool, hipStream_t s);
// The rays of one entry (base = 0 into the given arrays).
hipError_t launch_gen_one(const GenEntry& g, RayPool pool, hipStream_t s);

}  // namespace tetrt
