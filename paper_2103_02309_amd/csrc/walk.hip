// Closest-hit traversal kernels for gfx950: one lane per ray (wave64).
//
// Per ray (paper, Sec. "Tetrahedron Traversal"):
//   basis     2-D basis (u, v) orthogonal to the direction, scaled so that u has
//             a zero at the direction's smallest component and its largest
//             components are +-1 (subsection "Point projection using
//             specialized basis", Eq. 1-2; the divisor of v is the magnitude of
//             its largest component, which always sits at that index).
//   project   q(P) = (u.P - po_x, v.P - po_y) with po = (u.o, v.o) (Sec. "GPU
//             Implementation", Eq. 4-5).  u and v are kept as full 3-vectors:
//             their zero and +-1 entries make each fused multiply-add of the
//             corresponding term exact, which is Eq. 3 without per-lane
//             component selects.
//   start     the tet containing the origin (given, or located by a straight
//             line walk from a seed tet), whose exit face is found in 3-D once;
//             or, for secondary rays, the tet on the far side of the start face.
//   step      id3 = a0 ^ a1 ^ a2 ^ VX[tet]; q3 = q(P[id3]); e = Algorithm 1;
//             next = N[tet][rank of a[e] among {a0, a1, a2, id3}] (Algorithms
//             4-5); slot e of the kept face takes (id3, q3).
//   stop      at a neighbour field with the top bit set: a constrained face
//             (hit) or the boundary (miss).  The hit's t and barycentric
//             weights are evaluated once, in float64.
//   precision (optional, eps > 0) when one of Algorithm 1's determinants is
//             within eps (|q3|_1 + |q_i|_1) of zero -- the only case in which
//             float32 rounding of the projections can flip its sign -- the step
//             recomputes the four projections and determinants in float64 from
//             the float32 points, basis and origin and decides with those; the
//             start tet's exit face is then also found in float64.
//
// Memory (paper, Sec. "Tetrahedral Mesh Representation"):
//   Tet20  20 packed bytes {VX, N0, N1, N2, N3}, read as one 16-byte and one
//          4-byte load;
//   Tet16  16 bytes {VX, NX0, NX1, NX2} with NX_j = N_j ^ N_3, one aligned
//          16-byte load; the neighbour across the exit face is the field of the
//          entry face (known: it refers back to the previous tet) xor NX of the
//          entry vertex's rank xor NX of the exit vertex's rank (NX_3 = 0),
//          Algorithms 6-7.
//   With these the point is one 12-byte load after the record, so a step is
//   two dependent round trips (record, then point).  Points are stored as
//   12-byte triples, not padded to 16: more of them share a cache line, and
//   the walk's loads are bound by the L1's line lookups and fills.  The next record's load is
//   issued inside the step, as soon as the exit face is known.
//   Tet32N 32 bytes {N0..N3, W0..W3}: the neighbour fields and each
//          neighbour's xor-sum.  The xor-sum of the tet being entered comes
//          with the previous record, so the record and the point of a step are
//          loaded together: one round trip per step, for twice the bytes and
//          one more L1 lookup per lane than Tet16.  Not one of the paper's
//          layouts: the paper's xor idea moved one step ahead.
//   Tet32  32 bytes {V0, V1, V2, VX, N0..N3} (Fig. 2), two 16-byte loads; the
//          next tet is the neighbour field beside the stored vertex id that
//          equals the exit vertex, N3 when none does (Algorithms 2-3): no rank,
//          three compares.
// Records and points are read by id through structured buffer descriptors: an
// index past the array reads zero instead of faulting.  The step is
// branch-free: the loop test is its only branch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "device.h"
#include "tetrt.h"

using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Structured buffer loads (index * stride + offset, computed by the address
// unit): a record or point is read by its id, with no vector instruction to
// scale the id into a byte offset.  Clang has builtins for the raw (byte
// offset) forms only, so these name the LLVM intrinsics directly.
extern "C" __device__ u32x4 sbuf_load_b128(rsrc_t r, unsigned index, unsigned voffset,
                                           unsigned soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");
extern "C" __device__ u32x3 sbuf_load_b96(rsrc_t r, unsigned index, unsigned voffset,
                                          unsigned soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v3i32");
extern "C" __device__ unsigned sbuf_load_b32(rsrc_t r, unsigned index, unsigned voffset,
                                             unsigned soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.i32");

namespace tetrt {

namespace {

constexpr uint32_t kBoundary = 0xFFFFFFFFu;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;

// record layouts
constexpr int kTet20 = 0;
constexpr int kTet16 = 1;
constexpr int kTet32N = 2;
constexpr int kTet32 = 3;

template <int LAYOUT>
constexpr uint32_t rec_bytes() { return LAYOUT == kTet20 ? 20u : (LAYOUT == kTet16 ? 16u : 32u); }  // Tet32, Tet32N: 32

// gfx9-family buffer descriptor for `count` elements of `stride` bytes.  An
// access to an index at or past `count` reads zeros (the bound is given in
// elements, the unit the address unit checks an index against when the stride
// is non-zero).
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t stride, uint32_t count) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)stride, int(count), 0x00020000);
}

struct Mem {
    rsrc_t rec;
    rsrc_t pts;
};

template <int LAYOUT>
__device__ __forceinline__ Mem make_mem(const DevMesh& m) {
    Mem M;
    M.rec = make_rsrc(m.rec, rec_bytes<LAYOUT>(), uint32_t(m.nt));
    M.pts = make_rsrc(m.pts, 12u, uint32_t(m.np));
    return M;
}

// Pins a loaded value at this point of the program.  Without it the compiler
// may turn a select among loaded fields into a branch and move the load into
// it, which adds a dependent memory round trip to the step.
__device__ __forceinline__ void keep(uint32_t& v) { asm volatile("" : "+v"(v)); }

// A record as loaded: the xor field and four more words (Tet20: N0..N3 by
// ascending vertex id; Tet16: NX0..NX2 and 0; Tet32N: N0..N3 and the
// neighbours' xor-sums w0..w3, no xor field of its own; Tet32: N0..N3 and the
// stored vertex ids V0..V2 in w0..w2).
struct Rec {
    int32_t vx;
    uint32_t n0, n1, n2, n3;
    uint32_t w0, w1, w2, w3;
};

template <int LAYOUT>
__device__ __forceinline__ Rec load_rec(const Mem& M, uint32_t tet) {
    if (LAYOUT == kTet20) {
        const u32x4 a = sbuf_load_b128(M.rec, tet, 0u, 0u, 0);
        uint32_t b = sbuf_load_b32(M.rec, tet, 16u, 0u, 0);
        keep(b);
        return Rec{int32_t(a[0]), a[1], a[2], a[3], b, 0u, 0u, 0u, 0u};
    } else if (LAYOUT == kTet16) {
        const u32x4 a = sbuf_load_b128(M.rec, tet, 0u, 0u, 0);
        return Rec{int32_t(a[0]), a[1], a[2], a[3], 0u, 0u, 0u, 0u, 0u};
    } else if (LAYOUT == kTet32) {
        const u32x4 a = sbuf_load_b128(M.rec, tet, 0u, 0u, 0);    // V0, V1, V2, VX
        const u32x4 b = sbuf_load_b128(M.rec, tet, 16u, 0u, 0);   // N0..N3
        return Rec{int32_t(a[3]), b[0], b[1], b[2], b[3], a[0], a[1], a[2], 0u};
    } else {
        const u32x4 a = sbuf_load_b128(M.rec, tet, 0u, 0u, 0);
        const u32x4 b = sbuf_load_b128(M.rec, tet, 16u, 0u, 0);
        return Rec{0, a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    }
}

// Word r (0..3) of four, selected on the bits of r: three selects and no
// compare chain (which the compiler would turn into a branch).
__device__ __forceinline__ uint32_t pick4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, int r) {
    const bool b0 = (r & 1) != 0, b1 = (r & 2) != 0;
    const uint32_t lo = b0 ? w1 : w0;
    const uint32_t hi = b0 ? w3 : w2;
    return b1 ? hi : lo;
}

// Per-lane conditions as wave lane masks: a comparison becomes a 64-bit mask in
// scalar registers, masks combine with scalar ALU operations (and, or, xor on
// whole wavefronts), and a mask turns back into a per-lane condition for a
// vector select at no vector cost.  Used inside the walk, where every lane of
// the wave that is still active runs the same code.
__device__ __forceinline__ uint64_t lanes(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ bool lane(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Word (hi, lo) of four: word 2*hi + lo (three vector selects).
__device__ __forceinline__ uint32_t pick4b(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, bool lo,
                                           bool hi) {
    const uint32_t a = lo ? w1 : w0;
    const uint32_t b = lo ? w3 : w2;
    return hi ? b : a;
}

// Neighbour field across the face opposite the vertex of rank r (0..3) in a
// record; `back` is the field of the face the walk entered through and `ra`
// the rank of the vertex opposite it (used by Tet16 only).
template <int LAYOUT>
__device__ __forceinline__ uint32_t next_field(const Rec& R, int r, uint32_t back, int ra) {
    if (LAYOUT == kTet16) {
        return back ^ pick4(R.n0, R.n1, R.n2, 0u, ra) ^ pick4(R.n0, R.n1, R.n2, 0u, r);
    } else {
        return pick4(R.n0, R.n1, R.n2, R.n3, r);
    }
}

__device__ __forceinline__ float4 load_pt(const Mem& M, uint32_t id) {
    const u32x3 a = sbuf_load_b96(M.pts, id, 0u, 0u, 0);
    return make_float4(__uint_as_float(a[0]), __uint_as_float(a[1]), __uint_as_float(a[2]), 0.0f);
}

struct Frame {
    float ux, uy, uz;   // u (Eq. 1)
    float vx, vy, vz;   // v (Eq. 2)
    float pox, poy;     // projected origin (Eq. 4)
};

// 2-D determinant with both products rounded before the subtraction (no fused
// multiply-add), so that det(a, b) == -det(b, a) exactly.
__device__ __forceinline__ float det2(float ax, float ay, float bx, float by) {
#pragma clang fp contract(off)
    return ax * by - ay * bx;
}

// The sign tests of det2 as comparisons of the two rounded products: for
// finite values the rounded difference is negative, or not, exactly when the
// first product is below the second, or not.
__device__ __forceinline__ bool det2_neg(float ax, float ay, float bx, float by) {
#pragma clang fp contract(off)
    return ax * by < ay * bx;
}
__device__ __forceinline__ bool det2_nonneg(float ax, float ay, float bx, float by) {
#pragma clang fp contract(off)
    return ax * by >= ay * bx;
}

// Eq. 1-2 for direction n (not necessarily unit).  Index names: i = smallest
// component (lowest index of the smaller of the two non-largest ones), j = i+1,
// k = i+2 (mod 3), and the largest component is j or k.
__device__ __forceinline__ void specialized_basis(float nx, float ny, float nz, Frame& f) {
    const float ax = fabsf(nx), ay = fabsf(ny), az = fabsf(nz);
    const int mx = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    const int o1 = mx == 0 ? 1 : 0;    // the two other indices, increasing
    const int o2 = mx == 2 ? 1 : 2;
    const float a1 = o1 == 0 ? ax : ay;
    const float a2 = o2 == 1 ? ay : az;
    const int mn = a2 < a1 ? o2 : o1;
    const float ni = mn == 0 ? nx : (mn == 1 ? ny : nz);   // cyclic from mn
    const float nj = mn == 0 ? ny : (mn == 1 ? nz : nx);
    const float nk = mn == 0 ? nz : (mn == 1 ? nx : ny);
    const bool max_is_j = mx == (mn == 2 ? 0 : mn + 1);
    const float nmax = max_is_j ? nj : nk;
    // u_i = 0, u_j = n_k / n_max, u_k = -n_j / n_max (one of them is +-1 exactly)
    const float uj = max_is_j ? nk / nmax : 1.0f;
    const float uk = max_is_j ? -1.0f : -nj / nmax;
    // v = (n x u) / |(n x u)_i|: v_i = -sign(n_max), v_{j,k} = sign(n_max) n_i n_{j,k} / (n_j^2 + n_k^2)
    const float s = nmax > 0.0f ? 1.0f : -1.0f;
    const float w = 1.0f / (nj * nj + nk * nk);
    const float vi = -s;
    const float vj = s * ni * nj * w;
    const float vk = s * ni * nk * w;
    f.ux = mn == 0 ? 0.0f : (mn == 1 ? uk : uj);
    f.uy = mn == 1 ? 0.0f : (mn == 2 ? uk : uj);
    f.uz = mn == 2 ? 0.0f : (mn == 0 ? uk : uj);
    f.vx = mn == 0 ? vi : (mn == 1 ? vk : vj);
    f.vy = mn == 1 ? vi : (mn == 2 ? vk : vj);
    f.vz = mn == 2 ? vi : (mn == 0 ? vk : vj);
}

__device__ __forceinline__ void set_origin(Frame& f, float ox, float oy, float oz) {
    f.pox = fmaf(f.ux, ox, fmaf(f.uy, oy, f.uz * oz));
    f.poy = fmaf(f.vx, ox, fmaf(f.vy, oy, f.vz * oz));
}

__device__ __forceinline__ void project(const Frame& f, float4 p, float& qx, float& qy) {
    qx = fmaf(f.ux, p.x, fmaf(f.uy, p.y, fmaf(f.uz, p.z, -f.pox)));
    qy = fmaf(f.vx, p.x, fmaf(f.vy, p.y, fmaf(f.vz, p.z, -f.poy)));
}

// parameter along the ray (in units of its direction) of P's orthogonal projection
struct Depth {
    float gx, gy, gz, go;
};

__device__ __forceinline__ void set_depth(Depth& g, float dx, float dy, float dz, float ox, float oy,
                                          float oz) {
    const float inv = 1.0f / fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    g.gx = dx * inv;
    g.gy = dy * inv;
    g.gz = dz * inv;
    g.go = fmaf(g.gx, ox, fmaf(g.gy, oy, g.gz * oz));
}

__device__ __forceinline__ float depth(const Depth& g, float4 p) {
    return fmaf(g.gx, p.x, fmaf(g.gy, p.y, fmaf(g.gz, p.z, -g.go)));
}

// Algorithm 1: which of the three kept vertices the exit face drops.
__device__ __forceinline__ int exit_slot(float q0x, float q0y, float q1x, float q1y, float q2x,
                                         float q2y, float q3x, float q3y) {
    const float d0 = det2(q3x, q3y, q0x, q0y);
    const float d1 = det2(q3x, q3y, q1x, q1y);
    const float d2 = det2(q3x, q3y, q2x, q2y);
    return d0 < 0.0f ? (d2 >= 0.0f ? 1 : 0) : (d1 < 0.0f ? 2 : 0);
}

// Precision variant: threshold, the line its float64 decisions follow, and a
// count of the steps decided in float64.
// Ray walks (ray6 given) decide in float64 along the ray as given: origin and
// direction are read back from the lane's copy in LDS (ray6[k * kRayStash], k =
// 0..5; rare: unsure steps only).  The float32
// basis leans from the direction by float32 rounding, so float64 decisions in
// it would answer for a slightly different ray; the unsure test covers that
// lean as it covers float32 rounding, so the float32 decisions it lets stand
// hold for the ray as given too.  Location walks (ray6 null) follow the segment
// their float32 basis projects along, from (ox, oy, oz).
// A float64 decision whose determinant is zero to within float64 rounding is a
// tie: the ray meets a vertex or edge exactly, or lies in a face plane (a ray
// along the mesh boundary).  Such ties are flagged (degen) so the ray can take
// the closest hit by its definition; allow_degen decides them by Algorithm 1's
// plain inequalities instead.
struct Prec {
    float eps;
    float ox, oy, oz;
    int32_t n64;
    bool degen = false;
    bool allow_degen = true;
    const float* ray6 = nullptr;
};

// Stride of the per-lane ray copies in LDS (threads per block at most).
constexpr int kRayStash = 256;

// A float64 projection of a point carries an absolute error of a few units of
// float64 rounding of the coordinates (about 1e-16 of the scene's size S), so a
// determinant of two projected points a, b is decided to within
// 1e-16 S (|a|_1 + |b|_1); anything within 1e-14 S (|a|_1 + |b|_1) is a tie.
constexpr double kTie64 = 1e-14;

// float64 2-D determinant, both products rounded (as det2)
__device__ __forceinline__ double det2d(double ax, double ay, double bx, double by) {
#pragma clang fp contract(off)
    return ax * by - ay * bx;
}

// The frame of the float64 decisions: a basis (u, v) and an origin, in double.
// A point's 2-D coordinates are u.(P - O), v.(P - O): the difference first,
// exact for float32 inputs of like magnitude.
struct Frame64 {
    double ux, uy, uz, vx, vy, vz;
    double ox, oy, oz;
};

// The float32 basis, widened (location walks follow the line it projects along).
__device__ __forceinline__ Frame64 frame64_of(const Frame& f, float ox, float oy, float oz) {
    return Frame64{double(f.ux), double(f.uy), double(f.uz), double(f.vx), double(f.vy), double(f.vz),
                   double(ox), double(oy), double(oz)};
}

__device__ __forceinline__ void project64(const Frame64& F, float4 p, double& qx, double& qy) {
    const double rx = double(p.x) - F.ox, ry = double(p.y) - F.oy, rz = double(p.z) - F.oz;
    qx = fma(F.ux, rx, fma(F.uy, ry, F.uz * rz));
    qy = fma(F.vx, rx, fma(F.vy, ry, F.vz * rz));
}

// Along the direction d as given, the 2-D determinant of two projected points
// a, b is, up to a positive factor, the triple product d . ((a - O) x (b - O)):
// the projection's basis (u, v) is orthogonal to d with u x v along +d.  So a
// ray walk decides in float64 with d itself and no basis.  The products are
// exact for float32 inputs up to the last sums; anything within 1e-14 of the
// product of the three vectors' 1-norms is a tie.
__device__ __forceinline__ double triple64(double dx, double dy, double dz, double ax, double ay, double az,
                                           double bx, double by, double bz, double& scale) {
    scale = (fabs(dx) + fabs(dy) + fabs(dz)) * (fabs(ax) + fabs(ay) + fabs(az)) * (fabs(bx) + fabs(by) + fabs(bz));
    return fma(dx, ay * bz - az * by, fma(dy, az * bx - ax * bz, dz * (ax * by - ay * bx)));
}

// Algorithm 1 on float64 determinants of the kept vertices a0..a2 and P.
// EXACT: a ray walk (pc.ray6 given), decided along the ray as given.
template <bool EXACT>
__device__ int exit_slot64(const Mem& M, const Frame& f, Prec& pc, int32_t a0, int32_t a1,
                           int32_t a2, float4 P) {
    if (EXACT) {
        // a ray walk: along the ray as given
        const float* st = pc.ray6;
        const double ox = st[0], oy = st[kRayStash], oz = st[2 * kRayStash];
        const double dx = st[3 * kRayStash], dy = st[4 * kRayStash], dz = st[5 * kRayStash];
        const double rx = double(P.x) - ox, ry = double(P.y) - oy, rz = double(P.z) - oz;
        // d . (r3 x r_k) = (d x r3) . r_k: the cross product once for the three
        const double cx = dy * rz - dz * ry, cy = dz * rx - dx * rz, cz = dx * ry - dy * rx;
        const double s3 = (fabs(dx) + fabs(dy) + fabs(dz)) * (fabs(rx) + fabs(ry) + fabs(rz));
        double d[3], sc[3];
        const int32_t ids[3] = {a0, a1, a2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 Q = load_pt(M, uint32_t(ids[k]));
            const double qx = double(Q.x) - ox, qy = double(Q.y) - oy, qz = double(Q.z) - oz;
            d[k] = fma(cx, qx, fma(cy, qy, cz * qz));
            sc[k] = s3 * (fabs(qx) + fabs(qy) + fabs(qz));
        }
        if (!pc.allow_degen)
            pc.degen |= fabs(d[0]) <= kTie64 * sc[0] || fabs(d[1]) <= kTie64 * sc[1] || fabs(d[2]) <= kTie64 * sc[2];
        return d[0] < 0.0 ? (d[2] >= 0.0 ? 1 : 0) : (d[1] < 0.0 ? 2 : 0);
    }
    const Frame64 F = frame64_of(f, pc.ox, pc.oy, pc.oz);
    double x0, y0, x1, y1, x2, y2, x3, y3;
    project64(F, load_pt(M, uint32_t(a0)), x0, y0);
    project64(F, load_pt(M, uint32_t(a1)), x1, y1);
    project64(F, load_pt(M, uint32_t(a2)), x2, y2);
    project64(F, P, x3, y3);
    const double d0 = det2d(x3, y3, x0, y0);
    const double d1 = det2d(x3, y3, x1, y1);
    const double d2 = det2d(x3, y3, x2, y2);
    if (!pc.allow_degen) {
        const double S = kTie64 * (1.0 + fabs(F.ox) + fabs(F.oy) + fabs(F.oz));
        const double s3 = fabs(x3) + fabs(y3);
        pc.degen |= fabs(d0) <= S * (s3 + fabs(x0) + fabs(y0)) ||
                    fabs(d1) <= S * (s3 + fabs(x1) + fabs(y1)) ||
                    fabs(d2) <= S * (s3 + fabs(x2) + fabs(y2));
    }
    return d0 < 0.0 ? (d2 >= 0.0 ? 1 : 0) : (d1 < 0.0 ? 2 : 0);
}

// The kept face (ids a, 2-D points q, depths e) in counter-clockwise order
// around the ray, the neighbour field across it, and `cur`: the field that the
// next tet's record holds for this face -- the id of the tet the face belongs
// to, or the constrained-face field when a secondary ray starts on it.
struct Walk {
    int32_t a0, a1, a2;
    float q0x, q0y, q1x, q1y, q2x, q2y;
    float e0, e1, e2;
    uint32_t next;
    int32_t cur;
    int32_t vxn;   // Tet32N: xor-sum of the tet `next` refers to
};

__device__ __forceinline__ void make_ccw(Walk& w) {
    const float o = det2(w.q1x - w.q0x, w.q1y - w.q0y, w.q2x - w.q0x, w.q2y - w.q0y);
    const bool sw = o < 0.0f;
    const int32_t a1 = w.a1, a2 = w.a2;
    const float q1x = w.q1x, q1y = w.q1y, q2x = w.q2x, q2y = w.q2y, e1 = w.e1, e2 = w.e2;
    w.a1 = sw ? a2 : a1; w.a2 = sw ? a1 : a2;
    w.q1x = sw ? q2x : q1x; w.q2x = sw ? q1x : q2x;
    w.q1y = sw ? q2y : q1y; w.q2y = sw ? q1y : q2y;
    w.e1 = sw ? e2 : e1; w.e2 = sw ? e1 : e2;
}

// make_ccw with the orientation decided in float64 (precision variant): the
// three face vertices A, B, C (in slot order) are projected in float64 about
// the origin X.  A face that contains the ray's 2-D origin on or near one of
// its edges -- a ray along a mesh edge starts on two such faces -- has a
// float32 orientation of random sign, and a wrongly oriented face misleads
// every later exit decision.
// Returns true when the orientation is a float64 tie (the face's projection is
// a segment: its plane contains the ray direction).
// dir (ray walks): the orientation is that of the projection along the ray's
// direction as given, the sign of dir . ((B - A) x (C - A)); else along the
// float32 basis of f from X.
__device__ __forceinline__ bool make_ccw64(const Frame& f, float Xx, float Xy, float Xz, const float* dir,
                                           float4 A, float4 B, float4 C, Walk& w) {
    double o, tol;
    if (dir) {
        double sc;
        o = triple64(double(dir[0]), double(dir[1]), double(dir[2]), double(B.x) - A.x, double(B.y) - A.y,
                     double(B.z) - A.z, double(C.x) - A.x, double(C.y) - A.y, double(C.z) - A.z, sc);
        tol = kTie64 * sc;
    } else {
        const Frame64 F = frame64_of(f, Xx, Xy, Xz);
        double x0, y0, x1, y1, x2, y2;
        project64(F, A, x0, y0);
        project64(F, B, x1, y1);
        project64(F, C, x2, y2);
        const double ex = x1 - x0, ey = y1 - y0, fx = x2 - x0, fy = y2 - y0;
        o = det2d(ex, ey, fx, fy);
        tol = kTie64 * (1.0 + fabs(F.ox) + fabs(F.oy) + fabs(F.oz)) * (fabs(ex) + fabs(ey) + fabs(fx) + fabs(fy));
    }
    const bool sw = o < 0.0;
    const int32_t a1 = w.a1, a2 = w.a2;
    const float q1x = w.q1x, q1y = w.q1y, q2x = w.q2x, q2y = w.q2y, e1 = w.e1, e2 = w.e2;
    w.a1 = sw ? a2 : a1; w.a2 = sw ? a1 : a2;
    w.q1x = sw ? q2x : q1x; w.q2x = sw ? q1x : q2x;
    w.q1y = sw ? q2y : q1y; w.q2y = sw ? q1y : q2y;
    w.e1 = sw ? e2 : e1; w.e2 = sw ? e1 : e2;
    return fabs(o) <= tol;
}

// One step of the walk (Algorithm 1 with Algorithms 4-5 or 6-7), branch-free
// (apart from the rare float64 re-evaluation of the precision variant).
// LINK (Tet16): w.cur carries the xor of the previous tet's field and w.next
// instead of the field itself, before and after the step.  The step then
// updates both in place (w.cur ^= NX[a] ^ NX[b], w.next ^= w.cur) rather than
// rotating previous / current / next through registers.
// R is the record of w.next.  PIPE: as soon as the step knows the next tet,
// it loads that tet's record into *ahead, so the load is in flight while the
// step finishes; for a lane whose walk ends there the index is a face flag or
// the boundary mark, beyond the record count, and the buffer bound makes the
// load return zeros without touching memory.
// unsure (given, with PREC false): the step only tests whether its float32
// decision is unsure -- the test of the precision variant -- and reports it.
// EXACT (a ray walk of the precision variant): unsure steps are decided along
// the ray as given (pc.ray6), else along the float32 basis.
template <bool DEPTH, int LAYOUT, bool PREC, bool LINK = false, bool PIPE = false, bool EXACT = false>
__device__ __forceinline__ void walk_step_rec(const Mem& M, const Frame& f, const Depth& g, Walk& w,
                                              Prec& pc, const Rec& R, Rec* ahead, bool* unsure_out = nullptr) {
    const uint32_t tet = w.next;
    const int32_t id3 = w.a0 ^ w.a1 ^ w.a2 ^ (LAYOUT == kTet32N ? w.vxn : R.vx);
    const float4 P = load_pt(M, uint32_t(id3));
    float q3x, q3y;
    project(f, P, q3x, q3y);
    // Algorithm 1 as lane masks: the exit face drops slot 1 when det(q3,q0) < 0 and
    // det(q3,q2) >= 0, slot 2 when det(q3,q0) >= 0 and det(q3,q1) < 0, else slot 0
    uint64_t N0, N1, P2;
    bool unsure = false;
    if (PREC || unsure_out) {
        // the determinants as values, for the unsure test too; their signs decide as
        // the comparisons of the rounded products do (a rounded difference of finite
        // values is negative exactly when the first product is below the second)
        const float d0 = det2(q3x, q3y, w.q0x, w.q0y);
        const float d1 = det2(q3x, q3y, w.q1x, w.q1y);
        const float d2 = det2(q3x, q3y, w.q2x, w.q2y);
        N0 = lanes(d0 < 0.0f);
        N1 = lanes(d1 < 0.0f);
        P2 = lanes(d2 >= 0.0f);
        // |det(q3, q_i)| <= eps (|q3|_1 + |q_i|_1), evaluated in full (no short
        // circuit: branches would cost more than the tests)
        const float es3 = pc.eps * (fabsf(q3x) + fabsf(q3y));
        unsure = (fabsf(d0) <= fmaf(pc.eps, fabsf(w.q0x) + fabsf(w.q0y), es3)) |
                 (fabsf(d1) <= fmaf(pc.eps, fabsf(w.q1x) + fabsf(w.q1y), es3)) |
                 (fabsf(d2) <= fmaf(pc.eps, fabsf(w.q2x) + fabsf(w.q2y), es3));
        if (unsure_out) *unsure_out = unsure;
    } else {
        N0 = lanes(det2_neg(q3x, q3y, w.q0x, w.q0y));
        N1 = lanes(det2_neg(q3x, q3y, w.q1x, w.q1y));
        P2 = lanes(det2_nonneg(q3x, q3y, w.q2x, w.q2y));
    }
    uint64_t S1 = N0 & P2, S2 = N1 & ~N0;
    if (PREC) {
        // the unsure lanes' decisions are replaced by the float64 ones; a wave with
        // no unsure lane (nearly every step) skips all of it on one scalar branch
        const uint64_t U = lanes(unsure);
        if (U) {
            int e = 0;
            if (unsure) {
                e = exit_slot64<EXACT>(M, f, pc, w.a0, w.a1, w.a2, P);
                ++pc.n64;
            }
            S1 = (S1 & ~U) | lanes(unsure && e == 1);
            S2 = (S2 & ~U) | lanes(unsure && e == 2);
        }
    }
    const bool s1 = lane(S1), s2 = lane(S2), s0 = lane(~(S1 | S2));
    const int32_t x = s1 ? w.a1 : (s2 ? w.a2 : w.a0);
    bool rlo = false, rhi = false;
    if (LAYOUT != kTet32) {
        // rank of the exit vertex x among the tet's four ids (Algorithms 4-5), as its
        // two bits: the count of ids below x is odd (lo) / at least 2 (hi)
        const uint64_t b0 = lanes(w.a0 < x), b1 = lanes(w.a1 < x), b2 = lanes(w.a2 < x), b3 = lanes(id3 < x);
        rlo = lane(b0 ^ b1 ^ b2 ^ b3);
        rhi = lane(((b0 | b1) & (b2 | b3)) | (b0 & b1) | (b2 & b3));
    }
    if (LAYOUT == kTet32) {
        // Algorithm 3: the neighbour field beside the stored id equal to x, else N3
        const bool e0 = lane(lanes(x == int32_t(R.w0)));
        const bool e1 = lane(lanes(x == int32_t(R.w1)));
        const bool e2 = lane(lanes(x == int32_t(R.w2)));
        w.next = e0 ? R.n0 : (e1 ? R.n1 : (e2 ? R.n2 : R.n3));
        w.cur = int32_t(tet);
    } else if (LAYOUT == kTet16) {
        // Algorithms 6-7: next = prev ^ NX[rank of id3] ^ NX[rank of x], NX3 = 0
        const uint64_t c0 = lanes(w.a0 < id3), c1 = lanes(w.a1 < id3), c2 = lanes(w.a2 < id3);
        const bool alo = lane(c0 ^ c1 ^ c2);
        const bool ahi = lane((c0 & c1) | (c2 & (c0 | c1)));
        const uint32_t xa = pick4b(R.n0, R.n1, R.n2, 0u, alo, ahi);
        const uint32_t xb = pick4b(R.n0, R.n1, R.n2, 0u, rlo, rhi);
        if (LINK) {
            w.cur = int32_t(uint32_t(w.cur) ^ xa ^ xb);   // prev ^ tet ^ NX[a] ^ NX[b] = tet ^ next
            w.next = uint32_t(w.cur) ^ tet;
        } else {
            w.next = uint32_t(w.cur) ^ xa ^ xb;
            w.cur = int32_t(tet);
        }
    } else {
        w.next = pick4b(R.n0, R.n1, R.n2, R.n3, rlo, rhi);
        w.cur = int32_t(tet);
    }
    if (LAYOUT == kTet32N) w.vxn = int32_t(pick4b(R.w0, R.w1, R.w2, R.w3, rlo, rhi));
    if (PIPE) *ahead = load_rec<LAYOUT>(M, w.next);
    w.a0 = s0 ? id3 : w.a0;  w.q0x = s0 ? q3x : w.q0x;  w.q0y = s0 ? q3y : w.q0y;
    w.a1 = s1 ? id3 : w.a1;  w.q1x = s1 ? q3x : w.q1x;  w.q1y = s1 ? q3y : w.q1y;
    w.a2 = s2 ? id3 : w.a2;  w.q2x = s2 ? q3x : w.q2x;  w.q2y = s2 ? q3y : w.q2y;
    if (DEPTH) {
        const float e3 = depth(g, P);
        w.e0 = s0 ? e3 : w.e0;
        w.e1 = s1 ? e3 : w.e1;
        w.e2 = s2 ? e3 : w.e2;
    }
}

template <bool DEPTH, int LAYOUT, bool PREC, bool LINK = false>
__device__ __forceinline__ void walk_step(const Mem& M, const Frame& f, const Depth& g, Walk& w,
                                          Prec& pc) {
    const Rec R = load_rec<LAYOUT>(M, w.next);
    walk_step_rec<DEPTH, LAYOUT, PREC, LINK, false>(M, f, g, w, pc, R, nullptr);
}

// Exit face of tet `tet` (vertex ids v[0..3]) for the line X + s*D: the face
// whose outward normal has n.D > 0 with the smallest crossing parameter s.
// Fills the walk state (face ids, 2-D points in frame f, depths in g, the
// neighbour field) and returns s (+inf when no face is front-facing).
// The plane tests run in T: float, or double in the precision variant.
// EXACT (ray walks of the precision variant): D is the ray's direction as given,
// and the float64 tests and orientation follow it (see Prec).
template <bool DEPTH, int LAYOUT, typename T, bool EXACT = false>
__device__ float start_in_tet(const DevMesh& m, const Mem& M, int32_t tet, const int32_t v[4],
                              float Xx, float Xy, float Xz, float Dx, float Dy, float Dz,
                              const Frame& f, const Depth& g, Walk& w, bool* degen = nullptr) {
    float4 P[4];
    T rx[4], ry[4], rz[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        P[k] = load_pt(M, uint32_t(v[k]));
        rx[k] = T(P[k].x) - T(Xx);
        ry[k] = T(P[k].y) - T(Xy);
        rz[k] = T(P[k].z) - T(Xz);
    }
    // In float64 a location walk's plane tests use the direction its walk
    // projects along, u x v of the float32 basis, rather than D: the two differ
    // by float32 rounding, and for a segment that grazes an edge the start face
    // chosen for D need not surround the origin in the walk's projection.  A
    // ray walk's float64 decisions follow D itself.
    T ex = T(Dx), ey = T(Dy), ez = T(Dz);
    if (std::is_same<T, double>::value && !EXACT) {
        ex = T(f.uy) * T(f.vz) - T(f.uz) * T(f.vy);
        ey = T(f.uz) * T(f.vx) - T(f.ux) * T(f.vz);
        ez = T(f.ux) * T(f.vy) - T(f.uy) * T(f.vx);
    }
    T best = T(INFINITY);
    int bj = -1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int A = j == 0 ? 1 : 0;
        const int B = j <= 1 ? 2 : 1;
        const int C = j <= 2 ? 3 : 2;
        const T e1x = rx[B] - rx[A], e1y = ry[B] - ry[A], e1z = rz[B] - rz[A];
        const T e2x = rx[C] - rx[A], e2y = ry[C] - ry[A], e2z = rz[C] - rz[A];
        T nx = e1y * e2z - e1z * e2y;
        T ny = e1z * e2x - e1x * e2z;
        T nz = e1x * e2y - e1y * e2x;
        const T side = nx * (rx[j] - rx[A]) + ny * (ry[j] - ry[A]) + nz * (rz[j] - rz[A]);
        if (side > T(0)) { nx = -nx; ny = -ny; nz = -nz; }
        const T nd = nx * ex + ny * ey + nz * ez;
        if (nd > T(0)) {
            const T s = (nx * rx[A] + ny * ry[A] + nz * rz[A]) / nd;
            if (s < best) { best = s; bj = j; }
        }
    }
    if (bj < 0) return INFINITY;
    // face ids (the three slots other than bj) and the neighbour across it;
    // selects rather than indexing, so the arrays stay in registers
    const float4 PA = bj == 0 ? P[1] : P[0];
    const float4 PB = bj <= 1 ? P[2] : P[1];
    const float4 PC = bj <= 2 ? P[3] : P[2];
    w.a0 = bj == 0 ? v[1] : v[0];
    w.a1 = bj <= 1 ? v[2] : v[1];
    w.a2 = bj <= 2 ? v[3] : v[2];
    project(f, PA, w.q0x, w.q0y);
    project(f, PB, w.q1x, w.q1y);
    project(f, PC, w.q2x, w.q2y);
    if (DEPTH) {
        w.e0 = depth(g, PA); w.e1 = depth(g, PB); w.e2 = depth(g, PC);
    }
    const int32_t x = bj == 0 ? v[0] : (bj == 1 ? v[1] : (bj == 2 ? v[2] : v[3]));
    const int r = (v[0] < x) + (v[1] < x) + (v[2] < x) + (v[3] < x);
    const Rec R = load_rec<LAYOUT>(M, uint32_t(tet));
    // Tet16 keeps N3 of every tet in a cold array for starts: N_r = N3 ^ NX_r
    w.next = LAYOUT == kTet16 ? next_field<kTet16>(R, r, uint32_t(m.n3[tet]), 3)
                              : next_field<kTet20>(R, r, 0u, 0);
    if (LAYOUT == kTet32N) w.vxn = int32_t(pick4(R.w0, R.w1, R.w2, R.w3, r));
    w.cur = tet;
    if (std::is_same<T, double>::value) {
        const float D[3] = {Dx, Dy, Dz};
        const bool tie = make_ccw64(f, Xx, Xy, Xz, EXACT ? D : nullptr, PA, PB, PC, w);
        if (degen) *degen = tie;
    } else {
        make_ccw(w);
    }
    return float(best);
}

// Point location (paper, Sec. "Locating points in a tetrahedral mesh"): the
// traversal itself, along the segment from the centroid S of a seed tet to the
// point; in each tet the crossing of the exit face is compared with the point
// (parameter 1).  Constrained faces are crossed (location ignores geometry).
// Returns the internal tet (its four ids in v) or TM_RAY_INVALID (outside) /
// TM_RAY_STEP_CAP.
template <int LAYOUT, bool PREC>
__device__ int32_t locate_point(const DevMesh& m, const Mem& M, float px, float py, float pz,
                                int32_t max_steps, float eps, int32_t v[4]) {
    int cx = int(floorf((px - m.lo[0]) * m.inv_cell[0]));
    int cy = int(floorf((py - m.lo[1]) * m.inv_cell[1]));
    int cz = int(floorf((pz - m.lo[2]) * m.inv_cell[2]));
    cx = min(max(cx, 0), m.G - 1);
    cy = min(max(cy, 0), m.G - 1);
    cz = min(max(cz, 0), m.G - 1);
    const int32_t seed = m.seed[(cx * m.G + cy) * m.G + cz];
    const int4 sv = reinterpret_cast<const int4*>(m.tetv)[seed];
    v[0] = sv.x; v[1] = sv.y; v[2] = sv.z; v[3] = sv.w;
    float Sx = 0.f, Sy = 0.f, Sz = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 p = load_pt(M, uint32_t(v[k]));
        Sx += p.x; Sy += p.y; Sz += p.z;
    }
    Sx *= 0.25f; Sy *= 0.25f; Sz *= 0.25f;
    const float Dx = px - Sx, Dy = py - Sy, Dz = pz - Sz;
    if (Dx == 0.0f && Dy == 0.0f && Dz == 0.0f) return seed;
    Frame f;
    specialized_basis(Dx, Dy, Dz, f);
    set_origin(f, Sx, Sy, Sz);
    Depth g;
    set_depth(g, Dx, Dy, Dz, Sx, Sy, Sz);
    Walk w;
    using T = typename std::conditional<PREC, double, float>::type;
    const float s0 = start_in_tet<true, LAYOUT, T>(m, M, seed, v, Sx, Sy, Sz, Dx, Dy, Dz, f, g, w);
    Prec pc{eps, Sx, Sy, Sz, 0};   // ties decided by the plain inequalities
    if (!(s0 < 1.0f)) return seed;
    for (int32_t step = 0; step < max_steps; ++step) {
        const uint32_t field = w.next;
        int32_t tet;
        if (field == kBoundary) return TM_RAY_INVALID;
        if (field & 0x80000000u) {
            const uint32_t cf = field & kIdMask;
            if (cf >= uint32_t(m.ntri)) return TM_RAY_STEP_CAP;
            const int4 pr = reinterpret_cast<const int4*>(m.cft)[cf];
            const bool other_neg = pr.x == w.cur;
            tet = other_neg ? pr.y : pr.x;
            if (tet < 0) return TM_RAY_INVALID;
            w.cur = int32_t(field);   // the other tet's record holds this field for the face
            w.vxn = other_neg ? pr.w : pr.z;
        } else {
            tet = int32_t(field);
        }
        if (uint32_t(tet) >= uint32_t(m.nt)) return TM_RAY_STEP_CAP;
        w.next = uint32_t(tet);
        const int32_t a0 = w.a0, a1 = w.a1, a2 = w.a2;
        walk_step<true, LAYOUT, PREC>(M, f, g, w, pc);
        w.cur = tet;
        // the vertex the new face dropped: the tet is {a0, a1, a2, id3}
        const int32_t x = (w.a0 != a0) ? a0 : ((w.a1 != a1) ? a1 : a2);
        // the segment leaves this tet through the new face at the depth of the
        // 2-D origin's barycentric combination; at or beyond 1 the point is inside
        const float l0 = det2(w.q1x, w.q1y, w.q2x, w.q2y);
        const float l1 = det2(w.q2x, w.q2y, w.q0x, w.q0y);
        const float l2 = det2(w.q0x, w.q0y, w.q1x, w.q1y);
        if (l0 * (w.e0 - 1.0f) + l1 * (w.e1 - 1.0f) + l2 * (w.e2 - 1.0f) >= 0.0f) {
            v[0] = w.a0; v[1] = w.a1; v[2] = w.a2; v[3] = x;
            return tet;
        }
    }
    return TM_RAY_STEP_CAP;
}

// Precision variant: make sure the start tet contains the point, with
// orientations in float64.  The straight-line location decides its last
// crossing in float32, so a point within rounding distance of a face, edge or
// vertex (a ray that starts on a mesh edge) can land in a neighbour of the tet
// that holds it; a walk started in a tet that does not contain its origin
// breaks the invariant that the entry face surrounds the ray.  While the point
// is on the outer side of a face, step across that face (at most 16 times).
// v receives the ascending vertex ids of the returned tet.
template <int LAYOUT>
__device__ int32_t contain64(const DevMesh& m, const Mem& M, int32_t tet, int32_t v[4], float px,
                             float py, float pz) {
    for (int it = 0; it < 16; ++it) {
        const int4 sv = reinterpret_cast<const int4*>(m.tetv)[tet];
        v[0] = sv.x; v[1] = sv.y; v[2] = sv.z; v[3] = sv.w;
        double X[4], Y[4], Z[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4 P = load_pt(M, uint32_t(v[k]));
            X[k] = double(P.x) - double(px);
            Y[k] = double(P.y) - double(py);
            Z[k] = double(P.z) - double(pz);
        }
        // orientation of the tet, and of each face with the point in place of its
        // opposite vertex (the point is the origin of these coordinates)
        const double e1x = X[1] - X[0], e1y = Y[1] - Y[0], e1z = Z[1] - Z[0];
        const double e2x = X[2] - X[0], e2y = Y[2] - Y[0], e2z = Z[2] - Z[0];
        const double e3x = X[3] - X[0], e3y = Y[3] - Y[0], e3z = Z[3] - Z[0];
        const double vol = e1x * (e2y * e3z - e2z * e3y) - e1y * (e2x * e3z - e2z * e3x) +
                           e1z * (e2x * e3y - e2y * e3x);
        int out = -1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int A = j == 0 ? 1 : 0;
            const int B = j <= 1 ? 2 : 1;
            const int C = j <= 2 ? 3 : 2;
            // triple product of the face vertices seen from the point, signed as the
            // tet's volume with the point replacing vertex j
            double t = X[A] * (Y[B] * Z[C] - Z[B] * Y[C]) - Y[A] * (X[B] * Z[C] - Z[B] * X[C]) +
                       Z[A] * (X[B] * Y[C] - Y[B] * X[C]);
            if (j == 1 || j == 3) t = -t;   // odd permutations of (0, 1, 2, 3)
            if (out < 0 && t * vol < 0.0) out = j;
        }
        if (out < 0) return tet;
        const Rec R = load_rec<LAYOUT>(M, uint32_t(tet));
        const uint32_t field = LAYOUT == kTet16 ? next_field<kTet16>(R, out, uint32_t(m.n3[tet]), 3)
                                                : pick4(R.n0, R.n1, R.n2, R.n3, out);
        int32_t nt;
        if (field == kBoundary) return tet;
        if (field & 0x80000000u) {
            const uint32_t cf = field & kIdMask;
            if (cf >= uint32_t(m.ntri)) return tet;
            const int4 pr = reinterpret_cast<const int4*>(m.cft)[cf];
            nt = pr.x == tet ? pr.y : pr.x;
            if (nt < 0) return tet;
        } else {
            nt = int32_t(field);
        }
        if (uint32_t(nt) >= uint32_t(m.nt)) return tet;
        tet = nt;
    }
    const int4 sv = reinterpret_cast<const int4*>(m.tetv)[tet];
    v[0] = sv.x; v[1] = sv.y; v[2] = sv.z; v[3] = sv.w;
    return tet;
}

// Everything a lane keeps for one ray between set-up and the result.
struct Ray {
    Frame f;
    Depth g;
    Walk w;
    float tmax;
    int32_t steps;
};

struct Knobs {
    float eps;                // precision variant threshold (PREC kernels)
    uint32_t xcd_blocks;      // block renumbering for the XCDs: 0 = one contiguous range per
                              // XCD, > 0 = runs of this many consecutive blocks per XCD
    TieList ties;             // PREC one-pass kernel: where its ties are listed (count null: none)
};

__device__ __forceinline__ void write_result(const RayArgs& r, int64_t i, int32_t code, float t,
                                             float b1, float b2, int32_t front, int32_t back,
                                             int32_t steps, int32_t n64 = 0) {
    r.tri[i] = code;
    r.t[i] = t;
    reinterpret_cast<float2*>(r.bary)[i] = make_float2(b1, b2);
    if (r.hit_tets) reinterpret_cast<int2*>(r.hit_tets)[i] = make_int2(front, back);
    if (r.steps) r.steps[i] = steps;
    if (r.fp64_steps) r.fp64_steps[i] = n64;
}

__device__ __forceinline__ void write_code(const RayArgs& r, int64_t i, int32_t code, int32_t steps,
                                           int32_t n64 = 0) {
    const float NaN = __int_as_float(0x7fc00000);
    write_result(r, i, code, NaN, NaN, NaN, -1, -1, steps, n64);
}

// Set-up of ray i.  Returns true when the ray needs walking (state in s);
// false when its result is already written.  Precision variant: *degen reports
// a float64 tie in the orientation of the start face, and *lost that no start
// tet was found (the origin lies on the mesh boundary, or no face of the start
// tet faces the ray).
template <bool TMAX, int LAYOUT, bool PREC>
__device__ bool setup_ray(const DevMesh& m, const Mem& M, const RayArgs& r, int64_t i, Ray& s,
                          float eps, bool* degen = nullptr, bool* lost = nullptr) {
    const float ox = r.orig[3 * i], oy = r.orig[3 * i + 1], oz = r.orig[3 * i + 2];
    const float dx = r.dir[3 * i], dy = r.dir[3 * i + 1], dz = r.dir[3 * i + 2];
    s.tmax = (TMAX && r.tmax) ? r.tmax[i] : INFINITY;
    s.steps = 0;
    const float dd = dx * dx + dy * dy + dz * dz;
    if (!(dd > 0.0f) || !isfinite(dd) || !isfinite(ox + oy + oz) || isnan(s.tmax)) {
        write_code(r, i, TM_RAY_INVALID, 0);
        return false;
    }
    const int32_t sf = r.start_face ? r.start_face[i] : -1;
    if (sf >= 0) {
        // secondary ray: start in the tet on the side of the face that dir points into
        if (sf >= m.ntri) { write_code(r, i, TM_RAY_INVALID, 0); return false; }
        const int4 fv = reinterpret_cast<const int4*>(m.cfv)[sf];
        const int4 ft = reinterpret_cast<const int4*>(m.cft)[sf];
        const float4 PA = load_pt(M, uint32_t(fv.x)), PB = load_pt(M, uint32_t(fv.y)),
                     PC = load_pt(M, uint32_t(fv.z));
        const float e1x = PB.x - PA.x, e1y = PB.y - PA.y, e1z = PB.z - PA.z;
        const float e2x = PC.x - PA.x, e2y = PC.y - PA.y, e2z = PC.z - PA.z;
        const float nd = (e1y * e2z - e1z * e2y) * dx + (e1z * e2x - e1x * e2z) * dy +
                         (e1x * e2y - e1y * e2x) * dz;
        if (nd == 0.0f) { write_code(r, i, TM_RAY_INVALID, 0); return false; }
        const int32_t start = nd > 0.0f ? ft.x : ft.y;
        s.w.vxn = nd > 0.0f ? ft.z : ft.w;
        if (start < 0) { write_code(r, i, TM_RAY_MISS, 0); return false; }
        specialized_basis(dx, dy, dz, s.f);
        set_origin(s.f, ox, oy, oz);
        if (TMAX) set_depth(s.g, dx, dy, dz, ox, oy, oz);
        s.w.a0 = fv.x; s.w.a1 = fv.y; s.w.a2 = fv.z;
        project(s.f, PA, s.w.q0x, s.w.q0y);
        project(s.f, PB, s.w.q1x, s.w.q1y);
        project(s.f, PC, s.w.q2x, s.w.q2y);
        if (TMAX) { s.w.e0 = depth(s.g, PA); s.w.e1 = depth(s.g, PB); s.w.e2 = depth(s.g, PC); }
        if (PREC) {
            const float D[3] = {dx, dy, dz};
            const bool tie = make_ccw64(s.f, ox, oy, oz, D, PA, PB, PC, s.w);
            if (degen) *degen = tie;
        } else {
            make_ccw(s.w);
        }
        s.w.next = uint32_t(start);
        s.w.cur = int32_t(0x80000000u | uint32_t(sf));   // the start tet's field for this face
        return true;
    }
    int32_t v[4];
    int32_t tet;
    const int32_t st = r.start_tet ? r.start_tet[i] : -1;
    if (st >= 0) {
        if (st >= m.nt) { write_code(r, i, TM_RAY_INVALID, 0); return false; }
        tet = m.t_old2new[st];
        const int4 sv = reinterpret_cast<const int4*>(m.tetv)[tet];
        v[0] = sv.x; v[1] = sv.y; v[2] = sv.z; v[3] = sv.w;
    } else {
        tet = locate_point<LAYOUT, PREC>(m, M, ox, oy, oz, r.max_steps, eps, v);
        if (tet < 0) {
            if (lost) *lost = true;
            write_code(r, i, tet, 0);
            return false;
        }
    }
    if (PREC) tet = contain64<LAYOUT>(m, M, tet, v, ox, oy, oz);
    specialized_basis(dx, dy, dz, s.f);
    set_origin(s.f, ox, oy, oz);
    if (TMAX) set_depth(s.g, dx, dy, dz, ox, oy, oz);
    using T = typename std::conditional<PREC, double, float>::type;
    const float sx = start_in_tet<TMAX, LAYOUT, T, PREC>(m, M, tet, v, ox, oy, oz, dx, dy, dz, s.f, s.g, s.w, degen);
    if (!(sx < INFINITY)) {
        if (lost) *lost = true;
        write_code(r, i, TM_RAY_INVALID, 0);
        return false;
    }
    return true;
}

// Whether the walk of s goes on: the field ahead is a tet, the step cap is not
// reached and (with tmax) the face ahead is not entirely beyond tmax.
template <bool TMAX>
__device__ __forceinline__ bool walk_on(const Ray& s, int32_t max_steps) {
    bool go = (int32_t(s.w.next) >= 0) & (s.steps < max_steps);
    if (TMAX) go = go & !(fminf(s.w.e0, fminf(s.w.e1, s.w.e2)) > s.tmax);
    return go;
}

// The walk of a set-up ray until it stops, in the plain float32 form.  With
// STEPS false s.steps ends at 0: a per-lane step count costs a vector
// instruction per step, and it is only written when the caller asks for it.
template <bool TMAX, int LAYOUT, bool STEPS>
__device__ __forceinline__ void walk_ray(const Mem& M, Ray& s, int32_t max_steps) {
    Prec pc{0.0f, 0.0f, 0.0f, 0.0f, 0};
    if (LAYOUT == kTet16) s.w.cur ^= int32_t(s.w.next);   // the LINK form of walk_step
    Rec R = load_rec<LAYOUT>(M, s.w.next);
    while (walk_on<TMAX>(s, max_steps)) {
        walk_step_rec<TMAX, LAYOUT, false, true, true>(M, s.f, s.g, s.w, pc, R, &R);
        ++s.steps;
    }
    if (LAYOUT == kTet16) s.w.cur ^= int32_t(s.w.next);
    if (!STEPS) s.steps = 0;
}

// Result of a walk that stopped; the hit's t and barycentric weights come from
// the Moller-Trumbore form in float64 with the triangle's vertices in ascending
// caller-id order, so the weights are those of its 2nd and 3rd vertex.
template <bool TMAX>
__device__ void finish_ray(const DevMesh& m, const Mem& M, const RayArgs& r, int64_t i, const Ray& s,
                           int32_t n64 = 0) {
    // tested afresh here: reusing the walk loop's own test of the field would
    // carry its outcome through every step in scalar registers
    uint32_t nx = s.w.next;
    keep(nx);
    if (!(nx & 0x80000000u)) {
        // tmax early-out, else the step cap
        const bool beyond = TMAX && (fminf(s.w.e0, fminf(s.w.e1, s.w.e2)) > s.tmax);
        write_code(r, i, beyond ? TM_RAY_MISS : TM_RAY_STEP_CAP, s.steps, n64);
        return;
    }
    if (nx == kBoundary) { write_code(r, i, TM_RAY_MISS, s.steps, n64); return; }
    const uint32_t cf = nx & kIdMask;
    if (cf >= uint32_t(m.ntri)) { write_code(r, i, TM_RAY_STEP_CAP, s.steps, n64); return; }
    // reload the ray from memory rather than keeping it in registers through the walk
    asm volatile("" ::: "memory");
    const int4 fv = reinterpret_cast<const int4*>(m.cfv)[cf];
    const float4 A = load_pt(M, uint32_t(fv.x)), B = load_pt(M, uint32_t(fv.y)),
                 C = load_pt(M, uint32_t(fv.z));
    const double ox = r.orig[3 * i], oy = r.orig[3 * i + 1], oz = r.orig[3 * i + 2];
    const double Dx = r.dir[3 * i], Dy = r.dir[3 * i + 1], Dz = r.dir[3 * i + 2];
    const double e1x = double(B.x) - A.x, e1y = double(B.y) - A.y, e1z = double(B.z) - A.z;
    const double e2x = double(C.x) - A.x, e2y = double(C.y) - A.y, e2z = double(C.z) - A.z;
    const double sx = ox - A.x, sy = oy - A.y, sz = oz - A.z;
    const double px = Dy * e2z - Dz * e2y, py = Dz * e2x - Dx * e2z, pz = Dx * e2y - Dy * e2x;
    const double det = e1x * px + e1y * py + e1z * pz;
    const double inv = 1.0 / det;
    const double bu = (sx * px + sy * py + sz * pz) * inv;
    const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    const double bv = (Dx * qx + Dy * qy + Dz * qz) * inv;
    const double th = (e2x * qx + e2y * qy + e2z * qz) * inv;
    if (TMAX && th > double(s.tmax)) { write_code(r, i, TM_RAY_MISS, s.steps, n64); return; }
    int32_t front = -1, back = -1;
    if (r.hit_tets) {
        const int4 ft = reinterpret_cast<const int4*>(m.cft)[cf];
        const int32_t other = ft.x == s.w.cur ? ft.y : ft.x;
        front = m.t_new2old[s.w.cur];
        back = other >= 0 ? m.t_new2old[other] : -1;
    }
    write_result(r, i, int32_t(cf), float(th), float(bu), float(bv), front, back, s.steps, n64);
}

// One lane per ray: set-up, walk, result.
// 8 waves per SIMD (at most 64 VGPRs): the walk is latency-bound, so occupancy
// is what hides the memory round trips.  The precision variant carries float64
// code; it runs 7 waves (without tmax) or 6 (with): at these register budgets
// its step loop's common path keeps every value in registers, and the spilled
// values are those of the rare float64 path and of set-up.  Its float64 path
// reads the ray from the lane's copy in LDS, so no address stays live for it.
// At 8 waves without tmax (64 VGPRs) the compiler parks scalar registers in
// vector-register lanes across the float64 branch, and whole waves came back
// wrong; 7 waves keep the loop free of such spills.
// The dispatcher deals blocks to the XCDs round-robin (block b runs on XCD
// b mod X), and each XCD has an L2 of its own.  Renumbering blocks so that
// consecutive ones share an XCD keeps neighbouring rays -- which visit the same
// tets, and read and write the same lines of the ray arrays -- on one L2.
// G = 0: one contiguous range per XCD (the whole launch split X ways; walks of
// uneven length then leave XCDs idle at the end).  G > 0: within each span of
// X*G dispatched blocks, XCD x takes G consecutive blocks; a span is dispatched
// at about the same time, so the balance of round-robin placement is kept.
// Both are bijections on [0, nb); the blocks past the last whole span keep
// their numbers.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb, uint32_t X, uint32_t G) {
    if (X <= 1) return b;
    if (G == 0) {
        const uint32_t q = nb / X, rem = nb % X;
        const uint32_t x = b % X, k = b / X;
        return x < rem ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
    }
    const uint32_t span = X * G;
    if (b >= nb / span * span) return b;
    const uint32_t r = b % span;
    return (b - r) + (r % X) * G + r / X;
}

// ---- precision variant ------------------------------------------------------
//
// A walk step whose float32 exit determinants are unsure (within eps) is decided
// in float64; the start tet and the start face's orientation are decided in
// float64 too.  A ray that meets an exact float64 tie -- it lies in a face plane,
// e.g. a ray along the mesh boundary, where Algorithm 1's zero determinants leave
// the walk undefined -- takes the closest hit by its definition instead: FP64
// Moller-Trumbore over every constrained triangle (inclusive edges, t in
// (0, tmax], the start face excluded, hits within 1e-12 of the nearest going to
// the lowest id): listed and computed by the whole grid (k_tie_scan) when a
// workspace holds the list, else by the ray's wave together.  So does a ray whose
// origin lies on the mesh boundary (within 1e-6 of the bounds) where location
// finds no start tet.

// The closest constrained triangle along one ray, by the definition; called by
// every lane of a wave with the same ray (lanes take every 64th triangle).
struct DefHit {
    int32_t tri;
    double t, u, v;
};

__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) x = fmin(x, __shfl_xor(x, k, 64));
    return x;
}

__device__ __forceinline__ int32_t wave_min_i(int32_t x) {
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) x = min(x, __shfl_xor(x, k, 64));
    return x;
}

// Moller-Trumbore in float64 from the float32 points; false when the line misses
// the closed triangle or the plane is parallel.  No fused multiply-adds, so every
// caller rounds alike.
__device__ __forceinline__ bool mt64_tri(float4 A, float4 B, float4 C, double ox, double oy, double oz, double dx,
                                         double dy, double dz, double& t, double& u, double& v) {
#pragma clang fp contract(off)
    const double e1x = double(B.x) - A.x, e1y = double(B.y) - A.y, e1z = double(B.z) - A.z;
    const double e2x = double(C.x) - A.x, e2y = double(C.y) - A.y, e2z = double(C.z) - A.z;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const double det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0) return false;
    const double sx = ox - A.x, sy = oy - A.y, sz = oz - A.z;
    u = (sx * px + sy * py + sz * pz) / det;
    const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    v = (dx * qx + dy * qy + dz * qz) / det;
    t = (e2x * qx + e2y * qy + e2z * qz) / det;
    return u >= 0.0 && v >= 0.0 && u + v <= 1.0;
}

__device__ __forceinline__ bool mt64(const Mem& M, const int4 fv, double ox, double oy, double oz, double dx,
                                     double dy, double dz, double& t, double& u, double& v) {
    return mt64_tri(load_pt(M, uint32_t(fv.x)), load_pt(M, uint32_t(fv.y)), load_pt(M, uint32_t(fv.z)), ox, oy, oz,
                    dx, dy, dz, t, u, v);
}

__device__ DefHit wave_closest_hit(const DevMesh& m, const Mem& M, double ox, double oy, double oz, double dx,
                                   double dy, double dz, double tmax, int32_t exclude) {
    const int32_t ln = int32_t(threadIdx.x & 63);
    const int4* cfv = reinterpret_cast<const int4*>(m.cfv);
    double best = INFINITY;
    for (int32_t f = ln; f < m.ntri; f += 64) {
        double t, u, v;
        if (f != exclude && mt64(M, cfv[f], ox, oy, oz, dx, dy, dz, t, u, v) && t > 0.0 && t <= tmax)
            best = fmin(best, t);
    }
    const double tmin = wave_min(best);
    DefHit h{TM_RAY_MISS, NAN, NAN, NAN};
    if (!(tmin < INFINITY)) return h;
    // the lowest id among the hits within 1e-12 of the nearest
    int32_t id = 0x7FFFFFFF;
    for (int32_t f = ln; f < m.ntri; f += 64) {
        double t, u, v;
        if (f != exclude && mt64(M, cfv[f], ox, oy, oz, dx, dy, dz, t, u, v) && t > 0.0 && t <= tmax &&
            t <= tmin + 1e-12)
            id = min(id, f);
    }
    h.tri = wave_min_i(id);
    (void)mt64(M, cfv[h.tri], ox, oy, oz, dx, dy, dz, h.t, h.u, h.v);
    return h;
}

// Whether p lies within 1e-6 of the extent on or outside the mesh's bounds.
__device__ __forceinline__ bool on_bounds(const DevMesh& m, float px, float py, float pz) {
    const float p[3] = {px, py, pz};
    float ext = 0.0f;
    for (int a = 0; a < 3; ++a) ext = fmaxf(ext, float(m.G) / m.inv_cell[a]);
    bool on = false;
    for (int a = 0; a < 3; ++a) {
        const float hi = m.lo[a] + float(m.G) / m.inv_cell[a];
        on |= (p[a] <= m.lo[a] + 1e-6f * ext) | (p[a] >= hi - 1e-6f * ext);
    }
    return on;
}

// The result of ray k from the closest hit by definition h: a miss, or the hit
// with its front and back tets (the front one on the side the ray comes from).
template <bool TMAX>
__device__ void write_def_hit(const DevMesh& m, const Mem& M, const RayArgs& r, int64_t k, const DefHit& h,
                              int32_t steps, int32_t n64) {
    if (h.tri < 0) {
        write_code(r, k, TM_RAY_MISS, steps, n64);
        return;
    }
    int32_t front = -1, back = -1;
    if (r.hit_tets) {
        const double dx = r.dir[3 * k], dy = r.dir[3 * k + 1], dz = r.dir[3 * k + 2];
        const int4 fv = reinterpret_cast<const int4*>(m.cfv)[h.tri];
        const int4 ft = reinterpret_cast<const int4*>(m.cft)[h.tri];
        const float4 A = load_pt(M, uint32_t(fv.x)), B = load_pt(M, uint32_t(fv.y)), C = load_pt(M, uint32_t(fv.z));
        const double e1x = double(B.x) - A.x, e1y = double(B.y) - A.y, e1z = double(B.z) - A.z;
        const double e2x = double(C.x) - A.x, e2y = double(C.y) - A.y, e2z = double(C.z) - A.z;
        const double nd = (e1y * e2z - e1z * e2y) * dx + (e1z * e2x - e1x * e2z) * dy + (e1x * e2y - e1y * e2x) * dz;
        const int32_t f = nd > 0.0 ? ft.y : ft.x, b = nd > 0.0 ? ft.x : ft.y;
        front = f >= 0 ? m.t_new2old[f] : -1;
        back = b >= 0 ? m.t_new2old[b] : -1;
    }
    write_result(r, k, h.tri, float(h.t), float(h.u), float(h.v), front, back, steps, n64);
}

// The ties of a wave's lanes (ballot), one after the other, each by the whole
// wave; lane `tie` writes its ray's result.  Every lane of the wave must call it.
template <bool TMAX>
__device__ void resolve_ties(const DevMesh& m, const Mem& M, const RayArgs& r, bool tie, int64_t i, int32_t steps,
                             int32_t n64) {
    uint64_t T = lanes(tie);
    while (T) {
        const int l = __builtin_ctzll(T);
        T &= T - 1;
        const int64_t k = __builtin_amdgcn_readlane(int32_t(i), l);
        const double ox = r.orig[3 * k], oy = r.orig[3 * k + 1], oz = r.orig[3 * k + 2];
        const double dx = r.dir[3 * k], dy = r.dir[3 * k + 1], dz = r.dir[3 * k + 2];
        const double tmax = (TMAX && r.tmax) ? double(r.tmax[k]) : INFINITY;
        const int32_t sf = r.start_face ? r.start_face[k] : -1;
        const DefHit h = wave_closest_hit(m, M, ox, oy, oz, dx, dy, dz, tmax, sf);
        if (int(threadIdx.x & 63) == l) write_def_hit<TMAX>(m, M, r, k, h, steps, n64);
    }
}

// The ties of a wave: listed in L when it is given (entries past its capacity,
// and every tie without a list, are resolved by the wave itself).  Every lane of
// the wave must call it.
template <bool TMAX>
__device__ void list_or_resolve_ties(const DevMesh& m, const Mem& M, const RayArgs& r, const TieList& L, bool tie,
                                     int64_t i, int32_t steps, int32_t n64) {
    bool own = tie;
    const uint64_t T = lanes(tie);
    if (L.count && T) {
        const int lead = __builtin_ctzll(T);
        uint32_t base = 0;
        if (int(threadIdx.x & 63) == lead) base = atomicAdd(L.count, uint32_t(__popcll(T)));
        base = __builtin_amdgcn_readlane(base, lead);
        const uint32_t slot = base + __builtin_amdgcn_mbcnt_hi(uint32_t(T >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(T), 0u));
        if (tie && slot < L.cap) {
            L.ray[slot] = int32_t(i);
            L.steps[slot] = steps;
            L.n64[slot] = n64;
            L.tmin[slot] = 0x7FF0000000000000ull;   // +inf
            L.best[slot] = 0x7FFFFFFF;
            own = false;
        }
    }
    resolve_ties<TMAX>(m, M, r, own, i, steps, n64);
}

// Grid-wide closest hit by definition of the listed ties.  Work item (b, c) tests
// the constrained triangles of slice b (one per thread) against the ties of chunk
// c (staged in LDS).  A tie whose segment (0, t limit] misses the slice's
// bounding box, padded by 1e-6 of its coordinates' size, skips the slice: a hit
// that mt64 reports lies within float64 rounding of its triangle, so skipping
// changes no result.  (The exception would be a ray within about 1e-15 of
// parallel to a triangle's plane, where the quotients by a near-zero
// determinant lose their digits; an exactly coplanar ray has a zero
// determinant and no hit.)  Pass 0 takes the nearest t (atomic minimum on its bits),
// pass 1 the lowest id hit within 1e-12 of it; the rules of wave_closest_hit,
// so the results are those the wave would write.
constexpr int kTieChunk = 64;

// Whether the segment o + t d, t in [0, tl], meets the box [lo, hi]; a NaN
// anywhere reads as a miss.
__device__ __forceinline__ bool segment_meets_box(const double o[3], const double d[3], double tl, const double lo[3],
                                                  const double hi[3]) {
    double t0 = 0.0, t1 = tl;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (!(o[a] >= lo[a] && o[a] <= hi[a])) return false;
            continue;
        }
        const double inv = 1.0 / d[a];
        const double ta = (lo[a] - o[a]) * inv, tb = (hi[a] - o[a]) * inv;
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
    }
    return t0 <= t1;
}

template <bool TMAX, int LAYOUT>
__global__ void __launch_bounds__(256) k_tie_scan(DevMesh m, RayArgs r, TieList L, int32_t pass) {
    __shared__ double s_o[3][kTieChunk], s_d[3][kTieChunk], s_tl[kTieChunk];
    __shared__ int32_t s_sf[kTieChunk];
    __shared__ float s_box[4][6];
    const Mem M = make_mem<LAYOUT>(m);
    const int32_t n = int32_t(min(*L.count, L.cap));
    const int32_t nb = (m.ntri + 255) / 256, nc = (n + kTieChunk - 1) / kTieChunk;
    const int4* cfv = reinterpret_cast<const int4*>(m.cfv);
    const int w = int(threadIdx.x >> 6);
    for (int32_t it = blockIdx.x; it < nb * nc; it += gridDim.x) {
        const int32_t b = it % nb, c = it / nb;
        const int32_t f = b * 256 + int32_t(threadIdx.x);
        const bool have = f < m.ntri;
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A, C = A;
        if (have) {
            const int4 fv = cfv[f];
            A = load_pt(M, uint32_t(fv.x));
            B = load_pt(M, uint32_t(fv.y));
            C = load_pt(M, uint32_t(fv.z));
        }
        // the slice's bounding box
        float bx[6] = {fminf(A.x, fminf(B.x, C.x)), fminf(A.y, fminf(B.y, C.y)), fminf(A.z, fminf(B.z, C.z)),
                       -fmaxf(A.x, fmaxf(B.x, C.x)), -fmaxf(A.y, fmaxf(B.y, C.y)), -fmaxf(A.z, fmaxf(B.z, C.z))};
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            float x = have ? bx[e] : INFINITY;
#pragma unroll
            for (int k = 32; k >= 1; k >>= 1) x = fminf(x, __shfl_xor(x, k, 64));
            if ((threadIdx.x & 63) == 0) s_box[w][e] = x;
        }
        // the chunk's ties: origin, direction, the limit on t (negative: nothing to find)
        if (threadIdx.x < kTieChunk) {
            const int32_t k = c * kTieChunk + int32_t(threadIdx.x);
            if (k < n) {
                const int64_t ray = L.ray[k];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    s_o[a][threadIdx.x] = r.orig[3 * ray + a];
                    s_d[a][threadIdx.x] = r.dir[3 * ray + a];
                }
                double tl = (TMAX && r.tmax) ? double(r.tmax[ray]) : INFINITY;
                if (pass == 1) {
                    const double tmin = __longlong_as_double(static_cast<long long>(L.tmin[k]));
                    tl = tmin < INFINITY ? fmin(tl, tmin + 1e-12) : -1.0;
                }
                s_tl[threadIdx.x] = tl;
                s_sf[threadIdx.x] = r.start_face ? r.start_face[ray] : -1;
            }
        }
        __syncthreads();
        double lo[3], hi[3];
        double size = 1.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(fminf(s_box[0][a], s_box[1][a]), fminf(s_box[2][a], s_box[3][a]));
            hi[a] = -fminf(fminf(s_box[0][a + 3], s_box[1][a + 3]), fminf(s_box[2][a + 3], s_box[3][a + 3]));
            size = fmax(size, fmax(fabs(lo[a]), fabs(hi[a])));
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] -= 1e-6 * size;
            hi[a] += 1e-6 * size;
        }
        // lane j tests tie j against the box; the wave then runs the exact test for
        // the ties that meet it, one after the other
        const int32_t kn = min(kTieChunk, n - c * kTieChunk);
        const int ln = int(threadIdx.x & 63);
        bool meets = false;
        if (ln < kn && s_tl[ln] > 0.0) {
            const double o[3] = {s_o[0][ln], s_o[1][ln], s_o[2][ln]};
            const double d[3] = {s_d[0][ln], s_d[1][ln], s_d[2][ln]};
            meets = segment_meets_box(o, d, s_tl[ln], lo, hi);
        }
        for (uint64_t J = lanes(meets); J; J &= J - 1) {
            const int32_t j = __builtin_ctzll(J);
            const double tl = s_tl[j];
            const double o[3] = {s_o[0][j], s_o[1][j], s_o[2][j]};
            const double d[3] = {s_d[0][j], s_d[1][j], s_d[2][j]};
            double t, u, v;
            const bool hit = have && f != s_sf[j] && mt64_tri(A, B, C, o[0], o[1], o[2], d[0], d[1], d[2], t, u, v) &&
                             t > 0.0 && t <= tl;
            if (!lanes(hit)) continue;
            const int32_t k = c * kTieChunk + j;
            if (pass == 0) {
                const double best = wave_min(hit ? t : INFINITY);
                if ((threadIdx.x & 63) == 0)
                    atomicMin(L.tmin + k, static_cast<unsigned long long>(__double_as_longlong(best)));
            } else {
                const int32_t id = wave_min_i(hit ? f : 0x7FFFFFFF);
                if ((threadIdx.x & 63) == 0) atomicMin(L.best + k, id);
            }
        }
        __syncthreads();
    }
}

// The listed ties' results, from the hits found by the scans.
template <bool TMAX, int LAYOUT>
__global__ void __launch_bounds__(256) k_tie_write(DevMesh m, RayArgs r, TieList L) {
    const Mem M = make_mem<LAYOUT>(m);
    const int64_t n = min(*L.count, L.cap);
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x) {
        const int64_t ray = L.ray[k];
        DefHit h{TM_RAY_MISS, NAN, NAN, NAN};
        if (L.best[k] != 0x7FFFFFFF) {
            h.tri = L.best[k];
            const double ox = r.orig[3 * ray], oy = r.orig[3 * ray + 1], oz = r.orig[3 * ray + 2];
            const double dx = r.dir[3 * ray], dy = r.dir[3 * ray + 1], dz = r.dir[3 * ray + 2];
            (void)mt64(M, reinterpret_cast<const int4*>(m.cfv)[h.tri], ox, oy, oz, dx, dy, dz, h.t, h.u, h.v);
        }
        write_def_hit<TMAX>(m, M, r, ray, h, L.steps[k], L.n64[k]);
    }
}

// One ray of the precision variant, up to its result or its tie.  Returns true
// when the ray is a tie (its result then comes from resolve_ties).  DEFER (the
// first pass of the two-pass form): the walk stops at its first unsure step
// instead of deciding it in float64, and *deferred is set; the result is then
// left to the second pass.
template <bool TMAX, int LAYOUT, bool DEFER>
__device__ __forceinline__ bool trace_prec(const DevMesh& m, const Mem& M, const RayArgs& r, int64_t i, float eps,
                                           int32_t& steps_out, int32_t& n64_out, bool* deferred) {
    Ray s;
    bool degen = false, lost = false;
    steps_out = 0;
    n64_out = 0;
    if (!setup_ray<TMAX, LAYOUT, true>(m, M, r, i, s, eps, &degen, &lost)) {
        // no start tet: an origin on the boundary takes the definition (the result of
        // setup_ray, TM_RAY_INVALID, stands otherwise)
        if (!lost || !on_bounds(m, r.orig[3 * i], r.orig[3 * i + 1], r.orig[3 * i + 2])) return false;
        if (DEFER) { *deferred = true; return false; }
        return true;
    }
    if (degen) {
        if (DEFER) { *deferred = true; return false; }
        return true;
    }
    // float64 decisions along the ray as given, from the lane's copy of it in LDS
    // (read back when a step is unsure: one LDS round trip, no address to keep)
    __shared__ float ray_stash[6][kRayStash];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ray_stash[c][threadIdx.x] = r.orig[3 * i + c];
        ray_stash[3 + c][threadIdx.x] = r.dir[3 * i + c];
    }
    Prec pc{eps, 0.0f, 0.0f, 0.0f, 0};
    pc.ray6 = &ray_stash[0][threadIdx.x];
    pc.allow_degen = false;
    // the pipelined form of walk_ray (next record loaded inside the step)
    if (LAYOUT == kTet16) s.w.cur ^= int32_t(s.w.next);
    Rec R = load_rec<LAYOUT>(M, s.w.next);
    bool unsure = false;
    if (DEFER) {
        while (walk_on<TMAX>(s, r.max_steps)) {
            walk_step_rec<TMAX, LAYOUT, false, true, true>(M, s.f, s.g, s.w, pc, R, &R, &unsure);
            if (unsure) break;
            ++s.steps;
        }
    } else if (walk_on<TMAX>(s, r.max_steps)) {
        do {
            walk_step_rec<TMAX, LAYOUT, true, true, true, true>(M, s.f, s.g, s.w, pc, R, &R);
            ++s.steps;
        } while (!pc.degen && walk_on<TMAX>(s, r.max_steps));
    }
    if (LAYOUT == kTet16) s.w.cur ^= int32_t(s.w.next);
    steps_out = s.steps;
    n64_out = pc.n64;
    if (DEFER && unsure) { *deferred = true; return false; }
    if (pc.degen) return true;
    finish_ray<TMAX>(m, M, r, i, s, pc.n64);
    return false;
}

template <bool TMAX, int LAYOUT, bool PREC, bool STEPS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC ? (TMAX ? 6 : 7) : 8)))
k_trace(DevMesh m, RayArgs r, uint32_t xcds, Knobs kn) {
    const int64_t j = int64_t(xcd_block(blockIdx.x, gridDim.x, xcds, kn.xcd_blocks)) * blockDim.x + threadIdx.x;
    const Mem M = make_mem<LAYOUT>(m);
    if (!PREC) {
        if (j >= r.n) return;
        const int64_t i = r.perm ? int64_t(r.perm[j]) : j;
        if (uint64_t(i) >= uint64_t(r.n)) return;   // a caller's order that is no permutation
        Ray s;
        if (!setup_ray<TMAX, LAYOUT, false>(m, M, r, i, s, 0.0f)) return;
        walk_ray<TMAX, LAYOUT, STEPS>(M, s, r.max_steps);
        finish_ray<TMAX>(m, M, r, i, s);
        return;
    }
    // precision variant: every lane stays to the end (ties are listed for the grid,
    // or, past the list or without one, resolved by the wave)
    const int64_t i = j < r.n ? (r.perm ? int64_t(r.perm[j]) : j) : -1;
    const bool valid = j < r.n && uint64_t(i) < uint64_t(r.n);
    int32_t steps = 0, n64 = 0;
    const bool tie = valid && trace_prec<TMAX, LAYOUT, false>(m, M, r, i, kn.eps, steps, n64, nullptr);
    list_or_resolve_ties<TMAX>(m, M, r, kn.ties, tie, i, steps, n64);
}

// Two-pass precision variant, first pass: the float32 walk with the unsure test
// at the plain kernel's occupancy; a ray whose walk meets an unsure step (or
// whose start is a float64 tie) is appended to a list -- one atomic per wave, the
// lanes' slots from their rank in the ballot -- and left unwritten.
template <bool TMAX, int LAYOUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_trace_defer(DevMesh m, RayArgs r, uint32_t xcds, Knobs kn, uint32_t* count, int32_t* list) {
    const int64_t j = int64_t(xcd_block(blockIdx.x, gridDim.x, xcds, kn.xcd_blocks)) * blockDim.x + threadIdx.x;
    const Mem M = make_mem<LAYOUT>(m);
    const int64_t i = j < r.n ? (r.perm ? int64_t(r.perm[j]) : j) : -1;
    const bool valid = j < r.n && uint64_t(i) < uint64_t(r.n);
    bool deferred = false;
    int32_t steps = 0, n64 = 0;
    if (valid) (void)trace_prec<TMAX, LAYOUT, true>(m, M, r, i, kn.eps, steps, n64, &deferred);
    const uint64_t D = lanes(deferred);
    if (D) {
        uint32_t base = 0;
        if ((threadIdx.x & 63) == uint32_t(__builtin_ctzll(D))) base = atomicAdd(count, uint32_t(__popcll(D)));
        base = __builtin_amdgcn_readlane(base, __builtin_ctzll(D));
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(uint32_t(D >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(D), 0u));
        if (deferred) list[base + rank] = int32_t(i);
    }
}

// Second pass: the precision variant on the listed rays (count read on the
// device), in a grid-stride loop whose trip count is the same for every lane of
// a wave (ties are resolved by whole waves).
template <bool TMAX, int LAYOUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TMAX ? 4 : 7)))
k_trace_listed(DevMesh m, RayArgs r, Knobs kn, const uint32_t* count, const int32_t* list) {
    const Mem M = make_mem<LAYOUT>(m);
    const int64_t n = *count;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t base = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
        const int64_t j = base + (threadIdx.x & 63);
        const int64_t i = j < n ? int64_t(list[j]) : -1;
        const bool valid = j < n && uint64_t(i) < uint64_t(r.n);
        int32_t steps = 0, n64 = 0;
        const bool tie = valid && trace_prec<TMAX, LAYOUT, false>(m, M, r, i, kn.eps, steps, n64, nullptr);
        resolve_ties<TMAX>(m, M, r, tie, i, steps, n64);
    }
}

// Persistent lanes: lane g of the grid owns the rays at positions g, g + L,
// g + 2L, ... of the ray order (L = lanes in the grid), so neighbouring lanes
// start on neighbouring rays.  A
// wave walks until `refill` of its lanes have finished, then writes those
// results and sets up their next rays together, so the dependent loads of
// set-up and result are paid once per batch rather than on every step.
template <bool TMAX, int LAYOUT>
__global__ void __launch_bounds__(256) k_trace_persistent(DevMesh m, RayArgs r, int32_t refill) {
    const int64_t L = int64_t(gridDim.x) * blockDim.x;
    int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;   // position in the ray order
    int64_t i = 0;                                                 // the ray at that position
    const Mem M = make_mem<LAYOUT>(m);
    Ray s;
    bool has = false;   // the lane holds ray i
    bool done = false;  // ... and its walk has stopped
    for (;;) {
        if (done) {
            finish_ray<TMAX>(m, M, r, i, s);
            done = false;
            has = false;
            j += L;
        }
        if (!has) {
            while (j < r.n) {
                i = r.perm ? int64_t(r.perm[j]) : j;
                if (uint64_t(i) < uint64_t(r.n) && setup_ray<TMAX, LAYOUT, false>(m, M, r, i, s, 0.0f)) {
                    has = true;
                    break;
                }
                j += L;
            }
        }
        if (!__any(has)) break;
        for (;;) {
            const bool go = has && !done && walk_on<TMAX>(s, r.max_steps);
            done = has && !go;
            if (__popcll(__ballot(done)) >= uint32_t(refill) || !__any(go)) break;
            if (go) {
                Prec pc{0.0f, 0.0f, 0.0f, 0.0f, 0};
                walk_step<TMAX, LAYOUT, false>(M, s.f, s.g, s.w, pc);
                ++s.steps;
            }
        }
    }
}

// Batched launch: block b belongs to the job whose block range holds it (a
// binary search that every lane of the block takes alike, so the job's
// descriptors are read with scalar loads); the rest is the walk of k_trace.
// PREC: the precision variant with eps (every lane stays to the end, for the
// ties its wave resolves together).
template <int LAYOUT, bool STEPS, bool PREC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC ? 6 : 8)))
k_trace_batch(const Job* __restrict__ jobs, int32_t n_jobs, uint32_t xcds, float eps) {
    const int64_t b = xcd_block(blockIdx.x, gridDim.x, xcds, 0u);
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].block0 <= b) lo = mid; else hi = mid;
    }
    const DevMesh m = jobs[lo].m;
    const RayArgs r = jobs[lo].r;
    const int64_t j = (b - jobs[lo].block0) * blockDim.x + threadIdx.x;
    const Mem M = make_mem<LAYOUT>(m);
    if (PREC) {
        const int64_t i = j < r.n ? (r.perm ? int64_t(r.perm[j]) : j) : -1;
        const bool valid = j < r.n && uint64_t(i) < uint64_t(r.n);
        int32_t steps = 0, n64 = 0;
        const bool tie = valid && trace_prec<true, LAYOUT, false>(m, M, r, i, eps, steps, n64, nullptr);
        resolve_ties<true>(m, M, r, tie, i, steps, n64);
        return;
    }
    if (j >= r.n) return;
    const int64_t i = r.perm ? int64_t(r.perm[j]) : j;
    if (uint64_t(i) >= uint64_t(r.n)) return;
    Ray s;
    if (!setup_ray<true, LAYOUT, false>(m, M, r, i, s, 0.0f)) return;
    walk_ray<true, LAYOUT, STEPS>(M, s, r.max_steps);
    finish_ray<true>(m, M, r, i, s, 0);
}

// Persistent waves draining a work queue (one launch over one or many jobs).
// The ray order of every job is cut into chunks of q.chunk rays (rays per wave
// fetch), numbered over all jobs in table order and split into q.xcds
// contiguous ranges, one per accelerator die: block b runs on die b mod X (the
// dispatcher deals blocks to the dies round-robin), so the waves of a die take
// their chunks from its own range first -- neighbouring chunks then share that
// die's L2 -- through an atomic counter per range, and take chunks from the
// other dies' ranges once theirs is exhausted, so no die idles while work is
// left.
// A wave stages the ray ids of its chunk in LDS, 64 at a time (its ray queue).
// Lanes walk one ray each; once q.refill of them have finished (a ballot), those
// write their results and take the next rays from the queue: each needy lane's
// rank among the needy lanes (mbcnt of the ballot) indexes the queue, so the
// wave's rays stay packed in its lanes with no lane-to-lane exchange.
// Registers: across a refill the lanes' ray frames, 2-D face points and tmax go
// to LDS (one 64-lane row per word, so the stores and loads are conflict-free),
// so that set-up does not stack its registers on top of the walk state; the
// kernel then fits 64 VGPRs and 8 waves per SIMD like the one-lane-per-ray
// kernel.
// A wave moves to a chunk of another job (another mesh) only when all its
// lanes are idle: the buffer descriptors of a step are wave-wide.  Every wave
// ends when all ranges are exhausted and its lanes are idle.
constexpr int kQWaves = 4;     // waves per 256-thread block

template <bool TMAX>
constexpr int stash_words() { return TMAX ? 19 : 14; }

__device__ __forceinline__ int job_of_chunk(const Job* __restrict__ jobs, int n_jobs, uint32_t c) {
    int lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (uint64_t(jobs[mid].qchunk0) <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// The stashed part of a ray's state: word k of lane l at S[64 k + l].
template <bool TMAX>
__device__ __forceinline__ void stash_put(float* S, uint32_t l, const Ray& s) {
    float* p = S + l;
    p[0] = s.f.ux; p[64] = s.f.uy; p[128] = s.f.uz; p[192] = s.f.vx; p[256] = s.f.vy; p[320] = s.f.vz;
    p[384] = s.f.pox; p[448] = s.f.poy;
    p[512] = s.w.q0x; p[576] = s.w.q0y; p[640] = s.w.q1x; p[704] = s.w.q1y; p[768] = s.w.q2x; p[832] = s.w.q2y;
    if (TMAX) {
        p[896] = s.g.gx; p[960] = s.g.gy; p[1024] = s.g.gz; p[1088] = s.g.go; p[1152] = s.tmax;
    }
}

template <bool TMAX>
__device__ __forceinline__ void stash_get(const float* S, uint32_t l, Ray& s) {
    const float* p = S + l;
    s.f.ux = p[0]; s.f.uy = p[64]; s.f.uz = p[128]; s.f.vx = p[192]; s.f.vy = p[256]; s.f.vz = p[320];
    s.f.pox = p[384]; s.f.poy = p[448];
    s.w.q0x = p[512]; s.w.q0y = p[576]; s.w.q1x = p[640]; s.w.q1y = p[704]; s.w.q2x = p[768]; s.w.q2y = p[832];
    if (TMAX) {
        s.g.gx = p[896]; s.g.gy = p[960]; s.g.gz = p[1024]; s.g.go = p[1088]; s.tmax = p[1152];
    } else {
        s.tmax = INFINITY;
    }
}

// Keeps the compiler from holding values loaded before this point in registers
// past it: the job's descriptors are then loaded where set-up and results use
// them, and only the step's buffer descriptors stay in scalar registers through
// the walk.
__device__ __forceinline__ void reload_point() { asm volatile("" ::: "memory"); }

template <bool TMAX, int LAYOUT, bool STEPS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_trace_queue(const Job* __restrict__ jobs, int32_t n_jobs, Queue q) {
    __shared__ float stash[kQWaves][stash_words<TMAX>() * 64];
    __shared__ int32_t qbuf[kQWaves][64];
    float* S = stash[threadIdx.x >> 6];
    int32_t* Q = qbuf[threadIdx.x >> 6];
    const uint32_t ln = threadIdx.x & 63u;
    const uint32_t X = q.xcds;
    const uint32_t home = blockIdx.x % X;
    // wave-uniform state
    uint32_t visit = 0;            // ranges visited so far (home first)
    int job = -1;                  // the job of the rays in the lanes and the queue
    int64_t cbase = 0;             // the current chunk: rays cbase + (cn .. ce-1) of the job
    uint32_t cn = 0, ce = 0;
    uint32_t qn = 0, qe = 0;       // staged queue: positions qn .. qe-1 of Q
    uint32_t held = 0xFFFFFFFFu;   // a chunk of another job, taken while lanes were busy
    bool exhausted = false;
    // lane state
    Ray s;
    Rec R;
    int64_t i = 0;
    bool has = false, done = false;
    for (;;) {
        reload_point();
        if (done) {
            const Job& J = jobs[__builtin_amdgcn_readfirstlane(job)];
            const Mem M = make_mem<LAYOUT>(J.m);
            if (LAYOUT == kTet16) s.w.cur ^= int32_t(s.w.next);
            if (!STEPS) s.steps = 0;
            finish_ray<TMAX>(J.m, M, J.r, i, s);
            has = false;
            done = false;
        }
        stash_put<TMAX>(S, ln, s);
        // refill the idle lanes
        for (;;) {
            const uint64_t need = lanes(!has);
            if (need == 0 || exhausted) break;
            reload_point();
            if (qn == qe) {
                if (cn == ce) {
                    uint32_t c = held;
                    if (c == 0xFFFFFFFFu) {
                        // the next chunk: from the home range, else the next range that has one
                        c = q.n_chunks;
                        while (visit < X) {
                            const uint32_t x = (home + visit) % X;
                            const uint32_t lo = uint32_t(uint64_t(q.n_chunks) * x / X);
                            const uint32_t hi = uint32_t(uint64_t(q.n_chunks) * (x + 1) / X);
                            uint32_t k = 0;
                            if (ln == 0) k = atomicAdd(q.cursor + 32 * x, 1u);
                            k = __builtin_amdgcn_readfirstlane(k);
                            if (lo + k < hi) { c = lo + k; break; }
                            ++visit;
                        }
                        if (c >= q.n_chunks) { exhausted = true; break; }
                    }
                    const int jb = job_of_chunk(jobs, n_jobs, c);
                    if (jb != job) {
                        // another mesh: only once every lane of the wave is idle
                        if (~need != 0) { held = c; break; }
                        job = __builtin_amdgcn_readfirstlane(jb);
                    }
                    held = 0xFFFFFFFFu;
                    cbase = (int64_t(c) - jobs[job].qchunk0) * q.chunk;
                    cn = 0;
                    ce = uint32_t(min<int64_t>(q.chunk, jobs[job].r.n - cbase));
                }
                // stage the next 64 rays of the chunk
                const uint32_t cnt = min(64u, ce - cn);
                if (ln < cnt) {
                    const int64_t j = cbase + cn + ln;
                    const int32_t* perm = jobs[job].r.perm;
                    Q[ln] = perm ? perm[j] : int32_t(j);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                cn += cnt;
                qn = 0;
                qe = cnt;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // the needy lanes take the next positions, in lane order
            const uint32_t take = min(uint32_t(__popcll(need)), qe - qn);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(uint32_t(need >> 32),
                                                            __builtin_amdgcn_mbcnt_lo(uint32_t(need), 0u));
            if (!has && rank < take) {
                const Job& J = jobs[__builtin_amdgcn_readfirstlane(job)];
                const Mem M = make_mem<LAYOUT>(J.m);
                i = Q[qn + rank];
                Ray t;
                if (uint64_t(i) < uint64_t(J.r.n) && setup_ray<TMAX, LAYOUT, false>(J.m, M, J.r, i, t, 0.0f)) {
                    has = true;
                    if (LAYOUT == kTet16) t.w.cur ^= int32_t(t.w.next);   // the LINK form of the step
                    stash_put<TMAX>(S, ln, t);
                    s.w = t.w;
                    s.steps = t.steps;
                    R = load_rec<LAYOUT>(M, s.w.next);
                }
            }
            qn += take;
        }
        if (lanes(has) == 0) {
            if (exhausted || held == 0xFFFFFFFFu) break;
            continue;   // switch to the held chunk's job
        }
        stash_get<TMAX>(S, ln, s);
        const Job& JW = jobs[__builtin_amdgcn_readfirstlane(job)];
        const Mem M = make_mem<LAYOUT>(JW.m);
        const int32_t max_steps = JW.r.max_steps;
        // walk until q.refill lanes have finished (or none is left walking)
        for (;;) {
            const bool go = has && !done && walk_on<TMAX>(s, max_steps);
            done = done || (has && !go);
            const uint64_t G = lanes(go);
            if (G == 0 || __popcll(lanes(done)) >= uint32_t(q.refill)) break;
            if (go) {
                Prec pc{0.0f, 0.0f, 0.0f, 0.0f, 0};
                walk_step_rec<TMAX, LAYOUT, false, true, true>(M, s.f, s.g, s.w, pc, R, &R);
                ++s.steps;
            }
        }
    }
}

// One job entry written on the device (the single-mesh form of the queue kernel
// reads its mesh and rays from a one-entry table like a batch).
__global__ void k_put_job(Job j, Job* dst) { *dst = j; }

__global__ void k_zero(uint32_t* p, int32_t n) {
    const int k = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < n) p[k] = 0u;
}

template <int LAYOUT>
__global__ void __launch_bounds__(256) k_locate(DevMesh m, int64_t n, const float* pts, int32_t* out,
                                                int32_t max_steps) {
    // location is always decided with the float64 re-evaluation of near-zero
    // determinants: it is short, and a wrong tet there would start every ray wrong
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Mem M = make_mem<LAYOUT>(m);
    const float px = pts[3 * i], py = pts[3 * i + 1], pz = pts[3 * i + 2];
    if (!isfinite(px + py + pz)) { out[i] = -1; return; }
    int32_t v[4];
    int32_t t = locate_point<LAYOUT, true>(m, M, px, py, pz, max_steps, 1e-6f, v);
    if (t >= 0) t = contain64<LAYOUT>(m, M, t, v, px, py, pz);
    out[i] = t >= 0 ? m.t_new2old[t] : (t == TM_RAY_STEP_CAP ? -2 : -1);
}

// The persistent-wave kernel: its counters zeroed (a kernel, so the pair can be
// captured in a graph), then a grid that fills every CU at 8 waves per SIMD (or
// fewer blocks, when there are fewer chunks than waves).
template <bool TMAX, int LAYOUT>
void launch_queue_t(const Job* jobs, int32_t n_jobs, const Queue& q, bool steps, int32_t cus, hipStream_t s) {
    if (q.n_chunks == 0) return;
    const int32_t words = int32_t(32 * q.xcds);
    hipLaunchKernelGGL(k_zero, dim3(unsigned((words + 255) / 256)), dim3(256), 0, s, q.cursor, words);
    const int64_t full = int64_t(std::max(1, cus)) * (8 * 4 * 64 / 256);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(full, (int64_t(q.n_chunks) + kQWaves - 1) / kQWaves));
    if (steps)
        hipLaunchKernelGGL((k_trace_queue<TMAX, LAYOUT, true>), dim3(unsigned(grid)), dim3(256), 0, s, jobs, n_jobs, q);
    else
        hipLaunchKernelGGL((k_trace_queue<TMAX, LAYOUT, false>), dim3(unsigned(grid)), dim3(256), 0, s, jobs, n_jobs, q);
}

template <bool TMAX, int LAYOUT>
void launch_trace_t(const DevMesh& m, const RayArgs& r, const LaunchCfg& c, hipStream_t s) {
    const int block = (c.block == 64 || c.block == 128) ? c.block : 256;
    const int64_t simple_grid = (r.n + block - 1) / block;
    if (c.kernel == 3) {
        // a one-entry job table in the workspace, beside the queue's counters
        Job j{};
        j.m = m;
        j.r = r;
        Job* table = c.queue_job;
        hipLaunchKernelGGL(k_put_job, dim3(1), dim3(1), 0, s, j, table);
        launch_queue_t<TMAX, LAYOUT>(table, 1, c.queue, r.steps != nullptr, c.cus, s);
    } else if (c.kernel == 2) {
        // enough lanes to fill every CU with `waves_per_simd` waves per SIMD
        const int64_t blocks_per_cu = int64_t(c.waves_per_simd) * 4 * 64 / block;
        int64_t grid = std::min<int64_t>(simple_grid, std::max<int64_t>(1, c.cus * blocks_per_cu));
        if (c.grid_cap > 0) grid = std::min<int64_t>(grid, c.grid_cap);
        const int32_t refill = std::min(64, std::max(1, c.refill));
        hipLaunchKernelGGL((k_trace_persistent<TMAX, LAYOUT>), dim3(unsigned(grid)), dim3(block), 0, s,
                           m, r, refill);
    } else if (c.eps > 0.0f && c.defer_count) {
        // two passes: the float32 walk defers its unsure rays to a list, which the
        // float64-capable kernel then traces (a grid that fills the device at its
        // occupancy, reading the list's length on the device)
        const Knobs kn{c.eps, uint32_t(c.xcd_blocks)};
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, c.defer_count, 1);
        hipLaunchKernelGGL((k_trace_defer<TMAX, LAYOUT>), dim3(unsigned(simple_grid)), dim3(block), 0, s, m, r,
                           uint32_t(std::max(1, c.xcds)), kn, c.defer_count, c.defer_list);
        const int64_t full = int64_t(std::max(1, c.cus)) * (TMAX ? 4 : 7) * 4 * 64 / 256;
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(full, (r.n + 255) / 256));
        hipLaunchKernelGGL((k_trace_listed<TMAX, LAYOUT>), dim3(unsigned(grid)), dim3(256), 0, s, m, r, kn,
                           c.defer_count, c.defer_list);
    } else if (c.eps > 0.0f) {
        // ties go to a list (when there is room for one), whose closest hits by
        // definition the whole grid then finds: a scan pass for the nearest t, one
        // for the lowest id at it, and the results
        if (c.ties.count) hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, c.ties.count, 1);
        hipLaunchKernelGGL((k_trace<TMAX, LAYOUT, true, true>), dim3(unsigned(simple_grid)), dim3(block), 0,
                           s, m, r, uint32_t(std::max(1, c.xcds)), Knobs{c.eps, uint32_t(c.xcd_blocks), c.ties});
        if (c.ties.count) {
            const unsigned grid = unsigned(std::max(1, c.cus) * 8);
            hipLaunchKernelGGL((k_tie_scan<TMAX, LAYOUT>), dim3(grid), dim3(256), 0, s, m, r, c.ties, 0);
            hipLaunchKernelGGL((k_tie_scan<TMAX, LAYOUT>), dim3(grid), dim3(256), 0, s, m, r, c.ties, 1);
            hipLaunchKernelGGL((k_tie_write<TMAX, LAYOUT>), dim3((kTieCap + 255) / 256), dim3(256), 0, s, m, r,
                               c.ties);
        }
    } else if (r.steps) {
        hipLaunchKernelGGL((k_trace<TMAX, LAYOUT, false, true>), dim3(unsigned(simple_grid)), dim3(block), 0,
                           s, m, r, uint32_t(std::max(1, c.xcds)), Knobs{0.0f, uint32_t(c.xcd_blocks)});
    } else {
        hipLaunchKernelGGL((k_trace<TMAX, LAYOUT, false, false>), dim3(unsigned(simple_grid)), dim3(block), 0,
                           s, m, r, uint32_t(std::max(1, c.xcds)), Knobs{0.0f, uint32_t(c.xcd_blocks)});
    }
}

}  // namespace

hipError_t launch_trace(const DevMesh& m, const RayArgs& r, const LaunchCfg& c, hipStream_t s) {
    if (r.n <= 0) return hipSuccess;
    if (m.layout == kTet16) {
        if (r.tmax) launch_trace_t<true, kTet16>(m, r, c, s);
        else launch_trace_t<false, kTet16>(m, r, c, s);
    } else if (m.layout == kTet32N) {
        if (r.tmax) launch_trace_t<true, kTet32N>(m, r, c, s);
        else launch_trace_t<false, kTet32N>(m, r, c, s);
    } else if (m.layout == kTet32) {
        if (r.tmax) launch_trace_t<true, kTet32>(m, r, c, s);
        else launch_trace_t<false, kTet32>(m, r, c, s);
    } else {
        if (r.tmax) launch_trace_t<true, kTet20>(m, r, c, s);
        else launch_trace_t<false, kTet20>(m, r, c, s);
    }
    return hipGetLastError();
}

template <int LAYOUT>
void launch_trace_batch_t(const Job* d_jobs, int32_t n_jobs, dim3 g, dim3 b, uint32_t X, bool steps, float eps,
                          hipStream_t s) {
    if (eps > 0.0f)
        hipLaunchKernelGGL((k_trace_batch<LAYOUT, true, true>), g, b, 0, s, d_jobs, n_jobs, X, eps);
    else if (steps)
        hipLaunchKernelGGL((k_trace_batch<LAYOUT, true, false>), g, b, 0, s, d_jobs, n_jobs, X, 0.0f);
    else
        hipLaunchKernelGGL((k_trace_batch<LAYOUT, false, false>), g, b, 0, s, d_jobs, n_jobs, X, 0.0f);
}

hipError_t launch_trace_batch(const Job* d_jobs, int32_t n_jobs, int64_t total_blocks, int32_t block,
                              int32_t layout, int32_t xcds, bool steps, float eps, hipStream_t s) {
    const uint32_t X = uint32_t(std::max(1, xcds));
    if (total_blocks <= 0 || n_jobs <= 0) return hipSuccess;
    const dim3 g{unsigned(total_blocks)}, b{unsigned(block)};
    if (layout == kTet16) launch_trace_batch_t<kTet16>(d_jobs, n_jobs, g, b, X, steps, eps, s);
    else if (layout == kTet32N) launch_trace_batch_t<kTet32N>(d_jobs, n_jobs, g, b, X, steps, eps, s);
    else if (layout == kTet32) launch_trace_batch_t<kTet32>(d_jobs, n_jobs, g, b, X, steps, eps, s);
    else launch_trace_batch_t<kTet20>(d_jobs, n_jobs, g, b, X, steps, eps, s);
    return hipGetLastError();
}

int64_t queue_workspace_bytes() { return kQueueCursorBytes + (int64_t(sizeof(Job)) + 255) / 256 * 256; }

// [count: 256 B][ray, steps, n64, best: 4 B each][tmin: 8 B], each part 256-byte aligned
int64_t tie_workspace_bytes() { return 256 + 4 * (int64_t(kTieCap) * 4) + int64_t(kTieCap) * 8; }

TieList tie_list_at(void* p) {
    char* b = static_cast<char*>(p);
    const int64_t q = int64_t(kTieCap) * 4;
    TieList L;
    L.count = reinterpret_cast<uint32_t*>(b);
    L.ray = reinterpret_cast<int32_t*>(b + 256);
    L.steps = reinterpret_cast<int32_t*>(b + 256 + q);
    L.n64 = reinterpret_cast<int32_t*>(b + 256 + 2 * q);
    L.best = reinterpret_cast<int32_t*>(b + 256 + 3 * q);
    L.tmin = reinterpret_cast<unsigned long long*>(b + 256 + 4 * q);
    L.cap = kTieCap;
    return L;
}

hipError_t launch_trace_batch_queue(const Job* d_jobs, int32_t n_jobs, const Queue& q, int32_t layout,
                                    bool steps, int32_t cus, hipStream_t s) {
    if (n_jobs <= 0 || q.n_chunks == 0) return hipSuccess;
    // batches carry tmax for every job (+inf where a job has none)
    if (layout == kTet16) launch_queue_t<true, kTet16>(d_jobs, n_jobs, q, steps, cus, s);
    else if (layout == kTet32N) launch_queue_t<true, kTet32N>(d_jobs, n_jobs, q, steps, cus, s);
    else if (layout == kTet32) launch_queue_t<true, kTet32>(d_jobs, n_jobs, q, steps, cus, s);
    else launch_queue_t<true, kTet20>(d_jobs, n_jobs, q, steps, cus, s);
    return hipGetLastError();
}

hipError_t launch_locate(const DevMesh& m, int64_t n, const float* pts, int32_t* out,
                         int32_t max_steps, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    if (m.layout == kTet16)
        hipLaunchKernelGGL(k_locate<kTet16>, dim3(unsigned(grid)), dim3(block), 0, s, m, n, pts, out, max_steps);
    else if (m.layout == kTet32N)
        hipLaunchKernelGGL(k_locate<kTet32N>, dim3(unsigned(grid)), dim3(block), 0, s, m, n, pts, out, max_steps);
    else if (m.layout == kTet32)
        hipLaunchKernelGGL(k_locate<kTet32>, dim3(unsigned(grid)), dim3(block), 0, s, m, n, pts, out, max_steps);
    else
        hipLaunchKernelGGL(k_locate<kTet20>, dim3(unsigned(grid)), dim3(block), 0, s, m, n, pts, out, max_steps);
    return hipGetLastError();
}

}  // namespace tetrt
