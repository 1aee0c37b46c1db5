// Host-side packing of a caller mesh into the device layout (no HIP types).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "tetrt.h"

namespace tetrt {

// Neighbour-field encoding: a tet id (top bit clear), a constrained-face
// record (top bit set, low 31 bits = triangle id), or the mesh boundary.
constexpr uint32_t kConstrainedBit = 0x80000000u;
constexpr uint32_t kBoundaryField = 0xFFFFFFFFu;

struct PackedMesh {
    int64_t np = 0, nt = 0, ntri = 0;
    int32_t layout = 0, sfc = 0;
    std::vector<float> pts;              // [np*3]   x, y, z in internal point order
    std::vector<int32_t> rec;            // Tet20 [nt*5]: xor of the four internal vertex ids, then
                                         //   the neighbour fields N0..N3 by ascending vertex id;
                                         // Tet16 [nt*4]: xor, then NX_j = N_j ^ N_3 for j < 3;
                                         // Tet32N [nt*8]: N0..N3, then each neighbour's xor
                                         //   (0 where the field is not a tet);
                                         // Tet32 [nt*8]: V0, V1, V2 (ascending internal ids),
                                         //   the xor, then N0..N3 (N_j across V_j)
    std::vector<int32_t> n3;             // Tet16 only [nt]: N_3 (cold, to start walks)
    std::vector<int32_t> tetv;           // [nt*4]   internal vertex ids, ascending (cold)
    std::vector<int32_t> cfv;            // [ntri*4] internal ids of the triangle's vertices in
                                         //          ascending caller-id order, then 0
    std::vector<int32_t> cft;            // [ntri*4] internal tet on the + side of
                                         //          (v1-v0)x(v2-v0), the - side (-1 = none),
                                         //          then the xor fields of those two tets
    std::vector<int32_t> t_new2old;      // [nt]
    std::vector<int32_t> t_old2new;      // [nt]
    std::vector<int32_t> tri_verts_user; // [ntri*3] caller vertex ids, ascending
    std::vector<int32_t> seed;           // [G^3]    internal start tet per seed-grid cell
    int64_t n_regions = 0;               // TM_SFC_HILBERT_REGIONS: regions found
    int32_t G = 1;
    float lo[3] = {0, 0, 0};
    float inv_cell[3] = {0, 0, 0};
};

// Validate (if requested), renumber along the space-filling curve and build the
// packed arrays.  Returns TM_OK or TM_ERR_ARG / TM_ERR_MESH with *err set.
int pack_mesh(const float* points, int64_t np, const int32_t* tets, const int32_t* nbrs,
              const uint8_t* cflag, int64_t nt, const tm_upload_opts& opts, PackedMesh* out,
              std::string* err);

// Space-filling-curve key of integer coordinates (each < 2^bits, bits <= 21).
uint64_t hilbert_key(uint32_t x, uint32_t y, uint32_t z, int bits);
uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z, int bits);

}  // namespace tetrt
