// Host-only driver for the mesh packer, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py: packs a mesh read
// from a binary file in every record layout and curve order, then runs the
// validation on corrupted copies of it.  Prints one line per run.
#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>

#include "pack.h"

namespace {

template <class T>
bool read_all(FILE* f, std::vector<T>& v, size_t n) {
    v.resize(n);
    return n == 0 || fread(v.data(), sizeof(T), n, f) == n;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[2];
    if (fread(hdr, sizeof hdr, 1, f) != 1) return 2;
    const int64_t np = hdr[0], nt = hdr[1];
    std::vector<float> P;
    std::vector<int32_t> tets, nbrs;
    std::vector<uint8_t> cflag;
    if (!read_all(f, P, size_t(3 * np)) || !read_all(f, tets, size_t(4 * nt)) ||
        !read_all(f, nbrs, size_t(4 * nt)) || !read_all(f, cflag, size_t(4 * nt)))
        return 2;
    fclose(f);
    // regions by a plain flood fill (independent of the packer's union-find):
    // tets joined across faces that are neither constrained nor the boundary
    std::vector<int32_t> label(size_t(nt), -1);
    int64_t n_regions = 0;
    for (int64_t s = 0; s < nt; ++s) {
        if (label[size_t(s)] >= 0) continue;
        std::vector<int64_t> stack{s};
        label[size_t(s)] = int32_t(n_regions);
        while (!stack.empty()) {
            const int64_t t = stack.back();
            stack.pop_back();
            for (int j = 0; j < 4; ++j) {
                const int32_t nb = nbrs[size_t(4 * t + j)];
                if (nb < 0 || cflag[size_t(4 * t + j)] || label[size_t(nb)] >= 0) continue;
                label[size_t(nb)] = int32_t(n_regions);
                stack.push_back(nb);
            }
        }
        ++n_regions;
    }
    for (int layout = 0; layout < 4; ++layout) {
        for (int sfc = 0; sfc < 4; ++sfc) {
            tm_upload_opts o{layout, sfc, 1, 0, 0};
            tetrt::PackedMesh m;
            std::string err;
            const int rc = tetrt::pack_mesh(P.data(), np, tets.data(), nbrs.data(), cflag.data(), nt, o, &m, &err);
            // in region order every region's tets are one contiguous run
            int64_t runs = 0;
            for (int64_t i = 0; i < nt && rc == 0; ++i)
                if (i == 0 || label[size_t(m.t_new2old[size_t(i)])] != label[size_t(m.t_new2old[size_t(i - 1)])])
                    ++runs;
            printf("pack layout %d sfc %d rc %d ntri %lld G %d rec %zu regions %lld flood %lld runs %lld\n",
                   layout, sfc, rc, (long long)m.ntri, m.G, m.rec.size(), (long long)m.n_regions,
                   (long long)n_regions, (long long)runs);
        }
    }
    // corrupted copies: each must be rejected by validation
    struct Bad { const char* what; int64_t at; int kind; };
    const Bad bad[] = {{"vertex out of range", 0, 0}, {"negative vertex", nt / 2, 1},
                       {"repeated vertex", nt - 1, 2}, {"neighbour out of range", 3, 3},
                       {"flag on one side", 5, 4}};
    for (const Bad& b : bad) {
        std::vector<int32_t> t2 = tets, n2 = nbrs;
        std::vector<uint8_t> c2 = cflag;
        const int64_t t = b.at;
        if (b.kind == 0) t2[4 * t + 2] = int32_t(np + 3);
        if (b.kind == 1) t2[4 * t + 1] = -5;
        if (b.kind == 2) t2[4 * t + 3] = t2[4 * t];
        if (b.kind == 3) n2[4 * t] = int32_t(nt + 10);
        if (b.kind == 4) {
            int j = 0;
            while (j < 4 && n2[4 * t + j] < 0) ++j;
            if (j < 4) c2[4 * t + j] = uint8_t(!c2[4 * t + j]);
        }
        tm_upload_opts o{1, 0, 1, 0, 0};
        tetrt::PackedMesh m;
        std::string err;
        const int rc = tetrt::pack_mesh(P.data(), np, t2.data(), n2.data(), c2.data(), nt, o, &m, &err);
        printf("bad %s rc %d: %s\n", b.what, rc, err.c_str());
    }
    printf("done\n");
    return 0;
}
