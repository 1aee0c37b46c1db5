// Host-side packing: validation, canonical triangle ids, space-filling-curve
// renumbering, Tet20 records, the constrained-face table and the point-location
// seed grid.  Everything here runs once per upload.
#include "pack.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <thread>

namespace tetrt {

namespace {

unsigned worker_count() {
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 4;
    return std::min(n, 32u);
}

// Run f(begin, end) over [0, n) split across threads.
template <class F>
void parallel_for(int64_t n, F&& f) {
    unsigned k = worker_count();
    if (n < (1 << 15) || k <= 1) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + k - 1) / k;
    for (unsigned i = 0; i < k; ++i) {
        int64_t b = int64_t(i) * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back([&f, b, e] { f(b, e); });
    }
    for (auto& t : th) t.join();
}

struct KeyId {
    uint64_t key;
    uint32_t id;
    bool operator<(const KeyId& o) const { return key < o.key || (key == o.key && id < o.id); }
};

// Sort in parallel: sort 2^p chunks, then merge pairwise.
void parallel_sort(std::vector<KeyId>& v) {
    unsigned k = worker_count();
    size_t n = v.size();
    if (n < (1u << 16) || k <= 1) {
        std::sort(v.begin(), v.end());
        return;
    }
    unsigned p = 1;
    while (p * 2 <= k) p *= 2;
    std::vector<size_t> bound(p + 1);
    for (unsigned i = 0; i <= p; ++i) bound[i] = n * i / p;
    {
        std::vector<std::thread> th;
        for (unsigned i = 0; i < p; ++i)
            th.emplace_back([&, i] { std::sort(v.begin() + bound[i], v.begin() + bound[i + 1]); });
        for (auto& t : th) t.join();
    }
    for (unsigned w = 1; w < p; w *= 2) {
        std::vector<std::thread> th;
        for (unsigned i = 0; i + w < p; i += 2 * w) {
            size_t a = bound[i], m = bound[i + w], e = bound[std::min(i + 2 * w, p)];
            th.emplace_back([&v, a, m, e] {
                std::inplace_merge(v.begin() + a, v.begin() + m, v.begin() + e);
            });
        }
        for (auto& t : th) t.join();
    }
}

double orient3d(const float* P, const int32_t* t) {
    const float *a = P + 3 * (int64_t)t[0], *b = P + 3 * (int64_t)t[1], *c = P + 3 * (int64_t)t[2],
                *d = P + 3 * (int64_t)t[3];
    double bx = double(b[0]) - a[0], by = double(b[1]) - a[1], bz = double(b[2]) - a[2];
    double cx = double(c[0]) - a[0], cy = double(c[1]) - a[1], cz = double(c[2]) - a[2];
    double dx = double(d[0]) - a[0], dy = double(d[1]) - a[1], dz = double(d[2]) - a[2];
    return bx * (cy * dz - cz * dy) - by * (cx * dz - cz * dx) + bz * (cx * dy - cy * dx);
}

// Checks of one tet; returns an empty string when it is consistent.
std::string check_tet(int64_t t, int64_t np, int64_t nt, const float* P, const int32_t* tets,
                      const int32_t* nbrs, const uint8_t* cflag) {
    char buf[256];
    const int32_t* v = tets + 4 * t;
    for (int s = 0; s < 4; ++s)
        if (v[s] < 0 || v[s] >= np) {
            snprintf(buf, sizeof buf, "tet %lld: vertex id %d out of range", (long long)t, v[s]);
            return buf;
        }
    for (int s = 0; s < 4; ++s)
        for (int r = s + 1; r < 4; ++r)
            if (v[s] == v[r]) {
                snprintf(buf, sizeof buf, "tet %lld: repeated vertex %d", (long long)t, v[s]);
                return buf;
            }
    if (orient3d(P, v) == 0.0) {
        snprintf(buf, sizeof buf, "tet %lld: zero volume", (long long)t);
        return buf;
    }
    for (int j = 0; j < 4; ++j) {
        int32_t nb = nbrs[4 * t + j];
        if (nb == -1) continue;
        if (nb < -1 || nb >= nt || nb == t) {
            snprintf(buf, sizeof buf, "tet %lld: neighbour %d of slot %d out of range", (long long)t, nb, j);
            return buf;
        }
        const int32_t* w = tets + 4 * (int64_t)nb;
        int back = -1;
        for (int s = 0; s < 4; ++s)
            if (nbrs[4 * (int64_t)nb + s] == t) back = s;
        if (back < 0) {
            snprintf(buf, sizeof buf, "tet %lld: neighbour %d (slot %d) does not link back",
                     (long long)t, nb, j);
            return buf;
        }
        // the three vertices of face j must be the vertices of nb other than w[back]
        for (int s = 0; s < 4; ++s) {
            if (s == j) continue;
            bool found = false;
            for (int r = 0; r < 4; ++r)
                if (r != back && w[r] == v[s]) found = true;
            if (!found) {
                snprintf(buf, sizeof buf, "tet %lld: face %d is not shared with neighbour %d",
                         (long long)t, j, nb);
                return buf;
            }
        }
        if ((cflag[4 * t + j] != 0) != (cflag[4 * (int64_t)nb + back] != 0)) {
            snprintf(buf, sizeof buf, "tet %lld: constrained flag of face %d differs from neighbour %d",
                     (long long)t, j, nb);
            return buf;
        }
    }
    return std::string();
}

// Region label of every tet (caller numbering): tets joined across faces that
// are neither constrained nor on the boundary share a label (the smallest tet
// id of their component).  Union-find with path halving.
std::vector<int32_t> tet_regions(const int32_t* nbrs, const uint8_t* cflag, int64_t nt) {
    std::vector<int32_t> parent(static_cast<size_t>(nt));
    for (int64_t t = 0; t < nt; ++t) parent[size_t(t)] = int32_t(t);
    auto find = [&parent](int32_t x) {
        while (parent[size_t(x)] != x) {
            parent[size_t(x)] = parent[size_t(parent[size_t(x)])];
            x = parent[size_t(x)];
        }
        return x;
    };
    for (int64_t t = 0; t < nt; ++t)
        for (int j = 0; j < 4; ++j) {
            const int32_t nb = nbrs[4 * t + j];
            if (nb < 0 || nb <= t || cflag[4 * t + j]) continue;
            int32_t a = find(int32_t(t)), b = find(nb);
            if (a == b) continue;
            if (a < b) std::swap(a, b);
            parent[size_t(a)] = b;
        }
    for (int64_t t = 0; t < nt; ++t) parent[size_t(t)] = find(int32_t(t));
    return parent;
}

inline uint64_t spread3(uint32_t x, int bits) {
    uint64_t r = 0;
    for (int b = 0; b < bits; ++b) r |= uint64_t((x >> b) & 1u) << (3 * b);
    return r;
}

}  // namespace

uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z, int bits) {
    return (spread3(x, bits) << 2) | (spread3(y, bits) << 1) | spread3(z, bits);
}

// Hilbert key via Skilling's construction: the coordinates are turned in place
// into the "transposed" Hilbert index (undo the per-level reflections and axis
// exchanges from the top bit down, then Gray-decode across axes), whose bits,
// interleaved most significant first, are the position along the curve.
uint64_t hilbert_key(uint32_t x, uint32_t y, uint32_t z, int bits) {
    uint32_t X[3] = {x, y, z};
    const uint32_t top = 1u << (bits - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t low = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & q) {
                X[0] ^= low;                       // reflect the low bits of axis 0
            } else {
                uint32_t diff = (X[0] ^ X[i]) & low;   // swap the low bits of axes 0 and i
                X[0] ^= diff;
                X[i] ^= diff;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t flip = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (X[2] & q) flip ^= q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= flip;
    return morton_key(X[0], X[1], X[2], bits);
}

int pack_mesh(const float* P, int64_t np, const int32_t* tets, const int32_t* nbrs,
              const uint8_t* cflag, int64_t nt, const tm_upload_opts& opts, PackedMesh* out,
              std::string* err) {
    char buf[256];
    PackedMesh& M = *out;
    M.np = np;
    M.nt = nt;
    M.layout = opts.layout;
    M.sfc = opts.sfc;

    // ---- validation ----------------------------------------------------------
    if (opts.validate) {
        std::atomic<int64_t> first_bad(std::numeric_limits<int64_t>::max());
        parallel_for(nt, [&](int64_t b, int64_t e) {
            for (int64_t t = b; t < e && t < first_bad.load(std::memory_order_relaxed); ++t) {
                if (!check_tet(t, np, nt, P, tets, nbrs, cflag).empty()) {
                    int64_t cur = first_bad.load();
                    while (t < cur && !first_bad.compare_exchange_weak(cur, t)) {
                    }
                    break;
                }
            }
        });
        if (first_bad.load() != std::numeric_limits<int64_t>::max()) {
            *err = check_tet(first_bad.load(), np, nt, P, tets, nbrs, cflag);
            return TM_ERR_MESH;
        }
        for (int64_t i = 0; i < 3 * np; ++i)
            if (!std::isfinite(P[i])) {
                snprintf(buf, sizeof buf, "point %lld is not finite", (long long)(i / 3));
                *err = buf;
                return TM_ERR_MESH;
            }
    }

    // ---- canonical triangle ids (faces t-major, first sighting) -------------
    std::vector<int32_t> face_tri(size_t(4 * nt), -1);
    std::vector<int32_t> tri_tets;
    M.tri_verts_user.clear();
    int64_t ntri = 0;
    for (int64_t t = 0; t < nt; ++t) {
        for (int j = 0; j < 4; ++j) {
            int64_t fj = 4 * t + j;
            if (!cflag[fj] || face_tri[fj] >= 0) continue;
            if (ntri >= int64_t(0x7FFFFFFE)) {
                *err = "too many constrained triangles";
                return TM_ERR_ARG;
            }
            int32_t f[3];
            int k = 0;
            for (int s = 0; s < 4; ++s)
                if (s != j) f[k++] = tets[4 * t + s];
            std::sort(f, f + 3);
            int32_t id = int32_t(ntri++);
            face_tri[fj] = id;
            M.tri_verts_user.insert(M.tri_verts_user.end(), f, f + 3);
            int32_t nb = nbrs[fj];
            tri_tets.push_back(int32_t(t));
            tri_tets.push_back(nb);
            if (nb < 0) continue;
            int mirror = -1;
            for (int s = 0; s < 4; ++s) {
                int32_t v = tets[4 * (int64_t)nb + s];
                if (v != f[0] && v != f[1] && v != f[2]) mirror = s;
            }
            if (mirror < 0 || !cflag[4 * (int64_t)nb + mirror]) {
                snprintf(buf, sizeof buf, "tet %lld: constrained face %d is not mirrored by tet %d",
                         (long long)t, j, nb);
                *err = buf;
                return TM_ERR_MESH;
            }
            face_tri[4 * (int64_t)nb + mirror] = id;
        }
    }
    M.ntri = ntri;

    // ---- space-filling-curve order ------------------------------------------
    float lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    for (int64_t i = 0; i < np; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], P[3 * i + a]);
            hi[a] = std::max(hi[a], P[3 * i + a]);
        }
    double ext = std::max({double(hi[0]) - lo[0], double(hi[1]) - lo[1], double(hi[2]) - lo[2]});
    const int bits = 21;
    const double qmax = double((1u << bits) - 1);
    const double scale = ext > 0 ? qmax / ext : 0.0;
    auto quant = [&](double c, int a) -> uint32_t {
        double q = std::floor((c - lo[a]) * scale);
        return uint32_t(std::min(qmax, std::max(0.0, q)));
    };
    auto key = [&](double x, double y, double z) -> uint64_t {
        uint32_t qx = quant(x, 0), qy = quant(y, 1), qz = quant(z, 2);
        return opts.sfc == TM_SFC_MORTON ? morton_key(qx, qy, qz, bits) : hilbert_key(qx, qy, qz, bits);
    };

    std::vector<int32_t> p_old2new(np), p_new2old(np);
    M.t_new2old.resize(nt);
    M.t_old2new.resize(nt);
    if (opts.sfc == TM_SFC_NONE) {
        for (int64_t i = 0; i < np; ++i) p_old2new[i] = p_new2old[i] = int32_t(i);
        for (int64_t i = 0; i < nt; ++i) M.t_old2new[i] = M.t_new2old[i] = int32_t(i);
    } else {
        std::vector<KeyId> kp(np);
        parallel_for(np, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; ++i)
                kp[i] = {key(P[3 * i], P[3 * i + 1], P[3 * i + 2]), uint32_t(i)};
        });
        parallel_sort(kp);
        for (int64_t i = 0; i < np; ++i) {
            p_new2old[i] = int32_t(kp[i].id);
            p_old2new[kp[i].id] = int32_t(i);
        }
        std::vector<KeyId>().swap(kp);
        std::vector<KeyId> kt(nt);
        parallel_for(nt, [&](int64_t b, int64_t e) {
            for (int64_t t = b; t < e; ++t) {
                double c[3] = {0, 0, 0};
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) c[a] += P[3 * (int64_t)tets[4 * t + s] + a];
                kt[t] = {key(0.25 * c[0], 0.25 * c[1], 0.25 * c[2]), uint32_t(t)};
            }
        });
        parallel_sort(kt);
        if (opts.sfc == TM_SFC_HILBERT_REGIONS) {
            // Regions first (paper, Sec. "Reordering tetrahedral mesh data"): the
            // tets that constrained faces enclose together -- a walk never leaves
            // its region -- are stored contiguously, regions in the curve order of
            // their first tet, and tets inside a region in curve order.  Region
            // labels: components of the face-adjacency graph without its
            // constrained faces.
            std::vector<int32_t> region = tet_regions(nbrs, cflag, nt);
            std::vector<int32_t> rank(size_t(nt), -1);   // region label -> rank
            int32_t nreg = 0;
            for (int64_t i = 0; i < nt; ++i) {
                int32_t& r = rank[size_t(region[kt[i].id])];
                if (r < 0) r = nreg++;
            }
            std::vector<int64_t> start(size_t(nreg) + 1, 0);
            for (int64_t i = 0; i < nt; ++i) ++start[size_t(rank[size_t(region[kt[i].id])]) + 1];
            for (int32_t r = 0; r < nreg; ++r) start[size_t(r) + 1] += start[size_t(r)];
            for (int64_t i = 0; i < nt; ++i) {   // stable: curve order inside a region
                const int64_t pos = start[size_t(rank[size_t(region[kt[i].id])])]++;
                M.t_new2old[pos] = int32_t(kt[i].id);
            }
            for (int64_t i = 0; i < nt; ++i) M.t_old2new[M.t_new2old[i]] = int32_t(i);
            M.n_regions = nreg;
        } else {
            for (int64_t i = 0; i < nt; ++i) {
                M.t_new2old[i] = int32_t(kt[i].id);
                M.t_old2new[kt[i].id] = int32_t(i);
            }
        }
    }

    // ---- points ----------------------------------------------------------------
    M.pts.assign(size_t(3 * np), 0.0f);
    for (int64_t i = 0; i < np; ++i) {
        const float* s = P + 3 * (int64_t)p_new2old[i];
        M.pts[3 * i] = s[0];
        M.pts[3 * i + 1] = s[1];
        M.pts[3 * i + 2] = s[2];
    }

    // ---- tet records (Tet20, Tet16, Tet32 or Tet32N) -----------------------
    const bool t16 = opts.layout == TM_LAYOUT_TET16;
    const bool t32n = opts.layout == TM_LAYOUT_TET32N;
    const bool t32 = opts.layout == TM_LAYOUT_TET32;
    M.rec.resize(size_t((t16 ? 4 : ((t32n || t32) ? 8 : 5)) * nt));
    if (t16) M.n3.resize(size_t(nt));
    M.tetv.resize(size_t(4 * nt));
    std::vector<int32_t> vx_of(nt);   // xor field of every (new) tet
    parallel_for(nt, [&](int64_t b, int64_t e) {
        for (int64_t tn = b; tn < e; ++tn) {
            int64_t t = M.t_new2old[tn];
            vx_of[tn] = p_old2new[tets[4 * t]] ^ p_old2new[tets[4 * t + 1]] ^ p_old2new[tets[4 * t + 2]] ^
                        p_old2new[tets[4 * t + 3]];
        }
    });
    parallel_for(nt, [&](int64_t b, int64_t e) {
        for (int64_t tn = b; tn < e; ++tn) {
            int64_t t = M.t_new2old[tn];
            int32_t v[4], slot[4];
            for (int s = 0; s < 4; ++s) {
                v[s] = p_old2new[tets[4 * t + s]];
                slot[s] = s;
            }
            for (int a = 1; a < 4; ++a)  // order by internal vertex id, carrying the slot
                for (int c = a; c > 0 && v[c] < v[c - 1]; --c) {
                    std::swap(v[c], v[c - 1]);
                    std::swap(slot[c], slot[c - 1]);
                }
            uint32_t field[4];
            int32_t nvx[4];
            for (int r = 0; r < 4; ++r) {
                int64_t f = 4 * t + slot[r];
                nvx[r] = 0;
                if (cflag[f]) {
                    field[r] = kConstrainedBit | uint32_t(face_tri[f]);
                } else if (nbrs[f] < 0) {
                    field[r] = kBoundaryField;
                } else {
                    field[r] = uint32_t(M.t_old2new[nbrs[f]]);
                    nvx[r] = vx_of[field[r]];
                }
                M.tetv[4 * tn + r] = v[r];
            }
            const int32_t vx = vx_of[tn];
            if (t16) {
                M.rec[4 * tn] = vx;
                for (int r = 0; r < 3; ++r) M.rec[4 * tn + 1 + r] = int32_t(field[r] ^ field[3]);
                M.n3[tn] = int32_t(field[3]);
            } else if (t32n) {
                for (int r = 0; r < 4; ++r) {
                    M.rec[8 * tn + r] = int32_t(field[r]);
                    M.rec[8 * tn + 4 + r] = nvx[r];
                }
            } else if (t32) {
                // Fig. 2: V0, V1, V2, the xor-sum, then N0..N3 with N_j across V_j
                // (vertices in ascending id, so the fields are those of Tet20)
                for (int r = 0; r < 3; ++r) M.rec[8 * tn + r] = v[r];
                M.rec[8 * tn + 3] = vx;
                for (int r = 0; r < 4; ++r) M.rec[8 * tn + 4 + r] = int32_t(field[r]);
            } else {
                M.rec[5 * tn] = vx;
                for (int r = 0; r < 4; ++r) M.rec[5 * tn + 1 + r] = int32_t(field[r]);
            }
        }
    });

    // ---- constrained-face table --------------------------------------------
    M.cfv.assign(size_t(4 * ntri), 0);
    M.cft.assign(size_t(4 * ntri), -1);
    for (int64_t f = 0; f < ntri; ++f) {
        const int32_t* u = &M.tri_verts_user[3 * f];
        for (int k = 0; k < 3; ++k) M.cfv[4 * f + k] = p_old2new[u[k]];
        const float *A = P + 3 * (int64_t)u[0], *B = P + 3 * (int64_t)u[1], *C = P + 3 * (int64_t)u[2];
        double e1[3], e2[3], n[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = double(B[a]) - A[a];
            e2[a] = double(C[a]) - A[a];
        }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        int32_t ta = tri_tets[2 * f], tb = tri_tets[2 * f + 1];
        int32_t w = -1;
        for (int s = 0; s < 4; ++s) {
            int32_t v = tets[4 * (int64_t)ta + s];
            if (v != u[0] && v != u[1] && v != u[2]) w = v;
        }
        const float* W = P + 3 * (int64_t)w;
        double side = n[0] * (double(W[0]) - A[0]) + n[1] * (double(W[1]) - A[1]) +
                      n[2] * (double(W[2]) - A[2]);
        int32_t na = M.t_old2new[ta], nbn = tb >= 0 ? M.t_old2new[tb] : -1;
        const int32_t pos = side > 0 ? na : nbn, neg = side > 0 ? nbn : na;
        M.cft[4 * f] = pos;
        M.cft[4 * f + 1] = neg;
        M.cft[4 * f + 2] = pos >= 0 ? vx_of[pos] : 0;
        M.cft[4 * f + 3] = neg >= 0 ? vx_of[neg] : 0;
    }

    // ---- seed grid for point location --------------------------------------
    int G = opts.seed_grid > 0 ? opts.seed_grid
                               : int(std::lround(std::cbrt(double(nt) / 6.0) / 2.0));
    G = std::max(1, std::min(G, 256));
    M.G = G;
    for (int a = 0; a < 3; ++a) {
        M.lo[a] = lo[a];
        double e = double(hi[a]) - lo[a];
        M.inv_cell[a] = e > 0 ? float(G / e) : 0.0f;
    }
    const int64_t ncell = int64_t(G) * G * G;
    M.seed.assign(size_t(ncell), -1);
    std::vector<double> best(size_t(ncell), std::numeric_limits<double>::infinity());
    for (int64_t tn = 0; tn < nt; ++tn) {
        double c[3] = {0, 0, 0};
        for (int r = 0; r < 4; ++r)
            for (int a = 0; a < 3; ++a) c[a] += M.pts[3 * (int64_t)M.tetv[4 * tn + r] + a];
        int ci[3];
        double d2 = 0;
        for (int a = 0; a < 3; ++a) {
            c[a] *= 0.25;
            double g = (c[a] - lo[a]) * M.inv_cell[a];
            ci[a] = std::max(0, std::min(G - 1, int(std::floor(g))));
            double off = g - (ci[a] + 0.5);
            d2 += off * off;
        }
        int64_t cell = (int64_t(ci[0]) * G + ci[1]) * G + ci[2];
        if (d2 < best[cell]) {
            best[cell] = d2;
            M.seed[cell] = int32_t(tn);
        }
    }
    // cells that hold no centroid take a face neighbour's seed
    for (bool changed = true; changed;) {
        changed = false;
        std::vector<int32_t> next = M.seed;
        for (int x = 0; x < G; ++x)
            for (int y = 0; y < G; ++y)
                for (int z = 0; z < G; ++z) {
                    int64_t cell = (int64_t(x) * G + y) * G + z;
                    if (M.seed[cell] >= 0) continue;
                    const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
                    for (auto& o : d) {
                        int a = x + o[0], b = y + o[1], c = z + o[2];
                        if (a < 0 || b < 0 || c < 0 || a >= G || b >= G || c >= G) continue;
                        int32_t s = M.seed[(int64_t(a) * G + b) * G + c];
                        if (s >= 0) {
                            next[cell] = s;
                            changed = true;
                            break;
                        }
                    }
                }
        M.seed.swap(next);
    }
    return TM_OK;
}

}  // namespace tetrt
