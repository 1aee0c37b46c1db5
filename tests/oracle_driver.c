/* Driver for the oracle's C walk (oracle/walk.c), built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_host_sanitized.py.  Reads a mesh
 * and a ray set from a binary file, traces the rays (with and without tmax and
 * start faces as given) and locates their origins, and writes the outputs. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void* oracle_mesh_new(const float* pts, int64_t np, const int32_t* tets, const int32_t* nbrs,
                      const uint8_t* cflag, int64_t nt, char* err, int64_t errlen);
void oracle_mesh_free(void* h);
int oracle_locate(void* h, int64_t n, const float* xyz, int32_t source_tet, int32_t* out);
int oracle_trace(void* h, int64_t n, const float* orig, const float* dir, const float* tmax,
                 const int32_t* start_face, const int32_t* start_tet, int32_t source_tet,
                 int early_out, int64_t max_steps, int32_t* out_tri, double* out_t, double* out_bary,
                 int32_t* out_tets, int32_t* out_steps, int32_t* out_start);

static void* read_n(FILE* f, size_t size, size_t n) {
    void* p = malloc(size * (n ? n : 1));
    if (!p || (n && fread(p, size, n, f) != n)) exit(2);
    return p;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[3];
    if (fread(hdr, sizeof hdr, 1, f) != 1) return 2;
    const int64_t np = hdr[0], nt = hdr[1], n = hdr[2];
    float* P = read_n(f, sizeof(float), (size_t)(3 * np));
    int32_t* tets = read_n(f, sizeof(int32_t), (size_t)(4 * nt));
    int32_t* nbrs = read_n(f, sizeof(int32_t), (size_t)(4 * nt));
    uint8_t* cflag = read_n(f, 1, (size_t)(4 * nt));
    float* o = read_n(f, sizeof(float), (size_t)(3 * n));
    float* d = read_n(f, sizeof(float), (size_t)(3 * n));
    float* tm = read_n(f, sizeof(float), (size_t)n);
    int32_t* sf = read_n(f, sizeof(int32_t), (size_t)n);
    fclose(f);
    char err[256];
    void* h = oracle_mesh_new(P, np, tets, nbrs, cflag, nt, err, sizeof err);
    if (!h) { fprintf(stderr, "mesh: %s\n", err); return 3; }
    int32_t* tri = malloc(sizeof(int32_t) * (size_t)n);
    double* t = malloc(sizeof(double) * (size_t)n);
    double* bary = malloc(sizeof(double) * 2 * (size_t)n);
    int32_t* tt = malloc(sizeof(int32_t) * 2 * (size_t)n);
    int32_t* steps = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* start = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* loc = malloc(sizeof(int32_t) * (size_t)n);
    FILE* g = fopen(argv[2], "wb");
    if (!g) return 2;
    /* pass 1: located origins, no tmax; pass 2: tmax and start faces */
    for (int pass = 0; pass < 2; ++pass) {
        if (oracle_trace(h, n, o, d, pass ? tm : NULL, pass ? sf : NULL, NULL, 0, 1, 0, tri, t, bary, tt,
                         steps, start) != 0)
            return 4;
        fwrite(tri, sizeof(int32_t), (size_t)n, g);
        fwrite(t, sizeof(double), (size_t)n, g);
        fwrite(bary, sizeof(double), 2 * (size_t)n, g);
        fwrite(steps, sizeof(int32_t), (size_t)n, g);
    }
    if (oracle_locate(h, n, o, 0, loc) != 0) return 5;
    fwrite(loc, sizeof(int32_t), (size_t)n, g);
    fclose(g);
    oracle_mesh_free(h);
    free(P); free(tets); free(nbrs); free(cflag); free(o); free(d); free(tm); free(sf);
    free(tri); free(t); free(bary); free(tt); free(steps); free(start); free(loc);
    printf("done\n");
    return 0;
}
