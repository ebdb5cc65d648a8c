/*
 * Test driver for a sanitizer build of the oracle (test infrastructure only): reads a scene
 * (n x 9 float32) and rays (m x 8 float32) from two raw files, runs every oracle function on
 * them, and prints one line of results that the calling test compares with the regular build.
 * Built by tests/test_oracle_sanitize.py with gcc -fsanitize=address,undefined together with
 * hcc_oracle.c; any out-of-bounds access, leak or undefined operation ends the run with an error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_scene_box(const float* tris, uint32_t n, float* out6);
uint32_t oracle_morton3(uint32_t qx, uint32_t qy, uint32_t qz);
void oracle_morton_codes(const float* tris, uint32_t n, uint32_t* codes);
int oracle_build_bvh(const float* tris, uint32_t n, uint32_t* child, uint32_t* leaf_prim, float* boxes,
                     uint32_t* sorted_codes);
void oracle_had(uint32_t n, const uint32_t* child, const float* boxes, double lambda, double* had);
int oracle_select_cut(uint32_t n, const uint32_t* child, const double* had, uint32_t cut_size, uint32_t* cut_ids);
int oracle_select_mlhcc_cut(uint32_t n, const uint32_t* child, const double* had, uint32_t top, uint32_t low,
                            uint32_t* top_ids, uint32_t* low_ids);
void oracle_grid_boxes(const float* scene_lohi, uint32_t gx, uint32_t gy, uint32_t gz, float* boxes);
int oracle_slab(const float* ray8, const float* box6);
void oracle_encode_hcc(const float* rays, uint32_t n, const float* cut_boxes, uint32_t c_eff, uint32_t key_bits,
                       uint64_t* keys);
void oracle_encode_mlhcc(const float* rays, uint32_t n, const float* top_boxes, uint32_t t_eff,
                         const float* low_boxes, uint32_t low, uint32_t key_bits, uint64_t* keys);
void oracle_encode_ppc(const float* rays, uint32_t n, uint32_t n_tris, const uint32_t* child, const float* boxes,
                       uint32_t key_bits, uint64_t* keys);
void oracle_encode_twopoint(const float* rays, uint32_t n, const float* scene_lohi, uint32_t key_bits,
                            uint64_t* keys);
int oracle_sort(const uint64_t* keys, uint32_t n, uint32_t* perm);
void oracle_trace(uint32_t n_tris, const uint32_t* child, const uint32_t* leaf_prim, const float* boxes,
                  const float* tris, const float* rays, const uint32_t* perm, uint32_t k0, uint32_t k1, int closest,
                  float* hits, uint8_t* occluded, uint32_t* n_nodes, uint32_t* n_tests);
void oracle_brute_force(const float* tris, uint32_t n_tris, const float* rays, uint32_t n_rays, int closest,
                        float* hits, uint8_t* occluded);
double oracle_anc(const uint64_t* keys, const uint32_t* perm, uint32_t n, uint32_t width);
int oracle_wave_fetches(uint32_t n_tris, const uint32_t* child, const uint32_t* leaf_prim, const float* boxes,
                        const float* tris, const float* rays, const uint32_t* perm, uint32_t n, uint32_t width,
                        int closest, int order, const uint32_t* waves, uint32_t n_waves, uint64_t* out_nodes,
                        uint64_t* out_tris, uint32_t* out_steps);

static void* read_all(const char* path, size_t* bytes) {
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long len = ftell(f);
    fseek(f, 0, SEEK_SET);
    void* p = malloc(len > 0 ? (size_t)len : 1);
    if (p && len > 0 && fread(p, 1, (size_t)len, f) != (size_t)len) { free(p); p = NULL; }
    fclose(f);
    *bytes = (size_t)len;
    return p;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    size_t tb = 0, rb = 0;
    float* tris = (float*)read_all(argv[1], &tb);
    float* rays = (float*)read_all(argv[2], &rb);
    if (!tris || !rays) return 3;
    const uint32_t n = (uint32_t)(tb / 36), m = (uint32_t)(rb / 32);
    float box[6];
    oracle_scene_box(tris, n, box);
    uint32_t* codes = malloc(sizeof(uint32_t) * n);
    oracle_morton_codes(tris, n, codes);
    uint32_t* child = malloc(sizeof(uint32_t) * 2 * (n > 1 ? n - 1 : 1));
    uint32_t* leaf = malloc(sizeof(uint32_t) * n);
    float* boxes = malloc(sizeof(float) * 6 * (2 * (size_t)n - 1));
    uint32_t* sorted = malloc(sizeof(uint32_t) * n);
    if (oracle_build_bvh(tris, n, child, leaf, boxes, sorted) != 0) return 4;
    double* had = malloc(sizeof(double) * (2 * (size_t)n - 1));
    oracle_had(n, child, boxes, 0.125, had);
    uint32_t cut[64 + 2];
    int c = oracle_select_cut(n, child, had, 64, cut);
    if (c <= 0) return 5;
    float* cb = malloc(sizeof(float) * 6 * (size_t)c);
    for (int i = 0; i < c; ++i)
        for (int a = 0; a < 6; ++a) cb[6 * i + a] = boxes[6 * (size_t)cut[i] + a];
    uint64_t* keys = malloc(sizeof(uint64_t) * m);
    uint64_t* keys2 = malloc(sizeof(uint64_t) * m);
    uint32_t* perm = malloc(sizeof(uint32_t) * m);
    oracle_encode_hcc(rays, m, cb, (uint32_t)c, 32, keys);
    if (oracle_sort(keys, m, perm) != 0) return 6;
    uint64_t sum = 0;
    for (uint32_t i = 0; i < m; ++i) sum = sum * 1000003u + keys[i] + 7u * perm[i];
    oracle_encode_twopoint(rays, m, box, 64, keys2);
    for (uint32_t i = 0; i < m; ++i) sum = sum * 1000003u + keys2[i];
    oracle_encode_ppc(rays, m, n, child, boxes, 64, keys2);
    for (uint32_t i = 0; i < m; ++i) sum = sum * 1000003u + keys2[i];
    uint32_t top[8 + 2], low[(8 + 2) * 8];
    int t = oracle_select_mlhcc_cut(n, child, had, 8, 8, top, low);
    if (t <= 0) return 7;
    float* tb6 = malloc(sizeof(float) * 6 * (size_t)t);
    float* lb6 = malloc(sizeof(float) * 6 * (size_t)t * 8);
    for (int i = 0; i < t; ++i)
        for (int a = 0; a < 6; ++a) tb6[6 * i + a] = boxes[6 * (size_t)top[i] + a];
    for (int i = 0; i < t * 8; ++i)
        for (int a = 0; a < 6; ++a) lb6[6 * i + a] = boxes[6 * (size_t)low[i] + a];
    oracle_encode_mlhcc(rays, m, tb6, (uint32_t)t, lb6, 8, 16, keys2);
    for (uint32_t i = 0; i < m; ++i) sum = sum * 1000003u + keys2[i];
    float grid[64 * 6];
    oracle_grid_boxes(box, 4, 4, 4, grid);
    oracle_encode_hcc(rays, m, grid, 64, 64, keys2);
    for (uint32_t i = 0; i < m; ++i) sum = sum * 1000003u + keys2[i] + (uint64_t)oracle_slab(rays + 8 * (size_t)i, boxes);
    float* hits = malloc(sizeof(float) * 4 * m);
    float* hits2 = malloc(sizeof(float) * 4 * m);
    uint8_t* occ = malloc(m);
    uint8_t* occ2 = malloc(m);
    uint32_t* nn = malloc(sizeof(uint32_t) * m);
    uint32_t* nt = malloc(sizeof(uint32_t) * m);
    oracle_trace(n, child, leaf, boxes, tris, rays, perm, 0, m, 1, hits, NULL, nn, nt);
    oracle_trace(n, child, leaf, boxes, tris, rays, NULL, 0, m, 0, NULL, occ, NULL, NULL);
    oracle_brute_force(tris, n, rays, m, 1, hits2, NULL);
    oracle_brute_force(tris, n, rays, m, 0, NULL, occ2);
    uint32_t agree = 0, occ_agree = 0;
    for (uint32_t i = 0; i < m; ++i) {
        agree += ((const uint32_t*)hits)[4 * i + 1] == ((const uint32_t*)hits2)[4 * i + 1];
        occ_agree += occ[i] == occ2[i];
    }
    double anc = oracle_anc(keys, perm, m, 32);
    const uint32_t waves_n = (m + 63) / 64;
    uint32_t* waves = malloc(sizeof(uint32_t) * waves_n);
    uint64_t* wn = malloc(sizeof(uint64_t) * waves_n);
    uint64_t* wt = malloc(sizeof(uint64_t) * waves_n);
    uint32_t* ws = malloc(sizeof(uint32_t) * waves_n);
    for (uint32_t i = 0; i < waves_n; ++i) waves[i] = i;
    uint64_t fetch[2] = {0, 0};
    for (int order = 0; order < 2; ++order) {
        if (oracle_wave_fetches(n, child, leaf, boxes, tris, rays, perm, m, 64, 1, order, waves, waves_n, wn, wt, ws))
            return 8;
        for (uint32_t i = 0; i < waves_n; ++i) fetch[order] += wn[i] + wt[i];
    }
    printf("%u %u %u %u %llu %.6f %llu %llu %u\n", n, m, agree, occ_agree, (unsigned long long)sum, anc,
           (unsigned long long)fetch[0], (unsigned long long)fetch[1], oracle_morton3(1, 2, 3));
    free(tris); free(rays); free(codes); free(child); free(leaf); free(boxes); free(sorted); free(had); free(cb);
    free(keys); free(keys2); free(perm); free(tb6); free(lb6); free(hits); free(hits2); free(occ); free(occ2);
    free(nn); free(nt); free(waves); free(wn); free(wt); free(ws);
    return 0;
}
