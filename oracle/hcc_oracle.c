/*
 * Plain CPU oracle for the hierarchy-cut-code ray-reordering path
 * (Xiang et al., "Faster Ray Tracing through Hierarchy Cut Code", 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU path is checked against.  It is used by the tests, by the smoke
 * check and by the benchmark's CPU-baseline leg, and by nothing else.  It shares
 * no code, header, table or constant with the GPU library, and it includes none
 * of that library's files.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no FMA contraction, IEEE single-precision arithmetic on x86-64 SSE, so every
 * float operation below rounds exactly as written).
 *
 * Each function names the passage of the paper it follows.  Where the paper is
 * silent, the reading taken is stated at the function.  Functions without an
 * independent pin in the test-suite are marked "parity unpinned" (none at present).
 *
 * Conventions shared with the callers (Python side):
 *   triangles  : n x 9 float32, [v0xyz v1xyz v2xyz]
 *   rays       : n x 8 float32, [ox oy oz tmin dx dy dz tmax]
 *   node ids   : "unified" ids; internal node i -> i (0 <= i < n-1),
 *                leaf j (j-th triangle in Morton order) -> n-1+j.  Root = 0.
 *   boxes      : (2n-1) x 6 float32, [lo.x lo.y lo.z hi.x hi.y hi.z] by unified id
 *   child      : (n-1) x 2 uint32 unified ids (left, right)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MISS_PRIM 0xFFFFFFFFu

/* ------------------------------------------------------------------ helpers */

static float minf3(float a, float b, float c) { return fminf(fminf(a, b), c); }
static float maxf3(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

/* Scene bounding box over every vertex of every triangle. */
static void scene_box(const float* tris, uint32_t n, float lo[3], float hi[3]) {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (uint32_t i = 0; i < n; ++i)
        for (int v = 0; v < 3; ++v)
            for (int a = 0; a < 3; ++a) {
                float x = tris[9 * (size_t)i + 3 * v + a];
                if (x < lo[a]) lo[a] = x;
                if (x > hi[a]) hi[a] = x;
            }
}

void oracle_scene_box(const float* tris, uint32_t n, float* out6) {
    scene_box(tris, n, out6, out6 + 3);
}

/* ------------------------------------------------------------------ O1: Morton code
 * Morton code of a point (Section 3.2: interleaved quantised coordinates).  The
 * builder's reading: 10 bits per axis of the triangle-AABB centre, quantised
 * against the scene box, x taking the most significant bit of each triple. */
static uint32_t quantize10(float c, float lo, float hi) {
    float ext = hi - lo;
    float u = (ext > 0.0f) ? (c - lo) / ext : 0.0f;
    float q = floorf(u * 1024.0f);
    if (q < 0.0f) q = 0.0f;
    if (q > 1023.0f) q = 1023.0f;
    return (uint32_t)q;
}

uint32_t oracle_morton3(uint32_t qx, uint32_t qy, uint32_t qz) {
    uint32_t code = 0;
    for (int b = 9; b >= 0; --b) {
        code = (code << 1) | ((qx >> b) & 1u);
        code = (code << 1) | ((qy >> b) & 1u);
        code = (code << 1) | ((qz >> b) & 1u);
    }
    return code;
}

void oracle_morton_codes(const float* tris, uint32_t n, uint32_t* codes) {
    float lo[3], hi[3];
    scene_box(tris, n, lo, hi);
    for (uint32_t i = 0; i < n; ++i) {
        const float* t = tris + 9 * (size_t)i;
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            float mn = minf3(t[a], t[3 + a], t[6 + a]);
            float mx = maxf3(t[a], t[3 + a], t[6 + a]);
            float c = 0.5f * (mn + mx);
            q[a] = quantize10(c, lo[a], hi[a]);
        }
        codes[i] = oracle_morton3(q[0], q[1], q[2]);
    }
}

/* ------------------------------------------------------------------ O1: LBVH
 * Binary radix tree over the Morton-sorted triangles (the BVH of Section 3.1,
 * built as a linear BVH).  Sort: stable by Morton code, i.e. by (code, prim id).
 * Tree: over augmented keys (code << 32 | sorted position), a range [f, l] is
 * split after the last position that still shares more leading bits with key f
 * than key l does (split at the highest differing bit).  Numbering (Karras 2012):
 * root = internal 0; left child of a range [f, l] split at g is leaf g if f == g
 * else internal g; right child is leaf g+1 if g+1 == l else internal g+1.
 * Leaf box = triangle AABB; internal box = exact union of its children's boxes. */

typedef struct { uint32_t code; uint32_t prim; } code_prim;

static int cmp_code_prim(const void* pa, const void* pb) {
    const code_prim* a = (const code_prim*)pa;
    const code_prim* b = (const code_prim*)pb;
    if (a->code != b->code) return a->code < b->code ? -1 : 1;
    if (a->prim != b->prim) return a->prim < b->prim ? -1 : 1;
    return 0;
}

static int clz64(uint64_t x) { return x == 0 ? 64 : __builtin_clzll(x); }

static void tri_box(const float* t, float out[6]) {
    for (int a = 0; a < 3; ++a) {
        out[a] = minf3(t[a], t[3 + a], t[6 + a]);
        out[3 + a] = maxf3(t[a], t[3 + a], t[6 + a]);
    }
}

/* Returns 0 on success, -1 on bad input, -2 on allocation failure. */
int oracle_build_bvh(const float* tris, uint32_t n, uint32_t* child, uint32_t* leaf_prim,
                     float* boxes, uint32_t* sorted_codes) {
    if (n == 0) return -1;
    uint32_t* codes = (uint32_t*)malloc(sizeof(uint32_t) * n);
    code_prim* cp = (code_prim*)malloc(sizeof(code_prim) * n);
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * n);
    /* explicit work list of (first, last, id) in creation order */
    uint32_t* wf = (uint32_t*)malloc(sizeof(uint32_t) * n);
    uint32_t* wl = (uint32_t*)malloc(sizeof(uint32_t) * n);
    uint32_t* wi = (uint32_t*)malloc(sizeof(uint32_t) * n);
    if (!codes || !cp || !key || !wf || !wl || !wi) {
        free(codes); free(cp); free(key); free(wf); free(wl); free(wi);
        return -2;
    }
    oracle_morton_codes(tris, n, codes);
    for (uint32_t i = 0; i < n; ++i) { cp[i].code = codes[i]; cp[i].prim = i; }
    qsort(cp, n, sizeof(code_prim), cmp_code_prim);
    for (uint32_t j = 0; j < n; ++j) {
        leaf_prim[j] = cp[j].prim;
        key[j] = ((uint64_t)cp[j].code << 32) | (uint64_t)j;
        if (sorted_codes) sorted_codes[j] = cp[j].code;
        tri_box(tris + 9 * (size_t)cp[j].prim, boxes + 6 * (size_t)(n - 1 + j));
    }
    if (n > 1) {
        size_t top = 0, count = 0;
        wf[0] = 0; wl[0] = n - 1; wi[0] = 0; count = 1;
        while (top < count) {
            uint32_t f = wf[top], l = wl[top], id = wi[top];
            ++top;
            int d = clz64(key[f] ^ key[l]);
            uint32_t g = f;
            for (uint32_t j = f; j < l; ++j)
                if (clz64(key[f] ^ key[j]) > d) g = j;
            uint32_t left = (f == g) ? (n - 1 + g) : g;
            uint32_t right = (g + 1 == l) ? (n - 1 + g + 1) : (g + 1);
            child[2 * (size_t)id] = left;
            child[2 * (size_t)id + 1] = right;
            if (f != g) { wf[count] = f; wl[count] = g; wi[count] = g; ++count; }
            if (g + 1 != l) { wf[count] = g + 1; wl[count] = l; wi[count] = g + 1; ++count; }
        }
        /* children are created after their parent: union boxes in reverse order */
        for (size_t k = count; k-- > 0;) {
            uint32_t id = wi[k];
            const float* bl = boxes + 6 * (size_t)child[2 * (size_t)id];
            const float* br = boxes + 6 * (size_t)child[2 * (size_t)id + 1];
            float* b = boxes + 6 * (size_t)id;
            for (int a = 0; a < 3; ++a) {
                b[a] = fminf(bl[a], br[a]);
                b[3 + a] = fmaxf(bl[3 + a], br[3 + a]);
            }
        }
    }
    free(codes); free(cp); free(key); free(wf); free(wl); free(wi);
    return 0;
}

/* ------------------------------------------------------------------ O2: HAD, Eq. (1)
 * Leaf: TC * SA (TC = triangles in the leaf = 1 here); internal:
 * HAD_left + HAD_right + lambda * SA.  SA = full surface area of the node's box,
 * in double precision from the float box.  Reading: "density" of a leaf is taken
 * from Eq. (1) (TC*SA), not the prose (TC alone). */
static double box_sa(const float* b) {
    double dx = (double)b[3] - (double)b[0];
    double dy = (double)b[4] - (double)b[1];
    double dz = (double)b[5] - (double)b[2];
    return 2.0 * ((dx * dy + dy * dz) + dz * dx);
}

/* Post-order recursion over the tree (depth is at most 63 for 62-bit keys). */
static double had_rec(uint32_t n, const uint32_t* child, const float* boxes, double lambda,
                      uint32_t id, double* had) {
    if (id >= n - 1) {            /* leaf */
        double h = 1.0 * box_sa(boxes + 6 * (size_t)id);
        had[id] = h;
        return h;
    }
    double hl = had_rec(n, child, boxes, lambda, child[2 * (size_t)id], had);
    double hr = had_rec(n, child, boxes, lambda, child[2 * (size_t)id + 1], had);
    double h = (hl + hr) + lambda * box_sa(boxes + 6 * (size_t)id);
    had[id] = h;
    return h;
}

void oracle_had(uint32_t n, const uint32_t* child, const float* boxes, double lambda, double* had) {
    if (n == 0) return;
    if (n == 1) { had[0] = 1.0 * box_sa(boxes); return; }
    had_rec(n, child, boxes, lambda, 0, had);
}

/* ------------------------------------------------------------------ O3: cut, Alg. 2
 * Priority = HAD (largest first); ties broken by smaller unified id.  The queue
 * starts with the root; while it holds fewer than MaxQueueSize nodes, the head is
 * removed: a leaf goes to the cut list and MaxQueueSize shrinks by one, an internal
 * node is replaced by its two children.  Whatever is left in the queue joins the
 * cut.  Reading for a request larger than the number of leaves: stop when the
 * queue empties (cut = all leaves).  The cut is then ordered by HAD descending
 * (ties: id ascending), which is the bit order of the code (Section 4.2.2).
 * The queue is a plain array searched linearly: slow and obviously correct. */
static int before(double ha, uint32_t ia, double hb, uint32_t ib) {
    if (ha != hb) return ha > hb;
    return ia < ib;
}

/* Returns the cut size (<= cut_size), or -1 on bad input, -2 on allocation failure. */
int oracle_select_cut(uint32_t n, const uint32_t* child, const double* had, uint32_t cut_size,
                      uint32_t* cut_ids) {
    if (n == 0 || cut_size == 0) return -1;
    uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)cut_size + 2));
    uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)cut_size + 2));
    if (!q || !list) { free(q); free(list); return -2; }
    size_t qn = 0, ln = 0;
    int64_t max_q = cut_size;
    q[qn++] = 0;
    while ((int64_t)qn < max_q) {
        if (qn == 0) break;
        size_t best = 0;
        for (size_t k = 1; k < qn; ++k)
            if (before(had[q[k]], q[k], had[q[best]], q[best])) best = k;
        uint32_t node = q[best];
        q[best] = q[qn - 1];
        --qn;
        if (n == 1 || node >= n - 1) {
            list[ln++] = node;
            max_q -= 1;
        } else {
            q[qn++] = child[2 * (size_t)node];
            q[qn++] = child[2 * (size_t)node + 1];
        }
    }
    size_t m = 0;
    for (size_t k = 0; k < ln; ++k) cut_ids[m++] = list[k];
    for (size_t k = 0; k < qn; ++k) cut_ids[m++] = q[k];
    /* insertion sort by (HAD desc, id asc) */
    for (size_t i = 1; i < m; ++i) {
        uint32_t x = cut_ids[i];
        size_t j = i;
        while (j > 0 && before(had[x], x, had[cut_ids[j - 1]], cut_ids[j - 1])) {
            cut_ids[j] = cut_ids[j - 1];
            --j;
        }
        cut_ids[j] = x;
    }
    free(q); free(list);
    return (int)m;
}

/* ------------------------------------------------------------------ MLHCC cut, Alg. 3
 * Two-level cut of the multi-level hierarchy cut code (Section 4.3).  Top level: the
 * priority-queue search of Alg. 2 (largest HAD first, ties by smaller id) that keeps only
 * nodes with a sufficient subtree.  Reading of "sufficient": at least L leaves, so that a
 * low-level cut of exactly L nodes exists below the node.  When a node is removed from the
 * queue, its children with at least L leaves are pushed and the others are discarded; a node
 * none of whose children qualifies cannot be refined and joins the top-level list (as a leaf
 * does in Alg. 2, the target shrinking by one).  Top-level cut = that list + the queue,
 * ordered by HAD descending.  Low level: for each top node, the Alg. 2 cut of size L of its
 * subtree, ordered by HAD descending.  Returns the number of top nodes T' (<= top), or -1
 * on bad input, -2 on allocation failure.  low_ids: top x low entries (row i for top node i). */
static uint32_t count_leaves(uint32_t n, const uint32_t* child, uint32_t id, uint32_t* cache) {
    if (n == 1 || id >= n - 1) return 1;
    if (cache[id]) return cache[id];
    uint32_t c = count_leaves(n, child, child[2 * (size_t)id], cache) +
                 count_leaves(n, child, child[2 * (size_t)id + 1], cache);
    cache[id] = c;
    return c;
}

/* Alg. 2 below an arbitrary node (the same search as oracle_select_cut, rooted at 'root'). */
static int subtree_cut(uint32_t n, const uint32_t* child, const double* had, uint32_t root, uint32_t cut_size,
                       uint32_t* cut_ids) {
    uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)cut_size + 2));
    uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)cut_size + 2));
    if (!q || !list) { free(q); free(list); return -2; }
    size_t qn = 0, ln = 0;
    int64_t max_q = cut_size;
    q[qn++] = root;
    while ((int64_t)qn < max_q) {
        if (qn == 0) break;
        size_t best = 0;
        for (size_t k = 1; k < qn; ++k)
            if (before(had[q[k]], q[k], had[q[best]], q[best])) best = k;
        uint32_t node = q[best];
        q[best] = q[qn - 1];
        --qn;
        if (n == 1 || node >= n - 1) { list[ln++] = node; max_q -= 1; }
        else { q[qn++] = child[2 * (size_t)node]; q[qn++] = child[2 * (size_t)node + 1]; }
    }
    size_t m = 0;
    for (size_t k = 0; k < ln; ++k) cut_ids[m++] = list[k];
    for (size_t k = 0; k < qn; ++k) cut_ids[m++] = q[k];
    for (size_t i = 1; i < m; ++i) {
        uint32_t x = cut_ids[i];
        size_t j = i;
        while (j > 0 && before(had[x], x, had[cut_ids[j - 1]], cut_ids[j - 1])) { cut_ids[j] = cut_ids[j - 1]; --j; }
        cut_ids[j] = x;
    }
    free(q); free(list);
    return (int)m;
}

int oracle_select_mlhcc_cut(uint32_t n, const uint32_t* child, const double* had, uint32_t top, uint32_t low,
                            uint32_t* top_ids, uint32_t* low_ids) {
    if (n == 0 || top == 0 || low == 0) return -1;
    uint32_t* cache = (uint32_t*)calloc(n, sizeof(uint32_t));
    uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)top + 2));
    uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)top + 2));
    if (!cache || !q || !list) { free(cache); free(q); free(list); return -2; }
    size_t qn = 0, ln = 0;
    int64_t max_q = top;
    if (count_leaves(n, child, 0, cache) >= low) q[qn++] = 0;
    while ((int64_t)qn < max_q && qn > 0) {
        size_t best = 0;
        for (size_t k = 1; k < qn; ++k)
            if (before(had[q[k]], q[k], had[q[best]], q[best])) best = k;
        uint32_t node = q[best];
        q[best] = q[qn - 1];
        --qn;
        int pushed = 0;
        if (!(n == 1 || node >= n - 1)) {
            for (int c = 0; c < 2; ++c) {
                uint32_t ch = child[2 * (size_t)node + c];
                if (count_leaves(n, child, ch, cache) >= low) { q[qn++] = ch; ++pushed; }
            }
        }
        if (!pushed) { list[ln++] = node; max_q -= 1; }
    }
    size_t m = 0;
    for (size_t k = 0; k < ln; ++k) top_ids[m++] = list[k];
    for (size_t k = 0; k < qn; ++k) top_ids[m++] = q[k];
    for (size_t i = 1; i < m; ++i) {
        uint32_t x = top_ids[i];
        size_t j = i;
        while (j > 0 && before(had[x], x, had[top_ids[j - 1]], top_ids[j - 1])) { top_ids[j] = top_ids[j - 1]; --j; }
        top_ids[j] = x;
    }
    int rc = (int)m;
    for (size_t i = 0; i < m && rc >= 0; ++i) {
        int got = subtree_cut(n, child, had, top_ids[i], low, low_ids + (size_t)i * low);
        if (got != (int)low) rc = got < 0 ? got : -1;
    }
    free(cache); free(q); free(list);
    return rc;
}

/* ------------------------------------------------------------------ regular grid (control)
 * The regular-grid encoding of Section 5: the cut boxes are replaced by the cells of a uniform
 * gx x gy x gz grid over the scene box.  Reading: cell boundaries at lo + ext * i / g computed
 * in double and rounded to float; cells numbered x fastest, then y, then z, and cell 0 takes
 * the most significant bit (there is no HAD to order them). */
void oracle_grid_boxes(const float* scene_lohi, uint32_t gx, uint32_t gy, uint32_t gz, float* boxes) {
    const uint32_t g[3] = {gx, gy, gz};
    size_t k = 0;
    for (uint32_t z = 0; z < gz; ++z)
        for (uint32_t y = 0; y < gy; ++y)
            for (uint32_t x = 0; x < gx; ++x) {
                const uint32_t idx[3] = {x, y, z};
                for (int a = 0; a < 3; ++a) {
                    double lo = scene_lohi[a], ext = (double)scene_lohi[3 + a] - (double)scene_lohi[a];
                    boxes[6 * k + a] = (float)(lo + ext * (double)idx[a] / (double)g[a]);
                    boxes[6 * k + 3 + a] = (float)(lo + ext * (double)(idx[a] + 1) / (double)g[a]);
                }
                ++k;
            }
}

/* ------------------------------------------------------------------ slab test
 * Ray against an axis-aligned box over the ray's own segment [tmin, tmax].  The
 * paper does not spell the test out; reading: IEEE division for 1/d, minNum /
 * maxNum (fminf / fmaxf, which drop a NaN operand), and the far distance scaled
 * by 1 + 3*2^-23 so that rounding never loses a true intersection (Ize 2013). */
static int slab_hit(const float o[3], const float inv[3], float tmin, float tmax, const float* b,
                    float* tnear_out) {
    float tn[3], tf[3];
    for (int a = 0; a < 3; ++a) {
        float t0 = (b[a] - o[a]) * inv[a];
        float t1 = (b[3 + a] - o[a]) * inv[a];
        tn[a] = fminf(t0, t1);
        tf[a] = fmaxf(t0, t1) * 0x1.000006p+0f;
    }
    float tnear = fmaxf(fmaxf(fmaxf(tn[0], tn[1]), tn[2]), tmin);
    float tfar = fminf(fminf(fminf(tf[0], tf[1]), tf[2]), tmax);
    if (tnear_out) *tnear_out = tnear;
    return tnear <= tfar;
}

int oracle_slab(const float* ray8, const float* box6) {
    float o[3] = {ray8[0], ray8[1], ray8[2]};
    float inv[3] = {1.0f / ray8[4], 1.0f / ray8[5], 1.0f / ray8[6]};
    return slab_hit(o, inv, ray8[3], ray8[7], box6, 0);
}

/* ------------------------------------------------------------------ O4: HCC key, Alg. 1
 * One bit per cut node: bit (K-1-i) is set iff the ray meets cut node i, the cut
 * being ordered by HAD descending so the highest-HAD node is the most significant
 * bit (Section 4.2.2).  Reading when the cut and the key length differ: only the
 * first min(C, K) cut nodes are encoded; remaining low bits are zero. */
void oracle_encode_hcc(const float* rays, uint32_t n, const float* cut_boxes, uint32_t c_eff,
                       uint32_t key_bits, uint64_t* keys) {
    uint32_t m = c_eff < key_bits ? c_eff : key_bits;
    for (uint32_t r = 0; r < n; ++r) {
        const float* ry = rays + 8 * (size_t)r;
        float o[3] = {ry[0], ry[1], ry[2]};
        float inv[3] = {1.0f / ry[4], 1.0f / ry[5], 1.0f / ry[6]};
        uint64_t key = 0;
        for (uint32_t i = 0; i < m; ++i)
            if (slab_hit(o, inv, ry[3], ry[7], cut_boxes + 6 * (size_t)i, 0))
                key |= (uint64_t)1 << (key_bits - 1 - i);
        keys[r] = key;
    }
}

/* ------------------------------------------------------------------ MLHCC key (Section 4.3)
 * The key has key_bits = top + low bits.  Bit (key_bits-1-i) records whether the ray meets
 * top node i (top nodes in HAD order, i < t_eff <= top); the representative is the first top
 * node met in that order; bit (low-1-j) records whether the ray meets node j of the
 * representative's low-level cut.  A ray meeting no top node has zero low bits. */
void oracle_encode_mlhcc(const float* rays, uint32_t n, const float* top_boxes, uint32_t t_eff,
                         const float* low_boxes, uint32_t low, uint32_t key_bits, uint64_t* keys) {
    for (uint32_t r = 0; r < n; ++r) {
        const float* ry = rays + 8 * (size_t)r;
        float o[3] = {ry[0], ry[1], ry[2]};
        float inv[3] = {1.0f / ry[4], 1.0f / ry[5], 1.0f / ry[6]};
        uint64_t key = 0;
        int rep = -1;
        for (uint32_t i = 0; i < t_eff; ++i) {
            if (slab_hit(o, inv, ry[3], ry[7], top_boxes + 6 * (size_t)i, 0)) {
                key |= (uint64_t)1 << (key_bits - 1 - i);
                if (rep < 0) rep = (int)i;
            }
        }
        if (rep >= 0) {
            const float* lb = low_boxes + 6 * (size_t)rep * low;
            for (uint32_t j = 0; j < low; ++j)
                if (slab_hit(o, inv, ry[3], ry[7], lb + 6 * (size_t)j, 0)) key |= (uint64_t)1 << (low - 1 - j);
        }
        keys[r] = key;
    }
}

/* ------------------------------------------------------------------ PPC key (Section 4.1)
 * Prefix path code: every ray walks the BVH in one and the same forced order and each box
 * test on the walk appends one bit (1 = the ray meets the box), most significant first, until
 * key_bits tests have been made.  Readings: expanding a node tests its two children, child 0
 * then child 1; the walk is depth first with child 0's subtree before child 1's; only
 * internal children that were met are expanded; the segment is the ray's own [tmin, tmax]
 * throughout (no shortening by hits, since no triangle is tested); a walk that runs out of
 * nodes leaves the remaining low bits zero.  A one-triangle BVH makes the single test of its
 * root leaf's box.  n_tris is the triangle count, child the (n-1) x 2 unified child ids and
 * boxes the (2n-1) x 6 node boxes. */
void oracle_encode_ppc(const float* rays, uint32_t n, uint32_t n_tris, const uint32_t* child, const float* boxes,
                       uint32_t key_bits, uint64_t* keys) {
    uint32_t* stack = (uint32_t*)malloc(sizeof(uint32_t) * (key_bits + 2));
    for (uint32_t r = 0; r < n; ++r) {
        const float* ry = rays + 8 * (size_t)r;
        float o[3] = {ry[0], ry[1], ry[2]};
        float inv[3] = {1.0f / ry[4], 1.0f / ry[5], 1.0f / ry[6]};
        uint64_t key = 0;
        if (n_tris == 1) {
            if (slab_hit(o, inv, ry[3], ry[7], boxes, 0)) key = (uint64_t)1 << (key_bits - 1);
            keys[r] = key;
            continue;
        }
        uint32_t bits = 0, sp = 0;
        stack[sp++] = 0;
        while (sp > 0 && bits < key_bits) {
            uint32_t node = stack[--sp];
            int met[2] = {0, 0};
            for (int c = 0; c < 2 && bits < key_bits; ++c) {
                met[c] = slab_hit(o, inv, ry[3], ry[7], boxes + 6 * (size_t)child[2 * node + c], 0);
                if (met[c]) key |= (uint64_t)1 << (key_bits - 1 - bits);
                ++bits;
            }
            /* child 1 goes below child 0 so that child 0's subtree is walked first */
            for (int c = 1; c >= 0; --c)
                if (met[c] && child[2 * node + c] < n_tris - 1) stack[sp++] = child[2 * node + c];
        }
        keys[r] = key;
    }
    free(stack);
}

/* ------------------------------------------------------------------ O5: TwoPoint key
 * Baseline of Section 3.2 / Section 5: 6-D Morton code of the origin and an
 * estimated termination point at fixed distance 0.25 * (largest scene extent)
 * along the normalised direction (clipped to the ray's own segment).  Reading for
 * the missing bit-layout figure: each of the six coordinates is quantised against
 * the scene box; dimension d gets floor(K/6) bits plus one if d < K mod 6; bits
 * are interleaved from the most significant level down, cycling dims 0..5
 * (ox, oy, oz, ex, ey, ez). */
void oracle_encode_twopoint(const float* rays, uint32_t n, const float* scene_lohi, uint32_t key_bits,
                            uint64_t* keys) {
    const float* lo = scene_lohi;
    const float* hi = scene_lohi + 3;
    float ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    float L = fmaxf(fmaxf(ext[0], ext[1]), ext[2]);
    float t_est = 0.25f * L;
    uint32_t bits[6];
    for (int d = 0; d < 6; ++d) bits[d] = key_bits / 6 + ((uint32_t)d < key_bits % 6 ? 1u : 0u);
    for (uint32_t r = 0; r < n; ++r) {
        const float* ry = rays + 8 * (size_t)r;
        float len = sqrtf((ry[4] * ry[4] + ry[5] * ry[5]) + ry[6] * ry[6]);
        float dist = fminf(t_est, ry[7] * len);
        float p[6];
        for (int a = 0; a < 3; ++a) {
            float dn = ry[4 + a] / len;
            p[a] = ry[a];
            p[3 + a] = ry[a] + dn * dist;
        }
        uint32_t q[6];
        for (int d = 0; d < 6; ++d) {
            int a = d % 3;
            float u = ext[a] > 0.0f ? (p[d] - lo[a]) / ext[a] : 0.0f;
            u = fminf(fmaxf(u, 0.0f), 1.0f);
            float scale = (float)(1u << bits[d]);
            float qf = floorf(u * scale);
            uint32_t qi = (bits[d] == 0) ? 0u : (uint32_t)qf;
            uint32_t qmax = (bits[d] == 0) ? 0u : ((1u << bits[d]) - 1u);
            q[d] = qi > qmax ? qmax : qi;
        }
        uint64_t key = 0;
        for (uint32_t level = 0; level < bits[0]; ++level)
            for (int d = 0; d < 6; ++d)
                if (level < bits[d])
                    key = (key << 1) | ((q[d] >> (bits[d] - 1 - level)) & 1u);
        keys[r] = key;
    }
}

/* ------------------------------------------------------------------ O6: sort
 * Keys sorted as unsigned integers (Section 4.2.3), ascending; the output is the
 * permutation of ray indices (the paper sorts ray indices, Section 5).  Stable:
 * equal keys keep their input order (the comparison on the index makes qsort
 * stable). */
typedef struct { uint64_t key; uint32_t idx; } key_idx;

static int cmp_key_idx(const void* pa, const void* pb) {
    const key_idx* a = (const key_idx*)pa;
    const key_idx* b = (const key_idx*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

int oracle_sort(const uint64_t* keys, uint32_t n, uint32_t* perm) {
    key_idx* v = (key_idx*)malloc(sizeof(key_idx) * (n ? n : 1));
    if (!v) return -2;
    for (uint32_t i = 0; i < n; ++i) { v[i].key = keys[i]; v[i].idx = i; }
    qsort(v, n, sizeof(key_idx), cmp_key_idx);
    for (uint32_t i = 0; i < n; ++i) perm[i] = v[i].idx;
    free(v);
    return 0;
}

/* ------------------------------------------------------------------ O7: trace
 * Ray/triangle test: Moller-Trumbore (1997), double sided, single precision, in
 * this operation order; det == 0 is a miss; a hit needs u >= 0, v >= 0, u+v <= 1
 * and tmin < t < tmax.  Closest hit = the smallest (t, prim id) pair over every
 * triangle hit, so the answer does not depend on traversal order; any hit = true
 * iff some triangle is hit in the segment. */
static int tri_hit(const float* tri, const float o[3], const float d[3], float tmin, float tmax,
                   float* t_out, float* u_out, float* v_out) {
    float e1[3] = {tri[3] - tri[0], tri[4] - tri[1], tri[5] - tri[2]};
    float e2[3] = {tri[6] - tri[0], tri[7] - tri[1], tri[8] - tri[2]};
    float p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    float det = (e1[0] * p[0] + e1[1] * p[1]) + e1[2] * p[2];
    if (det == 0.0f) return 0;
    float inv = 1.0f / det;
    float s[3] = {o[0] - tri[0], o[1] - tri[1], o[2] - tri[2]};
    float u = ((s[0] * p[0] + s[1] * p[1]) + s[2] * p[2]) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return 0;
    float q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    float v = ((d[0] * q[0] + d[1] * q[1]) + d[2] * q[2]) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return 0;
    float t = ((e2[0] * q[0] + e2[1] * q[1]) + e2[2] * q[2]) * inv;
    if (!(t > tmin && t < tmax)) return 0;
    *t_out = t; *u_out = u; *v_out = v;
    return 1;
}

typedef struct {
    uint32_t n;
    const uint32_t* child;
    const uint32_t* leaf_prim;
    const float* boxes;
    const float* tris;
} bvh_view;

/* Near-first depth-first traversal with an explicit stack.  'closest' selects
 * closest-hit (1) or any-hit (0).  A popped node is tested against the segment
 * [tmin, best t so far]; an internal node pushes the children whose boxes pass,
 * far child first so that the nearer one (smaller entry distance; child 0 on a
 * tie) is popped next.  Every triangle reached is tested against the ray's full
 * segment and kept if its (t, prim id) pair is smaller than the best so far.
 * Counters: boxes passed at pop time, and triangle tests. */
static void trace_one(const bvh_view* b, const float* ray, int closest, float* t_out, uint32_t* prim_out,
                      float* u_out, float* v_out, uint8_t* occ_out, uint32_t* n_nodes, uint32_t* n_tris) {
    float o[3] = {ray[0], ray[1], ray[2]};
    float d[3] = {ray[4], ray[5], ray[6]};
    float inv[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
    float tmin = ray[3], tmax = ray[7];
    float best_t = tmax;
    uint32_t best_prim = MISS_PRIM;
    float best_u = 0.0f, best_v = 0.0f;
    int found = 0;
    uint32_t visits = 0, tests = 0;
    uint32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;   /* root: unified id 0 (internal 0, or leaf 0 when n == 1) */
    while (sp > 0) {
        uint32_t id = stack[--sp];
        if (!slab_hit(o, inv, tmin, best_t, b->boxes + 6 * (size_t)id, 0)) continue;
        ++visits;
        if (b->n == 1 || id >= b->n - 1) {
            uint32_t leaf = (b->n == 1) ? 0 : id - (b->n - 1);
            uint32_t prim = b->leaf_prim[leaf];
            float t, u, v;
            ++tests;
            if (!tri_hit(b->tris + 9 * (size_t)prim, o, d, tmin, tmax, &t, &u, &v)) continue;
            if (!closest) { found = 1; break; }
            if (!found || t < best_t || (t == best_t && prim < best_prim)) {
                best_t = t; best_prim = prim; best_u = u; best_v = v; found = 1;
            }
            continue;
        }
        uint32_t c0 = b->child[2 * (size_t)id], c1 = b->child[2 * (size_t)id + 1];
        float n0, n1;
        int h0 = slab_hit(o, inv, tmin, best_t, b->boxes + 6 * (size_t)c0, &n0);
        int h1 = slab_hit(o, inv, tmin, best_t, b->boxes + 6 * (size_t)c1, &n1);
        if (h0 && h1) {
            if (n1 < n0) { stack[sp++] = c0; stack[sp++] = c1; }
            else { stack[sp++] = c1; stack[sp++] = c0; }
        } else if (h0) {
            stack[sp++] = c0;
        } else if (h1) {
            stack[sp++] = c1;
        }
    }
    if (closest) {
        *t_out = found ? best_t : INFINITY;
        *prim_out = found ? best_prim : MISS_PRIM;
        *u_out = found ? best_u : 0.0f;
        *v_out = found ? best_v : 0.0f;
    } else {
        *occ_out = (uint8_t)found;
    }
    if (n_nodes) *n_nodes = visits;
    if (n_tris) *n_tris = tests;
}

/* Trace rays[perm[k]] for k in [k0, k1) (perm may be NULL = identity); results go
 * to the ORIGINAL ray index.  hits: 4 words per ray (t, prim, u, v). */
void oracle_trace(uint32_t n_tris, const uint32_t* child, const uint32_t* leaf_prim, const float* boxes,
                  const float* tris, const float* rays, const uint32_t* perm, uint32_t k0, uint32_t k1,
                  int closest, float* hits, uint8_t* occluded, uint32_t* n_nodes, uint32_t* n_tests) {
    bvh_view b = {n_tris, child, leaf_prim, boxes, tris};
    for (uint32_t k = k0; k < k1; ++k) {
        uint32_t r = perm ? perm[k] : k;
        float t = 0, u = 0, v = 0;
        uint32_t prim = 0;
        uint8_t occ = 0;
        trace_one(&b, rays + 8 * (size_t)r, closest, &t, &prim, &u, &v, &occ,
                  n_nodes ? n_nodes + r : 0, n_tests ? n_tests + r : 0);
        if (closest) {
            hits[4 * (size_t)r] = t;
            memcpy(hits + 4 * (size_t)r + 1, &prim, 4);
            hits[4 * (size_t)r + 2] = u;
            hits[4 * (size_t)r + 3] = v;
        } else {
            occluded[r] = occ;
        }
    }
}

/* Brute force over every triangle, same triangle test and tie rule. */
void oracle_brute_force(const float* tris, uint32_t n_tris, const float* rays, uint32_t n_rays, int closest,
                        float* hits, uint8_t* occluded) {
    for (uint32_t r = 0; r < n_rays; ++r) {
        const float* ry = rays + 8 * (size_t)r;
        float o[3] = {ry[0], ry[1], ry[2]};
        float d[3] = {ry[4], ry[5], ry[6]};
        float best_t = INFINITY, best_u = 0, best_v = 0;
        uint32_t best_prim = MISS_PRIM;
        int found = 0;
        for (uint32_t p = 0; p < n_tris; ++p) {
            float t, u, v;
            if (!tri_hit(tris + 9 * (size_t)p, o, d, ry[3], ry[7], &t, &u, &v)) continue;
            if (!found || t < best_t || (t == best_t && p < best_prim)) {
                best_t = t; best_prim = p; best_u = u; best_v = v; found = 1;
            }
            if (!closest) break;
        }
        if (closest) {
            hits[4 * (size_t)r] = best_t;
            memcpy(hits + 4 * (size_t)r + 1, &best_prim, 4);
            hits[4 * (size_t)r + 2] = best_u;
            hits[4 * (size_t)r + 3] = best_v;
        } else {
            occluded[r] = (uint8_t)found;
        }
    }
}

/* ------------------------------------------------------------------ O8: wave model, ANC
 * Metrics, not parity.  Average number of distinct codes per group of 'width'
 * consecutive rays in trace order (Section 6.5, Table 6: per warp). */
double oracle_anc(const uint64_t* keys, const uint32_t* perm, uint32_t n, uint32_t width) {
    if (n == 0 || width == 0) return 0.0;
    uint64_t* buf = (uint64_t*)malloc(sizeof(uint64_t) * width);
    if (!buf) return -1.0;
    double total = 0.0;
    uint32_t groups = 0;
    for (uint32_t g0 = 0; g0 < n; g0 += width) {
        uint32_t m = (n - g0 < width) ? n - g0 : width;
        uint32_t distinct = 0;
        for (uint32_t i = 0; i < m; ++i) {
            uint64_t k = keys[perm ? perm[g0 + i] : g0 + i];
            int seen = 0;
            for (uint32_t j = 0; j < distinct; ++j)
                if (buf[j] == k) { seen = 1; break; }
            if (!seen) buf[distinct++] = k;
        }
        total += distinct;
        ++groups;
    }
    free(buf);
    return total / groups;
}

/* ------------------------------------------------------------------ O8: lockstep wave model
 * Order-dependent fetch count behind the paper's coherence argument (Section 3.1: rays
 * of one warp that walk similar paths share their node fetches; Table 6 in Section 6.5
 * measures the same property as codes per warp).  Rays are taken in trace order
 * (perm[k], or k when perm is NULL) and grouped into waves of `width` consecutive rays.
 * Every ray's traversal is a sequence of steps.  In lockstep execution step s of a wave
 * runs for every lane whose traversal has more than s steps, and each distinct node and
 * each distinct triangle those lanes touch at step s is fetched once for the wave.  The
 * wave's node (triangle) fetches are these distinct counts summed over its steps.
 *
 * Two traversal orders are modelled:
 *   order 0 -- the traversal of O7 above: one step per popped node whose box passes the
 *              segment [tmin, best t]; an internal node is a node fetch, a leaf is a
 *              triangle fetch.
 *   order 1 -- child-test traversal: a step fetches the current internal node and tests
 *              both children's boxes against [tmin, best t] (tmax for any hit); the
 *              triangle of every hit leaf child is tested in the same step (triangle
 *              fetches); the step then continues with the hit internal child of smaller
 *              entry distance (child 0 on a tie) and pushes the other hit internal
 *              child, or, with no hit internal child, pops the stack, the popped node
 *              being fetched at the next step without a new box test.  The traversal
 *              ends when nothing is left to pop, and for any hit after the step that
 *              found one.  A BVH of one triangle has no node fetch and one triangle
 *              fetch at step 0.
 * Node ids are unified ids (internal node i -> i, leaf j -> n-1+j); a triangle fetch is
 * identified by its leaf.
 * Metrics, not parity: pinned by hand-counted cases and an independent re-implementation
 * in the tests. */

typedef struct {
    uint32_t* node;      /* per step: node id fetched, or MISS_PRIM for none */
    uint32_t* leaf_a;    /* per step: first triangle (leaf id) fetched, or MISS_PRIM */
    uint32_t* leaf_b;    /* per step: second triangle (order 1: the other child), or MISS_PRIM */
    uint32_t len, cap;
} step_list;

static int steps_push(step_list* L, uint32_t node, uint32_t la, uint32_t lb) {
    if (L->len == L->cap) {
        uint32_t cap = L->cap ? 2 * L->cap : 64;
        uint32_t* a = (uint32_t*)realloc(L->node, sizeof(uint32_t) * cap);
        if (!a) return -1;
        L->node = a;
        a = (uint32_t*)realloc(L->leaf_a, sizeof(uint32_t) * cap);
        if (!a) return -1;
        L->leaf_a = a;
        a = (uint32_t*)realloc(L->leaf_b, sizeof(uint32_t) * cap);
        if (!a) return -1;
        L->leaf_b = a;
        L->cap = cap;
    }
    L->node[L->len] = node;
    L->leaf_a[L->len] = la;
    L->leaf_b[L->len] = lb;
    ++L->len;
    return 0;
}

/* Closest-hit bookkeeping shared by both orders: test the triangle of leaf `leaf`, keep the
 * smallest (t, prim) pair; returns 1 on a hit in the segment. */
static int model_leaf(const bvh_view* b, uint32_t leaf, const float o[3], const float d[3], float tmin,
                      float tmax, int* found, float* best_t, uint32_t* best_prim) {
    uint32_t prim = b->leaf_prim[leaf];
    float t, u, v;
    if (!tri_hit(b->tris + 9 * (size_t)prim, o, d, tmin, tmax, &t, &u, &v)) return 0;
    if (!*found || t < *best_t || (t == *best_t && prim < *best_prim)) {
        *best_t = t;
        *best_prim = prim;
        *found = 1;
    }
    return 1;
}

/* The steps of one ray's traversal in the given order (see above). */
static int ray_steps(const bvh_view* b, const float* ray, int closest, int order, step_list* L) {
    float o[3] = {ray[0], ray[1], ray[2]};
    float d[3] = {ray[4], ray[5], ray[6]};
    float inv[3] = {1.0f / d[0], 1.0f / d[1], 1.0f / d[2]};
    float tmin = ray[3], tmax = ray[7];
    float best_t = tmax;
    uint32_t best_prim = MISS_PRIM;
    int found = 0;
    uint32_t stack[128];
    int sp = 0;
    const uint32_t n_int = b->n - 1;
    L->len = 0;
    if (b->n == 1) {   /* the root is the only leaf */
        return steps_push(L, MISS_PRIM, 0, MISS_PRIM);
    }
    if (order == 0) {
        stack[sp++] = 0;
        while (sp > 0) {
            uint32_t id = stack[--sp];
            if (!slab_hit(o, inv, tmin, best_t, b->boxes + 6 * (size_t)id, 0)) continue;
            if (id >= n_int) {
                if (steps_push(L, MISS_PRIM, id, MISS_PRIM)) return -1;
                int hit = model_leaf(b, id - n_int, o, d, tmin, tmax, &found, &best_t, &best_prim);
                if (hit && !closest) break;
                continue;
            }
            if (steps_push(L, id, MISS_PRIM, MISS_PRIM)) return -1;
            uint32_t c0 = b->child[2 * (size_t)id], c1 = b->child[2 * (size_t)id + 1];
            float n0, n1;
            int h0 = slab_hit(o, inv, tmin, best_t, b->boxes + 6 * (size_t)c0, &n0);
            int h1 = slab_hit(o, inv, tmin, best_t, b->boxes + 6 * (size_t)c1, &n1);
            if (h0 && h1) {
                if (n1 < n0) { stack[sp++] = c0; stack[sp++] = c1; }
                else { stack[sp++] = c1; stack[sp++] = c0; }
            } else if (h0) {
                stack[sp++] = c0;
            } else if (h1) {
                stack[sp++] = c1;
            }
            if (sp > 126) return -2;
        }
        return 0;
    }
    /* order 1 */
    uint32_t node = 0;
    while (1) {
        uint32_t c0 = b->child[2 * (size_t)node], c1 = b->child[2 * (size_t)node + 1];
        float lim = closest ? best_t : tmax;
        float n0, n1;
        int h0 = slab_hit(o, inv, tmin, lim, b->boxes + 6 * (size_t)c0, &n0);
        int h1 = slab_hit(o, inv, tmin, lim, b->boxes + 6 * (size_t)c1, &n1);
        int leaf0 = h0 && c0 >= n_int, leaf1 = h1 && c1 >= n_int;
        if (steps_push(L, node, leaf0 ? c0 : MISS_PRIM, leaf1 ? c1 : MISS_PRIM)) return -1;
        int any = 0;
        if (leaf0) any |= model_leaf(b, c0 - n_int, o, d, tmin, tmax, &found, &best_t, &best_prim);
        if (leaf1) any |= model_leaf(b, c1 - n_int, o, d, tmin, tmax, &found, &best_t, &best_prim);
        if (!closest && any) break;
        int in0 = h0 && !leaf0, in1 = h1 && !leaf1;
        if (in0 && in1) {
            if (n1 < n0) { stack[sp++] = c0; node = c1; }
            else { stack[sp++] = c1; node = c0; }
            if (sp > 126) return -2;
        } else if (in0) {
            node = c0;
        } else if (in1) {
            node = c1;
        } else {
            if (sp == 0) break;
            node = stack[--sp];
        }
    }
    return 0;
}

/* Distinct values among v[0..m) that are not MISS_PRIM (m is at most a few hundred). */
static uint32_t count_distinct(uint32_t* v, uint32_t m) {
    uint32_t distinct = 0;
    for (uint32_t i = 0; i < m; ++i) {
        if (v[i] == MISS_PRIM) continue;
        int seen = 0;
        for (uint32_t j = 0; j < i; ++j)
            if (v[j] == v[i]) { seen = 1; break; }
        if (!seen) ++distinct;
    }
    return distinct;
}

/* Wave fetches of the listed waves: wave w holds trace positions [w*width, (w+1)*width)
 * clipped to n.  out_nodes[i] / out_tris[i] receive the fetches of waves[i]; out_steps[i]
 * (nullable) the number of lockstep steps (the longest traversal of the wave).
 * Returns 0, or a negative value on a bad argument or exhausted memory. */
int oracle_wave_fetches(uint32_t n_tris, const uint32_t* child, const uint32_t* leaf_prim, const float* boxes,
                        const float* tris, const float* rays, const uint32_t* perm, uint32_t n, uint32_t width,
                        int closest, int order, const uint32_t* waves, uint32_t n_waves, uint64_t* out_nodes,
                        uint64_t* out_tris, uint32_t* out_steps) {
    if (width == 0 || width > 1024 || n_tris == 0 || (order != 0 && order != 1)) return -3;
    bvh_view b = {n_tris, child, leaf_prim, boxes, tris};
    step_list* lanes = (step_list*)calloc(width, sizeof(step_list));
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * 2 * width);
    int rc = 0;
    if (!lanes || !ids) { rc = -1; goto done; }
    for (uint32_t i = 0; i < n_waves; ++i) {
        uint64_t k0 = (uint64_t)waves[i] * width;
        uint32_t m = k0 >= n ? 0 : (uint32_t)((n - k0 < width) ? n - k0 : width);
        uint32_t longest = 0;
        for (uint32_t l = 0; l < m; ++l) {
            uint32_t r = perm ? perm[k0 + l] : (uint32_t)(k0 + l);
            rc = ray_steps(&b, rays + 8 * (size_t)r, closest, order, &lanes[l]);
            if (rc) goto done;
            if (lanes[l].len > longest) longest = lanes[l].len;
        }
        uint64_t nodes = 0, trisf = 0;
        for (uint32_t s = 0; s < longest; ++s) {
            uint32_t c = 0;
            for (uint32_t l = 0; l < m; ++l)
                if (s < lanes[l].len) ids[c++] = lanes[l].node[s];
            nodes += count_distinct(ids, c);
            c = 0;
            for (uint32_t l = 0; l < m; ++l)
                if (s < lanes[l].len) { ids[c++] = lanes[l].leaf_a[s]; ids[c++] = lanes[l].leaf_b[s]; }
            trisf += count_distinct(ids, c);
        }
        out_nodes[i] = nodes;
        out_tris[i] = trisf;
        if (out_steps) out_steps[i] = longest;
    }
done:
    if (lanes) {
        for (uint32_t l = 0; l < width; ++l) { free(lanes[l].node); free(lanes[l].leaf_a); free(lanes[l].leaf_b); }
        free(lanes);
    }
    free(ids);
    return rc;
}
