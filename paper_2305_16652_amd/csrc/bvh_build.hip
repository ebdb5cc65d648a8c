// LBVH construction and HAD on gfx950 (the acceleration structure of Section 3.1 and
// the hierarchically accumulated density of Eq. 1, Section 4.2.2).
//
//   scene box (two-level min/max reduction, exact)
//   -> 30-bit Morton code of each triangle's AABB centre (10 bits per axis, x on top)
//   -> stable radix sort of (code, triangle index)
//   -> Karras (2012) radix tree: every internal node finds its range and split on its own
//   -> leaves: triangles re-laid in Morton order as (v0, e1, e2, index), leaf boxes, leaf HAD
//   -> bottom-up pass with one arrival counter per internal node: the second child to
//      arrive unions the two boxes, fills the parent's 64-byte node and its HAD.
// Everything is exact or rounds in a fixed operation order, so the tree, boxes and HAD
// are identical from run to run and to a plain sequential build.
#include "hcc_internal.h"

namespace hcc {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;

__global__ __launch_bounds__(256) void k_bounds_partial(const float* __restrict__ tris, uint32_t n,
                                                        float* __restrict__ partial) {
    __shared__ float s[6][256];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const size_t nv = (size_t)n * 3;
    for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (size_t)gridDim.x * 256) {
        const float* p = tris + 3 * v;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], p[a]);
            hi[a] = fmaxf(hi[a], p[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + off]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_bounds_final(const float* __restrict__ partial, uint32_t nblocks,
                                                      float* __restrict__ box) {
    __shared__ float s[6][256];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], partial[b * 6 + a]);
            hi[a] = fmaxf(hi[a], partial[b * 6 + 3 + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + off]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) box[threadIdx.x] = s[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t spread3(uint32_t x) {   // 10 bits -> every third bit
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t quant10(float c, float lo, float hi) {
    const float ext = hi - lo;
    const float u = ext > 0.0f ? (c - lo) / ext : 0.0f;
    float q = floorf(u * 1024.0f);
    q = fminf(fmaxf(q, 0.0f), 1023.0f);
    return (uint32_t)q;
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ tris, uint32_t n,
                                                const float* __restrict__ box, uint32_t* __restrict__ codes) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float* t = tris + 9 * (size_t)i;
    uint32_t q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float mn = fminf(fminf(t[a], t[3 + a]), t[6 + a]);
        const float mx = fmaxf(fmaxf(t[a], t[3 + a]), t[6 + a]);
        const float c = 0.5f * (mn + mx);
        q[a] = quant10(c, box[a], box[3 + a]);
    }
    codes[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
}

// Common-prefix length of the augmented keys (code << 32 | position); -1 out of range.
__device__ __forceinline__ int delta(const uint32_t* __restrict__ codes, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    const uint64_t a = ((uint64_t)codes[i] << 32) | (uint64_t)i;
    const uint64_t b = ((uint64_t)codes[j] << 32) | (uint64_t)j;
    return __clzll((long long)(a ^ b));
}

__global__ __launch_bounds__(256) void k_karras(const uint32_t* __restrict__ codes, uint32_t n,
                                                uint32_t* __restrict__ child, uint32_t* __restrict__ parent) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n_int = (int64_t)n - 1;
    if (i >= n_int) return;
    const int64_t d = (delta(codes, n, i, i + 1) - delta(codes, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = delta(codes, n, i, i - d);
    int64_t lmax = 2;
    while (delta(codes, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(codes, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = delta(codes, n, i, j);
    int64_t s = 0;
    for (int64_t div = 2;; div <<= 1) {
        const int64_t t = (l + div - 1) / div;
        if (delta(codes, n, i, i + (s + t) * d) > dnode) s += t;
        if (t == 1) break;
    }
    const int64_t g = i + s * d + (d < 0 ? -1 : 0);
    const int64_t first = i < j ? i : j, last = i < j ? j : i;
    const uint32_t left = (uint32_t)(first == g ? n_int + g : g);
    const uint32_t right = (uint32_t)(last == g + 1 ? n_int + g + 1 : g + 1);
    child[2 * i] = left;
    child[2 * i + 1] = right;
    parent[left] = (uint32_t)i;
    parent[right] = (uint32_t)i;
}

__device__ __forceinline__ double box_sa(float lx, float ly, float lz, float hx, float hy, float hz) {
    const double dx = (double)hx - (double)lx, dy = (double)hy - (double)ly, dz = (double)hz - (double)lz;
    return 2.0 * ((dx * dy + dy * dz) + dz * dx);
}

__global__ __launch_bounds__(256) void k_leaves(const float* __restrict__ tris, uint32_t n,
                                                const uint32_t* __restrict__ leaf_prim, Tri* __restrict__ out,
                                                float* __restrict__ boxes, double* __restrict__ had) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const uint32_t prim = leaf_prim[j];
    const float* t = tris + 9 * (size_t)prim;
    const float v0x = t[0], v0y = t[1], v0z = t[2];
    const float e1x = t[3] - v0x, e1y = t[4] - v0y, e1z = t[5] - v0z;
    const float e2x = t[6] - v0x, e2y = t[7] - v0y, e2z = t[8] - v0z;
    Tri tr;
    tr.p = make_float4(v0x, v0y, v0z, e1x);
    tr.q = make_float4(e1y, e1z, e2x, e2y);
    tr.r = make_float4(e2z, __uint_as_float(prim), 0.0f, 0.0f);
    out[j] = tr;
    float b[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b[a] = fminf(fminf(t[a], t[3 + a]), t[6 + a]);
        b[3 + a] = fmaxf(fmaxf(t[a], t[3 + a]), t[6 + a]);
    }
    const size_t id = (size_t)(n - 1) + j;
#pragma unroll
    for (int a = 0; a < 6; ++a) boxes[6 * id + a] = b[a];
    had[id] = 1.0 * box_sa(b[0], b[1], b[2], b[3], b[4], b[5]);
}

// Loads of values another thread published before its arrival on the counter; agent
// scope so that a copy cached for another XCD is never used.
__device__ __forceinline__ float load_agent(const float* p) {
    return __uint_as_float(__hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ double load_agent(const double* p) {
    return __longlong_as_double(
        (long long)__hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void store_agent(float* p, float v) {
    __hip_atomic_store((uint32_t*)p, __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(double* p, double v) {
    __hip_atomic_store((uint64_t*)p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bottom-up pass.  kBoxes: union boxes and fill nodes; always: HAD with 'lambda'.
template <bool kBoxes>
__global__ __launch_bounds__(256) void k_refit(uint32_t n, const uint32_t* __restrict__ child,
                                               const uint32_t* __restrict__ parent, uint32_t* flags,
                                               float* boxes, double* had, Node* __restrict__ nodes, double lambda) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const uint32_t n_int = n - 1;
    uint32_t node = parent[n_int + j];
    // Boxes and HAD values that other threads read are stored and loaded with device-scope
    // atomic accesses (coherent across the XCDs' L2 caches); a thread counts its arrival at the
    // parent only once its stores have completed.  Device-scope fences instead would write back
    // and invalidate the L2 at every step.
    while (node != kNone) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);                    // this child's results are stored
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (atomicAdd(&flags[node], 1u) == 0) return;     // sibling not done: it continues
        __atomic_signal_fence(__ATOMIC_SEQ_CST);          // the sibling's results are read after
        const uint32_t c0 = child[2 * node], c1 = child[2 * node + 1];
        const float* b0 = boxes + 6 * (size_t)c0;
        const float* b1 = boxes + 6 * (size_t)c1;
        float b[6];
        if (kBoxes) {
            float x0[6], x1[6];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                x0[a] = load_agent(b0 + a);
                x1[a] = load_agent(b1 + a);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                b[a] = fminf(x0[a], x1[a]);
                b[3 + a] = fmaxf(x0[3 + a], x1[3 + a]);
            }
#pragma unroll
            for (int a = 0; a < 6; ++a) store_agent(boxes + 6 * (size_t)node + a, b[a]);
            Node nd;
            nd.a = make_float4(x0[0], x0[1], x0[2], x0[3]);
            nd.b = make_float4(x0[4], x0[5], x1[0], x1[1]);
            nd.c = make_float4(x1[2], x1[3], x1[4], x1[5]);
            nd.d = make_uint4(c0, c1, 0u, 0u);
            nodes[node] = nd;
        } else {
#pragma unroll
            for (int a = 0; a < 6; ++a) b[a] = boxes[6 * (size_t)node + a];
        }
        const double h0 = load_agent(had + c0);
        const double h1 = load_agent(had + c1);
        store_agent(had + node, (h0 + h1) + lambda * box_sa(b[0], b[1], b[2], b[3], b[4], b[5]));
        node = parent[node];
    }
}

// 4-wide nodes, one level of the wide tree per launch: a frontier node starts from its two
// children and, while it has fewer than four and one of them is internal, replaces the
// internal child of largest surface area by that child's two children (greedy SAH-style
// collapse).  Internal members become the next level's frontier.  Wide nodes are stored
// compactly in level order: frontier entry i of this level is wide node level_base + i, and
// the next level starts right after this one, each node's internal members taking consecutive
// places there (one reservation per node), so siblings sit next to each other in memory.
__global__ __launch_bounds__(256) void k_wide_level(const uint32_t* __restrict__ frontier, uint32_t count,
                                                    uint32_t level_base, uint32_t n_int,
                                                    const uint32_t* __restrict__ child,
                                                    const float* __restrict__ boxes, Node4* __restrict__ wide,
                                                    uint32_t* __restrict__ next, uint32_t* __restrict__ next_count) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const uint32_t next_base = level_base + count;
    const uint32_t x = frontier[i];
    uint32_t list[4] = {child[2 * (size_t)x], child[2 * (size_t)x + 1], kNone, kNone};
    uint32_t m = 2;
    while (m < 4) {
        int best = -1;
        float best_sa = -1.0f;
        for (uint32_t j = 0; j < m; ++j) {
            const uint32_t u = list[j];
            if (u >= n_int) continue;
            const float* bx = boxes + 6 * (size_t)u;
            const float ex = bx[3] - bx[0], ey = bx[4] - bx[1], ez = bx[5] - bx[2];
            const float sa = (ex * ey + ey * ez) + ez * ex;
            if (sa > best_sa) {
                best_sa = sa;
                best = (int)j;
            }
        }
        if (best < 0) break;
        const uint32_t u = list[best];
        for (uint32_t j = m; j > (uint32_t)best + 1; --j) list[j] = list[j - 1];
        list[best] = child[2 * (size_t)u];
        list[best + 1] = child[2 * (size_t)u + 1];
        ++m;
    }
    uint32_t n_in = 0;
    for (uint32_t j = 0; j < m; ++j) n_in += list[j] < n_int ? 1u : 0u;
    uint32_t at = n_in ? atomicAdd(next_count, n_in) : 0u;
    float lo[3][4], hi[3][4];
    uint32_t ref[4];
    for (uint32_t j = 0; j < 4; ++j) {
        if (j < m) {
            const uint32_t u = list[j];
            const float* bx = boxes + 6 * (size_t)u;
            for (int a = 0; a < 3; ++a) {
                lo[a][j] = bx[a];
                hi[a][j] = bx[3 + a];
            }
            if (u >= n_int) {
                ref[j] = kWideLeaf | (u - n_int);
            } else {
                ref[j] = next_base + at;
                next[at++] = u;
            }
        } else {
            // inverted box: rejected by the sign-selected child test without a check of ref
            for (int a = 0; a < 3; ++a) {
                lo[a][j] = INFINITY;
                hi[a][j] = -INFINITY;
            }
            ref[j] = kWideEmpty;
        }
    }
    Node4 w;
    w.lox = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
    w.loy = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
    w.loz = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
    w.hix = make_float4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
    w.hiy = make_float4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
    w.hiz = make_float4(hi[2][0], hi[2][1], hi[2][2], hi[2][3]);
    w.ref = make_uint4(ref[0], ref[1], ref[2], ref[3]);
    w.pad = make_uint4(0, 0, 0, 0);
    wide[level_base + i] = w;
}

// Quantised copy of wide node i (the Node4Q layout).  Axis a: corner p = the least lower plane
// of the slots, scale s = the least power of two (at least 2^-126) whose step 255 decodes to at
// least the node's upper plane; each slot's lower step is the largest decoding to at most its
// lower plane, its upper step the smallest decoding to at least its upper plane, both found by
// decoding exactly as the traversal does (fmaf(q, s, p)).  A node with a non-finite corner or
// upper plane counts into *bad and keeps zero steps (the library then does not offer the
// quantised traversal for this BVH).
__device__ __forceinline__ float qdec(uint32_t q, float s, float p) { return fmaf((float)q, s, p); }

__global__ __launch_bounds__(256) void k_quantize_wide(const Node4* __restrict__ wide, uint32_t count,
                                                       Node4Q* __restrict__ qn, uint32_t* __restrict__ bad) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const Node4 w = wide[i];
    const uint32_t refs[4] = {w.ref.x, w.ref.y, w.ref.z, w.ref.w};
    const float lo[3][4] = {{w.lox.x, w.lox.y, w.lox.z, w.lox.w},
                            {w.loy.x, w.loy.y, w.loy.z, w.loy.w},
                            {w.loz.x, w.loz.y, w.loz.z, w.loz.w}};
    const float hi[3][4] = {{w.hix.x, w.hix.y, w.hix.z, w.hix.w},
                            {w.hiy.x, w.hiy.y, w.hiy.z, w.hiy.w},
                            {w.hiz.x, w.hiz.y, w.hiz.z, w.hiz.w}};
    float p[3], sc[3];
    uint32_t lw[3] = {0, 0, 0}, hw[3] = {0, 0, 0};
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        float c = INFINITY, top = -INFINITY;
        for (int j = 0; j < 4; ++j) {
            if (refs[j] == kWideEmpty) continue;
            c = fminf(c, lo[a][j]);
            top = fmaxf(top, hi[a][j]);
        }
        p[a] = c;
        sc[a] = 0.0f;
        if (!(fabsf(c) < INFINITY) || !(fabsf(top) < INFINITY) || !(top >= c)) {
            ok = false;
            continue;
        }
        // the least power of two whose 255 steps reach top (start from the extent's estimate)
        const double need = ((double)top - (double)c) / 255.0;
        int e = need > 0.0 ? (int)ceil(log2(need)) : -126;
        if (e < -126) e = -126;
        float s = ldexpf(1.0f, e);
        while (e > -126 && qdec(255u, ldexpf(1.0f, e - 1), c) >= top) s = ldexpf(1.0f, --e);
        while (qdec(255u, s, c) < top && e < 127) s = ldexpf(1.0f, ++e);
        if (!(qdec(255u, s, c) >= top) || !(fabsf(qdec(255u, s, c)) < INFINITY)) {
            ok = false;
            continue;
        }
        sc[a] = s;
        for (int j = 0; j < 4; ++j) {
            uint32_t ql = 255u, qh = 0u;   // empty slot: inverted
            if (refs[j] != kWideEmpty) {
                // lower: the largest step decoding to <= lo (step 0 decodes to c <= lo)
                const double fl = floor(((double)lo[a][j] - (double)c) / (double)s);
                ql = fl <= 0.0 ? 0u : (fl >= 255.0 ? 255u : (uint32_t)fl);
                while (ql > 0u && qdec(ql, s, c) > lo[a][j]) --ql;
                while (ql < 255u && qdec(ql + 1u, s, c) <= lo[a][j]) ++ql;
                // upper: the smallest step decoding to >= hi (step 255 decodes to >= top >= hi)
                const double fh = ceil(((double)hi[a][j] - (double)c) / (double)s);
                qh = fh <= 0.0 ? 0u : (fh >= 255.0 ? 255u : (uint32_t)fh);
                while (qh < 255u && qdec(qh, s, c) < hi[a][j]) ++qh;
                while (qh > 0u && qdec(qh - 1u, s, c) >= hi[a][j]) --qh;
            }
            lw[a] |= ql << (8 * j);
            hw[a] |= qh << (8 * j);
        }
    }
    if (!ok) atomicAdd(bad, 1u);
    Node4Q q;
    q.a = make_float4(p[0], p[1], p[2], sc[0]);
    q.b = make_float4(sc[1], sc[2], __uint_as_float(lw[0]), __uint_as_float(hw[0]));
    q.c = make_uint4(lw[1], hw[1], lw[2], hw[2]);
    q.ref = w.ref;
    qn[i] = q;
}

__global__ void k_fill(uint32_t* p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_leaf_had(const float* __restrict__ boxes, uint32_t n, double* __restrict__ had) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const size_t id = (size_t)(n - 1) + j;
    const float* b = boxes + 6 * id;
    had[id] = 1.0 * box_sa(b[0], b[1], b[2], b[3], b[4], b[5]);
}

template <typename T>
hcc_status dalloc(const Allocator& A, hipStream_t s, T** p, size_t count, size_t& bytes) {
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    *p = (T*)A.get(b, s);
    if (!*p) return fail(HCC_ERR_OOM, "device allocation failed in hcc_build_bvh");
    bytes += b;
    return HCC_OK;
}

inline unsigned blocks_for(size_t n, unsigned per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void free_bvh(hcc_bvh_s* b) {
    if (!b) return;
    const Allocator& A = b->alloc;
    A.put(b->nodes, nullptr);
    A.put(b->wnodes, nullptr);
    A.put(b->qnodes, nullptr);
    A.put(b->tris, nullptr);
    A.put(b->boxes, nullptr);
    A.put(b->had, nullptr);
    A.put(b->child, nullptr);
    A.put(b->leaf_prim, nullptr);
    A.put(b->parent, nullptr);
    b->magic = 0;
    delete b;
}

hcc_status build_bvh(const float* d_tris, uint32_t n, hipStream_t stream, hcc_bvh_s** out) {
    hcc_bvh_s* b = new hcc_bvh_s();
    b->alloc = current_allocator();
    const Allocator A = b->alloc;
    b->n = n;
    b->n_int = n - 1;
    (void)hipGetDevice(&b->device);
    size_t bytes = 0;
    const size_t nn = 2 * (size_t)n - 1;
    hcc_status st;
#define TRY(x)                      \
    do {                            \
        st = (x);                   \
        if (st != HCC_OK) {         \
            free_bvh(b);            \
            return st;              \
        }                           \
    } while (0)
    TRY(dalloc(A, stream, &b->nodes, b->n_int, bytes));
    TRY(dalloc(A, stream, &b->wnodes, b->n_int, bytes));
    TRY(dalloc(A, stream, &b->tris, n, bytes));
    TRY(dalloc(A, stream, &b->boxes, nn * 6, bytes));
    TRY(dalloc(A, stream, &b->had, nn, bytes));
    TRY(dalloc(A, stream, &b->child, 2 * (size_t)b->n_int, bytes));
    TRY(dalloc(A, stream, &b->leaf_prim, n, bytes));
    TRY(dalloc(A, stream, &b->parent, nn, bytes));
    b->bytes = bytes;

    // temporaries
    size_t tmp_bytes = 0;
    const unsigned nb_bounds = std::min<unsigned>(1024u, std::max(1u, blocks_for((size_t)n * 3)));
    float* partial = nullptr;
    float* d_box = nullptr;
    uint32_t* codes = nullptr;
    uint32_t* codes_sorted = nullptr;
    uint32_t* flags = nullptr;
    void* ws = nullptr;
    const size_t ws_bytes = sort_workspace_bytes(n, 30);
    auto cleanup = [&]() {
        A.put(partial, stream);
        A.put(d_box, stream);
        A.put(codes, stream);
        A.put(codes_sorted, stream);
        A.put(flags, stream);
        A.put(ws, stream);
    };
#define TRYT(x)                     \
    do {                            \
        st = (x);                   \
        if (st != HCC_OK) {         \
            cleanup();              \
            free_bvh(b);            \
            return st;              \
        }                           \
    } while (0)
    TRYT(dalloc(A, stream, &partial, (size_t)nb_bounds * 6, tmp_bytes));
    TRYT(dalloc(A, stream, &d_box, 6, tmp_bytes));
    TRYT(dalloc(A, stream, &codes, n, tmp_bytes));
    TRYT(dalloc(A, stream, &codes_sorted, n, tmp_bytes));
    TRYT(dalloc(A, stream, &flags, std::max<size_t>(b->n_int, 1), tmp_bytes));
    if ((ws = A.get(ws_bytes, stream)) == nullptr) {
        cleanup();
        free_bvh(b);
        return fail(HCC_ERR_OOM, "hipMalloc failed in hcc_build_bvh (sort workspace)");
    }

    k_bounds_partial<<<nb_bounds, 256, 0, stream>>>(d_tris, n, partial);
    k_bounds_final<<<1, 256, 0, stream>>>(partial, nb_bounds, d_box);
    k_morton<<<blocks_for(n), 256, 0, stream>>>(d_tris, n, d_box, codes);
    TRYT(radix_sort(codes, 30, n, b->leaf_prim, codes_sorted, nullptr, ws, ws_bytes, stream));
    k_fill<<<blocks_for(nn), 256, 0, stream>>>(b->parent, nn, kNone);
    if (b->n_int > 0) {
        k_karras<<<blocks_for(b->n_int), 256, 0, stream>>>(codes_sorted, n, b->child, b->parent);
        k_fill<<<blocks_for(b->n_int), 256, 0, stream>>>(flags, b->n_int, 0u);
    }
    k_leaves<<<blocks_for(n), 256, 0, stream>>>(d_tris, n, b->leaf_prim, b->tris, b->boxes, b->had);
    if (b->n_int > 0)
        k_refit<true><<<blocks_for(n), 256, 0, stream>>>(n, b->child, b->parent, flags, b->boxes, b->had, b->nodes,
                                                        0.125);
    hipError_t e = hipGetLastError();
    // 4-wide nodes, level by level from the root (codes / codes_sorted are free again and serve
    // as the frontier ping-pong buffers, flags[0] as the next level's counter)
    if (e == hipSuccess && b->n_int > 0) {
        uint32_t* cur = codes;
        uint32_t* nxt = codes_sorted;
        uint32_t count = 1, level_base = 0;
        k_fill<<<1, 256, 0, stream>>>(cur, 1, 0u);
        for (int level = 0; count > 0 && level < 256 && e == hipSuccess; ++level) {
            k_fill<<<1, 256, 0, stream>>>(flags, 1, 0u);
            k_wide_level<<<blocks_for(count), 256, 0, stream>>>(cur, count, level_base, b->n_int, b->child, b->boxes,
                                                                b->wnodes, nxt, flags);
            level_base += count;
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(&count, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            std::swap(cur, nxt);
        }
        if (e == hipSuccess && count > 0) {   // deeper than any radix tree over 62-bit keys can be
            cleanup();
            free_bvh(b);
            return fail(HCC_ERR_DEVICE, "hcc_build_bvh: 4-wide collapse did not finish");
        }
        b->n_wide = level_base;
        // quantised copy of the wide nodes (flags[0] counts nodes that cannot be quantised)
        if (e == hipSuccess) {
            const hcc_status qs = dalloc(A, stream, &b->qnodes, b->n_wide, b->bytes);
            if (qs != HCC_OK) {
                cleanup();
                free_bvh(b);
                return qs;
            }
            uint32_t nbad = 1;
            k_fill<<<1, 256, 0, stream>>>(flags, 1, 0u);
            k_quantize_wide<<<blocks_for(b->n_wide), 256, 0, stream>>>(b->wnodes, b->n_wide, b->qnodes, flags);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(&nbad, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            b->quant_ok = e == hipSuccess && nbad == 0;
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(b->scene_box, d_box, 6 * sizeof(float), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    cleanup();
    if (e != hipSuccess) {
        free_bvh(b);
        return hip_fail(e, "hcc_build_bvh");
    }
    b->had_lambda = 0.125;
    *out = b;
    return HCC_OK;
#undef TRY
#undef TRYT
}

// Recompute HAD for another lambda (boxes unchanged).  Blocking.
hcc_status recompute_had(hcc_bvh_s* b, double lambda, hipStream_t stream) {
    if (b->n == 1) {
        b->had_lambda = lambda;   // a single leaf: HAD = TC * SA regardless of lambda
        return HCC_OK;
    }
    uint32_t* flags = nullptr;
    if ((flags = (uint32_t*)b->alloc.get(sizeof(uint32_t) * b->n_int, stream)) == nullptr)
        return fail(HCC_ERR_OOM, "device allocation failed in hcc_select_cut");
    k_fill<<<blocks_for(b->n_int), 256, 0, stream>>>(flags, b->n_int, 0u);
    k_leaf_had<<<blocks_for(b->n), 256, 0, stream>>>(b->boxes, b->n, b->had);
    k_refit<false><<<blocks_for(b->n), 256, 0, stream>>>(b->n, b->child, b->parent, flags, b->boxes, b->had,
                                                         b->nodes, lambda);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    b->alloc.put(flags, stream);
    if (e != hipSuccess) return hip_fail(e, "hcc_select_cut (HAD)");
    b->had_lambda = lambda;
    return HCC_OK;
}

}  // namespace hcc
