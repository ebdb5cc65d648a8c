// Internal declarations of the gfx950 library: device data layouts, shared device
// helpers, error plumbing.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hcc.h"

namespace hcc {

// ------------------------------------------------------------------------- layouts

// BVH2 node, 64 bytes = one aligned fetch.  The node stores the boxes of its two
// children so that one load gives everything a traversal step tests.
//   a = (lo0.x, lo0.y, lo0.z, hi0.x)   b = (hi0.y, hi0.z, lo1.x, lo1.y)
//   c = (lo1.z, hi1.x, hi1.y, hi1.z)   d = (child0, child1, 0, 0) as uint bits
// child ids are unified: < n_internal -> internal node, else leaf (id - n_internal).
struct alignas(64) Node {
    float4 a, b, c;
    uint4 d;
};

// 4-wide node for traversal, 128 bytes (two cache lines): the BVH2 collapsed top down.  The
// wide node of BVH2 node X holds up to four BVH2 descendants of X that together cover its
// subtree (X's children, internal ones replaced by their children, largest surface area first).
// Slot j: box (lox[j], loy[j], loz[j]) - (hix[j], hiy[j], hiz[j]); ref[j] = index of the wide
// node of an internal member (wide nodes are stored in level order, the root at 0),
// kWideLeaf | triangle slot, or kWideEmpty.
struct alignas(64) Node4 {
    float4 lox, loy, loz, hix, hiy, hiz;
    uint4 ref;
    uint4 pad;
};
constexpr uint32_t kWideLeaf = 0x80000000u;
constexpr uint32_t kWideEmpty = 0xFFFFFFFFu;

// Quantised 4-wide node, 64 bytes (one cache line, four 16-byte loads instead of the seven a
// Node4 step reads): the slot boxes of the Node4 with the same index as 8-bit steps from the
// node's corner.  On axis a, step q decodes to the plane fmaf(q, s_a, p_a) (q * s_a is exact,
// one rounding), with p the corner (the least lower plane over the slots) and s_a a power of
// two for which step 255 reaches the node's upper plane.  A slot's lower steps are the largest
// that decode to at most its lower planes and its upper steps the smallest that decode to at
// least its upper planes, so every decoded box contains its slot's box and a ray that meets a
// slot's box meets its decoded box.  An empty slot has lower steps 255, upper steps 0 and ref
// kWideEmpty.
//   a = (p.x, p.y, p.z, s.x)   b = (s.y, s.z, lower x steps, upper x steps)
//   c = (lower y, upper y, lower z, upper z steps)   ref = the Node4's refs
// Each steps word holds slot j in byte j.
struct alignas(64) Node4Q {
    float4 a, b;
    uint4 c;
    uint4 ref;
};

__device__ __forceinline__ float qplane(uint32_t steps, int j, float s, float p) {
    return fmaf((float)((steps >> (8 * j)) & 255u), s, p);
}
constexpr int kWideStack = 192;   // <= 3 pushes per wide level, at most 63 levels (BVH2 depth over 62-bit keys)

// Triangle in Morton order, 48 bytes: v0, e1 = v1 - v0, e2 = v2 - v0 (float32,
// rounded exactly as the Moller-Trumbore test computes them), original index.
//   p = (v0.x, v0.y, v0.z, e1.x)  q = (e1.y, e1.z, e2.x, e2.y)  r = (e2.z, prim bits, 0, 0)
struct alignas(16) Tri {
    float4 p, q, r;
};

// Cut box in LDS / global: lo.xyz, pad, hi.xyz, pad (32 bytes, two 16-byte loads).
struct alignas(16) CutBox {
    float4 lo, hi;
};

constexpr uint32_t kMissPrim = 0xFFFFFFFFu;
constexpr int kStackDepth = 64;   // >= depth of a radix tree over 62-bit keys

// ------------------------------------------------------------------------- device math
// Slab test of a ray against a box over [tmin, tmax] (IEEE 1/d precomputed, minNum /
// maxNum, far distance scaled by 1 + 3*2^-23).  Compiled without FMA contraction so
// it rounds exactly like the reference definition.
__device__ __forceinline__ bool slab(float ox, float oy, float oz, float ix, float iy, float iz, float tmin,
                                     float tmax, float lx, float ly, float lz, float hx, float hy, float hz,
                                     float& tnear) {
    float t0x = (lx - ox) * ix, t1x = (hx - ox) * ix;
    float t0y = (ly - oy) * iy, t1y = (hy - oy) * iy;
    float t0z = (lz - oz) * iz, t1z = (hz - oz) * iz;
    float nx = fminf(t0x, t1x), fx = fmaxf(t0x, t1x);
    float ny = fminf(t0y, t1y), fy = fmaxf(t0y, t1y);
    float nz = fminf(t0z, t1z), fz = fmaxf(t0z, t1z);
    tnear = fmaxf(fmaxf(fmaxf(nx, ny), nz), tmin);
    // scaling after the minimum equals scaling each axis first: rounding of a product by a
    // positive constant is monotone, and a NaN axis is dropped by fminf either way
    float tfar = fminf(fminf(fminf(fx, fy), fz) * 0x1.000006p+0f, tmax);
    return tnear <= tfar;
}

// Child-box test of a 4-wide node.  For a ray with a finite origin and an inverse direction that
// is finite and nonzero on every axis ("fast" ray), the entry plane of axis a is lo_a when 1/d_a
// has its sign bit clear and hi_a otherwise, so (entry - o_a) * inv_a is exactly min(t0, t1) of
// the slab test above, and the exit plane gives max(t0, t1): the slab's per-axis min/max pairs
// are replaced by choosing which plane to fetch.  Entry planes sit at byte offsets x: 0 or 48,
// y: 16 or 64, z: 32 or 80 inside the node; the exit plane of an axis is at the entry offset XOR
// 48 / 80 / 112.  Empty slots hold the inverted box (+inf, -inf): for a fast ray (+-inf - o) * inv
// is an infinity, never NaN, so such a slot gets entry +inf and exit -inf and is rejected without
// looking at ref.  Any other ray needs the slab test itself (where 0 * inf can make an axis NaN)
// and the check of ref.
struct WideRay {
    uint32_t ex, ey, ez;   // entry-plane byte offsets within a node
    bool fast;
};

__device__ __forceinline__ bool finite_nonzero(float x) { return fabsf(x) < INFINITY && x != 0.0f; }

__device__ __forceinline__ WideRay wide_ray(float ox, float oy, float oz, float ix, float iy, float iz) {
    WideRay w;
    w.fast = fabsf(ox) < INFINITY && fabsf(oy) < INFINITY && fabsf(oz) < INFINITY && finite_nonzero(ix) &&
             finite_nonzero(iy) && finite_nonzero(iz);
    w.ex = signbit(ix) ? 48u : 0u;
    w.ey = signbit(iy) ? 64u : 16u;
    w.ez = signbit(iz) ? 80u : 32u;
    return w;
}

// Byte offsets into the node array are 32-bit on the selected-plane path.
constexpr uint32_t kWideFastNodes = 0xFFFFFFFFu / (uint32_t)sizeof(Node4);

// The four child tests of node `node` for the calling lane: kFast, the selected-plane form (only
// for fast rays, and node arrays whose byte offsets fit 32 bits); else the slab test.
template <bool kFast>
__device__ __forceinline__ void wide_test(const Node4* __restrict__ wn, uint32_t node, const WideRay& w, float ox,
                                          float oy, float oz, float ix, float iy, float iz, float tmin, float lim,
                                          uint4& ref, bool (&h)[4], float (&t)[4]) {
    if constexpr (kFast) {
        const char* base = reinterpret_cast<const char*>(wn);
        const uint32_t at = node * (uint32_t)sizeof(Node4);
        const float4 nx = *reinterpret_cast<const float4*>(base + (at + w.ex));
        const float4 fx = *reinterpret_cast<const float4*>(base + (at + (w.ex ^ 48u)));
        const float4 ny = *reinterpret_cast<const float4*>(base + (at + w.ey));
        const float4 fy = *reinterpret_cast<const float4*>(base + (at + (w.ey ^ 80u)));
        const float4 nz = *reinterpret_cast<const float4*>(base + (at + w.ez));
        const float4 fz = *reinterpret_cast<const float4*>(base + (at + (w.ez ^ 112u)));
        ref = *reinterpret_cast<const uint4*>(base + (at + 96u));
        const float enx[4] = {nx.x, nx.y, nx.z, nx.w}, eny[4] = {ny.x, ny.y, ny.z, ny.w};
        const float enz[4] = {nz.x, nz.y, nz.z, nz.w}, exx[4] = {fx.x, fx.y, fx.z, fx.w};
        const float exy[4] = {fy.x, fy.y, fy.z, fy.w}, exz[4] = {fz.x, fz.y, fz.z, fz.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float tn = fmaxf(fmaxf(fmaxf((enx[j] - ox) * ix, (eny[j] - oy) * iy), (enz[j] - oz) * iz), tmin);
            const float tf = fminf(fminf(fminf((exx[j] - ox) * ix, (exy[j] - oy) * iy), (exz[j] - oz) * iz) *
                                       0x1.000006p+0f, lim);
            t[j] = tn;
            h[j] = tn <= tf;
        }
    } else {
        const Node4 nd = wn[node];
        ref = nd.ref;
        h[0] = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.lox.x, nd.loy.x, nd.loz.x, nd.hix.x, nd.hiy.x, nd.hiz.x,
                    t[0]) && ref.x != kWideEmpty;
        h[1] = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.lox.y, nd.loy.y, nd.loz.y, nd.hix.y, nd.hiy.y, nd.hiz.y,
                    t[1]) && ref.y != kWideEmpty;
        h[2] = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.lox.z, nd.loy.z, nd.loz.z, nd.hix.z, nd.hiy.z, nd.hiz.z,
                    t[2]) && ref.z != kWideEmpty;
        h[3] = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.lox.w, nd.loy.w, nd.loz.w, nd.hix.w, nd.hiy.w, nd.hiz.w,
                    t[3]) && ref.w != kWideEmpty;
    }
}

// The four child tests of quantised node `node`: the tests of wide_test on the decoded boxes
// (kFast: the selected-plane form, for fast rays), plus the check of ref for empty slots, whose
// decoded box is inverted but not by infinities.
template <bool kFast>
__device__ __forceinline__ void wide_test_q(const Node4Q* __restrict__ qn, uint32_t node, const WideRay& w, float ox,
                                            float oy, float oz, float ix, float iy, float iz, float tmin, float lim,
                                            uint4& ref, bool (&h)[4], float (&t)[4]) {
    const Node4Q nd = qn[node];
    ref = nd.ref;
    const float px = nd.a.x, py = nd.a.y, pz = nd.a.z, sx = nd.a.w, sy = nd.b.x, sz = nd.b.y;
    const uint32_t lox = __float_as_uint(nd.b.z), hix = __float_as_uint(nd.b.w);
    const uint32_t loy = nd.c.x, hiy = nd.c.y, loz = nd.c.z, hiz = nd.c.w;
    const uint32_t refs[4] = {ref.x, ref.y, ref.z, ref.w};
    if constexpr (kFast) {
        // entry steps: the lower ones where 1/d has its sign bit clear, else the upper ones
        const uint32_t enx = w.ex ? hix : lox, exx = w.ex ? lox : hix;
        const uint32_t eny = w.ey != 16u ? hiy : loy, exy = w.ey != 16u ? loy : hiy;
        const uint32_t enz = w.ez != 32u ? hiz : loz, exz = w.ez != 32u ? loz : hiz;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float tn = fmaxf(fmaxf(fmaxf((qplane(enx, j, sx, px) - ox) * ix, (qplane(eny, j, sy, py) - oy) * iy),
                                         (qplane(enz, j, sz, pz) - oz) * iz),
                                   tmin);
            const float tf = fminf(fminf(fminf((qplane(exx, j, sx, px) - ox) * ix, (qplane(exy, j, sy, py) - oy) * iy),
                                         (qplane(exz, j, sz, pz) - oz) * iz) *
                                       0x1.000006p+0f,
                                   lim);
            t[j] = tn;
            h[j] = tn <= tf && refs[j] != kWideEmpty;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            h[j] = slab(ox, oy, oz, ix, iy, iz, tmin, lim, qplane(lox, j, sx, px), qplane(loy, j, sy, py),
                        qplane(loz, j, sz, pz), qplane(hix, j, sx, px), qplane(hiy, j, sy, py), qplane(hiz, j, sz, pz),
                        t[j]) &&
                   refs[j] != kWideEmpty;
    }
}

// Moller-Trumbore, double sided, float32, fixed operation order, no FMA contraction.
__device__ __forceinline__ bool tri_test(const Tri& tr, float ox, float oy, float oz, float dx, float dy, float dz,
                                         float tmin, float tmax, float& t, float& u, float& v) {
    const float v0x = tr.p.x, v0y = tr.p.y, v0z = tr.p.z;
    const float e1x = tr.p.w, e1y = tr.q.x, e1z = tr.q.y;
    const float e2x = tr.q.z, e2y = tr.q.w, e2z = tr.r.x;
    const float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const float det = (e1x * px + e1y * py) + e1z * pz;
    // s before the first exit, so that all of the triangle is fetched in one round trip
    const float sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
    if (det == 0.0f) return false;
    const float inv = 1.0f / det;
    u = ((sx * px + sy * py) + sz * pz) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    v = ((dx * qx + dy * qy) + dz * qz) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    t = ((e2x * qx + e2y * qy) + e2z * qz) * inv;
    return t > tmin && t < tmax;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Host-side tracing: every public entry point opens a named roctx range for its host call
// (the queued kernels show in a kernel trace under it), so `rocprofv3 --marker-trace` shows
// which library call issued which work.  Without a profiler attached the calls cost a few
// nanoseconds.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

// Host-side error helpers ---------------------------------------------------------------
void set_error(const std::string& msg);
hcc_status fail(hcc_status st, const std::string& msg);

// Device memory the library owns: hipMalloc / hipFree unless hcc_set_allocator installed
// hooks.  Objects keep the allocator they were created with and free through it.
struct Allocator {
    hcc_alloc_fn alloc = nullptr;
    hcc_free_fn release = nullptr;
    void* ctx = nullptr;
    void* get(size_t bytes, hipStream_t s) const {
        if (alloc) return alloc(bytes, (hcc_stream)s, ctx);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void* p, hipStream_t s) const {
        if (!p) return;
        if (release) release(p, (hcc_stream)s, ctx);
        else (void)hipFree(p);
    }
};
Allocator current_allocator();
hcc_status hip_fail(hipError_t e, const char* what);

#define HCC_HIP(call)                                                  \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return ::hcc::hip_fail(_e, #call);       \
    } while (0)

// Radix sort used by the BVH build and by hcc_sort.
size_t sort_workspace_bytes(uint32_t n, uint32_t key_bits);
hcc_status radix_sort(const void* d_keys, uint32_t key_bits, uint32_t n, uint32_t* d_perm, void* d_sorted_keys,
                      const uint32_t* d_vals_in, void* d_ws, size_t ws_bytes, hipStream_t stream);
size_t sort_static_bytes();
hcc_status radix_sort_static(const void* d_keys, uint32_t key_bits, uint32_t n, uint32_t* d_perm,
                             void* d_sorted_keys, hipStream_t stream);
hcc_status radix_sort_ex(const void* d_keys, uint32_t key_bits, uint32_t skip, uint32_t tile, uint32_t n,
                         uint32_t* d_perm, void* d_sorted_keys, void* d_ws, size_t ws_bytes, hipStream_t stream);

// XCD-aware block index: the hardware deals workgroups to the 8 XCDs round robin;
// this maps them so that each XCD runs a contiguous range of logical blocks.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t g) {
    uint32_t per = g >> 3, rem = g & 7u;
    uint32_t x = b & 7u, k = b >> 3;
    return x * per + (x < rem ? x : rem) + k;
}

}  // namespace hcc

// Library-owned handle layouts.
struct hcc_bvh_s {
    uint32_t n = 0;                 // triangles
    uint32_t n_int = 0;             // internal nodes = n - 1
    hcc::Node* nodes = nullptr;     // n_int
    hcc::Node4* wnodes = nullptr;   // 4-wide nodes in level order from the root (at most n_int)
    hcc::Node4Q* qnodes = nullptr;  // the same nodes quantised (n_wide), when quant_ok
    uint32_t n_wide = 0;            // 4-wide nodes
    bool quant_ok = false;          // every wide node's corner and extent are finite
    hcc::Tri* tris = nullptr;       // n (Morton order)
    float* boxes = nullptr;         // (2n-1) x 6
    double* had = nullptr;          // 2n-1
    uint32_t* child = nullptr;      // n_int x 2 (unified ids)
    uint32_t* leaf_prim = nullptr;  // n
    uint32_t* parent = nullptr;     // 2n-1 (root: 0xFFFFFFFF)
    float scene_box[6] = {0, 0, 0, 0, 0, 0};
    double had_lambda = 0.125;
    size_t bytes = 0;
    int device = 0;
    // host mirror for the cut search
    std::vector<uint32_t> h_child;
    std::vector<double> h_had;
    std::vector<uint32_t> h_leaves; // leaves below each node (two-level cut search)
    double h_had_lambda = -1.0;
    hcc::Allocator alloc;           // the device memory above came from here
    uint64_t magic = 0x6863636276680001ull;
};

struct hcc_cut_s {
    const hcc_bvh_s* bvh = nullptr;
    uint32_t kind = 0;              // 0 cut (Alg. 2), 1 two-level cut (Alg. 3), 2 regular grid
    uint32_t c_eff = 0;             // cut nodes / top-level nodes / grid cells
    uint32_t low = 0;               // two-level cut: low-level nodes per top node
    uint32_t top_req = 0;           // two-level cut: requested top-level size
    std::vector<uint32_t> ids;      // c_eff (grid: 0xFFFFFFFF)
    std::vector<double> had;
    std::vector<float> boxes;       // c_eff x 6
    std::vector<uint32_t> low_ids;  // c_eff x low
    std::vector<float> low_boxes;   // c_eff x low x 6
    hcc::CutBox* d_boxes = nullptr; // c_eff boxes, then (two-level) c_eff x low boxes
    hcc::Allocator alloc;           // d_boxes came from here
    uint64_t magic = 0x6863636375740001ull;
};
