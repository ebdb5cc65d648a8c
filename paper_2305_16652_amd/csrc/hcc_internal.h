// Internal declarations of the gfx950 library: device data layouts, shared device
// helpers, error plumbing.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
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
// Slot j: box (lox[j], loy[j], loz[j]) - (hix[j], hiy[j], hiz[j]); ref[j] = BVH2 id of an internal
// member (whose wide node is stored at that same index), kWideLeaf | triangle slot, or kWideEmpty.
struct alignas(64) Node4 {
    float4 lox, loy, loz, hix, hiy, hiz;
    uint4 ref;
    uint4 pad;
};
constexpr uint32_t kWideLeaf = 0x80000000u;
constexpr uint32_t kWideEmpty = 0xFFFFFFFFu;
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

// Moller-Trumbore, double sided, float32, fixed operation order, no FMA contraction.
__device__ __forceinline__ bool tri_test(const Tri& tr, float ox, float oy, float oz, float dx, float dy, float dz,
                                         float tmin, float tmax, float& t, float& u, float& v) {
    const float v0x = tr.p.x, v0y = tr.p.y, v0z = tr.p.z;
    const float e1x = tr.p.w, e1y = tr.q.x, e1z = tr.q.y;
    const float e2x = tr.q.z, e2y = tr.q.w, e2z = tr.r.x;
    const float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const float det = (e1x * px + e1y * py) + e1z * pz;
    if (det == 0.0f) return false;
    const float inv = 1.0f / det;
    const float sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
    u = ((sx * px + sy * py) + sz * pz) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return false;
    const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    v = ((dx * qx + dy * qy) + dz * qz) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return false;
    t = ((e2x * qx + e2y * qy) + e2z * qz) * inv;
    return t > tmin && t < tmax;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

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
    hcc::Node4* wnodes = nullptr;   // n_int slots, filled at even-depth internal ids
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
