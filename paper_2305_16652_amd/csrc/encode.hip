// Sorting-key kernels for gfx950.
//
// HCC (Algorithm 1, Section 4.2.1): every ray is tested against the first min(C, K) cut
// boxes (HAD order) and bit K-1-i records cut node i.  All lanes of a wavefront test the same
// box at the same time, so the boxes are read with scalar loads (one 32-byte load per box and
// wavefront, through the scalar cache, into SGPRs that the slab test reads directly).  Staged
// in LDS instead, each box cost two 16-byte reads per lane, and at 32 boxes per ray the LDS
// bandwidth bound the kernel.
//
// TwoPoint (Section 3.2; fixed-length end point of Section 5): 6-D Morton code of
// (origin, origin + 0.25 L * d/|d|), L the largest scene extent.
//
// Rays are 32-byte records read as two 16-byte loads per lane (fully coalesced).
#include "hcc_internal.h"

namespace hcc {
namespace {

constexpr uint32_t kBlock = 256;

// Bits of the boxes box[0 .. m) met by the ray, box 0 in bit m-1 (m <= 64).  The box index is
// the same for every lane, so the boxes come through scalar loads.
template <typename K>
__device__ __forceinline__ K box_bits(const CutBox* __restrict__ box, uint32_t m, float ox, float oy, float oz,
                                      float ix, float iy, float iz, float tmin, float tmax, int* first_hit) {
    K bits = 0;
    int first = -1;
#pragma unroll 4
    for (uint32_t i = 0; i < m; ++i) {
        const CutBox c = box[i];
        float tn;
        const bool hit = slab(ox, oy, oz, ix, iy, iz, tmin, tmax, c.lo.x, c.lo.y, c.lo.z, c.hi.x, c.hi.y, c.hi.z, tn);
        bits = (bits << 1) | (K)hit;
        if (first_hit && hit && first < 0) first = (int)i;
    }
    if (first_hit) *first_hit = first;
    return bits;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_encode_hcc(const float4* __restrict__ rays, uint32_t n,
                                                       const CutBox* __restrict__ cut, uint32_t m,
                                                       uint32_t key_bits, K* __restrict__ keys) {
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const float4 a = rays[2 * (size_t)r];
        const float4 b = rays[2 * (size_t)r + 1];
        const float ix = 1.0f / b.x, iy = 1.0f / b.y, iz = 1.0f / b.z;
        // 1 <= m <= key_bits: the m box bits go to the top of the key
        keys[r] = box_bits<K>(cut, m, a.x, a.y, a.z, ix, iy, iz, a.w, b.w, nullptr) << (key_bits - m);
    }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_encode_twopoint(const float4* __restrict__ rays, uint32_t n, float lox,
                                                            float loy, float loz, float hix, float hiy, float hiz,
                                                            uint32_t key_bits, K* __restrict__ keys) {
    const float lo[3] = {lox, loy, loz};
    const float ext[3] = {hix - lox, hiy - loy, hiz - loz};
    const float L = fmaxf(fmaxf(ext[0], ext[1]), ext[2]);
    const float t_est = 0.25f * L;
    uint32_t bits[6];
#pragma unroll
    for (uint32_t d = 0; d < 6; ++d) bits[d] = key_bits / 6 + (d < key_bits % 6 ? 1u : 0u);
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const float4 a = rays[2 * (size_t)r];
        const float4 b = rays[2 * (size_t)r + 1];
        const float len = sqrtf((b.x * b.x + b.y * b.y) + b.z * b.z);
        const float dist = fminf(t_est, b.w * len);
        const float dir[3] = {b.x, b.y, b.z};
        const float org[3] = {a.x, a.y, a.z};
        float p[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float dn = dir[k] / len;
            p[k] = org[k];
            p[3 + k] = org[k] + dn * dist;
        }
        uint32_t q[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const int ax = d % 3;
            float u = ext[ax] > 0.0f ? (p[d] - lo[ax]) / ext[ax] : 0.0f;
            u = fminf(fmaxf(u, 0.0f), 1.0f);
            const float qf = floorf(u * (float)(1u << bits[d]));
            const uint32_t qmax = (1u << bits[d]) - 1u;
            const uint32_t qi = (uint32_t)qf;
            q[d] = qi > qmax ? qmax : qi;
        }
        K key = 0;
        for (uint32_t level = 0; level < bits[0]; ++level) {
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                if (level < bits[d]) key = (key << 1) | (K)((q[d] >> (bits[d] - 1 - level)) & 1u);
            }
        }
        keys[r] = key;
    }
}

// MLHCC (Section 4.3): the top-level boxes are read like HCC's cut boxes (scalar loads); every
// top node's low-level boxes are staged in LDS (top x low <= 2048 boxes, 64 KB), since lanes
// whose rays meet different top nodes first read different rows.  Top bits as in HCC; the
// first top node met is the representative, whose low-level boxes give the low bits.
constexpr uint32_t kMaxLowBoxes = 2048;

template <typename K>
__global__ __launch_bounds__(kBlock) void k_encode_mlhcc(const float4* __restrict__ rays, uint32_t n,
                                                         const CutBox* __restrict__ boxes, uint32_t t_eff,
                                                         uint32_t low, uint32_t key_bits, K* __restrict__ keys) {
    __shared__ CutBox s_low[kMaxLowBoxes];
    for (uint32_t i = threadIdx.x; i < t_eff * low; i += kBlock) s_low[i] = boxes[t_eff + i];
    __syncthreads();
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const float4 a = rays[2 * (size_t)r];
        const float4 b = rays[2 * (size_t)r + 1];
        const float ix = 1.0f / b.x, iy = 1.0f / b.y, iz = 1.0f / b.z;
        int rep = -1;
        // 1 <= t_eff and t_eff + low <= key_bits
        K key = box_bits<K>(boxes, t_eff, a.x, a.y, a.z, ix, iy, iz, a.w, b.w, &rep) << (key_bits - t_eff);
        if (rep >= 0) {
            const CutBox* lb = s_low + (uint32_t)rep * low;
            for (uint32_t j = 0; j < low; ++j) {
                const CutBox c = lb[j];
                float tn;
                const bool hit = slab(a.x, a.y, a.z, ix, iy, iz, a.w, b.w, c.lo.x, c.lo.y, c.lo.z, c.hi.x, c.hi.y,
                                      c.hi.z, tn);
                key |= (K)hit << (low - 1 - j);
            }
        }
        keys[r] = key;
    }
}

// PPC (Section 4.1): each lane walks the BVH in the one forced order shared by all rays
// (expanding a node tests child 0 then child 1; child 0's subtree first; only met internal
// children are expanded) and appends one bit per box test until key_bits tests are made.
// Every expansion uses up to two bits and pushes at most one net entry, so the walk never
// holds more than key_bits / 2 + 1 <= 33 nodes.
constexpr uint32_t kPpcStack = 34;

template <typename K>
__global__ __launch_bounds__(kBlock) void k_encode_ppc(const float4* __restrict__ rays, uint32_t n,
                                                       const Node* __restrict__ nodes, uint32_t n_int,
                                                       const float* __restrict__ root_box, uint32_t key_bits,
                                                       K* __restrict__ keys) {
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const float4 a = rays[2 * (size_t)r];
        const float4 b = rays[2 * (size_t)r + 1];
        const float ix = 1.0f / b.x, iy = 1.0f / b.y, iz = 1.0f / b.z;
        K key = 0;
        float tn;
        if (n_int == 0) {
            if (slab(a.x, a.y, a.z, ix, iy, iz, a.w, b.w, root_box[0], root_box[1], root_box[2], root_box[3],
                     root_box[4], root_box[5], tn))
                key = (K)1 << (key_bits - 1);
        } else {
            uint32_t stack[kPpcStack];
            uint32_t sp = 0, bits = 0;
            stack[sp++] = 0;
            while (sp > 0 && bits < key_bits) {
                const Node nd = nodes[stack[--sp]];
                const bool m0 = slab(a.x, a.y, a.z, ix, iy, iz, a.w, b.w, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x,
                                     nd.b.y, tn);
                key |= (K)m0 << (key_bits - 1 - bits);
                ++bits;
                bool m1 = false;
                if (bits < key_bits) {
                    m1 = slab(a.x, a.y, a.z, ix, iy, iz, a.w, b.w, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w,
                              tn);
                    key |= (K)m1 << (key_bits - 1 - bits);
                    ++bits;
                }
                if (m1 && nd.d.y < n_int && sp < kPpcStack) stack[sp++] = nd.d.y;
                if (m0 && nd.d.x < n_int && sp < kPpcStack) stack[sp++] = nd.d.x;
            }
        }
        keys[r] = key;
    }
}

// Blocks for n rays: enough to fill 256 CUs several times over, a grid-stride loop covering the
// rest.  Memory-bound encodes (few boxes per ray, TwoPoint) take one ray per thread instead: more
// loads in flight (measured on 16.6M rays: 4 boxes 0.121 -> 0.110 ms, TwoPoint 0.123 -> 0.107 ms;
// with 16 or 32 boxes per ray the capped grid is 5% faster).
inline unsigned grid_for(uint32_t n, bool light = false) {
    const uint32_t want = (n + kBlock - 1) / kBlock;
    return std::max(1u, std::min(want, light ? 256u * 256u : 256u * 32u));
}

}  // namespace

hcc_status encode_hcc(const hcc_cut_s* cut, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                      hipStream_t stream) {
    const uint32_t m = std::min(cut->c_eff, key_bits);
    if (key_bits <= 32)
        k_encode_hcc<uint32_t><<<grid_for(n, m <= 8), kBlock, 0, stream>>>((const float4*)d_rays, n, cut->d_boxes, m,
                                                                   key_bits, (uint32_t*)d_keys);
    else
        k_encode_hcc<uint64_t><<<grid_for(n, m <= 8), kBlock, 0, stream>>>((const float4*)d_rays, n, cut->d_boxes, m,
                                                                   key_bits, (uint64_t*)d_keys);
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

hcc_status encode_mlhcc(const hcc_cut_s* cut, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                        hipStream_t stream) {
    if (key_bits <= 32)
        k_encode_mlhcc<uint32_t><<<grid_for(n), kBlock, 0, stream>>>((const float4*)d_rays, n, cut->d_boxes,
                                                                     cut->c_eff, cut->low, key_bits,
                                                                     (uint32_t*)d_keys);
    else
        k_encode_mlhcc<uint64_t><<<grid_for(n), kBlock, 0, stream>>>((const float4*)d_rays, n, cut->d_boxes,
                                                                     cut->c_eff, cut->low, key_bits,
                                                                     (uint64_t*)d_keys);
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

hcc_status encode_ppc(const hcc_bvh_s* bvh, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                      hipStream_t stream) {
    if (key_bits <= 32)
        k_encode_ppc<uint32_t><<<grid_for(n), kBlock, 0, stream>>>((const float4*)d_rays, n, bvh->nodes, bvh->n_int,
                                                                   bvh->boxes, key_bits, (uint32_t*)d_keys);
    else
        k_encode_ppc<uint64_t><<<grid_for(n), kBlock, 0, stream>>>((const float4*)d_rays, n, bvh->nodes, bvh->n_int,
                                                                   bvh->boxes, key_bits, (uint64_t*)d_keys);
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

hcc_status encode_twopoint(const hcc_bvh_s* bvh, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                           hipStream_t stream) {
    const float* s = bvh->scene_box;
    if (key_bits <= 32)
        k_encode_twopoint<uint32_t><<<grid_for(n, true), kBlock, 0, stream>>>((const float4*)d_rays, n, s[0], s[1], s[2],
                                                                        s[3], s[4], s[5], key_bits,
                                                                        (uint32_t*)d_keys);
    else
        k_encode_twopoint<uint64_t><<<grid_for(n, true), kBlock, 0, stream>>>((const float4*)d_rays, n, s[0], s[1], s[2],
                                                                        s[3], s[4], s[5], key_bits,
                                                                        (uint64_t*)d_keys);
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

}  // namespace hcc
