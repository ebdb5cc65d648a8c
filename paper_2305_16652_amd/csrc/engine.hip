// Batched engine: many ray batches of different sizes over several resident scenes in ONE
// persistent launch (encode -> per-batch radix sort -> trace), for gfx950.
//
// The launch works through a queue of items in batch-major order; for every batch:
//   E   tiles of 1024 rays: sorting keys (HCC of the batch's scene, or TwoPoint) and the
//       batch's digit histograms for every sort pass (wavefront-aggregated atomics);
//   S_p for each 8-bit pass p, tiles of 1024 keys: stable ranking with wavefront ballots,
//       decoupled look-back over the batch's earlier tiles, scatter to the pass's output;
//   T   chunks of rays traced through the batch's final permutation with lane refill and
//       batched leaf tests (as the persistent trace kernel).
// A wavefront takes the next item from a global counter.  Before an item of phase q it waits
// until every item of phase q-1 of the same batch has signalled completion; look-back waits
// only on earlier tiles of the same pass.  Everything waited on sits earlier in the queue and
// is therefore already held by a running wavefront that waits only on still earlier items, so
// the launch always drains.  Completion is signalled with a release fence + counter increment
// and observed with an agent-scope load + acquire fence.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "hcc_internal.h"

namespace hcc {

// the full-device kernels (encode.hip, trace.hip) used for direct launches
hcc_status encode_hcc(const hcc_cut_s* cut, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                      hipStream_t stream);
hcc_status encode_twopoint(const hcc_bvh_s* bvh, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                           hipStream_t stream);
hcc_status trace(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                 hcc_hit* hits, uint8_t* occ, const hcc_trace_opts& o, hipStream_t s);

struct EngScene {
    const Node* nodes;
    const Node4* wnodes;
    const Node4Q* qnodes;  // quantised 4-wide nodes (HCC_TRACE_QUANT and the BVH has them), else null
    const Tri* tris;
    const CutBox* cut;
    uint32_t n_int;
    uint32_t m;            // cut boxes encoded (min(c_eff, key_bits)); 0 for TwoPoint / NoSort
    float lo[3], hi[3];    // scene box (TwoPoint)
};

struct EngHeader {
    uint32_t nb, total_items, mode, key_bits, passes, refill, total_tiles, slab;   // slab: HCC_TRACE_SLAB given
    uint32_t* zero;        // region cleared before the engine runs (starts with the queue counter)
    uint32_t* queue;
    uint64_t zero_words;
};

struct EngBatch {
    const float4* rays;
    float4* hits;
    uint8_t* occ;
    void* keys_a;
    void* keys_b;
    uint32_t* vals_a;
    uint32_t* vals_b;
    uint32_t* hist;        // passes x 256
    uint32_t* lookback;    // passes x tiles x 256
    uint32_t* done;        // passes + 1 completion counters
    // tile0 / trace0: tiles / trace items of the batches before this one; chunk: rays per trace item
    uint32_t scene, n, closest, tiles, trace_items, tile0, trace0, chunk;
};

namespace {

constexpr uint32_t kTile = 1024;      // keys per encode / sort tile (64 lanes x 16)
constexpr uint32_t kDirectFloor = 65536;   // smallest batch that may take a direct launch
constexpr int kEngShort = 12;              // 4-wide trace: default stack entries per lane kept in LDS
constexpr int kEngLds = 24;                // 4-wide trace with HCC_STACK_LDS: LDS entries per lane

// LDS stack entries per lane of the engine's 4-wide trace phase for an hcc_stack_mode.
inline int engine_stack_entries(uint32_t stack) {
    return stack == HCC_BATCH_STACK_SCRATCH ? 0 : (stack == HCC_STACK_LDS ? kEngLds : kEngShort);
}
constexpr uint32_t kPerLane = 16;
constexpr uint32_t kRadix = 256;
constexpr uint32_t kFlagAgg = 1u << 30, kFlagIncl = 2u << 30, kCountMask = (1u << 30) - 1u;
constexpr uint32_t kNone = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t below_mask() {
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

__device__ __forceinline__ uint64_t same_digit(uint32_t d, uint32_t nbits, bool alive) {
    uint64_t m = __ballot(alive);
    for (uint32_t b = 0; b < nbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t& total) {
    const uint32_t lane = __lane_id();
    uint32_t incl = x;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    total = __shfl(incl, 63, 64);
    return incl - x;
}

// Every wait is bounded: after about a second of spinning the wave gives up, records the
// fault in 'err' and carries on, so a broken dependency yields wrong results, never a hang.
constexpr uint32_t kSpinLimit = 1u << 24;

// Data handed from one phase to the next inside the launch (keys, permutation values, pass
// histograms) is stored and loaded with device-scope atomic accesses, which are coherent across
// the XCDs' separate L2 caches.  A phase's completion count is raised only after the wavefront's
// stores have completed, and the next phase reads that data only after seeing the count, so no
// L2 write-back or invalidation (a device-scope fence) is needed: those flushed and emptied the
// L2 under every tile, the trace phase's scene data included.
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wait_count(const uint32_t* p, uint32_t target, uint32_t* err) {
    uint32_t spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins == kSpinLimit) {
            if (__lane_id() == 0) atomicOr(err, 1u);
            break;
        }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);   // the phase's loads stay after the wait
}

__device__ __forceinline__ void signal(uint32_t* p) {
    // every memory operation of this wavefront, its device-scope stores included, completes
    // before the count is raised
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (__lane_id() == 0) atomicAdd(p, 1u);
}

// HCC key of one ray.  The cut's boxes stay unchanged while the engine runs and every lane of
// the wavefront reads the same box, so they are read through the constant address space:
// scalar loads into SGPRs (a wavefront-uniform 32-byte load per box) instead of a copy in LDS
// that every lane reads.
typedef const __attribute__((address_space(4))) float* ConstFloats;

template <typename K>
__device__ K hcc_key(const CutBox* cut, uint32_t m, uint32_t key_bits, float4 a, float4 b) {
    const ConstFloats box = (ConstFloats)cut;   // CutBox i: lo.xyz at 8i, hi.xyz at 8i + 4
    const float ix = 1.0f / b.x, iy = 1.0f / b.y, iz = 1.0f / b.z;
    K bits = 0;
#pragma unroll 4
    for (uint32_t i = 0; i < m; ++i) {
        const ConstFloats c = box + 8 * i;
        float tn;
        const bool hit = slab(a.x, a.y, a.z, ix, iy, iz, a.w, b.w, c[0], c[1], c[2], c[4], c[5], c[6], tn);
        bits = (bits << 1) | (K)hit;
    }
    // 1 <= m <= key_bits: the m box bits go to the top of the key
    return bits << (key_bits - m);
}

template <typename K>
__device__ K twopoint_key(const EngScene& sc, uint32_t key_bits, float4 a, float4 b) {
    const float lo[3] = {sc.lo[0], sc.lo[1], sc.lo[2]};
    const float ext[3] = {sc.hi[0] - sc.lo[0], sc.hi[1] - sc.lo[1], sc.hi[2] - sc.lo[2]};
    const float L = fmaxf(fmaxf(ext[0], ext[1]), ext[2]);
    const float len = sqrtf((b.x * b.x + b.y * b.y) + b.z * b.z);
    const float dist = fminf(0.25f * L, b.w * len);
    const float dir[3] = {b.x, b.y, b.z}, org[3] = {a.x, a.y, a.z};
    float p[6];
    for (int k = 0; k < 3; ++k) {
        p[k] = org[k];
        p[3 + k] = org[k] + (dir[k] / len) * dist;
    }
    uint32_t bits[6], q[6];
    for (uint32_t d = 0; d < 6; ++d) bits[d] = key_bits / 6 + (d < key_bits % 6 ? 1u : 0u);
    for (int d = 0; d < 6; ++d) {
        const int ax = d % 3;
        float u = ext[ax] > 0.0f ? (p[d] - lo[ax]) / ext[ax] : 0.0f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const uint32_t qi = (uint32_t)floorf(u * (float)(1u << bits[d]));
        const uint32_t qmax = (1u << bits[d]) - 1u;
        q[d] = qi > qmax ? qmax : qi;
    }
    K key = 0;
    for (uint32_t level = 0; level < bits[0]; ++level)
        for (int d = 0; d < 6; ++d)
            if (level < bits[d]) key = (key << 1) | (K)((q[d] >> (bits[d] - 1 - level)) & 1u);
    return key;
}

// ---- E: keys of one tile + histogram of every pass.  The first pass's digits are counted in
// LDS and added to the batch's histogram once per tile (every tile of a batch adds to the same
// few bins, so per-key global atomics would queue on them); later passes add per wavefront
// group of equal digits.
template <typename K>
__device__ void encode_tile(const EngScene& sc, const EngBatch& bt, uint32_t tile, uint32_t mode, uint32_t key_bits,
                            uint32_t passes, uint32_t* s_h0) {
    const uint32_t lane = __lane_id();
    for (uint32_t j = 0; j < 4; ++j) s_h0[lane * 4 + j] = 0;
    __syncthreads();
    const uint64_t lt = below_mask();
    K* keys = (K*)bt.keys_a;
    for (uint32_t i = 0; i < kPerLane; ++i) {
        const uint32_t idx = tile * kTile + i * 64 + lane;
        const bool valid = idx < bt.n;
        K key = 0;
        if (valid) {
            const float4 a = bt.rays[2 * (size_t)idx], b = bt.rays[2 * (size_t)idx + 1];
            key = mode == HCC_KEY_HCC ? hcc_key<K>(sc.cut, sc.m, key_bits, a, b) : twopoint_key<K>(sc, key_bits, a, b);
            st_dev(keys + idx, key);
        }
        for (uint32_t p = 0; p < passes; ++p) {
            const uint32_t nb = min(8u, key_bits - 8u * p);
            const uint32_t d = (uint32_t)(key >> (8u * p)) & ((1u << nb) - 1u);
            const uint64_t m = same_digit(d, nb, valid);
            if (valid && (m & lt) == 0) {
                if (p == 0) atomicAdd(&s_h0[d], (uint32_t)__popcll(m));
                else atomicAdd(&bt.hist[p * kRadix + d], (uint32_t)__popcll(m));
            }
        }
    }
    __syncthreads();
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t c = s_h0[lane * 4 + j];
        if (c) atomicAdd(&bt.hist[lane * 4 + j], c);
    }
    __syncthreads();
}

// ---- S_p: one tile of one pass
// Register budget: the 1,024 ranks wait in LDS (16-bit) across the look-back; keys are read
// once to rank them and once more (from L2) to scatter them, so the engine kernel keeps the
// trace phase's register count and occupancy.
template <typename K>
__device__ void scatter_tile(const EngBatch& bt, uint32_t tile, uint32_t p, uint32_t key_bits, uint32_t* s_whist,
                             uint32_t* s_gbase, uint16_t* s_rank, uint32_t* err) {
    const uint32_t lane = __lane_id();
    const K* kin = (const K*)((p & 1) ? bt.keys_b : bt.keys_a);
    K* kout = (K*)((p & 1) ? bt.keys_a : bt.keys_b);
    const uint32_t* vin = (p & 1) ? bt.vals_b : bt.vals_a;
    uint32_t* vout = (p & 1) ? bt.vals_a : bt.vals_b;
    const uint32_t shift = 8u * p, nbits = min(8u, key_bits - 8u * p), mask = (1u << nbits) - 1u;
    for (uint32_t j = 0; j < 4; ++j) s_whist[lane * 4 + j] = 0;
    __syncthreads();
    const uint64_t lt = below_mask();
    const uint32_t base_idx = tile * kTile + lane;
#pragma unroll 4
    for (uint32_t i = 0; i < kPerLane; ++i) {
        const uint32_t idx = base_idx + i * 64;
        const bool valid = idx < bt.n;
        const K key = valid ? ld_dev(kin + idx) : K(0);
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        const uint64_t m = same_digit(d, nbits, valid);
        const uint32_t below = (uint32_t)__popcll(m & lt);
        const uint32_t prev = valid ? s_whist[d] : 0u;
        s_rank[i * 64 + lane] = (uint16_t)(prev + below);
        if (valid && below == 0) s_whist[d] = prev + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // lane owns digits 4 lane .. 4 lane + 3
    uint32_t cnt[4], excl[4];
    uint32_t* lb = bt.lookback + ((size_t)p * bt.tiles + tile) * kRadix;
    for (uint32_t j = 0; j < 4; ++j) {
        cnt[j] = s_whist[lane * 4 + j];
        excl[j] = 0;
        __hip_atomic_store(lb + lane * 4 + j, (tile == 0 ? kFlagIncl : kFlagAgg) | cnt[j], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tile > 0) {
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t d = lane * 4 + j;
            int64_t t = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (true) {
                const uint32_t x = __hip_atomic_load(bt.lookback + ((size_t)p * bt.tiles + t) * kRadix + d,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t f = x & ~kCountMask;
                if (f == 0) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins == kSpinLimit) {
                        atomicOr(err, 2u);
                        break;
                    }
                    continue;
                }
                excl[j] += x & kCountMask;
                if (f == kFlagIncl) break;
                --t;
            }
            __hip_atomic_store(lb + d, kFlagIncl | (excl[j] + cnt[j]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // global start of each digit: exclusive scan of the pass histogram + earlier tiles
    uint32_t h[4], hs = 0, total;
    for (uint32_t j = 0; j < 4; ++j) {
        h[j] = ld_dev(bt.hist + p * kRadix + lane * 4 + j);
        hs += h[j];
    }
    uint32_t base = wave_excl_scan(hs, total);
    for (uint32_t j = 0; j < 4; ++j) {
        s_gbase[lane * 4 + j] = base + excl[j];
        base += h[j];
    }
    __syncthreads();
#pragma unroll 4
    for (uint32_t i = 0; i < kPerLane; ++i) {
        const uint32_t idx = base_idx + i * 64;
        if (idx < bt.n) {
            const K key = ld_dev(kin + idx);
            const uint32_t val = p == 0 ? idx : ld_dev(vin + idx);
            const uint32_t d = (uint32_t)(key >> shift) & mask;
            const uint32_t pos = s_gbase[d] + s_rank[i * 64 + lane];
            if (pos < bt.n) {   // always true unless a dependency failed (then 'err' is set)
                st_dev(kout + pos, key);
                st_dev(vout + pos, val);
            }
        }
    }
    __syncthreads();
}

// ---- T: trace rays [begin, end) of the batch's order with lane refill and batched leaves
__device__ void trace_range(const EngScene& sc, const EngBatch& bt, const uint32_t* perm, uint32_t begin,
                            uint32_t end, uint32_t refill) {
    const bool closest = bt.closest != 0;
    const uint64_t below = below_mask();
    uint32_t stk[kStackDepth];
    uint32_t next = begin;
    bool has = false;
    uint32_t rid = 0, node = kNone, sp = 0, best_prim = kMissPrim, pend0 = kNone, pend1 = kNone, pend2 = kNone;
    float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, ix = 0, iy = 0, iz = 0, tmin = 0, tmax = 0;
    float best_t = 0, best_u = 0, best_v = 0;
    bool found = false;
    const uint32_t n_int = sc.n_int;
    auto test_tri = [&](uint32_t slot) {
        const Tri tr = sc.tris[slot];
        const uint32_t prim = __float_as_uint(tr.r.y);
        float t, u, v;
        if (tri_test(tr, ox, oy, oz, dx, dy, dz, tmin, tmax, t, u, v)) {
            if (!closest) {
                found = true;
            } else if (t < best_t || (t == best_t && prim < best_prim)) {
                best_t = t; best_u = u; best_v = v; best_prim = prim;
                found = true;
            }
        }
    };
    while (true) {
        const uint64_t idle = __ballot(!has);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (nidle >= refill || nidle == 64) {
            if (next < end) {
                const uint32_t k = next + (uint32_t)__popcll(idle & below);
                if (!has && k < end) {
                    rid = perm ? ld_dev(perm + k) : k;
                    if (rid < bt.n) {
                        const float4 ra = bt.rays[2 * (size_t)rid], rb = bt.rays[2 * (size_t)rid + 1];
                        ox = ra.x; oy = ra.y; oz = ra.z; tmin = ra.w;
                        dx = rb.x; dy = rb.y; dz = rb.z; tmax = rb.w;
                        ix = 1.0f / dx; iy = 1.0f / dy; iz = 1.0f / dz;
                        best_t = tmax; best_u = 0.0f; best_v = 0.0f; best_prim = kMissPrim;
                        found = false;
                        sp = 0;
                        pend0 = pend1 = pend2 = kNone;
                        node = 0;
                        if (n_int == 0) {          // single-triangle scene: the root is leaf 0
                            node = kNone;
                            pend0 = 0;
                        }
                        has = true;
                    }
                }
                next = min(next + nidle, end);
            } else if (nidle == 64) {
                break;
            }
        }
        if (has && node != kNone && pend1 == kNone) {
            const Node nd = sc.nodes[node];
            const float lim = closest ? best_t : tmax;
            float tn0, tn1;
            bool h0 = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, tn0);
            bool h1 = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, tn1);
            const uint32_t c0 = nd.d.x, c1 = nd.d.y;
            const bool leaf0 = h0 && c0 >= n_int, leaf1 = h1 && c1 >= n_int;
            if (leaf0 || leaf1) {
                const uint32_t a = leaf0 ? c0 - n_int : c1 - n_int;
                const uint32_t b = (leaf0 && leaf1) ? c1 - n_int : kNone;
                if (pend0 == kNone) { pend0 = a; pend1 = b; } else { pend1 = a; pend2 = b; }
            }
            h0 = h0 && !leaf0;
            h1 = h1 && !leaf1;
            if (h0 && h1) {
                const bool near1 = tn1 < tn0;
                stk[sp++] = near1 ? c0 : c1;
                node = near1 ? c1 : c0;
            } else if (h0) {
                node = c0;
            } else if (h1) {
                node = c1;
            } else if (sp == 0) {
                node = kNone;
            } else {
                node = stk[--sp];
            }
        }
        const bool can_step = has && node != kNone && pend1 == kNone;
        const uint64_t busy = __ballot(has);
        const uint64_t waiting = __ballot(has && pend0 != kNone && !can_step);
        const uint64_t stepping = __ballot(can_step);
        if (waiting != 0 && (2 * __popcll(waiting) >= __popcll(busy) || stepping == 0)) {
            if (has && pend0 != kNone) {
                test_tri(pend0);
                if (pend1 != kNone && (closest || !found)) test_tri(pend1);
                if (pend2 != kNone && (closest || !found)) test_tri(pend2);
                pend0 = pend1 = pend2 = kNone;
                if (!closest && found) node = kNone;
            }
        }
        if (has && node == kNone && pend0 == kNone) {
            if (closest)
                bt.hits[rid] = make_float4(found ? best_t : INFINITY, __uint_as_float(found ? best_prim : kMissPrim),
                                           found ? best_u : 0.0f, found ? best_v : 0.0f);
            else
                bt.occ[rid] = found ? 1 : 0;
            has = false;
        }
    }
}

// compare-exchange by selects (no branch)
__device__ __forceinline__ void cswap4(float& ka, uint32_t& ia, float& kb, uint32_t& ib) {
    const bool sw = kb < ka;
    const float k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const uint32_t i0 = sw ? ib : ia, i1 = sw ? ia : ib;
    ka = k0;
    kb = k1;
    ia = i0;
    ib = i1;
}

// ---- T over the 4-wide nodes (the persistent 4-wide trace kernel's step, for rays
// [begin, end) of the batch's order)
template <bool closest, int kShort>
__device__ void trace_range_wide_t(const EngScene& sc, const EngBatch& bt, const uint32_t* perm, uint32_t begin,
                                   uint32_t end, uint32_t refill, uint32_t slab, uint32_t* s_stk) {
    const uint64_t below = below_mask();
    // first kShort entries per lane in LDS (lane-interleaved), deeper ones in scratch
    uint32_t deep[kWideStack - kShort];
    uint32_t* lds = s_stk + __lane_id();
    auto push = [&](uint32_t i, uint32_t x) {
        if (i < (uint32_t)kShort) lds[i * 64] = x;
        else deep[i - kShort] = x;
    };
    auto pop = [&](uint32_t i) { return i < (uint32_t)kShort ? lds[i * 64] : deep[i - kShort]; };
    uint32_t next = begin;
    bool has = false;
    uint32_t rid = 0, node = kNone, sp = 0, best_prim = kMissPrim, pnode = 0, pmask = 0;
    float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, ix = 0, iy = 0, iz = 0, tmin = 0, tmax = 0;
    float best_t = 0, best_u = 0, best_v = 0;
    WideRay wr{0, 0, 0, false};
    bool found = false;
    const uint32_t n_int = sc.n_int;
    const bool fast_nodes = !slab && n_int <= kWideFastNodes;
    auto test_tri = [&](uint32_t slot) {
        const Tri tr = sc.tris[slot];
        const uint32_t prim = __float_as_uint(tr.r.y);
        float t, u, v;
        const bool hit = tri_test(tr, ox, oy, oz, dx, dy, dz, tmin, tmax, t, u, v);
        if (!closest) {
            found = found || hit;
        } else {
            const bool take = hit && (t < best_t || (t == best_t && prim < best_prim));
            best_t = take ? t : best_t;
            best_u = take ? u : best_u;
            best_v = take ? v : best_v;
            best_prim = take ? prim : best_prim;
            found = found || take;
        }
    };
    while (true) {
        const uint64_t idle = __ballot(!has);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (nidle >= refill || nidle == 64) {
            if (next < end) {
                const uint32_t k = next + (uint32_t)__popcll(idle & below);
                if (!has && k < end) {
                    rid = perm ? ld_dev(perm + k) : k;
                    if (rid < bt.n) {
                        const float4 ra = bt.rays[2 * (size_t)rid], rb = bt.rays[2 * (size_t)rid + 1];
                        ox = ra.x; oy = ra.y; oz = ra.z; tmin = ra.w;
                        dx = rb.x; dy = rb.y; dz = rb.z; tmax = rb.w;
                        ix = 1.0f / dx; iy = 1.0f / dy; iz = 1.0f / dz;
                        wr = wide_ray(ox, oy, oz, ix, iy, iz);
                        best_t = tmax; best_u = 0.0f; best_v = 0.0f; best_prim = kMissPrim;
                        found = false;
                        sp = 0;
                        pmask = 0;
                        node = 0;
                        if (n_int == 0) {          // single-triangle scene: test its triangle now
                            node = kNone;
                            test_tri(0);
                        }
                        has = true;
                    }
                }
                next = min(next + nidle, end);
            } else if (nidle == 64) {
                break;
            }
        }
        const bool step = has && node != kNone && pmask == 0;
        // the node step is specialised on the (wavefront-uniform) form of the child test
        auto node_step = [&](auto kind) {
            uint4 r;
            bool hh[4];
            float tt[4];
            constexpr int kKind = decltype(kind)::value;   // 0 slab, 1 selected planes, 2 / 3 quantised
            if constexpr (kKind >= 2)
                wide_test_q<kKind == 3>(sc.qnodes, node, wr, ox, oy, oz, ix, iy, iz, tmin, closest ? best_t : tmax, r,
                                        hh, tt);
            else
                wide_test<kKind == 1>(sc.wnodes, node, wr, ox, oy, oz, ix, iy, iz, tmin, closest ? best_t : tmax, r,
                                      hh, tt);
            const bool h0 = hh[0], h1 = hh[1], h2 = hh[2], h3 = hh[3];
            const float t0 = tt[0], t1 = tt[1], t2 = tt[2], t3 = tt[3];
            const bool l0 = h0 && (r.x & kWideLeaf), l1 = h1 && (r.y & kWideLeaf);
            const bool l2 = h2 && (r.z & kWideLeaf), l3 = h3 && (r.w & kWideLeaf);
            const uint32_t lm = (l0 ? 1u : 0u) | (l1 ? 2u : 0u) | (l2 ? 4u : 0u) | (l3 ? 8u : 0u);
            if (lm) {
                pnode = node;
                pmask = lm;
            }
            float k0 = (h0 && !l0) ? t0 : INFINITY, k1 = (h1 && !l1) ? t1 : INFINITY;
            float k2 = (h2 && !l2) ? t2 : INFINITY, k3 = (h3 && !l3) ? t3 : INFINITY;
            uint32_t i0 = (h0 && !l0) ? r.x : kNone, i1 = (h1 && !l1) ? r.y : kNone;
            uint32_t i2 = (h2 && !l2) ? r.z : kNone, i3 = (h3 && !l3) ? r.w : kNone;
            cswap4(k0, i0, k1, i1);
            cswap4(k2, i2, k3, i3);
            cswap4(k0, i0, k2, i2);
            cswap4(k1, i1, k3, i3);
            cswap4(k1, i1, k2, i2);
            if (kShort >= 3 && __ballot(sp + 3 > (uint32_t)kShort) == 0) {
                // every stepping lane has three free LDS slots above its stack top: candidates
                // are written there and kept if valid, and the top is read back for the pop
                lds[sp * 64] = i3;
                sp += i3 < n_int ? 1u : 0u;
                lds[sp * 64] = i2;
                sp += i2 < n_int ? 1u : 0u;
                lds[sp * 64] = i1;
                sp += i1 < n_int ? 1u : 0u;
                const uint32_t top = lds[(sp > 0 ? sp - 1 : 0) * 64];
                const bool descend = i0 < n_int;
                node = descend ? i0 : (sp == 0 ? kNone : top);
                sp -= (!descend && sp > 0) ? 1u : 0u;
            } else {
                if (i3 < n_int && sp < kWideStack) push(sp++, i3);
                if (i2 < n_int && sp < kWideStack) push(sp++, i2);
                if (i1 < n_int && sp < kWideStack) push(sp++, i1);
                if (i0 < n_int) node = i0;
                else if (sp == 0) node = kNone;
                else node = pop(--sp);
            }
        };
        if (sc.qnodes) {
            if (!slab && __ballot(step && !wr.fast) == 0) {
                if (step) node_step(std::integral_constant<int, 3>{});
            } else {
                if (step) node_step(std::integral_constant<int, 2>{});
            }
        } else if (fast_nodes && __ballot(step && !wr.fast) == 0) {
            if (step) node_step(std::integral_constant<int, 1>{});
        } else {
            if (step) node_step(std::integral_constant<int, 0>{});
        }
        const bool can_step = has && node != kNone && pmask == 0;
        const uint64_t busy = __ballot(has);
        const uint64_t waiting = __ballot(has && pmask != 0);
        const uint64_t stepping = __ballot(can_step);
        // a leaf batch once a third of the busy lanes wait on one (measured: a half or two thirds
        // leave too many lanes idle in the node steps; a quarter is no better, fewer is worse)
        if (waiting != 0 && (3 * __popcll(waiting) >= __popcll(busy) || stepping == 0)) {
            const bool mine = has && pmask != 0;
            uint4 r = make_uint4(kNone, kNone, kNone, kNone);
            if (mine) r = sc.wnodes[pnode].ref;
            // pending triangles lowest slot first, one per lane and round
            uint32_t left = mine ? pmask : 0u;
            while (__ballot(left != 0) != 0) {
                if (left != 0) {
                    const uint32_t j = __builtin_ctz(left);
                    left &= left - 1u;
                    const uint32_t ref = j == 0 ? r.x : (j == 1 ? r.y : (j == 2 ? r.z : r.w));
                    test_tri(ref & ~kWideLeaf);
                    if (!closest && found) left = 0;
                }
            }
            if (mine) {
                pmask = 0;
                if (!closest && found) node = kNone;
            }
        }
        if (has && node == kNone && pmask == 0) {
            if (closest)
                bt.hits[rid] = make_float4(found ? best_t : INFINITY, __uint_as_float(found ? best_prim : kMissPrim),
                                           found ? best_u : 0.0f, found ? best_v : 0.0f);
            else
                bt.occ[rid] = found ? 1 : 0;
            has = false;
        }
    }
}

template <int kShort>
__device__ __forceinline__ void trace_range_wide(const EngScene& sc, const EngBatch& bt, const uint32_t* perm,
                                                 uint32_t begin, uint32_t end, uint32_t refill, uint32_t slab,
                                                 uint32_t* s_stk) {
    if (bt.closest) trace_range_wide_t<true, kShort>(sc, bt, perm, begin, end, refill, slab, s_stk);
    else trace_range_wide_t<false, kShort>(sc, bt, perm, begin, end, refill, slab, s_stk);
}

template <typename K, bool kWide, int kShort>
__device__ __forceinline__ void engine_loop(const EngScene* __restrict__ scenes, const EngBatch* __restrict__ batches,
                                            uint32_t nb, uint32_t total_items, uint32_t total_tiles, uint32_t* queue,
                                            uint32_t mode, uint32_t key_bits, uint32_t passes, uint32_t refill,
                                            uint32_t slab) {
    __shared__ uint32_t s_whist[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    // the scatter's ranks and the 4-wide trace's short stacks are never live at the same time
    __shared__ uint32_t s_share[kTile / 2 > kShort * 64 ? kTile / 2 : kShort * 64];
    uint16_t* s_rank = reinterpret_cast<uint16_t*>(s_share);
    uint32_t* s_stk = s_share;
    __shared__ uint32_t s_item;
    // Items are phase-major: the encode tiles of every batch, then the tiles of sort pass 0 of
    // every batch, ..., then the trace items of every batch.  An item depends only on its own
    // batch's previous phase, which was handed out before the whole current phase, so waits are
    // rare (only the last batches of a phase can still be running) and never circular.
    const uint32_t sort_items = mode == HCC_KEY_NONE ? 0u : (passes + 1) * total_tiles;
    while (true) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);   // wave-uniform: scalar from here
        __syncthreads();
        if (item >= total_items) break;
        const bool sorting = item < sort_items;
        const uint32_t phase = sorting ? item / max(total_tiles, 1u) : 0u;
        const uint32_t r = sorting ? item - phase * total_tiles : item - sort_items;
        // batch owning position r of this phase: the last one starting at or before it
        uint32_t lo = 0, hi = nb - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if ((sorting ? batches[mid].tile0 : batches[mid].trace0) <= r) lo = mid; else hi = mid - 1;
        }
        const EngBatch& bt = batches[lo];
        const EngScene& sc = scenes[bt.scene];
        if (!sorting) {
            const uint32_t c = r - bt.trace0;
            const uint32_t* perm = nullptr;
            if (mode != HCC_KEY_NONE) {
                wait_count(bt.done + passes, bt.tiles, queue + 1);
                perm = ((passes - 1) & 1) ? bt.vals_a : bt.vals_b;
            }
            if (kWide)
                trace_range_wide<kShort>(sc, bt, perm, c * bt.chunk, min(bt.n, (c + 1) * bt.chunk), refill, slab,
                                         s_stk);
            else
                trace_range(sc, bt, perm, c * bt.chunk, min(bt.n, (c + 1) * bt.chunk), refill);
            continue;
        }
        const uint32_t tile = r - bt.tile0;
        if (phase == 0) {
            encode_tile<K>(sc, bt, tile, mode, key_bits, passes, s_whist);
            signal(bt.done);
        } else {
            const uint32_t p = phase - 1;
            wait_count(bt.done + p, bt.tiles, queue + 1);
            scatter_tile<K>(bt, tile, p, key_bits, s_whist, s_gbase, s_rank, queue + 1);
            signal(bt.done + p + 1);
        }
    }
}

template <typename K, bool kWide, int kShort>
__global__ __launch_bounds__(64) void k_engine(const EngScene* __restrict__ scenes, const EngBatch* __restrict__ batches,
                                               uint32_t nb, uint32_t total_items, uint32_t total_tiles,
                                               uint32_t* queue, uint32_t mode,
                                               uint32_t key_bits, uint32_t passes, uint32_t refill, uint32_t slab) {
    engine_loop<K, kWide, kShort>(scenes, batches, nb, total_items, total_tiles, queue, mode, key_bits, passes,
                                  refill, slab);
}

__global__ void k_zero(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Graph-launched form: the launch parameters that change from group to group come from a
// header the same graph copies to the device first, so one captured graph (copy, clear,
// engine) serves every group.
template <typename K, bool kWide, int kShort>
__global__ __launch_bounds__(64) void k_engine_hdr(const EngHeader* __restrict__ h, const EngScene* __restrict__ scenes,
                                                   const EngBatch* __restrict__ batches) {
    engine_loop<K, kWide, kShort>(scenes, batches, h->nb, h->total_items, h->total_tiles, h->queue, h->mode, h->key_bits,
                          h->passes,
                          h->refill, h->slab);
}

__global__ void k_zero_hdr(const EngHeader* __restrict__ h) {
    uint32_t* p = h->zero;
    const size_t n = h->zero_words;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
    size_t tables, scenes_off, batches_off, zero_off, zero_bytes, total;
    std::vector<size_t> keys_a, keys_b, vals_a, vals_b, hist, lookback, done;
    uint32_t total_items = 0;
};

}  // namespace

// Workspace layout for a batch list (the caller allocates it once, e.g. for the largest set).
static Plan plan_batches(const hcc_batch_desc* d, uint32_t nb, uint32_t n_scenes, uint32_t mode, uint32_t key_bits,
                         uint32_t chunk) {
    Plan P;
    const size_t ks = key_bits <= 32 ? 4 : 8;
    const uint32_t passes = mode == HCC_KEY_NONE ? 0 : (key_bits + 7) / 8;
    size_t off = 0;
    // zeroed region first: queue counter and error flag (bytes 0 and 4 of every workspace),
    // histograms, look-back state, completion counters
    P.zero_off = off;
    off += 256;
    P.hist.resize(nb); P.lookback.resize(nb); P.done.resize(nb);
    for (uint32_t b = 0; b < nb; ++b) {
        const size_t tiles = (d[b].n + kTile - 1) / kTile;
        P.hist[b] = off; off += al((size_t)passes * kRadix * 4);
        P.lookback[b] = off; off += al((size_t)passes * tiles * kRadix * 4);
        P.done[b] = off; off += al((passes + 1) * 4);
    }
    P.zero_bytes = off - P.zero_off;
    // descriptor tables (copied from the host at launch)
    P.scenes_off = off; off += al(sizeof(EngScene) * n_scenes);
    P.batches_off = off; off += al(sizeof(EngBatch) * nb);
    P.tables = off - P.scenes_off;
    P.keys_a.resize(nb); P.keys_b.resize(nb); P.vals_a.resize(nb); P.vals_b.resize(nb);
    for (uint32_t b = 0; b < nb; ++b) {
        const size_t n = d[b].n;
        if (mode == HCC_KEY_NONE) continue;
        P.keys_a[b] = off; off += al(n * ks);
        P.keys_b[b] = off; off += al(n * ks);
        P.vals_a[b] = off; off += al(n * 4);
        P.vals_b[b] = off; off += al(n * 4);
    }
    P.total = off;
    (void)chunk;
    return P;
}

// A batch run outside the engine (direct launch): its keys, permutation and sort workspace.
static size_t direct_bytes(uint32_t n, uint32_t mode, uint32_t key_bits) {
    if (mode == HCC_KEY_NONE) return 0;
    const size_t ks = key_bits <= 32 ? 4 : 8;
    return al((size_t)n * ks) + al((size_t)n * 4) + al(sort_workspace_bytes(n, key_bits));
}

// Engine layout of every batch, then room for a direct launch of every batch that could take
// one (at least kDirectFloor rays), whatever opts.direct_min the run uses.
hcc_status batch_workspace(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits, size_t* bytes) {
    size_t total = al(plan_batches(d, nb, nb, mode, key_bits, 0).total);
    for (uint32_t b = 0; b < nb; ++b)
        if (d[b].n >= kDirectFloor) total += direct_bytes(d[b].n, mode, key_bits);
    *bytes = total;
    return HCC_OK;
}

// The engine part alone (the request server runs its large requests itself).
hcc_status engine_workspace(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits, size_t* bytes) {
    *bytes = plan_batches(d, nb, nb, mode, key_bits, 0).total;
    return HCC_OK;
}

// Host size of the descriptor tables a launch copies to the device.
size_t batch_table_bytes(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits) {
    return plan_batches(d, nb, nb, mode, key_bits, 0).tables;
}

// Device descriptor tables of a batch list whose workspace is d_ws.
struct Tables {
    Plan P;
    std::vector<EngScene> hs;
    std::vector<EngBatch> hb;
    EngHeader hdr{};
};

static hcc_status fill_tables(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                              const hcc_batch_opts& o, void* d_ws, size_t ws_bytes, Tables& T) {
    const uint32_t chunk = std::max<uint32_t>(64u, o.chunk ? o.chunk : 256u);
    const uint32_t refill = std::min<uint32_t>(64u, std::max<uint32_t>(1u, o.refill ? o.refill : 32u));
    // scenes: distinct (bvh, cut) pairs
    std::vector<const hcc_bvh_s*> sb;
    std::vector<const hcc_cut_s*> sc;
    std::vector<uint32_t> scene_of(nb);
    for (uint32_t b = 0; b < nb; ++b) {
        uint32_t s = 0;
        while (s < sb.size() && !(sb[s] == d[b].bvh && sc[s] == d[b].cut)) ++s;
        if (s == sb.size()) {
            sb.push_back(d[b].bvh);
            sc.push_back(d[b].cut);
        }
        scene_of[b] = s;
    }
    T.P = plan_batches(d, nb, (uint32_t)sb.size(), mode, key_bits, chunk);
    const Plan& P = T.P;
    if (ws_bytes < P.total) return fail(HCC_ERR_INVALID, "hcc_batch_run: workspace too small (see hcc_batch_workspace)");
    const uint32_t passes = mode == HCC_KEY_NONE ? 0 : (key_bits + 7) / 8;
    char* ws = (char*)d_ws;
    T.hs.assign(sb.size(), EngScene{});
    for (size_t s = 0; s < sb.size(); ++s) {
        EngScene& e = T.hs[s];
        e.nodes = sb[s]->nodes;
        e.wnodes = sb[s]->wnodes;
        // quantised nodes where asked for and available (a scene without them traces its exact
        // nodes: the same hits but for the rounding cases the quantised boxes also reach)
        e.qnodes = ((o.flags & HCC_TRACE_QUANT) && sb[s]->quant_ok) ? sb[s]->qnodes : nullptr;
        e.tris = sb[s]->tris;
        e.n_int = sb[s]->n_int;
        e.cut = sc[s] ? sc[s]->d_boxes : nullptr;
        e.m = (mode == HCC_KEY_HCC && sc[s]) ? std::min(sc[s]->c_eff, key_bits) : 0;
        for (int a = 0; a < 3; ++a) {
            e.lo[a] = sb[s]->scene_box[a];
            e.hi[a] = sb[s]->scene_box[3 + a];
        }
    }
    T.hb.assign(nb, EngBatch{});
    uint32_t tiles_before = 0, trace_before = 0;
    for (uint32_t b = 0; b < nb; ++b) {
        EngBatch& e = T.hb[b];
        e.rays = (const float4*)d[b].d_rays;
        e.hits = (float4*)d[b].d_hits;
        e.occ = d[b].d_occluded;
        e.scene = scene_of[b];
        e.n = d[b].n;
        e.closest = d[b].mode == HCC_TRACE_CLOSEST ? 1u : 0u;
        e.tiles = (d[b].n + kTile - 1) / kTile;
        // a batch too small to give every wavefront a full chunk gets smaller chunks (down to one
        // wavefront's worth), so its rays spread over ~2,048 wavefronts instead of a few
        e.chunk = std::max<uint32_t>(64u, std::min<uint32_t>(chunk, d[b].n / 2048u));
        e.trace_items = (d[b].n + e.chunk - 1) / e.chunk;
        e.hist = (uint32_t*)(ws + P.hist[b]);
        e.lookback = (uint32_t*)(ws + P.lookback[b]);
        e.done = (uint32_t*)(ws + P.done[b]);
        if (mode != HCC_KEY_NONE) {
            e.keys_a = ws + P.keys_a[b];
            e.keys_b = ws + P.keys_b[b];
            e.vals_a = (uint32_t*)(ws + P.vals_a[b]);
            e.vals_b = (uint32_t*)(ws + P.vals_b[b]);
        } else {
            e.keys_a = e.keys_b = nullptr;
            e.vals_a = e.vals_b = nullptr;
        }
        e.tile0 = tiles_before;
        e.trace0 = trace_before;
        tiles_before += e.tiles;
        trace_before += e.trace_items;
    }
    EngHeader& h = T.hdr;
    h.nb = nb;
    h.total_tiles = tiles_before;
    h.total_items = (mode == HCC_KEY_NONE ? 0u : tiles_before * (1 + passes)) + trace_before;
    h.mode = mode;
    h.key_bits = key_bits;
    h.passes = passes;
    h.refill = refill;
    h.slab = (o.flags & HCC_TRACE_SLAB) ? 1u : 0u;
    h.zero = (uint32_t*)(ws + P.zero_off);
    h.queue = (uint32_t*)(ws + P.zero_off);
    h.zero_words = P.zero_bytes / 4;
    return HCC_OK;
}

// One batch through the full-device kernels (encode, radix sort, persistent 4-wide trace) on
// the stream, with its buffers at ws.
static hcc_status run_direct(const hcc_batch_desc& d, uint32_t mode, uint32_t key_bits, bool quant, char* ws,
                             hipStream_t stream) {
    hcc_trace_opts to{};
    to.persistent = 1;
    to.stack = HCC_STACK_SHORT;
    to.refill = 32;
    to.chunk = 64;
    to.flags = HCC_TRACE_WIDE | ((quant && d.bvh->quant_ok) ? HCC_TRACE_QUANT : 0u);
    const uint32_t* perm = nullptr;
    if (mode != HCC_KEY_NONE) {
        const size_t ks = key_bits <= 32 ? 4 : 8;
        void* keys = ws;
        uint32_t* pm = (uint32_t*)(ws + al((size_t)d.n * ks));
        void* sws = ws + al((size_t)d.n * ks) + al((size_t)d.n * 4);
        const size_t swb = al(sort_workspace_bytes(d.n, key_bits));
        hcc_status st = mode == HCC_KEY_HCC ? encode_hcc(d.cut, key_bits, d.d_rays, d.n, keys, stream)
                                            : encode_twopoint(d.bvh, key_bits, d.d_rays, d.n, keys, stream);
        if (st != HCC_OK) return st;
        if ((st = radix_sort(keys, key_bits, d.n, pm, nullptr, nullptr, sws, swb, stream)) != HCC_OK) return st;
        perm = pm;
    }
    return trace(d.bvh, d.d_rays, perm, d.n, d.mode == HCC_TRACE_CLOSEST, d.d_hits, d.d_occluded, to, stream);
}

// Launch a batch list.  With 'pinned' (page-locked host memory of at least
// batch_table_bytes, kept alive by the caller until the stream has passed this launch) the
// descriptor copy is asynchronous; without it a private buffer is used and the copy waited for.
static hcc_status engine_launch(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                                const hcc_batch_opts& o, void* d_ws, size_t ws_bytes, hipStream_t stream, void* pinned,
                                size_t pinned_bytes);

hcc_status batch_launch(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                        const hcc_batch_opts& o, void* d_ws, size_t ws_bytes, hipStream_t stream, void* pinned,
                        size_t pinned_bytes) {
    if (o.direct_min == 0) return engine_launch(d, nb, mode, key_bits, o, d_ws, ws_bytes, stream, pinned, pinned_bytes);
    // batches of at least direct_min rays run through the full-device kernels after the engine
    // launch of the others; their buffers follow the engine layout of the whole list
    std::vector<hcc_batch_desc> rest;
    for (uint32_t b = 0; b < nb; ++b)
        if (d[b].n < o.direct_min) rest.push_back(d[b]);
    size_t off = al(plan_batches(d, nb, nb, mode, key_bits, 0).total);
    if (!rest.empty()) {
        const hcc_status st = engine_launch(rest.data(), (uint32_t)rest.size(), mode, key_bits, o, d_ws, off, stream,
                                            pinned, pinned_bytes);
        if (st != HCC_OK) return st;
    } else {   // no engine launch: still clear the error flag that hcc_batch_check reads
        k_zero<<<1, 64, 0, stream>>>((uint32_t*)d_ws, 64);
        HCC_HIP(hipGetLastError());
    }
    for (uint32_t b = 0; b < nb; ++b) {
        if (d[b].n < o.direct_min) continue;
        const size_t need = direct_bytes(d[b].n, mode, key_bits);
        if (off + need > ws_bytes) return fail(HCC_ERR_INVALID, "hcc_batch_run: workspace too small (see hcc_batch_workspace)");
        const hcc_status st = run_direct(d[b], mode, key_bits, (o.flags & HCC_TRACE_QUANT) != 0, (char*)d_ws + off,
                                         stream);
        if (st != HCC_OK) return st;
        off += need;
    }
    return HCC_OK;
}

static hcc_status engine_launch(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                                const hcc_batch_opts& o, void* d_ws, size_t ws_bytes, hipStream_t stream, void* pinned,
                                size_t pinned_bytes) {
    Tables T;
    hcc_status st = fill_tables(d, nb, mode, key_bits, o, d_ws, ws_bytes, T);
    if (st != HCC_OK) return st;
    const Plan& P = T.P;
    const EngHeader& h = T.hdr;
    char* ws = (char*)d_ws;
    // the descriptor tables travel with the launch on the stream; the host copies are kept
    // alive until the stream has consumed them
    static thread_local std::vector<char> staging;
    char* host = (char*)pinned;
    if (pinned) {
        if (pinned_bytes < P.tables) return fail(HCC_ERR_INVALID, "batch launch: staging buffer too small");
    } else {
        staging.assign(P.tables, 0);
        host = staging.data();
    }
    std::memcpy(host, T.hs.data(), sizeof(EngScene) * T.hs.size());
    std::memcpy(host + (P.batches_off - P.scenes_off), T.hb.data(), sizeof(EngBatch) * T.hb.size());
    HCC_HIP(hipMemcpyAsync(ws + P.scenes_off, host, P.tables, hipMemcpyHostToDevice, stream));
    if (!pinned) HCC_HIP(hipStreamSynchronize(stream));
    const size_t zw = h.zero_words;
    k_zero<<<(unsigned)std::min<size_t>(2048, (zw + 255) / 256), 256, 0, stream>>>(h.zero, zw);
    const EngScene* dsc = (const EngScene*)(ws + P.scenes_off);
    const EngBatch* dbt = (const EngBatch*)(ws + P.batches_off);
    const uint32_t waves = o.waves ? o.waves : 8192u;
    const unsigned grid = std::max(1u, std::min(waves, h.total_items));
    const bool wide = (o.flags & HCC_TRACE_WIDE) != 0;
    const int lds = engine_stack_entries(o.stack);
#define HCC_ENGINE(KT, WD, SH)                                                                                    \
    k_engine<KT, WD, SH><<<grid, 64, 0, stream>>>(dsc, dbt, nb, h.total_items, h.total_tiles, h.queue, mode,   \
                                                  key_bits, h.passes, h.refill, h.slab)
#define HCC_ENGINE_K(KT)                                                                                          \
    if (!wide) HCC_ENGINE(KT, false, kEngShort);                                                                  \
    else if (lds == 0) HCC_ENGINE(KT, true, 0);                                                                   \
    else if (lds == kEngLds) HCC_ENGINE(KT, true, kEngLds);                                                       \
    else HCC_ENGINE(KT, true, kEngShort)
    if (key_bits <= 32) {
        HCC_ENGINE_K(uint32_t);
    } else {
        HCC_ENGINE_K(uint64_t);
    }
#undef HCC_ENGINE_K
#undef HCC_ENGINE
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

// ---- graph-launched groups (the request server's continuous mode)
//
// A slot owns a pinned staging buffer, a device table buffer of fixed capacity (header,
// scenes, batches) and a graph captured once: copy staging -> device tables, clear the
// group's counters (k_zero_hdr), run the engine (k_engine_hdr) on a fixed grid.  Launching a
// group = writing its tables into the slot's staging buffer + one hipGraphLaunch.  The slot
// stays with the group until the group's completion event has fired.
size_t graph_table_bytes(uint32_t max_batches) {
    return al(sizeof(EngHeader)) + al(sizeof(EngScene) * max_batches) + al(sizeof(EngBatch) * max_batches);
}

hcc_status graph_capture(uint32_t max_batches, uint32_t key_bits, const hcc_batch_opts& o, void* pinned,
                         void* d_tables, hipStream_t capture_stream, hipGraphExec_t* exec) {
    const size_t bytes = graph_table_bytes(max_batches);
    char* dt = (char*)d_tables;
    const EngHeader* dh = (const EngHeader*)dt;
    const EngScene* dsc = (const EngScene*)(dt + al(sizeof(EngHeader)));
    const EngBatch* dbt = (const EngBatch*)(dt + al(sizeof(EngHeader)) + al(sizeof(EngScene) * max_batches));
    const unsigned grid = o.waves ? o.waves : 8192u;
    const bool wide = (o.flags & HCC_TRACE_WIDE) != 0;
    const int lds = engine_stack_entries(o.stack);
    HCC_HIP(hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipMemcpyAsync(dt, pinned, bytes, hipMemcpyHostToDevice, capture_stream);
    if (e == hipSuccess) {
        k_zero_hdr<<<512, 256, 0, capture_stream>>>(dh);
#define HCC_ENGINE_HDR(KT, WD, SH) k_engine_hdr<KT, WD, SH><<<grid, 64, 0, capture_stream>>>(dh, dsc, dbt)
#define HCC_ENGINE_HDR_K(KT)                                                                                      \
    if (!wide) HCC_ENGINE_HDR(KT, false, kEngShort);                                                              \
    else if (lds == 0) HCC_ENGINE_HDR(KT, true, 0);                                                               \
    else if (lds == kEngLds) HCC_ENGINE_HDR(KT, true, kEngLds);                                                   \
    else HCC_ENGINE_HDR(KT, true, kEngShort)
        if (key_bits <= 32) {
            HCC_ENGINE_HDR_K(uint32_t);
        } else {
            HCC_ENGINE_HDR_K(uint64_t);
        }
#undef HCC_ENGINE_HDR_K
#undef HCC_ENGINE_HDR
        e = hipGetLastError();
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(capture_stream, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "engine graph capture");
    return HCC_OK;
}

// Write a group's tables into a slot's staging buffer (the workspace d_ws holds the group's
// counters and sort buffers) and launch the slot's graph.
hcc_status graph_launch(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                        const hcc_batch_opts& o, void* d_ws, size_t ws_bytes, uint32_t max_batches, void* pinned,
                        void* d_tables, hipGraphExec_t exec, hipStream_t stream) {
    if (nb > max_batches) return fail(HCC_ERR_INVALID, "graph launch: more batches than the slot holds");
    Tables T;
    hcc_status st = fill_tables(d, nb, mode, key_bits, o, d_ws, ws_bytes, T);
    if (st != HCC_OK) return st;
    // the scenes' and batches' addresses inside the slot's device table
    char* host = (char*)pinned;
    (void)d_tables;   // the slot's graph copies the staging buffer there
    const size_t soff = al(sizeof(EngHeader)), boff = soff + al(sizeof(EngScene) * max_batches);
    std::memcpy(host, &T.hdr, sizeof(EngHeader));
    std::memcpy(host + soff, T.hs.data(), sizeof(EngScene) * T.hs.size());
    std::memcpy(host + boff, T.hb.data(), sizeof(EngBatch) * T.hb.size());
    HCC_HIP(hipGraphLaunch(exec, stream));
    return HCC_OK;
}

// Distinct (bvh, cut) pairs of a batch list, the scene table fill_tables builds.
static uint32_t count_scenes(const hcc_batch_desc* d, uint32_t nb) {
    std::vector<std::pair<const hcc_bvh_s*, const hcc_cut_s*>> seen;
    for (uint32_t b = 0; b < nb; ++b) {
        const auto key = std::make_pair((const hcc_bvh_s*)d[b].bvh, (const hcc_cut_s*)d[b].cut);
        if (std::find(seen.begin(), seen.end(), key) == seen.end()) seen.push_back(key);
    }
    return (uint32_t)seen.size();
}

template <typename K>
__global__ void k_gather_keys(const K* __restrict__ keys, const uint32_t* __restrict__ perm, uint32_t n,
                              K* __restrict__ out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = keys[perm[i]];
}

// Batch b's final permutation and its keys in that order, as the last run on d_ws (with the
// same batch list, mode, key length and options) left them: for an engine batch the last sort
// pass's output buffers, for a direct launch its permutation and its keys gathered through it.
hcc_status batch_export(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                        const hcc_batch_opts& o, const void* d_ws, size_t ws_bytes, uint32_t b, uint32_t* d_perm,
                        void* d_sorted_keys, hipStream_t stream) {
    const uint32_t n = d[b].n;
    if (n == 0) return HCC_OK;
    const size_t ks = key_bits <= 32 ? 4 : 8;
    const char* ws = (const char*)d_ws;
    if (o.direct_min != 0 && n >= o.direct_min) {
        size_t off = al(plan_batches(d, nb, nb, mode, key_bits, 0).total);
        for (uint32_t i = 0; i < b; ++i)
            if (d[i].n >= o.direct_min) off += direct_bytes(d[i].n, mode, key_bits);
        if (off + direct_bytes(n, mode, key_bits) > ws_bytes) return fail(HCC_ERR_INVALID, "hcc_batch_export: workspace too small");
        const void* keys = ws + off;
        const uint32_t* pm = (const uint32_t*)(ws + off + al((size_t)n * ks));
        if (d_perm) HCC_HIP(hipMemcpyAsync(d_perm, pm, (size_t)n * 4, hipMemcpyDeviceToDevice, stream));
        if (d_sorted_keys) {
            const unsigned grid = std::min<unsigned>(4096u, (n + 255) / 256);
            if (ks == 4) k_gather_keys<uint32_t><<<grid, 256, 0, stream>>>((const uint32_t*)keys, pm, n, (uint32_t*)d_sorted_keys);
            else k_gather_keys<uint64_t><<<grid, 256, 0, stream>>>((const uint64_t*)keys, pm, n, (uint64_t*)d_sorted_keys);
            HCC_HIP(hipGetLastError());
        }
        return HCC_OK;
    }
    // engine batch: offsets within the plan of the list the engine launch received
    std::vector<hcc_batch_desc> list;
    uint32_t at = b;
    if (o.direct_min != 0) {
        for (uint32_t i = 0; i < nb; ++i) {
            if (d[i].n >= o.direct_min) continue;
            if (i == b) at = (uint32_t)list.size();
            list.push_back(d[i]);
        }
    } else {
        list.assign(d, d + nb);
    }
    const uint32_t nl = (uint32_t)list.size();
    const Plan P = plan_batches(list.data(), nl, count_scenes(list.data(), nl), mode, key_bits, 0);
    if (P.total > ws_bytes) return fail(HCC_ERR_INVALID, "hcc_batch_export: workspace too small");
    const uint32_t passes = (key_bits + 7) / 8;
    const bool in_a = ((passes - 1) & 1) != 0;
    const void* keys = ws + (in_a ? P.keys_a[at] : P.keys_b[at]);
    const void* vals = ws + (in_a ? P.vals_a[at] : P.vals_b[at]);
    if (d_perm) HCC_HIP(hipMemcpyAsync(d_perm, vals, (size_t)n * 4, hipMemcpyDeviceToDevice, stream));
    if (d_sorted_keys) HCC_HIP(hipMemcpyAsync(d_sorted_keys, keys, (size_t)n * ks, hipMemcpyDeviceToDevice, stream));
    return HCC_OK;
}

// The engine's error flag (word 1 of every workspace): nonzero when a bounded wait gave up.
hcc_status batch_check(const void* d_ws, hipStream_t stream, uint32_t* ok) {
    uint32_t flag = 0;
    HCC_HIP(hipMemcpyAsync(&flag, (const char*)d_ws + 4, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    HCC_HIP(hipStreamSynchronize(stream));
    *ok = flag == 0 ? 1u : 0u;
    return HCC_OK;
}

}  // namespace hcc

namespace hcc {
hcc_status batch_run(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits, const hcc_batch_opts& o,
                     void* d_ws, size_t ws_bytes, hipStream_t stream) {
    return batch_launch(d, nb, mode, key_bits, o, d_ws, ws_bytes, stream, nullptr, 0);
}
}  // namespace hcc
