// BVH traversal for gfx950 (the trace kernel of Section 5: it fetches the rays through
// the sorted indices, so reordered rays of one wavefront walk similar paths).
//
// One lane per ray, wavefront of 64 lanes.  Loop per lane: fetch the current internal
// node (one 64-byte load holding both child boxes), slab-test both children against
// [tmin, best t], test leaf children's triangles at once (one triangle per leaf),
// descend into the nearer hit child and push the farther one, pop when nothing is hit.
// Stack placement is a template parameter (LDS, private scratch, or LDS for the first
// entries and scratch beyond).  Results are written at the original ray index.
//
// Closest hit keeps the smallest (t, triangle index) pair, which makes the answer
// independent of traversal order; any hit stops at the first triangle in the segment.
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "hcc_internal.h"

namespace hcc {
namespace {

constexpr int kShortDepth = 16;

template <int kStack, int kBlock>
struct Stack;

template <int kBlock>
struct Stack<HCC_STACK_LDS, kBlock> {
    uint32_t* s;
    __device__ void init(uint32_t* lds) { s = lds + threadIdx.x; }
    __device__ void push(uint32_t sp, uint32_t x) { s[sp * kBlock] = x; }
    __device__ uint32_t pop(uint32_t sp) { return s[sp * kBlock]; }
};

template <int kBlock>
struct Stack<HCC_STACK_SCRATCH, kBlock> {
    uint32_t s[kStackDepth];
    __device__ void init(uint32_t*) {}
    __device__ void push(uint32_t sp, uint32_t x) { s[sp] = x; }
    __device__ uint32_t pop(uint32_t sp) { return s[sp]; }
};

template <int kBlock>
struct Stack<HCC_STACK_SHORT, kBlock> {
    uint32_t* s;
    uint32_t deep[kStackDepth - kShortDepth];
    __device__ void init(uint32_t* lds) { s = lds + threadIdx.x; }
    __device__ void push(uint32_t sp, uint32_t x) {
        if (sp < kShortDepth) s[sp * kBlock] = x;
        else deep[sp - kShortDepth] = x;
    }
    __device__ uint32_t pop(uint32_t sp) { return sp < kShortDepth ? s[sp * kBlock] : deep[sp - kShortDepth]; }
};

template <int kStack>
constexpr int lds_entries() {
    return kStack == HCC_STACK_LDS ? kStackDepth : (kStack == HCC_STACK_SHORT ? kShortDepth : 1);
}

// Number of distinct values of x among the active lanes (measurement only).
__device__ __forceinline__ uint32_t wave_distinct(uint32_t x) {
    uint64_t rem = __ballot(1);
    uint32_t count = 0;
    while (rem) {
        const int src = __ffsll((unsigned long long)rem) - 1;
        const uint32_t id = __shfl(x, src, 64);
        rem &= ~__ballot(x == id);
        ++count;
    }
    return count;
}

__device__ __forceinline__ bool first_active_lane() {
    const uint64_t act = __ballot(1);
    return (int)__lane_id() == __ffsll((unsigned long long)act) - 1;
}

template <bool kClosest, int kStack, int kBlock, bool kStats>
__global__ __launch_bounds__(kBlock) void k_trace(const Node* __restrict__ nodes, const Tri* __restrict__ tris,
                                                  uint32_t n_int, const float4* __restrict__ rays,
                                                  const uint32_t* __restrict__ perm, uint32_t n,
                                                  float4* __restrict__ hits, uint8_t* __restrict__ occ,
                                                  uint32_t remap, uint32_t* __restrict__ cnt_nodes,
                                                  uint32_t* __restrict__ cnt_tris, uint32_t* wave_nodes,
                                                  uint32_t* wave_tris) {
    __shared__ uint32_t s_stack[lds_entries<kStack>() * kBlock];
    const uint32_t blk = remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t k = blk * kBlock + threadIdx.x;
    if (k >= n) return;
    const uint32_t rid = perm ? perm[k] : k;
    if (rid >= n) return;   // a permutation entry out of range is skipped, never dereferenced
    const float4 ra = rays[2 * (size_t)rid];
    const float4 rb = rays[2 * (size_t)rid + 1];
    const float ox = ra.x, oy = ra.y, oz = ra.z, tmin = ra.w;
    const float dx = rb.x, dy = rb.y, dz = rb.z, tmax = rb.w;
    const float ix = 1.0f / dx, iy = 1.0f / dy, iz = 1.0f / dz;
    float best_t = tmax, best_u = 0.0f, best_v = 0.0f;
    uint32_t best_prim = kMissPrim;
    bool found = false;
    uint32_t n_nodes = 0, n_tris = 0;
    const uint32_t wave = k >> 6;

    auto test_leaf = [&](uint32_t leaf) {
        const Tri tr = tris[leaf];
        const uint32_t prim = __float_as_uint(tr.r.y);
        float t, u, v;
        if (kStats) ++n_tris;
        if (tri_test(tr, ox, oy, oz, dx, dy, dz, tmin, tmax, t, u, v)) {
            if (!kClosest) {
                found = true;
            } else if (t < best_t || (t == best_t && prim < best_prim)) {
                best_t = t;
                best_u = u;
                best_v = v;
                best_prim = prim;
                found = true;
            }
        }
    };

    if (n_int == 0) {
        test_leaf(0);
        if (kStats && first_active_lane()) atomicAdd(wave_tris + wave, 1u);
    } else {
        Stack<kStack, kBlock> st;
        st.init(s_stack);
        uint32_t sp = 0;
        uint32_t node = 0;
        // One traversal step: fetch `node`, test its children's boxes and the triangles of hit
        // leaf children, then descend, pop, or end the traversal (false).
        auto step = [&]() -> bool {
            if (kStats) {
                ++n_nodes;
                const uint32_t dn = wave_distinct(node);
                if (first_active_lane()) atomicAdd(wave_nodes + wave, dn);
            }
            const Node nd = nodes[node];
            const float lim = kClosest ? best_t : tmax;
            float tn0, tn1;
            bool h0 = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, tn0);
            bool h1 = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, tn1);
            const uint32_t c0 = nd.d.x, c1 = nd.d.y;
            const bool leaf0 = h0 && c0 >= n_int;
            const bool leaf1 = h1 && c1 >= n_int;
            if (kStats) {
                const uint32_t t0 = wave_distinct(leaf0 ? c0 : 0xFFFFFFFFu) - (__ballot(!leaf0) != 0 ? 1u : 0u);
                const uint32_t t1 = wave_distinct(leaf1 ? c1 : 0xFFFFFFFFu) - (__ballot(!leaf1) != 0 ? 1u : 0u);
                if (first_active_lane()) atomicAdd(wave_tris + wave, t0 + t1);
            }
            if (leaf0) test_leaf(c0 - n_int);
            if (leaf1) test_leaf(c1 - n_int);
            if (!kClosest && found) return false;
            h0 = h0 && !leaf0;
            h1 = h1 && !leaf1;
            if (h0 && h1) {
                const bool near1 = tn1 < tn0;
                st.push(sp, near1 ? c0 : c1);
                ++sp;
                node = near1 ? c1 : c0;
            } else if (h0) {
                node = c0;
            } else if (h1) {
                node = c1;
            } else {
                if (sp == 0) return false;
                --sp;
                node = st.pop(sp);
            }
            return true;
        };
        if (kStats) {
            // Counting launch: every lane that is still traversing takes exactly one step per
            // iteration of a wavefront-uniform loop, so iteration s holds each lane's s-th step
            // (lockstep).  Left to itself the compiler nests the descend path in an inner loop
            // (lanes that pop wait while the others keep descending), which would make the
            // per-iteration counts depend on that schedule.
            bool active = true;
            while (__ballot(active) != 0) {
                if (active) active = step();
            }
        } else {
            while (step()) {
            }
        }
    }
    if (kClosest) {
        hits[rid] = make_float4(found ? best_t : INFINITY, __uint_as_float(found ? best_prim : kMissPrim),
                                found ? best_u : 0.0f, found ? best_v : 0.0f);
    } else {
        occ[rid] = found ? 1 : 0;
    }
    if (kStats) {
        if (cnt_nodes) cnt_nodes[rid] = n_nodes;
        if (cnt_tris) cnt_tris[rid] = n_tris;
    }
}

// Distinct values of x among the lanes with `on` set; every lane gets the count.  Called
// with the whole wavefront active (measurement only).
__device__ __forceinline__ uint32_t wave_distinct_on(uint32_t x, bool on) {
    uint64_t rem = __ballot(on);
    uint32_t count = 0;
    while (rem) {
        const int src = __ffsll((unsigned long long)rem) - 1;
        const uint32_t id = __shfl(x, src, 64);
        rem &= ~__ballot(on && x == id);
        ++count;
    }
    return count;
}

// Compare-exchange by selects (no branch: a branch per exchange costs more than the four
// selects in a wavefront whose lanes disagree).
__device__ __forceinline__ void cswap(float& ka, uint32_t& ia, float& kb, uint32_t& ib) {
    const bool sw = kb < ka;
    const float k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const uint32_t i0 = sw ? ib : ia, i1 = sw ? ia : ib;
    ka = k0;
    kb = k1;
    ia = i0;
    ib = i1;
}

__device__ __forceinline__ uint64_t lanes_below() {
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

// Chunks of a persistent launch: it deals out the sorted positions in chunks of `chunk`
// consecutive ones.  With a queue slot a wavefront takes the next chunk from a device counter
// whenever its own runs out, so wavefronts that drew cheap rays take more chunks and all of them
// finish together; without one (counting launches, launches captured into a graph, streams
// beyond the slots) wavefront w takes chunks w, w + grid, w + 2 grid, ...  A slot is 128 bytes
// per stream that launches persistent traces, claimed on the stream's first launch: word 0 is
// the number of chunks taken, word 1 the number of wavefronts done; the launch's last wavefront
// puts both back to 0, so a slot reads zero whenever no launch of its stream runs (launches on
// one stream never overlap).
//
// Spread dealing (HCC_TRACE_SPREAD, with a queue slot): take t goes to chunk (t mod S) Q + t / S
// over an S x Q arrangement of the chunks (S = 64), skipping the positions past the last chunk,
// so that the wavefronts running at one time hold chunks from 64 parts of the order instead of
// one stretch of it.  Each chunk is still a run of consecutive positions; a sorted order's
// neighbouring rays stay together in a wavefront while the device as a whole works on many
// keys at once.  (Giving each XCD a contiguous eighth of the chunks instead, the opposite
// arrangement, was measured 10-13% slower on every order of the frame workload's rays.)
constexpr uint32_t kQueueSlots = 256, kQueueWords = 32, kNoQueue = 0xFFFFFFFFu;
constexpr uint32_t kSpread = 64;
__device__ uint32_t g_chunk_queue[kQueueSlots * kQueueWords];

struct Chunks {
    uint32_t* q;
    uint32_t n, chunk, nchunks, cidx, next, end;
    bool spread;
    // wavefront-uniform calls only (every lane of the wavefront active).  deal: bit 0 = XCD
    // remap of the static order, bit 1 = spread dealing from the queue
    __device__ void init(uint32_t slot, uint32_t n_, uint32_t chunk_, uint32_t deal) {
        q = slot == kNoQueue ? nullptr : g_chunk_queue + (size_t)slot * kQueueWords;
        n = n_;
        chunk = chunk_;
        nchunks = (n + chunk - 1) / chunk;
        spread = q && (deal & 2u);
        // static order with remap: the wavefronts the hardware deals to one XCD start on
        // consecutive chunks
        cidx = q ? take() : ((deal & 1u) ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x);
        set();
    }
    __device__ uint32_t take() {
        uint32_t c = nchunks;
        if (__lane_id() == 0) {
            if (!spread) {
                c = atomicAdd(q, 1u);
            } else {
                const uint32_t rows = (nchunks + kSpread - 1) / kSpread;
                // at most kSpread - 1 takes land past the last chunk, so this loop ends
                while (true) {
                    const uint32_t t = atomicAdd(q, 1u);
                    if (t >= kSpread * rows) break;
                    const uint32_t m = (t % kSpread) * rows + t / kSpread;
                    if (m < nchunks) {
                        c = m;
                        break;
                    }
                }
            }
        }
        return __shfl(c, 0);
    }
    __device__ void set() {
        next = cidx < nchunks ? cidx * chunk : n;
        end = cidx < nchunks ? min(next + chunk, n) : n;
    }
    // the wavefront's next chunk, once the current one is dealt out (chunks are never empty)
    __device__ void advance() {
        if (next < end || cidx >= nchunks) return;
        cidx = q ? take() : cidx + gridDim.x;
        set();
    }
    __device__ void finish() {
        if (q && __lane_id() == 0 && atomicAdd(q + 1, 1u) == gridDim.x - 1) {
            atomicExch(q, 0u);
            atomicExch(q + 1, 0u);
        }
    }
};

// Persistent wavefronts (one wavefront per block).  Wavefront b owns chunks b, b + grid,
// b + 2 grid, ... of the trace order; whenever at least 'refill' of its lanes are idle it
// hands them the next rays of its current chunk.  Lanes whose ray finished early therefore
// pick up new work instead of idling until the wavefront's slowest ray completes, and the
// rays in flight in one wavefront stay neighbours in the (sorted) order.
//
// Leaf triangles are not tested inside the node step: a lane that meets leaves records up
// to two of them and pauses; the wavefront runs the triangle tests as one batch once at
// least half of its busy lanes have some pending (or no lane can step), so the triangle
// code runs with most lanes active instead of in a branch taken by a few.  Every wave-level
// decision is taken on ballots (uniform values); the loop ends once the wavefront's chunks
// are exhausted and all lanes are idle.
template <bool kClosest, int kStack, bool kSpec, bool kStats>
__global__ __launch_bounds__(64) void k_trace_persistent(const Node* __restrict__ nodes, const Tri* __restrict__ tris,
                                                         uint32_t n_int, const float4* __restrict__ rays,
                                                         const uint32_t* __restrict__ perm, uint32_t n,
                                                         float4* __restrict__ hits, uint8_t* __restrict__ occ,
                                                         uint32_t refill, uint32_t chunk, uint32_t deal,
                                                         uint32_t qslot, unsigned long long* __restrict__ counts) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    __shared__ uint32_t s_stack[lds_entries<kStack>() * 64];
    Chunks ch;
    ch.init(qslot, n, chunk, deal);
    const uint64_t below = lanes_below();
    Stack<kStack, 64> st;
    st.init(s_stack);
    bool has = false;
    uint32_t rid = 0, node = kNone, sp = 0, best_prim = kMissPrim;
    uint32_t pend0 = kNone, pend1 = kNone, pend2 = kNone;   // postponed leaves (triangle slots)
    float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, ix = 0, iy = 0, iz = 0, tmin = 0, tmax = 0;
    float best_t = 0, best_u = 0, best_v = 0;
    bool found = false;
    uint32_t c_nodes = 0, c_tris = 0;

    auto test_tri = [&](uint32_t slot) {
        const Tri tr = tris[slot];
        const uint32_t prim = __float_as_uint(tr.r.y);
        float t, u, v;
        if (tri_test(tr, ox, oy, oz, dx, dy, dz, tmin, tmax, t, u, v)) {
            if (!kClosest) {
                found = true;
            } else if (t < best_t || (t == best_t && prim < best_prim)) {
                best_t = t; best_u = u; best_v = v; best_prim = prim;
                found = true;
            }
        }
    };

    while (true) {
        // ---- refill idle lanes from the current chunk
        const uint64_t idle = __ballot(!has);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (nidle >= refill) {
            ch.advance();
            if (ch.next < ch.end) {
                const uint32_t k = ch.next + (uint32_t)__popcll(idle & below);
                if (!has && k < ch.end) {
                    rid = perm ? perm[k] : k;
                    if (rid < n) {
                        const float4 ra = rays[2 * (size_t)rid];
                        const float4 rb = rays[2 * (size_t)rid + 1];
                        ox = ra.x; oy = ra.y; oz = ra.z; tmin = ra.w;
                        dx = rb.x; dy = rb.y; dz = rb.z; tmax = rb.w;
                        ix = 1.0f / dx; iy = 1.0f / dy; iz = 1.0f / dz;
                        best_t = tmax; best_u = 0.0f; best_v = 0.0f;
                        best_prim = kMissPrim;
                        found = false;
                        node = 0;
                        sp = 0;
                        pend0 = pend1 = pend2 = kNone;
                        has = true;
                    }
                }
                ch.next = min(ch.next + nidle, ch.end);
            } else if (nidle == 64) {
                break;
            }
        }

        // ---- one node step for lanes with a node and room for two more postponed leaves
        // (kSpec: a lane keeps descending while it holds one postponed leaf)
        const bool step = has && node != kNone && (kSpec ? pend1 == kNone : pend0 == kNone);
        if (kStats) c_nodes += wave_distinct_on(node, step);
        if (step) {
            const Node nd = nodes[node];
            const float lim = kClosest ? best_t : tmax;
            float tn0, tn1;
            bool h0 = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, tn0);
            bool h1 = slab(ox, oy, oz, ix, iy, iz, tmin, lim, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, tn1);
            const uint32_t c0 = nd.d.x, c1 = nd.d.y;
            const bool leaf0 = h0 && c0 >= n_int;
            const bool leaf1 = h1 && c1 >= n_int;
            // append the hit leaves to the postponed list
            if (leaf0 || leaf1) {
                const uint32_t a = leaf0 ? c0 - n_int : c1 - n_int;
                const uint32_t b = (leaf0 && leaf1) ? c1 - n_int : kNone;
                if (pend0 == kNone) {
                    pend0 = a;
                    pend1 = b;
                } else {
                    pend1 = a;
                    pend2 = b;
                }
            }
            h0 = h0 && !leaf0;
            h1 = h1 && !leaf1;
            if (h0 && h1) {
                const bool near1 = tn1 < tn0;
                st.push(sp, near1 ? c0 : c1);
                ++sp;
                node = near1 ? c1 : c0;
            } else if (h0) {
                node = c0;
            } else if (h1) {
                node = c1;
            } else if (sp == 0) {
                node = kNone;
            } else {
                --sp;
                node = st.pop(sp);
            }
        }

        // ---- batched leaf tests
        const uint64_t busy = __ballot(has);
        const bool can_step = has && node != kNone && (kSpec ? pend1 == kNone : pend0 == kNone);
        const uint64_t waiting = __ballot(has && pend0 != kNone && !can_step);
        const uint64_t stepping = __ballot(can_step);
        if (waiting != 0 && (2 * __popcll(waiting) >= __popcll(busy) || stepping == 0)) {
            if (kStats) {
                const bool mine = has && pend0 != kNone;
                c_tris += wave_distinct_on(pend0, mine);
                c_tris += wave_distinct_on(pend1, mine && pend1 != kNone);
                c_tris += wave_distinct_on(pend2, kSpec && mine && pend2 != kNone);
            }
            if (has && pend0 != kNone) {
                test_tri(pend0);
                if (pend1 != kNone && (kClosest || !found)) test_tri(pend1);
                if (kSpec && pend2 != kNone && (kClosest || !found)) test_tri(pend2);
                pend0 = pend1 = pend2 = kNone;
                if (!kClosest && found) node = kNone;
            }
        }

        // ---- finished rays
        if (has && node == kNone && pend0 == kNone) {
            if (kClosest)
                hits[rid] = make_float4(found ? best_t : INFINITY, __uint_as_float(found ? best_prim : kMissPrim),
                                        found ? best_u : 0.0f, found ? best_v : 0.0f);
            else
                occ[rid] = found ? 1 : 0;
            has = false;
        }
    }
    if (kStats && __lane_id() == 0) {
        atomicAdd(counts, (unsigned long long)c_nodes);
        atomicAdd(counts + 1, (unsigned long long)c_tris);
    }
    ch.finish();
}

// Persistent wavefronts over the 4-wide nodes (same refill and batched-leaf scheme as
// k_trace_persistent).  A node step tests the four child boxes, records the hit leaf slots of
// the node as pending (node index + 4-bit mask), orders the hit internal children by entry
// distance with a 5-comparator network, descends into the nearest and pushes the others
// farthest first.  kStats: counts, per lockstep iteration, the distinct 4-wide nodes fetched
// by the stepping lanes and the distinct triangles fetched by a leaf batch (summed over the
// wavefront into counts[0] and counts[1]).
// Per-lane stack of the 4-wide traversal: the first entries in LDS (lane-interleaved, conflict
// free), deeper ones in scratch; or all of it in scratch.
// kLds = 0: all in scratch; otherwise the number of entries kept in LDS (16 for
// HCC_STACK_SHORT: with the 1 KB of pending-leaf refs that is 5 KB per wavefront, so the LDS
// of a CU holds exactly its 32 wavefronts; 24 for HCC_STACK_LDS).
template <int kLds>
struct WideStack {
    uint32_t* lds;
    uint32_t deep[kWideStack - kLds];
    __device__ void init(uint32_t* l) { lds = l + __lane_id(); }
    __device__ void push(uint32_t sp, uint32_t x) {
        if (sp < (uint32_t)kLds) lds[sp * 64] = x;
        else deep[sp - kLds] = x;
    }
    __device__ uint32_t pop(uint32_t sp) { return sp < (uint32_t)kLds ? lds[sp * 64] : deep[sp - kLds]; }
    // entries known to sit in the LDS part (sp < kLds)
    __device__ void push_lds(uint32_t sp, uint32_t x) { lds[sp * 64] = x; }
    __device__ uint32_t pop_lds(uint32_t sp) { return lds[sp * 64]; }
};

template <>
struct WideStack<0> {
    uint32_t s[kWideStack];
    __device__ void init(uint32_t*) {}
    __device__ void push(uint32_t sp, uint32_t x) { s[sp] = x; }
    __device__ uint32_t pop(uint32_t sp) { return s[sp]; }
    __device__ void push_lds(uint32_t sp, uint32_t x) { s[sp] = x; }
    __device__ uint32_t pop_lds(uint32_t sp) { return s[sp]; }
};

template <bool kClosest, bool kStats, int kLds>
__global__ __launch_bounds__(64) void k_trace_wide(const Node4* __restrict__ wn, const Node4Q* __restrict__ qn,
                                                   const Tri* __restrict__ tris,
                                                   uint32_t n_int, const float4* __restrict__ rays,
                                                   const uint32_t* __restrict__ perm, uint32_t n,
                                                   float4* __restrict__ hits, uint8_t* __restrict__ occ,
                                                   uint32_t refill, uint32_t chunk, uint32_t deal, uint32_t slab,
                                                   uint32_t qslot, unsigned long long* __restrict__ counts) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    Chunks ch;
    ch.init(qslot, n, chunk, deal);
    const uint64_t below = lanes_below();
    __shared__ uint32_t s_stack[kLds ? kLds * 64 : 1];
    __shared__ uint4 s_leaf[64];   // refs of the node whose hit leaves a lane has pending
    WideStack<kLds> stack;
    stack.init(s_stack);
    bool has = false;
    uint32_t rid = 0, node = kNone, sp = 0, best_prim = kMissPrim;
    uint32_t pmask = 0;
    float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, ix = 0, iy = 0, iz = 0, tmin = 0, tmax = 0;
    float best_t = 0, best_u = 0, best_v = 0;
    WideRay wr{0, 0, 0, false};
    const bool fast_nodes = !slab && n_int <= kWideFastNodes;
    bool found = false;
    uint32_t c_nodes = 0, c_tris = 0;

    auto test_tri = [&](uint32_t slot) {
        const Tri tr = tris[slot];
        const uint32_t prim = __float_as_uint(tr.r.y);
        float t, u, v;
        const bool hit = tri_test(tr, ox, oy, oz, dx, dy, dz, tmin, tmax, t, u, v);
        if (!kClosest) {
            found = found || hit;
        } else {
            // nearer hit, or an equally near one of a smaller triangle id: taken by selects
            const bool take = hit && (t < best_t || (t == best_t && prim < best_prim));
            best_t = take ? t : best_t;
            best_u = take ? u : best_u;
            best_v = take ? v : best_v;
            best_prim = take ? prim : best_prim;
            found = found || take;
        }
    };

    while (true) {
        // ---- refill idle lanes from the current chunk
        const uint64_t idle = __ballot(!has);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (nidle >= refill) {
            ch.advance();
            if (ch.next < ch.end) {
                const uint32_t k = ch.next + (uint32_t)__popcll(idle & below);
                if (!has && k < ch.end) {
                    rid = perm ? perm[k] : k;
                    if (rid < n) {
                        const float4 ra = rays[2 * (size_t)rid];
                        const float4 rb = rays[2 * (size_t)rid + 1];
                        ox = ra.x; oy = ra.y; oz = ra.z; tmin = ra.w;
                        dx = rb.x; dy = rb.y; dz = rb.z; tmax = rb.w;
                        ix = 1.0f / dx; iy = 1.0f / dy; iz = 1.0f / dz;
                        wr = wide_ray(ox, oy, oz, ix, iy, iz);
                        best_t = tmax; best_u = 0.0f; best_v = 0.0f;
                        best_prim = kMissPrim;
                        found = false;
                        node = 0;
                        sp = 0;
                        pmask = 0;
                        has = true;
                    }
                }
                ch.next = min(ch.next + nidle, ch.end);
            } else if (nidle == 64) {
                break;
            }
        }

        // ---- one 4-wide node step for lanes with a node and no pending leaves
        const bool step = has && node != kNone && pmask == 0;
        if (kStats) c_nodes += wave_distinct_on(node, step);
        // the whole node step is specialised on the (wavefront-uniform) form of the child test:
        // 0 slab test, 1 selected planes, 2 / 3 the same on the quantised nodes
        auto node_step = [&](auto kind) {
            uint4 r;
            bool hh[4];
            float tt[4];
            constexpr int kKind = decltype(kind)::value;
            if constexpr (kKind >= 2)
                wide_test_q<kKind == 3>(qn, node, wr, ox, oy, oz, ix, iy, iz, tmin, kClosest ? best_t : tmax, r, hh, tt);
            else
                wide_test<kKind == 1>(wn, node, wr, ox, oy, oz, ix, iy, iz, tmin, kClosest ? best_t : tmax, r, hh, tt);
            s_leaf[__lane_id()] = r;   // read back only if this step leaves hit leaves pending
            const bool h0 = hh[0], h1 = hh[1], h2 = hh[2], h3 = hh[3];
            const float t0 = tt[0], t1 = tt[1], t2 = tt[2], t3 = tt[3];
            const bool l0 = h0 && (r.x & kWideLeaf), l1 = h1 && (r.y & kWideLeaf);
            const bool l2 = h2 && (r.z & kWideLeaf), l3 = h3 && (r.w & kWideLeaf);
            const uint32_t lm = (l0 ? 1u : 0u) | (l1 ? 2u : 0u) | (l2 ? 4u : 0u) | (l3 ? 8u : 0u);
            pmask = lm;   // a stepping lane has none pending
            // hit internal children, nearest first (a missed or leaf slot sorts last as kNone)
            float k0 = (h0 && !l0) ? t0 : INFINITY, k1 = (h1 && !l1) ? t1 : INFINITY;
            float k2 = (h2 && !l2) ? t2 : INFINITY, k3 = (h3 && !l3) ? t3 : INFINITY;
            uint32_t i0 = (h0 && !l0) ? r.x : kNone, i1 = (h1 && !l1) ? r.y : kNone;
            uint32_t i2 = (h2 && !l2) ? r.z : kNone, i3 = (h3 && !l3) ? r.w : kNone;
            cswap(k0, i0, k1, i1);
            cswap(k2, i2, k3, i3);
            cswap(k0, i0, k2, i2);
            cswap(k1, i1, k3, i3);
            cswap(k1, i1, k2, i2);
            if (kLds > 0 && __ballot(sp + 3 > (uint32_t)kLds) == 0) {
                // every stepping lane has room for three more entries in the LDS part of its
                // stack: no per-entry choice between LDS and scratch
                // without branches: each candidate is written at the top and kept if valid (the
                // three slots above sp exist), and the top is read back for the pop
                stack.push_lds(sp, i3);
                sp += i3 < n_int ? 1u : 0u;
                stack.push_lds(sp, i2);
                sp += i2 < n_int ? 1u : 0u;
                stack.push_lds(sp, i1);
                sp += i1 < n_int ? 1u : 0u;
                const uint32_t top = stack.pop_lds(sp > 0 ? sp - 1 : 0);
                const bool descend = i0 < n_int;
                node = descend ? i0 : (sp == 0 ? kNone : top);
                sp -= (!descend && sp > 0) ? 1u : 0u;
            } else {
                if (i3 < n_int && sp < kWideStack) stack.push(sp++, i3);
                if (i2 < n_int && sp < kWideStack) stack.push(sp++, i2);
                if (i1 < n_int && sp < kWideStack) stack.push(sp++, i1);
                if (i0 < n_int) {
                    node = i0;
                } else if (sp == 0) {
                    node = kNone;
                } else {
                    node = stack.pop(--sp);
                }
            }
        };
        if (qn) {
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

        // ---- batched leaf tests
        const uint64_t busy = __ballot(has);
        const bool can_step = has && node != kNone && pmask == 0;
        const uint64_t waiting = __ballot(has && pmask != 0);
        const uint64_t stepping = __ballot(can_step);
        // a leaf batch once a third of the busy lanes wait on one (measured: a half or two thirds
        // leave too many lanes idle in the node steps; a quarter is no better, fewer is worse)
        if (waiting != 0 && (3 * __popcll(waiting) >= __popcll(busy) || stepping == 0)) {
            const bool mine = has && pmask != 0;
            uint4 r = make_uint4(kNone, kNone, kNone, kNone);
            if (mine) r = s_leaf[__lane_id()];
            if (kStats) {
                c_tris += wave_distinct_on(r.x, mine && (pmask & 1u));
                c_tris += wave_distinct_on(r.y, mine && (pmask & 2u));
                c_tris += wave_distinct_on(r.z, mine && (pmask & 4u));
                c_tris += wave_distinct_on(r.w, mine && (pmask & 8u));
            }
            // each lane tests its pending triangles lowest slot first, one per round: the
            // wavefront runs as many rounds as its fullest lane has triangles, not one per slot
            uint32_t left = mine ? pmask : 0u;
            while (__ballot(left != 0) != 0) {
                if (left != 0) {
                    const uint32_t j = __builtin_ctz(left);
                    left &= left - 1u;
                    const uint32_t ref = j == 0 ? r.x : (j == 1 ? r.y : (j == 2 ? r.z : r.w));
                    test_tri(ref & ~kWideLeaf);
                    if (!kClosest && found) left = 0;
                }
            }
            if (mine) {
                pmask = 0;
                if (!kClosest && found) node = kNone;
            }
        }

        // ---- finished rays
        if (has && node == kNone && pmask == 0) {
            if (kClosest)
                hits[rid] = make_float4(found ? best_t : INFINITY, __uint_as_float(found ? best_prim : kMissPrim),
                                        found ? best_u : 0.0f, found ? best_v : 0.0f);
            else
                occ[rid] = found ? 1 : 0;
            has = false;
        }
    }
    if (kStats && __lane_id() == 0) {
        atomicAdd(counts, (unsigned long long)c_nodes);
        atomicAdd(counts + 1, (unsigned long long)c_tris);
    }
    ch.finish();
}

// Wavefront packets over the 4-wide nodes.  A wavefront takes 64 consecutive rays of the trace
// order (one chunk of 64 from the stream's counter) and walks the tree once for all of them: the
// node of a step is the same on every lane, so it is fetched by one scalar load shared by the
// wavefront, and the vector memory path (which bounds the per-lane traversal above) carries only
// the rays and the results.  Each lane tests its own ray against the node's four child boxes
// (culling with its own best distance); a child is visited when some lane's test passes, the
// triangles of hit leaves are tested at once by the lanes that hit them, and the hit internal
// children are taken in the entry order of the lowest lane that hits one of them (descend into
// the first, push the others last first).  The stack is shared by the wavefront: entry e sits in
// lane e mod 64 of register e / 64, so a push writes one lane and a pop reads one.  An any-hit
// packet ends once every lane has found a hit.  A packet costs one step per node of the union of
// its rays' traversals: close to one ray's for coherent rays, many times that for incoherent ones.
struct PacketStack {
    uint32_t r0 = 0, r1 = 0, r2 = 0;   // kWideStack = 3 x 64 entries
    __device__ void push(uint32_t sp, uint32_t x) {
        const bool here = __lane_id() == (sp & 63u);
        const uint32_t g = sp >> 6;
        if (g == 0) r0 = here ? x : r0;
        else if (g == 1) r1 = here ? x : r1;
        else r2 = here ? x : r2;
    }
    __device__ uint32_t pop(uint32_t sp) const {
        const uint32_t l = sp & 63u, g = sp >> 6;
        return __builtin_amdgcn_readlane(g == 0 ? r0 : (g == 1 ? r1 : r2), l);
    }
};
static_assert(kWideStack == 3 * 64, "the packet stack holds three registers of 64 entries");

// Order-preserving map of a float to an unsigned key (negative values flipped).
__device__ __forceinline__ uint32_t ordered_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ void cswap_u(uint32_t& ka, uint32_t& ia, uint32_t& kb, uint32_t& ib) {
    const bool sw = kb < ka;
    const uint32_t k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const uint32_t i0 = sw ? ib : ia, i1 = sw ? ia : ib;
    ka = k0;
    kb = k1;
    ia = i0;
    ib = i1;
}

// tri_test without its early exits: every lane of a packet runs the whole test anyway, and the
// exits cost scalar exec-mask work per triangle.  Same operations in the same order, so the same
// (t, u, v) wherever a hit is reported.
__device__ __forceinline__ bool tri_test_flat(const Tri& tr, float ox, float oy, float oz, float dx, float dy,
                                              float dz, float tmin, float tmax, float& t, float& u, float& v) {
    const float v0x = tr.p.x, v0y = tr.p.y, v0z = tr.p.z;
    const float e1x = tr.p.w, e1y = tr.q.x, e1z = tr.q.y;
    const float e2x = tr.q.z, e2y = tr.q.w, e2z = tr.r.x;
    const float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const float det = (e1x * px + e1y * py) + e1z * pz;
    const float sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
    const float inv = 1.0f / det;
    u = ((sx * px + sy * py) + sz * pz) * inv;
    const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    v = ((dx * qx + dy * qy) + dz * qz) * inv;
    t = ((e2x * qx + e2y * qy) + e2z * qz) * inv;
    return (det != 0.0f) & (u >= 0.0f) & (u <= 1.0f) & (v >= 0.0f) & (u + v <= 1.0f) & (t > tmin) & (t < tmax);
}

template <bool kClosest>
__global__ __launch_bounds__(64) void k_trace_packet(const Node4* __restrict__ wn, const Node4Q* __restrict__ qn,
                                                     const Tri* __restrict__ tris, uint32_t n_int,
                                                     const float4* __restrict__ rays, const uint32_t* __restrict__ perm,
                                                     uint32_t n, float4* __restrict__ hits, uint8_t* __restrict__ occ,
                                                     uint32_t deal, uint32_t slab, uint32_t qslot) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    Chunks ch;
    ch.init(qslot, n, 64u, deal);
    const uint32_t lane = __lane_id();
    while (true) {
        ch.advance();
        if (ch.next >= ch.end) break;
        const uint32_t k = ch.next + lane;
        bool valid = k < ch.end;
        ch.next = ch.end;
        uint32_t rid = 0;
        if (valid) {
            rid = perm ? perm[k] : k;
            valid = rid < n;
        }
        float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 0, tmin = 0, tmax = 0;
        if (valid) {
            const float4 ra = rays[2 * (size_t)rid];
            const float4 rb = rays[2 * (size_t)rid + 1];
            ox = ra.x; oy = ra.y; oz = ra.z; tmin = ra.w;
            dx = rb.x; dy = rb.y; dz = rb.z; tmax = rb.w;
        }
        const float ix = 1.0f / dx, iy = 1.0f / dy, iz = 1.0f / dz;
        const WideRay wr = wide_ray(ox, oy, oz, ix, iy, iz);
        float best_t = tmax, best_u = 0.0f, best_v = 0.0f;
        uint32_t best_prim = kMissPrim;
        bool found = false;

        // on the lanes with `on` set (no branch: the whole wavefront runs the test)
        auto test_tri = [&](const Tri& tr, bool on) {
            const uint32_t prim = __float_as_uint(tr.r.y);
            float t, u, v;
            const bool hit = on & tri_test_flat(tr, ox, oy, oz, dx, dy, dz, tmin, tmax, t, u, v);
            if (!kClosest) {
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

        // the walk, specialised on the (packet-uniform) form of the child test: 0 slab test / 1
        // selected planes on the exact nodes, 2 slab test / 3 selected planes on the quantised nodes.
        // w: the lane's own plane choice, or one shared by the packet (every ray with the same
        // direction signs), which makes the choice a scalar one and the exact planes scalar loads
        auto walk = [&](auto kind, const WideRay& w) {
            constexpr int kKind = decltype(kind)::value;
            PacketStack st;
            uint32_t sp = 0, node = 0;
            while (true) {
                node = __builtin_amdgcn_readfirstlane(node);
                const bool alive = valid && (kClosest || !found);
                if (!kClosest && __ballot(alive) == 0) break;
                uint4 r;
                bool hh[4];
                float tt[4];
                if constexpr (kKind >= 2)
                    wide_test_q<kKind == 3>(qn, node, w, ox, oy, oz, ix, iy, iz, tmin, kClosest ? best_t : tmax, r, hh,
                                            tt);
                else
                    wide_test<kKind == 1>(wn, node, w, ox, oy, oz, ix, iy, iz, tmin, kClosest ? best_t : tmax, r, hh, tt);
                const uint32_t refs[4] = {r.x, r.y, r.z, r.w};
                // leaves first: the hits they give shrink every lane's segment before the descent
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool hl = alive && hh[j] && (refs[j] & kWideLeaf);
                    if (__ballot(hl) != 0) test_tri(tris[refs[j] & ~kWideLeaf], hl && (kClosest || !found));
                }
                // internal children some lane hits, keyed by the entry distance of the lowest such
                // lane (children that lane misses after those it hits, missed children last)
                bool hi[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) hi[j] = alive && hh[j] && !(refs[j] & kWideLeaf);
                const uint64_t any = __ballot(hi[0] || hi[1] || hi[2] || hi[3]);
                if (any == 0) {
                    if (sp == 0) break;
                    node = st.pop(--sp);
                    continue;
                }
                const uint32_t rep = (uint32_t)__ffsll((unsigned long long)any) - 1u;
                uint32_t key[4], id[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool some = __ballot(hi[j]) != 0;
                    const uint32_t mine = __builtin_amdgcn_readlane(hi[j] ? ordered_bits(tt[j]) : 0xFFFFFFFEu, rep);
                    key[j] = some ? mine : 0xFFFFFFFFu;
                    id[j] = some ? refs[j] : kNone;
                }
                cswap_u(key[0], id[0], key[1], id[1]);
                cswap_u(key[2], id[2], key[3], id[3]);
                cswap_u(key[0], id[0], key[2], id[2]);
                cswap_u(key[1], id[1], key[3], id[3]);
                cswap_u(key[1], id[1], key[2], id[2]);
                if (id[3] != kNone && sp < (uint32_t)kWideStack) st.push(sp++, id[3]);
                if (id[2] != kNone && sp < (uint32_t)kWideStack) st.push(sp++, id[2]);
                if (id[1] != kNone && sp < (uint32_t)kWideStack) st.push(sp++, id[1]);
                node = id[0];
            }
        };
        const uint64_t live = __ballot(valid);
        if (live == 0) continue;
        const bool all_fast = !slab && __ballot(valid && !wr.fast) == 0;
        // the first valid lane's plane choice, and whether every valid lane makes the same one
        const int src = __ffsll((unsigned long long)live) - 1;
        WideRay shared;
        shared.ex = __builtin_amdgcn_readfirstlane(__shfl(wr.ex, src, 64));
        shared.ey = __builtin_amdgcn_readfirstlane(__shfl(wr.ey, src, 64));
        shared.ez = __builtin_amdgcn_readfirstlane(__shfl(wr.ez, src, 64));
        shared.fast = true;
        const bool same = all_fast && __ballot(valid && (wr.ex != shared.ex || wr.ey != shared.ey ||
                                                         wr.ez != shared.ez)) == 0;
        if (!qn) {
            if (same && n_int <= kWideFastNodes) walk(std::integral_constant<int, 1>{}, shared);
            else walk(std::integral_constant<int, 0>{}, wr);
        } else if (same) {
            walk(std::integral_constant<int, 3>{}, shared);
        } else if (all_fast) {
            walk(std::integral_constant<int, 3>{}, wr);
        } else {
            walk(std::integral_constant<int, 2>{}, wr);
        }
        if (valid) {
            if (kClosest)
                hits[rid] = make_float4(found ? best_t : INFINITY, __uint_as_float(found ? best_prim : kMissPrim),
                                        found ? best_u : 0.0f, found ? best_v : 0.0f);
            else
                occ[rid] = found ? 1 : 0;
        }
    }
    ch.finish();
}

template <bool kClosest, int kStack, int kBlock, bool kStats>
void launch(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, hcc_hit* hits, uint8_t* occ,
            uint32_t remap, uint32_t* cn, uint32_t* ct, uint32_t* wn, uint32_t* wt, hipStream_t stream) {
    const unsigned grid = (n + kBlock - 1) / kBlock;
    k_trace<kClosest, kStack, kBlock, kStats><<<grid, kBlock, 0, stream>>>(
        b->nodes, b->tris, b->n_int, (const float4*)rays, perm, n, (float4*)hits, occ, remap, cn, ct, wn, wt);
}

template <bool kClosest, bool kStats>
hcc_status dispatch_stack(uint32_t stack, uint32_t block, const hcc_bvh_s* b, const hcc_ray* rays,
                          const uint32_t* perm, uint32_t n, hcc_hit* hits, uint8_t* occ, uint32_t remap, uint32_t* cn,
                          uint32_t* ct, uint32_t* wn, uint32_t* wt, hipStream_t s) {
#define HCC_BLOCKS(STK)                                                                       \
    switch (block) {                                                                          \
        case 64: launch<kClosest, STK, 64, kStats>(b, rays, perm, n, hits, occ, remap, cn, ct, wn, wt, s); break;   \
        case 128: launch<kClosest, STK, 128, kStats>(b, rays, perm, n, hits, occ, remap, cn, ct, wn, wt, s); break; \
        case 256: launch<kClosest, STK, 256, kStats>(b, rays, perm, n, hits, occ, remap, cn, ct, wn, wt, s); break; \
        default: return fail(HCC_ERR_INVALID, "hcc_trace: block must be 64, 128 or 256");    \
    }
    switch (stack) {
        case HCC_STACK_LDS: HCC_BLOCKS(HCC_STACK_LDS); break;
        case HCC_STACK_SCRATCH: HCC_BLOCKS(HCC_STACK_SCRATCH); break;
        case HCC_STACK_SHORT: HCC_BLOCKS(HCC_STACK_SHORT); break;
        default: return fail(HCC_ERR_INVALID, "hcc_trace: unknown stack mode");
    }
#undef HCC_BLOCKS
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}


// The chunk-queue slot of stream s on the current device; kNoQueue while s is being captured
// into a graph (a replay could overlap a launch on the stream the slot belongs to) and once
// every slot of the device is taken.
uint32_t queue_slot(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return kNoQueue;
    }
    int dev = 0;
    if (cs != hipStreamCaptureStatusNone || hipGetDevice(&dev) != hipSuccess) return kNoQueue;
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, uint32_t> slots;
    static std::map<int, uint32_t> taken;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(dev, s);
    const auto it = slots.find(key);
    if (it != slots.end()) return it->second;
    uint32_t& used = taken[dev];
    if (used >= kQueueSlots) return kNoQueue;
    slots.emplace(key, used);
    return used++;
}

// Persistent launches (BVH2 or 4-wide), optionally counting wavefront-distinct fetches.
template <bool kStats>
hcc_status trace_persistent(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                            hcc_hit* hits, uint8_t* occ, const hcc_trace_opts& o, unsigned long long* counts,
                            hipStream_t s) {
    const uint32_t refill = std::min<uint32_t>(64u, std::max<uint32_t>(1u, o.refill ? o.refill : 16u));
    const uint32_t chunk = std::max<uint32_t>(64u, o.chunk ? o.chunk : 256u);
    const uint32_t nchunks = (uint32_t)(((uint64_t)n + chunk - 1) / chunk);
    const uint32_t waves = std::min<uint32_t>(nchunks, o.waves ? o.waves : 8192u);
    // counting launches keep the static assignment, so that their counts are reproducible
    const uint32_t qslot = kStats ? kNoQueue : queue_slot(s);
    const uint32_t deal = (o.xcd_remap ? 1u : 0u) | ((o.flags & HCC_TRACE_SPREAD) ? 2u : 0u);
    const float4* r = (const float4*)rays;
    float4* h = (float4*)hits;
    if constexpr (!kStats) {
        if (o.flags & HCC_TRACE_PACKET) {
            // one chunk of 64 rays per packet; the wide flags (QUANT, SLAB, SPREAD) apply
            const uint32_t packets = (uint32_t)(((uint64_t)n + 63) / 64);
            const uint32_t pw = std::min<uint32_t>(packets, o.waves ? o.waves : 8192u);
            const Node4Q* qn = (o.flags & HCC_TRACE_QUANT) ? b->qnodes : nullptr;
            const uint32_t sl = (o.flags & HCC_TRACE_SLAB) ? 1u : 0u;
            if (closest)
                k_trace_packet<true><<<pw, 64, 0, s>>>(b->wnodes, qn, b->tris, b->n_int, r, perm, n, h, occ, deal, sl,
                                                       qslot);
            else
                k_trace_packet<false><<<pw, 64, 0, s>>>(b->wnodes, qn, b->tris, b->n_int, r, perm, n, h, occ, deal, sl,
                                                        qslot);
            HCC_HIP(hipGetLastError());
            return HCC_OK;
        }
    }
    if (o.flags & HCC_TRACE_WIDE) {
        // stack: scratch (HCC_STACK_SCRATCH, and always when counting), the first 16 entries in
        // LDS (HCC_STACK_SHORT) or the first 24 (HCC_STACK_LDS)
        const int lds = kStats ? 0 : (o.stack == HCC_STACK_SHORT ? 16 : (o.stack == HCC_STACK_LDS ? 24 : 0));
        // quantised nodes (HCC_TRACE_QUANT): checked available by the caller
        const Node4Q* qn = (o.flags & HCC_TRACE_QUANT) ? b->qnodes : nullptr;
#define HCC_WIDE(CL, LD)                                                                                           \
    k_trace_wide<CL, kStats, LD><<<waves, 64, 0, s>>>(b->wnodes, qn, b->tris, b->n_int, r, perm, n, h, occ, refill, \
                                                      chunk, deal, (o.flags & HCC_TRACE_SLAB) ? 1u : 0u, qslot, counts)
        if (closest) {
            if (lds == 16) HCC_WIDE(true, 16); else if (lds == 24) HCC_WIDE(true, 24); else HCC_WIDE(true, 0);
        } else {
            if (lds == 16) HCC_WIDE(false, 16); else if (lds == 24) HCC_WIDE(false, 24); else HCC_WIDE(false, 0);
        }
#undef HCC_WIDE
        HCC_HIP(hipGetLastError());
        return HCC_OK;
    }
#define HCC_PERSIST(CL, STK)                                                                                  \
    do {                                                                                                      \
        if (o.flags & HCC_TRACE_SPECULATE)                                                                    \
            k_trace_persistent<CL, STK, true, kStats><<<waves, 64, 0, s>>>(b->nodes, b->tris, b->n_int, r, perm, \
                                                                           n, h, occ, refill, chunk,           \
                                                                           deal, qslot, counts);               \
        else                                                                                                  \
            k_trace_persistent<CL, STK, false, kStats><<<waves, 64, 0, s>>>(b->nodes, b->tris, b->n_int, r,      \
                                                                            perm, n, h, occ, refill, chunk,     \
                                                                            deal, qslot, counts);               \
    } while (0)
    if (kStats && o.stack != HCC_STACK_SCRATCH)
        return fail(HCC_ERR_UNSUPPORTED, "hcc_trace_count: counting runs with the scratch stack only");
    switch (o.stack) {
        case HCC_STACK_SCRATCH:
            if (closest) HCC_PERSIST(true, HCC_STACK_SCRATCH); else HCC_PERSIST(false, HCC_STACK_SCRATCH);
            break;
        case HCC_STACK_LDS:
            if constexpr (!kStats) {
                if (closest) HCC_PERSIST(true, HCC_STACK_LDS); else HCC_PERSIST(false, HCC_STACK_LDS);
            }
            break;
        case HCC_STACK_SHORT:
            if constexpr (!kStats) {
                if (closest) HCC_PERSIST(true, HCC_STACK_SHORT); else HCC_PERSIST(false, HCC_STACK_SHORT);
            }
            break;
        default:
            return fail(HCC_ERR_INVALID, "hcc_trace: unknown stack mode");
    }
#undef HCC_PERSIST
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

}  // namespace

hcc_status trace(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                 hcc_hit* hits, uint8_t* occ, const hcc_trace_opts& o, hipStream_t s) {
    if ((o.flags & HCC_TRACE_QUANT) && (!(o.flags & HCC_TRACE_WIDE) || (b->n_int > 0 && !b->quant_ok)))
        return fail(HCC_ERR_UNSUPPORTED, "hcc_trace: HCC_TRACE_QUANT needs HCC_TRACE_WIDE and a BVH whose boxes are "
                                         "finite");
    if ((o.flags & HCC_TRACE_PACKET) && !(o.flags & HCC_TRACE_WIDE))
        return fail(HCC_ERR_UNSUPPORTED, "hcc_trace: HCC_TRACE_PACKET needs HCC_TRACE_WIDE");
    if ((o.persistent || (o.flags & HCC_TRACE_WIDE)) && b->n_int > 0)
        return trace_persistent<false>(b, rays, perm, n, closest, hits, occ, o, nullptr, s);
    const uint32_t block = o.block ? o.block : 64;
    if (closest)
        return dispatch_stack<true, false>(o.stack, block, b, rays, perm, n, hits, occ, o.xcd_remap, nullptr, nullptr,
                                           nullptr, nullptr, s);
    return dispatch_stack<false, false>(o.stack, block, b, rays, perm, n, hits, occ, o.xcd_remap, nullptr, nullptr,
                                        nullptr, nullptr, s);
}

hcc_status trace_count(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                       hcc_hit* hits, uint8_t* occ, const hcc_trace_opts& o, unsigned long long* counts,
                       hipStream_t s) {
    if (!(o.persistent || (o.flags & HCC_TRACE_WIDE)) || b->n_int == 0)
        return fail(HCC_ERR_UNSUPPORTED, "hcc_trace_count: counts the persistent launches only");
    if (o.flags & HCC_TRACE_PACKET)
        return fail(HCC_ERR_UNSUPPORTED, "hcc_trace_count: packet launches are not counted");
    if ((o.flags & HCC_TRACE_QUANT) && (!(o.flags & HCC_TRACE_WIDE) || !b->quant_ok))
        return fail(HCC_ERR_UNSUPPORTED, "hcc_trace_count: HCC_TRACE_QUANT needs HCC_TRACE_WIDE and a BVH whose "
                                         "boxes are finite");
    return trace_persistent<true>(b, rays, perm, n, closest, hits, occ, o, counts, s);
}

hcc_status trace_stats(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                       hcc_hit* hits, uint8_t* occ, uint32_t* cn, uint32_t* ct, uint32_t* wn, uint32_t* wt,
                       hipStream_t s) {
    if (closest)
        return dispatch_stack<true, true>(HCC_STACK_SCRATCH, 64, b, rays, perm, n, hits, occ, 0, cn, ct, wn, wt, s);
    return dispatch_stack<false, true>(HCC_STACK_SCRATCH, 64, b, rays, perm, n, hits, occ, 0, cn, ct, wn, wt, s);
}

}  // namespace hcc
