// Stable LSD radix sort of (key, index) pairs for gfx950, 8-bit digits.
//
// Sorting the ray keys as unsigned integers and handing the trace kernel the sorted
// ray indices is the reorder step of the method (Sections 4.2.3 and 5).  Each pass over one
// 8-bit digit is a reduce-then-scan over tiles of consecutive keys (4,096 of 32 bits or 2,048
// of 64 bits), three launches with no waiting between workgroups:
//   1. k_count: each tile's digit counts (one read of the keys, every load of a thread issued
//      at once; runs of equal digits added to LDS with one atomic), stored digit-major;
//   2. k_scan: per digit, the exclusive scan of its counts over the tiles (in place) and the
//      digit's total;
//   3. k_scatter: each tile ranks its keys with wavefront ballots (the lanes holding the same
//      digit are found from one ballot per digit bit; their count below a lane is its stable
//      rank), reorders (key, value) pairs in LDS so that equal digits are consecutive, and
//      writes them at (keys of smaller digits) + (this digit in earlier tiles) + rank.
// Once the key bits still to be ordered fit beside the element index in 32 bits, a pass writes
// packed words ((remaining key bits) << index bits | index) and the passes after it move those
// 4-byte words instead of a key and a value (when the sorted keys are not asked for).
// Tiles are dealt to the eight XCDs in contiguous ranges (the hardware deals workgroups round
// robin): the runs that consecutive tiles write for one digit are adjacent, and when the
// tiles sit on one XCD its L2 merges them into whole lines before they reach HBM.
// Keys: uint32 (key_bits <= 32) or uint64.  Only bits [0, key_bits) take part.
#include "hcc_internal.h"

#include <mutex>

namespace hcc {
namespace {

constexpr uint32_t kBlock = 256;          // 4 wavefronts
// Keys per thread and tile: 16 (4,096-key tiles) for 32-bit keys; 8 (2,048-key tiles) for
// 64-bit keys, whose LDS staging of a 4,096-key tile (48 KB) would leave room for only two
// workgroups per CU.
template <typename K>
constexpr uint32_t items_of() { return sizeof(K) == 4 ? 16u : 8u; }
template <typename K>
constexpr uint32_t tile_of() { return kBlock * items_of<K>(); }
constexpr uint32_t kRadix = 256;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a 256-thread block.  s must hold 4 words
// not used by any other concurrent scan.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* s) {
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    uint32_t incl = wave_incl_scan(x);
    if (lane == 63) s[w] = incl;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) pre += (j < w) ? s[j] : 0u;
    return pre + incl - x;
}

// Lanes of the wavefront (among 'alive') whose low 'nbits' bits of d equal this lane's.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint32_t nbits, bool alive) {
    uint64_t m = __ballot(alive);
    for (uint32_t b = 0; b < nbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Digit counts of one tile per block: counts[d * T + tile].  Thread t reads the kItems
// consecutive keys starting at t * kItems of its tile with 16-byte loads, all in flight
// together, and adds each run of equal digits among them to its wavefront's LDS histogram
// with one atomic (keys of coherent rays repeat: few atomics, little contention).
template <typename K>
__global__ __launch_bounds__(kBlock) void k_count(const K* __restrict__ keys, uint32_t n, uint32_t shift,
                                                  uint32_t nbits, uint32_t* __restrict__ counts) {
    constexpr uint32_t kPerLoad = 16 / sizeof(K);
    constexpr uint32_t kItems = items_of<K>(), kTile = tile_of<K>();
    __shared__ uint32_t s_h[4 * kRadix];
    const uint32_t t = threadIdx.x, w = t >> 6;
    const uint32_t T = gridDim.x;
    const uint32_t tile = xcd_block(blockIdx.x, T);
    for (uint32_t i = t; i < 4 * kRadix; i += kBlock) s_h[i] = 0;
    const uint32_t mask = (1u << nbits) - 1u;
    const size_t first = (size_t)tile * kTile + (size_t)t * kItems;
    const uint32_t nv = first >= n ? 0u : ((size_t)n - first >= kItems ? kItems : (uint32_t)((size_t)n - first));
    K k[kItems];
    if (nv == kItems && ((uintptr_t)keys & 15u) == 0) {
#pragma unroll
        for (uint32_t q = 0; q < kItems / kPerLoad; ++q) {
            const uint4 v = *reinterpret_cast<const uint4*>(keys + first + kPerLoad * q);
            if (sizeof(K) == 4) {
                k[4 * q] = (K)v.x; k[4 * q + 1] = (K)v.y; k[4 * q + 2] = (K)v.z; k[4 * q + 3] = (K)v.w;
            } else {
                k[2 * q] = (K)(((uint64_t)v.y << 32) | v.x);
                k[2 * q + 1] = (K)(((uint64_t)v.w << 32) | v.z);
            }
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < kItems; ++i) k[i] = i < nv ? keys[first + i] : K(0);
    }
    __syncthreads();
    uint32_t* h = s_h + w * kRadix;
    uint32_t cur = (uint32_t)(k[0] >> shift) & mask, run = nv ? 1u : 0u;
    // a wavefront whose 64 x kItems keys all share one digit (common for coherent rays' keys)
    // adds them with one atomic instead of 64 on the same LDS word
    bool uniform = nv == kItems && cur == __builtin_amdgcn_readfirstlane(cur);
#pragma unroll
    for (uint32_t i = 1; i < kItems; ++i) uniform = uniform && ((uint32_t)(k[i] >> shift) & mask) == cur;
    if (__ballot(uniform) == ~0ull) {
        if ((t & 63u) == 0) atomicAdd(&h[cur], 64u * kItems);
        run = 0;
    } else {
#pragma unroll
        for (uint32_t i = 1; i < kItems; ++i) {
            if (i < nv) {
                const uint32_t d = (uint32_t)(k[i] >> shift) & mask;
                if (d == cur) {
                    ++run;
                } else {
                    atomicAdd(&h[cur], run);
                    cur = d;
                    run = 1u;
                }
            }
        }
    }
    if (run) atomicAdd(&h[cur], run);
    __syncthreads();
    counts[(size_t)t * T + tile] = s_h[t] + s_h[kRadix + t] + s_h[2 * kRadix + t] + s_h[3 * kRadix + t];
}

// Block d: exclusive scan of digit d's tile counts (row d of counts, T entries, in place),
// staged through LDS in segments of 4096 (padded one word in 16 so that a thread's 16
// consecutive entries sit in different banks); the digit's total goes to tot[d].
__global__ __launch_bounds__(kBlock) void k_scan(uint32_t* __restrict__ counts, uint32_t T, uint32_t* __restrict__ tot) {
    constexpr uint32_t kSeg = 4096;
    __shared__ uint32_t s[kSeg + kSeg / 16];
    __shared__ uint32_t s_scan[4];
    __shared__ uint32_t s_total;
    const uint32_t t = threadIdx.x, d = blockIdx.x;
    uint32_t* row = counts + (size_t)d * T;
    uint32_t carry = 0;
    for (uint32_t seg = 0; seg < T; seg += kSeg) {
        const uint32_t m = min(kSeg, T - seg);
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) {
            const uint32_t i = t + 256 * j;
            s[i + (i >> 4)] = i < m ? row[seg + i] : 0u;
        }
        __syncthreads();
        uint32_t x[16], sum = 0;
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) {
            x[j] = s[17 * t + j];
            sum += x[j];
        }
        uint32_t run = block_excl_scan256(sum, s_scan) + carry;
        if (t == kBlock - 1) s_total = run + sum;
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) {
            s[17 * t + j] = run;
            run += x[j];
        }
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) {
            const uint32_t i = t + 256 * j;
            if (i < m) row[seg + i] = s[i + (i >> 4)];
        }
        carry = s_total;
        __syncthreads();
    }
    if (t == 0) tot[d] = carry;
}

// What a pass reads besides its keys, and what it writes.  Once the key bits a sort still has
// to order fit beside the ray index in 32 bits, a pass writes one packed word per element,
// (key >> consumed bits) << index bits | index, and the later passes read and move that word
// alone: 4 bytes per element instead of a key and a value.
enum : int { kInIota = 0, kInVals = 1, kInPacked = 2 };
enum : int { kOutKeysVals = 0, kOutVals = 1, kOutPacked = 2 };

// LDS staging of a tile's reordered elements: one 8-byte record per (32-bit key, value) pair,
// separate key and value arrays for 64-bit keys, the word alone for packed words.
template <typename K, bool kWordOnly>
struct TileStage {
    K key[tile_of<K>()];
    uint32_t val[tile_of<K>()];
    __device__ void put(uint32_t i, K k, uint32_t v) { key[i] = k; val[i] = v; }
    __device__ void get(uint32_t i, K& k, uint32_t& v) const { k = key[i]; v = val[i]; }
};
template <>
struct TileStage<uint32_t, false> {
    uint2 kv[tile_of<uint32_t>()];
    __device__ void put(uint32_t i, uint32_t k, uint32_t v) { kv[i] = make_uint2(k, v); }
    __device__ void get(uint32_t i, uint32_t& k, uint32_t& v) const {
        const uint2 p = kv[i];
        k = p.x;
        v = p.y;
    }
};
template <>
struct TileStage<uint32_t, true> {
    uint32_t w[tile_of<uint32_t>()];
    __device__ void put(uint32_t i, uint32_t k, uint32_t) { w[i] = k; }
    __device__ void get(uint32_t i, uint32_t& k, uint32_t& v) const { k = w[i]; v = 0u; }
};

// One pass: digit (kin >> shift) & (2^nbits - 1).  Packed input: the value is the word's low
// ib bits.  Packed output: (key part >> pshift) << ib | value, where the key part is the key
// or, for packed input, the word without its index bits.
template <typename K, int kIn, int kOut>
__global__ __launch_bounds__(kBlock) void k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    void* __restrict__ kout_, uint32_t* __restrict__ vout, uint32_t n,
                                                    uint32_t shift, uint32_t nbits, uint32_t ib, uint32_t pshift,
                                                    const uint32_t* __restrict__ offs,
                                                    const uint32_t* __restrict__ tot) {
    constexpr uint32_t kItems = items_of<K>(), kTile = tile_of<K>();
    constexpr bool kPackedIn = kIn == kInPacked;
    static_assert(!kPackedIn || sizeof(K) == 4, "packed words are 32-bit");
    __shared__ uint32_t s_whist[4 * kRadix];
    __shared__ uint32_t s_gofs[kRadix];
    __shared__ uint32_t s_scan[8];
    __shared__ TileStage<K, kPackedIn> s_tile;
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint32_t T = gridDim.x;
    const uint32_t tile = xcd_block(blockIdx.x, T);
    const uint32_t mask = (1u << nbits) - 1u;
    const uint32_t imask = ib >= 32 ? ~0u : (1u << ib) - 1u;
    for (uint32_t i = t; i < 4 * kRadix; i += kBlock) s_whist[i] = 0;
    const uint32_t base = tile * kTile + w * (64u * kItems) + lane;
    const uint64_t lt = lanemask_lt();
    uint32_t* wh = s_whist + w * kRadix;

    K k[kItems];
    uint32_t v[kItems];
    uint32_t r[kItems];
    if ((tile + 1) * kTile <= n) {
#pragma unroll
        for (uint32_t i = 0; i < kItems; ++i) {
            const uint32_t idx = base + i * 64u;
            k[i] = kin[idx];
            v[i] = kIn == kInIota ? idx : (kIn == kInVals ? vin[idx] : 0u);
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < kItems; ++i) {
            const uint32_t idx = base + i * 64u;
            const bool valid = idx < n;
            k[i] = valid ? kin[idx] : K(0);
            v[i] = kIn == kInIota ? idx : ((kIn == kInVals && valid) ? vin[idx] : 0u);
        }
    }
    // the tile's global offsets do not depend on its keys: read them while the keys load
    const uint32_t gtot = tot[t];
    const uint32_t gofs = offs[(size_t)t * T + tile];
    __syncthreads();

    // stable rank of every key among the keys of its wavefront with the same digit
#pragma unroll
    for (uint32_t i = 0; i < kItems; ++i) {
        const bool valid = base + i * 64u < n;
        const uint32_t d = (uint32_t)(k[i] >> shift) & mask;
        const uint64_t m = match_digit(d, nbits, valid);
        const uint32_t below = (uint32_t)__popcll(m & lt);
        const uint32_t prev = valid ? wh[d] : 0u;
        r[i] = prev + below;
        // every lane of the group has read wh[d] before the group's lowest lane writes it:
        // a wavefront's LDS operations complete in issue order
        if (valid && below == 0) wh[d] = prev + (uint32_t)__popcll(m);
    }
    __syncthreads();

    // thread t owns digit t: where each wavefront's keys of digit t start in the tile, and the
    // distance from a position in the tile to its position in the output
    const uint32_t d = t;
    const uint32_t c0 = s_whist[d], c1 = s_whist[kRadix + d], c2 = s_whist[2 * kRadix + d],
                   c3 = s_whist[3 * kRadix + d];
    const uint32_t dexcl = block_excl_scan256(c0 + c1 + c2 + c3, s_scan);
    const uint32_t gbase = block_excl_scan256(gtot, s_scan + 4) + gofs;
    s_whist[d] = dexcl;
    s_whist[kRadix + d] = dexcl + c0;
    s_whist[2 * kRadix + d] = dexcl + c0 + c1;
    s_whist[3 * kRadix + d] = dexcl + c0 + c1 + c2;
    s_gofs[d] = gbase - dexcl;
    __syncthreads();

#pragma unroll
    for (uint32_t i = 0; i < kItems; ++i) {
        if (base + i * 64u < n) {
            const uint32_t dd = (uint32_t)(k[i] >> shift) & mask;
            s_tile.put(wh[dd] + r[i], k[i], v[i]);
        }
    }
    __syncthreads();
    const uint32_t count = min(kTile, n - tile * kTile);
#pragma unroll
    for (uint32_t i = 0; i < kItems; ++i) {
        const uint32_t j = t + i * kBlock;
        if (j < count) {
            K key;
            uint32_t val;
            s_tile.get(j, key, val);
            if (kPackedIn) val = (uint32_t)key & imask;
            const uint32_t g = s_gofs[(uint32_t)(key >> shift) & mask] + j;
            if (kOut == kOutKeysVals) ((K*)kout_)[g] = key;
            if (kOut == kOutPacked) {
                const K part = kPackedIn ? (K)(key >> ib) : key;
                ((uint32_t*)kout_)[g] = ((uint32_t)(part >> pshift) << ib) | val;
            }
            if (kOut != kOutPacked) vout[g] = val;
        }
    }
}

// Tile-local sort: block b sorts keys [b*T, b*T + T) on its own (T = 256 x kTItems) with
// the same wavefront-ballot ranking, one LDS exchange per 8-bit pass, and writes the
// permutation of its tile (global ray indices) and optionally the sorted keys.  Elements past
// n take the largest key; they sit after every real key of the tile and stay behind them
// (stable), so the first count outputs are the tile's sorted real keys.
template <typename K, uint32_t kTItems>
__global__ __launch_bounds__(kBlock) void k_tile_sort(const K* __restrict__ kin, uint32_t n, uint32_t skip,
                                                      uint32_t passes, uint32_t key_bits, uint32_t* __restrict__ perm,
                                                      K* __restrict__ kout) {
    constexpr uint32_t T = kBlock * kTItems;
    __shared__ uint32_t s_whist[4 * kRadix];
    __shared__ uint32_t s_dexcl[kRadix];
    __shared__ uint32_t s_scan[4];
    __shared__ K s_keys[T];
    __shared__ uint32_t s_vals[T];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint32_t tile0 = blockIdx.x * T;
    const uint32_t seg = w * (64u * kTItems) + lane;     // this lane's first element in the tile
    const uint64_t lt = lanemask_lt();
    uint32_t* wh = s_whist + w * kRadix;
    K k[kTItems];
    uint32_t v[kTItems];
#pragma unroll
    for (uint32_t i = 0; i < kTItems; ++i) {
        const uint32_t e = seg + i * 64u;
        k[i] = tile0 + e < n ? kin[tile0 + e] : ~K(0);
        v[i] = e;
    }
    for (uint32_t p = 0; p < passes; ++p) {
        const uint32_t shift = skip + 8u * p;
        const uint32_t nb = min(8u, key_bits - shift);
        const uint32_t mask = (1u << nb) - 1u;
        for (uint32_t i = t; i < 4 * kRadix; i += kBlock) s_whist[i] = 0;
        __syncthreads();
        uint32_t r[kTItems];
#pragma unroll
        for (uint32_t i = 0; i < kTItems; ++i) {
            const uint32_t d = (uint32_t)(k[i] >> shift) & mask;
            const uint64_t m = match_digit(d, nb, true);
            const uint32_t below = (uint32_t)__popcll(m & lt);
            const uint32_t prev = wh[d];
            r[i] = prev + below;
            if (below == 0) wh[d] = prev + (uint32_t)__popcll(m);
        }
        __syncthreads();
        const uint32_t c0 = s_whist[t], c1 = s_whist[kRadix + t], c2 = s_whist[2 * kRadix + t],
                       c3 = s_whist[3 * kRadix + t];
        s_whist[t] = 0;
        s_whist[kRadix + t] = c0;
        s_whist[2 * kRadix + t] = c0 + c1;
        s_whist[3 * kRadix + t] = c0 + c1 + c2;
        s_dexcl[t] = block_excl_scan256(c0 + c1 + c2 + c3, s_scan);
        __syncthreads();
#pragma unroll
        for (uint32_t i = 0; i < kTItems; ++i) {
            const uint32_t d = (uint32_t)(k[i] >> shift) & mask;
            const uint32_t pos = s_dexcl[d] + wh[d] + r[i];
            s_keys[pos] = k[i];
            s_vals[pos] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (uint32_t i = 0; i < kTItems; ++i) {
            k[i] = s_keys[seg + i * 64u];
            v[i] = s_vals[seg + i * 64u];
        }
        __syncthreads();
    }
#pragma unroll
    for (uint32_t i = 0; i < kTItems; ++i) {
        const uint32_t e = seg + i * 64u;
        if (tile0 + e < n) {
            perm[tile0 + e] = tile0 + v[i];
            if (kout) kout[tile0 + e] = k[i];
        }
    }
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t keys_a, keys_b, vals, counts, tot, total;
};

// Workspace of a global sort: two key buffers, one value buffer, the digit-major tile counts
// of one pass (reused by every pass) and the digit totals.  Nothing in it needs clearing.
constexpr Layout layout(uint32_t n, uint32_t key_bits, uint32_t skip = 0) {
    const size_t ks = key_bits <= 32 ? 4 : 8;
    const size_t tile = key_bits <= 32 ? tile_of<uint32_t>() : tile_of<uint64_t>();
    const size_t tiles = ((size_t)n + tile - 1) / tile;
    (void)skip;
    Layout L{};
    size_t off = 0;
    L.keys_a = off; off += align256((size_t)n * ks);
    L.keys_b = off; off += align256((size_t)n * ks);
    L.vals = off; off += align256((size_t)n * 4);
    L.counts = off; off += align256(tiles * kRadix * 4);
    L.tot = off; off += align256(kRadix * 4);
    L.total = off;
    return L;
}

// Launches one pass's scatter for the input / output forms chosen by run_sort.
template <typename K>
void scatter_pass(int in, int out, uint32_t tiles, const K* kin, const uint32_t* vin, void* kout, uint32_t* vout,
                  uint32_t n, uint32_t shift, uint32_t nb, uint32_t ib, uint32_t pshift, const uint32_t* counts,
                  const uint32_t* tot, hipStream_t stream) {
    const dim3 grid(tiles), block(kBlock);
#define HCC_SCATTER(I, O) \
    k_scatter<K, I, O><<<grid, block, 0, stream>>>(kin, vin, kout, vout, n, shift, nb, ib, pshift, counts, tot)
    if (in == kInIota) {
        if (out == kOutKeysVals) HCC_SCATTER(kInIota, kOutKeysVals);
        else if (out == kOutVals) HCC_SCATTER(kInIota, kOutVals);
        else HCC_SCATTER(kInIota, kOutPacked);
    } else {
        if (out == kOutKeysVals) HCC_SCATTER(kInVals, kOutKeysVals);
        else if (out == kOutVals) HCC_SCATTER(kInVals, kOutVals);
        else HCC_SCATTER(kInVals, kOutPacked);
    }
#undef HCC_SCATTER
}

void scatter_packed(int out, uint32_t tiles, const uint32_t* kin, void* kout, uint32_t* vout, uint32_t n,
                    uint32_t shift, uint32_t nb, uint32_t ib, const uint32_t* counts, const uint32_t* tot,
                    hipStream_t stream) {
    const dim3 grid(tiles), block(kBlock);
    if (out == kOutVals)
        k_scatter<uint32_t, kInPacked, kOutVals><<<grid, block, 0, stream>>>(kin, nullptr, kout, vout, n, shift, nb,
                                                                          ib, 0u, counts, tot);
    else
        k_scatter<uint32_t, kInPacked, kOutPacked><<<grid, block, 0, stream>>>(kin, nullptr, kout, vout, n, shift,
                                                                            nb, ib, 0u, counts, tot);
}

// Passes over the digits [skip, key_bits), lowest first.  Without sorted keys out, the first
// pass whose remaining key bits fit beside the index in 32 bits writes packed words, and the
// passes after it sort those words (the digit then sits above the index bits).
template <typename K>
hcc_status run_sort(const K* keys, uint32_t key_bits, uint32_t skip, uint32_t n, uint32_t* perm, K* sorted_keys,
                    char* ws, hipStream_t stream) {
    const uint32_t passes = (key_bits - skip + 7) / 8;
    const Layout L = layout(n, key_bits, skip);
    const uint32_t tiles_k = (n + tile_of<K>() - 1) / tile_of<K>();
    const uint32_t tiles_w = (n + tile_of<uint32_t>() - 1) / tile_of<uint32_t>();
    uint32_t ib = 0;
    while (ib < 32 && (1ull << ib) < n) ++ib;
    uint32_t* counts = (uint32_t*)(ws + L.counts);
    uint32_t* tot = (uint32_t*)(ws + L.tot);
    void* final_keys = sorted_keys ? (void*)sorted_keys : (void*)(ws + L.keys_a);
    void* other_keys = ws + L.keys_b;
    uint32_t* vals_tmp = (uint32_t*)(ws + L.vals);
    const void* kin = keys;
    const uint32_t* vin = nullptr;
    bool packed = false;       // kin holds packed words
    uint32_t dropped = 0;      // key bits below the packed words' key part
    for (uint32_t p = 0; p < passes; ++p) {
        const bool to_final = ((passes - 1 - p) % 2) == 0;
        void* kout = to_final ? final_keys : other_keys;
        uint32_t* vout = to_final ? perm : vals_tmp;
        const bool last = p + 1 == passes;
        const uint32_t at = skip + 8u * p;
        const uint32_t nb = std::min<uint32_t>(8u, key_bits - at);
        const uint32_t left = key_bits - (at + nb);
        int out = kOutKeysVals;
        if (last) out = sorted_keys ? kOutKeysVals : kOutVals;
        else if (packed || (!sorted_keys && left + ib <= 32)) out = kOutPacked;
        if (packed) {
            const uint32_t shift = ib + (at - dropped);
            k_count<uint32_t><<<dim3(tiles_w), dim3(kBlock), 0, stream>>>((const uint32_t*)kin, n, shift, nb, counts);
            k_scan<<<dim3(kRadix), dim3(kBlock), 0, stream>>>(counts, tiles_w, tot);
            scatter_packed(out, tiles_w, (const uint32_t*)kin, kout, vout, n, shift, nb, ib, counts, tot, stream);
        } else {
            k_count<K><<<dim3(tiles_k), dim3(kBlock), 0, stream>>>((const K*)kin, n, at, nb, counts);
            k_scan<<<dim3(kRadix), dim3(kBlock), 0, stream>>>(counts, tiles_k, tot);
            scatter_pass<K>(p == 0 ? kInIota : kInVals, out, tiles_k, (const K*)kin, vin, kout, vout, n, at, nb, ib,
                            at + nb, counts, tot, stream);
            if (out == kOutPacked) {
                packed = true;
                dropped = at + nb;
            }
        }
        kin = kout;
        vin = vout;
    }
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

template <typename K>
hcc_status run_tile_sort(const K* keys, uint32_t key_bits, uint32_t skip, uint32_t tile, uint32_t n, uint32_t* perm,
                         K* sorted_keys, hipStream_t stream) {
    const uint32_t passes = (key_bits - skip + 7) / 8;
    const dim3 grid((n + tile - 1) / tile), block(kBlock);
    switch (tile) {
        case 256: k_tile_sort<K, 1><<<grid, block, 0, stream>>>(keys, n, skip, passes, key_bits, perm, sorted_keys); break;
        case 512: k_tile_sort<K, 2><<<grid, block, 0, stream>>>(keys, n, skip, passes, key_bits, perm, sorted_keys); break;
        case 1024: k_tile_sort<K, 4><<<grid, block, 0, stream>>>(keys, n, skip, passes, key_bits, perm, sorted_keys); break;
        case 2048: k_tile_sort<K, 8><<<grid, block, 0, stream>>>(keys, n, skip, passes, key_bits, perm, sorted_keys); break;
        default: k_tile_sort<K, 16><<<grid, block, 0, stream>>>(keys, n, skip, passes, key_bits, perm, sorted_keys); break;
    }
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

// Workspace of hcc_sort_static: one fixed device array per GPU, so that the call allocates
// nothing.  It is sized for the largest sort the call accepts (64-bit keys, the most passes);
// a smaller sort uses a prefix of it.  Host code never passes the array's name to a kernel
// (on the host it only names the symbol): the per-device address comes from
// hipGetSymbolAddress on the first call on each device.
constexpr size_t kStaticBytes = layout(HCC_SORT_STATIC_MAX_KEYS, 64).total;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hcc_status static_scratch(void** out) {
    int dev = -1;
    HCC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HCC_ERR_UNSUPPORTED, "hcc_sort_static: device index above 63");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(HCC_ERR_DEVICE, "hcc_sort_static: no device address for the static workspace");
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return HCC_OK;
}

}  // namespace

size_t sort_workspace_bytes(uint32_t n, uint32_t key_bits) { return layout(n, key_bits).total; }

size_t sort_static_bytes() { return kStaticBytes; }

// hcc_sort with the library's static workspace: the same kernels as radix_sort_ex over the
// whole key range.  Every part of the workspace a pass reads was written earlier in the same
// call, so nothing carries over between calls and nothing needs clearing.
hcc_status radix_sort_static(const void* d_keys, uint32_t key_bits, uint32_t n, uint32_t* d_perm,
                             void* d_sorted_keys, hipStream_t stream) {
    if (key_bits < 1 || key_bits > 64) return fail(HCC_ERR_INVALID, "hcc_sort_static: key_bits must be in [1, 64]");
    if (n > HCC_SORT_STATIC_MAX_KEYS)
        return fail(HCC_ERR_INVALID, "hcc_sort_static: n exceeds HCC_SORT_STATIC_MAX_KEYS (1048576); "
                                     "use hcc_sort with a caller workspace");
    if (n == 0) return HCC_OK;
    if (!d_keys || !d_perm) return fail(HCC_ERR_INVALID, "hcc_sort_static: null pointer");
    void* ws = nullptr;
    const hcc_status st = static_scratch(&ws);
    if (st != HCC_OK) return st;
    return radix_sort_ex(d_keys, key_bits, 0, 0, n, d_perm, d_sorted_keys, ws, kStaticBytes, stream);
}

hcc_status fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return HCC_OK;
    const unsigned grid = (unsigned)std::min<size_t>(1024, (n + 255) / 256);
    k_fill_u32<<<grid, 256, 0, s>>>(p, n, v);
    HCC_HIP(hipGetLastError());
    return HCC_OK;
}

// skip: the low bits left out of the order; tile: 0 for one sort over all n keys, else the
// size of the independently sorted groups (256 ... 4096, a power of two).
hcc_status radix_sort_ex(const void* d_keys, uint32_t key_bits, uint32_t skip, uint32_t tile, uint32_t n,
                         uint32_t* d_perm, void* d_sorted_keys, void* d_ws, size_t ws_bytes, hipStream_t stream) {
    if (key_bits < 1 || key_bits > 64) return fail(HCC_ERR_INVALID, "hcc_sort: key_bits must be in [1, 64]");
    if (skip >= key_bits) return fail(HCC_ERR_INVALID, "hcc_sort_ex: skip_bits must be below key_bits");
    if (tile != 0 && (tile < 256 || tile > 4096 || (tile & (tile - 1)) != 0))
        return fail(HCC_ERR_INVALID, "hcc_sort_ex: tile must be 0 or a power of two in [256, 4096]");
    if (n >= (1u << 30)) return fail(HCC_ERR_INVALID, "hcc_sort: n must be below 2^30");
    if (n == 0) return HCC_OK;
    if (!d_keys || !d_perm) return fail(HCC_ERR_INVALID, "hcc_sort: null pointer");
    if (tile != 0) {
        if (key_bits <= 32)
            return run_tile_sort<uint32_t>((const uint32_t*)d_keys, key_bits, skip, tile, n, d_perm,
                                           (uint32_t*)d_sorted_keys, stream);
        return run_tile_sort<uint64_t>((const uint64_t*)d_keys, key_bits, skip, tile, n, d_perm,
                                       (uint64_t*)d_sorted_keys, stream);
    }
    if (!d_ws) return fail(HCC_ERR_INVALID, "hcc_sort: null workspace");
    if (((uintptr_t)d_ws & 255u) != 0) return fail(HCC_ERR_INVALID, "hcc_sort: workspace must be 256-byte aligned");
    if (ws_bytes < layout(n, key_bits, skip).total)
        return fail(HCC_ERR_INVALID, "hcc_sort: workspace too small (see hcc_sort_workspace)");
    if (key_bits <= 32)
        return run_sort<uint32_t>((const uint32_t*)d_keys, key_bits, skip, n, d_perm, (uint32_t*)d_sorted_keys,
                                  (char*)d_ws, stream);
    return run_sort<uint64_t>((const uint64_t*)d_keys, key_bits, skip, n, d_perm, (uint64_t*)d_sorted_keys,
                              (char*)d_ws, stream);
}

hcc_status radix_sort(const void* d_keys, uint32_t key_bits, uint32_t n, uint32_t* d_perm, void* d_sorted_keys,
                      const uint32_t* /*d_vals_in*/, void* d_ws, size_t ws_bytes, hipStream_t stream) {
    return radix_sort_ex(d_keys, key_bits, 0, 0, n, d_perm, d_sorted_keys, d_ws, ws_bytes, stream);
}

}  // namespace hcc
