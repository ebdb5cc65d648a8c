// Stable LSD radix sort of (key, index) pairs for gfx950, 8-bit digits.
//
// Sorting the ray keys as unsigned integers and handing the trace kernel the sorted
// ray indices is the reorder step of the method (Sections 4.2.3 and 5).  Design:
//   1. one read of the keys builds the digit histograms of every pass at once;
//   2. per pass, one kernel ranks a tile of 4096 keys (4 wavefronts x 16 keys per lane)
//      with wavefront ballots: the lanes holding the same digit are found from one
//      ballot per digit bit, and their count below a lane gives its stable rank;
//      the tile's per-digit totals are combined with earlier tiles by a decoupled
//      look-back (tiles are numbered in the order blocks start, so every tile waited
//      on is already running); the tile is reordered in LDS and written out so that
//      equal digits land on consecutive addresses.
// Keys: uint32 (key_bits <= 32) or uint64.  Only bits [0, key_bits) take part.
#include "hcc_internal.h"

#include <mutex>

namespace hcc {
namespace {

constexpr uint32_t kBlock = 256;          // 4 wavefronts
constexpr uint32_t kItems = 16;
constexpr uint32_t kTile = kBlock * kItems;
constexpr uint32_t kRadix = 256;
constexpr uint32_t kMaxPasses = 8;
constexpr uint32_t kFlagAgg = 1u << 30, kFlagIncl = 2u << 30, kCountMask = (1u << 30) - 1u;

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

// Digit histograms of every pass in one read of the keys.  Thread g takes the four consecutive
// keys 4g .. 4g+3 and, per pass, adds each run of equal digits among them with one LDS atomic;
// when all 256 keys of a full wavefront share the digit, one lane adds 256.  Keys are skewed
// and locally coherent (many rays share a code, neighbours often do), so this keeps most
// lanes of a wavefront from hitting one bin in the same atomic.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_hist(const K* __restrict__ keys, uint32_t n, uint32_t key_bits,
                                                 uint32_t skip, uint32_t passes, uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[kMaxPasses * kRadix];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < passes * kRadix; i += kBlock) s_h[i] = 0;
    __syncthreads();
    const uint32_t groups = (n + 3u) / 4u, full = n / 4u;
    const bool aligned = ((uintptr_t)keys & 15u) == 0;
    for (uint32_t base = blockIdx.x * kBlock; base < groups; base += gridDim.x * kBlock) {
        const uint32_t g = base + t;
        // keys of this thread: a prefix of the four is valid
        const uint32_t nv = g < full ? 4u : (g < groups ? n - 4u * g : 0u);
        K kk[4];
        if (nv == 4u && aligned && sizeof(K) == 4) {
            const uint4 q = *reinterpret_cast<const uint4*>(keys + 4 * (size_t)g);
            kk[0] = (K)q.x; kk[1] = (K)q.y; kk[2] = (K)q.z; kk[3] = (K)q.w;
        } else {
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) kk[j] = j < nv ? keys[4 * (size_t)g + j] : K(0);
        }
        // this thread's wavefront covers 64 full groups
        const bool wave_full = (base + (t & ~63u) + 64u) <= full;
        for (uint32_t p = 0; p < passes; ++p) {
            const uint32_t sh = skip + 8u * p;
            const uint32_t msk = (1u << min(8u, key_bits - sh)) - 1u;
            uint32_t d[4];
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) d[j] = (uint32_t)(kk[j] >> sh) & msk;
            uint32_t* h = s_h + p * kRadix;
            const uint32_t v0 = __builtin_amdgcn_readfirstlane(d[0]);
            const bool same = d[0] == v0 && d[1] == v0 && d[2] == v0 && d[3] == v0;
            if (wave_full && __ballot(same) == ~0ull) {
                if ((t & 63u) == 0) atomicAdd(&h[v0], 256u);
                continue;
            }
            uint32_t cur = d[0], run = nv ? 1u : 0u;
#pragma unroll
            for (uint32_t j = 1; j < 4; ++j) {
                if (j < nv) {
                    if (d[j] == cur) {
                        ++run;
                    } else {
                        atomicAdd(&h[cur], run);
                        cur = d[j];
                        run = 1u;
                    }
                }
            }
            if (run) atomicAdd(&h[cur], run);
        }
    }
    __syncthreads();
    for (uint32_t i = t; i < passes * kRadix; i += kBlock)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

template <typename K, bool kIota, bool kWriteKeys>
__global__ __launch_bounds__(kBlock) void k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    K* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n,
                                                    uint32_t shift, uint32_t nbits,
                                                    const uint32_t* __restrict__ hist, uint32_t* lookback,
                                                    uint32_t* counter) {
    __shared__ uint32_t s_whist[4 * kRadix];
    __shared__ uint32_t s_dexcl[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_scan[8];
    __shared__ uint32_t s_tile;
    __shared__ K s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];

    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    if (t == 0) s_tile = atomicAdd(counter, 1u);
    for (uint32_t i = t; i < 4 * kRadix; i += kBlock) s_whist[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t base = tile * kTile + w * (64u * kItems) + lane;
    const uint32_t mask = (1u << nbits) - 1u;
    const uint64_t lt = lanemask_lt();
    uint32_t* wh = s_whist + w * kRadix;

    K k[kItems];
    uint32_t v[kItems];
    uint32_t r[kItems];
#pragma unroll
    for (uint32_t i = 0; i < kItems; ++i) {
        const uint32_t idx = base + i * 64u;
        const bool valid = idx < n;
        k[i] = valid ? kin[idx] : K(0);
        v[i] = kIota ? idx : (valid ? vin[idx] : 0u);
    }
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

    // thread t owns digit t: tile total, per-wavefront exclusive offsets
    const uint32_t d = t;
    const uint32_t c0 = s_whist[d], c1 = s_whist[kRadix + d], c2 = s_whist[2 * kRadix + d],
                   c3 = s_whist[3 * kRadix + d];
    const uint32_t cnt = c0 + c1 + c2 + c3;
    s_whist[d] = 0;
    s_whist[kRadix + d] = c0;
    s_whist[2 * kRadix + d] = c0 + c1;
    s_whist[3 * kRadix + d] = c0 + c1 + c2;

    // decoupled look-back over earlier tiles for digit d
    uint32_t excl = 0;
    uint32_t* mine = lookback + (size_t)tile * kRadix + d;
    if (tile == 0) {
        __hip_atomic_store(mine, kFlagIncl | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(mine, kFlagAgg | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // walk back over the earlier tiles four at a time (four loads in flight per round trip);
        // tile 0 always holds an inclusive prefix, so the walk ends at or above it
        constexpr int kLookWindow = 4;
        int64_t j = (int64_t)tile - 1;
        while (true) {
            uint32_t x[kLookWindow];
#pragma unroll
            for (int q = 0; q < kLookWindow; ++q)
                x[q] = j - q >= 0 ? __hip_atomic_load(lookback + (size_t)(j - q) * kRadix + d, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)
                                  : kFlagIncl;
            int used = kLookWindow;
            bool done = false;
#pragma unroll
            for (int q = 0; q < kLookWindow; ++q) {
                if (done || used < kLookWindow) continue;
                const uint32_t f = x[q] & ~kCountMask;
                if (f == 0) {
                    used = q;          // not yet published: take what came before, poll again
                } else {
                    excl += x[q] & kCountMask;
                    done = f == kFlagIncl;
                }
            }
            if (done) break;
            j -= used;
            if (used < kLookWindow) __builtin_amdgcn_s_sleep(1);
        }
        __hip_atomic_store(mine, kFlagIncl | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t hexcl = block_excl_scan256(hist[d], s_scan);
    const uint32_t dexcl = block_excl_scan256(cnt, s_scan + 4);
    s_gbase[d] = hexcl + excl;
    s_dexcl[d] = dexcl;
    __syncthreads();

#pragma unroll
    for (uint32_t i = 0; i < kItems; ++i) {
        if (base + i * 64u < n) {
            const uint32_t dd = (uint32_t)(k[i] >> shift) & mask;
            const uint32_t pos = s_dexcl[dd] + wh[dd] + r[i];
            s_keys[pos] = k[i];
            s_vals[pos] = v[i];
        }
    }
    __syncthreads();
    const uint32_t count = min(kTile, n - tile * kTile);
    for (uint32_t j = t; j < count; j += kBlock) {
        const K key = s_keys[j];
        const uint32_t dd = (uint32_t)(key >> shift) & mask;
        const uint32_t g = s_gbase[dd] + (j - s_dexcl[dd]);
        if (kWriteKeys) kout[g] = key;
        vout[g] = s_vals[j];
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
    size_t keys_a, keys_b, vals, hist, counters, lookback, total;
};

constexpr Layout layout(uint32_t n, uint32_t key_bits, uint32_t skip = 0) {
    const size_t ks = key_bits <= 32 ? 4 : 8;
    const uint32_t passes = (key_bits - skip + 7) / 8;
    const size_t tiles = ((size_t)n + kTile - 1) / kTile;
    Layout L{};
    size_t off = 0;
    L.keys_a = off; off += align256((size_t)n * ks);
    L.keys_b = off; off += align256((size_t)n * ks);
    L.vals = off; off += align256((size_t)n * 4);
    L.hist = off; off += align256((size_t)kMaxPasses * kRadix * 4);
    L.counters = off; off += align256(kMaxPasses * 4);
    L.lookback = off; off += align256((size_t)passes * tiles * kRadix * 4);
    L.total = off;
    return L;
}

template <typename K>
hcc_status run_sort(const K* keys, uint32_t key_bits, uint32_t skip, uint32_t n, uint32_t* perm, K* sorted_keys,
                    char* ws, hipStream_t stream) {
    const uint32_t passes = (key_bits - skip + 7) / 8;
    const Layout L = layout(n, key_bits, skip);
    const uint32_t tiles = (n + kTile - 1) / kTile;
    uint32_t* hist = (uint32_t*)(ws + L.hist);
    uint32_t* counters = (uint32_t*)(ws + L.counters);
    uint32_t* lookback = (uint32_t*)(ws + L.lookback);
    // zero histogram, counters and look-back state (hist, counters and lookback are contiguous)
    const size_t zero_words = (L.total - L.hist) / 4;
    k_fill_u32<<<dim3((unsigned)std::min<size_t>(1024, (zero_words + 255) / 256)), dim3(256), 0, stream>>>(
        hist, zero_words, 0u);
    const uint32_t hist_blocks = std::min<uint32_t>(2048u, ((n + 3) / 4 + kBlock - 1) / kBlock);
    k_hist<K><<<dim3(hist_blocks), dim3(kBlock), 0, stream>>>(keys, n, key_bits, skip, passes, hist);

    K* final_keys = sorted_keys ? sorted_keys : (K*)(ws + L.keys_a);
    K* other_keys = (K*)(ws + L.keys_b);
    uint32_t* vals_tmp = (uint32_t*)(ws + L.vals);
    const K* kin = keys;
    const uint32_t* vin = nullptr;
    for (uint32_t p = 0; p < passes; ++p) {
        const bool to_final = ((passes - 1 - p) % 2) == 0;
        K* kout = to_final ? final_keys : other_keys;
        uint32_t* vout = to_final ? perm : vals_tmp;
        const bool last = p + 1 == passes;
        const uint32_t shift = skip + 8u * p;
        const uint32_t nb = std::min<uint32_t>(8u, key_bits - shift);
        const uint32_t* h = hist + p * kRadix;
        uint32_t* lb = lookback + (size_t)p * tiles * kRadix;
        uint32_t* ctr = counters + p;
        dim3 grid(tiles), block(kBlock);
        if (p == 0) {
            if (last && !sorted_keys)
                k_scatter<K, true, false><<<grid, block, 0, stream>>>(kin, vin, kout, vout, n, shift, nb, h, lb, ctr);
            else
                k_scatter<K, true, true><<<grid, block, 0, stream>>>(kin, vin, kout, vout, n, shift, nb, h, lb, ctr);
        } else {
            if (last && !sorted_keys)
                k_scatter<K, false, false><<<grid, block, 0, stream>>>(kin, vin, kout, vout, n, shift, nb, h, lb, ctr);
            else
                k_scatter<K, false, true><<<grid, block, 0, stream>>>(kin, vin, kout, vout, n, shift, nb, h, lb, ctr);
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
// whole key range; the zero-initialised parts of the workspace (histograms, tile counters,
// look-back state) are cleared by a kernel on every call, as in every sort.
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
