/*
 * hcc.h -- C ABI of the hierarchy-cut-code ray-reordering library for MI355X (gfx950).
 *
 * The library implements the data-parallel path of Xiang et al., "Faster Ray Tracing
 * through Hierarchy Cut Code" (2023): build a BVH, choose a cut of it, encode each ray
 * as a sorting key, sort the rays by key, and trace the reordered rays.
 *
 * Conventions for every call
 *   - Pointers prefixed d_ are device pointers (hipMalloc'd or from a caching allocator)
 *     owned by the caller; pointers prefixed h_ are host pointers owned by the caller.
 *   - Handles (hcc_bvh, hcc_cut) are owned by the library and freed with *_destroy.
 *   - Calls taking a stream enqueue their device work on it and return without waiting,
 *     unless stated as blocking.  A NULL stream is the default stream.
 *   - Arguments are validated before any work is queued; on an error nothing is written
 *     to the out-parameters and hcc_last_error() (per thread) describes the failure.
 *   - A device fault surfaces as HCC_ERR_DEVICE from the next call that synchronises.
 *   - hcc_encode, hcc_sort and hcc_trace never allocate memory.
 *
 * Data layouts
 *   triangles : n x 9 float32, [v0.xyz v1.xyz v2.xyz] (36 bytes each)
 *   rays      : hcc_ray, 32 bytes: origin, tmin, direction, tmax.  The ray is the segment
 *               o + t d for tmin <= t <= tmax (tmax may be +inf); d need not be unit length.
 *   keys      : uint32 per ray when key_bits <= 32, else uint64.  Bits >= key_bits are 0.
 *   hits      : hcc_hit per ray (closest hit), or one uint8 per ray (any hit), both indexed
 *               by the ORIGINAL ray index whatever permutation the rays were traced in.
 *   node ids  : internal node i -> i (0 <= i < n-1), leaf j (j-th triangle in Morton
 *               order) -> n-1+j.  The root is id 0 (also when n == 1: then it is leaf 0).
 */
#ifndef HCC_H
#define HCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HCC_OK = 0,
    HCC_ERR_INVALID = 1,      /* bad argument (null pointer, size out of range, wrong handle) */
    HCC_ERR_OOM = 2,          /* device or host allocation failed */
    HCC_ERR_DEVICE = 3,       /* HIP runtime error or device fault */
    HCC_ERR_UNSUPPORTED = 4,  /* option not implemented */
    HCC_ERR_BUDGET = 5        /* request refused by an admission budget */
} hcc_status;

typedef enum {
    HCC_KEY_NONE = 0,         /* no key: rays traced in generation order ("NoSort") */
    HCC_KEY_HCC = 1,          /* hierarchy cut code (Section 4.2, Algorithm 1) */
    HCC_KEY_TWOPOINT = 2,     /* origin + estimated end point 6-D Morton code (Section 3.2) */
    HCC_KEY_MLHCC = 3,        /* multi-level hierarchy cut code (Section 4.3), two-level cut */
    HCC_KEY_PPC = 4           /* prefix path code (Section 4.1): forced-order walk, one bit per box test */
} hcc_key_mode;

typedef enum { HCC_TRACE_CLOSEST = 0, HCC_TRACE_ANY = 1 } hcc_trace_mode;

typedef enum {
    HCC_STACK_SCRATCH = 0,    /* per-lane traversal stack in private (scratch) memory (default) */
    HCC_STACK_LDS = 1,        /* BVH2 kernels: whole stack in LDS (64 entries); 4-wide: first 24 in LDS */
    HCC_STACK_SHORT = 2       /* first entries in LDS (BVH2: 16, 4-wide: 16), deeper ones in scratch */
} hcc_stack_mode;

typedef struct hcc_bvh_s* hcc_bvh;
typedef struct hcc_cut_s* hcc_cut;
typedef void* hcc_stream;     /* a hipStream_t */

/* ---------------------------------------------------------------------------------------
 * hcc_set_allocator -- where the library's own device memory comes from (not part of the
 * paper's method; the memory plumbing around it).  By default BVH and cut handles and the
 * build's temporaries use hipMalloc / hipFree, and request servers use stream-ordered
 * hipMallocAsync / hipFreeAsync for their per-launch workspaces.  With hooks installed all
 * of these go through them instead, e.g. a framework's caching allocator:
 *   alloc(bytes, stream, ctx)  returns device memory of at least `bytes` for use on `stream`,
 *                              or NULL, which makes the requesting call fail with HCC_ERR_OOM;
 *   free(ptr, stream, ctx)     takes back a block alloc returned, once no queued work uses it.
 * The setting is process-wide and affects objects created after the call.  Each handle and
 * server keeps the pair it was created with and frees through it, so both functions and ctx
 * must stay valid until those objects are destroyed.  A server calls them from its worker
 * thread.  Both NULL restores the defaults; exactly one NULL is HCC_ERR_INVALID.
 * hcc_encode, hcc_sort and hcc_trace allocate nothing either way.
 */
typedef void* (*hcc_alloc_fn)(size_t bytes, hcc_stream stream, void* ctx);
typedef void (*hcc_free_fn)(void* ptr, hcc_stream stream, void* ctx);
hcc_status hcc_set_allocator(hcc_alloc_fn alloc, hcc_free_fn free_fn, void* ctx);

typedef struct hcc_ray { float ox, oy, oz, tmin, dx, dy, dz, tmax; } hcc_ray;
typedef struct hcc_hit { float t; uint32_t prim; float u, v; } hcc_hit;   /* miss: t = +inf, prim = 0xFFFFFFFF */

/* Launch options of the trace kernel (the autotuner's knobs).  Zero-initialised = defaults. */
typedef struct hcc_trace_opts {
    uint32_t block;           /* one-ray-per-lane launch: threads per block, 64, 128 or 256 (0 = 64) */
    uint32_t stack;           /* hcc_stack_mode */
    uint32_t xcd_remap;       /* 1 = give each XCD a contiguous range of rays / chunks (0 = hardware order);
                                 persistent launches: the static chunk order only (see chunk) */
    uint32_t persistent;      /* 1 = persistent wavefronts that refill idle lanes with new rays */
    uint32_t refill;          /* persistent: refill when at least this many lanes are idle, 1..64 (0 = 16) */
    uint32_t chunk;           /* persistent: consecutive rays a wavefront owns at a time, >= 64 (0 = 256).
                                 A wavefront whose chunk runs out takes the next one from a
                                 per-stream device counter the library keeps (one of 256 slots per
                                 device, taken on the stream's first persistent launch); while
                                 the stream is being captured into a graph, once the slots are
                                 taken, and in hcc_trace_count, wavefront w takes chunks w,
                                 w + waves, w + 2 waves, ... instead.  Results are the same
                                 either way. */
    uint32_t waves;           /* persistent: wavefronts launched (0 = 8192) */
    uint32_t flags;           /* HCC_TRACE_SPECULATE | HCC_TRACE_WIDE | HCC_TRACE_SLAB | HCC_TRACE_SPREAD |
                                 HCC_TRACE_QUANT | HCC_TRACE_PACKET */
} hcc_trace_opts;

/* hcc_trace_opts.flags */
#define HCC_TRACE_SPECULATE 1u  /* persistent BVH2: keep descending while one leaf is postponed */
#define HCC_TRACE_WIDE 2u       /* traverse the 4-wide nodes (the BVH2 collapsed top down, built by
                                   hcc_build_bvh) with persistent wavefronts; refill, chunk, waves,
                                   stack and xcd_remap apply, block does not */
#define HCC_TRACE_SLAB 4u       /* with HCC_TRACE_WIDE: test every child box with the plain slab test.
                                   Without it, rays with a finite origin and finite nonzero direction
                                   components fetch each axis's entry and exit plane by the sign of the
                                   direction instead (the same hit / miss decisions and distances,
                                   fewer instructions; measured faster where the nodes stay in the
                                   caches, slower on scenes far larger than them) */
#define HCC_TRACE_SPREAD 8u     /* persistent launches taking chunks from the stream's counter: the counter
                                   deals the chunks in 64 interleaved streams (take t -> chunk
                                   (t mod 64) * ceil(chunks / 64) + t / 64), so the wavefronts running
                                   together work on 64 parts of the order; same results */
#define HCC_TRACE_QUANT 16u     /* with HCC_TRACE_WIDE: traverse the quantised copy of the 4-wide nodes that
                                   hcc_build_bvh also builds (64 bytes per node instead of 128: each slot's
                                   box as 8-bit steps from the node's corner, rounded outwards, so every
                                   decoded box contains the exact one; the node step reads four 16-byte
                                   words instead of seven).  The traversal then tests a superset of the
                                   boxes the exact nodes pass and finds the same closest or any hit.
                                   HCC_ERR_UNSUPPORTED without HCC_TRACE_WIDE, or for a BVH with a
                                   non-finite box */
#define HCC_TRACE_PACKET 32u    /* with HCC_TRACE_WIDE: wavefront packets instead of one traversal per lane.
                                   Each wavefront takes 64 consecutive rays of the trace order and walks
                                   the 4-wide tree once for all of them: a node is visited when some
                                   lane's child-box test passes, and its fetch is one load shared by the
                                   wavefront.  Pays where the 64 rays are coherent (primary and shadow
                                   rays, reordered rays: the per-warp coherence of Section 3.1); costs
                                   many times more steps on incoherent rays.  The same hits as the
                                   per-lane traversal, except that a lane also tests triangles whose
                                   boxes only other lanes pass, so a ray passing within rounding of a
                                   triangle's edge may report that triangle (as HCC_TRACE_QUANT).
                                   HCC_TRACE_QUANT, HCC_TRACE_SLAB, HCC_TRACE_SPREAD, xcd_remap and
                                   waves apply; chunk (64 rays per packet), refill and stack do not.
                                   HCC_ERR_UNSUPPORTED without HCC_TRACE_WIDE and in hcc_trace_count */

/* ---------------------------------------------------------------------------------------
 * hcc_build_bvh -- linear BVH over n_tris triangles (Section 3.1: the acceleration structure
 * the code is defined on; the builder is the Morton-code LBVH, one triangle per leaf).
 * Steps on the device: scene box; 30-bit Morton code of each triangle's AABB centre
 * (10 bits per axis, x most significant); stable sort by code; binary radix tree over
 * (code << 32 | position) (Karras 2012 numbering); bottom-up boxes; HAD with lambda 0.125.
 * d_tris: device, n_tris x 9 float32, read only during the call.  Blocking: returns when the
 * BVH is complete.  n_tris must be in [1, 2^28].  *out receives a new handle.
 */
hcc_status hcc_build_bvh(const float* d_tris, uint32_t n_tris, hcc_stream stream, hcc_bvh* out);

/* Sizes of a BVH: triangles, nodes (2n-1), scene box (6 floats lo.xyz hi.xyz) and device bytes
 * held.  Any out pointer may be NULL. */
hcc_status hcc_bvh_info(hcc_bvh bvh, uint32_t* n_tris, uint32_t* n_nodes, float* h_scene_box6,
                        size_t* device_bytes);

/* Copy the BVH to host memory (parity checks, inspection).  Blocking.  Any pointer may be NULL.
 * h_child: (n-1) x 2 uint32 unified ids; h_leaf_prim: n uint32 (triangle index of leaf j);
 * h_boxes: (2n-1) x 6 float32 by unified id; h_had: (2n-1) float64 HAD (Eq. 1) with the
 * lambda of the most recent hcc_select_cut (0.125 before the first). */
hcc_status hcc_bvh_export(hcc_bvh bvh, uint32_t* h_child, uint32_t* h_leaf_prim, float* h_boxes, double* h_had);

/* Copy the 4-wide traversal nodes to host memory (parity checks, inspection; the BVH2 collapsed
 * top down, see HCC_TRACE_WIDE and HCC_TRACE_QUANT).  Blocking.  Any pointer may be NULL; call
 * with null buffers first to learn *n_wide (0 for a one-triangle BVH).
 * h_wide: n_wide x 128 bytes, wide node i in level order (the root first): 6 x 4 float32 planes
 *   (lower x of slots 0..3, lower y, lower z, upper x, upper y, upper z), 4 uint32 refs (an
 *   internal member's wide node index; 0x80000000 | leaf index for a triangle, the leaf index as
 *   in h_leaf_prim; 0xFFFFFFFF for an empty slot), 4 uint32 zero.
 * h_quant: n_wide x 64 bytes, the quantised copy: float32 p.x p.y p.z s.x s.y s.z (corner and
 *   power-of-two step per axis), then uint32 step words lower x, upper x, lower y, upper y, lower
 *   z, upper z (slot j in byte j; plane = fmaf(step, s, p) rounded once), then the 4 refs.
 * *quant_ok: 1 when the quantised nodes exist and the quantised traversal is offered. */
hcc_status hcc_bvh_export_wide(hcc_bvh bvh, uint32_t* n_wide, void* h_wide, void* h_quant, uint32_t* quant_ok);

void hcc_bvh_destroy(hcc_bvh bvh);

/* ---------------------------------------------------------------------------------------
 * hcc_select_cut -- choose cut_size nodes of the BVH by Algorithm 2 (Section 4.2.2): a priority
 * queue keyed by HAD (Eq. 1 with the given lambda; the paper uses 0.125) starts at the root;
 * while it holds fewer nodes than the target, the largest-HAD node (ties: smaller id) is
 * removed and replaced by its children, or, if it is a leaf, moved to the cut while the target
 * shrinks by one.  The cut is ordered by HAD descending (ties: id ascending): cut node 0 owns
 * the most significant key bit.  A target above the leaf count yields all leaves.
 * HAD is recomputed on the device when lambda changes; the search runs on the host; the cut's
 * boxes are uploaded on the stream.  Blocking.  cut_size in [1, 2^20], lambda >= 0 and finite.
 */
hcc_status hcc_select_cut(hcc_bvh bvh, uint32_t cut_size, double lambda, hcc_stream stream, hcc_cut* out);

/* Number of nodes in the cut (min(cut_size, n_tris)). */
hcc_status hcc_cut_info(hcc_cut cut, uint32_t* c_eff);

/* Copy the cut to host memory, in bit order: h_ids (c_eff uint32 unified ids), h_had
 * (c_eff float64), h_boxes (c_eff x 6 float32).  Any pointer may be NULL.  Blocking. */
hcc_status hcc_cut_export(hcc_cut cut, uint32_t* h_ids, double* h_had, float* h_boxes);

void hcc_cut_destroy(hcc_cut cut);

/* hcc_select_mlhcc_cut -- two-level cut of the multi-level hierarchy cut code (Section 4.3,
 * Algorithm 3).  Top level: the Algorithm 2 search (largest HAD first, ties by smaller id) over
 * nodes with a sufficient subtree -- at least 'low' leaves, so that each top node can be split
 * into 'low' low-level nodes; a removed node pushes its children with at least 'low' leaves and
 * discards the others, and a node none of whose children qualifies joins the top level as it
 * is.  At most 'top' top nodes (HAD descending); for each, the Algorithm 2 cut of size 'low' of
 * its subtree (HAD descending).  1 <= top, low <= 64, top * low <= 2048.  Blocking.
 * Encode with HCC_KEY_MLHCC and key_bits >= top nodes + low: bit (key_bits-1-i) <=> the ray
 * meets top node i; the representative is the first top node met; bit (low-1-j) <=> the ray
 * meets node j of the representative's low-level cut (zero when no top node is met). */
hcc_status hcc_select_mlhcc_cut(hcc_bvh bvh, uint32_t top, uint32_t low, double lambda, hcc_stream stream,
                                hcc_cut* out);

/* hcc_grid_cut -- the regular-grid control encoding (Section 5): a "cut" whose boxes are the
 * cells of a uniform gx x gy x gz grid over the scene box (boundaries lo + ext*i/g computed in
 * double, rounded to float; cells numbered x fastest, then y, then z; cell 0 = most significant
 * bit).  Encode with HCC_KEY_HCC.  1 <= gx*gy*gz <= 64.  Blocking. */
hcc_status hcc_grid_cut(hcc_bvh bvh, uint32_t gx, uint32_t gy, uint32_t gz, hcc_stream stream, hcc_cut* out);

/* Kind of a cut (0 Algorithm 2 cut, 1 two-level cut, 2 regular grid), its (top-level) size and,
 * for a two-level cut, the low-level size.  Any out pointer may be NULL. */
hcc_status hcc_cut_shape(hcc_cut cut, uint32_t* kind, uint32_t* top, uint32_t* low);

/* Low level of a two-level cut: h_low_ids (top x low uint32 node ids, row i for top node i) and
 * h_low_boxes (top x low x 6 float32).  Either pointer may be NULL. */
hcc_status hcc_cut_export_low(hcc_cut cut, uint32_t* h_low_ids, float* h_low_boxes);

/* ---------------------------------------------------------------------------------------
 * hcc_encode -- one sorting key per ray.
 *   HCC_KEY_HCC (Algorithm 1, Section 4.2.1): bit (key_bits-1-i) is set iff the ray's segment
 *     meets the box of cut node i, for i < min(c_eff, key_bits); the cut's boxes are staged in
 *     LDS once per block.  Requires cut (from this bvh).
 *   HCC_KEY_TWOPOINT (Section 3.2 / Section 5): 6-D Morton code of the origin and the point at
 *     distance 0.25 x (largest scene extent) along the normalised direction (clipped to the
 *     segment); dimension d of (ox,oy,oz,ex,ey,ez) gets key_bits/6 bits plus one if
 *     d < key_bits % 6, interleaved from the top level down.  cut is ignored.
 *   HCC_KEY_MLHCC (Section 4.3): needs a two-level cut (hcc_select_mlhcc_cut); see there.
 *   HCC_KEY_PPC (Section 4.1): every ray walks the BVH in one forced order (expanding a node
 *     tests child 0 then child 1; child 0's subtree first; only met internal children are
 *     expanded) over its own segment; box test number j (from 0) sets bit (key_bits-1-j) when
 *     met; the walk stops after key_bits tests, and bits of a walk that ends earlier stay 0.
 *     A one-triangle BVH makes one test, of the root leaf's box.  cut is ignored.
 * key_bits in [1, 64]; d_keys: uint32[n] if key_bits <= 32 else uint64[n].  n may be 0.
 */
hcc_status hcc_encode(hcc_bvh bvh, hcc_cut cut, hcc_key_mode mode, uint32_t key_bits, const hcc_ray* d_rays,
                      uint32_t n, void* d_keys, hcc_stream stream);

/* ---------------------------------------------------------------------------------------
 * hcc_sort -- stable ascending sort of the keys as unsigned integers (Section 4.2.3), output
 * as the permutation of ray indices (Section 5: the trace kernel fetches rays through it):
 * d_perm[k] = index of the k-th smallest key, equal keys in input order.  LSD radix sort,
 * ceil(key_bits/8) passes of 8 bits.  d_sorted_keys (nullable) receives the sorted keys.
 * d_ws must hold hcc_sort_workspace(n, key_bits) bytes, 256-byte aligned.  n < 2^30.
 */
hcc_status hcc_sort_workspace(uint32_t n, uint32_t key_bits, size_t* bytes);
hcc_status hcc_sort(const void* d_keys, uint32_t key_bits, uint32_t n, uint32_t* d_perm, void* d_sorted_keys,
                    void* d_ws, size_t ws_bytes, hcc_stream stream);

/* hcc_sort_static -- hcc_sort without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops that must not call hipMalloc,
 * harnesses that forbid it).  It allocates nothing: its workspace is a fixed array in the
 * library's device memory, one per GPU (hcc_sort_static_bytes: about 21 MB, held from the
 * library's load until the process ends), and it runs the kernels of hcc_sort.  Same keys,
 * permutation, sorted keys and stream ordering as hcc_sort.  n <= HCC_SORT_STATIC_MAX_KEYS,
 * else HCC_ERR_INVALID (use hcc_sort with a caller workspace).  Every call on one GPU shares
 * that GPU's array: calls that overlap on a GPU (on other streams, or from other threads
 * without ordering between them) race and give wrong results; order them on one stream. */
#define HCC_SORT_STATIC_MAX_KEYS 1048576u
hcc_status hcc_sort_static(const void* d_keys, uint32_t key_bits, uint32_t n, uint32_t* d_perm,
                           void* d_sorted_keys, hcc_stream stream);
hcc_status hcc_sort_static_bytes(size_t* bytes);

/* hcc_sort_ex -- shorter sorts for the reorder overhead (Sections 6.5 and 6.6.1: rays within one warp need
 * no order among themselves, so the sort may skip the key's last bits or stop early).
 *   skip_bits: the low skip_bits bits take no part: stable ascending by key >> skip_bits, in
 *              ceil((key_bits - skip_bits) / 8) passes.  0 <= skip_bits < key_bits.
 *   tile:      0 = one sort over all n keys (workspace as for hcc_sort with the same n and
 *              key_bits); else a power of two in [256, 4096]: consecutive groups of `tile` keys
 *              (the last one ragged) are each sorted stably on their own, in one kernel with no
 *              workspace (d_ws may be NULL), and no index leaves its group.
 * d_perm and d_sorted_keys as for hcc_sort (sorted keys keep their skipped bits). */
hcc_status hcc_sort_ex(const void* d_keys, uint32_t key_bits, uint32_t skip_bits, uint32_t tile, uint32_t n,
                       uint32_t* d_perm, void* d_sorted_keys, void* d_ws, size_t ws_bytes, hcc_stream stream);

/* ---------------------------------------------------------------------------------------
 * hcc_trace -- BVH traversal of n rays taken in the order d_perm (NULL = 0..n-1), Section 5.
 *   HCC_TRACE_CLOSEST: d_hits[r] = the hit with the smallest (t, triangle index) among all
 *     triangles met with tmin < t < tmax (Moller-Trumbore, double sided); miss: t = +inf,
 *     prim = 0xFFFFFFFF, u = v = 0.
 *   HCC_TRACE_ANY: d_occluded[r] = 1 iff some triangle is met with tmin < t < tmax.
 * Results are written at the original ray index r = d_perm[k].  opts may be NULL (defaults).
 */
hcc_status hcc_trace(hcc_bvh bvh, const hcc_ray* d_rays, const uint32_t* d_perm, uint32_t n, hcc_trace_mode mode,
                     hcc_hit* d_hits, uint8_t* d_occluded, hcc_stream stream);
hcc_status hcc_trace_ex(hcc_bvh bvh, const hcc_ray* d_rays, const uint32_t* d_perm, uint32_t n, hcc_trace_mode mode,
                        hcc_hit* d_hits, uint8_t* d_occluded, const hcc_trace_opts* opts, hcc_stream stream);

/* hcc_trace_count -- hcc_trace_ex plus fetch counting, for the roofline's algorithmic bytes.
 * The same launch (persistent or HCC_TRACE_WIDE options only, scratch stack; other options
 * give HCC_ERR_UNSUPPORTED) also counts, at each lockstep iteration of each wavefront, the
 * distinct nodes fetched by its stepping lanes, and at each leaf batch the distinct triangles
 * fetched; it ADDS the totals to d_counts[0] (node fetches) and d_counts[1] (triangle fetches),
 * device uint64, zeroed by the caller.  Results are those of hcc_trace_ex; it runs slower. */
hcc_status hcc_trace_count(hcc_bvh bvh, const hcc_ray* d_rays, const uint32_t* d_perm, uint32_t n, hcc_trace_mode mode,
                           hcc_hit* d_hits, uint8_t* d_occluded, const hcc_trace_opts* opts, uint64_t* d_counts,
                           hcc_stream stream);

/* Measurement variant of hcc_trace (same results, slower): also counts, per ray, the BVH nodes
 * fetched (d_nodes, nullable) and triangles tested (d_tris, nullable), and per wavefront of 64
 * consecutive rays in trace order the distinct node and triangle fetches summed over its
 * lockstep iterations (d_wave_nodes, d_wave_tris: ceil(n/64) uint32 each, required; cleared by
 * the call).  Always uses 64-lane blocks with the scratch stack and hardware block order. */
hcc_status hcc_trace_stats(hcc_bvh bvh, const hcc_ray* d_rays, const uint32_t* d_perm, uint32_t n,
                           hcc_trace_mode mode, hcc_hit* d_hits, uint8_t* d_occluded, uint32_t* d_nodes,
                           uint32_t* d_tris, uint32_t* d_wave_nodes, uint32_t* d_wave_tris, hcc_stream stream);

/* ---------------------------------------------------------------------------------------
 * Batched engine: encode + sort + trace of many ray batches of different sizes over several
 * resident scenes in ONE persistent launch (not in the paper: the engine around its path).
 * Each batch is sorted on its own (stable, by its own keys) and traced through its own
 * permutation, exactly as hcc_encode + hcc_sort + hcc_trace would do it batch by batch, so
 * the results are identical to that sequence.
 */
typedef struct hcc_batch_desc {
    hcc_bvh bvh;              /* scene of the batch */
    hcc_cut cut;              /* cut of that scene (HCC_KEY_HCC); ignored otherwise */
    const hcc_ray* d_rays;    /* device, n rays */
    uint32_t n;               /* rays in the batch, < 2^30 (0 allowed) */
    uint32_t mode;            /* hcc_trace_mode */
    hcc_hit* d_hits;          /* closest hit: n records, by original index within the batch */
    uint8_t* d_occluded;      /* any hit: n flags, by original index within the batch */
} hcc_batch_desc;

typedef struct hcc_batch_opts {
    uint32_t chunk;           /* rays per trace item (>= 64; 0 = 256) */
    uint32_t refill;          /* lane refill threshold 1..64 (0 = 32) */
    uint32_t waves;           /* persistent wavefronts launched (0 = 8192) */
    uint32_t flags;           /* HCC_TRACE_WIDE: trace over the 4-wide nodes, HCC_TRACE_SLAB as for
                                 hcc_trace_opts, HCC_TRACE_QUANT (with HCC_TRACE_WIDE): the quantised
                                 4-wide nodes of each scene that has them; other bits must be 0 */
    uint32_t direct_min;      /* 0 = every batch in the one engine launch (default); else >= 65536:
                                 batches of at least this many rays run afterwards through the
                                 full-device encode / sort / trace kernels on the same stream */
    uint32_t stack;           /* stack placement of the 4-wide trace phase: 0 or HCC_STACK_SHORT = the
                                 first 12 entries per lane in LDS, deeper ones in scratch (default);
                                 HCC_STACK_LDS = the first 24 in LDS; 3 = every entry in scratch.
                                 The BVH2 trace phase keeps its stack in scratch. */
} hcc_batch_opts;

#define HCC_BATCH_STACK_SCRATCH 3u   /* hcc_batch_opts.stack: the 4-wide trace phase's stack in scratch only */

/* Device workspace needed by hcc_batch_run for this batch list, key mode and key length (for
 * any opts.direct_min). */
hcc_status hcc_batch_workspace(const hcc_batch_desc* batches, uint32_t nb, hcc_key_mode mode, uint32_t key_bits,
                               size_t* bytes);

/* Run the batch list in one persistent launch on the stream (mode HCC_KEY_NONE: trace only, in
 * generation order).  The host copies a small descriptor table to the workspace and waits for
 * that copy; the launch itself is asynchronous.  d_ws: hcc_batch_workspace bytes, 256-byte
 * aligned, not used by another call until this one has finished.  opts may be NULL. */
hcc_status hcc_batch_run(const hcc_batch_desc* batches, uint32_t nb, hcc_key_mode mode, uint32_t key_bits,
                         const hcc_batch_opts* opts, void* d_ws, size_t ws_bytes, hcc_stream stream);

/* Wait for the stream, then report in *h_ok whether the last hcc_batch_run on this workspace
 * resolved every dependency inside its launch (1), or whether a bounded wait gave up (0: the
 * results of that run are not valid; this indicates a library fault, never a user error). */
hcc_status hcc_batch_check(const void* d_ws, hcc_stream stream, uint32_t* h_ok);

/* Inspection of a finished hcc_batch_run (parity checks of the in-launch encode and sort):
 * stream-ordered copies of batch `batch`'s final permutation (d_perm: n uint32, the batch's ray
 * indices in sorted order) and of its keys in that order (d_sorted_keys: n keys, uint32 when
 * key_bits <= 32 else uint64), read from d_ws as the last run left it.  Pass the batch list,
 * mode, key length and options of that run; another call on d_ws in between invalidates the
 * result.  Either output may be NULL.  HCC_ERR_UNSUPPORTED for mode HCC_KEY_NONE. */
hcc_status hcc_batch_export(const hcc_batch_desc* batches, uint32_t nb, hcc_key_mode mode, uint32_t key_bits,
                            const hcc_batch_opts* opts, const void* d_ws, size_t ws_bytes, uint32_t batch,
                            uint32_t* d_perm, void* d_sorted_keys, hcc_stream stream);

/* ---------------------------------------------------------------------------------------
 * Request server with continuous batching (not in the paper: serving around its path).
 * A worker thread admits queued requests in arrival order while the device ray-state budget
 * and the slot limit allow, launches each set of newly admitted requests on the next of its
 * streams (so later requests overlap with earlier ones still running) -- the small ones together
 * as one engine batch, each large one (direct_min), or a small one admitted alone, through the
 * full-device kernels -- and retires them when their completion events fire.  A request's budget charge is its rays and
 * results plus the engine workspace for its size.  Results are exactly those of a lone
 * hcc_encode + hcc_sort + hcc_trace of the request.  plain = 1 runs one request at a time
 * through those three calls instead (the baseline).  Buffers named in a request stay owned by
 * the caller and must stay valid until the request is done or cancelled.
 */
typedef struct hcc_server_s* hcc_server;

typedef struct hcc_server_opts {
    uint64_t budget_bytes;    /* device bytes of admitted requests (0 = 64 GiB) */
    uint32_t max_inflight;    /* admitted requests at once (0 = 64) */
    uint32_t max_group;       /* requests per launch (0 = 16) */
    uint32_t streams;         /* HIP streams used for launches, <= 32 (0 = 4) */
    uint32_t key_mode;        /* hcc_key_mode for every request */
    uint32_t key_bits;        /* 1..64 (0 = 32) */
    uint32_t plain;           /* 1 = one request at a time through encode / sort / trace */
    uint32_t graphs;          /* 1 = launch each group through a captured HIP graph (table copy,
                                 counter clear, engine) kept per launch slot; 0 = three calls */
    uint32_t direct_min;      /* continuous mode: a request of at least this many rays runs through
                                 the full-device encode / sort / trace kernels on its own stream
                                 instead of the engine (0 = 65536; 0xFFFFFFFF = never, and then
                                 also a small request admitted alone shares the engine path) */
    hcc_batch_opts batch;     /* engine options */
} hcc_server_opts;

typedef struct hcc_server_stats {
    uint64_t launches, completed, queued, running, used_bytes;
} hcc_server_counters;

enum { HCC_REQ_QUEUED = 0, HCC_REQ_RUNNING = 1, HCC_REQ_DONE = 2, HCC_REQ_CANCELLED = 3, HCC_REQ_FAILED = 4 };

hcc_status hcc_server_create(const hcc_server_opts* opts, hcc_server* out);
/* Queue a request; HCC_ERR_BUDGET if it alone needs more than the whole budget. */
hcc_status hcc_server_submit(hcc_server server, const hcc_batch_desc* request, uint64_t* id);
/* State of a request (HCC_REQ_*) and, once done, its latency from submission in microseconds. */
hcc_status hcc_server_poll(hcc_server server, uint64_t id, uint32_t* state, double* latency_us);
/* Cancel a request that has not been admitted yet (HCC_ERR_INVALID once it has). */
hcc_status hcc_server_cancel(hcc_server server, uint64_t id);
/* Block until every submitted request is done or cancelled. */
hcc_status hcc_server_drain(hcc_server server);
hcc_status hcc_server_stats(hcc_server server, hcc_server_counters* out);
/* Cancels queued requests, waits for admitted ones, releases the server. */
void hcc_server_destroy(hcc_server server);

/* Text of the last error on the calling thread ("" if none). */
const char* hcc_last_error(void);
const char* hcc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HCC_H */
