// C ABI entry points: argument validation, handle management, the host-side cut search
// (Algorithm 2), and dispatch to the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "hcc_internal.h"

namespace hcc {

// defined in the kernel translation units
hcc_status build_bvh(const float* d_tris, uint32_t n, hipStream_t stream, hcc_bvh_s** out);
void free_bvh(hcc_bvh_s* b);
hcc_status recompute_had(hcc_bvh_s* b, double lambda, hipStream_t stream);
hcc_status encode_hcc(const hcc_cut_s* cut, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                      hipStream_t stream);
hcc_status encode_mlhcc(const hcc_cut_s* cut, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                        hipStream_t stream);
hcc_status encode_twopoint(const hcc_bvh_s* bvh, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n,
                           void* d_keys, hipStream_t stream);
hcc_status encode_ppc(const hcc_bvh_s* bvh, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                      hipStream_t stream);
hcc_status trace(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                 hcc_hit* hits, uint8_t* occ, const hcc_trace_opts& o, hipStream_t s);
hcc_status trace_stats(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                       hcc_hit* hits, uint8_t* occ, uint32_t* cn, uint32_t* ct, uint32_t* wn, uint32_t* wt,
                       hipStream_t s);
hcc_status trace_count(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                       hcc_hit* hits, uint8_t* occ, const hcc_trace_opts& o, unsigned long long* counts,
                       hipStream_t s);
hcc_status fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
hcc_status batch_workspace(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits, size_t* bytes);
hcc_status batch_run(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits, const hcc_batch_opts& o,
                     void* d_ws, size_t ws_bytes, hipStream_t stream);
hcc_status batch_check(const void* d_ws, hipStream_t stream, uint32_t* ok);
hcc_status batch_export(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                        const hcc_batch_opts& o, const void* d_ws, size_t ws_bytes, uint32_t b, uint32_t* d_perm,
                        void* d_sorted_keys, hipStream_t stream);

namespace {
thread_local std::string g_error;
std::mutex g_alloc_mu;
Allocator g_alloc;
}

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

void set_error(const std::string& msg) { g_error = msg; }

hcc_status fail(hcc_status st, const std::string& msg) {
    g_error = msg;
    return st;
}

hcc_status hip_fail(hipError_t e, const char* what) {
    g_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? HCC_ERR_OOM : HCC_ERR_DEVICE;
}

namespace {

bool valid_bvh(const hcc_bvh_s* b) { return b && b->magic == 0x6863636276680001ull; }
bool valid_cut(const hcc_cut_s* c) { return c && c->magic == 0x6863636375740001ull; }

hcc_status ensure_host_mirror(hcc_bvh_s* b, hipStream_t stream) {
    if (b->h_had_lambda == b->had_lambda && b->h_had.size() == 2 * (size_t)b->n - 1) return HCC_OK;
    b->h_child.resize(2 * (size_t)b->n_int);
    b->h_had.resize(2 * (size_t)b->n - 1);
    if (b->n_int)
        HCC_HIP(hipMemcpyAsync(b->h_child.data(), b->child, sizeof(uint32_t) * b->h_child.size(),
                               hipMemcpyDeviceToHost, stream));
    HCC_HIP(hipMemcpyAsync(b->h_had.data(), b->had, sizeof(double) * b->h_had.size(), hipMemcpyDeviceToHost, stream));
    HCC_HIP(hipStreamSynchronize(stream));
    b->h_had_lambda = b->had_lambda;
    return HCC_OK;
}

// Algorithm 2 with a binary heap ordered by (HAD descending, id ascending).
std::vector<uint32_t> cut_search(const hcc_bvh_s* b, uint32_t cut_size, uint32_t root = 0) {
    const std::vector<double>& had = b->h_had;
    auto lower = [&](uint32_t x, uint32_t y) {   // true if x has lower priority than y
        if (had[x] != had[y]) return had[x] < had[y];
        return x > y;
    };
    std::priority_queue<uint32_t, std::vector<uint32_t>, decltype(lower)> q(lower);
    std::vector<uint32_t> cut;
    int64_t max_q = cut_size;
    q.push(root);
    while ((int64_t)q.size() < max_q && !q.empty()) {
        const uint32_t node = q.top();
        q.pop();
        if (b->n_int == 0 || node >= b->n_int) {
            cut.push_back(node);
            --max_q;
        } else {
            q.push(b->h_child[2 * (size_t)node]);
            q.push(b->h_child[2 * (size_t)node + 1]);
        }
    }
    while (!q.empty()) {
        cut.push_back(q.top());
        q.pop();
    }
    std::sort(cut.begin(), cut.end(), [&](uint32_t x, uint32_t y) {
        if (had[x] != had[y]) return had[x] > had[y];
        return x < y;
    });
    return cut;
}

inline hipStream_t S(hcc_stream s) { return (hipStream_t)s; }

// Leaves below every node (post-order over the host mirror).
void ensure_leaf_counts(hcc_bvh_s* b) {
    const size_t nn = 2 * (size_t)b->n - 1;
    if (b->h_leaves.size() == nn) return;
    b->h_leaves.assign(nn, 1);
    if (b->n_int == 0) return;
    // children of internal node i have ids > i is not guaranteed, so walk an explicit stack
    std::vector<uint32_t> order;
    order.reserve(b->n_int);
    std::vector<uint32_t> st{0};
    while (!st.empty()) {
        const uint32_t x = st.back();
        st.pop_back();
        order.push_back(x);
        for (int c = 0; c < 2; ++c) {
            const uint32_t ch = b->h_child[2 * (size_t)x + c];
            if (ch < b->n_int) st.push_back(ch);
        }
    }
    for (size_t k = order.size(); k-- > 0;) {
        const uint32_t x = order[k];
        b->h_leaves[x] = b->h_leaves[b->h_child[2 * (size_t)x]] + b->h_leaves[b->h_child[2 * (size_t)x + 1]];
    }
}

// Two-level cut (Alg. 3): a node removed from the queue pushes its children that have at least
// 'low' leaves; if none has, the node itself joins the top-level list and the target shrinks.
std::vector<uint32_t> mlhcc_top_search(const hcc_bvh_s* b, uint32_t top, uint32_t low) {
    const std::vector<double>& had = b->h_had;
    auto lower = [&](uint32_t x, uint32_t y) {
        if (had[x] != had[y]) return had[x] < had[y];
        return x > y;
    };
    std::priority_queue<uint32_t, std::vector<uint32_t>, decltype(lower)> q(lower);
    std::vector<uint32_t> out;
    int64_t max_q = top;
    if (b->h_leaves[0] >= low) q.push(0);
    while ((int64_t)q.size() < max_q && !q.empty()) {
        const uint32_t node = q.top();
        q.pop();
        int pushed = 0;
        if (node < b->n_int) {
            for (int c = 0; c < 2; ++c) {
                const uint32_t ch = b->h_child[2 * (size_t)node + c];
                if (b->h_leaves[ch] >= low) {
                    q.push(ch);
                    ++pushed;
                }
            }
        }
        if (!pushed) {
            out.push_back(node);
            --max_q;
        }
    }
    while (!q.empty()) {
        out.push_back(q.top());
        q.pop();
    }
    std::sort(out.begin(), out.end(), [&](uint32_t x, uint32_t y) {
        if (had[x] != had[y]) return had[x] > had[y];
        return x < y;
    });
    return out;
}

hcc_status download_boxes(const hcc_bvh_s* b, std::vector<float>& all) {
    all.resize(6 * (2 * (size_t)b->n - 1));
    HCC_HIP(hipMemcpy(all.data(), b->boxes, sizeof(float) * all.size(), hipMemcpyDeviceToHost));
    return HCC_OK;
}

// Upload a cut's boxes (top/cut boxes, then low boxes) and hand out the handle.
hcc_status finish_cut(hcc_cut_s* c, hipStream_t stream, hcc_cut* out) {
    const size_t nb = c->boxes.size() / 6 + c->low_boxes.size() / 6;
    std::vector<CutBox> up(std::max<size_t>(nb, 1));
    for (size_t i = 0; i < c->boxes.size() / 6; ++i) {
        const float* bx = &c->boxes[6 * i];
        up[i].lo = make_float4(bx[0], bx[1], bx[2], 0.0f);
        up[i].hi = make_float4(bx[3], bx[4], bx[5], 0.0f);
    }
    const size_t off = c->boxes.size() / 6;
    for (size_t i = 0; i < c->low_boxes.size() / 6; ++i) {
        const float* bx = &c->low_boxes[6 * i];
        up[off + i].lo = make_float4(bx[0], bx[1], bx[2], 0.0f);
        up[off + i].hi = make_float4(bx[3], bx[4], bx[5], 0.0f);
    }
    c->alloc = current_allocator();
    c->d_boxes = (CutBox*)c->alloc.get(sizeof(CutBox) * up.size(), stream);
    if (!c->d_boxes) {
        delete c;
        return fail(HCC_ERR_OOM, "device allocation failed for the cut's boxes");
    }
    hipError_t e = hipMemcpyAsync(c->d_boxes, up.data(), sizeof(CutBox) * up.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        c->alloc.put(c->d_boxes, stream);
        delete c;
        return hip_fail(e, "cut upload");
    }
    *out = c;
    return HCC_OK;
}

}  // namespace
}  // namespace hcc

using namespace hcc;

extern "C" {

__attribute__((visibility("default"))) hcc_status hcc_set_allocator(hcc_alloc_fn alloc, hcc_free_fn free_fn,
                                                                    void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(HCC_ERR_INVALID, "hcc_set_allocator: give both functions or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.release = free_fn;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return HCC_OK;
}

__attribute__((visibility("default"))) const char* hcc_last_error(void) { return g_error.c_str(); }

__attribute__((visibility("default"))) const char* hcc_version(void) { return "hcc-gfx950 0.1"; }

__attribute__((visibility("default"))) hcc_status hcc_build_bvh(const float* d_tris, uint32_t n_tris,
                                                                hcc_stream stream, hcc_bvh* out) {
    hcc::Range range("hcc_build_bvh");
    if (!d_tris || !out) return fail(HCC_ERR_INVALID, "hcc_build_bvh: null pointer");
    if (n_tris == 0 || n_tris > (1u << 28)) return fail(HCC_ERR_INVALID, "hcc_build_bvh: n_tris must be in [1, 2^28]");
    hcc_bvh_s* b = nullptr;
    hcc_status st = build_bvh(d_tris, n_tris, S(stream), &b);
    if (st != HCC_OK) return st;
    *out = b;
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_bvh_info(hcc_bvh bvh, uint32_t* n_tris, uint32_t* n_nodes,
                                                               float* h_scene_box6, size_t* device_bytes) {
    if (!valid_bvh(bvh)) return fail(HCC_ERR_INVALID, "hcc_bvh_info: invalid handle");
    if (n_tris) *n_tris = bvh->n;
    if (n_nodes) *n_nodes = 2 * bvh->n - 1;
    if (h_scene_box6) std::memcpy(h_scene_box6, bvh->scene_box, sizeof(bvh->scene_box));
    if (device_bytes) *device_bytes = bvh->bytes;
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_bvh_export(hcc_bvh bvh, uint32_t* h_child, uint32_t* h_leaf_prim,
                                                                 float* h_boxes, double* h_had) {
    if (!valid_bvh(bvh)) return fail(HCC_ERR_INVALID, "hcc_bvh_export: invalid handle");
    const size_t nn = 2 * (size_t)bvh->n - 1;
    if (h_child && bvh->n_int)
        HCC_HIP(hipMemcpy(h_child, bvh->child, sizeof(uint32_t) * 2 * bvh->n_int, hipMemcpyDeviceToHost));
    if (h_leaf_prim) HCC_HIP(hipMemcpy(h_leaf_prim, bvh->leaf_prim, sizeof(uint32_t) * bvh->n, hipMemcpyDeviceToHost));
    if (h_boxes) HCC_HIP(hipMemcpy(h_boxes, bvh->boxes, sizeof(float) * 6 * nn, hipMemcpyDeviceToHost));
    if (h_had) HCC_HIP(hipMemcpy(h_had, bvh->had, sizeof(double) * nn, hipMemcpyDeviceToHost));
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_bvh_export_wide(hcc_bvh bvh, uint32_t* n_wide, void* h_wide,
                                                                      void* h_quant, uint32_t* quant_ok) {
    if (!valid_bvh(bvh)) return fail(HCC_ERR_INVALID, "hcc_bvh_export_wide: invalid handle");
    if (n_wide) *n_wide = bvh->n_wide;
    if (quant_ok) *quant_ok = bvh->quant_ok ? 1u : 0u;
    if (h_wide && bvh->n_wide)
        HCC_HIP(hipMemcpy(h_wide, bvh->wnodes, sizeof(hcc::Node4) * bvh->n_wide, hipMemcpyDeviceToHost));
    if (h_quant && bvh->n_wide) {
        if (bvh->qnodes)
            HCC_HIP(hipMemcpy(h_quant, bvh->qnodes, sizeof(hcc::Node4Q) * bvh->n_wide, hipMemcpyDeviceToHost));
        else
            std::memset(h_quant, 0, sizeof(hcc::Node4Q) * bvh->n_wide);
    }
    return HCC_OK;
}

__attribute__((visibility("default"))) void hcc_bvh_destroy(hcc_bvh bvh) {
    if (valid_bvh(bvh)) free_bvh(bvh);
}

__attribute__((visibility("default"))) hcc_status hcc_select_cut(hcc_bvh bvh, uint32_t cut_size, double lambda,
                                                                 hcc_stream stream, hcc_cut* out) {
    hcc::Range range("hcc_select_cut");
    if (!valid_bvh(bvh) || !out) return fail(HCC_ERR_INVALID, "hcc_select_cut: invalid handle or null out");
    if (cut_size == 0 || cut_size > (1u << 20)) return fail(HCC_ERR_INVALID, "hcc_select_cut: cut_size must be in [1, 2^20]");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(HCC_ERR_INVALID, "hcc_select_cut: lambda must be finite and >= 0");
    hcc_status st;
    if (lambda != bvh->had_lambda) {
        st = recompute_had(bvh, lambda, S(stream));
        if (st != HCC_OK) return st;
    }
    st = ensure_host_mirror(bvh, S(stream));
    if (st != HCC_OK) return st;
    std::vector<uint32_t> ids = cut_search(bvh, cut_size);
    hcc_cut_s* c = new hcc_cut_s();
    c->bvh = bvh;
    c->c_eff = (uint32_t)ids.size();
    c->ids = ids;
    std::vector<float> all;
    if ((st = download_boxes(bvh, all)) != HCC_OK) {
        delete c;
        return st;
    }
    for (uint32_t id : ids) {
        c->had.push_back(bvh->h_had[id]);
        c->boxes.insert(c->boxes.end(), &all[6 * (size_t)id], &all[6 * (size_t)id] + 6);
    }
    return finish_cut(c, S(stream), out);
}

__attribute__((visibility("default"))) hcc_status hcc_cut_info(hcc_cut cut, uint32_t* c_eff) {
    if (!valid_cut(cut) || !c_eff) return fail(HCC_ERR_INVALID, "hcc_cut_info: invalid handle");
    *c_eff = cut->c_eff;
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_cut_export(hcc_cut cut, uint32_t* h_ids, double* h_had,
                                                                 float* h_boxes) {
    if (!valid_cut(cut)) return fail(HCC_ERR_INVALID, "hcc_cut_export: invalid handle");
    if (h_ids) std::memcpy(h_ids, cut->ids.data(), sizeof(uint32_t) * cut->c_eff);
    if (h_had) std::memcpy(h_had, cut->had.data(), sizeof(double) * cut->c_eff);
    if (h_boxes) std::memcpy(h_boxes, cut->boxes.data(), sizeof(float) * 6 * cut->c_eff);
    return HCC_OK;
}

__attribute__((visibility("default"))) void hcc_cut_destroy(hcc_cut cut) {
    if (!valid_cut(cut)) return;
    cut->alloc.put(cut->d_boxes, nullptr);
    cut->magic = 0;
    delete cut;
}

__attribute__((visibility("default"))) hcc_status hcc_encode(hcc_bvh bvh, hcc_cut cut, hcc_key_mode mode,
                                                             uint32_t key_bits, const hcc_ray* d_rays, uint32_t n,
                                                             void* d_keys, hcc_stream stream) {
    hcc::Range range("hcc_encode");
    if (!valid_bvh(bvh)) return fail(HCC_ERR_INVALID, "hcc_encode: invalid bvh handle");
    if (key_bits < 1 || key_bits > 64) return fail(HCC_ERR_INVALID, "hcc_encode: key_bits must be in [1, 64]");
    if (n == 0) return HCC_OK;
    if (!d_rays || !d_keys) return fail(HCC_ERR_INVALID, "hcc_encode: null pointer");
    switch (mode) {
        case HCC_KEY_HCC:
            if (!valid_cut(cut)) return fail(HCC_ERR_INVALID, "hcc_encode: HCC needs a cut");
            if (cut->bvh != bvh) return fail(HCC_ERR_INVALID, "hcc_encode: cut belongs to another BVH");
            if (cut->kind == 1) return fail(HCC_ERR_INVALID, "hcc_encode: a two-level cut needs HCC_KEY_MLHCC");
            return encode_hcc(cut, key_bits, d_rays, n, d_keys, S(stream));
        case HCC_KEY_MLHCC:
            if (!valid_cut(cut) || cut->kind != 1) return fail(HCC_ERR_INVALID, "hcc_encode: MLHCC needs a two-level cut");
            if (cut->bvh != bvh) return fail(HCC_ERR_INVALID, "hcc_encode: cut belongs to another BVH");
            if (key_bits < cut->low + cut->c_eff)
                return fail(HCC_ERR_INVALID, "hcc_encode: key_bits must be at least top nodes + low nodes");
            return encode_mlhcc(cut, key_bits, d_rays, n, d_keys, S(stream));
        case HCC_KEY_TWOPOINT:
            return encode_twopoint(bvh, key_bits, d_rays, n, d_keys, S(stream));
        case HCC_KEY_PPC:
            return encode_ppc(bvh, key_bits, d_rays, n, d_keys, S(stream));
        default:
            return fail(HCC_ERR_INVALID, "hcc_encode: mode must be HCC_KEY_HCC, HCC_KEY_TWOPOINT, HCC_KEY_MLHCC or HCC_KEY_PPC");
    }
}

__attribute__((visibility("default"))) hcc_status hcc_sort_workspace(uint32_t n, uint32_t key_bits, size_t* bytes) {
    if (!bytes) return fail(HCC_ERR_INVALID, "hcc_sort_workspace: null pointer");
    if (key_bits < 1 || key_bits > 64) return fail(HCC_ERR_INVALID, "hcc_sort_workspace: key_bits must be in [1, 64]");
    if (n >= (1u << 30)) return fail(HCC_ERR_INVALID, "hcc_sort_workspace: n must be below 2^30");
    *bytes = sort_workspace_bytes(n, key_bits);
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_sort(const void* d_keys, uint32_t key_bits, uint32_t n,
                                                           uint32_t* d_perm, void* d_sorted_keys, void* d_ws,
                                                           size_t ws_bytes, hcc_stream stream) {
    hcc::Range range("hcc_sort");
    return radix_sort(d_keys, key_bits, n, d_perm, d_sorted_keys, nullptr, d_ws, ws_bytes, S(stream));
}

__attribute__((visibility("default"))) hcc_status hcc_sort_static(const void* d_keys, uint32_t key_bits,
                                                                  uint32_t n, uint32_t* d_perm, void* d_sorted_keys,
                                                                  hcc_stream stream) {
    return radix_sort_static(d_keys, key_bits, n, d_perm, d_sorted_keys, S(stream));
}

__attribute__((visibility("default"))) hcc_status hcc_sort_static_bytes(size_t* bytes) {
    if (!bytes) return fail(HCC_ERR_INVALID, "hcc_sort_static_bytes: null pointer");
    *bytes = sort_static_bytes();
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_sort_ex(const void* d_keys, uint32_t key_bits,
                                                              uint32_t skip_bits, uint32_t tile, uint32_t n,
                                                              uint32_t* d_perm, void* d_sorted_keys, void* d_ws,
                                                              size_t ws_bytes, hcc_stream stream) {
    hcc::Range range("hcc_sort_ex");
    return radix_sort_ex(d_keys, key_bits, skip_bits, tile, n, d_perm, d_sorted_keys, d_ws, ws_bytes, S(stream));
}

static hcc_status check_trace(hcc_bvh bvh, const hcc_ray* d_rays, uint32_t n, hcc_trace_mode mode, hcc_hit* d_hits,
                              uint8_t* d_occluded) {
    if (!valid_bvh(bvh)) return fail(HCC_ERR_INVALID, "hcc_trace: invalid bvh handle");
    if (mode != HCC_TRACE_CLOSEST && mode != HCC_TRACE_ANY) return fail(HCC_ERR_INVALID, "hcc_trace: bad mode");
    if (n == 0) return HCC_OK;
    if (!d_rays) return fail(HCC_ERR_INVALID, "hcc_trace: null rays");
    if (mode == HCC_TRACE_CLOSEST && !d_hits) return fail(HCC_ERR_INVALID, "hcc_trace: closest hit needs d_hits");
    if (mode == HCC_TRACE_ANY && !d_occluded) return fail(HCC_ERR_INVALID, "hcc_trace: any hit needs d_occluded");
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_trace_ex(hcc_bvh bvh, const hcc_ray* d_rays,
                                                               const uint32_t* d_perm, uint32_t n, hcc_trace_mode mode,
                                                               hcc_hit* d_hits, uint8_t* d_occluded,
                                                               const hcc_trace_opts* opts, hcc_stream stream) {
    hcc::Range range("hcc_trace_ex");
    hcc_status st = check_trace(bvh, d_rays, n, mode, d_hits, d_occluded);
    if (st != HCC_OK || n == 0) return st;
    hcc_trace_opts o{};
    if (opts) o = *opts;
    if (o.flags & ~(HCC_TRACE_SPECULATE | HCC_TRACE_WIDE | HCC_TRACE_SLAB | HCC_TRACE_SPREAD | HCC_TRACE_QUANT |
                    HCC_TRACE_PACKET))
        return fail(HCC_ERR_INVALID, "hcc_trace: unknown opts.flags bits");
    return trace(bvh, d_rays, d_perm, n, mode == HCC_TRACE_CLOSEST, d_hits, d_occluded, o, S(stream));
}

__attribute__((visibility("default"))) hcc_status hcc_trace_count(hcc_bvh bvh, const hcc_ray* d_rays,
                                                                  const uint32_t* d_perm, uint32_t n,
                                                                  hcc_trace_mode mode, hcc_hit* d_hits,
                                                                  uint8_t* d_occluded, const hcc_trace_opts* opts,
                                                                  uint64_t* d_counts, hcc_stream stream) {
    hcc::Range range("hcc_trace_count");
    hcc_status st = check_trace(bvh, d_rays, n, mode, d_hits, d_occluded);
    if (st != HCC_OK || n == 0) return st;
    if (!d_counts) return fail(HCC_ERR_INVALID, "hcc_trace_count: null d_counts");
    hcc_trace_opts o{};
    if (opts) o = *opts;
    if (o.flags & ~(HCC_TRACE_SPECULATE | HCC_TRACE_WIDE | HCC_TRACE_SLAB | HCC_TRACE_SPREAD | HCC_TRACE_QUANT |
                    HCC_TRACE_PACKET))
        return fail(HCC_ERR_INVALID, "hcc_trace_count: unknown opts.flags bits");
    return trace_count(bvh, d_rays, d_perm, n, mode == HCC_TRACE_CLOSEST, d_hits, d_occluded, o,
                       (unsigned long long*)d_counts, S(stream));
}

__attribute__((visibility("default"))) hcc_status hcc_trace(hcc_bvh bvh, const hcc_ray* d_rays, const uint32_t* d_perm,
                                                            uint32_t n, hcc_trace_mode mode, hcc_hit* d_hits,
                                                            uint8_t* d_occluded, hcc_stream stream) {
    hcc::Range range("hcc_trace");
    return hcc_trace_ex(bvh, d_rays, d_perm, n, mode, d_hits, d_occluded, nullptr, stream);
}

__attribute__((visibility("default"))) hcc_status hcc_trace_stats(hcc_bvh bvh, const hcc_ray* d_rays,
                                                                  const uint32_t* d_perm, uint32_t n,
                                                                  hcc_trace_mode mode, hcc_hit* d_hits,
                                                                  uint8_t* d_occluded, uint32_t* d_nodes,
                                                                  uint32_t* d_tris, uint32_t* d_wave_nodes,
                                                                  uint32_t* d_wave_tris, hcc_stream stream) {
    hcc::Range range("hcc_trace_stats");
    hcc_status st = check_trace(bvh, d_rays, n, mode, d_hits, d_occluded);
    if (st != HCC_OK || n == 0) return st;
    if (!d_wave_nodes || !d_wave_tris)
        return fail(HCC_ERR_INVALID, "hcc_trace_stats: d_wave_nodes and d_wave_tris are required");
    const size_t waves = ((size_t)n + 63) / 64;
    // the per-wave counters are accumulated with atomics: clear them first
    st = fill_u32(d_wave_nodes, waves, 0u, S(stream));
    if (st == HCC_OK) st = fill_u32(d_wave_tris, waves, 0u, S(stream));
    if (st != HCC_OK) return st;
    return trace_stats(bvh, d_rays, d_perm, n, mode == HCC_TRACE_CLOSEST, d_hits, d_occluded, d_nodes, d_tris,
                       d_wave_nodes, d_wave_tris, S(stream));
}

}  // extern "C"

static hcc_status check_batches(const hcc_batch_desc* d, uint32_t nb, hcc_key_mode mode, uint32_t key_bits) {
    if (!d || nb == 0) return fail(HCC_ERR_INVALID, "hcc_batch: empty batch list");
    if (mode != HCC_KEY_NONE && mode != HCC_KEY_HCC && mode != HCC_KEY_TWOPOINT)
        return fail(HCC_ERR_INVALID, "hcc_batch: bad key mode");
    if (key_bits < 1 || key_bits > 64) return fail(HCC_ERR_INVALID, "hcc_batch: key_bits must be in [1, 64]");
    for (uint32_t b = 0; b < nb; ++b) {
        const hcc_batch_desc& x = d[b];
        const std::string at = " (batch " + std::to_string(b) + ")";
        if (!valid_bvh(x.bvh)) return fail(HCC_ERR_INVALID, "hcc_batch: invalid bvh" + at);
        if (mode == HCC_KEY_HCC && (!valid_cut(x.cut) || x.cut->bvh != x.bvh))
            return fail(HCC_ERR_INVALID, "hcc_batch: HCC needs a cut of the batch's bvh" + at);
        if (x.n >= (1u << 30)) return fail(HCC_ERR_INVALID, "hcc_batch: n must be below 2^30" + at);
        if (x.mode != HCC_TRACE_CLOSEST && x.mode != HCC_TRACE_ANY) return fail(HCC_ERR_INVALID, "hcc_batch: bad trace mode" + at);
        if (x.n > 0 && !x.d_rays) return fail(HCC_ERR_INVALID, "hcc_batch: null rays" + at);
        if (x.n > 0 && x.mode == HCC_TRACE_CLOSEST && !x.d_hits) return fail(HCC_ERR_INVALID, "hcc_batch: null hits" + at);
        if (x.n > 0 && x.mode == HCC_TRACE_ANY && !x.d_occluded) return fail(HCC_ERR_INVALID, "hcc_batch: null occluded" + at);
    }
    return HCC_OK;
}

extern "C" {

__attribute__((visibility("default"))) hcc_status hcc_batch_workspace(const hcc_batch_desc* batches, uint32_t nb,
                                                                      hcc_key_mode mode, uint32_t key_bits,
                                                                      size_t* bytes) {
    if (!bytes) return fail(HCC_ERR_INVALID, "hcc_batch_workspace: null bytes");
    hcc_status st = check_batches(batches, nb, mode, key_bits);
    if (st != HCC_OK) return st;
    return batch_workspace(batches, nb, mode, key_bits, bytes);
}

__attribute__((visibility("default"))) hcc_status hcc_batch_run(const hcc_batch_desc* batches, uint32_t nb,
                                                                hcc_key_mode mode, uint32_t key_bits,
                                                                const hcc_batch_opts* opts, void* d_ws,
                                                                size_t ws_bytes, hcc_stream stream) {
    hcc::Range range("hcc_batch_run");
    hcc_status st = check_batches(batches, nb, mode, key_bits);
    if (st != HCC_OK) return st;
    if (!d_ws || ((uintptr_t)d_ws & 255u)) return fail(HCC_ERR_INVALID, "hcc_batch_run: workspace must be 256-byte aligned");
    hcc_batch_opts o{};
    if (opts) o = *opts;
    if ((o.flags & ~(HCC_TRACE_WIDE | HCC_TRACE_SLAB | HCC_TRACE_QUANT)) != 0)
        return fail(HCC_ERR_INVALID, "hcc_batch_run: unknown opts.flags bits");
    if (o.direct_min != 0 && o.direct_min < 65536)
        return fail(HCC_ERR_INVALID, "hcc_batch_run: opts.direct_min must be 0 or at least 65536");
    if (o.stack > HCC_BATCH_STACK_SCRATCH) return fail(HCC_ERR_INVALID, "hcc_batch_run: opts.stack must be 0..3");
    return batch_run(batches, nb, mode, key_bits, o, d_ws, ws_bytes, S(stream));
}

__attribute__((visibility("default"))) hcc_status hcc_batch_export(const hcc_batch_desc* batches, uint32_t nb,
                                                                   hcc_key_mode mode, uint32_t key_bits,
                                                                   const hcc_batch_opts* opts, const void* d_ws,
                                                                   size_t ws_bytes, uint32_t batch, uint32_t* d_perm,
                                                                   void* d_sorted_keys, hcc_stream stream) {
    hcc_status st = check_batches(batches, nb, mode, key_bits);
    if (st != HCC_OK) return st;
    if (mode == HCC_KEY_NONE) return fail(HCC_ERR_UNSUPPORTED, "hcc_batch_export: a trace-only run has no keys");
    if (!d_ws || ((uintptr_t)d_ws & 255u)) return fail(HCC_ERR_INVALID, "hcc_batch_export: workspace must be 256-byte aligned");
    if (batch >= nb) return fail(HCC_ERR_INVALID, "hcc_batch_export: batch index out of range");
    hcc_batch_opts o{};
    if (opts) o = *opts;
    if (o.direct_min != 0 && o.direct_min < 65536)
        return fail(HCC_ERR_INVALID, "hcc_batch_export: opts.direct_min must be 0 or at least 65536");
    return batch_export(batches, nb, mode, key_bits, o, d_ws, ws_bytes, batch, d_perm, d_sorted_keys, S(stream));
}

__attribute__((visibility("default"))) hcc_status hcc_batch_check(const void* d_ws, hcc_stream stream,
                                                                  uint32_t* h_ok) {
    if (!d_ws || !h_ok) return fail(HCC_ERR_INVALID, "hcc_batch_check: null argument");
    return batch_check(d_ws, S(stream), h_ok);
}

__attribute__((visibility("default"))) hcc_status hcc_select_mlhcc_cut(hcc_bvh bvh, uint32_t top, uint32_t low,
                                                                       double lambda, hcc_stream stream,
                                                                       hcc_cut* out) {
    hcc::Range range("hcc_select_mlhcc_cut");
    if (!valid_bvh(bvh) || !out) return fail(HCC_ERR_INVALID, "hcc_select_mlhcc_cut: invalid handle or null out");
    if (top == 0 || low == 0 || top > 64 || low > 64 || top * low > 2048)
        return fail(HCC_ERR_INVALID, "hcc_select_mlhcc_cut: need 1 <= top, low <= 64 and top * low <= 2048");
    if (!(lambda >= 0.0) || !std::isfinite(lambda))
        return fail(HCC_ERR_INVALID, "hcc_select_mlhcc_cut: lambda must be finite and >= 0");
    hcc_status st;
    if (lambda != bvh->had_lambda && (st = recompute_had(bvh, lambda, S(stream))) != HCC_OK) return st;
    if ((st = ensure_host_mirror(bvh, S(stream))) != HCC_OK) return st;
    ensure_leaf_counts(bvh);
    std::vector<float> all;
    if ((st = download_boxes(bvh, all)) != HCC_OK) return st;
    hcc_cut_s* c = new hcc_cut_s();
    c->bvh = bvh;
    c->kind = 1;
    c->low = low;
    c->top_req = top;
    c->ids = mlhcc_top_search(bvh, top, low);
    c->c_eff = (uint32_t)c->ids.size();
    for (uint32_t id : c->ids) {
        c->had.push_back(bvh->h_had[id]);
        c->boxes.insert(c->boxes.end(), &all[6 * (size_t)id], &all[6 * (size_t)id] + 6);
        const std::vector<uint32_t> lo = cut_search(bvh, low, id);
        if (lo.size() != low) {
            delete c;
            return fail(HCC_ERR_INVALID, "hcc_select_mlhcc_cut: internal error (short low-level cut)");
        }
        for (uint32_t x : lo) {
            c->low_ids.push_back(x);
            c->low_boxes.insert(c->low_boxes.end(), &all[6 * (size_t)x], &all[6 * (size_t)x] + 6);
        }
    }
    return finish_cut(c, S(stream), out);
}

__attribute__((visibility("default"))) hcc_status hcc_grid_cut(hcc_bvh bvh, uint32_t gx, uint32_t gy, uint32_t gz,
                                                               hcc_stream stream, hcc_cut* out) {
    hcc::Range range("hcc_grid_cut");
    if (!valid_bvh(bvh) || !out) return fail(HCC_ERR_INVALID, "hcc_grid_cut: invalid handle or null out");
    if (gx == 0 || gy == 0 || gz == 0 || (uint64_t)gx * gy * gz > 64)
        return fail(HCC_ERR_INVALID, "hcc_grid_cut: need 1 <= gx*gy*gz <= 64");
    hcc_cut_s* c = new hcc_cut_s();
    c->bvh = bvh;
    c->kind = 2;
    const uint32_t g[3] = {gx, gy, gz};
    const float* sb = bvh->scene_box;
    for (uint32_t z = 0; z < gz; ++z)
        for (uint32_t y = 0; y < gy; ++y)
            for (uint32_t x = 0; x < gx; ++x) {
                const uint32_t idx[3] = {x, y, z};
                float bx[6];
                for (int a = 0; a < 3; ++a) {
                    const double lo = sb[a], ext = (double)sb[3 + a] - (double)sb[a];
                    bx[a] = (float)(lo + ext * (double)idx[a] / (double)g[a]);
                    bx[3 + a] = (float)(lo + ext * (double)(idx[a] + 1) / (double)g[a]);
                }
                c->boxes.insert(c->boxes.end(), bx, bx + 6);
                c->ids.push_back(0xFFFFFFFFu);
                c->had.push_back(0.0);
            }
    c->c_eff = gx * gy * gz;
    return finish_cut(c, S(stream), out);
}

__attribute__((visibility("default"))) hcc_status hcc_cut_shape(hcc_cut cut, uint32_t* kind, uint32_t* top,
                                                                uint32_t* low) {
    if (!valid_cut(cut)) return fail(HCC_ERR_INVALID, "hcc_cut_shape: invalid handle");
    if (kind) *kind = cut->kind;
    if (top) *top = cut->c_eff;
    if (low) *low = cut->low;
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_cut_export_low(hcc_cut cut, uint32_t* h_low_ids,
                                                                     float* h_low_boxes) {
    if (!valid_cut(cut) || cut->kind != 1) return fail(HCC_ERR_INVALID, "hcc_cut_export_low: not a two-level cut");
    if (h_low_ids) std::memcpy(h_low_ids, cut->low_ids.data(), sizeof(uint32_t) * cut->low_ids.size());
    if (h_low_boxes) std::memcpy(h_low_boxes, cut->low_boxes.data(), sizeof(float) * cut->low_boxes.size());
    return HCC_OK;
}

}  // extern "C"
