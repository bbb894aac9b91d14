// Host side of the fastloop C ABI: validation, workspace and pinned staging
// (allocated once and grown, never per call), batch descriptor upload,
// kernel launches, HIP-graph capture/replay and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "fastloop.h"
#include "fl_internal.h"
#include "fl_residual.h"
#include "fl_search.h"

using namespace fl;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define FL_HIP(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(FL_EHIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int next_pow2(int x) {
    int p = 16;
    while (p < x) p <<= 1;
    return p;
}

// A device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t size = 0;
    int ensure(size_t need) {
        if (need <= size) return FL_OK;
        if (p) {
            hipDeviceSynchronize();   // work queued on any stream may still use the old buffer
            hipFree(p);
        }
        p = nullptr;
        size = 0;
        size_t n = std::max(need, (size_t)1 << 20);
        n = align_up(n + n / 4, 4096);
        if (hipMalloc(&p, n) != hipSuccess) {
            p = nullptr;
            return fail(FL_ENOMEM, "hipMalloc of %zu bytes failed", n);
        }
        size = n;
        return FL_OK;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        size = 0;
    }
};

// Pinned staging buffer with an event marking when its last upload finished.
struct Pinned {
    void* p = nullptr;
    size_t size = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

// Offsets of the workspace regions of one batch.
struct Layout {
    size_t hdr, kf, ev, cell_start, recs, desc_sorted, cell_kp, hash, claim, tile, add_list, match_list,
        counters, stats, ev_match, refine_done, event_S32, refine_partial, total;
    size_t blob_bytes;   // hdr + kf + ev (uploaded per call)
};

}  // namespace

struct fl_ctx {
    int device = 0;
    int n_cu = 256;
    DevBuf ws;           // batched workspace (header, tables, grids, lists)
    DevBuf plain;        // plain-path workspace
    DevBuf res;          // residual partials and done counter
    Pinned pin[2];
    int pin_next = 0;
    hipStream_t cap_stream = nullptr;
    fl_tuning tune{2, 256, 16, 1};
    int stats = 0;
    int add_cap_override = 0;   // test hook: >0 forces a small ADD / match list capacity
    int prof = 0;               // record events around eager search kernels
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
    // captured graph and its key
    hipGraphExec_t gexec = nullptr;
    void* g_ws = nullptr;
    fl_tuning g_tune{};
    int g_stats = -1;
    int g_refine = -1;
};

namespace {

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

int check_params(const fl_params* P) {
    if (!P) return fail(FL_EINVAL, "params is NULL");
    if (P->flags != 0) return fail(FL_EINVAL, "params.flags must be 0");
    if (!finite_pos(P->win_px)) return fail(FL_EINVAL, "win_px must be finite and > 0");
    if (!finite_pos(P->scale_factor)) return fail(FL_EINVAL, "scale_factor must be finite and > 0");
    if (P->n_octaves < 1 || P->n_octaves > FL_MAX_OCTAVES)
        return fail(FL_ERANGE, "n_octaves %d outside [1, %d]", P->n_octaves, FL_MAX_OCTAVES);
    if (P->grid_cols < 1 || P->grid_rows < 1) return fail(FL_EINVAL, "grid_cols and grid_rows must be >= 1");
    if ((int64_t)P->grid_cols * P->grid_rows > FL_MAX_CELLS)
        return fail(FL_ERANGE, "grid_cols * grid_rows = %lld exceeds %d", (long long)P->grid_cols * P->grid_rows,
                    FL_MAX_CELLS);
    if (!std::isfinite(P->nn_ratio)) return fail(FL_EINVAL, "nn_ratio must be finite");
    return FL_OK;
}

int check_cam(const fl_pinhole* K, const char* what) {
    if (!K) return fail(FL_EINVAL, "%s camera is NULL", what);
    if (!std::isfinite(K->fx) || !std::isfinite(K->fy) || !std::isfinite(K->cx) || !std::isfinite(K->cy))
        return fail(FL_EINVAL, "%s camera has non-finite intrinsics", what);
    if (!finite_pos(K->width) || !finite_pos(K->height))
        return fail(FL_EINVAL, "%s camera width/height must be finite and > 0", what);
    return FL_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

void fill_search_const(const fl_params* P, SearchConst& sc, float* sf) {
    for (int n = 0; n < 32; ++n) sf[n] = n < P->n_octaves ? (float)std::pow((double)P->scale_factor, (double)n) : 0.0f;
    for (int n = 0; n < 32; ++n) sc.sf[n] = sf[n];
    sc.N = P->n_octaves;
    sc.C = P->grid_cols;
    sc.R = P->grid_rows;
    sc.th = P->hamming_th;
    sc.ratio = P->nn_ratio;
    sc.r0 = P->win_px;
}

void fill_kf_geometry(KfDesc& k, const fl_sim3& S, const fl_pinhole& K, const fl_params* P) {
    for (int i = 0; i < 9; ++i) k.A[i] = S.sR[i];
    for (int i = 0; i < 3; ++i) k.t[i] = S.t[i];
    k.inv_s = S.inv_s;
    k.fx = K.fx;
    k.fy = K.fy;
    k.cx = K.cx;
    k.cy = K.cy;
    k.W = K.width;
    k.H = K.height;
    k.invw = (float)P->grid_cols / K.width;
    k.invh = (float)P->grid_rows / K.height;
    for (int i = 0; i < 12; ++i) k.T[i] = (i == 0 || i == 4 || i == 8) ? 1.0f : 0.0f;
}

int get_pinned(fl_ctx* c, size_t need, Pinned** out) {
    Pinned& p = c->pin[c->pin_next];
    c->pin_next ^= 1;
    if (p.pending) {
        FL_HIP(hipEventSynchronize(p.done));
        p.pending = false;
    }
    if (p.size < need) {
        if (p.p) hipHostFree(p.p);
        p.p = nullptr;
        p.size = 0;
        size_t n = align_up(std::max(need + need / 4, (size_t)1 << 16), 4096);
        if (hipHostMalloc(&p.p, n, hipHostMallocDefault) != hipSuccess) {
            p.p = nullptr;
            return fail(FL_ENOMEM, "hipHostMalloc of %zu bytes failed", n);
        }
        p.size = n;
    }
    *out = &p;
    return FL_OK;
}

// ---------------------------------------------------------------------------
// batch preparation

struct Prepared {
    Layout L;
    std::vector<KfDesc> kf;
    std::vector<EventDesc> ev;
    BatchHdr hdr;
    int n_tiles = 0;
    int refine_blocks = 1;
};

int validate_batch(const fl_batch* B, const fl_params* P, const fl_fuse_out* out) {
    if (!B) return fail(FL_EINVAL, "batch is NULL");
    if (!out) return fail(FL_EINVAL, "outputs are NULL");
    int rc = check_params(P);
    if (rc) return rc;
    if (B->n_events < 0 || B->n_kf < 0 || B->n_mp < 0 || B->n_kp_total < 0 || B->n_pairs < 0)
        return fail(FL_EINVAL, "negative count in batch");
    if (B->n_pairs > FL_MAX_PAIRS) return fail(FL_ERANGE, "n_pairs %lld exceeds 2^31-1", (long long)B->n_pairs);
    if (!B->event_kf_offset || !B->event_mp_offset || !B->kp_offset || !B->pair_offset)
        return fail(FL_EINVAL, "batch offset tables must not be NULL");
    if (B->n_kf > 0 && (!B->kf_sim3 || !B->kf_K)) return fail(FL_EINVAL, "kf_sim3 / kf_K must not be NULL");
    const int32_t* ekf = B->event_kf_offset;
    const int32_t* emp = B->event_mp_offset;
    if (ekf[0] != 0 || emp[0] != 0) return fail(FL_EINVAL, "event offsets must start at 0");
    for (int e = 0; e < B->n_events; ++e) {
        if (ekf[e + 1] < ekf[e]) return fail(FL_EINVAL, "event_kf_offset decreases at event %d", e);
        if (emp[e + 1] < emp[e]) return fail(FL_EINVAL, "event_mp_offset decreases at event %d", e);
    }
    if (ekf[B->n_events] != B->n_kf) return fail(FL_EINVAL, "event_kf_offset[n_events] != n_kf");
    if (emp[B->n_events] != B->n_mp) return fail(FL_EINVAL, "event_mp_offset[n_events] != n_mp");
    if (B->kp_offset[0] != 0 || B->pair_offset[0] != 0)
        return fail(FL_EINVAL, "kp_offset / pair_offset must start at 0");
    for (int k = 0; k < B->n_kf; ++k) {
        const int32_t nk = B->kp_offset[k + 1] - B->kp_offset[k];
        if (nk < 0) return fail(FL_EINVAL, "kp_offset decreases at keyframe %d", k);
        if (nk > FL_MAX_KP) return fail(FL_ERANGE, "keyframe %d has %d keypoints (max %d)", k, nk, FL_MAX_KP);
        if (B->pair_offset[k + 1] < B->pair_offset[k]) return fail(FL_EINVAL, "pair_offset decreases at keyframe %d", k);
        rc = check_cam(&B->kf_K[k], "keyframe");
        if (rc) return rc;
    }
    if (B->kp_offset[B->n_kf] != B->n_kp_total) return fail(FL_EINVAL, "kp_offset[n_kf] != n_kp_total");
    if (B->pair_offset[B->n_kf] != B->n_pairs) return fail(FL_EINVAL, "pair_offset[n_kf] != n_pairs");
    if (!B->pair_mp) {
        for (int e = 0; e < B->n_events; ++e)
            for (int k = ekf[e]; k < ekf[e + 1]; ++k)
                if (B->pair_offset[k + 1] - B->pair_offset[k] != emp[e + 1] - emp[e])
                    return fail(FL_EINVAL, "dense pairs: keyframe %d must have one pair per point of its event", k);
    }
    if (B->n_kp_total > 0 && (!B->kp_xy || !B->kp_octave || !B->kp_desc || !B->kp_owner))
        return fail(FL_EINVAL, "keypoint arrays must not be NULL");
    if (B->n_mp > 0 && (!B->mp_xyz || !B->mp_desc)) return fail(FL_EINVAL, "point arrays must not be NULL");
    if ((B->kp_desc && !aligned16(B->kp_desc)) || (B->mp_desc && !aligned16(B->mp_desc)))
        return fail(FL_EINVAL, "descriptor arrays must be 16-byte aligned");
    if (B->n_pairs > 0 &&
        (!out->best_idx || !out->best_dist || !out->second_dist || !out->decision || !out->target))
        return fail(FL_EINVAL, "output arrays must not be NULL");
    return FL_OK;
}

int prepare_batch(fl_ctx* c, const fl_batch* B, const fl_params* P, const fl_fuse_out* out, const fl_refine* R,
                  int ppl, Prepared& pr) {
    const int cells = P->grid_cols * P->grid_rows;
    const int n_kf = B->n_kf, n_ev = B->n_events;
    const int tile_pairs = kWave * ppl;
    const bool refine = R && R->n_iters > 0;
    pr.kf.assign(n_kf, KfDesc{});
    pr.ev.assign(n_ev, EventDesc{});
    // per-keyframe geometry, ranges and tables
    int64_t hash_total = 0;
    int64_t list_total = 0;
    std::vector<double> cost(n_kf);
    for (int e = 0; e < n_ev; ++e) {
        EventDesc& ed = pr.ev[e];
        ed.kf_begin = B->event_kf_offset[e];
        ed.kf_end = B->event_kf_offset[e + 1];
        ed.mp_off = B->event_mp_offset[e];
        ed.n_mp = B->event_mp_offset[e + 1] - ed.mp_off;
        ed.pair_begin = B->pair_offset[ed.kf_begin];
        ed.pair_end = B->pair_offset[ed.kf_end];
        int64_t kp_ev = B->kp_offset[ed.kf_end] - B->kp_offset[ed.kf_begin];
        int64_t cap = std::min<int64_t>(ed.pair_end - ed.pair_begin, std::max<int64_t>(2 * kp_ev, 4096));
        if (c->add_cap_override > 0) cap = std::min<int64_t>(cap, c->add_cap_override);
        ed.list_off = refine ? (int32_t)list_total : 0;
        ed.list_cap = refine ? (int32_t)cap : 0;
        if (refine) list_total += cap;
        for (int k = ed.kf_begin; k < ed.kf_end; ++k) {
            KfDesc& kd = pr.kf[k];
            fill_kf_geometry(kd, B->kf_sim3[k], B->kf_K[k], P);
            if (B->kf_T)
                for (int i = 0; i < 12; ++i) kd.T[i] = B->kf_T[12 * (int64_t)k + i];
            kd.kp_off = B->kp_offset[k];
            kd.n_kp = B->kp_offset[k + 1] - B->kp_offset[k];
            kd.grid_off = k * (cells + 1);
            kd.event = e;
            kd.mp_off = ed.mp_off;
            kd.n_mp = ed.n_mp;
            const int hsize = next_pow2(2 * kd.n_kp);
            kd.hash_off = (int32_t)hash_total;
            kd.hash_mask = hsize - 1;
            hash_total += hsize;
            kd.pair_off = B->pair_offset[k];
            kd.n_pairs = B->pair_offset[k + 1] - B->pair_offset[k];
            kd.n_tiles = (int32_t)((kd.n_pairs + tile_pairs - 1) / tile_pairs);
            // cost per pair grows with keypoint density (candidates scanned)
            cost[k] = (double)kd.n_pairs * (1.0 + 4.0 * kd.n_kp / std::max(1, cells));
        }
    }
    // tile order: keyframes by decreasing cost, tiles of a keyframe consecutive
    std::vector<int> order(n_kf);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    int64_t tiles = 0;
    std::vector<double> tile_cost_prefix(1, 0.0);
    for (int k : order) {
        pr.kf[k].tile_off = (int32_t)tiles;
        tiles += pr.kf[k].n_tiles;
    }
    if (tiles > INT32_MAX / 2) return fail(FL_ERANGE, "too many tiles");
    pr.n_tiles = (int)tiles;
    // split the tile sequence into per-XCD queues of about equal estimated cost
    BatchHdr& h = pr.hdr;
    memset(&h, 0, sizeof(h));
    const int nq = c->tune.xcd_queues ? kMaxQueues : 1;
    h.n_queues = nq;
    {
        double total = 0.0;
        for (int k = 0; k < n_kf; ++k) total += cost[k];
        int q = 1;
        double acc = 0.0;
        h.queue_begin[0] = 0;
        for (int k : order) {
            const KfDesc& kd = pr.kf[k];
            const double per_tile = kd.n_tiles ? cost[k] / kd.n_tiles : 0.0;
            for (int j = 0; j < kd.n_tiles && q < nq; ++j) {
                acc += per_tile;
                while (q < nq && acc >= total * q / nq) h.queue_begin[q++] = kd.tile_off + j + 1;
            }
        }
        while (q <= nq) h.queue_begin[q++] = pr.n_tiles;
        h.queue_begin[nq] = pr.n_tiles;
        for (int i = 1; i <= nq; ++i) h.queue_begin[i] = std::max(h.queue_begin[i], h.queue_begin[i - 1]);
    }
    // workspace layout
    Layout& L = pr.L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.hdr = take(sizeof(BatchHdr));
    L.kf = take(sizeof(KfDesc) * (size_t)n_kf);
    L.ev = take(sizeof(EventDesc) * (size_t)n_ev);
    L.blob_bytes = off;
    L.cell_start = take(sizeof(int32_t) * (size_t)n_kf * (cells + 1));
    L.recs = take(sizeof(KpRec) * (size_t)B->n_kp_total);
    L.desc_sorted = take(32 * (size_t)B->n_kp_total);
    L.cell_kp = take(sizeof(int32_t) * (size_t)B->n_kp_total);
    L.hash = take(sizeof(int32_t) * (size_t)hash_total);
    L.claim = take(sizeof(int32_t) * (size_t)B->n_kp_total);
    L.tile = take(sizeof(int2) * (size_t)pr.n_tiles);
    int64_t add_cap = std::min<int64_t>(B->n_pairs, std::max<int64_t>(2 * (int64_t)B->n_kp_total, 4096));
    if (c->add_cap_override > 0) add_cap = std::min<int64_t>(add_cap, c->add_cap_override);
    L.add_list = take(sizeof(PairRef) * (size_t)add_cap);
    L.match_list = take(sizeof(PairRef) * (size_t)list_total);
    L.counters = take(sizeof(uint32_t) * kCounterWords);
    L.stats = take(sizeof(unsigned long long) * 4);
    L.ev_match = take(sizeof(uint32_t) * (size_t)n_ev);
    L.refine_done = take(sizeof(uint32_t) * (size_t)n_ev);
    L.event_S32 = take(sizeof(fl_sim3) * (size_t)n_ev);
    pr.refine_blocks = std::max(1, std::min(64, 1024 / std::max(1, n_ev)));
    L.refine_partial = take(sizeof(double) * kNAcc * (size_t)n_ev * pr.refine_blocks);
    L.total = off;
    int rc = c->ws.ensure(L.total);
    if (rc) return rc;
    char* base = (char*)c->ws.p;
    // header
    h.n_events = n_ev;
    h.n_kf = n_kf;
    h.n_mp = B->n_mp;
    h.n_kp_total = B->n_kp_total;
    h.n_pairs = B->n_pairs;
    h.n_tiles = pr.n_tiles;
    h.tile_pairs = tile_pairs;
    h.cells = cells;
    h.grid_cols = P->grid_cols;
    h.grid_rows = P->grid_rows;
    h.n_octaves = P->n_octaves;
    h.hamming_th = P->hamming_th;
    h.nn_ratio = P->nn_ratio;
    h.r0 = P->win_px;
    h.gate = B->mp_dmax != nullptr;
    h.dense = B->pair_mp == nullptr;
    h.add_cap = (int32_t)add_cap;
    h.stats = c->stats;
    SearchConst sc;
    fill_search_const(P, sc, h.sf);
    h.kf = (const KfDesc*)(base + L.kf);
    h.ev = (const EventDesc*)(base + L.ev);
    h.tile = (int2*)(base + L.tile);
    h.kp_xy = B->kp_xy;
    h.kp_oct = B->kp_octave;
    h.kp_desc = B->kp_desc;
    h.kp_owner = B->kp_owner;
    h.mp_xyz = B->mp_xyz;
    h.mp_desc = B->mp_desc;
    h.mp_dmax = B->mp_dmax;
    h.mp_id = B->mp_id;
    h.pair_mp = B->pair_mp;
    h.best_idx = out->best_idx;
    h.best_dist = out->best_dist;
    h.second_dist = out->second_dist;
    h.decision = out->decision;
    h.target = out->target;
    h.cell_start = (int32_t*)(base + L.cell_start);
    h.recs = (KpRec*)(base + L.recs);
    h.desc_sorted = (uint4*)(base + L.desc_sorted);
    h.cell_kp = (int32_t*)(base + L.cell_kp);
    h.hash = (int32_t*)(base + L.hash);
    h.claim = (int32_t*)(base + L.claim);
    h.add_list = (PairRef*)(base + L.add_list);
    h.match_list = (PairRef*)(base + L.match_list);
    h.counters = (uint32_t*)(base + L.counters);
    h.stats_out = (unsigned long long*)(base + L.stats);
    h.ev_match_count = (uint32_t*)(base + L.ev_match);
    h.refine_done = (uint32_t*)(base + L.refine_done);
    h.event_S32 = (fl_sim3*)(base + L.event_S32);
    h.refine_partial = (double*)(base + L.refine_partial);
    h.refine_blocks = pr.refine_blocks;
    if (refine) {
        h.refine_iters = R->n_iters;
        h.huber_delta = R->huber_delta;
        h.event_S = R->event_S;
        h.event_S32_out = R->event_S32;
        h.event_n_matched = R->event_n_matched;
    }
    return FL_OK;
}

int upload_batch(fl_ctx* c, Prepared& pr, hipStream_t stream) {
    Pinned* pin = nullptr;
    int rc = get_pinned(c, pr.L.blob_bytes, &pin);
    if (rc) return rc;
    char* hb = (char*)pin->p;
    memcpy(hb + pr.L.hdr, &pr.hdr, sizeof(BatchHdr));
    if (!pr.kf.empty()) memcpy(hb + pr.L.kf, pr.kf.data(), sizeof(KfDesc) * pr.kf.size());
    if (!pr.ev.empty()) memcpy(hb + pr.L.ev, pr.ev.data(), sizeof(EventDesc) * pr.ev.size());
    FL_HIP(hipMemcpyAsync(c->ws.p, hb, pr.L.blob_bytes, hipMemcpyHostToDevice, stream));
    FL_HIP(hipEventRecord(pin->done, stream));
    pin->pending = true;
    return FL_OK;
}

int search_grid_size(const fl_ctx* c) {
    const int waves_per_block = std::max(1, c->tune.block / kWave);
    return std::max(1, c->n_cu * c->tune.waves_per_cu / waves_per_block);
}

constexpr int kPrepGrid = 512;
constexpr int kResolveGrid = 256;
constexpr int kRefineGrid = 1024;

int launch_search(fl_ctx* c, const BatchHdr* dh, hipStream_t s, bool eager_sizes, int n_kf) {
    const int pg = eager_sizes ? std::max(1, std::min(n_kf, kPrepGrid)) : kPrepGrid;
    hipLaunchKernelGGL(prep_batched_kernel, dim3(pg), dim3(kPrepBlock), 0, s, dh);
    const int g = search_grid_size(c);
    const int b = c->tune.block;
    const int ppl = c->tune.pairs_per_lane;
    const bool timed = eager_sizes && c->prof;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (timed) {
        FL_HIP(hipEventCreate(&t0));
        FL_HIP(hipEventCreate(&t1));
        FL_HIP(hipEventRecord(t0, s));
    }
    if (c->stats) {
        if (ppl == 1) hipLaunchKernelGGL((search_batched_kernel<1, true>), dim3(g), dim3(b), 0, s, dh);
        else if (ppl == 2) hipLaunchKernelGGL((search_batched_kernel<2, true>), dim3(g), dim3(b), 0, s, dh);
        else hipLaunchKernelGGL((search_batched_kernel<4, true>), dim3(g), dim3(b), 0, s, dh);
    } else {
        if (ppl == 1) hipLaunchKernelGGL((search_batched_kernel<1, false>), dim3(g), dim3(b), 0, s, dh);
        else if (ppl == 2) hipLaunchKernelGGL((search_batched_kernel<2, false>), dim3(g), dim3(b), 0, s, dh);
        else hipLaunchKernelGGL((search_batched_kernel<4, false>), dim3(g), dim3(b), 0, s, dh);
    }
    if (timed) {
        FL_HIP(hipEventRecord(t1, s));
        c->prof_ev.emplace_back(t0, t1);
    }
    hipLaunchKernelGGL(resolve_batched_kernel, dim3(kResolveGrid), dim3(256), 0, s, dh);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int launch_refine(const BatchHdr* dh, int n_iters, hipStream_t s) {
    hipLaunchKernelGGL(refine_init_kernel, dim3(1), dim3(256), 0, s, dh);
    for (int it = 0; it < n_iters; ++it)
        hipLaunchKernelGGL(refine_iter_kernel, dim3(kRefineGrid), dim3(kResBlock), 0, s, dh);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int check_refine(const fl_batch* B, const fl_refine* R) {
    if (!R || R->n_iters == 0) return FL_OK;
    if (R->n_iters < 0 || R->n_iters > 1000) return fail(FL_ERANGE, "refine.n_iters %d outside [0, 1000]", R->n_iters);
    if (!finite_pos(R->huber_delta)) return fail(FL_EINVAL, "refine.huber_delta must be finite and > 0");
    if (B->n_events > 0 && !R->event_S) return fail(FL_EINVAL, "refine.event_S must not be NULL");
    return FL_OK;
}

}  // namespace

// ===========================================================================
// C ABI

static void clear_profile(fl_ctx* c);

extern "C" {

const char* fl_last_error(void) { return g_err; }

int fl_version(void) { return 10000; }

int fl_create(fl_ctx** out, int device) {
    if (!out) return fail(FL_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    FL_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(FL_EINVAL, "device %d not present (%d devices)", device, n);
    FL_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    FL_HIP(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FL_ENOTSUP, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    fl_ctx* c = new fl_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    for (auto& p : c->pin) {
        if (hipEventCreateWithFlags(&p.done, hipEventDisableTiming) != hipSuccess) {
            fl_destroy(c);
            return fail(FL_EHIP, "hipEventCreate failed");
        }
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        fl_destroy(c);
        return fail(FL_EHIP, "hipStreamCreate failed");
    }
    // residual partials: 1024 blocks x kNAcc doubles + a done counter
    if (c->res.ensure(sizeof(double) * 1024 * kNAcc + 256) != FL_OK ||
        hipMemset(c->res.p, 0, c->res.size) != hipSuccess) {
        fl_destroy(c);
        return fail(FL_ENOMEM, "residual workspace allocation failed");
    }
    *out = c;
    return FL_OK;
}

void fl_destroy(fl_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    clear_profile(c);
    for (auto& p : c->pin) {
        if (p.p) hipHostFree(p.p);
        if (p.done) hipEventDestroy(p.done);
    }
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    c->ws.release();
    c->plain.release();
    c->res.release();
    delete c;
}

int fl_build_grid(fl_ctx* c, int32_t n_kp, const float* kp_xy, const fl_pinhole* K, const fl_params* P,
                  int32_t* cell_start, int32_t* cell_kp, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_params(P);
    if (rc) return rc;
    rc = check_cam(K, "keyframe");
    if (rc) return rc;
    if (n_kp < 0) return fail(FL_EINVAL, "n_kp is negative");
    if (n_kp > FL_MAX_KP) return fail(FL_ERANGE, "n_kp %d exceeds %d", n_kp, FL_MAX_KP);
    if (!cell_start || (n_kp > 0 && (!kp_xy || !cell_kp))) return fail(FL_EINVAL, "NULL array");
    KfDesc kd{};
    fl_sim3 I{};
    fill_kf_geometry(kd, I, *K, P);
    kd.n_kp = n_kp;
    hipLaunchKernelGGL(grid_single_kernel, dim3(1), dim3(kPrepBlock), 0, stream, kd,
                       P->grid_cols * P->grid_rows, P->grid_cols, P->grid_rows, kp_xy, cell_start, cell_kp);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_search_fuse(fl_ctx* c, int32_t n_mp, const float* mp_xyz, const uint8_t* mp_desc, const float* mp_dmax,
                   const int32_t* mp_id, const fl_keyframe* kf, const fl_sim3* S, const fl_pinhole* K,
                   const fl_params* P, const fl_fuse_out* out, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_params(P);
    if (rc) return rc;
    rc = check_cam(K, "keyframe");
    if (rc) return rc;
    if (!kf || !S || !out) return fail(FL_EINVAL, "keyframe, Sim3 and outputs must not be NULL");
    if (n_mp < 0 || kf->n_kp < 0) return fail(FL_EINVAL, "negative count");
    if (kf->n_kp > FL_MAX_KP) return fail(FL_ERANGE, "n_kp %d exceeds %d", kf->n_kp, FL_MAX_KP);
    if (n_mp > 0 && (!mp_xyz || !mp_desc)) return fail(FL_EINVAL, "point arrays must not be NULL");
    if (kf->n_kp > 0 && (!kf->kp_xy || !kf->kp_octave || !kf->kp_desc || !kf->kp_owner))
        return fail(FL_EINVAL, "keypoint arrays must not be NULL");
    if ((kf->cell_start == nullptr) != (kf->cell_kp == nullptr))
        return fail(FL_EINVAL, "cell_start and cell_kp must both be given or both be NULL");
    if ((mp_desc && !aligned16(mp_desc)) || (kf->kp_desc && !aligned16(kf->kp_desc)))
        return fail(FL_EINVAL, "descriptor arrays must be 16-byte aligned");
    if (n_mp > 0 && (!out->best_idx || !out->best_dist || !out->second_dist || !out->decision || !out->target))
        return fail(FL_EINVAL, "output arrays must not be NULL");
    if (n_mp == 0) return FL_OK;
    const int cells = P->grid_cols * P->grid_rows;
    const int n_kp = kf->n_kp;
    const int hsize = next_pow2(2 * n_kp);
    int64_t cap = std::min<int64_t>(n_mp, std::max<int64_t>(2 * (int64_t)n_kp, 4096));
    if (c->add_cap_override > 0) cap = std::min<int64_t>(cap, c->add_cap_override);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_cs = take(sizeof(int32_t) * (cells + 1));
    const size_t o_ck = take(sizeof(int32_t) * (size_t)std::max(n_kp, 1));
    const size_t o_hash = take(sizeof(int32_t) * (size_t)hsize);
    const size_t o_claim = take(sizeof(int32_t) * (size_t)std::max(n_kp, 1));
    const size_t o_ctr = take(sizeof(uint32_t) * kCounterWords);
    const size_t o_list = take(sizeof(PairRef) * (size_t)cap);
    rc = c->plain.ensure(off);
    if (rc) return rc;
    char* base = (char*)c->plain.p;
    PlainArgs a{};
    fill_kf_geometry(a.kd, *S, *K, P);
    a.kd.n_kp = n_kp;
    a.kd.hash_mask = hsize - 1;
    float sf[32];
    fill_search_const(P, a.sc, sf);
    a.sc.gate = mp_dmax != nullptr;
    a.n_mp = n_mp;
    a.add_cap = (int32_t)cap;
    a.mp_xyz = mp_xyz;
    a.mp_desc = mp_desc;
    a.mp_dmax = mp_dmax;
    a.mp_id = mp_id;
    a.kp_xy = kf->kp_xy;
    a.kp_oct = kf->kp_octave;
    a.kp_desc = kf->kp_desc;
    a.kp_owner = kf->kp_owner;
    a.hash = (const int32_t*)(base + o_hash);
    a.claim = (int32_t*)(base + o_claim);
    a.counters = (uint32_t*)(base + o_ctr);
    a.add_list = (PairRef*)(base + o_list);
    a.best_idx = out->best_idx;
    a.best_dist = out->best_dist;
    a.second_dist = out->second_dist;
    a.decision = out->decision;
    a.target = out->target;
    if (kf->cell_start) {
        a.cell_start = kf->cell_start;
        a.cell_kp = kf->cell_kp;
    } else {
        int32_t* cs = (int32_t*)(base + o_cs);
        int32_t* ck = (int32_t*)(base + o_ck);
        hipLaunchKernelGGL(grid_single_kernel, dim3(1), dim3(kPrepBlock), 0, stream, a.kd, cells, P->grid_cols,
                           P->grid_rows, kf->kp_xy, cs, ck);
        a.cell_start = cs;
        a.cell_kp = ck;
    }
    hipLaunchKernelGGL(plain_prep_kernel, dim3(1), dim3(kPrepBlock), 0, stream, n_kp, kf->kp_owner,
                       (int32_t*)(base + o_hash), hsize - 1, a.claim, a.counters);
    const int grid = (n_mp + 255) / 256;
    hipLaunchKernelGGL(search_plain_kernel, dim3(grid), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(resolve_plain_kernel, dim3(std::min(grid, 256)), dim3(256), 0, stream, n_mp,
                       (const uint32_t*)a.counters, (const PairRef*)a.add_list, (int32_t)cap,
                       (const int32_t*)a.claim, mp_id, (const int32_t*)out->best_idx, out->decision, out->target);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_validate_batch(const fl_batch* B, const fl_params* P, const fl_fuse_out* out) {
    return validate_batch(B, P, out);
}

int fl_search_fuse_batched(fl_ctx* c, const fl_batch* B, const fl_params* P, const fl_fuse_out* out,
                           hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = validate_batch(B, P, out);
    if (rc) return rc;
    if (B->n_pairs == 0 && B->n_kf == 0) return FL_OK;
    Prepared pr;
    rc = prepare_batch(c, B, P, out, nullptr, c->tune.pairs_per_lane, pr);
    if (rc) return rc;
    rc = upload_batch(c, pr, stream);
    if (rc) return rc;
    return launch_search(c, (const BatchHdr*)c->ws.p, stream, true, B->n_kf);
}

int fl_refine_events(fl_ctx* c, const fl_batch* B, const fl_fuse_out* out, const fl_refine* R, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    fl_params P{3.0f, 1.2f, 1, 1, 1, 0, 0.0f, 0};   // search thresholds are not used by refinement
    int rc = validate_batch(B, &P, out);
    if (rc) return rc;
    rc = check_refine(B, R);
    if (rc) return rc;
    if (!R || R->n_iters == 0 || B->n_events == 0) return FL_OK;
    Prepared pr;
    rc = prepare_batch(c, B, &P, out, R, c->tune.pairs_per_lane, pr);
    if (rc) return rc;
    pr.hdr.refine_scan = 1;
    rc = upload_batch(c, pr, stream);
    if (rc) return rc;
    return launch_refine((const BatchHdr*)c->ws.p, R->n_iters, stream);
}

int fl_search_fuse_graph_launch(fl_ctx* c, const fl_batch* B, const fl_params* P, const fl_fuse_out* out,
                                const fl_refine* R, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = validate_batch(B, P, out);
    if (rc) return rc;
    rc = check_refine(B, R);
    if (rc) return rc;
    if (B->n_pairs == 0 && B->n_kf == 0) return FL_OK;
    const int n_iters = (R && R->n_iters > 0) ? R->n_iters : 0;
    Prepared pr;
    rc = prepare_batch(c, B, P, out, R, c->tune.pairs_per_lane, pr);
    if (rc) return rc;
    const bool stale = !c->gexec || c->g_ws != c->ws.p || memcmp(&c->g_tune, &c->tune, sizeof(fl_tuning)) != 0 ||
                       c->g_stats != c->stats || c->g_refine != n_iters;
    if (stale) {
        if (c->gexec) {
            FL_HIP(hipStreamSynchronize(stream));
            hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        const BatchHdr* dh = (const BatchHdr*)c->ws.p;
        hipGraph_t graph = nullptr;
        FL_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        int lrc = launch_search(c, dh, c->cap_stream, false, B->n_kf);
        if (lrc == FL_OK && n_iters > 0) lrc = launch_refine(dh, n_iters, c->cap_stream);
        hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
        if (lrc) {
            if (graph) hipGraphDestroy(graph);
            return lrc;
        }
        if (ce != hipSuccess) return fail(FL_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            c->gexec = nullptr;
            return fail(FL_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
        }
        c->g_ws = c->ws.p;
        c->g_tune = c->tune;
        c->g_stats = c->stats;
        c->g_refine = n_iters;
    }
    rc = upload_batch(c, pr, stream);
    if (rc) return rc;
    FL_HIP(hipGraphLaunch(c->gexec, stream));
    return FL_OK;
}

// ---------------------------------------------------------------------------
// residual

static int residual_args(fl_ctx* c, int32_t n, const float* xyz, const float* uv, const int32_t* kf_idx,
                         int32_t n_kf, const float* kf_T, const fl_sim3* S, const fl_pinhole* K, float delta,
                         ResArgs& a, int& grid) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (n < 0 || n_kf < 0) return fail(FL_EINVAL, "negative count");
    if (!S) return fail(FL_EINVAL, "S is NULL");
    if (n > 0 && (!xyz || !uv)) return fail(FL_EINVAL, "xyz / uv must not be NULL");
    if (kf_idx && n_kf < 1) return fail(FL_EINVAL, "kf_idx given but n_kf < 1");
    int rc = check_cam(K, "residual");
    if (rc) return rc;
    if (!finite_pos(delta)) return fail(FL_EINVAL, "huber_delta must be finite and > 0");
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.n_kf = n_kf;
    a.xyz = xyz;
    a.uv = uv;
    a.kf_idx = kf_idx;
    a.kf_T = kf_T;
    a.S = S;
    a.fx = K->fx;
    a.fy = K->fy;
    a.cx = K->cx;
    a.cy = K->cy;
    a.delta = delta;
    a.partial = (double*)c->res.p;
    a.done = (uint32_t*)((char*)c->res.p + sizeof(double) * 1024 * kNAcc);
    grid = std::max(1, std::min((n + kResBlock - 1) / kResBlock, 1024));
    return FL_OK;
}

int fl_reproj_residual_fwd(fl_ctx* c, int32_t n, const float* xyz, const float* uv, const int32_t* kf_idx,
                           int32_t n_kf, const float* kf_T, const fl_sim3* S, const fl_pinhole* K, float huber_delta,
                           float* r, float* w, double* loss, hipStream_t stream) {
    ResArgs a;
    int grid = 1;
    int rc = residual_args(c, n, xyz, uv, kf_idx, n_kf, kf_T, S, K, huber_delta, a, grid);
    if (rc) return rc;
    if (!loss) return fail(FL_EINVAL, "loss must not be NULL");
    a.r = r;
    a.w = w;
    a.loss = loss;
    hipLaunchKernelGGL(residual_fwd_kernel, dim3(grid), dim3(kResBlock), 0, stream, a);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_reproj_residual_bwd(fl_ctx* c, int32_t n, const float* xyz, const float* uv, const int32_t* kf_idx,
                           int32_t n_kf, const float* kf_T, const fl_sim3* S, const fl_pinhole* K, float huber_delta,
                           double grad_scale, double* g, double* H, hipStream_t stream) {
    ResArgs a;
    int grid = 1;
    int rc = residual_args(c, n, xyz, uv, kf_idx, n_kf, kf_T, S, K, huber_delta, a, grid);
    if (rc) return rc;
    if (!g) return fail(FL_EINVAL, "g must not be NULL");
    if (!std::isfinite(grad_scale)) return fail(FL_EINVAL, "grad_scale must be finite");
    a.g = g;
    a.H = H;
    a.grad_scale = grad_scale;
    hipLaunchKernelGGL(residual_bwd_kernel, dim3(grid), dim3(kResBlock), 0, stream, a);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_sim3_exp_mul(fl_ctx* c, const double* xi, const double* S_in, double* S_out, fl_sim3* S32_out,
                    hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!xi || !S_in || !S_out) return fail(FL_EINVAL, "NULL argument");
    hipLaunchKernelGGL(sim3_exp_mul_kernel, dim3(1), dim3(64), 0, stream, xi, S_in, S_out, S32_out);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_gn_step(fl_ctx* c, const double* g, const double* H, double lambda, double* S, fl_sim3* S32,
               hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!g || !H || !S) return fail(FL_EINVAL, "NULL argument");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(FL_EINVAL, "lambda must be finite and >= 0");
    hipLaunchKernelGGL(gn_step_kernel, dim3(1), dim3(64), 0, stream, g, H, lambda, S, S32);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

// ---------------------------------------------------------------------------
// tuning and statistics

int fl_get_tuning(fl_ctx* c, fl_tuning* out) {
    if (!c || !out) return fail(FL_EINVAL, "NULL argument");
    *out = c->tune;
    return FL_OK;
}

int fl_set_tuning(fl_ctx* c, const fl_tuning* t) {
    if (!c || !t) return fail(FL_EINVAL, "NULL argument");
    if (t->pairs_per_lane != 1 && t->pairs_per_lane != 2 && t->pairs_per_lane != 4)
        return fail(FL_EINVAL, "pairs_per_lane must be 1, 2 or 4");
    if (t->block != 64 && t->block != 128 && t->block != 256) return fail(FL_EINVAL, "block must be 64, 128 or 256");
    if (t->waves_per_cu < 1 || t->waves_per_cu > 32) return fail(FL_EINVAL, "waves_per_cu must be in [1, 32]");
    if (t->xcd_queues != 0 && t->xcd_queues != 1) return fail(FL_EINVAL, "xcd_queues must be 0 or 1");
    c->tune = *t;
    return FL_OK;
}

int fl_autotune(fl_ctx* c, const fl_batch* B, const fl_params* P, const fl_fuse_out* out, int32_t reps,
                fl_tuning* best, float* best_ms, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = validate_batch(B, P, out);
    if (rc) return rc;
    if (reps < 1) reps = 3;
    hipEvent_t e0, e1;
    FL_HIP(hipEventCreate(&e0));
    FL_HIP(hipEventCreate(&e1));
    const fl_tuning saved = c->tune;
    fl_tuning top = saved;
    float top_ms = 1e30f;
    const int ppls[] = {1, 2, 4};
    const int blocks[] = {128, 256};
    const int wpcs[] = {8, 16, 32};
    for (int ppl : ppls)
        for (int blk : blocks)
            for (int wpc : wpcs)
                for (int xq = 0; xq <= 1; ++xq) {
                    c->tune = fl_tuning{ppl, blk, wpc, xq};
                    rc = fl_search_fuse_batched(c, B, P, out, stream);   // warm-up
                    if (rc) break;
                    hipEventRecord(e0, stream);
                    for (int r = 0; r < reps && rc == FL_OK; ++r) rc = fl_search_fuse_batched(c, B, P, out, stream);
                    hipEventRecord(e1, stream);
                    if (rc) break;
                    if (hipEventSynchronize(e1) != hipSuccess) {
                        rc = fail(FL_EHIP, "hipEventSynchronize failed");
                        break;
                    }
                    float ms = 0.0f;
                    hipEventElapsedTime(&ms, e0, e1);
                    ms /= (float)reps;
                    if (ms < top_ms) {
                        top_ms = ms;
                        top = c->tune;
                    }
                }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tune = rc == FL_OK ? top : saved;
    if (rc) return rc;
    if (best) *best = top;
    if (best_ms) *best_ms = top_ms;
    return FL_OK;
}

int fl_set_stats(fl_ctx* c, int enable) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    c->stats = enable ? 1 : 0;
    return FL_OK;
}

int fl_get_stats(fl_ctx* c, int64_t* out4) {
    if (!c || !out4) return fail(FL_EINVAL, "NULL argument");
    if (!c->ws.p) return fail(FL_EINVAL, "no batched search has run on this context");
    // the stats block follows the fixed-size regions; its device address is in the header
    BatchHdr h;
    FL_HIP(hipMemcpy(&h, c->ws.p, sizeof(h), hipMemcpyDeviceToHost));
    unsigned long long v[4];
    FL_HIP(hipMemcpy(v, h.stats_out, sizeof(v), hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) out4[i] = (int64_t)v[i];
    return FL_OK;
}

static void clear_profile(fl_ctx* c) {
    for (auto& pr : c->prof_ev) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
    }
    c->prof_ev.clear();
}

int fl_set_profiling(fl_ctx* c, int enable) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    c->prof = enable ? 1 : 0;
    clear_profile(c);
    return FL_OK;
}

int fl_get_profile(fl_ctx* c, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches) return fail(FL_EINVAL, "NULL argument");
    double sum = 0.0;
    if (!c->prof_ev.empty()) FL_HIP(hipEventSynchronize(c->prof_ev.back().second));
    for (auto& pr : c->prof_ev) {
        float ms = 0.0f;
        FL_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)c->prof_ev.size();
    clear_profile(c);
    return FL_OK;
}

// Test hook: cap the provisional-ADD and matched-pair lists at `cap` entries
// (0 restores the default) so the overflow paths can be exercised.
int fl_debug_set_list_cap(fl_ctx* c, int32_t cap) {
    if (!c || cap < 0) return fail(FL_EINVAL, "bad argument");
    c->add_cap_override = cap;
    return FL_OK;
}

}  // extern "C"
