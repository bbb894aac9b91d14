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
#include <mutex>
#include <queue>
#include <vector>

#include "fastloop.h"
#include "fl_internal.h"
#include "fl_pgo.h"
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
    // Grow to at least `need` bytes; a new allocation is filled with `fill`
    // (-1: left uninitialised).
    int ensure(size_t need, int fill = -1) {
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
        if (fill >= 0 && hipMemset(p, fill, n) != hipSuccess) return fail(FL_EHIP, "hipMemset failed");
        return FL_OK;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        size = 0;
    }
};

// Pinned staging buffer with an event marking when its last upload finished.
constexpr int kPinRing = 16;   // staging buffers in flight

struct Pinned {
    void* p = nullptr;
    size_t size = 0;
    size_t used = 0;            // bytes of tables staged in it
    bool pending = false;       // a fetch from it may still be queued
    uint64_t seq = 0;           // upload number of its last fetch
    hipStream_t stream = nullptr;   // ... and the stream it was queued on
};

// Table fetches (eager uploads and graph replays) record an event only every
// kFenceEvery fetches.  A staging buffer is rewritten at least kFenceEvery
// fetches after its last one (kPinRing distinct eager uploads, kGraphRing
// graph replays), by which time a fence recorded on the same stream after
// that fetch exists.
constexpr int kFenceEvery = 8;
constexpr int kFences = 4;
constexpr int kGraphRing = 8;   // graph executables replayed in turn, each with its own tables
static_assert(kPinRing >= kFenceEvery && kGraphRing >= kFenceEvery,
              "a fence must follow every fetch before its buffer returns");
struct Fence {
    hipEvent_t ev = nullptr;
    uint64_t seq = 0;           // upload number it follows; 0: never recorded
    hipStream_t stream = nullptr;
};


}  // namespace

struct fl_ctx {
    int device = 0;
    int n_cu = 256;
    size_t lds_max = 65536;     // dynamic LDS per workgroup the device allows
    DevBuf ws;                  // batched workspace (tables, global grids, lists, partials)
    DevBuf claims;              // ADD claims, 0xFF.. between epochs
    DevBuf ctrs;                // stats + per-keyframe + per-event counters, zero at rest
    DevBuf diag;                // sink of the VALU issue-rate probe
    DevBuf plain;               // plain-path workspace
    DevBuf res;                 // residual partials and done counter
    DevBuf part;                // refinement partial sums and their tags, zero when the epoch restarts
    DevBuf pgo;                 // pose-graph tables and workspace
    Pinned pin[kPinRing];
    int pin_next = 0;
    Fence fence[kFences];
    int fence_next = 0;
    uint64_t upload_seq = 0;    // eager uploads so far
    hipStream_t cap_stream = nullptr;
    fl_tuning tune{1, kModeLdsDesc, 1, 1};
    uint32_t launches = 0;      // table fetches since the claims were last reset
    Pinned* pin_last = nullptr; // ring buffer of the last eager upload
    int stats = 0;
    int add_cap_override = 0;   // test hook: >0 forces small accepted-pair (and plain-path ADD) list capacities
    int prof = 0;               // record events around eager search and refinement kernels
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[2];   // by FL_PROF_* class
    std::vector<hipEvent_t> ev_pool;   // events of read profiles, reused (no event creation per launch)
    // captured graph and its key
    hipGraphExec_t gexec[kGraphRing] = {};   // replayed in turn
    Pinned gpin[kGraphRing];    // the pinned tables each graph fetches from
    int g_next = 0;
    void* g_ws = nullptr;
    void* g_claims = nullptr;
    void* g_ctrs = nullptr;
    int g_mode = -1, g_ppl = -1, g_grid = -1, g_refine = -1;
    size_t g_lds = 0;
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

// Wait until the last fetch from p has run: the oldest fence recorded after
// it on its stream, or a device-wide wait if the fetches changed streams.
int wait_fetched(fl_ctx* c, Pinned& p) {
    if (!p.pending) return FL_OK;
    const Fence* f = nullptr;
    for (const Fence& g : c->fence)
        if (g.seq != 0 && g.seq >= p.seq && g.stream == p.stream && (!f || g.seq < f->seq)) f = &g;
    if (f) FL_HIP(hipEventSynchronize(f->ev));
    else FL_HIP(hipDeviceSynchronize());
    p.pending = false;
    return FL_OK;
}

// A fetch from p was just queued on stream.
int note_fetch(fl_ctx* c, Pinned& p, hipStream_t stream) {
    const uint64_t seq = ++c->upload_seq;
    p.seq = seq;
    p.stream = stream;
    p.pending = true;
    if (seq % kFenceEvery == 0) {
        Fence& f = c->fence[c->fence_next];
        c->fence_next = (c->fence_next + 1) % kFences;
        FL_HIP(hipEventRecord(f.ev, stream));
        f.seq = seq;
        f.stream = stream;
    }
    return FL_OK;
}

int get_pinned(fl_ctx* c, size_t need, Pinned** out) {
    Pinned& p = c->pin[c->pin_next];
    c->pin_next = (c->pin_next + 1) % kPinRing;
    const int rc = wait_fetched(c, p);
    if (rc) return rc;
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


// ---------------------------------------------------------------------------
// batch preparation

constexpr int kPrepGrid = 512;     // workgroups of the global-grid build
constexpr int kRefineGrid = 256;   // workgroups of a refinement step

struct Prepared {
    std::vector<char> blob;     // header + tables, uploaded per call
    BatchHdr* hdr = nullptr;
    int mode = kModeGlobal;
    int ppl = 1;
    int grid = 1;
    size_t lds = 16;
    size_t blob_cap = 0;
    int refine_iters = 0;
    int refine_variant = 0;           // refinement kernel: bit 0 Levenberg-Marquardt, bit 1 rounds
    bool resolve_in_refine = false;   // the refinement launch resolves the ADD conflicts
};

template <typename T>
size_t blob_take(std::vector<char>& blob, size_t n) {
    size_t off = align_up(blob.size(), 256);
    blob.resize(off + sizeof(T) * std::max<size_t>(n, 1), 0);
    return off;
}

// Pairs per tile of every keyframe; returns the number of tiles.  A
// workgroup runs on one CU and spreads a tile's waves over its four SIMDs,
// so a tile takes time in proportion to its waves per SIMD.  Full tiles
// (tile_cap pairs) are the fewest; while they number fewer than the
// workgroup slots, the spare slots go one at a time to the keyframe whose
// tiles cost most (pairs times the keypoint density the candidate scan
// meets), which cuts that keyframe into more, smaller tiles.  A tile of more
// than 256 pairs is a multiple of 256 (the same waves on every SIMD), a
// smaller one a multiple of 64.
int64_t plan_tiles(const std::vector<int64_t>& pairs, const std::vector<int32_t>& kps, int cells, int64_t tile_cap,
                   int slots, std::vector<int32_t>& tile) {
    const int n_kf = (int)pairs.size();
    tile.assign(n_kf, (int32_t)tile_cap);
    std::vector<int64_t> nt(n_kf, 0), most(n_kf, 0);
    std::vector<double> cost(n_kf, 0.0);
    int64_t total = 0;
    for (int k = 0; k < n_kf; ++k) {
        const int64_t np = pairs[k];
        const int n_kp = kps[k];
        nt[k] = (np + tile_cap - 1) / tile_cap;
        most[k] = (np + kWave - 1) / kWave;
        cost[k] = (double)np * (1.0 + 2.0 * n_kp / std::max(1, cells));
        total += nt[k];
    }
    if (total < slots) {
        std::priority_queue<std::pair<double, int>> q;   // (cost per tile, keyframe)
        for (int k = 0; k < n_kf; ++k)
            if (nt[k] > 0 && nt[k] < most[k]) q.push({cost[k] / (double)nt[k], k});
        while (total < slots && !q.empty()) {
            const int k = q.top().second;
            q.pop();
            ++nt[k];
            ++total;
            if (nt[k] < most[k]) q.push({cost[k] / (double)nt[k], k});
        }
    }
    int64_t n = 0;
    for (int k = 0; k < n_kf; ++k) {
        const int64_t np = pairs[k];
        if (np <= 0) continue;
        int64_t ts = (np + nt[k] - 1) / nt[k];
        const int64_t unit = ts > 256 ? 256 : kWave;
        ts = std::min(tile_cap, (ts + unit - 1) / unit * unit);
        tile[k] = (int32_t)ts;
        n += (np + ts - 1) / ts;
    }
    return n;
}

// Choose the staging mode and the octave groups per cell: the most groups
// (up to one per octave, at most max_nb) whose LDS footprint fits in the
// tuned mode or a smaller one, and whose record slots (two per keypoint with
// more than one group) stay below 65536.
int pick_mode(const fl_ctx* c, int want, int kp_cap, int cells, int hash_cap, int max_nb, int* nb_out) {
    for (int nb = max_nb; nb >= 1; nb = nb > 4 ? 4 : nb / 2) {
        if (search_slots(kp_cap, nb) > FL_MAX_KP) continue;
        for (int m = want; m > kModeGlobal; --m)
            if (search_lds_bytes(m, kp_cap, cells, hash_cap, nb) <= c->lds_max) {
                *nb_out = nb;
                return m;
            }
    }
    *nb_out = 1;
    return kModeGlobal;
}

// graph: the launch shape is kept stable across batches of different sizes,
// so a captured graph can be replayed for them (the grid is always every
// workgroup slot, empty ranges exit at once; the dynamic LDS is rounded up to
// a 16 KB step).
// passes: n_pass searches of the batch in one launch (NULL: one, with P, out
// and the batch's kf_sim3).  P holds the grid and octave fields every pass
// shares.  Each (keyframe, pass) gets a descriptor of its own, keyframe-major,
// so the passes of a keyframe are consecutive in the tile order.
int prepare_batch(fl_ctx* c, const fl_batch* B, const fl_params* P, const fl_fuse_out* out, const fl_refine* R,
                  bool refine_scan, Prepared& pr, bool graph = false, int n_pass = 1,
                  const fl_pass* passes = nullptr) {
    const int cells = P->grid_cols * P->grid_rows;
    const int n_kf = B->n_kf, n_ev = B->n_events;
    const int n_vk = n_kf * n_pass;   // descriptors
    if ((int64_t)n_pass * B->n_kp_total > INT32_MAX) return fail(FL_ERANGE, "too many keypoints for %d passes", n_pass);
    const int ppl = c->tune.pairs_per_lane;
    const int64_t tile_cap = (int64_t)kSearchBlock * ppl;
    const bool refine = R && R->n_iters > 0;
    pr.ppl = ppl;
    pr.refine_iters = refine ? R->n_iters : 0;
    pr.refine_variant = refine ? (R->lm_lambda > 0.0f ? 1 : 0) | (R->n_rounds > 1 ? 2 : 0) : 0;
    int kp_cap = 1;
    for (int k = 0; k < n_kf; ++k) kp_cap = std::max(kp_cap, B->kp_offset[k + 1] - B->kp_offset[k]);
    const int lds_hash_cap = std::max(64, next_pow2(kp_cap + 1));
    // octave groups: one per octave (at most 8) with the gate on; one group
    // (the plain grid) with the gate off and for counting launches, whose
    // keypoint counts are per grid cell
    const bool gate = B->mp_dmax != nullptr;
    const int max_nb = (gate && !c->stats) ? std::min(P->n_octaves, 8) : 1;
    int nb = 1;
    pr.mode = pick_mode(c, c->tune.lds_mode, kp_cap, cells, lds_hash_cap, max_nb, &nb);
    pr.lds = search_lds_bytes(pr.mode, kp_cap, cells, lds_hash_cap, nb);
    if (graph && pr.mode != kModeGlobal) pr.lds = std::min(c->lds_max, align_up(pr.lds, 16384));

    // workgroups of the search launch (every slot in graph mode, at most one
    // per tile otherwise)
    const int slots = std::max(1, c->n_cu * std::max(1, c->tune.wg_per_cu));
    std::vector<int32_t> kf_tile;
    int64_t n_tiles_all = 0;
    {
        std::vector<int64_t> vp(n_vk);
        std::vector<int32_t> vk(n_vk);
        for (int v = 0; v < n_vk; ++v) {
            const int k = v / n_pass;
            vp[v] = B->pair_offset[k + 1] - B->pair_offset[k];
            vk[v] = B->kp_offset[k + 1] - B->kp_offset[k];
        }
        n_tiles_all = plan_tiles(vp, vk, cells, tile_cap, slots, kf_tile);
    }
    int grid = slots;
    if (!graph) grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, n_tiles_all));
    pr.grid = grid;

    // Table blob: header, the workgroups' tile ranges and the keyframe table
    // first, at offsets the kernel derives from its grid size alone.
    std::vector<char>& blob = pr.blob;
    blob.clear();
    const size_t o_hdr = blob_take<BatchHdr>(blob, 1);
    const size_t o_range = blob_take<WgRange>(blob, grid);
    const size_t o_kf = blob_take<KfDesc>(blob, n_vk);
    if (o_hdr != 0 || o_range != blob_range_offset() || o_kf != blob_kf_offset(grid))
        return fail(FL_EINVAL, "internal: table layout mismatch");
    const size_t o_ev = blob_take<EventDesc>(blob, n_ev);
    const size_t o_order = blob_take<int32_t>(blob, n_vk);
    const size_t o_prefix = blob_take<int32_t>(blob, n_vk + 1);
    KfDesc* kfd = (KfDesc*)(blob.data() + o_kf);
    EventDesc* evd = (EventDesc*)(blob.data() + o_ev);

    // keyframes, events, list regions, tiles
    int64_t hash_total = 0, list_total = 0;
    std::vector<double> tile_cost;    // cost of each keyframe's tiles (per tile)
    tile_cost.resize(n_vk);
    for (int e = 0; e < n_ev; ++e) {
        EventDesc& ed = evd[e];
        const int kb = B->event_kf_offset[e], ke = B->event_kf_offset[e + 1];
        ed.kf_begin = kb * n_pass;   // descriptor range
        ed.kf_end = ke * n_pass;
        ed.mp_off = B->event_mp_offset[e];
        ed.n_mp = B->event_mp_offset[e + 1] - ed.mp_off;
        ed.pair_begin = B->pair_offset[kb];
        ed.pair_end = B->pair_offset[ke];
        const int64_t kp_ev = B->kp_offset[ke] - B->kp_offset[kb];
        int64_t cap = std::min<int64_t>(ed.pair_end - ed.pair_begin, std::max<int64_t>(2 * kp_ev, 4096));
        if (c->add_cap_override > 0) cap = std::min<int64_t>(cap, c->add_cap_override);
        ed.list_off = refine ? (int32_t)list_total : 0;
        ed.list_cap = refine ? (int32_t)cap : 0;
        const fl_refine_inverse* V = refine ? R->inverse : nullptr;
        ed.inv_off = V ? (int32_t)V->event_offset[e] : 0;
        ed.inv_n = V ? (int32_t)(V->event_offset[e + 1] - V->event_offset[e]) : 0;
        if (refine) list_total += cap;
        for (int k = kb; k < ke; ++k) {
            // the keyframe's global grid and owner hash set serve every pass
            const int n_kp = B->kp_offset[k + 1] - B->kp_offset[k];
            const int hsize = next_pow2(2 * n_kp);
            const int32_t hash_off = (int32_t)hash_total;
            hash_total += hsize;
            for (int p = 0; p < n_pass; ++p) {
                const int v = k * n_pass + p;
                KfDesc& kd = kfd[v];
                const fl_sim3& S = (passes && passes[p].kf_sim3) ? passes[p].kf_sim3[k] : B->kf_sim3[k];
                fill_kf_geometry(kd, S, B->kf_K[k], P);
                if (B->kf_T)
                    for (int i = 0; i < 12; ++i) kd.T[i] = B->kf_T[12 * (int64_t)k + i];
                kd.kp_off = B->kp_offset[k];
                kd.n_kp = n_kp;
                kd.grid_off = k * (cells + 1);
                kd.event = e;
                kd.mp_off = ed.mp_off;
                kd.n_mp = ed.n_mp;
                kd.hash_off = hash_off;
                kd.hash_mask = hsize - 1;
                kd.pair_off = B->pair_offset[k];
                kd.n_pairs = B->pair_offset[k + 1] - B->pair_offset[k];
                kd.tile_pairs = kf_tile[v];
                kd.n_tiles = (int32_t)((kd.n_pairs + kd.tile_pairs - 1) / kd.tile_pairs);
                kd.pass = p;
                kd.stage_key = k;
                kd.claim_off = p * B->n_kp_total + kd.kp_off;
                // a pair costs more where keypoints are dense (more candidates scanned)
                tile_cost[v] = (double)kd.tile_pairs * (1.0 + 2.0 * kd.n_kp / std::max(1, cells));
            }
        }
    }
    // every (keyframe, pass) descriptor's pairs, in tile order: the index
    // space of the workgroups' list regions
    int64_t n_virtual = 0;
    for (int v = 0; v < n_vk; ++v) n_virtual += kfd[v].n_pairs;
    if (n_virtual > INT32_MAX || list_total > INT32_MAX || hash_total > INT32_MAX)
        return fail(FL_ERANGE, "batch too large for the workspace indexing");
    // tile order: keyframes in batch order
    int32_t* order = (int32_t*)(blob.data() + o_order);
    int32_t* prefix = (int32_t*)(blob.data() + o_prefix);
    int64_t n_tiles = 0;
    for (int k = 0; k < n_vk; ++k) {
        order[k] = k;
        prefix[k] = (int32_t)n_tiles;
        n_tiles += kfd[k].n_tiles;
        if (n_tiles > INT32_MAX / 2) return fail(FL_ERANGE, "too many tiles");
    }
    prefix[n_vk] = (int32_t)n_tiles;
    if (n_tiles != n_tiles_all) return fail(FL_EINVAL, "internal: tile count mismatch");
    // the workgroups' contiguous, cost-balanced tile ranges
    WgRange* wr = (WgRange*)(blob.data() + o_range);
    {
        // first pair of tile t in the list index space (t = n_tiles: its end)
        std::vector<int64_t> vbase(n_vk + 1, 0);
        for (int k = 0; k < n_vk; ++k) vbase[k + 1] = vbase[k] + kfd[order[k]].n_pairs;
        auto tile_pair = [&](int64_t t) -> int64_t {
            if (t >= n_tiles) return n_virtual;
            const int s = (int)(std::upper_bound(prefix, prefix + n_vk + 1, (int32_t)t) - prefix) - 1;
            const KfDesc& kd = kfd[order[s]];
            return vbase[s] + std::min<int64_t>((t - prefix[s]) * (int64_t)kd.tile_pairs, kd.n_pairs);
        };
        // cumulative cost at each tile boundary, by keyframe
        std::vector<double> kcum(n_vk + 1, 0.0);
        for (int k = 0; k < n_vk; ++k) kcum[k + 1] = kcum[k] + tile_cost[k] * kfd[k].n_tiles;
        auto tile_at_cost = [&](double target) -> int64_t {   // first tile whose end cost >= target
            if (target <= 0.0) return 0;
            int k = (int)(std::upper_bound(kcum.begin(), kcum.end(), target) - kcum.begin()) - 1;
            k = std::min(std::max(k, 0), n_vk - 1);
            const double per = tile_cost[k] > 0 ? tile_cost[k] : 1.0;
            int64_t j = (int64_t)std::ceil((target - kcum[k]) / per);
            j = std::min<int64_t>(std::max<int64_t>(j, 0), kfd[k].n_tiles);
            return prefix[k] + j;
        };
        const double total = kcum[n_vk];
        // The tiles are laid out over ge = min(grid, tiles) workgroups, as an
        // eager launch has them; a graph's further workgroups (its grid is
        // fixed) get empty ranges and exit at once.
        const int ge = (int)std::max<int64_t>(1, std::min<int64_t>(grid, n_tiles));
        std::vector<int64_t> bound(ge + 1);
        bound[0] = 0;
        bound[ge] = n_tiles;
        if (n_tiles <= 2 * (int64_t)ge) {
            // at most two tiles per workgroup: equal counts (a single wave of
            // tiles is latency bound, so a workgroup must not take more)
            for (int i = 1; i < ge; ++i) bound[i] = n_tiles * i / ge;
        } else {
            for (int i = 1; i < ge; ++i) bound[i] = tile_at_cost(total * i / ge);
        }
        for (int i = 1; i <= ge; ++i) bound[i] = std::max(bound[i], bound[i - 1]);
        for (int i = ge - 1; i >= 0; --i) bound[i] = std::min(bound[i], bound[i + 1]);
        // chunk i of the sequence goes to workgroup w(i); with xcd_aware the
        // chunks of one XCD's share are consecutive in the sequence
        std::vector<int> wg_of(ge);
        if (c->tune.xcd_aware && ge >= 2 * kMaxQueues) {
            int i = 0;
            for (int x = 0; x < kMaxQueues; ++x)
                for (int b = x; b < ge; b += kMaxQueues) wg_of[i++] = b;
        } else {
            for (int i = 0; i < ge; ++i) wg_of[i] = i;
        }
        for (int i = 0; i < ge; ++i) {
            // slot of the first tile: prefix[slot] <= tile < prefix[slot + 1]
            const int64_t t0 = bound[i];
            int slot = (int)(std::upper_bound(prefix, prefix + n_vk + 1, (int32_t)t0) - prefix) - 1;
            slot = std::min(std::max(slot, 0), std::max(n_vk - 1, 0));
            WgRange& g = wr[wg_of[i]];
            g.t0 = (int32_t)t0;
            g.t1 = (int32_t)bound[i + 1];
            g.slot = slot;
            g.kf = order[slot];
            const int64_t p0 = tile_pair(t0), p1 = tile_pair(bound[i + 1]);
            g.priv_off = (int32_t)p0;
            g.priv_cap = (int32_t)(p1 - p0);
        }
        for (int i = ge; i < grid; ++i) {
            WgRange& g = wr[i];
            g.t0 = g.t1 = (int32_t)n_tiles;
            g.slot = 0;
            g.kf = order[0];
            g.priv_off = (int32_t)n_virtual;
            g.priv_cap = 0;
        }
    }

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 16), 256);
        return o;
    };
    // the tables region has a power-of-two capacity: a captured graph fetches
    // the whole capacity from its pinned buffer
    pr.blob_cap = std::max<size_t>(65536, 1);
    while (pr.blob_cap < blob.size()) pr.blob_cap <<= 1;
    const size_t L_blob = take(pr.blob_cap);
    const bool global_grid = pr.mode == kModeGlobal;
    const size_t L_cs = take(global_grid ? sizeof(int32_t) * (size_t)n_kf * (cells + 1) : 0);
    const size_t L_recs = take(global_grid ? sizeof(KpRec) * (size_t)B->n_kp_total : 0);
    const size_t L_desc = take(global_grid ? 32 * (size_t)B->n_kp_total : 0);
    const size_t L_ck = take(global_grid ? sizeof(int32_t) * (size_t)B->n_kp_total : 0);
    const size_t L_hash = take(global_grid ? sizeof(int32_t) * (size_t)hash_total : 0);
    const size_t L_add = take(sizeof(AddRef) * (size_t)n_virtual);
    const size_t L_add_count = take(sizeof(uint32_t) * (size_t)grid);
    const size_t L_stage = take(refine ? sizeof(MatchRec) * (size_t)n_virtual : 0);
    const size_t L_match = take(sizeof(MatchRec) * (size_t)list_total);
    const int refine_blocks = std::max(1, std::min(kRefMaxB, kRefineGrid / std::max(1, n_ev)));
    const size_t n_rows = 2 * (size_t)n_ev * refine_blocks;
    int rc = c->ws.ensure(off);
    if (rc) return rc;
    // Tags in the partial-sum buffer must never match a tag of a later
    // launch: the buffer is zeroed when allocated and whenever the epoch
    // restarts.
    const void* old_part = c->part.p;
    rc = c->part.ensure(sizeof(unsigned long long) * kRefWords * n_rows, 0x00);
    if (rc) return rc;
    rc = c->claims.ensure(sizeof(unsigned long long) * (size_t)std::max(n_pass * B->n_kp_total, 1), 0xFF);
    if (rc) return rc;
    const void* old_ctrs = c->ctrs.p;
    rc = c->ctrs.ensure(64 + sizeof(uint32_t) * (size_t)kEvCtrs * n_ev, 0x00);
    if (rc) return rc;
    if (c->ctrs.p != old_ctrs && old_ctrs != nullptr) {
        // a fresh counter block restarts the epoch: every stored claim must be reset too
        if (hipMemset(c->claims.p, 0xFF, c->claims.size) != hipSuccess) return fail(FL_EHIP, "hipMemset failed");
        if (c->part.p == old_part && hipMemset(c->part.p, 0, c->part.size) != hipSuccess)
            return fail(FL_EHIP, "hipMemset failed");
        c->launches = 0;
    }
    char* base = (char*)c->ws.p;
    char* cb = (char*)c->ctrs.p;

    BatchHdr& h = *(BatchHdr*)(blob.data() + o_hdr);
    pr.hdr = &h;
    h.n_events = n_ev;
    h.n_kf = n_vk;
    h.n_mp = B->n_mp;
    h.n_kp_total = B->n_kp_total;
    h.n_pairs = B->n_pairs;
    h.n_tiles = (int32_t)n_tiles;
    h.tile_cap = (int32_t)tile_cap;
    h.cells = cells;
    h.grid_cols = P->grid_cols;
    h.grid_rows = P->grid_rows;
    h.n_octaves = P->n_octaves;
    h.n_pass = n_pass;
    for (int p = 0; p < n_pass; ++p) {
        const fl_params& Pp = passes ? passes[p].params : *P;
        const fl_fuse_out& op = passes ? passes[p].out : *out;
        PassOut& po = h.out[p];
        po.best_idx = op.best_idx;
        po.best_dist = op.best_dist;
        po.second_dist = op.second_dist;
        po.decision = op.decision;
        po.target = op.target;
        po.hamming_th = Pp.hamming_th;
        po.nn_ratio = Pp.nn_ratio;
        po.r0 = Pp.win_px;
    }
    h.gate = B->mp_dmax != nullptr;
    h.dense = B->pair_mp == nullptr;
    h.stats = c->stats;
    h.lds_hash_mask = lds_hash_cap - 1;
    h.lds_kp_cap = kp_cap;   // the record capacity search_lds_bytes sized
    h.oct_buckets = nb;
    h.n_wg = grid;
    SearchConst sc;
    fill_search_const(P, sc, h.sf);
    h.kf = (const KfDesc*)(base + L_blob + o_kf);
    h.ev = (const EventDesc*)(base + L_blob + o_ev);
    h.kf_order = (const int32_t*)(base + L_blob + o_order);
    h.tile_prefix = (const int32_t*)(base + L_blob + o_prefix);
    h.wg_range = (const WgRange*)(base + L_blob + o_range);
    h.kp_xy = B->kp_xy;
    h.kp_oct = B->kp_octave;
    h.kp_desc = B->kp_desc;
    h.kp_owner = B->kp_owner;
    h.mp_xyz = B->mp_xyz;
    h.mp_desc = B->mp_desc;
    h.mp_dmax = B->mp_dmax;
    h.mp_id = B->mp_id;
    h.pair_mp = B->pair_mp;
    h.cell_start = (int32_t*)(base + L_cs);
    h.recs = (KpRec*)(base + L_recs);
    h.desc_sorted = (uint4*)(base + L_desc);
    h.cell_kp = (int32_t*)(base + L_ck);
    h.hash = (int32_t*)(base + L_hash);
    h.claim = (unsigned long long*)c->claims.p;
    h.stats_out = (unsigned long long*)cb;
    h.epoch = (const uint32_t*)(cb + 32);
    h.ev_ctr = (uint32_t*)(cb + 64);
    h.add_list = (AddRef*)(base + L_add);
    h.add_count = (uint32_t*)(base + L_add_count);
    h.match_stage = (MatchRec*)(base + L_stage);
    h.match_list = (MatchRec*)(base + L_match);
    h.refine_blocks = refine_blocks;
    h.refine_scan = refine_scan ? 1 : 0;
    // a refinement that follows a search in the same call resolves its ADD
    // conflicts; otherwise launch_search adds the resolution kernel
    pr.resolve_in_refine = refine && !refine_scan;
    h.resolve_in_refine = pr.resolve_in_refine ? 1 : 0;
    h.refine_rows = (unsigned long long*)c->part.p;
    if (refine) {
        h.refine_iters = R->n_iters;
        h.huber_delta = R->huber_delta;
        h.refine_rounds = std::max(R->n_rounds, 1);
        h.outlier_px = R->n_rounds > 1 ? R->outlier_px : INFINITY;
        h.lm_lambda = R->lm_lambda;
        h.event_S = R->event_S;
        h.event_S32_out = R->event_S32;
        h.event_n_matched = R->event_n_matched;
        if (const fl_refine_inverse* V = R->inverse) {
            h.inv_xyz = V->xyz;
            h.inv_uv = V->uv;
            h.inv_kf = V->kf_idx;
            h.inv_T = V->kf_T;
            h.inv_cam = V->kf_cam;
            h.inv_n_kf = V->n_kf;
        }
    }
    return FL_OK;
}

// Fill n 32-bit words with a value (used in place of memset nodes, which a
// caller's stream capture would record).
__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u32(void* p, size_t bytes, uint32_t v, hipStream_t stream) {
    const size_t n = bytes / 4;
    if (n == 0) return;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid), dim3(256), 0, stream, (uint32_t*)p, n, v);
}

// Count launches.  When the device epoch (decremented by every table fetch)
// is about to run out, reset every claim and the epoch.  The refinement's
// partial-sum rows are zeroed whenever their tags are about to repeat
// (every 2^kTagEpochBits launches) and at every epoch reset.
int next_epoch(fl_ctx* c, hipStream_t stream) {
    if (++c->launches >= 0xFFFFFFF0u) {
        fill_u32(c->claims.p, c->claims.size, 0xFFFFFFFFu, stream);
        fill_u32((char*)c->ctrs.p + 32, 4, 0u, stream);
        if (c->part.p) fill_u32(c->part.p, c->part.size, 0u, stream);
        c->launches = 1;
    } else if (refine_rows_cleared_before(c->launches) && c->part.p) {
        // a refinement of this context still running on another stream would
        // lose its rows: let it finish first (once per 2^22 launches)
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        FL_HIP(hipStreamIsCapturing(stream, &cs));
        if (cs == hipStreamCaptureStatusNone) FL_HIP(hipDeviceSynchronize());
        fill_u32(c->part.p, c->part.size, 0u, stream);
    }
    FL_HIP(hipGetLastError());
    return FL_OK;
}

void launch_fetch(fl_ctx* c, const void* src, size_t bytes, hipStream_t stream) {
    const int n16 = (int)((bytes + 15) / 16);
    const int grid = std::max(1, std::min((n16 + 255) / 256, 64));
    hipLaunchKernelGGL(fetch_blob_kernel, dim3(grid), dim3(256), 0, stream, (const uint4*)src, (uint4*)c->ws.p, n16,
                       (uint32_t*)((char*)c->ctrs.p + 32));
}

// Eager calls: stage the header and tables in a pinned ring buffer and fetch
// them into the workspace with a copy kernel on the launch stream.
int upload_batch(fl_ctx* c, Prepared& pr, hipStream_t stream) {
    int rc = next_epoch(c, stream);
    if (rc) return rc;
    Pinned* last = c->pin_last;
    Pinned* pin = nullptr;
    if (last && last->used == pr.blob.size() && memcmp(last->p, pr.blob.data(), pr.blob.size()) == 0) {
        pin = last;   // unchanged tables: fetch again from the same buffer, nothing is overwritten
    } else {
        rc = get_pinned(c, pr.blob.size(), &pin);
        if (rc) return rc;
        memcpy(pin->p, pr.blob.data(), pr.blob.size());
        pin->used = pr.blob.size();
    }
    launch_fetch(c, pin->p, pr.blob.size(), stream);
    FL_HIP(hipGetLastError());
    c->pin_last = pin;
    return note_fetch(c, *pin, stream);
}

template <int PPL, int MODE, bool STATS>
void launch_fused(const BatchHdr* dh, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((search_fused_kernel<PPL, MODE, STATS>), dim3(grid), dim3(kSearchBlock), lds, s, dh);
}

template <int PPL, int MODE>
void launch_fused_s(bool stats, const BatchHdr* dh, int grid, size_t lds, hipStream_t s) {
    if (stats) launch_fused<PPL, MODE, true>(dh, grid, lds, s);
    else launch_fused<PPL, MODE, false>(dh, grid, lds, s);
}

template <int PPL>
void launch_fused_m(int mode, bool stats, const BatchHdr* dh, int grid, size_t lds, hipStream_t s) {
    if (mode == kModeLdsDesc) launch_fused_s<PPL, kModeLdsDesc>(stats, dh, grid, lds, s);
    else if (mode == kModeLdsRec) launch_fused_s<PPL, kModeLdsRec>(stats, dh, grid, lds, s);
    else launch_fused_s<PPL, kModeGlobal>(stats, dh, grid, lds, s);
}


// An event for a profiled launch: from the context's pool, else new.
int prof_event(fl_ctx* c, hipEvent_t* e) {
    if (!c->ev_pool.empty()) {
        *e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return FL_OK;
    }
    FL_HIP(hipEventCreate(e));
    return FL_OK;
}

int launch_search(fl_ctx* c, const Prepared& pr, const BatchHdr* dh, hipStream_t s, bool eager, bool stats) {
    if (pr.mode == kModeGlobal) {
        const int pg = eager ? std::max(1, std::min(pr.hdr->n_kf, kPrepGrid)) : kPrepGrid;
        hipLaunchKernelGGL(prep_global_kernel, dim3(pg), dim3(kPrepBlock), 0, s, dh);
    }
    const bool timed = eager && c->prof;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (timed) {
        int rc = prof_event(c, &t0);
        if (!rc) rc = prof_event(c, &t1);
        if (rc) return rc;
        FL_HIP(hipEventRecord(t0, s));
    }
    if (pr.ppl == 1) launch_fused_m<1>(pr.mode, stats, dh, pr.grid, pr.lds, s);
    else if (pr.ppl == 2) launch_fused_m<2>(pr.mode, stats, dh, pr.grid, pr.lds, s);
    else launch_fused_m<4>(pr.mode, stats, dh, pr.grid, pr.lds, s);
    if (timed) {
        FL_HIP(hipEventRecord(t1, s));
        c->prof_ev[FL_PROF_SEARCH].emplace_back(t0, t1);
    }
    if (!pr.resolve_in_refine) {
        const int rg = eager ? std::max(1, std::min(pr.hdr->n_wg, kResolveGrid)) : kResolveGrid;
        hipLaunchKernelGGL(resolve_adds_kernel, dim3(rg), dim3(kResolveBlock), 0, s, dh);
    }
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int launch_refine(fl_ctx* c, const BatchHdr* dh, int n_iters, int variant, hipStream_t s, bool eager) {
    if (n_iters <= 0) return FL_OK;
    const bool timed = eager && c->prof;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (timed) {
        int rc = prof_event(c, &t0);
        if (!rc) rc = prof_event(c, &t1);
        if (rc) return rc;
        FL_HIP(hipEventRecord(t0, s));
    }
    // variant: bit 0 Levenberg-Marquardt, bit 1 more than one round
    if (variant == 0) hipLaunchKernelGGL((refine_kernel<false, false>), dim3(kRefineGrid), dim3(kRefBlock), 0, s, dh);
    else if (variant == 1) hipLaunchKernelGGL((refine_kernel<true, false>), dim3(kRefineGrid), dim3(kRefBlock), 0, s, dh);
    else if (variant == 2) hipLaunchKernelGGL((refine_kernel<false, true>), dim3(kRefineGrid), dim3(kRefBlock), 0, s, dh);
    else hipLaunchKernelGGL((refine_kernel<true, true>), dim3(kRefineGrid), dim3(kRefBlock), 0, s, dh);
    if (timed) {
        FL_HIP(hipEventRecord(t1, s));
        c->prof_ev[FL_PROF_REFINE].emplace_back(t0, t1);
    }
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int check_refine(const fl_batch* B, const fl_refine* R) {
    if (!R || R->n_iters == 0) return FL_OK;
    if (R->n_iters < 0 || R->n_iters > 1000) return fail(FL_ERANGE, "refine.n_iters %d outside [0, 1000]", R->n_iters);
    if (!finite_pos(R->huber_delta)) return fail(FL_EINVAL, "refine.huber_delta must be finite and > 0");
    if (R->flags != 0) return fail(FL_EINVAL, "refine.flags must be 0");
    if (R->n_rounds < 0 || (int64_t)R->n_iters * std::max(R->n_rounds, 1) > 1000)
        return fail(FL_ERANGE, "refine.n_iters * n_rounds must be at most 1000");
    if (R->n_rounds > 1 && !(R->outlier_px > 0.0f)) return fail(FL_EINVAL, "refine.outlier_px must be > 0");
    if (!(R->lm_lambda >= 0.0f) || !std::isfinite(R->lm_lambda))
        return fail(FL_EINVAL, "refine.lm_lambda must be finite and >= 0");
    if (B->n_events > 0 && !R->event_S) return fail(FL_EINVAL, "refine.event_S must not be NULL");
    if (const fl_refine_inverse* V = R->inverse) {
        if (R->n_rounds > 1 || R->lm_lambda > 0.0f)
            return fail(FL_ENOTSUP, "refine.inverse: two-sided refinement is Gauss-Newton only "
                                    "(n_rounds <= 1, lm_lambda = 0)");
        if (V->flags != 0) return fail(FL_EINVAL, "refine.inverse.flags must be 0");
        if (!V->event_offset) return fail(FL_EINVAL, "refine.inverse.event_offset must not be NULL");
        if (V->event_offset[0] != 0) return fail(FL_EINVAL, "refine.inverse.event_offset[0] must be 0");
        for (int e = 0; e < B->n_events; ++e)
            if (V->event_offset[e + 1] < V->event_offset[e])
                return fail(FL_EINVAL, "refine.inverse.event_offset must be non-decreasing (event %d)", e);
        const int64_t n = V->event_offset[B->n_events];
        if (n > INT32_MAX) return fail(FL_ERANGE, "refine.inverse: %lld pairs, at most 2^31-1", (long long)n);
        if (n > 0) {
            if (!V->xyz || !V->uv || !V->kf_idx || !V->kf_T || !V->kf_cam)
                return fail(FL_EINVAL, "refine.inverse: xyz, uv, kf_idx, kf_T and kf_cam must not be NULL");
            if (V->n_kf <= 0) return fail(FL_EINVAL, "refine.inverse.n_kf must be > 0");
            if ((uintptr_t)V->xyz % 16 || (uintptr_t)V->uv % 8 || (uintptr_t)V->kf_idx % 4 ||
                (uintptr_t)V->kf_T % 4 || (uintptr_t)V->kf_cam % 16)
                return fail(FL_EINVAL, "refine.inverse: misaligned array (xyz 16, uv 8, kf_cam 16, others 4 bytes)");
        }
    }
    return FL_OK;
}

// Every instantiation of the fused kernel may use up to lds_max bytes of LDS.
template <int PPL, int MODE, bool STATS>
void allow_lds(size_t bytes) {
    (void)hipFuncSetAttribute((const void*)search_fused_kernel<PPL, MODE, STATS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int PPL>
void allow_lds_all(size_t bytes) {
    allow_lds<PPL, kModeLdsDesc, false>(bytes);
    allow_lds<PPL, kModeLdsDesc, true>(bytes);
    allow_lds<PPL, kModeLdsRec, false>(bytes);
    allow_lds<PPL, kModeLdsRec, true>(bytes);
}

}  // namespace

// ===========================================================================
// C ABI

static void clear_profile(fl_ctx* c);
namespace {
int scratch_of_current_device(void** out);
}

extern "C" {

const char* fl_last_error(void) { return g_err; }

int fl_version(void) { return 10100; }

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
    {
        void* sp = nullptr;   // the allocation-free search's scratch on this device, resolved at set-up
        const int rs = scratch_of_current_device(&sp);
        if (rs) return rs;
    }
    fl_ctx* c = new fl_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->lds_max = std::max<size_t>(prop.sharedMemPerBlock, 65536) - kSearchStaticLds;   // room for static LDS
    allow_lds_all<1>(c->lds_max);
    allow_lds_all<2>(c->lds_max);
    allow_lds_all<4>(c->lds_max);
    // the band solve's window at the widest band (above 64 KB)
    (void)hipFuncSetAttribute((const void*)pgo_band_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)band_solve_lds_bytes(kBandMaxW));
    for (auto& f : c->fence) {
        if (hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) != hipSuccess) {
            fl_destroy(c);
            return fail(FL_EHIP, "hipEventCreate failed");
        }
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        fl_destroy(c);
        return fail(FL_EHIP, "hipStreamCreate failed");
    }
    // residual partials: 1024 blocks x kNAcc doubles + a done counter
    if (c->res.ensure(sizeof(double) * 1024 * kNAcc + 256, 0x00) != FL_OK) {
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
    for (auto& g : c->gexec)
        if (g) hipGraphExecDestroy(g);
    clear_profile(c);
    for (auto e : c->ev_pool) hipEventDestroy(e);
    for (auto& p : c->pin)
        if (p.p) hipHostFree(p.p);
    for (auto& f : c->fence)
        if (f.ev) hipEventDestroy(f.ev);
    for (auto& p : c->gpin)
        if (p.p) hipHostFree(p.p);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    c->ws.release();
    c->claims.release();
    c->ctrs.release();
    c->diag.release();
    c->plain.release();
    c->res.release();
    c->part.release();
    c->pgo.release();
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


}  // extern "C"

namespace {

// Checks of a plain search call (before any launch).
int check_plain(int32_t n_mp, const float* mp_xyz, const uint8_t* mp_desc, const fl_keyframe* kf, const fl_sim3* S,
                const fl_pinhole* K, const fl_params* P, const fl_fuse_out* out) {
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
    return FL_OK;
}

// Scratch layout of a plain search: the keyframe's grid (when the caller
// gives none), owner hash set, ADD claims, the ADD counter and the ADD list.
struct PlainLayout {
    int hsize = 0;
    int64_t cap = 0;
    size_t o_cs = 0, o_ck = 0, o_hash = 0, o_claim = 0, o_ctr = 0, o_list = 0, bytes = 0;
};

PlainLayout plain_layout(int32_t n_mp, int n_kp, int cells, int cap_override) {
    PlainLayout L;
    L.hsize = next_pow2(2 * n_kp);
    L.cap = std::min<int64_t>(n_mp, std::max<int64_t>(2 * (int64_t)n_kp, 4096));
    if (cap_override > 0) L.cap = std::min<int64_t>(L.cap, cap_override);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.o_cs = take(sizeof(int32_t) * (cells + 1));
    L.o_ck = take(sizeof(int32_t) * (size_t)std::max(n_kp, 1));
    L.o_hash = take(sizeof(int32_t) * (size_t)L.hsize);
    L.o_claim = take(sizeof(int32_t) * (size_t)std::max(n_kp, 1));
    L.o_ctr = take(sizeof(uint32_t) * 4);
    L.o_list = take(sizeof(AddRef) * (size_t)L.cap);
    L.bytes = off;
    return L;
}

// The plain search's launches with its scratch at `base` (laid out as L).
// Every scratch word the kernels read is written first in the same call:
// plain_prep_kernel resets the hash set, the claims and the counter, and
// the grid is built when the caller gives none.
int plain_launch(char* base, const PlainLayout& L, int32_t n_mp, const float* mp_xyz, const uint8_t* mp_desc,
                 const float* mp_dmax, const int32_t* mp_id, const fl_keyframe* kf, const fl_sim3* S,
                 const fl_pinhole* K, const fl_params* P, const fl_fuse_out* out, hipStream_t stream) {
    const int cells = P->grid_cols * P->grid_rows;
    const int n_kp = kf->n_kp;
    PlainArgs a{};
    fill_kf_geometry(a.kd, *S, *K, P);
    a.kd.n_kp = n_kp;
    a.kd.hash_mask = L.hsize - 1;
    float sf[32];
    fill_search_const(P, a.sc, sf);
    a.sc.gate = mp_dmax != nullptr;
    a.n_mp = n_mp;
    a.add_cap = (int32_t)L.cap;
    a.mp_xyz = mp_xyz;
    a.mp_desc = mp_desc;
    a.mp_dmax = mp_dmax;
    a.mp_id = mp_id;
    a.kp_xy = kf->kp_xy;
    a.kp_oct = kf->kp_octave;
    a.kp_desc = kf->kp_desc;
    a.kp_owner = kf->kp_owner;
    a.hash = (const int32_t*)(base + L.o_hash);
    a.claim = (int32_t*)(base + L.o_claim);
    a.counter = (uint32_t*)(base + L.o_ctr);
    a.add_list = (AddRef*)(base + L.o_list);
    a.best_idx = out->best_idx;
    a.best_dist = out->best_dist;
    a.second_dist = out->second_dist;
    a.decision = out->decision;
    a.target = out->target;
    if (kf->cell_start) {
        a.cell_start = kf->cell_start;
        a.cell_kp = kf->cell_kp;
    } else {
        int32_t* cs = (int32_t*)(base + L.o_cs);
        int32_t* ck = (int32_t*)(base + L.o_ck);
        hipLaunchKernelGGL(grid_single_kernel, dim3(1), dim3(kPrepBlock), 0, stream, a.kd, cells, P->grid_cols,
                           P->grid_rows, kf->kp_xy, cs, ck);
        a.cell_start = cs;
        a.cell_kp = ck;
    }
    hipLaunchKernelGGL(plain_prep_kernel, dim3(1), dim3(kPrepBlock), 0, stream, n_kp, kf->kp_owner,
                       (int32_t*)(base + L.o_hash), L.hsize - 1, a.claim, a.counter);
    const int grid = (n_mp + 255) / 256;
    hipLaunchKernelGGL(search_plain_kernel, dim3(grid), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(resolve_plain_kernel, dim3(std::min(grid, 256)), dim3(256), 0, stream, n_mp,
                       (const uint32_t*)a.counter, (const AddRef*)a.add_list, (int32_t)L.cap,
                       (const int32_t*)a.claim, mp_id, (const int32_t*)out->best_idx, out->decision, out->target);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free plain search: one static device array per
// GPU (each device holds its own copy at its own address, found once per
// device with hipGetSymbolAddress).  The array's name in host code is not a
// device address; only the resolved pointer is passed to kernels.
constexpr size_t kNoAllocScratch = 1u << 20;   // bytes per GPU
__device__ __align__(256) unsigned char scratch[kNoAllocScratch];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array (resolved on the
// first request for that device).
int scratch_of_current_device(void** out) {
    int dev = 0;
    FL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FL_ENOTSUP, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FL_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FL_OK;
}

}  // namespace

extern "C" {

int fl_search_fuse(fl_ctx* c, int32_t n_mp, const float* mp_xyz, const uint8_t* mp_desc, const float* mp_dmax,
                   const int32_t* mp_id, const fl_keyframe* kf, const fl_sim3* S, const fl_pinhole* K,
                   const fl_params* P, const fl_fuse_out* out, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_plain(n_mp, mp_xyz, mp_desc, kf, S, K, P, out);
    if (rc) return rc;
    if (n_mp == 0) return FL_OK;
    const PlainLayout L = plain_layout(n_mp, kf->n_kp, P->grid_cols * P->grid_rows, c->add_cap_override);
    rc = c->plain.ensure(L.bytes);
    if (rc) return rc;
    return plain_launch((char*)c->plain.p, L, n_mp, mp_xyz, mp_desc, mp_dmax, mp_id, kf, S, K, P, out, stream);
}

int fl_search_fuse_noalloc(int32_t n_mp, const float* mp_xyz, const uint8_t* mp_desc, const float* mp_dmax,
                           const int32_t* mp_id, const fl_keyframe* kf, const fl_sim3* S, const fl_pinhole* K,
                           const fl_params* P, const fl_fuse_out* out, hipStream_t stream) {
    int rc = check_plain(n_mp, mp_xyz, mp_desc, kf, S, K, P, out);
    if (rc) return rc;
    const PlainLayout L = plain_layout(n_mp, kf->n_kp, P->grid_cols * P->grid_rows, 0);
    if (L.bytes > kNoAllocScratch)
        return fail(FL_ERANGE, "n_kp %d with %d grid cells needs %zu bytes of scratch; the allocation-free search "
                    "holds %zu (use fl_search_fuse)", kf->n_kp, P->grid_cols * P->grid_rows, L.bytes,
                    kNoAllocScratch);
    void* base = nullptr;
    rc = scratch_of_current_device(&base);
    if (rc) return rc;
    if (n_mp == 0) return FL_OK;
    return plain_launch((char*)base, L, n_mp, mp_xyz, mp_desc, mp_dmax, mp_id, kf, S, K, P, out, stream);
}


int fl_validate_batch(const fl_batch* B, const fl_params* P, const fl_fuse_out* out) {
    return validate_batch(B, P, out);
}

int fl_search_fuse_batched(fl_ctx* c, const fl_batch* B, const fl_params* P, const fl_fuse_out* out,
                           const fl_refine* R, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = validate_batch(B, P, out);
    if (rc) return rc;
    rc = check_refine(B, R);
    if (rc) return rc;
    if (B->n_pairs == 0) return FL_OK;
    Prepared pr;
    rc = prepare_batch(c, B, P, out, R, false, pr);
    if (rc) return rc;
    rc = upload_batch(c, pr, stream);
    if (rc) return rc;
    if (c->stats) FL_HIP(hipMemsetAsync(c->ctrs.p, 0, 32, stream));
    const BatchHdr* dh = (const BatchHdr*)c->ws.p;
    rc = launch_search(c, pr, dh, stream, true, c->stats != 0);
    if (rc) return rc;
    return launch_refine(c, dh, pr.refine_iters, pr.refine_variant, stream, true);
}

int fl_search_fuse_passes(fl_ctx* c, const fl_batch* B, int32_t n_pass, const fl_pass* passes, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!passes) return fail(FL_EINVAL, "passes is NULL");
    if (n_pass < 1 || n_pass > FL_MAX_PASSES) return fail(FL_EINVAL, "n_pass %d outside [1, %d]", n_pass, FL_MAX_PASSES);
    const fl_params* P = &passes[0].params;
    for (int p = 0; p < n_pass; ++p) {
        const int rc = validate_batch(B, &passes[p].params, &passes[p].out);
        if (rc) return rc;
        const fl_params& Q = passes[p].params;
        if (Q.scale_factor != P->scale_factor || Q.n_octaves != P->n_octaves || Q.grid_cols != P->grid_cols ||
            Q.grid_rows != P->grid_rows)
            return fail(FL_EINVAL, "pass %d: scale_factor, n_octaves and the grid must equal those of pass 0", p);
        for (int q = 0; q < p && B->n_pairs > 0; ++q) {
            const fl_fuse_out &a = passes[p].out, &b = passes[q].out;
            if (a.best_idx == b.best_idx || a.best_dist == b.best_dist || a.second_dist == b.second_dist ||
                a.decision == b.decision || a.target == b.target)
                return fail(FL_EINVAL, "passes %d and %d share an output array", q, p);
        }
    }
    if (B->n_pairs == 0) return FL_OK;
    Prepared pr;
    int rc = prepare_batch(c, B, P, &passes[0].out, nullptr, false, pr, false, n_pass, passes);
    if (rc) return rc;
    rc = upload_batch(c, pr, stream);
    if (rc) return rc;
    if (c->stats) FL_HIP(hipMemsetAsync(c->ctrs.p, 0, 32, stream));
    return launch_search(c, pr, (const BatchHdr*)c->ws.p, stream, true, c->stats != 0);
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
    rc = prepare_batch(c, B, &P, out, R, true, pr);
    if (rc) return rc;
    rc = upload_batch(c, pr, stream);
    if (rc) return rc;
    return launch_refine(c, (const BatchHdr*)c->ws.p, R->n_iters, pr.refine_variant, stream, true);
}

int fl_search_fuse_graph_launch(fl_ctx* c, const fl_batch* B, const fl_params* P, const fl_fuse_out* out,
                                const fl_refine* R, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = validate_batch(B, P, out);
    if (rc) return rc;
    rc = check_refine(B, R);
    if (rc) return rc;
    if (B->n_pairs == 0) return FL_OK;
    Prepared pr;
    rc = prepare_batch(c, B, P, out, R, false, pr, true);
    if (rc) return rc;
    pr.hdr->stats = 0;   // counters are an eager-path feature
    const int refine_on = pr.refine_iters > 0 ? 1 + pr.refine_variant : 0;   // the captured kernel
    const bool stale = !c->gexec[0] || c->g_ws != c->ws.p || c->g_claims != c->claims.p || c->g_ctrs != c->ctrs.p ||
                       c->g_mode != pr.mode || c->g_ppl != pr.ppl || c->g_grid != pr.grid ||
                       c->g_refine != refine_on || c->g_lds != pr.lds || c->gpin[0].size != pr.blob_cap;
    if (stale) {
        FL_HIP(hipStreamSynchronize(stream));
        for (int gi = 0; gi < kGraphRing; ++gi) {
            Pinned& gp = c->gpin[gi];
            const int wrc = wait_fetched(c, gp);   // a replay may still fetch from it
            if (wrc) return wrc;
            if (c->gexec[gi]) hipGraphExecDestroy(c->gexec[gi]);
            c->gexec[gi] = nullptr;
            gp.used = 0;
            if (gp.size != pr.blob_cap) {
                if (gp.p) hipHostFree(gp.p);
                gp.p = nullptr;
                gp.size = 0;
                const size_t n = pr.blob_cap;
                if (hipHostMalloc(&gp.p, n, hipHostMallocDefault) != hipSuccess) {
                    gp.p = nullptr;
                    return fail(FL_ENOMEM, "hipHostMalloc of %zu bytes failed", n);
                }
                gp.size = n;
            }
        }
        const BatchHdr* dh = (const BatchHdr*)c->ws.p;
        for (int gi = 0; gi < kGraphRing; ++gi) {
            hipGraph_t graph = nullptr;
            FL_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            const int saved_prof = c->prof;
            c->prof = 0;
            launch_fetch(c, c->gpin[gi].p, c->gpin[gi].size, c->cap_stream);
            int lrc = launch_search(c, pr, dh, c->cap_stream, false, false);
            c->prof = saved_prof;
            if (lrc == FL_OK && refine_on)
                lrc = launch_refine(c, dh, pr.refine_iters, pr.refine_variant, c->cap_stream, false);
            hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
            if (lrc) {
                if (graph) hipGraphDestroy(graph);
                return lrc;
            }
            if (ce != hipSuccess) return fail(FL_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
            hipError_t ie = hipGraphInstantiate(&c->gexec[gi], graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                c->gexec[gi] = nullptr;
                return fail(FL_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
            }
            // resources of the executable set up now, not on its first replay
            FL_HIP(hipGraphUpload(c->gexec[gi], c->cap_stream));
        }
        FL_HIP(hipStreamSynchronize(c->cap_stream));
        c->g_ws = c->ws.p;
        c->g_claims = c->claims.p;
        c->g_ctrs = c->ctrs.p;
        c->g_mode = pr.mode;
        c->g_ppl = pr.ppl;
        c->g_grid = pr.grid;
        c->g_refine = refine_on;
        c->g_lds = pr.lds;
    }
    // The graph fetches its tables from its own pinned buffer.  Unchanged
    // tables are left in place; otherwise wait until the previous replay of
    // this graph (kGraphRing replays ago) has fetched them before overwriting.
    Pinned& gp = c->gpin[c->g_next];
    if (!(gp.used == pr.blob.size() && memcmp(gp.p, pr.blob.data(), pr.blob.size()) == 0)) {
        rc = wait_fetched(c, gp);
        if (rc) return rc;
        memcpy(gp.p, pr.blob.data(), pr.blob.size());
        gp.used = pr.blob.size();
    }
    rc = next_epoch(c, stream);
    if (rc) return rc;
    FL_HIP(hipGraphLaunch(c->gexec[c->g_next], stream));
    c->g_next = (c->g_next + 1) % kGraphRing;
    return note_fetch(c, gp, stream);
}


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
    hipLaunchKernelGGL(residual_bwd_kernel<false>, dim3(grid), dim3(kResBlock), 0, stream, a);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_reproj_residual_bwd_inv(fl_ctx* c, int32_t n, const float* xyz, const float* uv, const int32_t* kf_idx,
                               int32_t n_kf, const float* kf_T, const fl_sim3* S_inv, const fl_pinhole* K,
                               float huber_delta, double grad_scale, double* g, double* H, hipStream_t stream) {
    ResArgs a;
    int grid = 1;
    int rc = residual_args(c, n, xyz, uv, kf_idx, n_kf, kf_T, S_inv, K, huber_delta, a, grid);
    if (rc) return rc;
    if (!g) return fail(FL_EINVAL, "g must not be NULL");
    if (!std::isfinite(grad_scale)) return fail(FL_EINVAL, "grad_scale must be finite");
    a.g = g;
    a.H = H;
    a.grad_scale = grad_scale;
    hipLaunchKernelGGL(residual_bwd_kernel<true>, dim3(grid), dim3(kResBlock), 0, stream, a);
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_pose_graph_optimize(fl_ctx* c, const fl_pose_graph* G, const fl_pgo_params* P, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!G || !P) return fail(FL_EINVAL, "graph or params is NULL");
    const int N = G->n_nodes, E = G->n_edges;
    if (N < 1 || E < 0) return fail(FL_EINVAL, "n_nodes must be >= 1 and n_edges >= 0");
    if (N > (1 << 24) || E > (1 << 26)) return fail(FL_ERANGE, "graph too large (%d nodes, %d edges)", N, E);
    if (!G->S || (E > 0 && (!G->M || !G->edges))) return fail(FL_EINVAL, "NULL graph array");
    if (P->iters < 0 || P->iters > 1000) return fail(FL_ERANGE, "iters %d outside [0, 1000]", P->iters);
    if (P->cg_iters < 1 || P->cg_iters > 100000) return fail(FL_ERANGE, "cg_iters %d outside [1, 100000]", P->cg_iters);
    if (!(P->lambda >= 0.0) || !std::isfinite(P->lambda)) return fail(FL_EINVAL, "lambda must be finite and >= 0");
    if (!(P->cg_tol >= 0.0) || !std::isfinite(P->cg_tol)) return fail(FL_EINVAL, "cg_tol must be finite and >= 0");
    if (P->solver < FL_PGO_SOLVER_AUTO || P->solver > FL_PGO_SOLVER_DIRECT_WIDE || P->reserved != 0)
        return fail(FL_EINVAL, "solver %d / reserved %d", P->solver, P->reserved);
    // incident edges of every node, in edge order (the gathers' fixed order),
    // then the band position of every node and the node of every position
    std::vector<int32_t> tab((size_t)2 * E + (N + 1) + 2 * (size_t)E + 2 * (size_t)N, 0);
    int32_t* t_edges = tab.data();
    int32_t* off = t_edges + 2 * (size_t)E;
    int32_t* adj = off + (N + 1);
    int32_t* posn = adj + 2 * (size_t)E;
    int32_t* order = posn + N;
    for (int k = 0; k < E; ++k) {
        const int i = G->edges[2 * k], j = G->edges[2 * k + 1];
        if (i < 0 || i >= N || j < 0 || j >= N || i == j)
            return fail(FL_EINVAL, "edge %d joins %d and %d (n_nodes %d)", k, i, j, N);
        t_edges[2 * k] = i;
        t_edges[2 * k + 1] = j;
        ++off[i + 1];
        ++off[j + 1];
    }
    for (int n = 0; n < N; ++n) off[n + 1] += off[n];
    {
        std::vector<int32_t> fill(off, off + N);
        for (int k = 0; k < E; ++k) {
            adj[fill[t_edges[2 * k]]++] = 2 * k;
            adj[fill[t_edges[2 * k + 1]]++] = 2 * k + 1;
        }
    }
    // Band ordering of the free nodes: reverse Cuthill-McKee (breadth-first
    // from a node of least degree in each component, neighbours by rising
    // degree, the whole order reversed); b = the widest span of an edge
    // between free nodes.
    std::vector<uint8_t> held(N);
    for (int n = 0; n < N; ++n) held[n] = G->fixed ? (G->fixed[n] != 0) : (n == 0);
    int nf = 0, bw = 0;
    {
        std::vector<int32_t> deg(N, 0), seq, nb;
        for (int k = 0; k < E; ++k)
            if (!held[t_edges[2 * k]] && !held[t_edges[2 * k + 1]]) {
                ++deg[t_edges[2 * k]];
                ++deg[t_edges[2 * k + 1]];
            }
        std::vector<int32_t> roots;
        for (int n = 0; n < N; ++n)
            if (!held[n]) roots.push_back(n);
        std::stable_sort(roots.begin(), roots.end(), [&](int x, int y) { return deg[x] < deg[y]; });
        std::vector<uint8_t> seen(N, 0);
        seq.reserve(roots.size());
        for (int root : roots) {
            if (seen[root]) continue;
            seen[root] = 1;
            size_t head = seq.size();
            seq.push_back(root);
            while (head < seq.size()) {
                const int v = seq[head++];
                nb.clear();
                for (int t = off[v]; t < off[v + 1]; ++t) {
                    const int k = adj[t] >> 1, u = t_edges[2 * k + 1 - (adj[t] & 1)];
                    if (!held[u] && !seen[u]) {
                        seen[u] = 1;
                        nb.push_back(u);
                    }
                }
                std::stable_sort(nb.begin(), nb.end(), [&](int x, int y) {
                    return deg[x] != deg[y] ? deg[x] < deg[y] : x < y;
                });
                seq.insert(seq.end(), nb.begin(), nb.end());
            }
        }
        nf = (int)seq.size();
        for (int n = 0; n < N; ++n) posn[n] = -1;
        for (int p = 0; p < nf; ++p) {
            order[p] = seq[nf - 1 - p];
            posn[order[p]] = p;
        }
        for (int k = 0; k < E; ++k) {
            const int pi = posn[t_edges[2 * k]], pj = posn[t_edges[2 * k + 1]];
            if (pi >= 0 && pj >= 0) bw = std::max(bw, std::abs(pi - pj));
        }
    }
    const bool band_fits = bw + 1 <= FL_PGO_MAX_BAND_NODES;
    if ((P->solver == FL_PGO_SOLVER_DIRECT || P->solver == FL_PGO_SOLVER_DIRECT_WIDE) && !band_fits && E > 0 &&
        nf > 0)
        return fail(FL_ERANGE, "reordered band spans %d keyframes (at most %d)", bw + 1, FL_PGO_MAX_BAND_NODES);
    const bool direct = E > 0 && nf > 0 && band_fits && P->solver != FL_PGO_SOLVER_CG;
    // the LDS window up to kBandLdsNodes keyframes, the device-memory one above
    const bool wide = direct && (bw + 1 > kBandLdsNodes || P->solver == FL_PGO_SOLVER_DIRECT_WIDE);
    const int band_w = 7 * (bw + 1);
    const int64_t band_vs = 7 * (int64_t)nf;
    const size_t tab_bytes = sizeof(int32_t) * tab.size();
    size_t off_b = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off_b;
        off_b = align_up(off_b + std::max<size_t>(bytes, 16), 256);
        return o;
    };
    const size_t L_tab = take(tab_bytes);
    const size_t L_fix = take((size_t)N);
    const size_t L_e = take(sizeof(double) * 7 * (size_t)E);
    const size_t L_J = take(sizeof(double) * 98 * (size_t)E);
    const size_t L_u = take(sizeof(double) * 7 * (size_t)E);
    const size_t L_vec = take(sizeof(double) * 6 * 7 * (size_t)N);
    const size_t L_D = take(sizeof(double) * 49 * (size_t)N);
    // co-resident solve workgroups: enough threads for every edge and node,
    // at most one per CU (each grid barrier costs every workgroup a fence)
    const int solve_grid = (int)std::max<int64_t>(
        1, std::min<int64_t>(c->n_cu, (std::max(E, N) + (int64_t)kPgoBlock - 1) / kPgoBlock));
    const size_t L_bar = take(sizeof(uint32_t));
    const size_t L_red = take(sizeof(double) * 2 * 4 * (size_t)solve_grid);
    const size_t L_band = take(direct ? sizeof(double) * (size_t)band_vs * band_w : 0);
    const size_t L_rhs = take(direct ? sizeof(double) * (size_t)band_vs : 0);
    const size_t L_xs = take(direct ? sizeof(double) * (size_t)band_vs : 0);
    const size_t L_lm = take(sizeof(double) * kLmWords);
    const size_t L_Sc = take(sizeof(double) * 13 * (size_t)N);
    const size_t L_ec = take(sizeof(double) * (size_t)E);
    int rc = c->pgo.ensure(off_b);
    if (rc) return rc;
    char* base = (char*)c->pgo.p;
    // tables and fixed flags through the pinned ring (node 0 held when no flags are given)
    const size_t up = L_fix + (size_t)N;
    Pinned* pin = nullptr;
    rc = get_pinned(c, up, &pin);
    if (rc) return rc;
    memcpy(pin->p, tab.data(), tab_bytes);
    uint8_t* fx = (uint8_t*)pin->p + L_fix;
    for (int n = 0; n < N; ++n) fx[n] = held[n];
    pin->used = up;
    FL_HIP(hipMemcpyAsync(base, pin->p, up, hipMemcpyHostToDevice, stream));
    rc = note_fetch(c, *pin, stream);
    if (rc) return rc;
    PgoArgs a{};
    a.n_nodes = N;
    a.n_edges = E;
    a.S = G->S;
    a.M = G->M;
    a.edges = (const int32_t*)(base + L_tab);
    a.adj_off = a.edges + 2 * (size_t)E;
    a.adj = a.adj_off + (N + 1);
    a.fixed = (const uint8_t*)(base + L_fix);
    a.cg_iters = P->cg_iters;
    a.cg_tol = P->cg_tol;
    a.e = (double*)(base + L_e);
    a.J = (double*)(base + L_J);
    a.u = (double*)(base + L_u);
    a.vec = (double*)(base + L_vec);
    a.Dfac = (double*)(base + L_D);
    a.bar = (uint32_t*)(base + L_bar);
    a.red = (double*)(base + L_red);
    a.band_w = band_w;
    a.band_vs = (int32_t)band_vs;
    a.pos = a.adj + 2 * (size_t)E;
    a.order = a.pos + N;
    a.band = (double*)(base + L_band);
    a.rhs = (double*)(base + L_rhs);
    a.xs = (double*)(base + L_xs);
    a.lm = (double*)(base + L_lm);
    a.S_c = (double*)(base + L_Sc);
    a.ecost = (double*)(base + L_ec);
    a.cost = P->cost;
    a.cg_used = P->cg_used;
    a.lambdas = P->lambdas;
    a.accepted = P->accepted;
    // Every iteration enqueues the same kernels: the damping, the decision
    // and whether to relinearise are read from the device state.
    const int edge_grid = std::max(1, (E + kPgoBlock - 1) / kPgoBlock);
    const int jac_grid = std::max(1, (E + kPgoJacBlock - 1) / kPgoJacBlock);
    const int node_grid = std::max(1, (int)((13 * (int64_t)N + kPgoBlock - 1) / kPgoBlock));
    hipLaunchKernelGGL(pgo_edge_cost_kernel, dim3(edge_grid), dim3(kPgoBlock), 0, stream, a, (const double*)a.S);
    hipLaunchKernelGGL(pgo_init_kernel, dim3(1), dim3(kPgoBlock), 0, stream, a, P->lambda);
    for (int it = 0; it < P->iters; ++it) {
        a.step = it;
        if (E > 0) hipLaunchKernelGGL(pgo_jacobian_kernel, dim3(jac_grid), dim3(kPgoJacBlock), 0, stream, a);
        if (direct) {
            hipLaunchKernelGGL(pgo_band_assemble_kernel, dim3((unsigned)((band_vs + kBandBlock - 1) / kBandBlock)),
                               dim3(kBandBlock), 0, stream, a);
            if (wide)
                hipLaunchKernelGGL(pgo_band_solve_wide_kernel, dim3(1), dim3(kWideBlock), 0, stream, a);
            else
                hipLaunchKernelGGL(pgo_band_solve_kernel, dim3(1), dim3(kBandBlock),
                                   band_solve_lds_bytes(band_w), stream, a);
        } else {
            fill_u32(a.bar, sizeof(uint32_t), 0u, stream);
            hipLaunchKernelGGL(pgo_solve_kernel, dim3(solve_grid), dim3(kPgoBlock), 0, stream, a);
        }
        hipLaunchKernelGGL(pgo_edge_cost_kernel, dim3(edge_grid), dim3(kPgoBlock), 0, stream, a, (const double*)a.S_c);
        hipLaunchKernelGGL(pgo_decide_kernel, dim3(1), dim3(kPgoBlock), 0, stream, a);
        hipLaunchKernelGGL(pgo_accept_kernel, dim3(node_grid), dim3(kPgoBlock), 0, stream, a);
    }
    FL_HIP(hipGetLastError());
    return FL_OK;
}

int fl_sim3_inverse(fl_ctx* c, const double* S_in, double* S_out, fl_sim3* S32_out, hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!S_in || (!S_out && !S32_out)) return fail(FL_EINVAL, "NULL argument");
    hipLaunchKernelGGL(sim3_inverse_kernel, dim3(1), dim3(64), 0, stream, S_in, S_out, S32_out);
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

int fl_sim3_grad_xi(fl_ctx* c, const double* xi, const double* g, const double* scale, double* out,
                    hipStream_t stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!xi || !g || !out) return fail(FL_EINVAL, "NULL argument");
    hipLaunchKernelGGL(sim3_grad_xi_kernel, dim3(1), dim3(64), 0, stream, xi, g, scale, out);
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
// tuning, statistics, profiling

int fl_get_tuning(fl_ctx* c, fl_tuning* out) {
    if (!c || !out) return fail(FL_EINVAL, "NULL argument");
    *out = c->tune;
    return FL_OK;
}

int fl_set_tuning(fl_ctx* c, const fl_tuning* t) {
    if (!c || !t) return fail(FL_EINVAL, "NULL argument");
    if (t->pairs_per_lane != 1 && t->pairs_per_lane != 2 && t->pairs_per_lane != 4)
        return fail(FL_EINVAL, "pairs_per_lane must be 1, 2 or 4");
    if (t->lds_mode < kModeGlobal || t->lds_mode > kModeLdsDesc) return fail(FL_EINVAL, "lds_mode must be 0, 1 or 2");
    if (t->wg_per_cu != 1 && t->wg_per_cu != 2) return fail(FL_EINVAL, "wg_per_cu must be 1 or 2");
    if (t->xcd_aware != 0 && t->xcd_aware != 1) return fail(FL_EINVAL, "xcd_aware must be 0 or 1");
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
    const int saved_stats = c->stats, saved_prof = c->prof;
    c->stats = 0;
    c->prof = 0;
    fl_tuning top = saved;
    float top_ms = 1e30f;
    const int ppls[] = {1, 2, 4};
    const int modes[] = {kModeLdsDesc, kModeLdsRec, kModeGlobal};
    for (int ppl : ppls)
        for (int mode : modes)
            for (int wpc = 1; wpc <= 2; ++wpc)
                for (int xa = 0; xa <= 1 && rc == FL_OK; ++xa) {
                    c->tune = fl_tuning{ppl, mode, wpc, xa};
                    rc = fl_search_fuse_batched(c, B, P, out, nullptr, stream);   // warm-up
                    if (rc) break;
                    (void)hipEventRecord(e0, stream);
                    for (int r = 0; r < reps && rc == FL_OK; ++r) rc = fl_search_fuse_batched(c, B, P, out, nullptr, stream);
                    (void)hipEventRecord(e1, stream);
                    if (rc) break;
                    if (hipEventSynchronize(e1) != hipSuccess) {
                        rc = fail(FL_EHIP, "hipEventSynchronize failed");
                        break;
                    }
                    float ms = 0.0f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms /= (float)reps;
                    if (ms < top_ms) {
                        top_ms = ms;
                        top = c->tune;
                    }
                }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->stats = saved_stats;
    c->prof = saved_prof;
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
    if (!c->ctrs.p) return fail(FL_EINVAL, "no batched search has run on this context");
    unsigned long long v[4];
    FL_HIP(hipMemcpy(v, c->ctrs.p, sizeof(v), hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) out4[i] = (int64_t)v[i];
    return FL_OK;
}

}  // extern "C"

static void clear_profile(fl_ctx* c, int kernel) {
    for (auto& pr : c->prof_ev[kernel]) {
        c->ev_pool.push_back(pr.first);
        c->ev_pool.push_back(pr.second);
    }
    c->prof_ev[kernel].clear();
}

static void clear_profile(fl_ctx* c) {
    clear_profile(c, FL_PROF_SEARCH);
    clear_profile(c, FL_PROF_REFINE);
}

extern "C" {

int fl_set_profiling(fl_ctx* c, int enable) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    c->prof = enable ? 1 : 0;
    clear_profile(c);
    return FL_OK;
}

int fl_get_profile(fl_ctx* c, int kernel, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches) return fail(FL_EINVAL, "NULL argument");
    if (kernel != FL_PROF_SEARCH && kernel != FL_PROF_REFINE) return fail(FL_EINVAL, "unknown kernel class %d", kernel);
    auto& ev = c->prof_ev[kernel];
    double sum = 0.0;
    if (!ev.empty()) FL_HIP(hipEventSynchronize(ev.back().second));
    for (auto& pr : ev) {
        float ms = 0.0f;
        FL_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)ev.size();
    clear_profile(c, kernel);
    return FL_OK;
}

namespace fl {
// Issue rate of the search's Hamming instructions: eight independent chains
// of v_xor_b32 + v_bcnt_u32_b32 per lane, 16 lane-ops per iteration, on every
// CU at full occupancy.  The sink is written only if the chains end on one
// particular value, which keeps them live without memory traffic.
__global__ __launch_bounds__(256) void valu_rate_kernel(uint32_t* sink, int iters) {
    uint32_t a[8], b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = threadIdx.x * 0x9E3779B1u + (uint32_t)j;
        b[j] = blockIdx.x + 77u * (uint32_t)j;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a[j] ^= b[j];
            b[j] = (uint32_t)__popc(a[j]) + b[j];
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= a[j] + b[j];
    if (r == 0x9E3779B9u) sink[0] = r;
}
}  // namespace fl

int fl_valu_rate(fl_ctx* c, int32_t iters, double* lane_ops_per_s, hipStream_t stream) {
    if (!c || !lane_ops_per_s) return fail(FL_EINVAL, "NULL argument");
    if (iters < 1 || iters > (1 << 20)) return fail(FL_ERANGE, "iters %d outside [1, 2^20]", iters);
    const int rc = c->diag.ensure(4096, 0x00);
    if (rc) return rc;
    const int grid = c->n_cu * 8, block = 256;
    hipEvent_t e0, e1;
    FL_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(FL_EHIP, "hipEventCreate failed");
    }
    hipError_t err = hipEventRecord(e0, stream);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(fl::valu_rate_kernel, dim3(grid), dim3(block), 0, stream,
                           reinterpret_cast<uint32_t*>(c->diag.p), iters);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(FL_EHIP, "valu rate: %s", hipGetErrorString(err));
    if (!(ms > 0.0f)) return fail(FL_EHIP, "valu rate: no elapsed time");
    *lane_ops_per_s = (double)grid * block * (double)iters * 16.0 / ((double)ms * 1e-3);
    return FL_OK;
}

uint32_t fl_debug_refine_tag(uint32_t epoch, int32_t step) { return refine_tag(epoch, step); }

int fl_debug_refine_rows_cleared(uint32_t launches) { return refine_rows_cleared_before(launches) ? 1 : 0; }

int fl_debug_set_list_cap(fl_ctx* c, int32_t cap) {
    if (!c || cap < 0) return fail(FL_EINVAL, "bad argument");
    c->add_cap_override = cap;
    return FL_OK;
}

}  // extern "C"
