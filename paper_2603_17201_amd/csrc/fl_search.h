// Search-and-fuse kernels: the fused batched search, its global-grid
// fallback, the plain per-keyframe search and ADD-conflict resolution.
//
// Loop fusion (paper Sec. III-B, Sec. IV-D3): every map point of the loop
// region is projected through the corrected Sim3 into each connected
// keyframe; keypoints inside a window whose size follows the point's
// predicted octave are compared by 256-bit Hamming distance and the point is
// fused into an owned keypoint or added to a free one.  The work is
// independent per (point, keyframe) pair; the only coupling is several
// points claiming one free keypoint, resolved by the lowest point index.
#pragma once

#include "fl_internal.h"

namespace fl {

constexpr uint8_t kDecUndecided = 0xFF;
constexpr int kSearchBlock = 1024;   // threads of a batched-search workgroup (16 waves)
constexpr int kWavesPerWG = kSearchBlock / 64;

struct SearchConst {
    float sf[32];
    int N;
    int gate;
    int C, R;
    int th;
    float ratio;
    float r0;
};

__device__ __forceinline__ void load_desc(const uint8_t* __restrict__ base, int64_t row, uint4& a, uint4& b) {
    const uint4* p = reinterpret_cast<const uint4*>(base + row * 32);
    a = p[0];
    b = p[1];
}

__device__ __forceinline__ bool accept_match(const Best& b, int th, float ratio) {
    if (b.key == 0xFFFFFFFFu) return false;
    const int bh = (int)(b.key >> 16);
    if (bh > th) return false;
    if (ratio > 0.0f && ratio < 1.0f) return (float)bh < ratio * (float)b.second;
    return true;
}

// Window box and cell range of a visible point.
struct Window {
    float lx, hx, ly, hy;
    int c0, c1, r0, r1;
};

__device__ __forceinline__ Window make_window(const Proj& p, const KfDesc& kd, const float* sf, float r0w, int C,
                                              int R) {
    Window w;
    const float rad = r0w * sf[p.pred];
    w.lx = p.u - rad;
    w.hx = p.u + rad;
    w.ly = p.v - rad;
    w.hy = p.v + rad;
    w.c0 = cell_of(w.lx, kd.invw, C);
    w.c1 = cell_of(w.hx, kd.invw, C);
    w.r0 = cell_of(w.ly, kd.invh, R);
    w.r1 = cell_of(w.hy, kd.invh, R);
    return w;
}

__device__ __forceinline__ bool in_window(const Window& w, float x, float y, int oct, int pred, int gate) {
    if (!(x >= w.lx && x <= w.hx && y >= w.ly && y <= w.hy)) return false;
    if (gate && (oct < pred - 1 || oct > pred)) return false;
    return true;
}

__device__ __forceinline__ uint32_t owner_slot(int32_t id, int32_t mask) {
    return (hash_id(id) >> 7) & (uint32_t)mask;
}

// Insert an owner id into an open-addressing set with at least one free slot.
__device__ __forceinline__ void owner_insert(int32_t* tab, int32_t mask, int32_t o) {
    uint32_t hh = owner_slot(o, mask);
    for (int probe = 0; probe <= mask; ++probe) {
        const int32_t prev = atomicCAS(&tab[hh], -1, o);
        if (prev == -1 || prev == o) return;
        hh = (hh + 1) & (uint32_t)mask;
    }
}

// Workgroup exclusive scan of a[0..n) in place (n may exceed blockDim): each
// thread sums a run of consecutive elements, the runs are scanned inside each
// wave and the wave totals by wave 0.  s_tmp needs blockDim / 64 + 1 ints
// (s_tmp[blockDim / 64] = total); blockDim is a multiple of 64, at most 4096.
__device__ void block_exclusive_scan(int32_t* a, int n, int32_t* s_tmp) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = wave_lane(), wid = tid / kWave, nw = nt / kWave;
    const int chunk = (n + nt - 1) / nt;
    const int b = min(tid * chunk, n), e = min(b + chunk, n);
    constexpr int kRun = 4;   // runs up to this length are loaded at once
    int v[kRun];
    int sum = 0;
    if (chunk <= kRun) {
#pragma unroll
        for (int j = 0; j < kRun; ++j) v[j] = b + j < e ? a[b + j] : 0;
#pragma unroll
        for (int j = 0; j < kRun; ++j) sum += v[j];
    } else {
        for (int i = b; i < e; ++i) sum += a[i];
    }
    const int incl = wave_incl_scan(sum);
    if (lane == kWave - 1) s_tmp[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const int t = lane < nw ? s_tmp[lane] : 0;
        const int x = wave_incl_scan(t);
        if (lane < nw) s_tmp[lane] = x - t;
        if (lane == nw - 1) s_tmp[nw] = x;
    }
    __syncthreads();
    int run = s_tmp[wid] + incl - sum;
    if (chunk <= kRun) {
#pragma unroll
        for (int j = 0; j < kRun; ++j)
            if (b + j < e) {
                a[b + j] = run;
                run += v[j];
            }
    } else {
        for (int i = b; i < e; ++i) {
            const int x = a[i];
            a[i] = run;
            run += x;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Keyframe grid in LDS: histogram of cells, exclusive scan, scatter of
// cell-ordered records (and descriptors), owner hash set.  On return s_cs[c]
// is the first slot of cell c and s_cs[cells] = n_kp.  The order of the
// keypoints inside a cell is arbitrary: the packed (distance, index) key
// makes every output independent of it.

template <bool STAGE_DESC>
__device__ void stage_keyframe(const BatchHdr& h, const KfDesc& kd, int32_t* s_cs, KpRec* s_rec, uint4* s_desc,
                               int32_t* s_own, int32_t* s_hash, int32_t* s_tmp) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n = kd.n_kp;
    const int cells = h.cells, C = h.grid_cols, R = h.grid_rows;
    const int hmask = h.lds_hash_mask;
    const float* xy = h.kp_xy + 2 * (int64_t)kd.kp_off;
    for (int c = tid; c <= cells; c += nt) s_cs[c] = 0;
    for (int s = tid; s <= hmask; s += nt) s_hash[s] = -1;
    __syncthreads();
    // The first kStageRegs keypoints of each thread are loaded once, with
    // their descriptors, and kept in registers across the scan; any further
    // keypoints (keyframes larger than kStageRegs * blockDim) are reloaded.
    constexpr int kStageRegs = 1;
    float kx[kStageRegs], ky[kStageRegs];
    int ko[kStageRegs], kc[kStageRegs], kw[kStageRegs];
    uint4 kd0[kStageRegs], kd1[kStageRegs];
#pragma unroll
    for (int q = 0; q < kStageRegs; ++q) {
        const int i = tid + q * nt;
        kc[q] = -1;
        if (i < n) {
            kx[q] = xy[2 * i];
            ky[q] = xy[2 * i + 1];
            ko[q] = (int)h.kp_oct[kd.kp_off + i];
            if (STAGE_DESC) {
                const uint4* src = reinterpret_cast<const uint4*>(h.kp_desc + 32 * ((int64_t)kd.kp_off + i));
                kd0[q] = src[0];
                kd1[q] = src[1];
            }
            const int32_t o = h.kp_owner[kd.kp_off + i];
            kw[q] = o;
            kc[q] = cell_of(ky[q], kd.invh, R) * C + cell_of(kx[q], kd.invw, C);
            atomicAdd(&s_cs[kc[q] + 1], 1);
            if (o >= 0) owner_insert(s_hash, hmask, o);
        }
    }
    for (int i = tid + kStageRegs * nt; i < n; i += nt) {
        const int c = cell_of(xy[2 * i + 1], kd.invh, R) * C + cell_of(xy[2 * i], kd.invw, C);
        atomicAdd(&s_cs[c + 1], 1);
        const int32_t o = h.kp_owner[kd.kp_off + i];
        if (o >= 0) owner_insert(s_hash, hmask, o);
    }
    __syncthreads();
    block_exclusive_scan(s_cs + 1, cells, s_tmp);   // s_cs[1 + c] = first slot of c
#pragma unroll
    for (int q = 0; q < kStageRegs; ++q) {
        if (kc[q] < 0) continue;
        const int slot = atomicAdd(&s_cs[kc[q] + 1], 1);   // ends as the first slot of c + 1
        KpRec r;
        r.x = kx[q];
        r.y = ky[q];
        r.idx = tid + q * nt;
        r.oct = ko[q];
        s_rec[slot] = r;
        s_own[slot] = kw[q];
        if (STAGE_DESC) {
            s_desc[2 * slot] = kd0[q];
            s_desc[2 * slot + 1] = kd1[q];
        }
    }
    for (int i = tid + kStageRegs * nt; i < n; i += nt) {
        const float x = xy[2 * i], y = xy[2 * i + 1];
        const int c = cell_of(y, kd.invh, R) * C + cell_of(x, kd.invw, C);
        const int slot = atomicAdd(&s_cs[c + 1], 1);
        KpRec r;
        r.x = x;
        r.y = y;
        r.idx = i;
        r.oct = (int)h.kp_oct[kd.kp_off + i];
        s_rec[slot] = r;
        s_own[slot] = h.kp_owner[kd.kp_off + i];
        if (STAGE_DESC) {
            const uint4* src = reinterpret_cast<const uint4*>(h.kp_desc + 32 * ((int64_t)kd.kp_off + i));
            s_desc[2 * slot] = src[0];
            s_desc[2 * slot + 1] = src[1];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Global keyframe grids (fallback for keyframes too large for LDS, and
// fl_build_grid): one workgroup per keyframe.

constexpr int kPrepBlock = 256;

__device__ void build_grid_global(const KfDesc& kd, int cells, int C, int R, const float* __restrict__ kp_xy,
                                  int32_t* __restrict__ cs, int32_t* __restrict__ ck, int32_t* s_cnt,
                                  int32_t* s_tmp) {
    const int tid = threadIdx.x, nb = blockDim.x;
    const int n = kd.n_kp;
    const float* xy = kp_xy + 2 * (int64_t)kd.kp_off;
    for (int c = tid; c <= cells; c += nb) s_cnt[c] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += nb) {
        const int c = cell_of(xy[2 * i + 1], kd.invh, R) * C + cell_of(xy[2 * i], kd.invw, C);
        atomicAdd(&s_cnt[c], 1);
    }
    __syncthreads();
    block_exclusive_scan(s_cnt, cells, s_tmp);
    for (int c = tid; c < cells; c += nb) cs[c] = s_cnt[c];
    if (tid == 0) cs[cells] = n;
    __syncthreads();
    for (int i = tid; i < n; i += nb) {
        const int c = cell_of(xy[2 * i + 1], kd.invh, R) * C + cell_of(xy[2 * i], kd.invw, C);
        ck[atomicAdd(&s_cnt[c], 1)] = i;
    }
    __syncthreads();
    // keypoints of a cell in increasing index order (deterministic layout)
    for (int c = tid; c < cells; c += nb) {
        const int b = cs[c], e = cs[c + 1];
        for (int a = b + 1; a < e; ++a) {
            const int v = ck[a];
            int j = a - 1;
            while (j >= b && ck[j] > v) {
                ck[j + 1] = ck[j];
                --j;
            }
            ck[j + 1] = v;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kPrepBlock) void prep_global_kernel(const BatchHdr* __restrict__ hp) {
    __shared__ int32_t s_cnt[FL_MAX_CELLS + 1];
    __shared__ int32_t s_tmp[kPrepBlock / kWave + 1];
    const BatchHdr& h = *hp;
    for (int k = blockIdx.x; k < h.n_kf; k += gridDim.x) {
        const KfDesc& kd = h.kf[k];
        if (kd.pass != 0) continue;   // the other passes of a keyframe share its grid
        int32_t* cs = h.cell_start + kd.grid_off;
        int32_t* ck = h.cell_kp + kd.kp_off;
        build_grid_global(kd, h.cells, h.grid_cols, h.grid_rows, h.kp_xy, cs, ck, s_cnt, s_tmp);
        for (int s = threadIdx.x; s < kd.n_kp; s += blockDim.x) {
            const int i = ck[s];
            KpRec r;
            r.x = h.kp_xy[2 * ((int64_t)kd.kp_off + i)];
            r.y = h.kp_xy[2 * ((int64_t)kd.kp_off + i) + 1];
            r.idx = i;
            r.oct = (int)h.kp_oct[kd.kp_off + i];
            h.recs[kd.kp_off + s] = r;
            const uint4* src = reinterpret_cast<const uint4*>(h.kp_desc + 32 * ((int64_t)kd.kp_off + i));
            h.desc_sorted[2 * ((int64_t)kd.kp_off + s)] = src[0];
            h.desc_sorted[2 * ((int64_t)kd.kp_off + s) + 1] = src[1];
        }
        int32_t* tab = h.hash + kd.hash_off;
        for (int s = threadIdx.x; s <= kd.hash_mask; s += blockDim.x) tab[s] = -1;
        __syncthreads();
        for (int i = threadIdx.x; i < kd.n_kp; i += blockDim.x) {
            const int32_t o = h.kp_owner[kd.kp_off + i];
            if (o >= 0) owner_insert(tab, kd.hash_mask, o);
        }
        __syncthreads();
    }
}

// Grid of a single keyframe into caller buffers (fl_build_grid).
__global__ __launch_bounds__(kPrepBlock) void grid_single_kernel(KfDesc kd, int cells, int C, int R,
                                                               const float* __restrict__ kp_xy,
                                                               int32_t* __restrict__ cell_start,
                                                               int32_t* __restrict__ cell_kp) {
    __shared__ int32_t s_cnt[FL_MAX_CELLS + 1];
    __shared__ int32_t s_tmp[kPrepBlock / kWave + 1];
    build_grid_global(kd, cells, C, R, kp_xy, cell_start, cell_kp, s_cnt, s_tmp);
}

// ---------------------------------------------------------------------------
// Per-call tables are fetched by the device from pinned host memory (a plain
// copy kernel, in stream order with the kernels that read them).

// It also advances the claim epoch of the launch that follows (counting
// down, so claims of earlier launches always compare larger).
__global__ __launch_bounds__(256) void fetch_blob_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                       int n16, uint32_t* __restrict__ epoch) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += gridDim.x * blockDim.x) dst[i] = src[i];
    if (epoch && blockIdx.x == 0 && threadIdx.x == 0) *epoch = *epoch - 1u;
}

// ---------------------------------------------------------------------------
// Wave-aggregated append to a bounded list: one atomic per wave.

template <typename T>
__device__ __forceinline__ void wave_append(bool want, uint32_t* counter, T* list, int32_t cap, const T& e) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const int lane = wave_lane();
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader);
    if (want) {
        const uint32_t idx = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (idx < (uint32_t)cap) list[idx] = e;
    }
}

// ---------------------------------------------------------------------------
// Fused batched search.  Each workgroup owns a contiguous, cost-balanced run
// of tiles inside the range of its XCD (workgroups are dispatched to the 8
// XCDs round-robin), so the keyframes of an XCD stay in its L2 and no atomic
// is spent on scheduling.  A tile is up to 1024 * PPL consecutive pairs of
// one keyframe, a whole number of waves; pair j of a tile goes to thread
// j mod 1024, so a tile smaller than the workgroup leaves its last waves
// idle.  When its tile moves to a new keyframe the workgroup builds that
// keyframe's grid, records (and descriptors) and owner hash set in LDS.  The
// ADD conflicts are resolved by the next kernel on the stream.

struct KfView {
    const int32_t* cs;
    const KpRec* rec;
    const uint4* desc;          // cell-ordered descriptors (LDS or workspace), or null
    const uint8_t* desc_orig;   // keypoint descriptors by original index (when desc is null)
    const int32_t* own;         // cell-ordered owners (LDS), or null: read kp_owner by index
    const int32_t* hash;
    int32_t hash_mask;
};

// LDS bytes of the search kernel (shared with the host).
__host__ __device__ inline size_t search_lds_bytes(int mode, int kp_cap, int cells, int hash_cap) {
    if (mode == kModeGlobal) return 16;
    size_t b = 20 * (size_t)kp_cap;   // records + owners
    if (mode == kModeLdsDesc) b += 32 * (size_t)kp_cap;
    b += 4 * (size_t)((cells + 4 + 3) & ~3);
    b += 4 * (size_t)hash_cap;
    b += 4 * (size_t)(kSearchBlock / kWave + 4);
    return b;
}

template <int PPL, int MODE, bool STATS>
__global__ __launch_bounds__(kSearchBlock) void search_fused_kernel(const BatchHdr* __restrict__ hp) {
    extern __shared__ __align__(16) unsigned char s_mem[];
    const BatchHdr& h = *hp;
    const int tid = threadIdx.x;
    const int lane = wave_lane();
    KpRec* s_rec = reinterpret_cast<KpRec*>(s_mem);
    uint4* s_desc = nullptr;
    int32_t* s_cs = nullptr;
    int32_t* s_own = nullptr;
    int32_t* s_hash = nullptr;
    int32_t* s_tmp = nullptr;
    __shared__ uint32_t s_cnt[2 * PPL * kWavesPerWG + 2];   // per-wave list counts, then the two bases
    const int wid = tid / kWave;
    if (MODE != kModeGlobal) {
        unsigned char* p = s_mem + 16 * (size_t)h.lds_kp_cap;
        if (MODE == kModeLdsDesc) {
            s_desc = reinterpret_cast<uint4*>(p);
            p += 32 * (size_t)h.lds_kp_cap;
        }
        s_own = reinterpret_cast<int32_t*>(p);
        p += 4 * (size_t)h.lds_kp_cap;
        s_cs = reinterpret_cast<int32_t*>(p);
        p += 4 * (size_t)((h.cells + 4 + 3) & ~3);
        s_hash = reinterpret_cast<int32_t*>(p);
        p += 4 * (size_t)(h.lds_hash_mask + 1);
        s_tmp = reinterpret_cast<int32_t*>(p);
        p += 4 * (size_t)(kSearchBlock / kWave + 4);
    }

    // the octave scale table in LDS: the octave search and the window radius
    // index it per lane.  In the LDS modes the barrier that opens the first
    // keyframe's staging publishes it, so the tile's table and point loads
    // below are issued without waiting here.
    __shared__ float s_sf[FL_MAX_OCTAVES];
    if (tid < FL_MAX_OCTAVES) s_sf[tid] = h.sf[tid];
    if (MODE == kModeGlobal) __syncthreads();
    const float* sf = s_sf;
    const int N = h.n_octaves, gate = h.gate, C = h.grid_cols, R = h.grid_rows;
    const bool dense = h.dense != 0;
    const bool want_matches = h.refine_iters > 0;
    const unsigned long long tag = (unsigned long long)(*h.epoch) << 32;
    unsigned long long st_vis = 0, st_cells = 0, st_kp = 0, st_cand = 0;

    // tiles [x, y); the first one belongs to slot z (keyframe w) of the tile
    // order.  The ranges and the keyframe table sit at offsets of the table
    // blob that follow from the grid size, so neither waits for a pointer.
    const char* blob = reinterpret_cast<const char*>(hp);
    const int4 range = reinterpret_cast<const int4*>(blob + blob_range_offset())[blockIdx.x];
    const KfDesc* kf_tab = reinterpret_cast<const KfDesc*>(blob + blob_kf_offset((int)gridDim.x));
    int slot = range.z;
    int staged = -1;
    for (int t = range.x; t < range.y; ++t) {
        while (t >= h.tile_prefix[slot + 1]) ++slot;
        const int k = t == range.x ? range.w : h.kf_order[slot];
        const KfDesc kd = kf_tab[k];          // by value: kept in registers across the stores below
        const EventDesc ed = h.ev[kd.event];
        const PassOut& po = h.out[kd.pass];
        const int64_t pb = kd.pair_off + (int64_t)(t - h.tile_prefix[slot]) * kd.tile_pairs;
        const int64_t pe = min(pb + (int64_t)kd.tile_pairs, kd.pair_off + kd.n_pairs);
        // A provisional ADD is written as ADD here; the ADD conflicts are
        // resolved after the whole search, by the next kernel on the stream
        // (the refinement, or the resolution kernel when there is none), which
        // relabels the losers.  No tile waits for another.

        // Point loads of every pair of this thread are issued first, so their
        // latency overlaps the keyframe staging below.
        uint8_t dec[PPL];
        int32_t gp[PPL], id[PPL];
        float px[PPL], py[PPL], pz[PPL], pdm[PPL];
        uint4 a0[PPL], a1[PPL];
        bool add_want[PPL], acc_want[PPL];
        int32_t add_kp[PPL];
        float acc_u[PPL], acc_v[PPL];
#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            const int64_t o = pb + (int64_t)r * kSearchBlock + tid;
            dec[r] = o < pe ? kDecUndecided : (uint8_t)0;
            gp[r] = 0;
            id[r] = -1;
            px[r] = py[r] = pz[r] = pdm[r] = 0.0f;
            a0[r] = a1[r] = make_uint4(0, 0, 0, 0);
            if (o < pe) {
                const int64_t j = o - kd.pair_off;
                const int32_t lp = dense ? (int32_t)j : h.pair_mp[o];
                if (lp < 0 || lp >= kd.n_mp) {
                    dec[r] = FL_INVALID;
                } else {
                    gp[r] = kd.mp_off + lp;
                    id[r] = h.mp_id ? h.mp_id[gp[r]] : gp[r];
                    px[r] = h.mp_xyz[3 * (int64_t)gp[r]];
                    py[r] = h.mp_xyz[3 * (int64_t)gp[r] + 1];
                    pz[r] = h.mp_xyz[3 * (int64_t)gp[r] + 2];
                    if (gate) pdm[r] = h.mp_dmax[gp[r]];
                    load_desc(h.mp_desc, gp[r], a0[r], a1[r]);
                }
            }
        }

        KfView v;
        if (MODE == kModeGlobal) {
            v.cs = h.cell_start + kd.grid_off;
            v.rec = h.recs + kd.kp_off;
            v.desc = h.desc_sorted + 2 * (int64_t)kd.kp_off;
            v.desc_orig = nullptr;
            v.own = nullptr;
            v.hash = h.hash + kd.hash_off;
            v.hash_mask = kd.hash_mask;
        } else {
            if (staged != kd.stage_key) {
                __syncthreads();   // every reader of the previous keyframe is done
                stage_keyframe<MODE == kModeLdsDesc>(h, kd, s_cs, s_rec, s_desc, s_own, s_hash, s_tmp);
                staged = kd.stage_key;
            }
            v.cs = s_cs;
            v.rec = s_rec;
            v.desc = MODE == kModeLdsDesc ? s_desc : nullptr;
            v.desc_orig = h.kp_desc + 32 * (int64_t)kd.kp_off;
            v.own = s_own;
            v.hash = s_hash;
            v.hash_mask = h.lds_hash_mask;
        }

#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            const int64_t o = pb + (int64_t)r * kSearchBlock + tid;
            const bool active = o < pe;
            // owner probe: a point already observed in this keyframe is skipped
            if (dec[r] == kDecUndecided && id[r] >= 0) {
                uint32_t hh = owner_slot(id[r], v.hash_mask);
                for (int probe = 0; probe <= v.hash_mask; ++probe) {
                    const int32_t hv = v.hash[hh];
                    if (hv == id[r]) {
                        dec[r] = FL_SKIP;
                        break;
                    }
                    if (hv < 0) break;
                    hh = (hh + 1) & (uint32_t)v.hash_mask;
                }
            }
            Best best;
            best.init();
            int32_t target = -1;
            float ku = 0.0f, kv = 0.0f;
            int bslot = 0;
            if (dec[r] == kDecUndecided) {
                Proj p;
                if (!project(kd, px[r], py[r], pz[r], pdm[r], gate, sf, N, p)) {
                    dec[r] = FL_NOT_VISIBLE;
                } else {
                    if (STATS) ++st_vis;
                    const Window w = make_window(p, kd, sf, po.r0, C, R);
                    for (int row = w.r0; row <= w.r1; ++row) {
                        const int s = v.cs[row * C + w.c0];
                        const int e = v.cs[row * C + w.c1 + 1];
                        if (STATS) {
                            st_cells += (unsigned long long)(w.c1 - w.c0 + 1);
                            st_kp += (unsigned long long)(e - s);
                        }
                        for (int i = s; i < e; ++i) {
                            const KpRec rc = v.rec[i];
                            if (!in_window(w, rc.x, rc.y, rc.oct, p.pred, gate)) continue;
                            if (STATS) ++st_cand;
                            uint4 b0, b1;
                            if (MODE == kModeLdsRec) {
                                load_desc(v.desc_orig, rc.idx, b0, b1);
                            } else {
                                b0 = v.desc[2 * i];
                                b1 = v.desc[2 * i + 1];
                            }
                            const uint32_t before = best.key;
                            best.offer(hamming(a0[r], a1[r], b0, b1), rc.idx);
                            if (best.key != before) {
                                ku = rc.x;
                                kv = rc.y;
                                bslot = i;
                            }
                        }
                    }
                    if (!accept_match(best, po.hamming_th, po.nn_ratio)) {
                        dec[r] = FL_NO_MATCH;
                    } else {
                        const int32_t ow = v.own ? v.own[bslot]
                                                 : h.kp_owner[kd.kp_off + (int32_t)(best.key & 0xFFFFu)];
                        if (ow >= 0) {
                            dec[r] = FL_FUSE;
                            target = ow;
                        } else {
                            dec[r] = FL_ADD;   // provisional; losers are relabelled by the resolver
                        }
                    }
                }
            }
            const int bidx = best.key == 0xFFFFFFFFu ? -1 : (int)(best.key & 0xFFFFu);
            const int kpg = kd.claim_off + (bidx < 0 ? 0 : bidx);   // claim slot
            const bool is_add = active && dec[r] == FL_ADD;
            if (active) {
                po.best_idx[o] = bidx;
                po.best_dist[o] = (int16_t)(best.key == 0xFFFFFFFFu ? FL_NO_DIST : (int)(best.key >> 16));
                po.second_dist[o] = (int16_t)best.second;
                po.decision[o] = dec[r];
                po.target[o] = target;
            }
            if (is_add) atomicMin(&h.claim[kpg], tag | (uint32_t)gp[r]);
            // list entries are written after the tile with one atomic per list
            add_want[r] = is_add;
            add_kp[r] = kpg;
            acc_want[r] = want_matches && active && (dec[r] == FL_ADD || dec[r] == FL_FUSE);
            acc_u[r] = ku;
            acc_v[r] = kv;
            const unsigned long long ma = __ballot(add_want[r]);
            const unsigned long long mm = __ballot(acc_want[r]);
            if (lane == 0) {
                s_cnt[(2 * r) * kWavesPerWG + wid] = (uint32_t)__popcll(ma);
                s_cnt[(2 * r + 1) * kWavesPerWG + wid] = (uint32_t)__popcll(mm);
            }
        }
        __syncthreads();
        if (wid == 0) {
            // wave 0 turns the per-wave counts (pair slot major, wave minor)
            // into offsets and reserves both lists
            static_assert(PPL * kWavesPerWG <= kWave, "one count per lane");
            constexpr int nv = PPL * kWavesPerWG;
            const int r = lane / kWavesPerWG, w = lane % kWavesPerWG;
            const bool in = lane < nv;
            const int ca = in ? (int)s_cnt[(2 * r) * kWavesPerWG + w] : 0;
            const int cm = in ? (int)s_cnt[(2 * r + 1) * kWavesPerWG + w] : 0;
            const int ia = wave_incl_scan(ca), im = wave_incl_scan(cm);
            if (in) {
                s_cnt[(2 * r) * kWavesPerWG + w] = (uint32_t)(ia - ca);
                s_cnt[(2 * r + 1) * kWavesPerWG + w] = (uint32_t)(im - cm);
            }
            const uint32_t run_a = (uint32_t)__builtin_amdgcn_readlane(ia, nv - 1);
            const uint32_t run_m = (uint32_t)__builtin_amdgcn_readlane(im, nv - 1);
            if (lane == 0) {
                // both list reservations are issued before either result is used
                const uint32_t ba = run_a ? atomicAdd(&h.kf_ctr[k * kKfCtrs + kKfAdd], run_a) : 0u;
                const uint32_t bm = run_m ? atomicAdd(&h.ev_ctr[kd.event * kEvCtrs + kEvMatch], run_m) : 0u;
                s_cnt[2 * PPL * kWavesPerWG] = ba;
                s_cnt[2 * PPL * kWavesPerWG + 1] = bm;
            }
        }
        __syncthreads();
        {
            const uint32_t base_a = s_cnt[2 * PPL * kWavesPerWG], base_m = s_cnt[2 * PPL * kWavesPerWG + 1];
            const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                const int64_t o = pb + (int64_t)r * kSearchBlock + tid;
                const unsigned long long ma = __ballot(add_want[r]);
                const unsigned long long mm = __ballot(acc_want[r]);
                if (add_want[r]) {
                    const uint32_t idx = base_a + s_cnt[(2 * r) * kWavesPerWG + wid] + (uint32_t)__popcll(ma & below);
                    if (idx < (uint32_t)kd.add_cap) {
                        AddRef e;
                        e.pair = (int32_t)o;
                        e.kp = add_kp[r];
                        e.gp = gp[r];
                        e.pad = 0;
                        h.add_list[kd.add_off + idx] = e;
                    }
                }
                if (acc_want[r]) {
                    const uint32_t idx =
                        base_m + s_cnt[(2 * r + 1) * kWavesPerWG + wid] + (uint32_t)__popcll(mm & below);
                    if (idx < (uint32_t)ed.list_cap) {
                        MatchRec me;
                        me.x = px[r];
                        me.y = py[r];
                        me.z = pz[r];
                        me.u = acc_u[r];
                        me.v = acc_v[r];
                        me.kf = k;
                        me.pad0 = me.pad1 = 0;
                        h.match_list[ed.list_off + idx] = me;
                    }
                }
            }
        }
    }
    if (STATS) {
        unsigned long long vals[4] = {st_vis, st_cells, st_kp, st_cand};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            unsigned long long xv = vals[i];
            for (int off = 32; off > 0; off >>= 1) xv += __shfl_xor(xv, off);
            if (lane == 0 && xv) atomicAdd(&h.stats_out[i], xv);
        }
    }
}

// ADD resolution after a batched search launched without refinement: one
// workgroup per keyframe, grid-stride.
constexpr int kResolveBlock = 256;
constexpr int kResolveGrid = 1024;   // workgroups in graph mode (any count is correct)

__global__ __launch_bounds__(kResolveBlock) void resolve_adds_kernel(const BatchHdr* __restrict__ hp) {
    const BatchHdr& h = *hp;
    const unsigned long long tag = (unsigned long long)(*h.epoch) << 32;
    for (int k = blockIdx.x; k < h.n_kf; k += gridDim.x) resolve_keyframe_adds(h, k, tag);
}

// ---------------------------------------------------------------------------
// Plain search: one lane per map point against one keyframe, candidates
// gathered through the caller's (or a freshly built) cell_start / cell_kp
// grid from the keyframe's own arrays.

// Owner hash set and claim reset of a single keyframe (plain path).
__global__ __launch_bounds__(kPrepBlock) void plain_prep_kernel(int n, const int32_t* __restrict__ kp_owner,
                                                              int32_t* __restrict__ tab, int32_t mask,
                                                              int32_t* __restrict__ claim,
                                                              uint32_t* __restrict__ counter) {
    const int tid = threadIdx.x;
    for (int s = tid; s <= mask; s += blockDim.x) tab[s] = -1;
    for (int i = tid; i < n; i += blockDim.x) claim[i] = 0x7FFFFFFF;
    if (tid == 0) *counter = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
        const int32_t o = kp_owner[i];
        if (o >= 0) owner_insert(tab, mask, o);
    }
}

struct PlainArgs {
    KfDesc kd;
    SearchConst sc;
    int32_t n_mp;
    int32_t add_cap;
    const float* mp_xyz;
    const uint8_t* mp_desc;
    const float* mp_dmax;
    const int32_t* mp_id;
    const float* kp_xy;
    const int8_t* kp_oct;
    const uint8_t* kp_desc;
    const int32_t* kp_owner;
    const int32_t* cell_start;
    const int32_t* cell_kp;
    const int32_t* hash;
    int32_t* claim;
    uint32_t* counter;
    AddRef* add_list;
    int32_t* best_idx;
    int16_t* best_dist;
    int16_t* second_dist;
    uint8_t* decision;
    int32_t* target;
};

__global__ __launch_bounds__(256) void search_plain_kernel(PlainArgs a) {
    __shared__ float s_sf[FL_MAX_OCTAVES];
    if (threadIdx.x < FL_MAX_OCTAVES) s_sf[threadIdx.x] = a.sc.sf[threadIdx.x];
    __syncthreads();
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = o < a.n_mp;
    const KfDesc& kd = a.kd;
    const SearchConst& sc = a.sc;
    uint8_t dec = active ? kDecUndecided : (uint8_t)0;
    const int32_t gp = (int32_t)o;
    const int32_t id = active ? (a.mp_id ? a.mp_id[gp] : gp) : 0;
    if (active && owner_lookup(a.hash, kd.hash_mask, id)) dec = FL_SKIP;
    Best best;
    best.init();
    int32_t target = -1;
    if (dec == kDecUndecided) {
        const float x = a.mp_xyz[3 * o], y = a.mp_xyz[3 * o + 1], z = a.mp_xyz[3 * o + 2];
        const float dmax = sc.gate ? a.mp_dmax[o] : 0.0f;
        Proj p;
        if (!project(kd, x, y, z, dmax, sc.gate, s_sf, sc.N, p)) {
            dec = FL_NOT_VISIBLE;
        } else {
            uint4 a0, a1;
            load_desc(a.mp_desc, o, a0, a1);
            const Window w = make_window(p, kd, s_sf, sc.r0, sc.C, sc.R);
            for (int row = w.r0; row <= w.r1; ++row) {
                // a caller-supplied grid is clamped to the keypoint range
                const int s = max(a.cell_start[row * sc.C + w.c0], 0);
                const int e = min(a.cell_start[row * sc.C + w.c1 + 1], kd.n_kp);
                for (int i = s; i < e; ++i) {
                    const int kp = a.cell_kp[i];
                    if ((unsigned)kp >= (unsigned)kd.n_kp) continue;
                    const float kx = a.kp_xy[2 * kp], ky = a.kp_xy[2 * kp + 1];
                    if (!in_window(w, kx, ky, (int)a.kp_oct[kp], p.pred, sc.gate)) continue;
                    uint4 b0, b1;
                    load_desc(a.kp_desc, kp, b0, b1);
                    best.offer(hamming(a0, a1, b0, b1), kp);
                }
            }
            if (!accept_match(best, sc.th, sc.ratio)) {
                dec = FL_NO_MATCH;
            } else {
                const int32_t ow = a.kp_owner[best.key & 0xFFFFu];
                if (ow >= 0) {
                    dec = FL_FUSE;
                    target = ow;
                } else {
                    dec = FL_ADD;
                }
            }
        }
    }
    const int bidx = best.key == 0xFFFFFFFFu ? -1 : (int)(best.key & 0xFFFFu);
    if (active) {
        a.best_idx[o] = bidx;
        a.best_dist[o] = (int16_t)(best.key == 0xFFFFFFFFu ? FL_NO_DIST : (int)(best.key >> 16));
        a.second_dist[o] = (int16_t)best.second;
        a.decision[o] = dec;
        a.target[o] = target;
    }
    const bool is_add = active && dec == FL_ADD;
    if (is_add) atomicMin(&a.claim[bidx], gp);
    AddRef e;
    e.pair = (int32_t)o;
    e.kp = bidx < 0 ? 0 : bidx;
    e.gp = gp;
    e.pad = 0;
    wave_append(is_add, a.counter, a.add_list, a.add_cap, e);
}

__global__ __launch_bounds__(256) void resolve_plain_kernel(int32_t n_mp, const uint32_t* __restrict__ counter,
                                                          const AddRef* __restrict__ list, int32_t cap,
                                                          const int32_t* __restrict__ claim,
                                                          const int32_t* __restrict__ mp_id,
                                                          const int32_t* __restrict__ best_idx,
                                                          uint8_t* __restrict__ decision,
                                                          int32_t* __restrict__ target) {
    const uint32_t n = *counter;
    const int stride = gridDim.x * blockDim.x;
    if (n <= (uint32_t)cap) {
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            const AddRef e = list[i];
            const int32_t w = claim[e.kp];
            if (w != e.gp) {
                decision[e.pair] = FL_FUSE;
                target[e.pair] = mp_id ? mp_id[w] : w;
            }
        }
        return;
    }
    for (int32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < n_mp; o += stride) {
        if (decision[o] != FL_ADD) continue;
        const int32_t w = claim[best_idx[o]];
        if (w != o) {
            decision[o] = FL_FUSE;
            target[o] = mp_id ? mp_id[w] : w;
        }
    }
}

}  // namespace fl
