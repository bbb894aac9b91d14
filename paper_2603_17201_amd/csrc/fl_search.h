// Search-and-fuse kernels: keypoint grid build, the persistent batched
// search, the plain per-keyframe search and ADD-conflict resolution.
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

// ---------------------------------------------------------------------------
// Grid build: one workgroup per keyframe (strided).  LDS histogram of cells,
// exclusive prefix scan into cell_start, scatter of keypoint indices into
// cell_kp, then per-cell sort so the layout is deterministic.  Optionally
// also writes the cell-ordered records / descriptors, the owner hash set,
// resets the ADD claims and fills the tile table.

constexpr int kPrepBlock = 256;

template <bool FULL>
__device__ void prep_keyframe(const KfDesc& kd, int k, int cells, int C, int R, const float* __restrict__ kp_xy,
                              const int8_t* __restrict__ kp_oct, const uint8_t* __restrict__ kp_desc,
                              const int32_t* __restrict__ kp_owner, int32_t* __restrict__ cell_start,
                              int32_t* __restrict__ cell_kp, KpRec* __restrict__ recs,
                              uint4* __restrict__ desc_sorted, int32_t* __restrict__ hash,
                              int32_t* __restrict__ claim, int2* __restrict__ tiles, int32_t* s_cnt,
                              int32_t* s_part) {
    const int tid = threadIdx.x;
    const int nb = blockDim.x;
    const int n = kd.n_kp;
    const float* xy = kp_xy + 2 * (int64_t)kd.kp_off;
    for (int c = tid; c < cells; c += nb) s_cnt[c] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += nb) {
        const int c = cell_of(xy[2 * i + 1], kd.invh, R) * C + cell_of(xy[2 * i], kd.invw, C);
        atomicAdd(&s_cnt[c], 1);
    }
    __syncthreads();
    // exclusive scan: each thread owns a contiguous chunk of cells
    const int chunk = (cells + nb - 1) / nb;
    const int cb = min(tid * chunk, cells), ce = min(cb + chunk, cells);
    int sum = 0;
    for (int c = cb; c < ce; ++c) sum += s_cnt[c];
    s_part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < nb; off <<= 1) {
        const int v = tid >= off ? s_part[tid - off] : 0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    int run = s_part[tid] - sum;   // exclusive prefix of this chunk
    int32_t* cs = cell_start + kd.grid_off;
    for (int c = cb; c < ce; ++c) {
        const int v = s_cnt[c];
        cs[c] = run;
        s_cnt[c] = run;
        run += v;
    }
    if (tid == nb - 1) cs[cells] = s_part[nb - 1];
    __syncthreads();
    int32_t* ck = cell_kp + kd.kp_off;
    for (int i = tid; i < n; i += nb) {
        const int c = cell_of(xy[2 * i + 1], kd.invh, R) * C + cell_of(xy[2 * i], kd.invw, C);
        const int slot = atomicAdd(&s_cnt[c], 1);
        ck[slot] = i;
    }
    __syncthreads();
    // keypoints of a cell in increasing index order
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
    if (!FULL) return;
    __syncthreads();
    for (int s = tid; s < n; s += nb) {
        const int i = ck[s];
        KpRec r;
        r.x = xy[2 * i];
        r.y = xy[2 * i + 1];
        r.idx = i;
        r.oct = (int)kp_oct[kd.kp_off + i];
        recs[kd.kp_off + s] = r;
        const uint4* src = reinterpret_cast<const uint4*>(kp_desc + 32 * ((int64_t)kd.kp_off + i));
        uint4* dst = desc_sorted + 2 * ((int64_t)kd.kp_off + s);
        dst[0] = src[0];
        dst[1] = src[1];
    }
    int32_t* tab = hash + kd.hash_off;
    for (int s = tid; s <= kd.hash_mask; s += nb) tab[s] = -1;
    for (int i = tid; i < n; i += nb) claim[kd.kp_off + i] = 0x7FFFFFFF;
    for (int j = tid; j < kd.n_tiles; j += nb) tiles[kd.tile_off + j] = make_int2(k, j);
    __syncthreads();
    for (int i = tid; i < n; i += nb) {
        const int32_t o = kp_owner[kd.kp_off + i];
        if (o < 0) continue;
        uint32_t hh = (hash_id(o) >> 7) & (uint32_t)kd.hash_mask;
        for (;;) {
            const int32_t prev = atomicCAS(&tab[hh], -1, o);
            if (prev == -1 || prev == o) break;
            hh = (hh + 1) & (uint32_t)kd.hash_mask;
        }
    }
}

__global__ __launch_bounds__(kPrepBlock) void prep_batched_kernel(const BatchHdr* __restrict__ hp) {
    __shared__ int32_t s_cnt[FL_MAX_CELLS];
    __shared__ int32_t s_part[kPrepBlock];
    const BatchHdr& h = *hp;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < kCounterWords; i += blockDim.x) h.counters[i] = 0;
        for (int i = threadIdx.x; i < 4; i += blockDim.x) h.stats_out[i] = 0ull;
        for (int i = threadIdx.x; i < h.n_events; i += blockDim.x) {
            h.ev_match_count[i] = 0;
            h.refine_done[i] = 0;
        }
    }
    for (int k = blockIdx.x; k < h.n_kf; k += gridDim.x) {
        const KfDesc& kd = h.kf[k];
        prep_keyframe<true>(kd, k, h.cells, h.grid_cols, h.grid_rows, h.kp_xy, h.kp_oct, h.kp_desc, h.kp_owner,
                            h.cell_start, h.cell_kp, h.recs, h.desc_sorted, h.hash, h.claim,
                            h.tile, s_cnt, s_part);
        __syncthreads();
    }
}

// Grid of a single keyframe into caller buffers (fl_build_grid).
__global__ __launch_bounds__(kPrepBlock) void grid_single_kernel(KfDesc kd, int cells, int C, int R,
                                                               const float* __restrict__ kp_xy,
                                                               int32_t* __restrict__ cell_start,
                                                               int32_t* __restrict__ cell_kp) {
    __shared__ int32_t s_cnt[FL_MAX_CELLS];
    __shared__ int32_t s_part[kPrepBlock];
    prep_keyframe<false>(kd, 0, cells, C, R, kp_xy, nullptr, nullptr, nullptr, cell_start, cell_kp, nullptr,
                         nullptr, nullptr, nullptr, nullptr, s_cnt, s_part);
}

// Owner hash set and claim reset of a single keyframe (plain path).
__global__ __launch_bounds__(kPrepBlock) void plain_prep_kernel(int n, const int32_t* __restrict__ kp_owner,
                                                              int32_t* __restrict__ tab, int32_t mask,
                                                              int32_t* __restrict__ claim,
                                                              uint32_t* __restrict__ counters) {
    const int tid = threadIdx.x;
    for (int s = tid; s <= mask; s += blockDim.x) tab[s] = -1;
    for (int i = tid; i < n; i += blockDim.x) claim[i] = 0x7FFFFFFF;
    for (int i = tid; i < kCounterWords; i += blockDim.x) counters[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
        const int32_t o = kp_owner[i];
        if (o < 0) continue;
        uint32_t hh = (hash_id(o) >> 7) & (uint32_t)mask;
        for (;;) {
            const int32_t prev = atomicCAS(&tab[hh], -1, o);
            if (prev == -1 || prev == o) break;
            hh = (hh + 1) & (uint32_t)mask;
        }
    }
}

// ---------------------------------------------------------------------------
// Wave-aggregated append to a list: one atomic per wave.

__device__ __forceinline__ void wave_append(bool want, uint32_t* counter, PairRef* list, int32_t cap,
                                            const PairRef& e) {
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
// Persistent batched search.  Each wave takes tiles of 64 * PPL consecutive
// pairs of one keyframe from an atomic work queue; with one queue per XCD,
// a workgroup serves the queue of the XCD it was dispatched to (workgroups
// are dispatched to the 8 XCDs round-robin) and steals from the next queues
// once its own is empty, so the keyframes of a queue stay in one L2.

template <int PPL, bool STATS>
__global__ __launch_bounds__(256) void search_batched_kernel(const BatchHdr* __restrict__ hp) {
    const BatchHdr& h = *hp;
    const int lane = wave_lane();
    const int nq = h.n_queues;
    int q = (int)(blockIdx.x % (unsigned)nq);
    int exhausted = 0;
    SearchConst sc;   // scalars only; the octave table is read from the header
    const float* sf = h.sf;
    sc.N = h.n_octaves;
    sc.gate = h.gate;
    sc.C = h.grid_cols;
    sc.R = h.grid_rows;
    sc.th = h.hamming_th;
    sc.ratio = h.nn_ratio;
    sc.r0 = h.r0;
    const bool dense = h.dense != 0;
    const bool want_matches = h.refine_iters > 0;
    unsigned long long st_vis = 0, st_cells = 0, st_kp = 0, st_cand = 0;

    for (;;) {
        int t = 0;
        if (lane == 0) t = (int)atomicAdd(&h.counters[kCtrQueue + q], 1u);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0)) + h.queue_begin[q];
        if (t >= h.queue_begin[q + 1]) {
            if (++exhausted >= nq) break;
            q = (q + 1 == nq) ? 0 : q + 1;
            continue;
        }
        const int2 te = h.tile[t];
        const int k = __builtin_amdgcn_readfirstlane(te.x);
        const int tk = __builtin_amdgcn_readfirstlane(te.y);
        const KfDesc& kd = h.kf[k];
        const EventDesc& ed = h.ev[kd.event];
        const int64_t pb = kd.pair_off + (int64_t)tk * h.tile_pairs;
        const int64_t pe = min(pb + (int64_t)h.tile_pairs, kd.pair_off + kd.n_pairs);
        const int32_t* cs = h.cell_start + kd.grid_off;
        const KpRec* recs = h.recs + kd.kp_off;
        const uint4* kdesc = h.desc_sorted + 2 * (int64_t)kd.kp_off;
        const int32_t* tab = h.hash + kd.hash_off;

#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            const int64_t o = pb + (int64_t)r * kWave + lane;
            const bool active = o < pe;
            uint8_t dec = active ? kDecUndecided : (uint8_t)0;
            int32_t gp = 0, id = 0;
            if (active) {
                const int64_t j = o - kd.pair_off;
                const int32_t lp = dense ? (int32_t)j : h.pair_mp[o];
                if (lp < 0 || lp >= kd.n_mp) {
                    dec = FL_INVALID;
                } else {
                    gp = kd.mp_off + lp;
                    id = h.mp_id ? h.mp_id[gp] : gp;
                    if (owner_lookup(tab, kd.hash_mask, id)) dec = FL_SKIP;
                }
            }
            Best best;
            best.init();
            int32_t target = -1;
            if (dec == kDecUndecided) {
                const float x = h.mp_xyz[3 * (int64_t)gp];
                const float y = h.mp_xyz[3 * (int64_t)gp + 1];
                const float z = h.mp_xyz[3 * (int64_t)gp + 2];
                const float dmax = sc.gate ? h.mp_dmax[gp] : 0.0f;
                Proj p;
                if (!project(kd, x, y, z, dmax, sc.gate, sf, sc.N, p)) {
                    dec = FL_NOT_VISIBLE;
                } else {
                    if (STATS) ++st_vis;
                    uint4 a0, a1;
                    load_desc(h.mp_desc, gp, a0, a1);
                    const Window w = make_window(p, kd, sf, sc.r0, sc.C, sc.R);
                    for (int row = w.r0; row <= w.r1; ++row) {
                        const int s = cs[row * sc.C + w.c0];
                        const int e = cs[row * sc.C + w.c1 + 1];
                        if (STATS) {
                            st_cells += (unsigned long long)(w.c1 - w.c0 + 1);
                            st_kp += (unsigned long long)(e - s);
                        }
                        for (int i = s; i < e; ++i) {
                            const KpRec rc = recs[i];
                            if (!in_window(w, rc.x, rc.y, rc.oct, p.pred, sc.gate)) continue;
                            if (STATS) ++st_cand;
                            const uint4 b0 = kdesc[2 * i];
                            const uint4 b1 = kdesc[2 * i + 1];
                            best.offer(hamming(a0, a1, b0, b1), rc.idx);
                        }
                    }
                    if (!accept_match(best, sc.th, sc.ratio)) {
                        dec = FL_NO_MATCH;
                    } else {
                        const int32_t ow = h.kp_owner[kd.kp_off + (int32_t)(best.key & 0xFFFFu)];
                        if (ow >= 0) {
                            dec = FL_FUSE;
                            target = ow;
                        } else {
                            dec = FL_ADD;   // provisional; losers are relabelled by the resolve kernel
                        }
                    }
                }
            }
            const int bidx = best.key == 0xFFFFFFFFu ? -1 : (int)(best.key & 0xFFFFu);
            const int kpg = kd.kp_off + (bidx < 0 ? 0 : bidx);
            if (active) {
                h.best_idx[o] = bidx;
                h.best_dist[o] = (int16_t)(best.key == 0xFFFFFFFFu ? FL_NO_DIST : (int)(best.key >> 16));
                h.second_dist[o] = (int16_t)best.second;
                h.decision[o] = dec;
                h.target[o] = target;
            }
            const bool is_add = active && dec == FL_ADD;
            if (is_add) atomicMin(&h.claim[kpg], gp);
            PairRef e;
            e.pair = (int32_t)o;
            e.kp = kpg;
            e.gp = gp;
            e.kf = k;
            wave_append(is_add, &h.counters[kCtrAdd], h.add_list, h.add_cap, e);
            if (want_matches) {
                const bool acc = active && (dec == FL_ADD || dec == FL_FUSE);
                wave_append(acc, &h.ev_match_count[kd.event], h.match_list + ed.list_off, ed.list_cap, e);
            }
        }
    }
    if (STATS) {
        unsigned long long v[4] = {st_vis, st_cells, st_kp, st_cand};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            unsigned long long x = v[i];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            if (lane == 0 && x) atomicAdd(&h.stats_out[i], x);
        }
    }
}

// Conflict resolution: every provisional ADD whose point is not the lowest
// claimant of its keypoint becomes a FUSE into that claimant.  Uses the ADD
// list, or, when it overflowed, a scan of all pairs.
__global__ __launch_bounds__(256) void resolve_batched_kernel(const BatchHdr* __restrict__ hp) {
    const BatchHdr& h = *hp;
    const uint32_t n = h.counters[kCtrAdd];
    if (n <= (uint32_t)h.add_cap) {
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const PairRef e = h.add_list[i];
            const int32_t w = h.claim[e.kp];
            if (w != e.gp) {
                h.decision[e.pair] = FL_FUSE;
                h.target[e.pair] = h.mp_id ? h.mp_id[w] : w;
            }
        }
        return;
    }
    for (int k = blockIdx.x; k < h.n_kf; k += gridDim.x) {
        const KfDesc& kd = h.kf[k];
        for (int64_t j = threadIdx.x; j < kd.n_pairs; j += blockDim.x) {
            const int64_t o = kd.pair_off + j;
            if (h.decision[o] != FL_ADD) continue;
            const int32_t gp = kd.mp_off + (h.dense ? (int32_t)j : h.pair_mp[o]);
            const int32_t w = h.claim[kd.kp_off + h.best_idx[o]];
            if (w != gp) {
                h.decision[o] = FL_FUSE;
                h.target[o] = h.mp_id ? h.mp_id[w] : w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Plain search: one lane per map point against one keyframe, candidates
// gathered through the caller's (or a freshly built) cell_start / cell_kp
// grid from the keyframe's own arrays.

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
    uint32_t* counters;
    PairRef* add_list;
    int32_t* best_idx;
    int16_t* best_dist;
    int16_t* second_dist;
    uint8_t* decision;
    int32_t* target;
};

__global__ __launch_bounds__(256) void search_plain_kernel(PlainArgs a) {
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
        if (!project(kd, x, y, z, dmax, sc.gate, sc.sf, sc.N, p)) {
            dec = FL_NOT_VISIBLE;
        } else {
            uint4 a0, a1;
            load_desc(a.mp_desc, o, a0, a1);
            const Window w = make_window(p, kd, sc.sf, sc.r0, sc.C, sc.R);
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
    PairRef e;
    e.pair = (int32_t)o;
    e.kp = bidx < 0 ? 0 : bidx;
    e.gp = gp;
    e.kf = 0;
    wave_append(is_add, &a.counters[kCtrAdd], a.add_list, a.add_cap, e);
}

__global__ __launch_bounds__(256) void resolve_plain_kernel(int32_t n_mp, const uint32_t* __restrict__ counters,
                                                          const PairRef* __restrict__ list, int32_t cap,
                                                          const int32_t* __restrict__ claim,
                                                          const int32_t* __restrict__ mp_id,
                                                          const int32_t* __restrict__ best_idx,
                                                          uint8_t* __restrict__ decision,
                                                          int32_t* __restrict__ target) {
    const uint32_t n = counters[kCtrAdd];
    const int stride = gridDim.x * blockDim.x;
    if (n <= (uint32_t)cap) {
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            const PairRef e = list[i];
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
