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
    a = ldg_u4(p);
    b = ldg_u4(p + 1);
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

// Closed box and octave gate, evaluated without branches.
__device__ __forceinline__ bool in_window(const Window& w, float x, float y, int oct, int pred, int gate) {
    const bool box = (x >= w.lx) & (x <= w.hx) & (y >= w.ly) & (y <= w.hy);
    const bool oct_ok = (gate == 0) | ((oct >= pred - 1) & (oct <= pred));
    return box & oct_ok;
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

// Workgroup exclusive scan of n_words packed pairs of 16-bit counts in place
// (low half first): word k becomes (P, P + lo) for P the sum of every count
// before it.  Every sum must stay below 65536.  Same shape as
// block_exclusive_scan.
__device__ void block_exclusive_scan_u16(uint32_t* w, int n, int32_t* s_tmp) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = wave_lane(), wid = tid / kWave, nw = nt / kWave;
    const int chunk = (n + nt - 1) / nt;
    const int b = min(tid * chunk, n), e = min(b + chunk, n);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += (int)(w[i] & 0xFFFFu) + (int)(w[i] >> 16);
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
    uint32_t run = (uint32_t)(s_tmp[wid] + incl - sum);
    for (int i = b; i < e; ++i) {
        const uint32_t x = w[i], lo = x & 0xFFFFu, hi = x >> 16;
        w[i] = run | ((run + lo) << 16);
        run += lo + hi;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Keyframe grid in LDS by octave group.  With the octave gate on, a pair
// whose point is predicted at octave p has as candidates the keypoints of
// octaves p - 1 and p; group g = min(p, nb - 1) holds exactly those
// keypoints for g < nb - 1, and the last group every octave from nb - 2 up,
// so a pair reads the cells of one group.  A keypoint of octave o therefore
// sits in up to two groups (o and o + 1 below nb - 1, the last group from
// o = nb - 2 up; octaves below -1 can never be candidates).  With nb = 1
// (the gate off, or too little LDS) group 0 is the plain grid of every
// keypoint.  Slots are ordered by row, then group, then column, so a pair's
// candidates are one run of slots per grid row.  Histogram of the (row,
// group, column) cells (16-bit counts, two per 32-bit word), exclusive scan,
// scatter of slot-ordered records (and descriptors), owner hash set.  On
// return s_cs[j] is the first slot of cell j and s_cs[R * nb * C] the
// number of slots (below 65536).  The order of the records inside a cell is
// arbitrary: the packed (distance, index) key makes every output
// independent of it.

// The groups of a keypoint of octave o: a (or -1) and b (or -1).
__device__ __forceinline__ void groups_of(int o, int nb, int& a, int& b) {
    if (nb == 1) {
        a = 0;
        b = -1;
        return;
    }
    a = (o >= 0 && o <= nb - 2) ? o : -1;
    b = (o + 1 >= 0 && o + 1 <= nb - 2) ? o + 1 : (o >= nb - 2 ? nb - 1 : -1);
}

// 16-bit entry j of a packed array, incremented; returns its old value.
__device__ __forceinline__ int u16_fetch_add(uint32_t* w, int j) {
    const int sh = (j & 1) * 16;
    return (int)((atomicAdd(&w[j >> 1], 1u << sh) >> sh) & 0xFFFFu);
}

template <bool STAGE_DESC>
__device__ void stage_keyframe(const BatchHdr& h, const KfDesc& kd, uint16_t* s_cs, KpRec* s_rec, uint4* s_desc,
                               int32_t* s_hash, int32_t* s_tmp) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n = kd.n_kp;
    const int C = h.grid_cols, R = h.grid_rows, nb = h.oct_buckets;
    const int entries = R * nb * C + 1;          // cell starts and the end
    const int words = (entries + 1) / 2;
    uint32_t* w = reinterpret_cast<uint32_t*>(s_cs);
    const int hmask = h.lds_hash_mask;
    const float* xy = h.kp_xy + 2 * (int64_t)kd.kp_off;
    for (int c = tid; c < words; c += nt) w[c] = 0;
    for (int s = tid; s <= hmask; s += nt) s_hash[s] = -1;
    __syncthreads();
    // cell of group g of keypoint i: (row * nb + g) * C + col
    for (int i = tid; i < n; i += nt) {
        const float x = xy[2 * i], y = xy[2 * i + 1];
        const int base = cell_of(y, kd.invh, R) * nb * C + cell_of(x, kd.invw, C);
        int ga, gb;
        groups_of((int)h.kp_oct[kd.kp_off + i], nb, ga, gb);
        if (ga >= 0) u16_fetch_add(w, base + ga * C + 1);
        if (gb >= 0) u16_fetch_add(w, base + gb * C + 1);
        const int32_t o = h.kp_owner[kd.kp_off + i];
        if (o >= 0) owner_insert(s_hash, hmask, o);
    }
    __syncthreads();
    block_exclusive_scan_u16(w, words, s_tmp);   // entry 1 + j = first slot of cell j
    for (int i = tid; i < n; i += nt) {
        const float x = xy[2 * i], y = xy[2 * i + 1];
        const int oct = (int)h.kp_oct[kd.kp_off + i];
        const int base = cell_of(y, kd.invh, R) * nb * C + cell_of(x, kd.invw, C);
        int ga, gb;
        groups_of(oct, nb, ga, gb);
        KpRec r;
        r.x = x;
        r.y = y;
        r.idx = i;
        r.oct = oct;
        uint4 d0 = make_uint4(0, 0, 0, 0), d1 = d0;
        if (STAGE_DESC && (ga >= 0 || gb >= 0)) {
            const uint4* src = reinterpret_cast<const uint4*>(h.kp_desc + 32 * ((int64_t)kd.kp_off + i));
            d0 = src[0];
            d1 = src[1];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int g = q ? gb : ga;
            if (g < 0) continue;
            const int slot = u16_fetch_add(w, base + g * C + 1);   // ends as the first slot of the next cell
            s_rec[slot] = r;
            if (STAGE_DESC) {
                s_desc[2 * slot] = d0;
                s_desc[2 * slot + 1] = d1;
            }
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
// of tiles (workgroups are dispatched to the 8 XCDs round-robin, and the runs
// of one XCD are neighbours in the tile order, so the keyframes of an XCD
// stay in its L2).  The workgroup's consecutive tiles of one keyframe
// descriptor form a segment.  When a segment's keyframe is not the one in
// LDS, the workgroup builds that keyframe's grid, records (and descriptors)
// and owner hash set in LDS; then its waves take the segment's pairs in
// chunks of 64 x PPL (pair j of a chunk on lane j mod 64), each wave on its
// own, with no barrier between chunks.  Provisional ADDs and accepted pairs
// go to the workgroup's own list regions through LDS counters; at the end of
// a segment its accepted pairs join their event's list with one device-scope
// reservation.  The ADD conflicts are resolved by the next kernel on the
// stream.

struct KfView {
    const int32_t* cs;          // global grid: cell starts (one bucket per cell)
    const uint16_t* cs16;       // LDS: octave-bucket starts
    int nb;                     // octave buckets per cell
    const KpRec* rec;
    const uint4* desc;          // cell-ordered descriptors (LDS or workspace), or null
    const uint8_t* desc_orig;   // keypoint descriptors by original index (when desc is null)
    const int32_t* own;         // unused: the owner of the best keypoint is read from kp_owner
    const int32_t* hash;
    int32_t hash_mask;
    int32_t n_rec;              // records (slots) in rec
};

// Bytes of the 16-bit octave-bucket starts in LDS (a whole number of 16-byte
// units).
__host__ __device__ inline size_t search_cs_bytes(int cells, int nb) {
    return ((size_t)cells * nb + 2 + 7) / 8 * 16;
}

// Record slots of a keyframe of kp_cap keypoints in nb octave groups (a
// keypoint sits in up to two groups when nb > 1).
__host__ __device__ inline int search_slots(int kp_cap, int nb) { return nb > 1 ? 2 * kp_cap : kp_cap; }

// LDS bytes of the search kernel (shared with the host).
__host__ __device__ inline size_t search_lds_bytes(int mode, int kp_cap, int cells, int hash_cap, int nb) {
    if (mode == kModeGlobal) return 16;
    const size_t slots = (size_t)search_slots(kp_cap, nb);
    size_t b = 16 * slots;   // records
    if (mode == kModeLdsDesc) b += 32 * slots;
    b += search_cs_bytes(cells, nb);
    b += 4 * (size_t)hash_cap;
    b += 4 * (size_t)(kSearchBlock / kWave + 4);
    return b;
}

// One pair's point, loaded before its evaluation (its descriptor is read
// only for the pair's candidates, when their distances are computed).
struct PairIn {
    int32_t gp, id;
    float x, y, z, dm;
    uint8_t dec;
};

__device__ __forceinline__ void load_pair(const BatchHdr& h, const KfDesc& kd, bool dense, int gate, int64_t o,
                                          int64_t se, PairIn& p) {
    p.dec = o < se ? kDecUndecided : (uint8_t)0;
    p.gp = 0;
    p.id = -1;
    p.x = p.y = p.z = p.dm = 0.0f;
    if (o < se) {
        const int64_t j = o - kd.pair_off;
        const int32_t lp = dense ? (int32_t)j : ldg(h.pair_mp + o);
        if (lp < 0 || lp >= kd.n_mp) {
            p.dec = FL_INVALID;
        } else {
            p.gp = kd.mp_off + lp;
            p.id = h.mp_id ? ldg(h.mp_id + p.gp) : p.gp;
            p.x = ldg(h.mp_xyz + 3 * (int64_t)p.gp);
            p.y = ldg(h.mp_xyz + 3 * (int64_t)p.gp + 1);
            p.z = ldg(h.mp_xyz + 3 * (int64_t)p.gp + 2);
            if (gate) p.dm = ldg(h.mp_dmax + p.gp);
        }
    }
}

// Search result of one pair beyond its decision.
struct PairRes {
    Best best;
    int32_t target;
    float ku, kv;   // the best candidate's keypoint
};

// The octave scale table sf[n] = scale_factor^n of a launch: its first
// kOctReg entries in registers, every entry in LDS; and the pass's window
// half-width at octave 0.
constexpr int kOctReg = 8;
struct OctaveTable {
    float sf[kOctReg];
    const float* all;   // LDS, n_octaves entries
    int N;
    float r0;
};

// The first n with d * sf[n] >= dmax, else N - 1 (the oracle's loop; the
// first kOctReg tests without branches).
__device__ __forceinline__ int predict_octave(const OctaveTable& T, float d, float dmax) {
    int pred = T.N - 1;
    bool found = false;
#pragma unroll
    for (int n = 0; n < kOctReg; ++n) {
        const bool hit = (!found) & (n < T.N) & (d * T.sf[n] >= dmax);
        pred = hit ? n : pred;
        found = found | hit;
    }
    if (!found)
        for (int n = kOctReg; n < T.N; ++n)
            if (d * T.all[n] >= dmax) {
                pred = n;
                break;
            }
    return pred;
}

// Window half-width r0 * sf[pred] (sf from LDS: a lane-dependent index into
// registers would be compiled as a table in scratch memory).
__device__ __forceinline__ float window_radius(const OctaveTable& T, int pred) { return T.r0 * T.all[pred]; }

// Evaluation of one pair (point p, keyframe kd) in three parts.  The front
// (per lane): observed-set test, Sim3 projection, predicted octave, window,
// and the runs of record slots to read: the window's grid rows of the pair's
// octave group (with the octave gate on, the group holds octaves pred - 1
// and pred only: a quarter of the window's keypoints when the eight octaves
// are equally common).  The scan (the whole wave together): every lane walks
// its runs as one flat sequence, testing box and octave; the records that
// pass go to a per-wave queue, and each time the queue fills (and at the end)
// the wave computes the queued Hamming distances one per lane, so the
// distance instructions run with their lanes full instead of with the few
// lanes that happen to have a candidate at one step.  Best and second best
// are kept per lane in LDS with atomic minima: the packed (distance, index)
// key of a candidate goes to the best slot, and whichever key the update
// leaves out (the old best, or the candidate) offers its distance to the
// second slot; so the second slot ends at the smallest distance of every
// candidate but the best, whatever the order.  The back (per lane): the
// fuse / add decision (provisional for ADD).  st: visible pairs, cells
// scanned, keypoints in them (every octave), candidates.
constexpr int kRowSeg = 4;
static_assert(kRowSeg == 4, "four row runs");

// What the front leaves for the scan of one pair.
struct PairScan {
    Window w;
    int pred, grp;
    int b0, d1, d2, d3, c1, c2, c3, total;   // slot = m + b0 + (d_j where m >= c_j)
    int nrows;
};

// Per wave: the candidate queue, each lane's best key and second distance,
// and the marks of the scan's item ranges (-1 between uses).
struct WaveCand {
    uint32_t q[kWave];        // owner lane << 17 | slot
    uint32_t best[kWave];
    uint32_t second[kWave];
    int32_t mark[kWave];
};
constexpr size_t kSearchStaticLds = sizeof(WaveCand) * kWavesPerWG + 1024;   // beside the dynamic LDS

template <int MODE, bool STATS>
__device__ __forceinline__ bool search_front(const KfDesc& kd, const KfView& v, const OctaveTable& T, int gate,
                                             int C, int R, PairIn& p, PairScan& q, unsigned long long* st) {
    q.total = 0;
    q.nrows = 0;
    // owner probe (a point already observed in this keyframe is skipped):
    // its first read is issued here and the probe finished after the
    // window, so its latency overlaps the projection
    const bool probe = p.dec == kDecUndecided && p.id >= 0;
    uint32_t hh = 0;
    int32_t hv = -1;
    if (probe) {
        hh = owner_slot(p.id, v.hash_mask);
        hv = v.hash[hh];
    }
    Proj pr{};
    const bool vis = p.dec == kDecUndecided && project_uv(kd, p.x, p.y, p.z, pr);
    q.pred = gate ? predict_octave(T, pr.d, p.dm) : T.N - 1;
    const float rad = window_radius(T, q.pred);
    Window& w = q.w;
    w.lx = pr.u - rad;
    w.hx = pr.u + rad;
    w.ly = pr.v - rad;
    w.hy = pr.v + rad;
    w.c0 = cell_of(w.lx, kd.invw, C);
    w.c1 = cell_of(w.hx, kd.invw, C);
    w.r0 = cell_of(w.ly, kd.invh, R);
    w.r1 = cell_of(w.hy, kd.invh, R);
    const int nb = MODE == kModeGlobal ? 1 : v.nb;
    auto cs_at = [&](int j) -> int { return MODE == kModeGlobal ? v.cs[j] : (int)v.cs16[j]; };
    q.grp = min(q.pred, nb - 1);
    q.nrows = w.r1 - w.r0 + 1;
    // the runs of the first kRowSeg rows (named values, not arrays: an array
    // indexed by a lane-dependent value would be placed in scratch memory)
    auto run = [&](int j, int c_in, int& b_out, int& c_out) {
        const bool in = j < q.nrows;
        const int idx = ((in ? w.r0 + j : w.r0) * nb + q.grp) * C;
        const int s0 = cs_at(idx + w.c0), e0 = cs_at(idx + w.c1 + 1);
        b_out = s0 - c_in;
        c_out = c_in + (in ? e0 - s0 : 0);
    };
    int b1, b2, b3;
    run(0, 0, q.b0, q.c1);
    run(1, q.c1, b1, q.c2);
    run(2, q.c2, b2, q.c3);
    run(3, q.c3, b3, q.total);
    q.d1 = b1 - q.b0;
    q.d2 = b2 - b1;
    q.d3 = b3 - b2;
    if (probe) {
        for (int n = 0; n <= v.hash_mask; ++n) {
            if (hv == p.id) {
                p.dec = FL_SKIP;
                break;
            }
            if (hv < 0) break;
            hh = (hh + 1) & (uint32_t)v.hash_mask;
            hv = v.hash[hh];
        }
    }
    // SKIP before NOT_VISIBLE; neither is searched
    if (p.dec == kDecUndecided && !vis) p.dec = FL_NOT_VISIBLE;
    if (p.dec != kDecUndecided) {
        q.total = 0;
        q.nrows = 0;
        return false;
    }
    if (STATS) {
        ++st[0];
        // cells and keypoints of the window's cells (every octave: the
        // counting launch stages one group)
        for (int row = w.r0; row <= w.r1; ++row) {
            st[1] += (unsigned long long)(w.c1 - w.c0 + 1);
            for (int g = 0; g < nb; ++g) {
                const int j = (row * nb + g) * C;
                st[2] += (unsigned long long)(cs_at(j + w.c1 + 1) - cs_at(j + w.c0));
            }
        }
    }
    return true;
}

__device__ __forceinline__ int scan_slot(const PairScan& q, int m) {
    // masks, not a chain of selects, which the compiler would turn into a
    // table in scratch memory
    return m + q.b0 + (q.d1 & -(int)(m >= q.c1)) + (q.d2 & -(int)(m >= q.c2)) + (q.d3 & -(int)(m >= q.c3));
}

// Descriptor of record slot i (keypoint index idx).
template <int MODE>
__device__ __forceinline__ void record_desc(const KfView& v, int i, int idx, uint4& b0, uint4& b1) {
    if (MODE == kModeLdsRec) {
        load_desc(v.desc_orig, idx, b0, b1);
    } else if (MODE == kModeLdsDesc) {
        b0 = v.desc[2 * i];
        b1 = v.desc[2 * i + 1];
    } else {
        b0 = ldg_u4(v.desc + 2 * i);
        b1 = ldg_u4(v.desc + 2 * i + 1);
    }
}

// A candidate of key k for the pair of `owner`: the atomic-minimum update of
// its best and second slots (see above).
__device__ __forceinline__ void offer_lds(WaveCand& wc, int owner, uint32_t k) {
    const uint32_t old = atomicMin(&wc.best[owner], k);
    const uint32_t out = k < old ? old : k;
    if (out != 0xFFFFFFFFu) atomicMin(&wc.second[owner], out >> 16);
}

// The queued candidates, one per lane: the owner's point descriptor (its
// point index from the owner lane) against the keypoint's.  Every lane of
// the wave takes part in the cross-lane read.
template <int MODE>
__device__ __forceinline__ void drain_queue(WaveCand& wc, int qn, const KfView& v, const uint8_t* mp_desc,
                                            int32_t gp) {
    const int lane = wave_lane();
    const uint32_t e = lane < qn ? wc.q[lane] : 0u;
    const int owner = (int)(e >> 17);
    const int32_t ogp = __builtin_amdgcn_ds_bpermute(owner << 2, gp);
    if (lane < qn) {
        const int slot = (int)(e & 0x1FFFFu);
        const int idx = v.rec[slot].idx;
        uint4 a0, a1, b0, b1;
        load_desc(mp_desc, ogp, a0, a1);
        record_desc<MODE>(v, slot, idx, b0, b1);
        offer_lds(wc, owner, ((uint32_t)hamming(a0, a1, b0, b1) << 16) | (uint32_t)idx);
    }
}

// The wave's scan of its lanes' pairs (every lane of the wave calls it; a
// lane with no pair to search has q.total = 0 and q.nrows = 0).  The records
// of the lanes' runs form one sequence of items, lane after lane (lane l's
// q.total items from P_l, the exclusive prefix sum of the totals), taken 64
// at a time, one per lane: a wave makes ceil(N / 64) steps for its N items
// instead of as many as its busiest lane has records.  Lane l marks where its
// items start; the owner of an item is the last mark at or before it, and
// the owner's window and run layout come from the owner lane.
template <int MODE, bool STATS>
__device__ __forceinline__ void search_scan(const KfView& v, int gate, int C, const uint8_t* mp_desc,
                                            const PairIn& p, const PairScan& q, WaveCand& wc,
                                            unsigned long long* st) {
    const int lane = wave_lane();
    wc.best[lane] = 0xFFFFFFFFu;
    wc.second[lane] = FL_NO_DIST;
    int qn = 0;
    const int L = q.total;
    const int incl = wave_incl_scan(L);
    const int P = incl - L;
    const int N = __builtin_amdgcn_readlane(incl, kWave - 1);
    // item k of this lane (P <= k < P + L) is record slot
    // k + B + (d1 if k >= A1) + (d2 if k >= A2) + (d3 if k >= A3)
    const int B = q.b0 - P, A1 = P + q.c1, A2 = P + q.c2, A3 = P + q.c3;
    const float lx = q.w.lx, hx = q.w.hx, ly = q.w.ly, hy = q.w.hy;
    int cur = 0;   // owner of the step's first item when no range starts there
    for (int base = 0; base < N; base += kWave) {
        // (one wave's LDS accesses complete in order: the read below sees
        // the marks, and the reset follows the read)
        if (L > 0 && P >= base && P < base + kWave) wc.mark[P - base] = lane;
        int mk = wc.mark[lane];
        wc.mark[lane] = -1;
        if (lane == 0 && mk < 0) mk = cur;
        const unsigned long long starts = __ballot(mk >= 0);   // bit 0 always set
        const unsigned long long upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
        const int pos = 63 - __builtin_clzll(starts & upto);
        const int o = __shfl(mk, pos);   // owner lane of item base + lane
        cur = __builtin_amdgcn_readlane(o, kWave - 1);
        const int k = base + lane;
        const bool act = k < N;
        const int oB = __shfl(B, o), oA1 = __shfl(A1, o), oA2 = __shfl(A2, o), oA3 = __shfl(A3, o);
        const int od1 = __shfl(q.d1, o), od2 = __shfl(q.d2, o), od3 = __shfl(q.d3, o);
        Window w;
        w.lx = __shfl(lx, o);
        w.hx = __shfl(hx, o);
        w.ly = __shfl(ly, o);
        w.hy = __shfl(hy, o);
        const int opred = __shfl(q.pred, o);
        const int i = k + oB + (od1 & -(int)(k >= oA1)) + (od2 & -(int)(k >= oA2)) + (od3 & -(int)(k >= oA3));
        KpRec rc{};
        if (act) rc = v.rec[min((unsigned)i, (unsigned)(v.n_rec - 1))];   // (in range by construction)
        const bool cand = act && in_window(w, rc.x, rc.y, rc.oct, opred, gate);
        const unsigned long long cm = __ballot(cand);
        if (cm) {
            const int n = __popcll(cm);
            if (qn + n > kWave) {
                drain_queue<MODE>(wc, qn, v, mp_desc, p.gp);
                qn = 0;
            }
            if (cand) {
                wc.q[qn + __popcll(cm & ((1ull << lane) - 1ull))] = ((uint32_t)o << 17) | (uint32_t)i;
                if (STATS) ++st[3];
            }
            qn += n;
        }
    }
    if (qn) drain_queue<MODE>(wc, qn, v, mp_desc, p.gp);
    // rows beyond the first kRowSeg (wide windows): each lane its own, the
    // distances computed on the spot
    if (q.nrows > kRowSeg) {
        const int nb = MODE == kModeGlobal ? 1 : v.nb;
        uint4 a0, a1;
        load_desc(mp_desc, p.gp, a0, a1);
        for (int row = q.w.r0 + kRowSeg; row <= q.w.r1; ++row) {
            const int j = (row * nb + q.grp) * C;
            const int s0 = MODE == kModeGlobal ? v.cs[j + q.w.c0] : (int)v.cs16[j + q.w.c0];
            const int e0 = MODE == kModeGlobal ? v.cs[j + q.w.c1 + 1] : (int)v.cs16[j + q.w.c1 + 1];
            for (int i = s0; i < e0; ++i) {
                const KpRec rc = v.rec[i];
                if (!in_window(q.w, rc.x, rc.y, rc.oct, q.pred, gate)) continue;
                if (STATS) ++st[3];
                uint4 b0, b1;
                record_desc<MODE>(v, i, rc.idx, b0, b1);
                offer_lds(wc, lane, ((uint32_t)hamming(a0, a1, b0, b1) << 16) | (uint32_t)rc.idx);
            }
        }
    }
}

// The decision of a searched pair from its best and second.
__device__ __forceinline__ void search_back(const KfDesc& kd, int hamming_th, float nn_ratio,
                                            const int32_t* kp_owner, PairIn& p, PairRes& res) {
    if (!accept_match(res.best, hamming_th, nn_ratio)) {
        p.dec = FL_NO_MATCH;
    } else {
        const int32_t ow = ldg(kp_owner + kd.kp_off + (int32_t)(res.best.key & 0xFFFFu));
        if (ow >= 0) {
            p.dec = FL_FUSE;
            res.target = ow;
        } else {
            p.dec = FL_ADD;   // provisional; losers are relabelled by the resolver
        }
    }
}

template <int PPL, int MODE, bool STATS>
__global__ __launch_bounds__(kSearchBlock) void search_fused_kernel(const BatchHdr* __restrict__ hp) {
    extern __shared__ __align__(16) unsigned char s_mem[];
    const BatchHdr& h = *hp;
    const int tid = threadIdx.x;
    const int lane = wave_lane();
    KpRec* s_rec = reinterpret_cast<KpRec*>(s_mem);
    uint4* s_desc = nullptr;
    uint16_t* s_cs = nullptr;
    int32_t* s_hash = nullptr;
    int32_t* s_tmp = nullptr;
    // running counts of the workgroup's ADD and accepted-pair regions, then
    // the segment's accepted-pair total and its base in the event's list
    __shared__ uint32_t s_list[4];
    __shared__ WaveCand s_wc[kWavesPerWG];   // each wave's candidate queue, best and second
    const int wid = tid / kWave, nw = (int)(blockDim.x / kWave);
    if (MODE != kModeGlobal) {
        const size_t slots = (size_t)search_slots(h.lds_kp_cap, h.oct_buckets);
        unsigned char* p = s_mem + 16 * slots;
        if (MODE == kModeLdsDesc) {
            s_desc = reinterpret_cast<uint4*>(p);
            p += 32 * slots;
        }
        s_cs = reinterpret_cast<uint16_t*>(p);
        p += search_cs_bytes(h.cells, h.oct_buckets);
        s_hash = reinterpret_cast<int32_t*>(p);
        p += 4 * (size_t)(h.lds_hash_mask + 1);
        s_tmp = reinterpret_cast<int32_t*>(p);
        p += 4 * (size_t)(kSearchBlock / kWave + 4);
    }
    if (tid == 0) {
        s_list[0] = 0;
        s_list[1] = 0;
    }
    s_wc[tid / kWave].mark[lane] = -1;

    // the octave scale table in LDS: the octave search and the window radius
    // index it per lane.  In the LDS modes the barrier that opens the first
    // keyframe's staging publishes it (and the counters above), so the first
    // point loads are issued without waiting here.
    __shared__ float s_sf[FL_MAX_OCTAVES];
    if (tid < FL_MAX_OCTAVES) s_sf[tid] = h.sf[tid];
    if (MODE == kModeGlobal) __syncthreads();
    OctaveTable T;
    T.all = s_sf;
    T.N = h.n_octaves;
#pragma unroll
    for (int n = 0; n < kOctReg; ++n) T.sf[n] = uniform_f(h.sf[n]);
    T.N = uniform_i(T.N);
    const int gate = uniform_i(h.gate), C = uniform_i(h.grid_cols), R = uniform_i(h.grid_rows);
    const bool dense = uniform_i(h.dense) != 0;
    const bool want_matches = uniform_i(h.refine_iters) > 0;
    const unsigned long long tag = (unsigned long long)(uint32_t)uniform_i((int32_t)*h.epoch) << 32;
    // header fields read per pair, held in scalar registers (the output
    // stores below could otherwise be taken to alias the header)
    const int32_t* const kp_owner = uniform_p(h.kp_owner);
    const float* const kp_xy = uniform_p(h.kp_xy);
    const uint8_t* const mp_desc = uniform_p(h.mp_desc);
    unsigned long long* const claim = uniform_p(h.claim);
    AddRef* const add_list = uniform_p(h.add_list);
    MatchRec* const match_stage = uniform_p(h.match_stage);
    unsigned long long st[4] = {0, 0, 0, 0};

    // The range and the keyframe table sit at offsets of the table blob that
    // follow from the grid size, so neither waits for a pointer.
    const char* blob = reinterpret_cast<const char*>(hp);
    const WgRange rg = reinterpret_cast<const WgRange*>(blob + blob_range_offset())[blockIdx.x];
    const KfDesc* kf_tab = reinterpret_cast<const KfDesc*>(blob + blob_kf_offset((int)gridDim.x));
    int slot = rg.slot;
    int staged = -1;
    uint32_t seg_m0 = 0;   // first staged accepted pair of the current segment
    for (int t = rg.t0; t < rg.t1;) {
        while (t >= h.tile_prefix[slot + 1]) ++slot;
        const int k = t == rg.t0 ? rg.kf : h.kf_order[slot];
        const int tb = h.tile_prefix[slot];
        const int t_end = min(rg.t1, h.tile_prefix[slot + 1]);
        const KfDesc kd = uniform_kf(kf_tab[k]);   // scalar registers, kept across the stores below
        PassOut po = h.out[kd.pass];
        po.best_idx = uniform_p(po.best_idx);
        po.best_dist = uniform_p(po.best_dist);
        po.second_dist = uniform_p(po.second_dist);
        po.decision = uniform_p(po.decision);
        po.target = uniform_p(po.target);
        po.hamming_th = uniform_i(po.hamming_th);
        po.nn_ratio = uniform_f(po.nn_ratio);
        po.r0 = uniform_f(po.r0);
        T.r0 = po.r0;
        const int64_t kend = kd.pair_off + kd.n_pairs;
        const int64_t sb = kd.pair_off + (int64_t)(t - tb) * kd.tile_pairs;
        const int64_t se = min(kd.pair_off + (int64_t)(t_end - tb) * kd.tile_pairs, kend);
        t = t_end;

        KfView v;
        if (MODE == kModeGlobal) {
            v.cs = h.cell_start + kd.grid_off;
            v.cs16 = nullptr;
            v.nb = 1;
            v.rec = h.recs + kd.kp_off;
            v.n_rec = max(kd.n_kp, 1);
            v.desc = h.desc_sorted + 2 * (int64_t)kd.kp_off;
            v.desc_orig = nullptr;
            v.own = nullptr;
            v.hash = h.hash + kd.hash_off;
            v.hash_mask = kd.hash_mask;
        } else {
            if (staged != kd.stage_key) {
                __syncthreads();   // every reader of the previous keyframe is done
                stage_keyframe<MODE == kModeLdsDesc>(h, kd, s_cs, s_rec, s_desc, s_hash, s_tmp);
                staged = kd.stage_key;
            }
            v.cs = nullptr;
            v.cs16 = s_cs;
            v.nb = uniform_i(h.oct_buckets);
            v.rec = s_rec;
            v.n_rec = search_slots(uniform_i(h.lds_kp_cap), uniform_i(h.oct_buckets));
            v.desc = MODE == kModeLdsDesc ? s_desc : nullptr;
            v.desc_orig = h.kp_desc + 32 * (int64_t)kd.kp_off;
            v.own = nullptr;
            v.hash = s_hash;
            v.hash_mask = h.lds_hash_mask;
        }

        constexpr int kChunk = kWave * PPL;
        const int64_t n_chunks = (se - sb + kChunk - 1) / kChunk;
        const unsigned long long below = (1ull << lane) - 1ull;
        // The points of a wave's next chunk are loaded while its current
        // chunk is evaluated (their latency overlaps the evaluation).
        PairIn pn[PPL];
        if (wid < n_chunks) {
#pragma unroll
            for (int r = 0; r < PPL; ++r)
                load_pair(h, kd, dense, gate, sb + wid * kChunk + r * kWave + lane, se, pn[r]);
        }
        for (int64_t c = wid; c < n_chunks; c += nw) {
            const int64_t cb = sb + c * kChunk;
            PairIn p[PPL];
#pragma unroll
            for (int r = 0; r < PPL; ++r) p[r] = pn[r];
            if (c + nw < n_chunks) {
#pragma unroll
                for (int r = 0; r < PPL; ++r)
                    load_pair(h, kd, dense, gate, cb + nw * kChunk + r * kWave + lane, se, pn[r]);
            }
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                const int64_t o = cb + r * kWave + lane;
                const bool active = o < se;
                PairRes res;
                res.target = -1;
                res.ku = res.kv = 0.0f;
                PairScan sq;
                const bool searching = search_front<MODE, STATS>(kd, v, T, gate, C, R, p[r], sq, st);
                WaveCand& wc = s_wc[wid];
                search_scan<MODE, STATS>(v, gate, C, mp_desc, p[r], sq, wc, st);
                res.best.key = wc.best[lane];
                res.best.second = (int)wc.second[lane];
                if (searching) search_back(kd, po.hamming_th, po.nn_ratio, kp_owner, p[r], res);
                const uint32_t key = res.best.key;
                const int bidx = key == 0xFFFFFFFFu ? -1 : (int)(key & 0xFFFFu);
                const int kpg = kd.claim_off + (bidx < 0 ? 0 : bidx);   // claim slot
                if (active) {
                    stg(po.best_idx + o, (int32_t)bidx);
                    stg(po.best_dist + o, (int16_t)(key == 0xFFFFFFFFu ? FL_NO_DIST : (int)(key >> 16)));
                    stg(po.second_dist + o, (int16_t)res.best.second);
                    stg(po.decision + o, p[r].dec);
                    stg(po.target + o, res.target);
                }
                const bool is_add = active && p[r].dec == FL_ADD;
                const bool acc = want_matches && active && (p[r].dec == FL_ADD || p[r].dec == FL_FUSE);
                if (is_add)
                    __hip_atomic_fetch_min((gmem<unsigned long long>*)(claim + kpg),
                                           tag | (uint32_t)p[r].gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // one LDS reservation per wave and list
                const unsigned long long ma = __ballot(is_add), mm = __ballot(acc);
                uint32_t ba = 0, bm = 0;
                if (lane == 0) {
                    if (ma) ba = atomicAdd(&s_list[0], (uint32_t)__popcll(ma));
                    if (mm) bm = atomicAdd(&s_list[1], (uint32_t)__popcll(mm));
                }
                ba = (uint32_t)__shfl((int)ba, 0);
                bm = (uint32_t)__shfl((int)bm, 0);
                if (is_add) {
                    AddRef e;
                    e.pair = (int32_t)o;
                    e.kp = kpg;
                    e.gp = p[r].gp;
                    e.pass = kd.pass;
                    stg_rec(add_list + rg.priv_off + ba + (uint32_t)__popcll(ma & below), e);
                }
                if (acc) {
                    // the matched keypoint's observation
                    const int64_t kg = (int64_t)kd.kp_off + bidx;
                    MatchRec me;
                    me.x = p[r].x;
                    me.y = p[r].y;
                    me.z = p[r].z;
                    me.u = ldg(kp_xy + 2 * kg);
                    me.v = ldg(kp_xy + 2 * kg + 1);
                    me.kf = k;
                    me.pad0 = me.pad1 = 0;
                    stg_rec(match_stage + rg.priv_off + bm + (uint32_t)__popcll(mm & below), me);
                }
            }
        }
        if (want_matches) {
            // the segment's accepted pairs join their event's list
            __syncthreads();
            if (tid == 0) {
                const uint32_t tot = s_list[1];
                s_list[2] = tot;
                s_list[3] = tot > seg_m0 ? atomicAdd(&h.ev_ctr[kd.event * kEvCtrs + kEvMatch], tot - seg_m0) : 0u;
            }
            __syncthreads();
            const uint32_t tot = s_list[2], base = s_list[3];
            const EventDesc& ed = h.ev[kd.event];
            const int32_t list_off = ed.list_off, list_cap = ed.list_cap;
            for (uint32_t i = seg_m0 + tid; i < tot; i += blockDim.x) {
                const uint32_t idx = base + (i - seg_m0);
                if (idx < (uint32_t)list_cap) h.match_list[list_off + idx] = h.match_stage[rg.priv_off + i];
            }
            seg_m0 = tot;
        }
    }
    __syncthreads();   // every ADD of the workgroup is counted
    if (tid == 0) h.add_count[blockIdx.x] = s_list[0];
    if (STATS) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            unsigned long long xv = st[i];
            for (int off = 32; off > 0; off >>= 1) xv += __shfl_xor(xv, off);
            if (lane == 0 && xv) atomicAdd(&h.stats_out[i], xv);
        }
    }
}

// ADD resolution after a batched search launched without refinement: the
// search workgroups' ADD regions, grid-stride.
constexpr int kResolveBlock = 256;
constexpr int kResolveGrid = 1024;   // workgroups in graph mode (any count is correct)

__global__ __launch_bounds__(kResolveBlock) void resolve_adds_kernel(const BatchHdr* __restrict__ hp) {
    const BatchHdr& h = *hp;
    const unsigned long long tag = (unsigned long long)(*h.epoch) << 32;
    for (int r = blockIdx.x; r < h.n_wg; r += gridDim.x) resolve_region_adds(h, r, tag);
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
    e.pass = 0;
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
