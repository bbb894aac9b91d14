// Internal layouts and device helpers of the fastloop library (gfx950).
//
// The batch descriptor lives in device memory (uploaded once per call from a
// pinned staging buffer); every kernel takes only a pointer to it, so one
// captured HIP graph serves batches of any size up to the workspace capacity.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastloop.h"

namespace fl {

constexpr int kWave = 64;
constexpr int kMaxQueues = 8;        // one work queue per XCD
constexpr int kNAccPad = 36;        // doubles per partial of a float64 reduction

// One keyframe of a batch: search transform, camera, grid and ranges.
struct alignas(16) KfDesc {
    float A[9];          // sR, row-major
    float t[3];
    float inv_s;
    float fx, fy, cx, cy, W, H;
    float invw, invh;    // grid_cols / W, grid_rows / H (float32, rounded once)
    float T[12];         // world->camera SE3 for refinement (R row-major, t)
    int32_t kp_off;      // first keypoint (global index)
    int32_t n_kp;
    int32_t grid_off;    // first cell_start entry (global-grid mode)
    int32_t event;
    int32_t mp_off;      // first point of the event (global index)
    int32_t n_mp;        // points in the event
    int32_t hash_off;    // owner hash table of this keyframe (global-grid mode)
    int32_t hash_mask;
    int32_t n_tiles;
    int32_t pad0, pad2;
    int32_t tile_pairs;  // pairs per tile of this keyframe (a whole number of waves)
    int64_t pair_off;
    int64_t n_pairs;
    // A launch may search its batch several times (passes); each (keyframe,
    // pass) has a descriptor of its own, keyframe-major.
    int32_t pass;        // thresholds and outputs: BatchHdr::out[pass]
    int32_t stage_key;   // the keyframe in the batch (its grid is the same in every pass)
    int32_t claim_off;   // first ADD claim slot: pass * n_kp_total + kp_off
    int32_t pad1;
};

// One search pass of a launch: its thresholds and its outputs (caller-owned).
struct PassOut {
    int32_t* best_idx;
    int16_t* best_dist;
    int16_t* second_dist;
    uint8_t* decision;
    int32_t* target;
    int32_t hamming_th;
    float nn_ratio;
    float r0;            // window half-width at octave 0, pixels
    int32_t pad;
};

struct alignas(16) EventDesc {
    int32_t kf_begin, kf_end;
    int32_t mp_off, n_mp;
    int32_t list_off, list_cap;    // region of the matched-pair list
    int64_t pair_begin, pair_end;  // pair range (pairs of the event are contiguous)
    int32_t inv_off, inv_n;        // the event's pairs of the other direction (two-sided refinement)
    int32_t pad0, pad1;
};

// Offsets in the table blob (which starts at the batch header) of the
// workgroups' tile ranges and of the keyframe table: fixed by the header size
// and the search grid, so a workgroup finds its range and first keyframe
// without first loading pointers.
constexpr size_t kBlobAlign = 256;
__host__ __device__ constexpr size_t blob_align(size_t x) { return (x + kBlobAlign - 1) / kBlobAlign * kBlobAlign; }

// Provisional ADD: a pair whose point claimed a free keypoint.
struct alignas(16) AddRef {
    int32_t pair;     // global pair index
    int32_t kp;       // claim slot of the keypoint (KfDesc::claim_off + index)
    int32_t gp;       // global point index
    int32_t pass;     // search pass (its outputs)
};

// The share of the search launch of one workgroup: tiles [t0, t1) of the
// tile order, the slot of tile t0 and its keyframe descriptor, and the
// workgroup's region of the provisional-ADD and accepted-pair staging lists:
// entries [priv_off, priv_off + priv_cap), as many as the pairs it searches
// (each pair adds at most one entry to each list).
struct alignas(16) WgRange {
    int32_t t0, t1, slot, kf;
    int32_t priv_off, priv_cap, pad0, pad1;
};

// Accepted pair kept for refinement: point, observation, keyframe.
struct alignas(16) MatchRec {
    float x, y, z;
    float u, v;
    int32_t kf;
    int32_t pad0, pad1;
};

// Cell-ordered keypoint record: 16 bytes, one dwordx4 load.  idx is the
// keypoint index within its keyframe.
struct alignas(16) KpRec {
    float x, y;
    int32_t idx;
    int32_t oct;
};

// Per-event counters (the accepted-pair count, zero between launches: the
// refinement that reads the list resets it).  Each event's counters sit on a
// 128-byte line of their own: device-scope atomics on one line serialise
// (about 12 ns apiece).
enum : int { kEvMatch = 0, kEvCtrs = 32 };

enum : int { kModeGlobal = 0, kModeLdsRec = 1, kModeLdsDesc = 2 };

struct alignas(16) BatchHdr {
    int32_t n_events, n_kf, n_mp, n_kp_total;
    int64_t n_pairs;
    int32_t n_tiles, tile_cap;   // tiles of the batch; the largest tile (workgroup size x pairs per lane)
    int32_t cells, grid_cols, grid_rows, n_octaves;
    int32_t n_pass;             // search passes of the launch (1 .. FL_MAX_PASSES)
    int32_t gate;               // 1: point distance invariance given (octave gate on)
    int32_t dense;
    int32_t stats;              // 1: count visible / cells / keypoints / candidates
    uint32_t pad_epoch;
    int32_t lds_hash_mask;      // owner hash capacity - 1 in the LDS modes
    int32_t n_wg;               // workgroups of the search launch
    int32_t refine_iters;       // evaluations per round
    float huber_delta;
    int32_t refine_rounds;      // >= 1; rounds after the first keep the pairs within outlier_px
    float outlier_px;
    float lm_lambda;            // > 0: Levenberg-Marquardt from this damping; 0: Gauss-Newton
    int32_t pad_refine;
    int32_t refine_blocks;      // blocks per event
    int32_t refine_scan;        // 1: take accepted pairs from the decisions, not the list
    int32_t resolve_in_refine;  // 1: the refinement kernel resolves the search's ADD conflicts
    int32_t lds_kp_cap;         // keypoint capacity of the LDS records in the LDS modes
    int32_t oct_buckets;        // octave buckets per grid cell in the LDS modes (1 .. 8)
    int32_t pad_buckets[3];
    float sf[32];               // scale_factor^n rounded to float32
    // tables in the uploaded blob
    const KfDesc* kf;
    const EventDesc* ev;
    const int32_t* kf_order;    // keyframes in tile order
    const int32_t* tile_prefix; // [n_kf+1] first tile of each keyframe in tile order
    const WgRange* wg_range;    // [n_wg] each workgroup's tiles and list regions
    // inputs (caller-owned)
    const float* kp_xy;
    const int8_t* kp_oct;
    const uint8_t* kp_desc;
    const int32_t* kp_owner;
    const float* mp_xyz;
    const uint8_t* mp_desc;
    const float* mp_dmax;
    const int32_t* mp_id;
    const int32_t* pair_mp;
    // thresholds and outputs of each pass
    PassOut out[FL_MAX_PASSES];
    // workspace (library-owned)
    int32_t* cell_start;        // global-grid mode: [n_kf * (cells + 1)]
    KpRec* recs;                // global-grid mode: [n_kp_total]
    uint4* desc_sorted;         // global-grid mode: [n_kp_total * 2]
    int32_t* cell_kp;           // global-grid mode: [n_kp_total]
    int32_t* hash;              // global-grid mode: owner hash tables
    unsigned long long* claim;  // [n_pass * n_kp_total] (epoch << 32 | lowest claiming point)
    const uint32_t* epoch;      // tag of this launch's claims, decremented by the table fetch
    uint32_t* ev_ctr;           // [n_events * kEvCtrs]
    AddRef* add_list;           // per-workgroup regions (WgRange::priv_off)
    uint32_t* add_count;        // [n_wg] entries of each workgroup's ADD region
    MatchRec* match_stage;      // per-workgroup regions of accepted pairs, before they join their event's list
    MatchRec* match_list;       // per-event regions
    unsigned long long* stats_out;  // [4]
    // refinement
    double* event_S;            // [n_events][13] caller's, in/out
    fl_sim3* event_S32_out;     // caller's (may be null)
    int32_t* event_n_matched;   // caller's (may be null)
    unsigned long long* refine_rows;   // [2][n_events * refine_blocks][2 * kNAccPad] tagged partial-sum words
    // two-sided refinement (caller's; null without it): points of the other
    // side observed through S^-1 in keyframes of their own
    const float* inv_xyz;       // [n][3]
    const float* inv_uv;        // [n][2]
    const int32_t* inv_kf;      // [n] into inv_T / inv_cam
    const float* inv_T;         // [inv_n_kf][12]
    const float* inv_cam;       // [inv_n_kf][4] fx, fy, cx, cy
    int32_t inv_n_kf;
    int32_t pad_inv[3];
};

__host__ __device__ constexpr size_t blob_range_offset() { return blob_align(sizeof(BatchHdr)); }
__host__ __device__ constexpr size_t blob_kf_offset(int grid) {
    return blob_align(blob_range_offset() + sizeof(WgRange) * (size_t)(grid > 1 ? grid : 1));
}


// ---------------------------------------------------------------------------
// float32 helpers whose rounding is fixed: every multiply-add written as
// fmaf is one fused operation, every other operation rounds on its own (the
// library is compiled with -ffp-contract=off).

// floor(x * inv) clamped to [0, n): a negative or NaN product gives cell 0.
// Branch free: fmaxf returns its other operand for a NaN, and floor of a
// product below n is at most n - 1.
__device__ __forceinline__ int cell_of(float x, float inv, int n) {
    const float f = floorf(x * inv);
    return (int)fminf(fmaxf(f, 0.0f), (float)(n - 1));
}

struct Proj {
    float u, v, d;
    int pred;
};

// Transform by the keyframe's Sim3, pinhole projection and image test:
// false when the point is not visible; u, v and the metric distance d
// otherwise.
__device__ __forceinline__ bool project_uv(const KfDesc& k, float x, float y, float z, Proj& p) {
    const float q0 = fmaf(k.A[2], z, fmaf(k.A[1], y, fmaf(k.A[0], x, k.t[0])));
    const float q1 = fmaf(k.A[5], z, fmaf(k.A[4], y, fmaf(k.A[3], x, k.t[1])));
    const float q2 = fmaf(k.A[8], z, fmaf(k.A[7], y, fmaf(k.A[6], x, k.t[2])));
    if (!(q2 > 0.0f)) return false;
    const float iz = 1.0f / q2;
    const float u = fmaf(k.fx, q0 * iz, k.cx);
    const float v = fmaf(k.fy, q1 * iz, k.cy);
    if (!(u >= 0.0f && u < k.W && v >= 0.0f && v < k.H)) return false;
    p.u = u;
    p.v = v;
    p.d = sqrtf(fmaf(q0, q0, fmaf(q1, q1, q2 * q2))) * k.inv_s;
    return true;
}

// Transform, projection, image test and predicted octave: the first n with
// d * sf[n] >= dmax, else N - 1 (gate off: N - 1).
__device__ __forceinline__ bool project(const KfDesc& k, float x, float y, float z, float dmax, int gate,
                                        const float* sf, int N, Proj& p) {
    if (!project_uv(k, x, y, z, p)) return false;
    int pred = N - 1;
    if (gate) {
        for (int n = 0; n < N; ++n) {
            if (p.d * sf[n] >= dmax) { pred = n; break; }
        }
    }
    p.pred = pred;
    return true;
}

__device__ __forceinline__ int hamming(const uint4& a0, const uint4& a1, const uint4& b0, const uint4& b1) {
    int h = __popc(a0.x ^ b0.x);
    h += __popc(a0.y ^ b0.y);
    h += __popc(a0.z ^ b0.z);
    h += __popc(a0.w ^ b0.w);
    h += __popc(a1.x ^ b1.x);
    h += __popc(a1.y ^ b1.y);
    h += __popc(a1.z ^ b1.z);
    h += __popc(a1.w ^ b1.w);
    return h;
}

// Running best / second best over packed keys (h << 16 | idx): the minimum
// key is the lexicographic minimum of (distance, keypoint index), so the
// result does not depend on the order candidates are visited in.
struct Best {
    uint32_t key;   // 0xFFFFFFFF: none
    int second;     // FL_NO_DIST: none
    __device__ __forceinline__ void init() {
        key = 0xFFFFFFFFu;
        second = FL_NO_DIST;
    }
    __device__ __forceinline__ void offer(int h, int idx) {
        const uint32_t k = ((uint32_t)h << 16) | (uint32_t)idx;
        if (k < key) {
            if (key != 0xFFFFFFFFu) second = min(second, (int)(key >> 16));
            key = k;
        } else {
            second = min(second, h);
        }
    }
};

__device__ __forceinline__ uint32_t hash_id(int32_t id) {
    return (uint32_t)id * 0x9E3779B1u;
}

// Is `id` among the owners stored in a keyframe's open-addressing table?
__device__ __forceinline__ bool owner_lookup(const int32_t* __restrict__ table, int32_t mask, int32_t id) {
    if (id < 0) return false;
    uint32_t h = (hash_id(id) >> 7) & (uint32_t)mask;
    for (int probe = 0; probe <= mask; ++probe) {
        const int32_t v = table[h];
        if (v == id) return true;
        if (v < 0) return false;
        h = (h + 1) & (uint32_t)mask;
    }
    return false;
}

// Tag of the refinement's partial-sum words: the low kTagEpochBits bits of
// the launch epoch (decremented by every table fetch) above ten bits of
// step number (step + 1 < 1024).  Tags repeat every 2^kTagEpochBits
// launches, so the host zeroes the partial-sum rows before every launch
// whose count is a multiple of that period (refine_rows_cleared_before):
// between two clears no two launches share a tag, and a zeroed word (tag 0)
// matches none.
constexpr uint32_t kTagEpochBits = 22;
__host__ __device__ constexpr uint32_t refine_tag(uint32_t epoch, int step) {
    return (epoch << 10) | (uint32_t)(step + 1);
}
__host__ __device__ constexpr bool refine_rows_cleared_before(uint32_t launches) {
    return (launches & ((1u << kTagEpochBits) - 1u)) == 0u;
}

__device__ __forceinline__ int wave_lane() { return threadIdx.x & (kWave - 1); }

// Global-memory accesses through the global address space: the compiler
// then issues global (not flat) loads and stores, with a scalar base where
// it can.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const gmem<T>*)p;   // address-space cast: generic to global
}
template <typename T>
__device__ __forceinline__ void stg(T* p, const T& v) {
    *(gmem<T>*)p = v;
}
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ldg_u4(const uint4* p) {
    const v4u x = *(const gmem<v4u>*)p;
    return make_uint4(x.x, x.y, x.z, x.w);
}
// A record of n 16-byte units stored with n dwordx4 global stores.
template <typename T>
__device__ __forceinline__ void stg_rec(T* p, const T& v) {
    static_assert(sizeof(T) % 16 == 0, "whole 16-byte units");
    const v4u* src = reinterpret_cast<const v4u*>(&v);
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 16; ++i) ((gmem<v4u>*)p)[i] = src[i];
}

// A value known to be the same in every lane, moved to a scalar register
// (the compiler cannot always tell that a loaded value is uniform, and
// would otherwise hold it in a vector register of every lane).
__device__ __forceinline__ int32_t uniform_i(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int64_t uniform_l(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uniform_p(T* p) {
    return reinterpret_cast<T*>(uniform_l((int64_t)reinterpret_cast<uintptr_t>(p)));
}

// The search fields of a keyframe descriptor, in scalar registers.
__device__ __forceinline__ KfDesc uniform_kf(const KfDesc& s) {
    KfDesc k;
#pragma unroll
    for (int i = 0; i < 9; ++i) k.A[i] = uniform_f(s.A[i]);
#pragma unroll
    for (int i = 0; i < 3; ++i) k.t[i] = uniform_f(s.t[i]);
    k.inv_s = uniform_f(s.inv_s);
    k.fx = uniform_f(s.fx);
    k.fy = uniform_f(s.fy);
    k.cx = uniform_f(s.cx);
    k.cy = uniform_f(s.cy);
    k.W = uniform_f(s.W);
    k.H = uniform_f(s.H);
    k.invw = uniform_f(s.invw);
    k.invh = uniform_f(s.invh);
#pragma unroll
    for (int i = 0; i < 12; ++i) k.T[i] = 0.0f;   // not used by the search
    k.kp_off = uniform_i(s.kp_off);
    k.n_kp = uniform_i(s.n_kp);
    k.grid_off = uniform_i(s.grid_off);
    k.event = uniform_i(s.event);
    k.mp_off = uniform_i(s.mp_off);
    k.n_mp = uniform_i(s.n_mp);
    k.hash_off = uniform_i(s.hash_off);
    k.hash_mask = uniform_i(s.hash_mask);
    k.n_tiles = uniform_i(s.n_tiles);
    k.pad0 = k.pad2 = 0;
    k.tile_pairs = uniform_i(s.tile_pairs);
    k.pair_off = uniform_l(s.pair_off);
    k.n_pairs = uniform_l(s.n_pairs);
    k.pass = uniform_i(s.pass);
    k.stage_key = uniform_i(s.stage_key);
    k.claim_off = uniform_i(s.claim_off);
    k.pad1 = 0;
    return k;
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8
// lanes inside each row of 16 (DPP row_shr), then the last lane of row 0 is
// added to row 1 and of row 2 to row 3 (row_bcast:15), and the last lane of
// row 1 to rows 2 and 3 (row_bcast:31).  Lanes with no source add 0.  Every
// lane of the wave must be active.
__device__ __forceinline__ int wave_incl_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15, rows 1 and 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31, rows 2 and 3
    return x;
}

// ADD conflicts, resolved by a kernel that runs after the whole batched
// search on the same stream.  Of the provisional ADDs on one keypoint the
// lowest point index (the claim it left, tagged with the launch epoch) keeps
// ADD; the others become FUSE to that point (Sec. IV-D3, with the
// lowest-index reading of concurrent additions).  Workgroup r of the search
// listed its provisional ADDs in its region of the ADD list; every thread of
// the calling workgroup takes part.
__device__ inline void resolve_region_adds(const BatchHdr& h, int r, unsigned long long tag) {
    const WgRange g = h.wg_range[r];
    const uint32_t n = h.add_count[r];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const AddRef e = h.add_list[g.priv_off + i];
        const int32_t w = (int32_t)(h.claim[e.kp] - tag);
        if (w != e.gp) {
            const PassOut& po = h.out[e.pass];
            po.decision[e.pair] = FL_FUSE;
            po.target[e.pair] = h.mp_id ? h.mp_id[w] : w;
        }
    }
}

}  // namespace fl
