/*
 * CPU oracle for Sim3-corrected search-and-fuse (loop fusion, Sec. IV-D3 of
 * the FastLoop paper; the fusion criteria are stated in Sec. III-B).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that the
 * GPU library is checked against.  It shares no code, header, table or
 * constant generator with the GPU library and must never be linked into it.
 *
 * Definition (per (map point p, keyframe k) pair), all float32 with the
 * operation order written below; every multiply-add written as fmaf() is a
 * single fused multiply-add, every other operation is rounded on its own:
 *
 *   sf[n]   = (float) pow(scale_factor, n), n < n_octaves (computed in double)
 *   r0      = win_px,  invw = (float)grid_cols / W,  invh = (float)grid_rows / H
 *   id(p)   = mp_id[p] if given, else the global index of p
 *   SKIP    (4) if id(p) equals kp_owner[i] >= 0 for some keypoint i of k
 *           (kp_owner < 0 marks a free keypoint)
 *   q_j     = fmaf(A[j][2], z, fmaf(A[j][1], y, fmaf(A[j][0], x, t[j])))
 *   NOT_VISIBLE (0) unless q_2 > 0
 *   iz = 1/q_2,  u = fmaf(fx, q_0*iz, cx),  v = fmaf(fy, q_1*iz, cy)
 *   NOT_VISIBLE (0) unless 0 <= u < W and 0 <= v < H
 *   d       = sqrtf(fmaf(q_0, q_0, fmaf(q_1, q_1, q_2*q_2))) * inv_s
 *   pred    = smallest n with d*sf[n] >= dmax[p], else n_octaves-1
 *             (dmax absent: pred = n_octaves-1 and the octave gate is off)
 *   rad     = r0 * sf[pred];  box = [u-rad, u+rad] x [v-rad, v+rad] (closed)
 *   Cset    = { i : x_i, y_i in box, pred-1 <= octave_i <= pred }
 *   h_i     = popcount(desc_p XOR desc_i) over 256 bits
 *   best    = lexicographic min of (h_i, i) over Cset; second = min h over
 *             the rest (0x7FFF when absent); best_idx = -1 when Cset empty
 *   accept  iff best_idx >= 0, best <= hamming_th and (ratio off or
 *             (float)best < nn_ratio * (float)second)
 *   NO_MATCH (1) if not accepted
 *   FUSE (3, target = kp_owner[best_idx]) if that keypoint is owned,
 *   else provisional ADD.  Among provisional ADDs on one keypoint of one
 *   keyframe, the lowest point index keeps ADD (2, target -1); all others
 *   become FUSE with target = id(lowest point).
 *   INVALID (5) when a sparse pair names a point outside its event.
 *
 * The brute-force variant evaluates Cset over every keypoint of the
 * keyframe.  The grid variant builds a cell grid (cell of a keypoint =
 * clamp(floor(x*invw)), clamp(floor(y*invh))) and scans the clamped cell
 * range of the box; it must give identical outputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { D_NOT_VISIBLE = 0, D_NO_MATCH = 1, D_ADD = 2, D_FUSE = 3, D_SKIP = 4, D_INVALID = 5 };
#define NO_DIST 0x7FFF
#define PROVISIONAL_ADD 250

typedef struct {
    float win_px;
    float scale_factor;
    int32_t n_octaves;
    int32_t grid_cols;
    int32_t grid_rows;
    int32_t hamming_th;
    float nn_ratio;
    int32_t flags;
} orc_params;

static int popcount8(uint8_t b) {
    int c = 0;
    while (b) { c += b & 1; b >>= 1; }
    return c;
}

static int hamming256(const uint8_t* a, const uint8_t* b) {
    int h = 0;
    for (int i = 0; i < 32; ++i) h += popcount8((uint8_t)(a[i] ^ b[i]));
    return h;
}

static int cell_of(float x, float inv, int n) {
    float f = floorf(x * inv);
    if (!(f >= 0.0f)) return 0;           /* negative or NaN */
    if (f >= (float)n) return n - 1;
    return (int)f;
}

/* Grid of one keyframe: cell_start[cells+1], cell_kp[n] (CSR, keypoints of a
 * cell in increasing index order). */
static void build_grid(int n, const float* xy, int C, int R, float invw, float invh,
                       int32_t* cell_start, int32_t* cell_kp) {
    int cells = C * R;
    memset(cell_start, 0, sizeof(int32_t) * (size_t)(cells + 1));
    for (int i = 0; i < n; ++i) {
        int c = cell_of(xy[2 * i + 1], invh, R) * C + cell_of(xy[2 * i], invw, C);
        cell_start[c + 1]++;
    }
    for (int c = 0; c < cells; ++c) cell_start[c + 1] += cell_start[c];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)cells);
    memcpy(fill, cell_start, sizeof(int32_t) * (size_t)cells);
    for (int i = 0; i < n; ++i) {
        int c = cell_of(xy[2 * i + 1], invh, R) * C + cell_of(xy[2 * i], invw, C);
        cell_kp[fill[c]++] = i;
    }
    free(fill);
}


/* Transform, projection, visibility and predicted octave of one point in one
 * keyframe (float32, the order stated at the top).  Returns 1 if visible. */
static int project_point(const float* S, const float* K, const float* X, const float* sf, int N,
                         float dmax, int gate, float* pu, float* pv, float* pd, int* ppred) {
    const float fx = K[0], fy = K[1], cx = K[2], cy = K[3], W = K[4], H = K[5];
    const float x = X[0], y = X[1], z = X[2];
    const float q0 = fmaf(S[2], z, fmaf(S[1], y, fmaf(S[0], x, S[9])));
    const float q1 = fmaf(S[5], z, fmaf(S[4], y, fmaf(S[3], x, S[10])));
    const float q2 = fmaf(S[8], z, fmaf(S[7], y, fmaf(S[6], x, S[11])));
    if (!(q2 > 0.0f)) return 0;
    const float iz = 1.0f / q2;
    const float u = fmaf(fx, q0 * iz, cx);
    const float v = fmaf(fy, q1 * iz, cy);
    if (!(u >= 0.0f && u < W && v >= 0.0f && v < H)) return 0;
    const float d = sqrtf(fmaf(q0, q0, fmaf(q1, q1, q2 * q2))) * S[12];
    int pred = N - 1;
    if (gate) {
        for (int n = 0; n < N; ++n)
            if (d * sf[n] >= dmax) { pred = n; break; }
    }
    *pu = u;
    *pv = v;
    *pd = d;
    *ppred = pred;
    return 1;
}

/* Offer candidate (h, i) to the running best / second-best. */
static void offer(int h, int i, int* best_h, int* best_i, int* second_h) {
    if (*best_i < 0 || h < *best_h || (h == *best_h && i < *best_i)) {
        if (*best_i >= 0 && *best_h < *second_h) *second_h = *best_h;
        *best_h = h;
        *best_i = i;
    } else if (h < *second_h) {
        *second_h = h;
    }
}

/*
 * Search-and-fuse over a batch of keyframes.
 *   kf_sim3 : [n_kf][16]  sR row-major (9), t (3), inv_s, pad
 *   kf_cam  : [n_kf][8]   fx, fy, cx, cy, W, H, pad
 *   kf_event: [n_kf] event of each keyframe; event_mp_offset: [n_events+1]
 *   pair_offset: [n_kf+1]; pair_mp: local point index per pair, NULL = dense
 *   counters (nullable, grid variant): n_visible, n_cells, n_kp_scanned, n_cand
 */
int orc_search_fuse(int n_kf, const int32_t* kp_offset, const float* kp_xy, const int8_t* kp_oct,
                    const uint8_t* kp_desc, const int32_t* kp_owner, const float* kf_sim3,
                    const float* kf_cam, const int32_t* kf_event, const int32_t* event_mp_offset,
                    const float* mp_xyz, const uint8_t* mp_desc, const float* mp_dmax,
                    const int32_t* mp_id, const int64_t* pair_offset, const int32_t* pair_mp,
                    const orc_params* P, int use_grid, int32_t* best_idx, int16_t* best_dist,
                    int16_t* second_dist, uint8_t* decision, int32_t* target, int64_t* counters) {
    const int N = P->n_octaves;
    if (N < 1 || N > 32 || P->grid_cols < 1 || P->grid_rows < 1) return -1;
    float sf[32];
    for (int n = 0; n < N; ++n) sf[n] = (float)pow((double)P->scale_factor, (double)n);
    const float r0 = P->win_px;
    int64_t n_visible = 0, n_cells = 0, n_kp_scanned = 0, n_cand = 0;

    for (int k = 0; k < n_kf; ++k) {
        const int kp0 = kp_offset[k];
        const int nkp = kp_offset[k + 1] - kp0;
        const float* xy = kp_xy + 2 * (int64_t)kp0;
        const int8_t* oc = kp_oct + kp0;
        const uint8_t* kd = kp_desc + 32 * (int64_t)kp0;
        const int32_t* ow = kp_owner + kp0;
        const float* S = kf_sim3 + 16 * k;
        const float* K = kf_cam + 8 * k;
        const int C = P->grid_cols, R = P->grid_rows;
        const float invw = (float)C / K[4], invh = (float)R / K[5];
        const int ev = kf_event[k];
        const int mp0 = event_mp_offset[ev];
        const int nmp = event_mp_offset[ev + 1] - mp0;
        const int64_t pb = pair_offset[k];
        const int64_t np_k = pair_offset[k + 1] - pb;

        int32_t* cell_start = NULL;
        int32_t* cell_kp = NULL;
        if (use_grid) {
            cell_start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(C * R + 1));
            cell_kp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nkp > 0 ? nkp : 1));
            build_grid(nkp, xy, C, R, invw, invh, cell_start, cell_kp);
        }
        /* lowest global point index with a provisional ADD on each keypoint */
        int32_t* claim = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nkp > 0 ? nkp : 1));
        for (int i = 0; i < nkp; ++i) claim[i] = INT32_MAX;

        for (int64_t j = 0; j < np_k; ++j) {
            const int64_t o = pb + j;
            best_idx[o] = -1;
            best_dist[o] = NO_DIST;
            second_dist[o] = NO_DIST;
            target[o] = -1;
            const int64_t lp = pair_mp ? (int64_t)pair_mp[o] : j;
            if (lp < 0 || lp >= nmp) { decision[o] = D_INVALID; continue; }
            const int64_t gp = mp0 + lp;
            const int32_t id = mp_id ? mp_id[gp] : (int32_t)gp;

            int observed = 0;
            for (int i = 0; i < nkp; ++i)
                if (ow[i] >= 0 && ow[i] == id) { observed = 1; break; }
            if (observed) { decision[o] = D_SKIP; continue; }

            float u, v, d;
            int pred;
            const int gate = mp_dmax != NULL;
            if (!project_point(S, K, mp_xyz + 3 * gp, sf, N, gate ? mp_dmax[gp] : 0.0f, gate, &u, &v, &d,
                               &pred)) {
                decision[o] = D_NOT_VISIBLE;
                continue;
            }
            ++n_visible;
            const float rad = r0 * sf[pred];
            const float lx = u - rad, hx = u + rad, ly = v - rad, hy = v + rad;
            const uint8_t* pd = mp_desc + 32 * gp;

            int bh = NO_DIST, bi = -1, sh = NO_DIST;
            if (!use_grid) {
                for (int i = 0; i < nkp; ++i) {
                    const float kx = xy[2 * i], ky = xy[2 * i + 1];
                    if (!(kx >= lx && kx <= hx && ky >= ly && ky <= hy)) continue;
                    if (gate && (oc[i] < pred - 1 || oc[i] > pred)) continue;
                    offer(hamming256(pd, kd + 32 * i), i, &bh, &bi, &sh);
                }
            } else {
                const int c0 = cell_of(lx, invw, C), c1 = cell_of(hx, invw, C);
                const int r0c = cell_of(ly, invh, R), r1c = cell_of(hy, invh, R);
                for (int r = r0c; r <= r1c; ++r) {
                    for (int c = c0; c <= c1; ++c) {
                        ++n_cells;
                        const int cell = r * C + c;
                        for (int s = cell_start[cell]; s < cell_start[cell + 1]; ++s) {
                            const int i = cell_kp[s];
                            ++n_kp_scanned;
                            const float kx = xy[2 * i], ky = xy[2 * i + 1];
                            if (!(kx >= lx && kx <= hx && ky >= ly && ky <= hy)) continue;
                            if (gate && (oc[i] < pred - 1 || oc[i] > pred)) continue;
                            ++n_cand;
                            offer(hamming256(pd, kd + 32 * i), i, &bh, &bi, &sh);
                        }
                    }
                }
            }
            best_idx[o] = bi;
            best_dist[o] = (int16_t)bh;
            second_dist[o] = (int16_t)sh;
            int accept = bi >= 0 && bh <= P->hamming_th;
            if (accept && P->nn_ratio > 0.0f && P->nn_ratio < 1.0f)
                accept = (float)bh < P->nn_ratio * (float)sh;
            if (!accept) { decision[o] = D_NO_MATCH; continue; }
            if (ow[bi] >= 0) {
                decision[o] = D_FUSE;
                target[o] = ow[bi];
            } else {
                decision[o] = PROVISIONAL_ADD;
                if (gp < claim[bi]) claim[bi] = (int32_t)gp;
            }
        }
        /* conflict resolution among provisional ADDs of this keyframe */
        for (int64_t j = 0; j < np_k; ++j) {
            const int64_t o = pb + j;
            if (decision[o] != PROVISIONAL_ADD) continue;
            const int64_t gp = mp0 + (pair_mp ? (int64_t)pair_mp[o] : j);
            const int32_t w = claim[best_idx[o]];
            if (w == gp) {
                decision[o] = D_ADD;
                target[o] = -1;
            } else {
                decision[o] = D_FUSE;
                target[o] = mp_id ? mp_id[w] : w;
            }
        }
        free(claim);
        free(cell_start);
        free(cell_kp);
    }
    if (counters) {
        counters[0] = n_visible;
        counters[1] = n_cells;
        counters[2] = n_kp_scanned;
        counters[3] = n_cand;
    }
    return 0;
}

/*
 * FP64 boundary census.  For every valid, unobserved pair, recompute the
 * projection, visibility, predicted octave and candidate set in double
 * precision from the same (float) inputs and compare with float32:
 *   out[0] = pairs whose visibility, pred or candidate set differ
 *   out[1] = pairs with a keypoint within eps px of an edge of the (FP64)
 *            window: an eligible-octave keypoint whose x (or y) is within
 *            eps of a box edge while its y (or x) lies in the box widened
 *            by eps (the window-edge cases the bound is stated for)
 *   out[2] = pairs examined
 *   out[3] = pairs whose FP64 projection lies within eps px of an image
 *            edge: |u|, |u-W|, |v|, |v-H| < eps (the visibility boundary;
 *            such a pair is not examined for window edges)
 */
int orc_census_fp64(int n_kf, const int32_t* kp_offset, const float* kp_xy, const int8_t* kp_oct,
                    const int32_t* kp_owner, const float* kf_sim3, const float* kf_cam,
                    const int32_t* kf_event, const int32_t* event_mp_offset, const float* mp_xyz,
                    const float* mp_dmax, const int32_t* mp_id, const int64_t* pair_offset,
                    const int32_t* pair_mp, const orc_params* P, double eps, int64_t* out) {
    const int N = P->n_octaves;
    if (N < 1 || N > 32) return -1;
    float sf[32];
    double sf64[32];
    for (int n = 0; n < N; ++n) {
        sf64[n] = pow((double)P->scale_factor, (double)n);
        sf[n] = (float)sf64[n];
    }
    int64_t n_diff = 0, n_near = 0, n_exam = 0, n_image = 0;
    for (int k = 0; k < n_kf; ++k) {
        const int kp0 = kp_offset[k];
        const int nkp = kp_offset[k + 1] - kp0;
        const float* xy = kp_xy + 2 * (int64_t)kp0;
        const int8_t* oc = kp_oct + kp0;
        const int32_t* ow = kp_owner + kp0;
        const float* S = kf_sim3 + 16 * k;
        const float* K = kf_cam + 8 * k;
        const int ev = kf_event[k];
        const int mp0 = event_mp_offset[ev];
        const int nmp = event_mp_offset[ev + 1] - mp0;
        for (int64_t j = 0; j < pair_offset[k + 1] - pair_offset[k]; ++j) {
            const int64_t o = pair_offset[k] + j;
            const int64_t lp = pair_mp ? (int64_t)pair_mp[o] : j;
            if (lp < 0 || lp >= nmp) continue;
            const int64_t gp = mp0 + lp;
            const int32_t id = mp_id ? mp_id[gp] : (int32_t)gp;
            int observed = 0;
            for (int i = 0; i < nkp; ++i)
                if (ow[i] >= 0 && ow[i] == id) { observed = 1; break; }
            if (observed) continue;
            ++n_exam;
            const float x = mp_xyz[3 * gp], y = mp_xyz[3 * gp + 1], z = mp_xyz[3 * gp + 2];
            /* float32 path */
            const float q0 = fmaf(S[2], z, fmaf(S[1], y, fmaf(S[0], x, S[9])));
            const float q1 = fmaf(S[5], z, fmaf(S[4], y, fmaf(S[3], x, S[10])));
            const float q2 = fmaf(S[8], z, fmaf(S[7], y, fmaf(S[6], x, S[11])));
            int vis32 = 0, pred32 = N - 1;
            float u = 0, v = 0, rad = 0;
            if (q2 > 0.0f) {
                const float iz = 1.0f / q2;
                u = fmaf(K[0], q0 * iz, K[2]);
                v = fmaf(K[1], q1 * iz, K[3]);
                vis32 = u >= 0.0f && u < K[4] && v >= 0.0f && v < K[5];
                if (vis32 && mp_dmax) {
                    const float d = sqrtf(fmaf(q0, q0, fmaf(q1, q1, q2 * q2))) * S[12];
                    for (int n = 0; n < N; ++n)
                        if (d * sf[n] >= mp_dmax[gp]) { pred32 = n; break; }
                }
                rad = P->win_px * sf[pred32];
            }
            /* float64 path from the same inputs */
            const double Q0 = (double)S[0] * x + (double)S[1] * y + (double)S[2] * z + (double)S[9];
            const double Q1 = (double)S[3] * x + (double)S[4] * y + (double)S[5] * z + (double)S[10];
            const double Q2 = (double)S[6] * x + (double)S[7] * y + (double)S[8] * z + (double)S[11];
            int vis64 = 0, pred64 = N - 1;
            double U = 0, V = 0, RAD = 0;
            if (Q2 > 0.0) {
                U = (double)K[0] * (Q0 / Q2) + (double)K[2];
                V = (double)K[1] * (Q1 / Q2) + (double)K[3];
                vis64 = U >= 0.0 && U < K[4] && V >= 0.0 && V < K[5];
                if (vis64 && mp_dmax) {
                    const double d = sqrt(Q0 * Q0 + Q1 * Q1 + Q2 * Q2) * (double)S[12];
                    for (int n = 0; n < N; ++n)
                        if (d * sf64[n] >= (double)mp_dmax[gp]) { pred64 = n; break; }
                }
                RAD = (double)P->win_px * sf64[pred64];
                if (fabs(U) < eps || fabs(U - K[4]) < eps || fabs(V) < eps || fabs(V - K[5]) < eps) {
                    ++n_image;
                    if (vis32 != vis64) ++n_diff;
                    continue;
                }
            }
            if (vis32 != vis64 || pred32 != pred64) { ++n_diff; continue; }
            if (!vis32) continue;
            int differ = 0, near = 0;
            for (int i = 0; i < nkp; ++i) {
                if (mp_dmax && (oc[i] < pred32 - 1 || oc[i] > pred32)) continue;
                const double kx = xy[2 * i], ky = xy[2 * i + 1];
                const int in32 = (float)kx >= u - rad && (float)kx <= u + rad && (float)ky >= v - rad &&
                                 (float)ky <= v + rad;
                const int in64 = kx >= U - RAD && kx <= U + RAD && ky >= V - RAD && ky <= V + RAD;
                if (in32 != in64) differ = 1;
                const int inx = kx >= U - RAD - eps && kx <= U + RAD + eps;
                const int iny = ky >= V - RAD - eps && ky <= V + RAD + eps;
                const int nearx = fabs(kx - (U - RAD)) < eps || fabs(kx - (U + RAD)) < eps;
                const int neary = fabs(ky - (V - RAD)) < eps || fabs(ky - (V + RAD)) < eps;
                if ((nearx && iny) || (neary && inx)) near = 1;
            }
            n_diff += differ;
            n_near += near;
        }
    }
    out[0] = n_diff;
    out[1] = n_near;
    out[2] = n_exam;
    out[3] = n_image;
    return 0;
}

/* Hamming distance of two 256-bit rows (exposed for the popcount pins). */
int orc_hamming256(const uint8_t* a, const uint8_t* b) { return hamming256(a, b); }

/* Per-pair projection (u, v, metric distance, predicted octave, visible) of
 * points X[n] through one keyframe transform, for the projection pins. */
int orc_project(int n, const float* X, const float* S, const float* K, const float* dmax,
                const orc_params* P, float* u, float* v, float* d, int32_t* pred, uint8_t* vis) {
    const int N = P->n_octaves;
    if (N < 1 || N > 32) return -1;
    float sf[32];
    for (int k = 0; k < N; ++k) sf[k] = (float)pow((double)P->scale_factor, (double)k);
    for (int i = 0; i < n; ++i) {
        int pr = -1;
        float uu = 0, vv = 0, dd = 0;
        vis[i] = (uint8_t)project_point(S, K, X + 3 * i, sf, N, dmax ? dmax[i] : 0.0f, dmax != NULL, &uu,
                                        &vv, &dd, &pr);
        u[i] = uu;
        v[i] = vv;
        d[i] = dd;
        pred[i] = vis[i] ? pr : -1;
    }
    return 0;
}

/* Keypoint cell grid of one keyframe (the CSR the search scans). */
int orc_build_grid(int n, const float* xy, int C, int R, float W, float H, int32_t* cell_start,
                   int32_t* cell_kp) {
    if (n < 0 || C < 1 || R < 1) return -1;
    build_grid(n, xy, C, R, (float)C / W, (float)R / H, cell_start, cell_kp);
    return 0;
}
