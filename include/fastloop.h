/*
 * fastloop.h - C ABI of an MI355X (gfx950) library for the data-parallel core
 * of loop closing in visual SLAM: Sim3-corrected search-and-fuse and the
 * Sim3 reprojection residual with its hand-written backward.
 *
 * Paper: "FastLoop: Parallel Loop Closing with GPU-Acceleration in Visual
 * SLAM" (arXiv 2603.17201).  Loop fusion (Sec. III-B, Sec. IV-D3) projects the
 * map points of the loop region through the loop-corrected Sim3 into every
 * connected keyframe and merges points with keypoints that are close in the
 * image and similar in descriptor.  Keyframes are mutually independent
 * (Sec. IV-D3), data stays resident on the GPU and is transferred once, in
 * compact wrapper structures, into memory allocated once (Sec. IV-E).
 *
 * Conventions for every entry point
 *  - Pointers named in the argument comments as "host" point to host memory;
 *    all others are device pointers into HBM owned by the caller.  The
 *    library never frees caller memory.
 *  - All work is enqueued on the given stream; no call synchronises the
 *    stream unless it says so.  Host arrays are copied before the call
 *    returns, so the caller may reuse them immediately.
 *  - Every function returns FL_OK (0) or a negative FL_E* code; the message
 *    of the last failure on the calling thread is in fl_last_error().  All
 *    checks that can run on the host run before anything is enqueued.
 *  - Descriptor rows (32 bytes each) must start at a 16-byte aligned address.
 *  - A Sim3 acts as X -> s R X + t (world to camera).  The search form
 *    fl_sim3 stores sR row-major, t and 1/s in float32.  The float64 form
 *    used by refinement is 13 doubles [R row-major (9), t (3), s].  Tangent
 *    vectors are xi = (omega, upsilon, sigma) with left perturbation
 *    S <- exp(xi) S.
 */
#ifndef FASTLOOP_H
#define FASTLOOP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FL_OK 0
#define FL_EINVAL (-1)   /* an argument is invalid (NULL, negative, misaligned, inconsistent) */
#define FL_ENOMEM (-2)   /* device or pinned host allocation failed */
#define FL_EHIP (-3)     /* a HIP runtime call failed */
#define FL_ERANGE (-4)   /* a size exceeds a documented limit */
#define FL_ENOTSUP (-5)  /* the device is not supported */

/* decision per (map point, keyframe) pair */
#define FL_NOT_VISIBLE 0 /* behind the camera or projects outside the image */
#define FL_NO_MATCH 1    /* visible, no candidate accepted */
#define FL_ADD 2         /* accepted; the keypoint was free and this point takes it */
#define FL_FUSE 3        /* accepted; merge into target (owner id) */
#define FL_SKIP 4        /* the point already owns a keypoint of this keyframe */
#define FL_INVALID 5     /* a sparse pair names a point outside its event */

#define FL_NO_DIST 0x7FFF
#define FL_MAX_KP 65535      /* keypoints per keyframe (16-bit index in the packed key) */
#define FL_MAX_OCTAVES 32
#define FL_MAX_CELLS 8192    /* grid_cols * grid_rows */
#define FL_MAX_PAIRS 2147483647LL

typedef struct fl_ctx fl_ctx;

/* Search form of a (keyframe-composed) Sim3: q = sR X + t, metric distance
 * |q| * inv_s.  64 bytes. */
typedef struct {
    float sR[9];
    float t[3];
    float inv_s;
    float pad[3];
} fl_sim3;

/* Pinhole camera: u = fx x/z + cx, v = fy y/z + cy, image [0,width) x [0,height). */
typedef struct {
    float fx, fy, cx, cy, width, height;
    float pad[2];
} fl_pinhole;

/* Search thresholds.  Window half-width win_px * scale_factor^pred where
 * pred is the point's predicted octave; keypoint octave gate {pred-1, pred};
 * accept iff Hamming distance <= hamming_th (and, when 0 < nn_ratio < 1,
 * best < nn_ratio * second).  Typical: 3.0, 1.2, 8, 64, 48, 50, 0. */
typedef struct {
    float win_px;
    float scale_factor;
    int32_t n_octaves;   /* 1..32 */
    int32_t grid_cols;   /* grid_cols * grid_rows <= FL_MAX_CELLS */
    int32_t grid_rows;
    int32_t hamming_th;
    float nn_ratio;      /* <= 0 or >= 1: ratio test off */
    int32_t flags;       /* must be 0 */
} fl_params;

/* Per-pair outputs (device arrays, one entry per pair).  best_idx is the
 * keypoint index within its keyframe (-1: no candidate); best_dist and
 * second_dist are Hamming distances (FL_NO_DIST when absent); target is the
 * owner id merged into for FL_FUSE, else -1. */
typedef struct {
    int32_t* best_idx;
    int16_t* best_dist;
    int16_t* second_dist;
    uint8_t* decision;
    int32_t* target;
} fl_fuse_out;

/* One keyframe's keypoints (device arrays of n_kp entries).  kp_owner < 0
 * marks a free keypoint, otherwise the id of the map point observed there.
 * cell_start [grid_cols*grid_rows + 1] / cell_kp [n_kp] is the keypoint grid
 * produced by fl_build_grid; both NULL: the library builds it. */
typedef struct {
    int32_t n_kp;
    const float* kp_xy;        /* [n_kp][2] */
    const int8_t* kp_octave;   /* [n_kp] */
    const uint8_t* kp_desc;    /* [n_kp][32] */
    const int32_t* kp_owner;   /* [n_kp] */
    const int32_t* cell_start;
    const int32_t* cell_kp;
} fl_keyframe;

/* A batch of loop events.  Keyframes, keypoints and points of all events are
 * concatenated; pairs are grouped by keyframe.  Small tables are host arrays
 * (validated and uploaded by the library), bulk data are device arrays. */
typedef struct {
    int32_t n_events;
    int32_t n_kf;
    int32_t n_mp;                     /* total points */
    int32_t n_kp_total;               /* total keypoints */
    int64_t n_pairs;                  /* total pairs (< 2^31) */
    const int32_t* event_kf_offset;   /* host [n_events+1] keyframe range of each event */
    const int32_t* event_mp_offset;   /* host [n_events+1] point range of each event */
    const int32_t* kp_offset;         /* host [n_kf+1] keypoint range of each keyframe */
    const int64_t* pair_offset;       /* host [n_kf+1] pair range of each keyframe */
    const fl_sim3* kf_sim3;           /* host [n_kf] search transform of each keyframe */
    const fl_pinhole* kf_K;           /* host [n_kf] camera of each keyframe */
    const float* kf_T;                /* host [n_kf][12] world->camera SE3 (R row-major, t); refinement only, may be NULL */
    const int32_t* pair_mp;           /* device [n_pairs] point index within the event; NULL = dense
                                         (pair j of keyframe k is point j of its event) */
    const float* kp_xy;               /* device [n_kp_total][2] */
    const int8_t* kp_octave;          /* device [n_kp_total] */
    const uint8_t* kp_desc;           /* device [n_kp_total][32] */
    const int32_t* kp_owner;          /* device [n_kp_total] */
    const float* mp_xyz;              /* device [n_mp][3] */
    const uint8_t* mp_desc;           /* device [n_mp][32] */
    const float* mp_dmax;             /* device [n_mp] distance invariance; NULL: pred = n_octaves-1, no octave gate */
    const int32_t* mp_id;             /* device [n_mp]; NULL: id = index in the batch */
} fl_batch;

/* Refinement of each event's loop Sim3 after matching (Gauss-Newton on the
 * Huber reprojection residual of the accepted pairs).
 * The workgroups that refine one event exchange partial sums every step and
 * wait for one another, so they must be resident together: one launch keeps
 * at most one such workgroup per compute unit (at most 64 per event, 256 in
 * all), and a single-event launch uses at most 64.  Launches from several
 * contexts may overlap on different streams (for instance consecutive events
 * alternating between two contexts) as long as their events' workgroups
 * together stay within the compute units, which two single-event launches
 * always do.  A wait that does not end within its bound reports the event as
 * failed (event_n_matched = -1); it never blocks the device. */
/* The other direction of a loop's matches, for two-sided refinement (the
 * loop's Sim3 is refined on the matches seen from both keyframes of the
 * loop, Sec. IV-C): points of the current side observed in loop-side
 * keyframes through S^-1, p = S^-1 X, q = R_m p + t_m, r = pi(q) - uv, with
 * the Jacobian taken with respect to the same left perturbation of S as the
 * accepted pairs'.  Pair i of event e is in [event_offset[e],
 * event_offset[e+1]).  A pair whose kf_idx is outside [0, n_kf) or whose q_z
 * is not positive adds nothing.  Gauss-Newton only (n_rounds <= 1,
 * lm_lambda = 0). */
typedef struct {
    const int64_t* event_offset;  /* host [n_events+1], event_offset[0] = 0, non-decreasing, total < 2^31 */
    const float* xyz;             /* device [n][3] point, in the frame S maps into (16-byte aligned base) */
    const float* uv;              /* device [n][2] observation, pixels */
    const int32_t* kf_idx;        /* device [n] observing keyframe (index into kf_T and kf_cam) */
    const float* kf_T;            /* device [n_kf][12] world->camera SE3 of each observing keyframe (R row-major, t) */
    const float* kf_cam;          /* device [n_kf][4] fx, fy, cx, cy of each observing keyframe */
    int32_t n_kf;                 /* observing keyframes (> 0 when any pair is given) */
    int32_t flags;                /* must be 0 */
} fl_refine_inverse;

typedef struct {
    int32_t n_iters;        /* evaluations per round; 0 = no refinement */
    float huber_delta;      /* pixels */
    double* event_S;        /* device [n_events][13] in: start, out: refined (float64 Sim3) */
    fl_sim3* event_S32;     /* device [n_events] out: float32 form of the refined Sim3 (may be NULL) */
    int32_t* event_n_matched; /* device [n_events] out: pairs of the result's last evaluation (may be NULL) */
    /* Robust refinement (all zero: one round of Gauss-Newton).  Round 0 uses
     * every accepted pair; each later round uses the pairs in front of their
     * keyframe whose reprojection error at the round's starting Sim3 is at
     * most outlier_px.  lm_lambda > 0 selects Levenberg-Marquardt: the first
     * evaluation of a round is at its starting Sim3, each later one at the
     * candidate exp(d) S_acc with (H + lambda diag H) d = -g at the accepted
     * S_acc; a candidate with a lower Huber loss is accepted (lambda / 10),
     * otherwise rejected (lambda x 10); lambda restarts at lm_lambda each
     * round, and the round ends at S_acc.  n_iters * max(n_rounds, 1) <= 1000. */
    int32_t n_rounds;       /* 0 or 1: one round */
    float outlier_px;       /* > 0 when n_rounds > 1 (may be +inf) */
    float lm_lambda;        /* 0: Gauss-Newton */
    int32_t flags;          /* must be 0 */
    /* Two-sided refinement: every evaluation also sums the terms of these
     * pairs at S^-1 (NULL: the accepted pairs only).  event_n_matched then
     * counts the pairs of both directions. */
    const fl_refine_inverse* inverse;   /* host, may be NULL */
} fl_refine;

/* ------------------------------------------------------------------ */
/* Context: workspace memory, pinned staging and captured graphs, allocated
 * once and reused (Sec. IV-E).  One context per device and host thread. */
int fl_create(fl_ctx** out, int device);
void fl_destroy(fl_ctx* ctx);
const char* fl_last_error(void);
int fl_version(void);

/* Keypoint cell grid of one keyframe (the "grid" input of the search): the
 * paper's loop fusion gathers a point's candidate keypoints from the cells
 * around its projection (Sec. IV-D3, the projection search of Sec. IV-D1).
 * Cell of a keypoint = (clamp(floor(y*R/H)), clamp(floor(x*C/W))) in float32;
 * cell_start [C*R+1] is the exclusive prefix sum of the per-cell counts and
 * cell_kp [n_kp] lists keypoint indices cell by cell, increasing within a
 * cell.  Errors: FL_EINVAL (NULL with n_kp > 0, bad params), FL_ERANGE
 * (n_kp > FL_MAX_KP, cells > FL_MAX_CELLS). */
int fl_build_grid(fl_ctx* ctx, int32_t n_kp, const float* kp_xy, const fl_pinhole* K /* host */,
                  const fl_params* P /* host */, int32_t* cell_start, int32_t* cell_kp, hipStream_t stream);

/* Plain search-and-fuse: every one of n_mp points against ONE keyframe, one
 * lane per point, the per-call form of the paper's projection-search kernel
 * (Sec. IV-D1, loop fusion Sec. IV-D3).  Pair index = point index; ids are
 * mp_id[i] (or i when mp_id is NULL).  Outputs: see fl_fuse_out.  Errors:
 * FL_EINVAL, FL_ERANGE as for fl_build_grid; misaligned descriptors. */
int fl_search_fuse(fl_ctx* ctx, int32_t n_mp, const float* mp_xyz, const uint8_t* mp_desc,
                   const float* mp_dmax, const int32_t* mp_id, const fl_keyframe* kf /* host */,
                   const fl_sim3* S /* host */, const fl_pinhole* K /* host */,
                   const fl_params* P /* host */, const fl_fuse_out* out /* host */, hipStream_t stream);

/* fl_search_fuse without a context and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid it).  Same arguments (less the
 * context), same outputs and the same kernels.  Its scratch (the keyframe's
 * grid when none is given, the owner hash set, the ADD claims and list) is
 * one static device array of 1 MiB per GPU, resolved once per device (in
 * fl_create, or at the first call on the current device): a keyframe of
 * n_kp keypoints needs about 8 * n_kp + 4 * pow2(2 n_kp) + 16 * min(n_mp,
 * max(2 n_kp, 4096)) + 4 * cells bytes, so keyframes of up to about 16,000
 * keypoints fit whatever n_mp.
 * Every call on one GPU shares that array and rewrites what it reads first;
 * calls that overlap on one GPU (two streams, or threads, in flight at once)
 * race on it and must be serialised by the caller.  Runs on the current
 * device.  Errors: as fl_search_fuse; FL_ERANGE when the scratch would not
 * hold the call (use fl_search_fuse); FL_EHIP when the array's address
 * cannot be resolved. */
int fl_search_fuse_noalloc(int32_t n_mp, const float* mp_xyz, const uint8_t* mp_desc, const float* mp_dmax,
                           const int32_t* mp_id, const fl_keyframe* kf /* host */, const fl_sim3* S /* host */,
                           const fl_pinhole* K /* host */, const fl_params* P /* host */,
                           const fl_fuse_out* out /* host */, hipStream_t stream);

/* Host-only check of a batch (every test fl_search_fuse_batched makes before
 * enqueuing anything; no device memory is touched, no context needed).
 * Returns FL_OK or the error code the batched call would return. */
int fl_validate_batch(const fl_batch* B /* host */, const fl_params* P /* host */, const fl_fuse_out* out /* host */);

/* Batched search-and-fuse over whole loop events (Sec. IV-D3: connected
 * keyframes evaluated concurrently on resident data, Sec. IV-E: one transfer
 * of compact tables): one upload of the batch tables and one fused kernel
 * that stages each keyframe's grid in LDS and searches all pairs of all
 * events; the ADD conflicts of each keyframe are resolved by the kernel that
 * follows on the stream (the refinement, or a resolution kernel when refine
 * is NULL), so the outputs are final when the stream reaches the end of the
 * call's work.  Results are identical to
 * fl_search_fuse applied per keyframe.  With refine non-NULL the search also
 * records each event's accepted pairs and per-event Sim3 refinement follows
 * on the same stream, as in fl_search_fuse_graph_launch.
 * Errors: FL_EINVAL (inconsistent offsets or NULL arrays), FL_ERANGE. */
int fl_search_fuse_batched(fl_ctx* ctx, const fl_batch* B /* host */, const fl_params* P /* host */,
                           const fl_fuse_out* out /* host */, const fl_refine* refine /* host, may be NULL */,
                           hipStream_t stream);

/* The same work as fl_search_fuse_batched, optionally followed by per-event
 * Sim3 refinement, replayed from a HIP graph captured on first use: one
 * upload and one graph launch per call.  The graph is independent of the
 * batch sizes and re-captured only when the workspace grows or the tuning
 * changes.  refine may be NULL. */
int fl_search_fuse_graph_launch(fl_ctx* ctx, const fl_batch* B /* host */, const fl_params* P /* host */,
                                const fl_fuse_out* out /* host */, const fl_refine* refine /* host */,
                                hipStream_t stream);

/* One search of a batch in fl_search_fuse_passes: the search transform of
 * each keyframe, the thresholds and the outputs of this pass. */
#define FL_MAX_PASSES 4
typedef struct {
    const fl_sim3* kf_sim3;   /* host [n_kf] search transform of each keyframe for this pass; NULL: the batch's */
    fl_params params;         /* win_px, hamming_th and nn_ratio may differ between passes; scale_factor,
                                 n_octaves, grid_cols and grid_rows must equal those of pass 0 */
    fl_fuse_out out;          /* device [n_pairs] each; no array shared with another pass */
} fl_pass;

/* Several independent searches of one resident batch, launched together
 * (task parallelism, Sec. IV-C: searches of the same kind of input with no
 * dependency between them, such as the projection searches on the current
 * keyframe before and after the Sim3 optimization, run concurrently from one
 * transfer and keep their outputs in separate batches).  The tiles of every
 * pass share one launch, and a workgroup stages a keyframe's grid once for
 * all passes of it.  Pass p's outputs are identical to those of
 * fl_search_fuse_batched on the batch with passes[p].kf_sim3 (when given),
 * &passes[p].params and &passes[p].out; the ADD conflicts of a pass are
 * resolved within that pass.  No refinement.  Errors: those of
 * fl_search_fuse_batched for any pass; FL_EINVAL for passes NULL, n_pass
 * outside [1, FL_MAX_PASSES], grid or octave fields that differ from pass 0,
 * or two passes sharing an output array; FL_ERANGE when n_pass * n_kp_total
 * exceeds 2^31-1. */
int fl_search_fuse_passes(fl_ctx* ctx, const fl_batch* B /* host */, int32_t n_pass,
                          const fl_pass* passes /* host [n_pass] */, hipStream_t stream);

/* Per-event Sim3 refinement on the pairs a previous search accepted (ADD or
 * FUSE; observation = matched keypoint position), eagerly launched.
 * B must describe the same batch and out hold that search's results. */
int fl_refine_events(fl_ctx* ctx, const fl_batch* B /* host */, const fl_fuse_out* out /* host */,
                     const fl_refine* refine /* host */, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Sim3 reprojection residual over n matched pairs (the refinement that
 * follows matching, Sec. IV-C): p = sR X + t, q = R_k p + t_k,
 * r = pi(q) - uv, e = |r|, Huber rho(e) with threshold huber_delta,
 * w = min(1, delta/e); pairs with q_z <= 0 give r = 0, w = 0.
 * xyz [n][3], uv [n][2], kf_idx [n] (NULL: all 0), kf_T [n_kf][12] device
 * (NULL: identity), S device pointer to one fl_sim3.  Outputs r [n][2],
 * w [n] (either may be NULL) and loss [1] (float64, sum of rho). */
int fl_reproj_residual_fwd(fl_ctx* ctx, int32_t n, const float* xyz, const float* uv,
                           const int32_t* kf_idx, int32_t n_kf, const float* kf_T, const fl_sim3* S,
                           const fl_pinhole* K /* host */, float huber_delta, float* r, float* w,
                           double* loss, hipStream_t stream);

/* Hand-written backward of the residual: with J = d r / d xi (2x7, left
 * perturbation at xi = 0), g = grad_scale * sum w J^T r (7 doubles) and,
 * if H is not NULL, the Gauss-Newton matrix sum w J^T J as its 28 upper-
 * triangle entries row by row.  Per-pair terms in float32, sums in float64. */
int fl_reproj_residual_bwd(fl_ctx* ctx, int32_t n, const float* xyz, const float* uv,
                           const int32_t* kf_idx, int32_t n_kf, const float* kf_T, const fl_sim3* S,
                           const fl_pinhole* K /* host */, float huber_delta, double grad_scale,
                           double* g, double* H, hipStream_t stream);

/* The other direction of a loop match: a point X of the current side mapped
 * to the loop side by S^-1 and observed in keyframe k there,
 * r = pi(T_k S^-1 X) - uv.  fl_reproj_residual_fwd given the float32 form of
 * S^-1 (fl_sim3_inverse) computes these residuals, weights and loss.  This
 * backward takes that same form, S_inv, but returns g and H with respect to
 * the left perturbation of S itself (S^-1 <- S^-1 exp(-xi)):
 * J = dpi/dq R_k (-(1/s) R^T) [ -[X]x | I | X ], so the sums of both
 * directions add into one Gauss-Newton system for S (fl_gn_step).
 * Arguments, layouts and errors as fl_reproj_residual_bwd. */
int fl_reproj_residual_bwd_inv(fl_ctx* ctx, int32_t n, const float* xyz, const float* uv,
                               const int32_t* kf_idx, int32_t n_kf, const float* kf_T, const fl_sim3* S_inv,
                               const fl_pinhole* K /* host */, float huber_delta, double grad_scale,
                               double* g, double* H, hipStream_t stream);

/* S^-1 = (R^T, -R^T t / s, 1 / s) of S_in (device [13], float64) into
 * S_out (device [13], may be NULL) and its float32 form S32_out (device,
 * may be NULL; not both NULL).  Errors: FL_EINVAL for NULL arguments. */
int fl_sim3_inverse(fl_ctx* ctx, const double* S_in, double* S_out, fl_sim3* S32_out, hipStream_t stream);

/* S_out = exp(xi) S_in (float64, device [7], [13], [13]): the update of the
 * Sim3 refinement that follows matching (Sec. IV-C), with the closed-form
 * Sim3 exponential of Strasdat et al. (RSS 2010); S32_out (device, may be
 * NULL) receives the float32 search form.  Errors: FL_EINVAL for NULL
 * arguments. */
int fl_sim3_exp_mul(fl_ctx* ctx, const double* xi, const double* S_in, double* S_out, fl_sim3* S32_out,
                    hipStream_t stream);

/* Gradient of a loss L(S) with respect to the tangent coordinates xi of
 * S = exp(xi) S0 (the Sim3 refinement of Sec. IV-C differentiated with
 * respect to its parameters, Sec. IV-F): given g = dL/d(left perturbation
 * of S) from fl_reproj_residual_bwd at S, out = scale * J_l(xi)^T g, where
 * J_l(xi) = sum_k ad(xi)^k / (k+1)! is the Sim3 left Jacobian
 * (exp(xi + d) = exp(J_l(xi) d) exp(xi) to first order).  xi, g, out:
 * device float64 [7] in the order (omega, upsilon, sigma); scale: device
 * float64 [1], or NULL for 1.  The series is summed to float64 rounding for
 * |omega| <= pi and |sigma| of order one.  out may alias g.
 * Errors: FL_EINVAL for NULL xi, g or out. */
int fl_sim3_grad_xi(fl_ctx* ctx, const double* xi, const double* g, const double* scale, double* out,
                    hipStream_t stream);

/* One Gauss-Newton / Levenberg-Marquardt step of the Sim3 refinement
 * (Sec. IV-C; the paper's pose optimisation is Levenberg-Marquardt, Sec. VI):
 * solve (H + lambda diag(H)) d = -g
 * by float64 Cholesky (g [7], H [28] upper as above, device), then
 * S <- exp(d) S in place (device [13]) and S32 (device, may be NULL) <- its
 * float32 form.  A non-positive pivot leaves S unchanged. */
int fl_gn_step(fl_ctx* ctx, const double* g, const double* H, double lambda, double* S, fl_sim3* S32,
               hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Essential-graph optimisation (loop correction, Sec. III-B; graph
 * optimisation, Sec. IV-F).  Nodes are keyframe poses S_i (world -> camera
 * Sim3s, 13 doubles each: R row-major, t, s); an edge (i, j) measures
 * M_ij ~ S_j S_i^-1 and contributes e_ij = log(M_ij^-1 S_j S_i^-1) to
 * F = sum e^T e.  Nodes move by left perturbations S_i <- exp(d_i) S_i; the
 * Jacobians of e_ij are exact (J_j = J_l(e)^-1 Ad(M^-1),
 * J_i = -J_l(e)^-1 Ad(M^-1 S_j S_i^-1), J_l the Sim3 left Jacobian; the
 * paper obtains exact derivatives by automatic differentiation).  The poses
 * are optimised by `iters` Levenberg-Marquardt iterations (Sec. VI): each
 * solves (H + lambda diag H) d = -g at the accepted poses and evaluates F at
 * the candidate exp(d_i) S_i, which is taken if F decreases (lambda / 10,
 * at least 1e-12) and refused otherwise (lambda x 10, at most 1e12; the
 * linearisation is kept).  lambda = 0 takes every Gauss-Newton step.  The
 * solve is one of two (`solver`):
 *  - direct: the free nodes are renumbered by reverse Cuthill-McKee on the
 *    host; when no edge then spans more than FL_PGO_MAX_BAND_NODES - 1
 *    positions, the banded H is factored by float64 Cholesky in one
 *    workgroup and solved exactly (cg_used = 0; a pivot that is not
 *    positive reports -1 and refuses that iteration's candidate).  A band
 *    of at most 12 keyframes is factored through a window of rows in LDS,
 *    a wider one (several loops, for instance) with the band itself in
 *    device memory as the window; both take the same floating-point steps
 *    in the same order and give identical results where both apply;
 *  - block-Jacobi preconditioned conjugate gradients (at most cg_iters,
 *    stopping when |r| <= cg_tol |g|).  This solve runs one workgroup per
 *    compute unit, all resident together and synchronised by a grid
 *    barrier; other work on the device at the same time can keep them from
 *    being resident, and a barrier wait that runs past its bound in any
 *    workgroup reports the iteration as failed (cg_used = -1) and refuses
 *    its candidate instead of blocking.
 * A graph with no edges or no free node takes the conjugate gradients under
 * every setting.  Deterministic: every sum has a fixed order; the host
 * enqueues the same kernels every iteration and never waits for the
 * device (the damping and the decision stay in device memory). */
#define FL_PGO_MAX_BAND_NODES 64   /* widest band of the direct solver, in keyframes */
#define FL_PGO_SOLVER_AUTO 0       /* direct when the band fits, else conjugate gradients */
#define FL_PGO_SOLVER_CG 1
#define FL_PGO_SOLVER_DIRECT 2     /* FL_ERANGE when the band does not fit */
#define FL_PGO_SOLVER_DIRECT_WIDE 3   /* direct, with the device-memory window at every band width
                                         (FL_ERANGE when the band does not fit) */
typedef struct {
    int32_t n_nodes;
    int32_t n_edges;
    double* S;              /* device [n_nodes][13] in: start, out: optimised */
    const double* M;        /* device [n_edges][13] measured S_j S_i^-1 */
    const int32_t* edges;   /* host [n_edges][2] (i, j), i != j */
    const uint8_t* fixed;   /* host [n_nodes] nonzero: held; NULL: node 0 held */
} fl_pose_graph;

typedef struct {
    int32_t iters;          /* Levenberg-Marquardt iterations, 0..1000 */
    int32_t cg_iters;       /* 1..100000 */
    double lambda;          /* first damping, >= 0; 0: Gauss-Newton */
    double cg_tol;          /* >= 0 */
    double* cost;           /* device [iters + 1] (may be NULL): F of the accepted poses before each
                               iteration and after the last */
    int32_t* cg_used;       /* device [iters] (may be NULL): conjugate-gradient iterations of each
                               iteration (0 for a direct solve), -1: the solve failed */
    double* lambdas;        /* device [iters] (may be NULL): the damping each iteration solved with */
    uint8_t* accepted;      /* device [iters] (may be NULL): 1 when the iteration's candidate was taken */
    int32_t solver;         /* FL_PGO_SOLVER_* */
    int32_t reserved;       /* 0 */
} fl_pgo_params;

/* Errors: FL_EINVAL (NULL arrays, an edge outside the graph or joining a
 * node to itself, bad parameters), FL_ERANGE (sizes), FL_ENOMEM. */
int fl_pose_graph_optimize(fl_ctx* ctx, const fl_pose_graph* G /* host */, const fl_pgo_params* P /* host */,
                           hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Tuning of the batched search kernel.  Any tuning gives identical
 * results; fl_autotune times the candidates on the given batch (the stream
 * is synchronised) and keeps the fastest in the context. */
typedef struct {
    int32_t pairs_per_lane;  /* 1, 2 or 4: a tile is 1024 * pairs_per_lane pairs of one keyframe */
    int32_t lds_mode;        /* 2: keyframe grid, records and descriptors in LDS; 1: grid and
                                records in LDS, descriptors from HBM; 0: grids prebuilt in HBM.
                                A mode whose LDS footprint does not fit falls back to the next. */
    int32_t wg_per_cu;       /* 1 or 2 workgroups of 1024 threads per compute unit */
    int32_t xcd_aware;       /* 1: the tiles of a keyframe stay on one XCD (shared L2) */
} fl_tuning;

int fl_get_tuning(fl_ctx* ctx, fl_tuning* out /* host */);
int fl_set_tuning(fl_ctx* ctx, const fl_tuning* t /* host */);
int fl_autotune(fl_ctx* ctx, const fl_batch* B /* host */, const fl_params* P /* host */,
                const fl_fuse_out* out /* host */, int32_t reps, fl_tuning* best /* host, may be NULL */,
                float* best_ms /* host, may be NULL */, hipStream_t stream);

/* Optional per-call counters of the last batched search on this context
 * (pairs visible, grid cells scanned, keypoints scanned, descriptor
 * comparisons), enabled by fl_set_stats(ctx, 1); read after the stream
 * completes.  Counting costs time and is off by default. */
int fl_set_stats(fl_ctx* ctx, int enable);
int fl_get_stats(fl_ctx* ctx, int64_t* out4 /* host [4] */);

/* Kernel timing: when enabled, eager calls on this context record a pair of
 * HIP events on the launch stream around every search kernel
 * (FL_PROF_SEARCH) and every refinement kernel (FL_PROF_REFINE).
 * fl_get_profile waits for the last pair of the class `kernel` and returns
 * its summed kernel time in milliseconds and its number of launches since
 * profiling was enabled or the class was last read (then clears the class).
 * Graph launches are not timed. */
#define FL_PROF_SEARCH 0
#define FL_PROF_REFINE 1
int fl_set_profiling(fl_ctx* ctx, int enable);
int fl_get_profile(fl_ctx* ctx, int kernel, double* total_ms /* host */, int64_t* launches /* host */);

/* Measured VALU issue rate for roofline reporting (not a step of the
 * method): a kernel on every compute unit runs `iters` rounds of eight
 * independent v_xor_b32 + v_bcnt_u32_b32 chains per lane (the instructions
 * of the 256-bit Hamming distance), timed by HIP events on `stream`, which
 * is synchronised.  *lane_ops_per_s receives lanes x instructions per
 * second.  FL_ERANGE for iters outside [1, 2^20]; FL_ENOMEM / FL_EHIP from
 * the 4 KB sink allocation or the launch. */
int fl_valu_rate(fl_ctx* ctx, int32_t iters, double* lane_ops_per_s /* host */, hipStream_t stream);

/* Test hook: cap the provisional-ADD and matched-pair lists at `cap`
 * entries (0 restores the default) so that their overflow paths, full scans
 * of the pair outputs, run.  Results are unchanged. */
int fl_debug_set_list_cap(fl_ctx* ctx, int32_t cap);

/* Test hooks of the refinement's tagged partial sums (host-only, no GPU
 * needed): the 32-bit tag a launch with device epoch `epoch` gives step
 * `step` (0 <= step < 1000; the epoch is decremented by every table fetch,
 * so launch L of a context has epoch -L mod 2^32), and whether the partial
 * sums are zeroed before the launch numbered `launches` (1, 2, ... since the
 * last epoch reset).  Between two clears no two launches share a tag. */
uint32_t fl_debug_refine_tag(uint32_t epoch, int32_t step);
int fl_debug_refine_rows_cleared(uint32_t launches);

#ifdef __cplusplus
}
#endif
#endif /* FASTLOOP_H */
