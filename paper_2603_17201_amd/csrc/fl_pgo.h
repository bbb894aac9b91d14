// Essential-graph (Sim3 pose-graph) optimisation.
//
// Loop correction spreads the loop's Sim3 to every keyframe by optimising
// the essential graph (Sec. III-B, Sec. IV-F).  Nodes are keyframe poses S_i
// (world -> camera Sim3s); an edge (i, j) measures M_ij ~ S_j S_i^-1 and
// contributes e_ij = log(M_ij^-1 S_j S_i^-1) to F = sum e^T e.  Nodes move by
// left perturbations S_i <- exp(d_i) S_i.  The Jacobians are exact (the
// paper differentiates automatically): with E = M^-1 S_j S_i^-1 and
// e = log E, J_j = J_l(e)^-1 Ad(M^-1) and J_i = -J_l(e)^-1 Ad(E), J_l the
// Sim3 left Jacobian.  The poses are optimised by Levenberg-Marquardt
// (Sec. VI): an iteration solves (H + lambda diag H) d = -g at the accepted
// poses, evaluates F at the candidate exp(d_i) S_i and takes it when F
// decreases (lambda / 10; the next iteration relinearises) or refuses it
// (lambda x 10; the linearisation is kept).  The damping and the decision
// live in device memory, so the host enqueues the same kernels every
// iteration and never waits.
//
// Per iteration pgo_jacobian_kernel runs one thread per edge (it exits at
// once after a refusal), then one of two solves writes the candidate:
//  - direct (the paper's is a direct LDL^T): with the free nodes renumbered
//    so that every edge spans at most b positions (reverse Cuthill-McKee on
//    the host), H is a band of W = 7 (b + 1) scalars.  pgo_band_assemble_kernel
//    writes each band row from its node's incident edges;
//    pgo_band_solve_kernel, one workgroup, factors the band by Cholesky in
//    block columns of one keyframe (7 columns) with the forward substitution
//    folded in, keeping the W rows still being updated in an LDS window that
//    slides down the matrix, then back-substitutes by blocks of 7 rows
//    (pgo_band_solve_wide_kernel, for bands of more than 12 keyframes, keeps
//    the window in device memory instead);
//  - pgo_solve_kernel, one co-resident workgroup per CU synchronised by a
//    grid barrier, which gathers g and the diagonal blocks per node over its
//    incident edges (fixed order, no floating-point atomics) and runs block-
//    Jacobi preconditioned conjugate gradients with fixed-order float64
//    reductions.
// pgo_edge_cost_kernel then evaluates every edge at the candidate,
// pgo_decide_kernel sums F in a fixed order and decides, and
// pgo_accept_kernel copies an accepted candidate into the poses.

#pragma once

#include "fl_residual.h"

namespace fl {

constexpr int kPgoBlock = 256;      // threads of a solve workgroup (one per CU, all co-resident)
constexpr int kPgoJacBlock = 256;   // threads of a Jacobian workgroup
constexpr int kBandBlock = 512;     // threads of the band assembly and of the one band-solve workgroup
constexpr int kBandLdsNodes = 12;   // widest band, in keyframes, whose window the LDS holds
constexpr int kBandMaxW = 7 * kBandLdsNodes;   // widest band row of the LDS-window solve, in scalars
constexpr int kWideBlock = 1024;    // threads of the device-memory-window band solve
constexpr int kWideMaxW = 7 * FL_PGO_MAX_BAND_NODES;   // widest band row of any direct solve
constexpr int kWideRing = 512;      // right-hand-side ring of that solve (a power of two)
static_assert(kWideMaxW + 14 <= kWideRing && kWideMaxW <= kWideBlock, "one thread per window row");
static_assert(kBandLdsNodes <= FL_PGO_MAX_BAND_NODES, "the LDS window is the narrow case");
// entries per thread of the two parts of the band solve's trailing update
constexpr int kBandPart1 = (7 * (kBandMaxW - 7) + kBandBlock - 1) / kBandBlock;
constexpr int kBandPart2 = ((kBandMaxW - 14) * (kBandMaxW - 13) / 2 + kBandBlock - kWave - 1) / (kBandBlock - kWave);
static_assert(kBandMaxW <= kBandBlock, "one thread per band offset");

struct PgoArgs {
    int32_t n_nodes, n_edges;
    double* S;                  // [n_nodes][13] in/out
    const double* M;            // [n_edges][13]
    const int32_t* edges;       // [n_edges][2]
    const int32_t* adj_off;     // [n_nodes + 1] incident edges of each node
    const int32_t* adj;         // [2 n_edges] 2 * edge + (1 if the node is the edge's j)
    const uint8_t* fixed;       // [n_nodes]
    int32_t cg_iters;
    double cg_tol;
    int32_t step;               // outer step index (cost and count outputs)
    // workspace
    // Component-major layouts (entry, then edge or node), so that the
    // threads of a wave, which take consecutive edges or nodes, load
    // consecutive addresses.
    double* e;                  // [7][n_edges]
    double* J;                  // [2][49][n_edges]: J_i then J_j, entry 7 r + c of each
    double* u;                  // [7][n_edges] conjugate-gradient edge products
    double* vec;                // [6][7][n_nodes]: g, x, r, z, p, q
    double* Dfac;               // [49][n_nodes] LDL^T factors of the preconditioner blocks
    uint32_t* bar;              // grid-barrier counter, zero at launch
    double* red;                // [2][gridDim][4] reduction rows
    // direct solve: free nodes by band position, the band [Vs][W] (row R
    // holds columns R - W + 1 .. R, the diagonal last; H, then L in place),
    // the right-hand side (-g, then the forward solution) and the step
    int32_t band_w;             // W
    int32_t band_vs;            // Vs = 7 free nodes
    const int32_t* order;       // [Vs / 7] node of each position
    const int32_t* pos;         // [n_nodes] position of each node, -1 held
    double* band;
    double* rhs;                // [Vs]
    double* xs;                 // [Vs]
    // Levenberg-Marquardt state (device): lm[kLmLambda] damping of the next
    // solve, lm[kLmF] F of the accepted poses, lm[kLmRelin] 1 when the next
    // iteration relinearises, lm[kLmFail] set by a solve that failed,
    // lm[kLmUsed] conjugate-gradient iterations of the last solve,
    // lm[kLmTake] 1 when the last candidate was accepted
    double* lm;
    double* S_c;                // [n_nodes][13] candidate poses
    double* ecost;              // [n_edges] e^T e of each edge at the evaluated poses
    // outputs (may be null)
    double* cost;               // [iters + 1]
    int32_t* cg_used;           // [iters]
    double* lambdas;            // [iters]
    uint8_t* accepted;          // [iters]
};

enum : int { kLmLambda = 0, kLmF = 1, kLmRelin = 2, kLmFail = 3, kLmUsed = 4, kLmTake = 5, kLmWords = 8 };
constexpr double kLmLambdaMin = 1e-12, kLmLambdaMax = 1e12;

// A fixed-order block sum that may be called back to back (the closing
// barrier keeps the next call's partials from overwriting ones still read).
__device__ __forceinline__ double pgo_sum(double v, double* s_w) {
    const double sum = block_sum_f64(v, s_w);
    __syncthreads();
    return sum;
}

// e = log(M^-1 S_j S_i^-1)
__device__ inline void pgo_edge_error(const Sim3d& Si, const Sim3d& Sj, const Sim3d& Minv, double* e) {
    sim3_log(sim3_mul(Minv, sim3_mul(Sj, sim3_inv(Si))), e);
}

// The Sim3 left Jacobian J_l(x) = sum_k ad(x)^k / (k + 1)! of x = (w, u, sig)
// in its block form: with ad(x) = [[W, 0, 0], [U, W + sig I, -u], [0, 0, 0]]
// (W = [w]x, U = [u]x) every term T_k = ad(x) T_{k-1} / (k + 1) keeps the
// blocks T11, T21, T22 and the column t23 (rows 3..5 of column 6); the
// sum runs until a term's entries fall below 1e-18 of the sum's (at most
// 64 terms).  J = [[J11, 0, 0], [J21, J22, j23], [0, 0, 1]].
struct LeftJac {
    double J11[9], J21[9], J22[9], j23[3];
};

__device__ inline void mul33(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = fma(A[3 * i], B[j], fma(A[3 * i + 1], B[3 + j], A[3 * i + 2] * B[6 + j]));
}

__device__ inline void inv33(const double* A, double* B) {
    const double c0 = A[4] * A[8] - A[5] * A[7], c1 = A[5] * A[6] - A[3] * A[8], c2 = A[3] * A[7] - A[4] * A[6];
    const double id = 1.0 / (A[0] * c0 + A[1] * c1 + A[2] * c2);
    B[0] = c0 * id;
    B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    B[3] = c1 * id;
    B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    B[6] = c2 * id;
    B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

__device__ inline LeftJac sim3_left_jacobian(const double* x) {
    double W[9], Wd[9], U[9], W2[9];
    hat_sq(x[0], x[1], x[2], W, W2);
    hat_sq(x[3], x[4], x[5], U, W2);
    for (int i = 0; i < 9; ++i) Wd[i] = W[i] + ((i % 4 == 0) ? x[6] : 0.0);
    double T11[9], T21[9], T22[9], t23[3];
    LeftJac J;
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        T11[i] = T22[i] = J.J11[i] = J.J22[i] = I;
        T21[i] = J.J21[i] = 0.0;
    }
    for (int i = 0; i < 3; ++i) t23[i] = J.j23[i] = 0.0;
    for (int k = 1; k < 64; ++k) {
        const double f = 1.0 / (double)(k + 1);
        double N11[9], N21[9], N22[9], A[9], B[9], n23[3];
        mul33(W, T11, N11);
        mul33(U, T11, A);
        mul33(Wd, T21, B);
        for (int i = 0; i < 9; ++i) N21[i] = A[i] + B[i];
        mul33(Wd, T22, N22);
        for (int i = 0; i < 3; ++i) {
            n23[i] = fma(Wd[3 * i], t23[0], fma(Wd[3 * i + 1], t23[1], Wd[3 * i + 2] * t23[2]));
            if (k == 1) n23[i] -= x[3 + i];   // -u times row 6 of T_0 = I
        }
        double tmax = 0.0, jmax = 0.0;
        for (int i = 0; i < 9; ++i) {
            T11[i] = N11[i] * f;
            T21[i] = N21[i] * f;
            T22[i] = N22[i] * f;
            J.J11[i] += T11[i];
            J.J21[i] += T21[i];
            J.J22[i] += T22[i];
            tmax = fmax(tmax, fmax(fabs(T11[i]), fmax(fabs(T21[i]), fabs(T22[i]))));
            jmax = fmax(jmax, fmax(fabs(J.J11[i]), fmax(fabs(J.J21[i]), fabs(J.J22[i]))));
        }
        for (int i = 0; i < 3; ++i) {
            t23[i] = n23[i] * f;
            J.j23[i] += t23[i];
            tmax = fmax(tmax, fabs(t23[i]));
            jmax = fmax(jmax, fabs(J.j23[i]));
        }
        if (tmax <= 1e-18 * jmax) break;
    }
    return J;
}

// P = sign * J^-1 Ad(S) for J = J_l (block lower triangular as above) and
// Ad(S) = [[R, 0, 0], [[t]x R, sR, -t], [0, 0, 1]]: with K = J^-1,
// K11 = J11^-1, K22 = J22^-1, K21 = -K22 J21 K11, k23 = -K22 j23,
//   P11 = K11 R, P21 = K21 R + K22 [t]x R, P22 = s K22 R, p23 = k23 - K22 t,
// row 6 = e6 (times sign).  Written as the 7x7 row-major P.
__device__ inline void jl_inv_adjoint(const double* K11, const double* K21, const double* K22, const double* k23,
                                      const Sim3d& S, double sign, double* P) {
    double TR[9], Tx[9], W2[9], A[9], B[9];
    hat_sq(S.t[0], S.t[1], S.t[2], Tx, W2);
    mul33(Tx, S.R, TR);
    for (int i = 0; i < 49; ++i) P[i] = 0.0;
    mul33(K11, S.R, A);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) P[7 * r + c] = sign * A[3 * r + c];
    mul33(K21, S.R, A);
    mul33(K22, TR, B);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) P[7 * (3 + r) + c] = sign * (A[3 * r + c] + B[3 * r + c]);
    mul33(K22, S.R, A);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) P[7 * (3 + r) + 3 + c] = sign * S.s * A[3 * r + c];
        const double kt = fma(K22[3 * r], S.t[0], fma(K22[3 * r + 1], S.t[1], K22[3 * r + 2] * S.t[2]));
        P[7 * (3 + r) + 6] = sign * (k23[r] - kt);
    }
    P[48] = sign;
}

// e and the exact J_i, J_j of edge k (one thread per edge); nothing after a
// refused step (the linearisation at the accepted poses is kept).
__global__ __launch_bounds__(kPgoJacBlock) void pgo_jacobian_kernel(PgoArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_edges || a.lm[kLmRelin] == 0.0) return;
    const int i = a.edges[2 * k], j = a.edges[2 * k + 1];
    const Sim3d Minv = sim3_inv(sim3_load(a.M + 13 * (int64_t)k));
    const Sim3d Ed = sim3_mul(Minv, sim3_mul(sim3_load(a.S + 13 * (int64_t)j), sim3_inv(sim3_load(a.S + 13 * (int64_t)i))));
    double e[7];
    sim3_log(Ed, e);
    for (int r = 0; r < 7; ++r) a.e[(int64_t)r * a.n_edges + k] = e[r];
    const LeftJac J = sim3_left_jacobian(e);
    double K11[9], K22[9], K21[9], k23[3], A[9];
    inv33(J.J11, K11);
    inv33(J.J22, K22);
    mul33(J.J21, K11, A);
    mul33(K22, A, K21);
    for (int q = 0; q < 9; ++q) K21[q] = -K21[q];
    for (int r = 0; r < 3; ++r) k23[r] = -fma(K22[3 * r], J.j23[0], fma(K22[3 * r + 1], J.j23[1], K22[3 * r + 2] * J.j23[2]));
    double P[49];
    jl_inv_adjoint(K11, K21, K22, k23, Ed, -1.0, P);   // J_i = -J_l^-1 Ad(E)
    double* Ji = a.J + k;
    for (int q = 0; q < 49; ++q) Ji[(int64_t)q * a.n_edges] = P[q];
    jl_inv_adjoint(K11, K21, K22, k23, Minv, 1.0, P);  // J_j = J_l^-1 Ad(M^-1)
    double* Jj = a.J + (int64_t)49 * a.n_edges + k;
    for (int q = 0; q < 49; ++q) Jj[(int64_t)q * a.n_edges] = P[q];
}

// y += J^T v with J's entry 7 r + c at J[(7 r + c) st] and v's entry r at
// v[r st] (the component-major layouts)
__device__ __forceinline__ void add_JTv(const double* J, const double* v, int64_t st, double* y) {
    double vr[7];
    for (int r = 0; r < 7; ++r) vr[r] = v[r * st];
    for (int c = 0; c < 7; ++c) {
        double s = y[c];
        for (int r = 0; r < 7; ++r) s = fma(J[(7 * r + c) * st], vr[r], s);
        y[c] = s;
    }
}

// LDL^T of a 7x7 symmetric positive-definite block (row-major, in place: L
// below the diagonal, D on it); returns false for a pivot that is not
// positive.
__device__ inline bool ldl7(double* A) {
    for (int j = 0; j < 7; ++j) {
        double dj = A[8 * j];
        for (int m = 0; m < j; ++m) dj -= A[7 * j + m] * A[7 * j + m] * A[8 * m];
        if (!(dj > 0.0)) return false;
        A[8 * j] = dj;
        for (int i = j + 1; i < 7; ++i) {
            double v = A[7 * i + j];
            for (int m = 0; m < j; ++m) v -= A[7 * i + m] * A[7 * j + m] * A[8 * m];
            A[7 * i + j] = v / dj;
        }
    }
    return true;
}

__device__ inline void ldl7_solve(const double* F, const double* b, double* x) {
    double y[7];
    for (int i = 0; i < 7; ++i) {
        double v = b[i];
        for (int m = 0; m < i; ++m) v -= F[7 * i + m] * y[m];
        y[i] = v;
    }
    for (int i = 6; i >= 0; --i) {
        double v = y[i] / F[8 * i];
        for (int m = i + 1; m < 7; ++m) v -= F[7 * m + i] * x[m];
        x[i] = v;
    }
}

// Grid-wide barrier of the solve kernel's co-resident workgroups: a
// counter that every workgroup increments once per barrier (zeroed before
// the launch), with device-scope release and acquire around it so that the
// vectors written before it are visible on every XCD after it.  The wait is
// bounded: on a timeout the kernel reports failure instead of hanging.
__device__ inline bool pgo_grid_sync(uint32_t* bar, uint32_t target) {
    __shared__ int s_ok;
    __syncthreads();
    if (gridDim.x == 1) return true;   // one workgroup: its own barrier is enough
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this workgroup's writes, before the count
        atomicAdd(bar, 1u);
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpinLimit) {
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every workgroup's writes, after the count
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Fixed-order grid sum of up to 4 values: each workgroup's block sums go to
// its row of red[buf], then every workgroup adds the rows in workgroup order
// (all of them end with the same bits).  Consecutive reductions alternate
// between two row buffers: a buffer is written again only after the barrier
// that follows every workgroup's reading of it.
template <int NV>
__device__ inline bool pgo_grid_sum(double* v, double* red, int buf, uint32_t* bar, uint32_t& seq, double* s_w) {
    double tot[NV];
    for (int i = 0; i < NV; ++i) tot[i] = pgo_sum(v[i], s_w);
    const int G = gridDim.x;
    double* rows = red + (size_t)buf * 4 * G;
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) rows[4 * blockIdx.x + i] = tot[i];
    if (!pgo_grid_sync(bar, ++seq * (uint32_t)G)) return false;
    for (int i = 0; i < NV; ++i) {
        double sum = 0.0;
        for (int w = 0; w < G; ++w) sum += rows[4 * w + i];
        v[i] = sum;
    }
    return true;
}

// One outer step after the Jacobians: cost, g and the preconditioner blocks
// node by node, the conjugate gradients, the node update.  Every workgroup
// of the grid takes part; nodes and edges are spread over all threads.
__global__ __launch_bounds__(kPgoBlock) void pgo_solve_kernel(PgoArgs a) {
    __shared__ double s_w[kPgoBlock / kWave];
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x, gnt = gridDim.x * blockDim.x;
    const int N = a.n_nodes, E = a.n_edges;
    const int64_t V = 7 * (int64_t)N;
    double* g = a.vec;
    double* x = a.vec + V;
    double* r = a.vec + 2 * V;
    double* z = a.vec + 3 * V;
    double* p = a.vec + 4 * V;
    double* q = a.vec + 5 * V;
    uint32_t seq = 0;
    int rb = 0;   // row buffer of the next reduction
    bool ok = true;

    const double lambda = a.lm[kLmLambda];
    // g, preconditioner blocks, r = -g, z = M^-1 r, p = z
    double red3[3] = {0.0, 0.0, 0.0};   // (unused), |g|^2, r.z
    for (int n = gtid; n < N; n += gnt) {
        double gn[7] = {0, 0, 0, 0, 0, 0, 0};
        double D[49];
        for (int t = 0; t < 49; ++t) D[t] = 0.0;
        if (!a.fixed[n]) {
            for (int t = a.adj_off[n]; t < a.adj_off[n + 1]; ++t) {
                const int k = a.adj[t] >> 1, side = a.adj[t] & 1;
                const double* Jk = a.J + (int64_t)49 * side * E + k;
                add_JTv(Jk, a.e + k, E, gn);
                double Jl[49];
                for (int q2 = 0; q2 < 49; ++q2) Jl[q2] = Jk[(int64_t)q2 * E];
                for (int c1 = 0; c1 < 7; ++c1)
                    for (int c2 = 0; c2 < 7; ++c2) {
                        double s = D[7 * c1 + c2];
                        for (int rr = 0; rr < 7; ++rr) s = fma(Jl[7 * rr + c1], Jl[7 * rr + c2], s);
                        D[7 * c1 + c2] = s;
                    }
            }
            for (int c = 0; c < 7; ++c) D[8 * c] *= 1.0 + lambda;
            if (!ldl7(D)) {
                // no information on this node: hold it
                for (int t = 0; t < 49; ++t) D[t] = 0.0;
                for (int c = 0; c < 7; ++c) {
                    D[8 * c] = 1.0;
                    gn[c] = 0.0;
                }
            }
        } else {
            for (int c = 0; c < 7; ++c) D[8 * c] = 1.0;
        }
        for (int t = 0; t < 49; ++t) a.Dfac[(int64_t)t * N + n] = D[t];
        double rn[7], zn[7];
        for (int c = 0; c < 7; ++c) rn[c] = -gn[c];
        ldl7_solve(D, rn, zn);
        for (int c = 0; c < 7; ++c) {
            g[(int64_t)c * N + n] = gn[c];
            x[(int64_t)c * N + n] = 0.0;
            r[(int64_t)c * N + n] = rn[c];
            z[(int64_t)c * N + n] = zn[c];
            p[(int64_t)c * N + n] = zn[c];
            red3[1] = fma(gn[c], gn[c], red3[1]);
            red3[2] = fma(rn[c], zn[c], red3[2]);
        }
    }
    ok = pgo_grid_sum<3>(red3, a.red, rb, a.bar, seq, s_w);
    rb ^= 1;
    const double gnorm2 = red3[1];
    double rz = red3[2];

    // Conjugate gradients on H x = -g over the free nodes (fixed nodes keep
    // p = r = z = 0).  The direction update p = z + beta p of an iteration is
    // folded into the next: its edge products use z + beta p directly, and
    // each node's p is rewritten in the node phase that follows.
    int used = 0;
    double beta = 0.0;
    const double stop2 = a.cg_tol * a.cg_tol * gnorm2;
    for (int it = 0; ok && it < a.cg_iters && gnorm2 > 0.0; ++it) {
        // u_k = J_i p'_i + J_j p'_j with p' = z + beta p (p' = p at it = 0)
        for (int k = gtid; k < E; k += gnt) {
            const int i = a.edges[2 * k], j = a.edges[2 * k + 1];
            const double* Ji = a.J + k;
            const double* Jj = a.J + (int64_t)49 * E + k;
            double pi[7], pj[7];
            for (int c = 0; c < 7; ++c) {
                const int64_t ci = (int64_t)c * N + i, cj = (int64_t)c * N + j;
                pi[c] = it ? fma(beta, p[ci], z[ci]) : p[ci];
                pj[c] = it ? fma(beta, p[cj], z[cj]) : p[cj];
            }
            for (int rr = 0; rr < 7; ++rr) {
                double s = 0.0;
                for (int c = 0; c < 7; ++c) s = fma(Ji[(int64_t)(7 * rr + c) * E], pi[c], s);
                for (int c = 0; c < 7; ++c) s = fma(Jj[(int64_t)(7 * rr + c) * E], pj[c], s);
                a.u[(int64_t)rr * E + k] = s;
            }
        }
        ok = pgo_grid_sync(a.bar, ++seq * (uint32_t)gridDim.x);
        if (!ok) break;
        // p_n = p'_n; q_n = sum over incident edges of J^T u (+ lambda diag H p)
        double pq[1] = {0.0};
        for (int n = gtid; n < N; n += gnt) {
            double pn[7], qn[7] = {0, 0, 0, 0, 0, 0, 0};
            for (int c = 0; c < 7; ++c) {
                const int64_t cn = (int64_t)c * N + n;
                pn[c] = it ? fma(beta, p[cn], z[cn]) : p[cn];
                p[cn] = pn[c];
            }
            if (!a.fixed[n]) {
                double dg[7] = {0, 0, 0, 0, 0, 0, 0};
                for (int t = a.adj_off[n]; t < a.adj_off[n + 1]; ++t) {
                    const int k = a.adj[t] >> 1, side = a.adj[t] & 1;
                    const double* Jk = a.J + (int64_t)49 * side * E + k;
                    add_JTv(Jk, a.u + k, E, qn);
                    if (lambda > 0.0)
                        for (int c = 0; c < 7; ++c)
                            for (int rr = 0; rr < 7; ++rr) {
                                const double jv = Jk[(int64_t)(7 * rr + c) * E];
                                dg[c] = fma(jv, jv, dg[c]);
                            }
                }
                if (lambda > 0.0)
                    for (int c = 0; c < 7; ++c) qn[c] = fma(lambda * dg[c], pn[c], qn[c]);
            }
            for (int c = 0; c < 7; ++c) {
                q[(int64_t)c * N + n] = qn[c];
                pq[0] = fma(pn[c], qn[c], pq[0]);
            }
        }
        ok = pgo_grid_sum<1>(pq, a.red, rb, a.bar, seq, s_w);
        rb ^= 1;
        if (!ok || !(pq[0] > 0.0)) break;
        const double alpha = rz / pq[0];
        double red2[2] = {0.0, 0.0};   // |r|^2, r.z
        for (int n = gtid; n < N; n += gnt) {
            double rn[7], zn[7];
            for (int c = 0; c < 7; ++c) {
                const int64_t cn = (int64_t)c * N + n;
                x[cn] = fma(alpha, p[cn], x[cn]);
                rn[c] = fma(-alpha, q[cn], r[cn]);
                r[cn] = rn[c];
                red2[0] = fma(rn[c], rn[c], red2[0]);
            }
            double F[49];
            for (int t = 0; t < 49; ++t) F[t] = a.Dfac[(int64_t)t * N + n];
            ldl7_solve(F, rn, zn);
            for (int c = 0; c < 7; ++c) {
                const double zc = a.fixed[n] ? 0.0 : zn[c];
                z[(int64_t)c * N + n] = zc;
                red2[1] = fma(rn[c], zc, red2[1]);
            }
        }
        ok = pgo_grid_sum<2>(red2, a.red, rb, a.bar, seq, s_w);
        rb ^= 1;
        if (!ok) break;
        used = it + 1;
        if (red2[0] <= stop2) break;
        beta = red2[1] / rz;
        rz = red2[1];
    }
    // Any workgroup whose barrier wait ran out marks the solve failed; the
    // decision, a later kernel, then refuses the candidate whatever the
    // other workgroups wrote.
    if (!ok) {
        if (threadIdx.x == 0) a.lm[kLmFail] = 1.0;
        return;
    }
    if (gtid == 0) a.lm[kLmUsed] = (double)used;
    // candidate C_n = exp(x_n) S_n (each node by the thread that owns it)
    for (int n = gtid; n < N; n += gnt) {
        const Sim3d Sn = sim3_load(a.S + 13 * (int64_t)n);
        if (a.fixed[n]) {
            sim3_store(Sn, a.S_c + 13 * (int64_t)n);
            continue;
        }
        double d[7];
        for (int c = 0; c < 7; ++c) d[c] = x[(int64_t)c * N + n];
        sim3_store(sim3_mul(sim3_exp(d), Sn), a.S_c + 13 * (int64_t)n);
    }
}

// Row R = 7 P + r of the band (free node n at position P): entries
// (J_a^T J_a)[r][c <= r] over the node's edges on the diagonal block, and
// (J_a^T J_b)[r][.] of each edge to a free node m at an earlier position in
// block (P, pos m); lambda scales the diagonal; rhs = -g.  A node without
// edges is held (unit diagonal, zero right-hand side).  Each thread owns its
// row, so the sums take the incident edges in their fixed order.
__global__ __launch_bounds__(kBandBlock) void pgo_band_assemble_kernel(PgoArgs a) {
    const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (R >= a.band_vs) return;
    const int W = a.band_w, w = W - 1, E = a.n_edges;
    const int P = (int)(R / 7), r = (int)(R % 7);
    const int n = a.order[P];
    double* row = a.band + R * W;
    for (int o = 0; o < W; ++o) row[o] = 0.0;
    double gr = 0.0;
    for (int t = a.adj_off[n]; t < a.adj_off[n + 1]; ++t) {
        const int k = a.adj[t] >> 1, side = a.adj[t] & 1;
        const int m = a.edges[2 * k + 1 - side];
        const double* Ja = a.J + (int64_t)49 * side * E + k;
        const double* Jb = a.J + (int64_t)49 * (1 - side) * E + k;
        double ja[7];
        for (int rr = 0; rr < 7; ++rr) {
            ja[rr] = Ja[(int64_t)(7 * rr + r) * E];
            gr = fma(ja[rr], a.e[(int64_t)rr * E + k], gr);
        }
        for (int c = 0; c <= r; ++c) {
            double v = 0.0;
            for (int rr = 0; rr < 7; ++rr) v = fma(ja[rr], Ja[(int64_t)(7 * rr + c) * E], v);
            row[c - r + w] += v;
        }
        const int pm = a.pos[m];
        const int64_t base = 7 * (int64_t)pm - R + w;
        if (pm >= 0 && pm < P && base >= 0) {
            for (int c = 0; c < 7; ++c) {
                double v = 0.0;
                for (int rr = 0; rr < 7; ++rr) v = fma(ja[rr], Jb[(int64_t)(7 * rr + c) * E], v);
                row[base + c] += v;
            }
        }
    }
    if (a.adj_off[n] == a.adj_off[n + 1]) {
        row[w] = 1.0;
        gr = 0.0;
    } else {
        row[w] *= 1.0 + a.lm[kLmLambda];
    }
    a.rhs[R] = -gr;
}

// Barrier for LDS traffic only: waits for this wave's LDS operations, not
// for its outstanding global loads (the prefetches below stay in flight
// across it).  Global data is exchanged between threads only across a full
// __syncthreads().
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Row stride, in doubles, of the band solve's LDS window: even, so that
// the entries of one band column in consecutive rows (W - 1 apart in the
// band layout, W + 1 or W apart with the padding) fall in different banks.
__host__ __device__ constexpr int band_win_stride(int W) { return (W | 1) + 1; }

// Dynamic LDS of the band solve: the window, the right-hand-side ring, and
// the staged rows of the next block with their right-hand sides.
__host__ __device__ constexpr size_t band_solve_lds_bytes(int W) {
    return sizeof(double) * ((size_t)W * band_win_stride(W) + (W + 1) + 7 * (size_t)W + 7);
}

// A float64 value of lane l (l wave-uniform).
__device__ __forceinline__ double readlane_f64(double x, int l) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The candidate poses of a direct solve: S_n <- exp(x_n) S_n for every free
// node (x in a.xs, by band position), held nodes copied.
__device__ inline void band_candidate_poses(const PgoArgs& a) {
    for (int n = threadIdx.x; n < a.n_nodes; n += blockDim.x) {
        const int P = a.pos[n];
        const Sim3d Sn = sim3_load(a.S + 13 * (int64_t)n);
        if (P < 0) {
            sim3_store(Sn, a.S_c + 13 * (int64_t)n);
            continue;
        }
        double dn[7];
        for (int c = 0; c < 7; ++c) dn[c] = a.xs[7 * (int64_t)P + c];
        sim3_store(sim3_mul(sim3_exp(dn), Sn), a.S_c + 13 * (int64_t)n);
    }
}

// Back substitution L^T x = y (L and y in device memory, visible to the
// whole workgroup), by blocks of 7 rows from the last: wave 0 solves the
// block's 7 unknowns, lane l holding row l's running right-hand side
// (x_i = s_i / L(i,i), then s_l -= L(i,l) x_i for the block's earlier rows),
// then thread u subtracts the block's 7 products from the running
// right-hand side of row r0 - w + u.  The running right-hand sides of the
// rows still open, [r0 - w, r0 + 6] at block K, live in an LDS ring of
// RM + 1 >= W + 14 entries (RM + 1 a power of two); x goes to a.xs.  Each
// s_j takes its products in falling row order, one fused multiply-add each,
// each block's loads issued two blocks ahead.  Needs w < blockDim.x and 7
// doubles of LDS at sX.
__device__ inline void band_back_substitute(const PgoArgs& a, double* sB, int RM, double* sX) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int W = a.band_w, w = W - 1, Vs = a.band_vs;
    const int NB = Vs / 7;
    {
        const int lo = 7 * (NB - 1) - w < 0 ? 0 : 7 * (NB - 1) - w;
        for (int j = lo + tid; j < Vs; j += nth) sB[j & RM] = a.rhs[j];
    }
    // this thread's loads for block K: wave 0 lane l < 7 the block's column l
    // (Lc[ii] = L(r0 + ii, r0 + l), ii > l) and L(r0 + l, r0 + l); thread
    // u < w the block's entries of row j = r0 - w + u (zero outside the band)
    // and, for u < 7, the y of the row entering the window next.  Two sets,
    // for the blocks alternately, each loaded two blocks ahead; nothing is
    // computed from the loaded values until the block is solved, so no load
    // is waited for early.
    struct Set {
        double Lc[7], dg, Lr[7], ye;
    };
    auto load_block = [&](int K, Set& st) {
        const int r0 = 7 * K;
#pragma unroll
        for (int ii = 0; ii < 7; ++ii) {
            st.Lc[ii] = tid < 7 && ii > tid ? a.band[(int64_t)(r0 + ii) * W + w - (ii - tid)] : 0.0;
            const int j = r0 - w + tid;
            st.Lr[ii] = tid < w && j >= 0 && ii <= tid ? a.band[(int64_t)(r0 + ii) * W + w - (r0 + ii - j)] : 0.0;
        }
        st.dg = tid < 7 ? a.band[(int64_t)(r0 + tid) * W + w] : 1.0;
        const int je = r0 - 7 - w + tid;
        st.ye = tid < 7 && je >= 0 ? a.rhs[je] : 0.0;
    };
    auto block = [&](int K, const Set& st) {
        const int r0 = 7 * K;
        if (tid < kWave) {
            const int l = tid;
            const double dinv = 1.0 / st.dg;   // lanes 0 .. 6: 1 / L(r0 + l, r0 + l)
            double sl = l < 7 ? sB[(r0 + l) & RM] : 0.0;
#pragma unroll
            for (int ii = 6; ii >= 0; --ii) {
                const double xi = readlane_f64(sl, ii) * readlane_f64(dinv, ii);
                if (l < ii) sl = fma(-st.Lc[ii], xi, sl);
                if (l == ii) {
                    a.xs[r0 + ii] = xi;
                    sX[ii] = xi;
                }
            }
        }
        lds_barrier();
        if (tid < w && r0 - w + tid >= 0) {
            const int j = r0 - w + tid;
            double s = sB[j & RM];
#pragma unroll
            for (int ii = 6; ii >= 0; --ii) s = fma(-st.Lr[ii], sX[ii], s);
            sB[j & RM] = s;
        }
        if (tid < 7 && r0 - 7 - w + tid >= 0) sB[(r0 - 7 - w + tid) & RM] = st.ye;
    };
    Set A, B;
    load_block(NB - 1, A);
    if (NB >= 2) load_block(NB - 2, B);
    __syncthreads();
    for (int K = NB - 1; K >= 0; K -= 2) {
        block(K, A);
        if (K >= 2) load_block(K - 2, A);
        lds_barrier();
        if (K == 0) break;
        block(K - 1, B);
        if (K >= 3) load_block(K - 3, B);
        lds_barrier();
    }
    __syncthreads();   // every x in device memory
}

// The banded Cholesky H = L L^T with L y = rhs solved alongside, L^T x = y,
// and S_n <- exp(x_n) S_n, in one workgroup.
//
// Factorisation by block columns of 7 (one keyframe): every edge joins
// keyframes at most b positions apart, so block column K (columns 7K ..
// 7K + 6) has entries in rows 7K .. 7K + W - 1 only, the W rows the LDS
// window holds (row R in slot R mod W, its W band entries).  Per block:
//  1. one wave factors the panel (those W rows by 7 columns) in registers,
//     lane t holding row t (and t + 64): column by column, the pivot comes
//     from the diagonal lane, the rows below are scaled and the panel's later
//     columns and the right-hand sides are updated, with the values of one
//     lane read by all (readlane) and no barrier;
//  2. the workgroup subtracts the panel's rank-7 product from the window's
//     remaining triangle, while the finished rows 7K .. 7K + 6 go back to
//     HBM and the rows of block K + b + 1, staged during the previous step,
//     take their slots.  With look-ahead, the entries of the next panel's
//     columns are updated first, and the rest of the triangle while wave 0
//     factors that next panel (step 1 of block K + 1).
// Every entry sees the same fused multiply-adds, in the same order, as a
// column-by-column factorisation: two barriers per block instead of two per
// column.  Back substitution goes by blocks of 7 rows (band_back_substitute),
// its running right-hand sides in a ring over the window's LDS.
__global__ __launch_bounds__(kBandBlock) void pgo_band_solve_kernel(PgoArgs a) {
    extern __shared__ __align__(16) unsigned char s_mem[];
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    const int W = a.band_w, w = W - 1, Vs = a.band_vs;
    const int Ws = band_win_stride(W);
    double* win = (double*)s_mem;      // [W][Ws]
    double* sv = win + W * Ws;         // [W + 1]
    double* stg = sv + W + 1;          // [7 W] the rows of the block that enters next
    double* stgb = stg + 7 * W;        // [7] and their right-hand sides

    // This thread's entries (i, j), i >= j, of a block's trailing triangle
    // (local rows of the block's window), in two parts: the 7 columns that
    // form the next panel (7 <= j <= 13), over the whole workgroup, and the
    // rest (j >= 14), over waves 1 .. 7 while wave 0 factors that panel.
    // Packed as i << 8 | j, -1: none.
    int pk1[kBandPart1], pk2[kBandPart2];
    {
        const int n1 = 7 * (W - 7);   // i - 7 in [0, W - 8], j - 7 in [0, 6], j > i skipped
#pragma unroll
        for (int q = 0; q < kBandPart1; ++q) {
            const int t = tid + q * kBandBlock;
            const int i = 7 + t / 7, j = 7 + t % 7;
            pk1[q] = t < n1 && j <= i ? (i << 8 | j) : -1;
        }
        const int m = W - 14;   // the triangle 14 <= j <= i < W
        const int n2 = m > 0 ? m * (m + 1) / 2 : 0;
#pragma unroll
        for (int q = 0; q < kBandPart2; ++q) {
            const int t = tid - kWave + q * (kBandBlock - kWave);
            pk2[q] = -1;
            if (tid >= kWave && t < n2) {
                int ra = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
                while (ra * (ra + 1) / 2 > t) --ra;
                while ((ra + 1) * (ra + 2) / 2 <= t) ++ra;
                pk2[q] = (14 + ra) << 8 | (14 + t - ra * (ra + 1) / 2);
            }
        }
    }
    for (int idx = tid; idx < W * W; idx += kBandBlock) {
        const int R = idx / W;
        win[R * Ws + idx % W] = R < Vs ? a.band[(int64_t)R * W + idx % W] : 0.0;
    }
    for (int idx = tid; idx < W; idx += kBandBlock) sv[idx] = idx < Vs ? a.rhs[idx] : 0.0;
    if (tid == 0) s_fail = 0;
    __syncthreads();

    // The panel of block K (window rows from slot s0), by wave 0: lane t
    // holds row t (and t + 64); column by column, the pivot comes from the
    // diagonal lane, the rows below are scaled and the panel's later columns
    // and the right-hand sides are updated, with the values of one lane read
    // by all (readlane) and no barrier.
    auto panel = [&](int K, int s0) {
        const int r0 = 7 * K;
        const int t = tid, t2 = tid + kWave;
        int sa = s0 + t;   // below 2 W
        if (sa >= W) sa -= W;
        int sb = s0 + t2;  // below 3 W when W < 2 x 64
        if (sb >= W) sb -= W;
        if (sb >= W) sb -= W;
        const bool ha = t < W && r0 + t < Vs, hb = t2 < W && r0 + t2 < Vs;
        double p[7], p2[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            p[c] = ha && c <= t ? win[sa * Ws + w + c - t] : 0.0;
            p2[c] = hb ? win[sb * Ws + w + c - t2] : 0.0;
        }
        double b1 = ha ? sv[sa] : 0.0, b2 = hb ? sv[sb] : 0.0;
        bool okp = true;
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            const double d = readlane_f64(p[c], c);
            okp = okp && d > 0.0;   // the same in every lane; a failed block is discarded whole
            // 1 / sqrt(d) from the hardware estimate and two Newton steps
            // (a short dependency chain on this serial path), sqrt(d) =
            // d / sqrt(d)
            double ird = __builtin_amdgcn_rsq(d);
#pragma unroll
            for (int it = 0; it < 2; ++it) {
                const double e = fma(-d * ird, ird, 1.0);
                ird = fma(0.5 * ird, e, ird);
            }
            const double rd = d * ird;
            const double yc = readlane_f64(b1, c) * ird;
            if (t == c) {
                p[c] = rd;
                b1 = yc;
            } else if (t > c) {
                p[c] *= ird;
                b1 = fma(-p[c], yc, b1);
            }
            p2[c] *= ird;
            b2 = fma(-p2[c], yc, b2);
#pragma unroll
            for (int j = c + 1; j < 7; ++j) {
                const double ljc = readlane_f64(p[c], j);   // L(j, c)
                if (t >= j) p[j] = fma(-p[c], ljc, p[j]);
                p2[j] = fma(-p2[c], ljc, p2[j]);
            }
        }
        if (!okp) {
            if (t == 0) s_fail = 1;
        } else {
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                if (ha && c <= t) win[sa * Ws + w + c - t] = p[c];
                if (hb) win[sb * Ws + w + c - t2] = p2[c];
            }
            if (ha) sv[sa] = b1;
            if (hb) sv[sb] = b2;
        }
    };
    // Rows 7K + W .. 7K + W + 6 (block K + b + 1, entering the window at the
    // end of block K) into the staging rows, by waves 1 .. 7.
    auto stage = [&](int K) {
        const int r = 7 * K + W;
        for (int idx = tid - kWave; idx < 7 * W; idx += kBandBlock - kWave) {
            const int q = idx / W, e = idx - q * W;
            stg[idx] = r + q < Vs ? a.band[(int64_t)(r + q) * W + e] : 0.0;
        }
        if (tid - kWave < 7) stgb[tid - kWave] = r + tid - kWave < Vs ? a.rhs[r + tid - kWave] : 0.0;
    };
    // Entries of block K's trailing triangle, all read and computed before
    // any is written back (a store could otherwise be taken to alias the
    // next entry's loads and serialise them); the panel columns they read
    // are not written meanwhile.
    auto update = [&](const int* pk, auto NP, int r0, int s0) {
        double nv[decltype(NP)::value];
        int at[decltype(NP)::value];
#pragma unroll
        for (int q = 0; q < decltype(NP)::value; ++q) {
            at[q] = -1;
            if (pk[q] < 0) continue;
            const int i = pk[q] >> 8, j = pk[q] & 255;
            if (r0 + i >= Vs) continue;
            int si = s0 + i, sj = s0 + j;   // both below 2 W
            if (si >= W) si -= W;
            if (sj >= W) sj -= W;
            const double* Li = win + si * Ws + w - i;   // Li[c] = L(7K + i, 7K + c)
            const double* Lj = win + sj * Ws + w - j;
            at[q] = si * Ws + w - (i - j);
            double av = win[at[q]];
#pragma unroll
            for (int c = 0; c < 7; ++c) av = fma(-Li[c], Lj[c], av);
            nv[q] = av;
        }
#pragma unroll
        for (int q = 0; q < decltype(NP)::value; ++q)
            if (at[q] >= 0) win[at[q]] = nv[q];
    };

    // Per block K, with look-ahead: 1. the whole workgroup updates the
    // entries of the next panel's columns, writes the finished rows 7K ..
    // 7K + 6 back to HBM and moves the staged rows into their slots; 2. wave
    // 0 factors the panel of block K + 1 while waves 1 .. 7 stage the rows
    // that enter after it and update the rest of block K's triangle (no
    // entry either side reads is written by the other).  Two LDS-only
    // barriers per block; the row stores stay in flight across them.
    const int NB = Vs / 7;
    if (tid < kWave) panel(0, 0);
    else stage(0);
    lds_barrier();
    int s0 = 0;   // slot of row 7K
    for (int K = 0; K < NB && !s_fail; ++K) {
        const int r0 = 7 * K;
        update(pk1, std::integral_constant<int, kBandPart1>{}, r0, s0);
        for (int idx = tid; idx < 7 * W; idx += kBandBlock) {
            const int q = idx / W, e = idx - q * W;
            if (r0 + q >= Vs) continue;
            int sq = s0 + q;
            if (sq >= W) sq -= W;
            a.band[(int64_t)(r0 + q) * W + e] = win[sq * Ws + e];
            win[sq * Ws + e] = stg[idx];
        }
        if (tid < 7 && r0 + tid < Vs) {
            int sq = s0 + tid;
            if (sq >= W) sq -= W;
            a.rhs[r0 + tid] = sv[sq];
            sv[sq] = stgb[tid];
        }
        lds_barrier();
        int s1 = s0 + 7;
        if (s1 >= W) s1 -= W;
        if (tid < kWave) {
            if (K + 1 < NB) panel(K + 1, s1);
        } else {
            if (K + 1 < NB) stage(K + 1);
            update(pk2, std::integral_constant<int, kBandPart2>{}, r0, s0);
        }
        lds_barrier();   // s_fail is read at the loop's test, the same in every thread
        s0 = s1;
    }
    if (s_fail) {   // the same in every thread
        if (tid == 0) a.lm[kLmFail] = 1.0;
        return;
    }
    if (tid == 0) a.lm[kLmUsed] = 0.0;
    __syncthreads();   // L and y in global memory, visible to every thread

    // Back substitution by blocks of 7 rows, the running right-hand sides
    // in a ring over the window's LDS (W + 14 <= 128 entries)
    int ring = 16;
    while (ring < W + 14) ring *= 2;
    band_back_substitute(a, win, ring - 1, sv);
    band_candidate_poses(a);
}

// The same banded Cholesky for bands too wide for an LDS window (up to
// FL_PGO_MAX_BAND_NODES keyframes): the band itself, in device memory (the
// active rows stay in L2), is the window, updated in place, in one workgroup
// of kWideBlock threads.  Per block column K (rows r0 = 7K ..):
//  A. thread t holds window row r0 + t's 7 panel entries and right-hand side;
//     wave 0 factors the 7 x 7 diagonal block exactly as the LDS solve's
//     panel wave does and publishes 1 / L(c,c), y_c and L(j,c) in LDS, from
//     which the other rows finish (the same fused multiply-adds in the same
//     order as in that wave); the finished entries go to device memory and
//     the panel to LDS;
//  B. the workgroup subtracts the panel's rank-7 product from the window's
//     trailing triangle, read and written in device memory in tiles of 4 x 4
//     entries, consecutive threads on consecutive tiles of a tile row; the
//     entries that form the next panel are also kept in LDS, so the next
//     step A reads its rows from LDS (only the rows entering the window come
//     from device memory, loaded during this step).
// Back substitution as in the LDS-window solve (band_back_substitute).
// Every entry, right-hand side and unknown sees the same fused multiply-adds,
// in the same order, as in the LDS-window solve, so the two give identical
// results on any band both take.
__global__ __launch_bounds__(kWideBlock) void pgo_band_solve_wide_kernel(PgoArgs a) {
    constexpr int MW = kWideMaxW, RM = kWideRing - 1;
    constexpr int PW = MW + 8;      // panel column stride: row t at t + 1, so rows 8, 12, .. start 32-byte units
    __shared__ __align__(16) double sP[7 * PW];   // the panel by column: sP[c PW + t + 1] = L(r0 + t, r0 + c)
    __shared__ double sN[7 * MW];   // the next panel's entries, as updated by step B
    __shared__ double sB[kWideRing];   // right-hand sides by row (mod kWideRing)
    __shared__ double sK[14 + 49];   // 1 / L(c,c), y_c and L(j,c) of a block; x of a block
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    const int W = a.band_w, w = W - 1, Vs = a.band_vs;
    const int NB = Vs / 7;
    const int nT = (W - 7 + 3) / 4;   // tile rows of the trailing triangle
    const int ntile = nT * (nT + 1) / 2;
    for (int t = tid; t < W; t += kWideBlock) sB[t & RM] = t < Vs ? a.rhs[t] : 0.0;
    if (tid == 0) s_fail = 0;
    double pf[7], pfb = 0.0;   // a row entering the window at the next block
#pragma unroll
    for (int c = 0; c < 7; ++c) pf[c] = 0.0;
    __syncthreads();

    for (int K = 0; K < NB; ++K) {
        const int r0 = 7 * K;
        const int t = tid, R = r0 + t;
        const bool hr = t < W && R < Vs;
        // A. the panel
        double p[7], b = 0.0;
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            const bool in = hr && (t >= 7 || c <= t);
            p[c] = !in ? 0.0 : K == 0 ? a.band[(int64_t)R * W + w + c - t] : t >= W - 7 ? pf[c] : sN[c * MW + t];
        }
        if (hr) b = sB[R & RM];
        if (tid < kWave) {
            bool okp = true;
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                const double d = readlane_f64(p[c], c);
                okp = okp && d > 0.0;
                double ird = __builtin_amdgcn_rsq(d);
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    const double e = fma(-d * ird, ird, 1.0);
                    ird = fma(0.5 * ird, e, ird);
                }
                const double rd = d * ird;
                const double yc = readlane_f64(b, c) * ird;
                if (t == c) {
                    p[c] = rd;
                    b = yc;
                } else if (t > c) {
                    p[c] *= ird;
                    b = fma(-p[c], yc, b);
                }
                if (tid == 0) {
                    sK[c] = ird;
                    sK[7 + c] = yc;
                }
#pragma unroll
                for (int j = c + 1; j < 7; ++j) {
                    const double ljc = readlane_f64(p[c], j);   // L(j, c)
                    if (t >= j) p[j] = fma(-p[c], ljc, p[j]);
                    if (tid == 0) sK[14 + 7 * j + c] = ljc;
                }
            }
            if (tid == 0 && !okp) s_fail = 1;
        }
        lds_barrier();
        if (s_fail) break;   // the same in every thread
        if (tid >= kWave && hr) {
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                const double ird = sK[c], yc = sK[7 + c];
                p[c] *= ird;
                b = fma(-p[c], yc, b);
#pragma unroll
                for (int j = c + 1; j < 7; ++j) p[j] = fma(-p[c], sK[14 + 7 * j + c], p[j]);
            }
        }
        if (hr) {
#pragma unroll
            for (int c = 0; c < 7; ++c)
                if (t >= 7 || c <= t) a.band[(int64_t)R * W + w + c - t] = p[c];
            if (t >= 7) {
#pragma unroll
                for (int c = 0; c < 7; ++c) sP[c * PW + t + 1] = p[c];
            } else {
                a.rhs[R] = b;   // y of the block's rows, final
            }
            sB[R & RM] = b;
        }
        lds_barrier();
        // B. the trailing update.  The rows entering the window at the next
        // block (rows r0 + W .. r0 + W + 6, untouched so far) are loaded first.
        const int Rn = r0 + 7 + t;
        const bool hn = t >= W - 7 && t < W && Rn < Vs;
        if (hn) {
#pragma unroll
            for (int c = 0; c < 7; ++c)
                pf[c] = t >= 7 || c <= t ? a.band[(int64_t)Rn * W + w + c - t] : 0.0;
            pfb = a.rhs[Rn];
        }
        // The trailing triangle in tiles of 4 x 4 entries (local rows i0 ..
        // i0 + 3, columns j0 .. j0 + 3), one per thread at a time: a tile
        // reads 8 panel entries per column for its 16 entries, the columns'
        // 4 as one 32-byte LDS read, and consecutive threads take
        // consecutive tiles of a tile row (consecutive device-memory
        // entries of the same 4 rows).
        for (int T = tid; T < ntile; T += kWideBlock) {
            int I = (int)((sqrtf(8.0f * (float)T + 1.0f) - 1.0f) * 0.5f);
            while (I * (I + 1) / 2 > T) --I;
            while ((I + 1) * (I + 2) / 2 <= T) ++I;
            const int J = T - I * (I + 1) / 2;
            const int i0 = 7 + 4 * I, j0 = 7 + 4 * J;
            double acc[4][4];
            // entry (i, j) of the window at band[(r0 + i) W + w - i + j]
            double* tb = a.band + (int64_t)(r0 + i0) * W + w - i0 + j0;
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const int i = i0 + x, j = j0 + y;
                    acc[x][y] = i < W && j <= i && r0 + i < Vs ? tb[x * w + y] : 0.0;
                }
#pragma unroll 1
            for (int c = 0; c < 7; ++c) {
                const double2 q0 = *(const double2*)&sP[c * PW + j0 + 1];
                const double2 q1 = *(const double2*)&sP[c * PW + j0 + 3];
                const double pj[4] = {q0.x, q0.y, q1.x, q1.y};
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const double pi = sP[c * PW + i0 + x + 1];
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = fma(-pi, pj[y], acc[x][y]);
                }
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const int i = i0 + x, j = j0 + y;
                    if (!(i < W && j <= i && r0 + i < Vs)) continue;
                    tb[x * w + y] = acc[x][y];
                    if (j < 14) sN[(j - 7) * MW + (i - 7)] = acc[x][y];
                }
        }
        if (hn) sB[Rn & RM] = pfb;
        // step B's device-memory entries are read by other threads next block
        __syncthreads();
    }
    if (s_fail) {   // the same in every thread
        if (tid == 0) a.lm[kLmFail] = 1.0;
        return;
    }
    if (tid == 0) a.lm[kLmUsed] = 0.0;
    __syncthreads();   // L and y in device memory, visible to every thread

    band_back_substitute(a, sB, RM, sK);
    band_candidate_poses(a);
}

// e^T e of every edge at the poses P (one thread per edge).
__global__ __launch_bounds__(kPgoBlock) void pgo_edge_cost_kernel(PgoArgs a, const double* __restrict__ P) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_edges) return;
    const int i = a.edges[2 * k], j = a.edges[2 * k + 1];
    double e[7];
    pgo_edge_error(sim3_load(P + 13 * (int64_t)i), sim3_load(P + 13 * (int64_t)j),
                   sim3_inv(sim3_load(a.M + 13 * (int64_t)k)), e);
    double v = 0.0;
    for (int c = 0; c < 7; ++c) v = fma(e[c], e[c], v);
    a.ecost[k] = v;
}

// F = the edge costs summed in a fixed order (thread strides, then the block sum).
__device__ inline double pgo_total_cost(const PgoArgs& a, double* s_w) {
    double part = 0.0;
    for (int k = threadIdx.x; k < a.n_edges; k += blockDim.x) part += a.ecost[k];
    return block_sum_f64(part, s_w);
}

// Start: F of the starting poses (edge costs already evaluated), the first
// damping, relinearise.
__global__ __launch_bounds__(kPgoBlock) void pgo_init_kernel(PgoArgs a, double lambda0) {
    __shared__ double s_w[kPgoBlock / kWave];
    const double F = pgo_total_cost(a, s_w);
    if (threadIdx.x == 0) {
        for (int q = 0; q < kLmWords; ++q) a.lm[q] = 0.0;
        a.lm[kLmLambda] = lambda0;
        a.lm[kLmF] = F;
        a.lm[kLmRelin] = 1.0;
        if (a.cost) a.cost[0] = F;
    }
}

// The decision of iteration a.step (edge costs of the candidate evaluated):
// take the candidate if its F is below the accepted F (every candidate when
// the damping is 0: Gauss-Newton) and the solve did not fail.
__global__ __launch_bounds__(kPgoBlock) void pgo_decide_kernel(PgoArgs a) {
    __shared__ double s_w[kPgoBlock / kWave];
    const double Fc = pgo_total_cost(a, s_w);
    if (threadIdx.x == 0) {
        const double lam = a.lm[kLmLambda];
        const bool fail = a.lm[kLmFail] != 0.0;
        const bool take = !fail && (lam == 0.0 || Fc < a.lm[kLmF]);
        if (a.lambdas) a.lambdas[a.step] = lam;
        if (a.accepted) a.accepted[a.step] = take ? 1 : 0;
        if (a.cg_used) a.cg_used[a.step] = fail ? -1 : (int32_t)a.lm[kLmUsed];
        if (take) {
            a.lm[kLmF] = Fc;
            if (lam > 0.0) a.lm[kLmLambda] = fmax(lam / 10.0, kLmLambdaMin);   // lambda / 10, as the definition states
        } else {
            a.lm[kLmLambda] = fmin(lam * 10.0, kLmLambdaMax);
        }
        a.lm[kLmRelin] = take ? 1.0 : 0.0;
        a.lm[kLmTake] = take ? 1.0 : 0.0;
        a.lm[kLmFail] = 0.0;
        if (a.cost) a.cost[a.step + 1] = a.lm[kLmF];
    }
}

// An accepted candidate becomes the poses.
__global__ __launch_bounds__(kPgoBlock) void pgo_accept_kernel(PgoArgs a) {
    if (a.lm[kLmTake] == 0.0) return;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < 13 * (int64_t)a.n_nodes) a.S[q] = a.S_c[q];
}

}  // namespace fl
