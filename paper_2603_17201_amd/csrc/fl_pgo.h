// Essential-graph (Sim3 pose-graph) optimisation.
//
// Loop correction spreads the loop's Sim3 to every keyframe by optimising
// the essential graph (Sec. III-B, Sec. IV-F).  Nodes are keyframe poses S_i
// (world -> camera Sim3s); an edge (i, j) measures M_ij ~ S_j S_i^-1 and
// contributes e_ij = log(M_ij^-1 S_j S_i^-1) to F = sum e^T e.  Nodes move by
// left perturbations S_i <- exp(d_i) S_i.  The Jacobians of e_ij with respect
// to d_i and d_j are central differences of the float64 Sim3 algebra.  Each
// outer step solves (H + lambda diag H) d = -g by block-Jacobi preconditioned
// conjugate gradients.
//
// Per outer step two kernels run: pgo_jacobian_kernel over (edge, column)
// items on every CU, then pgo_solve_kernel, one workgroup that gathers g and
// the diagonal blocks per node over its incident edges (fixed order, no
// floating-point atomics), runs the conjugate gradients with fixed-order
// float64 reductions and updates the nodes.

#pragma once

#include "fl_residual.h"

namespace fl {

constexpr int kPgoBlock = 1024;     // threads of the solve workgroup
constexpr int kPgoJacBlock = 256;   // threads of a Jacobian workgroup

struct PgoArgs {
    int32_t n_nodes, n_edges;
    double* S;                  // [n_nodes][13] in/out
    const double* M;            // [n_edges][13]
    const int32_t* edges;       // [n_edges][2]
    const int32_t* adj_off;     // [n_nodes + 1] incident edges of each node
    const int32_t* adj;         // [2 n_edges] 2 * edge + (1 if the node is the edge's j)
    const uint8_t* fixed;       // [n_nodes]
    double fd_step;
    double lambda;
    int32_t cg_iters;
    double cg_tol;
    int32_t step;               // outer step index (cost and count outputs)
    // workspace
    double* e;                  // [n_edges][7]
    double* J;                  // [n_edges][2][49] J_i then J_j, row-major 7x7
    double* u;                  // [n_edges][7] conjugate-gradient edge products
    double* vec;                // [6][n_nodes][7]: g, x, r, z, p, q
    double* Dfac;               // [n_nodes][49] LDL^T factors of the preconditioner blocks
    // outputs (may be null)
    double* cost;               // [iters + 1]
    int32_t* cg_used;           // [iters]
};

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

// Column c of J_i and J_j of edge k (item k * 7 + c); item c = 0 also
// writes e.
__global__ __launch_bounds__(kPgoJacBlock) void pgo_jacobian_kernel(PgoArgs a) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= 7 * (int64_t)a.n_edges) return;
    const int k = (int)(item / 7), c = (int)(item % 7);
    const int i = a.edges[2 * k], j = a.edges[2 * k + 1];
    const Sim3d Si = sim3_load(a.S + 13 * (int64_t)i);
    const Sim3d Sj = sim3_load(a.S + 13 * (int64_t)j);
    const Sim3d Minv = sim3_inv(sim3_load(a.M + 13 * (int64_t)k));
    if (c == 0) {
        double e[7];
        pgo_edge_error(Si, Sj, Minv, e);
        for (int r = 0; r < 7; ++r) a.e[7 * (int64_t)k + r] = e[r];
    }
    const double h = a.fd_step;
    double d[7] = {0, 0, 0, 0, 0, 0, 0};
    double ep[7], em[7];
    for (int side = 0; side < 2; ++side) {
        d[c] = h;
        const Sim3d Pp = sim3_mul(sim3_exp(d), side ? Sj : Si);
        d[c] = -h;
        const Sim3d Pm = sim3_mul(sim3_exp(d), side ? Sj : Si);
        d[c] = 0.0;
        if (side) {
            pgo_edge_error(Si, Pp, Minv, ep);
            pgo_edge_error(Si, Pm, Minv, em);
        } else {
            pgo_edge_error(Pp, Sj, Minv, ep);
            pgo_edge_error(Pm, Sj, Minv, em);
        }
        double* Jk = a.J + 98 * (int64_t)k + 49 * side;
        for (int r = 0; r < 7; ++r) Jk[7 * r + c] = (ep[r] - em[r]) / (2.0 * h);
    }
}

// y += J^T v (J 7x7 row-major)
__device__ __forceinline__ void add_JTv(const double* J, const double* v, double* y) {
    for (int c = 0; c < 7; ++c) {
        double s = y[c];
        for (int r = 0; r < 7; ++r) s = fma(J[7 * r + c], v[r], s);
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

__global__ __launch_bounds__(kPgoBlock) void pgo_solve_kernel(PgoArgs a) {
    __shared__ double s_w[kPgoBlock / kWave];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = a.n_nodes, E = a.n_edges;
    const int64_t V = 7 * (int64_t)N;
    double* g = a.vec;
    double* x = a.vec + V;
    double* r = a.vec + 2 * V;
    double* z = a.vec + 3 * V;
    double* p = a.vec + 4 * V;
    double* q = a.vec + 5 * V;

    // cost of the current poses
    double part = 0.0;
    for (int k = tid; k < E; k += nt)
        for (int c = 0; c < 7; ++c) part = fma(a.e[7 * (int64_t)k + c], a.e[7 * (int64_t)k + c], part);
    const double F = pgo_sum(part, s_w);
    if (tid == 0 && a.cost) a.cost[a.step] = F;

    // g and the preconditioner blocks, node by node over incident edges
    double gg = 0.0;
    for (int n = tid; n < N; n += nt) {
        double gn[7] = {0, 0, 0, 0, 0, 0, 0};
        double D[49];
        for (int t = 0; t < 49; ++t) D[t] = 0.0;
        if (!a.fixed[n]) {
            for (int t = a.adj_off[n]; t < a.adj_off[n + 1]; ++t) {
                const int k = a.adj[t] >> 1, side = a.adj[t] & 1;
                const double* Jk = a.J + 98 * (int64_t)k + 49 * side;
                add_JTv(Jk, a.e + 7 * (int64_t)k, gn);
                for (int c1 = 0; c1 < 7; ++c1)
                    for (int c2 = 0; c2 < 7; ++c2) {
                        double s = D[7 * c1 + c2];
                        for (int rr = 0; rr < 7; ++rr) s = fma(Jk[7 * rr + c1], Jk[7 * rr + c2], s);
                        D[7 * c1 + c2] = s;
                    }
            }
            for (int c = 0; c < 7; ++c) D[8 * c] *= 1.0 + a.lambda;
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
        for (int t = 0; t < 49; ++t) a.Dfac[49 * (int64_t)n + t] = D[t];
        for (int c = 0; c < 7; ++c) {
            g[7 * n + c] = gn[c];
            x[7 * n + c] = 0.0;
            r[7 * n + c] = -gn[c];
            gg = fma(gn[c], gn[c], gg);
        }
        double zn[7];
        ldl7_solve(D, r + 7 * n, zn);
        for (int c = 0; c < 7; ++c) {
            z[7 * n + c] = zn[c];
            p[7 * n + c] = zn[c];
        }
    }
    const double gnorm2 = pgo_sum(gg, s_w);
    double rz = 0.0;
    for (int64_t v = tid; v < V; v += nt) rz = fma(r[v], z[v], rz);
    rz = pgo_sum(rz, s_w);

    // conjugate gradients on H x = -g over the free nodes (fixed nodes keep
    // p = r = 0)
    int used = 0;
    const double stop2 = a.cg_tol * a.cg_tol * gnorm2;
    for (int it = 0; it < a.cg_iters && gnorm2 > 0.0; ++it) {
        // u_k = J_i p_i + J_j p_j
        for (int k = tid; k < E; k += nt) {
            const int i = a.edges[2 * k], j = a.edges[2 * k + 1];
            const double* Ji = a.J + 98 * (int64_t)k;
            const double* Jj = Ji + 49;
            for (int rr = 0; rr < 7; ++rr) {
                double s = 0.0;
                for (int c = 0; c < 7; ++c) s = fma(Ji[7 * rr + c], p[7 * i + c], s);
                for (int c = 0; c < 7; ++c) s = fma(Jj[7 * rr + c], p[7 * j + c], s);
                a.u[7 * (int64_t)k + rr] = s;
            }
        }
        __syncthreads();
        // q_n = sum over incident edges of J^T u (+ lambda diag H p via the blocks)
        double pq = 0.0;
        for (int n = tid; n < N; n += nt) {
            double qn[7] = {0, 0, 0, 0, 0, 0, 0};
            if (!a.fixed[n]) {
                double dg[7] = {0, 0, 0, 0, 0, 0, 0};
                for (int t = a.adj_off[n]; t < a.adj_off[n + 1]; ++t) {
                    const int k = a.adj[t] >> 1, side = a.adj[t] & 1;
                    const double* Jk = a.J + 98 * (int64_t)k + 49 * side;
                    add_JTv(Jk, a.u + 7 * (int64_t)k, qn);
                    if (a.lambda > 0.0)
                        for (int c = 0; c < 7; ++c)
                            for (int rr = 0; rr < 7; ++rr) dg[c] = fma(Jk[7 * rr + c], Jk[7 * rr + c], dg[c]);
                }
                if (a.lambda > 0.0)
                    for (int c = 0; c < 7; ++c) qn[c] = fma(a.lambda * dg[c], p[7 * n + c], qn[c]);
            }
            for (int c = 0; c < 7; ++c) {
                q[7 * n + c] = qn[c];
                pq = fma(p[7 * n + c], qn[c], pq);
            }
        }
        pq = pgo_sum(pq, s_w);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        double rr2 = 0.0, rz_new = 0.0;
        for (int n = tid; n < N; n += nt) {
            for (int c = 0; c < 7; ++c) {
                x[7 * n + c] = fma(alpha, p[7 * n + c], x[7 * n + c]);
                r[7 * n + c] = fma(-alpha, q[7 * n + c], r[7 * n + c]);
                rr2 = fma(r[7 * n + c], r[7 * n + c], rr2);
            }
            double zn[7];
            ldl7_solve(a.Dfac + 49 * (int64_t)n, r + 7 * n, zn);
            for (int c = 0; c < 7; ++c) {
                z[7 * n + c] = a.fixed[n] ? 0.0 : zn[c];
                rz_new = fma(r[7 * n + c], z[7 * n + c], rz_new);
            }
        }
        rr2 = pgo_sum(rr2, s_w);
        rz_new = pgo_sum(rz_new, s_w);
        used = it + 1;
        if (rr2 <= stop2) break;
        const double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t v = tid; v < V; v += nt) p[v] = fma(beta, p[v], z[v]);
        __syncthreads();
    }
    if (tid == 0 && a.cg_used) a.cg_used[a.step] = used;
    __syncthreads();
    // S_n <- exp(x_n) S_n
    for (int n = tid; n < N; n += nt) {
        if (a.fixed[n]) continue;
        double d[7];
        for (int c = 0; c < 7; ++c) d[c] = x[7 * n + c];
        const Sim3d Sn = sim3_mul(sim3_exp(d), sim3_load(a.S + 13 * (int64_t)n));
        sim3_store(Sn, a.S + 13 * (int64_t)n);
    }
}

// Cost after the last step (e of the final poses, summed in fixed order).
__global__ __launch_bounds__(kPgoBlock) void pgo_cost_kernel(PgoArgs a) {
    __shared__ double s_w[kPgoBlock / kWave];
    double part = 0.0;
    for (int k = threadIdx.x; k < a.n_edges; k += blockDim.x) {
        const int i = a.edges[2 * k], j = a.edges[2 * k + 1];
        double e[7];
        pgo_edge_error(sim3_load(a.S + 13 * (int64_t)i), sim3_load(a.S + 13 * (int64_t)j),
                       sim3_inv(sim3_load(a.M + 13 * (int64_t)k)), e);
        for (int c = 0; c < 7; ++c) part = fma(e[c], e[c], part);
    }
    const double F = block_sum_f64(part, s_w);
    if (threadIdx.x == 0 && a.cost) a.cost[a.step] = F;
}

}  // namespace fl
