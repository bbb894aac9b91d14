// Sim3 reprojection residual, its hand-written backward, the float64 Sim3
// exponential and the Gauss-Newton step, plus per-event refinement of the
// loop Sim3 on the pairs a search accepted.
//
// The paper refines the loop Sim3 between its two projection searches
// (Sec. IV-C) and optimises poses with Jacobians it obtains by automatic
// differentiation (Sec. IV-F).  Here the residual of a matched pair is
//   p = sR X + t,  q = R_k p + t_k,  r = pi(q) - uv,
// its Jacobian with respect to a left perturbation xi = (omega, upsilon,
// sigma) of the Sim3 is written out by hand,
//   J = dpi/dq R_k [ -[p]x | I | p ],
// per-pair arithmetic is float32 and every sum is float64 with a fixed
// reduction order (thread, wave, block, then blocks in index order).
#pragma once

#include "fl_internal.h"

namespace fl {

constexpr int kResBlock = 256;
constexpr int kNAcc = kNAccPad;   // 7 gradient + 28 upper-triangle H + 1 count / loss

// ---------------------------------------------------------------------------
// float64 Sim3 algebra

struct Sim3d {
    double R[9];
    double t[3];
    double s;
};

// 1 / (i + 1), i < 72
struct RecipTable {
    double v[72];
    constexpr RecipTable() : v() {
        for (int i = 0; i < 72; ++i) v[i] = 1.0 / (double)(i + 1);
    }
};
__device__ constexpr RecipTable kRecip{};

// 1/x to within about one ulp: the hardware estimate refined by two Newton
// steps (cheaper on the serial path of a step than a correctly rounded
// division).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// The first NT terms of e^sigma = sum_k sigma^k / k! and of
// I_n(sigma) = integral_0^1 tau^n e^{sigma tau} d tau = sum_k sigma^k / (k! (n + k + 1)), n = 0..6.
template <int NT>
__device__ __forceinline__ void sigma_series(double sig, double* I, double& es) {
    double p[NT];
    p[0] = 1.0;
#pragma unroll
    for (int k = 1; k < NT; ++k) p[k] = p[k - 1] * sig * kRecip.v[k - 1];   // sigma^k / k!
    es = 0.0;
#pragma unroll
    for (int k = NT - 1; k >= 0; --k) es += p[k];
#pragma unroll
    for (int n = 0; n < 7; ++n) {
        double v = 0.0;
#pragma unroll
        for (int k = NT - 1; k >= 0; --k) v = fma(p[k], kRecip.v[n + k], v);
        I[n] = v;
    }
}

// Coefficients of the exponential of xi = (omega, upsilon, sigma):
// R = I + a W + b W^2 with W = [omega]x, s = e^sigma, and
// V = c0 I + c1 W + c2 W^2 = integral_0^1 e^{sigma tau} exp(tau W) d tau
// (closed form; series for small rotation angles), t = V upsilon.
struct ExpCoef {
    double a, b, c0, c1, c2, es;
};

__device__ __noinline__ ExpCoef sim3_exp_coef_full(double w0, double w1, double w2, double sig) {
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const bool small = th2 < 1e-4;   // angle below 1e-2: the series need only th^2
    // th, sin th and cos th only where the series do not serve (taken inside
    // the branch, so that the common small-angle path does not wait for a
    // square root whose result it never uses)
    double th = 0.0, sn = 0.0, cs = 1.0;
    ExpCoef k;
    if (small) {
        // sin(th)/th and (1 - cos(th))/th^2 by their Taylor series: the next
        // terms are below th^8/9! < 3e-22 here
        const double t4 = th2 * th2;
        k.a = 1.0 - th2 * (1.0 / 6.0) + t4 * (1.0 / 120.0) - t4 * th2 * (1.0 / 5040.0);
        k.b = 0.5 - th2 * (1.0 / 24.0) + t4 * (1.0 / 720.0) - t4 * th2 * (1.0 / 40320.0);
    } else {
        th = sqrt(th2);
        sn = sin(th);
        cs = cos(th);
        k.a = sn / th;
        k.b = (1.0 - cs) / th2;
    }
    // I_n(sigma) for n = 0..6 and e^sigma = sum_k sigma^k / k! share one series
    double I[7];
    double es;
    const double asig = fabs(sig);
    if (asig < 2.5e-4) {
        sigma_series<5>(sig, I, es);   // remainder below 2.5e-4^5 / 5! < 1e-20
    } else if (asig < 4e-3) {
        sigma_series<7>(sig, I, es);   // below 4e-3^7 / 7! < 1e-20
    } else if (asig < 0.01) {
        sigma_series<9>(sig, I, es);   // below 0.01^9 / 9! < 3e-24
    } else if (fabs(sig) < 2.0) {
        double term = 1.0, e = 0.0;
        for (int n = 0; n < 7; ++n) I[n] = 0.0;
        for (int kk = 0; kk < 60; ++kk) {
            e += term;
#pragma unroll
            for (int n = 0; n < 7; ++n) I[n] += term * kRecip.v[n + kk];
            if (fabs(term) < 1e-18 * e) break;
            term *= sig * kRecip.v[kk];
        }
        es = e;
    } else {
        es = exp(sig);
        I[0] = expm1(sig) / sig;
        for (int m = 1; m < 7; ++m) I[m] = (es - (double)m * I[m - 1]) / sig;
    }
    k.es = es;
    k.c0 = I[0];
    if (small) {
        k.c1 = I[1] - th2 * (1.0 / 6.0) * I[3] + th2 * th2 * (1.0 / 120.0) * I[5];
        k.c2 = 0.5 * I[2] - th2 * (1.0 / 24.0) * I[4] + th2 * th2 * (1.0 / 720.0) * I[6];
    } else {
        const double den = sig * sig + th2;
        k.c1 = (es * (sig * sn - th * cs) + th) / (th * den);
        k.c2 = (k.c0 - (es * (sig * cs + th * sn) - sig) / den) / th2;
    }
    return k;
}

// The same coefficients, with the usual Gauss-Newton step (rotation angle
// below 1e-2, |sigma| below 1e-2) computed in line by the very same series
// and every other step by the out-of-line function above: the common case
// costs no call, and the code placed in line stays small enough not to push
// a kernel that holds many registers into spilling them.
__device__ __forceinline__ ExpCoef sim3_exp_coef(double w0, double w1, double w2, double sig) {
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double asig = fabs(sig);
    if (!(th2 < 1e-4 && asig < 0.01)) return sim3_exp_coef_full(w0, w1, w2, sig);
    ExpCoef k;
    const double t4 = th2 * th2;
    k.a = 1.0 - th2 * (1.0 / 6.0) + t4 * (1.0 / 120.0) - t4 * th2 * (1.0 / 5040.0);
    k.b = 0.5 - th2 * (1.0 / 24.0) + t4 * (1.0 / 720.0) - t4 * th2 * (1.0 / 40320.0);
    double I[7];
    double es;
    if (asig < 2.5e-4) sigma_series<5>(sig, I, es);
    else if (asig < 4e-3) sigma_series<7>(sig, I, es);
    else sigma_series<9>(sig, I, es);
    k.es = es;
    k.c0 = I[0];
    k.c1 = I[1] - th2 * (1.0 / 6.0) * I[3] + th2 * th2 * (1.0 / 120.0) * I[5];
    k.c2 = 0.5 * I[2] - th2 * (1.0 / 24.0) * I[4] + th2 * th2 * (1.0 / 720.0) * I[6];
    return k;
}

__device__ inline void hat_sq(double w0, double w1, double w2, double* W, double* W2) {
    W[0] = 0.0; W[1] = -w2; W[2] = w1;
    W[3] = w2; W[4] = 0.0; W[5] = -w0;
    W[6] = -w1; W[7] = w0; W[8] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            W2[3 * i + j] = W[3 * i] * W[j] + W[3 * i + 1] * W[3 + j] + W[3 * i + 2] * W[6 + j];
}

// exp of a tangent xi = (omega, upsilon, sigma)
__device__ inline Sim3d sim3_exp(const double* xi) {
    const ExpCoef k = sim3_exp_coef(xi[0], xi[1], xi[2], xi[6]);
    double W[9], W2[9];
    hat_sq(xi[0], xi[1], xi[2], W, W2);
    Sim3d S;
    double V[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        S.R[i] = I + k.a * W[i] + k.b * W2[i];
        V[i] = k.c0 * I + k.c1 * W[i] + k.c2 * W2[i];
    }
    for (int i = 0; i < 3; ++i) S.t[i] = V[3 * i] * xi[3] + V[3 * i + 1] * xi[4] + V[3 * i + 2] * xi[5];
    S.s = k.es;
    return S;
}

// log of a Sim3: omega from R (axis-angle, atan2 of the skew part's norm and
// the trace), sigma = ln s, upsilon solving V upsilon = t (Cramer's rule).
__device__ inline void sim3_log(const Sim3d& S, double* xi) {
    const double* R = S.R;
    const double v0 = 0.5 * (R[7] - R[5]), v1 = 0.5 * (R[2] - R[6]), v2 = 0.5 * (R[3] - R[1]);
    const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    const double sn = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const double th = atan2(sn, c);
    double w0, w1, w2;
    if (sn > 1e-7 || c > 0.0) {
        // omega = th / sin(th) v; the series 1 + th^2/6 + 7 th^4/360 below 1e-4
        const double f = th < 1e-4 ? 1.0 + th * th * (1.0 / 6.0) + 7.0 * th * th * th * th / 360.0 : th / sn;
        w0 = f * v0;
        w1 = f * v1;
        w2 = f * v2;
    } else {
        // th near pi: the axis from the largest diagonal entry of (R + I) / 2
        int m = 0;
        if (R[4] > R[0]) m = 1;
        if (R[8] > R[4 * m]) m = 2;
        double ax[3];
        ax[m] = sqrt(fmax(0.0, 0.5 * (R[4 * m] + 1.0)));
        for (int j = 0; j < 3; ++j)
            if (j != m) ax[j] = 0.5 * (R[3 * m + j] + R[3 * j + m]) / (2.0 * ax[m]);
        w0 = th * ax[0];
        w1 = th * ax[1];
        w2 = th * ax[2];
    }
    const double sig = log(S.s);
    const ExpCoef k = sim3_exp_coef(w0, w1, w2, sig);
    double W[9], W2[9], V[9];
    hat_sq(w0, w1, w2, W, W2);
    for (int i = 0; i < 9; ++i) V[i] = k.c0 * ((i % 4 == 0) ? 1.0 : 0.0) + k.c1 * W[i] + k.c2 * W2[i];
    const double A0 = V[4] * V[8] - V[5] * V[7], A1 = V[5] * V[6] - V[3] * V[8], A2 = V[3] * V[7] - V[4] * V[6];
    const double det = V[0] * A0 + V[1] * A1 + V[2] * A2;
    const double id = 1.0 / det;
    const double* t = S.t;
    // upsilon = V^-1 t = adj(V) t / det(V)
    xi[3] = (A0 * t[0] + (V[2] * V[7] - V[1] * V[8]) * t[1] + (V[1] * V[5] - V[2] * V[4]) * t[2]) * id;
    xi[4] = (A1 * t[0] + (V[0] * V[8] - V[2] * V[6]) * t[1] + (V[2] * V[3] - V[0] * V[5]) * t[2]) * id;
    xi[5] = (A2 * t[0] + (V[1] * V[6] - V[0] * V[7]) * t[1] + (V[0] * V[4] - V[1] * V[3]) * t[2]) * id;
    xi[0] = w0;
    xi[1] = w1;
    xi[2] = w2;
    xi[6] = sig;
}

// S^-1 = (R^T, -R^T t / s, 1 / s)
__device__ inline Sim3d sim3_inv(const Sim3d& S) {
    Sim3d V;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V.R[3 * i + j] = S.R[3 * j + i];
    V.s = 1.0 / S.s;
    for (int i = 0; i < 3; ++i)
        V.t[i] = -(V.R[3 * i] * S.t[0] + V.R[3 * i + 1] * S.t[1] + V.R[3 * i + 2] * S.t[2]) * V.s;
    return V;
}

// A o B  (X -> A(B(X)))
__device__ inline Sim3d sim3_mul(const Sim3d& A, const Sim3d& B) {
    Sim3d C;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            C.R[3 * i + j] = A.R[3 * i] * B.R[j] + A.R[3 * i + 1] * B.R[3 + j] + A.R[3 * i + 2] * B.R[6 + j];
        C.t[i] = A.s * (A.R[3 * i] * B.t[0] + A.R[3 * i + 1] * B.t[1] + A.R[3 * i + 2] * B.t[2]) + A.t[i];
    }
    C.s = A.s * B.s;
    return C;
}

__device__ inline Sim3d sim3_load(const double* p) {
    Sim3d S;
    for (int i = 0; i < 9; ++i) S.R[i] = p[i];
    for (int i = 0; i < 3; ++i) S.t[i] = p[9 + i];
    S.s = p[12];
    return S;
}

__device__ inline void sim3_store(const Sim3d& S, double* p) {
    for (int i = 0; i < 9; ++i) p[i] = S.R[i];
    for (int i = 0; i < 3; ++i) p[9 + i] = S.t[i];
    p[12] = S.s;
}

__device__ inline void sim3_to_f32(const Sim3d& S, fl_sim3* o) {
    for (int i = 0; i < 9; ++i) o->sR[i] = (float)(S.s * S.R[i]);
    for (int i = 0; i < 3; ++i) o->t[i] = (float)S.t[i];
    o->inv_s = (float)(1.0 / S.s);
    o->pad[0] = o->pad[1] = o->pad[2] = 0.0f;
}

// The part of the float32 form the residual reads (sR, t), for the steps
// inside a refinement; inv_s is filled in once at the end.
__device__ inline void sim3_to_f32_pose(const Sim3d& S, fl_sim3* o) {
    for (int i = 0; i < 9; ++i) o->sR[i] = (float)(S.s * S.R[i]);
    for (int i = 0; i < 3; ++i) o->t[i] = (float)S.t[i];
}

// Solve (H + lambda diag H) d = -g by an LDL^T factorisation (no square
// roots; one reciprocal per pivot); H given as its 28 upper entries row by
// row.  Returns false (d = 0) for a pivot that is not clearly positive.
// Right-looking, on the packed lower triangle (a[i(i+1)/2 + j] = H[i][j]):
// each pivot's column is scaled and its rank-1 product subtracted from the
// rest at once, with the forward substitution folded in, and the back
// substitution likewise updates every open right-hand side once an unknown is
// known.  It runs on one lane, so its dependency chain is its cost: per pivot
// one reciprocal, one multiply and one fused multiply-add deep, the updates
// themselves independent of one another.
__device__ inline bool solve7(const double* g, const double* Hu, double lambda, double* d) {
    double a[28];
    double dmax = 0.0;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) a[i * (i + 1) / 2 + j] = Hu[j * 7 - j * (j - 1) / 2 + (i - j)];
        a[i * (i + 1) / 2 + i] *= (1.0 + lambda);
        dmax = fmax(dmax, fabs(a[i * (i + 1) / 2 + i]));
    }
    double y[7], Dinv[7], L[21];   // L[i(i-1)/2 + j] = L[i][j], j < i
#pragma unroll
    for (int i = 0; i < 7; ++i) y[i] = -g[i];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const double dj = a[j * (j + 1) / 2 + j];
        ok = ok && dj > 1e-14 * dmax;
        Dinv[j] = recip(dj);
#pragma unroll
        for (int i = j + 1; i < 7; ++i) L[i * (i - 1) / 2 + j] = a[i * (i + 1) / 2 + j] * Dinv[j];
#pragma unroll
        for (int i = j + 1; i < 7; ++i) {
            const double lij = L[i * (i - 1) / 2 + j];
#pragma unroll
            for (int k = j + 1; k <= i; ++k)
                a[i * (i + 1) / 2 + k] = fma(-lij, a[k * (k + 1) / 2 + j], a[i * (i + 1) / 2 + k]);
            y[i] = fma(-lij, y[j], y[i]);
        }
    }
    // L^T d = D^-1 y
#pragma unroll
    for (int i = 0; i < 7; ++i) y[i] *= Dinv[i];
#pragma unroll
    for (int i = 6; i >= 0; --i) {
        d[i] = y[i];
#pragma unroll
        for (int m = 0; m < i; ++m) y[m] = fma(-L[i * (i - 1) / 2 + m], d[i], y[m]);
    }
    if (!ok) {
#pragma unroll
        for (int i = 0; i < 7; ++i) d[i] = 0.0;
    }
    return ok;
}

// ---------------------------------------------------------------------------
// per-pair residual and Jacobian (float32)

struct PairTerm {
    float r0, r1, w, rho;
    float e;             // |r| (0 when not valid)
    float J[2][7];
    bool valid;
};

// INV: (A, tS) is the float32 form of S^-1 and the pair is a point of the
// current side observed on the loop side, p = S^-1 X; its Jacobian is still
// taken with respect to the left perturbation of S, under which
// S^-1 <- S^-1 exp(-xi):  J = dpi/dq R_k (-A) [ -[X]x | I | X ].
template <bool INV = false>
__device__ __forceinline__ void pair_term(const float* A, const float* tS, const float* T, float fx, float fy,
                                          float cx, float cy, float x, float y, float z, float uo, float vo,
                                          float delta, bool need_J, PairTerm& o) {
    const float p0 = A[0] * x + A[1] * y + A[2] * z + tS[0];
    const float p1 = A[3] * x + A[4] * y + A[5] * z + tS[1];
    const float p2 = A[6] * x + A[7] * y + A[8] * z + tS[2];
    float q0 = p0, q1 = p1, q2 = p2;
    if (T) {
        q0 = T[0] * p0 + T[1] * p1 + T[2] * p2 + T[9];
        q1 = T[3] * p0 + T[4] * p1 + T[5] * p2 + T[10];
        q2 = T[6] * p0 + T[7] * p1 + T[8] * p2 + T[11];
    }
    o.valid = q2 > 0.0f;
    if (!o.valid) {
        o.r0 = o.r1 = o.w = o.rho = o.e = 0.0f;
        return;
    }
    const float iz = __builtin_amdgcn_rcpf(q2);   // within 1 ulp
    o.r0 = fx * q0 * iz + cx - uo;
    o.r1 = fy * q1 * iz + cy - vo;
    const float e = sqrtf(o.r0 * o.r0 + o.r1 * o.r1);
    o.e = e;
    if (e <= delta) {
        o.w = 1.0f;
        o.rho = 0.5f * e * e;
    } else {
        o.w = delta * __builtin_amdgcn_rcpf(e);
        o.rho = delta * e - 0.5f * delta * delta;
    }
    if (!need_J) return;
    // M = dpi/dq R_k (2 x 3)
    const float a0 = fx * iz, a2 = -fx * q0 * iz * iz;
    const float b1 = fy * iz, b2 = -fy * q1 * iz * iz;
    float M[2][3];
    if (T) {
        for (int c = 0; c < 3; ++c) {
            M[0][c] = a0 * T[c] + a2 * T[6 + c];
            M[1][c] = b1 * T[3 + c] + b2 * T[6 + c];
        }
    } else {
        M[0][0] = a0; M[0][1] = 0.0f; M[0][2] = a2;
        M[1][0] = 0.0f; M[1][1] = b1; M[1][2] = b2;
    }
    for (int r = 0; r < 2; ++r) {
        float m0 = M[r][0], m1 = M[r][1], m2 = M[r][2];
        float a0 = p0, a1 = p1, a2 = p2;   // the point the perturbation acts on
        if (INV) {
            // row of -M A, acting on X
            const float b0 = -(m0 * A[0] + m1 * A[3] + m2 * A[6]);
            const float b1 = -(m0 * A[1] + m1 * A[4] + m2 * A[7]);
            const float b2 = -(m0 * A[2] + m1 * A[5] + m2 * A[8]);
            m0 = b0;
            m1 = b1;
            m2 = b2;
            a0 = x;
            a1 = y;
            a2 = z;
        }
        o.J[r][0] = a1 * m2 - a2 * m1;   // a x m: derivative along omega
        o.J[r][1] = a2 * m0 - a0 * m2;
        o.J[r][2] = a0 * m1 - a1 * m0;
        o.J[r][3] = m0;                  // upsilon
        o.J[r][4] = m1;
        o.J[r][5] = m2;
        o.J[r][6] = m0 * a0 + m1 * a1 + m2 * a2;   // sigma
    }
}

// acc[0..6] += w J^T r, acc[7..34] += w J^T J (upper, row by row): each
// pair's terms in float32 (as its residual and Jacobian are), accumulated
// over pairs in float64.
__device__ __forceinline__ void accumulate(const PairTerm& t, double* acc) {
    const float w = t.w, r0 = t.r0, r1 = t.r1;
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] += (double)(w * fmaf(t.J[0][i], r0, t.J[1][i] * r1));
    int k = 7;
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int j = i; j < 7; ++j) acc[k++] += (double)(w * fmaf(t.J[0][i], t.J[0][j], t.J[1][i] * t.J[1][j]));
}

// Block reduction of NV <= 64 doubles per thread, fixed order.  Inside a
// wave a butterfly reduce-scatter halves the values a lane carries at every
// step (63 exchanges for any NV instead of 6 * NV), leaving the wave total of
// value l in lane l; the block then adds the wave totals in wave order.
// Result in s_out[0..NV) after the call.
template <int NV>
__device__ __forceinline__ void block_reduce(double* v, double* s_red, double* s_out) {
    static_assert(NV <= 64, "at most 64 values");
    const int lane = wave_lane();
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    double w[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const double lo = i < NV ? v[i] : 0.0;
        const double hi = i + 32 < NV ? v[i + 32] : 0.0;
        const bool up = (lane & 32) != 0;
        const double send = up ? lo : hi;
        w[i] = (up ? hi : lo) + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int h = 16; h >= 1; h >>= 1) {
        const bool up = (lane & h) != 0;
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const double send = up ? w[i] : w[i + h];
            w[i] = (up ? w[i + h] : w[i]) + __shfl_xor(send, h);
        }
    }
    if (lane < NV) s_red[wid * NV + lane] = w[0];
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double s = 0.0;
        for (int q = 0; q < nw; ++q) s += s_red[q * NV + threadIdx.x];
        s_out[threadIdx.x] = s;
    }
    __syncthreads();
}

// The same sums in float32, for a thread's few register-held pairs (it adds
// at most two terms before they are widened to float64).
__device__ __forceinline__ void accumulate_f32(const PairTerm& t, float* acc) {
    const float w = t.w, r0 = t.r0, r1 = t.r1;
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] += w * fmaf(t.J[0][i], r0, t.J[1][i] * r1);
    int k = 7;
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int j = i; j < 7; ++j) acc[k++] += w * fmaf(t.J[0][i], t.J[0][j], t.J[1][i] * t.J[1][j]);
}

// Fixed-order block reduction for the refinement.  The four lanes of each
// quad first add their values pairwise in float32 (DPP quad permutations:
// lanes 2i and 2i + 1 swap halves and add, then lanes 4i + {0, 1} and
// 4i + {2, 3} swap quarters and add), so each lane keeps NV / 4 of the quad's
// sums.  Those go through LDS column-major (column stride NT / 4 + 1), kSeg
// NV threads each add one of kSeg segments of a column in float64 and NV
// threads add the segments pairwise.  s_t holds NV (NT / 4 + 1) floats, s_q
// kSeg NV doubles; the block has NT threads (whole waves), a multiple of
// 4 kSeg and at least kSeg NV; NV is a multiple of 4.  Result in
// s_out[0..NV) after the call.
constexpr int kSeg = 8;

static_assert(kSeg == 4 || kSeg == 8, "segments are added as a pairwise tree of 4 or 8");

template <int NV>
__device__ __forceinline__ double add_segments(const double* s_q, int c) {
    const double a = (s_q[c] + s_q[NV + c]) + (s_q[2 * NV + c] + s_q[3 * NV + c]);
    if constexpr (kSeg == 4) return a;
    else return a + ((s_q[4 * NV + c] + s_q[5 * NV + c]) + (s_q[6 * NV + c] + s_q[7 * NV + c]));
}

template <int CTRL>
__device__ __forceinline__ float quad_perm_f32(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

template <int NV, int NT>
__device__ __forceinline__ void block_reduce_quad(const float* v, float* s_t, double* s_q, double* s_out) {
    static_assert(NV % 4 == 0 && NT % (4 * kSeg) == 0 && NT >= kSeg * NV && NT % kWave == 0, "block shape");
    constexpr int H = NV / 2, Q = NV / 4, NQ = NT / 4, ld = NQ + 1, per = NQ / kSeg;
    const int tid = threadIdx.x;
    const bool odd = tid & 1, hi = tid & 2;
    float h[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const float keep = odd ? v[j + H] : v[j];
        const float send = odd ? v[j] : v[j + H];
        h[j] = keep + quad_perm_f32<0xB1>(send);   // quad_perm [1, 0, 3, 2]
    }
    float q[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const float keep = hi ? h[j + Q] : h[j];
        const float send = hi ? h[j] : h[j + Q];
        q[j] = keep + quad_perm_f32<0x4E>(send);   // quad_perm [2, 3, 0, 1]
    }
    const int base = (odd ? H : 0) + (hi ? Q : 0);
#pragma unroll
    for (int j = 0; j < Q; ++j) s_t[(base + j) * ld + (tid >> 2)] = q[j];
    __syncthreads();
    if (tid < kSeg * NV) {
        const int c = tid % NV, sg = tid / NV;
        const float* col = s_t + c * ld + sg * per;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int r = 0; r + 1 < per; r += 2) {
            a0 += (double)col[r];
            a1 += (double)col[r + 1];
        }
        if (per & 1) a0 += (double)col[per - 1];
        s_q[sg * NV + c] = a0 + a1;
    }
    __syncthreads();
    if (tid < NV) s_out[tid] = add_segments<NV>(s_q, tid);
    __syncthreads();
}

struct ResArgs {
    int32_t n;
    int32_t n_kf;
    const float* xyz;
    const float* uv;
    const int32_t* kf_idx;
    const float* kf_T;
    const fl_sim3* S;
    float fx, fy, cx, cy;
    float delta;
    double grad_scale;
    float* r;
    float* w;
    double* loss;
    double* g;
    double* H;
    double* partial;      // [gridDim.x][kNAcc]
    uint32_t* done;       // one counter, zero on entry and on exit
};

__device__ __forceinline__ bool load_pair(const ResArgs& a, int i, float& x, float& y, float& z, float& uo,
                                          float& vo, const float*& T) {
    x = a.xyz[3 * (int64_t)i];
    y = a.xyz[3 * (int64_t)i + 1];
    z = a.xyz[3 * (int64_t)i + 2];
    uo = a.uv[2 * (int64_t)i];
    vo = a.uv[2 * (int64_t)i + 1];
    T = nullptr;
    if (a.kf_idx) {
        const int k = a.kf_idx[i];
        if (k < 0 || k >= a.n_kf) return false;
        if (a.kf_T) T = a.kf_T + 12 * (int64_t)k;
    } else if (a.kf_T) {
        T = a.kf_T;
    }
    return true;
}

// Last-block-done: true in the one block that finishes last (all blocks'
// partials are then visible to it).
__device__ __forceinline__ bool last_block(uint32_t* done, unsigned n_blocks) {
    __shared__ int s_last;
    __syncthreads();   // every wave's partial is written before thread 0 releases
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(done, 1u) == n_blocks - 1;
        if (s_last) __threadfence();   // acquire: see every block's partial (L2s of other XCDs)
    }
    __syncthreads();
    return s_last != 0;
}

// Sum `rows` partials of NV doubles (row stride kNAcc) in row order into
// s_out[0..NV): rows are staged through LDS in chunks by the whole block so
// the loads are issued in parallel, then column i is summed by thread i.
template <int NV, int MAXR>
__device__ __forceinline__ void sum_partials(const double* part, int rows, double* s_chunk, double* s_out) {
    double acc = 0.0;
    for (int r0 = 0; r0 < rows; r0 += MAXR) {
        const int nr = min(MAXR, rows - r0);
        for (int i = threadIdx.x; i < nr * NV; i += blockDim.x) {
            const int r = i / NV, c = i - r * NV;
            s_chunk[i] = part[(int64_t)(r0 + r) * kNAcc + c];
        }
        __syncthreads();
        if ((int)threadIdx.x < NV)
            for (int r = 0; r < nr; ++r) acc += s_chunk[r * NV + threadIdx.x];
        __syncthreads();
    }
    if ((int)threadIdx.x < NV) s_out[threadIdx.x] = acc;
    __syncthreads();
}

__global__ __launch_bounds__(kResBlock) void residual_fwd_kernel(ResArgs a) {
    __shared__ double s_red[(kResBlock / kWave) * 1];
    __shared__ double s_out[1];
    __shared__ double s_chunk[32 * 1];
    const fl_sim3 S = *a.S;
    double acc[1] = {0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
        float x, y, z, uo, vo;
        const float* T;
        PairTerm t;
        if (load_pair(a, i, x, y, z, uo, vo, T)) {
            pair_term(S.sR, S.t, T, a.fx, a.fy, a.cx, a.cy, x, y, z, uo, vo, a.delta, false, t);
        } else {
            t.valid = false;
            t.r0 = t.r1 = t.w = t.rho = 0.0f;
        }
        if (a.r) {
            a.r[2 * (int64_t)i] = t.r0;
            a.r[2 * (int64_t)i + 1] = t.r1;
        }
        if (a.w) a.w[i] = t.w;
        acc[0] += (double)t.rho;
    }
    block_reduce<1>(acc, s_red, s_out);
    if (threadIdx.x == 0) a.partial[blockIdx.x * kNAcc] = s_out[0];
    if (last_block(a.done, gridDim.x)) {
        sum_partials<1, 32>(a.partial, gridDim.x, s_chunk, s_out);
        if (threadIdx.x == 0) {
            *a.loss = s_out[0];
            *a.done = 0;
        }
    }
}

template <bool INV>
__global__ __launch_bounds__(kResBlock) void residual_bwd_kernel(ResArgs a) {
    __shared__ double s_red[(kResBlock / kWave) * 35];
    __shared__ double s_out[35];
    __shared__ double s_chunk[32 * 35];
    const fl_sim3 S = *a.S;
    double acc[35];
#pragma unroll
    for (int i = 0; i < 35; ++i) acc[i] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
        float x, y, z, uo, vo;
        const float* T;
        if (!load_pair(a, i, x, y, z, uo, vo, T)) continue;
        PairTerm t;
        pair_term<INV>(S.sR, S.t, T, a.fx, a.fy, a.cx, a.cy, x, y, z, uo, vo, a.delta, true, t);
        if (t.valid) accumulate(t, acc);
    }
    block_reduce<35>(acc, s_red, s_out);
    if ((int)threadIdx.x < 35) a.partial[blockIdx.x * kNAcc + threadIdx.x] = s_out[threadIdx.x];
    if (last_block(a.done, gridDim.x)) {
        sum_partials<35, 32>(a.partial, gridDim.x, s_chunk, s_out);
        if (threadIdx.x < 7) a.g[threadIdx.x] = a.grad_scale * s_out[threadIdx.x];
        else if ((int)threadIdx.x < 35 && a.H) a.H[threadIdx.x - 7] = s_out[threadIdx.x];
        if (threadIdx.x == 0) *a.done = 0;
    }
}

__global__ void sim3_exp_mul_kernel(const double* __restrict__ xi, const double* __restrict__ S_in,
                                    double* __restrict__ S_out, fl_sim3* __restrict__ S32) {
    if (threadIdx.x != 0) return;
    const Sim3d E = sim3_exp(xi);
    const Sim3d S = sim3_mul(E, sim3_load(S_in));
    sim3_store(S, S_out);
    if (S32) sim3_to_f32(S, S32);
}

// Gradient with respect to the coordinates xi of S = exp(xi) S0, from the
// gradient g with respect to a left perturbation of S: exp(xi + d) equals
// exp(J_l(xi) d) exp(xi) to first order, so dL/dxi = J_l(xi)^T g, with the
// left Jacobian J_l(xi) = sum_k ad(xi)^k / (k + 1)!.  For xi = (w, u, sig)
// (omega, upsilon, sigma) the commutator of the 4x4 generators gives, in
// the rows and columns (omega, upsilon, sigma),
//   ad(xi) = [ [w]x        0          0 ]
//            [ [u]x   [w]x + sig I   -u ]
//            [ 0           0          0 ].
// The series is summed in float64 until a term's largest entry falls below
// 1e-18 of the sum's (at most 64 terms; |w| <= pi and |sig| of order one
// converge in about 25).  out = scale * J_l^T g (scale: device, may be null).
__global__ void sim3_grad_xi_kernel(const double* __restrict__ xi, const double* __restrict__ g,
                                    const double* __restrict__ scale, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double A[49];
    for (int i = 0; i < 49; ++i) A[i] = 0.0;
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2], u0 = xi[3], u1 = xi[4], u2 = xi[5], sg = xi[6];
    auto set_hat = [&](int r, int c, double a0, double a1, double a2) {   // [a]x at block (r, c)
        A[(r + 0) * 7 + c + 1] = -a2;
        A[(r + 0) * 7 + c + 2] = a1;
        A[(r + 1) * 7 + c + 0] = a2;
        A[(r + 1) * 7 + c + 2] = -a0;
        A[(r + 2) * 7 + c + 0] = -a1;
        A[(r + 2) * 7 + c + 1] = a0;
    };
    set_hat(0, 0, w0, w1, w2);
    set_hat(3, 0, u0, u1, u2);
    set_hat(3, 3, w0, w1, w2);
    for (int i = 3; i < 6; ++i) A[i * 7 + i] += sg;
    A[3 * 7 + 6] = -u0;
    A[4 * 7 + 6] = -u1;
    A[5 * 7 + 6] = -u2;
    // J = sum_k T_k with T_0 = I, T_k = A T_{k-1} / (k + 1)
    double T[49], J[49], N[49];
    for (int i = 0; i < 49; ++i) T[i] = J[i] = (i % 8 == 0) ? 1.0 : 0.0;
    for (int k = 1; k < 64; ++k) {
        double tmax = 0.0, jmax = 0.0;
        const double f = 1.0 / (double)(k + 1);
        for (int r = 0; r < 7; ++r)
            for (int c = 0; c < 7; ++c) {
                double v = 0.0;
                for (int m = 0; m < 7; ++m) v = fma(A[r * 7 + m], T[m * 7 + c], v);
                N[r * 7 + c] = v * f;
            }
        for (int i = 0; i < 49; ++i) {
            T[i] = N[i];
            J[i] += N[i];
            tmax = fmax(tmax, fabs(N[i]));
            jmax = fmax(jmax, fabs(J[i]));
        }
        if (tmax <= 1e-18 * jmax) break;
    }
    const double sc = scale ? *scale : 1.0;
    for (int c = 0; c < 7; ++c) {
        double v = 0.0;
        for (int r = 0; r < 7; ++r) v = fma(J[r * 7 + c], g[r], v);
        out[c] = sc * v;
    }
}

// S_inv = S^-1 = (R^T, -R^T t / s, 1 / s) in float64, and its float32 form.
__global__ void sim3_inverse_kernel(const double* __restrict__ S_in, double* __restrict__ S_out,
                                    fl_sim3* __restrict__ S32) {
    if (threadIdx.x != 0) return;
    const Sim3d V = sim3_inv(sim3_load(S_in));
    if (S_out) sim3_store(V, S_out);
    if (S32) sim3_to_f32(V, S32);
}

__global__ void gn_step_kernel(const double* __restrict__ g, const double* __restrict__ H, double lambda,
                               double* __restrict__ S_io, fl_sim3* __restrict__ S32) {
    if (threadIdx.x != 0) return;
    double d[7];
    Sim3d S = sim3_load(S_io);
    if (solve7(g, H, lambda, d)) {
        S = sim3_mul(sim3_exp(d), S);
        sim3_store(S, S_io);
    }
    if (S32) sim3_to_f32(S, S32);
}

// ---------------------------------------------------------------------------
// Per-event refinement inside a batch, all Gauss-Newton steps in one launch.
// refine_blocks workgroups per event accumulate g and H over the event's
// accepted pairs (recorded by the search as point + observation + keyframe,
// held in registers across the steps), publish their partial sums as tagged
// rows and wait until every row of the step is tagged; every workgroup then
// sums the rows in the same order and solves the same 7x7 system, so all of
// them hold the bitwise-identical next Sim3 without a second exchange.  The
// wait only involves workgroups of the same event, which are co-resident (the
// whole grid is one workgroup per CU); its spin is bounded and a timeout is
// reported as n_matched = -1.

constexpr unsigned kSpinLimit = 1u << 22;

// One pair's terms at S (float32), added when the pair is in front of its
// keyframe; acc[35] counts the pairs added.
__device__ __forceinline__ void refine_accumulate_f32(const float* T, float fx, float fy, float cx, float cy, float x,
                                                      float y, float z, float uo, float vo, const fl_sim3& S,
                                                      float delta, float* acc) {
    PairTerm t;
    pair_term(S.sR, S.t, T, fx, fy, cx, cy, x, y, z, uo, vo, delta, true, t);
    if (t.valid) {
        accumulate_f32(t, acc);
        acc[35] += 1.0f;
    }
}

// A pair of the other direction (a point of the current side observed in a
// loop-side keyframe through S^-1, Si = float32 form of S^-1): its terms with
// respect to the left perturbation of S, added when the point is in front of
// that keyframe.  The keyframe's pose and intrinsics come from LDS (16 floats
// per keyframe: T, fx, fy, cx, cy) or from the caller's arrays.
__device__ __forceinline__ void refine_inverse_f32(const BatchHdr& h, const float* s_ikf, bool lds, int k, float x,
                                                   float y, float z, float uo, float vo, const fl_sim3& Si,
                                                   float delta, float* acc) {
    const float* T;
    float fx, fy, cx, cy;
    if (lds) {
        T = s_ikf + 16 * k;
        fx = T[12];
        fy = T[13];
        cx = T[14];
        cy = T[15];
    } else {
        T = h.inv_T + 12 * (int64_t)k;
        const float* c = h.inv_cam + 4 * (int64_t)k;
        fx = c[0];
        fy = c[1];
        cx = c[2];
        cy = c[3];
    }
    PairTerm t;
    pair_term<true>(Si.sR, Si.t, T, fx, fy, cx, cy, x, y, z, uo, vo, delta, true, t);
    if (t.valid) {
        accumulate_f32(t, acc);
        acc[35] += 1.0f;
    }
}

// A pair's reprojection error at a float64 Sim3 (13 doubles: R, t, s), in
// float64 throughout; false when the pair is behind its keyframe.  The
// quantities that decide something (a Levenberg-Marquardt step's Huber loss,
// whether a pair is an inlier of a round) are evaluated this way: their
// float32 form carries ~1e-5 px of rounding per pair, enough to turn a
// near-tie either way.
__device__ __forceinline__ bool pair_error64(const double* S, const float* T, float fx, float fy, float cx, float cy,
                                             float x, float y, float z, float uo, float vo, double& e) {
    const double X = x, Y = y, Z = z, sc = S[12];
    double p[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = sc * (S[3 * i] * X + S[3 * i + 1] * Y + S[3 * i + 2] * Z) + S[9 + i];
    double q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        q[i] = (double)T[3 * i] * p[0] + (double)T[3 * i + 1] * p[1] + (double)T[3 * i + 2] * p[2] + (double)T[9 + i];
    if (!(q[2] > 0.0)) {
        e = 0.0;
        return false;
    }
    const double r0 = (double)fx * q[0] / q[2] + (double)cx - (double)uo;
    const double r1 = (double)fy * q[1] / q[2] + (double)cy - (double)vo;
    e = sqrt(r0 * r0 + r1 * r1);
    return true;
}

__device__ __forceinline__ double huber64(double e, double delta) {
    return e <= delta ? 0.5 * e * e : delta * e - 0.5 * delta * delta;
}

// Fixed-order float64 sum over the block: a wave butterfly (every lane ends
// with the same value: each stage adds the same two numbers in both lanes),
// then the wave totals in wave order.  s_w holds one double per wave.
__device__ __forceinline__ double block_sum_f64(double v, double* s_w) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (wave_lane() == 0) s_w[threadIdx.x / kWave] = v;
    __syncthreads();
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) sum += s_w[w];
    return sum;
}

// S <- exp(d) S by the lanes of one wave: every lane holds the same step d
// and evaluates the exponential's coefficients; lane l < 13 then computes
// entry l of the product (R row-major, t, s) from the rows of exp(d)
// (R_d = I + a W + b W^2 and V = c0 I + c1 W + c2 W^2 with W = [omega]x and
// W^2 = omega omega^T - |omega|^2 I) and from S in LDS, writes it to S64 and
// its float32 pose to o32; with inv32 the lanes then write the float32 pose
// of the product's inverse (R^T / s, -R^T t / s).  S64 is read by every lane
// before any lane writes it (one wave: its LDS accesses are in order).
__device__ __forceinline__ void compose_exp_lanes(const double* d, double* S64, fl_sim3* o32, fl_sim3* inv32) {
    const int l = wave_lane();
    const ExpCoef k = sim3_exp_coef(d[0], d[1], d[2], d[6]);
    const double w0 = d[0], w1 = d[1], w2 = d[2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    // this lane's row i of R_d and V: lanes 0-8 entry (i, j) = (l / 3, l % 3)
    // of the rotation, lanes 9-11 row l - 9 of the translation
    const int i = l < 9 ? l / 3 : (l < 12 ? l - 9 : 0);
    const int j = l < 9 ? l % 3 : 0;
    const double wi = i == 0 ? w0 : (i == 1 ? w1 : w2);
    // row i of W: (0, -w2, w1), (w2, 0, -w0), (-w1, w0, 0)
    const double W0 = i == 0 ? 0.0 : (i == 1 ? w2 : -w1);
    const double W1 = i == 0 ? -w2 : (i == 1 ? 0.0 : w0);
    const double W2 = i == 0 ? w1 : (i == 1 ? -w0 : 0.0);
    const double Q0 = wi * w0 - (i == 0 ? th2 : 0.0);   // row i of W^2
    const double Q1 = wi * w1 - (i == 1 ? th2 : 0.0);
    const double Q2 = wi * w2 - (i == 2 ? th2 : 0.0);
    const double R0 = (i == 0 ? 1.0 : 0.0) + k.a * W0 + k.b * Q0;
    const double R1 = (i == 1 ? 1.0 : 0.0) + k.a * W1 + k.b * Q1;
    const double R2 = (i == 2 ? 1.0 : 0.0) + k.a * W2 + k.b * Q2;
    const double s_new = k.es * S64[12];
    double v;
    if (l < 9) {
        v = R0 * S64[j] + R1 * S64[3 + j] + R2 * S64[6 + j];
    } else if (l < 12) {
        const double V0 = (i == 0 ? k.c0 : 0.0) + k.c1 * W0 + k.c2 * Q0;
        const double V1 = (i == 1 ? k.c0 : 0.0) + k.c1 * W1 + k.c2 * Q1;
        const double V2 = (i == 2 ? k.c0 : 0.0) + k.c1 * W2 + k.c2 * Q2;
        v = k.es * (R0 * S64[9] + R1 * S64[10] + R2 * S64[11]) + (V0 * d[3] + V1 * d[4] + V2 * d[5]);
    } else {
        v = s_new;
    }
    if (l < 13) S64[l] = v;
    if (l < 9) o32->sR[l] = (float)(s_new * v);
    else if (l < 12) o32->t[l - 9] = (float)v;
    // the new entries are written before any lane reads them
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (inv32) {
        const double inv_s = 1.0 / s_new;
        if (l < 9) {
            inv32->sR[l] = (float)(inv_s * S64[3 * j + i]);
        } else if (l < 12) {
            inv32->t[i] = (float)(-(S64[i] * S64[9] + S64[3 + i] * S64[10] + S64[6 + i] * S64[11]) * inv_s);
        }
    }
}

constexpr int kRefCache = 2;     // accepted pairs a thread keeps in registers across the steps
constexpr int kRefKfLds = 64;    // keyframes of one event whose pose and intrinsics sit in LDS
constexpr int kRefMaxB = 64;     // workgroups per event
constexpr int kRefBlock = 512;   // threads of a refinement workgroup: 64 x 512 pairs at one per thread
constexpr int kNAccLM = 40;      // the sums plus the Huber loss (slot 36), padded to a multiple of 4
// Each float64 partial travels as two 64-bit words, (high half << 32 | tag)
// and (low half << 32 | tag): a word is written and read in one piece, so a
// reader that sees the tag of the current launch and step in both words has
// the value, without a separate flag or any cache maintenance.  Rows are
// laid out for the larger (Levenberg-Marquardt) sum set.
constexpr int kRefWords = 2 * kNAccLM;
constexpr double kLmConverged = 1e-6;   // relative loss change that ends a round

// The refinement of each event in rounds.  Round 0 uses every accepted
// pair; a later round uses the pairs in front of their keyframe whose error
// at the round's starting Sim3 is within outlier_px.  A round is
// refine_iters evaluations of the sums.  Gauss-Newton (LM false) steps to
// S <- exp(d) S after every evaluation, d solving H d = -g.  Levenberg-
// Marquardt (LM true) evaluates the round's starting Sim3, then candidates
// exp(d) S_acc with (H + lambda diag H) d = -g at the accepted S_acc.  With
// rho the candidate's relative drop of the Huber loss below S_acc's: rho >
// 1e-6 takes it (lambda / 10, at least 1e-12), |rho| <= 1e-6 ends the round
// (converged; every workgroup holds the same sums, so all of them leave the
// round together), rho < -1e-6 drops it (lambda x 10, at most 1e16).
// lambda restarts at lm_lambda each round and the round ends at S_acc.
// ROUNDS false compiles the single-round kernel (no inlier tests).
template <bool LM, bool ROUNDS>
__global__ __launch_bounds__(kRefBlock) void refine_kernel(const BatchHdr* __restrict__ hp) {
    constexpr int NV = LM ? kNAccLM : kNAcc;
    __shared__ float s_big[NV * (kRefBlock / 4 + 1)];   // the block reduction's transpose
    __shared__ double s_q[kSeg * NV];
    __shared__ double s_out[NV];
    __shared__ float s_kf[kRefKfLds * 16];   // per keyframe: T (12), fx, fy, cx, cy
    __shared__ float s_ikf[(LM || ROUNDS) ? 16 : kRefKfLds * 16];   // the same for the other direction's keyframes
    __shared__ double s_S64[13];
    __shared__ fl_sim3 s_S;
    __shared__ fl_sim3 s_Sinv;               // float32 form of S^-1 (two-sided refinement)
    __shared__ double s_Srs64[13];           // the round's starting Sim3 (inlier tests)
    __shared__ double s_wsum[kRefBlock / kWave];
    __shared__ double s_acc[kNAcc];          // LM: g, H and count at S_acc
    __shared__ double s_Sacc[13];            // LM: S_acc
    __shared__ double s_lm[2];               // LM: loss at S_acc, lambda
    __shared__ int s_fail;
    __shared__ int s_round_end;              // LM: the round converged at this step
    const BatchHdr& h = *hp;
    const int B = h.refine_blocks;
    const int n_units = h.n_events * B;
    const int iters = h.refine_iters;
    const int total = iters * (ROUNDS ? h.refine_rounds : 1);
    const float delta = h.huber_delta;
    const float tau = h.outlier_px;
    const int tid = threadIdx.x;
    const uint32_t epoch = *h.epoch;
    for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
        const int ev = unit / B, b = unit % B;
        const EventDesc ed = h.ev[ev];
        const int n_kf_ev = ed.kf_end - ed.kf_begin;
        const bool kf_lds = n_kf_ev <= kRefKfLds;
        if (tid < 13) s_S64[tid] = h.event_S[13 * (int64_t)ev + tid];
        if (tid == 0) s_fail = 0;
        if (kf_lds) {
            for (int i = tid; i < n_kf_ev * 16; i += blockDim.x) {
                const KfDesc& kd = h.kf[ed.kf_begin + (i >> 4)];
                const int f = i & 15;
                s_kf[i] = f < 12 ? kd.T[f] : f == 12 ? kd.fx : f == 13 ? kd.fy : f == 14 ? kd.cx : kd.cy;
            }
        }
        // two-sided refinement (Gauss-Newton only): the event's pairs of the
        // other direction and their keyframes
        const int n_inv = (LM || ROUNDS) ? 0 : ed.inv_n;
        const bool ikf_lds = h.inv_n_kf <= kRefKfLds;
        if (n_inv > 0 && ikf_lds) {
            for (int i = tid; i < h.inv_n_kf * 16; i += blockDim.x) {
                const int k = i >> 4, f = i & 15;
                s_ikf[i] = f < 12 ? h.inv_T[12 * k + f] : h.inv_cam[4 * k + f - 12];
            }
        }
        __syncthreads();
        if (tid == 0) {
            const Sim3d S0 = sim3_load(s_S64);
            sim3_to_f32(S0, &s_S);
            if (n_inv > 0) sim3_to_f32_pose(sim3_inv(S0), &s_Sinv);
        }
        const uint32_t cnt = h.ev_ctr[ev * kEvCtrs + kEvMatch];
        const bool use_list = !h.refine_scan && cnt <= (uint32_t)ed.list_cap;
        // With the list, the event uses only as many workgroups as give each
        // thread one pair of each direction (every workgroup reads the same
        // counts, so all agree on Be); the others have nothing to add and
        // skip the event.
        const uint32_t per_dir = max(cnt, (uint32_t)n_inv);
        const int Be = use_list ? max(1, min(B, (int)((per_dir + blockDim.x - 1) / blockDim.x))) : B;
        if (b >= Be) {
            __syncthreads();
            continue;
        }
        const int stride = Be * blockDim.x;
        // this thread's first kRefCache accepted pairs, loaded once, and
        // whether each is an inlier of the current round
        float cx_[kRefCache], cy_[kRefCache], cz_[kRefCache], cu_[kRefCache], cv_[kRefCache];
        int ck_[kRefCache];
        bool in_[kRefCache];
#pragma unroll
        for (int r = 0; r < kRefCache; ++r) {
            const int i = b * blockDim.x + tid + r * stride;
            ck_[r] = -1;
            in_[r] = true;
            if (use_list && i < (int)cnt) {
                const MatchRec m = h.match_list[ed.list_off + i];
                cx_[r] = m.x;
                cy_[r] = m.y;
                cz_[r] = m.z;
                cu_[r] = m.u;
                cv_[r] = m.v;
                ck_[r] = m.kf;
            }
        }
        // and its first pair of the other direction
        float ix_ = 0.0f, iy_ = 0.0f, iz_ = 0.0f, iu_ = 0.0f, iv_ = 0.0f;
        int ik_ = -1;
        if (b * (int)blockDim.x + tid < n_inv) {
            const int64_t g = ed.inv_off + (int64_t)b * blockDim.x + tid;
            ix_ = h.inv_xyz[3 * g];
            iy_ = h.inv_xyz[3 * g + 1];
            iz_ = h.inv_xyz[3 * g + 2];
            iu_ = h.inv_uv[2 * g];
            iv_ = h.inv_uv[2 * g + 1];
            const int k = h.inv_kf[g];
            ik_ = (k >= 0 && k < h.inv_n_kf) ? k : -1;
        }
        __syncthreads();
        // it: evaluation index (round it / iters); seq: exchanges done, which
        // picks the row buffer and the tag (a converged round skips the rest
        // of its evaluations, in every workgroup alike)
        for (int it = 0, seq = 0; it < total; ++it, ++seq) {
            const int rnd = it / iters, j = it - rnd * iters;
            const fl_sim3 S = s_S;
            // a round after the first keeps its inliers: a pair held in
            // registers is classified at the round's first evaluation (at the
            // round's starting Sim3); any other pair is tested against that
            // Sim3 at every step
            const bool bounded = ROUNDS && rnd > 0;
            const bool classify = bounded && j == 0;
            // Each thread adds its few pairs' terms in float32 (one pair per
            // thread when the list fits the workgroups, a couple of dozen at
            // most when the event's pairs are scanned); everything across
            // threads and workgroups is summed in float64.
            float accf[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) accf[i] = 0.0f;
            double lossd = 0.0;   // LM: the Huber loss of this thread's pairs, float64
            if (use_list) {
#pragma unroll
                for (int r = 0; r < kRefCache; ++r) {
                    if (ck_[r] < 0 || !(in_[r] || classify)) continue;
                    const float* T;
                    float fx, fy, px, py;
                    if (kf_lds) {
                        const float* q = &s_kf[16 * (ck_[r] - ed.kf_begin)];
                        T = q;
                        fx = q[12];
                        fy = q[13];
                        px = q[14];
                        py = q[15];
                    } else {
                        const KfDesc& kd = h.kf[ck_[r]];
                        T = kd.T;
                        fx = kd.fx;
                        fy = kd.fy;
                        px = kd.cx;
                        py = kd.cy;
                    }
                    double e;
                    if (classify) {
                        in_[r] = pair_error64(s_Srs64, T, fx, fy, px, py, cx_[r], cy_[r], cz_[r], cu_[r], cv_[r], e) &&
                                 e <= (double)tau;
                        if (!in_[r]) continue;
                    }
                    refine_accumulate_f32(T, fx, fy, px, py, cx_[r], cy_[r], cz_[r], cu_[r], cv_[r], S, delta, accf);
                    if (LM && pair_error64(s_S64, T, fx, fy, px, py, cx_[r], cy_[r], cz_[r], cu_[r], cv_[r], e))
                        lossd += huber64(e, (double)delta);
                }
                for (int i = b * blockDim.x + tid + kRefCache * stride; i < (int)cnt; i += stride) {
                    const MatchRec m = h.match_list[ed.list_off + i];
                    const KfDesc& kd = h.kf[m.kf];
                    double e;
                    if (bounded && !(pair_error64(s_Srs64, kd.T, kd.fx, kd.fy, kd.cx, kd.cy, m.x, m.y, m.z, m.u, m.v,
                                                  e) && e <= (double)tau))
                        continue;
                    refine_accumulate_f32(kd.T, kd.fx, kd.fy, kd.cx, kd.cy, m.x, m.y, m.z, m.u, m.v, S, delta, accf);
                    if (LM && pair_error64(s_S64, kd.T, kd.fx, kd.fy, kd.cx, kd.cy, m.x, m.y, m.z, m.u, m.v, e))
                        lossd += huber64(e, (double)delta);
                }
            } else {
                // no list (or it overflowed): scan the event's pairs keyframe by keyframe
                for (int k = ed.kf_begin; k < ed.kf_end; ++k) {
                    const KfDesc& kd = h.kf[k];
                    for (int64_t jj = b * blockDim.x + tid; jj < kd.n_pairs; jj += stride) {
                        const int64_t o = kd.pair_off + jj;
                        const uint8_t dec = h.out[0].decision[o];
                        if (dec != FL_ADD && dec != FL_FUSE) continue;
                        const int32_t lp = h.dense ? (int32_t)jj : h.pair_mp[o];
                        const int32_t bi = h.out[0].best_idx[o];
                        if (lp < 0 || lp >= kd.n_mp || bi < 0 || bi >= kd.n_kp) continue;
                        const int64_t gp = kd.mp_off + lp, kp = kd.kp_off + bi;
                        const float x = h.mp_xyz[3 * gp], y = h.mp_xyz[3 * gp + 1], z = h.mp_xyz[3 * gp + 2];
                        const float uo = h.kp_xy[2 * kp], vo = h.kp_xy[2 * kp + 1];
                        double e;
                        if (bounded && !(pair_error64(s_Srs64, kd.T, kd.fx, kd.fy, kd.cx, kd.cy, x, y, z, uo, vo, e) &&
                                         e <= (double)tau))
                            continue;
                        refine_accumulate_f32(kd.T, kd.fx, kd.fy, kd.cx, kd.cy, x, y, z, uo, vo, S, delta, accf);
                        if (LM && pair_error64(s_S64, kd.T, kd.fx, kd.fy, kd.cx, kd.cy, x, y, z, uo, vo, e))
                            lossd += huber64(e, (double)delta);
                    }
                }
            }
            if (n_inv > 0) {
                const fl_sim3 Si = s_Sinv;
                if (ik_ >= 0)
                    refine_inverse_f32(h, s_ikf, ikf_lds, ik_, ix_, iy_, iz_, iu_, iv_, Si, delta, accf);
                for (int i = b * blockDim.x + tid + stride; i < n_inv; i += stride) {
                    const int64_t g = ed.inv_off + (int64_t)i;
                    const int k = h.inv_kf[g];
                    if (k < 0 || k >= h.inv_n_kf) continue;
                    refine_inverse_f32(h, s_ikf, ikf_lds, k, h.inv_xyz[3 * g], h.inv_xyz[3 * g + 1],
                                       h.inv_xyz[3 * g + 2], h.inv_uv[2 * g], h.inv_uv[2 * g + 1], Si, delta, accf);
                }
            }
            // the per-thread float32 sums go through LDS as they are and are
            // widened as the segments are added
            block_reduce_quad<NV, kRefBlock>(accf, s_big, s_q, s_out);
            if (LM) {
                const double loss = block_sum_f64(lossd, s_wsum);
                if (tid == 0) s_out[36] = loss;
                __syncthreads();
            }
            if (Be > 1) {
                // Exchange of the Be partial sums of this step as tagged words
                // (device-coherent stores and loads).  Rows alternate between
                // two buffers by step: a workgroup writes step it + 2 only
                // after it has read every row of step it + 1, which every
                // workgroup writes only after reading all rows of step it.
                const size_t slot = ((size_t)(seq & 1) * n_units + (size_t)ev * B);   // rows of this step: Be
                unsigned long long* rows = h.refine_rows + slot * kRefWords;
                const uint32_t tag = refine_tag(epoch, seq);
                if (tid < 2 * NV) {
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(s_out[tid >> 1]);
                    const uint32_t half = (tid & 1) ? (uint32_t)bits : (uint32_t)(bits >> 32);
                    __hip_atomic_store(&rows[(size_t)b * kRefWords + tid], ((unsigned long long)half << 32) | tag,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                // Thread (c, q) loads the two words of value c of rows q,
                // q + kSeg, ... (words whose tag is not yet the current one are
                // loaded again) and adds those rows in that order; then the
                // segments are added pairwise.  The order is the same in every
                // workgroup, so all of them solve for bitwise the same step.
                if (tid < kSeg * NV) {
                    const int c = tid % NV, q = tid / NV;
                    constexpr int kRowsPer = kRefMaxB / kSeg;
                    unsigned long long wh[kRowsPer], wl[kRowsPer];
                    uint32_t pending = 0;
#pragma unroll
                    for (int jr = 0; jr < kRowsPer; ++jr)
                        if (q + kSeg * jr < Be) pending |= 1u << jr;
                    unsigned spins = 0;
                    while (pending) {
#pragma unroll
                        for (int jr = 0; jr < kRowsPer; ++jr)
                            if (pending >> jr & 1u) {
                                const unsigned long long* w = rows + (size_t)(q + kSeg * jr) * kRefWords + 2 * c;
                                wh[jr] = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                wl[jr] = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            }
#pragma unroll
                        for (int jr = 0; jr < kRowsPer; ++jr)
                            if ((pending >> jr & 1u) && (uint32_t)wh[jr] == tag && (uint32_t)wl[jr] == tag)
                                pending &= ~(1u << jr);
                        if (pending) {
                            // no back-off: each round is a device-memory round
                            // trip already, and a pause only delays the last row
                            if (++spins > kSpinLimit) {
                                s_fail = 1;
                                break;
                            }
                        }
                    }
                    double a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int jr = 0; jr < kRowsPer; ++jr) {
                        if (q + kSeg * jr < Be) {
                            const double x = __longlong_as_double(
                                (long long)((wh[jr] >> 32 << 32) | (wl[jr] >> 32)));
                            if (jr & 1) a1 += x; else a0 += x;
                        }
                    }
                    s_q[q * NV + c] = a0 + a1;
                }
                __syncthreads();
                if (s_fail) break;
                if (tid < NV) s_out[tid] = add_segments<NV>(s_q, tid);
                __syncthreads();
            }
            if (!LM && tid < kWave) {
                // Gauss-Newton: every lane of wave 0 solves for the same step,
                // then the lanes compose it with S together
                double d[7];
                if (solve7(s_out, s_out + 7, 0.0, d)) compose_exp_lanes(d, s_S64, &s_S, n_inv > 0 ? &s_Sinv : nullptr);
            }
            if (tid == 0) {
                bool round_end = j == iters - 1;
                if (LM) {
                    // the evaluation just summed was at s_S64: the round's start
                    // (j = 0) or the last candidate
                    bool take = j == 0;
                    if (j == 0) {
                        s_lm[1] = (double)h.lm_lambda;
                    } else {
                        const double rho = s_lm[0] > 0.0 ? (s_lm[0] - s_out[36]) / s_lm[0] : 0.0;
                        take = rho > kLmConverged;
                        if (!take && rho >= -kLmConverged) round_end = true;   // converged
                    }
                    if (take) {
                        for (int i = 0; i < kNAcc; ++i) s_acc[i] = s_out[i];
                        for (int i = 0; i < 13; ++i) s_Sacc[i] = s_S64[i];
                        s_lm[0] = s_out[36];
                        if (j > 0) s_lm[1] = fmax(s_lm[1] * 0.1, 1e-12);
                    } else if (!round_end) {
                        s_lm[1] = fmin(s_lm[1] * 10.0, 1e16);
                    }
                    const Sim3d Sa = sim3_load(s_Sacc);
                    double d[7];
                    if (!round_end && solve7(s_acc, s_acc + 7, s_lm[1], d)) {
                        const Sim3d Sd = sim3_mul(sim3_exp(d), Sa);
                        sim3_store(Sd, s_S64);
                        sim3_to_f32_pose(Sd, &s_S);
                    } else {
                        sim3_store(Sa, s_S64);
                        sim3_to_f32_pose(Sa, &s_S);
                    }
                }
                if (round_end)
                    for (int i = 0; i < 13; ++i) s_Srs64[i] = s_S64[i];   // the next round's starting Sim3
                s_round_end = round_end;
            }
            __syncthreads();
            if (LM && s_round_end) it = (rnd + 1) * iters - 1;   // on to the next round
        }
        if (b == 0 && tid == 0) {
            if (!s_fail) {
                for (int i = 0; i < 13; ++i) h.event_S[13 * (int64_t)ev + i] = s_S64[i];
                if (h.event_S32_out) sim3_to_f32(sim3_load(s_S64), &h.event_S32_out[ev]);
            }
            if (h.event_n_matched)
                h.event_n_matched[ev] = s_fail ? -1 : (int32_t)(LM ? s_acc[35] : s_out[35]);
            h.ev_ctr[ev * kEvCtrs + kEvMatch] = 0;   // the event's list is spent
        }
        __syncthreads();
    }
    // The ADD conflicts of the search that precedes this launch: the search
    // workgroups' ADD regions go to workgroups from the last one down, so
    // workgroups with no refinement work (most of them for a single event)
    // take them while the others iterate.  The refinement reads accepted
    // pairs only, which an ADD and its relabelling as FUSE both are.
    if (h.resolve_in_refine) {
        const unsigned long long tag = (unsigned long long)(*h.epoch) << 32;
        for (int r = (int)(gridDim.x - 1 - blockIdx.x); r < h.n_wg; r += (int)gridDim.x)
            resolve_region_adds(h, r, tag);
    }
}

}  // namespace fl
