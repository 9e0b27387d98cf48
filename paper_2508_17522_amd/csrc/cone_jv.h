// Jacobian-vector products of the projections onto the dual cones (Appendix A), written as
// device templates shared by the single-problem and the batched kernels. Each takes an
// input functor in(r) and an output functor out(r, value) over global y-row indices r.
#pragma once

#include "qcpd_internal.h"

namespace qcpd {

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kRsqrt2 = 0.70710678118654752440;

__device__ inline int exp_row(const Problem &p, int cone) {
    return p.exp_rows ? p.exp_rows[cone] : p.exp_row0 + 3 * cone;
}

// ---------------------------------------------------------------------------------------
// cone Jacobian-vector products, J = DPi_{K*}(z_y) per block
// ---------------------------------------------------------------------------------------

// Second-order cone (self-dual), one thread per cone. par = (mode, 1/||u||, c1, c2):
// mode 0: J = 0; mode 1: J = I; mode 2 (||u|| > |t|):
//   J(dt, du) = (1/2 (dt + uh'du),  1/2 uh dt + c1 du - c2 (uh'du) uh),
//   uh = u/||u||, c1 = (t + ||u||)/(2||u||), c2 = t/(2||u||).
template <class IN, class OUT>
__device__ inline void soc_jv(const Problem &p, int cone, IN in, OUT out) {
    const int r0 = p.soc_row[cone], k = p.soc_dim[cone];
    const double *par = p.soc_par + 4 * cone;
    const int mode = (int)par[0];
    if (mode == 0) {
        for (int i = 0; i < k; ++i) out(r0 + i, 0.0);
        return;
    }
    if (mode == 1) {
        for (int i = 0; i < k; ++i) out(r0 + i, in(r0 + i));
        return;
    }
    const double inv_nu = par[1], c1 = par[2], c2 = par[3];
    const double *u = p.zy + r0 + 1;
    const double dt = in(r0);
    double a = 0.0;
    for (int i = 1; i < k; ++i) a += u[i - 1] * inv_nu * in(r0 + i);
    out(r0, 0.5 * (dt + a));
    for (int i = 1; i < k; ++i) {
        const double uh = u[i - 1] * inv_nu;
        out(r0 + i, 0.5 * uh * dt + c1 * in(r0 + i) - c2 * a * uh);
    }
}

// Dual exponential cone, one thread per cone: a stored 3x3 matrix (I - DPi_exp(-z)).
template <class IN, class OUT>
__device__ inline void exp_jv(const Problem &p, int cone, IN in, OUT out) {
    const int r0 = exp_row(p, cone);
    const double *J = p.exp_J + 9 * cone;
    const double a = in(r0), b = in(r0 + 1), c = in(r0 + 2);
    out(r0, J[0] * a + J[1] * b + J[2] * c);
    out(r0 + 1, J[3] * a + J[4] * b + J[5] * c);
    out(r0 + 2, J[6] * a + J[7] * b + J[8] * c);
}

__device__ inline int svec_index(int i, int j, int k) {  // i >= j
    return j * k - (j * (j - 1)) / 2 + (i - j);
}

// PSD cone on svec coordinates, one workgroup per cone:
//   J[dZ] = V (B o (V' dZ V)) V'.
// LDS: X, T, V as k x ld matrices (ld = k | 1, odd, to spread LDS banks).
template <class IN, class OUT>
__device__ inline void psd_jv(const Problem &p, int cone, double *sm, IN in, OUT out) {
    const int k = p.psd_k[cone], r0 = p.psd_row[cone];
    const int ld = k | 1, kk = k * k;
    const double *Vg = p.psd_pool + p.psd_off[cone];
    const double *Bg = Vg + kk;
    double *X = sm, *T = sm + k * ld, *V = sm + 2 * k * ld;
    const int tid = threadIdx.x;
    for (int e = tid; e < kk; e += kBlock) {
        const int i = e / k, j = e - (e / k) * k;
        V[i * ld + j] = Vg[e];
        if (i >= j) {
            double v = in(r0 + svec_index(i, j, k));
            if (i == j) {
                X[i * ld + i] = v;
            } else {
                v *= kRsqrt2;
                X[i * ld + j] = v;
                X[j * ld + i] = v;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < kk; e += kBlock) {  // T = X V
        const int i = e / k, j = e - (e / k) * k;
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc += X[i * ld + l] * V[l * ld + j];
        T[i * ld + j] = acc;
    }
    __syncthreads();
    for (int e = tid; e < kk; e += kBlock) {  // X = B o (V' T)
        const int i = e / k, j = e - (e / k) * k;
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc += V[l * ld + i] * T[l * ld + j];
        X[i * ld + j] = Bg[e] * acc;
    }
    __syncthreads();
    for (int e = tid; e < kk; e += kBlock) {  // T = V X
        const int i = e / k, j = e - (e / k) * k;
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc += V[i * ld + l] * X[l * ld + j];
        T[i * ld + j] = acc;
    }
    __syncthreads();
    for (int e = tid; e < kk; e += kBlock) {  // Y = T V', lower triangle into svec
        const int i = e / k, j = e - (e / k) * k;
        if (i >= j) {
            double acc = 0.0;
            for (int l = 0; l < k; ++l) acc += T[i * ld + l] * V[j * ld + l];
            out(r0 + svec_index(i, j, k), i == j ? acc : acc * kSqrt2);
        }
    }
    __syncthreads();
}

__host__ __device__ inline int psd_stage_offset(int k) { return 3 * k * (k | 1); }

}  // namespace qcpd
