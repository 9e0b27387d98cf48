// LSMR (Fong & Saunders 2011), the method the paper solves both least-squares problems with
// (Sec. 3.1 "Computing the derivative", Sec. 3.2 "Computing the adjoint"). It builds the same
// Golub-Kahan bidiagonalisation as LSQR, so the two product launches of an iteration are the
// LSQR loop kernels themselves (roles U and V, without LSQR's owed x update); a third launch,
// k_lsmr_step, takes the V launch's partial sums (alpha_{k+1}), runs LSMR's recurrences and
// updates the iterate:
//   first QR of the bidiagonal matrix:  rho_k = |(alphabar_k, beta_{k+1})|, c, s,
//                                       theta_{k+1} = s alpha_{k+1}, alphabar_{k+1} = c alpha_{k+1}
//   second QR:                          thetabar_k = sbar rho_k, rhobar_k = |(cbar rho_k, theta_{k+1})|,
//                                       zeta_k = cbar' zetabar, zetabar <- -sbar' zetabar
//   hbar_k = h_k - (thetabar_k rho_k / (rho_{k-1} rhobar_{k-1})) hbar_{k-1}
//   x_k    = x_{k-1} + (zeta_k / (rho_k rhobar_k)) hbar_k
//   h_{k+1} = v_{k+1} - (theta_{k+1} / rho_k) h_k
// and the estimate of ||r_k|| from a third QR (of Rbar_k'), whose leading entries are fixed
// once computed: ||r_k||^2 = fixed part + (betadot - taudot)^2 + betadd^2.
// Every workgroup sums the partials in the same fixed order and thread 0 of each runs the
// scalar recurrences (identical in every workgroup); workgroup 0 writes the state for the
// next iteration. The LSMR scalars are double-buffered by the parity of the iteration count,
// so the buffer a launch reads is never the one it writes.
#include <algorithm>

#include "qcpd_internal.h"

namespace qcpd {

namespace {

constexpr int kLsmrPartRegs = kMaxLoopGrid / kBlock;

// Sum of the partials (two doubles per slot, slots < nslots) over the workgroup, in a fixed
// order; valid in thread 0.
__device__ inline void partial_totals(const double *part, int nslots, double &t0, double &t1) {
    __shared__ double sh[2][kBlock];
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int j = 0; j < kLsmrPartRegs; ++j) {
        const int i = threadIdx.x + j * kBlock;
        if (i < nslots) {
            a += part[2 * i];
            b += part[2 * i + 1];
        }
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    t0 = sh[0][0];
    t1 = sh[1][0];
}

// The recurrences of one iteration (thread 0). Returns false when no update is to be
// applied (a zero rotation: the bidiagonalisation has terminated).
__device__ inline bool lsmr_scalars(LsqrState &st, LsmrState &L, double alpha, double coef[3]) {
    const double beta = st.beta, alphabar = L.alphabar;
    const double rho = sqrt(alphabar * alphabar + beta * beta);
    if (!(rho > 0.0)) return false;
    const double c = alphabar / rho, s = beta / rho;
    const double theta_next = s * alpha;
    L.alphabar = c * alpha;
    const double thetabar = L.sbar * rho;
    const double crho = L.cbar * rho;
    const double rhobar = sqrt(crho * crho + theta_next * theta_next);
    if (!(rhobar > 0.0)) return false;
    const double cbar = crho / rhobar, sbar = theta_next / rhobar;
    const double zeta = cbar * L.zetabar;
    L.zetabar = -sbar * L.zetabar;
    coef[0] = thetabar * rho / (L.rho_prev * L.rhobar_prev);  // of hbar_{k-1}
    coef[1] = zeta / (rho * rhobar);                          // of hbar_k in x
    coef[2] = theta_next / rho;                               // of h_k in h_{k+1}
    L.rho_prev = rho;
    L.rhobar_prev = rhobar;
    L.cbar = cbar;
    L.sbar = sbar;
    // residual estimate
    const double betahat = c * L.betadd;
    L.betadd = -s * L.betadd;
    const double rhodot = L.rhodot;
    const double rhotil = sqrt(rhodot * rhodot + thetabar * thetabar);
    const double ctil = rhodot / rhotil, stil = thetabar / rhotil;
    L.rhodot = ctil * rhobar;
    const double betatil = ctil * L.betadot + stil * betahat;
    L.betadot = -stil * L.betadot + ctil * betahat;
    if (st.iters > 0) {  // from the second iteration on, entry k-1 of tau is final
        const double tautil = (L.zeta_prev - L.thetatil * L.tautil_prev) / rhotil;
        const double d = betatil - tautil;
        L.fixed_sq += d * d;
        L.tautil_prev = tautil;
    }
    L.thetatil = stil * rhobar;
    const double taudot = (zeta - L.thetatil * L.tautil_prev) / L.rhodot;
    L.zeta_prev = zeta;
    const double e = L.betadot - taudot;
    st.phibar = sqrt(L.fixed_sq + e * e + L.betadd * L.betadd);
    return true;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_lsmr_step(LsmrArgs a) {
    __shared__ double coef[4];  // chb, phr, thr, 1/alpha
    __shared__ int go;
    const LsqrState *stp = a.st;
    const bool live = !stp->done && stp->pend_role == ROLE_V;
    double t0 = 0.0, t1 = 0.0;
    if (live) partial_totals(a.part, stp->pend_blocks, t0, t1);
    if (threadIdx.x == 0) {
        LsqrState st = *stp;
        go = 0;
        if (live) {
            const int par = st.iters & 1;
            LsmrState L = a.ls[par];
            const double alpha = sqrt(t0);
            if (st.pend_fwd) st.dot_fwd = t1; else st.dot_adj = t1;
            double cf[3];
            if (lsmr_scalars(st, L, alpha, cf)) {
                go = 1;
                coef[0] = cf[0];
                coef[1] = cf[1];
                coef[2] = cf[2];
                coef[3] = alpha > 0.0 ? 1.0 / alpha : 0.0;
                st.iters += 1;
                st.alpha = alpha;
                if (st.phibar <= st.tol * st.beta1 || !(alpha > 0.0)) {
                    st.done = 1;
                    st.conv = 1;
                } else if (st.iters >= st.max_iter) {
                    st.done = 1;
                }
            } else {
                st.done = 1;
                st.conv = 1;
            }
            st.pend_role = -1;
            st.pending = 0;
            if (blockIdx.x == 0 && go) a.ls[par ^ 1] = L;  // never the buffer being read
        }
        if (blockIdx.x == 0) *a.st_next = st;
    }
    __syncthreads();
    if (!go) return;
    const double chb = coef[0], phr = coef[1], thr = coef[2], ia = coef[3];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.N; i += gridDim.x * kBlock) {
        const double h = a.h[i];
        const double hb = h - chb * a.hb[i];
        a.hb[i] = hb;
        a.x[i] += phr * hb;
        a.h[i] = a.v[i] * ia - thr * h;
    }
}

// After the first product (alpha_1 v_1 = A'u_1): h_1 = v_1, hbar_0 = 0 and the LSMR scalars
// of iteration 1 in buffer 0.
__global__ __launch_bounds__(kBlock) void k_lsmr_init(LsmrArgs a) {
    const LsqrState *st = a.st;
    const double alpha = st->alpha, beta1 = st->beta1;
    const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        LsmrState L{};
        L.alphabar = alpha;
        L.rho_prev = 1.0;
        L.rhobar_prev = 1.0;
        L.cbar = 1.0;
        L.sbar = 0.0;
        L.zetabar = alpha * beta1;
        L.betadd = beta1;
        L.rhodot = 1.0;
        a.ls[0] = L;
    }
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.N; i += gridDim.x * kBlock) {
        a.h[i] = a.v[i] * ia;
        a.hb[i] = 0.0;
    }
}

void launch_lsmr_step(const LsmrArgs &a, hipStream_t s) {
    const int grid = std::max(1, std::min(div_up(a.N, kBlock), 2048));
    hipLaunchKernelGGL(k_lsmr_step, dim3(grid), dim3(kBlock), 0, s, a);
}

void launch_lsmr_init(const LsmrArgs &a, hipStream_t s) {
    const int grid = std::max(1, std::min(div_up(a.N, kBlock), 2048));
    hipLaunchKernelGGL(k_lsmr_init, dim3(grid), dim3(kBlock), 0, s, a);
}

}  // namespace qcpd
