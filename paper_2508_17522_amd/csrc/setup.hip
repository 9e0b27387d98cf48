// Setup at a solution (Sec. 3.1, "First, we compute Pi z ..."): A' and its slot map, Px,
// c = -2Px - q, x'Px, z_y = y - s, and the per-block factors of J = DPi_{K*}(z_y)
// (Appendix A), plus the Jacobi column scales.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "qcpd_internal.h"
#include "setup.h"

namespace qcpd {

// ---------------------------------------------------------------------------------------
// CSR transpose: a stable radix sort of the slots by column keeps each transposed row in
// increasing original-row order, so the transpose is deterministic.
// ---------------------------------------------------------------------------------------

__global__ void k_expand_rows(const int *rp, int nrows, int *rowidx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrows)
        for (int k = rp[i]; k < rp[i + 1]; ++k) rowidx[k] = i;
}

__global__ void k_iota(int *v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

__global__ void k_rowptr_from_sorted(const int *keys, int nnz, int ncols, int *rp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnz) {
        const int prev = (t == 0) ? -1 : keys[t - 1];
        for (int j = prev + 1; j <= keys[t]; ++j) rp[j] = t;
    }
    if (t == nnz) {
        const int last = (nnz == 0) ? -1 : keys[nnz - 1];
        for (int j = last + 1; j <= ncols; ++j) rp[j] = nnz;
    }
}

__global__ void k_gather_transpose(const int *perm, const int *rowidx, const double *val,
                                   int nnz, int *tci, double *tv) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnz) {
        const int k = perm[t];
        tci[t] = rowidx[k];
        tv[t] = val[k];
    }
}

hipError_t csr_transpose(int nrows, int ncols, int nnz, const int *rp, const int *ci,
                         const double *val, int *trp, int *tci, double *tv, int *perm,
                         hipStream_t s) {
    hipError_t e = hipSuccess;
    int *rowidx = nullptr, *keys_out = nullptr, *iota = nullptr;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    int end_bit = 1;
    while ((1LL << end_bit) <= ncols) ++end_bit;
    if (nnz > 0) {
        if ((e = hipMalloc(&rowidx, sizeof(int) * nnz))) goto done;
        if ((e = hipMalloc(&keys_out, sizeof(int) * nnz))) goto done;
        if ((e = hipMalloc(&iota, sizeof(int) * nnz))) goto done;
        hipLaunchKernelGGL(k_expand_rows, dim3(div_up(nrows, 256)), dim3(256), 0, s, rp, nrows, rowidx);
        hipLaunchKernelGGL(k_iota, dim3(div_up(nnz, 256)), dim3(256), 0, s, iota, nnz);
        if ((e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, ci, keys_out, iota, perm,
                                                    nnz, 0, end_bit, s)))
            goto done;
        if ((e = hipMalloc(&temp, std::max<size_t>(temp_bytes, 16)))) goto done;
        if ((e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, ci, keys_out, iota, perm,
                                                    nnz, 0, end_bit, s)))
            goto done;
        hipLaunchKernelGGL(k_gather_transpose, dim3(div_up(nnz, 256)), dim3(256), 0, s, perm,
                           rowidx, val, nnz, tci, tv);
    }
    hipLaunchKernelGGL(k_rowptr_from_sorted, dim3(div_up(nnz + 1, 256)), dim3(256), 0, s,
                       keys_out, nnz, ncols, trp);
    e = hipStreamSynchronize(s);
done:
    (void)hipFree(rowidx);
    (void)hipFree(keys_out);
    (void)hipFree(iota);
    (void)hipFree(temp);
    return e;
}

// Structural validity of a CSR matrix: rowptr[0] = 0, nondecreasing, rowptr[nrows] = nnz,
// and every column index in [0, ncols). Checked before anything indexes through it.
__global__ void k_check_csr(const int *rp, const int *ci, int nrows, int ncols, int nnz, int *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[nrows] != nnz)) atomicOr(flag, 1);
    if (i < nrows) {
        const int a = rp[i], b = rp[i + 1];
        if (a > b || a < 0 || b > nnz) {
            atomicOr(flag, 1);
            return;
        }
        for (int k = a; k < b; ++k)
            if (ci[k] < 0 || ci[k] >= ncols) {
                atomicOr(flag, 1);
                return;
            }
    }
}

// P must have strictly increasing column indices in every row, and equal its transpose.
__global__ void k_check_sorted(const int *rp, const int *ci, int nrows, int ncols, int *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrows) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= ncols || (k > rp[i] && ci[k] <= ci[k - 1])) {
                atomicOr(flag, 1);
                return;
            }
        }
    }
}

__global__ void k_check_symmetric(const int *rp, const int *ci, const double *v, const int *trp,
                                  const int *tci, const double *tv, int n, int nnz, int *flag) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= n && rp[t] != trp[t]) atomicOr(flag, 2);
    if (t < nnz) {
        if (ci[t] != tci[t]) atomicOr(flag, 2);
        const double a = v[t], b = tv[t];
        if (fabs(a - b) > 1e-12 * (fabs(a) + fabs(b)) && !(a == b)) atomicOr(flag, 4);
    }
}

// ---------------------------------------------------------------------------------------
// Px, c = -2Px - q, x'Px  (the tau-row of D_u Q at tau = 1, Sec. 2.4)
// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_px(Problem p, RowGrid g, double *c, double *xpx_out,
                                               double *partials, int *counter) {
    const int tid = threadIdx.x;
    const int L = g.lx;
    const long long gt = (long long)blockIdx.x * kBlock + tid;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    double acc = 0.0;
    if (row < p.n)
        for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) acc += p.Pv[k] * p.x[p.Pci[k]];
    for (int off = L >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    double s0 = 0.0;
    if (lane == 0 && row < p.n) {
        c[row] = -2.0 * acc - p.q[row];
        s0 = p.x[row] * acc;
    }
    double tot[3];
    if (last_block_sum3(s0, 0.0, 0.0, partials, counter, gridDim.x, tot) && tid == 0) *xpx_out = tot[0];
}

__global__ void k_sub(const double *a, const double *b, double *out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

// ---------------------------------------------------------------------------------------
// cone factors of J = DPi_{K*}(z_y)
// ---------------------------------------------------------------------------------------

constexpr double kKinkTol = 1e-10;

// zero cone rows: the dual cone is R, J = 1. nonnegative rows: J = 1{z > 0}. Every factor
// kernel also writes Pi_{K*}(z_y) of its rows to proj when that is given.
__global__ void k_diag_factors(const double *zy, int n_zero, int n_diag, double *jdiag,
                               int *nondiff, double *proj) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n_diag) {
        const double z = zy[r];
        if (r < n_zero) {
            jdiag[r] = 1.0;
            if (proj) proj[r] = z;
        } else {
            jdiag[r] = z > 0.0 ? 1.0 : 0.0;
            if (proj) proj[r] = fmax(z, 0.0);
            if (fabs(z) <= kKinkTol) atomicOr(nondiff, 1);
        }
    }
}

// second-order cone {(t, u) : ||u|| <= t}; cases tested in the order of the appendix.
__global__ void k_soc_factors(const double *zy, const int *soc_row, const int *soc_dim, int n_soc,
                              double *par, double *jdiag, int *nondiff, double *proj) {
    const int cone = blockIdx.x * blockDim.x + threadIdx.x;
    if (cone >= n_soc) return;
    const int r0 = soc_row[cone], k = soc_dim[cone];
    const double t = zy[r0];
    double nu2 = 0.0, amax = fabs(t);
    for (int i = 1; i < k; ++i) {
        nu2 += zy[r0 + i] * zy[r0 + i];
        amax = fmax(amax, fabs(zy[r0 + i]));
    }
    const double nu = sqrt(nu2);
    double *pp = par + 4 * cone;
    if (fabs(nu - fabs(t)) <= kKinkTol * fmax(1.0, amax) || (k == 1 && fabs(t) <= kKinkTol))
        atomicOr(nondiff, 1);
    if (nu <= -t) {
        pp[0] = 0.0; pp[1] = 0.0; pp[2] = 0.0; pp[3] = 0.0;
        for (int i = 0; i < k; ++i) jdiag[r0 + i] = 0.0;
        if (proj)
            for (int i = 0; i < k; ++i) proj[r0 + i] = 0.0;
    } else if (nu <= t) {
        pp[0] = 1.0; pp[1] = 0.0; pp[2] = 0.0; pp[3] = 0.0;
        for (int i = 0; i < k; ++i) jdiag[r0 + i] = 1.0;
        if (proj)
            for (int i = 0; i < k; ++i) proj[r0 + i] = zy[r0 + i];
    } else {
        const double inv = 1.0 / nu;
        const double c1 = 0.5 * (t + nu) * inv, c2 = 0.5 * t * inv;
        pp[0] = 2.0; pp[1] = inv; pp[2] = c1; pp[3] = c2;
        jdiag[r0] = 0.5;
        for (int i = 1; i < k; ++i) {
            const double uh = zy[r0 + i] * inv;
            jdiag[r0 + i] = c1 - c2 * uh * uh;
        }
        if (proj) {  // (t + |u|)/2 (1, u/|u|)
            const double h = 0.5 * (t + nu);
            proj[r0] = h;
            for (int i = 1; i < k; ++i) proj[r0 + i] = h * zy[r0 + i] * inv;
        }
    }
}

// exponential cone K_exp = cl{(x,y,z): y e^{x/y} <= z, y > 0}.
__device__ inline bool exp_member(double x, double y, double z) {
    if (y > 0.0) return y * exp(x / y) <= z;
    return y == 0.0 && x <= 0.0 && z >= 0.0;
}
__device__ inline bool exp_dual_member(double u, double v, double w) {
    if (u < 0.0) return -u * exp(v / u) <= M_E * w;
    return u == 0.0 && v >= 0.0 && w >= 0.0;
}

// The smooth-boundary case: hat p = yh (r, 1, e^r) and p - hat p = mu (e^r, (1-r)e^r, -1)
// are orthogonal, so p lies in their span exactly when
//   h(r) = <p, (r,1,e^r) x (e^r,(1-r)e^r,-1)>
//        = x0 (-1 - (1-r)e^{2r}) + y0 (e^{2r} + r) + z0 e^r (r - r^2 - 1)
// vanishes; the projection is the root at which h crosses from below with yh, mu > 0.
__device__ inline double exp_h(double x0, double y0, double z0, double r, bool scaled) {
    const double E = exp(r), E2 = E * E;
    double h = x0 * (-1.0 - (1.0 - r) * E2) + y0 * (E2 + r) + z0 * E * (r - r * r - 1.0);
    return scaled ? h / (1.0 + E2) : h;
}
__device__ inline double exp_dh(double x0, double y0, double z0, double r) {
    const double E = exp(r), E2 = E * E;
    return x0 * E2 * (2.0 * r - 1.0) + y0 * (2.0 * E2 + 1.0) - z0 * E * r * (r + 1.0);
}

__device__ bool exp_root(double x0, double y0, double z0, double &r_out) {
    // scan for an upward sign change of h with positive coefficients, then safeguarded
    // Newton inside the bracket
    double best_a = 0.0, best_b = 0.0, best_g = -1.0;
    bool found = false;
    for (int pass = 0; pass < 2 && !found; ++pass) {
        const double lo = pass == 0 ? -30.0 : -300.0, hi = pass == 0 ? 30.0 : 300.0;
        const double step = pass == 0 ? 0.0625 : 0.5;
        double ra = lo, ha = exp_h(x0, y0, z0, ra, true);
        for (double rb = lo + step; rb <= hi + 1e-12; rb += step) {
            const double hb = exp_h(x0, y0, z0, rb, true);
            if (ha < 0.0 && hb >= 0.0) {
                const double rm = 0.5 * (ra + rb), E = exp(rm);
                const double n1 = sqrt(rm * rm + 1.0 + E * E);
                const double gval = (x0 * rm + y0 + z0 * E) / n1;  // <p, d1>/||d1||
                if (gval > best_g) { best_g = gval; best_a = ra; best_b = rb; found = true; }
            }
            ra = rb;
            ha = hb;
        }
    }
    if (!found || !(best_g > 0.0)) return false;
    double a = best_a, b = best_b, r = 0.5 * (a + b);
    for (int it = 0; it < 200; ++it) {
        const double h = exp_h(x0, y0, z0, r, false);
        if (h == 0.0) break;
        if (h < 0.0) a = r; else b = r;
        const double dh = exp_dh(x0, y0, z0, r);
        double rn = (dh != 0.0) ? r - h / dh : 0.5 * (a + b);
        if (!(rn > a && rn < b)) rn = 0.5 * (a + b);
        if (fabs(rn - r) <= 1e-16 * fmax(1.0, fabs(r)) || b - a <= 4e-16 * fmax(1.0, fabs(r))) {
            r = rn;
            break;
        }
        r = rn;
    }
    r_out = r;
    return true;
}

// J of the dual exponential cone: DPi_{exp*}(z) = I - DPi_exp(-z) (App. A, Moreau).
// In the smooth case DPi_exp is the leading 3x3 block of the inverse of the bordered
// matrix [[H, g], [g', 0]] with H = I + mu Hess(y e^{x/y}) and g = grad(y e^{x/y} - z),
// evaluated as H^-1 - (H^-1 g)(H^-1 g)'/(g' H^-1 g).
__global__ void k_exp_factors(const double *zy, int row0, const int *rows, int n_exp, double *Jout,
                              double *jdiag, int *nondiff, int *fail, double *proj) {
    const int cone = blockIdx.x * blockDim.x + threadIdx.x;
    if (cone >= n_exp) return;
    const int r0 = rows ? rows[cone] : row0 + 3 * cone;
    const double x0 = -zy[r0], y0 = -zy[r0 + 1], z0 = -zy[r0 + 2];  // p = -z
    const double scale = fmax(1.0, fmax(fabs(x0), fmax(fabs(y0), fabs(z0))));
    const double tol = kKinkTol * scale;
    double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // DPi_exp(p)
    double ph[3] = {0.0, 0.0, 0.0};              // Pi_exp(p)
    if (exp_member(x0, y0, z0)) {
        D[0] = D[4] = D[8] = 1.0;
        ph[0] = x0; ph[1] = y0; ph[2] = z0;
        if (y0 <= tol || z0 - y0 * exp(x0 / y0) <= tol) atomicOr(nondiff, 1);
    } else if (exp_dual_member(-x0, -y0, -z0)) {
        const double u = -x0, v = -y0, w = -z0;
        if (u >= -tol || M_E * w + u * exp(v / u) <= tol) atomicOr(nondiff, 1);
    } else if (x0 < 0.0 && y0 < 0.0) {
        D[0] = 1.0;
        D[8] = z0 > 0.0 ? 1.0 : 0.0;
        ph[0] = x0; ph[2] = fmax(z0, 0.0);
        if (fabs(z0) <= tol || x0 >= -tol || y0 >= -tol) atomicOr(nondiff, 1);
    } else {
        double r;
        if (!exp_root(x0, y0, z0, r)) {
            atomicOr(fail, 1);
            return;
        }
        const double E = exp(r);
        const double yh = (x0 * r + y0 + z0 * E) / (r * r + 1.0 + E * E);
        ph[0] = yh * r; ph[1] = yh; ph[2] = yh * E;
        const double g0 = E, g1 = (1.0 - r) * E, g2 = -1.0;
        const double mu = (x0 * g0 + y0 * g1 + z0 * g2) / (g0 * g0 + g1 * g1 + g2 * g2);
        if (yh <= tol || mu <= tol) atomicOr(nondiff, 1);
        const double kap = mu * E / yh;
        const double det = 1.0 + kap + kap * r * r;
        // H^-1: 2x2 block for (x, y) and 1 for z
        const double h00 = (1.0 + kap * r * r) / det, h01 = kap * r / det, h11 = (1.0 + kap) / det;
        const double q0 = h00 * g0 + h01 * g1, q1 = h01 * g0 + h11 * g1, q2 = g2;
        const double gam = g0 * q0 + g1 * q1 + g2 * q2;
        const double Hi[9] = {h00, h01, 0.0, h01, h11, 0.0, 0.0, 0.0, 1.0};
        const double qv[3] = {q0, q1, q2};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) D[3 * i + j] = Hi[3 * i + j] - qv[i] * qv[j] / gam;
    }
    double *J = Jout + 9 * cone;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[3 * i + j] = (i == j ? 1.0 : 0.0) - D[3 * i + j];
    if (proj)  // Moreau: Pi_{exp*}(z) = z + Pi_exp(-z)
        for (int i = 0; i < 3; ++i) proj[r0 + i] = zy[r0 + i] + ph[i];
    jdiag[r0] = J[0];
    jdiag[r0 + 1] = J[4];
    jdiag[r0 + 2] = J[8];
}

// Power cone K_pow,a = {(x,y,z): x^a y^(1-a) >= |z|, x, y >= 0} (App. A, "Power cone").
__device__ inline bool pow_member(double x, double y, double z, double a) {
    return x >= 0.0 && y >= 0.0 && pow(x, a) * pow(y, 1.0 - a) >= fabs(z);
}
// K_pow,a* = {(u,v,w): (u/a)^a (v/(1-a))^(1-a) >= |w|, u, v >= 0}
__device__ inline bool pow_dual_member(double u, double v, double w, double a) {
    return u >= 0.0 && v >= 0.0 && pow(u / a, a) * pow(v / (1.0 - a), 1.0 - a) >= fabs(w);
}
// (x + sqrt(x^2 + t)) / 2, t >= 0, without cancellation for x < 0
__device__ inline double half_root(double x, double t) {
    const double s = sqrt(x * x + t);
    return x >= 0.0 ? 0.5 * (x + s) : 0.5 * t / (s - x);
}

// DPi_pow,a(x, y, z) into D (row-major), by the appendix's cases in their order: the cone's
// interior, the polar cone's, the plane z = 0, and otherwise the closed form around the
// root r in (0, |z|) of r = f_x(r)^a f_y(r)^(1-a), found by bisection until the bracket stops
// shrinking (the root is unique; the function is positive just above 0 and negative at |z|).
__device__ void pow_jacobian(double x, double y, double z, double a, double tol, double D[9],
                             int *nondiff, double ph[3]) {
    for (int i = 0; i < 9; ++i) D[i] = 0.0;
    ph[0] = ph[1] = ph[2] = 0.0;  // Pi_pow,a(x, y, z)
    const double az = fabs(z);
    if (pow_member(x, y, z, a)) {
        D[0] = D[4] = D[8] = 1.0;
        ph[0] = x; ph[1] = y; ph[2] = z;
        if (x <= tol || y <= tol || pow(x, a) * pow(y, 1.0 - a) - az <= tol) atomicOr(nondiff, 1);
        return;
    }
    if (pow_dual_member(-x, -y, -z, a)) {
        if (-x <= tol || -y <= tol ||
            pow(-x / a, a) * pow(-y / (1.0 - a), 1.0 - a) - az <= tol)
            atomicOr(nondiff, 1);
        return;
    }
    if (z == 0.0) {
        double d = 0.0;
        if (x > 0.0 && y < 0.0) d = a > 0.5 ? 1.0 : a < 0.5 ? 0.0 : x / (2.0 * fabs(y) + x);
        else if (x < 0.0 && y > 0.0) d = a < 0.5 ? 1.0 : a > 0.5 ? 0.0 : y / (2.0 * fabs(x) + y);
        D[0] = x > 0.0 ? 1.0 : 0.0;
        D[4] = y > 0.0 ? 1.0 : 0.0;
        D[8] = d;
        ph[0] = fmax(x, 0.0); ph[1] = fmax(y, 0.0);
        if (fabs(x) <= tol || fabs(y) <= tol) atomicOr(nondiff, 1);
        return;
    }
    double lo = 0.0, hi = az;
    for (int it = 0; it < 2000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        const double t = mid * (az - mid);
        const double h = pow(half_root(x, 4.0 * a * t), a) *
                         pow(half_root(y, 4.0 * (1.0 - a) * t), 1.0 - a) - mid;
        if (h > 0.0) lo = mid; else hi = mid;
    }
    const double r = 0.5 * (lo + hi);
    const double t = r * (az - r);
    const double fx = half_root(x, 4.0 * a * t), fy = half_root(y, 4.0 * (1.0 - a) * t);
    const double gx = 2.0 * fx - x, gy = 2.0 * fy - y;
    const double S = a * x / gx + (1.0 - a) * y / gy;
    const double L = 2.0 * (az - r) / (az + (az - 2.0 * r) * S);
    const double sz = z > 0.0 ? 1.0 : -1.0;
    ph[0] = fx; ph[1] = fy; ph[2] = sz * r;
    const double m = (az - 2.0 * r) * r * L;
    D[0] = 0.5 + x / (2.0 * gx) + a * a * m / (gx * gx);
    D[1] = D[3] = (a - a * a) * m / (gx * gy);
    D[2] = D[6] = sz * a * r * L / gx;
    D[4] = 0.5 + y / (2.0 * gy) + (1.0 - a) * (1.0 - a) * m / (gy * gy);
    D[5] = D[7] = sz * (1.0 - a) * r * L / gy;
    D[8] = r / az - (r / az) * S * L;
    if (r <= tol || az - r <= tol) atomicOr(nondiff, 1);
}

// J of the power-cone blocks: par[i] > 0 is alpha of a power cone, whose dual cone is
// projected by Moreau, J = I - DPi_pow(-z); par[i] < 0 is -alpha of a dual power cone, whose
// dual cone is K_pow itself, J = DPi_pow(z). Cone i occupies rows row0 + 3 i ..; its J is the
// 3 x 3 row-major matrix at Jout + 9 i.
__global__ void k_pow_factors(const double *zy, int row0, int count, const double *par,
                              double *Jout, double *jdiag, int *nondiff, double *proj) {
    const int cone = blockIdx.x * blockDim.x + threadIdx.x;
    if (cone >= count) return;
    const int r0 = row0 + 3 * cone;
    const double a = fabs(par[cone]);
    const bool dual = par[cone] < 0.0;
    const double sg = dual ? 1.0 : -1.0;
    const double x0 = sg * zy[r0], y0 = sg * zy[r0 + 1], z0 = sg * zy[r0 + 2];
    const double scale = fmax(1.0, fmax(fabs(x0), fmax(fabs(y0), fabs(z0))));
    double D[9], ph[3];
    pow_jacobian(x0, y0, z0, a, kKinkTol * scale, D, nondiff, ph);
    double *J = Jout + 9 * cone;
    for (int i = 0; i < 9; ++i) J[i] = dual ? D[i] : ((i % 4 == 0) ? 1.0 : 0.0) - D[i];
    if (proj)  // dual power cone: Pi_pow(z); power cone: z + Pi_pow(-z) (Moreau)
        for (int i = 0; i < 3; ++i) proj[r0 + i] = dual ? ph[i] : zy[r0 + i] + ph[i];
    jdiag[r0] = J[0];
    jdiag[r0 + 1] = J[4];
    jdiag[r0 + 2] = J[8];
}

// PSD cone: eigendecomposition of each k x k block by cyclic Jacobi with a round-robin
// (tournament) ordering, so k/2 disjoint rotations are applied at once; then
//   B_ij = 1 (both eigenvalues >= 0), 0 (both < 0), (l_i+ - l_j+)/(l_i - l_j) (mixed),
// which equals the appendix's B for any eigenvalue order. V (row-major, columns are
// eigenvectors) and B are stored side by side in the pool, with the eigenpairs of the
// smaller side of the split first: those with eigenvalue >= 0 when they are at most half,
// else those < 0. psd_lr (when given) records c, the size of that side, plus 256 when it is
// the negative side (the low-rank form of the Jacobian in the loop kernels reads it).
__global__ __launch_bounds__(kBlock) void k_psd_factors(const double *zy, const int *psd_row,
                                                        const int *psd_k, const long long *psd_off,
                                                        double *pool, double *jdiag,
                                                        int *nondiff, int *fail, int *psd_lr,
                                                        double *proj) {
    extern __shared__ double sm[];
    const int cone = blockIdx.x;
    const int k = psd_k[cone], r0 = psd_row[cone];
    const int ld = k | 1;
    const int kp = k + (k & 1);  // even number of players, the extra one idles
    double *A = sm, *V = sm + k * ld;
    double *rot = V + k * ld;    // (c, s) per pair
    int *pq = reinterpret_cast<int *>(rot + kp);
    __shared__ double lam_s[kMaxPsd];
    const int tid = threadIdx.x;
    const double rs2 = 0.70710678118654752440;
    for (int e = tid; e < k * k; e += kBlock) {
        const int i = e / k, j = e % k;
        V[i * ld + j] = (i == j) ? 1.0 : 0.0;
        if (i >= j) {
            const int t = j * k - (j * (j - 1)) / 2 + (i - j);
            double v = zy[r0 + t];
            if (i != j) v *= rs2;
            A[i * ld + j] = v;
            A[j * ld + i] = v;
        }
    }
    __syncthreads();
    const int npair = kp / 2;
    // Sweeps stop once the off-diagonal mass is at rounding level (||off||_F <= 1e-15
    // ||A||_F), or once it stops shrinking after reaching 1e-10 ||A||_F; the factorisation
    // is reported as failed only if it never got below 1e-10 ||A||_F.
    bool converged = false;
    double off_prev = -1.0, off_last = 0.0, all_last = 0.0;
    for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
        for (int round = 0; round < kp - 1; ++round) {
            if (tid < npair) {
                auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (kp - 1)) + 1; };
                int p = player(tid), q = player(kp - 1 - tid);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < k) {
                    const double apq = A[p * ld + q];
                    if (apq != 0.0) {
                        const double app = A[p * ld + p], aqq = A[q * ld + q];
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                rot[2 * tid] = c;
                rot[2 * tid + 1] = s;
                pq[2 * tid] = p;
                pq[2 * tid + 1] = q;
            }
            __syncthreads();
            // A <- J' A (rows p, q of every pair)
            for (int e = tid; e < npair * k; e += kBlock) {
                const int pr = e / k, j = e % k;
                const int p = pq[2 * pr], q = pq[2 * pr + 1];
                if (q < k) {
                    const double c = rot[2 * pr], s = rot[2 * pr + 1];
                    const double ap = A[p * ld + j], aq = A[q * ld + j];
                    A[p * ld + j] = c * ap - s * aq;
                    A[q * ld + j] = s * ap + c * aq;
                }
            }
            __syncthreads();
            // A <- A J and V <- V J (columns p, q of every pair)
            for (int e = tid; e < npair * k; e += kBlock) {
                const int pr = e / k, i = e % k;
                const int p = pq[2 * pr], q = pq[2 * pr + 1];
                if (q < k) {
                    const double c = rot[2 * pr], s = rot[2 * pr + 1];
                    const double ap = A[i * ld + p], aq = A[i * ld + q];
                    A[i * ld + p] = c * ap - s * aq;
                    A[i * ld + q] = s * ap + c * aq;
                    const double vp = V[i * ld + p], vq = V[i * ld + q];
                    V[i * ld + p] = c * vp - s * vq;
                    V[i * ld + q] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
        double off = 0.0, all = 0.0, z3 = 0.0;
        for (int e = tid; e < k * k; e += kBlock) {
            const int i = e / k, j = e % k;
            const double v = A[i * ld + j];
            all += v * v;
            if (i != j) off += v * v;
        }
        block_sum3(off, all, z3);
        __shared__ int conv_s;
        __shared__ double off_s, all_s;
        if (tid == 0) {
            conv_s = (off <= 1e-30 * all) || off == 0.0 ||
                     (off_prev >= 0.0 && off >= off_prev && off <= 1e-20 * all);
            off_s = off;
            all_s = all;
        }
        __syncthreads();
        converged = conv_s != 0;
        off_last = off_s;
        all_last = all_s;
        off_prev = off_last;
        __syncthreads();
    }
    if (tid == 0 && !(off_last <= 1e-20 * all_last)) atomicOr(fail, 2);
    for (int i = tid; i < k; i += kBlock) lam_s[i] = A[i * ld + i];
    __syncthreads();
    __shared__ int perm_s[kMaxPsd];  // stored position -> eigenpair
    if (tid == 0) {
        int r = 0;
        for (int i = 0; i < k; ++i) r += lam_s[i] >= 0.0;
        const bool neg = r > k - r;
        const int c = neg ? k - r : r;
        int a = 0, b = c;
        for (int i = 0; i < k; ++i) {
            const bool side = neg ? lam_s[i] < 0.0 : lam_s[i] >= 0.0;
            perm_s[side ? a++ : b++] = i;
        }
        if (psd_lr) psd_lr[cone] = c | (neg ? 256 : 0);
    }
    __syncthreads();
    double *Vg = pool + psd_off[cone];
    double *Bg = Vg + k * k;
    double lmax = 0.0;
    for (int i = 0; i < k; ++i) lmax = fmax(lmax, fabs(lam_s[i]));
    if (tid == 0) {
        for (int i = 0; i < k; ++i)
            if (fabs(lam_s[i]) <= kKinkTol * fmax(1.0, lmax)) atomicOr(nondiff, 1);
    }
    auto bfun = [](double li, double lj) {
        if (li >= 0.0 && lj >= 0.0) return 1.0;
        if (li < 0.0 && lj < 0.0) return 0.0;
        return (fmax(li, 0.0) - fmax(lj, 0.0)) / (li - lj);
    };
    for (int e = tid; e < k * k; e += kBlock) {
        const int i = e / k, j = e % k;
        Vg[e] = V[i * ld + perm_s[j]];
        Bg[e] = bfun(lam_s[perm_s[i]], lam_s[perm_s[j]]);
        A[i * ld + j] = bfun(lam_s[i], lam_s[j]);  // B in eigenpair order, for the diagonal below
    }
    __syncthreads();
    // diag of J on svec coordinates: entry (i,i): sum_ab B_ab V_ia^2 V_ib^2;
    // entry (i,j), i > j: sum_ab B_ab (V_ia^2 V_jb^2 + V_ia V_ib V_ja V_jb)
    const int nr = k * (k + 1) / 2;
    for (int e = tid; e < k * k; e += kBlock) {
        const int i = e / k, j = e % k;
        if (i < j) continue;
        double acc = 0.0;
        for (int a = 0; a < k; ++a) {
            const double via = V[i * ld + a], vja = V[j * ld + a];
            for (int b2 = 0; b2 < k; ++b2) {
                const double vib = V[i * ld + b2], vjb = V[j * ld + b2];
                const double bab = A[a * ld + b2];
                acc += (i == j) ? bab * via * via * vib * vib
                                : bab * (via * via * vjb * vjb + via * vib * vja * vjb);
            }
        }
        const int t = j * k - (j * (j - 1)) / 2 + (i - j);
        jdiag[r0 + t] = acc;
    }
    (void)nr;
    if (proj) {  // Pi = V diag(max(lambda, 0)) V' in svec (off-diagonals times sqrt 2)
        for (int e = tid; e < k * k; e += kBlock) {
            const int i = e / k, j = e % k;
            if (i < j) continue;
            double acc = 0.0;
            for (int a = 0; a < k; ++a) acc += V[i * ld + a] * fmax(lam_s[a], 0.0) * V[j * ld + a];
            const int t = j * k - (j * (j - 1)) / 2 + (i - j);
            proj[r0 + t] = i == j ? acc : acc * 1.41421356237309504880;
        }
    }
}

// ---------------------------------------------------------------------------------------
// Jacobi scales: d_jvp = 1/column norms of F, d_vjp = 1/row norms of F, with each cone
// block's J replaced by its diagonal (exact for x, tau, zero and nonnegative columns).
//   col x_j: ||P_:j||^2 + ||A_:j||^2 + c_j^2          row x_i: ||P_i:||^2 + sum_k A_ki^2 J_kk^2 + q_i^2
//   col y_j: J_jj^2 (||A_j:||^2 + b_j^2) + (1-J_jj)^2   row y_i: ||A_i:||^2 + (1-J_ii)^2 + b_i^2
//   col tau: ||q||^2 + ||b||^2 + (x'Px)^2             row tau: ||c||^2 + sum_k b_k^2 J_kk^2 + (x'Px)^2
// ---------------------------------------------------------------------------------------

__device__ inline double inv_norm(double s2) { return s2 > 0.0 ? 1.0 / sqrt(s2) : 1.0; }

__global__ __launch_bounds__(kBlock) void k_scales(Problem p, RowGrid g, double *dj, double *dv,
                                                   double *partials, int *counter, int do_tau) {
    const int tid = threadIdx.x;
    const bool xr = blockIdx.x < (unsigned)g.bx;
    const int L = xr ? g.lx : g.ly;
    const long long gt = (long long)(xr ? blockIdx.x : blockIdx.x - g.bx) * kBlock + tid;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (xr && row < p.n) {
        for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) a0 += p.Pv[k] * p.Pv[k];
        for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L) {
            const double v2 = p.Tv[t] * p.Tv[t], jd = p.jdiag[p.Tci[t]];
            a1 += v2;
            a2 += v2 * jd * jd;
        }
    } else if (!xr && row < p.m) {
        for (int k = p.Arp[row] + lane; k < p.Arp[row + 1]; k += L) a0 += p.Av[k] * p.Av[k];
    }
    for (int off = L >> 1; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off);
        a1 += __shfl_xor(a1, off);
        a2 += __shfl_xor(a2, off);
    }
    double s0 = 0.0, s1 = 0.0;
    if (lane == 0) {
        if (xr && row < p.n) {
            const double c = p.c[row], q = p.q[row];
            dj[row] = inv_norm(a0 + a1 + c * c);
            dv[row] = inv_norm(a0 + a2 + q * q);
            s0 = q * q;
            s1 = c * c;
        } else if (!xr && row < p.m) {
            const double jd = p.jdiag[row], b = p.b[row];
            dj[p.n + row] = inv_norm(jd * jd * (a0 + b * b) + (1.0 - jd) * (1.0 - jd));
            dv[p.n + row] = inv_norm(a0 + (1.0 - jd) * (1.0 - jd) + b * b);
            s0 = b * b;
            s1 = b * b * jd * jd;
        }
    }
    double tot[3];
    if (last_block_sum3(s0, s1, 0.0, partials, counter, gridDim.x, tot) && tid == 0 && do_tau) {
        const double x2 = p.xPx * p.xPx;
        dj[p.N - 1] = inv_norm(tot[0] + x2);
        dv[p.N - 1] = inv_norm(tot[1] + x2);
    }
}

// ---------------------------------------------------------------------------------------
// Two-sided equilibration of F-hat (F with each cone block's J replaced by its diagonal):
// one sweep divides every row and every column of M = DL F-hat DR by the square root of its
// 2-norm, DL_i /= sqrt(||M_i.||), DR_j /= sqrt(||M_.j||), both from the same M. Entries:
//   x row i:  P_i., (A'_i. J), q_i      y row r:  -A_r., (1 - J_rr) at (r, r), b_r
//   tau row:  c', -(b o J)', x'Px
// Repeated sweeps balance row and column norms (the LSQR systems are consistent, so a row
// scaling leaves their solutions unchanged).
// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_equil_sweep(Problem p, RowGrid g, const double *DL,
                                                        const double *DR, double *DLo, double *DRo,
                                                        double *partials, int *counter) {
    const int tid = threadIdx.x, n = p.n, N = p.N;
    const bool xr = blockIdx.x < (unsigned)g.bx;
    const int L = xr ? g.lx : g.ly;
    const long long gt = (long long)(xr ? blockIdx.x : blockIdx.x - g.bx) * kBlock + tid;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    const double dlN = DL[N - 1], drN = DR[N - 1];
    double rs = 0.0, cs = 0.0;
    if (xr && row < n) {
        for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) {
            const double v2 = p.Pv[k] * p.Pv[k];
            const int j = p.Pci[k];
            rs += v2 * DR[j] * DR[j];
            cs += v2 * DL[j] * DL[j];  // P symmetric: column i = row i
        }
        for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L) {
            const int r = p.Tci[t];
            const double v2 = p.Tv[t] * p.Tv[t], jd = p.jdiag[r];
            rs += v2 * jd * jd * DR[n + r] * DR[n + r];
            cs += v2 * DL[n + r] * DL[n + r];
        }
    } else if (!xr && row < p.m) {
        for (int k = p.Arp[row] + lane; k < p.Arp[row + 1]; k += L) {
            const double v2 = p.Av[k] * p.Av[k];
            const int j = p.Aci[k];
            rs += v2 * DR[j] * DR[j];
            cs += v2 * DL[j] * DL[j];
        }
    }
    for (int off = L >> 1; off > 0; off >>= 1) {
        rs += __shfl_xor(rs, off);
        cs += __shfl_xor(cs, off);
    }
    double s0 = 0.0, s1 = 0.0;
    auto upd = [&](int i, double rsum, double csum) {
        const double rn = DL[i] * sqrt(rsum), cn = DR[i] * sqrt(csum);
        DLo[i] = rn > 0.0 ? DL[i] / sqrt(rn) : DL[i];
        DRo[i] = cn > 0.0 ? DR[i] / sqrt(cn) : DR[i];
    };
    if (lane == 0) {
        if (xr && row < n) {
            const double q = p.q[row], c = p.c[row];
            upd(row, rs + q * q * drN * drN, cs + c * c * dlN * dlN);
            s0 = c * c * DR[row] * DR[row];  // tau row
            s1 = q * q * DL[row] * DL[row];  // tau column
        } else if (!xr && row < p.m) {
            const int i = n + row;
            const double jd = p.jdiag[row], b = p.b[row], o = 1.0 - jd;
            upd(i, rs + o * o * DR[i] * DR[i] + b * b * drN * drN,
                jd * jd * cs + o * o * DL[i] * DL[i] + b * b * jd * jd * dlN * dlN);
            s0 = b * b * jd * jd * DR[i] * DR[i];
            s1 = b * b * DL[i] * DL[i];
        }
    }
    double tot[3];
    if (last_block_sum3(s0, s1, 0.0, partials, counter, gridDim.x, tot) && tid == 0) {
        const double x2 = p.xPx * p.xPx;
        upd(N - 1, tot[0] + x2 * drN * drN, tot[1] + x2 * dlN * dlN);
    }
}

void launch_equilibrate(const Problem &p, const RowGrid &g, double *DL, double *DR, double *tmpL,
                        double *tmpR, int sweeps, double *partials, int *counter, hipStream_t s) {
    // starts from DL = DR = 1 (filled by the caller); an even number of sweeps ends in DL, DR
    for (int k = 0; k < sweeps; ++k) {
        const bool even = (k % 2) == 0;
        hipLaunchKernelGGL(k_equil_sweep, dim3(g.total()), dim3(kBlock), 0, s, p, g,
                           even ? DL : tmpL, even ? DR : tmpR, even ? tmpL : DL, even ? tmpR : DR,
                           partials, counter);
    }
}

// ---------------------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------------------

void launch_check_csr(const int *rp, const int *ci, int nrows, int ncols, int nnz, int *flag,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_check_csr, dim3(div_up(std::max(nrows, 1), 256)), dim3(256), 0, s, rp, ci,
                       nrows, ncols, nnz, flag);
}
void launch_check_sorted(const int *rp, const int *ci, int nrows, int ncols, int *flag, hipStream_t s) {
    if (nrows > 0)
        hipLaunchKernelGGL(k_check_sorted, dim3(div_up(nrows, 256)), dim3(256), 0, s, rp, ci, nrows, ncols, flag);
}
void launch_check_symmetric(const int *rp, const int *ci, const double *v, const int *trp,
                            const int *tci, const double *tv, int n, int nnz, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_symmetric, dim3(div_up(std::max(n + 1, nnz), 256)), dim3(256), 0, s,
                       rp, ci, v, trp, tci, tv, n, nnz, flag);
}
void launch_px(const Problem &p, const RowGrid &g, double *c, double *xpx, double *partials,
               int *counter, hipStream_t s) {
    hipLaunchKernelGGL(k_px, dim3(std::max(g.bx, 1)), dim3(kBlock), 0, s, p, g, c, xpx, partials, counter);
}
// ---------------------------------------------------------------------------------------
// Solution refinement (the forward re-solve): the KKT map of the QCP at a point (x, eta),
// with y = Pi_{K*}(eta) and s = y - eta (Moreau: y and s in K* and K, orthogonal),
//   G(x, eta) = (P x + A' y + q, -A x + b - y + eta),
// zero exactly at a primal-dual solution (Sec. 2.1 optimality conditions). One thread per
// row of the n + m rows, the stored CSR copies of P, A and A'.
// ---------------------------------------------------------------------------------------

__global__ void k_kkt_map(Problem p, const double *x, const double *y, const double *eta,
                          double *g) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = p.n, m = p.m;
    if (i < n) {
        double acc = p.q[i];
        for (int k = p.Prp[i]; k < p.Prp[i + 1]; ++k) acc += p.Pv[k] * x[p.Pci[k]];
        for (int k = p.Trp[i]; k < p.Trp[i + 1]; ++k) acc += p.Tv[k] * y[p.Tci[k]];
        g[i] = acc;
    } else if (i < (long long)n + m) {
        const int r = (int)(i - n);
        double acc = 0.0;
        for (int k = p.Arp[r]; k < p.Arp[r + 1]; ++k) acc += p.Av[k] * x[p.Aci[k]];
        g[i] = -acc + p.b[r] - y[r] + eta[r];
    }
}

// x += dx, eta += dy - ds: the Newton step of the refinement from a derivative's outputs
__global__ void k_newton_update(double *x, double *eta, const double *dx, const double *dy,
                                const double *ds, int n, int m) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += dx[i];
    else if (i < (long long)n + m) eta[i - n] += dy[i - n] - ds[i - n];
}

// sum of squares: per-workgroup partial sums, then one workgroup adds them in a fixed order
__global__ __launch_bounds__(kBlock) void k_sumsq_part(const double *v, long long n, double *part) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        a += v[i] * v[i];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}
__global__ __launch_bounds__(kBlock) void k_sum_final(const double *part, int np, double *out) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) a += part[i];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) out[0] = a;
}

void launch_kkt_map(const Problem &p, const double *x, const double *y, const double *eta,
                    double *g, hipStream_t s) {
    const long long rows = (long long)p.n + p.m;
    if (rows > 0)
        hipLaunchKernelGGL(k_kkt_map, dim3(div_up(rows, kBlock)), dim3(kBlock), 0, s, p, x, y, eta, g);
}
void launch_newton_update(double *x, double *eta, const double *dx, const double *dy,
                          const double *ds, int n, int m, hipStream_t s) {
    const long long rows = (long long)n + m;
    if (rows > 0)
        hipLaunchKernelGGL(k_newton_update, dim3(div_up(rows, kBlock)), dim3(kBlock), 0, s, x, eta,
                           dx, dy, ds, n, m);
}
void launch_sumsq(const double *v, long long n, double *part, double *out, hipStream_t s) {
    const int g = std::max(1, std::min(kSumsqParts, div_up(n, kBlock)));
    hipLaunchKernelGGL(k_sumsq_part, dim3(g), dim3(kBlock), 0, s, v, n, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, part, g, out);
}

void launch_sub(const double *a, const double *b, double *out, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_sub, dim3(div_up(n, 256)), dim3(256), 0, s, a, b, out, n);
}
void launch_cone_factors(const Problem &p, const ConeHost &ch, double *jdiag, double *soc_par,
                         double *exp_J, double *pool, int *nondiff, int *fail, int psd_lds,
                         hipStream_t s, double *proj) {
    if (p.n_diag > 0)
        hipLaunchKernelGGL(k_diag_factors, dim3(div_up(p.n_diag, 256)), dim3(256), 0, s, p.zy,
                           ch.n_zero, p.n_diag, jdiag, nondiff, proj);
    if (p.n_soc > 0)
        hipLaunchKernelGGL(k_soc_factors, dim3(div_up(p.n_soc, 128)), dim3(128), 0, s, p.zy,
                           p.soc_row, p.soc_dim, p.n_soc, soc_par, jdiag, nondiff, proj);
    if (ch.n_exp > 0)
        hipLaunchKernelGGL(k_exp_factors, dim3(div_up(ch.n_exp, 64)), dim3(64), 0, s, p.zy,
                           p.exp_row0, p.exp_rows, ch.n_exp, exp_J, jdiag, nondiff, fail, proj);
    if (ch.n_pow > 0)  // power cones follow the exponential cones (one contiguous row range)
        hipLaunchKernelGGL(k_pow_factors, dim3(div_up(ch.n_pow, 64)), dim3(64), 0, s, p.zy,
                           p.exp_row0 + 3 * ch.n_exp, ch.n_pow, ch.pow_par, exp_J + 9LL * ch.n_exp,
                           jdiag, nondiff, proj);
    if (p.n_psd > 0) {
        (void)hipFuncSetAttribute((const void *)k_psd_factors, hipFuncAttributeMaxDynamicSharedMemorySize, psd_lds);
        hipLaunchKernelGGL(k_psd_factors, dim3(p.n_psd), dim3(kBlock), psd_lds, s, p.zy, p.psd_row,
                           p.psd_k, p.psd_off, pool, jdiag, nondiff, fail, ch.psd_lr, proj);
    }
}
void launch_scales(const Problem &p, const RowGrid &g, double *dj, double *dv, double *partials,
                   int *counter, hipStream_t s, int do_tau) {
    hipLaunchKernelGGL(k_scales, dim3(g.total()), dim3(kBlock), 0, s, p, g, dj, dv, partials, counter,
                       do_tau);
}

int psd_factor_lds_bytes(int kmax) {
    if (kmax <= 0) return 0;
    const int ld = kmax | 1, kp = kmax + (kmax & 1);
    return (2 * kmax * ld + kp) * (int)sizeof(double) + kp * (int)sizeof(int) + 64;
}

}  // namespace qcpd
