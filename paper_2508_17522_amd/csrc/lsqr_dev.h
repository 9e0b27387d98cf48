// Device helpers of one LSQR product step, shared by the single-problem grid kernels and
// the batched (one workgroup per problem) kernel.
#pragma once

#include "cone_jv.h"
#include "qcpd_internal.h"

namespace qcpd {

// ---------------------------------------------------------------------------------------
// LSQR bookkeeping
// ---------------------------------------------------------------------------------------

// t0: the sum of squares of the launch's output; t1: the dot product it accumulated (or, for
// ROLE_RESID, the squared norm of the right-hand side)
__device__ inline void finalize(LsqrState *st, int role, double t0, double t1, bool dot_is_fwd) {
    switch (role) {
    case ROLE_U: {
        const double beta = sqrt(t0);
        st->beta = beta;
        st->pending = 0;
        if (dot_is_fwd) st->dot_fwd = t1; else st->dot_adj = t1;
        if (!(beta > 0.0)) { st->done = 1; st->conv = 1; }
        break;
    }
    case ROLE_V0: {
        const double alpha = sqrt(t0);
        st->alpha = alpha;
        st->rhobar = alpha;
        st->phibar = st->beta1;
        st->phr = 0.0;
        st->thr = 0.0;
        st->pending = 0;
        if (dot_is_fwd) st->dot_fwd = t1; else st->dot_adj = t1;
        if (!(alpha > 0.0)) { st->done = 1; st->conv = 1; }
        break;
    }
    case ROLE_V: {
        // plane rotation that eliminates beta (Paige & Saunders), then the x/w update is
        // owed to the next iteration's first kernel (or the final flush)
        // one thread evaluates this between two barriers of every launch, so the chain of
        // dependent FP64 operations is kept short: rho = sqrt(rhobar^2 + beta^2) (both are
        // norms of scaled vectors, far from overflow) and one reciprocal for the four
        // quotients by rho
        const double alpha = sqrt(t0);
        const double beta = st->beta, rhobar = st->rhobar;
        const double rho = sqrt(rhobar * rhobar + beta * beta);
        if (!(rho > 0.0)) { st->done = 1; st->conv = 1; st->pending = 0; break; }
        const double ri = 1.0 / rho;
        const double c = rhobar * ri, s = beta * ri;
        const double theta = s * alpha;
        const double phi = c * st->phibar;
        st->rhobar = -c * alpha;
        st->phibar = s * st->phibar;
        st->phr = phi * ri;
        st->thr = theta * ri;
        st->pending = 1;
        st->iters += 1;
        st->alpha = alpha;
        if (dot_is_fwd) st->dot_fwd = t1; else st->dot_adj = t1;
        if (st->phibar <= st->tol * st->beta1 || !(alpha > 0.0)) {
            st->done = 1;
            st->conv = 1;
        } else if (st->iters >= st->max_iter) {
            st->done = 1;
        }
        break;
    }
    case ROLE_RESID:
        st->resid = sqrt(t0);
        st->tau_rhs = sqrt(t1);  // ||rhs|| of the unscaled system
        break;
    default:
        if (dot_is_fwd) st->dot_fwd = t1; else st->dot_adj = t1;
        break;
    }
}

struct Ctx {  // per-launch scalars every thread derives from the state block
    double inv, cU, cV, inv_alpha_up, phr, thr, in_N;
    const double *isc;  // scale applied when reading the input (sc for v, scl for u)
    const double *osc;  // scale applied to the operator's output in the role update
    const double *nxs;  // scale the next product applies when it reads this output
};

// The LSQR matrix is M = L F R (JVP) or L F' R (VJP) with diagonal L = scl, R = sc. The
// v-side vectors are read through sc, the u-side vectors through scl; M v = L op(R v) and
// M'u = R op'(L u), so a u-step output is scaled by scl and a v-step output by sc.
__device__ inline Ctx make_ctx(const StepArgs &a, int tau_idx) {
    const LsqrState *st = a.st;
    const double *sv = reinterpret_cast<const double *>(st);
    Ctx c;
    c.inv = 1.0 / sv[a.in_nrm];
    c.cU = (a.role == ROLE_U) ? st->alpha / st->beta : 0.0;
    c.cV = (a.role == ROLE_V) ? st->beta / st->alpha : 0.0;
    c.inv_alpha_up = a.do_update ? 1.0 / st->alpha : 0.0;
    c.phr = st->phr;
    c.thr = st->thr;
    c.isc = a.in_is_v ? a.sc : a.scl;
    c.osc = (a.role == ROLE_U) ? a.scl : (a.role == ROLE_V || a.role == ROLE_V0) ? a.sc : nullptr;
    c.nxs = a.out_is_v ? a.sc : a.scl;
    c.in_N = a.in[tau_idx] * c.inv * (c.isc ? c.isc[tau_idx] : 1.0);
    return c;
}

__device__ inline double ldin(const StepArgs &a, const Ctx &c, int i) {
    const double v = a.in[i] * c.inv;
    return c.isc ? v * c.isc[i] : v;
}

__device__ inline double nscale(const Ctx &c, int idx) { return c.nxs ? c.nxs[idx] : 1.0; }

__device__ inline double role_value(const StepArgs &a, const Ctx &c, int idx, double val) {
    const double sv = c.osc ? c.osc[idx] * val : val;
    switch (a.role) {
    case ROLE_U: return sv - c.cU * a.out[idx];
    case ROLE_V: return sv - c.cV * a.out[idx];
    case ROLE_V0: return sv;
    case ROLE_RESID: return val - a.rhs[idx];
    default: return val;
    }
}

__device__ inline void lsqr_update(const StepArgs &a, const Ctx &c, int idx) {
    const double w = a.wk[idx];
    a.xk[idx] += c.phr * w;
    a.wk[idx] = a.in[idx] * c.inv_alpha_up - c.thr * w;
}

__device__ inline double group_sum(double v, int L) {
    for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}



// One work unit of the fused product with F' (see k_fused_FT), executed by the whole
// workgroup. Accumulates this thread's share of ||out||^2 (s0) and of the F tau-row dot
// for the next product (s1). The tau entry is handled by the caller.
__device__ inline void fused_unit(const Problem &p, const StepArgs &a, const Ctx &c, int lx,
                                  int ly, const Unit &u, double *sm, double &s0, double &s1) {
    const int n = p.n;
    const int tid = threadIdx.x;
    auto nsc = [&](int idx) { return nscale(c, idx); };
    auto finish = [&](int idx, double val) {
        const double o = role_value(a, c, idx, val);
        a.out[idx] = o;
        s0 += o * o;
        if (a.role == ROLE_RESID) s1 += a.rhs[idx] * a.rhs[idx];
        return o;
    };
    // t_r = A_r. r_x - b_r r_N - r_y for y rows [r0, r1), L lanes per row, into buf
    auto yrows = [&](int r0, int r1, double *buf) {
        const int L = ly, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = r0; rb < r1; rb += ngrp) {
            const int r = rb + grp;
            double acc = 0.0;
            if (r < r1)
                for (int k = p.Arp[r] + lane; k < p.Arp[r + 1]; k += L)
                    acc += p.Av[k] * ldin(a, c, p.Aci[k]);
            acc = group_sum(acc, L);
            if (r < r1 && lane == 0) buf[r - r0] = acc - p.b[r] * c.in_N - ldin(a, c, n + r);
        }
    };
    if (u.type == U_XROWS) {
        const int L = lx, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = u.begin; rb < u.end; rb += ngrp) {
            const int row = rb + grp;
            double acc = 0.0, accT = 0.0;
            if (row < u.end) {
                for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L)
                    acc += p.Pv[k] * ldin(a, c, p.Pci[k]);
                for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L)
                    accT += p.Tv[t] * ldin(a, c, n + p.Tci[t]);
            }
            acc = group_sum(acc, L);
            accT = group_sum(accT, L);
            if (row < u.end && lane == 0) {
                const double o = finish(row, acc - accT + p.c[row] * c.in_N);
                if (a.do_pre) s1 += p.c[row] * nsc(row) * o;
                if (a.do_update) lsqr_update(a, c, row);
            }
        }
    } else if (u.type == U_DIAG) {
        const int L = ly, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = u.begin; rb < u.end; rb += ngrp) {
            const int r = rb + grp;
            double acc = 0.0;
            if (r < u.end)
                for (int k = p.Arp[r] + lane; k < p.Arp[r + 1]; k += L)
                    acc += p.Av[k] * ldin(a, c, p.Aci[k]);
            acc = group_sum(acc, L);
            if (r < u.end && lane == 0) {
                const int idx = n + r;
                const double ry = ldin(a, c, idx);
                const double t = acc - p.b[r] * c.in_N - ry;
                const double o = finish(idx, p.jdiag[r] * t + ry);
                if (a.do_pre) {
                    const double w = p.jdiag[r] * nsc(idx) * o;
                    a.wy[r] = w;
                    s1 -= p.b[r] * w;
                }
                if (a.do_update) lsqr_update(a, c, idx);
            }
        }
    } else if (u.type == U_SOC || u.type == U_EXP) {
        double *tb = sm, *ob = sm + kUnitRows;
        const int r0 = u.row0;
        const int r1 = (u.type == U_SOC) ? p.soc_row[u.end - 1] + p.soc_dim[u.end - 1]
                                         : exp_row(p, u.end - 1) + 3;
        yrows(r0, r1, tb);
        __syncthreads();
        const int cone = u.begin + tid;
        if (cone < u.end) {
            auto tin = [&](int r) { return tb[r - r0]; };
            auto fout = [&](int r, double jt) {
                const double o = finish(n + r, jt + ldin(a, c, n + r));
                ob[r - r0] = nsc(n + r) * o;
                if (a.do_update) lsqr_update(a, c, n + r);
            };
            auto oin = [&](int r) { return ob[r - r0]; };
            auto wout = [&](int r, double w) { a.wy[r] = w; s1 -= p.b[r] * w; };
            if (u.type == U_SOC) {
                soc_jv(p, cone, tin, fout);
                if (a.do_pre) soc_jv(p, cone, oin, wout);
            } else {
                exp_jv(p, cone, tin, fout);
                if (a.do_pre) exp_jv(p, cone, oin, wout);
            }
        }
    } else {  // one PSD cone
        const int cone = u.begin;
        const int k = p.psd_k[cone], r0 = p.psd_row[cone], nr = k * (k + 1) / 2;
        double *tb = sm + psd_stage_offset(k), *ob = tb + nr;
        yrows(r0, r0 + nr, tb);
        __syncthreads();
        psd_jv(p, cone, sm, [&](int r) { return tb[r - r0]; },
               [&](int r, double jt) {
                   const double o = finish(n + r, jt + ldin(a, c, n + r));
                   ob[r - r0] = nsc(n + r) * o;
                   if (a.do_update) lsqr_update(a, c, n + r);
               });
        if (a.do_pre)
            psd_jv(p, cone, sm, [&](int r) { return ob[r - r0]; },
                   [&](int r, double w) { a.wy[r] = w; s1 -= p.b[r] * w; });
    }
}

}  // namespace qcpd
