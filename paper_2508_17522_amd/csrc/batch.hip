// Many QCPs of uneven sizes in one launch.
//
// Setup treats the batch as one block-diagonal problem (its CSR transpose, Px, cone factors
// and Jacobi scales are exactly those of the single-problem path), except for the per-problem
// tau entries (x'Px and the tau scales). The vectors of the batch are laid out as
//   [ x of every problem | y of every problem | tau of every problem ].
// A derivative evaluation runs in three phases. Begin and end are persistent kernels in which
// each workgroup takes whole problems from an atomic work queue (longest first): the begin
// kernel forms a problem's right-hand side and the first product of its bidiagonalisation,
// the end kernel applies the owed update, recomputes the explicit residual and forms the
// outputs. In between, the LSQR iterations of all problems advance together in the segmented
// loop kernels (loop.hip), two launches per iteration captured in HIP graphs, each work item
// within one problem and each problem with its own state and stopping test, so results match
// the single-problem path up to rounding.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "cone_jv.h"
#include "lsqr_dev.h"
#include "qcpd_internal.h"
#include "setup.h"

namespace qcpd {

struct BatchDev {
    Problem p;  // union of the problems; p.n = sum n, p.m = sum m, p.N = p.n + p.m + nprob
    int B;
    const int *n_off, *m_off, *u_off;  // nprob + 1 prefix offsets
    const int *lxs, *lys;              // lanes per CSR row, per problem
    const Unit *units;
    const double *xPx;
    const int *order;
    int *queue;
    double *u, *v, *xk, *wk, *rhs, *sol, *wy, *scratch;
    double *wy_res;    // J applied to the solution, for the explicit residual and outputs
    const double *sc;  // column (v-side) scale of the current direction, or null
    const double *scl; // row (u-side) scale of the current direction, or null
    int *resume;       // per problem: LSQR resumed after its explicit residual check
    int *nresumed;
    double *prev_rel;  // per problem: explicit relative residual before its last resume, or 0
    LsqrState *st_out;
    double tol;
    int max_iter;
};

struct BCtx {
    int b, n0, n1, m0, m1, tix, lx, ly, u0, u1;
    double xPx;
};

// ---------------------------------------------------------------------------------------
// block-level pieces of one problem's evaluation (all threads of the workgroup call them)
// ---------------------------------------------------------------------------------------

__device__ inline void blk_reduce_finalize(LsqrState *S, int role, double s0, double s1, double s2,
                                           bool dot_is_fwd) {
    block_sum3(s0, s1, s2);
    if (threadIdx.x == 0) {
        const double tot[3] = {s0, s1, s2};
        finalize(S, role, tot[0], tot[1], dot_is_fwd);
    }
    __syncthreads();
}

// product with F over the problem's rows (CSR rows of P and A' for x, of A for y, the tau row)
__device__ void blk_rows_F(const Problem &p, const StepArgs &a, const Ctx &c, const BCtx &bc,
                           double &s0, double &s1) {
    const int n = p.n, tid = threadIdx.x;
    {
        const int L = bc.lx, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = bc.n0; rb < bc.n1; rb += ngrp) {
            const int row = rb + grp;
            double acc = 0.0, accT = 0.0;
            if (row < bc.n1) {
                for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L)
                    acc += p.Pv[k] * ldin(a, c, p.Pci[k]);
                for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L)
                    accT += p.Tv[t] * a.wy[p.Tci[t]];
            }
            acc = group_sum(acc, L);
            accT = group_sum(accT, L);
            if (row < bc.n1 && lane == 0) {
                const double o = role_value(a, c, row, acc + accT * c.inv + p.q[row] * c.in_N);
                a.out[row] = o;
                s0 += o * o;
                s1 += (a.role == ROLE_RESID) ? a.rhs[row] * a.rhs[row] : p.q[row] * nscale(c, row) * o;
                if (a.do_update) lsqr_update(a, c, row);
            }
        }
    }
    {
        const int L = bc.ly, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = bc.m0; rb < bc.m1; rb += ngrp) {
            const int r = rb + grp;
            double acc = 0.0;
            if (r < bc.m1)
                for (int k = p.Arp[r] + lane; k < p.Arp[r + 1]; k += L)
                    acc += p.Av[k] * ldin(a, c, p.Aci[k]);
            acc = group_sum(acc, L);
            if (r < bc.m1 && lane == 0) {
                const int idx = n + r;
                const double val = -acc + p.b[r] * c.in_N - a.wy[r] * c.inv + ldin(a, c, idx);
                const double o = role_value(a, c, idx, val);
                a.out[idx] = o;
                s0 += o * o;
                s1 += (a.role == ROLE_RESID) ? a.rhs[idx] * a.rhs[idx] : p.b[r] * nscale(c, idx) * o;
                if (a.do_update) lsqr_update(a, c, idx);
            }
        }
    }
    if (tid == 0) {
        const double o = role_value(a, c, bc.tix, a.st->dot_fwd * c.inv + bc.xPx * c.in_N);
        a.out[bc.tix] = o;
        s0 += o * o;
        if (a.role == ROLE_RESID) s1 += a.rhs[bc.tix] * a.rhs[bc.tix];
        if (a.do_update) lsqr_update(a, c, bc.tix);
    }
}

// fused product with F' over the problem's work units
__device__ void blk_fused_FT(const Problem &p, const BatchDev &d, const StepArgs &a, const Ctx &c,
                             const BCtx &bc, double *sm, double &s0, double &s1) {
    for (int ui = bc.u0; ui < bc.u1; ++ui) {
        fused_unit(p, a, c, bc.lx, bc.ly, d.units[ui], sm, s0, s1);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double o = role_value(a, c, bc.tix, a.st->dot_adj * c.inv + bc.xPx * c.in_N);
        a.out[bc.tix] = o;
        s0 += o * o;
        if (a.role == ROLE_RESID) s1 += a.rhs[bc.tix] * a.rhs[bc.tix];
        if (a.do_update) lsqr_update(a, c, bc.tix);
    }
}

// wy = J(s o in_y) (raw) and the F tau-row dot c'(s o in)_x - b'wy, over the problem's units
__device__ void blk_pre(const Problem &p, const BatchDev &d, const double *in, const double *scl,
                        double *wy, const BCtx &bc, double *sm, double &s1) {
    const int n = p.n, tid = threadIdx.x;
    auto ld = [&](int idx) { return scl ? scl[idx] * in[idx] : in[idx]; };
    auto wout = [&](int r, double w) { wy[r] = w; s1 -= p.b[r] * w; };
    for (int ui = bc.u0; ui < bc.u1; ++ui) {
        const Unit u = d.units[ui];
        if (u.type == U_XROWS) {
            for (int i = u.begin + tid; i < u.end; i += kBlock) s1 += p.c[i] * ld(i);
        } else if (u.type == U_DIAG) {
            for (int r = u.begin + tid; r < u.end; r += kBlock) wout(r, p.jdiag[r] * ld(n + r));
        } else if (u.type == U_SOC) {
            const int cone = u.begin + tid;
            if (cone < u.end) soc_jv(p, cone, [&](int r) { return ld(n + r); }, wout);
        } else if (u.type == U_EXP) {
            const int cone = u.begin + tid;
            if (cone < u.end) exp_jv(p, cone, [&](int r) { return ld(n + r); }, wout);
        } else {
            psd_jv(p, u.begin, sm, [&](int r) { return ld(n + r); }, wout);
        }
        __syncthreads();
    }
}

// JVP right-hand side: u~ = -D_theta N[dtheta] on the problem's rows
__device__ void blk_jvp_rhs(const Problem &p, const BatchDev &d, const BCtx &bc, const double *dP,
                            const double *dA, const double *dq, const double *db, double &s0,
                            double &s1, double &s2) {
    const int n = p.n, tid = threadIdx.x;
    {
        const int L = bc.lx, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = bc.n0; rb < bc.n1; rb += ngrp) {
            const int row = rb + grp;
            double acc = 0.0, accT = 0.0;
            if (row < bc.n1) {
                for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) acc += dP[k] * p.x[p.Pci[k]];
                for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L)
                    accT += dA[p.Tperm[t]] * p.y[p.Tci[t]];
            }
            acc = group_sum(acc, L);
            accT = group_sum(accT, L);
            if (row < bc.n1 && lane == 0) {
                // LSQR starts from u~ = L(-d) (L the row scale); -d itself is kept in rhs
                const double o = -(acc + accT + dq[row]), l = d.scl ? d.scl[row] : 1.0;
                d.u[row] = l * o;
                d.rhs[row] = o;
                s0 += l * o * l * o;
                s1 += p.q[row] * o * l * l;
                s2 += p.x[row] * acc + dq[row] * p.x[row];
            }
        }
    }
    {
        const int L = bc.ly, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = bc.m0; rb < bc.m1; rb += ngrp) {
            const int r = rb + grp;
            double acc = 0.0;
            if (r < bc.m1)
                for (int k = p.Arp[r] + lane; k < p.Arp[r + 1]; k += L) acc += dA[k] * p.x[p.Aci[k]];
            acc = group_sum(acc, L);
            if (r < bc.m1 && lane == 0) {
                const double o = acc - db[r], l = d.scl ? d.scl[n + r] : 1.0;
                d.u[n + r] = l * o;
                d.rhs[n + r] = o;
                s0 += l * o * l * o;
                s1 += p.b[r] * o * l * l;
                s2 += db[r] * p.y[r];
            }
        }
    }
}

// VJP right-hand side: u~ = -D phi'(gx, gy, gs) on the problem's units
__device__ void blk_vjp_rhs(const Problem &p, const BatchDev &d, const BCtx &bc, const double *gx,
                            const double *gy, const double *gs, double *sm, double &s0, double &s2) {
    const int n = p.n, tid = threadIdx.x;
    auto put = [&](int idx, double o) {  // u~ = L o, o kept in rhs
        const double l = d.scl ? d.scl[idx] : 1.0;
        d.u[idx] = l * o;
        d.rhs[idx] = o;
        s0 += l * o * l * o;
    };
    auto gsum = [&](int r) { return gy[r] + gs[r]; };
    auto yout = [&](int r, double jt) {
        put(n + r, -(jt - gs[r]));
        s2 += p.y[r] * gy[r] + p.s[r] * gs[r];
    };
    for (int ui = bc.u0; ui < bc.u1; ++ui) {
        const Unit u = d.units[ui];
        if (u.type == U_XROWS) {
            for (int i = u.begin + tid; i < u.end; i += kBlock) {
                put(i, -gx[i]);
                s2 += p.x[i] * gx[i];
            }
        } else if (u.type == U_DIAG) {
            for (int r = u.begin + tid; r < u.end; r += kBlock) yout(r, p.jdiag[r] * gsum(r));
        } else if (u.type == U_SOC) {
            const int cone = u.begin + tid;
            if (cone < u.end) soc_jv(p, cone, gsum, yout);
        } else if (u.type == U_EXP) {
            const int cone = u.begin + tid;
            if (cone < u.end) exp_jv(p, cone, gsum, yout);
        } else {
            psd_jv(p, u.begin, sm, gsum, yout);
        }
        __syncthreads();
    }
}

__device__ inline BCtx bctx_of(const BatchDev &d, int b) {
    BCtx bc;
    bc.b = b;
    bc.n0 = d.n_off[b]; bc.n1 = d.n_off[b + 1];
    bc.m0 = d.m_off[b]; bc.m1 = d.m_off[b + 1];
    bc.tix = d.p.n + d.p.m + b;
    bc.lx = d.lxs[b]; bc.ly = d.lys[b];
    bc.u0 = d.u_off[b]; bc.u1 = d.u_off[b + 1];
    bc.xPx = d.xPx[b];
    return bc;
}

__device__ inline StepArgs base_of(const BatchDev &d, LsqrState *S) {
    StepArgs base{};
    base.sc = d.sc; base.scl = d.scl; base.wy = d.wy; base.xk = d.xk; base.wk = d.wk; base.rhs = d.rhs;
    base.st = S; base.in_nrm = NRM_ONE; base.role = ROLE_PLAIN;
    return base;
}

// One problem's JVP (dir 0) or VJP (dir 1) up to its LSQR loop: state, right-hand side and
// the first product of the bidiagonalisation (state in S, LDS).
__device__ void solve_begin(const BatchDev &d, int dir, int b, LsqrState *S, double *sm,
                            const double *i0, const double *i1, const double *i2, const double *i3) {
    const Problem &p = d.p;
    const int tid = threadIdx.x, n = p.n;
    const BCtx bc = bctx_of(d, b);
    const int Nb = (bc.n1 - bc.n0) + (bc.m1 - bc.m0) + 1;
    if (tid == 0) {
        LsqrState z = {};
        z.one = 1.0;
        z.tol = d.tol;
        z.max_iter = d.max_iter > 0 ? d.max_iter : 100 * Nb;
        *S = z;
    }
    auto each_index = [&](auto f) {
        for (int i = bc.n0 + tid; i < bc.n1; i += kBlock) f(i);
        for (int r = bc.m0 + tid; r < bc.m1; r += kBlock) f(n + r);
        if (tid == 0) f(bc.tix);
    };
    each_index([&](int i) { d.xk[i] = 0.0; d.wk[i] = 0.0; });
    __syncthreads();

    const StepArgs base = base_of(d, S);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;

    if (dir == 0) {
        blk_jvp_rhs(p, d, bc, i0, i1, i2, i3, s0, s1, s2);
        block_sum3(s0, s1, s2);
        if (tid == 0) {
            const double oN = s2, lN = d.scl ? d.scl[bc.tix] : 1.0;
            d.u[bc.tix] = lN * oN;
            d.rhs[bc.tix] = oN;
            const double beta = sqrt(s0 + lN * oN * lN * oN);
            S->beta = beta; S->beta1 = beta; S->phibar = beta; S->dot_adj = s1;
            if (!(beta > 0.0)) { S->done = 1; S->conv = 1; }
        }
        __syncthreads();
        if (!S->done) {  // v~ = sc o F'u, and J(sc o v~)
            StepArgs t = base;
            t.in = d.u; t.in_nrm = NRM_BETA; t.out = d.v; t.role = ROLE_V0; t.out_is_v = 1; t.do_pre = 1;
            const Ctx c = make_ctx(t, bc.tix);
            s0 = s1 = 0.0;
            blk_fused_FT(p, d, t, c, bc, sm, s0, s1);
            blk_reduce_finalize(S, ROLE_V0, s0, s1, 0.0, true);
        }
    } else {
        blk_vjp_rhs(p, d, bc, i0, i1, i2, sm, s0, s2);
        block_sum3(s0, s1, s2);
        if (tid == 0) {
            const double oN = s2, lN = d.scl ? d.scl[bc.tix] : 1.0;
            d.u[bc.tix] = lN * oN;
            d.rhs[bc.tix] = oN;
            const double beta = sqrt(s0 + lN * oN * lN * oN);
            S->beta = beta; S->beta1 = beta; S->phibar = beta;
            if (!(beta > 0.0)) { S->done = 1; S->conv = 1; }
        }
        __syncthreads();
        if (!S->done) {  // J(u~) and the F tau-row dot, then v~ = sc o F u
            s1 = 0.0;
            blk_pre(p, d, d.u, d.scl, d.wy, bc, sm, s1);
            block_sum3(s0, s1, s2);
            if (tid == 0) S->dot_fwd = s1;
            __syncthreads();
            StepArgs f = base;
            f.in = d.u; f.in_nrm = NRM_BETA; f.out = d.v; f.role = ROLE_V0; f.out_is_v = 1;
            const Ctx c = make_ctx(f, bc.tix);
            s0 = s1 = 0.0;
            blk_rows_F(p, f, c, bc, s0, s1);
            blk_reduce_finalize(S, ROLE_V0, s0, s1, 0.0, false);
        }
    }
}

// One problem's evaluation after its LSQR loop (final state in S): the owed update, the
// explicit residual and the outputs.
__device__ void solve_end(const BatchDev &d, int dir, int b, LsqrState *S, double *sm,
                          double *o0, double *o1, double *o2, double *o3) {
    const Problem &p = d.p;
    const int tid = threadIdx.x, n = p.n;
    const BCtx bc = bctx_of(d, b);
    auto each_index = [&](auto f) {
        for (int i = bc.n0 + tid; i < bc.n1; i += kBlock) f(i);
        for (int r = bc.m0 + tid; r < bc.m1; r += kBlock) f(n + r);
        if (tid == 0) f(bc.tix);
    };
    const StepArgs base = base_of(d, S);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    // owed x update, sol = sc o x, q'sol_x + b'sol_y for a product with F'
    {
        const bool pend = S->pending != 0;
        const double phr = S->phr;
        s1 = 0.0;
        each_index([&](int i) {
            double x = d.xk[i];
            if (pend) x += phr * d.wk[i];
            d.xk[i] = x;
            const double v = d.sc ? d.sc[i] * x : x;
            d.sol[i] = v;
            if (i < n) s1 += p.q[i] * v;
            else if (i < n + p.m) s1 += p.b[i - n] * v;
        });
        s0 = s2 = 0.0;
        block_sum3(s0, s1, s2);
        if (tid == 0) { S->pending = 0; S->dot_adj = s1; }
        __syncthreads();
    }
    if (dir == 0) {
        // explicit residual ||F sol + d|| and (dx, dy, ds) = D phi sol
        s1 = 0.0;
        blk_pre(p, d, d.sol, nullptr, d.wy_res, bc, sm, s1);
        s0 = s2 = 0.0;
        block_sum3(s0, s1, s2);
        if (tid == 0) S->dot_fwd = s1;
        __syncthreads();
        StepArgs f = base;  // the unscaled operator
        f.sc = nullptr; f.scl = nullptr; f.wy = d.wy_res;
        f.in = d.sol; f.in_nrm = NRM_ONE; f.out = d.scratch; f.role = ROLE_RESID;
        {
            const Ctx c = make_ctx(f, bc.tix);
            s0 = s1 = 0.0;
            blk_rows_F(p, f, c, bc, s0, s1);
        }
        blk_reduce_finalize(S, ROLE_RESID, s0, s1, 0.0, false);
        const double dzN = d.sol[bc.tix];
        for (int i = bc.n0 + tid; i < bc.n1; i += kBlock) o0[i] = d.sol[i] - dzN * p.x[i];
        for (int r = bc.m0 + tid; r < bc.m1; r += kBlock) {
            const double jd = d.wy_res[r];
            o1[r] = jd - dzN * p.y[r];
            o2[r] = jd - d.sol[n + r] - dzN * p.s[r];
        }
    } else {
        // explicit residual ||F'sol + dz|| and dtheta = D_theta N'[sol]
        StepArgs t = base;  // the unscaled operator
        t.sc = nullptr; t.scl = nullptr;
        t.in = d.sol; t.in_nrm = NRM_ONE; t.out = d.scratch; t.role = ROLE_RESID;
        {
            const Ctx c = make_ctx(t, bc.tix);
            s0 = s1 = 0.0;
            blk_fused_FT(p, d, t, c, bc, sm, s0, s1);
        }
        blk_reduce_finalize(S, ROLE_RESID, s0, s1, 0.0, true);
        const double *w = d.sol;
        const double wN = w[bc.tix];
        {
            const int L = bc.lx, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
            for (int rb = bc.n0; rb < bc.n1; rb += ngrp) {
                const int row = rb + grp;
                if (row < bc.n1) {
                    const double wi = w[row], xi = p.x[row];
                    for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) {
                        const int j = p.Pci[k];
                        const double xj = p.x[j];
                        o0[k] = 0.5 * (wi * xj + xi * w[j]) - wN * xi * xj;
                    }
                    if (lane == 0) o2[row] = wi - wN * xi;
                }
            }
        }
        {
            const int L = bc.ly, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
            for (int rb = bc.m0; rb < bc.m1; rb += ngrp) {
                const int r = rb + grp;
                if (r < bc.m1) {
                    const double yi = p.y[r], wyi = w[n + r];
                    for (int k = p.Arp[r] + lane; k < p.Arp[r + 1]; k += L) {
                        const int j = p.Aci[k];
                        o1[k] = yi * w[j] - wyi * p.x[j];
                    }
                    if (lane == 0) o3[r] = wyi - wN * yi;
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) d.st_out[b] = *S;
    __syncthreads();
}

// Begin and end phases: persistent workgroups taking problems from queue[q] (longest first).
__device__ inline int next_problem(const BatchDev &d, int q) {
    __shared__ int next;
    if (threadIdx.x == 0) {
        const int t = atomicAdd(d.queue + q, 1);
        next = t < d.B ? d.order[t] : -1;
    }
    __syncthreads();
    const int b = next;
    __syncthreads();
    return b;
}

__global__ __launch_bounds__(kBlock) void k_batch_begin(BatchDev d, int dir, const double *i0,
                                                        const double *i1, const double *i2,
                                                        const double *i3, LsqrState *st_loop,
                                                        int *ndone) {
    extern __shared__ double sm[];
    __shared__ LsqrState S;
    for (int b = next_problem(d, 0); b >= 0; b = next_problem(d, 0)) {
        solve_begin(d, dir, b, &S, sm, i0, i1, i2, i3);
        if (threadIdx.x == 0) {
            LsqrState s = S;
            s.pend_role = -1;  // the first product finalised its own reduction
            st_loop[b] = s;
            if (s.done) atomicAdd(ndone, 1);
        }
        __syncthreads();
    }
}

// The LSQR stopping test sees its own estimate (of the scaled residual, with a row scaling):
// a problem whose explicit (unscaled) relative residual is above tol resumes its LSQR from its
// loop state with a tighter internal tolerance, at most a few times and, as in the
// single-problem path, not again after a resume that lowered that residual by less than a
// tenth while the estimate went far below tol (its rounding floor).
__global__ __launch_bounds__(kBlock) void k_batch_end(BatchDev d, int dir, double *o0, double *o1,
                                                      double *o2, double *o3, LsqrState *st0,
                                                      LsqrState *st1, int only_resumed,
                                                      int allow_resume) {
    extern __shared__ double sm[];
    __shared__ LsqrState S;
    for (int b = next_problem(d, 1); b >= 0; b = next_problem(d, 1)) {
        if (only_resumed && !d.resume[b]) continue;
        if (threadIdx.x == 0) S = st0[b];
        __syncthreads();
        const LsqrState loop_state = S;
        solve_end(d, dir, b, &S, sm, o0, o1, o2, o3);
        if (threadIdx.x == 0) {
            const double rel = S.tau_rhs > 0.0 ? S.resid / S.tau_rhs : 0.0;
            const double prev = d.prev_rel[b];
            const double est = loop_state.beta1 > 0.0 ? loop_state.phibar / loop_state.beta1 : 0.0;
            const bool floor = prev > 0.0 && rel > 0.9 * prev && est <= 0.05 * d.tol;
            const bool again = allow_resume && !(rel <= d.tol) && loop_state.conv &&
                               loop_state.iters < loop_state.max_iter && loop_state.tol > 0.0 &&
                               !floor;
            d.resume[b] = again ? 1 : 0;
            if (again) {
                d.prev_rel[b] = rel;
                LsqrState r = loop_state;
                r.tol *= fmax(0.02, 0.5 * d.tol / rel);
                r.done = 0;
                r.conv = 0;
                r.phr = 0.0;       // the owed x update was applied above
                r.pending = 0;
                r.pend_role = -1;
                st0[b] = r;
                st1[b] = r;
                atomicAdd(d.nresumed, 1);
            }
        }
        __syncthreads();
    }
}

// One two-sided 2-norm balancing sweep of every problem's F with each cone block's Jacobian
// replaced by its diagonal (see k_equil_sweep of the single-problem path), one workgroup per
// problem: its x rows (P, A'), y rows (A) and its own tau row and column.
__global__ __launch_bounds__(kBlock) void k_batch_equil_sweep(BatchDev d, const double *DL,
                                                              const double *DR, double *DLo,
                                                              double *DRo) {
    const Problem &p = d.p;
    const BCtx bc = bctx_of(d, blockIdx.x);
    const int n = p.n, tid = threadIdx.x, tix = bc.tix;
    const double dlN = DL[tix], drN = DR[tix];
    auto upd = [&](int i, double rsum, double csum) {
        const double rn = DL[i] * sqrt(rsum), cn = DR[i] * sqrt(csum);
        DLo[i] = rn > 0.0 ? DL[i] / sqrt(rn) : DL[i];
        DRo[i] = cn > 0.0 ? DR[i] / sqrt(cn) : DR[i];
    };
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    {
        const int L = bc.lx, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = bc.n0; rb < bc.n1; rb += ngrp) {
            const int row = rb + grp;
            double rs = 0.0, cs = 0.0;
            if (row < bc.n1) {
                for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) {
                    const double v2 = p.Pv[k] * p.Pv[k];
                    const int j = p.Pci[k];
                    rs += v2 * DR[j] * DR[j];
                    cs += v2 * DL[j] * DL[j];
                }
                for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L) {
                    const int r = p.Tci[t];
                    const double v2 = p.Tv[t] * p.Tv[t], jd = p.jdiag[r];
                    rs += v2 * jd * jd * DR[n + r] * DR[n + r];
                    cs += v2 * DL[n + r] * DL[n + r];
                }
            }
            rs = group_sum(rs, L);
            cs = group_sum(cs, L);
            if (row < bc.n1 && lane == 0) {
                const double q = p.q[row], c = p.c[row];
                upd(row, rs + q * q * drN * drN, cs + c * c * dlN * dlN);
                s0 += c * c * DR[row] * DR[row];
                s1 += q * q * DL[row] * DL[row];
            }
        }
    }
    {
        const int L = bc.ly, lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
        for (int rb = bc.m0; rb < bc.m1; rb += ngrp) {
            const int r = rb + grp;
            double rs = 0.0, cs = 0.0;
            if (r < bc.m1)
                for (int k = p.Arp[r] + lane; k < p.Arp[r + 1]; k += L) {
                    const double v2 = p.Av[k] * p.Av[k];
                    const int j = p.Aci[k];
                    rs += v2 * DR[j] * DR[j];
                    cs += v2 * DL[j] * DL[j];
                }
            rs = group_sum(rs, L);
            cs = group_sum(cs, L);
            if (r < bc.m1 && lane == 0) {
                const int i = n + r;
                const double jd = p.jdiag[r], bb = p.b[r], o = 1.0 - jd;
                upd(i, rs + o * o * DR[i] * DR[i] + bb * bb * drN * drN,
                    jd * jd * cs + o * o * DL[i] * DL[i] + bb * bb * jd * jd * dlN * dlN);
                s0 += bb * bb * jd * jd * DR[i] * DR[i];
                s1 += bb * bb * DL[i] * DL[i];
            }
        }
    }
    block_sum3(s0, s1, s2);
    if (tid == 0) {
        const double x2 = bc.xPx * bc.xPx;
        upd(tix, s0 + x2 * drN * drN, s1 + x2 * dlN * dlN);
    }
}

// ---------------------------------------------------------------------------------------
// batch setup kernels
// ---------------------------------------------------------------------------------------

// Local CSR blocks (problem after problem, row pointers starting at 0) -> one block-diagonal
// CSR with global column indices; validates each block. One workgroup per problem.
__global__ void k_batch_csr(const int *rp_loc, const int *ci_loc, const int *row_off,
                            const int *col_off, const int *nz_off, int *rp, int *ci, int last_row,
                            int *flag) {
    const int b = blockIdx.x;
    const int r0 = row_off[b], nr = row_off[b + 1] - r0;
    const int c0 = col_off[b], nc = col_off[b + 1] - c0;
    const int z0 = nz_off[b], nz = nz_off[b + 1] - z0;
    const int *lrp = rp_loc + r0 + b;  // each block has nr + 1 row pointers
    if (threadIdx.x == 0 && (lrp[0] != 0 || lrp[nr] != nz)) atomicOr(flag, 1);
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
        const int a = lrp[i], e = lrp[i + 1];
        rp[r0 + i] = z0 + a;
        if (a > e || a < 0 || e > nz) { atomicOr(flag, 1); continue; }
    }
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
        const int j = ci_loc[z0 + k];
        if (j < 0 || j >= nc) atomicOr(flag, 1);
        ci[z0 + k] = j + c0;
    }
    if (b == (int)gridDim.x - 1 && threadIdx.x == 0) rp[last_row] = z0 + nz;
}

// per problem: x'Px (P x is already in c = -2Px - q: x'Px = -(x'c + x'q)/2 would lose
// digits, so it is recomputed from the CSR rows)
__global__ __launch_bounds__(kBlock) void k_batch_xpx(Problem p, const int *n_off, double *xpx) {
    const int b = blockIdx.x;
    double acc = 0.0, z1 = 0.0, z2 = 0.0;
    for (int i = n_off[b] + threadIdx.x; i < n_off[b + 1]; i += kBlock) {
        double r = 0.0;
        for (int k = p.Prp[i]; k < p.Prp[i + 1]; ++k) r += p.Pv[k] * p.x[p.Pci[k]];
        acc += p.x[i] * r;
    }
    block_sum3(acc, z1, z2);
    if (threadIdx.x == 0) xpx[b] = acc;
}

// zero / nonnegative rows of every problem: J = 1, resp. 1{z > 0}
__global__ void k_batch_diag(const double *zy, const int *m_off, const int *nz, const int *nn,
                             double *jdiag, int *nondiff) {
    const int b = blockIdx.x;
    const int r0 = m_off[b];
    for (int t = threadIdx.x; t < nz[b] + nn[b]; t += blockDim.x) {
        const int r = r0 + t;
        if (t < nz[b]) {
            jdiag[r] = 1.0;
        } else {
            const double z = zy[r];
            jdiag[r] = z > 0.0 ? 1.0 : 0.0;
            if (fabs(z) <= 1e-10) atomicOr(nondiff, 1);
        }
    }
}

// tau column / row norms of every problem (see the single-problem scales)
__global__ __launch_bounds__(kBlock) void k_batch_tau_scales(Problem p, const int *n_off,
                                                             const int *m_off, const double *xpx,
                                                             double *dj, double *dv) {
    const int b = blockIdx.x;
    double s0 = 0.0, s1 = 0.0, z = 0.0;
    for (int i = n_off[b] + threadIdx.x; i < n_off[b + 1]; i += kBlock) {
        s0 += p.q[i] * p.q[i];
        s1 += p.c[i] * p.c[i];
    }
    for (int r = m_off[b] + threadIdx.x; r < m_off[b + 1]; r += kBlock) {
        const double jd = p.jdiag[r];
        s0 += p.b[r] * p.b[r];
        s1 += p.b[r] * p.b[r] * jd * jd;
    }
    block_sum3(s0, s1, z);
    if (threadIdx.x == 0) {
        const int t = p.n + p.m + b;
        const double x2 = xpx[b] * xpx[b];
        dj[t] = (s0 + x2) > 0.0 ? 1.0 / sqrt(s0 + x2) : 1.0;
        dv[t] = (s1 + x2) > 0.0 ? 1.0 / sqrt(s1 + x2) : 1.0;
    }
}

}  // namespace qcpd

// ---------------------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------------------

using namespace qcpd;

struct qcpd_batch {
    hipStream_t stream = nullptr;
    qcpd_opts opts{};
    BatchDev d{};
    int lds = 0;
    int grid = 0;
    int grid_default = 0;  // all workgroups that fit on the device at once (capped at B)
    std::vector<void *> allocs;
    double *scale[2] = {nullptr, nullptr};  // Jacobi: [0] columns of F, [1] columns of F'
    double *equil[2] = {nullptr, nullptr};  // two-sided equilibration: [0] columns, [1] rows
    const double *graph_scl[2] = {nullptr, nullptr};
    int nnzP = 0, nnzA = 0;
    int *flag = nullptr, *host_flag = nullptr;
    LsqrState *st = nullptr;
    std::vector<LsqrState> host_st;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    uint32_t create_flags = 0;
    // segmented LSQR loop
    hipStream_t cap = nullptr;  // private stream used only for graph capture
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_chunk[2] = {0, 0};
    const double *graph_sc[2] = {nullptr, nullptr};
    SegGrid seg{};
    int lds_seg = 0;
    LsqrState *stl[2] = {nullptr, nullptr};  // one state per problem, double-buffered
    double *spart[2] = {nullptr, nullptr};   // per-item partial sums, double-buffered
    int *host_ndone = nullptr;               // pinned
    std::vector<int> nb_rows;                // n + m + 1 per problem
    // work lists of the running problems only: host copies of the full lists, device
    // buffers for the compacted ones, and the running count at the last compaction
    std::vector<SegItem> h_fitems;
    std::vector<Unit> h_tunits;
    std::vector<int> h_tprob;
    const SegItem *full_fitems = nullptr;
    const Unit *full_tunits = nullptr;
    const int *full_tprob = nullptr;
    SegItem *c_fitems = nullptr;
    Unit *c_tunits = nullptr;
    int *c_tprob = nullptr, *c_fslot = nullptr, *c_tslot = nullptr;
    int running_at = 0;
    int seg_version = 0;
    // values of the union's P, A, A' with a scale folded in: [0] sc, [1] scl (per run)
    double *sval[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int graph_version[2] = {-1, -1};
};

namespace {

template <class T>
qcpd_status balloc(qcpd_batch *h, T **ptr, long long count) {
    *ptr = nullptr;
    if (count <= 0) count = 1;
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (size_t)count) != hipSuccess) return QCPD_ERR_OOM;
    h->allocs.push_back(p);
    *ptr = static_cast<T *>(p);
    return QCPD_OK;
}

#define BALLOC(ptr, count)                                   \
    do {                                                     \
        qcpd_status s_ = balloc(h, &(ptr), (long long)(count)); \
        if (s_ != QCPD_OK) return s_;                        \
    } while (0)
#define BCHK(expr)                                 \
    do {                                           \
        if ((expr) != hipSuccess) return QCPD_ERR_HIP; \
    } while (0)

template <class T>
qcpd_status upload(qcpd_batch *h, T **dst, const std::vector<T> &src) {
    qcpd_status rc = balloc(h, dst, (long long)src.size());
    if (rc != QCPD_OK) return rc;
    if (!src.empty() && hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess)
        return QCPD_ERR_HIP;
    return QCPD_OK;
}

#define UPLOAD(dst, src)                                 \
    do {                                                 \
        qcpd_status s_ = upload(h, &(dst), (src));       \
        if (s_ != QCPD_OK) return s_;                    \
    } while (0)

// Lanes per CSR row of the batched loop: a power of two (<= 64) that gives each lane about
// `per_lane` stored entries (opts.nnz_per_lane_F, else kSegPerLane; the autotuner picks it).
constexpr double kSegPerLane = 32.0;
int lanes_of(double avg, double per_lane) {
    int L = 1;
    while (L < 64 && 2 * L * per_lane <= avg) L *= 2;
    return L;
}

void free_batch(qcpd_batch *h) {
    if (!h) return;
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->host_flag) (void)hipHostFree(h->host_flag);
    if (h->host_ndone) (void)hipHostFree(h->host_ndone);
    for (int d = 0; d < 2; ++d)
        if (h->graph[d]) (void)hipGraphExecDestroy(h->graph[d]);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

qcpd_status flag_sync(qcpd_batch *h) {
    BCHK(hipMemcpyAsync(h->host_flag, h->flag, 8 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    BCHK(hipStreamSynchronize(h->stream));
    return QCPD_OK;
}

qcpd_status batch_create_impl(qcpd_batch *h, const qcpd_batch_layout *L, const int32_t *P_rp,
                              const int32_t *P_ci, const double *P_v, const int32_t *A_rp,
                              const int32_t *A_ci, const double *A_v, const double *q,
                              const double *bv, const double *x, const double *y, const double *s) {
    const int B = L->nprob;
    hipStream_t st = h->stream;
    std::vector<int> n_off(B + 1, 0), m_off(B + 1, 0), pz(B + 1, 0), az(B + 1, 0);
    for (int i = 0; i < B; ++i) {
        n_off[i + 1] = n_off[i] + L->n[i];
        m_off[i + 1] = m_off[i] + L->m[i];
        pz[i + 1] = pz[i] + L->nnz_P[i];
        az[i + 1] = az[i] + L->nnz_A[i];
    }
    const int n = n_off[B], m = m_off[B], NT = n + m + B;
    h->nnzP = pz[B];
    h->nnzA = az[B];
    Problem &p = h->d.p;
    p.n = n; p.m = m; p.N = NT; p.nnzP = pz[B]; p.nnzA = az[B];
    int *Prp, *Pci, *Arp, *Aci, *Trp, *Tci, *Tperm, *d_noff, *d_moff, *d_pz, *d_az;
    double *Pv, *Av, *Tv, *dq_, *db_, *dx_, *dy_, *ds_, *c, *zy, *xpx, *jdiag;
    BALLOC(Prp, n + 1); BALLOC(Pci, pz[B]); BALLOC(Pv, pz[B]);
    BALLOC(Arp, m + 1); BALLOC(Aci, az[B]); BALLOC(Av, az[B]);
    BALLOC(Trp, n + 1); BALLOC(Tci, az[B]); BALLOC(Tv, az[B]); BALLOC(Tperm, az[B]);
    BALLOC(dq_, n); BALLOC(db_, m); BALLOC(dx_, n); BALLOC(dy_, m); BALLOC(ds_, m);
    BALLOC(c, n); BALLOC(zy, m); BALLOC(xpx, B); BALLOC(jdiag, m);
    BALLOC(h->flag, 8);  // 0 CSR, 1 NaN, 2 pattern, 3 cone failure, 4 non-differentiable
    UPLOAD(d_noff, n_off); UPLOAD(d_moff, m_off); UPLOAD(d_pz, pz); UPLOAD(d_az, az);
    BCHK(hipMemsetAsync(h->flag, 0, 8 * sizeof(int), st));
    if (pz[B]) BCHK(hipMemcpyAsync(Pv, P_v, 8LL * pz[B], hipMemcpyDeviceToDevice, st));
    if (az[B]) BCHK(hipMemcpyAsync(Av, A_v, 8LL * az[B], hipMemcpyDeviceToDevice, st));
    BCHK(hipMemcpyAsync(dq_, q, 8LL * n, hipMemcpyDeviceToDevice, st));
    BCHK(hipMemcpyAsync(dx_, x, 8LL * n, hipMemcpyDeviceToDevice, st));
    if (m) {
        BCHK(hipMemcpyAsync(db_, bv, 8LL * m, hipMemcpyDeviceToDevice, st));
        BCHK(hipMemcpyAsync(dy_, y, 8LL * m, hipMemcpyDeviceToDevice, st));
        BCHK(hipMemcpyAsync(ds_, s, 8LL * m, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_batch_csr, dim3(B), dim3(256), 0, st, P_rp, P_ci, d_noff, d_noff, d_pz, Prp,
                       Pci, n, h->flag);
    hipLaunchKernelGGL(k_batch_csr, dim3(B), dim3(256), 0, st, A_rp, A_ci, d_moff, d_noff, d_az, Arp,
                       Aci, m, h->flag);
    qcpd_status rc = flag_sync(h);
    if (rc != QCPD_OK) return rc;
    if (h->host_flag[0]) return QCPD_ERR_INVALID_ARG;
    {
        std::vector<const double *> ptrs = {Pv, Av, dq_, db_, dx_, dy_, ds_};
        std::vector<long long> lens = {pz[B], az[B], n, m, n, m, m};
        const double **dp;
        long long *dl;
        BALLOC(dp, 8);
        BALLOC(dl, 8);
        BCHK(hipMemcpy(dp, ptrs.data(), sizeof(double *) * ptrs.size(), hipMemcpyHostToDevice));
        BCHK(hipMemcpy(dl, lens.data(), sizeof(long long) * lens.size(), hipMemcpyHostToDevice));
        launch_nan_scan(dp, dl, (int)ptrs.size(), h->flag + 1, st);
        rc = flag_sync(h);
        if (rc != QCPD_OK) return rc;
        if (h->host_flag[1]) return QCPD_ERR_NAN;
    }
    BCHK(csr_transpose(m, n, az[B], Arp, Aci, Av, Trp, Tci, Tv, Tperm, st));
    if (h->opts.check_symmetry) {
        int *Srp, *Sci, *Sperm;
        double *Sv;
        BALLOC(Srp, n + 1); BALLOC(Sci, pz[B]); BALLOC(Sv, pz[B]); BALLOC(Sperm, pz[B]);
        launch_check_sorted(Prp, Pci, n, n, h->flag + 2, st);
        BCHK(csr_transpose(n, n, pz[B], Prp, Pci, Pv, Srp, Sci, Sv, Sperm, st));
        launch_check_symmetric(Prp, Pci, Pv, Srp, Sci, Sv, n, pz[B], h->flag + 2, st);
        rc = flag_sync(h);
        if (rc != QCPD_OK) return rc;
        if (h->host_flag[2]) return QCPD_ERR_PATTERN;
    }
    p.Prp = Prp; p.Pci = Pci; p.Pv = Pv; p.Arp = Arp; p.Aci = Aci; p.Av = Av;
    p.Trp = Trp; p.Tci = Tci; p.Tv = Tv; p.Tperm = Tperm;
    p.q = dq_; p.b = db_; p.x = dx_; p.y = dy_; p.s = ds_; p.c = c; p.zy = zy; p.jdiag = jdiag;
    // per-problem lanes, cone tables (global y rows), work units
    const double spl = h->opts.nnz_per_lane_F > 0 ? (double)h->opts.nnz_per_lane_F : kSegPerLane;
    std::vector<int> lx(B), ly(B), soc_row, soc_dim, psd_row, psd_k, exp_rows, nzv(B), nnv(B);
    std::vector<long long> psd_off;
    std::vector<Unit> units;
    std::vector<int> u_off(B + 1, 0);
    std::vector<double> cost(B);
    long long pool_sz = 0;
    int kmax = 0;
    for (int b = 0; b < B; ++b) {
        const qcpd_cones &K = L->cones[b];
        const int nb = L->n[b], mb = L->m[b];
        lx[b] = lanes_of(nb ? (double)(L->nnz_P[b] + L->nnz_A[b]) / nb : 1.0, spl);
        ly[b] = lanes_of(mb ? (double)L->nnz_A[b] / mb : 1.0, spl);
        nzv[b] = K.n_zero;
        nnv[b] = K.n_nonneg;
        units.push_back({U_XROWS, n_off[b], n_off[b + 1], 0});
        const int ndiag = K.n_zero + K.n_nonneg;
        int row = m_off[b];
        if (ndiag) units.push_back({U_DIAG, row, row + ndiag, 0});
        row += ndiag;
        const int soc0 = (int)soc_row.size();
        for (int i = 0; i < K.n_soc; ++i) { soc_row.push_back(row); soc_dim.push_back(K.soc_dims[i]); row += K.soc_dims[i]; }
        for (int i = 0; i < K.n_soc;) {
            int j = i, rws = 0;
            while (j < K.n_soc && j - i < kBlock && (j == i || rws + K.soc_dims[j] <= 256) &&
                   rws + K.soc_dims[j] <= kUnitRows) {
                rws += K.soc_dims[j];
                ++j;
            }
            if (j == i) return QCPD_ERR_CONE;
            units.push_back({U_SOC, soc0 + i, soc0 + j, soc_row[soc0 + i]});
            i = j;
        }
        double psd_cost = 0.0;
        for (int i = 0; i < K.n_psd; ++i) {
            const int k = K.psd_orders[i];
            units.push_back({U_PSD, (int)psd_row.size(), (int)psd_row.size() + 1, row});
            psd_row.push_back(row); psd_k.push_back(k); psd_off.push_back(pool_sz);
            row += k * (k + 1) / 2; pool_sz += 2LL * k * k; kmax = std::max(kmax, k);
            psd_cost += 8.0 * k * k * k;
        }
        const int exp0 = (int)exp_rows.size();
        for (int i = 0; i < K.n_exp; ++i) { exp_rows.push_back(row); row += 3; }
        for (int i = 0; i < K.n_exp; i += 85)
            units.push_back({U_EXP, exp0 + i, exp0 + std::min(K.n_exp, i + 85), exp_rows[exp0 + i]});
        u_off[b + 1] = (int)units.size();
        cost[b] = 12.0 * (L->nnz_P[b] + 2.0 * L->nnz_A[b]) + 40.0 * (nb + mb) + psd_cost;
    }
    // work items of the segmented loop, grouped by problem: the product with F over chunks of
    // x rows and of y rows; the fused product with F' over PSD cones (longest first), runs of
    // exponential and SOC cones, chunks of diagonal rows and of x rows
    std::vector<SegItem> fitems;
    std::vector<Unit> tunits;
    std::vector<int> tprob, foff(B + 1, 0), toff(B + 1, 0);
    h->nb_rows.resize(B);
    for (int b = 0; b < B; ++b) {
        const int rx = kBlock / lx[b], ry = kBlock / ly[b];
        h->nb_rows[b] = L->n[b] + L->m[b] + 1;
        for (int r = n_off[b]; r < n_off[b + 1]; r += rx)
            fitems.push_back({0, r, std::min(n_off[b + 1], r + rx), b});
        for (int r = m_off[b]; r < m_off[b + 1]; r += ry)
            fitems.push_back({1, r, std::min(m_off[b + 1], r + ry), b});
        foff[b + 1] = (int)fitems.size();
        std::vector<Unit> mine(units.begin() + u_off[b], units.begin() + u_off[b + 1]);
        std::stable_sort(mine.begin(), mine.end(), [&](const Unit &x, const Unit &y) {
            auto rank = [](int t) { return t == U_PSD ? 0 : t == U_EXP ? 1 : t == U_SOC ? 2 : t == U_DIAG ? 3 : 4; };
            return rank(x.type) < rank(y.type);
        });
        for (const Unit &u : mine) {
            if (u.type == U_XROWS || u.type == U_DIAG) {
                const int step = u.type == U_XROWS ? rx : ry;
                for (int r = u.begin; r < u.end; r += step) {
                    tunits.push_back({u.type, r, std::min(u.end, r + step), 0});
                    tprob.push_back(b);
                }
            } else {
                tunits.push_back(u);
                tprob.push_back(b);
            }
        }
        toff[b + 1] = (int)tunits.size();
    }
    // longest problems first (a greedy longest-processing-time schedule for the queue)
    std::vector<int> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return cost[a] > cost[b2]; });
    int *d_lx, *d_ly, *d_soc_row, *d_soc_dim, *d_psd_row, *d_psd_k, *d_exp_rows, *d_uoff, *d_order, *d_nz, *d_nn;
    long long *d_psd_off;
    Unit *d_units;
    double *soc_par, *exp_J, *pool;
    UPLOAD(d_lx, lx); UPLOAD(d_ly, ly); UPLOAD(d_soc_row, soc_row); UPLOAD(d_soc_dim, soc_dim);
    UPLOAD(d_psd_row, psd_row); UPLOAD(d_psd_k, psd_k); UPLOAD(d_psd_off, psd_off);
    UPLOAD(d_exp_rows, exp_rows); UPLOAD(d_uoff, u_off); UPLOAD(d_order, order); UPLOAD(d_units, units);
    UPLOAD(d_nz, nzv); UPLOAD(d_nn, nnv);
    BALLOC(soc_par, 4LL * soc_row.size()); BALLOC(exp_J, 9LL * exp_rows.size()); BALLOC(pool, pool_sz);
    p.n_diag = 0;
    p.n_soc = (int)soc_row.size(); p.soc_row = d_soc_row; p.soc_dim = d_soc_dim; p.soc_par = soc_par;
    p.n_exp = (int)exp_rows.size(); p.exp_row0 = 0; p.exp_rows = d_exp_rows; p.exp_J = exp_J;
    p.n_psd = (int)psd_row.size(); p.psd_row = d_psd_row; p.psd_k = d_psd_k; p.psd_off = d_psd_off;
    p.psd_pool = pool;
    p.psd_lr = nullptr;  // the batch kernels apply the full form
    p.Prp4 = p.Arp4 = nullptr;
    p.Pc4 = p.Ac4 = nullptr;
    p.Pv4 = p.Av4 = nullptr;
    // Px, c, x'Px per problem, z_y, cone factors, scales
    double *partials;
    int *counter;
    RowGrid rg;
    rg.lx = lanes_of(n ? (double)(pz[B] + az[B]) / n : 1.0, spl);
    rg.ly = lanes_of(m ? (double)az[B] / m : 1.0, spl);
    rg.bx = div_up((long long)n * rg.lx, kBlock);
    rg.by = div_up((long long)(m + 1) * rg.ly, kBlock);
    BALLOC(partials, 3LL * (rg.total() + 1)); BALLOC(counter, 1);
    BCHK(hipMemsetAsync(counter, 0, sizeof(int), st));
    RowGrid pg = rg;
    pg.by = 0;
    double *xpx_all;
    BALLOC(xpx_all, 1);
    launch_px(p, pg, c, xpx_all, partials, counter, st);
    hipLaunchKernelGGL(k_batch_xpx, dim3(B), dim3(kBlock), 0, st, p, d_noff, xpx);
    launch_sub(dy_, ds_, zy, m, st);
    ConeHost ch{0, p.n_exp, 0, nullptr};
    launch_cone_factors(p, ch, jdiag, soc_par, exp_J, pool, h->flag + 4, h->flag + 3,
                        psd_factor_lds_bytes(kmax), st);
    hipLaunchKernelGGL(k_batch_diag, dim3(B), dim3(256), 0, st, zy, d_moff, d_nz, d_nn, jdiag, h->flag + 4);
    BALLOC(h->scale[0], NT); BALLOC(h->scale[1], NT);
    launch_scales(p, rg, h->scale[0], h->scale[1], partials, counter, st, 0);
    hipLaunchKernelGGL(k_batch_tau_scales, dim3(B), dim3(kBlock), 0, st, p, d_noff, d_moff, xpx,
                       h->scale[0], h->scale[1]);
    rc = flag_sync(h);
    if (rc != QCPD_OK) return rc;
    BCHK(hipGetLastError());
    if (h->host_flag[3]) return QCPD_ERR_CONE;
    // workspace
    BatchDev &d = h->d;
    d.B = B; d.n_off = d_noff; d.m_off = d_moff; d.u_off = d_uoff; d.lxs = d_lx; d.lys = d_ly;
    d.units = d_units; d.xPx = xpx; d.order = d_order;
    BALLOC(d.queue, 2);
    BALLOC(d.u, NT); BALLOC(d.v, NT); BALLOC(d.xk, NT); BALLOC(d.wk, NT); BALLOC(d.rhs, NT);
    BALLOC(d.sol, NT); BALLOC(d.scratch, NT); BALLOC(d.wy, m); BALLOC(d.wy_res, m);
    BALLOC(d.resume, B); BALLOC(d.nresumed, 1); BALLOC(d.prev_rel, B);
    BCHK(hipMemsetAsync(d.resume, 0, sizeof(int) * B, st));
    // two-sided equilibration of every problem (even number of sweeps: ends in equil[])
    {
        double *tl, *tr;
        BALLOC(h->equil[0], NT); BALLOC(h->equil[1], NT); BALLOC(tl, NT); BALLOC(tr, NT);
        launch_fill(h->equil[0], NT, 1.0, st);
        launch_fill(h->equil[1], NT, 1.0, st);
        BatchDev de = d;
        de.p = p;
        for (int k = 0; k < 20; ++k) {
            const bool even = (k % 2) == 0;
            hipLaunchKernelGGL(k_batch_equil_sweep, dim3(B), dim3(kBlock), 0, st, de,
                               even ? h->equil[1] : tl, even ? h->equil[0] : tr,
                               even ? tl : h->equil[1], even ? tr : h->equil[0]);
        }
        BCHK(hipGetLastError());
    }
    BALLOC(h->st, B);
    d.st_out = h->st;
    h->host_st.resize(B);
    h->lds = fused_lds_bytes(kmax);
    BCHK(hipFuncSetAttribute((const void *)k_batch_begin, hipFuncAttributeMaxDynamicSharedMemorySize, h->lds));
    BCHK(hipFuncSetAttribute((const void *)k_batch_end, hipFuncAttributeMaxDynamicSharedMemorySize, h->lds));
    // the segmented loop
    {
        SegItem *d_fitems;
        Unit *d_tunits;
        int *d_tprob, *d_foff, *d_toff;
        UPLOAD(d_fitems, fitems); UPLOAD(d_tunits, tunits); UPLOAD(d_tprob, tprob);
        UPLOAD(d_foff, foff); UPLOAD(d_toff, toff);
        SegGrid &g = h->seg;
        g.B = B; g.nf = (int)fitems.size(); g.nt = (int)tunits.size();
        g.fitems = d_fitems; g.foff = d_foff; g.tunits = d_tunits; g.tprob = d_tprob; g.toff = d_toff;
        g.fslot = g.tslot = nullptr;
        g.small_psd = kmax <= 16 ? 1 : 0;
        fill_unit_ranges(p, d_tunits, g.nt, st);
        h->h_fitems = fitems;
        h->h_tunits.resize(tunits.size());
        BCHK(hipMemcpyAsync(h->h_tunits.data(), d_tunits, sizeof(Unit) * tunits.size(),
                            hipMemcpyDeviceToHost, st));
        BCHK(hipStreamSynchronize(st));
        h->h_tprob = tprob;
        h->full_fitems = d_fitems; h->full_tunits = d_tunits; h->full_tprob = d_tprob;
        BALLOC(h->c_fitems, g.nf); BALLOC(h->c_tunits, g.nt); BALLOC(h->c_tprob, g.nt);
        BALLOC(h->c_fslot, g.nf); BALLOC(h->c_tslot, g.nt);
        g.lxs = d_lx; g.lys = d_ly; g.xPx = xpx;
        BALLOC(g.ndone, 1);
        const int slots = std::max(g.nf, g.nt);
        BALLOC(h->spart[0], 2LL * slots); BALLOC(h->spart[1], 2LL * slots);
        BALLOC(h->stl[0], B); BALLOC(h->stl[1], B);
        h->lds_seg = loop_lds_bytes(psd_k.data(), (int)psd_k.size());
        set_seg_kernel_lds(h->lds_seg);
        if (hipHostMalloc((void **)&h->host_ndone, sizeof(int), hipHostMallocDefault) != hipSuccess)
            return QCPD_ERR_OOM;
        BCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    }
    int dev = 0, ncu = 0, per_cu = 0;
    BCHK(hipGetDevice(&dev));
    BCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    BCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch_begin, kBlock, h->lds));
    h->grid = std::max(1, std::min(B, ncu * std::max(per_cu, 1)));
    h->grid_default = h->grid;
    h->create_flags = h->host_flag[4] ? 2u : 0u;
    return h->host_flag[4] ? QCPD_WARN_NONDIFF : QCPD_OK;
}

// One LSQR iteration of every problem (two launches, states and partials double-buffered).
// Fold the run's scales into copies of the union's CSR values (the loop kernels then read
// one value per entry instead of a value and a gathered scale).
qcpd_status seg_bake(qcpd_batch *h) {
    const Problem &p = h->d.p;
    const double *sv[2] = {h->d.sc, h->d.scl};
    for (int j = 0; j < 2; ++j) {
        if (!sv[j] || p.nnzP == 0 || p.nnzA == 0) continue;
        if (!h->sval[j][0]) {
            BALLOC(h->sval[j][0], p.nnzP);
            BALLOC(h->sval[j][1], p.nnzA);
            BALLOC(h->sval[j][2], p.nnzA);
        }
        launch_scale_vals(p.Pci, p.Pv, p.nnzP, sv[j], 0, h->sval[j][0], h->stream);
        launch_scale_vals(p.Aci, p.Av, p.nnzA, sv[j], 0, h->sval[j][1], h->stream);
        launch_scale_vals(p.Tci, p.Tv, p.nnzA, sv[j], p.n, h->sval[j][2], h->stream);
    }
    BCHK(hipGetLastError());
    return QCPD_OK;
}

void seg_baked(const qcpd_batch *h, StepArgs &a) {
    const int j = a.in_is_v ? 0 : 1;
    const double *isc = a.in_is_v ? a.sc : a.scl;
    if (isc && h->sval[j][0]) {
        a.Pvs = h->sval[j][0];
        a.Avs = h->sval[j][1];
        a.Tvs = h->sval[j][2];
    }
}

void enqueue_seg_iteration(const qcpd_batch *h, int dir, hipStream_t s) {
    const BatchDev &d = h->d;
    StepArgs a{};
    a.sc = d.sc; a.scl = d.scl; a.wy = d.wy; a.xk = d.xk; a.wk = d.wk;
    StepArgs first = a, second = a;
    first.st = h->stl[0]; first.st_next = h->stl[1]; first.part_prev = h->spart[0]; first.part_next = h->spart[1];
    second.st = h->stl[1]; second.st_next = h->stl[0]; second.part_prev = h->spart[1]; second.part_next = h->spart[0];
    if (dir == 0) {
        StepArgs &f = first;  // u~ <- F(sc o v) - alpha u~ (and the owed x, w update)
        f.in = d.v; f.in_nrm = NRM_ALPHA; f.in_is_v = 1; f.out = d.u; f.role = ROLE_U; f.do_update = 1;
        seg_baked(h, f);
        launch_seg_F(d.p, f, h->seg, s);
        StepArgs &t = second;  // v~ <- sc o F'u - beta v~, then J(sc o v~)
        t.in = d.u; t.in_nrm = NRM_BETA; t.out = d.v; t.role = ROLE_V; t.out_is_v = 1; t.do_pre = 1;
        seg_baked(h, t);
        launch_seg_FT(d.p, t, h->seg, h->lds_seg, s);
    } else {
        StepArgs &t = first;  // u~ <- F'(sc o v) - alpha u~ (and the owed update), J(u~)
        t.in = d.v; t.in_nrm = NRM_ALPHA; t.in_is_v = 1; t.out = d.u; t.role = ROLE_U;
        t.do_update = 1; t.do_pre = 1;
        seg_baked(h, t);
        launch_seg_FT(d.p, t, h->seg, h->lds_seg, s);
        StepArgs &f = second;  // v~ <- sc o F u - beta v~
        f.in = d.u; f.in_nrm = NRM_BETA; f.out = d.v; f.role = ROLE_V; f.out_is_v = 1;
        seg_baked(h, f);
        launch_seg_F(d.p, f, h->seg, s);
    }
}

// Launch lists of the segmented loop: every item (all = true), or only the items of the
// problems still running (their LSQR state not done; a stop is written to both state
// buffers, so either shows it). Items keep their partial-sum slot, so the per-problem slot
// ranges and the entry reductions are unchanged. Called between graph launches.
qcpd_status seg_lists(qcpd_batch *h, bool all) {
    SegGrid &g = h->seg;
    const int B = h->d.B;
    if (all) {
        g.fitems = h->full_fitems; g.tunits = h->full_tunits; g.tprob = h->full_tprob;
        g.fslot = g.tslot = nullptr;
        g.nf = (int)h->h_fitems.size(); g.nt = (int)h->h_tunits.size();
        h->running_at = B;
        ++h->seg_version;
        return QCPD_OK;
    }
    BCHK(hipMemcpyAsync(h->host_st.data(), h->stl[0], sizeof(LsqrState) * B, hipMemcpyDeviceToHost,
                        h->stream));
    BCHK(hipStreamSynchronize(h->stream));
    std::vector<SegItem> fi;
    std::vector<Unit> tu;
    std::vector<int> tp, fs, ts;
    int running = 0;
    for (int b = 0; b < B; ++b) running += h->host_st[b].done ? 0 : 1;
    for (size_t i = 0; i < h->h_fitems.size(); ++i)
        if (!h->host_st[h->h_fitems[i].prob].done) { fi.push_back(h->h_fitems[i]); fs.push_back((int)i); }
    for (size_t i = 0; i < h->h_tunits.size(); ++i)
        if (!h->host_st[h->h_tprob[i]].done) {
            tu.push_back(h->h_tunits[i]); tp.push_back(h->h_tprob[i]); ts.push_back((int)i);
        }
    if (fi.empty() || tu.empty()) return QCPD_OK;  // nothing runs: the caller stops
    BCHK(hipMemcpyAsync(h->c_fitems, fi.data(), sizeof(SegItem) * fi.size(), hipMemcpyHostToDevice, h->stream));
    BCHK(hipMemcpyAsync(h->c_fslot, fs.data(), sizeof(int) * fs.size(), hipMemcpyHostToDevice, h->stream));
    BCHK(hipMemcpyAsync(h->c_tunits, tu.data(), sizeof(Unit) * tu.size(), hipMemcpyHostToDevice, h->stream));
    BCHK(hipMemcpyAsync(h->c_tprob, tp.data(), sizeof(int) * tp.size(), hipMemcpyHostToDevice, h->stream));
    BCHK(hipMemcpyAsync(h->c_tslot, ts.data(), sizeof(int) * ts.size(), hipMemcpyHostToDevice, h->stream));
    BCHK(hipStreamSynchronize(h->stream));  // the host vectors go out of scope
    g.fitems = h->c_fitems; g.fslot = h->c_fslot; g.nf = (int)fi.size();
    g.tunits = h->c_tunits; g.tprob = h->c_tprob; g.tslot = h->c_tslot; g.nt = (int)tu.size();
    h->running_at = running;
    ++h->seg_version;
    return QCPD_OK;
}

// Iterations per graph launch of the segmented loop: at most 32, so the host can shrink the
// launch lists (and stop) soon after problems finish (measured: 32 beats 128 here, while
// the single-problem loop prefers 128).
constexpr int kSegChunkMax = 32;

qcpd_status seg_graph(qcpd_batch *h, int dir) {
    const int chunk = std::min(kSegChunkMax, std::max(1, h->opts.graph_chunk));
    if (h->graph[dir] && h->graph_chunk[dir] == chunk && h->graph_sc[dir] == h->d.sc &&
        h->graph_scl[dir] == h->d.scl && h->graph_version[dir] == h->seg_version)
        return QCPD_OK;
    if (h->graph[dir]) {
        (void)hipGraphExecDestroy(h->graph[dir]);
        h->graph[dir] = nullptr;
    }
    hipGraph_t g = nullptr;
    BCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < chunk; ++i) enqueue_seg_iteration(h, dir, h->cap);
    BCHK(hipStreamEndCapture(h->cap, &g));
    const hipError_t e = hipGraphInstantiate(&h->graph[dir], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph[dir] = nullptr;
        return QCPD_ERR_HIP;
    }
    h->graph_chunk[dir] = chunk;
    h->graph_sc[dir] = h->d.sc;
    h->graph_scl[dir] = h->d.scl;
    h->graph_version[dir] = h->seg_version;
    return QCPD_OK;
}

qcpd_status batch_run(qcpd_batch *h, int dir, const double *i0, const double *i1, const double *i2,
                      const double *i3, double *o0, double *o1, double *o2, double *o3,
                      qcpd_info *info) {
    hipStream_t s = h->stream;
    BCHK(hipEventRecord(h->ev0, s));
    switch (h->opts.precond) {  // as the single-problem path: the VJP swaps the two sides
    case QCPD_PRECOND_JACOBI: h->d.sc = h->scale[dir]; h->d.scl = nullptr; break;
    case QCPD_PRECOND_EQUIL: h->d.sc = h->equil[dir]; h->d.scl = h->equil[1 - dir]; break;
    default: h->d.sc = nullptr; h->d.scl = nullptr; break;
    }
    h->d.tol = h->opts.tol;
    h->d.max_iter = h->opts.max_iter;
    qcpd_status rc = seg_bake(h);
    if (rc != QCPD_OK) return rc;
    rc = seg_lists(h, true);
    if (rc != QCPD_OK) return rc;
    rc = seg_graph(h, dir);
    if (rc != QCPD_OK) return rc;
    BCHK(hipMemsetAsync(h->d.queue, 0, 2 * sizeof(int), s));
    BCHK(hipMemsetAsync(h->seg.ndone, 0, sizeof(int), s));
    BCHK(hipMemsetAsync(h->d.prev_rel, 0, sizeof(double) * h->d.B, s));
    hipLaunchKernelGGL(k_batch_begin, dim3(h->grid), dim3(kBlock), h->lds, s, h->d, dir, i0, i1, i2,
                       i3, h->stl[0], h->seg.ndone);
    BCHK(hipGetLastError());
    // iterate until every problem's LSQR has stopped (each stops by its own iteration cap at
    // the latest)
    long long cap_iter = 0;
    for (int b = 0; b < h->d.B; ++b)
        cap_iter = std::max<long long>(cap_iter, h->opts.max_iter > 0 ? h->opts.max_iter : 100LL * h->nb_rows[b]);
    const long long max_launch = cap_iter / h->graph_chunk[dir] + 4;
    for (int round = 0;; ++round) {
        for (long long l = 0;; ++l) {
            BCHK(hipMemcpyAsync(h->host_ndone, h->seg.ndone, sizeof(int), hipMemcpyDeviceToHost, s));
            BCHK(hipStreamSynchronize(s));
            if (*h->host_ndone >= h->d.B || l >= max_launch) break;
            // once half of the problems launched for have stopped, launch only the rest
            if (2 * (h->d.B - *h->host_ndone) <= h->running_at) {
                rc = seg_lists(h, false);
                if (rc == QCPD_OK) rc = seg_graph(h, dir);
                if (rc != QCPD_OK) return rc;
            }
            BCHK(hipGraphLaunch(h->graph[dir], s));
        }
        BCHK(hipMemsetAsync(h->d.queue + 1, 0, sizeof(int), s));
        BCHK(hipMemsetAsync(h->d.nresumed, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_batch_end, dim3(h->grid), dim3(kBlock), h->lds, s, h->d, dir, o0, o1,
                           o2, o3, h->stl[0], h->stl[1], round > 0 ? 1 : 0, round < 8 ? 1 : 0);
        BCHK(hipGetLastError());
        BCHK(hipMemcpyAsync(h->host_ndone, h->d.nresumed, sizeof(int), hipMemcpyDeviceToHost, s));
        BCHK(hipStreamSynchronize(s));
        const int resumed = *h->host_ndone;
        if (resumed == 0) break;
        *h->host_ndone = h->d.B - resumed;  // the resumed problems count as running again
        BCHK(hipMemcpyAsync(h->seg.ndone, h->host_ndone, sizeof(int), hipMemcpyHostToDevice, s));
        rc = seg_lists(h, false);
        if (rc == QCPD_OK) rc = seg_graph(h, dir);
        if (rc != QCPD_OK) return rc;
    }
    BCHK(hipEventRecord(h->ev1, s));
    BCHK(hipMemcpyAsync(h->host_st.data(), h->st, sizeof(LsqrState) * h->d.B, hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    hipEventElapsedTime(&ms, h->ev0, h->ev1);
    bool all_conv = true;
    for (int b = 0; b < h->d.B; ++b) {
        const LsqrState &st = h->host_st[b];
        // converged: LSQR stopped on its test AND the recomputed unscaled residual meets tol
        const double rel = st.tau_rhs > 0.0 ? st.resid / st.tau_rhs : 0.0;
        const bool conv = st.conv && !(h->opts.tol > 0.0 && !(rel <= h->opts.tol));
        all_conv = all_conv && conv;
        if (info) {
            info[b].iters = st.iters;
            info[b].est_residual = st.beta1 > 0.0 ? st.phibar / st.beta1 : 0.0;
            info[b].rel_residual = rel;
            info[b].flags = (conv ? 0u : 1u) | h->create_flags;
            info[b].ms_total = ms;
        }
    }
    return all_conv ? QCPD_OK : QCPD_WARN_NOT_CONVERGED;
}

}  // namespace

extern "C" {

qcpd_status qcpd_batch_create(qcpd_batch **out, const qcpd_batch_layout *L, const int32_t *P_rowptr,
                              const int32_t *P_colind, const double *P_val, const int32_t *A_rowptr,
                              const int32_t *A_colind, const double *A_val, const double *q,
                              const double *b, const double *x, const double *y, const double *s,
                              const qcpd_opts *opts, void *stream) {
    if (!out) return QCPD_ERR_INVALID_ARG;
    *out = nullptr;
    if (!L || L->nprob < 1 || !L->n || !L->m || !L->nnz_P || !L->nnz_A || !L->cones)
        return QCPD_ERR_INVALID_ARG;
    if (!P_rowptr || !A_rowptr || !q || !x) return QCPD_ERR_INVALID_ARG;
    long long sn = 0, sm = 0, sp = 0, sa = 0;
    for (int i = 0; i < L->nprob; ++i) {
        const qcpd_cones &K = L->cones[i];
        if (L->n[i] < 1 || L->m[i] < 0 || L->nnz_P[i] < 0 || L->nnz_A[i] < 0) return QCPD_ERR_INVALID_ARG;
        if (K.n_zero < 0 || K.n_nonneg < 0 || K.n_soc < 0 || K.n_psd < 0 || K.n_exp < 0) return QCPD_ERR_CONE;
        if (K.n_pow != 0 || K.n_dpow != 0) return QCPD_ERR_CONE;  // single-problem path only
        if ((K.n_soc > 0 && !K.soc_dims) || (K.n_psd > 0 && !K.psd_orders)) return QCPD_ERR_CONE;
        long long rows = (long long)K.n_zero + K.n_nonneg + 3LL * K.n_exp;
        for (int j = 0; j < K.n_soc; ++j) {
            if (K.soc_dims[j] < 1 || K.soc_dims[j] > kUnitRows) return QCPD_ERR_CONE;
            rows += K.soc_dims[j];
        }
        for (int j = 0; j < K.n_psd; ++j) {
            const int k = K.psd_orders[j];
            if (k < 1 || k > kMaxPsd) return QCPD_ERR_CONE;
            rows += (long long)k * (k + 1) / 2;
        }
        if (rows != L->m[i]) return QCPD_ERR_CONE;
        sn += L->n[i]; sm += L->m[i]; sp += L->nnz_P[i]; sa += L->nnz_A[i];
    }
    if (sn + sm + L->nprob >= (1LL << 31) || sp >= (1LL << 31) || sa >= (1LL << 31)) return QCPD_ERR_DIM;
    if ((sp > 0 && (!P_colind || !P_val)) || (sa > 0 && (!A_colind || !A_val))) return QCPD_ERR_INVALID_ARG;
    if (sm > 0 && (!b || !y || !s)) return QCPD_ERR_INVALID_ARG;
    qcpd_opts o;
    qcpd_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.tol >= 0.0) || o.max_iter < 0 ||
        (o.precond != QCPD_PRECOND_NONE && o.precond != QCPD_PRECOND_JACOBI &&
         o.precond != QCPD_PRECOND_EQUIL) || o.graph_chunk < 1 || o.graph_chunk > 4096 ||
        o.solver != QCPD_SOLVER_LSQR)
        return QCPD_ERR_INVALID_ARG;
    qcpd_batch *h = new (std::nothrow) qcpd_batch();
    if (!h) return QCPD_ERR_OOM;
    h->opts = o;
    h->stream = static_cast<hipStream_t>(stream);
    if (hipHostMalloc((void **)&h->host_flag, 8 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
        free_batch(h);
        return QCPD_ERR_HIP;
    }
    qcpd_status rc = batch_create_impl(h, L, P_rowptr, P_colind, P_val, A_rowptr, A_colind, A_val,
                                       q, b, x, y, s);
    if (rc < 0) {
        hipStreamSynchronize(h->stream);
        free_batch(h);
        return rc;
    }
    *out = h;
    return rc;
}

qcpd_status qcpd_batch_jvp(qcpd_batch *h, const double *dP, const double *dA, const double *dq,
                           const double *db, double *dx, double *dy, double *ds, qcpd_info *info) {
    if (!h || (h->nnzP && !dP) || (h->nnzA && !dA) || !dq || !dx) return QCPD_ERR_INVALID_ARG;
    if (h->d.p.m && (!db || !dy || !ds)) return QCPD_ERR_INVALID_ARG;
    return batch_run(h, 0, dP, dA, dq, db, dx, dy, ds, nullptr, info);
}

qcpd_status qcpd_batch_vjp(qcpd_batch *h, const double *gx, const double *gy, const double *gs,
                           double *dP, double *dA, double *dq, double *db, qcpd_info *info) {
    if (!h || !gx || !dq || (h->nnzP && !dP) || (h->nnzA && !dA)) return QCPD_ERR_INVALID_ARG;
    if (h->d.p.m && (!gy || !gs || !db)) return QCPD_ERR_INVALID_ARG;
    return batch_run(h, 1, gx, gy, gs, nullptr, dP, dA, dq, db, info);
}

qcpd_status qcpd_batch_set_opts(qcpd_batch *h, const qcpd_opts *opts) {
    if (!h || !opts || !(opts->tol >= 0.0) || opts->max_iter < 0 ||
        (opts->precond != QCPD_PRECOND_NONE && opts->precond != QCPD_PRECOND_JACOBI &&
         opts->precond != QCPD_PRECOND_EQUIL) || opts->graph_chunk < 1 || opts->graph_chunk > 4096 ||
        opts->solver != QCPD_SOLVER_LSQR)
        return QCPD_ERR_INVALID_ARG;
    h->opts = *opts;
    return QCPD_OK;
}

qcpd_status qcpd_batch_set_launch(qcpd_batch *h, int32_t grid) {
    if (!h || grid < 0) return QCPD_ERR_INVALID_ARG;
    h->grid = grid ? std::min(grid, h->d.B) : h->grid_default;
    return QCPD_OK;
}

qcpd_status qcpd_batch_get_launch(qcpd_batch *h, int32_t *out) {
    if (!h || !out) return QCPD_ERR_INVALID_ARG;
    out[0] = h->grid;
    out[1] = h->grid_default;
    return QCPD_OK;
}

void qcpd_batch_destroy(qcpd_batch *h) {
    if (!h) return;
    hipStreamSynchronize(h->stream);
    free_batch(h);
}

}  // extern "C"
