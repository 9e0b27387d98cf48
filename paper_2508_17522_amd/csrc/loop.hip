// The two launches of one LSQR iteration (products with F and with F', Sec. 2.4 / 3.1-3.2),
// written so that memory latency overlaps the reduction that ends the previous launch.
//
// A launch needs the LSQR scalars (alpha or beta, the plane rotation) that only the previous
// launch's partial sums determine, but nothing else it loads depends on them: the CSR sums
// of the product are linear in the input, so they are accumulated on the unnormalised input
// (the 1/alpha or 1/beta factor is applied afterwards), the cone Jacobians are linear too,
// and the operands of the role update (old output, scales, x and w of the owed update) are
// plain loads. Each workgroup therefore
//   1. issues the loads of the state and of its share of the previous launch's partials,
//   2. computes the state-free part of its first work item (CSR sums, and for cone units
//      the Jacobian applied to the raw rows, in LDS) and prefetches the update operands,
//   3. finalises the previous launch's reduction (fixed order, every workgroup the same),
//   4. finishes its work item (normalisation, role update, owed x/w update, stores), then
//      any further items it owns, and leaves its own partial sums for the next launch.
// Steps 1 and 2 run concurrently in the memory system. Cone units finish one thread per
// row, and their Jacobian applications read and write LDS only.
#include <algorithm>

#include "cone_jv.h"
#include "lsqr_dev.h"
#include "qcpd_internal.h"

namespace qcpd {

constexpr int kPartRegs = kMaxLoopGrid / kBlock;  // previous-launch partials per thread

// ---------------------------------------------------------------------------------------
// entry: state and the previous launch's partial sums
// ---------------------------------------------------------------------------------------

struct Entry {
    LsqrState st;
    double pa[kPartRegs], pb[kPartRegs];
};

// Issue the loads (values are consumed in entry_finish). The partial buffers hold
// kMaxLoopGrid slots, so the loads stay in bounds; slots beyond pend_blocks are ignored.
__device__ inline void entry_issue(const StepArgs &a, Entry &e) {
    e.st = *a.st;
#pragma unroll
    for (int j = 0; j < kPartRegs; ++j) {
        const int i = threadIdx.x + j * kBlock;
        e.pa[j] = a.part_prev[3 * i];
        e.pb[j] = a.part_prev[3 * i + 1];
    }
}

// Finalise the previous launch's reduction into S; false in every thread once LSQR stopped.
__device__ inline bool entry_finish(const StepArgs &a, const Entry &e, LsqrState *S, int my_fwd) {
    const int tid = threadIdx.x;
    if (e.st.done) {
        if (blockIdx.x == 0 && tid == 0) *a.st_next = e.st;
        return false;
    }
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    if (e.st.pend_role >= 0) {
#pragma unroll
        for (int j = 0; j < kPartRegs; ++j)
            if (tid + j * kBlock < e.st.pend_blocks) {
                t0 += e.pa[j];
                t1 += e.pb[j];
            }
        block_sum3(t0, t1, t2);
    }
    if (tid == 0) {
        LsqrState s = e.st;
        if (s.pend_role >= 0) {
            finalize(&s, s.pend_role, t0, t1, s.pend_fwd != 0);
        }
        if (s.done) {
            s.pend_role = -1;
        } else {
            s.pend_role = a.role;
            s.pend_blocks = gridDim.x;
            s.pend_fwd = my_fwd;
        }
        if (blockIdx.x == 0) {
            *a.st_next = s;
            // on the stop decision both buffers get the final state
            if (s.done) *a.st = s;
        }
        *S = s;
    }
    __syncthreads();
    return !S->done;
}

// ---------------------------------------------------------------------------------------
// state-free operands of one output entry, and its finish
// ---------------------------------------------------------------------------------------

struct Ptrs {  // scales by role; none depends on the LSQR scalars
    const double *isc, *osc, *nxs;
};

__device__ inline Ptrs ptrs_of(const StepArgs &a) {
    Ptrs q;
    q.isc = a.in_is_v ? a.sc : a.scl;
    q.osc = (a.role == ROLE_U) ? a.scl : (a.role == ROLE_V || a.role == ROLE_V0) ? a.sc : nullptr;
    q.nxs = a.out_is_v ? a.sc : a.scl;
    return q;
}

__device__ inline double in_raw(const StepArgs &a, const Ptrs &q, int j) {
    const double v = a.in[j];
    return q.isc ? v * q.isc[j] : v;
}

struct Fin {
    double out_old, osc, nxs, wk, xk, in;
};

__device__ inline void fin_load(const StepArgs &a, const Ptrs &q, int idx, Fin &f) {
    f.out_old = (a.role == ROLE_U || a.role == ROLE_V) ? a.out[idx] : 0.0;
    f.osc = q.osc ? q.osc[idx] : 1.0;
    f.nxs = q.nxs ? q.nxs[idx] : 1.0;
    if (a.do_update) {
        f.wk = a.wk[idx];
        f.xk = a.xk[idx];
        f.in = a.in[idx];
    } else {
        f.wk = f.xk = f.in = 0.0;
    }
}

// LSQR scalars of this launch, from the finalised state
__device__ inline Ctx scalars(const StepArgs &a, const LsqrState &S, const Ptrs &q,
                              double in_N_raw) {
    const double *sv = reinterpret_cast<const double *>(&S);
    Ctx c;
    c.inv = 1.0 / sv[a.in_nrm];
    c.cU = (a.role == ROLE_U) ? S.alpha / S.beta : 0.0;
    c.cV = (a.role == ROLE_V) ? S.beta / S.alpha : 0.0;
    c.inv_alpha_up = a.do_update ? 1.0 / S.alpha : 0.0;
    c.phr = S.phr;
    c.thr = S.thr;
    c.isc = q.isc;
    c.osc = q.osc;
    c.nxs = q.nxs;
    c.in_N = in_N_raw * c.inv;
    return c;
}

// role update of one entry with operator value val; returns the stored output
__device__ inline double fin_store(const StepArgs &a, const Ctx &c, int idx, const Fin &f,
                                   double val, double &s0) {
    const double sv = f.osc * val;
    double o;
    switch (a.role) {
    case ROLE_U: o = sv - c.cU * f.out_old; break;
    case ROLE_V: o = sv - c.cV * f.out_old; break;
    case ROLE_V0: o = sv; break;
    default: o = val; break;
    }
    a.out[idx] = o;
    s0 += o * o;
    if (a.do_update) {
        a.xk[idx] = f.xk + c.phr * f.wk;
        a.wk[idx] = f.in * c.inv_alpha_up - c.thr * f.wk;
    }
    return o;
}

// ---------------------------------------------------------------------------------------
// product with F over CSR rows
// ---------------------------------------------------------------------------------------

struct RowPre {
    int idx;           // output entry held by this thread (lane 0 of its row group), or -1
    double acc, accT;  // raw CSR sums: x rows P(isc o in) and A'wy; y rows A(isc o in)
    double self;       // y rows: (isc o in) at the row
    double qb;         // q (x rows) or b (y rows) at the entry
    double wyr;        // y rows: J applied to the input, at the row
    Fin f;
};

__device__ inline void rows_pre(const Problem &p, const StepArgs &a, const Ptrs &q,
                                const RowGrid &g, int vb, RowPre &r) {
    const int n = p.n, m = p.m, N = p.N;
    const int tid = threadIdx.x;
    const bool xr = vb < g.bx;
    const int L = xr ? g.lx : g.ly;
    const long long gt = (long long)(xr ? vb : vb - g.bx) * kBlock + tid;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    double acc = 0.0, accT = 0.0;
    int idx = -1;
    if (xr) {
        if (row < n) {
            const int k0 = p.Prp[row], k1 = p.Prp[row + 1];
            const int t0 = p.Trp[row], t1 = p.Trp[row + 1];
#pragma unroll 4
            for (int k = k0 + lane; k < k1; k += L) acc += p.Pv[k] * in_raw(a, q, p.Pci[k]);
#pragma unroll 4
            for (int t = t0 + lane; t < t1; t += L) accT += p.Tv[t] * a.wy[p.Tci[t]];
            idx = row;
        }
    } else {
        if (row < m) {
            const int k0 = p.Arp[row], k1 = p.Arp[row + 1];
#pragma unroll 4
            for (int k = k0 + lane; k < k1; k += L) acc += p.Av[k] * in_raw(a, q, p.Aci[k]);
            idx = n + row;
        } else if (row == m) {
            idx = N - 1;
        }
    }
    r.acc = group_sum(acc, L);
    r.accT = group_sum(accT, L);
    r.idx = (lane == 0) ? idx : -1;
    double qb = 0.0, self = 0.0, wyr = 0.0;
    if (r.idx >= 0) {
        fin_load(a, q, r.idx, r.f);
        if (r.idx < n) {
            qb = p.q[r.idx];
        } else if (r.idx < N - 1) {
            const int y = r.idx - n;
            qb = p.b[y];
            self = in_raw(a, q, r.idx);
            wyr = a.wy[y];
        }
    }
    r.qb = qb;
    r.self = self;
    r.wyr = wyr;
}

__device__ inline void rows_post(const Problem &p, const StepArgs &a, const Ctx &c,
                                 const LsqrState &S, const RowPre &r, double &s0, double &s1) {
    const int n = p.n, N = p.N;
    if (r.idx < 0) return;
    double val;
    if (r.idx < n)
        val = (r.acc + r.accT) * c.inv + r.qb * c.in_N;
    else if (r.idx < N - 1)
        val = (r.self - r.acc - r.wyr) * c.inv + r.qb * c.in_N;
    else
        val = S.dot_fwd * c.inv + p.xPx * c.in_N;
    const double o = fin_store(a, c, r.idx, r.f, val, s0);
    if (r.idx < N - 1) s1 += r.qb * r.f.nxs * o;
}

__global__ __launch_bounds__(kBlock) void k_loop_F(Problem p, StepArgs a, RowGrid g) {
    __shared__ LsqrState S;
    Entry e;
    entry_issue(a, e);
    const Ptrs q = ptrs_of(a);
    const double in_N_raw = in_raw(a, q, p.N - 1);
    RowPre r;
    rows_pre(p, a, q, g, blockIdx.x, r);
    if (!entry_finish(a, e, &S, 0)) return;
    const Ctx c = scalars(a, S, q, in_N_raw);
    double s0 = 0.0, s1 = 0.0;
    rows_post(p, a, c, S, r, s0, s1);
    for (int vb = blockIdx.x + gridDim.x; vb < g.bx + g.by; vb += gridDim.x) {
        rows_pre(p, a, q, g, vb, r);
        rows_post(p, a, c, S, r, s0, s1);
    }
    deferred_leave(a, s0, s1);
}

// ---------------------------------------------------------------------------------------
// product with F', fused with the cone Jacobians (work units as in k_fused_FT)
// ---------------------------------------------------------------------------------------

struct UnitPre {
    int idx;                   // entry of this thread (x / diagonal rows: lane 0), or -1
    double acc, accT, self, coef, jd;
    double bv;                 // cone units: b at this thread's first row
    Fin f;
};

// LDS layout of a cone unit: [PSD scratch X, T, V][tb: raw rows][rb: raw r_y, then the
// scaled outputs][jt: J applied]
__device__ inline int unit_rows(const Problem &p, const Unit &u, int &r0) {
    if (u.type == U_PSD) {
        const int k = p.psd_k[u.begin];
        r0 = p.psd_row[u.begin];
        return k * (k + 1) / 2;
    }
    r0 = u.row0;
    const int r1 = (u.type == U_SOC) ? p.soc_row[u.end - 1] + p.soc_dim[u.end - 1]
                                     : exp_row(p, u.end - 1) + 3;
    return r1 - r0;
}

__device__ inline double *unit_base(const Problem &p, const Unit &u, double *sm) {
    if (u.type == U_PSD) {
        const int k = p.psd_k[u.begin];
        return sm + psd_stage_offset(k);
    }
    return sm;
}

__device__ inline void unit_pre(const Problem &p, const StepArgs &a, const Ptrs &q, int lx,
                                int ly, const Unit &u, double *sm, double in_N_raw,
                                UnitPre &P) {
    const int n = p.n;
    const int tid = threadIdx.x;
    P.idx = -1;
    if (u.type == U_XROWS) {
        const int L = lx, lane = tid & (L - 1), row = u.begin + tid / L;
        double acc = 0.0, accT = 0.0;
        if (row < u.end) {
            const int k0 = p.Prp[row], k1 = p.Prp[row + 1];
            const int t0 = p.Trp[row], t1 = p.Trp[row + 1];
#pragma unroll 4
            for (int k = k0 + lane; k < k1; k += L) acc += p.Pv[k] * in_raw(a, q, p.Pci[k]);
#pragma unroll 4
            for (int t = t0 + lane; t < t1; t += L) accT += p.Tv[t] * in_raw(a, q, n + p.Tci[t]);
        }
        P.acc = group_sum(acc, L);
        P.accT = group_sum(accT, L);
        if (row < u.end && lane == 0) {
            P.idx = row;
            P.coef = p.c[row];
            fin_load(a, q, row, P.f);
        }
        return;
    }
    if (u.type == U_DIAG) {
        const int L = ly, lane = tid & (L - 1), r = u.begin + tid / L;
        double acc = 0.0;
        if (r < u.end) {
            const int k0 = p.Arp[r], k1 = p.Arp[r + 1];
#pragma unroll 4
            for (int k = k0 + lane; k < k1; k += L) acc += p.Av[k] * in_raw(a, q, p.Aci[k]);
        }
        P.acc = group_sum(acc, L);
        if (r < u.end && lane == 0) {
            P.idx = n + r;
            P.self = in_raw(a, q, n + r);
            P.coef = p.b[r];
            P.jd = p.jdiag[r];
            fin_load(a, q, n + r, P.f);
        }
        return;
    }
    // cone units: raw rows t = A r_x - b r_N - r_y (unnormalised) into tb, then J t into jt
    int r0;
    const int nr = unit_rows(p, u, r0);
    double *tb = unit_base(p, u, sm), *rb = tb + nr, *jt = rb + nr;
    int L = ly;
    while (L > 1 && L * nr > kBlock) L >>= 1;
    const int lane = tid & (L - 1), grp = tid / L, ngrp = kBlock / L;
    for (int i0 = 0; i0 < nr; i0 += ngrp) {
        const int i = i0 + grp, r = r0 + i;
        double acc = 0.0;
        if (i < nr) {
            const int k0 = p.Arp[r], k1 = p.Arp[r + 1];
#pragma unroll 4
            for (int k = k0 + lane; k < k1; k += L) acc += p.Av[k] * in_raw(a, q, p.Aci[k]);
        }
        acc = group_sum(acc, L);
        if (i < nr && lane == 0) {
            const double ry = in_raw(a, q, n + r);
            rb[i] = ry;
            tb[i] = acc - p.b[r] * in_N_raw - ry;
        }
    }
    if (tid < nr) {
        P.idx = n + r0 + tid;
        P.bv = p.b[r0 + tid];
        fin_load(a, q, n + r0 + tid, P.f);
    }
    __syncthreads();
    auto tin = [&](int r) { return tb[r - r0]; };
    auto jout = [&](int r, double v) { jt[r - r0] = v; };
    if (u.type == U_PSD) {
        psd_jv(p, u.begin, sm, tin, jout);  // ends with a barrier
    } else {
        const int cone = u.begin + tid;
        if (cone < u.end) {
            if (u.type == U_SOC) soc_jv(p, cone, tin, jout);
            else exp_jv(p, cone, tin, jout);
        }
        __syncthreads();
    }
}

__device__ inline void unit_post(const Problem &p, const StepArgs &a, const Ptrs &q,
                                 const Ctx &c, const Unit &u, double *sm, const UnitPre &P,
                                 double &s0, double &s1) {
    const int n = p.n;
    const int tid = threadIdx.x;
    if (u.type == U_XROWS) {
        if (P.idx >= 0) {
            const double o = fin_store(a, c, P.idx, P.f, (P.acc - P.accT) * c.inv + P.coef * c.in_N, s0);
            if (a.do_pre) s1 += P.coef * P.f.nxs * o;
        }
        return;
    }
    if (u.type == U_DIAG) {
        if (P.idx >= 0) {
            const double t = (P.acc - P.self) * c.inv - P.coef * c.in_N;
            const double o = fin_store(a, c, P.idx, P.f, P.jd * t + P.self * c.inv, s0);
            if (a.do_pre) {
                const double w = P.jd * P.f.nxs * o;
                a.wy[P.idx - n] = w;
                s1 -= P.coef * w;
            }
        }
        return;
    }
    int r0;
    const int nr = unit_rows(p, u, r0);
    double *tb = unit_base(p, u, sm), *rb = tb + nr, *jt = rb + nr;
    for (int i = tid; i < nr; i += kBlock) {
        Fin f;
        if (i == tid) f = P.f;
        else fin_load(a, q, n + r0 + i, f);
        const double o = fin_store(a, c, n + r0 + i, f, (jt[i] + rb[i]) * c.inv, s0);
        rb[i] = f.nxs * o;  // the next product's input, in place of r_y
    }
    if (!a.do_pre) return;
    __syncthreads();
    // J of the next product with F, on the scaled outputs
    auto oin = [&](int r) { return rb[r - r0]; };
    auto jout = [&](int r, double v) { jt[r - r0] = v; };
    if (u.type == U_PSD) {
        psd_jv(p, u.begin, sm, oin, jout);
    } else {
        const int cone = u.begin + tid;
        if (cone < u.end) {
            if (u.type == U_SOC) soc_jv(p, cone, oin, jout);
            else exp_jv(p, cone, oin, jout);
        }
        __syncthreads();
    }
    for (int i = tid; i < nr; i += kBlock) {
        const double w = jt[i];
        a.wy[r0 + i] = w;
        s1 -= (i == tid ? P.bv : p.b[r0 + i]) * w;
    }
}

__global__ __launch_bounds__(kBlock) void k_loop_FT(Problem p, StepArgs a, FusedGrid g) {
    extern __shared__ double sm[];
    __shared__ LsqrState S;
    Entry e;
    entry_issue(a, e);
    const Ptrs q = ptrs_of(a);
    const double in_N_raw = in_raw(a, q, p.N - 1);
    UnitPre P;
    Unit u = g.units[blockIdx.x];
    unit_pre(p, a, q, g.lx, g.ly, u, sm, in_N_raw, P);
    if (!entry_finish(a, e, &S, 1)) return;
    const Ctx c = scalars(a, S, q, in_N_raw);
    double s0 = 0.0, s1 = 0.0;
    unit_post(p, a, q, c, u, sm, P, s0, s1);
    for (int ui = blockIdx.x + gridDim.x; ui < g.nunits; ui += gridDim.x) {
        __syncthreads();  // LDS of the previous unit is free
        u = g.units[ui];
        unit_pre(p, a, q, g.lx, g.ly, u, sm, in_N_raw, P);
        unit_post(p, a, q, c, u, sm, P, s0, s1);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // the tau entry
        const int N = p.N;
        Fin f;
        fin_load(a, q, N - 1, f);
        const double o = fin_store(a, c, N - 1, f, S.dot_adj * c.inv + p.xPx * c.in_N, s0);
        (void)o;
    }
    deferred_leave(a, s0, s1);
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------

int loop_lds_bytes(int kmax) {
    const int psd = kmax > 0 ? psd_stage_offset(kmax) + 3 * (kmax * (kmax + 1) / 2) : 0;
    return (int)sizeof(double) * std::max(3 * kUnitRows, psd);
}

void set_loop_kernel_lds(int bytes) {
    (void)hipFuncSetAttribute((const void *)k_loop_FT, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void launch_loop_F(const Problem &p, const StepArgs &a, const RowGrid &g, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_loop_F, dim3(grid), dim3(kBlock), 0, s, p, a, g);
}

void launch_loop_FT(const Problem &p, const StepArgs &a, const FusedGrid &g, int lds, int grid,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_loop_FT, dim3(grid), dim3(kBlock), lds, s, p, a, g);
}

}  // namespace qcpd
