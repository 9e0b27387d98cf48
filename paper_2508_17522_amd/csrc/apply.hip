// Hot-path kernels of the derivative evaluation: the products with F and F' that LSQR
// needs (Sec. 3.1 / 3.2), the cone Jacobian-vector products (Appendix A), and the maps
// into and out of the least-squares problems.
//
// F = D_u Q(Pi z) DPi(z) - DPi(z) + I at z_N = 1 (Sec. 2.4), with
//   D_u Q w = (P w_x + A' w_y + q w_N,  -A w_x + b w_N,  c'w_x - b'w_y + x'Px w_N),
//   c = -2Px - q,  DPi = blockdiag(I_n, J, 1),  J = DPi_{K*}(z_y).
// So F v = (P v_x + A'(J v_y) + q v_N,
//           -A v_x + b v_N - J v_y + v_y,
//           c'v_x - b'(J v_y) + x'Px v_N)
// and  F'r = (P r_x - A'r_y + c r_N,
//             J(A r_x - b r_N - r_y) + r_y,
//             q'r_x + b'r_y + x'Px r_N).
//
// The kernels here serve the steps outside the LSQR loop (its first product, the explicit
// residual, the persistent driver): one product with F over CSR rows (k_rows_F) and one
// fused product with F' in which each workgroup forms the rows of a work unit and applies
// that unit's block of J in LDS (k_fused_FT). The J needed by the next product with F is
// applied inside the fused product (block-local), and the tau-row dot products of each
// product are accumulated by the kernel that produces its input. The loop itself runs the
// latency-overlapped kernels of loop.hip.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "cone_jv.h"
#include "lsqr_dev.h"
#include "qcpd_internal.h"

namespace qcpd {

namespace cg = cooperative_groups;

// ---------------------------------------------------------------------------------------
// product with F: CSR rows
// ---------------------------------------------------------------------------------------

// The rows of one virtual workgroup `vb` of the product with F: x rows (P and A'), then y
// rows and the tau row (A). Accumulates ||out||^2 (s0) and the F' tau-row dot (s1).
__device__ inline void rows_F_vblock(const Problem &p, const StepArgs &a, const Ctx &c,
                                     const RowGrid &g, int vb, double &s0, double &s1) {
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
            for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L)
                acc += p.Pv[k] * ldin(a, c, p.Pci[k]);
            for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L)
                accT += p.Tv[t] * a.wy[p.Tci[t]];
            idx = row;
        }
    } else {
        if (row < m) {
            for (int k = p.Arp[row] + lane; k < p.Arp[row + 1]; k += L)
                acc += p.Av[k] * ldin(a, c, p.Aci[k]);
            idx = n + row;
        } else if (row == m) {
            idx = N - 1;
        }
    }
    acc = group_sum(acc, L);
    accT = group_sum(accT, L);
    if (lane == 0 && idx >= 0) {
        double val;
        if (idx < n) {
            val = acc + accT * c.inv + p.q[idx] * c.in_N;
        } else if (idx < N - 1) {
            const int r = idx - n;
            val = -acc + p.b[r] * c.in_N - a.wy[r] * c.inv + ldin(a, c, idx);
        } else {
            val = a.st->dot_fwd * c.inv + p.xPx * c.in_N;
        }
        const double o = role_value(a, c, idx, val);
        a.out[idx] = o;
        s0 += o * o;
        if (a.role == ROLE_RESID) {
            s1 += a.rhs[idx] * a.rhs[idx];  // for the unscaled relative residual
        } else {
            const double nsc = nscale(c, idx);
            if (idx < n) s1 += p.q[idx] * nsc * o;
            else if (idx < N - 1) s1 += p.b[idx - n] * nsc * o;
        }
        if (a.do_update) lsqr_update(a, c, idx);
    }
}

__global__ __launch_bounds__(kBlock) void k_rows_F(Problem p, StepArgs a, RowGrid g) {
    LsqrState *st = a.st;
    if (a.check_done && st->done) return;
    const Ctx c = make_ctx(a, p.N - 1);
    double s0 = 0.0, s1 = 0.0;
    rows_F_vblock(p, a, c, g, blockIdx.x, s0, s1);
    double tot[3];
    if (last_block_sum3(s0, s1, 0.0, a.partials, a.counter, gridDim.x, tot) && threadIdx.x == 0)
        finalize(st, a.role, tot[0], tot[1], false);
}

// ---------------------------------------------------------------------------------------
// product with F', fused: each workgroup forms the rows of D_u Q'r for one work unit and
// applies that unit's block of J in LDS, so no launch boundary separates the two halves:
//   x rows:  (F'r)_x = P r_x - A'r_y + c r_N
//   y rows:  t = A r_x - b r_N - r_y,  (F'r)_y = J t + r_y      (per cone block)
//   tau:     (F'r)_N = q'r_x + b'r_y + x'Px r_N                  (dot accumulated earlier)
// then the LSQR role update and, when asked, the J of the next product with F.
// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_fused_FT(Problem p, StepArgs a, FusedGrid g) {
    extern __shared__ double sm[];
    LsqrState *st = a.st;
    if (a.check_done && st->done) return;
    const int N = p.N;
    const Ctx c = make_ctx(a, N - 1);
    const int tid = threadIdx.x;
    double s0 = 0.0, s1 = 0.0;
    fused_unit(p, a, c, g.lx, g.ly, g.units[blockIdx.x], sm, s0, s1);
    if (blockIdx.x == 0 && tid == 0) {  // the tau entry
        const double o = role_value(a, c, N - 1, st->dot_adj * c.inv + p.xPx * c.in_N);
        a.out[N - 1] = o;
        s0 += o * o;
        if (a.role == ROLE_RESID) s1 += a.rhs[N - 1] * a.rhs[N - 1];
        if (a.do_update) lsqr_update(a, c, N - 1);
    }
    double tot[3];
    if (last_block_sum3(s0, s1, 0.0, a.partials, a.counter, gridDim.x, tot) && tid == 0)
        finalize(st, a.role, tot[0], tot[1], true);
}

void set_fused_kernel_lds(int bytes) {
    (void)hipFuncSetAttribute((const void *)k_fused_FT, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

int fused_lds_bytes(int kmax) {
    const int psd = kmax > 0 ? (3 * kmax * (kmax | 1) + kmax * (kmax + 1)) : 0;
    return (int)sizeof(double) * std::max(2 * kUnitRows, psd);
}

// ---------------------------------------------------------------------------------------
// The whole LSQR loop in one cooperative launch. Each iteration is two phases (the product
// with F over CSR rows, the fused product with F'), each ending in one grid barrier. After a
// barrier every workgroup reduces the per-block partial sums in the same fixed order and runs
// the same LSQR scalar update into its own LDS copy of the state, so the copies stay
// identical without a second barrier. Partials are double-buffered by phase: a block can only
// overwrite a buffer after the next barrier, by which time every block has read it.
// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_lsqr_persistent(Problem p, StepArgs fa, StepArgs ta,
                                                            RowGrid rg, FusedGrid fg, int dir,
                                                            LsqrState *gst, double *partials) {
    extern __shared__ double sm[];
    __shared__ LsqrState S;
    cg::grid_group grid = cg::this_grid();
    const int tid = threadIdx.x, G = gridDim.x, N = p.N;
    if (tid == 0) S = *gst;
    __syncthreads();
    fa.st = &S;
    ta.st = &S;
    while (!S.done) {
        for (int phase = 0; phase < 2; ++phase) {
            const bool isF = (dir == 0) ? (phase == 0) : (phase == 1);
            const StepArgs &a = isF ? fa : ta;
            const Ctx c = make_ctx(a, N - 1);
            double s0 = 0.0, s1 = 0.0, z = 0.0;
            if (isF) {
                for (int vb = blockIdx.x; vb < rg.bx + rg.by; vb += G) rows_F_vblock(p, a, c, rg, vb, s0, s1);
            } else {
                for (int ui = blockIdx.x; ui < fg.nunits; ui += G) {
                    fused_unit(p, a, c, fg.lx, fg.ly, fg.units[ui], sm, s0, s1);
                    __syncthreads();
                }
                if (blockIdx.x == 0 && tid == 0) {
                    const double o = role_value(a, c, N - 1, S.dot_adj * c.inv + p.xPx * c.in_N);
                    a.out[N - 1] = o;
                    s0 += o * o;
                    if (a.do_update) lsqr_update(a, c, N - 1);
                }
            }
            block_sum3(s0, s1, z);
            double *buf = partials + (size_t)phase * 3 * G;
            if (tid == 0) {
                store_coherent(&buf[3 * blockIdx.x], s0);
                store_coherent(&buf[3 * blockIdx.x + 1], s1);
            }
            grid.sync();
            double t0 = 0.0, t1 = 0.0, t2 = 0.0;
            for (int i = tid; i < G; i += kBlock) {
                t0 += load_coherent(&buf[3 * i]);
                t1 += load_coherent(&buf[3 * i + 1]);
            }
            block_sum3(t0, t1, t2);
            if (tid == 0) {
                const double tot[3] = {t0, t1, 0.0};
                finalize(&S, a.role, tot[0], tot[1], !isF);
            }
            __syncthreads();
            if (S.done) break;
        }
    }
    if (blockIdx.x == 0 && tid == 0) *gst = S;
}

int persistent_blocks_per_cu(int lds_bytes) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_lsqr_persistent, kBlock,
                                                     lds_bytes) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_lsqr_persistent(const Problem &p, const StepArgs &fa, const StepArgs &ta,
                                  const RowGrid &rg, const FusedGrid &fg, int dir, LsqrState *st,
                                  double *partials, int grid, int lds, hipStream_t s) {
    Problem pp = p;
    StepArgs f = fa, t = ta;
    RowGrid r = rg;
    FusedGrid u = fg;
    void *args[] = {&pp, &f, &t, &r, &u, &dir, &st, &partials};
    (void)hipFuncSetAttribute((const void *)k_lsqr_persistent, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return hipLaunchCooperativeKernel((const void *)k_lsqr_persistent, dim3(grid), dim3(kBlock), args,
                                      (unsigned)lds, s);
}

// wy = J(s o in_y) (raw, no normaliser) and dot_fwd = c'(s o in)_x - b'wy, for a product
// with F whose input was not produced by cone_FT.
__global__ __launch_bounds__(kBlock) void k_cone_pre(Problem p, StepArgs a, ConeGrid g) {
    extern __shared__ double sm[];
    LsqrState *st = a.st;
    if (a.check_done && st->done) return;
    const int n = p.n, N = p.N;
    const int tid = threadIdx.x;
    const double *isc = a.in_is_v ? a.sc : a.scl;
    auto ld = [&](int idx) { return isc ? isc[idx] * a.in[idx] : a.in[idx]; };
    double s1 = 0.0;
    const int bid = blockIdx.x;
    if (bid < g.bE) {
        const int e = bid * kBlock + tid;
        if (e < g.nE - 1) {
            if (e < n) {
                s1 += p.c[e] * ld(e);
            } else {
                const int r = e - n;
                const double w = p.jdiag[r] * ld(e);
                a.wy[r] = w;
                s1 -= p.b[r] * w;
            }
        }
    } else if (bid < g.bE + g.bS) {
        const int cone = (bid - g.bE) * kBlock + tid;
        if (cone < p.n_soc)
            soc_jv(p, cone, [&](int r) { return ld(n + r); },
                   [&](int r, double w) { a.wy[r] = w; s1 -= p.b[r] * w; });
    } else if (bid < g.bE + g.bS + g.bX) {
        const int cone = (bid - g.bE - g.bS) * kBlock + tid;
        if (cone < p.n_exp)
            exp_jv(p, cone, [&](int r) { return ld(n + r); },
                   [&](int r, double w) { a.wy[r] = w; s1 -= p.b[r] * w; });
    } else {
        const int cone = bid - g.bE - g.bS - g.bX;
        psd_jv(p, cone, sm, [&](int r) { return ld(n + r); },
               [&](int r, double w) { a.wy[r] = w; s1 -= p.b[r] * w; });
    }
    (void)N;
    double tot[3];
    if (last_block_sum3(0.0, s1, 0.0, a.partials, a.counter, gridDim.x, tot) && tid == 0)
        st->dot_fwd = tot[1];
}

// ---------------------------------------------------------------------------------------
// LSQR start / finish
// ---------------------------------------------------------------------------------------

__global__ void k_state_init(LsqrState *st, double tol, int max_iter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        LsqrState s = {};
        s.one = 1.0;
        s.tol = tol;
        s.max_iter = max_iter;
        s.pend_role = -1;
        *st = s;
    }
}

__global__ void k_fill(double *p, long long n, double v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Apply the owed x update, map the LSQR iterate back through the diagonal scale
// (sol = sc o x), and accumulate q'sol_x + b'sol_y for a following product with F'.
__global__ __launch_bounds__(kBlock) void k_flush(Problem p, StepArgs a, double *sol) {
    LsqrState *st = a.st;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool pend = st->pending != 0;
    const double phr = st->phr;
    double s1 = 0.0;
    if (i < p.N) {
        double x = a.xk[i];
        if (pend) x += phr * a.wk[i];
        a.xk[i] = x;
        const double v = a.sc ? a.sc[i] * x : x;
        sol[i] = v;
        if (i < p.n) s1 = p.q[i] * v;
        else if (i < p.N - 1) s1 = p.b[i - p.n] * v;
    }
    double tot[3];
    if (last_block_sum3(0.0, s1, 0.0, a.partials, a.counter, gridDim.x, tot) && threadIdx.x == 0) {
        st->pending = 0;
        (a.st_next ? a.st_next : st)->dot_adj = tot[1];  // for a product with F' at sol
    }
}

// q'in_x + b'in_y (the tau-row dot of a product with F' at `in`) into st->dot_adj.
__global__ __launch_bounds__(kBlock) void k_adj_dot(Problem p, StepArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double s1 = 0.0;
    if (i < p.n) s1 = p.q[i] * a.in[i];
    else if (i < p.N - 1) s1 = p.b[i - p.n] * a.in[i];
    double tot[3];
    if (last_block_sum3(0.0, s1, 0.0, a.partials, a.counter, gridDim.x, tot) && threadIdx.x == 0)
        a.st->dot_adj = tot[1];
}

// JVP right-hand side (Sec. 2.4, D_theta N at z_N = 1, Pi z = (x, y, 1)):
//   d = (dP x + dA'y + dq,  -dA x + db,  -x'dP x - dq'x - db'y);
// LSQR starts from u~ = -d (also kept in rhs for the explicit residual).
__global__ __launch_bounds__(kBlock) void k_jvp_rhs(Problem p, StepArgs a, RowGrid g,
                                                    const double *dP, const double *dA,
                                                    const double *dq, const double *db) {
    LsqrState *st = a.st;
    const int n = p.n, m = p.m, N = p.N;
    const int tid = threadIdx.x;
    const bool xr = blockIdx.x < (unsigned)g.bx;
    const int L = xr ? g.lx : g.ly;
    const long long gt = (long long)(xr ? blockIdx.x : blockIdx.x - g.bx) * kBlock + tid;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    double acc = 0.0, accT = 0.0;
    int idx = -1;
    if (xr) {
        if (row < n) {
            for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) acc += dP[k] * p.x[p.Pci[k]];
            for (int t = p.Trp[row] + lane; t < p.Trp[row + 1]; t += L)
                accT += dA[p.Tperm[t]] * p.y[p.Tci[t]];
            idx = row;
        }
    } else if (row < m) {
        for (int k = p.Arp[row] + lane; k < p.Arp[row + 1]; k += L) acc += dA[k] * p.x[p.Aci[k]];
        idx = n + row;
    }
    acc = group_sum(acc, L);
    accT = group_sum(accT, L);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (lane == 0 && idx >= 0) {
        double o;
        if (idx < n) {
            o = -(acc + accT + dq[idx]);
            s1 = p.q[idx] * o;
            s2 = p.x[idx] * acc + dq[idx] * p.x[idx];
        } else {
            const int r = idx - n;
            o = -(-acc + db[r]);
            s1 = p.b[r] * o;
            s2 = db[r] * p.y[r];
        }
        // LSQR starts from u~ = L(-d) (L = scl, the row scale); the unscaled -d is kept for
        // the explicit residual
        const double l = a.scl ? a.scl[idx] : 1.0;
        a.out[idx] = l * o;
        const_cast<double *>(a.rhs)[idx] = o;
        s0 = l * o * l * o;
        s1 *= l * l;
    }
    double tot[3];
    if (last_block_sum3(s0, s1, s2, a.partials, a.counter, gridDim.x, tot) && tid == 0) {
        const double oN = tot[2];  // -d_N = x'dP x + dq'x + db'y
        const double lN = a.scl ? a.scl[N - 1] : 1.0;
        a.out[N - 1] = lN * oN;
        const_cast<double *>(a.rhs)[N - 1] = oN;
        const double beta = sqrt(tot[0] + lN * oN * lN * oN);
        st->beta = beta;
        st->beta1 = beta;
        st->phibar = beta;
        st->dot_adj = tot[1];
        if (!(beta > 0.0)) { st->done = 1; st->conv = 1; }
    }
}

// VJP right-hand side (Sec. 3.2): dz = D phi'(gx, gy, gs)
//   = (gx, J(gy + gs) - gs, -x'gx - y'gy - s'gs); LSQR starts from u~ = -dz.
__global__ __launch_bounds__(kBlock) void k_vjp_rhs(Problem p, StepArgs a, ConeGrid g,
                                                    const double *gx, const double *gy,
                                                    const double *gs) {
    extern __shared__ double sm[];
    LsqrState *st = a.st;
    const int n = p.n, N = p.N;
    const int tid = threadIdx.x;
    double *rhs = const_cast<double *>(a.rhs);
    double s0 = 0.0, s2 = 0.0;
    auto put = [&](int idx, double o) {
        const double l = a.scl ? a.scl[idx] : 1.0;  // scaled LSQR start, unscaled copy
        a.out[idx] = l * o;
        rhs[idx] = o;
        s0 += l * o * l * o;
    };
    auto gsum = [&](int r) { return gy[r] + gs[r]; };
    auto yout = [&](int r, double jt) {
        put(n + r, -(jt - gs[r]));
        s2 += p.y[r] * gy[r] + p.s[r] * gs[r];
    };
    const int bid = blockIdx.x;
    if (bid < g.bE) {
        const int e = bid * kBlock + tid;
        if (e < g.nE - 1) {
            if (e < n) {
                put(e, -gx[e]);
                s2 += p.x[e] * gx[e];
            } else {
                const int r = e - n;
                yout(r, p.jdiag[r] * gsum(r));
            }
        }
    } else if (bid < g.bE + g.bS) {
        const int cone = (bid - g.bE) * kBlock + tid;
        if (cone < p.n_soc) soc_jv(p, cone, gsum, yout);
    } else if (bid < g.bE + g.bS + g.bX) {
        const int cone = (bid - g.bE - g.bS) * kBlock + tid;
        if (cone < p.n_exp) exp_jv(p, cone, gsum, yout);
    } else {
        const int cone = bid - g.bE - g.bS - g.bX;
        psd_jv(p, cone, sm, gsum, yout);
    }
    double tot[3];
    if (last_block_sum3(s0, 0.0, s2, a.partials, a.counter, gridDim.x, tot) && tid == 0) {
        const double oN = tot[2];  // -dz_N
        const double lN = a.scl ? a.scl[N - 1] : 1.0;
        a.out[N - 1] = lN * oN;
        rhs[N - 1] = oN;
        const double beta = sqrt(tot[0] + lN * oN * lN * oN);
        st->beta = beta;
        st->beta1 = beta;
        st->phibar = beta;
        if (!(beta > 0.0)) { st->done = 1; st->conv = 1; }
    }
}

// JVP output (Sec. 3.1): dx = dz_x - dz_N x, dy = J dz_y - dz_N y,
// ds = J dz_y - dz_y - dz_N s; jdz = J dz_y precomputed.
__global__ __launch_bounds__(kBlock) void k_jvp_out(Problem p, const double *sol,
                                                    const double *jdz, double *dx, double *dy,
                                                    double *ds) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int n = p.n, m = p.m;
    const double dzN = sol[p.N - 1];
    if (i < n) {
        dx[i] = sol[i] - dzN * p.x[i];
    } else if (i < n + m) {
        const int r = i - n;
        dy[r] = jdz[r] - dzN * p.y[r];
        ds[r] = jdz[r] - sol[i] - dzN * p.s[r];
    }
}

// VJP output (Sec. 3.2, tau = 1), on the stored patterns of P and A:
//   dP_ij = 1/2 (w_i x_j + x_i w_j) - w_N x_i x_j,  dA_ij = y_i w_j - w_{n+i} x_j,
//   dq = w_x - w_N x,  db = w_y - w_N y.
__global__ __launch_bounds__(kBlock) void k_vjp_out(Problem p, RowGrid g, const double *w,
                                                    double *dP, double *dA, double *dq,
                                                    double *db) {
    const int n = p.n, m = p.m;
    const int tid = threadIdx.x;
    const bool xr = blockIdx.x < (unsigned)g.bx;
    const int L = xr ? g.lx : g.ly;
    const long long gt = (long long)(xr ? blockIdx.x : blockIdx.x - g.bx) * kBlock + tid;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    const double wN = w[p.N - 1];
    if (xr) {
        if (row < n) {
            const double wi = w[row], xi = p.x[row];
            for (int k = p.Prp[row] + lane; k < p.Prp[row + 1]; k += L) {
                const int j = p.Pci[k];
                const double xj = p.x[j];
                dP[k] = 0.5 * (wi * xj + xi * w[j]) - wN * xi * xj;
            }
            if (lane == 0) dq[row] = wi - wN * xi;
        }
    } else if (row < m) {
        const double yi = p.y[row], wyi = w[n + row];
        for (int k = p.Arp[row] + lane; k < p.Arp[row + 1]; k += L) {
            const int j = p.Aci[k];
            dA[k] = yi * w[j] - wyi * p.x[j];
        }
        if (lane == 0) db[row] = wyi - wN * yi;
    }
}

__global__ void k_nan_scan(const double *const *ptrs, const long long *lens, int nseg,
                           int *flag) {
    for (int sgi = 0; sgi < nseg; ++sgi) {
        const double *ptr = ptrs[sgi];
        const long long len = lens[sgi];
        bool bad = false;
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len;
             i += (long long)gridDim.x * blockDim.x)
            if (!isfinite(ptr[i])) bad = true;
        if (bad) atomicOr(flag, 1);
    }
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------

void launch_rows_F(const Problem &p, const StepArgs &a, const RowGrid &g, hipStream_t s, int grid) {
    hipLaunchKernelGGL(k_rows_F, dim3(grid > 0 ? grid : g.total()), dim3(kBlock), 0, s, p, a, g);
}
void launch_fused_FT(const Problem &p, const StepArgs &a, const FusedGrid &g, int lds, hipStream_t s,
                     int grid) {
    hipLaunchKernelGGL(k_fused_FT, dim3(grid > 0 ? grid : g.nunits), dim3(kBlock), lds, s, p, a, g);
}
void launch_cone_pre(const Problem &p, const StepArgs &a, const ConeGrid &g, int lds, hipStream_t s) {
    hipLaunchKernelGGL(k_cone_pre, dim3(g.total()), dim3(kBlock), lds, s, p, a, g);
}
void launch_state_init(LsqrState *st, double tol, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, tol, max_iter);
}
void launch_fill(double *ptr, long long n, double v, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<long long>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, s, ptr, n, v);
}
void launch_adj_dot(const Problem &p, const StepArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_dot, dim3(div_up(p.N, kBlock)), dim3(kBlock), 0, s, p, a);
}
void launch_flush(const Problem &p, const StepArgs &a, double *sol, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_flush, dim3(nblk), dim3(kBlock), 0, s, p, a, sol);
}
void launch_jvp_rhs(const Problem &p, const StepArgs &a, const RowGrid &g, const double *dP,
                    const double *dA, const double *dq, const double *db, hipStream_t s) {
    hipLaunchKernelGGL(k_jvp_rhs, dim3(g.total()), dim3(kBlock), 0, s, p, a, g, dP, dA, dq, db);
}
void launch_vjp_rhs(const Problem &p, const StepArgs &a, const ConeGrid &g, int lds,
                    const double *gx, const double *gy, const double *gs, hipStream_t s) {
    hipLaunchKernelGGL(k_vjp_rhs, dim3(g.total()), dim3(kBlock), lds, s, p, a, g, gx, gy, gs);
}
void launch_jvp_out(const Problem &p, const double *sol, const double *wy, double *dx,
                    double *dy, double *ds, hipStream_t s) {
    const int nb = div_up((long long)p.n + p.m, kBlock);
    if (nb > 0) hipLaunchKernelGGL(k_jvp_out, dim3(nb), dim3(kBlock), 0, s, p, sol, wy, dx, dy, ds);
}
void launch_vjp_out(const Problem &p, const RowGrid &g, const double *w, double *dP,
                    double *dA, double *dq, double *db, hipStream_t s) {
    hipLaunchKernelGGL(k_vjp_out, dim3(g.total()), dim3(kBlock), 0, s, p, g, w, dP, dA, dq, db);
}
void launch_nan_scan(const double *const *ptrs, const long long *lens, int nseg, int *flag,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_nan_scan, dim3(256), dim3(kBlock), 0, s, ptrs, lens, nseg, flag);
}

// the cone kernels may need more than the default 64 KB of dynamic LDS for PSD blocks
void set_cone_kernel_lds(int bytes) {
    (void)hipFuncSetAttribute((const void *)k_cone_pre, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void *)k_vjp_rhs, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);

}

}  // namespace qcpd
