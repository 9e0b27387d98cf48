// The two launches of one LSQR iteration (products with F and with F', Sec. 2.4 / 3.1-3.2),
// written so that memory latency overlaps the reduction that ends the previous launch.
//
// A launch needs the LSQR scalars (alpha or beta, the plane rotation) that only the previous
// launch's partial sums determine, but nothing else it loads depends on them: the CSR sums
// of the product are linear in the input, so they are accumulated on the unnormalised input
// (the 1/alpha or 1/beta factor is applied afterwards), the cone Jacobians are linear too,
// and the operands of the role update (old output, scales, x and w of the owed update) are
// plain loads. Each workgroup therefore
//   1. computes the state-free part of its first work item (CSR sums, and for cone units
//      the Jacobian applied to the raw rows, in LDS) and prefetches the update operands,
//   2. issues the loads of the state and of the previous launch's partials (after the work
//      item's own loads: a wait for a load also waits for all loads issued before it, and
//      the partials, read by every workgroup, arrive last),
//   3. finalises the previous launch's reduction (fixed order, every workgroup the same),
//   4. finishes its work item (normalisation, role update, owed x/w update, stores), then
//      any further items it owns, and leaves its own partial sums for the next launch.
// Cone units finish one thread per row, and their Jacobian applications read and write LDS
// only. Where the solve has diagonal scales, the CSR values come with the input scale
// folded in, so a product reads one value per entry and gathers only the input.
#include <algorithm>

#include "cone_jv.h"
#include "lsqr_dev.h"
#include "qcpd_internal.h"

namespace qcpd {

constexpr int kPartRegs = kMaxLoopGrid / kBlock;  // previous-launch partials per thread


// ---------------------------------------------------------------------------------------
// reductions on DPP lane moves (a __shfl_xor step is an LDS permute on this GPU; a DPP move
// is a register operand modifier)
// ---------------------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xf>
__device__ inline double dpp_mov(double v) {  // lanes without a source read 0
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, true),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, true));
}

// Sum over aligned groups of L lanes (L a power of two <= 64), valid in every lane of the
// group: butterflies within a row of 16 lanes (xor 1, xor 2, half-row mirror, row mirror),
// then permutes across rows.
__device__ inline double group_sum_dpp(double v, int L) {
    if (L >= 2) v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    if (L >= 4) v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    if (L >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
    if (L >= 16) v += dpp_mov<0x140>(v);  // row_mirror
    if (L >= 32) v += __shfl_xor(v, 16);
    if (L >= 64) v += __shfl_xor(v, 32);
    return v;
}

// Sum over the wave, valid in lane 63: row sums, then row_bcast15 / row_bcast31.
__device__ inline double wave_total_dpp(double v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    v += dpp_mov<0x142, 0xa>(v);
    v += dpp_mov<0x143, 0xc>(v);
    return v;
}

// Sums of a and b over a workgroup of BS threads, valid in thread 0 (fixed order: wave 0,
// 1, ...).
template <int BS = kBlock>
__device__ inline void block_sum2(double &a, double &b) {
    __shared__ double sh[2][BS / kWave];
    a = wave_total_dpp(a);
    b = wave_total_dpp(b);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == kWave - 1) {
        sh[0][w] = a;
        sh[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = sh[0][0];
        b = sh[1][0];
        for (int i = 1; i < BS / kWave; ++i) {
            a += sh[0][i];
            b += sh[1][i];
        }
    }
    __syncthreads();
}

// This workgroup's partial sums for the next launch (plain stores).
template <int BS = kBlock>
__device__ inline void leave(const StepArgs &a, double s0, double s1, int slot) {
    block_sum2<BS>(s0, s1);
    if (threadIdx.x == 0) {
        reinterpret_cast<double2 *>(a.part_next)[slot] = make_double2(s0, s1);
    }
}

// ---------------------------------------------------------------------------------------
// entry: state and the previous launch's partial sums
// ---------------------------------------------------------------------------------------

template <int BS>
struct EntryT {
    static constexpr int kRegs = kMaxLoopGrid / BS;  // previous-launch partials per thread
    LsqrState st;
    double pa[kRegs], pb[kRegs];
};
using Entry = EntryT<kBlock>;

// Issue the loads (values are consumed in entry_finish). The partial buffers hold
// kMaxLoopGrid slots, so the loads stay in bounds; slots beyond pend_blocks are ignored.
// A wait for a load also waits for every load issued before it, so the kernels issue these
// after the first loads of their own work.
template <int BS>
__device__ inline void entry_issue(const StepArgs &a, EntryT<BS> &e) {
    e.st = *a.st;
#pragma unroll
    for (int j = 0; j < EntryT<BS>::kRegs; ++j) {
        const int i = threadIdx.x + j * BS;
        const double2 v = reinterpret_cast<const double2 *>(a.part_prev)[i];  // one 16-byte load
        e.pa[j] = v.x;
        e.pb[j] = v.y;
    }
}

// Sums of a and b over the workgroup, valid in every thread (the same fixed order as
// block_sum2, so every thread holds the same bits).
template <int BS = kBlock>
__device__ inline void block_sum2_all(double &a, double &b) {
    __shared__ double sh[2][BS / kWave];
    a = wave_total_dpp(a);
    b = wave_total_dpp(b);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == kWave - 1) {
        sh[0][w] = a;
        sh[1][w] = b;
    }
    __syncthreads();
    a = sh[0][0];
    b = sh[1][0];
    for (int i = 1; i < BS / kWave; ++i) {
        a += sh[0][i];
        b += sh[1][i];
    }
}

// Finalise the previous launch's reduction into S (a copy per thread: every thread holds
// the totals and evaluates the same scalars, so no broadcast or second barrier is needed);
// false in every thread once LSQR stopped.
template <int BS>
__device__ inline bool entry_finish(const StepArgs &a, const EntryT<BS> &e, LsqrState *S, int my_fwd) {
    const int tid = threadIdx.x;
    if (e.st.done) {
        if (blockIdx.x == 0 && tid == 0) *a.st_next = e.st;
        return false;
    }
    double t0 = 0.0, t1 = 0.0;
    if (e.st.pend_role >= 0) {
#pragma unroll
        for (int j = 0; j < EntryT<BS>::kRegs; ++j)
            if (tid + j * BS < e.st.pend_blocks) {
                t0 += e.pa[j];
                t1 += e.pb[j];
            }
        block_sum2_all<BS>(t0, t1);
    }
    LsqrState s = e.st;
    if (s.pend_role >= 0) finalize(&s, s.pend_role, t0, t1, s.pend_fwd != 0);
    if (s.done) {
        s.pend_role = -1;
    } else {
        s.pend_role = a.role;
        s.pend_blocks = gridDim.x + a.extra_slots;
        s.pend_fwd = my_fwd;
    }
    // Only the buffer of the next launch is written: other workgroups of this launch may
    // still be loading *a.st. A stop decided here reaches the other buffer through the next
    // launch's copy at its entry (every graph holds whole pairs of launches), so after a
    // graph both buffers hold the final state.
    if (blockIdx.x == 0 && tid == 0) *a.st_next = s;
    *S = s;
    return !s.done;
}

// ---------------------------------------------------------------------------------------
// state-free operands of one output entry, and its finish
// ---------------------------------------------------------------------------------------

struct Ptrs {  // scales by role; none depends on the LSQR scalars
    const double *isc, *osc, *nxs;
    // CSR values of the products with the input: the input scale folded in (Pv o isc[col]
    // etc., prepared per solve) when the launch has them, then gsc is null; else the plain
    // values, gathered with gsc = isc
    const double *Pv, *Av, *Tv, *gsc;
};

__device__ inline Ptrs ptrs_of(const Problem &p, const StepArgs &a) {
    Ptrs q;
    q.isc = a.in_is_v ? a.sc : a.scl;
    const bool baked = q.isc && a.Pvs;
    q.Pv = baked ? a.Pvs : p.Pv;
    q.Av = baked ? a.Avs : p.Av;
    q.Tv = baked ? a.Tvs : p.Tv;
    q.gsc = baked ? nullptr : q.isc;
    q.osc = (a.role == ROLE_U) ? a.scl : (a.role == ROLE_V || a.role == ROLE_V0) ? a.sc : nullptr;
    q.nxs = a.out_is_v ? a.sc : a.scl;
    return q;
}

__device__ inline double in_raw(const StepArgs &a, const Ptrs &q, int j) {
    const double v = a.in[j];
    return q.isc ? v * q.isc[j] : v;
}

// Strided CSR dot product sum_k val[k] (sc o x)[col[k] + off] over k = k0 + lane, k0 + lane
// + L, ... below k1, with sc absent meaning all ones. Four entries per pass, each pass's loads
// issued together: indices past k1 are clamped to k1 - 1 (a valid entry) and their value is
// replaced by zero, so the loop body has no branch between its loads.
template <bool SC>
__device__ inline double csr_dot4(const int *col, const double *val, int k0, int k1, int lane,
                                  int L, const double *x, const double *sc, int off) {
    double acc = 0.0;
    for (int k = k0 + lane; k < k1; k += 4 * L) {
        int j[4];
        double v[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = min(k + u * L, k1 - 1);
            j[u] = col[kk] + off;
            v[u] = val[kk];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = SC ? x[j[u]] * sc[j[u]] : x[j[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k + u * L < k1) acc += v[u] * xv[u];
    }
    return acc;
}

// csr_dot4's first pass (entries k, k + L, k + 2L, k + 3L of a lane, clamped to the row's
// last entry and, for an empty row, to entry 0) loaded ahead of other work, and the sum that
// starts from it: the same terms in the same order as csr_dot4.
struct Pass4 {
    int j[4];
    double v[4];
};
__device__ inline void pass4_load(const int *col, const double *val, int k, int k1, int L,
                                  int off, Pass4 &ps) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int kk = max(min(k + u * L, k1 - 1), 0);
        ps.j[u] = col[kk] + off;
        ps.v[u] = val[kk];
    }
}
template <bool SC>
__device__ inline double csr_dot4_from(const Pass4 &ps, const int *col, const double *val,
                                       int k0, int k1, int lane, int L, const double *x,
                                       const double *sc, int off) {
    double acc = 0.0;
    int k = k0 + lane;
    if (k < k1) {
        double xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = SC ? x[ps.j[u]] * sc[ps.j[u]] : x[ps.j[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k + u * L < k1) acc += ps.v[u] * xv[u];
    }
    for (k += 4 * L; k < k1; k += 4 * L) {
        int j[4];
        double v[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = min(k + u * L, k1 - 1);
            j[u] = col[kk] + off;
            v[u] = val[kk];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = SC ? x[j[u]] * sc[j[u]] : x[j[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k + u * L < k1) acc += v[u] * xv[u];
    }
    return acc;
}

__device__ inline double csr_dot(const int *col, const double *val, int k0, int k1, int lane,
                                 int L, const double *x, const double *sc, int off) {
    return sc ? csr_dot4<true>(col, val, k0, k1, lane, L, x, sc, off)
              : csr_dot4<false>(col, val, k0, k1, lane, L, x, sc, off);
}

// Two strided CSR dot products of one row (P and A' of an x row) in the same passes, so
// the loads of both are in flight together: pass i issues four entries of each.
template <bool SCA, bool SCB>
__device__ inline void csr_dot_pair(const int *colA, const double *valA, int a0, int a1,
                                    const double *xA, const double *scA, int offA,
                                    const int *colB, const double *valB, int b0, int b1,
                                    const double *xB, const double *scB, int offB, int lane,
                                    int L, double &accA, double &accB) {
    accA = 0.0;
    accB = 0.0;
    for (int ka = a0 + lane, kb = b0 + lane; ka < a1 || kb < b1; ka += 4 * L, kb += 4 * L) {
        int ja[4], jb[4];
        double va[4], vb[4], xa[4], xb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int ia = max(min(ka + u * L, a1 - 1), 0), ib = max(min(kb + u * L, b1 - 1), 0);
            ja[u] = a1 > a0 ? colA[ia] + offA : 0;
            va[u] = a1 > a0 ? valA[ia] : 0.0;
            jb[u] = b1 > b0 ? colB[ib] + offB : 0;
            vb[u] = b1 > b0 ? valB[ib] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xa[u] = SCA ? xA[ja[u]] * scA[ja[u]] : xA[ja[u]];
            xb[u] = SCB ? xB[jb[u]] * scB[jb[u]] : xB[jb[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (ka + u * L < a1) accA += va[u] * xa[u];
            if (kb + u * L < b1) accB += vb[u] * xb[u];
        }
    }
}

// As csr_dot4 with kDeep entries per lane in flight: the batched loop gives each lane about
// that many entries (fewer lanes per row, more rows per workgroup), so a launch needs far
// fewer workgroups and each keeps more of the memory system busy.
constexpr int kDeep = 16;

template <bool SC, int D = kDeep>
__device__ inline double csr_dot_deep(const int *col, const double *val, int k0, int k1,
                                      int lane, int L, const double *x, const double *sc,
                                      int off) {
    double acc = 0.0;
    for (int k = k0 + lane; k < k1; k += D * L) {
        int j[D];
        double v[D], xv[D];
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int kk = min(k + u * L, k1 - 1);
            j[u] = col[kk] + off;
            v[u] = val[kk];
        }
#pragma unroll
        for (int u = 0; u < D; ++u) xv[u] = SC ? x[j[u]] * sc[j[u]] : x[j[u]];
#pragma unroll
        for (int u = 0; u < D; ++u)
            if (k + u * L < k1) acc += v[u] * xv[u];
    }
    return acc;
}

// The staged kernels' sums with the input in LDS, over the packed copy of P or A: each lane
// reads whole quads of consecutive entries (one 8-byte load of four 16-bit columns, two
// 16-byte loads of their values), two quads per pass, lanes strided by quads. Padding
// entries (column 0, value 0) add nothing. Measured on the n = 20 000 workload against
// strided single entries: probes of P's and A's shapes 14 % and 13 % faster; eight entries
// per lane in flight instead of four, masked loads past a row's end and non-temporal CSR
// streams (to keep the gathered vectors in L2) gained nothing or lost (up to 40 %).
__device__ inline double csr_dot_quads(const int *rp4, const unsigned short *c4,
                                       const double *v4, int row, int lane, int L,
                                       const double *xs) {
    const int q0 = rp4[row] >> 2, q1 = rp4[row + 1] >> 2;
    const ushort4 *C = reinterpret_cast<const ushort4 *>(c4);
    const double2 *V = reinterpret_cast<const double2 *>(v4);
    double acc = 0.0;
    for (int qq = q0 + lane; qq < q1; qq += 2 * L) {
        ushort4 c[2];
        double2 va[2], vb[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int qk = min(qq + u * L, q1 - 1);
            c[u] = C[qk];
            va[u] = V[2 * qk];
            vb[u] = V[2 * qk + 1];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (qq + u * L < q1)
                acc += va[u].x * xs[c[u].x] + va[u].y * xs[c[u].y] + vb[u].x * xs[c[u].z] +
                       vb[u].y * xs[c[u].w];
    }
    return acc;
}

template <bool DEEP>
__device__ inline double csr_dot_d(const int *col, const double *val, int k0, int k1, int lane,
                                   int L, const double *x, const double *sc, int off) {
    if (!DEEP) return csr_dot(col, val, k0, k1, lane, L, x, sc, off);
    return sc ? csr_dot_deep<true>(col, val, k0, k1, lane, L, x, sc, off)
              : csr_dot_deep<false>(col, val, k0, k1, lane, L, x, sc, off);
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
    // two independent reciprocals instead of four dependent quotients
    const double ia = 1.0 / S.alpha, ib = 1.0 / S.beta;
    Ctx c;
    c.inv = a.in_nrm == NRM_ALPHA ? ia : a.in_nrm == NRM_BETA ? ib : 1.0 / S.one;
    c.cU = (a.role == ROLE_U) ? S.alpha * ib : 0.0;
    c.cV = (a.role == ROLE_V) ? S.beta * ia : 0.0;
    c.inv_alpha_up = a.do_update ? ia : 0.0;
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

template <bool DEEP>
__device__ inline void rows_pre(const Problem &p, const StepArgs &a, const Ptrs &q,
                                const RowGrid &g, int vb, RowPre &r) {
    const int n = p.n, m = p.m, N = p.N;
    const int tid = threadIdx.x;
    const bool xr = vb < g.bx;
    const int L = xr ? g.lx : g.ly;
    const long long gt = (long long)(xr ? vb : vb - g.bx) * kBlock + tid;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    // the output entry of lane 0 of each row group and its operands, loaded before the sums
    // (no arithmetic on them until the sums are done)
    int idx = -1;
    if (lane == 0) {
        if (xr) idx = row < n ? row : -1;
        else if (row < m) idx = n + row;
        else if (row == m) idx = N - 1;
    }
    double qb = 0.0, self = 0.0, self_sc = 1.0, wyr = 0.0;
    if (idx >= 0) {
        fin_load(a, q, idx, r.f);
        if (idx < n) {
            qb = p.q[idx];
        } else if (idx < N - 1) {
            const int y = idx - n;
            qb = p.b[y];
            self = a.in[idx];
            if (q.isc) self_sc = q.isc[idx];
            wyr = a.wy[y];
        }
    }
    double acc = 0.0, accT = 0.0;
    if (xr) {
        if (row < n) {
            const int k0 = p.Prp[row], k1 = p.Prp[row + 1];
            const int t0 = p.Trp[row], t1 = p.Trp[row + 1];
            // two separate passes measure faster here than csr_dot_pair (fewer registers)
            acc = csr_dot_d<DEEP>(p.Pci, q.Pv, k0, k1, lane, L, a.in, q.gsc, 0);
            accT = csr_dot_d<DEEP>(p.Tci, p.Tv, t0, t1, lane, L, a.wy, nullptr, 0);
        }
    } else if (row < m) {
        const int k0 = p.Arp[row], k1 = p.Arp[row + 1];
        acc = csr_dot_d<DEEP>(p.Aci, q.Av, k0, k1, lane, L, a.in, q.gsc, 0);
    }
    r.acc = group_sum_dpp(acc, L);
    r.accT = group_sum_dpp(accT, L);
    r.idx = idx;
    r.qb = qb;
    r.self = q.isc ? self * self_sc : self;  // in_raw of the row's own entry
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

template <bool DEEP>
__device__ inline void loop_F_body(const Problem &p, const StepArgs &a, const RowGrid &g) {
    LsqrState S;  // per thread (entry_finish)
    Entry e;
    const Ptrs q = ptrs_of(p, a);
    const double in_N_raw = in_raw(a, q, p.N - 1);
    RowPre r;
    rows_pre<DEEP>(p, a, q, g, blockIdx.x, r);
    entry_issue(a, e);  // after the row loads: the memory counter is in order
    if (!entry_finish(a, e, &S, 0)) return;
    const Ctx c = scalars(a, S, q, in_N_raw);
    double s0 = 0.0, s1 = 0.0;
    rows_post(p, a, c, S, r, s0, s1);
    for (int vb = blockIdx.x + gridDim.x; vb < g.bx + g.by; vb += gridDim.x) {
        rows_pre<DEEP>(p, a, q, g, vb, r);
        rows_post(p, a, c, S, r, s0, s1);
    }
    leave(a, s0, s1, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_loop_F(Problem p, StepArgs a, RowGrid g) {
    loop_F_body<false>(p, a, g);
}


// ---------------------------------------------------------------------------------------
// product with F', fused with the cone Jacobians (work units as in k_fused_FT)
// ---------------------------------------------------------------------------------------

constexpr int kPostPref = 4;  // PSD units of the cone launch: later rows prefetched per thread

struct UnitPre {
    int idx;                   // entry of this thread (x / diagonal rows: lane 0), or -1
    double acc, accT, self, coef, jd;
    double bv;                 // cone units: b at this thread's first row
    double cp[4];              // SOC factors of this thread's cone: mode, 1/|u|, c1, c2
    int ii, jj;                // PSD units: the matrix entry of this thread's first row
    Fin f;
    // PSD units of the cone launch: finish operands and b of rows tid + j kBlock,
    // j = 1 .. kPostPref (clamped to the last row), loaded before the first Jacobian so
    // that they arrive while it runs
    Fin fq[kPostPref];
    double bq[kPostPref];
};

// LDS of a cone unit. Runs of SOC / exponential cones: tb (raw rows), rb (raw r_y, then the
// scaled outputs), jt (J applied), ub (SOC: u/|u| at each row; exponential: each cone's
// 3x3 Jacobian), kUnitRows each. One PSD cone of order k: X, T, V and, when it fits, B as
// kp x ld matrices (kp = k rounded up to a multiple of 16, zero-padded, ld = kp + 1), then
// tb, rb, jt (k(k+1)/2 each). Each unit also has a gather buffer gb of kGather products for
// its CSR rows, used before the cone factors are staged: jt and ub of a SOC / exponential
// unit, X, T, V and B of a PSD unit when they are large enough, else after jt.
constexpr int kPsdLdsCap = 16384;  // doubles a PSD unit may stage B into
constexpr int kPsdPref = 4;        // V, B entries per thread loaded ahead (kp*kp <= 1024)
constexpr int kSocPref = 8;        // u entries per cone loaded ahead (dimensions <= 9)
constexpr int kGatherRegs = 8;     // CSR entries in flight per thread in a cone unit
constexpr int kGather = kGatherRegs * kBlock;
static_assert(kGather <= 2 * kUnitRows, "gather buffer of a SOC / exponential unit");

struct PsdLds {
    int kp, ld, nr, b, tb, gb;  // b: offset of B, or -1 when B is read from global memory
};

__host__ __device__ inline PsdLds psd_lds(int k) {
    PsdLds L;
    L.kp = (k + 15) / 16 * 16;
    L.ld = L.kp + 1;
    L.nr = k * (k + 1) / 2;
    const int mat = L.kp * L.ld;
    if (4 * mat + 3 * L.nr <= kPsdLdsCap) {
        L.b = 3 * mat;
        L.tb = 4 * mat;
    } else {
        L.b = -1;
        L.tb = 3 * mat;
    }
    L.gb = L.tb >= kGather ? 0 : L.tb + 3 * L.nr;
    return L;
}

// rows of a cone run from the cone tables (fill_unit_ranges stores them in the unit)
__device__ inline int unit_rows_of(const Problem &p, const Unit &u, int &r0) {
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

__device__ inline int unit_rows(const Unit &u, int &r0) {
    r0 = u.row0;
    return u.nrows;
}

__device__ inline void unit_bufs(const Problem &p, const Unit &u, double *sm, int nr,
                                 double *&tb, double *&rb, double *&jt, double *&ub,
                                 double *&gb) {
    if (u.type == U_PSD) {
        const PsdLds L = psd_lds(u.k);
        tb = sm + L.tb;
        rb = tb + nr;
        jt = rb + nr;
        ub = nullptr;
        gb = sm + L.gb;
    } else {
        tb = sm;
        rb = sm + kUnitRows;
        jt = sm + 2 * kUnitRows;
        ub = sm + 3 * kUnitRows;
        gb = jt;
    }
}

// Products val[k] * (sc o x)[col[k]] of the entries base .. base + cnt - 1 (1 <= cnt <=
// kGather) into gb, kGatherRegs per thread with all loads issued before the first use;
// entries past cnt load entry cnt - 1 (valid) and are not stored.
template <bool SC>
__device__ inline void gather_products(const int *col, const double *val, int base, int cnt,
                                       const double *x, const double *sc, double *gb) {
    const int tid = threadIdx.x;
    int j[kGatherRegs];
    double v[kGatherRegs], xv[kGatherRegs];
#pragma unroll
    for (int u = 0; u < kGatherRegs; ++u) {
        const int k = base + min(tid + u * kBlock, cnt - 1);
        j[u] = col[k];
        v[u] = val[k];
    }
#pragma unroll
    for (int u = 0; u < kGatherRegs; ++u) xv[u] = SC ? x[j[u]] * sc[j[u]] : x[j[u]];
#pragma unroll
    for (int u = 0; u < kGatherRegs; ++u)
        if (tid + u * kBlock < cnt) gb[tid + u * kBlock] = v[u] * xv[u];
}

// SOC Jacobian (see soc_jv) on unit-relative rows [i0, i0 + dim), u/|u| read from ub
template <class IN, class OUT>
__device__ inline void soc_apply(const double *cp, const double *ub, int i0, int dim, IN in,
                                 OUT out) {
    const int mode = (int)cp[0];
    if (mode == 0) {
        for (int i = 0; i < dim; ++i) out(i0 + i, 0.0);
        return;
    }
    if (mode == 1) {
        for (int i = 0; i < dim; ++i) out(i0 + i, in(i0 + i));
        return;
    }
    const double c1 = cp[2], c2 = cp[3];
    const double dt = in(i0);
    double a = 0.0;
    for (int i = 1; i < dim; ++i) a += ub[i0 + i] * in(i0 + i);
    out(i0, 0.5 * (dt + a));
    for (int i = 1; i < dim; ++i) {
        const double uh = ub[i0 + i];
        out(i0 + i, 0.5 * uh * dt + c1 * in(i0 + i) - c2 * a * uh);
    }
}

template <class IN, class OUT>
__device__ inline void exp_apply(const double *J, int i0, IN in, OUT out) {
    const double a = in(i0), b = in(i0 + 1), c = in(i0 + 2);
    out(i0, J[0] * a + J[1] * b + J[2] * c);
    out(i0 + 1, J[3] * a + J[4] * b + J[5] * c);
    out(i0 + 2, J[6] * a + J[7] * b + J[8] * c);
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// The K = 4 KS sum of one 16 x 16 tile, lanes and accumulator entries as in mfma_product below:
// all 2 KS operands are loaded before the first product (one wave per SIMD: nothing else
// would hide the LDS latency), even and odd steps in two accumulators.
template <int KS, class AF, class BF>
__device__ inline dbl4 mfma_tile(int i0, int j0, AF af, BF bf) {
    const int lane = threadIdx.x & (kWave - 1), li = lane & 15, lk = lane >> 4;
    double av[KS], bv[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        av[s] = af(i0 + li, 4 * s + lk);
        bv[s] = bf(4 * s + lk, j0 + li);
    }
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s + 1 < KS; s += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s + 1], bv[s + 1], acc1, 0, 0, 0);
    }
    if constexpr (KS % 2 == 1)
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[KS - 1], bv[KS - 1], acc0, 0, 0, 0);
    return acc0 + acc1;
}

// One KP x KP product C = A B on the FP64 matrix cores, operands read through af(i, kk) and
// bf(kk, j) (LDS, zero beyond the cone's order): wave w computes the 16 x 16 tiles w, w + 4,
// ... in row-major tile order with V_MFMA_F64_16X16X4F64. In step s lane l supplies
// A[i0 + l%16][4s + l/16] and B[4s + l/16][j0 + l%16]; accumulator entry r of lane l is
// C[i0 + 4r + l/16][j0 + l%16]. The operands of a chunk of up to eight steps (a divisor of
// the step count: six for KP = 48) are loaded before its first product, and even and odd
// steps accumulate separately (two short dependency chains instead of one long one).
// epi(i, j, acc) receives i = i0 + l/16 (rows i + 4r) and j = j0 + l%16. KS < KP / 4: the
// sum over the first 4 KS entries of K only (the rest of A's columns or B's rows are zero),
// its operands all loaded ahead.
template <int KP, int KS = KP / 4, class AF, class BF, class EPI>
__device__ inline void mfma_product(AF af, BF bf, EPI epi) {
    constexpr int NT = KP / 16, NS = KP / 4;
    constexpr int CH = NS % 8 == 0 ? 8 : NS % 6 == 0 ? 6 : 4;
    static_assert(NS % CH == 0 && CH % 2 == 0, "a chunk must divide the steps into pairs");
    static_assert(KS == NS || KS <= 8, "a cut sum is loaded whole");
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 1
    for (int t = wave; t < NT * NT; t += kBlock / kWave) {
        const int i0 = (t / NT) * 16, j0 = (t % NT) * 16;
        if constexpr (KS < NS) {
            epi(i0 + lk, j0 + li, mfma_tile<KS>(i0, j0, af, bf));
            continue;
        }
        dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
        for (int s0 = 0; s0 < NS; s0 += CH) {
            double av[CH], bv[CH];
#pragma unroll
            for (int s = 0; s < CH; ++s) {
                const int kk = 4 * (s0 + s) + lk;
                av[s] = af(i0 + li, kk);
                bv[s] = bf(kk, j0 + li);
            }
#pragma unroll
            for (int s = 0; s < CH; s += 2) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s + 1], bv[s + 1], acc1, 0, 0, 0);
            }
        }
        epi(i0 + lk, j0 + li, acc0 + acc1);
    }
}

// PSD Jacobian Y = J[X] = V (B o (V' X V)) V' (see psd_jv) of the symmetric matrix X held
// in the X region (zero beyond the order), with V (and B) staged in LDS as KP x (KP + 1)
// matrices; the four products on the matrix cores. Y replaces X (zero beyond the order, as
// V is). The callers write X from the svec rows and read Y back into them (svec_rc), so the
// products themselves do no index arithmetic. KS < KP / 4 (orders up to 4 KS): each product's
// sum over the first 4 KS entries only, those beyond the order being zero in X, V and T.
template <int KP, int KS = KP / 4>
__device__ inline void psd_apply_kp(int k, const PsdLds &L, double *sm, const double *Bg) {
    constexpr int ld = KP + 1, mat = KP * ld;
    double *X = sm, *T = sm + mat;
    const double *V = sm + 2 * mat, *B = L.b >= 0 ? sm + L.b : nullptr;
    auto vf = [&](int i, int j) { return V[i * ld + j]; };
    auto vt = [&](int i, int j) { return V[j * ld + i]; };
    auto tf = [&](int i, int j) { return T[i * ld + j]; };
    auto xm = [&](int i, int j) { return X[i * ld + j]; };
    auto to_t = [&](int i, int j, const dbl4 &c) {
        for (int r = 0; r < 4; ++r) T[(i + 4 * r) * ld + j] = c[r];
    };
    mfma_product<KP, KS>(xm, vf, to_t);  // T = X V
    __syncthreads();
    mfma_product<KP, KS>(vt, tf, [&](int i, int j, const dbl4 &c) {  // X = B o (V'T)
        for (int r = 0; r < 4; ++r) {
            const int ii = i + 4 * r;
            double bij = 0.0;
            if (ii < k && j < k) bij = B ? B[ii * ld + j] : Bg[ii * k + j];
            X[ii * ld + j] = bij * c[r];
        }
    });
    __syncthreads();
    mfma_product<KP, KS>(vf, xm, to_t);  // T = V X
    __syncthreads();
    mfma_product<KP, KS>(tf, vt, [&](int i, int j, const dbl4 &c) {  // X = Y = T V'
        for (int r = 0; r < 4; ++r) X[(i + 4 * r) * ld + j] = c[r];
    });
    __syncthreads();
}

// The last product of the low-rank Jacobian: Y = U V_S' + V_S U' (neg: X minus it) on the
// lower triangle of 16 x 16 tiles, as the product of the KP x 8 CS panel [U_:, <4CS | V_:, <4CS]
// with [V_:, <4CS | U_:, <4CS]' (U's columns from c <= 4 CS on are zero, so the columns
// dropped add nothing). Tiles t = wave, wave + 4, ... of the lower triangle in row order; a
// wave short of its last tile recomputes tile 0 and drops the result. W holds U (KP x 17).
template <int KP, int CS>
__device__ inline void lr_sym_product(double *X, const double *W, const double *V, bool neg) {
    constexpr int ld = KP + 1, lc = 17, MT = KP / 16;
    constexpr int NLT = MT * (MT + 1) / 2, NJ = (NLT + kBlock / kWave - 1) / (kBlock / kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    auto af = [&](int i, int kk) { return kk < 4 * CS ? W[i * lc + kk] : V[i * ld + kk - 4 * CS]; };
    auto bf = [&](int kk, int j) { return kk < 4 * CS ? V[j * ld + kk] : W[j * lc + kk - 4 * CS]; };
    dbl4 acc[NJ];
    int ti[NJ], tj[NJ];
#pragma unroll
    for (int jn = 0; jn < NJ; ++jn) {
        const int t = wave + jn * (kBlock / kWave), tt = t < NLT ? t : 0;
        ti[jn] = tt >= 6 ? 3 : tt >= 3 ? 2 : tt >= 1 ? 1 : 0;
        tj[jn] = tt - ti[jn] * (ti[jn] + 1) / 2;
        acc[jn] = mfma_tile<2 * CS>(16 * ti[jn], 16 * tj[jn], af, bf);
    }
#pragma unroll
    for (int jn = 0; jn < NJ; ++jn) {
        if (wave + jn * (kBlock / kWave) >= NLT) break;
        for (int r = 0; r < 4; ++r) {
            double &x = X[(16 * ti[jn] + lk + 4 * r) * ld + 16 * tj[jn] + li];
            x = neg ? x - acc[jn][r] : acc[jn][r];
        }
    }
}

// Low-rank form of the same Jacobian, for a cone whose eigenvalues leave c <= 16 on one side
// of zero: setup stores those eigenpairs first in V and B (S, the first c columns). With
// M = V'XV and Bs = B (S: eigenvalues >= 0) or 1 - B (S: eigenvalues < 0), both equal to one
// on S x S and
//   V (Bs o M) V' = E + E' - V_S M_SS V_S',   E = V (Bs o M)[:, S] V_S'
// (Bs o M is nonzero on the rows or columns of S only), and J[X] = V (B o M) V' equals that
// sum (S >= 0) or X minus it (V orthogonal). With H = (V'(X V_S)) times Bs[:, S] elementwise,
// its S x S block halved, and U = V H: the sum is U V_S' + V_S U', one product of the
// KP x 32 panel [U V_S] with [V_S U]'. Three KP x KP x 16 products and that one, on the
// lower triangle of 16 x 16 tiles only: about 4 KP^2 16 multiply-adds instead of 4 KP^3.
// X (symmetric, zero beyond the order) is replaced by Y on and below the diagonal (the
// callers read the lower triangle only; above it X is left as it was, zero beyond the
// order); W and H are KP x 16 panels in the T region. Bs[:, S] comes from B in LDS, else
// from the KP x 16 panel of B's first columns staged after W and H (KP = 64: the cone
// launch stages it with V). Waves own whole tiles: the first three products have
// KP / 16 <= 4 of them, one per wave. KS: the k-steps of 4 of the first three products' sums
// (KP / 4, or fewer when the order leaves the last rows and columns of X and V zero).
template <int KP, int KS = KP / 4>
__device__ inline void psd_apply_lr(int k, int c, bool neg, const PsdLds &L, double *sm,
                                    const double *Bg) {
    constexpr int ld = KP + 1, mat = KP * ld, lc = 17, MT = KP / 16;
    static_assert(KS >= 1 && KS <= KP / 4, "steps within the padded order");
    static_assert(2 * KP * lc <= mat, "two KP x 16 panels fit in the T region");
    static_assert(MT <= kBlock / kWave, "one row tile per wave");
    double *X = sm, *W = sm + mat, *H = sm + mat + KP * lc;
    const double *V = sm + 2 * mat, *B = L.b >= 0 ? sm + L.b : nullptr;
    const double *Bp = nullptr;
    if constexpr (3 * KP * lc <= mat) Bp = sm + mat + 2 * KP * lc;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    auto vf = [&](int i, int j) { return V[i * ld + j]; };
    auto vt = [&](int i, int j) { return V[j * ld + i]; };
    if (wave < MT) {  // W = X V_S
        const dbl4 a = mfma_tile<KS>(16 * wave, 0, [&](int i, int j) { return X[i * ld + j]; }, vf);
        for (int r = 0; r < 4; ++r) W[(16 * wave + lk + 4 * r) * lc + li] = a[r];
    }
    __syncthreads();
    if (wave < MT) {  // H = Bs' o (V'W), the factors read before the products
        double f[4];
        for (int r = 0; r < 4; ++r) {
            const int ii = 16 * wave + lk + 4 * r;
            f[r] = 0.0;
            if (ii < k && li < c) {
                if (ii < c) {
                    f[r] = 0.5;
                } else {
                    const double b = B ? B[ii * ld + li] : Bp ? Bp[ii * lc + li] : Bg[ii * k + li];
                    f[r] = neg ? 1.0 - b : b;
                }
            }
        }
        const dbl4 a = mfma_tile<KS>(16 * wave, 0, vt, [&](int i, int j) { return W[i * lc + j]; });
        for (int r = 0; r < 4; ++r) H[(16 * wave + lk + 4 * r) * lc + li] = f[r] * a[r];
    }
    __syncthreads();
    if (wave < MT) {  // U = V H, into the W panel
        const dbl4 a = mfma_tile<KS>(16 * wave, 0, vf, [&](int i, int j) { return H[i * lc + j]; });
        for (int r = 0; r < 4; ++r) W[(16 * wave + lk + 4 * r) * lc + li] = a[r];
    }
    __syncthreads();
    // Y = U V_S' + V_S U' (or X minus it) on the lower tiles, over the 4 CS columns of each
    // panel that can be nonzero (U's columns from c on are zero)
    switch ((c + 3) >> 2) {
    case 0:
    case 1: lr_sym_product<KP, 1>(X, W, V, neg); break;
    case 2: lr_sym_product<KP, 2>(X, W, V, neg); break;
    case 3: lr_sym_product<KP, 3>(X, W, V, neg); break;
    default: lr_sym_product<KP, 4>(X, W, V, neg); break;
    }
    __syncthreads();
}

// MAXKP: the largest padded order the caller can meet (fewer instances, fewer registers)
template <int MAXKP = 64>
__device__ inline void psd_apply(int k, const PsdLds &L, double *sm, const double *Bg) {
    if (MAXKP <= 16) {
        psd_apply_kp<16>(k, L, sm, Bg);
        return;
    }
    switch (L.kp) {
    case 16: psd_apply_kp<16>(k, L, sm, Bg); break;
    case 32:  // orders 17-20: sums over the order only (5 k-steps)
        if (k <= 20) psd_apply_kp<32, 5>(k, L, sm, Bg);
        else psd_apply_kp<32>(k, L, sm, Bg);
        break;
    case 48: psd_apply_kp<48>(k, L, sm, Bg); break;
    default: psd_apply_kp<64>(k, L, sm, Bg); break;
    }
}

// The Jacobian of PSD cone `cone`: the low-rank form where LR is set, the factors record a
// side of at most 16 eigenvalues and the padded order is 48 or 64; else the full form.
template <int MAXKP = 64, bool LR = false>
__device__ __forceinline__ void psd_apply_sel(const int *psd_lr, int cone, int k, const PsdLds &L,
                                     double *sm, const double *Bg) {
    if (LR && MAXKP >= 48 && L.kp >= 48 && psd_lr) {
        const int lr = psd_lr[cone], c = lr & 255;
        if (c <= 16) {
            if (L.kp == 48) psd_apply_lr<48>(k, c, lr >= 256, L, sm, Bg);
            else if (k <= 52) psd_apply_lr<64, 13>(k, c, lr >= 256, L, sm, Bg);  // 13 k-steps
            else psd_apply_lr<64>(k, c, lr >= 256, L, sm, Bg);
            return;
        }
    }
    psd_apply<MAXKP>(k, L, sm, Bg);
}

// svec row i of an order-k cone is the matrix entry (ii, jj), ii >= jj (column jj holds the
// rows ii = jj .. k-1)
__device__ inline void svec_rc(int i, int k, int &ii, int &jj) {
    // column j starts at row off(j) = j (2k + 1 - j) / 2: the root of off(j) = i, rounded
    // down, then corrected by one either way for the rounding of the square root
    const int b = 2 * k + 1;
    int j = (int)((b - sqrtf((float)(b * b - 8 * i))) * 0.5f);
    j = max(0, min(j, k - 1));
    if (j * (b - j) / 2 > i) --j;
    else if ((j + 1) * (b - j - 1) / 2 <= i) ++j;
    jj = j;
    ii = j + (i - j * (b - j) / 2);
}

// svec value v of entry (ii, jj) into the symmetric matrix X (both triangles)
__device__ inline void smat_put(double *X, int ld, int ii, int jj, double v) {
    if (ii == jj) {
        X[ii * ld + ii] = v;
    } else {
        v *= kRsqrt2;
        X[ii * ld + jj] = v;
        X[jj * ld + ii] = v;
    }
}

// svec value of entry (ii, jj) of the symmetric matrix Y
__device__ inline double smat_get(const double *Y, int ld, int ii, int jj) {
    return ii == jj ? Y[ii * ld + ii] : Y[ii * ld + jj] * kSqrt2;
}

// e / kp for 0 <= e < 8192 and kp a multiple of 16 up to 64, rkp = 1 / kp in FP32: the
// quotient (e + 1/2) / kp is at least 1 / (2 kp) >= 2^-7 from an integer and the FP32
// product is within 2^-22 (e + 1/2) / kp <= 2^-13 of it, so truncation gives the integer
// quotient (an integer division by a value known only at run time costs tens of
// instructions per use)
__device__ inline int quot_kp(int e, float rkp) {
    return (int)(((float)e + 0.5f) * rkp);
}

// DEEP: the row units' CSR sums keep kDeep entries per lane in flight (batched loop).
// TROWS: the raw rows of a PSD unit come from a.tmp (written by the rows launch of the same
// product) instead of the unit's own CSR gather.
template <bool DEEP = false, int MAXKP = 64, bool TROWS = false, bool LR = false>
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
            if (DEEP) {
                acc = csr_dot_d<DEEP>(p.Pci, q.Pv, k0, k1, lane, L, a.in, q.gsc, 0);
                accT = csr_dot_d<DEEP>(p.Tci, q.Tv, t0, t1, lane, L, a.in, q.gsc, n);
            } else if (q.gsc) {
                csr_dot_pair<true, true>(p.Pci, q.Pv, k0, k1, a.in, q.gsc, 0, p.Tci, q.Tv, t0, t1,
                                         a.in, q.gsc, n, lane, L, acc, accT);
            } else {
                csr_dot_pair<false, false>(p.Pci, q.Pv, k0, k1, a.in, nullptr, 0, p.Tci, q.Tv, t0,
                                           t1, a.in, nullptr, n, lane, L, acc, accT);
            }
        }
        P.acc = group_sum_dpp(acc, L);
        P.accT = group_sum_dpp(accT, L);
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
            acc = csr_dot_d<DEEP>(p.Aci, q.Av, k0, k1, lane, L, a.in, q.gsc, 0);
        }
        P.acc = group_sum_dpp(acc, L);
        if (r < u.end && lane == 0) {
            P.idx = n + r;
            P.self = in_raw(a, q, n + r);
            P.coef = p.b[r];
            P.jd = p.jdiag[r];
            fin_load(a, q, n + r, P.f);
        }
        return;
    }
    if (u.type == U_PSDROWS) {  // raw t of PSD rows for the PSD launch; nothing to finish
        const int L = ly, lane = tid & (L - 1), r = u.begin + tid / L;
        double acc = 0.0;
        if (r < u.end) {
            const int k0 = p.Arp[r], k1 = p.Arp[r + 1];
            acc = csr_dot_d<DEEP>(p.Aci, q.Av, k0, k1, lane, L, a.in, q.gsc, 0);
        }
        acc = group_sum_dpp(acc, L);
        if (r < u.end && lane == 0)
            a.tmp[n + r] = acc - p.b[r] * in_N_raw - in_raw(a, q, n + r);
        return;
    }
    // cone units: issue the loads of the cone factors and of this thread's finish operands,
    // then the raw rows t = A r_x - b r_N - r_y (unnormalised) into tb, then stage the
    // factors in LDS and apply J to t into jt. Each cone kind has its own branch so that
    // the registers holding its prefetched factors are not live in the others.
    int r0;
    const int nr = unit_rows(u, r0);
    double *tb, *rb, *jt, *ub, *gb;
    unit_bufs(p, u, sm, nr, tb, rb, jt, ub, gb);
    // this thread's row operands; a PSD unit of the cone launch issues them after the loads
    // of its factors (whose addresses would otherwise wait for these loads to return)
    int rs = 0, re = 0;
    double ry = 0.0;
    auto row_ops = [&]() {
        if (tid < nr) {
            P.idx = n + r0 + tid;
            P.bv = p.b[r0 + tid];
            if (!TROWS) {
                rs = p.Arp[r0 + tid];
                re = p.Arp[r0 + tid + 1];
                ry = in_raw(a, q, n + r0 + tid);
            }
            fin_load(a, q, n + r0 + tid, P.f);
        }
    };
    const bool late_ops = TROWS && u.type == U_PSD;
    if (!late_ops) row_ops();
    // raw rows t = A r_x - b r_N - r_y of the unit (unnormalised). The unit's rows are
    // consecutive CSR rows, so their entries are one range [e0, e1): the workgroup gathers
    // the products of kGather entries at a time into gb, then each row adds its own entries
    // in CSR order (a fixed order, whatever the launch shape).
    auto yrows = [&]() {
        const int e0 = u.e0, e1 = u.e1;
        for (int base = e0; base < e1; base += kGather) {
            const int cnt = min(e1 - base, kGather);
            if (q.gsc) gather_products<true>(p.Aci, q.Av, base, cnt, a.in, q.gsc, gb);
            else gather_products<false>(p.Aci, q.Av, base, cnt, a.in, nullptr, gb);
            __syncthreads();
            for (int i = tid; i < nr; i += kBlock) {
                const int k0 = max(i == tid ? rs : p.Arp[r0 + i], base);
                const int k1 = min(i == tid ? re : p.Arp[r0 + i + 1], base + cnt);
                double acc = base == e0 ? 0.0 : tb[i];
                for (int k = k0; k < k1; ++k) acc += gb[k - base];
                tb[i] = acc;
            }
            __syncthreads();
        }
        for (int i = tid; i < nr; i += kBlock) {
            const int r = r0 + i;
            const double y = i == tid ? ry : in_raw(a, q, n + r);
            const double bb = i == tid ? P.bv : p.b[r];
            rb[i] = y;
            tb[i] = (e1 > e0 ? tb[i] : 0.0) - bb * in_N_raw - y;
        }
    };
    // the same rows from a.tmp (raw t of the rows launch) and the input, the loads of eight
    // rows per thread in flight at once (past the last row they read the last row, kept
    // unconditional); xld > 0: a PSD unit, whose rows also go into the symmetric matrix X
    // (leading dimension xld) while the loads are in flight
    auto trows = [&](int xld) {
        constexpr int R = 8;
        for (int i0 = tid; i0 < nr; i0 += R * kBlock) {
            double y[R], t[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = min(i0 + j * kBlock, nr - 1);
                y[j] = in_raw(a, q, n + r0 + i);
                t[j] = a.tmp[n + r0 + i];
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = i0 + j * kBlock;
                if (i < nr) {
                    rb[i] = y[j];
                    tb[i] = t[j];
                    if (xld > 0) {
                        int ii, jj;
                        svec_rc(i, u.k, ii, jj);
                        smat_put(sm, xld, ii, jj, t[j]);
                    }
                }
            }
        }
        __syncthreads();
    };
    auto tin = [&](int i) { return tb[i]; };
    auto jout = [&](int i, double v) { jt[i] = v; };
    const int cone = u.begin + tid;
    if (u.type == U_PSD) {
        const int k = u.k;
        const PsdLds Ld = psd_lds(k);
        const int kp = Ld.kp;
        const double *Vg = p.psd_pool + u.voff, *Bg = Vg + k * k;
        double *V = sm + 2 * kp * Ld.ld, *B = Ld.b >= 0 ? sm + Ld.b : nullptr;
        const float rkp = 1.0f / (float)kp;
        if (kp * kp <= kPsdPref * kBlock) {
            double vpre[kPsdPref], bpre[kPsdPref];
#pragma unroll
            for (int j = 0; j < kPsdPref; ++j) {
                const int e = tid + j * kBlock, i = quot_kp(e, rkp), jj = e - i * kp;
                const bool in_k = e < kp * kp && i < k && jj < k;
                vpre[j] = in_k ? Vg[i * k + jj] : 0.0;
                bpre[j] = (in_k && B) ? Bg[i * k + jj] : 0.0;
            }
            if (late_ops) row_ops();
            if (tid < nr) svec_rc(tid, k, P.ii, P.jj);  // while the loads are in flight
            if (TROWS) trows(Ld.ld); else yrows();
#pragma unroll
            for (int j = 0; j < kPsdPref; ++j) {
                const int e = tid + j * kBlock, i = quot_kp(e, rkp), jj = e - i * kp;
                if (e < kp * kp) {
                    V[i * Ld.ld + jj] = vpre[j];
                    if (B) B[i * Ld.ld + jj] = bpre[j];
                    if (i >= k || jj >= k) sm[i * Ld.ld + jj] = 0.0;  // X beyond order k
                }
            }
        } else if (TROWS) {
            // the cone launch: all of V (and B) in flight with the rows' loads, and with
            // kp = 64 (B not in LDS) the panel of B's first 16 columns for the low-rank form
            // after the W and H panels of the T region (also staged when it goes unused).
            // Thread tid takes column c = tid % 64 of rows tid / 64 + 4 j, of V and of the
            // panel's transpose (B is symmetric: column j of the panel is row j of B, whole
            // lines instead of 16 entries of every row); every load is issued, from a valid
            // address, and its value kept or replaced by zero.
            constexpr int RJ = 16, RB = 4;
            static_assert(RJ * (kBlock / 64) >= 64 && RB * (kBlock / 64) >= 16, "one batch");
            const int c = tid & 63, rq = tid / 64;
            const bool cin = c < k, panel = LR && kp == 64 && !B;
            const double *vp = Vg + (cin ? c : 0) + rq * k, *bq = Bg + (cin ? c : 0) + rq * k;
            double vv[RJ], bb[RJ], bp[RB];
#pragma unroll
            for (int j = 0; j < RJ; ++j) {
                const bool ok = cin && rq + 4 * j < k;
                const double v = vp[ok ? 4 * j * k : 0];
                vv[j] = ok ? v : 0.0;
            }
            if (B) {
#pragma unroll
                for (int j = 0; j < RJ; ++j) {
                    const bool ok = cin && rq + 4 * j < k;
                    const double v = bq[ok ? 4 * j * k : 0];
                    bb[j] = ok ? v : 0.0;
                }
            }
            if (panel) {
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    const bool ok = cin && rq + 4 * j < k;
                    const double v = bq[ok ? 4 * j * k : 0];
                    bp[j] = ok ? v : 0.0;
                }
            }
            asm volatile("" ::: "memory");  // keeps the row operands' loads after these
            row_ops();
            if (tid < nr) svec_rc(tid, k, P.ii, P.jj);
            trows(Ld.ld);
            if (c < kp) {
#pragma unroll
                for (int j = 0; j < RJ; ++j) {
                    const int r = rq + 4 * j;
                    if (r < kp) {
                        V[r * Ld.ld + c] = vv[j];
                        if (B) B[r * Ld.ld + c] = bb[j];
                        if (r >= k || c >= k) sm[r * Ld.ld + c] = 0.0;  // X beyond order k
                    }
                }
            }
            if (panel) {
                double *Bp = sm + kp * Ld.ld + 2 * kp * 17;
#pragma unroll
                for (int j = 0; j < RB; ++j) Bp[c * 17 + rq + 4 * j] = bp[j];  // c < kp = 64
            }
        } else {
            if (tid < nr) svec_rc(tid, k, P.ii, P.jj);
            yrows();
            for (int e = tid; e < kp * kp; e += kBlock) {
                const int i = quot_kp(e, rkp), jj = e - i * kp;
                const bool in_k = i < k && jj < k;
                V[i * Ld.ld + jj] = in_k ? Vg[i * k + jj] : 0.0;
                if (B) B[i * Ld.ld + jj] = in_k ? Bg[i * k + jj] : 0.0;
                if (!in_k) sm[i * Ld.ld + jj] = 0.0;
            }
        }
        // the raw rows as the symmetric matrix X (the gather buffer may have used the region;
        // trows wrote it already)
        if (!TROWS) {
            for (int i = tid; i < nr; i += kBlock) {
                int ii = P.ii, jj = P.jj;
                if (i != tid) svec_rc(i, k, ii, jj);
                smat_put(sm, Ld.ld, ii, jj, tb[i]);
            }
        }
        __syncthreads();
        if constexpr (TROWS && LR) {
#pragma unroll
            for (int j = 0; j < kPostPref; ++j) {
                const int i = min(tid + (j + 1) * kBlock, nr - 1);
                fin_load(a, q, n + r0 + i, P.fq[j]);
                P.bq[j] = p.b[r0 + i];
            }
        }
        psd_apply_sel<MAXKP, LR>(p.psd_lr, u.begin, k, Ld, sm, Bg);  // ends with a barrier
    } else if (u.type == U_SOC) {
        int cr0 = 0, cdim = 0;
        if (cone < u.end) {
            const double *par = p.soc_par + 4 * cone;
            P.cp[0] = par[0]; P.cp[1] = par[1]; P.cp[2] = par[2]; P.cp[3] = par[3];
            cr0 = p.soc_row[cone];
            cdim = p.soc_dim[cone];
        }
        // the first kSocPref entries of u are loaded ahead, the rest (longer cones) after the
        // rows; yrows has barriers, so every thread takes the same path to it
        double upre[kSocPref];
#pragma unroll
        for (int j = 0; j < kSocPref; ++j) upre[j] = j < cdim - 1 ? p.zy[cr0 + 1 + j] : 0.0;
        if (TROWS) trows(0); else yrows();
#pragma unroll
        for (int j = 0; j < kSocPref; ++j)
            if (j < cdim - 1) ub[cr0 - r0 + 1 + j] = upre[j] * P.cp[1];
        for (int j = kSocPref; j < cdim - 1; ++j) ub[cr0 - r0 + 1 + j] = p.zy[cr0 + 1 + j] * P.cp[1];
        __syncthreads();
        if (cone < u.end) soc_apply(P.cp, ub, cr0 - r0, cdim, tin, jout);
        __syncthreads();
    } else {  // exponential cones: each cone's 3x3 Jacobian staged in ub
        double J[9];
        const bool own = cone < u.end;
#pragma unroll
        for (int j = 0; j < 9; ++j) J[j] = own ? p.exp_J[9 * cone + j] : 0.0;
        if (TROWS) trows(0); else yrows();
        if (own) {
#pragma unroll
            for (int j = 0; j < 9; ++j) ub[9 * tid + j] = J[j];
        }
        __syncthreads();
        if (own) exp_apply(J, exp_row(p, cone) - r0, tin, jout);
        __syncthreads();
    }
}

// CL: the cone launch (k_loop_FT_cones): low-rank PSD Jacobians, and the loads of four rows
// per thread in flight in the row loops
template <int MAXKP = 64, bool CL = false>
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
    if (u.type == U_PSDROWS) return;
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
    const int nr = unit_rows(u, r0);
    double *tb, *rb, *jt, *ub, *gb;
    unit_bufs(p, u, sm, nr, tb, rb, jt, ub, gb);
    (void)gb;
    const bool psd = u.type == U_PSD;
    const int k = u.k, ld = psd ? psd_lds(k).ld : 0;
    if constexpr (CL) {  // as below, the operands of four rows per thread loaded first
        auto fin_row = [&](int i, const Fin &f) {
            int ii = P.ii, jj = P.jj;
            if (psd && i != tid) svec_rc(i, k, ii, jj);
            const double jv = psd ? smat_get(sm, ld, ii, jj) : jt[i];
            const double o = fin_store(a, c, n + r0 + i, f, (jv + rb[i]) * c.inv, s0);
            rb[i] = f.nxs * o;
            if (psd && a.do_pre) smat_put(sm, ld, ii, jj, rb[i]);
        };
        int from = tid;
        if (psd) {  // the first rows from the operands unit_pre loaded
#pragma unroll
            for (int j = 0; j <= kPostPref; ++j) {
                const int i = tid + j * kBlock;
                if (i < nr) fin_row(i, j == 0 ? P.f : P.fq[j - 1]);
            }
            from = tid + (kPostPref + 1) * kBlock;
        }
        constexpr int R = 4;
        for (int i0 = from; i0 < nr; i0 += R * kBlock) {
            Fin f[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = i0 + j * kBlock;
                if (i == tid) f[j] = P.f;
                else if (i < nr) fin_load(a, q, n + r0 + i, f[j]);
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = i0 + j * kBlock;
                if (i >= nr) break;
                fin_row(i, f[j]);
            }
        }
    } else {
        for (int i = tid; i < nr; i += kBlock) {
            Fin f;
            if (i == tid) f = P.f;
            else fin_load(a, q, n + r0 + i, f);
            int ii = P.ii, jj = P.jj;
            if (psd && i != tid) svec_rc(i, k, ii, jj);
            // PSD: J t is the matrix Y in the X region; each thread reads its own lower-triangle
            // entries before it writes them, and no thread reads the upper triangle
            const double jv = psd ? smat_get(sm, ld, ii, jj) : jt[i];
            const double o = fin_store(a, c, n + r0 + i, f, (jv + rb[i]) * c.inv, s0);
            rb[i] = f.nxs * o;  // the next product's input, in place of r_y
            if (psd && a.do_pre) smat_put(sm, ld, ii, jj, rb[i]);
        }
    }
    if (!a.do_pre) return;
    __syncthreads();
    // J of the next product with F, on the scaled outputs (factors still staged)
    auto oin = [&](int i) { return rb[i]; };
    auto jout = [&](int i, double v) { jt[i] = v; };
    if (psd) {
        const double *Bg = p.psd_pool + u.voff + k * k;
        psd_apply_sel<MAXKP, CL>(p.psd_lr, u.begin, k, psd_lds(k), sm, Bg);  // Y in X
        for (int i = tid; i < nr; i += kBlock) {
            int ii = P.ii, jj = P.jj;
            if (i != tid) svec_rc(i, k, ii, jj);
            jt[i] = smat_get(sm, ld, ii, jj);
        }
    } else {
        const int cone = u.begin + tid;
        if (cone < u.end) {
            if (u.type == U_SOC) soc_apply(P.cp, ub, p.soc_row[cone] - r0, p.soc_dim[cone], oin, jout);
            else exp_apply(ub + 9 * tid, exp_row(p, cone) - r0, oin, jout);
        }
        __syncthreads();
    }
    if constexpr (CL) {
        int from = tid;
        if (psd) {
#pragma unroll
            for (int j = 0; j <= kPostPref; ++j) {
                const int i = tid + j * kBlock;
                if (i < nr) {
                    const double w = jt[i];
                    a.wy[r0 + i] = w;
                    s1 -= (j == 0 ? P.bv : P.bq[j - 1]) * w;
                }
            }
            from = tid + (kPostPref + 1) * kBlock;
        }
        constexpr int R = 4;
        for (int i0 = from; i0 < nr; i0 += R * kBlock) {
            double bb[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = i0 + j * kBlock;
                bb[j] = i >= nr ? 0.0 : i == tid ? P.bv : p.b[r0 + i];
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = i0 + j * kBlock;
                if (i < nr) {
                    const double w = jt[i];
                    a.wy[r0 + i] = w;
                    s1 -= bb[j] * w;
                }
            }
        }
    } else {
        for (int i = tid; i < nr; i += kBlock) {
            const double w = jt[i];
            a.wy[r0 + i] = w;
            s1 -= (i == tid ? P.bv : p.b[r0 + i]) * w;
        }
    }
}

// MULTI: a workgroup runs units blockIdx.x, blockIdx.x + gridDim.x, ... (launches with
// fewer workgroups than units); else exactly unit blockIdx.x. The single-unit form needs
// about half the registers (a loop around the unit code keeps more of it live), so it runs
// at twice the occupancy.
template <bool MULTI, bool DEEP>
__device__ inline void loop_FT_body(const Problem &p, const StepArgs &a, const FusedGrid &g,
                                    double *sm, LsqrState &S) {
    Entry e;
    const Ptrs q = ptrs_of(p, a);
    const double in_N_raw = in_raw(a, q, p.N - 1);
    UnitPre P;
    Ctx c;
    double s0 = 0.0, s1 = 0.0;
    if (!MULTI) {
        const Unit u = g.units[blockIdx.x];
        unit_pre<DEEP>(p, a, q, g.lx, g.ly, u, sm, in_N_raw, P);
        entry_issue(a, e);  // after the unit's loads: the memory counter is in order
        if (!entry_finish(a, e, &S, 1)) return;
        c = scalars(a, S, q, in_N_raw);
        unit_post(p, a, q, c, u, sm, P, s0, s1);
    } else {
        for (int ui = blockIdx.x; ui < g.nunits; ui += gridDim.x) {
            if (ui != (int)blockIdx.x) __syncthreads();  // LDS of the previous unit is free
            const Unit u = g.units[ui];
            unit_pre<DEEP>(p, a, q, g.lx, g.ly, u, sm, in_N_raw, P);
            if (ui == (int)blockIdx.x) {
                entry_issue(a, e);
                if (!entry_finish(a, e, &S, 1)) return;
                c = scalars(a, S, q, in_N_raw);
            }
            unit_post(p, a, q, c, u, sm, P, s0, s1);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // the tau entry
        const int N = p.N;
        Fin f;
        fin_load(a, q, N - 1, f);
        fin_store(a, c, N - 1, f, S.dot_adj * c.inv + p.xPx * c.in_N, s0);
    }
    leave(a, s0, s1, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_loop_FT(Problem p, StepArgs a, FusedGrid g) {
    extern __shared__ double sm[];
    LsqrState S;  // per thread (entry_finish)
    loop_FT_body<false, false>(p, a, g, sm, S);
}

__global__ __launch_bounds__(kBlock) void k_loop_FT_multi(Problem p, StepArgs a, FusedGrid g) {
    extern __shared__ double sm[];
    LsqrState S;
    loop_FT_body<true, false>(p, a, g, sm, S);
}

__global__ __launch_bounds__(kBlock) void k_loop_FT_deep(Problem p, StepArgs a, FusedGrid g) {
    extern __shared__ double sm[];
    LsqrState S;
    loop_FT_body<false, true>(p, a, g, sm, S);
}

__global__ __launch_bounds__(kBlock) void k_loop_FT_multi_deep(Problem p, StepArgs a, FusedGrid g) {
    extern __shared__ double sm[];
    LsqrState S;
    loop_FT_body<true, true>(p, a, g, sm, S);
}

// g.units[i] by scalar loads (the table is constant during a launch): its words read
// through a pointer into the constant address space
__device__ inline Unit unit_at(const Unit *units, int i) {
    using CWord = const __attribute__((address_space(4))) int;
    constexpr int NW = sizeof(Unit) / sizeof(int);
    static_assert(NW * sizeof(int) == sizeof(Unit), "whole words");
    CWord *w = (CWord *)(units + i);
    int v[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) v[j] = w[j];
    Unit u;
    __builtin_memcpy(&u, v, sizeof(Unit));
    return u;
}

// The cone units of a product with F' whose rows launch (k_loop_FT* with U_PSDROWS units,
// or k_loop_FT_xs) left their raw rows t = A r_x - b r_N - r_y in a.tmp: one workgroup per
// unit (a PSD cone, or a run of SOC or exponential cones), the scalars of the state that
// launch finalised (a.st), partial sums from slot a.slot0 on. Large PSD cones stage up to
// 130 KB of LDS; in their own launch they no longer hold every other unit to one workgroup
// per CU.
__global__ __launch_bounds__(kBlock) void k_loop_FT_cones(Problem p, StepArgs a, FusedGrid g) {
    extern __shared__ double sm[];
    // the unit first, through the scalar cache (read only here): the loads of its factors
    // and rows depend on it, and in vector registers its fields would wait for every vector
    // load issued before their first use (the raw rows come from a.tmp, so unit_pre does
    // not read in_N_raw)
    const Unit u = unit_at(g.units, blockIdx.x);
    const Ptrs q = ptrs_of(p, a);
    UnitPre P;
    unit_pre<false, 64, true, true>(p, a, q, g.lx, g.ly, u, sm, 0.0, P);
    const double in_N_raw = in_raw(a, q, p.N - 1);
    const LsqrState S = *a.st;
    if (S.done) return;
    const Ctx c = scalars(a, S, q, in_N_raw);
    double s0 = 0.0, s1 = 0.0;
    unit_post<64, true>(p, a, q, c, u, sm, P, s0, s1);
    leave(a, s0, s1, a.slot0 + blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// products with the input's x part staged in LDS
//
// When n doubles fit in LDS, (isc o in)_x is staged there by every workgroup (kXsBlock
// threads, one workgroup per CU), and the CSR sums with P and A gather from LDS instead of
// through the L1 and L2 caches (one 8-byte entry per 128-byte line on random columns).
// The workgroup's waves then take 64-thread blocks of rows round robin over the launch.
// The sums with A' gather the y part (m long) from global memory. Product with F: x rows,
// y rows and the tau row, as k_loop_F. Product with F': x rows and the diagonal y rows are
// finished here, the raw rows of the cones go to a.tmp for k_loop_FT_cones (their blocks
// of J are not diagonal), and the tau entry is finished by the first thread.
// ---------------------------------------------------------------------------------------

struct XsPre {
    int idx;  // output entry of this thread (lane 0 of its row group), or -1
    double acc, accT;
    double coef;  // F: q (x rows) or b (y rows); F': c (x rows) or b (diagonal rows)
    double self;  // y rows: (isc o in) at the row
    double aux;   // F y rows: J applied to the previous input at the row; F': diag of J
    Fin f;
};

template <bool FT>
__device__ inline void xs_pre(const Problem &p, const StepArgs &a, const Ptrs &q,
                              const double *xs, const XsGrid &g, int wb, int lane64,
                              double in_N_raw, XsPre &r) {
    const int n = p.n, m = p.m, N = p.N;
    const bool xr = wb < g.bxw;
    const int L = xr ? g.lx : g.ly;
    const long long gt = (long long)(xr ? wb : wb - g.bxw) * kWave + lane64;
    const int row = (int)(gt / L), lane = (int)(gt & (L - 1));
    // this thread's output entry (lane 0 of its row group) and its operands, loaded before
    // the sums so that they arrive with them (no arithmetic on them until the sums are done:
    // a product here would wait for the loads before the sums' own loads are issued)
    int idx = -1;
    if (lane == 0) {
        if (xr) idx = row < n ? row : -1;
        else if (row < m) idx = n + row;
        else if (!FT && row == m) idx = N - 1;
    }
    double coef = 0.0, self = 0.0, self_sc = 1.0, aux = 0.0;
    bool cone_row = false;
    if (idx >= 0 && idx < n) {
        coef = FT ? p.c[idx] : p.q[idx];
    } else if (idx >= n && idx < N - 1) {
        const int y = idx - n;
        self = a.in[idx];
        if (q.isc) self_sc = q.isc[idx];
        coef = p.b[y];
        cone_row = FT && y >= p.n_diag;  // its raw row goes to the cone launch
        if (!cone_row) aux = FT ? p.jdiag[y] : a.wy[y];
    }
    if (idx >= 0 && !cone_row) fin_load(a, q, idx, r.f);
    double acc = 0.0, accT = 0.0;
    if (xr) {
        if (row < n) {
            // the first pass of the A' sums loaded before P's quads: its column and value
            // loads are in flight while P's sums run, its gathers follow them
            const int t0 = p.Trp[row], t1 = p.Trp[row + 1];
            const double *Tv = FT ? q.Tv : p.Tv;
            Pass4 tp;
            pass4_load(p.Tci, Tv, t0 + lane, t1, L, FT ? n : 0, tp);
            acc = csr_dot_quads(p.Prp4, p.Pc4, p.Pv4, row, lane, L, xs);
            if (!FT) accT = csr_dot4_from<false>(tp, p.Tci, Tv, t0, t1, lane, L, a.wy, nullptr, 0);
            else if (q.gsc) accT = csr_dot4_from<true>(tp, p.Tci, Tv, t0, t1, lane, L, a.in, q.gsc, n);
            else accT = csr_dot4_from<false>(tp, p.Tci, Tv, t0, t1, lane, L, a.in, nullptr, n);
        }
    } else if (row < m) {
        acc = csr_dot_quads(p.Arp4, p.Ac4, p.Av4, row, lane, L, xs);
    }
    r.acc = group_sum_dpp(acc, L);
    r.accT = group_sum_dpp(accT, L);
    if (q.isc) self *= self_sc;  // in_raw of the row's own entry
    if (cone_row) {
        a.tmp[idx] = r.acc - coef * in_N_raw - self;
        idx = -1;
    }
    r.idx = idx;
    r.coef = coef;
    r.self = self;
    r.aux = aux;
}

template <bool FT>
__device__ inline void xs_post(const Problem &p, const StepArgs &a, const Ctx &c,
                               const LsqrState &S, const XsPre &r, double &s0, double &s1) {
    const int n = p.n, N = p.N;
    if (r.idx < 0) return;
    if (FT) {
        if (r.idx < n) {
            const double o = fin_store(a, c, r.idx, r.f, (r.acc - r.accT) * c.inv + r.coef * c.in_N, s0);
            if (a.do_pre) s1 += r.coef * r.f.nxs * o;
        } else {
            const double t = (r.acc - r.self) * c.inv - r.coef * c.in_N;
            const double o = fin_store(a, c, r.idx, r.f, r.aux * t + r.self * c.inv, s0);
            if (a.do_pre) {
                const double w = r.aux * r.f.nxs * o;
                a.wy[r.idx - n] = w;
                s1 -= r.coef * w;
            }
        }
        return;
    }
    double val;
    if (r.idx < n)
        val = (r.acc + r.accT) * c.inv + r.coef * c.in_N;
    else if (r.idx < N - 1)
        val = (r.self - r.acc - r.aux) * c.inv + r.coef * c.in_N;
    else
        val = S.dot_fwd * c.inv + p.xPx * c.in_N;
    const double o = fin_store(a, c, r.idx, r.f, val, s0);
    if (r.idx < N - 1) s1 += r.coef * r.f.nxs * o;
}

template <bool FT>
__device__ inline void loop_xs_body(const Problem &p, const StepArgs &a, const XsGrid &g,
                                    double *xs) {
    constexpr int kW = kXsBlock / kWave;
    const int tid = threadIdx.x;
    const Ptrs q = ptrs_of(p, a);
    for (int j = tid; j < p.n; j += kXsBlock) xs[j] = in_raw(a, q, j);
    const double in_N_raw = in_raw(a, q, p.N - 1);
    __syncthreads();
    const int lane64 = tid & (kWave - 1), total = g.total(), W = gridDim.x * kW;
    int wb = blockIdx.x * kW + tid / kWave;
    XsPre r;
    r.idx = -1;
    if (wb < total) xs_pre<FT>(p, a, q, xs, g, wb, lane64, in_N_raw, r);
    EntryT<kXsBlock> e;
    entry_issue(a, e);  // after the first rows' loads: the memory counter is in order
    LsqrState S;
    if (!entry_finish(a, e, &S, FT ? 1 : 0)) return;
    const Ctx c = scalars(a, S, q, in_N_raw);
    double s0 = 0.0, s1 = 0.0;
    xs_post<FT>(p, a, c, S, r, s0, s1);
    for (wb += W; wb < total; wb += W) {
        xs_pre<FT>(p, a, q, xs, g, wb, lane64, in_N_raw, r);
        xs_post<FT>(p, a, c, S, r, s0, s1);
    }
    if (FT && blockIdx.x == 0 && tid == 0) {  // the tau entry
        const int N = p.N;
        Fin f;
        fin_load(a, q, N - 1, f);
        fin_store(a, c, N - 1, f, S.dot_adj * c.inv + p.xPx * c.in_N, s0);
    }
    leave<kXsBlock>(a, s0, s1, blockIdx.x);
}

__global__ __launch_bounds__(kXsBlock) void k_loop_F_xs(Problem p, StepArgs a, XsGrid g) {
    extern __shared__ double xs[];
    loop_xs_body<false>(p, a, g, xs);
}

__global__ __launch_bounds__(kXsBlock) void k_loop_FT_xs(Problem p, StepArgs a, XsGrid g) {
    extern __shared__ double xs[];
    loop_xs_body<true>(p, a, g, xs);
}

// The packed copy of a CSR matrix whose columns are below 65 536 (P's and A's columns index
// x, whose n doubles the staged kernels hold in LDS): one thread per row copies its entries
// to the row's padded start and fills the rest of its last quad with column 0, value 0.
__global__ void k_pack_rows(const int *rp, const int *ci, const double *v, const int *rp4,
                            unsigned short *c4, double *v4, int rows) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int k0 = rp[r], k1 = rp[r + 1], o = rp4[r], o1 = rp4[r + 1];
    for (int k = k0; k < k1; ++k) {
        c4[o + k - k0] = (unsigned short)ci[k];
        v4[o + k - k0] = v[k];
    }
    for (int t = o + (k1 - k0); t < o1; ++t) {
        c4[t] = 0;
        v4[t] = 0.0;
    }
}

// ---------------------------------------------------------------------------------------
// segmented form: the LSQR loops of many problems (the batch, one block-diagonal union)
// advanced together. Every work item belongs to one problem; each problem has its own state
// (double-buffered, one per problem) and reduces its own items' partial sums, in item order,
// at the entry of the next launch. Items of finished problems exit at entry; the first item
// of a problem counts the problem in *ndone when its stop decision is taken.
// ---------------------------------------------------------------------------------------

struct SegEntry {
    LsqrState st;
    double pa[kPartRegs], pb[kPartRegs];
    int c0, cnt;  // the problem's partial slots in the previous launch
};

__device__ inline void seg_entry_issue(const StepArgs &a, int b, const int *prev_off, SegEntry &e) {
    e.st = a.st[b];
    e.c0 = prev_off[b];
    e.cnt = prev_off[b + 1] - e.c0;
#pragma unroll
    for (int j = 0; j < kPartRegs; ++j) {
        const int i = threadIdx.x + j * kBlock;
        const int slot = e.c0 + min(i, max(e.cnt - 1, 0));  // in bounds; masked below
        const double2 v = reinterpret_cast<const double2 *>(a.part_prev)[slot];
        e.pa[j] = v.x;
        e.pb[j] = v.y;
    }
}

__device__ inline bool seg_entry_finish(const StepArgs &a, const SegEntry &e, int b, bool first,
                                        int *ndone, LsqrState *S, int my_fwd) {
    const int tid = threadIdx.x;
    if (e.st.done) {
        if (first && tid == 0) a.st_next[b] = e.st;
        return false;
    }
    double t0 = 0.0, t1 = 0.0;
    if (e.st.pend_role >= 0) {
#pragma unroll
        for (int j = 0; j < kPartRegs; ++j)
            if (tid + j * kBlock < e.cnt) {
                t0 += e.pa[j];
                t1 += e.pb[j];
            }
        for (int i = tid + kPartRegs * kBlock; i < e.cnt; i += kBlock) {  // very large problems
            const double2 v = reinterpret_cast<const double2 *>(a.part_prev)[e.c0 + i];
            t0 += v.x;
            t1 += v.y;
        }
        block_sum2_all(t0, t1);
    }
    LsqrState s = e.st;  // per thread, as entry_finish
    if (s.pend_role >= 0) finalize(&s, s.pend_role, t0, t1, s.pend_fwd != 0);
    if (s.done) {
        s.pend_role = -1;
    } else {
        s.pend_role = a.role;
        s.pend_fwd = my_fwd;
    }
    if (first && tid == 0) {  // as entry_finish: never the buffer this launch reads
        a.st_next[b] = s;
        if (s.done) atomicAdd(ndone, 1);
    }
    *S = s;
    return !s.done;
}

// rows of one item of the product with F (x rows: P and A'wy; y rows: A), as rows_pre
__device__ inline void seg_rows_pre(const Problem &p, const StepArgs &a, const Ptrs &q,
                                    const SegItem &it, int L, RowPre &r) {
    const int n = p.n;
    const int tid = threadIdx.x, lane = tid & (L - 1), row = it.begin + tid / L;
    double acc = 0.0, accT = 0.0;
    if (row < it.end) {
        if (it.type == 0) {
            acc = csr_dot_d<true>(p.Pci, q.Pv, p.Prp[row], p.Prp[row + 1], lane, L, a.in, q.gsc, 0);
            accT = csr_dot_d<true>(p.Tci, p.Tv, p.Trp[row], p.Trp[row + 1], lane, L, a.wy, nullptr, 0);
        } else {
            acc = csr_dot_d<true>(p.Aci, q.Av, p.Arp[row], p.Arp[row + 1], lane, L, a.in, q.gsc, 0);
        }
    }
    r.acc = group_sum_dpp(acc, L);
    r.accT = group_sum_dpp(accT, L);
    r.idx = (lane == 0 && row < it.end) ? (it.type == 0 ? row : n + row) : -1;
    double qb = 0.0, self = 0.0, wyr = 0.0;
    if (r.idx >= 0) {
        fin_load(a, q, r.idx, r.f);
        if (it.type == 0) {
            qb = p.q[row];
        } else {
            qb = p.b[row];
            self = in_raw(a, q, r.idx);
            wyr = a.wy[row];
        }
    }
    r.qb = qb;
    r.self = self;
    r.wyr = wyr;
}

__device__ inline void seg_rows_post(const StepArgs &a, const Ctx &c, const SegItem &it,
                                     const RowPre &r, double &s0, double &s1) {
    if (r.idx < 0) return;
    const double val = it.type == 0 ? (r.acc + r.accT) * c.inv + r.qb * c.in_N
                                    : (r.self - r.acc - r.wyr) * c.inv + r.qb * c.in_N;
    const double o = fin_store(a, c, r.idx, r.f, val, s0);
    s1 += r.qb * r.f.nxs * o;
}

__global__ __launch_bounds__(kBlock) void k_seg_F(Problem p, StepArgs a, SegGrid g) {
    LsqrState S;  // per thread (entry_finish)
    const SegItem it = g.fitems[blockIdx.x];
    const int slot = g.fslot ? g.fslot[blockIdx.x] : (int)blockIdx.x;
    const int b = it.prob;
    const bool first = slot == g.foff[b];
    SegEntry e;
    seg_entry_issue(a, b, g.toff, e);
    const Ptrs q = ptrs_of(p, a);
    const int tix = p.n + p.m + b;
    const double in_N_raw = in_raw(a, q, tix);
    RowPre r;
    seg_rows_pre(p, a, q, it, it.type == 0 ? g.lxs[b] : g.lys[b], r);
    if (!seg_entry_finish(a, e, b, first, g.ndone, &S, 0)) return;
    const Ctx c = scalars(a, S, q, in_N_raw);
    double s0 = 0.0, s1 = 0.0;
    seg_rows_post(a, c, it, r, s0, s1);
    if (first && threadIdx.x == 0) {  // the problem's tau entry
        Fin f;
        fin_load(a, q, tix, f);
        fin_store(a, c, tix, f, S.dot_fwd * c.inv + g.xPx[b] * c.in_N, s0);
    }
    leave(a, s0, s1, slot);
}

template <int MAXKP>
__device__ inline void seg_FT_body(const Problem &p, const StepArgs &a, const SegGrid &g,
                                   double *sm) {
    LsqrState S;  // per thread (entry_finish)
    const Unit u = g.tunits[blockIdx.x];
    const int b = g.tprob[blockIdx.x];
    const int slot = g.tslot ? g.tslot[blockIdx.x] : (int)blockIdx.x;
    const bool first = slot == g.toff[b];
    SegEntry e;
    seg_entry_issue(a, b, g.foff, e);
    const Ptrs q = ptrs_of(p, a);
    const int tix = p.n + p.m + b;
    const double in_N_raw = in_raw(a, q, tix);
    UnitPre P;
    unit_pre<true, MAXKP>(p, a, q, g.lxs[b], g.lys[b], u, sm, in_N_raw, P);
    if (!seg_entry_finish(a, e, b, first, g.ndone, &S, 1)) return;
    const Ctx c = scalars(a, S, q, in_N_raw);
    double s0 = 0.0, s1 = 0.0;
    unit_post<MAXKP>(p, a, q, c, u, sm, P, s0, s1);
    if (first && threadIdx.x == 0) {  // the problem's tau entry
        Fin f;
        fin_load(a, q, tix, f);
        fin_store(a, c, tix, f, S.dot_adj * c.inv + g.xPx[b] * c.in_N, s0);
    }
    leave(a, s0, s1, slot);
}

__global__ __launch_bounds__(kBlock) void k_seg_FT(Problem p, StepArgs a, SegGrid g) {
    extern __shared__ double sm[];
    seg_FT_body<64>(p, a, g, sm);
}

// batches whose PSD cones all have order <= 16: one product instance, fewer registers
__global__ __launch_bounds__(kBlock) void k_seg_FT_small(Problem p, StepArgs a, SegGrid g) {
    extern __shared__ double sm[];
    seg_FT_body<16>(p, a, g, sm);
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------

__global__ void k_unit_ranges(Problem p, Unit *units, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Unit u = units[i];
    u.nrows = u.e0 = u.e1 = u.k = 0;
    if (u.type == U_PSD || u.type == U_SOC || u.type == U_EXP) {
        int r0;
        u.nrows = unit_rows_of(p, u, r0);
        u.e0 = p.Arp[r0];
        u.e1 = p.Arp[r0 + u.nrows];
        if (u.type == U_PSD) {
            u.k = p.psd_k[u.begin];
            u.voff = p.psd_off[u.begin];
        }
    }
    units[i] = u;
}

__global__ void k_scale_vals(const int *col, const double *val, long long nnz, const double *sc,
                             int off, double *out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) out[i] = val[i] * sc[off + col[i]];
}

void launch_scale_vals(const int *col, const double *val, long long nnz, const double *sc,
                       int off, double *out, hipStream_t s) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_scale_vals, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           col, val, nnz, sc, off, out);
}

void fill_unit_ranges(const Problem &p, Unit *units, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_unit_ranges, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, units, n);
}

int loop_lds_bytes(const int *psd_orders, int n_psd) {
    int need = 4 * kUnitRows;
    for (int i = 0; i < n_psd; ++i) {
        const PsdLds L = psd_lds(psd_orders[i]);
        need = std::max({need, L.tb + 3 * L.nr, L.gb + kGather});
    }
    return (int)sizeof(double) * need;
}

void set_loop_kernel_lds(int bytes) {
    (void)hipFuncSetAttribute((const void *)k_loop_FT_cones, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void *)k_loop_FT, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void *)k_loop_FT_multi, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void *)k_loop_FT_deep, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void *)k_loop_FT_multi_deep, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void launch_loop_F(const Problem &p, const StepArgs &a, const RowGrid &g, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_loop_F, dim3(grid), dim3(kBlock), 0, s, p, a, g);
}

void launch_loop_FT(const Problem &p, const StepArgs &a, const FusedGrid &g, int lds, int grid,
                    hipStream_t s) {
    const bool one = grid >= g.nunits;
    if (one) grid = g.nunits;
    if (g.deep)
        hipLaunchKernelGGL(one ? k_loop_FT_deep : k_loop_FT_multi_deep, dim3(grid), dim3(kBlock), lds, s, p, a, g);
    else
        hipLaunchKernelGGL(one ? k_loop_FT : k_loop_FT_multi, dim3(grid), dim3(kBlock), lds, s, p, a, g);
}

void launch_loop_FT_cones(const Problem &p, const StepArgs &a, const FusedGrid &g, int lds,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_loop_FT_cones, dim3(g.nunits), dim3(kBlock), lds, s, p, a, g);
}

int xs_lds_bytes(int n) { return (int)sizeof(double) * n; }

void launch_pack_rows(const int *rp, const int *ci, const double *v, const int *rp4,
                      unsigned short *c4, double *v4, int rows, hipStream_t s) {
    if (rows > 0)
        hipLaunchKernelGGL(k_pack_rows, dim3(div_up(rows, kBlock)), dim3(kBlock), 0, s, rp, ci, v,
                           rp4, c4, v4, rows);
}

void set_xs_kernel_lds(int bytes) {
    (void)hipFuncSetAttribute((const void *)k_loop_F_xs, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void *)k_loop_FT_xs, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void launch_loop_xs(const Problem &p, const StepArgs &a, const XsGrid &g, bool ft, int grid,
                    hipStream_t s) {
    hipLaunchKernelGGL(ft ? k_loop_FT_xs : k_loop_F_xs, dim3(grid), dim3(kXsBlock), xs_lds_bytes(p.n), s, p, a, g);
}

void set_seg_kernel_lds(int bytes) {
    (void)hipFuncSetAttribute((const void *)k_seg_FT, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void *)k_seg_FT_small, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void launch_seg_F(const Problem &p, const StepArgs &a, const SegGrid &g, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_F, dim3(g.nf), dim3(kBlock), 0, s, p, a, g);
}

void launch_seg_FT(const Problem &p, const StepArgs &a, const SegGrid &g, int lds, hipStream_t s) {
    if (g.small_psd)
        hipLaunchKernelGGL(k_seg_FT_small, dim3(g.nt), dim3(kBlock), lds, s, p, a, g);
    else
        hipLaunchKernelGGL(k_seg_FT, dim3(g.nt), dim3(kBlock), lds, s, p, a, g);
}

}  // namespace qcpd
