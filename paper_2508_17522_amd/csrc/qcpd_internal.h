// Internal device data layout and helpers shared by the library's HIP sources.
// gfx950 only: 64-lane wavefronts, 256-thread workgroups, FP64 arithmetic throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qcpd.h"

namespace qcpd {

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kWave = 64;
constexpr int kMaxPsd = 64;      // largest PSD order kept in LDS
constexpr int kMaxLoopGrid = 1024;  // most workgroups of one LSQR-loop launch

// LSQR scalars live in device memory so that a captured graph of many iterations runs
// without host round trips; the host only reads `done` once per graph launch.
struct LsqrState {
    double alpha;     // ||v~||  (v = v~ / alpha)
    double beta;      // ||u~||  (u = u~ / beta)
    double rhobar, phibar, beta1;
    double phr, thr;  // phi/rho and theta/rho of the last rotation (pending x, w update)
    double dot_fwd;   // c'(s o in)_x - b'(J s o in)_y for the next product with F
    double dot_adj;   // q'(s o in)_x + b'(s o in)_y for the next product with F'
    double one;       // 1.0: normaliser for plain (non-LSQR) products
    double tol;
    double resid;     // explicit residual norm (absolute)
    double tau_rhs;   // scratch
    int32_t pending;  // an x/w update is owed (set by the v-step, cleared by the u-step)
    int32_t done;     // stop flag read by every kernel on entry
    int32_t iters;
    int32_t max_iter;
    int32_t conv;     // 1 when the stopping test passed
    // deferred protocol of the LSQR loop kernels: the role, block count and dot kind of the
    // partial sums the previous launch left for the next launch to finalise (-1: none)
    int32_t pend_role, pend_blocks, pend_fwd;
};

// Offsets of doubles inside LsqrState, used to select a normaliser by index.
enum NrmSel { NRM_ALPHA = 0, NRM_BETA = 1, NRM_ONE = 9 };

// Read-only view of one problem on the device (passed by value to kernels).
struct Problem {
    int n, m, N;
    int nnzP, nnzA;
    const int *Prp, *Pci;
    const double *Pv;
    const int *Arp, *Aci;
    const double *Av;
    const int *Trp, *Tci, *Tperm;   // A' in CSR and, per A' slot, the A slot it came from
    const double *Tv;
    const double *q, *b, *x, *y, *s;
    const double *c;                // c = -2Px - q (the tau-row of D_u Q at tau = 1)
    const double *zy;               // z_y = y - s
    double xPx;
    // cones
    int n_diag;                     // zero + nonnegative rows (leading rows of y)
    const double *jdiag;            // diag of J for every y row
    int n_soc;
    const int *soc_row, *soc_dim;   // first y-row and dimension of each SOC
    const double *soc_par;          // 4 per cone: mode, 1/||u||, c1, c2
    int n_exp;
    int exp_row0;                   // first y-row of the exponential cones (3 rows each)
    const int *exp_rows;            // or, when not null, the first y-row of each cone
    const double *exp_J;            // 9 per cone, row-major, J of the dual exponential cone
    int n_psd;
    const int *psd_row, *psd_k;
    const long long *psd_off;       // offset of (V, B) in psd_pool, 2 k^2 doubles per cone
    const double *psd_pool;
    const int *psd_lr;              // per cone: the low-rank side of its Jacobian (c, + 256 when
                                    // it is the negative side), or null
    // packed copies of P and A for the staged kernels (or null): rows padded to whole quads of
    // entries (row starts Prp4 / Arp4, multiples of 4), 16-bit columns, padding 0 and 0.0
    const int *Prp4, *Arp4;
    const unsigned short *Pc4, *Ac4;
    const double *Pv4, *Av4;
};

// Cone-kernel grid: [elementwise | SOC | exp | PSD] block ranges.
struct ConeGrid {
    int nE;         // elementwise items: x-part (n) + diagonal y rows (n_diag) + tau (1)
    int bE, bS, bX, bP;
    int total() const { return bE + bS + bX + bP; }
};

// Rows-kernel grid: x rows with lx lanes each, then y rows (+ tau) with ly lanes each.
struct RowGrid {
    int lx, ly;
    int bx, by;
    int total() const { return bx + by; }
};

// LSQR loop kernels with the input's x part staged in LDS (loop.hip): one workgroup of
// kXsBlock threads per CU; x rows with lx lanes each in bxw blocks of 64 threads, then y rows
// (+ tau) with ly lanes each in byw blocks, taken by the waves round robin.
constexpr int kXsBlock = 1024;
struct XsGrid {
    int lx, ly;
    int bxw, byw;
    __host__ __device__ int total() const { return bxw + byw; }
};

// ---------------------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum of three values over the workgroup; result valid in thread 0.
__device__ inline void block_sum3(double &a, double &b, double &c) {
    __shared__ double sh[3][kBlock / kWave];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) { sh[0][w] = a; sh[1][w] = b; sh[2][w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = sh[0][0]; b = sh[1][0]; c = sh[2][0];
        for (int i = 1; i < kBlock / kWave; ++i) { a += sh[0][i]; b += sh[1][i]; c += sh[2][i]; }
    }
    __syncthreads();
}

__device__ inline void store_coherent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double load_coherent(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish this block's three partial sums (3 doubles per block in `partials`). Returns true
// in every thread of the last block to arrive; that block then holds the totals, summed in
// a fixed order so the result does not depend on which block arrived last. The last block
// also rearms the counter for the next launch.
__device__ inline bool last_block_sum3(double a, double b, double c, double *partials,
                                       int *counter, int nblocks, double tot[3]) {
    __shared__ int is_last;
    __shared__ double tsh[3];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) {
        store_coherent(&partials[3 * blockIdx.x], a);
        store_coherent(&partials[3 * blockIdx.x + 1], b);
        store_coherent(&partials[3 * blockIdx.x + 2], c);
        __threadfence();
        int t = atomicAdd(counter, 1);
        is_last = (t == nblocks - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double sa = 0.0, sb = 0.0, sc = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kBlock) {
        sa += load_coherent(&partials[3 * i]);
        sb += load_coherent(&partials[3 * i + 1]);
        sc += load_coherent(&partials[3 * i + 2]);
    }
    block_sum3(sa, sb, sc);
    if (threadIdx.x == 0) {
        tsh[0] = sa; tsh[1] = sb; tsh[2] = sc;
        __hip_atomic_store(counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    tot[0] = tsh[0]; tot[1] = tsh[1]; tot[2] = tsh[2];
    return true;
}

inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace qcpd

namespace qcpd {

// Roles of an operator product inside LSQR (Paige & Saunders bidiagonalisation):
//   U:     u~ <- op(in) - (alpha/beta) u~        (product with the LSQR matrix)
//   V:     v~ <- sc o op(in) - (beta/alpha) v~   (product with its transpose), then the
//          plane rotation and the convergence test
//   V0:    v~ <- sc o op(in)                     (first v of the bidiagonalisation)
//   RESID: out <- op(in) - rhs                   (explicit residual)
//   PLAIN: out <- op(in)
enum Role { ROLE_U = 0, ROLE_V = 1, ROLE_V0 = 2, ROLE_RESID = 3, ROLE_PLAIN = 4 };

struct StepArgs {
    const double *in;   // operator input buffer (N)
    int in_nrm;         // NrmSel: input is in / state[in_nrm]
    int in_is_v;        // the input is the v-side vector: read it through sc
    double *out;        // output buffer (N), updated in place
    int role;
    int out_is_v;       // the output is the v-side vector (scaled by sc)
    const double *sc;   // v-side (column) diagonal scale of the LSQR matrix, or null
    const double *scl;  // u-side (row) diagonal scale of the LSQR matrix, or null
    const double *rhs;  // ROLE_RESID right-hand side
    double *wy;         // J applied to the next product's y-input (unnormalised), m
    int do_pre;         // compute wy and the F tau-row dot for the next product
    int do_update;      // apply the owed LSQR x/w update (first kernel of an iteration)
    double *xk, *wk;    // LSQR iterate and direction (N)
    double *tmp;        // staging between the two kernels of a product with F' (N)
    double *partials;   // 3 doubles per block
    int *counter;
    LsqrState *st;
    int check_done;     // return at once when st->done is set (kernels inside the loop)
    // LSQR loop (loop.hip): read the state from st and the previous launch's partials from
    // part_prev (kMaxLoopGrid slots of two doubles, 16-byte aligned), finalise them at entry,
    // write the state to st_next and this launch's partials to part_next. No fences or
    // atomics: launch order gives visibility.
    LsqrState *st_next;
    const double *part_prev;
    double *part_next;
    // values of P, A and A' with the input scale of the launch folded into each entry
    // (val * isc[col], isc = sc or scl as in_is_v says), or null: the loop kernels then
    // gather isc per entry
    const double *Pvs, *Avs, *Tvs;
    // a product with F' in two launches (rows, then the cones): the rows launch counts
    // extra_slots more partial sums for the next launch to reduce; the cone launch writes its
    // partials from slot slot0 on
    int extra_slots, slot0;
};

// Work units of the fused product with F' (one workgroup each): x rows, diagonal y rows,
// runs of whole SOC or exponential cones, or one PSD cone. Rows of D_u Q' r for the unit
// are formed in LDS and the unit's block of J is applied to them in the same workgroup.
// U_PSDROWS (LSQR loop with the PSD cones in a launch of their own): rows of PSD cones whose
// raw CSR rows t = A r_x - b r_N - r_y go to StepArgs::tmp for that launch.
enum UnitType { U_XROWS = 0, U_DIAG = 1, U_SOC = 2, U_EXP = 3, U_PSD = 4, U_PSDROWS = 5 };
struct Unit {
    int type, begin, end, row0;  // row0: first y row of a cone run (SOC / exp / PSD)
    // cone runs, filled on the device once the CSR copies exist (fill_unit_ranges): the
    // number of y rows, the range [e0, e1) of their CSR entries in A, and a PSD cone's order
    // and the offset of its (V, B) in the factor pool (one dependent load less at the start
    // of a PSD unit)
    int nrows, e0, e1, k;
    long long voff;
};
constexpr int kUnitRows = 1024;   // most y rows staged by one SOC / exp unit

struct FusedGrid {
    int nunits;
    const Unit *units;   // device table
    int lx, ly;
    int deep = 0;        // the loop kernel keeps kDeep CSR entries per lane in flight
};

// host launchers (apply.hip)
void launch_fused_FT(const Problem &p, const StepArgs &a, const FusedGrid &g, int lds_bytes,
                     hipStream_t s, int grid = 0);
int fused_lds_bytes(int kmax);
int persistent_blocks_per_cu(int lds_bytes);
hipError_t launch_lsqr_persistent(const Problem &p, const StepArgs &fa, const StepArgs &ta,
                                  const RowGrid &rg, const FusedGrid &fg, int dir, LsqrState *st,
                                  double *partials, int grid, int lds, hipStream_t s);
void set_fused_kernel_lds(int bytes);
void launch_rows_F(const Problem &p, const StepArgs &a, const RowGrid &g, hipStream_t s, int grid = 0);
void launch_cone_pre(const Problem &p, const StepArgs &a, const ConeGrid &g, int lds_bytes,
                     hipStream_t s);
void launch_state_init(LsqrState *st, double tol, int max_iter, hipStream_t s);
void launch_fill(double *p, long long n, double v, hipStream_t s);
void launch_flush(const Problem &p, const StepArgs &a, double *sol, int nblk, hipStream_t s);
void launch_adj_dot(const Problem &p, const StepArgs &a, hipStream_t s);
void launch_jvp_rhs(const Problem &p, const StepArgs &a, const RowGrid &g, const double *dP,
                    const double *dA, const double *dq, const double *db, hipStream_t s);
void launch_vjp_rhs(const Problem &p, const StepArgs &a, const ConeGrid &g, int lds_bytes,
                    const double *gx, const double *gy, const double *gs, hipStream_t s);
void launch_jvp_out(const Problem &p, const double *sol, const double *wy, double *dx,
                    double *dy, double *ds, hipStream_t s);
void launch_vjp_out(const Problem &p, const RowGrid &g, const double *w, double *dP,
                    double *dA, double *dq, double *db, hipStream_t s);
void launch_nan_scan(const double *const *ptrs, const long long *lens, int nseg, int *flag,
                     hipStream_t s);

// segmented LSQR loop of a batch (loop.hip): items of the product with F (x rows or y rows
// of one problem, at most kBlock / lanes rows) and units of the fused product with F' (each
// within one problem, at most kBlock / lanes rows for x and diagonal units), both grouped by
// problem; st / st_next of the StepArgs point to one state per problem.
struct SegItem {
    int type;  // 0: x rows, 1: y rows
    int begin, end, prob;
};
struct SegGrid {
    int B, nf, nt;        // items launched (all, or those of the running problems)
    const SegItem *fitems;
    const int *foff;      // B + 1: items of problem b are [foff[b], foff[b + 1]) (all items)
    const Unit *tunits;
    const int *tprob;     // problem of each F' unit
    const int *toff;      // B + 1
    // launched item i is item fslot[i] / tslot[i] of the full lists (its partial-sum slot);
    // null: the launch covers every item in order
    const int *fslot, *tslot;
    int small_psd;        // every PSD cone of the batch has order <= 16
    const int *lxs, *lys; // lanes per CSR row, per problem
    const double *xPx;    // per problem
    int *ndone;           // problems whose LSQR has stopped
};
void set_seg_kernel_lds(int bytes);
void launch_seg_F(const Problem &p, const StepArgs &a, const SegGrid &g, hipStream_t s);
void launch_seg_FT(const Problem &p, const StepArgs &a, const SegGrid &g, int lds, hipStream_t s);

// the LSQR loop (loop.hip)
void fill_unit_ranges(const Problem &p, Unit *units, int n, hipStream_t s);
void launch_scale_vals(const int *col, const double *val, long long nnz, const double *sc,
                       int off, double *out, hipStream_t s);
int loop_lds_bytes(const int *psd_orders, int n_psd);
void set_loop_kernel_lds(int bytes);
void launch_loop_F(const Problem &p, const StepArgs &a, const RowGrid &g, int grid, hipStream_t s);
void launch_loop_FT(const Problem &p, const StepArgs &a, const FusedGrid &g, int lds, int grid,
                    hipStream_t s);
void launch_loop_FT_cones(const Problem &p, const StepArgs &a, const FusedGrid &g, int lds,
                          hipStream_t s);
int xs_lds_bytes(int n);
void set_xs_kernel_lds(int bytes);
void launch_loop_xs(const Problem &p, const StepArgs &a, const XsGrid &g, bool ft, int grid,
                    hipStream_t s);
void launch_pack_rows(const int *rp, const int *ci, const double *v, const int *rp4,
                      unsigned short *c4, double *v4, int rows, hipStream_t s);

// LSMR (lsmr.hip): its scalars beyond the LSQR state block, and the arguments of its
// per-iteration launch (after the U and V product launches of the LSQR loop kernels)
struct LsmrState {
    double alphabar;                         // first QR: unfinished diagonal
    double rho_prev, rhobar_prev, cbar, sbar, zetabar;   // second QR
    double betadd, betadot, rhodot, thetatil, tautil_prev, zeta_prev, fixed_sq;  // estimate
};
struct LsmrArgs {
    const LsqrState *st;   // state the V launch wrote (its partials pending)
    LsqrState *st_next;    // state the next U launch reads
    const double *part;    // the V launch's partial sums (kMaxLoopGrid slots of two doubles)
    LsmrState *ls;         // two buffers, read [iters % 2], write the other
    const double *v;       // v~_{k+1} (unnormalised)
    double *x, *h, *hb;    // iterate and directions (N each)
    int N;
};
void launch_lsmr_step(const LsmrArgs &a, hipStream_t s);
void launch_lsmr_init(const LsmrArgs &a, hipStream_t s);

// learned preconditioner (learned.hip)
struct FeatMeta {
    int n_zero, n_diag, soc_end, psd_end;  // y-row boundaries of the cone kinds
};
hipError_t launch_features(const Problem &p, const FeatMeta &fm, const double *jcol,
                           const double *jrow, float *feat, hipStream_t s);
hipError_t launch_targets(int N, const double *jcol, const double *jrow, const double *ecol,
                          const double *erow, float *target, hipStream_t s);
hipError_t launch_mlp_scales(const float *feat, int N, const float *w, const double *jcol,
                             const double *jrow, double *col, double *row, hipStream_t s);

}  // namespace qcpd
