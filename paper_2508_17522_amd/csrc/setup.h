// Host-side declarations of the create-time kernels.
#pragma once

#include "qcpd_internal.h"

namespace qcpd {

struct ConeHost {
    int n_zero;
    int n_exp;                // exponential cones (the first 3 x 3 blocks)
    int n_pow;                // power and dual power cones after them
    const double *pow_par;    // [device] alpha (power cone) or -alpha (dual power cone)
    int *psd_lr = nullptr;    // [device] per PSD cone: low-rank side (k_psd_factors), or null
};

hipError_t csr_transpose(int nrows, int ncols, int nnz, const int *rp, const int *ci,
                         const double *val, int *trp, int *tci, double *tv, int *perm,
                         hipStream_t s);
void launch_check_csr(const int *rp, const int *ci, int nrows, int ncols, int nnz, int *flag,
                      hipStream_t s);
void launch_check_sorted(const int *rp, const int *ci, int nrows, int ncols, int *flag, hipStream_t s);
void launch_check_symmetric(const int *rp, const int *ci, const double *v, const int *trp,
                            const int *tci, const double *tv, int n, int nnz, int *flag,
                            hipStream_t s);
void launch_px(const Problem &p, const RowGrid &g, double *c, double *xpx, double *partials,
               int *counter, hipStream_t s);
void launch_sub(const double *a, const double *b, double *out, int n, hipStream_t s);
// solution refinement: G(x, eta) of the QCP's KKT conditions at y = Pi_{K*}(eta) (n + m
// entries), the Newton update x += dx, eta += dy - ds, and the sum of squares of n entries into
// out[0] (part: kSumsqParts doubles of scratch)
constexpr int kSumsqParts = 256;
void launch_kkt_map(const Problem &p, const double *x, const double *y, const double *eta,
                    double *g, hipStream_t s);
void launch_newton_update(double *x, double *eta, const double *dx, const double *dy,
                          const double *ds, int n, int m, hipStream_t s);
void launch_sumsq(const double *v, long long n, double *part, double *out, hipStream_t s);

// proj (optional): Pi_{K*}(z_y) of every cone row (zero and nonnegative rows included)
void launch_cone_factors(const Problem &p, const ConeHost &ch, double *jdiag, double *soc_par,
                         double *exp_J, double *pool, int *nondiff, int *fail, int psd_lds,
                         hipStream_t s, double *proj = nullptr);
void launch_scales(const Problem &p, const RowGrid &g, double *dj, double *dv, double *partials,
                   int *counter, hipStream_t s, int do_tau = 1);
int psd_factor_lds_bytes(int kmax);
void launch_equilibrate(const Problem &p, const RowGrid &g, double *DL, double *DR, double *tmpL,
                        double *tmpR, int sweeps, double *partials, int *counter, hipStream_t s);
void set_cone_kernel_lds(int bytes);

}  // namespace qcpd
