// Internal declarations shared by the host side of the library and the
// kernel translation units.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "rp.h"

namespace rp {

constexpr double kPi = 3.14159265358979323846;
constexpr double kHartreeEv = 27.211386245988;  // CODATA 2018

// A device buffer that grows on demand and is freed with the context.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Bits of the device-side fault flag.
enum : int { kFlagZeroPivot = 1, kFlagNonFinite = 2 };

// Radix plan of one FFT length: n = prod(rad[0..nrad-1]), radices in {2,3,4,5}.
struct FftPlan {
    int n;
    int nrad;
    int rad[12];
};

bool make_plan(int n, FftPlan *plan);

// Geometry of one call, computed on the host.
struct Geometry {
    double lat[9];
    double rec[9];     // rows b_i, a_i.b_j = 2 pi delta_ij
    double volume;
    int fft[3];
    int kmesh[3];
    int iq[3];
    int nk;
};

}  // namespace rp

struct rp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int *flag = nullptr;            // device int[4] fault flags
    void *scratch = nullptr;        // this device's fixed workspace (rp_chi0_accumulate_noalloc)
    rp::DevBuf ugrid;               // u-grids of one k: [nO + nE][N1][N2][N3] c128
    rp::DevBuf ugrid32;             // the same grids in FP32 (split-precision path)
    rp::DevBuf weights;             // w[nfreq][npair] c128
    rp::DevBuf glist;               // int[...] copies of host G lists
    rp::DevBuf freq;                // c128[nfreq]
    rp::DevBuf kinfo;               // per-k tables
    rp::DevBuf vsqrt;               // double[ng]
    rp::DevBuf work;                // eps / inversion workspace
    rp::DevBuf split_a;             // split-BF16 row operand (FP32 complex)
    rp::DevBuf split_b;             // split-BF16 column operand (BF16 planes)
    rp::DevBuf split_w;             // split-BF16 weights (FP32)
    rp::DevBuf chi_part;            // split-BF16 partial tiles of sliced pair steps
    rp::DevBuf rho;                 // Wannier densities
    rp::DevBuf piv;                 // pivots
    rp::DevBuf mbuf;                // pair densities of one k batch (batch entry point)
    rp::DevBuf bstage;              // device copies of a batch's G and frequency lists
    // the last batch's graphs (launched in order) and the launch arguments
    // they were captured with; batch_nodes counts their kernel nodes
    std::vector<hipGraphExec_t> batch_execs;
    long batch_nodes = 0;
    std::string batch_key;
    bool capturing = false;         // stage timers stay off while a graph is captured
    std::vector<rp_tune_entry> tuning;  // launch shapes per size class, matched in order
    double fermi_eV = std::nan("");  // Fermi level of the metallic weights (RP_W_TETRA_METAL)
    double drude_wq = 0.0;           // intraband head term qhat.Omega.qhat (eV^2) of rp_screen_head
    double drude_delta = 0.0;        // its broadening (eV)
    // stage timers
    bool profiling = false;
    struct Mark {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> spare;
};

namespace rp {

rp_status fail(rp_ctx *ctx, rp_status st, const char *fmt, ...);
rp_status ensure(rp_ctx *ctx, DevBuf &b, size_t bytes);
rp_status check_launch(rp_ctx *ctx, const char *what);
rp_status geometry(rp_ctx *ctx, const rp_cell *cell, const int iq[3], Geometry *g);

// Launch shapes of one call: the first tuning entry whose class holds N_G and
// the largest FFT edge, else the defaults (2 frequencies per contraction
// workgroup, slicing towards 1024 workgroups, FFT lines per block by length).
struct Tune {
    int chi_nw = 2;
    int chi_fill = 1024;
    int fft_lines = 0;
    int chi_kernel = 0;
};
Tune tune_for(const rp_ctx *ctx, int ng, const int fft[3]);

// Brackets the launches of one stage with events when profiling is on.
class StageTimer {
  public:
    StageTimer(rp_ctx *ctx, int stage);
    ~StageTimer();

  private:
    rp_ctx *ctx_;
    int stage_;
    hipEvent_t a_ = nullptr;
};

// ---- kernel launchers (one translation unit each) --------------------------

// fft.hip: u-grids (scatter + pruned 3-D transform) of two band sets stored
// one after the other in u (nA grids from millerA/coefA, then nB from
// millerB/coefB), FP32 or FP64; u holds ugrid_bytes (the grids, then a small
// sort workspace; band_stride is the npw_max of the coefficient rows).
size_t ugrid_bytes(const int fft[3], int nbands, int npw_max, bool fp32);
void launch_ugrid2(hipStream_t s, const FftPlan plans[3], const int fft[3], const int mmax[3], int nA, int npwA,
                   const int *millerA, const double2 *coefA, int nB, int npwB, const int *millerB,
                   const double2 *coefB, int band_stride, void *u, bool fp32, int lines);

// fft.hip: in-place batched positive-exponent transform of whole grids.
void launch_fft3d(hipStream_t s, const FftPlan plans[3], const int fft[3], int ngrids,
                  double2 *data);

// Split-BF16 operands of one contraction call (layout in split_ops.h): the
// FP32 row blocks A, the BF16 planes B, the padded sizes, and p0, the index
// within the call's pairs of the first pair a pair-kernel launch writes.
struct SplitOps {
    void *A = nullptr;
    void *B = nullptr;
    long p0 = 0;
    int NGP = 0, npg = 0, nterm = 0;
};

// pair.hip: pair densities of one k (grids in FP64, or FP32 when fp32).
size_t pair_lds_bytes(const int fft[3], int L3, int rows, size_t csize, int npairs);
int pair_rows(const int fft[3]);
// whether a pair kernel can run this grid, sphere size and m3 window
bool pair_supported(const int fft[3], int ng, int L3, bool fp32);
// the smallest line length n of the lane kernels with need <= n <= limit that
// takes this sphere and m3 window as N2 = N3 = n, or 0
int pair_lane_edge(int need, int limit, int ng, int L3, bool fp32);
void launch_pair_k(hipStream_t s, const FftPlan plans[3], const int fft[3], const void *u_occ,
                   const void *u_emp, int nO, int nE, int ng, const int *gsph, const int g0[3],
                   int lo3, int L3, bool fp32, double2 *M);
// the same pair densities written as split operands (FP32 grids only): pair
// (a, b) of this k goes to pair p0 + a nO + b of ops
void launch_pair_ops(hipStream_t s, const FftPlan plans[3], const int fft[3], const void *u_occ,
                     const void *u_emp, int nO, int nE, int ng, const int *gsph, const int g0[3], int lo3, int L3,
                     const SplitOps &ops);

// tetra.hip: weights of a pair range.
void launch_weights(hipStream_t s, const int kmesh[3], const int iq[3], int nband,
                    const double *E_eV, const double *T, int o0, int o1, int e0, int e1,
                    int k0, int k1, int nfreq, const double2 *freq_eV, double delta_eV,
                    int mode, double ef_eV, double2 *w);

// chi_f64.hip: chi += sum_p w_p M_p M_p^H on FP64 matrix cores.  herm: the
// weights are real and only the upper tiles are formed (chi Hermitian).
void launch_chi_f64(hipStream_t s, long npair, int ng, const double2 *M, int nfreq,
                    const double2 *w, int accumulate, bool herm, double2 *chi);

// chi_bf16.hip: split-BF16 contraction (herm as above; part holds the
// partial tiles when the pair steps are sliced, chi_part_bytes of them).
size_t split_a_bytes(long npair, int ng);
size_t split_b_bytes(long npair, int ng);
size_t split_w_bytes(long npair, int nfreq);
size_t chi_part_bytes(long npair, int ng, int nfreq, bool herm, int nw, int fill, int kernel, int nterm);
// the operand layout of npair pairs at ng rows in split_a / split_b (p0 = 0)
SplitOps split_ops(void *split_a, void *split_b, long npair, int ng, int nterm);
// the operands of M (FP64, npair x ng) into split_a / split_b
void launch_split_prep(hipStream_t s, int nterm, long npair, int ng, const double2 *M, void *split_a,
                       void *split_b);
// zeros into the padding slots of the operands of npair pairs (rows ng..NGP-1
// of every pair, pairs npair..KP-1 of every row), for operands whose pairs
// the pair kernels write
void launch_ops_pad(hipStream_t s, const SplitOps &ops, long npair, int ng);
// the FP32 weights [nfreq][KP] of the contraction
void launch_weight_prep(hipStream_t s, long npair, int nfreq, const double2 *w, bool herm, void *split_w);
// before_reduce (may be empty) is called on the host between the contraction
// launch and the launch that sums its partial tiles, when there is one
void launch_chi_bf16(hipStream_t s, int nterm, long npair, int ng, int nfreq, int accumulate,
                     double2 *chi, const void *split_a, const void *split_b, const void *split_w,
                     bool herm, int nw, int fill, int kernel, void *part,
                     const std::function<void()> &before_reduce);

// screen.hip
void launch_vsqrt(hipStream_t s, const Geometry &g, int ng, const int *gsph, double *vs, int *flag,
                  bool head = false);
void launch_eps(hipStream_t s, int nfreq, int ng, const double *vs, const double2 *chi,
                double2 *eps, int *flag);
size_t invert_scratch_bytes(int ng, int nfreq);
void launch_invert(hipStream_t s, int nfreq, int ng, double2 *a, double2 *scratch, int *piv, int *flag);
void launch_W(hipStream_t s, int nfreq, int ng, const double *vs, const double2 *einv,
              double2 *W);

// head.hip: q -> 0 head densities into column col of M (row stride ldm),
// and the optical quantities {Re eps_M, Im eps_M, L, Re sigma, R} per
// frequency from eps^-1_00.
void launch_head(hipStream_t s, const Geometry &g, const int *miller, const double2 *coef, const double *E,
                 const int *npw_dev, int nband, int npw_max, int o0, int o1, int e0, int e1, int k0, int k1,
                 const double qhat[3], int ldm, int col, double2 *M, int *flag);
void launch_optics(hipStream_t s, int nfreq, int ng, const double2 *einv, const double2 *freq, double *out);
// head.hip: diagonal moments p[k][b1 - b0][3] (Cartesian) of bands [b0, b1)
void launch_pdiag(hipStream_t s, const Geometry &g, const int *miller, const double2 *coef, const int *npw_dev,
                  int nband, int npw_max, int b0, int b1, double *p);
// head.hip: the intraband term of eps_00 (before the inversion) and the zero
// head of eps^-1 where it is infinite (after it)
void launch_drude_head(hipStream_t s, int nfreq, int ng, const double2 *freq, double wq, double delta, double2 *eps);
void launch_drude_zero(hipStream_t s, int nfreq, int ng, const double2 *freq, double delta, double2 *einv);
// tetra.hip: Fermi-surface weights times (1 - T^2) p p^T per (k, band), summed
// into out[6] = {xx, yy, zz, xy, xz, yz} (contrib: [Nk][b1 - b0][6] workspace)
void launch_fermi_plasma(hipStream_t s, const int kmesh[3], int nband, const double *E_eV, const double *T, int b0,
                         int b1, double ef_eV, const double *p, double *contrib, double *out);

// wannier.hip
void launch_wannier_density(hipStream_t s, const Geometry &g, const FftPlan plans[3], int nwan,
                            const double *phi, const double *centre_frac_dev, double2 *f);
// zero_ok: where q + G = 0 store ntilde(0) instead of flagging the division
void launch_wannier_gather(hipStream_t s, const Geometry &g, int nwan, int nlist,
                           const int *glist, const double2 *fgrid, double2 *rho, int *flag,
                           bool zero_ok = false);
void launch_wannier_W(hipStream_t s, int nfreq, int nwan, int ng, const double2 *rho_eps,
                      int ntail, const double2 *rho_tail, const double2 *einv, double pre,
                      double2 *T, double2 *Wij);

// symmetry.hip: unfolding of coefficients and of G-indexed matrices
void launch_unfold_coef(hipStream_t s, int nband, int npw, const int *idx, const int *miller, const int delta[3],
                        const double t[3], const double2 *src, long ld_src, double2 *dst, long ld_dst);
void launch_unfold_matrix(hipStream_t s, int nfreq, int ng, int ng_src, const int *idx, const int *gsph,
                          const double t[3], double2 *ph, const double2 *src, double2 *dst);

// qsum.hip: one q-point's term of the q-sums of U, V, J, X
void launch_xdens(hipStream_t s, const Geometry &g, const FftPlan plans[3], int nwan, const double *phi,
                  const double *centre_dev, const int *R_dev, long v0, int nvc, double2 *grids);
int wgemm_row_tiles(int ng);
void launch_wgemm(hipStream_t s, bool diag, int nfreq, int ng, int klo, int nv, const double2 *P, long ldp,
                  const double2 *E, double2 *out);
void launch_wcross(hipStream_t s, int nfreq, int nwan, int ng, int klo, const double2 *P, long ldp,
                   const double2 *T, double2 *body);
void launch_wgram(hipStream_t s, int nout, int nb, bool diag, int ng, int klo, int ntail, const double2 *P,
                  long ldp, double2 *bare, double2 *tail);
void launch_wsum_u(hipStream_t s, const Geometry &g, int nfreq, int nR, int nwan, int ng, const int *R_dev,
                   double pre, bool head, double avg, const double2 *E, const double2 *P, long ldp,
                   const double2 *body, const double2 *bare, const double2 *tail, int accumulate, double2 *U,
                   double2 *V);
void launch_wsum_x(hipStream_t s, int nfreq, long nvt, long v0, int nvc, int ng, double pre, bool head, double avg,
                   const double2 *E, const double2 *P, long ldp, const double2 *part, const double2 *bare,
                   const double2 *tail, int accumulate, double2 *J, double2 *X);

}  // namespace rp
