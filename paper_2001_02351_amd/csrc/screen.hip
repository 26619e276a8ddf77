// Steps a7-a9 (Eqs. epsGG, Wq):
//   eps_GG'(w)   = delta_GG' - v^1/2_G chi_GG'(w) v^1/2_G',  v^1/2_G = sqrt(4 pi/Omega)/|q+G|
//   eps^-1(w)    by in-place Gauss-Jordan elimination with partial (row)
//                pivoting, blocked, all frequencies of a q-point batched,
//                FP64 throughout
//   W_GG'(w)     = HA * v^1/2_G eps^-1_GG'(w) v^1/2_G'   (eV)
//
// Elimination step c (per matrix): pick the row r >= c of largest |a_rc|,
// swap rows r and c, scale row c by 1/a_cc (leaving 1/a_cc in place), and
// subtract a_ic * row c from every other row i (leaving -a_ic/a_cc in column
// c).  After the last step the recorded row swaps are undone as column swaps
// in reverse order, which leaves A^-1 in place.
//
// Blocked form: the steps of a panel of columns K = [c0, c0 + nb) are run on
// the panel's columns only (after the full-row swaps), and the other columns
// R are brought up to date afterwards in one pass.  The steps on K act on the
// matrix as the sweep on block K: with P the panel columns after the panel
// steps (rows K: A_KK^-1, other rows: -A_OK A_KK^-1) and A_KR the pivot rows
// of R before the panel, the updated R columns are
//     A[:, R] = P A_KR + (rows outside K: A[:, R] as they were),
// a complex matrix product with an inner dimension of nb, run on the FP64
// matrix cores.  The arithmetic is that of the unblocked steps regrouped, and
// the pivots are the same.
//
// eps is dimensionless with a unit-scale diagonal, so a pivot below
// kPivotFloor (a condition number beyond ~1e13, where an FP64 inverse has no
// correct digits left) is reported as singular; a non-finite pivot as a
// non-finite input.
#include "fft_lds.h"

namespace rp {

namespace {

constexpr double kPivotFloor = 1e-13;

// vs[i] = sqrt(4 pi / Omega) / |q + G_i|; with head set, the q -> 0 form:
// |q + G| = 0 (G = 0) takes sqrt(4 pi / Omega), the q factor being in chi
__global__ void k_vsqrt(int ng, const int *g, double r0, double r1, double r2, double r3, double r4,
                        double r5, double r6, double r7, double r8, double q1, double q2, double q3,
                        double pref, int head, double *vs, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    const double f1 = q1 + g[3 * i], f2 = q2 + g[3 * i + 1], f3 = q3 + g[3 * i + 2];
    const double x = f1 * r0 + f2 * r3 + f3 * r6;
    const double y = f1 * r1 + f2 * r4 + f3 * r7;
    const double z = f1 * r2 + f2 * r5 + f3 * r8;
    const double qg = sqrt(x * x + y * y + z * z);
    if (head && qg == 0.0) {
        vs[i] = pref;
        return;
    }
    vs[i] = pref / qg;
    if (!(qg > 0.0)) atomicOr(flag, kFlagNonFinite);
}

__global__ void k_eps(int nfreq, int ng, const double *vs, const double2 *chi, double2 *eps, int *flag)
{
    const long n2 = (long)ng * ng;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2 * nfreq) return;
    const long e = t % n2;
    const int g = (int)(e / ng), h = (int)(e - (long)g * ng);
    const double s = vs[g] * vs[h];
    const double2 c = chi[t];
    if (!isfinite(c.x) || !isfinite(c.y)) atomicOr(flag, kFlagNonFinite);
    eps[t] = make_double2((g == h ? 1.0 : 0.0) - s * c.x, -s * c.y);
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGjNb = 64;            // panel width
constexpr int kGjPivotThreads = 1024;
constexpr int kGjElimRows = 16;      // rows per elimination workgroup (4 per thread)

// (|v|, row) of the larger pivot candidate; ties go to the lower row
__device__ __forceinline__ void pivot_max(double &m, int &r, double om, int orow)
{
    if (om > m || (om == m && orow < r)) { m = om; r = orow; }
}

// Step c of panel [c0, c0 + nb), first half, one block per matrix: pivot
// search over rows >= c of column c, swap of the full rows r and c, and the
// scaled pivot row's panel entries into prow[f][0 .. nb) (1/a_cc in column
// c itself).
__global__ void __launch_bounds__(kGjPivotThreads)
k_gj_pivot(int ng, int c0, int nb, int c, double2 *a, double2 *prow, int *piv, int *flag)
{
    constexpr int NWV = kGjPivotThreads / 64;
    __shared__ double bv[NWV];
    __shared__ int bi[NWV];
    const int f = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double2 *A = a + (long)f * ng * ng;
    double best = -1.0;
    int bidx = c;
    for (int i = c + tid; i < ng; i += kGjPivotThreads) {
        const double2 v = A[(long)i * ng + c];
        const double m = isfinite(v.x) && isfinite(v.y) ? hypot(v.x, v.y) : INFINITY;
        pivot_max(best, bidx, m, i);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pivot_max(best, bidx, __shfl_xor(best, o), __shfl_xor(bidx, o));
    if (lane == 0) {
        bv[wave] = best;
        bi[wave] = bidx;
    }
    __syncthreads();
    best = bv[0];
    bidx = bi[0];
#pragma unroll
    for (int w = 1; w < NWV; w++) pivot_max(best, bidx, bv[w], bi[w]);
    const int r = bidx;
    if (tid == 0) {
        piv[(long)f * ng + c] = r;
        if (!isfinite(best)) atomicOr(flag, kFlagNonFinite);
        else if (!(best > kPivotFloor)) atomicOr(flag, kFlagZeroPivot);
    }
    if (r != c) {
        for (int j = tid; j < ng; j += kGjPivotThreads) {
            const double2 t = A[(long)c * ng + j];
            A[(long)c * ng + j] = A[(long)r * ng + j];
            A[(long)r * ng + j] = t;
        }
    }
    __syncthreads();
    const double2 p = A[(long)c * ng + c];
    const double den = p.x * p.x + p.y * p.y;
    const double2 ip = make_double2(p.x / den, -p.y / den);
    if (tid < nb) {
        const int j = c0 + tid;
        prow[(long)f * kGjNb + tid] = (j == c) ? ip : cmul(A[(long)c * ng + j], ip);
    }
}

// Step c, second half: the panel columns of every row, grid (row blocks of
// kGjElimRows, matrices).  Row c takes the scaled pivot row; column c of the
// other rows takes -a_ic/a_cc; the other entries a_ij - a_ic prow_j.  Each
// thread reads the a_ic of its rows before any thread of the block (which
// owns those rows whole) writes column c.
__global__ void __launch_bounds__(256)
k_gj_elim(int ng, int c0, int nb, int c, double2 *a, const double2 *prow)
{
    const int f = blockIdx.y, tid = threadIdx.x, jj = tid & 63, rr = tid >> 6;
    double2 *A = a + (long)f * ng * ng;
    const double2 *pr = prow + (long)f * kGjNb;
    const int i0 = blockIdx.x * kGjElimRows + rr;
    double2 fi[kGjElimRows / 4];
#pragma unroll
    for (int q = 0; q < kGjElimRows / 4; q++) {
        const int i = i0 + 4 * q;
        fi[q] = i < ng ? A[(long)i * ng + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (jj >= nb) return;
    const int j = c0 + jj;
    const double2 pj = pr[jj], ip = pr[c - c0];
#pragma unroll
    for (int q = 0; q < kGjElimRows / 4; q++) {
        const int i = i0 + 4 * q;
        if (i >= ng) continue;
        double2 *x = A + (long)i * ng + j;
        double2 v;
        if (i == c) v = pj;
        else v = (j == c) ? cmul(make_double2(-fi[q].x, -fi[q].y), ip) : csub(*x, cmul(fi[q], pj));
        *x = v;
    }
}

// After the panel: its pivot rows (all columns) into rk [f][nb][ng] for the
// update of the other columns.
__global__ void k_gj_saverows(int ng, int c0, int nb, const double2 *a, double2 *rk)
{
    const int f = blockIdx.y;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nb * ng) return;
    const int kk = (int)(t / ng), j = (int)(t - (long)kk * ng);
    rk[((long)f * kGjNb + kk) * ng + j] = a[(long)f * ng * ng + (long)(c0 + kk) * ng + j];
}

__device__ __forceinline__ d4 mfma64(double x, double y, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// Update of the columns outside panel [c0, c0 + nb) (see the header):
//   A[i][j] = sum_k A[i][c0 + k] rk[k][j] + (i outside the panel rows ? A[i][j] : 0)
// A 256-thread block owns a 64x64 tile of one matrix; each wave a 32x32
// sub-tile (2x2 blocks of 16x16) on v_mfma_f64_16x16x4f64 (A operand lane
// i + 16k, B operand lane j + 16k, result register r of lane l at row
// l / 16 + 4 r, column l % 16).  The panel columns of the tile's rows and the
// pivot rows of its columns are staged in LDS.
__global__ void __launch_bounds__(256, 3)
k_gj_update(int ng, int c0, int nb, double2 *a, const double2 *rk)
{
    // the panel's 64 columns pass through LDS in chunks of 16, so that a CU
    // holds several workgroups and one's loads overlap another's matrix work;
    // the registers are held to three waves per SIMD (three workgroups per
    // CU; four would spill)
    constexpr int KC = 16;
    __shared__ double2 sP[64][KC + 1];
    __shared__ double2 sR[KC][64];
    const int f = blockIdx.z, tid = threadIdx.x;
    const int rt0 = blockIdx.y * 64, ct0 = blockIdx.x * 64;
    if (ct0 >= c0 && ct0 + 64 <= c0 + nb) return;   // tile inside the panel columns
    double2 *A = a + (long)f * ng * ng;
    const double2 *R = rk + (long)f * kGjNb * ng;
    const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    d4 accR[2][2], accI[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++) {
            accR[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
            accI[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
        }
    // each thread moves 4 panel and 4 pivot-row elements of a chunk; the next
    // chunk's are loaded into registers before the current chunk's matrix
    // work, so their latency is covered by it
    constexpr int PER = 64 * KC / 256;
    double2 pp[PER], pr[PER];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = tid + q * 256;
            const int rr = e / KC, k = e - rr * KC, i = rt0 + rr;
            pp[q] = (i < ng && kc + k < nb) ? A[(long)i * ng + c0 + kc + k] : make_double2(0.0, 0.0);
            const int k2 = e >> 6, cc = e & 63, j = ct0 + cc;
            pr[q] = (kc + k2 < nb && j < ng) ? R[(long)(kc + k2) * ng + j] : make_double2(0.0, 0.0);
        }
    };
    fetch(0);
    for (int kc = 0; kc < nb; kc += KC) {
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = tid + q * 256;
            sP[e / KC][e % KC] = pp[q];
            sR[e >> 6][e & 63] = pr[q];
        }
        __syncthreads();
        if (kc + KC < nb) fetch(kc + KC);
#pragma unroll
        for (int k0 = 0; k0 < KC; k0 += 4) {
            double2 x[2], y[2];
#pragma unroll
            for (int rb = 0; rb < 2; rb++) x[rb] = sP[wr + rb * 16 + li][k0 + lk];
#pragma unroll
            for (int cb = 0; cb < 2; cb++) y[cb] = sR[k0 + lk][wc + cb * 16 + li];
#pragma unroll
            for (int rb = 0; rb < 2; rb++)
#pragma unroll
                for (int cb = 0; cb < 2; cb++) {
                    accR[rb][cb] = mfma64(x[rb].x, y[cb].x, accR[rb][cb]);
                    accR[rb][cb] = mfma64(-x[rb].y, y[cb].y, accR[rb][cb]);
                    accI[rb][cb] = mfma64(x[rb].x, y[cb].y, accI[rb][cb]);
                    accI[rb][cb] = mfma64(x[rb].y, y[cb].x, accI[rb][cb]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = rt0 + wr + rb * 16 + lk + 4 * r, j = ct0 + wc + cb * 16 + li;
                if (i >= ng || j >= ng || (j >= c0 && j < c0 + nb)) continue;
                double2 v = make_double2(accR[rb][cb][r], accI[rb][cb][r]);
                if (i < c0 || i >= c0 + nb) v = cadd(v, A[(long)i * ng + j]);
                A[(long)i * ng + j] = v;
            }
}

// undo the row swaps as column swaps in reverse order; one thread per row
__global__ void k_gj_unswap(int nfreq, int ng, double2 *a, const int *piv)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nfreq * ng) return;
    const int f = (int)(t / ng);
    double2 *row = a + t * ng;
    const int *pv = piv + (long)f * ng;
    for (int c = ng - 1; c >= 0; c--) {
        const int r = pv[c];
        if (r != c) {
            const double2 x = row[c];
            row[c] = row[r];
            row[r] = x;
        }
    }
}

__global__ void k_W(int nfreq, int ng, const double *vs, const double2 *einv, double2 *W)
{
    const long n2 = (long)ng * ng;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2 * nfreq) return;
    const long e = t % n2;
    const int g = (int)(e / ng), h = (int)(e - (long)g * ng);
    W[t] = cscale(einv[t], kHartreeEv * vs[g] * vs[h]);
}

}  // namespace

void launch_vsqrt(hipStream_t s, const Geometry &g, int ng, const int *gsph, double *vs, int *flag, bool head)
{
    const double pref = sqrt(4.0 * kPi / g.volume);
    hipLaunchKernelGGL(k_vsqrt, dim3((ng + 255) / 256), dim3(256), 0, s, ng, gsph, g.rec[0], g.rec[1],
                       g.rec[2], g.rec[3], g.rec[4], g.rec[5], g.rec[6], g.rec[7], g.rec[8],
                       (double)g.iq[0] / g.kmesh[0], (double)g.iq[1] / g.kmesh[1],
                       (double)g.iq[2] / g.kmesh[2], pref, (int)head, vs, flag);
}

void launch_eps(hipStream_t s, int nfreq, int ng, const double *vs, const double2 *chi, double2 *eps,
                int *flag)
{
    const long tot = (long)nfreq * ng * ng;
    hipLaunchKernelGGL(k_eps, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nfreq, ng, vs, chi,
                       eps, flag);
}

// the pivot rows of a panel [nfreq][kGjNb][ng], then the scaled pivot rows [nfreq][kGjNb]
size_t invert_scratch_bytes(int ng, int nfreq) { return sizeof(double2) * (size_t)kGjNb * (ng + 1) * nfreq; }

void launch_invert(hipStream_t s, int nfreq, int ng, double2 *a, double2 *scratch, int *piv, int *flag)
{
    const unsigned t = (unsigned)((ng + 63) / 64);
    double2 *prow = scratch + (size_t)kGjNb * ng * nfreq;
    const dim3 eg((unsigned)((ng + kGjElimRows - 1) / kGjElimRows), (unsigned)nfreq);
    for (int c0 = 0; c0 < ng; c0 += kGjNb) {
        const int nb = std::min(kGjNb, ng - c0);
        for (int c = c0; c < c0 + nb; c++) {
            hipLaunchKernelGGL(k_gj_pivot, dim3(nfreq), dim3(kGjPivotThreads), 0, s, ng, c0, nb, c, a, prow, piv,
                               flag);
            hipLaunchKernelGGL(k_gj_elim, eg, dim3(256), 0, s, ng, c0, nb, c, a, prow);
        }
        const long nrow = (long)nb * ng;
        hipLaunchKernelGGL(k_gj_saverows, dim3((unsigned)((nrow + 255) / 256), (unsigned)nfreq), dim3(256), 0, s,
                           ng, c0, nb, a, scratch);
        hipLaunchKernelGGL(k_gj_update, dim3(t, t, nfreq), dim3(256), 0, s, ng, c0, nb, a, scratch);
    }
    const long rows = (long)nfreq * ng;
    hipLaunchKernelGGL(k_gj_unswap, dim3((unsigned)((rows + 127) / 128)), dim3(128), 0, s, nfreq, ng, a,
                       piv);
}

void launch_W(hipStream_t s, int nfreq, int ng, const double *vs, const double2 *einv, double2 *W)
{
    const long tot = (long)nfreq * ng * ng;
    hipLaunchKernelGGL(k_W, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nfreq, ng, vs, einv, W);
}

}  // namespace rp
