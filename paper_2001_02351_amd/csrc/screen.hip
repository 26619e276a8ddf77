// Steps a7-a9 (Eqs. epsGG, Wq):
//   eps_GG'(w)   = delta_GG' - v^1/2_G chi_GG'(w) v^1/2_G',  v^1/2_G = sqrt(4 pi/Omega)/|q+G|
//   eps^-1(w)    by in-place Gauss-Jordan elimination with partial (row)
//                pivoting, all frequencies of a q-point in one batched launch
//                per elimination step, FP64 throughout
//   W_GG'(w)     = HA * v^1/2_G eps^-1_GG'(w) v^1/2_G'   (eV)
//
// Elimination step c (per matrix): pick the row r >= c of largest |a_rc|,
// swap rows r and c, scale row c by 1/a_cc (leaving 1/a_cc in place), and
// subtract a_ic * row c from every other row i (leaving -a_ic/a_cc in column
// c).  After the last step the recorded row swaps are undone as column swaps
// in reverse order, which leaves A^-1 in place.
//
// eps is dimensionless with a unit-scale diagonal, so a pivot below
// kPivotFloor (a condition number beyond ~1e13, where an FP64 inverse has no
// correct digits left) is reported as singular; a non-finite pivot as a
// non-finite input.
#include "fft_lds.h"

namespace rp {

namespace {

constexpr double kPivotFloor = 1e-13;

__global__ void k_vsqrt(int ng, const int *g, double r0, double r1, double r2, double r3, double r4,
                        double r5, double r6, double r7, double r8, double q1, double q2, double q3,
                        double pref, double *vs, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    const double f1 = q1 + g[3 * i], f2 = q2 + g[3 * i + 1], f3 = q3 + g[3 * i + 2];
    const double x = f1 * r0 + f2 * r3 + f3 * r6;
    const double y = f1 * r1 + f2 * r4 + f3 * r7;
    const double z = f1 * r2 + f2 * r5 + f3 * r8;
    const double qg = sqrt(x * x + y * y + z * z);
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

// pivot search, row swap and pivot-row scaling for step c; one block per matrix
__global__ void __launch_bounds__(256) k_gj_pivot(int ng, int c, double2 *a, double2 *col, int *piv,
                                                  int *flag)
{
    __shared__ double bv[256];
    __shared__ int bi[256];
    const int f = blockIdx.x, tid = threadIdx.x;
    double2 *A = a + (long)f * ng * ng;
    double best = -1.0;
    int bidx = c;
    for (int i = c + tid; i < ng; i += 256) {
        const double2 v = A[(long)i * ng + c];
        const double m = isfinite(v.x) && isfinite(v.y) ? hypot(v.x, v.y) : INFINITY;
        if (m > best || (m == best && i < bidx)) { best = m; bidx = i; }
    }
    bv[tid] = best;
    bi[tid] = bidx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            const double o = bv[tid + s];
            const int oi = bi[tid + s];
            if (o > bv[tid] || (o == bv[tid] && oi < bi[tid])) { bv[tid] = o; bi[tid] = oi; }
        }
        __syncthreads();
    }
    const int r = bi[0];
    const double pm = bv[0];
    if (tid == 0) {
        piv[(long)f * ng + c] = r;
        if (!isfinite(pm)) atomicOr(flag, kFlagNonFinite);
        else if (!(pm > kPivotFloor)) atomicOr(flag, kFlagZeroPivot);
    }
    if (r != c) {
        for (int j = tid; j < ng; j += 256) {
            const double2 t = A[(long)c * ng + j];
            A[(long)c * ng + j] = A[(long)r * ng + j];
            A[(long)r * ng + j] = t;
        }
    }
    __syncthreads();
    const double2 p = A[(long)c * ng + c];
    const double den = p.x * p.x + p.y * p.y;
    const double2 ip = make_double2(p.x / den, -p.y / den);
    // save column c (after the swap) for the elimination kernel
    for (int i = tid; i < ng; i += 256) col[(long)f * ng + i] = A[(long)i * ng + c];
    __syncthreads();
    for (int j = tid; j < ng; j += 256) {
        const double2 v = (j == c) ? make_double2(1.0, 0.0) : A[(long)c * ng + j];
        A[(long)c * ng + j] = cmul(v, ip);
    }
}

// rows i != c: a_ij -= a_ic a_cj (j != c), a_ic = -a_ic a_cc
__global__ void k_gj_elim(int ng, int c, double2 *a, const double2 *col)
{
    const int f = blockIdx.z;
    const int i = blockIdx.y;
    if (i == c) return;
    double2 *A = a + (long)f * ng * ng;
    const double2 fi = col[(long)f * ng + i];
    if (fi.x == 0.0 && fi.y == 0.0) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ng; j += gridDim.x * blockDim.x) {
        const double2 pc = A[(long)c * ng + j];
        const double2 prod = cmul(fi, pc);
        if (j == c) A[(long)i * ng + j] = make_double2(-prod.x, -prod.y);
        else A[(long)i * ng + j] = csub(A[(long)i * ng + j], prod);
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

void launch_vsqrt(hipStream_t s, const Geometry &g, int ng, const int *gsph, double *vs, int *flag)
{
    const double pref = sqrt(4.0 * kPi / g.volume);
    hipLaunchKernelGGL(k_vsqrt, dim3((ng + 255) / 256), dim3(256), 0, s, ng, gsph, g.rec[0], g.rec[1],
                       g.rec[2], g.rec[3], g.rec[4], g.rec[5], g.rec[6], g.rec[7], g.rec[8],
                       (double)g.iq[0] / g.kmesh[0], (double)g.iq[1] / g.kmesh[1],
                       (double)g.iq[2] / g.kmesh[2], pref, vs, flag);
}

void launch_eps(hipStream_t s, int nfreq, int ng, const double *vs, const double2 *chi, double2 *eps,
                int *flag)
{
    const long tot = (long)nfreq * ng * ng;
    hipLaunchKernelGGL(k_eps, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nfreq, ng, vs, chi,
                       eps, flag);
}

void launch_invert(hipStream_t s, int nfreq, int ng, double2 *a, double2 *col, int *piv, int *flag)
{
    const unsigned xb = (unsigned)std::min(8, (ng + 255) / 256);
    for (int c = 0; c < ng; c++) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(nfreq), dim3(256), 0, s, ng, c, a, col, piv, flag);
        hipLaunchKernelGGL(k_gj_elim, dim3(xb, ng, nfreq), dim3(256), 0, s, ng, c, a, col);
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
