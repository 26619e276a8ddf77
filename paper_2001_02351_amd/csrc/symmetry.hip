// Symmetry unfolding (section "Symmetry", Eqs. coef-G and symeps) for an
// operation x -> W x + t on fractional coordinates, S = W^{-T} on fractional
// reciprocal coordinates, k = S k* + Delta:
//
//   C_G(k)          = C_{S^{-1}(G+Delta)}(k*) e^{-2 pi i (m + Delta).t}
//   X_{G,G'}(q)     = X_{S^{-1}(G+Delta), S^{-1}(G'+Delta)}(q*) e^{+2 pi i (m - m').t}
//
// (m, m' the Miller indices of G, G'; X = eps^-1 or chi).  The source index
// of every target vector is resolved on the host; the kernels gather and
// apply the phases.  Both are bound by HBM traffic: one read and one write of
// every element.
#include "fft_lds.h"

namespace rp {

namespace {

// coef[b][g] = src[b][idx[g]] e^{-2 pi i (m_g + Delta).t}; one thread per (b, g)
__global__ void k_unfold_coef(int nband, int npw, const int *__restrict__ idx, const int *__restrict__ miller,
                              int d0, int d1, int d2, double t0, double t1, double t2, const double2 *__restrict__ src,
                              long ld_src, double2 *__restrict__ dst, long ld_dst)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nband * npw) return;
    const int b = (int)(t / npw), g = (int)(t - (long)b * npw);
    const int *m = miller + 3 * g;
    // the phase argument reduced mod 1 before the sine and cosine
    double a = (double)(m[0] + d0) * t0 + (double)(m[1] + d1) * t1 + (double)(m[2] + d2) * t2;
    a -= floor(a);
    double s, c;
    sincospi(-2.0 * a, &s, &c);
    dst[(long)b * ld_dst + g] = cmul(src[(long)b * ld_src + idx[g]], make_double2(c, s));
}

// ph[g] = e^{+2 pi i m_g.t}
__global__ void k_unfold_phase(int ng, const int *__restrict__ gsph, double t0, double t1, double t2,
                               double2 *__restrict__ ph)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int *m = gsph + 3 * g;
    double a = (double)m[0] * t0 + (double)m[1] * t1 + (double)m[2] * t2;
    a -= floor(a);
    double s, c;
    sincospi(2.0 * a, &s, &c);
    ph[g] = make_double2(c, s);
}

// dst[f][g][h] = src[f][idx[g]][idx[h]] ph[g] conj(ph[h]); block per (row
// chunk, f), the source indices staged in LDS (4 ng bytes), the phases read
// through the cache
__global__ void __launch_bounds__(256) k_unfold_matrix(int ng, int ng_src, const int *__restrict__ idx,
                                                       const double2 *__restrict__ ph, const double2 *__restrict__ src,
                                                       double2 *__restrict__ dst)
{
    constexpr int kRows = 4;
    extern __shared__ int sidx[];
    const int f = blockIdx.y, tid = threadIdx.x;
    for (int h = tid; h < ng; h += 256) sidx[h] = idx[h];
    __syncthreads();
    const double2 *S = src + (long)f * ng_src * ng_src;
    double2 *D = dst + (long)f * ng * ng;
    for (int r = 0; r < kRows; r++) {
        const int g = blockIdx.x * kRows + r;
        if (g >= ng) break;
        const double2 pg = ph[g];
        const double2 *row = S + (long)sidx[g] * ng_src;
        for (int h = tid; h < ng; h += 256) D[(long)g * ng + h] = cmulc(ph[h], cmul(row[sidx[h]], pg));
    }
}

}  // namespace

void launch_unfold_coef(hipStream_t s, int nband, int npw, const int *idx, const int *miller, const int delta[3],
                        const double t[3], const double2 *src, long ld_src, double2 *dst, long ld_dst)
{
    const long n = (long)nband * npw;
    if (n == 0) return;
    hipLaunchKernelGGL(k_unfold_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nband, npw, idx, miller,
                       delta[0], delta[1], delta[2], t[0], t[1], t[2], src, ld_src, dst, ld_dst);
}

size_t unfold_matrix_lds(int ng) { return sizeof(int) * (size_t)ng; }

void launch_unfold_matrix(hipStream_t s, int nfreq, int ng, int ng_src, const int *idx, const int *gsph,
                          const double t[3], double2 *ph, const double2 *src, double2 *dst)
{
    hipLaunchKernelGGL(k_unfold_phase, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, ng, gsph, t[0], t[1],
                       t[2], ph);
    hipLaunchKernelGGL(k_unfold_matrix, dim3((unsigned)((ng + 3) / 4), (unsigned)nfreq), dim3(256),
                       unfold_matrix_lds(ng), s, ng, ng_src, idx, ph, src, dst);
}

}  // namespace rp
