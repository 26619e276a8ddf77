// Step a6 in FP64 (Eq. chi): chi_GG'(w) (+)= sum_p w_p(w) M_p(G) conj(M_p(G'))
// on FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// Each pair p contributes a rank-one term, so over a batch of pairs chi(w) is
// the complex product (M o w(w))^T conj(M) with the pair index as the
// contraction dimension.  Complex arithmetic uses four real products:
//   Re chi += Re(a) Re(b) + Im(a) Im(b),   Im chi += Im(a) Re(b) - Re(a) Im(b)
// with a = w_p M_p(G) and b = M_p(G').
//
// Tiling: a 256-thread block owns a 64x64 tile of (G, G') for NW frequencies;
// each wave owns a 32x32 sub-tile (2x2 blocks of 16x16).  Operands are read
// straight from global memory in the matrix-core lane layout (lane = i + 16 k:
// 16 consecutive G of one pair, 256 contiguous bytes), prefetched one step ahead.
#include "fft_lds.h"

namespace rp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NW>
__global__ void __launch_bounds__(256)
k_chi_f64(long npair, int ng, const double2 *__restrict__ M, int nfreq, const double2 *__restrict__ w,
          int accumulate, double2 *__restrict__ chi)
{
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int row0 = blockIdx.y * 64 + (wave >> 1) * 32;   // G
    const int col0 = blockIdx.x * 64 + (wave & 1) * 32;    // G'
    const int f0 = blockIdx.z * NW;

    d4 accR[NW][2][2], accI[NW][2][2];
#pragma unroll
    for (int iw = 0; iw < NW; iw++)
#pragma unroll
        for (int rb = 0; rb < 2; rb++)
#pragma unroll
            for (int cb = 0; cb < 2; cb++) {
                accR[iw][rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
                accI[iw][rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
            }

    const int gr[2] = {row0 + li, row0 + 16 + li};
    const int gc[2] = {col0 + li, col0 + 16 + li};
    const bool okr[2] = {gr[0] < ng, gr[1] < ng};
    const bool okc[2] = {gc[0] < ng, gc[1] < ng};
    bool okf[NW];
#pragma unroll
    for (int iw = 0; iw < NW; iw++) okf[iw] = f0 + iw < nfreq;

    const double2 zero = make_double2(0.0, 0.0);
    double2 ar[2], bc[2], wv[NW];
    auto load = [&](long p0) {
        const long p = p0 + lk;
        const bool ok = p < npair;
        const double2 *row = M + p * ng;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            ar[t] = (ok && okr[t]) ? row[gr[t]] : zero;
            bc[t] = (ok && okc[t]) ? row[gc[t]] : zero;
        }
#pragma unroll
        for (int iw = 0; iw < NW; iw++) wv[iw] = (ok && okf[iw]) ? w[(long)(f0 + iw) * npair + p] : zero;
    };

    load(0);
    for (long p0 = 0; p0 < npair; p0 += 4) {
        const double2 a0 = ar[0], a1 = ar[1], b0 = bc[0], b1 = bc[1];
        double2 wc[NW];
#pragma unroll
        for (int iw = 0; iw < NW; iw++) wc[iw] = wv[iw];
        if (p0 + 4 < npair) load(p0 + 4);
        const double2 av[2] = {a0, a1}, bv[2] = {b0, b1};
#pragma unroll
        for (int iw = 0; iw < NW; iw++) {
#pragma unroll
            for (int rb = 0; rb < 2; rb++) {
                const double2 a = cmul(av[rb], wc[iw]);
#pragma unroll
                for (int cb = 0; cb < 2; cb++) {
                    accR[iw][rb][cb] = mfma64(a.x, bv[cb].x, accR[iw][rb][cb]);
                    accR[iw][rb][cb] = mfma64(a.y, bv[cb].y, accR[iw][rb][cb]);
                    accI[iw][rb][cb] = mfma64(a.y, bv[cb].x, accI[iw][rb][cb]);
                    accI[iw][rb][cb] = mfma64(-a.x, bv[cb].y, accI[iw][rb][cb]);
                }
            }
        }
    }

    // result register r of lane (li, lk) holds row lk + 4 r, column li of a 16x16 block
#pragma unroll
    for (int iw = 0; iw < NW; iw++) {
        if (!okf[iw]) continue;
        double2 *C = chi + (long)(f0 + iw) * ng * ng;
#pragma unroll
        for (int rb = 0; rb < 2; rb++)
#pragma unroll
            for (int cb = 0; cb < 2; cb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = row0 + rb * 16 + lk + 4 * r;
                    const int j = col0 + cb * 16 + li;
                    if (i < ng && j < ng) {
                        double2 v = make_double2(accR[iw][rb][cb][r], accI[iw][rb][cb][r]);
                        const long idx = (long)i * ng + j;
                        if (accumulate) v = cadd(C[idx], v);
                        C[idx] = v;
                    }
                }
    }
}

}  // namespace

void launch_chi_f64(hipStream_t s, long npair, int ng, const double2 *M, int nfreq, const double2 *w,
                    int accumulate, double2 *chi)
{
    const unsigned t = (unsigned)((ng + 63) / 64);
    if (nfreq >= 4) {
        hipLaunchKernelGGL(k_chi_f64<4>, dim3(t, t, (nfreq + 3) / 4), dim3(256), 0, s, npair, ng, M, nfreq,
                           w, accumulate, chi);
    } else if (nfreq >= 2) {
        hipLaunchKernelGGL(k_chi_f64<2>, dim3(t, t, (nfreq + 1) / 2), dim3(256), 0, s, npair, ng, M, nfreq,
                           w, accumulate, chi);
    } else {
        hipLaunchKernelGGL(k_chi_f64<1>, dim3(t, t, nfreq), dim3(256), 0, s, npair, ng, M, nfreq, w,
                           accumulate, chi);
    }
}

}  // namespace rp
