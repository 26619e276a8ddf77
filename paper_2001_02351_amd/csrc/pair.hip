// Steps a3-a4: pair densities of one k (Eq. ism, FFT route).
//
//   M_p(G) = (1/N_r) sum_j conj(u_{a,k+q}(r_j)) u_{b,k}(r_j) e^{i(G+G0).r_j}
//
// One workgroup per pair (a, b).  The grid is walked plane by plane along
// j1; each plane of the product is transformed along j3 (in row chunks, only
// the m3 window of the sphere is kept), then along j2, and the sphere points
// accumulate their j1 phase e^{2 pi i m1 j1 / N1} directly, so that no
// full-size intermediate ever leaves LDS.  The u-grids are read once per pair
// straight from HBM/L2 with coalesced row loads.
#include "fft_lds.h"

namespace rp {

namespace {

template <int MAXG>
__global__ void __launch_bounds__(256)
k_pair(const double2 *__restrict__ u_occ, const double2 *__restrict__ u_emp, int nO, int N1, int N2,
       int N3, FftPlan p2, FftPlan p3, int ng, const int *__restrict__ gsph, int g01, int g02,
       int g03, int lo3, int L3, int rows, double2 *__restrict__ M)
{
    extern __shared__ double2 smem[];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int pair = blockIdx.x;
    const int a = pair / nO, b = pair - a * nO;
    const long nr = (long)N1 * N2 * N3;
    const double2 *ua = u_emp + (long)a * nr;
    const double2 *ub = u_occ + (long)b * nr;

    double2 *tw1 = smem;
    double2 *tw2 = tw1 + N1;
    double2 *tw3 = tw2 + N2;
    double2 *C = tw3 + N3;               // [N2][L3]
    double2 *D = C + (size_t)N2 * L3;    // ping-pong partner of C
    const int ld3 = N3 + 1;
    double2 *P0 = D + (size_t)N2 * L3;   // [rows][N3+1]
    double2 *P1 = P0 + (size_t)rows * ld3;

    fill_twiddles(tw1, N1, tid, nth);
    fill_twiddles(tw2, N2, tid, nth);
    fill_twiddles(tw3, N3, tid, nth);

    // sphere points owned by this thread
    double2 acc[MAXG];
    int cidx[MAXG], step1[MAXG], ph[MAXG];
#pragma unroll
    for (int t = 0; t < MAXG; t++) {
        const int g = tid + t * 256;
        acc[t] = make_double2(0.0, 0.0);
        cidx[t] = 0;
        step1[t] = 0;
        ph[t] = 0;
        if (g < ng) {
            const int m1 = gsph[3 * g] + g01, m2 = gsph[3 * g + 1] + g02, m3 = gsph[3 * g + 2] + g03;
            cidx[t] = pmod(m2, N2) * L3 + (m3 - lo3);
            step1[t] = pmod(m1, N1);
        }
    }
    __syncthreads();

    for (int j1 = 0; j1 < N1; j1++) {
        const long plane = (long)j1 * N2 * N3;
        // transform along j3, row chunk by row chunk; keep the m3 window
        for (int rc = 0; rc < N2; rc += rows) {
            const int nl = min(rows, N2 - rc);
            const long base = plane + (long)rc * N3;
            for (int e = tid; e < nl * N3; e += nth) {
                const int l = e / N3, i = e - l * N3;
                P0[l * ld3 + i] = cmulc(ua[base + e], ub[base + e]);
            }
            __syncthreads();
            const double2 *R = fft_lines(P0, P1, p3, nl, ld3, 1, tw3, tid, nth);
            for (int e = tid; e < nl * L3; e += nth) {
                const int l = e / L3, t3 = e - l * L3;
                C[(rc + l) * L3 + t3] = R[l * ld3 + pmod(lo3 + t3, N3)];
            }
            __syncthreads();
        }
        // transform along j2: L3 lines of length N2, element stride L3
        const double2 *R2 = fft_lines(C, D, p2, L3, 1, L3, tw2, tid, nth);
        // accumulate the j1 phase of every sphere point
#pragma unroll
        for (int t = 0; t < MAXG; t++) {
            const int g = tid + t * 256;
            if (g < ng) {
                const double2 v = R2[cidx[t]];
                const double2 e = tw1[ph[t]];
                acc[t].x += v.x * e.x - v.y * e.y;
                acc[t].y += v.x * e.y + v.y * e.x;
                ph[t] += step1[t];
                if (ph[t] >= N1) ph[t] -= N1;
            }
        }
        __syncthreads();
    }
    const double inv = 1.0 / (double)nr;
    double2 *out = M + (long)pair * ng;
#pragma unroll
    for (int t = 0; t < MAXG; t++) {
        const int g = tid + t * 256;
        if (g < ng) out[g] = cscale(acc[t], inv);
    }
}

}  // namespace

size_t pair_lds_bytes(const int fft[3], int L3, int rows)
{
    return sizeof(double2) * ((size_t)fft[0] + fft[1] + fft[2] + 2 * (size_t)fft[1] * L3 +
                              2 * (size_t)rows * (fft[2] + 1));
}

int pair_rows(const int fft[3]) { return std::max(1, std::min(fft[1], 768 / fft[2])); }

void launch_pair_k(hipStream_t s, const FftPlan plans[3], const int fft[3], const double2 *u_occ,
                   const double2 *u_emp, int nO, int nE, int ng, const int *gsph, const int g0[3],
                   int lo3, int L3, double2 *M)
{
    const int rows = pair_rows(fft);
    const size_t shm = pair_lds_bytes(fft, L3, rows);
    const dim3 grid((unsigned)(nO * nE)), block(256);
#define RP_PAIR(G)                                                                                     \
    hipLaunchKernelGGL(k_pair<G>, grid, block, shm, s, u_occ, u_emp, nO, fft[0], fft[1], fft[2],      \
                       plans[1], plans[2], ng, gsph, g0[0], g0[1], g0[2], lo3, L3, rows, M)
    if (ng <= 512) RP_PAIR(2);
    else if (ng <= 1024) RP_PAIR(4);
    else if (ng <= 2048) RP_PAIR(8);
    else if (ng <= 4096) RP_PAIR(16);
    else RP_PAIR(24);
#undef RP_PAIR
}

}  // namespace rp
