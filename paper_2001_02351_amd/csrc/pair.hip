// Steps a3-a4: pair densities of one k (Eq. ism, FFT route).
//
//   M_p(G) = (1/N_r) sum_j conj(u_{a,k+q}(r_j)) u_{b,k}(r_j) e^{i(G+G0).r_j}
//
// One workgroup per block of NA empty x NB occupied bands (NA*NB pairs), so
// each u-grid row read from memory serves several pairs.  The grid is walked
// plane by plane along j1; each plane of each product is transformed along j3
// (in row chunks, keeping only the m3 window of the sphere), then along j2,
// and the sphere points accumulate their j1 phase e^{2 pi i m1 j1/N1} in
// registers, so no full-size intermediate ever leaves LDS.  The grids and
// transforms run in FP64 (double2) or FP32 (float2); M is written in FP64.
#include <algorithm>

#include "fft_lds.h"

namespace rp {

namespace {

template <typename C, int NA, int NB, int MAXG>
__global__ void __launch_bounds__(256)
k_pair(const C *__restrict__ u_occ, const C *__restrict__ u_emp, int nO, int nE, int N1, int N2, int N3,
       FftPlan p2, FftPlan p3, int ng, const int *__restrict__ gsph, int g01, int g02, int g03, int lo3,
       int L3, int rows, double2 *__restrict__ M)
{
    typedef typename CxT<C>::T T;
    constexpr int NP = NA * NB;
    extern __shared__ double2 smem_d[];
    C *smem = (C *)smem_d;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int nbB = (nO + NB - 1) / NB;
    const int a0 = (blockIdx.x / nbB) * NA, b0 = (blockIdx.x % nbB) * NB;
    const long nr = (long)N1 * N2 * N3;
    const C *ua[NA];
    const C *ub[NB];
#pragma unroll
    for (int i = 0; i < NA; i++) ua[i] = u_emp + (long)min(a0 + i, nE - 1) * nr;
#pragma unroll
    for (int i = 0; i < NB; i++) ub[i] = u_occ + (long)min(b0 + i, nO - 1) * nr;

    C *tw1 = smem;
    C *tw2 = tw1 + N1;
    C *tw3 = tw2 + N2;
    C *Cb = tw3 + N3;                        // [NP][N2][L3]
    C *D = Cb + (size_t)NP * N2 * L3;        // ping-pong partner, [N2][L3]
    const int ld3 = N3 + 1;
    C *P0 = D + (size_t)N2 * L3;             // [rows][N3+1]
    C *P1 = P0 + (size_t)rows * ld3;

    fill_twiddles(tw1, N1, tid, nth);
    fill_twiddles(tw2, N2, tid, nth);
    fill_twiddles(tw3, N3, tid, nth);

    // sphere points owned by this thread
    C acc[NP][MAXG];
    int cidx[MAXG], step1[MAXG], ph[MAXG];
#pragma unroll
    for (int t = 0; t < MAXG; t++) {
        const int g = tid + t * 256;
#pragma unroll
        for (int q = 0; q < NP; q++) acc[q][t] = mkc<C>(0, 0);
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
#pragma unroll
            for (int ia = 0; ia < NA; ia++)
#pragma unroll
                for (int ib = 0; ib < NB; ib++) {
                    for (int e = tid; e < nl * N3; e += nth) {
                        const int l = e / N3, i = e - l * N3;
                        P0[l * ld3 + i] = cmulc(ua[ia][base + e], ub[ib][base + e]);
                    }
                    __syncthreads();
                    const C *R = fft_lines(P0, P1, p3, nl, ld3, 1, tw3, tid, nth);
                    C *dst = Cb + (size_t)(ia * NB + ib) * N2 * L3;
                    for (int e = tid; e < nl * L3; e += nth) {
                        const int l = e / L3, t3 = e - l * L3;
                        dst[(rc + l) * L3 + t3] = R[l * ld3 + pmod(lo3 + t3, N3)];
                    }
                    __syncthreads();
                }
        }
        // transform along j2 (L3 lines of length N2, element stride L3) and
        // accumulate the j1 phase of every sphere point
#pragma unroll
        for (int q = 0; q < NP; q++) {
            const C *R2 = fft_lines(Cb + (size_t)q * N2 * L3, D, p2, L3, 1, L3, tw2, tid, nth);
#pragma unroll
            for (int t = 0; t < MAXG; t++) {
                const int g = tid + t * 256;
                if (g < ng) {
                    const C v = R2[cidx[t]];
                    const C e = tw1[ph[t]];
                    acc[q][t].x += v.x * e.x - v.y * e.y;
                    acc[q][t].y += v.x * e.y + v.y * e.x;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < MAXG; t++) {
            ph[t] += step1[t];
            if (ph[t] >= N1) ph[t] -= N1;
        }
    }
    const double inv = 1.0 / (double)nr;
#pragma unroll
    for (int ia = 0; ia < NA; ia++)
#pragma unroll
        for (int ib = 0; ib < NB; ib++) {
            const int a = a0 + ia, b = b0 + ib;
            if (a >= nE || b >= nO) continue;
            double2 *out = M + ((long)a * nO + b) * ng;
#pragma unroll
            for (int t = 0; t < MAXG; t++) {
                const int g = tid + t * 256;
                if (g < ng) out[g] = make_double2((double)acc[ia * NB + ib][t].x * inv,
                                                  (double)acc[ia * NB + ib][t].y * inv);
            }
        }
    (void)sizeof(T);
}

// Register-FFT form for compile-time N2 = N3 = N: per plane, (A) thread
// (pair q, row j2) forms the product row and transforms it along j3 in
// registers, keeping the m3 window; (B) thread (q, column t3) transforms along
// j2 in registers, in place; (C) every sphere point accumulates its j1 phase.
// The window buffer is double-buffered across planes: two barriers per plane.
template <typename C, int N, int NA, int NB, int MAXG>
__global__ void __launch_bounds__(256)
k_pair_reg(const C *__restrict__ u_occ, const C *__restrict__ u_emp, int nO, int nE, int N1, int ng,
           const int *__restrict__ gsph, int g01, int g02, int g03, int lo3, int L3, double2 *__restrict__ M)
{
    constexpr int NP = NA * NB;
    extern __shared__ double2 smem_d[];
    C *smem = (C *)smem_d;
    const int tid = threadIdx.x;
    const int nbB = (nO + NB - 1) / NB;
    const int a0 = (blockIdx.x / nbB) * NA, b0 = (blockIdx.x % nbB) * NB;
    const long nr = (long)N1 * N * N;

    C *tw1 = smem;
    C *twN = tw1 + N1;
    C *buf0 = twN + N;                                       // two [NP][N][L3] windows
    fill_twiddles(tw1, N1, tid, 256);
    fill_twiddles(twN, N, tid, 256);

    C acc[NP][MAXG];
    int cidx[MAXG], step1[MAXG], ph[MAXG];
#pragma unroll
    for (int t = 0; t < MAXG; t++) {
        const int g = tid + t * 256;
#pragma unroll
        for (int q = 0; q < NP; q++) acc[q][t] = mkc<C>(0, 0);
        cidx[t] = 0;
        step1[t] = 0;
        ph[t] = 0;
        if (g < ng) {
            const int m1 = gsph[3 * g] + g01, m2 = gsph[3 * g + 1] + g02, m3 = gsph[3 * g + 2] + g03;
            cidx[t] = pmod(m2, N) * L3 + (m3 - lo3);
            step1[t] = pmod(m1, N1);
        }
    }
    __syncthreads();

    for (int j1 = 0; j1 < N1; j1++) {
        C *B = buf0 + (size_t)(j1 & 1) * NP * N * L3;
        // (A) rows along j3
        for (int L = tid; L < NP * N; L += 256) {
            const int q = L / N, j2 = L - q * N;
            const int a = min(a0 + q / NB, nE - 1), b = min(b0 + q % NB, nO - 1);
            const long off = ((long)j1 * N + j2) * N;
            const C *ra = u_emp + (long)a * nr + off;
            const C *rb = u_occ + (long)b * nr + off;
            C x[N];
#pragma unroll
            for (int i = 0; i < N; i++) x[i] = cmulc(ra[i], rb[i]);
            reg_fft<N>(x, twN);
            C *dst = B + ((size_t)q * N + j2) * L3;
#pragma unroll
            for (int i = 0; i < N; i++) {
                int t3 = i - lo3;
                t3 = t3 < 0 ? t3 + N : (t3 >= N ? t3 - N : t3);
                if (t3 < L3) dst[t3] = x[i];
            }
        }
        __syncthreads();
        // (B) columns along j2, in place
        for (int L = tid; L < NP * L3; L += 256) {
            const int q = L / L3, t3 = L - q * L3;
            C *col = B + (size_t)q * N * L3 + t3;
            C y[N];
#pragma unroll
            for (int j2 = 0; j2 < N; j2++) y[j2] = col[j2 * L3];
            reg_fft<N>(y, twN);
#pragma unroll
            for (int m2 = 0; m2 < N; m2++) col[m2 * L3] = y[m2];
        }
        __syncthreads();
        // (C) sphere points
#pragma unroll
        for (int t = 0; t < MAXG; t++) {
            const int g = tid + t * 256;
            if (g < ng) {
                const C e = tw1[ph[t]];
#pragma unroll
                for (int q = 0; q < NP; q++) {
                    const C v = B[(size_t)q * N * L3 + cidx[t]];
                    acc[q][t].x += v.x * e.x - v.y * e.y;
                    acc[q][t].y += v.x * e.y + v.y * e.x;
                }
                ph[t] += step1[t];
                if (ph[t] >= N1) ph[t] -= N1;
            }
        }
    }
    const double inv = 1.0 / (double)nr;
#pragma unroll
    for (int q = 0; q < NP; q++) {
        const int a = a0 + q / NB, b = b0 + q % NB;
        if (a >= nE || b >= nO) continue;
        double2 *out = M + ((long)a * nO + b) * ng;
#pragma unroll
        for (int t = 0; t < MAXG; t++) {
            const int g = tid + t * 256;
            if (g < ng) out[g] = make_double2((double)acc[q][t].x * inv, (double)acc[q][t].y * inv);
        }
    }
}

// Workgroup barrier over LDS only: waits for this wave's LDS operations, not
// for global-to-LDS DMAs still in flight (which __syncthreads would drain).
__device__ __forceinline__ void lds_sync()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// widest m3 window the quad form holds in LDS (FP32 2x2 pair blocks, FP64
// 2x1 pair blocks: either way under 80 KB, two workgroups per CU)
template <typename C, int N> constexpr int quad_l3max()
{
    return sizeof(C) == 8 ? (N >= 48 ? N / 2 : N) : (N >= 48 ? N / 3 : (N >= 32 ? 24 : N));
}

// Quad-FFT form (FP32 or FP64), the path for N2 = N3 in {16, 24, 32, 48}.  Per plane
// j1: (A) each quad of lanes (pair q, row j2) loads its two grid rows (each
// lane a contiguous quarter, in 16-byte loads), forms the product and
// transforms it along j3 (quad_fft), keeping the m3 window; (B) each quad
// (q, column t3) transforms along j2 in place; (C) every sphere point
// accumulates its j1 phase in registers.  All four waves share phases A and B
// evenly, and a lane holds N/4 points of a line instead of N, which leaves
// room for the sphere accumulators.  The two m3-window buffers alternate
// between planes, so phase A of plane j1+1 may start while other waves still
// read plane j1's window in phase C: two barriers per plane.  LDS stays under
// half a CU's, so two workgroups share a CU and cover each other's load and
// barrier waits.
template <typename C, int N, int NA, int NB, int MAXG>
__global__ void __launch_bounds__(256, 2)
k_pair_quad(const C *__restrict__ u_occ, const C *__restrict__ u_emp, int nO, int nE, int N1, int ng,
            const int *__restrict__ gsph, int g01, int g02, int g03, int lo3, int L3, double2 *__restrict__ M)
{
    constexpr int Q = N / 4, NP = NA * NB;
    constexpr int L3M = quad_l3max<C, N>();
    constexpr int TA = (NP * N + 63) / 64;    // phase-A lines per quad
    __shared__ C win0[NP * N * L3M];          // [NP][N][L3]
    __shared__ C win1[NP * N * L3M];
    __shared__ C tw1[256];
    __shared__ C twN[N];
    __shared__ C twQ[Q];
    const int tid = threadIdx.x;
    const int s = tid & 3, quad = tid >> 2, r = quad_row(s);
    const int nbB = (nO + NB - 1) / NB;
    const int a0 = (blockIdx.x / nbB) * NA, b0 = (blockIdx.x % nbB) * NB;
    const long nr = (long)N1 * N * N;
    fill_twiddles(tw1, N1, tid, 256);
    fill_twiddles(twN, N, tid, 256);
    fill_twiddles(twQ, Q, tid, 256);

    C acc[NP][MAXG];
    int cidx[MAXG], step1[MAXG], ph[MAXG];
#pragma unroll
    for (int t = 0; t < MAXG; t++) {
        const int g = tid + t * 256;
#pragma unroll
        for (int q = 0; q < NP; q++) acc[q][t] = mkc<C>(0, 0);
        cidx[t] = 0;
        step1[t] = 0;
        ph[t] = 0;
        if (g < ng) {
            const int m1 = gsph[3 * g] + g01, m2 = gsph[3 * g + 1] + g02, m3 = gsph[3 * g + 2] + g03;
            cidx[t] = pmod(m2, N) * L3 + (m3 - lo3);
            step1[t] = pmod(m1, N1);
        }
    }
    __syncthreads();

    auto plane = [&](int j1, C *B) {
        // (A) product rows along j3
#pragma unroll 1
        for (int it = 0; it < TA; it++) {
            const int task = quad + 64 * it;
            if (task < NP * N) {
                const int q = task / N, j2 = task - q * N;
                const long off = ((long)j1 * N + j2) * N + Q * s;
                const C *ra = u_emp + (long)min(a0 + q / NB, nE - 1) * nr + off;
                const C *rb = u_occ + (long)min(b0 + q % NB, nO - 1) * nr + off;
                C x[Q];
                if constexpr (sizeof(C) == 8) {   // two FP32 complex values per 16-byte load
#pragma unroll
                    for (int n = 0; n < Q / 2; n++) {
                        const float4 va = ((const float4 *)ra)[n], vb = ((const float4 *)rb)[n];
                        x[2 * n] = cmulc(mkc<C>(va.x, va.y), mkc<C>(vb.x, vb.y));
                        x[2 * n + 1] = cmulc(mkc<C>(va.z, va.w), mkc<C>(vb.z, vb.w));
                    }
                } else {
#pragma unroll
                    for (int n = 0; n < Q; n++) x[n] = cmulc(ra[n], rb[n]);
                }
                quad_fft<Q>(x, twQ, twN, s);
                C *dst = B + ((size_t)q * N + j2) * L3;
#pragma unroll
                for (int k = 0; k < Q; k++) {
                    int t3 = 4 * k + r - lo3;
                    t3 = t3 < 0 ? t3 + N : (t3 >= N ? t3 - N : t3);
                    if (t3 < L3) dst[t3] = x[k];
                }
            }
        }
        lds_sync();
        // (B) columns along j2, in place (a quad reads its whole column
        // before any of its lanes writes)
        for (int task = quad; task < NP * L3; task += 64) {
            const int qq = task / L3, t3 = task - qq * L3;
            C *col = B + (size_t)qq * N * L3 + t3;
            C y[Q];
#pragma unroll
            for (int n = 0; n < Q; n++) y[n] = col[(Q * s + n) * L3];
            quad_fft<Q>(y, twQ, twN, s);
#pragma unroll
            for (int k = 0; k < Q; k++) col[(4 * k + r) * L3] = y[k];
        }
        lds_sync();
        // (C) sphere points
#pragma unroll
        for (int t = 0; t < MAXG; t++) {
            const int g = tid + t * 256;
            if (g < ng) {
                const C e = tw1[ph[t]];
#pragma unroll
                for (int qq = 0; qq < NP; qq++) {
                    const C v = B[(size_t)qq * N * L3 + cidx[t]];
                    acc[qq][t].x += v.x * e.x - v.y * e.y;
                    acc[qq][t].y += v.x * e.y + v.y * e.x;
                }
                ph[t] += step1[t];
                if (ph[t] >= N1) ph[t] -= N1;
            }
        }
    };
    // window j1 & 1 is rewritten by phase A of plane j1 + 2, which every
    // thread starts only after the barriers of plane j1 + 1
    for (int j1 = 0; j1 < N1; j1 += 2) {
        plane(j1, win0);
        if (j1 + 1 < N1) plane(j1 + 1, win1);
    }
    const double inv = 1.0 / (double)nr;
#pragma unroll
    for (int qq = 0; qq < NP; qq++) {
        const int a = a0 + qq / NB, b = b0 + qq % NB;
        if (a >= nE || b >= nO) continue;
        double2 *out = M + ((long)a * nO + b) * ng;
#pragma unroll
        for (int t = 0; t < MAXG; t++) {
            const int g = tid + t * 256;
            if (g < ng) out[g] = make_double2((double)acc[qq][t].x * inv, (double)acc[qq][t].y * inv);
        }
    }
}

template <typename C, int N, int NA, int NB>
void launch_pair_quad(hipStream_t s, int N1, const C *u_occ, const C *u_emp, int nO, int nE, int ng,
                      const int *gsph, const int g0[3], int lo3, int L3, double2 *M)
{
    const unsigned nblk = (unsigned)(((nE + NA - 1) / NA) * ((nO + NB - 1) / NB));
#define RP_PAIRQ(G)                                                                                          \
    hipLaunchKernelGGL((k_pair_quad<C, N, NA, NB, G>), dim3(nblk), dim3(256), 0, s, u_occ, u_emp, nO, nE, N1,\
                       ng, gsph, g0[0], g0[1], g0[2], lo3, L3, M)
    if (ng <= 512) RP_PAIRQ(2);
    else if (ng <= 1024) RP_PAIRQ(4);
    else if (ng <= 1536) RP_PAIRQ(6);
    else RP_PAIRQ(8);
#undef RP_PAIRQ
}

template <typename C, int N, int NA, int NB>
void launch_pair_reg(hipStream_t s, int N1, const C *u_occ, const C *u_emp, int nO, int nE, int ng,
                     const int *gsph, const int g0[3], int lo3, int L3, double2 *M)
{
    const size_t shm = sizeof(C) * ((size_t)N1 + N + 2 * (size_t)NA * NB * N * L3);
    const unsigned nblk = (unsigned)(((nE + NA - 1) / NA) * ((nO + NB - 1) / NB));
#define RP_PAIRR(G)                                                                                            \
    hipLaunchKernelGGL((k_pair_reg<C, N, NA, NB, G>), dim3(nblk), dim3(256), shm, s, u_occ, u_emp, nO, nE, N1, \
                       ng, gsph, g0[0], g0[1], g0[2], lo3, L3, M)
    if (ng <= 512) RP_PAIRR(2);
    else if (ng <= 1024) RP_PAIRR(4);
    else RP_PAIRR(8);
#undef RP_PAIRR
}

template <typename C, int NA, int NB>
void launch_pair_t(hipStream_t s, const FftPlan plans[3], const int fft[3], const C *u_occ, const C *u_emp,
                   int nO, int nE, int ng, const int *gsph, const int g0[3], int lo3, int L3, double2 *M)
{
    const int rows = pair_rows(fft);
    const size_t shm = pair_lds_bytes(fft, L3, rows, sizeof(C), NA * NB);
    const unsigned nblk = (unsigned)(((nE + NA - 1) / NA) * ((nO + NB - 1) / NB));
#define RP_PAIR(G)                                                                                          \
    hipLaunchKernelGGL((k_pair<C, NA, NB, G>), dim3(nblk), dim3(256), shm, s, u_occ, u_emp, nO, nE, fft[0], \
                       fft[1], fft[2], plans[1], plans[2], ng, gsph, g0[0], g0[1], g0[2], lo3, L3, rows, M)
    if (ng <= 512) RP_PAIR(2);
    else if (ng <= 1024) RP_PAIR(4);
    else if (ng <= 2048) RP_PAIR(8);
    else if (ng <= 4096) RP_PAIR(16);
    else RP_PAIR(24);
#undef RP_PAIR
}


}  // namespace

size_t pair_lds_bytes(const int fft[3], int L3, int rows, size_t csize, int npairs)
{
    return csize * ((size_t)fft[0] + fft[1] + fft[2] + (size_t)(npairs + 1) * fft[1] * L3 +
                    2 * (size_t)rows * (fft[2] + 1));
}

int pair_rows(const int fft[3]) { return std::max(1, std::min(fft[1], 768 / fft[2])); }

// lengths with a register-FFT instantiation (FP64 lines of 48 do not fit in
// registers and use the LDS form)
bool pair_reg_supported(const int fft[3], int ng, bool fp32)
{
    if (ng > 2048 || fft[1] != fft[2]) return false;
    switch (fft[1]) {
    case 16: case 24: case 32: return true;
    case 48: return fp32;
    default: return false;
    }
}

// the quad form: N2 = N3 in {16, 24, 32, 48}, N1 <= 256, ng <= 2048, and the
// m3 window within its LDS plan
template <typename C> static bool pair_quad_supported(const int fft[3], int ng, int L3)
{
    if (fft[0] > 256 || fft[1] != fft[2] || ng > 2048) return false;
    switch (fft[1]) {
    case 16: return L3 <= quad_l3max<C, 16>();
    case 24: return L3 <= quad_l3max<C, 24>();
    case 32: return L3 <= quad_l3max<C, 32>();
    case 48: return L3 <= quad_l3max<C, 48>();
    default: return false;
    }
}

void launch_pair_k(hipStream_t s, const FftPlan plans[3], const int fft[3], const void *u_occ,
                   const void *u_emp, int nO, int nE, int ng, const int *gsph, const int g0[3], int lo3,
                   int L3, bool fp32, double2 *M)
{
    if (fp32 && pair_quad_supported<float2>(fft, ng, L3)) {
        const float2 *uo = (const float2 *)u_occ, *ue = (const float2 *)u_emp;
        switch (fft[1]) {
        case 16: launch_pair_quad<float2, 16, 2, 2>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        case 24: launch_pair_quad<float2, 24, 2, 2>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        case 32: launch_pair_quad<float2, 32, 2, 2>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        case 48: launch_pair_quad<float2, 48, 2, 2>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        default: break;
        }
    }
    if (!fp32 && pair_quad_supported<double2>(fft, ng, L3)) {
        const double2 *uo = (const double2 *)u_occ, *ue = (const double2 *)u_emp;
        switch (fft[1]) {
        case 16: launch_pair_quad<double2, 16, 2, 1>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        case 24: launch_pair_quad<double2, 24, 2, 1>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        case 32: launch_pair_quad<double2, 32, 2, 1>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        case 48: launch_pair_quad<double2, 48, 2, 1>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M); return;
        default: break;
        }
    }
    if (fp32)
        launch_pair_t<float2, 2, 2>(s, plans, fft, (const float2 *)u_occ, (const float2 *)u_emp, nO, nE, ng,
                                    gsph, g0, lo3, L3, M);
    else
        launch_pair_t<double2, 1, 1>(s, plans, fft, (const double2 *)u_occ, (const double2 *)u_emp, nO, nE,
                                     ng, gsph, g0, lo3, L3, M);
}


}  // namespace rp
