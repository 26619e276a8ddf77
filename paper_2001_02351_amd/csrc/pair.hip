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
#include <type_traits>

#include "fft_lds.h"
#include "split_ops.h"

namespace rp {

namespace {

// The block's pair densities as split operands: pair (a, b) of this k is
// pair p0 + a nO + b of the contraction call.  The value is the FP64 M of the
// plain output, (double) acc / N_r, rounded to FP32, so the operands equal
// those the split preparation makes from M.  Two pairs b, b + 1 that share a
// group of 8 at an even position go out in one store.
// The band block of this workgroup.  Workgroup i is dispatched to XCD i mod 8;
// the blocks are renumbered so that each XCD takes a contiguous run of them:
// the blocks of one empty band (which read the same u-grid rows) and the
// blocks whose pairs share a group of 8 in the split operands (whose partial
// lines then merge in one L2) run on the same XCD.  A bijection of [0, n).
__device__ __forceinline__ int xcd_block()
{
    const int n = gridDim.x, x = blockIdx.x & 7;
    return x * (n >> 3) + min(x, n & 7) + (blockIdx.x >> 3);
}

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

template <typename C, int NA, int NB, int MAXG>
__device__ __forceinline__ void pair_ops_out(const C (&acc)[NA * NB][MAXG], int a0, int b0, int nO, int nE,
                                             int ng, int tid, double inv, const SplitOps &ops)
{
    auto val = [&](int q, int t) {
        return make_float2((float)((double)acc[q][t].x * inv), (float)((double)acc[q][t].y * inv));
    };
    // compile-time band indices, so that acc stays in registers
    static_for<0, NA>([&](auto IA) {
        constexpr int ia = decltype(IA)::value;
        const int a = a0 + ia;
        if (a >= nE) return;
        const long P0 = ops.p0 + (long)a * nO + b0;
        if constexpr (NB == 2) {
            if (b0 + 1 < nO && (P0 & 1) == 0) {
#pragma unroll
                for (int t = 0; t < MAXG; t++) {
                    const int g = tid + t * 256;
                    if (g < ng) ops_store2(ops, P0, g, val(ia * NB, t), val(ia * NB + 1, t));
                }
                return;
            }
        }
        static_for<0, NB>([&](auto IB) {
            constexpr int ib = decltype(IB)::value;
            if (b0 + ib >= nO) return;
#pragma unroll
            for (int t = 0; t < MAXG; t++) {
                const int g = tid + t * 256;
                if (g < ng) {
                    const float2 v = val(ia * NB + ib, t);
                    ops_store(ops, P0 + ib, g, v.x, v.y);
                }
            }
        });
    });
}

template <typename C, int NA, int NB, int MAXG>
__global__ void __launch_bounds__(256)
k_pair(const C *__restrict__ u_occ, const C *__restrict__ u_emp, int nO, int nE, int N1, int N2, int N3,
       FftPlan p2, FftPlan p3, int ng, const int *__restrict__ gsph, int g01, int g02, int g03, int lo3,
       int L3, int rows, double2 *__restrict__ M, SplitOps ops)
{
    typedef typename CxT<C>::T T;
    constexpr int NP = NA * NB;
    extern __shared__ double2 smem_d[];
    C *smem = (C *)smem_d;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int nbB = (nO + NB - 1) / NB;
    const int bid = xcd_block();
    const int a0 = (bid / nbB) * NA, b0 = (bid % nbB) * NB;
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
    if (ops.A) {
        pair_ops_out<C, NA, NB, MAXG>(acc, a0, b0, nO, nE, ng, tid, inv, ops);
        return;
    }
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

// Workgroup barrier over LDS only: waits for this wave's LDS operations, not
// for global-to-LDS DMAs still in flight (which __syncthreads would drain).
__device__ __forceinline__ void lds_sync()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// lanes per line for the lane-group form: 8 for the 96-point lines (12
// points per lane keep the registers for large spheres), else 4 when N is a
// multiple of 4, 2 when even, 1 when odd
template <int N> constexpr int pair_group()
{
    return N == 96 ? 8 : (N % 4 == 0 ? 4 : (N % 2 == 0 ? 2 : 1));
}

// widest m3 window the lane-group form holds in LDS: two windows of
// [NP][N][L3M] under 72 KB (FP32) or 48 KB (FP64), so that at least two
// workgroups share a CU (the windows are allocated at the call's own width)
template <typename C, int N, int NP> constexpr int lanes_l3max()
{
    constexpr int budget = sizeof(C) == 8 ? 73728 : 49152;
    constexpr int m = budget / (2 * NP * N * (int)sizeof(C));
    return m < N ? m : N;
}

// Lane-group form (FP32 or FP64), the path for N2 = N3 = N with a compile-time
// instantiation.  Per plane j1: (A) each group of G lanes (pair q, row j2)
// loads its two grid rows (each lane a contiguous 1/G of the row), forms the
// product and transforms it along j3 (group_fft), keeping the m3 window;
// (B) each group (q, column t3) transforms along j2 in place; (C) every
// sphere point accumulates its j1 phase in registers.  All four waves share
// phases A and B evenly, and a lane holds N/G points of a line, which leaves
// room for the sphere accumulators.  The two m3-window buffers alternate
// between planes, so phase A of plane j1+1 may start while other waves still
// read plane j1's window in phase C: two barriers per plane.  The windows take
// dynamic LDS of the call's window width: at least two workgroups share a CU
// (three for the 15-wide window of a 32-point grid, where the registers then
// limit it) and cover each other's load and barrier waits.
// waves per SIMD the lane-group form asks of the compiler: four for FP32 lines
// of up to 32 points on four lanes with at most 6 sphere points per thread
// (which then fit 128 registers), else two
template <typename C, int N, int MAXG> constexpr int pair_lanes_waves()
{
    return sizeof(C) == 8 && N % 4 == 0 && N <= 32 && MAXG <= 6 ? 4 : 2;
}

template <typename C, int N, int NA, int NB, int MAXG>
__global__ void __launch_bounds__(256, (pair_lanes_waves<C, N, MAXG>()))
k_pair_lanes(const C *__restrict__ u_occ, const C *__restrict__ u_emp, int nO, int nE, int N1, int ng,
             const int *__restrict__ gsph, int g01, int g02, int g03, int lo3, int L3, double2 *__restrict__ M,
             SplitOps ops)
{
    constexpr int G = pair_group<N>(), Q = N / G, NP = NA * NB;
    constexpr int NGRP = 256 / G;             // lane groups per workgroup
    constexpr int TA = (NP * N + NGRP - 1) / NGRP;    // phase-A lines per group
    extern __shared__ float4 pair_lanes_dyn[];
    C *win[2] = {(C *)pair_lanes_dyn, (C *)pair_lanes_dyn + (size_t)NP * N * L3};   // two windows [NP][N][L3]
    __shared__ C tw1[256];
    __shared__ C twN[N];
    __shared__ C twQ[Q];
    const int tid = threadIdx.x;
    const int s = tid & (G - 1), grp = tid / G, r = group_row<G>(s);
    const int nbB = (nO + NB - 1) / NB;
    const int bid = xcd_block();
    const int a0 = (bid / nbB) * NA, b0 = (bid % nbB) * NB;
    const long nr = (long)N1 * N * N;
    fill_twiddles(tw1, N1, tid, 256);
    fill_twiddles(twN, N, tid, 256);
    fill_twiddles(twQ, Q, tid, 256);

    C acc[NP][MAXG];
    // per sphere point, packed into one register: bits 0-13 the window index
    // (m2 mod N) L3 + m3 - lo3 (< N times the widest window <= 2304), bits 14-21 the j1 phase step
    // m1 mod N1, bits 22-29 the running phase index (N1 <= 256)
    unsigned pk[MAXG];
#pragma unroll
    for (int t = 0; t < MAXG; t++) {
        const int g = tid + t * 256;
#pragma unroll
        for (int q = 0; q < NP; q++) acc[q][t] = mkc<C>(0, 0);
        pk[t] = 0;
        if (g < ng) {
            const int m1 = gsph[3 * g] + g01, m2 = gsph[3 * g + 1] + g02, m3 = gsph[3 * g + 2] + g03;
            pk[t] = (unsigned)(pmod(m2, N) * L3 + (m3 - lo3)) | ((unsigned)pmod(m1, N1) << 14);
        }
    }
    __syncthreads();

    // (A) one product row along j3 (line task q, j2 of plane j1) into window B
    auto row_task = [&](int j1, int q, int j2, C *B) {
        const long off = ((long)j1 * N + j2) * N + Q * s;
        const C *ra = u_emp + (long)min(a0 + q / NB, nE - 1) * nr + off;
        const C *rb = u_occ + (long)min(b0 + q % NB, nO - 1) * nr + off;
        C x[Q];
        if constexpr (sizeof(C) == 8 && N % 2 == 0 && Q % 2 == 0) {
            // two FP32 complex values per 16-byte load (row and lane offsets
            // are even, grids 16-byte aligned)
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
        group_fft<G, Q>(x, twQ, twN, s);
        C *dst = B + ((size_t)q * N + j2) * L3;
#pragma unroll
        for (int k = 0; k < Q; k++) {
            int t3 = G * k + r - lo3;
            t3 = t3 < 0 ? t3 + N : (t3 >= N ? t3 - N : t3);
            if (t3 < L3) dst[t3] = x[k];
        }
    };
    // (B) one column along j2, in place (a group reads its whole column
    // before any of its lanes writes)
    auto col_task = [&](int qq, int t3, C *B) {
        C *col = B + (size_t)qq * N * L3 + t3;
        C y[Q];
#pragma unroll
        for (int n = 0; n < Q; n++) y[n] = col[(Q * s + n) * L3];
        group_fft<G, Q>(y, twQ, twN, s);
#pragma unroll
        for (int k = 0; k < Q; k++) col[(G * k + r) * L3] = y[k];
    };
    // (C) the sphere points accumulate one plane's window with its j1 phase
    auto sphere = [&](const C *B) {
#pragma unroll
        for (int t = 0; t < MAXG; t++) {
            const int g = tid + t * 256;
            if (g < ng) {
                const unsigned u = pk[t];
                const int ci = (int)(u & 0x3fffu), st = (int)((u >> 14) & 0xffu);
                int ph = (int)(u >> 22);
                const C e = tw1[ph];
#pragma unroll
                for (int qq = 0; qq < NP; qq++) {
                    const C v = B[(size_t)qq * N * L3 + ci];
                    acc[qq][t].x += v.x * e.x - v.y * e.y;
                    acc[qq][t].y += v.x * e.y + v.y * e.x;
                }
                ph += st;
                if (ph >= N1) ph -= N1;
                pk[t] = (u & 0x3fffffu) | ((unsigned)ph << 22);
            }
        }
    };
    if constexpr (G <= 2) {
        // one or two lanes per line leave too few line tasks in one plane to
        // occupy the workgroup: phases A and B take two planes at a time, and
        // a third barrier keeps the next pair's rows out of the windows until
        // every sphere point has read them
        constexpr int TA2 = (2 * NP * N + NGRP - 1) / NGRP;
        for (int j1 = 0; j1 < N1; j1 += 2) {
            const int npl = min(2, N1 - j1);
#pragma unroll 1
            for (int it = 0; it < TA2; it++) {
                const int task = grp + NGRP * it;
                if (task < npl * NP * N) {
                    const int pl = task / (NP * N), t2 = task - pl * (NP * N);
                    row_task(j1 + pl, t2 / N, t2 % N, win[pl]);
                }
            }
            lds_sync();
            for (int task = grp; task < npl * NP * L3; task += NGRP) {
                const int pl = task / (NP * L3), t2 = task - pl * (NP * L3);
                col_task(t2 / L3, t2 % L3, win[pl]);
            }
            lds_sync();
            sphere(win[0]);
            if (npl == 2) sphere(win[1]);
            lds_sync();
        }
    } else {
        auto plane = [&](int j1, C *B) {
#pragma unroll 1
            for (int it = 0; it < TA; it++) {
                const int task = grp + NGRP * it;
                if (task < NP * N) row_task(j1, task / N, task % N, B);
            }
            lds_sync();
            for (int task = grp; task < NP * L3; task += NGRP) col_task(task / L3, task % L3, B);
            lds_sync();
            sphere(B);
        };
        // window j1 & 1 is rewritten by phase A of plane j1 + 2, which every
        // thread starts only after the barriers of plane j1 + 1
        for (int j1 = 0; j1 < N1; j1 += 2) {
            plane(j1, win[0]);
            if (j1 + 1 < N1) plane(j1 + 1, win[1]);
        }
    }
    const double inv = 1.0 / (double)nr;
    if (ops.A) {
        pair_ops_out<C, NA, NB, MAXG>(acc, a0, b0, nO, nE, ng, tid, inv, ops);
        return;
    }
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
void launch_pair_lanes(hipStream_t s, int N1, const C *u_occ, const C *u_emp, int nO, int nE, int ng,
                       const int *gsph, const int g0[3], int lo3, int L3, double2 *M, const SplitOps &ops)
{
    const unsigned nblk = (unsigned)(((nE + NA - 1) / NA) * ((nO + NB - 1) / NB));
    // the two m3 windows, sized by this window (not its largest allowed width):
    // narrow windows leave room for a third workgroup per CU
    const size_t shm = 2 * sizeof(C) * (size_t)(NA * NB) * N * L3;
#define RP_PAIRL(G)                                                                                          \
    do {                                                                                                     \
        if (shm > 65536)                                                                                     \
            (void)hipFuncSetAttribute((const void *)&k_pair_lanes<C, N, NA, NB, G>,                          \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);                 \
        hipLaunchKernelGGL((k_pair_lanes<C, N, NA, NB, G>), dim3(nblk), dim3(256), shm, s, u_occ, u_emp, nO, \
                           nE, N1, ng, gsph, g0[0], g0[1], g0[2], lo3, L3, M, ops);                          \
    } while (0)
    if constexpr (N >= 96) {
        // large grids come with large spheres: 2048, 4096 or 6144 points
        if (ng <= 2048) RP_PAIRL(8);
        else if (ng <= 4096) RP_PAIRL(16);
        else RP_PAIRL(24);
    } else {
        if (ng <= 512) RP_PAIRL(2);
        else if (ng <= 1024) RP_PAIRL(4);
        else if (ng <= 1536) RP_PAIRL(6);
        else RP_PAIRL(8);
    }
#undef RP_PAIRL
}

template <typename C, int NA, int NB>
void launch_pair_t(hipStream_t s, const FftPlan plans[3], const int fft[3], const C *u_occ, const C *u_emp,
                   int nO, int nE, int ng, const int *gsph, const int g0[3], int lo3, int L3, double2 *M,
                   const SplitOps &ops)
{
    const int rows = pair_rows(fft);
    const size_t shm = pair_lds_bytes(fft, L3, rows, sizeof(C), NA * NB);
    const unsigned nblk = (unsigned)(((nE + NA - 1) / NA) * ((nO + NB - 1) / NB));
#define RP_PAIR(G)                                                                                          \
    hipLaunchKernelGGL((k_pair<C, NA, NB, G>), dim3(nblk), dim3(256), shm, s, u_occ, u_emp, nO, nE, fft[0], \
                       fft[1], fft[2], plans[1], plans[2], ng, gsph, g0[0], g0[1], g0[2], lo3, L3, rows, M, \
                       ops)
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

// The lane-group form's lengths: N2 = N3 = N in these lists, N1 <= 256,
// ng <= 2048, and the m3 window within its LDS plan.  The band blocks are
// 2x2 pairs in FP32 and 2x1 in FP64.  FP32 N = 96 (the supercell grid) takes
// 2x1 blocks, so that a window of 24 fits, and spheres up to 6144 points.  FP64 lines of 25, 27 and 30 (one or two
// lanes per line) do not fit in registers and use the generic form.
#define RP_LANE_LENGTHS_F32(X) X(16) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(48)
#define RP_LANE_LENGTHS_F64(X) X(16) X(24) X(32) X(36) X(40) X(48)

static bool pair_lanes_f32(const int fft[3], int ng, int L3)
{
    if (fft[0] > 256 || fft[1] != fft[2]) return false;
    if (fft[1] == 96) return ng <= 6144 && L3 <= lanes_l3max<float2, 96, 2>();
    if (ng > 2048) return false;
    switch (fft[1]) {
#define RP_CASE(n) \
    case n: return L3 <= lanes_l3max<float2, n, 4>();
        RP_LANE_LENGTHS_F32(RP_CASE)
#undef RP_CASE
    default: return false;
    }
}

static bool pair_lanes_f64(const int fft[3], int ng, int L3)
{
    if (fft[0] > 256 || fft[1] != fft[2] || ng > 2048) return false;
    switch (fft[1]) {
#define RP_CASE(n) \
    case n: return L3 <= lanes_l3max<double2, n, 2>();
        RP_LANE_LENGTHS_F64(RP_CASE)
#undef RP_CASE
    default: return false;
    }
}

int pair_lane_edge(int need, int limit, int ng, int L3, bool fp32)
{
    int best = 0;
    auto take = [&](int n) {
        const int f[3] = {1, n, n};
        if (n < need || n > limit || (best && n >= best)) return;
        if (fp32 ? pair_lanes_f32(f, ng, L3) : pair_lanes_f64(f, ng, L3)) best = n;
    };
#define RP_CASE(n) take(n);
    if (fp32) {
        RP_LANE_LENGTHS_F32(RP_CASE)
        take(96);
    } else {
        RP_LANE_LENGTHS_F64(RP_CASE)
    }
#undef RP_CASE
    return best;
}

bool pair_supported(const int fft[3], int ng, int L3, bool fp32)
{
    if (fp32 ? pair_lanes_f32(fft, ng, L3) : pair_lanes_f64(fft, ng, L3)) return true;
    // the generic form's LDS plan (band blocks of 2x2 in FP32, 1x1 in FP64)
    return pair_lds_bytes(fft, L3, pair_rows(fft), fp32 ? 8 : 16, fp32 ? 4 : 1) <= 160 * 1024;
}

// the FP32 or FP64 pair kernel for this grid: the lane-group form when it
// takes the grid, sphere and window, else the generic LDS form
static void launch_pair_any(hipStream_t s, const FftPlan plans[3], const int fft[3], const void *u_occ,
                            const void *u_emp, int nO, int nE, int ng, const int *gsph, const int g0[3], int lo3,
                            int L3, bool fp32, double2 *M, const SplitOps &ops)
{
    if (fp32 && pair_lanes_f32(fft, ng, L3)) {
        const float2 *uo = (const float2 *)u_occ, *ue = (const float2 *)u_emp;
        switch (fft[1]) {
#define RP_CASE(n)                                                                                          \
        case n:                                                                                             \
            launch_pair_lanes<float2, n, 2, 2>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M, ops);   \
            return;
            RP_LANE_LENGTHS_F32(RP_CASE)
#undef RP_CASE
        case 96: launch_pair_lanes<float2, 96, 2, 1>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M, ops); return;
        default: break;
        }
    }
    if (!fp32 && pair_lanes_f64(fft, ng, L3)) {
        const double2 *uo = (const double2 *)u_occ, *ue = (const double2 *)u_emp;
        switch (fft[1]) {
#define RP_CASE(n)                                                                                          \
        case n:                                                                                             \
            launch_pair_lanes<double2, n, 2, 1>(s, fft[0], uo, ue, nO, nE, ng, gsph, g0, lo3, L3, M, ops);  \
            return;
            RP_LANE_LENGTHS_F64(RP_CASE)
#undef RP_CASE
        default: break;
        }
    }
    if (fp32)
        launch_pair_t<float2, 2, 2>(s, plans, fft, (const float2 *)u_occ, (const float2 *)u_emp, nO, nE, ng,
                                    gsph, g0, lo3, L3, M, ops);
    else
        launch_pair_t<double2, 1, 1>(s, plans, fft, (const double2 *)u_occ, (const double2 *)u_emp, nO, nE,
                                     ng, gsph, g0, lo3, L3, M, ops);
}

void launch_pair_k(hipStream_t s, const FftPlan plans[3], const int fft[3], const void *u_occ,
                   const void *u_emp, int nO, int nE, int ng, const int *gsph, const int g0[3], int lo3,
                   int L3, bool fp32, double2 *M)
{
    launch_pair_any(s, plans, fft, u_occ, u_emp, nO, nE, ng, gsph, g0, lo3, L3, fp32, M, SplitOps{});
}

void launch_pair_ops(hipStream_t s, const FftPlan plans[3], const int fft[3], const void *u_occ,
                     const void *u_emp, int nO, int nE, int ng, const int *gsph, const int g0[3], int lo3, int L3,
                     const SplitOps &ops)
{
    launch_pair_any(s, plans, fft, u_occ, u_emp, nO, nE, ng, gsph, g0, lo3, L3, true, nullptr, ops);
}

}  // namespace rp
