// Step a6 in FP64 (Eq. chi): chi_GG'(w) (+)= sum_p w_p(w) M_p(G) conj(M_p(G'))
// on FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// Each pair p contributes a rank-one term, so over a batch of pairs chi(w) is
// the complex product (M o w(w))^T conj(M) with the pair index as the
// contraction dimension.  Complex arithmetic uses four real products:
//   Re chi += Re(a) Re(b) + Im(a) Im(b),   Im chi += Im(a) Re(b) - Re(a) Im(b)
// with a = w_p M_p(G) and b = M_p(G').
//
// Tiling: a 256-thread block owns a 64x64 tile of (G, G') for NW = 4
// frequencies; each wave owns a 32x32 sub-tile (2x2 blocks of 16x16).  The
// pair dimension is consumed in chunks of 16 pairs staged through LDS with two
// buffers: while the matrix cores work on one chunk, the next chunk's 32 rows
// of 1 KB (16 pairs x 64 G, and 16 pairs x 64 G') stream from HBM/L2 straight
// into the other buffer (global_load_lds, no staging registers).  Rows and
// pairs past the end are clamped to valid addresses: clamped rows are never
// stored and clamped pairs carry zero weight.
#include "fft_lds.h"

namespace rp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kT = 64;     // tile edge
constexpr int kKC = 16;    // pairs per chunk
constexpr int kNW = 4;     // frequencies per block

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void dma16(const void *src, void *lds)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

// Tile (rt, ct) of block index id: row-major over the t x t tiles, or over
// the upper triangle rt <= ct when only that half is formed.
__device__ __forceinline__ void tile_of(int id, int t, int herm, int &rt, int &ct)
{
    if (!herm) {
        rt = id / t;
        ct = id - rt * t;
        return;
    }
    rt = 0;
    while (id >= t - rt) {
        id -= t - rt;
        rt++;
    }
    ct = rt + id;
}

// herm: the weights are real (imaginary frequencies, no broadening), so chi
// is Hermitian: their imaginary parts (rounding residue) are dropped, only
// the tiles rt <= ct are formed, and an off-diagonal tile also writes its
// conjugate transpose into the mirrored tile.
template <int NW>
__global__ void __launch_bounds__(256)
k_chi_f64(long npair, int ng, const double2 *__restrict__ M, int nfreq, const double2 *__restrict__ w,
          int accumulate, int herm, double2 *__restrict__ chi)
{
    // [stage][A rows | B cols][pair][64] double2, then [stage][NW][pair] weights
    __shared__ double2 sm[2][2][kKC][kT];
    __shared__ double2 sw[2][NW][kKC];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    int rt, ct;
    tile_of(blockIdx.x, (ng + kT - 1) / kT, herm, rt, ct);
    const int rt0 = rt * kT, ct0 = ct * kT;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int f0 = blockIdx.z * NW;
    const long nchunk = (npair + kKC - 1) / kKC;

    // DMA assignment: wave w moves pairs 4w..4w+3 of both operands
    const int rowA = min(rt0 + lane, ng - 1);
    const int colB = min(ct0 + lane, ng - 1);
    auto issue = [&](int stg, long c) {
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int pp = wave * 4 + t;
            const long p = min(c * kKC + pp, npair - 1);
            dma16(M + p * ng + rowA, &sm[stg][0][pp][0]);
            dma16(M + p * ng + colB, &sm[stg][1][pp][0]);
        }
    };
    // weights: thread tid < NW*16 stages one value through a register
    const int wiw = tid / kKC, wpp = tid % kKC;
    auto wload = [&](long c) -> double2 {
        const long p = c * kKC + wpp;
        if (tid < NW * kKC && p < npair && f0 + wiw < nfreq) {
            const double2 v = w[(long)(f0 + wiw) * npair + p];
            return make_double2(v.x, herm ? 0.0 : v.y);
        }
        return make_double2(0.0, 0.0);
    };

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

    if (nchunk > 0) {
        issue(0, 0);
        const double2 w0 = wload(0);
        if (tid < NW * kKC) sw[0][wiw][wpp] = w0;
    }
    for (long c = 0; c < nchunk; c++) {
        const int stg = (int)(c & 1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        double2 wnext = make_double2(0.0, 0.0);
        if (c + 1 < nchunk) {
            issue(stg ^ 1, c + 1);
            wnext = wload(c + 1);
        }
#pragma unroll
        for (int s = 0; s < kKC / 4; s++) {
            const int pp = 4 * s + lk;
            const double2 a0 = sm[stg][0][pp][wr + li], a1 = sm[stg][0][pp][wr + 16 + li];
            const double2 b0 = sm[stg][1][pp][wc + li], b1 = sm[stg][1][pp][wc + 16 + li];
            const double2 av[2] = {a0, a1}, bv[2] = {b0, b1};
#pragma unroll
            for (int iw = 0; iw < NW; iw++) {
                const double2 wv = sw[stg][iw][pp];
                const double2 a[2] = {cmul(av[0], wv), cmul(av[1], wv)};
                // first halves of the four products for all 8 accumulators, then the
                // second halves: dependent matrix-core ops are 8 instructions apart
#pragma unroll
                for (int rb = 0; rb < 2; rb++)
#pragma unroll
                    for (int cb = 0; cb < 2; cb++) {
                        accR[iw][rb][cb] = mfma64(a[rb].x, bv[cb].x, accR[iw][rb][cb]);
                        accI[iw][rb][cb] = mfma64(a[rb].y, bv[cb].x, accI[iw][rb][cb]);
                    }
#pragma unroll
                for (int rb = 0; rb < 2; rb++)
#pragma unroll
                    for (int cb = 0; cb < 2; cb++) {
                        accR[iw][rb][cb] = mfma64(a[rb].y, bv[cb].y, accR[iw][rb][cb]);
                        accI[iw][rb][cb] = mfma64(-a[rb].x, bv[cb].y, accI[iw][rb][cb]);
                    }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // the other stage's weights: its readers finished before this chunk's barrier
        if (c + 1 < nchunk && tid < NW * kKC) sw[stg ^ 1][wiw][wpp] = wnext;
    }

    // result register r of lane (li, lk) holds row lk + 4 r, column li of a 16x16 block
    const bool mirror = herm && rt != ct;
#pragma unroll
    for (int iw = 0; iw < NW; iw++) {
        if (f0 + iw >= nfreq) continue;
        double2 *C = chi + (long)(f0 + iw) * ng * ng;
#pragma unroll
        for (int rb = 0; rb < 2; rb++)
#pragma unroll
            for (int cb = 0; cb < 2; cb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = rt0 + wr + rb * 16 + lk + 4 * r;
                    const int j = ct0 + wc + cb * 16 + li;
                    if (i < ng && j < ng) {
                        const double2 a = make_double2(accR[iw][rb][cb][r], accI[iw][rb][cb][r]);
                        const long idx = (long)i * ng + j;
                        C[idx] = accumulate ? cadd(C[idx], a) : a;
                        if (mirror) {
                            const long jdx = (long)j * ng + i;
                            const double2 b = make_double2(a.x, -a.y);
                            C[jdx] = accumulate ? cadd(C[jdx], b) : b;
                        }
                    }
                }
    }
}

}  // namespace

void launch_chi_f64(hipStream_t s, long npair, int ng, const double2 *M, int nfreq, const double2 *w,
                    int accumulate, bool herm, double2 *chi)
{
    const unsigned t = (unsigned)((ng + kT - 1) / kT);
    const unsigned tiles = herm ? t * (t + 1) / 2 : t * t;
    hipLaunchKernelGGL(k_chi_f64<kNW>, dim3(tiles, 1, (nfreq + kNW - 1) / kNW), dim3(256), 0, s, npair, ng, M,
                       nfreq, w, accumulate, (int)herm, chi);
}

}  // namespace rp
