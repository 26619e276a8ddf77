// Step a6 with split-BF16 operands (Eq. chi, reduced-precision contraction):
//
//   chi_GG'(w) (+)= sum_p a_p(G) conj(b_p(G')),  a = w(w) M (row side), b = M (column side)
//
// Each FP32 value x is written as x ~ x_h + x_m + x_l with three BF16 terms
// (x_h = bf16(x), x_m = bf16(x - x_h), x_l = bf16(x - x_h - x_m); each
// remainder is exact in FP32), and a product x y is formed from the six
// partial products with s + t <= 2 (h=0, m=1, l=2), which keeps it to about
// 2^-24 relative.  The products run on v_mfma_f32_16x16x32_bf16 with FP32
// accumulators; each call's partial sums are added into chi in FP64.
//
// A prep pass converts the FP64 pair densities once per call into
//   Ap: FP32 complex, [KP/8][NGP][8]      (row side, scaled by w in registers)
//   Bp: 6 BF16 planes [6][KP/8][NGP][8]   (column side; re h,m,l then im h,m,l)
// with KP = pairs padded to 32 and NGP = ng padded to 128 (zeros), so that a
// lane's 8 consecutive pairs are one contiguous 64-byte / 16-byte load.
//
// Tiling: a 256-thread block owns a 128x128 tile of (G, G') for NW
// frequencies; each wave a 64x64 sub-tile (4x4 blocks of 16x16).
#include "fft_lds.h"

namespace rp {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;
constexpr int kStep = 32;  // pairs per matrix-core step

__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l)
{
    h = (__bf16)x;
    const float r1 = x - (float)h;
    m = (__bf16)r1;
    const float r2 = r1 - (float)m;
    l = (__bf16)r2;
}

__device__ __forceinline__ bf8 negate(bf8 v)
{
    u4 u = __builtin_bit_cast(u4, v);
    u ^= (u4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    return __builtin_bit_cast(bf8, u);
}

// one thread per (pair group of 8, G)
__global__ void k_split_prep(long npair, int ng, int npg, int NGP, const double2 *__restrict__ M,
                             float2 *__restrict__ Ap, bf8 *__restrict__ Bp)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)npg * NGP) return;
    const int pg = (int)(t / NGP), G = (int)(t - (long)pg * NGP);
    float2 a[8];
    bf8 pl[6];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const long p = (long)pg * 8 + j;
        double2 v = make_double2(0.0, 0.0);
        if (p < npair && G < ng) v = M[p * ng + G];
        const float re = (float)v.x, im = (float)v.y;
        a[j] = make_float2(re, im);
        __bf16 h, m, l;
        split3(re, h, m, l);
        pl[0][j] = h;
        pl[1][j] = m;
        pl[2][j] = l;
        split3(im, h, m, l);
        pl[3][j] = h;
        pl[4][j] = m;
        pl[5][j] = l;
    }
    float2 *ao = Ap + t * 8;
#pragma unroll
    for (int j = 0; j < 8; j++) ao[j] = a[j];
    const long plane = (long)npg * NGP;
#pragma unroll
    for (int s = 0; s < 6; s++) Bp[s * plane + t] = pl[s];
}

template <int NW>
__global__ void __launch_bounds__(256)
k_chi_bf16(int npg, int NGP, long npair, int ng, const float2 *__restrict__ Ap, const bf8 *__restrict__ Bp,
           int nfreq, const double2 *__restrict__ w, int accumulate, double2 *__restrict__ chi)
{
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int row0 = blockIdx.y * kTile + (wave >> 1) * 64;
    const int col0 = blockIdx.x * kTile + (wave & 1) * 64;
    const int f0 = blockIdx.z * NW;
    const long plane = (long)npg * NGP;

    f4 accR[NW][4][4], accI[NW][4][4];
#pragma unroll
    for (int iw = 0; iw < NW; iw++)
#pragma unroll
        for (int rb = 0; rb < 4; rb++)
#pragma unroll
            for (int cb = 0; cb < 4; cb++) {
                accR[iw][rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
                accI[iw][rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
            }

    for (int kg0 = 0; kg0 < npg; kg0 += kStep / 8) {
        const int kg = kg0 + lk;
        // column operand: 4 blocks x 6 planes
        bf8 B[4][6];
#pragma unroll
        for (int cb = 0; cb < 4; cb++)
#pragma unroll
            for (int s = 0; s < 6; s++) B[cb][s] = Bp[s * plane + (long)kg * NGP + col0 + cb * 16 + li];
        // weights of this lane's 8 pairs
        float2 wf[NW][8];
#pragma unroll
        for (int iw = 0; iw < NW; iw++)
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const long p = (long)kg * 8 + j;
                double2 v = make_double2(0.0, 0.0);
                if (p < npair && f0 + iw < nfreq) v = w[(long)(f0 + iw) * npair + p];
                wf[iw][j] = make_float2((float)v.x, (float)v.y);
            }
#pragma unroll
        for (int rb = 0; rb < 4; rb++) {
            const float2 *src = Ap + ((long)kg * NGP + row0 + rb * 16 + li) * 8;
            float2 araw[8];
#pragma unroll
            for (int j = 0; j < 8; j++) araw[j] = src[j];
#pragma unroll
            for (int iw = 0; iw < NW; iw++) {
                bf8 rh, rm, rl, ih, im, il;
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const float2 x = araw[j], y = wf[iw][j];
                    const float re = x.x * y.x - x.y * y.y;
                    const float imv = x.x * y.y + x.y * y.x;
                    __bf16 h, m, l;
                    split3(re, h, m, l);
                    rh[j] = h;
                    rm[j] = m;
                    rl[j] = l;
                    split3(imv, h, m, l);
                    ih[j] = h;
                    im[j] = m;
                    il[j] = l;
                }
#pragma unroll
                for (int cb = 0; cb < 4; cb++) {
                    f4 cr = accR[iw][rb][cb], ci = accI[iw][rb][cb];
                    // Re += Re a Re b + Im a Im b   (terms with s + t <= 2)
                    cr = mfma_bf16(rh, B[cb][0], cr);
                    cr = mfma_bf16(rh, B[cb][1], cr);
                    cr = mfma_bf16(rm, B[cb][0], cr);
                    cr = mfma_bf16(rh, B[cb][2], cr);
                    cr = mfma_bf16(rm, B[cb][1], cr);
                    cr = mfma_bf16(rl, B[cb][0], cr);
                    cr = mfma_bf16(ih, B[cb][3], cr);
                    cr = mfma_bf16(ih, B[cb][4], cr);
                    cr = mfma_bf16(im, B[cb][3], cr);
                    cr = mfma_bf16(ih, B[cb][5], cr);
                    cr = mfma_bf16(im, B[cb][4], cr);
                    cr = mfma_bf16(il, B[cb][3], cr);
                    // Im += Im a Re b - Re a Im b
                    ci = mfma_bf16(ih, B[cb][0], ci);
                    ci = mfma_bf16(ih, B[cb][1], ci);
                    ci = mfma_bf16(im, B[cb][0], ci);
                    ci = mfma_bf16(ih, B[cb][2], ci);
                    ci = mfma_bf16(im, B[cb][1], ci);
                    ci = mfma_bf16(il, B[cb][0], ci);
                    accR[iw][rb][cb] = cr;
                    accI[iw][rb][cb] = ci;
                }
                const bf8 nh = negate(rh), nm = negate(rm), nl = negate(rl);
#pragma unroll
                for (int cb = 0; cb < 4; cb++) {
                    f4 ci = accI[iw][rb][cb];
                    ci = mfma_bf16(nh, B[cb][3], ci);
                    ci = mfma_bf16(nh, B[cb][4], ci);
                    ci = mfma_bf16(nm, B[cb][3], ci);
                    ci = mfma_bf16(nh, B[cb][5], ci);
                    ci = mfma_bf16(nm, B[cb][4], ci);
                    ci = mfma_bf16(nl, B[cb][3], ci);
                    accI[iw][rb][cb] = ci;
                }
            }
        }
    }

    // result register r of lane (li, lk) holds row 4 lk + r, column li of a 16x16 block
#pragma unroll
    for (int iw = 0; iw < NW; iw++) {
        if (f0 + iw >= nfreq) continue;
        double2 *C = chi + (long)(f0 + iw) * ng * ng;
#pragma unroll
        for (int rb = 0; rb < 4; rb++)
#pragma unroll
            for (int cb = 0; cb < 4; cb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = row0 + rb * 16 + 4 * lk + r;
                    const int j = col0 + cb * 16 + li;
                    if (i < ng && j < ng) {
                        double2 v = make_double2((double)accR[iw][rb][cb][r], (double)accI[iw][rb][cb][r]);
                        const long idx = (long)i * ng + j;
                        if (accumulate) v = cadd(C[idx], v);
                        C[idx] = v;
                    }
                }
    }
}

long pad_pairs(long npair) { return (npair + kStep - 1) / kStep * kStep; }
int pad_ng(int ng) { return (ng + kTile - 1) / kTile * kTile; }

}  // namespace

size_t split_a_bytes(long npair, int ng) { return (size_t)pad_pairs(npair) * pad_ng(ng) * sizeof(float2); }
size_t split_b_bytes(long npair, int ng) { return (size_t)6 * pad_pairs(npair) * pad_ng(ng) * 2; }

void launch_split_prep(hipStream_t s, long npair, int ng, const double2 *M, void *split_a, void *split_b)
{
    const long KP = pad_pairs(npair);
    const int NGP = pad_ng(ng);
    const int npg = (int)(KP / 8);
    const long nt = (long)npg * NGP;
    if (nt > 0)
        hipLaunchKernelGGL(k_split_prep, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, npair, ng, npg,
                           NGP, M, (float2 *)split_a, (bf8 *)split_b);
}

void launch_chi_bf16(hipStream_t s, long npair, int ng, int nfreq, const double2 *w, int accumulate,
                     double2 *chi, const void *split_a, const void *split_b)
{
    const long KP = pad_pairs(npair);
    const int NGP = pad_ng(ng);
    const int npg = (int)(KP / 8);
    const float2 *Ap = (const float2 *)split_a;
    const bf8 *Bp = (const bf8 *)split_b;
    const unsigned t = (unsigned)(NGP / kTile);
    if (nfreq >= 2)
        hipLaunchKernelGGL(k_chi_bf16<2>, dim3(t, t, (nfreq + 1) / 2), dim3(256), 0, s, npg, NGP, npair, ng,
                           Ap, Bp, nfreq, w, accumulate, chi);
    else
        hipLaunchKernelGGL(k_chi_bf16<1>, dim3(t, t, nfreq), dim3(256), 0, s, npg, NGP, npair, ng, Ap, Bp,
                           nfreq, w, accumulate, chi);
}

}  // namespace rp
