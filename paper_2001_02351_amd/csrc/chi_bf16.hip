// Step a6 with split-BF16 operands (Eq. chi, reduced-precision contraction):
//
//   chi_GG'(w) (+)= sum_p a_p(G) conj(b_p(G')),  a = w(w) M (row side), b = M (column side)
//
// Each FP32 value x is written as a sum of NT BF16 terms x_0 + x_1 (+ x_2),
// x_0 = bf16(x), x_1 = bf16(x - x_0), x_2 = bf16(x - x_0 - x_1) (each
// remainder is exact in FP32), and a product x y is formed from the partial
// products x_s y_t with s + t < NT:
//   NT = 2: x_0 y_0 + x_0 y_1 + x_1 y_0   (three-term compensated product,
//           relative error about 3 2^-16 per product)
//   NT = 3: the six terms with s + t <= 2  (about 2^-24, i.e. FP32)
// The products run on v_mfma_f32_16x16x32_bf16 with FP32 accumulators; each
// call's partial sums are added into chi in FP64.
//
// The operands (layout in split_ops.h) are the FP32 row blocks Ap (scaled by
// w and split in registers), the 2 NT BF16 column planes Bp and the FP32
// weights Wq [nfreq][KP], with KP = pairs padded to 32 and NGP = ng padded to
// 128 (zeros).  The FP32 pair kernels write Ap and Bp directly; k_split_prep
// makes them from FP64 M for callers that hold M.
//
// Tiling (row form, k_chi_rows, the default for two frequencies per block): a
// 256-thread block owns a 128x128 tile of (G, G') for 2 frequencies; wave w
// holds rows 64 (w / 2) .. + 63 and all 128 columns for frequency w % 2 (4 x 8
// blocks of 16x16), so each weighted row operand is split by one wave only.
// With a multiple of four frequencies the same form runs as 64-row strips x
// 128 columns for 4 frequencies (a Hermitian chi with a multiple of eight: as
// 32-row strips x 128 columns for 8): the same work per wave, a half or a
// quarter of the row operand per workgroup and the column operand shared by
// four or eight frequencies; for a Hermitian chi each strip's column tiles
// start at its own diagonal.  k_chi_bf16 (one frequency per
// block, four 64x64 sub-tiles) and the eight-wave 256-row forms are the tuning
// alternatives.  Steps of 32 pairs
// stream through two LDS buffers (32 KB of A and 16 NT KB of B each) by
// global_load_lds DMA, so the next step's operands arrive while the matrix
// cores work on the current one.
#include <algorithm>

#include "fft_lds.h"
#include "split_ops.h"

namespace rp {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;
constexpr int kStep = 32;  // pairs per matrix-core step
// The FP32 accumulators of one block sum at most kFlush steps of 32 pairs
// (16 384 pairs): a longer contraction is cut into slices of the pair steps
// whose FP32 partial tiles are summed in FP64, so the accumulation error does
// not grow with the pairs per launch.
constexpr int kFlush = 512;

__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 negate(bf8 v)
{
    u4 u = __builtin_bit_cast(u4, v);
    u ^= (u4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    return __builtin_bit_cast(bf8, u);
}

__device__ __forceinline__ void dma16(const void *src, void *lds)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

// one thread per (pair group of 8, G)
template <int NT>
__global__ void k_split_prep(long npair, int ng, int npg, int NGP, const double2 *__restrict__ M,
                             float2 *__restrict__ Ap, bf8 *__restrict__ Bp)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)npg * NGP) return;
    const int pg = (int)(t / NGP), G = (int)(t - (long)pg * NGP);
    float2 a[8];
    bf8 pl[2 * NT];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const long p = (long)pg * 8 + j;
        double2 v = make_double2(0.0, 0.0);
        if (p < npair && G < ng) v = M[p * ng + G];
        const float re = (float)v.x, im = (float)v.y;
        a[j] = make_float2(re, im);
        __bf16 tr[NT], ti[NT];
        split<NT>(re, tr);
        split<NT>(im, ti);
#pragma unroll
        for (int s = 0; s < NT; s++) {
            pl[s][j] = tr[s];
            pl[NT + s][j] = ti[s];
        }
    }
    float2 *blk = Ap + ((long)pg * (NGP / 16) + G / 16) * 128 + (G % 16) * 2;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        blk[q * 32] = a[2 * q];
        blk[q * 32 + 1] = a[2 * q + 1];
    }
    const long plane = (long)npg * NGP;
#pragma unroll
    for (int s = 0; s < 2 * NT; s++) Bp[s * plane + t] = pl[s];
}

// zeros into the padding slots of the operands: the first nrow threads take
// (pair group, padding row), the rest (pair group holding padding pairs, row)
__global__ void k_ops_pad(SplitOps o, long npair, int ng, long nrow, long ntot)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntot) return;
    long pg;
    int g, j0;
    if (t < nrow) {
        const int pad = o.NGP - ng;
        pg = t / pad;
        g = ng + (int)(t - pg * pad);
        j0 = 0;
    } else {
        const long u = t - nrow;
        pg = npair / 8 + u / ng;
        g = (int)(u - (u / ng) * ng);
        j0 = (int)max(0L, npair - pg * 8);
    }
    for (int j = j0; j < 8; j++) ops_store(o, pg * 8 + j, g, 0.f, 0.f);
}

// real_w: the weights are real (imaginary frequencies, no broadening) and
// their imaginary parts, rounding residue only, are dropped
__global__ void k_weight_prep(long npair, long KP, int nfreq, const double2 *__restrict__ w, int real_w,
                              float2 *__restrict__ wq)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= KP * nfreq) return;
    const int f = (int)(t / KP);
    const long p = t - (long)f * KP;
    double2 v = make_double2(0.0, 0.0);
    if (p < npair) v = w[(long)f * npair + p];
    wq[t] = make_float2((float)v.x, real_w ? 0.f : (float)v.y);
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

// Strip tiling of a Hermitian chi (the upper triangle G <= G'): strips of h
// rows (h = 64 or 32), r = 0 .. ceil(ng / h) - 1, whose 128-column tiles start
// at the strip's own first row, columns h r + 128 j, j < ceil((ng - h r) /
// 128).  Only the lower half of each strip's leading h x h block and the
// columns past ng are formed without being needed, where 128 x 128 tiles of
// the upper triangle also form the lower half of every diagonal tile and the
// padding up to the next multiple of 128.
__host__ __device__ __forceinline__ int strip_tiles(int ng, int h, int r) { return (ng - h * r + kTile - 1) / kTile; }

__host__ __device__ inline long strip_tiles_total(int ng, int h)
{
    long n = 0;
    for (int r = 0; r * h < ng; r++) n += strip_tiles(ng, h, r);
    return n;
}

// strip r and column tile j of block index id
__device__ __forceinline__ void strip_tile_of(int id, int ng, int h, int &r, int &j)
{
    r = 0;
    for (int m = strip_tiles(ng, h, 0); id >= m; m = strip_tiles(ng, h, r)) {
        id -= m;
        r++;
    }
    j = id;
}

// Grid: x = tile (all t x t tiles, or the upper triangle when herm), y =
// frequency group, z = slice of the pair steps (sps steps each).  With one slice the
// block adds its tile into chi (and, for an off-diagonal tile of a Hermitian
// chi, the conjugate transpose into the mirrored tile); with several slices
// it writes its FP32 partial tile to part[slice][f][NGP][NGP] for k_chi_reduce.
//
// Tail split (stail > 0): the grid is one-dimensional over the units (tile,
// frequency group), unit = group * tiles + tile.  The first nfull units (whole
// waves of the chip) run whole; each of the remaining units runs as stail
// slices of sps pair steps, which write FP32 partial tiles
// part[(unit - nfull) * stail + slice][NW][128][128] for k_chi_reduce_tail, so
// that the last wave's work is spread over every compute unit.
template <int NT, int NW>
__global__ void __launch_bounds__(256)
k_chi_bf16(int npg, int NGP, long KP, int ng, const float2 *__restrict__ Ap, const bf8 *__restrict__ Bp,
           int nfreq, const float2 *__restrict__ wq, int accumulate, double2 *__restrict__ chi, int herm,
           int sps, float2 *__restrict__ part, int nfull, int stail)
{
    constexpr int NPL = 2 * NT;  // B planes
    // per stage: A [4 kg][8 row blocks][4 q][16][2] float2 (32 KB) and
    //            B [NPL planes][4 kg][128 cols] bf8 (8 NPL KB)
    __shared__ float2 sA[2][4 * 8 * 128];
    __shared__ bf8 sB[2][NPL * 4 * 128];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = NGP / kTile;
    const int ntiles = herm ? nt * (nt + 1) / 2 : nt * nt;
    // grid: x = tile, y = frequency group, z = slice of the pair steps (slowest,
    // so that the blocks in flight share one slice's operands)
    int tile = blockIdx.x, group = blockIdx.y, step0 = blockIdx.z * sps, nstep;
    float2 *tailp = nullptr;          // tail split: this slice's partial tile
    if (stail > 0) {
        const int b = blockIdx.x;
        int unit = b;
        step0 = 0;
        nstep = npg / 4;
        if (b >= nfull) {
            const int t = b - nfull;
            unit = nfull + t / stail;
            step0 = (t % stail) * sps;
            nstep = max(0, min(sps, npg / 4 - step0));
            tailp = part + (long)t * NW * kTile * kTile;
        }
        tile = unit % ntiles;
        group = unit / ntiles;
    } else {
        nstep = min(sps, npg / 4 - step0);
    }
    int rt, ct;
    tile_of(tile, nt, herm, rt, ct);
    const int rt0 = rt * kTile, ct0 = ct * kTile;
    const int wr = wave >> 1, wc = wave & 1;
    const int f0 = group * NW;
    const long plane = (long)npg * NGP;

    // DMA segments of 1 KB; wave w moves pair group kg = w: its 8 A row
    // blocks and its NPL x 2 B half-rows
    const float2 *srcA = Ap + ((long)wave * (NGP / 16) + rt0 / 16) * 128 + lane * 2;
    const bf8 *srcB = Bp + (long)wave * NGP + ct0 + lane;
    auto issue = [&](float2 *dA, bf8 *dB, int kg0) {
        const float2 *a = srcA + (long)kg0 * (NGP / 16) * 128;
        float2 *da = dA + wave * 8 * 128;
#pragma unroll
        for (int rb = 0; rb < 8; rb++) dma16(a + rb * 128, da + rb * 128);
        const bf8 *b = srcB + (long)kg0 * NGP;
#pragma unroll
        for (int sp = 0; sp < NPL; sp++)
#pragma unroll
            for (int h = 0; h < 2; h++) dma16(b + sp * plane + 64 * h, dB + (sp * 4 + wave) * 128 + 64 * h);
    };
    auto wload = [&](int step, float2 (&dst)[NW][8]) {
#pragma unroll
        for (int iw = 0; iw < NW; iw++) {
            const int f = min(f0 + iw, nfreq - 1);
            const float4 *src = (const float4 *)(wq + (long)f * KP + (long)(step * 4 + lk) * 8);
#pragma unroll
            for (int h = 0; h < 4; h++) {
                const float4 v = src[h];
                dst[iw][2 * h] = make_float2(v.x, v.y);
                dst[iw][2 * h + 1] = make_float2(v.z, v.w);
            }
        }
    };

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

    // One step: issue the DMA of the next step into the other stage and
    // compute the current one.  The stage pointers are restrict-qualified
    // parameters, so the compiler knows that the current stage's LDS reads do
    // not touch what the DMA writes and leaves the DMA in flight during the
    // matrix-core work (with plain indexing of one array it would wait for
    // the DMA before the first LDS read).
    auto step = [&](float2 *__restrict__ nA, bf8 *__restrict__ nB, const float2 *__restrict__ cA,
                    const bf8 *__restrict__ cB, int kgn, const float2 (&wcur)[NW][8]) {
        if (kgn >= 0) issue(nA, nB, kgn);
        // column operand: 4 blocks x NPL planes
        bf8 B[4][NPL];
#pragma unroll
        for (int cb = 0; cb < 4; cb++)
#pragma unroll
            for (int sp = 0; sp < NPL; sp++) B[cb][sp] = cB[(sp * 4 + lk) * 128 + wc * 64 + cb * 16 + li];
#pragma unroll
        for (int rb = 0; rb < 4; rb++) {
            const float2 *blk = cA + (lk * 8 + wr * 4 + rb) * 128 + li * 2;
            float2 araw[8];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 v = *(const float4 *)(blk + q * 32);
                araw[2 * q] = make_float2(v.x, v.y);
                araw[2 * q + 1] = make_float2(v.z, v.w);
            }
#pragma unroll
            for (int iw = 0; iw < NW; iw++) {
                bf8 ar[NT], ai[NT], an[NT];
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const float2 x = araw[j], y = wcur[iw][j];
                    __bf16 tr[NT], ti[NT];
                    split<NT>(x.x * y.x - x.y * y.y, tr);
                    split<NT>(x.x * y.y + x.y * y.x, ti);
#pragma unroll
                    for (int s = 0; s < NT; s++) {
                        ar[s][j] = tr[s];
                        ai[s][j] = ti[s];
                    }
                }
#pragma unroll
                for (int s = 0; s < NT; s++) an[s] = negate(ar[s]);
                // Re += Re a Re b + Im a Im b;  Im += Im a Re b - Re a Im b, over
                // the products s + t < NT; the column block is the innermost index
                // so consecutive matrix-core ops update 8 independent accumulators
                f4 cr[4], ci[4];
#pragma unroll
                for (int cb = 0; cb < 4; cb++) {
                    cr[cb] = accR[iw][rb][cb];
                    ci[cb] = accI[iw][rb][cb];
                }
#pragma unroll
                for (int s = 0; s < NT; s++)
#pragma unroll
                    for (int u = 0; u < NT; u++) {
                        if (s + u >= NT) continue;
#pragma unroll
                        for (int cb = 0; cb < 4; cb++) {
                            cr[cb] = mfma_bf16(ar[s], B[cb][u], cr[cb]);
                            ci[cb] = mfma_bf16(ai[s], B[cb][u], ci[cb]);
                        }
                    }
#pragma unroll
                for (int s = 0; s < NT; s++)
#pragma unroll
                    for (int u = 0; u < NT; u++) {
                        if (s + u >= NT) continue;
#pragma unroll
                        for (int cb = 0; cb < 4; cb++) {
                            cr[cb] = mfma_bf16(ai[s], B[cb][NT + u], cr[cb]);
                            ci[cb] = mfma_bf16(an[s], B[cb][NT + u], ci[cb]);
                        }
                    }
#pragma unroll
                for (int cb = 0; cb < 4; cb++) {
                    accR[iw][rb][cb] = cr[cb];
                    accI[iw][rb][cb] = ci[cb];
                }
            }
        }
    };

    // The weights of step t+1 are loaded into registers before the DMA of
    // step t+1 is issued: they are waited for at the top of the next step,
    // together with that DMA, so no wait inside a step covers the DMA.
    float2 wcur[NW][8], wnext[NW][8];
    if (nstep > 0) {
        wload(step0, wnext);
        issue(sA[0], sB[0], 4 * step0);
    }
    for (int t = 0; t < nstep; t++) {
        const int stg = t & 1;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int iw = 0; iw < NW; iw++)
#pragma unroll
            for (int j = 0; j < 8; j++) wcur[iw][j] = wnext[iw][j];
        const bool more = t + 1 < nstep;
        if (more) wload(step0 + t + 1, wnext);
        step(sA[stg ^ 1], sB[stg ^ 1], sA[stg], sB[stg], more ? 4 * (step0 + t + 1) : -1, wcur);
    }

    // result register r of lane (li, lk) holds row 4 lk + r, column li of a 16x16 block
    if (tailp) {
#pragma unroll
        for (int iw = 0; iw < NW; iw++)
#pragma unroll
            for (int rb = 0; rb < 4; rb++)
#pragma unroll
                for (int cb = 0; cb < 4; cb++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int i = wr * 64 + rb * 16 + 4 * lk + r;
                        const int j = wc * 64 + cb * 16 + li;
                        tailp[((long)iw * kTile + i) * kTile + j] =
                            make_float2(accR[iw][rb][cb][r], accI[iw][rb][cb][r]);
                    }
        return;
    }
    if (part && stail == 0) {
#pragma unroll
        for (int iw = 0; iw < NW; iw++) {
            if (f0 + iw >= nfreq) continue;
            float2 *P = part + ((long)blockIdx.z * nfreq + f0 + iw) * NGP * NGP;
#pragma unroll
            for (int rb = 0; rb < 4; rb++)
#pragma unroll
                for (int cb = 0; cb < 4; cb++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int i = rt0 + wr * 64 + rb * 16 + 4 * lk + r;
                        const int j = ct0 + wc * 64 + cb * 16 + li;
                        P[(long)i * NGP + j] = make_float2(accR[iw][rb][cb][r], accI[iw][rb][cb][r]);
                    }
        }
        return;
    }
    const bool mirror = herm && rt != ct;
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
                    const int i = rt0 + wr * 64 + rb * 16 + 4 * lk + r;
                    const int j = ct0 + wc * 64 + cb * 16 + li;
                    if (i < ng && j < ng) {
                        const double2 a = make_double2((double)accR[iw][rb][cb][r], (double)accI[iw][rb][cb][r]);
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

// Row form of the 128 x 128 tile (the default for two frequencies per
// block): wave w owns rows 64 (w / 2) .. 64 (w / 2) + 63 of the tile and all
// 128 columns for frequency f0 + w % 2, so every (row, pair, frequency) of
// the row operand is weighted and split by exactly one wave of the block,
// and each split row block feeds 8 column blocks x 12 matrix-core ops.  The
// split is done two values at a time (packed BF16 conversion, the hi terms
// widened back to FP32 by shifts), so a 16-row x 32-pair block of the row
// operand costs 88 vector instructions (2 NT = 4: weighting 32, split 48,
// negation 8) for its 96 matrix-core ops.  Operand layouts, the two DMA
// stages, the grid (tiles, frequency groups, slices, tail split) and the
// outputs are those of k_chi_bf16 with NW = 2.  RW: real weights (their
// imaginary parts are zero), weighting by two products instead of four.
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef __bf16 bh2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned pk_bf16(float a, float b)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector((fl2){a, b}, bh2));
}

// two FP32 values -> NT packed words of BF16 terms (hi, mid[, lo]); every
// remainder is exact in FP32
template <int NT> __device__ __forceinline__ void split_pair(float x0, float x1, unsigned (&t)[NT])
{
#pragma unroll
    for (int s = 0; s < NT; s++) {
        t[s] = pk_bf16(x0, x1);
        if (s + 1 < NT) {
            x0 -= __uint_as_float(t[s] << 16);
            x1 -= __uint_as_float(t[s] & 0xffff0000u);
        }
    }
}

// SM, the strip tiling (stail = 0): SM = 4, a block owns a 64-row strip x 128
// columns for 4 frequencies, wave w the strip for frequency f0 + w; SM = 8, a
// 32-row strip x 128 columns for 8 frequencies, wave w the strip for
// frequencies f0 + 2 w and f0 + 2 w + 1.  Either way every wave forms four
// (16-row block, frequency) combinations x 128 columns, the same work as in
// the 128 x 128 form (SM = 0); grid x runs over the strip tiles of the upper
// triangle (herm) or over all NGP / h x t strip tiles (row-major).
template <int NT, bool RW, int SM>
__global__ void __launch_bounds__(256)
k_chi_rows(int npg, int NGP, long KP, int ng, const float2 *__restrict__ Ap, const bf8 *__restrict__ Bp, int nfreq,
           const float2 *__restrict__ wq, int accumulate, double2 *__restrict__ chi, int herm, int sps,
           float2 *__restrict__ part, int nfull, int stail)
{
    constexpr bool ST = SM != 0;
    constexpr int NW = ST ? SM : 2;           // frequencies per block
    constexpr int WW = SM == 8 ? 2 : 1;       // frequencies per wave
    constexpr int SH = SM == 8 ? 32 : 64;     // strip height
    constexpr int NRB = ST ? SH / 16 : 8;     // 16-row blocks of the block's rows
    // combination c of a wave: 16-row block crb(c) of its rows, its frequency cw(c)
    auto crb = [](int c) { return WW == 2 ? (c & 1) : c; };
    auto cw = [](int c) { return WW == 2 ? (c >> 1) : 0; };
    constexpr int NPL = 2 * NT;
    __shared__ float2 sA[2][4 * 8 * 128];
    __shared__ bf8 sB[2][NPL * 4 * 128];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = NGP / kTile;
    const int ntiles = herm ? nt * (nt + 1) / 2 : nt * nt;
    int tile = blockIdx.x, group = blockIdx.y, step0 = blockIdx.z * sps, nstep;
    float2 *tailp = nullptr;
    if (stail > 0) {
        const int b = blockIdx.x;
        int unit = b;
        step0 = 0;
        nstep = npg / 4;
        if (b >= nfull) {
            const int t = b - nfull;
            unit = nfull + t / stail;
            step0 = (t % stail) * sps;
            nstep = max(0, min(sps, npg / 4 - step0));
            tailp = part + (long)t * NW * kTile * kTile;
        }
        tile = unit % ntiles;
        group = unit / ntiles;
    } else {
        nstep = min(sps, npg / 4 - step0);
    }
    int rt, ct, rt0, ct0;
    if constexpr (ST) {
        if (herm) {
            strip_tile_of(tile, ng, SH, rt, ct);
            rt0 = rt * SH;
            ct0 = rt0 + ct * kTile;
        } else {
            rt = tile / nt;
            ct = tile - rt * nt;
            rt0 = rt * SH;
            ct0 = ct * kTile;
        }
    } else {
        tile_of(tile, nt, herm, rt, ct);
        rt0 = rt * kTile;
        ct0 = ct * kTile;
    }
    const int wr = ST ? 0 : wave >> 1, iw = ST ? wave : wave & 1;
    const int f0 = group * NW;
    const int fv = f0 + WW * iw;              // the wave's first frequency
    const long plane = (long)npg * NGP;

    // DMA as in k_chi_bf16: wave w moves pair group kg = w of the step.  A
    // strip tile's columns can run past NGP: those lanes read column NGP - 1
    // (their results are never stored).
    const float2 *srcA = Ap + ((long)wave * (NGP / 16) + rt0 / 16) * 128 + lane * 2;
    const bf8 *srcB = Bp + (long)wave * NGP + (ST ? min(ct0 + lane, NGP - 1) : ct0 + lane);
    const bf8 *srcB1 = ST ? Bp + (long)wave * NGP + min(ct0 + 64 + lane, NGP - 1) : srcB + 64;
    auto issue = [&](float2 *dA, bf8 *dB, int kg0) {
        const float2 *a = srcA + (long)kg0 * (NGP / 16) * 128;
        float2 *da = dA + wave * 8 * 128;
#pragma unroll
        for (int rb = 0; rb < NRB; rb++) dma16(a + rb * 128, da + rb * 128);
        const bf8 *b0 = srcB + (long)kg0 * NGP, *b1 = srcB1 + (long)kg0 * NGP;
#pragma unroll
        for (int sp = 0; sp < NPL; sp++) {
            dma16(b0 + sp * plane, dB + (sp * 4 + wave) * 128);
            dma16(b1 + sp * plane, dB + (sp * 4 + wave) * 128 + 64);
        }
    };
    // this lane's 8 pairs (8 lk .. 8 lk + 7 of the step) at the wave's frequencies
    const float4 *wsrc[WW];
#pragma unroll
    for (int v = 0; v < WW; v++) wsrc[v] = (const float4 *)(wq + (long)min(fv + v, nfreq - 1) * KP) + lk * 4;
    auto wload = [&](int step, float4 (&dst)[WW][4]) {
#pragma unroll
        for (int v = 0; v < WW; v++)
#pragma unroll
            for (int h = 0; h < 4; h++) dst[v][h] = wsrc[v][(long)step * 16 + h];
    };

    f4 accR[4][8], accI[4][8];
#pragma unroll
    for (int rb = 0; rb < 4; rb++)
#pragma unroll
        for (int cb = 0; cb < 8; cb++) {
            accR[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
            accI[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
        }

    // the weighted, split row operand of row block rb of the wave
    auto split_rows = [&](const float2 *__restrict__ cA, int rb, const float4 (&wc)[4], bf8 (&ar)[NT],
                          bf8 (&ai)[NT], bf8 (&an)[NT]) {
        const float2 *blk = cA + (lk * 8 + wr * 4 + rb) * 128 + li * 2;
        u4 wr_[NT], wi_[NT];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float4 v = *(const float4 *)(blk + q * 32);   // pairs 2q, 2q+1: (re, im, re, im)
            const float4 w = wc[q];
            float r0, i0, r1, i1;
            if (RW) {
                r0 = v.x * w.x;
                i0 = v.y * w.x;
                r1 = v.z * w.z;
                i1 = v.w * w.z;
            } else {
                r0 = v.x * w.x - v.y * w.y;
                i0 = v.x * w.y + v.y * w.x;
                r1 = v.z * w.z - v.w * w.w;
                i1 = v.z * w.w + v.w * w.z;
            }
            unsigned tr[NT], ti[NT];
            split_pair<NT>(r0, r1, tr);
            split_pair<NT>(i0, i1, ti);
#pragma unroll
            for (int s = 0; s < NT; s++) {
                wr_[s][q] = tr[s];
                wi_[s][q] = ti[s];
            }
        }
#pragma unroll
        for (int s = 0; s < NT; s++) {
            ar[s] = __builtin_bit_cast(bf8, wr_[s]);
            ai[s] = __builtin_bit_cast(bf8, wi_[s]);
            an[s] = negate(ar[s]);
        }
    };
    // Re += Re a Re b + Im a Im b;  Im += Im a Re b - Re a Im b over the
    // products s + u < NT, for row block rb and column block cb
    auto products = [&](int rb, int cb, const bf8 (&ar)[NT], const bf8 (&ai)[NT], const bf8 (&an)[NT],
                        const bf8 (&B)[NPL]) {
#pragma unroll
        for (int s = 0; s < NT; s++)
#pragma unroll
            for (int u = 0; u < NT; u++) {
                if (s + u >= NT) continue;
                accR[rb][cb] = mfma_bf16(ar[s], B[u], accR[rb][cb]);
                accI[rb][cb] = mfma_bf16(ai[s], B[u], accI[rb][cb]);
                accR[rb][cb] = mfma_bf16(ai[s], B[NT + u], accR[rb][cb]);
                accI[rb][cb] = mfma_bf16(an[s], B[NT + u], accI[rb][cb]);
            }
    };
    constexpr int NPROD = 4 * NT * (NT + 1) / 2;   // matrix-core ops per (row block, column block)

    auto step = [&](float2 *__restrict__ nA, bf8 *__restrict__ nB, const float2 *__restrict__ cA,
                    const bf8 *__restrict__ cB, int kgn, const float4 (&wc)[WW][4]) {
        if (kgn >= 0) issue(nA, nB, kgn);
        bf8 ar[4][NT], ai[4][NT], an[4][NT];
        bf8 B[NPL], Bn[NPL];   // this column block's fragments and the next one's
#pragma unroll
        for (int sp = 0; sp < NPL; sp++) B[sp] = cB[(sp * 4 + lk) * 128 + li];
        split_rows(cA, crb(0), wc[cw(0)], ar[0], ai[0], an[0]);
        __builtin_amdgcn_sched_barrier(0);
        // column block 0, one row block after the other: the split of row
        // block rb + 1 is issued among the matrix-core ops of row block rb,
        // and column block 1's fragments are read during row block 3's
#pragma unroll
        for (int rb = 0; rb < 4; rb++) {
            products(rb, 0, ar[rb], ai[rb], an[rb], B);
            if (rb + 1 < 4) {
                split_rows(cA, crb(rb + 1), wc[cw(rb + 1)], ar[rb + 1], ai[rb + 1], an[rb + 1]);
                __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);       // the row block's LDS reads
#pragma unroll
                for (int i = 0; i < NPROD; i++) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one matrix-core op
                    __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);   // then vector instructions
                }
            } else {
#pragma unroll
                for (int sp = 0; sp < NPL; sp++) Bn[sp] = cB[(sp * 4 + lk) * 128 + 16 + li];
                // one matrix-core op (after the wait for this block's data),
                // then the next fragments' reads, then the other ops
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, NPL, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NPROD - 1, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // the other column blocks: 8 independent accumulators per product;
        // the next column block's fragments are read ahead of each block's
        // matrix-core ops, so their LDS latency is covered by those ops
#pragma unroll
        for (int cb = 1; cb < 8; cb++) {
#pragma unroll
            for (int sp = 0; sp < NPL; sp++) B[sp] = Bn[sp];
            if (cb + 1 < 8) {
#pragma unroll
                for (int sp = 0; sp < NPL; sp++) Bn[sp] = cB[(sp * 4 + lk) * 128 + (cb + 1) * 16 + li];
            }
#pragma unroll
            for (int s = 0; s < NT; s++)
#pragma unroll
                for (int u = 0; u < NT; u++) {
                    if (s + u >= NT) continue;
#pragma unroll
                    for (int rb = 0; rb < 4; rb++) {
                        accR[rb][cb] = mfma_bf16(ar[rb][s], B[u], accR[rb][cb]);
                        accI[rb][cb] = mfma_bf16(ai[rb][s], B[u], accI[rb][cb]);
                    }
#pragma unroll
                    for (int rb = 0; rb < 4; rb++) {
                        accR[rb][cb] = mfma_bf16(ai[rb][s], B[NT + u], accR[rb][cb]);
                        accI[rb][cb] = mfma_bf16(an[rb][s], B[NT + u], accI[rb][cb]);
                    }
                }
            if (cb + 1 < 8) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, NPL, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 4 * NPROD - 1, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    float4 wcur[WW][4], wnext[WW][4];
    if (nstep > 0) {
        wload(step0, wnext);
        issue(sA[0], sB[0], 4 * step0);
    }
    for (int t = 0; t < nstep; t++) {
        const int stg = t & 1;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int v = 0; v < WW; v++)
#pragma unroll
            for (int h = 0; h < 4; h++) wcur[v][h] = wnext[v][h];
        const bool more = t + 1 < nstep;
        if (more) wload(step0 + t + 1, wnext);
        step(sA[stg ^ 1], sB[stg ^ 1], sA[stg], sB[stg], more ? 4 * (step0 + t + 1) : -1, wcur);
    }

    // result register r of lane (li, lk) holds row 4 lk + r, column li of a 16x16 block
    if (tailp) {
#pragma unroll
        for (int rb = 0; rb < 4; rb++)
#pragma unroll
            for (int cb = 0; cb < 8; cb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = wr * 64 + rb * 16 + 4 * lk + r;
                    const int j = cb * 16 + li;
                    tailp[((long)iw * kTile + i) * kTile + j] = make_float2(accR[rb][cb][r], accI[rb][cb][r]);
                }
        return;
    }
    // combination c: rows rt0 + wr 64 + 16 crb(c) .., frequency fv + cw(c)
    if (part && stail == 0) {
#pragma unroll
        for (int c = 0; c < 4; c++) {
            if (fv + cw(c) >= nfreq) continue;
            float2 *P = part + ((long)blockIdx.z * nfreq + fv + cw(c)) * NGP * NGP;
#pragma unroll
            for (int cb = 0; cb < 8; cb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = rt0 + wr * 64 + crb(c) * 16 + 4 * lk + r;
                    const int j = ct0 + cb * 16 + li;
                    if (!ST || j < NGP) P[(long)i * NGP + j] = make_float2(accR[c][cb][r], accI[c][cb][r]);
                }
        }
        return;
    }
    // Hermitian: the conjugate of an element outside the block's diagonal
    // tile (128 x 128 form) or outside its strip's leading SH columns (strip
    // form) also goes to the mirrored position, formed by no other block
    const bool mirror_tile = herm && rt != ct;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        if (fv + cw(c) >= nfreq) continue;
        double2 *C = chi + (long)(fv + cw(c)) * ng * ng;
#pragma unroll
        for (int cb = 0; cb < 8; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = rt0 + wr * 64 + crb(c) * 16 + 4 * lk + r;
                const int j = ct0 + cb * 16 + li;
                const bool mirror = ST ? herm && j >= rt0 + SH : mirror_tile;
                if (i < ng && j < ng) {
                    const double2 a = make_double2((double)accR[c][cb][r], (double)accI[c][cb][r]);
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

__device__ __forceinline__ f16v mfma32_bf16(bf8 a, bf8 b, f16v c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Wide form: a 512-thread block owns a 256 x 32 CB tile of (G, G') for NW
// frequencies (CB = 2: 256 x 64, NW = 1 or 2; CB = 4: 256 x 128, NW = 1); each
// of its 8 waves (two per SIMD) owns 32 whole rows of the tile as CB 32 x 32
// blocks on v_mfma_f32_32x32x16_bf16, so every row of A is
// weighted and split by one wave only.  Steps of 16 pairs (one pair group of
// 8 per wave half) stream through two LDS stages (32 KB of A, 2 NT KB of B and
// the step's weights each) by global_load_lds DMA.  The operand layouts are
// those of the prep pass above (a block of 16 rows x 8 pairs in quarter
// order for A; per plane 8 consecutive pairs of one column for B).  The
// contraction of one (a, b) pair is the same sum of split products as in
// k_chi_bf16; only the tiling differs.  Not for a Hermitian chi.  Three LDS
// stages (120 KB) let a step's DMA run two steps ahead of its use.

template <int NT, int NW, int CB>
__global__ void __launch_bounds__(512)
k_chi_bf16_wide(int npg, int NGP, long KP, int ng, const float2 *__restrict__ Ap, const bf8 *__restrict__ Bp,
                int nfreq, const float2 *__restrict__ wq, int accumulate, double2 *__restrict__ chi, int sps,
                float2 *__restrict__ part)
{
    constexpr int NPL = 2 * NT;
    constexpr int TN = 32 * CB;               // tile columns
    constexpr int NBH = NPL * 2 * (TN / 32) / 8;   // B half-segments (512 B) per wave per step
    constexpr int NOPS = 4 + NBH + 1;         // DMA operations per wave per step
    // per stage: A [2 pair groups][16 row blocks][128] float2 (32 KB),
    //            B [NPL planes][2 pair groups][64 cols] bf8, W [NW][16 pairs] float2
    // three stages as distinct objects, so the compiler sees that a stage's
    // reads never touch the two stages whose DMA is in flight
    __shared__ float2 sA0[2 * 16 * 128], sA1[2 * 16 * 128], sA2[2 * 16 * 128];
    __shared__ bf8 sB0[NPL * 2 * TN], sB1[NPL * 2 * TN], sB2[NPL * 2 * TN];
    __shared__ float2 sW0[2 * 16], sW1[2 * 16], sW2[2 * 16];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int r32 = lane & 31, h = lane >> 5;
    const int TC = NGP / TN;
    const int rt0 = (blockIdx.x / TC) * 256, ct0 = (blockIdx.x % TC) * TN;
    const int f0 = blockIdx.z * NW;
    const long plane = (long)npg * NGP;
    const int step0 = blockIdx.y * sps;
    const int nstep = min(sps, npg / 2 - step0);

    // DMA of step t (pair groups 2t, 2t+1), the same number of operations in
    // every wave: wave w moves the A blocks of pair group w/4, row blocks
    // 4(w%4)..4(w%4)+3, NBH of the 4 NPL half-segments of B (32 lanes each),
    // and two of the 16 weight chunks of 16 B (2 lanes; two frequencies)
    auto issue = [&](float2 *dA, bf8 *dB, float2 *dW, int t) {
        const int pgw = 2 * t + (wave >> 2);
        const float2 *a = Ap + ((long)pgw * (NGP / 16) + rt0 / 16 + (wave & 3) * 4) * 128 + lane * 2;
        float2 *da = dA + ((wave >> 2) * 16 + (wave & 3) * 4) * 128;
#pragma unroll
        for (int i = 0; i < 4; i++) dma16(a + i * 128, da + i * 128);
#pragma unroll
        for (int i = 0; i < NBH; i++) {
            const int hs = wave * NBH + i;            // half-segment: plane, pair group, 32 columns
            const int sid = hs / (TN / 32), c32 = hs % (TN / 32);
            const int sp = sid >> 1, g = sid & 1;
            if (lane < 32)
                dma16(Bp + sp * plane + (long)(2 * t + g) * NGP + ct0 + c32 * 32 + lane, dB + sid * TN + c32 * 32);
        }
        if (lane < 2) {
            const int c = wave * 2 + lane;           // chunk: frequency c / 8, pairs 2 (c % 8)
            const int f = min(f0 + min(c / 8, NW - 1), nfreq - 1);
            dma16(wq + (long)f * KP + (long)t * 16 + (c & 7) * 2, dW + wave * 4);
        }
    };

    f16v accR[NW][CB], accI[NW][CB];
#pragma unroll
    for (int iw = 0; iw < NW; iw++)
#pragma unroll
        for (int cb = 0; cb < CB; cb++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                accR[iw][cb][e] = 0.f;
                accI[iw][cb][e] = 0.f;
            }

    auto step = [&](float2 *__restrict__ nA, bf8 *__restrict__ nB, float2 *__restrict__ nW,
                    const float2 *__restrict__ cA, const bf8 *__restrict__ cB, const float2 *__restrict__ cW,
                    int tn) {
        if (tn >= 0) issue(nA, nB, nW, tn);
        const float2 *blk = cA + (h * 16 + 2 * wave + (r32 >> 4)) * 128 + (r32 & 15) * 2;
        float2 araw[8];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float4 v = *(const float4 *)(blk + q * 32);
            araw[2 * q] = make_float2(v.x, v.y);
            araw[2 * q + 1] = make_float2(v.z, v.w);
        }
#pragma unroll
        for (int iw = 0; iw < NW; iw++) {
            float2 wv[8];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 v = *(const float4 *)(cW + iw * 16 + h * 8 + 2 * q);
                wv[2 * q] = make_float2(v.x, v.y);
                wv[2 * q + 1] = make_float2(v.z, v.w);
            }
            bf8 ar[NT], ai[NT], an[NT];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const float2 x = araw[j], y = wv[j];
                __bf16 tr[NT], ti[NT];
                split<NT>(x.x * y.x - x.y * y.y, tr);
                split<NT>(x.x * y.y + x.y * y.x, ti);
#pragma unroll
                for (int s2 = 0; s2 < NT; s2++) {
                    ar[s2][j] = tr[s2];
                    ai[s2][j] = ti[s2];
                }
            }
#pragma unroll
            for (int s2 = 0; s2 < NT; s2++) an[s2] = negate(ar[s2]);
            // column blocks one at a time (their B planes loaded just before use)
#pragma unroll
            for (int cb = 0; cb < CB; cb++) {
                bf8 B[NPL];
#pragma unroll
                for (int sp = 0; sp < NPL; sp++) B[sp] = cB[(sp * 2 + h) * TN + cb * 32 + r32];
                f16v cr = accR[iw][cb], ci = accI[iw][cb];
#pragma unroll
                for (int s2 = 0; s2 < NT; s2++)
#pragma unroll
                    for (int u = 0; u < NT; u++) {
                        if (s2 + u >= NT) continue;
                        cr = mfma32_bf16(ar[s2], B[u], cr);
                        ci = mfma32_bf16(ai[s2], B[u], ci);
                        cr = mfma32_bf16(ai[s2], B[NT + u], cr);
                        ci = mfma32_bf16(an[s2], B[NT + u], ci);
                    }
                accR[iw][cb] = cr;
                accI[iw][cb] = ci;
            }
        }
    };

    auto body = [&](int t, float2 *__restrict__ nA, bf8 *__restrict__ nB, float2 *__restrict__ nW,
                    const float2 *__restrict__ cA, const bf8 *__restrict__ cB, const float2 *__restrict__ cW) {
        if (t + 1 < nstep) __builtin_amdgcn_s_waitcnt(0x0f70 | (NOPS & 0xf) | ((NOPS >> 4) << 14));
        else __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        step(nA, nB, nW, cA, cB, cW, t + 2 < nstep ? step0 + t + 2 : -1);
    };
    if (nstep > 0) issue(sA0, sB0, sW0, step0);
    if (nstep > 1) issue(sA1, sB1, sW1, step0 + 1);
    for (int t = 0; t < nstep; t += 3) {
        body(t, sA2, sB2, sW2, sA0, sB0, sW0);
        if (t + 1 < nstep) body(t + 1, sA0, sB0, sW0, sA1, sB1, sW1);
        if (t + 2 < nstep) body(t + 2, sA1, sB1, sW1, sA2, sB2, sW2);
    }

    // result register e of lane (r32, h) holds row 8 (e / 4) + 4 h + e % 4,
    // column r32 of a 32 x 32 block
#pragma unroll
    for (int iw = 0; iw < NW; iw++) {
        if (f0 + iw >= nfreq) continue;
#pragma unroll
        for (int cb = 0; cb < CB; cb++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int i = rt0 + 32 * wave + 8 * (e >> 2) + 4 * h + (e & 3);
                const int j = ct0 + cb * 32 + r32;
                if (part) {
                    part[((long)blockIdx.y * nfreq + f0 + iw) * NGP * NGP + (long)i * NGP + j] =
                        make_float2(accR[iw][cb][e], accI[iw][cb][e]);
                } else if (i < ng && j < ng) {
                    const double2 a = make_double2((double)accR[iw][cb][e], (double)accI[iw][cb][e]);
                    double2 *C = chi + (long)(f0 + iw) * ng * ng + (long)i * ng + j;
                    *C = accumulate ? cadd(*C, a) : a;
                }
            }
    }
}

// chi (+)= sum over slices of the partial tiles, in FP64, for the computed
// tiles; for a Hermitian chi formed by row strips of hs rows (128 x 128 tiles
// of the upper triangle: hs = 128; the strip tiling: hs = 64) the conjugate
// transpose of a chunk past its strip's leading hs columns goes to the
// mirrored chunk through LDS.  Block: 32 x 32 elements of one
// frequency (grid x over the NGP/32 x NGP/32 chunks, z over frequencies).
__global__ void __launch_bounds__(256)
k_chi_reduce(int nslice, int nfreq, int ng, int NGP, const float2 *__restrict__ part, int accumulate, int herm,
             int hs, double2 *__restrict__ chi)
{
    __shared__ double2 tr[32][33];
    const int nc = NGP / 32;
    const int ci = blockIdx.x / nc, cj = blockIdx.x - ci * nc;
    // Hermitian: the chunk's rows lie in strip rs of hs rows, whose blocks
    // formed the columns from the strip's first row on; the columns past the
    // strip's own hs also go to the mirrored chunk
    const int rs = ci * 32 / hs;
    if (herm && cj * 32 < rs * hs) return;
    const int f = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long plane = (long)NGP * NGP;
    double2 *C = chi + (long)f * ng * ng;
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const int i = ci * 32 + ty + 8 * m, j = cj * 32 + tx;
        const float2 *src = part + (long)f * plane + (long)i * NGP + j;
        double2 v = make_double2(0.0, 0.0);
        for (int sl = 0; sl < nslice; sl++) {
            const float2 x = src[(long)sl * nfreq * plane];
            v.x += (double)x.x;
            v.y += (double)x.y;
        }
        if (i < ng && j < ng) {
            const long idx = (long)i * ng + j;
            C[idx] = accumulate ? cadd(C[idx], v) : v;
        }
        tr[ty + 8 * m][tx] = v;
    }
    if (!(herm && cj * 32 >= (rs + 1) * hs)) return;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; m++) {
        // element (row cj*32 + ty + 8m, column ci*32 + tx) of the mirrored tile
        const int i = cj * 32 + ty + 8 * m, j = ci * 32 + tx;
        const double2 a = tr[tx][ty + 8 * m];
        const double2 v = make_double2(a.x, -a.y);
        if (i < ng && j < ng) {
            const long idx = (long)i * ng + j;
            C[idx] = accumulate ? cadd(C[idx], v) : v;
        }
    }
}

// chi (+)= sum over the stail slices of a tail unit's partial tiles (FP64
// sum), with the mirrored conjugate transpose of an off-diagonal tile of a
// Hermitian chi.  Block: 32 x 32 elements of one tail unit and one frequency
// of its group (grid x = tail unit * 16 + chunk, z = frequency in the group).
__global__ void __launch_bounds__(256)
k_chi_reduce_tail(int nfull, int stail, int NGP, int nw, int nfreq, int ng, int herm, int accumulate,
                  const float2 *__restrict__ part, double2 *__restrict__ chi)
{
    __shared__ double2 tr[32][33];
    const int nt = NGP / kTile;
    const int ntiles = herm ? nt * (nt + 1) / 2 : nt * nt;
    const int u = blockIdx.x / 16, ch = blockIdx.x % 16;
    const int unit = nfull + u;
    const int tile = unit % ntiles, group = unit / ntiles;
    const int iw = blockIdx.z, f = group * nw + iw;
    if (f >= nfreq) return;
    int rt, ct;
    tile_of(tile, nt, herm, rt, ct);
    const int ci = ch / 4, cj = ch % 4;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double2 *C = chi + (long)f * ng * ng;
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const int il = ci * 32 + ty + 8 * m, jl = cj * 32 + tx;
        const float2 *src = part + (((long)u * stail) * nw + iw) * kTile * kTile + (long)il * kTile + jl;
        double2 v = make_double2(0.0, 0.0);
        for (int sl = 0; sl < stail; sl++) {
            const float2 x = src[(long)sl * nw * kTile * kTile];
            v.x += (double)x.x;
            v.y += (double)x.y;
        }
        const int i = rt * kTile + il, j = ct * kTile + jl;
        if (i < ng && j < ng) {
            const long idx = (long)i * ng + j;
            C[idx] = accumulate ? cadd(C[idx], v) : v;
        }
        tr[ty + 8 * m][tx] = v;
    }
    if (!(herm && rt != ct)) return;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; m++) {
        // element (row ct*128 + cj*32 + ty + 8m, column rt*128 + ci*32 + tx) of the mirrored tile
        const int i = ct * kTile + cj * 32 + ty + 8 * m, j = rt * kTile + ci * 32 + tx;
        const double2 a = tr[tx][ty + 8 * m];
        const double2 v = make_double2(a.x, -a.y);
        if (i < ng && j < ng) {
            const long idx = (long)i * ng + j;
            C[idx] = accumulate ? cadd(C[idx], v) : v;
        }
    }
}

long pad_pairs(long npair) { return (npair + kStep - 1) / kStep * kStep; }
int pad_ng(int ng) { return (ng + kTile - 1) / kTile * kTile; }

}  // namespace

size_t split_a_bytes(long npair, int ng) { return (size_t)pad_pairs(npair) * pad_ng(ng) * sizeof(float2); }
size_t split_b_bytes(long npair, int ng) { return (size_t)6 * pad_pairs(npair) * pad_ng(ng) * 2; }
size_t split_w_bytes(long npair, int nfreq) { return (size_t)pad_pairs(npair) * nfreq * sizeof(float2); }

// The contraction form that runs for a requested one: the wide forms take
// complex weights only (no Hermitian half) and rows in blocks of 256, and the
// 256 x 128 form needs the two-term split (three stages of the six-plane B
// operand would not fit in LDS); otherwise the 128 x 128 form.
static int eff_kernel(int kernel, int ng, bool herm, int nterm)
{
    if (kernel == 0 || herm || pad_ng(ng) % 256 != 0) return 0;
    return (kernel == 2 && nterm == 2) ? 2 : 1;
}

// Slices of the pair steps for one contraction: with fill > 0, enough slices
// that the grid holds about `fill` blocks (one block per CU fits), each slice
// at least 8 steps; fill = 0 never slices.
// The strip tiling takes the row form's place (two-frequency groups
// requested) when the frequencies come in groups of four: always for a
// Hermitian chi; for complex weights (strips over all rows, the same
// workgroups and the same arithmetic per element as the 128 x 128 tiles) when
// the pair steps are sliced or the 128 x 128 form's tail split would not
// apply, as the strips do not split their tail.
static bool strips_allowed(bool herm, int nw, int nfreq, int wide)
{
    (void)herm;
    return nw == 2 && !wide && nfreq % 4 == 0;
}

static void tail_plan(long units, int nstep, int fill, int *nfull, int *stail);

static bool use_strips(bool herm, int nw, int nfreq, int wide, long npair, int ng, int fill, int S)
{
    if (!strips_allowed(herm, nw, nfreq, wide)) return false;
    if (herm || S > 1) return true;
    const long t = pad_ng(ng) / kTile;
    int nfull, stail;
    tail_plan(t * t * (nfreq / 2), (int)(pad_pairs(npair) / kStep), fill, &nfull, &stail);
    return stail == 0;
}

// frequencies per workgroup of the strip tiling and its strip height: for a
// Hermitian chi with frequencies in groups of eight, 8 on 32-row strips (whose
// leading blocks waste a quarter of the 64-row strips' lower halves); else 4
// on 64-row strips (for complex weights the 32-row strips measured no faster)
static int strip_sm(int nfreq, bool herm) { return herm && nfreq % 8 == 0 ? 8 : 4; }
static int strip_height(int nfreq, bool herm) { return strip_sm(nfreq, herm) == 8 ? 32 : 64; }

// workgroups per frequency group and slice of the strip tiling
static long strip_blocks(int ng, int nfreq, bool herm)
{
    const int h = strip_height(nfreq, herm);
    const long t = pad_ng(ng) / kTile;
    return herm ? strip_tiles_total(ng, h) : (long)(pad_ng(ng) / h) * t;
}

static void chi_slices(long npair, int ng, int nfreq, bool herm, int nw, int fill, int wide, int *nslice,
                       int *sps)
{
    const int t = pad_ng(ng) / kTile;
    long tiles = herm ? (long)t * (t + 1) / 2 : (long)t * t;
    if (herm && strips_allowed(herm, nw, nfreq, wide)) {
        // (for complex weights the strips hold as many workgroups as the tiles)
        tiles = strip_blocks(ng, nfreq, herm);
        nw = strip_sm(nfreq, herm);
    }
    int nstep = (int)(pad_pairs(npair) / kStep);
    if (wide) {
        const int tn = wide == 2 ? 128 : 64;
        if (wide == 2) nw = 1;
        tiles = (long)(pad_ng(ng) / 256) * (pad_ng(ng) / tn);
        nstep = (int)(pad_pairs(npair) / 16);
    }
    const long blocks = tiles * ((nfreq + nw - 1) / nw);
    int S = 1;
    if (fill > 0 && blocks < fill / 2 && nstep >= 16) {
        S = (int)std::min<long>((fill + blocks - 1) / blocks, nstep / 8);
        S = std::max(1, std::min(S, 64));
    }
    // no slice longer than kFlush steps of the 128 x 128 form (the wide
    // forms' steps hold 16 pairs)
    const int lim = wide ? 2 * kFlush : kFlush;
    S = std::max(S, (nstep + lim - 1) / lim);
    const int per = std::max(1, (nstep + S - 1) / S);
    *sps = per;
    *nslice = std::max(1, (nstep + per - 1) / per);
}

// Compute units of the current device (cached per device).
static int cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        hipDeviceProp_t prop;
        cached[dev] = hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0
                          ? prop.multiProcessorCount
                          : 256;
    }
    return cached[dev];
}

// Tail split of the 128 x 128 form when the pair steps are not sliced: the
// units (tile, frequency group) beyond the last whole wave of the chip run as
// stail slices each, stail (2..16, each slice >= 8 steps) chosen to minimize
// the time of the tail, ceil(R stail / CUs) / stail unit-times for R tail
// units; *stail = 0 when no split helps (or slicing is off, fill = 0).
static void tail_plan(long units, int nstep, int fill, int *nfull, int *stail)
{
    *nfull = (int)units;
    *stail = 0;
    const int cu = cu_count();
    if (fill == 0 || units < cu) return;
    const long R = units % cu;
    if (R == 0) return;
    double best = 1.0;
    for (int sl = 2; sl <= 16 && nstep / sl >= 8; sl++) {
        const double cost = (double)((R * sl + cu - 1) / cu) / sl;
        if (cost < best - 1e-9) {
            best = cost;
            *stail = sl;
        }
    }
    if (*stail) *nfull = (int)(units - R);
}

size_t chi_part_bytes(long npair, int ng, int nfreq, bool herm, int nw, int fill, int kernel, int nterm)
{
    int S, sps;
    const int form = eff_kernel(kernel, ng, herm, nterm);
    nw = nw == 1 ? 1 : 2;
    chi_slices(npair, ng, nfreq, herm, nw, fill, form, &S, &sps);
    if (S == 1) {
        if (form != 0 || use_strips(herm, nw, nfreq, form, npair, ng, fill, S)) return 0;
        const int t = pad_ng(ng) / kTile;
        const long units = (herm ? (long)t * (t + 1) / 2 : (long)t * t) * ((nfreq + nw - 1) / nw);
        int nfull, stail;
        tail_plan(units, (int)(pad_pairs(npair) / kStep), fill, &nfull, &stail);
        if (!stail) return 0;
        return (size_t)(units - nfull) * stail * nw * kTile * kTile * sizeof(float2);
    }
    return (size_t)S * nfreq * (size_t)pad_ng(ng) * pad_ng(ng) * sizeof(float2);
}

SplitOps split_ops(void *split_a, void *split_b, long npair, int ng, int nterm)
{
    SplitOps o;
    o.A = split_a;
    o.B = split_b;
    o.p0 = 0;
    o.NGP = pad_ng(ng);
    o.npg = (int)(pad_pairs(npair) / 8);
    o.nterm = nterm;
    return o;
}

void launch_split_prep(hipStream_t s, int nterm, long npair, int ng, const double2 *M, void *split_a,
                       void *split_b)
{
    const long KP = pad_pairs(npair);
    const int NGP = pad_ng(ng);
    const int npg = (int)(KP / 8);
    const long nt = (long)npg * NGP;
    if (nt == 0) return;
    const dim3 grid((unsigned)((nt + 255) / 256));
    if (nterm == 2)
        hipLaunchKernelGGL(k_split_prep<2>, grid, dim3(256), 0, s, npair, ng, npg, NGP, M, (float2 *)split_a,
                           (bf8 *)split_b);
    else
        hipLaunchKernelGGL(k_split_prep<3>, grid, dim3(256), 0, s, npair, ng, npg, NGP, M, (float2 *)split_a,
                           (bf8 *)split_b);
}

void launch_ops_pad(hipStream_t s, const SplitOps &ops, long npair, int ng)
{
    if (npair <= 0) return;
    const long nrow = (long)ops.npg * (ops.NGP - ng);
    const long ntot = nrow + (ops.npg - npair / 8) * (long)ng;
    if (ntot == 0) return;
    hipLaunchKernelGGL(k_ops_pad, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, ops, npair, ng, nrow,
                       ntot);
}

void launch_weight_prep(hipStream_t s, long npair, int nfreq, const double2 *w, bool herm, void *split_w)
{
    const long KP = pad_pairs(npair);
    const long nw = KP * nfreq;
    if (nw == 0) return;
    hipLaunchKernelGGL(k_weight_prep, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, npair, KP, nfreq, w,
                       (int)herm, (float2 *)split_w);
}

void launch_chi_bf16(hipStream_t s, int nterm, long npair, int ng, int nfreq, int accumulate, double2 *chi,
                     const void *split_a, const void *split_b, const void *split_w, bool herm, int nw, int fill,
                     int kernel, void *part, const std::function<void()> &before_reduce)
{
    const long KP = pad_pairs(npair);
    const int NGP = pad_ng(ng);
    const int npg = (int)(KP / 8);
    const int t = NGP / kTile;
    nw = nw == 1 ? 1 : 2;
    const int wide = eff_kernel(kernel, ng, herm, nterm);
    int S, sps;
    chi_slices(npair, ng, nfreq, herm, nw, fill, wide, &S, &sps);
    float2 *P = S > 1 ? (float2 *)part : nullptr;
    const unsigned nfg = (unsigned)((nfreq + nw - 1) / nw);
    if (wide) {
        const int CBW = wide == 2 ? 4 : 2;
        if (CBW == 4) nw = 1;
        const dim3 grid((unsigned)((NGP / 256) * (NGP / (32 * CBW))), (unsigned)S,
                        (unsigned)((nfreq + nw - 1) / nw));
#define RP_CHIW(NT, NW, CB)                                                                                      \
    hipLaunchKernelGGL((k_chi_bf16_wide<NT, NW, CB>), grid, dim3(512), 0, s, npg, NGP, KP, ng,                   \
                       (const float2 *)split_a, (const bf8 *)split_b, nfreq, (const float2 *)split_w, accumulate, \
                       chi, sps, P)
        if (CBW == 4) {
            RP_CHIW(2, 1, 4);
        } else if (nterm == 2) {
            if (nw == 1) RP_CHIW(2, 1, 2);
            else RP_CHIW(2, 2, 2);
        } else {
            if (nw == 1) RP_CHIW(3, 1, 2);
            else RP_CHIW(3, 2, 2);
        }
#undef RP_CHIW
    } else if (use_strips(herm, nw, nfreq, wide, npair, ng, fill, S)) {
        const int sm = strip_sm(nfreq, herm);
        const dim3 grid((unsigned)strip_blocks(ng, nfreq, herm), (unsigned)(nfreq / sm), (unsigned)S);
#define RP_STRIPS(NT, RW, SM)                                                                                 \
    hipLaunchKernelGGL((k_chi_rows<NT, RW, SM>), grid, dim3(256), 0, s, npg, NGP, KP, ng,                     \
                       (const float2 *)split_a, (const bf8 *)split_b, nfreq, (const float2 *)split_w, accumulate, \
                       chi, (int)herm, sps, P, 0, 0)
#define RP_STRIPS_SM(NT, RW)     \
    if (sm == 8) {               \
        RP_STRIPS(NT, RW, 8);    \
    } else {                     \
        RP_STRIPS(NT, RW, 4);    \
    }
        if (herm) {
            if (nterm == 2) {
                RP_STRIPS_SM(2, true)
            } else {
                RP_STRIPS_SM(3, true)
            }
        } else {
            if (nterm == 2) RP_STRIPS(2, false, 4);
            else RP_STRIPS(3, false, 4);
        }
#undef RP_STRIPS_SM
#undef RP_STRIPS
    } else {
        const unsigned tiles = herm ? (unsigned)(t * (t + 1) / 2) : (unsigned)(t * t);
        int nfull = 0, stail = 0;
        if (S == 1) tail_plan((long)tiles * nfg, npg / 4, fill, &nfull, &stail);
        const long ntail = stail ? (long)tiles * nfg - nfull : 0;
        if (stail) {
            sps = (npg / 4 + stail - 1) / stail;
            P = (float2 *)part;
        }
        const dim3 grid = stail ? dim3((unsigned)(nfull + ntail * stail)) : dim3(tiles, nfg, (unsigned)S);
#define RP_CHI(NT, NW)                                                                                         \
    hipLaunchKernelGGL((k_chi_bf16<NT, NW>), grid, dim3(256), 0, s, npg, NGP, KP, ng, (const float2 *)split_a, \
                       (const bf8 *)split_b, nfreq, (const float2 *)split_w, accumulate, chi, (int)herm, sps, P, \
                       nfull, stail)
#define RP_ROWS(NT, RW)                                                                                       \
    hipLaunchKernelGGL((k_chi_rows<NT, RW, 0>), grid, dim3(256), 0, s, npg, NGP, KP, ng, (const float2 *)split_a,  \
                       (const bf8 *)split_b, nfreq, (const float2 *)split_w, accumulate, chi, (int)herm, sps, P, \
                       nfull, stail)
        if (nw == 1) {
            if (nterm == 2) RP_CHI(2, 1);
            else RP_CHI(3, 1);
        } else if (nterm == 2) {
            if (herm) RP_ROWS(2, true);
            else RP_ROWS(2, false);
        } else {
            if (herm) RP_ROWS(3, true);
            else RP_ROWS(3, false);
        }
#undef RP_ROWS
#undef RP_CHI
        if (stail && before_reduce) before_reduce();
        if (stail)
            hipLaunchKernelGGL(k_chi_reduce_tail, dim3((unsigned)(ntail * 16), 1, (unsigned)nw), dim3(256), 0, s,
                               nfull, stail, NGP, nw, nfreq, ng, (int)herm, accumulate, (const float2 *)P, chi);
    }
    if (S > 1) {
        if (before_reduce) before_reduce();
        const int nc = NGP / 32;
        const int hs = herm && strips_allowed(herm, nw, nfreq, wide) ? strip_height(nfreq, herm) : kTile;
        hipLaunchKernelGGL(k_chi_reduce, dim3((unsigned)(nc * nc), 1, (unsigned)nfreq), dim3(256), 0, s, S, nfreq, ng,
                           NGP, (const float2 *)P, accumulate, (int)herm, hs, chi);
    }
}

}  // namespace rp
