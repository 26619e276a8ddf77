// Periodic parts of Bloch functions on the real-space grid (step a2, Eq. pak):
//     u_{nk}(r_j) = sum_{G in S_psi(k)} C_{Gn}(k) e^{iG.r_j}
// by scattering the sphere coefficients into the N1 x N2 x N3 box and applying
// three batched 1-D transforms, one axis at a time.  The first two passes are
// pruned to the lines that can hold a non-zero coefficient (|m_a| <= mmax_a).
// The grids are FP64 (double2) or, for the split-precision path, FP32
// (float2: coefficients rounded to FP32, transforms in FP32).
#include <algorithm>

#include "fft_lds.h"

namespace rp {

namespace {

// Lines of one pass.  Flat line index L = o*C + c; the line's first element
// is at  band*bstride + j1*s1 + j2*s2 + c*cs,  element i at  + i*is,
// with o = (band*B1 + b1)*B2 + b2 and j_a = (b_a - mm_a) mod N_a.
struct LineSet {
    int n;        // transform length
    int is;       // element stride
    long nlines;  // O*C
    int C, cs;
    int B1, mm1, N1, s1;
    int B2, mm2, N2, s2;
    long bstride;
};

__device__ __forceinline__ long line_base(const LineSet &ls, long L)
{
    long o = L / ls.C;
    int c = (int)(L - o * ls.C);
    int b2 = (int)(o % ls.B2);
    long o1 = o / ls.B2;
    int b1 = (int)(o1 % ls.B1);
    long band = o1 / ls.B1;
    int j1 = pmod(b1 - ls.mm1, ls.N1);
    int j2 = pmod(b2 - ls.mm2, ls.N2);
    return band * ls.bstride + (long)j1 * ls.s1 + (long)j2 * ls.s2 + (long)c * ls.cs;
}

// One block transforms `lpb` consecutive lines of the set in LDS.
template <typename C>
__global__ void __launch_bounds__(256) k_fft_lines(C *data, LineSet ls, FftPlan plan, int lpb)
{
    extern __shared__ double2 smem_d[];
    C *smem = (C *)smem_d;
    const int n = ls.n;
    const int ld = n + 1;  // padded line stride against LDS bank conflicts
    C *tw = smem;
    C *a = smem + n;
    C *b = a + (size_t)lpb * ld;
    const int tid = threadIdx.x, nth = blockDim.x;
    const long L0 = (long)blockIdx.x * lpb;
    const int nl = (int)min((long)lpb, ls.nlines - L0);
    fill_twiddles(tw, n, tid, nth);
    // strided lines are adjacent in memory along c: let consecutive threads
    // take consecutive lines so the loads coalesce; contiguous lines let
    // consecutive threads take consecutive elements
    const bool contiguous = (ls.is == 1);
    for (int e = tid; e < nl * n; e += nth) {
        int l, i;
        if (contiguous) { l = e / n; i = e - l * n; }
        else { i = e / nl; l = e - i * nl; }
        a[l * ld + i] = data[line_base(ls, L0 + l) + (long)i * ls.is];
    }
    __syncthreads();
    C *r = fft_lines(a, b, plan, nl, ld, 1, tw, tid, nth);
    for (int e = tid; e < nl * n; e += nth) {
        int l, i;
        if (contiguous) { l = e / n; i = e - l * n; }
        else { i = e / nl; l = e - i * nl; }
        data[line_base(ls, L0 + l) + (long)i * ls.is] = r[l * ld + i];
    }
}

template <typename C> __global__ void k_zero(C *p, long n)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long stride = (long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = mkc<C>(0, 0);
}

// u[band][m mod N] = C[band][g] for g < npw (each Miller index appears once),
// rounded to the grid's precision
template <typename C>
__global__ void k_scatter(const int *miller, const double2 *coef, int npw, int band_stride,
                          int nbands, int N1, int N2, int N3, C *u)
{
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)npw * nbands) return;
    int band = (int)(t / npw), g = (int)(t - (long)band * npw);
    int m1 = pmod(miller[3 * g], N1), m2 = pmod(miller[3 * g + 1], N2), m3 = pmod(miller[3 * g + 2], N3);
    const double2 c = coef[(long)band * band_stride + g];
    typedef typename CxT<C>::T T;
    u[(long)band * N1 * N2 * N3 + ((long)m1 * N2 + m2) * N3 + m3] = mkc<C>((T)c.x, (T)c.y);
}

// lines per block: the tuned count when given (clamped to 64 KB of LDS), else
// 32, 16 or 8 by length
template <typename C> int lines_per_block(int n, int tuned)
{
    int lpb = tuned > 0 ? std::min(tuned, 64) : (n <= 64 ? 32 : (n <= 128 ? 16 : 8));
    while (lpb > 1 && sizeof(C) * ((size_t)n + 2 * (size_t)lpb * (n + 1)) > 65536) lpb /= 2;
    return lpb;
}

template <typename C> void run_pass(hipStream_t s, C *data, const LineSet &ls, const FftPlan &plan, int tuned)
{
    int lpb = lines_per_block<C>(ls.n, tuned);
    long nblk = (ls.nlines + lpb - 1) / lpb;
    size_t shm = sizeof(C) * ((size_t)ls.n + 2 * (size_t)lpb * (ls.n + 1));
    hipLaunchKernelGGL(k_fft_lines<C>, dim3((unsigned)nblk), dim3(256), shm, s, data, ls, plan, lpb);
}

// box extents along an axis: B lines starting at -mm (mod N); full axis if the
// pruned range would cover it
void axis_box(int mmax, int N, int *B, int *mm)
{
    if (mmax < 0 || 2 * mmax + 1 >= N) { *B = N; *mm = 0; }
    else { *B = 2 * mmax + 1; *mm = mmax; }
}

template <typename C>
void fft3d_passes(hipStream_t s, const FftPlan plans[3], const int fft[3], int ngrids,
                  const int mmax[3], C *data, int lines)
{
    const int N1 = fft[0], N2 = fft[1], N3 = fft[2];
    const long nr = (long)N1 * N2 * N3;
    int B1, mm1, B2, mm2;
    axis_box(mmax[0], N1, &B1, &mm1);
    axis_box(mmax[1], N2, &B2, &mm2);
    // axis 3: lines (band, j1 in box, j2 in box), contiguous
    LineSet l3{N3, 1, (long)ngrids * B1 * B2, 1, 0, B1, mm1, N1, N2 * N3, B2, mm2, N2, N3, nr};
    run_pass(s, data, l3, plans[2], lines);
    // axis 2: lines (band, j1 in box, j3), stride N3
    LineSet l2{N2, N3, (long)ngrids * B1 * N3, N3, 1, B1, mm1, N1, N2 * N3, 1, 0, 1, 0, nr};
    run_pass(s, data, l2, plans[1], lines);
    // axis 1: lines (band, j2, j3), stride N2*N3
    LineSet l1{N1, N2 * N3, (long)ngrids * N2 * N3, N2 * N3, 1, 1, 0, 1, 0, 1, 0, 1, 0, nr};
    run_pass(s, data, l1, plans[0], lines);
}

// The u-grids of two band sets (occupied bands at k, empty bands at k+q) that
// sit one after the other in u: one zero fill, a scatter per set, and one set
// of transforms over all nA + nB grids.
template <typename C>
void ugrid2_t(hipStream_t s, const FftPlan plans[3], const int fft[3], const int mmax[3], int nA, int npwA,
              const int *millerA, const double2 *coefA, int nB, int npwB, const int *millerB,
              const double2 *coefB, int band_stride, C *u, int lines)
{
    const long nr = (long)fft[0] * fft[1] * fft[2];
    const long tot = nr * (nA + nB);
    unsigned zb = (unsigned)std::min<long>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero<C>, dim3(zb), dim3(256), 0, s, u, tot);
    const long nsA = (long)npwA * nA, nsB = (long)npwB * nB;
    if (nsA > 0)
        hipLaunchKernelGGL(k_scatter<C>, dim3((unsigned)((nsA + 255) / 256)), dim3(256), 0, s, millerA, coefA, npwA,
                           band_stride, nA, fft[0], fft[1], fft[2], u);
    if (nsB > 0)
        hipLaunchKernelGGL(k_scatter<C>, dim3((unsigned)((nsB + 255) / 256)), dim3(256), 0, s, millerB, coefB, npwB,
                           band_stride, nB, fft[0], fft[1], fft[2], u + nr * nA);
    fft3d_passes(s, plans, fft, nA + nB, mmax, u, lines);
}

}  // namespace

void launch_ugrid2(hipStream_t s, const FftPlan plans[3], const int fft[3], const int mmax[3], int nA, int npwA,
                   const int *millerA, const double2 *coefA, int nB, int npwB, const int *millerB,
                   const double2 *coefB, int band_stride, void *u, bool fp32, int lines)
{
    if (fp32)
        ugrid2_t(s, plans, fft, mmax, nA, npwA, millerA, coefA, nB, npwB, millerB, coefB, band_stride, (float2 *)u,
                 lines);
    else
        ugrid2_t(s, plans, fft, mmax, nA, npwA, millerA, coefA, nB, npwB, millerB, coefB, band_stride, (double2 *)u,
                 lines);
}

void launch_fft3d(hipStream_t s, const FftPlan plans[3], const int fft[3], int ngrids,
                  double2 *data)
{
    const int full[3] = {-1, -1, -1};
    fft3d_passes(s, plans, fft, ngrids, full, data, 0);
}

}  // namespace rp
