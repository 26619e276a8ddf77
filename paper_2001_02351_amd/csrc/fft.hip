// Periodic parts of Bloch functions on the real-space grid (step a2, Eq. pak):
//     u_{nk}(r_j) = sum_{G in S_psi(k)} C_{Gn}(k) e^{iG.r_j}
// by scattering the sphere coefficients into the N1 x N2 x N3 box and applying
// three batched 1-D transforms, one axis at a time.  The first two passes are
// pruned to the lines that can hold a non-zero coefficient (|m_a| <= mmax_a).
// Where an N2 x N3 plane fits in LDS, the scatter and the first two passes run
// plane by plane in LDS (k_ugrid_planes, on the coefficients sorted by plane),
// so the grids go through HBM once before the last pass; otherwise a zero
// fill, a scatter and the first two passes go through HBM.
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

// Counting sort of the plane-wave lists of the two band sets by grid plane:
// block `set` lists the g < npw of plane j1 = m1 mod N1 at perm[set][off[j1]
// .. off[j1 + 1]) (the order within a plane is free: every g has its own
// grid point).  N1 <= 256.
__global__ void __launch_bounds__(256)
k_plane_sort(const int *millerA, int npwA, const int *millerB, int npwB, int N1, int npw_max, int *perm, int *off)
{
    __shared__ int cnt[256];
    const int set = blockIdx.x, tid = threadIdx.x;
    const int *mil = set ? millerB : millerA;
    const int npw = set ? npwB : npwA;
    int *pm = perm + (long)set * npw_max;
    int *of = off + set * (N1 + 1);
    for (int j = tid; j < N1; j += 256) cnt[j] = 0;
    __syncthreads();
    for (int g = tid; g < npw; g += 256) atomicAdd(&cnt[pmod(mil[3 * g], N1)], 1);
    __syncthreads();
    if (tid == 0) {
        int sum = 0;
        for (int j = 0; j < N1; j++) {
            const int c = cnt[j];
            cnt[j] = sum;
            of[j] = sum;
            sum += c;
        }
        of[N1] = sum;
    }
    __syncthreads();
    for (int g = tid; g < npw; g += 256) pm[atomicAdd(&cnt[pmod(mil[3 * g], N1)], 1)] = g;
}

// Axes 3 and 2 of the u-grids plane by plane in LDS: block (j1, band)
// scatters the band's coefficients of plane j1 (from k_plane_sort) into a
// zeroed N2 x N3 plane, transforms the rows that can hold a non-zero
// coefficient (|m2| <= mmax2, as the pruned pass along axis 3 does), then
// every column along axis 2, and writes the plane; planes outside the box
// |m1| <= mmax1 are written as zeros.  The same transforms of the same values
// as the zero fill, scatter and first two passes of fft3d_passes.
template <typename C>
__global__ void __launch_bounds__(256)
k_ugrid_planes(const int *millerA, const double2 *coefA, int nA, const int *millerB, const double2 *coefB,
               int band_stride, const int *perm, const int *off, int npw_max, int N1, int N2, int N3, int B1,
               int mm1, int B2, int mm2, FftPlan p2, FftPlan p3, C *u)
{
    typedef typename CxT<C>::T T;
    extern __shared__ double2 smem_d[];
    C *smem = (C *)smem_d;
    const int ld = N3 + 1;
    C *tw2 = smem, *tw3 = tw2 + N2, *a = tw3 + N3, *b = a + (size_t)N2 * ld;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int j1 = blockIdx.x, band = blockIdx.y;
    C *dst = u + ((long)band * N1 + j1) * N2 * N3;
    if (pmod(j1 + mm1, N1) >= B1) {
        for (int e = tid; e < N2 * N3; e += nth) dst[e] = mkc<C>(0, 0);
        return;
    }
    const int set = band >= nA ? 1 : 0;
    const int *mil = set ? millerB : millerA;
    const double2 *cf = (set ? coefB : coefA) + (long)(band - set * nA) * band_stride;
    const int *pm = perm + (long)set * npw_max;
    const int *of = off + set * (N1 + 1);
    fill_twiddles(tw2, N2, tid, nth);
    fill_twiddles(tw3, N3, tid, nth);
    for (int e = tid; e < 2 * N2 * ld; e += nth) a[e] = mkc<C>(0, 0);
    __syncthreads();
    for (int e = of[j1] + tid; e < of[j1 + 1]; e += nth) {
        const int g = pm[e];
        const double2 c = cf[g];
        a[pmod(mil[3 * g + 1], N2) * ld + pmod(mil[3 * g + 2], N3)] = mkc<C>((T)c.x, (T)c.y);
    }
    __syncthreads();
    // axis 3 over the box rows j2 = (b2 - mm2) mod N2, b2 < B2: two runs of rows
    const int lo = B2 - mm2;                  // rows 0 .. lo - 1
    C *r = fft_lines(a, b, p3, lo, ld, 1, tw3, tid, nth);
    if (mm2 > 0) fft_lines(a + (size_t)(N2 - mm2) * ld, b + (size_t)(N2 - mm2) * ld, p3, mm2, ld, 1, tw3, tid, nth);
    // axis 2 over every column (the result of both runs is in r)
    C *o = r == a ? b : a;
    C *r2 = fft_lines(r, o, p2, N3, 1, ld, tw2, tid, nth);
    for (int e = tid; e < N2 * N3; e += nth) {
        const int j2 = e / N3, j3 = e - j2 * N3;
        dst[e] = r2[j2 * ld + j3];
    }
}

// LDS of k_ugrid_planes: twiddles of axes 2 and 3 and two padded planes
template <typename C> size_t planes_lds_bytes(const int fft[3])
{
    return sizeof(C) * ((size_t)fft[1] + fft[2] + 2 * (size_t)fft[1] * (fft[2] + 1));
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
    const size_t shm = planes_lds_bytes<C>(fft);
    if (fft[0] <= 256 && shm <= 160 * 1024 && nA + nB > 0) {
        // sort workspace after the grids (ugrid_bytes counts it)
        int *perm = (int *)(u + tot);
        int *off = perm + 2 * (long)band_stride;
        hipLaunchKernelGGL(k_plane_sort, dim3(2), dim3(256), 0, s, millerA, npwA, millerB, npwB, fft[0], band_stride,
                           perm, off);
        int B1, mm1, B2, mm2;
        axis_box(mmax[0], fft[0], &B1, &mm1);
        axis_box(mmax[1], fft[1], &B2, &mm2);
        if (shm > 65536)
            (void)hipFuncSetAttribute((const void *)&k_ugrid_planes<C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)shm);
        hipLaunchKernelGGL(k_ugrid_planes<C>, dim3((unsigned)fft[0], (unsigned)(nA + nB)), dim3(256), shm, s, millerA,
                           coefA, nA, millerB, coefB, band_stride, perm, off, band_stride, fft[0], fft[1], fft[2], B1,
                           mm1, B2, mm2, plans[1], plans[2], u);
        // axis 1: lines (band, j2, j3), stride N2*N3
        const int N2 = fft[1], N3 = fft[2];
        LineSet l1{fft[0], N2 * N3, (long)(nA + nB) * N2 * N3, N2 * N3, 1, 1, 0, 1, 0, 1, 0, 1, 0, nr};
        run_pass(s, u, l1, plans[0], lines);
        return;
    }
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

size_t ugrid_bytes(const int fft[3], int nbands, int npw_max, bool fp32)
{
    const size_t nr = (size_t)fft[0] * fft[1] * fft[2];
    return nr * nbands * (fp32 ? sizeof(float2) : sizeof(double2)) + sizeof(int) * (2 * (size_t)npw_max + 2 * 257);
}

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
