// Batched 1-D FFTs staged in LDS (device code shared by the grid kernels).
//
// Transform convention used throughout the library:
//     y[k] = sum_j x[j] e^{+2 pi i j k / n}      (no scaling)
// which is both the plane-wave synthesis u(r) = sum_G C_G e^{iG.r} and the
// analysis sum_r f(r) e^{iG.r} that the pair densities need (Eq. ism).
//
// Algorithm: Stockham autosort with radix-4/2/3/5 stages.  At a stage of
// radix R, after Ns points have already been combined, butterfly j of a line
// reads x[j + r n/R] (r < R), multiplies by e^{2 pi i (j mod Ns) r/(Ns R)},
// applies an R-point DFT and writes y[(j div Ns) Ns R + (j mod Ns) + r Ns].
// The output comes out in natural order after the last stage.
#pragma once

#include <hip/hip_runtime.h>

#include "rp_internal.h"

namespace rp {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)  // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 mul_i(double2 a) { return make_double2(-a.y, a.x); }

// tw[t] = e^{+2 pi i t/n}, t < n
__device__ __forceinline__ void fill_twiddles(double2 *tw, int n, int tid, int nth)
{
    for (int t = tid; t < n; t += nth) {
        double s, c;
        sincospi(2.0 * (double)t / (double)n, &s, &c);
        tw[t] = make_double2(c, s);
    }
}

template <int R> struct Dft;

template <> struct Dft<2> {
    __device__ static __forceinline__ void run(double2 *v)
    {
        double2 a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    }
};

template <> struct Dft<3> {
    __device__ static __forceinline__ void run(double2 *v)
    {
        const double h = 0.86602540378443864676;  // sqrt(3)/2
        double2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        double2 t = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
        v[0] = cadd(v[0], s);
        double2 id = mul_i(d);
        v[1] = make_double2(t.x + h * id.x, t.y + h * id.y);
        v[2] = make_double2(t.x - h * id.x, t.y - h * id.y);
    }
};

template <> struct Dft<4> {
    __device__ static __forceinline__ void run(double2 *v)
    {
        double2 s0 = cadd(v[0], v[2]), s1 = csub(v[0], v[2]);
        double2 s2 = cadd(v[1], v[3]), s3 = mul_i(csub(v[1], v[3]));
        v[0] = cadd(s0, s2);
        v[2] = csub(s0, s2);
        v[1] = cadd(s1, s3);
        v[3] = csub(s1, s3);
    }
};

template <> struct Dft<5> {
    __device__ static __forceinline__ void run(double2 *v)
    {
        const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;  // cos 2pi/5, cos 4pi/5
        const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;   // sin 2pi/5, sin 4pi/5
        double2 a = v[0];
        double2 be = cadd(v[1], v[4]), bme = csub(v[1], v[4]);
        double2 cd = cadd(v[2], v[3]), cmd = csub(v[2], v[3]);
        double2 r1 = make_double2(a.x + c1 * be.x + c2 * cd.x, a.y + c1 * be.y + c2 * cd.y);
        double2 r2 = make_double2(a.x + c2 * be.x + c1 * cd.x, a.y + c2 * be.y + c1 * cd.y);
        double2 i1 = mul_i(make_double2(s1 * bme.x + s2 * cmd.x, s1 * bme.y + s2 * cmd.y));
        double2 i2 = mul_i(make_double2(s2 * bme.x - s1 * cmd.x, s2 * bme.y - s1 * cmd.y));
        v[0] = cadd(a, cadd(be, cd));
        v[1] = cadd(r1, i1);
        v[4] = csub(r1, i1);
        v[2] = cadd(r2, i2);
        v[3] = csub(r2, i2);
    }
};

// One Stockham stage over `nlines` lines; element i of line l sits at
// buf[l*ls + i*es] in both the input and the output buffer.
template <int R>
__device__ __forceinline__ void fft_stage(const double2 *in, double2 *out, int n, int ns, int nlines,
                                          int ls, int es, const double2 *tw, int tid, int nth)
{
    const int nb = n / R;
    const int total = nlines * nb;
    const int tstep = n / (ns * R);
    for (int idx = tid; idx < total; idx += nth) {
        int l = idx / nb;
        int j = idx - l * nb;
        const double2 *src = in + l * ls;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = src[(j + r * nb) * es];
        int jm = j % ns;
        int t = jm * tstep;
#pragma unroll
        for (int r = 1; r < R; r++) v[r] = cmul(v[r], tw[t * r]);
        Dft<R>::run(v);
        int od = (j / ns) * ns * R + jm;
        double2 *dst = out + l * ls;
#pragma unroll
        for (int r = 0; r < R; r++) dst[(od + r * ns) * es] = v[r];
    }
}

// Full transform of `nlines` lines held in a (ping-pong partner b).  Every
// thread of the block must call it.  Returns the buffer holding the result.
__device__ __forceinline__ double2 *fft_lines(double2 *a, double2 *b, const FftPlan &p, int nlines,
                                              int ls, int es, const double2 *tw, int tid, int nth)
{
    int ns = 1;
    for (int s = 0; s < p.nrad; s++) {
        int R = p.rad[s];
        if (R == 4) fft_stage<4>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        else if (R == 2) fft_stage<2>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        else if (R == 3) fft_stage<3>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        else fft_stage<5>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        __syncthreads();
        double2 *t = a;
        a = b;
        b = t;
        ns *= R;
    }
    return a;
}

__device__ __forceinline__ int pmod(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

}  // namespace rp
