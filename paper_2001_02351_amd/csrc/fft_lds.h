// Batched 1-D FFTs staged in LDS (device code shared by the grid kernels),
// for complex FP64 (double2) and FP32 (float2) data.
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

template <typename C> struct CxT;
template <> struct CxT<double2> { typedef double T; };
template <> struct CxT<float2> { typedef float T; };

template <typename C> __device__ __forceinline__ C mkc(typename CxT<C>::T x, typename CxT<C>::T y)
{
    C c;
    c.x = x;
    c.y = y;
    return c;
}

template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return mkc<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cmulc(C a, C b)  // conj(a) * b
{
    return mkc<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mkc<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mkc<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, typename CxT<C>::T s)
{
    return mkc<C>(a.x * s, a.y * s);
}
template <typename C> __device__ __forceinline__ C mul_i(C a) { return mkc<C>(-a.y, a.x); }

// tw[t] = e^{+2 pi i t/n}, t < n (evaluated in FP64)
template <typename C> __device__ __forceinline__ void fill_twiddles(C *tw, int n, int tid, int nth)
{
    for (int t = tid; t < n; t += nth) {
        double s, c;
        sincospi(2.0 * (double)t / (double)n, &s, &c);
        tw[t] = mkc<C>((typename CxT<C>::T)c, (typename CxT<C>::T)s);
    }
}

template <int R, typename C> struct Dft;

template <typename C> struct Dft<2, C> {
    __device__ static __forceinline__ void run(C *v)
    {
        C a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    }
};

template <typename C> struct Dft<3, C> {
    __device__ static __forceinline__ void run(C *v)
    {
        typedef typename CxT<C>::T T;
        const T h = (T)0.86602540378443864676;  // sqrt(3)/2
        C s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        C t = mkc<C>(v[0].x - (T)0.5 * s.x, v[0].y - (T)0.5 * s.y);
        v[0] = cadd(v[0], s);
        C id = mul_i(d);
        v[1] = mkc<C>(t.x + h * id.x, t.y + h * id.y);
        v[2] = mkc<C>(t.x - h * id.x, t.y - h * id.y);
    }
};

template <typename C> struct Dft<4, C> {
    __device__ static __forceinline__ void run(C *v)
    {
        C s0 = cadd(v[0], v[2]), s1 = csub(v[0], v[2]);
        C s2 = cadd(v[1], v[3]), s3 = mul_i(csub(v[1], v[3]));
        v[0] = cadd(s0, s2);
        v[2] = csub(s0, s2);
        v[1] = cadd(s1, s3);
        v[3] = csub(s1, s3);
    }
};

template <typename C> struct Dft<5, C> {
    __device__ static __forceinline__ void run(C *v)
    {
        typedef typename CxT<C>::T T;
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;  // cos 2pi/5, cos 4pi/5
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;   // sin 2pi/5, sin 4pi/5
        C a = v[0];
        C be = cadd(v[1], v[4]), bme = csub(v[1], v[4]);
        C cd = cadd(v[2], v[3]), cmd = csub(v[2], v[3]);
        C r1 = mkc<C>(a.x + c1 * be.x + c2 * cd.x, a.y + c1 * be.y + c2 * cd.y);
        C r2 = mkc<C>(a.x + c2 * be.x + c1 * cd.x, a.y + c2 * be.y + c1 * cd.y);
        C i1 = mul_i(mkc<C>(s1 * bme.x + s2 * cmd.x, s1 * bme.y + s2 * cmd.y));
        C i2 = mul_i(mkc<C>(s2 * bme.x - s1 * cmd.x, s2 * bme.y - s1 * cmd.y));
        v[0] = cadd(a, cadd(be, cd));
        v[1] = cadd(r1, i1);
        v[4] = csub(r1, i1);
        v[2] = cadd(r2, i2);
        v[3] = csub(r2, i2);
    }
};

// One Stockham stage over `nlines` lines; element i of line l sits at
// buf[l*ls + i*es] in both the input and the output buffer.
template <int R, typename C>
__device__ __forceinline__ void fft_stage(const C *in, C *out, int n, int ns, int nlines, int ls, int es,
                                          const C *tw, int tid, int nth)
{
    const int nb = n / R;
    const int total = nlines * nb;
    const int tstep = n / (ns * R);
    for (int idx = tid; idx < total; idx += nth) {
        int l = idx / nb;
        int j = idx - l * nb;
        const C *src = in + l * ls;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = src[(j + r * nb) * es];
        int jm = j % ns;
        int t = jm * tstep;
#pragma unroll
        for (int r = 1; r < R; r++) v[r] = cmul(v[r], tw[t * r]);
        Dft<R, C>::run(v);
        int od = (j / ns) * ns * R + jm;
        C *dst = out + l * ls;
#pragma unroll
        for (int r = 0; r < R; r++) dst[(od + r * ns) * es] = v[r];
    }
}

// Full transform of `nlines` lines held in a (ping-pong partner b).  Every
// thread of the block must call it.  Returns the buffer holding the result.
template <typename C>
__device__ __forceinline__ C *fft_lines(C *a, C *b, const FftPlan &p, int nlines, int ls, int es, const C *tw,
                                        int tid, int nth)
{
    int ns = 1;
    for (int s = 0; s < p.nrad; s++) {
        int R = p.rad[s];
        if (R == 4) fft_stage<4>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        else if (R == 2) fft_stage<2>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        else if (R == 3) fft_stage<3>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        else fft_stage<5>(a, b, p.n, ns, nlines, ls, es, tw, tid, nth);
        __syncthreads();
        C *t = a;
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

namespace rp {

// ---------------------------------------------------------------------------
// Register FFT: one thread transforms a whole line of compile-time length N
// held in registers (same Stockham stages as above, fully unrolled, no
// synchronization).  tw is a table e^{+2 pi i t/N}, t < N, whose reads are
// uniform across the wave.

constexpr int fft_nstages(int n)
{
    int c = 0;
    for (int r = 4; r >= 2; r -= 2)
        while (n % r == 0) { n /= r; c++; }
    while (n % 3 == 0) { n /= 3; c++; }
    while (n % 5 == 0) { n /= 5; c++; }
    return n == 1 ? c : -1;
}

constexpr int fft_radix(int n, int s)
{
    int c = 0;
    for (int r = 4; r >= 2; r -= 2)
        while (n % r == 0) { if (c == s) return r; n /= r; c++; }
    while (n % 3 == 0) { if (c == s) return 3; n /= 3; c++; }
    while (n % 5 == 0) { if (c == s) return 5; n /= 5; c++; }
    return 1;
}

constexpr int fft_span(int n, int s)
{
    int p = 1;
    for (int i = 0; i < s; i++) p *= fft_radix(n, i);
    return p;
}

template <int N, int S, typename C>
__device__ __forceinline__ void reg_fft_stage(const C (&in)[N], C (&out)[N], const C *tw)
{
    constexpr int R = fft_radix(N, S), NS = fft_span(N, S), NB = N / R, TSTEP = N / (NS * R);
#pragma unroll
    for (int j = 0; j < NB; j++) {
        C v[R];
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = in[j + r * NB];
        const int jm = j % NS;
        const int t = jm * TSTEP;
        if (t != 0) {
#pragma unroll
            for (int r = 1; r < R; r++) v[r] = cmul(v[r], tw[t * r]);
        }
        Dft<R, C>::run(v);
        const int od = (j / NS) * NS * R + jm;
#pragma unroll
        for (int r = 0; r < R; r++) out[od + r * NS] = v[r];
    }
}

template <int N, int S, typename C> struct RegFft {
    // transforms a (scratch b); the result ends in a
    __device__ static __forceinline__ void run(C (&a)[N], C (&b)[N], const C *tw)
    {
        reg_fft_stage<N, S>(a, b, tw);
        if constexpr (S + 1 < fft_nstages(N)) {
            RegFft<N, S + 1, C>::run(b, a, tw);
#pragma unroll
            for (int i = 0; i < N; i++) a[i] = b[i];
        } else {
#pragma unroll
            for (int i = 0; i < N; i++) a[i] = b[i];
        }
    }
};

template <int N, typename C> __device__ __forceinline__ void reg_fft(C (&a)[N], const C *tw)
{
    static_assert(fft_nstages(N) > 0, "FFT length must factor into 2, 3, 5");
    C b[N];
    RegFft<N, 0, C>::run(a, b, tw);
}

// ---------------------------------------------------------------------------
// Quad FFT: a line of length N = 4Q spread over the four lanes of a quad
// (lanes 4i .. 4i+3 of a wave, all active together), decimated in frequency.
// Lane s holds the contiguous inputs x[Q s + n], n < Q.  Writing the output
// index as 4k + r,
//     X[4k + r] = sum_n e^{2 pi i k n/Q} e^{2 pi i r n/N} sum_s i^{r s} x[Q s + n],
// so a 4-point DFT across the quad (two radix-2 steps with DPP quad
// permutations: lane xor 2, then lane xor 1) comes first, then a twiddle and
// a length-Q transform inside each lane.  On return lane s holds
// X[4k + qrow(s)] in x[k], with qrow(s) = (s >> 1) | ((s & 1) << 1).

__device__ __forceinline__ int quad_row(int s) { return (s >> 1) | ((s & 1) << 1); }

template <int CTRL> __device__ __forceinline__ float quad_perm(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL> __device__ __forceinline__ double quad_perm(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// y_r = sum_s i^{r s} v_s across the quad; lane s ends with r = qrow(s)
template <int Q, typename C> __device__ __forceinline__ void quad_dft4(C (&x)[Q], int s)
{
    typedef typename CxT<C>::T T;
    // step 1, partner s ^ 2: lanes with bit 1 clear keep own + partner, the
    // others partner - own; step 2, partner s ^ 1, after lane 3 (odd s, r
    // bit 0 set) has multiplied its value by i
    const T sg1 = (s & 2) ? (T)-1 : (T)1, sg0 = (s & 1) ? (T)-1 : (T)1;
    const bool rot = s == 3;
#pragma unroll
    for (int k = 0; k < Q; k++) {
        const T px = quad_perm<0x4E>(x[k].x), py = quad_perm<0x4E>(x[k].y);
        const T vx = px + sg1 * x[k].x, vy = py + sg1 * x[k].y;
        const T rx = rot ? -vy : vx, ry = rot ? vx : vy;
        const T qx = quad_perm<0xB1>(rx), qy = quad_perm<0xB1>(ry);
        x[k] = mkc<C>(qx + sg0 * rx, qy + sg0 * ry);
    }
}

// twQ[t] = e^{2 pi i t/Q}, t < Q; twN[t] = e^{2 pi i t/N}, t < N
template <int Q, typename C>
__device__ __forceinline__ void quad_fft(C (&x)[Q], const C *twQ, const C *twN, int s)
{
    quad_dft4<Q>(x, s);
    const int r = quad_row(s);
#pragma unroll
    for (int n = 1; n < Q; n++) x[n] = cmul(x[n], twN[r * n]);
    reg_fft<Q>(x, twQ);
}

// ---------------------------------------------------------------------------
// Lane-group FFT: a line of length N = G Q over G adjacent lanes, G in
// {1, 2, 4, 8} (the group's lanes are active together).  G = 4 is the quad form
// above; G = 2 is the same decimation in frequency with a 2-point DFT across
// the lane pair (DPP swap of lanes s and s ^ 1): lane s holds x[Q s + n] and
// ends with X[2k + s] in x[k]; G = 1 is the register FFT of the whole line.
// group_row<G>(s) is the output residue of lane s: X[G k + group_row(s)].

template <int G> __device__ __forceinline__ int group_row(int s)
{
    if constexpr (G == 8) return 2 * quad_row(s & 3) + ((s >> 2) & 1);
    else if constexpr (G == 4) return quad_row(s & 3);
    else if constexpr (G == 2) return s & 1;
    else return 0;
}

// lane 0 ends with x0 + x1, lane 1 with x0 - x1 (x_s the value of lane s)
template <int Q, typename C> __device__ __forceinline__ void pair_dft2(C (&x)[Q], int s)
{
    typedef typename CxT<C>::T T;
    const T sg = (s & 1) ? (T)-1 : (T)1;
#pragma unroll
    for (int k = 0; k < Q; k++) {
        const T px = quad_perm<0xB1>(x[k].x), py = quad_perm<0xB1>(x[k].y);
        x[k] = mkc<C>(px + sg * x[k].x, py + sg * x[k].y);
    }
}

// twQ[t] = e^{2 pi i t/Q}, t < Q; twN[t] = e^{2 pi i t/N}, t < N (for G = 1
// the two tables are the same length and only twQ is read)
// G = 8: a radix-2 step across lanes s and s ^ 4 (lanes 0-3 keep x_s + x_s+4,
// lanes 4-7 take (x_s-4 - x_s) e^{2 pi i (s-4)/8}), then a 4-point DFT across
// each quad: lane s ends with output residue 2 qrow(s & 3) + (s >> 2 & 1).
template <int Q, typename C> __device__ __forceinline__ void oct_dft2(C (&x)[Q], int s)
{
    typedef typename CxT<C>::T T;
    const bool hi = (s & 4) != 0;
    const int m = s & 3;
    // e^{2 pi i m / 8}, m < 4
    const T h = (T)0.70710678118654752440;
    const T wr = m == 0 ? (T)1 : (m == 1 ? h : (m == 2 ? (T)0 : -h));
    const T wi = m == 0 ? (T)0 : (m == 1 ? h : (m == 2 ? (T)1 : h));
#pragma unroll
    for (int k = 0; k < Q; k++) {
        const T px = __shfl_xor(x[k].x, 4), py = __shfl_xor(x[k].y, 4);
        if (!hi) {
            x[k] = mkc<C>(x[k].x + px, x[k].y + py);
        } else {
            const T dx = px - x[k].x, dy = py - x[k].y;
            x[k] = mkc<C>(dx * wr - dy * wi, dx * wi + dy * wr);
        }
    }
}

template <int G, int Q, typename C>
__device__ __forceinline__ void group_fft(C (&x)[Q], const C *twQ, const C *twN, int s)
{
    if constexpr (G == 8) {
        oct_dft2<Q>(x, s);
        quad_dft4<Q>(x, s & 3);
        const int r = group_row<8>(s);
#pragma unroll
        for (int n = 1; n < Q; n++) x[n] = cmul(x[n], twN[r * n]);
        reg_fft<Q>(x, twQ);
    } else if constexpr (G == 4) {
        quad_fft<Q>(x, twQ, twN, s);
    } else if constexpr (G == 2) {
        pair_dft2<Q>(x, s);
        const int r = s & 1;
#pragma unroll
        for (int n = 1; n < Q; n++) x[n] = cmul(x[n], twN[r * n]);
        reg_fft<Q>(x, twQ);
    } else {
        reg_fft<Q>(x, twQ);
    }
}

}  // namespace rp
