// q -> 0 head of the pair densities and the optical quantities
// (Eqs. eps00-cRPA, momentum, epsilonM, eels, optical-conductivity,
// reflectance).
//
// Head density.  For q -> 0 the G = 0 pair density of an empty band a and an
// occupied band b at the same k is, to first order in q (k.p perturbation of
// the periodic parts), q . p_ab(k) / (E_a(k) - E_b(k)) with the transition
// moment p_ab = <psi_a| -i grad |psi_b> (the non-local pseudopotential term
// dropped).  In the plane-wave expansion
//     qhat . p_ab(k) = sum_G conj(C_Ga(k)) (qhat . (k + G)) C_Gb(k),
// so the head density h_ab = qhat . p_ab / (E_a - E_b) replaces M(q, G = 0) / |q|
// and the contraction of Eq. chi then gives lim chi_00 / q^2 and
// lim chi_0G / q; eps keeps its form with v^1/2_0 = sqrt(4 pi / Omega).
//
// Intraband (Drude) term of the head (Eqs. eps00, plasma): the diagonal
// moments p_a(k) feed the Fermi-surface sum of the plasma tensor (with the
// tetrahedron weights of the Fermi surface), and its projection wq on the
// direction of q enters eps_00 as -wq / (w (w + i delta)).
//
// Optics from eps^-1_00 per frequency: eps_M = 1 / eps^-1_00,
// L = -Im eps^-1_00, Re sigma = (w / 4 pi) Im eps_M (w in hartree, atomic
// units), R = |(sqrt(eps_M) - 1) / (sqrt(eps_M) + 1)|^2 (principal root).
#include "fft_lds.h"

namespace rp {

namespace {

constexpr int kHT = 8;    // bands per tile side (8 empty x 8 occupied per block)
constexpr int kHG = 64;   // plane waves per LDS stage

// Block (chunk of 8 occupied, chunk of 8 empty, k): 64 (a, b) sums, each
// split over 4 lanes that take every fourth plane wave of a stage; the 16
// coefficient rows of a stage and the weights qhat . (k + G) sit in LDS.
__global__ void __launch_bounds__(256)
k_head(const int *__restrict__ miller, const double2 *__restrict__ coef, const double *__restrict__ E,
       const int *__restrict__ npw, int nband, int npw_max, int o0, int nO, int e0, int nE, int k0, int K1, int K2,
       int K3, double r0, double r1, double r2, double r3, double r4, double r5, double r6, double r7, double r8,
       double qx, double qy, double qz, int ldm, int col, double2 *__restrict__ M, int *flag)
{
    __shared__ double2 sa[kHT][kHG + 1];
    __shared__ double2 sb[kHT][kHG + 1];
    __shared__ double ss[kHG];
    const int tid = threadIdx.x;
    const int k = k0 + blockIdx.z;
    const int a0 = e0 + blockIdx.y * kHT, b0 = o0 + blockIdx.x * kHT;
    const int n = npw[k];
    const double kf1 = (double)(k / (K2 * K3)) / K1, kf2 = (double)((k / K3) % K2) / K2, kf3 = (double)(k % K3) / K3;
    // qhat . (k + G) = f . (rec qhat) for fractional f = k + m
    const double c1 = r0 * qx + r1 * qy + r2 * qz, c2 = r3 * qx + r4 * qy + r5 * qz, c3 = r6 * qx + r7 * qy + r8 * qz;
    const int out = tid >> 2, l4 = tid & 3;
    const int ia = out >> 3, ib = out & 7;
    double2 acc = make_double2(0.0, 0.0);
    for (int g0 = 0; g0 < n; g0 += kHG) {
        for (int e = tid; e < kHT * kHG; e += 256) {
            const int r = e / kHG, gg = e - r * kHG, g = g0 + gg;
            double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
            if (g < n && a0 + r < e0 + nE) va = coef[((long)k * nband + a0 + r) * npw_max + g];
            if (g < n && b0 + r < o0 + nO) vb = coef[((long)k * nband + b0 + r) * npw_max + g];
            sa[r][gg] = va;
            sb[r][gg] = vb;
        }
        if (tid < kHG) {
            const int g = g0 + tid;
            double s = 0.0;
            if (g < n) {
                const int *m = miller + ((long)k * npw_max + g) * 3;
                s = (kf1 + m[0]) * c1 + (kf2 + m[1]) * c2 + (kf3 + m[2]) * c3;
            }
            ss[tid] = s;
        }
        __syncthreads();
#pragma unroll 4
        for (int gg = l4; gg < kHG; gg += 4) {
            const double2 x = sa[ia][gg], y = sb[ib][gg];
            const double s = ss[gg];
            acc.x += s * (x.x * y.x + x.y * y.y);
            acc.y += s * (x.x * y.y - x.y * y.x);
        }
        __syncthreads();
    }
    acc.x += __shfl_xor(acc.x, 1);
    acc.y += __shfl_xor(acc.y, 1);
    acc.x += __shfl_xor(acc.x, 2);
    acc.y += __shfl_xor(acc.y, 2);
    const int a = a0 + ia, b = b0 + ib;
    if (l4 == 0 && a < e0 + nE && b < o0 + nO) {
        const double de = (E[(long)k * nband + a] - E[(long)k * nband + b]) / kHartreeEv;
        const long p = ((long)(k - k0) * nE + (a - e0)) * nO + (b - o0);
        // an intraband pair (a = b, overlapping band ranges of a metal) belongs
        // to the intraband term of the head, not to the head density
        double2 h = make_double2(0.0, 0.0);
        if (a == b) h = make_double2(0.0, 0.0);
        else if (de != 0.0) h = make_double2(acc.x / de, acc.y / de);
        else atomicOr(flag, kFlagNonFinite);
        M[p * ldm + col] = h;
    }
}

__device__ __forceinline__ double2 csqrt_principal(double2 z)
{
    const double r = hypot(z.x, z.y);
    return make_double2(sqrt(0.5 * (r + z.x)), copysign(sqrt(0.5 * fmax(r - z.x, 0.0)), z.y));
}

// Diagonal moments p_a(k) = <psi_a| -i grad |psi_a> = sum_G |C_Ga(k)|^2 (k + G)
// (Eq. momentum, local part), Cartesian: one block per (band a, k), written to
// p[(k * nb + a - b0) * 3 + mu].
__global__ void __launch_bounds__(256)
k_pdiag(const int *__restrict__ miller, const double2 *__restrict__ coef, const int *__restrict__ npw, int nband,
        int npw_max, int b0, int nb, int K1, int K2, int K3, double r0, double r1, double r2, double r3, double r4,
        double r5, double r6, double r7, double r8, double *__restrict__ p)
{
    __shared__ double red[3][4];
    const int tid = threadIdx.x, a = b0 + blockIdx.x, k = blockIdx.y;
    const int n = npw[k];
    const double kf1 = (double)(k / (K2 * K3)) / K1, kf2 = (double)((k / K3) % K2) / K2, kf3 = (double)(k % K3) / K3;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;    // fractional components of sum |C|^2 (k + m)
    const double2 *c = coef + ((long)k * nband + a) * npw_max;
    const int *m = miller + (long)k * npw_max * 3;
    for (int g = tid; g < n; g += 256) {
        const double2 v = c[g];
        const double w = v.x * v.x + v.y * v.y;
        s1 += w * (kf1 + m[3 * g]);
        s2 += w * (kf2 + m[3 * g + 1]);
        s3 += w * (kf3 + m[3 * g + 2]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
        s3 += __shfl_xor(s3, o);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = s1;
        red[1][tid >> 6] = s2;
        red[2][tid >> 6] = s3;
    }
    __syncthreads();
    if (tid == 0) {
        const double f1 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const double f2 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        const double f3 = red[2][0] + red[2][1] + red[2][2] + red[2][3];
        double *out = p + ((long)k * nb + blockIdx.x) * 3;
        out[0] = f1 * r0 + f2 * r3 + f3 * r6;
        out[1] = f1 * r1 + f2 * r4 + f3 * r7;
        out[2] = f1 * r2 + f2 * r5 + f3 * r8;
    }
}

// w (w + i delta) in eV^2 for w = freq (eV, complex)
__device__ __forceinline__ double2 drude_den(double2 w, double delta)
{
    return make_double2(w.x * w.x - w.y * (w.y + delta), w.x * (w.y + delta) + w.y * w.x);
}

// The intraband term of the head: eps_00 -= wq / (w (w + i delta)).  Where
// w (w + i delta) = 0 the term is infinite; the head row and column of eps are
// then replaced by those of the identity, so that the inversion returns the
// body's inverse (the limit), and k_drude_zero clears the head afterwards.
// One thread per (frequency, i), i along the head row and column.
__global__ void k_drude_head(int nfreq, int ng, const double2 *__restrict__ freq, double wq, double delta,
                             double2 *__restrict__ eps)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nfreq * ng) return;
    const int f = (int)(t / ng), i = (int)(t - (long)f * ng);
    const double2 den = drude_den(freq[f], delta);
    double2 *E = eps + (long)f * ng * ng;
    if (den.x == 0.0 && den.y == 0.0) {
        E[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
        E[(long)i * ng] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
    } else if (i == 0) {
        const double d = den.x * den.x + den.y * den.y;
        E[0] = make_double2(E[0].x - wq * den.x / d, E[0].y + wq * den.y / d);
    }
}

__global__ void k_drude_zero(int nfreq, int ng, const double2 *__restrict__ freq, double delta,
                             double2 *__restrict__ einv)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfreq) return;
    const double2 den = drude_den(freq[f], delta);
    if (den.x == 0.0 && den.y == 0.0) einv[(long)f * ng * ng] = make_double2(0.0, 0.0);
}

// out[f] = {Re eps_M, Im eps_M, L, Re sigma, R}; an infinite head (eps^-1_00
// = 0, a metal's static limit) gives L = 0, R = 1 and NaN for the others
__global__ void k_optics(int nfreq, int ng, const double2 *__restrict__ einv, const double2 *__restrict__ freq,
                         double *__restrict__ out)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfreq) return;
    const double2 e = einv[(long)f * ng * ng];
    const double d = e.x * e.x + e.y * e.y;
    if (d == 0.0) {
        double *z = out + 5L * f;
        const double nan = __builtin_nan("");
        z[0] = nan;
        z[1] = nan;
        z[2] = 0.0;
        z[3] = nan;
        z[4] = 1.0;
        return;
    }
    const double2 em = make_double2(e.x / d, -e.y / d);
    const double w = freq[f].x / kHartreeEv;
    const double2 s = csqrt_principal(em);
    const double2 num = make_double2(s.x - 1.0, s.y), den = make_double2(s.x + 1.0, s.y);
    const double R = (num.x * num.x + num.y * num.y) / (den.x * den.x + den.y * den.y);
    double *o = out + 5L * f;
    o[0] = em.x;
    o[1] = em.y;
    o[2] = -e.y;
    o[3] = w / (4.0 * kPi) * em.y;
    o[4] = R;
}

}  // namespace

void launch_head(hipStream_t s, const Geometry &g, const int *miller, const double2 *coef, const double *E,
                 const int *npw_dev, int nband, int npw_max, int o0, int o1, int e0, int e1, int k0, int k1,
                 const double qhat[3], int ldm, int col, double2 *M, int *flag)
{
    const int nO = o1 - o0, nE = e1 - e0;
    const dim3 grid((unsigned)((nO + kHT - 1) / kHT), (unsigned)((nE + kHT - 1) / kHT), (unsigned)(k1 - k0));
    hipLaunchKernelGGL(k_head, grid, dim3(256), 0, s, miller, coef, E, npw_dev, nband, npw_max, o0, nO, e0, nE, k0,
                       g.kmesh[0], g.kmesh[1], g.kmesh[2], g.rec[0], g.rec[1], g.rec[2], g.rec[3], g.rec[4],
                       g.rec[5], g.rec[6], g.rec[7], g.rec[8], qhat[0], qhat[1], qhat[2], ldm, col, M, flag);
}

void launch_pdiag(hipStream_t s, const Geometry &g, const int *miller, const double2 *coef, const int *npw_dev,
                  int nband, int npw_max, int b0, int b1, double *p)
{
    if (b1 <= b0 || g.nk == 0) return;
    hipLaunchKernelGGL(k_pdiag, dim3((unsigned)(b1 - b0), (unsigned)g.nk), dim3(256), 0, s, miller, coef, npw_dev,
                       nband, npw_max, b0, b1 - b0, g.kmesh[0], g.kmesh[1], g.kmesh[2], g.rec[0], g.rec[1], g.rec[2],
                       g.rec[3], g.rec[4], g.rec[5], g.rec[6], g.rec[7], g.rec[8], p);
}

void launch_drude_head(hipStream_t s, int nfreq, int ng, const double2 *freq, double wq, double delta, double2 *eps)
{
    const long n = (long)nfreq * ng;
    hipLaunchKernelGGL(k_drude_head, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nfreq, ng, freq, wq, delta,
                       eps);
}

void launch_drude_zero(hipStream_t s, int nfreq, int ng, const double2 *freq, double delta, double2 *einv)
{
    hipLaunchKernelGGL(k_drude_zero, dim3((unsigned)((nfreq + 63) / 64)), dim3(64), 0, s, nfreq, ng, freq, delta,
                       einv);
}

void launch_optics(hipStream_t s, int nfreq, int ng, const double2 *einv, const double2 *freq, double *out)
{
    hipLaunchKernelGGL(k_optics, dim3((unsigned)((nfreq + 63) / 64)), dim3(64), 0, s, nfreq, ng, einv, freq, out);
}

}  // namespace rp
