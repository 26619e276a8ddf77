// Step a10 (Eqs. matrix_U, rhoiqG): Wannier densities and the projected
// screened interaction of one q-point.
//
//   f_i(r_j)  = phi_i(r_j)^2 e^{i q.rt_ij},  rt_ij = R_i + minimum image of (r_j - R_i)
//   rho_i(G)  = (Omega/N_r) [sum_j f_i(r_j) e^{iG.r_j}] / |q+G|
//   W_ij(w)   = pre * ( sum_{G,G'} rho_i(G) eps^-1_GG'(w) conj(rho_j(G'))
//                      + sum_{G in tail} rho_i(G) conj(rho_j(G)) ),  pre = HA 4 pi/(Omega Nq)
//
// The e^{iq.rt} factor carries the Bloch phase of the orbital's true position,
// since the home-cell orbital is stored folded into one cell.
#include "fft_lds.h"

namespace rp {

namespace {

__global__ void k_wdens(int nwan, int N1, int N2, int N3, const double *phi, const double *centre,
                        double q1, double q2, double q3, double2 *f)
{
    const long nr = (long)N1 * N2 * N3;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nr * nwan) return;
    const int i = (int)(t / nr);
    const long j = t - (long)i * nr;
    const int j1 = (int)(j / ((long)N2 * N3)), j2 = (int)((j / N3) % N2), j3 = (int)(j % N3);
    const double c1 = centre[3 * i], c2 = centre[3 * i + 1], c3 = centre[3 * i + 2];
    double d1 = (double)j1 / N1 - c1, d2 = (double)j2 / N2 - c2, d3 = (double)j3 / N3 - c3;
    d1 -= floor(d1 + 0.5);
    d2 -= floor(d2 + 0.5);
    d3 -= floor(d3 + 0.5);
    // q.rt = 2 pi sum_a qf_a rtf_a in fractional coordinates
    const double ph = 2.0 * (q1 * (c1 + d1) + q2 * (c2 + d2) + q3 * (c3 + d3));
    double s, c;
    sincospi(ph, &s, &c);
    const double n = phi[t] * phi[t];
    f[t] = make_double2(n * c, n * s);
}

__global__ void k_wgather(int nwan, int N1, int N2, int N3, int nlist, const int *g, double r0,
                          double r1, double r2, double r3, double r4, double r5, double r6, double r7,
                          double r8, double q1, double q2, double q3, double scale, const double2 *fg,
                          double2 *rho, int *flag, int zero_ok)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nlist * nwan) return;
    const int i = (int)(t / nlist), gi = (int)(t - (long)i * nlist);
    const int m1 = g[3 * gi], m2 = g[3 * gi + 1], m3 = g[3 * gi + 2];
    const double f1 = q1 + m1, f2 = q2 + m2, f3 = q3 + m3;
    const double x = f1 * r0 + f2 * r3 + f3 * r6;
    const double y = f1 * r1 + f2 * r4 + f3 * r7;
    const double z = f1 * r2 + f2 * r5 + f3 * r8;
    const double qg = sqrt(x * x + y * y + z * z);
    const long nr = (long)N1 * N2 * N3;
    const double2 v = fg[(long)i * nr + ((long)pmod(m1, N1) * N2 + pmod(m2, N2)) * N3 + pmod(m3, N3)];
    if (qg > 0.0) {
        rho[t] = cscale(v, scale / qg);
    } else if (zero_ok) {
        rho[t] = cscale(v, scale);   // q + G = 0: ntilde(0) itself
    } else {
        atomicOr(flag, kFlagNonFinite);
        rho[t] = cscale(v, scale / qg);
    }
}

// T[f][G][j] = sum_G' eps^-1[f][G][G'] conj(rho_j(G')); one block per (G, f)
__global__ void __launch_bounds__(256) k_wproj1(int nwan, int ng, const double2 *rho, const double2 *einv,
                                                double2 *T)
{
    extern __shared__ double2 red[];  // [256][nwan]
    const int G = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
    const double2 *row = einv + ((long)f * ng + G) * ng;
    for (int j = 0; j < nwan; j++) red[tid * nwan + j] = make_double2(0.0, 0.0);
    for (int h = tid; h < ng; h += 256) {
        const double2 e = row[h];
        for (int j = 0; j < nwan; j++) {
            const double2 r = rho[(long)j * ng + h];
            // e * conj(r)
            red[tid * nwan + j].x += e.x * r.x + e.y * r.y;
            red[tid * nwan + j].y += e.y * r.x - e.x * r.y;
        }
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            for (int j = 0; j < nwan; j++) red[tid * nwan + j] = cadd(red[tid * nwan + j], red[(tid + s) * nwan + j]);
        __syncthreads();
    }
    if (tid < nwan) T[((long)f * ng + G) * nwan + tid] = red[tid];
}

// W[f][i][j] = pre (sum_G rho_i(G) T[f][G][j] + sum_tail rho_i conj(rho_j)); one block per (i,j,f)
__global__ void __launch_bounds__(256) k_wproj2(int nwan, int ng, const double2 *rho, int ntail,
                                                const double2 *rtail, const double2 *T, double pre,
                                                double2 *W)
{
    __shared__ double2 red[256];
    const int i = blockIdx.x / nwan, j = blockIdx.x % nwan, f = blockIdx.y, tid = threadIdx.x;
    double2 s = make_double2(0.0, 0.0);
    for (int G = tid; G < ng; G += 256) s = cadd(s, cmul(rho[(long)i * ng + G], T[((long)f * ng + G) * nwan + j]));
    for (int G = tid; G < ntail; G += 256) s = cadd(s, cmulc(rtail[(long)j * ntail + G], rtail[(long)i * ntail + G]));
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] = cadd(red[tid], red[tid + h]);
        __syncthreads();
    }
    if (tid == 0) W[((long)f * nwan + i) * nwan + j] = cscale(red[0], pre);
}

}  // namespace

void launch_wannier_density(hipStream_t s, const Geometry &g, const FftPlan plans[3], int nwan,
                            const double *phi, const double *centre_frac_dev, double2 *f)
{
    const long tot = (long)g.fft[0] * g.fft[1] * g.fft[2] * nwan;
    hipLaunchKernelGGL(k_wdens, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nwan, g.fft[0],
                       g.fft[1], g.fft[2], phi, centre_frac_dev, (double)g.iq[0] / g.kmesh[0],
                       (double)g.iq[1] / g.kmesh[1], (double)g.iq[2] / g.kmesh[2], f);
    launch_fft3d(s, plans, g.fft, nwan, f);
}

void launch_wannier_gather(hipStream_t s, const Geometry &g, int nwan, int nlist, const int *glist,
                           const double2 *fgrid, double2 *rho, int *flag, bool zero_ok)
{
    const long tot = (long)nlist * nwan;
    if (tot == 0) return;
    const double scale = g.volume / ((double)g.fft[0] * g.fft[1] * g.fft[2]);
    hipLaunchKernelGGL(k_wgather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nwan, g.fft[0],
                       g.fft[1], g.fft[2], nlist, glist, g.rec[0], g.rec[1], g.rec[2], g.rec[3], g.rec[4],
                       g.rec[5], g.rec[6], g.rec[7], g.rec[8], (double)g.iq[0] / g.kmesh[0],
                       (double)g.iq[1] / g.kmesh[1], (double)g.iq[2] / g.kmesh[2], scale, fgrid, rho, flag,
                       (int)zero_ok);
}

void launch_wannier_W(hipStream_t s, int nfreq, int nwan, int ng, const double2 *rho_eps, int ntail,
                      const double2 *rho_tail, const double2 *einv, double pre, double2 *T, double2 *Wij)
{
    const size_t shm = sizeof(double2) * 256 * (size_t)nwan;
    hipLaunchKernelGGL(k_wproj1, dim3(ng, nfreq), dim3(256), shm, s, nwan, ng, rho_eps, einv, T);
    hipLaunchKernelGGL(k_wproj2, dim3(nwan * nwan, nfreq), dim3(256), 0, s, nwan, ng, rho_eps, ntail,
                       rho_tail, T, pre, Wij);
}

}  // namespace rp
