// One q-point's term of the q-mesh sums of the interaction parameters
// (Eqs. W, Wq, matrix_U, rhoiqG, matrix_V, matrix_J, matrix_X):
//
//   U_i0jR(w) += e^{-iq.R} pre [ sum_{G,G' in S_eps} rho_i(G) eps^-1_GG'(w) conj(rho_j(G'))
//                                + sum_{G in tail} rho_i conj(rho_j) + head ]
//   V_i0jR    += e^{-iq.R} pre [ sum_{G in S_eps + tail} rho_i conj(rho_j) + head ]
//   J_i0jR(w) += pre [ sum_{G,G'} rho_v(G) eps^-1_GG'(w) conj(rho_v(G')) + tail + head ]
//   X_i0jR    += pre [ sum_{G in S_eps + tail} |rho_v(G)|^2 + head ]
//
// with pre = HA 4 pi / (Omega N_q), rho = ntilde(q+G)/|q+G|, the direct
// densities rho_i of the orbitals' own densities and the exchange densities
// rho_v, v = (R, i, j), of the overlap densities phi_i0 phi_jR.  The overlap
// density is taken on the images of the grid points nearest the midpoint
// (c_i + c_j + R)/2, phi_i0 where the image lies within half a cell of c_i
// and phi_jR within half a cell of c_j + R (each orbital is stored folded
// into one cell and stands for a function localized within half a cell of
// its centre).
//
// At q = 0 the first G is G = 0: its density is stored as ntilde(0) (not
// divided by |q|) and enters only through the head term
// A eps^-1_00 ntilde_a(0) conj(ntilde_b(0)) (eps^-1_00 -> 1 for V, X), A the
// mean of 1/|q|^2 over the q-cell around Gamma; the wings are dropped (odd
// in q to leading order).
//
// The quadratic forms run as T = eps^-1 conj(P)^T on the FP64 matrix cores
// (64 x 64 tiles of (G, vector), 16x16x4 FP64 MFMAs), then per vector or per
// orbital pair a reduction with the densities themselves.
#include "fft_lds.h"

namespace rp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double x, double y, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// Overlap-density grids of vectors v0 .. v0 + nvc - 1 (v = (r nwan + i) nwan
// + j), each times e^{iq.rt}; one thread per (vector, grid point).
__global__ void k_xdens(int nwan, int N1, int N2, int N3, const double *__restrict__ phi,
                        const double *__restrict__ centre, const int *__restrict__ R, long v0, int nvc,
                        double q1, double q2, double q3, double2 *__restrict__ f)
{
    const long nr = (long)N1 * N2 * N3;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nr * nvc) return;
    const long lv = t / nr, p = t - lv * nr;
    const long v = v0 + lv;
    const int j = (int)(v % nwan), i = (int)((v / nwan) % nwan), r = (int)(v / ((long)nwan * nwan));
    const int p1 = (int)(p / ((long)N2 * N3)), p2 = (int)((p / N3) % N2), p3 = (int)(p % N3);
    const double x[3] = {(double)p1 / N1, (double)p2 / N2, (double)p3 / N3};
    const double qf[3] = {q1, q2, q3};
    const double *ci = centre + 3 * i, *cj = centre + 3 * j;
    const int *Rv = R + 3 * r;
    bool in = true;
    double ph = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double m = 0.5 * (ci[a] + cj[a] + (double)Rv[a]);
        double d = x[a] - m;
        d -= floor(d + 0.5);
        const double rt = m + d;
        const double di = rt - ci[a], dj = rt - (double)Rv[a] - cj[a];
        in = in && di >= -0.5 && di < 0.5 && dj >= -0.5 && dj < 0.5;
        ph += qf[a] * rt;
    }
    const double val = in ? phi[(long)i * nr + p] * phi[(long)j * nr + p] : 0.0;
    double s, c;
    sincospi(2.0 * ph, &s, &c);
    f[t] = make_double2(val * c, val * s);
}

// T = E conj(P)^T over K in [klo, ng) for one frequency (grid z), a 64 x 64
// tile of (G, vector) per block; E [nfreq][ng][ng], P [nv][ldp].
// DIAG: out[tile row][f][v] = sum over the tile's rows G in [klo, ng) of
//       P[v][G] T[G][v];  otherwise out[f][G][v] = T[G][v] (ld nv).
template <bool DIAG>
__global__ void __launch_bounds__(256)
k_wgemm(int ng, int klo, int nv, int nfreq, const double2 *__restrict__ P, long ldp,
        const double2 *__restrict__ E, double2 *__restrict__ out)
{
    constexpr int KC = 16;
    __shared__ double2 sE[64][KC + 1];
    __shared__ double2 sP[KC][64 + 1];
    __shared__ double2 red[2][64];
    const int f = blockIdx.z, tid = threadIdx.x;
    const int rt0 = blockIdx.y * 64, v0 = blockIdx.x * 64;
    const double2 *Ef = E + (long)f * ng * ng;
    const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    d4 accR[2][2], accI[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++) {
            accR[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
            accI[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
        }
    for (int kc = 0; kc < ng; kc += KC) {
        for (int e = tid; e < 64 * KC; e += 256) {
            const int rr = e / KC, k = e - rr * KC, i = rt0 + rr, K = kc + k;
            sE[rr][k] = (i < ng && K < ng && K >= klo) ? Ef[(long)i * ng + K] : make_double2(0.0, 0.0);
        }
        for (int e = tid; e < 64 * KC; e += 256) {
            const int cc = e / KC, k = e - cc * KC, v = v0 + cc, K = kc + k;
            double2 p = make_double2(0.0, 0.0);
            if (v < nv && K < ng) p = P[(long)v * ldp + K];
            sP[k][cc] = make_double2(p.x, -p.y);
        }
        __syncthreads();
#pragma unroll
        for (int k0 = 0; k0 < KC; k0 += 4) {
            double2 x[2], y[2];
#pragma unroll
            for (int rb = 0; rb < 2; rb++) x[rb] = sE[wr + rb * 16 + li][k0 + lk];
#pragma unroll
            for (int cb = 0; cb < 2; cb++) y[cb] = sP[k0 + lk][wc + cb * 16 + li];
#pragma unroll
            for (int rb = 0; rb < 2; rb++)
#pragma unroll
                for (int cb = 0; cb < 2; cb++) {
                    accR[rb][cb] = mfma64(x[rb].x, y[cb].x, accR[rb][cb]);
                    accR[rb][cb] = mfma64(-x[rb].y, y[cb].y, accR[rb][cb]);
                    accI[rb][cb] = mfma64(x[rb].x, y[cb].y, accI[rb][cb]);
                    accI[rb][cb] = mfma64(x[rb].y, y[cb].x, accI[rb][cb]);
                }
        }
        __syncthreads();
    }
    // result register r of lane (li, lk) holds row lk + 4 r, column li of a 16x16 block
    if constexpr (DIAG) {
#pragma unroll
        for (int cb = 0; cb < 2; cb++) {
            const int j = v0 + wc + cb * 16 + li;
            double2 s = make_double2(0.0, 0.0);
            if (j < nv) {
#pragma unroll
                for (int rb = 0; rb < 2; rb++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int i = rt0 + wr + rb * 16 + lk + 4 * r;
                        if (i >= klo && i < ng)
                            s = cadd(s, cmul(P[(long)j * ldp + i], make_double2(accR[rb][cb][r], accI[rb][cb][r])));
                    }
            }
            // the four lanes of column li (lk = 0..3) hold disjoint rows
            s.x += __shfl_xor(s.x, 16);
            s.y += __shfl_xor(s.y, 16);
            s.x += __shfl_xor(s.x, 32);
            s.y += __shfl_xor(s.y, 32);
            if (lk == 0) red[wave >> 1][wc + cb * 16 + li] = s;
        }
        __syncthreads();
        if (tid < 64 && v0 + tid < nv)
            out[((long)blockIdx.y * nfreq + f) * nv + v0 + tid] = cadd(red[0][tid], red[1][tid]);
    } else {
#pragma unroll
        for (int rb = 0; rb < 2; rb++)
#pragma unroll
            for (int cb = 0; cb < 2; cb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = rt0 + wr + rb * 16 + lk + 4 * r, j = v0 + wc + cb * 16 + li;
                    if (i < ng && j < nv)
                        out[((long)f * ng + i) * nv + j] = make_double2(accR[rb][cb][r], accI[rb][cb][r]);
                }
    }
}

__device__ __forceinline__ double2 block_sum(double2 s, double2 *red)
{
    const int tid = threadIdx.x;
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] = cadd(red[tid], red[tid + h]);
        __syncthreads();
    }
    return red[0];
}

// body[f][i][j] = sum_{G in [klo, ng)} P[i][G] T[f][G][j]; block per (i j, f)
__global__ void __launch_bounds__(256) k_wcross(int nwan, int ng, int klo, const double2 *__restrict__ P, long ldp,
                                                const double2 *__restrict__ T, double2 *__restrict__ body)
{
    __shared__ double2 red[256];
    const int i = blockIdx.x / nwan, j = blockIdx.x % nwan, f = blockIdx.y;
    double2 s = make_double2(0.0, 0.0);
    for (int G = klo + threadIdx.x; G < ng; G += 256)
        s = cadd(s, cmul(P[(long)i * ldp + G], T[((long)f * ng + G) * nwan + j]));
    s = block_sum(s, red);
    if (threadIdx.x == 0) body[((long)f * nwan + i) * nwan + j] = s;
}

// Gram sums of the densities: for output o (pair (a, b) = (o / nb, o % nb),
// or a = b = o when diag) bare[o] = sum_{G in [klo, ng)} P[a][G] conj(P[b][G])
// and tail[o] = the same over [ng, ng + ntail).
__global__ void __launch_bounds__(256) k_wgram(int nb, int diag, int ng, int klo, int ntail,
                                               const double2 *__restrict__ P, long ldp,
                                               double2 *__restrict__ bare, double2 *__restrict__ tail)
{
    __shared__ double2 red[256];
    const int o = blockIdx.x;
    const int a = diag ? o : o / nb, b = diag ? o : o % nb;
    const double2 *pa = P + (long)a * ldp, *pb = P + (long)b * ldp;
    double2 s = make_double2(0.0, 0.0), t = make_double2(0.0, 0.0);
    for (int G = klo + threadIdx.x; G < ng; G += 256) s = cadd(s, cmulc(pb[G], pa[G]));
    for (int G = ng + threadIdx.x; G < ng + ntail; G += 256) t = cadd(t, cmulc(pb[G], pa[G]));
    s = block_sum(s, red);
    __syncthreads();
    t = block_sum(t, red);
    if (threadIdx.x == 0) {
        tail[o] = t;
        bare[o] = cadd(s, t);
    }
}

// U[f][r][i][j], V[r][i][j] (+)= e^{-iq.R_r} pre (...); one thread per
// (f, r, i, j) of U, the f = 0 threads also write V
__global__ void k_wsum_u(int nfreq, int nR, int nwan, int ng, const int *__restrict__ R, double q1, double q2,
                         double q3, double pre, int head, double avg, const double2 *__restrict__ E,
                         const double2 *__restrict__ P, long ldp, const double2 *__restrict__ body,
                         const double2 *__restrict__ bare, const double2 *__restrict__ tail, int accumulate,
                         double2 *__restrict__ U, double2 *__restrict__ V)
{
    const long n2 = (long)nwan * nwan;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nfreq * nR * n2) return;
    const int f = (int)(t / (nR * n2));
    const long rem = t - (long)f * nR * n2;
    const int r = (int)(rem / n2);
    const int ij = (int)(rem - (long)r * n2), i = ij / nwan, j = ij % nwan;
    double s, c;
    sincospi(-2.0 * (q1 * R[3 * r] + q2 * R[3 * r + 1] + q3 * R[3 * r + 2]), &s, &c);
    const double2 ph = make_double2(pre * c, pre * s);
    double2 h = make_double2(0.0, 0.0);
    if (head) h = cscale(cmulc(P[(long)j * ldp], P[(long)i * ldp]), avg);   // A n_i(0) conj(n_j(0))
    if (U) {
        const double2 e00 = E[(long)f * ng * ng];
        double2 x = cadd(cadd(body[(long)f * n2 + ij], tail[ij]), cmul(e00, h));
        x = cmul(ph, x);
        U[t] = accumulate ? cadd(U[t], x) : x;
    }
    if (V && f == 0) {
        const double2 x = cmul(ph, cadd(bare[ij], h));
        const long o = (long)r * n2 + ij;
        V[o] = accumulate ? cadd(V[o], x) : x;
    }
}

// J[f][v], X[v] (+)= pre (...) for the vectors v0 .. v0 + nvc - 1 (one
// thread per (f, vector)); part [nrt][nfreq][nvc]
__global__ void k_wsum_x(int nfreq, long nvt, long v0, int nvc, int nrt, int ng, double pre, int head, double avg,
                         const double2 *__restrict__ E, const double2 *__restrict__ P, long ldp,
                         const double2 *__restrict__ part, const double2 *__restrict__ bare,
                         const double2 *__restrict__ tail, int accumulate, double2 *__restrict__ J,
                         double2 *__restrict__ X)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nfreq * nvc) return;
    const int f = (int)(t / nvc), lv = (int)(t - (long)f * nvc);
    double hv = 0.0;
    if (head) {
        const double2 n0 = P[(long)lv * ldp];
        hv = avg * (n0.x * n0.x + n0.y * n0.y);
    }
    if (J) {
        double2 s = tail[lv];
        for (int rt = 0; rt < nrt; rt++) s = cadd(s, part[((long)rt * nfreq + f) * nvc + lv]);
        s = cadd(s, cscale(E[(long)f * ng * ng], hv));
        s = cscale(s, pre);
        const long o = (long)f * nvt + v0 + lv;
        J[o] = accumulate ? cadd(J[o], s) : s;
    }
    if (X && f == 0) {
        const double2 x = cscale(make_double2(bare[lv].x + hv, bare[lv].y), pre);
        const long o = v0 + lv;
        X[o] = accumulate ? cadd(X[o], x) : x;
    }
}

unsigned blocks_for(long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void launch_xdens(hipStream_t s, const Geometry &g, const FftPlan plans[3], int nwan, const double *phi,
                  const double *centre_dev, const int *R_dev, long v0, int nvc, double2 *grids)
{
    const long nr = (long)g.fft[0] * g.fft[1] * g.fft[2];
    hipLaunchKernelGGL(k_xdens, dim3(blocks_for(nr * nvc, 256)), dim3(256), 0, s, nwan, g.fft[0], g.fft[1],
                       g.fft[2], phi, centre_dev, R_dev, v0, nvc, (double)g.iq[0] / g.kmesh[0],
                       (double)g.iq[1] / g.kmesh[1], (double)g.iq[2] / g.kmesh[2], grids);
    launch_fft3d(s, plans, g.fft, nvc, grids);
}

int wgemm_row_tiles(int ng) { return (ng + 63) / 64; }

void launch_wgemm(hipStream_t s, bool diag, int nfreq, int ng, int klo, int nv, const double2 *P, long ldp,
                  const double2 *E, double2 *out)
{
    if (nv == 0) return;
    const dim3 grid(blocks_for(nv, 64), (unsigned)wgemm_row_tiles(ng), (unsigned)nfreq);
    if (diag)
        hipLaunchKernelGGL(k_wgemm<true>, grid, dim3(256), 0, s, ng, klo, nv, nfreq, P, ldp, E, out);
    else
        hipLaunchKernelGGL(k_wgemm<false>, grid, dim3(256), 0, s, ng, klo, nv, nfreq, P, ldp, E, out);
}

void launch_wcross(hipStream_t s, int nfreq, int nwan, int ng, int klo, const double2 *P, long ldp,
                   const double2 *T, double2 *body)
{
    hipLaunchKernelGGL(k_wcross, dim3((unsigned)(nwan * nwan), (unsigned)nfreq), dim3(256), 0, s, nwan, ng, klo,
                       P, ldp, T, body);
}

void launch_wgram(hipStream_t s, int nout, int nb, bool diag, int ng, int klo, int ntail, const double2 *P,
                  long ldp, double2 *bare, double2 *tail)
{
    if (nout == 0) return;
    hipLaunchKernelGGL(k_wgram, dim3((unsigned)nout), dim3(256), 0, s, nb, (int)diag, ng, klo, ntail, P, ldp, bare,
                       tail);
}

void launch_wsum_u(hipStream_t s, const Geometry &g, int nfreq, int nR, int nwan, int ng, const int *R_dev,
                   double pre, bool head, double avg, const double2 *E, const double2 *P, long ldp,
                   const double2 *body, const double2 *bare, const double2 *tail, int accumulate, double2 *U,
                   double2 *V)
{
    const long n = (long)nfreq * nR * nwan * nwan;
    hipLaunchKernelGGL(k_wsum_u, dim3(blocks_for(n, 128)), dim3(128), 0, s, nfreq, nR, nwan, ng, R_dev,
                       (double)g.iq[0] / g.kmesh[0], (double)g.iq[1] / g.kmesh[1], (double)g.iq[2] / g.kmesh[2], pre,
                       (int)head, avg, E, P, ldp, body, bare, tail, accumulate, U, V);
}

void launch_wsum_x(hipStream_t s, int nfreq, long nvt, long v0, int nvc, int ng, double pre, bool head, double avg,
                   const double2 *E, const double2 *P, long ldp, const double2 *part, const double2 *bare,
                   const double2 *tail, int accumulate, double2 *J, double2 *X)
{
    const long n = (long)nfreq * nvc;
    hipLaunchKernelGGL(k_wsum_x, dim3(blocks_for(n, 128)), dim3(128), 0, s, nfreq, nvt, v0, nvc,
                       wgemm_row_tiles(ng), ng, pre, (int)head, avg, E, P, ldp, part, bare, tail, accumulate, J, X);
}

}  // namespace rp
