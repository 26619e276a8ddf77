/*
 * FP64 CPU oracle for the constrained-RPA polarization path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code with the device library and is written from the paper's equations:
 *
 *   Eq. pak      plane-wave Bloch functions psi_{nk}
 *   Eq. ism      pair densities M^G_{ab}(k+q,k) = <psi_{a,k+q}| e^{i(q+G).r} |psi_{b,k}>
 *   Eq. Xakqbk   the resonant + antiresonant factor X(omega)
 *   Eq. tetrahedron / generalized tetrahedron integration of X over the BZ
 *   Eq. tak      the constrained-RPA factor (1 - T T)
 *   Eq. chi      chi_GG'(q,w) = (2/Nk) sum_k sum_a sum_b (1-TT) M^G M^G'* X
 *   Eq. epsGG    eps_GG' = delta_GG' - (4pi/Omega) chi_GG' / (|q+G||q+G'|)
 *   Eq. Wq       W_GG' = (4pi/Omega) eps^-1_GG' / (|q+G||q+G'|)
 *   Eqs. matrix_U, rhoiqG   the per-q direct (U-type) Wannier projection
 *
 * Conventions (readings of the paper; they are the same on the device side):
 *   - lattice rows a1,a2,a3 in bohr; reciprocal rows b_i with a_i.b_j = 2 pi d_ij
 *   - Gamma-centred k mesh k = n/K, mesh index (n1*K2 + n2)*K3 + n3
 *   - real-space grid r_j = (j1/N1, j2/N2, j3/N3) in fractional coordinates,
 *     stored [j1][j2][j3]
 *   - u_{nk}(r) = sum_G C_{Gn}(k) e^{iG.r} (the periodic part, no 1/sqrt(V))
 *   - k+q = k' + G0 with k' on the mesh; then
 *       M(G) = (1/N_r) sum_j conj(u_{a,k'}(r_j)) u_{b,k}(r_j) e^{i(G+G0).r_j}
 *     which equals the exact plane-wave convolution
 *       M(G) = sum_{G2} conj(C_{G2+G+G0,a}(k')) C_{G2,b}(k)
 *     whenever the grid is free of aliasing.
 *   - energies, frequencies and the broadening are in eV at the interface and
 *     converted to hartree with 1 Ha = 27.211386245988 eV.
 *   - complex arrays are interleaved (re,im) doubles (C99 double complex).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_PI 3.14159265358979323846
#define OR_HA_EV 27.211386245988

/* ------------------------------------------------------------------ */
/* geometry helpers                                                    */
/* ------------------------------------------------------------------ */

static int imod(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }
static int idiv_floor(int a, int n) { return (a - imod(a, n)) / n; }

static void recip_rows(const double *lat, double *b)
{
    /* b = 2 pi (A^-1)^T with A the matrix whose rows are a1,a2,a3 */
    const double *a = lat;
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                 a[2] * (a[3] * a[7] - a[4] * a[6]);
    double inv[9];
    inv[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    inv[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    inv[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    inv[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    inv[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    inv[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    inv[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    inv[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    inv[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) b[i * 3 + j] = 2.0 * OR_PI * inv[j * 3 + i];
}

static double cell_volume(const double *a)
{
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                 a[2] * (a[3] * a[7] - a[4] * a[6]);
    return fabs(det);
}

/* |q+G| for q = iq/K (fractional) and Miller index m */
static double qg_norm(const double *b, const int *kmesh, const int *iq, const int *m)
{
    double f[3], v[3] = {0, 0, 0};
    for (int a = 0; a < 3; a++) f[a] = (double)iq[a] / kmesh[a] + m[a];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) v[c] += f[a] * b[a * 3 + c];
    return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

/* e^{2 pi i n / N} evaluated from the reduced integer n mod N */
static cplx unit_root(long n, int N)
{
    long r = n % N;
    if (r < 0) r += N;
    double t = 2.0 * OR_PI * (double)r / (double)N;
    return cos(t) + I * sin(t);
}

/* table t[n] = e^{2 pi i n / N}, n < N (caller frees) */
static cplx *root_table(int N)
{
    cplx *t = malloc(sizeof(cplx) * N);
    for (int n = 0; n < N; n++) t[n] = unit_root(n, N);
    return t;
}

static cplx root_at(const cplx *t, long n, int N)
{
    long r = n % N;
    return t[r < 0 ? r + N : r];
}

/* ------------------------------------------------------------------ */
/* step a1: k+q on the mesh with its umklapp vector                    */
/* ------------------------------------------------------------------ */

void or_kq(const int *kmesh, const int *iq, int *kp, int *g0)
{
    int nk = kmesh[0] * kmesh[1] * kmesh[2];
    for (int k = 0; k < nk; k++) {
        int n[3] = {k / (kmesh[1] * kmesh[2]), (k / kmesh[2]) % kmesh[1], k % kmesh[2]};
        int s[3], r[3];
        for (int a = 0; a < 3; a++) {
            s[a] = n[a] + iq[a];
            r[a] = imod(s[a], kmesh[a]);
            g0[3 * k + a] = idiv_floor(s[a], kmesh[a]);
        }
        kp[k] = (r[0] * kmesh[1] + r[1]) * kmesh[2] + r[2];
    }
}

/* ------------------------------------------------------------------ */
/* step a2: u_{nk}(r_j) = sum_{G in S_psi(k)} C_G e^{iG.r_j}  (Eq. pak)  */
/* ------------------------------------------------------------------ */

/* plain triple sum: every grid point, every plane wave */
void or_u_direct(const int *fft, int npw, const int *miller, const cplx *c, cplx *u)
{
    int N1 = fft[0], N2 = fft[1], N3 = fft[2];
    long nr = (long)N1 * N2 * N3;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < nr; j++) {
        int j1 = (int)(j / ((long)N2 * N3)), j2 = (int)((j / N3) % N2), j3 = (int)(j % N3);
        cplx s = 0;
        for (int g = 0; g < npw; g++) {
            const int *m = miller + 3 * g;
            s += c[g] * unit_root((long)m[0] * j1, N1) * unit_root((long)m[1] * j2, N2) *
                 unit_root((long)m[2] * j3, N3);
        }
        u[j] = s;
    }
}

/* the same sum, with e^{iG.r} = prod_a e^{2 pi i m_a j_a / N_a} summed one
 * axis at a time over the Miller box that holds the sphere */
void or_u_separable(const int *fft, int npw, const int *miller, const cplx *c, cplx *u)
{
    int N[3] = {fft[0], fft[1], fft[2]};
    int lo[3], hi[3], L[3];
    for (int a = 0; a < 3; a++) { lo[a] = 1 << 30; hi[a] = -(1 << 30); }
    for (int g = 0; g < npw; g++)
        for (int a = 0; a < 3; a++) {
            if (miller[3 * g + a] < lo[a]) lo[a] = miller[3 * g + a];
            if (miller[3 * g + a] > hi[a]) hi[a] = miller[3 * g + a];
        }
    if (npw == 0) { memset(u, 0, sizeof(cplx) * (size_t)N[0] * N[1] * N[2]); return; }
    for (int a = 0; a < 3; a++) L[a] = hi[a] - lo[a] + 1;
    cplx *tw[3];
    for (int a = 0; a < 3; a++) tw[a] = root_table(N[a]);
    cplx *box = calloc((size_t)L[0] * L[1] * L[2], sizeof(cplx));
    for (int g = 0; g < npw; g++) {
        const int *m = miller + 3 * g;
        box[((size_t)(m[0] - lo[0]) * L[1] + (m[1] - lo[1])) * L[2] + (m[2] - lo[2])] += c[g];
    }
    /* over m3: t1[m1][m2][j3] */
    cplx *t1 = calloc((size_t)L[0] * L[1] * N[2], sizeof(cplx));
    for (int a1 = 0; a1 < L[0]; a1++)
        for (int a2 = 0; a2 < L[1]; a2++)
            for (int j3 = 0; j3 < N[2]; j3++) {
                cplx s = 0;
                for (int a3 = 0; a3 < L[2]; a3++)
                    s += box[((size_t)a1 * L[1] + a2) * L[2] + a3] * root_at(tw[2], (long)(a3 + lo[2]) * j3, N[2]);
                t1[((size_t)a1 * L[1] + a2) * N[2] + j3] = s;
            }
    /* over m2: t2[m1][j2][j3] */
    cplx *t2 = calloc((size_t)L[0] * N[1] * N[2], sizeof(cplx));
    for (int a1 = 0; a1 < L[0]; a1++)
        for (int j2 = 0; j2 < N[1]; j2++)
            for (int j3 = 0; j3 < N[2]; j3++) {
                cplx s = 0;
                for (int a2 = 0; a2 < L[1]; a2++)
                    s += t1[((size_t)a1 * L[1] + a2) * N[2] + j3] * root_at(tw[1], (long)(a2 + lo[1]) * j2, N[1]);
                t2[((size_t)a1 * N[1] + j2) * N[2] + j3] = s;
            }
    /* over m1 */
    for (int j1 = 0; j1 < N[0]; j1++)
        for (int j2 = 0; j2 < N[1]; j2++)
            for (int j3 = 0; j3 < N[2]; j3++) {
                cplx s = 0;
                for (int a1 = 0; a1 < L[0]; a1++)
                    s += t2[((size_t)a1 * N[1] + j2) * N[2] + j3] * root_at(tw[0], (long)(a1 + lo[0]) * j1, N[0]);
                u[((size_t)j1 * N[1] + j2) * N[2] + j3] = s;
            }
    free(box); free(t1); free(t2);
    for (int a = 0; a < 3; a++) free(tw[a]);
}

/* u-grids of nb bands sharing one Miller list (bands in parallel) */
void or_u_batch(const int *fft, int nb, int npw, const int *miller, const cplx *c, long cstride, cplx *u)
{
    long nr = (long)fft[0] * fft[1] * fft[2];
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; b++) or_u_separable(fft, npw, miller, c + (long)b * cstride, u + (long)b * nr);
}

/* ------------------------------------------------------------------ */
/* steps a3-a4: pair densities (Eq. ism)                               */
/* ------------------------------------------------------------------ */

/* plain direct DFT of rho_j = conj(ua_j) ub_j over every grid point */
void or_pair_direct(const int *fft, const cplx *ua, const cplx *ub, const int *g0,
                    int ng, const int *gsph, cplx *M)
{
    int N1 = fft[0], N2 = fft[1], N3 = fft[2];
    long nr = (long)N1 * N2 * N3;
#pragma omp parallel for schedule(static)
    for (int g = 0; g < ng; g++) {
        long m1 = gsph[3 * g] + g0[0], m2 = gsph[3 * g + 1] + g0[1], m3 = gsph[3 * g + 2] + g0[2];
        cplx s = 0;
        for (long j = 0; j < nr; j++) {
            int j1 = (int)(j / ((long)N2 * N3)), j2 = (int)((j / N3) % N2), j3 = (int)(j % N3);
            s += conj(ua[j]) * ub[j] * unit_root(m1 * j1, N1) * unit_root(m2 * j2, N2) *
                 unit_root(m3 * j3, N3);
        }
        M[g] = s / (double)nr;
    }
}

/* the same sum done one axis at a time over the box of needed (G+G0) */
void or_pair_separable(const int *fft, const cplx *ua, const cplx *ub, const int *g0,
                       int ng, const int *gsph, cplx *M)
{
    int N[3] = {fft[0], fft[1], fft[2]};
    long nr = (long)N[0] * N[1] * N[2];
    int lo[3], hi[3], L[3];
    for (int a = 0; a < 3; a++) { lo[a] = 1 << 30; hi[a] = -(1 << 30); }
    for (int g = 0; g < ng; g++)
        for (int a = 0; a < 3; a++) {
            int v = gsph[3 * g + a] + g0[a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    if (ng == 0) return;
    for (int a = 0; a < 3; a++) L[a] = hi[a] - lo[a] + 1;
    cplx *tw[3];
    for (int a = 0; a < 3; a++) tw[a] = root_table(N[a]);
    cplx *rho = malloc(sizeof(cplx) * nr);
    for (long j = 0; j < nr; j++) rho[j] = conj(ua[j]) * ub[j];
    /* over j3: t1[j1][j2][m3] */
    cplx *t1 = malloc(sizeof(cplx) * (size_t)N[0] * N[1] * L[2]);
    for (int j1 = 0; j1 < N[0]; j1++)
        for (int j2 = 0; j2 < N[1]; j2++)
            for (int a3 = 0; a3 < L[2]; a3++) {
                cplx s = 0;
                for (int j3 = 0; j3 < N[2]; j3++)
                    s += rho[((size_t)j1 * N[1] + j2) * N[2] + j3] * root_at(tw[2], (long)(a3 + lo[2]) * j3, N[2]);
                t1[((size_t)j1 * N[1] + j2) * L[2] + a3] = s;
            }
    /* over j2: t2[j1][m2][m3] */
    cplx *t2 = malloc(sizeof(cplx) * (size_t)N[0] * L[1] * L[2]);
    for (int j1 = 0; j1 < N[0]; j1++)
        for (int a2 = 0; a2 < L[1]; a2++)
            for (int a3 = 0; a3 < L[2]; a3++) {
                cplx s = 0;
                for (int j2 = 0; j2 < N[1]; j2++)
                    s += t1[((size_t)j1 * N[1] + j2) * L[2] + a3] * root_at(tw[1], (long)(a2 + lo[1]) * j2, N[1]);
                t2[((size_t)j1 * L[1] + a2) * L[2] + a3] = s;
            }
    /* over j1, only at the requested vectors */
    for (int g = 0; g < ng; g++) {
        int a1 = gsph[3 * g] + g0[0] - lo[0];
        int a2 = gsph[3 * g + 1] + g0[1] - lo[1];
        int a3 = gsph[3 * g + 2] + g0[2] - lo[2];
        cplx s = 0;
        for (int j1 = 0; j1 < N[0]; j1++)
            s += t2[((size_t)j1 * L[1] + a2) * L[2] + a3] * root_at(tw[0], (long)(a1 + lo[0]) * j1, N[0]);
        M[g] = s / (double)nr;
    }
    free(rho); free(t1); free(t2);
    for (int a = 0; a < 3; a++) free(tw[a]);
}

/* all pairs (a, b) of nA grids ua (at k') and nB grids ub (at k):
 * M[a][b][g], pairs in parallel */
void or_pair_batch(const int *fft, int nA, const cplx *ua, int nB, const cplx *ub, const int *g0,
                   int ng, const int *gsph, cplx *M)
{
    long nr = (long)fft[0] * fft[1] * fft[2];
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int a = 0; a < nA; a++)
        for (int b = 0; b < nB; b++)
            or_pair_separable(fft, ua + (long)a * nr, ub + (long)b * nr, g0, ng, gsph,
                              M + ((long)a * nB + b) * ng);
}

/* exact plane-wave form: M(G) = sum_{G2 in S_b} conj(C_a[G2+G+G0]) C_b[G2] */
void or_pair_conv(int npw_a, const int *miller_a, const cplx *ca, int npw_b,
                  const int *miller_b, const cplx *cb, const int *g0, int ng,
                  const int *gsph, cplx *M)
{
#pragma omp parallel for schedule(static)
    for (int g = 0; g < ng; g++) {
        cplx s = 0;
        for (int i = 0; i < npw_b; i++) {
            int t[3];
            for (int a = 0; a < 3; a++) t[a] = miller_b[3 * i + a] + gsph[3 * g + a] + g0[a];
            for (int j = 0; j < npw_a; j++)
                if (miller_a[3 * j] == t[0] && miller_a[3 * j + 1] == t[1] &&
                    miller_a[3 * j + 2] == t[2]) {
                    s += conj(ca[j]) * cb[i];
                    break;
                }
        }
        M[g] = s;
    }
}

/* ------------------------------------------------------------------ */
/* step a5: generalized-tetrahedron weights                            */
/* ------------------------------------------------------------------ */
/*
 * For a tetrahedron with vertex transition energies e_1..e_4 and a linear
 * interpolant e(k) = sum_i lambda_i e_i, the vertex integral is
 *     I_i(z) = < lambda_i / (z - e) >_T      (average over the tetrahedron)
 * By the Hermite-Genocchi formula this equals the fourth-order divided
 * difference of g(x) = (z-x)^3 ln(z-x) over the nodes (e_i, e_i, e_j, e_k, e_l)
 * (the repeated node carries the lambda_i weight; g'''' = 6/(z-x)).
 * A consistent branch of ln is enough: a branch jump adds a cubic, which the
 * fourth-order difference removes.
 *
 * Divided differences are taken on sorted nodes.  Every entry g[x_a..x_b] of
 * the table is computed either by the recurrence
 *     (g[x_{a+1}..x_b] - g[x_a..x_{b-1}]) / (x_b - x_a)
 * or, when the nodes x_a..x_b lie within a quarter of their distance to the
 * singularity z, by the Taylor series about their midpoint c
 *     g[x_a..x_b] = sum_{m>=n} g^(m)(c)/m! h_{m-n}(x_a-c, .., x_b-c)
 * (n = b-a, h the complete homogeneous symmetric polynomial), which is exact
 * for coincident nodes and avoids cancellation for near-degenerate ones.
 * This plays the role of the paper's degeneracy thresholds delta_a, delta_r.
 */

/* Taylor coefficient g^(m)(c)/m! for g(x) = (z-x)^3 ln(z-x), w = z-c */
static cplx gtaylor(int m, cplx w, cplx lw)
{
    switch (m) {
    case 0: return w * w * w * lw;
    case 1: return -(3.0 * w * w * lw + w * w);
    case 2: return (6.0 * w * lw + 5.0 * w) / 2.0;
    case 3: return -(6.0 * lw + 11.0) / 6.0;
    default: {
        /* 6 (m-4)! / (m! w^(m-3)) = 6 / (m (m-1) (m-2) (m-3) w^(m-3)) */
        cplx p = 1.0;
        for (int t = 0; t < m - 3; t++) p *= w;
        return 6.0 / ((double)m * (m - 1) * (m - 2) * (m - 3) * p);
    }
    }
}

static cplx dd_taylor(cplx z, const double *x, int n /* order: n+1 nodes */)
{
    double c = 0.5 * (x[0] + x[n]);
    double y[5];
    for (int i = 0; i <= n; i++) y[i] = x[i] - c;
    cplx w = z - c, lw = clog(w);
    enum { KMAX = 80 };
    /* h[k] = complete homogeneous symmetric polynomial of degree k in y[0..n] */
    double h[KMAX + 1];
    for (int k = 0; k <= KMAX; k++) h[k] = 0.0;
    h[0] = 1.0;
    for (int i = 0; i <= n; i++)
        for (int k = 1; k <= KMAX; k++) h[k] += y[i] * h[k - 1];
    cplx s = 0;
    int small = 0;
    for (int m = n; m <= n + KMAX; m++) {
        cplx t = gtaylor(m, w, lw) * h[m - n];
        s += t;
        if (cabs(t) <= 1e-18 * cabs(s)) { if (++small >= 3) break; } else small = 0;
    }
    return s;
}

static cplx g_at(cplx z, double x)
{
    cplx w = z - x;
    return w * w * w * clog(w);
}

/* fourth-order divided difference of g over 5 nodes (any order, may repeat) */
cplx or_dd4(cplx z, const double *nodes)
{
    double x[5];
    for (int i = 0; i < 5; i++) x[i] = nodes[i];
    for (int i = 1; i < 5; i++)               /* insertion sort */
        for (int j = i; j > 0 && x[j] < x[j - 1]; j--) { double t = x[j]; x[j] = x[j - 1]; x[j - 1] = t; }
    cplx t[5][5];                             /* t[a][n] = g[x_a .. x_{a+n}] */
    for (int n = 0; n <= 4; n++)
        for (int a = 0; a + n <= 4; a++) {
            double spread = x[a + n] - x[a];
            double c = 0.5 * (x[a] + x[a + n]);
            if (n == 0) t[a][0] = g_at(z, x[a]);
            else if (spread <= 0.25 * cabs(z - c)) t[a][n] = dd_taylor(z, x + a, n);
            else t[a][n] = (t[a + 1][n - 1] - t[a][n - 1]) / spread;
        }
    return t[0][4];
}

/* I_i(z) = < lambda_i / (z - e) >_T */
cplx or_vertex_integral(cplx z, const double *e, int i)
{
    double nodes[5] = {e[i], e[0], e[1], e[2], e[3]};
    return or_dd4(z, nodes);
}

/* < 1/(z-e) >_T by the scalar closed form (distinct energies only) */
cplx or_tetra_scalar(cplx z, const double *e)
{
    cplx s = 0;
    for (int j = 0; j < 4; j++) {
        double p = 1.0;
        for (int k = 0; k < 4; k++)
            if (k != j) p *= (e[j] - e[k]);
        cplx w = z - e[j];
        s += w * w * clog(w) / p;
    }
    return -3.0 * s;
}

/* the six tetrahedra of a mesh subcell that share its (0,0,0)-(1,1,1)
 * diagonal: for each ordering (s0,s1,s2) of the axes the corners are
 * 0, e_s0, e_s0+e_s1, e_s0+e_s1+e_s2 */
static const int OR_PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static void tetra_corners(int t, int corner[4][3])
{
    for (int v = 0; v < 4; v++)
        for (int a = 0; a < 3; a++) corner[v][a] = 0;
    for (int v = 1; v < 4; v++) {
        for (int a = 0; a < 3; a++) corner[v][a] = corner[v - 1][a];
        corner[v][OR_PERM[t][v - 1]] = 1;
    }
}

static int mesh_index(const int *kmesh, const int *n)
{
    int r[3];
    for (int a = 0; a < 3; a++) r[a] = imod(n[a], kmesh[a]);
    return (r[0] * kmesh[1] + r[1]) * kmesh[2] + r[2];
}

/*
 * w[f][p] = (2/Nk) (1 - T_{a,k+q} T_{b,k}) x_p(omega_f) for the pairs
 * p = ((k-k0)*(e1-e0) + (a-e0))*(o1-o0) + (b-o0)   (b fastest)
 * mode 0: generalized tetrahedron; mode 1: sampling x = X(E_a(k+q)-E_b(k)).
 * Returns 0, or -1 on bad arguments.
 */
int or_weights(const int *kmesh, const int *iq, int nband, const double *E_eV,
               const double *T, int o0, int o1, int e0, int e1, int k0, int k1,
               int nfreq, const cplx *freq_eV, double delta_eV, int mode, cplx *w)
{
    int nk = kmesh[0] * kmesh[1] * kmesh[2];
    int nO = o1 - o0, nE = e1 - e0, nK = k1 - k0;
    if (nO < 0 || nE < 0 || nK < 0 || k0 < 0 || k1 > nk) return -1;
    long npair = (long)nK * nE * nO;
    int *kp = malloc(sizeof(int) * nk), *g0 = malloc(sizeof(int) * 3 * nk);
    or_kq(kmesh, iq, kp, g0);
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int f = 0; f < nfreq; f++)
        for (long p = 0; p < npair; p++) {
            int b = o0 + (int)(p % nO);
            int a = e0 + (int)((p / nO) % nE);
            int k = k0 + (int)(p / ((long)nO * nE));
            cplx om = freq_eV[f] / OR_HA_EV;
            double dl = delta_eV / OR_HA_EV;
            cplx z = om + I * dl, zp = -om + I * dl;
            cplx x = 0;
            if (mode == 1) {
                double e = (E_eV[(long)kp[k] * nband + a] - E_eV[(long)k * nband + b]) / OR_HA_EV;
                x = 1.0 / (z - e) + 1.0 / (zp - e);
            } else {
                int n[3] = {k / (kmesh[1] * kmesh[2]), (k / kmesh[2]) % kmesh[1], k % kmesh[2]};
                for (int s = 0; s < 8; s++) {
                    int off[3] = {(s >> 2) & 1, (s >> 1) & 1, s & 1}; /* k = corner + off */
                    for (int t = 0; t < 6; t++) {
                        int cr[4][3];
                        tetra_corners(t, cr);
                        int iv = -1;
                        for (int v = 0; v < 4; v++)
                            if (cr[v][0] == off[0] && cr[v][1] == off[1] && cr[v][2] == off[2]) iv = v;
                        if (iv < 0) continue;
                        double e[4];
                        for (int v = 0; v < 4; v++) {
                            int m[3], mq[3];
                            for (int c = 0; c < 3; c++) {
                                m[c] = n[c] - off[c] + cr[v][c];
                                mq[c] = m[c] + iq[c];
                            }
                            int kv = mesh_index(kmesh, m), kvq = mesh_index(kmesh, mq);
                            e[v] = (E_eV[(long)kvq * nband + a] - E_eV[(long)kv * nband + b]) / OR_HA_EV;
                        }
                        x += or_vertex_integral(z, e, iv) + or_vertex_integral(zp, e, iv);
                    }
                }
                x /= 6.0;
            }
            double crpa = 1.0;
            if (T) crpa = 1.0 - T[(long)kp[k] * nband + a] * T[(long)k * nband + b];
            w[(long)f * npair + p] = (2.0 / nk) * crpa * x;
        }
    free(kp); free(g0);
    return 0;
}

/* ------------------------------------------------------------------ */
/* step a6: chi_GG'(w) = sum_p w_p M_p(G) conj(M_p(G'))   (Eq. chi)      */
/* ------------------------------------------------------------------ */

void or_chi0(long npair, int ng, const cplx *M, int nfreq, const cplx *w, cplx *chi)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int f = 0; f < nfreq; f++)
        for (int g = 0; g < ng; g++)
            for (int h = 0; h < ng; h++) {
                /* compensated (Kahan) summation of real and imaginary parts */
                double sr = 0, cr = 0, si = 0, ci = 0;
                for (long p = 0; p < npair; p++) {
                    cplx t = w[(long)f * npair + p] * M[p * ng + g] * conj(M[p * ng + h]);
                    double yr = creal(t) - cr, tr = sr + yr;
                    cr = (tr - sr) - yr; sr = tr;
                    double yi = cimag(t) - ci, ti = si + yi;
                    ci = (ti - si) - yi; si = ti;
                }
                chi[((long)f * ng + g) * ng + h] = sr + I * si;
            }
}

/* ------------------------------------------------------------------ */
/* steps a7-a9: eps, eps^-1, W   (Eqs. epsGG, Wq)                      */
/* ------------------------------------------------------------------ */

/* Gauss-Jordan inversion with partial pivoting; returns 0 or -2 if singular */
int or_invert(int n, const cplx *A, cplx *Ainv)
{
    cplx *a = malloc(sizeof(cplx) * (size_t)n * n);
    memcpy(a, A, sizeof(cplx) * (size_t)n * n);
    for (long i = 0; i < (long)n * n; i++) Ainv[i] = 0;
    for (int i = 0; i < n; i++) Ainv[(long)i * n + i] = 1;
    int rc = 0;
    for (int c = 0; c < n; c++) {
        int piv = c;
        double best = cabs(a[(long)c * n + c]);
        for (int r = c + 1; r < n; r++)
            if (cabs(a[(long)r * n + c]) > best) { best = cabs(a[(long)r * n + c]); piv = r; }
        if (best == 0.0) { rc = -2; break; }
        if (piv != c)
            for (int j = 0; j < n; j++) {
                cplx t = a[(long)c * n + j]; a[(long)c * n + j] = a[(long)piv * n + j]; a[(long)piv * n + j] = t;
                t = Ainv[(long)c * n + j]; Ainv[(long)c * n + j] = Ainv[(long)piv * n + j]; Ainv[(long)piv * n + j] = t;
            }
        cplx d = 1.0 / a[(long)c * n + c];
        for (int j = 0; j < n; j++) { a[(long)c * n + j] *= d; Ainv[(long)c * n + j] *= d; }
#pragma omp parallel for schedule(static) if (n >= 384)
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            cplx f = a[(long)r * n + c];
            if (f == 0) continue;
            for (int j = 0; j < n; j++) {
                a[(long)r * n + j] -= f * a[(long)c * n + j];
                Ainv[(long)r * n + j] -= f * Ainv[(long)c * n + j];
            }
        }
    }
    free(a);
    return rc;
}

/* eps = I - v^1/2 chi v^1/2 (v^1/2_G = sqrt(4pi/Omega)/|q+G|), eps^-1, and
 * W = v^1/2 eps^-1 v^1/2 in eV.  eps_out / eps_inv / W may be NULL.
 * Returns 0, or -2 if some eps(w) is singular. */
int or_screen(const double *lat, const int *kmesh, const int *iq, int ng, const int *gsph,
              int nfreq, const cplx *chi, cplx *eps_out, cplx *eps_inv, cplx *W)
{
    double b[9];
    recip_rows(lat, b);
    double vol = cell_volume(lat);
    double *vs = malloc(sizeof(double) * ng);
    for (int g = 0; g < ng; g++) vs[g] = sqrt(4.0 * OR_PI / vol) / qg_norm(b, kmesh, iq, gsph + 3 * g);
    cplx *eps = malloc(sizeof(cplx) * (size_t)ng * ng);
    cplx *inv = malloc(sizeof(cplx) * (size_t)ng * ng);
    int rc = 0;
    for (int f = 0; f < nfreq && rc == 0; f++) {
        const cplx *c = chi + (size_t)f * ng * ng;
        for (int g = 0; g < ng; g++)
            for (int h = 0; h < ng; h++)
                eps[(long)g * ng + h] = (g == h ? 1.0 : 0.0) - vs[g] * c[(long)g * ng + h] * vs[h];
        if (eps_out) memcpy(eps_out + (size_t)f * ng * ng, eps, sizeof(cplx) * (size_t)ng * ng);
        rc = or_invert(ng, eps, inv);
        if (eps_inv) memcpy(eps_inv + (size_t)f * ng * ng, inv, sizeof(cplx) * (size_t)ng * ng);
        if (W)
            for (int g = 0; g < ng; g++)
                for (int h = 0; h < ng; h++)
                    W[((size_t)f * ng + g) * ng + h] = OR_HA_EV * vs[g] * inv[(long)g * ng + h] * vs[h];
    }
    free(vs); free(eps); free(inv);
    return rc;
}

/* ------------------------------------------------------------------ */
/* step a10: Wannier densities and the projected interaction           */
/* ------------------------------------------------------------------ */
/*
 * rho_i(G) = ntilde_i(q+G) / |q+G| with
 *     ntilde_i(Q) = (Omega/N_r) sum_j phi_i(r_j)^2 e^{iQ.rt_ij},
 * rt_ij = R_i + (r_j - R_i wrapped to the minimum image), so that the
 * density of the home-cell orbital carries the Bloch phase of its true
 * position (Eq. rhoiqG read as the density of orbital i).
 * direct = 1: plain sum over grid points; 0: the same sum one axis at a time.
 */
void or_wannier_rho(const double *lat, const int *fft, const int *kmesh, const int *iq,
                    int nwan, const double *phi, const double *centre_frac, int nglist,
                    const int *glist, int direct, cplx *rho)
{
    int N[3] = {fft[0], fft[1], fft[2]};
    long nr = (long)N[0] * N[1] * N[2];
    double b[9];
    recip_rows(lat, b);
    double vol = cell_volume(lat);
    double qf[3];
    for (int a = 0; a < 3; a++) qf[a] = (double)iq[a] / kmesh[a];
    for (int i = 0; i < nwan; i++) {
        const double *ph = phi + (size_t)i * nr;
        const double *R = centre_frac + 3 * i;
        /* f_j = n(r_j) e^{i q.rt_j} and the integer image shift of r_j */
        cplx *f = malloc(sizeof(cplx) * nr);
        for (long j = 0; j < nr; j++) {
            int jj[3] = {(int)(j / ((long)N[1] * N[2])), (int)((j / N[2]) % N[1]), (int)(j % N[2])};
            double rt[3];
            for (int a = 0; a < 3; a++) {
                double d = (double)jj[a] / N[a] - R[a];
                d -= floor(d + 0.5);
                rt[a] = R[a] + d;   /* fractional position of the true image */
            }
            double ph_q = 2.0 * OR_PI * (qf[0] * rt[0] + qf[1] * rt[1] + qf[2] * rt[2]);
            f[j] = ph[j] * ph[j] * (cos(ph_q) + I * sin(ph_q));
        }
        if (direct) {
#pragma omp parallel for schedule(static)
            for (int g = 0; g < nglist; g++) {
                const int *m = glist + 3 * g;
                cplx s = 0;
                for (long j = 0; j < nr; j++) {
                    int jj[3] = {(int)(j / ((long)N[1] * N[2])), (int)((j / N[2]) % N[1]), (int)(j % N[2])};
                    s += f[j] * unit_root((long)m[0] * jj[0], N[0]) * unit_root((long)m[1] * jj[1], N[1]) *
                         unit_root((long)m[2] * jj[2], N[2]);
                }
                rho[(size_t)i * nglist + g] = s * (vol / nr) / qg_norm(b, kmesh, iq, m);
            }
        } else {
            int zero[3] = {0, 0, 0};
            /* or_pair_separable computes (1/N_r) sum_j conj(ua) ub e^{iG.r_j};
             * with ua = 1 and ub = f it is the sum needed here */
            cplx *one = malloc(sizeof(cplx) * nr);
            for (long j = 0; j < nr; j++) one[j] = 1.0;
            cplx *tmp = malloc(sizeof(cplx) * nglist);
            or_pair_separable(fft, one, f, zero, nglist, glist, tmp);
            for (int g = 0; g < nglist; g++)
                rho[(size_t)i * nglist + g] = tmp[g] * (double)nr * (vol / nr) /
                                              qg_norm(b, kmesh, iq, glist + 3 * g);
            free(one); free(tmp);
        }
        free(f);
    }
}

/* W_ij(w) = HA_EV * (4pi/(Omega Nq)) [ sum_{G,G' in S_eps} rho_i(G) eps^-1_GG' conj(rho_j(G'))
 *                                     + sum_{G in tail} rho_i(G) conj(rho_j(G)) ]
 * rho_eps [nwan][ng], rho_tail [nwan][ntail], eps_inv [nfreq][ng][ng] */
void or_wannier_W(const double *lat, const int *kmesh, int nwan, int ng, const cplx *rho_eps,
                  int ntail, const cplx *rho_tail, int nfreq, const cplx *eps_inv, cplx *Wij)
{
    double vol = cell_volume(lat);
    int nq = kmesh[0] * kmesh[1] * kmesh[2];
    double pre = OR_HA_EV * 4.0 * OR_PI / (vol * nq);
#pragma omp parallel for collapse(3) schedule(static)
    for (int f = 0; f < nfreq; f++)
        for (int i = 0; i < nwan; i++)
            for (int j = 0; j < nwan; j++) {
                const cplx *e = eps_inv + (size_t)f * ng * ng;
                cplx s = 0;
                for (int g = 0; g < ng; g++) {
                    cplx r = 0;
                    for (int h = 0; h < ng; h++) r += e[(long)g * ng + h] * conj(rho_eps[(size_t)j * ng + h]);
                    s += rho_eps[(size_t)i * ng + g] * r;
                }
                for (int g = 0; g < ntail; g++)
                    s += rho_tail[(size_t)i * ntail + g] * conj(rho_tail[(size_t)j * ntail + g]);
                Wij[((size_t)f * nwan + i) * nwan + j] = pre * s;
            }
}

/* pointer-argument forms for foreign-function callers */
void or_dd4_py(const cplx *z, const double *nodes, cplx *out) { *out = or_dd4(*z, nodes); }
void or_vertex_integral_py(const cplx *z, const double *e, int i, cplx *out)
{
    *out = or_vertex_integral(*z, e, i);
}
void or_tetra_scalar_py(const cplx *z, const double *e, cplx *out) { *out = or_tetra_scalar(*z, e); }
