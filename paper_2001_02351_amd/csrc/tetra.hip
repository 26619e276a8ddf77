// Step a5: generalized-tetrahedron weights (Eqs. Xakqbk, tetrahedron, tak).
//
//   w_p(omega) = (2/Nk) (1 - T_{a,k+q} T_{b,k}) x_p(omega)
//   x_p(omega) = (1/6) sum_{T containing k} [ I_v(z) + I_v(z') ],
//   z = omega + i delta,  z' = -omega + i delta,
//
// where T runs over the 24 tetrahedra of the mesh that have k as a vertex
// (each mesh cell is cut into 6 tetrahedra around its (0,0,0)-(1,1,1)
// diagonal), v is k's vertex in T, and I_v(z) is the average over T of
// lambda_v / (z - e) for the linear interpolant e of the transition energies
// e = E_a(k+q) - E_b(k) at the four corners.  I_v(z) is the fourth divided
// difference of g(x) = (z-x)^3 log(z-x) with the node e_v doubled
// (Hermite-Genocchi).  With all four energies equal, x reduces to the
// textbook X(omega) of Eq. Xakqbk.
//
// Divided differences are evaluated top-down on sorted nodes: a set of
// nodes whose spread is at most a quarter of its distance to z is summed as a
// Taylor series of g about the set's midpoint; any other set is split by the
// recurrence (g[x1..xn] - g[x0..x(n-1)]) / (xn - x0), whose denominator is
// then large enough that nothing cancels.  This replaces the degeneracy
// thresholds delta_a, delta_r the paper's tetrahedron routine takes.
#include "fft_lds.h"

namespace rp {

namespace {

struct TetraTable {
    // for each of the 24 tetrahedra around a mesh point: neighbour codes
    // (d1+1)*9 + (d2+1)*3 + (d3+1) of its 4 corners and the corner that is k
    int nb[24][4];
    int self[24];
};

__constant__ TetraTable c_tetra;

__device__ __forceinline__ double2 clog_d(double2 w)
{
    return make_double2(log(hypot(w.x, w.y)), atan2(w.y, w.x));
}

__device__ __forceinline__ double2 cdiv_real(double2 a, double d) { return make_double2(a.x / d, a.y / d); }

__device__ __forceinline__ double2 crecip(double2 w)
{
    double s = 1.0 / (w.x * w.x + w.y * w.y);
    return make_double2(w.x * s, -w.y * s);
}

// sum_{m>=n} g^(m)(c)/m! * h_{m-n}(x_0-c, .., x_n-c) over the n+1 nodes x[a..a+n]
__device__ double2 dd_series(double2 z, const double *x, int a, int n)
{
    const double c = 0.5 * (x[a] + x[a + n]);
    const double2 w = make_double2(z.x - c, z.y);
    const double2 lw = clog_d(w);
    const double2 wi = crecip(w);
    double y[5], P[5];
#pragma unroll
    for (int i = 0; i < 5; i++) {
        y[i] = (i <= n) ? x[a + i] - c : 0.0;
        P[i] = 1.0;
    }
    // Taylor coefficients of g(x) = (z-x)^3 log(z-x) about c, with w = z - c:
    // m=0: w^3 L, 1: -(3w^2 L + w^2), 2: (6wL + 5w)/2, 3: -(6L + 11)/6,
    // m>=4: 6 / (m(m-1)(m-2)(m-3)) w^-(m-3)
    const double2 w2 = cmul(w, w);
    double2 lo[4];
    lo[0] = cmul(cmul(w2, w), lw);
    lo[1] = make_double2(-(3.0 * (w2.x * lw.x - w2.y * lw.y) + w2.x),
                         -(3.0 * (w2.x * lw.y + w2.y * lw.x) + w2.y));
    lo[2] = make_double2(0.5 * (6.0 * (w.x * lw.x - w.y * lw.y) + 5.0 * w.x),
                         0.5 * (6.0 * (w.x * lw.y + w.y * lw.x) + 5.0 * w.y));
    lo[3] = make_double2(-(6.0 * lw.x + 11.0) / 6.0, -(6.0 * lw.y) / 6.0);
    double2 wp = make_double2(1.0, 0.0);  // w^-(m-3) for m >= 4
    double2 sum = make_double2(0.0, 0.0);
    int quiet = 0;
    for (int m = n; m < n + 64; m++) {
        const int k = m - n;
        if (k > 0) {
            // raise P to degree k: h_k(y_0..y_i) = h_k(y_0..y_{i-1}) + y_i h_{k-1}(y_0..y_i)
            P[0] *= y[0];
#pragma unroll
            for (int i = 1; i < 5; i++)
                if (i <= n) P[i] = P[i - 1] + y[i] * P[i];
        }
        const double h = P[n];
        double2 coef;
        if (m < 4) {
            coef = lo[m];
        } else {
            wp = cmul(wp, wi);
            const double f = 6.0 / ((double)m * (m - 1) * (m - 2) * (m - 3));
            coef = make_double2(f * wp.x, f * wp.y);
        }
        const double2 t = make_double2(coef.x * h, coef.y * h);
        sum = cadd(sum, t);
        if (m >= 4) {
            const double tm = fabs(t.x) + fabs(t.y), sm = fabs(sum.x) + fabs(sum.y);
            if (tm <= 1e-18 * sm) {
                if (++quiet == 2) break;
            } else {
                quiet = 0;
            }
        }
    }
    return sum;
}

__device__ __forceinline__ double2 g_at(double2 z, double xv)
{
    const double2 w = make_double2(z.x - xv, z.y);
    return cmul(cmul(cmul(w, w), w), clog_d(w));
}

// fourth divided difference of g over five sorted nodes
__device__ double2 dd4_sorted(double2 z, const double *x)
{
    // entry (a, n) = g[x_a .. x_{a+n}] at slot id(a,n) = 5n - n(n-1)/2 + a
    bool need[15], ser[15];
    double2 val[15];
#pragma unroll
    for (int i = 0; i < 15; i++) { need[i] = false; ser[i] = false; }
    need[14] = true;
#pragma unroll
    for (int n = 4; n >= 1; n--) {
#pragma unroll
        for (int a = 0; a + n <= 4; a++) {
            const int id = 5 * n - n * (n - 1) / 2 + a;
            if (!need[id]) continue;
            const double spread = x[a + n] - x[a];
            const double c = 0.5 * (x[a] + x[a + n]);
            const double dz = hypot(z.x - c, z.y);
            if (4.0 * spread <= dz) {
                ser[id] = true;
            } else {
                const int lid = 5 * (n - 1) - (n - 1) * (n - 2) / 2 + a;
                need[lid] = true;
                need[lid + 1] = true;
            }
        }
    }
#pragma unroll
    for (int n = 0; n <= 4; n++) {
#pragma unroll
        for (int a = 0; a + n <= 4; a++) {
            const int id = 5 * n - n * (n - 1) / 2 + a;
            if (!need[id]) continue;
            if (n == 0) {
                val[id] = g_at(z, x[a]);
            } else if (ser[id]) {
                val[id] = dd_series(z, x, a, n);
            } else {
                const int lid = 5 * (n - 1) - (n - 1) * (n - 2) / 2 + a;
                val[id] = cdiv_real(csub(val[lid + 1], val[lid]), x[a + n] - x[a]);
            }
        }
    }
    return val[14];
}

// I_v(z) for corner energies e[4] (hartree)
__device__ double2 vertex_integral(double2 z, const double *e, int v)
{
    double x[5] = {e[0], e[1], e[2], e[3], e[v]};
    // sorting network on five keys
#define RP_CSWAP(i, j) { double lo_ = fmin(x[i], x[j]), hi_ = fmax(x[i], x[j]); x[i] = lo_; x[j] = hi_; }
    RP_CSWAP(0, 1) RP_CSWAP(3, 4) RP_CSWAP(2, 4) RP_CSWAP(2, 3) RP_CSWAP(0, 3)
    RP_CSWAP(0, 2) RP_CSWAP(1, 4) RP_CSWAP(1, 3) RP_CSWAP(1, 2)
#undef RP_CSWAP
    return dd4_sorted(z, x);
}

__device__ __forceinline__ int mesh_wrap(int n, int K) { return pmod(n, K); }

__global__ void __launch_bounds__(256)
k_weights(int K1, int K2, int K3, int q1, int q2, int q3, int nband, const double *E, const double *T,
          int o0, int nO, int e0, int nE, int k0, long npair, int nfreq, const double2 *freq,
          double delta, int mode, double2 *w)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npair * nfreq) return;
    const int f = (int)(t / npair);
    const long p = t - (long)f * npair;
    const int b = o0 + (int)(p % nO);
    const int a = e0 + (int)((p / nO) % nE);
    const int k = k0 + (int)(p / ((long)nO * nE));
    const int n1 = k / (K2 * K3), n2 = (k / K3) % K2, n3 = k % K3;
    const double ha = 1.0 / kHartreeEv;
    const double2 om = make_double2(freq[f].x * ha, freq[f].y * ha);
    const double dl = delta * ha;
    const double2 z = make_double2(om.x, om.y + dl);
    const double2 zp = make_double2(-om.x, -om.y + dl);
    const int kq = (mesh_wrap(n1 + q1, K1) * K2 + mesh_wrap(n2 + q2, K2)) * K3 + mesh_wrap(n3 + q3, K3);
    double2 x;
    if (mode == RP_W_SAMPLING) {
        const double e = (E[(long)kq * nband + a] - E[(long)k * nband + b]) * ha;
        x = cadd(crecip(make_double2(z.x - e, z.y)), crecip(make_double2(zp.x - e, zp.y)));
    } else {
        x = make_double2(0.0, 0.0);
        for (int tt = 0; tt < 24; tt++) {
            double e[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int code = c_tetra.nb[tt][v];
                const int d1 = code / 9 - 1, d2 = (code / 3) % 3 - 1, d3 = code % 3 - 1;
                const int m1 = n1 + d1, m2 = n2 + d2, m3 = n3 + d3;
                const int kv = (mesh_wrap(m1, K1) * K2 + mesh_wrap(m2, K2)) * K3 + mesh_wrap(m3, K3);
                const int kvq = (mesh_wrap(m1 + q1, K1) * K2 + mesh_wrap(m2 + q2, K2)) * K3 +
                                mesh_wrap(m3 + q3, K3);
                e[v] = (E[(long)kvq * nband + a] - E[(long)kv * nband + b]) * ha;
            }
            const int sv = c_tetra.self[tt];
            x = cadd(x, cadd(vertex_integral(z, e, sv), vertex_integral(zp, e, sv)));
        }
        x = cscale(x, 1.0 / 6.0);
    }
    double fac = 2.0 / (double)(K1 * K2 * K3);
    if (T) fac *= 1.0 - T[(long)kq * nband + a] * T[(long)k * nband + b];
    w[t] = cscale(x, fac);
}

TetraTable build_table()
{
    TetraTable tb{};
    int cnt = 0;
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int s = 0; s < 8; s++) {                 // k = cell corner + s
        const int so[3] = {(s >> 2) & 1, (s >> 1) & 1, s & 1};
        for (int pi = 0; pi < 6; pi++) {
            int corner[4][3] = {{0, 0, 0}};
            for (int v = 1; v < 4; v++) {
                for (int d = 0; d < 3; d++) corner[v][d] = corner[v - 1][d];
                corner[v][perms[pi][v - 1]] = 1;
            }
            int self = -1;
            for (int v = 0; v < 4; v++)
                if (corner[v][0] == so[0] && corner[v][1] == so[1] && corner[v][2] == so[2]) self = v;
            if (self < 0) continue;
            for (int v = 0; v < 4; v++) {
                const int d1 = corner[v][0] - so[0], d2 = corner[v][1] - so[1], d3 = corner[v][2] - so[2];
                tb.nb[cnt][v] = (d1 + 1) * 9 + (d2 + 1) * 3 + (d3 + 1);
            }
            tb.self[cnt] = self;
            cnt++;
        }
    }
    return tb;  // cnt == 24
}

}  // namespace

void launch_weights(hipStream_t s, const int kmesh[3], const int iq[3], int nband,
                    const double *E_eV, const double *T, int o0, int o1, int e0, int e1,
                    int k0, int k1, int nfreq, const double2 *freq_eV, double delta_eV,
                    int mode, double2 *w)
{
    static bool uploaded = false;
    static int uploaded_dev = -1;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (!uploaded || uploaded_dev != dev) {
        TetraTable tb = build_table();
        (void)hipMemcpyToSymbol(HIP_SYMBOL(c_tetra), &tb, sizeof(tb), 0, hipMemcpyHostToDevice);
        uploaded = true;
        uploaded_dev = dev;
    }
    const long npair = (long)(k1 - k0) * (e1 - e0) * (o1 - o0);
    const long tot = npair * nfreq;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, kmesh[0],
                       kmesh[1], kmesh[2], iq[0], iq[1], iq[2], nband, E_eV, T, o0, o1 - o0, e0,
                       e1 - e0, k0, npair, nfreq, freq_eV, delta_eV, mode, w);
}

}  // namespace rp
