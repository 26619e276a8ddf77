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
// nodes whose deviation from its median node is at most a quarter of that
// node's distance to z is summed as a Taylor series of g about the median
// node; any other set is split by the recurrence
// (g[x1..xn] - g[x0..x(n-1)]) / (xn - x0), whose denominator is then large
// enough that nothing cancels.  This replaces the degeneracy thresholds
// delta_a, delta_r the paper's tetrahedron routine takes.  Every series is
// centred on a node, so the only logarithms are log(z - e_j) at the 15
// distinct corners of the 24 tetrahedra around k: they are computed once per
// (pair, frequency) and kept in LDS, and each tetrahedron is pure arithmetic.
#include "fft_lds.h"

namespace rp {

namespace {

// The 24 tetrahedra around a mesh point (each mesh cell cut into 6 around its
// (0,0,0)-(1,1,1) diagonal): corners as slots into the 15 distinct
// neighbours, neighbour offsets as codes (d1+1)*9 + (d2+1)*3 + (d3+1).
struct TetraTable {
    int slot[24][4];
    int nbr[15];
    int self;   // slot of k itself (code 13)
    int ntet, nnbr;
};

constexpr TetraTable make_tetra_table()
{
    TetraTable tb{};
    int codes[24][4] = {};
    int cnt = 0;
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int s = 0; s < 8; s++) {                 // k = cell corner + s
        const int so[3] = {(s >> 2) & 1, (s >> 1) & 1, s & 1};
        for (int pi = 0; pi < 6; pi++) {
            int corner[4][3] = {};
            for (int v = 1; v < 4; v++) {
                for (int d = 0; d < 3; d++) corner[v][d] = corner[v - 1][d];
                corner[v][perms[pi][v - 1]] = 1;
            }
            bool has = false;
            for (int v = 0; v < 4; v++)
                if (corner[v][0] == so[0] && corner[v][1] == so[1] && corner[v][2] == so[2]) has = true;
            if (!has) continue;
            for (int v = 0; v < 4; v++)
                codes[cnt][v] = (corner[v][0] - so[0] + 1) * 9 + (corner[v][1] - so[1] + 1) * 3 +
                                (corner[v][2] - so[2] + 1);
            cnt++;
        }
    }
    int n = 0;
    for (int t = 0; t < 24; t++)
        for (int v = 0; v < 4; v++) {
            int found = -1;
            for (int j = 0; j < n; j++)
                if (tb.nbr[j] == codes[t][v]) found = j;
            if (found < 0 && n < 15) {
                tb.nbr[n] = codes[t][v];
                found = n++;
            }
            tb.slot[t][v] = found;
        }
    for (int j = 0; j < n; j++)
        if (tb.nbr[j] == 13) tb.self = j;
    tb.ntet = cnt;
    tb.nnbr = n;
    return tb;
}

constexpr TetraTable kTet = make_tetra_table();
static_assert(kTet.ntet == 24 && kTet.nnbr == 15, "24 tetrahedra over 15 distinct corners expected");

__constant__ TetraTable c_tetra = kTet;

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

// Series coefficients 6 / (m (m-1) (m-2) (m-3)) of the m-th Taylor term,
// m = 4 .. kSeriesMax - 1 (the m-th entry; entries below 4 unused).
constexpr int kSeriesMax = 4 + 96;
struct SeriesTable {
    double f[kSeriesMax];
};
constexpr SeriesTable make_series_table()
{
    SeriesTable t{};
    for (int m = 4; m < kSeriesMax; m++) t.f[m] = 6.0 / ((double)m * (m - 1) * (m - 2) * (m - 3));
    return t;
}
__constant__ SeriesTable c_series = make_series_table();

// sum_{m>=N} g^(m)(c)/m! * h_{m-N}(x_0-c, .., x_N-c) over the N+1 nodes
// x[a..a+N], about the node c = x[cm] with lw = log(z - c)
template <int N>
__device__ __forceinline__ double2 dd_series(double2 z, const double *x, int a, int cm, double2 lw)
{
    const double c = x[cm];
    const double2 w = make_double2(z.x - c, z.y);
    const double2 wi = crecip(w);
    double y[N + 1], P[N + 1];
#pragma unroll
    for (int i = 0; i <= N; i++) {
        y[i] = x[a + i] - c;
        P[i] = 1.0;
    }
    // Taylor coefficients of g(x) = (z-x)^3 log(z-x) about c, with w = z - c:
    // m=0: w^3 L, 1: -(3w^2 L + w^2), 2: (6wL + 5w)/2, 3: -(6L + 11)/6,
    // m>=4: 6 / (m(m-1)(m-2)(m-3)) w^-(m-3)
    double2 sum = make_double2(0.0, 0.0);
    const double2 w2 = cmul(w, w);
#pragma unroll
    for (int m = N; m < 4; m++) {
        if (m > N) {
            P[0] *= y[0];
#pragma unroll
            for (int i = 1; i <= N; i++) P[i] = P[i - 1] + y[i] * P[i];
        }
        double2 coef;
        if (m == 0) coef = cmul(cmul(w2, w), lw);
        else if (m == 1)
            coef = make_double2(-(3.0 * (w2.x * lw.x - w2.y * lw.y) + w2.x), -(3.0 * (w2.x * lw.y + w2.y * lw.x) + w2.y));
        else if (m == 2)
            coef = make_double2(0.5 * (6.0 * (w.x * lw.x - w.y * lw.y) + 5.0 * w.x),
                                0.5 * (6.0 * (w.x * lw.y + w.y * lw.x) + 5.0 * w.y));
        else coef = make_double2(-(6.0 * lw.x + 11.0) / 6.0, -lw.y);
        sum = make_double2(sum.x + coef.x * P[N], sum.y + coef.y * P[N]);
    }
    double2 wp = make_double2(1.0, 0.0);  // w^-(m-3)
    int quiet = 0;
    for (int m = 4; m < kSeriesMax; m++) {
        if (m > N) {
            // raise P to degree m - N: h_k(y_0..y_i) = h_k(y_0..y_{i-1}) + y_i h_{k-1}(y_0..y_i)
            P[0] *= y[0];
#pragma unroll
            for (int i = 1; i <= N; i++) P[i] = P[i - 1] + y[i] * P[i];
        }
        wp = cmul(wp, wi);
        const double fh = c_series.f[m] * P[N];
        const double2 t = make_double2(wp.x * fh, wp.y * fh);
        sum = cadd(sum, t);
        // stop after two consecutive terms below 1e-17 of the sum: the terms
        // shrink at least fourfold, and FP64 resolves 1.1e-16 of the sum
        const double tm = fabs(t.x) + fabs(t.y), sm = fabs(sum.x) + fabs(sum.y);
        if (tm <= 1e-17 * sm) {
            if (++quiet == 2) break;
        } else {
            quiet = 0;
        }
    }
    return sum;
}

// fourth divided difference of g over five sorted nodes x with lw[i] =
// log(z - x[i])
__device__ double2 dd4_sorted(double2 z, const double *x, const double2 *lw)
{
    // entry (a, n) = g[x_a .. x_{a+n}] at slot id(a,n) = 5n - n(n-1)/2 + a
    bool need[15], ser[15];
    double2 val[15];
#pragma unroll
    for (int i = 0; i < 15; i++) { need[i] = false; ser[i] = false; }
    need[14] = true;
    const double zy2 = z.y * z.y;
#pragma unroll
    for (int n = 4; n >= 1; n--) {
#pragma unroll
        for (int a = 0; a + n <= 4; a++) {
            const int id = 5 * n - n * (n - 1) / 2 + a;
            if (!need[id]) continue;
            const int cm = a + n / 2;
            const double dev = fmax(x[a + n] - x[cm], x[cm] - x[a]);
            const double dx = z.x - x[cm];
            if (16.0 * dev * dev <= dx * dx + zy2) {   // 4 dev <= |z - x_cm|
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
                const double2 w = make_double2(z.x - x[a], z.y);
                val[id] = cmul(cmul(cmul(w, w), w), lw[a]);
            } else if (ser[id]) {
                if (n == 1) val[id] = dd_series<1>(z, x, a, a + n / 2, lw[a + n / 2]);
                else if (n == 2) val[id] = dd_series<2>(z, x, a, a + n / 2, lw[a + n / 2]);
                else if (n == 3) val[id] = dd_series<3>(z, x, a, a + n / 2, lw[a + n / 2]);
                else val[id] = dd_series<4>(z, x, a, a + n / 2, lw[a + n / 2]);
            } else {
                const int lid = 5 * (n - 1) - (n - 1) * (n - 2) / 2 + a;
                val[id] = cdiv_real(csub(val[lid + 1], val[lid]), x[a + n] - x[a]);
            }
        }
    }
    return val[14];
}

__device__ __forceinline__ int mesh_wrap(int n, int K) { return pmod(n, K); }

// ---- metallic cut: the part of a tetrahedron where E_b < E_F < E_a ----
//
// Points are barycentric coordinates with respect to the tetrahedron T.  A
// tetrahedron P is clipped to {phi < 0} for a linear phi given at its
// corners: one corner inside leaves a corner tetrahedron; two or three leave
// a triangular prism (bottom and top triangles joined by three lateral
// edges), cut into three tetrahedra.

__device__ __forceinline__ void lerp4(const double (&a)[4], const double (&b)[4], double s, double (&out)[4])
{
#pragma unroll
    for (int d = 0; d < 4; d++) out[d] = a[d] + s * (b[d] - a[d]);
}

template <typename Emit>
__device__ __forceinline__ void prism3(const double (&p0)[4], const double (&p1)[4], const double (&p2)[4],
                                       const double (&q0)[4], const double (&q1)[4], const double (&q2)[4], Emit &emit)
{
    emit(p0, p1, p2, q0);
    emit(p1, p2, q0, q1);
    emit(p2, q0, q1, q2);
}

template <typename Emit>
__device__ void clip_tet(const double (&P)[4][4], const double (&phi)[4], Emit &emit)
{
    int in[4], out[4], ni = 0, no = 0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        if (phi[c] < 0.0) in[ni++] = c;
        else out[no++] = c;
    }
    if (ni == 0) return;
    if (ni == 4) {
        emit(P[0], P[1], P[2], P[3]);
        return;
    }
    // the point where phi = 0 on the edge from inside corner a to outside corner b
    auto cut = [&](int a, int b, double (&q)[4]) { lerp4(P[a], P[b], phi[a] / (phi[a] - phi[b]), q); };
    double x0[4], x1[4], x2[4];
    if (ni == 1) {
        cut(in[0], out[0], x0);
        cut(in[0], out[1], x1);
        cut(in[0], out[2], x2);
        emit(P[in[0]], x0, x1, x2);
    } else if (ni == 3) {
        cut(in[0], out[0], x0);
        cut(in[1], out[0], x1);
        cut(in[2], out[0], x2);
        prism3(P[in[0]], P[in[1]], P[in[2]], x0, x1, x2, emit);
    } else {
        double y1[4], y2[4];
        cut(in[0], out[0], x1);
        cut(in[0], out[1], x2);
        cut(in[1], out[0], y1);
        cut(in[1], out[1], y2);
        prism3(P[in[0]], x1, x2, P[in[1]], y1, y2, emit);
    }
}

__device__ __forceinline__ double det4(const double (&a)[4], const double (&b)[4], const double (&c)[4],
                                       const double (&d)[4])
{
    // expansion along the first row
    auto m3 = [](double a0, double a1, double a2, double b0, double b1, double b2, double c0, double c1, double c2) {
        return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
    };
    return a[0] * m3(b[1], b[2], b[3], c[1], c[2], c[3], d[1], d[2], d[3]) -
           a[1] * m3(b[0], b[2], b[3], c[0], c[2], c[3], d[0], d[2], d[3]) +
           a[2] * m3(b[0], b[1], b[3], c[0], c[1], c[3], d[0], d[1], d[3]) -
           a[3] * m3(b[0], b[1], b[2], c[0], c[1], c[2], d[0], d[1], d[2]);
}

// sorting network on five keys, carrying the logarithms
__device__ __forceinline__ void sort5(double (&xs)[5], double2 (&ls)[5])
{
#define RP_CSWAP(i, j)                                                                             \
    {                                                                                              \
        const bool sw_ = xs[j] < xs[i];                                                            \
        const double xi_ = xs[i], xj_ = xs[j];                                                     \
        const double2 li_ = ls[i], lj_ = ls[j];                                                    \
        xs[i] = sw_ ? xj_ : xi_;                                                                   \
        xs[j] = sw_ ? xi_ : xj_;                                                                   \
        ls[i] = sw_ ? lj_ : li_;                                                                   \
        ls[j] = sw_ ? li_ : lj_;                                                                   \
    }
    RP_CSWAP(0, 1) RP_CSWAP(3, 4) RP_CSWAP(2, 4) RP_CSWAP(2, 3) RP_CSWAP(0, 3)
    RP_CSWAP(0, 2) RP_CSWAP(1, 4) RP_CSWAP(1, 3) RP_CSWAP(1, 2)
#undef RP_CSWAP
}

// (1/|T|) int over {E_b < E_F < E_a} within T of lambda_v / (z - e): the
// region is tiled by clipping T first to E_b < E_F, then each piece to
// E_a > E_F; a piece S contributes (|S|/|T|) sum_j lambda_v(s_j) I_j^S(z),
// I_j^S the vertex integral of S on the transition energies at its corners
// (lambda_v is linear, so it is the barycentric combination of its corner
// values).
__device__ double2 clipped_vertex_integral(double2 zz, const double (&e)[4], const double (&eb)[4],
                                           const double (&ea)[4], double ef, int v)
{
    const double T[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    double phi1[4];
#pragma unroll
    for (int c = 0; c < 4; c++) phi1[c] = eb[c] - ef;
    double2 acc = make_double2(0.0, 0.0);
    auto inner = [&](const double (&r0)[4], const double (&r1)[4], const double (&r2)[4], const double (&r3)[4]) {
        const double ratio = fabs(det4(r0, r1, r2, r3));
        if (!(ratio > 0.0)) return;
        const double *R[4] = {r0, r1, r2, r3};
        double eS[4];
        double2 lS[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            eS[j] = R[j][0] * e[0] + R[j][1] * e[1] + R[j][2] * e[2] + R[j][3] * e[3];
            lS[j] = clog_d(make_double2(zz.x - eS[j], zz.y));
        }
        for (int j = 0; j < 4; j++) {
            const double lam = R[j][v];
            if (lam == 0.0) continue;
            double xs[5] = {eS[0], eS[1], eS[2], eS[3], eS[j]};
            double2 ls[5] = {lS[0], lS[1], lS[2], lS[3], lS[j]};
            sort5(xs, ls);
            const double2 d = dd4_sorted(zz, xs, ls);
            acc.x += ratio * lam * d.x;
            acc.y += ratio * lam * d.y;
        }
    };
    auto outer = [&](const double (&q0)[4], const double (&q1)[4], const double (&q2)[4], const double (&q3)[4]) {
        const double Q[4][4] = {{q0[0], q0[1], q0[2], q0[3]}, {q1[0], q1[1], q1[2], q1[3]},
                                {q2[0], q2[1], q2[2], q2[3]}, {q3[0], q3[1], q3[2], q3[3]}};
        double phi2[4];
#pragma unroll
        for (int j = 0; j < 4; j++)
            phi2[j] = ef - (Q[j][0] * ea[0] + Q[j][1] * ea[1] + Q[j][2] * ea[2] + Q[j][3] * ea[3]);
        clip_tet(Q, phi2, inner);
    };
    clip_tet(T, phi1, outer);
    return acc;
}

constexpr int kWThreads = 128;

// One thread per (pair, frequency).  The corner energies e_j of the 15
// distinct corners live in registers (the tetrahedron table indexes them with
// the same slot in every lane, which the compiler turns into register-relative
// moves) and the logarithms log(z - e_j) in LDS ([slot][thread]), so five
// 128-thread blocks share a CU; each of the 24 tetrahedra sorts its five nodes
// (four corners, k's corner doubled) together with their logarithms and
// evaluates I_v(z) and I_v(z') (only I_v(z) when z' = z*).
//
// METAL: the Fermi level ef (hartree) cuts the tetrahedra.  With E_b < ef at
// all four corners of a tetrahedron and E_a > ef at all four, the insulating
// integral applies; with E_b >= ef or E_a <= ef at all four, the tetrahedron
// contributes nothing; otherwise clipped_vertex_integral tiles the part where
// E_b < ef < E_a (the corner energies of both bands are kept in LDS too).
template <bool METAL>
__global__ void __launch_bounds__(kWThreads)
k_weights(int K1, int K2, int K3, int q1, int q2, int q3, int nband, const double *E, const double *T,
          int o0, int nO, int e0, int nE, int k0, long npair, int nfreq, const double2 *freq,
          double delta, int mode, double ef, double2 *w)
{
    double eR[15];
    __shared__ double2 sL[15][kWThreads];
    __shared__ double sB[METAL ? 15 : 1][kWThreads];
    __shared__ double sA[METAL ? 15 : 1][kWThreads];
    const int tid = threadIdx.x;
    const long t = (long)blockIdx.x * blockDim.x + tid;
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
#pragma unroll
        for (int j = 0; j < 15; j++) {
            const int code = kTet.nbr[j];
            const int m1 = n1 + code / 9 - 1, m2 = n2 + (code / 3) % 3 - 1, m3 = n3 + code % 3 - 1;
            const int kv = (mesh_wrap(m1, K1) * K2 + mesh_wrap(m2, K2)) * K3 + mesh_wrap(m3, K3);
            const int kvq = (mesh_wrap(m1 + q1, K1) * K2 + mesh_wrap(m2 + q2, K2)) * K3 + mesh_wrap(m3 + q3, K3);
            const double eb = E[(long)kv * nband + b] * ha, ea = E[(long)kvq * nband + a] * ha;
            eR[j] = (E[(long)kvq * nband + a] - E[(long)kv * nband + b]) * ha;
            if constexpr (METAL) {
                sB[j][tid] = eb;
                sA[j][tid] = ea;
            }
        }
        // on the imaginary axis without broadening z' = z*, and since the
        // corner energies are real I_v(z*) = conj(I_v(z)): x = 2 Re sum I_v(z)/6
        const bool conj_pair = dl == 0.0 && om.x == 0.0;
        x = make_double2(0.0, 0.0);
        for (int zi = 0; zi < (conj_pair ? 1 : 2); zi++) {
            const double2 zz = zi ? zp : z;
#pragma unroll
            for (int j = 0; j < 15; j++) sL[j][tid] = clog_d(make_double2(zz.x - eR[j], zz.y));
            for (int tt = 0; tt < 24; tt++) {
                if constexpr (METAL) {
                    double e4[4], b4[4], a4[4];
                    bool all_in = true, none_b = true, none_a = true;
                    int iv = 0;
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int sl = c_tetra.slot[tt][v];
                        e4[v] = eR[sl];
                        b4[v] = sB[sl][tid];
                        a4[v] = sA[sl][tid];
                        if (sl == kTet.self) iv = v;
                        all_in = all_in && b4[v] < ef && a4[v] > ef;
                        none_b = none_b && !(b4[v] < ef);
                        none_a = none_a && !(a4[v] > ef);
                    }
                    if (none_b || none_a) continue;
                    if (!all_in) {
                        x = cadd(x, clipped_vertex_integral(zz, e4, b4, a4, ef, iv));
                        continue;
                    }
                }
                double xs[5];
                double2 ls[5];
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int sl = c_tetra.slot[tt][v];
                    xs[v] = eR[sl];
                    ls[v] = sL[sl][tid];
                }
                xs[4] = eR[kTet.self];
                ls[4] = sL[kTet.self][tid];
                // sorting network on five keys, carrying the logarithms
#define RP_CSWAP(i, j)                                                                             \
    {                                                                                              \
        const bool sw_ = xs[j] < xs[i];                                                            \
        const double xi_ = xs[i], xj_ = xs[j];                                                     \
        const double2 li_ = ls[i], lj_ = ls[j];                                                    \
        xs[i] = sw_ ? xj_ : xi_;                                                                   \
        xs[j] = sw_ ? xi_ : xj_;                                                                   \
        ls[i] = sw_ ? lj_ : li_;                                                                   \
        ls[j] = sw_ ? li_ : lj_;                                                                   \
    }
                RP_CSWAP(0, 1) RP_CSWAP(3, 4) RP_CSWAP(2, 4) RP_CSWAP(2, 3) RP_CSWAP(0, 3)
                RP_CSWAP(0, 2) RP_CSWAP(1, 4) RP_CSWAP(1, 3) RP_CSWAP(1, 2)
#undef RP_CSWAP
                x = cadd(x, dd4_sorted(zz, xs, ls));
            }
        }
        if (conj_pair) x = make_double2(2.0 * x.x, 0.0);
        x = cscale(x, 1.0 / 6.0);
    }
    double fac = 2.0 / (double)(K1 * K2 * K3);
    if (T) fac *= 1.0 - T[(long)kq * nband + a] * T[(long)k * nband + b];
    w[t] = cscale(x, fac);
}

// ---- Fermi-surface weights of the intraband term (Eq. plasma) ----
//
// D_v = (1/|T|) int_T lambda_v delta(e - E) d^3k for the linear interpolant e
// of the corner energies over T.  The section {e = E} is a triangle (one
// corner on one side of E) or a quadrilateral (two on each side) with its
// corners on the edges that E separates.  In the reference tetrahedron (corner
// 0 at the origin, corner j at the j-th unit vector, volume 1/6) the delta
// turns the volume integral into a section integral over |grad e|, and the
// mean of the linear lambda_v over each triangle of the section is the mean of
// its corner values.
__device__ double fermi_corner(const double (&e)[4], int v, double E)
{
    int lo[4], hi[4], nl = 0, nh = 0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        if (e[c] < E) lo[nl++] = c;
        else hi[nh++] = c;
    }
    if (nl == 0 || nh == 0) return 0.0;
    const double gx = e[1] - e[0], gy = e[2] - e[0], gz = e[3] - e[0];
    const double gn = sqrt(gx * gx + gy * gy + gz * gz);
    double P[4][3], L[4];
    int np = 0;
    // the point of edge (i, j) where e = E, and lambda_v there
    auto edge = [&](int i, int j) {
        const double t = (E - e[i]) / (e[j] - e[i]);
#pragma unroll
        for (int d = 0; d < 3; d++) P[np][d] = (i == d + 1 ? 1.0 - t : 0.0) + (j == d + 1 ? t : 0.0);
        L[np] = (v == i ? 1.0 - t : 0.0) + (v == j ? t : 0.0);
        np++;
    };
    if (nl == 1) {
        edge(lo[0], hi[0]);
        edge(lo[0], hi[1]);
        edge(lo[0], hi[2]);
    } else if (nh == 1) {
        edge(lo[0], hi[0]);
        edge(lo[1], hi[0]);
        edge(lo[2], hi[0]);
    } else {
        // in cyclic order: consecutive corners share a face of T
        edge(lo[0], hi[0]);
        edge(lo[0], hi[1]);
        edge(lo[1], hi[1]);
        edge(lo[1], hi[0]);
    }
    auto area = [&](int a, int b, int c) {
        const double u0 = P[b][0] - P[a][0], u1 = P[b][1] - P[a][1], u2 = P[b][2] - P[a][2];
        const double w0 = P[c][0] - P[a][0], w1 = P[c][1] - P[a][1], w2 = P[c][2] - P[a][2];
        const double x = u1 * w2 - u2 * w1, y = u2 * w0 - u0 * w2, z = u0 * w1 - u1 * w0;
        return 0.5 * sqrt(x * x + y * y + z * z);
    };
    double sum = area(0, 1, 2) * (L[0] + L[1] + L[2]) / 3.0;
    if (np == 4) sum += area(0, 2, 3) * (L[0] + L[2] + L[3]) / 3.0;
    return 6.0 * sum / gn;
}

// One thread per (k, band a in [b0, b0 + nb)): the Fermi-surface weight
// D(k) = (1/(6 N_k)) sum over the 24 tetrahedra around k of k's corner weight,
// times (1 - T^2), times p p^T: contrib[t] = {xx, yy, zz, xy, xz, yz}.
__global__ void __launch_bounds__(256)
k_fermi_plasma(int K1, int K2, int K3, int nband, const double *__restrict__ E, const double *__restrict__ T,
               int b0, int nb, double ef, const double *__restrict__ p, double *__restrict__ contrib)
{
    const int nk = K1 * K2 * K3;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nk * nb) return;
    const int k = (int)(t / nb), a = b0 + (int)(t - (long)k * nb);
    const int n1 = k / (K2 * K3), n2 = (k / K3) % K2, n3 = k % K3;
    const double ha = 1.0 / kHartreeEv;
    double e15[15];
#pragma unroll
    for (int j = 0; j < 15; j++) {
        const int code = kTet.nbr[j];
        const int kv = (mesh_wrap(n1 + code / 9 - 1, K1) * K2 + mesh_wrap(n2 + (code / 3) % 3 - 1, K2)) * K3 +
                       mesh_wrap(n3 + code % 3 - 1, K3);
        e15[j] = E[(long)kv * nband + a] * ha;
    }
    double D = 0.0;
#pragma unroll
    for (int tt = 0; tt < 24; tt++) {
        double e[4];
        int v = 0;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            e[c] = e15[kTet.slot[tt][c]];
            if (kTet.slot[tt][c] == kTet.self) v = c;
        }
        D += fermi_corner(e, v, ef);
    }
    D /= 6.0 * nk;
    if (T) D *= 1.0 - T[(long)k * nband + a] * T[(long)k * nband + a];
    const double px = p[3 * t], py = p[3 * t + 1], pz = p[3 * t + 2];
    double *o = contrib + 6 * t;
    o[0] = D * px * px;
    o[1] = D * py * py;
    o[2] = D * pz * pz;
    o[3] = D * px * py;
    o[4] = D * px * pz;
    o[5] = D * py * pz;
}

// out[q] = sum_t c[t][q], q < 6, in one block
__global__ void __launch_bounds__(256) k_sum6(long n, const double *__restrict__ c, double *__restrict__ out)
{
    __shared__ double red[6][256];
    const int tid = threadIdx.x;
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long i = tid; i < n; i += 256)
#pragma unroll
        for (int q = 0; q < 6; q++) s[q] += c[6 * i + q];
#pragma unroll
    for (int q = 0; q < 6; q++) red[q][tid] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
#pragma unroll
            for (int q = 0; q < 6; q++) red[q][tid] += red[q][tid + w];
        __syncthreads();
    }
    if (tid < 6) out[tid] = red[tid][0];
}

}  // namespace

void launch_weights(hipStream_t s, const int kmesh[3], const int iq[3], int nband,
                    const double *E_eV, const double *T, int o0, int o1, int e0, int e1,
                    int k0, int k1, int nfreq, const double2 *freq_eV, double delta_eV,
                    int mode, double ef_eV, double2 *w)
{
    const long npair = (long)(k1 - k0) * (e1 - e0) * (o1 - o0);
    const long tot = npair * nfreq;
    if (tot == 0) return;
    const dim3 grid((unsigned)((tot + kWThreads - 1) / kWThreads));
    if (mode == RP_W_TETRA_METAL)
        hipLaunchKernelGGL(k_weights<true>, grid, dim3(kWThreads), 0, s, kmesh[0], kmesh[1], kmesh[2], iq[0], iq[1],
                           iq[2], nband, E_eV, T, o0, o1 - o0, e0, e1 - e0, k0, npair, nfreq, freq_eV, delta_eV,
                           (int)RP_W_TETRA, ef_eV / kHartreeEv, w);
    else
        hipLaunchKernelGGL(k_weights<false>, grid, dim3(kWThreads), 0, s, kmesh[0], kmesh[1], kmesh[2], iq[0], iq[1],
                           iq[2], nband, E_eV, T, o0, o1 - o0, e0, e1 - e0, k0, npair, nfreq, freq_eV, delta_eV,
                           mode, 0.0, w);
}

void launch_fermi_plasma(hipStream_t s, const int kmesh[3], int nband, const double *E_eV, const double *T, int b0,
                         int b1, double ef_eV, const double *p, double *contrib, double *out)
{
    const long n = (long)kmesh[0] * kmesh[1] * kmesh[2] * (b1 - b0);
    if (n > 0)
        hipLaunchKernelGGL(k_fermi_plasma, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kmesh[0], kmesh[1],
                           kmesh[2], nband, E_eV, T, b0, b1 - b0, ef_eV / kHartreeEv, p, contrib);
    hipLaunchKernelGGL(k_sum6, dim3(1), dim3(256), 0, s, n, contrib, out);
}

}  // namespace rp
