// Host side of the C ABI: argument validation, workspace management and the
// order of launches for each entry point.  All device work goes to the
// context's stream; nothing here synchronizes except rp_synchronize.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <optional>
#include <unordered_map>
#include <vector>

#include "rp_internal.h"

namespace rp {

rp_status fail(rp_ctx *ctx, rp_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

rp_status ensure(rp_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.bytes) return RP_OK;
    if (b.p) {
        // the stream may still be using the old buffer
        if (hipStreamSynchronize(ctx->stream) != hipSuccess)
            return fail(ctx, RP_E_DEVICE, "stream synchronize failed before workspace growth");
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)256);
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(ctx, RP_E_NOMEM, "device workspace allocation of %zu bytes failed", want);
    }
    b.bytes = want;
    return RP_OK;
}

rp_status check_launch(rp_ctx *ctx, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, RP_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return RP_OK;
}

bool make_plan(int n, FftPlan *plan)
{
    if (n < 1 || n > 256) return false;
    plan->n = n;
    plan->nrad = 0;
    int m = n;
    const int order[4] = {4, 2, 3, 5};
    for (int r : order)
        while (m % r == 0) {
            if (plan->nrad >= 12) return false;
            plan->rad[plan->nrad++] = r;
            m /= r;
        }
    return m == 1;
}

rp_status geometry(rp_ctx *ctx, const rp_cell *cell, const int iq[3], Geometry *g)
{
    if (!cell) return fail(ctx, RP_E_NULL, "cell is NULL");
    if (!iq) return fail(ctx, RP_E_NULL, "iq is NULL");
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) g->lat[3 * a + b] = cell->lat[a][b];
        g->fft[a] = cell->fft[a];
        g->kmesh[a] = cell->kmesh[a];
        g->iq[a] = iq[a];
        if (cell->fft[a] < 1 || cell->kmesh[a] < 1)
            return fail(ctx, RP_E_SHAPE, "fft and kmesh entries must be >= 1");
        if (iq[a] < 0 || iq[a] >= cell->kmesh[a])
            return fail(ctx, RP_E_RANGE, "iq[%d] = %d outside the mesh", a, iq[a]);
    }
    const double *A = g->lat;
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det))
        return fail(ctx, RP_E_RANGE, "lattice vectors are degenerate");
    double inv[9];
    inv[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    inv[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    inv[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    inv[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    inv[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    inv[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    inv[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    inv[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    inv[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) g->rec[3 * i + j] = 2.0 * kPi * inv[3 * j + i];
    g->volume = std::fabs(det);
    g->nk = cell->kmesh[0] * cell->kmesh[1] * cell->kmesh[2];
    return RP_OK;
}

Tune tune_for(const rp_ctx *ctx, int ng, const int fft[3])
{
    Tune t;
    const int edge = std::max(fft[0], std::max(fft[1], fft[2]));
    for (const rp_tune_entry &e : ctx->tuning) {
        if (ng > e.ng_max || edge > e.grid_max) continue;
        if (e.chi_nw) t.chi_nw = e.chi_nw;
        if (e.chi_fill >= 0) t.chi_fill = e.chi_fill;
        t.fft_lines = e.fft_lines;
        t.chi_kernel = e.chi_kernel;
        break;
    }
    return t;
}

static hipEvent_t take_event(rp_ctx *ctx)
{
    if (!ctx->spare.empty()) {
        hipEvent_t e = ctx->spare.back();
        ctx->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

StageTimer::StageTimer(rp_ctx *ctx, int stage) : ctx_(ctx), stage_(stage)
{
    if (!ctx_->profiling || ctx_->capturing) return;
    a_ = take_event(ctx_);
    if (a_) (void)hipEventRecord(a_, ctx_->stream);
}

StageTimer::~StageTimer()
{
    if (!a_) return;
    hipEvent_t b = take_event(ctx_);
    if (!b) {
        ctx_->spare.push_back(a_);
        return;
    }
    (void)hipEventRecord(b, ctx_->stream);
    ctx_->marks.push_back({stage_, a_, b});
}

static double qg_norm(const Geometry &g, const int *m)
{
    double f[3], v[3] = {0, 0, 0};
    for (int a = 0; a < 3; a++) f[a] = (double)g.iq[a] / g.kmesh[a] + m[a];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) v[c] += f[a] * g.rec[3 * a + c];
    return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

static rp_status plans3(rp_ctx *ctx, const Geometry &g, FftPlan plans[3])
{
    for (int a = 0; a < 3; a++)
        if (!make_plan(g.fft[a], &plans[a]))
            return fail(ctx, RP_E_UNSUPPORTED, "FFT length %d is not 2^a 3^b 5^c <= 256", g.fft[a]);
    return RP_OK;
}

static rp_status upload(rp_ctx *ctx, DevBuf &b, const void *host, size_t bytes)
{
    rp_status st = ensure(ctx, b, bytes);
    if (st != RP_OK) return st;
    if (bytes && hipMemcpyAsync(b.p, host, bytes, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        return fail(ctx, RP_E_DEVICE, "host-to-device copy failed");
    return RP_OK;
}

static rp_status check_ranges(rp_ctx *ctx, const Geometry &g, int nband, int o0, int o1, int e0, int e1,
                              int k0, int k1)
{
    if (nband < 1) return fail(ctx, RP_E_SHAPE, "nband must be >= 1");
    if (o0 < 0 || o1 < o0 || o1 > nband) return fail(ctx, RP_E_SHAPE, "bad occupied range [%d,%d)", o0, o1);
    if (e0 < 0 || e1 < e0 || e1 > nband) return fail(ctx, RP_E_SHAPE, "bad empty range [%d,%d)", e0, e1);
    if (k0 < 0 || k1 < k0 || k1 > g.nk) return fail(ctx, RP_E_SHAPE, "bad k range [%d,%d)", k0, k1);
    return RP_OK;
}

static rp_status check_gsph(rp_ctx *ctx, const Geometry &g, int ng, const int *gsph, const char *name)
{
    if (ng < 0) return fail(ctx, RP_E_SHAPE, "%s count < 0", name);
    if (ng > 0 && !gsph) return fail(ctx, RP_E_NULL, "%s is NULL", name);
    for (int i = 0; i < ng; i++)
        if (!(qg_norm(g, gsph + 3 * i) > 0.0))
            return fail(ctx, RP_E_RANGE, "%s[%d]: |q+G| = 0 (drop G = 0 at q = 0)", name, i);
    return RP_OK;
}

// ---- steps a2-a4: validated pair-density work, enqueued without allocation --

// Host-side description of one pair-density request after validation.
struct PairJob {
    Geometry g;
    FftPlan plans[3];
    int nband = 0, npw_max = 0;
    const int *npw = nullptr;       // host [Nk]
    int mmax[3] = {0, 0, 0};
    const int *miller = nullptr;    // device [Nk][npw_max][3]
    const double2 *coef = nullptr;  // device [Nk][nband][npw_max]
    int o0 = 0, o1 = 0, e0 = 0, e1 = 0;
    int ng = 0;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    bool fp32 = false;
    bool empty = true;  // no band pairs in the requested ranges
    int fft_lines = 0;  // tuned lines per workgroup of the u-grid transforms
};

static bool valid_prec(rp_precision prec)
{
    return prec == RP_FP64 || prec == RP_SPLIT_BF16 || prec == RP_SPLIT_BF16_X6;
}

// The Miller window [lo, hi] of the sphere per axis, and the grid that steps
// a2-a4 run on.  The cell's grid must hold the sphere products alias-free:
// N_a > 2 mmax_a + max |m_a + G0_a| (G0_a in {0, 1} when iq_a > 0).  The pair
// densities at the sphere points (Eq. ism) are then the same on every such
// grid, so the steps run on the smallest one the lane kernels take (N2 = N3
// from their lengths, N1 any length with a plan), never larger than the
// cell's; where no lane length fits, on the cell's grid.
static rp_status pair_grid(rp_ctx *ctx, const Geometry &g, const int mmax[3], int ng, const int *gsph, bool fp32,
                           int lo[3], int hi[3], int grid[3])
{
    int need[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = 1 << 30;
        hi[a] = -(1 << 30);
        for (int i = 0; i < ng; i++) {
            lo[a] = std::min(lo[a], gsph[3 * i + a]);
            hi[a] = std::max(hi[a], gsph[3 * i + a]);
        }
        const int up = hi[a] + (g.iq[a] > 0 ? 1 : 0);
        const int gmax = std::max(std::abs(lo[a]), std::abs(up));
        if (mmax[a] < 0) return fail(ctx, RP_E_SHAPE, "mmax[%d] < 0", a);
        if (g.fft[a] <= 2 * mmax[a] + gmax)
            return fail(ctx, RP_E_ALIAS, "axis %d: N=%d <= 2*mmax+|G|max = %d (pair products alias)", a,
                        g.fft[a], 2 * mmax[a] + gmax);
        need[a] = 2 * mmax[a] + gmax + 1;
        grid[a] = g.fft[a];
    }
    if (g.fft[1] != g.fft[2]) return RP_OK;
    const int n23 = pair_lane_edge(std::max(need[1], need[2]), g.fft[1], ng, hi[2] - lo[2] + 1, fp32);
    if (!n23) return RP_OK;
    FftPlan p;
    for (int n = need[0]; n < g.fft[0]; n++)
        if (make_plan(n, &p)) {
            grid[0] = n;
            break;
        }
    grid[1] = grid[2] = n23;
    return RP_OK;
}

static rp_status pair_check(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband, int npw_max,
                            const int *npw, const int mmax[3], const int *miller, const double *coef, int o0,
                            int o1, int e0, int e1, int k0, int k1, int ng, const int *gsph, rp_precision prec,
                            PairJob *j)
{
    rp_status st = geometry(ctx, cell, iq, &j->g);
    if (st != RP_OK) return st;
    const Geometry &g = j->g;
    if (!npw || !mmax || !miller || !coef) return fail(ctx, RP_E_NULL, "NULL array argument");
    if ((st = check_ranges(ctx, g, nband, o0, o1, e0, e1, k0, k1)) != RP_OK) return st;
    if (ng < 1 || ng > 6144) return fail(ctx, RP_E_UNSUPPORTED, "ng = %d outside [1, 6144]", ng);
    // (G = 0 at q = 0 is allowed here: the pair density there is an overlap;
    // the Coulomb factor that forbids it belongs to the screening step)
    if (!gsph) return fail(ctx, RP_E_NULL, "gsph is NULL");
    if (npw_max < 1) return fail(ctx, RP_E_SHAPE, "npw_max must be >= 1");
    if (!valid_prec(prec)) return fail(ctx, RP_E_RANGE, "unknown precision");
    j->fp32 = prec != RP_FP64;
    if ((st = plans3(ctx, g, j->plans)) != RP_OK) return st;
    for (int k = 0; k < g.nk; k++)
        if (npw[k] < 0 || npw[k] > npw_max) return fail(ctx, RP_E_SHAPE, "npw[%d] outside [0, npw_max]", k);
    int grid[3];
    if ((st = pair_grid(ctx, g, mmax, ng, gsph, j->fp32, j->lo, j->hi, grid)) != RP_OK) return st;
    j->fft_lines = tune_for(ctx, ng, g.fft).fft_lines;
    for (int a = 0; a < 3; a++) {
        j->mmax[a] = mmax[a];
        j->g.fft[a] = grid[a];
    }
    if ((st = plans3(ctx, g, j->plans)) != RP_OK) return st;
    j->nband = nband;
    j->npw_max = npw_max;
    j->npw = npw;
    j->miller = miller;
    j->coef = (const double2 *)coef;
    j->o0 = o0;
    j->o1 = o1;
    j->e0 = e0;
    j->e1 = e1;
    j->ng = ng;
    j->empty = (long)(o1 - o0) * (e1 - e0) * (k1 - k0) == 0;
    if (j->empty) return RP_OK;
    // the pair kernels' LDS plans (m3 window of the sphere, hi - lo + 1)
    if (!pair_supported(g.fft, ng, j->hi[2] - j->lo[2] + 1, j->fp32))
        return fail(ctx, RP_E_UNSUPPORTED, "grid %dx%dx%d too large for the pair kernel's LDS plan", g.fft[0],
                    g.fft[1], g.fft[2]);
    return RP_OK;
}

// u-grid workspace of one k: the occupied and the empty bands' grids.
static size_t pair_grid_bytes(const PairJob &j)
{
    return ugrid_bytes(j.g.fft, (j.o1 - j.o0) + (j.e1 - j.e0), j.npw_max, j.fp32);
}

// Enqueues steps a2-a4 for k in [k0, k1): per k, the u-grids of the occupied
// bands at k and of the empty bands at k+q (into `grid`), then the pair
// kernel into M[k - k0], or, when ops is given (FP32 grids), into the split
// operands of one contraction over the pairs of [k0, k1) in M's order.  dg is
// the device copy of the G list.  No allocation, copy or synchronization.
static rp_status pair_enqueue(rp_ctx *ctx, const PairJob &j, int k0, int k1, const int *dg, void *grid,
                              double2 *M, const SplitOps *ops = nullptr)
{
    const Geometry &g = j.g;
    const int nO = j.o1 - j.o0, nE = j.e1 - j.e0;
    if ((long)nO * nE * (k1 - k0) == 0) return RP_OK;
    const long nr = (long)g.fft[0] * g.fft[1] * g.fft[2];
    const int L3 = j.hi[2] - j.lo[2] + 1;
    for (int k = k0; k < k1; k++) {
        const int n1 = k / (g.kmesh[1] * g.kmesh[2]), n2 = (k / g.kmesh[2]) % g.kmesh[1], n3 = k % g.kmesh[2];
        const int s[3] = {n1 + g.iq[0], n2 + g.iq[1], n3 + g.iq[2]};
        int r[3], g0[3];
        for (int a = 0; a < 3; a++) {
            r[a] = s[a] % g.kmesh[a];
            g0[a] = s[a] / g.kmesh[a];
        }
        const int kp = (r[0] * g.kmesh[1] + r[1]) * g.kmesh[2] + r[2];
        const int *mil_k = j.miller + (long)k * j.npw_max * 3, *mil_kp = j.miller + (long)kp * j.npw_max * 3;
        const double2 *c_k = j.coef + ((long)k * j.nband + j.o0) * j.npw_max;
        const double2 *c_kp = j.coef + ((long)kp * j.nband + j.e0) * j.npw_max;
        {
            StageTimer t(ctx, RP_STAGE_UGRID);
            launch_ugrid2(ctx->stream, j.plans, g.fft, j.mmax, nO, j.npw[k], mil_k, c_k, nE, j.npw[kp], mil_kp, c_kp,
                          j.npw_max, grid, j.fp32, j.fft_lines);
        }
        const int lo3 = j.lo[2] + g0[2];
        {
            StageTimer t(ctx, RP_STAGE_PAIR);
            if (ops) {
                SplitOps o = *ops;
                o.p0 = (long)(k - k0) * nE * nO;
                const float2 *v = (const float2 *)grid;
                launch_pair_ops(ctx->stream, j.plans, g.fft, v, v + nr * nO, nO, nE, j.ng, dg, g0, lo3, L3, o);
            } else if (j.fp32) {
                double2 *Mk = M + (long)(k - k0) * nE * nO * j.ng;
                const float2 *v = (const float2 *)grid;
                launch_pair_k(ctx->stream, j.plans, g.fft, v, v + nr * nO, nO, nE, j.ng, dg, g0, lo3, L3, true, Mk);
            } else {
                double2 *Mk = M + (long)(k - k0) * nE * nO * j.ng;
                const double2 *u = (const double2 *)grid;
                launch_pair_k(ctx->stream, j.plans, g.fft, u, u + nr * nO, nO, nE, j.ng, dg, g0, lo3, L3, false,
                              Mk);
            }
        }
        rp_status st = check_launch(ctx, "pair density");
        if (st != RP_OK) return st;
    }
    return RP_OK;
}

// ---- steps a5-a6: validated weight and contraction work -------------------

struct ChiJob {
    Geometry g;
    int nband = 0;
    const double *E = nullptr, *T = nullptr;  // device [Nk][nband]
    int o0 = 0, o1 = 0, e0 = 0, e1 = 0;
    int ng = 0;
    int nfreq = 0;
    double delta = 0.0;
    rp_weight_mode wm = RP_W_TETRA;
    double ef = 0.0;    // Fermi level (eV) of RP_W_TETRA_METAL
    rp_precision prec = RP_FP64;
    bool herm = false;  // real weights: chi Hermitian
    Tune tune;          // contraction launch shape
};

static rp_status weights_check(rp_ctx *ctx, const double *E, int nfreq, const double *freq_eV, double delta_eV,
                               rp_weight_mode wm)
{
    if (!E || !freq_eV) return fail(ctx, RP_E_NULL, "NULL energy or frequency array");
    if (nfreq < 1) return fail(ctx, RP_E_SHAPE, "nfreq must be >= 1");
    if (!(delta_eV >= 0.0) || !std::isfinite(delta_eV)) return fail(ctx, RP_E_RANGE, "delta must be >= 0");
    if (wm != RP_W_TETRA && wm != RP_W_SAMPLING && wm != RP_W_TETRA_METAL)
        return fail(ctx, RP_E_RANGE, "unknown weight mode");
    if (wm == RP_W_TETRA_METAL && !std::isfinite(ctx->fermi_eV))
        return fail(ctx, RP_E_RANGE, "metallic weights need a Fermi level (rp_set_fermi_level)");
    for (int f = 0; f < 2 * nfreq; f++)
        if (!std::isfinite(freq_eV[f])) return fail(ctx, RP_E_RANGE, "non-finite frequency");
    return RP_OK;
}

static rp_status chi_check(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband, const double *E,
                           const double *T, int o0, int o1, int e0, int e1, int k0, int k1, int ng, int nfreq,
                           const double *freq_eV, double delta_eV, rp_weight_mode wm, rp_precision prec,
                           int accumulate, ChiJob *c)
{
    rp_status st = geometry(ctx, cell, iq, &c->g);
    if (st != RP_OK) return st;
    if ((st = check_ranges(ctx, c->g, nband, o0, o1, e0, e1, k0, k1)) != RP_OK) return st;
    if (ng < 1) return fail(ctx, RP_E_SHAPE, "ng must be >= 1");
    if (!valid_prec(prec)) return fail(ctx, RP_E_RANGE, "unknown precision");
    if (accumulate != 0 && accumulate != 1) return fail(ctx, RP_E_RANGE, "accumulate must be 0 or 1");
    if ((st = weights_check(ctx, E, nfreq, freq_eV, delta_eV, wm)) != RP_OK) return st;
    c->nband = nband;
    c->E = E;
    c->T = T;
    c->o0 = o0;
    c->o1 = o1;
    c->e0 = e0;
    c->e1 = e1;
    c->ng = ng;
    c->nfreq = nfreq;
    c->delta = delta_eV;
    c->wm = wm;
    c->ef = wm == RP_W_TETRA_METAL ? ctx->fermi_eV : 0.0;
    c->prec = prec;
    // on the imaginary axis (w = i nu) without broadening, z = i nu and
    // z' = -i nu = z* in Eqs. Xakqbk and tetrahedron, whose two terms are then
    // complex conjugates: the weights are real and chi is Hermitian
    c->tune = tune_for(ctx, ng, c->g.fft);
    c->herm = delta_eV == 0.0;
    for (int f = 0; f < nfreq; f++)
        if (freq_eV[2 * f] != 0.0) c->herm = false;
    return RP_OK;
}

// Workspace of one contraction over npair pairs.
struct ChiBytes {
    size_t w = 0, a = 0, b = 0, sw = 0, part = 0;
};

static ChiBytes chi_bytes(const ChiJob &c, long npair)
{
    ChiBytes b;
    b.w = sizeof(double2) * (size_t)std::max(1L, npair) * c.nfreq;
    if (c.prec != RP_FP64) {
        b.a = split_a_bytes(npair, c.ng);
        b.b = split_b_bytes(npair, c.ng);
        b.sw = split_w_bytes(npair, c.nfreq);
        b.part = chi_part_bytes(npair, c.ng, c.nfreq, c.herm, c.tune.chi_nw, c.tune.chi_fill, c.tune.chi_kernel,
                                c.prec == RP_SPLIT_BF16 ? 2 : 3);
    }
    return b;
}

struct ChiBufs {
    double2 *w;
    void *a, *b, *sw, *part;
};

// Enqueues the weights of the pairs of k in [k0, k1) into bufs.w (dfreq is the
// device copy of the frequencies) and the contraction of M into chi.  With
// ops_ready (split forms) the pair kernels have already written the pairs'
// operands into bufs.a / bufs.b and M is not read: only their padding is
// cleared.  No allocation, copy or synchronization.
static rp_status chi_enqueue(rp_ctx *ctx, const ChiJob &c, int k0, int k1, const double2 *M,
                             const double2 *dfreq, const ChiBufs &bufs, int accumulate, double2 *chi,
                             bool ops_ready = false)
{
    const long npair = (long)(k1 - k0) * (c.e1 - c.e0) * (c.o1 - c.o0);
    rp_status st;
    if (npair > 0) {
        {
            StageTimer t(ctx, RP_STAGE_WEIGHTS);
            launch_weights(ctx->stream, c.g.kmesh, c.g.iq, c.nband, c.E, c.T, c.o0, c.o1, c.e0, c.e1, k0, k1,
                           c.nfreq, dfreq, c.delta, (int)c.wm, c.ef, bufs.w);
        }
        if ((st = check_launch(ctx, "weights")) != RP_OK) return st;
    }
    if (c.prec == RP_FP64) {
        StageTimer t(ctx, RP_STAGE_CHI);
        launch_chi_f64(ctx->stream, npair, c.ng, M, c.nfreq, bufs.w, accumulate, c.herm, chi);
    } else {
        const int nterm = c.prec == RP_SPLIT_BF16 ? 2 : 3;
        {
            StageTimer t(ctx, RP_STAGE_PREP);
            if (ops_ready)
                launch_ops_pad(ctx->stream, split_ops(bufs.a, bufs.b, npair, c.ng, nterm), npair, c.ng);
            else
                launch_split_prep(ctx->stream, nterm, npair, c.ng, M, bufs.a, bufs.b);
            launch_weight_prep(ctx->stream, npair, c.nfreq, bufs.w, c.herm, bufs.sw);
        }
        // the contraction and the FP64 sum of its partial tiles on separate timers
        std::optional<StageTimer> tc, tr;
        tc.emplace(ctx, RP_STAGE_CHI);
        launch_chi_bf16(ctx->stream, nterm, npair, c.ng, c.nfreq, accumulate, chi, bufs.a, bufs.b, bufs.sw, c.herm,
                        c.tune.chi_nw, c.tune.chi_fill, c.tune.chi_kernel, bufs.part, [&] {
                            tc.reset();
                            tr.emplace(ctx, RP_STAGE_REDUCE);
                        });
    }
    return check_launch(ctx, "chi0 contraction");
}

// Launch arguments of a batch, serialized to decide whether a graph can be reused.
static void key_put(std::string &key, const void *p, size_t n) { key.append((const char *)p, n); }

template <typename T> static void key_val(std::string &key, const T &v) { key_put(key, &v, sizeof v); }

// Fixed workspace of rp_chi0_accumulate_noalloc: a device array in the
// library's code object, so each GPU that loads the library holds one copy of
// kScratchBytes until the process ends.  Host code never uses the name
// `scratch` as an address: the device address comes from hipGetSymbolAddress,
// once per device with that device current, and is kept per device.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];
static bool g_scratch_done[64];

// The address of this device's scratch array (the device must be current),
// or nullptr when the runtime cannot resolve it.
static void *scratch_address(int device)
{
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ptr = nullptr;
        }
        g_scratch_ptr[device] = ptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_ptr[device];
}

}  // namespace rp

using namespace rp;

extern "C" {

rp_status rp_create(rp_ctx **out, int device, void *hip_stream)
{
    if (!out) return RP_E_NULL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return RP_E_DEVICE;
    }
    if (device < 0 || device >= ndev) return RP_E_RANGE;
    if (hipSetDevice(device) != hipSuccess) return RP_E_DEVICE;
    rp_ctx *ctx = new rp_ctx();
    ctx->device = device;
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return RP_E_DEVICE;
        }
        ctx->own_stream = true;
    }
    if (hipMalloc((void **)&ctx->flag, 4 * sizeof(int)) != hipSuccess ||
        hipMemsetAsync(ctx->flag, 0, 4 * sizeof(int), ctx->stream) != hipSuccess) {
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return RP_E_DEVICE;
    }
    ctx->scratch = scratch_address(device);
    *out = ctx;
    return RP_OK;
}

static void release_marks(rp_ctx *ctx)
{
    for (auto &m : ctx->marks) {
        ctx->spare.push_back(m.a);
        ctx->spare.push_back(m.b);
    }
    ctx->marks.clear();
}

rp_status rp_profile(rp_ctx *ctx, int enable)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, RP_E_DEVICE, "stream synchronize failed");
    release_marks(ctx);
    ctx->profiling = enable != 0;
    return RP_OK;
}

rp_status rp_profile_read(rp_ctx *ctx, double *ms, long *count)
{
    if (!ctx) return RP_E_NULL;
    if (!ms || !count) return fail(ctx, RP_E_NULL, "NULL output array");
    (void)hipSetDevice(ctx->device);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, RP_E_DEVICE, "stream synchronize failed");
    for (int i = 0; i < RP_NSTAGE; i++) {
        ms[i] = 0.0;
        count[i] = 0;
    }
    for (auto &m : ctx->marks) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, m.a, m.b) != hipSuccess) return fail(ctx, RP_E_DEVICE, "event timing failed");
        ms[m.stage] += t;
        count[m.stage] += 1;
    }
    return RP_OK;
}

rp_status rp_destroy(rp_ctx *ctx)
{
    if (!ctx) return RP_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    release_marks(ctx);
    for (hipEvent_t e : ctx->spare) (void)hipEventDestroy(e);
    ctx->spare.clear();
    DevBuf *bufs[] = {&ctx->ugrid, &ctx->ugrid32, &ctx->weights, &ctx->glist, &ctx->freq,  &ctx->kinfo, &ctx->vsqrt,
                      &ctx->work,  &ctx->split_a, &ctx->split_b, &ctx->split_w, &ctx->rho, &ctx->piv,
                      &ctx->mbuf,  &ctx->bstage,  &ctx->chi_part};
    for (hipGraphExec_t e : ctx->batch_execs) (void)hipGraphExecDestroy(e);
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->flag) (void)hipFree(ctx->flag);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return RP_OK;
}

const char *rp_last_error(const rp_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

rp_status rp_synchronize(rp_ctx *ctx)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess)
        return fail(ctx, RP_E_DEVICE, "stream synchronize: %s", hipGetErrorString(hipGetLastError()));
    int flag[4] = {0, 0, 0, 0};
    if (hipMemcpy(flag, ctx->flag, sizeof flag, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(ctx, RP_E_DEVICE, "flag read failed");
    if (flag[0]) {
        (void)hipMemset(ctx->flag, 0, sizeof flag);
        if (flag[0] & kFlagZeroPivot) return fail(ctx, RP_E_SINGULAR, "zero pivot in the dielectric matrix");
        return fail(ctx, RP_E_RANGE, "non-finite value detected on the device");
    }
    return RP_OK;
}

rp_status rp_pair_density(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband, int npw_max,
                          const int *npw, const int mmax[3], const int *miller, const double *coef,
                          int o0, int o1, int e0, int e1, int k0, int k1, int ng, const int *gsph,
                          rp_precision prec, double *M)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    PairJob j;
    rp_status st = pair_check(ctx, cell, iq, nband, npw_max, npw, mmax, miller, coef, o0, o1, e0, e1, k0, k1, ng,
                              gsph, prec, &j);
    if (st != RP_OK) return st;
    if (!M) return fail(ctx, RP_E_NULL, "M is NULL");
    if (j.empty) return RP_OK;
    DevBuf &grid = j.fp32 ? ctx->ugrid32 : ctx->ugrid;
    if ((st = ensure(ctx, grid, pair_grid_bytes(j))) != RP_OK) return st;
    if ((st = upload(ctx, ctx->glist, gsph, sizeof(int) * 3 * ng)) != RP_OK) return st;
    return pair_enqueue(ctx, j, k0, k1, (const int *)ctx->glist.p, grid.p, (double2 *)M);
}

rp_status rp_pair_grid(const rp_cell *cell, const int iq[3], const int mmax[3], int ng, const int *gsph,
                       rp_precision prec, int grid[3])
{
    if (!mmax || !gsph || !grid) return RP_E_NULL;
    Geometry g;
    rp_status st = geometry(nullptr, cell, iq, &g);
    if (st != RP_OK) return st;
    if (ng < 1 || ng > 6144) return RP_E_UNSUPPORTED;
    if (!valid_prec(prec)) return RP_E_RANGE;
    FftPlan plans[3];
    if ((st = plans3(nullptr, g, plans)) != RP_OK) return st;
    int lo[3], hi[3];
    return pair_grid(nullptr, g, mmax, ng, gsph, prec != RP_FP64, lo, hi, grid);
}

rp_status rp_weights(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband,
                     const double *energy_eV, const double *T, int o0, int o1, int e0, int e1, int k0,
                     int k1, int nfreq, const double *freq_eV, double delta_eV, rp_weight_mode wm,
                     double *w)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    Geometry g;
    rp_status st = geometry(ctx, cell, iq, &g);
    if (st != RP_OK) return st;
    if ((st = check_ranges(ctx, g, nband, o0, o1, e0, e1, k0, k1)) != RP_OK) return st;
    if (!w) return fail(ctx, RP_E_NULL, "w is NULL");
    if ((st = weights_check(ctx, energy_eV, nfreq, freq_eV, delta_eV, wm)) != RP_OK) return st;
    if ((st = upload(ctx, ctx->freq, freq_eV, sizeof(double2) * nfreq)) != RP_OK) return st;
    {
        StageTimer t(ctx, RP_STAGE_WEIGHTS);
        launch_weights(ctx->stream, g.kmesh, g.iq, nband, energy_eV, T, o0, o1, e0, e1, k0, k1, nfreq,
                       (const double2 *)ctx->freq.p, delta_eV, (int)wm, ctx->fermi_eV, (double2 *)w);
    }
    return check_launch(ctx, "weights");
}

rp_status rp_chi0_accumulate(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband,
                             const double *energy_eV, const double *T, int o0, int o1, int e0, int e1,
                             int k0, int k1, int ng, const double *M, int nfreq, const double *freq_eV,
                             double delta_eV, rp_weight_mode wm, rp_precision prec, int accumulate,
                             double *chi)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    ChiJob c;
    rp_status st = chi_check(ctx, cell, iq, nband, energy_eV, T, o0, o1, e0, e1, k0, k1, ng, nfreq, freq_eV,
                             delta_eV, wm, prec, accumulate, &c);
    if (st != RP_OK) return st;
    if (!M || !chi) return fail(ctx, RP_E_NULL, "NULL M or chi");
    const long npair = (long)(k1 - k0) * (e1 - e0) * (o1 - o0);
    const ChiBytes nb = chi_bytes(c, npair);
    if ((st = ensure(ctx, ctx->weights, nb.w)) != RP_OK) return st;
    if (prec != RP_FP64) {
        if ((st = ensure(ctx, ctx->split_a, nb.a)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->split_b, nb.b)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->split_w, nb.sw)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->chi_part, nb.part)) != RP_OK) return st;
    }
    if ((st = upload(ctx, ctx->freq, freq_eV, sizeof(double2) * nfreq)) != RP_OK) return st;
    const ChiBufs bufs{(double2 *)ctx->weights.p, ctx->split_a.p, ctx->split_b.p, ctx->split_w.p,
                       ctx->chi_part.p};
    return chi_enqueue(ctx, c, k0, k1, (const double2 *)M, (const double2 *)ctx->freq.p, bufs, accumulate,
                       (double2 *)chi);
}

rp_status rp_chi0_accumulate_noalloc(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband,
                                     const double *energy_eV, const double *T, int o0, int o1, int e0, int e1,
                                     int k0, int k1, int ng, const double *M, int nfreq, const double *freq_eV,
                                     double delta_eV, rp_weight_mode wm, rp_precision prec, int accumulate,
                                     double *chi)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    ChiJob c;
    rp_status st = chi_check(ctx, cell, iq, nband, energy_eV, T, o0, o1, e0, e1, k0, k1, ng, nfreq, freq_eV,
                             delta_eV, wm, prec, accumulate, &c);
    if (st != RP_OK) return st;
    if (!M || !chi) return fail(ctx, RP_E_NULL, "NULL M or chi");
    if (!ctx->scratch) return fail(ctx, RP_E_DEVICE, "the fixed workspace has no device address on this GPU");
    // the workspace of rp_chi0_accumulate, carved from the fixed array in
    // 256-byte aligned pieces: frequencies, weights, split operands, partial tiles
    const long npair = (long)(k1 - k0) * (e1 - e0) * (o1 - o0);
    const ChiBytes nb = chi_bytes(c, npair);
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    const size_t off_f = 0, off_w = up(sizeof(double2) * nfreq);
    const size_t off_a = off_w + up(nb.w), off_b = off_a + up(nb.a), off_sw = off_b + up(nb.b);
    const size_t off_part = off_sw + up(nb.sw), need = off_part + up(nb.part);
    if (need > kScratchBytes)
        return fail(ctx, RP_E_SHAPE,
                    "this call needs %zu bytes of workspace, more than the fixed %zu (fewer pairs per call)", need,
                    kScratchBytes);
    char *base = (char *)ctx->scratch;
    if (hipMemcpyAsync(base + off_f, freq_eV, sizeof(double2) * nfreq, hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, RP_E_DEVICE, "host-to-device copy of the frequencies failed");
    }
    const ChiBufs bufs{(double2 *)(base + off_w), base + off_a, base + off_b, base + off_sw, base + off_part};
    return chi_enqueue(ctx, c, k0, k1, (const double2 *)M, (const double2 *)(base + off_f), bufs, accumulate,
                       (double2 *)chi);
}

rp_status rp_set_tuning(rp_ctx *ctx, int n, const rp_tune_entry *table)
{
    if (!ctx) return RP_E_NULL;
    if (n < 0) return fail(ctx, RP_E_RANGE, "n < 0");
    if (n > 0 && !table) return fail(ctx, RP_E_NULL, "table is NULL");
    for (int i = 0; i < n; i++) {
        const rp_tune_entry &e = table[i];
        if (e.ng_max < 1 || e.grid_max < 1) return fail(ctx, RP_E_RANGE, "entry %d: class bounds must be >= 1", i);
        if (e.chi_nw < 0 || e.chi_nw > 2) return fail(ctx, RP_E_RANGE, "entry %d: chi_nw must be 0, 1 or 2", i);
        if (e.chi_fill < -1 || e.chi_fill > (1 << 20))
            return fail(ctx, RP_E_RANGE, "entry %d: chi_fill outside [-1, 2^20]", i);
        if (e.fft_lines < 0 || e.fft_lines > 64) return fail(ctx, RP_E_RANGE, "entry %d: fft_lines outside [0, 64]", i);
        if (e.chi_kernel < 0 || e.chi_kernel > 2) return fail(ctx, RP_E_RANGE, "entry %d: chi_kernel must be 0, 1 or 2", i);
    }
    ctx->tuning.assign(table, table + n);
    return RP_OK;
}

// Enqueues steps a2-a6 for the k batch [ka, kb) of one problem: in FP64 the
// pair densities into ctx->mbuf and the contraction of them; in the split
// forms the pair kernels write the contraction's operands into bufs.a /
// bufs.b directly (no FP64 M), then the contraction.  dg and df are the
// device copies of the problem's G and frequency lists.
static rp_status kbatch_enqueue(rp_ctx *ctx, const PairJob &pj, const ChiJob &cj, int ka, int kb, const int *dg,
                                const double2 *df, void *grid, const ChiBufs &bufs, int accumulate, double2 *chi)
{
    rp_status st;
    if (cj.prec == RP_FP64) {
        double2 *M = (double2 *)ctx->mbuf.p;
        if ((st = pair_enqueue(ctx, pj, ka, kb, dg, grid, M)) != RP_OK) return st;
        return chi_enqueue(ctx, cj, ka, kb, M, df, bufs, accumulate, chi);
    }
    const long npair = (long)(kb - ka) * (pj.e1 - pj.e0) * (pj.o1 - pj.o0);
    const SplitOps ops = split_ops(bufs.a, bufs.b, npair, pj.ng, cj.prec == RP_SPLIT_BF16 ? 2 : 3);
    if ((st = pair_enqueue(ctx, pj, ka, kb, dg, grid, nullptr, &ops)) != RP_OK) return st;
    return chi_enqueue(ctx, cj, ka, kb, nullptr, df, bufs, accumulate, chi, true);
}

rp_status rp_chi0_run(rp_ctx *ctx, const rp_problem *p, rp_precision prec)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    if (!p) return fail(ctx, RP_E_NULL, "problem is NULL");
    if (!valid_prec(prec)) return fail(ctx, RP_E_RANGE, "unknown precision");
    PairJob pj;
    ChiJob cj;
    rp_status st = pair_check(ctx, &p->cell, p->iq, p->nband, p->npw_max, p->npw, p->mmax, p->miller, p->coef,
                              p->o0, p->o1, p->e0, p->e1, p->k0, p->k1, p->ng, p->gsph, prec, &pj);
    if (st != RP_OK) return st;
    if ((st = chi_check(ctx, &p->cell, p->iq, p->nband, p->energy_eV, p->T, p->o0, p->o1, p->e0, p->e1, p->k0,
                        p->k1, p->ng, p->nfreq, p->freq_eV, p->delta_eV, p->wm, prec, p->accumulate, &cj)) != RP_OK)
        return st;
    if (p->kbatch < 1) return fail(ctx, RP_E_SHAPE, "kbatch must be >= 1");
    if (!p->chi) return fail(ctx, RP_E_NULL, "chi is NULL");
    const long npk = (long)(p->o1 - p->o0) * (p->e1 - p->e0);
    const long npair = npk * std::min(p->kbatch, std::max(1, p->k1 - p->k0));
    const ChiBytes nb = chi_bytes(cj, pj.empty ? 0 : npair);
    DevBuf &grid = pj.fp32 ? ctx->ugrid32 : ctx->ugrid;
    if (!pj.empty) {
        if ((st = ensure(ctx, grid, pair_grid_bytes(pj))) != RP_OK) return st;
        if (prec == RP_FP64 && (st = ensure(ctx, ctx->mbuf, sizeof(double2) * (size_t)npair * p->ng)) != RP_OK)
            return st;
    }
    if ((st = ensure(ctx, ctx->weights, nb.w)) != RP_OK) return st;
    if (prec != RP_FP64) {
        if ((st = ensure(ctx, ctx->split_a, nb.a)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->split_b, nb.b)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->split_w, nb.sw)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->chi_part, nb.part)) != RP_OK) return st;
    }
    if ((st = upload(ctx, ctx->glist, p->gsph, sizeof(int) * 3 * p->ng)) != RP_OK) return st;
    if ((st = upload(ctx, ctx->freq, p->freq_eV, sizeof(double2) * p->nfreq)) != RP_OK) return st;
    const int *dg = (const int *)ctx->glist.p;
    const double2 *df = (const double2 *)ctx->freq.p;
    const ChiBufs bufs{(double2 *)ctx->weights.p, ctx->split_a.p, ctx->split_b.p, ctx->split_w.p,
                       ctx->chi_part.p};
    double2 *chi = (double2 *)p->chi;
    if (pj.empty) return chi_enqueue(ctx, cj, p->k0, p->k0, nullptr, df, bufs, p->accumulate, chi);
    for (int ka = p->k0; ka < p->k1; ka += p->kbatch) {
        const int kb = std::min(p->k1, ka + p->kbatch);
        if ((st = kbatch_enqueue(ctx, pj, cj, ka, kb, dg, df, grid.p, bufs, ka == p->k0 ? p->accumulate : 1,
                                 chi)) != RP_OK)
            return st;
    }
    return RP_OK;
}

// ---- batch of chi0 problems as one graph launch ----------------------------

// bound on the kernel nodes of one captured graph of a batch
constexpr long kGraphNodes = 2048;


rp_status rp_chi0_batch(rp_ctx *ctx, int nprob, const rp_problem *probs, rp_precision prec)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    if (nprob < 0) return fail(ctx, RP_E_SHAPE, "nprob < 0");
    if (nprob > 0 && !probs) return fail(ctx, RP_E_NULL, "probs is NULL");
    if (!valid_prec(prec)) return fail(ctx, RP_E_RANGE, "unknown precision");
    if (nprob == 0) return RP_OK;
    std::vector<PairJob> pj(nprob);
    std::vector<ChiJob> cj(nprob);
    std::vector<size_t> goff(nprob), foff(nprob);
    size_t grid_b = 0, m_b = 0, stage_b = 0;
    ChiBytes cb;
    auto round_up = [](size_t n) { return (n + 255) / 256 * 256; };
    for (int i = 0; i < nprob; i++) {
        const rp_problem &p = probs[i];
        rp_status st = pair_check(ctx, &p.cell, p.iq, p.nband, p.npw_max, p.npw, p.mmax, p.miller, p.coef, p.o0,
                                  p.o1, p.e0, p.e1, p.k0, p.k1, p.ng, p.gsph, prec, &pj[i]);
        if (st == RP_OK)
            st = chi_check(ctx, &p.cell, p.iq, p.nband, p.energy_eV, p.T, p.o0, p.o1, p.e0, p.e1, p.k0, p.k1, p.ng,
                           p.nfreq, p.freq_eV, p.delta_eV, p.wm, prec, p.accumulate, &cj[i]);
        if (st == RP_OK && p.kbatch < 1) st = fail(ctx, RP_E_SHAPE, "kbatch must be >= 1");
        if (st == RP_OK && !p.chi) st = fail(ctx, RP_E_NULL, "chi is NULL");
        if (st != RP_OK) {
            ctx->err = "problem " + std::to_string(i) + ": " + ctx->err;
            return st;
        }
        const long npk = (long)(p.o1 - p.o0) * (p.e1 - p.e0);
        const long npair = npk * std::min(p.kbatch, std::max(1, p.k1 - p.k0));
        if (!pj[i].empty) {
            grid_b = std::max(grid_b, pair_grid_bytes(pj[i]));
            if (prec == RP_FP64) m_b = std::max(m_b, sizeof(double2) * (size_t)npair * p.ng);
        }
        const ChiBytes b = chi_bytes(cj[i], pj[i].empty ? 0 : npair);
        cb.w = std::max(cb.w, b.w);
        cb.a = std::max(cb.a, b.a);
        cb.b = std::max(cb.b, b.b);
        cb.sw = std::max(cb.sw, b.sw);
        cb.part = std::max(cb.part, b.part);
        goff[i] = stage_b;
        stage_b += round_up(sizeof(int) * 3 * p.ng);
        foff[i] = stage_b;
        stage_b += round_up(sizeof(double2) * p.nfreq);
    }
    const bool fp32 = prec != RP_FP64;
    DevBuf &grid = fp32 ? ctx->ugrid32 : ctx->ugrid;
    rp_status st;
    if ((st = ensure(ctx, grid, grid_b)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->mbuf, m_b)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->weights, cb.w)) != RP_OK) return st;
    if (fp32) {
        if ((st = ensure(ctx, ctx->split_a, cb.a)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->split_b, cb.b)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->split_w, cb.sw)) != RP_OK) return st;
        if ((st = ensure(ctx, ctx->chi_part, cb.part)) != RP_OK) return st;
    }
    // host staging of every G list and frequency list, one copy to the device
    std::vector<char> stage(stage_b, 0);
    for (int i = 0; i < nprob; i++) {
        memcpy(stage.data() + goff[i], probs[i].gsph, sizeof(int) * 3 * probs[i].ng);
        memcpy(stage.data() + foff[i], probs[i].freq_eV, sizeof(double2) * probs[i].nfreq);
    }
    // the graph depends on every launch argument: the problems' scalars and
    // pointers, the host arrays read at enqueue time, and the workspaces
    std::string key;
    key_val(key, prec);
    key_val(key, nprob);
    for (int i = 0; i < nprob; i++) {
        const rp_problem &p = probs[i];
        key_val(key, p.cell);
        key_put(key, p.iq, sizeof p.iq);
        const int ints[] = {p.nband, p.npw_max, p.o0, p.o1, p.e0, p.e1, p.k0, p.k1, p.ng, p.nfreq, (int)p.wm,
                            p.kbatch, p.accumulate};
        key_put(key, ints, sizeof ints);
        key_put(key, p.mmax, sizeof p.mmax);
        key_put(key, p.npw, sizeof(int) * pj[i].g.nk);
        const void *ptrs[] = {p.miller, p.coef, p.energy_eV, p.T, p.chi};
        key_put(key, ptrs, sizeof ptrs);
        key_val(key, p.delta_eV);
        key_val(key, cj[i].ef);
        const int tn[] = {cj[i].tune.chi_nw, cj[i].tune.chi_fill, cj[i].tune.chi_kernel, pj[i].fft_lines};
        key_put(key, tn, sizeof tn);
    }
    key_put(key, stage.data(), stage.size());
    const void *ws[] = {grid.p,          ctx->mbuf.p,    ctx->weights.p, ctx->split_a.p,
                        ctx->split_b.p, ctx->split_w.p, ctx->chi_part.p};
    key_put(key, ws, sizeof ws);

    if (ctx->batch_execs.empty() || key != ctx->batch_key) {
        if (!ctx->batch_execs.empty()) {
            if (hipStreamSynchronize(ctx->stream) != hipSuccess)
                return fail(ctx, RP_E_DEVICE, "stream synchronize failed before replacing the batch graphs");
            for (hipGraphExec_t e : ctx->batch_execs) (void)hipGraphExecDestroy(e);
            ctx->batch_execs.clear();
            ctx->batch_nodes = 0;
            ctx->batch_key.clear();
        }
        if ((st = upload(ctx, ctx->bstage, stage.data(), stage.size())) != RP_OK) return st;
        const char *dstage = (const char *)ctx->bstage.p;
        const ChiBufs bufs{(double2 *)ctx->weights.p, ctx->split_a.p, ctx->split_b.p, ctx->split_w.p,
                           ctx->chi_part.p};
        // The launches are captured as a sequence of graphs of at most about
        // kGraphNodes kernel nodes each (a graph closes after the k batch that
        // reaches the bound), launched in order on the stream: the same launches
        // as one graph, without a serial chain of tens of thousands of nodes
        // for the runtime (or a profiler) to walk.
        std::vector<hipGraphExec_t> execs;
        long nodes = 0, piece = 0;
        bool in_capture = false;
        auto drop = [&]() {
            for (hipGraphExec_t e : execs) (void)hipGraphExecDestroy(e);
        };
        auto begin_piece = [&]() -> rp_status {
            if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, RP_E_DEVICE, "stream capture could not begin");
            }
            ctx->capturing = true;
            in_capture = true;
            piece = 0;
            return RP_OK;
        };
        auto end_piece = [&](rp_status prior) -> rp_status {
            ctx->capturing = false;
            in_capture = false;
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
            if (prior != RP_OK || ec != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                if (prior != RP_OK) {
                    ctx->err = "batch capture: " + ctx->err;
                    return prior;
                }
                return fail(ctx, RP_E_DEVICE, "stream capture failed: %s", hipGetErrorString(ec));
            }
            size_t n = 0;
            (void)hipGraphGetNodes(graph, nullptr, &n);
            hipGraphExec_t exec = nullptr;
            const hipError_t ei = n ? hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) : hipSuccess;
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, RP_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
            }
            if (exec) execs.push_back(exec);
            nodes += (long)n;
            return RP_OK;
        };
        // an upper bound on the kernels one k batch of kb k-points enqueues:
        // per k the u-grids (a plane sort, the planar transforms and the axis-1
        // pass; or, for grids too large for that, a zero fill, two scatters and
        // three passes) and the pair kernel; per batch the weights, two
        // preparation kernels (operands or their padding, and the weights), the
        // contraction and the sum of its partial tiles
        auto bound = [](int kb) { return 8L * kb + 6; };
        st = begin_piece();
        for (int i = 0; i < nprob && st == RP_OK; i++) {
            const rp_problem &p = probs[i];
            const int *dg = (const int *)(dstage + goff[i]);
            const double2 *df = (const double2 *)(dstage + foff[i]);
            double2 *chi = (double2 *)p.chi;
            if (pj[i].empty) {
                // no pairs: chi is overwritten with zero or left as it is
                st = chi_enqueue(ctx, cj[i], p.k0, p.k0, nullptr, df, bufs, p.accumulate, chi);
                piece += bound(0);
                continue;
            }
            for (int ka = p.k0; ka < p.k1 && st == RP_OK; ka += p.kbatch) {
                const int kb = std::min(p.k1, ka + p.kbatch);
                if (piece > 0 && piece + bound(kb - ka) > kGraphNodes) {
                    if ((st = end_piece(RP_OK)) != RP_OK || (st = begin_piece()) != RP_OK) break;
                }
                st = kbatch_enqueue(ctx, pj[i], cj[i], ka, kb, dg, df, grid.p, bufs, ka == p.k0 ? p.accumulate : 1,
                                    chi);
                piece += bound(kb - ka);
            }
        }
        if (in_capture) st = end_piece(st);
        if (st != RP_OK) {
            drop();
            return st;
        }
        ctx->batch_execs = std::move(execs);
        ctx->batch_nodes = nodes;
        ctx->batch_key = key;
    }
    {
        StageTimer t(ctx, RP_STAGE_BATCH);
        for (hipGraphExec_t e : ctx->batch_execs)
            if (hipGraphLaunch(e, ctx->stream) != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, RP_E_DEVICE, "graph launch failed");
            }
    }
    return RP_OK;
}

rp_status rp_chi0_batch_graphs(rp_ctx *ctx, int *graphs, long *nodes)
{
    if (!ctx) return RP_E_NULL;
    if (!graphs || !nodes) return fail(ctx, RP_E_NULL, "NULL output");
    *graphs = (int)ctx->batch_execs.size();
    *nodes = ctx->batch_nodes;
    return RP_OK;
}

rp_status rp_screen_W(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int ng, const int *gsph,
                      int nfreq, const double *chi, double *eps_inv, double *W)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    Geometry g;
    rp_status st = geometry(ctx, cell, iq, &g);
    if (st != RP_OK) return st;
    if (!chi) return fail(ctx, RP_E_NULL, "chi is NULL");
    if (ng < 1 || nfreq < 1) return fail(ctx, RP_E_SHAPE, "ng and nfreq must be >= 1");
    if (ng > 6144) return fail(ctx, RP_E_UNSUPPORTED, "ng = %d above 6144", ng);
    if ((st = check_gsph(ctx, g, ng, gsph, "gsph")) != RP_OK) return st;
    const size_t mat = sizeof(double2) * (size_t)ng * ng * nfreq;
    double2 *a = (double2 *)eps_inv;
    if (!a) {
        if ((st = ensure(ctx, ctx->work, mat)) != RP_OK) return st;
        a = (double2 *)ctx->work.p;
    }
    if ((st = upload(ctx, ctx->glist, gsph, sizeof(int) * 3 * ng)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->vsqrt, sizeof(double) * ng)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->piv, sizeof(int) * (size_t)ng * nfreq)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->rho, invert_scratch_bytes(ng, nfreq))) != RP_OK) return st;
    double *vs = (double *)ctx->vsqrt.p;
    StageTimer t(ctx, RP_STAGE_SCREEN);
    launch_vsqrt(ctx->stream, g, ng, (const int *)ctx->glist.p, vs, ctx->flag);
    launch_eps(ctx->stream, nfreq, ng, vs, (const double2 *)chi, a, ctx->flag);
    launch_invert(ctx->stream, nfreq, ng, a, (double2 *)ctx->rho.p, (int *)ctx->piv.p, ctx->flag);
    if (W) launch_W(ctx->stream, nfreq, ng, vs, a, (double2 *)W);
    return check_launch(ctx, "screen");
}

rp_status rp_head_density(rp_ctx *ctx, const rp_cell *cell, int nband, int npw_max, const int *npw,
                          const int *miller, const double *coef, const double *energy_eV, int o0, int o1, int e0,
                          int e1, int k0, int k1, const double qhat[3], int ng, int col, double *M)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    Geometry g;
    const int iq0[3] = {0, 0, 0};
    rp_status st = geometry(ctx, cell, iq0, &g);
    if (st != RP_OK) return st;
    if (!npw || !miller || !coef || !energy_eV || !qhat || !M) return fail(ctx, RP_E_NULL, "NULL array argument");
    if ((st = check_ranges(ctx, g, nband, o0, o1, e0, e1, k0, k1)) != RP_OK) return st;
    if (npw_max < 1) return fail(ctx, RP_E_SHAPE, "npw_max must be >= 1");
    for (int k = 0; k < g.nk; k++)
        if (npw[k] < 0 || npw[k] > npw_max) return fail(ctx, RP_E_SHAPE, "npw[%d] outside [0, npw_max]", k);
    if (ng < 1 || col < 0 || col >= ng) return fail(ctx, RP_E_SHAPE, "col = %d outside [0, ng = %d)", col, ng);
    const double qn = std::sqrt(qhat[0] * qhat[0] + qhat[1] * qhat[1] + qhat[2] * qhat[2]);
    if (!(qn > 0.0) || !std::isfinite(qn)) return fail(ctx, RP_E_RANGE, "qhat must be a finite non-zero vector");
    if ((long)(o1 - o0) * (e1 - e0) * (k1 - k0) == 0) return RP_OK;
    const double qu[3] = {qhat[0] / qn, qhat[1] / qn, qhat[2] / qn};
    if ((st = upload(ctx, ctx->kinfo, npw, sizeof(int) * g.nk)) != RP_OK) return st;
    {
        StageTimer t(ctx, RP_STAGE_PAIR);
        launch_head(ctx->stream, g, miller, (const double2 *)coef, energy_eV, (const int *)ctx->kinfo.p, nband,
                    npw_max, o0, o1, e0, e1, k0, k1, qu, ng, col, (double2 *)M, ctx->flag);
    }
    return check_launch(ctx, "head density");
}

rp_status rp_plasma_frequency(rp_ctx *ctx, const rp_cell *cell, int nband, int npw_max, const int *npw,
                              const int *miller, const double *coef, const double *energy_eV, const double *T, int b0,
                              int b1, double ef_eV, double *omega2_eV2)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    Geometry g;
    const int iq0[3] = {0, 0, 0};
    rp_status st = geometry(ctx, cell, iq0, &g);
    if (st != RP_OK) return st;
    if (!npw || !miller || !coef || !energy_eV || !omega2_eV2) return fail(ctx, RP_E_NULL, "NULL array argument");
    if (nband < 1 || b0 < 0 || b1 > nband || b0 > b1)
        return fail(ctx, RP_E_RANGE, "band range [%d, %d) outside [0, nband = %d)", b0, b1, nband);
    if (npw_max < 1) return fail(ctx, RP_E_SHAPE, "npw_max must be >= 1");
    for (int k = 0; k < g.nk; k++)
        if (npw[k] < 0 || npw[k] > npw_max) return fail(ctx, RP_E_SHAPE, "npw[%d] outside [0, npw_max]", k);
    if (!std::isfinite(ef_eV)) return fail(ctx, RP_E_RANGE, "non-finite Fermi level");
    const long n = (long)g.nk * (b1 - b0);
    // workspace (doubles): p [n][3] | contributions [n][6] | sums [6]
    if ((st = ensure(ctx, ctx->work, sizeof(double) * (9 * (size_t)n + 6))) != RP_OK) return st;
    if ((st = upload(ctx, ctx->kinfo, npw, sizeof(int) * g.nk)) != RP_OK) return st;
    double *p = (double *)ctx->work.p, *contrib = p + 3 * n, *sums = contrib + 6 * n;
    launch_pdiag(ctx->stream, g, miller, (const double2 *)coef, (const int *)ctx->kinfo.p, nband, npw_max, b0, b1, p);
    launch_fermi_plasma(ctx->stream, g.kmesh, nband, energy_eV, T, b0, b1, ef_eV, p, contrib, sums);
    if ((st = check_launch(ctx, "plasma frequency")) != RP_OK) return st;
    double h[6];
    if (hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return fail(ctx, RP_E_DEVICE, "plasma frequency: copy to host failed");
    // (4 pi / Omega) x 2 (spin) in hartree^2, then eV^2
    const double s = 4.0 * kPi / g.volume * 2.0 * kHartreeEv * kHartreeEv;
    const int ix[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
    for (int i = 0; i < 9; i++) omega2_eV2[i] = s * h[ix[i]];
    return RP_OK;
}

rp_status rp_set_drude(rp_ctx *ctx, double wq_eV2, double delta_eV)
{
    if (!ctx) return RP_E_NULL;
    if (!std::isfinite(wq_eV2) || !std::isfinite(delta_eV) || delta_eV < 0.0)
        return fail(ctx, RP_E_RANGE, "the intraband term needs finite wq and delta >= 0");
    ctx->drude_wq = wq_eV2;
    ctx->drude_delta = delta_eV;
    return RP_OK;
}

rp_status rp_screen_head(rp_ctx *ctx, const rp_cell *cell, int ng, const int *gsph, int nfreq,
                         const double *freq_eV, const double *chi, double *eps_inv, double *optics)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    Geometry g;
    const int iq0[3] = {0, 0, 0};
    rp_status st = geometry(ctx, cell, iq0, &g);
    if (st != RP_OK) return st;
    if (!chi || !gsph || !freq_eV) return fail(ctx, RP_E_NULL, "NULL array argument");
    if (ng < 1 || nfreq < 1) return fail(ctx, RP_E_SHAPE, "ng and nfreq must be >= 1");
    if (ng > 6144) return fail(ctx, RP_E_UNSUPPORTED, "ng = %d above 6144", ng);
    if (gsph[0] != 0 || gsph[1] != 0 || gsph[2] != 0) return fail(ctx, RP_E_RANGE, "gsph[0] must be G = 0");
    if ((st = check_gsph(ctx, g, ng - 1, gsph + 3, "gsph[1:]")) != RP_OK) return st;
    for (int f = 0; f < 2 * nfreq; f++)
        if (!std::isfinite(freq_eV[f])) return fail(ctx, RP_E_RANGE, "non-finite frequency");
    const size_t mat = sizeof(double2) * (size_t)ng * ng * nfreq;
    double2 *a = (double2 *)eps_inv;
    if (!a) {
        if ((st = ensure(ctx, ctx->work, mat)) != RP_OK) return st;
        a = (double2 *)ctx->work.p;
    }
    if ((st = upload(ctx, ctx->glist, gsph, sizeof(int) * 3 * ng)) != RP_OK) return st;
    if ((st = upload(ctx, ctx->freq, freq_eV, sizeof(double2) * nfreq)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->vsqrt, sizeof(double) * ng)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->piv, sizeof(int) * (size_t)ng * nfreq)) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->rho, invert_scratch_bytes(ng, nfreq))) != RP_OK) return st;
    double *vs = (double *)ctx->vsqrt.p;
    StageTimer t(ctx, RP_STAGE_SCREEN);
    launch_vsqrt(ctx->stream, g, ng, (const int *)ctx->glist.p, vs, ctx->flag, true);
    launch_eps(ctx->stream, nfreq, ng, vs, (const double2 *)chi, a, ctx->flag);
    const double2 *fq = (const double2 *)ctx->freq.p;
    const bool drude = ctx->drude_wq != 0.0;
    if (drude) launch_drude_head(ctx->stream, nfreq, ng, fq, ctx->drude_wq, ctx->drude_delta, a);
    launch_invert(ctx->stream, nfreq, ng, a, (double2 *)ctx->rho.p, (int *)ctx->piv.p, ctx->flag);
    if (drude) launch_drude_zero(ctx->stream, nfreq, ng, fq, ctx->drude_delta, a);
    if (optics) launch_optics(ctx->stream, nfreq, ng, a, fq, optics);
    return check_launch(ctx, "screen head");
}

rp_status rp_wannier_W(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nwan, const double *phi,
                       const double *centre_frac, int ng, const int *gsph, int ntail, const int *gtail,
                       int nfreq, const double *eps_inv, double *Wij)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    Geometry g;
    rp_status st = geometry(ctx, cell, iq, &g);
    if (st != RP_OK) return st;
    if (!phi || !centre_frac || !eps_inv || !Wij) return fail(ctx, RP_E_NULL, "NULL array argument");
    if (nwan < 1 || nwan > 32) return fail(ctx, RP_E_UNSUPPORTED, "nwan = %d outside [1, 32]", nwan);
    if (ng < 1 || nfreq < 1 || ntail < 0) return fail(ctx, RP_E_SHAPE, "bad ng, ntail or nfreq");
    if ((st = check_gsph(ctx, g, ng, gsph, "gsph")) != RP_OK) return st;
    if ((st = check_gsph(ctx, g, ntail, gtail, "gtail")) != RP_OK) return st;
    for (int i = 0; i < 3 * nwan; i++)
        if (!std::isfinite(centre_frac[i])) return fail(ctx, RP_E_RANGE, "non-finite centre");
    FftPlan plans[3];
    if ((st = plans3(ctx, g, plans)) != RP_OK) return st;
    const long nr = (long)g.fft[0] * g.fft[1] * g.fft[2];
    // layout of the Wannier workspace (double2 units):
    //   grids [nwan][nr] | rho_eps [nwan][ng] | rho_tail [nwan][ntail] | T [nfreq][ng][nwan]
    const size_t n_grid = (size_t)nwan * nr, n_re = (size_t)nwan * ng, n_rt = (size_t)nwan * ntail;
    const size_t n_T = (size_t)nfreq * ng * nwan;
    if ((st = ensure(ctx, ctx->work, sizeof(double2) * (n_grid + n_re + n_rt + n_T))) != RP_OK) return st;
    // host lists: centres, gsph, gtail packed into one upload
    std::vector<char> host(sizeof(double) * 3 * nwan + sizeof(int) * 3 * (ng + ntail));
    std::memcpy(host.data(), centre_frac, sizeof(double) * 3 * nwan);
    std::memcpy(host.data() + sizeof(double) * 3 * nwan, gsph, sizeof(int) * 3 * ng);
    if (ntail) std::memcpy(host.data() + sizeof(double) * 3 * nwan + sizeof(int) * 3 * ng, gtail, sizeof(int) * 3 * ntail);
    if ((st = upload(ctx, ctx->kinfo, host.data(), host.size())) != RP_OK) return st;
    const double *dcen = (const double *)ctx->kinfo.p;
    const int *dgs = (const int *)((const char *)ctx->kinfo.p + sizeof(double) * 3 * nwan);
    const int *dgt = dgs + 3 * ng;
    double2 *grids = (double2 *)ctx->work.p;
    double2 *rho_e = grids + n_grid;
    double2 *rho_t = rho_e + n_re;
    double2 *T = rho_t + n_rt;
    StageTimer t(ctx, RP_STAGE_WANNIER);
    launch_wannier_density(ctx->stream, g, plans, nwan, phi, dcen, grids);
    launch_wannier_gather(ctx->stream, g, nwan, ng, dgs, grids, rho_e, ctx->flag);
    launch_wannier_gather(ctx->stream, g, nwan, ntail, dgt, grids, rho_t, ctx->flag);
    const double pre = kHartreeEv * 4.0 * kPi / (g.volume * g.nk);
    launch_wannier_W(ctx->stream, nfreq, nwan, ng, rho_e, ntail, rho_t, (const double2 *)eps_inv, pre, T,
                     (double2 *)Wij);
    return check_launch(ctx, "wannier projection");
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the
// Legendre recurrence, starting from the usual cosine estimates).
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; i++) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Mean of 1/|q|^2 over the q-cell around Gamma: the cell (edges e_a = b_a /
// K_a, x in [-1/2, 1/2)^3) is cut into six pyramids with apex at Gamma, one
// per face; with q = t p (p on the face, t in [0, 1]) a pyramid over a face
// at distance h contributes h int_face dA / |p|^2, integrated by composite
// Gauss-Legendre quadrature (8 panels x 16 nodes per side).
static double cell_average(const Geometry &g)
{
    constexpr int kNodes = 16, kPanels = 8;
    double gx[kNodes], gw[kNodes];
    gauss_legendre(kNodes, gx, gw);
    double e[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) e[a][b] = g.rec[3 * a + b] / g.kmesh[a];
    double total = 0.0;
    for (int a = 0; a < 3; a++) {
        const double *u = e[(a + 1) % 3], *v = e[(a + 2) % 3];
        const double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        const double area = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const double c[3] = {0.5 * sgn * e[a][0], 0.5 * sgn * e[a][1], 0.5 * sgn * e[a][2]};
            const double h = std::fabs(c[0] * n[0] + c[1] * n[1] + c[2] * n[2]) / area;
            double face = 0.0;
            for (int px = 0; px < kPanels; px++)
                for (int ix = 0; ix < kNodes; ix++) {
                    const double x = -0.5 + (px + 0.5 * (gx[ix] + 1.0)) / kPanels;
                    for (int py = 0; py < kPanels; py++)
                        for (int iy = 0; iy < kNodes; iy++) {
                            const double y = -0.5 + (py + 0.5 * (gx[iy] + 1.0)) / kPanels;
                            double p2 = 0.0;
                            for (int d = 0; d < 3; d++) {
                                const double pd = c[d] + x * u[d] + y * v[d];
                                p2 += pd * pd;
                            }
                            face += gw[ix] * gw[iy] / p2;
                        }
                }
            // each panel maps [-1, 1] onto a width of 1/kPanels: Jacobian (1/(2 kPanels))^2
            total += h * area * face / (4.0 * kPanels * kPanels);
        }
    }
    return (double)g.nk * g.volume / std::pow(2.0 * kPi, 3) * total;
}

// Eq. grid.  The first branch is omega_i = dw (1 + s + ... + s^(i-2)); the
// condition omega_{N_max} = E_max makes s the root of
// g(s) = 1 + s + ... + s^(N_max-2) - E_max/dw, increasing on s > 0 with
// g(0) = 1 - E_max/dw < 0, found by bisection.  The second branch is
// E_max 3^((i - N_max)/(N_Omega - N_max)).
rp_status rp_frequency_grid(double emax_eV, double dw_eV, int nomega, int nmax, double *omega_eV)
{
    if (!omega_eV) return RP_E_NULL;
    if (nomega < 3) return RP_E_SHAPE;
    if (nmax == 0) nmax = 9 * nomega / 10;
    if (nmax < 2 || nmax >= nomega) return RP_E_SHAPE;
    if (!(dw_eV > 0.0) || !(emax_eV > dw_eV) || !std::isfinite(emax_eV)) return RP_E_RANGE;
    const double r = emax_eV / dw_eV;
    auto g = [&](double x) {
        double sum = 0.0, p = 1.0;
        for (int j = 0; j <= nmax - 2; j++) {
            sum += p;
            p *= x;
        }
        return sum - r;
    };
    double lo = 0.0, hi = 2.0;
    while (g(hi) <= 0.0) hi *= 2.0;
    for (int it = 0; it < 200 && hi - lo > 0.0; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        (g(mid) < 0.0 ? lo : hi) = mid;
    }
    const double sr = 0.5 * (lo + hi);
    double sum = 0.0, p = 1.0;
    omega_eV[0] = 0.0;
    for (int i = 2; i <= nmax; i++) {
        sum += p;
        p *= sr;
        omega_eV[i - 1] = dw_eV * sum;
    }
    for (int i = nmax + 1; i <= nomega; i++)
        omega_eV[i - 1] = emax_eV * std::exp(std::log(3.0) * (double)(i - nmax) / (double)(nomega - nmax));
    return RP_OK;
}

// ---- symmetry unfolding (Eqs. coef-G, symeps) ----

// S = W^{-T} for an integer W with det W = +-1 (row-major); false otherwise
static bool op_inverse_transpose(const int W[9], int S[9])
{
    const long det = (long)W[0] * (W[4] * W[8] - W[5] * W[7]) - (long)W[1] * (W[3] * W[8] - W[5] * W[6]) +
                     (long)W[2] * (W[3] * W[7] - W[4] * W[6]);
    if (det != 1 && det != -1) return false;
    // W^{-1} = adj(W) / det, so S[i][j] = W^{-1}[j][i] = cof(W)[i][j] / det
    const int c[9] = {W[4] * W[8] - W[5] * W[7], W[5] * W[6] - W[3] * W[8], W[3] * W[7] - W[4] * W[6],
                      W[2] * W[7] - W[1] * W[8], W[0] * W[8] - W[2] * W[6], W[1] * W[6] - W[0] * W[7],
                      W[1] * W[5] - W[2] * W[4], W[2] * W[3] - W[0] * W[5], W[0] * W[4] - W[1] * W[3]};
    for (int i = 0; i < 9; i++) S[i] = (int)(c[i] / det);
    return true;
}

// Delta = k - S k* for mesh indices n, n* (k = n / K), required integral
static rp_status op_rewind(rp_ctx *ctx, const Geometry &g, const int S[9], const int nirr[3], const int n[3],
                           int delta[3])
{
    for (int a = 0; a < 3; a++)
        if (nirr[a] < 0 || nirr[a] >= g.kmesh[a] || n[a] < 0 || n[a] >= g.kmesh[a])
            return fail(ctx, RP_E_RANGE, "mesh index outside the mesh");
    for (int a = 0; a < 3; a++) {
        double sk = 0.0;
        for (int b = 0; b < 3; b++) sk += S[3 * a + b] * ((double)nirr[b] / g.kmesh[b]);
        const double d = (double)n[a] / g.kmesh[a] - sk;
        const double r = std::nearbyint(d);
        if (std::fabs(d - r) > 1e-9) return fail(ctx, RP_E_RANGE, "the point is not the image of k* under the operation");
        delta[a] = (int)r;
    }
    return RP_OK;
}

static inline long long miller_key(int a, int b, int c)
{
    return ((long long)(a + (1 << 20)) << 42) | ((long long)(b + (1 << 20)) << 21) | (long long)(c + (1 << 20));
}

// src_idx[g] = position in `from` of W^T (m_g + Delta) for each vector of `to`
static rp_status op_source_index(rp_ctx *ctx, const int W[9], const int delta[3], int nfrom, const int *from, int nto,
                                 const int *to, std::vector<int> &src_idx)
{
    std::unordered_map<long long, int> where;
    where.reserve((size_t)nfrom * 2);
    for (int i = 0; i < nfrom; i++) where.emplace(miller_key(from[3 * i], from[3 * i + 1], from[3 * i + 2]), i);
    src_idx.resize(nto);
    for (int g = 0; g < nto; g++) {
        const int v[3] = {to[3 * g] + delta[0], to[3 * g + 1] + delta[1], to[3 * g + 2] + delta[2]};
        int m[3];
        for (int a = 0; a < 3; a++) m[a] = W[a] * v[0] + W[3 + a] * v[1] + W[6 + a] * v[2];   // (W^T v)_a
        const auto it = where.find(miller_key(m[0], m[1], m[2]));
        if (it == where.end())
            return fail(ctx, RP_E_RANGE, "target vector %d (%d %d %d) has no source vector", g, to[3 * g],
                        to[3 * g + 1], to[3 * g + 2]);
        src_idx[g] = it->second;
    }
    return RP_OK;
}

static rp_status check_op(rp_ctx *ctx, const int W[9], const double t[3], int S[9])
{
    if (!W || !t) return fail(ctx, RP_E_NULL, "W or t is NULL");
    if (!op_inverse_transpose(W, S)) return fail(ctx, RP_E_RANGE, "W is not an integer matrix of determinant +-1");
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(t[a])) return fail(ctx, RP_E_RANGE, "non-finite translation");
    return RP_OK;
}

rp_status rp_unfold_coef(rp_ctx *ctx, const rp_cell *cell, const int W[9], const double t[3], const int ik_irr[3],
                         int nband, int npw_irr, const int *miller_irr, const double *coef_irr, long ld_irr,
                         const int ik[3], int npw, const int *miller, double *coef, long ld)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    const int iq0[3] = {0, 0, 0};
    Geometry g;
    rp_status st = geometry(ctx, cell, iq0, &g);
    if (st != RP_OK) return st;
    int S[9], delta[3];
    if ((st = check_op(ctx, W, t, S)) != RP_OK) return st;
    if (!ik_irr || !ik) return fail(ctx, RP_E_NULL, "mesh index is NULL");
    if ((st = op_rewind(ctx, g, S, ik_irr, ik, delta)) != RP_OK) return st;
    if (nband < 1 || npw_irr < 1 || npw < 0 || ld_irr < npw_irr || ld < npw)
        return fail(ctx, RP_E_SHAPE, "bad nband, plane-wave counts or leading dimensions");
    if (!miller_irr || !coef_irr || (npw > 0 && (!miller || !coef))) return fail(ctx, RP_E_NULL, "NULL array argument");
    std::vector<int> idx;
    if ((st = op_source_index(ctx, W, delta, npw_irr, miller_irr, npw, miller, idx)) != RP_OK) return st;
    if (npw == 0) return RP_OK;
    std::vector<int> host((size_t)4 * npw);
    std::memcpy(host.data(), idx.data(), sizeof(int) * npw);
    std::memcpy(host.data() + npw, miller, sizeof(int) * 3 * npw);
    if ((st = upload(ctx, ctx->kinfo, host.data(), sizeof(int) * host.size())) != RP_OK) return st;
    const int *didx = (const int *)ctx->kinfo.p;
    StageTimer tm(ctx, RP_STAGE_UNFOLD);
    launch_unfold_coef(ctx->stream, nband, npw, didx, didx + npw, delta, t, (const double2 *)coef_irr, ld_irr,
                       (double2 *)coef, ld);
    return check_launch(ctx, "coefficient unfolding");
}

rp_status rp_unfold_eps_inv(rp_ctx *ctx, const rp_cell *cell, const int W[9], const double t[3], const int iq_irr[3],
                            int ng_irr, const int *gsph_irr, const int iq[3], int ng, const int *gsph, int nfreq,
                            const double *src, double *dst)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    const int iq0[3] = {0, 0, 0};
    Geometry g;
    rp_status st = geometry(ctx, cell, iq0, &g);
    if (st != RP_OK) return st;
    int S[9], delta[3];
    if ((st = check_op(ctx, W, t, S)) != RP_OK) return st;
    if (!iq_irr || !iq) return fail(ctx, RP_E_NULL, "mesh index is NULL");
    if ((st = op_rewind(ctx, g, S, iq_irr, iq, delta)) != RP_OK) return st;
    if (ng_irr < 1 || ng < 1 || ng > 6144 || nfreq < 1) return fail(ctx, RP_E_SHAPE, "bad ng, ng_irr or nfreq");
    if (!gsph_irr || !gsph || !src || !dst) return fail(ctx, RP_E_NULL, "NULL array argument");
    if (src == dst) return fail(ctx, RP_E_ALIAS, "source and destination must differ");
    std::vector<int> idx;
    if ((st = op_source_index(ctx, W, delta, ng_irr, gsph_irr, ng, gsph, idx)) != RP_OK) return st;
    std::vector<int> host((size_t)4 * ng);
    std::memcpy(host.data(), idx.data(), sizeof(int) * ng);
    std::memcpy(host.data() + ng, gsph, sizeof(int) * 3 * ng);
    if ((st = upload(ctx, ctx->kinfo, host.data(), sizeof(int) * host.size())) != RP_OK) return st;
    if ((st = ensure(ctx, ctx->work, sizeof(double2) * (size_t)ng)) != RP_OK) return st;
    const int *didx = (const int *)ctx->kinfo.p;
    StageTimer tm(ctx, RP_STAGE_UNFOLD);
    launch_unfold_matrix(ctx->stream, nfreq, ng, ng_irr, didx, didx + ng, t, (double2 *)ctx->work.p,
                         (const double2 *)src, (double2 *)dst);
    return check_launch(ctx, "eps^-1 unfolding");
}

rp_status rp_set_fermi_level(rp_ctx *ctx, double ef_eV)
{
    if (!ctx) return RP_E_NULL;
    ctx->fermi_eV = ef_eV;
    return RP_OK;
}

rp_status rp_coulomb_cell_average(const rp_cell *cell, double *avg)
{
    if (!avg) return RP_E_NULL;
    const int iq0[3] = {0, 0, 0};
    Geometry g;
    const rp_status st = geometry(nullptr, cell, iq0, &g);
    if (st != RP_OK) return st;
    *avg = cell_average(g);
    return RP_OK;
}

rp_status rp_wannier_qterm(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nwan, const double *phi,
                           const double *centre_frac, int nR, const int *R, int ng, const int *gsph, int ntail,
                           const int *gtail, int nfreq, const double *eps_inv, int accumulate, double *U,
                           double *J, double *V, double *X)
{
    if (!ctx) return RP_E_NULL;
    (void)hipSetDevice(ctx->device);
    Geometry g;
    rp_status st = geometry(ctx, cell, iq, &g);
    if (st != RP_OK) return st;
    if (!phi || !centre_frac || !R || !eps_inv) return fail(ctx, RP_E_NULL, "NULL array argument");
    if (!U && !J && !V && !X) return fail(ctx, RP_E_NULL, "no output requested");
    if (nwan < 1 || nwan > 32) return fail(ctx, RP_E_UNSUPPORTED, "nwan = %d outside [1, 32]", nwan);
    if (nR < 1 || nR > 4096) return fail(ctx, RP_E_UNSUPPORTED, "nR = %d outside [1, 4096]", nR);
    if (ng < 1 || nfreq < 1 || ntail < 0) return fail(ctx, RP_E_SHAPE, "bad ng, ntail or nfreq");
    if (accumulate != 0 && accumulate != 1) return fail(ctx, RP_E_RANGE, "accumulate must be 0 or 1");
    const bool head = iq[0] == 0 && iq[1] == 0 && iq[2] == 0;
    if (!gsph) return fail(ctx, RP_E_NULL, "gsph is NULL");
    if (head) {
        if (gsph[0] != 0 || gsph[1] != 0 || gsph[2] != 0)
            return fail(ctx, RP_E_RANGE, "at q = 0 gsph[0] must be G = 0");
        if ((st = check_gsph(ctx, g, ng - 1, gsph + 3, "gsph")) != RP_OK) return st;
    } else if ((st = check_gsph(ctx, g, ng, gsph, "gsph")) != RP_OK) {
        return st;
    }
    if ((st = check_gsph(ctx, g, ntail, gtail, "gtail")) != RP_OK) return st;
    for (int i = 0; i < 3 * nwan; i++)
        if (!std::isfinite(centre_frac[i])) return fail(ctx, RP_E_RANGE, "non-finite centre");
    FftPlan plans[3];
    if ((st = plans3(ctx, g, plans)) != RP_OK) return st;
    const long nr = (long)g.fft[0] * g.fft[1] * g.fft[2];
    const long ldp = (long)ng + ntail;
    const long nvt = (long)nR * nwan * nwan;
    // exchange densities per pass: grids of about 512 MB at most
    const long nvc = std::max(1L, std::min({512L, nvt, (512L << 20) / (nr * (long)sizeof(double2))}));
    const long nrt = wgemm_row_tiles(ng);
    // workspace (double2 units):
    //   grids [max(nvc, nwan)][nr] | PU [nwan][ldp] | PJ [nvc][ldp] | TU [nfreq][ng][nwan]
    //   | part [nrt][nfreq][nvc] | bodyU [nfreq][nwan^2] | bareU, tailU [nwan^2] | bareJ, tailJ [nvc]
    const size_t n2 = (size_t)nwan * nwan;
    const size_t sz[] = {(size_t)std::max<long>(nvc, nwan) * nr, (size_t)nwan * ldp, (size_t)nvc * ldp,
                         (size_t)nfreq * ng * nwan, (size_t)nrt * nfreq * nvc, (size_t)nfreq * n2, n2, n2,
                         (size_t)nvc, (size_t)nvc};
    size_t tot = 0;
    for (size_t x : sz) tot += x;
    if ((st = ensure(ctx, ctx->work, sizeof(double2) * tot)) != RP_OK) return st;
    double2 *bufs[10];
    bufs[0] = (double2 *)ctx->work.p;
    for (int b = 1; b < 10; b++) bufs[b] = bufs[b - 1] + sz[b - 1];
    double2 *grids = bufs[0], *PU = bufs[1], *PJ = bufs[2], *TU = bufs[3], *part = bufs[4], *bodyU = bufs[5];
    double2 *bareU = bufs[6], *tailU = bufs[7], *bareJ = bufs[8], *tailJ = bufs[9];
    // host lists: centres | gsph + gtail | R, packed into one upload
    const size_t hc = sizeof(double) * 3 * nwan, hg = sizeof(int) * 3 * ldp, hr = sizeof(int) * 3 * nR;
    std::vector<char> host(hc + hg + hr);
    std::memcpy(host.data(), centre_frac, hc);
    std::memcpy(host.data() + hc, gsph, sizeof(int) * 3 * ng);
    if (ntail) std::memcpy(host.data() + hc + sizeof(int) * 3 * ng, gtail, sizeof(int) * 3 * ntail);
    std::memcpy(host.data() + hc + hg, R, hr);
    if ((st = upload(ctx, ctx->kinfo, host.data(), host.size())) != RP_OK) return st;
    const double *dcen = (const double *)ctx->kinfo.p;
    const int *dgl = (const int *)((const char *)ctx->kinfo.p + hc);
    const int *dR = (const int *)((const char *)ctx->kinfo.p + hc + hg);
    const double pre = kHartreeEv * 4.0 * kPi / (g.volume * g.nk);
    const double avg = head ? cell_average(g) : 0.0;
    const int klo = head ? 1 : 0;
    const double2 *E = (const double2 *)eps_inv;
    hipStream_t s = ctx->stream;
    StageTimer t(ctx, RP_STAGE_WANNIER);
    if (U || V) {
        launch_wannier_density(s, g, plans, nwan, phi, dcen, grids);
        launch_wannier_gather(s, g, nwan, (int)ldp, dgl, grids, PU, ctx->flag, head);
        if (U) {
            launch_wgemm(s, false, nfreq, ng, klo, nwan, PU, ldp, E, TU);
            launch_wcross(s, nfreq, nwan, ng, klo, PU, ldp, TU, bodyU);
        }
        launch_wgram(s, (int)n2, nwan, false, ng, klo, ntail, PU, ldp, bareU, tailU);
        launch_wsum_u(s, g, nfreq, nR, nwan, ng, dR, pre, head, avg, E, PU, ldp, bodyU, bareU, tailU, accumulate,
                      (double2 *)U, (double2 *)V);
    }
    if (J || X) {
        for (long v0 = 0; v0 < nvt; v0 += nvc) {
            const int n = (int)std::min(nvc, nvt - v0);
            launch_xdens(s, g, plans, nwan, phi, dcen, dR, v0, n, grids);
            launch_wannier_gather(s, g, n, (int)ldp, dgl, grids, PJ, ctx->flag, head);
            if (J) launch_wgemm(s, true, nfreq, ng, klo, n, PJ, ldp, E, part);
            launch_wgram(s, n, 0, true, ng, klo, ntail, PJ, ldp, bareJ, tailJ);
            launch_wsum_x(s, nfreq, nvt, v0, n, ng, pre, head, avg, E, PJ, ldp, part, bareJ, tailJ, accumulate,
                          (double2 *)J, (double2 *)X);
        }
    }
    return check_launch(ctx, "wannier q-term");
}

}  // extern "C"
