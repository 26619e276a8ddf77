/*
 * rp.h - C ABI of the MI355X polarization / screened-interaction library.
 *
 * The library computes, for one q-point, the constrained-RPA chain of the
 * RESPACK paper (Nakamura et al., section "Response function with random
 * phase approximation" and section "Direct-Coulomb and exchange integrals"):
 *
 *   pair densities  M^G_{ab}(k+q,k) = <psi_{a,k+q}| e^{i(q+G).r} |psi_{b,k}>   Eq. ism
 *   polarization    chi_GG'(q,w) = (2/Nk) sum_k sum_a sum_b (1 - T T)
 *                                  M^G M^G'* X_{a k+q, b k}(w)                  Eq. chi
 *                   with X integrated by the generalized tetrahedron method    Eqs. Xakqbk, tetrahedron, tak
 *   dielectric      eps_GG' = delta_GG' - (4 pi/Omega) chi_GG'/(|q+G||q+G'|)   Eq. epsGG
 *   screened        W_GG' = (4 pi/Omega) eps^-1_GG' / (|q+G||q+G'|)             Eq. Wq
 *   projection      W_ij(q,w) = (4 pi/(Omega Nq)) [ sum_GG' rho_i(G) eps^-1 rho_j(G')*
 *                                 + sum_{G in tail} rho_i(G) rho_j(G)* ]       Eqs. matrix_U, rhoiqG
 *
 * and around it: the q -> 0 head, wings, intraband (Drude) term and optical
 * quantities (Eqs. eps00, eps00-cRPA, plasma, momentum, epsilonM, eels,
 * optical-conductivity, reflectance),
 * one q-point's term of the q-mesh sums of the screened and bare direct and
 * exchange integrals U, V, J, X (Eqs. matrix_U, matrix_V, matrix_J,
 * matrix_X), metallic tetrahedron weights (the Fermi level cutting the
 * tetrahedra), the symmetry unfolding of coefficients and eps^-1 (Eqs.
 * coef-G, symeps) and the logarithmic frequency grid (Eq. grid).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Units: lattice in bohr; energies, frequencies and the broadening in eV;
 *   chi in hartree^-1 (atomic units); W and W_ij in eV.  1 Ha = 27.211386245988 eV.
 * - k mesh: Gamma-centred, k = n/K (fractional), mesh index (n1*K2 + n2)*K3 + n3.
 *   q = iq/K with iq a mesh index; the q grid is the k grid (Eq. W).
 * - Real-space grid r_j = (j1/N1, j2/N2, j3/N3) fractional, stored [j1][j2][j3].
 * - Reciprocal vectors G = m1 b1 + m2 b2 + m3 b3 with integer Miller indices.
 * - Complex arrays ("c128") are interleaved (re, im) doubles, C-contiguous.
 * - Pair order: p = ((k-k0)*(e1-e0) + (a-e0))*(o1-o0) + (b-o0): occupied
 *   band b fastest, then empty band a, then k.
 * - Memory: the caller owns every array it passes.  "dev" pointers are device
 *   memory on the context's GPU, "host" pointers are ordinary host memory read
 *   during the call only.  The context owns its device workspace, which grows
 *   on demand and is released by rp_destroy.
 * - Execution: device work is enqueued on the context's stream and is
 *   asynchronous with respect to the host; host arrays may be reused as soon
 *   as the call returns.
 * - Errors: arguments are validated before anything is enqueued; a non-OK
 *   status means nothing was enqueued (or, for RP_E_DEVICE, that a launch
 *   failed) and the outputs are undefined.  Faults detected inside kernels
 *   (a zero pivot, a non-finite value) are reported by rp_synchronize.
 *   rp_last_error gives a message for the most recent failure.
 * - One context per host thread.
 */
#ifndef RP_H
#define RP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RP_OK = 0,
    RP_E_NULL = 1,        /* a required pointer is NULL */
    RP_E_SHAPE = 2,       /* inconsistent sizes, ranges or counts */
    RP_E_RANGE = 3,       /* a value outside its domain (e.g. |q+G| = 0, delta < 0) */
    RP_E_ALIAS = 4,       /* FFT grid too small for alias-free pair products */
    RP_E_NOMEM = 5,       /* device workspace could not be allocated */
    RP_E_DEVICE = 6,      /* HIP runtime error */
    RP_E_SINGULAR = 7,    /* the dielectric matrix had a zero pivot */
    RP_E_UNSUPPORTED = 8  /* e.g. an FFT length with a prime factor above 5 */
} rp_status;

typedef enum {
    RP_FP64 = 0,          /* FP64 everywhere (FP64 matrix cores for chi) */
    RP_SPLIT_BF16 = 1,    /* chi contraction on BF16 matrix cores: each operand
                             x = x_hi + x_mid (BF16 terms of its FP32 value),
                             products by the three-term compensated form
                             x_hi y_hi + x_hi y_mid + x_mid y_hi, FP32
                             accumulation, FP64 reduction into chi; pair
                             densities computed on FP32 grids; weights,
                             eps^-1 and W_ij in FP64 */
    RP_SPLIT_BF16_X6 = 2  /* as RP_SPLIT_BF16 with x = x_hi + x_mid + x_lo and
                             the six products of order <= 2 (each product to
                             about FP32 accuracy, twice the matrix-core work);
                             chi's error is then set by the FP32 pair
                             densities and the FP32 accumulation within a
                             slice of pair steps, about 1e-6 relative */
} rp_precision;

typedef enum {
    RP_W_TETRA = 0,     /* generalized tetrahedron integration of X (Eq. tetrahedron) */
    RP_W_SAMPLING = 1,  /* X evaluated at the mesh point (Eq. Xakqbk as written) */
    RP_W_TETRA_METAL = 2 /* generalized tetrahedron restricted, within every
                            tetrahedron, to the part where the linear
                            interpolants satisfy E_b(k) < E_F < E_a(k+q)
                            (E_F from rp_set_fermi_level); the occupied and
                            empty band ranges may then overlap */
} rp_weight_mode;

typedef struct rp_ctx rp_ctx;

typedef struct {
    double lat[3][3]; /* rows a1, a2, a3 (bohr) */
    int fft[3];       /* real-space grid N1, N2, N3 (factors 2,3,5 only, each <= 256) */
    int kmesh[3];     /* k mesh K1, K2, K3 */
} rp_cell;

/* Create a context on GPU `device`.  hip_stream is a hipStream_t to enqueue
 * on, or NULL for a stream the context creates (default priority) and owns. */
rp_status rp_create(rp_ctx **ctx, int device, void *hip_stream);

/* Release the workspace and the owned stream.  NULL is accepted. */
rp_status rp_destroy(rp_ctx *ctx);

/* Wait for the context's stream; report device-side faults (RP_E_SINGULAR for
 * a zero pivot, RP_E_RANGE for a non-finite value) raised since the last call. */
rp_status rp_synchronize(rp_ctx *ctx);

/* Message of the most recent failure on ctx ("" if none).  Owned by ctx and
 * valid until the next call on it. */
const char *rp_last_error(const rp_ctx *ctx);

/*
 * Steps a2-a4: pair densities (Eq. ism), evaluated by the FFT route:
 *   u_{nk}(r_j) = sum_{G in S_psi(k)} C_{Gn}(k) e^{iG.r_j}                       (Eq. pak)
 *   M_p(G) = (1/N_r) sum_j conj(u_{a,k'}(r_j)) u_{b,k}(r_j) e^{i(G+G0).r_j}
 * where k+q = k' + G0 with k' on the mesh.  This equals the plane-wave
 * definition exactly when N_a > 2 mmax_a + max|m_a + G0_a| on each axis, on
 * cell->fft or on any smaller grid that satisfies it: the steps run on the
 * grid rp_pair_grid reports.
 *
 * nband, npw_max     : bands and padded plane-wave count of coef/miller
 * npw      (host)    : int[Nk] plane waves per k
 * mmax     (host)    : int[3] bound on |m_a| over all wavefunction Miller
 *                      indices (used for the aliasing check and to prune the
 *                      transforms; a wrong bound gives wrong results)
 * miller   (dev)     : int[Nk][npw_max][3]
 * coef     (dev)     : c128[Nk][nband][npw_max], sum_G |C_Gn|^2 = 1
 * o0..o1 / e0..e1    : occupied bands b at k / empty bands a at k+q
 * k0..k1             : k range of this call
 * gsph     (host)    : int[ng][3] Miller indices of the polarization sphere
 * prec               : RP_FP64 computes the grids and transforms in FP64; the
 *                      split modes in FP32 (M then carries ~1e-7 relative
 *                      error, far below what the split contraction keeps)
 * M        (dev)     : c128[k1-k0][e1-e0][o1-o0][ng] output
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_ALIAS, RP_E_UNSUPPORTED,
 * RP_E_NOMEM, RP_E_DEVICE.
 */
rp_status rp_pair_density(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband,
                          int npw_max, const int *npw, const int mmax[3], const int *miller,
                          const double *coef, int o0, int o1, int e0, int e1, int k0, int k1,
                          int ng, const int *gsph, rp_precision prec, double *M);

/*
 * The grid that rp_pair_density and the chi0 entry points that build pair
 * densities run steps a2-a4 on, for these arguments; host computation only
 * (no context).  Once N_a > 2 mmax_a + max|m_a + G0_a| on every axis, the
 * FFT route gives the plane-wave definition of Eq. ism exactly, whatever the
 * grid; the library then takes the smallest such grid that its lane kernels
 * take (N2 = N3 from their line lengths, N1 any 2^a 3^b 5^c), never larger
 * than cell->fft, and keeps cell->fft where none fits.  cell->fft itself
 * must satisfy the condition (else RP_E_ALIAS, as in rp_pair_density).
 * mmax (host) int[3], gsph (host) int[ng][3], prec: as rp_pair_density.
 * grid (host) int[3] output.
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_ALIAS, RP_E_UNSUPPORTED.
 */
rp_status rp_pair_grid(const rp_cell *cell, const int iq[3], const int mmax[3], int ng,
                       const int *gsph, rp_precision prec, int grid[3]);

/*
 * Step a5: weights w_p(omega_f) = (2/Nk)(1 - T_{a,k+q} T_{b,k}) x_p(omega_f)
 * (Eqs. chi, tak), x from the generalized tetrahedron method on the linear
 * interpolant of E_a(k+q) - E_b(k) over the 6 tetrahedra per mesh cell that
 * share the cell's (0,0,0)-(1,1,1) diagonal (Eq. tetrahedron), with
 * z = w + i delta and z' = -w + i delta (Eq. Xakqbk), or x = X at the mesh
 * point for RP_W_SAMPLING.
 *
 * energy_eV (dev)    : double[Nk][nband]
 * T         (dev)    : double[Nk][nband] transition probabilities (Eq. tak),
 *                      or NULL for the usual RPA (T = 0)
 * freq_eV   (host)   : c128[nfreq] (real w, or i*nu on the imaginary axis)
 * delta_eV           : broadening >= 0
 * w         (dev)    : c128[nfreq][npair] output, hartree^-1
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_NOMEM, RP_E_DEVICE.
 */
rp_status rp_weights(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband,
                     const double *energy_eV, const double *T, int o0, int o1, int e0, int e1,
                     int k0, int k1, int nfreq, const double *freq_eV, double delta_eV,
                     rp_weight_mode wm, double *w);

/*
 * Steps a5-a6: chi_GG'(w) (+)= sum_p w_p(w) M_p(G) conj(M_p(G'))   (Eq. chi)
 * for the pairs of one rp_pair_density call (same ranges, same M layout).
 * prec selects the contraction: RP_FP64 (FP64 matrix cores), RP_SPLIT_BF16
 * or RP_SPLIT_BF16_X6 (BF16 split products with FP32 accumulation, added into
 * chi in FP64).  Weights are always FP64.
 *
 * M          (dev)   : c128[npair][ng] from rp_pair_density
 * accumulate         : 0 overwrite chi, 1 add into chi
 * chi        (dev)   : c128[nfreq][ng][ng], hartree^-1
 * Errors: as rp_weights.
 */
rp_status rp_chi0_accumulate(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband,
                             const double *energy_eV, const double *T, int o0, int o1, int e0,
                             int e1, int k0, int k1, int ng, const double *M, int nfreq,
                             const double *freq_eV, double delta_eV, rp_weight_mode wm,
                             rp_precision prec, int accumulate, double *chi);

/*
 * rp_chi0_accumulate without allocating, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * rp_chi0_accumulate; its workspace (frequencies, weights, split operands,
 * partial tiles) is carved from a fixed device array of 128 MiB that the
 * library holds on each GPU it runs on until the process ends, instead of
 * the context's growable buffers, and nothing is allocated or freed.  A call
 * whose workspace would exceed 128 MiB fails with RP_E_SHAPE before anything
 * is enqueued (fewer pairs per call fit: e.g. 12 288 pairs at N_G = 89 and
 * 10 frequencies take about 98 MiB in the split form).  Every call on one GPU
 * shares that array: calls that overlap on one GPU (contexts on different
 * streams) race and must be ordered by the caller; each call writes every
 * workspace byte it reads.
 * Errors: as rp_chi0_accumulate; RP_E_SHAPE beyond the fixed workspace;
 * RP_E_DEVICE when the array has no device address on this GPU.
 */
rp_status rp_chi0_accumulate_noalloc(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nband,
                                     const double *energy_eV, const double *T, int o0, int o1, int e0,
                                     int e1, int k0, int k1, int ng, const double *M, int nfreq,
                                     const double *freq_eV, double delta_eV, rp_weight_mode wm,
                                     rp_precision prec, int accumulate, double *chi);

/*
 * Steps a2-a6 for a batch of independent chi0 problems (section "Parallel
 * calculation": q-points are independent, and chi of one q is a sum of
 * band-pair blocks), enqueued as one HIP graph launch.  Each problem carries
 * the arguments of rp_pair_density and rp_chi0_accumulate; its k range
 * [k0, k1) is processed kbatch k-points at a time: the pair densities of a
 * batch go to context-owned buffers, then their weights and contraction are
 * added into the problem's chi (the first batch overwrites chi when
 * accumulate = 0).  In FP64 the buffer holds M as rp_pair_density writes it;
 * in the split forms the pair kernels write the contraction's operands
 * directly (each M value rounded to FP32, and its BF16 terms), the same
 * operands rp_chi0_accumulate prepares from M, so chi is the same as from
 * rp_pair_density and rp_chi0_accumulate per batch, bit for bit.  A problem
 * with no pairs only clears chi (accumulate = 0).
 * Problems may differ in cell, grid, k mesh, bands, N_G and frequencies;
 * they run one after the other on the context's stream, sharing workspace.
 *
 * The first call captures every launch of the batch into a sequence of
 * graphs (rp_chi0_batch_graphs) and launches them.  A later call with the
 * same problems (the same scalars and pointers, and the same contents of the
 * host arrays npw, gsph and freq_eV) relaunches those graphs without
 * capturing again; any difference captures anew.  The device arrays are read
 * when the graphs run.
 *
 * Fields of rp_problem, as in rp_pair_density and rp_chi0_accumulate:
 *   npw (host int[Nk]), mmax, miller (dev), coef (dev), energy_eV (dev),
 *   T (dev or NULL), gsph (host int[ng][3]), freq_eV (host c128[nfreq]),
 *   chi (dev c128[nfreq][ng][ng] output, hartree^-1).
 * kbatch >= 1 sets the pair-density buffers for the largest problem, with
 * P = kbatch*(o1-o0)*(e1-e0): FP64 16*P*ng bytes; split forms 20*KP*NGP bytes
 * (KP = P rounded up to 32, NGP = ng rounded up to 128).
 * prec applies to every problem.
 * Errors: those of rp_pair_density and rp_chi0_accumulate, with "problem i:"
 * in the message; RP_E_SHAPE for kbatch < 1 or nprob < 0.  On a non-OK
 * status nothing has been launched.
 */
typedef struct rp_problem {
    rp_cell cell;
    int iq[3];
    int nband, npw_max;
    const int *npw;
    int mmax[3];
    const int *miller;
    const double *coef;
    const double *energy_eV;
    const double *T;
    int o0, o1, e0, e1, k0, k1;
    int ng;
    const int *gsph;
    int nfreq;
    const double *freq_eV;
    double delta_eV;
    rp_weight_mode wm;
    int kbatch;
    int accumulate;
    double *chi;
} rp_problem;

rp_status rp_chi0_batch(rp_ctx *ctx, int nprob, const rp_problem *probs, rp_precision prec);

/*
 * The graphs of the most recent rp_chi0_batch capture: a batch is captured
 * as a sequence of graphs of at most about 2048 kernel nodes each (a graph
 * closes after the k batch that reaches the bound), launched in order on the
 * context's stream; graphs (host) gets their number and nodes (host) their
 * kernel nodes in total (0 and 0 before the first batch).
 * Errors: RP_E_NULL.
 */
rp_status rp_chi0_batch_graphs(rp_ctx *ctx, int *graphs, long *nodes);

/*
 * Steps a2-a6 of one chi0 problem (Eqs. ism and chi), enqueued directly on
 * the context's stream (no graph): the k range [k0, k1) of *p is processed
 * kbatch k-points at a time exactly as one problem of rp_chi0_batch, with
 * the same buffers (in the split forms the pair kernels write the
 * contraction's operands, and no FP64 M exists), so chi equals that of
 * rp_chi0_batch, and of rp_pair_density and rp_chi0_accumulate per k batch,
 * bit for bit.  Fields of *p as in rp_chi0_batch; p is read during the call
 * only.
 * Errors: those of rp_pair_density and rp_chi0_accumulate; RP_E_NULL for a
 * NULL p or chi; RP_E_SHAPE for kbatch < 1.  Argument errors are found before
 * anything is enqueued; a failed launch (RP_E_DEVICE) can leave chi holding
 * the k batches enqueued before it.
 */
rp_status rp_chi0_run(rp_ctx *ctx, const rp_problem *p, rp_precision prec);

/*
 * Steps a7-a9: eps = I - v^1/2 chi v^1/2 with v^1/2_G = sqrt(4 pi/Omega)/|q+G|
 * (Eq. epsGG), eps^-1 per frequency by FP64 Gauss-Jordan elimination with
 * partial pivoting (blocked in panels of 64 columns), and W = v^1/2 eps^-1
 * v^1/2 in eV (Eq. Wq, inside S_eps).
 *
 * ng              : 1 .. 6144 (RP_E_UNSUPPORTED above)
 * gsph    (host)  : int[ng][3], |q+G| > 0 for every entry
 * chi     (dev)   : c128[nfreq][ng][ng]
 * eps_inv (dev)   : c128[nfreq][ng][ng] output, or NULL
 * W       (dev)   : c128[nfreq][ng][ng] output in eV, or NULL
 * A pivot of magnitude below 1e-13 (eps is dimensionless with a unit-scale
 * diagonal, so this means a condition number beyond ~1e13) is reported by
 * rp_synchronize as RP_E_SINGULAR; a non-finite value as RP_E_RANGE.
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_UNSUPPORTED, RP_E_NOMEM,
 * RP_E_DEVICE.
 */
rp_status rp_screen_W(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int ng,
                      const int *gsph, int nfreq, const double *chi, double *eps_inv,
                      double *W);

/*
 * Step a10: W_ij(q,w) = HA * (4 pi/(Omega Nq)) [ sum_{G,G' in S_eps}
 *     rho_i(G) eps^-1_GG'(w) conj(rho_j(G')) + sum_{G in tail} rho_i(G) conj(rho_j(G)) ]
 * (the q-term of Eq. matrix_U at R = 0), with rho_i(G) = ntilde_i(q+G)/|q+G|,
 * ntilde_i(Q) = (Omega/N_r) sum_j phi_i(r_j)^2 e^{iQ.rt_ij}, rt_ij the image
 * of r_j nearest to the orbital centre (Eq. rhoiqG for the density of orbital i).
 *
 * phi         (dev)  : double[nwan][N1][N2][N3], (Omega/N_r) sum_j phi^2 = 1
 * centre_frac (host) : double[nwan][3] orbital centres, fractional
 * gsph        (host) : int[ng][3], the rows/columns of eps_inv
 * gtail       (host) : int[ntail][3], vectors of the bare tail (may be 0)
 * eps_inv     (dev)  : c128[nfreq][ng][ng]
 * Wij         (dev)  : c128[nfreq][nwan][nwan] output, eV
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_UNSUPPORTED, RP_E_NOMEM,
 * RP_E_DEVICE.
 */
rp_status rp_wannier_W(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nwan,
                       const double *phi, const double *centre_frac, int ng, const int *gsph,
                       int ntail, const int *gtail, int nfreq, const double *eps_inv,
                       double *Wij);

/*
 * One q-point's term of the q-mesh sums of the interaction parameters
 * between orbital i in the home cell and orbital j in cell R (section
 * "Interaction parameters", Eqs. W, Wq, matrix_U, rhoiqG, matrix_V, matrix_J,
 * matrix_X).  Summed over every q of the mesh (accumulate = 0 for the first,
 * 1 for the rest) it gives, in eV, with pre = HA 4 pi/(Omega N_q):
 *   U_i0jR(w) = sum_q e^{-iq.R} pre [ sum_{G,G' in S_eps} rho_iq(G) eps^-1_GG'(q,w) conj(rho_jq(G'))
 *                                     + sum_{G in tail} rho_iq(G) conj(rho_jq(G)) ]   screened direct
 *   V_i0jR    = the same with eps^-1 = delta                                           bare direct
 *   J_i0jR(w) = sum_q pre [ sum_{G,G'} rho_v(G) eps^-1_GG' conj(rho_v(G')) + tail ]      screened exchange
 *   X_i0jR    = the same with eps^-1 = delta                                           bare exchange
 * Direct densities rho_iq(G) = ntilde_i(q+G)/|q+G| as in rp_wannier_W.
 * Exchange densities rho_v(G) = ntilde_v(q+G)/|q+G|, v = (R, i, j), with
 * ntilde_v(Q) = (Omega/N_r) sum_p phi_i0(rt_p) phi_jR(rt_p) e^{iQ.rt_p}: rt_p
 * the image of grid point p nearest the midpoint (c_i + c_j + R)/2,
 * phi_i0(rt) = phi_i(p) where rt lies within half a cell of c_i (each
 * fractional component of rt - c_i in [-1/2, 1/2)), else 0, and phi_jR(rt)
 * = phi_j(p) where rt - R lies within half a cell of c_j, else 0.  X sums
 * over S_eps and the tail like V.
 * q = 0 (iq = 0): gsph[0] must be G = 0 (no other G = 0 in gsph or gtail)
 * and eps_inv the inverse with head and wings (rp_screen_head).  The G = 0
 * row and column then enter only through the head term
 * A eps^-1_00 ntilde_a(0) conj(ntilde_b(0)) (eps^-1_00 -> 1 for V and X),
 * A = rp_coulomb_cell_average(cell); the wings are dropped.  Elsewhere
 * |q + G| = 0 is an error (RP_E_RANGE).
 *
 * phi (dev) double[nwan][N1][N2][N3], centre_frac (host) double[nwan][3]:
 *   as rp_wannier_W.
 * R (host) int[nR][3]: lattice vectors in units of a1, a2, a3.
 * gsph (host) int[ng][3], gtail (host) int[ntail][3]: as rp_wannier_W.
 * eps_inv (dev) c128[nfreq][ng][ng].
 * U, J (dev) c128[nfreq][nR][nwan][nwan]; V, X (dev) c128[nR][nwan][nwan];
 *   each may be NULL (not computed), not all four.  accumulate = 1 adds the
 *   term to what they hold.
 * Device workspace: about (nwan + C)(N_r + ng + ntail) + nfreq ng nwan complex
 * values, C <= 512 exchange densities at a time (fewer on large grids).
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_UNSUPPORTED (nwan > 32,
 * nR > 4096, an FFT length), RP_E_NOMEM, RP_E_DEVICE.
 */
rp_status rp_wannier_qterm(rp_ctx *ctx, const rp_cell *cell, const int iq[3], int nwan,
                           const double *phi, const double *centre_frac, int nR, const int *R,
                           int ng, const int *gsph, int ntail, const int *gtail, int nfreq,
                           const double *eps_inv, int accumulate, double *U, double *J,
                           double *V, double *X);

/*
 * A = (N_q Omega/(2 pi)^3) int_cell d^3q/|q|^2, the mean of 1/|q|^2 over the
 * q-cell {sum_a x_a b_a/K_a : x in [-1/2, 1/2)^3} around Gamma, which replaces
 * 1/|q|^2 in the q = 0 term of the mesh sums (the treatment of the Coulomb
 * singularity the paper cites for Eq. rhoiqG).  Host computation only (no
 * context, no device): six face pyramids, each h int_face dA/|p|^2 by
 * composite Gauss-Legendre quadrature.
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE (degenerate lattice).
 */
rp_status rp_coulomb_cell_average(const rp_cell *cell, double *avg);

/*
 * The logarithmic frequency grid of the polarization function (section
 * "Frequency grid", Eq. grid), host computation only (no context):
 *   omega_i = (dw/(s-1)) (s^(i-1) - 1)                       i = 1 .. nmax
 *   omega_i = emax 3^((i - nmax)/(nomega - nmax))             i = nmax+1 .. nomega
 * with s fixed by omega_nmax = emax, i.e. s^(nmax-1) - (emax/dw)(s - 1) = 1
 * (the sign the boundary condition requires), s != 1; so omega_1 = 0,
 * omega_2 = dw, omega_nmax = emax and omega_nomega = 3 emax.  The paper's
 * defaults: nomega = 70, nmax = 9 nomega/10 (pass nmax = 0), dw = 0.05 eV,
 * emax = max E - min E over the bands.
 * omega_eV (host) double[nomega] output.
 * Errors: RP_E_NULL; RP_E_SHAPE (nomega < 3, nmax outside [2, nomega));
 * RP_E_RANGE (dw <= 0, emax <= dw, non-finite).
 */
rp_status rp_frequency_grid(double emax_eV, double dw_eV, int nomega, int nmax, double *omega_eV);

/*
 * The Fermi level E_F (eV, on the scale of energy_eV) that RP_W_TETRA_METAL
 * weights cut the tetrahedra with; NaN clears it.  A call with
 * RP_W_TETRA_METAL while none is set fails with RP_E_RANGE.  For a pair of a
 * band a at k+q and a band b at k the tetrahedron integral of Eq.
 * tetrahedron then runs over the part of each tetrahedron where
 * E_b < E_F < E_a (b occupied, a empty); a tetrahedron where that holds at
 * all four corners gives the insulating integral, one where E_b >= E_F or
 * E_a <= E_F at all four gives nothing.
 * Errors: RP_E_NULL.
 */
rp_status rp_set_fermi_level(rp_ctx *ctx, double ef_eV);

/*
 * Symmetry unfolding of plane-wave coefficients (section "Symmetry", Eqs.
 * red-wavefunction, k-and-kirr, G-and-Girr, coef-G).  The operation maps
 * fractional real-space coordinates x -> W x + t (W: integer, row-major,
 * det +-1; t: fractional translation); on fractional reciprocal coordinates
 * it acts as S = W^{-T}.  For k = S k* + Delta (k, k* given by mesh indices;
 * Delta, the rewind vector, must come out integral):
 *   C_G(k) = C_{S^{-1}(G + Delta)}(k*) e^{-i (G + Delta).T}
 * i.e. for Miller indices m the source is W^T (m + Delta) and the phase
 * e^{-2 pi i (m + Delta).t} (a global phase of the band is dropped, as in
 * the paper).
 * miller_irr (host) int[npw_irr][3], coef_irr (dev) c128[nband][ld_irr];
 * miller (host) int[npw][3], the target list at k, each of whose source
 * vectors must be in miller_irr; coef (dev) c128[nband][ld] output (columns
 * npw .. ld-1 untouched).
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE (W not unimodular, k not an
 * image of k*, a target without source, a mesh index outside the mesh),
 * RP_E_NOMEM, RP_E_DEVICE.
 */
rp_status rp_unfold_coef(rp_ctx *ctx, const rp_cell *cell, const int W[9], const double t[3],
                         const int ik_irr[3], int nband, int npw_irr, const int *miller_irr,
                         const double *coef_irr, long ld_irr, const int ik[3], int npw,
                         const int *miller, double *coef, long ld);

/*
 * Symmetry unfolding of a G-indexed matrix (Eq. symeps): eps^-1, or chi
 * and W, which transform alike.  For q = S q* + Delta (as above):
 *   X_{G,G'}(q, w) = X_{S^{-1}(G + Delta), S^{-1}(G' + Delta)}(q*, w) e^{+i (G - G').T}
 * The phase sign is the one that Eq. chi's order M(G) conj(M(G')) and
 * Eq. red-wavefunction's operator give (the paper prints e^{-i(G - G').T});
 * it reproduces chi computed directly at q from the symmetric bands.
 * gsph_irr (host) int[ng_irr][3], src (dev) c128[nfreq][ng_irr][ng_irr];
 * gsph (host) int[ng][3], the list at q (usually S G* - Delta over gsph_irr),
 * every source in gsph_irr; dst (dev) c128[nfreq][ng][ng], not src.
 * Errors: RP_E_NULL, RP_E_SHAPE (ng > 6144), RP_E_RANGE, RP_E_ALIAS,
 * RP_E_NOMEM, RP_E_DEVICE.
 */
rp_status rp_unfold_eps_inv(rp_ctx *ctx, const rp_cell *cell, const int W[9], const double t[3],
                            const int iq_irr[3], int ng_irr, const int *gsph_irr, const int iq[3], int ng,
                            const int *gsph, int nfreq, const double *src, double *dst);

/*
 * The q -> 0 head (section "Response function with random phase
 * approximation", Eqs. eps00-cRPA and momentum): for an empty band a and an
 * occupied band b at the same k, the G = 0 pair density tends to
 * q . p_ab(k) / (E_a(k) - E_b(k)) with p_ab = <psi_a| -i grad |psi_b> (the
 * non-local pseudopotential term dropped, as in the paper).  This call writes
 * the head density h_ab = qhat . p_ab / (E_a - E_b) (bohr, hartree) into
 * column col of M (c128 [npair][ng], the layout of rp_pair_density), so that
 * M holds M(q, G) for G != 0 and lim M(q, 0)/|q| in that column; the
 * contraction of such an M gives lim chi_00 / q^2 and lim chi_0G / q.
 * The usual use is rp_pair_density at iq = 0 with G = 0 in gsph at index
 * col, then this call, then rp_chi0_accumulate and rp_screen_head.
 *
 * npw (host int[Nk]), miller (dev), coef (dev): as rp_pair_density;
 * energy_eV (dev double[Nk][nband]).
 * qhat (host double[3]): direction of q, Cartesian, normalized here.
 * Where the band ranges overlap (a metal) the intraband pairs a = b get 0:
 * at q -> 0 they belong to the intraband term (rp_plasma_frequency,
 * rp_set_drude).
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_NOMEM, RP_E_DEVICE; any
 * other pair with E_a = E_b is flagged non-finite (rp_synchronize) and gets 0.
 */
rp_status rp_head_density(rp_ctx *ctx, const rp_cell *cell, int nband, int npw_max, const int *npw,
                          const int *miller, const double *coef, const double *energy_eV, int o0,
                          int o1, int e0, int e1, int k0, int k1, const double qhat[3], int ng,
                          int col, double *M);

/*
 * eps at q -> 0 with head and wings, its inverse, and the optical quantities
 * (Eqs. eps00-cRPA, epsilonM, eels, optical-conductivity, reflectance):
 * eps_GG' = delta_GG' - v^1/2_G chi_GG' v^1/2_G' with v^1/2_0 = sqrt(4 pi/Omega)
 * (the q factors of head and wings are in chi, see rp_head_density) and
 * v^1/2_G = sqrt(4 pi/Omega)/|G| otherwise; then per frequency
 *   optics[f] = {Re eps_M, Im eps_M, L, Re sigma, R}
 * with eps_M = 1/eps^-1_00, L = -Im eps^-1_00, Re sigma = (w/4 pi) Im eps_M
 * (w = Re freq in hartree, sigma in atomic units) and the reflectance
 * R = |(sqrt(eps_M) - 1)/(sqrt(eps_M) + 1)|^2.  The intraband term of Eq.
 * eps00 enters the head when rp_set_drude has set one: eps_00 -= wq /
 * (w (w + i delta)) (w = freq_eV, complex).  Where w (w + i delta) = 0 that
 * term is infinite: eps^-1 gets a zero head row and column and the inverse
 * of eps's body (the limit), and that frequency's optics are
 * {NaN, NaN, 0, NaN, 1} (L = 0 and R = 1 in the limit, eps_M and sigma
 * undefined).
 *
 * gsph     (host) : int[ng][3], G = 0 first, no other zero vector
 * freq_eV  (host) : c128[nfreq]
 * chi      (dev)  : c128[nfreq][ng][ng] with the head row and column
 * eps_inv  (dev)  : c128[nfreq][ng][ng] output, or NULL
 * optics   (dev)  : double[nfreq][5] output, or NULL
 * Errors: as rp_screen_W; a zero pivot surfaces in rp_synchronize.
 */
rp_status rp_screen_head(rp_ctx *ctx, const rp_cell *cell, int ng, const int *gsph, int nfreq,
                         const double *freq_eV, const double *chi, double *eps_inv,
                         double *optics);

/*
 * The plasma tensor of the intraband term (Eqs. eps00, plasma, momentum), in
 * eV^2:
 *   Omega^{mu nu} = (4 pi / Omega) (2 / N_k) sum_k sum_{a in [b0, b1)}
 *                   (1 - T_ak^2) p^mu_a(k) p^nu_a(k) delta(E_ak - E_F)
 * with the diagonal moments p_a(k) = <psi_a| -i grad |psi_a> = sum_G
 * |C_Ga(k)|^2 (k + G) (Cartesian, the non-local term dropped as in the
 * paper) and the Fermi-surface delta integrated on the linear tetrahedra of
 * the weights (6 per mesh cell around its (0,0,0)-(1,1,1) diagonal).  The
 * paper prints the Fermi-surface sum without the factor 4 pi / Omega and the
 * spin sum 2; with them a free-electron gas gives 4 pi n.  The head term
 * along qhat is wq = qhat . Omega . qhat (rp_set_drude).
 *
 * npw (host int[Nk]), miller (dev), coef (dev): as rp_pair_density;
 * energy_eV (dev double[Nk][nband]); T (dev double[Nk][nband]) or NULL (no
 * cRPA factor); bands [b0, b1) enter the sum (those that cross E_F matter).
 * omega2_eV2 (host double[3][3]) output.  The call waits for the device.
 * Errors: RP_E_NULL, RP_E_SHAPE, RP_E_RANGE, RP_E_NOMEM, RP_E_DEVICE.
 */
rp_status rp_plasma_frequency(rp_ctx *ctx, const rp_cell *cell, int nband, int npw_max,
                              const int *npw, const int *miller, const double *coef,
                              const double *energy_eV, const double *T, int b0, int b1,
                              double ef_eV, double *omega2_eV2);

/*
 * The intraband term that rp_screen_head subtracts from eps_00 (Eq. eps00):
 * wq = qhat . Omega . qhat (eV^2) and the broadening delta (eV) of
 * -wq / (w (w + i delta)); wq = 0 removes it (the default, and Eq.
 * eps00-cRPA).
 * Errors: RP_E_NULL, RP_E_RANGE (non-finite, delta < 0).
 */
rp_status rp_set_drude(rp_ctx *ctx, double wq_eV2, double delta_eV);

/*
 * Launch-shape tuning per size class (the autotuner in the Python package
 * measures the candidates and installs its table with this call).  A call
 * with N_G sphere vectors and largest FFT edge E uses the first entry with
 * ng_max >= N_G and grid_max >= E; with no match, or no table, the defaults
 * apply.  The table is copied; n = 0 clears it.
 *   chi_nw     frequencies per workgroup of the split-BF16 contraction, 1 or
 *              2 (0: the default, 2); with 2 and a multiple of four
 *              frequencies, form 0 runs as 64-row strips x 128 columns for
 *              four frequencies (a Hermitian chi with a multiple of eight:
 *              32-row strips for eight, each strip's tiles starting at its
 *              diagonal), except unsliced complex-weight launches whose last
 *              wave of 128 x 128 tiles is split over the chip
 *   chi_fill   workgroups the slicing of the pair steps aims for when the
 *              tiles alone give fewer than half of it (0: never slice, -1:
 *              the default, 1024)
 *   fft_lines  lines per workgroup of the u-grid transforms, 1..64 (0: 32,
 *              16 or 8 by length)
 *   chi_kernel split-BF16 contraction form: 0 = 128 x 128 tiles on four
 *              waves, 1 = 256 x 64 tiles on eight waves (two per SIMD, 32x32
 *              matrix-core ops), 2 = 256 x 128 tiles on eight waves, one
 *              frequency per workgroup (RP_SPLIT_BF16 only, else form 1).
 *              Forms 1 and 2 run where N_G pads to a multiple of 256 and the
 *              weights are complex; elsewhere form 0 runs.
 * Only launch shapes change: every choice computes the same sums (the
 * contraction's FP32 partial sums are grouped differently when sliced).
 * Errors: RP_E_NULL, RP_E_RANGE.
 */
typedef struct {
    int ng_max;
    int grid_max;
    int chi_nw;
    int chi_fill;
    int fft_lines;
    int chi_kernel;
} rp_tune_entry;

rp_status rp_set_tuning(rp_ctx *ctx, int n, const rp_tune_entry *table);

/*
 * Stage timers.  While enabled, the context records a pair of HIP events on
 * its stream around every kernel launch of a stage and accumulates the
 * elapsed device time per stage.  Stages:
 *   RP_STAGE_UGRID    u-grids (coefficient scatter and 3-D transform), a2
 *   RP_STAGE_PAIR     pair-density kernel, a3-a4
 *   RP_STAGE_WEIGHTS  tetrahedron weights, a5
 *   RP_STAGE_PREP     split-BF16 operand preparation, a6
 *   RP_STAGE_CHI      chi contraction kernel (FP64 or split-BF16), a6
 *   RP_STAGE_SCREEN   eps, inversion and W, a7-a9
 *   RP_STAGE_WANNIER  Wannier densities and projection, a10
 *   RP_STAGE_BATCH    one rp_chi0_batch graph launch, a2-a6 of every problem
 *                     (the per-stage timers do not run inside the graph)
 *   RP_STAGE_UNFOLD   symmetry unfolding of coefficients and eps^-1
 *   RP_STAGE_REDUCE   FP64 sums of the split-BF16 contraction's FP32 partial
 *                     tiles into chi, a6 (sliced or tail-split launches)
 * rp_profile(ctx, 1) enables and resets; rp_profile(ctx, 0) disables.
 * rp_profile_read synchronizes the stream and returns, per stage, the summed
 * milliseconds and the number of timed launches (arrays of RP_NSTAGE).
 */
enum {
    RP_STAGE_UGRID = 0,
    RP_STAGE_PAIR = 1,
    RP_STAGE_WEIGHTS = 2,
    RP_STAGE_PREP = 3,
    RP_STAGE_CHI = 4,
    RP_STAGE_SCREEN = 5,
    RP_STAGE_WANNIER = 6,
    RP_STAGE_BATCH = 7,
    RP_STAGE_UNFOLD = 8,
    RP_STAGE_REDUCE = 9,
    RP_NSTAGE = 10
};

rp_status rp_profile(rp_ctx *ctx, int enable);
rp_status rp_profile_read(rp_ctx *ctx, double *ms, long *count);

#ifdef __cplusplus
}
#endif

#endif /* RP_H */
