/*
 * kr.h -- C ABI of the per-cell implicit thermochemistry library (libkr.so).
 *
 * The library integrates, for every cell independently, the stiff
 * thermochemical ODE system of the paper (Sec. 2.2, eq. method-ode-thermochem)
 *
 *     dn^i/dt = sum_r nu_ri w_r(n, T),      d eps/dt = Q(n, T),
 *     eps = T * sum_s c_s n_s   (T = eps / c_V),
 *
 * over one step dt, starting from the state left by the preceding fluid step
 * (Sec. 2.2.2).  w_r are mass-action rates with modified Arrhenius
 * coefficients k = A T^b exp(-E/T) (Sec. 2.2.1, item 1); reverse coefficients
 * follow from detailed balance; Q = sum_r qhat_r w_r is the chemical heat
 * release.  Each substep is backward Euler solved by Newton iteration with the
 * analytic Jacobian (Sec. 2.2.1, eq. method-jacobian) and a small dense LU
 * factorisation (Sec. 2.3.2, Algorithm algo:lu-decomp); the substep size is
 * adaptive.  Results are post-processed and failing cells are retried or
 * reverted as in Sec. 2.2.3.  All compute runs in HIP kernels on the device.
 *
 * Conventions
 *   - cgs units; energies divided by k_B (so in K).
 *   - Every device pointer is caller-owned device memory (e.g. a torch
 *     tensor's storage).  The library never frees caller memory.  Host
 *     pointers are read during the call only.
 *   - Return codes: KR_OK (0) or a negative KR_E* value.  No exception
 *     crosses the ABI.  On error no output has been written unless stated.
 *   - Calls are asynchronous on the given stream (NULL = the default stream)
 *     unless a host-side output (stats, max_out) is requested, in which case
 *     the call synchronises the stream before returning.
 *   - A network handle is immutable after creation and may be shared by
 *     calls on different streams, except that concurrent kr_chem_integrate
 *     / kr_work_order calls on one handle race on its work counter and its
 *     cell-order scratch: serialise them per handle (one stream per
 *     handle).
 */
#ifndef KR_H
#define KR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *kr_stream_t; /* a hipStream_t; NULL selects the null stream */

enum {
  KR_OK = 0,
  KR_EINVAL = -1,  /* bad argument (NULL pointer, size, non-conserving
                      reaction, reservoir carrying other rows, ...) */
  KR_EDEVICE = -2, /* a HIP runtime call failed */
  KR_ENOMEM = -3,  /* host or device allocation failed */
  KR_ECOMPILE = -4 /* the network's device code failed to compile */
};

/* ------------------------------------------------------------------------ */
/* Network description and handle                                            */
/* ------------------------------------------------------------------------ */

/* A user-chosen set of species and reactions (the paper lets the user pick
 * the species subset and reaction database in the input file, Sec. 2).
 * All pointers are host memory, copied at creation.
 *
 *   composition [n_rows][n_species]  atoms of element row v in species s
 *                                    (Sec. 2.1, N_{v,s}); rows at index
 *                                    >= n_elem are charge rows (+1 per
 *                                    positive charge, -1 for e-).
 *   reservoir   [n_rows]             the species that absorbs each row's
 *                                    post-processing correction (Sec. 2.2.3
 *                                    "single-element species"); it must carry
 *                                    only its own row.
 *   cv          [n_species]          per-particle c_V / k_B.
 *   h_form, s_form [n_species]       formation energy (K) and entropy (k_B)
 *                                    at the standard-state pressure p_ref.
 *   reac, prod  [n_reactions][3]     species of each side (multisets, -1
 *                                    padded); every reaction must conserve
 *                                    every row.
 *   arr_f       [n_reactions][3]     forward (A, b, E): k = A T^b e^{-E/T}.
 *   arr_r       [n_reactions][3]     explicit reverse (A, b, E), or NULL for
 *                                    detailed balance: k_r = k_f / K_eq with
 *                                    K_eq = (p_ref/(k_B T))^dnu exp(dS - dH/T).
 *   T_min, T_max                     temperature limits applied to the input
 *                                    state (Sec. 2.2.2).
 *   cv_poly [n_species][2][5]        optional (NULL: c_V constant, cv):
 *                                    temperature-dependent heat capacities,
 *                                    c_V/k_B = sum_k a_k T^k with one set of
 *                                    coefficients for T < T_mid and one for
 *                                    T >= T_mid (Sec. 4.2: NASA-style
 *                                    piecewise polynomials; cv is then
 *                                    unused).  The energy equation is written
 *                                    in eps = sum_s n_s e_s(T), e_s the
 *                                    integral of c_V,s from 0 (its upper
 *                                    piece shifted to be continuous at
 *                                    T_mid).
 *   tab_of [n_reactions], tab_log2k [n_tables][n_tab_nodes]
 *                                    optional (tab_of NULL: none): tabulated
 *                                    rate factors (Sec. 2.2.1, third rate
 *                                    type).  Reaction r with tab_of[r] = t >=
 *                                    0 has its forward coefficient multiplied
 *                                    by tau_t(T), log2 tau_t linear in log2 T
 *                                    between the nodes log2 T = tab_log2T0 +
 *                                    i tab_dlog2T (values tab_log2k[t][i];
 *                                    the end segments extended beyond the
 *                                    nodes); with detailed-balance reverse
 *                                    rates (arr_r NULL) the reverse
 *                                    coefficient carries the same factor.
 *                                    Set arr_f[r] = (1, 0, 0) for a purely
 *                                    tabulated coefficient.
 *   sigma_abs [n_species], photo [n_reactions]
 *                                    optional (NULL: none): photoreactions
 *                                    (Sec. 2.2.1, second rate type).
 *                                    photo[r] = 1 makes reaction r's forward
 *                                    coefficient A F_eff (arr_f[r] = (A, 0,
 *                                    0), A its cross-section in cm^2) and
 *                                    its reverse coefficient 0; F_eff is the
 *                                    cell's photon flux averaged over its
 *                                    path, attenuated by the absorbers
 *                                    sigma_abs (cm^2) of the cell
 *                                    (kr_options.photo_flux, photo_length).
 *                                    The Jacobian takes the flux derivative
 *                                    in n_i times min{1, n_i sigma_i /
 *                                    lambda^-1} (the paper's dominant-
 *                                    absorber cutoff).  Lane layout only.
 *   heat_extra [n_reactions][3]      optional (NULL: none): gas heating per
 *                                    net forward event besides the
 *                                    formation energies, q0 + q1 T + q2 T ln
 *                                    T (K): absorbed photon energy, radiated
 *                                    recombination energy (the heating and
 *                                    cooling of eq. method-ode-thermochem).
 *                                    Lane layout only.
 * Limits: 1 <= n_species <= KR_MAX_SPECIES, 0 <= n_rows <= KR_MAX_ROWS,
 * n_reactions >= 0, 2 <= n_tab_nodes <= KR_MAX_TAB_NODES, n_tables <=
 * n_reactions. */
#define KR_MAX_TAB_NODES 1024
#define KR_MAX_SPECIES 63
#define KR_MAX_ROWS 8

typedef struct {
  int32_t n_species;
  int32_t n_rows;
  int32_t n_elem;
  int32_t n_reactions;
  const int32_t *composition;
  const int32_t *reservoir;
  const double *cv;
  const double *h_form;
  const double *s_form;
  const int32_t *reac;
  const int32_t *prod;
  const double *arr_f;
  const double *arr_r;
  double p_ref;
  double T_min;
  double T_max;
  const double *cv_poly;
  double T_mid;
  int32_t n_tables;
  int32_t n_tab_nodes;
  const int32_t *tab_of;
  const double *tab_log2k;
  double tab_log2T0;
  double tab_dlog2T;
  const double *sigma_abs;
  const int32_t *photo;
  const double *heat_extra;
} kr_network_desc;

typedef struct kr_network kr_network;

/* Validates the description, derives reverse Arrhenius parameters, generates
 * the network's device code and compiles it for the current device (gfx950)
 * with hipRTC.  On success *out owns device memory until kr_network_destroy.
 * Errors: KR_EINVAL (invalid description; *out = NULL), KR_ECOMPILE,
 * KR_EDEVICE, KR_ENOMEM. */
int kr_network_create(const kr_network_desc *desc, kr_network **out);
void kr_network_destroy(kr_network *net);

/* Compile-time tuning of the generated kernels (chosen by the autotuner):
 *   waves_per_eu  occupancy the register allocator budgets for (1..8; the
 *                 lane's Newton matrix lives in VGPRs, so more waves means
 *                 fewer registers per lane and possibly scratch spills).
 *                 0 (default) chooses per network: 1 for the lane layout,
 *                 for the wavefront layout 2 where its LDS block leaves
 *                 room for two waves per SIMD, else 1; a several-network
 *                 launch runs lane- and wavefront-layout networks in
 *                 separate kernels when their choices differ
 *   pivot_tau     threshold of the LU's partial pivoting, (0, 1]: the
 *                 diagonal is kept unless its scaled magnitude is below
 *                 pivot_tau times the best candidate's (lane-per-cell
 *                 layout; the wave-per-cell LU takes the best candidate)
 *   layout        KR_LAYOUT_AUTO: one cell per lane below
 *                 KR_WIDE_MIN_SPECIES species, one cell per 32-lane group
 *                 from there up to 30 species, one cell per wavefront
 *                 beyond (measured on gfx950: the lane layout is 2-10x
 *                 faster at 5 and 9 species, the wavefront layout 5x faster
 *                 at 23, 32-lane groups another 8-15 % at 23); networks
 *                 with photoreactions or extra heat terms stay one cell per
 *                 lane at any size (the only layout that has them);
 *                 KR_LAYOUT_LANE / KR_LAYOUT_WAVE force one.  The
 *                 wavefront layout holds the Newton matrix one row per lane
 *                 and needs n_species <= 62 and 5 * 2 * n_reactions
 *                 rounded up to 320 <= 4095 (n_reactions <= 384).
 *                 KR_LAYOUT_GROUP16 / KR_LAYOUT_GROUP32: one cell per group
 *                 of 16 / 32 lanes (4 / 2 cells per wavefront), rows as in
 *                 the wavefront layout; needs n_species <= 14 / 30 besides
 *                 the wavefront layout's limits, and supports what it
 *                 supports (KR_FP64, KR_FP32LU_REFINE; its other kernels
 *                 are the wavefront layout's).
 *   lu_mfma       1: the FP32 LU of the KR_FP32LU_REFINE form runs blocked,
 *                 its trailing updates on FP32 MFMA tiles (wavefront layout
 *                 with n_species >= 31, where the rate table's LDS holds the
 *                 panel blocks; elsewhere ignored); 0 (default): the
 *                 unblocked LU on the vector ALUs.  Same solution up to
 *                 rounding; measured slower or faster per network (see the
 *                 autotuner). */
#define KR_LAYOUT_AUTO 0
#define KR_LAYOUT_LANE 1
#define KR_LAYOUT_WAVE 2
#define KR_LAYOUT_GROUP16 3
#define KR_LAYOUT_GROUP32 4
#define KR_WIDE_MIN_SPECIES 16
typedef struct {
  int32_t waves_per_eu;
  float pivot_tau;
  int32_t layout;
  int32_t lu_mfma;
} kr_build_opts;

void kr_default_build_options(kr_build_opts *opt);
/* kr_network_create with explicit build options (NULL = defaults). */
int kr_network_create_ex(const kr_network_desc *desc, const kr_build_opts *opt,
                         kr_network **out);

/* Number of unknowns per cell (n_species + 1: abundances and temperature). */
int kr_network_unknowns(const kr_network *net);
/* Layout the network was compiled for: KR_LAYOUT_LANE, KR_LAYOUT_WAVE,
 * KR_LAYOUT_GROUP16 or KR_LAYOUT_GROUP32. */
int kr_network_layout(const kr_network *net);

/* Derived Arrhenius table actually used: out[r][dir][3] = (A, b, E), dir 0
 * forward, 1 reverse (host memory, n_reactions * 6 doubles). */
int kr_network_arrhenius(const kr_network *net, double *out);

/* Size of the generated device source (bytes incl. NUL) and a copy of it
 * (truncated to buf_len - 1 bytes) when buf is not NULL. */
int64_t kr_network_source(const kr_network *net, char *buf, int64_t buf_len);

/* Validates a description and generates its device source without touching
 * a device; with compile != 0 also compiles it with hipRTC for gfx950.  The
 * source is copied to src_buf (truncated to src_len - 1 bytes) when src_buf
 * is not NULL.  Returns KR_OK or the error kr_network_create would return
 * for the same description. */
int kr_network_check(const kr_network_desc *desc, int compile, char *src_buf,
                     int64_t src_len);
/* kr_network_check with explicit build options (NULL = defaults). */
int kr_network_check_ex(const kr_network_desc *desc, const kr_build_opts *opt, int compile,
                        char *src_buf, int64_t src_len);

/* ------------------------------------------------------------------------ */
/* Integration                                                               */
/* ------------------------------------------------------------------------ */

/* Precision of the per-cell integration:
 *   KR_FP64           everything in FP64
 *   KR_FP32LU_REFINE  the LU in FP32; residual, iterative refinement and the
 *                     element projection in FP64 (same root as KR_FP64)
 *   KR_SINGLE         the paper's full single-precision mode (Sec. 2): the
 *                     cell's integration in FP32 (rates with the hardware's
 *                     exp2/log2, Jacobian, LU, iterate, error estimate; the
 *                     substep clock stays FP64), post-processing in FP64
 *   KR_MIXED          the paper's mixed-precision mode: as KR_SINGLE, but the
 *                     final abundance update of the call is FP64 (n_out =
 *                     n_in + the FP32 change); lane layout only (n_species <
 *                     KR_WIDE_MIN_SPECIES or KR_LAYOUT_LANE), as KR_SINGLE
 * In the FP32 modes a Newton iteration also stops once its update is within
 * 4 FP32 ulps of the iterate, and the retry thresholds (element residual,
 * negative abundance) are 1e-5 instead of 1e-10: rtol well below 1e-5 asks
 * for more than FP32 holds. */
enum { KR_FP64 = 0, KR_FP32LU_REFINE = 1, KR_SINGLE = 2, KR_MIXED = 3 };
enum { KR_ADAPTIVE = 0, KR_FIXED_STEP = 1 }; /* substep control */
/* Order in which the persistent kernel hands out a batch's cells.  Results
 * per cell are the same either way.  KR_ORDER_WORK first sorts the cells by
 * an estimate of their work, largest first, so that long cells do not start
 * last and leave the rest of their wavefront (and the GPU) idle: the
 * estimate is dt (sum_s |f_s| / sum_s n_s + |Q| / eps) at the input state,
 * bucketed in half-octaves (three extra kernels on the stream, one rate
 * evaluation per cell; the first call with a larger batch than before
 * allocates n_cells * 5 bytes and synchronises the device).  It pays for
 * batches of long, uneven cells (10 % faster on 2^20 combustion cells of
 * ~1e4 Newton iterations each) and costs more than it saves on cheap ones
 * (one substep per cell: the extra evaluation and the scattered, no longer
 * coalesced state accesses make the launch up to 7x slower), hence the
 * default KR_ORDER_INPUT; the autotuner measures both. */
enum { KR_ORDER_INPUT = 0, KR_ORDER_WORK = 1 };

/* Totals of one kr_chem_integrate call (requested through kr_options.stats;
 * the call then synchronises its stream).  Counts cover both attempts of a
 * retried cell. */
typedef struct {
  int64_t cells;             /* cells finished (every status) */
  int64_t substeps;          /* accepted substeps */
  int64_t newton_iterations;
  int64_t rejected;          /* substeps rejected by the error control */
  int64_t newton_failures;
  int64_t retried;           /* cells with status 1 */
  int64_t reverted;          /* cells with status 2 (the paper's "terminate"
                                decision is the caller's: check this) */
  int64_t refinement_sweeps; /* FP32 solves in refinement sweeps */
  int64_t fp64_fallbacks;    /* systems refinement did not settle (FP64 LU) */
  int64_t guess_fallbacks;   /* learned starts that Newton abandoned */
  double max_element_residual; /* over the cells not reverted, after
                                  post-processing, relative to the
                                  pre-processed input (see
                                  kr_element_residual) */
} kr_stats;

typedef struct {
  int32_t precision;    /* KR_FP64 (default), KR_FP32LU_REFINE, KR_SINGLE
                           or KR_MIXED (see above) */
  int32_t mode;         /* KR_ADAPTIVE (default) or KR_FIXED_STEP */
  int32_t n_fixed;      /* substeps per cell in KR_FIXED_STEP (>= 1) */
  int32_t max_newton;   /* Newton iterations per substep (default 10) */
  int32_t max_substeps; /* substep attempts per cell and attempt (100000) */
  int32_t order;        /* KR_ORDER_INPUT (default) or KR_ORDER_WORK */
  double floor;         /* absolute tolerance as a fraction of the nuclei
                           density (default 1e-20) */
  double newton_tol;    /* weighted max-norm bound on the Newton update
                           (default 1e-3) */
  double rho_floor;     /* density floor: cells with rho < rho_floor have
                           their abundances scaled by rho_floor/rho
                           (Sec. 2.2.2); default 0 = off */
  const double *guess;  /* device [n_species + 1][guess_ld] or NULL: Newton
                           starting point for each cell's first substep of
                           its first attempt (e.g. from kr_guess_predict);
                           if Newton fails from it, the same substep is
                           redone from the plain starting point (the
                           substep's initial state) before any step cut */
  int64_t guess_ld;
  unsigned long long *counters; /* device [8] or NULL, accumulated: [0]
                           substeps started from a guess, [1] guess
                           fallbacks, [2] row exchanges taken by the LU,
                           [3] FP32 solves in refinement sweeps (FP32 LU
                           form), [4] linear systems that refinement did
                           not settle and FP64 LU solved, [5..7] reserved */
  double *h_hint;       /* device [n_cells] in/out, or NULL.  In: the first
                           substep length of a cell's first attempt, used
                           when positive and finite (else dt), so that a
                           simulation loop carries each cell's step from one
                           call (fluid step, Sec. 2.2.2) to the next.  Out
                           (adaptive mode, cells not reverted): the
                           controller's proposed length after the last
                           accepted substep -- its update of that substep,
                           or the length before that substep was clipped to
                           land on dt if larger.  Other cells keep it. */
  double *h_log;        /* device [h_log_cap][h_log_ld], or NULL: the
                           accepted substep lengths, in order, of the
                           attempt that produced each cell's result (the
                           first h_log_cap of them; entries past the count
                           are unspecified) */
  int64_t h_log_ld;     /* >= n_cells when h_log is given */
  int32_t h_log_cap;    /* >= 0 */
  int32_t reserved;
  int32_t *h_log_n;     /* device [n_cells] or NULL: the number of accepted
                           substeps of that attempt (may exceed h_log_cap;
                           0 for reverted cells and cells with dt = 0) */
  kr_stats *stats;      /* host, or NULL: totals of this call (synchronises) */
  const double *photo_flux;   /* device [n_cells] or NULL (no radiation):
                           each cell's optically thin photon flux F (cm^-2
                           s^-1) for the network's photoreactions */
  const double *photo_length; /* device [n_cells] or NULL (optically thin):
                           each cell's path length L (cm) along the rays;
                           the photoreactions see F_eff = F (1 - e^-tau) /
                           tau, tau = L sum_s sigma_s n_s (Sec. 2.2.1 and
                           eq. method-rad-equiv-flux: the path average over
                           the cell) */
} kr_options;

void kr_default_options(kr_options *opt);

/* Advances every cell by its step.
 *   states  device [n_species][ld] (SoA), in/out, cm^-3; ld >= n_cells
 *   T       device [n_cells], in/out, K
 *   rho     device [n_cells] g cm^-3 (used by the density floor) or NULL
 *   dt      device [n_cells] s, or NULL to use dt_scalar for every cell
 *   rtol    relative tolerance (> 0) of the substep error control and of
 *           the Newton convergence test
 *   opt     NULL for defaults
 *   status  device [n_cells] or NULL: 0 ok, 1 ok after the retry with a
 *           reduced first substep, 2 reverted (the cell's inputs are left
 *           untouched: the paper's reversion to pre-evolution values)
 *   cell_stats device [n_cells][4] int32 or NULL: accepted substeps, Newton
 *           iterations, rejected substeps, Newton failures
 * Errors: KR_EINVAL (NULL handle/arrays, n_cells < 0, ld < n_cells,
 * rtol <= 0, bad options), KR_EDEVICE, KR_ENOMEM (cell-order scratch with
 * KR_ORDER_WORK).  n_cells == 0 is a no-op. */
int kr_chem_integrate(const kr_network *net, int64_t n_cells, double *states,
                      int64_t ld, double *T, const double *rho,
                      const double *dt, double dt_scalar, double rtol,
                      const kr_options *opt, int32_t *status,
                      int32_t *cell_stats, kr_stream_t stream);

/* kr_chem_integrate for callers that cannot allocate (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, kernels and results, but no allocation of any kind.  Its
 * workspace (work counter, totals, cell-order buffers) is a static device
 * array of KR_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends;
 * its device address is looked up when the first network is created on that
 * GPU.  KR_ORDER_WORK is limited to KR_NOALLOC_MAX_ORDER_CELLS cells
 * (KR_EINVAL beyond); input order has no size limit.  Every call on one GPU
 * shares the array: calls that overlap on one GPU (different streams, or
 * different networks concurrently) race and give wrong results, so
 * serialise them per GPU.  Errors as kr_chem_integrate. */
#define KR_NOALLOC_SCRATCH_BYTES (8ll << 20)
#define KR_NOALLOC_MAX_ORDER_CELLS ((KR_NOALLOC_SCRATCH_BYTES - 4096) / 5)
int kr_chem_integrate_noalloc(const kr_network *net, int64_t n_cells, double *states,
                              int64_t ld, double *T, const double *rho,
                              const double *dt, double dt_scalar, double rtol,
                              const kr_options *opt, int32_t *status,
                              int32_t *cell_stats, kr_stream_t stream);

/* The order in which kr_chem_integrate with KR_ORDER_WORK hands out this
 * batch's cells: order[i] = index of the i-th cell handed out, largest
 * expected work first (see KR_ORDER_WORK; cells of one half-octave bucket
 * in arbitrary order).  states, ld, T, rho, dt, dt_scalar as for
 * kr_chem_integrate (read only); opt supplies floor and rho_floor (NULL for
 * defaults); order device [n_cells] uint32.  Shares the network's ordering
 * scratch with kr_chem_integrate: calls on one network are serialised by
 * the caller.  Errors: KR_EINVAL (NULL arrays, ld < n_cells,
 * n_cells > 2^32 - 1), KR_EDEVICE, KR_ENOMEM. */
int kr_work_order(const kr_network *net, int64_t n_cells, const double *states, int64_t ld,
                  const double *T, const double *rho, const double *dt, double dt_scalar,
                  const kr_options *opt, uint32_t *order, kr_stream_t stream);

/* Per-cell conservation residual (the constant-element-abundance invariant,
 * Sec. 2.1 eq. method-const-elem, taken per cell between two states):
 *   resid[c] = max_v |sum_s N_vs (after - before)_s| / D_v,
 *   D_v = sum_s |N_vs| before_s for element rows, the nuclei density for
 *   charge rows.
 *   before, after device [n_species][ld]; resid device [n_cells] or NULL;
 *   max_out host pointer or NULL (then the call synchronises).
 * Errors: KR_EINVAL, KR_EDEVICE, KR_ENOMEM. */
int kr_element_residual(const kr_network *net, int64_t n_cells,
                        const double *before, const double *after, int64_t ld,
                        double *resid, double *max_out, kr_stream_t stream);

/* Post-processing alone (Sec. 2.2.3), the three stages kr_chem_integrate
 * applies to each integrated cell: (1) negative abundances to zero; (2) each
 * conserved row's reservoir species absorbs the difference between the
 * row's total in `before` (after pre-processing: negatives clipped) and in
 * `after`; (3) a reservoir left negative is refilled by breaking up, just
 * enough, the most abundant species that carries its row with its sign
 * (into the reservoirs of all that species' rows), then the next one.
 *   before  device [n_species][ld] (read only)
 *   after   device [n_species][ld], post-processed in place
 *   flags   device [n_cells] int32 or NULL: bit 0 a clip, bit 1 a break-up
 * Non-finite values propagate.  Temperatures are not involved.
 * Errors: KR_EINVAL, KR_EDEVICE. */
int kr_postprocess(const kr_network *net, int64_t n_cells, const double *before,
                   double *after, int64_t ld, int32_t *flags, kr_stream_t stream);

/* One forward-Euler stage of the stoichiometry-compatible PLM advection of
 * the species (Sec. 2.1, eqs. method-flux-sp, method-plm-general,
 * method-sto-plm-def, method-sto-plm-proj, method-sto-plm-recon) along lines
 * of cells with periodic ends: every face takes its upwind cell's species
 * per mass x = n / rho (upwind by the sign of the face's mass flux),
 * extrapolated to the face with the modified van Leer slope for non-uniform
 * grids (the limiter of Mignone 2014 that the paper names), the correction
 * projected onto the null space of the network's element-species matrix
 * (P = V V^T), so that the species fluxes F_s = x_face,s F_rho carry element
 * fluxes proportional to the mass flux; then
 *   n_out = alpha base + beta (n_in - dt / dx (F(i+1/2) - F(i-1/2)))
 * (alpha is ignored when base is NULL; two such stages with (alpha, beta) =
 * (0, 1) and (1/2, 1/2), base = the step's initial state, make the SSP-RK2
 * step).  The density's own update (by the same mass fluxes) is the
 * caller's.
 *   n_lines, n_cells   lines and cells per line (>= 3); cell i of line l is
 *                      column l * line_stride + i of the [S][ld] arrays
 *   n_in, n_out, base  device [n_species][ld]; n_out must not alias n_in
 *   rho                device [cells]: density of the stage's input state
 *   flux               device [cells]: mass flux through each cell's left
 *                      face (face i-1/2 of cell i; periodic)
 *   xc, xf             device [n_cells] cell centres and [n_cells + 1] faces
 *                      of every line (xf[n_cells] - xf[0] the period)
 *   mode               1 projected PLM; 0 PLM without the projection (the
 *                      paper's non-conserving comparison); 2 donor cell
 * Errors: KR_EINVAL, KR_EDEVICE.  Asynchronous on the stream. */
int kr_advect_plm(const kr_network *net, int64_t n_lines, int64_t n_cells,
                  int64_t line_stride, const double *n_in, double *n_out,
                  int64_t ld, const double *rho, const double *flux,
                  const double *xc, const double *xf, double dt,
                  const double *base, double alpha, double beta, int32_t mode,
                  kr_stream_t stream);

/* One whole SSP-RK2 step of the same advection (Sec. 2.1; the time
 * integrator of the test of Sec. 4.1) in one pass over memory:
 *   u1    = n_in - dt / dx (F(i+1/2) - F(i-1/2))   the faces of n_in / rho0
 *                                                  with the mass fluxes flux0
 *   n_out = 1/2 n_in + 1/2 (u1 - dt / dx (F1(i+1/2) - F1(i-1/2)))
 *                                                  the faces of u1 / rho1
 *                                                  with the mass fluxes flux1
 * -- the two kr_advect_plm stages with (alpha, beta) = (0, 1) and (1/2,
 * 1/2), base n_in, with the same bits, but the intermediate u1 stays on
 * chip (registers up to 32 species, LDS beyond; each wavefront or
 * workgroup updates the first stage on a halo of two cells around its
 * own), so the step reads n_in and writes n_out once.  rho1 and
 * flux1 are the first stage's density and its face mass fluxes, which the
 * caller computes from rho0 and flux0 (the density's own update is the
 * caller's, as for kr_advect_plm).
 *   n_lines, n_cells   lines and cells per line (>= 4); cell i of line l is
 *                      column l * line_stride + i of the [S][ld] arrays
 *   n_in, n_out        device [n_species][ld]; n_out must not alias n_in
 *   rho0, flux0        device [cells]: density and left-face mass flux of
 *                      the step's start
 *   rho1, flux1        device [cells]: the same after the first stage
 *   xc, xf, dt, mode   as for kr_advect_plm
 * Errors: KR_EINVAL, KR_EDEVICE.  Asynchronous on the stream. */
int kr_advect_plm_ssprk2(const kr_network *net, int64_t n_lines, int64_t n_cells,
                         int64_t line_stride, const double *n_in, double *n_out,
                         int64_t ld, const double *rho0, const double *flux0,
                         const double *rho1, const double *flux1,
                         const double *xc, const double *xf, double dt,
                         int32_t mode, kr_stream_t stream);

/* Fastest self-coupling timescale of each cell at its (pre-processed) input
 * state, out[c] = 1 / max(max_s |df_s/dn_s|, |dQ/dT| / c_V), capped at 1e7 s
 * (device arrays; used to express steps in units of the cell's stiffness). */
int kr_fastest_timescale(const kr_network *net, int64_t n_cells,
                         const double *states, int64_t ld, const double *T,
                         double *out, kr_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Several networks in one launch                                            */
/* ------------------------------------------------------------------------ */

/* Up to 4 networks compiled into one module whose persistent kernel drains
 * each network's cell queue in turn (each wave works on one network at a
 * time, so lanes never diverge across networks; waves start on different
 * networks so the queues drain together).  The networks must outlive the
 * handle. */
typedef struct kr_multi kr_multi;

/* One network's cells for kr_chem_integrate_multi: the arrays and their
 * meaning are those of kr_chem_integrate. */
typedef struct {
  int64_t n_cells;
  double *states;
  int64_t ld;
  double *T;
  const double *rho;
  const double *dt;
  double dt_scalar;
  int32_t *status;
  int32_t *cell_stats;
} kr_batch;

int kr_multi_create(const kr_network *const *nets, int32_t n_nets,
                    const kr_build_opts *opt, kr_multi **out);
void kr_multi_destroy(kr_multi *m);
/* Integrates batches[k] with network k in one launch: one persistent
 * kernel for all networks, or one per occupancy group (lane- and
 * wavefront-layout networks compiled for different waves per SIMD), run in
 * order on the stream.  use_graph != 0: the launch ([order kernels] ->
 * [reset work counters] -> [integrate]) is
 * captured into a hipGraph on first use and replayed on later calls with
 * the same arguments (re-captured when they change).  Options apply to all
 * batches; the learned guess is not supported here (KR_EINVAL).  Calls on
 * one handle must be serialised. */
int kr_chem_integrate_multi(kr_multi *m, const kr_batch *batches, double rtol,
                            const kr_options *opt, int32_t use_graph,
                            kr_stream_t stream);
/* Graph replays so far (return value) and captures (*captures if not NULL). */
int64_t kr_multi_graph_stats(const kr_multi *m, int64_t *captures);
/* kr_network_check for a set of descriptions compiled into one module. */
int kr_multi_check(const kr_network_desc *const *descs, int32_t n_nets,
                   int compile, char *src_buf, int64_t src_len);

/* ------------------------------------------------------------------------ */
/* Learned Newton guess                                                      */
/* ------------------------------------------------------------------------ */

/* A small MLP that maps (log10 of each abundance over the nuclei density,
 * floored at 1e-20; log10 T; log10 h) to the change of those logarithms
 * (species and T) over one backward-Euler substep of length h.  Its output
 * is only a Newton starting point (kr_options.guess); the Newton residual
 * of the method decides the result.  The paper names a learned solver as
 * the direction for acceleration (Sec. 5, DeepODE).
 *
 * Architecture: (S + 2) inputs -> `layers` x [Linear(hidden) + GELU(tanh)]
 * -> Linear(S + 1).  BF16 weights and activations in every product (MFMA),
 * FP32 accumulation, FP32 biases, gradients and Adam master weights.
 * Inputs and targets are standardised by per-column mean and standard
 * deviation (normalisation block: mu_in[16], sd_in[16], mu_out[16],
 * sd_out[16]).  Parameter layout (FP32, flat): for each linear layer l,
 * W_l [fan_out][fan_in] row-major, then b_l [fan_out].
 * Supports networks of at most 14 species. */
typedef struct kr_guess kr_guess;

typedef struct {
  int64_t steps;   /* Adam steps in this call */
  int32_t batch;   /* rows per step, drawn uniformly with replacement */
  int32_t reserved;
  float lr, lr_min;        /* cosine decay from lr to lr_min over the call */
  float beta1, beta2, eps; /* Adam */
  uint64_t seed;           /* batch sampling stream; 0 = consecutive blocks
                              of rows (deterministic) */
} kr_train_opts;

/* Allocates the model on the network's device, initialised uniformly in
 * +-1/sqrt(fan_in) from a splitmix64 stream of `seed`.  Errors: KR_EINVAL
 * (sizes, more than 14 species), KR_EDEVICE. */
int kr_guess_create(const kr_network *net, int32_t hidden, int32_t layers,
                    uint64_t seed, kr_guess **out);
void kr_guess_destroy(kr_guess *g);
int64_t kr_guess_num_params(const kr_guess *g);
/* FP32 master parameters to / from host memory (kr_guess_num_params floats;
 * set also re-rounds the BF16 copies).  Synchronous. */
int kr_guess_get_params(const kr_guess *g, float *host);
int kr_guess_set_params(kr_guess *g, const float *host);
/* Normalisation block (64 floats, host).  Synchronous. */
int kr_guess_get_normalization(const kr_guess *g, float *norm64);
int kr_guess_set_normalization(kr_guess *g, const float *norm64);

/* Raw features X [n][S+2] (device FP32) of n cells (states SoA [S][ld],
 * T [n], step dt [n] or dt_scalar). */
int kr_guess_features(const kr_guess *g, int64_t n, const double *states,
                      int64_t ld, const double *T, const double *dt,
                      double dt_scalar, float *X, kr_stream_t stream);
/* Raw targets Y [n][S+1] (device FP32): change of the logarithms between
 * two states of the same cells (same layout and ld). */
int kr_guess_targets(const kr_guess *g, int64_t n, const double *before,
                     const double *T_before, const double *after,
                     const double *T_after, int64_t ld, float *Y,
                     kr_stream_t stream);
/* Sets the normalisation from the column means and standard deviations of
 * X and Y (n >= 2 rows, device). */
int kr_guess_fit_normalization(kr_guess *g, int64_t n, const float *X,
                               const float *Y, kr_stream_t stream);
/* Loss and gradient (FP32, device, kr_guess_num_params floats, may be NULL)
 * of the first B rows of X, Y without updating; *loss (host, may be NULL)
 * is the mean squared error in standardised units (synchronises). */
int kr_guess_gradients(kr_guess *g, int32_t B, const float *X, const float *Y,
                       float *grads, double *loss, kr_stream_t stream);
/* opts->steps Adam steps on batches drawn from the n rows of X, Y; *loss
 * (host, may be NULL) is the last batch's loss (synchronises). */
int kr_guess_train(kr_guess *g, int64_t n, const float *X, const float *Y,
                   const kr_train_opts *opts, double *last_loss,
                   kr_stream_t stream);
/* Standardised outputs out [n][S+1] (device FP32) for raw features X. */
int kr_guess_forward(kr_guess *g, int64_t n, const float *X, float *out,
                     kr_stream_t stream);
/* The Newton starting point for one substep of length dt of each cell:
 * guess [S+1][guess_ld] (device FP64; species rows then T).  X_scratch:
 * device FP32 [n][S+2] workspace (caller-owned). */
int kr_guess_predict(kr_guess *g, int64_t n, const double *states, int64_t ld,
                     const double *T, const double *dt, double dt_scalar,
                     float *X_scratch, double *guess, int64_t guess_ld,
                     kr_stream_t stream);

/* Last error message of the calling thread (static storage). */
const char *kr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
