/*
 * sr.h -- C ABI of libsr.so, the MI355X (gfx950) implementation of the
 * real-time synchrotron photon emission method of Wallin, Gonoskov & Marklund,
 * "Effects of high energy photon emissions in laser generated ultra-relativistic
 * plasmas: real-time synchrotron simulations" (arXiv 1409.5574).
 *
 * Units: normalised, c = m = e = 1, electron charge q = -1.  Time is in
 * 1/omega_r, length in c/omega_r, momentum in mc, energy in mc^2, fields in
 * eE/(mc omega_r) and eB/(m omega_r).  hbar_n = hbar omega_r/(mc^2).
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are HIP device pointers owned by the caller
 *    (typically PyTorch tensors).  The library never frees or retains them
 *    beyond the call.  Pointers marked "host" are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously on it unless the entry point says
 *    SYNCHRONOUS.
 *  - Return value: SR_OK (0) or a negative sr_error code.  Argument errors are
 *    detected on the host before anything is launched, so a failed call has
 *    enqueued no work.  Conditions the emission step finds on the device
 *    (photon-segment overflow, recoil clamping, non-finite inputs) travel with
 *    its ledger partials; sr_ledger_reduce latches them as bits in the
 *    caller's status word, read back by sr_status().
 *  - Hot calls (sr_gather_push_emit*, sr_ledger_reduce, sr_spectrum_histogram,
 *    sr_step_epilogue, sr_field_standing_wave, sr_sort_particles, sr_mlp_*)
 *    allocate nothing.  Only sr_table_build allocates device memory (released
 *    by sr_table_free).
 *  - Calls that share device buffers must be ordered by the caller (same
 *    stream or events); the library keeps no global mutable state apart from
 *    the tables it hands out.
 */
#ifndef SR_H
#define SR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
typedef enum {
    SR_OK = 0,
    SR_E_INVAL = -1,       /* bad argument (null pointer, size, mode)          */
    SR_E_HIP = -2,         /* a HIP runtime call failed                         */
    SR_E_NOMEM = -3,       /* sr_table_build could not allocate                 */
    SR_E_UNSUPPORTED = -4  /* valid request the library does not provide      */
} sr_error;

/* Bits latched in the device status word (sr_ledger.status). */
enum {
    SR_W_PHOTON_OVERFLOW = 1u, /* a chunk emitted more photons than its segment holds;
                                  the surplus is counted, not stored, and its energy
                                  goes to ledger column SR_LED_DROPPED             */
    SR_W_RECOIL_CLAMP = 2u,    /* recoil larger than |p|: p set to 0, remainder in
                                  ledger column SR_LED_CLAMPED                      */
    SR_W_NONFINITE = 4u,       /* a non-finite momentum or field value was met      */
    SR_W_CFL = 8u              /* sr_deposit_current: a particle moved a cell or more
                                  in one step; its current was not deposited         */
};

/* Ledger columns: one row of SR_LEDGER_COLS doubles per time step (FP64). */
enum {
    SR_LED_EMITTED = 0,  /* sum over emitted photons of weight * energy          */
    SR_LED_LL = 1,       /* sum w (2/3)(alpha/hbar_n) chi^2 beta^2 dt: the energy the
                            Landau-Lifshitz force (eq:LLformOfRRForce) removes     */
    SR_LED_RECOIL = 2,   /* sum w (gamma_after - gamma_before) of the recoil      */
    SR_LED_CLAMPED = 3,  /* sum w (recoil - |p|) where recoil exceeded |p|        */
    SR_LED_DROPPED = 4,  /* weight * energy of photons that did not fit           */
    SR_LED_PHOTONS = 5,  /* number of photons emitted (stored + dropped)          */
    SR_LED_WEIGHT = 6,   /* sum of particle weights processed                     */
    SR_LED_CHI_MAX = 7,  /* largest chi of the step                               */
    SR_LEDGER_COLS = 8
};

/* Particles per chunk when the caller gives no explicit chunking (one wave). */
#define SR_CHUNK 64

/* --------------------------------------------------------------- data types */
/* Macro-electrons, structure of arrays, FP32.  x[a] are positions measured from
 * the grid's lower corner (x[2] may be NULL for 2D, all may be NULL for the
 * uniform-field mode); p[a] = gamma v_a is the momentum at half step n-1/2 on
 * entry and n+1/2 on return; w are weights; id are persistent identifiers that
 * key the random streams (so results do not depend on the array order).  All
 * arrays are device, length n. */
typedef struct {
    int64_t n;
    float *x[3];
    float *p[3];
    float *w;          /* read only in the step */
    uint32_t *id;      /* read only in the step */
} sr_particles_f32;

/* Same, FP64 state (the precision-comparison path). */
typedef struct {
    int64_t n;
    double *x[3];
    double *p[3];
    double *w;         /* read only in the step */
    uint32_t *id;      /* read only in the step */
} sr_particles_f64;

/* Fields on a Yee grid, six device component arrays of n[0]*n[1]*n[2] FP32
 * values, x fastest.  Staggering in cells: Ex(1/2,0,0) Ey(0,1/2,0) Ez(0,0,1/2)
 * Bx(0,1/2,1/2) By(1/2,0,1/2) Bz(1/2,1/2,0).  Unused for dim == 0. */
typedef struct {
    const float *e[3];
    const float *b[3];
} sr_fields_f32;

/* Grid.  dim 0: uniform fields e0, b0 (no grid, positions not wrapped);
 * dim 2: n[2] == 1, positions x, y; dim 3: x, y, z.  Periodic in every axis;
 * the lower corner is the origin of the positions.  The emission step needs
 * n[0] >= 2 (SR_E_INVAL otherwise), fewer than 2^24 rows n[1] n[2] and fewer
 * than 2^30 cells (SR_E_UNSUPPORTED otherwise). */
typedef struct {
    int32_t dim;
    int32_t reserved;
    int64_t n[3];
    double dx[3];
    double e0[3];
    double b0[3];
} sr_grid;

enum { SR_SAMPLER_S = 0,          /* proposal S(x), section "Monte Carlo method"     */
       SR_SAMPLER_TABLE = 1,      /* direct: total rate, x from the inverse-CDF table */
       SR_SAMPLER_MLP = 2,        /* direct: total rate, x from the MLP surrogate     */
       SR_SAMPLER_QUANTUM = 3 };  /* proposal S(x) with the quantum-corrected kernel
                                     (chi approaching 1, section "Limitations"): the
                                     quantum synchrotron spectrum, delta = 1.5 chi x,
                                     xi = x/(1-delta),
                                     dN = dt (sqrt3/2pi) alpha H_eff Q / S(x),
                                     Q = (1-delta+1/(1-delta)) K_{2/3}(xi)
                                         - int_xi^inf K_{1/3},
                                     Q = 0 for delta >= 1 (kin_cut is implied);
                                     Q -> F(x)/x as chi -> 0                         */
enum { SR_RECOIL_NONE = 0, SR_RECOIL_PHOTON = 1, SR_RECOIL_LL = 2 };
enum { SR_DN_WEIGHT = 0, SR_DN_CLAMP = 1 };

typedef struct {
    double hbar_n;          /* hbar omega_r / (m c^2)                               */
    double alpha;           /* fine-structure constant                              */
    int32_t n_samples;      /* K >= 1 frequency trials per particle and step, each
                               carrying weight w/K (section "Monte Carlo method",
                               super-photon count and weights)                     */
    int32_t sampler;        /* SR_SAMPLER_*                                         */
    int32_t recoil;         /* SR_RECOIL_*                                          */
    int32_t dn_policy;      /* SR_DN_WEIGHT: dN >= 1 emits with weight w dN/K;
                               SR_DN_CLAMP: dN >= 1 emits with weight w/K           */
    int32_t kin_cut;        /* 1: no photon above the emitter's energy (x > 2/(3 chi)) */
    int32_t push_position;  /* 1: advance positions by dt p/gamma after the push    */
    const void *mlp_params; /* SR_SAMPLER_MLP: device bfloat16[SR_MLP_PARAMS]        */
    const uint8_t *mlp_fallback; /* SR_SAMPLER_MLP: device uint8[SR_MLP_FALLBACK_BINS]:
                               1 sends the trials of that log10 chi bin on
                               [-4, 2) (and any chi outside it) to the table       */
    double omega_grid;      /* > 0: the grid's cutoff frequency c/dx in units of
                               omega_r (section "The field setup": the grid resolves
                               radiation below it).  A photon of energy below
                               hbar_n omega_grid is not emitted (no record, no
                               recoil, not in the ledger's emitted column).  0: no
                               floor.  Not with SR_SAMPLER_MLP (SR_E_INVAL)        */
    int32_t gather;         /* SR_GATHER_DIRECT (0): every particle reads its stencil
                               from the grid in global memory.  SR_GATHER_BOX: on 3D
                               grids with uniform chunks, FP32 path, proposal, table
                               or quantum sampler, a block of 256 particles whose
                               stencils span at most SR_FIELD_BOX_NODES nodes (and do
                               not straddle a periodic boundary) first copies those
                               grid values into LDS with coalesced loads and
                               interpolates from there; other blocks, and other
                               configurations, read directly.  Both give
                               bit-identical results.                               */
    int32_t reserved;
} sr_params;
enum { SR_GATHER_DIRECT = 0, SR_GATHER_BOX = 1 };
#define SR_FIELD_BOX_NODES 1344

/* Chunking of the particle array.  Chunk c covers particles
 * [start[c], start[c+1]) when start != NULL (device, n_chunks+1 int64 values,
 * non-decreasing, start[0] = 0, start[n_chunks] = n), else
 * [c*SR_CHUNK, min((c+1)*SR_CHUNK, n)) with n_chunks = ceil(n / SR_CHUNK). */
typedef struct {
    int64_t n_chunks;
    const int64_t *start;
} sr_chunking;

/* Photon output.  The buffer is split into one segment per chunk: chunk c owns
 * slots [s_c * per_particle, e_c * per_particle) where [s_c, e_c) is its
 * particle range.  seg_count[c] receives the number of photons the chunk
 * emitted in this call; only the first min(seg_count[c], segment size) are
 * stored, in no particular order.  Arrays are device, sized n * per_particle
 * (seg_count: n_chunks).  k and step may be NULL. */
typedef struct {
    int64_t per_particle;
    uint32_t *seg_count;
    float *eps;         /* photon energy hbar omega in mc^2                        */
    float *w;           /* photon weight                                           */
    float *dir[3];      /* unit direction = mean momentum direction (section
                           "Modelling the relativistic case": photons along the
                           emitter's motion)                                        */
    float *pos[3];      /* emitter position x^n (pos[2] may be NULL in 2D)          */
    uint32_t *parent;   /* emitter id                                              */
    uint8_t *k;         /* trial index 0..K-1                                      */
    uint32_t *step;     /* step index                                              */
} sr_photon_buf;

/* FP64 energy ledger.  rows: device [n_rows][SR_LEDGER_COLS]; partials: device
 * workspace of at least sr_ledger_partials(n_chunks) doubles (the step writes
 * one partial row per group of four chunks, with the block's condition bits);
 * status: device uint32 into which sr_ledger_reduce ORs the condition bits of
 * the step it reduces (the caller zeroes it). */
typedef struct {
    double *rows;
    int64_t n_rows;
    double *partials;
    int64_t partials_len;
    uint32_t *status;
} sr_ledger;

/* Opaque spectrum tables built on the device in FP64 and read in FP32. */
typedef struct sr_table sr_table;

/* ------------------------------------------------------------ entry points */

/* Build the device tables (the "spectrum-table construction" of the FP64 split).
 * Their ranges and resolutions are fixed by the accuracy the step needs (the
 * trial density to ~1e-7 relative over every R' a 23-bit uniform can take, F
 * on x in [2^-18.5, 22.6], the cut fraction on log10 chi in [-6, 4]) and are
 * reported by sr_table_query; they are not arguments:
 *  - the synchrotron function F(x) = x int_x^inf K_{5/3} (section "Modelling
 *    the relativistic case"), as piecewise cubics in log2 x;
 *  - the trial density F(x)/(x S(x)) of the proposal sampler of section "Monte
 *    Carlo method" as piecewise cubics of its logarithm in log2 R' (lower
 *    branch) and log2(1 - R') (upper branch), so that a trial reads it directly
 *    from the uniform R';
 *  - the branch point P(a) of the proposal S(x), a^{4/3} + (7/9)e^{-a} = 1;
 *  - the inverse CDF of the photon-number spectrum F(x)/x with the optional
 *    kinematic cut, on a (log chi, u) grid, and the cut rate integral, for the
 *    direct samplers.
 * Allocates device memory, runs FP64 kernels on `stream` and synchronises it.
 * *out receives the handle.  SYNCHRONOUS. */
int sr_table_build(sr_table **out, void *stream);
void sr_table_free(sr_table *tab);

/* Host-side description of a built table (for tests and diagnostics). */
typedef struct {
    float proposal_pa;      /* binary32 branch point P(a)                          */
    int32_t f_pieces;       /* cubic pieces of log2 F                              */
    double proposal_a;      /* a, FP64                                             */
    int32_t t1_pieces;      /* cubic pieces of the uncut inverse number-CDF        */
    int32_t r_nodes;        /* nodes of the cut fraction r(chi)                     */
    double r_log10chi_lo, r_log10chi_hi;
    int32_t g_pieces;       /* cubic pieces of the trial density log2 F/(x S) in R' */
    int32_t q_pieces;       /* cubic pieces (each a pair) of the quantum kernel in
                               log2 xi                                              */
} sr_table_info;
int sr_table_query(const sr_table *tab, sr_table_info *info);

/* Evaluate the table's F at n device points x (device out). */
int sr_eval_synchrotron_F(const sr_table *tab, const float *x, float *out, int64_t n, void *stream);

/* dN of one proposal trial for n device (uniform word a, rate, chi) triples:
 * out_dn = rate F(x)/(x S(x)) (0 above the cut when kin_cut), out_x = x.
 * The same device functions the emission kernel uses (steps 3-5 of the list at
 * the end of section "Monte Carlo method"): F/(x S) is read from a table of
 * log2 F/(x S) built in FP64 as a function of R' itself. */
int sr_eval_trial(const sr_table *tab, const uint32_t *a, const float *rate, const float *chi,
                  int32_t kin_cut, float *out_dn, float *out_x, int64_t n, void *stream);

/* ---------------------------------------------------------- the PIC loop
 * The emission method runs inside a PIC code: particles on a grid, Maxwell's
 * equations for the field, the particles' currents feeding it (section "The
 * field setup"); the photons it emits are particles moving at c.  These calls
 * close that loop around sr_gather_push_emit.  Normalised units: E, B in
 * m c omega_r / e, lengths in c/omega_r, densities in n_r = m omega_r^2 /
 * (4 pi e^2): dB/dt = -curl E, dE/dt = curl B - J, div E = rho.  A particle of
 * weight w carries charge q w in units of n_r (c/omega_r)^3 (per unit length
 * in z for 2D).  Grid dim 2 or 3, periodic; arrays as sr_fields_f32 (x
 * fastest), J on the E points, rho on the nodes.  A step: sr_gather_push_emit
 * (gathers E, B at t^n, moves x^n -> x^{n+1}), sr_deposit_current (J of the
 * move, from a copy of x^n the caller kept), sr_field_step, sr_photon_advance.
 * All asynchronous on `stream`; the arrays are the caller's device memory. */

/* One Yee step with E and B kept at whole steps:
 *   B -= (dt/2) curl E;  E += dt (curl B - J);  B -= (dt/2) curl E
 * (forward differences for curl E on the B points, backward for curl B on the
 * E points).  j may be NULL (or j[0] NULL) for no current.  dt must satisfy
 * the Courant condition dt^2 sum_a 1/dx_a^2 < 1 (SR_E_INVAL otherwise). */
int sr_field_step(float *e[3], float *b[3], const float *j[3], const sr_grid *grid, double dt,
                  void *stream);

/* rho += charge w S / dV on the nodes, S the cloud-in-cell weights
 * (device float[cells], accumulated with float atomics: the order of the sums
 * is not fixed). */
int sr_deposit_rho(const sr_particles_f32 *parts, const sr_grid *grid, double charge, float *rho,
                   void *stream);

/* j += the charge-conserving current of the moves x_old -> parts->x (Esirkepov,
 * Comput. Phys. Commun. 135, 144 (2001), for the cloud-in-cell shape): the
 * discrete continuity equation rho(x) - rho(x_old) + dt div J = 0 holds for
 * the charge of sr_deposit_rho.  Moves are taken the shorter way round the
 * periodic box and must be below one cell per axis: a particle that moved
 * further deposits nothing and sets SR_W_CFL in *status (device uint32).  In
 * 2D, Jz is charge w v_z S / dV with v_z = p_z / gamma(p) of parts->p, the
 * momentum the position push used.  x_old: device arrays of the positions at
 * the start of the step (x_old[2] unused in 2D).  Each block of particles sums
 * its contributions exactly in fixed point, in units of 2^(e-21) where 2^e is
 * the power of two just above the largest bound B of a contribution in the
 * block (|c_a du_a| per axis, |c_z| for the 2D Jz), so that a contribution is
 * rounded by at most 2^-21 B; the block sums are then added to j with float
 * atomics, whose order is not fixed. */
int sr_deposit_current(const sr_particles_f32 *parts, const float *x_old[3], const sr_grid *grid,
                       double dt, double charge, float *j[3], uint32_t *status, void *stream);

/* Photons move at c along their direction: pos += dt dir for every stored
 * photon of the buffer (chunked as in sr_gather_push_emit), wrapped into the
 * periodic box on the grid's axes; pos arrays that are NULL are skipped. */
int sr_photon_advance(const sr_photon_buf *photons, const sr_chunking *chunks, int64_t n,
                      const sr_grid *grid, double dt, void *stream);

/* Validity diagnostics of the two limits the paper states for the method:
 *   SR_VALID_QUANTUM          chi >= 1: the classical emission formula fails and a
 *                             QED treatment is needed (section "Limitations");
 *   SR_VALID_NON_SYNCHROTRON  0 < H_eff tau_em <= 1: the field varies faster than
 *                             the particle turns by 1/gamma, tau_em <= 1/(gamma
 *                             omega_H), so the emission need not have the
 *                             synchrotron (wiggler) spectrum (section "Synchrotron
 *                             emission", the criterion a^-1 < omega_L tau_EM).
 * H_eff and chi are those the emission step computes (gather, Boris push,
 * eq:effective_H), without emission and without writing the particles.
 * tau_em > 0: the time scale of the field variation in units of 1/omega_r (for
 * a laser, 1/omega_L).  flags: device uint8[parts->n] or NULL.  sums: device
 * double[SR_VALID_SUMS] receiving {sum w, sum w [quantum], sum w
 * [non-synchrotron], sum w LL, sum w LL [quantum], sum w LL [non-synchrotron]},
 * LL the Landau-Lifshitz energy of the step (ledger column SR_LED_LL), summed
 * in a fixed order.  work: device double[sr_validity_work(parts->n)]. */
enum { SR_VALID_QUANTUM = 1u, SR_VALID_NON_SYNCHROTRON = 2u, SR_VALID_SUMS = 6 };
int sr_validity(const sr_particles_f32 *parts, const sr_fields_f32 *fields, const sr_grid *grid,
                double dt, const sr_params *prm, double tau_em, uint8_t *flags, double *sums,
                double *work, void *stream);
int64_t sr_validity_work(int64_t n);

/* dN of one quantum trial (SR_SAMPLER_QUANTUM) for n device (word a, rate, chi)
 * triples: out_dn = rate Q(x, chi)/S(x), out_x = x, with x and S from the
 * proposal exactly as sr_eval_trial; the emission kernel's device function.
 * Q is read from a table of log2 K_{2/3} and log2 int K_{1/3} in log2 xi built
 * in FP64; xi >= 128 (Q < e^-128) gives 0. */
int sr_eval_trial_quantum(const sr_table *tab, const uint32_t *a, const float *rate,
                          const float *chi, float *out_dn, float *out_x, int64_t n, void *stream);

/* Gather, Boris push and H_eff of every particle, exactly as the emission step
 * computes them (section "Numerical implementation": E and B interpolated to
 * the particle, the Boris scheme, and eq:effective_H from the momenta of the two
 * neighbouring steps with dp_perp/p limited to 1), without emission and
 * without writing the particles: out_heff = H_eff, out_chi = hbar_n H_eff
 * gamma_bar, out_gamma_bar = the mean gamma of the step (device FP64 arrays of
 * parts->n).  Only prm->hbar_n and prm->alpha are read.  The _f64 variant runs
 * the FP64 gather and push of sr_gather_push_emit_f64.  For the per-result
 * precision report of the FP32 / FP64 split. */
int sr_eval_push(const sr_particles_f32 *parts, const sr_fields_f32 *fields, const sr_grid *grid,
                 double dt, const sr_params *prm, double *out_heff, double *out_chi,
                 double *out_gamma_bar, void *stream);
int sr_eval_push_f64(const sr_particles_f64 *parts, const sr_fields_f32 *fields,
                     const sr_grid *grid, double dt, const sr_params *prm, double *out_heff,
                     double *out_chi, double *out_gamma_bar, void *stream);

/* Philox4x32-10 (Salmon et al., SC'11) as used by the kernels: n counters
 * ctr[i][4] (device) with key (seed low, seed high) -> out[i][4] (device). */
int sr_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out, int64_t n, void *stream);

/* One time step of the emission method for every particle (FP32 path):
 *   gather E, B at x^n (CIC on the Yee grid, or the uniform fields);
 *   Boris push p^{n-1/2} -> p^{n+1/2};
 *   H_eff from the two momenta (eq:effective_H) with dp_perp/p limited to 1;
 *   omega_c = 1.5 H_eff gamma^2 and chi = hbar_n H_eff gamma;
 *   K Monte-Carlo trials (the six steps listed at the end of section "Monte
 *   Carlo method"), random words from Philox4x32-10 with counter
 *   (id, step, k/2, 0) and key seed;
 *   photon append into the chunk's segment, recoil, position push.
 * Writes FP64 ledger partial rows, with the condition bits found, into
 * ledger->partials (sum them into a ledger row with sr_ledger_reduce, passing
 * the same n_chunks; that call latches the bits into ledger->status).  With
 * per_particle == 0 nothing is stored and every photon
 * is counted as dropped.  Explicit chunk starts are trusted: the caller
 * guarantees 0 = start[0] <= ... <= start[n_chunks] = n. */
int sr_gather_push_emit(sr_particles_f32 *parts, const sr_fields_f32 *fields, const sr_grid *grid,
                        double dt, uint64_t seed, uint64_t step, const sr_params *prm,
                        const sr_table *tab, const sr_chunking *chunks, sr_photon_buf *photons,
                        sr_ledger *ledger, void *stream);

/* The same step with FP64 state, FP64 gather (of the FP32 grid values), FP64
 * Boris push and H_eff; the trials run in FP32 as in the FP32 path. */
/* sr_gather_push_emit with timing: ev_start and ev_stop are HIP events
 * (hipEvent_t, created by the caller) that the kernel's own dispatch records at
 * its start and end (hipExtLaunchKernel), so their elapsed time is the
 * kernel's duration without the queue packets a separate event record adds.
 * Either may be NULL.  Results are those of sr_gather_push_emit. */
int sr_gather_push_emit_timed(sr_particles_f32 *parts, const sr_fields_f32 *fields,
                              const sr_grid *grid, double dt, uint64_t seed, uint64_t step,
                              const sr_params *prm, const sr_table *tab, const sr_chunking *chunks,
                              sr_photon_buf *photons, sr_ledger *ledger, void *ev_start,
                              void *ev_stop, void *stream);
int sr_gather_push_emit_f64(sr_particles_f64 *parts, const sr_fields_f32 *fields,
                            const sr_grid *grid, double dt, uint64_t seed, uint64_t step,
                            const sr_params *prm, const sr_table *tab, const sr_chunking *chunks,
                            sr_photon_buf *photons, sr_ledger *ledger, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation): sr_gather_push_emit followed by
 * sr_ledger_reduce into *ledger_row (device double[SR_LEDGER_COLS]), with the
 * step's partial ledger rows kept in a device array inside the library instead
 * of a caller workspace.  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call).  Results are those of the two calls with the same
 * arguments; the condition bits are ORed into *status (device uint32, zeroed
 * by the caller).  At most SR_NOALLOC_MAX_CHUNKS chunks (2^26 particles with
 * uniform chunks): SR_E_UNSUPPORTED above.  The array (about 21 MB) is held
 * by every device the library runs on until the process ends; all calls on
 * one device share it, so calls that overlap on one device (other streams,
 * other threads) race and must be ordered by the caller.  stream must belong
 * to the current device (SR_E_INVAL otherwise). */
#define SR_NOALLOC_MAX_CHUNKS (1 << 20)
int sr_gather_push_emit_noalloc(sr_particles_f32 *parts, const sr_fields_f32 *fields,
                                const sr_grid *grid, double dt, uint64_t seed, uint64_t step,
                                const sr_params *prm, const sr_table *tab,
                                const sr_chunking *chunks, sr_photon_buf *photons,
                                double *ledger_row, uint32_t *status, void *stream);

/* n_steps steps of sr_gather_push_emit in one launch for uniform fields (grid->dim
 * == 0, SR_E_UNSUPPORTED otherwise; uniform chunks; proposal, table or quantum
 * sampler; no grid floor): every particle stays in registers across the steps
 * (step numbers step0 .. step0 + n_steps - 1 key the random streams), and the
 * ledger of step step0 + s goes to ledger->rows[s] (n_rows >= n_steps), summed
 * in a fixed order, with the condition bits latched into *ledger->status.  The
 * photon segments are shared by all the steps of the call: chunk c's
 * seg_count[c] counts the photons of every step, photons->step (if not NULL)
 * receives each record's step, and a photon beyond the segment counts as
 * dropped in its step's row.  ledger->partials: sr_ledger_partials_steps(
 * n_chunks, n_steps) doubles.  The uniform-field case of section "Comparison
 * and benchmarking" (a particle in a constant magnetic field). */
int sr_gather_push_emit_steps(sr_particles_f32 *parts, const sr_grid *grid, double dt, uint64_t seed,
                              uint64_t step0, int64_t n_steps, const sr_params *prm,
                              const sr_table *tab, sr_photon_buf *photons, sr_ledger *ledger,
                              void *stream);
int64_t sr_ledger_partials_steps(int64_t n_chunks, int64_t n_steps);

/* Sum the partial rows a step over n_chunks chunks wrote into ledger->rows[row]
 * (FP64, fixed order, so the result is reproducible; column SR_LED_CHI_MAX is
 * a maximum) and OR the step's condition bits into *ledger->status.  The
 * energy ledger of the section "Comparison and benchmarking": emitted photon
 * energy against the Landau-Lifshitz loss. */
int sr_ledger_reduce(const sr_ledger *ledger, int64_t n_chunks, int64_t row, void *stream);

/* Workspace length (doubles) for ledger->partials with n_chunks chunks. */
int64_t sr_ledger_partials(int64_t n_chunks);

/* The per-step energy ledger of section "Comparison and benchmarking" (Fig. 3:
 * the energy the emitted photons carry against the Landau-Lifshitz radiation-
 * reaction loss of eq:LLformOfRRForce): copy ledger row `row` (columns
 * SR_LED_*, FP64) to host out[SR_LEDGER_COLS].  SYNCHRONOUS on stream. */
int sr_energy_ledger(const sr_ledger *ledger, int64_t row, double *out, void *stream);

/* Read (and, if clear != 0, zero) the latched status bits.  SYNCHRONOUS. */
int sr_status(const sr_ledger *ledger, uint32_t *flags, int32_t clear, void *stream);

/* Energy-weighted photon spectrum: hist[0..n_bins) += sum w*eps and
 * hist[n_bins..2 n_bins) += sum w over the stored photons of every chunk,
 * binned in log eps on [eps_lo, eps_hi).  hist is device FP64; work is a
 * device workspace of sr_hist_work(n_bins) doubles. */
int sr_spectrum_histogram(const sr_photon_buf *photons, const sr_chunking *chunks, int64_t n,
                          double eps_lo, double eps_hi, int32_t n_bins, double *hist,
                          double *work, void *stream);
int64_t sr_hist_work(int32_t n_bins);

/* The end of a step in two launches instead of four: exactly
 *   sr_ledger_reduce(ledger, n_chunks, row) and
 *   sr_spectrum_histogram(photons, chunks, n, eps_lo, eps_hi, n_bins, hist, work),
 * with the same arguments, argument checks and results (the ledger row
 * bit-identical; the histogram equal up to the order of its FP64 additions).
 * The first launch runs the ledger's first level beside the histogram's
 * accumulation, the second the ledger's last level beside the histogram's
 * reduction. */
int sr_step_epilogue(const sr_ledger *ledger, int64_t n_chunks, int64_t row,
                     const sr_photon_buf *photons, const sr_chunking *chunks, int64_t n,
                     double eps_lo, double eps_hi, int32_t n_bins, double *hist, double *work,
                     void *stream);

/* Angular distribution of the emitted energy over the front hemisphere around
 * `axis` (section "Comparison and benchmarking", Fig. 4: the front hemisphere
 * around the laser propagation direction):
 *   hist[it * n_phi + ip] += sum w*eps over the stored photons with theta, the
 *   angle between dir and axis, in [it, it+1) * (pi/2)/n_theta, and phi, the
 *   azimuth about the axis measured from the part of `ref` perpendicular to it
 *   (towards axis x ref), in [ip, ip+1) * 2 pi/n_phi;
 *   hist[n_theta * n_phi] += sum w*eps of the photons with dir . axis <= 0.
 * axis and ref: host vectors (any length; ref not parallel to axis).  hist is
 * device FP64 [n_theta * n_phi + 1]; work a device workspace of
 * sr_angular_work(n_theta, n_phi) doubles; n_theta * n_phi <= 4096. */
int sr_angular_histogram(const sr_photon_buf *photons, const sr_chunking *chunks, int64_t n,
                         const double axis[3], const double ref[3], int32_t n_theta,
                         int32_t n_phi, double *hist, double *work, void *stream);
int64_t sr_angular_work(int32_t n_theta, int32_t n_phi);

/* Prescribed field for the workloads: two counter-propagating circularly
 * polarised waves of amplitude a0 along x (k = omega = 1) forming
 *   E = 2 a0 cos x (0, cos t, -sin t),  B = 2 a0 sin x (0, -cos t, sin t),
 * written at the Yee points of the grid at time t (device outputs). */
int sr_field_standing_wave(float *e[3], float *b[3], const sr_grid *grid, double a0, double t,
                           void *stream);

/* Counting sort of the particles by tile of tile[0] x tile[1] x tile[2] cells
 * (tiles x fastest), for gather locality.  src and dst are two particle sets of
 * the same n (distinct storage); dst receives the permuted particles.  work:
 * device workspace of sr_sort_work(grid, tile, n) bytes.  Order inside a tile
 * is unspecified. */
int sr_sort_particles(const sr_particles_f32 *src, sr_particles_f32 *dst, const sr_grid *grid,
                      const int32_t tile[3], void *work, void *stream);
int64_t sr_sort_work(const sr_grid *grid, const int32_t tile[3], int64_t n);

/* ------------------------------------------------- MLP surrogate (direct sampler)
 * A 2 -> 64 -> 64 -> 64 -> 1 SiLU network mapping (f0, f1) = ((log10 chi + 1)/3,
 * logit(u)/16) to log2 x, x = inverse photon-number CDF at u (with the kinematic cut
 * when trained so).  Parameters: flat [SR_MLP_PARAMS] in the order W1[64][2],
 * b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4; bfloat16 copies
 * are what the kernels read, FP32 masters what Adam updates.  The 64x64 layers
 * run on the matrix cores (bfloat16 in, FP32 accumulate).  Not from the paper:
 * a learned stand-in for the inverse CDF of the spectrum of section "Monte Carlo
 * method", judged against the tables. */
#define SR_MLP_PARAMS 8577
#define SR_MLP_FALLBACK_BINS 24

/* out[i] = network(feats[i]) for M samples; feats device [M][2], out device [M]. */
int sr_mlp_forward(const void *params_bf16, const float *feats, float *out, int64_t M,
                   void *stream);
/* grads = gradient of the energy-weighted squared error
 *   (1/M) sum_i w_i (network(feats[i]) - target[i])^2,  w_i = 2^target[i] / E[x],
 * E[x] = 8/(15 sqrt 3) the mean x of the photon-number spectrum (targets are
 * log2 x, so w_i is the sample's share of the radiated energy), as device FP32
 * [SR_MLP_PARAMS]; work: device FP32 workspace of sr_mlp_grad_work() floats.
 * The sum is taken in a fixed order (reproducible). */
int sr_mlp_mse_grad(const void *params_bf16, const float *feats, const float *target, int64_t M,
                    float *grads, float *work, void *stream);
int64_t sr_mlp_grad_work(void);
/* grads = gradient of sum_i dout[i] * network(feats[i]) with respect to the
 * parameters (the vector-Jacobian product of the backward pass), device FP32
 * [SR_MLP_PARAMS]; dout device [M]; work as for sr_mlp_mse_grad.  Summed in a
 * fixed order (reproducible). */
int sr_mlp_backward(const void *params_bf16, const float *feats, const float *dout, float *grads,
                    int64_t M, float *work, void *stream);
/* `steps` Adam steps (beta 0.9, 0.999, eps 1e-8; step numbers t0+1 ...) on
 * fresh batches of `batch` pairs from sr_mlp_make_batch (seed, batch index
 * t0 + s), minimising the energy-weighted error of sr_mlp_mse_grad, with the
 * learning rate decayed from lr to lr_final on a cosine over the steps.  All
 * launches are enqueued on `stream` by the library (no host round trip per
 * step).  work: device FP32 workspace of sr_mlp_train_work(batch) floats. */
int sr_mlp_train(float *master, void *params_bf16, float *m, float *v, int64_t t0,
                 const sr_table *tab, uint64_t seed, int64_t steps, int64_t batch, float lr,
                 float lr_final, int32_t kin_cut, double log10chi_lo, double log10chi_hi,
                 float *work, void *stream);
int64_t sr_mlp_train_work(int64_t batch);
/* The judge of the surrogate against the table sampler (its fallback map).
 * For each of the SR_MLP_FALLBACK_BINS bins of log10 chi on [-4, 2): chi_per_bin
 * values of chi at the centres of the bin's equal sub-intervals, each with n_u
 * 23-bit midpoints u spread evenly over (0, 1); x from the table sampler
 * (sr_eval_direct, with the kinematic cut if kin_cut) and from the network; the
 * energy-weighted histograms (each sample adds x) over n_xbins log bins of
 * [x_lo, x_hi); err[b] = sum |h_net - h_table| / sum h_table (device FP64
 * [SR_MLP_FALLBACK_BINS]) and fallback[b] = err[b] > tol (device uint8, the map
 * sr_params.mlp_fallback reads).  work: device FP32 workspace of
 * sr_mlp_judge_work(n_u, chi_per_bin, n_xbins) floats. */
int sr_mlp_judge(const void *params_bf16, const sr_table *tab, int32_t kin_cut, int32_t n_u,
                 int32_t chi_per_bin, double x_lo, double x_hi, int32_t n_xbins, double tol,
                 double *err, uint8_t *fallback, float *work, void *stream);
int64_t sr_mlp_judge_work(int32_t n_u, int32_t chi_per_bin, int32_t n_xbins);
/* One Adam step (bias-corrected, step t >= 1) on the FP32 masters, refreshing
 * the bfloat16 copies.  All arrays device [SR_MLP_PARAMS]. */
int sr_mlp_adam(float *master, void *params_bf16, const float *grads, float *m, float *v,
                int64_t t, float lr, float beta1, float beta2, float eps, void *stream);
/* params_bf16 = round(master). */
int sr_mlp_cast(const float *master, void *params_bf16, void *stream);
/* M training pairs from the tables: log10 chi uniform on [lo, hi], u a 23-bit
 * midpoint (Philox, key seed, counter (i, batch, 3)), target log2 x clipped
 * below at -24.  feats device [M][2], target device [M]. */
int sr_mlp_make_batch(const sr_table *tab, uint64_t seed, uint64_t batch, int32_t kin_cut,
                      double log10chi_lo, double log10chi_hi, float *feats, float *target,
                      int64_t M, void *stream);
/* Table-direct sample: x for uniform words a (23-bit midpoints) at chi, the
 * device function of SR_SAMPLER_TABLE.  All arrays device [n]. */
int sr_eval_direct(const sr_table *tab, const uint32_t *a, const float *chi, int32_t kin_cut,
                   float *out_x, int64_t n, void *stream);

/* Human-readable text for a code. */
const char *sr_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* SR_H */
