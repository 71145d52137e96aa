/*
 * mdjk.h -- C ABI of an MI355X (gfx950) library for direct-SCF Coulomb (J) and
 * exchange (K) matrices and the nuclear gradient of the J/K energy, computed
 * from contracted Gaussian electron repulsion integrals over shells up to f
 * (l <= 3) by the McMurchie-Davidson scheme.
 *
 * The operations are the ones stated in arXiv 2406.14920 (Wang et al.,
 * "Extending GPU-accelerated Gaussian integrals in the TeraChem software
 * package to f type orbitals"):
 *   basis functions         section "Cartesian Gaussian basis functions",
 *                           eqs. contracted_basis, primtive_basis
 *   ERIs                    eqs. eri_definition, eri_formula
 *   J (J-engine)            eqs. j_definition, j_formula
 *   K                       eqs. k_definition, k_formula
 *   screening               eq. cauchy_schwarz_bound (pair and quartet level)
 *   energy and gradient     SI eqs. si_E_J_K, si_dE_J, si_dE_K, si_dE_J_step1,
 *                           si_dE_K_step1 (density held fixed)
 *   long-range operator     eqs. eri_longrange_definition, eri_longrange_formula
 *   one-electron integrals  eqs. overlap_formula, kinetic_formula, v1e_formula
 *                           (point charges: nuclei or QM/MM embedding) and SI
 *                           eqs. si_v1e_derivative_A/B/C
 *   density-weighted screen eq. kernel_upperbound (incremental builds)
 *   grid density, XC sums   eqs. xc_density_0, xc_density_1, xc_grid_sum_0,
 *                           xc_grid_sum_1, pair_derivative
 *
 * Conventions
 *   - Units: bohr, hartree.
 *   - Shell coefficients multiply normalised primitives; each contracted
 *     shell is renormalised so that its x^l component has unit norm.
 *   - AO order: shells in the order given to eri_setup.  Inside a shell,
 *     spherical=1 (default): real solid harmonics m = -l..l, except p which is
 *     (x, y, z); spherical=0: Cartesian components in lexicographic order
 *     (xx, xy, xz, yy, yz, zz; xxx, xxy, ... , zzz), all carrying the x^l
 *     normalisation.
 *   - Matrices are nbf x nbf, row-major, FP64, in DEVICE memory (for example
 *     the data_ptr() of a torch tensor on the GPU).
 *   - P is read as given and used as (P + P^T)/2.  J and K are returned
 *     symmetric.  E = 1/2 tr(PJ) - 1/4 tr(PK).
 *   - Screening is part of the result's definition: a shell quartet (ab|cd)
 *     enters iff Q_ab * Q_cd >= schwarz_thresh with
 *     Q_ab = sqrt(max over Cartesian components of |(ab|ab)|); inside it a
 *     primitive quartet enters iff q_ij * q_kl >= prim_thresh, q_ij being the
 *     same bound for one primitive pair (with its coefficients).
 *
 * Calls are stream-ordered and asynchronous on opts.stream (a hipStream_t;
 * NULL = the default stream) unless stated otherwise.  The library owns every
 * device buffer it allocates (released by eri_destroy); it never keeps caller
 * pointers after a call returns.  A context is not thread-safe; distinct
 * contexts may be used from distinct threads on distinct streams.
 *
 * Errors: every call returns 0 on success or a negative ERI_E* code; the
 * message of the last failure on the calling thread is in eri_last_error().
 */
#ifndef MDJK_H
#define MDJK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ERI_OK      0
#define ERI_EINVAL (-1) /* bad argument: null pointer, l outside 0..3, nprim < 1,
                           exponent <= 0 or not finite, atom index out of range,
                           negative threshold, unknown precision */
#define ERI_ENOMEM (-2) /* device or host allocation failed, or the library's device
                           buffers would pass the byte cap that the environment
                           variable ERI_MAX_DEVICE_BYTES sets (read at every
                           allocation; unset or 0: no cap).  A failed call leaves
                           no half-built context; a context stays usable. */
#define ERI_EHIP   (-3) /* HIP runtime error; the message carries hipGetErrorString */
#define ERI_ESTATE (-4) /* null/destroyed context or an inconsistent request */

#define ERI_FP64      0
#define ERI_MIXED     1  /* single-precision share where it pays (per launch; see eri_autotune) */
#define ERI_MIXED_ALL 2  /* the paper's rule on every launch: FP32 below the threshold everywhere */

typedef struct eri_ctx eri_ctx;

typedef struct {
    double xyz[3]; /* bohr */
} eri_atom;

typedef struct {
    int32_t atom;        /* index into the atoms array */
    int32_t l;           /* 0..3 */
    int32_t nprim;       /* >= 1 */
    const double *exps;  /* [nprim], > 0 (host memory, copied by eri_setup) */
    const double *coefs; /* [nprim], coefficients of normalised primitives */
} eri_shell;

typedef struct {
    double schwarz_thresh; /* shell-quartet threshold tau_S (>= 0) */
    double prim_thresh;    /* primitive-quartet threshold (>= 0); 0 keeps every
                              primitive of a kept shell quartet */
    double mixed_thresh;   /* mixed modes: a wavefront tile whose quartets all have
                              density-weighted bounds Q_ab*Q_cd*max|P_blk| below this
                              runs its primitive integrals in FP32 (>= 0) */
    int32_t precision;     /* ERI_FP64, ERI_MIXED or ERI_MIXED_ALL.  In ERI_MIXED a
                              launch takes the FP32 share only where that is faster:
                              by default the exchange classes with la+lb+lc+ld >= 5;
                              the J-engine stays FP64 (its FP32 share is dominated by
                              the FP64 Boys values and conversions); eri_autotune
                              re-decides per launch from timings.  Boys values,
                              bounds, digestion and accumulation are FP64 always. */
    int32_t spherical;     /* 1: real solid harmonics (default); 0: Cartesian */
    void *stream;          /* hipStream_t, NULL = default stream */
    double omega;          /* two-electron operator: 0 (default) the Coulomb 1/r;
                              > 0 the long-range erf(omega r)/r of eqs.
                              eri_longrange_definition / eri_longrange_formula
                              (J, K, energy and gradient).  Screening always uses
                              the 1/r bounds, which bound the long-range
                              integrals too. */
} eri_opts;

typedef struct {
    int32_t nshell, natom, nbf, nbf_cart;
    int64_t n_pairs;             /* contracted shell pairs kept (Q_ab > 0) */
    int64_t n_prim_pairs;        /* primitive pairs stored */
    int64_t n_quartets;          /* unique shell quartets passing the Schwarz rule */
    int64_t n_quartets_fp32;     /* of which run in FP32 (mixed modes, last build_jk) */
    double  eris_sph;            /* sum over kept unique quartets of prod (2l+1) */
    double  eris_cart;           /* same with Cartesian component counts */
    double  model_flops_k;       /* model FLOPs of one K build (unique quartets) */
    double  model_flops_j;       /* model FLOPs of one J build (J-engine) */
    double  last_ms;             /* device time of the last build_jk / jk_grad (ms) */
    int64_t n_prim_quartets_k;   /* primitive quartets one K build evaluates (after the
                                    primitive screen; unique quartets) */
    int64_t n_prim_quartets_j;   /* (bra, ket) primitive pairs one J-engine build evaluates */
} eri_stats_t;

/* Device time of one kernel family, accumulated while profiling is on. */
typedef struct {
    char    name[40];       /* kernel and class, e.g. "k_wave(31|10)", "jeng_small(4,2)" */
    int32_t launches;       /* launches accumulated */
    double  ms;             /* summed device time (HIP events recorded on the launch stream) */
    double  flops;          /* algorithmic FLOPs of one launch (fixed FLOP model per primitive quartet) */
    int64_t prim_quartets;  /* primitive quartets one launch evaluates (0 if not applicable) */
} eri_kernel_time;

/* Fill opts with defaults: schwarz 1e-11, prim 1e-2*schwarz, mixed 1e-5,
 * FP64, spherical, default stream, Coulomb operator (omega 0). */
void eri_default_opts(eri_opts *opts);

/* Build a context: normalise shells, form contracted and primitive shell pairs
 * (eq. pair_definition), compute Schwarz factors on the GPU, sort and bin the
 * pairs into the ten angular classes and allocate every device buffer later
 * calls need.  shells/atoms are host arrays, copied.  Synchronous.
 * On failure *out is set to NULL. */
int eri_setup(const eri_shell *shells, int32_t nshell, const eri_atom *atoms, int32_t natom,
              const eri_opts *opts, eri_ctx **out);

/* Number of basis functions (spherical or Cartesian, per opts.spherical). */
int eri_nbf(const eri_ctx *ctx, int32_t *nbf);

/* Move the atoms (same shells) and redo the pair/Schwarz setup.  Synchronous. */
int eri_set_geometry(eri_ctx *ctx, const eri_atom *atoms);

/* Change the precision mode (ERI_FP64 / ERI_MIXED / ERI_MIXED_ALL) and the
 * mixed threshold. */
int eri_set_precision(eri_ctx *ctx, int32_t precision, double mixed_thresh);

/* Switch the two-electron operator of later calls: omega = 0 for 1/r, > 0 for
 * erf(omega r)/r (eq. eri_longrange_formula); the pairs and screening bounds
 * are unchanged. */
int eri_set_omega(eri_ctx *ctx, double omega);

/* J_mn = sum_ls (mn|ls) P_ls (J-engine, eq. j_formula) and
 * K_ml = sum_ns (mn|ls) P_ns (eq. k_formula).  P, J, K: device, nbf*nbf
 * row-major FP64.  J or K may be NULL to skip it.  Asynchronous. */
int build_jk(eri_ctx *ctx, const double *P, double *J, double *K);

/* Density-weighted screen of later build_jk / build_jk_static calls (the
 * paper's density-weighted Schwarz bound, eq. kernel_upperbound and section
 * "Performance"): K skips a contracted quartet whose Q_ab Q_cd times the
 * largest |P| over the four Cartesian density blocks its digestion reads is
 * below tau; J skips a (bra wavefront, ket pair) tile whose largest Q_ab
 * times Q_cd max|P_cd| is below tau.  Each skipped term is bounded by its
 * bound, so incremental builds on a density change dP (J(P + dP) =
 * J(P) + J(dP)) skip most of the work as dP shrinks.  tau = 0 (default) turns
 * it off.  Gradients and potentials ignore it. */
int eri_set_density_screen(eri_ctx *ctx, double tau);

/* Overlap S_mn (eqs. overlap_definition, overlap_formula) and kinetic energy
 * T_mn (eqs. kinetic_definition, kinetic_formula) of the context's basis:
 * one workgroup per contracted shell pair, a thread per Cartesian component,
 * the pair's E coefficients with the ket index raised by two in LDS.  Pairs
 * that fail the Schwarz rule against every pair are absent, as in build_jk.
 * S, T: device nbf*nbf row-major, overwritten; either may be NULL, not both.
 * Asynchronous. */
int eri_one_electron(eri_ctx *ctx, double *S, double *T);

/* Electron density and its gradient at grid points (eqs. xc_density_0,
 * xc_density_1, with the pair derivative of eq. pair_derivative):
 * rho(r) = sum_mn P_mn m(r) n(r).  One lane per point; the contracted pairs
 * are walked per 64-point block, skipping every pair whose bounding sphere
 * (all points where one of its primitives has p |r - P|^2 <= 100) misses the
 * block's sphere, and inside a pair every such primitive.  Points should be
 * ordered so that consecutive points lie close together (atom by atom, shell
 * by shell), which keeps the block spheres small.  Deterministic.
 * P: device nbf*nbf, symmetric.  pts: device [npts][3] (bohr).  rho: device
 * [npts], overwritten; grad: device [npts][3] or NULL, overwritten.
 * npts = 0 is a no-op (pts, rho may then be NULL).  Asynchronous. */
int eri_grid_density(eri_ctx *ctx, const double *P, const double *pts, int64_t npts, double *rho, double *grad);

/* Grid sums of the exchange-correlation matrix (eqs. xc_grid_sum_0,
 * xc_grid_sum_1): V_mn = sum_g v0_g m(r_g) n(r_g) + sum_g v1_g . grad(m n)(r_g),
 * the quadrature weights folded into v0 and v1 by the caller (v0 = w de/drho,
 * v1 = w de/d(grad rho) of the functional, evaluated outside the library as
 * in the paper).  One wavefront per contracted pair over the point blocks
 * whose spheres meet the pair's (same cut-off as eri_grid_density), sums
 * reduced in a fixed order: deterministic.  pts: device [npts][3]; v0: device
 * [npts]; v1: device [npts][3] or NULL (no gradient term); V: device nbf*nbf,
 * overwritten (V = 0 for npts = 0).  Asynchronous. */
int eri_grid_matrix(eri_ctx *ctx, const double *pts, int64_t npts, const double *v0, const double *v1, double *V);

/* build_jk for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same double-precision J and K as build_jk, with the per-build work buffers
 * (Cartesian density and accumulators, Hermite density and Hermite J) taken
 * from a static device array of 64 MiB per GPU instead of the context's own
 * buffers; the call allocates nothing.  Needs 8*(3*nbf_cart^2 + 2*H) bytes,
 * H = sum over primitive pairs of the Hermite index count (rounded up to 256
 * bytes per region); a larger context is rejected with ERI_EINVAL.  Only the
 * double-precision path (ERI_FP64; otherwise ERI_ESTATE).  Every call on a
 * GPU shares that GPU's array and leaves its contents behind (each call
 * clears what it accumulates into), so calls that overlap on one GPU -- on
 * different streams or host threads -- race and must be serialised by the
 * caller.  P, J, K as for build_jk.  Asynchronous. */
int build_jk_static(eri_ctx *ctx, const double *P, double *J, double *K);

/* Nuclear gradient dE/dR of E = 1/2 tr(PJ) - 1/4 tr(PK) at fixed P
 * (SI eqs. si_E_J_K, si_dE_J, si_dE_K; the density-derivative terms are
 * absent), in hartree/bohr, atoms in the order given to eri_setup.
 * Coulomb part: the J-engine with the bra Hermite order raised by one and the
 * pair derivative of SI eq. si_pair_derivative (SI eq. si_dj_formula);
 * exchange part: derivative integrals of every canonical quartet on all four
 * centres (the fourth by translational invariance).  Same screening as
 * build_jk.  Precision: under ERI_MIXED_ALL (and where the autotuner chose
 * an FP32 share of a J-engine launch under ERI_MIXED) the Coulomb part's
 * J-engine launches of raised bra order <= 6 take the FP32 share by the same
 * density-weighted tile rule as build_jk, accumulated in FP64; the exchange
 * part, the pair-derivative contraction and every sum are FP64 (FP32 vector
 * arithmetic has no rate advantage over FP64 on this target).  Per-atom sums
 * are formed in a fixed order, so repeated calls give identical results.
 * P: device nbf*nbf.  grad: device [natom*3] or NULL; E: device [1] or NULL
 * (then a double-precision J and K build is done first); not both NULL.
 * Asynchronous. */
int jk_grad(eri_ctx *ctx, const double *P, double *grad, double *E);

/* Point-charge potential matrix V_mn = sum_C q_C int m(r) n(r) / |r - C|
 * (eqs. v1e_definition, v1e_summation_over_C; nuclear attraction with
 * q_C = -Z_C, or embedding charges of a QM/MM calculation), by eq.
 * v1e_formula: per primitive pair the Hermite potential
 * K_ab (2 pi/p) sum_C q_C R^0_t(p, P - C) (one lane per primitive pair, all
 * charges), then the pair's E coefficients.  Always the 1/r operator and
 * double precision, whatever eri_set_omega / eri_set_precision chose; no
 * primitive cut-off; the shell pairs are those the context keeps (pairs that
 * fail the Schwarz rule against every pair are absent, as in build_jk).
 * charges: device [ncharge][4] = x, y, z (bohr), q; ncharge >= 0 (0 gives
 * V = 0).  V: device nbf*nbf row-major, overwritten.  Asynchronous; the
 * context's work buffers are shared with build_jk on the same stream. */
int eri_potential(eri_ctx *ctx, const double *charges, int32_t ncharge, double *V);

/* Derivatives of E_V = sum_mn P_mn V_mn at fixed P (SI eqs.
 * si_v1e_derivative_A, si_v1e_derivative_B, si_v1e_derivative_C): with
 * respect to the atoms that carry the basis functions (the pair derivative of
 * SI eq. si_pair_derivative with the Hermite potential of order la+lb+1) and
 * to the charge positions (-q_C sum_t Dh_t R^0_{t+1_k}, Dh the pair's Hermite
 * density).  A nucleus that carries basis functions and a charge gets both
 * terms: the caller adds gatom[A] and gchg[C] for it.  Sums are formed in a
 * fixed order: repeated calls give identical results.
 * P: device nbf*nbf, symmetric.  gatom: device [natom*3] or NULL; gchg:
 * device [ncharge*3] or NULL; both overwritten.  Asynchronous. */
int eri_potential_grad(eri_ctx *ctx, const double *charges, int32_t ncharge, const double *P,
                       double *gatom, double *gchg);

/* E = 1/2 sum_ij P_ij J_ij - 1/4 sum_ij P_ij K_ij (SI eq. si_E_J_K) from
 * device P, J, K (nbf*nbf) into device E[1]; fixed-order reduction.
 * Asynchronous. */
int eri_energy(eri_ctx *ctx, const double *P, const double *J, const double *K, double *E);

/* Profiling: while on, every kernel launch of later calls is bracketed by HIP
 * events on the launch stream and build_jk runs all its launches on the
 * context stream (no concurrent J / exchange streams), so each pair of events
 * brackets one kernel alone; eri_profile_read synchronises, reports the
 * accumulated per-kernel times (up to cap entries, *n set to the count) and
 * clears them. */
int eri_set_profiling(eri_ctx *ctx, int32_t on);
int eri_profile_read(eri_ctx *ctx, eri_kernel_time *out, int32_t cap, int32_t *n);

/* Counters of the context (host struct).  Synchronises the stream. */
int eri_stats(const eri_ctx *ctx, eri_stats_t *out);

/* Release the context and all its device memory.  NULL is accepted. */
int eri_destroy(eri_ctx *ctx);

/* Autotuner: times the candidate launch shapes (J-engine ket chunk per class
 * pair; workgroup cap of each range-walking exchange launch; the ket
 * grouping of each lane-per-quartet exchange launch -- by the first ket
 * shell c or by the second shell d, the latter being the ordering the paper
 * calls inverted (section "Performance", closing remarks on the K
 * algorithm), chosen per angular class; under ERI_MIXED
 * also whether each launch takes the FP32 share at all) on this
 * context's own workload -- device density P, current precision -- best of
 * reps runs each, and keeps the fastest for later builds.  Replaces the
 * paper's fixed rule for splitting work between kernels.  Synchronous;
 * leaves J/K results unchanged except for the order of atomic additions
 * (under ERI_MIXED, launches moved between FP32 and FP64 change results
 * within the mixed-precision error). */
int eri_autotune(eri_ctx *ctx, const double *P, int32_t reps);

/* The launch shapes in use: kchunk100[10*X + Y] (may be NULL), the first
 * cap_len exchange caps into kcap (may be NULL; 0 = default), *n_kcap = the
 * number of exchange launches (may be NULL). */
int eri_tuning(const eri_ctx *ctx, int32_t *kchunk100, int32_t *kcap, int32_t cap_len, int32_t *n_kcap);

/* The launch shapes and precision splits in use, keyed by angular class so
 * that they can be saved and applied to a context of a similar workload.
 * kchunk/jsplit[10*X + Y]: J-engine ket chunk and FP32-share flag of bra
 * class X, ket class Y (classes ss, ps, pp, ds, dp, dd, fs, fp, fd, ff);
 * launch i < n_kwork of the exchange: class pair kwork_class[i] = 10*X + Y
 * (X >= Y), workgroup cap kcap[i] (0 = default), FP32-share flag ksplit[i]
 * and ket grouping kinv[i] (0: by the first ket shell, whose exchange targets
 * K_ac, K_bc the items of a row share; 1: by the second, sharing K_ad, K_bd;
 * only lane-per-quartet launches take 1, others keep 0). */
typedef struct {
    int32_t kchunk[100];
    int32_t jsplit[100];
    int32_t n_kwork;
    int32_t kwork_class[64];
    int32_t kcap[64];
    int32_t ksplit[64];
    int32_t kinv[64];
} eri_tuning_t;

/* Read the current choice (eri_get_tuning) or apply a saved one
 * (eri_set_tuning: entries are matched by class; chunks outside 8..1024 or
 * negative caps are rejected with ERI_EINVAL).  Results change only in the
 * order of floating-point additions, and under ERI_MIXED within the mixed
 * error where a launch moves between FP32 and FP64. */
int eri_get_tuning(const eri_ctx *ctx, eri_tuning_t *out);
int eri_set_tuning(eri_ctx *ctx, const eri_tuning_t *in);

/* Batches of independent molecules (many contexts, uneven sizes).
 * eri_batch_create: n >= 1 contexts on the current device, each keeping its
 * own basis, thresholds and precision; stream = hipStream_t the batch runs
 * on (NULL: the default stream).  The batch's own streams fork from that
 * stream at the start of each call and are joined back into it at the end, so
 * a call is ordered after the work queued before it on that stream and
 * before the work queued after it.  The contexts stay owned by the caller and
 * must outlive the batch.
 * eri_batch_build_jk: P, J, K are host arrays of n device pointers
 * (nbf_i x nbf_i each, as in build_jk; none NULL).  Results equal those of
 * build_jk on each context (up to the order of floating-point atomic
 * additions).  Asynchronous on the batch stream.  Two ways to run it
 * (eri_batch_set_mode):
 *  - ERI_BATCH_QUEUE (the default): the J-engine and exchange work of all
 *    molecules runs as ONE launch per kernel (angular class and arithmetic
 *    type; under ERI_MIXED* a class's double- and single-precision shares
 *    are two kernels, as in build_jk):
 *    the blocks every molecule's own launch would have had become the items
 *    of a device-side work list, the launches with the most work per block
 *    first, and workgroup b runs item b, so the hardware dispatcher hands
 *    the long items out first and fills the tail with the short ones (the
 *    paper's kernels are one launch per class and molecule, section
 *    "Implementation").  The plan
 *    (argument tables and item lists, on the device) is made on the first
 *    call and again after any context changes (precision, geometry, screen,
 *    tuning): that call allocates and copies; later calls launch kernels
 *    only (on the batch stream and on streams forked from it and joined
 *    back, as in build_jk), so a call after the first can be captured into
 *    a HIP graph.
 *  - ERI_BATCH_STREAMS: every molecule's build_jk is forked from the batch
 *    stream onto one of up to 8 batch streams and joined back, so molecules
 *    run concurrently.
 * (The library also holds a path that records the streams form into one HIP
 * graph itself; it is switched off in this library after host-side crashes of
 * that recording on the MI355X runtime.) */
typedef struct eri_batch eri_batch;
int eri_batch_create(eri_ctx *const *ctxs, int32_t n, void *stream, eri_batch **out);
int eri_batch_build_jk(eri_batch *b, const double *const *P, double *const *J, double *const *K);
#define ERI_BATCH_QUEUE   0
#define ERI_BATCH_STREAMS 1
/* Select how eri_batch_build_jk runs (ERI_EINVAL for another value). */
int eri_batch_set_mode(eri_batch *b, int32_t mode);
/* Launches per queue build and the items (blocks) they run in total, of the
 * current plan.  ERI_ESTATE before the first queue build. */
int eri_batch_queue_info(eri_batch *b, int32_t *launches, int64_t *items);
/* Per-molecule latency of the last eri_batch_build_jk: ms[i] = device time
 * from the start of that call on the batch stream to the end of molecule i's
 * build (HIP events on its batch stream), for the first n molecules.
 * Molecules are issued largest first (by the spherical ERIs of their unique
 * quartets), in the streams mode each onto the least-loaded of the batch
 * streams; in the queue mode every molecule finishes after the shared
 * batch launches, with its output transforms.  Synchronises with those
 * events.  ERI_ESTATE before the first batch build. */
int eri_batch_latency(eri_batch *b, float *ms, int32_t n);

int eri_batch_destroy(eri_batch *b);

/* Message of the last error on this thread ("" if none). */
const char *eri_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MDJK_H */
