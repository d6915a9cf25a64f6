/*
 * sfq.h -- C ABI of the MI355X strong-field QED Monte Carlo step.
 *
 * Method: Montefiori & Tamburini, "SFQEDtoolkit: a high-performance library for the accurate
 * modeling of strong-field QED processes in PIC and Monte Carlo codes", arXiv:2301.07684.
 * The calls follow the paper's App. A (user guide) in batched, device-pointer form.
 *
 * Conventions for every call below
 *   - Units are the paper's normalised units (Sec. 4.1 and App. A): energies gamma = eps/(m c^2),
 *     momenta in m c, fields E and B in m c omega_r/|e|, rates in omega_r, times in 1/omega_r.
 *   - Every array argument is a DEVICE pointer (hipMalloc'd or from a framework allocator) of
 *     the documented length; arrays are structure-of-arrays (one pointer per component).  The
 *     library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls are asynchronous:
 *     they validate their arguments, enqueue kernels on `stream` and return.  Results are valid
 *     after the stream has been synchronised.
 *   - n == 0 is a no-op returning SFQ_OK.
 *   - Errors: argument errors are reported synchronously as a non-zero sfq_status with a message
 *     available from sfq_last_error(); nothing is enqueued in that case.  Conditions found on
 *     the device (product-buffer overflow, chi beyond the tables) are reported in the
 *     sfq_counters structure of sfq_step.  No C++ exception crosses this interface.
 *   - A handle may be used from several host threads and streams at once.  sfq_step calls on
 *     different streams share the handle's emitter queue: the library orders them on the
 *     device (a step waits for the previous step of the handle when it was enqueued on another
 *     stream), so they are correct but do not overlap; use one handle per stream for
 *     concurrency.
 *   - sfq_step is not captured into graphs: on a stream that is capturing it returns
 *     SFQ_E_STATE and enqueues nothing (a graph would keep pointers to scratch memory the handle
 *     reuses).  Graphs of steps come from plans (sfq_plan_capture), which own theirs.
 */
#ifndef SFQ_H
#define SFQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfq_ctx* sfq_handle;

typedef enum {
    SFQ_OK = 0,
    SFQ_E_ARG = 1,      /* invalid argument (NULL pointer, bad enum, inconsistent config)      */
    SFQ_E_STATE = 2,    /* invalid handle, or a call not allowed in this state (sfq_step on a
                           capturing stream)                                                     */
    SFQ_E_NOMEM = 3,    /* device allocation failed                                              */
    SFQ_E_CAPACITY = 4, /* request exceeds a fixed limit of the library                          */
    SFQ_E_DEVICE = 5,   /* HIP runtime error                                                     */
    SFQ_E_TABLES = 6    /* approximation table file missing, corrupt or of another geometry      */
} sfq_status;

typedef enum { SFQ_ELECTRON = 0, SFQ_POSITRON = 1, SFQ_PHOTON = 2 } sfq_species;

/* FP64: everything in double precision.  MIXED: chi, optical depths and the inverse-CDF tails
 * with energy fraction above 0.999 in FP64; approximation evaluation and sampling in FP32. */
typedef enum { SFQ_FP64 = 0, SFQ_MIXED = 1 } sfq_precision;

/* Paper Sec. 2: optical-depth method (Eq. (any_event)) or local method (R dt > r). */
typedef enum { SFQ_OPTICAL_DEPTH = 0, SFQ_LOCAL = 1 } sfq_decision;

/* How a tile gives the fields at its particles (sfq_tile.field_mode).  ARRAYS: ex..bz are
 * arrays of n.  UNIFORM: ex..bz each point to ONE double, the field of every particle of the
 * tile (a constant, uniform external field such as the paper's Sec. 4.3 validation set-up).
 * PLANE_WAVE: the step computes the fields of a linearly polarised plane wave,
 * E = a_i cos(phi_i + theta) e, B = k x E, from the tile's wave_* members (ex..bz unused):
 * the field traffic is that of a_i and phi_i (16 B per particle instead of 48). */
typedef enum { SFQ_FIELDS_ARRAYS = 0, SFQ_FIELDS_UNIFORM = 1, SFQ_FIELDS_PLANE_WAVE = 2 } sfq_field_mode;

/* Evaluation form of the approximation tables (sfq_config.approx), the accuracy/speed dial in
 * the spirit of the paper's choice of coefficient counts (Sec. 4.5): FULL evaluates all 16
 * Chebyshev terms of each rate segment and all 8 x 8 coefficients of each inverse-CDF patch;
 * TRUNCATED only the leading 10 terms and 5 x 5 coefficients of the same tables (less work,
 * less accuracy).  The table generator measures each form's error (its report, data/
 * sfq_tables_report.json, "forms"). */
typedef enum { SFQ_APPROX_FULL = 0, SFQ_APPROX_TRUNCATED = 1 } sfq_approx;

/* Philox draw purposes (counter word 3).  See sfq_philox. */
enum { SFQ_P_INIT = 0, SFQ_P_EMIT = 1, SFQ_P_CHILD = 2, SFQ_P_CHILD2 = 3, SFQ_P_LOCAL = 4 };

typedef struct {
    double ref_omega;        /* reference angular frequency omega_r in rad/s (App. A function 2) */
    double ref_length;       /* reference length lambda_r = c/omega_r in m (App. A function 1);
                                exactly one of ref_omega and ref_length must be > 0             */
    double dt;               /* time step in units of 1/omega_r (App. A functions 1-2, "ts")    */
    int32_t precision;       /* sfq_precision                                                     */
    int32_t decision;        /* sfq_decision used by sfq_step                                     */
    int32_t blcfa;           /* 1: leptons use the beyond-LCFA emission of Sec. 5 in sfq_step;
                                requires decision == SFQ_LOCAL (Sec. 2, App. A)                   */
    int32_t bw_fast;         /* 1: pair rate is zero for chi < 0.3 (App. A function 7)           */
    int32_t device;          /* HIP device ordinal the handle's tables live on                   */
    int32_t approx;          /* sfq_approx: full or truncated evaluation of the tables           */
    const char* tables_path; /* approximation table file; NULL = data/sfq_tables.bin next to
                                the shared library                                                */
} sfq_config;

/* Initialisation (paper App. A functions 1 and 2, SFQED_INIT_ALL_ref_len / _ref_freq): loads
 * the approximation tables into device memory of cfg->device.  On success *out receives a new
 * handle and SFQ_OK is returned (the paper's `true`). */
sfq_status sfq_create(const sfq_config* cfg, sfq_handle* out);

/* Teardown (paper App. A function 14, SFQED_FINALIZE_ALL): frees the handle's device memory.
 * The caller must have synchronised every stream that used the handle.  NULL is ignored. */
void sfq_destroy(sfq_handle h);

/* Message of the last error on this host thread (h may be NULL); never NULL. */
const char* sfq_last_error(sfq_handle h);

/* Derived constants of a handle: lambda_C/lambda_r and lambda_r/lambda_C (dimensionless). */
sfq_status sfq_units(sfq_handle h, double* lc_over_lr, double* lr_over_lc);

/* Quantum parameter chi (paper Eq. (chi_exact); App. A functions 15-16) and energy gamma
 * (sqrt(1+p^2) for leptons, |p| for photons) of n particles of one species.  Inputs: momentum
 * and local fields (n doubles each).  Outputs: gamma_out (nullable), chi_out (n doubles). */
sfq_status sfq_chi(sfq_handle h, int species, size_t n, const double* px, const double* py,
                   const double* pz, const double* ex, const double* ey, const double* ez,
                   const double* bx, const double* by, const double* bz, double* gamma_out,
                   double* chi_out, void* stream);

/* LCFA rates W = R/omega_r (paper Eqs. (pe_rate_3) and (pp_tot_real); App. A functions 5-7):
 * species SFQ_ELECTRON or SFQ_POSITRON -> nonlinear Compton rate; SFQ_PHOTON -> nonlinear
 * Breit-Wheeler rate, zero for chi < 0.01 (Sec. 4.2) or chi < 0.3 with bw_fast.  Inputs gamma,
 * chi (n doubles each, gamma > 0, chi >= 0); output rate_out (n doubles). */
sfq_status sfq_rates(sfq_handle h, int species, size_t n, const double* gamma, const double* chi,
                     double* rate_out, void* stream);

/* LCFA photon energy (paper Sec. 4.3, Eq. (again); App. A function 9): for emitter energy gamma,
 * quantum parameter chi and uniform r in (0,1), gamma_photon_out receives the emitted photon
 * energy.  gamma_emitter_out (nullable) receives the emitter's energy after collinear recoil,
 * gamma - gamma_photon, computed without cancellation.  n doubles each. */
sfq_status sfq_sample_photon(sfq_handle h, size_t n, const double* gamma, const double* chi,
                             const double* r, double* gamma_photon_out, double* gamma_emitter_out,
                             void* stream);

/* Pair energies (paper Sec. 4.4, Eqs. (again_pp), (return_to_nrg); App. A function 11): for a
 * photon of energy gamma and quantum parameter chi (tabulated for chi >= 2^-7) and uniform r in
 * (0,1), gamma_electron_out receives the electron energy; gamma_positron_out (nullable) the
 * positron energy gamma - gamma_electron, computed without cancellation.  n doubles each. */
sfq_status sfq_sample_pair(sfq_handle h, size_t n, const double* gamma, const double* chi,
                           const double* r, double* gamma_electron_out,
                           double* gamma_positron_out, void* stream);

/* Philox4x32-10 draws (Salmon et al., SC'11) with key (seed mod 2^32, seed >> 32) and counter
 * (uid mod 2^32, uid >> 32, step mod 2^32, purpose).  a_out and b_out (n uint64 each) receive
 * the words x0:x1 and x2:x3.  The uniform used by the step is ((a >> 12) + 1/2) 2^-52. */
sfq_status sfq_philox(sfq_handle h, size_t n, const uint64_t* uid, uint64_t seed, uint64_t step,
                      uint32_t purpose, uint64_t* a_out, uint64_t* b_out, void* stream);

/* Initial optical depths tau_0 = -ln(1 - r) (paper Sec. 2, text after Eq. (any_event)) with r
 * from purpose SFQ_P_INIT at step 0.  tau_out: n doubles. */
sfq_status sfq_init_optical_depth(sfq_handle h, size_t n, const uint64_t* uid, uint64_t seed,
                                  double* tau_out, void* stream);

/* One tile of particles of one species for sfq_step.  All pointers are device pointers of n
 * elements unless stated. */
typedef struct {
    int32_t species;           /* sfq_species                                                     */
    int32_t product_set;       /* with desc->nsets > 0: index of the sfq_product_set receiving
                                  this tile's products; otherwise must be 0                       */
    uint64_t n;                /* number of particles                                             */
    double *px, *py, *pz;      /* momentum, updated in place by recoil.  With blcfa leptons this
                                  is the pushed momentum p_L^{(n+1/2)} of Sec. 5, or, with
                                  desc->push, p^{(n-1/2)} (the step pushes it)                    */
    const double *ex, *ey, *ez;/* electric field at the particle (blcfa leptons: only with push);
                                  see field_mode                                                  */
    const double *bx, *by, *bz;/* magnetic field at the particle (as E)                           */
    double* tau;               /* remaining optical depth tau_d (OPTICAL_DEPTH; else nullable).
                                  After the step: the decremented depth, a fresh one for a lepton
                                  that emitted; a photon that converted keeps its decremented
                                  (negative) depth                                                */
    const uint64_t* uid;       /* particle identifiers: the Philox counter of every draw          */
    uint8_t* alive;            /* nullable (all alive).  Converted photons are set to 0.  Dead
                                  particles are not processed; the step may rewrite their tau and
                                  momentum slots with the values they hold                       */
    /* beyond-LCFA state (blcfa handles, lepton tiles; else NULL): the momentum before the push
     * p^{(n-1/2)} (not read, and may be NULL, with desc->push), the stored transverse Lorentz
     * force F_perp^{(n-1)} and its last difference (3n doubles each, component-major:
     * x[0..n), y[0..n), z[0..n)), and the just-created flag                                    */
    const double *px_prev, *py_prev, *pz_prev;
    double* fperp;
    double* dfperp;
    uint8_t* just_created;
    double* chi_out;           /* nullable: chi of every alive particle                          */
    double* rate_out;          /* nullable: rate W of every alive particle                       */
    uint64_t step_offset;      /* this tile's draws use step index desc->step + step_offset
                                  (mod 2^32): lets one launch advance tiles that are at different
                                  steps of their own simulations                                  */
    int32_t field_mode;        /* sfq_field_mode                                                  */
    int32_t reserved3;         /* 0                                                               */
    const double* wave_amp;    /* PLANE_WAVE: amplitude a_i at each particle (n doubles, in
                                  m c omega_r / e)                                                */
    const double* wave_phase;  /* PLANE_WAVE: phase phi_i at each particle (n doubles, radians);
                                  |phi_i + wave_phase0| must stay below 2^20 pi/2 (about 1.6e6),
                                  the range of the step's cosine argument reduction             */
    double wave_k[3];          /* PLANE_WAVE: unit propagation direction k                        */
    double wave_pol[3];        /* PLANE_WAVE: unit polarisation e, perpendicular to k             */
    double wave_phase0;        /* PLANE_WAVE: theta, added to every phase (omega t of the step)  */
} sfq_tile;

/* Product buffers of one species (device SoA arrays of `capacity` elements). */
typedef struct {
    double *px, *py, *pz, *tau;
    uint64_t *uid, *parent;
    uint64_t capacity;
} sfq_products;

/* Device counters, accumulated by sfq_step (the caller zeroes them when it wants). */
typedef struct {
    unsigned long long processed;       /* alive particles taken through the step                */
    unsigned long long emitted;         /* Compton emissions kept                                */
    unsigned long long converted;       /* photons converted to pairs                            */
    unsigned long long blcfa_rejected;  /* beyond-LCFA candidates rejected by Eq. (rej_cond)     */
    unsigned long long out_of_domain;   /* chi above the tables (2^16): asymptotic forms used    */
    unsigned long long clamped;         /* leptons left with gamma <= 1 and put at rest          */
    unsigned long long overflow;        /* products that did not fit their buffer                */
    unsigned long long deferred;        /* particles whose step the deferred-share pass did (the
                                           emitter queue was too small for their share of a
                                           chunk; results are the same, only slower)            */
} sfq_counters;

/* Product buffers and their append counters, one set per owner (e.g. per simulation when one
 * step serves several): lets a single launch write every tile's products into its owner's own
 * buffers. */
typedef struct {
    sfq_products photons, electrons, positrons;
    unsigned long long* product_counts; /* device [3], as sfq_step_desc.product_counts          */
} sfq_product_set;

typedef struct {
    uint64_t seed;             /* Philox key                                                      */
    uint64_t step;             /* step index: Philox counter word 2 (mod 2^32), plus each tile's
                                  step_offset                                                     */
    int32_t ntiles;            /* 1 .. SFQ_MAX_TILES                                              */
    int32_t nsets;             /* 0: products go to the buffers below; 1 .. SFQ_MAX_TILES: each
                                  tile's products go to product_sets[tile.product_set] and the
                                  buffers and counts below are ignored                           */
    const sfq_tile* tiles;     /* HOST array of ntiles tile descriptors                           */
    sfq_products photons;      /* Compton photons                                                 */
    sfq_products electrons;    /* Breit-Wheeler electrons                                         */
    sfq_products positrons;    /* Breit-Wheeler positrons                                         */
    unsigned long long* product_counts; /* device [3]: photons, electrons, positrons already in
                                  the buffers; products are appended there and the counts grow
                                  (beyond capacity too: the final count is the size needed)      */
    sfq_counters* counters;    /* device, accumulated                                             */
    const sfq_product_set* product_sets; /* HOST array of nsets sets (copied by the call)         */
    int32_t push;              /* 1: before the QED step, every alive lepton's momentum gets the
                                  Boris push through its tile's E and B over one time step dt
                                  (charge -1 for electrons, +1 for positrons; time in 1/omega_r,
                                  fields in m c omega_r / e, the units of the QED step), and the
                                  step then works on the pushed momentum, which is what the tile
                                  holds afterwards.  Photons are not pushed.  This is the particle
                                  update of the PIC cycle fused with the QED step (paper Fig. 7),
                                  for callers whose fields are already at the particles.  With
                                  beyond-LCFA handles the tile's momentum is p^{(n-1/2)} and the
                                  push supplies p^{(n+1/2)} to the force update of Sec. 5, so
                                  px_prev.. are not needed; lepton tiles then need E and B.
                                  0: momenta are taken as given                                   */
    int32_t zero_product_counts; /* 1: the product counts (product_counts, or every set's) are
                                  set to zero on the stream before the step, so that the buffers
                                  receive this step's products only; 0: products are appended    */
} sfq_step_desc;

#define SFQ_MAX_TILES 4096

/* Launch shape of sfq_step for this handle (used by the autotuner): the streaming kernel runs
 * blocks_per_cu x (number of compute units) blocks of 256 threads, each taking `chunk`
 * consecutive particles of one tile at a time (chunk a multiple of 256 in [256, 2^22]).
 * Results do not depend on the launch shape. */
sfq_status sfq_set_launch(sfq_handle h, int blocks_per_cu, int chunk);
sfq_status sfq_get_launch(sfq_handle h, int* blocks_per_cu, int* chunk);


/* The Monte Carlo step (paper Fig. 7 workflow; App. A functions 4-6, 8-11, 15-17): for every
 * alive particle of every tile, gamma and chi (or, for blcfa leptons, the Sec. 5 force update),
 * the LCFA rate, the decision of cfg.decision, and for the particles that emit: Philox draws,
 * the energy sample, collinear recoil and the products.  All tiles run in one launch sequence
 * on `stream`.  Draws depend only on (seed, uid, step, purpose), so results do not depend on how
 * particles are split into tiles or batched with other work; only the order of products in
 * their buffers does (identify them by parent uid and species).  On product overflow the
 * particle state has still been advanced: restore it and re-run with larger buffers to get the
 * same result. */
sfq_status sfq_step(sfq_handle h, const sfq_step_desc* desc, void* stream);

/* sfq_step for callers that cannot allocate device memory (tight serving loops, code that may
 * not call hipMalloc): the same step and the same results, with no allocation of any kind in the
 * call.  Its scratch (the tile descriptors, at most 2 MiB of them; the emitter queue; the
 * deferred-share list) lives in a static device array of 256 MiB that the library holds on
 * each device it runs on until the process ends; sfq_create sets it up, with a pinned buffer
 * per handle for the descriptors.  The queue takes what the array leaves: shares that do not
 * fit are stepped by the deferred-share kernel, so results never depend on it (the call uses
 * the handle's launch shape, with the chunk halved while one share per slice would take more
 * than half of the queue's room).  Steps with more chunks than the array can list (about
 * sixteen million), or descriptors beyond 2 MiB, return SFQ_E_CAPACITY and enqueue nothing; a
 * capturing stream returns SFQ_E_STATE.  All calls on one
 * device share the array, and it keeps the last call's contents: calls that overlap on one
 * device (other streams, other handles, other threads) race and must be ordered by the caller;
 * calls on one stream are ordered by it.  Timing events (sfq_profile_*) are not recorded. */
sfq_status sfq_step_noalloc(sfq_handle h, const sfq_step_desc* desc, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Plans: a fixed set of tiles stepped repeatedly.  The descriptors are uploaded once, the plan
 * owns its emitter queue, and the Philox step index lives in device memory and advances by one
 * after every step, so a plan launch enqueues kernels only (no host copies, no allocation) and
 * a sequence of launches can be captured in a HIP graph and replayed.                          */
/* ------------------------------------------------------------------------------------------ */
typedef struct sfq_plan_t* sfq_plan;

/* Creates a plan for the tiles and buffers of `desc` (pointers are kept, the tile array is
 * copied; desc->step is the first step index).  zero_product_counts = 1 (or
 * desc->zero_product_counts = 1) zeroes the product counts at the start of every step (with a
 * kernel).  The handle's launch shape
 * (sfq_set_launch) at creation time is used.  The plan must be destroyed before the handle. */
sfq_status sfq_plan_create(sfq_handle h, const sfq_step_desc* desc, int zero_product_counts,
                           sfq_plan* out);
void sfq_plan_destroy(sfq_plan p);

/* One step of the plan on `stream` (same results as sfq_step with the current step index). */
sfq_status sfq_plan_launch(sfq_plan p, void* stream);

/* Sets the device step index of the plan (enqueued on `stream`). */
sfq_status sfq_plan_set_step(sfq_plan p, uint64_t step, void* stream);

/* Captures `steps` consecutive plan steps into a HIP graph (replacing a previous one) and
 * replays it: one graph launch advances the plan by `steps` steps. */
sfq_status sfq_plan_capture(sfq_plan p, int steps);
sfq_status sfq_plan_replay(sfq_plan p, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Scratch sizing and kernel timing                                                            */
/* ------------------------------------------------------------------------------------------ */
/* The emitter queue (device scratch owned by the handle) holds the particles that emit in a
 * step between the streaming pass and the emitter pass.  Each wave of the streaming pass owns a
 * slice of it, sized for the expected emitters, not for the worst case: a wave whose slice could
 * not take every particle of its next share of a chunk (chunk / 4 particles) leaves that share
 * untouched, and a further kernel of the same step steps it afterwards with the same arithmetic.
 * So the queue size never changes results, only speed (sfq_counters.deferred counts the
 * particles of such shares).  Streaming blocks take chunks as they become free, up to their
 * even share plus a sixteenth; a slice holds one share plus `2 * expected_fraction` of the
 * particles of that many shares (at most all of them, which makes deferral impossible).
 *
 * Pre-sizes the queue for sfq_step calls of up to `max_particles` particles in up to
 * `max_tiles` tiles with the current launch shape and queue fraction, so that such calls
 * allocate nothing.  A larger step, one after a change of launch shape, or one after the queue
 * fraction grew still grows the queue, which waits for the device.  SFQ_E_NOMEM if the
 * allocation fails. */
sfq_status sfq_reserve(sfq_handle h, uint64_t max_particles, int max_tiles);

/* Sizing of the emitter queue: `expected_fraction` in [0, 1] is the fraction of a step's
 * particles expected to emit (the slices hold twice that, plus one share; the default is 1/16,
 * adaptive); with adaptive = 1 the library raises it to twice the largest emitter fraction of
 * a wave's shares that the completed steps report (faster after deferrals), with adaptive = 0
 * it stays.  Takes effect from the next sfq_step, sfq_reserve or sfq_plan_create. */
sfq_status sfq_set_queue(sfq_handle h, double expected_fraction, int adaptive);

/* Bytes of device memory the handle's emitter queue holds now (0 before the first step). */
sfq_status sfq_queue_bytes(sfq_handle h, uint64_t* bytes);

/* Kernel timing (instrumentation).  With enable = 1, every sfq_step and sfq_plan_launch on this
 * handle records HIP events on its stream before the streaming kernel, between it and the
 * emitter pass, and after the step's last kernel; with enable = 2 only the first and the last
 * (the whole step); 0 stops.  Not inside sfq_plan_capture, nor in a launch the caller
 * captures.  They are timing-only events (hipEventDisableSystemFence), so recording them does
 * not write back the caches; each record still leaves the device idle for a few microseconds
 * before the next kernel starts, which the timings include (enable = 2 adds one such gap per
 * step, enable = 1 two).  sfq_profile_read waits for the recorded events, returns the summed
 * durations in ms of the streaming kernel and of the emitter pass (for steps timed whole: the
 * whole step, and 0) and the number of steps timed since the previous read, and clears them.
 * Any output may be NULL.  SFQ_E_ARG for another enable value. */
sfq_status sfq_profile_enable(sfq_handle h, int enable);
sfq_status sfq_profile_read(sfq_handle h, double* stream_ms, double* emit_ms, uint64_t* steps);

/* The same timings step by step (for latency percentiles): for each step timed since the
 * previous read, in order, the streaming kernel's and the emitter pass's (emitter and
 * deferred-share kernels) durations in ms go to stream_ms[k] and emit_ms[k] (a step timed
 * whole: its duration and 0; host arrays of max_steps floats, owned by the caller); *steps
 * receives the count, and the timings are cleared.  The events are
 * timing-only (no system-scope fence on record).  SFQ_E_CAPACITY, and nothing cleared, when
 * more than max_steps steps are pending; SFQ_E_ARG for NULL arrays when steps are pending. */
sfq_status sfq_profile_read_steps(sfq_handle h, uint64_t max_steps, float* stream_ms,
                                  float* emit_ms, uint64_t* steps);

#ifdef __cplusplus
}
#endif

#endif /* SFQ_H */
