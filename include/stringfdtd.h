/*
 * libstringfdtd: MI355X (gfx950) finite-difference time-domain synthesis of
 * stiff, lossy, nonlinear planar strings (transverse u and longitudinal zeta
 * coupled), after "String Sound Synthesizer on GPU-Accelerated Finite
 * Difference Scheme" (Lee, Choi, Lee; arXiv 2311.18505).
 *
 * One batch holds `capacity` independent string slots.  Each slot is given
 * physical and control parameters (Table 1 of the paper), an excitation by
 * pluck or hammer (Sec. 3.3), and is then advanced by the recursion of
 * eq. (7) from its initial conditions (Sec. 3.4); the readout of u at x_out is
 * written to device memory one sample per time step.
 *
 * Conventions
 *  - Every call returns an int status (SB_OK or a negative SB_E* code); no
 *    exception crosses the boundary.  string_batch_last_error() describes the
 *    last failure of a handle (pointer valid until the next call on it).
 *  - Host arrays passed in are copied before the call returns; the caller
 *    keeps ownership of every pointer it passes.
 *  - string_batch_step() is asynchronous on the HIP stream given at create
 *    time; outputs are valid after that stream is synchronised.
 *    string_batch_read_output() orders itself on the same stream.
 *  - A handle is not thread-safe: use one handle per host thread.
 *  - Units: the string has length L = 1 (positions are fractions of L),
 *    displacements are metres, time is seconds.
 */
#ifndef STRINGFDTD_H
#define STRINGFDTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SB_OK          0
#define SB_EINVAL     -1   /* invalid argument (range, NaN/Inf, index)              */
#define SB_ENOMEM     -2   /* device or host allocation failed                      */
#define SB_EBUDGET    -3   /* string larger than the per-wavefront budget (N > 1024) */
#define SB_EUNSTABLE  -4   /* energy monitor flagged a string, or the solve diverged */
#define SB_ESTATE     -5   /* call out of order (e.g. step before excite)            */
#define SB_EDEVICE    -6   /* HIP runtime error                                      */

/* precision of a batch */
#define SB_FP64        0   /* acceleration-form stepping in FP64                      */
#define SB_FP32C       1   /* FP32 stepping with compensated (Kahan) state updates    */
#define SB_FP64_PLAIN  2   /* eq. (7) as printed, FP64, serial banded LU per string   */

/* excitation types */
#define SB_EXC_NONE    0
#define SB_EXC_PLUCK   1
#define SB_EXC_HAMMER  2
#define SB_EXC_BOW     3

/* f0 modulation types */
#define SB_MOD_NONE    0
#define SB_MOD_VIBRATO 1   /* f0 * 2^{(depth/1200) sin(2 pi rate t)}                  */
#define SB_MOD_GLIDE   2   /* f0 * 2^{(semitones/12) t/T}, T = n_samples/fs           */

/* Transverse end conditions (zeta is always fixed at both ends).  Simply
 * supported: u = u_xx = 0, D_xxxx = D_xx^2, partials n f0 sqrt(1 + B n^2).
 * Clamped: u = u_x = 0 (the string of Sec. 4.1, whose partials eq. (10)
 * gives); D_xxxx takes mirrored ghost nodes u_{-1} = u_1, u_{N+1} = u_{N-1},
 * and N_t is lowered below the simply supported bound when needed until
 * 4 Theta - k^2 (gamma^2 (-D_xx) + kappa^2 D_xxxx) is positive definite. */
#define SB_BOUNDARY_SIMPLE  0
#define SB_BOUNDARY_CLAMPED 1

typedef struct sb_batch sb_batch;   /* opaque; owns all device memory of the batch */

/* Physical and control parameters of one string (Table 1; Sec. 3.2, 4.1).
 * gamma = 2 f0 (Sec. 4.1), kappa = gamma sqrt(B)/pi (inharmonicity
 * K = (pi kappa/gamma)^2 of Sec. 4.1 read as B).  theta <= 0 selects the
 * paper's (1+4/pi^2)/2; otherwise 1/2 < theta <= 1.  The grids are sized at
 * the stability bounds of the theta-scheme (transverse) and h_l >= gamma
 * alpha k (longitudinal) from the largest f0 the modulation reaches; grid_t /
 * grid_l > 0 force a size instead (testing).  alpha == 1 omits the
 * longitudinal grid (the system is then linear and zeta stays zero). */
typedef struct {
    double fs;                 /* sample rate [Hz], k = 1/fs                      */
    double f0;                 /* fundamental of the ideal string [Hz]            */
    double B;                  /* inharmonicity (>= 0)                            */
    double alpha;              /* stiffness-to-tension ratio (>= 1)               */
    double theta;              /* theta-scheme parameter                          */
    double sigma0_t, sigma1_t; /* transverse losses of eq. (4a) [1/s], [m^2/s]    */
    double sigma0_l, sigma1_l; /* longitudinal losses of eq. (4b)                 */
    double x_out;              /* readout position in (0,1)                       */
    int64_t n_samples;         /* output length (>= 2)                            */
    int32_t mod_type;          /* SB_MOD_*                                        */
    int32_t grid_t;            /* 0 or a forced N_t                               */
    double mod_depth_cents;    /* vibrato depth                                   */
    double mod_rate_hz;        /* vibrato rate                                    */
    double glide_semitones;    /* glide interval over the duration                */
    int32_t grid_l;            /* 0 or a forced N_l                               */
    int32_t boundary;          /* SB_BOUNDARY_*: transverse end condition         */
    int32_t readout_zeta;      /* 1: also record zeta at x_out (second channel)   */
    int32_t grid_interp;       /* order p of I_(l)->(t): 0 or 1 linear, 3 cubic   */
} sb_string_params;

/* Excitation (Sec. 3.3).  Pluck: initial triangle of peak c0 at x, released
 * from rest.  Hammer (eq. 6): lumped mass M_H [kg] at x with initial velocity
 * v_H [m/s], felt force K_H max(0, compression)^alpha_H, mass ratio
 * M_H / (rhoA * 1 m); starts touching the string at rest.  Bow (eq. 5): the
 * string starts at rest; the term -J_p(x_B) F_B phi(v_rel) acts on u with
 * v_rel = I_p(x_B) delta_t. u - v_B and the friction curve
 * phi(v) = sign(v) (fric_eps + (1 - fric_eps) exp(-fric_a |v|)); at
 * v_rel = 0 the string sticks (|phi| <= 1).  F_B (force per unit linear
 * density, m/s^2 on the string of length 1) and v_B [m/s] rise linearly over
 * `attack` seconds; the position moves linearly from x to x_end over the note
 * (n_samples / fs).  Each step solves the coupled system for its right-hand
 * side and for the bow's unit force, then the step's stick/slip problem
 * exactly (as a direct solve of eq. (7) would); SB_FP64_PLAIN carries the
 * unit force through its band elimination as a second right-hand side.
 * interp_order = 3 gives the hammer the cubic interpolant of Sec. 3.3
 * (p = 3): four nodes around x, nodes past an end mirrored with the sign of
 * the end condition, spreading J = I^T / h (batched precisions only;
 * SB_FP64_PLAIN refuses it). */
typedef struct {
    int32_t type;              /* SB_EXC_*                                        */
    int32_t interp_order;      /* hammer's I_p: 0 or 1 linear, 3 cubic (below)   */
    double x;                  /* position in (0,1); the bow's at t = 0           */
    double c0;                 /* pluck peak [m]                                  */
    double v_H, M_H, K_H, alpha_H, rhoA;
    double x_end;              /* bow position at the end of the note, in (0,1)   */
    double v_B, F_B, attack;   /* bow speed [m/s], force (>= 0), attack [s]       */
    double fric_a, fric_eps;   /* friction curve: a >= 0 [s/m], 0 <= eps <= 1     */
} sb_excitation;

/* Per-slot information (grid sizes and progress). */
typedef struct {
    int32_t N_t, N_l;          /* grid intervals (N_l = 0: no longitudinal grid)  */
    int64_t n_samples;         /* requested samples                               */
    int64_t samples_done;      /* samples available in the output                */
    int32_t flags;             /* 1: unstable (energy monitor), 2: no convergence */
    int32_t max_sweeps;        /* largest number of coupled-solve sweeps in a step */
    int64_t total_sweeps;      /* total sweeps                                    */
    int32_t size_class;        /* kernel size class 0..7 of the batched paths      */
    int32_t lanes;             /* lanes per string in that class (16, 32 or 64)   */
    int32_t slots_t, slots_l;  /* slots per lane of the transverse / longitudinal
                                  grid in the string's layout (FP32 batches: the
                                  fewest of the class's MM, 3MM/4 and MM/2 the
                                  grid fits in; FP64: MM; 0 on the plain path)   */
} sb_string_info;

/* Create a batch of `capacity` (>= 1) slots computing in `precision`
 * (SB_FP64, SB_FP32C or SB_FP64_PLAIN), launching on `hip_stream` (a
 * hipStream_t; NULL = the default stream).  *out receives the handle.
 * Errors: SB_EINVAL, SB_ENOMEM, SB_EDEVICE. */
int string_batch_create(int capacity, int precision, void *hip_stream, sb_batch **out);

/* Set the parameters of slots first .. first+count-1 from p[0..count-1]
 * (host array).  Plans the grids (Sec. 3.2), coefficient and interpolation
 * tables, and allocates the slots' device state and output (n_samples
 * samples each).  Resets the slots: excite must follow before step.
 * Errors: SB_EINVAL (ranges: fs, f0 > 0, B >= 0, alpha >= 1, 1/2 < theta <= 1,
 * sigmas >= 0, 0 < x_out < 1, n_samples >= 2, finite values), SB_EBUDGET
 * (N_t or N_l > 1024), SB_ENOMEM. */
int string_batch_set_params(sb_batch *b, int first, int count, const sb_string_params *p);

/* Excite slots first .. first+count-1 with e[0..count-1] (host array): writes
 * the initial conditions w^0, w^1 and samples y^0, y^1 (Sec. 3.3-3.4).
 * Errors: SB_EINVAL (type, 0 < x < 1, hammer M_H, K_H, rhoA > 0,
 * alpha_H >= 1, finite), SB_ESTATE (slot without parameters). */
int string_batch_excite(sb_batch *b, int first, int count, const sb_excitation *e);

/* Advance every excited slot by n_steps time steps of eq. (7) (clamped at
 * its n_samples), asynchronously on the batch stream.  Each step produces one
 * output sample.  Errors: SB_EINVAL (n_steps < 0), SB_ESTATE (no excited
 * slot), SB_EDEVICE.  Use string_batch_info() after a synchronisation to see
 * per-slot flags (the step of a flagged slot stops). */
int string_batch_step(sb_batch *b, int64_t n_steps);

/* Same as string_batch_step but only for slots first .. first+count-1. */
int string_batch_step_range(sb_batch *b, int first, int count, int64_t n_steps);

/* Several excitations per note: a new hammer or bow (e[i].type
 * SB_EXC_HAMMER or SB_EXC_BOW) on each of slots first .. first+count-1 while
 * they sound, applied before their next step n (the one computing sample
 * samples_done).  The string keeps its state and the new excitation replaces
 * the slot's hammer or bow: a hammer arrives touching the string at level
 * n-1 with velocity v_H toward it (the initial hammer when the string
 * rests); a bow's controls (attack, position sweep over the rest of the
 * note) restart from level n-1.  Synchronises the batch stream; a rewind of
 * a re-excited slot is refused until it is excited again.  Errors: SB_EINVAL
 * (plain path, other types, bad parameters), SB_ESTATE (slot not excited or
 * finished), SB_EDEVICE. */
int string_batch_restrike(sb_batch *b, int first, int count, const sb_excitation *e);

/* The same for count arbitrary slots slots[i] (each listed once), e[i]
 * applied to slots[i]; the slots of one call share two synchronisations. */
int string_batch_restrike_list(sb_batch *b, int count, const int32_t *slots, const sb_excitation *e);

/* Return slots first .. first+count-1 to their state right after
 * string_batch_excite (samples_done = 2, flags cleared) without host work:
 * a device copy of the excited state is kept for this.  Asynchronous on the
 * batch stream.  Errors: SB_EINVAL, SB_EDEVICE. */
int string_batch_rewind(sb_batch *b, int first, int count);

/* Checkpoint and resume of one slot.  The recursion of eq. (7) carries its
 * whole past in the two latest grid levels (Sec. 3.2), so a slot's stepping
 * state is small and self-contained: both grids at levels n and n-1 (as
 * value and velocity, with their compensations on the FP32 compensated
 * path), the hammer's lumped state, the energy monitor's reference and the
 * progress counters.  A snapshot copies exactly that; restoring it onto the
 * same slot makes the next steps reproduce, bit for bit, what they computed
 * after the snapshot was taken (output samples from samples_done on are
 * written again).  Output already written, the parameters and the
 * excitation tables are not part of it: a snapshot restores only onto the
 * slot it was taken from, and only while that slot keeps the excitation it
 * had (excite or restrike in between: SB_ESTATE).
 *
 * string_batch_snapshot_bytes: size in bytes of slot idx's snapshot (a
 *   256-byte header, then the state block).
 * string_batch_snapshot: waits for the batch's queued work, then copies the
 *   snapshot to dst (caller-owned, at least that many bytes; host memory, or
 *   device memory when dst_is_device) and returns when the copy is complete.
 * string_batch_restore: checks the snapshot's header against the slot
 *   (SB_EINVAL when it is not a snapshot of this slot's string or bytes
 *   differs from its size), waits for the batch's queued work, copies it back
 *   and returns when the copy is complete; the slot's samples_done and flags
 *   become the snapshot's.  A captured graph must be captured again.
 * Errors: SB_EINVAL, SB_ESTATE (slot not excited, or re-excited since the
 * snapshot), SB_EDEVICE. */
int string_batch_snapshot_bytes(sb_batch *b, int idx, int64_t *bytes);
int string_batch_snapshot(sb_batch *b, int idx, void *dst, int64_t bytes, int dst_is_device);
int string_batch_restore(sb_batch *b, int idx, const void *src, int64_t bytes, int src_is_device);

/* Launch capture (batched paths).  Records n_launches consecutive launches
 * of steps_per_launch steps each, of every slot excited at the time of the
 * call (the launches forked onto their streams and joined back, counters
 * cleared by a kernel), into a HIP graph owned by the batch; capture happens
 * on an internal stream, so nothing runs.  string_batch_graph_launch replays
 * it on the batch stream and advances every captured slot like the same
 * sequence of string_batch_step calls would (slots that reach n_samples idle).
 * set_params or excite on any slot invalidates the graph (launch then returns
 * SB_ESTATE); rewind does not.  Errors: SB_EINVAL (plain path, bad shape),
 * SB_ESTATE (nothing to step / stale graph), SB_EDEVICE. */
int string_batch_graph_capture(sb_batch *b, int64_t steps_per_launch, int n_launches);
int string_batch_graph_launch(sb_batch *b);

/* A batched step runs as SB_NUM_LAUNCHES concurrent units of kernel
 * launches, each on its own stream, forked from and joined back to the batch
 * stream:
 *   0: size classes 0..4 (up to 384 points), one persistent launch with one
 *      work queue, the classes' tasks dealt out in proportion;
 *   1: size class 5 (up to 512 points);
 *   2: size classes 6 (up to 640 points) and 7 (up to 1024), one launch
 *      after the other. */
#define SB_NUM_LAUNCHES 3

/* Durations of the launches of the last batched step (string_batch_step or a
 * captured graph's last launch), in ms, and the number of strings each
 * stepped; ms[u] = 0 for launches that did not run.  Synchronises the stream.
 * Errors: SB_EINVAL, SB_EDEVICE. */
int string_batch_launch_times(sb_batch *b, float ms[SB_NUM_LAUNCHES], int32_t strings[SB_NUM_LAUNCHES]);

/* Autotuner (batched paths): chooses the persistent blocks per CU of the
 * launches jointly.  Each probe is a whole step of probe_steps steps (all
 * launches concurrently, as string_batch_step runs them); coordinate descent
 * over the launches, largest strings first, tries 1, 2, 4, 6 and 8 blocks per
 * CU (up to the launch's occupancy limit) and keeps the shortest probe.  The
 * choice applies to later steps and is reported in chosen[SB_NUM_LAUNCHES]
 * (0 for launches with nothing to step; chosen may be NULL).  Every slot is
 * rewound to its excitation before and after, so call it right after excite.
 * Errors: SB_EINVAL, SB_ESTATE (nothing excited), SB_EDEVICE. */
int string_batch_autotune(sb_batch *b, int64_t probe_steps, int32_t *chosen);

/* Persistent blocks per CU of each launch for later steps
 * (blocks[SB_NUM_LAUNCHES]; 0 = the launch's occupancy limit), e.g. a
 * schedule found by the autotuner on a previous run.  Errors: SB_EINVAL. */
int string_batch_set_blocks_per_cu(sb_batch *b, const int32_t *blocks);

/* Copy samples offset .. offset+count-1 of slot idx to dst (count elements
 * of the batch precision: float for SB_FP32C, double otherwise), ordered on
 * the batch stream.  A host destination (dst_is_device == 0) is written
 * synchronously with the stream; samples the slot has not produced yet (at
 * or past its samples_done, e.g. after the energy monitor stopped it) are
 * written as zero, and a flagged slot returns SB_EUNSTABLE after the copy.
 * A device destination is an asynchronous copy of the buffer as it stands.
 * Errors: SB_EINVAL (range beyond n_samples), SB_ESTATE (slot not excited),
 * SB_EUNSTABLE, SB_EDEVICE. */
int string_batch_read_output(sb_batch *b, int idx, int64_t offset, int64_t count, void *dst, int dst_is_device);

/* The second readout channel: zeta at x_out, interpolated on the
 * longitudinal grid like u (the paper's Fig. 2 shows the transverse and the
 * longitudinal outputs and their spectra, discussed in Sec. 4.2; zero for
 * alpha = 1), recorded only for strings set with readout_zeta = 1 on the
 * batched paths; same arguments, ordering and zero filling as
 * string_batch_read_output.  Errors: SB_EINVAL (range beyond n_samples),
 * SB_ESTATE (slot not excited or set without the channel), SB_EUNSTABLE,
 * SB_EDEVICE. */
int string_batch_read_output_zeta(sb_batch *b, int idx, int64_t offset, int64_t count, void *dst,
                                  int dst_is_device);

/* Device pointer of slot idx's output samples (n_samples elements of the
 * batch precision); the batch owns the memory. */
int string_batch_output_ptr(sb_batch *b, int idx, void **dev_ptr);

/* Streaming readout of many slots at once (the output signal of Sec. 3.4's
 * recursion, one chunk per string): row i of dst (count elements of the
 * batch precision) receives samples offsets[i] .. offsets[i]+count-1 of slot
 * slots[i]; samples the slot has not produced (at or past its samples_done
 * or n_samples) are written as zero, so a row never holds stale audio.  One
 * gather kernel and one copy, ordered on the batch stream.  slots/offsets
 * are host arrays of n entries, copied before the call returns.
 * samples_done and flags (host arrays of n entries, or NULL) receive each
 * listed slot's progress and flags (as string_batch_info reports them).
 * Unless dst is on the device and both are NULL, the call is synchronous
 * with the batch stream and returns SB_EUNSTABLE when any listed slot is
 * flagged (the rows and arrays are written either way; last_error names the
 * slots).  Errors: SB_EINVAL (bad slot, offset outside [0, n_samples)),
 * SB_ESTATE (slot not excited), SB_EUNSTABLE, SB_ENOMEM, SB_EDEVICE. */
int string_batch_gather_output(sb_batch *b, int n, const int32_t *slots, const int64_t *offsets, int64_t count,
                               void *dst, int dst_is_device, int64_t *samples_done, int32_t *flags);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): string_batch_gather_output into a device
 * destination without any allocation.  The gathered slot indices, offsets
 * and per-row progress and flags live in a fixed scratch array of the
 * library (SB_NOALLOC_MAX_ROWS rows, about 384 KiB, held by each GPU the
 * library runs on until the process ends) instead of buffers of the batch.
 * Same rows, zero filling and return codes as string_batch_gather_output;
 * dst is device memory of n*count elements of the batch precision;
 * samples_done and flags are host arrays of n entries or NULL.  Synchronous
 * with the batch stream.  Every call on one GPU shares that GPU's scratch:
 * calls that overlap on one GPU (batches on different streams or threads at
 * the same time) race and must not be made.  Errors: SB_EINVAL (n above
 * SB_NOALLOC_MAX_ROWS or the capacity, bad slot, offset outside
 * [0, n_samples)), SB_ESTATE (slot not excited), SB_EUNSTABLE, SB_EDEVICE. */
#define SB_NOALLOC_MAX_ROWS 16384
int string_batch_gather_output_noalloc(sb_batch *b, int n, const int32_t *slots, const int64_t *offsets,
                                       int64_t count, void *dst, int64_t *samples_done, int32_t *flags);

/* Energy H^{n+1/2} of slot idx at its last monitor check (FP64, computed on
 * the GPU), and the step n of that check (-1 if none).  Synchronises the
 * stream.  Errors: SB_EINVAL, SB_EDEVICE. */
int string_batch_read_energy(sb_batch *b, int idx, double *H_latest, int64_t *step_of_H);

/* Grid sizes and progress of slot idx.  Synchronises the stream. */
int string_batch_info(sb_batch *b, int idx, sb_string_info *info);

/* Energy monitor period in steps (0 disables; default 480) and relative
 * growth tolerance (default 1e-9 for FP64, 1e-4 for FP32C). */
int string_batch_set_monitor(sb_batch *b, int period, double growth_tol);

/* Coupled-solve controls of the batched paths (block Gauss-Seidel between
 * the transverse and longitudinal grids, eq. (8)).  A string's step has
 * converged when the estimated error of its accelerations -- the largest
 * update of the last sweep times that sweep's contraction, the ratio of the
 * last two sweeps' largest updates -- or the update itself is below tol
 * times the string's largest acceleration after the first sweep (default
 * 1e-13 FP64, 1e-7 FP32C: the FP32 rounding of the acceleration).  Strings
 * in the kernels that carry bows, clamped ends or the zeta channel stop on
 * the update alone, below tol (FP64) or 100 tol (FP32C) times that value
 * (the stick/slip decision of a chaotic bowed string amplifies the solve's
 * error).  max_sweeps caps the sweeps per step (default 64; a step that
 * reaches it flags the string with 2). */
int string_batch_set_solver(sb_batch *b, double tol, int max_sweeps);

/* Grid sizes the library plans for p (host only, needs no device): N_t from
 * the stability bound of the theta-scheme (for clamped ends lowered further
 * if the energy test of SB_BOUNDARY_CLAMPED fails), N_l from
 * h_l >= gamma alpha k.  Errors: SB_EINVAL. */
int string_plan_grid(const sb_string_params *p, int32_t *N_t, int32_t *N_l);

/* Free every resource of the batch (synchronises its stream first). */
int string_batch_destroy(sb_batch *b);

/* Description of the last error on b (or of the last create failure if b is NULL). */
const char *string_batch_last_error(const sb_batch *b);

#ifdef __cplusplus
}
#endif
#endif
