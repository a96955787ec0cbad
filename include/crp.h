/*
 * crp.h -- C ABI of the MI355X (gfx950) charged-particle propagation library.
 *
 * The library advances many independent charged nuclei through a magnetic
 * field sampled on a regular periodic grid, the 3D mode of "Cosmic ray
 * propagation with CRPropa 3" (sections 2 and 3.2).  Each particle carries
 * position, direction, energy, charge and mass (section 3.1: the particle is
 * the single interface between modules).  Each step is an error-controlled
 * Cash-Karp Runge-Kutta step of the Lorentz force with trilinear field
 * interpolation at every stage; its length is the lowest bid among the
 * controller, the step limits, the distance to the observer sphere and the
 * remaining trajectory length (section 3.1, bidding system).  Propagation
 * ends at the observer sphere, at the length limit or when aborted
 * (section 3.1: "completed or aborted").  Energy is not changed (no losses,
 * as in section 3.3).  A negative charge with reversed direction propagates
 * backwards (section 3.3, backtracking).
 *
 * Conventions
 *   - [dev] marks device pointers; every buffer is owned by the caller (for
 *     example allocated through PyTorch).  The library never allocates device
 *     memory and keeps no global state other than a thread-local error string;
 *     the one exception is crp_propagate_noalloc's scratch array, a fixed
 *     array in the library's device image whose per-device address it keeps.
 *   - All work is enqueued on the caller's stream and is asynchronous; the
 *     call returns after enqueueing.  The exception is crp_lens_build, which
 *     waits for its stream to return the entry count and the row checks to
 *     the host.  No call throws across the ABI.
 *   - Units: positions and lengths in Mpc, energies in eV, fields in nG,
 *     times in seconds.  Status values are the CRP_ST_* codes below.
 *   - Argument errors are reported synchronously, before anything is
 *     enqueued, as CRP_ERR_INVALID; a failing HIP call as CRP_ERR_DEVICE.
 *     Problems of one particle only go into its status.
 */
#ifndef CRP_H
#define CRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRP_OK = 0,
    CRP_ERR_INVALID = -1,      /* bad argument; nothing was enqueued */
    CRP_ERR_DEVICE = -2,       /* a HIP runtime call failed */
    CRP_ERR_UNSUPPORTED = -3,  /* valid but not supported combination */
    CRP_ERR_WORKSPACE = -4     /* workspace missing or too small */
} crp_status;

typedef enum { CRP_F64 = 0, CRP_F32 = 1, CRP_F16 = 2, CRP_BF16 = 3 } crp_dtype;

/* Device storage layout of a field grid.
 * LINEAR: nodes [i][j][k][3] with one duplicated wrap node on every axis,
 *         (n0+1)(n1+1)(n2+1)*3 values; the 8 corners of a cell never wrap.
 * CELL8:  one record per cell holding its 8 corner vectors (24 values padded
 *         to 32), n0*n1*n2*32 values; a cell lookup reads one record. */
typedef enum { CRP_LAYOUT_LINEAR = 0, CRP_LAYOUT_CELL8 = 1 } crp_layout;

/* Arithmetic of the propagation kernel.
 * FP64: every stage in FP64 (the parity path).
 * MIXED_F64ACC: FP32 stages, position / length / time accumulated in FP64.
 * MIXED_DFACC: FP32 stages, position / length accumulated as double-float. */
typedef enum { CRP_PREC_FP64 = 0, CRP_PREC_MIXED_F64ACC = 1, CRP_PREC_MIXED_DFACC = 2 } crp_precision;

/* Particle status (per particle, in crp_particles.status). Only ACTIVE particles
 * are propagated; set MAX_STEPS or CANCELLED back to ACTIVE to resume. */
enum {
    CRP_ST_ACTIVE = 0,      /* still propagating */
    CRP_ST_ARRIVED = 1,     /* crossed the observer sphere (event located) */
    CRP_ST_MAX_LENGTH = 2,  /* trajectory length reached l_max exactly */
    CRP_ST_MAX_STEPS = 3,   /* accepted-step budget of this call used up */
    CRP_ST_NONFINITE = 4,   /* the error estimate or the event function was not finite */
    CRP_ST_CANCELLED = 5,   /* stopped by the caller's cancel word (crp_tuning.cancel) */
    CRP_ST_BAD_INPUT = 6    /* E <= 0, zero or non-finite direction or position, bad h_next */
};

/* A periodic scalar modulation grid (section 3.2, modulated grids: a small
 * high-resolution vector grid repeated periodically, times a large
 * low-resolution grid that carries the large-scale structure).  The field at
 * x becomes b(x) * m(x), m interpolated trilinearly on this grid (x, then y,
 * then z) and repeated with period n * spacing. */
typedef struct {
    int32_t n[3];          /* nodes per axis, each >= 2 */
    int32_t dtype;         /* CRP_F64 or CRP_F32 storage */
    double origin[3];      /* Mpc, position of node (0, 0, 0) */
    double spacing;        /* Mpc, > 0 */
    void *data;            /* [dev] crp_modulation_bytes(this) bytes, written by crp_modulation_upload */
} crp_modulation;

/* One periodic vector grid (section 3.2: regular grids; section 4: a vector
 * grid with a random Kolmogorov realisation).  Node (i,j,k) sits at
 * origin + spacing*(i,j,k); the field repeats with period n*spacing.
 * Domain: cell indices are 32-bit integers, so positions must stay within
 * 2^31 spacings of the origin along each axis (1.07e8 Mpc at 50 kpc); beyond
 * it the index saturates instead of wrapping, and results are not defined. */
typedef struct {
    int32_t n[3];          /* nodes per axis, each >= 2 */
    int32_t dtype;         /* crp_dtype of the stored values */
    int32_t layout;        /* crp_layout */
    int32_t reserved;
    double origin[3];      /* Mpc */
    double spacing;        /* Mpc, > 0 */
    double value_scale;    /* nG per stored unit (1 for F64/F32 grids) */
    void *data;            /* [dev] crp_field_bytes(this) bytes, written by crp_field_upload */
    const crp_modulation *modulation;  /* host pointer, NULL for none; no tape */
} crp_field;

/* Bidding and stopping parameters of one particle group (section 3.1).
 * Backtracking (section 3.3): with backtrack = 1 the particles' states are
 * where they were observed, and each is propagated as its antiparticle
 * (charge -Z) with the direction reversed; the direction written back is
 * reversed again, so input and output directions are the physical particle's
 * direction of motion (the output is the physical state a path length L
 * earlier).
 * Reflective box (the example of section 4 has reflective boundaries): with
 * reflect = 1 the distance to the nearest face also bids (after the sphere
 * distance, before the h_min floor), and a particle whose accepted step ends
 * outside the box on an axis, without arriving at the sphere, is mirrored on
 * that face: position 2 face - x, that direction component negated. */
typedef struct {
    double tol;            /* accuracy: error norm per step <= tol, > 0 */
    double h_min, h_max;   /* step limits in Mpc, 0 < h_min <= h_max */
    double obs_center[3];  /* observer sphere centre, Mpc */
    double obs_radius;     /* Mpc; <= 0 disables the sphere */
    double l_max;          /* length limit, Mpc, > 0; +inf disables it (then max_steps > 0) */
    int64_t max_steps;     /* accepted steps allowed per particle in one call; 0 = no limit */
    int32_t field_index;   /* which entry of the fields array this group uses */
    int32_t reflect;       /* 1: reflective box below; 0: none */
    double box_lo[3], box_hi[3];  /* Mpc, lo < hi on every axis when reflect = 1 */
    int32_t backtrack;     /* 1: backtracking (section 3.3); 0: forward */
    int32_t reserved;      /* 0 */
} crp_params;

/* Structure-of-arrays particle state; every pointer is [dev] with n entries
 * (may be NULL when n = 0).  In/out arrays are updated in place. */
typedef struct {
    double *x, *y, *z;        /* in/out position, Mpc */
    double *ux, *uy, *uz;     /* in/out direction; normalised on a fresh start */
    double *energy;           /* in, eV (unchanged) */
    int32_t *charge;          /* in, signed charge number Z (negative: backtracking) */
    int32_t *mass;            /* in, mass number A (carried, does not enter at beta = 1); may be NULL */
    double *length;           /* in/out trajectory length, Mpc */
    double *h_next;           /* in/out controller bid; 0 = fresh start */
    double *time;             /* out, length * Mpc / c in seconds; may be NULL */
    int32_t *status;          /* in/out CRP_ST_* */
    int32_t *param_index;     /* in, index into params; NULL = all use params[0] */
    int64_t *n_accepted;      /* in/out accepted steps (cumulative) */
    int64_t *n_rejected;      /* in/out rejected attempts (cumulative) */
} crp_particles;

/* Tape of a forward run for the adjoint (checkpointed replay).  Every K
 * accepted steps (and at the start of the call) the forward kernel takes the
 * next record of a shared pool (an atomic on *head) and writes the
 * particle's state into it: 8 doubles (x, y, z, ux, uy, uz, length,
 * controller bid), with links[record] = the particle's previous record (-1
 * for its first).  The head keeps counting past the capacity, so after a run
 * it holds the number of records the run needed; a particle that found the
 * pool exhausted sets the overflow flag.  For every particle the kernel writes
 * finals[4 i ..]: accepted steps N, the located crossing step s* (0 without
 * one), the index of its last record (as a double, -1 for none) and flags
 * (CRP_TAPE_* bits, as a double); all zero (last record -1) for a particle
 * that was not ACTIVE on entry.  The caller zeroes *head before the call.
 * The tape is valid only for crp_propagate_adjoint on the same particles,
 * field and parameters. */
typedef struct {
    double *checkpoints;          /* [dev] capacity records of 8 doubles */
    int64_t *links;               /* [dev] capacity previous-record indices */
    unsigned long long *head;     /* [dev] records handed out (caller zeroes) */
    double *finals;               /* [dev] 4 n doubles */
    int64_t capacity;             /* records in the pool, >= 1 */
    int32_t every_k;              /* checkpoint interval K, 1 .. 4096 */
    int32_t reserved;
} crp_tape;

enum {
    CRP_TAPE_EVENT = 1,        /* ended by a located sphere crossing */
    CRP_TAPE_OVERFLOW = 2,     /* the record pool ran out: no adjoint */
    CRP_TAPE_FRESH = 4,        /* started fresh (direction normalised on entry) */
    CRP_TAPE_COMPLETE = 8,     /* ended ARRIVED or MAX_LENGTH in this call */
    CRP_TAPE_MIRRORED = 16,    /* was mirrored by a reflective box at least once (its derivative
                                  is that of the replayed map; see crp_propagate_adjoint) */
    CRP_TAPE_GRAD_OVERFLOW = 32 /* set by crp_propagate_adjoint: the particle's cotangent left the
                                   FP64 range (a chaotic trajectory); its grid contributions from
                                   that point on were left out of grad_field */
};

/* Launch configuration; NULL selects the defaults. */
typedef struct {
    int32_t block_size;       /* threads per block: 64, 128 or 256 (default 256) */
    int32_t blocks_per_cu;    /* persistent blocks per compute unit (default 4); 0 = one lane per particle */
    int32_t refill_threshold; /* refill a wavefront when at least this many lanes are idle (default 32) */
    int32_t order_by_rigidity;/* 1: hand out low-rigidity particles first (longest first); default 1 */
    int32_t cache_cells;      /* keep each lane's last cell (in registers; in LDS for FP64 with
                                 per-particle groups) and skip repeated loads: 1 on, -1 off,
                                 0 automatic (default: on for LINEAR; for CELL8 on with more
                                 than 2048 particles per compute unit) */
    int32_t reserved;
    const int32_t *cancel;    /* NULL, or a [dev] word the caller may set nonzero while the call
                                 runs (from another stream, or mapped host memory) to stop it
                                 early: read by every wavefront once every 64 loop iterations;
                                 once seen, no further particle is started (those stay ACTIVE and
                                 untouched), a particle between accepted steps stops after its
                                 next accepted step with status CRP_ST_CANCELLED and its state
                                 saved, and one locating its sphere crossing finishes it.  Set
                                 CANCELLED back to ACTIVE (and the word to 0) to resume: the
                                 result is bit-identical to an uninterrupted call. */
} crp_tuning;

/* Counters accumulated by crp_propagate into an optional [dev] int64 array. */
enum {
    CRP_CNT_EVALS = 0,        /* Cash-Karp evaluations (each 6 field lookups) */
    CRP_CNT_ACCEPTED = 1,
    CRP_CNT_REJECTED = 2,
    CRP_CNT_EVENT_EVALS = 3,  /* evaluations spent locating sphere crossings */
    CRP_CNT_FLOOR_HITS = 4,   /* steps accepted at h_min with error above tolerance */
    CRP_CNT_PARTICLES = 5,    /* particles taken from the queue */
    CRP_CNT_CELL_LOADS = 6,   /* field lookups that read grid memory (the others hit the cell cache) */
    CRP_CNT_WAVE_ITERS = 7,   /* wavefront loop iterations (lane utilisation = EVALS / (64 x this)) */
    CRP_NCOUNTERS = 8
};

/* Bytes of device storage for a field in its dtype and layout; 0 if the
 * descriptor is invalid. */
size_t crp_field_bytes(const crp_field *f);

/* Fill f->data from src: [dev] C-order [n0][n1][n2][3] values in nG, of
 * src_dtype F64 or F32 (the grid of section 3.2 as produced by a field
 * generator).  Values are divided by f->value_scale and rounded to nearest
 * even into f->dtype, then written in f->layout.  src and f->data must not
 * overlap.  Stream s (hipStream_t, may be NULL for the default stream). */
crp_status crp_field_upload(const crp_field *f, const void *src, int32_t src_dtype, void *stream);

/* Bytes of device storage for a modulation grid; 0 if the descriptor is invalid. */
size_t crp_modulation_bytes(const crp_modulation *m);

/* Fill m->data from src: [dev] C-order [n0][n1][n2] values of src_dtype F64
 * or F32 (section 3.2, modulated grids), rounded to nearest even into
 * m->dtype and stored with the periodic wrap (one extra plane per axis).
 * src and m->data must not overlap.  Stream s may be NULL. */
crp_status crp_modulation_upload(const crp_modulation *m, const void *src, int32_t src_dtype, void *stream);

/* Device workspace needed by crp_propagate for n particles and the given
 * table sizes (field and parameter descriptors, work queue, ordering keys).
 * It is the same for every precision: no precision keeps per-particle
 * scratch in the workspace. */
size_t crp_workspace_bytes(int64_t n, int32_t n_fields, int32_t n_params);

/* Propagate n particles in place (sections 2, 3.1, 3.2): each ACTIVE particle
 * is stepped until it arrives at its observer sphere, reaches l_max, uses up
 * max_steps, or fails.  fields[n_fields] and params[n_params] are host
 * arrays; every field of one call must share dtype and layout.  tape: NULL,
 * or a tape to record for crp_propagate_adjoint (FP64 precision, one F64
 * or F32 field and one parameter group; else CRP_ERR_UNSUPPORTED).
 * precision is a crp_precision.  counters: optional [dev]
 * int64[CRP_NCOUNTERS], accumulated (caller zeroes).  workspace: [dev],
 * crp_workspace_bytes long, 256-byte aligned; its contents are scratch.
 * Calls that share a workspace must be ordered on one stream. */
crp_status crp_propagate(const crp_field *fields, int32_t n_fields, const crp_params *params,
                         int32_t n_params, const crp_particles *p, int64_t n, const crp_tape *tape,
                         int32_t precision, const crp_tuning *tuning, int64_t *counters, void *workspace,
                         size_t workspace_bytes, void *stream);

/* crp_propagate for callers that cannot allocate device memory: code under
 * hipGraph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, behaviour and results as crp_propagate, bit for bit, except
 * that there is no workspace argument: the library keeps one fixed scratch
 * array per GPU in its device image (crp_noalloc_scratch_bytes() bytes, about
 * 17 MB, held until the process ends) and uses it as the workspace.  The
 * call allocates nothing.  Limits: n <= CRP_NOALLOC_MAX_PARTICLES, n_fields
 * <= CRP_NOALLOC_MAX_FIELDS, n_params <= CRP_NOALLOC_MAX_PARAMS (else
 * CRP_ERR_INVALID before anything is enqueued).  Each call clears what must
 * start at zero and rewrites the rest, so no call depends on an earlier one;
 * but all calls on one GPU share its array, so calls that overlap on one GPU
 * (different streams or host threads without ordering) race and must not be
 * made. */
#define CRP_NOALLOC_MAX_PARTICLES 4194304
#define CRP_NOALLOC_MAX_FIELDS 64
#define CRP_NOALLOC_MAX_PARAMS 64
size_t crp_noalloc_scratch_bytes(void);
crp_status crp_propagate_noalloc(const crp_field *fields, int32_t n_fields, const crp_params *params,
                                 int32_t n_params, const crp_particles *p, int64_t n, const crp_tape *tape,
                                 int32_t precision, const crp_tuning *tuning, int64_t *counters, void *stream);

/* Workspace for crp_propagate_adjoint: n particles, checkpoint interval K.
 * The minimum: every particle's steps are replayed by the sweep itself. */
size_t crp_adjoint_workspace_bytes(int64_t n, int32_t every_k);

/* Workspace for crp_propagate_adjoint with room for the parallel replay of
 * replay_steps step records (616 bytes each: the record and the stages'
 * grid-value cotangents; plus about 8 bytes per checkpoint segment and 20 per
 * particle).  Before the reverse sweep, the particles with the most accepted
 * steps are replayed one checkpoint segment per thread (the segments are
 * independent given their checkpoints; section 3.1's step logic taken exactly
 * as the forward run took it), so the sweep of those particles, which sets
 * the time of the whole adjoint, is the reverse pass alone; their
 * grid-gradient contributions are added after the sweep, one thread per
 * segment, off its critical path.  They are taken in groups of 64 consecutive
 * particles of the adjoint's order (most steps first, sorted in buckets of 1/8
 * in log2 of the steps), each group needing 64 records per step of its longest
 * particle, for as many groups as fit.  The direction, position and energy
 * gradients are the same bits with any replay_steps (the grid gradient equal
 * to the order of its atomic sums).  Returns 0 for invalid arguments (n < 0,
 * K outside [1, 4096], replay_steps < 0). */
size_t crp_adjoint_replay_workspace_bytes(int64_t n, int32_t every_k, int64_t replay_steps);

/* Reverse-mode derivatives of the taped forward run (FP64).  The map
 * differentiated replays the forward pass's accepted steps (their sizes held
 * fixed) from the checkpoints, segment by segment from the last; the sphere
 * crossing in the last step is differentiated through its defining equation
 * |x - c| = R (implicit function theorem).  Inputs: the single field and
 * parameter group of the forward run; `initial` = the particles' state before
 * the forward run (raw direction, energy, charge); the cotangents gbar_dir
 * ([dev] n x 3) of the final direction and gbar_time ([dev] n, per second) of
 * the arrival time; gbar_energy ([dev] n, may be NULL) of the final energy,
 * which equals the initial one.  Outputs: grad_u0 ([dev] n x 3, written) with
 * respect to the initial direction (as given, before normalisation),
 * grad_x0 ([dev] n x 3, written, may be NULL), grad_energy ([dev] n, written,
 * may be NULL) with respect to the initial energy in eV: the rigidity
 * derivative (section 3.3: rigidity sets the deflection), kappa-bar * (-kappa /
 * E) with kappa = Z K / E and kappa-bar the cotangent of kappa summed over
 * every stage of the replay, plus gbar_energy; and grad_field ([dev]
 * [n0][n1][n2][3] of grad_dtype, CRP_F64 or CRP_F32, accumulated: the caller
 * zeroes it) with respect to the grid values in nG.  The contributions are
 * summed in FP64 per cell and added to grad_field with atomics of its type;
 * an FP32 gradient halves its memory and its atomic traffic.  Particles without a complete tape get zero gradients.
 * A backtracked run (params->backtrack = 1) is differentiated as the forward
 * run of the antiparticle it is: gradients and cotangents refer to the
 * physical directions of the input and output, as crp_propagate reads and
 * writes them.  In a reflective box (params->reflect = 1) the replay mirrors
 * where the forward run mirrored, and the mirrors are held fixed like the
 * step sizes: on each mirrored axis the position and direction cotangents
 * change sign (x -> 2 face - x, u -> -u).  The box faces themselves get no
 * gradient.  This is the derivative of the replayed map.  In a field-free box
 * it equals that of the forward run, and so it does for particles that never
 * reflect; for particles that reflect in a field it can differ from the
 * forward run's own derivative by large factors (mirrors act at step ends,
 * and next to a face the forward run's step sizes follow the state, so its
 * result depends on the whole step sequence).  A modulated field (section 3.2, modulated grids: B = b m) is
 * differentiated through both factors: grad_field is the gradient with
 * respect to the vector grid's values (its cotangent carries the factor m);
 * the modulation grid's own values get none.
 * Chaotic trajectories amplify cotangents exponentially; a contribution to
 * grad_field that is not finite in grad_dtype is left out (so grad_field
 * stays finite), and
 * a particle with such a contribution or a non-finite gradient gets
 * CRP_TAPE_GRAD_OVERFLOW in its tape flags (finals[4 i + 3], written by this
 * call).  Its grid contributions are then incomplete: to obtain grad_field
 * of the other particles exactly, zero the flagged particles' cotangents and
 * call again (the autograd wrapper does this).
 * workspace: [dev] at least crp_adjoint_workspace_bytes(n, K) bytes, 256-aligned;
 * what a larger workspace holds beyond that (see
 * crp_adjoint_replay_workspace_bytes) is used for parallel replay. */
crp_status crp_propagate_adjoint(const crp_field *field, const crp_params *params, const crp_particles *initial,
                                 int64_t n, const crp_tape *tape, const double *gbar_dir, const double *gbar_time,
                                 const double *gbar_energy, double *grad_u0, double *grad_x0,
                                 double *grad_energy, void *grad_field, int32_t grad_dtype, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* A captured propagation (hipGraph): the whole sequence of crp_propagate for
 * these exact arguments (descriptor tables, queue reset, longest-first order,
 * persistent kernel), replayed by crp_graph_launch with no host-side work.
 * Built for launch-bound repetition, e.g. many field realisations run again
 * and again (section 3.2: the same fields reused across runs).  Every pointer
 * captured must stay valid while the graph is used; each replay propagates
 * the particles' current state in place (callers reset it between replays if
 * they want the same input).  stream must be a non-default stream. */
typedef struct crp_graph crp_graph;
crp_status crp_graph_create(const crp_field *fields, int32_t n_fields, const crp_params *params, int32_t n_params,
                            const crp_particles *p, int64_t n, int32_t precision, const crp_tuning *tuning,
                            int64_t *counters, void *workspace, size_t workspace_bytes, void *stream,
                            crp_graph **out);
crp_status crp_graph_launch(crp_graph *g, void *stream);
crp_status crp_graph_destroy(crp_graph *g);

/* Device arithmetic conformance: apply operation op to n inputs in[] ([dev]
 * FP64) writing out[] ([dev] FP64).  op: 0 sqrt, 1 reciprocal (1/x), 2 fma(x, y,
 * z) on triples (n triples, in has 3n values), 3 floor, 4 the controller's
 * fifth root x^(-1/5), 5 the controller's shrink factor 1/sqrt(sqrt(x)), 6 the
 * quotient x/y on pairs (n pairs, in has 2n values).  Used to check that the
 * device rounds exactly like the host. */
crp_status crp_selftest_arith(const double *in, double *out, int64_t n, int32_t op, void *stream);

/* Gather microbenchmark (measurement only): lanes threads each perform
 * lookups_per_lane independent field lookups, with the propagation kernel's
 * layout, dtype and FP64 trilinear arithmetic (section 3.2: the lookup cost of
 * regular grids), at pseudo-random positions: uniform over the periodic box
 * when spread <= 0, else a cloud of standard deviation ~spread Mpc around the
 * origin.  sink: [dev] double[lanes], receives a checksum per lane.  Gives
 * the achievable lookup rate that bounds the propagation kernel. */
crp_status crp_bench_gather(const crp_field *f, int64_t lanes, int64_t lookups_per_lane, double spread,
                            uint64_t seed, double *sink, void *stream);

/* Replayed-lookup microbenchmark (measurement only): lanes threads each walk
 * a recorded stream of steps rec ([dev] FP64, layout [step][7][lane]: x, y,
 * z, ux, uy, uz of the state before the step and the step size h) and look
 * the field up at the six Cash-Karp stage points x + c_i h u of every step
 * (c = 0, 1/5, 3/10, 3/5, 1, 7/8), with the propagation kernel's lookup and,
 * if cache_cells = 1, its per-lane cell cache (section 3.2: the lookup cost
 * of regular grids).  The lookups do not depend on one another: the
 * achievable lookup rate for the cell sequences of real trajectories.  sink:
 * [dev] double[lanes] checksums; misses: [dev] int64[lanes] lookups that read
 * grid memory, or NULL.  F64 or F32 grids. */
crp_status crp_bench_gather_replay(const crp_field *f, const double *rec, int64_t lanes, int64_t steps,
                                   int32_t cache_cells, double *sink, int64_t *misses, void *stream);

/* Streaming microbenchmark (measurement only): reads bytes of src ([dev],
 * 16-byte aligned, bytes a multiple of 16) with blocks x 256 threads; copies
 * them to dst ([dev]) when dst is not NULL, else writes per-thread sums to
 * sink ([dev] double[blocks*256]).  A transfer of known size, used for the
 * bandwidth ceiling and to calibrate hardware byte counters. */
crp_status crp_bench_stream(const void *src, void *dst, size_t bytes, double *sink, int32_t blocks, void *stream);

/* ---- Lenses (section 3.3, the lensing technique of PARSEC) ----------------
 * For one rigidity, particles traced back from Earth (crp_propagate with
 * backtrack = 1, the observer sphere standing for the galactic border) give a
 * sparse matrix over sky pixels that maps cosmic-ray directions at the border
 * to the directions observed at Earth; arrival distributions are transformed
 * by matrix-vector products.  Pixels are HEALPix (Gorski et al. 2005, ApJ
 * 622:759) in the RING numbering, npix = 12 nside^2. */

/* Pixel of each direction (ux, uy, uz)[i]: any non-zero finite length, -1
 * for a zero or non-finite one.  1 <= nside <= 8192.  ux, uy, uz, pix: [dev]
 * n entries.  FP64 decision: z = uz/|u| and phi = atan2(uy, ux) in [0, 2 pi)
 * select the ring and the pixel in it.  Asynchronous on stream. */
crp_status crp_healpix_pixels(int32_t nside, const double *ux, const double *uy, const double *uz, int64_t n,
                              int32_t *pix, void *stream);

/* Workspace of crp_lens_build for nside and n launches (0 if out of range). */
size_t crp_lens_workspace_bytes(int32_t nside, int64_t n);

/* Lens of one rigidity from n backtracked launches.
 *   row: [dev] observed pixel of each launch, in [0, npix) (the pixel of the
 *        direction the particle was observed to come from, i.e. of the
 *        reversed velocity given to the backtracking run);
 *   ux, uy, uz, status: [dev] that run's output; a launch with status
 *        CRP_ST_ARRIVED adds to the entry at the pixel of its reversed
 *        velocity (the direction it came from at the border); every launch
 *        counts in its row's denominator;
 *   row_ptr: [dev] npix + 1 entries; col, val: [dev] capacity >= n entries;
 *        out: CSR with val[e] = (launches of row i reaching the border from
 *        pixel col[e]) / (launches of row i), FP64 ratio rounded to FP32,
 *        columns ascending within a row;
 *   nnz: [host] out, the number of entries (the call waits for the stream).
 * 1 <= nside <= 1024; any number of launches per row; a row whose launches
 * reach more than 4096 distinct border pixels gives CRP_ERR_UNSUPPORTED, a
 * row index out of range CRP_ERR_INVALID (both found
 * on the device, reported after the wait). */
crp_status crp_lens_build(int32_t nside, const int32_t *row, const double *ux, const double *uy, const double *uz,
                          const int32_t *status, int64_t n, int64_t *row_ptr, int32_t *col, float *val,
                          int64_t capacity, int64_t *nnz, void *workspace, size_t workspace_bytes, void *stream);

/* Lens application y = L x for nvec maps at once: y[i][v] = sum over the
 * entries e of row i of val[e] * x[col[e]][v], summed in FP64, stored FP32.
 * x, y: [dev] npix x nvec, pixel-major.  row_ptr, col, val: [dev] a lens as
 * crp_lens_build writes it (every col in [0, npix): the caller's to ensure);
 * nnz its entry count; 1 <= nvec <= 4096.  Allocates nothing; asynchronous. */
crp_status crp_lens_apply(int32_t nside, const int64_t *row_ptr, const int32_t *col, const float *val, int64_t nnz,
                          const float *x, float *y, int32_t nvec, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *crp_last_error(void);

/* Library version string. */
const char *crp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CRP_H */
