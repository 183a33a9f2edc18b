/*
 * tdpt.h -- C ABI of the MI355X (gfx950) two-dimensional parallel tempering
 * library.
 *
 * The method (Delacour, Sajeeb, Hespanha, Camsari, "Two-dimensional
 * Parallel Tempering for Constrained Optimization"):
 *   - an I x J grid of replicas; row i has inverse temperature beta_i, column
 *     j penalty strength P_j; the energy of a replica in column j is
 *     E_j = f + P_j g  (Eq. 1), g >= 0 the constraint function;
 *   - every replica performs Monte Carlo sweeps, then E and g are taken
 *     from the final state and one swap direction is tried (Algorithm 1):
 *     P-swaps between neighbouring columns of a row accept with
 *     min(1, exp(beta dP dg)) (Eq. 2), beta-swaps between neighbouring rows
 *     of a column with min(1, exp(dbeta dE)) (Eq. 3); pairs alternate
 *     between odd and even left indices and the direction flips after every
 *     even round; the bottom-right replica (largest beta and P) carries the
 *     answer.
 *   - the constraint is the copy constraint of graph sparsification,
 *     g = sum over copy edges (S_a - S_b)^2 (section on graph sparsification
 *     with copy constraints), or any sum of squared integer linear forms
 *     g = sum_t (sum_i a_ti S_i + d_t)^2 (tdpt_instance_create_terms), which
 *     holds equality constraints such as one-hot groups and capacity limits
 *     with slack spins (the constraint kinds named in the introduction).
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - Q12 fixed point: couplings J_q, fields b_q and penalties P_q are int32
 *     holding value * 2^12; f_q, E_q are int64 in the same scale, g is the
 *     integer sum of (s_a - s_b)^2 (4 per violated copy edge).
 *     f_q = -sum_{i<j} J_q[ij] s_i s_j - sum_i b_q[i] s_i.
 *   - Sweep: heat-bath updates colour class by colour class (ascending),
 *     P(s_i = +1) = 1 / (1 + exp(-2 beta h_i)) with
 *     h_i = sum_j J_ij s_j + b_i + 2 P sum_{copy neighbours k} s_k, or with
 *     general constraints h_i = sum_j J_ij s_j + b_i + 2 P c_i,
 *     c_i = -sum_t a_ti (sum_{j != i} a_tj s_j + d_t) (-s_i 2 c_i collects
 *     the terms of g that depend on s_i).
 *   - Random numbers: Philox4x32-10 keyed by the 64-bit seed; the counter of
 *     every draw is a function of (spin, sweep, grid position) or (pair,
 *     round, line, direction) only, so results do not depend on launch
 *     shape, batching or checkpoints.  Decisions are the double-precision
 *     expressions 2^32 u-threshold (heat bath) and u53 <= exp(x) (swaps).
 *   - Grid positions are row-major: p = i * J + j.  Outputs are reported per
 *     position; spins use the caller's original numbering.
 *
 * Errors: every int-returning call returns TDPT_OK or one of TDPT_E_*; the
 * message of the last failure on the calling thread is tdpt_last_error().
 * No call aborts or throws across the ABI.
 *
 * Threads and streams: an instance is immutable after creation and may be
 * shared.  A problem is bound to the stream given at creation; run calls
 * enqueue work on it and return without waiting; read/query calls wait for
 * that stream.  A problem must not be used from two threads at once.
 */
#ifndef TDPT_H
#define TDPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDPT_OK 0
#define TDPT_E_INVALID 1 /* malformed instance, schedule or argument */
#define TDPT_E_RANGE 2   /* fixed-point bounds exceeded (see tdpt_problem_create) */
#define TDPT_E_NOMEM 3   /* workspace too small / host allocation failed */
#define TDPT_E_DEVICE 4  /* HIP runtime error (code in the message) */
#define TDPT_E_STATE 5   /* call out of order: a batch whose member was destroyed or moved
                            to another batch, a histogram or logical read the problem was
                            not set up for */
#define TDPT_E_BUSY 6    /* the problem's batch has a run in flight (run, load, autotune) */

/* Flags of tdpt_run_cfg.flags */
#define TDPT_NO_PSWAP 1u /* J-column PT: no P-swaps; every round tries beta-swaps,
                            pair parity alternating every round */

typedef struct tdpt_instance tdpt_instance;
typedef struct tdpt_problem tdpt_problem;
typedef struct tdpt_batch tdpt_batch;

/* Run configuration (Algorithm 1 inputs). */
typedef struct tdpt_run_cfg {
    int32_t n_beta;          /* I >= 1 */
    const double *beta;      /* [I], strictly ascending, > 0, finite */
    int32_t n_p;             /* J >= 1 */
    const int32_t *p_q;      /* [J], Q12, non-decreasing, >= 0 */
    int32_t mcs_per_swap;    /* sweeps per swap round, >= 1 */
    uint64_t seed;           /* Philox key */
    const int8_t *s0;        /* nullable; [I*J*n] +-1, position-major, original spin
                                order; NULL draws every spin uniformly from the seed */
    int32_t has_target;      /* nonzero: record the first sweep at which the
                                bottom-right replica has g == 0 and f_q <= f_target_q */
    int64_t f_target_q;
    uint32_t flags;          /* TDPT_NO_PSWAP */
    int64_t trace_cap;       /* keep (f_q, g) of the bottom-right replica for the
                                first trace_cap rounds; 0 keeps none */
    int32_t hist_logical;    /* nonzero: after every round's swap step, count the
                                bottom-right replica's logical state in a device
                                histogram (the sampling measurement of Fig. 2; the
                                instance needs logical_of with at most 20 variables) */
} tdpt_run_cfg;

typedef struct tdpt_instance_info {
    int32_t n;          /* physical spins */
    int32_t n_pad;      /* colour-major padded length (classes rounded up to 4) */
    int32_t n_colors;
    int32_t max_degree; /* problem neighbours per spin (ELL width) */
    int32_t max_copy_degree;
    int32_t narrow;     /* 1 if problem indices and couplings fit 16 bits (packed layout; general-constraint rows stay 32-bit) */
    int64_t nnz;        /* directed problem couplings */
    int32_t m;          /* copy edges */
    int32_t n_terms;    /* general constraint terms (0 with copy edges) */
    int32_t max_constraint_degree; /* most spins one spin shares a term with */
    int32_t n_logical;  /* logical variables named by logical_of, 0 if none was given */
} tdpt_instance_info;

typedef struct tdpt_status {
    int64_t rounds_done;     /* swap rounds completed */
    int64_t sweeps_done;     /* rounds_done * mcs_per_swap */
    int64_t first_hit_sweep; /* -1 if the target was not reached (or no target) */
    int64_t best_f_q;        /* best feasible f_q seen at the bottom-right, INT64_MAX if none */
    int64_t best_sweep;      /* sweep count at which best_f_q was recorded, -1 if none */
    int32_t driver;          /* 1: one cooperative launch runs many rounds with every
                                replica resident in LDS; 0: one launch pair per round */
    int32_t slots;           /* per-round launches: replicas per sweep workgroup */
    int32_t spin;            /* per-round launches: 1 if one spin per lane (else one quad) */
} tdpt_status;

/* ---------------------------------------------------------------- instance */

/* Validate an Ising instance with copy constraints and lay it out for the
 * device (host memory only; nothing is allocated on the GPU).  Eq. 1 with
 * the copy constraint of the section on graph sparsification; the inputs
 * are Algorithm 1's problem instance.
 *   n           physical spins (> 0)
 *   row_ptr     [n+1] CSR offsets of the problem couplings, row_ptr[0] == 0
 *   col, J_q    [row_ptr[n]] neighbour index and Q12 coupling; the matrix must
 *               be symmetric (both directions present with equal values), with
 *               no self loops and no repeated neighbour in a row
 *   b_q         [n] Q12 fields, or NULL for zero
 *   m, copy_a, copy_b   copy-constraint edges (a != b, no repeats, not also a
 *               problem coupling); the constraint is g = sum (s_a - s_b)^2
 *   color       [n] colour class of every spin (>= 0); must be proper over
 *               problem and copy edges (a spin shares no class with any neighbour)
 *   logical_of  [n] or NULL: the logical variable (0 .. N-1, each used) each
 *               physical spin is a copy of.  A logical variable is read from
 *               its lowest-numbered copy (tdpt_problem_read_best_logical, the
 *               histogram of tdpt_run_cfg.hist_logical); on a state with g = 0
 *               every copy of a chain agrees.
 * At most 256 problem neighbours and 2 copy neighbours per spin, at most 32
 * colour classes.
 * All arrays are read during the call only.  On success *out owns a host
 * object released by tdpt_instance_destroy.  Returns TDPT_E_INVALID with a
 * message naming the first violation. */
int tdpt_instance_create(int32_t n, const int32_t *row_ptr, const int32_t *col,
                         const int32_t *J_q, const int32_t *b_q, int32_t m,
                         const int32_t *copy_a, const int32_t *copy_b,
                         const int32_t *color, const int32_t *logical_of,
                         tdpt_instance **out);

/* The same with a general constraint function in place of copy edges (Eq. 1
 * asks only g >= 0 with g = 0 exactly on feasible states):
 *   g = sum_{t < n_terms} (sum_{e = term_ptr[t]}^{term_ptr[t+1]-1}
 *                          term_coef[e] s[term_idx[e]] + term_const[t])^2.
 * An equality constraint sum_i w_i x_i = c on bits x = (1 + s) / 2 is the
 * term with coefficients w and constant sum_i w_i - 2c (its square is
 * 4 (w.x - c)^2); a copy edge is (1, -1) with constant 0, so copy chains
 * given this way run the same trajectory as through tdpt_instance_create.
 *   n_terms     >= 0; term_ptr [n_terms+1] offsets, term_ptr[0] == 0
 *   term_idx    spin of each entry (a spin at most once per term)
 *   term_coef   integer coefficient of each entry, term_const [n_terms]
 *   color       must be proper over the couplings and over every pair of
 *               spins whose expanded weight -sum_t a_ti a_tj is nonzero
 * Other arguments as tdpt_instance_create.  Such instances always use int8
 * replicas (no bit-packed replicas), so one replica must fit the LDS of a
 * workgroup; their constraint rows are 32-bit, their problem rows packed as
 * 16-bit pairs when indices and couplings allow it and the spin has at most
 * 8 problem neighbours.  Returns TDPT_E_INVALID for malformed
 * terms or a spin that shares terms with more than 1024 others, and
 * TDPT_E_RANGE if an expanded weight exceeds int32 or g could reach 2^62.
 * tdpt_problem_create bounds |h| by sum |J_q| + |b_q| + 2 P_q max_i |c_i|
 * and |E| by sum |J_q| + |b_q| + P_q max g. */
int tdpt_instance_create_terms(int32_t n, const int32_t *row_ptr, const int32_t *col,
                               const int32_t *J_q, const int32_t *b_q, int32_t n_terms,
                               const int32_t *term_ptr, const int32_t *term_idx,
                               const int32_t *term_coef, const int32_t *term_const,
                               const int32_t *color, const int32_t *logical_of,
                               tdpt_instance **out);
int tdpt_instance_info_get(const tdpt_instance *inst, tdpt_instance_info *out);
void tdpt_instance_destroy(tdpt_instance *inst);

/* Structure layout a problem of this instance and configuration runs with
 * (host only).  Problems of one batch whose group_key is equal share one
 * sweep kernel launch per round; a batch holds one group per key. */
typedef struct tdpt_layout {
    int32_t bits;       /* 1: replicas as bits, 4 per workgroup (replicas above 48 KiB as int8) */
    int32_t narrow;     /* 1: 16-bit packed structure rows */
    int32_t general;    /* 1: general constraint terms, 0: copy edges */
    int32_t ell_width;  /* problem-neighbour slots per spin in the device structure */
    int32_t group_key;  /* bits | narrow << 1 | (narrow && general) << 2 | ell_width << 3 |
                           pair16 << 12 */
    /* default launch shape of the per-round sweep (int8 replicas): */
    int32_t slots;      /* replicas per workgroup: 64 / lanes below 64 lanes (slots within
                           64 KiB of LDS), else 1 */
    int32_t lanes;      /* lanes per replica (0: one workgroup per replica at one quad per
                           lane): with spin, the power of two (>= 4) covering the largest
                           colour class's spins; else, when that class takes under 64
                           quads, the power of two (>= 4) covering its quads and the
                           per-phase bounds */
    int32_t held;       /* 1: the packed sweep holds each lane's structure in registers for
                           a round (one spin per lane: 2 to 4 colour classes; one quad per
                           lane: two classes, <= 4 neighbours and no fields) */
    int32_t per_round;  /* 1: tdpt_problem_create picks per-round launches over the
                           persistent driver (held, and mcs_per_swap >= 16) */
    int32_t spin;       /* 1: one spin per lane (packed copy-edge layout, <= 8 neighbours,
                           largest class <= 256 spins, the problem's round within 2048
                           waves, so latency-bound) */
    int32_t pair16;     /* 1: bit-packed replicas in pair form (two replicas per 32-bit word,
                           their coupling sums in 16-bit halves): every spin's sum of
                           2 |J_q| over its problem neighbours below 2^15 (environment
                           TDPT_PAIR16=0 turns it off) */
} tdpt_layout;
int tdpt_layout_get(const tdpt_instance *inst, const tdpt_run_cfg *cfg, tdpt_layout *out);

/* ---------------------------------------------------------------- problem */

/* Device bytes a problem needs (structure, all replica states, energies,
 * counters, tracking and trace) for an instance and Algorithm 1's run inputs
 * (the grid of beta and P values, sweeps per swap).  The caller allocates them (e.g. a torch
 * uint8 tensor) and passes the pointer to tdpt_problem_create. */
int tdpt_workspace_bytes(const tdpt_instance *inst, const tdpt_run_cfg *cfg, size_t *bytes);

/* Create a problem -- one run of Algorithm 1: the instance, the ordered beta
 * and P ladders, sweeps per swap and the initial spins -- in a caller-owned
 * device workspace (>= tdpt_workspace_bytes,
 * 256-byte aligned, on the current HIP device) and initialise it on `stream`
 * (a hipStream_t; NULL is the default stream): the workspace is cleared on
 * the device, the structure, ladders and any caller states are copied in,
 * and the call returns once the initial energies are computed (it waits for
 * the stream).  The instance may be destroyed afterwards.  The workspace must stay
 * allocated until tdpt_problem_destroy.  Returns TDPT_E_RANGE if a local
 * field could reach 2^31 in magnitude (sum |J_q| + |b_q| + 2 P_q * copy
 * degree) or an energy difference 2^52, or if an instance whose replica
 * exceeds 48 KiB as int8 (the bit-packed layout) has a coupling with
 * |J_q| >= 2^23 or a penalty P_q >= 2^22.  Returns TDPT_E_INVALID if such an instance has more than
 * 8 problem neighbours on a spin, or if one replica does not fit the LDS of
 * a workgroup. */
int tdpt_problem_create(const tdpt_instance *inst, const tdpt_run_cfg *cfg, void *dev_ws,
                        size_t ws_bytes, void *stream, tdpt_problem **out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation): the
 * same as tdpt_problem_create with the workspace taken from a static device
 * array of the library, TDPT_STATIC_WORKSPACE_BYTES per GPU, which each GPU
 * the library runs on holds until the process ends.  The call allocates no
 * device memory.  One such problem per GPU at a time: TDPT_E_BUSY while
 * another lives on the current device (tdpt_problem_destroy releases the
 * array after the problem's stream has finished); TDPT_E_NOMEM if the
 * problem's tdpt_workspace_bytes exceed the array.  Creation clears the part
 * of the array the problem uses, so nothing of an earlier holder leaks in. */
#define TDPT_STATIC_WORKSPACE_BYTES (64u << 20)
int tdpt_problem_create_static(const tdpt_instance *inst, const tdpt_run_cfg *cfg, void *stream,
                               tdpt_problem **out);

/* Enqueue n_rounds swap rounds of Algorithm 1 (each: mcs_per_swap sweeps of
 * every replica, f/g of the final states, one swap step by Eq. 2 or Eq. 3,
 * bottom-right tracking).  Resumable: calling it twice with a and b rounds
 * equals one call with a + b.  TDPT_E_BUSY if the problem's batch has a run
 * in flight; TDPT_E_RANGE past 2^32 sweeps.
 * Driver (tdpt_status.driver; results never depend on it): the persistent
 * one -- one cooperative launch runs all n_rounds, replicas resident in LDS
 * and exchanging through mailboxes -- when every replica's workgroup fits
 * the GPU at once, except for small replicas whose lanes hold their
 * structure in registers for a round (tdpt_layout.held: one spin per lane
 * and 2 to 4 colour classes, or one quad per lane, two classes, at most 4
 * neighbours and no fields) and whose rounds hold 16 sweeps or more: those run per-round
 * launches (tdpt_layout.per_round).  Per-round sweeps of small int8
 * replicas take one spin per lane while the problem's round is within 2048
 * waves (latency-bound; tdpt_status.spin), else one quad per lane, several
 * replicas per workgroup when the largest colour class takes under 64
 * lanes (tdpt_status.slots).  Otherwise one sweep launch and one swap
 * launch per round.  The environment variable
 * TDPT_PERSISTENT=0 at creation forbids the persistent driver, =1 prefers it
 * wherever it fits; tdpt_problem_autotune may change the choice. */
int tdpt_problem_run(tdpt_problem *prob, int64_t n_rounds);

/* Read calls wait for the problem's stream (and so for any batch run that
 * holds it) and write host memory the caller owns; the _async variants
 * enqueue the same data on the problem's stream into device memory the
 * caller owns (on the problem's device) and return at once. */

/* Counters and tracking: rounds and sweeps done; the first sweep at which
 * the bottom-right replica was feasible (g == 0) with f_q <= f_target_q (the
 * planted ground state of the Wishart study: the residual energy of Fig. 3
 * is read at the bottom-right replica); its best feasible f_q and sweep. */
int tdpt_problem_query(tdpt_problem *prob, tdpt_status *out);
/* dev_words[4] = rounds_done, first_hit_sweep, best_f_q, best_sweep. */
int tdpt_problem_query_async(tdpt_problem *prob, int64_t *dev_words);

/* E and g of the final state of every grid position's replica, the values
 * the swap step compares (Eq. 2, Eq. 3): f_q[R], g[R] per position
 * (R = I*J, row-major); either pointer may be NULL (not both). */
int tdpt_problem_read_energies(tdpt_problem *prob, int64_t *f_q, int64_t *g);
int tdpt_problem_read_energies_async(tdpt_problem *prob, int64_t *dev_f_q, int64_t *dev_g);
/* s[R*n] per position, original spin order. */
int tdpt_problem_read_states(tdpt_problem *prob, int8_t *s);
int tdpt_problem_read_states_async(tdpt_problem *prob, int8_t *dev_s);
/* pos_to_slot[R]: which internal replica slot sits at each position (a swap
 * exchanges the labels of two positions, never their spins). */
int tdpt_problem_read_perm(tdpt_problem *prob, int32_t *pos_to_slot);
/* Best feasible bottom-right state (Algorithm 1 stores the last replica's
 * spins after each swap step), original order, its f_q and sweep.  Any
 * pointer may be NULL. */
int tdpt_problem_read_best(tdpt_problem *prob, int8_t *s, int64_t *f_q, int64_t *sweep);
/* dev_s[n] (may be NULL) and dev_f_sweep[2] = best_f_q, best_sweep (may be NULL). */
int tdpt_problem_read_best_async(tdpt_problem *prob, int8_t *dev_s, int64_t *dev_f_sweep);
/* The same state decoded to its logical variables x[N] (+-1, each read from
 * its lowest-numbered copy); TDPT_E_STATE without logical_of. */
int tdpt_problem_read_best_logical(tdpt_problem *prob, int8_t *x, int64_t *f_q, int64_t *sweep);
/* Swap attempts/accepts: P pairs [I*(J-1)] indexed (row, left column), beta
 * pairs [J*(I-1)] indexed (column, upper row).  Any pointer may be NULL. */
int tdpt_problem_read_counters(tdpt_problem *prob, int64_t *p_att, int64_t *p_acc,
                               int64_t *b_att, int64_t *b_acc);
/* Bottom-right (f_q, g) of rounds 1..min(rounds_done, trace_cap). */
int tdpt_problem_read_trace(tdpt_problem *prob, int64_t *f_q, int64_t *g, int64_t *count);
/* The logical-state histogram of the bottom-right replica (hist_logical):
 * counts[2^N], bin sum_k [x_k = +1] 2^k, one sample per round done
 * (*samples, may be NULL).  TDPT_E_STATE if the run did not ask for it. */
int tdpt_problem_read_histogram(tdpt_problem *prob, uint32_t *counts, int64_t *samples);

/* Checkpoint (not a step of the paper; it makes long runs resumable): copy
 * the whole mutable device state to host memory.  With
 * host == NULL only *bytes is set.  tdpt_problem_load restores it into a
 * problem created from the same instance and configuration; a run resumed
 * from it is bit-identical to an uninterrupted one. */
int tdpt_problem_save(tdpt_problem *prob, void *host, size_t *bytes);
int tdpt_problem_load(tdpt_problem *prob, const void *host, size_t bytes);  /* TDPT_E_BUSY as run */

/* Release the handle (the caller frees the workspace afterwards).  A batch
 * member is first taken out of its batch, after the batch's work in flight;
 * that batch then needs tdpt_batch_set_members before its next run. */
void tdpt_problem_destroy(tdpt_problem *prob);

/* Measurement hook (not a step of the paper): from now on record a pair of
 * HIP events on the problem's stream around every `every`-th launch of the
 * sweep kernel (the per-round sweep kernel, or the persistent kernel that
 * runs many rounds); at most 4096 pairs; 0 switches it off and clears what
 * was recorded. */
int tdpt_problem_set_timing(tdpt_problem *prob, int32_t every);
/* Wait for the stream and report the summed duration (ms) of the timed
 * launches, how many were timed and how many swap rounds they covered. */
int tdpt_problem_read_timing(tdpt_problem *prob, double *total_ms, int64_t *launches,
                             int64_t *rounds);

/* Measurement hook of the persistent driver: from the next round on, for
 * `rounds` rounds, every replica slot writes four timestamps of the GPU's
 * 100 MHz real-time clock into dev_buf[round][slot][0..3] (caller-owned
 * device memory of rounds * R * 4 uint64, on the problem's device): the
 * round's start, the end of its sweeps, the moment the swap partner's
 * (f, g) is in hand (= the end of the sweeps when the slot has no partner
 * that round), and the end of the swap decision.  0 switches it off.  The
 * per-round driver records nothing.  Waits for the problem's stream. */
int tdpt_problem_set_stage_trace(tdpt_problem *prob, uint64_t *dev_buf, int32_t rounds);

/* Launch-shape autotuner (not a step of the paper: launch shapes never
 * change results).  Times each admissible (driver, threads per sweep
 * workgroup, replicas per workgroup) on the problem itself -- one warm-up
 * round, then rounds_per_trial rounds between HIP events on the problem's
 * stream -- and keeps the fastest for later runs.  Candidates: the per-round
 * driver at 64 to 1024 threads (768 for bit-packed replicas with fewer than
 * 4 sweeps per round, whose sweeps follow f and g per update), for int8
 * replicas of a small largest colour class also several replicas per
 * workgroup of 64, 128 or 256 threads (one to four passes over the class)
 * and one spin per lane (one or two passes), and, where every replica's
 * workgroup can be resident at once, the
 * persistent driver at 64 to 512, each no larger than the largest colour
 * class needs and no smaller than the per-phase 2^31 bounds allow.  The problem's state is saved before and
 * restored after (the trial rounds leave no trace); since random numbers do
 * not depend on launch shape, results after tuning equal those without.
 * Blocks the calling thread until the trials finish. */
typedef struct tdpt_tune_report {
    int32_t driver;              /* chosen: 1 persistent, 0 per-round */
    int32_t block;               /* chosen threads per sweep workgroup */
    double ms_per_round;         /* its measured time per round */
    int32_t n_trials;            /* candidates timed (<= 32), in this order: */
    int32_t trial_driver[32];
    int32_t trial_block[32];
    double trial_ms_per_round[32];
    int32_t slots;               /* chosen replicas per workgroup (per-round driver) */
    int32_t trial_slots[32];
    int32_t spin;                /* chosen: 1 one spin per lane, 0 one quad per lane */
    int32_t trial_spin[32];
} tdpt_tune_report;
int tdpt_problem_autotune(tdpt_problem *prob, int32_t rounds_per_trial, tdpt_tune_report *out);

/* ---------------------------------------------------------------- batches */

/* A batch advances many problems at once (many independent Algorithm 1
 * runs): every round is one sweep launch over all replica slots of all
 * members (grouped by structure layout, tdpt_layout.group_key, the largest
 * instances first) and one swap-and-track launch over all members, so
 * problems of uneven size and grid share the GPU.  Results are identical to
 * running each member alone (random streams are keyed per problem).
 * Members are ordinary problems; their own streams are ordered after every
 * batch run, so their read calls see its results.  While a batch run that
 * holds a problem is in flight, running, loading or autotuning that problem
 * returns TDPT_E_BUSY.  A problem belongs to at most one batch: naming it
 * in another batch's member list takes it out of the first, which then
 * needs tdpt_batch_set_members before it runs again (TDPT_E_STATE).
 *
 * Continuous batching with these calls: admitting a problem or retiring one
 * is tdpt_batch_set_members with the new list (at a round boundary: the
 * call waits for the work in flight); launching is tdpt_batch_run (returns
 * at once); polling is tdpt_batch_query (every member's first_hit_sweep,
 * rounds_done, best f at once) or tdpt_problem_query per member. */

/* Device bytes of the descriptor table of a batch with up to max_members. */
int tdpt_batch_workspace_bytes(int32_t max_members, size_t *bytes);
/* Create a batch in a caller-owned device workspace (256-byte aligned, at
 * least tdpt_batch_workspace_bytes) bound to `stream`. */
int tdpt_batch_create(int32_t max_members, void *dev_ws, size_t ws_bytes, void *stream,
                      tdpt_batch **out);
/* Replace the member list (count <= max_members, no repeats; count 0 empties
 * the batch).  Waits for pending work of the members and the batch.  On
 * failure the batch is left empty (no member). */
int tdpt_batch_set_members(tdpt_batch *batch, tdpt_problem *const *probs, int32_t count);
/* Enqueue n_rounds rounds of every member on the batch's stream.
 * TDPT_E_STATE if a member was destroyed or moved since set_members. */
int tdpt_batch_run(tdpt_batch *batch, int64_t n_rounds);
/* Poll every member at once: words[count][4] (in the order of the last
 * tdpt_batch_set_members) = rounds_done, first_hit_sweep, best_f_q,
 * best_sweep, as tdpt_problem_query reports them; one kernel and one copy
 * instead of a read per member.  Waits for the batch's stream.  The _async
 * form enqueues the same words into caller device memory on that stream. */
int tdpt_batch_query(tdpt_batch *batch, int64_t *words);
int tdpt_batch_query_async(tdpt_batch *batch, int64_t *dev_words);
/* Autotune the launch shape of each layout group of the current members,
 * one group after another, timing whole batch rounds; every member's state
 * is restored afterwards.  Candidates: one replica per workgroup of 64 to
 * 1024 threads (768 for bit-packed groups with a member of fewer than 4
 * sweeps per round; no smaller than the members' per-phase bounds allow),
 * run by the persistent driver where it fits; and, for int8 groups whose
 * largest colour class is small, several replicas per workgroup of 64, 128
 * or 256 threads (a power-of-two share of lanes each, one to four passes
 * over the class) and one spin per lane (one or two passes), run by
 * per-round launches.  Without tuning, per-round launches take one spin per
 * lane while the batch's round is within 2048 waves, else pack the
 * replicas of int8 groups whose largest class takes under 64 lanes, one
 * wave of 64 threads per workgroup.  The choice
 * holds until the next tdpt_batch_set_members; a packed choice keeps the
 * batch on per-round launches. */
typedef struct tdpt_batch_tune_report {
    int32_t persistent;                /* 1 if the tuned batch runs the persistent driver */
    int32_t n_groups;                  /* layout groups (<= 32) */
    int32_t group_block[32];           /* chosen threads per workgroup */
    double group_ms_per_round[32];     /* batch round time with that choice */
    int32_t n_trials;                  /* (group, shape) pairs timed (<= 128) */
    int32_t trial_group[128];
    int32_t trial_block[128];
    double trial_ms_per_round[128];
    int32_t group_slots[32];           /* chosen replicas per workgroup */
    int32_t trial_slots[128];
    int32_t group_spin[32];            /* chosen: 1 one spin per lane */
    int32_t trial_spin[128];
} tdpt_batch_tune_report;
int tdpt_batch_autotune(tdpt_batch *batch, int32_t rounds_per_trial, tdpt_batch_tune_report *out);
/* Driver of a batch.  By default (-1) tdpt_batch_run uses the persistent
 * driver -- per layout group one cooperative launch that runs all the
 * rounds, every member's replicas resident at once and exchanging through
 * their own mailboxes -- whenever every member allows it (int8 layout,
 * persistent driver not switched off) and each group's workgroups fit the
 * GPU together, unless every member is a replica of the kind that runs
 * per-round launches on its own (tdpt_problem_run: structure held in
 * registers, rounds of 16 sweeps or more);
 * otherwise one sweep launch per group and one swap launch per round.  0
 * forces the per-round launches.  Results are the same either way.  tdpt_batch_query_driver reports the current choice (1 persistent). */
int tdpt_batch_set_driver(tdpt_batch *batch, int32_t driver);
int tdpt_batch_query_driver(tdpt_batch *batch, int32_t *driver);
/* Replay rounds from a HIP graph: with rounds_per_graph = k > 0, the launches
 * of k rounds (every group's sweep, the swap step) are captured once into a
 * graph -- kernel launches only, on a private non-blocking stream -- and
 * tdpt_batch_run enqueues floor(n / k) replays of it on the batch's stream,
 * then the remaining rounds directly.  0 (the default) launches every round
 * directly.  The graph is rebuilt after tdpt_batch_set_members or
 * tdpt_batch_autotune; results are the same either way.  Graphs apply to the
 * per-round driver; the persistent driver needs one launch per group anyway. */
int tdpt_batch_set_graph(tdpt_batch *batch, int32_t rounds_per_graph);  /* per-round driver only */
void tdpt_batch_destroy(tdpt_batch *batch);

/* Thread-local message of the last failed call ("" if none). */
const char *tdpt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TDPT_H */
