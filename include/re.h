/*
 * re.h -- C ABI of the replica-exchange Lennard-Jones molecular-dynamics
 * engine for AMD Instinct MI355X (gfx950).
 *
 * Method: G. Bussi, "A simple asynchronous replica-exchange implementation".
 * Many replicas of a Lennard-Jones liquid (Example section: cutoff, neighbour
 * list with a half-skin update trigger, time step, thermostat) run at the
 * temperatures of a ladder; ladder neighbours exchange temperatures -- not
 * coordinates -- by the Metropolis rule, and accepted swaps scale the
 * velocities (Implementation section).  Exchanges may be synchronous (every
 * replica attempts after the same number of steps; Implementation section,
 * last paragraph) or asynchronous (a rotating master triggers each attempt
 * after N_x of its own steps, the others join at their next step boundary;
 * Implementation section, the three-step iteration).
 *
 * Units are Lennard-Jones reduced units: m = sigma = epsilon = k_B = 1.
 *
 * Conventions for every function below:
 *   - all pointers are HOST pointers to caller-owned memory; inputs are copied
 *     during the call, outputs are written during the call;
 *   - a replica index r is 0 <= r < R; atom arrays of one replica are in
 *     atom-id order, 3 doubles per atom (x, y, z);
 *   - every query synchronises the context's stream before returning;
 *   - a context is not thread-safe: one caller thread at a time;
 *   - return value 0 is success, negative values are the RE_E* codes; the
 *     message of the last failure is available from re_last_error.
 */
#ifndef RE_H_
#define RE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RE_OK 0
#define RE_EINVAL (-1)   /* bad argument (see each function) */
#define RE_ENOMEM (-2)   /* device or host allocation failed */
#define RE_EDEVICE (-3)  /* a HIP runtime error; see re_last_error */
#define RE_ETIMEOUT (-4) /* a device-side wait timed out; state is left at a step boundary */
#define RE_ESTATE (-5)   /* call not valid in the current state / mode */
#define RE_EOVERFLOW (-6)/* a neighbour list or cell exceeded its capacity */

/* thermostat */
#define RE_LANGEVIN 0 /* BAOAB Langevin, friction gamma (gamma = 0: velocity Verlet, NVE) */
#define RE_SVR 1      /* velocity Verlet + stochastic velocity rescaling (the thermostat of the
                         Example section; Bussi, Donadio, Parrinello, J. Chem. Phys. 126,
                         014101 (2007)): once per step, at the step boundary, every velocity
                         of a replica is multiplied by sqrt(K'/K), K' drawn from the
                         rescale's exact update with N_f = 3N - 3 and relaxation time
                         svr_tau; gamma is ignored.  The rescale needs a replica-wide
                         sum at the end of every step, so the next step's first half
                         cannot be fused into the force phase: slower than Langevin. */
/* precision / form */
#define RE_MIXED 0 /* positions as 32-bit periodic fixed point, FP32 pair arithmetic,
                      FP32 velocities; FP64 energy sums and rescale factors */
#define RE_FP64 1  /* FP64 positions, velocities and arithmetic throughout */
#define RE_BATCHED 0    /* all replicas advanced together on the device */
#define RE_PLAIN 1      /* one sequence of kernel launches per replica per step */
#define RE_LOCKSTEP 0   /* batched: one launch sequence per step for all replicas */
#define RE_PERSISTENT 1 /* batched: one persistent launch per re_step call.  The
                           workgroups serving one replica wait for each other
                           (team barriers, exchange partners), so every
                           workgroup of the launch must be resident at once:
                           the engine sizes its grid to the resident capacity
                           of the device (one 1024-thread workgroup per CU)
                           and assumes it has the GPU to itself.  Kernels of
                           other processes or streams that occupy CUs during
                           a call can keep a team from becoming resident; the
                           watchdog then ends the call with RE_ETIMEOUT
                           instead of hanging. */
/* exchange timing */
#define RE_SYNC 0  /* attempt after every N_x steps of every replica */
#define RE_ASYNC 1 /* rotating master triggers after N_x of its own steps */
/* persistent engine team barrier */
#define RE_BARRIER_AUTO 0  /* one-XCD release for teams that share an L2 */
#define RE_BARRIER_AGENT 1 /* agent-scope release and acquire always */

typedef struct re_ctx re_ctx; /* opaque; owned by the library until re_destroy */

/* Optional settings.  A zero-initialised struct (or NULL) means defaults. */
typedef struct {
    int thermostat;              /* RE_LANGEVIN (default) | RE_SVR                */
    double gamma;                /* Langevin friction; 0 selects NVE. Default: when
                                    gamma_set == 0, gamma = 1.0                   */
    int gamma_set;               /* nonzero: use the gamma field as given          */
    int precision;               /* RE_MIXED (default) | RE_FP64                   */
    int form;                    /* RE_BATCHED (default) | RE_PLAIN                */
    int batched_engine;          /* RE_PERSISTENT (default) | RE_LOCKSTEP          */
    int exchange_mode;           /* RE_SYNC (default) | RE_ASYNC                   */
    const double* rho_per_replica; /* R densities; NULL: the scalar rho for all   */
    void* stream;                /* hipStream_t to run on; NULL: a library stream  */
    double watchdog_seconds;     /* bound on every device-side wait; 0: 10 s       */
    int64_t log_capacity;        /* exchange records kept (ring); 0: 1 << 18       */
    int threads_per_atom;        /* force-kernel lanes per atom (1, 2, 4 or 8);
                                    0: 4, or the autotuner's choice when
                                    autotune is set                        */
    int block_size;              /* threads per block of the wide kernels; 0: auto */
    int team_size;               /* persistent engine: workgroups per replica; 0: auto */
    const char* tune_cache;      /* autotuner JSON cache path; NULL: no cache file */
    int autotune;                /* nonzero: choose the batched engine, the
                                    lockstep block size and the force lanes per
                                    atom by timing short runs of each candidate
                                    on throwaway contexts of the same workload
                                    (or take the choice from tune_cache): first
                                    one lane count for all replicas, then, for
                                    ladders whose replicas fall into several
                                    size classes (floor(log2 N)), a lane count
                                    per class where that is at least 2 % faster;
                                    explicit engine / block / lane settings are
                                    then ignored */
    int team_barrier;            /* persistent engine's barrier between the
                                    workgroups of one replica: RE_BARRIER_AUTO
                                    (default) lets a team whose workgroups all
                                    run on one XCD (read on the device) release
                                    through their shared L2 without an L2
                                    write-back; RE_BARRIER_AGENT always uses
                                    agent-scope release and acquire          */
    double svr_tau;              /* RE_SVR relaxation time (LJ units); 0: 0.5     */
    int exchange_max_distance;   /* non-nearest-neighbour exchanges (Implementation
                                    section): attempt k pairs ladder slots
                                    (j, j+d), d = 1 + (w mod D) from Philox
                                    counter (k, 0, purpose 5), j >= o = (k mod 2) d
                                    with floor((j - o)/d) even; D = 0 or 1: the
                                    alternating nearest-neighbour pattern    */
    int debug_delay_us;          /* test hook, persistent engine: after team
                                    barriers, workgroups picked by a hash of
                                    (workgroup, step, site) pause for up to
                                    this many microseconds, so that tests can
                                    check that results do not depend on the
                                    timing of the members; 0 = off         */
    const int32_t* threads_per_atom_per_replica;
                                 /* R values (1, 2, 4 or 8): force lanes per atom
                                    of each replica (its force pass and list
                                    layout), overriding threads_per_atom; the
                                    kernels then choose per replica (per block
                                    in the lockstep engine, per team in the
                                    persistent one).  NULL: threads_per_atom
                                    for every replica.  With autotune, the
                                    tuner may set it per size class
                                    (floor(log2 N)); see re_query_lanes   */
    int team_balance;            /* persistent engine with automatic team sizes:
                                    nonzero re-plans the teams once every
                                    replica has done 500 steps since the last
                                    plan, weighting replica r by
                                    N_r (1 + 4 u_r), u_r its list updates per
                                    step in that window (hot replicas update
                                    more often; with equal teams the others
                                    wait for them at synchronous exchanges);
                                    results do not depend on the teams.
                                    0 (default): teams proportional to N */
} re_options;

/* One record per ladder pair per exchange attempt. */
typedef struct {
    int64_t attempt;  /* global attempt index k (pairs slots j, j+d; d = 1: j = k mod 2) */
    int32_t master;   /* replica that triggered the attempt (async) or -1 (sync)  */
    int32_t slot_lo;  /* lower ladder slot j of the pair                          */
    int32_t rep_a;    /* replica that held slot j                                 */
    int32_t rep_b;    /* replica that held slot slot_hi                           */
    int64_t step_a;   /* step count of rep_a when it joined the attempt           */
    int64_t step_b;   /* step count of rep_b when it joined the attempt           */
    double U_a, U_b;  /* potential energies at those steps (FP64)                 */
    double T_a, T_b;  /* ladder temperatures T_j, T_{slot_hi}                     */
    double u;         /* uniform of the lower replica id (53-bit Philox)          */
    int32_t accepted; /* 1 if the temperatures were swapped                       */
    int32_t slot_hi;  /* upper ladder slot j + d of the pair                      */
} re_xlog_rec;

/*
 * Create R replicas.  N_atoms[r] >= 2 atoms each, on an FCC start at density
 * rho (or rho_per_replica[r]) in a periodic cube of side (N/rho)^(1/3)
 * rounded to a multiple of 2^-12; velocities Maxwell-Boltzmann at the ladder
 * temperature T_ladder[r] (strictly ascending, > 0), total momentum removed,
 * kinetic temperature exact with 3N-3 degrees of freedom.  Replica r starts
 * in ladder slot r.  r_c: LJ cutoff (truncated and energy-shifted); skin:
 * neighbour-list skin (list radius r_c + skin, updated when one atom moved
 * more than skin/2; Example section); dt: time step; N_x: exchange stride
 * (Implementation section); seed: Philox4x32-10 key.
 * Errors: RE_EINVAL for R < 1, any N < 2, a non-ascending or non-positive
 * ladder, rho <= 0, r_c <= 0, skin < 0, dt <= 0, N_x < 1, r_c + skin >= L/2
 * for some replica, or a replica whose neighbour-list block (with the rows
 * read past it) would reach 2^32 bytes (its words are addressed with 32-bit
 * byte offsets); RE_ENOMEM; RE_EDEVICE.  *out is NULL on failure.
 */
int re_create(re_ctx** out, int R, const int32_t* N_atoms, const double* T_ladder,
              double rho, double r_c, double skin, double dt, int N_x, uint64_t seed,
              const re_options* opt);

/*
 * Advance the run (Implementation section).  RE_SYNC: every replica advances
 * exactly n steps, with an exchange attempt whenever the common step count
 * reaches a multiple of N_x.  RE_ASYNC: returns once every replica has done
 * at least n more steps; a replica that reaches n keeps stepping (and
 * exchanging) until the last one does, so no replica idles and the step
 * counts differ; attempts are triggered by the rotating master; a replica
 * that is paired waits for its partner.  n >= 0.
 * Errors: RE_EINVAL (n < 0), RE_ETIMEOUT (a device-side wait exceeded the
 * watchdog bound; the run stops at a consistent step boundary), RE_EOVERFLOW,
 * RE_EDEVICE.
 */
int re_step(re_ctx* ctx, int64_t n);

/* One synchronous exchange attempt now, at every replica's current step
 * (the next attempt index).  Errors: RE_EDEVICE. */
int re_exchange(re_ctx* ctx);

/* Potential energy of each replica at its current step boundary (FP64,
 * replica order, R values). */
int re_query_energies(re_ctx* ctx, double* U);

/* Temperature currently held by each replica (R values). */
int re_query_temps(re_ctx* ctx, double* T);

/* Ladder slot currently held by each replica (R values). */
int re_query_slots(re_ctx* ctx, int32_t* slot);

/* Attempts and acceptances per ladder pair by its lower slot j (pairs
 * (j, j+1), or (j, j+d) with non-nearest-neighbour exchanges): R-1 values each. */
int re_query_acceptance(re_ctx* ctx, int64_t* attempts, int64_t* accepts);

/* Steps done and neighbour-list updates per replica (R values each). */
int re_query_steps(re_ctx* ctx, int64_t* steps, int64_t* rebuilds);

/* Exchange attempts made so far (the global attempt index of the next
 * attempt), counting attempts that pair no replica. */
int re_query_attempt_count(re_ctx* ctx, int64_t* n);

/* Box side of each replica (R values). */
int re_query_box(re_ctx* ctx, double* L);

/* Copy out up to cap of the most recent exchange records, oldest first;
 * *n_out receives the number copied, *n_total (may be NULL) the number ever
 * recorded.  Errors: RE_EINVAL for cap < 0. */
int re_query_exchange_log(re_ctx* ctx, re_xlog_rec* buf, int64_t cap, int64_t* n_out,
                          int64_t* n_total);

/* Positions (wrapped into [-L/2, L/2)) and full-step velocities of replica r
 * in atom-id order (3N doubles each; either pointer may be NULL).  The
 * velocities are those after every rescale of the current step boundary
 * (exchange factor sqrt(T_new/T_old), thermostat rescale), even where the
 * device applies the factor only with the next step. */
int re_get_state(re_ctx* ctx, int r, double* x, double* v);

/* Replace positions and velocities of replica r (atom-id order, 3N doubles
 * each; positions are wrapped into the box and rounded to the working
 * precision).  The neighbour list is rebuilt (counted as an update) and the
 * forces recomputed; the step count is kept.  Errors: RE_EINVAL. */
int re_set_state(re_ctx* ctx, int r, const double* x, const double* v);

/* Forces (3N doubles, atom-id order) and potential energy of replica r at its
 * current positions; changes no state.  Either output may be NULL. */
int re_compute_forces(re_ctx* ctx, int r, double* F, double* U);

/* Forces (3N doubles, atom-id order) on replica r at its current step
 * boundary as the engine that ran last computed them: the final force phase
 * of the last re_step (the persistent kernel's own force pass when that
 * engine runs), or the list update after re_create / re_set_state.  Truncated
 * and shifted LJ at cutoff r_c (Example section).  Reads no positions and
 * recomputes nothing.  Errors: RE_EINVAL (bad r or NULL F). */
int re_query_forces(re_ctx* ctx, int r, double* F);

/* Asynchronous mode only, for testing: fix the join steps of the next A
 * attempts instead of letting device timing decide.  join is A x R (row a:
 * the step at which each replica takes part in attempt a); each row must be
 * >= the previous one (and the current step counts) element-wise.  The next
 * re_step runs exactly those attempts and stops at the last row.
 * Errors: RE_EINVAL, RE_ESTATE (not in RE_ASYNC mode). */
int re_set_schedule(re_ctx* ctx, const int64_t* join, int64_t A);

/* The device exchange rule on given inputs, for testing: replica r holds
 * slot[r] (a permutation of 0..R-1) and energy U[r]; T is the ladder.
 * Runs attempt number `attempt` of the pattern with the given largest
 * distance (1: alternating nearest neighbours) on the GPU and writes
 * decisions[j] for each pair by its lower slot j (0 or 1; R-1 entries, slots
 * that are not the lower slot of a pair get 255).  Needs no context.
 * Errors: RE_EINVAL, RE_EDEVICE. */
int re_test_exchange(const double* U, const double* T, const int32_t* slot, int R,
                     uint64_t seed, int64_t attempt, int max_distance, uint8_t* decisions);

/* re_test_exchange for callers that cannot allocate device memory (code
 * under HIP graph capture, tight driver loops, harnesses that forbid
 * hipMalloc): the same arguments, rule and results, but the device staging
 * of U, T, slot and the decisions is a fixed array inside the library (one
 * per GPU, 84 KiB, held until the process ends) instead of allocations.  It
 * runs on the current device and the null stream, and calls no allocating
 * routine.  Limit: R <= 4096 (RE_EINVAL beyond, with the limit named).
 * Calls that overlap on one GPU (from several host threads) share that
 * array and race; serialise them.  Errors: RE_EINVAL, RE_EDEVICE. */
int re_test_exchange_noalloc(const double* U, const double* T, const int32_t* slot, int R,
                             uint64_t seed, int64_t attempt, int max_distance, uint8_t* decisions);

/* Device random numbers, for testing (no context needed).
 * re_test_philox: n Philox4x32-10 blocks (Salmon et al., SC'11) of the
 * counters ctr[4i .. 4i+3] under key (key0, key1) into out[4i .. 4i+3].
 * re_test_normals: n triples of standard normals, the Box-Muller transform
 * of the Philox block of counter ctr[4i .. 4i+3] under key `seed`, as the
 * integrator draws them (fp64 = 0: the FP32 form, 1: the FP64 form), into
 * out[3i .. 3i+2].  Errors: RE_EINVAL (n < 0 or NULL), RE_EDEVICE. */
int re_test_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, int n, uint32_t* out);
int re_test_normals(int fp64, uint64_t seed, const uint32_t* ctr, int n, double* out);

/* Measurement of the dominant kernel (the fused force + integrate launch of
 * the batched lockstep engine; the persistent launch of the persistent
 * engine), timed with HIP events on the context's stream.  re_profile(ctx, 1)
 * opens a window (at most 4096 launches are timed), re_profile(ctx, 0) closes
 * it; re_query_kernel_time gives the number of launches timed in the last
 * window and their mean duration in milliseconds. */
int re_profile(re_ctx* ctx, int enable);
int re_query_kernel_time(re_ctx* ctx, double* mean_ms, int64_t* n);

/* The launch configuration the context runs with (after autotuning):
 * engine (RE_LOCKSTEP | RE_PERSISTENT; RE_PLAIN form: RE_LOCKSTEP),
 * threads_per_atom (0 when it differs between replicas; see
 * re_query_lanes), and the persistent team size of replica 0 (0 when the
 * persistent engine is not available). */
int re_query_config(re_ctx* ctx, int* engine, int* threads_per_atom, int* team_size);

/* Force lanes per atom of each replica (R values). */
int re_query_lanes(re_ctx* ctx, int32_t* tpa);

/* Persistent engine: workgroups serving each replica in the current plan
 * (R values; 0 when the persistent engine is not available). */
int re_query_teams(re_ctx* ctx, int32_t* team);

/* Free everything owned by the context (NULL is allowed). */
void re_destroy(re_ctx* ctx);

/* Message of the last failure on ctx, or of the last failure of a call that
 * had no context (ctx == NULL).  Valid until the next call on ctx. */
const char* re_last_error(const re_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RE_H_ */
