/*
 * liblabs -- batched tabu search and memetic tabu search for Low
 * Autocorrelation Binary Sequences (LABS) on AMD Instinct MI355X (gfx950).
 *
 * The problem and the method follow Z. Zhang, J. Shen et al., "New
 * Improvements in Solving Large LABS Instances Using Massively Parallelizable
 * Memetic Tabu Search", arXiv:2504.00987.  Citations name the paper's
 * sections, equations, algorithms and tables.
 *
 * Conventions for every entry point
 *   - Sequences are int8 rows of +1/-1 (the spins s_i of Sec. II), row-major
 *     with a caller-given row stride in bytes (stride >= N).  Entries of a row
 *     beyond its length N are ignored on input and written as 0 on output.
 *   - Lengths satisfy LABS_MIN_N <= N <= LABS_MAX_N.
 *   - Energies are E(s) = sum_{k=1}^{N-1} C_k(s)^2 with
 *     C_k(s) = sum_{i=1}^{N-k} s_i s_{i+k} (Eq. 1, Eq. 2): exact int32.
 *   - "device" pointers are HIP device allocations (for example the
 *     data_ptr() of a torch tensor on the GPU); "host" pointers are ordinary
 *     process memory.  The caller owns every buffer it passes; the library
 *     never frees or retains caller memory after the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls documented as asynchronous only enqueue work on `stream`; their
 *     outputs are valid after the stream is synchronised.
 *   - Every call returns a labs_status.  Nothing throws or aborts across the
 *     ABI.  On failure, labs_last_error(h) holds a message; for LABS_E_HIP it
 *     names the HIP error.  Invalid arguments are rejected before any work is
 *     enqueued.
 *   - Randomness is Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit
 *     seed; every draw is addressed by (entity, generation, index, purpose),
 *     so results are a pure function of (seed, parameters, inputs, item
 *     index) and do not depend on the stream, batch composition, launch
 *     configuration or execution mode.
 *   - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef LIBLABS_H
#define LIBLABS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LABS_MIN_N 3
#define LABS_MAX_N 256
#define LABS_MAX_K 128 /* largest memetic population */

typedef enum labs_status {
    LABS_OK = 0,
    LABS_E_INVAL = 1,     /* an argument is out of range or a pointer is NULL */
    LABS_E_NOMEM = 2,     /* a device or pinned host allocation failed */
    LABS_E_HIP = 3,       /* a HIP runtime call failed */
    LABS_E_CANCELLED = 4, /* the request was cancelled */
    LABS_E_NOTFOUND = 5,  /* unknown request id */
    LABS_E_AGAIN = 6      /* the result is not ready yet */
} labs_status;

/* Walk length (maxIter) rule. */
typedef enum labs_steps_rule {
    LABS_STEPS_FIXED = 0,  /* maxIter = steps_a */
    LABS_STEPS_MULT_N = 1, /* maxIter = steps_a * N */
    LABS_STEPS_PAPER = 2,  /* maxIter = randomInt(0, N) + floor(N/2), Alg. 4 */
    /* maxIter uniform in [floor(slo_num*N/slo_den), floor(shi_num*N/shi_den)]
     * (both ends inclusive), from word 0 of the draw (walk, generation, 0,
     * LEN) as lo + ((w0 * (hi - lo + 1)) >> 32); Sec. III.B states the walk
     * length as randInt[N/2, 3N/2], which is RANGE(1/2, 3/2) and equals
     * LABS_STEPS_PAPER at every N */
    LABS_STEPS_RANGE = 3
} labs_steps_rule;

/* Tabu tenure rule: a move flipped at step t is tabu for steps
 * t+1 .. t+tenure, tenure uniform in [minTabu, maxTabu] (Alg. 2). */
typedef enum labs_tenure_rule {
    /* minTabu = floor(lo_num*N/lo_den) + lo_add,
     * maxTabu = floor(hi_num*N/hi_den) + hi_add */
    LABS_TENURE_LINEAR = 0,
    /* minTabu = floor(0.1*maxIter), maxTabu = floor(0.12*maxIter) (Sec. III.B) */
    LABS_TENURE_PAPER = 1
} labs_tenure_rule;

/* Parameters of one tabu walk (Alg. 2 / Alg. 4).  Valid when, for every N
 * used, 0 <= minTabu <= maxTabu < N (so some move is always admissible) and
 * 0 <= maxIter <= LABS_MAX_STEPS. */
typedef struct labs_tabu_params {
    int32_t steps_rule;  /* labs_steps_rule */
    int32_t steps_a;
    int32_t tenure_rule; /* labs_tenure_rule */
    int32_t lo_num, lo_den, lo_add;
    int32_t hi_num, hi_den, hi_add;
    int32_t aspiration;  /* 1: a tabu move is admissible when its energy is
                            strictly below the walk's best (not in the paper;
                            0 gives the paper's rule) */
    int32_t slo_num, slo_den, shi_num, shi_den; /* LABS_STEPS_RANGE bounds
                            (den > 0, num >= 0; ignored by the other rules) */
} labs_tabu_params;

#define LABS_MAX_STEPS (1 << 20)

/* Launch configuration of the batched walk kernels.  Lanes per walk =
 * group_lanes / walks_per_group: 64 (one wavefront per walk: {64, 1},
 * {128, 2}, {256, 4}), 128 ({128, 1}: the walks of 64 < N <= 128 run on
 * two wavefronts each, exchanging their minima through LDS; the batch's
 * other walks run one per wavefront, two per 128-lane workgroup), or 32 /
 * 16 ({64, 2} and {128, 4}: the walks of N <= 32 run two per wavefront, 32
 * lanes each; {64, 4}: those of N <= 16 four per wavefront and those of
 * 16 < N <= 32 two; the batch's longer walks run one per wavefront, one or
 * two per workgroup).  Four wavefronts per walk, and two walks of two
 * wavefronts in one workgroup ({256, 1}, {256, 2}), are not built
 * (LABS_E_INVAL). */
typedef struct labs_launch {
    int32_t group_lanes;     /* 64, 128 or 256 lanes per workgroup */
    int32_t walks_per_group; /* 1, 2 or 4 */
    int32_t persistent;      /* 1: a grid sized to the device drains a
                                longest-first work queue; 0: one walk per
                                wavefront (or per two) of the grid */
    int32_t groups_per_cu;   /* persistent grid = groups_per_cu x CUs (0: auto) */
    int32_t layout;          /* walks of 64 < N <= 128: 0 default (record form
                                on one wavefront, lag form on two), 1 lag form
                                (t_jk rows, 18.5 KB of LDS per walk), 2 record
                                form (sequence windows, 9.5 KB) */
} labs_launch;               /* default (untuned): {64, 2, 0, 0, 0} when
                                every walk has N <= 32, {64, 1, 0, 0, 0} up to
                                N = 128, {256, 4, 0, 0, 0} above */

typedef struct labs_handle labs_handle;

/* Create a handle bound to HIP device `device` (ordinal).  The handle owns
 * its device workspace, pinned staging memory, internal stream, tuned
 * launch table and cached graphs.  Returns LABS_E_INVAL for a bad ordinal. */
int labs_create(labs_handle **out, int device);

/* Destroy a handle after synchronising its work.  NULL is accepted. */
int labs_destroy(labs_handle *h);

/* Message describing the handle's most recent failure ("" if none).  The
 * pointer stays valid until the next call on the handle. */
const char *labs_last_error(const labs_handle *h);

/* Name of a status code (static string). */
const char *labs_status_name(int status);

/* Library version string (static). */
const char *labs_version(void);

/*
 * Energies of a batch of sequences: Eq. (2) of Sec. II.
 *   seqs      device int8 [count][stride], +-1 in the first N entries of a row
 *   ns        device int32 [count] per-row lengths, or NULL to use n_uniform
 *   n_uniform length of every row when ns == NULL
 *   energies  device int32 [count] output
 * Asynchronous on `stream`.  With per-row lengths the kernel clamps nothing:
 * the caller guarantees LABS_MIN_N <= ns[b] <= min(stride, LABS_MAX_N).
 */
int labs_energy_batch(labs_handle *h, const int8_t *seqs, const int32_t *ns,
                      int32_t n_uniform, int32_t stride, int64_t count,
                      int32_t *energies, void *stream);

/*
 * Deviation from skew-symmetry d(S) of App. A for a batch of sequences: the
 * least number of broken pairs t_{c+i} != (-1)^i t_{c-i} (the condition of
 * Sec. II.C for odd length 2c + 1) over the rotations of S (first r elements
 * moved to the end) -- for even N, each rotation followed by the deletion
 * of one element.  (App. A also admits one insertion; its printed values
 * follow deletion only.)
 *   seqs      device int8 [count][stride], +-1 in the first N entries of a row
 *   ns        device int32 [count] per-row lengths, or NULL to use n_uniform
 *   d         device int32 [count] output
 * Asynchronous on `stream`; the caller guarantees LABS_MIN_N <= ns[b] <=
 * min(stride, LABS_MAX_N).  Work per row: N^2 (odd N) or N^3 (even N) / 2
 * pair tests.
 */
int labs_skew_deviation_batch(labs_handle *h, const int8_t *seqs, const int32_t *ns,
                              int32_t n_uniform, int32_t stride, int64_t count, int32_t *d,
                              void *stream);

/*
 * Exhaustive minimum of Eq. (2) over all 2^n sequences of length n
 * (3 <= n <= LABS_MAX_BRUTE_N), the reference targets for time-to-solution
 * at small n.  E is invariant under negation (Sec. II.B), so the 2^(n-1)
 * sequences with s_0 = +1 are enumerated.
 *   min_e   HOST int32: the minimum energy
 *   count   HOST int64 (or NULL): how many of the 2^n sequences attain it
 *   argmin  HOST int8 [n] (or NULL): of the minima with s_0 = +1, the one
 *           whose bit pattern (bit i set <=> s_i = -1) is the smallest
 *           integer
 * Synchronous (on the handle's stream).  Work grows like 2^n n: n = 36
 * takes about a second, n = 40 about fifteen.
 */
#define LABS_MAX_BRUTE_N 40
int labs_bruteforce_min(labs_handle *h, int32_t n, int32_t *min_e, int64_t *count,
                        int8_t *argmin);

/*
 * The search restricted to skew-symmetric sequences (Sec. II.C): for odd
 * n = 2c + 1, the exhaustive minimum of Eq. (2) over the 2^(c+1) sequences
 * with s_{c+i} = (-1)^i s_{c-i} (0-based, centre c), whose C_k vanish for odd
 * k.  The paper's point is that this subspace need not hold the optimum
 * (Sec. II.C, Sec. VI); comparing the result with labs_bruteforce_min shows
 * where it does not.  Negating every spin keeps a sequence skew-symmetric, so
 * the 2^c sequences with s_0 = +1 are enumerated.
 *   min_e   HOST int32: the minimum energy over the skew-symmetric subspace
 *   count   HOST int64 (or NULL): how many of its 2^(c+1) sequences attain it
 *   argmin  HOST int8 [n] (or NULL): of the attaining ones with s_0 = +1, the
 *           one whose free spins s_0..s_c (bit i set <=> s_i = -1) form the
 *           smallest integer
 * Synchronous (on the handle's stream); LABS_E_INVAL for even n or n outside
 * [3, LABS_MAX_SKEW_BRUTE_N].  Work grows like 2^(n/2) n: n = 75 takes about
 * a second.
 */
#define LABS_MAX_SKEW_BRUTE_N 75
int labs_skew_bruteforce_min(labs_handle *h, int32_t n, int32_t *min_e, int64_t *count,
                             int8_t *argmin);

/*
 * Independent tabu walks (Alg. 2; the thread-parallel form of Alg. 4, one
 * walk per 64-lane wavefront).  Walk w (0 <= w < walks) starts from row w
 * of `starts`, or -- when starts == NULL -- from the 128-bit draws
 * (w, 0, q, START): bit i % 128 of draw q = i / 128 set means s_i = -1.  Each of its maxIter steps
 * scores all N single-flip neighbours, takes the lowest-energy admissible
 * one (ties: uniform by the step's draw), marks it tabu for a random tenure
 * and keeps the best sequence visited (strict improvement).
 *   p             walk parameters (host pointer)
 *   starts        device int8 [walks][start_stride] or NULL
 *   ns_host       HOST int32 [walks] per-walk lengths, or NULL (n_uniform)
 *   seed          Philox key
 *   best_seq      device int8 [walks][out_stride] best sequence of each walk
 *   best_e        device int32 [walks] its energy
 *   final_e       device int32 [walks] energy of the last pivot
 *   trace         optional device int16 [walks][trace_stride]: the 0-based
 *                 index flipped at step t goes to trace[w][t-1]
 *                 (trace_stride >= the longest walk), or NULL
 * walks may be up to 2^31 - 1; batches whose grid would pass 2^30
 * work-items run as several launches, in order, on `stream`.
 * Asynchronous on `stream`; ns_host is read before the call returns.
 */
int labs_tabu_batch(labs_handle *h, const labs_tabu_params *p,
                    const int8_t *starts, int32_t start_stride,
                    const int32_t *ns_host, int32_t n_uniform, int64_t walks,
                    uint64_t seed, int8_t *best_seq, int32_t out_stride,
                    int32_t *best_e, int32_t *final_e, int16_t *trace,
                    int32_t trace_stride, void *stream);

/*
 * labs_tabu_batch for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, same results, but no device or pinned host memory is
 * allocated or freed by the call.  Its queue heads, per-walk lengths and
 * processing order live in a fixed device array of LABS_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device for the life of the process.
 *   ns_host   HOST int32 [walks] or NULL; with per-walk lengths at most
 *             LABS_NOALLOC_MAX_WALKS walks (LABS_E_INVAL beyond; a batch of
 *             one length has no limit).  The lengths are copied by a
 *             transfer enqueued on `stream`: keep the array unchanged until
 *             the stream has passed this call.
 * Every call on a device shares that device's array (the handle's side
 * streams run the length classes of a mixed batch): calls that overlap in
 * time on one device -- from any handle or stream -- race and must be
 * ordered by the caller.
 */
#define LABS_NOALLOC_MAX_WALKS 65536
#define LABS_NOALLOC_SCRATCH_BYTES (1024 + 8 * LABS_NOALLOC_MAX_WALKS)
int labs_tabu_batch_noalloc(labs_handle *h, const labs_tabu_params *p,
                            const int8_t *starts, int32_t start_stride,
                            const int32_t *ns_host, int32_t n_uniform, int64_t walks,
                            uint64_t seed, int8_t *best_seq, int32_t out_stride,
                            int32_t *best_e, int32_t *final_e, int16_t *trace,
                            int32_t trace_stride, void *stream);

/* Set (launch != NULL) or clear (NULL: back to the tuned/default choice) the
 * launch configuration used by labs_tabu_batch on this handle. */
int labs_set_launch(labs_handle *h, const labs_launch *launch);

/* The launch configuration labs_tabu_batch would use for a batch whose
 * lengths span [n_min, n_max]. */
int labs_get_launch(labs_handle *h, int32_t n_min, int32_t n_max, labs_launch *out);

/*
 * Autotuner: times the launch configurations that apply to the length range
 * [n_min, n_max] -- {64, 1}, {128, 2}, {256, 4} (one wavefront per walk);
 * when the range reaches 64 < N <= 128, {128, 1} (two wavefronts per walk);
 * when n_min <= 32, {64, 2} and {128, 4} (two walks per wavefront), and
 * when n_min <= 16 also {64, 4} (four) -- each with both layouts of the
 * walks of 64 < N <= 128 where they are present, and each
 * as a grid of one walk per wavefront (or pair) and as a persistent queue
 * at 1, 2, 4 and 8 x 4 / (wavefronts per group) groups per CU -- on `walks`
 * random-start walks with lengths spread evenly over [n_min, n_max] and
 * parameters `p` (each: one warm-up call, then four calls back to back).
 * The default runs first until the GPU is at its steady clock (at least 16
 * calls and 25 ms), and stays unless a configuration is more than 2 % faster.
 * The choice is kept for batches whose shortest and longest lengths fall in
 * the length buckets (of 16) of n_min and n_max, so that tuning one range
 * leaves the others alone.  *tried (may be NULL) receives the number of
 * configurations timed.  Synchronous; results never depend on the choice
 * (only speed does).
 */
int labs_autotune(labs_handle *h, const labs_tabu_params *p, int32_t n_min,
                  int32_t n_max, int64_t walks, uint64_t seed, int32_t *tried);

/*
 * Measured throughput of the units the walk kernels are bound by (the
 * roofline's measured peaks; the published figures at 2.4 GHz are 157.3e12,
 * 39.3e12 and 78.6e12): v_dot4_i32_i8 int8 products per second (four per
 * lane per instruction), 32-bit integer adds per second, and bytes per
 * second of conflict-free 16-byte LDS reads; and the shader clock during
 * the dot-product load (its cycle counter against the 100 MHz constant
 * one).  Each is one timed launch of independent dependency chains on every
 * compute unit.  HOST outputs.  Synchronous (on the handle's stream); about
 * 3 ms.
 */
int labs_device_peaks(labs_handle *h, double *dot4_products_per_s, double *int32_ops_per_s,
                      double *lds_bytes_per_s, double *clock_hz);

/* Memetic search (Alg. 1; one replica per wavefront, Alg. 3). */
typedef enum labs_mut_rule {
    LABS_MUT_INV_N = 0, /* p_mutate = 1/N: flip when draw < floor(2^32 / N) */
    LABS_MUT_FIXED = 1  /* flip when draw < p_mut */
} labs_mut_rule;

typedef enum labs_exec_mode {
    LABS_MODE_PLAIN = 0,      /* one kernel launch per generation */
    LABS_MODE_GRAPH = 1,      /* a captured graph of `chunk` one-generation
                                 launches, replayed */
    LABS_MODE_PERSISTENT = 2  /* one launch runs `chunk` generations with the
                                 population resident on chip */
} labs_exec_mode;

typedef struct labs_memetic_params {
    int32_t K;           /* population size, 2..LABS_MAX_K (paper: 100) */
    uint32_t p_comb;     /* crossover when the draw < p_comb
                            (paper: 0.9 -> 3865470566) */
    int32_t mut_rule;    /* labs_mut_rule */
    uint32_t p_mut;      /* threshold for LABS_MUT_FIXED */
    labs_tabu_params tabu;
    int64_t generations; /* generations per replica */
    int32_t target_e;    /* a replica stops once its best energy <= target_e
                            (Alg. 1's loop condition); < 0 disables */
    int32_t mode;        /* labs_exec_mode */
    int32_t chunk;       /* generations between host checks (>= 1) */
    int32_t stop_all;    /* 1: once any replica reaches target_e, every
                            replica stops at the end of the current chunk
                            (the global termination flag of Sec. IV) */
    int32_t waves_per_replica; /* replicas with 64 < N <= 128: 1 or 2 wavefronts
                            (two split each step's neighbours and exchange
                            their minima: lower latency per generation, for
                            batches too small to fill the device); 0 picks
                            2 when those replicas number at most twice the
                            compute units */
    int32_t children;    /* children per generation, 1..8 (0 means 1).  1 is
                            Alg. 1 (steady state).  B > 1 is the batched-
                            generation variant: B children are made from
                            the population as it stands at the start of the
                            generation, walked concurrently (one wavefront
                            each), then merged in order b = 0..B-1 as Alg. 1
                            merges its one child; child b draws from
                            (replica, g, 2b | 2b+1, GEN), mutates with
                            (replica, g, 64b + i/4, MUT) and walks as
                            generation g*B + b.  Targets are checked once per
                            generation; hit_gen counts generations.  For
                            N > 128 a child's walk takes 17.7 KB of LDS, and
                            B is further limited to what one workgroup can
                            hold (LABS_E_INVAL beyond). */
    int32_t resume;      /* 1: continue the replicas this handle holds (left
                            by its last labs_memetic_run or put there by
                            labs_memetic_load) instead of drawing new
                            populations; pops, K, the lengths and the seed
                            must be those of the held state.  `generations`
                            stays the total per replica, so a run to G1 and a
                            resumed run to G give the results of one run to
                            G (with stop_all, when G1 is a multiple of
                            chunk). */
} labs_memetic_params;

#define LABS_MAX_CHILDREN 8
#define LABS_MAX_REPLICAS (1 << 22) /* replicas of one labs_memetic_run */

/*
 * Run `pops` independent memetic replicas (population id = index),
 * 0 <= pops <= LABS_MAX_REPLICAS.
 * Replica p: K members from the draws (p, m, q, INIT), bit i of member m
 * being bit i % 128 of draw q = i / 128 as for walk starts; per generation g,
 * crossover (binary-tournament parents, one-point cut) or sampling, per-bit
 * mutation, a tabu walk with entity p and generation g, strict best update
 * and replacement of a random member -- the order of Alg. 1.
 *   ns_host   HOST int32 [pops] per-replica lengths, or NULL (n_uniform)
 *   best_seq  device int8 [pops][out_stride] best sequence of each replica
 *   best_e    device int32 [pops]
 *   hit_gen   device int64 [pops]: children produced when best <= target
 *             first held (0: the initial population), -1 if never (or NULL)
 *   gens_done device int64 [pops]: generations executed (or NULL)
 * Asynchronous on `stream`: the population state lives in the handle's
 * device memory (a later run on any stream waits for this one on the GPU),
 * and every launch, copy and graph replay is enqueued on `stream`.  Chunk
 * boundaries (every `chunk` generations) carry a device-side stop flag: with
 * stop_all (Alg. 3's global termination flag) it is raised at the end of the
 * chunk in which the first replica reached the target, and every later
 * launch of the run does nothing.  Only then does the host wait: it reads
 * the flag back two chunks behind, on events of `stream`, to stop
 * enqueueing.  Without stop_all the call returns as soon as everything is
 * enqueued.  Returns LABS_E_CANCELLED when labs_cancel was called while the
 * call was still enqueueing; the outputs then hold each replica's state at
 * the chunk boundary where it stopped (gens_done < generations).
 */
int labs_memetic_run(labs_handle *h, const labs_memetic_params *p,
                     const int32_t *ns_host, int32_t n_uniform, int32_t pops,
                     uint64_t seed, int8_t *best_seq, int32_t out_stride,
                     int32_t *best_e, int64_t *hit_gen, int64_t *gens_done,
                     void *stream);

/*
 * Checkpoints of the memetic replicas a handle holds (after a
 * labs_memetic_run, also a cancelled one, or a labs_memetic_load): the
 * populations, their energies, each replica's best, generation count and hit
 * generation, and whether a replica has reached the target (the global flag
 * of Sec. IV).  The draws are counter-based, so no generator state is saved,
 * and a resumed run continues bit for bit (labs_memetic_params.resume).
 * The blob is host memory in a fixed layout: a 256-byte header (magic
 * "LABSMEM", version, pops, K, seed, the smallest generation count), the
 * per-replica lengths (int32, padded to 256 bytes), then the state arrays.
 *   labs_memetic_checkpoint_bytes  size of the blob for the held state
 *                                  (LABS_E_INVAL when the handle holds none)
 *   labs_memetic_save   copies the held state into `dst` (host, `bytes` >=
 *                       the size) after the work already on `stream`;
 *                       returns once the copy is complete
 *   labs_memetic_load   validates a blob (magic, version, sizes, lengths in
 *                       range) and makes it the held state, ordered on
 *                       `stream`; returns once `src` may be reused
 */
int labs_memetic_checkpoint_bytes(labs_handle *h, int64_t *bytes);
int labs_memetic_save(labs_handle *h, void *dst, int64_t bytes, void *stream);
int labs_memetic_load(labs_handle *h, const void *src, int64_t bytes, void *stream);

/*
 * Stop every labs_memetic_run of this handle that is running or still being
 * enqueued: each stops at its next chunk boundary (the device reads the
 * request from mapped host memory), and a call still enqueueing returns
 * LABS_E_CANCELLED.  Runs started after this call are not affected.  May be
 * called from any thread.
 */
int labs_cancel(labs_handle *h);

/*
 * Serving: a request loop that runs memetic solves of different N from a
 * stream of requests with continuous batching.  Requests wait in FIFO order
 * and are admitted as soon as enough resident population slots are free;
 * all admitted replicas advance together, `chunk` generations per kernel
 * launch, so requests that arrive while others run share the device.  A
 * request's result equals labs_memetic_run on the same (N, seed, pops,
 * params): the best of its replicas (lowest energy, then lowest replica id).
 * The server runs its own host thread and HIP stream.
 *   params     K, rules, target, chunk (generations/mode are per request)
 *   max_slots  resident replicas (device memory: about
 *              (K*36 + 64) bytes each); admission never exceeds it
 */
typedef struct labs_server labs_server;

int labs_server_create(labs_handle *h, const labs_memetic_params *params,
                       int32_t max_slots, labs_server **out);

/* Enqueue a solve of length n with `pops` replicas of `generations`
 * generations under `seed`.  *request_id receives the id.  Thread-safe. */
int labs_server_submit(labs_server *s, int32_t n, uint64_t seed, int32_t pops,
                       int64_t generations, int64_t *request_id);

/* Fetch a result: LABS_E_AGAIN while pending; LABS_OK with best_seq (HOST
 * int8 [n]), best_e and the latency in seconds (enqueue to completion)
 * once done.  A fetched result is released.  Thread-safe. */
int labs_server_poll(labs_server *s, int64_t request_id, int8_t *best_seq,
                     int32_t *best_e, double *latency_s);

/* Cancel a waiting or running request (its slots are freed at the next
 * chunk); polling it then returns LABS_E_CANCELLED.  Thread-safe. */
int labs_server_cancel(labs_server *s, int64_t request_id);

/* Counters: requests waiting, running, done; resident replicas. */
int labs_server_stats(labs_server *s, int64_t *waiting, int64_t *running,
                      int64_t *done, int64_t *resident);

/* Stop the loop (pending requests are dropped) and free the server. */
int labs_server_destroy(labs_server *s);

#ifdef __cplusplus
}
#endif

#endif /* LIBLABS_H */
