/*
 * labs_oracle.c -- plain CPU reference ("the oracle") for memetic tabu search
 * on Low Autocorrelation Binary Sequences (LABS).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct statement of
 * what the GPU library computes.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never calls
 * it and shares no code, header, table or helper with it.
 *
 * Paper: Z. Zhang, J. Shen, et al., "New Improvements in Solving Large LABS
 * Instances Using Massively Parallelizable Memetic Tabu Search",
 * arXiv:2504.00987.  Citations below name the paper's section, equation,
 * algorithm or table.
 *
 * Conventions
 *   - A sequence is int8_t s[0..n-1] with s_i in {-1,+1}; indices are 0-based
 *     (the paper is 1-based).
 *   - All arithmetic is exact integer arithmetic (int64 accumulators).
 *   - Randomness: every draw is Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed by the
 *     64-bit seed and addressed by a counter (entity, generation, index, tag).
 *     The paper only says that replicas use different seeds (Sec. IV); the
 *     counter layout below is this implementation's reading, written once and
 *     implemented independently on each side.
 *   - A uniform integer in [0, r) is drawn from a 32-bit word u as
 *     (u * r) >> 32.
 *
 * Parity pins: see tests/test_oracle_*.py.  Every function here is pinned by
 * at least one check that does not re-use this file's arithmetic.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* Longest sequence the walk and memetic routines accept. */
#define ORC_MAX_N 256

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from the published definition (SC'11, Sec. 2.3 / Fig. 2).   */
/* Round: (hi0,lo0) = M0*x0, (hi1,lo1) = M1*x2;                               */
/*        x' = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); the key is bumped by */
/*        the Weyl constants between rounds.                                  */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Purpose tags: the fourth counter word, one per kind of draw. */
enum {
    ORC_TAG_START = 1, /* random start of a stand-alone walk               */
    ORC_TAG_STEP  = 2, /* per tabu step: tie-break word, tenure word       */
    ORC_TAG_LEN   = 3, /* per walk: random walk length                     */
    ORC_TAG_INIT  = 4, /* per population member: initial sequence          */
    ORC_TAG_GEN   = 5, /* per generation: crossover/parents/cut/replacement */
    ORC_TAG_MUT   = 6  /* per generation: mutation words                   */
};

static void draw(uint64_t seed, uint32_t entity, uint32_t gen, uint32_t index,
                 uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = { entity, gen, index, tag };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

static uint32_t uniform_below(uint32_t u, uint32_t range)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)range) >> 32);
}

void orc_draw(uint64_t seed, uint32_t entity, uint32_t gen, uint32_t index,
              uint32_t tag, uint32_t out[4])
{
    draw(seed, entity, gen, index, tag, out);
}

/* ------------------------------------------------------------------------- */
/* Objective: Eq. (1) aperiodic autocorrelation, Eq. (2) energy.             */
/* ------------------------------------------------------------------------- */

/* C[k] = sum_{i=0}^{n-1-k} s_i s_{i+k} for k = 0..n-1 (Eq. 1; C[0] = n). */
void orc_autocorrelation(const int8_t *s, int n, int64_t *C)
{
    for (int k = 0; k < n; ++k) {
        int64_t c = 0;
        for (int i = 0; i + k < n; ++i)
            c += (int64_t)s[i] * (int64_t)s[i + k];
        C[k] = c;
    }
}

/* E(s) = sum_{k=1}^{n-1} C_k^2 (Eq. 2). */
int64_t orc_energy(const int8_t *s, int n)
{
    int64_t e = 0;
    for (int k = 1; k < n; ++k) {
        int64_t c = 0;
        for (int i = 0; i + k < n; ++i)
            c += (int64_t)s[i] * (int64_t)s[i + k];
        e += c * c;
    }
    return e;
}

/* Batch form of Eq. (2): energies of B sequences stored with a row stride. */
void orc_energy_batch(const int8_t *seqs, const int32_t *ns, int32_t n_uniform,
                      int32_t stride, int64_t B, int64_t *out)
{
    for (int64_t b = 0; b < B; ++b) {
        int n = ns ? ns[b] : n_uniform;
        out[b] = orc_energy(seqs + b * stride, n);
    }
}

/* Exhaustive minimum of Eq. (2) over all 2^n sequences (n <= 24), and the
 * number of sequences attaining it.  Every sequence is scored from Eq. (2)
 * directly; no symmetry is used. */
int orc_bruteforce_min(int n, int64_t *emin, int64_t *count)
{
    if (n < 1 || n > 24)
        return -1;
    int8_t s[24];
    int64_t best = -1, cnt = 0;
    uint32_t total = 1u << n;
    for (uint32_t code = 0; code < total; ++code) {
        for (int i = 0; i < n; ++i)
            s[i] = ((code >> i) & 1u) ? -1 : 1;
        int64_t e = orc_energy(s, n);
        if (best < 0 || e < best) {
            best = e;
            cnt = 1;
        } else if (e == best) {
            ++cnt;
        }
    }
    *emin = best;
    *count = cnt;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Skew-symmetric subspace (Sec. II.C).                                       */
/* ------------------------------------------------------------------------- */
/* The skew-symmetric sequence of odd length n = 2c + 1 whose free spins
 * s_0..s_c are given by code (bit i set <=> s_i = -1): the other half
 * follows from s_{c+i} = (-1)^i s_{c-i}, i = 1..c (Sec. II.C, 0-based with
 * the centre at c).  Returns -1 for even n or n outside [1, 63]. */
int orc_skew_sequence(int n, uint64_t code, int8_t *s)
{
    if (n < 1 || n > 63 || (n & 1) == 0)
        return -1;
    int c = (n - 1) / 2;
    for (int i = 0; i <= c; ++i)
        s[i] = ((code >> i) & 1u) ? -1 : 1;
    for (int i = 1; i <= c; ++i)
        s[c + i] = (int8_t)((i & 1) ? -s[c - i] : s[c - i]);
    return 0;
}

/* Exhaustive minimum of Eq. (2) over the 2^((n+1)/2) skew-symmetric
 * sequences of odd length n (n <= 45): the minimum, how many of them attain
 * it, and -- of those with s_0 = +1 -- the one whose free-spin code is the
 * smallest integer.  Every sequence is built by orc_skew_sequence and
 * scored from Eq. (2) directly; no symmetry is used. */
int orc_skew_bruteforce_min(int n, int64_t *emin, int64_t *count, int8_t *argmin)
{
    if (n < 1 || n > 45 || (n & 1) == 0)
        return -1;
    int8_t s[45];
    int c = (n - 1) / 2;
    int64_t best = -1, cnt = 0;
    uint64_t best_code = 0;
    uint64_t total = 1ull << (c + 1);
    for (uint64_t code = 0; code < total; ++code) {
        orc_skew_sequence(n, code, s);
        int64_t e = orc_energy(s, n);
        if (best < 0 || e < best) {
            best = e;
            cnt = 1;
            best_code = code;  /* ascending codes: the first is the smallest */
        } else if (e == best) {
            ++cnt;
        }
    }
    /* of the attaining codes, the smallest with s_0 = +1 (bit 0 clear):
     * negating every free spin negates the sequence, E unchanged, so the
     * smallest attaining code with bit 0 set has a partner without it */
    if (best_code & 1u) {
        for (uint64_t code = 0; code < total; code += 2) {
            orc_skew_sequence(n, code, s);
            if (orc_energy(s, n) == best) {
                best_code = code;
                break;
            }
        }
    }
    *emin = best;
    *count = cnt;
    if (argmin)
        orc_skew_sequence(n, best_code, argmin);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Neighbourhood energies.                                                    */
/* ------------------------------------------------------------------------- */

/* Definition: out[i] = E(flip(s, i)) for every i, each recomputed from
 * Eq. (2) (the O(N^3)-per-step route the paper calls prohibitive, Sec. III.C). */
void orc_neighbour_energies_recompute(const int8_t *s, int n, int64_t *out)
{
    int8_t t[ORC_MAX_N];
    if (n < 1 || n > ORC_MAX_N)
        return;
    memcpy(t, s, (size_t)n);
    for (int i = 0; i < n; ++i) {
        t[i] = (int8_t)-t[i];
        out[i] = orc_energy(t, n);
        t[i] = (int8_t)-t[i];
    }
}

/* The paper's data structures (Sec. III.C, Table "combinedTable"):
 * tableC[k][i] = s_i s_{i+k} (row k, the products behind C_k), and
 * vectorC[k] = C_k, the row sums.  Flipping bit i negates the products that
 * contain s_i: tableC[k][i] (when i+k < n) and tableC[k][i-k] (when i-k >= 0),
 * so each neighbour's energy costs O(n) and the update after a move touches
 * one "row and column" of products. */
typedef struct {
    int n;
    int8_t table[ORC_MAX_N][ORC_MAX_N]; /* table[k][i], valid for 1 <= k < n, 0 <= i < n-k */
    int64_t vec[ORC_MAX_N];             /* vec[k] = C_k */
} tables_t;

static void tables_build(tables_t *T, const int8_t *s, int n)
{
    T->n = n;
    for (int k = 1; k < n; ++k) {
        int64_t c = 0;
        for (int i = 0; i + k < n; ++i) {
            T->table[k][i] = (int8_t)(s[i] * s[i + k]);
            c += T->table[k][i];
        }
        T->vec[k] = c;
    }
}

/* Energy of flip(s, i) from the tables. */
static int64_t tables_neighbour_energy(const tables_t *T, int i)
{
    int n = T->n;
    int64_t e = 0;
    for (int k = 1; k < n; ++k) {
        int64_t c = T->vec[k];
        if (i + k < n)
            c -= 2 * (int64_t)T->table[k][i];
        if (i - k >= 0)
            c -= 2 * (int64_t)T->table[k][i - k];
        e += c * c;
    }
    return e;
}

/* Apply flip(s, i) to the tables. */
static void tables_flip(tables_t *T, int i)
{
    int n = T->n;
    for (int k = 1; k < n; ++k) {
        if (i + k < n) {
            T->vec[k] -= 2 * (int64_t)T->table[k][i];
            T->table[k][i] = (int8_t)-T->table[k][i];
        }
        if (i - k >= 0) {
            T->vec[k] -= 2 * (int64_t)T->table[k][i - k];
            T->table[k][i - k] = (int8_t)-T->table[k][i - k];
        }
    }
}

void orc_neighbour_energies_tables(const int8_t *s, int n, int64_t *out)
{
    if (n < 1 || n > ORC_MAX_N)
        return;
    tables_t *T = (tables_t *)malloc(sizeof(tables_t));
    tables_build(T, s, n);
    for (int i = 0; i < n; ++i)
        out[i] = tables_neighbour_energy(T, i);
    free(T);
}

/* ------------------------------------------------------------------------- */
/* Walk schedule: walk length maxIter and tenure range [minTabu, maxTabu].    */
/* ------------------------------------------------------------------------- */
enum { ORC_STEPS_FIXED = 0, ORC_STEPS_MULT_N = 1, ORC_STEPS_PAPER = 2, ORC_STEPS_RANGE = 3 };
enum { ORC_TENURE_LINEAR = 0, ORC_TENURE_PAPER = 1 };

/* The parameters of a walk (Alg. 2): how maxIter and the tenure range are
 * obtained for a length n, and whether aspiration is on. */
typedef struct {
    int steps_rule, steps_a, tenure_rule;
    int lo_num, lo_den, lo_add, hi_num, hi_den, hi_add;
    int aspiration;
    int slo_num, slo_den, shi_num, shi_den; /* ORC_STEPS_RANGE bounds */
} orc_rule_t;

/*
 * steps_rule
 *   FIXED : maxIter = a
 *   MULT_N: maxIter = a * n
 *   PAPER : maxIter = randomInt(0, n) + floor(n/2) (Alg. 4, both ends
 *           inclusive), one draw (entity, gen, 0, TAG_LEN), word 0.
 *   RANGE : maxIter uniform in [floor(slo_num*n/slo_den),
 *           floor(shi_num*n/shi_den)] (both ends inclusive) from the same
 *           draw: lo + ((w0 * (hi - lo + 1)) >> 32).  Sec. III.B states the
 *           walk length as randInt[N/2, 3N/2]; RANGE(1/2, 3/2) is that
 *           statement.
 * tenure_rule
 *   LINEAR: minTabu = floor(lo_num*n/lo_den) + lo_add,
 *           maxTabu = floor(hi_num*n/hi_den) + hi_add
 *   PAPER : minTabu = floor(0.1*maxIter), maxTabu = floor(0.12*maxIter)
 *           (Sec. III.B), in integers floor(T/10) and floor(3T/25).
 * Returns 0, or -1 when the schedule is invalid (0 <= lo <= hi < n fails).
 */
int orc_walk_schedule(int n, const orc_rule_t *r, uint64_t seed, uint32_t entity,
                      uint32_t gen, int *steps, int *lo, int *hi)
{
    int T;
    if (r->steps_rule == ORC_STEPS_FIXED) {
        T = r->steps_a;
    } else if (r->steps_rule == ORC_STEPS_MULT_N) {
        T = r->steps_a * n;
    } else if (r->steps_rule == ORC_STEPS_PAPER) {
        uint32_t w[4];
        draw(seed, entity, gen, 0, ORC_TAG_LEN, w);
        T = n / 2 + (int)uniform_below(w[0], (uint32_t)(n + 1));
    } else if (r->steps_rule == ORC_STEPS_RANGE) {
        if (r->slo_den <= 0 || r->shi_den <= 0 || r->slo_num < 0 || r->shi_num < 0)
            return -1;
        int tlo = r->slo_num * n / r->slo_den, thi = r->shi_num * n / r->shi_den;
        if (thi < tlo)
            return -1;
        uint32_t w[4];
        draw(seed, entity, gen, 0, ORC_TAG_LEN, w);
        T = tlo + (int)uniform_below(w[0], (uint32_t)(thi - tlo + 1));
    } else {
        return -1;
    }
    int l, h;
    if (r->tenure_rule == ORC_TENURE_LINEAR) {
        if (r->lo_den <= 0 || r->hi_den <= 0)
            return -1;
        l = r->lo_num * n / r->lo_den + r->lo_add;
        h = r->hi_num * n / r->hi_den + r->hi_add;
    } else if (r->tenure_rule == ORC_TENURE_PAPER) {
        l = T / 10;
        h = 3 * T / 25;
    } else {
        return -1;
    }
    if (T < 0 || l < 0 || h < l || h >= n)
        return -1;
    *steps = T;
    *lo = l;
    *hi = h;
    return 0;
}

/* Random start of stand-alone walk `walk`: s_i = -1 when bit i % 128 of the
 * 128-bit draw (walk, 0, i / 128, TAG_START) is set, the draw's word
 * (i % 128) / 32 holding bits 32 w .. 32 w + 31. */
void orc_random_start(int n, uint64_t seed, uint32_t walk, int8_t *s)
{
    uint32_t w[4];
    for (int i = 0; i < n; ++i) {
        if ((i & 127) == 0)
            draw(seed, walk, 0, (uint32_t)(i >> 7), ORC_TAG_START, w);
        s[i] = ((w[(i & 127) >> 5] >> (i & 31)) & 1u) ? -1 : 1;
    }
}

/* ------------------------------------------------------------------------- */
/* Tabu search: Alg. 2 (and its thread-parallel form, Alg. 4).                */
/* ------------------------------------------------------------------------- */
/*
 * One walk of `steps` iterations from `start`.
 *   - tabuList starts at 0 and bestSeqTS = start (the start counts as
 *     visited).
 *   - Step t = 1..steps: every neighbour flip(pivot, i) is scored; i is
 *     admissible when tabuList[i] < t, or -- with aspiration -- when its
 *     energy is strictly below the walk's best so far (aspiration is this
 *     implementation's addition; aspiration = 0 is the paper's rule).
 *   - The admissible minimum is taken; ties are broken uniformly: with
 *     (u0, u1) = words 0, 1 of draw (entity, gen, t, TAG_STEP), the tied
 *     indices in ascending order T[0..c-1] give the move T[(u0*c) >> 32].
 *   - pivot <- flip(pivot, i); tabuList[i] = t + lo + ((u1*(hi-lo+1)) >> 32).
 *   - bestSeqTS <- pivot when E(pivot) < E(bestSeqTS) (strict).
 * recompute = 1 scores every neighbour from Eq. (2) directly; recompute = 0
 * uses tableC/vectorC (Sec. III.C).  Both must give identical walks.
 * trace[t-1] (optional) receives the flipped index, trace_e[t-1] (optional)
 * the energy after step t, trace_x[t-1] (optional) the tabuList entry the
 * flipped index receives at step t (the last step at which it is tabu).
 * Returns 0, or -1 if a step has no admissible move (cannot happen when
 * hi < n: at most hi bits are tabu at any step).
 */
int orc_tabu_walk(int n, const int8_t *start, uint64_t seed, uint32_t entity,
                  uint32_t gen, int steps, int lo, int hi, int aspiration,
                  int recompute, int8_t *best, int64_t *best_e,
                  int64_t *final_e, int16_t *trace, int64_t *trace_e,
                  int64_t *trace_x)
{
    int8_t pivot[ORC_MAX_N];
    int64_t tabu[ORC_MAX_N];
    int64_t cand[ORC_MAX_N];
    int ties[ORC_MAX_N];
    if (n < 1 || n > ORC_MAX_N || lo < 0 || hi < lo)
        return -1;

    memcpy(pivot, start, (size_t)n);
    memcpy(best, start, (size_t)n);
    for (int i = 0; i < n; ++i)
        tabu[i] = 0;
    int64_t E = orc_energy(pivot, n);
    int64_t bestE = E;

    tables_t *T = NULL;
    if (!recompute) {
        T = (tables_t *)malloc(sizeof(tables_t));
        tables_build(T, pivot, n);
    }

    for (int t = 1; t <= steps; ++t) {
        if (recompute)
            orc_neighbour_energies_recompute(pivot, n, cand);
        else
            for (int i = 0; i < n; ++i)
                cand[i] = tables_neighbour_energy(T, i);

        int64_t m = INT64_MAX;
        int found = 0;
        for (int i = 0; i < n; ++i) {
            int admissible = (tabu[i] < t) || (aspiration && cand[i] < bestE);
            if (admissible && (!found || cand[i] < m)) {
                m = cand[i];
                found = 1;
            }
        }
        if (!found) {
            free(T);
            return -1;
        }
        int c = 0;
        for (int i = 0; i < n; ++i) {
            int admissible = (tabu[i] < t) || (aspiration && cand[i] < bestE);
            if (admissible && cand[i] == m)
                ties[c++] = i;
        }
        uint32_t w[4];
        draw(seed, entity, gen, (uint32_t)t, ORC_TAG_STEP, w);
        int pick = ties[uniform_below(w[0], (uint32_t)c)];

        pivot[pick] = (int8_t)-pivot[pick];
        if (!recompute)
            tables_flip(T, pick);
        E = m;
        tabu[pick] = (int64_t)t + lo + (int64_t)uniform_below(w[1], (uint32_t)(hi - lo + 1));
        if (E < bestE) {
            bestE = E;
            memcpy(best, pivot, (size_t)n);
        }
        if (trace)
            trace[t - 1] = (int16_t)pick;
        if (trace_e)
            trace_e[t - 1] = E;
        if (trace_x)
            trace_x[t - 1] = tabu[pick];
    }
    free(T);
    *best_e = bestE;
    *final_e = E;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Batched stand-alone walks (the batch driver), optionally over threads.     */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t W;
    const int32_t *ns;
    int32_t n_uniform;
    const int8_t *starts; /* [W][stride] or NULL for random starts */
    int32_t stride;
    uint64_t seed;
    orc_rule_t rule;
    int8_t *best_seq;     /* [W][stride], positions >= n are set to 0 */
    int64_t *best_e;
    int64_t *final_e;
    int64_t next;         /* next walk to take (guarded by lock) */
    pthread_mutex_t lock;
    int status;
} batch_job_t;

static int run_one_walk(batch_job_t *J, int64_t w)
{
    int n = J->ns ? J->ns[w] : J->n_uniform;
    int8_t start[ORC_MAX_N];
    int steps, lo, hi;
    if (n < 3 || n > ORC_MAX_N || n > J->stride)
        return -1;
    if (orc_walk_schedule(n, &J->rule, J->seed, (uint32_t)w, 0, &steps, &lo, &hi))
        return -1;
    if (J->starts)
        memcpy(start, J->starts + w * J->stride, (size_t)n);
    else
        orc_random_start(n, J->seed, (uint32_t)w, start);
    int8_t *out = J->best_seq + w * J->stride;
    memset(out, 0, (size_t)J->stride);
    return orc_tabu_walk(n, start, J->seed, (uint32_t)w, 0, steps, lo, hi,
                         J->rule.aspiration, 0, out, &J->best_e[w], &J->final_e[w],
                         NULL, NULL, NULL);
}

static void *batch_worker(void *arg)
{
    batch_job_t *J = (batch_job_t *)arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t w = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (w >= J->W)
            break;
        if (run_one_walk(J, w)) {
            pthread_mutex_lock(&J->lock);
            J->status = -1;
            pthread_mutex_unlock(&J->lock);
        }
    }
    return NULL;
}

int orc_tabu_batch(int64_t W, const int32_t *ns, int32_t n_uniform,
                   const int8_t *starts, int32_t stride, uint64_t seed,
                   const orc_rule_t *rule,
                   int8_t *best_seq, int64_t *best_e, int64_t *final_e,
                   int nthreads)
{
    batch_job_t J;
    memset(&J, 0, sizeof(J));
    J.W = W; J.ns = ns; J.n_uniform = n_uniform; J.starts = starts;
    J.stride = stride; J.seed = seed;
    J.rule = *rule;
    J.best_seq = best_seq; J.best_e = best_e; J.final_e = final_e;
    pthread_mutex_init(&J.lock, NULL);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 1; i < nthreads; ++i)
        if (pthread_create(&th[started], NULL, batch_worker, &J) == 0)
            ++started;
    batch_worker(&J);
    for (int i = 0; i < started; ++i)
        pthread_join(th[i], NULL);
    pthread_mutex_destroy(&J.lock);
    return J.status;
}

/* ------------------------------------------------------------------------- */
/* Memetic tabu search: Alg. 1 (per replica, Alg. 3).                         */
/* ------------------------------------------------------------------------- */
/*
 * Population state of one replica: pop[K][n] (+-1), popE[K], best[n], bestE.
 *
 * Initialisation (Alg. 1, first two lines): member m is read from the
 * draws (pop_id, m, i / 128, TAG_INIT) as orc_random_start reads its draws;
 * bestSeq is the lowest-index member of minimum energy.
 */
void orc_memetic_init(int n, int K, uint64_t seed, uint32_t pop_id,
                      int8_t *pop, int64_t *popE, int8_t *best, int64_t *best_e)
{
    int argmin = 0;
    for (int m = 0; m < K; ++m) {
        uint32_t w[4];
        int8_t *s = pop + (int64_t)m * n;
        for (int i = 0; i < n; ++i) {
            if ((i & 127) == 0)
                draw(seed, pop_id, (uint32_t)m, (uint32_t)(i >> 7), ORC_TAG_INIT, w);
            s[i] = ((w[(i & 127) >> 5] >> (i & 31)) & 1u) ? -1 : 1;
        }
        popE[m] = orc_energy(s, n);
        if (popE[m] < popE[argmin])
            argmin = m;
    }
    memcpy(best, pop + (int64_t)argmin * n, (size_t)n);
    *best_e = popE[argmin];
}

/* Binary tournament (selectParents is unspecified in Alg. 1; this reading):
 * two uniform draws with replacement, the lower energy wins, ties go to the
 * first draw. */
static int tournament(const int64_t *popE, int K, uint32_t u, uint32_t v)
{
    int i = (int)uniform_below(u, (uint32_t)K);
    int j = (int)uniform_below(v, (uint32_t)K);
    return popE[i] <= popE[j] ? i : j;
}

/*
 * Advance one replica from generation g0 by up to n_gens generations
 * (one generation = one pass of Alg. 1's loop body = one child).
 * Generation g uses words w0..w7 = draws (pop_id, g, 0|1, TAG_GEN):
 *   crossover when w0 < p_comb (randReal < p_comb with p_comb = p_comb/2^32):
 *     parents a = tournament(w1, w2), b = tournament(w3, w4);
 *     Combine = one-point crossover at cut = 1 + ((w5*(n-1)) >> 32):
 *     child = a[0:cut] ++ b[cut:n];
 *   otherwise Sample: child = pop[(w1*K) >> 32].
 *   Mutate: bit i flips when word i%4 of draw (pop_id, g, i/4, TAG_MUT) is
 *     below p_mut (probability p_mut/2^32).
 *   child <- Tabu-Search(child) with entity pop_id and generation g.
 *   bestSeq <- child when E(child) < E(bestSeq) (strict).
 *   The child replaces member (w6*K) >> 32 (a uniform random individual).
 * Stopping (Alg. 1's while condition): with target >= 0 the replica stops as
 * soon as bestE <= target; *hit_gen is then the number of children produced
 * when that first held (0 for the initial population); it stays -1 otherwise
 * and is left unchanged if already set.
 * Returns the number of generations executed, or -1 on an invalid schedule.
 */
int64_t orc_memetic_advance(int n, int K, uint32_t p_comb, uint32_t p_mut,
                            const orc_rule_t *rule, uint64_t seed, uint32_t pop_id, int64_t g0,
                            int64_t n_gens, int64_t target,
                            int8_t *pop, int64_t *popE, int8_t *best,
                            int64_t *best_e, int64_t *hit_gen)
{
    int8_t child[ORC_MAX_N], child_best[ORC_MAX_N];
    int64_t done = 0;
    if (n < 2 || n > ORC_MAX_N || K < 1)
        return -1;
    for (int64_t g = g0; g < g0 + n_gens; ++g) {
        if (target >= 0 && *best_e <= target) {
            if (*hit_gen < 0)
                *hit_gen = g;
            break;
        }
        uint32_t wa[4], wb[4];
        draw(seed, pop_id, (uint32_t)g, 0, ORC_TAG_GEN, wa);
        draw(seed, pop_id, (uint32_t)g, 1, ORC_TAG_GEN, wb);
        if (wa[0] < p_comb) {
            int a = tournament(popE, K, wa[1], wa[2]);
            int b = tournament(popE, K, wa[3], wb[0]);
            int cut = 1 + (int)uniform_below(wb[1], (uint32_t)(n - 1));
            for (int i = 0; i < n; ++i)
                child[i] = i < cut ? pop[(int64_t)a * n + i] : pop[(int64_t)b * n + i];
        } else {
            int c = (int)uniform_below(wa[1], (uint32_t)K);
            memcpy(child, pop + (int64_t)c * n, (size_t)n);
        }
        for (int i = 0; i < n; ++i) {
            uint32_t wm[4];
            draw(seed, pop_id, (uint32_t)g, (uint32_t)(i >> 2), ORC_TAG_MUT, wm);
            if (wm[i & 3] < p_mut)
                child[i] = (int8_t)-child[i];
        }
        int steps, lo, hi;
        if (orc_walk_schedule(n, rule, seed, pop_id, (uint32_t)g, &steps, &lo, &hi))
            return -1;
        int64_t ce, fe;
        if (orc_tabu_walk(n, child, seed, pop_id, (uint32_t)g, steps, lo, hi,
                          rule->aspiration, 0, child_best, &ce, &fe, NULL, NULL, NULL))
            return -1;
        if (ce < *best_e) {
            *best_e = ce;
            memcpy(best, child_best, (size_t)n);
        }
        int r = (int)uniform_below(wb[2], (uint32_t)K);
        memcpy(pop + (int64_t)r * n, child_best, (size_t)n);
        popE[r] = ce;
        ++done;
        if (target >= 0 && *best_e <= target) {
            if (*hit_gen < 0)
                *hit_gen = g + 1;
            break;
        }
    }
    return done;
}

/*
 * Batched-generation variant (a documented departure from Alg. 1, which is
 * steady state: one child per loop pass).  Generation g produces B children
 * from the population as it stands at the start of g; only then are they
 * merged, in the order b = 0..B-1, each exactly as Alg. 1 merges its one
 * child (strict best update, then replacement of a random member, a later
 * child overwriting an earlier one on the same slot).  Child b draws its
 * words from (pop_id, g, 2b | 2b+1, TAG_GEN), its mutation words from
 * (pop_id, g, 64 b + i/4, TAG_MUT), and walks as generation g*B + b.  With
 * B = 1 every draw and every step coincides with orc_memetic_advance.  The
 * target is checked once per generation, after the merge; *hit_gen counts
 * generations.  Returns the generations executed or -1.
 */
int64_t orc_memetic_advance_batched(int n, int K, int B, uint32_t p_comb, uint32_t p_mut,
                                    const orc_rule_t *rule, uint64_t seed, uint32_t pop_id, int64_t g0,
                                    int64_t n_gens, int64_t target,
                                    int8_t *pop, int64_t *popE, int8_t *best,
                                    int64_t *best_e, int64_t *hit_gen)
{
    int8_t child[ORC_MAX_N], kids[8][ORC_MAX_N];
    int64_t kid_e[8];
    int kid_slot[8];
    if (B < 1 || B > 8 || n < 2 || n > ORC_MAX_N || K < 1)
        return -1;
    int64_t done = 0;
    for (int64_t g = g0; g < g0 + n_gens; ++g) {
        if (target >= 0 && *best_e <= target) {
            if (*hit_gen < 0)
                *hit_gen = g;
            break;
        }
        /* every child of this generation sees the same population */
        for (int b = 0; b < B; ++b) {
            uint32_t wa[4], wb[4];
            draw(seed, pop_id, (uint32_t)g, (uint32_t)(2 * b), ORC_TAG_GEN, wa);
            draw(seed, pop_id, (uint32_t)g, (uint32_t)(2 * b + 1), ORC_TAG_GEN, wb);
            if (wa[0] < p_comb) {
                int pa = tournament(popE, K, wa[1], wa[2]);
                int pb = tournament(popE, K, wa[3], wb[0]);
                int cut = 1 + (int)uniform_below(wb[1], (uint32_t)(n - 1));
                for (int i = 0; i < n; ++i)
                    child[i] = i < cut ? pop[(int64_t)pa * n + i] : pop[(int64_t)pb * n + i];
            } else {
                int c = (int)uniform_below(wa[1], (uint32_t)K);
                memcpy(child, pop + (int64_t)c * n, (size_t)n);
            }
            for (int i = 0; i < n; ++i) {
                uint32_t wm[4];
                draw(seed, pop_id, (uint32_t)g, (uint32_t)(64 * b + (i >> 2)), ORC_TAG_MUT, wm);
                if (wm[i & 3] < p_mut)
                    child[i] = (int8_t)-child[i];
            }
            const uint32_t walk_gen = (uint32_t)(g * B + b);
            int steps, lo, hi;
            if (orc_walk_schedule(n, rule, seed, pop_id, walk_gen, &steps, &lo, &hi))
                return -1;
            int64_t fe;
            if (orc_tabu_walk(n, child, seed, pop_id, walk_gen, steps, lo, hi,
                              rule->aspiration, 0, kids[b], &kid_e[b], &fe, NULL, NULL, NULL))
                return -1;
            kid_slot[b] = (int)uniform_below(wb[2], (uint32_t)K);
        }
        for (int b = 0; b < B; ++b) {
            if (kid_e[b] < *best_e) {
                *best_e = kid_e[b];
                memcpy(best, kids[b], (size_t)n);
            }
            memcpy(pop + (int64_t)kid_slot[b] * n, kids[b], (size_t)n);
            popE[kid_slot[b]] = kid_e[b];
        }
        ++done;
        if (target >= 0 && *best_e <= target) {
            if (*hit_gen < 0)
                *hit_gen = g + 1;
            break;
        }
    }
    return done;
}

/* ------------------------------------------------------------------------- */
/* Deviation from skew-symmetry (App. A).                                     */
/* ------------------------------------------------------------------------- */
/* n_non-skew of an odd-length sequence t[0..m-1], m = 2c + 1: the number of
 * i = 1..c with t[c+i] != (-1)^i t[c-i] (App. A's sum of |differences| / 2;
 * skew-symmetry itself is Sec. II.C's condition).  Even m: -1 (undefined). */
int orc_non_skew(const int8_t *t, int m)
{
    if (m < 1 || (m & 1) == 0)
        return -1;
    int c = (m - 1) / 2, count = 0;
    for (int i = 1; i <= c; ++i) {
        int sign = (i & 1) ? -1 : 1;
        if (t[c + i] != sign * t[c - i])
            ++count;
    }
    return count;
}

/* d(S) of App. A: the least n_non-skew over the sequences reachable by one
 * rotation Rot(S; r) (the first r elements moved to the end) followed by one
 * insertion Ins(.; i, xi) (xi after the first i elements) or one deletion
 * Del(.; i) (the i-th element, 1-based, removed).  n_non-skew only exists
 * for odd lengths, so an odd N is measured on its rotations alone and an
 * even N on rotation + deletion; with_insertion = 1 also takes rotation +
 * insertion for even N (the printed values follow deletion only).
 * Returns -1 for n < 1 or n > ORC_MAX_N. */
int orc_skew_deviation(const int8_t *s, int n, int with_insertion)
{
    int8_t rot[ORC_MAX_N], t[ORC_MAX_N + 1];
    if (n < 1 || n > ORC_MAX_N)
        return -1;
    int best = n;
    for (int r = 0; r < n; ++r) {
        for (int k = 0; k < n; ++k)
            rot[k] = s[(k + r) % n];
        if (n & 1) {
            int v = orc_non_skew(rot, n);
            if (v < best)
                best = v;
            continue;
        }
        for (int i = 1; i <= n; ++i) {  /* Del(rot; i) */
            int m = 0;
            for (int k = 0; k < n; ++k)
                if (k != i - 1)
                    t[m++] = rot[k];
            int v = orc_non_skew(t, n - 1);
            if (v < best)
                best = v;
        }
        if (!with_insertion)
            continue;
        for (int i = 0; i <= n; ++i) {  /* Ins(rot; i, xi) */
            for (int xi = -1; xi <= 1; xi += 2) {
                int m = 0;
                for (int k = 0; k < i; ++k)
                    t[m++] = rot[k];
                t[m++] = (int8_t)xi;
                for (int k = i; k < n; ++k)
                    t[m++] = rot[k];
                int v = orc_non_skew(t, n + 1);
                if (v < best)
                    best = v;
            }
        }
    }
    return best;
}
