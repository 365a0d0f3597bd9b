/*
 * EBIC oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU statement of what EBIC computes, used
 * to check the GPU library. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the library never does.
 *
 * Paper: "EBIC.JL - an Efficient Implementation of Evolutionary Biclustering
 * Algorithm in Julia" (GECCO'21 Companion, arXiv 2105.01196).
 *   Sec. 2.3 (EBIC paragraph): an individual is a series of columns, and a
 *     row belongs to its bicluster when the row's values rise along that
 *     series; operators insertion/deletion/substitution/swap/crossover;
 *     elitism, tournament selection with an exponential penalty for overused
 *     columns (crowding), tabu list of individuals, stop on tabu hits.
 *   Sec. 2.4 (EBIC.jl): the nine-step generational loop, and the parameters
 *     (negative trends on/off, approximate-trend threshold, allowed overlap,
 *     iterations, number of biclusters).
 * The paper prints no formula for the tolerance, the size score, the overlap
 * measure, the crowding penalty or any default; the readings taken for them
 * are stated where they are used below.
 *
 * Floating point: the only FP results are exact FP64 values built with ldexp
 * from integers; compile with -ffp-contract=off.
 *
 * Parity status: evaluate() is pinned (brute force, Eulerian closed forms,
 * invariants, fitness identities, the size-score and overlap thresholds on
 * both sides). The size-score and overlap-penalty formulas themselves are a
 * reading, not printed in the paper: parity unpinned beyond those
 * identities. run() is pinned by RNG known-answer values (bounded draws
 * against a big-integer implementation included), the canonical tabu key,
 * determinism and planted recovery only: its trajectory is parity unpinned
 * against the paper.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_K_LIMIT 512

typedef struct oracle_params {
    int32_t approx_permille;   /* a: approximate-trend threshold, per mille   */
    int32_t negative_trends;   /* 0/1: reversed trends also count             */
    int32_t overlap_permille;  /* theta: allowed overlap, per mille           */
    int32_t min_rows;          /* r_min: fewer rows score 0                   */
    int32_t k_score_min;       /* fewer columns score 0                       */
    int32_t k_min, k_max;      /* allowed series lengths                      */
    int32_t archive_size;      /* K: top-rank list capacity                   */
    int32_t n_out;             /* b: biclusters returned                      */
    int32_t population;        /* P                                           */
    int32_t generations;       /* G: populations evaluated at most            */
    int32_t max_tabu_hits;     /* stop once this many mutants were rejected   */
    int32_t tournament;        /* T: tournament size                          */
    int32_t max_attempts;      /* attempts per population slot                */
    int32_t tie_rule;          /* equal values: 0 by column index, 1 strict,  */
                               /* 2 loose (see step_counts)                   */
    int32_t op_permille[5];    /* weights of insertion, deletion,             */
                               /* substitution, swap, crossover: per mille,   */
                               /* summing to 1000; all 0 means 200 each       */
} oracle_params;

/* ------------------------------------------------------------------------ */
/* Part 1: evaluation of one individual.                                    */
/* ------------------------------------------------------------------------ */

/* Row order (reading of ties, the paper does not say how equal values
 * count), for a step from column a to column b of row r; IEEE compares, so
 * -0 == +0. Adds to *v_inc when the step goes against the increasing trend
 * and to *v_dec when it goes against the decreasing one.
 *   rule 0: a precedes b when its value is smaller, or equal and a < b (a
 *           strict total order): every step goes against exactly one trend;
 *   rule 1 (strict): a tie goes against both trends;
 *   rule 2 (loose): a tie goes against neither. */
static void step_counts(const float *X, int C, int r, int a, int b, int rule,
                        int *v_inc, int *v_dec)
{
    float xa = X[(size_t)r * C + a];
    float xb = X[(size_t)r * C + b];
    if (xa < xb) {
        *v_dec += 1;
    } else if (xa > xb) {
        *v_inc += 1;
    } else if (rule == 0) {
        if (a < b)
            *v_dec += 1;
        else
            *v_inc += 1;
    } else if (rule == 1) {
        *v_inc += 1;
        *v_dec += 1;
    }
}

/* Tolerance (reading of the approximate-trend threshold, Sec. 2.4): the
 * number of the k-1 consecutive steps allowed to break the trend,
 * floor((k-1)(1000-a)/1000) in integers. */
static int tolerance(int k, int approx_permille)
{
    return (int)(((int64_t)(k - 1) * (1000 - approx_permille)) / 1000);
}

/* A row follows the series when at most t of its consecutive steps go
 * against the increasing order; with negative trends on, a row that follows
 * the reversed order counts too (each row once). */
static int row_fits(const float *X, int C, int r, const uint16_t *s, int k,
                    int t, int neg, int rule)
{
    int v_inc = 0, v_dec = 0;  /* steps against each trend */
    for (int j = 0; j + 1 < k; j++)
        step_counts(X, C, r, s[j], s[j + 1], rule, &v_inc, &v_dec);
    return v_inc <= t || (neg && v_dec <= t);
}

/* Size score (reading): s = n * 2^k when the bicluster has at least r_min
 * rows and k_score_min columns, else 0. */
static double size_score(int n, int k, const oracle_params *p)
{
    if (n >= p->min_rows && k >= p->k_score_min)
        return ldexp((double)n, k);
    return 0.0;
}

/* Overlap test (reading of the allowed overlap level): an archived bicluster
 * j covers h_j of the candidate's rows and g_j of its columns; it overlaps
 * too much when h_j*g_j exceeds theta per mille of the candidate's n*k
 * cells. Cross-multiplied in 64-bit integers. */
static int overlaps(int64_t h, int64_t g, int64_t n, int64_t k, int theta)
{
    return 1000 * h * g > (int64_t)theta * n * k;
}

static int count_common_cols(const uint16_t *a, int ka, const uint16_t *b, int kb)
{
    int g = 0;
    for (int i = 0; i < ka; i++)
        for (int j = 0; j < kb; j++)
            if (a[i] == b[j]) { g++; break; }
    return g;
}

typedef struct {
    int K;
    const uint8_t *rows;      /* K x R, 1 where the row is in the member */
    const int32_t *col_off;   /* K + 1 */
    const uint16_t *cols;     /* member series, concatenated */
} arch_view;

static void eval_individual(const float *X, int R, int C, const uint16_t *s, int k,
                            const arch_view *A, const oracle_params *p,
                            uint8_t *support, int32_t *n_out, int32_t *h_out,
                            double *score_out, double *fitness_out)
{
    int t = tolerance(k, p->approx_permille);
    int n = 0;
    for (int r = 0; r < R; r++) {
        support[r] = (uint8_t)row_fits(X, C, r, s, k, t, p->negative_trends, p->tie_rule);
        n += support[r];
    }
    int m = 0;
    for (int j = 0; j < A->K; j++) {
        const uint8_t *Sj = A->rows + (size_t)j * R;
        int h = 0;
        for (int r = 0; r < R; r++)
            h += support[r] & Sj[r];
        int g = count_common_cols(s, k, A->cols + A->col_off[j],
                                  A->col_off[j + 1] - A->col_off[j]);
        if (h_out) h_out[j] = h;
        m += overlaps(h, g, n, k, p->overlap_permille);
    }
    double sc = size_score(n, k, p);
    *n_out = n;
    *score_out = sc;
    /* penalty: halve the score once for every archived bicluster that
     * overlaps too much */
    *fitness_out = ldexp(sc, -m);
}

static int series_valid(const uint16_t *s, int k, int C)
{
    if (k < 2 || k > ORACLE_K_LIMIT) return 0;
    for (int i = 0; i < k; i++) {
        if (s[i] >= C) return 0;
        for (int j = 0; j < i; j++)
            if (s[i] == s[j]) return 0;
    }
    return 1;
}

/* Evaluate P individuals (CSR: offsets[P+1], cols) against an archive.
 * support (P x R flags), overlap (P x K) and score (P) may be NULL.
 * Returns 0, or -1 for an invalid argument. */
int oracle_evaluate(const float *X, int R, int C, int P,
                    const int32_t *offsets, const uint16_t *cols,
                    int K, const uint8_t *arch_rows, const int32_t *arch_off,
                    const uint16_t *arch_cols, const oracle_params *p, int nthreads,
                    double *fitness, int32_t *count, uint8_t *support,
                    int32_t *overlap, double *score)
{
    if (R < 1 || C < 2 || P < 0 || K < 0 || !X || !p) return -1;
    for (int i = 0; i < P; i++)
        if (!series_valid(cols + offsets[i], offsets[i + 1] - offsets[i], C)) return -1;
    for (int j = 0; j < K; j++)
        if (!series_valid(arch_cols + arch_off[j], arch_off[j + 1] - arch_off[j], C)) return -1;
    arch_view A = {K, arch_rows, arch_off, arch_cols};
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1) reduction(|:bad)
    for (int i = 0; i < P; i++) {
        uint8_t *sup = support ? support + (size_t)i * R : malloc((size_t)R);
        if (!sup) { bad = 1; continue; }
        int32_t n;
        double sc, f;
        eval_individual(X, R, C, cols + offsets[i], offsets[i + 1] - offsets[i], &A, p,
                        sup, &n, overlap ? overlap + (size_t)i * K : NULL, &sc, &f);
        count[i] = n;
        fitness[i] = f;
        if (score) score[i] = sc;
        if (!support) free(sup);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Part 2: the generational loop (Sec. 2.4, steps 1-9).                     */
/* ------------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the
 * golden-ratio increment and each output is the state put through the
 * variant-13 finaliser. One sequential stream per run, seeded with `seed`. */
typedef struct { uint64_t state; } splitmix64;

uint64_t oracle_splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform integer in [0, n): reject draws below 2^64 mod n, so that the
 * accepted range is a whole number of periods of n, then reduce mod n. */
uint64_t oracle_uniform(uint64_t *state, uint64_t n)
{
    uint64_t low = (0 - n) % n;
    uint64_t x;
    do {
        x = oracle_splitmix64_next(state);
    } while (x < low);
    return x % n;
}

typedef struct {
    int k;
    uint16_t c[ORACLE_K_LIMIT];
} series;

/* Lexicographic order on series; a proper prefix sorts first. */
static int series_cmp(const series *a, const series *b)
{
    int m = a->k < b->k ? a->k : b->k;
    for (int i = 0; i < m; i++)
        if (a->c[i] != b->c[i]) return a->c[i] < b->c[i] ? -1 : 1;
    return (a->k > b->k) - (a->k < b->k);
}

/* Canonical form used for the tabu list: with negative trends on, a series
 * and its reverse have identical supports, so the smaller of the two stands
 * for both. */
static void canonical(const series *s, int neg, series *out)
{
    *out = *s;
    if (!neg) return;
    series r;
    r.k = s->k;
    for (int i = 0; i < s->k; i++) r.c[i] = s->c[s->k - 1 - i];
    if (series_cmp(&r, s) < 0) *out = r;
}

/* Tabu list: an exact set of canonical series (Sec. 2.3 stores hashes; here
 * the hash only locates the slot and equality decides, so a collision cannot
 * change a result). Open addressing with linear probing; each entry holds its
 * own copy of the series. */
typedef struct {
    uint16_t **seq;   /* NULL = empty slot */
    int32_t *len;
    size_t cap, size;
} tabu_set;

static uint64_t seq_hash(const uint16_t *c, int k)
{
    uint64_t h = 1469598103934665603ULL;
    for (int i = 0; i < k; i++) {
        h ^= c[i];
        h *= 1099511628211ULL;
    }
    h ^= (uint64_t)k;
    h *= 1099511628211ULL;
    return h;
}

static int tabu_init(tabu_set *T, size_t cap)
{
    T->cap = cap;
    T->size = 0;
    T->seq = calloc(cap, sizeof(uint16_t *));
    T->len = calloc(cap, sizeof(int32_t));
    return T->seq && T->len ? 0 : -1;
}

static void tabu_free(tabu_set *T)
{
    if (T->seq)
        for (size_t i = 0; i < T->cap; i++) free(T->seq[i]);
    free(T->seq);
    free(T->len);
    T->seq = NULL;
    T->len = NULL;
}

static size_t tabu_find(const tabu_set *T, const uint16_t *c, int k)
{
    size_t i = seq_hash(c, k) % T->cap;
    while (T->seq[i]) {
        if (T->len[i] == k && memcmp(T->seq[i], c, sizeof(uint16_t) * k) == 0) return i;
        i = (i + 1) % T->cap;
    }
    return i;
}

static int tabu_contains(const tabu_set *T, const series *s)
{
    return T->seq[tabu_find(T, s->c, s->k)] != NULL;
}

static int tabu_grow(tabu_set *T)
{
    tabu_set N;
    if (tabu_init(&N, T->cap * 2)) return -1;
    for (size_t i = 0; i < T->cap; i++) {
        if (!T->seq[i]) continue;
        size_t j = tabu_find(&N, T->seq[i], T->len[i]);
        N.seq[j] = T->seq[i];
        N.len[j] = T->len[i];
        N.size++;
        T->seq[i] = NULL;
    }
    tabu_free(T);
    *T = N;
    return 0;
}

/* Insert a series known not to be in the set. */
static int tabu_insert(tabu_set *T, const series *s)
{
    if (2 * (T->size + 1) > T->cap && tabu_grow(T)) return -1;
    size_t i = tabu_find(T, s->c, s->k);
    T->seq[i] = malloc(sizeof(uint16_t) * (s->k ? s->k : 1));
    if (!T->seq[i]) return -1;
    memcpy(T->seq[i], s->c, sizeof(uint16_t) * s->k);
    T->len[i] = s->k;
    T->size++;
    return 0;
}

/* Top-rank list member. */
typedef struct {
    series s;
    uint8_t *rows;   /* R flags */
    int n;
    double score;
} member;

/* Order of the top-rank list: higher score first, then the smaller series. */
static int above(double sa, const series *a, double sb, const series *b)
{
    if (sa != sb) return sa > sb;
    return series_cmp(a, b) < 0;
}

typedef struct {
    const float *X;
    int R, C;
    const oracle_params *p;
    int nthreads;
    uint64_t rng;
    tabu_set tabu;
    int64_t tabu_hits;
    member *A;       /* archive, kept in top-rank order */
    int nA;
} ga_state;

/* Unused-column draw: a uniform index among the columns not in the series,
 * taken in ascending column order. */
static int draw_unused(ga_state *G, const series *s)
{
    int pick = (int)oracle_uniform(&G->rng, (uint64_t)(G->C - s->k));
    for (int c = 0; c < G->C; c++) {
        int in = 0;
        for (int i = 0; i < s->k; i++)
            if (s->c[i] == c) { in = 1; break; }
        if (in) continue;
        if (pick == 0) return c;
        pick--;
    }
    return -1; /* unreachable for k < C */
}

/* Evaluate a population against the current archive. */
static int eval_population(ga_state *G, const series *pop, int P, uint8_t *rows,
                           int32_t *n, double *score, double *fitness)
{
    int K = G->nA;
    uint8_t *arows = malloc((size_t)(K ? K : 1) * G->R);
    int32_t *aoff = malloc(sizeof(int32_t) * (K + 1));
    uint16_t *acols = malloc(sizeof(uint16_t) * (size_t)(K ? K : 1) * ORACLE_K_LIMIT);
    int32_t *off = malloc(sizeof(int32_t) * (P + 1));
    uint16_t *cols = malloc(sizeof(uint16_t) * (size_t)(P ? P : 1) * ORACLE_K_LIMIT);
    int rc = -1;
    if (!arows || !aoff || !acols || !off || !cols) goto done;
    aoff[0] = 0;
    for (int j = 0; j < K; j++) {
        memcpy(arows + (size_t)j * G->R, G->A[j].rows, G->R);
        memcpy(acols + aoff[j], G->A[j].s.c, sizeof(uint16_t) * G->A[j].s.k);
        aoff[j + 1] = aoff[j] + G->A[j].s.k;
    }
    off[0] = 0;
    for (int i = 0; i < P; i++) {
        memcpy(cols + off[i], pop[i].c, sizeof(uint16_t) * pop[i].k);
        off[i + 1] = off[i] + pop[i].k;
    }
    rc = oracle_evaluate(G->X, G->R, G->C, P, off, cols, K, arows, aoff, acols, G->p,
                         G->nthreads, fitness, n, rows, NULL, score);
done:
    free(arows); free(aoff); free(acols); free(off); free(cols);
    return rc;
}

static int common_rows(const uint8_t *a, const uint8_t *b, int R)
{
    int h = 0;
    for (int r = 0; r < R; r++) h += a[r] & b[r];
    return h;
}

static int archive_has(const ga_state *G, const series *s)
{
    series cs, ca;
    canonical(s, G->p->negative_trends, &cs);
    for (int j = 0; j < G->nA; j++) {
        canonical(&G->A[j].s, G->p->negative_trends, &ca);
        if (series_cmp(&cs, &ca) == 0) return 1;
    }
    return 0;
}

static void archive_remove(ga_state *G, int j)
{
    free(G->A[j].rows);
    for (int i = j; i + 1 < G->nA; i++) G->A[i] = G->A[i + 1];
    G->nA--;
}

static int archive_insert(ga_state *G, const series *s, const uint8_t *rows, int n, double sc)
{
    int pos = 0;
    while (pos < G->nA && above(G->A[pos].score, &G->A[pos].s, sc, s)) pos++;
    for (int i = G->nA; i > pos; i--) G->A[i] = G->A[i - 1];
    G->A[pos].s = *s;
    G->A[pos].rows = malloc(G->R);
    if (!G->A[pos].rows) return -1;
    memcpy(G->A[pos].rows, rows, G->R);
    G->A[pos].n = n;
    G->A[pos].score = sc;
    G->nA++;
    return 0;
}

/* Top-rank list update (steps 3 and 7). */
static int update_archive(ga_state *G, const series *pop, int P, const uint8_t *rows,
                          const int32_t *n, const double *score)
{
    const oracle_params *p = G->p;
    int K = p->archive_size;
    int *cand = malloc(sizeof(int) * (P ? P : 1));
    if (!cand) return -1;
    int nc = 0;
    for (int i = 0; i < P; i++)
        if (score[i] > 0 && !archive_has(G, &pop[i])) cand[nc++] = i;
    /* order candidates: score descending, then series ascending (insertion
     * sort keeps this plain) */
    for (int a = 1; a < nc; a++) {
        int x = cand[a], b = a - 1;
        while (b >= 0 && above(score[x], &pop[x], score[cand[b]], &pop[cand[b]])) {
            cand[b + 1] = cand[b];
            b--;
        }
        cand[b + 1] = x;
    }
    int rc = 0;
    for (int ci = 0; ci < nc; ci++) {
        int i = cand[ci];
        const uint8_t *Si = rows + (size_t)i * G->R;
        if (G->nA == K && !above(score[i], &pop[i], G->A[G->nA - 1].score, &G->A[G->nA - 1].s))
            break;
        int J[ORACLE_K_LIMIT];
        int nJ = 0, beats_all = 1;
        for (int j = 0; j < G->nA; j++) {
            int h = common_rows(Si, G->A[j].rows, G->R);
            int g = count_common_cols(pop[i].c, pop[i].k, G->A[j].s.c, G->A[j].s.k);
            if (overlaps(h, g, n[i], pop[i].k, p->overlap_permille)) {
                J[nJ++] = j;
                if (!above(score[i], &pop[i], G->A[j].score, &G->A[j].s)) beats_all = 0;
            }
        }
        if (nJ > 0 && !beats_all) continue;
        for (int q = nJ - 1; q >= 0; q--) archive_remove(G, J[q]);
        if (archive_insert(G, &pop[i], Si, n[i], score[i])) { rc = -1; break; }
        if (G->nA > K) archive_remove(G, G->nA - 1);
    }
    free(cand);
    return rc;
}

/* Crowding (reading of the exponential penalty for overused columns,
 * Sec. 2.3): a column is overused when more individuals hold it than the
 * mean share ceil(sum k / C); the tournament key is the fitness halved once
 * per overused column the individual holds. use[C] is scratch. */
static void crowding_keys(const series *pop, int P, int C, const double *fit, int32_t *use,
                          double *key)
{
    int64_t ksum = 0;
    memset(use, 0, sizeof(int32_t) * C);
    for (int i = 0; i < P; i++) {
        ksum += pop[i].k;
        for (int q = 0; q < pop[i].k; q++) use[pop[i].c[q]]++;
    }
    int64_t share = (ksum + C - 1) / C;
    for (int i = 0; i < P; i++) {
        int e = 0;
        for (int q = 0; q < pop[i].k; q++) e += use[pop[i].c[q]] > share;
        key[i] = ldexp(fit[i], -e);
    }
}

/* The crowding keys of a population given in CSR form (offsets[P+1], cols)
 * and its fitness, for testing. Returns 0, or -1 for an invalid argument. */
int oracle_crowding_keys(const int32_t *offsets, const uint16_t *cols, int P, int C,
                         const double *fitness, double *keys)
{
    if (P < 0 || C < 1) return -1;
    series *pop = malloc(sizeof(series) * (P ? P : 1));
    int32_t *use = malloc(sizeof(int32_t) * C);
    if (!pop || !use) { free(pop); free(use); return -1; }
    for (int i = 0; i < P; i++) {
        int k = offsets[i + 1] - offsets[i];
        if (!series_valid(cols + offsets[i], k, C)) { free(pop); free(use); return -1; }
        pop[i].k = k;
        memcpy(pop[i].c, cols + offsets[i], sizeof(uint16_t) * k);
    }
    crowding_keys(pop, P, C, fitness, use, keys);
    free(pop);
    free(use);
    return 0;
}

/* Tournament: T uniform draws with replacement; the largest key wins, the
 * lowest index among equal keys. */
static int tournament(ga_state *G, const double *key, int P)
{
    int best = -1;
    for (int d = 0; d < G->p->tournament; d++) {
        int i = (int)oracle_uniform(&G->rng, (uint64_t)P);
        if (best < 0 || key[i] > key[best] || (key[i] == key[best] && i < best)) best = i;
    }
    return best;
}

enum { OP_INSERT, OP_DELETE, OP_SUBST, OP_SWAP, OP_CROSS, OP_COUNT };

/* Weight of operator o (the paper names the five operators, Sec. 2.3, and
 * no probabilities: a parameter, uniform by default). */
static int op_weight(const oracle_params *p, int o)
{
    int any = 0;
    for (int q = 0; q < OP_COUNT; q++) any |= p->op_permille[q];
    return any ? p->op_permille[o] : 200;
}

/* One mutation attempt from the old population (step 5). The operator is
 * drawn among those that apply to the parent (insertion needs k < k_max
 * and k < C, deletion k > k_min, substitution k < C), in proportion to
 * their weights; when none of them has weight the attempt fails (the child
 * is left empty, outside every length range). */
static void mutate(ga_state *G, const series *pop, const double *key, int P, series *child)
{
    const oracle_params *p = G->p;
    const series *I = &pop[tournament(G, key, P)];
    int k = I->k, op;
    int applies[OP_COUNT] = {k < p->k_max && k < G->C, k > p->k_min, k < G->C, 1, 1};
    int total = 0;
    for (int o = 0; o < OP_COUNT; o++) total += applies[o] * op_weight(p, o);
    if (total == 0) {
        child->k = 0;
        return;
    }
    int x = (int)oracle_uniform(&G->rng, (uint64_t)total);
    for (op = 0;; op++) {
        int w = applies[op] * op_weight(p, op);
        if (x < w) break;
        x -= w;
    }
    *child = *I;
    if (op == OP_INSERT) {
        int pos = (int)oracle_uniform(&G->rng, (uint64_t)k + 1);
        int c = draw_unused(G, I);
        for (int i = k; i > pos; i--) child->c[i] = child->c[i - 1];
        child->c[pos] = (uint16_t)c;
        child->k = k + 1;
    } else if (op == OP_DELETE) {
        int pos = (int)oracle_uniform(&G->rng, (uint64_t)k);
        for (int i = pos; i + 1 < k; i++) child->c[i] = child->c[i + 1];
        child->k = k - 1;
    } else if (op == OP_SUBST) {
        int pos = (int)oracle_uniform(&G->rng, (uint64_t)k);
        child->c[pos] = (uint16_t)draw_unused(G, I);
    } else if (op == OP_SWAP) {
        int a = (int)oracle_uniform(&G->rng, (uint64_t)k);
        int b = (int)oracle_uniform(&G->rng, (uint64_t)k - 1);
        if (b >= a) b++;
        uint16_t x = child->c[a];
        child->c[a] = child->c[b];
        child->c[b] = x;
    } else {
        const series *J = &pop[tournament(G, key, P)];
        int a = 1 + (int)oracle_uniform(&G->rng, (uint64_t)k - 1);
        int b = 1 + (int)oracle_uniform(&G->rng, (uint64_t)J->k - 1);
        /* child = I[0:a] followed by the columns of J[b:] it lacks; a child
         * longer than the storage cap is longer than k_max and is only ever
         * length-checked */
        int len = a, stored = a;
        for (int i = b; i < J->k; i++) {
            int in = 0;
            for (int q = 0; q < stored; q++)
                if (child->c[q] == J->c[i]) { in = 1; break; }
            if (in) continue;
            if (stored < ORACLE_K_LIMIT) child->c[stored++] = J->c[i];
            len++;
        }
        child->k = len;
    }
}

/* Operator weights: each 0..1000 and summing to 1000, or all 0. */
static int ops_valid(const oracle_params *p)
{
    int sum = 0;
    for (int o = 0; o < OP_COUNT; o++) {
        if (p->op_permille[o] < 0 || p->op_permille[o] > 1000) return 0;
        sum += p->op_permille[o];
    }
    return sum == 0 || sum == 1000;
}

/* n mutation attempts (step 5) from a population given in CSR form, with
 * tournament keys `key` and the generator seeded with `seed`: child i goes
 * to child_cols[i * ORACLE_K_LIMIT ..], its length to child_len[i] (0 when
 * no weighted operator applied; a crossover child longer than the storage
 * keeps only its first ORACLE_K_LIMIT columns). Exposes the operators for
 * testing. Returns 0, or -1 for an invalid argument. */
int oracle_mutants(const int32_t *offsets, const uint16_t *cols, int P, const double *key,
                   int C, const oracle_params *p, uint64_t seed, int n, int32_t *child_len,
                   uint16_t *child_cols)
{
    if (P < 1 || C < 2 || n < 0 || !p || !ops_valid(p) || p->tournament < 1) return -1;
    series *pop = malloc(sizeof(series) * P);
    if (!pop) return -1;
    for (int i = 0; i < P; i++) {
        int k = offsets[i + 1] - offsets[i];
        if (k < 2 || k > ORACLE_K_LIMIT) { free(pop); return -1; }
        pop[i].k = k;
        memcpy(pop[i].c, cols + offsets[i], sizeof(uint16_t) * k);
    }
    ga_state G;
    memset(&G, 0, sizeof G);
    G.C = C; G.p = p; G.rng = seed;
    for (int i = 0; i < n; i++) {
        series child;
        mutate(&G, pop, key, P, &child);
        child_len[i] = child.k;
        int stored = child.k < ORACLE_K_LIMIT ? child.k : ORACLE_K_LIMIT;
        memcpy(child_cols + (size_t)i * ORACLE_K_LIMIT, child.c, sizeof(uint16_t) * stored);
    }
    free(pop);
    return 0;
}

/* Result of run(); caller-allocated arrays sized by n_out, R and G. */
typedef struct {
    int32_t *count;         /* biclusters written                      */
    int32_t *k;             /* [n_out]                                 */
    uint16_t *cols;         /* [n_out][ORACLE_K_LIMIT]                 */
    int32_t *n;             /* [n_out]                                 */
    double *score;          /* [n_out]                                 */
    uint8_t *rows;          /* [n_out][R] row flags                    */
    int64_t *stats;         /* generations, evaluations, tabu hits, stop reason */
    double *trace;          /* [G][4]: population size, archive size,  */
                            /* best score, cumulative tabu hits        */
} oracle_result;

enum { STOP_GENERATIONS = 1, STOP_TABU = 2, STOP_EXHAUSTED = 3 };

int oracle_run(const float *X, int R, int C, const oracle_params *p, uint64_t seed,
               int nthreads, oracle_result *out)
{
    if (!X || !p || !out || R < 1 || C < 2 || p->k_min < 2 || p->k_max < p->k_min ||
        p->k_max > ORACLE_K_LIMIT || p->k_max > C || p->population < 1 ||
        p->generations < 1 || p->archive_size < 1 || p->archive_size > 64 ||
        p->n_out < 0 || p->tournament < 1 || p->max_attempts < 1 || p->max_tabu_hits < 1 ||
        p->approx_permille < 0 || p->approx_permille > 1000 || !ops_valid(p))
        return -1;
    ga_state G;
    memset(&G, 0, sizeof G);
    G.X = X; G.R = R; G.C = C; G.p = p; G.nthreads = nthreads; G.rng = seed;
    int P = p->population;
    series *pop = malloc(sizeof(series) * P), *next = malloc(sizeof(series) * P);
    uint8_t *rows = malloc((size_t)P * R);
    int32_t *n = malloc(sizeof(int32_t) * P);
    double *score = malloc(sizeof(double) * P), *fit = malloc(sizeof(double) * P);
    double *key = malloc(sizeof(double) * P);
    int32_t *use = malloc(sizeof(int32_t) * C);
    G.A = calloc((size_t)p->archive_size + 2, sizeof(member));
    int rc = -1;
    if (!pop || !next || !rows || !n || !score || !fit || !key || !use || !G.A ||
        tabu_init(&G.tabu, 1024))
        goto done;

    int64_t evaluations = 0;
    int stop = 0;

    /* Step 1: random initial population; a series already seen is redrawn
     * (not a tabu hit). Lengths uniform in [k_min, k_max]; columns by a
     * partial Fisher-Yates shuffle of 0..C-1 (the drawn order is the series). */
    int Pn = 0;
    int *perm = malloc(sizeof(int) * C);
    if (!perm) goto done;
    for (int i = 0; i < P && !stop; i++) {
        int attempts = 0;
        for (;;) {
            if (attempts == p->max_attempts) { stop = STOP_EXHAUSTED; break; }
            attempts++;
            series s;
            s.k = p->k_min + (int)oracle_uniform(&G.rng, (uint64_t)(p->k_max - p->k_min + 1));
            for (int c = 0; c < C; c++) perm[c] = c;
            for (int j = 0; j < s.k; j++) {
                int r = j + (int)oracle_uniform(&G.rng, (uint64_t)(C - j));
                int x = perm[j]; perm[j] = perm[r]; perm[r] = x;
                s.c[j] = (uint16_t)perm[j];
            }
            series cs;
            canonical(&s, p->negative_trends, &cs);
            if (tabu_contains(&G.tabu, &cs)) continue;
            if (tabu_insert(&G.tabu, &cs)) { free(perm); goto done; }
            pop[Pn++] = s;
            break;
        }
    }
    free(perm);

    int g = 0;
    for (;;) {
        /* Steps 2-3 / 7: evaluate the population, then update the top-rank
         * list. */
        if (eval_population(&G, pop, Pn, rows, n, score, fit)) goto done;
        evaluations += Pn;
        if (update_archive(&G, pop, Pn, rows, n, score)) goto done;
        if (out->trace) {
            double *tr = out->trace + (size_t)g * 4;
            tr[0] = Pn;
            tr[1] = G.nA;
            tr[2] = G.nA ? G.A[0].score : 0.0;
            tr[3] = (double)G.tabu_hits;
        }
        g++;
        if (stop) break;
        if (g == p->generations) { stop = STOP_GENERATIONS; break; }

        /* Step 4: elitism -- the top-rank list, at most half the population. */
        int Nn = 0;
        int ne = G.nA < P / 2 ? G.nA : P / 2;
        for (int j = 0; j < ne; j++) next[Nn++] = G.A[j].s;

        crowding_keys(pop, Pn, C, fit, use, key);

        /* Step 5: replenish with mutants; step 6: tabu hits. */
        while (Nn < P && !stop) {
            int attempts = 0;
            for (;;) {
                if (attempts == p->max_attempts) { stop = STOP_EXHAUSTED; break; }
                attempts++;
                series child, cs;
                mutate(&G, pop, key, Pn, &child);
                if (child.k < p->k_min || child.k > p->k_max) continue;
                canonical(&child, p->negative_trends, &cs);
                if (tabu_contains(&G.tabu, &cs)) {
                    G.tabu_hits++;
                    if (G.tabu_hits >= p->max_tabu_hits) { stop = STOP_TABU; break; }
                    continue;
                }
                if (tabu_insert(&G.tabu, &cs)) goto done;
                next[Nn++] = child;
                break;
            }
        }
        if (stop) break;  /* step 6: go to the final step without scoring */
        series *tmp = pop; pop = next; next = tmp;
        Pn = Nn;
    }

    /* Step 9: evaluate the top-rank list alone and report the first b. */
    {
        int nb = G.nA < p->n_out ? G.nA : p->n_out;
        series *fin = malloc(sizeof(series) * (nb ? nb : 1));
        uint8_t *frows = malloc((size_t)(nb ? nb : 1) * R);
        int32_t *fn = malloc(sizeof(int32_t) * (nb ? nb : 1));
        double *fs = malloc(sizeof(double) * (nb ? nb : 1));
        double *ff = malloc(sizeof(double) * (nb ? nb : 1));
        int nA = G.nA;
        if (!fin || !frows || !fn || !fs || !ff) goto fin_done;
        for (int j = 0; j < nb; j++) fin[j] = G.A[j].s;
        G.nA = 0;  /* against an empty archive */
        if (eval_population(&G, fin, nb, frows, fn, fs, ff)) { G.nA = nA; goto fin_done; }
        G.nA = nA;
        *out->count = nb;
        for (int j = 0; j < nb; j++) {
            out->k[j] = fin[j].k;
            memcpy(out->cols + (size_t)j * ORACLE_K_LIMIT, fin[j].c, sizeof(uint16_t) * fin[j].k);
            out->n[j] = fn[j];
            out->score[j] = fs[j];
            memcpy(out->rows + (size_t)j * R, frows + (size_t)j * R, R);
        }
        out->stats[0] = g;
        out->stats[1] = evaluations;
        out->stats[2] = G.tabu_hits;
        out->stats[3] = stop;
        rc = 0;
    fin_done:
        free(fin); free(frows); free(fn); free(fs); free(ff);
    }
done:
    if (G.A) {
        for (int j = 0; j < G.nA; j++) free(G.A[j].rows);
        free(G.A);
    }
    tabu_free(&G.tabu);
    free(pop); free(next); free(rows); free(n); free(score); free(fit); free(key); free(use);
    return rc;
}
