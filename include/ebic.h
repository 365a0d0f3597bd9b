/*
 * ebic.h -- C ABI of the MI355X (gfx950) EBIC evaluation library.
 *
 * EBIC (evolutionary biclustering; arXiv 2105.01196, "EBIC.JL - an Efficient
 * Implementation of Evolutionary Biclustering Algorithm in Julia") searches a
 * numeric matrix for biclusters: a set of rows together with an ordered series
 * of columns such that every row follows the series' increasing order
 * (Sec. 2.3, EBIC paragraph). Each individual of the evolutionary search is
 * such a column series; scoring an individual means counting the rows that
 * follow its trend (Sec. 2.4, steps 2-3 and 7), then turning that count into
 * a fitness with a size score and a penalty for overlapping biclusters
 * already on the top-rank list. The final step reports the supporting row
 * indices of the top-rank list (Sec. 2.4, step 9).
 *
 * Definitions used throughout (the paper prints no formula; these are the
 * readings this library implements):
 *   row order    column a precedes column b in row r when X[r,a] < X[r,b], or
 *                X[r,a] == X[r,b] and a < b (IEEE compare, so -0 == +0);
 *   up-steps     u_r = #{ j < k-1 : c_j precedes c_{j+1} in row r };
 *   tolerance    t(k) = floor((k-1) * (1000 - approx_permille) / 1000);
 *   support      r fits when (k-1-u_r) <= t(k), or, with negative trends on,
 *                u_r <= t(k); n = number of fitting rows;
 *   size score   s = n * 2^k when n >= min_rows and k >= k_score_min, else 0;
 *   overlap      for archive member j: h_j = rows shared with the member's
 *                support, g_j = columns shared with its series; the member
 *                overlaps when 1000*h_j*g_j > overlap_permille*n*k (64-bit);
 *   fitness      s * 2^-m, m = number of overlapping members (exact FP64).
 *
 * Conventions:
 *   - Every pointer named d_* is device memory owned by the caller; h_* is
 *     host memory owned by the caller. The library keeps no reference to
 *     either after a call returns, except where stated.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked "asynchronous" only enqueue work on it.
 *   - Return values are EBIC_OK (0), EBIC_PENDING (1) or a negative EBIC_ERR_*
 *     code; ebic_last_error() gives a message for the calling thread. No C++
 *     exception crosses this interface.
 *   - Rows are padded to a multiple of 64 (rows_pad); a support bitmap holds
 *     W = rows_pad/64 64-bit words, bit (r % 64) of word (r / 64) for row r.
 *     Bits of padding rows are always 0.
 */
#ifndef EBIC_H
#define EBIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBIC_VERSION 200 /* 0.2.0: ebic_params gained op_permille */

#define EBIC_OK 0
#define EBIC_PENDING 1
#define EBIC_ERR_INVALID_ARG (-1)
#define EBIC_ERR_NONFINITE (-2)
#define EBIC_ERR_OOM (-3)
#define EBIC_ERR_DEVICE (-4)
#define EBIC_ERR_CAPACITY (-5)

#define EBIC_MAX_K 512        /* longest series                          */
#define EBIC_MAX_ARCHIVE 64   /* largest top-rank list                   */
#define EBIC_MAX_COLS 16384   /* widest matrix                           */
#define EBIC_MAX_ROWS (1 << 26)  /* and cols * rows_pad < 2^31 */

/* Method parameters; integers only, so that every result is exact. The
 * paper names negative trends on/off, the approximate-trend threshold, the
 * allowed overlap, the number of iterations and the number of biclusters as
 * its parameters (Sec. 2.4, last paragraph). */
typedef struct ebic_params {
    int32_t approx_permille;   /* approximate-trend threshold a, 0..1000 (1000 = exact) */
    int32_t negative_trends;   /* 0/1: rows following the reversed series also fit    */
    int32_t overlap_permille;  /* allowed overlap theta, 0..1000                      */
    int32_t min_rows;          /* fewer fitting rows score 0                           */
    int32_t k_score_min;       /* fewer columns score 0                                */
    int32_t k_min, k_max;      /* series lengths the search may create (ebic_run)      */
    int32_t archive_size;      /* top-rank list capacity K (ebic_run), <= 64           */
    int32_t n_out;             /* biclusters returned by ebic_run                      */
    int32_t population;        /* individuals per generation (ebic_run)                */
    int32_t generations;       /* populations evaluated at most (ebic_run)             */
    int32_t max_tabu_hits;     /* rejected mutants that end the run (ebic_run)         */
    int32_t tournament;        /* tournament size (ebic_run)                           */
    int32_t max_attempts;      /* mutation attempts per population slot (ebic_run)     */
    int32_t tie_rule;          /* equal values in a row (EBIC_TIE_*)                    */
    int32_t op_permille[5];    /* weights of the mutation operators (ebic_run), per
                                  mille, in the order insertion, deletion,
                                  substitution, swap, crossover (Sec. 2.3 names the
                                  five): each 0..1000 and summing to 1000, or all 0
                                  for 200 each. Each attempt draws one operator among
                                  those that apply to the parent (insertion needs
                                  k < k_max and k < cols, deletion k > k_min,
                                  substitution k < cols) in proportion to its weight;
                                  with no weighted operator applicable the attempt
                                  fails                                                   */
} ebic_params;

/* Equal values in a row (the paper does not say how ties count; a step of a
 * series goes from column a to column b):
 * EBIC_TIE_INDEX    the smaller column index comes first: a tie is an up-step
 *                   when a < b, a down-step otherwise (every step is one or
 *                   the other);
 * EBIC_TIE_STRICT   a tie is neither: it breaks the increasing and the
 *                   decreasing trend alike;
 * EBIC_TIE_LOOSE    a tie is both: it fits either trend.
 * The pair table serves EBIC_TIE_INDEX; with the strict table as well
 * (ebic_pairs_strict_prepare) the batched evaluator scores the other two
 * rules in the pair form too, else in the gather form. */
#define EBIC_TIE_INDEX 0
#define EBIC_TIE_STRICT 1
#define EBIC_TIE_LOOSE 2

/* A prepared matrix (ebic_matrix_prepare). */
typedef struct ebic_matrix {
    const uint16_t *d_ranks;   /* cols x rows_pad, column-major: for each cell the
                                  number of cells of its row with a smaller value
                                  (equal values share it), 0..cols-1              */
    int32_t rows, cols, rows_pad;
    const uint64_t *d_pairs;   /* optional pair table (ebic_pairs_prepare) or NULL */
    const uint64_t *d_pairs_strict; /* optional strict pair table
                                  (ebic_pairs_strict_prepare) or NULL: with d_pairs
                                  it lets the strict and loose tie rules take the
                                  pair form too                                   */
} ebic_matrix;

/* A population in compressed (CSR) form, as the paper sends it to the GPU
 * (Sec. 2.4, step 2): individual i is d_cols[d_offsets[i] .. d_offsets[i+1]). */
typedef struct ebic_population {
    int32_t size;              /* P >= 0 */
    int32_t length;            /* entries in d_cols; offsets beyond it mark the
                                  individual invalid */
    const int32_t *d_offsets;  /* P + 1 */
    const uint16_t *d_cols;    /* column indices, series order */
    const int32_t *d_order;    /* optional processing order for the batched
                                  evaluator: a permutation of 0..P-1, longest
                                  series first balances the load; NULL = 0..P-1.
                                  Results never depend on it. */
} ebic_population;

/* The top-rank list the overlap penalty is taken against. */
typedef struct ebic_archive {
    int32_t size;              /* K, 0..EBIC_MAX_ARCHIVE */
    int32_t length;            /* entries in d_cols */
    const uint64_t *d_support; /* K x W support bitmaps */
    const int32_t *d_offsets;  /* K + 1, CSR of the members' series */
    const uint16_t *d_cols;
} ebic_archive;

/* Outputs of an evaluation; all device arrays owned by the caller. */
typedef struct ebic_eval_out {
    double *d_fitness;         /* P: s * 2^-m; -1.0 for an invalid individual     */
    int32_t *d_count;          /* P: n; -1 for an invalid individual              */
    uint64_t *d_support;       /* P x W support bitmaps, or NULL                   */
    int32_t *d_overlap;        /* P x K rows shared with each member (h), or NULL */
} ebic_eval_out;

int ebic_version(void);
const char *ebic_last_error(void);

/* Bytes of the prepared rank matrix: cols * rows_pad * 2. */
size_t ebic_matrix_bytes(int32_t rows, int32_t cols);

/* Matrix ingest. Reads a float32 rows x cols row-major matrix d_x and writes
 * m->d_ranks (ebic_matrix_bytes(rows, cols) bytes, caller-owned): for every
 * row, the rank of each column in the row order defined above. Comparing two
 * columns' ranks is then exactly the row order of the paper's trend test,
 * which the evaluators read in column-major order. The paper keeps the matrix
 * on the GPU for the whole run and sends only populations per generation
 * (Sec. 2.4, step 2). Fills *m. Synchronous on `stream` (it waits for the
 * finiteness check). Errors: EBIC_ERR_INVALID_ARG for null pointers or sizes
 * outside 1..EBIC_MAX_ROWS x 2..EBIC_MAX_COLS; EBIC_ERR_NONFINITE if any value
 * is NaN or infinite (m->d_ranks is then unspecified). */
int ebic_matrix_prepare(const float *d_x, int32_t rows, int32_t cols, uint16_t *d_ranks,
                        ebic_matrix *m, void *stream);

/* Population upload: validates a host CSR population (every series has
 * 2..EBIC_MAX_K distinct columns below `cols`) and copies it into the
 * caller's device arrays d_offsets (P+1 int32) and d_cols (offsets[P]
 * uint16). Sec. 2.4, step 2 (the population is packed into one compact
 * array before it goes to the GPU). Synchronous. EBIC_ERR_INVALID_ARG on an invalid series (nothing
 * is copied). */
int ebic_population_upload(const int32_t *h_offsets, const uint16_t *h_cols, int32_t size,
                           int32_t cols, int32_t *d_offsets, uint16_t *d_cols, void *stream);

/* Plain evaluation, one launch for one population (Sec. 2.4, steps 2-3 and 7:
 * score every individual, counting its trend-preserving rows). For each
 * individual: support bitmap, n, h per archive member and fitness, as defined
 * above. Asynchronous. Host-side errors (EBIC_ERR_INVALID_ARG, nothing
 * enqueued): null required pointers, archive size outside 0..64, parameters
 * out of range. An individual whose length is outside 2..EBIC_MAX_K, or
 * whose columns are out of range or repeated, is marked invalid on the device
 * (count -1, fitness -1.0, support and overlap 0) and never read out of
 * bounds. */
int ebic_evaluate(const ebic_matrix *m, const ebic_population *pop, const ebic_archive *arch,
                  const ebic_params *p, const ebic_eval_out *out, void *stream);

/* Bytes of the pair-comparison table: C(C-1)/2 pairs x
 * ebic_pairs_words(rows) x 8 (0 when rows < 1 or cols < 2). */
size_t ebic_pairs_bytes(int32_t rows, int32_t cols);
/* Words per pair in the table: rows_pad/64 rounded up to a multiple of 16,
 * so every pair's bitmap starts on a 128-byte line (0 when rows < 1). */
int32_t ebic_pairs_words(int32_t rows);

/* Pair-comparison table (used by the batched evaluator). For every
 * unordered column pair lo < hi, the support-style bitmap (W = rows_pad/64
 * words) of the rows in which lo precedes hi, at d_pairs[pair * S + word]
 * with S = ebic_pairs_words(rows) and pair = lo*C - lo*(lo+1)/2 + (hi-lo-1);
 * words W..S-1 of a pair are not written. A series step c_j -> c_{j+1} keeps
 * the increasing trend (Sec. 2.3) exactly in the rows of its pair's bitmap,
 * inverted when c_j > c_{j+1}, so the trend test reduces to bitwise work.
 * d_pairs (ebic_pairs_bytes bytes) is caller-owned; sets m->d_pairs.
 * Asynchronous. EBIC_ERR_INVALID_ARG for a NULL or unprepared matrix. */
int ebic_pairs_prepare(ebic_matrix *m, uint64_t *d_pairs, void *stream);
/* Strict pair table: as ebic_pairs_prepare (same layout and size), with the
 * rows in which lo's value is strictly smaller than hi's. A tie is then
 * neither bit's, so the two tables tell the three outcomes of a compare
 * apart: a step keeps the increasing trend under the strict rule (ties
 * break both trends) exactly in the strict table's rows, under the loose
 * rule (ties keep both) in the other's, inverted for a step against the
 * column order as above. d_pairs_strict (ebic_pairs_bytes bytes) is
 * caller-owned; sets m->d_pairs_strict. Asynchronous. EBIC_ERR_INVALID_ARG
 * for a NULL or unprepared matrix. */
int ebic_pairs_strict_prepare(ebic_matrix *m, uint64_t *d_pairs_strict, void *stream);

/* One evaluation job of a batch: a matrix, a population, the archive it is
 * penalised against, the parameters and the outputs (as for ebic_evaluate;
 * out.d_support may be NULL, the batch then keeps its own scratch). */
typedef struct ebic_job {
    ebic_matrix matrix;
    ebic_population population;
    ebic_archive archive;
    ebic_params params;
    ebic_eval_out out;
} ebic_job;

#define EBIC_BATCH_GRAPH 1   /* replay the launch as a prebuilt HIP graph */
#define EBIC_BATCH_GATHER 2  /* ignore pair tables, use the gather form    */
#define EBIC_BATCH_TUNE 4    /* autotune the item shape on the first run   */

typedef struct ebic_batch ebic_batch;

/* Batched evaluation (Sec. 2.4, steps 2-3 and 7, for several populations
 * at once): every individual of every job in one kernel launch (its own
 * waves of a workgroup count and reduce each individual), each job with its own
 * matrix (pair-table form when the matrix has a table, else the gather
 * form), archive and parameters. Results are identical, bit for bit, to
 * ebic_evaluate on each job alone. create copies the job table to the
 * device (the caller's buffers are referenced, not copied: they must stay
 * valid until destroy; their contents may change between runs); run enqueues
 * one evaluation of all jobs on `stream` (asynchronous); destroy frees the
 * batch. Errors: EBIC_ERR_INVALID_ARG (as ebic_evaluate, per job),
 * EBIC_ERR_OOM, EBIC_ERR_DEVICE. Runs of one batch must not overlap. */
int ebic_batch_create(const ebic_job *jobs, int32_t njobs, int32_t flags, ebic_batch **out);
/* Item shape of the kernel: a wave takes one item of its individual's rows,
 * i.e. chunks_per_item groups (1, 2 or 4) of words_per_lane (1 or 2) chunks
 * of 4,096 rows, walking a group's chunks together (each lane holds one
 * 64-row word of each), with loads_in_flight (2 or 4, or 8 with one word
 * per lane) pair-bitmap loads issued per group of steps (an individual with
 * more than 16 items gets
 * proportionally larger ones). With EBIC_BATCH_TUNE the first run times every candidate
 * shape on the batch's own inputs, waits for the timings (that run is
 * synchronous), keeps the fastest, and caches the choice per batch shape in
 * the process and, when the environment variable EBIC_TUNE_CACHE names a
 * file, in that JSON file. Before tuning or pinning, a batch takes four
 * loads in flight, one word per lane and, per job, one chunk group per item
 * up to two chunks, two up to four, else four; ebic_batch_tuning reports that
 * default as chunks_per_item 0. ebic_batch_tuning reports the shape in use;
 * any output pointer may be NULL. */
int ebic_batch_tuning(ebic_batch *b, int32_t *chunks_per_item, int32_t *loads_in_flight,
                      int32_t *words_per_lane);
/* Pins the item shape, e.g. one reported by ebic_batch_tuning in an earlier
 * process; later runs use it and do not tune. Results never depend on the
 * shape. Synchronous; call between runs. Errors: EBIC_ERR_INVALID_ARG for a
 * shape outside the values above. */
int ebic_batch_set_tuning(ebic_batch *b, int32_t chunks_per_item, int32_t loads_in_flight,
                          int32_t words_per_lane);
int ebic_batch_run(ebic_batch *b, void *stream);
int ebic_batch_destroy(ebic_batch *b);

/* Kernel timing of a batch (metrics). ebic_batch_profile(b, n) makes the
 * next n runs record HIP events around the kernel (or the graph) on the
 * run's stream (n = 0 turns it off). ebic_batch_timings waits for the
 * recorded runs and writes up to *n per-run times in milliseconds to ms;
 * *n returns the number written. */
int ebic_batch_profile(ebic_batch *b, int32_t n);
int ebic_batch_timings(ebic_batch *b, float *ms, int32_t *n);

/* One-shot batched evaluation: create, run, wait, destroy. Synchronous. */
int ebic_evaluate_batched(const ebic_job *jobs, int32_t njobs, void *stream);

/* For callers that cannot allocate device or pinned memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same evaluation as ebic_evaluate_batched, bit for bit (the same kernel in
 * the same untuned item shape), with no hipMalloc, hipFree, hipHostMalloc or
 * other allocating call. The job table goes to a fixed device array of the
 * library (16 KiB per device, held until the process ends), so at most
 * EBIC_NOALLOC_MAX_JOBS jobs per call, and every job must bring its support
 * output (out.d_support; the others as for ebic_evaluate_batched). The
 * array's address is looked up once per device on the first call there.
 * Calls on one device run one at a time (a mutex per device, held until the
 * kernel has finished); the array keeps the last call's table, which no call
 * reads before writing it. Synchronous on `stream`. Errors: EBIC_ERR_INVALID_ARG
 * for more jobs than the limit, a missing support output or a bad job (the
 * outputs are then untouched); EBIC_ERR_DEVICE for a HIP failure. */
#define EBIC_NOALLOC_MAX_JOBS 64
int ebic_evaluate_batched_noalloc(const ebic_job *jobs, int32_t njobs, void *stream);

/* One bicluster of a run: rows ascending, columns in series order. */
typedef struct ebic_bicluster {
    int32_t n_rows;
    const int32_t *rows;
    int32_t n_cols;
    const uint16_t *cols;
    double score;              /* size score s = n * 2^k */
    const uint8_t *row_dir;    /* per row: 0 = follows the series' increasing trend
                                  (within the tolerance), 1 = only the reversed one */
} ebic_bicluster;

#define EBIC_STOP_GENERATIONS 1 /* the iteration limit was reached            */
#define EBIC_STOP_TABU 2        /* the tabu-hit threshold was reached         */
#define EBIC_STOP_EXHAUSTED 3   /* a population slot ran out of attempts      */

/* Result of ebic_run; library-owned, released with ebic_result_free. */
typedef struct ebic_result {
    int32_t count;                      /* biclusters returned (<= n_out)       */
    const ebic_bicluster *biclusters;   /* top-rank order: score desc, series asc */
    int32_t generations;                /* populations evaluated                */
    int64_t evaluations;                /* individuals evaluated                */
    int64_t tabu_hits;
    int32_t stop_reason;                /* EBIC_STOP_*                           */
    const double *trace;                /* generations x 4: population size,
                                           top-rank size, best score, tabu hits
                                           so far (after each evaluation)       */
} ebic_result;

/* Device memory for the method's runs (ebic_run, sessions): alloc returns
 * `bytes` of device memory usable on `stream` (NULL on failure, which the
 * call reports as EBIC_ERR_OOM), release returns it. A NULL allocator means
 * hipMalloc / hipFree. Every device buffer of a run (matrix, ranks, pair
 * table, populations, outputs, archive, job table) comes from it; pinned
 * host staging does not. */
typedef struct ebic_allocator {
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*release)(void *ctx, void *ptr, void *stream);
    void *ctx;
} ebic_allocator;

/* The whole method (Sec. 2.4, steps 1-9) on a host float32 rows x cols
 * row-major matrix: random initial population of series (step 1), GPU
 * evaluation of every population (steps 2 and 7), top-rank list update
 * (steps 3 and 7), elitism (step 4), tournament selection with the
 * column-overuse penalty and mutation (step 5), tabu list and tabu-hit stop
 * (step 6), and the final supports of the top-rank list (step 9). All draws
 * come from one SplitMix64 stream seeded with `seed`; the same seed gives the
 * same result. The host parts follow the readings stated at the top of this
 * file and in the parameter comments; evaluation uses the pair table when
 * it fits in a quarter of the free device memory, else the gather form
 * (identical results). Device memory comes from `alloc` (NULL: hipMalloc)
 * and is returned before the call ends. Each bicluster carries its rows'
 * directions. Synchronous on `stream`. Errors: EBIC_ERR_INVALID_ARG (parameters:
 * 2 <= k_min <= k_max <= min(cols, 512), population >= 1, generations >= 1,
 * 1 <= archive_size <= 64, tournament >= 1, max_attempts >= 1,
 * max_tabu_hits >= 1, n_out >= 0, op_permille as above), EBIC_ERR_NONFINITE, EBIC_ERR_OOM,
 * EBIC_ERR_DEVICE. On success *out is set. */
int ebic_run(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p, uint64_t seed,
             const ebic_allocator *alloc, void *stream, ebic_result **out);

/* ebic_run with every generation after the first on the device (Sec. 2.4,
 * steps 3-7; the paper names moving the CPU parts to the GPU as future work,
 * Sec. 4): the top-rank list update, elitism, the crowding keys, the
 * tournaments and mutations, the tabu set (a hash table of canonical series
 * in device memory) and the tabu-hit and attempt limits all run as kernels;
 * between generations the host reads only a status block. Step 1 (the first
 * population) and step 9 (the final supports) run as in ebic_run. The draws
 * are ebic_run's: SplitMix64 gives any draw of the stream directly, and an
 * attempt's draws do not depend on whether earlier children were rejected,
 * so each generation's attempts are drawn, built and checked in parallel and
 * the loop's rules are then applied in attempt order. The result equals
 * ebic_run's for the same seed (rows, series, scores, trace, counts).
 * Arguments, ownership and errors as for ebic_run; besides,
 * EBIC_ERR_INVALID_ARG for tournament > 16 or population > 8192, and
 * EBIC_ERR_CAPACITY when the tabu set for population * generations series
 * would take more than half the free device memory. */
int ebic_run_device(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                    uint64_t seed, const ebic_allocator *alloc, void *stream, ebic_result **out);
void ebic_result_free(ebic_result *r);

/* Clustering error (Sec. 2.2, Eq. 1) of detected biclusters against a
 * ground truth on a rows x cols matrix, for scoring recovery: the confusion
 * matrix counts the cells each detected bicluster shares with each true one
 * (rows x columns, so |rows ∩ rows'| * |cols ∩ cols'|), D_max is the largest
 * total of a one-to-one assignment between the two sets (Munkres), and U
 * collects every cell covered by any bicluster of either set. *score = D_max/|U|
 * (1 = perfect match, 0 = nothing shared: the paper's text reads CE this
 * way); *ce = (|U| - D_max)/|U|, Eq. 1 as printed. Both sets empty (or all
 * biclusters empty): score 1, ce 0. Only n_rows/rows/n_cols/cols of each
 * bicluster are read (e.g. straight from an ebic_result); order and repeats
 * do not matter. Host-only, synchronous. Errors: EBIC_ERR_INVALID_ARG (NULL,
 * negative counts, an index outside the matrix). */
int ebic_ce_score(const ebic_bicluster *found, int32_t n_found, const ebic_bicluster *truth,
                  int32_t n_truth, int32_t rows, int32_t cols, double *score, double *ce);

/* A run of the method that advances in steps and can be checkpointed: the
 * same computation as ebic_run, whose result it reproduces bit for bit,
 * however the steps are split and wherever it is checkpointed and restored.
 * create copies the matrix, ingests it and draws the first population
 * (step 1). step performs up to `steps` evaluations (each one population
 * scored against the top-rank list and the host steps that follow, or the
 * final scoring of the top-rank list, step 9) and sets *done once the run
 * has finished. checkpoint serialises the run's host state between steps
 * (parameters, generator state, generation, tabu list and hits, top-rank
 * list with supports, population, trace, and a hash of the matrix): with
 * buf NULL it sets *bytes to the size needed; else *bytes must be at least
 * that size and receives the size written. restore rebuilds a session from
 * a checkpoint and the same matrix (EBIC_ERR_INVALID_ARG for a malformed
 * checkpoint or another matrix). result returns the run's result once done
 * (caller frees it with ebic_result_free). The allocator, when given, must
 * outlive the session. Errors as ebic_run. */
typedef struct ebic_session ebic_session;
int ebic_session_create(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                        uint64_t seed, const ebic_allocator *alloc, void *stream,
                        ebic_session **out);
int ebic_session_step(ebic_session *s, int32_t steps, int32_t *done);
int ebic_session_checkpoint(ebic_session *s, void *buf, size_t *bytes);
int ebic_session_restore(const float *h_x, int32_t rows, int32_t cols, const void *buf,
                         size_t bytes, const ebic_allocator *alloc, void *stream,
                         ebic_session **out);
int ebic_session_result(ebic_session *s, ebic_result **out);
void ebic_session_free(ebic_session *s);

/* Job server: continuous batching of many runs of the method (each as in
 * ebic_run) on one GPU. A scheduler thread admits submitted jobs in arrival
 * order while their device footprint (matrix, ranks, pair table when it
 * takes at most an eighth of the budget, population, outputs, archive) fits
 * in the HBM budget and a slot is free; every admitted job keeps its state
 * resident on the device. Preparer threads set admitted jobs up (upload,
 * ranks, pair table, first population) on streams of their own while the
 * scheduler keeps ticking; a prepared job joins at the next tick. Each tick
 * scores the current populations of the jobs that want scores in one
 * batched launch; each job's host steps then run as a task of their own, and
 * the job joins the next tick once they are done. If asked for, a job with a
 * large population (device_loop_population) instead goes to a runner thread,
 * which sets it up and runs its generations on the device as
 * ebic_run_device does (its host steps would hold the ticks back); its
 * footprint then also counts the device loop's memory. A finished job frees its memory and slot, and
 * queued jobs are admitted at the next tick. Each job's result is identical to ebic_run with the same
 * matrix, parameters and seed. */
typedef struct ebic_server ebic_server;

typedef struct ebic_server_config {
    size_t hbm_budget;      /* bytes of device memory jobs may hold; 0 = 80% of free */
    int32_t max_active;     /* jobs resident at once; 0 = 64                         */
    int32_t device_loop_population; /* jobs with at least this population (and
                               within ebic_run_device's limits) run as device
                               loops on runner threads; 0 = none              */
    int32_t device_loop_runners;    /* runner threads (each with a stream); 0 = 2 */
} ebic_server_config;

typedef struct ebic_server_metrics {
    int64_t submitted, completed, failed, queued, active;
    int64_t evaluations;        /* individuals scored by completed jobs        */
    int64_t ticks;              /* batched launches                            */
    double p50_latency_s;       /* submit -> result, completed jobs            */
    double p99_latency_s;
    double mean_latency_s;
    double busy_s;              /* time with at least one active job           */
    size_t hbm_in_use, hbm_budget;
    double stage_s;             /* ticks' host packing                         */
    double device_s;            /* ticks' upload, launch, download and wait    */
    double host_s;              /* jobs' host steps (summed over worker tasks) */
    double setup_s;             /* admitted jobs' setup, beside the ticks      */
    double release_s;           /* ended jobs' frees                           */
    int64_t device_loop_jobs;   /* jobs admitted to the runners                */
    double device_loop_s;       /* runners' time on their jobs, summed         */
} ebic_server_metrics;

/* Creates the server on the current device; the scheduler and each
 * preparer thread use a stream of their own. Errors: EBIC_ERR_INVALID_ARG, EBIC_ERR_DEVICE. */
int ebic_server_create(const ebic_server_config *cfg, ebic_server **out);
/* Queues a job (the host matrix is copied before the call returns, by
 * several threads when it is large; parameters validated as for ebic_run);
 * never waits for the GPU. *job_id identifies it. Errors:
 * EBIC_ERR_INVALID_ARG, EBIC_ERR_OOM (no host memory for the copy). A job
 * whose footprint exceeds the whole budget fails with EBIC_ERR_CAPACITY when
 * the scheduler reaches it. */
int ebic_server_submit(ebic_server *s, const float *h_x, int32_t rows, int32_t cols,
                       const ebic_params *p, uint64_t seed, int64_t *job_id);
/* EBIC_PENDING while the job is queued or running; EBIC_OK with *out set
 * (caller frees it with ebic_result_free; the job is then forgotten); or the
 * job's error. */
int ebic_server_poll(ebic_server *s, int64_t job_id, ebic_result **out);
/* As poll, but blocks until the job has finished. */
int ebic_server_wait(ebic_server *s, int64_t job_id, ebic_result **out);
int ebic_server_stats(ebic_server *s, ebic_server_metrics *out);
/* Finishes the active jobs, fails the queued ones, joins the scheduler and
 * frees everything (unclaimed results included). */
int ebic_server_destroy(ebic_server *s);

/* Support compaction (Sec. 2.4, step 9: the trend-preserving rows' indices of
 * the top-rank list). For each of n_sel selected individuals sel[i] of a
 * P x W support array, writes its row indices in ascending order to
 * d_rows[d_row_offsets[i] .. d_row_offsets[i+1]). d_row_offsets (n_sel + 1,
 * caller-computed from the counts) bounds every write: an individual with more
 * rows than its slot is cut to the slot. Asynchronous. */
int ebic_support_rows(const uint64_t *d_support, int32_t size, int32_t words,
                      const int32_t *d_sel, int32_t n_sel, const int32_t *d_row_offsets,
                      int32_t *d_rows, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* EBIC_H */
