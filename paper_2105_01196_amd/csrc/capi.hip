// C ABI entry points: argument validation, error reporting, launches.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace ebic {

namespace {
thread_local char t_error[512] = "";
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_error, sizeof t_error, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { t_error[0] = 0; }

int check_hip(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(EBIC_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return fail(EBIC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_eval_params(const ebic_params *p) {
    if (!p) return fail(EBIC_ERR_INVALID_ARG, "params is NULL");
    if (p->approx_permille < 0 || p->approx_permille > 1000)
        return fail(EBIC_ERR_INVALID_ARG, "approx_permille %d outside 0..1000", p->approx_permille);
    if (p->overlap_permille < 0 || p->overlap_permille > 1000)
        return fail(EBIC_ERR_INVALID_ARG, "overlap_permille %d outside 0..1000",
                    p->overlap_permille);
    if (p->negative_trends != 0 && p->negative_trends != 1)
        return fail(EBIC_ERR_INVALID_ARG, "negative_trends must be 0 or 1");
    if (p->min_rows < 0 || p->k_score_min < 0)
        return fail(EBIC_ERR_INVALID_ARG, "min_rows and k_score_min must be >= 0");
    if (p->tie_rule < EBIC_TIE_INDEX || p->tie_rule > EBIC_TIE_LOOSE)
        return fail(EBIC_ERR_INVALID_ARG, "tie_rule %d is not an EBIC_TIE_* value", p->tie_rule);
    return EBIC_OK;
}

namespace {
std::mutex g_flag_mu;
std::vector<std::vector<int *>> g_free_flags;  // per device
constexpr int kFlagBlock = 64;                 // words per allocation
}  // namespace

int acquire_flag(int **flag, int *device) {
    int dev = 0;
    EBIC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_flag_mu);
    if ((int)g_free_flags.size() <= dev) g_free_flags.resize(dev + 1);
    std::vector<int *> &free_list = g_free_flags[dev];
    if (free_list.empty()) {
        void *p = nullptr;
        EBIC_HIP(hipMalloc(&p, kFlagBlock * sizeof(int)));
        for (int i = kFlagBlock; i-- > 0;) free_list.push_back(static_cast<int *>(p) + i);
    }
    *flag = free_list.back();
    free_list.pop_back();
    *device = dev;
    return EBIC_OK;
}

void release_flag(int *flag, int device) {
    std::lock_guard<std::mutex> lock(g_flag_mu);
    g_free_flags[device].push_back(flag);
}

static int check_matrix(const ebic_matrix *m) {
    if (!m || !m->d_ranks) return fail(EBIC_ERR_INVALID_ARG, "matrix or its ranks is NULL");
    if (m->rows < 1 || m->rows > EBIC_MAX_ROWS || m->cols < 2 || m->cols > EBIC_MAX_COLS ||
        m->rows_pad != rows_padded(m->rows) || (int64_t)m->cols * m->rows_pad > INT32_MAX)
        return fail(EBIC_ERR_INVALID_ARG, "matrix shape %d x %d (rows_pad %d) not supported",
                    m->rows, m->cols, m->rows_pad);
    return EBIC_OK;
}

static int check_archive(const ebic_archive *a) {
    if (!a) return EBIC_OK;
    if (a->size < 0 || a->size > EBIC_MAX_ARCHIVE)
        return fail(EBIC_ERR_INVALID_ARG, "archive size %d outside 0..%d", a->size,
                    EBIC_MAX_ARCHIVE);
    if (a->size > 0 && (!a->d_support || !a->d_offsets || !a->d_cols || a->length < 0))
        return fail(EBIC_ERR_INVALID_ARG, "archive arrays are NULL");
    return EBIC_OK;
}

}  // namespace ebic

using namespace ebic;

extern "C" {

int ebic_version(void) { return EBIC_VERSION; }

const char *ebic_last_error(void) { return t_error; }

size_t ebic_matrix_bytes(int32_t rows, int32_t cols) {
    if (rows < 1 || cols < 1) return 0;
    return (size_t)cols * rows_padded(rows) * sizeof(uint16_t);
}

int ebic_matrix_prepare(const float *d_x, int32_t rows, int32_t cols, uint16_t *d_ranks,
                        ebic_matrix *m, void *stream) {
    clear_error();
    if (!d_x || !d_ranks || !m) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    if (rows < 1 || rows > EBIC_MAX_ROWS || cols < 2 || cols > EBIC_MAX_COLS ||
        (int64_t)cols * rows_padded(rows) > INT32_MAX)
        return fail(EBIC_ERR_INVALID_ARG, "matrix shape %d x %d not supported", rows, cols);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int *flag = nullptr, dev = 0;
    int rc = acquire_flag(&flag, &dev);
    if (rc) return rc;
    // this call's own status word, zeroed, set by the check and read back
    // on this stream; returned to the pool once the read has landed
    int bad = 0;
    rc = launch_prepare(d_x, rows, cols, d_ranks, flag, s);
    if (rc == EBIC_OK) {
        hipError_t e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = check_hip(e, "matrix status word");
    }
    // the word goes back to the pool only once nothing of this call can still
    // write it; after a device error it stays out of the pool (4 bytes)
    if (rc == EBIC_OK) release_flag(flag, dev);
    if (rc) return rc;
    if (bad) return fail(EBIC_ERR_NONFINITE, "matrix holds NaN or infinite values");
    m->d_ranks = d_ranks;
    m->rows = rows;
    m->cols = cols;
    m->rows_pad = rows_padded(rows);
    m->d_pairs = nullptr;
    m->d_pairs_strict = nullptr;
    return EBIC_OK;
}

int ebic_population_upload(const int32_t *h_offsets, const uint16_t *h_cols, int32_t size,
                           int32_t cols, int32_t *d_offsets, uint16_t *d_cols, void *stream) {
    clear_error();
    if (size < 0 || !h_offsets || !d_offsets || (size > 0 && (!h_cols || !d_cols)))
        return fail(EBIC_ERR_INVALID_ARG, "NULL argument or negative size");
    if (h_offsets[0] != 0) return fail(EBIC_ERR_INVALID_ARG, "offsets[0] must be 0");
    std::vector<uint8_t> seen((size_t)cols > 0 ? cols : 1, 0);
    for (int32_t i = 0; i < size; i++) {
        const int32_t b = h_offsets[i], e = h_offsets[i + 1], k = e - b;
        if (k < 2 || k > EBIC_MAX_K)
            return fail(EBIC_ERR_INVALID_ARG, "individual %d has %d columns", i, k);
        int bad = 0;
        for (int32_t q = b; q < e; q++) {
            const uint16_t c = h_cols[q];
            if (c >= cols || seen[c]) bad = 1;
            if (c < cols) seen[c] = 1;
        }
        for (int32_t q = b; q < e; q++)
            if (h_cols[q] < cols) seen[h_cols[q]] = 0;
        if (bad)
            return fail(EBIC_ERR_INVALID_ARG, "individual %d repeats a column or exceeds %d", i,
                        cols);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    EBIC_HIP(hipMemcpyAsync(d_offsets, h_offsets, sizeof(int32_t) * (size + 1),
                            hipMemcpyHostToDevice, s));
    if (size > 0 && h_offsets[size] > 0)
        EBIC_HIP(hipMemcpyAsync(d_cols, h_cols, sizeof(uint16_t) * h_offsets[size],
                                hipMemcpyHostToDevice, s));
    EBIC_HIP(hipStreamSynchronize(s));
    return EBIC_OK;
}

int ebic_evaluate(const ebic_matrix *m, const ebic_population *pop, const ebic_archive *arch,
                  const ebic_params *p, const ebic_eval_out *out, void *stream) {
    clear_error();
    int rc = check_matrix(m);
    if (rc) return rc;
    if ((rc = check_eval_params(p)) || (rc = check_archive(arch))) return rc;
    if (!pop || pop->size < 0 || (pop->size > 0 && (!pop->d_offsets || !pop->d_cols)))
        return fail(EBIC_ERR_INVALID_ARG, "population is NULL or malformed");
    if (!out || (pop->size > 0 && (!out->d_fitness || !out->d_count)))
        return fail(EBIC_ERR_INVALID_ARG, "fitness and count outputs are required");
    EvalJob j{};
    j.ranks = m->d_ranks;
    j.rows = m->rows;
    j.cols = m->cols;
    j.rows_pad = m->rows_pad;
    j.words = m->rows_pad / 64;
    j.pairs = m->d_pairs;
    j.pop_size = pop->size;
    j.pop_len = pop->length;
    j.pop_off = pop->d_offsets;
    j.pop_cols = pop->d_cols;
    j.arch_size = arch ? arch->size : 0;
    j.arch_len = arch ? arch->length : 0;
    j.arch_support = arch ? arch->d_support : nullptr;
    j.arch_off = arch ? arch->d_offsets : nullptr;
    j.arch_cols = arch ? arch->d_cols : nullptr;
    j.approx_permille = p->approx_permille;
    j.negative_trends = p->negative_trends;
    j.overlap_permille = p->overlap_permille;
    j.min_rows = p->min_rows;
    j.k_score_min = p->k_score_min;
    j.tie_rule = p->tie_rule;
    j.fitness = out->d_fitness;
    j.count = out->d_count;
    j.support = out->d_support;
    j.overlap = out->d_overlap;
    return launch_evaluate_plain(j, static_cast<hipStream_t>(stream));
}

size_t ebic_pairs_bytes(int32_t rows, int32_t cols) {
    if (rows < 1 || cols < 2) return 0;
    return (size_t)cols * (cols - 1) / 2 * pair_words(rows_padded(rows)) * sizeof(uint64_t);
}

int32_t ebic_pairs_words(int32_t rows) {
    if (rows < 1) return 0;
    return pair_words(rows_padded(rows));
}

int ebic_pairs_prepare(ebic_matrix *m, uint64_t *d_pairs, void *stream) {
    clear_error();
    int rc = check_matrix(m);
    if (rc) return rc;
    if (!d_pairs) return fail(EBIC_ERR_INVALID_ARG, "pair table is NULL");
    rc = launch_build_pairs(m->d_ranks, m->rows, m->cols, m->rows_pad, d_pairs, false,
                            static_cast<hipStream_t>(stream));
    if (rc) return rc;
    m->d_pairs = d_pairs;
    return EBIC_OK;
}

int ebic_pairs_strict_prepare(ebic_matrix *m, uint64_t *d_pairs_strict, void *stream) {
    clear_error();
    int rc = check_matrix(m);
    if (rc) return rc;
    if (!d_pairs_strict) return fail(EBIC_ERR_INVALID_ARG, "strict pair table is NULL");
    rc = launch_build_pairs(m->d_ranks, m->rows, m->cols, m->rows_pad, d_pairs_strict, true,
                            static_cast<hipStream_t>(stream));
    if (rc) return rc;
    m->d_pairs_strict = d_pairs_strict;
    return EBIC_OK;
}

int ebic_batch_create(const ebic_job *jobs, int32_t njobs, int32_t flags, ebic_batch **out) {
    clear_error();
    if (!out) return fail(EBIC_ERR_INVALID_ARG, "out is NULL");
    Batch *b = nullptr;
    int rc = batch_create(jobs, njobs, flags, &b);
    if (rc) return rc;
    *out = reinterpret_cast<ebic_batch *>(b);
    return EBIC_OK;
}

int ebic_batch_run(ebic_batch *b, void *stream) {
    clear_error();
    return batch_run(reinterpret_cast<Batch *>(b), static_cast<hipStream_t>(stream));
}

int ebic_batch_destroy(ebic_batch *b) {
    clear_error();
    return batch_destroy(reinterpret_cast<Batch *>(b));
}

int ebic_batch_tuning(ebic_batch *b, int32_t *chunks_per_item, int32_t *loads_in_flight,
                      int32_t *words_per_lane) {
    clear_error();
    return batch_tuning(reinterpret_cast<Batch *>(b), chunks_per_item, loads_in_flight,
                        words_per_lane);
}

int ebic_batch_set_tuning(ebic_batch *b, int32_t chunks_per_item, int32_t loads_in_flight,
                          int32_t words_per_lane) {
    clear_error();
    return batch_set_tuning(reinterpret_cast<Batch *>(b), chunks_per_item, loads_in_flight,
                            words_per_lane);
}

int ebic_batch_profile(ebic_batch *b, int32_t n) {
    clear_error();
    return batch_profile(reinterpret_cast<Batch *>(b), n);
}

int ebic_batch_timings(ebic_batch *b, float *ms, int32_t *n) {
    clear_error();
    return batch_timings(reinterpret_cast<Batch *>(b), ms, n);
}

int ebic_evaluate_batched(const ebic_job *jobs, int32_t njobs, void *stream) {
    clear_error();
    Batch *b = nullptr;
    int rc = batch_create(jobs, njobs, 0, &b);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = batch_run(b, s);
    if (rc == EBIC_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = check_hip(e, "hipStreamSynchronize");
    }
    batch_destroy(b);
    return rc;
}

int ebic_evaluate_batched_noalloc(const ebic_job *jobs, int32_t njobs, void *stream) {
    clear_error();
    return batch_run_noalloc(jobs, njobs, static_cast<hipStream_t>(stream));
}

int ebic_run(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p, uint64_t seed,
             const ebic_allocator *alloc, void *stream, ebic_result **out) {
    clear_error();
    return run_method(h_x, rows, cols, p, seed, alloc, static_cast<hipStream_t>(stream), out);
}

int ebic_run_device(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                    uint64_t seed, const ebic_allocator *alloc, void *stream, ebic_result **out) {
    clear_error();
    return run_method_device(h_x, rows, cols, p, seed, alloc, static_cast<hipStream_t>(stream),
                             out);
}

int ebic_session_create(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                        uint64_t seed, const ebic_allocator *alloc, void *stream,
                        ebic_session **out) {
    clear_error();
    return session_create(h_x, rows, cols, p, seed, alloc, static_cast<hipStream_t>(stream),
                          reinterpret_cast<Session **>(out));
}

int ebic_session_step(ebic_session *s, int32_t steps, int32_t *done) {
    clear_error();
    return session_step(reinterpret_cast<Session *>(s), steps, done);
}

int ebic_session_checkpoint(ebic_session *s, void *buf, size_t *bytes) {
    clear_error();
    return session_checkpoint(reinterpret_cast<Session *>(s), buf, bytes);
}

int ebic_session_restore(const float *h_x, int32_t rows, int32_t cols, const void *buf,
                         size_t bytes, const ebic_allocator *alloc, void *stream,
                         ebic_session **out) {
    clear_error();
    return session_restore(h_x, rows, cols, buf, bytes, alloc, static_cast<hipStream_t>(stream),
                           reinterpret_cast<Session **>(out));
}

int ebic_session_result(ebic_session *s, ebic_result **out) {
    clear_error();
    return session_result(reinterpret_cast<Session *>(s), out);
}

void ebic_session_free(ebic_session *s) { session_free(reinterpret_cast<Session *>(s)); }

int ebic_ce_score(const ebic_bicluster *found, int32_t n_found, const ebic_bicluster *truth,
                  int32_t n_truth, int32_t rows, int32_t cols, double *score, double *ce) {
    clear_error();
    return ce_score(found, n_found, truth, n_truth, rows, cols, score, ce);
}

void ebic_result_free(ebic_result *r) {
    if (r) free_result(r);
}

int ebic_server_create(const ebic_server_config *cfg, ebic_server **out) {
    clear_error();
    if (!out) return fail(EBIC_ERR_INVALID_ARG, "out is NULL");
    Server *s = nullptr;
    int rc = server_create(cfg, &s);
    if (rc) return rc;
    *out = reinterpret_cast<ebic_server *>(s);
    return EBIC_OK;
}

int ebic_server_submit(ebic_server *s, const float *h_x, int32_t rows, int32_t cols,
                       const ebic_params *p, uint64_t seed, int64_t *job_id) {
    clear_error();
    if (!s) return fail(EBIC_ERR_INVALID_ARG, "server is NULL");
    return server_submit(reinterpret_cast<Server *>(s), h_x, rows, cols, p, seed, job_id);
}

int ebic_server_poll(ebic_server *s, int64_t job_id, ebic_result **out) {
    clear_error();
    if (!s) return fail(EBIC_ERR_INVALID_ARG, "server is NULL");
    return server_poll(reinterpret_cast<Server *>(s), job_id, out, false);
}

int ebic_server_wait(ebic_server *s, int64_t job_id, ebic_result **out) {
    clear_error();
    if (!s) return fail(EBIC_ERR_INVALID_ARG, "server is NULL");
    return server_poll(reinterpret_cast<Server *>(s), job_id, out, true);
}

int ebic_server_stats(ebic_server *s, ebic_server_metrics *out) {
    clear_error();
    if (!s || !out) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    server_stats(reinterpret_cast<Server *>(s), out);
    return EBIC_OK;
}

int ebic_server_destroy(ebic_server *s) {
    clear_error();
    if (s) server_destroy(reinterpret_cast<Server *>(s));
    return EBIC_OK;
}

int ebic_support_rows(const uint64_t *d_support, int32_t size, int32_t words,
                      const int32_t *d_sel, int32_t n_sel, const int32_t *d_row_offsets,
                      int32_t *d_rows, void *stream) {
    clear_error();
    if (size < 0 || words < 1 || n_sel < 0 ||
        (n_sel > 0 && (!d_support || !d_sel || !d_row_offsets || !d_rows)))
        return fail(EBIC_ERR_INVALID_ARG, "NULL argument or bad size");
    return launch_support_rows(d_support, size, words, d_sel, n_sel, d_row_offsets, d_rows,
                               static_cast<hipStream_t>(stream));
}

}  // extern "C"
