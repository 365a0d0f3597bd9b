// Internal declarations shared by the library's translation units (not part
// of the public interface; see include/ebic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "ebic.h"

namespace ebic {

constexpr int kWave = 64;

// Thread-local error message behind ebic_last_error().
int fail(int code, const char *fmt, ...);
void clear_error();

// Maps a HIP error to EBIC_ERR_DEVICE with a message naming the call.
int check_hip(hipError_t e, const char *what);

#define EBIC_HIP(call)                                            \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::ebic::check_hip(e_, #call); \
    } while (0)

inline int32_t rows_padded(int32_t rows) { return (rows + 63) / 64 * 64; }
// Words per pair in the pair table: the rows' 64-bit words rounded up to 16,
// so every pair's bitmap starts on a 128-byte line.
inline int32_t pair_words(int32_t rows_pad) { return (rows_pad / 64 + 15) / 16 * 16; }

inline int tolerance(int k, int approx_permille) {
    return (int)(((int64_t)(k - 1) * (1000 - approx_permille)) / 1000);
}

// Host-side validation of the evaluation parameters.
int check_eval_params(const ebic_params *p);

// 4-byte status words in device memory for matrix ingest, one per call in
// flight: acquire_flag takes a word of the current device for the caller
// alone (words come in blocks of 64, allocated when a device has none free
// and kept until the process ends), release_flag returns it. Concurrent
// ingests on several threads and streams therefore never share a word.
int acquire_flag(int **flag, int *device);
void release_flag(int *flag, int device);

// Arguments of one evaluation, as the kernels see them.
struct EvalJob {
    const uint16_t *ranks;
    int32_t rows, cols, rows_pad, words;
    const uint64_t *pairs;
    int32_t pop_size, pop_len;
    const int32_t *pop_off;
    const uint16_t *pop_cols;
    int32_t arch_size, arch_len;
    const uint64_t *arch_support;
    const int32_t *arch_off;
    const uint16_t *arch_cols;
    int32_t approx_permille, negative_trends, overlap_permille, min_rows, k_score_min, tie_rule;
    double *fitness;
    int32_t *count;
    uint64_t *support;
    int32_t *overlap;
};

int launch_evaluate_plain(const EvalJob &job, hipStream_t stream);
// A run of 64-bit words to copy: `words` words from src to dst + dst_at.
struct WordSpan {
    const uint64_t *src;
    uint64_t dst_at;
    int64_t words;
};
// Copies n spans (d_spans on the device) into dst, a workgroup per span.
int launch_gather_spans(const WordSpan *d_spans, int32_t n, uint64_t *dst, hipStream_t stream);
int launch_support_rows(const uint64_t *support, int32_t size, int32_t words, const int32_t *sel,
                        int32_t n_sel, const int32_t *row_off, int32_t *rows, hipStream_t stream);
int launch_prepare(const float *x, int32_t rows, int32_t cols, uint16_t *ranks, int *flag,
                   hipStream_t stream);
// The pair table ("lo precedes hi": rank[lo] <= rank[hi]) or, with strict,
// the strict one (rank[lo] < rank[hi]).
int launch_build_pairs(const uint16_t *ranks, int32_t rows, int32_t cols, int32_t rows_pad,
                       uint64_t *table, bool strict, hipStream_t stream);

int run_method(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p, uint64_t seed,
               const ebic_allocator *al, hipStream_t stream, ebic_result **out);
int run_method_device(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                      uint64_t seed, const ebic_allocator *al, hipStream_t stream,
                      ebic_result **out);
void free_result(ebic_result *r);
int ce_score(const ebic_bicluster *found, int32_t n_found, const ebic_bicluster *truth,
             int32_t n_truth, int32_t rows, int32_t cols, double *score, double *ce);

struct Session;
int session_create(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                   uint64_t seed, const ebic_allocator *al, hipStream_t stream, Session **out);
int session_step(Session *s, int32_t steps, int32_t *done);
int session_checkpoint(Session *s, void *buf, size_t *bytes);
int session_restore(const float *h_x, int32_t rows, int32_t cols, const void *buf, size_t bytes,
                    const ebic_allocator *al, hipStream_t stream, Session **out);
int session_result(Session *s, ebic_result **out);
void session_free(Session *s);

class Server;
int server_create(const ebic_server_config *cfg, Server **out);
int server_submit(Server *s, const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                  uint64_t seed, int64_t *id);
int server_poll(Server *s, int64_t id, ebic_result **out, bool block);
void server_stats(Server *s, ebic_server_metrics *st);
void server_destroy(Server *s);

struct Batch;
int batch_create(const ebic_job *jobs, int32_t njobs, int32_t flags, Batch **out);
int batch_run(Batch *b, hipStream_t stream);
// ebic_evaluate_batched_noalloc: the job table in the library's fixed
// device array, no allocation.
int batch_run_noalloc(const ebic_job *jobs, int32_t njobs, hipStream_t stream);
int batch_set(Batch **b, const ebic_job *jobs, int32_t njobs, hipStream_t stream,
              const ebic_allocator *al = nullptr);
// Device memory from the caller's allocator when one is given, else hipMalloc.
void *device_alloc(const ebic_allocator *al, size_t bytes, hipStream_t stream);
void device_release(const ebic_allocator *al, void *p, hipStream_t stream);
int batch_tuning(Batch *b, int32_t *cpi, int32_t *kb, int32_t *wpl);
int batch_set_tuning(Batch *b, int32_t cpi, int32_t kb, int32_t wpl);
// Device addresses of job `job`'s archive size and column count in the
// batch's job table, for code that changes the archive on the device
// between runs (the table must have room: its LDS sizing used the lengths
// given to batch_set).
int batch_archive_fields(Batch *b, int32_t job, int32_t **size, int32_t **len);
int batch_destroy(Batch *b);
int batch_profile(Batch *b, int32_t n);
int batch_timings(Batch *b, float *ms, int32_t *n);

}  // namespace ebic
