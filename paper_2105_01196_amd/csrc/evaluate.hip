// Plain per-generation evaluator and support compaction.
//
// Scoring an individual (Sec. 2.4, steps 2-3 and 7) means testing every row
// for the trend of its column series and counting the rows that keep it.
// Here one workgroup takes one individual and sweeps all 64-row blocks of the
// rank matrix: lane = row, the series' column offsets are wave-uniform, so
// every step is one coalesced 128-byte load, one compare and one add per
// lane. A wavefront ballot turns the 64 row verdicts into one word of the
// support bitmap, popcount gives the count, and AND + popcount against the
// archive words gives the rows shared with each archived bicluster. The
// workgroup then reduces these and computes the fitness itself, so the
// launch needs no atomics and no zeroed outputs.
#include "device.h"
#include "internal.h"

namespace ebic {
namespace {

constexpr int kEvalWaves = 4;
constexpr int kEvalThreads = kEvalWaves * kWave;

__global__ void __launch_bounds__(kEvalThreads) evaluate_plain_kernel(EvalJob a) {
    __shared__ int32_t s_off[EBIC_MAX_K];
    __shared__ uint32_t s_colbits[EBIC_MAX_COLS / 32];
    __shared__ int32_t s_count[kEvalWaves];
    __shared__ int32_t s_h[kEvalWaves][EBIC_MAX_ARCHIVE];
    __shared__ int32_t s_bad;

    const int i = blockIdx.x;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int32_t beg = a.pop_off[i], end = a.pop_off[i + 1];
    const int k = end - beg;

    for (int w = tid; w < (a.cols + 31) / 32; w += kEvalThreads) s_colbits[w] = 0;
    if (tid == 0) s_bad = !(beg >= 0 && end <= a.pop_len && k >= 2 && k <= EBIC_MAX_K);
    __syncthreads();
    if (!s_bad) {
        for (int j = tid; j < k; j += kEvalThreads) {
            const int c = a.pop_cols[beg + j];
            if (c >= a.cols) {
                s_bad = 1;
            } else {
                const uint32_t bit = 1u << (c % 32);
                if (atomicOr(&s_colbits[c / 32], bit) & bit) s_bad = 1;  // repeated column
                // byte offset of the column (< 2^32; passed as a bit pattern)
                s_off[j] = (int32_t)((uint32_t)c * (uint32_t)a.rows_pad * 2u);
            }
        }
    }
    __syncthreads();
    const int K = a.arch_size;
    if (s_bad) {
        for (int w = tid; w < a.words; w += kEvalThreads)
            if (a.support) a.support[(size_t)i * a.words + w] = 0;
        if (a.overlap && tid < K) a.overlap[(size_t)i * K + tid] = 0;
        if (tid == 0) {
            a.count[i] = -1;
            a.fitness[i] = -1.0;
        }
        return;
    }

    const int t = tol(k, a.approx_permille);
    const int neg = a.negative_trends;
    const __amdgpu_buffer_rsrc_t rs =
        make_rsrc(a.ranks, (uint32_t)((size_t)a.cols * a.rows_pad * 2));
    int32_t cnt = 0;   // wave-uniform
    int32_t hacc = 0;  // lane j < K: rows shared with member j
    for (int w = wave; w < a.words; w += kEvalWaves) {
        const int r = w * kWave + lane;
        const uint64_t word = block_support(rs, s_off, k, t, neg, a.tie_rule, r * 2, r < a.rows);
        if (a.support && lane == 0) a.support[(size_t)i * a.words + w] = word;
        cnt += __popcll(word);
        if (lane < K) hacc += __popcll(word & a.arch_support[(size_t)lane * a.words + w]);
    }
    if (lane == 0) s_count[wave] = cnt;
    if (lane < K) s_h[wave][lane] = hacc;
    __syncthreads();
    if (wave != 0) return;

    int32_t n = 0;
    for (int v = 0; v < kEvalWaves; v++) n += s_count[v];
    bool over = false;
    if (lane < K) {
        int32_t h = 0;
        for (int v = 0; v < kEvalWaves; v++) h += s_h[v][lane];
        // columns of the individual that member `lane` also holds
        int32_t mb = a.arch_off[lane], me = a.arch_off[lane + 1];
        if (mb < 0) mb = 0;
        if (me > a.arch_len) me = a.arch_len;
        int32_t g = 0;
        for (int32_t q = mb; q < me; q++) {
            const int c = a.arch_cols[q];
            if (c < a.cols) g += (s_colbits[c / 32] >> (c % 32)) & 1;
        }
        over = 1000LL * h * g > (long long)a.overlap_permille * n * k;
        if (a.overlap) a.overlap[(size_t)i * K + lane] = h;
    }
    const int m = __popcll(__ballot(over));
    if (lane == 0) {
        const double s = (n >= a.min_rows && k >= a.k_score_min) ? ldexp((double)n, k) : 0.0;
        a.count[i] = n;
        a.fitness[i] = ldexp(s, -m);
    }
}

// One workgroup per selected individual: popcount each support word, scan
// the counts across the workgroup, and write every set bit's row index.
constexpr int kCompactThreads = 256;

__global__ void __launch_bounds__(kCompactThreads)
    support_rows_kernel(const uint64_t *__restrict__ support, int32_t size, int32_t words,
                        const int32_t *__restrict__ sel, const int32_t *__restrict__ row_off,
                        int32_t *__restrict__ rows) {
    __shared__ int32_t s_scan[kCompactThreads];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int32_t i = sel[s];
    if (i < 0 || i >= size) return;
    const int32_t beg = row_off[s], end = row_off[s + 1];
    const uint64_t *sp = support + (size_t)i * words;
    int32_t base = beg;
    for (int32_t w0 = 0; w0 < words; w0 += kCompactThreads) {
        const int32_t w = w0 + tid;
        uint64_t word = w < words ? sp[w] : 0;
        const int32_t c = __popcll(word);
        s_scan[tid] = c;
        __syncthreads();
        for (int off = 1; off < kCompactThreads; off *= 2) {
            const int32_t v = tid >= off ? s_scan[tid - off] : 0;
            __syncthreads();
            s_scan[tid] += v;
            __syncthreads();
        }
        int32_t pos = base + s_scan[tid] - c;
        while (word) {
            const int b = __ffsll((unsigned long long)word) - 1;
            if (pos >= beg && pos < end) rows[pos] = w * 64 + b;
            pos++;
            word &= word - 1;
        }
        base += s_scan[kCompactThreads - 1];
        __syncthreads();
    }
}

}  // namespace

int launch_evaluate_plain(const EvalJob &job, hipStream_t stream) {
    if (job.pop_size == 0) return EBIC_OK;
    evaluate_plain_kernel<<<job.pop_size, kEvalThreads, 0, stream>>>(job);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

int launch_support_rows(const uint64_t *support, int32_t size, int32_t words, const int32_t *sel,
                        int32_t n_sel, const int32_t *row_off, int32_t *rows, hipStream_t stream) {
    if (n_sel == 0) return EBIC_OK;
    support_rows_kernel<<<n_sel, kCompactThreads, 0, stream>>>(support, size, words, sel, row_off,
                                                               rows);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

namespace {
constexpr int kGatherThreads = 256;

__global__ void __launch_bounds__(kGatherThreads)
    gather_spans_kernel(const WordSpan *__restrict__ spans, uint64_t *__restrict__ dst) {
    const WordSpan sp = spans[blockIdx.x];
    for (int64_t w = threadIdx.x; w < sp.words; w += kGatherThreads) dst[sp.dst_at + w] = sp.src[w];
}
}  // namespace

int launch_gather_spans(const WordSpan *d_spans, int32_t n, uint64_t *dst, hipStream_t stream) {
    if (n <= 0) return EBIC_OK;
    gather_spans_kernel<<<n, kGatherThreads, 0, stream>>>(d_spans, dst);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

}  // namespace ebic
