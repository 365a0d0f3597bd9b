// Batched evaluation: many populations (of one or several jobs, each with
// its own matrix, archive and parameters) in one launch of two kernels.
//
// Kernel A splits every individual into items of 2048 rows and gives each
// item to one wavefront; items of all jobs form one flat index space, so a
// single launch covers the whole batch, individuals of uneven length
// included. With a pair table a lane tests 32 rows at once: each step of the
// series is one 32-bit load of the pair's bitmap, and the rows' counts of
// steps against each trend are kept bit-sliced, saturating at t+1
// (thermometer code: plane m holds "at least m violations"), so an update is
// one AND-OR per plane. Without a table the item runs the gather form (lane =
// row) over its 32 blocks. Kernel B then reduces each individual's support
// words into the count, the rows shared with each archive member, and the
// FP64 fitness. The paper sends the whole population to the GPU at once
// (Sec. 2.4, step 2); here several populations share the launch.
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"

namespace ebic {

struct DevJob {
    const uint16_t *ranks;
    const uint32_t *pairs;
    int32_t rows, cols, rows_pad, w32, w64;
    int32_t mode;     // 1 = pair table, 0 = gather
    int32_t nchunks;  // items per individual
    int32_t pop_size, pop_len;
    int64_t item_begin;  // first item of this job in the batch
    int64_t ind_begin;   // first individual of this job in the batch
    const int32_t *pop_off;
    const uint16_t *pop_cols;
    const int32_t *order;
    int32_t arch_size, arch_len;
    const uint64_t *arch_support;
    const int32_t *arch_off;
    const uint16_t *arch_cols;
    int32_t approx_permille, negative_trends, overlap_permille, min_rows, k_score_min;
    double *fitness;
    int32_t *count;
    uint64_t *support;
    int32_t *overlap;
};

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = kWaves * kWave;
constexpr int kItemRows = 2048;  // 64 lanes x 32 rows, or 32 blocks x 64 rows

__device__ inline int find_job(const DevJob *jobs, int njobs, int64_t x, bool by_item) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        const int64_t b = by_item ? jobs[mid].item_begin : jobs[mid].ind_begin;
        if (b <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Thermometer counters of steps against the increasing trend (D) and against
// the decreasing trend (U), T = t+1 planes each; returns the fit word.
template <int T, bool NEG>
__device__ uint32_t pairs_thermo(const uint32_t *__restrict__ pairs, int64_t w32,
                                 const int32_t *s_pd, int k, int w, bool active) {
    uint32_t D[T], U[T];
#pragma unroll
    for (int m = 0; m < T; m++) D[m] = U[m] = 0;
    int j = 1;
    while (j < k) {
        const int n = (k - j) < 4 ? (k - j) : 4;
        uint32_t x[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            x[q] = 0;
            if (q < n) {
                const int pd = __builtin_amdgcn_readfirstlane(s_pd[j + q]);
                const uint32_t *vec = pairs + (int64_t)(pd & 0x7fffffff) * w32;
                const uint32_t bits = active ? vec[w] : 0u;
                x[q] = pd < 0 ? ~bits : bits;  // 1 = up-step in this row
            }
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (q >= n) break;
            const uint32_t up = x[q], down = ~x[q];
#pragma unroll
            for (int m = T - 1; m >= 1; m--) {
                D[m] |= D[m - 1] & down;
                if (NEG) U[m] |= U[m - 1] & up;
            }
            D[0] |= down;
            if (NEG) U[0] |= up;
        }
        j += n;
        const uint32_t dead = D[T - 1] & (NEG ? U[T - 1] : ~0u);
        if (__ballot(active && dead != ~0u) == 0) break;
    }
    return ~D[T - 1] | (NEG ? ~U[T - 1] : 0u);
}

// Bit-sliced compare of the 9-bit per-row counts b[] with a constant:
// returns rows with count < c in *lt and count == c in *eq.
__device__ inline void cmp_const(const uint32_t *b, int c, uint32_t *lt, uint32_t *eq) {
    uint32_t l = 0, e = ~0u;
#pragma unroll
    for (int p = 8; p >= 0; p--) {
        if ((c >> p) & 1) {
            l |= e & ~b[p];
            e &= b[p];
        } else {
            e &= ~b[p];
        }
    }
    *lt = l;
    *eq = e;
}

// Exact bit-sliced count of up-steps (9 planes, k <= 512) for large
// tolerances; returns the fit word.
template <bool NEG>
__device__ uint32_t pairs_binary(const uint32_t *__restrict__ pairs, int64_t w32,
                                 const int32_t *s_pd, int k, int t, int w, bool active) {
    uint32_t b[9];
#pragma unroll
    for (int p = 0; p < 9; p++) b[p] = 0;
    for (int j = 1; j < k; j++) {
        const int pd = __builtin_amdgcn_readfirstlane(s_pd[j]);
        const uint32_t *vec = pairs + (int64_t)(pd & 0x7fffffff) * w32;
        const uint32_t bits = active ? vec[w] : 0u;
        uint32_t carry = pd < 0 ? ~bits : bits;
#pragma unroll
        for (int p = 0; p < 9; p++) {
            const uint32_t c2 = b[p] & carry;
            b[p] ^= carry;
            carry = c2;
        }
    }
    uint32_t lt, eq;
    cmp_const(b, k - 1 - t, &lt, &eq);
    uint32_t fit = ~lt;  // ups >= k-1-t  <=>  downs <= t
    if (NEG) {
        cmp_const(b, t, &lt, &eq);
        fit |= lt | eq;  // ups <= t
    }
    return fit;
}

template <bool NEG>
__device__ uint32_t pairs_dispatch(const uint32_t *pairs, int64_t w32, const int32_t *s_pd, int k,
                                   int t, int w, bool active) {
    switch (t) {
#define EBIC_T(TT) \
    case TT - 1: return pairs_thermo<TT, NEG>(pairs, w32, s_pd, k, w, active);
        EBIC_T(1) EBIC_T(2) EBIC_T(3) EBIC_T(4) EBIC_T(5) EBIC_T(6) EBIC_T(7) EBIC_T(8)
        EBIC_T(9) EBIC_T(10) EBIC_T(11) EBIC_T(12) EBIC_T(13) EBIC_T(14) EBIC_T(15) EBIC_T(16)
#undef EBIC_T
        default: return pairs_binary<NEG>(pairs, w32, s_pd, k, t, w, active);
    }
}

__global__ void __launch_bounds__(kThreads)
    eval_items_kernel(const DevJob *__restrict__ jobs, int32_t njobs, int64_t total_items) {
    __shared__ int32_t s_buf[kWaves][EBIC_MAX_K];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t item = (int64_t)blockIdx.x * kWaves + wave;
    if (item >= total_items) return;
    const DevJob &J = jobs[find_job(jobs, njobs, item, true)];
    const int64_t local = item - J.item_begin;
    const int32_t oi = (int32_t)(local / J.nchunks), chunk = (int32_t)(local % J.nchunks);
    const int32_t ind = J.order ? J.order[oi] : oi;
    if (ind < 0 || ind >= J.pop_size) return;
    const int32_t beg = J.pop_off[ind], end = J.pop_off[ind + 1];
    const int k = end - beg;
    int32_t *s = s_buf[wave];
    bool bad = !(beg >= 0 && end <= J.pop_len && k >= 2 && k <= EBIC_MAX_K);
    if (!bad) {
        // stage the series (pair mode: one descriptor per step; gather mode:
        // each column's byte offset)
        int lbad = 0;
        for (int j = lane; j < k; j += kWave) {
            const int c = J.pop_cols[beg + j];
            lbad |= c >= J.cols;
            if (j > 0) lbad |= c == J.pop_cols[beg + j - 1];
            if (J.mode == 1) {
                if (j > 0) {
                    const int a = J.pop_cols[beg + j - 1];
                    const int lo = a < c ? a : c, hi = a < c ? c : a;
                    const int32_t p = (int32_t)pair_index(lo, hi, J.cols);
                    s[j] = p | (a > c ? (int32_t)0x80000000 : 0);
                }
            } else {
                s[j] = (int32_t)((uint32_t)c * (uint32_t)J.rows_pad * 2u);
            }
        }
        bad = __ballot(lbad) != 0;
    }
    if (bad) {  // malformed: kernel B marks it invalid; never read out of bounds
        const int32_t w0 = chunk * 32;
        if (lane < 32 && w0 + lane < J.w64) J.support[(int64_t)ind * J.w64 + w0 + lane] = 0;
        return;
    }
    const int t = tol(k, J.approx_permille);
    const bool neg = J.negative_trends != 0;
    if (J.mode == 1) {
        const int w = chunk * 64 + lane;  // this lane's 32-row dword
        const bool active = w < J.w32;
        uint32_t fit = neg ? pairs_dispatch<true>(J.pairs, J.w32, s, k, t, w, active)
                           : pairs_dispatch<false>(J.pairs, J.w32, s, k, t, w, active);
        const int r0 = w * 32;
        if (r0 + 32 > J.rows) fit &= r0 >= J.rows ? 0u : ((1u << (J.rows - r0)) - 1u);
        if (active) reinterpret_cast<uint32_t *>(J.support)[(int64_t)ind * J.w32 + w] = fit;
    } else {
        const __amdgpu_buffer_rsrc_t rs =
            make_rsrc(J.ranks, (uint32_t)((size_t)J.cols * J.rows_pad * 2));
        int lo = 0, hi = 0;
        const int b0 = chunk * 32;
        for (int b = 0; b < 32 && b0 + b < J.w64; b++) {
            const int r = (b0 + b) * kWave + lane;
            const uint64_t word = block_support(rs, s, k, t, neg, r * 2, r < J.rows);
            lo = writelane((int)(uint32_t)word, b, lo);
            hi = writelane((int)(uint32_t)(word >> 32), b, hi);
        }
        if (lane < 32 && b0 + lane < J.w64)
            J.support[(int64_t)ind * J.w64 + b0 + lane] =
                ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    }
}

// Kernel B: one wave per individual. Validates the series (length, range,
// no repeated column), reduces the support words into n and the rows shared
// with each archive member, and writes count, overlap and fitness.
__global__ void __launch_bounds__(kThreads)
    epilogue_kernel(const DevJob *__restrict__ jobs, int32_t njobs, int64_t total_ind) {
    __shared__ uint32_t s_bits[kWaves][EBIC_MAX_COLS / 32];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t gid = (int64_t)blockIdx.x * kWaves + wave;
    if (gid >= total_ind) return;
    const DevJob &J = jobs[find_job(jobs, njobs, gid, false)];
    const int32_t i = (int32_t)(gid - J.ind_begin);
    const int32_t beg = J.pop_off[i], end = J.pop_off[i + 1];
    const int k = end - beg;
    uint32_t *bits = s_bits[wave];
    const int K = J.arch_size;
    bool bad = !(beg >= 0 && end <= J.pop_len && k >= 2 && k <= EBIC_MAX_K);
    if (!bad) {
        for (int q = lane; q < (J.cols + 31) / 32; q += kWave) bits[q] = 0;
        __builtin_amdgcn_wave_barrier();
        int lbad = 0;
        for (int j = lane; j < k; j += kWave) {
            const int c = J.pop_cols[beg + j];
            if (c >= J.cols) {
                lbad = 1;
            } else {
                const uint32_t bit = 1u << (c % 32);
                if (atomicOr(&bits[c / 32], bit) & bit) lbad = 1;
            }
        }
        __builtin_amdgcn_wave_barrier();
        bad = __ballot(lbad) != 0;
    }
    uint64_t *S = J.support + (int64_t)i * J.w64;
    if (bad) {
        for (int w = lane; w < J.w64; w += kWave) S[w] = 0;
        if (J.overlap)
            for (int j = lane; j < K; j += kWave) J.overlap[(int64_t)i * K + j] = 0;
        if (lane == 0) {
            J.count[i] = -1;
            J.fitness[i] = -1.0;
        }
        return;
    }
    int c = 0;
    for (int w = lane; w < J.w64; w += kWave) c += __popcll(S[w]);
    const int n = wave_sum(c);
    int m = 0;
    int32_t my_h = 0;  // lane j keeps h of member j (j < 64)
    for (int j = 0; j < K; j++) {
        int32_t mb = J.arch_off[j], me = J.arch_off[j + 1];
        if (mb < 0) mb = 0;
        if (me > J.arch_len) me = J.arch_len;
        int g = 0;
        for (int q = mb + lane; q < me; q += kWave) {
            const int col = J.arch_cols[q];
            g += col < J.cols ? (int)((bits[col / 32] >> (col % 32)) & 1u) : 0;
        }
        g = wave_sum(g);
        int h = 0;
        if (n > 0 && (J.overlap || g > 0)) {
            const uint64_t *A = J.arch_support + (int64_t)j * J.w64;
            int hp = 0;
            for (int w = lane; w < J.w64; w += kWave) hp += __popcll(S[w] & A[w]);
            h = wave_sum(hp);
        }
        if (lane == j) my_h = h;
        m += 1000LL * h * g > (long long)J.overlap_permille * n * k;
    }
    if (J.overlap && lane < K) J.overlap[(int64_t)i * K + lane] = my_h;
    if (lane == 0) {
        const double s = (n >= J.min_rows && k >= J.k_score_min) ? ldexp((double)n, k) : 0.0;
        J.count[i] = n;
        J.fitness[i] = ldexp(s, -m);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: the batch object.
// ---------------------------------------------------------------------------

struct Batch {
    int device = 0;
    std::vector<DevJob> jobs;
    DevJob *d_jobs = nullptr;
    std::vector<void *> scratch;
    int64_t total_items = 0, total_ind = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // kernel arguments kept alive for the graph's nodes
    int32_t njobs = 0;
};

namespace {

int check_job(const ebic_job *j, int idx) {
    const ebic_matrix *m = &j->matrix;
    if (!m->d_ranks || m->rows < 1 || m->rows > EBIC_MAX_ROWS || m->cols < 2 ||
        m->cols > EBIC_MAX_COLS || m->rows_pad != rows_padded(m->rows) ||
        (int64_t)m->cols * m->rows_pad > INT32_MAX)
        return fail(EBIC_ERR_INVALID_ARG, "job %d: bad matrix view", idx);
    int rc = check_eval_params(&j->params);
    if (rc) return rc;
    const ebic_archive *a = &j->archive;
    if (a->size < 0 || a->size > EBIC_MAX_ARCHIVE ||
        (a->size > 0 && (!a->d_support || !a->d_offsets || !a->d_cols || a->length < 0)))
        return fail(EBIC_ERR_INVALID_ARG, "job %d: bad archive", idx);
    const ebic_population *p = &j->population;
    if (p->size < 0 || (p->size > 0 && (!p->d_offsets || !p->d_cols)))
        return fail(EBIC_ERR_INVALID_ARG, "job %d: bad population", idx);
    if (p->size > 0 && (!j->out.d_fitness || !j->out.d_count))
        return fail(EBIC_ERR_INVALID_ARG, "job %d: fitness and count outputs are required", idx);
    return EBIC_OK;
}

}  // namespace

int batch_create(const ebic_job *jobs, int32_t njobs, int32_t flags, Batch **out) {
    if (!out || njobs < 1 || !jobs) return fail(EBIC_ERR_INVALID_ARG, "no jobs");
    for (int i = 0; i < njobs; i++) {
        int rc = check_job(&jobs[i], i);
        if (rc) return rc;
    }
    Batch *b = new Batch();
    EBIC_HIP(hipGetDevice(&b->device));
    b->njobs = njobs;
    int64_t items = 0, inds = 0;
    for (int i = 0; i < njobs; i++) {
        const ebic_job &j = jobs[i];
        DevJob d{};
        d.ranks = j.matrix.d_ranks;
        d.pairs = reinterpret_cast<const uint32_t *>(j.matrix.d_pairs);
        d.rows = j.matrix.rows;
        d.cols = j.matrix.cols;
        d.rows_pad = j.matrix.rows_pad;
        d.w32 = j.matrix.rows_pad / 32;
        d.w64 = j.matrix.rows_pad / 64;
        d.mode = (j.matrix.d_pairs && !(flags & EBIC_BATCH_GATHER)) ? 1 : 0;
        d.nchunks = (j.matrix.rows_pad + kItemRows - 1) / kItemRows;
        d.pop_size = j.population.size;
        d.pop_len = j.population.length;
        d.pop_off = j.population.d_offsets;
        d.pop_cols = j.population.d_cols;
        d.order = j.population.d_order;
        d.item_begin = items;
        d.ind_begin = inds;
        d.arch_size = j.archive.size;
        d.arch_len = j.archive.length;
        d.arch_support = j.archive.d_support;
        d.arch_off = j.archive.d_offsets;
        d.arch_cols = j.archive.d_cols;
        d.approx_permille = j.params.approx_permille;
        d.negative_trends = j.params.negative_trends;
        d.overlap_permille = j.params.overlap_permille;
        d.min_rows = j.params.min_rows;
        d.k_score_min = j.params.k_score_min;
        d.fitness = j.out.d_fitness;
        d.count = j.out.d_count;
        d.support = j.out.d_support;
        d.overlap = j.out.d_overlap;
        if (!d.support && d.pop_size > 0) {
            void *p = nullptr;
            hipError_t e = hipMalloc(&p, (size_t)d.pop_size * d.w64 * sizeof(uint64_t));
            if (e != hipSuccess) {
                batch_destroy(b);
                return check_hip(e, "hipMalloc(support scratch)");
            }
            b->scratch.push_back(p);
            d.support = static_cast<uint64_t *>(p);
        }
        items += (int64_t)d.pop_size * d.nchunks;
        inds += d.pop_size;
        b->jobs.push_back(d);
    }
    b->total_items = items;
    b->total_ind = inds;
    hipError_t e = hipMalloc(&b->d_jobs, sizeof(DevJob) * njobs);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_jobs, b->jobs.data(), sizeof(DevJob) * njobs, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_destroy(b);
        return check_hip(e, "batch job table");
    }
    if ((flags & EBIC_BATCH_GRAPH) && b->total_ind > 0) {
        // Two kernel nodes, A then B, built explicitly (no stream capture).
        int rc = EBIC_OK;
        hipGraphNode_t na = nullptr, nb = nullptr;
        void *args_a[] = {&b->d_jobs, &b->njobs, &b->total_items};
        void *args_b[] = {&b->d_jobs, &b->njobs, &b->total_ind};
        hipKernelNodeParams pa{}, pb{};
        pa.func = reinterpret_cast<void *>(eval_items_kernel);
        pa.gridDim = dim3((unsigned)((b->total_items + kWaves - 1) / kWaves));
        pa.blockDim = dim3(kThreads);
        pa.kernelParams = args_a;
        pb.func = reinterpret_cast<void *>(epilogue_kernel);
        pb.gridDim = dim3((unsigned)((b->total_ind + kWaves - 1) / kWaves));
        pb.blockDim = dim3(kThreads);
        pb.kernelParams = args_b;
        e = hipGraphCreate(&b->graph, 0);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&na, b->graph, nullptr, 0, &pa);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&nb, b->graph, &na, 1, &pb);
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            rc = check_hip(e, "batch graph");
            batch_destroy(b);
            return rc;
        }
    }
    *out = b;
    return EBIC_OK;
}

int batch_run(Batch *b, hipStream_t stream) {
    if (!b) return fail(EBIC_ERR_INVALID_ARG, "batch is NULL");
    if (b->total_ind == 0) return EBIC_OK;
    if (b->exec) {
        EBIC_HIP(hipGraphLaunch(b->exec, stream));
        return EBIC_OK;
    }
    if (b->total_items > 0)
        eval_items_kernel<<<(unsigned)((b->total_items + kWaves - 1) / kWaves), kThreads, 0,
                            stream>>>(b->d_jobs, b->njobs, b->total_items);
    epilogue_kernel<<<(unsigned)((b->total_ind + kWaves - 1) / kWaves), kThreads, 0, stream>>>(
        b->d_jobs, b->njobs, b->total_ind);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

int batch_destroy(Batch *b) {
    if (!b) return EBIC_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    for (void *p : b->scratch) (void)hipFree(p);
    delete b;
    return EBIC_OK;
}

}  // namespace ebic
