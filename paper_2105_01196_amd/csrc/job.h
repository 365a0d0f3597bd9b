// Per-job state of the evolutionary loop (Sec. 2.4), shared by ebic_run and
// the job server. Internal to the library.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <iterator>
#include <vector>

#include "internal.h"

namespace ebic {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).
class SplitMix64 {
  public:
    explicit SplitMix64(uint64_t seed) : state_(seed) {}
    uint64_t state() const { return state_; }
    void set_state(uint64_t s) { state_ = s; }
    uint64_t next() {
        state_ += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state_;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    // Uniform in [0, n): draws below 2^64 mod n are rejected so that the
    // accepted range holds a whole number of periods of n.
    uint64_t below(uint64_t n) {
        const Divisor &d = divisor(n);
        for (;;) {
            const uint64_t x = next();
            if (x >= d.reject) return d.mod(x);
        }
    }
    int below_int(int64_t n) { return (int)below((uint64_t)n); }

  private:
    // x mod n without a division: with m = floor((2^64 - 1) / n), the
    // quotient estimate floor(x m / 2^64) is the true quotient or one less
    // (m n > 2^64 - 1 - n, so x / n - x m / 2^64 < x / 2^64 < 1), so the
    // remainder needs at most one correction.
    struct Divisor {
        uint64_t n = 0, m = 0, reject = 0;
        uint64_t mod(uint64_t x) const {
            const uint64_t q = (uint64_t)(((unsigned __int128)x * m) >> 64);
            uint64_t r = x - q * n;
            if (r >= n) r -= n;
            return r;
        }
    };
    // The few moduli a job draws with (the population, the operator count,
    // series lengths) repeat; each is set up once per slot of a small cache.
    const Divisor &divisor(uint64_t n) {
        Divisor &d = cache_[n & 7];
        if (d.n != n) {
            d.n = n;
            d.m = ~0ULL / n;
            d.reject = (0 - n) % n;
        }
        return d;
    }
    uint64_t state_;
    Divisor cache_[8];
};

using Series = std::vector<uint16_t>;

// With negative trends a series and its reverse have the same support; the
// smaller of the two stands for both in the tabu list and the top-rank list.
inline bool reverse_smaller(const uint16_t *s, size_t k) {
    for (size_t i = 0; i < k; i++)
        if (s[k - 1 - i] != s[i]) return s[k - 1 - i] < s[i];
    return false;
}
inline Series canonical(const Series &s, bool neg) {
    if (!neg || !reverse_smaller(s.data(), s.size())) return s;
    return Series(s.rbegin(), s.rend());
}
// Whether canonical(s, neg) equals the canonical series c, without a copy.
inline bool same_canonical(const Series &s, const Series &c, bool neg) {
    if (s.size() != c.size()) return false;
    return std::equal(s.begin(), s.end(), c.begin()) ||
           (neg && std::equal(s.rbegin(), s.rend(), c.begin()));
}

// The tabu list (Sec. 2.4, step 6): a set of canonical series, open
// addressing over one flat arena of columns, so an insert allocates only
// when a buffer doubles. Each slot keeps a 32-bit tag (part of the hash,
// never 0) in one compact array and the series' place in the arena in
// another, so a probe for a new series usually reads the tags alone. The
// hash only places series; membership is decided by comparing columns.
class TabuSet {
  public:
    // Inserts canonical(s, neg); false if it was present.
    bool insert(const uint16_t *s, size_t k, bool neg) {
        const uint16_t *c = s;
        if (neg && reverse_smaller(s, k)) {
            scratch_.assign(std::reverse_iterator<const uint16_t *>(s + k),
                            std::reverse_iterator<const uint16_t *>(s));
            c = scratch_.data();
        }
        if (2 * (n_ + 1) > tag_.size()) grow();
        const uint64_t h = hash(c, k);
        const uint32_t tg = tag_of(h);
        const size_t mask = tag_.size() - 1;
        for (size_t i = (size_t)h & mask;; i = (i + 1) & mask) {
            const uint32_t t = tag_[i];
            if (t == 0) {
                tag_[i] = tg;
                at_[i] = (uint64_t)arena_.size() << 16 | (uint64_t)k;
                arena_.insert(arena_.end(), c, c + k);
                n_++;
                return true;
            }
            if (t == tg && (at_[i] & 0xffff) == k &&
                std::equal(c, c + k, arena_.data() + (at_[i] >> 16)))
                return false;
        }
    }
    bool insert(const Series &s, bool neg) { return insert(s.data(), s.size(), neg); }
    size_t size() const { return n_; }
    void clear() {
        tag_.clear();
        at_.clear();
        arena_.clear();
        n_ = 0;
    }
    // f(columns, length) for every member, in no particular order.
    template <class F>
    void for_each(F &&f) const {
        for (size_t i = 0; i < tag_.size(); i++)
            if (tag_[i]) f(arena_.data() + (at_[i] >> 16), (size_t)(at_[i] & 0xffff));
    }

  private:
    // Four columns per multiply, then a final mix (series are at most
    // EBIC_MAX_K = 512 columns, which fits the 16-bit length field).
    static uint64_t hash(const uint16_t *c, size_t k) {
        uint64_t h = 0x9E3779B97F4A7C15ULL ^ k;
        size_t i = 0;
        for (; i + 4 <= k; i += 4) {
            uint64_t w;
            std::memcpy(&w, c + i, sizeof w);
            h = (h ^ w) * 0xBF58476D1CE4E5B9ULL;
            h ^= h >> 29;
        }
        uint64_t w = 0;
        for (size_t q = 0; i + q < k; q++) w |= (uint64_t)c[i + q] << (16 * q);
        h = (h ^ w) * 0x94D049BB133111EBULL;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ULL;
        return h ^ (h >> 32);
    }
    static uint32_t tag_of(uint64_t h) { return (uint32_t)(h >> 32) | 1u; }
    void grow() {
        const size_t cap = std::max<size_t>(1024, 2 * tag_.size());
        std::vector<uint32_t> tag(cap, 0);
        std::vector<uint64_t> at(cap, 0);
        const size_t mask = cap - 1;
        for (size_t j = 0; j < tag_.size(); j++) {
            if (!tag_[j]) continue;
            const uint64_t h = hash(arena_.data() + (at_[j] >> 16), (size_t)(at_[j] & 0xffff));
            size_t i = (size_t)h & mask;
            while (tag[i]) i = (i + 1) & mask;
            tag[i] = tag_[j];
            at[i] = at_[j];
        }
        tag_.swap(tag);
        at_.swap(at);
    }
    std::vector<uint32_t> tag_;  // per slot: 0 free, else part of the series' hash
    std::vector<uint64_t> at_;   // per slot: arena offset << 16 | length
    std::vector<uint16_t> arena_, scratch_;
    size_t n_ = 0;
};

// Top-rank order: larger score first, then the lexicographically smaller
// series (a proper prefix first).
inline bool ranks_above(double sa, const Series &a, double sb, const Series &b) {
    if (sa != sb) return sa > sb;
    return std::lexicographical_compare(a.begin(), a.end(), b.begin(), b.end());
}

struct Member {
    Series s;
    std::vector<uint64_t> support;
    int32_t n = 0;
    double score = 0.0;
};

struct ResultImpl {
    ebic_result pub{};
    std::vector<ebic_bicluster> bcs;
    std::vector<std::vector<int32_t>> rows;
    std::vector<std::vector<uint8_t>> dirs;
    std::vector<Series> cols;
    std::vector<double> trace;
};

template <typename T>
struct DeviceArray {
    T *p = nullptr;
    size_t n = 0;
    const ebic_allocator *al = nullptr;
    hipStream_t st = nullptr;
    DeviceArray() = default;
    DeviceArray(const DeviceArray &) = delete;
    DeviceArray &operator=(const DeviceArray &) = delete;
    ~DeviceArray() { reset(); }
    void reset() {
        if (p) device_release(al, p, st);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count, const ebic_allocator *a = nullptr, hipStream_t s = nullptr) {
        reset();
        n = count ? count : 1;
        al = a;
        st = s;
        p = static_cast<T *>(device_alloc(al, n * sizeof(T), st));
        return p ? hipSuccess : hipErrorOutOfMemory;
    }
};

template <typename T>
struct PinnedArray {
    T *p = nullptr;
    size_t n = 0;
    PinnedArray() = default;
    PinnedArray(const PinnedArray &) = delete;
    PinnedArray &operator=(const PinnedArray &) = delete;
    ~PinnedArray() {
        if (p) (void)hipHostFree(p);
    }
    hipError_t alloc(size_t count) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = count ? count : 1;
        const hipError_t e =
            hipHostMalloc(reinterpret_cast<void **>(&p), n * sizeof(T), hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            n = 0;
        }
        return e;
    }
};

#define RUN_HIP(call)                                     \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return check_hip(e_, #call); \
    } while (0)

struct DevLoopAccess;

class Job {
    friend struct DevLoopAccess;  // the generations on the device (devloop.hip)

  public:
    Job(const ebic_params &p, uint64_t seed, hipStream_t stream)
        : p_(p), rng_(seed), stream_(stream), neg_(p.negative_trends != 0) {
        bool any = false;
        for (int o = 0; o < 5; o++) any |= p.op_permille[o] != 0;
        for (int o = 0; o < 5; o++) op_w_[o] = any ? p.op_permille[o] : 200;
    }

    // Device bytes a job of this shape holds (matrix, ranks, pair table when
    // used, population, outputs, archive).
    static size_t footprint(int32_t rows, int32_t cols, const ebic_params &p, bool pairs);
    // Bytes of the pair tables a job with these parameters builds when it
    // uses the pair form (the strict table too under the strict and loose
    // tie rules).
    static size_t pair_table_bytes(int32_t rows, int32_t cols, const ebic_params &p) {
        return ebic_pairs_bytes(rows, cols) * (p.tie_rule == EBIC_TIE_INDEX ? 1 : 2);
    }
    // Allocate, ingest the matrix, build the pair table when `pairs`; with
    // own_staging false the job is only ever staged through stage_into()
    // and gets no staging buffers of its own.
    int setup(const float *h_x, int32_t rows, int32_t cols, bool pairs, bool own_staging = true);
    void start();                     // step 1
    int stage(ebic_job *job);         // upload what is to be scored next
    int fetch();                      // queue the outputs' download
    // After fetch()'s download has arrived: when it held no supports, the
    // ones the top-rank list update looks at first, gathered and downloaded
    // (waits for the stream).
    int fetch_first();
    // Staging through buffers shared by many jobs (one upload and one
    // download for all of them): the byte sizes of this job's slices for the
    // next stage (inputs; scores and counts; supports), then the packing of
    // its inputs into h_in (whose device copy is d_in), with its scores and
    // counts directed to d_out (read back from h_out, its host copy) and its
    // supports to d_sup (left on the device). Slices start 256-byte aligned.
    void slice_bytes(size_t *in_bytes, size_t *out_bytes, size_t *sup_bytes) const;
    void stage_into(ebic_job *job, uint8_t *h_in, uint8_t *d_in, uint8_t *h_out, uint8_t *d_out,
                    uint8_t *d_sup);
    // After a stage_into's scores have arrived: reads them and orders the
    // candidates for the top-rank list; *first (may be NULL) gets the first
    // up to `m` of them, the individuals whose supports the list update will
    // look at first (none in the final evaluation).
    int plan(size_t m, std::vector<int32_t> *first);
    // Host copies of the supports of plan()'s first candidates, in that
    // order, W words each; others are fetched from the device one by one.
    void set_first_supports(const uint64_t *h) { first_sup_ = h; }
    // The supports' words (rows_pad / 64) and their device copy.
    int32_t words() const { return W_; }
    const uint64_t *device_supports() const { return got_dsup_; }
    int advance();                    // host steps after the scores arrived
    bool done() const { return phase_ == Phase::Done; }
    ResultImpl *take_result() { return res_.release(); }
    int64_t evaluations() const { return evaluations_; }
    // Device memory from `al` (copied; NULL: hipMalloc); set before setup.
    void set_allocator(const ebic_allocator *al) {
        if (al) {
            alloc_ = *al;
            al_ = &alloc_;
        }
    }
    const ebic_allocator *allocator() const { return al_; }
    // The stream later steps queue on (set up on one stream, run on another);
    // the caller has synchronized the old one.
    void set_stream(hipStream_t s) { stream_ = s; }
    // The host matrix (rows x cols, row-major), read by the final step for
    // the rows' directions; it must stay valid while the job runs.
    void set_host_matrix(const float *hx) { hx_ = hx; }
    // Host state between steps, as bytes (see ebic_session_checkpoint).
    void save(std::vector<uint8_t> &out, uint64_t matrix_hash) const;
    // Reads a checkpoint's header; false if it is not one.
    static bool peek(const uint8_t *p, size_t n, ebic_params *params, int32_t *rows,
                     int32_t *cols, uint64_t *matrix_hash);
    // Restores the host state (after setup); EBIC_ERR_INVALID_ARG if malformed.
    int load(const uint8_t *p, size_t n);

  private:
    enum class Phase { Eval, FinalEval, Done };
    int take_scores();
    void order_candidates(size_t m);
    int update_archive();
    const uint64_t *support_of(int32_t i, size_t pos);
    void next_population();
    int finish();
    int tournament(const std::vector<double> &key, int n);
    int unused_column(const Series &s);
    // Writes a mutant of a tournament winner into child (its storage reused).
    void mutate(const std::vector<Series> &pop, const std::vector<double> &key, Series &child);
    double size_score(int32_t n, int k) const {
        return (n >= p_.min_rows && k >= p_.k_score_min) ? std::ldexp((double)n, k) : 0.0;
    }
    // Per row: 0 if it follows the series' increasing trend within the
    // tolerance, else 1 (it is in the support, so the reversed one fits).
    std::vector<uint8_t> row_directions(const std::vector<int32_t> &rows, const Series &s) const;
    int64_t shared_rows(const uint64_t *a, const uint64_t *b) const {
        int64_t h = 0;
        for (int w = 0; w < W_; w++) h += __builtin_popcountll(a[w] & b[w]);
        return h;
    }
    static int64_t shared_cols(const Series &a, const Series &b) {
        int64_t g = 0;
        for (uint16_t x : a)
            if (std::find(b.begin(), b.end(), x) != b.end()) g++;
        return g;
    }

    ebic_params p_;
    int32_t op_w_[5];  // operator weights (all-zero op_permille: 200 each)
    SplitMix64 rng_;
    hipStream_t stream_;
    bool neg_;
    ebic_allocator alloc_{};
    const ebic_allocator *al_ = nullptr;
    const float *hx_ = nullptr;
    int32_t R_ = 0, C_ = 0, W_ = 0;
    ebic_matrix m_{};
    DeviceArray<float> d_x_;
    DeviceArray<uint16_t> d_ranks_;
    DeviceArray<uint64_t> d_pairs_, d_pairs_strict_;
    DeviceArray<int32_t> d_sel_, d_roff_, d_rows_;
    // Own staging (stage() and fetch()): every input in one block each
    // way, and the scores, counts and then the supports in another, so a
    // generation takes one upload and one download; when the supports are
    // large only the ones the top-rank list update looks at come down,
    // gathered on the device (fetch_first()).
    PinnedArray<uint8_t> h_in_, h_out_;
    DeviceArray<uint8_t> d_in_, d_out_;
    PinnedArray<WordSpan> h_spans_;
    DeviceArray<WordSpan> d_spans_;
    PinnedArray<uint64_t> h_first_;
    DeviceArray<uint64_t> d_first_;
    size_t staged_down_ = 0;  // bytes fetch() downloads for this stage
    bool all_supports_ = true;

    Phase phase_ = Phase::Eval;
    int stop_ = 0;
    int32_t g_ = 0;
    int64_t evaluations_ = 0;
    std::vector<Series> pop_;   // being scored (or the final list)
    int32_t staged_P_ = 0;
    // where advance() reads the scores: the job's own pinned arrays, or its
    // slice of a shared download
    const double *got_fit_ = nullptr;
    const int32_t *got_cnt_ = nullptr;
    const uint64_t *got_sup_ = nullptr;
    const uint64_t *got_dsup_ = nullptr;  // the same supports on the device
    // the top-rank list update's candidates: scores, the ones not yet taken
    // (a heap, best on top, in its first heap_n_ entries), the first ones
    // taken off it in order, and their supports when the host has only those
    std::vector<double> score_;
    std::vector<int32_t> cand_, first_;
    size_t heap_n_ = 0;
    bool planned_ = false;
    const uint64_t *first_sup_ = nullptr;
    std::vector<uint64_t> fetched_;
    struct Slices {
        size_t off, cols, order, asup, aoff, acols, in_bytes;
        size_t fit, cnt, out_bytes, sup_bytes;
    };
    Slices slices() const;
    // The layout for P individuals with len columns in all, and K members
    // with alen columns, W support words each.
    static Slices layout(int32_t P, size_t len, int32_t K, size_t alen, int32_t W);
    size_t first_count() const { return 2 * (size_t)std::max(p_.archive_size, 0) + 8; }
    void pack(int32_t *off, uint16_t *cols, int32_t *order, uint64_t *asup, int32_t *aoff,
              uint16_t *acols) const;
    TabuSet tabu_;
    int64_t tabu_hits_ = 0;
    std::vector<Member> archive_;
    std::vector<Series> spare_;  // storage of an earlier population, for children
    std::vector<uint8_t> in_;    // scratch: a mark per column, all clear between uses
    std::vector<double> fitness_;
    std::vector<int32_t> count_;
    std::vector<int32_t> use_;
    std::unique_ptr<ResultImpl> res_{new ResultImpl()};
};

int check_run_params(int32_t rows, int32_t cols, const ebic_params *p);
// The device loop's own limits on the run parameters.
int devloop_check(int32_t cols, const ebic_params &p);
// Device memory the device loop of such a run takes beside the job's own
// (an upper bound: the tabu set as if every slot of every generation
// brought a new series).
size_t devloop_bytes(int32_t rows, int32_t cols, const ebic_params &p);
// Runs a started job's generations on the device (devloop.hip), scoring
// each population with *batch; on return the job is in its final step.
int devloop_run(Job &job, Batch **batch, hipStream_t stream);
// 64-bit hash of a float matrix's bytes (FNV-1a over 8-byte words).
uint64_t matrix_hash(const float *x, size_t n);

}  // namespace ebic
