// ebic_run: the evolutionary loop of Sec. 2.4 (steps 1-9) on the host, with
// every population scored on the GPU by the batched evaluator.
//
// Host parts follow the readings stated in include/ebic.h and the parameter
// comments: SplitMix64 draws, canonical tabu keys, top-rank admission by
// (score, series) with the overlap rule, elitism from the top-rank list,
// tournament on the fitness halved per overused column, five operators.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <unordered_set>
#include <vector>

#include "internal.h"

namespace ebic {
namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).
class SplitMix64 {
  public:
    explicit SplitMix64(uint64_t seed) : state_(seed) {}
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
        const uint64_t reject = (0 - n) % n;
        for (;;) {
            const uint64_t x = next();
            if (x >= reject) return x % n;
        }
    }
    int below_int(int64_t n) { return (int)below((uint64_t)n); }

  private:
    uint64_t state_;
};

using Series = std::vector<uint16_t>;

struct SeriesHash {
    size_t operator()(const Series &s) const {
        uint64_t h = 0x84222325CBF29CE4ULL ^ s.size();
        for (uint16_t c : s) h = (h ^ c) * 0x100000001B3ULL;
        return (size_t)h;
    }
};

// With negative trends a series and its reverse have the same support; the
// smaller of the two stands for both in the tabu list and the top-rank list.
Series canonical(const Series &s, bool neg) {
    if (!neg) return s;
    Series r(s.rbegin(), s.rend());
    return std::lexicographical_compare(r.begin(), r.end(), s.begin(), s.end()) ? r : s;
}

// Top-rank order: larger score first, then the lexicographically smaller
// series (a proper prefix first).
bool ranks_above(double sa, const Series &a, double sb, const Series &b) {
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
    std::vector<Series> cols;
    std::vector<double> trace;
};

template <typename T>
struct DeviceArray {
    T *p = nullptr;
    size_t n = 0;
    ~DeviceArray() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) {
        n = count ? count : 1;
        return hipMalloc(reinterpret_cast<void **>(&p), n * sizeof(T));
    }
};

template <typename T>
struct PinnedArray {
    T *p = nullptr;
    size_t n = 0;
    ~PinnedArray() {
        if (p) (void)hipHostFree(p);
    }
    hipError_t alloc(size_t count) {
        n = count ? count : 1;
        return hipHostMalloc(reinterpret_cast<void **>(&p), n * sizeof(T), hipHostMallocDefault);
    }
};

#define RUN_HIP(call)                                     \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return check_hip(e_, #call); \
    } while (0)

class Runner {
  public:
    Runner(const ebic_params &p, uint64_t seed, hipStream_t stream)
        : p_(p), rng_(seed), stream_(stream), neg_(p.negative_trends != 0) {}
    ~Runner() {
        if (batch_) batch_destroy(batch_);
    }

    int setup(const float *h_x, int32_t rows, int32_t cols);
    int run(ResultImpl *res);

  private:
    // Scores pop against the current top-rank list (or none): fills the
    // fitness, counts and support words (P x W) on the host.
    int evaluate(const std::vector<Series> &pop, bool with_archive);
    void update_archive(const std::vector<Series> &pop);
    int tournament(const std::vector<double> &key, int n);
    int unused_column(const Series &s);
    Series mutate(const std::vector<Series> &pop, const std::vector<double> &key);
    double size_score(int32_t n, int k) const {
        return (n >= p_.min_rows && k >= p_.k_score_min) ? std::ldexp((double)n, k) : 0.0;
    }
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
    SplitMix64 rng_;
    hipStream_t stream_;
    bool neg_;
    int32_t R_ = 0, C_ = 0, W_ = 0;
    ebic_matrix m_{};
    DeviceArray<float> d_x_;
    DeviceArray<uint16_t> d_ranks_;
    DeviceArray<uint64_t> d_pairs_;
    DeviceArray<int32_t> d_off_, d_order_, d_cnt_, d_aoff_, d_sel_, d_roff_, d_rows_;
    DeviceArray<uint16_t> d_cols_, d_acols_;
    DeviceArray<double> d_fit_;
    DeviceArray<uint64_t> d_sup_, d_asup_;
    PinnedArray<int32_t> h_off_, h_order_, h_cnt_, h_aoff_;
    PinnedArray<uint16_t> h_cols_, h_acols_;
    PinnedArray<double> h_fit_;
    PinnedArray<uint64_t> h_sup_, h_asup_;
    Batch *batch_ = nullptr;
    int32_t batch_P_ = -1, batch_K_ = -1;

    std::unordered_set<Series, SeriesHash> tabu_;
    int64_t tabu_hits_ = 0;
    std::vector<Member> archive_;
    std::vector<double> fitness_;
    std::vector<int32_t> count_;
};

int Runner::setup(const float *h_x, int32_t rows, int32_t cols) {
    R_ = rows;
    C_ = cols;
    const int32_t P = p_.population, K = p_.archive_size, kmax = p_.k_max;
    RUN_HIP(d_x_.alloc((size_t)rows * cols));
    RUN_HIP(hipMemcpyAsync(d_x_.p, h_x, sizeof(float) * rows * cols, hipMemcpyHostToDevice,
                           stream_));
    RUN_HIP(d_ranks_.alloc(ebic_matrix_bytes(rows, cols) / sizeof(uint16_t)));
    int rc = ebic_matrix_prepare(d_x_.p, rows, cols, d_ranks_.p, &m_, stream_);
    if (rc) return rc;
    W_ = m_.rows_pad / 64;
    size_t free_b = 0, total_b = 0;
    RUN_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t pair_bytes = ebic_pairs_bytes(rows, cols);
    if (pair_bytes > 0 && pair_bytes <= free_b / 4) {
        RUN_HIP(d_pairs_.alloc(pair_bytes / sizeof(uint64_t)));
        rc = ebic_pairs_prepare(&m_, d_pairs_.p, stream_);
        if (rc) return rc;
    }
    const int32_t nmax = std::max(P, K);
    RUN_HIP(d_off_.alloc(nmax + 1));
    RUN_HIP(d_order_.alloc(nmax));
    RUN_HIP(d_cols_.alloc((size_t)nmax * kmax));
    RUN_HIP(d_fit_.alloc(nmax));
    RUN_HIP(d_cnt_.alloc(nmax));
    RUN_HIP(d_sup_.alloc((size_t)nmax * W_));
    RUN_HIP(d_asup_.alloc((size_t)K * W_));
    RUN_HIP(d_aoff_.alloc(K + 1));
    RUN_HIP(d_acols_.alloc((size_t)K * kmax));
    RUN_HIP(h_off_.alloc(nmax + 1));
    RUN_HIP(h_order_.alloc(nmax));
    RUN_HIP(h_cols_.alloc((size_t)nmax * kmax));
    RUN_HIP(h_fit_.alloc(nmax));
    RUN_HIP(h_cnt_.alloc(nmax));
    RUN_HIP(h_sup_.alloc((size_t)nmax * W_));
    RUN_HIP(h_asup_.alloc((size_t)K * W_));
    RUN_HIP(h_aoff_.alloc(K + 1));
    RUN_HIP(h_acols_.alloc((size_t)K * kmax));
    return EBIC_OK;
}

int Runner::evaluate(const std::vector<Series> &pop, bool with_archive) {
    const int32_t P = (int32_t)pop.size();
    const int32_t K = with_archive ? (int32_t)archive_.size() : 0;
    // compressed population, longest series first
    h_off_.p[0] = 0;
    for (int32_t i = 0; i < P; i++) {
        std::copy(pop[i].begin(), pop[i].end(), h_cols_.p + h_off_.p[i]);
        h_off_.p[i + 1] = h_off_.p[i] + (int32_t)pop[i].size();
    }
    std::iota(h_order_.p, h_order_.p + P, 0);
    std::stable_sort(h_order_.p, h_order_.p + P,
                     [&](int32_t a, int32_t b) { return pop[a].size() > pop[b].size(); });
    const int32_t len = h_off_.p[P];
    RUN_HIP(hipMemcpyAsync(d_off_.p, h_off_.p, sizeof(int32_t) * (P + 1), hipMemcpyHostToDevice,
                           stream_));
    RUN_HIP(hipMemcpyAsync(d_cols_.p, h_cols_.p, sizeof(uint16_t) * std::max(len, 1),
                           hipMemcpyHostToDevice, stream_));
    RUN_HIP(hipMemcpyAsync(d_order_.p, h_order_.p, sizeof(int32_t) * std::max(P, 1),
                           hipMemcpyHostToDevice, stream_));
    if (K > 0) {
        h_aoff_.p[0] = 0;
        for (int32_t j = 0; j < K; j++) {
            const Member &a = archive_[j];
            std::copy(a.support.begin(), a.support.end(), h_asup_.p + (size_t)j * W_);
            std::copy(a.s.begin(), a.s.end(), h_acols_.p + h_aoff_.p[j]);
            h_aoff_.p[j + 1] = h_aoff_.p[j] + (int32_t)a.s.size();
        }
        RUN_HIP(hipMemcpyAsync(d_asup_.p, h_asup_.p, sizeof(uint64_t) * K * W_,
                               hipMemcpyHostToDevice, stream_));
        RUN_HIP(hipMemcpyAsync(d_aoff_.p, h_aoff_.p, sizeof(int32_t) * (K + 1),
                               hipMemcpyHostToDevice, stream_));
        RUN_HIP(hipMemcpyAsync(d_acols_.p, h_acols_.p, sizeof(uint16_t) * h_aoff_.p[K],
                               hipMemcpyHostToDevice, stream_));
    }
    if (P > 0) {
        if (!batch_ || batch_P_ != P || batch_K_ != K) {
            if (batch_) batch_destroy(batch_);
            batch_ = nullptr;
            ebic_job job{};
            job.matrix = m_;
            job.population = ebic_population{P, (int32_t)d_cols_.n, d_off_.p, d_cols_.p,
                                             d_order_.p};
            job.archive = ebic_archive{K, (int32_t)d_acols_.n, d_asup_.p, d_aoff_.p, d_acols_.p};
            job.params = p_;
            job.out = ebic_eval_out{d_fit_.p, d_cnt_.p, d_sup_.p, nullptr};
            int rc = batch_create(&job, 1, 0, &batch_);
            if (rc) return rc;
            batch_P_ = P;
            batch_K_ = K;
        }
        int rc = batch_run(batch_, stream_);
        if (rc) return rc;
        RUN_HIP(hipMemcpyAsync(h_fit_.p, d_fit_.p, sizeof(double) * P, hipMemcpyDeviceToHost,
                               stream_));
        RUN_HIP(hipMemcpyAsync(h_cnt_.p, d_cnt_.p, sizeof(int32_t) * P, hipMemcpyDeviceToHost,
                               stream_));
        RUN_HIP(hipMemcpyAsync(h_sup_.p, d_sup_.p, sizeof(uint64_t) * P * W_,
                               hipMemcpyDeviceToHost, stream_));
    }
    RUN_HIP(hipStreamSynchronize(stream_));
    fitness_.assign(h_fit_.p, h_fit_.p + P);
    count_.assign(h_cnt_.p, h_cnt_.p + P);
    for (int32_t i = 0; i < P; i++)
        if (count_[i] < 0) return fail(EBIC_ERR_DEVICE, "internal: invalid individual %d", i);
    return EBIC_OK;
}

void Runner::update_archive(const std::vector<Series> &pop) {
    const int32_t K = p_.archive_size;
    std::vector<Series> listed;
    for (const Member &a : archive_) listed.push_back(canonical(a.s, neg_));
    std::vector<int32_t> cand;
    std::vector<double> score(pop.size());
    for (size_t i = 0; i < pop.size(); i++) {
        score[i] = size_score(count_[i], (int)pop[i].size());
        if (score[i] > 0 &&
            std::find(listed.begin(), listed.end(), canonical(pop[i], neg_)) == listed.end())
            cand.push_back((int32_t)i);
    }
    std::sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
        return ranks_above(score[a], pop[a], score[b], pop[b]);
    });
    for (int32_t i : cand) {
        const Series &s = pop[i];
        if ((int32_t)archive_.size() == K &&
            !ranks_above(score[i], s, archive_.back().score, archive_.back().s))
            break;
        const uint64_t *sup = h_sup_.p + (size_t)i * W_;
        const int64_t n = count_[i], k = (int64_t)s.size();
        std::vector<size_t> clash;
        bool beats = true;
        for (size_t j = 0; j < archive_.size(); j++) {
            const int64_t h = shared_rows(sup, archive_[j].support.data());
            const int64_t g = shared_cols(s, archive_[j].s);
            if (1000 * h * g > (int64_t)p_.overlap_permille * n * k) {
                clash.push_back(j);
                if (!ranks_above(score[i], s, archive_[j].score, archive_[j].s)) beats = false;
            }
        }
        if (!clash.empty() && !beats) continue;
        for (size_t q = clash.size(); q-- > 0;) archive_.erase(archive_.begin() + clash[q]);
        Member m;
        m.s = s;
        m.support.assign(sup, sup + W_);
        m.n = count_[i];
        m.score = score[i];
        auto at = std::find_if(archive_.begin(), archive_.end(), [&](const Member &a) {
            return !ranks_above(a.score, a.s, m.score, m.s);
        });
        archive_.insert(at, std::move(m));
        if ((int32_t)archive_.size() > K) archive_.pop_back();
    }
}

int Runner::tournament(const std::vector<double> &key, int n) {
    int best = -1;
    for (int d = 0; d < p_.tournament; d++) {
        const int i = rng_.below_int(n);
        if (best < 0 || key[i] > key[best] || (key[i] == key[best] && i < best)) best = i;
    }
    return best;
}

int Runner::unused_column(const Series &s) {
    int pick = rng_.below_int((int64_t)C_ - (int64_t)s.size());
    std::vector<char> in(C_, 0);
    for (uint16_t c : s) in[c] = 1;
    for (int c = 0; c < C_; c++) {
        if (in[c]) continue;
        if (pick-- == 0) return c;
    }
    return -1;
}

Series Runner::mutate(const std::vector<Series> &pop, const std::vector<double> &key) {
    const int n = (int)pop.size();
    const Series &par = pop[tournament(key, n)];
    const int k = (int)par.size();
    enum { INSERT, DELETE, SUBST, SWAP, CROSS };
    int op;
    for (;;) {
        op = rng_.below_int(5);
        if (op == INSERT && !(k < p_.k_max && k < C_)) continue;
        if (op == DELETE && !(k > p_.k_min)) continue;
        if (op == SUBST && !(k < C_)) continue;
        break;
    }
    Series child = par;
    switch (op) {
        case INSERT: {
            const int pos = rng_.below_int(k + 1);
            child.insert(child.begin() + pos, (uint16_t)unused_column(par));
            break;
        }
        case DELETE:
            child.erase(child.begin() + rng_.below_int(k));
            break;
        case SUBST: {
            const int pos = rng_.below_int(k);
            child[pos] = (uint16_t)unused_column(par);
            break;
        }
        case SWAP: {
            const int a = rng_.below_int(k);
            int b = rng_.below_int(k - 1);
            if (b >= a) b++;
            std::swap(child[a], child[b]);
            break;
        }
        default: {
            const Series &other = pop[tournament(key, n)];
            const int a = 1 + rng_.below_int(k - 1);
            const int b = 1 + rng_.below_int((int)other.size() - 1);
            child.assign(par.begin(), par.begin() + a);
            for (int q = b; q < (int)other.size(); q++)
                if (std::find(child.begin(), child.begin() + a, other[q]) == child.begin() + a)
                    child.push_back(other[q]);
        }
    }
    return child;
}

int Runner::run(ResultImpl *res) {
    const int32_t P = p_.population;
    int stop = 0;
    // step 1: random initial population
    std::vector<Series> pop;
    std::vector<int> ident(C_);
    for (int32_t slot = 0; slot < P && !stop; slot++) {
        for (int attempts = 0;; attempts++) {
            if (attempts == p_.max_attempts) {
                stop = EBIC_STOP_EXHAUSTED;
                break;
            }
            const int k = p_.k_min + rng_.below_int(p_.k_max - p_.k_min + 1);
            std::iota(ident.begin(), ident.end(), 0);
            Series s(k);
            for (int j = 0; j < k; j++) {
                std::swap(ident[j], ident[j + rng_.below_int(C_ - j)]);
                s[j] = (uint16_t)ident[j];
            }
            if (!tabu_.insert(canonical(s, neg_)).second) continue;
            pop.push_back(std::move(s));
            break;
        }
    }
    int32_t g = 0;
    int64_t evaluations = 0;
    std::vector<int32_t> use(C_);
    for (;;) {
        // steps 2-3 and 7: score, update the top-rank list
        int rc = evaluate(pop, true);
        if (rc) return rc;
        evaluations += (int64_t)pop.size();
        update_archive(pop);
        res->trace.push_back((double)pop.size());
        res->trace.push_back((double)archive_.size());
        res->trace.push_back(archive_.empty() ? 0.0 : archive_[0].score);
        res->trace.push_back((double)tabu_hits_);
        g++;
        if (stop) break;
        if (g == p_.generations) {
            stop = EBIC_STOP_GENERATIONS;
            break;
        }
        // step 4: elitism
        std::vector<Series> next;
        const size_t elites = std::min(archive_.size(), (size_t)(P / 2));
        for (size_t j = 0; j < elites; j++) next.push_back(archive_[j].s);
        // step 5: tournament key with the column-overuse penalty
        std::fill(use.begin(), use.end(), 0);
        int64_t ksum = 0;
        for (const Series &s : pop) {
            ksum += (int64_t)s.size();
            for (uint16_t c : s) use[c]++;
        }
        const int64_t share = (ksum + C_ - 1) / C_;
        std::vector<double> key(pop.size());
        for (size_t i = 0; i < pop.size(); i++) {
            int over = 0;
            for (uint16_t c : pop[i]) over += use[c] > share;
            key[i] = std::ldexp(fitness_[i], -over);
        }
        // steps 5-6: replenish with mutants; tabu hits end the run
        while ((int32_t)next.size() < P && !stop) {
            for (int attempts = 0;; attempts++) {
                if (attempts == p_.max_attempts) {
                    stop = EBIC_STOP_EXHAUSTED;
                    break;
                }
                Series child = mutate(pop, key);
                if ((int)child.size() < p_.k_min || (int)child.size() > p_.k_max) continue;
                if (!tabu_.insert(canonical(child, neg_)).second) {
                    if (++tabu_hits_ >= p_.max_tabu_hits) {
                        stop = EBIC_STOP_TABU;
                        break;
                    }
                    continue;
                }
                next.push_back(std::move(child));
                break;
            }
        }
        if (stop) break;  // step 6: finish without scoring the new population
        pop.swap(next);
    }
    // step 9: the top-rank list alone, and its rows
    const int32_t nb = std::min((int32_t)archive_.size(), std::max(p_.n_out, 0));
    std::vector<Series> fin;
    for (int32_t j = 0; j < nb; j++) fin.push_back(archive_[j].s);
    int rc = evaluate(fin, false);
    if (rc) return rc;
    if (nb > 0) {
        std::vector<int32_t> sel(nb), roff(nb + 1, 0);
        std::iota(sel.begin(), sel.end(), 0);
        for (int32_t j = 0; j < nb; j++) roff[j + 1] = roff[j] + count_[j];
        RUN_HIP(d_sel_.alloc(nb));
        RUN_HIP(d_roff_.alloc(nb + 1));
        RUN_HIP(d_rows_.alloc(std::max(roff[nb], 1)));
        RUN_HIP(hipMemcpyAsync(d_sel_.p, sel.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice,
                               stream_));
        RUN_HIP(hipMemcpyAsync(d_roff_.p, roff.data(), sizeof(int32_t) * (nb + 1),
                               hipMemcpyHostToDevice, stream_));
        rc = launch_support_rows(d_sup_.p, nb, W_, d_sel_.p, nb, d_roff_.p, d_rows_.p, stream_);
        if (rc) return rc;
        std::vector<int32_t> rows(std::max(roff[nb], 1));
        RUN_HIP(hipMemcpyAsync(rows.data(), d_rows_.p, sizeof(int32_t) * rows.size(),
                               hipMemcpyDeviceToHost, stream_));
        RUN_HIP(hipStreamSynchronize(stream_));
        for (int32_t j = 0; j < nb; j++) {
            res->rows.emplace_back(rows.begin() + roff[j], rows.begin() + roff[j + 1]);
            res->cols.push_back(fin[j]);
        }
        for (int32_t j = 0; j < nb; j++) {
            ebic_bicluster b{};
            b.n_rows = (int32_t)res->rows[j].size();
            b.rows = res->rows[j].data();
            b.n_cols = (int32_t)res->cols[j].size();
            b.cols = res->cols[j].data();
            b.score = size_score(count_[j], (int)fin[j].size());
            res->bcs.push_back(b);
        }
    }
    res->pub.count = nb;
    res->pub.biclusters = res->bcs.data();
    res->pub.generations = g;
    res->pub.evaluations = evaluations;
    res->pub.tabu_hits = tabu_hits_;
    res->pub.stop_reason = stop;
    res->pub.trace = res->trace.data();
    return EBIC_OK;
}

}  // namespace

int run_method(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p, uint64_t seed,
               hipStream_t stream, ebic_result **out) {
    if (!h_x || !p || !out) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    int rc = check_eval_params(p);
    if (rc) return rc;
    if (rows < 1 || cols < 2 || p->k_min < 2 || p->k_max < p->k_min || p->k_max > EBIC_MAX_K ||
        p->k_max > cols || p->population < 1 || p->generations < 1 || p->archive_size < 1 ||
        p->archive_size > EBIC_MAX_ARCHIVE || p->tournament < 1 || p->max_attempts < 1 ||
        p->max_tabu_hits < 1 || p->n_out < 0)
        return fail(EBIC_ERR_INVALID_ARG, "run parameters out of range");
    std::unique_ptr<ResultImpl> res(new ResultImpl());
    {
        Runner r(*p, seed, stream);
        rc = r.setup(h_x, rows, cols);
        if (rc == EBIC_OK) rc = r.run(res.get());
    }
    if (rc) return rc;
    *out = &res.release()->pub;
    return EBIC_OK;
}

void free_result(ebic_result *r) {
    // pub is the first member of ResultImpl
    delete reinterpret_cast<ResultImpl *>(r);
}

}  // namespace ebic
