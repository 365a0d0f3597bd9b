// One run of the evolutionary loop of Sec. 2.4 (steps 1-9) as a state
// machine: the host parts run between GPU evaluations, and every population
// is scored by the batched evaluator. ebic_run drives one job alone; the
// server drives many and scores their populations in one launch.
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
#include <vector>

#include "job.h"

namespace ebic {

size_t Job::footprint(int32_t rows, int32_t cols, const ebic_params &p, bool pairs) {
    const size_t rp = (size_t)rows_padded(rows), W = rp / 64;
    const size_t nmax = (size_t)std::max(p.population, p.archive_size);
    size_t b = sizeof(float) * rows * cols + 2 * rp * cols;
    if (pairs) b += pair_table_bytes(rows, cols, p);
    b += nmax * (4 + 4 + 2 * (size_t)p.k_max + 8 + 4 + 8 * W) + 4;
    b += (size_t)p.archive_size * (8 * W + 4 + 2 * (size_t)p.k_max) + 4;
    b += (2 * (size_t)p.archive_size + 8) * (8 * W + sizeof(WordSpan));  // gathered supports
    return b + (1 << 20);  // slack for alignment and allocation granularity
}

int Job::setup(const float *h_x, int32_t rows, int32_t cols, bool pairs, bool own_staging) {
    R_ = rows;
    C_ = cols;
    const int32_t P = p_.population, K = p_.archive_size, kmax = p_.k_max;
    RUN_HIP(d_x_.alloc((size_t)rows * cols, al_, stream_));
    RUN_HIP(hipMemcpyAsync(d_x_.p, h_x, sizeof(float) * rows * cols, hipMemcpyHostToDevice,
                           stream_));
    RUN_HIP(d_ranks_.alloc(ebic_matrix_bytes(rows, cols) / sizeof(uint16_t), al_, stream_));
    int rc = ebic_matrix_prepare(d_x_.p, rows, cols, d_ranks_.p, &m_, stream_);
    if (rc) return rc;
    W_ = m_.rows_pad / 64;
    const size_t pair_bytes = ebic_pairs_bytes(rows, cols);
    if (pairs && pair_bytes > 0) {
        RUN_HIP(d_pairs_.alloc(pair_bytes / sizeof(uint64_t), al_, stream_));
        rc = ebic_pairs_prepare(&m_, d_pairs_.p, stream_);
        if (rc) return rc;
        if (p_.tie_rule != EBIC_TIE_INDEX) {  // both tables for the strict and loose rules
            RUN_HIP(d_pairs_strict_.alloc(pair_bytes / sizeof(uint64_t), al_, stream_));
            rc = ebic_pairs_strict_prepare(&m_, d_pairs_strict_.p, stream_);
            if (rc) return rc;
        }
    }
    if (!own_staging) return EBIC_OK;  // stage_into() only
    const int32_t nmax = std::max(P, K);
    const Slices most = layout(nmax, (size_t)nmax * kmax, K, (size_t)K * kmax, W_);
    RUN_HIP(d_in_.alloc(most.in_bytes, al_, stream_));
    RUN_HIP(d_out_.alloc(most.out_bytes + most.sup_bytes, al_, stream_));
    RUN_HIP(d_spans_.alloc(first_count(), al_, stream_));
    RUN_HIP(d_first_.alloc(first_count() * W_, al_, stream_));
    RUN_HIP(h_in_.alloc(most.in_bytes));
    RUN_HIP(h_out_.alloc(most.out_bytes + most.sup_bytes));
    RUN_HIP(h_spans_.alloc(first_count()));
    RUN_HIP(h_first_.alloc(first_count() * W_));
    return EBIC_OK;
}

// The population compressed (longest series first in the processing order)
// and, while generations run, the top-rank list the overlap is taken against.
void Job::pack(int32_t *off, uint16_t *cols, int32_t *order, uint64_t *asup, int32_t *aoff,
               uint16_t *acols) const {
    const std::vector<Series> &pop = pop_;
    const int32_t P = (int32_t)pop.size();
    const int32_t K = phase_ == Phase::Eval ? (int32_t)archive_.size() : 0;
    off[0] = 0;
    for (int32_t i = 0; i < P; i++) {
        std::copy(pop[i].begin(), pop[i].end(), cols + off[i]);
        off[i + 1] = off[i] + (int32_t)pop[i].size();
    }
    // longest first, ties by index: a counting sort over the lengths
    size_t kmax = 0;
    for (const Series &q : pop) kmax = std::max(kmax, q.size());
    std::vector<int32_t> start(kmax + 2, 0);
    for (const Series &q : pop) start[kmax - q.size() + 1]++;
    for (size_t b = 1; b <= kmax + 1; b++) start[b] += start[b - 1];
    for (int32_t i = 0; i < P; i++) order[start[kmax - pop[i].size()]++] = i;
    if (K == 0) return;
    aoff[0] = 0;
    for (int32_t j = 0; j < K; j++) {
        const Member &a = archive_[j];
        std::copy(a.support.begin(), a.support.end(), asup + (size_t)j * W_);
        std::copy(a.s.begin(), a.s.end(), acols + aoff[j]);
        aoff[j + 1] = aoff[j] + (int32_t)a.s.size();
    }
}

// Supports up to this many bytes come down whole with the scores; larger
// ones stay on the device but for the few the top-rank list update reads.
constexpr size_t kWholeSupportBytes = 1 << 20;

int Job::stage(ebic_job *job) {
    if (!h_in_.p) return fail(EBIC_ERR_INVALID_ARG, "internal: the job has no staging buffers");
    const Slices l = slices();
    const size_t sup = sizeof(uint64_t) * pop_.size() * W_;
    stage_into(job, h_in_.p, d_in_.p, h_out_.p, d_out_.p, d_out_.p + l.out_bytes);
    all_supports_ = sup <= kWholeSupportBytes;
    staged_down_ = l.out_bytes + (all_supports_ ? sup : 0);
    if (all_supports_) got_sup_ = reinterpret_cast<const uint64_t *>(h_out_.p + l.out_bytes);
    RUN_HIP(hipMemcpyAsync(d_in_.p, h_in_.p, l.in_bytes, hipMemcpyHostToDevice, stream_));
    return EBIC_OK;
}

Job::Slices Job::layout(int32_t P, size_t len, int32_t K, size_t alen, int32_t W) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    Slices l{};
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at = up(at + bytes);
        return here;
    };
    l.off = take(sizeof(int32_t) * (P + 1));
    l.cols = take(sizeof(uint16_t) * std::max<size_t>(len, 1));
    l.order = take(sizeof(int32_t) * std::max(P, 1));
    l.asup = take(sizeof(uint64_t) * K * W);
    l.aoff = take(sizeof(int32_t) * (K + 1));
    l.acols = take(sizeof(uint16_t) * std::max<size_t>(alen, 1));
    l.in_bytes = at;
    at = 0;
    l.fit = take(sizeof(double) * std::max(P, 1));
    l.cnt = take(sizeof(int32_t) * std::max(P, 1));
    l.out_bytes = at;
    l.sup_bytes = up(sizeof(uint64_t) * std::max(P, 1) * W);
    return l;
}

Job::Slices Job::slices() const {
    const int32_t K = phase_ == Phase::Eval ? (int32_t)archive_.size() : 0;
    size_t len = 0, alen = 0;
    for (const Series &q : pop_) len += q.size();
    for (int32_t j = 0; j < K; j++) alen += archive_[j].s.size();
    return layout((int32_t)pop_.size(), len, K, alen, W_);
}

void Job::slice_bytes(size_t *in_bytes, size_t *out_bytes, size_t *sup_bytes) const {
    const Slices l = slices();
    *in_bytes = l.in_bytes;
    *out_bytes = l.out_bytes;
    *sup_bytes = l.sup_bytes;
}

void Job::stage_into(ebic_job *job, uint8_t *h_in, uint8_t *d_in, uint8_t *h_out, uint8_t *d_out,
                     uint8_t *d_sup) {
    const Slices l = slices();
    const int32_t P = (int32_t)pop_.size();
    const int32_t K = phase_ == Phase::Eval ? (int32_t)archive_.size() : 0;
    staged_P_ = P;
    auto *off = reinterpret_cast<int32_t *>(h_in + l.off);
    auto *aoff = reinterpret_cast<int32_t *>(h_in + l.aoff);
    pack(off, reinterpret_cast<uint16_t *>(h_in + l.cols),
         reinterpret_cast<int32_t *>(h_in + l.order), reinterpret_cast<uint64_t *>(h_in + l.asup),
         aoff, reinterpret_cast<uint16_t *>(h_in + l.acols));
    *job = ebic_job{};
    job->matrix = m_;
    job->population = ebic_population{P, off[P], reinterpret_cast<const int32_t *>(d_in + l.off),
                                      reinterpret_cast<const uint16_t *>(d_in + l.cols),
                                      reinterpret_cast<const int32_t *>(d_in + l.order)};
    job->archive = ebic_archive{K, K > 0 ? aoff[K] : 0,
                                reinterpret_cast<const uint64_t *>(d_in + l.asup),
                                reinterpret_cast<const int32_t *>(d_in + l.aoff),
                                reinterpret_cast<const uint16_t *>(d_in + l.acols)};
    job->params = p_;
    job->out = ebic_eval_out{reinterpret_cast<double *>(d_out + l.fit),
                             reinterpret_cast<int32_t *>(d_out + l.cnt),
                             reinterpret_cast<uint64_t *>(d_sup), nullptr};
    got_fit_ = reinterpret_cast<const double *>(h_out + l.fit);
    got_cnt_ = reinterpret_cast<const int32_t *>(h_out + l.cnt);
    got_sup_ = nullptr;  // the supports stay on the device
    got_dsup_ = reinterpret_cast<const uint64_t *>(d_sup);
    first_sup_ = nullptr;
}

int Job::fetch() {
    if (staged_P_ == 0) return EBIC_OK;
    RUN_HIP(hipMemcpyAsync(h_out_.p, d_out_.p, staged_down_, hipMemcpyDeviceToHost, stream_));
    return EBIC_OK;
}

int Job::fetch_first() {
    if (all_supports_ || staged_P_ == 0) return EBIC_OK;
    int rc = plan(first_count(), nullptr);
    if (rc || first_.empty()) return rc;
    const size_t n = first_.size();
    for (size_t pos = 0; pos < n; pos++)
        h_spans_.p[pos] = WordSpan{got_dsup_ + (size_t)first_[pos] * W_, (uint64_t)(pos * W_), W_};
    RUN_HIP(hipMemcpyAsync(d_spans_.p, h_spans_.p, sizeof(WordSpan) * n, hipMemcpyHostToDevice,
                           stream_));
    rc = launch_gather_spans(d_spans_.p, (int32_t)n, d_first_.p, stream_);
    if (rc) return rc;
    RUN_HIP(hipMemcpyAsync(h_first_.p, d_first_.p, sizeof(uint64_t) * n * W_,
                           hipMemcpyDeviceToHost, stream_));
    RUN_HIP(hipStreamSynchronize(stream_));
    first_sup_ = h_first_.p;
    return EBIC_OK;
}

// Steps 3 and 7, first part: the size scores of the population and its
// candidates for the top-rank list (a positive score, not listed already),
// kept on a heap best first; the first `m` come off it into first_.
// Usually only the first few are ever looked at, hence a heap rather than a
// full sort (the series are distinct, so the order is the same).
void Job::order_candidates(size_t m) {
    const std::vector<Series> &pop = pop_;
    std::vector<Series> listed;
    for (const Member &a : archive_) listed.push_back(canonical(a.s, neg_));
    cand_.clear();
    first_.clear();
    score_.assign(pop.size(), 0.0);
    for (size_t i = 0; i < pop.size(); i++) {
        score_[i] = size_score(count_[i], (int)pop[i].size());
        if (score_[i] > 0 && std::none_of(listed.begin(), listed.end(), [&](const Series &c) {
                return same_canonical(pop[i], c, neg_);
            }))
            cand_.push_back((int32_t)i);
    }
    auto worse = [&](int32_t a, int32_t b) {
        return ranks_above(score_[b], pop[b], score_[a], pop[a]);
    };
    std::make_heap(cand_.begin(), cand_.end(), worse);
    heap_n_ = cand_.size();
    while (first_.size() < m && heap_n_ > 0) {
        std::pop_heap(cand_.begin(), cand_.begin() + heap_n_, worse);
        first_.push_back(cand_[--heap_n_]);
    }
}

// The support of pop_[i], the pos-th candidate taken.
const uint64_t *Job::support_of(int32_t i, size_t pos) {
    if (got_sup_) return got_sup_ + (size_t)i * W_;
    if (first_sup_ && pos < first_.size()) return first_sup_ + pos * W_;
    fetched_.resize(W_);
    if (hipMemcpy(fetched_.data(), got_dsup_ + (size_t)i * W_, sizeof(uint64_t) * W_,
                  hipMemcpyDeviceToHost) != hipSuccess)
        return nullptr;
    return fetched_.data();
}

// Steps 3 and 7, second part: candidates in rank order enter the list
// unless they clash with (overlap too much) a member that ranks above them;
// members they clash with and outrank leave it.
int Job::update_archive() {
    const std::vector<Series> &pop = pop_;
    const int32_t K = p_.archive_size;
    auto worse = [&](int32_t a, int32_t b) {
        return ranks_above(score_[b], pop[b], score_[a], pop[a]);
    };
    for (size_t pos = 0;; pos++) {
        int32_t i;
        if (pos < first_.size()) {
            i = first_[pos];
        } else if (heap_n_ > 0) {
            std::pop_heap(cand_.begin(), cand_.begin() + heap_n_, worse);
            i = cand_[--heap_n_];
        } else {
            break;
        }
        const Series &s = pop[i];
        if ((int32_t)archive_.size() == K &&
            !ranks_above(score_[i], s, archive_.back().score, archive_.back().s))
            break;
        const uint64_t *sup = support_of(i, pos);
        if (!sup) return fail(EBIC_ERR_DEVICE, "support download failed");
        const int64_t n = count_[i], k = (int64_t)s.size();
        std::vector<size_t> clash;
        bool beats = true;
        for (size_t j = 0; j < archive_.size(); j++) {
            // h <= min(n, n_j): when even that cannot clash (g = 0 among
            // others), the rows need no counting
            const int64_t g = shared_cols(s, archive_[j].s);
            const int64_t bound = (int64_t)p_.overlap_permille * n * k;
            if (1000 * std::min<int64_t>(n, archive_[j].n) * g <= bound) continue;
            const int64_t h = shared_rows(sup, archive_[j].support.data());
            if (1000 * h * g > bound) {
                clash.push_back(j);
                if (!ranks_above(score_[i], s, archive_[j].score, archive_[j].s)) beats = false;
            }
        }
        if (!clash.empty() && !beats) continue;
        for (size_t q = clash.size(); q-- > 0;) archive_.erase(archive_.begin() + clash[q]);
        Member m;
        m.s = s;
        m.support.assign(sup, sup + W_);
        m.n = count_[i];
        m.score = score_[i];
        auto at = std::find_if(archive_.begin(), archive_.end(), [&](const Member &a) {
            return !ranks_above(a.score, a.s, m.score, m.s);
        });
        archive_.insert(at, std::move(m));
        if ((int32_t)archive_.size() > K) archive_.pop_back();
    }
    return EBIC_OK;
}

int Job::tournament(const std::vector<double> &key, int n) {
    int best = -1;
    for (int d = 0; d < p_.tournament; d++) {
        const int i = rng_.below_int(n);
        if (best < 0 || key[i] > key[best] || (key[i] == key[best] && i < best)) best = i;
    }
    return best;
}

int Job::unused_column(const Series &s) {
    // The pick-th (from 0) column outside s in ascending order is the least
    // x with x = pick + #{c in s : c <= x}; iterating that map from x = pick
    // climbs to it (the map is monotone and the answer is its least fixed
    // point), usually in two or three passes over s.
    const int pick = rng_.below_int((int64_t)C_ - (int64_t)s.size());
    int x = pick;
    for (;;) {
        int below = 0;
        for (uint16_t c : s) below += c <= x;
        if (pick + below == x) return x;
        x = pick + below;
    }
}

void Job::mutate(const std::vector<Series> &pop, const std::vector<double> &key, Series &child) {
    const int n = (int)pop.size();
    const Series &par = pop[tournament(key, n)];
    const int k = (int)par.size();
    enum { INSERT, DELETE, SUBST, SWAP, CROSS };
    // one draw among the operators that apply, weighted
    const bool applies[5] = {k < p_.k_max && k < C_, k > p_.k_min, k < C_, true, true};
    int total = 0;
    for (int o = 0; o < 5; o++) total += applies[o] ? op_w_[o] : 0;
    if (total == 0) {  // no weighted operator applies: a failed attempt
        child.clear();
        return;
    }
    int op = 0;
    for (int x = rng_.below_int(total);; op++) {
        const int w = applies[op] ? op_w_[op] : 0;
        if (x < w) break;
        x -= w;
    }
    child.assign(par.begin(), par.end());
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
            // the second parent's tail, less the columns already taken from
            // the first (marked in a per-column scratch array, then cleared)
            if (in_.size() != (size_t)C_) in_.assign(C_, 0);
            for (int q = 0; q < a; q++) in_[child[q]] = 1;
            for (int q = b; q < (int)other.size(); q++)
                if (!in_[other[q]]) child.push_back(other[q]);
            for (int q = 0; q < a; q++) in_[child[q]] = 0;
        }
    }
}

void Job::start() {
    const int32_t P = p_.population;
    std::vector<int> ident(C_);
    use_.assign(C_, 0);
    for (int32_t slot = 0; slot < P && !stop_; slot++) {
        for (int attempts = 0;; attempts++) {
            if (attempts == p_.max_attempts) {
                stop_ = EBIC_STOP_EXHAUSTED;
                break;
            }
            const int k = p_.k_min + rng_.below_int(p_.k_max - p_.k_min + 1);
            std::iota(ident.begin(), ident.end(), 0);
            Series s(k);
            for (int j = 0; j < k; j++) {
                std::swap(ident[j], ident[j + rng_.below_int(C_ - j)]);
                s[j] = (uint16_t)ident[j];
            }
            if (!tabu_.insert(s, neg_)) continue;
            pop_.push_back(std::move(s));
            break;
        }
    }
    phase_ = Phase::Eval;
}

int Job::take_scores() {
    const int32_t P = staged_P_;
    fitness_.assign(got_fit_, got_fit_ + P);
    count_.assign(got_cnt_, got_cnt_ + P);
    for (int32_t i = 0; i < P; i++)
        if (count_[i] < 0) return fail(EBIC_ERR_DEVICE, "internal: invalid individual %d", i);
    return EBIC_OK;
}

int Job::plan(size_t m, std::vector<int32_t> *first) {
    int rc = take_scores();
    if (rc) return rc;
    if (phase_ == Phase::Eval) order_candidates(m);
    else first_.clear();
    planned_ = true;
    if (first) *first = first_;
    return EBIC_OK;
}

int Job::advance() {
    const int32_t P = staged_P_;
    if (!planned_) {
        int rc = take_scores();
        if (rc) return rc;
        if (phase_ == Phase::Eval) order_candidates(0);
    }
    planned_ = false;
    if (phase_ == Phase::FinalEval) return finish();
    // steps 3 and 7: top-rank list
    evaluations_ += P;
    int rc = update_archive();
    if (rc) return rc;
    ResultImpl *res = res_.get();
    res->trace.push_back((double)P);
    res->trace.push_back((double)archive_.size());
    res->trace.push_back(archive_.empty() ? 0.0 : archive_[0].score);
    res->trace.push_back((double)tabu_hits_);
    g_++;
    if (!stop_ && g_ == p_.generations) stop_ = EBIC_STOP_GENERATIONS;
    if (!stop_) next_population();
    if (stop_) {
        // step 9: score the top-rank list alone
        const int32_t nb = std::min((int32_t)archive_.size(), std::max(p_.n_out, 0));
        pop_.clear();
        for (int32_t j = 0; j < nb; j++) pop_.push_back(archive_[j].s);
        phase_ = Phase::FinalEval;
    }
    return EBIC_OK;
}

void Job::next_population() {
    const int32_t P = p_.population;
    // step 4: elitism
    std::vector<Series> next;
    const size_t elites = std::min(archive_.size(), (size_t)(P / 2));
    for (size_t j = 0; j < elites; j++) next.push_back(archive_[j].s);
    // step 5: tournament key with the column-overuse penalty
    std::fill(use_.begin(), use_.end(), 0);
    int64_t ksum = 0;
    for (const Series &s : pop_) {
        ksum += (int64_t)s.size();
        for (uint16_t c : s) use_[c]++;
    }
    const int64_t share = (ksum + C_ - 1) / C_;
    std::vector<double> key(pop_.size());
    for (size_t i = 0; i < pop_.size(); i++) {
        int over = 0;
        for (uint16_t c : pop_[i]) over += use_[c] > share;
        key[i] = std::ldexp(fitness_[i], -over);
    }
    // steps 5-6: replenish with mutants; tabu hits end the run
    while ((int32_t)next.size() < P && !stop_) {
        Series child;  // storage from an earlier population when there is some
        if (!spare_.empty()) {
            child.swap(spare_.back());
            spare_.pop_back();
        }
        for (int attempts = 0;; attempts++) {
            if (attempts == p_.max_attempts) {
                stop_ = EBIC_STOP_EXHAUSTED;
                break;
            }
            mutate(pop_, key, child);
            if ((int)child.size() < p_.k_min || (int)child.size() > p_.k_max) continue;
            if (!tabu_.insert(child, neg_)) {
                if (++tabu_hits_ >= p_.max_tabu_hits) {
                    stop_ = EBIC_STOP_TABU;
                    break;
                }
                continue;
            }
            next.push_back(std::move(child));
            break;
        }
    }
    if (stop_) return;  // step 6: a stop ends the run before scoring
    pop_.swap(next);
    for (Series &q : next) spare_.push_back(std::move(q));
}

int Job::finish() {
    ResultImpl *res = res_.get();
    const int32_t nb = (int32_t)pop_.size();
    if (nb > 0) {
        std::vector<int32_t> sel(nb), roff(nb + 1, 0);
        std::iota(sel.begin(), sel.end(), 0);
        for (int32_t j = 0; j < nb; j++) roff[j + 1] = roff[j] + count_[j];
        RUN_HIP(d_sel_.alloc(nb, al_, stream_));
        RUN_HIP(d_roff_.alloc(nb + 1, al_, stream_));
        RUN_HIP(d_rows_.alloc(std::max(roff[nb], 1), al_, stream_));
        RUN_HIP(hipMemcpyAsync(d_sel_.p, sel.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice,
                               stream_));
        RUN_HIP(hipMemcpyAsync(d_roff_.p, roff.data(), sizeof(int32_t) * (nb + 1),
                               hipMemcpyHostToDevice, stream_));
        int rc = launch_support_rows(got_dsup_, nb, W_, d_sel_.p, nb, d_roff_.p, d_rows_.p,
                                     stream_);
        if (rc) return rc;
        std::vector<int32_t> rows(std::max(roff[nb], 1));
        RUN_HIP(hipMemcpyAsync(rows.data(), d_rows_.p, sizeof(int32_t) * rows.size(),
                               hipMemcpyDeviceToHost, stream_));
        RUN_HIP(hipStreamSynchronize(stream_));
        for (int32_t j = 0; j < nb; j++) {
            res->rows.emplace_back(rows.begin() + roff[j], rows.begin() + roff[j + 1]);
            res->cols.push_back(pop_[j]);
            res->dirs.push_back(row_directions(res->rows[j], pop_[j]));
        }
        for (int32_t j = 0; j < nb; j++) {
            ebic_bicluster b{};
            b.n_rows = (int32_t)res->rows[j].size();
            b.rows = res->rows[j].data();
            b.n_cols = (int32_t)res->cols[j].size();
            b.cols = res->cols[j].data();
            b.score = size_score(count_[j], (int)pop_[j].size());
            b.row_dir = res->dirs[j].data();
            res->bcs.push_back(b);
        }
    }
    res->pub.count = nb;
    res->pub.biclusters = res->bcs.data();
    res->pub.generations = g_;
    res->pub.evaluations = evaluations_;
    res->pub.tabu_hits = tabu_hits_;
    res->pub.stop_reason = stop_;
    res->pub.trace = res->trace.data();
    phase_ = Phase::Done;
    return EBIC_OK;
}

int check_run_params(int32_t rows, int32_t cols, const ebic_params *p) {
    int rc = check_eval_params(p);
    if (rc) return rc;
    if (rows < 1 || cols < 2 || p->k_min < 2 || p->k_max < p->k_min || p->k_max > EBIC_MAX_K ||
        p->k_max > cols || p->population < 1 || p->generations < 1 || p->archive_size < 1 ||
        p->archive_size > EBIC_MAX_ARCHIVE || p->tournament < 1 || p->max_attempts < 1 ||
        p->max_tabu_hits < 1 || p->n_out < 0)
        return fail(EBIC_ERR_INVALID_ARG, "run parameters out of range");
    int32_t sum = 0;
    for (int o = 0; o < 5; o++) {
        if (p->op_permille[o] < 0 || p->op_permille[o] > 1000)
            return fail(EBIC_ERR_INVALID_ARG, "op_permille[%d] = %d outside 0..1000", o,
                        p->op_permille[o]);
        sum += p->op_permille[o];
    }
    if (sum != 0 && sum != 1000)
        return fail(EBIC_ERR_INVALID_ARG, "op_permille sums to %d, not 1000 (or all 0)", sum);
    return EBIC_OK;
}

void free_result(ebic_result *r) {
    // pub is the first member of ResultImpl
    delete reinterpret_cast<ResultImpl *>(r);
}

}  // namespace ebic

namespace ebic {

void *device_alloc(const ebic_allocator *al, size_t bytes, hipStream_t stream) {
    if (al && al->alloc) return al->alloc(al->ctx, bytes, stream);
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void device_release(const ebic_allocator *al, void *p, hipStream_t stream) {
    if (!p) return;
    if (al && al->release)
        al->release(al->ctx, p, stream);
    else if (!al || !al->alloc)
        (void)hipFree(p);
}

std::vector<uint8_t> Job::row_directions(const std::vector<int32_t> &rows, const Series &s) const {
    std::vector<uint8_t> dir(rows.size(), 0);
    if (!hx_ || s.size() < 2) return dir;
    const int k = (int)s.size();
    const int t = (int)(((int64_t)(k - 1) * (1000 - p_.approx_permille)) / 1000);
    for (size_t i = 0; i < rows.size(); i++) {
        const float *x = hx_ + (size_t)rows[i] * C_;
        int downs = 0;  // steps against the increasing trend
        for (int j = 0; j + 1 < k; j++) {
            const int a = s[j], b = s[j + 1];
            // the step fits the increasing trend: a smaller value, or a tie
            // that the tie rule lets through
            const bool tie_ok = p_.tie_rule == EBIC_TIE_LOOSE ||
                                (p_.tie_rule == EBIC_TIE_INDEX && a < b);
            const bool up = x[a] < x[b] || (x[a] == x[b] && tie_ok);
            downs += !up;
        }
        dir[i] = downs <= t ? 0 : 1;
    }
    return dir;
}

uint64_t matrix_hash(const float *x, size_t n) {
    uint64_t h = 0xCBF29CE484222325ULL ^ n;
    const size_t bytes = n * sizeof(float);
    const unsigned char *b = reinterpret_cast<const unsigned char *>(x);
    size_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
        uint64_t w;
        std::memcpy(&w, b + i, 8);
        h = (h ^ w) * 0x100000001B3ULL;
    }
    for (; i < bytes; i++) h = (h ^ b[i]) * 0x100000001B3ULL;
    return h;
}

// ---- checkpoint format: a flat little-endian byte stream ----

namespace {

constexpr char kMagic[8] = {'E', 'B', 'I', 'C', 'C', 'K', 'P', '1'};
constexpr uint32_t kVersion = 2;  // 2: ebic_params with op_permille

struct Writer {
    std::vector<uint8_t> &out;
    template <typename T>
    void put(const T &v) {
        const uint8_t *p = reinterpret_cast<const uint8_t *>(&v);
        out.insert(out.end(), p, p + sizeof(T));
    }
    void series(const Series &s) {
        put((uint16_t)s.size());
        for (uint16_t c : s) put(c);
    }
};

struct Reader {
    const uint8_t *p;
    size_t n, at = 0;
    bool ok = true;
    template <typename T>
    T get() {
        T v{};
        if (!ok || n - at < sizeof(T)) {
            ok = false;
            return v;
        }
        std::memcpy(&v, p + at, sizeof(T));
        at += sizeof(T);
        return v;
    }
    Series series(int32_t cols) {
        const uint16_t k = get<uint16_t>();
        Series s;
        if (!ok || k < 2 || k > EBIC_MAX_K) {
            ok = false;
            return s;
        }
        s.resize(k);
        for (auto &c : s) {
            c = get<uint16_t>();
            if (c >= cols) ok = false;
        }
        return s;
    }
};

}  // namespace

void Job::save(std::vector<uint8_t> &out, uint64_t mhash) const {
    out.clear();
    Writer w{out};
    for (char c : kMagic) w.put(c);
    w.put(kVersion);
    w.put(p_);
    w.put(R_);
    w.put(C_);
    w.put(mhash);
    w.put(rng_.state());
    w.put((int32_t)phase_);
    w.put((int32_t)stop_);
    w.put(g_);
    w.put(evaluations_);
    w.put(tabu_hits_);
    w.put((uint64_t)res_->trace.size());
    for (double v : res_->trace) w.put(v);
    w.put((uint32_t)pop_.size());
    for (const Series &s : pop_) w.series(s);
    w.put((uint32_t)archive_.size());
    for (const Member &m : archive_) {
        w.series(m.s);
        w.put(m.n);
        w.put(m.score);
        for (int32_t q = 0; q < W_; q++) w.put(m.support[q]);
    }
    // the tabu list in a canonical (sorted) order, so that equal states
    // give equal bytes
    std::vector<Series> tabu;
    tabu.reserve(tabu_.size());
    tabu_.for_each([&](const uint16_t *c, size_t k) { tabu.emplace_back(c, c + k); });
    std::sort(tabu.begin(), tabu.end(), [](const Series &a, const Series &b) {
        return a.size() != b.size() ? a.size() < b.size() : a < b;
    });
    w.put((uint64_t)tabu.size());
    for (const Series &s : tabu) w.series(s);
    for (char c : kMagic) w.put(c);
}

bool Job::peek(const uint8_t *p, size_t n, ebic_params *params, int32_t *rows, int32_t *cols,
               uint64_t *mhash) {
    Reader r{p, n};
    for (char c : kMagic)
        if (r.get<char>() != c) return false;
    if (r.get<uint32_t>() != kVersion) return false;
    *params = r.get<ebic_params>();
    *rows = r.get<int32_t>();
    *cols = r.get<int32_t>();
    *mhash = r.get<uint64_t>();
    return r.ok;
}

int Job::load(const uint8_t *p, size_t n) {
    Reader r{p, n};
    ebic_params params;
    int32_t rows, cols;
    uint64_t mhash;
    if (!peek(p, n, &params, &rows, &cols, &mhash) || rows != R_ || cols != C_)
        return fail(EBIC_ERR_INVALID_ARG, "not a checkpoint of this run");
    r.at = sizeof(kMagic) + sizeof(uint32_t) + sizeof(ebic_params) + 2 * sizeof(int32_t) +
           sizeof(uint64_t);
    rng_.set_state(r.get<uint64_t>());
    const int32_t phase = r.get<int32_t>(), stop = r.get<int32_t>();
    g_ = r.get<int32_t>();
    evaluations_ = r.get<int64_t>();
    tabu_hits_ = r.get<int64_t>();
    if (!r.ok || phase < (int32_t)Phase::Eval || phase > (int32_t)Phase::FinalEval || stop < 0 ||
        stop > EBIC_STOP_EXHAUSTED || g_ < 0 || g_ > p_.generations)
        return fail(EBIC_ERR_INVALID_ARG, "malformed checkpoint (state)");
    phase_ = (Phase)phase;
    stop_ = stop;
    const uint64_t nt = r.get<uint64_t>();
    if (!r.ok || nt != 4 * (uint64_t)g_) return fail(EBIC_ERR_INVALID_ARG, "malformed checkpoint (trace)");
    res_->trace.resize(nt);
    for (auto &v : res_->trace) v = r.get<double>();
    const uint32_t np = r.get<uint32_t>();
    if (!r.ok || np > (uint32_t)std::max(p_.population, p_.archive_size))
        return fail(EBIC_ERR_INVALID_ARG, "malformed checkpoint (population)");
    pop_.clear();
    for (uint32_t i = 0; i < np && r.ok; i++) pop_.push_back(r.series(C_));
    const uint32_t na = r.get<uint32_t>();
    if (!r.ok || na > (uint32_t)p_.archive_size)
        return fail(EBIC_ERR_INVALID_ARG, "malformed checkpoint (top-rank list)");
    archive_.clear();
    for (uint32_t j = 0; j < na && r.ok; j++) {
        Member m;
        m.s = r.series(C_);
        m.n = r.get<int32_t>();
        m.score = r.get<double>();
        m.support.resize(W_);
        for (auto &wd : m.support) wd = r.get<uint64_t>();
        archive_.push_back(std::move(m));
    }
    const uint64_t ntabu = r.get<uint64_t>();
    tabu_.clear();
    for (uint64_t i = 0; i < ntabu && r.ok; i++) tabu_.insert(r.series(C_), neg_);
    for (char c : kMagic)
        if (r.get<char>() != c) r.ok = false;
    if (!r.ok || r.at != n || tabu_.size() != ntabu)
        return fail(EBIC_ERR_INVALID_ARG, "malformed checkpoint");
    use_.assign(C_, 0);
    return EBIC_OK;
}

// ---- sessions: a run in steps, with checkpoints ----

struct Session {
    std::vector<float> own;  // the session's copy of the matrix (unless borrowed)
    const float *x = nullptr;
    int32_t rows = 0, cols = 0;
    hipStream_t stream = nullptr;
    std::unique_ptr<Job> job;
    Batch *batch = nullptr;
    bool taken = false;
    ~Session() {
        if (batch) batch_destroy(batch);
    }
};

namespace {

// Allocates the job's device state on the session's matrix.
int session_setup(Session *s, const ebic_params &p, uint64_t seed, const ebic_allocator *al) {
    size_t free_b = 0, total_b = 0;
    EBIC_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t pair_bytes = Job::pair_table_bytes(s->rows, s->cols, p);
    s->job.reset(new Job(p, seed, s->stream));
    s->job->set_allocator(al);
    s->job->set_host_matrix(s->x);
    return s->job->setup(s->x, s->rows, s->cols, pair_bytes > 0 && pair_bytes <= free_b / 4);
}

int session_open(const float *h_x, int32_t rows, int32_t cols, bool copy, hipStream_t stream,
                 std::unique_ptr<Session> *out) {
    std::unique_ptr<Session> s(new Session());
    s->rows = rows;
    s->cols = cols;
    s->stream = stream;
    if (copy) {
        s->own.assign(h_x, h_x + (size_t)rows * cols);
        s->x = s->own.data();
    } else {
        s->x = h_x;
    }
    *out = std::move(s);
    return EBIC_OK;
}

int session_begin(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                  uint64_t seed, const ebic_allocator *al, hipStream_t stream, bool copy,
                  std::unique_ptr<Session> *out) {
    if (!h_x || !p || !out) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    int rc = check_run_params(rows, cols, p);
    if (rc) return rc;
    std::unique_ptr<Session> s;
    rc = session_open(h_x, rows, cols, copy, stream, &s);
    if (rc == EBIC_OK) rc = session_setup(s.get(), *p, seed, al);
    if (rc) return rc;
    s->job->start();
    *out = std::move(s);
    return EBIC_OK;
}

}  // namespace

int session_step(Session *s, int32_t steps, int32_t *done) {
    if (!s || !s->job || steps < 0) return fail(EBIC_ERR_INVALID_ARG, "bad session or steps");
    Job &job = *s->job;
    int rc = EBIC_OK;
    for (int32_t i = 0; i < steps && rc == EBIC_OK && !job.done(); i++) {
        ebic_job view;
        rc = job.stage(&view);
        if (rc == EBIC_OK) rc = batch_set(&s->batch, &view, 1, s->stream, job.allocator());
        if (rc == EBIC_OK) rc = batch_run(s->batch, s->stream);
        if (rc == EBIC_OK) rc = job.fetch();
        if (rc == EBIC_OK) {
            hipError_t e = hipStreamSynchronize(s->stream);
            if (e != hipSuccess) rc = check_hip(e, "hipStreamSynchronize");
        }
        if (rc == EBIC_OK) rc = job.fetch_first();
        if (rc == EBIC_OK) rc = job.advance();
    }
    if (done) *done = job.done() ? 1 : 0;
    return rc;
}

int session_create(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                   uint64_t seed, const ebic_allocator *al, hipStream_t stream, Session **out) {
    if (!out) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    std::unique_ptr<Session> s;
    int rc = session_begin(h_x, rows, cols, p, seed, al, stream, true, &s);
    if (rc) return rc;
    *out = s.release();
    return EBIC_OK;
}

int session_checkpoint(Session *s, void *buf, size_t *bytes) {
    if (!s || !s->job || !bytes) return fail(EBIC_ERR_INVALID_ARG, "bad session or size");
    if (s->job->done()) return fail(EBIC_ERR_INVALID_ARG, "the run has finished");
    std::vector<uint8_t> blob;
    s->job->save(blob, matrix_hash(s->x, (size_t)s->rows * s->cols));
    if (!buf) {
        *bytes = blob.size();
        return EBIC_OK;
    }
    if (*bytes < blob.size()) return fail(EBIC_ERR_INVALID_ARG, "buffer too small");
    std::memcpy(buf, blob.data(), blob.size());
    *bytes = blob.size();
    return EBIC_OK;
}

int session_restore(const float *h_x, int32_t rows, int32_t cols, const void *buf, size_t bytes,
                    const ebic_allocator *al, hipStream_t stream, Session **out) {
    if (!h_x || !buf || !out) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    const uint8_t *b = static_cast<const uint8_t *>(buf);
    ebic_params p;
    int32_t r0, c0;
    uint64_t mh;
    if (!Job::peek(b, bytes, &p, &r0, &c0, &mh))
        return fail(EBIC_ERR_INVALID_ARG, "not a checkpoint");
    if (r0 != rows || c0 != cols) return fail(EBIC_ERR_INVALID_ARG, "checkpoint of another shape");
    int rc = check_run_params(rows, cols, &p);
    if (rc) return rc;
    if (matrix_hash(h_x, (size_t)rows * cols) != mh)
        return fail(EBIC_ERR_INVALID_ARG, "checkpoint of another matrix");
    std::unique_ptr<Session> s;
    rc = session_open(h_x, rows, cols, true, stream, &s);
    if (rc == EBIC_OK) rc = session_setup(s.get(), p, 0, al);
    if (rc == EBIC_OK) rc = s->job->load(b, bytes);
    if (rc) return rc;
    *out = s.release();
    return EBIC_OK;
}

int session_result(Session *s, ebic_result **out) {
    if (!s || !s->job || !out) return fail(EBIC_ERR_INVALID_ARG, "bad session");
    if (!s->job->done() || s->taken) return fail(EBIC_ERR_INVALID_ARG, "no result to take");
    s->taken = true;
    *out = &s->job->take_result()->pub;
    return EBIC_OK;
}

void session_free(Session *s) { delete s; }

int run_method_device(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                      uint64_t seed, const ebic_allocator *al, hipStream_t stream,
                      ebic_result **out) {
    if (!out || !p) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    int rc = devloop_check(cols, *p);
    if (rc) return rc;
    std::unique_ptr<Session> s;
    rc = session_begin(h_x, rows, cols, p, seed, al, stream, false, &s);
    if (rc == EBIC_OK) rc = devloop_run(*s->job, &s->batch, s->stream);
    int32_t done = 0;
    while (rc == EBIC_OK && !done) rc = session_step(s.get(), 1 << 30, &done);
    if (rc) return rc;
    return session_result(s.get(), out);
}

int run_method(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p, uint64_t seed,
               const ebic_allocator *al, hipStream_t stream, ebic_result **out) {
    if (!out) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    std::unique_ptr<Session> s;
    // the caller's matrix stays valid for the whole (synchronous) call
    int rc = session_begin(h_x, rows, cols, p, seed, al, stream, false, &s);
    int32_t done = 0;
    while (rc == EBIC_OK && !done) rc = session_step(s.get(), 1 << 30, &done);
    if (rc) return rc;
    return session_result(s.get(), out);
}

}  // namespace ebic
