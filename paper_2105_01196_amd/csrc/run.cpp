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
#include <unordered_set>
#include <vector>

#include "job.h"

namespace ebic {

size_t Job::footprint(int32_t rows, int32_t cols, const ebic_params &p, bool pairs) {
    const size_t rp = (size_t)rows_padded(rows), W = rp / 64;
    const size_t nmax = (size_t)std::max(p.population, p.archive_size);
    size_t b = sizeof(float) * rows * cols + 2 * rp * cols;
    if (pairs) b += ebic_pairs_bytes(rows, cols);
    b += nmax * (4 + 4 + 2 * (size_t)p.k_max + 8 + 4 + 8 * W) + 4;
    b += (size_t)p.archive_size * (8 * W + 4 + 2 * (size_t)p.k_max) + 4;
    return b + (1 << 20);  // slack for allocation granularity
}

int Job::setup(const float *h_x, int32_t rows, int32_t cols, bool pairs) {
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
    const size_t pair_bytes = ebic_pairs_bytes(rows, cols);
    if (pairs && pair_bytes > 0) {
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

int Job::stage(ebic_job *job) {
    const std::vector<Series> &pop = pop_;
    const bool with_archive = phase_ == Phase::Eval;
    const int32_t P = (int32_t)pop.size();
    const int32_t K = with_archive ? (int32_t)archive_.size() : 0;
    staged_P_ = P;
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
    *job = ebic_job{};
    job->matrix = m_;
    job->population = ebic_population{P, (int32_t)d_cols_.n, d_off_.p, d_cols_.p, d_order_.p};
    job->archive = ebic_archive{K, (int32_t)d_acols_.n, d_asup_.p, d_aoff_.p, d_acols_.p};
    job->params = p_;
    job->out = ebic_eval_out{d_fit_.p, d_cnt_.p, d_sup_.p, nullptr};
    return EBIC_OK;
}

int Job::fetch() {
    const int32_t P = staged_P_;
    if (P == 0) return EBIC_OK;
    RUN_HIP(hipMemcpyAsync(h_fit_.p, d_fit_.p, sizeof(double) * P, hipMemcpyDeviceToHost,
                           stream_));
    RUN_HIP(hipMemcpyAsync(h_cnt_.p, d_cnt_.p, sizeof(int32_t) * P, hipMemcpyDeviceToHost,
                           stream_));
    RUN_HIP(hipMemcpyAsync(h_sup_.p, d_sup_.p, sizeof(uint64_t) * P * W_, hipMemcpyDeviceToHost,
                           stream_));
    return EBIC_OK;
}

void Job::update_archive(const std::vector<Series> &pop) {
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

int Job::tournament(const std::vector<double> &key, int n) {
    int best = -1;
    for (int d = 0; d < p_.tournament; d++) {
        const int i = rng_.below_int(n);
        if (best < 0 || key[i] > key[best] || (key[i] == key[best] && i < best)) best = i;
    }
    return best;
}

int Job::unused_column(const Series &s) {
    int pick = rng_.below_int((int64_t)C_ - (int64_t)s.size());
    if (in_.size() != (size_t)C_) in_.assign(C_, 0);
    for (uint16_t c : s) in_[c] = 1;
    int found = -1;
    for (int c = 0; c < C_ && found < 0; c++) {
        if (in_[c]) continue;
        if (pick-- == 0) found = c;
    }
    for (uint16_t c : s) in_[c] = 0;
    return found;
}

Series Job::mutate(const std::vector<Series> &pop, const std::vector<double> &key) {
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
            if (!tabu_.insert(canonical(s, neg_)).second) continue;
            pop_.push_back(std::move(s));
            break;
        }
    }
    phase_ = Phase::Eval;
}

int Job::advance() {
    const int32_t P = staged_P_;
    fitness_.assign(h_fit_.p, h_fit_.p + P);
    count_.assign(h_cnt_.p, h_cnt_.p + P);
    for (int32_t i = 0; i < P; i++)
        if (count_[i] < 0) return fail(EBIC_ERR_DEVICE, "internal: invalid individual %d", i);
    if (phase_ == Phase::FinalEval) return finish();
    // steps 3 and 7: top-rank list
    evaluations_ += P;
    update_archive(pop_);
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
        for (int attempts = 0;; attempts++) {
            if (attempts == p_.max_attempts) {
                stop_ = EBIC_STOP_EXHAUSTED;
                break;
            }
            Series child = mutate(pop_, key);
            if ((int)child.size() < p_.k_min || (int)child.size() > p_.k_max) continue;
            if (!tabu_.insert(canonical(child, neg_)).second) {
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
    if (!stop_) pop_.swap(next);  // step 6: a stop ends the run before scoring
}

int Job::finish() {
    ResultImpl *res = res_.get();
    const int32_t nb = (int32_t)pop_.size();
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
        int rc = launch_support_rows(d_sup_.p, nb, W_, d_sel_.p, nb, d_roff_.p, d_rows_.p,
                                     stream_);
        if (rc) return rc;
        std::vector<int32_t> rows(std::max(roff[nb], 1));
        RUN_HIP(hipMemcpyAsync(rows.data(), d_rows_.p, sizeof(int32_t) * rows.size(),
                               hipMemcpyDeviceToHost, stream_));
        RUN_HIP(hipStreamSynchronize(stream_));
        for (int32_t j = 0; j < nb; j++) {
            res->rows.emplace_back(rows.begin() + roff[j], rows.begin() + roff[j + 1]);
            res->cols.push_back(pop_[j]);
        }
        for (int32_t j = 0; j < nb; j++) {
            ebic_bicluster b{};
            b.n_rows = (int32_t)res->rows[j].size();
            b.rows = res->rows[j].data();
            b.n_cols = (int32_t)res->cols[j].size();
            b.cols = res->cols[j].data();
            b.score = size_score(count_[j], (int)pop_[j].size());
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
    return EBIC_OK;
}

int run_method(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p, uint64_t seed,
               hipStream_t stream, ebic_result **out) {
    if (!h_x || !p || !out) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    int rc = check_run_params(rows, cols, p);
    if (rc) return rc;
    size_t free_b = 0, total_b = 0;
    EBIC_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t pair_bytes = ebic_pairs_bytes(rows, cols);
    Job job(*p, seed, stream);
    rc = job.setup(h_x, rows, cols, pair_bytes > 0 && pair_bytes <= free_b / 4);
    if (rc) return rc;
    job.start();
    Batch *batch = nullptr;
    while (rc == EBIC_OK && !job.done()) {
        ebic_job view;
        rc = job.stage(&view);
        if (rc == EBIC_OK) rc = batch_set(&batch, &view, 1, stream);
        if (rc == EBIC_OK) rc = batch_run(batch, stream);
        if (rc == EBIC_OK) rc = job.fetch();
        if (rc == EBIC_OK) {
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) rc = check_hip(e, "hipStreamSynchronize");
        }
        if (rc == EBIC_OK) rc = job.advance();
    }
    if (batch) batch_destroy(batch);
    if (rc) return rc;
    *out = &job.take_result()->pub;
    return EBIC_OK;
}

void free_result(ebic_result *r) {
    // pub is the first member of ResultImpl
    delete reinterpret_cast<ResultImpl *>(r);
}

}  // namespace ebic
