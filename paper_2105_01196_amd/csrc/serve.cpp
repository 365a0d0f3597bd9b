// Job server: continuous batching of many runs of the method on one GPU.
//
// A scheduler thread owns a stream. It admits queued jobs whose device
// footprint fits the remaining HBM budget (arrival order, so a large job is
// never starved by smaller ones behind it) and hands them to preparer
// threads, which set them up on streams of their own (allocation, upload,
// ranks, pair tables, first population) while the ticks go on. A tick takes
// every job that wants scores (just prepared, or its last host step done):
// it packs their populations and top-rank lists into one staging buffer,
// uploads it with one copy, scores them all in one batched launch,
// downloads scores and counts with one copy, orders each job's candidates
// and gathers the supports their top-rank list updates look at first. Each
// job's host step then runs as a task of its own on the worker pool, so no
// job waits for the slowest one; the tick's buffers (one of a few slots)
// stay reserved until those steps have read them. Finished jobs release
// their device memory and slot.
#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "job.h"

namespace ebic {
namespace {

// Threads (each with a stream) setting admitted jobs up beside the ticks.
constexpr int kPreparers = 3;
// Runner threads when device loops are asked for.
constexpr int kRunners = 2;
// Longest wait, in microseconds, for more jobs to join a tick.
constexpr int kGather = 500;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Fixed pool of host threads. Jobs' host steps are queued as tasks (each job
// runs its own as soon as its scores are in); parallel(n, fn) runs fn(0..n-1)
// on the calling thread and on workers ahead of the queued tasks, and
// returns when all n are done.
class WorkerPool {
  public:
    explicit WorkerPool(int n) {
        for (int i = 0; i < n; i++) threads_.emplace_back([this] { work(); });
    }
    ~WorkerPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        for (auto &t : threads_) t.join();
    }
    void submit(std::function<void()> task) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            tasks_.push_back(std::move(task));
        }
        cv_.notify_one();
    }
    // fn(0) .. fn(n - 1), the calling thread among the workers: it takes
    // items itself, so a pool busy with long tasks does not hold it up.
    // Helpers go to the front of the queue; one that starts after every item
    // is taken returns without touching fn (its state is shared, not on the
    // caller's stack).
    void parallel(size_t n, const std::function<void(size_t)> &fn) {
        if (n == 0) return;
        struct State {
            std::atomic<size_t> next{0};
            std::mutex m;
            std::condition_variable done;
            size_t finished = 0;
            const std::function<void(size_t)> *fn = nullptr;
        };
        auto st = std::make_shared<State>();
        st->fn = &fn;
        auto body = [](State &s, size_t n) {
            for (size_t i; (i = s.next.fetch_add(1)) < n;) {
                (*s.fn)(i);
                std::lock_guard<std::mutex> l(s.m);
                if (++s.finished == n) s.done.notify_all();
            }
        };
        const size_t helpers = std::min(n - 1, threads_.size());
        if (helpers > 0) {
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (size_t h = 0; h < helpers; h++)
                    tasks_.push_front([st, n, body] { body(*st, n); });
            }
            cv_.notify_all();
        }
        body(*st, n);
        std::unique_lock<std::mutex> l(st->m);
        st->done.wait(l, [&] { return st->finished == n; });
    }

  private:
    void work() {
        for (;;) {
            std::function<void()> task;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return quit_ || !tasks_.empty(); });
                if (tasks_.empty()) return;  // quitting with nothing queued
                task = std::move(tasks_.front());
                tasks_.pop_front();
            }
            task();
        }
    }
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<std::function<void()>> tasks_;
    bool quit_ = false;
};

// The server's own copy of a submitted matrix, made before submit returns
// (the caller may free theirs then). Fresh pages fault in on first write,
// which made one thread's copy of the serving mix's 1.75 GB take 0.39 s, so
// a large matrix is copied by several threads, into memory that may use
// 2 MB pages.
class HostCopy {
  public:
    HostCopy() = default;
    HostCopy(const HostCopy &) = delete;
    HostCopy &operator=(const HostCopy &) = delete;
    ~HostCopy() { clear(); }
    bool assign(const float *src, size_t n) {
        clear();
        const size_t bytes = n * sizeof(float);
        void *m = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
        if (m == MAP_FAILED) return false;
        (void)madvise(m, bytes, MADV_HUGEPAGE);  // a hint: refused where not enabled
        p_ = static_cast<float *>(m);
        bytes_ = bytes;
        // slices of at least kSlice bytes, at most kThreads of them
        constexpr size_t kSlice = size_t(32) << 20;
        constexpr size_t kThreads = 16;
        const size_t parts = std::min(kThreads, std::max<size_t>(1, bytes / kSlice));
        const size_t per = (n + parts - 1) / parts;
        auto copy = [&](size_t q) {
            const size_t b = q * per, e = std::min(n, b + per);
            if (b < e) std::memcpy(p_ + b, src + b, (e - b) * sizeof(float));
        };
        std::vector<std::thread> th;
        size_t q = 1;
        try {
            for (; q < parts; q++) th.emplace_back(copy, q);
        } catch (...) {  // no thread to be had: this one copies the rest
        }
        for (size_t r = q; r < parts; r++) copy(r);
        copy(0);
        for (auto &t : th) t.join();
        return true;
    }
    float *data() { return p_; }
    void clear() {
        if (p_) munmap(p_, bytes_);
        p_ = nullptr;
        bytes_ = 0;
    }

  private:
    float *p_ = nullptr;
    size_t bytes_ = 0;
};

struct ServerJob {
    int64_t id = 0;
    HostCopy x;
    int32_t rows = 0, cols = 0;
    ebic_params params{};
    uint64_t seed = 0;
    bool pairs = false;
    bool device_loop = false;  // runs on a runner thread (generations on the device)
    size_t footprint = 0;
    std::unique_ptr<Job> job;
    double t_submit = 0, t_done = 0;
    int status = EBIC_PENDING;  // published under the server's lock
    std::string error;
    int end_status = EBIC_OK;   // set by the thread that ends the job, then published
    std::string end_error;
    ResultImpl *result = nullptr;
};

}  // namespace

class Server {
  public:
    int init(const ebic_server_config *cfg);
    ~Server();
    int submit(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p, uint64_t seed,
               int64_t *id);
    int poll(int64_t id, ebic_result **out, bool block);
    void stats(ebic_server_metrics *st);

  private:
    // Staging buffers of one tick (inputs, scores and counts, supports, the
    // gathered first supports), reserved until the host steps of its jobs
    // have read them: pending counts the steps not yet finished.
    struct Slot {
        PinnedArray<uint8_t> h_in, h_out;
        DeviceArray<uint8_t> d_in, d_out, d_sup;
        PinnedArray<WordSpan> h_spans;
        DeviceArray<WordSpan> d_spans;
        PinnedArray<uint64_t> h_first;
        DeviceArray<uint64_t> d_first;
        Batch *batch = nullptr;
        int pending = 0;  // under mu_
    };
    static constexpr int kSlots = 4;

    void loop();
    void prepare_loop(hipStream_t stream);
    void runner_loop(hipStream_t stream);
    void tick(std::vector<std::shared_ptr<ServerJob>> &jobs, Slot &sl);
    void finish_job(const std::shared_ptr<ServerJob> &j, int status, const char *err);
    void release_loop();
    void end_jobs(const std::vector<std::shared_ptr<ServerJob>> &ended);
    bool admissible() const;
    int fetch_first_supports(Slot &sl, const std::vector<std::shared_ptr<ServerJob>> &jobs,
                             const std::vector<std::vector<int32_t>> &first,
                             std::vector<size_t> *at);

    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_, cv_prep_, cv_rel_, cv_run_;
    std::deque<std::shared_ptr<ServerJob>> queue_;
    // admitted, waiting for the preparer; prepared, waiting for a tick;
    // ended, waiting for their memory to be freed
    std::deque<std::shared_ptr<ServerJob>> prep_q_, ready_, rel_q_;
    std::deque<std::shared_ptr<ServerJob>> run_q_;  // admitted device-loop jobs
    std::deque<std::shared_ptr<ServerJob>> host_done_;  // host step finished
    std::unordered_map<int64_t, std::shared_ptr<ServerJob>> jobs_;
    std::vector<double> latencies_;
    int64_t next_id_ = 1, submitted_ = 0, completed_ = 0, failed_ = 0, evaluations_ = 0;
    int64_t ticks_ = 0, device_loop_jobs_ = 0;
    int32_t dl_population_ = 0;  // 0: no device loops
    int64_t n_active_ = 0;  // admitted, result not yet published
    int64_t n_held_ = 0;    // admitted, memory not yet freed (the slots in use)
    bool rel_quit_ = false;
    double busy_s_ = 0, stage_s_ = 0, device_s_ = 0, host_s_ = 0, setup_s_ = 0, release_s_ = 0;
    double device_loop_s_ = 0;
    size_t budget_ = 0, in_use_ = 0;
    int32_t max_active_ = 64;
    bool stop_ = false;
    int device_ = 0;
    hipStream_t stream_ = nullptr;
    std::vector<hipStream_t> prep_streams_;  // one per preparer thread
    std::vector<hipStream_t> run_streams_;   // one per runner thread
    Slot slots_[kSlots];
    std::unique_ptr<WorkerPool> pool_;
    std::thread thread_, rel_thread_;
    std::vector<std::thread> prep_threads_, run_threads_;
};

int Server::init(const ebic_server_config *cfg) {
    EBIC_HIP(hipGetDevice(&device_));
    size_t free_b = 0, total_b = 0;
    EBIC_HIP(hipMemGetInfo(&free_b, &total_b));
    budget_ = (cfg && cfg->hbm_budget) ? cfg->hbm_budget : free_b / 10 * 8;
    max_active_ = (cfg && cfg->max_active > 0) ? cfg->max_active : 64;
    if (cfg && cfg->device_loop_population > 0) dl_population_ = cfg->device_loop_population;
    const int runners = dl_population_ <= 0 ? 0
                        : (cfg && cfg->device_loop_runners > 0) ? cfg->device_loop_runners
                                                                : kRunners;
    EBIC_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
    for (int w = 0; w < kPreparers; w++) {
        hipStream_t st = nullptr;
        EBIC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        prep_streams_.push_back(st);
    }
    const unsigned hw = std::thread::hardware_concurrency();
    pool_.reset(new WorkerPool((int)std::max(1u, std::min(hw ? hw : 1u, 16u))));
    for (int r = 0; r < runners; r++) {
        hipStream_t st = nullptr;
        EBIC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        run_streams_.push_back(st);
    }
    for (hipStream_t st : prep_streams_) prep_threads_.emplace_back([this, st] { prepare_loop(st); });
    for (hipStream_t st : run_streams_) run_threads_.emplace_back([this, st] { runner_loop(st); });
    rel_thread_ = std::thread([this] { release_loop(); });
    thread_ = std::thread([this] { loop(); });
    return EBIC_OK;
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
    cv_prep_.notify_all();
    cv_run_.notify_all();
    // the scheduler ends once every admitted job is done, so the preparers
    // and runners have nothing left when they are told to stop
    if (thread_.joinable()) thread_.join();
    for (auto &t : prep_threads_) t.join();
    for (auto &t : run_threads_) t.join();
    {
        std::lock_guard<std::mutex> lk(mu_);
        rel_quit_ = true;  // nothing ends any more; free what is left
    }
    cv_rel_.notify_all();
    if (rel_thread_.joinable()) rel_thread_.join();
    pool_.reset();
    for (Slot &sl : slots_)
        if (sl.batch) batch_destroy(sl.batch);
    if (stream_) (void)hipStreamDestroy(stream_);
    for (hipStream_t st : prep_streams_) (void)hipStreamDestroy(st);
    for (hipStream_t st : run_streams_) (void)hipStreamDestroy(st);
    for (auto &kv : jobs_) delete kv.second->result;
}

int Server::submit(const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                   uint64_t seed, int64_t *id) {
    if (!h_x || !p || !id) return fail(EBIC_ERR_INVALID_ARG, "NULL argument");
    int rc = check_run_params(rows, cols, p);
    if (rc) return rc;
    if (rows > EBIC_MAX_ROWS || cols > EBIC_MAX_COLS ||
        (int64_t)cols * rows_padded(rows) > INT32_MAX)
        return fail(EBIC_ERR_INVALID_ARG, "matrix shape %d x %d not supported", rows, cols);
    auto j = std::make_shared<ServerJob>();
    if (!j->x.assign(h_x, (size_t)rows * cols))
        return fail(EBIC_ERR_OOM, "host copy of a %d x %d matrix", rows, cols);
    j->rows = rows;
    j->cols = cols;
    j->params = *p;
    j->seed = seed;
    {
        std::lock_guard<std::mutex> lk(mu_);
        const size_t pb = Job::pair_table_bytes(rows, cols, *p);
        j->pairs = pb > 0 && pb <= budget_ / 8;
        j->footprint = Job::footprint(rows, cols, *p, j->pairs);
        j->device_loop = !run_streams_.empty() && dl_population_ > 0 &&
                         p->population >= dl_population_ &&
                         devloop_check(cols, *p) == EBIC_OK;
        if (j->device_loop) {
            // the device loop's memory, and staging of the job's own for the
            // final step (inputs, scores, counts and supports)
            const size_t W = (size_t)rows_padded(rows) / 64;
            j->footprint += devloop_bytes(rows, cols, *p) +
                            (size_t)std::max(p->population, p->archive_size) *
                                (4 + 2 * (size_t)p->k_max + 8 + 4 + 8 * W);
        }
        j->id = next_id_++;
        j->t_submit = now_s();
        jobs_[j->id] = j;
        queue_.push_back(j);
        submitted_++;
        *id = j->id;
    }
    cv_work_.notify_all();
    return EBIC_OK;
}

int Server::poll(int64_t id, ebic_result **out, bool block) {
    if (!out) return fail(EBIC_ERR_INVALID_ARG, "out is NULL");
    std::unique_lock<std::mutex> lk(mu_);
    auto it = jobs_.find(id);
    if (it == jobs_.end()) return fail(EBIC_ERR_INVALID_ARG, "unknown job %lld", (long long)id);
    std::shared_ptr<ServerJob> j = it->second;
    if (block) cv_done_.wait(lk, [&] { return j->status != EBIC_PENDING; });
    if (j->status == EBIC_PENDING) return EBIC_PENDING;
    jobs_.erase(id);
    if (j->status != EBIC_OK) return fail(j->status, "job %lld: %s", (long long)id, j->error.c_str());
    *out = &j->result->pub;
    j->result = nullptr;
    return EBIC_OK;
}

void Server::stats(ebic_server_metrics *st) {
    std::lock_guard<std::mutex> lk(mu_);
    *st = ebic_server_metrics{};
    st->submitted = submitted_;
    st->completed = completed_;
    st->failed = failed_;
    st->queued = (int64_t)queue_.size();
    st->active = n_active_;
    st->evaluations = evaluations_;
    st->ticks = ticks_;
    if (!latencies_.empty()) {
        std::vector<double> l = latencies_;
        std::sort(l.begin(), l.end());
        auto q = [&](double f) {
            const size_t i = (size_t)std::min<double>(l.size() - 1, std::ceil(f * l.size()) - 1);
            return l[i];
        };
        st->p50_latency_s = q(0.50);
        st->p99_latency_s = q(0.99);
        double sum = 0;
        for (double v : l) sum += v;
        st->mean_latency_s = sum / l.size();
    }
    st->busy_s = busy_s_;
    st->stage_s = stage_s_;
    st->device_s = device_s_;
    st->host_s = host_s_;
    st->setup_s = setup_s_;
    st->release_s = release_s_;
    st->hbm_in_use = in_use_;
    st->hbm_budget = budget_;
    st->device_loop_jobs = device_loop_jobs_;
    st->device_loop_s = device_loop_s_;
}

// Called with mu_ held.
void Server::finish_job(const std::shared_ptr<ServerJob> &j, int status, const char *err) {
    j->status = status;
    if (err) j->error = err;
    j->t_done = now_s();
    if (status == EBIC_OK) {
        completed_++;
        latencies_.push_back(j->t_done - j->t_submit);
    } else {
        failed_++;
    }
}

namespace {
// Grows a pinned host buffer and its device twin to hold `count` elements.
template <typename T>
int grow(PinnedArray<T> &h, DeviceArray<T> &d, size_t count) {
    if (count <= h.n && h.p) return EBIC_OK;
    // doubling: every regrowth frees (device-synchronizing) and allocates
    // pinned memory, and a tick's buffers grow as more jobs join them
    const size_t room = 2 * count + 512;
    EBIC_HIP(h.alloc(room));
    EBIC_HIP(d.alloc(room));
    return EBIC_OK;
}
template <typename T>
int grow(DeviceArray<T> &d, size_t count) {
    if (count <= d.n && d.p) return EBIC_OK;
    EBIC_HIP(d.alloc(2 * count + 512));
    return EBIC_OK;
}
}  // namespace

// Downloads, for every job of the tick, the supports of the candidates its
// top-rank list update looks at first (gathered on the device into one
// buffer); job i's land at sl.h_first.p + (*at)[i].
int Server::fetch_first_supports(Slot &sl, const std::vector<std::shared_ptr<ServerJob>> &jobs,
                                 const std::vector<std::vector<int32_t>> &first,
                                 std::vector<size_t> *at) {
    const size_t n = jobs.size();
    at->assign(n + 1, 0);
    size_t spans = 0;
    for (size_t i = 0; i < n; i++) {
        (*at)[i + 1] = (*at)[i] + first[i].size() * (size_t)jobs[i]->job->words();
        spans += first[i].size();
    }
    if (spans == 0) return EBIC_OK;
    int rc = grow(sl.h_spans, sl.d_spans, spans);
    if (rc == EBIC_OK) rc = grow(sl.h_first, sl.d_first, (*at)[n]);
    if (rc) return rc;
    size_t q = 0;
    for (size_t i = 0; i < n; i++) {
        const Job &jb = *jobs[i]->job;
        const int64_t W = jb.words();
        for (size_t pos = 0; pos < first[i].size(); pos++)
            sl.h_spans.p[q++] = WordSpan{jb.device_supports() + (size_t)first[i][pos] * W,
                                         (uint64_t)((*at)[i] + pos * W), W};
    }
    EBIC_HIP(hipMemcpyAsync(sl.d_spans.p, sl.h_spans.p, sizeof(WordSpan) * spans,
                            hipMemcpyHostToDevice, stream_));
    rc = launch_gather_spans(sl.d_spans.p, (int32_t)spans, sl.d_first.p, stream_);
    if (rc) return rc;
    EBIC_HIP(hipMemcpyAsync(sl.h_first.p, sl.d_first.p, sizeof(uint64_t) * (*at)[n],
                            hipMemcpyDeviceToHost, stream_));
    EBIC_HIP(hipStreamSynchronize(stream_));
    return EBIC_OK;
}

// One tick over the jobs whose previous host step is done: pack (worker
// pool, largest populations first), one upload, one launch, one download of
// scores and counts, candidate order, the first candidates' supports; then
// every job's host step is queued as its own task, reading the slot's
// buffers, which stay reserved until the last of those steps has finished.
void Server::tick(std::vector<std::shared_ptr<ServerJob>> &jobs, Slot &sl) {
    const size_t n = jobs.size();
    std::vector<ebic_job> views(n);
    std::stable_sort(jobs.begin(), jobs.end(), [](const std::shared_ptr<ServerJob> &a,
                                                   const std::shared_ptr<ServerJob> &b) {
        return a->params.population > b->params.population;
    });
    const double t0 = now_s();
    std::vector<size_t> in_at(n + 1, 0), out_at(n + 1, 0), sup_at(n + 1, 0);
    for (size_t i = 0; i < n; i++) {
        size_t ib = 0, ob = 0, sb = 0;
        jobs[i]->job->slice_bytes(&ib, &ob, &sb);
        in_at[i + 1] = in_at[i] + ib;
        out_at[i + 1] = out_at[i] + ob;
        sup_at[i + 1] = sup_at[i] + sb;
    }
    int rc = grow(sl.h_in, sl.d_in, in_at[n]);
    if (rc == EBIC_OK) rc = grow(sl.h_out, sl.d_out, out_at[n]);
    if (rc == EBIC_OK) rc = grow(sl.d_sup, sup_at[n]);
    if (rc == EBIC_OK)
        pool_->parallel(n, [&](size_t i) {
            jobs[i]->job->stage_into(&views[i], sl.h_in.p + in_at[i], sl.d_in.p + in_at[i],
                                     sl.h_out.p + out_at[i], sl.d_out.p + out_at[i],
                                     sl.d_sup.p + sup_at[i]);
        });
    const double t1 = now_s();
    if (rc == EBIC_OK) {
        const hipError_t e =
            hipMemcpyAsync(sl.d_in.p, sl.h_in.p, in_at[n], hipMemcpyHostToDevice, stream_);
        if (e != hipSuccess) rc = check_hip(e, "hipMemcpyAsync");
    }
    if (rc == EBIC_OK) rc = batch_set(&sl.batch, views.data(), (int32_t)n, stream_);
    if (rc == EBIC_OK) rc = batch_run(sl.batch, stream_);
    if (rc == EBIC_OK) {
        hipError_t e =
            hipMemcpyAsync(sl.h_out.p, sl.d_out.p, out_at[n], hipMemcpyDeviceToHost, stream_);
        if (e == hipSuccess) e = hipStreamSynchronize(stream_);
        if (e != hipSuccess) rc = check_hip(e, "download");
    }
    std::vector<int> st(n, rc);
    std::vector<std::string> msg(n, rc ? ebic_last_error() : "");
    // which candidates' supports each top-rank list update looks at first
    std::vector<std::vector<int32_t>> first(n);
    const double t2a = now_s();
    if (rc == EBIC_OK)
        pool_->parallel(n, [&](size_t i) {
            const size_t m = 2 * (size_t)std::max(jobs[i]->params.archive_size, 0) + 8;
            st[i] = jobs[i]->job->plan(m, &first[i]);
            if (st[i]) {
                msg[i] = ebic_last_error();
                first[i].clear();
            }
        });
    const double t2b = now_s();
    std::vector<size_t> first_at;
    if (rc == EBIC_OK) {
        rc = fetch_first_supports(sl, jobs, first, &first_at);
        if (rc) {
            const std::string e = ebic_last_error();
            for (size_t i = 0; i < n; i++)
                if (st[i] == EBIC_OK) {
                    st[i] = rc;
                    msg[i] = e;
                }
        }
    }
    const double t3 = now_s();
    std::vector<std::shared_ptr<ServerJob>> failed;
    {
        std::lock_guard<std::mutex> lk(mu_);
        ticks_++;
        stage_s_ += t1 - t0;
        device_s_ += (t2a - t1) + (t3 - t2b);
        host_s_ += t2b - t2a;
        for (size_t i = 0; i < n; i++)
            if (st[i] == EBIC_OK) sl.pending++;
    }
    for (size_t i = 0; i < n; i++) {
        auto j = jobs[i];
        if (st[i] != EBIC_OK) {
            j->end_status = st[i];
            j->end_error = msg[i];
            failed.push_back(j);
            continue;
        }
        if (!first[i].empty()) j->job->set_first_supports(sl.h_first.p + first_at[i]);
        Slot *slot = &sl;
        pool_->submit([this, j, slot] {
            (void)hipSetDevice(device_);
            const double a = now_s();
            const int s = j->job->advance();
            std::string e = s ? ebic_last_error() : "";
            const double b = now_s();
            {
                std::lock_guard<std::mutex> lk(mu_);
                host_s_ += b - a;
                j->end_status = s;
                j->end_error = std::move(e);
                host_done_.push_back(j);
                slot->pending--;
            }
            cv_work_.notify_all();
        });
    }
    end_jobs(failed);
}

// Publishes the ended jobs' results (status in ServerJob::end_status)
// and hands them to the releaser; their footprint and slot stay taken until
// their memory is freed.
void Server::end_jobs(const std::vector<std::shared_ptr<ServerJob>> &ended) {
    if (ended.empty()) return;
    {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto &j : ended) {
            const int status = j->end_status;
            if (status == EBIC_OK) evaluations_ += j->job->evaluations();
            finish_job(j, status, status ? j->end_error.c_str() : nullptr);
            rel_q_.push_back(j);
        }
        n_active_ -= (int64_t)ended.size();
    }
    cv_done_.notify_all();
    cv_rel_.notify_all();
}

// Frees ended jobs' device and host memory on a thread of its own (a device
// free waits for all the GPU's queued work), then returns their footprint
// and slot to admission.
void Server::release_loop() {
    (void)hipSetDevice(device_);
    for (;;) {
        std::vector<std::shared_ptr<ServerJob>> gone;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_rel_.wait(lk, [&] { return rel_quit_ || !rel_q_.empty(); });
            if (rel_q_.empty()) return;
            gone.assign(rel_q_.begin(), rel_q_.end());
            rel_q_.clear();
        }
        const double t0 = now_s();
        for (auto &j : gone) {
            j->job.reset();
            j->x.clear();
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            release_s_ += now_s() - t0;
            for (auto &j : gone) in_use_ -= j->footprint;
            n_held_ -= (int64_t)gone.size();
        }
        cv_work_.notify_all();
    }
}

// With mu_ held: whether the queue's head can be decided now (admitted, or
// failed for exceeding the whole budget).
bool Server::admissible() const {
    if (queue_.empty()) return false;
    const size_t f = queue_.front()->footprint;
    return f > budget_ || (in_use_ + f <= budget_ && n_held_ < max_active_);
}

void Server::prepare_loop(hipStream_t stream) {
    (void)hipSetDevice(device_);
    for (;;) {
        std::shared_ptr<ServerJob> j;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_prep_.wait(lk, [&] { return stop_ || !prep_q_.empty(); });
            if (prep_q_.empty()) return;  // stopping, and nothing admitted is left
            j = prep_q_.front();
            prep_q_.pop_front();
        }
        const double t0 = now_s();
        j->job.reset(new Job(j->params, j->seed, stream));
        j->job->set_host_matrix(j->x.data());  // the job's own copy, for row directions
        int rc = j->job->setup(j->x.data(), j->rows, j->cols, j->pairs, false);
        if (rc == EBIC_OK) {
            const hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) rc = check_hip(e, "hipStreamSynchronize");
        }
        std::string err;
        if (rc == EBIC_OK) {
            j->job->start();
            j->job->set_stream(stream_);
        } else {
            err = ebic_last_error();
        }
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(mu_);
            setup_s_ += t1 - t0;
            if (rc == EBIC_OK) ready_.push_back(j);
        }
        if (rc != EBIC_OK) {
            j->end_status = rc;
            j->end_error = err;
            end_jobs({j});
        }
        cv_work_.notify_all();
    }
}

// A runner takes admitted device-loop jobs one at a time, sets each up as
// a preparer does, runs its generations on the device (devloop_run) and its
// final step with a batch of its own, all on the runner's stream, and ends
// it; its result is the job's ebic_run result, as from the ticks.
void Server::runner_loop(hipStream_t stream) {
    (void)hipSetDevice(device_);
    Batch *batch = nullptr;
    for (;;) {
        std::shared_ptr<ServerJob> j;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_run_.wait(lk, [&] { return stop_ || !run_q_.empty(); });
            if (run_q_.empty()) break;  // stopping, and nothing admitted is left
            j = run_q_.front();
            run_q_.pop_front();
        }
        const double t0 = now_s();
        j->job.reset(new Job(j->params, j->seed, stream));
        j->job->set_host_matrix(j->x.data());
        Job &job = *j->job;
        // staging buffers of its own: the final step is staged and fetched
        // as in a session, not packed by a tick
        int rc = job.setup(j->x.data(), j->rows, j->cols, j->pairs, true);
        if (rc == EBIC_OK) {
            const hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) rc = check_hip(e, "hipStreamSynchronize");
        }
        if (rc == EBIC_OK) {
            job.start();
            rc = devloop_run(job, &batch, stream);
        }
        while (rc == EBIC_OK && !job.done()) {  // the final step (step 9)
            ebic_job view;
            rc = job.stage(&view);
            if (rc == EBIC_OK) rc = batch_set(&batch, &view, 1, stream, job.allocator());
            if (rc == EBIC_OK) rc = batch_run(batch, stream);
            if (rc == EBIC_OK) rc = job.fetch();
            if (rc == EBIC_OK) {
                const hipError_t e = hipStreamSynchronize(stream);
                if (e != hipSuccess) rc = check_hip(e, "hipStreamSynchronize");
            }
            if (rc == EBIC_OK) rc = job.fetch_first();
            if (rc == EBIC_OK) rc = job.advance();
        }
        if (rc == EBIC_OK) {
            j->result = job.take_result();
        } else {
            j->end_status = rc;
            j->end_error = ebic_last_error();
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            device_loop_s_ += now_s() - t0;
        }
        end_jobs({j});
        cv_work_.notify_all();
    }
    if (batch) batch_destroy(batch);
}

void Server::loop() {
    (void)hipSetDevice(device_);
    std::vector<std::shared_ptr<ServerJob>> idle;  // scores wanted: prepared or stepped
    for (;;) {
        std::vector<std::shared_ptr<ServerJob>> ended;
        Slot *free_slot = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu_);
            auto slot_free = [&] {
                for (Slot &s : slots_)
                    if (s.pending == 0) return &s;
                return static_cast<Slot *>(nullptr);
            };
            cv_work_.wait(lk, [&] {
                return stop_ || !ready_.empty() || !host_done_.empty() || admissible() ||
                       (!idle.empty() && slot_free());
            });
            if (stop_ && !queue_.empty()) {  // queued jobs are dropped; admitted ones finish
                while (!queue_.empty()) {
                    finish_job(queue_.front(), EBIC_ERR_CAPACITY, "server stopped");
                    queue_.pop_front();
                }
                cv_done_.notify_all();
            }
            if (stop_ && n_active_ == 0) break;
            bool admitted = false;
            while (admissible()) {
                auto j = queue_.front();
                queue_.pop_front();
                if (j->footprint > budget_) {
                    finish_job(j, EBIC_ERR_CAPACITY, "footprint exceeds the HBM budget");
                    cv_done_.notify_all();
                    continue;
                }
                in_use_ += j->footprint;
                n_active_++;  // admitted jobs count as active
                n_held_++;
                if (j->device_loop) {
                    run_q_.push_back(j);
                    device_loop_jobs_++;
                } else {
                    prep_q_.push_back(j);
                }
                admitted = true;
            }
            if (admitted) {
                cv_prep_.notify_all();
                cv_run_.notify_all();
            }
            while (!ready_.empty()) {
                idle.push_back(ready_.front());
                ready_.pop_front();
            }
            while (!host_done_.empty()) {
                auto j = host_done_.front();
                host_done_.pop_front();
                if (j->end_status != EBIC_OK || j->job->done())
                    ended.push_back(j);
                else
                    idle.push_back(j);
            }
            free_slot = slot_free();
        }
        for (auto &j : ended)
            if (j->end_status == EBIC_OK) j->result = j->job->take_result();
        end_jobs(ended);
        ended.clear();
        if (idle.empty() || !free_slot) continue;
        {
            // a short window for more jobs to finish their host steps while
            // fewer than half of the running ones want scores, so a launch
            // carries more than a few populations
            std::unique_lock<std::mutex> lk(mu_);
            const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(kGather);
            auto stepping = [&] {
                size_t n = 0;
                for (const Slot &sl : slots_) n += (size_t)sl.pending;
                return n;
            };
            while (!stop_ && 2 * idle.size() < idle.size() + stepping() &&
                   cv_work_.wait_until(lk, until) != std::cv_status::timeout) {
                while (!host_done_.empty()) {
                    auto j = host_done_.front();
                    host_done_.pop_front();
                    if (j->end_status != EBIC_OK || j->job->done())
                        ended.push_back(j);
                    else
                        idle.push_back(j);
                }
            }
            while (!host_done_.empty()) {
                auto j = host_done_.front();
                host_done_.pop_front();
                if (j->end_status != EBIC_OK || j->job->done())
                    ended.push_back(j);
                else
                    idle.push_back(j);
            }
        }
        if (!ended.empty()) {
            for (auto &j : ended)
                if (j->end_status == EBIC_OK) j->result = j->job->take_result();
            end_jobs(ended);
            ended.clear();
        }
        const double t0 = now_s();
        tick(idle, *free_slot);
        idle.clear();
        std::lock_guard<std::mutex> lk(mu_);
        busy_s_ += now_s() - t0;
    }
    cv_prep_.notify_all();
}

int server_create(const ebic_server_config *cfg, Server **out) {
    Server *s = new Server();
    int rc = s->init(cfg);
    if (rc) {
        delete s;
        return rc;
    }
    *out = s;
    return EBIC_OK;
}
int server_submit(Server *s, const float *h_x, int32_t rows, int32_t cols, const ebic_params *p,
                  uint64_t seed, int64_t *id) {
    return s->submit(h_x, rows, cols, p, seed, id);
}
int server_poll(Server *s, int64_t id, ebic_result **out, bool block) {
    return s->poll(id, out, block);
}
void server_stats(Server *s, ebic_server_metrics *st) { s->stats(st); }
void server_destroy(Server *s) { delete s; }

}  // namespace ebic
