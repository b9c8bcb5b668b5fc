// Serving loop: continuous batching of independent Darcy + transport jobs.
//
// One FIFO queue, n worker threads, one HIP stream per worker.  A worker
// takes the head job when its estimated device footprint fits in the budget
// left by the running jobs and the cached handles (idle cached handles are
// evicted, least recently used first, to make room).  Each job runs on a
// handle of its own (vag_create, the pressure solve and the transport's
// set-up on the worker's stream, outputs copied to the caller's host
// buffers), so jobs on different workers overlap on the device.
//
// The transport steps of the jobs below kBatchRows control volumes run
// batched: per lane of job sizes, a batcher thread launches, tick after tick
// on a stream of its own, one kernel that takes one step of every active job
// of the lane (up to kBatchJobs per launch).  A job joins at the next tick
// once its set-up is done and leaves after its last step; its worker hands it
// over after the set-up and takes the next job, and a finisher thread waits
// for the last step, copies the outputs and completes the job.  A larger
// job's steps fill the device alone, and its worker launches them.  Each row
// of each job gets the arithmetic of the job run alone, so results are the
// same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <list>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "vag_internal.h"

namespace {

struct Job {
    uint64_t id = 0;
    // owned copies of the inputs
    int64_t nn = 0, nc = 0, nf = 0;
    std::vector<double> xyz, fwidth, fperm, fporo, perm, poro, p_bar, c_bar;
    std::vector<int32_t> hex8, fnodes;
    // a mesh given by its faces (hex8 empty): cell -> faces, face -> nodes,
    // fracture faces by face index
    int64_t n_faces = 0;
    std::vector<int64_t> cell_face_ptr, face_node_ptr;
    std::vector<int32_t> cell_faces, face_nodes, face_ids;
    std::vector<uint8_t> dir;
    double mu = 1.0;
    vag_options opt{};
    int64_t n_steps = 0;
    double t_final = 0.0;
    uint64_t key = 0;
    double *out[6] = {};  // u_node, u_cell, u_frac, c_cell, c_frac, c_node
    size_t est = 0;
    enum { QUEUED, RUNNING, DONE } state = QUEUED;
    vag_job_result res{};
    size_t charged = 0;  // the bytes it holds of the budget while it runs
    vag_status solve_status = VAG_OK;
    // a job whose transport steps run batched: its handle, the event its
    // set-up ends with, and the finisher that completes it
    vag_handle *h = nullptr;
    hipEvent_t ready = nullptr;
    int fin = 0;
};

struct Cached {
    uint64_t key;
    int64_t nn, nc, nf;
    int eliminate;
    vag_handle *h;
    size_t bytes;
};

template <class T>
std::vector<T> copy_in(const T *p, size_t n) {
    if (n && !p) throw std::invalid_argument("null input array");
    return n ? std::vector<T>(p, p + n) : std::vector<T>();
}

// The transport steps of the served jobs, batched per launch.  A worker
// hands a job over once its transport is set up (submit) and takes the next
// job; the batcher calls done(job, failed) once the job's last step is
// launched (the finisher then waits for it).
class StepBatcher {
public:
    using Done = std::function<void(Job *, bool)>;
    StepBatcher(int device, hipStream_t stream, Done done) : device_(device), stream_(stream), done_(std::move(done)) {
        for (auto &e : tick_) {
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
        }
        th_ = std::thread([this] { loop(); });
    }
    ~StepBatcher() {
        {
            std::lock_guard<std::mutex> l(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        th_.join();
        for (auto e : tick_)
            if (e) (void)hipEventDestroy(e);
    }
    // j->h has its transport set up (vag_serving_transport_begin); its steps
    // start after j->ready
    void submit(Job *j, int64_t N) {
        {
            std::lock_guard<std::mutex> l(mu_);
            pending_.push_back(Entry{j, N, 0});
        }
        cv_.notify_all();
    }
    void counts(int64_t *launches, int64_t *steps) {
        std::lock_guard<std::mutex> l(mu_);
        *launches = launches_;
        *steps = steps_;
    }

private:
    struct Entry {
        Job *j;
        int64_t N, k;
    };
    static constexpr int kDepth = 32;  // ticks in flight: the host runs ahead of the device, a new job joins within them

    void loop() {
        (void)hipSetDevice(device_);
        int64_t ticks = 0;
        std::vector<std::pair<Job *, bool>> finished;
        for (;;) {
            {
                std::unique_lock<std::mutex> l(mu_);
                cv_.wait(l, [&] { return stop_ || !pending_.empty() || !active_.empty(); });
                if (stop_ && pending_.empty() && active_.empty()) return;
                while (!pending_.empty()) {
                    Entry e = pending_.front();
                    pending_.pop_front();
                    if (hipStreamWaitEvent(stream_, e.j->ready, 0) != hipSuccess ||
                        hipEventRecord(vag_serving_event(e.j->h, 6), stream_) != hipSuccess)
                        finished.emplace_back(e.j, true);
                    else
                        active_.push_back(e);
                }
            }
            bool ok = true;
            if (!active_.empty()) {
                if (ticks >= kDepth && tick_[ticks % kDepth])
                    ok = hipEventSynchronize(tick_[ticks % kDepth]) == hipSuccess;
                try {
                    for (size_t g = 0; ok && g < active_.size(); g += vag::kBatchJobs) {
                        vag::TransportBatch B{};
                        B.n = (int32_t)std::min<size_t>(vag::kBatchJobs, active_.size() - g);
                        for (int32_t q = 0; q < B.n; ++q) {
                            Entry &e = active_[g + q];
                            vag_serving_transport_job(e.j->h, e.k, &B.job[q]);
                        }
                        vag::launch_transport_batch(stream_, B);
                        std::lock_guard<std::mutex> l(mu_);
                        ++launches_;
                        steps_ += B.n;
                    }
                } catch (...) {
                    ok = false;
                }
                if (ok && tick_[ticks % kDepth]) ok = hipEventRecord(tick_[ticks % kDepth], stream_) == hipSuccess;
                ++ticks;
                std::vector<Entry> still;
                for (Entry &e : active_) {
                    ++e.k;
                    if (!ok)
                        finished.emplace_back(e.j, true);
                    else if (e.k == e.N)
                        finished.emplace_back(e.j, hipEventRecord(vag_serving_event(e.j->h, 7), stream_) != hipSuccess);
                    else
                        still.push_back(e);
                }
                active_.swap(still);
            }
            for (auto &f : finished) done_(f.first, f.second);
            finished.clear();
        }
    }

    int device_;
    hipStream_t stream_;
    Done done_;
    hipEvent_t tick_[kDepth] = {};
    std::thread th_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Entry> pending_;
    std::vector<Entry> active_;  // only the batcher thread touches it
    int64_t launches_ = 0, steps_ = 0;
    bool stop_ = false;
};

}  // namespace

struct vag_server {
    int device = 0;
    size_t budget = 0;
    std::vector<hipStream_t> streams;
    // transport lanes by job size (rows of the upwind operator): a launch
    // takes one step of each job in its lane, so a step of a small job does
    // not wait for the step of a large one
    // Jobs of at least 2^18 rows step on their own: their launches fill the
    // device, and in a shared launch each step would wait for the others.
    static constexpr int kLanes = 3;
    static constexpr int64_t kBatchRows = int64_t(1) << 18;
    static int lane_of(int64_t rows) {  // rows below 2^16, 2^17, 2^18
        int l = 0;
        while (l + 1 < kLanes && rows >= (int64_t(1) << (16 + l))) ++l;
        return l;
    }
    hipStream_t lane_stream[kLanes] = {};
    std::unique_ptr<StepBatcher> lane[kLanes];
    // finishers: each waits for a batched job's last step, copies its
    // outputs (on its own stream, where the job's handle moved when it was
    // handed over), then keeps or destroys the handle and completes the job
    static constexpr int kFinishers = 4;
    hipStream_t fin_stream[kFinishers] = {};
    std::thread fin_thread[kFinishers];
    std::deque<std::pair<Job *, bool>> fin_queue[kFinishers];
    std::condition_variable cv_fin;
    bool fin_stop = false;
    int next_fin = 0;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    std::list<Cached> cache;  // front = most recently used
    size_t in_use = 0, peak = 0, cached_bytes = 0;
    int64_t submitted = 0, running = 0, finished = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    // Under the lock: takes idle cached handles out of the cache, least
    // recently used first, until need more bytes fit in the budget.  The
    // caller destroys them after releasing the lock.
    bool make_room(size_t need, std::vector<vag_handle *> &evicted) {
        while (in_use + cached_bytes + need > budget) {
            if (cache.empty()) return false;
            cached_bytes -= cache.back().bytes;
            evicted.push_back(cache.back().h);
            cache.pop_back();
        }
        return true;
    }

    // a run ends with the handle to keep (or null), or the job handed over
    struct Outcome {
        vag_handle *keep = nullptr;
        bool handed_over = false;
    };
    Outcome run(Job *j, int w, vag_handle *h);
    vag_handle *finish_outputs(Job *j, vag_handle *h, hipStream_t s);
    void complete(Job *j, vag_handle *keep);
    void loop(int w);
    void fin_loop(int f);
    // drains the finishers' queues, then ends their threads
    void stop_finisher() {
        {
            std::lock_guard<std::mutex> lk(mu);
            fin_stop = true;
        }
        cv_fin.notify_all();
        for (auto &t : fin_thread)
            if (t.joinable()) t.join();
    }
};

void vag_server::loop(int w) {
    (void)hipSetDevice(device);
    for (;;) {
        Job *j = nullptr;
        vag_handle *reuse = nullptr;
        size_t charged = 0;
        std::vector<vag_handle *> evicted;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop && queue.empty()) return;
                if (!queue.empty()) {
                    Job *head = queue.front();
                    auto hit = cache.end();
                    if (head->key)
                        for (auto it = cache.begin(); it != cache.end(); ++it)
                            if (it->key == head->key && it->nn == head->nn && it->nc == head->nc &&
                                it->nf == head->nf && it->eliminate == (head->opt.eliminate_frac_faces != 0)) {
                                hit = it;
                                break;
                            }
                    size_t need = head->est;
                    if (hit != cache.end()) {
                        // the cached handle leaves the cache and runs the job
                        reuse = hit->h;
                        need = std::max(hit->bytes, head->est);
                        cached_bytes -= hit->bytes;
                        cache.erase(hit);
                    }
                    if (make_room(need, evicted)) {
                        charged = need;
                        j = head;
                        queue.pop_front();
                        in_use += charged;
                        peak = std::max(peak, in_use + cached_bytes);
                        ++running;
                        j->state = Job::RUNNING;
                        j->charged = charged;
                        j->res.t_start = now();
                        j->res.worker = w;
                        j->res.reused = reuse != nullptr;
                        break;
                    }
                    if (reuse) {  // no room even after eviction: back into the cache
                        cache.push_front(Cached{head->key, head->nn, head->nc, head->nf,
                                                head->opt.eliminate_frac_faces != 0, reuse,
                                                vag_footprint_bytes(reuse)});
                        cached_bytes += cache.front().bytes;
                        reuse = nullptr;
                    }
                }
                cv_work.wait(lk);
            }
        }
        for (vag_handle *e : evicted) vag_destroy(e);
        const Outcome o = run(j, w, reuse);
        if (!o.handed_over) complete(j, o.keep);
    }
}

// Under no lock: the job's charge comes off, its handle goes to the cache
// (or nothing), the job is done.
void vag_server::complete(Job *j, vag_handle *keep) {
    std::vector<vag_handle *> evicted;
    {
        std::lock_guard<std::mutex> lk(mu);
        in_use -= j->charged;
        if (keep) {
            const size_t bytes = vag_footprint_bytes(keep);
            cache.push_front(Cached{j->key, j->nn, j->nc, j->nf, j->opt.eliminate_frac_faces != 0, keep, bytes});
            cached_bytes += bytes;
            make_room(0, evicted);  // the kept handle may have outgrown the estimate
        }
        --running;
        ++finished;
        j->state = Job::DONE;
        j->res.t_end = now();
    }
    cv_done.notify_all();
    cv_work.notify_all();
    for (vag_handle *e : evicted) vag_destroy(e);
}

// The outputs of a job whose work on h is done or queued on s; returns the
// handle to keep, or null (destroyed).
vag_handle *vag_server::finish_outputs(Job *j, vag_handle *h, hipStream_t s) {
    vag_job_result &r = j->res;
    const bool transport = j->n_steps > 0 || j->t_final > 0;
    vag_status st = vag_get_pressure(h, j->out[0], j->out[1], j->out[2], VAG_MEM_HOST);
    if (st == VAG_OK && transport) st = vag_get_concentration(h, j->out[3], j->out[4], j->out[5], VAG_MEM_HOST);
    if (st == VAG_OK) st = hipStreamSynchronize(s) == hipSuccess ? VAG_OK : VAG_ERR_HIP;
    if (st != VAG_OK) {
        r.status = st;
        std::snprintf(r.message, sizeof r.message, "%s", vag_last_error(h));
        vag_destroy(h);
        return nullptr;
    }
    r.ms_run = 1e3 * (now() - r.t_start);
    r.status = j->solve_status;  // VAG_OK or VAG_WARN_NOT_CONVERGED
    if (j->solve_status != VAG_OK) std::snprintf(r.message, sizeof r.message, "%s", vag_last_error(h));
    r.footprint_bytes = vag_footprint_bytes(h);
    if (j->key) return h;
    vag_destroy(h);
    return nullptr;
}

// Runs one job on worker w's stream, on h if given (a cached handle of the
// same mesh) or on a new handle: create (or update), the pressure solve and
// the transport's set-up; then hands the transport steps to the job's lane
// or, without transport, copies the outputs.
vag_server::Outcome vag_server::run(Job *j, int w, vag_handle *h) {
    vag::Phases ph("vag.job");
    hipStream_t s = streams[w];
    vag_job_result &r = j->res;
    vag_mesh mesh{j->nn, j->nc, j->xyz.data(), j->hex8.empty() ? nullptr : j->hex8.data()};
    vag_fractures fr{j->nf, j->fnodes.data(), j->fwidth.data(), j->fperm.data(), j->fporo.data()};
    if (j->hex8.empty()) {
        mesh.n_faces = j->n_faces;
        mesh.cell_face_ptr = j->cell_face_ptr.data();
        mesh.cell_faces = j->cell_faces.data();
        mesh.face_node_ptr = j->face_node_ptr.data();
        mesh.face_nodes = j->face_nodes.data();
        fr.face_nodes = nullptr;
        fr.face_ids = j->face_ids.data();
    }
    vag_rock rock{j->perm.data(), j->poro.data(), j->mu};
    vag_bc bc{j->dir.data(), j->p_bar.data(), j->c_bar.empty() ? nullptr : j->c_bar.data()};
    r.footprint_estimate = j->est;
    auto failed = [&](vag_status st) {
        r.status = st;
        std::snprintf(r.message, sizeof r.message, "%s", vag_last_error(h));
        return st < 0;
    };
    vag_status st;
    if (h) {
        st = vag_set_stream(h, s);
        if (st == VAG_OK) st = vag_set_options(h, &j->opt);
        if (st == VAG_OK)
            st = vag_update(h, &rock, j->nf ? &fr : nullptr, j->p_bar.data(),
                            j->c_bar.empty() ? nullptr : j->c_bar.data(), VAG_MEM_HOST);
        if (failed(st)) {
            vag_destroy(h);
            return {};
        }
    } else {
        const double tc = now();
        st = vag_create(&mesh, j->nf ? &fr : nullptr, &rock, &bc, &j->opt, VAG_MEM_HOST, s, &h);
        r.ms_create = 1e3 * (now() - tc);
        if (st != VAG_OK) {
            r.status = st;
            std::snprintf(r.message, sizeof r.message, "%s", vag_last_error(nullptr));
            return {};
        }
    }
    st = vag_solve_pressure(h, &r.solve);
    if (failed(st)) {
        vag_destroy(h);
        return {};
    }
    j->solve_status = st;
    if ((j->n_steps > 0 || j->t_final > 0) && j->nc + j->nf + j->nn >= kBatchRows) {
        st = vag_transport(h, j->n_steps, j->t_final, nullptr, nullptr, nullptr, VAG_MEM_HOST, &r.transport);
        if (failed(st)) {
            vag_destroy(h);
            return {};
        }
    } else if (j->n_steps > 0 || j->t_final > 0) {
        int64_t N = 0;
        st = vag_serving_transport_begin(h, j->n_steps, j->t_final, &N);
        if (st == VAG_OK && hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess) st = VAG_ERR_HIP;
        if (st == VAG_OK && hipEventRecord(j->ready, s) != hipSuccess) st = VAG_ERR_HIP;
        // the handle moves to its finisher's stream (its work on s ends here)
        if (st == VAG_OK) {
            {
                std::lock_guard<std::mutex> lk(mu);
                j->fin = next_fin;
                next_fin = (next_fin + 1) % kFinishers;
            }
            st = vag_set_stream(h, fin_stream[j->fin]);
        }
        if (failed(st)) {
            if (j->ready) (void)hipEventDestroy(j->ready);
            j->ready = nullptr;
            vag_destroy(h);
            return {};
        }
        j->h = h;
        lane[lane_of(j->nc + j->nf + j->nn)]->submit(j, N);
        Outcome o;
        o.handed_over = true;
        return o;
    }
    Outcome o;
    o.keep = finish_outputs(j, h, s);
    return o;
}

void vag_server::fin_loop(int f) {
    (void)hipSetDevice(device);
    for (;;) {
        std::pair<Job *, bool> item;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_fin.wait(lk, [&] { return fin_stop || !fin_queue[f].empty(); });
            if (fin_queue[f].empty()) return;  // stop
            item = fin_queue[f].front();
            fin_queue[f].pop_front();
        }
        Job *j = item.first;
        vag_handle *h = j->h, *keep = nullptr;
        j->h = nullptr;
        vag_status st = item.second ? VAG_ERR_HIP : vag_serving_transport_end(h, &j->res.transport);
        if (st == VAG_OK) {
            // the last step is done, so the lane's stream is past its wait on j->ready
            (void)hipEventDestroy(j->ready);
            j->ready = nullptr;
            keep = finish_outputs(j, h, fin_stream[f]);
        } else {  // j->ready stays: the lane's stream may still wait on it
            j->res.status = st;
            std::snprintf(j->res.message, sizeof j->res.message, "batched transport steps failed");
            (void)hipDeviceSynchronize();  // steps launched before the failure may still read the handle
            vag_destroy(h);
        }
        complete(j, keep);
    }
}

extern "C" {

vag_status vag_server_create(size_t hbm_budget, int n_workers, vag_server **out) {
    if (!out || n_workers < 1 || n_workers > 16) return VAG_ERR_ARG;
    *out = nullptr;
    std::unique_ptr<vag_server> s;
    try {
        s.reset(new vag_server());
    } catch (...) {
        return VAG_ERR_OOM;
    }
    if (hipGetDevice(&s->device) != hipSuccess) return VAG_ERR_HIP;
    if (hbm_budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return VAG_ERR_HIP;
        hbm_budget = free_b / 10 * 8;
    }
    s->budget = hbm_budget;
    for (int w = 0; w < n_workers; ++w) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            return VAG_ERR_HIP;
        }
        s->streams.push_back(st);
    }
    for (int l = 0; l < vag_server::kLanes; ++l)
        if (hipStreamCreateWithFlags(&s->lane_stream[l], hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            for (int m = 0; m < l; ++m) (void)hipStreamDestroy(s->lane_stream[m]);
            return VAG_ERR_HIP;
        }
    for (int f = 0; f < vag_server::kFinishers; ++f)
        if (hipStreamCreateWithFlags(&s->fin_stream[f], hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            for (auto x : s->lane_stream) (void)hipStreamDestroy(x);
            for (int g = 0; g < f; ++g) (void)hipStreamDestroy(s->fin_stream[g]);
            return VAG_ERR_HIP;
        }
    try {
        vag_server *p = s.get();
        auto to_finisher = [p](Job *j, bool failed) {
            {
                std::lock_guard<std::mutex> lk(p->mu);
                p->fin_queue[j->fin].emplace_back(j, failed);
            }
            p->cv_fin.notify_all();
        };
        for (int f = 0; f < vag_server::kFinishers; ++f) s->fin_thread[f] = std::thread([p, f] { p->fin_loop(f); });
        for (int l = 0; l < vag_server::kLanes; ++l)
            s->lane[l].reset(new StepBatcher(s->device, s->lane_stream[l], to_finisher));
        for (int w = 0; w < n_workers; ++w) s->workers.emplace_back([p = s.get(), w] { p->loop(w); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        for (auto &b : s->lane) b.reset();
        s->stop_finisher();
        for (auto x : s->streams) (void)hipStreamDestroy(x);
        for (auto x : s->lane_stream) (void)hipStreamDestroy(x);
        for (auto x : s->fin_stream) (void)hipStreamDestroy(x);
        return VAG_ERR_OOM;
    }
    *out = s.release();
    return VAG_OK;
}

vag_status vag_server_submit(vag_server *s, const vag_job *job, uint64_t *job_id) {
    if (!s || !job || !job_id || !job->mesh || !job->rock || !job->bc) return VAG_ERR_ARG;
    const vag_mesh *m = job->mesh;
    const int64_t nn = m->n_nodes, nc = m->n_cells, nf = job->frac ? job->frac->n_frac : 0;
    if (nn <= 0 || nc <= 0 || nf < 0 || job->n_steps < 0 || job->t_final < 0) return VAG_ERR_ARG;
    auto j = std::make_unique<Job>();
    try {
        j->nn = nn;
        j->nc = nc;
        j->nf = nf;
        j->xyz = copy_in(m->node_xyz, 3 * (size_t)nn);
        if (m->hex8) {
            j->hex8 = copy_in(m->hex8, 8 * (size_t)nc);
        } else {  // the general form: the two CSR lists (their sizes checked before the copies)
            const int64_t nF = m->n_faces;
            if (nF <= 0 || !m->cell_face_ptr || !m->face_node_ptr) return VAG_ERR_ARG;
            j->n_faces = nF;
            j->cell_face_ptr = copy_in(m->cell_face_ptr, (size_t)nc + 1);
            j->face_node_ptr = copy_in(m->face_node_ptr, (size_t)nF + 1);
            // non-decreasing offsets from 0, so that the lists' lengths are their last entries
            for (int64_t K = 0; K < nc; ++K)
                if (j->cell_face_ptr[K + 1] < j->cell_face_ptr[K]) return VAG_ERR_ARG;
            for (int64_t f = 0; f < nF; ++f)
                if (j->face_node_ptr[f + 1] < j->face_node_ptr[f]) return VAG_ERR_ARG;
            const int64_t ncf = j->cell_face_ptr[nc], nfn = j->face_node_ptr[nF];
            if (j->cell_face_ptr[0] != 0 || j->face_node_ptr[0] != 0) return VAG_ERR_ARG;
            j->cell_faces = copy_in(m->cell_faces, (size_t)ncf);
            j->face_nodes = copy_in(m->face_nodes, (size_t)nfn);
            if (nf) j->face_ids = copy_in(job->frac->face_ids, (size_t)nf);
        }
        if (nf) {
            if (m->hex8) j->fnodes = copy_in(job->frac->face_nodes, 4 * (size_t)nf);
            j->fwidth = copy_in(job->frac->width, (size_t)nf);
            j->fperm = copy_in(job->frac->perm, (size_t)nf);
            j->fporo = copy_in(job->frac->porosity, (size_t)nf);
        }
        j->perm = copy_in(job->rock->perm, 6 * (size_t)nc);
        j->poro = copy_in(job->rock->porosity, (size_t)nc);
        j->mu = job->rock->mu;
        j->dir = copy_in(job->bc->node_dirichlet, (size_t)nn);
        j->p_bar = copy_in(job->bc->p_bar, (size_t)nn);
        if (job->bc->c_bar) j->c_bar = copy_in(job->bc->c_bar, (size_t)nn);
    } catch (const std::invalid_argument &) {
        return VAG_ERR_ARG;
    } catch (...) {
        return VAG_ERR_OOM;
    }
    if (job->opt) j->opt = *job->opt; else vag_default_options(&j->opt);
    j->n_steps = job->n_steps;
    j->t_final = job->t_final;
    j->key = job->mesh_key;
    j->out[0] = job->u_node;
    j->out[1] = job->u_cell;
    j->out[2] = job->u_frac;
    j->out[3] = job->c_cell;
    j->out[4] = job->c_frac;
    j->out[5] = job->c_node;
    {
        vag_mesh em = *m;  // the copies, whose sizes were checked
        if (!m->hex8) {
            em.cell_face_ptr = j->cell_face_ptr.data();
            em.cell_faces = j->cell_faces.data();
            em.face_node_ptr = j->face_node_ptr.data();
            em.face_nodes = j->face_nodes.data();
        }
        j->est = vag_estimate_footprint_mesh(&em, nf, &j->opt);
        if (!j->est) return VAG_ERR_ARG;
    }
    if (j->est > s->budget) return VAG_ERR_OOM;
    j->res.worker = -1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return VAG_ERR_STATE;
        j->id = s->next_id++;
        j->res.t_submit = s->now();
        *job_id = j->id;
        s->queue.push_back(j.get());
        s->jobs.emplace(j->id, std::move(j));
        ++s->submitted;
    }
    s->cv_work.notify_all();
    return VAG_OK;
}

vag_status vag_server_wait(vag_server *s, uint64_t id, double timeout_s, vag_job_result *res) {
    if (!s) return VAG_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return VAG_ERR_ARG;
    Job *j = it->second.get();
    auto done = [&] { return j->state == Job::DONE; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        return VAG_ERR_TIMEOUT;
    }
    if (res) *res = j->res;
    s->jobs.erase(it);
    return VAG_OK;
}

vag_status vag_server_cancel(vag_server *s, uint64_t id) {
    if (!s) return VAG_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(id);
        if (it == s->jobs.end()) return VAG_ERR_ARG;
        Job *j = it->second.get();
        if (j->state != Job::QUEUED) return VAG_ERR_STATE;
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), j));
        j->state = Job::DONE;
        j->res.status = VAG_ERR_CANCELLED;
        std::snprintf(j->res.message, sizeof j->res.message, "cancelled before it started");
        j->res.t_end = s->now();
        ++s->finished;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();  // the next job may now be the head
    return VAG_OK;
}

vag_status vag_server_get_stats(vag_server *s, vag_server_stats *st) {
    if (!s || !st) return VAG_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->submitted;
    st->queued = (int64_t)s->queue.size();
    st->running = s->running;
    st->finished = s->finished;
    st->budget = s->budget;
    st->bytes_in_use = s->in_use;
    st->peak_bytes_in_use = s->peak;
    st->cached_bytes = s->cached_bytes;
    st->cached_handles = (int)s->cache.size();
    st->step_launches = st->job_steps = 0;
    for (auto &b : s->lane) {
        int64_t l = 0, k = 0;
        b->counts(&l, &k);
        st->step_launches += l;
        st->job_steps += k;
    }
    return VAG_OK;
}

double vag_server_clock(vag_server *s) { return s ? s->now() : 0.0; }

void vag_server_destroy(vag_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Job *j : s->queue) {
            j->state = Job::DONE;
            j->res.status = VAG_ERR_CANCELLED;
        }
        s->queue.clear();
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &b : s->lane) b.reset();  // their last jobs go to the finisher
    s->stop_finisher();
    for (auto &c : s->cache) vag_destroy(c.h);
    for (auto x : s->streams) (void)hipStreamDestroy(x);
    for (auto x : s->lane_stream) (void)hipStreamDestroy(x);
    for (auto x : s->fin_stream) (void)hipStreamDestroy(x);
    delete s;
}

}  // extern "C"
