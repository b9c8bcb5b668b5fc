// Serving loop: continuous batching of independent Darcy + transport jobs.
//
// One FIFO queue, n worker threads, one HIP stream per worker.  A worker
// takes the head job when its estimated device footprint fits in the budget
// left by the running jobs and the cached handles (idle cached handles are
// evicted, least recently used first, to make room).  Each job runs on a
// handle of its own (vag_create .. vag_transport, outputs copied to the
// caller's host buffers), so jobs on different workers overlap on the device
// while each job's kernels, and therefore its results, are those of the job
// run alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "vag.h"

namespace {

struct Job {
    uint64_t id = 0;
    // owned copies of the inputs
    int64_t nn = 0, nc = 0, nf = 0;
    std::vector<double> xyz, fwidth, fperm, fporo, perm, poro, p_bar, c_bar;
    std::vector<int32_t> hex8, fnodes;
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

}  // namespace

struct vag_server {
    int device = 0;
    size_t budget = 0;
    std::vector<hipStream_t> streams;
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

    vag_handle *run(Job *j, int w, vag_handle *h);
    void loop(int w);
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
        evicted.clear();
        vag_handle *keep = run(j, w, reuse);
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= charged;
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
}

// Runs one job on worker w's stream, on h if given (a cached handle of the
// same mesh) or on a new handle.  Returns the handle to cache, or null.
vag_handle *vag_server::run(Job *j, int w, vag_handle *h) {
    hipStream_t s = streams[w];
    vag_job_result &r = j->res;
    vag_mesh mesh{j->nn, j->nc, j->xyz.data(), j->hex8.data()};
    vag_fractures fr{j->nf, j->fnodes.data(), j->fwidth.data(), j->fperm.data(), j->fporo.data()};
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
            return nullptr;
        }
    } else {
        const double tc = now();
        st = vag_create(&mesh, j->nf ? &fr : nullptr, &rock, &bc, &j->opt, VAG_MEM_HOST, s, &h);
        r.ms_create = 1e3 * (now() - tc);
        if (st != VAG_OK) {
            r.status = st;
            std::snprintf(r.message, sizeof r.message, "%s", vag_last_error(nullptr));
            return nullptr;
        }
    }
    st = vag_solve_pressure(h, &r.solve);
    if (failed(st)) {
        vag_destroy(h);
        return nullptr;
    }
    const vag_status solve_status = st;
    if (j->n_steps > 0 || j->t_final > 0) {
        st = vag_transport(h, j->n_steps, j->t_final, nullptr, nullptr, nullptr, VAG_MEM_HOST, &r.transport);
        if (failed(st)) {
            vag_destroy(h);
            return nullptr;
        }
    }
    st = vag_get_pressure(h, j->out[0], j->out[1], j->out[2], VAG_MEM_HOST);
    if (st == VAG_OK && (j->n_steps > 0 || j->t_final > 0))
        st = vag_get_concentration(h, j->out[3], j->out[4], j->out[5], VAG_MEM_HOST);
    if (st == VAG_OK) st = hipStreamSynchronize(s) == hipSuccess ? VAG_OK : VAG_ERR_HIP;
    if (failed(st)) {
        vag_destroy(h);
        return nullptr;
    }
    r.ms_run = 1e3 * (now() - r.t_start);
    r.status = solve_status;  // VAG_OK or VAG_WARN_NOT_CONVERGED
    if (solve_status != VAG_OK) std::snprintf(r.message, sizeof r.message, "%s", vag_last_error(h));
    r.footprint_bytes = vag_footprint_bytes(h);
    if (j->key) return h;
    vag_destroy(h);
    return nullptr;
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
    try {
        for (int w = 0; w < n_workers; ++w) s->workers.emplace_back([p = s.get(), w] { p->loop(w); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        for (auto x : s->streams) (void)hipStreamDestroy(x);
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
    if (!m->hex8) return VAG_ERR_UNSUPPORTED;  // jobs take hex8 meshes
    auto j = std::make_unique<Job>();
    try {
        j->nn = nn;
        j->nc = nc;
        j->nf = nf;
        j->xyz = copy_in(m->node_xyz, 3 * (size_t)nn);
        j->hex8 = copy_in(m->hex8, 8 * (size_t)nc);
        if (nf) {
            j->fnodes = copy_in(job->frac->face_nodes, 4 * (size_t)nf);
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
    j->est = vag_estimate_footprint(nn, nc, nf, &j->opt);
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
    for (auto &c : s->cache) vag_destroy(c.h);
    for (auto x : s->streams) (void)hipStreamDestroy(x);
    delete s;
}

}  // extern "C"
