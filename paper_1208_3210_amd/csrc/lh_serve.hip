// lh_serve.hip -- continuous-batching server for susceptibility jobs.
//
// Jobs are queued in arrival order.  Worker threads (one per in-flight slot,
// each with its own HIP stream) admit the head of the queue as soon as a slot
// is free and the sum of the admitted jobs' device footprints stays within the
// HBM budget; admitted jobs build their plan (band, mu, tables, workspace kept
// resident on the device for the job's lifetime), run the hot path and the
// optional RPA epilogue on the worker's stream, and release the slot and the
// memory when the stream has drained.  Jobs on different workers overlap on
// the device.  A failed job reports its own status and does not affect others.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lh_internal.h"

using namespace lh;

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t id = 0;
    lindhard_problem p{};
    std::vector<double> omega, table, rho, pairw;
    double U = NAN;
    void *im = nullptr, *re = nullptr, *imr = nullptr, *rer = nullptr;
    size_t footprint = 0, points = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    lindhard_status status = LINDHARD_OK;
    Clock::time_point t_submit, t_done;
};

}  // namespace

struct lindhard_server_s {
    lindhard_serve_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    uint64_t next_id = 1;
    size_t inflight_bytes = 0, high_water = 0;
    int inflight = 0;
    bool stop = false;
    uint64_t submitted = 0, completed = 0, failed = 0, rejected = 0, canceled = 0;
    double points_done = 0.0;
    std::vector<double> lat_ms;
    Clock::time_point t0;
};

static lindhard_status run_job(Job &j, hipStream_t st)
{
    lindhard_problem p = j.p;
    p.omega = j.omega.data();
    p.eps_table = j.table.empty() ? nullptr : j.table.data();
    p.rho_table = j.rho.empty() ? nullptr : j.rho.data();
    p.pair_weight = j.pairw.empty() ? nullptr : j.pairw.data();
    lindhard_plan_t plan = nullptr;
    lindhard_status s = lindhard_plan(&p, &plan);
    if (s != LINDHARD_OK) return s;
    s = lindhard_exec(plan, j.im, st);
    if (s == LINDHARD_OK && std::isfinite(j.U)) s = lindhard_rpa(plan, j.U, j.re, j.imr, j.rer, st);
    if (hipStreamSynchronize(st) != hipSuccess && s == LINDHARD_OK) s = LINDHARD_EDEVICE;
    lindhard_plan_destroy(plan);
    return s;
}

static void worker_loop(lindhard_server_s *S, int w)
{
    (void)hipSetDevice(S->device);
    hipStream_t st = S->streams[w];
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // admit the head of the queue when it fits the budget
        S->cv_work.wait(lk, [&] {
            if (S->queue.empty()) return S->stop;
            auto &h = S->jobs[S->queue.front()];
            return S->inflight_bytes + h->footprint <= S->cfg.hbm_budget_bytes;
        });
        if (S->queue.empty() && S->stop) return;
        std::shared_ptr<Job> job = S->jobs[S->queue.front()];
        S->queue.pop_front();
        job->state = 1;
        S->inflight_bytes += job->footprint;
        S->inflight += 1;
        S->high_water = std::max(S->high_water, S->inflight_bytes);
        lk.unlock();
        S->cv_work.notify_all();

        lindhard_status s = run_job(*job, st);

        lk.lock();
        job->t_done = Clock::now();
        job->status = s;
        job->state = 2;
        S->inflight_bytes -= job->footprint;
        S->inflight -= 1;
        if (s == LINDHARD_OK) {
            S->completed += 1;
            S->points_done += (double)job->points;
            S->lat_ms.push_back(std::chrono::duration<double, std::milli>(job->t_done - job->t_submit).count());
        } else {
            S->failed += 1;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

extern "C" {

lindhard_status lindhard_serve_create(const lindhard_serve_config *cfg, lindhard_server_t *out)
{
    if (!cfg || !out || cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->max_queue < 1 ||
        cfg->hbm_budget_bytes == 0)
        return LINDHARD_EINVAL;
    *out = nullptr;
    lindhard_server_s *S = new (std::nothrow) lindhard_server_s();
    if (!S) return LINDHARD_ENOMEM;
    S->cfg = *cfg;
    S->t0 = Clock::now();
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return LINDHARD_EDEVICE;
    }
    S->streams.resize(cfg->max_inflight, nullptr);
    for (auto &st : S->streams) {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto &s2 : S->streams)
                if (s2) (void)hipStreamDestroy(s2);
            delete S;
            return LINDHARD_EDEVICE;
        }
    }
    for (int w = 0; w < cfg->max_inflight; ++w) S->workers.emplace_back(worker_loop, S, w);
    *out = S;
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_submit(lindhard_server_t S, const lindhard_problem *p, double U_or_nan, void *im_chi,
                                      void *re_chi, void *im_rpa, void *re_rpa, uint64_t *ticket)
{
    if (!S || !p || !im_chi || !ticket) return LINDHARD_EINVAL;
    auto job = std::make_shared<Job>();
    job->p = *p;
    job->p.want_rpa = std::isfinite(U_or_nan) ? 1 : p->want_rpa;
    Plan probe;
    lindhard_status s = plan_describe(&job->p, probe);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (s != LINDHARD_OK) {
            S->rejected += 1;
            return s;
        }
        if (probe.ws_bytes > S->cfg.hbm_budget_bytes) {
            S->rejected += 1;
            return LINDHARD_ETOOBIG;
        }
        if ((int)S->queue.size() >= S->cfg.max_queue) {
            S->rejected += 1;
            return LINDHARD_EBUSY;
        }
    }
    job->omega.assign(p->omega, p->omega + p->nomega);
    const size_t nb = (size_t)(p->n_bands > 1 ? p->n_bands : 1);
    const size_t nall = (size_t)p->nkx * p->nky * (size_t)(p->nkz > 1 ? p->nkz : 1) * nb;
    if (p->eps_table) job->table.assign(p->eps_table, p->eps_table + nall);
    if (p->rho_table) job->rho.assign(p->rho_table, p->rho_table + nall);
    if (p->pair_weight) job->pairw.assign(p->pair_weight, p->pair_weight + nb * nb);
    job->p.omega = nullptr;
    job->p.eps_table = nullptr;
    job->p.rho_table = nullptr;
    job->p.pair_weight = nullptr;
    job->U = U_or_nan;
    job->im = im_chi;
    job->re = re_chi;
    job->imr = im_rpa;
    job->rer = re_rpa;
    job->footprint = probe.ws_bytes;
    job->points = probe.out_elems;
    job->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return LINDHARD_ESTATE;
        job->id = S->next_id++;
        S->jobs[job->id] = job;
        S->queue.push_back(job->id);
        S->submitted += 1;
        *ticket = job->id;
    }
    S->cv_work.notify_all();
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_poll(lindhard_server_t S, uint64_t ticket, int32_t *done, lindhard_status *job_status)
{
    if (!S || !done) return LINDHARD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return LINDHARD_EINVAL;
    *done = it->second->state == 2;
    if (job_status) *job_status = it->second->status;
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_wait(lindhard_server_t S, uint64_t ticket, double timeout_s, lindhard_status *job_status)
{
    if (!S) return LINDHARD_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return LINDHARD_EINVAL;
    std::shared_ptr<Job> job = it->second;
    auto pred = [&] { return job->state == 2; };
    if (timeout_s < 0) {
        S->cv_done.wait(lk, pred);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        return LINDHARD_EBUSY;
    }
    if (job_status) *job_status = job->status;
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_cancel(lindhard_server_t S, uint64_t ticket)
{
    if (!S) return LINDHARD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return LINDHARD_EINVAL;
    if (it->second->state != 0) return LINDHARD_EBUSY;
    auto q = std::find(S->queue.begin(), S->queue.end(), ticket);
    if (q != S->queue.end()) S->queue.erase(q);
    it->second->state = 2;
    it->second->status = LINDHARD_ECANCELED;
    it->second->t_done = Clock::now();
    S->canceled += 1;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_stats_get(lindhard_server_t S, lindhard_serve_stats *o)
{
    if (!S || !o) return LINDHARD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *o = lindhard_serve_stats{};
    o->submitted = S->submitted;
    o->completed = S->completed;
    o->failed = S->failed;
    o->rejected = S->rejected;
    o->canceled = S->canceled;
    if (!S->lat_ms.empty()) {
        std::vector<double> v = S->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double f) {
            size_t i = (size_t)std::ceil(f * v.size()) - 1;
            return v[std::min(i, v.size() - 1)];
        };
        o->p50_ms = pct(0.50);
        o->p99_ms = pct(0.99);
    }
    const double wall = std::chrono::duration<double>(Clock::now() - S->t0).count();
    o->points_per_s = wall > 0 ? S->points_done / wall : 0.0;
    o->hbm_high_water = S->high_water;
    o->queue_depth = (int32_t)S->queue.size();
    o->inflight = S->inflight;
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_destroy(lindhard_server_t S)
{
    if (!S) return LINDHARD_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &st : S->streams)
        if (st) (void)hipStreamDestroy(st);
    delete S;
    return LINDHARD_OK;
}

}  // extern "C"
