// lh_serve.hip -- continuous-batching server for susceptibility jobs.
//
// Jobs are queued in arrival order.  Worker threads (one per in-flight slot,
// each with its own HIP stream) admit the head of the queue as soon as a slot
// is free and its memory fits the HBM budget, run the hot path and the
// optional RPA epilogue on the worker's stream, and hand the slot back when
// the stream has drained.  Jobs on different workers overlap on the device.
//
// Plans are cached by class (everything that fixes their tables and buffer
// layout).  An admitted job takes an idle plan of its class when there is
// one and rebinds it in place (band, mu, omega list; buffers grow when its
// lag range needs more), so the request path builds no tables, allocates
// nothing in the common case and times no window schedules; only a job of a
// new class plans from scratch.  The budget covers every plan the server
// holds, running or idle: idle plans are freed least recently used first when
// a job needs their memory.  Problems given at creation are planned (and
// their window schedules tuned) before the first job is taken.  A failed job
// reports its own status and does not affect the others.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lh_internal.h"

using namespace lh;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kLatencyWindow = 65536;  // latencies kept for the percentiles

size_t round_up(size_t b) { return (b + 255) & ~(size_t)255; }

struct Job {
    uint64_t id = 0;
    lindhard_problem p{};
    std::vector<double> omega, table, rho, pairw, m2;  // the job's copies (dropped when it ends)
    double U = NAN;
    void *im = nullptr, *re = nullptr, *imr = nullptr, *rer = nullptr;
    std::string key;            // plan class
    std::vector<size_t> sizes;  // buffer sizes its plan needs
    size_t footprint = 0, points = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    lindhard_status status = LINDHARD_OK;
    Clock::time_point t_submit, t_done;
};

struct Cached {
    lindhard_plan_t plan = nullptr;
    size_t bytes = 0;
    uint64_t last_use = 0;
};

// What a worker took from the queue: jobs of one class, each with the cached
// plan it runs on (or none: plan from scratch) and the bytes accounted for it,
// and idle plans that were evicted to make room (freed by the worker outside
// the lock).
struct Taken {
    std::shared_ptr<Job> job;
    lindhard_plan_t plan = nullptr;
    size_t reserved = 0;
};
struct Admit {
    std::vector<Taken> taken;
    std::vector<lindhard_plan_t> drop;
};

constexpr int kMergeMax = 8;  // jobs of one class a worker takes at once

// Bytes a cached plan must grow by to hold a job.
size_t growth(const std::vector<size_t> &cap, const std::vector<size_t> &need)
{
    size_t b = 0;
    for (size_t i = 0; i < need.size() && i < cap.size(); ++i)
        if (round_up(need[i]) > round_up(cap[i])) b += round_up(need[i]) - round_up(cap[i]);
    return b;
}

}  // namespace

struct lindhard_server_s {
    lindhard_serve_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;  // queued, running, or done and not yet reported
    std::unordered_map<std::string, std::vector<Cached>> idle;  // class -> idle plans
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<EvenInst *> desc;  // per worker: descriptors of a grouped launch (kMergeMax)
    uint64_t next_id = 1, use_clock = 0;
    size_t resident = 0, idle_bytes = 0, high_water = 0;  // bytes of all plans held / of the idle ones
    int inflight = 0, n_idle = 0;
    bool stop = false;
    uint64_t submitted = 0, completed = 0, failed = 0, rejected = 0, canceled = 0;
    uint64_t reuses = 0, builds = 0, evictions = 0, merged = 0;
    double points_done = 0.0;
    std::vector<double> lat_ms;  // ring of the last kLatencyWindow latencies
    size_t lat_next = 0;
    Clock::time_point t0;
};

// Remove the least recently used idle plan (caller holds the lock); false if none.
static bool evict_lru(lindhard_server_s *S, std::vector<lindhard_plan_t> &drop)
{
    std::vector<Cached> *best_v = nullptr;
    size_t best_i = 0;
    uint64_t best_t = UINT64_MAX;
    for (auto &kv : S->idle)
        for (size_t i = 0; i < kv.second.size(); ++i)
            if (kv.second[i].last_use < best_t) {
                best_t = kv.second[i].last_use;
                best_v = &kv.second;
                best_i = i;
            }
    if (!best_v) return false;
    const Cached c = (*best_v)[best_i];
    best_v->erase(best_v->begin() + best_i);
    S->resident -= c.bytes;
    S->idle_bytes -= c.bytes;
    S->n_idle -= 1;
    S->evictions += 1;
    drop.push_back(c.plan);
    return true;
}

// Try to admit queued job qi (caller holds the lock); on success it leaves the
// queue and joins a.taken.
static bool admit_job(lindhard_server_s *S, size_t qi, Admit &a)
{
    const std::shared_ptr<Job> h = S->queue[qi];
    const size_t budget = S->cfg.hbm_budget_bytes;
    // the idle plan of the job's class that needs the least growth (the most
    // recently used among equals)
    auto it = S->idle.find(h->key);
    long pick = -1;
    size_t pick_grow = 0;
    if (it != S->idle.end())
        for (size_t i = 0; i < it->second.size(); ++i) {
            const size_t gb = growth(plan_capacity(it->second[i].plan), h->sizes);
            if (pick < 0 || gb < pick_grow || (gb == pick_grow && it->second[i].last_use > it->second[pick].last_use)) {
                pick = (long)i;
                pick_grow = gb;
            }
        }
    // with that plan, the other idle plans may be evicted; from scratch, all
    bool reuse = false;
    if (pick >= 0) {
        const size_t other_idle = S->idle_bytes - it->second[pick].bytes;
        reuse = S->resident - other_idle + pick_grow <= budget;
    }
    if (!reuse && S->resident - S->idle_bytes + h->footprint > budget) return false;
    Taken t;
    t.job = h;
    if (reuse) {
        const Cached c = it->second[pick];
        it->second.erase(it->second.begin() + pick);
        S->idle_bytes -= c.bytes;
        S->n_idle -= 1;
        while (S->resident + pick_grow > budget && evict_lru(S, a.drop)) {
        }
        t.plan = c.plan;
        t.reserved = c.bytes + pick_grow;
        S->resident += pick_grow;
        S->reuses += 1;
    } else {
        while (S->resident + h->footprint > budget && evict_lru(S, a.drop)) {
        }
        t.plan = nullptr;
        t.reserved = h->footprint;
        S->resident += h->footprint;
    }
    S->high_water = std::max(S->high_water, S->resident);
    S->queue.erase(S->queue.begin() + qi);
    h->state = 1;
    S->inflight += 1;
    a.taken.push_back(t);
    return true;
}

// Admit the head of the queue and, behind it, further queued jobs of its
// class that fit (up to kMergeMax in all): they run together, the passes of
// those that can be grouped as one launch each.
static bool try_admit(lindhard_server_s *S, Admit &a)
{
    if (S->queue.empty() || !admit_job(S, 0, a)) return false;
    const std::string &key = a.taken[0].job->key;
    for (size_t qi = 0; qi < S->queue.size() && (int)a.taken.size() < kMergeMax;) {
        if (S->queue[qi]->key != key) {
            ++qi;
            continue;
        }
        if (!admit_job(S, qi, a)) break;
    }
    return true;
}

// Plan (or rebind) one job on stream st; *plan holds the plan afterwards
// (nullptr if planning failed).
static lindhard_status prepare_job(lindhard_server_s *S, Job &j, lindhard_plan_t *plan, hipStream_t st)
{
    lindhard_problem p = j.p;
    p.omega = j.omega.data();
    p.eps_table = j.table.empty() ? nullptr : j.table.data();
    p.rho_table = j.rho.empty() ? nullptr : j.rho.data();
    p.pair_weight = j.pairw.empty() ? nullptr : j.pairw.data();
    p.pair_m2 = j.m2.empty() ? nullptr : j.m2.data();
    lindhard_status s;
    if (*plan) {
        s = plan_rebind(*plan, &p, st);
    } else {
        s = lindhard_plan(&p, plan);
        std::lock_guard<std::mutex> lk(S->mu);
        S->builds += 1;
    }
    // the inputs are no longer needed
    std::vector<double>().swap(j.omega);
    std::vector<double>().swap(j.table);
    std::vector<double>().swap(j.rho);
    std::vector<double>().swap(j.pairw);
    std::vector<double>().swap(j.m2);
    return s;
}

// Plan and run the jobs a worker took: the even-path ones that share a group
// key as one launch per pass, the others one by one; then the RPA epilogues.
static void run_jobs(lindhard_server_s *S, std::vector<Taken> &tk, std::vector<lindhard_status> &st_out,
                     EvenInst *d_desc, hipStream_t st)
{
    const size_t n = tk.size();
    st_out.assign(n, LINDHARD_OK);
    for (size_t i = 0; i < n; ++i) st_out[i] = prepare_job(S, *tk[i].job, &tk[i].plan, st);
    std::vector<std::string> gkey(n);
    for (size_t i = 0; i < n; ++i)
        if (st_out[i] == LINDHARD_OK) gkey[i] = even_group_key(plan_of(tk[i].plan));
    std::vector<bool> done(n, false);
    std::vector<EvenInst> host;
    for (size_t i = 0; i < n; ++i) {
        if (st_out[i] != LINDHARD_OK || done[i] || gkey[i].empty()) continue;
        std::vector<lindhard_plan_t> plans;
        std::vector<void *> outs;
        std::vector<size_t> who;
        for (size_t k = i; k < n; ++k)
            if (st_out[k] == LINDHARD_OK && !done[k] && gkey[k] == gkey[i]) {
                plans.push_back(tk[k].plan);
                outs.push_back(tk[k].job->im);
                who.push_back(k);
            }
        if (plans.size() < 2) continue;
        const hipError_t e = plan_exec_group(plans.data(), (int)plans.size(), outs.data(), d_desc, host, st);
        for (size_t k : who) {
            done[k] = true;
            if (e != hipSuccess) st_out[k] = LINDHARD_EDEVICE;
        }
        // one group per merge: its descriptors are in use until the stream drains
        break;
    }
    for (size_t i = 0; i < n; ++i) {
        Job &j = *tk[i].job;
        if (st_out[i] != LINDHARD_OK) continue;
        if (!done[i]) st_out[i] = lindhard_exec(tk[i].plan, j.im, st);
        if (st_out[i] == LINDHARD_OK && std::isfinite(j.U)) st_out[i] = lindhard_rpa(tk[i].plan, j.U, j.re, j.imr, j.rer, st);
    }
    const bool ok = hipStreamSynchronize(st) == hipSuccess;
    for (size_t i = 0; i < n; ++i)
        if (!ok && st_out[i] == LINDHARD_OK) st_out[i] = LINDHARD_EDEVICE;
}

static void worker_loop(lindhard_server_s *S, int w)
{
    (void)hipSetDevice(S->device);
    hipStream_t st = S->streams[w];
    EvenInst *d_desc = S->desc[w];
    std::vector<lindhard_status> status;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        Admit a;
        S->cv_work.wait(lk, [&] { return (S->stop && S->queue.empty()) || try_admit(S, a); });
        if (a.taken.empty()) return;
        lk.unlock();
        S->cv_work.notify_all();
        for (lindhard_plan_t q : a.drop) lindhard_plan_destroy(q);

        run_jobs(S, a.taken, status, d_desc, st);
        std::vector<size_t> bytes(a.taken.size(), 0);
        for (size_t i = 0; i < a.taken.size(); ++i) {
            lindhard_plan_t plan = a.taken[i].plan;
            if (status[i] == LINDHARD_OK && plan)
                bytes[i] = plan_resident_bytes(plan);
            else if (plan)
                lindhard_plan_destroy(plan);
        }

        lk.lock();
        const Clock::time_point now = Clock::now();
        for (size_t i = 0; i < a.taken.size(); ++i) {
            Job &job = *a.taken[i].job;
            const lindhard_status s = status[i];
            job.t_done = now;
            job.status = s;
            job.state = 2;
            S->inflight -= 1;
            S->resident = S->resident - a.taken[i].reserved + bytes[i];
            if (s == LINDHARD_OK && a.taken[i].plan) {
                S->idle[job.key].push_back({a.taken[i].plan, bytes[i], ++S->use_clock});
                S->idle_bytes += bytes[i];
                S->n_idle += 1;
            }
            if (s == LINDHARD_OK) {
                S->completed += 1;
                S->points_done += (double)job.points;
                const double ms = std::chrono::duration<double, std::milli>(job.t_done - job.t_submit).count();
                if (S->lat_ms.size() < kLatencyWindow)
                    S->lat_ms.push_back(ms);
                else
                    S->lat_ms[S->lat_next] = ms;
                S->lat_next = (S->lat_next + 1) % kLatencyWindow;
            } else {
                S->failed += 1;
            }
        }
        if (a.taken.size() > 1) S->merged += a.taken.size();
        S->high_water = std::max(S->high_water, S->resident);
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

// Describe a problem for the server: its class, the buffer sizes and
// footprint of its plan, its output points.
static lindhard_status describe_job(const lindhard_problem *p, Job &j)
{
    Plan probe;
    const lindhard_status s = plan_describe(p, probe);
    if (s != LINDHARD_OK) return s;
    j.key = plan_class_key(probe);
    for (const BufSpec &b : plan_buffers(probe)) j.sizes.push_back(b.bytes);
    j.footprint = 0;
    for (size_t b : j.sizes) j.footprint += round_up(b);
    j.points = probe.out_elems;
    return LINDHARD_OK;
}

static void destroy_server(lindhard_server_s *S)
{
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &kv : S->idle)
        for (const Cached &c : kv.second) lindhard_plan_destroy(c.plan);
    for (auto &st : S->streams)
        if (st) (void)hipStreamDestroy(st);
    for (EvenInst *d : S->desc)
        if (d) (void)hipFree(d);
    delete S;
}

extern "C" {

lindhard_status lindhard_serve_create(const lindhard_serve_config *cfg, lindhard_server_t *out)
{
    if (!cfg || !out || cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->max_queue < 1 ||
        cfg->hbm_budget_bytes == 0 || cfg->n_warm < 0 || (cfg->n_warm > 0 && !cfg->warm))
        return LINDHARD_EINVAL;
    *out = nullptr;
    lindhard_server_s *S = new (std::nothrow) lindhard_server_s();
    if (!S) return LINDHARD_ENOMEM;
    S->cfg = *cfg;
    S->cfg.warm = nullptr;
    S->cfg.n_warm = 0;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return LINDHARD_EDEVICE;
    }
    S->streams.resize(cfg->max_inflight, nullptr);
    S->desc.resize(cfg->max_inflight, nullptr);
    for (int w = 0; w < cfg->max_inflight; ++w) {
        if (hipStreamCreateWithFlags(&S->streams[w], hipStreamNonBlocking) != hipSuccess ||
            hipMalloc((void **)&S->desc[w], kMergeMax * sizeof(EvenInst)) != hipSuccess) {
            (void)hipGetLastError();
            destroy_server(S);
            return LINDHARD_EDEVICE;
        }
    }
    // warm problems: plan each (which tunes its window schedule) and keep the
    // plan while the budget allows
    for (int i = 0; i < cfg->n_warm; ++i) {
        Job j;
        lindhard_status s = describe_job(&cfg->warm[i], j);
        lindhard_plan_t plan = nullptr;
        if (s == LINDHARD_OK) s = lindhard_plan(&cfg->warm[i], &plan);
        if (s != LINDHARD_OK) {
            destroy_server(S);
            return s;
        }
        S->builds += 1;
        const size_t bytes = plan_resident_bytes(plan);
        if (S->resident + bytes <= cfg->hbm_budget_bytes) {
            S->idle[plan_key(plan)].push_back({plan, bytes, ++S->use_clock});
            S->resident += bytes;
            S->idle_bytes += bytes;
            S->n_idle += 1;
            S->high_water = std::max(S->high_water, S->resident);
        } else {
            lindhard_plan_destroy(plan);
        }
    }
    S->t0 = Clock::now();
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
    lindhard_status s = describe_job(&job->p, *job);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (s != LINDHARD_OK) {
            S->rejected += 1;
            return s;
        }
        if (job->footprint > S->cfg.hbm_budget_bytes) {
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
    if (p->pair_m2)
        job->m2.assign(p->pair_m2, p->pair_m2 + nb * nb * (size_t)p->zones_x * p->nkx * (size_t)p->zones_y * p->nky);
    job->p.omega = nullptr;
    job->p.eps_table = nullptr;
    job->p.rho_table = nullptr;
    job->p.pair_weight = nullptr;
    job->p.pair_m2 = nullptr;
    job->U = U_or_nan;
    job->im = im_chi;
    job->re = re_chi;
    job->imr = im_rpa;
    job->rer = re_rpa;
    job->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return LINDHARD_ESTATE;
        job->id = S->next_id++;
        S->jobs[job->id] = job;
        S->queue.push_back(job);
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
    if (*done) S->jobs.erase(it);
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
    S->jobs.erase(job->id);
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_cancel(lindhard_server_t S, uint64_t ticket)
{
    if (!S) return LINDHARD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return LINDHARD_EINVAL;
    if (it->second->state != 0) return LINDHARD_EBUSY;
    auto q = std::find(S->queue.begin(), S->queue.end(), it->second);
    if (q != S->queue.end()) S->queue.erase(q);
    Job &j = *it->second;
    j.state = 2;
    j.status = LINDHARD_ECANCELED;
    j.t_done = Clock::now();
    std::vector<double>().swap(j.omega);
    std::vector<double>().swap(j.table);
    std::vector<double>().swap(j.rho);
    std::vector<double>().swap(j.pairw);
    std::vector<double>().swap(j.m2);
    S->canceled += 1;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_stats_get(lindhard_server_t S, lindhard_serve_stats *o)
{
    if (!S || !o) return LINDHARD_EINVAL;
    std::vector<double> v;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        *o = lindhard_serve_stats{};
        o->submitted = S->submitted;
        o->completed = S->completed;
        o->failed = S->failed;
        o->rejected = S->rejected;
        o->canceled = S->canceled;
        const double wall = std::chrono::duration<double>(Clock::now() - S->t0).count();
        o->points_per_s = wall > 0 ? S->points_done / wall : 0.0;
        o->hbm_high_water = S->high_water;
        o->queue_depth = (int32_t)S->queue.size();
        o->inflight = S->inflight;
        o->plan_reuses = S->reuses;
        o->plan_builds = S->builds;
        o->plan_evictions = S->evictions;
        o->cached_plans = S->n_idle;
        o->resident_bytes = S->resident;
        o->merged_jobs = S->merged;
        v = S->lat_ms;
    }
    if (!v.empty()) {
        auto pct = [&](double f) {
            const size_t i = std::min(v.size() - 1, (size_t)std::ceil(f * v.size()) - 1);
            std::nth_element(v.begin(), v.begin() + i, v.end());
            return v[i];
        };
        o->p50_ms = pct(0.50);
        o->p99_ms = pct(0.99);
    }
    return LINDHARD_OK;
}

lindhard_status lindhard_serve_destroy(lindhard_server_t S)
{
    if (!S) return LINDHARD_EINVAL;
    destroy_server(S);
    return LINDHARD_OK;
}

}  // extern "C"
