// Request loop: admits time-evolution jobs by HBM footprint into a fixed
// number of slots; each slot is a worker thread with its own HIP stream, so
// admitted jobs keep their tensors on the device and run concurrently.  A
// job that finishes frees its slot and memory at once and the next queued
// job that fits is admitted (queue order, skipping jobs that do not fit yet).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ipeps.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
    ipeps_job spec;
    size_t footprint = 0;
    int status = IPEPS_JOB_QUEUED;
    std::vector<ipeps_obs> series;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct ipeps_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, Job> jobs;
    std::deque<uint64_t> pending;
    uint64_t next_id = 1;
    size_t budget = 0, used = 0;
    int running = 0;
    bool stopping = false;
    int device = 0;
    std::vector<std::thread> workers;
};

namespace {

int run_job(ipeps_server* srv, Job& job, hipStream_t stream, std::vector<ipeps_obs>* series) {
    (void)srv;
    ipeps_state* st = nullptr;
    int rc = ipeps_init(&job.spec.cfg, stream, nullptr, nullptr, nullptr, &st);
    if (rc != IPEPS_OK) return rc;
    const int every = job.spec.observe_every > 0 ? job.spec.observe_every : job.spec.n_steps;
    int done = 0, nobs = 0;
    while (rc == IPEPS_OK && done < job.spec.n_steps) {
        int chunk = every;
        if (done + chunk > job.spec.n_steps) chunk = job.spec.n_steps - done;
        rc = ipeps_trotter_step(st, chunk, nullptr);
        if (rc != IPEPS_OK) break;
        done += chunk;
        int it = 0;
        double dl = 0;
        rc = ctmrg_converge(st, 0.0, job.spec.ctm_iters > 0 ? job.spec.ctm_iters : 10, nobs == 0, &it, &dl);
        if (rc != IPEPS_OK) break;
        ipeps_obs o;
        rc = ipeps_observe(st, &o);
        if (rc != IPEPS_OK) break;
        series->push_back(o);
        ++nobs;
    }
    ipeps_destroy(st);
    return rc;
}

void worker_main(ipeps_server* srv) {
    (void)hipSetDevice(srv->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    for (;;) {
        uint64_t id = 0;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            for (;;) {
                for (auto it = srv->pending.begin(); it != srv->pending.end(); ++it) {
                    Job& j = srv->jobs[*it];
                    if (srv->used + j.footprint <= srv->budget) {
                        id = *it;
                        srv->pending.erase(it);
                        break;
                    }
                }
                if (id) break;
                if (srv->stopping && srv->pending.empty()) {
                    if (stream) (void)hipStreamDestroy(stream);
                    return;
                }
                srv->cv_work.wait(lk);
            }
            Job& j = srv->jobs[id];
            srv->used += j.footprint;
            srv->running++;
            j.status = IPEPS_JOB_RUNNING;
            j.t_admit = now_s();
        }
        std::vector<ipeps_obs> series;
        Job copy;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            copy = srv->jobs[id];
        }
        const int rc = run_job(srv, copy, stream, &series);
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            Job& j = srv->jobs[id];
            j.series = std::move(series);
            j.status = (rc == IPEPS_OK) ? IPEPS_JOB_DONE : rc;
            j.t_done = now_s();
            srv->used -= j.footprint;
            srv->running--;
        }
        srv->cv_work.notify_all();
        srv->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

int solve_server_create(size_t hbm_budget, int max_slots, ipeps_server** out) {
    if (!out || max_slots < 1 || max_slots > 64) return IPEPS_EINVAL;
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return IPEPS_EDEVICE;
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return IPEPS_EDEVICE;
        hbm_budget = (size_t)(0.9 * (double)fr);
    }
    ipeps_server* srv = new ipeps_server();
    srv->budget = hbm_budget;
    srv->device = dev;
    for (int i = 0; i < max_slots; ++i) srv->workers.emplace_back(worker_main, srv);
    *out = srv;
    return IPEPS_OK;
}

int solve_submit(ipeps_server* srv, const ipeps_job* job, uint64_t* job_id) {
    if (!srv || !job || !job_id) return IPEPS_EINVAL;
    if (job->n_steps < 1 || job->observe_every < 0 || job->ctm_iters < 0) return IPEPS_EINVAL;
    const size_t fp = ipeps_footprint_bytes(&job->cfg);
    if (fp == 0) return IPEPS_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (fp > srv->budget || srv->stopping) return IPEPS_EINVAL;
    const uint64_t id = srv->next_id++;
    Job& j = srv->jobs[id];
    j.spec = *job;
    j.footprint = fp;
    j.t_submit = now_s();
    srv->pending.push_back(id);
    *job_id = id;
    srv->cv_work.notify_one();
    return IPEPS_OK;
}

int solve_poll(ipeps_server* srv, uint64_t job_id, int* status, ipeps_obs* series, int cap, int* n_out) {
    if (!srv) return IPEPS_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job_id);
    if (it == srv->jobs.end()) return IPEPS_ENOTFOUND;
    const Job& j = it->second;
    if (status) *status = j.status;
    if (j.status == IPEPS_JOB_QUEUED || j.status == IPEPS_JOB_RUNNING) return IPEPS_EAGAIN;
    if (j.status < 0) return j.status;
    const int n = (int)j.series.size();
    if (n_out) *n_out = n;
    if (series && cap > 0) std::memcpy(series, j.series.data(), sizeof(ipeps_obs) * (size_t)std::min(cap, n));
    return IPEPS_OK;
}

int solve_job_times(ipeps_server* srv, uint64_t job_id, double* t_submit, double* t_admit, double* t_done) {
    if (!srv) return IPEPS_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job_id);
    if (it == srv->jobs.end()) return IPEPS_ENOTFOUND;
    const Job& j = it->second;
    if (t_submit) *t_submit = j.t_submit;
    if (t_admit) *t_admit = j.t_admit;
    if (t_done) *t_done = j.t_done;
    if (j.status == IPEPS_JOB_QUEUED || j.status == IPEPS_JOB_RUNNING) return IPEPS_EAGAIN;
    return j.status < 0 ? j.status : IPEPS_OK;
}

void solve_server_destroy(ipeps_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (auto& t : srv->workers) t.join();
    delete srv;
}

}  // extern "C"
