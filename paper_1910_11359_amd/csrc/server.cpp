// Request loop with continuous batching.  Jobs are admitted by HBM footprint
// into slabs (one device allocation per layout: D, chi, d_A, precision,
// flags), where each keeps its state resident.  One executor thread advances
// the resident jobs from observation to observation: the idle jobs of one
// slab that are at the same point of their schedule (first observation or
// later, the same number of Trotter steps to the next observation, the same
// CTMRG iteration count) go as one lockstep batch, every kernel launch
// carrying all of them, and batches run side by side on the GPU (each slab
// its own streams) without waiting for each other: a batch that completes
// hands its jobs back at once, a job that finishes frees its slot, a slab
// with no job left returns its memory, and jobs that arrived meanwhile are
// admitted (queue order, skipping jobs that do not fit yet) and batched with
// the idle jobs of their slab.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/ipeps.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Bucket;

struct Job {
    ipeps_job spec;
    size_t footprint = 0;  // one slab region of its layout
    int status = IPEPS_JOB_QUEUED;
    std::vector<ipeps_obs> series;
    double t_submit = 0, t_admit = 0, t_done = 0;
    // resident part (executor thread only)
    ipeps_state* st = nullptr;
    Bucket* bucket = nullptr;
    int slot = -1;
    int done = 0;  // Trotter steps taken
    int nobs = 0;  // observations made
    bool busy = false;  // in a batch that has not completed yet
};

bool same_layout(const ipeps_config& a, const ipeps_config& b) {
    return a.D == b.D && a.chi == b.chi && a.d_A == b.d_A && a.dtype == b.dtype && a.flags == b.flags;
}

struct Bucket {
    ipeps_config layout;
    ipeps_slab* slab = nullptr;
    size_t bytes = 0;  // cap regions
    std::vector<uint64_t> slot_job;  // 0: free
    hipStream_t stream = nullptr;    // the stream of its states
    // the batch of the group that last completed with every job still
    // running, kept (with its captured graph) for the same group's next chunk
    ipeps_batch* kept = nullptr;
    std::vector<uint64_t> kept_ids;
    void drop_kept() {
        if (kept) ipeps_batch_destroy(kept);
        kept = nullptr;
        kept_ids.clear();
    }
    int used() const {
        int u = 0;
        for (uint64_t j : slot_job) u += j != 0;
        return u;
    }
};

}  // namespace

struct ipeps_server {
    std::mutex mu;
    std::condition_variable cv_work;
    std::map<uint64_t, Job> jobs;
    std::deque<uint64_t> pending;
    uint64_t next_id = 1;
    size_t budget = 0, used = 0;
    int max_slots = 1;
    int running = 0;
    bool stopping = false;
    std::atomic<bool> graphs{false};  // batches replay captured warm iterations
    int device = 0;
    std::vector<std::unique_ptr<Bucket>> buckets;  // executor thread only
    std::thread executor;
};

namespace {

// Admission (executor thread, server lock held): queued jobs in order, each
// into a free slot of a slab of its layout, or into a new slab sized for the
// queued jobs of that layout, as far as the budget and max_slots allow.
void admit(ipeps_server* srv, std::vector<uint64_t>& admitted) {
    for (auto it = srv->pending.begin(); it != srv->pending.end();) {
        if (srv->running >= srv->max_slots) break;
        Job& j = srv->jobs[*it];
        Bucket* bk = nullptr;
        int slot = -1;
        for (auto& b : srv->buckets) {
            if (!same_layout(b->layout, j.spec.cfg)) continue;
            for (size_t s = 0; s < b->slot_job.size(); ++s)
                if (!b->slot_job[s]) {
                    bk = b.get();
                    slot = (int)s;
                    break;
                }
            if (bk) break;
        }
        if (!bk) {
            const size_t region = j.footprint;
            int want = 0;
            for (uint64_t id : srv->pending) want += same_layout(srv->jobs[id].spec.cfg, j.spec.cfg);
            want = std::min(want, srv->max_slots - srv->running);
            const int fit = (int)((srv->budget - srv->used) / region);
            const int cap = std::min(want, fit);
            if (cap >= 1) {
                ipeps_slab* slab = nullptr;
                if (ipeps_slab_create(&j.spec.cfg, cap, &slab) == IPEPS_OK) {
                    auto b = std::make_unique<Bucket>();
                    b->layout = j.spec.cfg;
                    b->slab = slab;
                    b->bytes = region * cap;
                    b->slot_job.assign(cap, 0);
                    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) b->stream = nullptr;
                    srv->used += b->bytes;
                    bk = b.get();
                    slot = 0;
                    srv->buckets.push_back(std::move(b));
                }
            }
        }
        if (!bk) {  // does not fit yet: later jobs may
            ++it;
            continue;
        }
        bk->slot_job[slot] = *it;
        j.bucket = bk;
        j.slot = slot;
        j.status = IPEPS_JOB_RUNNING;
        j.t_admit = now_s();
        srv->running++;
        admitted.push_back(*it);
        it = srv->pending.erase(it);
    }
}

void finish(ipeps_server* srv, Job& j, uint64_t id, int rc) {
    if (j.st) ipeps_destroy(j.st);  // frees the slab region
    j.st = nullptr;
    std::lock_guard<std::mutex> lk(srv->mu);
    j.bucket->slot_job[j.slot] = 0;
    j.status = rc == IPEPS_OK ? IPEPS_JOB_DONE : rc;
    j.t_done = now_s();
    srv->running--;
    (void)id;
}

// A group: idle resident jobs of one slab at the same point of their
// schedules (first observation or later, the same number of Trotter steps
// to the next observation, the same CTMRG iteration count), advanced to
// their next observation as one lockstep batch.
struct Group {
    Bucket* bucket;
    bool cold;
    int chunk, iters;
    std::vector<uint64_t> ids;
    ipeps_batch* batch = nullptr;
    int rc = IPEPS_OK;
};

// Collect a finished group's readouts into its jobs' series.  The batch is
// kept in its bucket when every job goes on (the next chunk of the same
// group reuses it), else destroyed before any of its states is.
void complete(ipeps_server* srv, Group& g) {
    std::vector<ipeps_obs> obs(g.ids.size());
    std::vector<int> status(g.ids.size(), g.rc);
    if (g.rc == IPEPS_OK) {
        const int rc = ipeps_batch_observe_result(g.batch, obs.data(), status.data());
        // a NaN in one job poisons only that job; other failures hit all
        if (rc != IPEPS_OK && rc != IPEPS_ENUMERIC) status.assign(g.ids.size(), rc);
    }
    bool keep = g.batch != nullptr;
    for (size_t i = 0; i < g.ids.size(); ++i) {
        const Job& j = srv->jobs[g.ids[i]];
        keep = keep && status[i] == IPEPS_OK && j.done + g.chunk < j.spec.n_steps;
    }
    if (keep) {
        g.bucket->drop_kept();
        g.bucket->kept = g.batch;
        g.bucket->kept_ids = g.ids;
    } else if (g.batch) {
        ipeps_batch_destroy(g.batch);
    }
    g.batch = nullptr;
    for (size_t i = 0; i < g.ids.size(); ++i) {
        const uint64_t id = g.ids[i];
        Job& j = srv->jobs[id];
        j.busy = false;
        const int rc = status[i];
        if (rc != IPEPS_OK) {
            finish(srv, j, id, rc);
            continue;
        }
        j.done += g.chunk;
        j.nobs++;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            j.series.push_back(obs[i]);
        }
        if (j.done >= j.spec.n_steps) finish(srv, j, id, IPEPS_OK);
    }
}

void executor_main(ipeps_server* srv) {
    (void)hipSetDevice(srv->device);
    std::vector<Group> active;
    for (;;) {
        bool progress = false;
        // groups whose readout has completed
        for (auto it = active.begin(); it != active.end();) {
            const int q = it->rc == IPEPS_OK ? ipeps_batch_query(it->batch) : 1;
            if (q == 0) {
                ++it;
                continue;
            }
            if (q < 0) it->rc = q;
            complete(srv, *it);
            it = active.erase(it);
            progress = true;
        }
        std::vector<uint64_t> admitted, idle;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            for (;;) {
                // a slab with no job left returns its memory (its jobs' work
                // has completed: each job's batches were waited for)
                for (auto it = srv->buckets.begin(); it != srv->buckets.end();) {
                    if ((*it)->used() == 0) {
                        (*it)->drop_kept();
                        srv->used -= (*it)->bytes;
                        ipeps_slab_destroy((*it)->slab);
                        if ((*it)->stream) (void)hipStreamDestroy((*it)->stream);
                        it = srv->buckets.erase(it);
                    } else {
                        ++it;
                    }
                }
                admit(srv, admitted);
                if (srv->running > 0 || !active.empty()) break;
                if (srv->stopping && srv->pending.empty()) return;
                if (!srv->pending.empty() && srv->buckets.empty()) {
                    // the first queued job does not fit even alone: fail it
                    Job& j = srv->jobs[srv->pending.front()];
                    j.status = IPEPS_ENOMEM;
                    j.t_done = now_s();
                    srv->pending.pop_front();
                    continue;
                }
                srv->cv_work.wait(lk);
            }
            for (auto& kv : srv->jobs)
                if (kv.second.status == IPEPS_JOB_RUNNING && !kv.second.busy) idle.push_back(kv.first);
        }
        // states of the newly admitted jobs
        for (uint64_t id : admitted) {
            Job& j = srv->jobs[id];
            const int rc = ipeps_slab_init(j.bucket->slab, j.slot, &j.spec.cfg, j.bucket->stream, &j.st);
            if (rc != IPEPS_OK) {
                j.st = nullptr;
                finish(srv, j, id, rc);
            }
        }
        // idle jobs into groups, each launched as a batch (slabs on their own streams)
        std::vector<Group> fresh;
        for (uint64_t id : idle) {
            Job& j = srv->jobs[id];
            if (!j.st || j.status != IPEPS_JOB_RUNNING) continue;
            const int every = j.spec.observe_every > 0 ? j.spec.observe_every : j.spec.n_steps;
            const int chunk = std::min(every, j.spec.n_steps - j.done);
            const int iters = j.spec.ctm_iters > 0 ? j.spec.ctm_iters : 10;
            const bool cold = j.nobs == 0;
            Group* g = nullptr;
            for (auto& gg : fresh)
                if (gg.bucket == j.bucket && gg.cold == cold && gg.chunk == chunk && gg.iters == iters) g = &gg;
            if (!g) {
                fresh.push_back(Group{j.bucket, cold, chunk, iters, {}, nullptr, IPEPS_OK});
                g = &fresh.back();
            }
            g->ids.push_back(id);
        }
        for (auto& g : fresh) {
            std::vector<ipeps_state*> sts;
            for (uint64_t id : g.ids) {
                sts.push_back(srv->jobs[id].st);
                srv->jobs[id].busy = true;
            }
            Bucket* bk = g.bucket;
            if (bk->kept && bk->kept_ids == g.ids) {  // the same jobs as last time
                g.batch = bk->kept;
                bk->kept = nullptr;
                bk->kept_ids.clear();
            } else {
                // its jobs are idle; some may be in this group
                bk->drop_kept();
                g.rc = ipeps_batch_create(sts.data(), (int)sts.size(), &g.batch);
                if (g.rc == IPEPS_OK && srv->graphs.load()) g.rc = ipeps_batch_set_graph(g.batch, 1);
            }
            if (g.rc == IPEPS_OK) g.rc = ipeps_batch_trotter_step(g.batch, g.chunk);
            if (g.rc == IPEPS_OK) g.rc = ipeps_batch_ctmrg(g.batch, g.iters, g.cold ? 1 : 0);
            if (g.rc == IPEPS_OK) g.rc = ipeps_batch_observe_async(g.batch);
            active.push_back(std::move(g));
            progress = true;
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

}  // namespace

extern "C" {

int solve_server_create(size_t hbm_budget, int max_slots, ipeps_server** out) {
    if (!out || max_slots < 1 || max_slots > 256) return IPEPS_EINVAL;
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
    srv->max_slots = max_slots;
    srv->executor = std::thread(executor_main, srv);
    *out = srv;
    return IPEPS_OK;
}

int solve_submit(ipeps_server* srv, const ipeps_job* job, uint64_t* job_id) {
    if (!srv || !job || !job_id) return IPEPS_EINVAL;
    if (job->n_steps < 1 || job->observe_every < 0 || job->ctm_iters < 0) return IPEPS_EINVAL;
    if (ipeps_footprint_bytes(&job->cfg) == 0) return IPEPS_EINVAL;
    const size_t fp = ipeps_slab_region_bytes(&job->cfg);
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

int solve_server_set_graphs(ipeps_server* srv, int enable) {
    if (!srv) return IPEPS_EINVAL;
    srv->graphs.store(enable != 0);
    return IPEPS_OK;
}

void solve_server_destroy(ipeps_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    if (srv->executor.joinable()) srv->executor.join();
    delete srv;
}

}  // extern "C"
