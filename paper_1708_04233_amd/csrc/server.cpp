// Hologram server: continuous batching of hologram jobs (one hologram each, Sec. 2) over several
// streams of one device, admitted in submission order under a device-memory budget.
//
// One scheduler thread per server owns every device call of the jobs: it admits the head of the
// queue as soon as a slot (stream) is free and the job's bytes fit the budget, issues the job's
// work on that slot's stream (upload through the slot's pinned staging buffer, quantise, fused
// superposition + inverse, then an event), and polls the events of the running jobs.
// Memory: each slot keeps a device arena that holds a job's working memory (points, quantised
// points, the superposition's scratch), grown when a larger job comes and given back when an idle
// slot's arena is needed to admit a job; the result is allocated per job and stays charged to the
// budget until the caller releases it.  The budget counts the shared LUT, the arenas and the held
// results, i.e. the device memory the server's jobs hold.  Client calls (submit / wait / cancel / release / query)
// only touch host state under the server's mutex, except release, which frees the result.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace cgh {
namespace {

using Clock = std::chrono::steady_clock;

enum class JobState { Queued, Running, Ended };

struct ServerJob {
    uint64_t ticket = 0;
    int64_t n = 0;
    int32_t nx = 0, ny = 0;
    std::vector<double> host;  // the job's points (copied at submit; empty when simulated)
    size_t work_bytes = 0, result_bytes = 0;
    JobState state = JobState::Queued;
    bool cancel = false;
    bool result_held = false;  // result_bytes still charged to the budget
    int status = CGH_OK;
    int slot = -1;
    double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0, sim_end = 0, gpu_ms = 0;
    void *d_u = nullptr;
    hipStream_t result_stream = nullptr;  // stream the result was allocated on
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    uint64_t ticket = 0;      // 0 = free
    void *pinned = nullptr;   // staging buffer of the uploads issued on this slot
    size_t pinned_cap = 0;
    size_t arena_cap = 0;     // bytes of the slot's arena charged to the budget
    void *arena = nullptr;    // the arena as allocated (at most arena_cap bytes; grown on issue)
    size_t arena_real = 0;
};

// How often the scheduler looks at the running jobs' events while any job runs.
constexpr auto kPollInterval = std::chrono::microseconds(20);

}  // namespace
}  // namespace cgh

struct cgh_server {
    cgh_server_config cfg{};
    int device = 0;
    int B = 8;
    cgh::Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<cgh::ServerJob>> jobs;
    std::vector<cgh::Slot> slots;
    size_t used = 0;        // budgeted bytes: the LUT, the slots' arenas, the held results
    size_t lut_bytes = 0;
    cgh_server_stats st{};
    uint64_t next_ticket = 1;
    bool closing = false, stopped = false;
    // The scheduler sleeps on cv_kick / kick_mu between rounds.
    std::mutex kick_mu;
    std::condition_variable cv_kick;
    bool kicked = false;
    int waiters = 0;
    std::thread thread;

    double now() const
    {
        return std::chrono::duration<double>(cgh::Clock::now() - t0).count();
    }
};

namespace cgh {
namespace {

// Wake the scheduler after a change of host state (submit, cancel, release, destroy).
void kick(cgh_server *S)
{
    std::lock_guard<std::mutex> lock(S->kick_mu);
    S->kicked = true;
    S->cv_kick.notify_all();
}

// The job ended: account for it and wake its waiters.  Lock held.
void end_job(cgh_server *S, ServerJob &j, int status)
{
    j.state = JobState::Ended;
    j.status = status;
    if (status == CGH_OK) ++S->st.completed;
    else if (status == CGH_ECANCELED) ++S->st.canceled;
    else ++S->st.failed;
    S->cv_done.notify_all();
}

void free_result(cgh_server *S, ServerJob &j)
{
    if (j.d_u) (void)hipFreeAsync(j.d_u, j.result_stream);
    j.d_u = nullptr;
    if (j.result_held) S->used -= j.result_bytes;
    j.result_held = false;
}

size_t round_up(size_t b)
{
    return (b + 255) & ~(size_t)255;
}

// Working memory of a job in its slot's arena.
size_t work_bytes_of(const wasabi_lut *lut, int64_t n, int32_t nx, int32_t ny)
{
    size_t b = round_up(sizeof(double) * 4 * (size_t)n) + round_up(sizeof(wasabi_point) * (size_t)n);
    if (lut) b += (size_t)fused_scratch_bound(lut, n, nx, ny, false);
    return b;
}

// Issue the job's device work on its slot's stream.  Called without the lock: the job and its
// slot belong to the scheduler while the job runs.
int issue(cgh_server *S, ServerJob &j, Slot &sl)
{
    hipStream_t s = sl.stream;
    const wasabi_lut *lut = S->cfg.lut;
    const size_t bytes = sizeof(double) * 4 * (size_t)j.n;
    if (bytes > sl.pinned_cap) {
        // the slot's previous upload has completed (its job ended), so the buffer is free
        if (sl.pinned) CGH_TRY_HIP(hipHostFree(sl.pinned));
        sl.pinned = nullptr;
        sl.pinned_cap = 0;
        size_t c = size_t(1) << 20;
        while (c < bytes) c <<= 1;
        CGH_TRY_HIP(hipHostMalloc(&sl.pinned, c, hipHostMallocDefault));
        sl.pinned_cap = c;
    }
    if (bytes) std::memcpy(sl.pinned, j.host.data(), bytes);
    CGH_TRY_HIP(hipEventRecord(sl.ev0, s));
    if (sl.arena_real < sl.arena_cap) {
        if (sl.arena) CGH_TRY_HIP(hipFreeAsync(sl.arena, s));
        sl.arena = nullptr;
        sl.arena_real = 0;
        CGH_TRY_HIP(hipMallocAsync(&sl.arena, sl.arena_cap, s));
        sl.arena_real = sl.arena_cap;
    }
    CGH_TRY_HIP(hipMallocAsync(&j.d_u, sizeof(float) * 2 * (size_t)j.nx * j.ny, s));
    j.result_stream = s;
    if (j.ticket == S->cfg.fail_ticket)
        return fail(CGH_EHIP, "job %llu: issue failed (forced by fail_ticket)", (unsigned long long)j.ticket);
    // arena: device points | quantised points | superposition scratch
    const size_t pts_bytes = round_up(bytes), q_bytes = round_up(sizeof(wasabi_point) * (size_t)j.n);
    char *ar = (char *)sl.arena;
    if (j.n > 0) {
        CGH_TRY_HIP(hipMemcpyAsync(ar, sl.pinned, bytes, hipMemcpyHostToDevice, s));
        int rc = wasabi_quantize(lut, (const double *)ar, j.n, (wasabi_point *)(ar + pts_bytes), s);
        if (rc) return rc;
    }
    int rc = hologram_fused_shared(lut, (const wasabi_point *)(ar + pts_bytes), j.n, j.nx, j.ny, j.d_u, s,
                                   ar + pts_bytes + q_bytes, sl.arena_real - pts_bytes - q_bytes);
    if (rc) return rc;
    CGH_TRY_HIP(hipEventRecord(sl.ev1, s));
    return CGH_OK;
}

// Device work of a running job ended (or failed to be issued): give back its slot and working
// memory.  Lock held.
void retire(cgh_server *S, ServerJob &j, int status)
{
    Slot &sl = S->slots[j.slot];
    if (!S->cfg.simulate && status == CGH_OK) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, sl.ev0, sl.ev1) == hipSuccess) j.gpu_ms = ms;
        else (void)hipGetLastError();
    }
    sl.ticket = 0;
    --S->st.running;
    std::vector<double>().swap(j.host);
    if (j.cancel || status != CGH_OK) {
        free_result(S, j);
        end_job(S, j, status != CGH_OK ? status : CGH_ECANCELED);
    } else {
        end_job(S, j, CGH_OK);
    }
}

// Give back the arena of an idle slot.  Lock held; the enqueue does not block.
void drop_arena(cgh_server *S, Slot &sl)
{
    if (sl.arena) (void)hipFreeAsync(sl.arena, sl.stream);
    sl.arena = nullptr;
    sl.arena_real = 0;
    S->used -= sl.arena_cap;
    sl.arena_cap = 0;
}

// Free slot for the queue head, or -1: the free slot with the largest arena, after giving back
// the arenas of other idle slots if that is what makes the job fit.  Lock held.
int pick_slot(cgh_server *S, const ServerJob &j)
{
    int best = -1;
    size_t others = 0;
    for (int i = 0; i < (int)S->slots.size(); ++i) {
        const Slot &sl = S->slots[i];
        if (sl.ticket) continue;
        if (best < 0 || sl.arena_cap > S->slots[best].arena_cap) best = i;
        others += sl.arena_cap;
    }
    if (best < 0) return -1;
    others -= S->slots[best].arena_cap;
    const size_t grow = j.work_bytes > S->slots[best].arena_cap ? j.work_bytes - S->slots[best].arena_cap : 0;
    const size_t need = j.result_bytes + grow;
    if (S->used + need <= S->cfg.hbm_budget_bytes) return best;
    if (S->used - others + need > S->cfg.hbm_budget_bytes) return -1;
    for (int i = 0; i < (int)S->slots.size() && S->used + need > S->cfg.hbm_budget_bytes; ++i)
        if (i != best && S->slots[i].ticket == 0 && S->slots[i].arena_cap) drop_arena(S, S->slots[i]);
    return best;
}

void admit(cgh_server *S, ServerJob &j, int slot, std::unique_lock<std::mutex> &lk)
{
    j.state = JobState::Running;
    j.slot = slot;
    j.t_admit = S->now();
    Slot &arena_slot = S->slots[slot];
    if (j.work_bytes > arena_slot.arena_cap) {
        S->used += j.work_bytes - arena_slot.arena_cap;
        arena_slot.arena_cap = j.work_bytes;
    }
    S->used += j.result_bytes;
    j.result_held = true;
    S->st.peak_bytes = std::max(S->st.peak_bytes, S->used);
    ++S->st.running;
    S->st.max_running = std::max(S->st.max_running, S->st.running);
    Slot &sl = S->slots[slot];
    sl.ticket = j.ticket;
    j.t_start = j.t_admit;
    if (S->cfg.simulate) {
        if (j.ticket == S->cfg.fail_ticket) {   // the modelled issue fails: the same path as on the device
            j.t_done = S->now();
            retire(S, j, fail(CGH_EHIP, "job %llu: issue failed (forced by fail_ticket)", (unsigned long long)j.ticket));
            return;
        }
        j.sim_end = j.t_start + S->cfg.sim_ns_per_pixel * 1e-9 * (double)j.nx * (double)j.ny;
        return;
    }
    lk.unlock();
    const int rc = issue(S, j, sl);
    j.t_start = S->now();
    if (rc) {
        // Nothing behind the failure will run; wait for what was enqueued before giving the
        // staging buffer and memory back.  The slot stays taken meanwhile.
        (void)hipStreamSynchronize(sl.stream);
        (void)hipGetLastError();
    }
    lk.lock();
    if (rc) {
        j.t_done = S->now();
        retire(S, j, rc);
    }
}

void scheduler(cgh_server *S)
{
    if (!S->cfg.simulate) (void)hipSetDevice(S->device);
    for (;;) {
        double wake_at = -1.0;  // simulation: when the next modelled job ends
        bool polling = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // 1. running jobs whose work has ended
            const double t = S->now();
            for (Slot &sl : S->slots) {
                if (sl.ticket == 0) continue;
                ServerJob &j = *S->jobs.at(sl.ticket);
                if (S->cfg.simulate) {
                    if (j.sim_end > t) continue;
                    j.t_done = t;
                    retire(S, j, CGH_OK);
                    continue;
                }
                const hipError_t e = hipEventQuery(sl.ev1);
                if (e == hipErrorNotReady) continue;
                j.t_done = t;
                if (e != hipSuccess) (void)hipGetLastError();
                retire(S, j, e == hipSuccess ? CGH_OK : fail(CGH_EHIP, "job %llu: %s",
                                                             (unsigned long long)j.ticket, hipGetErrorString(e)));
            }
            // 2. admissions, strictly in submission order
            while (!S->queue.empty()) {
                ServerJob &j = *S->jobs.at(S->queue.front());
                const int slot = pick_slot(S, j);
                if (slot < 0) break;
                S->queue.pop_front();
                admit(S, j, slot, lk);
            }
            if (S->closing && S->queue.empty() && S->st.running == 0) return;
            if (S->st.running > 0) {
                if (S->cfg.simulate) {
                    wake_at = 1e300;
                    for (const Slot &sl : S->slots)
                        if (sl.ticket) wake_at = std::min(wake_at, S->jobs.at(sl.ticket)->sim_end);
                } else {
                    polling = true;
                }
            }
        }
        // 3. sleep until a client call changes something, a modelled job ends or it is time to
        //    look at the running jobs again
        std::unique_lock<std::mutex> kl(S->kick_mu);
        auto ready = [&] { return S->kicked; };
        if (polling) {
            S->cv_kick.wait_for(kl, kPollInterval, ready);
        } else if (wake_at >= 0) {
            const auto when = S->t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(wake_at));
            S->cv_kick.wait_until(kl, when, ready);
        } else {
            S->cv_kick.wait(kl, ready);
        }
        S->kicked = false;
    }
}

void fill_result(const ServerJob &j, cgh_result *out)
{
    out->u = j.d_u;
    out->nx = j.nx;
    out->ny = j.ny;
    out->t_submit = j.t_submit;
    out->t_admit = j.t_admit;
    out->t_start = j.t_start;
    out->t_done = j.t_done;
    out->gpu_ms = j.gpu_ms;
    out->status = j.status;
    out->slot = j.slot;
}

}  // namespace
}  // namespace cgh

extern "C" int cgh_server_create(const cgh_server_config *cfg, cgh_server **out)
{
    using namespace cgh;
    if (!out) return fail(CGH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(CGH_EINVAL, "config is NULL");
    if (cfg->hbm_budget_bytes == 0) return fail(CGH_EINVAL, "hbm_budget_bytes must be > 0");
    if (cfg->max_slots < 1 || cfg->max_slots > 64) return fail(CGH_EINVAL, "max_slots must be 1..64");
    if (cfg->simulate && !(cfg->sim_ns_per_pixel >= 0)) return fail(CGH_EINVAL, "sim_ns_per_pixel must be >= 0");
    if (!cfg->simulate && !cfg->lut) return fail(CGH_EINVAL, "lut is NULL");
    if (cfg->lut && cfg->lut->prm.wavelet != CGH_HAAR)
        return fail(CGH_EINVAL, "the server computes jobs on the fused path, which needs a Haar LUT");
    // the shared LUT is device memory the server's jobs hold too: charged to the budget once
    const size_t lut_bytes = cfg->lut ? cfg->lut->device_bytes : 0;
    if (lut_bytes >= cfg->hbm_budget_bytes)
        return fail(CGH_ENOMEM, "the LUT alone (%zu bytes) fills the budget of %zu", lut_bytes, cfg->hbm_budget_bytes);
    std::unique_ptr<cgh_server> S(new cgh_server);
    S->cfg = *cfg;
    S->lut_bytes = lut_bytes;
    S->used = lut_bytes;
    S->st.peak_bytes = lut_bytes;
    S->t0 = Clock::now();
    S->B = cfg->lut ? cfg->lut->B : 8;
    S->slots.resize(cfg->max_slots);
    if (!cfg->simulate) {
        CGH_TRY_HIP(hipGetDevice(&S->device));
        if (S->device != cfg->lut->device)
            return fail(CGH_EINVAL, "LUT lives on device %d, current is %d", cfg->lut->device, S->device);
        int rc = prepare_pool();
        if (rc) return rc;
        for (Slot &sl : S->slots) {
            hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreate(&sl.ev0);
            if (e == hipSuccess) e = hipEventCreate(&sl.ev1);
            if (e != hipSuccess) {
                for (Slot &t : S->slots) {
                    if (t.stream) (void)hipStreamDestroy(t.stream);
                    if (t.ev0) (void)hipEventDestroy(t.ev0);
                    if (t.ev1) (void)hipEventDestroy(t.ev1);
                }
                return fail(CGH_EHIP, "stream/event creation failed: %s", hipGetErrorString(e));
            }
        }
    }
    cgh_server *raw = S.get();
    raw->thread = std::thread(scheduler, raw);
    *out = S.release();
    return CGH_OK;
}

extern "C" int cgh_server_submit(cgh_server *S, const cgh_job *job, uint64_t *ticket)
{
    using namespace cgh;
    if (!S || !job || !ticket) return fail(CGH_EINVAL, "NULL argument");
    *ticket = 0;
    const int B = S->B;
    if (job->nx < B || job->ny < B || job->nx % B || job->ny % B || job->nx > 65536 || job->ny > 65536)
        return fail(CGH_EINVAL, "hologram %d x %d must be positive multiples of %d, at most 65536",
                    job->nx, job->ny, B);
    if (job->n < 0 || job->n > INT32_MAX) return fail(CGH_EINVAL, "n out of range");
    if (job->n > 0 && !job->host_pts) return fail(CGH_EINVAL, "host_pts is NULL");
    std::unique_ptr<ServerJob> j(new ServerJob);
    j->n = job->n;
    j->nx = job->nx;
    j->ny = job->ny;
    j->result_bytes = sizeof(float) * 2 * (size_t)job->nx * job->ny;
    j->work_bytes = work_bytes_of(S->cfg.lut, job->n, job->nx, job->ny);
    if (j->work_bytes + j->result_bytes > S->cfg.hbm_budget_bytes - S->lut_bytes)
        return fail(CGH_ENOMEM, "job needs %zu bytes, budget is %zu of which the LUT holds %zu",
                    j->work_bytes + j->result_bytes, S->cfg.hbm_budget_bytes, S->lut_bytes);
    if (job->n > 0 && !S->cfg.simulate) {
        try {
            j->host.assign(job->host_pts, job->host_pts + 4 * job->n);
        } catch (const std::bad_alloc &) {
            return fail(CGH_ENOMEM, "host copy of %lld points failed", (long long)job->n);
        }
    }
    std::lock_guard<std::mutex> lock(S->mu);
    if (S->closing) return fail(CGH_ECANCELED, "server is shutting down");
    j->ticket = S->next_ticket++;
    j->t_submit = S->now();
    *ticket = j->ticket;
    S->queue.push_back(j->ticket);
    S->jobs.emplace(j->ticket, std::move(j));
    ++S->st.submitted;
    kick(S);
    return CGH_OK;
}

extern "C" int cgh_server_wait(cgh_server *S, uint64_t ticket, int32_t timeout_ms, cgh_result *out)
{
    using namespace cgh;
    if (!S || !out) return fail(CGH_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    const auto deadline = Clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    ++S->waiters;
    int rc = CGH_OK;
    for (;;) {
        auto it = S->jobs.find(ticket);
        if (it == S->jobs.end()) {
            rc = fail(CGH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
            break;
        }
        if (it->second->state == JobState::Ended) {
            fill_result(*it->second, out);
            break;
        }
        if (S->stopped) {
            rc = fail(CGH_ECANCELED, "server destroyed");
            break;
        }
        if (timeout_ms < 0) {
            S->cv_done.wait(lk);
        } else if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            auto jt = S->jobs.find(ticket);
            if (jt != S->jobs.end() && jt->second->state == JobState::Ended) {
                fill_result(*jt->second, out);
                break;
            }
            rc = fail(CGH_ETIMEDOUT, "ticket %llu not done after %d ms", (unsigned long long)ticket, timeout_ms);
            break;
        }
    }
    --S->waiters;
    S->cv_done.notify_all();
    return rc;
}

extern "C" int cgh_server_cancel(cgh_server *S, uint64_t ticket)
{
    using namespace cgh;
    if (!S) return fail(CGH_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(CGH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    ServerJob &j = *it->second;
    if (j.state == JobState::Ended) return fail(CGH_EINVAL, "job %llu has already ended", (unsigned long long)ticket);
    if (j.state == JobState::Queued) {
        S->queue.erase(std::find(S->queue.begin(), S->queue.end(), ticket));
        std::vector<double>().swap(j.host);
        j.t_done = S->now();
        end_job(S, j, CGH_ECANCELED);
        kick(S);
    } else {
        j.cancel = true;
    }
    return CGH_OK;
}

extern "C" int cgh_server_release(cgh_server *S, uint64_t ticket)
{
    using namespace cgh;
    if (!S) return fail(CGH_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(CGH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != JobState::Ended)
        return fail(CGH_EAGAIN, "job %llu has not ended", (unsigned long long)ticket);
    free_result(S, *it->second);
    S->jobs.erase(it);
    kick(S);
    return CGH_OK;
}

extern "C" int cgh_server_query(cgh_server *S, cgh_server_stats *out)
{
    using namespace cgh;
    if (!S || !out) return fail(CGH_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(S->mu);
    *out = S->st;
    out->queued = (int64_t)S->queue.size();
    out->bytes_in_use = S->used;
    out->arena_bytes = 0;
    for (const Slot &sl : S->slots) out->arena_bytes += sl.arena_cap;
    out->lut_bytes = S->lut_bytes;
    return CGH_OK;
}

extern "C" int cgh_server_destroy(cgh_server *S)
{
    using namespace cgh;
    if (!S) return CGH_OK;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->closing = true;
        for (uint64_t t : S->queue) {
            ServerJob &j = *S->jobs.at(t);
            std::vector<double>().swap(j.host);
            j.t_done = S->now();
            end_job(S, j, CGH_ECANCELED);
        }
        S->queue.clear();
        for (auto &kv : S->jobs)
            if (kv.second->state == JobState::Running) kv.second->cancel = true;
    }
    kick(S);
    S->thread.join();
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->stopped = true;
        S->cv_done.notify_all();
        S->cv_done.wait(lk, [&] { return S->waiters == 0; });
        for (auto &kv : S->jobs) free_result(S, *kv.second);
        S->jobs.clear();
    }
    if (!S->cfg.simulate) {
        for (Slot &sl : S->slots) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
            (void)hipEventDestroy(sl.ev0);
            (void)hipEventDestroy(sl.ev1);
            if (sl.pinned) (void)hipHostFree(sl.pinned);
            if (sl.arena) (void)hipFree(sl.arena);
        }
    }
    delete S;
    return CGH_OK;
}
