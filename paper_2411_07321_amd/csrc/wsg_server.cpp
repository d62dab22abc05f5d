// Continuous-batching imaging server (include/wsg.h, "Serving").
//
// Slots are worker threads, each with a private context (stream + workspace),
// so admitted jobs run concurrently on separate streams and their staging
// copies, kernels and read-back overlap.  Admission is decided under one lock
// whenever a job arrives or finishes: the first queued job whose workspace
// fits in the budget next to what the other slots hold is given to a free
// slot.  Idle slots give their workspace back when a queued job would not fit
// otherwise.
#include "../../include/wsg.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

uint64_t wsg_ctx_device_bytes(const wsg_ctx *ctx);

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
    uint64_t ticket = 0;
    wsg_params p{};
    wsg_vis v{};
    double *image = nullptr;
    int32_t image_mem = WSG_MEM_DEVICE;
    uint64_t footprint = 0;
    bool done = false;
    wsg_job_info info{};
};

struct Slot {
    wsg_ctx *ctx = nullptr;
    std::thread th;
    std::shared_ptr<Job> job;     // assigned job (null when idle)
    uint64_t held = 0;            // device bytes the slot's context holds
    bool busy = false;
};

}  // namespace

struct wsg_server {
    int device = 0;
    uint64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<std::shared_ptr<Job>> queue;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    std::vector<Slot> slots;
    uint64_t peak = 0;
    // failure isolation checks: jobs of this mesh size fail in their slot before any
    // device work (WSG_SERVER_FAIL_GRID_N, read once when the server is created; 0: none)
    int fail_grid_n = 0;

    uint64_t held_total() const {
        uint64_t h = 0;
        for (const Slot &s : slots) h += s.held;
        return h;
    }

    // Start every queued job that can start now (caller holds mu).
    void pump() {
        bool progressed = true;
        while (progressed && !queue.empty()) {
            progressed = false;
            for (auto it = queue.begin(); it != queue.end(); ++it) {
                const std::shared_ptr<Job> &j = *it;
                int pick = -1;
                uint64_t other = 0;
                for (size_t i = 0; i < slots.size(); ++i) {
                    if (slots[i].busy) continue;
                    // prefer a free slot whose workspace already fits the job
                    if (pick < 0 || (slots[i].held >= j->footprint && slots[(size_t)pick].held < j->footprint))
                        pick = (int)i;
                }
                if (pick < 0) return;   // no free slot
                for (size_t i = 0; i < slots.size(); ++i)
                    if ((int)i != pick) other += slots[i].held;
                uint64_t need = std::max(slots[(size_t)pick].held, j->footprint);
                if (budget && other + need > budget) {
                    // idle slots may give their workspace back
                    uint64_t idle = 0;
                    for (size_t i = 0; i < slots.size(); ++i)
                        if ((int)i != pick && !slots[i].busy) idle += slots[i].held;
                    if (other - idle + j->footprint > budget) continue;   // try a later job
                    for (size_t i = 0; i < slots.size(); ++i)
                        if ((int)i != pick && !slots[i].busy && slots[i].held) {
                            wsg_trim(slots[i].ctx);
                            slots[i].held = 0;
                        }
                    if (slots[(size_t)pick].held > j->footprint) {
                        wsg_trim(slots[(size_t)pick].ctx);
                        slots[(size_t)pick].held = 0;
                    }
                }
                Slot &s = slots[(size_t)pick];
                s.busy = true;
                s.job = j;
                s.held = std::max(s.held, j->footprint);
                peak = std::max(peak, held_total());
                queue.erase(it);
                progressed = true;
                cv_work.notify_all();
                break;
            }
        }
    }

    void worker(size_t idx) {
        Slot &s = slots[idx];
        for (;;) {
            std::shared_ptr<Job> j;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || (s.busy && s.job); });
                if (!s.job) return;   // stopping and idle
                j = s.job;
            }
            j->info.t_start = now_s();
            wsg_stats st{};
            int n_img = wsg_n_images(&j->p, &j->v);
            std::vector<wsg_stats> all((size_t)std::max(1, n_img));
            wsg_status rc = (fail_grid_n && j->p.grid_n == fail_grid_n)
                                ? WSG_EDEVICE
                                : wsg_image(s.ctx, &j->p, &j->v, j->image, j->image_mem,
                                            wsg_context_stream(s.ctx), all.data());
            if (rc == WSG_OK) st = all[0];
            double t_end = now_s();
            {
                std::lock_guard<std::mutex> lk(mu);
                j->info.status = rc;
                j->info.t_end = t_end;
                j->info.stats = st;
                j->done = true;
                s.held = wsg_ctx_device_bytes(s.ctx);
                peak = std::max(peak, held_total());
                s.job.reset();
                s.busy = false;
                pump();
            }
            cv_done.notify_all();
        }
    }
};

extern "C" {

wsg_status wsg_server_create(int device, int32_t n_slots, uint64_t hbm_budget, wsg_server **out) {
    if (!out || n_slots < 1 || n_slots > 64) return WSG_EINVAL;
    *out = nullptr;
    wsg_server *srv = new (std::nothrow) wsg_server();
    if (!srv) return WSG_ENOMEM;
    srv->device = device;
    srv->budget = hbm_budget;
    if (const char *f = std::getenv("WSG_SERVER_FAIL_GRID_N")) srv->fail_grid_n = std::atoi(f);
    srv->slots.resize((size_t)n_slots);
    for (auto &s : srv->slots) {
        wsg_status rc = wsg_create(device, &s.ctx);
        if (rc != WSG_OK) {
            for (auto &t : srv->slots)
                if (t.ctx) wsg_destroy(t.ctx);
            delete srv;
            return rc;
        }
    }
    for (size_t i = 0; i < srv->slots.size(); ++i)
        srv->slots[i].th = std::thread([srv, i] {
            (void)hipSetDevice(srv->device);
            srv->worker(i);
        });
    *out = srv;
    return WSG_OK;
}

void wsg_server_destroy(wsg_server *srv) {
    if (!srv) return;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_done.wait(lk, [&] {
            if (!srv->queue.empty()) return false;
            for (auto &s : srv->slots)
                if (s.busy) return false;
            return true;
        });
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &s : srv->slots)
        if (s.th.joinable()) s.th.join();
    for (auto &s : srv->slots)
        if (s.ctx) wsg_destroy(s.ctx);
    delete srv;
}

wsg_status wsg_server_submit(wsg_server *srv, const wsg_params *p, const wsg_vis *v, double *image,
                             int32_t image_mem, uint64_t *ticket) {
    if (!srv || !p || !v || !image || !ticket) return WSG_EINVAL;
    wsg_status rc = wsg_check(p, v);
    if (rc != WSG_OK) return rc;
    uint64_t fp = 0;
    rc = wsg_footprint(p, v, &fp);
    if (rc != WSG_OK) return rc;
    if (srv->budget && fp > srv->budget) return WSG_ENOMEM;
    auto j = std::make_shared<Job>();
    j->p = *p;
    j->v = *v;
    j->image = image;
    j->image_mem = image_mem;
    j->footprint = fp;
    j->info.footprint = fp;
    j->info.t_submit = now_s();
    std::lock_guard<std::mutex> lk(srv->mu);
    j->ticket = srv->next_ticket++;
    srv->jobs[j->ticket] = j;
    srv->queue.push_back(j);
    *ticket = j->ticket;
    srv->pump();
    return WSG_OK;
}

wsg_status wsg_server_poll(wsg_server *srv, uint64_t ticket, int32_t *done, wsg_job_info *info) {
    if (!srv || !done) return WSG_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return WSG_EINVAL;
    *done = it->second->done ? 1 : 0;
    if (it->second->done) {
        if (info) *info = it->second->info;
        srv->jobs.erase(it);
    }
    return WSG_OK;
}

wsg_status wsg_server_wait(wsg_server *srv, uint64_t ticket, wsg_job_info *info) {
    if (!srv) return WSG_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return WSG_EINVAL;
    std::shared_ptr<Job> j = it->second;
    srv->cv_done.wait(lk, [&] { return j->done; });
    if (info) *info = j->info;
    srv->jobs.erase(ticket);
    return WSG_OK;
}

wsg_status wsg_server_cancel(wsg_server *srv, uint64_t ticket) {
    if (!srv) return WSG_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return WSG_EINVAL;
    const std::shared_ptr<Job> j = it->second;
    if (j->done) return WSG_OK;
    for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
        if (*q == j) {
            srv->queue.erase(q);
            j->info.status = WSG_ECANCELED;
            j->info.t_start = j->info.t_end = now_s();
            j->done = true;
            srv->cv_done.notify_all();
            return WSG_OK;
        }
    return WSG_EBUSY;   // admitted: its slot is running it
}

wsg_status wsg_server_memory(wsg_server *srv, uint64_t *held, uint64_t *peak) {
    if (!srv) return WSG_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (held) *held = srv->held_total();
    if (peak) *peak = srv->peak;
    return WSG_OK;
}

}  // extern "C"
