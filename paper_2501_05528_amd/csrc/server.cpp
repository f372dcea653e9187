// Request loop for compression jobs (blr_server_*, include/blr_tag.h): jobs are
// admitted in arrival order when a slot and enough of the HBM budget are free,
// and each slot runs blr_tag_compress on its own stream, so the device overlaps
// the jobs of different slots.  A job's arithmetic never depends on the others.
#include <hip/hip_runtime.h>

#include <chrono>
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct ServerJob {
    const blr_plan* plan = nullptr;
    const blr_operator* op = nullptr;
    const double* G = nullptr;
    const double* H = nullptr;
    blr_compress_opts opts{};
    bool has_opts = false;
    int64_t out_bytes = 0;  // bytes of the result handle, charged until the client claims it
    blr_ublr* result = nullptr;
    blr_server_job_stats st{};
    bool done = false;
    std::string msg;  // error message of a failed job
};

}  // namespace

struct blr_server {
    int device = -1;
    int64_t budget = 0;
    int64_t used = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<ServerJob>> jobs;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> ev_start, ev_end;  // per slot: device interval of the running job
    hipEvent_t ev_origin = nullptr;            // device time origin of the server
    bool stop = false;
    uint64_t next_id = 1;

    // Drops a completed result nobody can claim any more (the server is stopping).
    void discard_result(ServerJob& j) {
        if (j.result) blr_ublr_destroy(j.result);
        j.result = nullptr;
        used -= j.out_bytes;
        j.out_bytes = 0;
    }

    void work(int slot) {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lock(mu);
        for (;;) {
            cv_work.wait(lock, [&] {
                if (queue.empty()) return stop;
                const ServerJob& head = *jobs.at(queue.front());
                return used + head.st.footprint <= budget;
            });
            if (queue.empty()) return;  // stop requested and nothing left
            const uint64_t id = queue.front();
            queue.pop_front();
            ServerJob& j = *jobs.at(id);
            used += j.st.footprint;
            j.st.slot = slot;
            j.st.t_start = now_s();
            lock.unlock();
            cv_work.notify_all();  // the next head may fit as well
            blr_report rep{};
            blr_ublr* h = nullptr;
            (void)hipEventRecord(ev_start[slot], streams[slot]);
            const blr_status s = blr_tag_compress(j.plan, j.op, j.G, j.H, j.has_opts ? &j.opts : nullptr,
                                                  streams[slot], &h, &rep);
            const std::string msg = s == BLR_OK ? std::string() : std::string(blr_last_error_message());
            float t0 = -1.0f, t1 = -1.0f;
            if (hipEventRecord(ev_end[slot], streams[slot]) == hipSuccess &&
                hipEventSynchronize(ev_end[slot]) == hipSuccess &&
                hipEventElapsedTime(&t0, ev_origin, ev_start[slot]) == hipSuccess &&
                hipEventElapsedTime(&t1, ev_origin, ev_end[slot]) == hipSuccess) {
            } else {
                (void)hipGetLastError();
                t0 = t1 = -1.0f;
            }
            lock.lock();
            j.msg = msg;
            j.st.t_end = now_s();
            j.st.dev_start_ms = t0;
            j.st.dev_end_ms = t1;
            j.st.ms_device = rep.ms_total;
            j.st.status = s;
            j.result = h;
            j.done = true;
            // The temporaries are gone; the result keeps its bytes charged until claimed.
            j.out_bytes = (s == BLR_OK) ? std::min(j.out_bytes, j.st.footprint) : 0;
            used -= j.st.footprint - j.out_bytes;
            if (stop) discard_result(j);
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

extern "C" {

blr_status blr_server_create(int64_t hbm_budget, int32_t slots, blr_server** out) {
    if (out) *out = nullptr;
    try {
        if (!out) blr::fail(BLR_ERR_INVALID_ARG, "NULL output");
        if (slots < 1 || slots > 16) blr::fail(BLR_ERR_INVALID_ARG, "slots must be in 1..16");
        if (hbm_budget <= 0) blr::fail(BLR_ERR_INVALID_ARG, "the HBM budget must be positive");
        auto S = std::make_unique<blr_server>();
        if (hipGetDevice(&S->device) != hipSuccess) blr::fail(BLR_ERR_DEVICE, "no current device");
        S->budget = hbm_budget;
        auto release = [&] {
            for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
            for (hipEvent_t e : S->ev_start) (void)hipEventDestroy(e);
            for (hipEvent_t e : S->ev_end) (void)hipEventDestroy(e);
            if (S->ev_origin) (void)hipEventDestroy(S->ev_origin);
        };
        for (int q = 0; q < slots; ++q) {
            hipStream_t st = nullptr;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                release();
                blr::fail(BLR_ERR_DEVICE, "stream creation failed");
            }
            S->streams.push_back(st);
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
                if (e0) (void)hipEventDestroy(e0);
                release();
                blr::fail(BLR_ERR_DEVICE, "event creation failed");
            }
            S->ev_start.push_back(e0);
            S->ev_end.push_back(e1);
        }
        if (hipEventCreate(&S->ev_origin) != hipSuccess || hipEventRecord(S->ev_origin, S->streams[0]) != hipSuccess ||
            hipEventSynchronize(S->ev_origin) != hipSuccess) {
            release();
            blr::fail(BLR_ERR_DEVICE, "event creation failed");
        }
        blr_server* raw = S.get();
        for (int q = 0; q < slots; ++q) S->workers.emplace_back([raw, q] { raw->work(q); });
        *out = S.release();
        return BLR_OK;
    } catch (const blr::Error& e) {
        blr::set_last_error(e.what());
        return e.status;
    } catch (const std::exception& e) {
        blr::set_last_error(e.what());
        return BLR_ERR_INVALID_ARG;
    }
}

blr_status blr_server_submit(blr_server* srv, const blr_plan* plan, const blr_operator* op,
                             const double* G, const double* H, const blr_compress_opts* opts,
                             uint64_t* ticket) {
    if (ticket) *ticket = 0;
    try {
        if (!srv || !plan || !op || !G || !H || !ticket) blr::fail(BLR_ERR_INVALID_ARG, "NULL argument");
        const int prec = opts ? opts->precision : BLR_PREC_FP64;
        const int r_lo = opts ? opts->r_lo : 0;
        int64_t fp = 0;
        const blr_status fs = blr_plan_footprint(plan, prec, r_lo, &fp);
        if (fs != BLR_OK) blr::fail(fs, blr_last_error_message());
        if (fp > srv->budget) blr::fail(BLR_ERR_BUSY, "the job's footprint exceeds the server's HBM budget");
        const bool keep = opts && opts->keep_intermediates;
        const int64_t out_bytes = keep ? fp : blr::result_bytes(*plan->d);
        auto j = std::make_unique<ServerJob>();
        j->plan = plan;
        j->op = op;
        j->G = G;
        j->H = H;
        if (opts) {
            j->opts = *opts;
            j->has_opts = true;
        }
        j->st.footprint = fp;
        j->out_bytes = out_bytes;
        j->st.t_submit = now_s();
        j->st.slot = -1;
        {
            std::lock_guard<std::mutex> lock(srv->mu);
            if (srv->stop) blr::fail(BLR_ERR_INVALID_ARG, "server is shutting down");
            const uint64_t id = srv->next_id++;
            srv->jobs.emplace(id, std::move(j));
            srv->queue.push_back(id);
            *ticket = id;
        }
        srv->cv_work.notify_all();
        return BLR_OK;
    } catch (const blr::Error& e) {
        blr::set_last_error(e.what());
        return e.status;
    } catch (const std::exception& e) {
        blr::set_last_error(e.what());
        return BLR_ERR_INVALID_ARG;
    }
}

blr_status blr_server_poll(blr_server* srv, uint64_t ticket, int32_t* done) {
    if (!srv || !done) return BLR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) {
        blr::set_last_error("unknown or already claimed ticket");
        return BLR_ERR_INVALID_ARG;
    }
    *done = it->second->done ? 1 : 0;
    return BLR_OK;
}

blr_status blr_server_wait(blr_server* srv, uint64_t ticket, blr_ublr** out,
                           blr_server_job_stats* stats) {
    if (out) *out = nullptr;
    if (!srv || !out) return BLR_ERR_INVALID_ARG;
    std::unique_ptr<ServerJob> j;
    {
        std::unique_lock<std::mutex> lock(srv->mu);
        auto it = srv->jobs.find(ticket);
        if (it == srv->jobs.end()) {
            blr::set_last_error("unknown or already claimed ticket");
            return BLR_ERR_INVALID_ARG;
        }
        ServerJob* jp = it->second.get();  // stable: the map holds the job by pointer
        srv->cv_done.wait(lock, [&] { return jp->done; });
        it = srv->jobs.find(ticket);        // the map may have rehashed while waiting
        j = std::move(it->second);
        srv->jobs.erase(it);
        srv->used -= j->out_bytes;       // the handle leaves the server's accounting
    }
    srv->cv_work.notify_all();
    *out = j->result;
    if (stats) *stats = j->st;
    if (j->st.status != BLR_OK) blr::set_last_error(j->msg.empty() ? std::string("the job failed") : j->msg);
    return static_cast<blr_status>(j->st.status);
}

void blr_server_destroy(blr_server* srv) {
    if (!srv) return;
    {
        // Completed results can no longer be claimed: free them and their charge, so
        // that queued jobs still find room in the budget.
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
        for (auto& kv : srv->jobs)
            if (kv.second->done) srv->discard_result(*kv.second);
    }
    srv->cv_work.notify_all();
    for (auto& w : srv->workers) w.join();
    for (auto& kv : srv->jobs)
        if (kv.second->result) blr_ublr_destroy(kv.second->result);
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : srv->ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : srv->ev_end) (void)hipEventDestroy(e);
    if (srv->ev_origin) (void)hipEventDestroy(srv->ev_origin);
    delete srv;
}

}  // extern "C"
