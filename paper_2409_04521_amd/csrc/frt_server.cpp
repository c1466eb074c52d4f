// Serving layer of the ray-tracing library (include/frt.h, "serving"):
// requests arrive with their inputs, wait in arrival order until a slot
// and enough of the device-memory budget are free, are loaded as solves by
// loader threads (several requests at once, each solve on its own stream, so
// uploads overlap each other and the running steps) and then advance one
// step per tick together with every
// other admitted solve (one batched step per tick and per n_bins/precision
// group, driven by the worker thread).  A finished request's x_HI and ledger
// are copied to host memory and its solve is destroyed, which frees its
// share of the budget for the next arrivals.  The layer uses only the
// public C ABI of the library and the host services of frt_serving.h.
#include "frt.h"
#include "frt_serving.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

namespace {

struct Req {
    uint64_t id = 0;
    int state = FRT_REQ_QUEUED;
    int err = FRT_OK;
    std::string msg;
    frt_params params{};
    int nx = 0, ny = 0, nz = 0, n_src = 0, rot_steps = 0, n_steps = 0;
    double box_cm = 0.0, dt = 0.0;
    std::vector<float> nH, T, kappa;
    std::vector<double> x0, pos, ndot, rot;
    size_t resident = 0;              // device bytes of the solve's own buffers
    size_t pass = 0;                  // its share of the context's pass queues at their first size
    frt_solve solve = nullptr;
    int steps_done = 0;
    std::vector<double> x_out;
    std::vector<double> T_out;        // with the temperature on
    frt_ledger led{};
    double t_submit = 0.0, t_start = -1.0, t_done = -1.0;

    void free_inputs()
    {
        std::vector<float>().swap(nH);
        std::vector<float>().swap(T);
        std::vector<float>().swap(kappa);
        std::vector<double>().swap(x0);
        std::vector<double>().swap(pos);
        std::vector<double>().swap(ndot);
        std::vector<double>().swap(rot);
    }
};

template <typename T>
int copy_in(const T* p, size_t n, int kind, std::vector<T>& out)
{
    out.resize(n);
    if (!n) return FRT_OK;
    if (kind == FRT_HOST) {
        std::memcpy(out.data(), p, n * sizeof(T));
        return FRT_OK;
    }
    if (frt::copy_device_to_host(out.data(), p, n * sizeof(T)) != FRT_OK)
        return frt::set_error(FRT_EDEVICE, "copying a request's device input failed");
    return FRT_OK;
}

int validate(const frt_request* r)
{
    if (!r || r->size != sizeof(frt_request)) return frt::set_error(FRT_EINVAL, "frt_request.size must be sizeof(frt_request)");
    if (r->params.size != sizeof(frt_params)) return frt::set_error(FRT_EINVAL, "frt_request.params.size must be sizeof(frt_params)");
    if (r->nx < 1 || r->ny < 1 || r->nz < 1 || r->nx > 2048 || r->ny > 2048 || r->nz > 2048)
        return frt::set_error(FRT_EINVAL, "request grid outside 1..2048 per axis");
    if (!r->n_H) return frt::set_error(FRT_EINVAL, "request without n_H");
    if (r->n_src < 0 || (r->n_src > 0 && (!r->pos_cm || !r->ndot_bins)))
        return frt::set_error(FRT_EINVAL, "request sources incomplete");
    if (r->n_steps < 0 || !(r->dt_s > 0) || !std::isfinite(r->dt_s))
        return frt::set_error(FRT_EINVAL, "request needs n_steps >= 0 and a finite dt_s > 0");
    if (r->params.n_bins < 1 || r->params.n_bins > FRT_MAX_BINS) return frt::set_error(FRT_EINVAL, "request n_bins outside 1..8");
    if (r->ptr_kind != FRT_HOST && r->ptr_kind != FRT_DEVICE) return frt::set_error(FRT_EINVAL, "bad ptr_kind");
    if (r->rotation_steps < 0 || (r->rotation_steps > 0 && !r->rotation_uniforms))
        return frt::set_error(FRT_EINVAL, "rotation table incomplete");
    return FRT_OK;
}


}  // namespace

struct frt_server_s {
    frt_ctx ctx = nullptr;
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    double t0 = 0.0;                  // frt::clock_s() at creation
    std::mutex mu;
    std::condition_variable cv;       // worker: work arrived, a solve loaded, or stop
    std::condition_variable load_cv;  // loader: a request was admitted, or stop
    std::condition_variable done_cv;  // waiters: a request finished
    std::deque<Req*> queue;           // submitted, not admitted
    std::deque<Req*> to_load;         // admitted, waiting for the loader
    std::vector<Req*> ready;          // loaded, joining the next tick
    int loading = 0;                  // admitted requests not yet in `active`
    bool admit_check = false;         // a submission or freed bytes since the last admission pass
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all;
    std::vector<Req*> active;         // worker thread only
    uint64_t next_id = 1;
    bool stop = false;
    frt_server_stats st{};
    // device bytes: the admitted solves' own buffers, the sum of their
    // pass-queue shares, and what the context's shared pass workspace holds
    // (it grows with the largest pass and never shrinks); in use is the
    // first plus the larger of the other two
    size_t resident_in_use = 0, pass_in_use = 0, ws_bytes = 0;
    std::thread worker;
    std::vector<std::thread> loaders;   // requests are loaded this many at a time

    // caller holds mu
    void update_bytes()
    {
        st.bytes_in_use = resident_in_use + std::max(pass_in_use, ws_bytes);
        st.peak_bytes = std::max(st.peak_bytes, st.bytes_in_use);
    }

    // Publish a request's end.  After this call the request may be taken
    // (and deleted) by a client at any time: the calling thread must not
    // touch it again, and no list of the worker may still hold it.
    void finish(Req* r, int state)
    {
        std::lock_guard<std::mutex> lock(mu);
        r->state = state;
        r->t_done = (frt::clock_s() - t0);
        resident_in_use -= r->resident;
        pass_in_use -= r->pass;
        update_bytes();
        if (state == FRT_REQ_DONE) st.completed++;
        else st.failed++;
        admit_check = true;
        cv.notify_all();
        done_cv.notify_all();
    }

    // code and message of the failing call, taken by the thread that made it
    void fail_req(Req* r, int code, const std::string& msg)
    {
        r->err = code;
        r->msg = msg;
        if (r->solve) {
            frt_solve_destroy(r->solve);
            r->solve = nullptr;
        }
        r->free_inputs();
        finish(r, FRT_REQ_FAILED);
    }

    int load(Req* r)
    {
        int rc;
        // a stream of its own: the upload overlaps the steps of the others
        if ((rc = frt_solve_create(ctx, &r->params, nullptr, &r->solve))) return rc;
        if ((rc = frt_load_grid(r->solve, r->nx, r->ny, r->nz, r->box_cm, r->nH.data(), r->T.empty() ? nullptr : r->T.data(),
                                r->kappa.empty() ? nullptr : r->kappa.data(), r->x0.empty() ? nullptr : r->x0.data(),
                                FRT_HOST)))
            return rc;
        if ((rc = frt_load_sources(r->solve, r->n_src, r->pos.data(), r->ndot.data(), FRT_HOST))) return rc;
        if (r->rot_steps > 0 && (rc = frt_set_rotations(r->solve, r->rot_steps, r->rot.data()))) return rc;
        return frt_sync(r->solve);
    }

    void run_loader()
    {
        (void)frt::use_device(device);
        for (;;) {
            Req* r = nullptr;
            {
                std::unique_lock<std::mutex> lock(mu);
                load_cv.wait(lock, [&] { return stop || !to_load.empty(); });
                if (stop) break;
                r = to_load.front();
                to_load.pop_front();
            }
            const int rc = load(r);
            r->free_inputs();
            if (rc != FRT_OK) {
                {
                    std::lock_guard<std::mutex> lock(mu);
                    loading--;
                    cv.notify_all();
                }
                fail_req(r, rc, frt_last_error());
                continue;
            }
            std::lock_guard<std::mutex> lock(mu);
            ready.push_back(r);
            cv.notify_all();
        }
    }

    void complete(Req* r)
    {
        const size_t ncell = (size_t)r->nx * r->ny * r->nz;
        r->x_out.resize(ncell);
        int rc = frt_read_fields(r->solve, r->x_out.data(), nullptr, FRT_HOST);
        if (rc == FRT_OK && r->params.temperature) {
            r->T_out.resize(ncell);
            rc = frt_read_temperature(r->solve, r->T_out.data(), FRT_HOST);
        }
        if (rc == FRT_OK) rc = frt_read_ledger(r->solve, &r->led);
        if (rc == FRT_OK && r->led.err_flags) rc = frt::set_error(FRT_EDEVICE, "the solve ended with device error bits set");
        if (rc != FRT_OK) {
            fail_req(r, rc, frt_last_error());
            return;
        }
        frt_solve_destroy(r->solve);
        r->solve = nullptr;
        r->free_inputs();
        finish(r, FRT_REQ_DONE);
    }

    void run()
    {
        (void)frt::use_device(device);
        for (;;) {
            std::vector<Req*> joined;
            {
                std::unique_lock<std::mutex> lock(mu);
                cv.wait(lock, [&] { return stop || !queue.empty() || !active.empty() || !ready.empty(); });
                if (stop) break;
                // admission in arrival order: a slot and the request's bytes
                admit_check = false;
                while (!queue.empty() && (int)active.size() + loading < max_slots) {
                    Req* r = queue.front();
                    if (r->resident + r->pass > budget) {
                        queue.pop_front();
                        r->err = FRT_ENOMEM;
                        r->msg = "request needs more device memory than the server's whole budget";
                        r->state = FRT_REQ_FAILED;
                        r->t_done = (frt::clock_s() - t0);
                        r->free_inputs();
                        st.failed++;
                        done_cv.notify_all();
                        continue;
                    }
                    if (resident_in_use + r->resident + std::max(ws_bytes, pass_in_use + r->pass) > budget) {
                        // pass queues grown by earlier requests and kept while
                        // idle: give them back, so the request sees its own
                        if (active.empty() && loading == 0 && ready.empty() && ws_bytes > 0) {
                            frt::ctx_trim_workspace(ctx);
                            ws_bytes = 0;
                            update_bytes();
                            continue;
                        }
                        break;
                    }
                    queue.pop_front();
                    resident_in_use += r->resident;
                    pass_in_use += r->pass;
                    update_bytes();
                    r->state = FRT_REQ_RUNNING;
                    r->t_start = (frt::clock_s() - t0);
                    to_load.push_back(r);
                    loading++;
                    load_cv.notify_all();
                }
                joined.swap(ready);
                loading -= (int)joined.size();
                if (active.empty() && joined.empty()) {
                    // nothing to step yet: wait for a load, or for a submission
                    // or freed bytes that may admit another request meanwhile
                    // (its upload then overlaps the ones under way)
                    cv.wait(lock, [&] { return stop || !ready.empty() || admit_check; });
                    if (stop) break;
                    continue;
                }
            }
            for (Req* r : joined) {
                if (r->n_steps == 0) complete(r);
                else active.push_back(r);
            }
            {
                std::lock_guard<std::mutex> lock(mu);
                st.max_in_flight = std::max<uint32_t>(st.max_in_flight, (uint32_t)active.size());
            }
            if (active.empty()) continue;
            // the shared pass queues may grow up to what the budget leaves
            // beside the admitted solves' own buffers
            {
                std::lock_guard<std::mutex> lock(mu);
                frt::ctx_set_workspace_limit(ctx, budget > resident_in_use ? budget - resident_in_use : 1);
            }
            // one tick: a batched step per group of solves that one launch
            // sequence can take (same n_bins, precision and queue mode)
            std::map<std::tuple<int, int, int>, std::vector<Req*>> groups;
            for (Req* r : active)
                groups[{r->params.n_bins, r->params.march_precision, r->params.queue_capacity == 0}].push_back(r);
            std::vector<std::pair<Req*, std::pair<int, std::string>>> failed;
            for (auto& kv : groups) {
                std::vector<Req*>& g = kv.second;
                for (size_t at = 0; at < g.size(); at += FRT_MAX_SOLVES_PER_LAUNCH) {
                    const size_t n = std::min<size_t>(FRT_MAX_SOLVES_PER_LAUNCH, g.size() - at);
                    std::vector<frt_solve> ss(n);
                    std::vector<double> dts(n);
                    for (size_t i = 0; i < n; i++) {
                        ss[i] = g[at + i]->solve;
                        dts[i] = g[at + i]->dt;
                    }
                    int rc = frt_batch_step(ss.data(), (int)n, dts.data());
                    size_t stepped = 0;
                    if (rc == FRT_OK) {
                        for (size_t i = 0; i < n; i++) g[at + i]->steps_done++;
                        stepped = n;
                    } else if (n == 1 || rc == FRT_EDEVICE) {
                        const std::string msg = frt_last_error();
                        for (size_t i = 0; i < n; i++) failed.push_back({g[at + i], {rc, msg}});
                    } else {
                        // a failed batched step leaves every solve at the start of
                        // the step: step them one by one, so that only those that
                        // fail alone (too large for what is left, say) fail
                        for (size_t i = 0; i < n; i++) {
                            Req* r = g[at + i];
                            const int rc1 = frt_batch_step(&ss[i], 1, &dts[i]);
                            if (rc1 == FRT_OK) {
                                r->steps_done++;
                                stepped++;
                            } else {
                                failed.push_back({r, {rc1, frt_last_error()}});
                            }
                        }
                    }
                    std::lock_guard<std::mutex> lock(mu);
                    st.ticks++;
                    st.solve_steps += stepped;
                }
            }
            {
                std::lock_guard<std::mutex> lock(mu);
                ws_bytes = frt::ctx_workspace_bytes(ctx);
                update_bytes();
            }
            // drop finished and failed requests from `active` before their
            // end is published (a client may take, and so delete, them
            // as soon as it is)
            std::vector<Req*> still, done;
            for (Req* r : active) {
                bool bad = false;
                for (auto& f : failed) bad |= f.first == r;
                if (bad) continue;
                if (r->steps_done >= r->n_steps) done.push_back(r);
                else still.push_back(r);
            }
            active.swap(still);
            for (auto& f : failed) fail_req(f.first, f.second.first, f.second.second);
            for (Req* r : done) complete(r);
        }
        for (Req* r : active)
            if (r->solve) {
                frt_solve_destroy(r->solve);
                r->solve = nullptr;
            }
        active.clear();
    }

    // after both threads stopped: solves that were loaded but never stepped
    void drop_ready()
    {
        for (Req* r : ready)
            if (r->solve) {
                frt_solve_destroy(r->solve);
                r->solve = nullptr;
            }
        ready.clear();
    }
};

extern "C" {

int frt_request_bytes(const frt_request* req, size_t* bytes)
{
    if (!bytes) return frt::set_error(FRT_EINVAL, "null output");
    int rc = validate(req);
    if (rc) return rc;
    const uint64_t ncell = (uint64_t)req->nx * req->ny * req->nz;
    *bytes = (size_t)frt::solve_bytes(req->params, ncell, req->n_src, req->T != nullptr, nullptr, nullptr);
    return FRT_OK;
}

int frt_server_create(frt_ctx ctx, size_t hbm_budget_bytes, int max_slots, frt_server* out)
{
    if (!ctx || !out) return frt::set_error(FRT_EINVAL, "null argument");
    if (max_slots < 1 || max_slots > FRT_MAX_SOLVES_PER_LAUNCH) return frt::set_error(FRT_EINVAL, "max_slots outside 1..1024");
    if (hbm_budget_bytes == 0) return frt::set_error(FRT_EINVAL, "zero memory budget");
    const int dev = frt::ctx_device(ctx);
    if (frt::use_device(dev) != FRT_OK) return frt::set_error(FRT_EDEVICE, "cannot select the context's device");
    std::unique_ptr<frt_server_s> s(new frt_server_s());
    s->ctx = ctx;
    s->device = dev;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->t0 = frt::clock_s();
    frt_server_s* raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    // the host side of a load (input checks and conversions, pageable
    // copies) takes longer than a step of a small solve: several loaders
    // keep the admitted requests flowing when many arrive at once
    for (int k = 0; k < 4; k++) s->loaders.emplace_back([raw] { raw->run_loader(); });
    *out = s.release();
    return FRT_OK;
}

int frt_server_submit(frt_server srv, const frt_request* req, uint64_t* req_id)
{
    if (!srv || !req_id) return frt::set_error(FRT_EINVAL, "null argument");
    int rc = validate(req);
    if (rc) return rc;
    std::unique_ptr<Req> r(new Req());
    r->params = req->params;
    r->nx = req->nx;
    r->ny = req->ny;
    r->nz = req->nz;
    r->box_cm = req->box_cm;
    r->n_src = req->n_src;
    r->n_steps = req->n_steps;
    r->dt = req->dt_s;
    r->rot_steps = req->rotation_steps;
    const size_t ncell = (size_t)req->nx * req->ny * req->nz;
    const size_t nb = (size_t)req->params.n_bins;
    if ((rc = copy_in(req->n_H, ncell, req->ptr_kind, r->nH))) return rc;
    if (req->T && (rc = copy_in(req->T, ncell, req->ptr_kind, r->T))) return rc;
    if (req->kappa_sub && (rc = copy_in(req->kappa_sub, ncell, req->ptr_kind, r->kappa))) return rc;
    if (req->x_HI0 && (rc = copy_in(req->x_HI0, ncell, req->ptr_kind, r->x0))) return rc;
    if ((rc = copy_in(req->pos_cm, (size_t)req->n_src * 3, req->ptr_kind, r->pos))) return rc;
    if ((rc = copy_in(req->ndot_bins, (size_t)req->n_src * nb, req->ptr_kind, r->ndot))) return rc;
    if (req->rotation_steps > 0 &&
        (rc = copy_in(req->rotation_uniforms, (size_t)req->rotation_steps * req->n_src * 3, req->ptr_kind, r->rot)))
        return rc;
    uint64_t pass_bytes = 0;
    const uint64_t total = frt::solve_bytes(req->params, ncell, req->n_src, req->T != nullptr, nullptr, &pass_bytes);
    r->resident = (size_t)(total - pass_bytes);
    r->pass = (size_t)pass_bytes;
    std::lock_guard<std::mutex> lock(srv->mu);
    r->id = srv->next_id++;
    r->t_submit = (frt::clock_s() - srv->t0);
    *req_id = r->id;
    srv->queue.push_back(r.get());
    srv->all[r->id] = std::move(r);
    srv->st.submitted++;
    srv->admit_check = true;
    srv->cv.notify_all();
    return FRT_OK;
}

int frt_server_poll(frt_server srv, uint64_t req_id, int* state)
{
    if (!srv || !state) return frt::set_error(FRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->all.find(req_id);
    if (it == srv->all.end()) return frt::set_error(FRT_EINVAL, "unknown request");
    *state = it->second->state;
    return FRT_OK;
}

int frt_server_wait(frt_server srv, uint64_t req_id, double timeout_s, int* state)
{
    if (!srv || !state) return frt::set_error(FRT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lock(srv->mu);
    auto it = srv->all.find(req_id);
    if (it == srv->all.end()) return frt::set_error(FRT_EINVAL, "unknown request");
    Req* r = it->second.get();
    auto done = [&] { return r->state == FRT_REQ_DONE || r->state == FRT_REQ_FAILED; };
    if (timeout_s < 0) srv->done_cv.wait(lock, done);
    else srv->done_cv.wait_for(lock, std::chrono::duration<double>(timeout_s), done);
    *state = r->state;
    return FRT_OK;
}

int frt_server_take(frt_server srv, uint64_t req_id, double* x_HI, frt_ledger* ledger)
{
    if (!srv) return frt::set_error(FRT_EINVAL, "null server");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->all.find(req_id);
    if (it == srv->all.end()) return frt::set_error(FRT_EINVAL, "unknown request");
    Req* r = it->second.get();
    if (r->state == FRT_REQ_FAILED) {
        const int code = r->err ? r->err : FRT_EDEVICE;
        const std::string msg = r->msg;
        srv->all.erase(it);
        return frt::set_error(code, msg.c_str());
    }
    if (r->state != FRT_REQ_DONE) return frt::set_error(FRT_ESTATE, "request not finished");
    if (x_HI) std::memcpy(x_HI, r->x_out.data(), r->x_out.size() * sizeof(double));
    if (ledger) *ledger = r->led;
    srv->all.erase(it);
    return FRT_OK;
}

int frt_server_read_temperature(frt_server srv, uint64_t req_id, double* T)
{
    if (!srv || !T) return frt::set_error(FRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->all.find(req_id);
    if (it == srv->all.end()) return frt::set_error(FRT_EINVAL, "unknown request");
    const Req* r = it->second.get();
    if (r->state != FRT_REQ_DONE) return frt::set_error(FRT_ESTATE, "request not finished");
    if (r->T_out.empty()) return frt::set_error(FRT_ESTATE, "the request did not evolve its temperature");
    std::memcpy(T, r->T_out.data(), r->T_out.size() * sizeof(double));
    return FRT_OK;
}

int frt_server_times(frt_server srv, uint64_t req_id, double t[3])
{
    if (!srv || !t) return frt::set_error(FRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->all.find(req_id);
    if (it == srv->all.end()) return frt::set_error(FRT_EINVAL, "unknown request");
    t[0] = it->second->t_submit;
    t[1] = it->second->t_start;
    t[2] = it->second->t_done;
    return FRT_OK;
}

int frt_server_get_stats(frt_server srv, frt_server_stats* out)
{
    if (!srv || !out) return frt::set_error(FRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    *out = srv->st;
    return FRT_OK;
}

int frt_server_destroy(frt_server srv)
{
    if (!srv) return FRT_OK;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
        srv->load_cv.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    for (std::thread& t : srv->loaders)
        if (t.joinable()) t.join();
    srv->drop_ready();
    delete srv;
    return FRT_OK;
}

}  // extern "C"
