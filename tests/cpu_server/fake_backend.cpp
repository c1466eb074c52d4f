// CPU stand-in for the ray-tracing library under the serving layer
// (frt_server.cpp), for the scheduler's tests without a GPU: every call the
// layer makes (the ABI of include/frt.h it uses and the services of
// frt_serving.h) with the same contracts (a failed batched step changes no
// solve, solves of one batch share n_bins, precision and queue mode, the
// shared pass queues grow with the batch and respect the context's limit),
// a virtual clock advanced by the work done, and failures injected on
// request (fake_control.h).  A solve's "neutral fraction" after k steps is
// 1 / (1 + k) + 1e-6 tag + 1e-9 cell, with tag = n_H[0] of its grid, so a
// test can tell that every request received exactly its own steps; with the
// temperature on, its T is 1e4 + k + 1e-3 tag + 1e-6 cell.
#include "fake_control.h"

#include "frt.h"
#include "frt_serving.h"

#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

struct frt_ctx_s {
    int device = 0;
    uint64_t ws_bytes = 0, ws_limit = 0;
};

struct frt_solve_s {
    frt_ctx ctx = nullptr;
    frt_params P{};
    int nx = 0, ny = 0, nz = 0, n_src = -1;
    double tag = 0.0;
    uint64_t steps = 0;
    bool grid = false;
};

namespace {

std::mutex g_mu;                        // every piece of state below
fake::Faults g_faults;
int g_creates = 0, g_loads = 0, g_loaded = 0, g_live = 0;
bool g_hold = false, g_hold_steps = false;
std::condition_variable g_release;
uint64_t g_batches = 0, g_max_batch = 0;
std::atomic<int64_t> g_clock_ns{0};
thread_local std::string t_error;

int err(int code, const char* msg)
{
    t_error = msg;
    return code;
}

uint64_t ncell(const frt_solve_s* s) { return (uint64_t)s->nx * s->ny * s->nz; }

double value(double tag, uint64_t steps, uint64_t cell) { return 1.0 / (1.0 + (double)steps) + 1e-6 * tag + 1e-9 * (double)cell; }

void tick(int64_t ns) { g_clock_ns.fetch_add(ns); }

}  // namespace

namespace fake {

void reset(const Faults& f)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_faults = f;
    g_creates = g_loads = g_loaded = 0;
    g_hold = g_hold_steps = false;
    g_batches = g_max_batch = 0;
}

void hold_loads(bool hold)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_hold = hold;
    g_release.notify_all();
}

void hold_steps(bool hold)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_hold_steps = hold;
    g_release.notify_all();
}

int loads_started()
{
    std::lock_guard<std::mutex> lock(g_mu);
    return g_loads;
}

int loads_done()
{
    std::lock_guard<std::mutex> lock(g_mu);
    return g_loaded;
}

int live_solves()
{
    std::lock_guard<std::mutex> lock(g_mu);
    return g_live;
}

uint64_t batches()
{
    std::lock_guard<std::mutex> lock(g_mu);
    return g_batches;
}

uint64_t max_batch()
{
    std::lock_guard<std::mutex> lock(g_mu);
    return g_max_batch;
}

void advance_clock(double seconds) { tick((int64_t)std::llround(seconds * 1e9)); }

double expected_x(double tag, uint64_t steps, uint64_t cell) { return value(tag, steps, cell); }

double expected_T(double tag, uint64_t steps, uint64_t cell) { return 1e4 + (double)steps + 1e-3 * tag + 1e-6 * (double)cell; }

uint64_t cell_bytes() { return 36; }

uint64_t pass_bytes_per_cell() { return 32; }

}  // namespace fake

extern "C" {

const char* frt_last_error(void) { return t_error.c_str(); }

int frt_params_default(frt_params* p)
{
    if (!p) return err(FRT_EINVAL, "null params");
    std::memset(p, 0, sizeof(*p));
    p->size = sizeof(frt_params);
    p->n_bins = 1;
    p->sigma_bins[0] = 6.3e-18;
    p->alpha_B = 2.59e-13;
    p->max_level = 12;
    p->n_ray_min = 1.0;
    p->c_ray_cm_s = INFINITY;
    return FRT_OK;
}

int frt_ctx_create(int hip_device, frt_alloc_fn, frt_free_fn, void*, frt_ctx* out)
{
    if (!out) return err(FRT_EINVAL, "null output");
    frt_ctx c = new frt_ctx_s();
    c->device = hip_device;
    *out = c;
    return FRT_OK;
}

int frt_ctx_destroy(frt_ctx ctx)
{
    delete ctx;
    return FRT_OK;
}

int frt_solve_create(frt_ctx ctx, const frt_params* params, void*, frt_solve* out)
{
    if (!ctx || !params || !out) return err(FRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(g_mu);
    if (++g_creates == g_faults.create_fail_at) return err(FRT_ENOMEM, "injected: solve creation out of memory");
    frt_solve s = new frt_solve_s();
    s->ctx = ctx;
    s->P = *params;
    g_live++;
    *out = s;
    return FRT_OK;
}

int frt_solve_destroy(frt_solve s)
{
    if (!s) return FRT_OK;
    std::lock_guard<std::mutex> lock(g_mu);
    g_live--;
    delete s;
    return FRT_OK;
}

int frt_load_grid(frt_solve s, int nx, int ny, int nz, double, const float* n_H, const float*, const float*,
                  const double*, int ptr_kind)
{
    if (!s || !n_H || ptr_kind != FRT_HOST || nx < 1 || ny < 1 || nz < 1) return err(FRT_EINVAL, "bad grid");
    {
        std::unique_lock<std::mutex> lock(g_mu);
        if (++g_loads == g_faults.load_fail_at) return err(FRT_ENOMEM, "injected: grid upload out of memory");
        g_release.wait(lock, [] { return !g_hold; });
    }
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->tag = n_H[0];
    s->grid = true;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_loaded++;
    }
    tick(5000 + (int64_t)(0.1 * (double)ncell(s)));
    std::this_thread::yield();
    return FRT_OK;
}

int frt_load_sources(frt_solve s, int n_src, const double*, const double*, int)
{
    if (!s || n_src < 0) return err(FRT_EINVAL, "bad sources");
    if (!s->grid) return err(FRT_ESTATE, "sources before the grid");
    s->n_src = n_src;
    return FRT_OK;
}

int frt_set_rotations(frt_solve s, int n_steps, const double* u)
{
    if (!s || n_steps < 0 || (n_steps && !u)) return err(FRT_EINVAL, "bad rotations");
    return FRT_OK;
}

int frt_sync(frt_solve s) { return s ? FRT_OK : err(FRT_EINVAL, "null solve"); }

int frt_batch_step(frt_solve* ss, int n, const double* dts)
{
    if (!ss || n < 1 || n > FRT_MAX_SOLVES_PER_LAUNCH || !dts) return err(FRT_EINVAL, "bad batch");
    uint64_t need = 0, cells = 0;
    for (int i = 0; i < n; i++) {
        frt_solve s = ss[i];
        if (!s || !s->grid || s->n_src < 0) return err(FRT_ESTATE, "solve not loaded");
        if (s->ctx != ss[0]->ctx || s->P.n_bins != ss[0]->P.n_bins || s->P.march_precision != ss[0]->P.march_precision ||
            (s->P.queue_capacity == 0) != (ss[0]->P.queue_capacity == 0))
            return err(FRT_EINVAL, "the solves of a batch must share context, n_bins, precision and queue mode");
        if (!(dts[i] > 0)) return err(FRT_EINVAL, "dt must be > 0");
        need += ncell(s) * fake::pass_bytes_per_cell();
        cells += ncell(s);
    }
    frt_ctx ctx = ss[0]->ctx;
    {
        std::unique_lock<std::mutex> lock(g_mu);
        g_release.wait(lock, [] { return !g_hold_steps; });
        const fake::Faults& f = g_faults;
        need *= (uint64_t)f.pass_growth;
        for (int i = 0; i < n; i++)
            if (f.step_fail_code != 0 && ss[i]->tag == f.step_fail_tag && (int64_t)ss[i]->steps == f.step_fail_step)
                return err(f.step_fail_code, "injected: step failure");
        if (ctx->ws_limit && need > ctx->ws_limit) return err(FRT_ENOMEM, "pass queues would exceed the limit");
        if (need > ctx->ws_bytes) ctx->ws_bytes = need;
        g_batches++;
        if ((uint64_t)n > g_max_batch) g_max_batch = (uint64_t)n;
    }
    for (int i = 0; i < n; i++) ss[i]->steps++;
    tick(20000 + (int64_t)(0.5 * (double)cells));
    std::this_thread::yield();
    return FRT_OK;
}

int frt_read_fields(frt_solve s, double* x, float* gamma, int ptr_kind)
{
    if (!s || ptr_kind != FRT_HOST) return err(FRT_EINVAL, "bad read");
    const uint64_t n = ncell(s);
    if (x)
        for (uint64_t i = 0; i < n; i++) x[i] = value(s->tag, s->steps, i);
    if (gamma)
        for (uint64_t i = 0; i < n; i++) gamma[i] = 0.0f;
    return FRT_OK;
}

int frt_read_temperature(frt_solve s, double* T, int ptr_kind)
{
    if (!s || !T || ptr_kind != FRT_HOST) return err(FRT_EINVAL, "bad temperature read");
    if (!s->P.temperature) return err(FRT_ESTATE, "the solve holds no temperature");
    const uint64_t n = ncell(s);
    for (uint64_t i = 0; i < n; i++) T[i] = fake::expected_T(s->tag, s->steps, i);
    return FRT_OK;
}

int frt_read_ledger(frt_solve s, frt_ledger* out)
{
    if (!s || !out) return err(FRT_EINVAL, "bad ledger read");
    std::memset(out, 0, sizeof(*out));
    out->steps = s->steps;
    return FRT_OK;
}

}  // extern "C"

namespace frt {

int set_error(int code, const char* msg) { return err(code, msg); }

int ctx_device(frt_ctx ctx) { return ctx->device; }

uint64_t solve_bytes(const frt_params&, uint64_t n, int n_src, int, uint64_t* pass_records, uint64_t* pass_bytes)
{
    const uint64_t pass = n * fake::pass_bytes_per_cell();
    if (pass_records) *pass_records = n / 2;
    if (pass_bytes) *pass_bytes = pass;
    return n * fake::cell_bytes() + (uint64_t)(n_src > 0 ? n_src : 0) * 64 + pass;
}

uint64_t ctx_workspace_bytes(frt_ctx ctx)
{
    std::lock_guard<std::mutex> lock(g_mu);
    return ctx->ws_bytes;
}

void ctx_set_workspace_limit(frt_ctx ctx, uint64_t bytes)
{
    std::lock_guard<std::mutex> lock(g_mu);
    ctx->ws_limit = bytes;
}

void ctx_trim_workspace(frt_ctx ctx)
{
    std::lock_guard<std::mutex> lock(g_mu);
    ctx->ws_bytes = 0;
}

int use_device(int) { return FRT_OK; }

int copy_device_to_host(void*, const void*, size_t) { return err(FRT_EINVAL, "no device memory in the CPU stand-in"); }

double clock_s() { return 1e-9 * (double)g_clock_ns.load(); }

}  // namespace frt
