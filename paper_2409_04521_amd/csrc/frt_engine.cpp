// Host engine of the ray-tracing library: resident per-solve buffers in HBM,
// step orchestration (casting, march rounds, chemistry, bookkeeping),
// batches of solves, checkpoints and the C ABI declared in include/frt.h.
#include "frt.h"
#include "frt_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

struct frt_ctx_s {
    int device;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(FRT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

uint64_t mix64_host(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr double PI = 3.14159265358979323846;

}  // namespace

struct frt_solve_s {
    frt_ctx ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    frt_params P{};
    int fp64 = 0;
    size_t rs = 4;                     // bytes of one Real
    // grid
    bool have_grid = false, have_src = false;
    int nx = 0, ny = 0, nz = 0;
    double dx = 0;
    size_t ncell = 0;
    bool any_kappa = false;
    // descriptor
    FrtSolveDesc h{};
    FrtSolveDesc* d_desc = nullptr;
    // buffers
    void* op = nullptr;
    void* gam[2] = {nullptr, nullptr};
    double* x = nullptr;
    double* nH = nullptr;
    float* T = nullptr;
    double* src_pos = nullptr;
    float* spec = nullptr;
    double* specd = nullptr;
    double* quat = nullptr;
    uint32_t quat_steps = 0;
    double* user_u = nullptr;
    uint32_t user_steps = 0;
    int n_src = 0;
    uint32_t cap[FRT_NQ] = {0, 0, 0, 0};
    uint32_t* count = nullptr;
    FrtLedgerDev* L = nullptr;
    FrtLedgerDev* L_snap = nullptr;
    uint32_t* count_snap = nullptr;
    uint32_t* emit_prefix = nullptr;
    unsigned long long* cell_prefix = nullptr;
    FrtRoundPlan* plan = nullptr;
    uint32_t step = 0;
    int rounds = 1;
    double last_dt = 0;
    std::vector<double> host_uniforms;  // user table kept for checkpoints

    ~frt_solve_s() { release_all(); }

    void release_queue(int k)
    {
        FrtQueue& q = h.q[k];
        void* ptrs[] = {q.src, q.estep, q.lp, q.r, q.rstop, q.w0, q.tau, q.comp};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        q = FrtQueue{};
        cap[k] = 0;
    }

    void release_all()
    {
        for (int k = 0; k < FRT_NQ; k++) release_queue(k);
        void* ptrs[] = {d_desc, op, gam[0], gam[1], x, nH, T, src_pos, spec, specd, quat, user_u,
                        count, L, L_snap, count_snap, emit_prefix, cell_prefix, plan};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        d_desc = nullptr; op = nullptr; gam[0] = gam[1] = nullptr; x = nullptr; nH = nullptr; T = nullptr;
        src_pos = nullptr; spec = nullptr; specd = nullptr; quat = nullptr; user_u = nullptr; count = nullptr;
        L = nullptr; L_snap = nullptr; count_snap = nullptr; emit_prefix = nullptr; cell_prefix = nullptr;
        plan = nullptr;
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
};

namespace {

int dev_alloc(void** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(FRT_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    return FRT_OK;
}

// Allocate one SoA queue of `cap` entries; if `keep` entries of the old
// queue are to be preserved, copy them over.
int alloc_queue(frt_solve s, int k, uint32_t capn, uint32_t keep)
{
    FrtQueue nq{};
    nq.cap = capn;
    const int nb = s->P.n_bins;
    const size_t n = std::max<uint32_t>(capn, 1);
    int rc;
    if ((rc = dev_alloc((void**)&nq.src, n * 4)) || (rc = dev_alloc((void**)&nq.estep, n * 4)) ||
        (rc = dev_alloc((void**)&nq.lp, n * 4)) || (rc = dev_alloc(&nq.r, n * s->rs)) ||
        (rc = dev_alloc(&nq.rstop, n * s->rs)) || (rc = dev_alloc(&nq.w0, n * s->rs)) ||
        (rc = dev_alloc(&nq.tau, n * s->rs * nb)) || (rc = dev_alloc(&nq.comp, n * s->rs * nb))) {
        void* ptrs[] = {nq.src, nq.estep, nq.lp, nq.r, nq.rstop, nq.w0, nq.tau, nq.comp};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        return rc;
    }
    FrtQueue& oq = s->h.q[k];
    if (keep > 0 && oq.src) {
        keep = std::min(keep, oq.cap);
        HIPCHK(hipMemcpyAsync(nq.src, oq.src, keep * 4ull, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(nq.estep, oq.estep, keep * 4ull, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(nq.lp, oq.lp, keep * 4ull, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(nq.r, oq.r, keep * s->rs, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(nq.rstop, oq.rstop, keep * s->rs, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(nq.w0, oq.w0, keep * s->rs, hipMemcpyDeviceToDevice, s->stream));
        for (int b = 0; b < nb; b++) {
            HIPCHK(hipMemcpyAsync((char*)nq.tau + b * (size_t)capn * s->rs, (char*)oq.tau + b * (size_t)oq.cap * s->rs,
                                  keep * s->rs, hipMemcpyDeviceToDevice, s->stream));
            HIPCHK(hipMemcpyAsync((char*)nq.comp + b * (size_t)capn * s->rs, (char*)oq.comp + b * (size_t)oq.cap * s->rs,
                                  keep * s->rs, hipMemcpyDeviceToDevice, s->stream));
        }
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    s->release_queue(k);
    s->h.q[k] = nq;
    s->cap[k] = capn;
    return FRT_OK;
}

double split_radius_cells(const frt_params& P, int level)
{
    return std::ldexp(std::sqrt(3.0 / (PI * P.n_ray_min)), level);
}

// Number of march rounds a step needs: a packet can split at most once per
// level it can still reach inside the box (or within the distance cap).
int rounds_needed(frt_solve s)
{
    const double diag = std::sqrt((double)s->nx * s->nx + (double)s->ny * s->ny + (double)s->nz * s->nz);
    double reach = diag;
    if (s->P.max_distance_cm > 0) reach = std::min(reach, s->P.max_distance_cm / s->dx);
    int l = s->P.base_level;
    while (l < s->P.max_level && split_radius_cells(s->P, l) < reach) l++;
    return l - s->P.base_level + 1;
}

// Initial queue sizes.  Split parents at level l sit at r_split(l) where each
// covers dx^2 / N_min of the sphere; the part of that sphere inside the box
// has at most the box's surface area, so a source contributes at most
// min(12 4^l, N_min * 1.25 * surface) parents per round.
void initial_caps(frt_solve s, uint64_t* capF, uint64_t* capS)
{
    const double surf = 2.0 * ((double)s->nx * s->ny + (double)s->ny * s->nz + (double)s->nx * s->nz);
    const uint64_t ncast = 12ull << (2 * s->P.base_level);
    const double per_src_area = s->P.n_ray_min * 1.25 * surf + 64.0;
    double maxS = 0;
    for (int l = s->P.base_level; l < s->P.base_level + s->rounds - 1; l++) {
        double nl = std::min(std::ldexp(12.0, 2 * l), per_src_area);
        maxS = std::max(maxS, nl);
    }
    double S = maxS * s->n_src;
    double F = (double)ncast * s->n_src;
    if (std::isfinite(s->P.c_ray_cm_s)) F += std::min(per_src_area * s->n_src, 4.0 * (double)s->ncell);
    S = std::min(S, std::max(4.0 * (double)s->ncell, 4.0 * (double)ncast * s->n_src));
    const double lim = 2147483647.0;
    *capF = (uint64_t)std::min(lim, F + 1024);
    *capS = (uint64_t)std::min(lim, S + 1024);
    if (s->P.queue_capacity) {
        *capF = std::max<uint64_t>(*capF > s->P.queue_capacity ? s->P.queue_capacity : *capF, ncast * s->n_src + 1);
        *capS = s->P.queue_capacity;
    }
}

int ensure_quat(frt_solve s, uint32_t step)
{
    if (step < s->quat_steps) return FRT_OK;
    uint32_t nsteps = std::max<uint32_t>(step + 1, std::max<uint32_t>(64, 2 * s->quat_steps));
    double* nq = nullptr;
    int rc = dev_alloc((void**)&nq, (size_t)nsteps * std::max(1, s->n_src) * 4 * sizeof(double));
    if (rc) return rc;
    if (s->quat && s->quat_steps) {
        HIPCHK(hipMemcpyAsync(nq, s->quat, (size_t)s->quat_steps * s->n_src * 4 * sizeof(double),
                              hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        (void)hipFree(s->quat);
    }
    s->quat = nq;
    s->quat_steps = nsteps;
    s->h.quat = nq;
    s->h.quat_steps = nsteps;
    return FRT_OK;
}

// Per-step block of the descriptor.
void set_step_fields(frt_solve s, double dt)
{
    FrtSolveDesc& h = s->h;
    h.step = s->step;
    h.cur = s->step & 1u;
    h.dt = dt;
    h.budget = std::isfinite(s->P.c_ray_cm_s) ? s->P.c_ray_cm_s * dt / s->dx : HUGE_VAL;
    h.w0_cast = dt / (double)(12ull << (2 * s->P.base_level));
    for (int b = 0; b < FRT_MAX_BINS_I; b++) {
        double kb = b < s->P.n_bins ? h.R_ref * s->P.sigma_bins[b] / (s->dx * s->dx * dt) : 0.0;
        h.Kd[b] = kb;
        h.K[b] = (float)kb;
    }
}

int check_inputs_finite(const float* v, size_t n, const char* what)
{
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(v[i]) || v[i] < 0.f) return fail(FRT_EINVAL, "%s[%zu] = %g is negative or not finite", what, i, (double)v[i]);
    return FRT_OK;
}

int copy_in(void* dst, const void* src, size_t bytes, int kind, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, kind == FRT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    return FRT_OK;
}

// Host view of an input that may live on the device.
template <typename T>
int host_view(const T* p, size_t n, int kind, std::vector<T>& buf, const T** out)
{
    if (kind == FRT_HOST) {
        *out = p;
        return FRT_OK;
    }
    buf.resize(n);
    HIPCHK(hipMemcpy(buf.data(), p, n * sizeof(T), hipMemcpyDeviceToHost));
    *out = buf.data();
    return FRT_OK;
}

int upload_desc(frt_solve s)
{
    HIPCHK(hipMemcpyAsync(s->d_desc, &s->h, sizeof(FrtSolveDesc), hipMemcpyHostToDevice, s->stream));
    return FRT_OK;
}

int read_device_ledger(frt_solve s, FrtLedgerDev* out)
{
    HIPCHK(hipMemcpyAsync(out, s->L, sizeof(FrtLedgerDev), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

// Enqueue one step for a set of solves that share n_bins and precision.
// `d_descs` holds their descriptors contiguously on the device.
int enqueue_steps(frt_solve* ss, int n, FrtSolveDesc* d_descs, uint32_t* d_emit_prefix,
                  unsigned long long* d_cell_prefix, FrtRoundPlan* d_plan, hipStream_t st)
{
    const int nb = ss[0]->P.n_bins, fp64 = ss[0]->fp64;
    uint32_t emit_total = 0;
    unsigned long long cells = 0;
    int rounds = 1;
    for (int i = 0; i < n; i++) {
        emit_total += (uint32_t)ss[i]->n_src * (12u << (2 * ss[i]->P.base_level));
        cells += ss[i]->ncell;
        rounds = std::max(rounds, ss[i]->rounds);
    }
    hipError_t e;
    if ((e = frt::launch_emit(d_descs, d_emit_prefix, n, emit_total, fp64, st)) != hipSuccess)
        return fail(FRT_EDEVICE, "emit launch: %s", hipGetErrorString(e));
    for (int r = 0; r < rounds; r++) {
        if ((e = frt::launch_round(d_descs, d_plan, n, r, fp64, st)) != hipSuccess)
            return fail(FRT_EDEVICE, "plan launch: %s", hipGetErrorString(e));
        if ((e = frt::launch_round_march(d_descs, d_plan, r, nb, fp64, st)) != hipSuccess)
            return fail(FRT_EDEVICE, "march launch: %s", hipGetErrorString(e));
    }
    if ((e = frt::launch_chem(d_descs, d_cell_prefix, n, cells, fp64, st)) != hipSuccess)
        return fail(FRT_EDEVICE, "chem launch: %s", hipGetErrorString(e));
    if ((e = frt::launch_step_end(d_descs, n, st)) != hipSuccess)
        return fail(FRT_EDEVICE, "step-end launch: %s", hipGetErrorString(e));
    return FRT_OK;
}

int ready(frt_solve s)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid || !s->have_src) return fail(FRT_ESTATE, "load the grid and the sources before stepping");
    return FRT_OK;
}

}  // namespace

// =====================================================================  ABI
extern "C" {

const char* frt_last_error(void) { return g_err.c_str(); }

int frt_params_default(frt_params* p)
{
    if (!p) return fail(FRT_EINVAL, "null params");
    std::memset(p, 0, sizeof(*p));
    p->size = sizeof(frt_params);
    p->n_bins = 1;
    p->sigma_bins[0] = 6.3e-18;
    p->alpha_B = 2.59e-13;
    p->coll_ion = 0.0;
    p->base_level = 0;
    p->max_level = 12;
    p->n_ray_min = 1.0;
    p->flux_floor = 0.0;
    p->max_distance_cm = 0.0;
    p->c_ray_cm_s = 2.99792458e10;
    p->march_precision = FRT_F32;
    p->seed = 0;
    p->queue_capacity = 0;
    return FRT_OK;
}

int frt_ctx_create(int hip_device, frt_ctx* out)
{
    if (!out) return fail(FRT_EINVAL, "null output");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(FRT_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= n) return fail(FRT_EINVAL, "device %d out of range [0,%d)", hip_device, n);
    HIPCHK(hipSetDevice(hip_device));
    frt_ctx c = new (std::nothrow) frt_ctx_s;
    if (!c) return fail(FRT_ENOMEM, "context");
    c->device = hip_device;
    *out = c;
    return FRT_OK;
}

int frt_ctx_destroy(frt_ctx ctx)
{
    delete ctx;
    return FRT_OK;
}

int frt_solve_create(frt_ctx ctx, const frt_params* P, void* hip_stream, frt_solve* out)
{
    if (!ctx || !P || !out) return fail(FRT_EINVAL, "null argument");
    if (P->size != sizeof(frt_params)) return fail(FRT_EINVAL, "frt_params.size = %zu, expected %zu", P->size, sizeof(frt_params));
    if (P->n_bins < 1 || P->n_bins > FRT_MAX_BINS) return fail(FRT_EINVAL, "n_bins = %d outside 1..%d", P->n_bins, FRT_MAX_BINS);
    for (int b = 0; b < P->n_bins; b++)
        if (!(P->sigma_bins[b] > 0) || !std::isfinite(P->sigma_bins[b])) return fail(FRT_EINVAL, "sigma_bins[%d] must be finite and > 0", b);
    if (P->base_level < 0 || P->base_level > 8) return fail(FRT_EINVAL, "base_level %d outside 0..8", P->base_level);
    if (P->max_level < P->base_level || P->max_level > 13) return fail(FRT_EINVAL, "max_level %d outside base_level..13", P->max_level);
    if (!(P->n_ray_min > 0) || !std::isfinite(P->n_ray_min)) return fail(FRT_EINVAL, "n_ray_min must be finite and > 0");
    if (!(P->alpha_B >= 0) || !(P->coll_ion >= 0) || !std::isfinite(P->alpha_B) || !std::isfinite(P->coll_ion))
        return fail(FRT_EINVAL, "alpha_B and coll_ion must be finite and >= 0");
    if (!(P->flux_floor >= 0 && P->flux_floor < 1)) return fail(FRT_EINVAL, "flux_floor must lie in [0,1)");
    if (!(P->max_distance_cm >= 0) || !std::isfinite(P->max_distance_cm)) return fail(FRT_EINVAL, "max_distance_cm must be finite and >= 0");
    if (!(P->c_ray_cm_s > 0)) return fail(FRT_EINVAL, "c_ray_cm_s must be > 0 (or +inf)");
    if (P->march_precision != FRT_F32 && P->march_precision != FRT_F64) return fail(FRT_EINVAL, "march_precision must be FRT_F32 or FRT_F64");
    HIPCHK(hipSetDevice(ctx->device));
    frt_solve s = new (std::nothrow) frt_solve_s;
    if (!s) return fail(FRT_ENOMEM, "solve");
    s->ctx = ctx;
    s->P = *P;
    s->fp64 = P->march_precision == FRT_F64;
    s->rs = s->fp64 ? 8 : 4;
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return fail(FRT_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        s->own_stream = true;
    }
    int rc;
    if ((rc = dev_alloc((void**)&s->d_desc, sizeof(FrtSolveDesc))) || (rc = dev_alloc((void**)&s->count, FRT_NQ * 4)) ||
        (rc = dev_alloc((void**)&s->L, sizeof(FrtLedgerDev))) || (rc = dev_alloc((void**)&s->L_snap, sizeof(FrtLedgerDev))) ||
        (rc = dev_alloc((void**)&s->count_snap, FRT_NQ * 4)) || (rc = dev_alloc((void**)&s->emit_prefix, 2 * 4)) ||
        (rc = dev_alloc((void**)&s->cell_prefix, 2 * 8)) || (rc = dev_alloc((void**)&s->plan, sizeof(FrtRoundPlan)))) {
        delete s;
        return rc;
    }
    HIPCHK(hipMemsetAsync(s->count, 0, FRT_NQ * 4, s->stream));
    HIPCHK(hipMemsetAsync(s->L, 0, sizeof(FrtLedgerDev), s->stream));
    FrtSolveDesc& h = s->h;
    std::memset(&h, 0, sizeof(h));
    h.n_bins = P->n_bins;
    h.base_level = P->base_level;
    h.max_level = P->max_level;
    h.fp64 = s->fp64;
    h.sigma0 = P->sigma_bins[0];
    for (int b = 0; b < P->n_bins; b++) h.sig_rel[b] = (float)(P->sigma_bins[b] / P->sigma_bins[0]);
    h.r_split0 = std::sqrt(3.0 / (PI * P->n_ray_min));
    h.floor = (float)P->flux_floor;
    h.alpha_B = P->alpha_B;
    h.coll_ion = P->coll_ion;
    h.seed = P->seed;
    h.count = s->count;
    h.L = s->L;
    *out = s;
    return FRT_OK;
}

int frt_solve_destroy(frt_solve s)
{
    if (!s) return FRT_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    delete s;
    return FRT_OK;
}

int frt_load_grid(frt_solve s, int nx, int ny, int nz, double box_cm, const float* n_H, const float* T,
                  const float* kappa, const double* x0, int kind)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 2048 || ny > 2048 || nz > 2048) return fail(FRT_EINVAL, "grid %dx%dx%d outside 1..2048", nx, ny, nz);
    if (!(box_cm > 0) || !std::isfinite(box_cm)) return fail(FRT_EINVAL, "box_cm must be finite and > 0");
    if (!n_H) return fail(FRT_EINVAL, "n_H is required");
    if (kind != FRT_HOST && kind != FRT_DEVICE) return fail(FRT_EINVAL, "ptr_kind must be FRT_HOST or FRT_DEVICE");
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    const size_t n = (size_t)nx * ny * nz;
    std::vector<float> bn, bk;
    std::vector<double> bx;
    const float *hn = nullptr, *hk = nullptr;
    const double* hx = nullptr;
    int rc;
    if ((rc = host_view(n_H, n, kind, bn, &hn))) return rc;
    if ((rc = check_inputs_finite(hn, n, "n_H"))) return rc;
    if (kappa) {
        if ((rc = host_view(kappa, n, kind, bk, &hk))) return rc;
        if ((rc = check_inputs_finite(hk, n, "kappa_sub"))) return rc;
    }
    if (x0) {
        if ((rc = host_view(x0, n, kind, bx, &hx))) return rc;
        for (size_t i = 0; i < n; i++)
            if (!(hx[i] >= 0.0 && hx[i] <= 1.0)) return fail(FRT_EINVAL, "x_HI0[%zu] = %g outside [0,1]", i, hx[i]);
    }
    // (re)allocate grid buffers
    void* ptrs[] = {s->op, s->gam[0], s->gam[1], s->x, s->nH, s->T};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    s->op = s->gam[0] = s->gam[1] = nullptr;
    s->x = s->nH = nullptr;
    s->T = nullptr;
    if ((rc = dev_alloc(&s->op, n * 2 * s->rs)) || (rc = dev_alloc(&s->gam[0], n * s->rs)) ||
        (rc = dev_alloc(&s->gam[1], n * s->rs)) || (rc = dev_alloc((void**)&s->x, n * 8)) ||
        (rc = dev_alloc((void**)&s->nH, n * 8)))
        return rc;
    if (T && (rc = dev_alloc((void**)&s->T, n * 4))) return rc;
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->ncell = n;
    s->dx = box_cm / nx;
    // host-side conversion: n_H to double, opacity pairs {0, kappa dx}
    std::vector<double> nHd(n), xd(n, 1.0);
    for (size_t i = 0; i < n; i++) nHd[i] = (double)hn[i];
    if (hx) std::copy(hx, hx + n, xd.begin());
    s->any_kappa = false;
    if (s->fp64) {
        std::vector<double> opv(2 * n);
        for (size_t i = 0; i < n; i++) {
            opv[2 * i] = 0.0;
            opv[2 * i + 1] = hk ? (double)hk[i] * s->dx : 0.0;
            s->any_kappa |= hk && hk[i] > 0;
        }
        HIPCHK(hipMemcpy(s->op, opv.data(), n * 16, hipMemcpyHostToDevice));
    } else {
        std::vector<float> opv(2 * n);
        for (size_t i = 0; i < n; i++) {
            opv[2 * i] = 0.f;
            opv[2 * i + 1] = hk ? (float)((double)hk[i] * s->dx) : 0.f;
            s->any_kappa |= hk && hk[i] > 0;
        }
        HIPCHK(hipMemcpy(s->op, opv.data(), n * 8, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(s->nH, nHd.data(), n * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->x, xd.data(), n * 8, hipMemcpyHostToDevice));
    if (T) {
        if ((rc = copy_in(s->T, T, n * 4, kind, s->stream))) return rc;
    }
    HIPCHK(hipMemsetAsync(s->gam[0], 0, n * s->rs, s->stream));
    HIPCHK(hipMemsetAsync(s->gam[1], 0, n * s->rs, s->stream));
    HIPCHK(hipMemsetAsync(s->count, 0, FRT_NQ * 4, s->stream));
    HIPCHK(hipMemsetAsync(s->L, 0, sizeof(FrtLedgerDev), s->stream));
    FrtSolveDesc& h = s->h;
    h.nx = nx; h.ny = ny; h.nz = nz;
    h.dx_cm = s->dx;
    h.r_cap = s->P.max_distance_cm > 0 ? s->P.max_distance_cm / s->dx : HUGE_VAL;
    h.op = s->op;
    h.op_w = s->op;
    h.gamma[0] = s->gam[0];
    h.gamma[1] = s->gam[1];
    h.x = s->x;
    h.nH = s->nH;
    s->step = 0;
    s->have_grid = true;
    s->have_src = false;   // sources are checked against the box
    if ((rc = upload_desc(s))) return rc;
    hipError_t e = frt::launch_prep_opacity(s->d_desc, n, s->fp64, s->stream);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "prep launch: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int frt_load_sources(frt_solve s, int n_src, const double* pos_cm, const double* ndot, int kind)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid) return fail(FRT_ESTATE, "load the grid before the sources");
    if (n_src < 0) return fail(FRT_EINVAL, "n_src < 0");
    if (n_src > 0 && (!pos_cm || !ndot)) return fail(FRT_EINVAL, "null source arrays");
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    const int nb = s->P.n_bins;
    std::vector<double> bp, bd;
    const double *hp = nullptr, *hd = nullptr;
    int rc;
    if (n_src > 0) {
        if ((rc = host_view(pos_cm, (size_t)n_src * 3, kind, bp, &hp))) return rc;
        if ((rc = host_view(ndot, (size_t)n_src * nb, kind, bd, &hd))) return rc;
    }
    const double ext[3] = {s->nx * s->dx, s->ny * s->dx, s->nz * s->dx};
    double rmax = 0.0;
    std::vector<double> pos_cells((size_t)std::max(1, n_src) * 3);
    for (int i = 0; i < n_src; i++) {
        for (int a = 0; a < 3; a++) {
            double v = hp[3 * i + a];
            if (!std::isfinite(v) || v < 0.0 || v > ext[a]) return fail(FRT_EINVAL, "source %d lies outside the box", i);
            pos_cells[3 * i + a] = v / s->dx;
        }
        for (int b = 0; b < nb; b++) {
            double v = hd[(size_t)i * nb + b];
            if (!std::isfinite(v) || v < 0.0) return fail(FRT_EINVAL, "ndot[%d][%d] = %g is negative or not finite", i, b, v);
            rmax = std::max(rmax, v);
        }
    }
    const uint64_t ncast = 12ull << (2 * s->P.base_level);
    if ((uint64_t)n_src * ncast > 0x7fffffffull) return fail(FRT_EINVAL, "too many cast packets per step");
    const double R_ref = rmax > 0 ? rmax : 1.0;
    std::vector<float> spec((size_t)std::max(1, n_src) * nb);
    std::vector<double> specd((size_t)std::max(1, n_src) * nb);
    for (size_t i = 0; i < (size_t)n_src * nb; i++) {
        specd[i] = hd[i] / R_ref;
        spec[i] = (float)specd[i];
    }
    void* ptrs[] = {s->src_pos, s->spec, s->specd, s->quat, s->user_u};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    s->src_pos = nullptr; s->spec = nullptr; s->specd = nullptr; s->quat = nullptr; s->user_u = nullptr;
    s->quat_steps = 0;
    s->user_steps = 0;
    s->host_uniforms.clear();
    s->n_src = n_src;
    if ((rc = dev_alloc((void**)&s->src_pos, pos_cells.size() * 8)) || (rc = dev_alloc((void**)&s->spec, spec.size() * 4)) ||
        (rc = dev_alloc((void**)&s->specd, specd.size() * 8)))
        return rc;
    HIPCHK(hipMemcpy(s->src_pos, pos_cells.data(), pos_cells.size() * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->spec, spec.data(), spec.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->specd, specd.data(), specd.size() * 8, hipMemcpyHostToDevice));
    FrtSolveDesc& h = s->h;
    h.n_src = n_src;
    h.R_ref = R_ref;
    h.src_pos = s->src_pos;
    h.spec = s->spec;
    h.specd = s->specd;
    h.user_u = nullptr;
    h.user_steps = 0;
    s->rounds = rounds_needed(s);
    uint64_t capF, capS;
    initial_caps(s, &capF, &capS);
    for (int k = 0; k < FRT_NQ; k++) s->release_queue(k);
    if ((rc = alloc_queue(s, FRT_QF0, (uint32_t)capF, 0)) || (rc = alloc_queue(s, FRT_QF1, (uint32_t)capF, 0)) ||
        (rc = alloc_queue(s, FRT_QS0, (uint32_t)capS, 0)) || (rc = alloc_queue(s, FRT_QS1, (uint32_t)capS, 0)))
        return rc;
    if ((rc = ensure_quat(s, 0))) return rc;
    uint32_t ep[2] = {0, (uint32_t)(n_src * ncast)};
    unsigned long long cp[2] = {0, (unsigned long long)s->ncell};
    HIPCHK(hipMemcpy(s->emit_prefix, ep, sizeof(ep), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->cell_prefix, cp, sizeof(cp), hipMemcpyHostToDevice));
    HIPCHK(hipMemsetAsync(s->count, 0, FRT_NQ * 4, s->stream));
    HIPCHK(hipMemsetAsync(s->L, 0, sizeof(FrtLedgerDev), s->stream));
    s->step = 0;
    s->have_src = true;
    if ((rc = upload_desc(s))) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int frt_set_rotations(frt_solve s, int n_steps, const double* u)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_src) return fail(FRT_ESTATE, "load the sources before the rotation table");
    if (n_steps < 0 || (n_steps > 0 && !u)) return fail(FRT_EINVAL, "bad rotation table");
    const size_t n = (size_t)n_steps * s->n_src * 3;
    for (size_t i = 0; i < n; i++)
        if (!(u[i] >= 0.0 && u[i] < 1.0)) return fail(FRT_EINVAL, "uniform %zu = %g outside [0,1)", i, u[i]);
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->user_u) (void)hipFree(s->user_u);
    s->user_u = nullptr;
    int rc;
    if ((rc = dev_alloc((void**)&s->user_u, std::max<size_t>(n, 1) * 8))) return rc;
    if (n) HIPCHK(hipMemcpy(s->user_u, u, n * 8, hipMemcpyHostToDevice));
    s->user_steps = (uint32_t)n_steps;
    s->host_uniforms.assign(u, u + n);
    s->h.user_u = s->user_u;
    s->h.user_steps = s->user_steps;
    return upload_desc(s);
}

static int step_group(frt_solve* ss, int n, const double* dts, FrtSolveDesc* d_descs, uint32_t* d_ep,
                      unsigned long long* d_cp, FrtRoundPlan* d_plan, hipStream_t st, bool single)
{
    for (int i = 0; i < n; i++) {
        frt_solve s = ss[i];
        int rc;
        if ((rc = ensure_quat(s, s->step))) return rc;
        set_step_fields(s, dts[i]);
        s->last_dt = dts[i];
        if (single && (rc = upload_desc(s))) return rc;
    }
    return enqueue_steps(ss, n, d_descs, d_ep, d_cp, d_plan, st);
}

int frt_step(frt_solve s, double dt)
{
    int rc;
    if ((rc = ready(s))) return rc;
    if (!(dt > 0) || !std::isfinite(dt)) return fail(FRT_EINVAL, "dt must be finite and > 0");
    HIPCHK(hipSetDevice(s->ctx->device));
    const bool auto_grow = s->P.queue_capacity == 0;
    for (int attempt = 0; attempt < 12; attempt++) {
        if (auto_grow) {
            HIPCHK(hipMemcpyAsync(s->L_snap, s->L, sizeof(FrtLedgerDev), hipMemcpyDeviceToDevice, s->stream));
            HIPCHK(hipMemcpyAsync(s->count_snap, s->count, FRT_NQ * 4, hipMemcpyDeviceToDevice, s->stream));
        }
        if ((rc = step_group(&s, 1, &dt, s->d_desc, s->emit_prefix, s->cell_prefix, s->plan, s->stream, true))) return rc;
        if (!auto_grow) {
            s->step++;
            return FRT_OK;
        }
        FrtLedgerDev L;
        if ((rc = read_device_ledger(s, &L))) return rc;
        if (!(L.err_flags & FRT_DEVERR_QUEUE_OVERFLOW)) {
            s->step++;
            return FRT_OK;
        }
        // overflow: restore the step's starting state, enlarge, re-run
        uint32_t counts[FRT_NQ];
        HIPCHK(hipMemcpy(counts, s->count, sizeof(counts), hipMemcpyDeviceToHost));
        uint32_t keep;
        HIPCHK(hipMemcpy(&keep, s->count_snap + (s->step & 1u), 4, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(s->L, s->L_snap, sizeof(FrtLedgerDev), hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(s->count, s->count_snap, FRT_NQ * 4, hipMemcpyDeviceToDevice));
        HIPCHK(hipMemset(s->gam[s->step & 1u], 0, s->ncell * s->rs));
        const uint64_t lim = 2147483647ull;
        uint64_t needF = std::max<uint64_t>(2ull * s->cap[FRT_QF0], (uint64_t)std::max(counts[0], counts[1]) + 1024);
        uint64_t needS = std::max<uint64_t>(2ull * s->cap[FRT_QS0], (uint64_t)std::max(counts[2], counts[3]) + 1024);
        const uint64_t nF = std::min(lim, needF), nS = std::min(lim, needS);
        if ((uint64_t)s->cap[FRT_QF0] >= lim && (uint64_t)s->cap[FRT_QS0] >= lim)
            return fail(FRT_EOVERFLOW, "ray queues at their maximum size still overflow");
        const int cur = (int)(s->step & 1u);
        if ((rc = alloc_queue(s, cur, (uint32_t)nF, keep)) || (rc = alloc_queue(s, 1 - cur, (uint32_t)nF, 0)) ||
            (rc = alloc_queue(s, FRT_QS0, (uint32_t)nS, 0)) || (rc = alloc_queue(s, FRT_QS1, (uint32_t)nS, 0)))
            return rc == FRT_ENOMEM ? fail(FRT_EOVERFLOW, "ray queues could not grow: %s", g_err.c_str()) : rc;
        if ((rc = upload_desc(s))) return rc;
    }
    return fail(FRT_EOVERFLOW, "step kept overflowing its ray queues");
}

int frt_batch_step(frt_solve* ss, int n, const double* dts)
{
    if (!ss || n < 1 || !dts) return fail(FRT_EINVAL, "bad batch");
    if (n > FRT_MAX_SOLVES_PER_LAUNCH) return fail(FRT_EINVAL, "at most %d solves per batch", FRT_MAX_SOLVES_PER_LAUNCH);
    int rc;
    for (int i = 0; i < n; i++) {
        if ((rc = ready(ss[i]))) return rc;
        if (ss[i]->P.n_bins != ss[0]->P.n_bins || ss[i]->fp64 != ss[0]->fp64)
            return fail(FRT_EINVAL, "batched solves must share n_bins and march_precision");
        if (ss[i]->ctx->device != ss[0]->ctx->device) return fail(FRT_EINVAL, "batched solves must share a device");
        if (!(dts[i] > 0) || !std::isfinite(dts[i])) return fail(FRT_EINVAL, "dt must be finite and > 0");
        for (int j = 0; j < i; j++)
            if (ss[j] == ss[i]) return fail(FRT_EINVAL, "a solve appears twice in the batch");
    }
    hipStream_t st = ss[0]->stream;
    for (int i = 1; i < n; i++) HIPCHK(hipStreamSynchronize(ss[i]->stream));
    // batch-owned descriptor table and prefixes
    static thread_local FrtSolveDesc* d_descs = nullptr;
    static thread_local uint32_t* d_ep = nullptr;
    static thread_local unsigned long long* d_cp = nullptr;
    static thread_local FrtRoundPlan* d_plan = nullptr;
    static thread_local int cap_n = 0;
    if (cap_n < n) {
        if (d_descs) (void)hipFree(d_descs);
        if (d_ep) (void)hipFree(d_ep);
        if (d_cp) (void)hipFree(d_cp);
        if (d_plan) (void)hipFree(d_plan);
        d_descs = nullptr; d_ep = nullptr; d_cp = nullptr; d_plan = nullptr;
        int c = std::max(n, 64);
        if ((rc = dev_alloc((void**)&d_descs, c * sizeof(FrtSolveDesc))) || (rc = dev_alloc((void**)&d_ep, (c + 1) * 4)) ||
            (rc = dev_alloc((void**)&d_cp, (c + 1) * 8)) || (rc = dev_alloc((void**)&d_plan, sizeof(FrtRoundPlan)))) {
            cap_n = 0;
            return rc;
        }
        cap_n = c;
    }
    std::vector<FrtSolveDesc> hd(n);
    std::vector<uint32_t> ep(n + 1);
    std::vector<unsigned long long> cp(n + 1);
    ep[0] = 0;
    cp[0] = 0;
    for (int i = 0; i < n; i++) {
        frt_solve s = ss[i];
        if ((rc = ensure_quat(s, s->step))) return rc;
        set_step_fields(s, dts[i]);
        s->last_dt = dts[i];
        hd[i] = s->h;
        ep[i + 1] = ep[i] + (uint32_t)s->n_src * (12u << (2 * s->P.base_level));
        cp[i + 1] = cp[i] + s->ncell;
    }
    HIPCHK(hipMemcpyAsync(d_descs, hd.data(), n * sizeof(FrtSolveDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_ep, ep.data(), (n + 1) * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_cp, cp.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    if ((rc = enqueue_steps(ss, n, d_descs, d_ep, d_cp, d_plan, st))) return rc;
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < n; i++) {
        ss[i]->step++;
        if ((rc = upload_desc(ss[i]))) return rc;
    }
    return FRT_OK;
}

int frt_sync(frt_solve s)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    HIPCHK(hipStreamSynchronize(s->stream));
    if (!s->L) return FRT_OK;
    FrtLedgerDev L;
    int rc;
    if ((rc = read_device_ledger(s, &L))) return rc;
    if (L.err_flags & FRT_DEVERR_QUEUE_OVERFLOW) return fail(FRT_EOVERFLOW, "a ray queue overflowed; raise queue_capacity");
    return FRT_OK;
}

int frt_read_fields(frt_solve s, double* x_HI, float* gamma, int kind)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid) return fail(FRT_ESTATE, "no grid loaded");
    int rc;
    if ((rc = frt_sync(s)) && rc != FRT_EOVERFLOW) return rc;
    const size_t n = s->ncell;
    const hipMemcpyKind k = kind == FRT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (x_HI) HIPCHK(hipMemcpy(x_HI, s->x, n * 8, k));
    if (gamma) {
        const void* g = s->gam[(s->step + 1u) & 1u];   // buffer of the last completed step
        if (s->step == 0) {
            if (kind == FRT_DEVICE) HIPCHK(hipMemset(gamma, 0, n * 4));
            else std::memset(gamma, 0, n * 4);
        } else if (!s->fp64) {
            HIPCHK(hipMemcpy(gamma, g, n * 4, k));
        } else {
            std::vector<double> tmp(n);
            HIPCHK(hipMemcpy(tmp.data(), g, n * 8, hipMemcpyDeviceToHost));
            std::vector<float> f(n);
            for (size_t i = 0; i < n; i++) f[i] = (float)tmp[i];
            HIPCHK(hipMemcpy(gamma, f.data(), n * 4, kind == FRT_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
        }
    }
    return FRT_OK;
}

int frt_read_ledger(frt_solve s, frt_ledger* out)
{
    if (!s || !out) return fail(FRT_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(s->stream));
    FrtLedgerDev L;
    int rc;
    if ((rc = read_device_ledger(s, &L))) return rc;
    out->emitted = L.emitted;
    out->absorbed_HI = L.absorbed_HI;
    out->absorbed_sub = L.absorbed_sub;
    out->escaped = L.escaped;
    out->dropped = L.dropped;
    out->in_flight = L.in_flight;
    out->lost = L.lost;
    out->crossings = L.crossings;
    out->ray_visits = L.ray_visits;
    out->splits = L.splits;
    out->n_escaped = L.n_escaped;
    out->n_dropped = L.n_dropped;
    out->n_in_flight = L.n_in_flight;
    out->rays_emitted = L.rays_emitted;
    out->step_crossings = L.step_crossings;
    out->steps = s->step;
    out->err_flags = L.err_flags;
    out->max_items = L.max_items;
    return FRT_OK;
}

// Checkpoint layout: magic, version, step, n_src, ncell, nb, fp64, n_carried,
// ledger, x[ncell], quaternions of the steps so far, carried packets (SoA).
int frt_save_state(frt_solve s, void* buf, size_t* bytes)
{
    int rc;
    if ((rc = ready(s))) return rc;
    if (!bytes) return fail(FRT_EINVAL, "null size");
    HIPCHK(hipStreamSynchronize(s->stream));
    uint32_t counts[FRT_NQ];
    HIPCHK(hipMemcpy(counts, s->count, sizeof(counts), hipMemcpyDeviceToHost));
    const int cur = (int)(s->step & 1u);
    const uint32_t nc = std::min(counts[cur], s->cap[cur]);
    const int nb = s->P.n_bins;
    const size_t rec = 12 + 3 * s->rs + 2 * nb * s->rs;
    const size_t nq = (size_t)s->step * s->n_src * 4;
    const size_t need = 8 * 8 + sizeof(FrtLedgerDev) + s->ncell * 8 + nq * 8 + (size_t)nc * rec;
    if (!buf) {
        *bytes = need;
        return FRT_OK;
    }
    if (*bytes < need) return fail(FRT_EINVAL, "checkpoint buffer too small (%zu < %zu)", *bytes, need);
    char* p = (char*)buf;
    uint64_t hdr[8] = {0x4652544350543031ull, 1, s->step, (uint64_t)s->n_src, s->ncell, (uint64_t)nb, (uint64_t)s->fp64, nc};
    std::memcpy(p, hdr, sizeof(hdr));
    p += sizeof(hdr);
    HIPCHK(hipMemcpy(p, s->L, sizeof(FrtLedgerDev), hipMemcpyDeviceToHost));
    p += sizeof(FrtLedgerDev);
    HIPCHK(hipMemcpy(p, s->x, s->ncell * 8, hipMemcpyDeviceToHost));
    p += s->ncell * 8;
    if (nq) HIPCHK(hipMemcpy(p, s->quat, nq * 8, hipMemcpyDeviceToHost));
    p += nq * 8;
    const FrtQueue& q = s->h.q[cur];
    if (nc) {
        HIPCHK(hipMemcpy(p, q.src, nc * 4ull, hipMemcpyDeviceToHost)); p += nc * 4ull;
        HIPCHK(hipMemcpy(p, q.estep, nc * 4ull, hipMemcpyDeviceToHost)); p += nc * 4ull;
        HIPCHK(hipMemcpy(p, q.lp, nc * 4ull, hipMemcpyDeviceToHost)); p += nc * 4ull;
        HIPCHK(hipMemcpy(p, q.r, nc * s->rs, hipMemcpyDeviceToHost)); p += nc * s->rs;
        HIPCHK(hipMemcpy(p, q.rstop, nc * s->rs, hipMemcpyDeviceToHost)); p += nc * s->rs;
        HIPCHK(hipMemcpy(p, q.w0, nc * s->rs, hipMemcpyDeviceToHost)); p += nc * s->rs;
        for (int b = 0; b < nb; b++) {
            HIPCHK(hipMemcpy(p, (char*)q.tau + b * (size_t)q.cap * s->rs, nc * s->rs, hipMemcpyDeviceToHost)); p += nc * s->rs;
        }
        for (int b = 0; b < nb; b++) {
            HIPCHK(hipMemcpy(p, (char*)q.comp + b * (size_t)q.cap * s->rs, nc * s->rs, hipMemcpyDeviceToHost)); p += nc * s->rs;
        }
    }
    *bytes = need;
    return FRT_OK;
}

int frt_load_state(frt_solve s, const void* buf, size_t bytes)
{
    int rc;
    if ((rc = ready(s))) return rc;
    if (!buf || bytes < 64 + sizeof(FrtLedgerDev)) return fail(FRT_EINVAL, "checkpoint too small");
    const char* p = (const char*)buf;
    uint64_t hdr[8];
    std::memcpy(hdr, p, sizeof(hdr));
    p += sizeof(hdr);
    if (hdr[0] != 0x4652544350543031ull || hdr[1] != 1) return fail(FRT_EINVAL, "not a checkpoint of this library");
    if (hdr[3] != (uint64_t)s->n_src || hdr[4] != s->ncell || hdr[5] != (uint64_t)s->P.n_bins || hdr[6] != (uint64_t)s->fp64)
        return fail(FRT_EINVAL, "checkpoint does not match this solve (sources, grid, bins or precision)");
    const uint32_t step = (uint32_t)hdr[2], nc = (uint32_t)hdr[7];
    const int nb = s->P.n_bins;
    const size_t rec = 12 + 3 * s->rs + 2 * nb * s->rs;
    const size_t nq = (size_t)step * s->n_src * 4;
    if (bytes < 64 + sizeof(FrtLedgerDev) + s->ncell * 8 + nq * 8 + (size_t)nc * rec) return fail(FRT_EINVAL, "checkpoint truncated");
    HIPCHK(hipStreamSynchronize(s->stream));
    HIPCHK(hipMemcpy(s->L, p, sizeof(FrtLedgerDev), hipMemcpyHostToDevice));
    p += sizeof(FrtLedgerDev);
    HIPCHK(hipMemcpy(s->x, p, s->ncell * 8, hipMemcpyHostToDevice));
    p += s->ncell * 8;
    if ((rc = ensure_quat(s, step))) return rc;
    if (nq) HIPCHK(hipMemcpy(s->quat, p, nq * 8, hipMemcpyHostToDevice));
    p += nq * 8;
    const int cur = (int)(step & 1u);
    if (nc > s->cap[cur]) {
        if ((rc = alloc_queue(s, cur, nc + 1024, 0)) || (rc = alloc_queue(s, 1 - cur, nc + 1024, 0))) return rc;
    }
    const FrtQueue& q = s->h.q[cur];
    if (nc) {
        HIPCHK(hipMemcpy(q.src, p, nc * 4ull, hipMemcpyHostToDevice)); p += nc * 4ull;
        HIPCHK(hipMemcpy(q.estep, p, nc * 4ull, hipMemcpyHostToDevice)); p += nc * 4ull;
        HIPCHK(hipMemcpy(q.lp, p, nc * 4ull, hipMemcpyHostToDevice)); p += nc * 4ull;
        HIPCHK(hipMemcpy(q.r, p, nc * s->rs, hipMemcpyHostToDevice)); p += nc * s->rs;
        HIPCHK(hipMemcpy(q.rstop, p, nc * s->rs, hipMemcpyHostToDevice)); p += nc * s->rs;
        HIPCHK(hipMemcpy(q.w0, p, nc * s->rs, hipMemcpyHostToDevice)); p += nc * s->rs;
        for (int b = 0; b < nb; b++) {
            HIPCHK(hipMemcpy((char*)q.tau + b * (size_t)q.cap * s->rs, p, nc * s->rs, hipMemcpyHostToDevice)); p += nc * s->rs;
        }
        for (int b = 0; b < nb; b++) {
            HIPCHK(hipMemcpy((char*)q.comp + b * (size_t)q.cap * s->rs, p, nc * s->rs, hipMemcpyHostToDevice)); p += nc * s->rs;
        }
    }
    uint32_t counts[FRT_NQ] = {0, 0, 0, 0};
    counts[cur] = nc;
    HIPCHK(hipMemcpy(s->count, counts, sizeof(counts), hipMemcpyHostToDevice));
    s->step = step;
    s->h.step = step;
    // rebuild the opacity from the restored neutral fraction; clear deposits
    HIPCHK(hipMemset(s->gam[0], 0, s->ncell * s->rs));
    HIPCHK(hipMemset(s->gam[1], 0, s->ncell * s->rs));
    if ((rc = upload_desc(s))) return rc;
    hipError_t e = frt::launch_prep_opacity(s->d_desc, s->ncell, s->fp64, s->stream);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "prep launch: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int frt_rotation_uniforms(uint64_t seed, uint32_t step, uint32_t src, double out[3])
{
    if (!out) return fail(FRT_EINVAL, "null output");
    for (uint32_t k = 0; k < 3; k++) {
        uint64_t ctr = ((uint64_t)step << 32) | ((uint64_t)src << 2) | (uint64_t)k;
        out[k] = (double)(mix64_host(ctr ^ mix64_host(seed)) >> 11) * 0x1.0p-53;
    }
    return FRT_OK;
}

}  // extern "C"
