// Host engine of the ray-tracing library: resident per-solve buffers in HBM,
// step orchestration (seeding, brick passes, chemistry, ledger folding),
// batches of solves, queue growth, checkpoints and the C ABI declared in
// include/frt.h.
#include "frt.h"
#include "frt_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

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

#define RCCHK(expr)            \
    do {                       \
        int rc_ = (expr);      \
        if (rc_) return rc_;   \
    } while (0)

uint64_t mix64_host(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr double PI = 3.14159265358979323846;

// Device memory comes from the allocator hooks of the context a library
// call works on (frt_ctx_create), else from hipMalloc.  Each entry point
// that allocates names its context with an AllocScope for the calling
// thread; every block remembers the hooks that gave it, so it goes back to
// them whichever call frees it.
struct Allocator {
    frt_alloc_fn alloc = nullptr;
    frt_free_fn release = nullptr;
    void* user = nullptr;
};

thread_local const Allocator* t_alloc = nullptr;

struct AllocScope {
    const Allocator* prev;
    explicit AllocScope(const Allocator* a) : prev(t_alloc) { t_alloc = a; }
    ~AllocScope() { t_alloc = prev; }
};

std::mutex g_hooked_mu;
std::unordered_map<void*, Allocator> g_hooked;   // blocks from allocator hooks

int dev_alloc(void** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (t_alloc && t_alloc->alloc) {
        void* q = t_alloc->alloc(bytes, t_alloc->user);
        if (!q) return fail(FRT_ENOMEM, "the context's allocator returned no memory for %zu bytes", bytes);
        std::lock_guard<std::mutex> lock(g_hooked_mu);
        g_hooked[q] = *t_alloc;
        *p = q;
        return FRT_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(FRT_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    return FRT_OK;
}

void dev_free_ptr(void* p)
{
    if (!p) return;
    Allocator a;
    bool hooked = false;
    {
        std::lock_guard<std::mutex> lock(g_hooked_mu);
        auto it = g_hooked.find(p);
        if (it != g_hooked.end()) {
            a = it->second;
            hooked = true;
            g_hooked.erase(it);
        }
    }
    if (hooked) a.release(p, a.user);
    else (void)hipFree(p);
}

template <typename T>
void dev_free(T*& p)
{
    dev_free_ptr((void*)p);
    p = nullptr;
}

// Bytes of one packet record.
size_t rec_bytes(size_t rs) { return rs == 8 ? sizeof(FrtRec<double>) : sizeof(FrtRec<float>); }

// Device bytes of the pass queues for `records` packets per pass and
// `nkeys` brick keys (at least 4096 are held): two output buffers with their
// keys, the sorted index and the work list (items of at least 64 packets,
// plus one per brick).
uint64_t pass_queue_bytes(uint64_t records, size_t rs, uint64_t nkeys)
{
    return records * (2 * rec_bytes(rs) + 2 * 4 + sizeof(uint2)) +
           (records / 64 + std::max<uint64_t>(nkeys, 4096) + 64) * sizeof(FrtWork);
}

void free_recs(FrtRecs& q)
{
    dev_free(q.rec);
    q.cap = 0;
}

int alloc_recs(FrtRecs& q, uint32_t cap, int nb, size_t rs)
{
    (void)nb;
    FrtRecs n{};
    n.cap = cap;
    RCCHK(dev_alloc(&n.rec, (size_t)std::max<uint32_t>(cap, 1) * rec_bytes(rs)));
    q = n;
    return FRT_OK;
}

// Copy the first n records of src into dst.
int copy_recs(FrtRecs& dst, const FrtRecs& src, uint32_t n, int nb, size_t rs, hipStream_t st, hipMemcpyKind k)
{
    (void)nb;
    if (!n) return FRT_OK;
    HIPCHK(hipMemcpyAsync(dst.rec, src.rec, (size_t)n * rec_bytes(rs), k, st));
    return FRT_OK;
}

}  // namespace

// Per-context pass workspace, shared by the solves stepped on the context
// (one step at a time: the mutex serializes launches that use it).
struct Workspace {
    int fp64 = -1, nb = 0;
    // pass outputs (two buffers used in turn, with each record's key) and
    // the sorted input index of a pass
    FrtRecs O[2] = {};
    uint32_t* okey[2] = {nullptr, nullptr};
    uint2* sorted = nullptr;
    uint32_t pcap = 0;              // records per output buffer and sorted entries
    FrtRecs X{};                    // march scratch records (split children kept in their brick)
    uint32_t* segc = nullptr;
    uint32_t* segp = nullptr;
    uint32_t* ctr_host = nullptr;   // pinned copy of the counters
    frt_tuning tune{sizeof(frt_tuning), (int)FRT_ITEM_RAYS, 8};
    uint32_t* ctr = nullptr;
    uint32_t* hist = nullptr;
    uint32_t* cursor = nullptr;
    uint32_t nkeys_cap = 0;
    FrtWork* work = nullptr;
    uint32_t cap_work = 0;
    uint32_t* key_prefix = nullptr;
    uint32_t* seed_prefix = nullptr;
    unsigned long long* cell_prefix = nullptr;
    FrtSolveDesc* descs = nullptr;
    int solves_cap = 0;
    uint64_t limit = 0;             // most device bytes the workspace may hold (0: no limit)
    // ray merging: per-packet keys, flags and scans, the output queue and the
    // sort storage, for up to mcap carried packets and mold table entries
    struct Merge {
        uint32_t mcap = 0, mold = 0;
        size_t rec = 0, temp_bytes = 0;
        void *pkey = nullptr, *pkey_sorted = nullptr, *temp = nullptr;
        unsigned long long *gkey = nullptr, *gkey_s = nullptr, *stats = nullptr;
        uint32_t *idx = nullptr, *idx_s = nullptr, *flag_out = nullptr, *slot = nullptr, *flag_lead = nullptr,
                 *gid = nullptr, *ref = nullptr, *vmap = nullptr, *counts = nullptr, *acc_head = nullptr;
        double* acc = nullptr;
        double* residual = nullptr;
    } mg;

    // device bytes of the pass queues (the part that grows with the largest
    // pass; the march scratch and the small tables are a fixed cost)
    uint64_t bytes() const
    {
        if (fp64 < 0) return 0;
        const size_t rs = fp64 ? 8 : 4;
        return (uint64_t)pcap * (2 * rec_bytes(rs) + 2 * 4 + sizeof(uint2)) + (uint64_t)cap_work * sizeof(FrtWork);
    }

    void free_pass()
    {
        for (int k = 0; k < 2; k++) {
            free_recs(O[k]);
            dev_free(okey[k]);
        }
        dev_free(sorted);
        pcap = 0;
    }

    void free_merge()
    {
        dev_free(mg.pkey); dev_free(mg.pkey_sorted); dev_free(mg.temp); dev_free(mg.gkey);
        dev_free(mg.gkey_s); dev_free(mg.stats); dev_free(mg.idx); dev_free(mg.idx_s); dev_free(mg.flag_out);
        dev_free(mg.slot); dev_free(mg.flag_lead); dev_free(mg.gid); dev_free(mg.ref); dev_free(mg.vmap);
        dev_free(mg.acc); dev_free(mg.acc_head);
        dev_free(mg.counts); dev_free(mg.residual);
        mg = Merge{};
    }

    void release()
    {
        free_pass();
        free_merge();
        free_recs(X);
        dev_free(segc);
        dev_free(segp);
        if (ctr_host) (void)hipHostFree(ctr_host);
        ctr_host = nullptr;
        dev_free(ctr); dev_free(hist); dev_free(cursor); dev_free(work); dev_free(key_prefix);
        dev_free(seed_prefix); dev_free(cell_prefix); dev_free(descs);
        nkeys_cap = 0; cap_work = 0; solves_cap = 0; fp64 = -1; nb = 0;
    }
};

struct frt_ctx_s {
    int device = 0;
    std::mutex mu;
    Allocator al;                   // device memory hooks (none: hipMalloc / hipFree)
    Workspace ws;
    ~frt_ctx_s()
    {
        AllocScope scope(&al);
        ws.release();
    }
};

struct frt_solve_s {
    frt_ctx ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    frt_params P{};
    int fp64 = 0;
    size_t rs = 4;
    int bsh[3] = {FRT_BRICK_LOG_SUB[0], FRT_BRICK_LOG_SUB[1], FRT_BRICK_LOG_SUB[2]};   // log2 brick edges
    bool have_grid = false, have_src = false;
    int nx = 0, ny = 0, nz = 0;
    int bpx = 0, bpy = 0, bpz = 0;
    double dx = 0;
    double nH_mean = 0;                      // the grid's mean n_H (the density update's Delta)
    double w0_max = 0;                       // largest w0 any held packet can have
    size_t ncell = 0;
    FrtSolveDesc h{};
    FrtSolveDesc* d_desc = nullptr;
    void* op = nullptr;
    void* gam[2] = {nullptr, nullptr};
    double* x = nullptr;
    double* xavg = nullptr;                  // time-averaged chemistry only
    double* front = nullptr;                 // Generalized Opacity Mode only
    double* nH = nullptr;
    double* T = nullptr;                     // temperature (loaded, or evolving), K
    void* heat = nullptr;                    // this step's photo-heating, eV (temperature on)
    double* mark_T = nullptr;                // bookmark of T (temperature on)
    double* src_pos = nullptr;
    float* spec = nullptr;
    double* specd = nullptr;
    double* quat = nullptr;
    uint32_t quat_steps = 0;
    double* user_u = nullptr;
    uint32_t user_steps = 0;
    int n_src = 0;
    FrtRecs F[2]{};
    FrtVSrc* vt[2] = {nullptr, nullptr};     // virtual origins of merged packets (merging only)
    uint32_t vt_cap[2] = {0, 0};
    uint32_t* vcount = nullptr;              // [2] entries of each table
    float* w0_merged = nullptr;              // largest w0 of a merged packet
    FrtVSrc* mark_vt = nullptr;              // bookmark of the table the carried packets refer to
    uint32_t mark_vn = 0;
    uint32_t* fcount = nullptr;
    uint32_t* fcount_snap = nullptr;
    FrtLedgerDev* L = nullptr;
    FrtLedgerDev* L_snap = nullptr;
    uint32_t step = 0;
    // bookmark for frt_mark / frt_rewind
    double* mark_x = nullptr;
    void* kin = nullptr;                     // Generalized Opacity Mode with K marches: the input kappa dx
    void* mark_g = nullptr;                  // bookmark of the previous step's rate (see warm_rate)
    uint32_t* mark_fc = nullptr;
    FrtRecs mark_F{};
    uint32_t mark_n = 0, mark_step = 0;
    bool marked = false;
    // kernel timing (HIP events around launches)
    bool timing = false;
    struct Ev { hipEvent_t a, b; int kind; };
    std::vector<Ev> pending;
    double t_ms[5] = {0, 0, 0, 0, 0};       // seed, brick march, chem, other (scan, scatter, fold), merge
    uint64_t n_march = 0, n_chem = 0, n_steps_timed = 0;

    ~frt_solve_s() { release_all(); }

    void drain_events()
    {
        for (auto& e : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) t_ms[e.kind] += ms;
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        pending.clear();
    }

    void reset_timing()
    {
        drain_events();
        for (double& t : t_ms) t = 0;
        n_march = n_chem = n_steps_timed = 0;
    }

    void release_all()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        drain_events();
        free_recs(F[0]);
        free_recs(F[1]);
        free_recs(mark_F);
        dev_free(vt[0]); dev_free(vt[1]); dev_free(vcount); dev_free(w0_merged); dev_free(mark_vt);
        dev_free(mark_x);
        dev_free(heat);
        dev_free(mark_T);
        dev_free(mark_fc);
        dev_free(d_desc); dev_free(op); dev_free(gam[0]); dev_free(gam[1]); dev_free(x); dev_free(xavg); dev_free(front);
        dev_free(kin); dev_free(mark_g);
        dev_free(nH); dev_free(T); dev_free(src_pos); dev_free(spec); dev_free(specd); dev_free(quat); dev_free(user_u); dev_free(fcount);
        dev_free(fcount_snap); dev_free(L); dev_free(L_snap);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
};

namespace {

// Stream-ordered copy / fill followed by a wait on the solve's stream, so a
// host-side transfer never races work already enqueued on that stream.
int scopy(frt_solve s, void* dst, const void* src, size_t bytes, hipMemcpyKind kind)
{
    if (bytes == 0) return FRT_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, kind, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int sset(frt_solve s, void* dst, int value, size_t bytes)
{
    if (bytes == 0) return FRT_OK;
    HIPCHK(hipMemsetAsync(dst, value, bytes, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

double split_radius_cells(const frt_params& P, int level)
{
    return std::ldexp(std::sqrt(3.0 / (PI * P.n_ray_min)), level);
}

// Passes a step needs: along any lineage a visit ends at a brick boundary or
// a split, so visits <= 3 (ceil(L/B) + 1) + splits + 1 with L the distance a
// packet can cover in one step (travel budget, distance cap, box diagonal).
int passes_needed(frt_solve s)
{
    const double diag = std::sqrt((double)s->nx * s->nx + (double)s->ny * s->ny + (double)s->nz * s->nz);
    double reach = diag;
    if (s->P.max_distance_cm > 0) reach = std::min(reach, s->P.max_distance_cm / s->dx);
    int l = s->P.base_level;
    while (l < s->P.max_level && split_radius_cells(s->P, l) < reach) l++;
    int splits = l - s->P.base_level;
    double travel = reach;
    if (std::isfinite(s->P.c_ray_cm_s)) travel = std::min(travel, s->P.c_ray_cm_s * s->h.dt / s->dx + 1.0);
    // A lineage's distance from its source grows by at most `travel` in a
    // step, so it splits at most at the split radii inside one window of
    // that length: the radii no larger than the window, and at most one
    // more (radii above it are more than its length apart, as they double)
    int small = 0;
    for (int k = s->P.base_level; k < s->P.max_level && split_radius_cells(s->P, k) <= travel; k++) small++;
    splits = std::min(splits, small + 1);
    int cross = 0;
    for (int a = 0; a < 3; a++) cross += (int)std::ceil(travel / (double)(1 << s->bsh[a])) + 1;
    return cross + 2 * splits + 6;
}

int ensure_quat(frt_solve s, uint32_t step)
{
    if (step < s->quat_steps) return FRT_OK;
    uint32_t nsteps = std::max<uint32_t>(step + 1, std::max<uint32_t>(64, 2 * s->quat_steps));
    double* nq = nullptr;
    RCCHK(dev_alloc((void**)&nq, (size_t)nsteps * std::max(1, s->n_src) * 4 * sizeof(double)));
    if (s->quat && s->quat_steps) {
        HIPCHK(hipMemcpyAsync(nq, s->quat, (size_t)s->quat_steps * s->n_src * 4 * sizeof(double), hipMemcpyDeviceToDevice,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        dev_free(s->quat);
    }
    s->quat = nq;
    s->quat_steps = nsteps;
    s->h.quat = nq;
    s->h.quat_steps = nsteps;
    return FRT_OK;
}

void set_step_fields(frt_solve s, double dt)
{
    FrtSolveDesc& h = s->h;
    h.step = s->step;
    h.cur = s->step & 1u;
    h.dt = dt;
    h.budget = std::isfinite(s->P.c_ray_cm_s) ? s->P.c_ray_cm_s * dt / s->dx : HUGE_VAL;
    h.w0_cast = dt / (double)(12ull << (2 * s->P.base_level));
    // photo-heating rate (erg/cm^3/s) per eV left in a cell during the step
    h.heat_scale = 1.602176634e-12 / (s->dx * s->dx * s->dx * dt);
    // a packet holds at most w0 photons per bin (the rates are scaled to at
    // most 1), and no packet's w0 exceeds the largest cast weight so far
    s->w0_max = std::max(s->w0_max, h.w0_cast);
    h.dep_scale = (float)(std::ldexp(1.0, 46) / (s->w0_max * s->P.n_bins));
    for (int b = 0; b < FRT_MAX_BINS_I; b++) {
        double kb = b < s->P.n_bins ? h.R_ref * s->P.sigma_bins[b] / (s->dx * s->dx * dt) : 0.0;
        h.Kd[b] = kb;
        h.K[b] = (float)kb;
    }
    h.KSd = h.R_ref * s->P.sigma_bins[0] / (s->dx * s->dx * dt);
    h.KS = (float)h.KSd;
    h.dep_base = std::ldexp(1.0, 46) / s->P.n_bins;
    if (h.has_sub) {
        // with sub-grid opacity a crossing deposits K_nu N_nu ds phi, at most
        // the largest K_nu times the packet's photons times sqrt(3) < 2
        double kmax = 0.0;
        for (int b = 0; b < s->P.n_bins; b++) kmax = std::max(kmax, h.Kd[b]);
        h.dep_base = std::ldexp(1.0, 46) / (2.0 * kmax * s->P.n_bins);
        h.dep_scale = (float)(h.dep_base / s->w0_max);
    }
    // merged packets' w0 are known on the device only: the seeding plan takes
    // the larger of the two
    h.w0_hi = s->w0_max;
}

int check_inputs_finite(const float* v, size_t n, const char* what)
{
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(v[i]) || v[i] < 0.f)
            return fail(FRT_EINVAL, "%s[%zu] = %g is negative or not finite", what, i, (double)v[i]);
    return FRT_OK;
}

template <typename T>
int host_view(const T* p, size_t n, int kind, std::vector<T>& buf, const T** out)
{
    if (kind == FRT_HOST) {
        *out = p;
        return FRT_OK;
    }
    buf.resize(n);
    HIPCHK(hipDeviceSynchronize());
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
    HIPCHK(hipMemcpyAsync(out, s->L, offsetof(FrtLedgerDev, sd), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

// A Generalized Opacity Mode solve with K >= 1 marches per step starts each
// step's opacity iteration from the previous step's rate field, which is
// then part of its state (checkpoints and bookmarks keep it).
bool warm_rate(frt_solve s) { return s->P.opacity_mode == FRT_GENERALIZED && s->P.chem_iterations > 0; }

// Mean of a field, summed in cell order.
double mean_of(const std::vector<double>& v)
{
    double sum = 0.0;
    for (double a : v) sum += a;
    return v.empty() ? 0.0 : sum / (double)v.size();
}

// Photo-heating per recombination of ionized gas in photo-ionization
// equilibrium (§4.2, Eq. analytical_heating_HI), erg: 1 Ryd times the mean
// energy above 1 Ryd, in Ryd, of the photons HI absorbs from a spectrum
// J_nu ~ nu^-alpha cut off at 4 Ryd when sigma_HI ~ nu^-2.75.  With
// p = alpha + 2.75 that mean is
//   int_1^4 x^-p dx / int_1^4 x^-(p+1) dx - 1 = p/(p-1) (1 - 4^(1-p)) / (1 - 4^-p) - 1.
double reion_heat_per_recombination(double alpha)
{
    const double p = alpha + 2.75;
    const double mean = p / (p - 1.0) * (1.0 - std::pow(4.0, 1.0 - p)) / (1.0 - std::pow(4.0, -p));
    return (mean - 1.0) * 13.605693122994 * 1.602176634e-12;
}

int ready(frt_solve s)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid || !s->have_src) return fail(FRT_ESTATE, "load the grid and the sources before stepping");
    return FRT_OK;
}

// Initial carried-queue size: casting plus, for packets moving at a finite
// speed, room for many carried packets (grown on overflow).
uint32_t initial_fcap(frt_solve s)
{
    const double cast = (double)s->n_src * (12ull << (2 * s->P.base_level));
    double F = cast + 1024;
    if (std::isfinite(s->P.c_ray_cm_s)) F += std::min((double)s->ncell, 8.0 * cast + 65536.0);
    if (s->P.queue_capacity) F = (double)s->P.queue_capacity;
    return (uint32_t)std::min(F, 2147483647.0);
}

// Make the context workspace fit a launch of `n` solves with `nkeys` brick
// keys and at least `want_p` sorted records per pass.
int ensure_ws(Workspace& ws, int fp64, int nb, int n, uint32_t nkeys, uint64_t want_p)
{
    const size_t rs = fp64 ? 8 : 4;
    if (ws.fp64 != fp64 || ws.nb != nb) {
        ws.free_pass();
        free_recs(ws.X);
        ws.fp64 = fp64;
        ws.nb = nb;
    }
    want_p = std::min<uint64_t>(want_p, 2147483647ull);
    if (ws.pcap < want_p) {
        if (ws.limit) {
            const uint64_t nk = std::max<uint64_t>(ws.nkeys_cap, std::max<uint32_t>(nkeys, 4096));
            const uint64_t grown = want_p * (2 * rec_bytes(rs) + 2 * 4 + sizeof(uint2)) +
                                   (want_p / (uint64_t)ws.tune.item_rays + nk + 64) * sizeof(FrtWork);
            if (grown > ws.limit)
                return fail(FRT_ENOMEM, "pass queues of %llu records need %llu bytes, more than the %llu the context allows",
                            (unsigned long long)want_p, (unsigned long long)grown, (unsigned long long)ws.limit);
        }
        ws.free_pass();
        for (int k = 0; k < 2; k++) {
            RCCHK(alloc_recs(ws.O[k], (uint32_t)want_p, nb, rs));
            RCCHK(dev_alloc((void**)&ws.okey[k], (size_t)want_p * 4));
        }
        RCCHK(dev_alloc((void**)&ws.sorted, (size_t)want_p * sizeof(uint2)));
        ws.pcap = (uint32_t)want_p;
        dev_free(ws.work);
        ws.cap_work = 0;
    }
    if (!ws.X.rec) RCCHK(alloc_recs(ws.X, (uint32_t)frt::device_cu_count() * FRT_XREC_PER_CU, nb, rs));
    if (!ws.ctr) RCCHK(dev_alloc((void**)&ws.ctr, C_NCTR * 4));
    if (!ws.ctr_host && hipHostMalloc((void**)&ws.ctr_host, C_NCTR * 4, hipHostMallocDefault) != hipSuccess) {
        ws.ctr_host = nullptr;
        return fail(FRT_ENOMEM, "pinned counter buffer");
    }
    if (!ws.segc) RCCHK(dev_alloc((void**)&ws.segc, (size_t)FRT_QSEG * FRT_QSEG_STRIDE * 4));
    if (!ws.segp) RCCHK(dev_alloc((void**)&ws.segp, (FRT_QSEG + 1) * 4ull));
    if (ws.nkeys_cap < nkeys) {
        dev_free(ws.hist);
        dev_free(ws.cursor);
        ws.nkeys_cap = 0;
        uint32_t c = std::max<uint32_t>(nkeys, 4096);
        RCCHK(dev_alloc((void**)&ws.hist, c * 4ull));
        RCCHK(dev_alloc((void**)&ws.cursor, c * 4ull));
        HIPCHK(hipMemset(ws.hist, 0, c * 4ull));
        HIPCHK(hipDeviceSynchronize());
        ws.nkeys_cap = c;
        dev_free(ws.work);
        ws.cap_work = 0;
    }
    const uint64_t want_work = (uint64_t)ws.pcap / (uint64_t)ws.tune.item_rays + ws.nkeys_cap + 64;
    if (ws.cap_work < want_work) {
        dev_free(ws.work);
        RCCHK(dev_alloc((void**)&ws.work, want_work * sizeof(FrtWork)));
        ws.cap_work = (uint32_t)want_work;
    }
    if (ws.solves_cap < n) {
        dev_free(ws.key_prefix); dev_free(ws.seed_prefix); dev_free(ws.cell_prefix); dev_free(ws.descs);
        int c = std::max(n, 64);
        RCCHK(dev_alloc((void**)&ws.key_prefix, (c + 1) * 4ull));
        RCCHK(dev_alloc((void**)&ws.seed_prefix, (c + 1) * 4ull));
        RCCHK(dev_alloc((void**)&ws.cell_prefix, (c + 1) * 8ull));
        RCCHK(dev_alloc((void**)&ws.descs, c * sizeof(FrtSolveDesc)));
        ws.solves_cap = c;
    }
    return FRT_OK;
}

// Event pair around a launch when the timing solve has timing enabled.
struct Timed {
    frt_solve t;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    int kind;
    Timed(frt_solve t_, hipStream_t s_, int k) : t(t_), st(s_), kind(k)
    {
        if (t && t->timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, st);
        else
            a = b = nullptr;
    }
    ~Timed()
    {
        if (a && b) {
            (void)hipEventRecord(b, st);
            t->pending.push_back({a, b, kind});
        }
    }
};

// Host side of one step of a group of solves (same n_bins and precision):
// brick-key bases, descriptors, prefixes, the pass count and the launch
// workspace.
struct Group {
    std::vector<uint32_t> kp;
    std::vector<unsigned long long> cp;
    std::vector<FrtSolveDesc> hd;
    int passes = 1;
    FrtWS w{};
};

void plan_group(Workspace& ws, frt_solve* ss, int n, Group& g)
{
    g.kp.assign(n + 1, 0);
    g.cp.assign(n + 1, 0);
    g.hd.resize(n);
    g.passes = 1;
    for (int i = 0; i < n; i++) {
        frt_solve s = ss[i];
        s->h.key_base = g.kp[i];
        g.hd[i] = s->h;
        g.kp[i + 1] = g.kp[i] + (uint32_t)(s->bpx * s->bpy * s->bpz);
        g.cp[i + 1] = g.cp[i] + s->ncell;
        g.passes = std::max(g.passes, passes_needed(s));
    }
    FrtWS& w = g.w;
    w = FrtWS{};
    for (int k = 0; k < 2; k++) {
        w.buf[k] = ws.O[k];
        w.bkey[k] = ws.okey[k];
    }
    w.out = 0;
    w.sorted = ws.sorted;
    w.pcap = ws.pcap;
    w.xrec = ws.X.rec;
    w.xrec_cap = ws.X.cap;
    w.segc = ws.segc;
    w.segp = ws.segp;
    w.ctr = ws.ctr;
    w.hist = ws.hist;
    w.cursor = ws.cursor;
    w.work = ws.work;
    w.cap_work = ws.cap_work;
    w.nkeys = g.kp[n];
    w.key_prefix = ws.key_prefix;
    w.seed_prefix = ws.seed_prefix;
    w.n_solves = n;
    w.n_bins = ss[0]->P.n_bins;
    w.has_sub = 0;
    w.has_heat = 0;
    w.has_temp = 0;
    for (int i = 0; i < n; i++) {
        w.has_sub |= ss[i]->h.has_sub;
        w.has_heat |= ss[i]->h.heat != nullptr;
        w.has_temp |= ss[i]->h.temp;
    }
    // the 1024-thread march (FP32 without sub-grid opacity) takes
    // FRT_BIG_ITEM_SCALE times the tuned item size
    w.item_rays = (uint32_t)ws.tune.item_rays * ((!ss[0]->fp64 && !w.has_sub) ? FRT_BIG_ITEM_SCALE : 1u);
    w.scatter_bpc = ws.tune.scatter_blocks_per_cu;
    if (ss[0]->P.queue_capacity) {
        // fixed capacities: the shared workspace is used up to the solves' limit
        uint64_t lim = 0;
        for (int i = 0; i < n; i++) lim += ss[i]->P.queue_capacity;
        const uint32_t c = (uint32_t)std::min<uint64_t>(lim, w.pcap);
        w.buf[0].cap = c;
        w.buf[1].cap = c;
        w.pcap = c;
    }
}

// Descriptors and prefixes to the device (pageable host memory: never
// inside a stream capture).
int upload_group(Workspace& ws, const Group& g, int n, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(ws.descs, g.hd.data(), n * sizeof(FrtSolveDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ws.key_prefix, g.kp.data(), (n + 1) * 4ull, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ws.cell_prefix, g.cp.data(), (n + 1) * 8ull, hipMemcpyHostToDevice, st));
    return FRT_OK;
}

// Enqueue one step of a planned group on st.  With `graph` the step is
// being captured: it starts by saving each solve's ledger and carried count
// (for a re-run after an overflow) and ends by advancing the step index on
// the device; nothing in it reads host memory or records events.
int enqueue_step(Workspace& ws, frt_solve* ss, int n, const Group& g, hipStream_t st, bool graph, bool timed = true)
{
    const int fp64 = ss[0]->fp64;
    FrtWS w = g.w;
    frt_solve tm = (timed && !graph && ss[0]->timing) ? ss[0] : nullptr;
    // a replayed step does nothing after a replay that failed; a step
    // launched on its own starts by resetting every launch counter
    const uint32_t* halt = graph ? w.ctr + C_HALT : nullptr;
    hipError_t e;
    // every solve's ledger and carried-queue counters as the step starts, for
    // a re-run after an overflow (one kernel for the whole group)
    if ((e = frt::launch_snapshot(ws.descs, n, halt, st)) != hipSuccess) return fail(FRT_EDEVICE, "snapshot: %s", hipGetErrorString(e));
    // backward Euler: one march, then the update; time-averaged chemistry:
    // K marches from the same packets with <x> updated between them
    const int K = ss[0]->P.chem_iterations;   // the same for every solve of a group
    const int n_march = K > 0 ? K : 1;
    if (K > 0) {
        Timed t(tm, st, 2);
        if ((e = frt::launch_chem_avg(ws.descs, ws.cell_prefix, n, g.cp[n], fp64, w.has_temp, 0, w.ctr + C_ERR, halt, st)) != hipSuccess)
            return fail(FRT_EDEVICE, "chem: %s", hipGetErrorString(e));
    }
    for (int it = 0; it < n_march; it++) {
        if (it > 0) {
            Timed t(tm, st, 3);
            if ((e = frt::launch_iter_restart(ws.descs, n, halt, st)) != hipSuccess)
                return fail(FRT_EDEVICE, "restart: %s", hipGetErrorString(e));
        }
        {
            Timed t(tm, st, 0);
            w.out = 0;   // seeds fill buffer 0, the input of the first pass
            const int mode = it > 0 ? CLEAR_ITER : (graph ? CLEAR_STEP : CLEAR_ALL);
            if ((e = frt::launch_clear(w, mode, st)) != hipSuccess) return fail(FRT_EDEVICE, "clear: %s", hipGetErrorString(e));
            if ((e = frt::launch_seed(ws.descs, w, fp64, st)) != hipSuccess) return fail(FRT_EDEVICE, "seed: %s", hipGetErrorString(e));
        }
        for (int p = 0; p < g.passes; p++) {
            w.out = (p + 1) & 1;   // pass p reads buffer p & 1 and fills the other
            {
                Timed t(tm, st, 3);
                if ((e = frt::launch_pass(ws.descs, w, fp64, 0, st)) != hipSuccess) return fail(FRT_EDEVICE, "scan: %s", hipGetErrorString(e));
                if ((e = frt::launch_pass(ws.descs, w, fp64, 1, st)) != hipSuccess) return fail(FRT_EDEVICE, "scatter: %s", hipGetErrorString(e));
            }
            {
                Timed t(tm, st, 1);
                if ((e = frt::launch_pass(ws.descs, w, fp64, 2, st)) != hipSuccess) return fail(FRT_EDEVICE, "march: %s", hipGetErrorString(e));
                if (tm) tm->n_march++;
            }
        }
        {
            Timed t(tm, st, 3);
            if ((e = frt::launch_finish(ws.descs, w, st)) != hipSuccess) return fail(FRT_EDEVICE, "finish: %s", hipGetErrorString(e));
        }
        if (it + 1 < n_march) {
            Timed t(tm, st, 2);
            if ((e = frt::launch_chem_avg(ws.descs, ws.cell_prefix, n, g.cp[n], fp64, w.has_temp, 1, w.ctr + C_ERR, halt, st)) != hipSuccess)
                return fail(FRT_EDEVICE, "chem: %s", hipGetErrorString(e));
        }
    }
    {
        Timed t(tm, st, 2);
        if (K > 0) e = frt::launch_chem_avg(ws.descs, ws.cell_prefix, n, g.cp[n], fp64, w.has_temp, 2, w.ctr + C_ERR, halt, st);
        else e = frt::launch_chem(ws.descs, ws.cell_prefix, n, g.cp[n], fp64, w.has_temp, w.ctr + C_ERR, st);
        if (e != hipSuccess) return fail(FRT_EDEVICE, "chem: %s", hipGetErrorString(e));
        if (tm) tm->n_chem++;
    }
    if (graph && (e = frt::launch_advance(ws.descs, w, st)) != hipSuccess)
        return fail(FRT_EDEVICE, "advance: %s", hipGetErrorString(e));
    if (tm) tm->n_steps_timed++;
    return FRT_OK;
}

// Queue sizes of a group step before anything grew: brick keys and the
// first size of the pass queues.
int group_sizes(frt_solve* ss, int n, uint32_t* nkeys, uint64_t* want_p)
{
    uint64_t nk = 0, wp = 0;
    for (int i = 0; i < n; i++) {
        frt_solve s = ss[i];
        nk += (uint64_t)s->bpx * s->bpy * s->bpz;
        const uint64_t cast = (uint64_t)s->n_src * (12ull << (2 * s->P.base_level));
        wp += s->P.queue_capacity ? s->P.queue_capacity
                                  : (s->P.queue_hint ? s->P.queue_hint : std::max<uint64_t>(4 * cast + 65536, s->ncell / 2));
    }
    if (nk > FRT_KEY_MASK)
        return fail(FRT_EINVAL, "the solves of one launch hold %llu bricks, more than %u", (unsigned long long)nk, FRT_KEY_MASK);
    *nkeys = (uint32_t)nk;
    *want_p = wp;
    return FRT_OK;
}

// Put every solve of a step that overflowed back to the start of that step:
// ledger (with its error bits), carried-packet counts, this step's rate
// buffer and front counts.  The chemistry of an overflowed step does not run
// (its kernels skip a solve whose ledger has error bits), so the neutral
// fraction is already the one of the start of the step.
int restore_step_start(frt_solve* ss, int n, hipStream_t st)
{
    for (int i = 0; i < n; i++) {
        frt_solve s = ss[i];
        HIPCHK(hipMemcpyAsync(s->L, s->L_snap, sizeof(FrtLedgerDev), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(s->fcount, s->fcount_snap, 8, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemsetAsync(s->gam[s->step & 1u], 0, s->ncell * s->rs, st));
        if (s->front) HIPCHK(hipMemsetAsync(s->front, 0, s->ncell * 8, st));
        if (s->heat) HIPCHK(hipMemsetAsync(s->heat, 0, s->ncell * s->rs, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return FRT_OK;
}

// After a step that overflowed: put every solve back to the start of the
// step and enlarge what overflowed.
int recover_overflow(Workspace& ws, frt_solve* ss, int n, const uint32_t* ctr, uint64_t* want_p, hipStream_t st)
{
    // packets each solve tried to carry into the next step (the counter
    // counts every reservation, also those past the capacity)
    std::vector<uint32_t> fneed(n, 0);
    if (ctr[C_ERR] & FRT_DEVERR_CARRY_OVERFLOW) {
        HIPCHK(hipStreamSynchronize(st));
        for (int i = 0; i < n; i++) {
            uint32_t fc[2];
            HIPCHK(hipMemcpy(fc, ss[i]->fcount, 8, hipMemcpyDeviceToHost));
            const uint32_t nxt = fc[1 - (ss[i]->step & 1u)];
            if (nxt > ss[i]->F[0].cap) fneed[i] = nxt;
        }
    }
    for (int i = 0; i < n; i++)
        if (ss[i]->timing) ss[i]->reset_timing();
    RCCHK(restore_step_start(ss, n, st));
    if (ctr[C_ERR] & FRT_DEVERR_QUEUE_OVERFLOW) {
        if (ws.pcap >= 2147483647u) return fail(FRT_EOVERFLOW, "pass buffers at their maximum size still overflow");
        const uint64_t need = std::max<uint64_t>(2ull * ws.pcap, (uint64_t)ctr[C_MAXP] + (ctr[C_MAXP] >> 2) + 65536);
        *want_p = std::min<uint64_t>(need, 2147483647ull);
    }
    for (int i = 0; i < n; i++) {
        frt_solve s = ss[i];
        if (!fneed[i]) continue;
        const uint64_t nc = std::min<uint64_t>(std::max<uint64_t>(2ull * s->F[0].cap, fneed[i] + 65536ull), 2147483647ull);
        const int cur = (int)(s->step & 1u);
        uint32_t keep;
        HIPCHK(hipMemcpy(&keep, s->fcount + cur, 4, hipMemcpyDeviceToHost));
        FrtRecs nf[2];
        RCCHK(alloc_recs(nf[0], (uint32_t)nc, s->P.n_bins, s->rs));
        RCCHK(alloc_recs(nf[1], (uint32_t)nc, s->P.n_bins, s->rs));
        RCCHK(copy_recs(nf[cur], s->F[cur], std::min(keep, s->F[cur].cap), s->P.n_bins, s->rs, st, hipMemcpyDeviceToDevice));
        HIPCHK(hipStreamSynchronize(st));
        free_recs(s->F[0]);
        free_recs(s->F[1]);
        s->F[0] = nf[0];
        s->F[1] = nf[1];
        s->h.F[0] = nf[0];
        s->h.F[1] = nf[1];
        RCCHK(upload_desc(s));
    }
    return FRT_OK;
}

int read_counters(Workspace& ws, hipStream_t st, uint32_t* out)
{
    HIPCHK(hipMemcpyAsync(ws.ctr_host, ws.ctr, C_NCTR * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(out, ws.ctr_host, C_NCTR * 4);
    return FRT_OK;
}

// Solves of one launch share a brick shape; a batch mixing shapes (FP32
// solves with and without sub-grid opacity) runs as one launch sequence per
// shape.  Returns true and fills the parts when ss holds more than one.
bool split_by_shape(frt_solve* ss, int n, const double* dts, std::vector<std::vector<frt_solve>>& parts,
                    std::vector<std::vector<double>>& pdts)
{
    // solves of one launch share the brick shape and the chemistry's march count
    auto shape = [](frt_solve s) { return s->P.chem_iterations * 1000 + s->bsh[0] * 100 + s->bsh[1] * 10 + s->bsh[2]; };
    bool mixed = false;
    for (int i = 1; i < n; i++) mixed |= shape(ss[i]) != shape(ss[0]);
    if (!mixed) return false;
    std::vector<int> keys;
    for (int i = 0; i < n; i++) {
        const int k = shape(ss[i]);
        size_t at = std::find(keys.begin(), keys.end(), k) - keys.begin();
        if (at == keys.size()) {
            keys.push_back(k);
            parts.emplace_back();
            pdts.emplace_back();
        }
        parts[at].push_back(ss[i]);
        pdts[at].push_back(dts[i]);
    }
    return true;
}

int alloc_merge(Workspace& ws, uint32_t n, uint32_t n_old, int fp64);

// Room in the context's merge scratch for n carried packets referring to a
// table of n_old entries; on failure no scratch is held.
int ensure_merge(Workspace& ws, uint32_t n, uint32_t n_old, int fp64)
{
    const int rc = alloc_merge(ws, n, n_old, fp64);
    if (rc != FRT_OK) ws.free_merge();
    return rc;
}

int alloc_merge(Workspace& ws, uint32_t n, uint32_t n_old, int fp64)
{
    Workspace::Merge& m = ws.mg;
    const size_t rs = fp64 ? 8 : 4, rec = rec_bytes(rs);
    if (m.mcap < n || m.rec != rec || m.mold < n_old) {
        const uint32_t cap = std::max<uint32_t>(std::max(n, m.rec == rec ? m.mcap : 0u), 1024);
        const uint32_t old = std::max<uint32_t>(std::max(n_old, m.mold), 1024);
        ws.free_merge();
        RCCHK(dev_alloc(&m.pkey, (size_t)cap * rs));
        RCCHK(dev_alloc(&m.pkey_sorted, (size_t)cap * rs));
        RCCHK(dev_alloc((void**)&m.gkey, (size_t)cap * 8));
        RCCHK(dev_alloc((void**)&m.gkey_s, (size_t)cap * 8));
        RCCHK(dev_alloc((void**)&m.idx, (size_t)cap * 4));
        RCCHK(dev_alloc((void**)&m.idx_s, (size_t)cap * 4));
        RCCHK(dev_alloc((void**)&m.flag_out, (size_t)cap * 4));
        RCCHK(dev_alloc((void**)&m.slot, (size_t)cap * 4));
        RCCHK(dev_alloc((void**)&m.flag_lead, (size_t)cap * 4));
        RCCHK(dev_alloc((void**)&m.gid, (size_t)cap * 4));
        // sums of the groups that reach across a wave of 64 packets: one slot per wave
        const size_t slots = (size_t)cap / 64 + 2;
        RCCHK(dev_alloc((void**)&m.acc, slots * (7 + FRT_MAX_BINS_I) * sizeof(double)));
        RCCHK(dev_alloc((void**)&m.acc_head, slots * 4));
        RCCHK(dev_alloc((void**)&m.ref, (size_t)old * 4));
        RCCHK(dev_alloc((void**)&m.vmap, (size_t)old * 4));
        RCCHK(dev_alloc((void**)&m.counts, 16));
        RCCHK(dev_alloc((void**)&m.residual, 8));
        RCCHK(dev_alloc((void**)&m.stats, 16));
        m.temp_bytes = frt::merge_temp_bytes(cap, old, fp64);
        RCCHK(dev_alloc(&m.temp, m.temp_bytes));
        m.mcap = cap;
        m.mold = old;
        m.rec = rec;
    }
    return FRT_OK;
}

// A solve's table of virtual origins `k` with room for `cap` entries (its
// contents are not kept: only the table the next merge writes grows), grown
// to at least twice its size unless `exact`.  The old table is freed only
// once the new one is held.
int ensure_vtable(frt_solve s, int k, uint32_t cap, bool exact = false)
{
    if (s->vt_cap[k] >= cap) return FRT_OK;
    const uint32_t c = exact ? cap : std::max<uint32_t>(cap, 2 * s->vt_cap[k]);
    FrtVSrc* t = nullptr;
    RCCHK(dev_alloc((void**)&t, (size_t)c * sizeof(FrtVSrc)));
    dev_free(s->vt[k]);
    s->vt[k] = t;
    s->vt_cap[k] = c;
    s->h.vt[k] = t;
    return FRT_OK;
}

// Taken before a step of a merging solve, so that the step's packets can
// always be carried, merged or not: room in the next table for every entry
// of the current one.  The merge itself sizes its scratch and the next
// table from what the step left (merge_after_step).
int prepare_merge(frt_solve s)
{
    const int cur = (int)(s->step & 1u), nxt = cur ^ 1;
    uint32_t vc[2];
    HIPCHK(hipMemcpyAsync(vc, s->vcount, 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return ensure_vtable(s, nxt, vc[cur], true);
}

// The packets a merging solve carries into the next step, left unmerged:
// the current table of virtual origins becomes the next one as it is.
int carry_unmerged(frt_solve s, uint32_t n_old, hipStream_t st)
{
    const int cur = (int)(s->step & 1u), nxt = cur ^ 1;
    if (n_old)
        HIPCHK(hipMemcpyAsync(s->vt[nxt], s->vt[cur], (size_t)n_old * sizeof(FrtVSrc), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(s->vcount + nxt, &n_old, 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return FRT_OK;
}

// Ray merging (§3.3) of a solve after a step that ran without error: the
// packets it carries into the next step are merged, and the virtual origins
// they refer to renumbered into the table of the next step.  `d` is the
// solve's descriptor of that step on the device (its step index not yet
// advanced).  The merge scratch and the next table are sized from the
// step's own counts; if the device cannot hold them the packets are carried
// unmerged this step (the room for that was taken before the step).  Waits
// for the merge.
int merge_after_step(Workspace& ws, frt_solve s, FrtSolveDesc* d, hipStream_t st)
{
    const int cur = (int)(s->step & 1u), nxt = cur ^ 1;
    uint32_t fc[2], vc[2];
    HIPCHK(hipMemcpyAsync(fc, s->fcount, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(vc, s->vcount, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const uint32_t n = std::min(fc[nxt], s->F[nxt].cap);
    const uint32_t n_old = vc[cur];
    const uint64_t E = (uint64_t)std::floor(s->P.merge_exempt * (double)s->ncell);
    const bool all_exempt = E >= n;
    if (n == 0 || (all_exempt && n_old == 0)) {
        vc[nxt] = 0;
        HIPCHK(hipMemcpyAsync(s->vcount + nxt, &vc[nxt], 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return FRT_OK;
    }
    if (s->vt_cap[nxt] < n_old) return fail(FRT_EDEVICE, "next table of virtual origins smaller than reserved");
    if (ensure_merge(ws, n, n_old, s->fp64) != FRT_OK) return carry_unmerged(s, n_old, st);
    Workspace::Merge& m = ws.mg;
    FrtMergeArgs a{};
    a.n = n;
    a.n_old = n_old;
    a.E = E;
    a.level = s->P.merge_level;
    a.all_exempt = all_exempt ? 1 : 0;
    int cell_bits = 0;
    while (cell_bits < 40 && (1ull << cell_bits) < (uint64_t)s->ncell) cell_bits++;
    a.end_bit = 20 + cell_bits;
    a.key_mask = (a.end_bit >= 64) ? ~0ull : ((1ull << a.end_bit) - 1ull);
    a.pkey = m.pkey;
    a.pkey_sorted = m.pkey_sorted;
    a.gkey = m.gkey;
    a.gkey_s = m.gkey_s;
    a.idx = m.idx;
    a.idx_s = m.idx_s;
    a.flag_out = m.flag_out;
    a.slot = m.slot;
    a.flag_lead = m.flag_lead;
    a.gid = m.gid;
    a.ref = m.ref;
    a.vmap = m.vmap;
    a.counts = m.counts;
    a.residual = m.residual;
    a.stats = m.stats;
    a.dst = s->F[cur].rec;   // read by the step's seeding, free now; as large as F[nxt]
    a.acc = m.acc;
    a.acc_head = m.acc_head;
    a.n_slots = (n + 63) / 64;
    a.temp = m.temp;
    a.temp_bytes = m.temp_bytes;
    Timed t(s->timing ? s : nullptr, st, 4);
    hipError_t e = frt::launch_merge(d, a, s->fp64, s->P.n_bins, 0, st);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "merge: %s", hipGetErrorString(e));
    uint32_t counts[3];
    HIPCHK(hipMemcpyAsync(counts, m.counts, 12, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (counts[0] > s->F[cur].cap) return fail(FRT_EDEVICE, "merged queue larger than the carried queue");
    // the next table: the entries still referred to and one per merged group
    const uint32_t need = counts[1] + counts[2];
    if (s->vt_cap[nxt] < need) {
        if (ensure_vtable(s, nxt, need) != FRT_OK) return carry_unmerged(s, n_old, st);
        HIPCHK(hipMemcpyAsync((char*)d + offsetof(FrtSolveDesc, vt) + nxt * sizeof(FrtVSrc*), &s->vt[nxt],
                              sizeof(FrtVSrc*), hipMemcpyHostToDevice, st));
    }
    e = frt::launch_merge(d, a, s->fp64, s->P.n_bins, 1, st);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "merge: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(st));
    // the merged queue is the next step's carried queue
    std::swap(s->F[0], s->F[1]);
    s->h.F[0] = s->F[0];
    s->h.F[1] = s->F[1];
    return FRT_OK;
}

int step_group_locked(frt_solve* ss, int n, const double* dts);

// One step of a group with automatic queue growth: snapshot, run, check,
// and on overflow restore the starting state, enlarge and run again.
// The caller holds the context lock.
int step_group_locked(frt_solve* ss, int n, const double* dts)
{
    {
        std::vector<std::vector<frt_solve>> parts;
        std::vector<std::vector<double>> pdts;
        if (split_by_shape(ss, n, dts, parts, pdts)) {
            for (size_t k = 0; k < parts.size(); k++)
                RCCHK(step_group_locked(parts[k].data(), (int)parts[k].size(), pdts[k].data()));
            return FRT_OK;
        }
    }
    Workspace& ws = ss[0]->ctx->ws;
    hipStream_t st = ss[0]->stream;
    const bool auto_grow = ss[0]->P.queue_capacity == 0;
    uint32_t nkeys = 0;
    uint64_t want_p = 0;
    RCCHK(group_sizes(ss, n, &nkeys, &want_p));
    for (int i = 0; i < n; i++) {
        RCCHK(ensure_quat(ss[i], ss[i]->step));
        set_step_fields(ss[i], dts[i]);
    }
    for (int attempt = 0; attempt < 16; attempt++) {
        RCCHK(ensure_ws(ws, ss[0]->fp64, ss[0]->P.n_bins, n, nkeys, std::max<uint64_t>(want_p, ws.pcap)));
        for (int i = 0; i < n; i++)
            if (ss[i]->P.merge) RCCHK(prepare_merge(ss[i]));
        Group g;
        plan_group(ws, ss, n, g);
        RCCHK(upload_group(ws, g, n, st));
        RCCHK(enqueue_step(ws, ss, n, g, st, false));
        uint32_t ctr[C_NCTR];
        RCCHK(read_counters(ws, st, ctr));
        if (!auto_grow && (ctr[C_ERR] & (FRT_DEVERR_QUEUE_OVERFLOW | FRT_DEVERR_CARRY_OVERFLOW))) {
            // fixed capacities: the step is not applied
            RCCHK(restore_step_start(ss, n, st));
            return fail(FRT_EOVERFLOW, "a ray queue overflowed at step %u; raise queue_capacity (the step was not applied)",
                        ss[0]->step);
        }
        if (!(ctr[C_ERR] & (FRT_DEVERR_QUEUE_OVERFLOW | FRT_DEVERR_CARRY_OVERFLOW))) {
            if (ctr[C_ERR] & FRT_DEVERR_UNFINISHED) return fail(FRT_EDEVICE, "a step left packets after its last pass");
            for (int i = 0; i < n; i++)
                if (ss[i]->P.merge) RCCHK(merge_after_step(ws, ss[i], ws.descs + i, st));
            for (int i = 0; i < n; i++) ss[i]->step++;
            return FRT_OK;
        }
        RCCHK(recover_overflow(ws, ss, n, ctr, &want_p, st));
    }
    return fail(FRT_EOVERFLOW, "step kept overflowing its queues");
}

int step_group(frt_solve* ss, int n, const double* dts)
{
    std::lock_guard<std::mutex> lock(ss[0]->ctx->mu);
    return step_group_locked(ss, n, dts);
}

// A HIP graph of one step of a group, destroyed with the object.
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void reset()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~StepGraph() { reset(); }
};

// n_steps steps of a group; each step is one replay of a captured graph.
// Replays are enqueued `window` at a time and the launch counters are read
// back after each window: the replays after one that failed do nothing
// (C_HALT), C_DONE tells how many steps were applied, and an overflow
// restores the failed step's start, grows the queues, captures again and
// repeats the step.  The caller holds the lock.
int run_group_graph_locked(frt_solve* ss, int n, const double* dts, int n_steps, int window)
{
    {
        std::vector<std::vector<frt_solve>> parts;
        std::vector<std::vector<double>> pdts;
        if (split_by_shape(ss, n, dts, parts, pdts)) {
            for (size_t k = 0; k < parts.size(); k++)
                RCCHK(run_group_graph_locked(parts[k].data(), (int)parts[k].size(), pdts[k].data(), n_steps, window));
            return FRT_OK;
        }
    }
    Workspace& ws = ss[0]->ctx->ws;
    hipStream_t st = ss[0]->stream;
    const bool auto_grow = ss[0]->P.queue_capacity == 0;
    uint32_t nkeys = 0;
    uint64_t want_p = 0;
    RCCHK(group_sizes(ss, n, &nkeys, &want_p));
    int has_sub = 0, has_heat = 0;
    for (int i = 0; i < n; i++) {
        // rotations of every step of the run exist before the capture
        RCCHK(ensure_quat(ss[i], ss[i]->step + (uint32_t)n_steps));
        has_sub |= ss[i]->h.has_sub;
        has_heat |= ss[i]->h.heat != nullptr;
    }
    frt::prime_launch_shapes(ss[0]->fp64, ss[0]->P.n_bins, has_sub, has_heat);
    StepGraph sg;
    Group g;
    int done = 0, retries = 0;
    while (done < n_steps) {
        if (!sg.exec) {
            for (int i = 0; i < n; i++) set_step_fields(ss[i], dts[i]);
            RCCHK(ensure_ws(ws, ss[0]->fp64, ss[0]->P.n_bins, n, nkeys, std::max<uint64_t>(want_p, ws.pcap)));
            plan_group(ws, ss, n, g);
            RCCHK(upload_group(ws, g, n, st));
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue_step(ws, ss, n, g, st, true);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &graph);
            sg.graph = graph;
            if (rc != FRT_OK) return rc;
            if (ec != hipSuccess) return fail(FRT_EDEVICE, "graph capture: %s", hipGetErrorString(ec));
            HIPCHK(hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0));
        }
        const int k = std::min(window, n_steps - done);
        hipError_t e;
        if ((e = frt::launch_clear(g.w, CLEAR_ALL, st)) != hipSuccess) return fail(FRT_EDEVICE, "clear: %s", hipGetErrorString(e));
        for (int r = 0; r < k; r++) HIPCHK(hipGraphLaunch(sg.exec, st));
        uint32_t ctr[C_NCTR];
        RCCHK(read_counters(ws, st, ctr));
        const uint32_t applied = ctr[C_DONE];
        if (applied > (uint32_t)k || (applied < (uint32_t)k && !ctr[C_HALT]))
            return fail(FRT_EDEVICE, "%u of %d replayed steps reported applied", applied, k);
        for (int i = 0; i < n; i++) ss[i]->step += applied;
        done += (int)applied;
        if (applied) retries = 0;
        if (ctr[C_ERR] & (FRT_DEVERR_QUEUE_OVERFLOW | FRT_DEVERR_CARRY_OVERFLOW)) {
            if (!auto_grow) {
                // fixed capacities: the step is not applied
                RCCHK(restore_step_start(ss, n, st));
                for (int i = 0; i < n; i++) {
                    ss[i]->h.step = ss[i]->step;
                    ss[i]->h.cur = ss[i]->step & 1u;
                    RCCHK(upload_desc(ss[i]));
                }
                return fail(FRT_EOVERFLOW, "a ray queue overflowed at step %u; raise queue_capacity (the step was not applied)",
                            ss[0]->step);
            }
            if (++retries > 16) return fail(FRT_EOVERFLOW, "step kept overflowing its queues");
            RCCHK(recover_overflow(ws, ss, n, ctr, &want_p, st));
            sg.reset();
            continue;
        }
        if (ctr[C_ERR] & FRT_DEVERR_UNFINISHED) return fail(FRT_EDEVICE, "a step left packets after its last pass");
    }
    for (int i = 0; i < n; i++) {
        ss[i]->h.step = ss[i]->step;
        ss[i]->h.cur = ss[i]->step & 1u;
        RCCHK(upload_desc(ss[i]));
    }
    return FRT_OK;
}

// Device copy of everything a step changes in a solve, for the autotuner.
struct SolveSnap {
    double* x = nullptr;
    double* T = nullptr;
    void* gam_last = nullptr;
    FrtRecs F{};
    FrtLedgerDev* L = nullptr;
    uint32_t fc[2] = {0, 0};
    uint32_t step = 0;
    void release()
    {
        dev_free(x);
        dev_free(T);
        dev_free(gam_last);
        free_recs(F);
        dev_free(L);
    }
};

int snap_take(frt_solve s, SolveSnap& p)
{
    HIPCHK(hipStreamSynchronize(s->stream));
    RCCHK(scopy(s, p.fc, s->fcount, 8, hipMemcpyDeviceToHost));
    const int cur = (int)(s->step & 1u);
    const uint32_t nc = std::min(p.fc[cur], s->F[cur].cap);
    RCCHK(dev_alloc((void**)&p.x, s->ncell * 8));
    RCCHK(dev_alloc(&p.gam_last, s->ncell * s->rs));
    RCCHK(dev_alloc((void**)&p.L, sizeof(FrtLedgerDev)));
    RCCHK(alloc_recs(p.F, std::max<uint32_t>(nc, 1), s->P.n_bins, s->rs));
    HIPCHK(hipMemcpyAsync(p.x, s->x, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    if (s->h.temp) {
        RCCHK(dev_alloc((void**)&p.T, s->ncell * 8));
        HIPCHK(hipMemcpyAsync(p.T, s->T, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    }
    HIPCHK(hipMemcpyAsync(p.gam_last, s->gam[cur ^ 1], s->ncell * s->rs, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(p.L, s->L, sizeof(FrtLedgerDev), hipMemcpyDeviceToDevice, s->stream));
    RCCHK(copy_recs(p.F, s->F[cur], nc, s->P.n_bins, s->rs, s->stream, hipMemcpyDeviceToDevice));
    HIPCHK(hipStreamSynchronize(s->stream));
    p.step = s->step;
    return FRT_OK;
}

int snap_restore(frt_solve s, const SolveSnap& p)
{
    const int cur = (int)(p.step & 1u);
    const uint32_t nc = std::min(p.fc[cur], p.F.cap);
    if (nc > s->F[cur].cap) return fail(FRT_ESTATE, "carried queue shrank during tuning");
    HIPCHK(hipMemcpyAsync(s->x, p.x, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->gam[cur ^ 1], p.gam_last, s->ncell * s->rs, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipMemsetAsync(s->gam[cur], 0, s->ncell * s->rs, s->stream));
    if (s->front) HIPCHK(hipMemsetAsync(s->front, 0, s->ncell * 8, s->stream));
    if (p.T) HIPCHK(hipMemcpyAsync(s->T, p.T, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    if (s->heat) HIPCHK(hipMemsetAsync(s->heat, 0, s->ncell * s->rs, s->stream));
    HIPCHK(hipMemcpyAsync(s->L, p.L, sizeof(FrtLedgerDev), hipMemcpyDeviceToDevice, s->stream));
    RCCHK(copy_recs(s->F[cur], p.F, nc, s->P.n_bins, s->rs, s->stream, hipMemcpyDeviceToDevice));
    HIPCHK(hipMemcpyAsync(s->fcount, p.fc, 8, hipMemcpyHostToDevice, s->stream));
    s->step = p.step;
    s->h.step = p.step;
    s->h.cur = p.step & 1u;
    RCCHK(upload_desc(s));
    hipError_t e = frt::launch_prep_opacity(s->d_desc, s->ncell, s->fp64, s->stream);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "prep launch: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int check_batch(frt_solve* ss, int n, const double* dts)
{
    if (!ss || n < 1 || !dts) return fail(FRT_EINVAL, "bad batch");
    if (n > FRT_MAX_SOLVES_PER_LAUNCH) return fail(FRT_EINVAL, "at most %d solves per batch", FRT_MAX_SOLVES_PER_LAUNCH);
    for (int i = 0; i < n; i++) {
        RCCHK(ready(ss[i]));
        if (ss[i]->P.n_bins != ss[0]->P.n_bins || ss[i]->fp64 != ss[0]->fp64)
            return fail(FRT_EINVAL, "batched solves must share n_bins and march_precision");
        if (ss[i]->ctx != ss[0]->ctx) return fail(FRT_EINVAL, "batched solves must share a context");
        if ((ss[i]->P.queue_capacity == 0) != (ss[0]->P.queue_capacity == 0))
            return fail(FRT_EINVAL, "batched solves must all use automatic queues or all fixed ones");
        if (!(dts[i] > 0) || !std::isfinite(dts[i])) return fail(FRT_EINVAL, "dt must be finite and > 0");
        for (int j = 0; j < i; j++)
            if (ss[j] == ss[i]) return fail(FRT_EINVAL, "a solve appears twice in the batch");
    }
    return FRT_OK;
}

// One packet marched through a solve's current opacity by the production
// kernels (seeding of a carried packet, the brick passes, the ledger fold),
// in a solve object of its own: its descriptor, packet queues, ledger and
// rate buffer are temporary, while the opacity, n_H and x_HI it reads are
// the solve's (read only: no chemistry runs).  The packet is at level 12 and
// so never splits; it has no flux floor, distance cap or travel budget.
// The caller holds the context lock.
int debug_cast_locked(frt_solve s, const double o_cm[3], const double d_in[3], const double* N, double dt,
                      float* gamma_out, int kind, double* absorbed, double* escaped, uint64_t* crossings)
{
    const int nb = s->P.n_bins;
    double d[3], nrm = 0;
    for (int a = 0; a < 3; a++) nrm += d_in[a] * d_in[a];
    nrm = std::sqrt(nrm);
    for (int a = 0; a < 3; a++) d[a] = d_in[a] / nrm;
    double Rref = 0, total = 0;
    for (int b = 0; b < nb; b++) {
        Rref = std::max(Rref, N[b]);
        total += N[b];
    }
    if (!(Rref > 0)) Rref = 1.0;
    // the packet's cell: floor per axis, a point on a face belongs to the
    // cell being entered (the same rule as the march)
    int c[3];
    bool inside = true;
    const int dims[3] = {s->nx, s->ny, s->nz};
    for (int a = 0; a < 3; a++) {
        const double pc = o_cm[a] / s->dx;
        double f = std::floor(pc);
        if (pc == f && d[a] < 0) f -= 1.0;
        inside &= f >= 0 && f < dims[a];
        c[a] = inside ? (int)f : 0;
    }
    *absorbed = 0;
    *escaped = 0;
    *crossings = 0;
    std::unique_ptr<frt_solve_s> t(new (std::nothrow) frt_solve_s);
    if (!t) return fail(FRT_ENOMEM, "debug cast");
    t->ctx = s->ctx;
    t->stream = s->stream;
    t->own_stream = false;
    t->P = s->P;
    t->P.flux_floor = 0.0;
    t->P.max_distance_cm = 0.0;
    t->P.c_ray_cm_s = HUGE_VAL;
    t->P.chem_iterations = 0;
    t->P.queue_capacity = 0;
    t->P.merge = 0;
    t->P.temperature = 0;
    t->fp64 = s->fp64;
    t->rs = s->rs;
    for (int a = 0; a < 3; a++) t->bsh[a] = s->bsh[a];
    t->have_grid = t->have_src = true;
    t->nx = s->nx; t->ny = s->ny; t->nz = s->nz;
    t->bpx = s->bpx; t->bpy = s->bpy; t->bpz = s->bpz;
    t->dx = s->dx;
    t->ncell = s->ncell;
    t->n_src = 1;
    t->h = s->h;
    // the solve's temperature and heating stay as they are
    t->h.temp = 0;
    t->h.T = nullptr;
    t->h.heat = nullptr;
    RCCHK(dev_alloc((void**)&t->d_desc, sizeof(FrtSolveDesc)));
    RCCHK(dev_alloc((void**)&t->fcount, 8));
    RCCHK(dev_alloc((void**)&t->fcount_snap, 8));
    RCCHK(dev_alloc((void**)&t->L, sizeof(FrtLedgerDev)));
    RCCHK(dev_alloc((void**)&t->L_snap, sizeof(FrtLedgerDev)));
    RCCHK(dev_alloc(&t->gam[0], s->ncell * s->rs));
    RCCHK(dev_alloc((void**)&t->src_pos, 24));
    RCCHK(dev_alloc((void**)&t->spec, 4 * nb));
    RCCHK(dev_alloc((void**)&t->specd, 8 * nb));
    RCCHK(dev_alloc((void**)&t->quat, 32));
    RCCHK(alloc_recs(t->F[0], 1, nb, s->rs));
    RCCHK(alloc_recs(t->F[1], 1, nb, s->rs));
    if (s->front) RCCHK(dev_alloc((void**)&t->front, s->ncell * 8));
    const double pos_cells[3] = {o_cm[0] / s->dx, o_cm[1] / s->dx, o_cm[2] / s->dx};
    std::vector<float> spec(nb);
    std::vector<double> specd(nb);
    for (int b = 0; b < nb; b++) {
        specd[b] = N[b] / Rref;
        spec[b] = (float)specd[b];
    }
    const double q1[4] = {1, 0, 0, 0};
    RCCHK(scopy(t.get(), t->src_pos, pos_cells, 24, hipMemcpyHostToDevice));
    RCCHK(scopy(t.get(), t->spec, spec.data(), 4 * nb, hipMemcpyHostToDevice));
    RCCHK(scopy(t.get(), t->specd, specd.data(), 8 * nb, hipMemcpyHostToDevice));
    RCCHK(scopy(t.get(), t->quat, q1, 32, hipMemcpyHostToDevice));
    RCCHK(sset(t.get(), t->gam[0], 0, s->ncell * s->rs));
    RCCHK(sset(t.get(), t->L, 0, sizeof(FrtLedgerDev)));
    if (t->front) RCCHK(sset(t.get(), t->front, 0, s->ncell * 8));
    const uint32_t fc[2] = {inside ? 1u : 0u, 0u};
    RCCHK(scopy(t.get(), t->fcount, fc, 8, hipMemcpyHostToDevice));
    if (inside) {
        const uint32_t key = (uint32_t)((c[0] >> s->bsh[0]) + s->bpx * ((c[1] >> s->bsh[1]) + s->bpy * (c[2] >> s->bsh[2])));
        const uint32_t cell = (uint32_t)c[0] | ((uint32_t)c[1] << 11) | ((uint32_t)c[2] << 22);
        if (s->fp64) {
            FrtRec<double> r{};
            r.src = 0; r.estep = 0; r.lp = 12u << 28; r.cell = cell; r.key = key;
            r.r = 0; r.rstop = HUGE_VAL; r.w0 = 1.0;
            for (int a = 0; a < 3; a++) r.dir[a] = d[a];
            RCCHK(scopy(t.get(), t->F[0].rec, &r, sizeof(r), hipMemcpyHostToDevice));
        } else {
            FrtRec<float> r{};
            r.src = 0; r.estep = 0; r.lp = 12u << 28; r.cell = cell; r.key = key;
            r.r = 0.f; r.rstop = HUGE_VALF; r.w0 = 1.f;
            for (int a = 0; a < 3; a++) r.dir[a] = (float)d[a];
            RCCHK(scopy(t.get(), t->F[0].rec, &r, sizeof(r), hipMemcpyHostToDevice));
        }
    }
    FrtSolveDesc& h = t->h;
    h.n_src = 1;
    h.ncast = 0;                 // nothing is cast: the queue holds the one packet
    h.floor = 0.f;
    h.r_cap = HUGE_VAL;
    h.R_ref = Rref;
    h.src_pos = t->src_pos;
    h.spec = t->spec;
    h.specd = t->specd;
    h.quat = t->quat;
    h.quat_steps = 1;
    h.user_u = nullptr;
    h.user_steps = 0;
    h.F[0] = t->F[0];
    h.F[1] = t->F[1];
    h.fcount = t->fcount;
    h.fcount_snap = t->fcount_snap;
    h.L = t->L;
    h.L_snap = t->L_snap;
    h.gamma[0] = t->gam[0];
    h.gamma[1] = t->gam[0];
    h.front = t->front;
    h.xavg = nullptr;
    h.merge = 0;
    t->step = 0;
    set_step_fields(t.get(), dt);
    h.budget = HUGE_VAL;
    // the one packet has weight 1 and photon rates of at most 1 per bin: the
    // fixed-point deposit scale of the brightest packet is that of this one
    double kmax = 0.0;
    for (int b = 0; b < nb; b++) kmax = std::max(kmax, h.Kd[b]);
    h.dep_scale = (float)(std::ldexp(1.0, 46) / (h.has_sub ? 2.0 * kmax * nb : (double)nb));
    Workspace& ws = s->ctx->ws;
    frt_solve one = t.get();
    uint32_t nkeys = 0;
    uint64_t want_p = 0;
    RCCHK(group_sizes(&one, 1, &nkeys, &want_p));
    RCCHK(ensure_ws(ws, s->fp64, nb, 1, nkeys, std::max<uint64_t>(ws.pcap, 4096)));
    Group g;
    plan_group(ws, &one, 1, g);
    hipStream_t st = s->stream;
    RCCHK(upload_group(ws, g, 1, st));
    FrtWS w = g.w;
    hipError_t e;
    w.out = 0;
    if ((e = frt::launch_clear(w, CLEAR_ALL, st)) != hipSuccess) return fail(FRT_EDEVICE, "clear: %s", hipGetErrorString(e));
    if ((e = frt::launch_seed(ws.descs, w, s->fp64, st)) != hipSuccess) return fail(FRT_EDEVICE, "seed: %s", hipGetErrorString(e));
    for (int p = 0; p < g.passes; p++) {
        w.out = (p + 1) & 1;
        for (int part = 0; part < 3; part++)
            if ((e = frt::launch_pass(ws.descs, w, s->fp64, part, st)) != hipSuccess)
                return fail(FRT_EDEVICE, "pass: %s", hipGetErrorString(e));
    }
    if ((e = frt::launch_finish(ws.descs, w, st)) != hipSuccess) return fail(FRT_EDEVICE, "finish: %s", hipGetErrorString(e));
    FrtLedgerDev L;
    RCCHK(read_device_ledger(t.get(), &L));
    if (L.err_flags) return fail(FRT_EDEVICE, "debug cast raised device error bits 0x%x", L.err_flags);
    *absorbed = L.absorbed_HI + L.absorbed_sub + L.absorbed_front;
    *escaped = L.escaped + (inside ? 0.0 : total);
    *crossings = L.crossings;
    if (gamma_out) {
        const size_t n = s->ncell;
        const hipMemcpyKind k = kind == FRT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (!s->fp64) {
            RCCHK(scopy(t.get(), gamma_out, t->gam[0], n * 4, k));
        } else {
            std::vector<double> tmp(n);
            RCCHK(scopy(t.get(), tmp.data(), t->gam[0], n * 8, hipMemcpyDeviceToHost));
            std::vector<float> f(n);
            for (size_t i = 0; i < n; i++) f[i] = (float)tmp[i];
            if (kind == FRT_DEVICE) RCCHK(scopy(t.get(), gamma_out, f.data(), n * 4, hipMemcpyHostToDevice));
            else std::memcpy(gamma_out, f.data(), n * 4);
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    return FRT_OK;
}

int check_tuning(const frt_tuning* t)
{
    if (!t || t->size != sizeof(frt_tuning)) return fail(FRT_EINVAL, "frt_tuning.size must be sizeof(frt_tuning)");
    if (t->item_rays < 64 || t->item_rays > (int)FRT_ITEM_RAYS || t->item_rays % 64)
        return fail(FRT_EINVAL, "item_rays %d must be a multiple of 64 in 64..%u", t->item_rays, FRT_ITEM_RAYS);
    if (t->scatter_blocks_per_cu < 1 || t->scatter_blocks_per_cu > 16)
        return fail(FRT_EINVAL, "scatter workgroups per CU must be in 1..16");
    return FRT_OK;
}

}  // namespace

namespace frt {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int use_device(int device)
{
    HIPCHK(hipSetDevice(device));
    return FRT_OK;
}

int copy_device_to_host(void* dst, const void* src, size_t bytes)
{
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    return FRT_OK;
}

double clock_s()
{
    static const auto t0 = std::chrono::steady_clock::now();
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int ctx_device(frt_ctx ctx) { return ctx->device; }

uint64_t solve_bytes(const frt_params& P, uint64_t ncell, int n_src, int with_T, uint64_t* pass_records,
                     uint64_t* pass_bytes)
{
    const uint64_t rs = P.march_precision == FRT_F64 ? 8 : 4;
    const uint64_t rec = rec_bytes(rs);
    const uint64_t cast = (uint64_t)n_src * (12ull << (2 * P.base_level));
    // resident fields: opacity pair, two rate buffers, x_HI, n_H, T, <x> of
    // the time-averaged chemistry, front photons of the Generalized Opacity
    // Mode, photo-heating of the temperature evolution
    uint64_t b = ncell * (4 * rs + 16 + ((with_T || P.temperature) ? 8 : 0) + (P.chem_iterations > 0 ? 8 : 0) +
                          (P.opacity_mode == FRT_GENERALIZED ? 8 : 0) +
                          ((P.temperature && P.opacity_mode == FRT_STANDARD) ? rs : 0));
    // carried-packet queues (as first sized)
    double F = (double)cast + 1024;
    if (std::isfinite(P.c_ray_cm_s)) F += std::min((double)ncell, 8.0 * cast + 65536.0);
    if (P.queue_capacity) F = (double)P.queue_capacity;
    b += 2 * (uint64_t)F * rec;
    // sources, photon rates, 64 steps of rotations, ledgers
    b += (uint64_t)n_src * (24 + 12 * (uint64_t)P.n_bins) + 64ull * n_src * 32 + 2 * sizeof(FrtLedgerDev);
    // share of the pass queues: two output buffers with their keys, the
    // sorted index, work list
    const uint64_t wp = P.queue_capacity ? P.queue_capacity
                                         : (P.queue_hint ? P.queue_hint : std::max<uint64_t>(4 * cast + 65536, ncell / 2));
    if (pass_records) *pass_records = wp;
    // brick keys: at most one per 8^3 cells (the smallest brick)
    const uint64_t pq = pass_queue_bytes(wp, rs, ncell / 512 + 1);
    if (pass_bytes) *pass_bytes = pq;
    return b + pq;
}

uint64_t ctx_workspace_bytes(frt_ctx ctx)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    return ctx->ws.bytes();
}

void ctx_set_workspace_limit(frt_ctx ctx, uint64_t bytes)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->ws.limit = bytes;
}

void ctx_trim_workspace(frt_ctx ctx)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    (void)hipDeviceSynchronize();
    ctx->ws.free_pass();
    dev_free(ctx->ws.work);
    ctx->ws.cap_work = 0;
}

}  // namespace frt

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
    p->queue_hint = 0;
    p->merge = 0;
    p->merge_level = 0;
    p->merge_exempt = 4.0;
    p->temperature = 0;
    p->hubble_s = 0.0;
    p->cmb_z = -1.0;
    p->t_reion_k = 2e4;
    p->spectral_index = 1.5;
    return FRT_OK;
}

int frt_ctx_create(int hip_device, frt_alloc_fn alloc_fn, frt_free_fn free_fn, void* user, frt_ctx* out)
{
    if (!out) return fail(FRT_EINVAL, "null output");
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return fail(FRT_EINVAL, "give both allocator hooks or neither");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(FRT_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= n) return fail(FRT_EINVAL, "device %d out of range [0,%d)", hip_device, n);
    HIPCHK(hipSetDevice(hip_device));
    // the allocation-free step's scratch: its device address on this device
    void* scratch = nullptr;
    const hipError_t es = frt::static_scratch(hip_device, &scratch);
    if (es != hipSuccess) return fail(FRT_EDEVICE, "static scratch lookup: %s", hipGetErrorString(es));
    frt_ctx c = new (std::nothrow) frt_ctx_s;
    if (!c) return fail(FRT_ENOMEM, "context");
    c->device = hip_device;
    c->al.alloc = alloc_fn;
    c->al.release = free_fn;
    c->al.user = user;
    *out = c;
    return FRT_OK;
}

int frt_ctx_destroy(frt_ctx ctx)
{
    if (ctx) (void)hipDeviceSynchronize();
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
    if (P->max_level < P->base_level || P->max_level > 12) return fail(FRT_EINVAL, "max_level %d outside base_level..12", P->max_level);
    if (!(P->n_ray_min > 0) || !std::isfinite(P->n_ray_min)) return fail(FRT_EINVAL, "n_ray_min must be finite and > 0");
    if (!(P->alpha_B >= 0) || !(P->coll_ion >= 0) || !std::isfinite(P->alpha_B) || !std::isfinite(P->coll_ion))
        return fail(FRT_EINVAL, "alpha_B and coll_ion must be finite and >= 0");
    if (!(P->flux_floor >= 0 && P->flux_floor < 1)) return fail(FRT_EINVAL, "flux_floor must lie in [0,1)");
    if (!(P->max_distance_cm >= 0) || !std::isfinite(P->max_distance_cm)) return fail(FRT_EINVAL, "max_distance_cm must be finite and >= 0");
    if (!(P->c_ray_cm_s > 0)) return fail(FRT_EINVAL, "c_ray_cm_s must be > 0 (or +inf)");
    if (P->march_precision != FRT_F32 && P->march_precision != FRT_F64) return fail(FRT_EINVAL, "march_precision must be FRT_F32 or FRT_F64");
    if (P->chem_iterations < 0 || P->chem_iterations > FRT_MAX_CHEM_ITERATIONS)
        return fail(FRT_EINVAL, "chem_iterations %d outside 0..%d", P->chem_iterations, FRT_MAX_CHEM_ITERATIONS);
    if (P->opacity_mode != FRT_STANDARD && P->opacity_mode != FRT_GENERALIZED)
        return fail(FRT_EINVAL, "opacity_mode must be FRT_STANDARD or FRT_GENERALIZED");
    if (!(P->he_chi >= 0) || !std::isfinite(P->he_chi)) return fail(FRT_EINVAL, "he_chi must be finite and >= 0");
    if (P->merge != 0 && P->merge != 1) return fail(FRT_EINVAL, "merge must be 0 or 1");
    if (P->merge_level < 0 || P->merge_level > 8) return fail(FRT_EINVAL, "merge_level %d outside 0..8", P->merge_level);
    if (!(P->merge_exempt >= 0) || !std::isfinite(P->merge_exempt)) return fail(FRT_EINVAL, "merge_exempt must be finite and >= 0");
    if (P->temperature != 0 && P->temperature != 1) return fail(FRT_EINVAL, "temperature must be 0 or 1");
    if (!(P->t_reion_k > 0) || !std::isfinite(P->t_reion_k)) return fail(FRT_EINVAL, "t_reion_k must be finite and > 0");
    if (!(P->spectral_index >= 0) || !std::isfinite(P->spectral_index))
        return fail(FRT_EINVAL, "spectral_index must be finite and >= 0");
    for (int b = 0; b < P->n_bins; b++)
        if (!(P->heat_ev[b] >= 0) || !std::isfinite(P->heat_ev[b])) return fail(FRT_EINVAL, "heat_ev[%d] must be finite and >= 0", b);
    if (!(P->hubble_s >= 0) || !std::isfinite(P->hubble_s)) return fail(FRT_EINVAL, "hubble_s must be finite and >= 0");
    if (!std::isfinite(P->cmb_z)) return fail(FRT_EINVAL, "cmb_z must be finite");
    AllocScope scope(&ctx->al);
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
    if (P->merge && ((rc = dev_alloc((void**)&s->vcount, 8)) || (rc = dev_alloc((void**)&s->w0_merged, 4)))) {
        delete s;
        return rc;
    }
    if ((rc = dev_alloc((void**)&s->d_desc, sizeof(FrtSolveDesc))) || (rc = dev_alloc((void**)&s->fcount, 8)) ||
        (rc = dev_alloc((void**)&s->fcount_snap, 8)) || (rc = dev_alloc((void**)&s->L, sizeof(FrtLedgerDev))) ||
        (rc = dev_alloc((void**)&s->L_snap, sizeof(FrtLedgerDev)))) {
        delete s;
        return rc;
    }
    HIPCHK(hipMemsetAsync(s->fcount, 0, 8, s->stream));
    HIPCHK(hipMemsetAsync(s->L, 0, sizeof(FrtLedgerDev), s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    FrtSolveDesc& h = s->h;
    std::memset(&h, 0, sizeof(h));
    h.n_bins = P->n_bins;
    h.base_level = P->base_level;
    h.max_level = P->max_level;
    h.fp64 = s->fp64;
    for (int a = 0; a < 3; a++) h.bsh[a] = s->bsh[a];
    h.ncast = 12u << (2 * P->base_level);
    h.sigma0 = P->sigma_bins[0];
    for (int b = 0; b < P->n_bins; b++) {
        h.sig_rel[b] = (float)(P->sigma_bins[b] / P->sigma_bins[0]);
        h.sig_reld[b] = P->sigma_bins[b] / P->sigma_bins[0];
        h.sig_l2[b] = (float)(-1.4426950408889634 * P->sigma_bins[b] / P->sigma_bins[0]);
    }
    h.r_split0 = std::sqrt(3.0 / (PI * P->n_ray_min));
    h.floor = (float)P->flux_floor;
    h.alpha_B = P->alpha_B;
    h.coll_ion = P->coll_ion;
    h.seed = P->seed;
    h.fcount = s->fcount;
    h.L = s->L;
    h.fcount_snap = s->fcount_snap;
    h.L_snap = s->L_snap;
    h.merge = P->merge;
    h.vcount = s->vcount;
    h.w0_merged = s->w0_merged;
    if (P->merge) {
        HIPCHK(hipMemsetAsync(s->vcount, 0, 8, s->stream));
        HIPCHK(hipMemsetAsync(s->w0_merged, 0, 4, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
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
    if ((uint64_t)nx * ny * nz >= 0xffffffffull) return fail(FRT_EINVAL, "grid of %llu cells exceeds 2^32 - 1", (unsigned long long)nx * ny * nz);
    if (!(box_cm > 0) || !std::isfinite(box_cm)) return fail(FRT_EINVAL, "box_cm must be finite and > 0");
    if (!n_H) return fail(FRT_EINVAL, "n_H is required");
    if (kind != FRT_HOST && kind != FRT_DEVICE) return fail(FRT_EINVAL, "ptr_kind must be FRT_HOST or FRT_DEVICE");
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    const size_t n = (size_t)nx * ny * nz;
    AllocScope scope(&s->ctx->al);
    std::vector<float> bn, bk, bT;
    std::vector<double> bx;
    const float *hn = nullptr, *hk = nullptr, *hT = nullptr;
    const double* hx = nullptr;
    RCCHK(host_view(n_H, n, kind, bn, &hn));
    RCCHK(check_inputs_finite(hn, n, "n_H"));
    if (kappa) {
        RCCHK(host_view(kappa, n, kind, bk, &hk));
        RCCHK(check_inputs_finite(hk, n, "kappa_sub"));
    }
    if (x0) {
        RCCHK(host_view(x0, n, kind, bx, &hx));
        for (size_t i = 0; i < n; i++)
            if (!(hx[i] >= 0.0 && hx[i] <= 1.0)) return fail(FRT_EINVAL, "x_HI0[%zu] = %g outside [0,1]", i, hx[i]);
    }
    if (T) {
        RCCHK(host_view(T, n, kind, bT, &hT));
        for (size_t i = 0; i < n; i++)
            if (!(hT[i] > 0.f) || !std::isfinite(hT[i])) return fail(FRT_EINVAL, "T[%zu] = %g is not finite and > 0", i, (double)hT[i]);
    }
    const bool temp = s->P.temperature != 0;
    dev_free(s->heat); dev_free(s->mark_T);
    dev_free(s->op); dev_free(s->gam[0]); dev_free(s->gam[1]); dev_free(s->x); dev_free(s->xavg);
    dev_free(s->front); dev_free(s->nH); dev_free(s->T); dev_free(s->kin); dev_free(s->mark_g);
    const bool gen = s->P.opacity_mode == FRT_GENERALIZED;
    RCCHK(dev_alloc(&s->op, n * 2 * s->rs));
    RCCHK(dev_alloc(&s->gam[0], n * s->rs));
    RCCHK(dev_alloc(&s->gam[1], n * s->rs));
    RCCHK(dev_alloc((void**)&s->x, n * 8));
    if (s->P.chem_iterations > 0) RCCHK(dev_alloc((void**)&s->xavg, n * 8));
    if (gen) RCCHK(dev_alloc((void**)&s->front, n * 8));
    RCCHK(dev_alloc((void**)&s->nH, n * 8));
    if (T || temp) RCCHK(dev_alloc((void**)&s->T, n * 8));
    if (temp && !gen) RCCHK(dev_alloc(&s->heat, n * s->rs));   // the march's photo-heating
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->ncell = n;
    s->dx = box_cm / nx;
    // brick shape: 8^3 in FP64; in FP32 16^3 with sub-grid opacity (and in
    // the Generalized Opacity Mode, which stages the same pairs, and with the
    // temperature on, whose heating march uses that layout), else
    // 32 x 16 x 16 (the 1024-thread march)
    const bool any_kappa = gen || temp || (hk && std::any_of(hk, hk + n, [](float v) { return v > 0.f; }));
    const int* lg = s->fp64 ? FRT_BRICK_LOG_F64 : (any_kappa ? FRT_BRICK_LOG_SUB : FRT_BRICK_LOG_BIG);
    for (int a = 0; a < 3; a++) s->bsh[a] = lg[a];
    s->bpx = (nx + (1 << s->bsh[0]) - 1) >> s->bsh[0];
    s->bpy = (ny + (1 << s->bsh[1]) - 1) >> s->bsh[1];
    s->bpz = (nz + (1 << s->bsh[2]) - 1) >> s->bsh[2];
    std::vector<double> nHd(n), xd(n, 1.0);
    for (size_t i = 0; i < n; i++) nHd[i] = (double)hn[i];
    s->nH_mean = mean_of(nHd);
    if (hx) std::copy(hx, hx + n, xd.begin());
    // opacity: the HI part (first n values) is built from x_HI on the device;
    // the sub-grid part (next n values) is fixed.  Generalized Opacity Mode:
    // the first part is the ionized gas's kappa dx (fixed, floored like the
    // HI opacity), the second the ionized fraction, built on the device
    const double floor_a = s->fp64 ? 1e-300 : 1e-30;
    if (s->fp64) {
        std::vector<double> opv(2 * n, 0.0);
        if (hk)
            for (size_t i = 0; i < n; i++) opv[(gen ? 0 : n) + i] = (double)hk[i] * s->dx;
        if (gen)
            for (size_t i = 0; i < n; i++) opv[i] = std::max(opv[i], floor_a);
        RCCHK(scopy(s, s->op, opv.data(), n * 16, hipMemcpyHostToDevice));
    } else {
        std::vector<float> opv(2 * n, 0.f);
        if (hk)
            for (size_t i = 0; i < n; i++) opv[(gen ? 0 : n) + i] = (float)((double)hk[i] * s->dx);
        if (gen)
            for (size_t i = 0; i < n; i++) opv[i] = std::max(opv[i], (float)floor_a);
        RCCHK(scopy(s, s->op, opv.data(), n * 8, hipMemcpyHostToDevice));
    }
    if (gen) RCCHK(sset(s, s->front, 0, n * 8));
    if (warm_rate(s)) {
        // the input kappa dx, from which each march's opacity is rebuilt
        RCCHK(dev_alloc(&s->kin, n * s->rs));
        HIPCHK(hipMemcpyAsync(s->kin, s->op, n * s->rs, hipMemcpyDeviceToDevice, s->stream));
    }
    RCCHK(scopy(s, s->nH, nHd.data(), n * 8, hipMemcpyHostToDevice));
    RCCHK(scopy(s, s->x, xd.data(), n * 8, hipMemcpyHostToDevice));
    if (T || temp) {
        std::vector<double> Td(n, 1e4);
        if (hT)
            for (size_t i = 0; i < n; i++) Td[i] = (double)hT[i];
        RCCHK(scopy(s, s->T, Td.data(), n * 8, hipMemcpyHostToDevice));
    }
    if (s->heat) RCCHK(sset(s, s->heat, 0, n * s->rs));
    RCCHK(sset(s, s->gam[0], 0, n * s->rs));
    RCCHK(sset(s, s->gam[1], 0, n * s->rs));
    if (s->vcount) RCCHK(sset(s, s->vcount, 0, 8));
    RCCHK(sset(s, s->fcount, 0, 8));
    RCCHK(sset(s, s->L, 0, sizeof(FrtLedgerDev)));
    FrtSolveDesc& h = s->h;
    h.nx = nx; h.ny = ny; h.nz = nz;
    h.has_sub = (gen || temp) ? 1 : 0;
    if (hk)
        for (size_t i = 0; i < n && !h.has_sub; i++) h.has_sub = hk[i] > 0.f;
    h.temp = temp ? 1 : 0;
    h.T = temp ? s->T : nullptr;
    h.heat = s->heat;
    for (int b = 0; b < FRT_MAX_BINS_I; b++) h.heat_ev[b] = (b < s->P.n_bins && !gen) ? s->P.heat_ev[b] : 0.0;
    h.hubble = s->P.hubble_s;
    h.cmb_z = s->P.cmb_z;
    h.t_reion = s->P.t_reion_k;
    h.heat_rec = reion_heat_per_recombination(s->P.spectral_index);
    h.gen = gen ? 1 : 0;
    h.front_atoms = (1.0 + s->P.he_chi) * s->dx * s->dx * s->dx;
    h.front = s->front;
    h.kin = s->kin;
    h.bpx = s->bpx; h.bpy = s->bpy; h.bpz = s->bpz;
    for (int a = 0; a < 3; a++) h.bsh[a] = s->bsh[a];
    h.dx_cm = s->dx;
    h.r_cap = s->P.max_distance_cm > 0 ? s->P.max_distance_cm / s->dx : HUGE_VAL;
    h.op_a = s->op;
    h.op_b = (const char*)s->op + n * s->rs;
    h.op_aw = s->op;
    h.op_bw = (char*)s->op + n * s->rs;
    h.gamma[0] = s->gam[0];
    h.gamma[1] = s->gam[1];
    h.x = s->x;
    h.xavg = s->xavg;
    h.nH = s->nH;
    s->step = 0;
    s->have_grid = true;
    s->have_src = false;   // sources are checked against the new box
    RCCHK(upload_desc(s));
    hipError_t e = frt::launch_prep_opacity(s->d_desc, n, s->fp64, s->stream);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "prep launch: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int frt_set_opacity(frt_solve s, const float* kappa, int kind)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid) return fail(FRT_ESTATE, "load the grid before its opacity");
    if (!kappa) return fail(FRT_EINVAL, "null kappa");
    const bool gen = s->P.opacity_mode == FRT_GENERALIZED;
    if (!gen && !s->h.has_sub)
        return fail(FRT_EINVAL, "the grid was loaded without sub-grid opacity (its march has no kappa term)");
    HIPCHK(hipSetDevice(s->ctx->device));
    const size_t n = s->ncell;
    std::vector<float> bk;
    const float* hk = nullptr;
    RCCHK(host_view(kappa, n, kind, bk, &hk));
    RCCHK(check_inputs_finite(hk, n, "kappa"));
    for (size_t i = 0; i < n; i++)
        if (hk[i] < 0.f) return fail(FRT_EINVAL, "kappa[%zu] < 0", i);
    // the kappa half of the opacity pair: the first in the Generalized
    // Opacity Mode (floored like the HI opacity), else the second
    char* dst = (char*)s->op + (gen ? 0 : n * s->rs);
    const double floor_a = s->fp64 ? 1e-300 : 1e-30;
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->fp64) {
        std::vector<double> v(n);
        for (size_t i = 0; i < n; i++) {
            v[i] = (double)hk[i] * s->dx;
            if (gen) v[i] = std::max(v[i], floor_a);
        }
        RCCHK(scopy(s, dst, v.data(), n * 8, hipMemcpyHostToDevice));
        if (s->kin) RCCHK(scopy(s, s->kin, v.data(), n * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> v(n);
        for (size_t i = 0; i < n; i++) {
            v[i] = (float)((double)hk[i] * s->dx);
            if (gen) v[i] = std::max(v[i], (float)floor_a);
        }
        RCCHK(scopy(s, dst, v.data(), n * 4, hipMemcpyHostToDevice));
        if (s->kin) RCCHK(scopy(s, s->kin, v.data(), n * 4, hipMemcpyHostToDevice));
    }
    return FRT_OK;
}

int frt_set_density(frt_solve s, const float* n_H, int kind)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid) return fail(FRT_ESTATE, "load the grid before a new density");
    if (!n_H) return fail(FRT_EINVAL, "null n_H");
    if (kind != FRT_HOST && kind != FRT_DEVICE) return fail(FRT_EINVAL, "ptr_kind must be FRT_HOST or FRT_DEVICE");
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    const size_t n = s->ncell;
    AllocScope scope(&s->ctx->al);
    std::vector<float> bn;
    const float* hn = nullptr;
    RCCHK(host_view(n_H, n, kind, bn, &hn));
    RCCHK(check_inputs_finite(hn, n, "n_H"));
    std::vector<double> nd(n);
    for (size_t i = 0; i < n; i++) nd[i] = (double)hn[i];
    const double m1 = mean_of(nd);
    if (!(m1 > 0.0)) return fail(FRT_EINVAL, "the new density's mean must be > 0");
    if (!(s->nH_mean > 0.0)) return fail(FRT_ESTATE, "the loaded density's mean is 0: load a grid instead");
    double* dn = nullptr;
    RCCHK(dev_alloc((void**)&dn, n * 8));
    int rc = scopy(s, dn, nd.data(), n * 8, hipMemcpyHostToDevice);
    if (rc == FRT_OK) {
        hipError_t e = frt::launch_set_density(s->nH, dn, s->h.temp ? s->T : nullptr, s->nH_mean, m1, n, s->stream);
        if (e == hipSuccess) e = frt::launch_prep_opacity(s->d_desc, n, s->fp64, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) rc = fail(FRT_EDEVICE, "density update: %s", hipGetErrorString(e));
    }
    dev_free(dn);
    if (rc == FRT_OK) s->nH_mean = m1;
    return rc;
}

int frt_load_sources(frt_solve s, int n_src, const double* pos_cm, const double* ndot, int kind)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid) return fail(FRT_ESTATE, "load the grid before the sources");
    if (n_src < 0) return fail(FRT_EINVAL, "n_src < 0");
    if (n_src > 0 && (!pos_cm || !ndot)) return fail(FRT_EINVAL, "null source arrays");
    AllocScope scope(&s->ctx->al);
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    const int nb = s->P.n_bins;
    std::vector<double> bp, bd;
    const double *hp = nullptr, *hd = nullptr;
    if (n_src > 0) {
        RCCHK(host_view(pos_cm, (size_t)n_src * 3, kind, bp, &hp));
        RCCHK(host_view(ndot, (size_t)n_src * nb, kind, bd, &hd));
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
    dev_free(s->src_pos); dev_free(s->spec); dev_free(s->specd); dev_free(s->quat); dev_free(s->user_u);
    s->quat_steps = 0;
    s->user_steps = 0;
    s->n_src = n_src;
    RCCHK(dev_alloc((void**)&s->src_pos, pos_cells.size() * 8));
    RCCHK(dev_alloc((void**)&s->spec, spec.size() * 4));
    RCCHK(dev_alloc((void**)&s->specd, specd.size() * 8));
    RCCHK(scopy(s, s->src_pos, pos_cells.data(), pos_cells.size() * 8, hipMemcpyHostToDevice));
    RCCHK(scopy(s, s->spec, spec.data(), spec.size() * 4, hipMemcpyHostToDevice));
    RCCHK(scopy(s, s->specd, specd.data(), specd.size() * 8, hipMemcpyHostToDevice));
    FrtSolveDesc& h = s->h;
    h.n_src = n_src;
    h.R_ref = R_ref;
    h.src_pos = s->src_pos;
    h.spec = s->spec;
    h.specd = s->specd;
    h.user_u = nullptr;
    h.user_steps = 0;
    free_recs(s->F[0]);
    free_recs(s->F[1]);
    s->w0_max = 0;   // no packet is held
    const uint32_t fcap = initial_fcap(s);
    RCCHK(alloc_recs(s->F[0], fcap, nb, s->rs));
    RCCHK(alloc_recs(s->F[1], fcap, nb, s->rs));
    h.F[0] = s->F[0];
    h.F[1] = s->F[1];
    RCCHK(ensure_quat(s, 0));
    RCCHK(sset(s, s->fcount, 0, 8));
    RCCHK(sset(s, s->L, 0, sizeof(FrtLedgerDev)));
    if (s->P.merge) {
        RCCHK(sset(s, s->vcount, 0, 8));
        RCCHK(sset(s, s->w0_merged, 0, 4));
    }
    s->step = 0;
    s->have_src = true;
    RCCHK(upload_desc(s));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int frt_set_rotations(frt_solve s, int n_steps, const double* u)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_src) return fail(FRT_ESTATE, "load the sources before the rotation table");
    if (n_steps < 0 || (n_steps > 0 && !u)) return fail(FRT_EINVAL, "bad rotation table");
    AllocScope scope(&s->ctx->al);
    const size_t n = (size_t)n_steps * s->n_src * 3;
    for (size_t i = 0; i < n; i++)
        if (!(u[i] >= 0.0 && u[i] < 1.0)) return fail(FRT_EINVAL, "uniform %zu = %g outside [0,1)", i, u[i]);
    HIPCHK(hipStreamSynchronize(s->stream));
    dev_free(s->user_u);
    RCCHK(dev_alloc((void**)&s->user_u, std::max<size_t>(n, 1) * 8));
    if (n) RCCHK(scopy(s, s->user_u, u, n * 8, hipMemcpyHostToDevice));
    s->user_steps = (uint32_t)n_steps;
    s->h.user_u = s->user_u;
    s->h.user_steps = s->user_steps;
    return upload_desc(s);
}

int frt_step(frt_solve s, double dt)
{
    RCCHK(ready(s));
    AllocScope scope(&s->ctx->al);
    if (!(dt > 0) || !std::isfinite(dt)) return fail(FRT_EINVAL, "dt must be finite and > 0");
    HIPCHK(hipSetDevice(s->ctx->device));
    return step_group(&s, 1, &dt);
}

int frt_step_static(frt_solve s, double dt)
{
    RCCHK(ready(s));
    if (!(dt > 0) || !std::isfinite(dt)) return fail(FRT_EINVAL, "dt must be finite and > 0");
    HIPCHK(hipSetDevice(s->ctx->device));
    if (s->step >= s->quat_steps)
        return fail(FRT_ESTATE, "the solve's rotation table holds %u steps; an allocating call (frt_step) extends it",
                    s->quat_steps);
    if (s->P.merge) return fail(FRT_EINVAL, "the allocation-free step does not merge packets (frt_step does)");
    const uint64_t nkeys = (uint64_t)s->bpx * s->bpy * s->bpz;
    if (nkeys > FRT_STATIC_MAX_KEYS)
        return fail(FRT_EINVAL, "the grid holds %llu bricks; the allocation-free step takes at most %u",
                    (unsigned long long)nkeys, FRT_STATIC_MAX_KEYS);
    void* base = nullptr;
    const hipError_t es = frt::static_scratch(s->ctx->device, &base);
    if (es != hipSuccess) return fail(FRT_EDEVICE, "static scratch lookup: %s", hipGetErrorString(es));
    // every call in this process shares the array: one at a time, each to its end
    static std::mutex scratch_mu;
    std::lock_guard<std::mutex> lock(scratch_mu);
    // the smallest work items: a pass of a small solve is then spread over
    // many workgroups, and so over all the output segments (each holds a
    // 64th of the queue)
    Workspace sw;
    sw.tune.item_rays = 64;
    sw.tune.scatter_blocks_per_cu = 8;
    sw.fp64 = s->fp64;
    sw.nb = s->P.n_bins;
    // carve the scratch: small tables first, then the march scratch records,
    // then the pass queues in what is left
    const size_t rb = rec_bytes(s->rs);
    char* p = (char*)base;
    size_t left = FRT_STATIC_SCRATCH_BYTES;
    auto take = [&](size_t bytes) -> void* {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes > left) return nullptr;
        void* q = p;
        p += bytes;
        left -= bytes;
        return q;
    };
    sw.descs = (FrtSolveDesc*)take(sizeof(FrtSolveDesc));
    sw.solves_cap = 1;
    sw.key_prefix = (uint32_t*)take(8);
    sw.seed_prefix = (uint32_t*)take(8);
    sw.cell_prefix = (unsigned long long*)take(16);
    sw.ctr = (uint32_t*)take(C_NCTR * 4);
    sw.segc = (uint32_t*)take((size_t)FRT_QSEG * FRT_QSEG_STRIDE * 4);
    sw.segp = (uint32_t*)take((FRT_QSEG + 1) * 4);
    sw.hist = (uint32_t*)take(FRT_STATIC_MAX_KEYS * 4);
    sw.cursor = (uint32_t*)take(FRT_STATIC_MAX_KEYS * 4);
    sw.nkeys_cap = FRT_STATIC_MAX_KEYS;
    const uint32_t xcap = (uint32_t)frt::device_cu_count() * FRT_STATIC_XREC_PER_CU;
    sw.X.rec = take((size_t)xcap * rb);
    sw.X.cap = xcap;
    // pass queues: per record two output records, two keys, a sorted entry
    // and a share of the work list (items of at least 64 packets, plus one
    // per brick)
    const size_t work_fixed = ((size_t)FRT_STATIC_MAX_KEYS + 64) * sizeof(FrtWork) + 6 * 256;
    if (!sw.X.rec || left < work_fixed) return fail(FRT_EINVAL, "static scratch too small");
    const size_t per = 2 * rb + 2 * 4 + sizeof(uint2) + sizeof(FrtWork) / 64 + 1;
    const uint32_t pcap = (uint32_t)((left - work_fixed) / per);
    sw.pcap = pcap;
    for (int k = 0; k < 2; k++) {
        sw.O[k].rec = take((size_t)pcap * rb);
        sw.O[k].cap = pcap;
        sw.okey[k] = (uint32_t*)take((size_t)pcap * 4);
    }
    sw.sorted = (uint2*)take((size_t)pcap * sizeof(uint2));
    sw.cap_work = pcap / (uint32_t)sw.tune.item_rays + FRT_STATIC_MAX_KEYS + 64;
    sw.work = (FrtWork*)take((size_t)sw.cap_work * sizeof(FrtWork));
    if (!sw.O[0].rec || !sw.O[1].rec || !sw.okey[0] || !sw.okey[1] || !sw.sorted || !sw.work)
        return fail(FRT_EINVAL, "static scratch layout does not fit");
    hipStream_t st = s->stream;
    set_step_fields(s, dt);
    Group g;
    frt_solve one = s;
    plan_group(sw, &one, 1, g);
    RCCHK(upload_group(sw, g, 1, st));
    RCCHK(enqueue_step(sw, &one, 1, g, st, false, false));
    uint32_t ctr[C_NCTR];
    HIPCHK(hipMemcpyAsync(ctr, sw.ctr, sizeof(ctr), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ctr[C_ERR] & (FRT_DEVERR_QUEUE_OVERFLOW | FRT_DEVERR_CARRY_OVERFLOW)) {
        RCCHK(restore_step_start(&one, 1, st));
        if (ctr[C_ERR] & FRT_DEVERR_QUEUE_OVERFLOW)
            return fail(FRT_EOVERFLOW, "a pass of the step needs more than the static scratch's queue (%u packets, a "
                        "64th per output segment; largest pass %u); the step was not applied", pcap, ctr[C_MAXP]);
        return fail(FRT_EOVERFLOW, "the solve's carried-packet queue (%u) is too small for the step; it was not "
                    "applied (frt_step grows it)", s->F[0].cap);
    }
    if (ctr[C_ERR] & FRT_DEVERR_UNFINISHED) return fail(FRT_EDEVICE, "a step left packets after its last pass");
    s->step++;
    return FRT_OK;
}

int frt_batch_step(frt_solve* ss, int n, const double* dts)
{
    RCCHK(check_batch(ss, n, dts));
    AllocScope scope(&ss[0]->ctx->al);
    HIPCHK(hipSetDevice(ss[0]->ctx->device));
    for (int i = 1; i < n; i++) HIPCHK(hipStreamSynchronize(ss[i]->stream));
    RCCHK(step_group(ss, n, dts));
    HIPCHK(hipStreamSynchronize(ss[0]->stream));
    return FRT_OK;
}

int frt_batch_run(frt_solve* ss, int n, const double* dts, int n_steps, int use_graph)
{
    RCCHK(check_batch(ss, n, dts));
    AllocScope scope(&ss[0]->ctx->al);
    if (n_steps < 0) return fail(FRT_EINVAL, "n_steps must be >= 0");
    if (use_graph < 0) return fail(FRT_EINVAL, "use_graph must be >= 0 (0: no graph, w > 0: replays per host check)");
    if (n_steps == 0) return FRT_OK;
    HIPCHK(hipSetDevice(ss[0]->ctx->device));
    for (int i = 0; i < n; i++) HIPCHK(hipStreamSynchronize(ss[i]->stream));
    bool merging = false;
    for (int i = 0; i < n; i++) merging |= ss[i]->P.merge != 0;
    // a merge is sized from the carried count the step leaves, read on the
    // host: groups with merging solves are stepped launch by launch
    if (!use_graph || merging) {
        for (int k = 0; k < n_steps; k++) RCCHK(step_group(ss, n, dts));
    } else {
        std::lock_guard<std::mutex> lock(ss[0]->ctx->mu);
        RCCHK(run_group_graph_locked(ss, n, dts, n_steps, use_graph));
    }
    HIPCHK(hipStreamSynchronize(ss[0]->stream));
    return FRT_OK;
}

int frt_tuning_default(frt_tuning* t)
{
    if (!t) return fail(FRT_EINVAL, "null tuning");
    t->size = sizeof(frt_tuning);
    t->item_rays = (int)FRT_ITEM_RAYS;
    t->scatter_blocks_per_cu = 8;
    return FRT_OK;
}

int frt_ctx_set_tuning(frt_ctx ctx, const frt_tuning* t)
{
    if (!ctx) return fail(FRT_EINVAL, "null context");
    RCCHK(check_tuning(t));
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (t->item_rays < ctx->ws.tune.item_rays) {
        // smaller items need a longer work list: let ensure_ws size it again
        dev_free(ctx->ws.work);
        ctx->ws.cap_work = 0;
    }
    ctx->ws.tune = *t;
    return FRT_OK;
}

int frt_ctx_get_tuning(frt_ctx ctx, frt_tuning* t)
{
    if (!ctx || !t) return fail(FRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(ctx->mu);
    *t = ctx->ws.tune;
    return FRT_OK;
}

int frt_autotune(frt_solve* ss, int n, const double* dts, frt_tuning* best)
{
    RCCHK(check_batch(ss, n, dts));
    if (!best) return fail(FRT_EINVAL, "null output");
    frt_ctx ctx = ss[0]->ctx;
    AllocScope scope(&ctx->al);
    HIPCHK(hipSetDevice(ctx->device));
    for (int i = 0; i < n; i++) HIPCHK(hipStreamSynchronize(ss[i]->stream));
    std::lock_guard<std::mutex> lock(ctx->mu);
    std::vector<SolveSnap> snaps(n);
    struct Release {
        std::vector<SolveSnap>& v;
        ~Release() { for (auto& p : v) p.release(); }
    } rel{snaps};
    for (int i = 0; i < n; i++) RCCHK(snap_take(ss[i], snaps[i]));
    const frt_tuning keep = ctx->ws.tune;
    std::vector<frt_tuning> cand;
    for (int item : {256, 512, 1024})
        for (int sc : {4, 8}) cand.push_back(frt_tuning{sizeof(frt_tuning), item, sc});
    hipStream_t st = ss[0]->stream;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    auto restore_all = [&]() -> int {
        for (int i = 0; i < n; i++) RCCHK(snap_restore(ss[i], snaps[i]));
        return FRT_OK;
    };
    // a first step grows the queues to this group's size
    int rc = step_group_locked(ss, n, dts);
    if (rc == FRT_OK) rc = restore_all();
    float best_ms = -1.f;
    frt_tuning pick = keep;
    for (size_t c = 0; c < cand.size() && rc == FRT_OK; c++) {
        ctx->ws.tune = cand[c];
        if (cand[c].item_rays < keep.item_rays) {
            dev_free(ctx->ws.work);
            ctx->ws.cap_work = 0;
        }
        // the best of three timings of the same step (one step of a small
        // batch lasts a few ms, about as long as the launch jitter)
        float ms = -1.f;
        for (int rep = 0; rep < 3 && rc == FRT_OK; rep++) {
            (void)hipEventRecord(a, st);
            rc = step_group_locked(ss, n, dts);
            (void)hipEventRecord(b, st);
            if (rc != FRT_OK) break;
            (void)hipEventSynchronize(b);
            float t = 0.f;
            (void)hipEventElapsedTime(&t, a, b);
            if (ms < 0.f || t < ms) ms = t;
            rc = restore_all();
        }
        if (rc != FRT_OK) break;
        if (best_ms < 0.f || ms < best_ms) {
            best_ms = ms;
            pick = cand[c];
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    ctx->ws.tune = rc == FRT_OK ? pick : keep;
    dev_free(ctx->ws.work);
    ctx->ws.cap_work = 0;
    if (rc != FRT_OK) {
        (void)restore_all();
        return rc;
    }
    *best = pick;
    return FRT_OK;
}

int frt_sync(frt_solve s)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    HIPCHK(hipStreamSynchronize(s->stream));
    if (!s->L) return FRT_OK;
    FrtLedgerDev L;
    RCCHK(read_device_ledger(s, &L));
    if (L.err_flags & (FRT_DEVERR_QUEUE_OVERFLOW | FRT_DEVERR_CARRY_OVERFLOW))
        return fail(FRT_EOVERFLOW, "a ray queue overflowed; raise queue_capacity");
    if (L.err_flags & FRT_DEVERR_UNFINISHED) return fail(FRT_EDEVICE, "a step left packets after its last pass");
    return FRT_OK;
}

int frt_read_fields(frt_solve s, double* x_HI, float* gamma, int kind)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    if (!s->have_grid) return fail(FRT_ESTATE, "no grid loaded");
    RCCHK(frt_sync(s));
    const size_t n = s->ncell;
    const hipMemcpyKind k = kind == FRT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (x_HI) RCCHK(scopy(s, x_HI, s->x, n * 8, k));
    if (gamma) {
        const void* g = s->gam[(s->step + 1u) & 1u];   // buffer of the last completed step
        if (s->step == 0) {
            if (kind == FRT_DEVICE) RCCHK(sset(s, gamma, 0, n * 4));
            else std::memset(gamma, 0, n * 4);
        } else if (!s->fp64) {
            RCCHK(scopy(s, gamma, g, n * 4, k));
        } else {
            std::vector<double> tmp(n);
            RCCHK(scopy(s, tmp.data(), g, n * 8, hipMemcpyDeviceToHost));
            std::vector<float> f(n);
            for (size_t i = 0; i < n; i++) f[i] = (float)tmp[i];
            if (kind == FRT_DEVICE) RCCHK(scopy(s, gamma, f.data(), n * 4, hipMemcpyHostToDevice));
            else std::memcpy(gamma, f.data(), n * 4);
        }
    }
    return FRT_OK;
}

int frt_read_ledger(frt_solve s, frt_ledger* out)
{
    if (!s || !out) return fail(FRT_EINVAL, "null argument");
    FrtLedgerDev L;
    RCCHK(read_device_ledger(s, &L));
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
    out->absorbed_front = L.absorbed_front;
    out->merge_residual = L.merge_residual;
    out->merges = L.merges;
    out->rays_merged = L.rays_merged;
    out->front_excess = L.front_excess;
    out->heat_in = L.heat_in * 1.602176634e-12;   // eV -> erg
    return FRT_OK;
}

int frt_read_temperature(frt_solve s, double* T, int kind)
{
    if (!s || !T) return fail(FRT_EINVAL, "null argument");
    if (kind != FRT_HOST && kind != FRT_DEVICE) return fail(FRT_EINVAL, "ptr_kind must be FRT_HOST or FRT_DEVICE");
    if (!s->T) return fail(FRT_ESTATE, "the solve holds no temperature (none loaded, temperature off)");
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    RCCHK(scopy(s, T, s->T, s->ncell * 8, kind == FRT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

// Checkpoint layout: 8 u64 header (magic, version, step, n_src, ncell, nb,
// fp64, n_carried), ledger (without stripes), x[ncell], quaternions of the
// steps so far, the carried packets as FrtRec structs, the count and
// entries of the virtual-origin table, then the count (ncell or 0) and
// values of the previous step's rate field (solves that start their opacity
// iteration from it).
int frt_save_state(frt_solve s, void* buf, size_t* bytes)
{
    RCCHK(ready(s));
    if (!bytes) return fail(FRT_EINVAL, "null size");
    HIPCHK(hipStreamSynchronize(s->stream));
    uint32_t fc[2];
    RCCHK(scopy(s, fc, s->fcount, 8, hipMemcpyDeviceToHost));
    const int cur = (int)(s->step & 1u);
    const uint32_t nc = std::min(fc[cur], s->F[cur].cap);
    const int nb = s->P.n_bins;
    const size_t rec = rec_bytes(s->rs);
    const size_t led = offsetof(FrtLedgerDev, sd);
    const size_t nq = (size_t)s->step * s->n_src * 4;
    uint32_t vc[2] = {0, 0};
    if (s->vcount) RCCHK(scopy(s, vc, s->vcount, 8, hipMemcpyDeviceToHost));
    const uint64_t nv = vc[cur];
    const uint64_t ng = warm_rate(s) ? s->ncell : 0;
    const uint64_t nt = s->h.temp ? s->ncell : 0;
    const size_t need =
        64 + led + s->ncell * 8 + nq * 8 + (size_t)nc * rec + 8 + nv * sizeof(FrtVSrc) + 8 + ng * s->rs + 8 + nt * 8;
    if (!buf) {
        *bytes = need;
        return FRT_OK;
    }
    if (*bytes < need) return fail(FRT_EINVAL, "checkpoint buffer too small (%zu < %zu)", *bytes, need);
    char* p = (char*)buf;
    uint64_t hdr[8] = {0x4652544350543034ull, 9, s->step, (uint64_t)s->n_src, s->ncell, (uint64_t)nb, (uint64_t)s->fp64, nc};
    std::memcpy(p, hdr, sizeof(hdr));
    p += sizeof(hdr);
    RCCHK(scopy(s, p, s->L, led, hipMemcpyDeviceToHost));
    p += led;
    RCCHK(scopy(s, p, s->x, s->ncell * 8, hipMemcpyDeviceToHost));
    p += s->ncell * 8;
    if (nq) RCCHK(scopy(s, p, s->quat, nq * 8, hipMemcpyDeviceToHost));
    p += nq * 8;
    if (nc) {
        FrtRecs hv{};
        hv.cap = nc;
        hv.rec = p;
        RCCHK(copy_recs(hv, s->F[cur], nc, nb, s->rs, s->stream, hipMemcpyDeviceToHost));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    p += (size_t)nc * rec;
    std::memcpy(p, &nv, 8);
    p += 8;
    if (nv) RCCHK(scopy(s, p, s->vt[cur], nv * sizeof(FrtVSrc), hipMemcpyDeviceToHost));
    p += nv * sizeof(FrtVSrc);
    std::memcpy(p, &ng, 8);
    p += 8;
    if (ng) RCCHK(scopy(s, p, s->gam[(s->step + 1u) & 1u], ng * s->rs, hipMemcpyDeviceToHost));
    p += ng * s->rs;
    std::memcpy(p, &nt, 8);
    p += 8;
    if (nt) RCCHK(scopy(s, p, s->T, nt * 8, hipMemcpyDeviceToHost));
    *bytes = need;
    return FRT_OK;
}

int frt_load_state(frt_solve s, const void* buf, size_t bytes)
{
    RCCHK(ready(s));
    const size_t led = offsetof(FrtLedgerDev, sd);
    if (!buf || bytes < 64 + led) return fail(FRT_EINVAL, "checkpoint too small");
    const char* p = (const char*)buf;
    uint64_t hdr[8];
    std::memcpy(hdr, p, sizeof(hdr));
    p += sizeof(hdr);
    if (hdr[0] != 0x4652544350543034ull || hdr[1] != 9) return fail(FRT_EINVAL, "not a checkpoint of this library");
    AllocScope scope(&s->ctx->al);
    if (hdr[3] != (uint64_t)s->n_src || hdr[4] != s->ncell || hdr[5] != (uint64_t)s->P.n_bins || hdr[6] != (uint64_t)s->fp64)
        return fail(FRT_EINVAL, "checkpoint does not match this solve (sources, grid, bins or precision)");
    const uint32_t step = (uint32_t)hdr[2], nc = (uint32_t)hdr[7];
    const int nb = s->P.n_bins;
    const size_t rec = rec_bytes(s->rs);
    const size_t nq = (size_t)step * s->n_src * 4;
    if (bytes < 64 + led + s->ncell * 8 + nq * 8 + (size_t)nc * rec + 8) return fail(FRT_EINVAL, "checkpoint truncated");
    uint64_t nv = 0;
    std::memcpy(&nv, p + led + s->ncell * 8 + nq * 8 + (size_t)nc * rec, 8);
    const size_t at_ng = led + s->ncell * 8 + nq * 8 + (size_t)nc * rec + 8 + nv * sizeof(FrtVSrc);
    if (bytes < 64 + at_ng + 8) return fail(FRT_EINVAL, "checkpoint truncated");
    uint64_t ng = 0;
    std::memcpy(&ng, p + at_ng, 8);
    if (ng != (warm_rate(s) ? s->ncell : 0))
        return fail(FRT_EINVAL, "checkpoint's previous rate field does not match this solve's opacity iteration");
    if (bytes < 64 + at_ng + 8 + ng * s->rs + 8) return fail(FRT_EINVAL, "checkpoint truncated");
    const size_t at_nt = at_ng + 8 + ng * s->rs;
    uint64_t nt = 0;
    std::memcpy(&nt, p + at_nt, 8);
    if (nt != (s->h.temp ? s->ncell : 0)) return fail(FRT_EINVAL, "checkpoint's temperature field does not match this solve");
    if (bytes < 64 + at_nt + 8 + nt * 8) return fail(FRT_EINVAL, "checkpoint truncated");
    if (nv && !s->P.merge) return fail(FRT_EINVAL, "checkpoint holds merged packets; this solve does not merge");
    HIPCHK(hipStreamSynchronize(s->stream));
    RCCHK(sset(s, s->L, 0, sizeof(FrtLedgerDev)));
    RCCHK(scopy(s, s->L, p, led, hipMemcpyHostToDevice));
    p += led;
    RCCHK(scopy(s, s->x, p, s->ncell * 8, hipMemcpyHostToDevice));
    p += s->ncell * 8;
    RCCHK(ensure_quat(s, step));
    if (nq) RCCHK(scopy(s, s->quat, p, nq * 8, hipMemcpyHostToDevice));
    p += nq * 8;
    const int cur = (int)(step & 1u);
    if (nc > s->F[cur].cap) {
        FrtRecs nf[2];
        RCCHK(alloc_recs(nf[0], nc + 1024, nb, s->rs));
        RCCHK(alloc_recs(nf[1], nc + 1024, nb, s->rs));
        free_recs(s->F[0]);
        free_recs(s->F[1]);
        s->F[0] = nf[0];
        s->F[1] = nf[1];
        s->h.F[0] = nf[0];
        s->h.F[1] = nf[1];
    }
    if (nc) {
        // the carried packets may come from steps with a longer dt
        for (uint32_t i = 0; i < nc; i++) {
            double w0;
            if (s->fp64) {
                double v;
                std::memcpy(&v, p + i * rec + offsetof(FrtRec<double>, w0), sizeof(v));
                w0 = v;
            } else {
                float v;
                std::memcpy(&v, p + i * rec + offsetof(FrtRec<float>, w0), sizeof(v));
                w0 = v;
            }
            if (std::isfinite(w0)) s->w0_max = std::max(s->w0_max, w0);
        }
        FrtRecs hv{};
        hv.cap = nc;
        hv.rec = (void*)p;
        RCCHK(copy_recs(s->F[cur], hv, nc, nb, s->rs, s->stream, hipMemcpyHostToDevice));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    p += (size_t)nc * rec + 8;
    if (s->P.merge) {
        RCCHK(ensure_vtable(s, cur, (uint32_t)nv));
        if (nv) RCCHK(scopy(s, s->vt[cur], p, nv * sizeof(FrtVSrc), hipMemcpyHostToDevice));
        uint32_t vc[2] = {0, 0};
        vc[cur] = (uint32_t)nv;
        RCCHK(scopy(s, s->vcount, vc, 8, hipMemcpyHostToDevice));
    }
    uint32_t fc[2] = {0, 0};
    fc[cur] = nc;
    RCCHK(scopy(s, s->fcount, fc, 8, hipMemcpyHostToDevice));
    s->step = step;
    s->h.step = step;
    RCCHK(sset(s, s->gam[0], 0, s->ncell * s->rs));
    RCCHK(sset(s, s->gam[1], 0, s->ncell * s->rs));
    if (ng) {
        const char* pg = (const char*)buf + 64 + at_ng + 8;
        RCCHK(scopy(s, s->gam[(step + 1u) & 1u], pg, ng * s->rs, hipMemcpyHostToDevice));
    }
    if (s->front) RCCHK(sset(s, s->front, 0, s->ncell * 8));
    if (nt) RCCHK(scopy(s, s->T, (const char*)buf + 64 + at_nt + 8, nt * 8, hipMemcpyHostToDevice));
    if (s->heat) RCCHK(sset(s, s->heat, 0, s->ncell * s->rs));
    RCCHK(upload_desc(s));
    hipError_t e = frt::launch_prep_opacity(s->d_desc, s->ncell, s->fp64, s->stream);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "prep launch: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s->stream));
    return FRT_OK;
}

int frt_mark(frt_solve s)
{
    RCCHK(ready(s));
    AllocScope scope(&s->ctx->al);
    HIPCHK(hipStreamSynchronize(s->stream));
    uint32_t fc[2];
    RCCHK(scopy(s, fc, s->fcount, 8, hipMemcpyDeviceToHost));
    const int cur = (int)(s->step & 1u);
    const uint32_t nc = std::min(fc[cur], s->F[cur].cap);
    dev_free(s->mark_x);
    dev_free(s->mark_fc);
    free_recs(s->mark_F);
    RCCHK(dev_alloc((void**)&s->mark_x, s->ncell * 8));
    RCCHK(dev_alloc((void**)&s->mark_fc, 8));
    uint32_t mfc[2] = {0, 0};
    mfc[cur] = nc;
    RCCHK(scopy(s, s->mark_fc, mfc, 8, hipMemcpyHostToDevice));
    RCCHK(alloc_recs(s->mark_F, std::max<uint32_t>(nc, 1), s->P.n_bins, s->rs));
    HIPCHK(hipMemcpyAsync(s->mark_x, s->x, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    RCCHK(copy_recs(s->mark_F, s->F[cur], nc, s->P.n_bins, s->rs, s->stream, hipMemcpyDeviceToDevice));
    HIPCHK(hipStreamSynchronize(s->stream));
    dev_free(s->mark_vt);
    s->mark_vn = 0;
    if (s->vcount) {
        uint32_t vc[2];
        RCCHK(scopy(s, vc, s->vcount, 8, hipMemcpyDeviceToHost));
        s->mark_vn = vc[cur];
        RCCHK(dev_alloc((void**)&s->mark_vt, std::max<size_t>(s->mark_vn, 1) * sizeof(FrtVSrc)));
        if (s->mark_vn) RCCHK(scopy(s, s->mark_vt, s->vt[cur], (size_t)s->mark_vn * sizeof(FrtVSrc), hipMemcpyDeviceToDevice));
    }
    dev_free(s->mark_g);
    if (warm_rate(s)) {
        RCCHK(dev_alloc(&s->mark_g, s->ncell * s->rs));
        HIPCHK(hipMemcpyAsync(s->mark_g, s->gam[(s->step + 1u) & 1u], s->ncell * s->rs, hipMemcpyDeviceToDevice,
                              s->stream));
    }
    dev_free(s->mark_T);
    if (s->h.temp) {
        RCCHK(dev_alloc((void**)&s->mark_T, s->ncell * 8));
        HIPCHK(hipMemcpyAsync(s->mark_T, s->T, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    s->mark_n = nc;
    s->mark_step = s->step;
    s->marked = true;
    return FRT_OK;
}

int frt_rewind(frt_solve s)
{
    RCCHK(ready(s));
    if (!s->marked) return fail(FRT_ESTATE, "frt_rewind without frt_mark");
    const int cur = (int)(s->mark_step & 1u);
    if (s->mark_n > s->F[cur].cap) return fail(FRT_ESTATE, "carried queue shrank below the bookmark");
    HIPCHK(hipMemcpyAsync(s->x, s->mark_x, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    RCCHK(copy_recs(s->F[cur], s->mark_F, s->mark_n, s->P.n_bins, s->rs, s->stream, hipMemcpyDeviceToDevice));
    HIPCHK(hipMemcpyAsync(s->fcount, s->mark_fc, 8, hipMemcpyDeviceToDevice, s->stream));
    if (s->vcount) {
        if (s->vt_cap[cur] < s->mark_vn) return fail(FRT_ESTATE, "virtual-origin table shrank below the bookmark");
        if (s->mark_vn)
            HIPCHK(hipMemcpyAsync(s->vt[cur], s->mark_vt, (size_t)s->mark_vn * sizeof(FrtVSrc), hipMemcpyDeviceToDevice,
                                  s->stream));
        HIPCHK(hipMemcpyAsync(s->vcount + cur, &s->mark_vn, 4, hipMemcpyHostToDevice, s->stream));
    }
    HIPCHK(hipMemsetAsync(s->gam[cur], 0, s->ncell * s->rs, s->stream));
    if (s->mark_g)
        HIPCHK(hipMemcpyAsync(s->gam[cur ^ 1], s->mark_g, s->ncell * s->rs, hipMemcpyDeviceToDevice, s->stream));
    if (s->front) HIPCHK(hipMemsetAsync(s->front, 0, s->ncell * 8, s->stream));
    if (s->mark_T) HIPCHK(hipMemcpyAsync(s->T, s->mark_T, s->ncell * 8, hipMemcpyDeviceToDevice, s->stream));
    if (s->heat) HIPCHK(hipMemsetAsync(s->heat, 0, s->ncell * s->rs, s->stream));
    s->step = s->mark_step;
    s->h.step = s->step;
    RCCHK(upload_desc(s));
    hipError_t e = frt::launch_prep_opacity(s->d_desc, s->ncell, s->fp64, s->stream);
    if (e != hipSuccess) return fail(FRT_EDEVICE, "prep launch: %s", hipGetErrorString(e));
    return FRT_OK;
}

int frt_set_timing(frt_solve s, int enable)
{
    if (!s) return fail(FRT_EINVAL, "null solve");
    HIPCHK(hipStreamSynchronize(s->stream));
    s->reset_timing();
    s->timing = enable != 0;
    return FRT_OK;
}

int frt_read_timing(frt_solve s, frt_timing* out)
{
    if (!s || !out) return fail(FRT_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(s->stream));
    s->drain_events();
    out->emit_ms = s->t_ms[0];
    out->march_ms = s->t_ms[1];
    out->chem_ms = s->t_ms[2];
    out->other_ms = s->t_ms[3];
    out->march_launches = s->n_march;
    out->chem_launches = s->n_chem;
    out->steps = s->n_steps_timed;
    out->merge_ms = s->t_ms[4];
    return FRT_OK;
}

int frt_debug_cast(frt_solve s, const double o_cm[3], const double d[3], const double* N_bins, double dt_s,
                   float* gamma_out, int ptr_kind, double* absorbed, double* escaped, uint64_t* crossings)
{
    if (!s || !o_cm || !d || !N_bins || !absorbed || !escaped || !crossings) return fail(FRT_EINVAL, "null argument");
    if (!s->have_grid) return fail(FRT_ESTATE, "load the grid before casting through it");
    if (!(dt_s > 0) || !std::isfinite(dt_s)) return fail(FRT_EINVAL, "dt must be finite and > 0");
    if (ptr_kind != FRT_HOST && ptr_kind != FRT_DEVICE) return fail(FRT_EINVAL, "ptr_kind must be FRT_HOST or FRT_DEVICE");
    const double ext[3] = {s->nx * s->dx, s->ny * s->dx, s->nz * s->dx};
    double nrm = 0;
    for (int a = 0; a < 3; a++) {
        if (!std::isfinite(o_cm[a]) || o_cm[a] < 0 || o_cm[a] > ext[a]) return fail(FRT_EINVAL, "origin outside the box");
        if (!std::isfinite(d[a])) return fail(FRT_EINVAL, "direction not finite");
        nrm += d[a] * d[a];
    }
    if (!(nrm > 0)) return fail(FRT_EINVAL, "zero direction");
    for (int b = 0; b < s->P.n_bins; b++)
        if (!std::isfinite(N_bins[b]) || N_bins[b] < 0) return fail(FRT_EINVAL, "N_bins[%d] is negative or not finite", b);
    HIPCHK(hipSetDevice(s->ctx->device));
    HIPCHK(hipStreamSynchronize(s->stream));
    AllocScope scope(&s->ctx->al);
    std::lock_guard<std::mutex> lock(s->ctx->mu);
    return debug_cast_locked(s, o_cm, d, N_bins, dt_s, gamma_out, ptr_kind, absorbed, escaped, crossings);
}

int frt_microbench(frt_ctx ctx, size_t copy_bytes, size_t atomic_slots, frt_microbench_result* out)
{
    if (!ctx || !out) return fail(FRT_EINVAL, "null argument");
    if (out->size != sizeof(frt_microbench_result)) return fail(FRT_EINVAL, "frt_microbench_result.size must be its sizeof");
    if (copy_bytes < (1u << 20) || copy_bytes % 16) return fail(FRT_EINVAL, "copy_bytes must be a multiple of 16, at least 1 MiB");
    if (atomic_slots < 1024 || atomic_slots > 0xffffffffull) return fail(FRT_EINVAL, "atomic_slots outside 1024..2^32-1");
    std::lock_guard<std::mutex> lock(ctx->mu);
    AllocScope scope(&ctx->al);
    HIPCHK(hipSetDevice(ctx->device));
    struct Bufs {
        void *a = nullptr, *b = nullptr, *c = nullptr;
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Bufs()
        {
            if (st) (void)hipStreamSynchronize(st);
            dev_free_ptr(a);
            dev_free_ptr(b);
            dev_free_ptr(c);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (st) (void)hipStreamDestroy(st);
        }
    } m;
    RCCHK(dev_alloc(&m.a, copy_bytes));
    RCCHK(dev_alloc(&m.b, copy_bytes));
    RCCHK(dev_alloc(&m.c, atomic_slots * 4));
    HIPCHK(hipStreamCreateWithFlags(&m.st, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&m.e0));
    HIPCHK(hipEventCreate(&m.e1));
    HIPCHK(hipMemsetAsync(m.a, 0, copy_bytes, m.st));
    HIPCHK(hipMemsetAsync(m.c, 0, atomic_slots * 4, m.st));
    // the best of five timed runs after one untimed one
    auto best_ms = [&](auto launch, double* best) -> int {
        *best = -1.0;
        for (int r = 0; r < 6; r++) {
            HIPCHK(hipEventRecord(m.e0, m.st));
            hipError_t e = launch();
            if (e != hipSuccess) return fail(FRT_EDEVICE, "microbench launch: %s", hipGetErrorString(e));
            HIPCHK(hipEventRecord(m.e1, m.st));
            HIPCHK(hipEventSynchronize(m.e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, m.e0, m.e1));
            if (r > 0 && (*best < 0.0 || ms < *best)) *best = ms;
        }
        return FRT_OK;
    };
    double copy_ms = 0.0, atomic_ms = 0.0;
    for (int v = 0; v < 2; v++) {
        double ms = 0.0;
        RCCHK(best_ms([&] { return frt::microbench_copy(m.a, m.b, copy_bytes, v, m.st); }, &ms));
        if (v == 0 || ms < copy_ms) copy_ms = ms;
    }
    const int grid = frt::device_cu_count() * 8, per_lane = 64;
    const double ops = (double)grid * 256.0 * per_lane;
    RCCHK(best_ms([&] { return frt::microbench_atomic((float*)m.c, (uint32_t)atomic_slots, per_lane, grid, 12345u, m.st); },
                  &atomic_ms));
    out->copy_bytes = (double)copy_bytes;
    out->copy_GBps = 2.0 * (double)copy_bytes / (copy_ms * 1e-3) / 1e9;
    out->atomic_ops = ops;
    out->atomic_per_s = ops / (atomic_ms * 1e-3);
    out->atomic_slots = (double)atomic_slots;
    return FRT_OK;
}

int frt_merge_uniforms(uint64_t seed, uint32_t step, uint32_t cell, double out[3])
{
    if (!out) return fail(FRT_EINVAL, "null output");
    const uint64_t key = mix64_host(mix64_host(seed) ^ 0x6D65726765ull);
    for (uint32_t k = 0; k < 3; k++) {
        const uint64_t ctr = ((uint64_t)step << 34) | ((uint64_t)cell << 2) | (uint64_t)k;
        out[k] = (double)(mix64_host(ctr ^ key) >> 11) * 0x1.0p-53;
    }
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
