// HIP kernels for gfx950: casting, the brick-synchronous ray march, the
// hydrogen update (backward Euler, or the time-averaged update) and step
// bookkeeping of adaptive ray tracing of ionizing photon packets (Cain &
// D'Aloisio, FlexRT I, §3 and §4.1).
//
// A step runs as a sequence of passes.  The grid is cut into bricks
// (32 x 16 x 16 cells for the FP32 march without sub-grid opacity, 16^3 with
// it, 8^3 for FP64).  In each pass every brick that holds packets is given
// to workgroups: a workgroup stages the brick's opacity in LDS, walks each
// of its packets cell by cell until the packet leaves the brick, splits,
// ends or spends its travel budget, deposits the absorbed photons with LDS
// atomics, and adds the brick's deposits to the global rate field once.
// Packets that leave or split are appended to the pass's output buffer with
// the key of the brick they are in next; a counting pass and a scatter put
// their indices in brick order, and the next pass reads the records through
// them (the two output buffers alternate).  Item counts live on the device,
// so the host launches a fixed number of passes without reading anything
// back.
#include "frt_internal.h"
#include "frt_device.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>
#include <limits>
#include <mutex>
#include <unordered_map>
#include <utility>

namespace {

using namespace frt_dev;

constexpr int WAVE = 64;
constexpr int BLOCK = 256;

// ------------------------------------------------------------- wave helpers
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Add a per-lane value into a per-solve FP64 counter.  When every lane of
// the wave targets the same solve the wave reduces first and one lane adds.

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Exclusive prefix sum of v over the wave; *total gets the wave's sum.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total)
{
    const int lane = threadIdx.x & (WAVE - 1);
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, WAVE - 1, WAVE);
    return x - v;
}

// Reserve n_lane slots per lane in an array whose fill counter is *ctr, with
// one atomic per wave.  Every lane of the wave must call it.  Returns the
// lane's first slot.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* ctr, uint32_t n_lane)
{
    uint32_t total;
    const uint32_t off = wave_excl_scan(n_lane, &total);
    uint32_t base = 0;
    if ((threadIdx.x & (WAVE - 1)) == 0 && total) base = atomicAdd(ctr, total);
    base = __shfl(base, 0, WAVE);
    return base + off;
}

// Fill counters and sizes of the output segments (see FRT_QSEG).
__device__ __forceinline__ uint32_t* o_ctr(const FrtWS& ws, int k) { return ws.segc + k * FRT_QSEG_STRIDE; }
// A replayed step after one that failed: every kernel of the step returns
// at once (the same value for the whole grid, read before any barrier).
__device__ __forceinline__ bool halted(const FrtWS& ws) { return ws.ctr[C_HALT] != 0u; }
__device__ __forceinline__ uint32_t seg_cap(uint32_t cap) { return cap / FRT_QSEG; }
__device__ __forceinline__ int my_seg() { return (int)(blockIdx.x % FRT_QSEG); }

template <typename Real> __device__ __forceinline__ Real rinf();
template <> __device__ __forceinline__ float rinf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double rinf<double>() { return __builtin_huge_val(); }

// A wave-uniform value moved into a scalar register, so that it is read once
// per work item instead of from memory inside divergent loops.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double uni(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = uni((uint32_t)b), hi = uni((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Device memory through pointers the compiler cannot prove global (they
// come from the descriptor or a struct passed by value): their accesses
// are made global ones here rather than flat ones, which also count
// against the LDS wait counter, so that a later wait for an LDS result
// would wait for them as well.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ T ld_global(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}
// atomicAdd's relaxed, device-scope add on global memory
__device__ __forceinline__ uint32_t g_atomic_add(uint32_t* p, uint32_t v)
{
    return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_atomic_add(float* p, float v)
{
    (void)__hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_atomic_add(double* p, double v)
{
    (void)__hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename Real> struct Vec2;
template <> struct Vec2<float> { using T = float2; };
template <> struct Vec2<double> { using T = double2; };

// exp(-t): the hardware exponential in FP32.
__device__ __forceinline__ float exp_neg(float t) { return __expf(-t); }
__device__ __forceinline__ double exp_neg(double t) { return exp(-t); }

// --------------------------------------------------------------- the ledger
// Per-lane accumulation, block reduction, one atomic per field per flush
// into one of FRT_STRIPES stripes.  All threads of the block must call
// ledger_flush at the same point.
struct LaneLedger {
    double f[LF_NF];
    unsigned long long c[LC_NC];
    __device__ void clear()
    {
#pragma unroll
        for (int i = 0; i < LF_NF; i++) f[i] = 0.0;
#pragma unroll
        for (int i = 0; i < LC_NC; i++) c[i] = 0;
    }
};

// Direct add for the rare lane whose solve differs from its block's.
__device__ __forceinline__ void ledger_direct(FrtLedgerDev* L, int f, double v)
{
    if (v != 0.0) atomicAdd(&L->sd[blockIdx.x % FRT_STRIPES][f], v);
}

__device__ __forceinline__ void ledger_direct_c(FrtLedgerDev* L, int c, unsigned long long v)
{
    if (v) atomicAdd(&L->sc[blockIdx.x % FRT_STRIPES][c], v);
}

__device__ void ledger_flush(LaneLedger& a, FrtLedgerDev* L)
{
    __shared__ double s_f[BLOCK / WAVE][LF_NF];
    __shared__ unsigned long long s_c[BLOCK / WAVE][LC_NC];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int i = 0; i < LF_NF; i++) {
        double v = wave_sum(a.f[i]);
        if (lane == 0) s_f[w][i] = v;
    }
#pragma unroll
    for (int i = 0; i < LC_NC; i++) {
        unsigned long long v = wave_sum_u64(a.c[i]);
        if (lane == 0) s_c[w][i] = v;
    }
    __syncthreads();
    const int stripe = blockIdx.x % FRT_STRIPES;
    if (threadIdx.x < LF_NF) {
        double v = 0;
        for (int k = 0; k < BLOCK / WAVE; k++) v += s_f[k][threadIdx.x];
        if (v != 0.0) atomicAdd(&L->sd[stripe][threadIdx.x], v);
    } else if (threadIdx.x >= 32 && threadIdx.x < 32 + LC_NC) {
        const int i = threadIdx.x - 32;
        unsigned long long v = 0;
        for (int k = 0; k < BLOCK / WAVE; k++) v += s_c[k][i];
        if (v) atomicAdd(&L->sc[stripe][i], v);
    }
    __syncthreads();
    a.clear();
}

// ------------------------------------------------------------------ records
template <typename Real>
struct Pkt {
    uint32_t src, estep, lp, cell;
    Real r, rstop, w0;
    Real d[3];
};

// T[0] = A (HI optical depth at sigma_0), T[1] = K (sub-grid optical depth),
// T[2], T[3] their Kahan compensations.
template <typename Real>
__device__ __forceinline__ FrtRec<Real>* recs(const FrtRecs& q) { return (FrtRec<Real>*)q.rec; }

// The pass buffer a launch appends to and the one holding its input (both
// have the same capacity), and their key arrays.
__device__ __forceinline__ FrtRecs out_recs(const FrtWS& ws) { return FrtRecs{ws.out ? ws.buf[1].rec : ws.buf[0].rec, ws.buf[0].cap}; }
__device__ __forceinline__ FrtRecs in_recs(const FrtWS& ws) { return FrtRecs{ws.out ? ws.buf[0].rec : ws.buf[1].rec, ws.buf[0].cap}; }
__device__ __forceinline__ const uint32_t* in_keys(const FrtWS& ws) { return ws.out ? ws.bkey[0] : ws.bkey[1]; }

template <typename Real>
__device__ __forceinline__ void load_pkt(const FrtRecs& q, uint32_t i, Pkt<Real>& h, Real* T)
{
    const FrtRec<Real> x = recs<Real>(q)[i];
    h.src = x.src;
    h.estep = x.estep;
    h.lp = x.lp;
    h.cell = x.cell;
    h.r = x.r;
    h.rstop = x.rstop;
    h.w0 = x.w0;
#pragma unroll
    for (int a = 0; a < 3; a++) h.d[a] = x.dir[a];
#pragma unroll
    for (int b = 0; b < 4; b++) T[b] = x.tau[b];
}

template <typename Real>
__device__ __forceinline__ void store_pkt(const FrtRecs& q, uint32_t i, const Pkt<Real>& h, uint32_t key, const Real* T)
{
    FrtRec<Real> x;
    x.src = h.src;
    x.estep = h.estep;
    x.lp = h.lp;
    x.cell = h.cell;
    x.key = key;
    x.r = h.r;
    x.rstop = h.rstop;
    x.w0 = h.w0;
#pragma unroll
    for (int a = 0; a < 3; a++) x.dir[a] = h.d[a];
#pragma unroll
    for (int b = 0; b < 4; b++) x.tau[b] = T[b];
    // written as whole 16-byte words, global stores
    static_assert(sizeof(FrtRec<Real>) % 16 == 0, "records are whole 16-byte words");
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 wd[sizeof(FrtRec<Real>) / 16];
    __builtin_memcpy(wd, &x, sizeof(x));
    __attribute__((address_space(1))) u32x4* dst = (__attribute__((address_space(1))) u32x4*)(recs<Real>(q) + i);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(FrtRec<Real>) / 16); k++) dst[k] = wd[k];
}

// Append slot i of the launch's output buffer: the record and its key.
template <typename Real>
__device__ __forceinline__ void store_out(const FrtWS& ws, uint32_t i, const Pkt<Real>& h, uint32_t key, const Real* T)
{
    store_pkt<Real>(out_recs(ws), i, h, key, T);
    *gmem((ws.out ? ws.bkey[1] : ws.bkey[0]) + i) = key;
}

template <typename Real>
__device__ __forceinline__ void packet_dir(const FrtSolveDesc& D, uint32_t lp, uint32_t estep, uint32_t src, Real d[3])
{
    // the rotation's loads first, the pixel centre's arithmetic while they fly
    const double* qp = rot_of(D, estep, src);
    double q[4];
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = ld_global(qp + k);
    nest_pixel_centre<Real>((int)(lp >> 28), lp & 0x0fffffffu, d);
    quat_rotate<Real>(q, d);
}

// Cell of the point s + r d for a packet moving along d: floor per axis,
// a point exactly on a face belongs to the cell being entered.  Returns
// false when the point is outside the grid.
template <typename Real>
__device__ __forceinline__ bool locate(const FrtSolveDesc& D, const Real s[3], Real r, const Real d[3], int c[3])
{
    const int dims[3] = {D.nx, D.ny, D.nz};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        Real p = s[a] + r * d[a];
        Real f = floor(p);
        if (p == f && d[a] < Real(0)) f -= Real(1);
        in &= (f >= Real(0)) && (f < Real(dims[a]));
        c[a] = in ? (int)f : 0;
    }
    return in;
}

__device__ __forceinline__ uint32_t brick_key(const FrtSolveDesc& D, const int c[3])
{
    return D.key_base + (uint32_t)(c[0] >> D.bsh[0]) +
           (uint32_t)D.bpx * ((uint32_t)(c[1] >> D.bsh[1]) + (uint32_t)D.bpy * (uint32_t)(c[2] >> D.bsh[2]));
}

__device__ __forceinline__ int find_in_prefix(const uint32_t* prefix, int n, uint32_t g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void raise_error(FrtWS& ws, FrtLedgerDev* L, uint32_t bit)
{
    atomicOr(&ws.ctr[C_ERR], bit);
    atomicOr(&L->err_flags, bit);
}

template <typename Real>
__device__ __forceinline__ Real srel_of(const FrtSolveDesc& D, int b)
{
    if constexpr (sizeof(Real) == 8) return D.sig_reld[b];
    else return D.sig_rel[b];
}

template <typename Real>
__device__ __forceinline__ Real K_of(const FrtSolveDesc& D, int b)
{
    if constexpr (sizeof(Real) == 4) return D.K[b];
    else return (Real)D.Kd[b];
}

// 1/x: the hardware reciprocal in FP32 (about 1 ulp), a division in FP64.
template <typename Real>
__device__ __forceinline__ Real fast_rcp(Real x)
{
    if constexpr (sizeof(Real) == 4) return __builtin_amdgcn_rcpf(x);
    else return Real(1) / x;
}

// Crossings a packet at s + r d in cell c is expected to make in the brick
// holding c on its next visit: the distance to the first of brick exit,
// split radius, distance cap and the end of its travel budget (rstop),
// times |d|_1.  Only used to order the packets of a work item so that the
// lanes of a wave march similar lengths; stored in the key's top bits.
template <typename Real>
__device__ __forceinline__ Real split_radius(const FrtSolveDesc& D, int level)
{
    // r_split0 2^level (a power-of-two scaling, exact in either precision)
    return (level < D.max_level) ? (Real)ldexp((Real)D.r_split0, level) : rinf<Real>();
}

// Expected crossings of a packet in the brick of cell c before it leaves
// the brick or reaches its split radius, distance cap or budget end: the
// distance to the nearest of those times |dx| + |dy| + |dz|, in the bins of
// an output key.  inv[a] is 1 / d[a] (0 where d[a] is 0).
template <typename Real>
__device__ __forceinline__ uint32_t crossing_bin_inv(const FrtSolveDesc& D, const int c[3], const Real s[3], const Real d[3],
                                                     const Real inv[3], Real r, Real rstop, int level)
{
    const int dims[3] = {D.nx, D.ny, D.nz};
    Real lim = fmin(fmin(split_radius<Real>(D, level), (Real)D.r_cap), rstop);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int lo = (c[a] >> D.bsh[a]) << D.bsh[a], hi = min(lo + (1 << D.bsh[a]), dims[a]);
        if (d[a] > Real(0)) lim = fmin(lim, ((Real)hi - s[a]) * inv[a]);
        else if (d[a] < Real(0)) lim = fmin(lim, ((Real)lo - s[a]) * inv[a]);
    }
    const Real len = fmax(lim - r, Real(0)) * (fabs(d[0]) + fabs(d[1]) + fabs(d[2]));
    return (uint32_t)fmin(len, Real(FRT_KEY_BINS - 3)) + 1u;
}

template <typename Real>
__device__ __forceinline__ uint32_t crossing_bin(const FrtSolveDesc& D, const int c[3], const Real s[3], const Real d[3],
                                                 Real r, Real rstop, int level)
{
    Real inv[3];
#pragma unroll
    for (int a = 0; a < 3; a++) inv[a] = d[a] != Real(0) ? fast_rcp(d[a]) : Real(0);
    return crossing_bin_inv<Real>(D, c, s, d, inv, r, rstop, level);
}

__device__ __forceinline__ uint32_t key_with_bin(uint32_t key, uint32_t bin) { return key | (bin << FRT_KEY_BITS); }

// Output-key counts: an LDS table of KEY_SLOTS keys per workgroup, added to
// the histogram once per key.
constexpr int KEY_SLOTS = 128;

__device__ __forceinline__ void count_key(uint32_t* s_key, uint32_t* s_cnt, uint32_t* hist, uint32_t key, uint32_t n)
{
    uint32_t slot = (key * 2654435761u) & (KEY_SLOTS - 1);
    for (int probe = 0; probe < 16; probe++) {
        const uint32_t prev = atomicCAS(&s_key[slot], 0xffffffffu, key);
        if (prev == 0xffffffffu || prev == key) {
            atomicAdd(&s_cnt[slot], n);
            return;
        }
        slot = (slot + 1) & (KEY_SLOTS - 1);
    }
    atomicAdd(&hist[key], n);   // table crowded: count directly
}

// count_key for the lanes of a wave with `valid` set: one table update per
// distinct key of the wave.  Every lane of the wave must call it.
__device__ __forceinline__ void count_keys_wave(uint32_t* s_key, uint32_t* s_cnt, uint32_t* hist, uint32_t key, bool valid)
{
    const int lane = threadIdx.x & (WAVE - 1);
    unsigned long long todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll(todo) - 1;
        const uint32_t k = __shfl(key, leader, WAVE);
        const unsigned long long same = __ballot(valid && key == k);
        if (lane == leader) count_key(s_key, s_cnt, hist, k, (uint32_t)__popcll(same));
        todo &= ~same;
    }
}

// ================================================================= seeding
// Per solve: casting items (12 4^L0 per source) then the packets carried
// from the previous step.
__global__ void k_seed_plan(FrtSolveDesc* descs, FrtWS ws)
{
    // one wave: a solve per lane, the prefix by wave scans, 64 solves a round
    if (blockIdx.x != 0 || threadIdx.x >= WAVE || halted(ws)) return;
    uint32_t acc = 0;
    for (int s0 = 0; s0 < ws.n_solves; s0 += WAVE) {
        const int s = s0 + (int)threadIdx.x;
        uint32_t n = 0;
        if (s < ws.n_solves) {
            FrtSolveDesc& D = descs[s];
            uint32_t carried = D.fcount[D.cur];
            if (carried > D.F[D.cur].cap) carried = D.F[D.cur].cap;
            n = (uint32_t)D.n_src * D.ncast + carried;
            D.fcount[1 - D.cur] = 0;
            D.L->step_crossings = 0;
            // merged packets can hold more photons than any cast one: the
            // fixed-point deposit scale follows the brightest packet held
            if (D.merge) D.dep_scale = (float)(D.dep_base / fmax(D.w0_hi, (double)*D.w0_merged));
        }
        uint32_t tot;
        const uint32_t ex = wave_excl_scan(n, &tot);
        if (s < ws.n_solves) ws.seed_prefix[s] = acc + ex;
        acc += tot;
    }
    if (threadIdx.x == 0) ws.seed_prefix[ws.n_solves] = acc;
    for (int k = (int)threadIdx.x; k < FRT_QSEG; k += WAVE) ws.segc[k * FRT_QSEG_STRIDE] = 0;
}

// One lane per item: a cast packet gets r = 0 and Ndot_nu dt / (12 4^L0)
// photons per bin on its pixel of the source's sphere rotated for this step
// (§3.1, Eq. Nray); a carried packet is copied as it is.  Either goes to the
// pass output with the key of its brick.
template <typename Real, int NB>
__global__ void __launch_bounds__(BLOCK) k_seed(FrtSolveDesc* descs, FrtWS ws)
{
    __shared__ uint32_t spre[FRT_MAX_SOLVES_PER_LAUNCH + 1];
    __shared__ uint32_t s_key[KEY_SLOTS], s_cnt[KEY_SLOTS];   // output keys counted per round
    if (halted(ws)) return;
    for (int i = threadIdx.x; i <= ws.n_solves; i += blockDim.x) spre[i] = ws.seed_prefix[i];
    if (threadIdx.x < KEY_SLOTS) { s_key[threadIdx.x] = 0xffffffffu; s_cnt[threadIdx.x] = 0; }
    __syncthreads();
    const uint32_t total = spre[ws.n_solves];
    LaneLedger led;
    led.clear();
    int cs = -1;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < total; base += stride) {
        const uint32_t g = base + threadIdx.x;
        const bool active = g < total;
        const int si = find_in_prefix(spre, ws.n_solves, active ? g : base);
        // flush when the block moves to another solve (the solve of the
        // round's first item: block-uniform)
        const int bsolve = find_in_prefix(spre, ws.n_solves, base);
        if (bsolve != cs) {
            if (cs >= 0) ledger_flush(led, descs[cs].L);
            cs = bsolve;
        }
        FrtSolveDesc& D = descs[si];
        Pkt<Real> h;
        Real T[4] = {Real(0), Real(0), Real(0), Real(0)};
        uint32_t key = 0, want = 0, bin = 0;
        if (active) {
            const uint32_t local = g - spre[si];
            const uint32_t n_emit = (uint32_t)D.n_src * D.ncast;
            if (local < n_emit) {
                const uint32_t src = local / D.ncast, pix = local % D.ncast;
                double u[3];
                for (int k = 0; k < 3; k++)
                    u[k] = (D.step < D.user_steps) ? D.user_u[((size_t)D.step * D.n_src + src) * 3 + k]
                                                   : counter_uniform(D.seed, D.step, src, k);
                double q[4];
                shoemake_quat(u, q);
                if (pix == 0) {
                    double* dst = D.quat + ((size_t)D.step * D.n_src + src) * 4;
                    for (int k = 0; k < 4; k++) dst[k] = q[k];
                }
                Real d[3];
                nest_pixel_centre<Real>(D.base_level, pix, d);
                quat_rotate<Real>(q, d);
                h.src = src;
                h.estep = D.step;
                h.lp = ((uint32_t)D.base_level << 28) | pix;
                h.r = Real(0);
                h.rstop = Real(0);
                h.w0 = (Real)D.w0_cast;
                h.d[0] = d[0];
                h.d[1] = d[1];
                h.d[2] = d[2];
                double photons = 0.0;
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    if constexpr (sizeof(Real) == 8) photons += h.w0 * D.specd[(size_t)src * NB + b];
                    else photons += (double)(h.w0 * D.spec[(size_t)src * NB + b]);
                }
                photons *= D.R_ref;
                const bool own = (si == bsolve);
                if (own) {
                    led.f[LF_EMITTED] += photons;
                    led.c[LC_EMITTED] += 1;
                } else {
                    ledger_direct(D.L, LF_EMITTED, photons);
                    ledger_direct_c(D.L, LC_EMITTED, 1);
                }
                const double* sp = D.src_pos + (size_t)src * 3;
                const Real s3[3] = {(Real)sp[0], (Real)sp[1], (Real)sp[2]};
                int c[3];
                if (locate<Real>(D, s3, Real(0), d, c)) {
                    h.cell = pack_cell(c);
                    key = brick_key(D, c);
                    bin = crossing_bin<Real>(D, c, s3, h.d, Real(0), (Real)D.budget, D.base_level);
                    want = 1;
                } else if (own) {                  // points out of the box from a boundary source
                    led.f[LF_ESC] += photons;
                    led.c[LC_NESC] += 1;
                } else {
                    ledger_direct(D.L, LF_ESC, photons);
                    ledger_direct_c(D.L, LC_NESC, 1);
                }
            } else {
                const uint32_t i = local - n_emit;
                load_pkt<Real>(D.F[D.cur], i, h, T);
                key = D.key_base + recs<Real>(D.F[D.cur])[i].key;   // carried keys are solve-local
                const double* sp = src_pos_of(D, h.src);
                const Real s3[3] = {(Real)sp[0], (Real)sp[1], (Real)sp[2]};
                int c[3];
                unpack_cell(h.cell, c);
                const Real rs = h.rstop <= h.r ? h.r + (Real)D.budget : h.rstop;   // fresh budget this step
                bin = crossing_bin<Real>(D, c, s3, h.d, h.r, rs, (int)(h.lp >> 28));
                want = 1;
            }
        }
        const uint32_t at = wave_reserve(o_ctr(ws, my_seg()), want);
        bool stored = false;
        if (want) {
            if (at < seg_cap(ws.buf[0].cap)) {
                store_out<Real>(ws, (uint32_t)my_seg() * seg_cap(ws.buf[0].cap) + at, h, key_with_bin(key, bin), T);
                stored = true;
            } else {
                raise_error(ws, D.L, FRT_DEVERR_QUEUE_OVERFLOW);
            }
        }
        // the round's brick counts go to the histogram once per distinct key
        count_keys_wave(s_key, s_cnt, ws.hist, key, stored);
        __syncthreads();
        if (threadIdx.x < KEY_SLOTS) {
            const uint32_t k = s_key[threadIdx.x];
            if (k != 0xffffffffu) {
                atomicAdd(&ws.hist[k], s_cnt[threadIdx.x]);
                s_key[threadIdx.x] = 0xffffffffu;
                s_cnt[threadIdx.x] = 0;
            }
        }
        __syncthreads();
    }
    if (cs >= 0) ledger_flush(led, descs[cs].L);
}

// ============================================================ counting scan
// One block: offsets of each brick's packets in the sorted buffer, the work
// list (items of at most item_rays packets of one brick), scatter
// cursors; clears the histogram, the output counters and the counter the
// march workgroups take items from.
__global__ void __launch_bounds__(1024) k_scan(FrtWS ws)
{
    __shared__ uint32_t s_a[2 * WAVE + 1], s_b[2 * WAVE + 1];   // wave totals, their prefix, the total
    if (halted(ws)) return;
    const uint32_t nk = ws.nkeys;
    const uint32_t per = (nk + blockDim.x - 1) / blockDim.x;
    const uint32_t k0 = threadIdx.x * per, k1 = min(nk, k0 + per);
    uint32_t sum = 0, items = 0;
    for (uint32_t k = k0; k < k1; k++) {
        uint32_t h = ws.hist[k];
        sum += h;
        items += (h + ws.item_rays - 1) / ws.item_rays;
    }
    // exclusive scans of both counts: within each wave, then over the waves
    uint32_t wsum, witems;
    const uint32_t exs = wave_excl_scan(sum, &wsum);
    const uint32_t exi = wave_excl_scan(items, &witems);
    const int wid = (int)threadIdx.x / WAVE, nw = (int)blockDim.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        s_a[wid] = wsum;
        s_b[wid] = witems;
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
        const uint32_t a = (int)threadIdx.x < nw ? s_a[threadIdx.x] : 0u;
        const uint32_t b = (int)threadIdx.x < nw ? s_b[threadIdx.x] : 0u;
        uint32_t ta, tb;
        const uint32_t ea = wave_excl_scan(a, &ta), eb = wave_excl_scan(b, &tb);
        if ((int)threadIdx.x < nw) {
            s_a[WAVE + threadIdx.x] = ea;
            s_b[WAVE + threadIdx.x] = eb;
        }
        if (threadIdx.x == 0) {
            s_a[2 * WAVE] = ta;
            s_b[2 * WAVE] = tb;
        }
    }
    __syncthreads();
    uint32_t off = s_a[WAVE + wid] + exs;
    uint32_t it = s_b[WAVE + wid] + exi;
    const uint32_t total = s_a[2 * WAVE];
    const uint32_t total_items = s_b[2 * WAVE];
    // the previous pass's outputs in segment order; clear the fill counters
    if (threadIdx.x < WAVE) {
        const uint32_t cap = seg_cap(ws.buf[0].cap);
        const uint32_t c = *o_ctr(ws, threadIdx.x);
        if (c > cap) atomicOr(&ws.ctr[C_ERR], (uint32_t)FRT_DEVERR_QUEUE_OVERFLOW);
        uint32_t tot;
        const uint32_t ex = wave_excl_scan(c < cap ? c : cap, &tot);
        ws.segp[threadIdx.x] = ex;
        if (threadIdx.x == 0) {
            ws.segp[FRT_QSEG] = tot;
            ws.ctr[C_NOS] = tot;
        }
        *o_ctr(ws, threadIdx.x) = 0;
    }
    for (uint32_t k = k0; k < k1; k++) {
        uint32_t h = ws.hist[k];
        ws.cursor[k] = off;
        if (h) {
            const int solve = find_in_prefix(ws.key_prefix, ws.n_solves, k);
            for (uint32_t m = 0; m * ws.item_rays < h; m++) {
                if (it < ws.cap_work) {
                    FrtWork w;
                    w.key = k;
                    w.start = off + m * ws.item_rays;
                    w.count = min(ws.item_rays, h - m * ws.item_rays);
                    w.solve = (uint32_t)solve;
                    ws.work[it] = w;
                }
                it++;
            }
        }
        off += h;
        ws.hist[k] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ws.ctr[C_NP] = total;
        ws.ctr[C_NWORK] = total_items < ws.cap_work ? total_items : ws.cap_work;
        ws.ctr[C_NEXT] = 0;
        if (total > ws.ctr[C_MAXP]) ws.ctr[C_MAXP] = total;
        if (total > ws.pcap || total_items > ws.cap_work) ws.ctr[C_ERR] |= FRT_DEVERR_QUEUE_OVERFLOW;
    }
}

// ================================================================= scatter
// Put the previous pass's outputs in brick order without moving them: a
// block takes SLOTS consecutive outputs (written by few waves, so few
// distinct bricks), counts them per brick in an LDS hash table, reserves
// each brick's range with one atomic, and writes (record index, crossing
// bin) there.  Only the keys are read.
__global__ void __launch_bounds__(BLOCK) k_scatter(FrtWS ws)
{
    // PER outputs per thread and round; the table has a slot for every
    // output of the round, so an insertion always finds one
    constexpr int PER = 8;
    constexpr int SLOTS = PER * BLOCK;
    constexpr uint32_t EMPTY = 0xffffffffu;
    __shared__ uint32_t s_key[SLOTS], s_cnt[SLOTS], s_base[SLOTS];
    __shared__ uint32_t s_sp[FRT_QSEG + 1];
    if (halted(ws)) return;
    for (int i = threadIdx.x; i <= FRT_QSEG; i += blockDim.x) s_sp[i] = ws.segp[i];
    const uint32_t n = ws.ctr[C_NOS];
    const uint32_t scap = seg_cap(ws.buf[0].cap);
    const uint32_t* __restrict__ keys = in_keys(ws);
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned long long upto = (lane == WAVE - 1) ? ~0ull : ((2ull << lane) - 1ull);
    __syncthreads();
    for (uint32_t base = blockIdx.x * SLOTS; base < n; base += gridDim.x * SLOTS) {
        for (int i = threadIdx.x; i < SLOTS; i += blockDim.x) {
            s_key[i] = EMPTY;
            s_cnt[i] = 0;
        }
        // the round's keys, all loads issued together; a round inside one
        // output segment (the common case) needs no search for it
        const int sg0 = find_in_prefix(s_sp, FRT_QSEG, base);
        const bool one_seg = base + SLOTS <= s_sp[sg0 + 1];
        uint32_t idx[PER], kw[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const uint32_t v = base + (uint32_t)q * BLOCK + threadIdx.x;
            idx[q] = EMPTY;
            kw[q] = EMPTY;
            if (v < n) {
                const int sg = one_seg ? sg0 : find_in_prefix(s_sp, FRT_QSEG, v);
                idx[q] = (uint32_t)sg * scap + (v - s_sp[sg]);
                kw[q] = keys[idx[q]];
            }
        }
        __syncthreads();
        uint32_t slot[PER], rank[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            // empty slots (escaped split children) are skipped
            uint32_t key = (idx[q] == EMPTY || kw[q] == FRT_KEY_NONE) ? EMPTY : (kw[q] & FRT_KEY_MASK);
            if (key != EMPTY && key >= ws.nkeys) {      // never expected: flag and skip
                atomicOr(&ws.ctr[C_ERR], (uint32_t)FRT_DEVERR_QUEUE_OVERFLOW);
                key = EMPTY;
            }
            if (key == EMPTY) idx[q] = EMPTY;
            // lanes with equal keys next to each other (outputs of one wave of
            // the march mostly are) count as one run: its first lane inserts
            // the key once and reserves the run's ranks with one LDS atomic
            const uint32_t prev = __shfl_up(key, 1, WAVE);
            const bool head = lane == 0 || prev != key;
            const unsigned long long heads = __ballot(head);
            const int start = 63 - __clzll(heads & upto);
            uint32_t sl = 0, r0 = 0;
            if (head && key != EMPTY) {
                const unsigned long long after = heads & ~upto;
                const uint32_t len = (after ? (uint32_t)__ffsll(after) - 1u : (uint32_t)WAVE) - (uint32_t)lane;
                sl = (key * 2654435761u) & (SLOTS - 1);
                for (;;) {
                    const uint32_t prv = atomicCAS(&s_key[sl], EMPTY, key);
                    if (prv == EMPTY || prv == key) break;
                    sl = (sl + 1) & (SLOTS - 1);
                }
                r0 = atomicAdd(&s_cnt[sl], len);
            }
            slot[q] = __shfl(sl, start, WAVE);
            rank[q] = __shfl(r0, start, WAVE) + (uint32_t)(lane - start);
        }
        __syncthreads();
        for (int j = threadIdx.x; j < SLOTS; j += blockDim.x)
            if (s_key[j] != EMPTY) s_base[j] = atomicAdd(&ws.cursor[s_key[j]], s_cnt[j]);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; q++) {
            if (idx[q] == EMPTY) continue;
            const uint32_t pos = s_base[slot[q]] + rank[q];
            if (pos < ws.pcap) ws.sorted[pos] = make_uint2(idx[q], kw[q] >> FRT_KEY_BITS);
        }
        __syncthreads();
    }
}

// =============================================================== brick march
// Absorbed fraction 1 - e^-t of a segment given eb = e^-t: the series
// t (1 - t/2 + t^2/6 - t^3/24) below t = 0.03 (truncation < 7e-9
// relative), 1 - eb above.  Both forms are evaluated and one selected,
// which costs less than a branch per bin.
template <typename Real>
__device__ __forceinline__ Real absorbed(Real t, Real eb)
{
    if constexpr (sizeof(Real) == 4) {
        const Real ser = t * (Real(1) - t * (Real(0.5) - t * (Real(1.0 / 6.0) - t * Real(1.0 / 24.0))));
        const Real dif = Real(1) - eb;
        return t < Real(0.03) ? ser : dif;
    } else {
        return -expm1(-t);
    }
}

// The same in terms of u = -log2(e) t (so that e^-t = 2^u): 1 - 2^u for
// -0.0721 < u <= 0 (optical depths below 0.05) from its Taylor series, with
// w = -u ln 2, w - w^2/2 + w^3/6 - w^4/24: relative error below 6e-8 there,
// where 1 - 2^u from a rounded 2^u loses digits.
constexpr float ABSORBED_SERIES_U = 0.072134752f;
__device__ __forceinline__ float absorbed_series(float u)
{
    constexpr float c1 = -0.69314718f, c2 = -0.24022651f, c3 = -0.05550411f, c4 = -0.0096181291f;
    return u * (c1 + u * (c2 + u * (c3 + u * c4)));
}


// Lane-ordered prefix of a wave ballot: the number of set bits below the
// calling lane.
__device__ __forceinline__ uint32_t lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// wave_reserve for n_lane < 8, with three ballots in place of a shuffle scan.
__device__ __forceinline__ uint32_t wave_reserve_small(uint32_t* ctr, uint32_t n_lane)
{
    const unsigned long long m0 = __ballot(n_lane & 1u), m1 = __ballot(n_lane & 2u), m2 = __ballot(n_lane & 4u);
    const uint32_t total = (uint32_t)__popcll(m0) + 2u * (uint32_t)__popcll(m1) + 4u * (uint32_t)__popcll(m2);
    if (total == 0) return 0;
    uint32_t base = 0;
    if ((threadIdx.x & (WAVE - 1)) == 0) base = g_atomic_add(ctr, total);
    base = __shfl(base, 0, WAVE);
    return base + lanes_below(m0) + 2u * lanes_below(m1) + 4u * lanes_below(m2);
}

// wave_reserve_small in two halves, so that other work can run while the
// atomic is in flight: begin issues it (its result lands in lane 0's *raw)
// and returns the lane's offset; end broadcasts the base.
__device__ __forceinline__ uint32_t reserve_begin(uint32_t* ctr, uint32_t n_lane, uint32_t* raw)
{
    const unsigned long long m0 = __ballot(n_lane & 1u), m1 = __ballot(n_lane & 2u), m2 = __ballot(n_lane & 4u);
    const uint32_t total = (uint32_t)__popcll(m0) + 2u * (uint32_t)__popcll(m1) + 4u * (uint32_t)__popcll(m2);
    *raw = 0;
    if ((threadIdx.x & (WAVE - 1)) == 0 && total) *raw = g_atomic_add(ctr, total);
    return lanes_below(m0) + 2u * lanes_below(m1) + 4u * lanes_below(m2);
}

__device__ __forceinline__ uint32_t reserve_end(uint32_t raw, uint32_t off) { return uni(raw) + off; }

// A packet's origin and photons per bin per unit cast weight, from the
// solve's source tables or (merged packets) its virtual-origin table, all
// loads issued together.
template <typename Real, int NB>
__device__ __forceinline__ void source_of(uint32_t src, const double* pos_t, const Real* spec_t, const FrtVSrc* vt_t,
                                          Real s[3], Real spec[NB])
{
    if (!is_virtual(src)) {
        double o[3];
#pragma unroll
        for (int a = 0; a < 3; a++) o[a] = ld_global(pos_t + (size_t)src * 3 + a);
#pragma unroll
        for (int b = 0; b < NB; b++) spec[b] = ld_global(spec_t + (size_t)src * NB + b);
#pragma unroll
        for (int a = 0; a < 3; a++) s[a] = (Real)o[a];
    } else {
        const FrtVSrc* v = vt_t + (src & ~FRT_VSRC);
#pragma unroll
        for (int a = 0; a < 3; a++) s[a] = (Real)ld_global(&v->pos[a]);
#pragma unroll
        for (int b = 0; b < NB; b++) spec[b] = (Real)ld_global(&v->spec[b]);
    }
}

// One workgroup per work item (one brick, up to FRT_ITEM_RAYS packets).
// The item's packets are first ordered by their expected crossings (a
// counting sort in LDS), then each lane walks one packet cell by cell.
// Per segment of length ds (cells) in cell i and bin nu:
//   tau    = (s_nu a_i + b_i) ds,  a_i = n_HI sigma_0 dx, b_i = kappa dx
//   N_in   = N0 exp(-tau_sum)      (tau_sum carried with Kahan compensation)
//   Gamma_i += K_nu N_in ds phi(tau),  phi = (1 - e^-tau)/tau,
//   K_nu = R_ref sigma_nu / (dx^2 dt)
// which is Eq. gamma_avg_subgrid with lambda = 1/(n_HI sigma + kappa)
// (Eq. gamma_initial_standard when kappa = 0).  Without sub-grid opacity
// (SUB = false) K_nu ds phi = (K_nu / s_nu) (1 - e^-tau) / a_i, and
// K_nu / s_nu is the same for every bin, so the deposit is one constant
// times the absorbed photons over a_i: the march adds up each cell's
// absorbed photons and the sum is scaled once when the brick's deposits are
// added (a_i > 0 everywhere: the opacity has a tiny floor).  End states in order: distance cap,
// flux floor, split radius (Eq. r_split), leaving the box, travel budget;
// leaving the brick hands the packet to the next pass.  Ledger terms are
// reduced per wave and added into LDS; output keys are counted in an LDS
// table and added to the histogram once per work item.
template <typename Real, int NB, bool SUB, int LX, int LY, int LZ, int BT, bool HEAT = false>
__device__ __forceinline__ void brick_march(const FrtSolveDesc* __restrict__ descs, FrtWS& ws)
{
    using R2 = typename Vec2<Real>::T;
    constexpr bool F32 = sizeof(Real) == 4;
    constexpr int BX = 1 << LX, BY = 1 << LY, BZ = 1 << LZ;
    constexpr int BC = BX * BY * BZ;
    // a full item: FRT_ITEM_RAYS packets for 256 threads, FRT_ITEM_MAX for 1024
    constexpr int ITEM = BT >= 1024 ? (int)FRT_ITEM_MAX : (int)FRT_ITEM_RAYS;
    constexpr int PER = ITEM / BT;           // packets per thread in a full item
    constexpr int NST = BC / BT;             // brick cells staged per thread
    static_assert(BC % BT == 0 && ITEM % BT == 0 && ITEM <= 65536 && FRT_KEY_BINS == 64, "brick and item shapes");
    constexpr int NBIN = FRT_KEY_BINS;
    // staged opacity: {a_i, b_i} with sub-grid opacity, a_i alone without
    using OpT = typename std::conditional<SUB, R2, Real>::type;
    // the brick's opacity with one plane of guard cells on each side: the
    // march reads the next cell's opacity one step ahead, and a step across
    // a brick face lands at most one plane outside the brick (the value read
    // there is never used)
    constexpr int PADC = BX * BY;
    __shared__ OpT s_op[BC + 2 * PADC];
    // deposits: in the FP32 march as 64-bit fixed point (LDS integer atomics
    // run at the rate of plain stores here, FP32 LDS atomics far slower),
    // in the FP64 march as FP64
    constexpr bool INTDEP = F32;
    using GT = typename std::conditional<INTDEP, unsigned long long, Real>::type;
    __shared__ GT s_g[BC];
    // photo-heating (temperature evolution; the sub-grid layout only): each
    // cell's energy above 13.6 eV of the photons HI absorbed, LDS atomics in
    // the march's precision
    static_assert(!HEAT || SUB, "the heating march uses the sub-grid layout");
    __shared__ Real s_h[HEAT ? BC : 1];
    __shared__ double s_lf[LF_NF];
    __shared__ unsigned long long s_lc[LC_NC];
    __shared__ uint32_t s_key[KEY_SLOTS], s_cnt[KEY_SLOTS];
    __shared__ uint32_t s_bin[NBIN];
    // the current generation's packets in march order, as their record
    // indices (in the pass input for generation 0, in the scratch records
    // after it), so that a chunk's records are one load away
    __shared__ uint32_t s_order[ITEM];
    __shared__ uint32_t s_nv, s_chunk, s_next, s_xn;
    __shared__ uint8_t s_par[BT / WAVE][16];   // lanes of a round's split parents, per wave
    const uint32_t nwork = ws.ctr[C_NWORK];
    const uint32_t np = ws.ctr[C_NP] < ws.pcap ? ws.ctr[C_NP] : ws.pcap;
    const FrtRecs in_q = in_recs(ws);
    // this workgroup's scratch records for split children kept in the brick
    const uint32_t x_cap = min((uint32_t)(2 * ITEM), ws.xrec_cap / gridDim.x);
    const uint32_t x_base = blockIdx.x * x_cap;
    const FrtRecs x_q{ws.xrec, ws.xrec_cap};
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    if (threadIdx.x < LF_NF) s_lf[threadIdx.x] = 0.0;
    if (threadIdx.x < LC_NC) s_lc[threadIdx.x] = 0;
    if (threadIdx.x < KEY_SLOTS) { s_key[threadIdx.x] = 0xffffffffu; s_cnt[threadIdx.x] = 0; }
    int cs = -1;
    // workgroups take items in list order from a counter as they finish
    // one; the next index is fetched while the current item runs
    if (threadIdx.x == 0) s_next = atomicAdd(&ws.ctr[C_NEXT], 1u);
    __syncthreads();
    for (uint32_t item = uni(s_next); item < nwork; item = uni(s_next)) {
        FrtWork w = ws.work[item];
        w.key = uni(w.key);
        w.start = uni(w.start);
        w.count = uni(w.count);
        w.solve = uni(w.solve);
        __syncthreads();
        if ((int)w.solve != cs) {
            if (cs >= 0 && threadIdx.x < LF_NF + LC_NC) {
                FrtLedgerDev* L = descs[cs].L;
                const int stripe = blockIdx.x % FRT_STRIPES;
                if (threadIdx.x < LF_NF) {
                    if (s_lf[threadIdx.x] != 0.0) atomicAdd(&L->sd[stripe][threadIdx.x], s_lf[threadIdx.x]);
                    s_lf[threadIdx.x] = 0.0;
                } else {
                    const int c = threadIdx.x - LF_NF;
                    if (s_lc[c]) atomicAdd(&L->sc[stripe][c], s_lc[c]);
                    s_lc[c] = 0;
                }
            }
            cs = (int)w.solve;
        }
        const FrtSolveDesc& D = descs[w.solve];
        // per-solve constants of the march, held in scalar registers
        Real srel[NB], Kb[NB], sl2[NB], heps[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) {
            srel[b] = uni(srel_of<Real>(D, b));
            Kb[b] = SUB ? uni(K_of<Real>(D, b)) : Real(0);
            sl2[b] = uni((Real)D.sig_l2[b]);                // -log2(e) s_nu
            heps[b] = HEAT ? uni((Real)D.heat_ev[b]) : Real(0);   // eV per photon HI absorbs
        }
        const Real KS = uni(F32 ? (Real)D.KS : (Real)D.KSd);
        // the HI optical depth per segment (at sigma_0) below which every bin's
        // absorbed fraction comes from the series (the softest bin has the
        // largest |u|)
        Real smax = 0;
#pragma unroll
        for (int b = 0; b < NB; b++) smax = fmax(smax, -(Real)sl2[b]);
        const Real ta_ser = uni((Real)ABSORBED_SERIES_U / smax);
        const float dsc = uni(D.dep_scale);   // fixed-point units per photon
        const uint32_t lb = w.key - uni(D.key_base);
        const int bx = (int)(lb % (uint32_t)D.bpx), by = (int)((lb / (uint32_t)D.bpx) % (uint32_t)D.bpy),
                  bz = (int)(lb / ((uint32_t)D.bpx * (uint32_t)D.bpy));
        const int ox = bx * BX, oy = by * BY, oz = bz * BZ;
        const int nx = uni(D.nx), ny = uni(D.ny), nz = uni(D.nz);
        const Real* __restrict__ opa = (const Real*)D.op_a;
        const Real* __restrict__ opb = (const Real*)D.op_b;
        // all of the item's loads at once: its packets' crossing bins (NBIN
        // marks no packet), then the brick's opacities (-1 for cells outside
        // the grid, which a packet reaching them has left the box through)
        uint32_t eq[PER], ei[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const uint32_t j = (uint32_t)q * BT + threadIdx.x;
            eq[q] = NBIN;
            ei[q] = 0;
            if (j < w.count && w.start + j < np) {
                const uint2 e = ws.sorted[w.start + j];
                eq[q] = e.y;
                ei[q] = e.x;
            }
        }
        R2 st[NST];
#pragma unroll
        for (int k = 0; k < NST; k++) {
            const int t = k * BT + (int)threadIdx.x;
            const int lx = t & (BX - 1), ly = (t >> LX) & (BY - 1), lz = t >> (LX + LY);
            const int cx = ox + lx, cy = oy + ly, cz = oz + lz;
            st[k].x = Real(-1);
            st[k].y = Real(0);
            if (cx < nx && cy < ny && cz < nz) {
                const size_t ci = (size_t)cx + (size_t)nx * ((size_t)cy + (size_t)ny * (size_t)cz);
                st[k].x = opa[ci];
                if constexpr (SUB) st[k].y = opb[ci];
            }
        }
        // the next item's index, fetched while these loads are in flight
        uint32_t next_raw = 0;
        if (threadIdx.x == 0) next_raw = atomicAdd(&ws.ctr[C_NEXT], 1u);
#pragma unroll
        for (int k = 0; k < NST; k++) {
            const int t = k * BT + (int)threadIdx.x;
            if constexpr (SUB) s_op[PADC + t] = st[k];
            else s_op[PADC + t] = st[k].x;
            s_g[t] = GT(0);
            if constexpr (HEAT) s_h[t] = Real(0);
        }
        if (threadIdx.x < NBIN) s_bin[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            s_chunk = 0;
            s_xn = 0;
        }
        __syncthreads();
        // ---- order packets by expected crossings: a counting sort of up to
        // ITEM packets (bin NBIN: no packet) into s_order, whose bin counts
        // are taken once per distinct bin of a wave; s_bin starts at zero
        auto order_by_bin = [&](const uint32_t* eqv, const uint32_t* idxv) -> uint32_t {
            uint32_t slot_of[PER];
#pragma unroll
            for (int q = 0; q < PER; q++) {
                const uint32_t e = eqv[q];
                const bool valid = e < (uint32_t)NBIN;
                unsigned long long peers = __ballot(valid);
#pragma unroll
                for (int b = 0; b < 6; b++) {
                    const bool bit = (e >> b) & 1u;
                    const unsigned long long m = __ballot(bit);
                    peers &= bit ? m : ~m;
                }
                const int leader = valid ? __ffsll(peers) - 1 : lane;
                uint32_t base = 0;
                if (valid && lane == leader) base = atomicAdd(&s_bin[e], (uint32_t)__popcll(peers));
                base = (uint32_t)__shfl((int)base, leader, WAVE);
                slot_of[q] = valid ? ((e << 16) | (base + lanes_below(peers))) : 0xffffffffu;
            }
            __syncthreads();
            if (threadIdx.x < WAVE) {
                uint32_t tot;
                const uint32_t v = s_bin[threadIdx.x];
                s_bin[threadIdx.x] = wave_excl_scan(v, &tot);
                if (threadIdx.x == 0) s_nv = tot;
            }
            __syncthreads();
            const uint32_t n = s_nv;
#pragma unroll
            for (int q = 0; q < PER; q++)
                if (slot_of[q] != 0xffffffffu)
                    s_order[s_bin[slot_of[q] >> 16] + (slot_of[q] & 0xffffu)] = idxv[q];
            __syncthreads();
            return n;
        };
        if (threadIdx.x == 0) s_next = next_raw;   // read once this item is done
        // packets of the current generation (one wave's worth needs no order)
        const uint32_t n_item = w.start < np ? min(w.count, np - w.start) : 0u;
        uint32_t n_cur = n_item;
        if (n_item <= (uint32_t)WAVE) {
            if (threadIdx.x < n_item) s_order[threadIdx.x] = ei[0];
            __syncthreads();
        } else {
            n_cur = order_by_bin(eq, ei);
        }
        const Real r_cap = uni((Real)D.r_cap);
        const Real floor_f = uni((Real)D.floor);
        const double Rr = uni(D.R_ref);
        const int max_level = uni(D.max_level), base_level = uni(D.base_level);
        // Generalized Opacity Mode (only with the sub-grid layout): .x of a
        // staged cell is the ionized part's opacity per cell width at sigma_0,
        // .y the ionized volume fraction
        const bool gmode = SUB && uni(D.gen) != 0;
        const Real budget = uni((Real)D.budget);
        const uint32_t step = uni(D.step);
        // the source tables, taken once per item
        const double* const pos_t = D.src_pos;
        const Real* spec_t;
        if constexpr (F32) spec_t = D.spec;
        else spec_t = D.specd;
        const FrtVSrc* const vt_t = D.vt[D.cur];
        // absorbed photons and crossings of this lane's packets, reduced
        // over the wave once per item
        double acc_abs = 0.0;
        uint32_t acc_cross = 0;
        // Generation 0 marches the item's packets; split children that start
        // in this brick are kept in the workgroup's scratch records and
        // marched by the next generation while the brick is still staged
        // (their own children likewise), the rest go to the next pass.
        uint32_t g_lo = 0, g_hi = 0;   // scratch records of the current generation
        for (int gen = 0;; gen++) {
            // waves take chunks of 64 sorted packets as they finish, longest
            // chunks first, so that the waves end together
            const uint32_t n_chunks = (n_cur + WAVE - 1) / WAVE;
            for (;;) {
                uint32_t chunk = 0;
                if (lane == 0) chunk = atomicAdd(&s_chunk, 1u);
                chunk = uni(chunk);
                if (chunk >= n_chunks) break;
                const uint32_t p = (n_chunks - 1u - chunk) * WAVE + (uint32_t)lane;
                const bool active = p < n_cur;
                Pkt<Real> h;
                Real T[4], NE[NB], N0[NB], s[3];   // NE: photons of each bin (units of the cast weight)
                Real inv_d[3] = {Real(0), Real(0), Real(0)};   // 1 / direction, per axis
                int level = 0, end = -1;     // -1 inactive, 0 split, 1 escaped, 2 dropped, 3 in flight, 4 next brick
                int c[3] = {0, 0, 0};
                double v_abs = 0.0, v_sub = 0.0, v_end = 0.0;
                uint32_t v_cross = 0;
                if (active) {
                    if (gen == 0) load_pkt<Real>(in_q, s_order[p], h, T);
                    else load_pkt<Real>(x_q, s_order[p], h, T);
                    level = (int)(h.lp >> 28);
                    Real spec[NB];
                    source_of<Real, NB>(h.src, pos_t, spec_t, vt_t, s, spec);
                    if (h.estep != step && h.rstop <= h.r) h.rstop = h.r + budget;   // carried: fresh budget
                    if (h.estep == step && h.r == Real(0) && level == base_level) h.rstop = budget;
                    Real sum0 = 0;
                    double n_start = 0.0;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        N0[b] = h.w0 * spec[b];
                        NE[b] = N0[b] * (SUB ? exp_neg(srel[b] * T[0] + T[1]) : exp_neg(srel[b] * T[0]));
                        sum0 += N0[b];
                        n_start += (double)NE[b];
                    }
                    unpack_cell(h.cell, c);
                    const Real r_split = split_radius<Real>(D, level);
                    // the nearest of split radius, distance cap and budget end
                    const Real r_lim = fmin(fmin(r_split, r_cap), h.rstop);
                    // distance to the next face along each axis, and the distance
                    // between faces (Amanatides-Woo): the next face along an axis
                    // is reached after one more cell's distance along it
                    Real dtf[3], rf[3];
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        inv_d[a] = (h.d[a] != Real(0)) ? fast_rcp(h.d[a]) : Real(0);
                        dtf[a] = fabs(inv_d[a]);
                        rf[a] = (h.d[a] != Real(0)) ? ((Real)(c[a] + (h.d[a] > Real(0) ? 1 : 0)) - s[a]) * inv_d[a] : rinf<Real>();
                    }
                    // the cell's index in the staged brick, x fastest; a step along
                    // an axis changes only that axis's bit field of the index
                    // unless it leaves the brick (a carry or borrow out of the
                    // field), and the z guard planes keep the next cell's
                    // prefetch inside the array either way
                    const int inc[3] = {h.d[0] > Real(0) ? 1 : -1, h.d[1] > Real(0) ? BX : -BX,
                                        h.d[2] > Real(0) ? BX * BY : -(BX * BY)};
                    constexpr int NOT_X = ~(BX - 1), NOT_Y = ~((BY - 1) << LX), NOT_Z = ~((BZ - 1) << (LX + LY));
                    const int lc0 = c[0] - ox, lc1 = c[1] - oy, lc2 = c[2] - oz;
                    const bool in_brick = lc0 >= 0 && lc0 < BX && lc1 >= 0 && lc1 < BY && lc2 >= 0 && lc2 < BZ;
                    int li = in_brick ? lc0 + BX * (lc1 + BY * lc2) : 0;
                    if (!in_brick) end = 4;            // hand it to the brick that holds its cell
                    const bool floor_on = floor_f > Real(0);
                    const Real floor_abs = floor_f * sum0;
                    // photons left (in units of the cast weight), for the flux floor
                    Real S = 0;
#pragma unroll
                    for (int b = 0; b < NB; b++) S += NE[b];
                    // this visit's optical depth (HI part at sigma_0, sub-grid
                    // part), added to the packet's compensated sums at its end
                    Real tsum = 0, ksum = 0;
                    Real sub_acc = 0;
                    if (end < 0) {
                        // the opacity of the current cell; each step reads the next
                        // cell's one iteration ahead
                        OpT o_cur = s_op[PADC + li];
                        bool front = false;   // stopped at the cell's I-front (Generalized Opacity Mode)
                        // the loop keeps no per-step flags: at its exit, li, rf, S and
                        // h.r are those of its last step, which the exit recomputes
                        for (;;) {
                            const Real r_face = fmin(fmin(rf[0], rf[1]), rf[2]);
                            // the axis of the nearest face (ties to the lowest axis)
                            const bool a0 = rf[0] == r_face;
                            const bool a1 = !a0 && rf[1] == r_face;
                            const int li_n = li + (a0 ? inc[0] : (a1 ? inc[1] : inc[2]));
                            const bool out = ((li ^ li_n) & (a0 ? NOT_X : (a1 ? NOT_Y : NOT_Z))) != 0;
                            const OpT o_next = s_op[PADC + li_n];
                            Real r_end;
                            if constexpr (F32) r_end = __builtin_amdgcn_fmed3f(r_face, r_lim, h.r);
                            else r_end = fmax(fmin(r_face, r_lim), h.r);
                            const Real ds = r_end - h.r;
                            // the deposit's LDS atomic is issued on every path (adding
                            // 0 for an empty segment), so that waiting for the next
                            // cell's prefetched opacity never waits for it
                            Real dep = 0;
                            Real hdep = 0;   // photo-heating of the segment, eV (HEAT)
                            if constexpr (F32 && !SUB) {
                                // u = -log2(e) s_nu tau_0: each bin's transmission is
                                // 2^u.  The cell's absorbed photons: while even the
                                // softest bin's u is above -0.0721 (optical depth
                                // 0.05), the sum over bins of N_nu (1 - 2^u) from its
                                // series (valid there for every bin); beyond it the
                                // drop of the photons' sum, which is then at least 5%
                                // of the softest bin's photons (an empty segment
                                // changes nothing).  When every lane of the wave is
                                // in the series range the photons left are N_nu
                                // minus that series too, and no 2^u is evaluated.
                                const Real ta = o_cur * ds;
                                const bool thin = ta < ta_ser;
                                if (__ballot(!thin) == 0ull) {
                                    Real A = 0;
#pragma unroll
                                    for (int b = 0; b < NB; b++) {
                                        const Real d = NE[b] * absorbed_series(sl2[b] * ta);
                                        A += d;
                                        NE[b] -= d;
                                    }
                                    dep = A;
                                    S -= A;
                                } else {
                                    Real S_new = 0, A_ser = 0;
#pragma unroll
                                    for (int b = 0; b < NB; b++) {
                                        const Real u = sl2[b] * ta;
                                        A_ser += NE[b] * absorbed_series(u);
                                        NE[b] *= __builtin_amdgcn_exp2f(u);
                                        S_new += NE[b];
                                    }
                                    dep = thin ? A_ser : S - S_new;
                                    S = S_new;
                                }
                                tsum += ta;
                                v_cross += ds > Real(0) ? 1u : 0u;
                            } else if (ds > Real(0)) {
                                R2 o;
                                if constexpr (SUB) {
                                    o = o_cur;
                                } else {
                                    o.x = o_cur;
                                    o.y = Real(0);
                                }
                                // the path through absorbing gas: the ionized part
                                // x_ion ds in the Generalized Opacity Mode (whose
                                // rate keeps the whole ds: Eq. gamma_avg_subgrid
                                // with ds -> x_ion ds and V -> x_ion V)
                                const Real ta = o.x * (gmode ? o.y * ds : ds);
                                if (gmode) front = o.y < Real(1);
                                Real absd = 0;
                                if constexpr (SUB) {
                                    const Real tk = gmode ? Real(0) : o.y * ds;
#pragma unroll
                                    for (int b = 0; b < NB; b++) {
                                        const Real tb = srel[b] * ta + tk;
                                        const Real nin = NE[b];
                                        const Real eb = exp_neg(tb);
                                        const Real af = absorbed<Real>(tb, eb);
                                        const Real rt = fast_rcp(tb);
                                        const Real phi = (tb > Real(0)) ? af * rt : Real(1);
                                        dep += Kb[b] * nin * ds * phi;
                                        absd += nin * af;
                                        if (tk > Real(0)) sub_acc += nin * af * tk * rt;
                                        // the HI share of the bin's absorbed photons
                                        if constexpr (HEAT)
                                            hdep += (tb > Real(0)) ? heps[b] * nin * af * (srel[b] * ta) * rt : Real(0);
                                        NE[b] *= eb;
                                    }
                                    ksum += tk;
                                } else {
#pragma unroll
                                    for (int b = 0; b < NB; b++) {
                                        const Real tb = srel[b] * ta;
                                        const Real eb = exp_neg(tb);
                                        absd += NE[b] * absorbed<Real>(tb, eb);
                                        NE[b] *= eb;
                                    }
                                    // the cell's absorbed photons; times KS / a_i when
                                    // the brick's deposits are added
                                    dep = absd;
                                }
                                S -= absd;
                                tsum += ta;
                                v_cross++;
                            }
                            if constexpr (INTDEP) {
                                // whole units of the fixed point (dep <= 2^46 units),
                                // split exactly into the two words of the 64-bit add
                                const float x = __builtin_rintf(dep * dsc);
                                const uint32_t hi = (uint32_t)(x * 0x1p-32f);
                                const uint32_t lo = (uint32_t)__builtin_fmaf(-(float)hi, 0x1p32f, x);
                                atomicAdd(&s_g[li], ((unsigned long long)hi << 32) | lo);
                            } else {
                                atomicAdd(&s_g[li], dep);
                            }
                            if constexpr (HEAT) atomicAdd(&s_h[li], hdep);
                            h.r = r_end;
                            Real o_n;   // HI opacity of the next cell (< 0 outside the grid)
                            if constexpr (SUB) o_n = o_next.x;
                            else o_n = o_next;
                            // any end before or after the step: the exit below sorts it
                            // out (one test of all conditions, so that the next cell's
                            // opacity is read ahead of it rather than inside it)
                            const bool stop = front | (floor_on & (S < floor_abs)) | (h.r >= r_lim) | out | (o_n < Real(0));
                            if (stop) break;
                            li = li_n;
                            const Real rfa = r_face + (a0 ? dtf[0] : (a1 ? dtf[1] : dtf[2]));
                            rf[0] = a0 ? rfa : rf[0];
                            rf[1] = a1 ? rfa : rf[1];
                            rf[2] = (a0 || a1) ? rf[2] : rfa;
                            o_cur = o_next;
                        }
                        // the last step's face, axis, next cell and floor test,
                        // recomputed here (the empty asm keeps the compiler from
                        // carrying the loop's per-step flags out of it instead)
                        Real rx = rf[0], ry = rf[1], rz = rf[2];
                        asm volatile("" : "+v"(rx), "+v"(ry), "+v"(rz));
                        const Real r_face = fmin(fmin(rx, ry), rz);
                        const bool a0 = rx == r_face;
                        const bool a1 = !a0 && ry == r_face;
                        const int li_n = li + (a0 ? inc[0] : (a1 ? inc[1] : inc[2]));
                        const bool out = ((li ^ li_n) & (a0 ? NOT_X : (a1 ? NOT_Y : NOT_Z))) != 0;
                        const OpT o_next = s_op[PADC + li_n];
                        const bool floored = floor_on && S < floor_abs;
                        // end states before the step, in order: distance cap, flux
                        // floor, split, then the budget (a face reached with it is
                        // crossed first)
                        int e_pre = (h.r >= r_lim)
                                        ? ((h.r >= r_cap || floored) ? 2 : (h.r >= r_split ? 0 : (h.r < r_face ? 3 : -1)))
                                        : (floored ? 2 : -1);
                        if (front) e_pre = 5;   // (only in the Generalized Opacity Mode)
                        int lc[3] = {li & (BX - 1), (li >> LX) & (BY - 1), li >> (LX + LY)};
                        if (e_pre >= 0) {
                            end = e_pre;
                        } else {
                            // the face is crossed: leaving the brick (and the box,
                            // when the brick's face is the box's), a cell outside
                            // the grid within the brick (the box left), or the
                            // budget spent on the face
                            const int axis = a0 ? 0 : (a1 ? 1 : 2);
                            const int sgn = (axis == 0 ? h.d[0] : (axis == 1 ? h.d[1] : h.d[2])) > Real(0) ? 1 : -1;
                            lc[0] += axis == 0 ? sgn : 0;
                            lc[1] += axis == 1 ? sgn : 0;
                            lc[2] += axis == 2 ? sgn : 0;
                            const bool spent = h.r >= h.rstop;
                            Real o_n;
                            if constexpr (SUB) o_n = o_next.x;
                            else o_n = o_next;
                            if (out) {
                                const int ca = axis == 0 ? ox + lc[0] : (axis == 1 ? oy + lc[1] : oz + lc[2]);
                                const int dima = axis == 0 ? nx : (axis == 1 ? ny : nz);
                                end = (ca < 0 || ca >= dima) ? 1 : (spent ? 3 : 4);
                            } else {
                                end = o_n < Real(0) ? 1 : 3;
                            }
                        }
                        c[0] = ox + lc[0];
                        c[1] = oy + lc[1];
                        c[2] = oz + lc[2];
                        // the visit's optical depth into the packet's compensated sums
                        {
                            const Real y = tsum - T[2];
                            const Real t = T[0] + y;
                            T[2] = (t - T[0]) - y;
                            T[0] = t;
                        }
                        if constexpr (SUB) {
                            if (ksum > Real(0)) {
                                const Real y = ksum - T[3];
                                const Real t = T[1] + y;
                                T[3] = (t - T[1]) - y;
                                T[1] = t;
                            }
                        }
                    }
                    // photons at the end of the visit from the carried optical
                    // depth, exactly as the next visit will recompute them
                    double n_end = 0.0;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        n_end += (double)(N0[b] * (SUB ? exp_neg(srel[b] * T[0] + T[1]) : exp_neg(srel[b] * T[0])));
                    }
                    if constexpr (SUB) v_sub = (double)sub_acc * Rr;
                    v_abs = (n_start - n_end) * Rr - v_sub;
                    v_end = n_end * Rr;
                    h.cell = pack_cell(c);
                }
                // ---- slots in the next pass's input for packets entering another
                // brick, reserved with one atomic before the ledger reductions,
                // which run while it flies
                const unsigned long long m_next = __ballot(end == 4), m_par = __ballot(end == 0);
                const uint32_t n_out = (uint32_t)__popcll(m_next);
                uint32_t o_raw = 0;
                if (lane == 0 && n_out) o_raw = g_atomic_add(o_ctr(ws, my_seg()), n_out);
                const uint32_t ocap_seg = seg_cap(ws.buf[0].cap);
                const uint32_t oseg0 = (uint32_t)my_seg() * ocap_seg;
                // ---- ledger: counts from ballots, photon terms from wave sums
                // taken only when some lane of the wave has one
                {
                    const bool esc = end == 1, drop = end == 2, fl = end == 3;
                    const unsigned long long m_act = __ballot(active), m_split = __ballot(end == 0),
                                             m_esc = __ballot(esc), m_drop = __ballot(drop), m_fl = __ballot(fl);
                    acc_abs += v_abs;
                    acc_cross += v_cross;
                    double t_sub = 0.0, t_esc = 0.0, t_drop = 0.0, t_fl = 0.0;
                    if constexpr (SUB) t_sub = wave_sum(v_sub);
                    if (m_esc) t_esc = wave_sum(esc ? v_end : 0.0);
                    if (m_drop) t_drop = wave_sum(drop ? v_end : 0.0);
                    if (m_fl) t_fl = wave_sum(fl ? v_end : 0.0);
                    if (lane == 0) {
                        if (t_sub != 0.0) atomicAdd(&s_lf[LF_ABS_SUB], t_sub);
                        if (t_esc != 0.0) atomicAdd(&s_lf[LF_ESC], t_esc);
                        if (t_drop != 0.0) atomicAdd(&s_lf[LF_DROP], t_drop);
                        if (t_fl != 0.0) atomicAdd(&s_lf[LF_FLIGHT], t_fl);
                        if (m_act) atomicAdd(&s_lc[LC_VISITS], (unsigned long long)__popcll(m_act));
                        if (m_split) atomicAdd(&s_lc[LC_SPLITS], (unsigned long long)__popcll(m_split));
                        if (m_esc) atomicAdd(&s_lc[LC_NESC], (unsigned long long)__popcll(m_esc));
                        if (m_drop) atomicAdd(&s_lc[LC_NDROP], (unsigned long long)__popcll(m_drop));
                        if (m_fl) atomicAdd(&s_lc[LC_NFLIGHT], (unsigned long long)__popcll(m_fl));
                    }
                    // photons stopped at an I-front: the ledger term, and the
                    // cell's front counter that the chemistry turns into x_ion
                    if (gmode) {
                        const bool fr = end == 5;
                        if (__ballot(fr)) {
                            const double t_fr = wave_sum(fr ? v_end : 0.0);
                            if (lane == 0) atomicAdd(&s_lf[LF_ABS_SUB], t_fr);   // the front term here
                            if (fr) atomicAdd(&D.front[(size_t)c[0] + (size_t)nx * ((size_t)c[1] + (size_t)ny * (size_t)c[2])], v_end);
                        }
                    }
                }
                // keys of the packets entering another brick, computed while the
                // reservation flies
                uint32_t key = 0;
                if (end == 4) key = key_with_bin(brick_key(D, c), crossing_bin_inv<Real>(D, c, s, h.d, inv_d, h.r, h.rstop, level));
                const uint32_t o_base = n_out ? reserve_end(o_raw, 0u) : 0u;
                // ---- packets entering another brick go to the next pass
                {
                    bool stored = false;
                    if (end == 4) {
                        const uint32_t at = o_base + lanes_below(m_next);
                        if (at < ocap_seg) {
                            store_out<Real>(ws, oseg0 + at, h, key, T);
                            stored = true;
                        } else {
                            raise_error(ws, D.L, FRT_DEVERR_QUEUE_OVERFLOW);
                            atomicAdd(&s_lf[LF_LOST], v_end);
                        }
                    }
                    if (m_next) count_keys_wave(s_key, s_cnt, ws.hist, key & FRT_KEY_MASK, stored);
                }
                // ---- children of the packets at their split radius (Eq. lhpx):
                // level + 1, NESTED pixels 4p .. 4p + 3, a quarter of the photons
                // each, the parent's rotation, placed on their own pixel direction
                // at the split radius; a child whose position is outside the box
                // has escaped.  Up to 16 parents a round, four lanes per parent
                // and one child per lane, so that the wave's lanes stay busy.
                for (unsigned long long todo = m_par; todo;) {
                    const bool mine = ((todo >> lane) & 1ull) != 0;
                    const uint32_t rk = lanes_below(todo);
                    const bool now = mine && rk < 16u;
                    const uint32_t npar = min((uint32_t)__popcll(todo), 16u);
                    if (now) s_par[wv][rk] = (uint8_t)lane;
                    const uint32_t q = (uint32_t)lane >> 2, kq = (uint32_t)lane & 3u;
                    const bool cact = q < npar;
                    const int pl = cact ? (int)s_par[wv][q] : lane;
                    Pkt<Real> ch;
                    Real cT[4], cs[3];
                    ch.src = (uint32_t)__shfl((int)h.src, pl, WAVE);
                    ch.estep = (uint32_t)__shfl((int)h.estep, pl, WAVE);
                    const uint32_t plp = (uint32_t)__shfl((int)h.lp, pl, WAVE);
                    ch.r = __shfl(h.r, pl, WAVE);
                    ch.rstop = __shfl(h.rstop, pl, WAVE);
                    ch.w0 = __shfl(h.w0, pl, WAVE) * Real(0.25);
#pragma unroll
                    for (int b = 0; b < 4; b++) cT[b] = __shfl(T[b], pl, WAVE);
#pragma unroll
                    for (int a = 0; a < 3; a++) cs[a] = __shfl(s[a], pl, WAVE);
                    const double cph = 0.25 * __shfl(v_end, pl, WAVE);
                    const int clev = (int)(plp >> 28) + 1;
                    ch.lp = ((uint32_t)clev << 28) | (4u * (plp & 0x0fffffffu) + kq);
                    bool inside = false;
                    uint32_t ckey = 0;
                    if (cact) {
                        packet_dir<Real>(D, ch.lp, ch.estep, ch.src, ch.d);
                        int cc[3];
                        inside = locate<Real>(D, cs, ch.r, ch.d, cc);
                        if (inside) {
                            ch.cell = pack_cell(cc);
                            ckey = key_with_bin(brick_key(D, cc), crossing_bin<Real>(D, cc, cs, ch.d, ch.r, ch.rstop, clev));
                        }
                    }
                    // a child that starts in this brick is kept for the next
                    // generation while the scratch records last; the others go to
                    // the next pass
                    bool keep = inside && (ckey & FRT_KEY_MASK) == w.key;
                    const unsigned long long m_keep = __ballot(keep);
                    if (m_keep) {
                        uint32_t xb = 0;
                        if (lane == 0) xb = atomicAdd(&s_xn, (uint32_t)__popcll(m_keep));
                        const uint32_t xs = uni(xb) + lanes_below(m_keep);
                        // the record keeps the child's crossing bin for the next
                    // generation's ordering
                    if (keep && xs < x_cap) store_pkt<Real>(x_q, x_base + xs, ch, ckey >> FRT_KEY_BITS, cT);
                        else keep = false;
                    }
                    const bool to_o = inside && !keep;
                    bool stored = false;
                    if (__ballot(to_o)) {
                        const uint32_t at = wave_reserve_small(o_ctr(ws, my_seg()), to_o ? 1u : 0u);
                        if (to_o) {
                            if (at < ocap_seg) {
                                store_out<Real>(ws, oseg0 + at, ch, ckey, cT);
                                stored = true;
                            } else {
                                raise_error(ws, D.L, FRT_DEVERR_QUEUE_OVERFLOW);
                                atomicAdd(&s_lf[LF_LOST], cph);
                            }
                        }
                        count_keys_wave(s_key, s_cnt, ws.hist, ckey & FRT_KEY_MASK, stored);
                    }
                    const bool cesc = cact && !inside;
                    const unsigned long long m_cesc = __ballot(cesc);
                    if (m_cesc) {
                        const double t_cesc = wave_sum(cesc ? cph : 0.0);
                        if (lane == 0) {
                            atomicAdd(&s_lf[LF_ESC], t_cesc);
                            atomicAdd(&s_lc[LC_NESC], (unsigned long long)__popcll(m_cesc));
                        }
                    }
                    todo &= ~__ballot(now);
                }
                // ---- packets that spent their travel budget: carried to the next step
                if (__ballot(end == 3)) {
                    const int nxt = 1 - (int)D.cur;
                    const uint32_t fat = wave_reserve_small(&D.fcount[nxt], end == 3 ? 1u : 0u);
                    if (end == 3) {
                        if (fat < D.F[nxt].cap) {
                            store_pkt<Real>(D.F[nxt], fat, h, brick_key(D, c) - D.key_base, T);
                        } else {
                            raise_error(ws, D.L, FRT_DEVERR_CARRY_OVERFLOW);
                            atomicAdd(&s_lf[LF_LOST], v_end);
                        }
                    }
                }
            }
            // next generation: the children kept by this one (the scratch
            // records are written and read by this workgroup only, so the
            // barrier's workgroup-scope ordering makes them visible)
            __syncthreads();
            const uint32_t nx = min(s_xn, x_cap);
            if (nx <= g_hi) break;
            g_lo = g_hi;
            g_hi = min(nx, g_lo + (uint32_t)ITEM);   // the rest in a later round
            __syncthreads();
            if (threadIdx.x == 0) s_chunk = 0;
            if (g_hi - g_lo <= (uint32_t)WAVE) {
                // one wave marches them all: their order makes no difference
                if (threadIdx.x < g_hi - g_lo) s_order[threadIdx.x] = x_base + g_lo + threadIdx.x;
                __syncthreads();
                n_cur = g_hi - g_lo;
                continue;
            }
            if (threadIdx.x < NBIN) s_bin[threadIdx.x] = 0;
            uint32_t ex[PER], xi[PER];
#pragma unroll
            for (int q = 0; q < PER; q++) {
                const uint32_t j = (uint32_t)q * BT + threadIdx.x;
                xi[q] = x_base + g_lo + j;
                ex[q] = j < g_hi - g_lo ? recs<Real>(x_q)[xi[q]].key : (uint32_t)NBIN;
            }
            __syncthreads();
            n_cur = order_by_bin(ex, xi);
        }
        {
            const double t_abs = wave_sum(acc_abs);
            const uint32_t t_cross = wave_sum_u32(acc_cross);
            if (lane == 0) {
                if (t_abs != 0.0) atomicAdd(&s_lf[LF_ABS_HI], t_abs);
                if (t_cross) atomicAdd(&s_lc[LC_CROSS], (unsigned long long)t_cross);
            }
        }
        __syncthreads();
        // add the brick's deposits and its output-key counts once
        Real* __restrict__ gam = (Real*)D.gamma[D.step & 1u];
        const double dun = 1.0 / (double)dsc;
        for (int t = threadIdx.x; t < BC; t += BT) {
            const GT q = s_g[t];
            if (q != GT(0)) {
                Real v;
                if constexpr (INTDEP) v = (Real)((double)q * dun);
                else v = q;
                if constexpr (!SUB) v = v * (KS * fast_rcp<Real>(s_op[PADC + t]));
                const int lx = t & (BX - 1), ly = (t >> LX) & (BY - 1), lz = t >> (LX + LY);
                const size_t ci = (size_t)(ox + lx) + (size_t)nx * ((size_t)(oy + ly) + (size_t)ny * (size_t)(oz + lz));
                g_atomic_add(gam + ci, v);
            }
        }
        if constexpr (HEAT) {
            // the brick's photo-heating: its energy (eV; the march's photons
            // are in units of R_ref) summed for the ledger, and each cell's
            // heating rate (erg/cm^3/s, a range FP32 holds)
            Real* __restrict__ hp = (Real*)D.heat;
            const double hsc = uni(D.heat_scale);
            double hsum = 0.0;
            if (hp) {
                for (int t = threadIdx.x; t < BC; t += BT) {
                    const Real q = s_h[t];
                    if (q != Real(0)) {
                        const double e = (double)q * Rr;
                        const int lx = t & (BX - 1), ly = (t >> LX) & (BY - 1), lz = t >> (LX + LY);
                        const size_t ci = (size_t)(ox + lx) + (size_t)nx * ((size_t)(oy + ly) + (size_t)ny * (size_t)(oz + lz));
                        atomicAdd(hp + ci, (Real)(e * hsc));
                        hsum += e;
                    }
                }
            }
            hsum = wave_sum(hsum);
            if (lane == 0 && hsum != 0.0) atomicAdd(&s_lf[LF_HEAT], hsum);
        }
        if (threadIdx.x < KEY_SLOTS) {
            const uint32_t k = s_key[threadIdx.x];
            if (k != 0xffffffffu) {
                atomicAdd(&ws.hist[k], s_cnt[threadIdx.x]);
                s_key[threadIdx.x] = 0xffffffffu;
                s_cnt[threadIdx.x] = 0;
            }
        }
    }
    __syncthreads();
    if (cs >= 0 && threadIdx.x < LF_NF + LC_NC) {
        FrtLedgerDev* L = descs[cs].L;
        const int stripe = blockIdx.x % FRT_STRIPES;
        if (threadIdx.x < LF_NF) {
            if (s_lf[threadIdx.x] != 0.0) atomicAdd(&L->sd[stripe][threadIdx.x], s_lf[threadIdx.x]);
        } else {
            const int c = threadIdx.x - LF_NF;
            if (s_lc[c]) atomicAdd(&L->sc[stripe][c], s_lc[c]);
        }
    }
}

// 256-thread march on 16^3 (FP32 with sub-grid opacity) or 8^3 (FP64)
// bricks; HEAT adds the photo-heating deposits of temperature evolution
template <typename Real, int NB, bool SUB, bool HEAT = false>
__global__ void __launch_bounds__(BLOCK) k_brick(const FrtSolveDesc* __restrict__ descs, FrtWS ws)
{
    if (halted(ws)) return;
    if constexpr (sizeof(Real) == 4)
        brick_march<Real, NB, SUB, FRT_BRICK_LOG_SUB[0], FRT_BRICK_LOG_SUB[1], FRT_BRICK_LOG_SUB[2], BLOCK, HEAT>(descs, ws);
    else
        brick_march<Real, NB, SUB, FRT_BRICK_LOG_F64[0], FRT_BRICK_LOG_F64[1], FRT_BRICK_LOG_F64[2], BLOCK, HEAT>(descs, ws);
}

// 1024-thread march on 32 x 16 x 16 bricks (FP32 without sub-grid opacity):
// one workgroup of 16 waves per CU, 128 registers each
template <typename Real, int NB>
__global__ void __launch_bounds__(4 * BLOCK) k_brick_big(const FrtSolveDesc* __restrict__ descs, FrtWS ws)
{
    if (halted(ws)) return;
    brick_march<Real, NB, false, FRT_BRICK_LOG_BIG[0], FRT_BRICK_LOG_BIG[1], FRT_BRICK_LOG_BIG[2], 4 * BLOCK>(descs, ws);
}

// ============================================================ bookkeeping
// Clears the launch counters and the key histogram; a later march of the
// same step keeps the error bits and the largest pass size seen so far.
// Only CLEAR_ALL touches C_HALT and C_DONE, and only it runs under a halt.
__global__ void k_clear(FrtWS ws, int mode)
{
    if (mode != CLEAR_ALL && halted(ws)) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool keep = (mode == CLEAR_ITER && (t == C_ERR || t == C_MAXP)) ||
                      (mode != CLEAR_ALL && (t == C_HALT || t == C_DONE));
    if (t < C_NCTR && !keep) ws.ctr[t] = 0;
    for (uint32_t k = t; k < ws.nkeys; k += stride) ws.hist[k] = 0;
}

// One workgroup of one wave.
__global__ void k_advance(FrtSolveDesc* descs, FrtWS ws)
{
    if (halted(ws)) return;
    if (ws.ctr[C_ERR] != 0) {
        if (threadIdx.x == 0) ws.ctr[C_HALT] = 1u;
        return;
    }
    for (int i = threadIdx.x; i < ws.n_solves; i += blockDim.x) {
        descs[i].step += 1u;
        descs[i].cur ^= 1u;
    }
    if (threadIdx.x == 0) ws.ctr[C_DONE] += 1u;
}

// =============================================================== step close
// After the last pass: anything still queued means the pass count was too
// small (flagged, never expected); fold the ledger stripes.
__global__ void k_finish(FrtSolveDesc* descs, FrtWS ws)
{
    __shared__ int s_left;
    if (halted(ws)) return;
    if (threadIdx.x == 0) s_left = 0;
    __syncthreads();
    if (threadIdx.x < FRT_QSEG && *o_ctr(ws, threadIdx.x) > 0) s_left = 1;
    __syncthreads();
    for (int s = blockIdx.x; s < ws.n_solves; s += gridDim.x) {
        FrtSolveDesc& D = descs[s];
        FrtLedgerDev* L = D.L;
        if (threadIdx.x < LF_NF + LC_NC) {
            const int i = threadIdx.x;
            if (i < LF_NF) {
                double v = 0;
                for (int k = 0; k < FRT_STRIPES; k++) { v += L->sd[k][i]; L->sd[k][i] = 0.0; }
                switch (i) {
                    case LF_EMITTED: L->emitted += v; break;
                    case LF_ABS_HI: L->absorbed_HI += v; break;
                    case LF_ABS_SUB:
                        if (D.gen) L->absorbed_front += v;
                        else L->absorbed_sub += v;
                        break;
                    case LF_ESC: L->escaped += v; break;
                    case LF_DROP: L->dropped += v; break;
                    case LF_FLIGHT: L->in_flight = v; break;
                    case LF_LOST: L->lost += v; break;
                    case LF_HEAT: L->heat_in += v; break;
                }
            } else {
                const int j = i - LF_NF;
                unsigned long long v = 0;
                for (int k = 0; k < FRT_STRIPES; k++) { v += L->sc[k][j]; L->sc[k][j] = 0; }
                switch (j) {
                    case LC_CROSS: L->crossings += v; L->step_crossings = v; break;
                    case LC_VISITS: L->ray_visits += v; break;
                    case LC_SPLITS: L->splits += v; break;
                    case LC_NESC: L->n_escaped += v; break;
                    case LC_NDROP: L->n_dropped += v; break;
                    case LC_NFLIGHT: L->n_in_flight = v; break;
                    case LC_EMITTED: L->rays_emitted += v; break;
                }
            }
        }
        if (threadIdx.x == 0) {
            if (s_left) {
                L->err_flags |= FRT_DEVERR_UNFINISHED;
                atomicOr(&ws.ctr[C_ERR], (uint32_t)FRT_DEVERR_UNFINISHED);
            }
            if (ws.ctr[C_MAXP] > L->max_items) L->max_items = ws.ctr[C_MAXP];
        }
    }
}

// HI opacity per cell width, n_HI sigma_0 dx, with a floor far below any
// value that changes a result (1e-30 in FP32, 1e-300 in FP64): every cell
// then has a_i > 0, and the deposit K ds phi(tau) = (K / s) (1 - e^-tau) / a_i
// needs no separate form for a cell without neutral hydrogen.
template <typename Real>
__device__ __forceinline__ Real hi_opacity(double v)
{
    constexpr double lo = sizeof(Real) == 4 ? 1e-30 : 1e-300;
    return (Real)(v > lo ? v : lo);
}

// ================================================================ chemistry

// Temperature evolution (§4.1, Eq. temp_evolution_standard), pure H gas.
// Rates at temperature T (K), lambda = 2 T_HI / T with T_HI = 157807 K: the
// case-B recombination and collisional ionization coefficients (cm^3/s) of
// Hui & Gnedin 1997, which the paper cites, and cooling coefficients (erg
// cm^3/s): case-B recombination (Hui & Gnedin 1997), collisional ionization
// (k T_HI per ionization), collisional excitation (Cen 1992) and free-free
// (Gaunt factor 1.1 + 0.34 exp(-(5.5 - log10 T)^2 / 3)).
struct HRates {
    double alpha, coll, rec, ci, ce, ff;
};

constexpr double kBoltz = 1.380649e-16;     // erg/K
constexpr double kTHI = 157807.0;           // K
// Compton cooling off the CMB per electron and kelvin of T - T_CMB, at z = 0:
// 4 sigma_T a_rad k T_CMB0^4 / (m_e c), T_CMB0 = 2.725 K
constexpr double kCompton0 = 4.0 * 6.6524587321e-25 * 7.565733e-15 * kBoltz * (2.725 * 2.725 * 2.725 * 2.725) /
                             (9.1093837015e-28 * 2.99792458e10);

// Each power x^a of the fits is exp(a ln x), with ln lambda taken once and
// ln T = ln(2 T_HI) - ln lambda: under half the transcendental work of one
// pow per power.  With CASE_A also alpha_A (Hui & Gnedin 1997 case-A fit,
// 1.269e-13 lambda^1.503 / (1 + (lambda/0.522)^0.470)^1.923).
constexpr double kLn2THI = 12.662275226919286;   // ln(2 T_HI)
constexpr double kInvLn10 = 0.43429448190325176;

template <bool CASE_A = false>
__device__ HRates h_rates(double T, double* alpha_a = nullptr)
{
    HRates r;
    const double lam = 2.0 * kTHI / T;
    const double L = log(lam);
    const double lnT = kLn2THI - L;
    r.alpha = 2.753e-14 * exp(1.5 * L - 2.242 * log1p(exp(0.407 * (L - 1.007957920399979))));
    r.coll = 21.11 * exp(-1.5 * lnT - 0.5 * lam - 1.089 * L - 1.101 * log1p(exp(0.874 * (L + 1.0384583658483626))));
    r.rec = 3.435e-30 * T * exp(1.970 * L - 3.720 * log1p(exp(0.376 * (L - 0.8109302162163288))));
    r.ci = kBoltz * kTHI * r.coll;
    const double sT = sqrt(T);
    r.ce = 7.5e-19 * exp(-118348.0 / T) / (1.0 + sT * 3.1622776601683795e-3);
    const double g = 5.5 - lnT * kInvLn10;
    r.ff = 1.42e-27 * (1.1 + 0.34 * exp(-g * g / 3.0)) * sT;
    if constexpr (CASE_A) *alpha_a = 1.269e-13 * exp(1.503 * L - 1.923 * log1p(exp(0.470 * (L + 0.6500876910994983))));
    return r;
}

// Photo-heating minus cooling (erg/cm^3/s) of a cell at T with n_H and
// neutral fraction x; `heat` is the photo-heating rate.
__device__ double net_gain(const FrtSolveDesc& D, double T, double nH, double x, double heat)
{
    const HRates r = h_rates(T);
    const double ne = nH * (1.0 - x), nHI = nH * x;
    double cool = (r.rec + r.ff) * ne * ne + (r.ci + r.ce) * ne * nHI;
    if (D.cmb_z >= 0.0) {
        const double z1 = 1.0 + D.cmb_z, z4 = z1 * z1 * z1 * z1;
        cool += kCompton0 * z4 * (T - 2.725 * z1) * ne;
    }
    return heat - cool;
}

// dT/dt = rate(T) over dt in sub-steps that change T by at most a tenth,
// each solving the equation linearized about its start exactly (the slope
// from a relative step of 1e-6 in T); at most 4096 sub-steps, T >= 1 K.
template <typename F>
__device__ __forceinline__ double substep_temperature(double T, double dt, F&& rate)
{
    double t = 0.0;
    for (int k = 0; k < 4096 && t < dt; k++) {
        const double f = rate(T);
        const double Tp = T * (1.0 + 1e-6);
        const double slope = (rate(Tp) - f) / (Tp - T);
        double h = dt - t;
        if (fabs(f) * h > 0.1 * T) h = 0.1 * T / fabs(f);
        const double y = slope * h;
        T = T + ((fabs(y) > 1e-8) ? f * expm1(y) / slope : f * h);
        if (T < 1.0) T = 1.0;
        t += h;
    }
    return T;
}

// T at the end of a step in which x went from x0 to x1 (n_tot = n_H (2 - x)):
// n_tot T kept over the change of particle number, e^(-2 H dt) for the
// Hubble term, then dT/dt = 2 (heat - cool) / (3 k n_tot) at x1 over dt.
__device__ double evolve_temperature(const FrtSolveDesc& D, double T, double nH, double x0, double x1, double heat)
{
    const double n0 = nH * (2.0 - x0), n1 = nH * (2.0 - x1);
    if (n1 > 0.0) T = T * (n0 / n1);
    if (D.hubble > 0.0) T = T * exp(-2.0 * D.hubble * D.dt);
    if (!(n1 > 0.0)) return T;
    const double c = 2.0 / (3.0 * kBoltz * n1);
    return substep_temperature(T, D.dt, [&](double Tv) { return c * net_gain(D, Tv, nH, x1, heat); });
}

// Generalized Opacity Mode (§4.2): dT/dt of a cell's ionized part at T, K/s,
// with n_HI from photo-ionization equilibrium with its rate G: y = n_HI /
// n_H = min(1, alpha_B(T) n_H / G) (1 where G = 0), n_e = n_HII = n_H (1 - y);
// photo-heating heat_rec alpha_A(T) n_e n_HII (Eq. analytical_heating_HI)
// minus the cooling of Standard Mode, over 3/2 k n_tot, n_tot = n_H (2 - y).
__device__ double ionized_dTdt(const FrtSolveDesc& D, double T, double nH, double G)
{
    double aA;
    const HRates r = h_rates<true>(T, &aA);
    const double y = G > r.alpha * nH ? r.alpha * nH / G : 1.0;
    const double ne = nH * (1.0 - y), nHI = nH * y;
    double gain = D.heat_rec * aA * ne * ne - (r.rec + r.ff) * ne * ne - (r.ci + r.ce) * ne * nHI;
    if (D.cmb_z >= 0.0) {
        const double z1 = 1.0 + D.cmb_z, z4 = z1 * z1 * z1 * z1;
        gain -= kCompton0 * z4 * (T - 2.725 * z1) * ne;
    }
    return 2.0 * gain / (3.0 * kBoltz * nH * (2.0 - y));
}

// A cell's temperature at the end of a step in which its ionized fraction
// went from xi0 to xi1 (Generalized Opacity Mode): the part ionized before
// the step cools by e^(-2 H dt) and then follows ionized_dTdt with the
// step's rate G; the part the front ionized during the step enters at
// T_reion; the two mix by volume (ionized gas of one n_H: by particle number
// too).  A cell with no ionized gas keeps its temperature.
__device__ double front_cell_temperature(const FrtSolveDesc& D, double T, double nH, double G, double xi0, double xi1)
{
    double Ti = T;
    if (xi0 > 0.0) {
        if (D.hubble > 0.0) Ti = Ti * exp(-2.0 * D.hubble * D.dt);
        if (nH > 0.0) Ti = substep_temperature(Ti, D.dt, [&](double Tv) { return ionized_dTdt(D, Tv, nH, G); });
    }
    if (xi1 > xi0) return (xi0 * Ti + (xi1 - xi0) * D.t_reion) / xi1;
    return Ti;
}

// The step's photo-heating rate of cell i (erg/cm^3/s) that the march
// deposited, which it clears.
template <typename Real>
__device__ __forceinline__ double take_heat(const FrtSolveDesc& D, size_t i)
{
    Real* hp = (Real*)D.heat;
    const double h = (double)hp[i];
    hp[i] = Real(0);
    return h;
}

// The ionized fraction as staged for the march (Generalized Opacity Mode): a
// cell not fully ionized in FP64 stays below 1 in FP32 too, so that the
// march stops packets at its front exactly when the FP64 state has one.
template <typename Real>
__device__ __forceinline__ Real staged_ionized_fraction(double xi)
{
    Real v = (Real)xi;
    if (xi < 1.0 && !(v < Real(1))) v = Real(1) - Real(0.5) * std::numeric_limits<Real>::epsilon();
    return v;
}

// Moving screen (§4.2, Eq. dxidt) of one cell at the end of a step: each
// photon stopped at the cell's front ionizes 1 + chi atoms; x_ion is at
// most 1 and never decreases; x = 1 - x_ion is the neutral volume fraction.
// Photons beyond the atoms the cell had left ionize nothing: they move from
// the ledger's absorbed_front to front_excess.  Clears the front count.  With
// the temperature on, the cell's T follows (front_cell_temperature, with G
// the step's rate of the ionized gas).
template <typename Real, bool TEMP>
__device__ __forceinline__ void moving_screen(const FrtSolveDesc& D, size_t i, double G)
{
    const double atoms = D.front_atoms * D.nH[i];
    const double f = D.front[i];
    const double xion = 1.0 - D.x[i];
    double xi = 1.0, excess = 0.0;
    if (atoms > 0.0) {
        xi = xion + f / atoms;
        if (xi > 1.0) {
            const double left = (1.0 - xion) * atoms;
            excess = f > left ? f - left : 0.0;
            xi = 1.0;
        }
    } else {
        excess = f;   // no hydrogen: nothing to ionize
    }
    if (excess > 0.0) {
        atomicAdd(&D.L->front_excess, excess);
        atomicAdd(&D.L->absorbed_front, -excess);
    }
    D.x[i] = 1.0 - xi;
    ((Real*)D.op_bw)[i] = staged_ionized_fraction<Real>(xi);
    D.front[i] = 0.0;
    if (TEMP && D.temp) D.T[i] = front_cell_temperature(D, D.T[i], D.nH[i], G, xion, xi);
}

// Every cell of every solve of a launch, one per thread, in chunks of
// blockDim.x consecutive cells.  A chunk inside one solve (nearly all of
// them) finds that solve once and reads its descriptor with uniform scalar
// loads; a chunk across two solves finds each cell's solve by a binary
// search over the per-solve cell prefix (in LDS).  f(D, i) gets the solve
// and the cell index within it.
template <typename F>
__device__ __forceinline__ void for_each_cell(const FrtSolveDesc* __restrict__ descs, const unsigned long long* spre,
                                             int n_solves, unsigned long long total, F&& f)
{
    auto solve_of = [&](unsigned long long g) {
        int lo = 0, hi = n_solves - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (spre[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long base = (unsigned long long)blockIdx.x * blockDim.x; base < total; base += stride) {
        const unsigned long long g = base + threadIdx.x;
        const int s0 = uni(solve_of(base));
        if (base + blockDim.x <= spre[s0 + 1]) {
            f(descs[s0], (size_t)(g - spre[s0]));
        } else if (g < total) {
            const int s = solve_of(g);
            f(descs[s], (size_t)(g - spre[s]));
        }
    }
}

// Backward Euler for x = n_HI / n_H, pure H, n_e = n_HII = n_H (1 - x):
//   x' - x = dt [ -Gamma x' - C n_H (1-x') x' + alpha n_H (1-x')^2 ]
// (Eq. ion_balance_eqn), i.e. a x'^2 + b x' + c = 0 with the root in [0,1]
// taken as 2c / (-b + sqrt(b^2 - 4ac)).  Also rebuilds the opacity of the
// next step (in place) and clears the next step's deposit buffer.  A launch
// in which any solve's queues overflowed leaves every solve's state
// untouched: the whole launch is run again from the start of the step.
template <typename Real, bool TEMP>
__global__ void __launch_bounds__(BLOCK) k_chem(const FrtSolveDesc* __restrict__ descs, const unsigned long long* prefix,
                                                int n_solves, unsigned long long total, const uint32_t* launch_err)
{
    __shared__ unsigned long long spre[FRT_MAX_SOLVES_PER_LAUNCH + 1];
    if (*launch_err) return;
    for (int i = threadIdx.x; i <= n_solves; i += blockDim.x) spre[i] = prefix[i];
    __syncthreads();
    for_each_cell(descs, spre, n_solves, total, [&](const FrtSolveDesc& D, size_t i) {
        if (D.L->err_flags) return;
        Real* gcur = (Real*)D.gamma[D.step & 1u];
        Real* gnext = (Real*)D.gamma[(D.step + 1u) & 1u];
        if (D.gen) {
            moving_screen<Real, TEMP>(D, i, (double)gcur[i]);
            gnext[i] = Real(0);
            return;
        }
        const double G = (double)gcur[i];
        const double nH = D.nH[i];
        const double x = D.x[i];
        const double dt = D.dt;
        // recombination and collisional ionization at the step's starting
        // temperature when it evolves
        double alpha = D.alpha_B, coll = D.coll_ion;
        if (TEMP && D.temp) {
            const HRates r = h_rates(D.T[i]);
            alpha = r.alpha;
            coll = r.coll;
        }
        const double a = dt * nH * (alpha + coll);
        const double bq = -(1.0 + dt * (G + 2.0 * alpha * nH + coll * nH));
        const double cq = x + alpha * nH * dt;
        double disc = bq * bq - 4.0 * a * cq;
        disc = disc > 0.0 ? disc : 0.0;
        const double xn = 2.0 * cq / (-bq + sqrt(disc));
        D.x[i] = xn;
        ((Real*)D.op_aw)[i] = hi_opacity<Real>(nH * xn * D.sigma0 * D.dx_cm);
        gnext[i] = Real(0);
        if (TEMP && D.temp) D.T[i] = evolve_temperature(D, D.T[i], nH, x, xn, take_heat<Real>(D, i));
    });
}

// Time-averaged hydrogen update (§4.1, Eqs. xi_of_t, xeq, ti, avg_xi) for
// x = n_HI / n_H, which follows the same linear equation as x_i once n_e is
// held fixed over the step: dx/dt = alpha n_e (1 - x) - (Gamma + C n_e) x.
// With R = Gamma + C n_e + alpha n_e, x_eq = alpha n_e / R and y = R dt:
//   x(dt) = x_eq + (x0 - x_eq) e^-y,   <x> = x_eq + (x0 - x_eq) (1 - e^-y) / y.
// phase 0, before the first march: <x> = x0 and the opacity from x0;
// phase 1, between marches: <x> from this march's Gamma and n_e = n_H (1 - <x>)
//   of the previous estimate; the next march sees n_HI = n_H <x> (Eq.
//   gamma_updated_standard) and starts from a cleared deposit buffer;
// phase 2, after the last march: x = x(dt), the next step's opacity from it
//   and its deposit buffer cleared.
// A launch in which any solve's queues overflowed leaves every solve's state
// untouched (phases 1 and 2 do nothing); phase 0 starts every run of the
// step, the first and any re-run, from the state the step began with.
template <typename Real, bool TEMP>
__global__ void __launch_bounds__(BLOCK) k_chem_avg(const FrtSolveDesc* __restrict__ descs, const unsigned long long* prefix,
                                                    int n_solves, unsigned long long total, int phase,
                                                    const uint32_t* launch_err, const uint32_t* halt)
{
    __shared__ unsigned long long spre[FRT_MAX_SOLVES_PER_LAUNCH + 1];
    if ((halt && *halt) || (phase != 0 && *launch_err)) return;
    for (int i = threadIdx.x; i <= n_solves; i += blockDim.x) spre[i] = prefix[i];
    __syncthreads();
    for_each_cell(descs, spre, n_solves, total, [&](const FrtSolveDesc& D, size_t i) {
        if (D.L->err_flags) return;
        if (D.gen) {
            Real* gcur = (Real*)D.gamma[D.step & 1u];
            if (phase == 2) {
                moving_screen<Real, TEMP>(D, i, (double)gcur[i]);
                ((Real*)D.gamma[(D.step + 1u) & 1u])[i] = Real(0);
                return;
            }
            // the opacity iteration of the Generalized Opacity Mode: the
            // ionized gas's kappa dx for the next march is the input plus
            // sigma_0 dx n_HI of photo-ionization equilibrium (§5.1, Eqs.
            // subgrid_lambda and subgrid_nHI) with the last rate, the
            // previous step's before the first march; where no rate is
            // known the optically thin guess (n_HI = 0); alpha_B at the
            // step's starting temperature when it evolves
            const double g = (double)((const Real*)D.gamma[phase == 0 ? (D.step + 1u) & 1u : D.step & 1u])[i];
            const double nH = D.nH[i];
            const double ab = (TEMP && D.temp) ? h_rates(D.T[i]).alpha : D.alpha_B;
            double nhi = 0.0;
            if (g > 0.0) nhi = (ab * nH * nH < g * nH) ? ab * nH * nH / g : nH;
            ((Real*)D.op_aw)[i] = hi_opacity<Real>((double)((const Real*)D.kin)[i] + D.sigma0 * nhi * D.dx_cm);
            if (phase == 1) {
                gcur[i] = Real(0);
                D.front[i] = 0.0;
            }
            return;
        }
        const double nH = D.nH[i];
        const double x0 = D.x[i];
        double xo;   // the neutral fraction the opacity is built from
        if (phase == 0) {
            D.xavg[i] = x0;
            xo = x0;
        } else {
            Real* gcur = (Real*)D.gamma[D.step & 1u];
            const double G = (double)gcur[i];
            const double ne = nH * (1.0 - D.xavg[i]);
            double alpha = D.alpha_B, coll = D.coll_ion;
            if (TEMP && D.temp) {
                // the rates of the step's starting temperature, for every march
                const HRates r = h_rates(D.T[i]);
                alpha = r.alpha;
                coll = r.coll;
            }
            const double R = G + coll * ne + alpha * ne;
            const double y = R * D.dt;
            double xa = x0, xe = x0;
            if (y > 0.0) {
                const double xeq = alpha * ne / R;
                xe = xeq + (x0 - xeq) * exp(-y);
                xa = xeq + (x0 - xeq) * (-expm1(-y) / y);
            }
            if (phase == 1) {
                D.xavg[i] = xa;
                gcur[i] = Real(0);
                // only the last march's photo-heating counts, like its rate
                if (TEMP && D.temp) ((Real*)D.heat)[i] = Real(0);
                xo = xa;
            } else {
                D.x[i] = xe;
                ((Real*)D.gamma[(D.step + 1u) & 1u])[i] = Real(0);
                if (TEMP && D.temp) D.T[i] = evolve_temperature(D, D.T[i], nH, x0, xe, take_heat<Real>(D, i));
                xo = xe;
            }
        }
        ((Real*)D.op_aw)[i] = hi_opacity<Real>(nH * xo * D.sigma0 * D.dx_cm);
    });
}

// The ledger and carried-queue counters of every solve as a step starts, kept
// for a re-run of the step (queue growth) and for the later marches of the
// time-averaged chemistry.  One workgroup per solve.
__global__ void __launch_bounds__(BLOCK) k_snapshot(FrtSolveDesc* descs, const uint32_t* halt)
{
    if (halt && *halt) return;
    const FrtSolveDesc& D = descs[blockIdx.x];
    constexpr int NW = (int)(sizeof(FrtLedgerDev) / sizeof(unsigned long long));
    const unsigned long long* src = (const unsigned long long*)D.L;
    unsigned long long* dst = (unsigned long long*)D.L_snap;
    for (int k = threadIdx.x; k < NW; k += blockDim.x) dst[k] = src[k];
    if (threadIdx.x < 2) D.fcount_snap[threadIdx.x] = D.fcount[threadIdx.x];
}

// Every march of a step after the first starts from the step's packets: the
// ledger and the carried-queue counters go back to their values at the
// start of the step, keeping the device error bits.  One workgroup per solve.
__global__ void __launch_bounds__(BLOCK) k_iter_restart(FrtSolveDesc* descs, const uint32_t* halt)
{
    if (halt && *halt) return;
    const FrtSolveDesc& D = descs[blockIdx.x];
    __shared__ uint32_t s_err;
    if (threadIdx.x == 0) s_err = D.L->err_flags;
    __syncthreads();
    constexpr int NW = (int)(sizeof(FrtLedgerDev) / sizeof(unsigned long long));
    static_assert(sizeof(FrtLedgerDev) % sizeof(unsigned long long) == 0, "ledger copied as 8-byte words");
    const unsigned long long* src = (const unsigned long long*)D.L_snap;
    unsigned long long* dst = (unsigned long long*)D.L;
    for (int k = threadIdx.x; k < NW; k += blockDim.x) dst[k] = src[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        D.L->err_flags |= s_err;
        D.fcount[0] = D.fcount_snap[0];
        D.fcount[1] = D.fcount_snap[1];
    }
}

// Opacity from the loaded state: {n_H x sigma_0 dx, kappa dx} (kappa dx is
// written by the host beforehand into .y); in the Generalized Opacity Mode
// {kappa dx (written by the host), 1 - x}.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_prep(const FrtSolveDesc* __restrict__ desc, unsigned long long n)
{
    const FrtSolveDesc& D = *desc;
    Real* op = (Real*)D.op_aw;
    Real* ob = (Real*)D.op_bw;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        if (D.gen) ob[i] = staged_ionized_fraction<Real>(1.0 - D.x[i]);   // .x is kappa dx, set by the host
        else op[i] = hi_opacity<Real>(D.nH[i] * D.x[i] * D.sigma0 * D.dx_cm);
    }
}

// A new hydrogen density between steps: with the temperature on, the
// compression term of Eq. temp_evolution_standard, whose solution along any
// path keeps T Delta^(-2/3), Delta = n_H / <n_H> (m0, m1: the grid's mean
// before and after): T -> T (Delta_new / Delta_old)^(2/3), where both
// densities are > 0.  The staged opacity is rebuilt afterwards (k_prep).
__global__ void __launch_bounds__(BLOCK) k_set_density(double* __restrict__ nH, const double* __restrict__ nH_new,
                                                      double* __restrict__ T, double m0, double m1, unsigned long long n)
{
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        const double n0 = nH[i], n1 = nH_new[i];
        if (T && n0 > 0.0 && n1 > 0.0) T[i] = T[i] * pow((n1 / m1) / (n0 / m0), 2.0 / 3.0);
        nH[i] = n1;
    }
}

// The allocation-free step's scratch (FRT_STATIC_SCRATCH_BYTES per GPU).  In
// host code `scratch` names a host-side stand-in, not device memory: host code
// uses the device address that static_scratch() looks up, never the name.
static __device__ __align__(256) unsigned char scratch[FRT_STATIC_SCRATCH_BYTES];

// Compute units of the current device, queried once (the server's loader
// threads may ask for it at the same time: a function-local static is
// initialized exactly once)
int cu_count()
{
    static const int n = [] {
        int dev = 0, c = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        return c > 0 ? c : 256;
    }();
    return n;
}

int grid_for(unsigned long long items, int per_cu)
{
    unsigned long long want = (items + BLOCK - 1) / BLOCK;
    unsigned long long cap = (unsigned long long)cu_count() * per_cu;
    if (want < 1) want = 1;
    return (int)(want < cap ? want : cap);
}

template <typename Real, int NB>
void launch_seed_nb(FrtSolveDesc* d, const FrtWS& ws, hipStream_t s)
{
    hipLaunchKernelGGL((k_seed<Real, NB>), dim3(cu_count() * 4), dim3(BLOCK), 0, s, d, ws);
}

// Resident workgroups per CU of a kernel (at least 1), queried once per
// kernel.
int blocks_per_cu(void (*kernel)(const FrtSolveDesc*, FrtWS), int threads)
{
    static std::mutex mu;
    static std::unordered_map<const void*, int> known;
    std::lock_guard<std::mutex> lock(mu);
    const auto it = known.find((const void*)kernel);
    if (it != known.end()) return it->second;
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, threads, 0) != hipSuccess || b < 1) b = 1;
    known[(const void*)kernel] = b;
    return b;
}

// The march kernel of a launch, its workgroup size and its grid (resident
// workgroups on every CU; the occupancy query runs on the first call).
struct BrickLaunch {
    void (*kernel)(const FrtSolveDesc*, FrtWS);
    int threads, per_cu;
};

template <typename Real, int NB>
BrickLaunch brick_kernel(const FrtWS& ws)
{
    BrickLaunch b;
    if (ws.has_heat) {
        // temperature evolution: the solves of such a launch use the
        // sub-grid layout
        b.kernel = k_brick<Real, NB, true, true>;
        b.threads = BLOCK;
    } else if constexpr (sizeof(Real) == 4) {
        if (!ws.has_sub) {
            b.kernel = k_brick_big<Real, NB>;
            b.threads = 4 * BLOCK;
        } else {
            b.kernel = k_brick<Real, NB, true>;
            b.threads = BLOCK;
        }
    } else {
        b.kernel = ws.has_sub ? k_brick<Real, NB, true> : k_brick<Real, NB, false>;
        b.threads = BLOCK;
    }
    b.per_cu = blocks_per_cu(b.kernel, b.threads);
    return b;
}

template <typename Real, int NB>
void launch_pass_nb(FrtSolveDesc* d, const FrtWS& ws, int part, hipStream_t s)
{
    const BrickLaunch bk = brick_kernel<Real, NB>(ws);
    const dim3 grid(cu_count() * bk.per_cu);
    if (part == 0) hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, ws);
    else if (part == 1) hipLaunchKernelGGL(k_scatter, dim3(cu_count() * ws.scatter_bpc), dim3(BLOCK), 0, s, ws);
    else if (part == 2) hipLaunchKernelGGL(bk.kernel, grid, dim3(bk.threads), 0, s, d, ws);
}

template <typename Real>
hipError_t seed_t(FrtSolveDesc* d, const FrtWS& ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_seed_plan, dim3(1), dim3(64), 0, s, d, ws);
    switch (ws.n_bins) {
        case 1: launch_seed_nb<Real, 1>(d, ws, s); break;
        case 2: launch_seed_nb<Real, 2>(d, ws, s); break;
        case 3: launch_seed_nb<Real, 3>(d, ws, s); break;
        case 4: launch_seed_nb<Real, 4>(d, ws, s); break;
        case 5: launch_seed_nb<Real, 5>(d, ws, s); break;
        case 6: launch_seed_nb<Real, 6>(d, ws, s); break;
        case 7: launch_seed_nb<Real, 7>(d, ws, s); break;
        case 8: launch_seed_nb<Real, 8>(d, ws, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename Real>
hipError_t pass_t(FrtSolveDesc* d, const FrtWS& ws, int part, hipStream_t s)
{
    switch (ws.n_bins) {
        case 1: launch_pass_nb<Real, 1>(d, ws, part, s); break;
        case 2: launch_pass_nb<Real, 2>(d, ws, part, s); break;
        case 3: launch_pass_nb<Real, 3>(d, ws, part, s); break;
        case 4: launch_pass_nb<Real, 4>(d, ws, part, s); break;
        case 5: launch_pass_nb<Real, 5>(d, ws, part, s); break;
        case 6: launch_pass_nb<Real, 6>(d, ws, part, s); break;
        case 7: launch_pass_nb<Real, 7>(d, ws, part, s); break;
        case 8: launch_pass_nb<Real, 8>(d, ws, part, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

namespace frt {

int device_cu_count() { return cu_count(); }

hipError_t static_scratch(int device, void** ptr)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* addr[MAX_DEVICES] = {};
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_seed(FrtSolveDesc* d, const FrtWS& ws, int fp64, hipStream_t s)
{
    return fp64 ? seed_t<double>(d, ws, s) : seed_t<float>(d, ws, s);
}

hipError_t launch_pass(FrtSolveDesc* d, const FrtWS& ws, int fp64, int part, hipStream_t s)
{
    return fp64 ? pass_t<double>(d, ws, part, s) : pass_t<float>(d, ws, part, s);
}

hipError_t launch_finish(FrtSolveDesc* d, const FrtWS& ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish, dim3(ws.n_solves < 1024 ? ws.n_solves : 1024), dim3(64), 0, s, d, ws);
    return hipGetLastError();
}

hipError_t launch_chem(FrtSolveDesc* d, const unsigned long long* d_cell_prefix, int n_solves,
                       unsigned long long total_cells, int fp64, int temp, const uint32_t* launch_err, hipStream_t s)
{
    if (total_cells == 0) return hipSuccess;
    const int grid = grid_for(total_cells, 16);
    auto kern = fp64 ? (temp ? k_chem<double, true> : k_chem<double, false>) : (temp ? k_chem<float, true> : k_chem<float, false>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), 0, s, d, d_cell_prefix, n_solves, total_cells, launch_err);
    return hipGetLastError();
}

hipError_t launch_clear(const FrtWS& ws, int mode, hipStream_t s)
{
    const uint32_t n = ws.nkeys > C_NCTR ? ws.nkeys : C_NCTR;
    hipLaunchKernelGGL(k_clear, dim3(grid_for(n, 4)), dim3(BLOCK), 0, s, ws, mode);
    return hipGetLastError();
}

hipError_t launch_chem_avg(FrtSolveDesc* d, const unsigned long long* d_cell_prefix, int n_solves,
                           unsigned long long total_cells, int fp64, int temp, int phase, const uint32_t* launch_err,
                           const uint32_t* halt, hipStream_t s)
{
    if (total_cells == 0) return hipSuccess;
    const int grid = grid_for(total_cells, 16);
    auto kern = fp64 ? (temp ? k_chem_avg<double, true> : k_chem_avg<double, false>)
                     : (temp ? k_chem_avg<float, true> : k_chem_avg<float, false>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), 0, s, d, d_cell_prefix, n_solves, total_cells, phase, launch_err, halt);
    return hipGetLastError();
}

hipError_t launch_snapshot(FrtSolveDesc* d, int n_solves, const uint32_t* halt, hipStream_t s)
{
    hipLaunchKernelGGL(k_snapshot, dim3(n_solves), dim3(BLOCK), 0, s, d, halt);
    return hipGetLastError();
}

hipError_t launch_iter_restart(FrtSolveDesc* d, int n_solves, const uint32_t* halt, hipStream_t s)
{
    hipLaunchKernelGGL(k_iter_restart, dim3(n_solves), dim3(BLOCK), 0, s, d, halt);
    return hipGetLastError();
}

hipError_t launch_advance(FrtSolveDesc* d, const FrtWS& ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, d, ws);
    return hipGetLastError();
}

void prime_launch_shapes(int fp64, int n_bins, int has_sub, int has_heat)
{
    (void)cu_count();
    FrtWS w{};
    w.n_bins = n_bins;
    w.has_sub = has_sub;
    w.has_heat = has_heat;
    auto prime = [&](auto tag) {
        using Real = decltype(tag);
        switch (n_bins) {
            case 1: brick_kernel<Real, 1>(w); break;
            case 2: brick_kernel<Real, 2>(w); break;
            case 3: brick_kernel<Real, 3>(w); break;
            case 4: brick_kernel<Real, 4>(w); break;
            case 5: brick_kernel<Real, 5>(w); break;
            case 6: brick_kernel<Real, 6>(w); break;
            case 7: brick_kernel<Real, 7>(w); break;
            case 8: brick_kernel<Real, 8>(w); break;
            default: break;
        }
    };
    if (fp64) prime(double{});
    else prime(float{});
}

hipError_t launch_prep_opacity(FrtSolveDesc* d_desc, unsigned long long ncell, int fp64, hipStream_t s)
{
    if (ncell == 0) return hipSuccess;
    const int grid = grid_for(ncell, 16);
    if (fp64) hipLaunchKernelGGL(k_prep<double>, dim3(grid), dim3(BLOCK), 0, s, d_desc, ncell);
    else hipLaunchKernelGGL(k_prep<float>, dim3(grid), dim3(BLOCK), 0, s, d_desc, ncell);
    return hipGetLastError();
}

hipError_t launch_set_density(double* nH, const double* nH_new, double* T, double m0, double m1,
                              unsigned long long ncell, hipStream_t s)
{
    if (ncell == 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_density, dim3(grid_for(ncell, 16)), dim3(BLOCK), 0, s, nH, nH_new, T, m0, m1, ncell);
    return hipGetLastError();
}

}  // namespace frt
