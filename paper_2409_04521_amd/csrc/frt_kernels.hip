// HIP kernels for gfx950: casting, the per-round ray march, backward-Euler
// chemistry and step bookkeeping of adaptive ray tracing of ionizing photon
// packets (Cain & D'Aloisio, FlexRT I, §3 and §4.1).
//
// Work layout: one lane owns one packet for one "visit" (from where it
// starts this round until it splits, ends, or spends its travel budget).
// Each round is one grid-stride launch over the concatenated work items of
// every solve in the launch; item counts are read on the device.
#include "frt_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;

// ------------------------------------------------------------------ HEALPix
// Centre of NESTED pixel p at level l (Nside = 2^l), Gorski et al. 2005:
// the pixel index splits into base face f and in-face coordinates (ix, iy)
// (bits interleaved, ix in the even bits); the ring index counted from the
// north pole is j = jr(f) Nside - ix - iy - 1 and the pixel's longitude
// index within its ring is jp(f) nr + ix - iy, with nr the ring's
// half-width.  z follows from j on the polar caps (j < Nside, j > 3 Nside)
// and on the equatorial belt.
__device__ __forceinline__ uint32_t squeeze_even_bits(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

template <typename Real>
__device__ void nest_pixel_centre(int level, uint32_t pix, Real v[3])
{
    const int jr_face[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
    const int jp_face[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
    const int nside = 1 << level;
    const uint32_t face = pix >> (2 * level);
    const uint32_t sub = pix & ((1u << (2 * level)) - 1u);
    const int ix = (int)squeeze_even_bits(sub);
    const int iy = (int)squeeze_even_bits(sub >> 1);
    const int j = jr_face[face] * nside - ix - iy - 1;
    int nr;
    Real z, st;
    const Real inv3n2 = Real(1) / (Real(3) * Real(nside) * Real(nside));
    if (j < nside) {
        nr = j;
        Real t = Real(nr) * Real(nr) * inv3n2;   // 1 - z
        z = Real(1) - t;
        st = sqrt(t * (Real(2) - t));
    } else if (j > 3 * nside) {
        nr = 4 * nside - j;
        Real t = Real(nr) * Real(nr) * inv3n2;   // 1 + z
        z = t - Real(1);
        st = sqrt(t * (Real(2) - t));
    } else {
        nr = nside;
        z = Real(2 * nside - j) * (Real(2) / Real(3 * nside));
        st = sqrt((Real(1) - z) * (Real(1) + z));
    }
    int k = jp_face[face] * nr + ix - iy;
    if (k < 0) k += 8 * nr;
    else if (k >= 8 * nr) k -= 8 * nr;
    // phi = (pi/4) k / nr, evaluated as sincospi(k / (4 nr))
    Real s, c;
    if constexpr (sizeof(Real) == 8) sincospi(Real(k) / Real(4 * nr), &s, &c);
    else sincospif(Real(k) / Real(4 * nr), &s, &c);
    v[0] = st * c;
    v[1] = st * s;
    v[2] = z;
}

// ----------------------------------------------------------------- rotation
// Counter-based uniforms: SplitMix64 output function (Steele, Lea & Flood
// 2014) of (step<<32 | src<<2 | k) xor a key derived from the seed.
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double counter_uniform(uint64_t seed, uint32_t step, uint32_t src, uint32_t k)
{
    uint64_t ctr = ((uint64_t)step << 32) | ((uint64_t)src << 2) | (uint64_t)k;
    return (double)(mix64(ctr ^ mix64(seed)) >> 11) * 0x1.0p-53;
}

// Uniform random rotation as a unit quaternion (w, x, y, z) from three
// uniforms (Shoemake 1992).
__device__ void shoemake_quat(const double u[3], double q[4])
{
    double a = sqrt(1.0 - u[0]), b = sqrt(u[0]);
    double s2, c2, s3, c3;
    sincospi(2.0 * u[1], &s2, &c2);
    sincospi(2.0 * u[2], &s3, &c3);
    q[0] = b * c3;
    q[1] = a * s2;
    q[2] = a * c2;
    q[3] = b * s3;
}

// v' = q v q*, written with the vector part u of q:  t = 2 u x v,
// v' = v + w t + u x t.
template <typename Real>
__device__ __forceinline__ void quat_rotate(const double* qd, Real v[3])
{
    const Real w = (Real)qd[0], ux = (Real)qd[1], uy = (Real)qd[2], uz = (Real)qd[3];
    Real tx = Real(2) * (uy * v[2] - uz * v[1]);
    Real ty = Real(2) * (uz * v[0] - ux * v[2]);
    Real tz = Real(2) * (ux * v[1] - uy * v[0]);
    Real ox = v[0] + w * tx + (uy * tz - uz * ty);
    Real oy = v[1] + w * ty + (uz * tx - ux * tz);
    Real oz = v[2] + w * tz + (ux * ty - uy * tx);
    v[0] = ox; v[1] = oy; v[2] = oz;
}

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
__device__ __forceinline__ void ledger_add(double* target, double v, bool uniform)
{
    if (uniform) {
        double s = wave_sum(v);
        if ((threadIdx.x & (WAVE - 1)) == 0 && s != 0.0) atomicAdd(target, s);
    } else if (v != 0.0) {
        atomicAdd(target, v);
    }
}

__device__ __forceinline__ void ledger_add_u64(unsigned long long* target, unsigned long long v, bool uniform)
{
    if (uniform) {
        unsigned long long s = wave_sum_u64(v);
        if ((threadIdx.x & (WAVE - 1)) == 0 && s != 0) atomicAdd(target, s);
    } else if (v != 0) {
        atomicAdd(target, v);
    }
}

__device__ __forceinline__ int find_solve(const uint32_t* prefix, int n, uint32_t g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename Real> __device__ __forceinline__ Real rinf();
template <> __device__ __forceinline__ float rinf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double rinf<double>() { return __builtin_huge_val(); }

__device__ __forceinline__ float rexp(float x) { return expf(x); }
__device__ __forceinline__ double rexp(double x) { return exp(x); }
__device__ __forceinline__ float rexpm1(float x) { return expm1f(x); }
__device__ __forceinline__ double rexpm1(double x) { return expm1(x); }

template <typename Real> struct Vec2;
template <> struct Vec2<float> { using T = float2; };
template <> struct Vec2<double> { using T = double2; };

// ------------------------------------------------------------ record access
template <typename Real>
struct Rec {
    uint32_t src, estep, lp;
    Real r, rstop, w0;
};

template <typename Real>
__device__ __forceinline__ void push_record(const FrtQueue& q, uint32_t i, int nb, const Rec<Real>& h,
                                            const Real* tau, const Real* comp)
{
    q.src[i] = h.src;
    q.estep[i] = h.estep;
    q.lp[i] = h.lp;
    ((Real*)q.r)[i] = h.r;
    ((Real*)q.rstop)[i] = h.rstop;
    ((Real*)q.w0)[i] = h.w0;
    for (int b = 0; b < nb; b++) {
        ((Real*)q.tau)[(size_t)b * q.cap + i] = tau[b];
        ((Real*)q.comp)[(size_t)b * q.cap + i] = comp[b];
    }
}

// ==================================================================== emit
// One lane per (source, base pixel): append a packet with r = 0 and the
// photons Ndot_nu dt / (12 4^L0) per bin (§3.1, Eq. Nray), and make this
// step's rotation of the source's sphere.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_emit(FrtSolveDesc* descs, const uint32_t* prefix, int n_solves,
                                                uint32_t total)
{
    __shared__ uint32_t spre[FRT_MAX_SOLVES_PER_LAUNCH + 1];
    for (int i = threadIdx.x; i <= n_solves; i += blockDim.x) spre[i] = prefix[i];
    __syncthreads();
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < total; base += stride) {
        const uint32_t g = base + threadIdx.x;
        const bool active = g < total;
        int si = active ? find_solve(spre, n_solves, g) : 0;
        const bool uniform = __all(__shfl(si, 0, WAVE) == si);
        FrtSolveDesc& D = descs[si];
        double photons = 0.0;
        if (active) {
            const uint32_t local = g - spre[si];
            const uint32_t ncast = 12u << (2 * D.base_level);
            const uint32_t src = local / ncast, pix = local % ncast;
            if (pix == 0) {
                double u[3];
                for (int k = 0; k < 3; k++)
                    u[k] = (D.step < D.user_steps) ? D.user_u[((size_t)D.step * D.n_src + src) * 3 + k]
                                                   : counter_uniform(D.seed, D.step, src, k);
                double q[4];
                shoemake_quat(u, q);
                double* dst = D.quat + ((size_t)D.step * D.n_src + src) * 4;
                for (int k = 0; k < 4; k++) dst[k] = q[k];
            }
            Rec<Real> h;
            h.src = src;
            h.estep = D.step;
            h.lp = ((uint32_t)D.base_level << 28) | pix;
            h.r = Real(0);
            h.rstop = Real(0);
            h.w0 = (Real)D.w0_cast;
            Real zero[FRT_MAX_BINS_I] = {};
            for (int b = 0; b < D.n_bins; b++) {
                if constexpr (sizeof(Real) == 8) photons += h.w0 * D.specd[(size_t)src * D.n_bins + b];
                else photons += (double)(h.w0 * D.spec[(size_t)src * D.n_bins + b]);
            }
            const FrtQueue& q = D.q[D.cur];
            uint32_t at = atomicAdd(&D.count[D.cur], 1u);
            if (at < q.cap) {
                push_record<Real>(q, at, D.n_bins, h, zero, zero);
            } else {
                atomicOr(&D.L->err_flags, (unsigned)FRT_DEVERR_QUEUE_OVERFLOW);
                atomicAdd(&D.L->lost, photons * D.R_ref);
            }
        }
        ledger_add(&D.L->emitted, photons * D.R_ref, uniform);
        ledger_add_u64(&D.L->rays_emitted, active ? 1ull : 0ull, uniform);
    }
}

// =============================================================== round plan
// Prefix of this round's work items over the solves, and clearing of the
// queues this round writes.
__global__ void k_plan(FrtSolveDesc* descs, FrtRoundPlan* plan, int n_solves, int round)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int in_split = FRT_QS0 + ((round + 1) & 1);   // split queue read by rounds >= 1
    const int out_split = FRT_QS0 + (round & 1);
    uint32_t acc = 0;
    for (int s = 0; s < n_solves; s++) {
        FrtSolveDesc& D = descs[s];
        plan->prefix[s] = acc;
        uint32_t n;
        if (round == 0) {
            D.L->step_crossings = 0;
            n = D.count[D.cur];
            if (n > D.q[D.cur].cap) n = D.q[D.cur].cap;
            D.count[1 - D.cur] = 0;     // packets carried into the next step
        } else {
            n = D.count[in_split];
            if (n > D.q[in_split].cap) n = D.q[in_split].cap;
            n *= 4u;
        }
        D.count[out_split] = 0;
        if (n > D.L->max_items) D.L->max_items = n;
        acc += n;
    }
    plan->prefix[n_solves] = acc;
    plan->n_solves = n_solves;
    plan->in_slot = round == 0 ? -1 : in_split;
    plan->out_slot = out_split;
    plan->expand = round == 0 ? 0 : 1;
}

// ==================================================================== march
// Per lane: load a packet (or one child of a split parent), then walk cells
// along src + r dir.  Per segment of length ds (cells) in cell i, per bin:
//   tau    = (s_nu a_i + b_i) ds,  a_i = n_HI sigma_0 dx, b_i = kappa dx
//   N_in   = N0 exp(-tau_sum)      (tau_sum carried with Kahan compensation)
//   Gamma_i += K_nu N_in ds phi(tau),  phi = (1 - e^-tau)/tau,
//   K_nu = R_ref sigma_nu / (dx^2 dt)
// which is Eq. gamma_avg_subgrid with lambda = 1/(n_HI sigma + kappa)
// (Eq. gamma_initial_standard when kappa = 0).  End states in order:
// distance cap, flux floor, split radius (Eq. r_split), leaving the box,
// travel budget.
template <typename Real, int NB, bool EXPAND>
__global__ void __launch_bounds__(BLOCK) k_march(FrtSolveDesc* descs, const FrtRoundPlan* plan)
{
    using R2 = typename Vec2<Real>::T;
    constexpr bool F32 = sizeof(Real) == 4;
    __shared__ uint32_t spre[FRT_MAX_SOLVES_PER_LAUNCH + 1];
    const int n_solves = plan->n_solves;
    for (int i = threadIdx.x; i <= n_solves; i += blockDim.x) spre[i] = plan->prefix[i];
    __syncthreads();
    const uint32_t total = spre[n_solves];
    const int in_slot = plan->in_slot, out_slot = plan->out_slot;
    const uint32_t stride = gridDim.x * blockDim.x;

    for (uint32_t base = blockIdx.x * blockDim.x; base < total; base += stride) {
        const uint32_t g = base + threadIdx.x;
        const bool active = g < total;
        const int si = active ? find_solve(spre, n_solves, g) : find_solve(spre, n_solves, total - 1);
        const bool uniform = __all(__shfl(si, 0, WAVE) == si);
        FrtSolveDesc& D = descs[si];
        double d_abs = 0.0, d_sub = 0.0, d_esc = 0.0, d_drop = 0.0, d_fl = 0.0;
        unsigned long long n_cross = 0, n_esc = 0, n_drop = 0, n_split = 0;
        if (active) {
            const uint32_t local = g - spre[si];
            const int slot = EXPAND ? in_slot : (int)D.cur;
            const FrtQueue& qi = D.q[slot];
            const uint32_t e = EXPAND ? (local >> 2) : local;
            Rec<Real> h;
            h.src = qi.src[e];
            h.estep = qi.estep[e];
            h.lp = qi.lp[e];
            h.r = ((const Real*)qi.r)[e];
            h.rstop = ((const Real*)qi.rstop)[e];
            h.w0 = ((const Real*)qi.w0)[e];
            Real tau[NB], comp[NB], E[NB], N0[NB];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                tau[b] = ((const Real*)qi.tau)[(size_t)b * qi.cap + e];
                comp[b] = ((const Real*)qi.comp)[(size_t)b * qi.cap + e];
            }
            int level = (int)(h.lp >> 28);
            uint32_t pix = h.lp & 0x0fffffffu;
            if (EXPAND) {
                level += 1;
                pix = 4u * pix + (local & 3u);
                h.lp = ((uint32_t)level << 28) | pix;
                h.w0 = h.w0 * Real(0.25);
            } else {
                h.rstop = h.r + (Real)D.budget;   // fresh travel budget each step
            }
            Real sum0 = 0, sumE = 0;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                Real spec;
                if constexpr (F32) spec = D.spec[(size_t)h.src * NB + b];
                else spec = D.specd[(size_t)h.src * NB + b];
                N0[b] = h.w0 * spec;
                E[b] = rexp(-tau[b]);
                sum0 += N0[b];
            }
            double n_start = 0.0;
#pragma unroll
            for (int b = 0; b < NB; b++) n_start += (double)(N0[b] * E[b]);

            // direction of (level, pix) on the source's rotated sphere
            Real d[3];
            nest_pixel_centre<Real>(level, pix, d);
            quat_rotate<Real>(D.quat + ((size_t)h.estep * D.n_src + h.src) * 4, d);
            const double* sp = D.src_pos + (size_t)h.src * 3;
            const Real s[3] = {(Real)sp[0], (Real)sp[1], (Real)sp[2]};
            const Real r_split = (level < D.max_level) ? (Real)(D.r_split0 * (double)(1u << level)) : rinf<Real>();
            const Real r_cap = (Real)D.r_cap;
            const int nx = D.nx, ny = D.ny, nz = D.nz;
            const int dims[3] = {nx, ny, nz};
            int c[3];
            Real rf[3];
            bool out = false;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                Real p = s[a] + h.r * d[a];
                Real f = floor(p);
                if (p == f && d[a] < Real(0)) f -= Real(1);
                c[a] = (int)f;
                out |= (c[a] < 0) || (c[a] >= dims[a]);
            }
            Real Kb[NB], srel[NB];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                srel[b] = (Real)D.sig_rel[b];
                if constexpr (F32) Kb[b] = D.K[b];
                else Kb[b] = D.Kd[b];
            }
            const R2* __restrict__ op = (const R2*)D.op;
            Real* __restrict__ gam = (Real*)D.gamma[D.step & 1u];
            // 0 = split, 1 = escaped, 2 = dropped, 3 = in flight
            int end = 1;
            float sub_acc = 0.f;
            double sub_acc_d = 0.0;
            if (!out) {
                Real inv[3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    inv[a] = (d[a] != Real(0)) ? Real(1) / d[a] : Real(0);
                    rf[a] = (d[a] != Real(0)) ? ((Real)(c[a] + (d[a] > Real(0) ? 1 : 0)) - s[a]) * inv[a]
                                              : rinf<Real>();
                }
                for (;;) {
                    int axis = 0;
                    Real r_face = rf[0];
                    if (rf[1] < r_face) { r_face = rf[1]; axis = 1; }
                    if (rf[2] < r_face) { r_face = rf[2]; axis = 2; }
                    Real r_end = r_face;
                    r_end = fmin(r_end, r_split);
                    r_end = fmin(r_end, r_cap);
                    r_end = fmin(r_end, h.rstop);
                    r_end = fmax(r_end, h.r);
                    const Real ds = r_end - h.r;
                    if (ds > Real(0)) {
                        const size_t ci = (size_t)c[0] + (size_t)nx * ((size_t)c[1] + (size_t)ny * (size_t)c[2]);
                        const R2 o = op[ci];
                        Real dep = 0;
#pragma unroll
                        for (int b = 0; b < NB; b++) {
                            const Real th = srel[b] * o.x * ds;
                            const Real tb = th + o.y * ds;
                            const Real nin = N0[b] * E[b];
                            Real absf, phi;
                            if (tb < Real(1e-4)) {
                                phi = Real(1) - Real(0.5) * tb;
                                absf = tb * phi;
                            } else {
                                absf = -rexpm1(-tb);
                                phi = absf / tb;
                            }
                            dep += Kb[b] * nin * ds * phi;
                            if (o.y > Real(0)) {
                                if constexpr (F32) sub_acc += nin * absf * ((o.y * ds) / tb);
                                else sub_acc_d += nin * absf * ((o.y * ds) / tb);
                            }
                            if constexpr (F32) {
                                // Kahan-compensated running optical depth
                                const Real y = tb - comp[b];
                                const Real t = tau[b] + y;
                                comp[b] = (t - tau[b]) - y;
                                tau[b] = t;
                            } else {
                                tau[b] += tb;
                            }
                            E[b] = rexp(-tau[b]);
                        }
                        if constexpr (F32) unsafeAtomicAdd(gam + ci, dep);
                        else unsafeAtomicAdd(gam + ci, dep);
                        n_cross++;
                    }
                    h.r = r_end;
                    if (h.r >= r_cap) { end = 2; break; }
                    if (D.floor > 0.f) {
                        sumE = 0;
#pragma unroll
                        for (int b = 0; b < NB; b++) sumE += N0[b] * E[b];
                        if (sumE < (Real)D.floor * sum0) { end = 2; break; }
                    }
                    if (h.r >= r_split) { end = 0; break; }
                    if (h.r >= r_face) {
                        c[axis] += (d[axis] > Real(0)) ? 1 : -1;
                        if (c[axis] < 0 || c[axis] >= dims[axis]) { end = 1; break; }
                        rf[axis] = ((Real)(c[axis] + (d[axis] > Real(0) ? 1 : 0)) - s[axis]) * inv[axis];
                    }
                    if (h.r >= h.rstop) { end = 3; break; }
                }
            }
            double n_end = 0.0;
#pragma unroll
            for (int b = 0; b < NB; b++) n_end += (double)(N0[b] * E[b]);
            const double Rr = D.R_ref;
            d_abs = (n_start - n_end) * Rr;
            d_sub = (F32 ? (double)sub_acc : sub_acc_d) * Rr;
            if (end == 1) { d_esc = n_end * Rr; n_esc = 1; }
            else if (end == 2) { d_drop = n_end * Rr; n_drop = 1; }
            else {
                const int qs = (end == 0) ? out_slot : (int)(1 - D.cur);
                const FrtQueue& qo = D.q[qs];
                uint32_t at = atomicAdd(&D.count[qs], 1u);
                if (at < qo.cap) {
                    push_record<Real>(qo, at, NB, h, tau, comp);
                    if (end == 0) n_split = 1;
                    else d_fl = n_end * Rr;
                } else {
                    atomicOr(&D.L->err_flags, (unsigned)FRT_DEVERR_QUEUE_OVERFLOW);
                    atomicAdd(&D.L->lost, n_end * Rr);
                }
            }
        }
        FrtLedgerDev* L = D.L;
        ledger_add(&L->absorbed_HI, d_abs - d_sub, uniform);
        ledger_add(&L->absorbed_sub, d_sub, uniform);
        ledger_add(&L->escaped, d_esc, uniform);
        ledger_add(&L->dropped, d_drop, uniform);
        ledger_add(&L->in_flight_acc, d_fl, uniform);
        ledger_add_u64(&L->crossings, n_cross, uniform);
        ledger_add_u64(&L->step_crossings, n_cross, uniform);
        ledger_add_u64(&L->ray_visits, active ? 1ull : 0ull, uniform);
        ledger_add_u64(&L->n_escaped, n_esc, uniform);
        ledger_add_u64(&L->n_dropped, n_drop, uniform);
        ledger_add_u64(&L->splits, n_split, uniform);
    }
}

// ================================================================ chemistry
// Backward Euler for x = n_HI / n_H, pure H, n_e = n_HII = n_H (1 - x):
//   x' - x = dt [ -Gamma x' - C n_H (1-x') x' + alpha n_H (1-x')^2 ]
// (Eq. ion_balance_eqn), i.e. a x'^2 + b x' + c = 0 with the root in [0,1]
// taken as 2c / (-b + sqrt(b^2 - 4ac)).  Also rebuilds the opacity of the
// next step and clears the next step's deposit buffer.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_chem(FrtSolveDesc* descs, const unsigned long long* prefix,
                                                int n_solves, unsigned long long total)
{
    using R2 = typename Vec2<Real>::T;
    __shared__ unsigned long long spre[FRT_MAX_SOLVES_PER_LAUNCH + 1];
    for (int i = threadIdx.x; i <= n_solves; i += blockDim.x) spre[i] = prefix[i];
    __syncthreads();
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long g = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
        int lo = 0, hi = n_solves - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (spre[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const FrtSolveDesc& D = descs[lo];
        if (D.L->err_flags & FRT_DEVERR_QUEUE_OVERFLOW) continue;   // failed step: keep the state
        const size_t i = (size_t)(g - spre[lo]);
        Real* gcur = (Real*)D.gamma[D.step & 1u];
        Real* gnext = (Real*)D.gamma[(D.step + 1u) & 1u];
        const double G = (double)gcur[i];
        const double nH = D.nH[i];
        const double x = D.x[i];
        const double dt = D.dt;
        const double a = dt * nH * (D.alpha_B + D.coll_ion);
        const double bq = -(1.0 + dt * (G + 2.0 * D.alpha_B * nH + D.coll_ion * nH));
        const double cq = x + D.alpha_B * nH * dt;
        double disc = bq * bq - 4.0 * a * cq;
        disc = disc > 0.0 ? disc : 0.0;
        const double xn = 2.0 * cq / (-bq + sqrt(disc));
        D.x[i] = xn;
        R2* op = (R2*)D.op_w;
        op[i].x = (Real)(nH * xn * D.sigma0 * D.dx_cm);
        gnext[i] = Real(0);
    }
}

// Opacity from the loaded state: {n_H x sigma_0 dx, kappa dx} (kappa dx is
// written by the host beforehand into .y).
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_prep(FrtSolveDesc* desc, unsigned long long n)
{
    using R2 = typename Vec2<Real>::T;
    const FrtSolveDesc& D = *desc;
    R2* op = (R2*)D.op_w;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        op[i].x = (Real)(D.nH[i] * D.x[i] * D.sigma0 * D.dx_cm);
}

// Close the step: packets that ended in flight become the ledger's
// in-flight term; any split parents left after the last round (none by
// construction of the round count) are counted as lost.
__global__ void k_step_end(FrtSolveDesc* descs, int n_solves)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_solves) return;
    FrtSolveDesc& D = descs[s];
    FrtLedgerDev* L = D.L;
    L->in_flight = L->in_flight_acc;
    L->in_flight_acc = 0.0;
    uint32_t nf = D.count[1 - D.cur];
    L->n_in_flight = nf < D.q[1 - D.cur].cap ? nf : D.q[1 - D.cur].cap;
    L->step_visits = 0;
}

template <typename T>
__global__ void k_fill(T* p, T v, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int g_sm_count = 0;

int grid_for(unsigned long long items, int per_cu)
{
    if (g_sm_count == 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&g_sm_count, hipDeviceAttributeMultiprocessorCount, dev);
        if (g_sm_count <= 0) g_sm_count = 256;
    }
    unsigned long long want = (items + BLOCK - 1) / BLOCK;
    unsigned long long cap = (unsigned long long)g_sm_count * per_cu;
    if (want < 1) want = 1;
    return (int)(want < cap ? want : cap);
}

template <typename Real, bool EXPAND>
hipError_t launch_march_nb(FrtSolveDesc* d, FrtRoundPlan* p, int nb, hipStream_t s)
{
    const int grid = grid_for(1ull << 40, 8);
    switch (nb) {
#define CASE(N) case N: hipLaunchKernelGGL((k_march<Real, N, EXPAND>), dim3(grid), dim3(BLOCK), 0, s, d, p); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

namespace frt {

int device_sm_count()
{
    grid_for(1, 1);
    return g_sm_count;
}

hipError_t launch_emit(FrtSolveDesc* d_descs, const uint32_t* d_emit_prefix, int n_solves, uint32_t total_items,
                       int fp64, hipStream_t s)
{
    if (total_items == 0) return hipSuccess;
    const int grid = grid_for(total_items, 8);
    if (fp64) hipLaunchKernelGGL(k_emit<double>, dim3(grid), dim3(BLOCK), 0, s, d_descs, d_emit_prefix, n_solves, total_items);
    else hipLaunchKernelGGL(k_emit<float>, dim3(grid), dim3(BLOCK), 0, s, d_descs, d_emit_prefix, n_solves, total_items);
    return hipGetLastError();
}

hipError_t launch_round(FrtSolveDesc* d_descs, FrtRoundPlan* d_plan, int n_solves, int round, int fp64, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(64), 0, s, d_descs, d_plan, n_solves, round);
    return hipGetLastError();
}

hipError_t launch_round_march(FrtSolveDesc* d_descs, FrtRoundPlan* d_plan, int round, int nb, int fp64, hipStream_t s)
{
    if (fp64) return round == 0 ? launch_march_nb<double, false>(d_descs, d_plan, nb, s)
                                : launch_march_nb<double, true>(d_descs, d_plan, nb, s);
    return round == 0 ? launch_march_nb<float, false>(d_descs, d_plan, nb, s)
                      : launch_march_nb<float, true>(d_descs, d_plan, nb, s);
}

hipError_t launch_chem(FrtSolveDesc* d_descs, const unsigned long long* d_cell_prefix, int n_solves,
                       unsigned long long total_cells, int fp64, hipStream_t s)
{
    if (total_cells == 0) return hipSuccess;
    const int grid = grid_for(total_cells, 16);
    if (fp64) hipLaunchKernelGGL(k_chem<double>, dim3(grid), dim3(BLOCK), 0, s, d_descs, d_cell_prefix, n_solves, total_cells);
    else hipLaunchKernelGGL(k_chem<float>, dim3(grid), dim3(BLOCK), 0, s, d_descs, d_cell_prefix, n_solves, total_cells);
    return hipGetLastError();
}

hipError_t launch_step_end(FrtSolveDesc* d_descs, int n_solves, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_end, dim3((n_solves + 63) / 64), dim3(64), 0, s, d_descs, n_solves);
    return hipGetLastError();
}

hipError_t launch_prep_opacity(FrtSolveDesc* d_desc, unsigned long long ncell, int fp64, hipStream_t s)
{
    if (ncell == 0) return hipSuccess;
    const int grid = grid_for(ncell, 16);
    if (fp64) hipLaunchKernelGGL(k_prep<double>, dim3(grid), dim3(BLOCK), 0, s, d_desc, ncell);
    else hipLaunchKernelGGL(k_prep<float>, dim3(grid), dim3(BLOCK), 0, s, d_desc, ncell);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 16)), dim3(BLOCK), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, size_t n, hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 16)), dim3(BLOCK), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, size_t n, hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 16)), dim3(BLOCK), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace frt
