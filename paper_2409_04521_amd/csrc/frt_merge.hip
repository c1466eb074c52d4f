// Ray merging at the end of a step (Cain & D'Aloisio, FlexRT I, §3.3) on
// the GPU: the packets a solve carries into the next step are ranked by
// their photons and all but the floor(N_ex N_RT) brightest are grouped by
// their cell and by the pixel of that cell's randomly rotated level-l_merge
// HEALPix sphere that holds their direction; each group of two or more
// becomes one packet with the summed photons of every bin, travelling along
// the pixel's centre, its position, distance from its origin and level the
// photon-weighted means of its members'.  A merged packet refers to a virtual
// origin (position - r dir) with the rotation that takes the centre of its
// own level-l pixel onto the merged direction, so that the march moves and
// splits it like any packet.
//
// Two launch sequences per solve, after the step.  Counting: keys (photons,
// and cell x 2^20 + pixel), the exemption threshold from a descending sort
// of the photons, a sort of the packets by group key, group flags and three
// scans (output slots, merged packets, virtual-origin entries still referred
// to).  Writing, once the host has sized the next table from the counts:
// the kept entries, the merged packets and the carried ones to the queue the
// step's carried-in packets were read from (free once the step has run),
// which then becomes the solve's carried queue.
#include "frt_internal.h"
#include "frt_device.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

namespace {

using namespace frt_dev;

constexpr int BLOCK = 256;
constexpr unsigned long long KEY_EXEMPT = ~0ull;
constexpr int PIX_BITS = 20;
constexpr unsigned long long PIX_MASK = (1ull << PIX_BITS) - 1ull;

int blocks_for(uint32_t n) { return (int)((n + BLOCK - 1) / BLOCK) > 0 ? (int)((n + BLOCK - 1) / BLOCK) : 1; }

// Photons per bin of a carried packet, as the next march will compute them:
// N0_nu exp(-(s_nu A + K)), N0_nu = w0 spec_nu, times R_ref.
template <typename Real, int NB>
__device__ __forceinline__ void packet_photons(const FrtSolveDesc& D, const FrtRec<Real>& r, double N[NB])
{
#pragma unroll
    for (int b = 0; b < NB; b++) {
        Real s_rel;
        if constexpr (sizeof(Real) == 8) s_rel = D.sig_reld[b];
        else s_rel = D.sig_rel[b];
        const Real n0 = r.w0 * spec_of<Real>(D, r.src, NB, b);
        Real t = s_rel * r.tau[0] + r.tau[1];
        Real e;
        if constexpr (sizeof(Real) == 8) e = exp(-t);
        else e = __expf(-t);
        N[b] = (double)(n0 * e) * D.R_ref;
    }
}

// The cell's merging-sphere rotation at this step (Shoemake 1992 from three
// counter-based uniforms).
__device__ __forceinline__ void cell_rotation(const FrtSolveDesc& D, uint32_t cell, double q[4])
{
    double u[3];
    for (int k = 0; k < 3; k++) u[k] = merge_uniform(D.seed, D.step, cell, (uint32_t)k);
    shoemake_quat(u, q);
}

// Per carried packet: its photons (the ranking key) and its group key, cell
// index x 2^20 + the NESTED pixel of level l_merge holding R_c^-1 d.
template <typename Real, int NB>
__global__ void __launch_bounds__(BLOCK) k_merge_keys(const FrtSolveDesc* __restrict__ dp, FrtMergeArgs a)
{
    const FrtSolveDesc& D = *dp;
    const FrtRec<Real>* F = (const FrtRec<Real>*)D.F[1 - D.cur].rec;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < a.n; i += gridDim.x * BLOCK) {
        const FrtRec<Real> r = F[i];
        double N[NB];
        packet_photons<Real, NB>(D, r, N);
        // the ranking key in units of R_ref (photon counts overflow FP32)
        double P = 0.0;
#pragma unroll
        for (int b = 0; b < NB; b++) P += N[b];
        ((Real*)a.pkey)[i] = (Real)(P / D.R_ref);
        a.idx[i] = i;
        if (a.all_exempt) {
            a.gkey[i] = KEY_EXEMPT;
            continue;
        }
        int c[3];
        unpack_cell(r.cell, c);
        const uint32_t cell = (uint32_t)c[0] + (uint32_t)D.nx * ((uint32_t)c[1] + (uint32_t)D.ny * (uint32_t)c[2]);
        double q[4];
        cell_rotation(D, cell, q);
        // R^-1 d with the conjugate quaternion
        const double qc[4] = {q[0], -q[1], -q[2], -q[3]};
        double v[3] = {(double)r.dir[0], (double)r.dir[1], (double)r.dir[2]};
        quat_rotate<double>(qc, v);
        const uint32_t pix = nest_pixel_of(a.level, v);
        a.gkey[i] = ((unsigned long long)cell << PIX_BITS) | (unsigned long long)pix;
    }
}

// Packets with at least the photons of the E-th brightest are exempt.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_merge_exempt(FrtMergeArgs a)
{
    const Real T = ((const Real*)a.pkey_sorted)[a.E - 1];
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < a.n; i += gridDim.x * BLOCK)
        if (((const Real*)a.pkey)[i] >= T) a.gkey[i] = KEY_EXEMPT;
}

__device__ __forceinline__ bool exempt_key(unsigned long long k, unsigned long long mask) { return (k & mask) == mask; }

// Group flags over the packets in key order: an exempt packet or a group of
// one is carried as it is (out), a group of two or more is written by its
// first packet (out, lead).  Entries of the old virtual-origin table that a
// packet carried as it is refers to are marked.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_merge_flags(const FrtSolveDesc* __restrict__ dp, FrtMergeArgs a)
{
    const FrtSolveDesc& D = *dp;
    const FrtRec<Real>* F = (const FrtRec<Real>*)D.F[1 - D.cur].rec;
    for (uint32_t j = blockIdx.x * BLOCK + threadIdx.x; j < a.n; j += gridDim.x * BLOCK) {
        const unsigned long long k = a.gkey_s[j];
        uint32_t out = 1, lead = 0;
        if (!exempt_key(k, a.key_mask)) {
            const bool head = j == 0 || a.gkey_s[j - 1] != k;
            const bool tail = j + 1 == a.n || a.gkey_s[j + 1] != k;
            out = head ? 1u : 0u;
            lead = (head && !tail) ? 1u : 0u;
        }
        a.flag_out[j] = out;
        a.flag_lead[j] = lead;
        if (out && !lead) {
            const uint32_t src = F[a.idx_s[j]].src;
            if (is_virtual(src) && (src & ~FRT_VSRC) < a.n_old) a.ref[src & ~FRT_VSRC] = 1u;
        }
    }
}

__global__ void k_merge_clear(uint32_t* v, uint32_t n)
{
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) v[i] = 0u;
}

// Totals of the three scans: outputs, merged packets, kept table entries.
__global__ void k_merge_totals(FrtMergeArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    a.counts[0] = a.n ? a.slot[a.n - 1] + a.flag_out[a.n - 1] : 0u;
    a.counts[1] = a.n ? a.gid[a.n - 1] + a.flag_lead[a.n - 1] : 0u;
    a.counts[2] = a.n_old ? a.vmap[a.n_old - 1] + a.ref[a.n_old - 1] : 0u;
}

// Entries of the old table still referred to, to their places in the new one.
__global__ void __launch_bounds__(BLOCK) k_merge_keep_origins(const FrtSolveDesc* __restrict__ dp, FrtMergeArgs a)
{
    const FrtSolveDesc& D = *dp;
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < a.n_old; v += gridDim.x * BLOCK)
        if (a.ref[v]) D.vt[1 - D.cur][a.vmap[v]] = D.vt[D.cur][v];
}

__device__ __forceinline__ void atomic_max_pos_float(float* p, float v)
{
    // positive floats order as their bit patterns
    atomicMax((int*)p, __float_as_int(v));
}

// Per group member, the sums a merged packet is built from: photons W,
// photon-weighted position (3), distance and level, the member count, then
// the photons of each bin.
constexpr int ACC_FIXED = 7;
constexpr int ACC_N = ACC_FIXED + FRT_MAX_BINS_I;
constexpr int WAVE = 64;

// The packet merged from the group whose first packet is at sorted position
// h, from the group's sums v: direction the centre of its merging pixel
// (rotated), position, distance and level the photon-weighted means, photons
// per bin summed; it refers to a new virtual origin (position - r dir, the
// rotation that takes the centre of its own level-l pixel onto its
// direction, photons per bin relative to R_ref w0).
template <typename Real, int NB>
__device__ void write_merged(const FrtSolveDesc& D, const FrtMergeArgs& a, uint32_t h, const double* v, double& res,
                             unsigned long long& merged_in, unsigned long long& groups, float& w0_hi)
{
    FrtRec<Real>* dst = (FrtRec<Real>*)a.dst;
    const unsigned long long k = a.gkey_s[h];
    const double W = v[0];
    double pos[3];
    for (int c = 0; c < 3; c++) pos[c] = v[1 + c] / W;
    const double rbar = v[4] / W;
    const int level = (int)floor(v[5] / W + 0.5);
    const uint32_t cell = (uint32_t)(k >> PIX_BITS);
    const uint32_t p = (uint32_t)(k & PIX_MASK);
    const int lm = a.level;
    const uint32_t pix_v = level >= lm ? p << (2 * (level - lm)) : p >> (2 * (lm - level));
    double qc[4], dm[3], dv[3], qa[4], qv[4];
    cell_rotation(D, cell, qc);
    nest_pixel_centre<double>(lm, p, dm);
    nest_pixel_centre<double>(level, pix_v, dv);
    quat_between(dv, dm, qa);
    quat_mul(qc, qa, qv);
    quat_rotate<double>(qc, dm);            // the merged direction
    // photons per bin relative to R_ref w0, at most 1
    double mx = 0.0;
#pragma unroll
    for (int b = 0; b < NB; b++) mx = fmax(mx, v[ACC_FIXED + b]);
    const double w0 = mx / D.R_ref;
    const uint32_t vi = a.counts[2] + a.gid[h];
    FrtVSrc e;
    for (int c = 0; c < 3; c++) e.pos[c] = pos[c] - rbar * dm[c];
    for (int c = 0; c < 4; c++) e.q[c] = qv[c];
    for (int b = 0; b < FRT_MAX_BINS_I; b++) e.spec[b] = b < NB && w0 > 0.0 ? v[ACC_FIXED + b] / (D.R_ref * w0) : 0.0;
    D.vt[1 - D.cur][vi] = e;
    FrtRec<Real> r{};
    r.src = FRT_VSRC | vi;
    r.estep = D.step;
    r.lp = ((uint32_t)level << 28) | pix_v;
    // the merged position lies in the group's cell (a mean of points in
    // it); on a face the packet is in the cell it enters
    int cc[3] = {(int)(cell % (uint32_t)D.nx), (int)((cell / (uint32_t)D.nx) % (uint32_t)D.ny),
                 (int)(cell / ((uint32_t)D.nx * (uint32_t)D.ny))};
    const int dims[3] = {D.nx, D.ny, D.nz};
    for (int c = 0; c < 3; c++) {
        double f = floor(pos[c]);
        if (pos[c] == f && dm[c] < 0.0) f -= 1.0;
        if (f >= 0.0 && f < (double)dims[c]) cc[c] = (int)f;
    }
    r.cell = pack_cell(cc);
    r.key = (uint32_t)(cc[0] >> D.bsh[0]) +
            (uint32_t)D.bpx * ((uint32_t)(cc[1] >> D.bsh[1]) + (uint32_t)D.bpy * (uint32_t)(cc[2] >> D.bsh[2]));
    r.r = (Real)rbar;
    r.rstop = r.r;
    r.w0 = (Real)w0;
    for (int c = 0; c < 3; c++) r.dir[c] = (Real)dm[c];
    dst[a.slot[h]] = r;
    // photons the record now holds, as the march will compute them
    double after = 0.0;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const Real n0 = r.w0 * (Real)e.spec[b];
        after += (double)n0 * D.R_ref;
        res += v[ACC_FIXED + b];
    }
    res -= after;
    merged_in += (unsigned long long)v[6];
    groups++;
    w0_hi = fmaxf(w0_hi, (float)w0 * 1.0000002f);
}

// The wave's residual, counts and largest merged w0, added with one atomic
// each by its first lane (every lane of the wave calls this).
__device__ __forceinline__ void flush_merge_stats(const FrtSolveDesc& D, const FrtMergeArgs& a, double res,
                                                  unsigned long long merged_in, unsigned long long groups, float w0_hi)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        res += __shfl_xor(res, o, WAVE);
        merged_in += __shfl_xor(merged_in, o, WAVE);
        groups += __shfl_xor(groups, o, WAVE);
        w0_hi = fmaxf(w0_hi, __shfl_xor(w0_hi, o, WAVE));
    }
    if ((threadIdx.x & (WAVE - 1)) == 0 && groups) {
        atomicAdd(a.residual, res);
        atomicAdd(&a.stats[0], groups);
        atomicAdd(&a.stats[1], merged_in);
        atomic_max_pos_float(D.w0_merged, w0_hi);
    }
}

// One thread per packet in group-key order.  A packet that is exempt or
// alone in its group is carried as it is (its table entry renumbered).  The
// members of a group of two or more add up their sums by a segmented scan
// over the wave; the last member of a group in the wave then writes the
// merged packet if the whole group lies in this wave, or adds the wave's
// part to the group's accumulator otherwise (one per wave: the slot of the
// wave that holds the group's first packet, since only the last group of a
// wave can reach past it), which k_merge_finalize turns into the packet.
template <typename Real, int NB>
__global__ void __launch_bounds__(BLOCK) k_merge_emit(const FrtSolveDesc* __restrict__ dp, FrtMergeArgs a)
{
    static_assert(BLOCK % WAVE == 0, "waves cover whole 64-packet chunks");
    const FrtSolveDesc& D = *dp;
    const FrtRec<Real>* F = (const FrtRec<Real>*)D.F[1 - D.cur].rec;
    FrtRec<Real>* dst = (FrtRec<Real>*)a.dst;
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    double res = 0.0;
    unsigned long long merged_in = 0, groups = 0;
    float w0_hi = 0.f;
    const uint32_t n_pad = (a.n + WAVE - 1) / WAVE * WAVE;   // whole waves take part in the shuffles
    for (uint32_t j = blockIdx.x * BLOCK + threadIdx.x; j < n_pad; j += gridDim.x * BLOCK) {
        const bool valid = j < a.n;
        const unsigned long long k = valid ? a.gkey_s[j] : KEY_EXEMPT;
        bool member = false, head = false, tail = false;
        if (valid && !exempt_key(k, a.key_mask)) {
            head = j == 0 || a.gkey_s[j - 1] != k;
            tail = j + 1 == a.n || a.gkey_s[j + 1] != k;
            member = !(head && tail);
        }
        double v[ACC_FIXED + NB];
#pragma unroll
        for (int c = 0; c < ACC_FIXED + NB; c++) v[c] = 0.0;
        if (valid) {
            FrtRec<Real> r = F[a.idx_s[j]];
            if (!member) {
                if (is_virtual(r.src) && (r.src & ~FRT_VSRC) < a.n_old) r.src = FRT_VSRC | a.vmap[r.src & ~FRT_VSRC];
                dst[a.slot[j]] = r;
            } else {
                double N[NB];
                packet_photons<Real, NB>(D, r, N);
                double w = 0.0;
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    w += N[b];
                    v[ACC_FIXED + b] = N[b];
                }
                const double* o = src_pos_of(D, r.src);
                v[0] = w;
                for (int c = 0; c < 3; c++) v[1 + c] = w * (o[c] + (double)r.r * (double)r.dir[c]);
                v[4] = w * (double)r.r;
                v[5] = w * (double)(r.lp >> 28);
                v[6] = 1.0;
            }
        }
        if (!__ballot(member)) continue;   // no group member in this wave (whole waves iterate together)
        // the wave's runs of members with equal keys, each from its first lane
        const unsigned long long prev_k = __shfl_up(k, 1, WAVE);
        const int prev_member = __shfl_up((int)member, 1, WAVE);
        const bool start = member && (lane == 0 || !prev_member || prev_k != k);
        const unsigned long long starts = __ballot(start);
        const unsigned long long heads = __ballot(member && head);
        const unsigned long long upto = (lane == WAVE - 1) ? ~0ull : ((2ull << lane) - 1ull);
        const int s0 = member ? 63 - __clzll(starts & upto) : lane;
        for (int d = 1; d < WAVE; d <<= 1) {
#pragma unroll
            for (int c = 0; c < ACC_FIXED + NB; c++) {
                const double o = __shfl_up(v[c], d, WAVE);
                if (member && lane - d >= s0) v[c] += o;
            }
        }
        const unsigned long long next_k = __shfl_down(k, 1, WAVE);
        const int next_member = __shfl_down((int)member, 1, WAVE);
        const bool run_end = member && (lane == WAVE - 1 || !next_member || next_k != k);
        if (run_end) {
            const uint32_t base = j - (uint32_t)lane;
            const bool own_head = ((heads >> s0) & 1ull) != 0;
            if (own_head && tail) {
                write_merged<Real, NB>(D, a, base + (uint32_t)s0, v, res, merged_in, groups, w0_hi);
            } else {
                // the group's first packet: in this wave, or found by a search
                // of the keys before it
                uint32_t h = base + (uint32_t)s0;
                if (!own_head) {
                    uint32_t lo = 0, hi = base;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (a.gkey_s[mid] < k) lo = mid + 1;
                        else hi = mid;
                    }
                    h = lo;
                }
                const uint32_t sl = h / WAVE;
                double* acc = a.acc + (size_t)sl * ACC_N;
#pragma unroll
                for (int c = 0; c < ACC_FIXED + NB; c++) atomicAdd(acc + c, v[c]);
                if (own_head) a.acc_head[sl] = h;
            }
        }
    }
    flush_merge_stats(D, a, res, merged_in, groups, w0_hi);
}

// The groups that reach across waves: one thread per accumulator slot.
template <typename Real, int NB>
__global__ void __launch_bounds__(BLOCK) k_merge_finalize(const FrtSolveDesc* __restrict__ dp, FrtMergeArgs a)
{
    const FrtSolveDesc& D = *dp;
    double res = 0.0;
    unsigned long long merged_in = 0, groups = 0;
    float w0_hi = 0.f;
    for (uint32_t sl = blockIdx.x * BLOCK + threadIdx.x; sl < a.n_slots; sl += gridDim.x * BLOCK) {
        const uint32_t h = a.acc_head[sl];
        if (h == ~0u) continue;
        double v[ACC_FIXED + NB];
        const double* acc = a.acc + (size_t)sl * ACC_N;
#pragma unroll
        for (int c = 0; c < ACC_FIXED + NB; c++) v[c] = acc[c];
        write_merged<Real, NB>(D, a, h, v, res, merged_in, groups, w0_hi);
    }
    flush_merge_stats(D, a, res, merged_in, groups, w0_hi);
}

__global__ void __launch_bounds__(BLOCK) k_merge_acc_clear(FrtMergeArgs a)
{
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < a.n_slots; i += gridDim.x * BLOCK) {
        a.acc_head[i] = ~0u;
        double* acc = a.acc + (size_t)i * ACC_N;
        for (int c = 0; c < ACC_N; c++) acc[c] = 0.0;
    }
}

// Counts and ledger terms of the merged queue (which the host then makes
// the solve's carried queue).
template <typename Real>
__global__ void k_merge_finish(FrtSolveDesc* dp, FrtMergeArgs a)
{
    FrtSolveDesc& D = *dp;
    const uint32_t m = a.counts[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        D.fcount[1 - D.cur] = m;
        D.vcount[1 - D.cur] = a.counts[2] + a.counts[1];
        FrtLedgerDev* L = D.L;
        L->merge_residual += *a.residual;
        L->in_flight -= *a.residual;
        L->n_in_flight = m;
        L->merges += a.stats[0];
        L->rays_merged += a.stats[1];
    }
}

__global__ void k_merge_zero(FrtMergeArgs a)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *a.residual = 0.0;
        a.stats[0] = 0;
        a.stats[1] = 0;
    }
}

// Counting phase: keys, the exemption, the group sort, flags, the three
// scans and their totals (a.counts, read by the host to size the next table
// of virtual origins before the writing phase).
template <typename Real, int NB>
hipError_t count_nb(FrtSolveDesc* d, FrtMergeArgs a, hipStream_t st)
{
    hipError_t e;
    const int g = blocks_for(a.n);
    hipLaunchKernelGGL(k_merge_zero, dim3(1), dim3(64), 0, st, a);
    hipLaunchKernelGGL((k_merge_keys<Real, NB>), dim3(g), dim3(BLOCK), 0, st, d, a);
    size_t tb = a.temp_bytes;
    if (!a.all_exempt && a.E > 0) {
        if ((e = rocprim::radix_sort_keys_desc(a.temp, tb, (Real*)a.pkey, (Real*)a.pkey_sorted, a.n, 0,
                                               8 * (unsigned)sizeof(Real), st)) != hipSuccess)
            return e;
        hipLaunchKernelGGL((k_merge_exempt<Real>), dim3(g), dim3(BLOCK), 0, st, a);
    }
    if (!a.all_exempt) {
        tb = a.temp_bytes;
        if ((e = rocprim::radix_sort_pairs(a.temp, tb, a.gkey, a.gkey_s, a.idx, a.idx_s, a.n, 0, (unsigned)a.end_bit,
                                           st)) != hipSuccess)
            return e;
    } else {
        (void)hipMemcpyAsync(a.gkey_s, a.gkey, (size_t)a.n * 8, hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(a.idx_s, a.idx, (size_t)a.n * 4, hipMemcpyDeviceToDevice, st);
    }
    if (a.n_old) hipLaunchKernelGGL(k_merge_clear, dim3(blocks_for(a.n_old)), dim3(BLOCK), 0, st, a.ref, a.n_old);
    hipLaunchKernelGGL((k_merge_flags<Real>), dim3(g), dim3(BLOCK), 0, st, d, a);
    tb = a.temp_bytes;
    if ((e = rocprim::exclusive_scan(a.temp, tb, a.flag_out, a.slot, 0u, (size_t)a.n, rocprim::plus<uint32_t>(), st)) !=
        hipSuccess)
        return e;
    tb = a.temp_bytes;
    if ((e = rocprim::exclusive_scan(a.temp, tb, a.flag_lead, a.gid, 0u, (size_t)a.n, rocprim::plus<uint32_t>(), st)) !=
        hipSuccess)
        return e;
    if (a.n_old) {
        tb = a.temp_bytes;
        if ((e = rocprim::exclusive_scan(a.temp, tb, a.ref, a.vmap, 0u, (size_t)a.n_old, rocprim::plus<uint32_t>(), st)) !=
            hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_merge_totals, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}

// Writing phase: the kept table entries, the merged packets and the queue.
template <typename Real, int NB>
hipError_t write_nb(FrtSolveDesc* d, FrtMergeArgs a, hipStream_t st)
{
    const int g = blocks_for(a.n);
    if (a.n_old) hipLaunchKernelGGL(k_merge_keep_origins, dim3(blocks_for(a.n_old)), dim3(BLOCK), 0, st, d, a);
    hipLaunchKernelGGL(k_merge_acc_clear, dim3(blocks_for(a.n_slots)), dim3(BLOCK), 0, st, a);
    hipLaunchKernelGGL((k_merge_emit<Real, NB>), dim3(g), dim3(BLOCK), 0, st, d, a);
    hipLaunchKernelGGL((k_merge_finalize<Real, NB>), dim3(blocks_for(a.n_slots)), dim3(BLOCK), 0, st, d, a);
    hipLaunchKernelGGL((k_merge_finish<Real>), dim3(1), dim3(64), 0, st, d, a);
    return hipGetLastError();
}

template <typename Real>
hipError_t merge_t(FrtSolveDesc* d, const FrtMergeArgs& a, int nb, int phase, hipStream_t st)
{
#define FRT_MERGE_NB(K) \
    case K: return phase == 0 ? count_nb<Real, K>(d, a, st) : write_nb<Real, K>(d, a, st);
    switch (nb) {
        FRT_MERGE_NB(1)
        FRT_MERGE_NB(2)
        FRT_MERGE_NB(3)
        FRT_MERGE_NB(4)
        FRT_MERGE_NB(5)
        FRT_MERGE_NB(6)
        FRT_MERGE_NB(7)
        FRT_MERGE_NB(8)
        default: return hipErrorInvalidValue;
    }
#undef FRT_MERGE_NB
}

template <typename Real>
size_t temp_bytes_t(uint32_t n, uint32_t n_old)
{
    size_t need = 0, b = 0;
    Real* kf = nullptr;
    unsigned long long* k64 = nullptr;
    uint32_t* u = nullptr;
    (void)rocprim::radix_sort_keys_desc(nullptr, b, kf, kf, n, 0, 8 * (unsigned)sizeof(Real));
    need = b > need ? b : need;
    b = 0;
    (void)rocprim::radix_sort_pairs(nullptr, b, k64, k64, u, u, n, 0, 64u);
    need = b > need ? b : need;
    b = 0;
    const size_t ns = n > n_old ? n : n_old;
    (void)rocprim::exclusive_scan(nullptr, b, u, u, 0u, ns, rocprim::plus<uint32_t>());
    need = b > need ? b : need;
    return need;
}

}  // namespace

namespace frt {

hipError_t launch_merge(FrtSolveDesc* d, const FrtMergeArgs& a, int fp64, int n_bins, int phase, hipStream_t st)
{
    if (a.n == 0) return hipSuccess;
    return fp64 ? merge_t<double>(d, a, n_bins, phase, st) : merge_t<float>(d, a, n_bins, phase, st);
}

size_t merge_temp_bytes(uint32_t n, uint32_t n_old, int fp64)
{
    return fp64 ? temp_bytes_t<double>(n, n_old) : temp_bytes_t<float>(n, n_old);
}

}  // namespace frt
