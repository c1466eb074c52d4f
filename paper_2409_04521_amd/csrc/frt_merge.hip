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
// One launch sequence per solve, after the step: keys (photons, and cell x
// 2^20 + pixel), the exemption threshold from a descending sort of the
// photons, a sort of the packets by group key, group flags and three scans
// (output slots, merged packets, virtual-origin entries still referred to),
// the merged packets and the carried ones written to a scratch queue, then
// copied back over the solve's carried queue.
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

// Output: a packet carried as it is (its table entry renumbered), or the
// packet merged from a group, written by the group's first packet.
template <typename Real, int NB>
__global__ void __launch_bounds__(BLOCK) k_merge_emit(const FrtSolveDesc* __restrict__ dp, FrtMergeArgs a)
{
    const FrtSolveDesc& D = *dp;
    const FrtRec<Real>* F = (const FrtRec<Real>*)D.F[1 - D.cur].rec;
    FrtRec<Real>* dst = (FrtRec<Real>*)a.dst;
    const uint32_t n_kept = a.counts[2];
    double res = 0.0;
    unsigned long long merged_in = 0, groups = 0;
    for (uint32_t j = blockIdx.x * BLOCK + threadIdx.x; j < a.n; j += gridDim.x * BLOCK) {
        if (!a.flag_out[j]) continue;
        const uint32_t s = a.slot[j];
        if (!a.flag_lead[j]) {
            FrtRec<Real> r = F[a.idx_s[j]];
            if (is_virtual(r.src) && (r.src & ~FRT_VSRC) < a.n_old) r.src = FRT_VSRC | a.vmap[r.src & ~FRT_VSRC];
            dst[s] = r;
            continue;
        }
        // a group: photon sums and photon-weighted means in FP64
        const unsigned long long k = a.gkey_s[j];
        double W = 0.0, pos[3] = {0.0, 0.0, 0.0}, rs = 0.0, ls = 0.0, Nb[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) Nb[b] = 0.0;
        uint32_t m = 0;
        for (uint32_t q = j; q < a.n && a.gkey_s[q] == k; q++, m++) {
            const FrtRec<Real> r = F[a.idx_s[q]];
            double N[NB];
            packet_photons<Real, NB>(D, r, N);
            double w = 0.0;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                w += N[b];
                Nb[b] += N[b];
            }
            const double* o = src_pos_of(D, r.src);
            for (int c = 0; c < 3; c++) pos[c] += w * (o[c] + (double)r.r * (double)r.dir[c]);
            rs += w * (double)r.r;
            ls += w * (double)(r.lp >> 28);
            W += w;
        }
        for (int c = 0; c < 3; c++) pos[c] /= W;
        const double rbar = rs / W;
        int level = (int)floor(ls / W + 0.5);
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
        for (int b = 0; b < NB; b++) mx = fmax(mx, Nb[b]);
        const double w0 = mx / D.R_ref;
        const uint32_t v = n_kept + a.gid[j];
        FrtVSrc e;
        for (int c = 0; c < 3; c++) e.pos[c] = pos[c] - rbar * dm[c];
        for (int c = 0; c < 4; c++) e.q[c] = qv[c];
        for (int b = 0; b < FRT_MAX_BINS_I; b++) e.spec[b] = b < NB && w0 > 0.0 ? Nb[b] / (D.R_ref * w0) : 0.0;
        D.vt[1 - D.cur][v] = e;
        FrtRec<Real> r{};
        r.src = FRT_VSRC | v;
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
        dst[s] = r;
        // photons the record now holds, as the march will compute them
        double after = 0.0;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const Real n0 = r.w0 * (Real)e.spec[b];
            after += (double)n0 * D.R_ref;
            res += Nb[b];
        }
        res -= after;
        merged_in += m;
        groups++;
        atomic_max_pos_float(D.w0_merged, (float)w0 * 1.0000002f);
    }
    if (groups) {
        atomicAdd(a.residual, res);
        atomicAdd(&a.stats[0], groups);
        atomicAdd(&a.stats[1], merged_in);
    }
}

// The merged queue back over the carried queue; counts and ledger terms.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_merge_finish(FrtSolveDesc* dp, FrtMergeArgs a)
{
    FrtSolveDesc& D = *dp;
    FrtRec<Real>* F = (FrtRec<Real>*)D.F[1 - D.cur].rec;
    const FrtRec<Real>* src = (const FrtRec<Real>*)a.dst;
    const uint32_t m = a.counts[0];
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < m; i += gridDim.x * BLOCK) F[i] = src[i];
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

template <typename Real, int NB>
hipError_t merge_nb(FrtSolveDesc* d, FrtMergeArgs a, hipStream_t st)
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
    if (a.n_old) hipLaunchKernelGGL(k_merge_keep_origins, dim3(blocks_for(a.n_old)), dim3(BLOCK), 0, st, d, a);
    hipLaunchKernelGGL((k_merge_emit<Real, NB>), dim3(g), dim3(BLOCK), 0, st, d, a);
    hipLaunchKernelGGL((k_merge_finish<Real>), dim3(g), dim3(BLOCK), 0, st, d, a);
    return hipGetLastError();
}

template <typename Real>
hipError_t merge_t(FrtSolveDesc* d, const FrtMergeArgs& a, int nb, hipStream_t st)
{
    switch (nb) {
        case 1: return merge_nb<Real, 1>(d, a, st);
        case 2: return merge_nb<Real, 2>(d, a, st);
        case 3: return merge_nb<Real, 3>(d, a, st);
        case 4: return merge_nb<Real, 4>(d, a, st);
        case 5: return merge_nb<Real, 5>(d, a, st);
        case 6: return merge_nb<Real, 6>(d, a, st);
        case 7: return merge_nb<Real, 7>(d, a, st);
        case 8: return merge_nb<Real, 8>(d, a, st);
        default: return hipErrorInvalidValue;
    }
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

hipError_t launch_merge(FrtSolveDesc* d, const FrtMergeArgs& a, int fp64, int n_bins, hipStream_t st)
{
    if (a.n == 0) return hipSuccess;
    return fp64 ? merge_t<double>(d, a, n_bins, st) : merge_t<float>(d, a, n_bins, st);
}

size_t merge_temp_bytes(uint32_t n, uint32_t n_old, int fp64)
{
    return fp64 ? temp_bytes_t<double>(n, n_old) : temp_bytes_t<float>(n, n_old);
}

}  // namespace frt
