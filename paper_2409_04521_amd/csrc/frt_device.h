// Device helpers shared by the HIP kernels of the ray-tracing library:
// HEALPix NESTED pixel centres and pixel lookup (Gorski et al. 2005), the
// counter-based uniforms and uniform random rotations of the sources'
// spheres and of the cells' merging spheres, packed cell coordinates, and
// the origin, photon rates and rotation of a packet (its source's, or those
// of the merged packet's virtual origin).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "frt_internal.h"

namespace frt_dev {

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
__device__ inline void nest_pixel_centre(int level, uint32_t pix, Real v[3])
{
    const int nside = 1 << level;
    const uint32_t face = pix >> (2 * level);
    // ring of the face's southern corner (in units of Nside) and its
    // longitude index: faces 0-3 are the northern row, 4-7 the equatorial
    // row (shifted by half a face), 8-11 the southern row
    const int jr_face = (int)(face >> 2) + 2;
    const int jp_face = 2 * (int)(face & 3u) + ((face >> 2) == 1u ? 0 : 1);
    const uint32_t sub = pix & ((1u << (2 * level)) - 1u);
    const int ix = (int)squeeze_even_bits(sub);
    const int iy = (int)squeeze_even_bits(sub >> 1);
    const int j = jr_face * nside - ix - iy - 1;
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
    int k = jp_face * nr + ix - iy;
    if (k < 0) k += 8 * nr;
    else if (k >= 8 * nr) k -= 8 * nr;
    // phi = (pi/4) k / nr: sincospi(k / (4 nr)) in FP64; in FP32 the
    // hardware sine and cosine, which take their argument in turns
    // (phi / 2pi = k / (8 nr)), accurate to the precision of the FP32 march
    Real s, c;
    if constexpr (sizeof(Real) == 8) {
        sincospi(Real(k) / Real(4 * nr), &s, &c);
    } else {
        const float turns = (float)k / (float)(8 * nr);
        s = __builtin_amdgcn_sinf(turns);
        c = __builtin_amdgcn_cosf(turns);
    }
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
__device__ inline void shoemake_quat(const double u[3], double q[4])
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

// Pixel of level `level` holding unit vector v (NESTED; Gorski et al. 2005,
// ang2pix): on the equatorial belt (|z| <= 2/3) the pixel's face and in-face
// coordinates come from the two families of ring-crossing lines through
// (phi, z); on the polar caps from the distance to the pole.
__device__ __forceinline__ uint32_t spread_even_bits(uint32_t v)
{
    v &= 0x0000ffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ inline uint32_t nest_pixel_of(int level, const double v[3])
{
    const int nside = 1 << level;
    const double z = v[2];
    double phi = atan2(v[1], v[0]);
    if (phi < 0.0) phi += 2.0 * M_PI;
    const double tt = phi * (2.0 / M_PI);          // in [0, 4)
    int face, ix, iy;
    if (fabs(z) <= 2.0 / 3.0) {
        const double t1 = nside * (0.5 + tt), t2 = nside * z * 0.75;
        const int jp = (int)(t1 - t2), jm = (int)(t1 + t2);
        const int ifp = jp >> level, ifm = jm >> level;
        face = ifp == ifm ? (ifp | 4) : (ifp < ifm ? ifp : ifm + 8);
        ix = jm & (nside - 1);
        iy = nside - (jp & (nside - 1)) - 1;
    } else {
        int ntt = (int)tt;
        if (ntt > 3) ntt = 3;
        const double tp = tt - ntt;
        const double tmp = nside * sqrt(3.0 * (1.0 - fabs(z)));
        int jp = (int)(tp * tmp), jm = (int)((1.0 - tp) * tmp);
        if (jp > nside - 1) jp = nside - 1;
        if (jm > nside - 1) jm = nside - 1;
        if (z >= 0) {
            face = ntt;
            ix = nside - jm - 1;
            iy = nside - jp - 1;
        } else {
            face = ntt + 8;
            ix = jp;
            iy = jm;
        }
    }
    return ((uint32_t)face << (2 * level)) | spread_even_bits((uint32_t)ix) | (spread_even_bits((uint32_t)iy) << 1);
}

// Uniforms of a cell's merging sphere: the SplitMix64 output function of
// (step<<34 | cell<<2 | k) xor a key of its own stream derived from the seed.
constexpr uint64_t MERGE_STREAM = 0x6D65726765ull;   // ASCII "merge"

__device__ __forceinline__ double merge_uniform(uint64_t seed, uint32_t step, uint32_t cell, uint32_t k)
{
    const uint64_t ctr = ((uint64_t)step << 34) | ((uint64_t)cell << 2) | (uint64_t)k;
    return (double)(mix64(ctr ^ mix64(mix64(seed) ^ MERGE_STREAM)) >> 11) * 0x1.0p-53;
}

// Quaternion product a b (w, x, y, z).
__device__ __forceinline__ void quat_mul(const double a[4], const double b[4], double o[4])
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// The shortest rotation taking unit vector a onto unit vector b (a != -b),
// as the unit quaternion proportional to (1 + a.b, a x b).
__device__ __forceinline__ void quat_between(const double a[3], const double b[3], double q[4])
{
    q[0] = 1.0 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    q[1] = a[1] * b[2] - a[2] * b[1];
    q[2] = a[2] * b[0] - a[0] * b[2];
    q[3] = a[0] * b[1] - a[1] * b[0];
    const double n = rsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; k++) q[k] *= n;
}

// A packet's cell as packed coordinates x | y << 11 | z << 22 (grids have at
// most 2048 cells per axis), so that no division recovers them.
__device__ __forceinline__ uint32_t pack_cell(const int c[3])
{
    return (uint32_t)c[0] | ((uint32_t)c[1] << 11) | ((uint32_t)c[2] << 22);
}

__device__ __forceinline__ void unpack_cell(uint32_t p, int c[3])
{
    c[0] = (int)(p & 2047u);
    c[1] = (int)((p >> 11) & 2047u);
    c[2] = (int)(p >> 22);
}

// A packet's source index refers to the solve's sources, or (with this bit
// set) to an entry of the virtual-origin table its packets of this step
// refer to (merged packets, §3.3).
__device__ __forceinline__ bool is_virtual(uint32_t src) { return (src & FRT_VSRC) != 0u; }

__device__ __forceinline__ const double* src_pos_of(const FrtSolveDesc& D, uint32_t src)
{
    return is_virtual(src) ? D.vt[D.cur][src & ~FRT_VSRC].pos : D.src_pos + (size_t)src * 3;
}

template <typename Real>
__device__ __forceinline__ Real spec_of(const FrtSolveDesc& D, uint32_t src, int nb, int b)
{
    if (is_virtual(src)) return (Real)D.vt[D.cur][src & ~FRT_VSRC].spec[b];
    if constexpr (sizeof(Real) == 4) return D.spec[(size_t)src * nb + b];
    else return D.specd[(size_t)src * nb + b];
}

__device__ __forceinline__ const double* rot_of(const FrtSolveDesc& D, uint32_t estep, uint32_t src)
{
    return is_virtual(src) ? D.vt[D.cur][src & ~FRT_VSRC].q : D.quat + ((size_t)estep * D.n_src + src) * 4;
}

}  // namespace frt_dev
