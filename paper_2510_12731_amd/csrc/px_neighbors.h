// Neighbour searches over the Morton-ordered atoms (device code): a one-wave
// workgroup owns 64 row atoms (two groups of GROUP) and visits the source
// groups whose bounding box lies within a distance of its rows' box, in
// increasing order, with each group's atoms fetched by one vector load while
// the previous group is being processed.  The candidate groups of a row block
// can be shared out over nsub workgroups: subset s takes candidates s,
// s + nsub, ... of the sequence (every subset still tests all the boxes).
#pragma once

#include "px_internal.h"

#include <hip/hip_runtime.h>

namespace px {
namespace nbr {

// Squared gap between two axis-aligned boxes (0 when they overlap).
__device__ __forceinline__ float box_gap2(float4 alo, float4 ahi, float4 blo, float4 bhi)
{
    const float dx = fmaxf(0.0f, fmaxf(blo.x - ahi.x, alo.x - bhi.x));
    const float dy = fmaxf(0.0f, fmaxf(blo.y - ahi.y, alo.y - bhi.y));
    const float dz = fmaxf(0.0f, fmaxf(blo.z - ahi.z, alo.z - bhi.z));
    return dx * dx + dy * dy + dz * dz;
}

// Box of the 64 rows (groups g0 and g0 + 1) of a one-wave workgroup.
__device__ __forceinline__ void wave_box(const float4* __restrict__ glo, const float4* __restrict__ ghi, int64_t g0,
                                         float4& lo, float4& hi)
{
    const float4 a0 = glo[g0], a1 = glo[g0 + 1], b0 = ghi[g0], b1 = ghi[g0 + 1];
    lo = make_float4(fminf(a0.x, a1.x), fminf(a0.y, a1.y), fminf(a0.z, a1.z), 0.f);
    hi = make_float4(fmaxf(b0.x, b1.x), fmaxf(b0.y, b1.y), fmaxf(b0.z, b1.z), 0.f);
}

// The candidate source groups in increasing order, wave-uniform: the lanes
// test 64 groups at a time and the wave walks the set bits.
struct GroupWalk {
    float4 lo, hi;
    const float4* glo;
    const float4* ghi;
    int64_t ngroups;
    float lim2;
    int64_t base = -64;
    uint64_t mask = 0;

    __device__ int64_t next()
    {
        while (mask == 0) {
            base += 64;
            if (base >= ngroups) return -1;
            const int64_t g = base + (threadIdx.x & 63);
            const bool hit = g < ngroups && box_gap2(lo, hi, glo[g], ghi[g]) <= lim2;
            mask = __ballot(hit);
        }
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        return base + b;
    }
};

// Calls f(j, p_j) for every real atom j (< n) of the source groups of subset
// sub (of nsub) among those whose box lies within lim of the box of row block
// rb (64 rows), j increasing, wave-uniform.  Lane k < GROUP loads atom k of a
// group (the next group's load is issued before the current group is
// processed) and the atoms are broadcast from LDS.  For one-wave workgroups
// (64 threads).
template <typename F>
__device__ __forceinline__ void for_near_atoms(const double4* __restrict__ xyz, int64_t n,
                                               const float4* __restrict__ glo, const float4* __restrict__ ghi,
                                               float lim, int64_t rb, int sub, int nsub, F&& f)
{
    __shared__ double4 sp[GROUP];
    const int lane = threadIdx.x & 63;
    GroupWalk w;
    wave_box(glo, ghi, rb * (64 / GROUP), w.lo, w.hi);
    w.glo = glo;
    w.ghi = ghi;
    w.ngroups = (n + GROUP - 1) / GROUP;
    w.lim2 = lim * lim;
    // candidate sub, then every nsub-th
    for (int t = 0; t < sub; ++t)
        if (w.next() < 0) break;
    int64_t g = w.next();
    double4 cur = make_double4(0.0, 0.0, 0.0, 0.0);
    if (g >= 0) cur = xyz[g * GROUP + (lane & (GROUP - 1))];
    while (g >= 0) {
        int64_t gn = -1;
        for (int t = 0; t < nsub; ++t)
            if ((gn = w.next()) < 0) break;
        double4 nxt = cur;
        if (gn >= 0) nxt = xyz[gn * GROUP + (lane & (GROUP - 1))];
        __syncthreads();
        if (lane < GROUP) sp[lane] = cur;
        __syncthreads();
        const int64_t j0 = g * GROUP;
        const int kn = n - j0 < GROUP ? (int)(n - j0) : GROUP;
        for (int k = 0; k < kn; ++k) f(j0 + k, sp[k]);
        cur = nxt;
        g = gn;
    }
}

}  // namespace nbr
}  // namespace px
