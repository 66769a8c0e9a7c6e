// Post-processing (Section "Post-process Analysis"): the field and the
// density of the induced charges (and dipoles) at probe points.  The charges
// are Gaussians of width R_q and the dipoles Gaussian dipoles of width R_mu
// (Section 2): a charge q at r_i gives the density q G(r; R_q), G = exp(-r^2 /
// R^2) / (pi^{3/2} R^3), and the field q g(r) d / r^3 with d = p - r_i, r = |d|
// and g(r) = erf(x) - (2/sqrt(pi)) x exp(-x^2), x = r / R; a dipole mu gives
// the density (2 / R_mu^2) (mu . d) G(r; R_mu) and the field -mu g / r^3 +
// (mu . d) d [3 g / r^5 - (4/sqrt(pi)) exp(-x^2) / (R^3 r^2)].  Beyond 7
// widths the Gaussian corrections are below FP64 rounding and a source acts
// as a point charge or point dipole.
//
// For structures of 4096 atoms or more the points are sorted by their Morton
// code first (so that a wave's 64 points are close together) and the results
// scattered back.  One thread per
// probe point, the source atoms (Morton order) read wave-uniform through the
// scalar cache; a group of 32 atoms whose bounding box lies farther than 7
// widths from the box of the wave's 64 points takes the branch-free point
// path; inside the other groups a wave vote per atom takes the Gaussian
// formulas only where one of the wave's points lies within 7 widths of it.
// With few points the atoms are split over blockIdx.y and k_probe_sum adds
// the splits.

#include "px_internal.h"
#include "px_neighbors.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>

namespace px {

namespace {

constexpr double PROBE_NEAR = 7.0;   // widths beyond which a Gaussian is a point source
constexpr int PROBE_CHUNK = 256;     // atoms per split chunk

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Twice 1/sqrt(q) for q > 0 (hardware estimate and one Newton step; the
// caller halves it).
__device__ __forceinline__ double rsqrt2(double q)
{
    const double y = __builtin_amdgcn_rsq(q);
    return y * fma(-q, y * y, 3.0);
}

// Source of atom i for one column: charge (re, im) and, for the dipole model,
// the dipole's three components (re, im); ghosts and absent columns zero.
template <int S>
__global__ void k_probe_src(const double2* __restrict__ x, int ldx, int col, int64_t n, int64_t np,
                            double* __restrict__ src)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
#pragma unroll
    for (int c = 0; c < S / 2; ++c) {
        double2 v = make_double2(0.0, 0.0);
        if (i < n) v = x[((size_t)c * np + i) * ldx + col];
        src[(size_t)i * S + 2 * c] = v.x;
        src[(size_t)i * S + 2 * c + 1] = v.y;
    }
}

struct ProbeConst {
    double rq, rmu;          // widths (bohr)
    double gq, gmu;          // density normalisations pi^{-3/2} R^{-3}
    float near2;             // squared near distance of a group (bohr^2)
};

// g(r; R) / r^3, the dipole bracket [3 g / r^5 - (4/sqrt(pi)) e^{-x^2} / (R^3
// r^2)] and e^{-x^2}, x = r / R; Taylor series of erf and exp for x < 1/2,
// where the closed forms cancel.
__device__ __forceinline__ void probe_radial(double r, double R, double& g_r3, double& brk, double& ex)
{
    const double x = r / R, x2 = x * x;
    ex = exp(-x2);
    const double c = 1.1283791670955126;   // 2 / sqrt(pi)
    if (x < 0.5) {
        // g / x^3 = c sum_{k>=1} (-1)^{k+1} 2k / (2k+1) x^{2k-2} / k!
        // bracket R^5 = c sum_{k>=2} (-1)^k 4 / ((2k+1) (k-2)!) x^{2k-4}
        double s1 = 0.0, s2 = 0.0, xp = 1.0, xq = 1.0, inv_fact = 1.0, inv_fact2 = 1.0;
        for (int k = 1; k <= 14; ++k) {
            inv_fact /= k;
            const double sgn = (k & 1) ? 1.0 : -1.0;
            s1 += sgn * (2.0 * k / (2.0 * k + 1.0)) * xp * inv_fact;   // xp = x^{2k-2}
            if (k >= 2) {
                if (k >= 3) {
                    inv_fact2 /= (k - 2);
                    xq *= x2;                                           // xq = x^{2k-4}
                }
                s2 -= sgn * 4.0 / (2.0 * k + 1.0) * xq * inv_fact2;
            }
            xp *= x2;
        }
        const double r3 = R * R * R;
        g_r3 = c * s1 / r3;
        brk = c * s2 / (r3 * R * R);
        return;
    }
    const double g = erf(x) - c * x * ex;
    const double ir = 1.0 / r, ir2 = ir * ir, ir3 = ir2 * ir;
    g_r3 = g * ir3;
    brk = 3.0 * g * ir3 * ir2 - 2.0 * c * ex / (R * R * R) * ir2;
}

// Splits of the probe launch: enough waves for every CU (16 per CU as the
// narrow T-apply), at most one chunk of atoms per split.
int probe_splits(int64_t npad, int64_t np)
{
    // filled on first use; concurrent first calls store the same value
    static std::atomic<int> ncu_cache{0};
    int ncu = ncu_cache.load(std::memory_order_relaxed);
    if (ncu == 0) {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cu <= 0)
            cu = 256;
        ncu = cu;
        ncu_cache.store(ncu, std::memory_order_relaxed);
    }
    const int64_t blocks = npad / 256;
    const int64_t nchunk = (np + PROBE_CHUNK - 1) / PROBE_CHUNK;
    int64_t want = (16 * (int64_t)ncu + blocks - 1) / blocks;
    if (want > nchunk) want = nchunk;
    if (want < 1) want = 1;
    return (int)want;
}

template <int MODEL>
__global__ __launch_bounds__(256) void k_probe(const double4* __restrict__ xyz, const double* __restrict__ src,
                                               const float4* __restrict__ glo, const float4* __restrict__ ghi,
                                               int64_t np, const double4* __restrict__ pts,
                                               double* __restrict__ part, int64_t npad, ProbeConst k)
{
    constexpr int S = MODEL ? 8 : 2;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double4 p = pts[i];
    // box of the wave's points
    float lo[3] = {(float)p.x, (float)p.y, (float)p.z}, hi[3] = {lo[0], lo[1], lo[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int off = 32; off > 0; off >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, 64));
        }
    const float4 blo = make_float4(lo[0], lo[1], lo[2], 0.f);
    const float4 bhi = make_float4(hi[0], hi[1], hi[2], 0.f);
    double e[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // E_x, E_y, E_z real then imaginary
    double rho[2] = {0.0, 0.0};
    // one source atom in the point-charge (and point-dipole) form
    auto point_pair = [&](const double* s, double dx, double dy, double dz, double r2) {
        const double ir = 0.5 * rsqrt2(r2);
        const double ir2 = ir * ir, ir3 = ir2 * ir;
        const double fr = s[0] * ir3, fi = s[1] * ir3;
        e[0] = fma(fr, dx, e[0]);
        e[1] = fma(fr, dy, e[1]);
        e[2] = fma(fr, dz, e[2]);
        e[3] = fma(fi, dx, e[3]);
        e[4] = fma(fi, dy, e[4]);
        e[5] = fma(fi, dz, e[5]);
        if (MODEL) {
            const double ir5 = 3.0 * ir3 * ir2;
            const double mdr = fma(s[2], dx, fma(s[4], dy, s[6] * dz)) * ir5;
            const double mdi = fma(s[3], dx, fma(s[5], dy, s[7] * dz)) * ir5;
            e[0] = fma(mdr, dx, fma(-s[2], ir3, e[0]));
            e[1] = fma(mdr, dy, fma(-s[4], ir3, e[1]));
            e[2] = fma(mdr, dz, fma(-s[6], ir3, e[2]));
            e[3] = fma(mdi, dx, fma(-s[3], ir3, e[3]));
            e[4] = fma(mdi, dy, fma(-s[5], ir3, e[4]));
            e[5] = fma(mdi, dz, fma(-s[7], ir3, e[5]));
        }
    };
    // one source atom with its Gaussian charge (and dipole): field and density
    auto gauss_pair = [&](const double* s, double dx, double dy, double dz, double r2) {
        const double r = sqrt(r2);
        double g3, brk, ex;
        probe_radial(r, k.rq, g3, brk, ex);
        const double fr = s[0] * g3, fi = s[1] * g3;
        e[0] = fma(fr, dx, e[0]);
        e[1] = fma(fr, dy, e[1]);
        e[2] = fma(fr, dz, e[2]);
        e[3] = fma(fi, dx, e[3]);
        e[4] = fma(fi, dy, e[4]);
        e[5] = fma(fi, dz, e[5]);
        rho[0] = fma(s[0], k.gq * ex, rho[0]);
        rho[1] = fma(s[1], k.gq * ex, rho[1]);
        if (MODEL) {
            probe_radial(r, k.rmu, g3, brk, ex);
            const double mdr = fma(s[2], dx, fma(s[4], dy, s[6] * dz));
            const double mdi = fma(s[3], dx, fma(s[5], dy, s[7] * dz));
            e[0] = fma(mdr * brk, dx, fma(-s[2], g3, e[0]));
            e[1] = fma(mdr * brk, dy, fma(-s[4], g3, e[1]));
            e[2] = fma(mdr * brk, dz, fma(-s[6], g3, e[2]));
            e[3] = fma(mdi * brk, dx, fma(-s[3], g3, e[3]));
            e[4] = fma(mdi * brk, dy, fma(-s[5], g3, e[4]));
            e[5] = fma(mdi * brk, dz, fma(-s[7], g3, e[5]));
            const double w = 2.0 / (k.rmu * k.rmu) * k.gmu * ex;
            rho[0] = fma(mdr, w, rho[0]);
            rho[1] = fma(mdi, w, rho[1]);
        }
    };
    const double near2 = (double)k.near2;
    const int nchunk = (int)(np / PROBE_CHUNK);
    for (int ch = blockIdx.y; ch < nchunk; ch += gridDim.y)
    for (int gq = ch * (PROBE_CHUNK / GROUP); gq < (ch + 1) * (PROBE_CHUNK / GROUP); ++gq) {
        const int j0 = uniform_i(gq * GROUP);
        if (uniform_i(nbr::box_gap2(blo, bhi, glo[gq], ghi[gq]) >= k.near2)) {
            // the whole group beyond the near distance of the wave's box
#pragma unroll 8
            for (int jj = 0; jj < GROUP; ++jj) {
                const double4 a = xyz[j0 + jj];
                const double dx = p.x - a.x, dy = p.y - a.y, dz = p.z - a.z;
                point_pair(src + (size_t)(j0 + jj) * S, dx, dy, dz, fma(dx, dx, fma(dy, dy, dz * dz)));
            }
        } else {
            // per atom: the Gaussian forms only where one of the wave's points
            // is within the near distance (a wave vote), else the point forms
            for (int jj = 0; jj < GROUP; ++jj) {
                const double4 a = xyz[j0 + jj];
                const double* s = src + (size_t)(j0 + jj) * S;
                const double dx = p.x - a.x, dy = p.y - a.y, dz = p.z - a.z;
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                if (__ballot(r2 < near2) != 0) gauss_pair(s, dx, dy, dz, r2);
                else point_pair(s, dx, dy, dz, r2);
            }
        }
    }
    double* out = part + ((size_t)blockIdx.y * npad + i) * 8;
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = e[c];
    out[6] = rho[0];
    out[7] = rho[1];
}

__device__ __forceinline__ uint32_t spread_bits10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// keys[t] = 30-bit Morton code of point t in the box (lo, lo + 1023 / sc)
// above its index (morton = 0: the index alone, the caller's order); the
// padding up to npow sorts last.
__global__ void k_probe_keys(const double4* __restrict__ pts, int64_t npts, int64_t npow, double3 lo, double sc,
                             int morton, uint64_t* __restrict__ keys)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npow) return;
    if (t >= npts) {
        keys[t] = ~0ull;
        return;
    }
    if (!morton) {
        keys[t] = (uint64_t)t;
        return;
    }
    const double4 p = pts[t];
    const uint32_t qx = (uint32_t)fmin(1023.0, fmax(0.0, (p.x - lo.x) * sc));
    const uint32_t qy = (uint32_t)fmin(1023.0, fmax(0.0, (p.y - lo.y) * sc));
    const uint32_t qz = (uint32_t)fmin(1023.0, fmax(0.0, (p.z - lo.z) * sc));
    const uint32_t code = spread_bits10(qx) | (spread_bits10(qy) << 1) | (spread_bits10(qz) << 2);
    keys[t] = ((uint64_t)code << 32) | (uint64_t)t;
}

// Points in key order (padding: copies of the last real point) and their
// original indices.
__global__ void k_probe_order(const uint64_t* __restrict__ keys, const double4* __restrict__ pts, int64_t npts,
                              int64_t npad, double4* __restrict__ spts, int32_t* __restrict__ order)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npad) return;
    const int64_t s = t < npts ? (int64_t)(keys[t] & 0xffffffffull) : (int64_t)(keys[npts - 1] & 0xffffffffull);
    spts[t] = pts[s];
    order[t] = (int32_t)s;
}

// field[order[t]] = {E_x, E_y, E_z} complex (interleaved), rho[order[t]]
// complex: the sum of the splits of sorted point t < npts.
__global__ void k_probe_sum(const double* __restrict__ part, int nsplit, int64_t npad, int64_t npts,
                            const int32_t* __restrict__ order, double* __restrict__ field, double* __restrict__ rho)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < nsplit; ++s)
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] += part[((size_t)s * npad + t) * 8 + c];
    const int64_t o = order[t];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        field[(size_t)o * 6 + 2 * a] = v[a];
        field[(size_t)o * 6 + 2 * a + 1] = v[3 + a];
    }
    rho[(size_t)o * 2] = v[6];
    rho[(size_t)o * 2 + 1] = v[7];
}

int64_t pow2_at_least(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

void probe_sources(const Geometry& g, const double2* x, int ldx, int col, double* src, hipStream_t st)
{
    if (g.model == 0)
        hipLaunchKernelGGL(k_probe_src<2>, dim3((unsigned)((g.np + 255) / 256)), dim3(256), 0, st, x, ldx, col, g.n,
                           g.np, src);
    else
        hipLaunchKernelGGL(k_probe_src<8>, dim3((unsigned)((g.np + 255) / 256)), dim3(256), 0, st, x, ldx, col, g.n,
                           g.np, src);
}

size_t probe_part_doubles(const Geometry& g, int64_t npts)
{
    const int64_t npad = (npts + 255) / 256 * 256;
    return (size_t)probe_splits(npad, g.np) * npad * 8;
}

size_t probe_order_bytes(int64_t npts)
{
    const int64_t npad = (npts + 255) / 256 * 256;
    return (size_t)pow2_at_least(npad) * sizeof(uint64_t) + (size_t)npad * (sizeof(double4) + sizeof(int32_t));
}

void probe_field(const Geometry& g, const double* src, const double4* pts, int64_t npts, const double lo[3],
                 const double hi[3], void* order, double* part, double* field, double* rho, hipStream_t st)
{
    const int64_t npad = (npts + 255) / 256 * 256;
    const int64_t npow = pow2_at_least(npad);
    uint64_t* keys = static_cast<uint64_t*>(order);
    double4* spts = reinterpret_cast<double4*>(keys + npow);
    int32_t* perm = reinterpret_cast<int32_t*>(spts + npad);
    const double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    const double sc = ext > 0 ? 1023.0 / ext : 1.0;
    // sorting pays once the atoms are many (its ~log^2 npts launches against
    // the n_atoms-long loop of every point): 20k-atom sphere on a 128^3 grid
    // 50.5 -> 46.5 ms, 1122-atom dimer on 160k points 1.22 -> 1.55 ms
    const int morton = g.n >= 4096 ? 1 : 0;
    hipLaunchKernelGGL(k_probe_keys, dim3((unsigned)((npow + 255) / 256)), dim3(256), 0, st, pts, npts, npow,
                       make_double3(lo[0], lo[1], lo[2]), sc, morton, keys);
    if (morton) sort_keys(keys, npow, st);
    hipLaunchKernelGGL(k_probe_order, dim3((unsigned)(npad / 256)), dim3(256), 0, st, (const uint64_t*)keys, pts, npts,
                       npad, spts, perm);
    ProbeConst k;
    k.rq = g.r_q;
    k.rmu = g.model ? g.r_mu : g.r_q;
    const double ipi32 = 1.0 / (M_PI * std::sqrt(M_PI));
    k.gq = ipi32 / (k.rq * k.rq * k.rq);
    k.gmu = ipi32 / (k.rmu * k.rmu * k.rmu);
    const double rn = PROBE_NEAR * std::max(k.rq, g.model ? k.rmu : 0.0) * 1.0001 + 1e-3;
    k.near2 = (float)(rn * rn);
    const int nsplit = probe_splits(npad, g.np);
    const dim3 grid((unsigned)(npad / 256), (unsigned)nsplit);
    if (g.model == 0)
        hipLaunchKernelGGL(k_probe<0>, grid, dim3(256), 0, st, g.xyz64, src, g.glo, g.ghi, g.np, (const double4*)spts,
                           part, npad, k);
    else
        hipLaunchKernelGGL(k_probe<1>, grid, dim3(256), 0, st, g.xyz64, src, g.glo, g.ghi, g.np, (const double4*)spts,
                           part, npad, k);
    hipLaunchKernelGGL(k_probe_sum, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, part, nsplit, npad, npts,
                       (const int32_t*)perm, field, rho);
}

}  // namespace px
