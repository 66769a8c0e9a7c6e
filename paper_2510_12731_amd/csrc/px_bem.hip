// BEM in the DPCM formulation (plasmonX paper, Section 2.3, Eq. bem-dpcm, the
// "approximate" F): the surface of the nanostructure is a mesh of tesserae
// (barycentre s_i, outward unit normal n_i, area A_i); the unknowns are the
// tessera charges q_i (Section 7: d = sum_i q_i s_i) and the system is
//     [ M - z(w) I ] q = -A E_n,    z(w) = 2 pi (eps2 + eps1) / (eps2 - eps1),
//     M_ij = A_i (s_i - s_j) . n_i / |s_i - s_j|^3   (i != j),
//     M_ii = 1.0694 sqrt(4 pi A_i) / (2 R),  R the radius enclosing the mesh.
// M is real and shared by every frequency, so the structure runs through the
// omegaFQ solver with the tesserae as its sites, the identity in place of
// Kbar, M in place of T and z(w) in place of z_q(w): the shared-Krylov phase
// (one Arnoldi process per polarization for every frequency), the blocked
// solver's true FP64 residuals and the observables are the same code.
//
// The M-apply is generated on the fly in FP64 (M is not symmetric and not
// stored): one thread per row i, the source tesserae read wave-uniform
// (through the scalar cache) in source splits, a deterministic split sum.
#include "px_internal.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace px {
namespace {

constexpr double BEM_SELF = 1.0694;   // self-patch factor of the approximate F diagonal
constexpr int BEM_ROWS = 256;         // rows per workgroup
constexpr int BEM_UNIT = 256;         // sources per split unit
constexpr int BEM_NC = 8;             // real columns per launch (wider blocks: several launches)

// 2 / sqrt(q) for q > 0: the hardware estimate and one Newton step (the caller
// applies the factor 1/2, cubed, to its sums).
__device__ __forceinline__ double rsqrt2_pos(double q)
{
    const double y = __builtin_amdgcn_rsq(q);
    return y * fma(-q, y * y, 3.0);
}

// Split y of row block x: part[y][i][c] = A_i sum_j (s_i - s_j).n_i / r^3 X[j][c0 + c]
// over the source units y, y + nsplit, ... (the self pair excluded), plus the
// diagonal M_ii X[i][c0 + c] in split 0.  s, na: [np] (x, y, z, -) and
// (n_x, n_y, n_z, A); ghost tesserae have A = 0 and zero columns of X.
template <int NC>
__global__ __launch_bounds__(BEM_ROWS) void k_bem_apply(const double4* __restrict__ s, const double4* __restrict__ na,
                                                      const double* __restrict__ X, int ldx, int c0,
                                                      double* __restrict__ part, int np, double inv_2r,
                                                      const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int i = blockIdx.x * BEM_ROWS + threadIdx.x;
    const double4 si = s[i], ni = na[i];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const int nunit = np / BEM_UNIT;
    const int row_unit = (blockIdx.x * BEM_ROWS) / BEM_UNIT;
    for (int u = blockIdx.y; u < nunit; u += gridDim.y) {
        const int j0 = u * BEM_UNIT;
        const bool self = u == row_unit;
#pragma unroll 4
        for (int jj = 0; jj < BEM_UNIT; ++jj) {
            const int j = j0 + jj;
            const double4 sj = s[j];
            const double dx = si.x - sj.x, dy = si.y - sj.y, dz = si.z - sj.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double dn = fma(dx, ni.x, fma(dy, ni.y, dz * ni.z));
            const double y = rsqrt2_pos(self && j == i ? 1.0 : r2);
            double t = dn * (y * y * y);
            if (self && j == i) t = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = fma(t, X[(size_t)j * ldx + c0 + c], acc[c]);
        }
    }
    // (2 / r)^3 = 8 / r^3: the factor 1/8, the row's area, and the diagonal once
    const double w = 0.125 * ni.w;
    double* out = part + (size_t)blockIdx.y * np * NC + (size_t)i * NC;
    const double mii = BEM_SELF * sqrt(4.0 * M_PI * ni.w) * inv_2r;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double v = w * acc[c];
        if (blockIdx.y == 0) v = fma(mii, X[(size_t)i * ldx + c0 + c], v);
        out[c] = v;
    }
}

// Y[i][c0 + c] = sum over the splits of part[k][i][c] (c < nc), in a fixed order.
__global__ void k_bem_sum(const double* __restrict__ part, int nsplit, int np, int nc_part, int nc, double* __restrict__ Y,
                          int ldy, int c0, const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)np * nc) return;
    const int i = (int)(t / nc), c = (int)(t % nc);
    const size_t len = (size_t)np * nc_part;
    const size_t o = (size_t)i * nc_part + c;
    double s0 = 0.0, s1 = 0.0;
    int k = 0;
    for (; k + 2 <= nsplit; k += 2) {
        s0 += part[(size_t)k * len + o];
        s1 += part[(size_t)(k + 1) * len + o];
    }
    if (k < nsplit) s0 += part[(size_t)k * len + o];
    Y[(size_t)i * ldy + c0 + c] = s0 + s1;
}

// b[i][c] = -A_i E0 n_i,l for column c of polarization l = col_pol[c].
__global__ void k_bem_rhs(const double4* __restrict__ na, const int32_t* __restrict__ col_pol, double e0,
                          double2* __restrict__ b, int64_t n, int64_t np, int ncol, int ldb)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= np || c >= ldb) return;
    double v = 0.0;
    if (i < n && c < ncol) {
        const double4 a = na[i];
        const int l = col_pol[c];
        const double nl = l == 0 ? a.x : (l == 1 ? a.y : a.z);
        v = -a.w * e0 * nl;
    }
    b[(size_t)i * ldb + c] = make_double2(v, 0.0);
}

}  // namespace

int bem_splits(const Geometry& g)
{
    static const int ncu = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            return v;
        return 256;
    }();
    const int nunit = (int)(g.np / BEM_UNIT);
    const int rb = (int)(g.np / BEM_ROWS);
    int want = (32 * ncu + rb - 1) / rb;
    want = std::max(1, std::min(want, nunit));
    const int ups = (nunit + want - 1) / want;
    return (nunit + ups - 1) / ups;
}

size_t bem_scratch_bytes(const Geometry& g) { return (size_t)bem_splits(g) * g.np * BEM_NC * sizeof(double); }

void bem_apply_f64(const Geometry& g, const double* X, double* Y, int ldx, int ncols, hipStream_t st, double* scratch,
                   const int32_t* stop, const hipEvent_t* ev)
{
    const int np = (int)g.np;
    const int nsplit = bem_splits(g);
    const dim3 grid((unsigned)(np / BEM_ROWS), (unsigned)nsplit);
    const double inv_2r = 1.0 / (2.0 * g.bem_r);
    hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
    for (int c0 = 0; c0 < ncols; c0 += BEM_NC) {
        const int nc = std::min(BEM_NC, ncols - c0);
        const bool first = c0 == 0, last = c0 + nc >= ncols;
#define PX_BEM(NC)                                                                                                   \
    hipExtLaunchKernelGGL(k_bem_apply<NC>, grid, dim3(BEM_ROWS), 0, st, first ? e0 : nullptr, nullptr, 0,           \
                          (const double4*)g.xyz64, (const double4*)g.bem_na, X, ldx, c0, scratch, np, inv_2r, stop)
        switch (nc) {
        case 1: PX_BEM(1); break;
        case 2: PX_BEM(2); break;
        case 3: PX_BEM(3); break;
        case 4: PX_BEM(4); break;
        case 5: PX_BEM(5); break;
        case 6: PX_BEM(6); break;
        case 7: PX_BEM(7); break;
        default: PX_BEM(8); break;
        }
#undef PX_BEM
        const int64_t len = (int64_t)np * nc;
        hipExtLaunchKernelGGL(k_bem_sum, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, nullptr,
                              last ? e1 : nullptr, 0, (const double*)scratch, nsplit, np, nc, nc, Y, ldx, c0, stop);
    }
}

void bem_rhs(const Geometry& g, const int32_t* col_pol, double e0, double2* b, int ncol, int ldb, hipStream_t st)
{
    const dim3 grid((unsigned)((g.np + 3) / 4), (unsigned)((ldb + 63) / 64));
    hipLaunchKernelGGL(k_bem_rhs, grid, dim3(256), 0, st, (const double4*)g.bem_na, col_pol, e0, b, g.n, g.np, ncol,
                       ldb);
}

hipError_t build_bem_geometry(Geometry& g, const double* cen_bohr, const double* nrm, const double* area_bohr2,
                              double r_enc_bohr, hipStream_t st)
{
    const int64_t n = g.n, np = g.np;
    std::vector<double4> s((size_t)np), na((size_t)np);
    std::vector<float4> s32((size_t)np);
    for (int64_t i = 0; i < np; ++i) {
        if (i < n) {
            const double* p = cen_bohr + 3 * i;
            const double* v = nrm + 3 * i;
            const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            s[(size_t)i] = make_double4(p[0], p[1], p[2], 0.0);
            na[(size_t)i] = make_double4(v[0] / l, v[1] / l, v[2] / l, area_bohr2[i]);
        } else {
            // ghost tesserae: no area, on a line far outside the mesh
            s[(size_t)i] = make_double4(4.0 * r_enc_bohr + 50.0 * (double)(i - n + 1), 3.0 * r_enc_bohr, 0.0, 0.0);
            na[(size_t)i] = make_double4(0.0, 0.0, 1.0, 0.0);
        }
        s32[(size_t)i] = make_float4((float)s[(size_t)i].x, (float)s[(size_t)i].y, (float)s[(size_t)i].z, 0.0f);
    }
    // the identity in place of Kbar (CSR over the real tesserae)
    std::vector<int32_t> rp((size_t)n + 1), ci((size_t)std::max<int64_t>(n, 1));
    std::vector<double> cv((size_t)std::max<int64_t>(n, 1), 1.0);
    for (int64_t i = 0; i <= n; ++i) rp[(size_t)i] = (int32_t)i;
    for (int64_t i = 0; i < n; ++i) ci[(size_t)i] = (int32_t)i;
    hipError_t e;
#define PXCHK(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
    PXCHK(px::dev_malloc((void**)&g.xyz64, sizeof(double4) * np));
    PXCHK(px::dev_malloc((void**)&g.xyz32, sizeof(float4) * np));
    PXCHK(px::dev_malloc((void**)&g.bem_na, sizeof(double4) * np));
    PXCHK(px::dev_malloc((void**)&g.row_ptr, sizeof(int32_t) * (n + 1)));
    PXCHK(px::dev_malloc((void**)&g.col, sizeof(int32_t) * ci.size()));
    PXCHK(px::dev_malloc((void**)&g.val, sizeof(double) * cv.size()));
    PXCHK(hipMemcpyAsync(g.xyz64, s.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.xyz32, s32.data(), sizeof(float4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.bem_na, na.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.row_ptr, rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.col, ci.data(), sizeof(int32_t) * ci.size(), hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.val, cv.data(), sizeof(double) * cv.size(), hipMemcpyHostToDevice, st));
    PXCHK(hipStreamSynchronize(st));
#undef PXCHK
    g.nnz = n;
    g.bem = true;
    g.bem_r = r_enc_bohr;
    return hipSuccess;
}

}  // namespace px
