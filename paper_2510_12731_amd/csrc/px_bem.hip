// BEM (plasmonX paper, Section 2.3, the "approximate" F): the surface of the
// nanostructure is a mesh of tesserae (barycentre s_i, outward unit normal
// n_i, area A_i).
//
// DPCM (Eq. bem-dpcm), read for the tessera charges q_i (Section 7:
// d = sum_i q_i s_i):
//     [ M - z(w) I ] q = -A E_n,    z(w) = 2 pi (eps2 + eps1) / (eps2 - eps1),
//     M_ij = A_i (s_i - s_j) . n_i / |s_i - s_j|^3   (i != j),
//     M_ii = 1.0694 sqrt(4 pi A_i) / (2 R),  R the radius enclosing the mesh.
// IEFPCM (Eq. bem-iefpcm) with the unknown y = S A^-1 q, the potential the
// charges make at the barycentres:
//     [ F - z(w) I ] y = -(2 pi I + F) V,   z(w) = -2 pi (eps2 + eps1) / (eps2 - eps1),
//     F_ij = A_j (s_i - s_j) . n_j / |s_i - s_j|^3   (i != j),
//     F_ii = -1.0694 sqrt(4 pi A_i) / (2 R)   (the double layer's self patch),
//     V_i = -E0 (s_i - c)_l,  then q = (S A^-1)^-1 y with
//     (S A^-1)_ij = 1 / |s_i - s_j|,  (S A^-1)_ii = 1.0694 sqrt(4 pi / A_i),
// c the tesserae's area-weighted centroid (a constant in V would not drop
// out of the discrete equation).  S A^-1 is symmetric, so the dipole needs no
// charges: d_k = (s - c)_k . q = w_k . y with w_k = (S A^-1)^-1 (s - c)_k,
// three real solves per mesh.
// M and F are real and shared by every frequency, so the structure runs
// through the omegaFQ solver with the tesserae as its sites, the identity in
// place of Kbar, M or F in place of T and z(w) in place of z_q(w): the
// shared-Krylov phase (one block Arnoldi process over the polarizations, or
// one per polarization, for every frequency), the true FP64 residuals and
// the observables are the same code.
//
// The operators are generated on the fly in FP64 (M and F are not symmetric
// and not stored): one or two rows per thread, the source tesserae read
// wave-uniform (through the scalar cache) in source splits, a deterministic
// split sum.  The single-layer solves are Jacobi-preconditioned conjugate
// gradients with every scalar kept on the device.
#include "px_internal.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

namespace px {
namespace {

constexpr double BEM_SELF = 1.0694;   // self-patch factor of the approximate F diagonal
constexpr int BEM_ROWS = 256;         // rows per workgroup
constexpr int BEM_UNIT = 256;         // sources per split unit
constexpr int BEM_NC = 8;             // real columns per launch of a narrow block
constexpr int BEM_NC_WIDE = 16;       // per launch of a block wider than BEM_NC
// rows per thread of the apply: two for narrow launches, one for the wide
// launch (whose 16 accumulators per row already fill the registers)
constexpr int bem_rpt(int nc) { return nc <= BEM_NC ? 2 : 1; }
constexpr double kSingleLayerTol = 1e-12;   // the dipole weights' solve
constexpr int kSingleLayerMaxIter = 20000;

// 2 / sqrt(q) for q > 0: the hardware estimate and one Newton step (the caller
// applies the factor 1/2, cubed, to its sums).
__device__ __forceinline__ double rsqrt2_pos(double q)
{
    const double y = __builtin_amdgcn_rsq(q);
    return y * fma(-q, y * y, 3.0);
}

// Split y of row block x: part[y][i][c] = sum_j K_ij X[j][c0 + c] over the
// source units y, y + nsplit, ... (the self pair excluded), plus the diagonal
// K_ii X[i][c0 + c] in split 0, for K = M (MODE 0), F (MODE 1) or S A^-1
// (MODE 2).  A thread holds RPT rows (t, t + BEM_ROWS / RPT of the block), so
// every source's wave-uniform loads feed RPT rows.
//   pc [np]: positions relative to the mesh centre with |p|^2 in w, so that
//       r^2 = |p_i|^2 + |p_j|^2 - 2 p_i.p_j takes four instructions (its
//       rounding, a few units of FP64 rounding times |p|^2 / r^2, stays near
//       1e-12 of a term for the nearest tesserae of a 100k-tesserae sphere);
//   na [np]: (n, A); an [np]: (A n, A p.n) for the double layer, so that
//       A_j (s_i - s_j).n_j = p_i.(A_j n_j) - A_j p_j.n_j takes three.
// Ghost tesserae have A = 0: zero rows of all three, zero columns of F; the
// columns of X are zero on ghost rows (M and S A^-1 do not mask them), and
// S A^-1 has identity ghost rows.
template <int MODE, int NC, int RPT>
__global__ __launch_bounds__(BEM_ROWS / RPT) void k_bem_apply(const double4* __restrict__ pc,
                                                            const double4* __restrict__ na,
                                                            const double4* __restrict__ an,
                                                            const double* __restrict__ X, int ldx, int c0,
                                                            double* __restrict__ part, int np, double inv_2r,
                                                            const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int BT = BEM_ROWS / RPT;
    const int base = blockIdx.x * BEM_ROWS;
    // per row: -2 p_i, |p_i|^2; MODE 0: n_i and p_i.n_i; MODE 1: p_i
    double qx[RPT], qy[RPT], qz[RPT], qw[RPT], ux[RPT], uy[RPT], uz[RPT], uw[RPT];
    double acc[RPT][NC];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = base + threadIdx.x + r * BT;
        const double4 p = pc[i];
        qx[r] = -2.0 * p.x;
        qy[r] = -2.0 * p.y;
        qz[r] = -2.0 * p.z;
        qw[r] = p.w;
        if (MODE == 0) {
            const double4 n = na[i];
            ux[r] = n.x;
            uy[r] = n.y;
            uz[r] = n.z;
            uw[r] = fma(p.x, n.x, fma(p.y, n.y, p.z * n.z));
        } else {
            ux[r] = p.x;
            uy[r] = p.y;
            uz[r] = p.z;
            uw[r] = 0.0;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = 0.0;
    }
    const int nunit = np / BEM_UNIT;
    const int row_unit = base / BEM_UNIT;
    // one source j for every row of the thread; SELF: the unit holds the rows
    // themselves (the pair j == i is skipped), every other unit takes the
    // loop without that test
    auto pair = [&](int j, auto self_tag) {
        constexpr bool SELF = decltype(self_tag)::value;
        const double4 pj = pc[j];
        double xj[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) xj[c] = X[(size_t)j * ldx + c0 + c];
        double4 aj = make_double4(0.0, 0.0, 0.0, 0.0);
        if (MODE == 1) aj = an[j];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const double r2 = fma(qx[r], pj.x, fma(qy[r], pj.y, fma(qz[r], pj.z, qw[r]))) + pj.w;
            const bool diag = SELF && j == base + (int)threadIdx.x + r * BT;
            const double y = rsqrt2_pos(diag ? 1.0 : r2);
            double t;
            if (MODE == 0) t = fma(-pj.x, ux[r], fma(-pj.y, uy[r], fma(-pj.z, uz[r], uw[r]))) * (y * y * y);
            else if (MODE == 1) t = fma(ux[r], aj.x, fma(uy[r], aj.y, fma(uz[r], aj.z, -aj.w))) * (y * y * y);
            else t = y;
            if (diag) t = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[r][c] = fma(t, xj[c], acc[r][c]);
        }
    };
    for (int u = blockIdx.y; u < nunit; u += gridDim.y) {
        const int j0 = u * BEM_UNIT;
        if (u != row_unit) {
#pragma unroll 4
            for (int jj = 0; jj < BEM_UNIT; ++jj) pair(j0 + jj, std::false_type{});
        } else {
#pragma unroll 4
            for (int jj = 0; jj < BEM_UNIT; ++jj) pair(j0 + jj, std::true_type{});
        }
    }
    // 2 / r: the factor 1/2 (S A^-1), (2 / r)^3 = 8 / r^3: 1/8 (M, F); the
    // row's area (M) or ghost mask (F, S A^-1), and the diagonal once
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = base + threadIdx.x + r * BT;
        const double4 ni = na[i];
        const bool real_row = ni.w > 0.0;
        double w, kii;
        if (MODE == 0) {
            w = 0.125 * ni.w;
            kii = BEM_SELF * sqrt(4.0 * M_PI * ni.w) * inv_2r;
        } else if (MODE == 1) {
            w = real_row ? 0.125 : 0.0;
            kii = -BEM_SELF * sqrt(4.0 * M_PI * ni.w) * inv_2r;
        } else {
            w = real_row ? 0.5 : 0.0;
            kii = real_row ? BEM_SELF * sqrt(4.0 * M_PI / ni.w) : 1.0;
        }
        double* out = part + (size_t)blockIdx.y * np * NC + (size_t)i * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double v = w * acc[r][c];
            if (blockIdx.y == 0) v = fma(kii, X[(size_t)i * ldx + c0 + c], v);
            out[c] = v;
        }
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

// b[i][c] for column c of polarization l = col_pol[c]: -A_i E0 n_i,l (DPCM,
// rv = null) or E0 rv_i,l with rv = 2 pi s + F s (IEFPCM: -(2 pi I + F) V
// for V = -E0 s_l).
__global__ void k_bem_rhs(const double4* __restrict__ na, const double4* __restrict__ rv,
                          const int32_t* __restrict__ col_pol, double e0, double2* __restrict__ b, int64_t n,
                          int64_t np, int ncol, int ldb)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= np || c >= ldb) return;
    double v = 0.0;
    if (i < n && c < ncol) {
        const int l = col_pol[c];
        if (rv) {
            const double4 a = rv[i];
            v = e0 * (l == 0 ? a.x : (l == 1 ? a.y : a.z));
        } else {
            const double4 a = na[i];
            const double nl = l == 0 ? a.x : (l == 1 ? a.y : a.z);
            v = -a.w * e0 * nl;
        }
    }
    b[(size_t)i * ldb + c] = make_double2(v, 0.0);
}

// rv_i = 2 pi s_i + (F s)_i over the real tesserae, 0 for ghosts (fs holds F s).
__global__ void k_bem_ief_rv(const double4* __restrict__ s, const double4* __restrict__ na, double4* __restrict__ fs,
                             int64_t np)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const double4 p = s[i], f = fs[i];
    const double tp = 2.0 * M_PI;
    fs[i] = na[i].w > 0.0 ? make_double4(fma(tp, p.x, f.x), fma(tp, p.y, f.y), fma(tp, p.z, f.z), 0.0)
                          : make_double4(0.0, 0.0, 0.0, 0.0);
}

// ---- conjugate gradients on S A^-1 -----------------------------------------
// Vectors [np][nc] (nc <= CG_NC); per-column scalars on the device; the
// partial sums of each dot product over blocks of CG_ROWS rows are reduced
// in a fixed order, so the iteration is deterministic.
constexpr int CG_NC = 8;
constexpr int CG_ROWS = 256;

struct CgState {
    double rz[CG_NC], bb[CG_NC], rr[CG_NC], alpha[CG_NC], beta[CG_NC];
    int32_t active[CG_NC];
    int32_t n_active, breakdown;
};

__device__ __forceinline__ double jacobi_inv(double a)
{
    // 1 / (S A^-1)_ii for a real tessera, 1 for a ghost (identity row)
    return a > 0.0 ? 1.0 / (BEM_SELF * sqrt(4.0 * M_PI / a)) : 1.0;
}

// Sum of v over the CG_ROWS threads of the block; every thread gets it.
__device__ __forceinline__ double block_sum(double v, double* lds)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < CG_ROWS / 64; ++k) s += lds[k];
    return s;
}

// r = B - Q (Q = S A^-1 x, or null for x = 0), z = D^-1 r, p = z; partial
// sums of r.z and r.r per column into part[block][2][CG_NC]; x = 0 when Q is
// null.
__global__ __launch_bounds__(CG_ROWS) void k_cg_start(const double* __restrict__ B, int ldb, const double* __restrict__ Q,
                                                    const double4* __restrict__ na, int64_t np, int nc,
                                                    double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ z, double* __restrict__ p,
                                                    double* __restrict__ part)
{
    __shared__ double lds[CG_ROWS / 64];
    const int64_t i = (int64_t)blockIdx.x * CG_ROWS + threadIdx.x;
    const double a = na[i].w, dinv = jacobi_inv(a);
    for (int c = 0; c < nc; ++c) {
        const size_t o = (size_t)i * nc + c;
        const double b = a > 0.0 ? B[(size_t)i * ldb + c] : 0.0;
        const double rv = Q ? b - Q[o] : b;
        if (!Q) x[o] = 0.0;
        const double zv = dinv * rv;
        r[o] = rv;
        z[o] = zv;
        p[o] = zv;
        const double s_rz = block_sum(rv * zv, lds);
        const double s_rr = block_sum(rv * rv, lds);
        if (threadIdx.x == 0) {
            part[((size_t)blockIdx.x * 2 + 0) * CG_NC + c] = s_rz;
            part[((size_t)blockIdx.x * 2 + 1) * CG_NC + c] = s_rr;
        }
    }
}

// Column c's total of part[.][k][c] over nblk blocks (fixed order), for
// every thread of the block.
__device__ double part_total(const double* __restrict__ part, int nblk, int k, int c, double* lds)
{
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += CG_ROWS) s += part[((size_t)b * 2 + k) * CG_NC + c];
    return block_sum(s, lds);
}

// After k_cg_start: rz, rr (and ||B||^2 on the first start), the active set.
__global__ __launch_bounds__(CG_ROWS) void k_cg_begin(const double* __restrict__ part, int nblk, int nc, double tol2,
                                                    int first, CgState* __restrict__ cs)
{
    __shared__ double lds[CG_ROWS / 64];
    int na = 0;
    for (int c = 0; c < nc; ++c) {
        const double rz = part_total(part, nblk, 0, c, lds);
        const double rr = part_total(part, nblk, 1, c, lds);
        if (threadIdx.x == 0) {
            if (first) cs->bb[c] = rr;
            cs->rz[c] = rz;
            cs->rr[c] = rr;
            cs->alpha[c] = cs->beta[c] = 0.0;
            const int act = cs->bb[c] > 0.0 && rr > tol2 * cs->bb[c];
            cs->active[c] = act;
            na += act;
        }
    }
    if (threadIdx.x == 0) {
        cs->n_active = na;
        if (first) cs->breakdown = 0;
    }
}

// partial sums of p.q per column into part[block][0][CG_NC]
__global__ __launch_bounds__(CG_ROWS) void k_cg_pq(const double* __restrict__ p, const double* __restrict__ q, int nc,
                                                 double* __restrict__ part)
{
    __shared__ double lds[CG_ROWS / 64];
    const int64_t i = (int64_t)blockIdx.x * CG_ROWS + threadIdx.x;
    for (int c = 0; c < nc; ++c) {
        const size_t o = (size_t)i * nc + c;
        const double s = block_sum(p[o] * q[o], lds);
        if (threadIdx.x == 0) part[((size_t)blockIdx.x * 2) * CG_NC + c] = s;
    }
}

// alpha = r.z / p.q for the active columns (0 for the others); a
// non-positive p.q on an active column flags a breakdown.
__global__ __launch_bounds__(CG_ROWS) void k_cg_alpha(const double* __restrict__ part, int nblk, int nc,
                                                    CgState* __restrict__ cs)
{
    __shared__ double lds[CG_ROWS / 64];
    for (int c = 0; c < nc; ++c) {
        const double pq = part_total(part, nblk, 0, c, lds);
        if (threadIdx.x == 0) {
            double a = 0.0;
            if (cs->active[c]) {
                if (pq > 0.0) a = cs->rz[c] / pq;
                else cs->breakdown = 1;
            }
            cs->alpha[c] = a;
        }
    }
}

// x += alpha p, r -= alpha q, z = D^-1 r; partial sums of r.z and r.r.
__global__ __launch_bounds__(CG_ROWS) void k_cg_update(double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ z, const double* __restrict__ p,
                                                     const double* __restrict__ q, const double4* __restrict__ na,
                                                     int nc, const CgState* __restrict__ cs,
                                                     double* __restrict__ part)
{
    __shared__ double lds[CG_ROWS / 64];
    const int64_t i = (int64_t)blockIdx.x * CG_ROWS + threadIdx.x;
    const double dinv = jacobi_inv(na[i].w);
    for (int c = 0; c < nc; ++c) {
        const size_t o = (size_t)i * nc + c;
        const double a = cs->alpha[c];
        x[o] = fma(a, p[o], x[o]);
        const double rv = fma(-a, q[o], r[o]);
        const double zv = dinv * rv;
        r[o] = rv;
        z[o] = zv;
        const double s_rz = block_sum(rv * zv, lds);
        const double s_rr = block_sum(rv * rv, lds);
        if (threadIdx.x == 0) {
            part[((size_t)blockIdx.x * 2 + 0) * CG_NC + c] = s_rz;
            part[((size_t)blockIdx.x * 2 + 1) * CG_NC + c] = s_rr;
        }
    }
}

// beta = new r.z / old r.z; columns whose ||r|| <= tol ||B|| leave the
// active set (alpha = beta = 0 from then on).
__global__ __launch_bounds__(CG_ROWS) void k_cg_beta(const double* __restrict__ part, int nblk, int nc, double tol2,
                                                   CgState* __restrict__ cs)
{
    __shared__ double lds[CG_ROWS / 64];
    int na = 0;
    for (int c = 0; c < nc; ++c) {
        const double rz = part_total(part, nblk, 0, c, lds);
        const double rr = part_total(part, nblk, 1, c, lds);
        if (threadIdx.x == 0) {
            double b = 0.0;
            if (cs->active[c]) {
                cs->rr[c] = rr;
                b = rz / cs->rz[c];
                cs->rz[c] = rz;
                if (!(rr > tol2 * cs->bb[c])) {
                    cs->active[c] = 0;
                    b = 0.0;
                }
            }
            cs->beta[c] = b;
            na += cs->active[c];
        }
    }
    if (threadIdx.x == 0) cs->n_active = na;
}

// p = z + beta p
__global__ __launch_bounds__(CG_ROWS) void k_cg_dir(const double* __restrict__ z, double* __restrict__ p, int nc,
                                                  const CgState* __restrict__ cs)
{
    const int64_t i = (int64_t)blockIdx.x * CG_ROWS + threadIdx.x;
    for (int c = 0; c < nc; ++c) {
        const size_t o = (size_t)i * nc + c;
        p[o] = fma(cs->beta[c], p[o], z[o]);
    }
}

// w[i] = (w3[i][0], w3[i][1], w3[i][2], 0)
__global__ void k_bem_pack_w(const double* __restrict__ w3, double4* __restrict__ w, int64_t np)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    w[i] = make_double4(w3[3 * i], w3[3 * i + 1], w3[3 * i + 2], 0.0);
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

size_t bem_scratch_bytes(const Geometry& g, int ncols)
{
    return (size_t)bem_splits(g) * g.np * (ncols > BEM_NC ? BEM_NC_WIDE : BEM_NC) * sizeof(double);
}

namespace {

template <int MODE>
void bem_apply_mode(const Geometry& g, const double* X, double* Y, int ldx, int ncols, hipStream_t st,
                    double* scratch, const int32_t* stop, const hipEvent_t* ev)
{
    const int np = (int)g.np;
    const int nsplit = bem_splits(g);
    const dim3 grid((unsigned)(np / BEM_ROWS), (unsigned)nsplit);
    const double inv_2r = 1.0 / (2.0 * g.bem_r);
    hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
    for (int c0 = 0; c0 < ncols;) {
        const int nc = ncols - c0 >= BEM_NC_WIDE ? BEM_NC_WIDE : std::min(BEM_NC, ncols - c0);
        const bool first = c0 == 0, last = c0 + nc >= ncols;
#define PX_BEM(NC)                                                                                                   \
    hipExtLaunchKernelGGL((k_bem_apply<MODE, NC, bem_rpt(NC)>), grid, dim3(BEM_ROWS / bem_rpt(NC)), 0, st,         \
                          first ? e0 : nullptr, nullptr, 0, (const double4*)g.xyzc, (const double4*)g.bem_na,        \
                          (const double4*)g.bem_an, X, ldx, c0, scratch, np, inv_2r, stop)
        switch (nc) {
        case 1: PX_BEM(1); break;
        case 2: PX_BEM(2); break;
        case 3: PX_BEM(3); break;
        case 4: PX_BEM(4); break;
        case 5: PX_BEM(5); break;
        case 6: PX_BEM(6); break;
        case 7: PX_BEM(7); break;
        case 8: PX_BEM(8); break;
        default: PX_BEM(16); break;
        }
#undef PX_BEM
        const int64_t len = (int64_t)np * nc;
        hipExtLaunchKernelGGL(k_bem_sum, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, nullptr,
                              last ? e1 : nullptr, 0, (const double*)scratch, nsplit, np, nc, nc, Y, ldx, c0, stop);
        c0 += nc;
    }
}

}  // namespace

void bem_apply_f64(const Geometry& g, const double* X, double* Y, int ldx, int ncols, hipStream_t st, double* scratch,
                   const int32_t* stop, const hipEvent_t* ev)
{
    if (g.bem_ief) bem_apply_mode<1>(g, X, Y, ldx, ncols, st, scratch, stop, ev);
    else bem_apply_mode<0>(g, X, Y, ldx, ncols, st, scratch, stop, ev);
}

void bem_rhs(const Geometry& g, const int32_t* col_pol, double e0, double2* b, int ncol, int ldb, hipStream_t st)
{
    const dim3 grid((unsigned)((g.np + 3) / 4), (unsigned)((ldb + 63) / 64));
    hipLaunchKernelGGL(k_bem_rhs, grid, dim3(256), 0, st, (const double4*)g.bem_na,
                       (const double4*)(g.bem_ief ? g.bem_rv : nullptr), col_pol, e0, b, g.n, g.np, ncol, ldb);
}

hipError_t bem_single_layer_solve(const Geometry& g, const double* B, int ldb, int nc, double* X, double tol,
                                  int max_iter, hipStream_t st, int* status, int* iters, double* relres)
{
    *status = 1;
    if (nc < 1 || nc > CG_NC || g.np % CG_ROWS != 0) return hipErrorInvalidValue;
    const int64_t np = g.np;
    const int nblk = (int)(np / CG_ROWS);
    const size_t vec = (size_t)np * nc;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *part = nullptr, *scr = nullptr;
    CgState* cs = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        for (void* v : {(void*)r, (void*)z, (void*)p, (void*)q, (void*)part, (void*)scr, (void*)cs}) px::dev_free(v);
    };
#define PXCG(x)            \
    do {                   \
        e = (x);           \
        if (e != hipSuccess) { \
            cleanup();     \
            return e;      \
        }                  \
    } while (0)
    PXCG(px::dev_malloc((void**)&r, sizeof(double) * vec));
    PXCG(px::dev_malloc((void**)&z, sizeof(double) * vec));
    PXCG(px::dev_malloc((void**)&p, sizeof(double) * vec));
    PXCG(px::dev_malloc((void**)&q, sizeof(double) * vec));
    PXCG(px::dev_malloc((void**)&part, sizeof(double) * nblk * 2 * CG_NC));
    PXCG(px::dev_malloc((void**)&scr, bem_scratch_bytes(g, nc)));
    PXCG(px::dev_malloc((void**)&cs, sizeof(CgState)));
    const double4* na = (const double4*)g.bem_na;
    const double tol2 = tol * tol;
    const dim3 grid((unsigned)nblk), blk(CG_ROWS);
    CgState h{};
    int it = 0;
    // a restart from the current x when the recursive residual has drifted
    // from the true one by more than 10 tol
    for (int start = 0; start < 3; ++start) {
        if (start == 0) {
            hipLaunchKernelGGL(k_cg_start, grid, blk, 0, st, B, ldb, (const double*)nullptr, na, np, nc, X, r, z, p,
                               part);
        } else {
            bem_apply_mode<2>(g, X, q, nc, nc, st, scr, nullptr, nullptr);
            hipLaunchKernelGGL(k_cg_start, grid, blk, 0, st, B, ldb, (const double*)q, na, np, nc, X, r, z, p, part);
        }
        hipLaunchKernelGGL(k_cg_begin, dim3(1), blk, 0, st, (const double*)part, nblk, nc, tol2, start == 0 ? 1 : 0,
                           cs);
        PXCG(hipGetLastError());
        PXCG(hipMemcpyAsync(&h, cs, sizeof(CgState), hipMemcpyDeviceToHost, st));
        PXCG(hipStreamSynchronize(st));
        if (start > 0 && h.n_active == 0) break;
        while (h.n_active > 0 && !h.breakdown && it < max_iter) {
            // a few iterations between looks at the active set
            for (int k = 0; k < 8 && it < max_iter; ++k, ++it) {
                bem_apply_mode<2>(g, p, q, nc, nc, st, scr, nullptr, nullptr);
                hipLaunchKernelGGL(k_cg_pq, grid, blk, 0, st, (const double*)p, (const double*)q, nc, part);
                hipLaunchKernelGGL(k_cg_alpha, dim3(1), blk, 0, st, (const double*)part, nblk, nc, cs);
                hipLaunchKernelGGL(k_cg_update, grid, blk, 0, st, X, r, z, (const double*)p, (const double*)q, na, nc,
                                   (const CgState*)cs, part);
                hipLaunchKernelGGL(k_cg_beta, dim3(1), blk, 0, st, (const double*)part, nblk, nc, tol2, cs);
                hipLaunchKernelGGL(k_cg_dir, grid, blk, 0, st, (const double*)z, p, nc, (const CgState*)cs);
            }
            PXCG(hipGetLastError());
            PXCG(hipMemcpyAsync(&h, cs, sizeof(CgState), hipMemcpyDeviceToHost, st));
            PXCG(hipStreamSynchronize(st));
        }
        if (h.breakdown || h.n_active > 0) break;
    }
    // the true residual of the final x
    bem_apply_mode<2>(g, X, q, nc, nc, st, scr, nullptr, nullptr);
    hipLaunchKernelGGL(k_cg_start, grid, blk, 0, st, B, ldb, (const double*)q, na, np, nc, X, r, z, p, part);
    hipLaunchKernelGGL(k_cg_begin, dim3(1), blk, 0, st, (const double*)part, nblk, nc, tol2, 0, cs);
    PXCG(hipGetLastError());
    PXCG(hipMemcpyAsync(&h, cs, sizeof(CgState), hipMemcpyDeviceToHost, st));
    PXCG(hipStreamSynchronize(st));
    double worst = 0.0;
    for (int c = 0; c < nc; ++c)
        if (h.bb[c] > 0.0) worst = std::max(worst, std::sqrt(h.rr[c] / h.bb[c]));
    *status = h.breakdown ? 2 : (worst <= 10.0 * tol ? 0 : 1);
    if (iters) *iters = it;
    if (relres) *relres = worst;
    cleanup();
#undef PXCG
    return hipSuccess;
}

hipError_t build_bem_geometry(Geometry& g, const double* cen_bohr, const double* nrm, const double* area_bohr2,
                              double r_enc_bohr, bool ief, hipStream_t st, int* status)
{
    *status = 0;
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
    // the kernels' source data: positions relative to the centre of the
    // tesserae's bounding box with |p|^2 in w, and (A n, A p.n)
    double lo[3] = {s[0].x, s[0].y, s[0].z}, hi[3] = {s[0].x, s[0].y, s[0].z};
    for (int64_t i = 1; i < n; ++i) {
        const double v[3] = {s[(size_t)i].x, s[(size_t)i].y, s[(size_t)i].z};
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], v[k]);
            hi[k] = std::max(hi[k], v[k]);
        }
    }
    const double cx = 0.5 * (lo[0] + hi[0]), cy = 0.5 * (lo[1] + hi[1]), cz = 0.5 * (lo[2] + hi[2]);
    std::vector<double4> pcv((size_t)np), anv((size_t)np);
    for (int64_t i = 0; i < np; ++i) {
        const double x = s[(size_t)i].x - cx, y = s[(size_t)i].y - cy, z = s[(size_t)i].z - cz;
        pcv[(size_t)i] = make_double4(x, y, z, x * x + y * y + z * z);
        const double4 a = na[(size_t)i];
        anv[(size_t)i] = make_double4(a.w * a.x, a.w * a.y, a.w * a.z, a.w * (x * a.x + y * a.y + z * a.z));
    }
    g.cx = cx;
    g.cy = cy;
    g.cz = cz;
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
    PXCHK(px::dev_malloc((void**)&g.xyzc, sizeof(double4) * np));
    PXCHK(px::dev_malloc((void**)&g.bem_an, sizeof(double4) * np));
    PXCHK(px::dev_malloc((void**)&g.row_ptr, sizeof(int32_t) * (n + 1)));
    PXCHK(px::dev_malloc((void**)&g.col, sizeof(int32_t) * ci.size()));
    PXCHK(px::dev_malloc((void**)&g.val, sizeof(double) * cv.size()));
    PXCHK(hipMemcpyAsync(g.xyz64, s.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.xyz32, s32.data(), sizeof(float4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.bem_na, na.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.xyzc, pcv.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.bem_an, anv.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.row_ptr, rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.col, ci.data(), sizeof(int32_t) * ci.size(), hipMemcpyHostToDevice, st));
    PXCHK(hipMemcpyAsync(g.val, cv.data(), sizeof(double) * cv.size(), hipMemcpyHostToDevice, st));
    PXCHK(hipStreamSynchronize(st));
    g.nnz = n;
    g.bem = true;
    g.bem_r = r_enc_bohr;
    // positions relative to the tesserae's area-weighted centroid c: the
    // dipole's origin (the discrete charges are neutral only up to the
    // discretization), and for IEFPCM the zero of the applied field's
    // potential V (a constant in V does not drop out of the discrete equation)
    double cw = 0.0, cc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        const double a = area_bohr2[i];
        cw += a;
        for (int k = 0; k < 3; ++k) cc[k] += a * cen_bohr[3 * i + k];
    }
    for (int k = 0; k < 3; ++k) cc[k] /= cw;
    std::vector<double4> sc((size_t)np);
    for (int64_t i = 0; i < np; ++i)
        sc[(size_t)i] = i < n ? make_double4(s[(size_t)i].x - cc[0], s[(size_t)i].y - cc[1], s[(size_t)i].z - cc[2], 0.0)
                              : make_double4(0.0, 0.0, 0.0, 0.0);
    PXCHK(px::dev_malloc((void**)&g.bem_w, sizeof(double4) * np));
    if (!ief) {
        // DPCM's dipole weights: the centred positions (d_k = w_k . q)
        PXCHK(hipMemcpyAsync(g.bem_w, sc.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st));
        PXCHK(hipStreamSynchronize(st));
        return hipSuccess;
    }
    // IEFPCM, with u = s - c: rv = 2 pi u + F u, then the dipole weights
    // w = (S A^-1)^-1 u
    g.bem_ief = true;
    PXCHK(px::dev_malloc((void**)&g.bem_rv, sizeof(double4) * np));
    PXCHK(hipMemsetAsync(g.bem_rv, 0, sizeof(double4) * np, st));
    double *scr = nullptr, *w3 = nullptr;
    double4* scd = nullptr;
    e = px::dev_malloc((void**)&scr, bem_scratch_bytes(g, 3));
    if (e == hipSuccess) e = px::dev_malloc((void**)&w3, sizeof(double) * 3 * np);
    if (e == hipSuccess) e = px::dev_malloc((void**)&scd, sizeof(double4) * np);
    if (e == hipSuccess) e = hipMemcpyAsync(scd, sc.data(), sizeof(double4) * np, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        bem_apply_mode<1>(g, (const double*)scd, (double*)g.bem_rv, 4, 3, st, scr, nullptr, nullptr);
        hipLaunchKernelGGL(k_bem_ief_rv, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, (const double4*)scd,
                           (const double4*)g.bem_na, g.bem_rv, np);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = bem_single_layer_solve(g, (const double*)scd, 4, 3, w3, kSingleLayerTol, kSingleLayerMaxIter, st, status,
                                   nullptr, nullptr);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_bem_pack_w, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, (const double*)w3,
                           g.bem_w, np);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    px::dev_free(scr);
    px::dev_free(w3);
    px::dev_free(scd);
#undef PXCHK
    return e;
}

}  // namespace px
