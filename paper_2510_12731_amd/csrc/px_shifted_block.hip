// Shared-Krylov solve over a block of polarizations: one block Arnoldi
// process for the R = npol right-hand sides of a one-material omegaFQ
// structure.
//
// Eq. (wfq-system) for column (omega_w, l) reads (M - z_w I) q = b_l with
// M = Kbar T real and b_l real and the same at every frequency.  The block
// Krylov space of B = [b_0 .. b_{R-1}] is shift-invariant like the single
// ones and after k steps holds each polarization's own k-dimensional space,
// so every pair minimises its residual over all kR directions (fewer steps
// than one process per polarization for the same tolerance; each step is
// still one T-apply of R vectors).  With B = V_0 rho_0 and
// M V_k = V_{k+1} Hbar_k, Hbar block upper Hessenberg with R x R blocks whose
// subdiagonal blocks are upper triangular, pair (w, l) takes
// y = argmin |rho_0 e_l - (Hbar - z_w I~) y| (unrestarted GMRES, Section 6):
// one banded QR per frequency (R rotations per column) serves its R
// right-hand sides.
//
// Orthogonalisation: delayed block CGS2.  Step k holds U, the candidate block
// for V_k projected once against V_{<k} in step k-1, and Wt = M U.  One dot
// pass gives S_j = V_j^T U, C_j = V_j^T Wt (j < k), U^T U and U^T Wt; then
// rho = chol(U^T U - sum S_j^T S_j) (upper), V_k = (U - V S) rho^-1, block
// column k-1 of Hbar gains S (block rows < k) and rho (block row k); with
// Ck = rho^-T (U^T Wt - S^T C) and T = Hbar_{(k+1) x k} S, the first-pass
// column k is h_j = (C_j - T_j) rho^-1, h_k = (Ck - T_k) rho^-1, and the next
// candidate U' = M V_k - V_{<=k} h = (Wt - V_{<k} C - V_k Ck) rho^-1, written
// from U, Wt and V_{<k} by one update pass.  A column whose projected norm
// falls below 1e-12 of its norm before the projections is deflated: its
// pivot is taken as zero and its basis vector stays zero.
//
// Layout: the block's R vectors are interleaved, V[k][row][a], so the T-apply
// reads one block per pass over the atom pairs.  Hbar is dense row-major,
// Hb[row * ldh + col] with ldh = kcap R.  Pairs p = w R + l (the solver's
// column index); per frequency w the rotations of column K, rc/rs[(K R + i)
// NW + w] (i < R, the rotation of rows K and K + 1 + i), and the rotated
// right-hand sides g[(row NW + w) R + l].
#include "px_internal.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

namespace px {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// v from another lane by the data-parallel-primitive control CTRL (rows not
// in ROWMASK get 0), both 32-bit halves moved by VALU moves (no LDS).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_take(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum of v over the 64 lanes, returned to every lane (for the coefficient
// kernel's few sums: 13.8 against 15.3 us per launch; the dot pass's block
// sums of 18 values are faster with shuffles, 51 against 61 us): pairs and quads
// (quad permutations), half rows and rows (mirrors), then rows 0+1 and 2+3
// (broadcast of lane 15 into rows 1 and 3) and all four (lane 31 into rows
// 2 and 3): lane 63 holds the total, read as a scalar.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_take<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_take<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_take<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_take<0x140, 0xF>(v);   // row_mirror
    v += dpp_take<0x142, 0xA>(v);   // row_bcast:15
    v += dpp_take<0x143, 0xC>(v);   // row_bcast:31
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Block sum of W values over 256 threads in a fixed order; thread 0 returns it.
template <int W>
__device__ __forceinline__ void block_sum(double (&v)[W], double (*lds)[W])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int c = 0; c < W; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < W; ++c) lds[wave][c] = v[c];
    __syncthreads();
    if (tid == 0)
#pragma unroll
        for (int c = 0; c < W; ++c) v[c] = (lds[0][c] + lds[1][c]) + (lds[2][c] + lds[3][c]);
}

// (a, b) <- (c a + s b, -conj(s) a + c b).
__device__ __forceinline__ void rot(double c, double2 s, double2& a, double2& b)
{
    const double2 sb = cmul(s, b);
    const double2 sa = cmul(make_double2(s.x, -s.y), a);
    const double2 na = make_double2(c * a.x + sb.x, c * a.y + sb.y);
    b = make_double2(c * b.x - sa.x, c * b.y - sa.y);
    a = na;
}

// The rotation that zeroes b against a: c real, s complex, c a + s b = |(a, b)| a / |a|.
__device__ __forceinline__ void make_rot(double2 a, double2 b, double& c, double2& s)
{
    const double aa = sqrt(cabs2(a)), bb = sqrt(cabs2(b));
    if (bb == 0.0) {
        c = 1.0;
        s = make_double2(0.0, 0.0);
    } else if (aa == 0.0) {
        c = 0.0;
        s = make_double2(b.x / bb, -b.y / bb);
    } else {
        const double r = sqrt(aa * aa + bb * bb);
        c = aa / r;
        // (a / |a|) conj(b) / r
        const double2 u = make_double2(a.x / aa, a.y / aa);
        s = cmul(u, make_double2(b.x / r, -b.y / r));
    }
}

__device__ __forceinline__ size_t rpk(int l, int j) { return (size_t)l * (l + 1) / 2 + j; }

// Entry (row, col) of Hbar - z I~.
__device__ __forceinline__ double2 hsb(const double* __restrict__ Hb, int ldh, int row, int col, double2 z)
{
    const double h = Hb[(size_t)row * ldh + col];
    return row == col ? make_double2(h - z.x, -z.y) : make_double2(h, 0.0);
}

// Upper Cholesky factor of the R x R matrix X (row-major) with deflation: a
// pivot below 1e-12 of ref[i] (the column's squared norm before the
// projections) is taken as zero, and so is the rest of its row.
template <int R>
__device__ __forceinline__ void chol_defl(const double (&X)[R * R], const double (&ref)[R], double (&r)[R * R])
{
#pragma unroll
    for (int e = 0; e < R * R; ++e) r[e] = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        double d = X[i * R + i];
#pragma unroll
        for (int m = 0; m < i; ++m) d -= r[m * R + i] * r[m * R + i];
        if (!(d > 1e-12 * ref[i])) continue;
        const double p = sqrt(d);
        r[i * R + i] = p;
#pragma unroll
        for (int j = i + 1; j < R; ++j) {
            double v = X[i * R + j];
#pragma unroll
            for (int m = 0; m < i; ++m) v -= r[m * R + i] * r[m * R + j];
            r[i * R + j] = v / p;
        }
    }
}

// Inverse of an upper-triangular R x R matrix whose zero pivots (deflated
// columns) give zero rows and columns.
template <int R>
__device__ __forceinline__ void triu_inv(const double (&r)[R * R], double (&x)[R * R])
{
#pragma unroll
    for (int e = 0; e < R * R; ++e) x[e] = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (r[j * R + j] == 0.0) continue;
        x[j * R + j] = 1.0 / r[j * R + j];
#pragma unroll
        for (int i = j - 1; i >= 0; --i) {
            if (r[i * R + i] == 0.0) continue;
            double v = 0.0;
#pragma unroll
            for (int m = i + 1; m <= j; ++m) v += r[i * R + m] * x[m * R + j];
            x[i * R + j] = -v / r[i * R + i];
        }
    }
}

// c = a b (R x R, row-major)
template <int R>
__device__ __forceinline__ void mm(const double* a, const double* b, double* c)
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < R; ++m) v = fma(a[i * R + m], b[m * R + j], v);
            c[i * R + j] = v;
        }
}

}  // namespace

// u[row][c] = Re b[row][c] (the block B itself; step 0 normalises it).
template <int R>
__global__ void k_msb_init(const double2* __restrict__ b, int ldb, double* __restrict__ u, int64_t nup)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nup) return;
#pragma unroll
    for (int c = 0; c < R; ++c) u[(size_t)r * R + c] = b[(size_t)r * ldb + c].x;
}

// part[(j * nslab + slab)][.]: over the slab's rows, S_j[a][b] = sum x_j[row][a]
// u[row][b] at a R + b and C_j[a][b] (wt in place of u) at R^2 + a R + b, with
// x_j = V_j (j < k) or u (j = k).  A block takes MJB consecutive vectors.
constexpr int MJB = 1;

template <int R>
__global__ __launch_bounds__(256) void k_msb_dots(const double* __restrict__ V, int64_t vstride, int k,
                                                  const double* __restrict__ u, const double* __restrict__ wt,
                                                  double* __restrict__ part, int64_t nup, int64_t rows_per_slab,
                                                  const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int RR = R * R, W = 2 * RR;
    __shared__ double lds[4][MJB * W];
    const int j0 = blockIdx.y * MJB, slab = blockIdx.x, nslab = gridDim.x;
    const int nj = k + 1 - j0 < MJB ? k + 1 - j0 : MJB;
    const int64_t r0 = (int64_t)slab * rows_per_slab;
    const int64_t r1 = r0 + rows_per_slab < nup ? r0 + rows_per_slab : nup;
    double acc[MJB * W];
#pragma unroll
    for (int c = 0; c < MJB * W; ++c) acc[c] = 0.0;
    const double* xp[MJB];
#pragma unroll
    for (int jj = 0; jj < MJB; ++jj) {
        const int j = j0 + jj;
        xp[jj] = (jj < nj && j < k) ? V + (size_t)j * vstride : u;
    }
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        double uu[R], ww[R], xx[MJB][R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            uu[c] = u[(size_t)r * R + c];
            ww[c] = wt[(size_t)r * R + c];
        }
#pragma unroll
        for (int jj = 0; jj < MJB; ++jj)
#pragma unroll
            for (int c = 0; c < R; ++c) xx[jj][c] = xp[jj][(size_t)r * R + c];
#pragma unroll
        for (int jj = 0; jj < MJB; ++jj)
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = 0; b < R; ++b) {
                    acc[jj * W + a * R + b] = fma(xx[jj][a], uu[b], acc[jj * W + a * R + b]);
                    acc[jj * W + RR + a * R + b] = fma(xx[jj][a], ww[b], acc[jj * W + RR + a * R + b]);
                }
    }
    block_sum<MJB * W>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int jj = 0; jj < MJB; ++jj)
            if (jj < nj)
#pragma unroll
                for (int c = 0; c < W; ++c) part[((size_t)(j0 + jj) * nslab + slab) * W + c] = acc[jj * W + c];
}

// G[j][c] = sum over slabs of part[j][slab][c] (fixed order), W values per j.
template <int W>
__global__ void k_msb_reduce(const double* __restrict__ part, int nslab, int nvec, double* __restrict__ G,
                             const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nvec * W) return;
    const int j = t / W, c = t - j * W;
    double s = 0.0;
    for (int q = 0; q < nslab; ++q) s += part[((size_t)j * nslab + q) * W + c];
    G[t] = s;
}

// The coefficients of step k, one wave per block row j = 0..k of Hbar
// (CWPB waves per workgroup, which form sum S_i^T S_i and S_i^T C_i together):
// corrects block column k-1, writes the first-pass block column k (block rows
// 0..k), coefv_j = S_j rho^-1 and coefu_j = (C_j - S_j rho^-1 Ck) rho^-1 (j < k),
// scal = {rho^-1, -rho^-1 Ck rho^-1} and, at k = 0, rho0 = rho_0.
// fix_only: the last block column's correction alone.
constexpr int CWPB = 4;

template <int R>
__global__ __launch_bounds__(64 * CWPB) void k_msb_coef(const double* __restrict__ G, double* __restrict__ Hb,
                                                        int ldh, int k, int fix_only, double* __restrict__ coefv,
                                                        double* __restrict__ coefu, double* __restrict__ scal,
                                                        double* __restrict__ rho0,
                                                        const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int RR = R * R, W = 2 * RR;
    __shared__ double red[CWPB][2 * RR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = blockIdx.x * CWPB + wave;
    double ss[RR], sc[RR];
#pragma unroll
    for (int e = 0; e < RR; ++e) ss[e] = sc[e] = 0.0;
    for (int i = threadIdx.x; i < k; i += 64 * CWPB) {
        const double* Si = G + (size_t)i * W;
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b)
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    ss[a * R + b] = fma(Si[m * R + a], Si[m * R + b], ss[a * R + b]);
                    sc[a * R + b] = fma(Si[m * R + a], Si[RR + m * R + b], sc[a * R + b]);
                }
    }
#pragma unroll
    for (int e = 0; e < RR; ++e) {
        ss[e] = wave_sum(ss[e]);
        sc[e] = wave_sum(sc[e]);
    }
    if (lane == 0)
#pragma unroll
        for (int e = 0; e < RR; ++e) {
            red[wave][e] = ss[e];
            red[wave][RR + e] = sc[e];
        }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < RR; ++e) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < CWPB; ++q) {
            a += red[q][e];
            b += red[q][RR + e];
        }
        ss[e] = a;
        sc[e] = b;
    }
    if (j > k) return;
    const double* Gk = G + (size_t)k * W;
    double X[RR], ref[R], rho[RR], ri[RR], ck[RR];
#pragma unroll
    for (int e = 0; e < RR; ++e) X[e] = Gk[e] - ss[e];
#pragma unroll
    for (int a = 0; a < R; ++a) ref[a] = Gk[a * R + a];
    chol_defl<R>(X, ref, rho);
    triu_inv<R>(rho, ri);
    // Ck = rho^-T (U^T Wt - S^T C)
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < R; ++m) v = fma(ri[m * R + a], Gk[RR + m * R + b] - sc[m * R + b], v);
            ck[a * R + b] = v;
        }
    const double* Sj = G + (size_t)j * W;
    // block (j, k-1) corrected
    double hfix[RR];
#pragma unroll
    for (int e = 0; e < RR; ++e) hfix[e] = 0.0;
    if (k >= 1) {
        if (j < k) {
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = 0; b < R; ++b)
                    hfix[a * R + b] = Hb[(size_t)(j * R + a) * ldh + (k - 1) * R + b] + Sj[a * R + b];
        } else {
#pragma unroll
            for (int e = 0; e < RR; ++e) hfix[e] = rho[e];
        }
    }
    if (fix_only) {
        if (lane == 0 && k >= 1)
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = 0; b < R; ++b) Hb[(size_t)(j * R + a) * ldh + (k - 1) * R + b] = hfix[a * R + b];
        return;
    }
    // T_j = sum_{i >= j-1, i < k} H_{j,i} S_i with the corrected block column k-1
    double t[RR];
#pragma unroll
    for (int e = 0; e < RR; ++e) t[e] = 0.0;
    for (int i = (j > 0 ? j - 1 : 0) + lane; i < k; i += 64) {
        double h[RR];
        if (i == k - 1) {
#pragma unroll
            for (int e = 0; e < RR; ++e) h[e] = hfix[e];
        } else {
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = 0; b < R; ++b) h[a * R + b] = Hb[(size_t)(j * R + a) * ldh + i * R + b];
        }
        const double* Si = G + (size_t)i * W;
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b)
#pragma unroll
                for (int m = 0; m < R; ++m) t[a * R + b] = fma(h[a * R + m], Si[m * R + b], t[a * R + b]);
    }
#pragma unroll
    for (int e = 0; e < RR; ++e) t[e] = wave_sum(t[e]);
    if (lane != 0) return;
    if (k >= 1)
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b) Hb[(size_t)(j * R + a) * ldh + (k - 1) * R + b] = hfix[a * R + b];
    double d[RR], hk[RR];
#pragma unroll
    for (int e = 0; e < RR; ++e) d[e] = (j < k ? Sj[RR + e] : ck[e]) - t[e];
    mm<R>(d, ri, hk);
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) Hb[(size_t)(j * R + a) * ldh + k * R + b] = hk[a * R + b];
    double ckri[RR];
    mm<R>(ck, ri, ckri);
    if (j < k) {
        double cv[RR], cr[RR], tmp[RR];
        mm<R>(Sj, ri, cv);
        mm<R>(Sj + RR, ri, cr);
        mm<R>(cv, ckri, tmp);
#pragma unroll
        for (int e = 0; e < RR; ++e) {
            coefv[(size_t)j * RR + e] = cv[e];
            coefu[(size_t)j * RR + e] = cr[e] - tmp[e];
        }
    }
    if (j == 0) {
        double e2[RR];
        mm<R>(ri, ckri, e2);
#pragma unroll
        for (int e = 0; e < RR; ++e) {
            scal[e] = ri[e];
            scal[RR + e] = -e2[e];
        }
        if (k == 0)
#pragma unroll
            for (int e = 0; e < RR; ++e) rho0[e] = rho[e];
    }
}

// The finishing combination of one row: v_k = u rho^-1 - av and
// u' = wt rho^-1 + u E - au (E = scal[R^2..]).
template <int R>
__device__ __forceinline__ void msb_finish_row(int64_t r, const double (&av)[R], const double (&au)[R],
                                               const double* __restrict__ scal, double* __restrict__ u,
                                               const double* __restrict__ wt, double* __restrict__ vk)
{
    constexpr int RR = R * R;
    double uo[R], wo[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
        uo[a] = u[(size_t)r * R + a];
        wo[a] = wt[(size_t)r * R + a];
    }
#pragma unroll
    for (int b = 0; b < R; ++b) {
        double v = -av[b], w = -au[b];
#pragma unroll
        for (int a = 0; a < R; ++a) {
            v = fma(uo[a], scal[a * R + b], v);
            w = fma(wo[a], scal[a * R + b], w);
            w = fma(uo[a], scal[RR + a * R + b], w);
        }
        vk[(size_t)r * R + b] = v;
        u[(size_t)r * R + b] = w;
    }
}

// One pass over V_{<k}: av = V coefv, au = V coefu per row; the vectors are
// split over blockIdx.y, and with more than one split the sums go to part2
// for k_msb_finish (fixed order).
template <int R>
__global__ __launch_bounds__(256) void k_msb_update(const double* __restrict__ V, int64_t vstride, int k,
                                                    const double* __restrict__ coefv,
                                                    const double* __restrict__ coefu,
                                                    const double* __restrict__ scal, double* __restrict__ u,
                                                    const double* __restrict__ wt, double* __restrict__ vk,
                                                    double* __restrict__ part2, int64_t nup, int vecs_per_split,
                                                    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int RR = R * R;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nup) return;
    const int j0 = blockIdx.y * vecs_per_split;
    const int j1 = j0 + vecs_per_split < k ? j0 + vecs_per_split : k;
    double av[R], au[R];
#pragma unroll
    for (int c = 0; c < R; ++c) av[c] = au[c] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double* vj = V + (size_t)j * vstride + (size_t)r * R;
        const double* cv = coefv + (size_t)j * RR;
        const double* cu = coefu + (size_t)j * RR;
        double x[R];
#pragma unroll
        for (int a = 0; a < R; ++a) x[a] = vj[a];
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b) {
                av[b] = fma(x[a], cv[a * R + b], av[b]);
                au[b] = fma(x[a], cu[a * R + b], au[b]);
            }
    }
    if (gridDim.y == 1) {
        msb_finish_row<R>(r, av, au, scal, u, wt, vk);
    } else {
#pragma unroll
        for (int c = 0; c < R; ++c) {
            part2[((size_t)blockIdx.y * nup + r) * 2 * R + c] = av[c];
            part2[((size_t)blockIdx.y * nup + r) * 2 * R + R + c] = au[c];
        }
    }
}

template <int R>
__global__ void k_msb_finish(const double* __restrict__ part2, int nsplit, const double* __restrict__ scal,
                             double* __restrict__ u, const double* __restrict__ wt, double* __restrict__ vk,
                             int64_t nup, const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nup) return;
    double av[R], au[R];
#pragma unroll
    for (int c = 0; c < R; ++c) av[c] = au[c] = 0.0;
    for (int q = 0; q < nsplit; ++q)
#pragma unroll
        for (int c = 0; c < R; ++c) {
            av[c] += part2[((size_t)q * nup + r) * 2 * R + c];
            au[c] += part2[((size_t)q * nup + r) * 2 * R + R + c];
        }
    msb_finish_row<R>(r, av, au, scal, u, wt, vk);
}

// A batch of RFB columns' rotations and the fresh Hessenberg entries that
// enter the window of column l after each of them.
constexpr int RFB = 4;

template <int R>
struct RotBatchB {
    double c[RFB][R], h[RFB];
    double2 s[RFB][R];

    __device__ __forceinline__ void load(const double* __restrict__ rc, const double2* __restrict__ rs,
                                         const double* __restrict__ Hb, int ldh, int NW, int w, int l, int j0, int jn)
    {
#pragma unroll
        for (int u = 0; u < RFB; ++u) {
            const int j = j0 + u;
            if (j < jn) {
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    c[u][i] = rc[(size_t)(j * R + i) * NW + w];
                    s[u][i] = rs[(size_t)(j * R + i) * NW + w];
                }
                h[u] = Hb[(size_t)(j + R + 1) * ldh + l];
            }
        }
    }

    // columns j0 .. j0+RFB-1 (< jn) applied to the window a of column l; row j
    // of the factor goes to out[rpk(l, j)] (STORE)
    template <bool STORE>
    __device__ __forceinline__ void apply(double2 (&a)[R + 1], double2* __restrict__ out, int l, int j0, int jn,
                                          double2 zw) const
    {
#pragma unroll
        for (int u = 0; u < RFB; ++u) {
            const int j = j0 + u;
            if (j < jn) {
#pragma unroll
                for (int i = 0; i < R; ++i) rot(c[u][i], s[u][i], a[0], a[i + 1]);
                if (STORE) out[rpk(l, j)] = a[0];
#pragma unroll
                for (int m = 0; m < R; ++m) a[m] = a[m + 1];
                a[R] = j + R + 1 == l ? make_double2(h[u] - zw.x, -zw.y) : make_double2(h[u], 0.0);
            }
        }
    }
};

// ---- banded QR of every frequency's shifted block Hessenberg matrix --------
// Columns K0 .. K0+nc-1 (nc <= GBC) per launch.  Phase 1, one lane per
// (frequency, new column): the rotations of the columns before K0 are applied
// to the column through a window of R + 1 rows (rows j .. j+R while column
// j's R rotations are applied; row j is then final and a fresh row enters).
// Phase 2, one lane per frequency: each new column in turn takes the
// rotations of the batch's earlier columns and then its own R rotations,
// which zero its R subdiagonal entries against the diagonal; the same
// rotations act on the R right-hand sides, whose rows K+1 .. K+R then give
// the residual norms after K+1 columns.  A pair whose residual reaches its
// target is done with done[p] = K + 1 columns; the thread that finishes the
// last pair raises *stop.
constexpr int GBC = 12, LPW = 16;

template <int R>
__global__ __launch_bounds__(64) void k_msb_givens(const double* __restrict__ Hb, int ldh, int NW, int K0, int nc,
                                                   const double2* __restrict__ z, double* __restrict__ rc,
                                                   double2* __restrict__ rs, double2* __restrict__ g,
                                                   const double* __restrict__ rho0,
                                                   const double* __restrict__ target, int32_t* __restrict__ done,
                                                   double* __restrict__ resid, int32_t* __restrict__ ndone,
                                                   int32_t* __restrict__ stop)
{
    // (no early exit on *stop: another workgroup may raise it while this one
    // runs, and every thread must reach the barriers; once it is raised every
    // frequency is finished and skips below)
    constexpr int NR = GBC + R;
    __shared__ double2 win[4][GBC][R + 1];
    __shared__ double2 colv[4][NR];
    __shared__ double2 gl[4][NR][R];
    __shared__ double rcl[4][GBC][R];
    __shared__ double2 rsl[4][GBC][R];
    const int t = threadIdx.x, wl = t / LPW, q = t % LPW;
    const int w = blockIdx.x * (64 / LPW) + wl;
    bool live = w < NW;
    if (live) {
        bool all = true;
#pragma unroll
        for (int l = 0; l < R; ++l) all = all && done[w * R + l] != 0;
        live = !all;
    }
    const double2 zw = live ? z[(size_t)w * R] : make_double2(0.0, 0.0);
    // phase 1
    if (live && q < nc) {
        const int K = K0 + q;
        double2 a[R + 1];
#pragma unroll
        for (int m = 0; m <= R; ++m) a[m] = hsb(Hb, ldh, m, K, zw);
        // batches of RFB earlier columns (a double-buffered variant measured
        // 1.8x slower here)
        for (int j0 = 0; j0 < K0; j0 += RFB) {
            RotBatchB<R> b;
            b.load(rc, rs, Hb, ldh, NW, w, K, j0, K0);
            b.template apply<false>(a, nullptr, K, j0, K0, zw);
        }
#pragma unroll
        for (int m = 0; m <= R; ++m) win[wl][q][m] = a[m];
    }
    // the rotated right-hand sides of rows K0 .. K0 + nc + R - 1
    if (live && q < R) {
        const int l = q;
        for (int m = 0; m < nc + R; ++m) {
            const int row = K0 + m;
            double2 v = g[((size_t)row * NW + w) * R + l];
            if (K0 == 0 && row < R) v = make_double2(rho0[row * R + l], 0.0);
            gl[wl][m][l] = v;
        }
    }
    __syncthreads();
    if (live && q == 0) {
        int ndl = 0;
        bool dl[R];
#pragma unroll
        for (int l = 0; l < R; ++l) {
            dl[l] = done[w * R + l] != 0;
            ndl += dl[l] ? 1 : 0;
        }
        for (int qq = 0; qq < nc && ndl < R; ++qq) {
            const int K = K0 + qq;
            for (int m = 0; m <= qq + R; ++m)
                colv[wl][m] = m <= R ? win[wl][qq][m] : hsb(Hb, ldh, K0 + m, K, zw);
            for (int m = 0; m < qq; ++m)
#pragma unroll
                for (int i = 0; i < R; ++i) rot(rcl[wl][m][i], rsl[wl][m][i], colv[wl][m], colv[wl][m + i + 1]);
            double res2[R];
#pragma unroll
            for (int l = 0; l < R; ++l) res2[l] = 0.0;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                double c;
                double2 s;
                double2 a0 = colv[wl][qq], bi = colv[wl][qq + i + 1];
                make_rot(a0, bi, c, s);
                rot(c, s, a0, bi);
                colv[wl][qq] = a0;
                colv[wl][qq + i + 1] = bi;
                rcl[wl][qq][i] = c;
                rsl[wl][qq][i] = s;
                rc[(size_t)(K * R + i) * NW + w] = c;
                rs[(size_t)(K * R + i) * NW + w] = s;
#pragma unroll
                for (int l = 0; l < R; ++l) {
                    double2 ga = gl[wl][qq][l], gb = gl[wl][qq + i + 1][l];
                    rot(c, s, ga, gb);
                    gl[wl][qq][l] = ga;
                    gl[wl][qq + i + 1][l] = gb;
                }
            }
#pragma unroll
            for (int l = 0; l < R; ++l) {
#pragma unroll
                for (int i = 1; i <= R; ++i) res2[l] += cabs2(gl[wl][qq + i][l]);
                if (dl[l]) continue;
                const int p = w * R + l;
                const double res = sqrt(res2[l]);
                resid[p] = res;
                if (res <= target[p]) {
                    dl[l] = true;
                    ++ndl;
                    done[p] = K + 1;
                    if (atomicAdd(ndone, 1) + 1 == NW * R && stop) *stop = 1;
                }
            }
        }
    }
    __syncthreads();
    if (live && q < R) {
        const int l = q;
        for (int m = 0; m < nc + R; ++m) g[((size_t)(K0 + m) * NW + w) * R + l] = gl[wl][m][l];
    }
}

// Columns of every frequency's triangular factor, rebuilt by the same
// rotations: rst[w S + rpk(l, j)] = R_w[j][l] (S = rpk(kcols, 0), column l of
// frequency w contiguous).  Lanes take consecutive columns l of one frequency
// w = blockIdx.y (its rotations are loaded once per wave); columns past the
// frequency's last finished pair skip.
template <int R>
__global__ __launch_bounds__(64) void k_msb_rfactor(const double* __restrict__ Hb, int ldh, int NW, int kcols,
                                                    const double2* __restrict__ z, const double* __restrict__ rc,
                                                    const double2* __restrict__ rs, const int32_t* __restrict__ done,
                                                    double2* __restrict__ rst)
{
    const int w = blockIdx.y;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    int Kw = 0;
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int d = done[w * R + c];
        Kw = std::max(Kw, d ? d : kcols);
    }
    if (l >= Kw) return;
    double2* out = rst + (size_t)w * rpk(kcols, 0);
    const double2 zw = z[(size_t)w * R];
    double2 a[R + 1];
#pragma unroll
    for (int m = 0; m <= R; ++m) a[m] = hsb(Hb, ldh, m, l, zw);
    // batches of RFB earlier columns, the next batch's loads in flight while
    // the current one is applied
    RotBatchB<R> b0, b1;
    b0.load(rc, rs, Hb, ldh, NW, w, l, 0, l);
    for (int j0 = 0; j0 < l; j0 += 2 * RFB) {
        b1.load(rc, rs, Hb, ldh, NW, w, l, j0 + RFB, l);
        b0.template apply<true>(a, out, l, j0, l, zw);
        b0.load(rc, rs, Hb, ldh, NW, w, l, j0 + 2 * RFB, l);
        b1.template apply<true>(a, out, l, j0 + RFB, l, zw);
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
        rot(rc[(size_t)(l * R + i) * NW + w], rs[(size_t)(l * R + i) * NW + w], a[0], a[i + 1]);
    out[rpk(l, l)] = a[0];
}

// y_p = R_w^-1 g_p for the R pairs p = w R + l of frequency w = blockIdx.x
// together, each over its own K_p columns (done[p], else kcols <= BST MBS):
// column-oriented back substitution, thread t holding rows t + BST m of the R
// right-hand sides in registers; column c of R_w is read once (contiguous)
// for all of them, PD columns ahead of its use.  y[j][p] = 0 for j >= K_p.
constexpr int BST = 512, MBS = 8, PD = 3;

template <int R>
__device__ __forceinline__ void bs_load(const double2* __restrict__ Rw, int c, double2 (&v)[MBS])
{
    if (c < 0) return;
    const double2* col = Rw + rpk(c, 0);
#pragma unroll
    for (int m = 0; m < MBS; ++m) {
        const int j = threadIdx.x + BST * m;
        if (j <= c) v[m] = col[j];
    }
}

template <int R>
__global__ __launch_bounds__(BST) void k_msb_backsub(const double2* __restrict__ rst, int NW, int kcols,
                                                     const int32_t* __restrict__ done,
                                                     const double2* __restrict__ g, double2* __restrict__ y)
{
    __shared__ double2 ys[R];
    const int w = blockIdx.x, tid = threadIdx.x, P = NW * R;
    const double2* Rw = rst + (size_t)w * rpk(kcols, 0);
    int K[R], Kw = 0;
#pragma unroll
    for (int l = 0; l < R; ++l) {
        const int d = done[w * R + l];
        K[l] = d ? d : kcols;
        Kw = std::max(Kw, K[l]);
    }
    double2 gr[MBS][R], ring[PD][MBS];
#pragma unroll
    for (int m = 0; m < MBS; ++m) {
        const int j = tid + BST * m;
#pragma unroll
        for (int l = 0; l < R; ++l) {
            gr[m][l] = j < K[l] ? g[((size_t)j * NW + w) * R + l] : make_double2(0.0, 0.0);
            if (j >= K[l] && j < kcols) y[(size_t)j * P + w * R + l] = make_double2(0.0, 0.0);
        }
    }
#pragma unroll
    for (int u = 0; u < PD; ++u) bs_load<R>(Rw, Kw - 1 - u, ring[u]);
    for (int cb = Kw - 1; cb >= 0; cb -= PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
            const int c = cb - u;
            if (c < 0) break;
            double2 cur[MBS];
#pragma unroll
            for (int m = 0; m < MBS; ++m) cur[m] = ring[u][m];
            bs_load<R>(Rw, c - PD, ring[u]);
            if (tid == (c % BST)) {
                const int mo = c / BST;
                double2 rcc = make_double2(0.0, 0.0);
                double2 gv[R];
#pragma unroll
                for (int l = 0; l < R; ++l) gv[l] = make_double2(0.0, 0.0);
#pragma unroll
                for (int m = 0; m < MBS; ++m)
                    if (m == mo) {
                        rcc = cur[m];
#pragma unroll
                        for (int l = 0; l < R; ++l) gv[l] = gr[m][l];
                    }
                const double den = cabs2(rcc);
#pragma unroll
                for (int l = 0; l < R; ++l) {
                    const double2 v = (c < K[l] && den > 0.0)
                                          ? make_double2((gv[l].x * rcc.x + gv[l].y * rcc.y) / den,
                                                         (gv[l].y * rcc.x - gv[l].x * rcc.y) / den)
                                          : make_double2(0.0, 0.0);
                    ys[l] = v;
                    if (c < K[l]) y[(size_t)c * P + w * R + l] = v;
                }
            }
            __syncthreads();
            double2 yc[R];
#pragma unroll
            for (int l = 0; l < R; ++l) yc[l] = ys[l];
#pragma unroll
            for (int m = 0; m < MBS; ++m) {
                const int j = tid + BST * m;
                if (j < c)
#pragma unroll
                    for (int l = 0; l < R; ++l) {
                        const double2 t = cmul(cur[m], yc[l]);
                        gr[m][l] = make_double2(gr[m][l].x - t.x, gr[m][l].y - t.y);
                    }
            }
            __syncthreads();
        }
    }
}

// W[row][K] = Vcol_K[row] = V[K / R][row][K % R] for K < kcols, 0 up to ldw:
// the basis as one row-major matrix, for a single operator apply over it.
__global__ void k_msb_basis_gather(const double* __restrict__ V, int64_t vstride, int R, int kcols, int64_t nup,
                                   double* __restrict__ W, int ldw)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nup * ldw) return;
    const int64_t row = t / ldw;
    const int K = (int)(t - row * ldw);
    W[t] = K < kcols ? V[(size_t)(K / R) * vstride + (size_t)row * R + K % R] : 0.0;
}

// TV[K / R][row][K % R] = Z[row][K] for K < kcols: an operator's product with
// the basis back in the basis layout.
__global__ void k_msb_basis_scatter(const double* __restrict__ Z, int ldz, int R, int kcols, int64_t nup,
                                    double* __restrict__ TV, int64_t vstride)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nup * kcols) return;
    const int64_t row = t / kcols;
    const int K = (int)(t - row * kcols);
    TV[(size_t)(K / R) * vstride + (size_t)row * R + K % R] = Z[(size_t)row * ldz + K];
}

// x[row][p] = sum_K Vcol_K[row] y[K][p] over the pair's K_p columns,
// Vcol_K = V[K / R][row][K % R]: tiles of 32 rows x 64 pairs, TJB blocks of the
// basis per LDS stage, up to the tile's largest K_p (blocks of steps issued
// after every pair finished were skipped and are never read).
template <int R>
__global__ __launch_bounds__(256) void k_msb_xcombine(const double* __restrict__ V, int64_t vstride, int kcols,
                                                      const int32_t* __restrict__ done,
                                                      const double2* __restrict__ y, int P, double2* __restrict__ x,
                                                      int ldx, int64_t nup)
{
    constexpr int TR = 32, TP = 64, TJB = 8;
    __shared__ double sv[TJB][TR][R];
    __shared__ double2 sy[TJB * R][TP];
    __shared__ int kt;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    const int p0 = blockIdx.y * TP;
    const int p = p0 + tx;
    if (tid == 0) kt = 0;
    __syncthreads();
    if (ty == 0 && p < P) atomicMax(&kt, done[p] ? done[p] : kcols);
    __syncthreads();
    const int kblocks = (kt + R - 1) / R;
    double2 acc[8];
#pragma unroll
    for (int qv = 0; qv < 8; ++qv) acc[qv] = make_double2(0.0, 0.0);
    for (int j0 = 0; j0 < kblocks; j0 += TJB) {
        __syncthreads();
        for (int e = tid; e < TJB * TR * R; e += 256) {
            const int jj = e / (TR * R), rem = e - jj * TR * R;
            const int rr = rem / R, cc = rem - rr * R;
            const int64_t row = row0 + rr;
            sv[jj][rr][cc] =
                (j0 + jj < kblocks && row < nup) ? V[(size_t)(j0 + jj) * vstride + (size_t)row * R + cc] : 0.0;
        }
        for (int e = tid; e < TJB * R * TP; e += 256) {
            const int kk = e / TP, pp = e - kk * TP;
            const int Kc = j0 * R + kk;
            sy[kk][pp] = (Kc < kcols && p0 + pp < P) ? y[(size_t)Kc * P + p0 + pp] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int jj = 0; jj < TJB; ++jj)
#pragma unroll
            for (int cc = 0; cc < R; ++cc) {
                const double2 yv = sy[jj * R + cc][tx];
#pragma unroll
                for (int qv = 0; qv < 8; ++qv) {
                    const double v = sv[jj][ty * 8 + qv][cc];
                    acc[qv] = make_double2(fma(v, yv.x, acc[qv].x), fma(v, yv.y, acc[qv].y));
                }
            }
    }
    if (p >= P) return;
#pragma unroll
    for (int qv = 0; qv < 8; ++qv) {
        const int64_t row = row0 + ty * 8 + qv;
        if (row < nup) x[(size_t)row * ldx + p] = acc[qv];
    }
}

// ---------------------------------------------------------------- launchers

namespace {

int msb_slabs(int64_t nup, int ngroups)
{
    int64_t maxs = (nup + 255) / 256;
    int64_t want = (1024 + ngroups - 1) / ngroups;
    want = std::max<int64_t>(1, std::min(want, maxs));
    return (int)want;
}

void msb_update_split(int64_t nup, int k, int& vps, int& nsp)
{
    if (k <= 0) {
        vps = 0;
        nsp = 1;
        return;
    }
    const int64_t rb = (nup + 255) / 256;
    int64_t want = (1024 + rb - 1) / rb;
    const int64_t maxs = (k + 15) / 16;
    want = std::max<int64_t>(1, std::min(want, maxs));
    vps = (int)((k + want - 1) / want);
    nsp = (k + vps - 1) / vps;
}

template <int R>
void step_r(const double* V, int64_t vstride, int k, double* u, const double* wt, double* part, double* part2,
            double* G, double* Hb, int ldh, double* coefv, double* coefu, double* scal, double* rho0, int64_t nup,
            int fix_only, hipStream_t st, const int32_t* stop, hipEvent_t e0, hipEvent_t e1)
{
    constexpr int W = 2 * R * R;
    const int nvec = k + 1;
    const int ngroups = (nvec + MJB - 1) / MJB;
    const int nslab = msb_slabs(nup, ngroups);
    const int64_t rps = (nup + nslab - 1) / nslab;
    hipExtLaunchKernelGGL(k_msb_dots<R>, dim3((unsigned)nslab, (unsigned)ngroups), dim3(256), 0, st, e0, nullptr, 0,
                          V, vstride, k, (const double*)u, wt, part, nup, rps, stop);
    hipLaunchKernelGGL(k_msb_reduce<W>, dim3((unsigned)((nvec * W + 255) / 256)), dim3(256), 0, st, (const double*)part,
                       nslab, nvec, G, stop);
    const dim3 cg((unsigned)((k + CWPB) / CWPB)), cb(64 * CWPB);
    if (fix_only) {
        hipExtLaunchKernelGGL(k_msb_coef<R>, cg, cb, 0, st, nullptr, e1, 0, (const double*)G, Hb, ldh, k, 1, coefv,
                              coefu, scal, rho0, stop);
        return;
    }
    hipLaunchKernelGGL(k_msb_coef<R>, cg, cb, 0, st, (const double*)G, Hb, ldh, k, 0, coefv, coefu, scal, rho0, stop);
    int vps, nsp;
    msb_update_split(nup, k, vps, nsp);
    double* vk = const_cast<double*>(V) + (size_t)k * vstride;
    hipExtLaunchKernelGGL(k_msb_update<R>, dim3((unsigned)((nup + 255) / 256), (unsigned)nsp), dim3(256), 0, st,
                          nullptr, nsp > 1 ? nullptr : e1, 0, V, vstride, k, (const double*)coefv,
                          (const double*)coefu, (const double*)scal, u, wt, vk, part2, nup, vps, stop);
    if (nsp > 1)
        hipExtLaunchKernelGGL(k_msb_finish<R>, dim3((unsigned)((nup + 255) / 256)), dim3(256), 0, st, nullptr, e1, 0,
                              (const double*)part2, nsp, (const double*)scal, u, wt, vk, nup, stop);
}

}  // namespace

void msb_init(int R, const double2* b, int ldb, double* u, int64_t nup, hipStream_t st)
{
    const dim3 grid((unsigned)((nup + 255) / 256));
    if (R == 2) hipLaunchKernelGGL(k_msb_init<2>, grid, dim3(256), 0, st, b, ldb, u, nup);
    else hipLaunchKernelGGL(k_msb_init<3>, grid, dim3(256), 0, st, b, ldb, u, nup);
}

void msb_step(int R, double* V, int64_t vstride, int k, double* u, const double* wt, double* part, double* part2,
              double* G, double* Hb, int ldh, double* coefv, double* coefu, double* scal, double* rho0, int64_t nup,
              bool fix_only, hipStream_t st, const int32_t* stop, const hipEvent_t* ev)
{
    hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
    if (R == 2)
        step_r<2>(V, vstride, k, u, wt, part, part2, G, Hb, ldh, coefv, coefu, scal, rho0, nup, fix_only ? 1 : 0, st,
                  stop, e0, e1);
    else
        step_r<3>(V, vstride, k, u, wt, part, part2, G, Hb, ldh, coefv, coefu, scal, rho0, nup, fix_only ? 1 : 0, st,
                  stop, e0, e1);
}

size_t msb_part_doubles(int R, int kcap)
{
    return (size_t)(1024 + (kcap + 1 + MJB - 1) / MJB) * MJB * 2 * R * R;
}

size_t msb_part2_doubles(int R, int64_t nup, int kcap)
{
    int mx = 1;
    for (int k = 1; k <= kcap; ++k) {
        int vps, nsp;
        msb_update_split(nup, k, vps, nsp);
        mx = std::max(mx, nsp);
    }
    return (size_t)mx * nup * 2 * R;
}

int msb_givens_cols() { return GBC; }

void msb_givens(int R, const double* Hb, int ldh, int NW, int K0, int nc, const double2* z, double* rc, double2* rs,
                double2* g, const double* rho0, const double* target, int32_t* done, double* resid, int32_t* ndone,
                int32_t* stop, hipStream_t st)
{
    const dim3 grid((unsigned)((NW + 3) / 4));
    if (R == 2)
        hipLaunchKernelGGL(k_msb_givens<2>, grid, dim3(64), 0, st, Hb, ldh, NW, K0, nc, z, rc, rs, g, rho0, target,
                           done, resid, ndone, stop);
    else
        hipLaunchKernelGGL(k_msb_givens<3>, grid, dim3(64), 0, st, Hb, ldh, NW, K0, nc, z, rc, rs, g, rho0, target,
                           done, resid, ndone, stop);
}

size_t msb_rst_elems(int NW, int kcols) { return (size_t)kcols * (kcols + 1) / 2 * NW; }

void msb_basis_gather(int R, const double* V, int64_t vstride, int kcols, int64_t nup, double* W, int ldw,
                      hipStream_t st)
{
    const int64_t len = nup * ldw;
    hipLaunchKernelGGL(k_msb_basis_gather, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, V, vstride, R, kcols,
                       nup, W, ldw);
}

void msb_basis_scatter(int R, const double* Z, int ldz, int kcols, int64_t nup, double* TV, int64_t vstride,
                       hipStream_t st)
{
    const int64_t len = nup * kcols;
    if (len == 0) return;
    hipLaunchKernelGGL(k_msb_basis_scatter, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, Z, ldz, R, kcols,
                       nup, TV, vstride);
}

void msb_xcombine(int R, const double* V, int64_t vstride, int kcols, const int32_t* done, const double2* y, int P,
                  double2* x, int ldx, int64_t nup, hipStream_t st)
{
    if (kcols < 1) return;
    const dim3 gx((unsigned)((nup + 31) / 32), (unsigned)((P + 63) / 64));
    if (R == 2)
        hipLaunchKernelGGL(k_msb_xcombine<2>, gx, dim3(256), 0, st, V, vstride, kcols, done, y, P, x, ldx, nup);
    else
        hipLaunchKernelGGL(k_msb_xcombine<3>, gx, dim3(256), 0, st, V, vstride, kcols, done, y, P, x, ldx, nup);
}

void msb_finish_solve(int R, const double* Hb, int ldh, int NW, int kcols, const double2* z, const double* rc,
                      const double2* rs, const int32_t* done, double2* rst, const double2* g, double2* y,
                      const double* V, int64_t vstride, double2* x, int ldx, int64_t nup, hipStream_t st)
{
    if (kcols < 1) return;
    const int P = NW * R;
    const dim3 gr((unsigned)((kcols + 63) / 64), (unsigned)NW);
    const dim3 gx((unsigned)((nup + 31) / 32), (unsigned)((P + 63) / 64));
    if (R == 2) {
        hipLaunchKernelGGL(k_msb_rfactor<2>, gr, dim3(64), 0, st, Hb, ldh, NW, kcols, z, rc, rs, done, rst);
        hipLaunchKernelGGL(k_msb_backsub<2>, dim3((unsigned)NW), dim3(BST), 0, st, (const double2*)rst, NW, kcols,
                           done, g, y);
        hipLaunchKernelGGL(k_msb_xcombine<2>, gx, dim3(256), 0, st, V, vstride, kcols, done, (const double2*)y, P, x,
                           ldx, nup);
    } else {
        hipLaunchKernelGGL(k_msb_rfactor<3>, gr, dim3(64), 0, st, Hb, ldh, NW, kcols, z, rc, rs, done, rst);
        hipLaunchKernelGGL(k_msb_backsub<3>, dim3((unsigned)NW), dim3(BST), 0, st, (const double2*)rst, NW, kcols,
                           done, g, y);
        hipLaunchKernelGGL(k_msb_xcombine<3>, gx, dim3(256), 0, st, V, vstride, kcols, done, (const double2*)y, P, x,
                           ldx, nup);
    }
}

}  // namespace px
