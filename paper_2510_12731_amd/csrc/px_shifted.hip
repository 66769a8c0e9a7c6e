// Shared-Krylov solve of every frequency of a one-material omegaFQ structure.
//
// Eq. (wfq-system) for column (omega_j, l) reads (M - z_q(omega_j) I) q = b_l
// with M = Kbar T real and b_l = E0 Kbar r_l real and the same for every
// frequency (Eq. z_q_wfq gives the only frequency dependence).  A Krylov space
// does not change under a shift, K_k(M - z I, b) = K_k(M, b), and the Arnoldi
// relation M V_k = V_{k+1} Hbar_k gives (M - z I) V_k = V_{k+1} (Hbar_k - z I~),
// so one real Arnoldi process per polarization yields, for every frequency,
// exactly the iterate of unrestarted GMRES on that frequency's system
// (Section 6, "iterative on the fly"): each shift only adds its own Givens QR
// of the small shifted Hessenberg matrix.
//
// Layout: the basis of the R = npol polarizations is interleaved,
// V[k][row][slot], so the narrow FP64 T-apply reads one basis vector of every
// polarization in one pass over the atom pairs.  Hbar is stored row-major per
// polarization, H[(slot (kcap + 1) + row) kcap + column].  Per (frequency,
// polarization) pair p = w * npol + slot (the solver's column index): the
// rotations cs[k][p], sn[k][p] and the rotated right-hand side g[k][p],
// coalesced over p.
#include "px_internal.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace px {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cfma_real(double v, double2 y, double2 acc)
{
    return make_double2(fma(v, y.x, acc.x), fma(v, y.y, acc.y));
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

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace

// u[row][c] = b[row][c].x / bnorm[c] (the right-hand sides of the first
// frequency's columns, normalised).
template <int R>
__global__ void k_ms_init(const double2* __restrict__ b, int ldb, const double* __restrict__ bnorm,
                          double* __restrict__ u, int64_t nup)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nup) return;
#pragma unroll
    for (int c = 0; c < R; ++c) {
        double v = 0.0;
        if (bnorm[c] > 0.0) v = b[(size_t)r * ldb + c].x / bnorm[c];
        u[(size_t)r * R + c] = v;
    }
}

// w = Kbar Y over the R slots (rows of ghost atoms zero).
template <int R>
__global__ __launch_bounds__(256) void k_ms_spmv(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const double* __restrict__ cv, const double* __restrict__ Y,
                                                 double* __restrict__ w, int64_t n, int64_t np,
                                                 const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0;
    if (i < n) {
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const double k = cv[e];
            const double* y = Y + (size_t)ci[e] * R;
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = fma(k, y[c], acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) w[(size_t)i * R + c] = acc[c];
}

// ---- delayed classical Gram-Schmidt (DCGS2) --------------------------------
// Step k holds u, the candidate for v_k orthogonalised once against V_{<k} in
// step k-1, and wt = M u.  One dot pass gives s = V_{<k}^T u, c = V_{<k}^T wt,
// <u,u> and <u,wt>.  Then rho = sqrt(<u,u> - |s|^2) and v_k = (u - V_{<k} s)
// / rho; column k-1 of Hbar gains s (rows < k) and rho (row k); with
// c_k = (<u,wt> - s.c) / rho and t = Hbar_{(k+1) x k} s, the first-pass
// column k is h_j = (c_j - t_j) / rho (j < k), h_k = (c_k - t_k) / rho, and
// the next candidate is u' = M v_k - V_{<=k} h = wt / rho - (c_k / rho^2) u
// - V_{<k} d with d = (c - (c_k / rho) s) / rho: one update pass over V_{<k}
// writes v_k and u'.

// part[(j * nslab + slab)][c] = sum over the slab's rows of x_j[row][c] u[row][c]
// and part[..][R + c] the same with wt, where x_j = V_j (j < k) or u (j = k).
// A block takes MJ consecutive vectors, so u and wt are read once for MJ of them.
constexpr int MJ = 2;

template <int R>
__global__ __launch_bounds__(256) void k_ms_dots(const double* __restrict__ V, int64_t vstride, int k,
                                                 const double* __restrict__ u, const double* __restrict__ wt,
                                                 double* __restrict__ part, int64_t nup, int64_t rows_per_slab,
                                                 const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int W = 2 * R;
    __shared__ double lds[4][MJ * W];
    const int j0 = blockIdx.y * MJ, slab = blockIdx.x, nslab = gridDim.x;
    const int nj = k + 1 - j0 < MJ ? k + 1 - j0 : MJ;
    const int64_t r0 = (int64_t)slab * rows_per_slab;
    const int64_t r1 = r0 + rows_per_slab < nup ? r0 + rows_per_slab : nup;
    double acc[MJ * W];
#pragma unroll
    for (int c = 0; c < MJ * W; ++c) acc[c] = 0.0;
    // the block's vectors (u itself for j = k, and in place of the missing
    // ones of a short last group, whose sums are not written): chosen once, so
    // that the row loop has no branch and its loads overlap across rows
    const double* xp[MJ];
#pragma unroll
    for (int jj = 0; jj < MJ; ++jj) {
        const int j = j0 + jj;
        xp[jj] = (jj < nj && j < k) ? V + (size_t)j * vstride : u;
    }
#pragma unroll 2
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        double uu[R], ww[R], xx[MJ][R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            uu[c] = u[(size_t)r * R + c];
            ww[c] = wt[(size_t)r * R + c];
        }
#pragma unroll
        for (int jj = 0; jj < MJ; ++jj)
#pragma unroll
            for (int c = 0; c < R; ++c) xx[jj][c] = xp[jj][(size_t)r * R + c];
#pragma unroll
        for (int jj = 0; jj < MJ; ++jj)
#pragma unroll
            for (int c = 0; c < R; ++c) {
                acc[jj * W + c] = fma(xx[jj][c], uu[c], acc[jj * W + c]);
                acc[jj * W + R + c] = fma(xx[jj][c], ww[c], acc[jj * W + R + c]);
            }
    }
    block_sum<MJ * W>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int jj = 0; jj < MJ; ++jj)
            if (jj < nj)
#pragma unroll
                for (int c = 0; c < W; ++c) part[((size_t)(j0 + jj) * nslab + slab) * W + c] = acc[jj * W + c];
}

// G[j][c] = sum over slabs of part[j][slab][c] (fixed order), W values per j.
template <int W>
__global__ void k_ms_reduce(const double* __restrict__ part, int nslab, int nvec, double* __restrict__ G,
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

// The coefficients of step k from G (layout of k_ms_dots), one wave per row j
// of Hbar (j = 0..k) and slot c = blockIdx.y: corrects column k-1, writes the
// first-pass column k (rows 0..k), coefv[j][c] = s_j / rho and coefu[j][c] =
// d_j, and scal[c] = {1 / rho, 1 / rho, -c_k / rho^2}.  fix_only: the last
// column's correction alone.  A zero rho (an invariant subspace) zeroes v_k
// and u'.
template <int R>
__global__ __launch_bounds__(256) void k_ms_coef(const double* __restrict__ G, double* __restrict__ H, int kcap,
                                                 int k, int fix_only, double* __restrict__ coefv,
                                                 double* __restrict__ coefu, double* __restrict__ scal,
                                                 const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    constexpr int W = 2 * R;
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int c = blockIdx.y;
    if (j > k) return;
    double ss = 0.0, sc = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double si = G[i * W + c];
        ss = fma(si, si, ss);
        sc = fma(si, G[i * W + R + c], sc);
    }
    ss = wave_sum(ss);
    sc = wave_sum(sc);
    const double rho2 = G[k * W + c] - ss;
    const double rho = rho2 > 0.0 ? sqrt(rho2) : 0.0;
    const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
    const double ck = (G[k * W + R + c] - sc) * inv;
    double* hrow = H + ((size_t)c * (kcap + 1) + j) * kcap;
    const double sj = j < k ? G[j * W + c] : 0.0;
    double hfix = 0.0;
    if (k >= 1) hfix = j < k ? hrow[k - 1] + sj : rho;
    if (fix_only) {
        if (lane == 0 && k >= 1) hrow[k - 1] = hfix;
        return;
    }
    // t_j = sum_{i >= j-1, i < k} Hbar[j][i] s_i with the corrected column k-1
    double t = 0.0;
    for (int i = (j > 0 ? j - 1 : 0) + lane; i < k; i += 64) {
        const double h = i == k - 1 ? hfix : hrow[i];
        t = fma(h, G[i * W + c], t);
    }
    t = wave_sum(t);
    if (lane == 0) {
        if (k >= 1) hrow[k - 1] = hfix;
        const double cj = j < k ? G[j * W + R + c] : ck;
        hrow[k] = (cj - t) * inv;
        if (j < k) {
            coefv[j * R + c] = sj * inv;
            coefu[j * R + c] = (cj - ck * inv * sj) * inv;
        }
        if (j == 0) {
            scal[c * 3 + 0] = inv;
            scal[c * 3 + 1] = inv;
            scal[c * 3 + 2] = -ck * inv * inv;
        }
    }
}

// One pass over V_{<k}: v_k = scal0 u - V coefv and u' = scal1 wt + scal2 u -
// V coefu (in place).  The vectors are split over blockIdx.y; with one split
// the results are written directly, else the split sums go to part2 and
// k_ms_finish adds them in a fixed order.
template <int R>
__global__ __launch_bounds__(256) void k_ms_update(const double* __restrict__ V, int64_t vstride, int k,
                                                   const double* __restrict__ coefv, const double* __restrict__ coefu,
                                                   const double* __restrict__ scal, double* __restrict__ u,
                                                   const double* __restrict__ wt, double* __restrict__ vk,
                                                   double* __restrict__ part2, int64_t nup, int vecs_per_split,
                                                   const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nup) return;
    const int j0 = blockIdx.y * vecs_per_split;
    const int j1 = j0 + vecs_per_split < k ? j0 + vecs_per_split : k;
    double av[R], au[R];
#pragma unroll
    for (int c = 0; c < R; ++c) av[c] = au[c] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double* vj = V + (size_t)j * vstride + (size_t)r * R;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const double x = vj[c];
            av[c] = fma(x, coefv[j * R + c], av[c]);
            au[c] = fma(x, coefu[j * R + c], au[c]);
        }
    }
    if (gridDim.y == 1) {
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const size_t o = (size_t)r * R + c;
            const double uo = u[o];
            vk[o] = scal[c * 3] * uo - av[c];
            u[o] = scal[c * 3 + 1] * wt[o] + scal[c * 3 + 2] * uo - au[c];
        }
    } else {
#pragma unroll
        for (int c = 0; c < R; ++c) {
            part2[((size_t)blockIdx.y * nup + r) * 2 * R + c] = av[c];
            part2[((size_t)blockIdx.y * nup + r) * 2 * R + R + c] = au[c];
        }
    }
}

template <int R>
__global__ void k_ms_finish(const double* __restrict__ part2, int nsplit, const double* __restrict__ scal,
                            double* __restrict__ u, const double* __restrict__ wt, double* __restrict__ vk,
                            int64_t nup, const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nup * R) return;
    const int64_t r = t / R;
    const int c = (int)(t - r * R);
    double av = 0.0, au = 0.0;
    for (int q = 0; q < nsplit; ++q) {
        av += part2[((size_t)q * nup + r) * 2 * R + c];
        au += part2[((size_t)q * nup + r) * 2 * R + R + c];
    }
    const double uo = u[t];
    vk[t] = scal[c * 3] * uo - av;
    u[t] = scal[c * 3 + 1] * wt[t] + scal[c * 3 + 2] * uo - au;
}

// Entry (j, K) of Hbar for polarization c.
__device__ __forceinline__ double hget(const double* __restrict__ H, int kcap, int c, int j, int K)
{
    return H[((size_t)c * (kcap + 1) + j) * kcap + K];
}

// Entry (j, K) of Hbar - z I~ (the shift on the diagonal).
__device__ __forceinline__ double2 hs(const double* __restrict__ H, int kcap, int c, int K, int j, double2 zp)
{
    const double h = hget(H, kcap, c, j, K);
    return j == K ? make_double2(h - zp.x, -zp.y) : make_double2(h, 0.0);
}

// (a, b) <- (c a + s b, -conj(s) a + c b): returns the first, carries the second in a.
__device__ __forceinline__ double2 rotate(double cj, double2 sj, double2& a, double2 b)
{
    const double2 sb = cmul(sj, b);
    const double2 first = make_double2(cj * a.x + sb.x, cj * a.y + sb.y);
    const double2 sa = cmul(make_double2(sj.x, -sj.y), a);
    a = make_double2(cj * b.x - sa.x, cj * b.y - sa.y);
    return first;
}

// The rotations 0..k0-1 of pair p applied to the carried entries a[q] of the
// nb new columns k0 + q; each output R[j][k0 + q] goes to the packed factor.
// Two register buffers alternate: the loads of the next GU rotations are in
// flight while the current GU are applied to nb independent chains.
constexpr int GB = 8, GU = 4;

struct RotBatch {
    double c[GU];
    double2 s[GU];
    double h[GU][GB];
};

__device__ __forceinline__ size_t rpk(int l, int j) { return (size_t)l * (l + 1) / 2 + j; }

__device__ __forceinline__ void load_rots(RotBatch& b, const double* __restrict__ cs, const double2* __restrict__ sn,
                                          const double* __restrict__ H, int kcap, int c, int P, int p, int k0, int nb,
                                          int j0)
{
#pragma unroll
    for (int u = 0; u < GU; ++u) {
        const int j = j0 + u;
        if (j < k0) {
            b.c[u] = cs[(size_t)j * P + p];
            b.s[u] = sn[(size_t)j * P + p];
#pragma unroll
            for (int q = 0; q < GB; ++q) {
                const int l = k0 + q;
                if (q < nb) b.h[u][q] = hget(H, kcap, c, j + 1, l);
            }
        }
    }
}

__device__ __forceinline__ void apply_rots(const RotBatch& b, double2 (&a)[GB], int k0, int nb, int j0, double2 zp)
{
#pragma unroll
    for (int u = 0; u < GU; ++u) {
        const int j = j0 + u;
        if (j < k0) {
#pragma unroll
            for (int q = 0; q < GB; ++q) {
                const int l = k0 + q;
                if (q < nb) {
                    const double hv = b.h[u][q];
                    const double2 bb = j + 1 == l ? make_double2(hv - zp.x, -zp.y) : make_double2(hv, 0.0);
                    (void)rotate(b.c[u], b.s[u], a[q], bb);
                }
            }
        }
    }
}

// Columns k0 .. k0+kn-1 (kn <= GB) of every shifted Hessenberg matrix
// Hbar - z_p I~: the rotations of earlier columns are applied to all kn
// columns in one pass (each rotation loaded once, kn independent chains),
// then each column takes the batch's new rotations and its own, which
// annihilates its subdiagonal; the rotated right-hand side gives the GMRES
// residual norm |g[K+1][p]|.  One thread per (frequency, polarization) pair;
// the thread that finishes the last pair raises *stop.  Nothing is stored
// inside the chains (stores and loads share one completion counter here).
__global__ __launch_bounds__(64) void k_ms_givens(const double* __restrict__ H, int kcap, int npol, int P, int k0,
                                                  int kn, const double2* __restrict__ z, double* __restrict__ cs,
                                                  double2* __restrict__ sn, double2* __restrict__ g,
                                                  const double* __restrict__ target,
                                                  int32_t* __restrict__ done, double* __restrict__ resid,
                                                  int32_t* __restrict__ ndone, int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || done[p]) return;
    const int c = p % npol;
    const double2 zp = z[p];
    double2 a[GB];
#pragma unroll
    for (int q = 0; q < GB; ++q)
        if (q < kn) a[q] = hs(H, kcap, c, k0 + q, 0, zp);
    RotBatch b0, b1;
    load_rots(b0, cs, sn, H, kcap, c, P, p, k0, kn, 0);
    for (int j0 = 0; j0 < k0; j0 += 2 * GU) {
        load_rots(b1, cs, sn, H, kcap, c, P, p, k0, kn, j0 + GU);
        apply_rots(b0, a, k0, kn, j0, zp);
        load_rots(b0, cs, sn, H, kcap, c, P, p, k0, kn, j0 + 2 * GU);
        apply_rots(b1, a, k0, kn, j0 + GU, zp);
    }
    double rc[GB];
    double2 rs[GB];
    double2 gk = g[(size_t)k0 * P + p];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
        if (q >= kn) break;
        const int K = k0 + q;
        double2 u = a[q];
#pragma unroll
        for (int t = 0; t < GB; ++t)
            if (t < q) (void)rotate(rc[t], rs[t], u, hs(H, kcap, c, K, k0 + t + 1, zp));
        const double beta = hget(H, kcap, c, K + 1, K);
        const double aa = sqrt(u.x * u.x + u.y * u.y);
        double ck;
        double2 sk;
        if (aa == 0.0) {
            ck = 0.0;
            sk = make_double2(1.0, 0.0);
        } else {
            const double rr = sqrt(aa * aa + beta * beta);
            ck = aa / rr;
            sk = make_double2(u.x / aa * beta / rr, u.y / aa * beta / rr);
        }
        rc[q] = ck;
        rs[q] = sk;
        cs[(size_t)K * P + p] = ck;
        sn[(size_t)K * P + p] = sk;
        g[(size_t)K * P + p] = make_double2(ck * gk.x, ck * gk.y);
        gk = cmul(make_double2(-sk.x, sk.y), gk);
        g[(size_t)(K + 1) * P + p] = gk;
        const double res = sqrt(gk.x * gk.x + gk.y * gk.y);
        resid[p] = res;
        if (res <= target[p]) {
            done[p] = K + 1;
            if (atomicAdd(ndone, 1) + 1 == P && stop) *stop = 1;
            break;
        }
    }
}

// Column l = blockIdx.y of every pair's triangular factor R_p (pairs with
// K_p <= l skip), rebuilt by the same chain of rotations as k_ms_givens:
// rst[(l (l + 1) / 2 + j) P + p] = R_p[j][l].  One thread per pair; the many
// columns in flight hide the chains' memory latency.
__global__ __launch_bounds__(64) void k_ms_rfactor(const double* __restrict__ H, int kcap, int npol, int P, int kmax,
                                                   const double2* __restrict__ z, const double* __restrict__ cs,
                                                   const double2* __restrict__ sn, const int32_t* __restrict__ done,
                                                   double2* __restrict__ rst)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (p >= P) return;
    const int K = done[p] ? done[p] : kmax;
    if (l >= K) return;
    const int c = p % npol;
    const double2 zp = z[p];
    double2 a = hs(H, kcap, c, l, 0, zp);
#pragma unroll 4
    for (int j = 0; j < l; ++j) {
        const double hv = hget(H, kcap, c, j + 1, l);
        const double2 b = j + 1 == l ? make_double2(hv - zp.x, -zp.y) : make_double2(hv, 0.0);
        rst[rpk(l, j) * P + p] = rotate(cs[(size_t)j * P + p], sn[(size_t)j * P + p], a, b);
    }
    const double cl = cs[(size_t)l * P + p];
    const double2 sl = sn[(size_t)l * P + p];
    const double beta = hget(H, kcap, c, l + 1, l);
    rst[rpk(l, l) * P + p] = make_double2(cl * a.x + sl.x * beta, cl * a.y + sl.y * beta);
}

// Least-squares solution y_p = R_p^-1 g_p of every pair over its own number
// of steps K_p (done[p], else kmax), one workgroup per pair: column-oriented
// back substitution with g in LDS, the rows of each column spread over the
// threads.  y[j][p] = 0 for j >= K_p.
__global__ __launch_bounds__(256) void k_ms_backsub(const double2* __restrict__ rst, int P, int kmax,
                                                    const int32_t* __restrict__ done, const double2* __restrict__ g,
                                                    double2* __restrict__ y)
{
    extern __shared__ double2 gl[];
    const int p = blockIdx.x, tid = threadIdx.x;
    const int K = done[p] ? done[p] : kmax;
    for (int j = tid; j < kmax; j += blockDim.x) {
        if (j < K) gl[j] = g[(size_t)j * P + p];
        else y[(size_t)j * P + p] = make_double2(0.0, 0.0);
    }
    for (int l = K - 1; l >= 0; --l) {
        __syncthreads();
        const double2 rll = rst[rpk(l, l) * P + p];
        const double2 gv = gl[l];
        const double den = rll.x * rll.x + rll.y * rll.y;
        const double2 yl = den > 0.0 ? make_double2((gv.x * rll.x + gv.y * rll.y) / den,
                                                    (gv.y * rll.x - gv.x * rll.y) / den)
                                     : make_double2(0.0, 0.0);
        if (tid == 0) y[(size_t)l * P + p] = yl;
        for (int j = tid; j < l; j += blockDim.x) {
            const double2 r = cmul(rst[rpk(l, j) * P + p], yl);
            gl[j] = make_double2(gl[j].x - r.x, gl[j].y - r.y);
        }
    }
}

// x[row][p] = sum_j V_j[row][slot(p)] y[j][p] over the pair's K_p = done[p]
// (else kmax) basis vectors: tiles of 32 rows x 64 pairs, 16 basis vectors per
// LDS stage, up to the tile's largest K_p (vectors of steps issued after every
// pair finished were skipped and are never read).
template <int R>
__global__ __launch_bounds__(256) void k_ms_xcombine(const double* __restrict__ V, int64_t vstride, int kmax,
                                                     const int32_t* __restrict__ done,
                                                     const double2* __restrict__ y, int npol, int P,
                                                     double2* __restrict__ x, int ldx, int64_t nup)
{
    constexpr int TR = 32, TP = 64, TJ = 16;
    __shared__ double sv[TJ][TR][R];
    __shared__ double2 sy[TJ][TP];
    __shared__ int kt;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    const int p0 = blockIdx.y * TP;
    const int p = p0 + tx;
    const int c = p % npol;
    if (tid == 0) kt = 0;
    __syncthreads();
    if (ty == 0 && p < P) atomicMax(&kt, done[p] ? done[p] : kmax);
    __syncthreads();
    const int K = kt;
    double2 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int j0 = 0; j0 < K; j0 += TJ) {
        __syncthreads();
        for (int e = tid; e < TJ * TR * R; e += 256) {
            const int jj = e / (TR * R), rem = e - jj * TR * R;
            const int rr = rem / R, cc = rem - rr * R;
            const int64_t row = row0 + rr;
            sv[jj][rr][cc] = (j0 + jj < K && row < nup) ? V[(size_t)(j0 + jj) * vstride + (size_t)row * R + cc] : 0.0;
        }
        for (int e = tid; e < TJ * TP; e += 256) {
            const int jj = e / TP, pp = e - jj * TP;
            sy[jj][pp] = (j0 + jj < K && p0 + pp < P) ? y[(size_t)(j0 + jj) * P + p0 + pp] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 4
        for (int jj = 0; jj < TJ; ++jj) {
            const double2 yv = sy[jj][tx];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = cfma_real(sv[jj][ty * 8 + q][c], yv, acc[q]);
        }
    }
    if (p >= P) return;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t row = row0 + ty * 8 + q;
        if (row < nup) x[(size_t)row * ldx + p] = acc[q];
    }
}

// ---------------------------------------------------------------- launchers

namespace {

template <template <int> class F, typename... A>
void with_r(int R, A... a)
{
    if (R == 1) F<1>::run(a...);
    else if (R == 2) F<2>::run(a...);
    else F<3>::run(a...);
}

// row slabs of the dot pass over ngroups vector groups: about 1024 blocks
// (two vectors per block measured fastest: 47 us against 54 us for one and
// 73 us for four at step 800 of the 20k-atom sphere; 1024 blocks 1 ms per
// solve faster than 2048 there, 4096 5 ms slower)
int ms_slabs(int64_t nup, int ngroups)
{
    int64_t maxs = (nup + 255) / 256;
    int64_t want = (1024 + ngroups - 1) / ngroups;
    if (want < 1) want = 1;
    if (want > maxs) want = maxs;
    return (int)want;
}

// vectors per split and number of splits of the update pass over k vectors
void ms_update_split(int64_t nup, int k, int& vps, int& nsp)
{
    if (k <= 0) {
        vps = 0;
        nsp = 1;
        return;
    }
    const int64_t rb = (nup + 255) / 256;
    int64_t want = (1024 + rb - 1) / rb;
    const int64_t maxs = (k + 15) / 16;
    if (want > maxs) want = maxs;
    if (want < 1) want = 1;
    vps = (int)((k + want - 1) / want);
    nsp = (k + vps - 1) / vps;
}

template <int R>
struct InitL {
    static void run(const double2* b, int ldb, const double* bn, double* u, int64_t nup, hipStream_t st)
    {
        hipLaunchKernelGGL(k_ms_init<R>, dim3((unsigned)((nup + 255) / 256)), dim3(256), 0, st, b, ldb, bn, u, nup);
    }
};

template <int R>
struct SpmvL {
    static void run(const Geometry* g, const double* Y, double* w, hipStream_t st, const int32_t* stop,
                    hipEvent_t e0, hipEvent_t e1)
    {
        hipExtLaunchKernelGGL(k_ms_spmv<R>, dim3((unsigned)((g->np + 255) / 256)), dim3(256), 0, st, e0, e1, 0,
                              (const int32_t*)g->row_ptr, (const int32_t*)g->col, (const double*)g->val, Y, w, g->n,
                              g->np, stop);
    }
};

template <int R>
struct StepL {
    static void run(const double* V, int64_t vstride, int k, double* u, const double* wt, double* part,
                    double* part2, double* G, double* H, int kcap, double* coefv, double* coefu, double* scal,
                    int64_t nup, int fix_only, hipStream_t st, const int32_t* stop, hipEvent_t e0, hipEvent_t e1)
    {
        constexpr int W = 2 * R;
        const int nvec = k + 1;
        const int ngroups = (nvec + MJ - 1) / MJ;
        const int nslab = ms_slabs(nup, ngroups);
        const int64_t rps = (nup + nslab - 1) / nslab;
        hipExtLaunchKernelGGL(k_ms_dots<R>, dim3((unsigned)nslab, (unsigned)ngroups), dim3(256), 0, st, e0, nullptr, 0,
                              V, vstride, k, (const double*)u, wt, part, nup, rps, stop);
        hipLaunchKernelGGL(k_ms_reduce<W>, dim3((unsigned)((nvec * W + 255) / 256)), dim3(256), 0, st, part, nslab,
                           nvec, G, stop);
        if (fix_only) {
            hipExtLaunchKernelGGL(k_ms_coef<R>, dim3((unsigned)((k + 1 + 3) / 4), (unsigned)R), dim3(256), 0, st,
                                  nullptr, e1, 0, (const double*)G, H, kcap, k, fix_only, coefv, coefu, scal, stop);
            return;
        }
        hipLaunchKernelGGL(k_ms_coef<R>, dim3((unsigned)((k + 1 + 3) / 4), (unsigned)R), dim3(256), 0, st, G, H,
                           kcap, k, fix_only, coefv, coefu, scal, stop);
        int vps, nsp;
        ms_update_split(nup, k, vps, nsp);
        double* vk = const_cast<double*>(V) + (size_t)k * vstride;
        hipExtLaunchKernelGGL(k_ms_update<R>, dim3((unsigned)((nup + 255) / 256), (unsigned)nsp), dim3(256), 0, st,
                              nullptr, nsp > 1 ? nullptr : e1, 0, V, vstride, k, (const double*)coefv,
                              (const double*)coefu, (const double*)scal, u, wt, vk, part2, nup, vps, stop);
        if (nsp > 1)
            hipExtLaunchKernelGGL(k_ms_finish<R>, dim3((unsigned)((nup * R + 255) / 256)), dim3(256), 0, st, nullptr,
                                  e1, 0, (const double*)part2, nsp, (const double*)scal, u, wt, vk, nup, stop);
    }
};

template <int R>
struct XcombL {
    static void run(const double* V, int64_t vstride, int K, const int32_t* done, const double2* y, int P, double2* x,
                    int ldx, int64_t nup, hipStream_t st)
    {
        const dim3 grid((unsigned)((nup + 31) / 32), (unsigned)((P + 63) / 64));
        hipLaunchKernelGGL(k_ms_xcombine<R>, grid, dim3(256), 0, st, V, vstride, K, done, y, R, P, x, ldx, nup);
    }
};

}  // namespace

void ms_init(int R, const double2* b, int ldb, const double* bnorm, double* u, int64_t nup, hipStream_t st)
{
    with_r<InitL>(R, b, ldb, bnorm, u, nup, st);
}

void ms_spmv(int R, const Geometry& g, const double* Y, double* w, hipStream_t st, const int32_t* stop,
             const hipEvent_t* ev)
{
    with_r<SpmvL>(R, &g, Y, w, st, stop, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
}

void ms_step(int R, double* V, int64_t vstride, int k, double* u, const double* wt, double* part, double* part2,
             double* G, double* H, int kcap, double* coefv, double* coefu, double* scal, int64_t nup, bool fix_only,
             hipStream_t st, const int32_t* stop, const hipEvent_t* ev)
{
    with_r<StepL>(R, (const double*)V, vstride, k, u, wt, part, part2, G, H, kcap, coefv, coefu, scal, nup,
                  fix_only ? 1 : 0, st, stop, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
}

size_t ms_part_doubles(int R, int64_t nup, int kcap)
{
    // slabs x (vectors rounded up to MJ) <= (1024 + groups) x MJ for every length up to kcap + 1
    (void)nup;
    return (size_t)(1024 + (kcap + 1 + MJ - 1) / MJ) * MJ * 2 * R;
}

size_t ms_part2_doubles(int R, int64_t nup, int kcap)
{
    int mx = 1;
    for (int k = 1; k <= kcap; ++k) {
        int vps, nsp;
        ms_update_split(nup, k, vps, nsp);
        if (nsp > mx) mx = nsp;
    }
    return (size_t)mx * nup * 2 * R;
}

int ms_givens_batch() { return GB; }

void ms_givens(const double* H, int kcap, int npol, int P, int k0, int kn, const double2* z, double* cs, double2* sn,
               double2* g, const double* target, int32_t* done, double* resid, int32_t* ndone, int32_t* stop,
               hipStream_t st)
{
    hipLaunchKernelGGL(k_ms_givens, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, H, kcap, npol, P, k0, kn, z, cs,
                       sn, g, target, done, resid, ndone, stop);
}

void ms_rfactor(const double* H, int kcap, int npol, int P, int kmax, const double2* z, const double* cs,
                const double2* sn, const int32_t* done, double2* rst, hipStream_t st)
{
    if (kmax < 1) return;
    hipLaunchKernelGGL(k_ms_rfactor, dim3((unsigned)((P + 63) / 64), (unsigned)kmax), dim3(64), 0, st, H, kcap, npol,
                       P, kmax, z, cs, sn, done, rst);
}

size_t ms_rst_elems(int P, int kcap) { return (size_t)kcap * (kcap + 1) / 2 * P; }

void ms_backsub(const double2* rst, int P, int kmax, const int32_t* done, const double2* g, double2* y, hipStream_t st)
{
    hipLaunchKernelGGL(k_ms_backsub, dim3((unsigned)P), dim3(256), sizeof(double2) * kmax, st, rst, P, kmax, done, g,
                       y);
}

void ms_xcombine(int R, const double* V, int64_t vstride, int K, const int32_t* done, const double2* y, int P,
                 double2* x, int ldx, int64_t nup, hipStream_t st)
{
    with_r<XcombL>(R, V, vstride, K, done, y, P, x, ldx, nup, st);
}

}  // namespace px
