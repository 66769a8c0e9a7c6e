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
// Layout: the basis of the npol polarizations is interleaved, V[k][row][slot]
// (R = 2 or 4 real slots per row, slot = polarization index, unused slots
// zero), so the narrow FP64 T-apply reads one basis vector of every
// polarization in one pass over the atom pairs.  Per (frequency,
// polarization) pair p = w * npol + slot (the solver's column index): the
// rotations cs[k][p], sn[k][p] and the rotated right-hand side g[k][p],
// coalesced over p.  Hessenberg columns are stored packed: column k has rows
// 0..k+1 at row offset k (k + 3) / 2.
#include "px_internal.h"

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

// Block sum of R values over 256 threads in a fixed order; thread 0 returns it.
template <int R>
__device__ __forceinline__ void block_sum(double (&v)[R], double (*lds)[R])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int c = 0; c < R; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < R; ++c) lds[wave][c] = v[c];
    __syncthreads();
    if (tid == 0)
#pragma unroll
        for (int c = 0; c < R; ++c) v[c] = (lds[0][c] + lds[1][c]) + (lds[2][c] + lds[3][c]);
}

}  // namespace

// V0[row][c] = b[row][c].x / bnorm[c] for c < npol (the right-hand sides of
// the first frequency's columns), 0 otherwise.
template <int R>
__global__ void k_ms_init(const double2* __restrict__ b, int ldb, int npol, const double* __restrict__ bnorm,
                          double* __restrict__ V0, int64_t nup)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nup) return;
#pragma unroll
    for (int c = 0; c < R; ++c) {
        double v = 0.0;
        if (c < npol && bnorm[c] > 0.0) v = b[(size_t)r * ldb + c].x / bnorm[c];
        V0[(size_t)r * R + c] = v;
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

// part[(j * nslab + slab)][c] = sum over the slab's rows of V_j[row][c] w[row][c]
template <int R>
__global__ __launch_bounds__(256) void k_ms_dots(const double* __restrict__ V, int64_t vstride,
                                                 const double* __restrict__ w, double* __restrict__ part,
                                                 int64_t nup, int64_t rows_per_slab, const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    __shared__ double lds[4][R];
    const int j = blockIdx.y, slab = blockIdx.x, nslab = gridDim.x;
    const int64_t r0 = (int64_t)slab * rows_per_slab;
    const int64_t r1 = r0 + rows_per_slab < nup ? r0 + rows_per_slab : nup;
    const double* vj = V + (size_t)j * vstride;
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] = fma(vj[(size_t)r * R + c], w[(size_t)r * R + c], acc[c]);
    }
    block_sum<R>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < R; ++c) part[((size_t)j * nslab + slab) * R + c] = acc[c];
}

// s[j][c] = sum over slabs of part (fixed order); out[j][c] = s, and
// out2[j][c] = base[j][c] + s when out2 is given.
template <int R>
__global__ void k_ms_reduce(const double* __restrict__ part, int nslab, int nvec, double* __restrict__ out,
                            const double* __restrict__ base, double* __restrict__ out2,
                            const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nvec * R) return;
    const int j = t / R, c = t - j * R;
    double s = 0.0;
    for (int q = 0; q < nslab; ++q) s += part[((size_t)j * nslab + q) * R + c];
    out[t] = s;
    if (out2) out2[t] = base[t] + s;
}

// w -= sum_j V_j s[j] over the vectors of split blockIdx.y; with one split the
// result goes to w, else the split's sum goes to part2[split] for k_ms_combine.
template <int R>
__global__ __launch_bounds__(256) void k_ms_update(const double* __restrict__ V, int64_t vstride, int nvec,
                                                   const double* __restrict__ s, double* __restrict__ w,
                                                   double* __restrict__ part2, int64_t nup, int vecs_per_split,
                                                   const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nup) return;
    const int j0 = blockIdx.y * vecs_per_split;
    const int j1 = j0 + vecs_per_split < nvec ? j0 + vecs_per_split : nvec;
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double* vj = V + (size_t)j * vstride + (size_t)r * R;
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] = fma(vj[c], s[j * R + c], acc[c]);
    }
    if (gridDim.y == 1) {
#pragma unroll
        for (int c = 0; c < R; ++c) w[(size_t)r * R + c] -= acc[c];
    } else {
#pragma unroll
        for (int c = 0; c < R; ++c) part2[((size_t)blockIdx.y * nup + r) * R + c] = acc[c];
    }
}

template <int R>
__global__ void k_ms_combine(const double* __restrict__ part2, int nsplit, double* __restrict__ w, int64_t nup,
                             const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nup * R) return;
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += part2[(size_t)q * nup * R + t];
    w[t] -= s;
}

// V_next = w / ||w|| per slot (zero for a zero norm: an invariant subspace,
// where every shift of that polarization has converged); hnext[c] = ||w||.
template <int R>
__global__ void k_ms_normalize(const double* __restrict__ w, const double* __restrict__ nrm2,
                               double* __restrict__ vnext, double* __restrict__ hnext, int64_t nup,
                               const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < R) hnext[t] = sqrt(nrm2[t]);
    if (t >= nup * R) return;
    const int c = (int)(t % R);
    const double b = sqrt(nrm2[c]);
    vnext[t] = b > 0.0 ? w[t] / b : 0.0;
}

// Hessenberg column K of polarization c, entry j, with the shift on the diagonal.
__device__ __forceinline__ double2 hs(const double* __restrict__ hpk, int R, int c, int K, int j, double2 zp)
{
    const double h = hpk[((size_t)K * (K + 3) / 2 + j) * R + c];
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
                                          const double* __restrict__ hpk, int R, int c, int P, int p, int k0, int nb,
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
                if (q < nb) b.h[u][q] = hpk[((size_t)l * (l + 3) / 2 + j + 1) * R + c];
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
__global__ __launch_bounds__(64) void k_ms_givens(const double* __restrict__ hpk, int R, int npol, int P, int k0,
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
        if (q < kn) a[q] = hs(hpk, R, c, k0 + q, 0, zp);
    RotBatch b0, b1;
    load_rots(b0, cs, sn, hpk, R, c, P, p, k0, kn, 0);
    for (int j0 = 0; j0 < k0; j0 += 2 * GU) {
        load_rots(b1, cs, sn, hpk, R, c, P, p, k0, kn, j0 + GU);
        apply_rots(b0, a, k0, kn, j0, zp);
        load_rots(b0, cs, sn, hpk, R, c, P, p, k0, kn, j0 + 2 * GU);
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
            if (t < q) (void)rotate(rc[t], rs[t], u, hs(hpk, R, c, K, k0 + t + 1, zp));
        const double beta = hpk[((size_t)K * (K + 3) / 2 + K + 1) * R + c];
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
__global__ __launch_bounds__(64) void k_ms_rfactor(const double* __restrict__ hpk, int R, int npol, int P, int kmax,
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
    double2 a = hs(hpk, R, c, l, 0, zp);
    const double* hl = hpk + (size_t)l * (l + 3) / 2 * R;
#pragma unroll 4
    for (int j = 0; j < l; ++j) {
        const double hv = hl[(j + 1) * R + c];
        const double2 b = j + 1 == l ? make_double2(hv - zp.x, -zp.y) : make_double2(hv, 0.0);
        rst[rpk(l, j) * P + p] = rotate(cs[(size_t)j * P + p], sn[(size_t)j * P + p], a, b);
    }
    const double cl = cs[(size_t)l * P + p];
    const double2 sl = sn[(size_t)l * P + p];
    const double beta = hl[(l + 1) * R + c];
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

// x[row][p] = sum_j V_j[row][slot(p)] y[j][p] for K basis vectors: tiles of
// 32 rows x 64 pairs, 16 basis vectors per LDS stage.
template <int R>
__global__ __launch_bounds__(256) void k_ms_xcombine(const double* __restrict__ V, int64_t vstride, int K,
                                                     const double2* __restrict__ y, int npol, int P,
                                                     double2* __restrict__ x, int ldx, int64_t nup)
{
    constexpr int TR = 32, TP = 64, TJ = 16;
    __shared__ double sv[TJ][TR][R];
    __shared__ double2 sy[TJ][TP];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    const int p0 = blockIdx.y * TP;
    const int p = p0 + tx;
    const int c = p % npol;
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

int ms_slabs(int64_t nup, int nvec)
{
    int64_t maxs = (nup + 255) / 256;
    int64_t want = (2048 + nvec - 1) / nvec;
    if (want < 1) want = 1;
    if (want > maxs) want = maxs;
    return (int)want;
}

int ms_update_splits(int64_t nup, int nvec)
{
    const int64_t rb = (nup + 255) / 256;
    int64_t want = (1024 + rb - 1) / rb;
    const int64_t maxs = (nvec + 15) / 16;
    if (want > maxs) want = maxs;
    if (want < 1) want = 1;
    return (int)want;
}

void ms_init(int R, const double2* b, int ldb, int npol, const double* bnorm, double* V0, int64_t nup, hipStream_t st)
{
    const dim3 grid((unsigned)((nup + 255) / 256));
    if (R == 2) hipLaunchKernelGGL(k_ms_init<2>, grid, dim3(256), 0, st, b, ldb, npol, bnorm, V0, nup);
    else hipLaunchKernelGGL(k_ms_init<4>, grid, dim3(256), 0, st, b, ldb, npol, bnorm, V0, nup);
}

void ms_spmv(int R, const Geometry& g, const double* Y, double* w, hipStream_t st, const int32_t* stop)
{
    const dim3 grid((unsigned)((g.np + 255) / 256));
    if (R == 2)
        hipLaunchKernelGGL(k_ms_spmv<2>, grid, dim3(256), 0, st, g.row_ptr, g.col, g.val, Y, w, g.n, g.np, stop);
    else
        hipLaunchKernelGGL(k_ms_spmv<4>, grid, dim3(256), 0, st, g.row_ptr, g.col, g.val, Y, w, g.n, g.np, stop);
}

void ms_dots(int R, const double* V, int64_t vstride, int nvec, const double* w, double* part, int64_t nup,
             double* out, const double* base, double* out2, hipStream_t st, const int32_t* stop)
{
    const int nslab = ms_slabs(nup, nvec);
    const int64_t rps = (nup + nslab - 1) / nslab;
    const dim3 grid((unsigned)nslab, (unsigned)nvec);
    const dim3 rg((unsigned)((nvec * R + 255) / 256));
    if (R == 2) {
        hipLaunchKernelGGL(k_ms_dots<2>, grid, dim3(256), 0, st, V, vstride, w, part, nup, rps, stop);
        hipLaunchKernelGGL(k_ms_reduce<2>, rg, dim3(256), 0, st, part, nslab, nvec, out, base, out2, stop);
    } else {
        hipLaunchKernelGGL(k_ms_dots<4>, grid, dim3(256), 0, st, V, vstride, w, part, nup, rps, stop);
        hipLaunchKernelGGL(k_ms_reduce<4>, rg, dim3(256), 0, st, part, nslab, nvec, out, base, out2, stop);
    }
}

void ms_update(int R, const double* V, int64_t vstride, int nvec, const double* s, double* w, double* part2,
               int64_t nup, hipStream_t st, const int32_t* stop)
{
    const int nsplit = ms_update_splits(nup, nvec);
    const int vps = (nvec + nsplit - 1) / nsplit;
    const int nsp = (nvec + vps - 1) / vps;
    const dim3 grid((unsigned)((nup + 255) / 256), (unsigned)nsp);
    const dim3 cg((unsigned)((nup * R + 255) / 256));
    if (R == 2) {
        hipLaunchKernelGGL(k_ms_update<2>, grid, dim3(256), 0, st, V, vstride, nvec, s, w, part2, nup, vps, stop);
        if (nsp > 1) hipLaunchKernelGGL(k_ms_combine<2>, cg, dim3(256), 0, st, part2, nsp, w, nup, stop);
    } else {
        hipLaunchKernelGGL(k_ms_update<4>, grid, dim3(256), 0, st, V, vstride, nvec, s, w, part2, nup, vps, stop);
        if (nsp > 1) hipLaunchKernelGGL(k_ms_combine<4>, cg, dim3(256), 0, st, part2, nsp, w, nup, stop);
    }
}

size_t ms_part_doubles(int R, int64_t nup, int nvec_max)
{
    size_t a = 0;
    for (int nv : {1, nvec_max}) {
        const size_t s = (size_t)ms_slabs(nup, nv) * nv * R;
        if (s > a) a = s;
    }
    // ms_slabs(nup, nv) * nv is at most max(nv, 2048 + nv) over nv
    const size_t b = (size_t)(2048 + nvec_max) * R;
    return a > b ? a : b;
}

size_t ms_part2_doubles(int R, int64_t nup, int nvec_max)
{
    int mx = 1;
    for (int nv = 1; nv <= nvec_max; ++nv) {
        const int nsplit = ms_update_splits(nup, nv);
        const int vps = (nv + nsplit - 1) / nsplit;
        const int nsp = (nv + vps - 1) / vps;
        if (nsp > mx) mx = nsp;
    }
    return (size_t)mx * nup * R;
}

void ms_normalize(int R, const double* w, const double* nrm2, double* vnext, double* hnext, int64_t nup,
                  hipStream_t st, const int32_t* stop)
{
    const dim3 grid((unsigned)((nup * R + 255) / 256));
    if (R == 2) hipLaunchKernelGGL(k_ms_normalize<2>, grid, dim3(256), 0, st, w, nrm2, vnext, hnext, nup, stop);
    else hipLaunchKernelGGL(k_ms_normalize<4>, grid, dim3(256), 0, st, w, nrm2, vnext, hnext, nup, stop);
}

int ms_givens_batch() { return GB; }

void ms_givens(const double* hpk, int R, int npol, int P, int k0, int kn, const double2* z, double* cs, double2* sn,
               double2* g, const double* target, int32_t* done, double* resid, int32_t* ndone, int32_t* stop,
               hipStream_t st)
{
    hipLaunchKernelGGL(k_ms_givens, dim3((unsigned)((P + 63) / 64)), dim3(64), 0, st, hpk, R, npol, P, k0, kn, z, cs,
                       sn, g, target, done, resid, ndone, stop);
}

void ms_rfactor(const double* hpk, int R, int npol, int P, int kmax, const double2* z, const double* cs,
                const double2* sn, const int32_t* done, double2* rst, hipStream_t st)
{
    if (kmax < 1) return;
    hipLaunchKernelGGL(k_ms_rfactor, dim3((unsigned)((P + 63) / 64), (unsigned)kmax), dim3(64), 0, st, hpk, R, npol,
                       P, kmax, z, cs, sn, done, rst);
}

size_t ms_rst_elems(int P, int kcap) { return (size_t)kcap * (kcap + 1) / 2 * P; }

void ms_backsub(const double2* rst, int P, int kmax, const int32_t* done, const double2* g, double2* y, hipStream_t st)
{
    hipLaunchKernelGGL(k_ms_backsub, dim3((unsigned)P), dim3(256), sizeof(double2) * kmax, st, rst, P, kmax, done, g,
                       y);
}

void ms_xcombine(int R, const double* V, int64_t vstride, int K, const double2* y, int npol, int P, double2* x,
                 int ldx, int64_t nup, hipStream_t st)
{
    const dim3 grid((unsigned)((nup + 31) / 32), (unsigned)((P + 63) / 64));
    if (R == 2)
        hipLaunchKernelGGL(k_ms_xcombine<2>, grid, dim3(256), 0, st, V, vstride, K, y, npol, P, x, ldx, nup);
    else
        hipLaunchKernelGGL(k_ms_xcombine<4>, grid, dim3(256), 0, st, V, vstride, K, y, npol, P, x, ldx, nup);
}

}  // namespace px
