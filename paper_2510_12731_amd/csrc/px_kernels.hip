// Geometry set-up, sparse Kbar, and the column-blocked Krylov kernels.
//
// Column conventions: a block of na complex columns is stored row-major as
// double2 [rows][lda] (lda >= na, padded columns kept at zero), so every
// per-column operation is a coalesced sweep over consecutive columns.  Column
// reductions (dot products, norms, dipoles) use a fixed chunking of the rows
// and a fixed summation order, so a column's arithmetic never depends on which
// other columns share the block.
#include "px_internal.h"
#include "px_neighbors.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace px {
namespace {

constexpr double TWO_PI = 6.283185307179586;
constexpr double C_LIGHT = 137.035999084;   // speed of light, a.u. (CODATA 2018)
constexpr double ANG = 0.529177210903;       // Angstrom per bohr (CODATA 2018)

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b)   // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// ---------------------------------------------------------------- geometry

__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton(const double* __restrict__ xyz, int64_t n, int64_t npow, double3 lo, double3 scale,
                         uint64_t* __restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow) return;
    if (i >= n) {
        keys[i] = ~0ull;
        return;
    }
    uint32_t qx = (uint32_t)fmin(1023.0, fmax(0.0, (xyz[3 * i] - lo.x) * scale.x));
    uint32_t qy = (uint32_t)fmin(1023.0, fmax(0.0, (xyz[3 * i + 1] - lo.y) * scale.y));
    uint32_t qz = (uint32_t)fmin(1023.0, fmax(0.0, (xyz[3 * i + 2] - lo.z) * scale.z));
    uint32_t code = spread10(qx) | (spread10(qy) << 1) | (spread10(qz) << 2);
    keys[i] = ((uint64_t)code << 32) | (uint64_t)i;
}

__global__ void k_bitonic(uint64_t* __restrict__ a, uint32_t j, uint32_t k, uint32_t npow)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow) return;
    uint32_t l = i ^ j;
    if (l > i) {
        bool up = (i & k) == 0;
        uint64_t x = a[i], y = a[l];
        if ((x > y) == up) {
            a[i] = y;
            a[l] = x;
        }
    }
}

// Sorted coordinates; ghosts (rows n..np-1) parked on a far line, 50 bohr apart.
__global__ void k_gather_sorted(const double* __restrict__ xyz, const uint64_t* __restrict__ keys, int64_t n,
                                int64_t np, double3 far0, int32_t* __restrict__ perm, double4* __restrict__ x64,
                                float4* __restrict__ x32)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double4 p;
    if (i < n) {
        int64_t o = (int64_t)(keys[i] & 0xffffffffull);
        perm[i] = (int32_t)o;
        p = make_double4(xyz[3 * o], xyz[3 * o + 1], xyz[3 * o + 2], 0.0);
    } else {
        p = make_double4(far0.x + 50.0 * (double)(i - n), far0.y, far0.z, 0.0);
    }
    x64[i] = p;
    x32[i] = make_float4((float)p.x, (float)p.y, (float)p.z, 0.0f);
}

// Conservative FP32 bounding box of every group of GROUP atoms.
__global__ void k_group_bbox(const double4* __restrict__ x64, int64_t ngroups, float4* __restrict__ lo,
                             float4* __restrict__ hi)
{
    int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= ngroups) return;
    double l[3] = {1e300, 1e300, 1e300}, h[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < GROUP; ++k) {
        double4 p = x64[gi * GROUP + k];
        l[0] = fmin(l[0], p.x); l[1] = fmin(l[1], p.y); l[2] = fmin(l[2], p.z);
        h[0] = fmax(h[0], p.x); h[1] = fmax(h[1], p.y); h[2] = fmax(h[2], p.z);
    }
    const double pad = 1e-3;
    lo[gi] = make_float4((float)(l[0] - pad), (float)(l[1] - pad), (float)(l[2] - pad), 0.f);
    hi[gi] = make_float4((float)(h[0] + pad), (float)(h[1] + pad), (float)(h[2] + pad), 0.f);
}

struct KappaConst {
    double a_eff, fd, s_r0, rc, rc2, min_r;
};

// Exchange constants of the pair types AA, AB (= BA), BB; homogeneous
// structures use k[0] only (type == nullptr).
struct KappaSet {
    KappaConst k[3];
    double rc_max;
};

// Eqs. (fermi), (kappa): K_ij = [1 - f(r)] A / r for r <= cutoff.
__device__ __forceinline__ double kappa_val(double r, const KappaConst& k)
{
    double f = 1.0 / (1.0 + exp(-k.fd * (r / k.s_r0 - 1.0)));
    return (1.0 - f) * k.a_eff / r;
}

// Neighbour search over the real atoms, one thread per row atom, 64 rows per
// (one-wave) workgroup x = blockIdx.x, the row block's candidate source
// groups shared out over gridDim.y subsets (px_neighbors.h).  Pass 0 counts
// each subset's off-diagonal entries of the row (cntw[sub][i]) and flags
// coincident atoms; pass 1 fills them, subset after subset (columns
// increasing within a subset), leaving the row's last slot to k_kbar_diag.
template <int PASS>
__global__ __launch_bounds__(64) void k_kbar_rows(const double4* __restrict__ x64, const float4* __restrict__ glo,
                                                  const float4* __restrict__ ghi, int64_t n, int64_t np,
                                                  KappaSet ks, const uint8_t* __restrict__ type,
                                                  int32_t* __restrict__ cntw,
                                                  const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                  double* __restrict__ val, int* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int sub = blockIdx.y, nsub = gridDim.y;
    const double4 pi = x64[i];
    const bool row = i < n;
    const float lim = (float)(ks.rc_max * 1.0001 + 1e-3);
    const double lim2 = (double)lim * (double)lim;   // r^2 prefilter, above every pair type's cutoff
    const int ti = (type && row) ? type[i] : 0;
    int count = 0;
    int64_t out = 0;
    if (PASS == 1 && row) {
        out = row_ptr[i];
        for (int t = 0; t < sub; ++t) out += cntw[(size_t)t * np + i];
    }
    nbr::for_near_atoms(x64, n, glo, ghi, lim, (int64_t)blockIdx.x, sub, nsub, [&](int64_t j, const double4& pj) {
        if (!row) return;
        if (j == i) return;
        const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > lim2) return;
        const double r = sqrt(r2);
        const KappaConst& kc = ks.k[type ? ti + type[j] : 0];
        if (PASS == 0 && r < kc.min_r) *bad = 1;
        if (r <= kc.rc) {
            if (PASS == 0) {
                ++count;
            } else {
                col[out] = (int32_t)j;
                val[out] = kappa_val(r, kc);
                ++out;
            }
        }
    });
    if (PASS == 0 && row) cntw[(size_t)sub * np + i] = count;
}

// cnt[i] = add + sum over the nsub subsets of cntw[s][i], i < n.
__global__ void k_count_sum(const int32_t* __restrict__ cntw, int nsub, int64_t np, int64_t n, int32_t add,
                            int32_t* __restrict__ cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = add;
    for (int s = 0; s < nsub; ++s) c += cntw[(size_t)s * np + i];
    cnt[i] = c;
}

// The diagonal of each row of Kbar in its last slot: Kbar_ii = -sum_k K_ik
// over the row's other entries, in slot order.
__global__ void k_kbar_diag(const int32_t* __restrict__ row_ptr, int64_t n, int32_t* __restrict__ col,
                            double* __restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t d = row_ptr[i + 1] - 1;
    double s = 0.0;
    for (int32_t e = row_ptr[i]; e < d; ++e) s += val[e];
    col[d] = (int32_t)i;
    val[d] = -s;
}

// Exclusive scan of cnt[0..n) into row_ptr[0..n], single workgroup.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ cnt, int64_t n,
                                               int32_t* __restrict__ row_ptr)
{
    __shared__ int32_t s[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        int64_t i = base + threadIdx.x;
        int32_t v = (i < n) ? cnt[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int32_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) row_ptr[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) row_ptr[n] = carry;
}

// Atom types in Morton order (ghost atoms type A).
__global__ void k_gather_types(const uint8_t* __restrict__ types, const int32_t* __restrict__ perm, int64_t n,
                               int64_t np, uint8_t* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    out[i] = i < n ? types[perm[i]] : 0;
}

// Per row of a two-type structure: the exchange K summed over same-type and
// over other-type neighbours, and the two neighbour counts (Eq. polar-finale).
__global__ void k_het_rows(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ cv, const uint8_t* __restrict__ type, int64_t n,
                           double4* __restrict__ hrow)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ti = type[i];
    double ks = 0.0, ko = 0.0;
    int ns = 0, no = 0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = ci[e];
        if (j == i) continue;
        if (type[j] == ti) {
            ks += cv[e];
            ++ns;
        } else {
            ko += cv[e];
            ++no;
        }
    }
    hrow[i] = make_double4(ks, ko, (double)ns, (double)no);
}

// ---------------------------------------------------------------- sparse

// W = S [diag(Kbar, I) Y - diag(z_q, z_mu) X]        (mode B == nullptr)
// W = B - S [diag(Kbar, I) Y - diag(z_q, z_mu) X]    (residual mode)
// with S = diag(I, mu_sign I): the solver negates the dipole rows (mu_sign =
// -1), which leaves solution and residual norms unchanged and makes
// diag(Kbar, -I) T similar to a symmetric negative semidefinite matrix, so
// both diagonal shifts push every eigenvalue into the upper half plane.
// Y: real [nup][ldy] (FP32 or FP64), complex column c = real columns (2c, 2c+1).
template <typename TY>
__global__ __launch_bounds__(256) void k_spmm_shift(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                    const double* __restrict__ cv, const TY* __restrict__ Y, int ldy,
                                                    const double2* __restrict__ X, const double2* __restrict__ zq,
                                                    const double2* __restrict__ zmu,
                                                    const double2* __restrict__ B, double2* __restrict__ W,
                                                    int64_t n, int64_t np, int64_t nup, int na, int lda,
                                                    double mu_sign,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= lda) return;
    const size_t o = (size_t)r * lda + c;
    const int64_t comp = r / np, i = r - comp * np;
    if (c >= na || i >= n) {
        W[o] = make_double2(0.0, 0.0);
        return;
    }
    double ar = 0.0, ai = 0.0;
    double2 z;
    if (comp == 0) {
        const int32_t e1 = rp[i + 1];
        for (int32_t e = rp[i]; e < e1; ++e) {
            const double k = cv[e];
            const TY* yr = Y + (size_t)ci[e] * ldy + 2 * c;
            ar = fma(k, (double)yr[0], ar);
            ai = fma(k, (double)yr[1], ai);
        }
        z = zq[c];
    } else {
        const TY* yr = Y + (size_t)r * ldy + 2 * c;
        ar = (double)yr[0];
        ai = (double)yr[1];
        z = zmu[c];
    }
    const double2 x = X[o];
    double2 w = make_double2(ar - (z.x * x.x - z.y * x.y), ai - (z.x * x.y + z.y * x.x));
    if (comp != 0) w = make_double2(mu_sign * w.x, mu_sign * w.y);
    if (B != nullptr) {
        const double2 b = B[o];
        w = make_double2(b.x - w.x, b.y - w.y);
    }
    W[o] = w;
}

// b = E0 Kbar r_l (charge rows) and mu_sign E0 e_l (dipole rows) for column c
// with polarization col_pol[c]: the right-hand side -Kbar V, V_i = -E0 r_i.l,
// and the field E (dipole rows scaled like the operator's, see k_spmm_shift).
__global__ __launch_bounds__(256) void k_rhs(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                             const double* __restrict__ cv, const double4* __restrict__ x64,
                                             const int32_t* __restrict__ col_pol, double e0, double2* __restrict__ b,
                                             int64_t n, int64_t np, int64_t nup, int ncol, int ldb, double mu_sign)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= ldb) return;
    const size_t o = (size_t)r * ldb + c;
    const int64_t comp = r / np, i = r - comp * np;
    if (c >= ncol || i >= n) {
        b[o] = make_double2(0.0, 0.0);
        return;
    }
    const int l = col_pol[c];
    double v = 0.0;
    if (comp == 0) {
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const double4 p = x64[ci[e]];
            const double coord = (l == 0) ? p.x : (l == 1) ? p.y : p.z;
            v = fma(cv[e], coord, v);
        }
        v *= e0;
    } else {
        v = (comp - 1 == l) ? mu_sign * e0 : 0.0;
    }
    b[o] = make_double2(v, 0.0);
}

// Two atom types (Eq. wfqfmu-leghe): the charge rows apply
// S(w) = (Kbar + Hbar(w)) / 2, whose off-diagonal entries are K_ij for like
// pairs and gamma_{t_i}(w) K_ij for unlike ones, gamma_t = (1 + rho_t phi_t) / 2,
// and whose diagonal is -(Ks_i + gamma_{t_i} Ko_i) (hrow: same-type and
// other-type row sums of K).  Shifts per atom: z_q of the atom's type, and
// z_mu,i = -[(N_same + 1) / alpha_t + N_other / alpha_o] / (N + 1)
// (Eq. polar-finale).  het: [6][lda] complex per column: z_q,A, z_q,B,
// gamma_A, gamma_B, 1/alpha_IB,A, 1/alpha_IB,B.  Otherwise as k_spmm_shift.
template <typename TY>
__global__ __launch_bounds__(256) void k_spmm_het(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                  const double* __restrict__ cv, const uint8_t* __restrict__ type,
                                                  const double4* __restrict__ hrow, const TY* __restrict__ Y,
                                                  int ldy, const double2* __restrict__ X,
                                                  const double2* __restrict__ het, const double2* __restrict__ B,
                                                  double2* __restrict__ W, int64_t n, int64_t np, int64_t nup,
                                                  int na, int lda, double mu_sign, const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= lda) return;
    const size_t o = (size_t)r * lda + c;
    const int64_t comp = r / np, i = r - comp * np;
    if (c >= na || i >= n) {
        W[o] = make_double2(0.0, 0.0);
        return;
    }
    const int ti = type[i];
    double ar = 0.0, ai = 0.0;
    double2 z;
    if (comp == 0) {
        const double2 g = het[(2 + ti) * (size_t)lda + c];
        double lr = 0.0, li = 0.0, ur = 0.0, ui = 0.0;   // like and unlike neighbour sums
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int32_t j = ci[e];
            if (j == i) continue;
            const double k = cv[e];
            const TY* yr = Y + (size_t)j * ldy + 2 * c;
            if (type[j] == ti) {
                lr = fma(k, (double)yr[0], lr);
                li = fma(k, (double)yr[1], li);
            } else {
                ur = fma(k, (double)yr[0], ur);
                ui = fma(k, (double)yr[1], ui);
            }
        }
        const double4 h = hrow[i];
        const TY* yi = Y + (size_t)i * ldy + 2 * c;
        const double dr = -(h.x + g.x * h.y), di = -(g.y * h.y);          // S_ii
        const double y0 = (double)yi[0], y1 = (double)yi[1];
        ar = lr + (g.x * ur - g.y * ui) + (dr * y0 - di * y1);
        ai = li + (g.x * ui + g.y * ur) + (dr * y1 + di * y0);
        z = het[(size_t)ti * lda + c];
    } else {
        const TY* yr = Y + (size_t)r * ldy + 2 * c;
        ar = (double)yr[0];
        ai = (double)yr[1];
        const double4 h = hrow[i];
        const double2 own = het[(4 + ti) * (size_t)lda + c], oth = het[(5 - ti) * (size_t)lda + c];
        const double inv = 1.0 / (h.z + h.w + 1.0);
        z = make_double2(-((h.z + 1.0) * own.x + h.w * oth.x) * inv, -((h.z + 1.0) * own.y + h.w * oth.y) * inv);
    }
    const double2 x = X[o];
    double2 w = make_double2(ar - (z.x * x.x - z.y * x.y), ai - (z.x * x.y + z.y * x.x));
    if (comp != 0) w = make_double2(mu_sign * w.x, mu_sign * w.y);
    if (B != nullptr) {
        const double2 b = B[o];
        w = make_double2(b.x - w.x, b.y - w.y);
    }
    W[o] = w;
}

// Right-hand side of a two-type structure: diag(S(w_c), I) (-V; E) per
// column, -V_j = E0 r_j.l; gam: [2][ldg] gamma_A, gamma_B of each column.
__global__ __launch_bounds__(256) void k_rhs_het(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const double* __restrict__ cv, const uint8_t* __restrict__ type,
                                                 const double4* __restrict__ hrow, const double4* __restrict__ x64,
                                                 const int32_t* __restrict__ col_pol, const double2* __restrict__ gam,
                                                 double e0, double2* __restrict__ b, int64_t n, int64_t np,
                                                 int64_t nup, int ncol, int ldb, double mu_sign)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= ldb) return;
    const size_t o = (size_t)r * ldb + c;
    const int64_t comp = r / np, i = r - comp * np;
    if (c >= ncol || i >= n) {
        b[o] = make_double2(0.0, 0.0);
        return;
    }
    const int l = col_pol[c];
    if (comp != 0) {
        b[o] = make_double2((comp - 1 == l) ? mu_sign * e0 : 0.0, 0.0);
        return;
    }
    const int ti = type[i];
    const double2 g = gam[(size_t)ti * ldb + c];
    double lv = 0.0, uv = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = ci[e];
        if (j == i) continue;
        const double4 p = x64[j];
        const double coord = (l == 0) ? p.x : (l == 1) ? p.y : p.z;
        if (type[j] == ti) lv = fma(cv[e], coord, lv);
        else uv = fma(cv[e], coord, uv);
    }
    const double4 h = hrow[i];
    const double4 p = x64[i];
    const double xi = (l == 0) ? p.x : (l == 1) ? p.y : p.z;
    const double vr = lv + g.x * uv - (h.x + g.x * h.y) * xi;
    const double vi = g.y * uv - g.y * h.y * xi;
    b[o] = make_double2(e0 * vr, e0 * vi);
}

// ---------------------------------------------------------------- Arnoldi

// Column reductions over chunks of ARN_ROWS rows: a 256-thread block (4 waves
// x 64 columns) covers one chunk; wave w takes rows w, w+4, ... and the four
// wave sums are added in a fixed order through LDS.

// partial[chunk][j][c] = sum over the chunk's rows of conj(V_j[r][c]) w[r][c],
// for the ARN_JB basis vectors j0.. of this block (grid.z).
__global__ __launch_bounds__(256) void k_col_dots(const double2* __restrict__ V, int64_t vstride, int nvec,
                                                  const double2* __restrict__ w, double2* __restrict__ partial,
                                                  int na, int lda, int64_t nup)
{
    __shared__ double2 red[4][ARN_JB][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.y * 64 + lane;
    const int j0 = blockIdx.z * ARN_JB;
    const int nj = min(ARN_JB, nvec - j0);
    const int64_t r0 = (int64_t)blockIdx.x * ARN_ROWS;
    const int64_t r1 = min(nup, r0 + ARN_ROWS);
    double ar[ARN_JB], ai[ARN_JB];
#pragma unroll
    for (int q = 0; q < ARN_JB; ++q) ar[q] = ai[q] = 0.0;
    if (c < na) {
        const double2* vb = V + (size_t)j0 * vstride + c;
        for (int64_t r = r0 + wave; r < r1; r += 4) {
            const double2 x = w[(size_t)r * lda + c];
#pragma unroll
            for (int q = 0; q < ARN_JB; ++q) {
                if (q < nj) {
                    const double2 v = vb[(size_t)q * vstride + (size_t)r * lda];
                    ar[q] = fma(v.x, x.x, fma(v.y, x.y, ar[q]));
                    ai[q] = fma(v.x, x.y, fma(-v.y, x.x, ai[q]));
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < ARN_JB; ++q) red[wave][q][lane] = make_double2(ar[q], ai[q]);
    __syncthreads();
    if (wave == 0 && c < na) {
        for (int q = 0; q < nj; ++q) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sr += red[k][q][lane].x;
                si += red[k][q][lane].y;
            }
            partial[((size_t)blockIdx.x * nvec + j0 + q) * lda + c] = make_double2(sr, si);
        }
    }
}

__global__ void k_reduce_dots(const double2* __restrict__ partial, int nchunk, int nvec, double2* __restrict__ h,
                              int na, int lda)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nvec * lda) return;
    const int j = t / lda, c = t - j * lda;
    if (c >= na) return;
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < nchunk; ++k) {
        const double2 p = partial[((size_t)k * nvec + j) * lda + c];
        ar += p.x;
        ai += p.y;
    }
    h[(size_t)j * lda + c] = make_double2(ar, ai);
}

// w -= sum_j V_j h_j (per column); with norm_partial, also |w|^2 per chunk of
// UPD_ROWS rows.  A 256-thread block covers UPD_ROWS rows x 64 columns; each
// wave updates ARN_RG consecutive rows, so every h_j load feeds ARN_RG basis
// loads, and the basis loop is unrolled by two for more loads in flight.
__global__ __launch_bounds__(256) void k_col_update(const double2* __restrict__ V, int64_t vstride, int nvec,
                                                    const double2* __restrict__ h, double2* __restrict__ w,
                                                    double* __restrict__ norm_partial, int na, int lda, int64_t nup)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.y * 64 + lane;
    const int64_t rg = (int64_t)blockIdx.x * UPD_ROWS + wave * ARN_RG;
    const int nr = (int)max((int64_t)0, min((int64_t)ARN_RG, nup - rg));
    double nrm = 0.0;
    if (c < na && nr > 0) {
        double2 acc[ARN_RG];
#pragma unroll
        for (int q = 0; q < ARN_RG; ++q)
            acc[q] = (q < nr) ? w[(size_t)(rg + q) * lda + c] : make_double2(0.0, 0.0);
        const double2* vb = V + (size_t)rg * lda + c;
        int j = 0;
        for (; j + 1 < nvec; j += 2) {
            const double2 h0 = h[(size_t)j * lda + c];
            const double2 h1 = h[(size_t)(j + 1) * lda + c];
            const double2* v0 = vb + (size_t)j * vstride;
            const double2* v1 = v0 + vstride;
#pragma unroll
            for (int q = 0; q < ARN_RG; ++q) {
                if (q < nr) {
                    const double2 a = v0[(size_t)q * lda];
                    const double2 b = v1[(size_t)q * lda];
                    acc[q].x -= (a.x * h0.x - a.y * h0.y) + (b.x * h1.x - b.y * h1.y);
                    acc[q].y -= (a.x * h0.y + a.y * h0.x) + (b.x * h1.y + b.y * h1.x);
                }
            }
        }
        if (j < nvec) {
            const double2 h0 = h[(size_t)j * lda + c];
            const double2* v0 = vb + (size_t)j * vstride;
#pragma unroll
            for (int q = 0; q < ARN_RG; ++q) {
                if (q < nr) {
                    const double2 a = v0[(size_t)q * lda];
                    acc[q].x -= a.x * h0.x - a.y * h0.y;
                    acc[q].y -= a.x * h0.y + a.y * h0.x;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < ARN_RG; ++q) {
            if (q < nr) {
                w[(size_t)(rg + q) * lda + c] = acc[q];
                nrm = fma(acc[q].x, acc[q].x, fma(acc[q].y, acc[q].y, nrm));
            }
        }
    }
    if (norm_partial) {
        red[wave][lane] = nrm;
        __syncthreads();
        if (wave == 0 && c < na)
            norm_partial[(size_t)blockIdx.x * lda + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    }
}

__global__ __launch_bounds__(256) void k_col_norm_partial(const double2* __restrict__ w, double* __restrict__ partial,
                                                          int na, int lda, int64_t nup)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.y * 64 + lane;
    const int64_t r0 = (int64_t)blockIdx.x * ARN_ROWS;
    const int64_t r1 = min(nup, r0 + ARN_ROWS);
    double nrm = 0.0;
    if (c < na)
        for (int64_t r = r0 + wave; r < r1; r += 4) {
            const double2 a = w[(size_t)r * lda + c];
            nrm = fma(a.x, a.x, fma(a.y, a.y, nrm));
        }
    red[wave][lane] = nrm;
    __syncthreads();
    if (wave == 0 && c < na)
        partial[(size_t)blockIdx.x * lda + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// nrm[c] = sqrt(sum_k partial[k][c]); 256 threads = 64 columns x 4 waves, wave
// w sums chunks w, w+4, ...; the four sums are combined in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_norms(const double* __restrict__ partial, int nchunk,
                                                      double* __restrict__ nrm, int na, int lda,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (c < na)
        for (int k = wave; k < nchunk; k += 4) s += partial[(size_t)k * lda + c];
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && c < na) nrm[c] = sqrt(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
}

// v = w / ||w|| (zero for finished or padded columns), plus the FP32 copy in
// the real layout [rows][2*lda] when x32 != nullptr.
__global__ __launch_bounds__(256) void k_normalize(const double2* __restrict__ w, const double* __restrict__ nrm,
                                                   const int32_t* __restrict__ done, double2* __restrict__ v,
                                                   float* __restrict__ x32, int na, int lda, int64_t nup,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= lda) return;
    const size_t o = (size_t)r * lda + c;
    double2 out = make_double2(0.0, 0.0);
    if (c < na && !(done && done[c]) && nrm[c] > 0.0) {
        const double s = 1.0 / nrm[c];
        const double2 a = w[o];
        out = make_double2(a.x * s, a.y * s);
    }
    v[o] = out;
    if (x32) {
        float2* xp = reinterpret_cast<float2*>(x32 + (size_t)r * 2 * lda + 2 * c);
        *xp = make_float2((float)out.x, (float)out.y);
    }
}

__global__ __launch_bounds__(256) void k_to_f32(const double2* __restrict__ v, float* __restrict__ x32, int na,
                                                int lda, int64_t nup)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= lda) return;
    const double2 a = (c < na) ? v[(size_t)r * lda + c] : make_double2(0.0, 0.0);
    *reinterpret_cast<float2*>(x32 + (size_t)r * 2 * lda + 2 * c) = make_float2((float)a.x, (float)a.y);
}

// One Arnoldi column of the Hessenberg matrix through the stored Givens
// rotations (complex rotations, real cosine), the new rotation, and the
// least-squares residual estimate |g_{k+1}|.
//   R  [m][m+1][lda]  (column k holds R_{0..k,k}),  cs [m][lda], sn [m][lda]
//   g  [m+1][lda]
// Rotates column k of R (rows 0..k already hold the Hessenberg entries,
// bb = the real sub-diagonal entry H_{k+1,k}) through the stored rotations,
// forms rotation k and updates g, steps and done.
__device__ void rotate_column(int k, int m, int c, int lda, double bb, double2* __restrict__ R,
                              double* __restrict__ cs, double2* __restrict__ sn, double2* __restrict__ g,
                              const double* __restrict__ target, int32_t* __restrict__ done,
                              int32_t* __restrict__ steps)
{
    double2* Rk = R + (size_t)k * (m + 1) * lda;
    for (int j = 0; j < k; ++j) {
        const double cj = cs[(size_t)j * lda + c];
        const double2 sj = sn[(size_t)j * lda + c];
        const double2 a = Rk[(size_t)j * lda + c], b = Rk[(size_t)(j + 1) * lda + c];
        // [a; b] <- [c a + s b; -conj(s) a + c b]
        const double2 sb = cmul(sj, b);
        const double2 sa = cconjmul(sj, a);
        Rk[(size_t)j * lda + c] = make_double2(cj * a.x + sb.x, cj * a.y + sb.y);
        Rk[(size_t)(j + 1) * lda + c] = make_double2(cj * b.x - sa.x, cj * b.y - sa.y);
    }
    const double2 a = Rk[(size_t)k * lda + c];
    const double aa = hypot(a.x, a.y);
    const double rr = hypot(aa, bb);
    double ck;
    double2 sk;
    if (rr == 0.0) {
        ck = 1.0;
        sk = make_double2(0.0, 0.0);
    } else if (aa == 0.0) {
        ck = 0.0;
        sk = make_double2(1.0, 0.0);
    } else {
        ck = aa / rr;
        sk = make_double2(a.x / aa * bb / rr, a.y / aa * bb / rr);   // (a/|a|) conj(b)/r, b real
    }
    cs[(size_t)k * lda + c] = ck;
    sn[(size_t)k * lda + c] = sk;
    Rk[(size_t)k * lda + c] = make_double2(ck * a.x + sk.x * bb, ck * a.y + sk.y * bb);
    const double2 gk = g[(size_t)k * lda + c];
    const double2 gk1 = cconjmul(sk, gk);
    g[(size_t)(k + 1) * lda + c] = make_double2(-gk1.x, -gk1.y);
    g[(size_t)k * lda + c] = make_double2(ck * gk.x, ck * gk.y);
    steps[c] = k + 1;
    const double est = hypot(gk1.x, gk1.y);
    if (est <= target[c] || k + 1 >= m || bb == 0.0) done[c] = 1;
}

__global__ void k_givens(int k, int m, const double2* __restrict__ h1, const double2* __restrict__ h2,
                         const double* __restrict__ nrm, double2* __restrict__ R, double* __restrict__ cs,
                         double2* __restrict__ sn, double2* __restrict__ g, const double* __restrict__ target,
                         int32_t* __restrict__ done, int32_t* __restrict__ steps, int na, int lda)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= na || done[c]) return;
    double2* Rk = R + (size_t)k * (m + 1) * lda;
    for (int j = 0; j <= k; ++j) {
        const double2 a = h1[(size_t)j * lda + c], b = h2[(size_t)j * lda + c];
        Rk[(size_t)j * lda + c] = make_double2(a.x + b.x, a.y + b.y);
    }
    rotate_column(k, m, c, lda, nrm[c], R, cs, sn, g, target, done, steps);
}

// y = R^{-1} g over the first steps[c] rows (back substitution per column).
__global__ void k_lsq(int m, const double2* __restrict__ R, const double2* __restrict__ g,
                      const int32_t* __restrict__ steps, double2* __restrict__ y, int na, int lda)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= na) return;
    const int kc = steps[c];
    for (int j = kc - 1; j >= 0; --j) {
        double2 s = g[(size_t)j * lda + c];
        for (int l = j + 1; l < kc; ++l) {
            const double2 rjl = R[((size_t)l * (m + 1) + j) * lda + c];
            const double2 t = cmul(rjl, y[(size_t)l * lda + c]);
            s.x -= t.x;
            s.y -= t.y;
        }
        const double2 d = R[((size_t)j * (m + 1) + j) * lda + c];
        const double den = d.x * d.x + d.y * d.y;
        y[(size_t)j * lda + c] = make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den);
    }
}

// x += sum_{j < steps[c]} V_j y_j
__global__ __launch_bounds__(256) void k_x_update(const double2* __restrict__ V, int64_t vstride,
                                                  const double2* __restrict__ y, const int32_t* __restrict__ steps,
                                                  double2* __restrict__ x, int na, int lda, int64_t nup)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= na) return;
    const size_t o = (size_t)r * lda + c;
    double2 acc = x[o];
    const int kc = steps[c];
    for (int j = 0; j < kc; ++j) {
        const double2 t = cmul(V[j * vstride + o], y[(size_t)j * lda + c]);
        acc.x += t.x;
        acc.y += t.y;
    }
    x[o] = acc;
}

__global__ __launch_bounds__(256) void k_gather(const double2* __restrict__ src, int lds, double2* __restrict__ dst,
                                                int ldd, const int32_t* __restrict__ map, int na, int64_t nup)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= ldd) return;
    dst[(size_t)r * ldd + c] = (c < na) ? src[(size_t)r * lds + map[c]] : make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_scatter(const double2* __restrict__ src, int lds, double2* __restrict__ dst,
                                                 int ldd, const int32_t* __restrict__ map, int na, int64_t nup)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nup || c >= na) return;
    dst[(size_t)r * ldd + map[c]] = src[(size_t)r * lds + c];
}

// ---------------------------------------------------------------- observables

// dpart[chunk][k][c] over atom chunks: sum_i x_q[i][c] r_ik (+ sum_i x_mu_k[i][c])
__global__ __launch_bounds__(64) void k_dipole_partial(const double2* __restrict__ x, const double4* __restrict__ x64,
                                                       int64_t n, int64_t np, int model, int ncol, int ldx,
                                                       double2* __restrict__ dpart)
{
    const int c = blockIdx.y * 64 + threadIdx.x;
    if (c >= ncol) return;
    const int64_t i0 = (int64_t)blockIdx.x * RED_ROWS;
    const int64_t i1 = min(n, i0 + RED_ROWS);
    double d[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t i = i0; i < i1; ++i) {
        const double2 q = x[(size_t)i * ldx + c];
        const double4 p = x64[i];
        d[0][0] = fma(q.x, p.x, d[0][0]); d[0][1] = fma(q.y, p.x, d[0][1]);
        d[1][0] = fma(q.x, p.y, d[1][0]); d[1][1] = fma(q.y, p.y, d[1][1]);
        d[2][0] = fma(q.x, p.z, d[2][0]); d[2][1] = fma(q.y, p.z, d[2][1]);
        if (model == 1) {
            for (int k = 0; k < 3; ++k) {
                const double2 mu = x[(size_t)((k + 1) * np + i) * ldx + c];
                d[k][0] += mu.x;
                d[k][1] += mu.y;
            }
        }
    }
    for (int k = 0; k < 3; ++k) dpart[((size_t)blockIdx.x * 3 + k) * ldx + c] = make_double2(d[k][0], d[k][1]);
}

__global__ void k_dipole_reduce(const double2* __restrict__ dpart, int nchunk, int ncol, int ldx,
                                double2* __restrict__ d)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * ncol) return;
    const int k = t / ncol, c = t - k * ncol;
    double ar = 0.0, ai = 0.0;
    for (int q = 0; q < nchunk; ++q) {
        const double2 p = dpart[((size_t)q * 3 + k) * ldx + c];
        ar += p.x;
        ai += p.y;
    }
    d[(size_t)k * ncol + c] = make_double2(ar, ai);
}

// alpha[w][k][l] = d_k / E0 of the column (w, l); sigma = (4 pi w / c) mean_l Im alpha_ll
__global__ void k_spectrum(const double2* __restrict__ d, const int32_t* __restrict__ col_pol, int n_omega, int npol,
                           int ncol, const double* __restrict__ omega_au, double e0, double2* __restrict__ alpha,
                           double* __restrict__ sigma)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_omega) return;
    double2* a = alpha + (size_t)w * 9;
    for (int q = 0; q < 9; ++q) a[q] = make_double2(0.0, 0.0);
    double im = 0.0;
    for (int p = 0; p < npol; ++p) {
        const int c = w * npol + p;
        const int l = col_pol[c];
        for (int k = 0; k < 3; ++k) {
            const double2 dk = d[(size_t)k * ncol + c];
            a[3 * k + l] = make_double2(dk.x / e0, dk.y / e0);
        }
        im += a[3 * l + l].y;
    }
    sigma[w] = 2.0 * TWO_PI * omega_au[w] / C_LIGHT * (im / npol);
}

__global__ void k_unpermute(const double2* __restrict__ x, int ldx, int col, const int32_t* __restrict__ perm,
                            int64_t n, int64_t np, int ncomp, double2* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * ncomp) return;
    const int64_t comp = t / n, i = t - comp * n;
    out[comp * n + perm[i]] = x[(size_t)(comp * np + i) * ldx + col];
}

__global__ void k_permute_in(const double2* __restrict__ in, int ncol, int64_t n, int64_t np, int ncomp,
                             const int32_t* __restrict__ perm, double2* __restrict__ x, int ldx)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= np * ncomp || c >= ldx) return;
    const int64_t comp = r / np, i = r - comp * np;
    double2 v = make_double2(0.0, 0.0);
    if (c < ncol && i < n) v = in[(size_t)c * n * ncomp + comp * n + perm[i]];
    x[(size_t)r * ldx + c] = v;
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t words)
{
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; t < words; t += stride) p[t] = 0u;
}

// ============ CGS2 with delayed reorthogonalisation (two passes) =============
// Step k holds v_0..v_{k-1} orthonormal and u = V_k, a vector that had one
// projection pass.  With w~ = A u (the matvec of this step):
//   one dot pass   G[j][0] = <v_j, u>, G[j][1] = <v_j, w~>  (j <= k, v_k := u)
//   coefficients   s = G[<k][0], rho^2 = <u,u> - |s|^2, v_k = (u - V s) / rho;
//                  the previous Hessenberg column gets its lagged correction
//                  H[<k][k-1] += b s, H[k][k-1] = b rho (b = its tentative norm)
//                  and its Givens rotation; c = V_k^H w~, h = (c - H s) / rho
//   one update     v_k = u/rho - V (s/rho),  w' = w~/rho - (c_k/rho^2) u - V d
//                  with d = (c_<k - (c_k/rho) s) / rho, and |w'|^2 partials.
// w' is normalised into V_{k+1} for the next step; its own second pass is the
// next step's lagged correction.

// partial[chunk][j][t][c], t = 0: <V_j, V_{nvec-1}>, t = 1: <V_j, w>.
// One wave per (DOT_JB basis vectors, row chunk, 64 columns).  Loads are
// unconditional (the last group repeats its final vector), so a row's
// DOT_JB + 2 loads issue back to back.  The hardware hands block L to XCD
// L mod 8; the blocks are renumbered so that the j-groups of one row chunk,
// which all read the same rows of u and w, run on one XCD and share its L2.
constexpr int DOT_JB = 8;
__global__ __launch_bounds__(64) void k_dots2(const double2* __restrict__ V, int64_t vstride, int nvec,
                                              const double2* __restrict__ w, double2* __restrict__ partial, int na,
                                              int lda, int64_t nup, int rows_per, int njg, int nch,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int nb = gridDim.x, L = blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, x = L & 7;
    const int lam = (x < r8 ? x * (q8 + 1) : r8 * (q8 + 1) + (x - r8) * q8) + (L >> 3);
    const int jg = lam % njg;
    const int rest = lam / njg;
    const int chunk = rest % nch;
    const int c = (rest / nch) * 64 + (int)threadIdx.x;
    if (c >= na) return;
    const int j0 = jg * DOT_JB;
    const int64_t r0 = (int64_t)chunk * rows_per;
    const int64_t r1 = min(nup, r0 + rows_per);
    const double2* vq[DOT_JB];
#pragma unroll
    for (int q = 0; q < DOT_JB; ++q) vq[q] = V + (size_t)min(j0 + q, nvec - 1) * vstride + c;
    const double2* u = V + (size_t)(nvec - 1) * vstride + c;
    const double2* wc = w + c;
    double a0r[DOT_JB], a0i[DOT_JB], a1r[DOT_JB], a1i[DOT_JB];
#pragma unroll
    for (int q = 0; q < DOT_JB; ++q) a0r[q] = a0i[q] = a1r[q] = a1i[q] = 0.0;
#pragma unroll 2
    for (int64_t r = r0; r < r1; ++r) {
        const size_t o = (size_t)r * lda;
        const double2 x0 = u[o];
        const double2 x1 = wc[o];
        double2 v[DOT_JB];
#pragma unroll
        for (int q = 0; q < DOT_JB; ++q) v[q] = vq[q][o];
#pragma unroll
        for (int q = 0; q < DOT_JB; ++q) {
            a0r[q] = fma(v[q].x, x0.x, fma(v[q].y, x0.y, a0r[q]));
            a0i[q] = fma(v[q].x, x0.y, fma(-v[q].y, x0.x, a0i[q]));
            a1r[q] = fma(v[q].x, x1.x, fma(v[q].y, x1.y, a1r[q]));
            a1i[q] = fma(v[q].x, x1.y, fma(-v[q].y, x1.x, a1i[q]));
        }
    }
    const int nj = min(DOT_JB, nvec - j0);
#pragma unroll
    for (int q = 0; q < DOT_JB; ++q)
        if (q < nj) {
            double2* o = partial + (((size_t)chunk * nvec + j0 + q) * 2) * lda + c;
            o[0] = make_double2(a0r[q], a0i[q]);
            o[lda] = make_double2(a1r[q], a1i[q]);
        }
}

// G[j][t][f] = sum of the partials over the row chunks of f's segment.
// Without segments (seg_beg null) f = c < na and all nch chunks count; with
// segments f = seg * ld + c over nseg segments of ld columns, seg_beg holding
// each segment's first 256-row chunk.
__global__ void k_reduce_dots2(const double2* __restrict__ partial, int nch, int rows_per, int nvec,
                               double2* __restrict__ G, int na, int ld, const int32_t* __restrict__ seg_beg, int nseg,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int ldf = nseg * ld;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nvec * 2 * ldf) return;
    const int jt = t / ldf, f = t - jt * ldf;
    const int sg = f / ld, c = f - sg * ld;
    if (!seg_beg && c >= na) return;
    const int per = 256 / rows_per;
    const int k0 = seg_beg ? seg_beg[sg] * per : 0;
    const int k1 = seg_beg ? seg_beg[sg + 1] * per : nch;
    double ar = 0.0, ai = 0.0;
    for (int k = k0; k < k1; ++k) {
        const double2 p = partial[((size_t)k * nvec * 2 + jt) * ld + c];
        ar += p.x;
        ai += p.y;
    }
    G[(size_t)jt * ldf + f] = make_double2(ar, ai);
}

// Step k, per column (one thread each): rho of the corrected v_k, the lagged
// correction of Hessenberg column k-1 (H[<k][k-1] += b s, H[k][k-1] = b rho)
// with its Givens rotation, and c_k = <v_k, w~>.  aux[c] = (rho, c_k).
// final_only: the cycle's last correction, nothing after the rotation.
__global__ void k_dcgs2_fix(int k, int m, int final_only, const double2* __restrict__ G,
                            const double* __restrict__ nrm, double2* __restrict__ H, double2* __restrict__ R,
                            double* __restrict__ cs, double2* __restrict__ sn, double2* __restrict__ g,
                            const double* __restrict__ target, int32_t* __restrict__ done,
                            int32_t* __restrict__ steps, double2* __restrict__ aux, int na, int lda,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= na || done[c]) return;
    const size_t ld2 = 2 * (size_t)lda;
    const double2* Gs = G + c;              // s_j = Gs[j * ld2]
    const double2* Gt = G + lda + c;        // t_j = <v_j, w~> = Gt[j * ld2]
    double ss = 0.0;
#pragma unroll 4
    for (int j = 0; j < k; ++j) {
        const double2 sj = Gs[(size_t)j * ld2];
        ss = fma(sj.x, sj.x, fma(sj.y, sj.y, ss));
    }
    const double rho = sqrt(fmax(Gs[(size_t)k * ld2].x - ss, 1e-300));
    if (k >= 1) {
        const int col = k - 1;
        const double b = nrm[c];
        double2* Hc = H + (size_t)col * (m + 1) * lda + c;
        double2* Rc = R + (size_t)col * (m + 1) * lda + c;
        // corrected entries h_j = H[j][col] + b s_j, rotated on the fly by the
        // col stored rotations; a carries the partially rotated entry j
        double2 a;
        {
            const double2 h = Hc[0], sj = Gs[0];
            a = make_double2(fma(b, sj.x, h.x), fma(b, sj.y, h.y));
            Hc[0] = a;
        }
#pragma unroll 4
        for (int j = 0; j < col; ++j) {
            const double2 h = Hc[(size_t)(j + 1) * lda], sv = Gs[(size_t)(j + 1) * ld2];
            const double cj = cs[(size_t)j * lda + c];
            const double2 sj = sn[(size_t)j * lda + c];
            const double2 hb = make_double2(fma(b, sv.x, h.x), fma(b, sv.y, h.y));
            Hc[(size_t)(j + 1) * lda] = hb;
            // [a; hb] <- [c a + s hb; -conj(s) a + c hb]
            const double2 sb = cmul(sj, hb);
            const double2 sa = cconjmul(sj, a);
            Rc[(size_t)j * lda] = make_double2(cj * a.x + sb.x, cj * a.y + sb.y);
            a = make_double2(cj * hb.x - sa.x, cj * hb.y - sa.y);
        }
        const double bb = b * rho;
        Hc[(size_t)k * lda] = make_double2(bb, 0.0);
        const double aa = hypot(a.x, a.y);
        const double rr = hypot(aa, bb);
        double ck;
        double2 sk;
        if (rr == 0.0) {
            ck = 1.0;
            sk = make_double2(0.0, 0.0);
        } else if (aa == 0.0) {
            ck = 0.0;
            sk = make_double2(1.0, 0.0);
        } else {
            ck = aa / rr;
            sk = make_double2(a.x / aa * bb / rr, a.y / aa * bb / rr);
        }
        cs[(size_t)col * lda + c] = ck;
        sn[(size_t)col * lda + c] = sk;
        Rc[(size_t)col * lda] = make_double2(ck * a.x + sk.x * bb, ck * a.y + sk.y * bb);
        const double2 gk = g[(size_t)col * lda + c];
        const double2 gk1 = cconjmul(sk, gk);
        g[(size_t)(col + 1) * lda + c] = make_double2(-gk1.x, -gk1.y);
        g[(size_t)col * lda + c] = make_double2(ck * gk.x, ck * gk.y);
        steps[c] = col + 1;
        if (hypot(gk1.x, gk1.y) <= target[c] || col + 1 >= m || bb == 0.0) {
            done[c] = 1;
            return;
        }
    }
    if (final_only) return;
    double2 cv = Gt[(size_t)k * ld2];
#pragma unroll 4
    for (int j = 0; j < k; ++j) {
        const double2 st = cconjmul(Gs[(size_t)j * ld2], Gt[(size_t)j * ld2]);
        cv.x -= st.x;
        cv.y -= st.y;
    }
    aux[c] = make_double2(rho, 0.0);
    aux[lda + c] = make_double2(cv.x / rho, cv.y / rho);
}

// stop = 1 when every one of the n columns is done (one workgroup).
__global__ __launch_bounds__(256) void k_all_done(const int32_t* __restrict__ done, int n, int32_t* __restrict__ stop)
{
    int open = 0;
    for (int c = threadIdx.x; c < n; c += 256) open |= (done[c] == 0);
    open = __syncthreads_or(open);
    if (threadIdx.x == 0) stop[0] = open ? 0 : 1;
}

// Step k, one wave per (row i <= k, 64 columns): the tentative Hessenberg
// column h_i = (c_i - (H s)_i) / rho, and the update coefficients
// coefQ[i] = (s_i / rho, d_i) for i < k, coefV = (1/rho, c_k/rho^2) for i = k.
// Columns that are done get zero coefficients.
__global__ __launch_bounds__(256) void k_dcgs2_coef(int k, int m, const double2* __restrict__ G,
                                                    const double2* __restrict__ aux, double2* __restrict__ H,
                                                    const int32_t* __restrict__ done, double2* __restrict__ coefQ,
                                                    double2* __restrict__ coefV, int na, int lda,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i > k || c >= na) return;
    const size_t ld2 = 2 * (size_t)lda;
    double2* cq = (i < k) ? coefQ + (size_t)i * ld2 + c : coefV + c;
    if (done[c]) {
        cq[0] = make_double2(0.0, 0.0);
        cq[lda] = make_double2(0.0, 0.0);
        return;
    }
    const double rho = aux[c].x;
    const double2 ckr = aux[lda + c];        // c_k = <v_k, w~>
    const double2 e = make_double2(ckr.x / rho, ckr.y / rho);
    // (H s)_i over the columns j >= i - 1 (H is upper Hessenberg)
    double hr = 0.0, hi = 0.0;
    const double2* Hi = H + (size_t)i * lda + c;
    const double2* Gs = G + c;
#pragma unroll 4
    for (int j = (i > 0 ? i - 1 : 0); j < k; ++j) {
        const double2 h = Hi[(size_t)j * (m + 1) * lda], sj = Gs[(size_t)j * ld2];
        hr = fma(h.x, sj.x, fma(-h.y, sj.y, hr));
        hi = fma(h.x, sj.y, fma(h.y, sj.x, hi));
    }
    const double2 ci = (i < k) ? G[(size_t)i * ld2 + lda + c] : ckr;
    H[((size_t)k * (m + 1) + i) * lda + c] = make_double2((ci.x - hr) / rho, (ci.y - hi) / rho);
    if (i < k) {
        const double2 si = Gs[(size_t)i * ld2];
        const double2 es = cmul(e, si);
        cq[0] = make_double2(si.x / rho, si.y / rho);
        cq[lda] = make_double2((ci.x - es.x) / rho, (ci.y - es.y) / rho);
    } else {
        cq[0] = make_double2(1.0 / rho, 0.0);
        cq[lda] = make_double2(e.x / rho, e.y / rho);
    }
}

// V_k <- V_k/rho - sum_j V_j (s_j/rho);  w <- w/rho - (c_k/rho^2) V_k(old) - sum_j V_j d_j
// With segments (chunk_seg non-null) the coefficients of row r's column c sit
// at flat index chunk_seg[r / 256] * lda + c of leading dimension ldc.
__global__ __launch_bounds__(256) void k_dcgs2_update(double2* __restrict__ V, int64_t vstride, int k,
                                                      const double2* __restrict__ coefQ,
                                                      const double2* __restrict__ coefV, double2* __restrict__ w,
                                                      double* __restrict__ norm_partial, int na, int lda, int64_t nup,
                                                      const int32_t* __restrict__ chunk_seg, int ldc,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.y * 64 + lane;
    const int64_t rg = (int64_t)blockIdx.x * UPD_ROWS + wave * ARN_RG;
    const size_t ld2 = 2 * (size_t)ldc;
    double nrm = 0.0;
    if (c < na && rg < nup) {
        const int f = chunk_seg ? chunk_seg[rg >> 8] * lda + c : c;
        const double2 p = coefV[f], qv = coefV[ldc + f];
        double2* u = V + (size_t)k * vstride + (size_t)rg * lda + c;
        double2 av[ARN_RG], aw[ARN_RG];
#pragma unroll
        for (int q = 0; q < ARN_RG; ++q) {
            const double2 uu = u[(size_t)q * lda];
            const double2 ww = w[(size_t)(rg + q) * lda + c];
            const double2 t = cmul(qv, uu);
            av[q] = make_double2(p.x * uu.x, p.x * uu.y);
            aw[q] = make_double2(p.x * ww.x - t.x, p.x * ww.y - t.y);
        }
        const double2* vb = V + (size_t)rg * lda + c;
#pragma unroll 2
        for (int j = 0; j < k; ++j) {
            const double2 a = coefQ[(size_t)j * ld2 + f];
            const double2 d = coefQ[(size_t)j * ld2 + ldc + f];
            const double2* vj = vb + (size_t)j * vstride;
#pragma unroll
            for (int q = 0; q < ARN_RG; ++q) {
                const double2 v = vj[(size_t)q * lda];
                const double2 ta = cmul(v, a), td = cmul(v, d);
                av[q].x -= ta.x; av[q].y -= ta.y;
                aw[q].x -= td.x; aw[q].y -= td.y;
            }
        }
#pragma unroll
        for (int q = 0; q < ARN_RG; ++q) {
            u[(size_t)q * lda] = av[q];
            w[(size_t)(rg + q) * lda + c] = aw[q];
            nrm = fma(aw[q].x, aw[q].x, fma(aw[q].y, aw[q].y, nrm));
        }
    }
    red[wave][lane] = nrm;
    __syncthreads();
    if (wave == 0 && c < na)
        norm_partial[(size_t)blockIdx.x * lda + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// ============================ stacked segments ==============================
// A stacked block holds several segments (structure x block of Bc columns),
// each a contiguous, 256-row-aligned range of rows; chunk_seg maps every
// 256-row chunk to its segment.  Per-column state is indexed by the flat
// column seg * Bc + c (leading dimension nseg * Bc).

__global__ __launch_bounds__(256) void k_spmm_seg(const SegInfo* __restrict__ segs,
                                                  const int32_t* __restrict__ chunk_seg, const void* __restrict__ Yv,
                                                  int y_f32, int ldy, const double2* __restrict__ X,
                                                  const double2* __restrict__ zq, const double2* __restrict__ zmu,
                                                  const double2* __restrict__ B, double2* __restrict__ W, int64_t rows,
                                                  int Bc, int ldf, double mu_sign,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows || c >= Bc) return;
    const size_t o = (size_t)r * Bc + c;
    const int sg = chunk_seg[r >> 8];
    const SegInfo& S = segs[sg];
    const int64_t lr = r - S.row_off;
    const int64_t comp = lr / S.np, i = lr - comp * S.np;
    if (i >= S.n) {
        W[o] = make_double2(0.0, 0.0);
        return;
    }
    const int f = sg * Bc + c;
    double ar = 0.0, ai = 0.0;
    double2 z;
    if (comp == 0) {
        for (int32_t e = S.rp[i]; e < S.rp[i + 1]; ++e) {
            const double k = S.cv[e];
            const size_t yo = (size_t)(S.row_off + S.ci[e]) * ldy + 2 * c;
            const double yr = y_f32 ? (double)static_cast<const float*>(Yv)[yo] : static_cast<const double*>(Yv)[yo];
            const double yi = y_f32 ? (double)static_cast<const float*>(Yv)[yo + 1]
                                    : static_cast<const double*>(Yv)[yo + 1];
            ar = fma(k, yr, ar);
            ai = fma(k, yi, ai);
        }
        z = zq[f];
    } else {
        const size_t yo = (size_t)r * ldy + 2 * c;
        ar = y_f32 ? (double)static_cast<const float*>(Yv)[yo] : static_cast<const double*>(Yv)[yo];
        ai = y_f32 ? (double)static_cast<const float*>(Yv)[yo + 1] : static_cast<const double*>(Yv)[yo + 1];
        z = zmu[f];
    }
    const double2 x = X[o];
    double2 w = make_double2(ar - (z.x * x.x - z.y * x.y), ai - (z.x * x.y + z.y * x.x));
    if (comp != 0) w = make_double2(mu_sign * w.x, mu_sign * w.y);
    if (B != nullptr) {
        const double2 b = B[o];
        w = make_double2(b.x - w.x, b.y - w.y);
    }
    W[o] = w;
    (void)ldf;
}

// h[j][seg*Bc + c] = sum of partial[k][j][c] over the segment's chunks k
__global__ void k_reduce_dots_seg(const double2* __restrict__ partial, const int32_t* __restrict__ seg_beg,
                                  int nvec, double2* __restrict__ h, int nseg, int Bc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ldf = nseg * Bc;
    if (t >= nvec * ldf) return;
    const int j = t / ldf, f = t - j * ldf;
    const int sg = f / Bc, c = f - sg * Bc;
    double ar = 0.0, ai = 0.0;
    for (int k = seg_beg[sg]; k < seg_beg[sg + 1]; ++k) {
        const double2 p = partial[((size_t)k * nvec + j) * Bc + c];
        ar += p.x;
        ai += p.y;
    }
    h[(size_t)j * ldf + f] = make_double2(ar, ai);
}

// nrm[seg*Bc + c] = sqrt(sum of partial[k][c] over the segment's chunks k)
__global__ void k_reduce_norms_seg(const double* __restrict__ partial, const int32_t* __restrict__ seg_beg,
                                   double* __restrict__ nrm, int nseg, int Bc,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nseg * Bc) return;
    const int sg = f / Bc, c = f - sg * Bc;
    double s = 0.0;
    for (int k = seg_beg[sg]; k < seg_beg[sg + 1]; ++k) s += partial[(size_t)k * Bc + c];
    nrm[f] = sqrt(s);
}

// w -= sum_j V_j h_j with h per flat column; norm partials per UPD_ROWS rows.
__global__ __launch_bounds__(256) void k_col_update_seg(const double2* __restrict__ V, int64_t vstride, int nvec,
                                                        const double2* __restrict__ h, double2* __restrict__ w,
                                                        double* __restrict__ norm_partial,
                                                        const int32_t* __restrict__ chunk_seg, int Bc, int ldf,
                                                        int64_t rows)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.y * 64 + lane;
    const int64_t rg = (int64_t)blockIdx.x * UPD_ROWS + wave * ARN_RG;
    double nrm = 0.0;
    if (c < Bc && rg < rows) {
        const int f = chunk_seg[rg >> 8] * Bc + c;
        double2 acc[ARN_RG];
#pragma unroll
        for (int q = 0; q < ARN_RG; ++q) acc[q] = w[(size_t)(rg + q) * Bc + c];
        const double2* vb = V + (size_t)rg * Bc + c;
        for (int j = 0; j < nvec; ++j) {
            const double2 hj = h[(size_t)j * ldf + f];
            const double2* vj = vb + (size_t)j * vstride;
#pragma unroll
            for (int q = 0; q < ARN_RG; ++q) {
                const double2 a = vj[(size_t)q * Bc];
                acc[q].x -= a.x * hj.x - a.y * hj.y;
                acc[q].y -= a.x * hj.y + a.y * hj.x;
            }
        }
#pragma unroll
        for (int q = 0; q < ARN_RG; ++q) {
            w[(size_t)(rg + q) * Bc + c] = acc[q];
            nrm = fma(acc[q].x, acc[q].x, fma(acc[q].y, acc[q].y, nrm));
        }
    }
    if (norm_partial) {
        red[wave][lane] = nrm;
        __syncthreads();
        if (wave == 0 && c < Bc)
            norm_partial[(size_t)blockIdx.x * Bc + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    }
}

__global__ __launch_bounds__(256) void k_normalize_seg(const double2* __restrict__ w, const double* __restrict__ nrm,
                                                       const int32_t* __restrict__ done,
                                                       const int32_t* __restrict__ chunk_seg, double2* __restrict__ v,
                                                       float* __restrict__ x32, int Bc, int64_t rows,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows || c >= Bc) return;
    const size_t o = (size_t)r * Bc + c;
    const int f = chunk_seg[r >> 8] * Bc + c;
    double2 out = make_double2(0.0, 0.0);
    if (!done[f]) {
        const double s = 1.0 / nrm[f];
        const double2 a = w[o];
        out = make_double2(a.x * s, a.y * s);
    }
    v[o] = out;
    if (x32) *reinterpret_cast<float2*>(x32 + (size_t)r * 2 * Bc + 2 * c) = make_float2((float)out.x, (float)out.y);
}

__global__ __launch_bounds__(256) void k_x_update_seg(const double2* __restrict__ V, int64_t vstride,
                                                      const double2* __restrict__ y, const int32_t* __restrict__ steps,
                                                      const int32_t* __restrict__ chunk_seg, double2* __restrict__ x,
                                                      int Bc, int ldf, int64_t rows)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows || c >= Bc) return;
    const size_t o = (size_t)r * Bc + c;
    const int f = chunk_seg[r >> 8] * Bc + c;
    double2 acc = x[o];
    const int kc = steps[f];
    for (int j = 0; j < kc; ++j) {
        const double2 t = cmul(V[j * vstride + o], y[(size_t)j * ldf + f]);
        acc.x += t.x;
        acc.y += t.y;
    }
    x[o] = acc;
}

inline dim3 grid_rows_cols(int64_t rows, int cols) { return dim3((unsigned)((rows + 3) / 4), (unsigned)((cols + 63) / 64)); }
inline int nchunks(int64_t rows) { return (int)((rows + RED_ROWS - 1) / RED_ROWS); }
inline int arn_chunks(int64_t rows) { return (int)((rows + ARN_ROWS - 1) / ARN_ROWS); }

}  // namespace

// ============================================================== launchers

// Candidate subsets per row block of the neighbour builders: about 1024
// one-wave workgroups in all, at most 8 subsets.
void count_sum(const int32_t* cntw, int nsub, int64_t np, int64_t n, int32_t add, int32_t* cnt, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_count_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cntw, nsub, np, n, add,
                           cnt);
}

int neighbor_subsets(int64_t np)
{
    const int64_t rb = std::max<int64_t>(1, np / 64);
    return (int)std::max<int64_t>(1, std::min<int64_t>(8, (1024 + rb - 1) / rb));
}

hipError_t build_geometry(Geometry& g, const double* xyz_bohr_host, double cutoff_bohr, const pxMaterial& m,
                          double r0_bohr, std::vector<int32_t>& perm_host, int* bad_pair, hipStream_t st,
                          const uint8_t* types_host, const pxMaterial* mb)
{
    const int64_t n = g.n, np = g.np;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], xyz_bohr_host[3 * i + k]);
            hi[k] = std::max(hi[k], xyz_bohr_host[3 * i + k]);
        }
    double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    double sc = ext > 0 ? 1023.0 / ext : 1.0;
    g.cx = n > 0 ? 0.5 * (lo[0] + hi[0]) : 0.0;
    g.cy = n > 0 ? 0.5 * (lo[1] + hi[1]) : 0.0;
    g.cz = n > 0 ? 0.5 * (lo[2] + hi[2]) : 0.0;
    int64_t npow = 1;
    while (npow < n) npow <<= 1;
    double* d_xyz = nullptr;
    uint64_t* d_keys = nullptr;
    int32_t *d_cnt = nullptr, *d_perm = nullptr, *d_cntw = nullptr;
    int* d_bad = nullptr;
    uint8_t* d_types = nullptr;
    hipError_t e;
#define PXCHK(x) do { e = (x); if (e != hipSuccess) goto fail; } while (0)
    PXCHK(px::dev_malloc((void**)&d_xyz, sizeof(double) * 3 * n));
    PXCHK(px::dev_malloc((void**)&d_keys, sizeof(uint64_t) * npow));
    PXCHK(px::dev_malloc((void**)&d_cnt, sizeof(int32_t) * (n + 1)));
    PXCHK(px::dev_malloc((void**)&d_perm, sizeof(int32_t) * np));
    PXCHK(px::dev_malloc((void**)&d_bad, sizeof(int)));
    PXCHK(px::dev_malloc((void**)&g.xyz64, sizeof(double4) * np));
    PXCHK(px::dev_malloc((void**)&g.xyz32, sizeof(float4) * np));
    PXCHK(px::dev_malloc((void**)&g.glo, sizeof(float4) * (np / GROUP)));
    PXCHK(px::dev_malloc((void**)&g.ghi, sizeof(float4) * (np / GROUP)));
    PXCHK(px::dev_malloc((void**)&g.row_ptr, sizeof(int32_t) * (n + 1)));
    PXCHK(hipMemcpyAsync(d_xyz, xyz_bohr_host, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(d_bad), (size_t)1);
    hipLaunchKernelGGL(k_morton, dim3((unsigned)((npow + 255) / 256)), dim3(256), 0, st, d_xyz, n, npow,
                       make_double3(lo[0], lo[1], lo[2]), make_double3(sc, sc, sc), d_keys);
    for (uint32_t k = 2; k <= (uint32_t)npow; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic, dim3((unsigned)((npow + 255) / 256)), dim3(256), 0, st, d_keys, j, k,
                               (uint32_t)npow);
    {
        double3 far0 = make_double3(hi[0] + 1.0e4, hi[1] + 1.0e4, hi[2] + 1.0e4);
        hipLaunchKernelGGL(k_gather_sorted, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, d_xyz, d_keys, n,
                           np, far0, d_perm, g.xyz64, g.xyz32);
    }
    hipLaunchKernelGGL(k_group_bbox, dim3((unsigned)((np / GROUP + 255) / 256)), dim3(256), 0, st, g.xyz64,
                       np / GROUP, g.glo, g.ghi);
    {
        KappaSet ks;
        KappaConst& kc = ks.k[0];
        kc.a_eff = m.a_eff;
        kc.fd = m.fermi_d;
        kc.s_r0 = m.fermi_s * r0_bohr;
        kc.rc = cutoff_bohr;
        kc.rc2 = cutoff_bohr * cutoff_bohr;
        kc.min_r = 1e-6 / ANG;
        ks.k[1] = ks.k[2] = kc;
        ks.rc_max = kc.rc;
        if (types_host && mb) {
            // type B, and unlike pairs with the mean of the two types' A, r0, d, s and cutoff
            const double r0b = mb->r0_ang / ANG, rcb = mb->cutoff_ang / ANG;
            KappaConst& kb = ks.k[2];
            kb.a_eff = mb->a_eff;
            kb.fd = mb->fermi_d;
            kb.s_r0 = mb->fermi_s * r0b;
            kb.rc = rcb;
            kb.rc2 = rcb * rcb;
            KappaConst& kab = ks.k[1];
            kab.a_eff = 0.5 * (m.a_eff + mb->a_eff);
            kab.fd = 0.5 * (m.fermi_d + mb->fermi_d);
            kab.s_r0 = 0.5 * (m.fermi_s + mb->fermi_s) * 0.5 * (r0_bohr + r0b);
            kab.rc = 0.5 * (cutoff_bohr + rcb);
            kab.rc2 = kab.rc * kab.rc;
            ks.rc_max = std::max(kc.rc, std::max(kb.rc, kab.rc));
            PXCHK(px::dev_malloc((void**)&d_types, n));
            PXCHK(px::dev_malloc((void**)&g.type, np));
            PXCHK(hipMemcpyAsync(d_types, types_host, n, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_gather_types, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, d_types, d_perm, n,
                               np, g.type);
        }
        const int nsub = neighbor_subsets(np);
        PXCHK(px::dev_malloc((void**)&d_cntw, sizeof(int32_t) * (size_t)nsub * np));
        hipLaunchKernelGGL(k_kbar_rows<0>, dim3((unsigned)(np / 64), (unsigned)nsub), dim3(64), 0, st, g.xyz64, g.glo,
                           g.ghi, n, np, ks, g.type, d_cntw, nullptr, nullptr, nullptr, d_bad);
        // row lengths with the diagonal
        hipLaunchKernelGGL(k_count_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const int32_t*)d_cntw,
                           nsub, np, n, 1, d_cnt);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, d_cnt, n, g.row_ptr);
        int32_t nnz = 0;
        PXCHK(hipMemcpyAsync(&nnz, g.row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        PXCHK(hipMemcpyAsync(bad_pair, d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
        PXCHK(hipStreamSynchronize(st));
        g.nnz = nnz;
        PXCHK(px::dev_malloc((void**)&g.col, sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
        PXCHK(px::dev_malloc((void**)&g.val, sizeof(double) * std::max<int64_t>(nnz, 1)));
        hipLaunchKernelGGL(k_kbar_rows<1>, dim3((unsigned)(np / 64), (unsigned)nsub), dim3(64), 0, st, g.xyz64, g.glo,
                           g.ghi, n, np, ks, g.type, d_cntw, g.row_ptr, g.col, g.val, d_bad);
        hipLaunchKernelGGL(k_kbar_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           (const int32_t*)g.row_ptr, n, g.col, g.val);
        if (g.type) {
            PXCHK(px::dev_malloc((void**)&g.hrow, sizeof(double4) * n));
            hipLaunchKernelGGL(k_het_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.row_ptr, g.col, g.val,
                               g.type, n, g.hrow);
        }
    }
    perm_host.resize(n);
    PXCHK(hipMemcpyAsync(perm_host.data(), d_perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    PXCHK(hipStreamSynchronize(st));
    PXCHK(hipGetLastError());
fail:
#undef PXCHK
    px::dev_free(d_xyz);
    px::dev_free(d_keys);
    px::dev_free(d_cnt);
    px::dev_free(d_cntw);
    px::dev_free(d_perm);
    px::dev_free(d_bad);
    px::dev_free(d_types);
    return e;
}

void spmm_shift(const Geometry& g, const void* Y, bool y_is_f32, int ldy, const double2* X, const double2* zq,
                const double2* zmu, const double2* B, double2* W, int na, int lda, double mu_sign, hipStream_t st, const int32_t* stop)
{
    dim3 grid = grid_rows_cols(g.nup, lda);
    if (y_is_f32)
        hipLaunchKernelGGL(k_spmm_shift<float>, grid, dim3(256), 0, st, g.row_ptr, g.col, g.val,
                           static_cast<const float*>(Y), ldy, X, zq, zmu, B, W, g.n, g.np, g.nup, na, lda,
                           mu_sign, stop);
    else
        hipLaunchKernelGGL(k_spmm_shift<double>, grid, dim3(256), 0, st, g.row_ptr, g.col, g.val,
                           static_cast<const double*>(Y), ldy, X, zq, zmu, B, W, g.n, g.np, g.nup, na, lda,
                           mu_sign, stop);
}

void build_rhs(const Geometry& g, const int32_t* col_pol, double e0, double2* b, int ncol, int ldb, double mu_sign,
               hipStream_t st)
{
    hipLaunchKernelGGL(k_rhs, grid_rows_cols(g.nup, ldb), dim3(256), 0, st, g.row_ptr, g.col, g.val, g.xyz64,
                       col_pol, e0, b, g.n, g.np, g.nup, ncol, ldb, mu_sign);
}

void col_dots(const double2* V, int64_t vstride, int nvec, const double2* w, double2* partial, int na, int lda,
              int64_t nup, hipStream_t st)
{
    hipLaunchKernelGGL(k_col_dots, dim3(arn_chunks(nup), (unsigned)((na + 63) / 64), (unsigned)((nvec + ARN_JB - 1) / ARN_JB)),
                       dim3(256), 0, st, V, vstride, nvec, w, partial, na, lda, nup);
}

void reduce_dots(const double2* partial, int nchunk, int nvec, double2* h, int na, int lda, bool, hipStream_t st)
{
    int t = nvec * lda;
    hipLaunchKernelGGL(k_reduce_dots, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, partial, nchunk, nvec, h,
                       na, lda);
}

void col_update(const double2* V, int64_t vstride, int nvec, const double2* h, double2* w, double* norm_partial,
                int na, int lda, int64_t nup, hipStream_t st)
{
    hipLaunchKernelGGL(k_col_update, dim3(update_chunks(nup), (unsigned)((na + 63) / 64)), dim3(256), 0, st, V,
                       vstride, nvec, h, w, norm_partial, na, lda, nup);
}

void col_norm_partial(const double2* w, double* partial, int na, int lda, int64_t nup, hipStream_t st)
{
    hipLaunchKernelGGL(k_col_norm_partial, dim3(arn_chunks(nup), (unsigned)((na + 63) / 64)), dim3(256), 0, st, w,
                       partial, na, lda, nup);
}

void reduce_norms(const double* partial, int nchunk, double* nrm, int na, int lda, hipStream_t st, const int32_t* stop)
{
    hipLaunchKernelGGL(k_reduce_norms, dim3((unsigned)((na + 63) / 64)), dim3(256), 0, st, partial, nchunk, nrm, na,
                       lda, stop);
}

void normalize(const double2* w, const double* nrm, const int32_t* done, double2* v, float* x32, int na, int lda,
               int64_t nup, hipStream_t st, const int32_t* stop)
{
    hipLaunchKernelGGL(k_normalize, grid_rows_cols(nup, lda), dim3(256), 0, st, w, nrm, done, v, x32, na, lda, nup, stop);
}

void to_f32(const double2* v, float* x32, int na, int lda, int64_t nup, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_f32, grid_rows_cols(nup, lda), dim3(256), 0, st, v, x32, na, lda, nup);
}

void givens_step(int k, int m, const double2* h1, const double2* h2, const double* nrm, double2* R, double* cs,
                 double2* sn, double2* gvec, const double* target, int32_t* done, int32_t* steps, int32_t*, int na,
                 int lda, hipStream_t st)
{
    hipLaunchKernelGGL(k_givens, dim3((unsigned)((na + 63) / 64)), dim3(64), 0, st, k, m, h1, h2, nrm, R, cs, sn,
                       gvec, target, done, steps, na, lda);
}

void lsq_solve(int m, const double2* R, const double2* gvec, const int32_t* steps, double2* y, int na, int lda,
               hipStream_t st)
{
    hipLaunchKernelGGL(k_lsq, dim3((unsigned)((na + 63) / 64)), dim3(64), 0, st, m, R, gvec, steps, y, na, lda);
}

void x_update(const double2* V, int64_t vstride, const double2* y, const int32_t* steps, int, double2* x, int na,
              int lda, int64_t nup, hipStream_t st)
{
    hipLaunchKernelGGL(k_x_update, grid_rows_cols(nup, lda), dim3(256), 0, st, V, vstride, y, steps, x, na, lda, nup);
}

void gather_cols(const double2* src, int lds, double2* dst, int ldd, const int32_t* map, int na, int64_t nup,
                 hipStream_t st)
{
    hipLaunchKernelGGL(k_gather, grid_rows_cols(nup, ldd), dim3(256), 0, st, src, lds, dst, ldd, map, na, nup);
}

void scatter_cols(const double2* src, int lds, double2* dst, int ldd, const int32_t* map, int na, int64_t nup,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter, grid_rows_cols(nup, lds), dim3(256), 0, st, src, lds, dst, ldd, map, na, nup);
}

void observables(const Geometry& g, const double2* x, int ncol, int ldx, double2* dpart, double2* d, hipStream_t st)
{
    int nch = nchunks(g.n);
    // a BEM structure's dipole weights in place of the positions: the
    // positions from the tesserae's centroid (DPCM) or their single-layer
    // solve (IEFPCM, whose unknowns are potentials)
    const double4* pos = g.bem ? g.bem_w : g.xyz64;
    hipLaunchKernelGGL(k_dipole_partial, dim3(nch, (unsigned)((ncol + 63) / 64)), dim3(64), 0, st, x, pos, g.n,
                       g.np, g.model, ncol, ldx, dpart);
    hipLaunchKernelGGL(k_dipole_reduce, dim3((unsigned)((3 * ncol + 255) / 256)), dim3(256), 0, st, dpart, nch, ncol,
                       ldx, d);
}

void spectrum(const double2* d, const int32_t* col_pol, int n_omega, int npol, const double* omega_au, double e0,
              double2* alpha, double* sigma, hipStream_t st)
{
    hipLaunchKernelGGL(k_spectrum, dim3((unsigned)((n_omega + 63) / 64)), dim3(64), 0, st, d, col_pol, n_omega, npol,
                       n_omega * npol, omega_au, e0, alpha, sigma);
}

void unpermute(const Geometry& g, const double2* x, int ldx, int col, const int32_t* perm, double2* out,
               hipStream_t st)
{
    int ncomp = g.model ? 4 : 1;
    int64_t t = g.n * ncomp;
    hipLaunchKernelGGL(k_unpermute, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, x, ldx, col, perm, g.n,
                       g.np, ncomp, out);
}

void permute_in(const Geometry& g, const double2* in, int ncol, const int32_t* perm, double2* x, int ldx,
                hipStream_t st)
{
    int ncomp = g.model ? 4 : 1;
    hipLaunchKernelGGL(k_permute_in, grid_rows_cols(g.np * ncomp, ldx), dim3(256), 0, st, in, ncol, g.n, g.np, ncomp,
                       perm, x, ldx);
}

void sort_keys(uint64_t* keys, int64_t npow, hipStream_t st)
{
    for (uint32_t k = 2; k <= (uint32_t)npow; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic, dim3((unsigned)((npow + 255) / 256)), dim3(256), 0, st, keys, j, k,
                               (uint32_t)npow);
}

void scan_counts(const int32_t* cnt, int64_t n, int32_t* row_ptr, hipStream_t st)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, n, row_ptr);
}

void fill_zero(void* p, size_t bytes, hipStream_t st)
{
    size_t words = bytes / 4;
    if (words == 0) return;
    unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, st, reinterpret_cast<uint32_t*>(p), words);
}

// ---- stacked-segment launchers ----------------------------------------------

void spmm_seg(const SegInfo* segs, const int32_t* chunk_seg, const void* Y, bool y_is_f32, int ldy, const double2* X,
              const double2* zq, const double2* zmu, const double2* B, double2* W, int64_t rows, int Bc, int nseg,
              double mu_sign, hipStream_t st, const int32_t* stop)
{
    hipLaunchKernelGGL(k_spmm_seg, grid_rows_cols(rows, Bc), dim3(256), 0, st, segs, chunk_seg, Y, y_is_f32 ? 1 : 0,
                       ldy, X, zq, zmu, B, W, rows, Bc, nseg * Bc, mu_sign, stop);
}

void reduce_dots_seg(const double2* partial, const int32_t* seg_beg, int nvec, double2* h, int nseg, int Bc,
                     hipStream_t st)
{
    const int t = nvec * nseg * Bc;
    hipLaunchKernelGGL(k_reduce_dots_seg, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, partial, seg_beg, nvec,
                       h, nseg, Bc);
}

void reduce_norms_seg(const double* partial, const int32_t* seg_beg, double* nrm, int nseg, int Bc, hipStream_t st, const int32_t* stop)
{
    hipLaunchKernelGGL(k_reduce_norms_seg, dim3((unsigned)((nseg * Bc + 255) / 256)), dim3(256), 0, st, partial,
                       seg_beg, nrm, nseg, Bc, stop);
}

void col_update_seg(const double2* V, int64_t vstride, int nvec, const double2* h, double2* w, double* norm_partial,
                    const int32_t* chunk_seg, int Bc, int nseg, int64_t rows, hipStream_t st)
{
    hipLaunchKernelGGL(k_col_update_seg, dim3(update_chunks(rows), (unsigned)((Bc + 63) / 64)), dim3(256), 0, st, V,
                       vstride, nvec, h, w, norm_partial, chunk_seg, Bc, nseg * Bc, rows);
}

void normalize_seg(const double2* w, const double* nrm, const int32_t* done, const int32_t* chunk_seg, double2* v,
                   float* x32, int Bc, int64_t rows, hipStream_t st, const int32_t* stop)
{
    hipLaunchKernelGGL(k_normalize_seg, grid_rows_cols(rows, Bc), dim3(256), 0, st, w, nrm, done, chunk_seg, v, x32, Bc,
                       rows, stop);
}

void x_update_seg(const double2* V, int64_t vstride, const double2* y, const int32_t* steps, const int32_t* chunk_seg,
                  double2* x, int Bc, int nseg, int64_t rows, hipStream_t st)
{
    hipLaunchKernelGGL(k_x_update_seg, grid_rows_cols(rows, Bc), dim3(256), 0, st, V, vstride, y, steps, chunk_seg, x,
                       Bc, nseg * Bc, rows);
}

// ---- delayed-reorthogonalisation launchers ------------------------------------

int dot_rows(int nvec)
{
    // shorter row chunks for short bases keep enough waves in flight
    return nvec > 48 ? 256 : (nvec > 16 ? 128 : 64);
}

size_t dot_partial_slabs(int64_t nup, int nvec_max)
{
    size_t best = 0;
    for (int v = 1; v <= nvec_max; ++v) best = std::max(best, (size_t)dot_chunks(nup, v) * v);
    return best;
}

void dots2(const double2* V, int64_t vstride, int nvec, const double2* w, double2* partial, int na, int lda,
           int64_t nup, hipStream_t st, const int32_t* stop)
{
    const int rows = dot_rows(nvec), nch = dot_chunks(nup, nvec);
    const int njg = (nvec + DOT_JB - 1) / DOT_JB, ncb = (na + 63) / 64;
    hipLaunchKernelGGL(k_dots2, dim3((unsigned)(njg * nch * ncb)), dim3(64), 0, st, V, vstride, nvec, w, partial,
                       na, lda, nup, rows, njg, nch, stop);
}

void reduce_dots2(const double2* partial, int64_t nup, int nvec, double2* G, int na, int lda, hipStream_t st,
                  const int32_t* seg_beg, int nseg, const int32_t* stop)
{
    const int t = nvec * 2 * lda * nseg;
    hipLaunchKernelGGL(k_reduce_dots2, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, partial,
                       dot_chunks(nup, nvec), dot_rows(nvec), nvec, G, na, lda, seg_beg, nseg, stop);
}

void dcgs2_coef(int k, int m, bool final_only, const double2* G, const double* nrm, double2* H, double2* R,
                double* cs, double2* sn, double2* gvec, const double* target, int32_t* done, int32_t* steps,
                double2* aux, double2* coefQ, double2* coefV, int na, int lda, hipStream_t st, int32_t* stop)
{
    hipLaunchKernelGGL(k_dcgs2_fix, dim3((unsigned)((na + 63) / 64)), dim3(64), 0, st, k, m, final_only ? 1 : 0, G,
                       nrm, H, R, cs, sn, gvec, target, done, steps, aux, na, lda, stop);
    // with a stop flag: raise it as soon as the rotations have finished every column
    if (stop) hipLaunchKernelGGL(k_all_done, dim3(1), dim3(256), 0, st, done, na, stop);
    if (final_only) return;
    hipLaunchKernelGGL(k_dcgs2_coef, dim3((unsigned)((k + 4) / 4), (unsigned)((na + 63) / 64)), dim3(256), 0, st, k,
                       m, G, aux, H, done, coefQ, coefV, na, lda, stop);
}

void dcgs2_update(double2* V, int64_t vstride, int k, const double2* coefQ, const double2* coefV, double2* w,
                  double* norm_partial, int na, int lda, int64_t nup, hipStream_t st, const int32_t* chunk_seg,
                  int ldc, const int32_t* stop)
{
    hipLaunchKernelGGL(k_dcgs2_update, dim3(update_chunks(nup), (unsigned)((na + 63) / 64)), dim3(256), 0, st, V,
                       vstride, k, coefQ, coefV, w, norm_partial, na, lda, nup, chunk_seg, chunk_seg ? ldc : lda, stop);
}

void spmm_het(const Geometry& g, const void* Y, bool y_is_f32, int ldy, const double2* X, const double2* het,
              const double2* B, double2* W, int na, int lda, double mu_sign, hipStream_t st, const int32_t* stop)
{
    const dim3 grid((unsigned)((g.nup + 3) / 4), (unsigned)((lda + 63) / 64));
    if (y_is_f32)
        hipLaunchKernelGGL(k_spmm_het<float>, grid, dim3(256), 0, st, g.row_ptr, g.col, g.val, g.type, g.hrow,
                           static_cast<const float*>(Y), ldy, X, het, B, W, g.n, g.np, g.nup, na, lda, mu_sign, stop);
    else
        hipLaunchKernelGGL(k_spmm_het<double>, grid, dim3(256), 0, st, g.row_ptr, g.col, g.val, g.type, g.hrow,
                           static_cast<const double*>(Y), ldy, X, het, B, W, g.n, g.np, g.nup, na, lda, mu_sign, stop);
}

void build_rhs_het(const Geometry& g, const int32_t* col_pol, const double2* gam, double e0, double2* b, int ncol,
                   int ldb, double mu_sign, hipStream_t st)
{
    hipLaunchKernelGGL(k_rhs_het, dim3((unsigned)((g.nup + 3) / 4), (unsigned)((ldb + 63) / 64)), dim3(256), 0, st,
                       g.row_ptr, g.col, g.val, g.type, g.hrow, g.xyz64, col_pol, gam, e0, b, g.n, g.np, g.nup, ncol,
                       ldb, mu_sign);
}

}  // namespace px
