// Matrix-free interaction-kernel apply Y = T X (plasmonX paper: Eq. tqq for
// omegaFQ; the T^qq / T^qmu / T^muq / T^mumu blocks of Eq. wfqfmu-system,
// obtained by differentiating the Gaussian charge kernel, for omegaFQFmu).
//
// T is never stored: every tile is generated in registers directly in the
// A-operand layout of the matrix instructions and contracted against X tiles
// staged through LDS.  T is real and shared by every frequency and
// polarization, so a block of n_c complex columns is an N x 2n_c real
// contraction.
//
//   tapply_f32  omegaFQ: v_mfma_f32_32x32x2f32, wave tile 64 rows x 128 columns
//               omegaFQFmu: v_mfma_f32_32x32x2f32, wave tile 32 atoms x 4
//               components x 32 columns (one pair block feeds 16 MFMAs)
//   tapply_f64  >= 128 real columns: v_mfma_f64_16x16x4f64 tiles
//               narrow blocks (<= 8 real columns): FP64 VALU with a split over
//               the source atoms and a deterministic second-pass sum
//
// Near/far split: atoms are in Morton order and grouped by 32 with bounding
// boxes.  When the boxes of a row group and a source group are farther apart
// than x_far * R, erf(r/R) rounds to 1 in the working precision and the kernel
// takes the point-charge form (1/r and its derivatives); the decision is
// uniform per wave.  The diagonal T_ii is the Gaussian self-interaction
// sqrt(2/pi)/R_q; the dipole self blocks are zero.
#include "px_internal.h"
#include "px_neighbors.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <vector>

namespace px {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr float TWO_OVER_SQRTPI_F = 1.1283791670955126f;
constexpr double TWO_OVER_SQRTPI = 1.1283791670955126;

// erf(x), x >= 0, Abramowitz & Stegun (1964) formula 7.1.26 (absolute error
// <= 1.5e-7): used only in the single-precision near field.
__device__ __forceinline__ float erf_as(float x)
{
    const float p = 0.3275911f;
    const float a1 = 0.254829592f, a2 = -0.284496736f, a3 = 1.421413741f, a4 = -1.453152027f,
                a5 = 1.061405429f;
    float t = __builtin_amdgcn_rcpf(fmaf(p, x, 1.0f));
    float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, a5, a4), a3), a2), a1);
    return 1.0f - poly * __expf(-x * x);
}

// Squared distance between two axis-aligned boxes (0 if they overlap).
__device__ __forceinline__ float box_gap2(float4 alo, float4 ahi, float4 blo, float4 bhi)
{
    float dx = fmaxf(0.0f, fmaxf(blo.x - ahi.x, alo.x - bhi.x));
    float dy = fmaxf(0.0f, fmaxf(blo.y - ahi.y, alo.y - bhi.y));
    float dz = fmaxf(0.0f, fmaxf(blo.z - ahi.z, alo.z - bhi.z));
    return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Far-field thresholds x_far = r / R beyond which the Gaussian factors equal
// their point limits to working precision (erfc(4) < 2^-25; erfc(6) < 2^-54;
// for the dipole kernels the extra x^3 exp(-x^2) terms need 5 and 7).
constexpr double XFAR_Q32 = 4.0, XFAR_Q64 = 6.0, XFAR_D32 = 5.0, XFAR_D64 = 7.0;

// ============================ omegaFQ, FP32 MFMA ============================
// Workgroup: 8 waves, 256 rows x 128 real columns; the X tile of each source
// chunk is staged once in LDS for all eight.  Wave w: rows [row0, row0 + 32)
// as one 32-row MFMA block x four 32-column blocks, i.e. 64 accumulator
// registers, so four waves share each SIMD and hide one another's T
// generation, LDS reads and barriers behind their MFMAs.
// MFMA 32x32x2 operand layout (wave64): A lane l -> (row l%32, k l/32);
// B lane l -> (k l/32, col l%32); D register v of lane l -> (row 8(v/4) +
// 4(l/32) + v%4, col l%32).  MFMA column n of block cb is physical column
// 4n + cb, so one ds_read_b128 yields a lane's four B values and one 16-byte
// store writes its four outputs.
constexpr int Q32_COLS = 128;
constexpr int Q32_JC = 32;
constexpr int Q32_THREADS = 512;

// Work decomposition (stream-K): the (output tile, source chunk) iterations of
// all tiles are laid end to end and cut into one equal contiguous range per
// resident workgroup, so every CU gets the same MFMA work whatever the tile
// count.  A range covers the tail of one tile, any number of whole tiles and
// the head of another; whole tiles are written to Y directly, the partial
// first and last pieces to two scratch slots per workgroup, which
// k_sk_fixup adds in workgroup order (a fixed order for a given launch shape).
__device__ __forceinline__ void mfma4(f32x16 (&acc)[4], float a, float4 b)
{
    acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b.x, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b.y, acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b.z, acc[2], 0, 0, 0);
    acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b.w, acc[3], 0, 0, 0);
}

// Output tile (row block bx, column block by) over source chunks [cbeg, cend);
// the 256 x 128 result goes to out (its element (0, 0)), rows ldo apart.
__device__ __forceinline__ void tapply_wfq_f32_body(int bx, int by, int cbeg, int cend,
                                                        const float4* __restrict__ xyz,
                                                        const float4* __restrict__ glo,
                                                        const float4* __restrict__ ghi,
                                                        const float* __restrict__ X, float* __restrict__ out, int ldo,
                                                        int ldx, float inv_rqq, float t_self, float r_far2)
{
    __shared__ __attribute__((aligned(16))) float sx[2][Q32_JC][Q32_COLS];
    __shared__ float4 sxyz[2][Q32_JC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const int row0 = bx * 256 + wave * 32;
    const int col0 = by * Q32_COLS;

    const int ii = row0 + (lane & 31);
    const float4 pi = xyz[ii];
    const float xi = pi.x, yi = pi.y, zi = pi.z;
    const float4 rlo = glo[row0 >> 5], rhi = ghi[row0 >> 5];

    f32x16 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[cb][v] = 0.0f;

    // cooperative tile load: thread -> (row tid/16, 8 columns at 8*(tid%16))
    const int lr = tid >> 4;
    const int lc = (tid & 15) * 8;
    if (cbeg < cend) {
        const int j0 = cbeg * Q32_JC;
        const float4* src = reinterpret_cast<const float4*>(X + (size_t)(j0 + lr) * ldx + col0 + lc);
        float4* dst = reinterpret_cast<float4*>(&sx[0][lr][lc]);
        dst[0] = src[0];
        dst[1] = src[1];
        if (tid < Q32_JC) sxyz[0][tid] = xyz[j0 + tid];
    }
    __syncthreads();

    const int half = lane >> 5;
    const int col4 = 4 * (lane & 31);
    for (int ch = cbeg; ch < cend; ++ch) {
        const int buf = (ch - cbeg) & 1;
        const int j0 = ch * Q32_JC;
        const bool more = (ch + 1) < cend;
        // next chunk: global -> registers now, registers -> LDS in mid-loop
        // (on the last chunk the loads re-read this chunk's rows and are never stored)
        const int jn = more ? j0 + Q32_JC : j0;
        const float4* nsrc = reinterpret_cast<const float4*>(X + (size_t)(jn + lr) * ldx + col0 + lc);
        const float4 pre0 = nsrc[0];
        const float4 pre1 = nsrc[1];
        const float4 prexyz = xyz[jn + (tid & (Q32_JC - 1))];
        const int far = uniform(box_gap2(rlo, rhi, glo[ch], ghi[ch]) >= r_far2);
        // operands of the next k-step are read from LDS before this step's MFMAs
        float4 pj = sxyz[buf][half];
        float4 bq = *reinterpret_cast<const float4*>(&sx[buf][half][col4]);
#pragma unroll
        for (int kk = 0; kk < Q32_JC / 2; ++kk) {
            float4 pjn = pj, bqn = bq;
            if (kk + 1 < Q32_JC / 2) {
                pjn = sxyz[buf][2 * kk + 2 + half];
                bqn = *reinterpret_cast<const float4*>(&sx[buf][2 * kk + 2 + half][col4]);
            }
            const float dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            float a = __builtin_amdgcn_rsqf(r2);
            // Gaussian near field, only for the k-steps where some pair of the
            // wave is closer than the far threshold (wave-uniform branches;
            // only the A value changes)
            if (!far && __any(r2 < r_far2)) {
                const int j = j0 + 2 * kk + half;
                const float t = erf_as(r2 * a * inv_rqq) * a;
                a = (ii == j) ? t_self : t;
            }
            mfma4(acc, a, bq);
            pj = pjn;
            bq = bqn;
            if (kk == Q32_JC / 4 && more) {
                // the other buffer was released at the previous barrier
                float4* dst = reinterpret_cast<float4*>(&sx[buf ^ 1][lr][lc]);
                dst[0] = pre0;
                dst[1] = pre1;
                if (tid < Q32_JC) sxyz[buf ^ 1][tid] = prexyz;
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = wave * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        const float4 o = make_float4(acc[0][v], acc[1][v], acc[2][v], acc[3][v]);
        *reinterpret_cast<float4*>(out + (size_t)i * ldo + col4) = o;
    }
}

// ---- stream-K bookkeeping ----------------------------------------------------
// Tiles t = 0..T-1 with C_t chunks each start at iteration pre[t]; without a
// tile list (single structure) tile t is (row block t % RB, column block
// t / RB) with C chunks.  Workgroup b owns iterations [begin(b), begin(b+1)).
struct SkGrid {
    const int4* tiles;       // {segment, row block, column block, chunks} or null
    const int64_t* pre;      // [T + 1] or null
    int T, RB, C, G;
    int64_t total;
};

constexpr int SK_TILE_FLOATS = 256 * Q32_COLS;

__device__ __forceinline__ int64_t sk_begin(const SkGrid& s, int b) { return s.total * b / s.G; }
__device__ __forceinline__ int64_t sk_pre(const SkGrid& s, int t) { return s.pre ? s.pre[t] : (int64_t)t * s.C; }

__device__ int sk_tile_of(const SkGrid& s, int64_t i)
{
    if (!s.pre) return (int)(i / s.C);
    int lo = 0, hi = s.T - 1;   // largest t with pre[t] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.pre[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ int sk_block_of(const SkGrid& s, int64_t i)
{
    int b = (int)(i * s.G / s.total);   // largest b with begin(b) <= i
    while (b + 1 < s.G && sk_begin(s, b + 1) <= i) ++b;
    while (b > 0 && sk_begin(s, b) > i) --b;
    return b;
}

// Workgroup b's pieces: calls f(tile, c0, c1, slot) in order; slot is -1 for
// a whole tile, else the scratch slot (2b for the first piece, 2b+1 for the
// last).
template <class F>
__device__ __forceinline__ void sk_pieces(const SkGrid& s, int b, F&& f)
{
    int64_t it = sk_begin(s, b);
    const int64_t end = sk_begin(s, b + 1);
    bool first = true;
    while (it < end) {
        const int t = uniform(sk_tile_of(s, it));
        const int64_t p0 = sk_pre(s, t);
        const int ct = s.tiles ? s.tiles[t].w : s.C;
        const int c0 = (int)(it - p0);
        const int c1 = (int)min((int64_t)ct, (int64_t)c0 + (end - it));
        const int slot = (c0 == 0 && c1 == ct) ? -1 : 2 * b + (first ? 0 : 1);
        f(t, c0, c1, slot);
        it += c1 - c0;
        first = false;
    }
}

__global__ __launch_bounds__(Q32_THREADS) void k_tapply_wfq_f32(const float4* __restrict__ xyz,
                                                                const float4* __restrict__ glo,
                                                                const float4* __restrict__ ghi,
                                                                const float* __restrict__ X, float* __restrict__ Y,
                                                                float* __restrict__ partial, int ldx, SkGrid sk,
                                                                float inv_rqq, float t_self, float r_far2,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    sk_pieces(sk, blockIdx.x, [&](int t, int c0, int c1, int slot) {
        const int rb = t % sk.RB, cb = t / sk.RB;
        float* out = slot < 0 ? Y + (size_t)rb * 256 * ldx + cb * Q32_COLS : partial + (size_t)slot * SK_TILE_FLOATS;
        tapply_wfq_f32_body(rb, cb, c0, c1, xyz, glo, ghi, X, out, slot < 0 ? ldx : Q32_COLS, ldx, inv_rqq, t_self,
                            r_far2);
    });
}

// ---- stored T (the paper's in-memory solver), FP32 --------------------------
// Y = T X with T stored dense (row-major nup x nup, ld = ldt) for either model:
// the tiles and stream-K pieces of the on-the-fly kernel, the A operand read
// from memory instead of generated.  T is symmetric (T_ij = T_ji holds bit for
// bit in the dense builders: swapping i and j negates the components of r
// exactly), so lane l of k-step kk, which needs T[i][j] for row i = row0 +
// l%32 and source j = j0 + 2 kk + l/32, reads T[j][i]: the 32 lanes of a
// half-wave read 128 contiguous bytes.  The next chunk's 16 values per lane
// are loaded while the current chunk's MFMAs run.  NB = 4 computes all 128
// columns of a tile (MFMA column n of block cb is tile column 4n + cb); NB = 2
// only its first 64 (column 2n + cb), for a last column block whose other
// half holds no active column (the sparse apply never reads those).
template <int NB>
__device__ __forceinline__ void tstored_f32_body(int bx, int by, int cbeg, int cend, const float* __restrict__ Ts,
                                                 int ldt, const float* __restrict__ X, float* __restrict__ out,
                                                 int ldo, int ldx)
{
    static_assert(NB == 2 || NB == 4, "four or two 32-column MFMA blocks per tile");
    __shared__ __attribute__((aligned(16))) float sx[2][Q32_JC][Q32_COLS];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const int row0 = bx * 256 + wave * 32;
    const int col0 = by * Q32_COLS;
    const int ii = row0 + (lane & 31);
    const int half = lane >> 5;
    const int coln = NB * (lane & 31);

    f32x16 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[cb][v] = 0.0f;

    const int lr = tid >> 4;
    const int lc = (tid & 15) * 8;
    float tv[Q32_JC / 2];
    if (cbeg < cend) {
        const int j0 = cbeg * Q32_JC;
        const float4* src = reinterpret_cast<const float4*>(X + (size_t)(j0 + lr) * ldx + col0 + lc);
        float4* dst = reinterpret_cast<float4*>(&sx[0][lr][lc]);
        dst[0] = src[0];
        dst[1] = src[1];
#pragma unroll
        for (int kk = 0; kk < Q32_JC / 2; ++kk) tv[kk] = Ts[(size_t)(j0 + 2 * kk + half) * ldt + ii];
    }
    __syncthreads();

    for (int ch = cbeg; ch < cend; ++ch) {
        const int buf = (ch - cbeg) & 1;
        const int j0 = ch * Q32_JC;
        const bool more = (ch + 1) < cend;
        const int jn = more ? j0 + Q32_JC : j0;
        const float4* nsrc = reinterpret_cast<const float4*>(X + (size_t)(jn + lr) * ldx + col0 + lc);
        const float4 pre0 = nsrc[0];
        const float4 pre1 = nsrc[1];
        float tn[Q32_JC / 2];
#pragma unroll
        for (int kk = 0; kk < Q32_JC / 2; ++kk) tn[kk] = Ts[(size_t)(jn + 2 * kk + half) * ldt + ii];
        if constexpr (NB == 4) {
            float4 bq = *reinterpret_cast<const float4*>(&sx[buf][half][coln]);
#pragma unroll
            for (int kk = 0; kk < Q32_JC / 2; ++kk) {
                float4 bqn = bq;
                if (kk + 1 < Q32_JC / 2) bqn = *reinterpret_cast<const float4*>(&sx[buf][2 * kk + 2 + half][coln]);
                mfma4(acc, tv[kk], bq);
                bq = bqn;
                if (kk == Q32_JC / 4 && more) {
                    float4* dst = reinterpret_cast<float4*>(&sx[buf ^ 1][lr][lc]);
                    dst[0] = pre0;
                    dst[1] = pre1;
                }
            }
        } else {
            float2 bq = *reinterpret_cast<const float2*>(&sx[buf][half][coln]);
#pragma unroll
            for (int kk = 0; kk < Q32_JC / 2; ++kk) {
                float2 bqn = bq;
                if (kk + 1 < Q32_JC / 2) bqn = *reinterpret_cast<const float2*>(&sx[buf][2 * kk + 2 + half][coln]);
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(tv[kk], bq.x, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(tv[kk], bq.y, acc[1], 0, 0, 0);
                bq = bqn;
                if (kk == Q32_JC / 4 && more) {
                    float4* dst = reinterpret_cast<float4*>(&sx[buf ^ 1][lr][lc]);
                    dst[0] = pre0;
                    dst[1] = pre1;
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < Q32_JC / 2; ++kk) tv[kk] = tn[kk];
        __syncthreads();
    }

#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = wave * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        if constexpr (NB == 4) {
            const float4 o = make_float4(acc[0][v], acc[1][v], acc[2][v], acc[3][v]);
            *reinterpret_cast<float4*>(out + (size_t)i * ldo + coln) = o;
        } else {
            *reinterpret_cast<float2*>(out + (size_t)i * ldo + coln) = make_float2(acc[0][v], acc[1][v]);
        }
    }
}

template <int NB>
__global__ __launch_bounds__(Q32_THREADS) void k_tstored_f32(const float* __restrict__ Ts, int ldt,
                                                             const float* __restrict__ X, float* __restrict__ Y,
                                                             float* __restrict__ partial, int ldx, SkGrid sk,
                                                             const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    sk_pieces(sk, blockIdx.x, [&](int t, int c0, int c1, int slot) {
        const int rb = t % sk.RB, cb = t / sk.RB;
        float* out = slot < 0 ? Y + (size_t)rb * 256 * ldx + cb * Q32_COLS : partial + (size_t)slot * SK_TILE_FLOATS;
        tstored_f32_body<NB>(rb, cb, c0, c1, Ts, ldt, X, out, slot < 0 ? ldx : Q32_COLS, ldx);
    });
}

// ========================== omegaFQFmu, FP32 MFMA ===========================
// Workgroup: 4 waves x 32 atoms, 32 real columns.  Each lane builds the 4x4
// pair block of (row atom l%32, source atom 2kk + l/32) once and feeds the 16
// (output component, input component) MFMAs of the k-step with it.
constexpr int D32_COLS = 32;
constexpr int D32_JC = 32;

struct DipoleConstF {
    float inv_rqq, inv_rqm, inv_rmm;   // 1/R for the three widths
    float gauss_pref;                  // (4/sqrt(pi)) / R_mumu^3
    float t_self;                      // sqrt(2/pi)/R_q
    float r_far2;
};

// Pair block b[a][c] (a: output component of row atom, c: input component of
// source atom; 0 = q, 1..3 = mu_x..mu_z) for rv = r_i - r_j.
__device__ __forceinline__ void pair_block_f32(float dx, float dy, float dz, bool far, const DipoleConstF& k,
                                               float b[4][4])
{
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float rinv = __builtin_amdgcn_rsqf(r2);
    float rinv3 = rinv * rinv * rinv;
    float tqq, gq, gm, gs;
    if (far) {
        tqq = rinv;
        gq = 1.0f;
        gm = 1.0f;
        gs = 0.0f;
    } else {
        float r = r2 * rinv;
        float xq = r * k.inv_rqq, xm = r * k.inv_rqm, xmm = r * k.inv_rmm;
        tqq = erf_as(xq) * rinv;
        gq = erf_as(xm) - TWO_OVER_SQRTPI_F * xm * __expf(-xm * xm);
        float e = __expf(-xmm * xmm);
        gm = erf_as(xmm) - TWO_OVER_SQRTPI_F * xmm * e;
        gs = k.gauss_pref * e;
    }
    float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
    float u[3] = {ux, uy, uz};
    b[0][0] = tqq;
    float gr = gq * rinv * rinv;   // g / r^2
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b[0][1 + a] = gr * u[a];
        b[1 + a][0] = -gr * u[a];
    }
    float gm3 = gm * rinv3;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float uu = u[a] * u[c];
            b[1 + a][1 + c] = fmaf(gs - 3.0f * gm3, uu, (a == c) ? gm3 : 0.0f);
        }
}

__device__ __forceinline__ void tapply_wfqfmu_f32_body(int bx, int by, int bz, const float4* __restrict__ xyz,
                                                           const float4* __restrict__ glo,
                                                           const float4* __restrict__ ghi,
                                                           const float* __restrict__ X, float* __restrict__ Y,
                                                           int np, int ldx, DipoleConstF kc)
{
    __shared__ float sx[2][4][D32_JC][D32_COLS];
    __shared__ float4 sxyz[2][D32_JC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int row0 = bx * 128 + wave * 32;
    const int col0 = by * D32_COLS;
    const size_t cstride = (size_t)np * ldx;   // component block stride

    const int ii = row0 + (lane & 31);
    const float4 pi = xyz[ii];
    const float4 rlo = glo[row0 >> 5], rhi = ghi[row0 >> 5];

    f32x16 acc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][v] = 0.0f;

    // tile load: 4 comps x 32 atoms x 32 cols = 4096 floats; thread -> comp tid/64,
    // atom (tid%64)/2, 16 columns at 16*(tid%2)
    const int lcomp = tid >> 6;
    const int latom = (tid & 63) >> 1;
    const int lcol = (tid & 1) * 16;
    const int nchunk = np / D32_JC;
    {
        const float4* src = reinterpret_cast<const float4*>(X + lcomp * cstride + (size_t)latom * ldx + col0 + lcol);
        float4* dst = reinterpret_cast<float4*>(&sx[0][lcomp][latom][lcol]);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = src[q];
        if (tid < D32_JC) sxyz[0][tid] = xyz[tid];
    }
    __syncthreads();

    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        const int j0 = ch * D32_JC;
        const bool more = (ch + 1) < nchunk;
        float4 pre[4];
        float4 prexyz = make_float4(0.f, 0.f, 0.f, 0.f);
        if (more) {
            const float4* src = reinterpret_cast<const float4*>(X + lcomp * cstride +
                                                                (size_t)(j0 + D32_JC + latom) * ldx + col0 + lcol);
#pragma unroll
            for (int q = 0; q < 4; ++q) pre[q] = src[q];
            if (tid < D32_JC) prexyz = xyz[j0 + D32_JC + tid];
        }
        const int far = uniform(box_gap2(rlo, rhi, glo[ch], ghi[ch]) >= kc.r_far2);

#pragma unroll 2
        for (int kk = 0; kk < D32_JC / 2; ++kk) {
            const int jr = 2 * kk + (lane >> 5);
            const float4 pj = sxyz[buf][jr];
            const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            // point forms unless some pair of the wave is inside the far threshold
            const bool fstep = far || !__any(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < kc.r_far2);
            float b[4][4];
            pair_block_f32(dx, dy, dz, fstep, kc, b);
            if (!fstep && ii == j0 + jr) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) b[a][c] = 0.0f;
                b[0][0] = kc.t_self;
            }
            float xb[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) xb[c] = sx[buf][c][jr][lane & 31];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a] = __builtin_amdgcn_mfma_f32_32x32x2f32(b[a][c], xb[c], acc[a], 0, 0, 0);
        }
        if (more) {
            float4* dst = reinterpret_cast<float4*>(&sx[buf ^ 1][lcomp][latom][lcol]);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = pre[q];
            if (tid < D32_JC) sxyz[buf ^ 1][tid] = prexyz;
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = row0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            Y[a * cstride + (size_t)i * ldx + col0 + (lane & 31)] = acc[a][v];
        }
}

__global__ __launch_bounds__(256) void k_tapply_wfqfmu_f32(const float4* __restrict__ xyz,
                                                           const float4* __restrict__ glo,
                                                           const float4* __restrict__ ghi,
                                                           const float* __restrict__ X, float* __restrict__ Y,
                                                           int np, int ldx, DipoleConstF kc,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    tapply_wfqfmu_f32_body(blockIdx.x, blockIdx.y, blockIdx.z, xyz, glo, ghi, X, Y, np, ldx, kc);
}

// ============================ omegaFQ, FP64 MFMA ============================
// Workgroup: 4 waves x 32 rows, 64 real columns.  MFMA 16x16x4 f64 layout:
// A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16); D register v
// of lane l -> (row 4v + l/16, col l%16) (rows interleave across the four
// lane groups, unlike the f32 16x16x4 form).  MFMA column n of block cb is
// physical column 4n + cb.
constexpr int Q64_COLS = 64;
constexpr int Q64_JC = 32;

__device__ __forceinline__ void tapply_wfq_f64_body(int bx, int by, int bz, const double4* __restrict__ xyz,
                                                        const float4* __restrict__ glo,
                                                        const float4* __restrict__ ghi,
                                                        const double* __restrict__ X, double* __restrict__ Y,
                                                        int np, int ldx, double inv_rqq, double t_self,
                                                        float r_far2)
{
    __shared__ __attribute__((aligned(16))) double sx[2][Q64_JC][Q64_COLS];
    __shared__ double4 sxyz[2][Q64_JC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int row0 = bx * 128 + wave * 32;
    const int col0 = by * Q64_COLS;

    double xi[2], yi[2], zi[2];
    int ii[2];
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) {
        ii[sb] = row0 + sb * 16 + (lane & 15);
        double4 p = xyz[ii[sb]];
        xi[sb] = p.x; yi[sb] = p.y; zi[sb] = p.z;
    }
    const float4 rlo = glo[row0 >> 5], rhi = ghi[row0 >> 5];

    f64x4 acc[2][4];
#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[sb][cb][v] = 0.0;

    // tile load: 32 atoms x 64 doubles = 2048 doubles; thread -> row tid/8, 8 doubles at 8*(tid%8)
    const int lr = tid >> 3;
    const int lc = (tid & 7) * 8;
    const int nchunk = np / Q64_JC;
    {
        const double2* src = reinterpret_cast<const double2*>(X + (size_t)lr * ldx + col0 + lc);
        double2* dst = reinterpret_cast<double2*>(&sx[0][lr][lc]);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = src[q];
        if (tid < Q64_JC) sxyz[0][tid] = xyz[tid];
    }
    __syncthreads();

    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        const int j0 = ch * Q64_JC;
        const bool more = (ch + 1) < nchunk;
        double2 pre[4];
        double4 prexyz = make_double4(0, 0, 0, 0);
        if (more) {
            const double2* src = reinterpret_cast<const double2*>(X + (size_t)(j0 + Q64_JC + lr) * ldx + col0 + lc);
#pragma unroll
            for (int q = 0; q < 4; ++q) pre[q] = src[q];
            if (tid < Q64_JC) prexyz = xyz[j0 + Q64_JC + tid];
        }
        const int far = uniform(box_gap2(rlo, rhi, glo[ch], ghi[ch]) >= r_far2);

#pragma unroll 2
        for (int kk = 0; kk < Q64_JC / 4; ++kk) {
            const int jr = 4 * kk + (lane >> 4);
            const double4 pj = sxyz[buf][jr];
            const double2* bp = reinterpret_cast<const double2*>(&sx[buf][jr][4 * (lane & 15)]);
            const double2 b01 = bp[0], b23 = bp[1];
            double a[2], r2[2];
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                double dx = xi[sb] - pj.x, dy = yi[sb] - pj.y, dz = zi[sb] - pj.z;
                r2[sb] = fma(dx, dx, fma(dy, dy, dz * dz));
                a[sb] = rsqrt(r2[sb]);
            }
            // Gaussian form only for the k-steps with a pair inside the far threshold
            if (!far && __any(r2[0] < (double)r_far2 || r2[1] < (double)r_far2)) {
#pragma unroll
                for (int sb = 0; sb < 2; ++sb) {
                    const double t = erf(r2[sb] * a[sb] * inv_rqq) * a[sb];
                    a[sb] = (ii[sb] == j0 + jr) ? t_self : t;
                }
            }
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                acc[sb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sb], b01.x, acc[sb][0], 0, 0, 0);
                acc[sb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sb], b01.y, acc[sb][1], 0, 0, 0);
                acc[sb][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sb], b23.x, acc[sb][2], 0, 0, 0);
                acc[sb][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sb], b23.y, acc[sb][3], 0, 0, 0);
            }
        }
        if (more) {
            double2* dst = reinterpret_cast<double2*>(&sx[buf ^ 1][lr][lc]);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = pre[q];
            if (tid < Q64_JC) sxyz[buf ^ 1][tid] = prexyz;
        }
        __syncthreads();
    }

#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = row0 + sb * 16 + 4 * v + (lane >> 4);
            double2* dst = reinterpret_cast<double2*>(Y + (size_t)i * ldx + col0 + 4 * (lane & 15));
            dst[0] = make_double2(acc[sb][0][v], acc[sb][1][v]);
            dst[1] = make_double2(acc[sb][2][v], acc[sb][3][v]);
        }
}

__global__ __launch_bounds__(256) void k_tapply_wfq_f64(const double4* __restrict__ xyz,
                                                        const float4* __restrict__ glo,
                                                        const float4* __restrict__ ghi,
                                                        const double* __restrict__ X, double* __restrict__ Y,
                                                        int np, int ldx, double inv_rqq, double t_self,
                                                        float r_far2,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    tapply_wfq_f64_body(blockIdx.x, blockIdx.y, blockIdx.z, xyz, glo, ghi, X, Y, np, ldx, inv_rqq, t_self, r_far2);
}

// ---- stored T, FP64 (either model): the tiles of the on-the-fly FP64 MFMA
// kernel with the A operand read as T[j][i] (T symmetric): the 16 lanes of a
// row group read 128 contiguous bytes; the next chunk's 16 values per lane
// are loaded while the current chunk's MFMAs run.
__global__ __launch_bounds__(256) void k_tstored_f64(const double* __restrict__ Ts, int ldt,
                                                     const double* __restrict__ X, double* __restrict__ Y, int nup,
                                                     int ldx, const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    __shared__ __attribute__((aligned(16))) double sx[2][Q64_JC][Q64_COLS];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int row0 = blockIdx.x * 128 + wave * 32;
    const int col0 = blockIdx.y * Q64_COLS;
    int ii[2];
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) ii[sb] = row0 + sb * 16 + (lane & 15);
    f64x4 acc[2][4];
#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[sb][cb][v] = 0.0;
    const int lr = tid >> 3;
    const int lc = (tid & 7) * 8;
    const int nchunk = nup / Q64_JC;
    double tv[Q64_JC / 4][2];
    {
        const double2* src = reinterpret_cast<const double2*>(X + (size_t)lr * ldx + col0 + lc);
        double2* dst = reinterpret_cast<double2*>(&sx[0][lr][lc]);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = src[q];
#pragma unroll
        for (int kk = 0; kk < Q64_JC / 4; ++kk)
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) tv[kk][sb] = Ts[(size_t)(4 * kk + (lane >> 4)) * ldt + ii[sb]];
    }
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        const int j0 = ch * Q64_JC;
        const bool more = (ch + 1) < nchunk;
        const int jn = more ? j0 + Q64_JC : j0;
        double2 pre[4];
        const double2* src = reinterpret_cast<const double2*>(X + (size_t)(jn + lr) * ldx + col0 + lc);
#pragma unroll
        for (int q = 0; q < 4; ++q) pre[q] = src[q];
        double tn[Q64_JC / 4][2];
#pragma unroll
        for (int kk = 0; kk < Q64_JC / 4; ++kk)
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) tn[kk][sb] = Ts[(size_t)(jn + 4 * kk + (lane >> 4)) * ldt + ii[sb]];
#pragma unroll
        for (int kk = 0; kk < Q64_JC / 4; ++kk) {
            const int jr = 4 * kk + (lane >> 4);
            const double2* bp = reinterpret_cast<const double2*>(&sx[buf][jr][4 * (lane & 15)]);
            const double2 b01 = bp[0], b23 = bp[1];
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                acc[sb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[kk][sb], b01.x, acc[sb][0], 0, 0, 0);
                acc[sb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[kk][sb], b01.y, acc[sb][1], 0, 0, 0);
                acc[sb][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[kk][sb], b23.x, acc[sb][2], 0, 0, 0);
                acc[sb][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[kk][sb], b23.y, acc[sb][3], 0, 0, 0);
            }
        }
        if (more) {
            double2* dst = reinterpret_cast<double2*>(&sx[buf ^ 1][lr][lc]);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = pre[q];
        }
#pragma unroll
        for (int kk = 0; kk < Q64_JC / 4; ++kk)
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) tv[kk][sb] = tn[kk][sb];
        __syncthreads();
    }
#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = row0 + sb * 16 + 4 * v + (lane >> 4);
            double2* dst = reinterpret_cast<double2*>(Y + (size_t)i * ldx + col0 + 4 * (lane & 15));
            dst[0] = make_double2(acc[sb][0][v], acc[sb][1][v]);
            dst[1] = make_double2(acc[sb][2][v], acc[sb][3][v]);
        }
}

// Stored T, FP64, 1-8 real columns (the shared-Krylov phase's matvec on a
// stored T; a memory-bound pass over T): thread t of row block x takes row
// i = 256 x + t; split y of the sources sums T[j][i] x_j (T symmetric, so the
// 64 lanes of a wave read 512 contiguous bytes of row j, and x_j is a
// wave-uniform load) over its share of the rows j; k_sum_splits adds the
// splits.
template <int NC>
__global__ __launch_bounds__(256) void k_tstored_narrow(const double* __restrict__ Ts, int ldt,
                                                        const double* __restrict__ X, double* __restrict__ part,
                                                        int nup, int per_split, const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j0 = blockIdx.y * per_split;
    const int j1 = min(nup, j0 + per_split);
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
        const double t = Ts[(size_t)j * ldt + i];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = fma(t, X[(size_t)j * NC + c], acc[c]);
    }
    double* out = part + (size_t)blockIdx.y * nup * NC;
#pragma unroll
    for (int c = 0; c < NC; ++c) out[(size_t)i * NC + c] = acc[c];
}

// ========================== omegaFQFmu, FP64 MFMA ===========================
// Workgroup: 4 waves x 16 atoms, 16 real columns; 16 MFMAs per k-step.
struct DipoleConstD {
    double inv_rqq, inv_rqm, inv_rmm, gauss_pref, t_self;
    float r_far2;
};

__device__ __forceinline__ void pair_block_f64(double dx, double dy, double dz, bool far, const DipoleConstD& k,
                                               double b[4][4])
{
    double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    double rinv = rsqrt(r2);
    double rinv3 = rinv * rinv * rinv;
    double tqq, gq, gm, gs;
    if (far) {
        tqq = rinv;
        gq = 1.0;
        gm = 1.0;
        gs = 0.0;
    } else {
        double r = r2 * rinv;
        double xq = r * k.inv_rqq, xm = r * k.inv_rqm, xmm = r * k.inv_rmm;
        tqq = erf(xq) * rinv;
        gq = erf(xm) - TWO_OVER_SQRTPI * xm * exp(-xm * xm);
        double e = exp(-xmm * xmm);
        gm = erf(xmm) - TWO_OVER_SQRTPI * xmm * e;
        gs = k.gauss_pref * e;
    }
    double u[3] = {dx * rinv, dy * rinv, dz * rinv};
    b[0][0] = tqq;
    double gr = gq * rinv * rinv;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b[0][1 + a] = gr * u[a];
        b[1 + a][0] = -gr * u[a];
    }
    double gm3 = gm * rinv3;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double uu = u[a] * u[c];
            b[1 + a][1 + c] = fma(gs - 3.0 * gm3, uu, (a == c) ? gm3 : 0.0);
        }
}

constexpr int D64_COLS = 16;
constexpr int D64_JC = 32;

__device__ __forceinline__ void tapply_wfqfmu_f64_body(int bx, int by, int bz, const double4* __restrict__ xyz,
                                                           const float4* __restrict__ glo,
                                                           const float4* __restrict__ ghi,
                                                           const double* __restrict__ X, double* __restrict__ Y,
                                                           int np, int ldx, DipoleConstD kc)
{
    __shared__ double sx[2][4][D64_JC][D64_COLS];
    __shared__ double4 sxyz[2][D64_JC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int row0 = bx * 64 + wave * 16;
    const int col0 = by * D64_COLS;
    const size_t cstride = (size_t)np * ldx;

    const int ii = row0 + (lane & 15);
    const double4 pi = xyz[ii];
    const float4 rlo = glo[row0 >> 5], rhi = ghi[row0 >> 5];

    f64x4 acc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[a][v] = 0.0;

    // tile load: 4 comps x 32 atoms x 16 cols = 2048 doubles; thread -> comp tid/64,
    // atom (tid%64)/2, 8 doubles at 8*(tid%2)
    const int lcomp = tid >> 6;
    const int latom = (tid & 63) >> 1;
    const int lcol = (tid & 1) * 8;
    const int nchunk = np / D64_JC;
    {
        const double2* src = reinterpret_cast<const double2*>(X + lcomp * cstride + (size_t)latom * ldx + col0 + lcol);
        double2* dst = reinterpret_cast<double2*>(&sx[0][lcomp][latom][lcol]);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = src[q];
        if (tid < D64_JC) sxyz[0][tid] = xyz[tid];
    }
    __syncthreads();

    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        const int j0 = ch * D64_JC;
        const bool more = (ch + 1) < nchunk;
        double2 pre[4];
        double4 prexyz = make_double4(0, 0, 0, 0);
        if (more) {
            const double2* src = reinterpret_cast<const double2*>(X + lcomp * cstride +
                                                                  (size_t)(j0 + D64_JC + latom) * ldx + col0 + lcol);
#pragma unroll
            for (int q = 0; q < 4; ++q) pre[q] = src[q];
            if (tid < D64_JC) prexyz = xyz[j0 + D64_JC + tid];
        }
        const int far = uniform(box_gap2(rlo, rhi, glo[ch], ghi[ch]) >= kc.r_far2);

        for (int kk = 0; kk < D64_JC / 4; ++kk) {
            const int jr = 4 * kk + (lane >> 4);
            const double4 pj = sxyz[buf][jr];
            const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            const bool fstep = far || !__any(fma(dx, dx, fma(dy, dy, dz * dz)) < (double)kc.r_far2);
            double b[4][4];
            pair_block_f64(dx, dy, dz, fstep, kc, b);
            if (!fstep && ii == j0 + jr) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) b[a][c] = 0.0;
                b[0][0] = kc.t_self;
            }
            double xb[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) xb[c] = sx[buf][c][jr][lane & 15];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[a][c], xb[c], acc[a], 0, 0, 0);
        }
        if (more) {
            double2* dst = reinterpret_cast<double2*>(&sx[buf ^ 1][lcomp][latom][lcol]);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = pre[q];
            if (tid < D64_JC) sxyz[buf ^ 1][tid] = prexyz;
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = row0 + 4 * v + (lane >> 4);
            Y[a * cstride + (size_t)i * ldx + col0 + (lane & 15)] = acc[a][v];
        }
}

__global__ __launch_bounds__(256) void k_tapply_wfqfmu_f64(const double4* __restrict__ xyz,
                                                           const float4* __restrict__ glo,
                                                           const float4* __restrict__ ghi,
                                                           const double* __restrict__ X, double* __restrict__ Y,
                                                           int np, int ldx, DipoleConstD kc,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    tapply_wfqfmu_f64_body(blockIdx.x, blockIdx.y, blockIdx.z, xyz, glo, ghi, X, Y, np, ldx, kc);
}

// ====================== narrow blocks, FP64 VALU ============================
// One thread per row atom, NC real columns (x 4 components for the dipole
// model); the source atoms are split over gridDim.y and the partial sums are
// added in a fixed order by k_sum_splits.
constexpr int NW_CHUNK = 256;

template <int NC, int MODEL>
__global__ __launch_bounds__(256) void k_tapply_f64_narrow(const double4* __restrict__ xyz,
                                                           const float4* __restrict__ glo,
                                                           const float4* __restrict__ ghi,
                                                           const double* __restrict__ X,
                                                           double* __restrict__ part, int np, int chunks_per_split,
                                                           double inv_rqq, double t_self, float r_far2,
                                                           DipoleConstD kc,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    constexpr int NCOMP = MODEL ? 4 : 1;
    __shared__ double4 sxyz[NW_CHUNK];
    __shared__ double sxv[NCOMP][NW_CHUNK][NC];

    const int tid = threadIdx.x;
    const int i = blockIdx.x * 256 + tid;
    const int wave_row0 = blockIdx.x * 256 + (tid & ~63);
    const double4 pi = xyz[i];
    const float4 g0lo = glo[wave_row0 >> 5], g1lo = glo[(wave_row0 >> 5) + 1];
    const float4 g0hi = ghi[wave_row0 >> 5], g1hi = ghi[(wave_row0 >> 5) + 1];
    const float4 rlo = make_float4(fminf(g0lo.x, g1lo.x), fminf(g0lo.y, g1lo.y), fminf(g0lo.z, g1lo.z), 0.f);
    const float4 rhi = make_float4(fmaxf(g0hi.x, g1hi.x), fmaxf(g0hi.y, g1hi.y), fmaxf(g0hi.z, g1hi.z), 0.f);
    const size_t cstride = (size_t)np * NC;

    double acc[NCOMP][NC];
#pragma unroll
    for (int a = 0; a < NCOMP; ++a)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[a][c] = 0.0;

    const int nchunk = np / NW_CHUNK;
    // split y takes chunks y, y + nsplit, ...: the near-field chunks, which lie
    // close together in Morton order, spread over the splits
    (void)chunks_per_split;
    for (int ch = blockIdx.y; ch < nchunk; ch += gridDim.y) {
        const int j0 = ch * NW_CHUNK;
        __syncthreads();
        sxyz[tid] = xyz[j0 + tid];
#pragma unroll
        for (int a = 0; a < NCOMP; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c) sxv[a][tid][c] = X[a * cstride + (size_t)(j0 + tid) * NC + c];
        __syncthreads();
        for (int gq = 0; gq < NW_CHUNK / GROUP; ++gq) {
            const int gidx = (j0 >> 5) + gq;
            const int far = uniform(box_gap2(rlo, rhi, glo[gidx], ghi[gidx]) >= r_far2);
            for (int jj = gq * GROUP; jj < (gq + 1) * GROUP; ++jj) {
                const double4 pj = sxyz[jj];
                const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const bool fstep = far || !__any(r2 < (double)r_far2);
                if (MODEL == 0) {
                    double rinv = rsqrt(r2);
                    double t;
                    if (fstep) {
                        t = rinv;
                    } else {
                        t = erf(r2 * rinv * inv_rqq) * rinv;
                        t = (i == j0 + jj) ? t_self : t;
                    }
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[0][c] = fma(t, sxv[0][jj][c], acc[0][c]);
                } else {
                    double b[4][4];
                    pair_block_f64(dx, dy, dz, fstep, kc, b);
                    if (!fstep && i == j0 + jj) {
#pragma unroll
                        for (int a = 0; a < 4; ++a)
#pragma unroll
                            for (int c = 0; c < 4; ++c) b[a][c] = 0.0;
                        b[0][0] = kc.t_self;
                    }
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int c2 = 0; c2 < 4; ++c2)
#pragma unroll
                            for (int c = 0; c < NC; ++c) acc[a][c] = fma(b[a][c2], sxv[c2][jj][c], acc[a][c]);
                }
            }
        }
    }
    double* out = part + (size_t)blockIdx.y * NCOMP * cstride;
#pragma unroll
    for (int a = 0; a < NCOMP; ++a)
#pragma unroll
        for (int c = 0; c < NC; ++c) out[a * cstride + (size_t)i * NC + c] = acc[a][c];
}

// 1/sqrt(x) for finite x > 0: the hardware estimate refined by one
// third-order step y (1 + e/2 + 3e^2/8), e = 1 - x y^2, which takes the
// estimate's relative error eps to O(eps^3), below FP64 rounding; the library
// call adds only the special-input handling, which a pair distance never needs.
// Twice 1/sqrt(q) for q > 0: the hardware estimate y0 (about 23 correct bits)
// and one Newton step, y0 (3 - q y0^2), whose factor 1/2 the caller applies
// once to its sums.  Relative error below 1e-13 (the Newton step squares the
// estimate's error, times 3/2), in three instructions instead of the five of
// rsqrt_pos.
__device__ __forceinline__ double rsqrt_pos_x2(double q)
{
    const double y = __builtin_amdgcn_rsq(q);
    return y * fma(-q, y * y, 3.0);
}

// The omegaFQ narrow blocks, T = T_point + C.  Split y of a row block applies
// the point part 1/r over the source chunks y, y + nsplit, ... (the self pair
// excluded) and the slots y, y + nsplit, ... of the row block's stored
// near-field correction C (ELL layout, k_near_rows); k_sum_splits adds the
// splits.  The source atoms are read by wave-uniform loads (through the
// scalar cache) instead of LDS: every lane of a wave needs the same source
// atom at each step, so one scalar load serves the whole wave and the LDS
// pipe, which the CU's waves share, leaves the inner loop.  Positions are
// relative to the structure's centre with |p|^2 in w, so that r^2 = |p_i|^2 +
// |p_j|^2 - 2 p_i.p_j takes four instructions; its rounding error, a few
// units of FP64 rounding times the squared radius of the structure, is below
// 1e-12 of r^2 for the nearest pairs of a 100k-atom sphere.  Only the source
// groups that hold one of the wave's own rows need the self pair masked.  The
// correction list is read in the shadow of the ALU-bound pair loop.
template <int NC, int RPT, int RB, int SU>
__global__ __launch_bounds__(RB / RPT) void k_tapply_f64_narrow_q(const double4* __restrict__ xyzc,
                                                                   const double* __restrict__ X,
                                                                   double* __restrict__ part, int np,
                                                                   const int64_t* __restrict__ ell_off,
                                                                   const int32_t* __restrict__ ell_col,
                                                                   const double* __restrict__ ell_val,
                                                                   const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;
    // a block covers RB rows with RB / RPT threads: thread t holds rows
    // t, t + RB / RPT, ... of the block, so every source load feeds RPT rows
    static_assert(256 % RB == 0 && SU % GROUP == 0, "row blocks within the 256-row ELL blocks");
    constexpr int BT = RB / RPT;
    const int tid = threadIdx.x;
    const int base = blockIdx.x * RB;
    const int wave_row0 = uniform(base + (tid & ~63));
    double px_[RPT], py_[RPT], pz_[RPT], pw_[RPT];
    double acc[RPT][NC];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const double4 pi = xyzc[base + tid + r * BT];
        px_[r] = -2.0 * pi.x;
        py_[r] = -2.0 * pi.y;
        pz_[r] = -2.0 * pi.z;
        pw_[r] = pi.w;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = 0.0;
    }
    const int nunit = np / SU;
    for (int ch = blockIdx.y; ch < nunit; ch += gridDim.y)
    for (int gq = ch * (SU / GROUP); gq < (ch + 1) * (SU / GROUP); ++gq) {
        const int j0 = uniform(gq * GROUP);
        bool self = false;
#pragma unroll
        for (int r = 0; r < RPT; ++r) self = self || (j0 + GROUP > wave_row0 + r * BT && j0 < wave_row0 + r * BT + 64);
        if (!self) {
            // eight pairs per iteration: the next iteration's scalar loads are
            // in flight under this one's arithmetic (2: +15 %, 4: +4 % time)
#pragma unroll 8
            for (int jj = 0; jj < GROUP; ++jj) {
                const double4 pj = xyzc[j0 + jj];
                double xj[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) xj[c] = X[(size_t)(j0 + jj) * NC + c];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const double t = rsqrt_pos_x2(fma(px_[r], pj.x, fma(py_[r], pj.y, fma(pz_[r], pj.z, pw_[r]))) + pj.w);
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[r][c] = fma(t, xj[c], acc[r][c]);
                }
            }
        } else {
#pragma unroll 4
            for (int jj = 0; jj < GROUP; ++jj) {
                const double4 pj = xyzc[j0 + jj];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const double r2 = fma(px_[r], pj.x, fma(py_[r], pj.y, fma(pz_[r], pj.z, pw_[r]))) + pj.w;
                    const double t = (base + tid + r * BT == j0 + jj) ? 0.0 : rsqrt_pos_x2(r2);
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[r][c] = fma(t, X[(size_t)(j0 + jj) * NC + c], acc[r][c]);
                }
            }
        }
    }
    const int64_t e0 = ell_off[base / 256], e1 = ell_off[base / 256 + 1];
    double* out = part + (size_t)blockIdx.y * np * NC;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int lr = base % 256 + tid + r * BT;   // row within the 256-row ELL block
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] *= 0.5;
        for (int64_t e = e0 + (int64_t)blockIdx.y * 256 + lr; e < e1; e += (int64_t)gridDim.y * 256) {
            const double v = ell_val[e];
            const double* x = X + (size_t)ell_col[e] * NC;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[r][c] = fma(v, x[c], acc[r][c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) out[(size_t)(base + tid + r * BT) * NC + c] = acc[r][c];
    }
}

// Y[t] = sum over the splits of part[k][t], in four interleaved chains so that
// several loads of a thread are in flight (the launches have few waves).
__global__ void k_sum_splits(const double* __restrict__ part, double* __restrict__ Y, size_t len, int nsplit,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 4 <= nsplit; k += 4)
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] += part[(size_t)(k + q) * len + t];
    for (; k < nsplit; ++k) s[0] += part[(size_t)k * len + t];
    Y[t] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Near-field list of the omegaFQ T in FP64 over the real atoms: for every
// pair closer than r_far (erfc(x) < 2^-54 beyond), C_ij = -erfc(r/R_qq)/r,
// and C_ii = sqrt(2/pi)/R_q (the self term, Eq. tqq).  Pass 0 counts each
// row's entries per candidate subset (cntw[sub][i]); pass 1 fills the ELL
// layout: row block b (256 rows) holds width_b = (off[b+1] - off[b]) / 256
// slots, entry k of row i at off[b] + k * 256 + (i - 256 b), subset after
// subset (columns increasing within a subset), unused slots left as cleared
// (column 0, value 0).  One thread per row atom, 64 rows per (one-wave)
// workgroup x = blockIdx.x, the row block's candidate source groups shared out
// over gridDim.y subsets (px_neighbors.h).
template <int PASS>
__global__ __launch_bounds__(64) void k_near_rows(const double4* __restrict__ xyz, const float4* __restrict__ glo,
                                                  const float4* __restrict__ ghi, int64_t n, int64_t np,
                                                  double r_far, double inv_rqq, double t_self,
                                                  int32_t* __restrict__ cntw, const int64_t* __restrict__ off,
                                                  int32_t* __restrict__ col, double* __restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int sub = blockIdx.y, nsub = gridDim.y;
    const double4 pi = xyz[i];
    const bool row = i < n;
    const double rf2 = r_far * r_far;
    int count = 0;
    int64_t out = 0;
    if (PASS == 1 && row) {
        int64_t before = 0;
        for (int t = 0; t < sub; ++t) before += cntw[(size_t)t * np + i];
        out = off[i / 256] + (i % 256) + 256 * before;
    }
    nbr::for_near_atoms(xyz, n, glo, ghi, (float)(r_far * 1.0001 + 1e-3), (int64_t)blockIdx.x, sub, nsub,
                        [&](int64_t j, const double4& pj) {
        if (!row) return;
        const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        if (j != i && !(r2 < rf2)) return;
        if (PASS == 0) {
            ++count;
        } else {
            double v = t_self;
            if (j != i) {
                const double r = sqrt(r2);
                v = -erfc(r * inv_rqq) / r;
            }
            col[out] = (int32_t)j;
            val[out] = v;
            out += 256;
        }
    });
    if (PASS == 0 && row) cntw[(size_t)sub * np + i] = count;
}

// ELL slot counts: wid[b] = 256 * (the longest row of row block b), b < nb;
// with the exclusive scan of wid, off[b] is block b's first entry.
__global__ void k_near_widths(const int32_t* __restrict__ cnt, int64_t n, int64_t nb, int64_t* __restrict__ wid)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    int32_t w = 0;
    for (int64_t i = b * 256; i < (b + 1) * 256 && i < n; ++i) w = cnt[i] > w ? cnt[i] : w;
    wid[b] = 256 * (int64_t)w;
}

// Positions relative to the centre c, |p - c|^2 in w.
__global__ void k_centred(const double4* __restrict__ xyz, int64_t np, double cx, double cy, double cz,
                          double4* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const double4 p = xyz[i];
    const double x = p.x - cx, y = p.y - cy, z = p.z - cz;
    out[i] = make_double4(x, y, z, fma(x, x, fma(y, y, z * z)));
}

// ====================== grouped launches (many segments) ====================
// A stacked block holds several segments (structure x column block), each a
// contiguous range of rows starting at row_off; one launch covers every
// segment's tiles, listed as int4 {segment, row block, column block, split}.
struct GroupConst {
    const float4* xyz32;
    const double4* xyz64;
    const float4* glo;
    const float4* ghi;
    int64_t row_off;
    int np, model;
    float inv_rqq32, t_self32, rfar32;
    double inv_rqq64, t_self64;
    float rfar64;
    DipoleConstF d32;
    DipoleConstD d64;
};

__global__ __launch_bounds__(Q32_THREADS) void k_tapply_wfq_f32_grouped(const GroupConst* __restrict__ gc,
                                                                        const float* __restrict__ X,
                                                                        float* __restrict__ Y,
                                                                        float* __restrict__ partial, int ldx,
                                                                        SkGrid sk,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    sk_pieces(sk, blockIdx.x, [&](int t, int c0, int c1, int slot) {
        const int4 tl = sk.tiles[t];
        const GroupConst& c = gc[tl.x];
        float* out = slot < 0 ? Y + ((size_t)c.row_off + (size_t)tl.y * 256) * ldx + tl.z * Q32_COLS
                              : partial + (size_t)slot * SK_TILE_FLOATS;
        tapply_wfq_f32_body(tl.y, tl.z, c0, c1, c.xyz32, c.glo, c.ghi, X + (size_t)c.row_off * ldx, out,
                            slot < 0 ? ldx : Q32_COLS, ldx, c.inv_rqq32, c.t_self32, c.rfar32);
    });
}

// Sums the scratch slots of every tile that several workgroups share, in
// workgroup order, into Y.  Grid: 32 workgroups of 256 threads per tile, one
// float4 per thread.  gc / tiles null: the single-structure layout.
__global__ __launch_bounds__(256) void k_sk_fixup(const float* __restrict__ partial, float* __restrict__ Y, int ldx,
                                                  SkGrid sk, const GroupConst* __restrict__ gc,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int t = blockIdx.x >> 5;
    const int64_t p0 = sk_pre(sk, t);
    const int ct = sk.tiles ? sk.tiles[t].w : sk.C;
    const int blo = sk_block_of(sk, p0), bhi = sk_block_of(sk, p0 + ct - 1);
    if (blo == bhi) return;
    const int q = (blockIdx.x & 31) * 256 + threadIdx.x;   // float4 index in the tile
    const int row = q >> 5, col = (q & 31) * 4;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int b = blo; b <= bhi; ++b) {
        const int slot = (b == blo && sk_begin(sk, b) < p0) ? 2 * b + 1 : 2 * b;
        const float4 v = *reinterpret_cast<const float4*>(partial + (size_t)slot * SK_TILE_FLOATS + row * Q32_COLS + col);
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    size_t r0;
    int cb;
    if (sk.tiles) {
        const int4 tl = sk.tiles[t];
        r0 = (size_t)gc[tl.x].row_off + (size_t)tl.y * 256;
        cb = tl.z;
    } else {
        r0 = (size_t)(t % sk.RB) * 256;
        cb = t / sk.RB;
    }
    *reinterpret_cast<float4*>(Y + (r0 + row) * ldx + cb * Q32_COLS + col) = acc;
}

__global__ __launch_bounds__(256) void k_tapply_wfqfmu_f32_grouped(const GroupConst* __restrict__ gc,
                                                                   const int4* __restrict__ tiles,
                                                                   const float* __restrict__ X,
                                                                   float* __restrict__ Y, int ldx,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int4 t = tiles[blockIdx.x];
    const GroupConst& c = gc[t.x];
    tapply_wfqfmu_f32_body(t.y, t.z, 0, c.xyz32, c.glo, c.ghi, X + (size_t)c.row_off * ldx,
                           Y + (size_t)c.row_off * ldx, c.np, ldx, c.d32);
}

__global__ __launch_bounds__(256) void k_tapply_wfq_f64_grouped(const GroupConst* __restrict__ gc,
                                                                const int4* __restrict__ tiles,
                                                                const double* __restrict__ X, double* __restrict__ Y,
                                                                int ldx,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int4 t = tiles[blockIdx.x];
    const GroupConst& c = gc[t.x];
    tapply_wfq_f64_body(t.y, t.z, 0, c.xyz64, c.glo, c.ghi, X + (size_t)c.row_off * ldx, Y + (size_t)c.row_off * ldx,
                        c.np, ldx, c.inv_rqq64, c.t_self64, c.rfar64);
}

__global__ __launch_bounds__(256) void k_tapply_wfqfmu_f64_grouped(const GroupConst* __restrict__ gc,
                                                                   const int4* __restrict__ tiles,
                                                                   const double* __restrict__ X,
                                                                   double* __restrict__ Y, int ldx,
    const int32_t* __restrict__ stop)
{
    if (stop && *stop) return;   // every column of the block is done
    const int4 t = tiles[blockIdx.x];
    const GroupConst& c = gc[t.x];
    tapply_wfqfmu_f64_body(t.y, t.z, 0, c.xyz64, c.glo, c.ghi, X + (size_t)c.row_off * ldx,
                           Y + (size_t)c.row_off * ldx, c.np, ldx, c.d64);
}



DipoleConstD dipole_const_d(const Geometry& g)
{
    DipoleConstD k;
    double rqq = std::sqrt(2.0) * g.r_q;
    double rqm = std::sqrt(g.r_q * g.r_q + g.r_mu * g.r_mu);
    double rmm = std::sqrt(2.0) * g.r_mu;
    k.inv_rqq = 1.0 / rqq;
    k.inv_rqm = 1.0 / rqm;
    k.inv_rmm = 1.0 / rmm;
    k.gauss_pref = 2.0 * TWO_OVER_SQRTPI / (rmm * rmm * rmm);
    k.t_self = TWO_OVER_SQRTPI / rqq;
    double rmax = std::fmax(rqq, std::fmax(rqm, rmm));
    k.r_far2 = (float)((XFAR_D64 * rmax) * (XFAR_D64 * rmax));
    return k;
}

int device_cus()
{
    static const int ncu = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            return v;
        return 256;
    }();
    return ncu;
}

// Source splits of the narrow kernels: about 16 workgroups per CU (several
// rounds), which balances the rows' unequal near-field work better than one
// round of long workgroups (measured on the 20k-atom sphere).
int narrow_splits(const Geometry& g)
{
    const int ncu = device_cus();
    int rb = (int)(g.np / 256);
    int nchunk = (int)(g.np / NW_CHUNK);
    int want = (16 * ncu + rb - 1) / rb;
    if (want < 1) want = 1;
    if (want > nchunk) want = nchunk;
    int cps = (nchunk + want - 1) / want;
    return (nchunk + cps - 1) / cps;
}

// rows per thread of the point-charge kernel (2: +12 %, 4: +43 % time on the
// 20k-atom sphere: the extra registers cut the waves per SIMD from 8 to 3)
constexpr int kNarrowRpt = 1;
// rows per workgroup, source atoms per split unit and 256-row blocks x splits
// per CU aimed at by the point-charge kernel.  On the 20k-atom sphere (79
// splits of one unit each): 3 % less time than 40 splits of two units, while
// 64- or 128-row workgroups change nothing and 128-atom units (158 splits) or
// fewer splits cost 2-12 % (the split sum grows, resp. the last round of
// workgroups runs the CUs part empty).
constexpr int kQRows = 256;
constexpr int kQUnit = 256;
constexpr int kQWant = 32;

int narrow_q_splits(const Geometry& g)
{
    const int nunit = (int)(g.np / kQUnit);
    const int rb = (int)(g.np / 256);
    int want = (kQWant * device_cus() + rb - 1) / rb;
    want = std::max(1, std::min(want, nunit));
    const int ups = (nunit + want - 1) / want;
    return (nunit + ups - 1) / ups;
}

template <int NC, int MODEL>
void launch_narrow(const Geometry& g, const double* X, double* Y, hipStream_t st, double* scratch, const int32_t* stop,
                   hipEvent_t ev0, hipEvent_t ev1)
{
    int rb = (int)(g.np / 256);
    int nchunk = (int)(g.np / NW_CHUNK);
    int nsplit = narrow_splits(g);
    int cps = (nchunk + nsplit - 1) / nsplit;
    double rqq = std::sqrt(2.0) * g.r_q;
    DipoleConstD kc = dipole_const_d(g);
    float rf2 = MODEL ? kc.r_far2 : (float)((XFAR_Q64 * rqq) * (XFAR_Q64 * rqq));
    if (MODEL == 0 && g.near_off) {
        // point part on the fly, near-field correction from the stored list
        nsplit = narrow_q_splits(g);
        hipExtLaunchKernelGGL((k_tapply_f64_narrow_q<NC, kNarrowRpt, kQRows, kQUnit>),
                              dim3((unsigned)(g.np / kQRows), nsplit), dim3(kQRows / kNarrowRpt), 0, st,
                              ev0, nullptr, 0,
                              (const double4*)g.xyzc, X, scratch, (int)g.np, (const int64_t*)g.near_off,
                              (const int32_t*)g.near_col, (const double*)g.near_val, stop);
        const size_t len = (size_t)g.np * NC;
        hipExtLaunchKernelGGL(k_sum_splits, dim3((unsigned)((len + 63) / 64)), dim3(64), 0, st, nullptr, ev1, 0,
                              (const double*)scratch, Y, len, nsplit, stop);
        return;
    }
    hipExtLaunchKernelGGL((k_tapply_f64_narrow<NC, MODEL>), dim3(rb, nsplit), dim3(256), 0, st, ev0, nullptr, 0,
                          (const double4*)g.xyz64, (const float4*)g.glo, (const float4*)g.ghi, X, scratch, (int)g.np,
                          cps, 1.0 / rqq, TWO_OVER_SQRTPI / rqq, rf2, kc, stop);
    size_t len = (size_t)(MODEL ? 4 : 1) * g.np * NC;
    hipExtLaunchKernelGGL(k_sum_splits, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, nullptr, ev1, 0,
                          (const double*)scratch, Y, len, nsplit, stop);
}

// ---- dense T for the stored-T apply ---------------------------------------------
// T[u][v] over the padded unknowns u, v (row-major, ld = nup; component-major
// for the dipole model: u = a * np + i), the same formulas and far thresholds
// as the on-the-fly kernels of the precision; rows and columns of ghost atoms
// are zero.  One thread per element, 256 columns of one row per workgroup.
__global__ __launch_bounds__(256) void k_tdense_f32(const float4* __restrict__ xyz, int64_t n, int64_t np, int model,
                                                    float inv_rqq, float t_self, float r_far2, DipoleConstF kc,
                                                    float* __restrict__ T)
{
    const int64_t nup = model ? 4 * np : np;
    const int64_t v = (int64_t)blockIdx.y * 256 + threadIdx.x;
    const int64_t u = blockIdx.x;
    if (v >= nup) return;
    const int a = (int)(u / np), c = (int)(v / np);
    const int64_t i = u - a * np, j = v - c * np;
    float t = 0.0f;
    if (i < n && j < n) {
        const float4 pi = xyz[i], pj = xyz[j];
        const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (!model) {
            if (i == j) {
                t = t_self;
            } else {
                const float rinv = __builtin_amdgcn_rsqf(r2);
                t = r2 < r_far2 ? erf_as(r2 * rinv * inv_rqq) * rinv : rinv;
            }
        } else if (i == j) {
            t = (a == 0 && c == 0) ? kc.t_self : 0.0f;
        } else {
            float b[4][4];
            pair_block_f32(dx, dy, dz, r2 >= kc.r_far2, kc, b);
            t = b[a][c];
        }
    }
    T[u * nup + v] = t;
}

__global__ __launch_bounds__(256) void k_tdense_f64(const double4* __restrict__ xyz, int64_t n, int64_t np, int model,
                                                    double inv_rqq, double t_self, float r_far2, DipoleConstD kc,
                                                    double* __restrict__ T)
{
    const int64_t nup = model ? 4 * np : np;
    const int64_t v = (int64_t)blockIdx.y * 256 + threadIdx.x;
    const int64_t u = blockIdx.x;
    if (v >= nup) return;
    const int a = (int)(u / np), c = (int)(v / np);
    const int64_t i = u - a * np, j = v - c * np;
    double t = 0.0;
    if (i < n && j < n) {
        const double4 pi = xyz[i], pj = xyz[j];
        const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        if (!model) {
            if (i == j) {
                t = t_self;
            } else {
                const double rinv = rsqrt(r2);
                t = r2 < (double)r_far2 ? erf(r2 * rinv * inv_rqq) * rinv : rinv;
            }
        } else if (i == j) {
            t = (a == 0 && c == 0) ? kc.t_self : 0.0;
        } else {
            double b[4][4];
            pair_block_f64(dx, dy, dz, r2 >= (double)kc.r_far2, kc, b);
            t = b[a][c];
        }
    }
    T[u * nup + v] = t;
}

// Resident 512-thread FP32 workgroups: two per CU (LDS and registers allow
// two), counted once per device.
int sk_slots()
{
    // filled on first use per device; callers on several host threads store
    // the same value, so relaxed atomics suffice
    static std::atomic<int> slots[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int v = slots[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        v = 2 * cu;
        slots[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Workgroups of a stream-K launch over `total` iterations: every resident
// slot, but at least 8 source chunks (256 atoms) each.
int sk_workgroups(int64_t total) { return (int)std::max<int64_t>(1, std::min<int64_t>(sk_slots(), total / 8)); }

}  // namespace

hipError_t ensure_near_f64(Geometry& g, hipStream_t st)
{
    if (g.model != 0 || g.near_off || g.bem) return hipSuccess;
    const double rqq = std::sqrt(2.0) * g.r_q;
    const double r_far = XFAR_Q64 * rqq;
    const int64_t nb = g.np / 256;
    int32_t *cnt = nullptr, *cntw = nullptr;
    int64_t* wid = nullptr;
    const int nsub = neighbor_subsets(g.np);
    int64_t nnz = 0;
    hipError_t e;
#define PXCHK(x) do { e = (x); if (e != hipSuccess) goto fail; } while (0)
    PXCHK(px::dev_malloc((void**)&cnt, sizeof(int32_t) * g.np));
    PXCHK(px::dev_malloc((void**)&cntw, sizeof(int32_t) * (size_t)nsub * g.np));
    PXCHK(px::dev_malloc((void**)&wid, sizeof(int64_t) * nb));
    PXCHK(px::dev_malloc((void**)&g.near_off, sizeof(int64_t) * (nb + 1)));
    PXCHK(px::dev_malloc((void**)&g.xyzc, sizeof(double4) * g.np));
    hipLaunchKernelGGL(k_centred, dim3((unsigned)((g.np + 255) / 256)), dim3(256), 0, st, g.xyz64, g.np, g.cx, g.cy,
                       g.cz, g.xyzc);
    hipLaunchKernelGGL(k_near_rows<0>, dim3((unsigned)(g.np / 64), (unsigned)nsub), dim3(64), 0, st, g.xyz64, g.glo,
                       g.ghi, g.n, g.np, r_far, 1.0 / rqq, TWO_OVER_SQRTPI / rqq, cntw, nullptr, nullptr, nullptr);
    count_sum(cntw, nsub, g.np, g.n, 0, cnt, st);
    hipLaunchKernelGGL(k_near_widths, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, cnt, g.n, nb, wid);
    PXCHK(hipGetLastError());
    {
        // block offsets on the host (one value per 256 atoms)
        std::vector<int64_t> w((size_t)nb), o((size_t)nb + 1);
        PXCHK(hipMemcpyAsync(w.data(), wid, sizeof(int64_t) * nb, hipMemcpyDeviceToHost, st));
        PXCHK(hipStreamSynchronize(st));
        o[0] = 0;
        for (int64_t b = 0; b < nb; ++b) o[b + 1] = o[b] + w[b];
        nnz = o[nb];
        PXCHK(hipMemcpyAsync(g.near_off, o.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, st));
        g.near_nnz = nnz;
        PXCHK(px::dev_malloc((void**)&g.near_col, sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
        PXCHK(px::dev_malloc((void**)&g.near_val, sizeof(double) * std::max<int64_t>(nnz, 1)));
        fill_zero(g.near_col, sizeof(int32_t) * std::max<int64_t>(nnz, 1), st);
        fill_zero(g.near_val, sizeof(double) * std::max<int64_t>(nnz, 1), st);
        hipLaunchKernelGGL(k_near_rows<1>, dim3((unsigned)(g.np / 64), (unsigned)nsub), dim3(64), 0, st, g.xyz64,
                           g.glo, g.ghi, g.n, g.np, r_far, 1.0 / rqq, TWO_OVER_SQRTPI / rqq, cntw, g.near_off,
                           g.near_col, g.near_val);
        PXCHK(hipStreamSynchronize(st));
        PXCHK(hipGetLastError());
    }
    px::dev_free(cnt);
    px::dev_free(cntw);
    px::dev_free(wid);
    return hipSuccess;
fail:
#undef PXCHK
    px::dev_free(cnt);
    px::dev_free(cntw);
    px::dev_free(wid);
    px::dev_free(g.near_off);
    px::dev_free(g.near_col);
    px::dev_free(g.near_val);
    px::dev_free(g.xyzc);
    g.near_off = nullptr;
    g.near_col = nullptr;
    g.near_val = nullptr;
    g.xyzc = nullptr;
    g.near_nnz = 0;
    return e;
}


size_t tapply_f32_scratch_bytes(const Geometry& g, int ncols)
{
    (void)ncols;
    if (g.model != 0) return 0;
    return (size_t)2 * sk_slots() * SK_TILE_FLOATS * sizeof(float);
}

void tapply_f32(const Geometry& g, const float* X, float* Y, int ldx, int ncols, hipStream_t st, float* scratch, const int32_t* stop)
{
    if (g.model == 0) {
        double rqq = std::sqrt(2.0) * g.r_q;
        float rf = (float)(XFAR_Q32 * rqq);
        SkGrid sk{};
        sk.RB = (int)(g.np / 256);
        sk.C = (int)(g.np / Q32_JC);
        sk.T = sk.RB * (ncols / Q32_COLS);
        sk.total = (int64_t)sk.T * sk.C;
        sk.G = sk_workgroups(sk.total);
        hipLaunchKernelGGL(k_tapply_wfq_f32, dim3((unsigned)sk.G), dim3(Q32_THREADS), 0, st, g.xyz32, g.glo, g.ghi, X,
                           Y, scratch, ldx, sk, (float)(1.0 / rqq), (float)(TWO_OVER_SQRTPI / rqq), rf * rf, stop);
        hipLaunchKernelGGL(k_sk_fixup, dim3((unsigned)(32 * sk.T)), dim3(256), 0, st, scratch, Y, ldx, sk,
                           (const GroupConst*)nullptr, stop);
    } else {
        DipoleConstD d = dipole_const_d(g);
        DipoleConstF k;
        k.inv_rqq = (float)d.inv_rqq;
        k.inv_rqm = (float)d.inv_rqm;
        k.inv_rmm = (float)d.inv_rmm;
        k.gauss_pref = (float)d.gauss_pref;
        k.t_self = (float)d.t_self;
        double rmax = 1.0 / std::fmin(d.inv_rqq, std::fmin(d.inv_rqm, d.inv_rmm));
        k.r_far2 = (float)((XFAR_D32 * rmax) * (XFAR_D32 * rmax));
        hipLaunchKernelGGL(k_tapply_wfqfmu_f32, dim3((unsigned)(g.np / 128), (unsigned)(ncols / D32_COLS)),
                           dim3(256), 0, st, g.xyz32, g.glo, g.ghi, X, Y, (int)g.np, ldx, k, stop);
    }
}

size_t tapply_f64_scratch_bytes(const Geometry& g, int ncols)
{
    if (g.bem) return bem_scratch_bytes(g, ncols);
    if (ncols > 8) return 0;
    const int ns = g.model ? narrow_splits(g) : std::max(narrow_splits(g), narrow_q_splits(g));
    return (size_t)ns * (g.model ? 4 : 1) * g.np * ncols * sizeof(double);
}

void tapply_f64(const Geometry& g, const double* X, double* Y, int ldx, int ncols, hipStream_t st,
                double* scratch, size_t scratch_bytes, const int32_t* stop, const hipEvent_t* ev, int active)
{
    if (active <= 0 || active > ncols) active = ncols;
    (void)scratch_bytes;
    if (g.bem) {
        bem_apply_f64(g, X, Y, ldx, ncols, st, scratch, stop, ev);
        return;
    }
    hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
    if (ncols <= 8) {
        // narrow layout: ldx == ncols
        if (g.model == 0) {
            switch (ncols) {
            case 1: launch_narrow<1, 0>(g, X, Y, st, scratch, stop, e0, e1); break;
            case 2: launch_narrow<2, 0>(g, X, Y, st, scratch, stop, e0, e1); break;
            case 3: launch_narrow<3, 0>(g, X, Y, st, scratch, stop, e0, e1); break;
            case 4: launch_narrow<4, 0>(g, X, Y, st, scratch, stop, e0, e1); break;
            case 6: launch_narrow<6, 0>(g, X, Y, st, scratch, stop, e0, e1); break;
            default: launch_narrow<8, 0>(g, X, Y, st, scratch, stop, e0, e1); break;
            }
        } else {
            switch (ncols) {
            case 2: launch_narrow<2, 1>(g, X, Y, st, scratch, stop, e0, e1); break;
            case 4: launch_narrow<4, 1>(g, X, Y, st, scratch, stop, e0, e1); break;
            case 6: launch_narrow<6, 1>(g, X, Y, st, scratch, stop, e0, e1); break;
            default: launch_narrow<8, 1>(g, X, Y, st, scratch, stop, e0, e1); break;
            }
        }
        return;
    }
    if (g.model == 0) {
        double rqq = std::sqrt(2.0) * g.r_q;
        float rf = (float)(XFAR_Q64 * rqq);
        hipExtLaunchKernelGGL(k_tapply_wfq_f64, dim3((unsigned)(g.np / 128), (unsigned)((active + Q64_COLS - 1) / Q64_COLS)), dim3(256),
                              0, st, e0, e1, 0, (const double4*)g.xyz64, (const float4*)g.glo, (const float4*)g.ghi, X,
                              Y, (int)g.np, ldx, 1.0 / rqq, TWO_OVER_SQRTPI / rqq, rf * rf, stop);
    } else {
        DipoleConstD k = dipole_const_d(g);
        hipExtLaunchKernelGGL(k_tapply_wfqfmu_f64, dim3((unsigned)(g.np / 64), (unsigned)((active + D64_COLS - 1) / D64_COLS)),
                              dim3(256), 0, st, e0, e1, 0, (const double4*)g.xyz64, (const float4*)g.glo,
                              (const float4*)g.ghi, X, Y, (int)g.np, ldx, k, stop);
    }
}

// ---- grouped launches -------------------------------------------------------

struct GroupedTApply::Impl {
    GroupConst* d_gc = nullptr;
    int4* d_t32q = nullptr;   // FP32 omegaFQ tiles
    int4* d_t32d = nullptr;   // FP32 dipole tiles
    int4* d_t64q = nullptr;
    int4* d_t64d = nullptr;
    int64_t* d_pre32q = nullptr;   // stream-K iteration offsets of the FP32 omegaFQ tiles
    int n32q = 0, n32d = 0, n64q = 0, n64d = 0;
    SkGrid sk{};
    int64_t rows = 0;
    int ldx = 0;
    void release()
    {
        void* ps[] = {d_gc, d_t32q, d_t32d, d_t64q, d_t64d, d_pre32q};
        for (void* p : ps)
            if (p) px::dev_free(p);
        d_gc = nullptr;
        d_t32q = d_t32d = d_t64q = d_t64d = nullptr;
        d_pre32q = nullptr;
    }
};

GroupedTApply::GroupedTApply() : impl(new Impl) {}
GroupedTApply::~GroupedTApply()
{
    impl->release();
    delete impl;
}

static hipError_t upload(void** dst, const void* src, size_t bytes, hipStream_t st)
{
    hipError_t e = px::dev_malloc(dst, bytes > 0 ? bytes : 16);
    if (e != hipSuccess) return e;
    if (bytes > 0) e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, st);
    return e;
}

hipError_t GroupedTApply::setup(const std::vector<GroupSeg>& segs, int ldx, int64_t rows, hipStream_t st)
{
    impl->release();
    impl->rows = rows;
    impl->ldx = ldx;
    std::vector<GroupConst> gc(segs.size());
    std::vector<int4> t32q, t32d, t64q, t64d;
    std::vector<int64_t> pre32q(1, 0);
    for (size_t k = 0; k < segs.size(); ++k) {
        const Geometry& g = *segs[k].g;
        GroupConst c{};
        c.xyz32 = g.xyz32;
        c.xyz64 = g.xyz64;
        c.glo = g.glo;
        c.ghi = g.ghi;
        c.row_off = segs[k].row_off;
        c.np = (int)g.np;
        c.model = g.model;
        const double rqq = std::sqrt(2.0) * g.r_q;
        c.inv_rqq32 = (float)(1.0 / rqq);
        c.t_self32 = (float)(TWO_OVER_SQRTPI / rqq);
        c.rfar32 = (float)((XFAR_Q32 * rqq) * (XFAR_Q32 * rqq));
        c.inv_rqq64 = 1.0 / rqq;
        c.t_self64 = TWO_OVER_SQRTPI / rqq;
        c.rfar64 = (float)((XFAR_Q64 * rqq) * (XFAR_Q64 * rqq));
        const int nchunk = (int)(g.np / Q32_JC);
        if (g.model == 1) {
            c.d64 = dipole_const_d(g);
            c.d32.inv_rqq = (float)c.d64.inv_rqq;
            c.d32.inv_rqm = (float)c.d64.inv_rqm;
            c.d32.inv_rmm = (float)c.d64.inv_rmm;
            c.d32.gauss_pref = (float)c.d64.gauss_pref;
            c.d32.t_self = (float)c.d64.t_self;
            const double rmax = 1.0 / std::fmin(c.d64.inv_rqq, std::fmin(c.d64.inv_rqm, c.d64.inv_rmm));
            c.d32.r_far2 = (float)((XFAR_D32 * rmax) * (XFAR_D32 * rmax));
        }
        gc[k] = c;
        const int kk = (int)k;
        if (g.model == 0) {
            for (int cb = 0; cb < ldx / Q32_COLS; ++cb)
                for (int rb = 0; rb < (int)(g.np / 256); ++rb) {
                    t32q.push_back(make_int4(kk, rb, cb, nchunk));
                    pre32q.push_back(pre32q.back() + nchunk);
                }
            for (int cb = 0; cb < ldx / Q64_COLS; ++cb)
                for (int rb = 0; rb < (int)(g.np / 128); ++rb) t64q.push_back(make_int4(kk, rb, cb, 0));
        } else {
            for (int cb = 0; cb < ldx / D32_COLS; ++cb)
                for (int rb = 0; rb < (int)(g.np / 128); ++rb) t32d.push_back(make_int4(kk, rb, cb, 0));
            for (int cb = 0; cb < ldx / D64_COLS; ++cb)
                for (int rb = 0; rb < (int)(g.np / 64); ++rb) t64d.push_back(make_int4(kk, rb, cb, 0));
        }
    }
    impl->n32q = (int)t32q.size();
    impl->n32d = (int)t32d.size();
    impl->n64q = (int)t64q.size();
    impl->n64d = (int)t64d.size();
    hipError_t e;
    if ((e = upload((void**)&impl->d_gc, gc.data(), sizeof(GroupConst) * gc.size(), st)) != hipSuccess) return e;
    if ((e = upload((void**)&impl->d_t32q, t32q.data(), sizeof(int4) * t32q.size(), st)) != hipSuccess) return e;
    if ((e = upload((void**)&impl->d_t32d, t32d.data(), sizeof(int4) * t32d.size(), st)) != hipSuccess) return e;
    if ((e = upload((void**)&impl->d_t64q, t64q.data(), sizeof(int4) * t64q.size(), st)) != hipSuccess) return e;
    if ((e = upload((void**)&impl->d_t64d, t64d.data(), sizeof(int4) * t64d.size(), st)) != hipSuccess) return e;
    if ((e = upload((void**)&impl->d_pre32q, pre32q.data(), sizeof(int64_t) * pre32q.size(), st)) != hipSuccess)
        return e;
    impl->sk.tiles = impl->d_t32q;
    impl->sk.pre = impl->d_pre32q;
    impl->sk.T = impl->n32q;
    impl->sk.total = pre32q.back();
    impl->sk.G = impl->sk.total > 0 ? sk_workgroups(impl->sk.total) : 0;
    return hipStreamSynchronize(st);
}

size_t GroupedTApply::partial_bytes() const
{
    return impl->n32q > 0 ? (size_t)2 * sk_slots() * SK_TILE_FLOATS * sizeof(float) : 0;
}

int64_t GroupedTApply::f32_tiles() const { return impl->n32q + impl->n32d; }

void GroupedTApply::run_f32(const float* X, float* Y, float* partial, hipStream_t st, const int32_t* stop) const
{
    if (impl->n32q > 0) {
        hipLaunchKernelGGL(k_tapply_wfq_f32_grouped, dim3((unsigned)impl->sk.G), dim3(Q32_THREADS), 0, st, impl->d_gc,
                           X, Y, partial, impl->ldx, impl->sk, stop);
        hipLaunchKernelGGL(k_sk_fixup, dim3((unsigned)(32 * impl->n32q)), dim3(256), 0, st, partial, Y, impl->ldx,
                           impl->sk, impl->d_gc, stop);
    }
    if (impl->n32d > 0)
        hipLaunchKernelGGL(k_tapply_wfqfmu_f32_grouped, dim3(impl->n32d), dim3(256), 0, st, impl->d_gc, impl->d_t32d,
                           X, Y, impl->ldx, stop);
}

void GroupedTApply::run_f64(const double* X, double* Y, hipStream_t st, const int32_t* stop) const
{
    if (impl->n64q > 0)
        hipLaunchKernelGGL(k_tapply_wfq_f64_grouped, dim3(impl->n64q), dim3(256), 0, st, impl->d_gc, impl->d_t64q, X, Y,
                           impl->ldx, stop);
    if (impl->n64d > 0)
        hipLaunchKernelGGL(k_tapply_wfqfmu_f64_grouped, dim3(impl->n64d), dim3(256), 0, st, impl->d_gc, impl->d_t64d,
                           X, Y, impl->ldx, stop);
}

size_t tstored_f32_scratch_bytes() { return (size_t)2 * sk_slots() * SK_TILE_FLOATS * sizeof(float); }

void tstored_f32(const Geometry& g, const float* T, const float* X, float* Y, int ldx, int ncols, hipStream_t st,
                 float* scratch, const int32_t* stop, const hipEvent_t* ev, int active)
{
    // column blocks of 128; the last one as a 64-column tile when its active
    // columns fit one (a second stream-K launch over that block alone)
    const int nb = ncols / Q32_COLS;
    if (active <= 0 || active > ncols) active = ncols;
    const int last = active - (nb - 1) * Q32_COLS;
    const bool half = nb >= 1 && last > 0 && last <= Q32_COLS / 2;
    const int nfull = half ? nb - 1 : nb;
    hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
    auto launch = [&](int nblk, bool halftile, const float* Xb, float* Yb, hipEvent_t a, hipEvent_t b) {
        SkGrid sk{};
        sk.RB = (int)(g.nup / 256);
        sk.C = (int)(g.nup / Q32_JC);
        sk.T = sk.RB * nblk;
        sk.total = (int64_t)sk.T * sk.C;
        sk.G = sk_workgroups(sk.total);
        if (halftile)
            hipExtLaunchKernelGGL(k_tstored_f32<2>, dim3((unsigned)sk.G), dim3(Q32_THREADS), 0, st, a, nullptr, 0, T,
                                  (int)g.nup, Xb, Yb, scratch, ldx, sk, stop);
        else
            hipExtLaunchKernelGGL(k_tstored_f32<4>, dim3((unsigned)sk.G), dim3(Q32_THREADS), 0, st, a, nullptr, 0, T,
                                  (int)g.nup, Xb, Yb, scratch, ldx, sk, stop);
        hipExtLaunchKernelGGL(k_sk_fixup, dim3((unsigned)(32 * sk.T)), dim3(256), 0, st, nullptr, b, 0, scratch, Yb,
                              ldx, sk, (const GroupConst*)nullptr, stop);
    };
    if (nfull > 0) launch(nfull, false, X, Y, e0, half ? nullptr : e1);
    if (half)
        launch(1, true, X + (size_t)nfull * Q32_COLS, Y + (size_t)nfull * Q32_COLS, nfull > 0 ? nullptr : e0, e1);
}

void tstored_f64(const Geometry& g, const double* T, const double* X, double* Y, int ldx, int ncols, hipStream_t st,
                 double* scratch, const int32_t* stop, const hipEvent_t* ev, int active)
{
    if (active <= 0 || active > ncols) active = ncols;
    hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
    const int nup = (int)g.nup;
    if (ncols <= 8) {
        // narrow layout (ldx == ncols): split over the source rows, then the split sum
        const int nsplit = narrow_splits(g);
        const int per = (nup + nsplit - 1) / nsplit;
        const dim3 grid((unsigned)(nup / 256), (unsigned)nsplit);
#define PX_TSN(NC)                                                                                                   \
    hipExtLaunchKernelGGL(k_tstored_narrow<NC>, grid, dim3(256), 0, st, e0, nullptr, 0, T, nup, X, scratch, nup, per, stop)
        switch (ncols) {
        case 1: PX_TSN(1); break;
        case 2: PX_TSN(2); break;
        case 3: PX_TSN(3); break;
        case 4: PX_TSN(4); break;
        case 6: PX_TSN(6); break;
        default: PX_TSN(8); break;
        }
#undef PX_TSN
        const int nc = ncols <= 4 || ncols == 6 ? ncols : 8;
        const size_t len = (size_t)nup * nc;
        hipExtLaunchKernelGGL(k_sum_splits, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, nullptr, e1, 0,
                              (const double*)scratch, Y, len, nsplit, stop);
        return;
    }
    hipExtLaunchKernelGGL(k_tstored_f64, dim3((unsigned)(nup / 128), (unsigned)((active + Q64_COLS - 1) / Q64_COLS)), dim3(256), 0, st,
                          e0, e1, 0, T, nup, X, Y, nup, ldx, stop);
}

void tdense_f32(const Geometry& g, float* T, hipStream_t st)
{
    const double rqq = std::sqrt(2.0) * g.r_q;
    const float rf = (float)(XFAR_Q32 * rqq);
    DipoleConstF k{};
    if (g.model == 1) {
        const DipoleConstD d = dipole_const_d(g);
        k.inv_rqq = (float)d.inv_rqq;
        k.inv_rqm = (float)d.inv_rqm;
        k.inv_rmm = (float)d.inv_rmm;
        k.gauss_pref = (float)d.gauss_pref;
        k.t_self = (float)d.t_self;
        const double rmax = 1.0 / std::fmin(d.inv_rqq, std::fmin(d.inv_rqm, d.inv_rmm));
        k.r_far2 = (float)((XFAR_D32 * rmax) * (XFAR_D32 * rmax));
    }
    hipLaunchKernelGGL(k_tdense_f32, dim3((unsigned)g.nup, (unsigned)((g.nup + 255) / 256)), dim3(256), 0, st, g.xyz32,
                       g.n, g.np, g.model, (float)(1.0 / rqq), (float)(TWO_OVER_SQRTPI / rqq), rf * rf, k, T);
}

void tdense_f64(const Geometry& g, double* T, hipStream_t st)
{
    const double rqq = std::sqrt(2.0) * g.r_q;
    const float rf = (float)(XFAR_Q64 * rqq);
    const DipoleConstD k = dipole_const_d(g);
    hipLaunchKernelGGL(k_tdense_f64, dim3((unsigned)g.nup, (unsigned)((g.nup + 255) / 256)), dim3(256), 0, st, g.xyz64,
                       g.n, g.np, g.model, 1.0 / rqq, TWO_OVER_SQRTPI / rqq, rf * rf, k, T);
}

}  // namespace px
