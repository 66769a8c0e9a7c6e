// C ABI entry points and the blocked GMRES driver with FP64 iterative
// refinement (plasmonX paper, Section 6: the "iterative on the fly" solver of
// Eq. matrix-compact, here for all frequency/polarization columns at once).
//
// One restart cycle = m Arnoldi steps.  Each cycle starts from the true
// residual r = b - A x recomputed in FP64 (FP64 T-apply + FP64 sparse apply),
// so with PX_MIXED the cycle is the inner solve of an iterative-refinement
// step whose T-apply runs in FP32 on MFMA, while orthogonalisation (CGS2),
// the Givens least-squares update and the solution update stay in FP64.
// Columns whose true relative residual reached rel_tol are retired at the next
// cycle boundary and the active block is compacted, so the T-apply width
// follows the number of unfinished columns.
#include "px_internal.h"
#include "px_state.h"
#include "px_engine.h"

#include <condition_variable>
#include <memory>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace pxs;

namespace {

thread_local std::string g_err;

int pad_cols(int na, bool narrow_ok) { return (narrow_ok && na <= 4) ? na : ((na + px::COL_PAD - 1) / px::COL_PAD) * px::COL_PAD; }

// An IEFPCM column's charges from its potentials: conjugate gradients on
// S A^-1 to this relative residual.
constexpr double kChargeSolveTol = 1e-12;
constexpr int kChargeSolveMaxIter = 20000;

}  // namespace

namespace pxs {

pxStatus fail(pxStatus st, const std::string& msg)
{
    g_err = msg;
    return st;
}

void shift_q(double drude, double tau, double w, double& zr, double& zi)
{
    const double pref = -w / (2.0 * drude * tau);
    zr = pref * w * tau;
    zi = pref;
}

void shift_mu(double ar, double ai, double& zr, double& zi)
{
    const double den = ar * ar + ai * ai;
    zr = -ar / den;
    zi = ai / den;
}

void shift_bem(double e2r, double e2i, double e1r, double e1i, double& zr, double& zi)
{
    const double nr = e2r + e1r, ni = e2i + e1i, dr = e2r - e1r, di = e2i - e1i;
    const double den = dr * dr + di * di;
    zr = 2.0 * PI * (nr * dr + ni * di) / den;
    zi = 2.0 * PI * (ni * dr - nr * di) / den;
}

// The shift z of a BEM structure's operator M - z I (DPCM, Eq. bem-dpcm) or
// F - z I (IEFPCM, Eq. bem-iefpcm: z = -2 pi (eps2 + eps1) / (eps2 - eps1))
// for the metal permittivity e2 (interleaved complex).
void shift_bem_of(const pxStructure_t* s, const double* e2, double& zr, double& zi)
{
    shift_bem(e2[0], e2[1], s->eps1[0], s->eps1[1], zr, zi);
    if (s->g.bem_ief) {
        zr = -zr;
        zi = -zi;
    }
}

// The charge-row shift of frequency w: z_q(w) of Eq. (z_q_wfq), or for a BEM
// structure the shift above with the metal permittivity eps2(w) given with
// the frequencies.
void shift_of(const pxStructure_t* s, int w, double& zr, double& zi)
{
    if (s->model == PX_BEM) shift_bem_of(s, &s->aib[2 * w], zr, zi);
    else shift_q(s->drude, s->mat.tau, s->omega_au[w], zr, zi);
}

void het_factors(const pxStructure_t* s, double w, const double* aib4, double2 out[6])
{
    const double dr[2] = {s->drude, s->drude_b};
    const double tau[2] = {s->mat.tau, s->mat_b.tau};
    for (int t = 0; t < 2; ++t) {
        const int o = 1 - t;
        double zr, zi;
        shift_q(dr[t], tau[t], w, zr, zi);
        out[t] = make_double2(zr, zi);
        // rho_t phi_t = (n_o tau_o / n_t tau_t) (1 - i w tau_t) / (1 - i w tau_o)
        const double rho = dr[o] * tau[o] / (dr[t] * tau[t]);
        const double ai = -w * tau[t], bi = -w * tau[o];
        const double den = 1.0 + bi * bi;
        const double fr = (1.0 + ai * bi) / den, fi = (ai - bi) / den;
        out[2 + t] = make_double2(0.5 * (1.0 + rho * fr), 0.5 * rho * fi);
        out[4 + t] = make_double2(0.0, 0.0);
        if (aib4) {
            const double ar = aib4[2 * t], aim = aib4[2 * t + 1];
            const double d = ar * ar + aim * aim;
            out[4 + t] = make_double2(ar / d, -aim / d);
        }
    }
}

void prepare_solve(pxStructure_t* s)
{
    const int ncol = s->ncol;
    const int64_t nup = s->g.nup;
    double2* d_gam = nullptr;
    if (s->het) {
        // gamma_A, gamma_B of every column's frequency
        std::vector<double2> gam((size_t)2 * s->ldg, make_double2(0.0, 0.0));
        for (int c = 0; c < ncol; ++c) {
            double2 f[6];
            het_factors(s, s->omega_au[c / s->npol], nullptr, f);
            gam[c] = f[2];
            gam[s->ldg + c] = f[3];
        }
        d_gam = dalloc<double2>((size_t)2 * s->ldg);
        HC(hipMemcpyAsync(d_gam, gam.data(), sizeof(double2) * 2 * s->ldg, hipMemcpyHostToDevice, s->st));
        px::build_rhs_het(s->g, s->d_col_pol, d_gam, s->e0, s->b, ncol, s->ldg, SOLVER_MU_SIGN, s->st);
    } else if (s->model == PX_BEM) {
        px::bem_rhs(s->g, s->d_col_pol, s->e0, s->b, ncol, s->ldg, s->st);
    } else {
        px::build_rhs(s->g, s->d_col_pol, s->e0, s->b, ncol, s->ldg, SOLVER_MU_SIGN, s->st);
    }
    px::fill_zero(s->x, sizeof(double2) * (size_t)nup * s->ldg, s->st);
    s->bnorm.assign(ncol, 0.0);
    const int nchunk = px::arnoldi_chunks(nup);
    double* part = dalloc<double>((size_t)nchunk * s->ldg);
    double* nr = dalloc<double>(s->ldg);
    px::col_norm_partial(s->b, part, ncol, s->ldg, nup, s->st);
    px::reduce_norms(part, nchunk, nr, ncol, s->ldg, s->st);
    HC(hipMemcpyAsync(s->bnorm.data(), nr, sizeof(double) * ncol, hipMemcpyDeviceToHost, s->st));
    HC(hipStreamSynchronize(s->st));
    dfree(part);
    dfree(nr);
    dfree(d_gam);
    s->iters.assign(ncol, 0);
    s->cycles.assign(ncol, 0);
    s->stall.assign(ncol, 0);
    s->relres.assign(ncol, 0.0);
    s->solved = false;
}

void finish_solve(pxStructure_t* s)
{
    const int ncol = s->ncol;
    const int nchunk = (int)((s->g.n + px::RED_ROWS - 1) / px::RED_ROWS);
    double2* dpart = dalloc<double2>((size_t)nchunk * 3 * s->ldg);
    double2* d = dalloc<double2>((size_t)3 * ncol);
    double2* al = dalloc<double2>((size_t)9 * s->n_omega);
    double* sg = dalloc<double>(s->n_omega);
    px::observables(s->g, s->x, ncol, s->ldg, dpart, d, s->st);
    px::spectrum(d, s->d_col_pol, s->n_omega, s->npol, s->d_omega, s->e0, al, sg, s->st);
    s->alpha.assign((size_t)18 * s->n_omega, 0.0);
    s->sigma.assign(s->n_omega, 0.0);
    HC(hipMemcpyAsync(s->alpha.data(), al, sizeof(double2) * 9 * s->n_omega, hipMemcpyDeviceToHost, s->st));
    HC(hipMemcpyAsync(s->sigma.data(), sg, sizeof(double) * s->n_omega, hipMemcpyDeviceToHost, s->st));
    HC(hipStreamSynchronize(s->st));
    dfree(dpart);
    dfree(d);
    dfree(al);
    dfree(sg);
    s->solved = true;
}

}  // namespace pxs

namespace {

// The active block's vectors and the T-apply scratch: everything a true
// residual and an operator apply need (lda columns).
void ensure_vectors(pxStructure_t* s, int lda)
{
    Workspace& W = s->ws;
    const int64_t nup = s->g.nup;
    if (W.lda_cap >= lda && W.nup == nup) return;
    W.release();
    const size_t vec = (size_t)nup * lda;
    const int nchunk = px::arnoldi_chunks(nup);
    W.w = dalloc<double2>(vec);
    W.xs = dalloc<double2>(vec);
    W.rs = dalloc<double2>(vec);
    W.bs = dalloc<double2>(vec);
    W.tmp = dalloc<double2>(vec);
    W.X32 = dalloc<float>(2 * vec);
    W.Y32 = dalloc<float>(2 * vec);
    W.Y64 = dalloc<double>(2 * vec);
    W.npart = dalloc<double>((size_t)std::max(nchunk, px::update_chunks(nup)) * lda);
    W.nrm = dalloc<double>(lda);
    W.target = dalloc<double>(lda);
    W.done = dalloc<int32_t>(lda);
    W.steps = dalloc<int32_t>(lda);
    W.map = dalloc<int32_t>(lda);
    W.zq = dalloc<double2>(lda);
    W.zmu = dalloc<double2>(lda);
    W.het = dalloc<double2>((size_t)6 * lda);
    // (a BEM structure applies every column of the block in one call)
    W.narrow_bytes = px::tapply_f64_scratch_bytes(s->g, s->g.bem ? 2 * lda : 8);
    W.narrow = dalloc<double>(W.narrow_bytes / sizeof(double) + 1);
    W.split32 = dalloc<float>(px::tapply_f32_scratch_bytes(s->g, 2 * lda) / sizeof(float) + 1);
    // the omegaFQ narrow FP64 T-apply takes its near field from a stored list
    HC(px::ensure_near_f64(s->g, s->st));
    W.lda_cap = lda;
    W.m_cap = 0;
    W.nup = nup;
    px::fill_zero(W.X32, sizeof(float) * 2 * vec, s->st);
}

// The Krylov basis and the per-column Arnoldi state of restart length m, for
// the vectors' lda, allocated the first time a restart cycle needs them (a
// solve that the shared-Krylov phase finishes never does).
void ensure_basis(pxStructure_t* s, int m)
{
    Workspace& W = s->ws;
    if (W.m_cap >= m) return;
    const int64_t nup = s->g.nup;
    const int lda = W.lda_cap;
    const size_t vec = (size_t)nup * lda;
    const int nchunk = px::arnoldi_chunks(nup);
    void* old[] = {W.V, W.partial, W.h1, W.h2, W.R, W.H, W.G, W.coefQ, W.coefV, W.aux, W.sn, W.gv, W.y, W.cs};
    for (void* p : old) dfree(p);
    W.V = dalloc<double2>((size_t)(m + 1) * vec);
    W.partial = dalloc<double2>(std::max((size_t)nchunk * (m + 1), px::dot_partial_slabs(nup, m + 1)) * 2 * lda);
    W.h1 = dalloc<double2>((size_t)(m + 1) * lda);
    W.h2 = dalloc<double2>((size_t)(m + 1) * lda);
    W.R = dalloc<double2>((size_t)m * (m + 1) * lda);
    W.H = dalloc<double2>((size_t)m * (m + 1) * lda);
    W.G = dalloc<double2>((size_t)(m + 1) * 2 * lda);
    W.coefQ = dalloc<double2>((size_t)m * 2 * lda);
    W.coefV = dalloc<double2>((size_t)2 * lda);
    W.aux = dalloc<double2>((size_t)2 * lda);
    W.sn = dalloc<double2>((size_t)m * lda);
    W.gv = dalloc<double2>((size_t)(m + 1) * lda);
    W.y = dalloc<double2>((size_t)m * lda);
    W.cs = dalloc<double>((size_t)m * lda);
    W.m_cap = m;
    s->sync.ensure(m + 1);
    px::fill_zero(W.V, sizeof(double2) * (size_t)(m + 1) * vec, s->st);
}



// ---- T-apply method: on-the-fly kernels or the stored T with one GEMM --------
// The autotuner times both on the structure itself (after one warm-up launch
// each) the first time a (model, atoms, columns, precision) shape is applied
// and keeps the faster for the rest of the process.  The stored T costs
// nup^2 x 4 (FP32) or 8 (FP64) bytes and is only tried when that fits in a
// quarter of the free device memory.
enum { TA_FLY = 1, TA_STORED = 2 };
std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int, int>, int> g_tune;

bool stored_fits(pxStructure_t* s, bool f32)
{
    if ((f32 ? (void*)s->t32 : (void*)s->t64) != nullptr) return true;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
    const double bytes = (double)s->g.nup * (double)s->g.nup * (f32 ? 4.0 : 8.0);
    return bytes <= 0.25 * (double)fr;
}

void ensure_stored(pxStructure_t* s, bool f32)
{
    const size_t n2 = (size_t)s->g.nup * (size_t)s->g.nup;
    if (f32 && !s->t32) {
        s->t32 = static_cast<float*>(pxs::BlockCache::get().take(n2 * sizeof(float)));
        px::tdense_f32(s->g, s->t32, s->st);
    }
    if (f32 && !s->ws.sk32) s->ws.sk32 = dalloc<float>(px::tstored_f32_scratch_bytes() / sizeof(float));
    if (!f32 && !s->t64) {
        s->t64 = static_cast<double*>(pxs::BlockCache::get().take(n2 * sizeof(double)));
        px::tdense_f64(s->g, s->t64, s->st);
    }
}

// Y = T X on the stored T (hand-written kernels: FP32 or FP64 MFMA tiles, or
// a split pass over T for the narrow FP64 blocks).
// active (FP32): the real columns that hold data; 0 = all
void apply_stored(pxStructure_t* s, bool f32, const void* X, void* Y, int ldx, int ncols, const int32_t* stop = nullptr,
                  const hipEvent_t* ev = nullptr, int active = 0)
{
    Workspace& W = s->ws;
    if (f32)
        px::tstored_f32(s->g, s->t32, static_cast<const float*>(X), static_cast<float*>(Y), ldx, ncols, s->st, W.sk32,
                        stop, ev, active);
    else
        px::tstored_f64(s->g, s->t64, static_cast<const double*>(X), static_cast<double*>(Y), ldx, ncols, s->st,
                        W.narrow, stop, ev, active);
}

void apply_fly(pxStructure_t* s, bool f32, const void* X, void* Y, int ldx, int ncols, const int32_t* stop,
               const hipEvent_t* ev = nullptr, int active = 0)
{
    Workspace& W = s->ws;
    if (f32) {
        if (ev) HC(hipEventRecord(ev[0], s->st));
        px::tapply_f32(s->g, static_cast<const float*>(X), static_cast<float*>(Y), ldx, ncols, s->st, W.split32,
                       stop);
        if (ev) HC(hipEventRecord(ev[1], s->st));
    } else {
        px::tapply_f64(s->g, static_cast<const double*>(X), static_cast<double*>(Y), ldx, ncols, s->st, W.narrow,
                       W.narrow_bytes, stop, ev, active);
    }
}

float time_apply(pxStructure_t* s, bool f32, int method, const void* X, void* Y, int ldx, int ncols)
{
    hipEvent_t a, b;
    HC(hipEventCreate(&a));
    HC(hipEventCreate(&b));
    HC(hipEventRecord(a, s->st));
    if (method == TA_STORED) apply_stored(s, f32, X, Y, ldx, ncols);
    else apply_fly(s, f32, X, Y, ldx, ncols, nullptr);
    HC(hipEventRecord(b, s->st));
    HC(hipEventSynchronize(b));
    float ms = 0.f;
    HC(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

// The method for this shape: forced by the options, else the tuner's choice.
// The shared-Krylov phase stops a (frequency, polarization) pair once its
// GMRES residual estimate is below this fraction of rel_tol: the estimate
// agrees with the true FP64 residual recomputed afterwards to about four
// digits (20k-atom sphere: 9.000e-9 at 0.9), and a pair left above rel_tol
// goes on in the blocked solver.  (0.5 took 750 steps there against 731.)
constexpr double kPhaseTarget = 0.9;

// Above this many bytes the stored FP64 T is not tried for the narrow (1-8
// column) apply: that product streams T from HBM (8 N^2 bytes per apply)
// while the point-charge kernel is ALU-bound on the same N^2 pairs, about 3x
// faster (20k atoms: 570 against 182 us); only a T that stays in the
// last-level cache can compete.
constexpr double kNarrowStoredMaxBytes = 256.0 * (1 << 20);
// Largest dense T built to tune a single-use residual shape.
constexpr double kSingleUseTuneMaxBytes = 4.0 * (1 << 30);

// single_use: the apply is a true residual that the solve may need only once
// or twice (after the shared phase).  A dense T built for it then costs its
// generation and a device allocation (and its release) of 8 N_u^2 bytes per
// structure, more than the one apply saves unless the block cache already
// holds a block for it (a structure of the same size solved before).
int tapply_method(pxStructure_t* s, bool f32, const void* X, void* Y, int ldx, int ncols, const pxSolveOptions& o,
                  bool single_use = false)
{
    // the BEM operator is generated on the fly only (it is not symmetric)
    if (o.t_apply == PX_TAPPLY_ON_THE_FLY || s->g.bem) return TA_FLY;
    if (o.t_apply == PX_TAPPLY_STORED) {
        ensure_stored(s, f32);
        return TA_STORED;
    }
    const double t_bytes = (double)s->g.nup * (double)s->g.nup * (f32 ? 4.0 : 8.0);
    if (!f32 && ncols <= 8 && t_bytes > kNarrowStoredMaxBytes && !s->t64) return TA_FLY;
    if (single_use && !(f32 ? (void*)s->t32 : (void*)s->t64) &&
        !pxs::BlockCache::get().can_serve((size_t)t_bytes)) {
        // the T would need a new allocation: on the fly, except to tune a
        // new shape whose T is small enough (its block then serves the
        // structures of that size that follow)
        bool tuned;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tuned = g_tune.count(std::make_tuple((int)s->g.model, (int64_t)s->g.n, ncols, f32 ? 32 : 64)) > 0;
        }
        if (tuned || t_bytes > kSingleUseTuneMaxBytes) return TA_FLY;
    }
    const auto key = std::make_tuple((int)s->g.model, (int64_t)s->g.n, ncols, f32 ? 32 : 64);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            if (it->second == TA_STORED) {
                if (!stored_fits(s, f32)) return TA_FLY;
                ensure_stored(s, f32);
            }
            return it->second;
        }
    }
    if (!stored_fits(s, f32)) return TA_FLY;
    ensure_stored(s, f32);
    // one warm-up each, then three alternating rounds, the fastest launch of
    // each method (other streams, such as a batch's other solves, may share
    // the GPU during any one of them)
    (void)time_apply(s, f32, TA_FLY, X, Y, ldx, ncols);
    (void)time_apply(s, f32, TA_STORED, X, Y, ldx, ncols);
    float t_fly = 1e30f, t_st = 1e30f;
    for (int r = 0; r < 3; ++r) {
        t_fly = std::min(t_fly, time_apply(s, f32, TA_FLY, X, Y, ldx, ncols));
        t_st = std::min(t_st, time_apply(s, f32, TA_STORED, X, Y, ldx, ncols));
    }
    const int m = t_st < t_fly ? TA_STORED : TA_FLY;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = m;
    return m;
}

// ev (optional): start/stop events around the apply (carried by the launches
// of the on-the-fly FP64 kernels, recorded on the stream otherwise).
// active: the real columns that hold data (columns beyond are not read
// afterwards, so the stored FP32 product may skip them); 0 = all
void tapply(pxStructure_t* s, int method, bool f32, const void* X, void* Y, int ldx, int ncols, const int32_t* stop,
            const hipEvent_t* ev = nullptr, int active = 0)
{
    if (method == TA_STORED) {
        apply_stored(s, f32, X, Y, ldx, ncols, stop, ev, active);
    } else {
        apply_fly(s, f32, X, Y, ldx, ncols, stop, ev, active);
    }
}

// The sparse part of the operator on the active block, Y = T X given: the
// homogeneous Kbar apply with per-column shifts, or the two-type S(w) apply.
void sparse_apply(pxStructure_t* s, const void* Y, bool f32, int ldy, const double2* X, const double2* B,
                  double2* out, int na, int lda, double mu_sign, const int32_t* stop = nullptr)
{
    Workspace& W = s->ws;
    if (s->het) px::spmm_het(s->g, Y, f32, ldy, X, W.het, B, out, na, lda, mu_sign, s->st, stop);
    else px::spmm_shift(s->g, Y, f32, ldy, X, W.zq, W.zmu, B, out, na, lda, mu_sign, s->st, stop);
}

// r = b - A x for the active block (FP64 T-apply and FP64 sparse apply).
// single_use: the first residual of a solve (see tapply_method).
void residual(pxStructure_t* s, const double2* xs, const double2* bs, double2* rs, int na, int lda,
              const pxSolveOptions& o, bool single_use = false)
{
    Workspace& W = s->ws;
    const int method = tapply_method(s, false, xs, W.Y64, 2 * lda, 2 * lda, o, single_use);
    tapply(s, method, false, xs, W.Y64, 2 * lda, 2 * lda, nullptr, nullptr, 2 * na);
    s->tstats[method == TA_STORED ? 3 : 2] += 1;
    s->counts[3] += 1;
    s->counts[4] += 2 * lda;
    s->counts[5] += 2 * na;
    const double nu = (double)s->g.nu;
    s->work[1] += 2.0 * nu * nu * 2.0 * na;
    s->work[2] += 80.0 * nu * na;
    sparse_apply(s, W.Y64, false, 2 * lda, xs, bs, rs, na, lda, SOLVER_MU_SIGN);
}

void col_norms(pxStructure_t* s, const double2* v, int na, int lda, std::vector<double>& out)
{
    Workspace& W = s->ws;
    const int nchunk = px::arnoldi_chunks(s->g.nup);
    px::col_norm_partial(v, W.npart, na, lda, s->g.nup, s->st);
    px::reduce_norms(W.npart, nchunk, W.nrm, na, lda, s->st);
    out.resize(na);
    HC(hipMemcpyAsync(out.data(), W.nrm, sizeof(double) * na, hipMemcpyDeviceToHost, s->st));
    HC(hipStreamSynchronize(s->st));
}

void upload_shifts(pxStructure_t* s, const std::vector<int>& act, int lda)
{
    if (s->het) {
        std::vector<double2> h((size_t)6 * lda, make_double2(0, 0));
        for (size_t k = 0; k < act.size(); ++k) {
            const int w = act[k] / s->npol;
            double2 f[6];
            het_factors(s, s->omega_au[w], s->model == PX_WFQFMU ? &s->aib[4 * w] : nullptr, f);
            for (int q = 0; q < 6; ++q) h[(size_t)q * lda + k] = f[q];
        }
        HC(hipMemcpyAsync(s->ws.het, h.data(), sizeof(double2) * 6 * lda, hipMemcpyHostToDevice, s->st));
        return;
    }
    std::vector<double2> zq(lda, make_double2(0, 0)), zm(lda, make_double2(0, 0));
    for (size_t k = 0; k < act.size(); ++k) {
        const int c = act[k];
        const int w = c / s->npol;
        double zr, zi;
        shift_of(s, w, zr, zi);
        zq[k] = make_double2(zr, zi);
        if (s->model == PX_WFQFMU) {
            shift_mu(s->aib[2 * w], s->aib[2 * w + 1], zr, zi);
            zm[k] = make_double2(zr, zi);
        }
    }
    HC(hipMemcpyAsync(s->ws.zq, zq.data(), sizeof(double2) * lda, hipMemcpyHostToDevice, s->st));
    HC(hipMemcpyAsync(s->ws.zmu, zm.data(), sizeof(double2) * lda, hipMemcpyHostToDevice, s->st));
}

// Steps the host enqueues ahead of the last stop flag it looked at.
constexpr int kLag = 2;

// ---- blocked GMRES over a set of columns, advanced step by step -------------
// Solves the columns `act` (global indices) of a structure as one block: the
// true FP64 residual of every column, then a restart cycle of m Arnoldi steps,
// repeated until every column reached rel_tol (or gave up).  advance()
// enqueues work without waiting for the device wherever it can (the steps run
// ahead of the host and a device flag ends them), so one host thread can keep
// several solves busy on their own streams.
class BlockRun {
  public:
    BlockRun(pxStructure_t* s, std::vector<int> act, const pxSolveOptions& o)
        : s_(s), o_(o), act_(std::move(act)), tm_(o.timings != 0)
    {
        Workspace& W = s->ws;
        m_ = o.restart_m;
        m_max_ = std::max(o.restart_m, o.max_restart_m);
        mixed_ = o.precision == PX_MIXED;
        dcgs2_ = o.ortho == PX_ORTHO_DCGS2;
        na_ = (int)act_.size();
        lda_ = pad_cols(na_, true);
        const int64_t nup = s->g.nup;
        std::vector<int32_t> map(act_.begin(), act_.end());
        HC(hipMemcpyAsync(W.map, map.data(), sizeof(int32_t) * na_, hipMemcpyHostToDevice, s->st));
        px::gather_cols(s->x, s->ldg, W.xs, lda_, W.map, na_, nup, s->st);
        px::gather_cols(s->b, s->ldg, W.bs, lda_, W.map, na_, nup, s->st);
        upload_shifts(s, act_, lda_);
    }
    bool finished() const { return state_ == DONE; }
    // Enqueues at most max_steps Arnoldi steps (a residual pass counts as
    // one).  Without `wait` it returns instead of waiting for a step still on
    // the device.  Returns the work enqueued (0: it would have had to wait).
    int advance(int max_steps, bool wait)
    {
        int did = 0;
        while (state_ != DONE && did < max_steps) {
            if (state_ == RESIDUAL) {
                begin_cycle();
                ++did;
                continue;
            }
            bool blocked = false;
            did += steps(max_steps - did, wait, blocked);
            if (blocked) break;
        }
        return did;
    }

  private:
    enum State { RESIDUAL, STEPS, DONE };

    // True residual, retirement of finished columns, then the set-up of one
    // restart cycle (or DONE when no column is left).
    void begin_cycle()
    {
        pxStructure_t* s = s_;
        Workspace& W = s->ws;
        const int64_t nup = s->g.nup;
        residual(s, W.xs, W.bs, W.rs, na_, lda_, o_, first_residual_);
        first_residual_ = false;
        col_norms(s, W.rs, na_, lda_, beta_);
        std::vector<int> keep;
        bool slow = false;
        for (int k = 0; k < na_; ++k) {
            const int c = act_[k];
            const double prev = s->relres[c];
            s->relres[c] = s->bnorm[c] > 0.0 ? beta_[k] / s->bnorm[c] : 0.0;
            if (s->cycles[c] > 0 && s->relres[c] > 0.98 * prev) s->stall[c] += 1;
            else s->stall[c] = 0;
            if (s->relres[c] > o_.rel_tol && s->cycles[c] < o_.max_cycles &&
                (o_.stall_cycles == 0 || s->stall[c] < o_.stall_cycles)) {
                keep.push_back(k);
                if (s->cycles[c] > 0 && s->relres[c] > 0.7 * prev) slow = true;
            }
        }
        if (slow && m_ < m_max_) {
            // a longer Krylov space for every remaining column of the block
            m_ = std::min(2 * m_, m_max_);
            for (int k : keep) s->stall[act_[k]] = 0;
        }
        if (keep.empty()) {
            state_ = DONE;
            return;
        }
        if ((int)keep.size() < na_) {
            // retire finished columns: compact the slot layout
            const int na2 = (int)keep.size();
            const int lda2 = pad_cols(na2, true);
            std::vector<int32_t> smap(keep.begin(), keep.end());
            HC(hipMemcpyAsync(W.map, smap.data(), sizeof(int32_t) * na2, hipMemcpyHostToDevice, s->st));
            px::gather_cols(W.xs, lda_, W.tmp, lda2, W.map, na2, nup, s->st);
            std::swap(W.xs, W.tmp);
            px::gather_cols(W.rs, lda_, W.tmp, lda2, W.map, na2, nup, s->st);
            std::swap(W.rs, W.tmp);
            px::gather_cols(W.bs, lda_, W.tmp, lda2, W.map, na2, nup, s->st);
            std::swap(W.bs, W.tmp);
            std::vector<int> act2;
            std::vector<double> beta2;
            for (int k : keep) {
                act2.push_back(act_[k]);
                beta2.push_back(beta_[k]);
            }
            act_.swap(act2);
            beta_.swap(beta2);
            na_ = na2;
            lda_ = lda2;
            upload_shifts(s, act_, lda_);
        }
        // ---- set-up of one restart cycle
        ensure_basis(s, m_max_);
        const int m = m_;
        std::vector<double> tgt(lda_, 0.0);
        std::vector<double2> g0(lda_, make_double2(0, 0));
        for (int k = 0; k < na_; ++k) {
            const int c = act_[k];
            tgt[k] = std::max(0.5 * o_.rel_tol * s->bnorm[c], mixed_ ? beta_[k] * o_.inner_reduction : 0.0);
            g0[k] = make_double2(beta_[k], 0.0);
        }
        HC(hipMemcpyAsync(W.target, tgt.data(), sizeof(double) * lda_, hipMemcpyHostToDevice, s->st));
        px::fill_zero(W.gv, sizeof(double2) * (size_t)(m + 1) * lda_, s->st);
        HC(hipMemcpyAsync(W.gv, g0.data(), sizeof(double2) * lda_, hipMemcpyHostToDevice, s->st));
        px::fill_zero(W.done, sizeof(int32_t) * lda_, s->st);
        px::fill_zero(W.steps, sizeof(int32_t) * lda_, s->st);
        HC(hipMemcpyAsync(W.nrm, beta_.data(), sizeof(double) * na_, hipMemcpyHostToDevice, s->st));
        vstride_ = nup * lda_;
        px::normalize(W.rs, W.nrm, nullptr, W.V, mixed_ ? W.X32 : nullptr, na_, lda_, nup, s->st);
        // the BEM operator has an FP64 apply only
        wide32_ = mixed_ && lda_ > 4 && !s->g.bem;
        method_ = wide32_ ? tapply_method(s, true, W.X32, W.Y32, 2 * lda_, 2 * lda_, o_)
                          : tapply_method(s, false, W.V, W.Y64, 2 * lda_, 2 * lda_, o_);
        lag_ = kLag;
        // delayed orthogonalisation: the host enqueues steps ahead of the device and a
        // device flag, raised once the rotations have finished every column, ends them
        stop_ = dcgs2_ ? s->sync.flag() : nullptr;
        if (stop_) s->sync.reset(s->st);
        tm_.ensure(m);
        launched_ = 0;
        k_ = 0;
        done_h_.assign(na_, 0);
        state_ = STEPS;
    }

    // Steps of the current cycle; ends the cycle when its loop is over.
    int steps(int max_steps, bool wait, bool& blocked)
    {
        pxStructure_t* s = s_;
        Workspace& W = s->ws;
        const int64_t nup = s->g.nup;
        const int m = m_, na = na_, lda = lda_;
        const int nchunk = px::arnoldi_chunks(nup);
        int did = 0;
        while (did < max_steps) {
            const int k = k_;
            bool end = k >= m;
            if (!end && stop_ && k >= lag_) {
                if (!wait && !s->sync.ready(k - lag_)) {
                    blocked = true;
                    return did;
                }
                end = s->sync.stopped(k - lag_);
            }
            if (end) {
                end_cycle();
                return did;
            }
            double2* vk = W.V + k * vstride_;
            tm_.mark(k, 0, s->st);
            if (wide32_) tapply(s, method_, true, W.X32, W.Y32, 2 * lda, 2 * lda, stop_, nullptr, 2 * na);
            else tapply(s, method_, false, vk, W.Y64, 2 * lda, 2 * lda, stop_, nullptr, 2 * na);
            tm_.mark(k, 1, s->st);
            sparse_apply(s, wide32_ ? (const void*)W.Y32 : (const void*)W.Y64, wide32_, 2 * lda, vk, nullptr, W.w, na,
                         lda, SOLVER_MU_SIGN, stop_);
            tm_.mark(k, 2, s->st);
            if (dcgs2_) {
                // one dot pass and one update pass; column k-1 is finished here
                px::dots2(W.V, vstride_, k + 1, W.w, W.partial, na, lda, nup, s->st, stop_);
                px::reduce_dots2(W.partial, nup, k + 1, W.G, na, lda, s->st, nullptr, 1, stop_);
                px::dcgs2_coef(k, m, false, W.G, W.nrm, W.H, W.R, W.cs, W.sn, W.gv, W.target, W.done, W.steps, W.aux,
                               W.coefQ, W.coefV, na, lda, s->st, stop_);
                px::dcgs2_update(W.V, vstride_, k, W.coefQ, W.coefV, W.w, W.npart, na, lda, nup, s->st, nullptr, 0,
                                 stop_);
            } else {
                // CGS2 against v_0..v_k
                px::col_dots(W.V, vstride_, k + 1, W.w, W.partial, na, lda, nup, s->st);
                px::reduce_dots(W.partial, nchunk, k + 1, W.h1, na, lda, false, s->st);
                px::col_update(W.V, vstride_, k + 1, W.h1, W.w, nullptr, na, lda, nup, s->st);
                px::col_dots(W.V, vstride_, k + 1, W.w, W.partial, na, lda, nup, s->st);
                px::reduce_dots(W.partial, nchunk, k + 1, W.h2, na, lda, false, s->st);
                px::col_update(W.V, vstride_, k + 1, W.h2, W.w, W.npart, na, lda, nup, s->st);
            }
            px::reduce_norms(W.npart, px::update_chunks(nup), W.nrm, na, lda, s->st, stop_);
            if (!dcgs2_)
                px::givens_step(k, m, W.h1, W.h2, W.nrm, W.R, W.cs, W.sn, W.gv, W.target, W.done, W.steps, nullptr,
                                na, lda, s->st);
            px::normalize(W.w, W.nrm, W.done, W.V + (k + 1) * vstride_, mixed_ ? W.X32 : nullptr, na, lda, nup, s->st,
                          stop_);
            if (dcgs2_ && k == m - 1) {
                // the last basis vector's correction finishes column m-1
                px::dots2(W.V, vstride_, m + 1, W.V + m * vstride_, W.partial, na, lda, nup, s->st, stop_);
                px::reduce_dots2(W.partial, nup, m + 1, W.G, na, lda, s->st, nullptr, 1, stop_);
                px::dcgs2_coef(m, m, true, W.G, W.nrm, W.H, W.R, W.cs, W.sn, W.gv, W.target, W.done, W.steps, W.aux,
                               W.coefQ, W.coefV, na, lda, s->st, stop_);
            }
            tm_.mark(k, 3, s->st);
            ++launched_;
            ++k_;
            ++did;
            if (stop_) {
                s->sync.publish(k, s->st);
            } else {
                HC(hipMemcpyAsync(done_h_.data(), W.done, sizeof(int32_t) * na, hipMemcpyDeviceToHost, s->st));
                HC(hipStreamSynchronize(s->st));
                bool all = true;
                for (int q = 0; q < na; ++q) all = all && done_h_[q];
                if (all) {
                    end_cycle();
                    return did;
                }
            }
        }
        return did;
    }

    // Least squares, x update, statistics of the finished cycle.
    void end_cycle()
    {
        pxStructure_t* s = s_;
        Workspace& W = s->ws;
        const int64_t nup = s->g.nup;
        const int m = m_, na = na_, lda = lda_;
        px::lsq_solve(m, W.R, W.gv, W.steps, W.y, na, lda, s->st);
        px::x_update(W.V, vstride_, W.y, W.steps, m, W.xs, na, lda, nup, s->st);
        std::vector<int32_t> steps_h(na, 0);
        HC(hipMemcpyAsync(steps_h.data(), W.steps, sizeof(int32_t) * na, hipMemcpyDeviceToHost, s->st));
        HC(hipMemcpyAsync(W.map, act_.data(), sizeof(int32_t) * na, hipMemcpyHostToDevice, s->st));
        px::scatter_cols(W.xs, lda, s->x, s->ldg, W.map, na, nup, s->st);
        HC(hipStreamSynchronize(s->st));
        const bool stored = method_ == TA_STORED;
        {
            double t_ap = 0.0;
            tm_.collect(launched_, t_ap, s->ms[3], s->ms[4]);
            s->ms[wide32_ ? 1 : 2] += t_ap;
            s->tms[(wide32_ ? 0 : 2) + (stored ? 1 : 0)] += t_ap;
        }
        // accounting: column q took part in the matvecs of its first M_q steps (the delayed
        // variant learns that a column is done one step after its last useful matvec)
        const double nu = (double)s->g.nu;
        int executed = 0;
        int64_t colsum = 0;
        for (int q = 0; q < na; ++q) {
            const int mq = dcgs2_ ? std::min(steps_h[q] + 1, m) : steps_h[q];
            executed = std::max(executed, mq);
            colsum += mq;
            for (int k = 0; k < mq; ++k) s->work[2] += nu * (80.0 + 16.0 * (dcgs2_ ? 2.0 * k + 6.0 : 4.0 * k + 10.0));
            if (dcgs2_ && steps_h[q] == m) s->work[2] += nu * 16.0 * (m + 2);   // final correction pass
            s->iters[act_[q]] += steps_h[q];
            s->cycles[act_[q]] += 1;
            s->work[2] += 16.0 * nu * (steps_h[q] + 2);
        }
        s->tstats[(wide32_ ? 0 : 2) + (stored ? 1 : 0)] += executed;
        s->counts[wide32_ ? 0 : 3] += executed;
        s->counts[wide32_ ? 1 : 4] += (int64_t)executed * 2 * lda;
        s->counts[wide32_ ? 2 : 5] += 2 * colsum;
        s->work[wide32_ ? 0 : 1] += 2.0 * nu * nu * 2.0 * (double)colsum;
        s->tflop[(wide32_ ? 0 : 2) + (stored ? 1 : 0)] += 2.0 * nu * nu * 2.0 * (double)colsum;
        state_ = RESIDUAL;
    }

    pxStructure_t* s_;
    pxSolveOptions o_;
    std::vector<int> act_;
    StepTimer tm_;
    State state_ = RESIDUAL;
    int m_ = 0, m_max_ = 0, na_ = 0, lda_ = 0;
    bool mixed_ = false, dcgs2_ = false, wide32_ = false;
    bool first_residual_ = true;
    std::vector<double> beta_;
    std::vector<int32_t> done_h_;
    int64_t vstride_ = 0;
    int method_ = TA_FLY, lag_ = kLag, launched_ = 0, k_ = 0;
    int32_t* stop_ = nullptr;
};

// ---- shared-Krylov phase: every frequency of a one-material omegaFQ structure
// from one real Arnoldi process per polarization (px_shifted.hip) or one block
// Arnoldi process over the polarizations (px_shifted_block.hip) ----------------

// Device buffers that live for one call, from the block cache: given back to
// it once the call has marked them idle (its streams synchronised), else freed.
struct Scratch {
    std::vector<void*> ps;
    bool idle = false;
    template <typename T>
    T* get(size_t count)
    {
        T* p = static_cast<T*>(pxs::BlockCache::get().take(std::max<size_t>(count, 1) * sizeof(T)));
        ps.push_back(p);
        return p;
    }
    ~Scratch()
    {
        for (void* p : ps) {
            if (idle) pxs::BlockCache::get().give(p);
            else pxs::BlockCache::get().drop(p);
        }
    }
};

bool shifted_applies(const pxStructure_t* s, const pxSolveOptions& o)
{
    return o.shifted >= 1 && (s->model == PX_WFQ || s->model == PX_BEM) && !s->het;
}

// Structures that pxSolveBatch and the server solve whole (each on a stream of
// its own, several at a time) instead of in the stacked block: those of the
// shared-Krylov phase, and structures of kPoolMinAtoms atoms or more, whose
// own launches fill the GPU and whose restart escalation would otherwise hold
// every segment of the block (dipole-model requests of 1k-4k atoms ran 1.7x
// slower stacked than alone).
constexpr int64_t kPoolMinAtoms = 1024;
bool pooled_solve(const pxStructure_t* s, const pxSolveOptions& o)
{
    return shifted_applies(s, o) || s->g.n >= kPoolMinAtoms;
}

// A block Krylov space of R columns per step spans all nu unknowns after
// ceil(nu / R) steps, where every pair's GMRES iterate is exact: the phase
// never needs more (two steps of margin for the rounding).
int phase_step_limit(const pxStructure_t* s, int R)
{
    return (int)std::min<int64_t>((s->g.nu + R - 1) / R + 2, 1 << 20);
}

// The step loop of a shared-Krylov phase: steps on the structure's stream, the
// frequencies' Givens QRs in batches on a second stream of the same priority
// (beside the next steps' T-applies), the stop flag published once per batch
// and polled by the host a few steps behind.
class PhaseRun {
  public:
    virtual ~PhaseRun()
    {
        if (side_e_) (void)hipEventDestroy(side_e_);
        if (side_s_) (void)hipStreamDestroy(side_s_);
    }
    bool ended() const { return ended_; }
    // After finish(): relres holds every pair's true FP64 residual (not the
    // Givens estimate), so the blocked solver need only take the pairs above
    // rel_tol.
    bool verified() const { return verified_; }
    // Enqueues at most max_steps steps; without `wait`, returns (blocked set)
    // rather than wait for a Givens batch still on the device.
    int advance(int max_steps, bool wait, bool& blocked)
    {
        int did = 0;
        while (!ended_ && did < max_steps) {
            const int k = launched_;
            if (k >= kcap_) {
                end_loop();
                break;
            }
            bool stopped = false;
            while (polled_ < (int)batch_step_.size() && batch_step_[polled_] <= k - lag_) {
                if (!wait && !s_->sync.ready(polled_)) {
                    blocked = true;
                    return did;
                }
                if (s_->sync.stopped(polled_++)) {
                    stopped = true;
                    break;
                }
            }
            if (stopped) {
                end_loop();
                break;
            }
            step(k);
            if (k - gnext_ >= gb_) {
                givens_side(gnext_, gb_, k);
                gnext_ += gb_;
            }
            ++launched_;
            ++did;
        }
        return did;
    }
    // Finishing kernels (factors, back substitution, x = V y), a wait for the
    // structure's stream, statistics.
    void finish()
    {
        bool blocked = false;
        while (!ended_) advance(1 << 30, true, blocked);
        finish_kernels(launched_);
    }

  protected:
    PhaseRun(pxStructure_t* s, const pxSolveOptions& o) : s_(s), o_(o), tm_(o.timings != 0) {}
    // after the buffers: the stop flag, the side stream
    void start(int kcap, int lag, int gb)
    {
        kcap_ = kcap;
        lag_ = lag;
        gb_ = gb;
        s_->sync.ensure(kcap / gb + 2);
        stop_ = s_->sync.flag();
        s_->sync.reset(s_->st);
        HC(hipStreamCreateWithFlags(&side_s_, hipStreamNonBlocking));
        HC(hipEventCreateWithFlags(&side_e_, hipEventDisableTiming));
    }
    virtual void step(int k) = 0;
    virtual void givens(int k0, int kn) = 0;   // on side_s_
    virtual void last_step(int launched) = 0;
    virtual void finish_kernels(int launched) = 0;

    pxStructure_t* s_;
    pxSolveOptions o_;
    LaunchTimer tm_;
    Scratch sc_;
    int32_t* stop_ = nullptr;
    hipStream_t side_s_ = nullptr;
    hipEvent_t side_e_ = nullptr;
    int method_ = TA_FLY;
    bool verified_ = false;

  private:
    void givens_side(int k0, int kn, int at_step)
    {
        HC(hipEventRecord(side_e_, s_->st));
        HC(hipStreamWaitEvent(side_s_, side_e_, 0));
        givens(k0, kn);
        s_->sync.publish((int)batch_step_.size(), side_s_);
        batch_step_.push_back(at_step);
    }
    // the last column's correction (a no-op once every pair converged), the
    // remaining Givens batches, the side stream joined into the main one
    void end_loop()
    {
        last_step(launched_);
        while (gnext_ < launched_) {
            const int kn = std::min(gb_, launched_ - gnext_);
            givens_side(gnext_, kn, launched_);
            gnext_ += kn;
        }
        HC(hipEventRecord(side_e_, side_s_));
        HC(hipStreamWaitEvent(s_->st, side_e_, 0));
        ended_ = true;
    }
    int kcap_ = 0, lag_ = 0, gb_ = 1;
    int launched_ = 0, gnext_ = 0, polled_ = 0;
    bool ended_ = false;
    std::vector<int> batch_step_;
};

// One real Arnoldi process per polarization (shifted = 1, and the fallback for
// one polarization or a zero right-hand side).
class ShiftedRun : public PhaseRun {
  public:
    ShiftedRun(pxStructure_t* s, const pxSolveOptions& o) : PhaseRun(s, o)
    {
        npol_ = s->npol;
        R_ = npol_;
        P_ = s->ncol;
        const int R = R_, P = P_;
        const int64_t nup = s->g.nup;
        hipStream_t st = s->st;
        // basis, Hessenberg matrices and triangular factors within a quarter of the free device memory
        size_t fr = 0, tot = 0;
        HC(hipMemGetInfo(&fr, &tot));
        int kcap = std::min(o.shifted_max_steps, phase_step_limit(s, 1));
        auto bytes_for = [&](double k) {
            return (k + 1) * (double)nup * R * 8.0 + (k + 1) * k * R * 8.0 + k * (double)P * (8 + 16 + 16 + 16) +
                   k * (k + 1) / 2 * P * 16.0 + (double)px::ms_part2_doubles(R, nup, (int)k) * 8.0;
        };
        while (kcap > 8 && bytes_for(kcap) > 0.25 * (double)fr) kcap = kcap * 3 / 4;
        kc_ = kcap;
        vstride_ = nup * R;
        V_ = sc_.get<double>((size_t)(kcap + 1) * vstride_);
        u_ = sc_.get<double>((size_t)vstride_);
        Y_ = sc_.get<double>((size_t)vstride_);
        wt_ = sc_.get<double>((size_t)vstride_);
        part_ = sc_.get<double>(px::ms_part_doubles(R, nup, kcap));
        part2_ = sc_.get<double>(px::ms_part2_doubles(R, nup, kcap));
        G_ = sc_.get<double>((size_t)(kcap + 1) * 2 * R);
        H_ = sc_.get<double>((size_t)(kcap + 1) * kcap * R);
        coefv_ = sc_.get<double>((size_t)kcap * R);
        coefu_ = sc_.get<double>((size_t)kcap * R);
        scal_ = sc_.get<double>((size_t)3 * R);
        z_ = sc_.get<double2>(P);
        cs_ = sc_.get<double>((size_t)kcap * P);
        sn_ = sc_.get<double2>((size_t)kcap * P);
        g_ = sc_.get<double2>((size_t)(kcap + 1) * P);
        rst_ = sc_.get<double2>(px::ms_rst_elems(P, kcap));
        ycoef_ = sc_.get<double2>((size_t)kcap * P);
        target_ = sc_.get<double>(P);
        resid_ = sc_.get<double>(P);
        double* bn = sc_.get<double>(npol_);
        done_ = sc_.get<int32_t>(P);
        ndone_ = sc_.get<int32_t>(1);

        std::vector<double2> zh(P), g0(P);
        std::vector<double> th(P);
        for (int p = 0; p < P; ++p) {
            double zr, zi;
            shift_of(s, p / npol_, zr, zi);
            zh[p] = make_double2(zr, zi);
            g0[p] = make_double2(s->bnorm[p % npol_], 0.0);
            th[p] = kPhaseTarget * o.rel_tol * s->bnorm[p];
        }
        HC(hipMemcpyAsync(z_, zh.data(), sizeof(double2) * P, hipMemcpyHostToDevice, st));
        HC(hipMemcpyAsync(g_, g0.data(), sizeof(double2) * P, hipMemcpyHostToDevice, st));
        HC(hipMemcpyAsync(target_, th.data(), sizeof(double) * P, hipMemcpyHostToDevice, st));
        HC(hipMemcpyAsync(bn, s->bnorm.data(), sizeof(double) * npol_, hipMemcpyHostToDevice, st));
        px::fill_zero(done_, sizeof(int32_t) * P, st);
        px::fill_zero(ndone_, sizeof(int32_t), st);
        px::ms_init(R, s->b, s->ldg, bn, u_, nup, st);
        method_ = tapply_method(s, false, u_, Y_, R, R, o);
        // the T-apply kernels return at once once the stop flag is set; a lag
        // of a few steps keeps the host from waiting on a Givens batch the main
        // stream has not overtaken yet
        start(kcap, 2 * kLag, px::ms_givens_batch());
    }

  protected:
    void step(int k) override
    {
        pxStructure_t* s = s_;
        // wt = Kbar T u for the candidate u of v_k
        tapply(s, method_, false, u_, Y_, R_, R_, stop_, tm_.events(k, 0));
        px::ms_spmv(R_, s->g, Y_, wt_, s->st, stop_, tm_.events(k, 1));
        // one dot and one update pass: v_k final, column k-1 of Hbar final
        px::ms_step(R_, V_, vstride_, k, u_, wt_, part_, part2_, G_, H_, kc_, coefv_, coefu_, scal_, s->g.nup, false,
                    s->st, stop_, tm_.events(k, 2));
    }
    void givens(int k0, int kn) override
    {
        px::ms_givens(H_, kc_, npol_, P_, k0, kn, z_, cs_, sn_, g_, target_, done_, resid_, ndone_, stop_, side_s_);
    }
    void last_step(int launched) override
    {
        px::ms_step(R_, V_, vstride_, launched, u_, u_, part_, part2_, G_, H_, kc_, coefv_, coefu_, scal_, s_->g.nup,
                    true, s_->st, stop_);
    }
    void finish_kernels(int launched) override
    {
        pxStructure_t* s = s_;
        hipStream_t st = s->st;
        const int P = P_, npol = npol_, R = R_;
        px::ms_rfactor(H_, kc_, npol, P, launched, z_, cs_, sn_, done_, rst_, st);
        px::ms_backsub(rst_, P, launched, done_, g_, ycoef_, st);
        px::ms_xcombine(R, V_, vstride_, launched, done_, ycoef_, P, s->x, s->ldg, s->g.nup, st);
        std::vector<int32_t> dh(P);
        std::vector<double> rh(P);
        HC(hipMemcpyAsync(dh.data(), done_, sizeof(int32_t) * P, hipMemcpyDeviceToHost, st));
        HC(hipMemcpyAsync(rh.data(), resid_, sizeof(double) * P, hipMemcpyDeviceToHost, st));
        HC(hipStreamSynchronize(st));
        sc_.idle = true;   // nothing on either stream uses the scratch any more
        int executed = 0;
        for (int p = 0; p < P; ++p) {
            s->iters[p] = dh[p] ? dh[p] : launched;
            s->cycles[p] = 1;
            s->relres[p] = s->bnorm[p] > 0.0 ? rh[p] / s->bnorm[p] : 0.0;
            executed = std::max(executed, s->iters[p]);
        }
        // the device ran one step past the last column it needed (that column's correction)
        executed = std::min(launched, executed + 1);
        double t_ap = 0.0;
        tm_.collect(executed, t_ap, s->ms[3], s->ms[4]);
        s->ms[2] += t_ap;
        s->tms[method_ == TA_STORED ? 3 : 2] += t_ap;
        const double nu = (double)s->g.nu;
        s->tstats[method_ == TA_STORED ? 3 : 2] += executed;
        s->counts[3] += executed;
        s->counts[4] += (int64_t)executed * R;
        s->counts[5] += (int64_t)executed * npol;
        s->tflop[method_ == TA_STORED ? 3 : 2] += 2.0 * nu * nu * npol * executed;
        s->work[1] += 2.0 * nu * nu * npol * executed;
        // one dot and one update pass over the basis per step
        s->work[2] += 2.0 * 8.0 * (double)s->g.n * npol * (double)executed * (executed + 1) / 2.0;
    }

  private:
    int npol_ = 0, R_ = 0, P_ = 0, kc_ = 0;
    int64_t vstride_ = 0;
    double *V_, *u_, *Y_, *wt_, *part_, *part2_, *G_, *H_, *coefv_, *coefu_, *scal_, *cs_, *target_, *resid_;
    double2 *z_, *sn_, *g_, *rst_, *ycoef_;
    int32_t *done_, *ndone_;
};

// The shared-Krylov phase over a block of polarizations: one block Arnoldi
// process for the npol right-hand sides (px_shifted_block.hip), for 2 or 3
// polarizations whose right-hand sides are all non-zero.
bool block_applies(const pxStructure_t* s, const pxSolveOptions& o)
{
    if (o.shifted != 2 || s->npol < 2 || s->npol > 3) return false;
    for (int l = 0; l < s->npol; ++l)
        if (!(s->bnorm[l] > 0.0)) return false;
    return true;
}

class BlockShiftedRun : public PhaseRun {
  public:
    BlockShiftedRun(pxStructure_t* s, const pxSolveOptions& o) : PhaseRun(s, o)
    {
        R_ = s->npol;
        P_ = s->ncol;
        NW_ = P_ / R_;
        const int R = R_, P = P_, NW = NW_;
        const int64_t nup = s->g.nup;
        hipStream_t st = s->st;
        size_t fr = 0, tot = 0;
        HC(hipMemGetInfo(&fr, &tot));
        // the back substitution holds a frequency's kcap R rows of its right-hand
        // sides in registers (at most 4096)
        int kcap = std::min(std::min(o.shifted_max_steps, 4096 / R), phase_step_limit(s, R));
        auto bytes_for = [&](double k) {
            const double kc = k * R;
            return (k + 1) * (double)nup * R * 8.0 + (kc + R) * kc * 8.0 + kc * R * NW * 24.0 +
                   (kc + R) * NW * R * 16.0 + kc * (kc + 1) / 2 * NW * 16.0 + kc * P * 16.0 +
                   (double)px::msb_part2_doubles(R, nup, (int)k) * 8.0;
        };
        while (kcap > 8 && bytes_for(kcap) > 0.25 * (double)fr) kcap = kcap * 3 / 4;
        const int RR = R * R;
        ldh_ = kcap * R;
        vstride_ = nup * R;
        V_ = sc_.get<double>((size_t)(kcap + 1) * vstride_);
        u_ = sc_.get<double>((size_t)vstride_);
        Y_ = sc_.get<double>((size_t)vstride_);
        wt_ = sc_.get<double>((size_t)vstride_);
        part_ = sc_.get<double>(px::msb_part_doubles(R, kcap));
        part2_ = sc_.get<double>(px::msb_part2_doubles(R, nup, kcap));
        G_ = sc_.get<double>((size_t)(kcap + 1) * 2 * RR);
        Hb_ = sc_.get<double>((size_t)(kcap + 1) * R * ldh_);
        coefv_ = sc_.get<double>((size_t)kcap * RR);
        coefu_ = sc_.get<double>((size_t)kcap * RR);
        scal_ = sc_.get<double>((size_t)2 * RR);
        rho0_ = sc_.get<double>((size_t)RR);
        z_ = sc_.get<double2>(P);
        rc_ = sc_.get<double>((size_t)kcap * R * R * NW);
        rs_ = sc_.get<double2>((size_t)kcap * R * R * NW);
        g_ = sc_.get<double2>((size_t)(kcap + 1) * R * NW * R);
        target_ = sc_.get<double>(P);
        resid_ = sc_.get<double>(P);
        done_ = sc_.get<int32_t>(P);
        ndone_ = sc_.get<int32_t>(1);

        std::vector<double2> zh(P);
        std::vector<double> th(P);
        for (int p = 0; p < P; ++p) {
            double zr, zi;
            shift_of(s, p / R, zr, zi);
            zh[p] = make_double2(zr, zi);
            th[p] = kPhaseTarget * o.rel_tol * s->bnorm[p];
        }
        HC(hipMemcpyAsync(z_, zh.data(), sizeof(double2) * P, hipMemcpyHostToDevice, st));
        HC(hipMemcpyAsync(target_, th.data(), sizeof(double) * P, hipMemcpyHostToDevice, st));
        px::fill_zero(Hb_, sizeof(double) * (size_t)(kcap + 1) * R * ldh_, st);
        px::fill_zero(g_, sizeof(double2) * (size_t)(kcap + 1) * R * NW * R, st);
        px::fill_zero(done_, sizeof(int32_t) * P, st);
        px::fill_zero(ndone_, sizeof(int32_t), st);
        px::msb_init(R, s->b, s->ldg, u_, nup, st);
        method_ = tapply_method(s, false, u_, Y_, R, R, o);
        // the banded QRs run on the side stream, a launch every GBB block steps
        start(kcap, 2 * kLag, px::msb_givens_cols() / R);
    }

  protected:
    void step(int k) override
    {
        pxStructure_t* s = s_;
        // Wt = Kbar T U for the candidate block U of V_k
        tapply(s, method_, false, u_, Y_, R_, R_, stop_, tm_.events(k, 0));
        px::ms_spmv(R_, s->g, Y_, wt_, s->st, stop_, tm_.events(k, 1));
        px::msb_step(R_, V_, vstride_, k, u_, wt_, part_, part2_, G_, Hb_, ldh_, coefv_, coefu_, scal_, rho0_,
                     s->g.nup, false, s->st, stop_, tm_.events(k, 2));
    }
    void givens(int kb0, int nkb) override
    {
        px::msb_givens(R_, Hb_, ldh_, NW_, kb0 * R_, nkb * R_, z_, rc_, rs_, g_, rho0_, target_, done_, resid_, ndone_,
                       stop_, side_s_);
    }
    void last_step(int launched) override
    {
        px::msb_step(R_, V_, vstride_, launched, u_, u_, part_, part2_, G_, Hb_, ldh_, coefv_, coefu_, scal_, rho0_,
                     s_->g.nup, true, s_->st, stop_);
    }
    void finish_kernels(int launched) override
    {
        pxStructure_t* s = s_;
        hipStream_t st = s->st;
        const int R = R_, P = P_, NW = NW_;
        const int kcols = launched * R;
        double2* rst = sc_.get<double2>(std::max<size_t>(1, px::msb_rst_elems(NW, kcols)));
        double2* ycoef = sc_.get<double2>(std::max<size_t>(1, (size_t)kcols * P));
        px::msb_finish_solve(R, Hb_, ldh_, NW, kcols, z_, rc_, rs_, done_, rst, g_, ycoef, V_, vstride_, s->x, s->ldg,
                             s->g.nup, st);
        // When the basis is narrow beside the pairs (BEM: 15 block steps for
        // 192 pairs), every pair's true FP64 residual comes from one operator
        // apply over the basis: T x = (T V) y, the same coefficients as x =
        // V y, then b - (Kbar T x - z x); the blocked solver then takes only
        // the pairs above rel_tol instead of applying T to all of them.
        const int64_t nup = s->g.nup;
        const int kpad = s->g.bem ? (kcols + 15) / 16 * 16 : (kcols + 127) / 128 * 128;
        std::vector<double> tn;
        if (kcols > 0 && kpad <= P) {
            double* Wb = sc_.get<double>((size_t)nup * kpad);
            double* Zb = sc_.get<double>((size_t)nup * kpad);
            double* TV = sc_.get<double>((size_t)launched * vstride_);
            double2* TX = sc_.get<double2>((size_t)nup * s->ldg);
            double2* Rr = sc_.get<double2>((size_t)nup * s->ldg);
            const int nchunk = px::arnoldi_chunks(nup);
            double* npart = sc_.get<double>((size_t)nchunk * s->ldg);
            double* nrm = sc_.get<double>(s->ldg);
            px::msb_basis_gather(R, V_, vstride_, kcols, nup, Wb, kpad, st);
            const int meth = tapply_method(s, false, Wb, Zb, kpad, kpad, o_, true);
            tapply(s, meth, false, Wb, Zb, kpad, kpad, nullptr, nullptr, kpad);
            px::msb_basis_scatter(R, Zb, kpad, kcols, nup, TV, vstride_, st);
            px::msb_xcombine(R, TV, vstride_, kcols, done_, ycoef, P, TX, s->ldg, nup, st);
            px::spmm_shift(s->g, TX, false, 2 * s->ldg, s->x, z_, z_, s->b, Rr, P, s->ldg, SOLVER_MU_SIGN, st);
            px::col_norm_partial(Rr, npart, P, s->ldg, nup, st);
            px::reduce_norms(npart, nchunk, nrm, P, s->ldg, st);
            tn.resize(P);
            HC(hipMemcpyAsync(tn.data(), nrm, sizeof(double) * P, hipMemcpyDeviceToHost, st));
            const double nu = (double)s->g.nu;
            s->counts[3] += 1;
            s->counts[4] += kpad;
            s->counts[5] += kcols;
            s->work[1] += 2.0 * nu * nu * kcols;
            s->work[2] += 80.0 * nu * P;
            verified_ = true;
        }
        std::vector<int32_t> dh(P);
        std::vector<double> rh(P);
        HC(hipMemcpyAsync(dh.data(), done_, sizeof(int32_t) * P, hipMemcpyDeviceToHost, st));
        HC(hipMemcpyAsync(rh.data(), resid_, sizeof(double) * P, hipMemcpyDeviceToHost, st));
        HC(hipStreamSynchronize(st));
        if (verified_) rh = tn;
        sc_.idle = true;   // nothing on either stream uses the scratch any more
        int executed = 0;
        for (int p = 0; p < P; ++p) {
            s->iters[p] = dh[p] ? (dh[p] + R - 1) / R : launched;
            s->cycles[p] = 1;
            s->relres[p] = s->bnorm[p] > 0.0 ? rh[p] / s->bnorm[p] : 0.0;
            executed = std::max(executed, s->iters[p]);
        }
        executed = std::min(launched, executed + 1);
        double t_ap = 0.0;
        tm_.collect(executed, t_ap, s->ms[3], s->ms[4]);
        s->ms[2] += t_ap;
        s->tms[method_ == TA_STORED ? 3 : 2] += t_ap;
        const double nu = (double)s->g.nu;
        s->tstats[method_ == TA_STORED ? 3 : 2] += executed;
        s->counts[3] += executed;
        s->counts[4] += (int64_t)executed * R;
        s->counts[5] += (int64_t)executed * R;
        s->tflop[method_ == TA_STORED ? 3 : 2] += 2.0 * nu * nu * R * executed;
        s->work[1] += 2.0 * nu * nu * R * executed;
        // one dot pass (2 R^2 products per basis block and row) and one update
        // pass (2 R^2) per step
        s->work[2] += 2.0 * 2.0 * 2.0 * R * R * (double)s->g.n * (double)executed * (executed + 1) / 2.0;
    }

  private:
    int R_ = 0, P_ = 0, NW_ = 0, ldh_ = 0;
    int64_t vstride_ = 0;
    double *V_, *u_, *Y_, *wt_, *part_, *part2_, *G_, *Hb_, *coefv_, *coefu_, *scal_, *rho0_, *rc_, *target_, *resid_;
    double2 *z_, *rs_, *g_;
    int32_t *done_, *ndone_;
};

pxStatus check_options(const pxSolveOptions& o)
{
    if (o.restart_m < 1 || o.restart_m > 1000 || o.max_restart_m > 1000)
        return fail(PX_E_INVALID, "restart_m and max_restart_m must be in [1, 1000]");
    if (!(o.rel_tol > 0.0) || o.max_cycles < 1 || o.max_block_cols < 0 || o.inner_reduction < 0.0 ||
        o.stall_cycles < 0 || o.block_cols < 0 || o.block_cols % 64 != 0 || o.block_cols > 1024 ||
        (o.ortho != PX_ORTHO_CGS2 && o.ortho != PX_ORTHO_DCGS2) || o.graph_steps < 0 || o.graph_steps > 64 ||
        (o.t_apply != PX_TAPPLY_AUTO && o.t_apply != PX_TAPPLY_ON_THE_FLY && o.t_apply != PX_TAPPLY_STORED) ||
        (o.shifted < 0 || o.shifted > 2) || o.shifted_max_steps < 1 || o.shifted_max_steps > 4000 ||
        (o.precision != PX_FP64 && o.precision != PX_MIXED))
        return fail(PX_E_INVALID, "invalid solve options");
    return PX_OK;
}

// Status of a structure the stacked engine finished.
void set_engine_status(pxStructure_t* s, const pxSolveOptions& o)
{
    s->last_status = PX_OK;
    s->last_error.clear();
    for (int c = 0; c < s->ncol; ++c)
        if (!(s->relres[c] <= o.rel_tol)) {
            s->last_status = PX_E_NOTCONV;
            s->last_error = "some columns did not reach rel_tol";
        }
}

// ---- one structure's whole solve, advanced step by step ----------------------
// Right-hand sides and norms, the shared-Krylov phase where it applies, the
// blocked solver over every column block (the true FP64 residual of every
// column, restart cycles for any column above rel_tol), the observables.
// pxSolveSpectrum drives it to the end on the structure's stream; the batch
// and the server drive several at once from the calling thread, each on a
// stream of its own (ordered after the structure's stream when it starts, and
// the structure's stream after it when it ends), so their launches overlap on
// the device without host threads.
class WholeSolve {
  public:
    WholeSolve(pxStructure_t* s, const pxSolveOptions& o, bool own_stream) : s_(s), o_(o)
    {
        t0_ = std::chrono::steady_clock::now();
        for (double& v : s->ms) v = 0.0;
        for (int64_t& v : s->counts) v = 0;
        for (double& v : s->work) v = 0.0;
        for (int64_t& v : s->tstats) v = 0;
        for (double& v : s->tms) v = 0.0;
        for (double& v : s->tflop) v = 0.0;
        s->last_status = PX_E_STATE;
        s->last_error = "solve in progress";
        if (own_stream) {
            HC(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
            HC(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
            HC(hipEventRecord(ev_, s->st));
            HC(hipStreamWaitEvent(st_, ev_, 0));
            home_ = s->st;
            s->st = st_;
            moved_ = true;
        }
        try {
            blk_ = o.max_block_cols > 0 ? std::min(o.max_block_cols, s->ncol) : s->ncol;
            ensure_vectors(s, pad_cols(blk_, true));
            prepare_solve(s);
            if (shifted_applies(s, o)) {
                if (block_applies(s, o)) phase_.reset(new BlockShiftedRun(s, o));
                else phase_.reset(new ShiftedRun(s, o));
            } else {
                next_block();
            }
        } catch (...) {
            phase_.reset();
            block_.reset();
            hand_back();
            if (ev_) (void)hipEventDestroy(ev_);
            if (st_) (void)hipStreamDestroy(st_);
            throw;
        }
    }
    ~WholeSolve()
    {
        phase_.reset();
        block_.reset();
        hand_back();
        if (ev_) (void)hipEventDestroy(ev_);
        if (st_) (void)hipStreamDestroy(st_);
    }
    WholeSolve(const WholeSolve&) = delete;
    WholeSolve& operator=(const WholeSolve&) = delete;

    bool finished() const { return fin_; }
    pxStructure_t* structure() const { return s_; }
    // Enqueues at most about max_steps steps; without `wait` it returns
    // rather than wait for work still on the device.  Returns the work done
    // (0: it would have had to wait).
    int advance(int max_steps, bool wait)
    {
        int did = 0;
        while (!fin_ && did < max_steps) {
            if (phase_) {
                bool blocked = false;
                did += phase_->advance(max_steps - did, wait, blocked);
                if (phase_->ended()) {
                    phase_->finish();
                    if (phase_->verified()) {
                        // only the pairs whose true residual is above rel_tol go on
                        pending_.clear();
                        for (int c = 0; c < s_->ncol; ++c)
                            if (!(s_->relres[c] <= o_.rel_tol)) pending_.push_back(c);
                        use_pending_ = true;
                    }
                    phase_.reset();
                    next_block();
                    ++did;
                } else if (blocked) {
                    break;
                }
                continue;
            }
            const int n = block_->advance(max_steps - did, wait);
            did += n;
            if (block_->finished()) {
                block_.reset();
                next_block();
                ++did;
            } else if (n == 0) {
                break;
            }
        }
        return did;
    }

  private:
    void next_block()
    {
        if (use_pending_) {
            if (p0_ < pending_.size()) {
                const size_t e = std::min(pending_.size(), p0_ + (size_t)blk_);
                std::vector<int> cols(pending_.begin() + p0_, pending_.begin() + e);
                p0_ = e;
                block_.reset(new BlockRun(s_, cols, o_));
                return;
            }
        } else if (c0_ < s_->ncol) {
            std::vector<int> cols;
            for (int c = c0_; c < std::min(s_->ncol, c0_ + blk_); ++c) cols.push_back(c);
            c0_ += blk_;
            block_.reset(new BlockRun(s_, cols, o_));
            return;
        }
        finish_solve(s_);
        hand_back();
        s_->ms[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
        s_->ms[5] = s_->ms[0] - s_->ms[1] - s_->ms[2] - s_->ms[3] - s_->ms[4];
        s_->last_status = PX_OK;
        s_->last_error.clear();
        for (int c = 0; c < s_->ncol; ++c)
            if (!(s_->relres[c] <= o_.rel_tol)) {
                s_->last_status = PX_E_NOTCONV;
                s_->last_error = "some columns did not reach rel_tol";
            }
        fin_ = true;
    }
    // the structure back on its own stream, ordered after everything this solve enqueued
    void hand_back()
    {
        if (!moved_) return;
        moved_ = false;
        if (hipEventRecord(ev_, st_) == hipSuccess) (void)hipStreamWaitEvent(home_, ev_, 0);
        (void)hipStreamSynchronize(st_);
        s_->st = home_;
    }

    pxStructure_t* s_;
    pxSolveOptions o_;
    std::chrono::steady_clock::time_point t0_;
    hipStream_t st_ = nullptr, home_ = nullptr;
    hipEvent_t ev_ = nullptr;
    bool moved_ = false, fin_ = false;
    int blk_ = 0, c0_ = 0;
    // the columns left after a phase that checked every true residual
    std::vector<int> pending_;
    size_t p0_ = 0;
    bool use_pending_ = false;
    std::unique_ptr<PhaseRun> phase_;
    std::unique_ptr<BlockRun> block_;
};

pxStatus solve_impl(pxStructure_t* s, const pxSolveOptions& o)
{
    if (s->ncol == 0) return fail(PX_E_STATE, "pxSolveSpectrum: call pxSetFrequencies first");
    if (check_options(o) != PX_OK) return PX_E_INVALID;
    WholeSolve w(s, o, false);
    while (!w.finished()) w.advance(1 << 30, true);
    if (s->last_status != PX_OK) return fail(s->last_status, s->last_error);
    return PX_OK;
}


bool finite3(const double* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

pxStatus status_of(const HipError& h) { return h.e == hipErrorOutOfMemory ? PX_E_OOM : PX_E_DEVICE; }

template <typename F>
pxStatus guarded(F&& f)
{
    try {
        return f();
    } catch (const HipError& h) {
        return fail(status_of(h), std::string(h.where) + ": " + hipGetErrorString(h.e));
    } catch (const std::bad_alloc&) {
        return fail(PX_E_OOM, "host allocation failed");
    } catch (...) {
        return fail(PX_E_DEVICE, "unexpected exception");
    }
}

// A solve of pxSolveSpectrumAsync: the whole solve on the structure's stream,
// advanced by later calls.
class AsyncSolve : public pxs::PendingSolve {
  public:
    AsyncSolve(pxStructure_t* s, const pxSolveOptions& o) : w(s, o, false) {}
    WholeSolve w;
};

// Steps enqueued per non-blocking call of an asynchronous solve.
constexpr int kAsyncSteps = 64;

// Advances s's asynchronous solve (to its end when `wait`); the solve is
// dropped once finished or when it fails.  Returns whether it finished.
bool advance_pending(pxStructure_t* s, bool wait)
{
    auto* a = static_cast<AsyncSolve*>(s->pending.get());
    try {
        if (wait) {
            while (!a->w.finished()) a->w.advance(1 << 30, true);
        } else {
            a->w.advance(kAsyncSteps, false);
        }
    } catch (...) {
        (void)hipDeviceSynchronize();
        s->pending.reset();
        s->last_status = PX_E_DEVICE;
        s->last_error = "the asynchronous solve failed";
        throw;
    }
    if (!a->w.finished()) return false;
    s->pending.reset();
    return true;
}

// Every call on a structure first completes an asynchronous solve in
// progress (its own status stays readable with pxGetSolveStatus).
pxStatus settle(pxStructure_t* s)
{
    if (!s || !s->pending) return PX_OK;
    return guarded([&]() -> pxStatus {
        advance_pending(s, true);
        return PX_OK;
    });
}

#define PX_SETTLE(s)                            \
    do {                                        \
        const pxStatus st_ = settle(s);         \
        if (st_ != PX_OK) return st_;           \
    } while (0)

// ---- several whole solves at once from one host thread (batch and server) ----
// Each structure runs as a WholeSolve on a stream of its own; the driver
// enqueues a few steps of each in turn without waiting for the device, and
// only waits (on the oldest) when none of them can go on.  A solve that
// throws is ended on its own: its structure records the status and the
// message, the others go on.
constexpr int kConcurrentSolves = 4;   // GPU_MAX_HW_QUEUES is 4 by default
constexpr int kStepsPerTurn = 8;

class SolveDriver {
  public:
    explicit SolveDriver(const pxSolveOptions& o) : o_(o) {}
    ~SolveDriver() { run_.clear(); }
    bool busy() const { return !run_.empty(); }
    int running() const { return (int)run_.size(); }
    bool has_room() const { return (int)run_.size() < kConcurrentSolves; }
    // starts s (it must have frequencies set); a failure to start is recorded in s
    void start(pxStructure_t* s)
    {
        try {
            run_.emplace_back(new WholeSolve(s, o_, true));
        } catch (const HipError& h) {
            record(s, status_of(h), std::string(h.where) + ": " + hipGetErrorString(h.e));
        } catch (const std::bad_alloc&) {
            record(s, PX_E_OOM, "host allocation failed");
        }
    }
    // One turn over the running solves; returns the structures that finished
    // (successfully or not).  With `may_wait`, waits for the device when no
    // solve could go on without waiting.
    std::vector<pxStructure_t*> turn(bool may_wait)
    {
        int did = 0;
        for (size_t i = 0; i < run_.size(); ++i) did += step(i, kStepsPerTurn, false);
        if (did == 0 && may_wait && !run_.empty()) step(0, 1, true);
        return collect();
    }
    std::vector<pxStructure_t*> take_failed_starts()
    {
        std::vector<pxStructure_t*> out;
        out.swap(failed_);
        return out;
    }

  private:
    int step(size_t i, int n, bool wait)
    {
        WholeSolve* w = run_[i].get();
        if (!w || w->finished()) return 0;
        try {
            return w->advance(n, wait);
        } catch (const HipError& h) {
            end_failed(i, status_of(h), std::string(h.where) + ": " + hipGetErrorString(h.e));
        } catch (const std::bad_alloc&) {
            end_failed(i, PX_E_OOM, "host allocation failed");
        }
        return 1;
    }
    void end_failed(size_t i, pxStatus st, const std::string& msg)
    {
        pxStructure_t* s = run_[i]->structure();
        run_[i].reset();   // waits for its stream, hands the structure back
        record(s, st, msg);
    }
    void record(pxStructure_t* s, pxStatus st, const std::string& msg)
    {
        s->last_status = st;
        s->last_error = msg;
        s->solved = false;
        failed_.push_back(s);
    }
    std::vector<pxStructure_t*> collect()
    {
        std::vector<pxStructure_t*> out;
        out.swap(failed_);
        for (auto& w : run_)
            if (w && w->finished()) {
                out.push_back(w->structure());
                w.reset();
            }
        run_.erase(std::remove_if(run_.begin(), run_.end(), [](const std::unique_ptr<WholeSolve>& w) { return !w; }),
                   run_.end());
        return out;
    }
    pxSolveOptions o_;
    std::vector<std::unique_ptr<WholeSolve>> run_;
    std::vector<pxStructure_t*> failed_;
};

// HBM bytes of one whole solve (admission of the server's whole solves): the
// active block's vectors and T-apply scratch, the near-field list, and the
// shared-Krylov phase's basis and factors or the blocked solver's basis.
double solve_footprint(const pxStructure_t* s, const pxSolveOptions& o)
{
    const int blk = o.max_block_cols > 0 ? std::min(o.max_block_cols, s->ncol) : s->ncol;
    const double lda = pad_cols(blk, true);
    const double nup = (double)s->g.nup, vec = nup * lda;
    double b = vec * (5 * 16 + 8 + 8 + 16) + (double)px::tapply_f64_scratch_bytes(s->g, s->g.bem ? 2 * (int)lda : 8) +
               (double)px::tapply_f32_scratch_bytes(s->g, 2 * (int)lda);
    if (s->model == PX_WFQ) b += 6000.0 * (double)s->g.n;   // near-field list (about 400 entries per atom)
    if (!s->g.bem) {
        // a stored T the tuner may build and the structure then keeps: FP64
        // for the true residuals (up to the size it tunes), FP32 for the
        // mixed-precision blocked cycles
        const double t64 = nup * nup * 8.0;
        if (t64 <= kSingleUseTuneMaxBytes) b += t64;
        if (o.precision == PX_MIXED) b += nup * nup * 4.0;
    }
    const int m_max = std::max(o.restart_m, o.max_restart_m);
    if (shifted_applies(s, o)) {
        const double R = s->npol, P = s->ncol;
        // the block phase's step limit (one process per polarization, its
        // fallback for a zero right-hand side, can take up to nu steps)
        const int rk = o.shifted == 2 && s->npol >= 2 ? s->npol : 1;
        const double k = std::min(o.shifted_max_steps, phase_step_limit(s, rk));
        b += (k + 1) * nup * R * 8.0 + (k + 1) * k * R * R * 8.0 + k * P * 56.0 + k * (k + 1) / 2.0 * P * 16.0;
        // the true residuals through the basis (taken when its padded width
        // is at most P): the basis as a matrix and its product (each at most
        // P columns), the product in the basis layout, T x and the residuals
        b += 2.0 * nup * P * 8.0 + std::min(k + 1, P / R + 1) * nup * R * 8.0 + 2.0 * nup * (double)s->ldg * 16.0;
    } else {
        b += (m_max + 1.0) * vec * 16.0 + 2.0 * m_max * (m_max + 1.0) * lda * 16.0;
    }
    return b;
}


}  // namespace

// ---- device scratch of pxApplyOperatorNoAlloc --------------------------------
// A fixed array per GPU, held until the process ends, for callers that cannot
// allocate.  Host code never uses its name as an address: the device address
// is taken once per device with hipGetSymbolAddress and kept.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64] = {};

// This device's address of the scratch array (looked up on the first call on
// each device, with that device current).
char* noalloc_scratch()
{
    int dev = 0;
    HC(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw HipError{hipErrorInvalidDevice, "hipGetDevice"};
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        HC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress"};
        g_noalloc_ptr[dev] = p;
    }
    return static_cast<char*>(g_noalloc_ptr[dev]);
}

}  // namespace

extern "C" {

pxStatus pxSetAllocator(pxDeviceAllocFn alloc, pxDeviceFreeFn free, void* user)
{
    if ((alloc == nullptr) != (free == nullptr))
        return fail(PX_E_INVALID, "pxSetAllocator: give both alloc and free, or neither");
    return guarded([&]() -> pxStatus {
        // blocks kept from earlier solves were made by the previous allocator
        pxs::BlockCache::get().release();
        px::set_allocator(alloc, free, user);
        return PX_OK;
    });
}

pxStatus pxReleaseCache(void)
{
    return guarded([&]() -> pxStatus {
        pxs::BlockCache::get().release();
        return PX_OK;
    });
}

void pxDefaultSolveOptions(pxSolveOptions* o)
{
    if (!o) return;
    o->precision = PX_FP64;
    o->restart_m = 100;
    o->rel_tol = 1e-8;
    o->max_cycles = 400;
    o->max_block_cols = 0;
    o->inner_reduction = 1e-5;
    o->timings = 0;
    o->stall_cycles = 8;
    o->max_restart_m = 200;
    o->block_cols = 0;
    o->ortho = PX_ORTHO_DCGS2;
    o->graph_steps = 8;
    o->t_apply = PX_TAPPLY_AUTO;
    o->shifted = 2;
    o->shifted_max_steps = 2000;
}

const char* pxLastError(void) { return g_err.c_str(); }

namespace {

// Drude weight n/m* of a material (graphene: E_F / (pi t_g)); the checks of
// pxCreateStructure on its parameters.
double drude_of(const pxMaterial& m)
{
    return m.fermi_energy_ev > 0.0 ? (m.fermi_energy_ev / EV_PER_HARTREE) / (PI * m.sheet_thickness)
                                   : m.density / m.eff_mass;
}

pxStatus check_material(const pxMaterial& m, pxModel model)
{
    const double drude = drude_of(m);
    if (!(m.a_eff > 0) || !(m.r_q > 0) || !(m.tau > 0) || !(drude > 0) || !std::isfinite(drude) || !(m.r0_ang > 0) ||
        !(m.cutoff_ang > 0) || !(m.fermi_s > 0) || !std::isfinite(m.fermi_d))
        return fail(PX_E_INVALID, "invalid material parameters");
    if (model == PX_WFQFMU && !(m.r_mu > 0)) return fail(PX_E_INVALID, "r_mu must be > 0 for the dipole model");
    return PX_OK;
}

pxStatus create_impl(pxModel model, int64_t n_atoms, const double* xyz_ang, const uint8_t* types,
                     const pxMaterial* mat, const pxMaterial* mat_b, void* hip_stream, pxStructure* out)
{
    g_err.clear();
    if (!out || !xyz_ang || !mat) return fail(PX_E_INVALID, "null argument");
    *out = nullptr;
    if (model != PX_WFQ && model != PX_WFQFMU)
        return fail(PX_E_INVALID, model == PX_BEM ? "a BEM structure is made with pxCreateBem" : "unknown model");
    if (n_atoms < 1 || n_atoms > (int64_t)1 << 28) return fail(PX_E_INVALID, "n_atoms out of range");
    for (int64_t i = 0; i < n_atoms; ++i)
        if (!finite3(xyz_ang + 3 * i)) return fail(PX_E_INVALID, "non-finite coordinate");
    const pxMaterial& m = *mat;
    if (check_material(m, model) != PX_OK) return PX_E_INVALID;
    if (types) {
        if (check_material(*mat_b, model) != PX_OK) return PX_E_INVALID;
        if (mat_b->r_q != m.r_q || (model == PX_WFQFMU && mat_b->r_mu != m.r_mu))
            return fail(PX_E_INVALID, "the two materials must share r_q (and r_mu)");
        for (int64_t i = 0; i < n_atoms; ++i)
            if (types[i] > 1) return fail(PX_E_INVALID, "atom types must be 0 or 1");
    }
    return guarded([&]() -> pxStatus {
        int dev = 0;
        hipDeviceProp_t prop;
        HC(hipGetDevice(&dev));
        HC(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(PX_E_DEVICE, std::string("built for gfx950, device is ") + prop.gcnArchName);
        auto* s = new pxStructure_t();
        s->model = model;
        s->mat = m;
        s->drude = drude_of(m);
        if (types) {
            s->het = true;
            s->mat_b = *mat_b;
            s->drude_b = drude_of(*mat_b);
        }
        s->st = static_cast<hipStream_t>(hip_stream);
        s->g.model = (int)model;
        s->g.n = n_atoms;
        s->g.np = ((n_atoms + px::ATOM_PAD - 1) / px::ATOM_PAD) * px::ATOM_PAD;
        s->g.nu = model == PX_WFQFMU ? 4 * n_atoms : n_atoms;
        s->g.nup = model == PX_WFQFMU ? 4 * s->g.np : s->g.np;
        s->g.r_q = m.r_q;
        s->g.r_mu = m.r_mu;
        std::vector<double> xb(3 * n_atoms);
        for (int64_t i = 0; i < 3 * n_atoms; ++i) xb[i] = xyz_ang[i] / ANG_PER_BOHR;
        int bad = 0;
        hipError_t e = px::build_geometry(s->g, xb.data(), m.cutoff_ang / ANG_PER_BOHR, m, m.r0_ang / ANG_PER_BOHR,
                                          s->perm, &bad, s->st, types, types ? mat_b : nullptr);
        if (e != hipSuccess) {
            delete s;
            throw HipError{e, "build_geometry"};
        }
        if (bad) {
            delete s;
            return fail(PX_E_INVALID, "two atoms closer than 1e-6 Angstrom");
        }
        try {
            // the omegaFQ narrow FP64 T-apply takes its near field from a list built here
            HC(px::ensure_near_f64(s->g, s->st));
            s->d_perm = dalloc<int32_t>(n_atoms);
            HC(hipMemcpyAsync(s->d_perm, s->perm.data(), sizeof(int32_t) * n_atoms, hipMemcpyHostToDevice, s->st));
            HC(hipStreamSynchronize(s->st));
        } catch (...) {
            delete s;
            throw;
        }
        *out = s;
        return PX_OK;
    });
}

}  // namespace

pxStatus pxCreateStructure(pxModel model, int64_t n_atoms, const double* xyz_ang, const pxMaterial* mat,
                           void* hip_stream, pxStructure* out)
{
    return create_impl(model, n_atoms, xyz_ang, nullptr, mat, nullptr, hip_stream, out);
}

pxStatus pxCreateStructureHetero(pxModel model, int64_t n_atoms, const double* xyz_ang, const uint8_t* types,
                                 const pxMaterial* mat_a, const pxMaterial* mat_b, void* hip_stream,
                                 pxStructure* out)
{
    if (!types || !mat_b) {
        g_err.clear();
        if (out) *out = nullptr;
        return fail(PX_E_INVALID, "null argument");
    }
    return create_impl(model, n_atoms, xyz_ang, types, mat_a, mat_b, hip_stream, out);
}

namespace {

pxStatus create_bem(int64_t n_tess, const double* cen_ang, const double* normals, const double* area_ang2,
                    double r_enc_ang, const double* eps_env, void* hip_stream, bool ief, pxStructure* out)
{
    g_err.clear();
    if (!out || !cen_ang || !normals || !area_ang2) return fail(PX_E_INVALID, "null argument");
    *out = nullptr;
    if (n_tess < 1 || n_tess > (int64_t)1 << 26) return fail(PX_E_INVALID, "n_tess out of range");
    if (!(r_enc_ang > 0) || !std::isfinite(r_enc_ang)) return fail(PX_E_INVALID, "r_enc must be > 0");
    const double e1r = eps_env ? eps_env[0] : 1.0, e1i = eps_env ? eps_env[1] : 0.0;
    if (!std::isfinite(e1r) || !std::isfinite(e1i)) return fail(PX_E_INVALID, "eps_env must be finite");
    for (int64_t i = 0; i < n_tess; ++i) {
        const double* v = normals + 3 * i;
        const double l2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (!finite3(cen_ang + 3 * i) || !finite3(v) || !(l2 > 0) || !std::isfinite(l2))
            return fail(PX_E_INVALID, "non-finite barycentre or normal, or a zero normal");
        if (!(area_ang2[i] > 0) || !std::isfinite(area_ang2[i])) return fail(PX_E_INVALID, "tessera areas must be > 0");
    }
    return guarded([&]() -> pxStatus {
        int dev = 0;
        hipDeviceProp_t prop;
        HC(hipGetDevice(&dev));
        HC(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(PX_E_DEVICE, std::string("built for gfx950, device is ") + prop.gcnArchName);
        std::unique_ptr<pxStructure_t> s(new pxStructure_t());
        s->model = PX_BEM;
        s->eps1[0] = e1r;
        s->eps1[1] = e1i;
        s->st = static_cast<hipStream_t>(hip_stream);
        s->g.model = 0;
        s->g.n = n_tess;
        s->g.np = ((n_tess + px::ATOM_PAD - 1) / px::ATOM_PAD) * px::ATOM_PAD;
        s->g.nu = n_tess;
        s->g.nup = s->g.np;
        std::vector<double> cb(3 * n_tess), ab(n_tess);
        for (int64_t i = 0; i < 3 * n_tess; ++i) cb[i] = cen_ang[i] / ANG_PER_BOHR;
        for (int64_t i = 0; i < n_tess; ++i) ab[i] = area_ang2[i] / (ANG_PER_BOHR * ANG_PER_BOHR);
        int cg = 0;
        HC(px::build_bem_geometry(s->g, cb.data(), normals, ab.data(), r_enc_ang / ANG_PER_BOHR, ief, s->st, &cg));
        if (cg == 2) return fail(PX_E_INVALID, "S A^-1 is not positive definite on this mesh");
        if (cg == 1) return fail(PX_E_NOTCONV, "the single-layer solve for the dipole weights did not converge");
        s->perm.resize(n_tess);
        for (int64_t i = 0; i < n_tess; ++i) s->perm[i] = (int32_t)i;
        s->d_perm = dalloc<int32_t>(n_tess);
        HC(hipMemcpyAsync(s->d_perm, s->perm.data(), sizeof(int32_t) * n_tess, hipMemcpyHostToDevice, s->st));
        HC(hipStreamSynchronize(s->st));
        *out = s.release();
        return PX_OK;
    });
}

}  // namespace

pxStatus pxCreateBem(int64_t n_tess, const double* cen_ang, const double* normals, const double* area_ang2,
                     double r_enc_ang, const double* eps_env, void* hip_stream, pxStructure* out)
{
    return create_bem(n_tess, cen_ang, normals, area_ang2, r_enc_ang, eps_env, hip_stream, false, out);
}

pxStatus pxCreateBemIefpcm(int64_t n_tess, const double* cen_ang, const double* normals, const double* area_ang2,
                           double r_enc_ang, const double* eps_env, void* hip_stream, pxStructure* out)
{
    return create_bem(n_tess, cen_ang, normals, area_ang2, r_enc_ang, eps_env, hip_stream, true, out);
}

pxStatus pxSetFrequencies(pxStructure s, int32_t n_omega, const double* omega_ev, uint32_t pol_mask, double e0_au,
                          const double* alpha_ib)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !omega_ev) return fail(PX_E_INVALID, "null argument");
    if (n_omega < 1) return fail(PX_E_INVALID, "n_omega must be >= 1");
    if ((pol_mask & 7u) == 0 || (pol_mask & ~7u)) return fail(PX_E_INVALID, "pol_mask must be a non-empty subset of 0b111");
    if (!(e0_au > 0) || !std::isfinite(e0_au)) return fail(PX_E_INVALID, "e0 must be > 0");
    for (int w = 0; w < n_omega; ++w)
        if (!(omega_ev[w] > 0) || !std::isfinite(omega_ev[w])) return fail(PX_E_INVALID, "frequencies must be > 0");
    if (s->model == PX_WFQFMU) {
        if (!alpha_ib) return fail(PX_E_INVALID, "alpha_ib required for the dipole model");
        const int na = s->het ? 2 * n_omega : n_omega;
        for (int w = 0; w < na; ++w)
            if (!std::isfinite(alpha_ib[2 * w]) || !std::isfinite(alpha_ib[2 * w + 1]) ||
                (alpha_ib[2 * w] == 0.0 && alpha_ib[2 * w + 1] == 0.0))
                return fail(PX_E_INVALID, "alpha_ib must be finite and non-zero");
    }
    if (s->model == PX_BEM) {
        // eps2(w): the metal permittivity per frequency
        if (!alpha_ib) return fail(PX_E_INVALID, "a BEM structure needs eps2(w) (alpha_ib argument)");
        for (int w = 0; w < n_omega; ++w)
            if (!std::isfinite(alpha_ib[2 * w]) || !std::isfinite(alpha_ib[2 * w + 1]) ||
                (alpha_ib[2 * w] == s->eps1[0] && alpha_ib[2 * w + 1] == s->eps1[1]))
                return fail(PX_E_INVALID, "eps2 must be finite and differ from the medium's eps1");
    }
    return guarded([&]() -> pxStatus {
        s->solved = false;
        s->n_omega = n_omega;
        s->pol_mask = pol_mask;
        s->npol = __builtin_popcount(pol_mask);
        s->ncol = n_omega * s->npol;
        s->ldg = ((s->ncol + px::COL_PAD - 1) / px::COL_PAD) * px::COL_PAD;
        s->e0 = e0_au;
        s->omega_au.resize(n_omega);
        for (int w = 0; w < n_omega; ++w) s->omega_au[w] = omega_ev[w] / EV_PER_HARTREE;
        const int naib = s->het ? 4 : 2;
        s->aib.assign((size_t)naib * n_omega, 0.0);
        if (s->model != PX_WFQ) std::copy(alpha_ib, alpha_ib + naib * n_omega, s->aib.begin());
        s->col_pol.clear();
        for (int w = 0; w < n_omega; ++w)
            for (int l = 0; l < 3; ++l)
                if (pol_mask & (1u << l)) s->col_pol.push_back(l);
        dfree(s->d_col_pol);
        dfree(s->d_omega);
        dfree(s->x);
        dfree(s->b);
        s->d_col_pol = nullptr;
        s->d_omega = nullptr;
        s->x = s->b = nullptr;
        s->d_col_pol = dalloc<int32_t>(s->ncol);
        s->d_omega = dalloc<double>(n_omega);
        s->x = dalloc<double2>((size_t)s->g.nup * s->ldg);
        s->b = dalloc<double2>((size_t)s->g.nup * s->ldg);
        HC(hipMemcpyAsync(s->d_col_pol, s->col_pol.data(), sizeof(int32_t) * s->ncol, hipMemcpyHostToDevice, s->st));
        HC(hipMemcpyAsync(s->d_omega, s->omega_au.data(), sizeof(double) * n_omega, hipMemcpyHostToDevice, s->st));
        HC(hipStreamSynchronize(s->st));
        return PX_OK;
    });
}

pxStatus pxSolveSpectrum(pxStructure s, const pxSolveOptions* opt)
{
    g_err.clear();
    if (!s) return fail(PX_E_INVALID, "null structure");
    PX_SETTLE(s);
    pxSolveOptions o;
    pxDefaultSolveOptions(&o);
    if (opt) o = *opt;
    return guarded([&]() -> pxStatus { return solve_impl(s, o); });
}

pxStatus pxSolveSpectrumAsync(pxStructure s, const pxSolveOptions* opt)
{
    g_err.clear();
    if (!s) return fail(PX_E_INVALID, "null structure");
    PX_SETTLE(s);
    pxSolveOptions o;
    pxDefaultSolveOptions(&o);
    if (opt) o = *opt;
    if (s->ncol == 0) return fail(PX_E_STATE, "pxSolveSpectrumAsync: call pxSetFrequencies first");
    if (check_options(o) != PX_OK) return PX_E_INVALID;
    return guarded([&]() -> pxStatus {
        s->pending.reset(new AsyncSolve(s, o));
        advance_pending(s, false);
        return PX_OK;
    });
}

pxStatus pxSolveProgress(pxStructure s, int32_t* done)
{
    g_err.clear();
    if (!s || !done) return fail(PX_E_INVALID, "null argument");
    *done = 1;
    if (!s->pending) return PX_OK;
    return guarded([&]() -> pxStatus {
        *done = advance_pending(s, false) ? 1 : 0;
        return PX_OK;
    });
}

pxStatus pxSolveWait(pxStructure s)
{
    g_err.clear();
    if (!s) return fail(PX_E_INVALID, "null structure");
    PX_SETTLE(s);
    if (s->last_status != PX_OK) return fail(s->last_status, s->last_error);
    return PX_OK;
}

pxStatus pxSolveBatch(const pxStructure* ss, int32_t n, const pxSolveOptions* opt)
{
    g_err.clear();
    if (ss)
        for (int32_t k = 0; k < n; ++k)
            if (ss[k]) PX_SETTLE(ss[k]);
    if (!ss || n < 0) return fail(PX_E_INVALID, "null argument");
    if (n == 0) return PX_OK;
    pxSolveOptions o;
    pxDefaultSolveOptions(&o);
    if (opt) o = *opt;
    if (check_options(o) != PX_OK) return PX_E_INVALID;
    for (int32_t k = 0; k < n; ++k) {
        if (!ss[k]) return fail(PX_E_INVALID, "null structure");
        if (ss[k]->ncol == 0) return fail(PX_E_STATE, "pxSolveBatch: every structure needs pxSetFrequencies");
        if (ss[k]->st != ss[0]->st) return fail(PX_E_INVALID, "pxSolveBatch: structures use different streams");
        if (ss[k]->het) return fail(PX_E_INVALID, "pxSolveBatch: two-type structures are solved with pxSolveSpectrum");
        if (ss[k]->model == PX_BEM && o.shifted < 1)
            return fail(PX_E_INVALID, "pxSolveBatch: BEM structures are solved whole (shifted >= 1)");
        for (int32_t j = 0; j < k; ++j)
            if (ss[j] == ss[k]) return fail(PX_E_INVALID, "pxSolveBatch: a structure is listed twice");
    }
    return guarded([&]() -> pxStatus {
        auto t0 = std::chrono::steady_clock::now();
        const int Bc = o.block_cols > 0 ? o.block_cols : 64;
        const int m_max = std::max(o.restart_m, o.max_restart_m);
        hipStream_t st = ss[0]->st;
        // whole solves (several at once, each on a stream of its own) beside
        // the stacked engine that takes the small structures
        std::vector<pxStructure_t*> pooled, stacked;
        for (int32_t k = 0; k < n; ++k) {
            ss[k]->last_status = PX_E_STATE;
            ss[k]->last_error = "not solved";
            (pooled_solve(ss[k], o) ? pooled : stacked).push_back(ss[k]);
        }
        std::unique_ptr<Engine> eng;
        std::deque<pxStructure_t*> queue;
        if (!stacked.empty()) {
            int64_t rows = 0;
            int nseg = 0;
            for (pxStructure_t* p : stacked) {
                nseg += (p->ncol + Bc - 1) / Bc;
                rows += (int64_t)((p->ncol + Bc - 1) / Bc) * p->g.nup;
            }
            size_t free_b = 0, total_b = 0;
            HC(hipMemGetInfo(&free_b, &total_b));
            const int64_t fit = (int64_t)(0.8 * (double)free_b / (double)Engine::bytes_per_row(Bc, m_max));
            const int64_t cap = std::min(rows, fit);
            int64_t biggest = 0;
            for (pxStructure_t* p : stacked)
                biggest = std::max<int64_t>(biggest, (int64_t)((p->ncol + Bc - 1) / Bc) * p->g.nup);
            if (cap < biggest) return fail(PX_E_OOM, "pxSolveBatch: the largest structure does not fit in device memory");
            eng.reset(new Engine(st, Bc, o, std::max(cap, biggest), nseg));
            for (pxStructure_t* p : stacked) {
                for (double& v : p->ms) v = 0.0;
                for (int64_t& v : p->counts) v = 0;
                prepare_solve(p);
                queue.push_back(p);
            }
        }
        SolveDriver drv(o);
        std::deque<pxStructure_t*> waiting(pooled.begin(), pooled.end());
        auto engine_work = [&]() { return eng && (!queue.empty() || !eng->idle()); };
        while (!waiting.empty() || drv.busy() || engine_work()) {
            while (drv.has_room() && !waiting.empty()) {
                drv.start(waiting.front());
                waiting.pop_front();
            }
            const bool ew = engine_work();
            (void)drv.turn(!ew);
            if (ew) {
                while (!queue.empty() && eng->can_admit(queue.front())) {
                    eng->admit(queue.front());
                    queue.pop_front();
                }
                for (pxStructure_t* p : eng->cycle()) set_engine_status(p, o);
                (void)drv.turn(false);
            }
        }
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (pxStructure_t* p : stacked) {
            p->ms[0] = ms;
            p->ms[5] = ms;
            p->counts[0] = eng->stats().tapply_f32;
            p->counts[3] = eng->stats().tapply_f64 + eng->stats().residuals;
        }
        // the worst status: a device or memory failure before a convergence shortfall
        pxStatus worst = PX_OK;
        std::string msg;
        for (int32_t k = 0; k < n; ++k) {
            const pxStatus sk = ss[k]->last_status;
            if (sk == PX_OK) continue;
            if (worst == PX_OK || (worst == PX_E_NOTCONV && sk != PX_E_NOTCONV)) {
                worst = sk;
                msg = "structure " + std::to_string(k) + ": " + ss[k]->last_error;
            }
        }
        if (worst != PX_OK) return fail(worst, msg);
        return PX_OK;
    });
}

pxStatus pxGetCharges(pxStructure s, int32_t i_omega, int32_t pol, double* q, double* mu)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !q) return fail(PX_E_INVALID, "null argument");
    if (!s->solved) return fail(PX_E_STATE, "no solved spectrum");
    if (i_omega < 0 || i_omega >= s->n_omega || pol < 0 || pol > 2 || !(s->pol_mask & (1u << pol)))
        return fail(PX_E_INVALID, "column not in the solved set");
    int p = 0;
    for (int l = 0; l < pol; ++l)
        if (s->pol_mask & (1u << l)) ++p;
    const int col = i_omega * s->npol + p;
    if (s->g.bem_ief) {
        // the charges of an IEFPCM column: (S A^-1) q = y, the real and
        // imaginary parts as two real columns
        return guarded([&]() -> pxStatus {
            const int64_t np = s->g.np;
            double* qd = dalloc<double>((size_t)2 * np);
            int cg = 0;
            HC(px::bem_single_layer_solve(s->g, reinterpret_cast<const double*>(s->x) + 2 * col, 2 * s->ldg, 2, qd,
                                          kChargeSolveTol, kChargeSolveMaxIter, s->st, &cg, nullptr, nullptr));
            HC(hipMemcpyAsync(q, qd, sizeof(double2) * s->g.n, hipMemcpyDeviceToHost, s->st));
            HC(hipStreamSynchronize(s->st));
            dfree(qd);
            if (cg == 2) return fail(PX_E_INVALID, "S A^-1 is not positive definite on this mesh");
            if (cg == 1) return fail(PX_E_NOTCONV, "the single-layer solve for the charges did not converge");
            return PX_OK;
        });
    }
    return guarded([&]() -> pxStatus {
        const int ncomp = s->model == PX_WFQFMU ? 4 : 1;
        double2* d = dalloc<double2>((size_t)ncomp * s->g.n);
        px::unpermute(s->g, s->x, s->ldg, col, s->d_perm, d, s->st);
        std::vector<double> h((size_t)2 * ncomp * s->g.n);
        HC(hipMemcpyAsync(h.data(), d, sizeof(double2) * ncomp * s->g.n, hipMemcpyDeviceToHost, s->st));
        HC(hipStreamSynchronize(s->st));
        dfree(d);
        std::copy(h.begin(), h.begin() + 2 * s->g.n, q);
        if (mu && ncomp == 4) std::copy(h.begin() + 2 * s->g.n, h.end(), mu);
        return PX_OK;
    });
}

// ---- post-processing: field and density at probe points --------------------

namespace {

// Field and density at npts points (Angstrom, host) from the per-atom sources
// src (device, Morton order, np x 2 or np x 8), in batches of 2^20 points.
pxStatus probe_run(pxStructure_t* s, const double* src, int64_t npts, const double* pts_ang, double* field,
                   double* density)
{
    constexpr int64_t kBatch = int64_t(1) << 20;
    s->probe[0] = 0.0;
    s->probe[1] = (double)npts * (double)s->g.n;
    if (npts == 0) return PX_OK;
    for (int64_t t = 0; t < 3 * npts; ++t)
        if (!std::isfinite(pts_ang[t])) return fail(PX_E_INVALID, "probe points must be finite");
    const int64_t nb0 = std::min(npts, kBatch);
    // split counts differ between a full batch and the last one
    const int64_t nlast = npts - (npts - 1) / kBatch * kBatch;
    Scratch sc;
    double4* pts = sc.get<double4>((size_t)nb0);
    double* part = sc.get<double>(std::max(px::probe_part_doubles(s->g, nb0), px::probe_part_doubles(s->g, nlast)));
    void* order = sc.get<uint8_t>(px::probe_order_bytes(nb0));
    double* f_d = sc.get<double>((size_t)nb0 * 6);
    double* r_d = sc.get<double>((size_t)nb0 * 2);
    std::vector<double4> ph((size_t)nb0);
    std::vector<double> fh((size_t)nb0 * 6), rh((size_t)nb0 * 2);
    hipEvent_t ev[2];
    HC(hipEventCreate(&ev[0]));
    HC(hipEventCreate(&ev[1]));
    const double ang = ANG_PER_BOHR;
    for (int64_t b0 = 0; b0 < npts; b0 += kBatch) {
        const int64_t nb = std::min(kBatch, npts - b0);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t t = 0; t < nb; ++t) {
            const double* p = pts_ang + 3 * (b0 + t);
            ph[(size_t)t] = make_double4(p[0] / ang, p[1] / ang, p[2] / ang, 0.0);
            const double v[3] = {ph[(size_t)t].x, ph[(size_t)t].y, ph[(size_t)t].z};
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], v[a]);
                hi[a] = std::max(hi[a], v[a]);
            }
        }
        HC(hipMemcpyAsync(pts, ph.data(), sizeof(double4) * nb, hipMemcpyHostToDevice, s->st));
        HC(hipEventRecord(ev[0], s->st));
        px::probe_field(s->g, src, pts, nb, lo, hi, order, part, f_d, r_d, s->st);
        HC(hipEventRecord(ev[1], s->st));
        HC(hipGetLastError());
        HC(hipMemcpyAsync(fh.data(), f_d, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, s->st));
        HC(hipMemcpyAsync(rh.data(), r_d, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, s->st));
        HC(hipStreamSynchronize(s->st));
        float ms = 0.f;
        HC(hipEventElapsedTime(&ms, ev[0], ev[1]));
        s->probe[0] += ms;
        if (field) std::copy(fh.begin(), fh.begin() + 6 * nb, field + 6 * b0);
        if (density) std::copy(rh.begin(), rh.begin() + 2 * nb, density + 2 * b0);
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return PX_OK;
}

}  // namespace

pxStatus pxInducedField(pxStructure s, int32_t i_omega, int32_t pol, int64_t npts, const double* pts_ang,
                        double* field, double* density)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || npts < 0 || (npts > 0 && !pts_ang)) return fail(PX_E_INVALID, "pxInducedField: invalid argument");
    if (s->model == PX_BEM) return fail(PX_E_INVALID, "pxInducedField: the Gaussian densities are those of the atomistic models");
    if (!s->solved) return fail(PX_E_STATE, "pxInducedField: no solved spectrum");
    if (i_omega < 0 || i_omega >= s->n_omega || pol < 0 || pol > 2 || !(s->pol_mask & (1u << pol)))
        return fail(PX_E_INVALID, "pxInducedField: column not in the solved set");
    int p = 0;
    for (int l = 0; l < pol; ++l)
        if (s->pol_mask & (1u << l)) ++p;
    const int col = i_omega * s->npol + p;
    return guarded([&]() -> pxStatus {
        Scratch sc;
        const int S = s->model == PX_WFQFMU ? 8 : 2;
        double* src = sc.get<double>((size_t)S * s->g.np);
        px::probe_sources(s->g, s->x, s->ldg, col, src, s->st);
        return probe_run(s, src, npts, pts_ang, field, density);
    });
}

pxStatus pxProbeField(pxStructure s, const double* q, const double* mu, int64_t npts, const double* pts_ang,
                      double* field, double* density)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !q || npts < 0 || (npts > 0 && !pts_ang)) return fail(PX_E_INVALID, "pxProbeField: invalid argument");
    if (s->model == PX_BEM) return fail(PX_E_INVALID, "pxProbeField: the Gaussian densities are those of the atomistic models");
    if (mu && s->model != PX_WFQFMU) return fail(PX_E_INVALID, "pxProbeField: dipoles given for an omegaFQ structure");
    return guarded([&]() -> pxStatus {
        const int S = s->model == PX_WFQFMU ? 8 : 2;
        const int64_t n = s->g.n, np = s->g.np;
        std::vector<double> h((size_t)S * np, 0.0);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t o = s->perm[(size_t)i];
            h[(size_t)S * i] = q[2 * o];
            h[(size_t)S * i + 1] = q[2 * o + 1];
            if (mu)
                for (int a = 0; a < 3; ++a) {
                    h[(size_t)S * i + 2 + 2 * a] = mu[2 * (a * n + o)];
                    h[(size_t)S * i + 3 + 2 * a] = mu[2 * (a * n + o) + 1];
                }
        }
        Scratch sc;
        double* src = sc.get<double>((size_t)S * np);
        HC(hipMemcpyAsync(src, h.data(), sizeof(double) * S * np, hipMemcpyHostToDevice, s->st));
        return probe_run(s, src, npts, pts_ang, field, density);
    });
}

pxStatus pxGetProbeStats(pxStructure s, double* out2)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !out2) return fail(PX_E_INVALID, "null argument");
    out2[0] = s->probe[0];
    out2[1] = s->probe[1];
    return PX_OK;
}

pxStatus pxGetSpectrum(pxStructure s, double* alpha, double* sigma_abs)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s) return fail(PX_E_INVALID, "null structure");
    if (!s->solved) return fail(PX_E_STATE, "no solved spectrum");
    if (alpha) std::copy(s->alpha.begin(), s->alpha.end(), alpha);
    if (sigma_abs) std::copy(s->sigma.begin(), s->sigma.end(), sigma_abs);
    return PX_OK;
}

pxStatus pxGetSolveStats(pxStructure s, int32_t* iterations, int32_t* cycles, double* rel_res)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s) return fail(PX_E_INVALID, "null structure");
    if (!s->solved) return fail(PX_E_STATE, "no solved spectrum");
    if (iterations) std::copy(s->iters.begin(), s->iters.end(), iterations);
    if (cycles) std::copy(s->cycles.begin(), s->cycles.end(), cycles);
    if (rel_res) std::copy(s->relres.begin(), s->relres.end(), rel_res);
    return PX_OK;
}

pxStatus pxApplyOperator(pxStructure s, int32_t precision, int32_t ncol, const double* omega_ev,
                         const double* alpha_ib, const double* x, double* y)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !omega_ev || !x || !y) return fail(PX_E_INVALID, "null argument");
    if (ncol < 1) return fail(PX_E_INVALID, "ncol must be >= 1");
    if (precision != PX_FP64 && precision != PX_MIXED) return fail(PX_E_INVALID, "unknown precision");
    if (s->model == PX_WFQFMU && !alpha_ib) return fail(PX_E_INVALID, "alpha_ib required for the dipole model");
    if (s->model == PX_BEM && (!alpha_ib || precision != PX_FP64))
        return fail(PX_E_INVALID, "a BEM structure needs eps2 per column (alpha_ib) and PX_FP64");
    for (int c = 0; c < ncol; ++c)
        if (!(omega_ev[c] > 0)) return fail(PX_E_INVALID, "frequencies must be > 0");
    const int naib = s->het ? 4 : 2;
    return guarded([&]() -> pxStatus {
        const bool mixed = precision == PX_MIXED;
        const int lda = pad_cols(ncol, !mixed);
        ensure_vectors(s, std::max(lda, s->ws.lda_cap));
        Workspace& W = s->ws;
        const int64_t nu = s->g.nu, nup = s->g.nup;
        double2* din = dalloc<double2>((size_t)ncol * nu);
        HC(hipMemcpyAsync(din, x, sizeof(double2) * ncol * nu, hipMemcpyHostToDevice, s->st));
        px::permute_in(s->g, din, ncol, s->d_perm, W.xs, lda, s->st);
        std::vector<double2> zq(lda, make_double2(0, 0)), zm(lda, make_double2(0, 0));
        std::vector<double2> h((size_t)6 * lda, make_double2(0, 0));
        for (int c = 0; c < ncol; ++c) {
            const double w = omega_ev[c] / EV_PER_HARTREE;
            const double* a = s->model == PX_WFQFMU ? alpha_ib + naib * c : nullptr;
            if (s->het) {
                double2 f[6];
                het_factors(s, w, a, f);
                for (int q = 0; q < 6; ++q) h[(size_t)q * lda + c] = f[q];
                continue;
            }
            double zr, zi;
            if (s->model == PX_BEM) shift_bem_of(s, alpha_ib + 2 * c, zr, zi);
            else shift_q(s->drude, s->mat.tau, w, zr, zi);
            zq[c] = make_double2(zr, zi);
            if (a) {
                shift_mu(a[0], a[1], zr, zi);
                zm[c] = make_double2(zr, zi);
            }
        }
        HC(hipMemcpyAsync(W.zq, zq.data(), sizeof(double2) * lda, hipMemcpyHostToDevice, s->st));
        HC(hipMemcpyAsync(W.zmu, zm.data(), sizeof(double2) * lda, hipMemcpyHostToDevice, s->st));
        HC(hipMemcpyAsync(W.het, h.data(), sizeof(double2) * 6 * lda, hipMemcpyHostToDevice, s->st));
        if (mixed) {
            px::to_f32(W.xs, W.X32, ncol, lda, nup, s->st);
            px::tapply_f32(s->g, W.X32, W.Y32, 2 * lda, 2 * lda, s->st, W.split32);
            sparse_apply(s, W.Y32, true, 2 * lda, W.xs, nullptr, W.w, ncol, lda, 1.0);
        } else {
            px::tapply_f64(s->g, reinterpret_cast<const double*>(W.xs), W.Y64, 2 * lda, 2 * lda, s->st, W.narrow,
                           W.narrow_bytes);
            sparse_apply(s, W.Y64, false, 2 * lda, W.xs, nullptr, W.w, ncol, lda, 1.0);
        }
        const int ncomp = s->model == PX_WFQFMU ? 4 : 1;
        double2* dout = dalloc<double2>((size_t)ncol * nu);
        for (int c = 0; c < ncol; ++c) px::unpermute(s->g, W.w, lda, c, s->d_perm, dout + (size_t)c * nu, s->st);
        (void)ncomp;
        HC(hipMemcpyAsync(y, dout, sizeof(double2) * ncol * nu, hipMemcpyDeviceToHost, s->st));
        HC(hipStreamSynchronize(s->st));
        dfree(din);
        dfree(dout);
        return PX_OK;
    });
}

pxStatus pxApplyOperatorNoAlloc(pxStructure s, int32_t ncol, const double* omega_ev, const double* alpha_ib,
                                const double* x, double* y)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !omega_ev || !x || !y) return fail(PX_E_INVALID, "null argument");
    if (ncol < 1 || ncol > 4) return fail(PX_E_INVALID, "pxApplyOperatorNoAlloc: ncol must be in [1, 4]");
    if (s->model == PX_WFQFMU && !alpha_ib) return fail(PX_E_INVALID, "alpha_ib required for the dipole model");
    if (s->model == PX_BEM && !alpha_ib) return fail(PX_E_INVALID, "a BEM structure needs eps2 per column (alpha_ib)");
    for (int c = 0; c < ncol; ++c)
        if (!(omega_ev[c] > 0) || !std::isfinite(omega_ev[c])) return fail(PX_E_INVALID, "frequencies must be > 0");
    const int naib = s->het ? 4 : 2;
    return guarded([&]() -> pxStatus {
        if (s->model == PX_WFQ && !s->het && !s->g.near_off) return fail(PX_E_STATE, "near-field list missing");
        const int64_t nu = s->g.nu, nup = s->g.nup;
        const int lda = ncol;
        const size_t vec = (size_t)nup * lda;
        // the layout in the scratch array: shifts, permuted columns, T x, the
        // operator's result, the narrow T-apply's split partial sums
        size_t off = 0;
        auto carve = [&off](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) / 256 * 256;
            return o;
        };
        const size_t part_bytes = px::tapply_f64_scratch_bytes(s->g, 2 * lda);
        const size_t o_sh = carve(sizeof(double2) * 8 * lda), o_xs = carve(sizeof(double2) * vec),
                     o_y = carve(sizeof(double) * 2 * vec), o_w = carve(sizeof(double2) * vec),
                     o_part = carve(part_bytes);
        if (off > kNoAllocScratchBytes)
            return fail(PX_E_OOM, "pxApplyOperatorNoAlloc: needs " + std::to_string(off) +
                                      " bytes of scratch, the fixed device array holds " +
                                      std::to_string(kNoAllocScratchBytes));
        char* base = noalloc_scratch();
        double2* zq = reinterpret_cast<double2*>(base + o_sh);
        double2* zm = zq + lda;
        double2* het = zq + 2 * lda;
        double2* xs = reinterpret_cast<double2*>(base + o_xs);
        double* Y64 = reinterpret_cast<double*>(base + o_y);
        double2* w = reinterpret_cast<double2*>(base + o_w);
        double* part = reinterpret_cast<double*>(base + o_part);
        // shifts of every column (host), one copy into the array
        std::vector<double2> h((size_t)8 * lda, make_double2(0, 0));
        for (int c = 0; c < ncol; ++c) {
            const double wv = omega_ev[c] / EV_PER_HARTREE;
            const double* a = s->model == PX_WFQFMU ? alpha_ib + naib * c : nullptr;
            if (s->het) {
                double2 f[6];
                het_factors(s, wv, a, f);
                for (int q = 0; q < 6; ++q) h[(size_t)(2 + q) * lda + c] = f[q];
                continue;
            }
            double zr, zi;
            if (s->model == PX_BEM) shift_bem_of(s, alpha_ib + 2 * c, zr, zi);
            else shift_q(s->drude, s->mat.tau, wv, zr, zi);
            h[c] = make_double2(zr, zi);
            if (a) {
                shift_mu(a[0], a[1], zr, zi);
                h[(size_t)lda + c] = make_double2(zr, zi);
            }
        }
        HC(hipMemcpyAsync(zq, h.data(), sizeof(double2) * 8 * lda, hipMemcpyHostToDevice, s->st));
        px::permute_in(s->g, reinterpret_cast<const double2*>(x), ncol, s->d_perm, xs, lda, s->st);
        px::tapply_f64(s->g, reinterpret_cast<const double*>(xs), Y64, 2 * lda, 2 * lda, s->st, part, part_bytes);
        if (s->het) px::spmm_het(s->g, Y64, false, 2 * lda, xs, het, nullptr, w, ncol, lda, 1.0, s->st);
        else px::spmm_shift(s->g, Y64, false, 2 * lda, xs, zq, zm, nullptr, w, ncol, lda, 1.0, s->st);
        for (int c = 0; c < ncol; ++c)
            px::unpermute(s->g, w, lda, c, s->d_perm, reinterpret_cast<double2*>(y) + (size_t)c * nu, s->st);
        HC(hipGetLastError());
        HC(hipStreamSynchronize(s->st));
        return PX_OK;
    });
}

pxStatus pxGetSize(pxStructure s, int64_t* n_atoms, int64_t* n_unknowns)
{
    g_err.clear();
    if (!s) return fail(PX_E_INVALID, "null structure");
    if (n_atoms) *n_atoms = s->g.n;
    if (n_unknowns) *n_unknowns = s->g.nu;
    return PX_OK;
}

pxStatus pxGetTApplyStats(pxStructure s, int64_t* launches4, double* ms4, double* flop4)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s) return fail(PX_E_INVALID, "null structure");
    if (launches4) std::copy(s->tstats, s->tstats + 4, launches4);
    if (ms4) std::copy(s->tms, s->tms + 4, ms4);
    if (flop4) std::copy(s->tflop, s->tflop + 4, flop4);
    return PX_OK;
}

pxStatus pxGetWork(pxStructure s, double* work3)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !work3) return fail(PX_E_INVALID, "null argument");
    std::copy(s->work, s->work + 3, work3);
    return PX_OK;
}

pxStatus pxGetTimings(pxStructure s, double* ms6, int64_t* counts6)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s) return fail(PX_E_INVALID, "null structure");
    if (ms6) std::copy(s->ms, s->ms + 6, ms6);
    if (counts6) std::copy(s->counts, s->counts + 6, counts6);
    return PX_OK;
}

void pxDestroyStructure(pxStructure s)
{
    if (!s) return;
    // an asynchronous solve in progress is abandoned once the stream is idle
    const hipError_t e = s->st ? hipStreamSynchronize(s->st) : hipDeviceSynchronize();
    s->idle = e == hipSuccess;
    if (s->pending) {
        (void)hipDeviceSynchronize();   // its second stream too
        s->pending.reset();
    }
    delete s;
}

struct pxServer_t {
    pxs::Engine* eng = nullptr;
    std::unique_ptr<SolveDriver> drv;               // whole solves, several at once
    std::deque<pxStructure_t*> queue;               // stacked-engine requests not yet admitted
    std::deque<pxStructure_t*> waiting;             // whole-solve requests not yet admitted
    std::map<pxStructure_t*, double> whole_bytes;   // footprints of the admitted whole solves
    double whole_in_use = 0.0;
    std::deque<pxStructure_t*> done;
    hipStream_t st = nullptr;
    pxSolveOptions o{};
    double budget = 0.0;
    double row_bytes = 0.0;
    double engine_bytes() const { return (double)eng->rows_in_use() * row_bytes; }
};

pxStatus pxServerCreate(double memory_budget_bytes, const pxSolveOptions* opt, void* hip_stream, pxServer* out)
{
    g_err.clear();
    if (!out) return fail(PX_E_INVALID, "null argument");
    *out = nullptr;
    pxSolveOptions o;
    pxDefaultSolveOptions(&o);
    if (opt) o = *opt;
    if (check_options(o) != PX_OK) return PX_E_INVALID;
    if (!(memory_budget_bytes > 0)) return fail(PX_E_INVALID, "memory budget must be > 0");
    return guarded([&]() -> pxStatus {
        const int Bc = o.block_cols > 0 ? o.block_cols : 64;
        const int m_max = std::max(o.restart_m, o.max_restart_m);
        const int64_t rows = (int64_t)(memory_budget_bytes / (double)Engine::bytes_per_row(Bc, m_max));
        if (rows < 256) return fail(PX_E_OOM, "memory budget below one segment");
        std::unique_ptr<pxServer_t> sv(new pxServer_t());
        sv->st = static_cast<hipStream_t>(hip_stream);
        sv->o = o;
        sv->o.block_cols = Bc;
        sv->budget = memory_budget_bytes;
        sv->row_bytes = (double)Engine::bytes_per_row(Bc, m_max);
        sv->eng = new Engine(sv->st, Bc, o, rows, (int)std::max<int64_t>(1, rows / 256));
        sv->drv.reset(new SolveDriver(sv->o));
        *out = sv.release();
        return PX_OK;
    });
}

pxStatus pxServerSubmit(pxServer sv, pxStructure s)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!sv || !s) return fail(PX_E_INVALID, "null argument");
    if (s->ncol == 0) return fail(PX_E_STATE, "pxServerSubmit: call pxSetFrequencies first");
    if (s->st != sv->st) return fail(PX_E_INVALID, "pxServerSubmit: structure uses another stream");
    if (s->het) return fail(PX_E_INVALID, "pxServerSubmit: two-type structures are solved with pxSolveSpectrum");
    if (s->model == PX_BEM && sv->o.shifted < 1)
        return fail(PX_E_INVALID, "pxServerSubmit: BEM structures are solved whole (shifted >= 1)");
    const bool whole = pooled_solve(s, sv->o);
    if (whole ? solve_footprint(s, sv->o) > sv->budget : sv->eng->rows_for(s) > sv->eng->rows_capacity())
        return fail(PX_E_OOM, "pxServerSubmit: the structure can never fit the memory budget");
    return guarded([&]() -> pxStatus {
        s->last_status = PX_E_STATE;
        s->last_error = "queued";
        s->solved = false;
        if (whole) {
            sv->waiting.push_back(s);
            return PX_OK;
        }
        for (double& v : s->ms) v = 0.0;
        for (int64_t& v : s->counts) v = 0;
        prepare_solve(s);
        sv->queue.push_back(s);
        return PX_OK;
    });
}

pxStatus pxServerStep(pxServer sv, pxStructure* finished, int32_t max_finished, int32_t* n_finished)
{
    g_err.clear();
    if (!sv || !n_finished || (max_finished > 0 && !finished)) return fail(PX_E_INVALID, "null argument");
    return guarded([&]() -> pxStatus {
        // admission by HBM footprint, in arrival order within each kind: the
        // stacked rows in use and the whole solves' footprints share the budget
        while (!sv->queue.empty() && sv->eng->can_admit(sv->queue.front()) &&
               (double)(sv->eng->rows_in_use() + sv->eng->rows_for(sv->queue.front())) * sv->row_bytes +
                       sv->whole_in_use <= sv->budget) {
            sv->eng->admit(sv->queue.front());
            sv->queue.pop_front();
        }
        while (!sv->waiting.empty() && sv->drv->has_room()) {
            pxStructure_t* s = sv->waiting.front();
            const double fp = solve_footprint(s, sv->o);
            if (sv->engine_bytes() + sv->whole_in_use + fp > sv->budget) break;
            sv->waiting.pop_front();
            sv->whole_bytes[s] = fp;
            sv->whole_in_use += fp;
            sv->drv->start(s);
        }
        auto take = [&](const std::vector<pxStructure_t*>& fin) {
            for (pxStructure_t* s : fin) {
                auto it = sv->whole_bytes.find(s);
                if (it != sv->whole_bytes.end()) {
                    sv->whole_in_use -= it->second;
                    sv->whole_bytes.erase(it);
                }
                sv->done.push_back(s);
            }
        };
        take(sv->drv->turn(false));
        const bool cycled = !sv->eng->idle();
        if (cycled)
            for (pxStructure_t* s : sv->eng->cycle()) {
                set_engine_status(s, sv->o);
                sv->done.push_back(s);
            }
        // without an engine cycle to run, wait for the device rather than spin
        take(sv->drv->turn(!cycled && sv->done.empty()));
        if (sv->whole_bytes.empty()) sv->whole_in_use = 0.0;
        int32_t k = 0;
        while (k < max_finished && !sv->done.empty()) {
            finished[k++] = sv->done.front();
            sv->done.pop_front();
        }
        *n_finished = k;
        return PX_OK;
    });
}

pxStatus pxServerQuery(pxServer sv, int32_t* n_queued, int32_t* n_active, int64_t* rows_in_use,
                       int64_t* rows_capacity)
{
    g_err.clear();
    if (!sv) return fail(PX_E_INVALID, "null server");
    if (n_queued) *n_queued = (int32_t)(sv->queue.size() + sv->waiting.size());
    if (n_active) *n_active = sv->eng->n_structures() + sv->drv->running();
    if (rows_in_use) *rows_in_use = sv->eng->rows_in_use();
    if (rows_capacity) *rows_capacity = sv->eng->rows_capacity();
    return PX_OK;
}

pxStatus pxServerMemory(pxServer sv, double* bytes_in_use, double* budget_bytes, int32_t* n_whole)
{
    g_err.clear();
    if (!sv) return fail(PX_E_INVALID, "null server");
    if (bytes_in_use) *bytes_in_use = sv->engine_bytes() + sv->whole_in_use;
    if (budget_bytes) *budget_bytes = sv->budget;
    if (n_whole) *n_whole = sv->drv->running();
    return PX_OK;
}

pxStatus pxSolveFootprint(pxStructure s, const pxSolveOptions* opt, double* bytes)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !bytes) return fail(PX_E_INVALID, "null argument");
    if (s->ncol == 0) return fail(PX_E_STATE, "pxSolveFootprint: call pxSetFrequencies first");
    pxSolveOptions o;
    pxDefaultSolveOptions(&o);
    if (opt) o = *opt;
    if (check_options(o) != PX_OK) return PX_E_INVALID;
    *bytes = solve_footprint(s, o);
    return PX_OK;
}

pxStatus pxGetSolveStatus(pxStructure s, int32_t* status, char* message, int32_t message_len)
{
    g_err.clear();
    if (s) PX_SETTLE(s);
    if (!s || !status) return fail(PX_E_INVALID, "null argument");
    *status = (int32_t)s->last_status;
    if (message && message_len > 0) {
        const size_t n = std::min<size_t>((size_t)message_len - 1, s->last_error.size());
        std::memcpy(message, s->last_error.data(), n);
        message[n] = '\0';
    }
    return PX_OK;
}

void pxServerDestroy(pxServer sv)
{
    if (!sv) return;
    sv->drv.reset();   // waits for the running whole solves' streams
    if (sv->st) (void)hipStreamSynchronize(sv->st);
    else (void)hipDeviceSynchronize();
    delete sv->eng;
    delete sv;
}

}  // extern "C"

