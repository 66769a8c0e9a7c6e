// Internal state shared by the C ABI entry points (px_api.cpp) and the
// stacked multi-structure engine (px_engine.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "plasmonx.h"
#include "px_internal.h"

namespace pxs {

constexpr double ANG_PER_BOHR = 0.529177210903;   // CODATA 2018
constexpr double EV_PER_HARTREE = 27.211386245988;
constexpr double PI = 3.14159265358979323846;
// The solver works on Eq. (wfqfmu-system) with its dipole rows multiplied by
// -1 (same solution, same residual norms); see k_spmm_shift.
constexpr double SOLVER_MU_SIGN = -1.0;

pxStatus fail(pxStatus st, const std::string& msg);

struct HipError {
    hipError_t e;
    const char* where;
};

inline void hcheck(hipError_t e, const char* where)
{
    if (e != hipSuccess) throw HipError{e, where};
}

#define HC(x) pxs::hcheck((x), #x)

template <typename T>
T* dalloc(size_t count)
{
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw HipError{e, "hipMalloc"};
    return static_cast<T*>(p);
}

inline void dfree(void* p)
{
    if (p) (void)hipFree(p);
}

struct Workspace {
    int lda_cap = 0, m_cap = 0;
    int64_t nup = 0;
    double2 *V = nullptr, *w = nullptr, *xs = nullptr, *rs = nullptr, *bs = nullptr, *tmp = nullptr;
    float *X32 = nullptr, *Y32 = nullptr;
    double* Y64 = nullptr;
    double2* partial = nullptr;
    double* npart = nullptr;
    double2 *h1 = nullptr, *h2 = nullptr, *R = nullptr, *sn = nullptr, *gv = nullptr, *y = nullptr;
    double2 *H = nullptr, *G = nullptr, *coefQ = nullptr, *coefV = nullptr, *aux = nullptr;   // delayed reorth.
    double *cs = nullptr, *nrm = nullptr, *target = nullptr;
    int32_t *done = nullptr, *steps = nullptr, *map = nullptr;
    double2 *zq = nullptr, *zmu = nullptr;
    double* narrow = nullptr;
    size_t narrow_bytes = 0;
    float* split32 = nullptr;

    void release()
    {
        void* ps[] = {V, w, xs, rs, bs, tmp, X32, Y32, Y64, partial, npart, h1, h2, R, H, G, coefQ, coefV, aux, sn, gv, y, cs, nrm, target,
                      done, steps, map, zq, zmu, narrow, split32};
        for (void* p : ps) dfree(p);
        *this = Workspace();
    }
};

// z_q(omega) of Eq. (z_q_wfq) with the Drude weight n/m* (graphene: E_F/(pi t_g)), omega in Hartree
void shift_q(double drude, double tau, double w, double& zr, double& zi);
// Eq. (z-mu): z_mu = -1 / alpha_IB
void shift_mu(double ar, double ai, double& zr, double& zi);

}  // namespace pxs

struct pxStructure_t {
    px::Geometry g;
    pxModel model = PX_WFQ;
    pxMaterial mat{};
    double drude = 0.0;
    hipStream_t st = nullptr;
    std::vector<int32_t> perm;
    int32_t* d_perm = nullptr;
    // frequencies and columns (frequency-major: column = w * npol + p)
    int n_omega = 0, npol = 0, ncol = 0, ldg = 0;
    std::vector<double> omega_au;
    std::vector<double> aib;   // 2 * n_omega
    std::vector<int32_t> col_pol;
    uint32_t pol_mask = 0;
    double e0 = 0.0;
    int32_t* d_col_pol = nullptr;
    double* d_omega = nullptr;
    double2* x = nullptr;   // [nup][ldg]
    double2* b = nullptr;
    std::vector<double> bnorm;
    // results
    bool solved = false;
    std::vector<int32_t> iters, cycles, stall;
    std::vector<double> relres, alpha, sigma;
    // workspace and timings
    pxs::Workspace ws;
    // ms: total, T-apply FP32, T-apply FP64 inside cycles, sparse apply, Arnoldi+Givens, rest
    double ms[6] = {0, 0, 0, 0, 0, 0};
    // counts: FP32 T-apply launches, padded real columns, algorithmic real
    // columns; the same three for the FP64 T-apply (cycles and residuals)
    int64_t counts[6] = {0, 0, 0, 0, 0, 0};
    double work[3] = {0, 0, 0};   // algorithmic FP32 FLOP, FP64 FLOP, HBM bytes of the last solve

    ~pxStructure_t()
    {
        ws.release();
        void* ps[] = {g.xyz32, g.xyz64, g.glo, g.ghi, g.row_ptr, g.col, g.val, d_perm, d_col_pol, d_omega, x, b};
        for (void* p : ps) pxs::dfree(p);
    }
};

namespace pxs {
// Right-hand sides, x = 0, ||b|| and fresh statistics for every column of s.
void prepare_solve(pxStructure_t* s);
// Dipole moments, polarizability and cross sections from s->x; marks s solved.
void finish_solve(pxStructure_t* s);
}  // namespace pxs
