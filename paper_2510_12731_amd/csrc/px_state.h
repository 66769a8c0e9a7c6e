// Internal state shared by the C ABI entry points (px_api.cpp) and the
// stacked multi-structure engine (px_engine.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
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
    hipError_t e = px::dev_malloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw HipError{e, "device allocation"};
    return static_cast<T*>(p);
}

inline void dfree(void* p)
{
    if (p) px::dev_free(p);
}

// Device blocks kept for the next allocation of a similar size (the shared
// phases' scratch and the stored T: hipMalloc and hipFree of several GB cost
// milliseconds of host time per solve).  A block is given back only once no
// stream uses it any more (its user has synchronised); a block of at least
// kMinBytes serves a request of at least half its size on the same device;
// at most kCacheBytes are kept, and a failed allocation releases them and
// tries again.  The blocks are never freed at process exit.  With a caller
// allocator installed nothing is kept: the caller's allocator caches instead.
// Blocks come from px::dev_malloc and go back through px::dev_free.
class BlockCache {
  public:
    static constexpr size_t kMinBytes = size_t(1) << 24, kCacheBytes = size_t(24) << 30;

    static BlockCache& get()
    {
        static BlockCache* c = new BlockCache();
        return *c;
    }

    void* take(size_t bytes)
    {
        if (bytes == 0) bytes = 1;
        int dev = 0;
        hcheck(hipGetDevice(&dev), "hipGetDevice");
        if (!px::caller_allocator()) {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto it = blocks_.lower_bound(bytes); it != blocks_.end() && it->first <= 2 * bytes; ++it)
                if (it->second.dev == dev) {
                    void* p = it->second.p;
                    live_[p] = Live{it->first, dev};
                    held_ -= it->first;
                    blocks_.erase(it);
                    return p;
                }
        }
        void* p = nullptr;
        hipError_t e = px::dev_malloc(&p, bytes);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            release();
            e = px::dev_malloc(&p, bytes);
        }
        if (e != hipSuccess) throw HipError{e, "device allocation"};
        std::lock_guard<std::mutex> lk(mu_);
        live_[p] = Live{bytes, dev};
        return p;
    }

    // a take(bytes) on this device would be served from the kept blocks
    bool can_serve(size_t bytes)
    {
        if (bytes == 0) bytes = 1;
        if (px::caller_allocator()) return false;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return false;
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = blocks_.lower_bound(bytes); it != blocks_.end() && it->first <= 2 * bytes; ++it)
            if (it->second.dev == dev) return true;
        return false;
    }

    // p came from take() and no stream uses it any more
    void give(void* p)
    {
        if (!p) return;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = live_.find(p);
            if (it != live_.end()) {
                const Live l = it->second;
                live_.erase(it);
                if (l.bytes >= kMinBytes && held_ + l.bytes <= kCacheBytes && !px::caller_allocator()) {
                    blocks_.emplace(l.bytes, Block{p, l.dev});
                    held_ += l.bytes;
                    return;
                }
            }
        }
        px::dev_free(p);
    }

    // p came from take() but may still be in use: freed (dev_free waits for the device)
    void drop(void* p)
    {
        if (!p) return;
        {
            std::lock_guard<std::mutex> lk(mu_);
            live_.erase(p);
        }
        px::dev_free(p);
    }

    void release()
    {
        std::multimap<size_t, Block> b;
        {
            std::lock_guard<std::mutex> lk(mu_);
            b.swap(blocks_);
            held_ = 0;
        }
        for (auto& e : b) px::dev_free(e.second.p);
    }

  private:
    struct Block {
        void* p;
        int dev;
    };
    struct Live {
        size_t bytes;
        int dev;
    };
    std::mutex mu_;
    std::multimap<size_t, Block> blocks_;
    std::unordered_map<void*, Live> live_;
    size_t held_ = 0;
};

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
    double2* het = nullptr;   // two-type shifts and factors, [6][lda]
    double* narrow = nullptr;
    size_t narrow_bytes = 0;
    float* split32 = nullptr;
    float* sk32 = nullptr;   // stream-K tiles of the stored FP32 apply (allocated with the stored T)

    void release()
    {
        void* ps[] = {V, w, xs, rs, bs, tmp, X32, Y32, Y64, partial, npart, h1, h2, R, H, G, coefQ, coefV, aux, sn, gv, y, cs, nrm, target,
                      done, steps, map, zq, zmu, het, narrow, split32, sk32};
        for (void* p : ps) dfree(p);
        *this = Workspace();
    }
};

// Lagged host polling of the device stop flag that every kernel of an Arnoldi
// step reads: the host enqueues steps ahead of the device and only looks at
// the flag published after step k - lag, so it never waits for the step it
// just enqueued, and the steps enqueued after the last column finished cost
// one near-empty launch per kernel.
class StepSync {
  public:
    StepSync() = default;
    StepSync(const StepSync&) = delete;
    StepSync& operator=(const StepSync&) = delete;
    ~StepSync() { release(); }
    void ensure(int steps)
    {
        if (steps <= cap_) return;
        release();
        d_flag_ = dalloc<int32_t>(1);
        if (hipHostMalloc((void**)&h_flags_, sizeof(int32_t) * steps, hipHostMallocDefault) != hipSuccess)
            throw HipError{hipErrorOutOfMemory, "hipHostMalloc"};
        ev_.resize(steps);
        for (auto& e : ev_) HC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        cap_ = steps;
    }
    int32_t* flag() const { return d_flag_; }
    // device-side reset, a kernel (so that the sequence can be graph-captured)
    void reset(hipStream_t st) { px::fill_zero(d_flag_, sizeof(int32_t), st); }
    void publish(int k, hipStream_t st)
    {
        HC(hipMemcpyAsync(h_flags_ + k, d_flag_, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HC(hipEventRecord(ev_[k], st));
    }
    // true once the flag published as k has reached the host (never waits)
    bool ready(int k)
    {
        const hipError_t e = hipEventQuery(ev_[k]);
        if (e == hipSuccess) return true;
        if (e == hipErrorNotReady) return false;
        throw HipError{e, "hipEventQuery"};
    }
    bool stopped(int k)
    {
        HC(hipEventSynchronize(ev_[k]));
        return h_flags_[k] != 0;
    }

  private:
    void release()
    {
        for (auto& e : ev_) (void)hipEventDestroy(e);
        ev_.clear();
        if (h_flags_) (void)hipHostFree(h_flags_);
        dfree(d_flag_);
        h_flags_ = nullptr;
        d_flag_ = nullptr;
        cap_ = 0;
    }
    int cap_ = 0;
    int32_t* d_flag_ = nullptr;
    int32_t* h_flags_ = nullptr;
    std::vector<hipEvent_t> ev_;
};

// Per-step phase timing with HIP events, read after the cycle's final sync.
// An event costs a few microseconds of stream time, so only every kStride-th
// step of a cycle is marked and collect() scales the sampled steps' mean to
// all steps.
class StepTimer {
  public:
    static constexpr int kStride = 16;
    explicit StepTimer(bool on) : on_(on) {}
    StepTimer(const StepTimer&) = delete;
    StepTimer& operator=(const StepTimer&) = delete;
    ~StepTimer()
    {
        for (auto& e : ev_) (void)hipEventDestroy(e);
    }
    void ensure(int steps)
    {
        if (!on_) return;
        const int slots = (steps + kStride - 1) / kStride;
        while ((int)ev_.size() < 4 * slots) {
            hipEvent_t e;
            HC(hipEventCreate(&e));
            ev_.push_back(e);
        }
    }
    void mark(int k, int i, hipStream_t st)
    {
        if (on_ && k % kStride == 0) HC(hipEventRecord(ev_[4 * (k / kStride) + i], st));
    }
    // adds the estimated phase times of steps [0, nsteps) to a, b, c (t01, t12, t23)
    void collect(int nsteps, double& a, double& b, double& c)
    {
        if (!on_ || nsteps <= 0) return;
        const int m = (nsteps + kStride - 1) / kStride;
        double sa = 0.0, sb = 0.0, sc = 0.0;
        for (int q = 0; q < m; ++q) {
            float t = 0.f;
            HC(hipEventElapsedTime(&t, ev_[4 * q], ev_[4 * q + 1]));
            sa += t;
            HC(hipEventElapsedTime(&t, ev_[4 * q + 1], ev_[4 * q + 2]));
            sb += t;
            HC(hipEventElapsedTime(&t, ev_[4 * q + 2], ev_[4 * q + 3]));
            sc += t;
        }
        a += sa * nsteps / m;
        b += sb * nsteps / m;
        c += sc * nsteps / m;
    }
    bool on() const { return on_; }

  private:
    bool on_;
    std::vector<hipEvent_t> ev_;
};

// Sampled per-step kernel timing for the shared-Krylov phase.  An event costs
// a few microseconds of stream time, so only every kStride-th step is timed
// (its phases' first and last launches carry start and stop events); the
// sampled event sets form a ring of kRing, read on the host when a slot comes
// round again (the host has waited for later steps by then) or at the end, and
// the totals are scaled from the sampled steps to all steps.
class LaunchTimer {
  public:
    static constexpr int kStride = 16, kRing = 16, kPhases = 3;
    explicit LaunchTimer(bool on) : on_(on)
    {
        if (!on_) return;
        ev_.resize((size_t)kRing * kPhases * 2);
        for (auto& e : ev_) HC(hipEventCreate(&e));
    }
    LaunchTimer(const LaunchTimer&) = delete;
    LaunchTimer& operator=(const LaunchTimer&) = delete;
    ~LaunchTimer()
    {
        for (auto& e : ev_) (void)hipEventDestroy(e);
    }
    // start/stop events of phase i for step k, or null when step k is not
    // timed; call for phase 0 of step k before its other phases
    const hipEvent_t* events(int k, int i)
    {
        if (!on_ || k % kStride != 0) return nullptr;
        const int q = k / kStride;
        if (i == 0) {
            if (q >= kRing) read(q - kRing);
            if ((int)ms_.size() < q + 1) ms_.resize((size_t)q + 1, {0.0, 0.0, 0.0});
            recorded_ = q + 1;
        }
        return &ev_[((size_t)(q % kRing) * kPhases + i) * 2];
    }
    // adds the estimated phase times of steps [0, nsteps) to a, b, c: the
    // sampled steps' mean times nsteps
    void collect(int nsteps, double& a, double& b, double& c)
    {
        if (!on_ || nsteps <= 0) return;
        for (int q = recorded_ - kRing > 0 ? recorded_ - kRing : 0; q < recorded_; ++q) read(q);
        int m = 0;
        double sa = 0.0, sb = 0.0, sc = 0.0;
        for (int q = 0; q < recorded_ && q * kStride < nsteps; ++q, ++m) {
            sa += ms_[q][0];
            sb += ms_[q][1];
            sc += ms_[q][2];
        }
        if (m == 0) return;
        a += sa * nsteps / m;
        b += sb * nsteps / m;
        c += sc * nsteps / m;
    }

  private:
    void read(int q)
    {
        for (int i = 0; i < kPhases; ++i) {
            const hipEvent_t* e = &ev_[((size_t)(q % kRing) * kPhases + i) * 2];
            HC(hipEventSynchronize(e[1]));
            float t = 0.f;
            HC(hipEventElapsedTime(&t, e[0], e[1]));
            ms_[q][i] = t;
        }
    }
    bool on_;
    int recorded_ = 0;
    std::vector<hipEvent_t> ev_;
    std::vector<std::array<double, 3>> ms_;
};

// z_q(omega) of Eq. (z_q_wfq) with the Drude weight n/m* (graphene: E_F/(pi t_g)), omega in Hartree
void shift_q(double drude, double tau, double w, double& zr, double& zi);
// Eq. (z-mu): z_mu = -1 / alpha_IB
void shift_mu(double ar, double ai, double& zr, double& zi);
// Eq. (bem-dpcm): the BEM shift 2 pi (eps2 + eps1) / (eps2 - eps1)
void shift_bem(double e2r, double e2i, double e1r, double e1i, double& zr, double& zi);

}  // namespace pxs

struct pxStructure_t;
namespace pxs {
// The shift z of a BEM structure's operator (DPCM: the one above; IEFPCM: its
// negative) for the metal permittivity e2 (interleaved complex)
void shift_bem_of(const pxStructure_t* s, const double* e2, double& zr, double& zi);
}  // namespace pxs

namespace pxs {
// A solve started by pxSolveSpectrumAsync and not finished yet (px_api.cpp).
class PendingSolve {
  public:
    virtual ~PendingSolve() = default;
};
}  // namespace pxs

struct pxStructure_t {
    px::Geometry g;
    pxModel model = PX_WFQ;
    pxMaterial mat{};
    double eps1[2] = {1.0, 0.0};   // BEM: permittivity of the medium around the mesh
    double drude = 0.0;
    // two atom types: the second material, its Drude weight (types live in g)
    bool het = false;
    pxMaterial mat_b{};
    double drude_b = 0.0;
    hipStream_t st = nullptr;
    std::vector<int32_t> perm;
    int32_t* d_perm = nullptr;
    // frequencies and columns (frequency-major: column = w * npol + p)
    int n_omega = 0, npol = 0, ncol = 0, ldg = 0;
    std::vector<double> omega_au;
    std::vector<double> aib;   // 2 * n_omega (4 * n_omega for two types)
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
    pxs::StepSync sync;           // stop flag of the Arnoldi steps

    // stored-T apply: dense T in FP32 / FP64 (allocated when the tuner or the
    // options pick it), launches per method
    float* t32 = nullptr;
    double* t64 = nullptr;
    int64_t tstats[4] = {0, 0, 0, 0};   // FP32 on the fly, FP32 stored, FP64 on the fly, FP64 stored
    double tms[4] = {0, 0, 0, 0};       // their HIP-event milliseconds inside cycles (options.timings)
    double tflop[4] = {0, 0, 0, 0};     // their algorithmic FLOP inside cycles
    double probe[2] = {0, 0};           // last probe call: kernel milliseconds, pair evaluations

    bool idle = false;   // set once the structure's stream has been synchronised for destruction
    // status and message of the last solve (pxSolveSpectrum, pxSolveBatch, the server)
    pxStatus last_status = PX_E_STATE;
    std::string last_error = "not solved";

    std::unique_ptr<pxs::PendingSolve> pending;   // an asynchronous solve in progress

    ~pxStructure_t()
    {
        pending.reset();
        ws.release();
        void* ps[] = {g.xyz32, g.xyz64, g.glo, g.ghi, g.row_ptr, g.col, g.val, g.type, g.hrow, g.near_off, g.near_col, g.near_val, g.xyzc, g.bem_na, g.bem_an, g.bem_rv, g.bem_w, d_perm, d_col_pol, d_omega, x, b};
        for (void* p : ps) pxs::dfree(p);
        // the stored T came from the block cache
        for (void* p : {(void*)t32, (void*)t64}) {
            if (idle) pxs::BlockCache::get().give(p);
            else pxs::BlockCache::get().drop(p);
        }
    }
};

namespace pxs {
// Right-hand sides, x = 0, ||b|| and fresh statistics for every column of s.
void prepare_solve(pxStructure_t* s);
// Dipole moments, polarizability and cross sections from s->x; marks s solved.
void finish_solve(pxStructure_t* s);
}  // namespace pxs
