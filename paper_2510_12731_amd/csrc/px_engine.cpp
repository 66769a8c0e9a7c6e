// Stacked multi-structure engine: one block Krylov iteration over many
// structures at once (pxSolveBatch, and the continuous-batching server).
//
// Every structure's columns are cut into segments of Bc columns; the active
// segments of all structures are stacked row-wise in one block (each segment
// a 256-row-aligned range of rows), so each phase of an Arnoldi step is a
// single launch for all of them: a grouped T-apply over a tile list, one
// sparse apply, one pass of each CGS2 kernel with segment-wise reductions,
// one Givens update over the flat (segment, column) index.  Segments are
// admitted and retired only at restart-cycle boundaries, where the true
// residual is recomputed in FP64 for every segment (iterative refinement as in
// the single-structure solver).  A retired segment hands its columns back to
// its structure; a structure whose segments are all retired gets its
// observables computed and is returned to the caller.
#include "px_engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace px {
namespace {

__global__ void k_gather_range(const double2* __restrict__ src, int lds, int col0, int ncols,
                               double2* __restrict__ dst, int ldd, int64_t rows)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows || c >= ldd) return;
    dst[(size_t)r * ldd + c] = (c < ncols) ? src[(size_t)r * lds + col0 + c] : make_double2(0.0, 0.0);
}

__global__ void k_scatter_range(const double2* __restrict__ src, int lds, int ncols, double2* __restrict__ dst,
                                int ldd, int col0, int64_t rows)
{
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows || c >= ncols) return;
    dst[(size_t)r * ldd + col0 + c] = src[(size_t)r * lds + c];
}

inline dim3 grid_rc(int64_t rows, int cols) { return dim3((unsigned)((rows + 3) / 4), (unsigned)((cols + 63) / 64)); }

}  // namespace
}  // namespace px

namespace pxs {

using px::GroupSeg;

// Steps the host enqueues ahead of the last stop flag it looked at.
constexpr int kLag = 2;

size_t Engine::bytes_per_row(int Bc, int m_max)
{
    // Krylov basis + 7 column blocks (w, x, r, b and the repacking copies) in
    // FP64 complex, FP32 operands/results and the FP64 T-apply result
    return (size_t)Bc * 16 * (m_max + 1 + 7) + (size_t)Bc * (8 + 8 + 16);
}

Engine::Engine(hipStream_t st, int Bc, const pxSolveOptions& o, int64_t rows_cap, int nseg_cap)
    : caller_(st), Bc_(Bc), o_(o), rows_cap_(rows_cap), nseg_cap_(nseg_cap)
{
    // the engine's own stream (default priority, non-blocking so that it can be
    // captured into graphs), ordered after the caller's stream at every cycle
    HC(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
    HC(hipEventCreateWithFlags(&ev_in_, hipEventDisableTiming));
    m_max_ = std::max(o.restart_m, o.max_restart_m);
    m_ = o.restart_m;
    sync_.ensure(m_max_ + 1);
    rows_cap_ = ((rows_cap + 255) / 256) * 256;
    const size_t vec = (size_t)rows_cap_ * Bc_;
    const int ldf = nseg_cap_ * Bc_;
    V_ = dalloc<double2>((size_t)(m_max_ + 1) * vec);
    w_ = dalloc<double2>(vec);
    xs_ = dalloc<double2>(vec);
    rs_ = dalloc<double2>(vec);
    bs_ = dalloc<double2>(vec);
    xs2_ = dalloc<double2>(vec);
    bs2_ = dalloc<double2>(vec);
    X32_ = dalloc<float>(2 * vec);
    Y32_ = dalloc<float>(2 * vec);
    Y64_ = dalloc<double>(2 * vec);
    partial_ = dalloc<double2>(std::max((size_t)(rows_cap_ / 256) * (m_max_ + 1),
                                        px::dot_partial_slabs(rows_cap_, m_max_ + 1)) * 2 * Bc_);
    npart_ = dalloc<double>((size_t)px::update_chunks(rows_cap_) * Bc_);
    h1_ = dalloc<double2>((size_t)(m_max_ + 1) * ldf);
    h2_ = dalloc<double2>((size_t)(m_max_ + 1) * ldf);
    R_ = dalloc<double2>((size_t)m_max_ * (m_max_ + 1) * ldf);
    H_ = dalloc<double2>((size_t)m_max_ * (m_max_ + 1) * ldf);
    G_ = dalloc<double2>((size_t)(m_max_ + 1) * 2 * ldf);
    coefQ_ = dalloc<double2>((size_t)m_max_ * 2 * ldf);
    coefV_ = dalloc<double2>((size_t)2 * ldf);
    aux_ = dalloc<double2>((size_t)2 * ldf);
    sn_ = dalloc<double2>((size_t)m_max_ * ldf);
    gv_ = dalloc<double2>((size_t)(m_max_ + 1) * ldf);
    y_ = dalloc<double2>((size_t)m_max_ * ldf);
    cs_ = dalloc<double>((size_t)m_max_ * ldf);
    nrm_ = dalloc<double>(ldf);
    target_ = dalloc<double>(ldf);
    done_ = dalloc<int32_t>(ldf);
    steps_ = dalloc<int32_t>(ldf);
    zq_ = dalloc<double2>(ldf);
    zmu_ = dalloc<double2>(ldf);
    seginfo_ = dalloc<px::SegInfo>(nseg_cap_);
    chunk_seg_ = dalloc<int32_t>(rows_cap_ / 256 + 1);
    beg256_ = dalloc<int32_t>(nseg_cap_ + 1);
    beg32_ = dalloc<int32_t>(nseg_cap_ + 1);
    px::fill_zero(V_, sizeof(double2) * (size_t)(m_max_ + 1) * vec, st_);
    px::fill_zero(X32_, sizeof(float) * 2 * vec, st_);
}

Engine::~Engine()
{
    (void)hipStreamSynchronize(st_);
    drop_graphs();
    void* ps[] = {V_, w_, xs_, rs_, bs_, xs2_, bs2_, X32_, Y32_, Y64_, partial_, npart_, h1_, h2_, R_, H_, G_,
                  coefQ_, coefV_, aux_, sn_, gv_, y_,
                  cs_, nrm_, target_, done_, steps_, zq_, zmu_, seginfo_, chunk_seg_, beg256_, beg32_, split_};
    for (void* p : ps) dfree(p);
    (void)hipEventDestroy(ev_in_);
    (void)hipStreamDestroy(st_);
}

int Engine::segments_for(const pxStructure_t* s) const { return (s->ncol + Bc_ - 1) / Bc_; }

int64_t Engine::rows_for(const pxStructure_t* s) const { return (int64_t)segments_for(s) * s->g.nup; }

bool Engine::can_admit(const pxStructure_t* s) const
{
    return rows_ + pending_rows_ + rows_for(s) <= rows_cap_ &&
           (int)segs_.size() + segments_for(s) <= nseg_cap_;
}

void Engine::admit(pxStructure_t* s)
{
    for (int c0 = 0; c0 < s->ncol; c0 += Bc_) {
        EngineSeg e;
        e.s = s;
        e.c0 = c0;
        e.nc = std::min(Bc_, s->ncol - c0);
        e.rows = s->g.nup;
        e.fresh = true;
        segs_.push_back(e);
        pending_rows_ += e.rows;
    }
    open_[s] = segments_for(s);
    dirty_ = true;
}

void Engine::layout()
{
    drop_graphs();   // captured launches hold this layout's sizes and pointers
    // new row offsets; copy surviving segments' x and b, gather fresh ones from their structure
    int64_t off = 0;
    for (EngineSeg& e : segs_) {
        const int64_t old = e.row_off;
        e.row_off = off;
        if (e.fresh) {
            px_launch_gather(e.s->x, e.s->ldg, e.c0, e.nc, xs2_ + (size_t)off * Bc_, e.rows);
            px_launch_gather(e.s->b, e.s->ldg, e.c0, e.nc, bs2_ + (size_t)off * Bc_, e.rows);
            e.fresh = false;
        } else {
            HC(hipMemcpyAsync(xs2_ + (size_t)off * Bc_, xs_ + (size_t)old * Bc_, sizeof(double2) * e.rows * Bc_,
                              hipMemcpyDeviceToDevice, st_));
            HC(hipMemcpyAsync(bs2_ + (size_t)off * Bc_, bs_ + (size_t)old * Bc_, sizeof(double2) * e.rows * Bc_,
                              hipMemcpyDeviceToDevice, st_));
        }
        off += e.rows;
    }
    std::swap(xs_, xs2_);
    std::swap(bs_, bs2_);
    rows_ = off;
    pending_rows_ = 0;
    const int nseg = (int)segs_.size();
    const int ldf = nseg * Bc_;
    std::vector<px::SegInfo> info(nseg);
    std::vector<int32_t> chunk((size_t)(rows_ / 256) + 1, 0), b256(nseg + 1), b32(nseg + 1);
    std::vector<double2> zq(ldf, make_double2(1.0, 0.0)), zm(ldf, make_double2(1.0, 0.0));
    std::vector<GroupSeg> gs(nseg);
    for (int k = 0; k < nseg; ++k) {
        const EngineSeg& e = segs_[k];
        const px::Geometry& g = e.s->g;
        info[k] = px::SegInfo{e.row_off, g.n, g.np, g.model, 0, g.row_ptr, g.col, g.val};
        for (int64_t r = e.row_off / 256; r < (e.row_off + e.rows) / 256; ++r) chunk[r] = k;
        b256[k] = (int32_t)(e.row_off / 256);
        b32[k] = (int32_t)(e.row_off / px::UPD_ROWS);
        for (int c = 0; c < e.nc; ++c) {
            const int gc = e.c0 + c;
            const int w = gc / e.s->npol;
            double zr, zi;
            shift_q(e.s->drude, e.s->mat.tau, e.s->omega_au[w], zr, zi);
            zq[k * Bc_ + c] = make_double2(zr, zi);
            if (e.s->model == PX_WFQFMU) {
                shift_mu(e.s->aib[2 * w], e.s->aib[2 * w + 1], zr, zi);
                zm[k * Bc_ + c] = make_double2(zr, zi);
            }
        }
        gs[k] = GroupSeg{&g, e.row_off};
    }
    b256[nseg] = (int32_t)(rows_ / 256);
    b32[nseg] = (int32_t)(rows_ / px::UPD_ROWS);
    HC(hipMemcpyAsync(seginfo_, info.data(), sizeof(px::SegInfo) * nseg, hipMemcpyHostToDevice, st_));
    HC(hipMemcpyAsync(chunk_seg_, chunk.data(), sizeof(int32_t) * chunk.size(), hipMemcpyHostToDevice, st_));
    HC(hipMemcpyAsync(beg256_, b256.data(), sizeof(int32_t) * (nseg + 1), hipMemcpyHostToDevice, st_));
    HC(hipMemcpyAsync(beg32_, b32.data(), sizeof(int32_t) * (nseg + 1), hipMemcpyHostToDevice, st_));
    HC(hipMemcpyAsync(zq_, zq.data(), sizeof(double2) * ldf, hipMemcpyHostToDevice, st_));
    HC(hipMemcpyAsync(zmu_, zm.data(), sizeof(double2) * ldf, hipMemcpyHostToDevice, st_));
    HC(gt_.setup(gs, 2 * Bc_, rows_, st_));
    if (gt_.partial_bytes() > split_bytes_) {
        dfree(split_);
        split_ = dalloc<float>(gt_.partial_bytes() / sizeof(float) + 1);
        split_bytes_ = gt_.partial_bytes();
    }
    dirty_ = false;
}

void Engine::px_launch_gather(const double2* src, int lds, int col0, int ncols, double2* dst, int64_t rows)
{
    hipLaunchKernelGGL(px::k_gather_range, px::grid_rc(rows, Bc_), dim3(256), 0, st_, src, lds, col0, ncols, dst, Bc_,
                       rows);
}

void Engine::drop_graphs()
{
    for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second);
    graphs_.clear();
}

// Steps k0 .. k1-1 of a cycle of restart length m (delayed orthogonalisation,
// stop flag): the launch sequence that is captured into a graph.
void Engine::enqueue_steps(int k0, int k1, int m, int32_t* stop)
{
    const int nseg = (int)segs_.size();
    const int ldf = nseg * Bc_;
    const bool mixed = o_.precision == PX_MIXED;
    const int64_t rows = rows_;
    const int64_t vstride = rows * Bc_;
    for (int k = k0; k < k1; ++k) {
        double2* vk = V_ + k * vstride;
        if (mixed)
            gt_.run_f32(X32_, Y32_, split_, st_, stop);
        else
            gt_.run_f64(reinterpret_cast<const double*>(vk), Y64_, st_, stop);
        px::spmm_seg(seginfo_, chunk_seg_, mixed ? (const void*)Y32_ : (const void*)Y64_, mixed, 2 * Bc_, vk, zq_,
                     zmu_, nullptr, w_, rows, Bc_, nseg, SOLVER_MU_SIGN, st_, stop);
        px::dots2(V_, vstride, k + 1, w_, partial_, Bc_, Bc_, rows, st_, stop);
        px::reduce_dots2(partial_, rows, k + 1, G_, Bc_, Bc_, st_, beg256_, nseg, stop);
        px::dcgs2_coef(k, m, false, G_, nrm_, H_, R_, cs_, sn_, gv_, target_, done_, steps_, aux_, coefQ_, coefV_, ldf,
                       ldf, st_, stop);
        px::dcgs2_update(V_, vstride, k, coefQ_, coefV_, w_, npart_, Bc_, Bc_, rows, st_, chunk_seg_, ldf, stop);
        px::reduce_norms_seg(npart_, beg32_, nrm_, nseg, Bc_, st_, stop);
        px::normalize_seg(w_, nrm_, done_, chunk_seg_, V_ + (k + 1) * vstride, mixed ? X32_ : nullptr, Bc_, rows, st_,
                          stop);
        if (k == m - 1) {
            // the last basis vector's correction finishes column m-1
            px::dots2(V_, vstride, m + 1, V_ + m * vstride, partial_, Bc_, Bc_, rows, st_, stop);
            px::reduce_dots2(partial_, rows, m + 1, G_, Bc_, Bc_, st_, beg256_, nseg, stop);
            px::dcgs2_coef(m, m, true, G_, nrm_, H_, R_, cs_, sn_, gv_, target_, done_, steps_, aux_, coefQ_, coefV_,
                           ldf, ldf, st_, stop);
        }
    }
}

// Launches steps k0 .. k1-1 as a graph, capturing it on first use; the graph
// reads everything a cycle changes (targets, g, flags, shifts) from device
// memory, so it stays valid until the layout or the restart length changes.
void Engine::launch_steps_graph(int k0, int k1, int m, int32_t* stop)
{
    const int64_t key = ((int64_t)m << 20) | ((int64_t)k0 << 10) | (int64_t)(k1 - k0);
    auto it = graphs_.find(key);
    if (it == graphs_.end()) {
        hipGraph_t g = nullptr;
        HC(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_steps(k0, k1, m, stop);
        } catch (...) {
            (void)hipStreamEndCapture(st_, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        HC(hipStreamEndCapture(st_, &g));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HC(e);
        it = graphs_.emplace(key, ex).first;
        stats_.graphs += 1;
    }
    HC(hipGraphLaunch(it->second, st_));
}

std::vector<pxStructure_t*> Engine::cycle()
{
    std::vector<pxStructure_t*> finished;
    if (segs_.empty()) return finished;
    // work the caller queued on its stream (frequencies, x, b) comes first
    HC(hipEventRecord(ev_in_, caller_));
    HC(hipStreamWaitEvent(st_, ev_in_, 0));
    if (dirty_) layout();
    const int nseg = (int)segs_.size();
    const int ldf = nseg * Bc_;
    const bool mixed = o_.precision == PX_MIXED;
    const bool dcgs2 = o_.ortho == PX_ORTHO_DCGS2;
    const int64_t rows = rows_;

    // ---- true residual of every segment (FP64)
    gt_.run_f64(reinterpret_cast<const double*>(xs_), Y64_, st_);
    px::spmm_seg(seginfo_, chunk_seg_, Y64_, false, 2 * Bc_, xs_, zq_, zmu_, bs_, rs_, rows, Bc_, nseg, SOLVER_MU_SIGN,
                 st_);
    px::col_norm_partial(rs_, npart_, Bc_, Bc_, rows, st_);
    px::reduce_norms_seg(npart_, beg256_, nrm_, nseg, Bc_, st_);
    std::vector<double> beta(ldf);
    HC(hipMemcpyAsync(beta.data(), nrm_, sizeof(double) * ldf, hipMemcpyDeviceToHost, st_));
    HC(hipStreamSynchronize(st_));
    stats_.residuals += 1;

    std::vector<int32_t> done(ldf, 1);
    std::vector<double> tgt(ldf, 0.0);
    std::vector<double2> g0(ldf, make_double2(0.0, 0.0));
    bool slow = false, any_retired = false;
    for (int k = 0; k < nseg; ++k) {
        EngineSeg& e = segs_[k];
        pxStructure_t* s = e.s;
        bool active = false;
        for (int c = 0; c < e.nc; ++c) {
            const int gc = e.c0 + c, f = k * Bc_ + c;
            const double prev = s->relres[gc];
            s->relres[gc] = s->bnorm[gc] > 0.0 ? beta[f] / s->bnorm[gc] : 0.0;
            // x is unchanged since the last residual if that pass only retired segments
            const bool moved = !relaid_only_ && s->cycles[gc] > 0;
            if (moved && s->relres[gc] > 0.98 * prev) s->stall[gc] += 1;
            else if (moved) s->stall[gc] = 0;
            if (s->relres[gc] > o_.rel_tol && s->cycles[gc] < o_.max_cycles &&
                (o_.stall_cycles == 0 || s->stall[gc] < o_.stall_cycles)) {
                active = true;
                done[f] = 0;
                tgt[f] = std::max(0.5 * o_.rel_tol * s->bnorm[gc], mixed ? beta[f] * o_.inner_reduction : 0.0);
                g0[f] = make_double2(beta[f], 0.0);
                if (moved && s->relres[gc] > 0.7 * prev) slow = true;
            }
        }
        if (!active) {
            hipLaunchKernelGGL(px::k_scatter_range, px::grid_rc(e.rows, e.nc), dim3(256), 0, st_,
                               xs_ + (size_t)e.row_off * Bc_, Bc_, e.nc, s->x, s->ldg, e.c0, e.rows);
            e.finished = true;
            any_retired = true;
            if (--open_[s] == 0) {
                HC(hipStreamSynchronize(st_));
                finish_solve(s);
                open_.erase(s);
                finished.push_back(s);
            }
        }
    }
    if (any_retired) {
        segs_.erase(std::remove_if(segs_.begin(), segs_.end(), [](const EngineSeg& e) { return e.finished; }),
                    segs_.end());
        dirty_ = true;
        relaid_only_ = true;
        HC(hipStreamSynchronize(st_));
        return finished;   // the remaining segments restart from a fresh layout
    }
    relaid_only_ = false;
    if (slow && m_ < m_max_) {
        m_ = std::min(2 * m_, m_max_);
        for (EngineSeg& e : segs_)
            for (int c = 0; c < e.nc; ++c) e.s->stall[e.c0 + c] = 0;
    }

    // ---- one restart cycle over all segments
    const int m = m_;
    const int64_t vstride = rows * Bc_;
    HC(hipMemcpyAsync(target_, tgt.data(), sizeof(double) * ldf, hipMemcpyHostToDevice, st_));
    px::fill_zero(gv_, sizeof(double2) * (size_t)(m + 1) * ldf, st_);
    HC(hipMemcpyAsync(gv_, g0.data(), sizeof(double2) * ldf, hipMemcpyHostToDevice, st_));
    HC(hipMemcpyAsync(done_, done.data(), sizeof(int32_t) * ldf, hipMemcpyHostToDevice, st_));
    px::fill_zero(steps_, sizeof(int32_t) * ldf, st_);
    HC(hipMemcpyAsync(nrm_, beta.data(), sizeof(double) * ldf, hipMemcpyHostToDevice, st_));
    px::normalize_seg(rs_, nrm_, done_, chunk_seg_, V_, mixed ? X32_ : nullptr, Bc_, rows, st_);
    std::vector<int32_t> done_h(ldf);
    if (dcgs2) {
        // steps run ahead of the host; a device flag, raised once the rotations have
        // finished every column, turns the remaining launches into no-ops
        int32_t* stop = sync_.flag();
        sync_.reset(st_);
        const int chunk = o_.graph_steps > 0 ? o_.graph_steps : 1;
        for (int k0 = 0, j = 0; k0 < m; k0 += chunk, ++j) {
            if (j >= kLag && sync_.stopped(j - kLag)) break;
            const int k1 = std::min(m, k0 + chunk);
            if (o_.graph_steps > 0) launch_steps_graph(k0, k1, m, stop);
            else enqueue_steps(k0, k1, m, stop);
            sync_.publish(j, st_);
        }
    } else {
        for (int k = 0; k < m; ++k) {
            double2* vk = V_ + k * vstride;
            if (mixed) gt_.run_f32(X32_, Y32_, split_, st_);
            else gt_.run_f64(reinterpret_cast<const double*>(vk), Y64_, st_);
            px::spmm_seg(seginfo_, chunk_seg_, mixed ? (const void*)Y32_ : (const void*)Y64_, mixed, 2 * Bc_, vk, zq_,
                         zmu_, nullptr, w_, rows, Bc_, nseg, SOLVER_MU_SIGN, st_);
            px::col_dots(V_, vstride, k + 1, w_, partial_, Bc_, Bc_, rows, st_);
            px::reduce_dots_seg(partial_, beg256_, k + 1, h1_, nseg, Bc_, st_);
            px::col_update_seg(V_, vstride, k + 1, h1_, w_, nullptr, chunk_seg_, Bc_, nseg, rows, st_);
            px::col_dots(V_, vstride, k + 1, w_, partial_, Bc_, Bc_, rows, st_);
            px::reduce_dots_seg(partial_, beg256_, k + 1, h2_, nseg, Bc_, st_);
            px::col_update_seg(V_, vstride, k + 1, h2_, w_, npart_, chunk_seg_, Bc_, nseg, rows, st_);
            px::reduce_norms_seg(npart_, beg32_, nrm_, nseg, Bc_, st_);
            px::givens_step(k, m, h1_, h2_, nrm_, R_, cs_, sn_, gv_, target_, done_, steps_, nullptr, ldf, ldf, st_);
            px::normalize_seg(w_, nrm_, done_, chunk_seg_, V_ + (k + 1) * vstride, mixed ? X32_ : nullptr, Bc_, rows,
                              st_);
            HC(hipMemcpyAsync(done_h.data(), done_, sizeof(int32_t) * ldf, hipMemcpyDeviceToHost, st_));
            HC(hipStreamSynchronize(st_));
            stats_.steps += 1;
            (mixed ? stats_.tapply_f32 : stats_.tapply_f64) += 1;
            bool all = true;
            for (int f = 0; f < ldf && all; ++f) all = done_h[f] != 0;
            if (all) break;
        }
    }
    px::lsq_solve(m, R_, gv_, steps_, y_, ldf, ldf, st_);
    px::x_update_seg(V_, vstride, y_, steps_, chunk_seg_, xs_, Bc_, nseg, rows, st_);
    std::vector<int32_t> steps_h(ldf);
    HC(hipMemcpyAsync(steps_h.data(), steps_, sizeof(int32_t) * ldf, hipMemcpyDeviceToHost, st_));
    HC(hipStreamSynchronize(st_));
    int executed = 0;
    for (int k = 0; k < nseg; ++k) {
        const EngineSeg& e = segs_[k];
        for (int c = 0; c < e.nc; ++c) {
            const int f = k * Bc_ + c;
            if (done[f]) continue;   // column was already finished at the cycle start
            e.s->iters[e.c0 + c] += steps_h[f];
            e.s->cycles[e.c0 + c] += 1;
            executed = std::max(executed, dcgs2 ? std::min(steps_h[f] + 1, m) : steps_h[f]);
        }
    }
    if (dcgs2) stats_.steps += executed;
    (mixed ? stats_.tapply_f32 : stats_.tapply_f64) += dcgs2 ? executed : 0;
    stats_.cycles += 1;
    return finished;
}

}  // namespace pxs
