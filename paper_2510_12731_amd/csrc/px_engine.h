// Stacked multi-structure engine (see px_engine.cpp).
#pragma once

#include <map>
#include <vector>

#include "px_state.h"

namespace pxs {

struct EngineSeg {
    pxStructure_t* s = nullptr;
    int c0 = 0, nc = 0;        // global columns [c0, c0 + nc) of s
    int64_t rows = 0;          // s->g.nup
    int64_t row_off = 0;       // first row in the current stacked layout
    bool fresh = true;         // not yet placed in a layout
    bool finished = false;
};

struct EngineStats {
    int64_t cycles = 0, steps = 0, residuals = 0, tapply_f32 = 0, tapply_f64 = 0, graphs = 0;
};

class Engine {
  public:
    // rows_cap: capacity of the stacked block in rows; nseg_cap: maximum number of segments.
    Engine(hipStream_t st, int Bc, const pxSolveOptions& o, int64_t rows_cap, int nseg_cap);
    ~Engine();
    Engine(const Engine&) = delete;
    Engine& operator=(const Engine&) = delete;

    // HBM bytes of engine storage per stacked row.
    static size_t bytes_per_row(int Bc, int m_max);
    int segments_for(const pxStructure_t* s) const;
    int64_t rows_for(const pxStructure_t* s) const;
    bool can_admit(const pxStructure_t* s) const;
    // s must have been through prepare_solve(); its segments join at the next cycle.
    void admit(pxStructure_t* s);
    // One restart cycle over every active segment; returns the structures whose
    // last segment retired (their results are final).
    std::vector<pxStructure_t*> cycle();
    bool idle() const { return segs_.empty(); }
    int64_t rows_in_use() const { return rows_ + pending_rows_; }
    int64_t rows_capacity() const { return rows_cap_; }
    int n_structures() const { return (int)open_.size(); }
    const EngineStats& stats() const { return stats_; }

  private:
    void layout();
    void drop_graphs();
    void enqueue_steps(int k0, int k1, int m, int32_t* stop);
    void launch_steps_graph(int k0, int k1, int m, int32_t* stop);
    void px_launch_gather(const double2* src, int lds, int col0, int ncols, double2* dst, int64_t rows);

    hipStream_t caller_;           // the stream the structures and the caller use
    hipStream_t st_ = nullptr;     // the engine's own stream
    hipEvent_t ev_in_ = nullptr;
    std::map<int64_t, hipGraphExec_t> graphs_;   // captured step chunks of the current layout
    int Bc_;
    pxSolveOptions o_;
    int m_max_ = 0, m_ = 0;
    int64_t rows_cap_ = 0;
    int nseg_cap_ = 0;
    std::vector<EngineSeg> segs_;
    std::map<pxStructure_t*, int> open_;   // structure -> segments not yet retired
    bool dirty_ = true;
    bool relaid_only_ = false;   // last cycle() only retired segments (x unchanged)
    int64_t rows_ = 0, pending_rows_ = 0;
    EngineStats stats_;
    px::GroupedTApply gt_;
    double2 *V_ = nullptr, *w_ = nullptr, *xs_ = nullptr, *rs_ = nullptr, *bs_ = nullptr, *xs2_ = nullptr,
            *bs2_ = nullptr;
    float *X32_ = nullptr, *Y32_ = nullptr, *split_ = nullptr;
    size_t split_bytes_ = 0;
    double* Y64_ = nullptr;
    double2* partial_ = nullptr;
    double* npart_ = nullptr;
    double2 *h1_ = nullptr, *h2_ = nullptr, *R_ = nullptr, *sn_ = nullptr, *gv_ = nullptr, *y_ = nullptr;
    double2 *H_ = nullptr, *G_ = nullptr, *coefQ_ = nullptr, *coefV_ = nullptr, *aux_ = nullptr;
    double *cs_ = nullptr, *nrm_ = nullptr, *target_ = nullptr;
    int32_t *done_ = nullptr, *steps_ = nullptr;
    double2 *zq_ = nullptr, *zmu_ = nullptr;
    px::SegInfo* seginfo_ = nullptr;
    int32_t *chunk_seg_ = nullptr, *beg256_ = nullptr, *beg32_ = nullptr;
    StepSync sync_;   // stop flag of the Arnoldi steps
};

}  // namespace pxs
