// Internal declarations of the HIP solver library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "plasmonx.h"

namespace px {

// Device memory of the library.  With no caller allocator installed
// (pxSetAllocator) these are hipMalloc and hipFree; with one, blocks come from
// it, and each block goes back to the allocator that made it after the device
// has finished with it (as hipFree waits for the device).
hipError_t dev_malloc(void** p, size_t bytes);
void dev_free(void* p);
// true while a caller allocator is installed
bool caller_allocator();
void set_allocator(pxDeviceAllocFn alloc, pxDeviceFreeFn free, void* user);

// Atom padding: every device vector holds np >= n rows per component; rows
// n..np-1 belong to ghost atoms parked far away with zero unknowns.
constexpr int ATOM_PAD = 256;
// Atoms per bounding-box group used by the near/far split of the T-apply.
constexpr int GROUP = 32;
// Complex columns of every active block are padded to a multiple of this.
constexpr int COL_PAD = 64;
// Rows per partial-sum chunk of the dipole reduction.
constexpr int RED_ROWS = 64;
// Rows per partial-sum chunk of the Arnoldi reductions (dots, norms), basis
// vectors per dot-product block, rows per thread in the basis update.
constexpr int ARN_ROWS = 256;
constexpr int ARN_JB = 8;
constexpr int ARN_RG = 8;
inline int arnoldi_chunks(int64_t rows) { return (int)((rows + ARN_ROWS - 1) / ARN_ROWS); }
// Rows per block of the basis update (its norm partials come in these chunks).
constexpr int UPD_ROWS = 4 * ARN_RG;
inline int update_chunks(int64_t rows) { return (int)((rows + UPD_ROWS - 1) / UPD_ROWS); }

struct Geometry {
    int model = 0;         // 0 omegaFQ, 1 omegaFQFmu
    int64_t n = 0;         // real atoms
    int64_t np = 0;        // padded atoms
    int64_t nu = 0;        // unknowns (n or 4n)
    int64_t nup = 0;       // padded unknown rows (np or 4np)
    float4* xyz32 = nullptr;   // [np] bohr, Morton order, ghosts far away
    double4* xyz64 = nullptr;  // [np]
    float4* glo = nullptr;     // [np/GROUP] group bounding boxes (conservative)
    float4* ghi = nullptr;
    // CSR of Kbar over the n real atoms (FP64 values, diagonal included)
    int32_t* row_ptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    int64_t nnz = 0;
    // kernel constants (bohr)
    double r_q = 0, r_mu = 0;
    // two atom types (null for homogeneous structures): type per atom in
    // Morton order, and per real atom (same-type K row sum, other-type K row
    // sum, same-type and other-type neighbour counts)
    uint8_t* type = nullptr;
    double4* hrow = nullptr;
    // omegaFQ near field in FP64 (built by ensure_near_f64): T - T_point over
    // the real atoms for the pairs closer than the FP64 far threshold,
    // -erfc(r/R)/r off the diagonal and the self term on it, in ELL layout per
    // block of 256 rows: near_off[b] is block b's first entry ([np/256 + 1]),
    // slot k of row i at near_off[i/256] + 256 k + i % 256, unused slots zero
    int64_t* near_off = nullptr;
    int32_t* near_col = nullptr;
    double* near_val = nullptr;
    int64_t near_nnz = 0;   // entries including the unused slots
    // centre of the real atoms' bounding box (bohr), and for the point-charge
    // kernel every atom's position relative to it with its squared norm in w
    double cx = 0, cy = 0, cz = 0;
    double4* xyzc = nullptr;   // [np], built with the near-field list
    // BEM: the sites are tesserae (barycentres in xyz64, and relative to the
    // centre (cx, cy, cz) with |p|^2 in w in xyzc), with their outward unit
    // normal and area in bem_na [np] (ghosts: area 0) and (A n, A p.n) in
    // bem_an, the identity in place of Kbar and the radius enclosing the mesh
    // (bohr).  With u = s - c (c the tesserae's area-weighted centroid), DPCM
    // solves for the charges with the dipole weights bem_w [np] = u (d_k =
    // w_k . q); IEFPCM (bem_ief) for the potential y = S A^-1 q they make,
    // with bem_rv [np] = 2 pi u + F u (the right-hand side per unit field,
    // component l for polarization l) and bem_w [np] = (S A^-1)^-1 u (d_k =
    // w_k . y, S A^-1 being symmetric)
    bool bem = false;
    bool bem_ief = false;
    double4* bem_na = nullptr;
    double4* bem_an = nullptr;
    double4* bem_rv = nullptr;
    double4* bem_w = nullptr;
    double bem_r = 0.0;
};

// ---- BEM, DPCM and IEFPCM (px_bem.hip) -------------------------------------------
// The mesh on the device (caller order; positions and areas in bohr units);
// for IEFPCM also bem_rv and bem_w (the latter by bem_single_layer_solve;
// *status as there).
hipError_t build_bem_geometry(Geometry& g, const double* cen_bohr, const double* nrm, const double* area_bohr2,
                              double r_enc_bohr, bool ief, hipStream_t st, int* status);
// Y = M X (DPCM) or Y = F X (IEFPCM) for ncols real columns (X, Y row-major,
// ld ldx), generated on the fly in FP64; scratch of bem_scratch_bytes(g, ncols)
// (wider launches above 8 columns).
size_t bem_scratch_bytes(const Geometry& g, int ncols);
void bem_apply_f64(const Geometry& g, const double* X, double* Y, int ldx, int ncols, hipStream_t st, double* scratch,
                   const int32_t* stop = nullptr, const hipEvent_t* ev = nullptr);
// Solves (S A^-1) X = B for nc <= 8 real columns (IEFPCM's single layer, ghost
// rows of B ignored): B rows of stride ldb, X [np][nc] contiguous on return,
// Jacobi-preconditioned conjugate gradients to ||B - S A^-1 X|| <= tol ||B||
// per column.  *status: 0 converged, 1 not within max_iter, 2 a direction of
// non-positive curvature (S A^-1 not positive definite on this mesh).
hipError_t bem_single_layer_solve(const Geometry& g, const double* B, int ldb, int nc, double* X, double tol,
                                  int max_iter, hipStream_t st, int* status, int* iters, double* relres);
// b per column: -A E0 n_l (DPCM) or E0 (2 pi s_l + (F s)_l) (IEFPCM), complex
// with imaginary part 0
void bem_rhs(const Geometry& g, const int32_t* col_pol, double e0, double2* b, int ncol, int ldb, hipStream_t st);

// Ascending bitonic sort of npow (a power of two) 64-bit keys in place.
void sort_keys(uint64_t* keys, int64_t npow, hipStream_t st);
// Candidate subsets per 64-row block of the neighbour builders (px_neighbors.h)
int neighbor_subsets(int64_t np);
// cnt[i] = add + sum over nsub subsets of cntw[s][i] (row stride np), i < n
void count_sum(const int32_t* cntw, int nsub, int64_t np, int64_t n, int32_t add, int32_t* cnt, hipStream_t st);
// Exclusive scan of cnt[0..n) into row_ptr[0..n] (one workgroup).
void scan_counts(const int32_t* cnt, int64_t n, int32_t* row_ptr, hipStream_t st);
// Builds g's FP64 near-field list for the omegaFQ narrow T-apply once
// (a no-op when built or for the dipole model); synchronises st.
hipError_t ensure_near_f64(Geometry& g, hipStream_t st);

// ---- T-apply launchers (px_tapply.hip) -------------------------------------
// Y = T X over real columns: X, Y are [nup][ldx] (row-major, component-major
// blocks for the dipole model); ncols real columns, multiple of 2*COL_PAD for
// the wide kernels.  Ghost rows of Y are unspecified.
// scratch: tapply_f32_scratch_bytes(g, ncols) bytes (split-K partial sums).
void tapply_f32(const Geometry& g, const float* X, float* Y, int ldx, int ncols, hipStream_t st, float* scratch, const int32_t* stop = nullptr);
size_t tapply_f32_scratch_bytes(const Geometry& g, int ncols);
// ev: optional start/stop events carried by the first and last launch (timing
// without extra stream packets).
// active (blocks of more than 8 columns): the real columns that hold data;
// column blocks past them are skipped (their outputs are not read); 0 = all
void tapply_f64(const Geometry& g, const double* X, double* Y, int ldx, int ncols, hipStream_t st,
                double* scratch, size_t scratch_bytes, const int32_t* stop = nullptr, const hipEvent_t* ev = nullptr,
                int active = 0);
size_t tapply_f64_scratch_bytes(const Geometry& g, int ncols);

// Dense T over the padded unknowns (row-major, nup x nup; ghost rows and
// columns zero) for the stored-T apply: Y = T X is then one GEMM.
// Y = T X with T stored dense (tdense_f32 / tdense_f64: row-major, nup x nup,
// symmetric), either model: FP32 on MFMA with the stream-K pieces of
// tapply_f32 (ncols a multiple of 128; scratch of tstored_f32_scratch_bytes());
// FP64 on MFMA (ncols a multiple of 64), or for 1-8 real columns (ldx ==
// ncols) a split pass over T with scratch of tapply_f64_scratch_bytes(g, 8).
// ev: optional start/stop events carried by the first and last launch.
size_t tstored_f32_scratch_bytes();
// active: the real columns that hold data (the others are never read); 0 = all
void tstored_f32(const Geometry& g, const float* T, const float* X, float* Y, int ldx, int ncols, hipStream_t st,
                 float* scratch, const int32_t* stop = nullptr, const hipEvent_t* ev = nullptr, int active = 0);
void tstored_f64(const Geometry& g, const double* T, const double* X, double* Y, int ldx, int ncols, hipStream_t st,
                 double* scratch, const int32_t* stop = nullptr, const hipEvent_t* ev = nullptr, int active = 0);
void tdense_f32(const Geometry& g, float* T, hipStream_t st);
void tdense_f64(const Geometry& g, double* T, hipStream_t st);

// Grouped T-apply over the segments of a stacked block (each segment one
// structure's padded rows starting at row_off; real columns ldx, a multiple
// of 128).  setup() builds and uploads the tile lists; run_* launch one kernel
// per precision and model for all segments.
struct GroupSeg {
    const Geometry* g;
    int64_t row_off;
};
class GroupedTApply {
  public:
    GroupedTApply();
    ~GroupedTApply();
    GroupedTApply(const GroupedTApply&) = delete;
    GroupedTApply& operator=(const GroupedTApply&) = delete;
    hipError_t setup(const std::vector<GroupSeg>& segs, int ldx, int64_t rows, hipStream_t st);
    size_t partial_bytes() const;   // split-K scratch needed by run_f32
    int64_t f32_tiles() const;
    void run_f32(const float* X, float* Y, float* partial, hipStream_t st, const int32_t* stop = nullptr) const;
    void run_f64(const double* X, double* Y, hipStream_t st, const int32_t* stop = nullptr) const;

  private:
    struct Impl;
    Impl* impl;
};

// ---- other kernels (px_kernels.hip) ----------------------------------------
// types_host (n atoms, 0/1, may be null) with mb: a two-type structure; unlike
// pairs exchange with the mean of the two materials' A, r0, d, s and cutoff.
hipError_t build_geometry(Geometry& g, const double* xyz_bohr_host, double cutoff_bohr, const pxMaterial& m,
                          double r0_bohr, std::vector<int32_t>& perm_host, int* bad_pair, hipStream_t st,
                          const uint8_t* types_host = nullptr, const pxMaterial* mb = nullptr);
// Two-type sparse apply and right-hand side (the structure must have types):
// het [6][lda] per column: z_q,A, z_q,B, gamma_A, gamma_B, 1/alpha_IB,A, 1/alpha_IB,B;
// gam [2][ldb]: gamma_A, gamma_B per column.
void spmm_het(const Geometry& g, const void* Y, bool y_is_f32, int ldy, const double2* X, const double2* het,
              const double2* B, double2* W, int na, int lda, double mu_sign, hipStream_t st,
              const int32_t* stop = nullptr);
void build_rhs_het(const Geometry& g, const int32_t* col_pol, const double2* gam, double e0, double2* b, int ncol,
                   int ldb, double mu_sign, hipStream_t st);

struct Shifts {            // per active slot
    double2* zq = nullptr;
    double2* zmu = nullptr;
};

// mu_sign: +1 gives the paper's operator, -1 the solver's form with negated dipole rows.
void spmm_shift(const Geometry& g, const void* Y, bool y_is_f32, int ldy, const double2* X, const double2* zq,
                const double2* zmu, const double2* B, double2* W, int na, int lda, double mu_sign, hipStream_t st, const int32_t* stop = nullptr);
void build_rhs(const Geometry& g, const int32_t* col_pol, double e0, double2* b, int ncol, int ldb, double mu_sign,
               hipStream_t st);
void col_dots(const double2* V, int64_t vstride, int nvec, const double2* w, double2* partial, int na, int lda,
              int64_t nup, hipStream_t st);
void reduce_dots(const double2* partial, int nchunk, int nvec, double2* h, int na, int lda, bool accumulate,
                 hipStream_t st);
// norm_partial (may be null): update_chunks(nup) x lda partial sums of |w|^2.
void col_update(const double2* V, int64_t vstride, int nvec, const double2* h, double2* w, double* norm_partial,
                int na, int lda, int64_t nup, hipStream_t st);
void reduce_norms(const double* partial, int nchunk, double* nrm, int na, int lda, hipStream_t st, const int32_t* stop = nullptr);
void col_norm_partial(const double2* w, double* partial, int na, int lda, int64_t nup, hipStream_t st);
void normalize(const double2* w, const double* nrm, const int32_t* done, double2* v, float* x32, int na, int lda,
               int64_t nup, hipStream_t st, const int32_t* stop = nullptr);
void to_f32(const double2* v, float* x32, int na, int lda, int64_t nup, hipStream_t st);
void givens_step(int k, int m, const double2* h1, const double2* h2, const double* nrm, double2* R, double* cs,
                 double2* sn, double2* gvec, const double* target, int32_t* done, int32_t* steps, int32_t* n_open,
                 int na, int lda, hipStream_t st);
void lsq_solve(int m, const double2* R, const double2* gvec, const int32_t* steps, double2* y, int na, int lda,
               hipStream_t st);
void x_update(const double2* V, int64_t vstride, const double2* y, const int32_t* steps, int m, double2* x,
              int na, int lda, int64_t nup, hipStream_t st);
void gather_cols(const double2* src, int lds, double2* dst, int ldd, const int32_t* map, int na, int64_t nup,
                 hipStream_t st);
void scatter_cols(const double2* src, int lds, double2* dst, int ldd, const int32_t* map, int na, int64_t nup,
                  hipStream_t st);
void observables(const Geometry& g, const double2* x, int ncol, int ldx, double2* dpart, double2* d,
                 hipStream_t st);
void spectrum(const double2* d, const int32_t* col_pol, int n_omega, int npol, const double* omega_au, double e0,
              double2* alpha, double* sigma, hipStream_t st);
void unpermute(const Geometry& g, const double2* x, int ldx, int col, const int32_t* perm, double2* out,
               hipStream_t st);
void permute_in(const Geometry& g, const double2* in, int ncol, const int32_t* perm, double2* x, int ldx,
                hipStream_t st);
void fill_zero(void* p, size_t bytes, hipStream_t st);

// CGS2 with delayed reorthogonalisation (px_kernels.hip): G is [nvec][2][lda],
// H the raw Hessenberg [m][m+1][lda], coefQ [m][2][lda], coefV [2][lda].
// The dot pass sums dot_rows(nvec) rows per partial; partial holds
// dot_chunks(nup, nvec) x nvec x 2 x lda values, at most
// dot_partial_slabs(nup, nvec_max) x 2 x lda for bases up to nvec_max vectors.
int dot_rows(int nvec);
inline int dot_chunks(int64_t nup, int nvec) { return (int)((nup + dot_rows(nvec) - 1) / dot_rows(nvec)); }
size_t dot_partial_slabs(int64_t nup, int nvec_max);
void dots2(const double2* V, int64_t vstride, int nvec, const double2* w, double2* partial, int na, int lda,
           int64_t nup, hipStream_t st, const int32_t* stop = nullptr);
// With segments (seg_beg: first 256-row chunk of each of nseg segments of lda
// columns), G is indexed by the flat column seg * lda + c.
void reduce_dots2(const double2* partial, int64_t nup, int nvec, double2* G, int na, int lda, hipStream_t st,
                  const int32_t* seg_beg = nullptr, int nseg = 1, const int32_t* stop = nullptr);
// aux: [2][lda] scratch (rho, c_k) between the column-serial and the row-parallel part.
// stop (optional): set to 1 once the rotations have finished every one of the na
// columns; every kernel of an Arnoldi step that is given the flag returns at once
// when it is set.
void dcgs2_coef(int k, int m, bool final_only, const double2* G, const double* nrm, double2* H, double2* R,
                double* cs, double2* sn, double2* gvec, const double* target, int32_t* done, int32_t* steps,
                double2* aux, double2* coefQ, double2* coefV, int na, int lda, hipStream_t st, int32_t* stop = nullptr);
// chunk_seg (per 256-row chunk: its segment) switches to flat coefficients of
// leading dimension ldc.
void dcgs2_update(double2* V, int64_t vstride, int k, const double2* coefQ, const double2* coefV, double2* w,
                  double* norm_partial, int na, int lda, int64_t nup, hipStream_t st,
                  const int32_t* chunk_seg = nullptr, int ldc = 0, const int32_t* stop = nullptr);

// ---- stacked segments (px_engine.cpp) ---------------------------------------
// One segment of a stacked block: a structure's padded rows (np or 4 np) with
// Bc columns, starting at row_off (a multiple of 256).
struct SegInfo {
    int64_t row_off, n, np;
    int32_t model, pad;
    const int32_t* rp;
    const int32_t* ci;
    const double* cv;
};
void spmm_seg(const SegInfo* segs, const int32_t* chunk_seg, const void* Y, bool y_is_f32, int ldy, const double2* X,
              const double2* zq, const double2* zmu, const double2* B, double2* W, int64_t rows, int Bc, int nseg,
              double mu_sign, hipStream_t st, const int32_t* stop = nullptr);
void reduce_dots_seg(const double2* partial, const int32_t* seg_beg, int nvec, double2* h, int nseg, int Bc,
                     hipStream_t st);
void reduce_norms_seg(const double* partial, const int32_t* seg_beg, double* nrm, int nseg, int Bc, hipStream_t st, const int32_t* stop = nullptr);
void col_update_seg(const double2* V, int64_t vstride, int nvec, const double2* h, double2* w, double* norm_partial,
                    const int32_t* chunk_seg, int Bc, int nseg, int64_t rows, hipStream_t st);
void normalize_seg(const double2* w, const double* nrm, const int32_t* done, const int32_t* chunk_seg, double2* v,
                   float* x32, int Bc, int64_t rows, hipStream_t st, const int32_t* stop = nullptr);
void x_update_seg(const double2* V, int64_t vstride, const double2* y, const int32_t* steps, const int32_t* chunk_seg,
                  double2* x, int Bc, int nseg, int64_t rows, hipStream_t st);

// ---- post-processing: field and density at probe points (px_probe.hip) ------
// Sources of one column (charge, and for the dipole model the dipole, per atom
// in Morton order; np x 2 or np x 8 doubles) from the solution x.
void probe_sources(const Geometry& g, const double2* x, int ldx, int col, double* src, hipStream_t st);
// Partial-sum scratch (doubles) for npts points.
size_t probe_part_doubles(const Geometry& g, int64_t npts);
// Scratch of probe_field for npts points: keys (npow = the power of two >=
// npad), sorted points (npad) and their order (npad), in bytes.
size_t probe_order_bytes(int64_t npts);
// field [npts][3] complex and rho [npts] complex at pts [npts] (bohr, w
// unused), in the caller's order; lo/hi: the points' bounding box (bohr).  The
// points are evaluated in Morton order (compact waves) and the results
// scattered back.  order: probe_order_bytes(npts) bytes of scratch.
void probe_field(const Geometry& g, const double* src, const double4* pts, int64_t npts, const double lo[3],
                 const double hi[3], void* order, double* part, double* field, double* rho, hipStream_t st);

// ---- shared-Krylov solve (px_shifted.hip) ----------------------------------
// R = npol real slots per row (1..3), one per polarization; Hbar row-major per
// slot with row stride kcap; see px_shifted.hip.
void ms_init(int R, const double2* b, int ldb, const double* bnorm, double* u, int64_t nup, hipStream_t st);
// ev (optional): start and stop events carried by the first and last launch.
void ms_spmv(int R, const Geometry& g, const double* Y, double* w, hipStream_t st, const int32_t* stop,
             const hipEvent_t* ev = nullptr);
// One DCGS2 step k: dots of [V_{<k}, u] with u and wt, the coefficients (column
// k-1 corrected, column k first pass) and the update pass writing V_k and the
// next candidate u; fix_only: the last column's correction alone.
void ms_step(int R, double* V, int64_t vstride, int k, double* u, const double* wt, double* part, double* part2,
             double* G, double* H, int kcap, double* coefv, double* coefu, double* scal, int64_t nup, bool fix_only,
             hipStream_t st, const int32_t* stop, const hipEvent_t* ev = nullptr);
size_t ms_part_doubles(int R, int64_t nup, int kcap);
size_t ms_part2_doubles(int R, int64_t nup, int kcap);
// Hessenberg columns k0 .. k0+kn-1 (kn <= ms_givens_batch()) for every (frequency, polarization) pair
int ms_givens_batch();
void ms_givens(const double* H, int kcap, int npol, int P, int k0, int kn, const double2* z, double* cs, double2* sn,
               double2* g, const double* target, int32_t* done, double* resid, int32_t* ndone, int32_t* stop,
               hipStream_t st);
// every pair's triangular factor, packed, into rst (ms_rst_elems(P, kcap) complex)
size_t ms_rst_elems(int P, int kcap);
void ms_rfactor(const double* H, int kcap, int npol, int P, int kmax, const double2* z, const double* cs,
                const double2* sn, const int32_t* done, double2* rst, hipStream_t st);
// y = R^-1 g per pair (kmax <= 4000: g is staged in LDS)
void ms_backsub(const double2* rst, int P, int kmax, const int32_t* done, const double2* g, double2* y, hipStream_t st);
// x = V y per pair over its done[p] (else K) basis vectors
void ms_xcombine(int R, const double* V, int64_t vstride, int K, const int32_t* done, const double2* y, int P,
                 double2* x, int ldx, int64_t nup, hipStream_t st);

// ---- shared-Krylov solve over a block of polarizations (px_shifted_block.hip)
// One block Arnoldi process for R = npol in {2, 3} right-hand sides; Hbar
// dense row-major with ldh = kcap R; pairs p = w R + l; see px_shifted_block.hip.
void msb_init(int R, const double2* b, int ldb, double* u, int64_t nup, hipStream_t st);
// One delayed block CGS2 step k (block column k-1 corrected, block column k
// first pass, V_k and the next candidate block u written); rho0 receives
// rho_0 (R x R) at k = 0; fix_only: the last block column's correction alone.
void msb_step(int R, double* V, int64_t vstride, int k, double* u, const double* wt, double* part, double* part2,
              double* G, double* Hb, int ldh, double* coefv, double* coefu, double* scal, double* rho0, int64_t nup,
              bool fix_only, hipStream_t st, const int32_t* stop, const hipEvent_t* ev = nullptr);
size_t msb_part_doubles(int R, int kcap);
size_t msb_part2_doubles(int R, int64_t nup, int kcap);
// banded QR columns K0 .. K0+nc-1 (nc <= msb_givens_cols()) of every frequency
int msb_givens_cols();
void msb_givens(int R, const double* Hb, int ldh, int NW, int K0, int nc, const double2* z, double* rc, double2* rs,
                double2* g, const double* rho0, const double* target, int32_t* done, double* resid, int32_t* ndone,
                int32_t* stop, hipStream_t st);
// triangular factors (rst: msb_rst_elems(NW, kcols) complex), back
// substitution (kcols <= 4096) and x = V y over kcols columns
size_t msb_rst_elems(int NW, int kcols);
// The basis (kcols columns in the block layout) as a row-major [nup][ldw]
// matrix (columns kcols..ldw-1 zero), and a product Z [nup][ldz] with it back
// in the block layout; x = V y per pair over its done[p] (else kcols) columns
// for any basis in that layout.
void msb_basis_gather(int R, const double* V, int64_t vstride, int kcols, int64_t nup, double* W, int ldw,
                      hipStream_t st);
void msb_basis_scatter(int R, const double* Z, int ldz, int kcols, int64_t nup, double* TV, int64_t vstride,
                       hipStream_t st);
void msb_xcombine(int R, const double* V, int64_t vstride, int kcols, const int32_t* done, const double2* y, int P,
                  double2* x, int ldx, int64_t nup, hipStream_t st);
void msb_finish_solve(int R, const double* Hb, int ldh, int NW, int kcols, const double2* z, const double* rc,
                      const double2* rs, const int32_t* done, double2* rst, const double2* g, double2* y,
                      const double* V, int64_t vstride, double2* x, int ldx, int64_t nup, hipStream_t st);

}  // namespace px
