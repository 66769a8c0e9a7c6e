/*
 * plasmonx.h -- C ABI of the MI355X (gfx950) frequency-domain solver for the
 * atomistic omegaFQ and omegaFQFmu plasmonics models (plasmonX paper,
 * arXiv 2510.12731, Sections 2.1, 2.2, 6 and 7).
 *
 * One call sequence per nanostructure:
 *   pxCreateStructure  -> geometry, neighbour list, Kbar (Eqs. kappa, kappa_bar, fermi)
 *   pxSetFrequencies   -> frequency grid, polarizations, field amplitude
 *   pxSolveSpectrum    -> solve Eq. (wfq-system) / Eq. (wfqfmu-system) for every
 *                         (frequency, polarization) column by blocked GMRES
 *                         (Section 6, "iterative on the fly")
 *   pxGetCharges / pxGetSpectrum / pxGetSolveStats -> results (Section 7)
 *   pxInducedField / pxProbeField -> induced field and density at probe points
 *                         (Section "Post-process Analysis")
 *   pxDestroyStructure
 *
 * Conventions
 *   - Every call returns pxStatus; nothing throws across this boundary.  On a
 *     non-OK status pxLastError() returns a thread-local description.
 *   - Coordinates are in Angstrom (the paper's input unit), frequencies in eV,
 *     everything else in Hartree atomic units unless the field name says so.
 *   - Complex numbers are interleaved (re, im) doubles.
 *   - All caller buffers are host memory, read (inputs) or written (outputs)
 *     before the call returns; the library copies what it keeps (the device
 *     arrays of pxApplyOperatorNoAlloc aside).  Device memory comes from
 *     hipMalloc, or from the caller's allocator once pxSetAllocator installed
 *     one (the Python binding offers the framework's caching allocator); a
 *     structure's memory is released by pxDestroyStructure.
 *   - Outputs are in the caller's atom order.
 *   - A handle is not thread-safe; distinct handles may be used concurrently
 *     from different threads.
 *   - Streams: each structure's device work is ordered on the HIP stream given
 *     at creation (NULL = the default stream): it starts after the work the
 *     caller queued on that stream before the call, and work the caller
 *     queues after a call returns sees its results.  A solve drives restart
 *     cycles and convergence checks from the host, so pxSolveSpectrum,
 *     pxSolveBatch and pxServerStep return only once their steps are done (a
 *     solve is not left running on the stream; the server's pxServerStep is
 *     the way to interleave solves with other host work).  Inside a solve
 *     the library may also use streams of its own (default priority), joined
 *     back to the structure's stream before the call returns.  pxGet*
 *     synchronise the structure's stream.
 *   - Unknown order of the dipole model: [q_0..q_{N-1} | mu_x | mu_y | mu_z].
 */
#ifndef PLASMONX_H
#define PLASMONX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PX_OK = 0,
    PX_E_INVALID = 1,   /* bad argument: NaN/Inf or coincident atoms, omega <= 0, tau <= 0, ... */
    PX_E_OOM = 2,       /* device allocation failed or the memory budget would be exceeded */
    PX_E_NOTCONV = 3,   /* some columns missed rel_tol; results readable, see pxGetSolveStats */
    PX_E_DEVICE = 4,    /* HIP runtime error or the library was built for another device */
    PX_E_STATE = 5      /* call out of order (e.g. results before a solve) */
} pxStatus;

typedef enum { PX_WFQ = 0, PX_WFQFMU = 1, PX_BEM = 2 } pxModel;

typedef enum {
    PX_FP64 = 0,   /* every step in FP64 */
    PX_MIXED = 1   /* the blocked GMRES cycles apply T in FP32 on MFMA; FP64
                      Arnoldi, Givens, solution update and true residual
                      (iterative refinement).  The shared-Krylov phase
                      (pxSolveOptions.shifted) is FP64 either way: PX_MIXED
                      changes only the cycles of the columns that phase leaves
                      above rel_tol, and every cycle of shifted = 0 */
} pxPrecision;

typedef enum {
    PX_TAPPLY_AUTO = 0,        /* the autotuner times both methods per shape and keeps the faster */
    PX_TAPPLY_ON_THE_FLY = 1,  /* T generated in registers by the hand-written kernels */
    PX_TAPPLY_STORED = 2       /* dense T stored once per structure, one hand-written product per apply */
} pxTApply;

typedef enum {
    PX_ORTHO_CGS2 = 0,   /* classical Gram-Schmidt, two passes per Arnoldi step */
    PX_ORTHO_DCGS2 = 1   /* the second pass delayed into the next step */
} pxOrtho;

/* Material parameters of one homogeneous nanostructure.
 *   a_eff            effective area A of Eq. (kappa), bohr^2
 *   r_q, r_mu        Gaussian widths of charges (Eq. tqq) and dipoles, bohr
 *   tau              Drude scattering time of Eq. (z_q_wfq), a.u.
 *   density, eff_mass  n and m* (a.u.); the Drude weight entering z_q is n/m*
 *   fermi_d, fermi_s  d and s of Eq. (fermi)
 *   r0_ang           nearest-neighbour distance r^0 of Eq. (fermi), Angstrom
 *   cutoff_ang       charge exchange is kept for pairs with r_ij <= cutoff, Angstrom
 *   fermi_energy_ev  > 0 selects the graphene reading of the Drude weight,
 *                    E_F / (pi * sheet_thickness) (Eq. 2d-eff-mass with the
 *                    Dirac-cone density); 0 for metals
 *   sheet_thickness  effective graphene thickness, bohr (used iff fermi_energy_ev > 0)
 */
typedef struct {
    double a_eff;
    double r_q;
    double r_mu;
    double tau;
    double density;
    double eff_mass;
    double fermi_d;
    double fermi_s;
    double r0_ang;
    double cutoff_ang;
    double fermi_energy_ev;
    double sheet_thickness;
} pxMaterial;

/* Solver options (pxDefaultSolveOptions fills the defaults shown).
 *   precision        PX_FP64 (default) or PX_MIXED (see pxPrecision)
 *   restart_m        GMRES restart length m at the start (100)
 *   max_restart_m    the restart length doubles, up to this value, whenever
 *                    some column's true residual fell by less than 30 % over
 *                    its last cycle (restarted GMRES stagnates at the sharp
 *                    plasmon resonances); <= restart_m keeps m fixed (200)
 *   rel_tol          per column ||b - A x||_2 / ||b||_2 target (1e-8)
 *   max_cycles       maximum number of restart cycles per column (400)
 *   max_block_cols   columns solved together in one block; 0 = all (0).
 *                    1 gives the one-column-at-a-time solver.
 *   inner_reduction  mixed precision: a cycle stops for a column once its
 *                    estimated residual fell by this factor (1e-5); 0 = only
 *                    the rel_tol target stops it
 *   timings          1 = time each phase with HIP events, sampled
 *                    (pxGetTimings) (0)
 *   block_cols       columns per segment of the stacked multi-structure block
 *                    used by pxSolveBatch and the server (multiple of 64;
 *                    0 = 64)
 *   stall_cycles     a column is given up (and reported unconverged) after
 *                    this many consecutive cycles that each removed less than
 *                    2 % of its true residual; 0 = never (8)
 *   ortho            Arnoldi orthogonalisation: PX_ORTHO_DCGS2 (default),
 *                    classical Gram-Schmidt twice with the second pass delayed
 *                    into the next step (one dot and one update pass over the
 *                    basis per step), or PX_ORTHO_CGS2, both passes in the
 *                    same step (two of each)
 *   graph_steps      pxSolveBatch and the server with PX_ORTHO_DCGS2: the
 *                    Arnoldi steps of a cycle are captured into HIP graphs of
 *                    this many steps, once per block layout and restart
 *                    length, and replayed; 0 launches every kernel directly.
 *                    In [0, 64] (8).  pxSolveSpectrum ignores it (its block
 *                    layout changes at nearly every restart as columns retire).
 *   t_apply          how pxSolveSpectrum applies T in its cycles and true
 *                    residuals: PX_TAPPLY_AUTO (default) times, on the
 *                    structure itself, the on-the-fly kernels and the
 *                    hand-written products with T stored densely (the
 *                    paper's in-memory solver; N_u^2 x 4 B in FP32,
 *                    x 8 B in FP64, only when that fits a quarter of the free
 *                    device memory) the first time a (model, atoms, columns,
 *                    precision) shape occurs in the process, and keeps the
 *                    faster; PX_TAPPLY_ON_THE_FLY / PX_TAPPLY_STORED force one
 *                    (STORED fails with PX_E_OOM if T does not fit).  Under
 *                    AUTO a stored FP64 T above 256 MiB is not tried for the
 *                    narrow (1-8 column) apply of the shared phase, and a
 *                    solve's first true residual builds no dense T unless a
 *                    block kept from an earlier solve serves it (or, once per
 *                    new shape up to 4 GiB, to tune it).
 *                    The stacked block of pxSolveBatch and the server always
 *                    generates T on the fly.
 *   shifted          pxSolveSpectrum on a one-material PX_WFQ structure: 1
 *                    first runs one real Arnoldi process on Kbar T
 *                    per polarization, in FP64, and takes every frequency's
 *                    GMRES iterate from it (the right-hand side does not depend
 *                    on the frequency and the frequency only shifts the
 *                    operator, so all frequencies share one Krylov space);
 *                    columns it leaves above rel_tol continue in the blocked
 *                    solver from its iterate (the phase counts as one cycle).
 *                    A pair stops once its GMRES residual estimate is below
 *                    0.9 rel_tol.
 *                    2 (default): one block Arnoldi process over the polarizations
 *                    instead (2 or 3 polarizations with non-zero right-hand
 *                    sides, else as 1): the block Krylov space of all
 *                    right-hand sides holds each polarization's own space, so
 *                    every pair minimises its residual over all of it (fewer
 *                    steps for the same tolerance, each one T-apply of the
 *                    same vectors); one banded QR per frequency serves its
 *                    polarizations; steps at most min(shifted_max_steps,
 *                    4096 / npol).
 *                    0 = blocked solver only.  Ignored for PX_WFQFMU and
 *                    two-type structures.  pxSolveBatch and the server solve
 *                    the structures it applies to, and every structure of
 *                    1024 atoms or more, whole (as pxSolveSpectrum does), a
 *                    few steps of each in turn on streams of their own,
 *                    beside the stacked block that takes the others.
 *   shifted_max_steps  Arnoldi steps of that phase at most, in [1, 4000]
 *                    (2000; lowered to keep its basis and the frequencies'
 *                    triangular factors, k^2/2 x 16 B per column, within a
 *                    quarter of the free device memory)
 */
typedef struct {
    int32_t precision;
    int32_t restart_m;
    double rel_tol;
    int32_t max_cycles;
    int32_t max_block_cols;
    double inner_reduction;
    int32_t timings;
    int32_t stall_cycles;
    int32_t max_restart_m;
    int32_t block_cols;
    int32_t ortho;
    int32_t graph_steps;
    int32_t t_apply;
    int32_t shifted;
    int32_t shifted_max_steps;
} pxSolveOptions;

typedef struct pxStructure_t* pxStructure;

/* Fills *opt with the defaults listed above. */
void pxDefaultSolveOptions(pxSolveOptions* opt);

/* Creates a nanostructure from n_atoms coordinates (xyz_ang: n_atoms x 3,
 * row-major, Angstrom, copied).  Builds on the device: the Morton order of the
 * atoms, the neighbour list within cutoff_ang and the CSR matrix Kbar
 * (Eqs. fermi, kappa, kappa_bar).  hip_stream: a hipStream_t or NULL.
 * Errors: PX_E_INVALID for n_atoms < 1, non-finite coordinates, two atoms
 * closer than 1e-6 Angstrom, or non-positive a_eff, r_q, tau, Drude weight,
 * r0 or cutoff (r_mu > 0 required for PX_WFQFMU); PX_E_OOM; PX_E_DEVICE. */
pxStatus pxCreateStructure(pxModel model, int64_t n_atoms, const double* xyz_ang, const pxMaterial* mat,
                           void* hip_stream, pxStructure* out);

/* Creates a structure of two atom types (Section 2.2, Eqs. wfqfmu-leghe and
 * polar-finale: alloys, core-shell particles): types[n_atoms] (copied) holds 0
 * for an atom of mat_a and 1 for one of mat_b.  The charge rows solve
 * S(w) T q - z_q,i q_i = -S(w) V with S = (Kbar + Hbar(w)) / 2, where Hbar
 * carries the exchange back through the ratio of the two atoms' Drude factors
 * 2 n tau / (1 - i w tau); z_q,i is the z_q of atom i's type.  Like pairs
 * exchange with their material's A, r0, d, s and cutoff, unlike pairs with
 * the mean of the two; the dipole rows use the per-atom interband
 * polarizability of Eq. (polar-finale) with the neighbours within the
 * exchange cutoff.  Both materials must have the same r_q (and r_mu for
 * PX_WFQFMU): T is that of one material.  Such a structure is solved with
 * pxSolveSpectrum; pxSolveBatch and the server refuse it (PX_E_INVALID).
 * Errors as pxCreateStructure, and PX_E_INVALID for a type other than 0 or 1
 * or for different widths. */
pxStatus pxCreateStructureHetero(pxModel model, int64_t n_atoms, const double* xyz_ang, const uint8_t* types,
                                 const pxMaterial* mat_a, const pxMaterial* mat_b, void* hip_stream,
                                 pxStructure* out);

/* Creates a BEM structure in the DPCM formulation (Section 2.3, Eq.
 * bem-dpcm, the "approximate" F): a closed surface mesh of n_tess tesserae
 * with barycentres cen_ang (n_tess x 3, Angstrom), outward normals normals
 * (n_tess x 3, normalised here) and areas area_ang2 (Angstrom^2), all copied;
 * r_enc_ang is the radius of the sphere enclosing the mesh (the R of F's
 * diagonal); eps_env (2 doubles, complex; NULL = vacuum) is the medium's
 * permittivity eps1.  The unknowns are the tessera charges q_i (pxGetCharges
 * returns them in the caller's tessera order) and the solved system is
 *   [ M - 2 pi (eps2 + eps1) / (eps2 - eps1) I ] q = -A E_n,
 *   M_ij = A_i (s_i - s_j).n_i / |s_i - s_j|^3, M_ii = 1.0694 sqrt(4 pi A_i) / (2R),
 * with E_n,i = E0 e_l . n_i; d = sum_i q_i (s_i - c) (Section 7, c the
 * area-weighted centroid of the tesserae: the discrete charges are neutral
 * only up to the discretization, so the dipole's origin is fixed on the mesh)
 * and alpha, sigma_abs as for the atomistic models.  pxSetFrequencies takes the metal permittivity
 * eps2(omega_w) per frequency in its alpha_ib argument (2 * n_omega doubles,
 * interleaved complex, != eps1).  M is real and the same at every frequency,
 * so pxSolveSpectrum (shifted >= 1) runs the shared-Krylov phase over all
 * frequencies, then the true FP64 residual of every column; M is generated on
 * the fly in FP64 (t_apply is ignored; PX_MIXED runs the FP64 apply).
 * pxApplyOperator (PX_FP64 only) and pxApplyOperatorNoAlloc take eps2 per
 * column in alpha_ib; pxInducedField and pxProbeField refuse a BEM structure;
 * pxSolveBatch and the server solve it whole (shifted >= 1, else
 * PX_E_INVALID).  Errors: PX_E_INVALID for n_tess < 1, non-finite inputs, a
 * zero normal, an area <= 0 or r_enc <= 0; barycentres must be distinct.
 * PX_E_OOM; PX_E_DEVICE. */
pxStatus pxCreateBem(int64_t n_tess, const double* cen_ang, const double* normals, const double* area_ang2,
                     double r_enc_ang, const double* eps_env, void* hip_stream, pxStructure* out);

/* Creates a BEM structure in the IEFPCM formulation (Section 2.3, Eq.
 * bem-iefpcm, the "approximate" F), with the arguments, ownership and errors
 * of pxCreateBem.  The paper's matrices, for the tessera charges q:
 *   [ 2 pi f I + F ] S A^-1 q = -(2 pi I + F) V,  f = (eps2 + eps1) / (eps2 - eps1),
 *   S_ij = A_j / |s_i - s_j|, S_ii = 1.0694 sqrt(4 pi A_i),
 *   F_ij = A_j (s_i - s_j).n_j / |s_i - s_j|^3, F_ii = -1.0694 sqrt(4 pi A_i) / (2R),
 *   V_i = -E0 (s_i - c)_l (the applied field's potential), d = sum_i q_i (s_i - c),
 * with c the area-weighted centroid of the tesserae: a constant in V drops
 * out of the continuous equation but not of the discrete one, so V's zero is
 * put at c and the result does not depend on where the mesh sits.
 * F's diagonal is the double layer's self patch on a sphere (negative; the
 * printed positive value belongs to the DPCM operator).  The solver's unknown
 * is the potential y = S A^-1 q of every column, from [F - z I] y = b with
 * z = -2 pi f, so pxSolveSpectrum (shifted >= 1) runs the shared-Krylov
 * phase as for DPCM, rel_tol and pxGetSolveStats refer to this system, and
 * pxApplyOperator / pxApplyOperatorNoAlloc apply y -> [F + 2 pi f I] y.  The
 * creation also solves S A^-1 w_k = s_k (k = x, y, z; conjugate gradients to
 * 1e-12) so that d_k = w_k . y without the charges (S A^-1 is symmetric);
 * pxGetCharges solves S A^-1 q = y for its column the same way (one solve per
 * call, PX_E_NOTCONV if it stalls).  Extra errors: PX_E_NOTCONV if the
 * creation's solve does not converge, PX_E_INVALID if S A^-1 is not positive
 * definite on the mesh. */
pxStatus pxCreateBemIefpcm(int64_t n_tess, const double* cen_ang, const double* normals, const double* area_ang2,
                           double r_enc_ang, const double* eps_env, void* hip_stream, pxStructure* out);

/* Sets the frequency grid (omega_ev[n_omega], > 0, copied), the polarizations
 * (pol_mask bit0 = x, bit1 = y, bit2 = z; one column per set bit and
 * frequency, frequency-major) and the field amplitude e0_au (> 0; the paper
 * uses 1e-4).  alpha_ib: 2*n_omega interleaved complex interband
 * polarizabilities alpha^IB(omega) (bohr^3) of Eq. (z-mu), required for
 * PX_WFQFMU and ignored for PX_WFQ.  For a two-type structure alpha_ib holds
 * 4*n_omega doubles: per frequency alpha^IB of mat_a, then of mat_b (each
 * interleaved complex).  Discards previous results. */
pxStatus pxSetFrequencies(pxStructure s, int32_t n_omega, const double* omega_ev, uint32_t pol_mask,
                          double e0_au, const double* alpha_ib);

/* Solves all columns (synchronously: the call returns when the solve is
 * done).  opt may be NULL (defaults).  Returns PX_E_NOTCONV if any column
 * missed rel_tol within max_cycles (results stay readable). */
pxStatus pxSolveSpectrum(pxStructure s, const pxSolveOptions* opt);

/* The same solve, started without waiting for it: the call enqueues the
 * solve's first steps on the structure's stream and returns.  The solve's
 * restart and convergence decisions are taken on the host, so it advances
 * only inside later calls: pxSolveProgress enqueues what it can without
 * waiting for the device (call it between other host work), pxSolveWait
 * drives it to the end, and every other call on the structure (pxGet*,
 * pxSetFrequencies, another solve, pxApplyOperator, the probe fields,
 * pxSolveBatch, pxServerSubmit, pxSolveFootprint) first completes it.
 * pxDestroyStructure abandons a solve in progress once the device is idle.
 * Errors: as pxSolveSpectrum for the arguments (PX_E_STATE without
 * frequencies, PX_E_INVALID for bad options); PX_E_OOM / PX_E_DEVICE from the
 * first steps. */
pxStatus pxSolveSpectrumAsync(pxStructure s, const pxSolveOptions* opt);

/* Advances an asynchronous solve without waiting for the device; *done = 1
 * once it has finished (also when none was started), else 0.  The solve's
 * status is then read with pxGetSolveStatus (or pxSolveWait).  Errors:
 * PX_E_INVALID for null arguments; PX_E_DEVICE / PX_E_OOM if the solve failed
 * (it is dropped). */
pxStatus pxSolveProgress(pxStructure s, int32_t* done);

/* Completes an asynchronous solve (returns at once if none is in progress)
 * and returns the status of the structure's last solve: PX_OK, PX_E_NOTCONV
 * (results readable), or the error that ended it. */
pxStatus pxSolveWait(pxStructure s);

/* Solves several structures together (all must use the same HIP stream, have
 * their frequencies set, and appear once).  One-material PX_WFQ structures
 * with opt->shifted >= 1 (default 2), and every structure of 1024 atoms or
 * more, are solved whole, each as by pxSolveSpectrum, up to four at a time,
 * each on a HIP stream of its own (default priority, ordered after the
 * structures' stream): the calling thread enqueues a few steps of each in
 * turn without waiting for the device, so their launches overlap; the library
 * starts no host threads.  Every other structure's columns are cut into
 * segments of opt->block_cols columns; the segments of all of them form one
 * stacked block whose Arnoldi steps run as single grouped launches (one
 * T-apply over a tile list covering every structure, one sparse apply, one
 * pass of each orthogonalisation kernel), with segments retiring at restart
 * boundaries.  Results are read per structure with pxGet*; each structure's
 * own status and message with pxGetSolveStatus.  Returns the worst status
 * (a device or memory failure before PX_E_NOTCONV) with the first failing
 * structure's message; the other structures' results stay valid. */
pxStatus pxSolveBatch(const pxStructure* s, int32_t n, const pxSolveOptions* opt);

/* ---- continuous batching ----------------------------------------------------
 * A server keeps one stacked block resident on the device and runs restart
 * cycles over it, and beside it solves up to four larger requests whole, each
 * on a stream of its own, a few steps per pxServerStep.  Requests submitted
 * while others are being solved are admitted by HBM footprint as memory
 * frees up (first come, first served within each kind); finished stacked
 * requests leave at cycle boundaries, so requests of different sizes overlap
 * on the device.  Structures stay owned by the caller and must outlive their
 * time in the server; their results are read with pxGet* once pxServerStep
 * returned them, their status with pxGetSolveStatus.  Calls on one server are
 * not thread-safe; the library starts no host threads. */
typedef struct pxServer_t* pxServer;

/* memory_budget_bytes bounds the resident storage of the admitted requests:
 * the stacked block's rows in use times its bytes per row (the basis of the
 * largest restart length and the block's vectors) plus the footprints of the
 * whole solves in flight (pxSolveFootprint).  The stacked block's storage for
 * its full row capacity (the budget over the bytes per row) is allocated at
 * creation; the whole solves allocate theirs when admitted, so the device
 * holds at most about twice the budget.  opt as for pxSolveSpectrum (may be
 * NULL), including block_cols.  The stream is the one every submitted
 * structure must use. */
pxStatus pxServerCreate(double memory_budget_bytes, const pxSolveOptions* opt, void* hip_stream, pxServer* out);

/* Queues a structure whose frequencies are set.  PX_E_OOM if it can never fit
 * the budget; PX_E_INVALID for a different stream.  A structure of 1024
 * atoms or more, or (opt->shifted >= 1) a one-material PX_WFQ structure, is
 * solved whole once admitted; the others join the stacked block. */
pxStatus pxServerSubmit(pxServer sv, pxStructure s);

/* Admits queued structures that fit the budget, advances the whole solves by
 * a few steps each, runs one restart cycle of the stacked block, and writes up
 * to max_finished structures that completed (converged or not, or failed:
 * see pxGetSolveStatus) into finished[] (*n_finished of them; more are
 * returned by later calls).  With only whole solves in flight and none
 * finished it waits for the device instead of returning at once. */
pxStatus pxServerStep(pxServer sv, pxStructure* finished, int32_t max_finished, int32_t* n_finished);

/* Queue length (both kinds), structures in flight (stacked block and whole
 * solves), rows of the stacked block in use and its row capacity. */
pxStatus pxServerQuery(pxServer sv, int32_t* n_queued, int32_t* n_active, int64_t* rows_in_use,
                       int64_t* rows_capacity);

/* Bytes charged against the budget (stacked rows in use times bytes per row
 * plus the admitted whole solves' footprints), the budget, and the number of
 * whole solves in flight.  Any pointer may be NULL. */
pxStatus pxServerMemory(pxServer sv, double* bytes_in_use, double* budget_bytes, int32_t* n_whole);

void pxServerDestroy(pxServer sv);

/* HBM footprint (bytes) of solving s whole with the options opt (NULL:
 * defaults): the active column block's vectors and T-apply scratch, the
 * near-field list, a stored T the tuner may build (FP64 up to 4 GiB, FP32
 * for PX_MIXED; kept by the structure), and the shared-Krylov phase's basis,
 * factors and true-residual buffers at opt->shifted_max_steps or the blocked
 * solver's basis at max_restart_m; the figure the server admits whole solves
 * by.  PX_E_STATE before pxSetFrequencies. */
pxStatus pxSolveFootprint(pxStructure s, const pxSolveOptions* opt, double* bytes);

/* Status of the structure's last solve (pxSolveSpectrum, pxSolveBatch or the
 * server: PX_OK, PX_E_NOTCONV, PX_E_OOM, PX_E_DEVICE; PX_E_STATE while not
 * solved) and its message, copied into message[message_len] (NUL-terminated,
 * truncated; message may be NULL). */
pxStatus pxGetSolveStatus(pxStructure s, int32_t* status, char* message, int32_t message_len);

/* Induced charges q (2*n_atoms doubles) and, for PX_WFQFMU, dipoles mu
 * (6*n_atoms doubles: mu_x, mu_y, mu_z blocks) of column (i_omega, pol) in
 * the caller's atom order; pol is 0, 1 or 2 and must be in pol_mask.  mu may
 * be NULL.  PX_E_STATE before a solve. */
pxStatus pxGetCharges(pxStructure s, int32_t i_omega, int32_t pol, double* q, double* mu);

/* Polarizability alpha[n_omega][3][3] (interleaved complex, alpha[k][l] =
 * d_k / E_l, zero for unsolved l) and absorption cross section
 * sigma_abs[n_omega] (bohr^2): (4 pi omega / c) times the mean of Im alpha_ll
 * over the solved polarizations, i.e. the paper's (4 pi omega / 3c) Tr Im alpha
 * when all three are solved.  Either pointer may be NULL. */
pxStatus pxGetSpectrum(pxStructure s, double* alpha, double* sigma_abs);

/* Per column (frequency-major, n_omega * n_pol entries): GMRES iterations,
 * restart cycles and final true relative residual ||b - A x|| / ||b||
 * (recomputed in FP64).  Any pointer may be NULL. */
pxStatus pxGetSolveStats(pxStructure s, int32_t* iterations, int32_t* cycles, double* rel_res);

/* Applies the operator of the solved system, y_c = A(omega_c) x_c, to ncol
 * complex columns (x, y: [ncol][n_unknowns] interleaved complex, caller atom
 * order), column c at frequency omega_ev[c] (and alpha_ib[c] for PX_WFQFMU:
 * 2 doubles per column, 4 for a two-type structure as in pxSetFrequencies),
 * in the requested precision, with the same kernels the solver uses.  The
 * dipole rows are those of Eq. (wfqfmu-system), not negated. */
pxStatus pxApplyOperator(pxStructure s, int32_t precision, int32_t ncol, const double* omega_ev,
                         const double* alpha_ib, const double* x, double* y);

/* Device memory.  alloc(bytes, device, user) returns at least bytes of
 * device memory on that device (the current one), 256-byte aligned, or NULL
 * when none is left (the library call then fails with PX_E_OOM);
 * free(ptr, device, user) gives back a block that alloc returned.  The
 * library waits for the device after alloc returns and before it calls free,
 * so the allocator may hand out a block whose previous user's work is still
 * queued on some stream, and may reuse a freed block at once.  Every device
 * allocation of the library goes through it (structures, solve workspaces,
 * stored T), except the fixed array of pxApplyOperatorNoAlloc; each block
 * goes back to the allocator that made it, also after a later
 * pxSetAllocator.  alloc = free = NULL restores hipMalloc/hipFree.  With an
 * allocator installed the library keeps no freed blocks of its own: the
 * blocks it keeps for reuse between solves are released and later ones are
 * given back at once.  The callbacks run on the thread that made the
 * library call.  Errors: PX_E_INVALID if exactly one of alloc and free is
 * NULL. */
typedef void* (*pxDeviceAllocFn)(size_t bytes, int32_t device, void* user);
typedef void (*pxDeviceFreeFn)(void* ptr, int32_t device, void* user);
pxStatus pxSetAllocator(pxDeviceAllocFn alloc, pxDeviceFreeFn free, void* user);

/* Frees the device blocks the library keeps for reuse between solves (solve
 * workspaces and stored T of at least 16 MiB, up to 24 GiB in all, with
 * hipMalloc as the allocator).  Blocks in use are not touched. */
pxStatus pxReleaseCache(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * pxApplyOperator, y_c = A(omega_c) x_c for 1 <= ncol <= 4 columns, with x
 * and y in DEVICE memory ([ncol][n_unknowns] interleaved complex, caller atom
 * order, as pxApplyOperator's host arrays), the same kernels and the same
 * result as pxApplyOperator with PX_FP64.  Its scratch (the permuted columns,
 * T x, the operator's result before un-permuting, the narrow T-apply's split
 * partial sums and the shifts) lives in a fixed 128 MiB device array of the
 * library, one per GPU, held until the process ends; the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).  Runs on the
 * structure's stream and returns once y is written.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller.  Errors: PX_E_INVALID
 * for a null pointer, ncol outside [1, 4], omega <= 0 or a missing alpha_ib
 * (PX_WFQFMU); PX_E_OOM, with the sizes in the message, when the structure
 * needs more scratch than the array holds (e.g. ncol = 4 on a 20k-atom
 * PX_WFQFMU structure); PX_E_DEVICE. */
pxStatus pxApplyOperatorNoAlloc(pxStructure s, int32_t ncol, const double* omega_ev, const double* alpha_ib,
                                const double* x, double* y);

/* Number of unknowns (n_atoms or 4 n_atoms) and of atoms. */
pxStatus pxGetSize(pxStructure s, int64_t* n_atoms, int64_t* n_unknowns);

/* Measurements of the last solve.
 * ms6 (may be NULL): [0] wall time of the solve; with options.timings = 1 the
 * HIP-event times summed over all Arnoldi steps of [1] the FP32 T-apply, [2]
 * the FP64 T-apply inside cycles, [3] the sparse Kbar apply, [4] the
 * orthogonalisation/Givens kernels, and [5] the remainder (residuals,
 * updates, host work); zeros otherwise.  Only every 16th Arnoldi step of a
 * cycle or of the shared-Krylov phase is timed (an event costs a few
 * microseconds of stream time) and the sampled steps' mean is scaled to all
 * steps; the shared phase's Givens kernels run on a second stream and count in
 * [5] only where they delay the main stream.
 * counts6 (may be NULL): [0] FP32 T-apply launches, [1] real columns they
 * processed including padding, [2] real columns without padding; [3..5] the
 * same for the FP64 T-apply (inside cycles and true residuals). */
pxStatus pxGetTimings(pxStructure s, double* ms6, int64_t* counts6);

/* Algorithmic work of the last pxSolveSpectrum (the method's own work, no
 * padding, no re-reads): work3[0] FLOP of the FP32 T-apply (2 N_u^2 per real
 * column and Arnoldi step), work3[1] FLOP of the FP64 T-apply (steps of FP64
 * cycles and true residuals), work3[2] HBM bytes of the bandwidth-bound
 * phases: per step and column the sparse apply (N_u x 40 B: FP32 T X, FP64
 * X, FP64 result), the orthogonalisation (one dot and one update pass:
 * N_u x 16 B x (2k + 6) at step k; two of each for CGS2: N_u x 16 B x
 * (4k + 10)) and the normalisation (N_u x 40 B); per cycle the residual's
 * vector traffic (N_u x 80 B) and the solution update (N_u x 16 B x
 * (steps + 2)).  N_u = unknowns (atoms, or 4 x atoms for PX_WFQFMU).
 * Dividing each by its peak gives the ideal time of the solve. */
pxStatus pxGetWork(pxStructure s, double* work3);

/* T-apply of the last pxSolveSpectrum by method (autotuner or options):
 * launches4 (may be NULL) [0] FP32 on the fly, [1] FP32 stored T, [2] FP64 on
 * the fly, [3] FP64 stored T (cycles and true residuals); ms4 (may be NULL)
 * the HIP-event milliseconds of the same launches inside cycles (zeros unless
 * options.timings = 1; true residuals are not timed); flop4 (may be NULL)
 * their algorithmic FLOP inside cycles (2 N_u^2 per real column of a column
 * that was still iterating). */
pxStatus pxGetTApplyStats(pxStructure s, int64_t* launches4, double* ms4, double* flop4);

/* Post-processing (Section "Post-process Analysis"): the electric field and
 * the charge density of induced charges (and, for PX_WFQFMU, dipoles) at
 * probe points, for CUBE grids and plane maps.  The charges are the model's
 * Gaussians (Section 2): a charge q at r_i contributes the density
 * q exp(-r^2/R_q^2) / (pi^{3/2} R_q^3) and the field q g(r) d / r^3, with
 * d = p - r_i, r = |d|, g(r) = erf(r/R_q) - (2/sqrt(pi)) (r/R_q)
 * exp(-(r/R_q)^2); a dipole mu (width R_mu) the density -mu . grad of its
 * Gaussian and the field -grad [mu . d g(r; R_mu) / r^3].  Points may lie
 * anywhere, atom centres included.
 *   pxInducedField: the sources of the solved column (i_omega, pol) of s
 *     (after pxSolveSpectrum; the field per E0 of pxSetFrequencies).
 *   pxProbeField: caller-given sources on s's atoms, caller's atom order:
 *     q [n_atoms] complex; mu [3 n_atoms] complex, component-major
 *     ([mu_x | mu_y | mu_z], the layout of pxGetCharges), PX_WFQFMU only
 *     (NULL there leaves the dipoles out; must be NULL for PX_WFQ).
 * pts_ang: [npts][3] host, Angstrom.  field (may be NULL): [npts][3] complex
 * (E_x, E_y, E_z), Hartree / (e bohr); density (may be NULL): [npts] complex,
 * e / bohr^3.  The work is npts x n_atoms pair evaluations; points in spatial
 * order (grid lines, planes) run fastest.  Device buffers for the points and
 * results are allocated and released inside the call (points in batches of
 * 2^20; for 4096 atoms or more each batch is evaluated in Morton order and
 * returned in the caller's order);
 * synchronises s's stream.  Errors: PX_E_INVALID (null s, pts with npts > 0
 * or q; npts < 0; a non-finite point; a column outside the solved set; mu for
 * PX_WFQ),
 * PX_E_STATE (pxInducedField before a solve), PX_E_OOM, PX_E_DEVICE. */
pxStatus pxInducedField(pxStructure s, int32_t i_omega, int32_t pol, int64_t npts, const double* pts_ang,
                        double* field, double* density);
pxStatus pxProbeField(pxStructure s, const double* q, const double* mu, int64_t npts, const double* pts_ang,
                      double* field, double* density);

/* The last pxInducedField / pxProbeField call of s: out2[0] HIP-event
 * milliseconds of its probe kernels (the field and density sums, without the
 * copies), out2[1] its pair evaluations (npts x n_atoms). */
pxStatus pxGetProbeStats(pxStructure s, double* out2);

void pxDestroyStructure(pxStructure s);

/* Thread-local description of the last error of this thread ("" if none). */
const char* pxLastError(void);

#ifdef __cplusplus
}
#endif

#endif /* PLASMONX_H */
