"""Benchmark: omegaFQ frequency solves per second on a 20,000-atom Ag sphere.

Workload (one "step" = the whole path once): an Ag fcc sphere of 20,000 atoms,
128 frequencies 2-5 eV x 3 polarizations = 384 (frequency, polarization)
columns, each driven to a true relative residual of 1e-8 (recomputed in
FP64).  A step creates the structure on the GPU (neighbour list, Kbar,
near-field list), sets the frequencies, solves (the shared-Krylov phase: one
FP64 block Arnoldi process over the three polarizations serves every
frequency, then every column's true FP64 residual) and reads the spectrum
back; the inputs are host arrays as they arrive at the C ABI.

Reported next to the headline number (one JSON line):
  * roofline of the dominant kernel (the narrow FP64 T-apply), from HIP-event
    times of its launches on the library's stream, against the FP64 vector peak;
  * the small spectrum (249 atoms x 50 w) against the oracle's direct solve,
    and the oracle residual of sampled columns of the headline spectrum;
  * the plain FP64 solver (one column at a time, sampled) and FP64 blocked,
    the blocked mixed-precision solver, the per-polarization phase;
  * the other workloads: the 10,000-atom Au rod (omegaFQFmu), the 64-structure
    graphene batch, the serving mix, and the BEM sphere;
  * the oracle timed on the host's cores (a bounded sample, scaled).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ensure_built():
    import paper_2510_12731_amd as px
    if not os.path.exists(px.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return px.load()


def one_step(px, case, precision, timings, max_block_cols=0, t_apply=None, shifted=None):
    om = case["omega_ev"]
    s = px.Structure(case["model"], case["xyz"], case["params"], px.default_stream())
    pol = case["pol_mask"]
    s.set_frequencies(om, pol, case["e0"], case["alpha_ib"])
    st = s.solve(precision=precision, rel_tol=1e-8, max_block_cols=max_block_cols, timings=timings,
                 t_apply=t_apply, shifted=shifted)
    alpha, sigma = s.spectrum()
    it, cyc, rr = s.stats()
    tm = s.timings()
    wk = s.work()
    ta = s.tapply_stats()
    s.close()
    return dict(status=st, sigma=sigma, alpha=alpha, iters=it, cycles=cyc, relres=rr, timings=tm, work=wk, tapply=ta)


# FP64 arithmetic per atom pair of the narrow omegaFQ T-apply besides the
# products with the columns: r^2 = |p_i|^2 + |p_j|^2 - 2 p_i.p_j over centred
# positions (one add and three fused multiply-adds, 7; the per-atom -2 p_i and
# |p|^2 are computed once), the reciprocal square root estimate (1) and one
# Newton step to FP64 accuracy (two multiplies and a fused multiply-add, 4);
# each column adds one fused multiply-add (2).
PAIR_FLOP = 12


def tapply_roofline(runs, n, npol, traffic, traffic_note):
    """Roofline of the T-apply method that took the most time in these runs,
    from the HIP-event times the library records around each launch on its
    stream.  FP64 on the fly with a few columns is the narrow omegaFQ kernel
    (point part + stored near-field correction), bound by FP64 vector
    arithmetic; FP32 on the fly and the stored-T GEMMs are MFMA-bound."""
    keys = ("f32_on_the_fly", "f32_stored", "f64_on_the_fly", "f64_stored")
    ms = {k: sum(r["tapply"]["ms_" + k] for r in runs) for k in keys}
    nl = {k: int(sum(r["tapply"][k] for r in runs)) for k in keys}
    dom = max(keys, key=lambda k: ms[k])
    if dom == "f64_on_the_fly":
        fl = float(n) * n * (PAIR_FLOP + 2 * npol) * nl[dom]
        peak, bound, kname = FP64_VECTOR_PEAK_TFLOPS, "alu", \
            "k_tapply_f64_narrow_q (point part and stored near-field correction) + k_sum_splits (split sum), FP64"
        flop_note = (f"{PAIR_FLOP} + 2 x {npol} FP64 FLOP per atom pair (N^2 pairs; the near-field list adds "
                     f"< 1 %), peak = FP64 vector")
    else:
        fl = sum(r["tapply"]["flop_" + dom] for r in runs)
        f32 = dom.startswith("f32")
        peak, bound = (FP32_MFMA_PEAK_TFLOPS if f32 else FP64_MFMA_PEAK_TFLOPS), "mfma"
        kname = {"f32_on_the_fly": "k_tapply_wfq_f32 (+ k_sk_fixup), T generated on the fly",
                 "f32_stored": "k_tstored_f32 (+ k_sk_fixup) on the stored T",
                 "f64_stored": "k_tstored_f64 / k_tstored_narrow on the stored T"}[dom]
        flop_note = "2 N^2 FLOP per real column still iterating, peak = matrix"
    achieved = fl / (ms[dom] * 1e-3) / 1e12 if ms[dom] > 0 else 0.0
    return dict(bound=bound, achieved=round(achieved, 2), peak=peak, unit="TFLOP/s", frac=round(achieved / peak, 4),
                traffic=traffic if dom == "f64_on_the_fly" else None, traffic_note=traffic_note,
                kernel=kname, flop_note=flop_note, launches=nl[dom],
                avg_launch_ms=round(ms[dom] / max(nl[dom], 1), 4),
                avg_algorithmic_gflop_per_launch=round(fl / max(nl[dom], 1) / 1e9, 2),
                method_ms={k: round(v, 1) for k, v in ms.items()}, method_launches=nl)


def blocked_roofline(runs, n, traffic, traffic_cols):
    """Roofline of the FP32 T-apply of the blocked mixed-precision solver."""
    keys = ("f32_on_the_fly", "f32_stored")
    ms = {k: sum(r["tapply"]["ms_" + k] for r in runs) for k in keys}
    dom = max(keys, key=lambda k: ms[k])
    fl = sum(r["tapply"]["flop_" + dom] for r in runs)
    nl = sum(r["tapply"][dom] for r in runs)
    achieved = fl / (ms[dom] * 1e-3) / 1e12 if ms[dom] > 0 else 0.0
    fly = dom == "f32_on_the_fly"
    note = None
    if fly and traffic is not None:
        note = (f"HBM bytes per launch at {traffic_cols} real columns (counter runs); "
                f"algorithmic {2 * 4 * n * traffic_cols} B (X read once, Y written once)")
    if not fly:
        traffic, traffic_cols, kname = measured_traffic_stored("tapply_f32_stored_sphere20k_hbm_counters.md")
        if traffic is not None:
            nup = ((n + 255) // 256) * 256
            note = (f"HBM bytes per launch at {traffic_cols} real columns (counter runs, {kname}); "
                    f"algorithmic {4 * nup * nup + 2 * 4 * nup * traffic_cols} B (stored T read once, X, Y)")
    return dict(bound="mfma", achieved=round(achieved, 2), peak=FP32_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / FP32_MFMA_PEAK_TFLOPS, 4), traffic=traffic, traffic_note=note,
                kernel=("k_tapply_wfq_f32 (+ k_sk_fixup), T generated on the fly" if fly else
                        "k_tstored_f32 (+ k_sk_fixup) on the stored T (autotuner's choice for this width)"),
                launches=int(nl), avg_launch_ms=round(ms[dom] / max(nl, 1), 4),
                avg_algorithmic_gflop_per_launch=round(fl / max(nl, 1) / 1e9, 2),
                method_ms={k: round(v, 1) for k, v in ms.items()},
                method_launches={k: int(sum(r["tapply"][k] for r in runs)) for k in keys})


def measured_traffic_stored(summary, kernel_src="paper_2510_12731_amd/csrc/px_tapply.hip"):
    """HBM bytes per full-width stored-T product launch from the committed
    counter summary, or None if the kernel source changed since the counters
    were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        src = open(os.path.join(ROOT, kernel_src), "rb").read()
    except OSError:
        return None, None, None
    kv = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith(("-", "#")))
    if "traffic_bytes_per_launch" not in kv or kv.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None, None, None
    return int(kv["traffic_bytes_per_launch"]), int(kv["traffic_launch_real_columns"]), kv.get("kernel_name")


def measured_traffic(kernel_src, summary):
    """HBM bytes per full-width launch from the committed counter summary, or
    None if the kernel source changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        src = open(os.path.join(ROOT, kernel_src), "rb").read()
    except OSError:
        return None, None
    kv = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith(("-", "#")))
    if kv.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None, None
    return int(kv["traffic_bytes_per_launch"]), int(kv["traffic_launch_real_columns"])


def measured_traffic_narrow(kernel_src, summary):
    """HBM bytes per narrow FP64 T-apply launch (point part + near-field
    correction) from the committed counter summary, or None if the kernel
    source changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        src = open(os.path.join(ROOT, kernel_src), "rb").read()
    except OSError:
        return None, None
    kv = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith(("-", "#")))
    if kv.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None, None
    return int(kv["traffic_bytes_per_launch"]), kv.get("traffic_note")


def host_info():
    """Host CPU model and core counts (the box the oracle baseline ran on)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(cpu_model=model, nproc=os.cpu_count(), usable_cores=usable)


# Oracle timing tasks, each run in a child process pinned to one core (the
# oracle is single-threaded C): 'c1' the small spectrum in full, 'lu' one
# frequency of an N-atom sphere of the headline's lattice (dense assembly of
# A(w), its complete LU, three polarizations' solves), 'asm' the dense
# assembly alone at the headline's size; 'bem' / 'bemief' one frequency of an
# icosphere of R = 80 A (refinement level argv[4]) in the DPCM / IEFPCM form,
# three polarizations (matrices, the IEFPCM product, LU, solves).
_ORACLE_TASK = r"""
import json, os, sys, time
os.sched_setaffinity(0, {int(sys.argv[2])})
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle as O
from workloads import configs as C
from workloads import geometry as G
from workloads import materials as M
task = sys.argv[3]
t0 = time.perf_counter()
if task == "c1":
    c = C.small_sphere()
    O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    out = dict(seconds=time.perf_counter() - t0, columns=len(c["omega_ev"]))
elif task in ("bem", "bemief"):
    from workloads import mesh as ME
    m = ME.sphere(80.0, int(sys.argv[4]))
    om = np.array([3.6])
    eps = M.drude_permittivity(M.load("ag_bem"), om)
    solve = O.bem_ief_solve_spectrum if task == "bemief" else O.bem_solve_spectrum
    solve(m, om, eps, 1.0, 0b111, 1e-4)
    out = dict(seconds=time.perf_counter() - t0, n=len(m["area"]))
else:
    n = int(sys.argv[4])
    c = C.sphere_20k(n, 3)
    pv = M.param_vector(c["params"])
    a = O.assemble(0, c["xyz"], pv, 3.5)
    t1 = time.perf_counter()
    if task == "asm":
        out = dict(seconds=t1 - t0, n=n)
    else:
        b = np.stack([O.rhs(0, c["xyz"], pv, l, 1e-4) for l in range(3)], axis=1)
        O.lu_solve(a, b)
        out = dict(seconds=time.perf_counter() - t0, assembly_s=t1 - t0, lu_solve_s=time.perf_counter() - t1, n=n)
print(json.dumps(out), flush=True)
"""


def _oracle_children(tasks):
    """Run the oracle tasks concurrently, one child process per (core, task)."""
    import subprocess
    procs = [subprocess.Popen([sys.executable, "-c", _ORACLE_TASK, ROOT, str(core), *map(str, t)],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for core, t in tasks]
    out = []
    for p in procs:
        so, se = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle child failed: {se[-400:]}")
        out.append(json.loads(so.strip().splitlines()[-1]))
    return out


def cpu_baseline(n_head, npol, n_lu=3000, all_core_cap=16):
    """The oracle (dense FP64 direct solve, its own LU) on the host's cores.

    One pinned core: the small spectrum in full; one frequency at N = n_lu
    (assembly + complete LU + 3 solves); the dense assembly at the headline's
    N.  The headline's rate is extrapolated: assembly measured at N, LU and
    solves scaled from n_lu by (N / n_lu)^3.  All cores: one n_lu frequency on
    each usable core at once (independent frequency shards), measured, scaled
    the same way."""
    info = host_info()
    cores = sorted(os.sched_getaffinity(0))
    c0 = cores[0]
    t0 = time.perf_counter()
    c1 = _oracle_children([(c0, ("c1",))])[0]
    lu = _oracle_children([(c0, ("lu", n_lu))])[0]
    asm = _oracle_children([(c0, ("asm", n_head))])[0]
    k = min(len(cores), all_core_cap)
    allc = _oracle_children([(cores[i], ("lu", n_lu)) for i in range(k)])
    scale = (n_head / n_lu) ** 3
    per_freq = asm["seconds"] + lu["lu_solve_s"] * scale
    rate = npol / per_freq
    t_all = max(r["seconds"] for r in allc)
    lu_all = float(np.mean([r["lu_solve_s"] for r in allc]))
    asm_all = float(np.mean([r["assembly_s"] for r in allc]))
    # k shards at once: each core's frequency costs its assembly (scaled by N^2) and LU (by N^3)
    per_freq_all = asm_all * (n_head / n_lu) ** 2 + lu_all * scale
    rate_all = k * npol / per_freq_all
    return dict(value=round(rate, 8), unit="freq-solves/s", cores=1, kind="oracle",
                sample=(f"one core (pinned): dense assembly of A(w) at N={n_head} measured "
                        f"({asm['seconds']:.1f} s); one frequency at N={n_lu} (assembly {lu['assembly_s']:.1f} s, "
                        f"complete LU + {npol} solves {lu['lu_solve_s']:.1f} s) with the LU scaled by "
                        f"(N/{n_lu})^3 = {scale:.0f} to {lu['lu_solve_s'] * scale / 3600:.1f} h; {npol} "
                        f"polarizations per factorization; extrapolated, not run at N={n_head}"),
                host=info,
                config1_full=dict(columns=c1["columns"], seconds=round(c1["seconds"], 3),
                                  freq_solves_per_s=round(c1["columns"] / c1["seconds"], 2),
                                  note="249-atom sphere, 50 frequencies, x: the complete oracle spectrum, measured"),
                all_cores=dict(cores=k, value=round(rate_all, 8), unit="freq-solves/s",
                               measured_wall_s=round(t_all, 1),
                               note=(f"{k} independent frequency shards at N={n_lu} on {k} pinned cores at once "
                                     "(measured), each scaled to the headline's N as above")),
                measured_s=round(time.perf_counter() - t0, 1))


def bem_cpu_baseline(k_mesh=3, k_bench=5):
    """The oracle's BEM direct solve on the host, both forms at once on two
    pinned cores: one frequency (three polarizations) of the level-k_mesh
    icosphere, scaled by (n_bench / n)^3 to the benchmark's level-k_bench
    sphere (the LU and, for IEFPCM, the dense product dominate)."""
    cores = sorted(os.sched_getaffinity(0))
    c0, c1 = cores[0], cores[1 % len(cores)]
    r = _oracle_children([(c0, ("bem", k_mesh)), (c1, ("bemief", k_mesh))])
    n_bench = 20 * 4 ** k_bench
    out = {}
    for form, x in zip(("dpcm", "iefpcm"), r):
        scale = (n_bench / x["n"]) ** 3
        out[form] = dict(value=round(3.0 / (x["seconds"] * scale), 8), unit="freq-solves/s", cores=1, kind="oracle",
                         sample=(f"one core (pinned): one frequency, 3 polarizations, of the {x['n']}-tesserae "
                                 f"sphere in full ({x['seconds']:.1f} s: matrices"
                                 f"{', the product F S A^-1' if form == 'iefpcm' else ''}, LU, solves), scaled by "
                                 f"({n_bench}/{x['n']})^3 = {scale:.0f}; extrapolated, not run at {n_bench}"))
    return out


def config1_parity(pxm):
    """The small spectrum (249-atom Ag sphere, 50 w, x) on the GPU against the
    oracle's direct solve: sigma_abs relative error of the default (mixed
    options) and of the FP64 path at rel_tol 1e-12."""
    import oracle as O
    from workloads import configs as C
    from workloads import materials as M
    c = C.small_sphere()
    ref = O.solve_spectrum(0, c["xyz"], M.param_vector(c["params"]), c["omega_ev"], c["pol_mask"], c["e0"])
    out = {}
    for label, prec, tol in (("default_rel_tol_1e-8", pxm.PX_MIXED, 1e-8), ("fp64_rel_tol_1e-12", pxm.PX_FP64, 1e-12)):
        s = make_structure(pxm, c)
        st = s.solve(precision=prec, rel_tol=tol)
        sig = s.spectrum()[1]
        s.close()
        out[label] = dict(status=int(st), sigma_rel_err=float(np.max(np.abs(sig - ref["sigma"])) /
                                                              np.max(np.abs(ref["sigma"]))))
    return out


# sampled (frequency index, polarization) columns of the headline spectrum for
# the oracle residual: three in the 3.30-3.44 eV band at the dipolar plasmon,
# where restarted GMRES stagnates, the others spread over the grid
SAMPLED_COLUMNS = ((0, 0), (30, 1), (55, 0), (57, 1), (60, 2), (80, 2), (110, 0), (127, 1))


def oracle_residuals(pxm, case):
    """Solve the headline spectrum once more (untimed, same options), then
    the residual of sampled columns under the oracle's own operator and
    right-hand side (matrix-free, FP64 on the host)."""
    import oracle as O
    from workloads import materials as M
    s = make_structure(pxm, case)
    st = s.solve(precision=pxm.PX_MIXED, rel_tol=1e-8)
    om = case["omega_ev"]
    cols = [(w, l) for w, l in SAMPLED_COLUMNS if w < len(om)]
    q = np.stack([s.charges(w, l) for w, l in cols])
    s.close()
    pv = M.param_vector(case["params"])
    t0 = time.perf_counter()
    y = O.apply(0, case["xyz"], pv, om[[w for w, _ in cols]], q)
    b = {l: O.rhs(0, case["xyz"], pv, l, case["e0"]) for l in {l for _, l in cols}}
    res = [float(np.linalg.norm(b[l] - y[k]) / np.linalg.norm(b[l])) for k, (w, l) in enumerate(cols)]
    return dict(status=int(st), columns=[dict(omega_ev=round(float(om[w]), 4), pol="xyz"[l], oracle_rel_residual=r)
                                         for (w, l), r in zip(cols, res)],
                max_oracle_rel_residual=max(res), oracle_seconds=round(time.perf_counter() - t0, 1),
                note="||b - A q|| / ||b|| with A and b from the oracle (or_apply, or_rhs) for the GPU's charges")


def rod_extra(pxm):
    """The 10,000-atom Au rod (omegaFQFmu, 40,000 unknowns), 96 w, z: mixed
    against the plain FP64 blocked solver."""
    from workloads import configs as C
    c = C.rod_10k()
    ncol = len(c["omega_ev"])
    runs = {}
    for label, prec in (("mixed", pxm.PX_MIXED), ("fp64", pxm.PX_FP64)):
        one_step(pxm, c, prec, False)   # the T-apply tuner times its shapes once per process
        t0 = time.perf_counter()
        r = one_step(pxm, c, prec, True)
        runs[label] = (time.perf_counter() - t0, r)
    (tm, rm), (t64, r64) = runs["mixed"], runs["fp64"]
    return dict(workload="au_rod_10000_wfqfmu_96w_z", columns=ncol, mixed_s=round(tm, 2),
                mixed_solves_per_s=round(ncol / tm, 2), fp64_s=round(t64, 2), fp64_solves_per_s=round(ncol / t64, 2),
                speedup=round(t64 / tm, 2), mixed_iterations_max=int(rm["iters"].max()),
                fp64_iterations_max=int(r64["iters"].max()), status=[rm["status"], r64["status"]],
                relres_max=[float(rm["relres"].max()), float(r64["relres"].max())],
                sigma_rel_err_mixed_vs_fp64=float(np.max(np.abs(rm["sigma"] - r64["sigma"])) /
                                                  np.max(np.abs(r64["sigma"]))),
                tapply_launches={k: v for k, v in rm["tapply"].items() if not k.startswith(("ms_", "flop_"))})


def batch_full_extra(pxm, fp64_every=8):
    """The 64 graphene disks and ribbons (2k-60k atoms, 64 w each) in one
    pxSolveBatch call, against the plain FP64 solver per structure on every
    fp64_every-th structure."""
    from workloads import configs as C
    cases = C.graphene_batch()
    # the first call also runs the T-apply tuner on every new shape (64 atom counts)
    rc = batch_run(pxm, cases, pxm.PX_MIXED)
    rb = batch_run(pxm, cases, pxm.PX_MIXED)
    cols = sum(ncols(c) for c in cases)
    pick = list(range(0, len(cases), fp64_every))
    sub = [cases[k] for k in pick]
    seq = sequential_run(pxm, sub, pxm.PX_FP64, shifted=0)
    t64 = sum(r["seconds"] for r in seq)
    cols64 = sum(ncols(c) for c in sub)
    err = max(float(np.max(np.abs(rb["sigma"][k] - r["sigma"])) / np.max(np.abs(r["sigma"])))
              for k, r in zip(pick, seq))
    return dict(workload="graphene_batch_64", structures=len(cases),
                n_range=[min(len(c["xyz"]) for c in cases), max(len(c["xyz"]) for c in cases)], columns=cols,
                batched_s=round(rb["seconds"], 2), batched_solves_per_s=round(cols / rb["seconds"], 2),
                first_call_s=round(rc["seconds"], 2),
                first_call_note="the same batch the first time its shapes occur in the process (T-apply tuner included)",
                status=rb["status"], relres_max=rb["relres_max"],
                fp64_sample=f"every {fp64_every}th structure ({len(sub)} of {len(cases)}, {cols64} columns)",
                fp64_per_structure_solves_per_s=round(cols64 / t64, 2),
                speedup_vs_fp64=round((cols / rb["seconds"]) / (cols64 / t64), 2), sigma_rel_err_vs_fp64=err)


# FP64 arithmetic per tessera pair of the BEM operator kernels besides the
# products with the columns: s_i - s_j (3), r^2 (a multiply and two fused
# multiply-adds, 5), d.n (5), the reciprocal square root estimate and one
# Newton step (5), y^3 (2) and the kernel's value (1); the double layer F
# multiplies by the source area too.
BEM_PAIR_FLOP = {"dpcm": 21, "iefpcm": 22}


def bem_extra(pxm, form="dpcm", cpu=None):
    """BEM (DPCM or IEFPCM): a 20,480-tesserae Ag sphere (R = 80 A), 64 w x 3
    pol, the default solve against the FP64 blocked solver, and the oracle
    residual of a sampled column (IEFPCM: its charges in the printed
    equation).  For IEFPCM also the creation (mesh, F s and the dipole
    weights' single-layer solve) and one column's charge solve, timed apart."""
    import oracle as O
    from workloads import materials as M
    from workloads import mesh as ME
    m = ME.sphere(80.0, 5)
    om = np.linspace(3.2, 4.4, 64)
    eps = M.drude_permittivity(M.load("ag_bem"), om)

    def run(**kw):
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = pxm.Structure.bem(m, 1.0, pxm.default_stream(), form=form)
        t_create = time.perf_counter() - t0
        s.set_frequencies(om, 0b111, 1e-4, eps)
        st = s.solve(rel_tol=1e-8, **kw)
        sig = s.spectrum()[1]
        it = s.stats()[0]
        torch.cuda.synchronize()
        return s, dict(seconds=time.perf_counter() - t0, create_s=t_create, status=int(st), sigma=sig,
                       steps=int(it.max()), tapply=s.tapply_stats())

    s, r = run()
    s.close()
    s, r = run()
    # the shared phase's operator applies (one k_bem_apply over the three
    # real basis columns + k_bem_sum per step), timed by the library's HIP
    # events on its stream in a third solve with timings on
    s_t, r_t = run(timings=True)
    s_t.close()
    ta = r_t["tapply"]
    n = len(m["area"])
    pair_flop = BEM_PAIR_FLOP[form] + 2 * 3
    launches = int(ta["f64_on_the_fly"])
    ms_ap = float(ta["ms_f64_on_the_fly"])
    ach = n * n * pair_flop * launches / (ms_ap * 1e-3) / 1e12 if ms_ap > 0 else 0.0
    roof = dict(bound="alu", achieved=round(ach, 2), peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                frac=round(ach / FP64_VECTOR_PEAK_TFLOPS, 4),
                kernel=f"k_bem_apply<{1 if form == 'iefpcm' else 0}, 3> + k_bem_sum (the shared phase's step)",
                launches=launches, avg_launch_ms=round(ms_ap / max(launches, 1), 4),
                flop_note=f"{BEM_PAIR_FLOP[form]} + 2 x 3 FP64 FLOP per tessera pair (N^2 pairs), peak = FP64 vector")
    w = int(np.argmax(r["sigma"]))
    t0 = time.perf_counter()
    q = s.charges(w, 0)
    t_q = time.perf_counter() - t0
    s.close()
    if form == "iefpcm":
        b = O.bem_ief_rhs(m, 0, 1e-4)
        y = O.bem_ief_potential(m, q[None, :])
        res = float(np.linalg.norm(b - O.bem_ief_apply(m, eps[w:w + 1], 1.0, y)[0]) / np.linalg.norm(b))
    else:
        b = O.bem_rhs(m, 0, 1e-4)
        res = float(np.linalg.norm(b - O.bem_apply(m, eps[w:w + 1], 1.0, q[None, :])[0]) / np.linalg.norm(b))
    s64, r64 = run(precision=pxm.PX_FP64, shifted=0)
    s64.close()
    ncol = len(om) * 3
    out = dict(workload=f"ag_bem_{form}_sphere_20480_64w_xyz", tesserae=len(m["area"]), columns=ncol,
               seconds=round(r["seconds"], 3), solves_per_s=round(ncol / r["seconds"], 2), status=r["status"],
               phase_steps_max=r["steps"], fp64_blocked_s=round(r64["seconds"], 2),
               fp64_blocked_solves_per_s=round(ncol / r64["seconds"], 2),
               speedup_vs_fp64_blocked=round(r64["seconds"] / r["seconds"], 2),
               sigma_rel_err_vs_fp64_blocked=float(np.max(np.abs(r["sigma"] - r64["sigma"])) /
                                                   np.max(np.abs(r64["sigma"]))),
               oracle_rel_residual_at_peak=res, peak_ev=round(float(om[w]), 3), roofline=roof)
    if form == "iefpcm":
        out.update(create_s=round(r["create_s"], 3), charges_one_column_s=round(t_q, 4))
    if cpu is not None:
        out["cpu_baseline"] = cpu[form]
    return out


def make_structure(pxm, case):
    s = pxm.Structure(case["model"], case["xyz"], case["params"], pxm.default_stream())
    s.set_frequencies(case["omega_ev"], case["pol_mask"], case["e0"], case["alpha_ib"])
    return s


def ncols(case):
    return len(case["omega_ev"]) * bin(case["pol_mask"]).count("1")


def batch_run(pxm, cases, precision, block_cols=64):
    """All structures in one pxSolveBatch call (solved whole, several at once on
    their own streams, or stacked in the block); returns timing and statuses."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ss = [make_structure(pxm, c) for c in cases]
    st = pxm.solve_batch(ss, precision=precision, rel_tol=1e-8, block_cols=block_cols, max_restart_m=100)
    sig = [s.spectrum()[1] for s in ss]
    rr = max(float(s.stats()[2].max()) for s in ss)
    for s in ss:
        s.close()
    torch.cuda.synchronize()
    return dict(seconds=time.perf_counter() - t0, status=int(st), relres_max=rr, sigma=sig)


def sequential_run(pxm, cases, precision, max_block_cols=0, shifted=None, progress=False):
    """One structure after the other, each with pxSolveSpectrum (shifted = 0:
    the blocked solver alone, the plain FP64 baseline with PX_FP64)."""
    import torch
    out = []
    for k, c in enumerate(cases):
        if progress:
            log(f"[bench]   structure {k + 1}/{len(cases)}: N={len(c['xyz'])}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = make_structure(pxm, c)
        st = s.solve(precision=precision, rel_tol=1e-8, max_block_cols=max_block_cols, max_restart_m=100,
                     shifted=shifted)
        sig = s.spectrum()[1]
        s.close()
        torch.cuda.synchronize()
        out.append(dict(seconds=time.perf_counter() - t0, status=int(st), sigma=sig))
    return out


def serving_run(pxm, cases, arrivals, budget_bytes, block_cols=64):
    """Continuous batching: request k arrives at arrivals[k] (s after start) and
    joins the server's block at the next restart boundary that has room."""
    import torch
    sv = pxm.Server(budget_bytes, pxm.default_stream(), precision=pxm.PX_MIXED, rel_tol=1e-8,
                    block_cols=block_cols, max_restart_m=100)
    t0 = time.perf_counter()
    pending = list(range(len(cases)))
    live = {}
    lat = [None] * len(cases)
    sig = [None] * len(cases)
    peak_rows = 0
    while pending or live:
        now = time.perf_counter() - t0
        while pending and arrivals[pending[0]] <= now:
            k = pending.pop(0)
            s = make_structure(pxm, cases[k])
            sv.submit(s)
            live[s.h.value] = (k, s)
        q = sv.query()
        if q["active"] == 0 and q["queued"] == 0:
            if pending:
                time.sleep(max(0.0, arrivals[pending[0]] - (time.perf_counter() - t0)))
            continue
        for h in sv.step():
            k, s = live.pop(h)
            lat[k] = time.perf_counter() - t0 - arrivals[k]
            sig[k] = s.spectrum()[1]
            s.close()
        peak_rows = max(peak_rows, sv.query()["rows_in_use"])
    makespan = time.perf_counter() - t0
    cap = sv.query()["rows_capacity"]
    sv.close()
    return dict(latency=lat, makespan=makespan, sigma=sig, peak_rows=peak_rows, rows_capacity=cap)


def serving_extra(pxm, n_req, n_min, n_max, seed, load, block_cols=64, model=None, fp64=True):
    """The serving mix: n_req seeded requests (model: only those of that model
    out of the n_req drawn), served by the server under Poisson arrivals at
    `load` of the one-at-a-time capacity, against one request at a time (and,
    with fp64, the plain FP64 solver one at a time), then all queued at once."""
    from workloads import configs as C
    rng = np.random.default_rng(seed)
    cases = [C.serving_request(rng, n_min, n_max) for _ in range(n_req)]
    if model is not None:
        cases = [c for c in cases if c["model"] == model]
        n_req = len(cases)
    cols = sum(ncols(c) for c in cases)
    seq = sequential_run(pxm, cases, pxm.PX_MIXED)
    t_seq = sum(r["seconds"] for r in seq)
    lam = load * n_req / t_seq
    arrivals = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / lam, n_req)) - 0.0
    arrivals -= arrivals[0]
    # sequential one-at-a-time under the same arrivals: FIFO queue
    t, lat_seq = 0.0, []
    for a, r in zip(arrivals, seq):
        t = max(t, a) + r["seconds"]
        lat_seq.append(t - a)
    # the plain FP64 solver (blocked, no shared-Krylov phase) one request at a time, same arrivals, FIFO
    seq64 = sequential_run(pxm, cases, pxm.PX_FP64, shifted=0) if fp64 else seq
    t64, lat64 = 0.0, []
    for a, r in zip(arrivals, seq64):
        t64 = max(t64, a) + r["seconds"]
        lat64.append(t64 - a)
    budget = 0.5 * torch_free_bytes()
    srv = serving_run(pxm, cases, arrivals, budget, block_cols)
    err = max(float(np.max(np.abs(a - b["sigma"])) / np.max(np.abs(b["sigma"]))) for a, b in zip(srv["sigma"], seq))
    lat = np.array(srv["latency"])
    # saturated: every request queued at once, against the same requests one after the other
    sat = serving_run(pxm, cases, np.zeros(n_req), budget, block_cols)
    return dict(requests=n_req, columns=cols, n_range=[n_min, n_max], arrival_rate_per_s=round(lam, 3),
                load=load, solves_per_s=round(cols / srv["makespan"], 2),
                p50_s=round(float(np.percentile(lat, 50)), 3), p99_s=round(float(np.percentile(lat, 99)), 3),
                one_at_a_time_solves_per_s=round(cols / max(t, 1e-9), 2),
                one_at_a_time_p50_s=round(float(np.percentile(lat_seq, 50)), 3),
                one_at_a_time_p99_s=round(float(np.percentile(lat_seq, 99)), 3),
                fp64_one_at_a_time_solves_per_s=round(cols / max(t64, 1e-9), 2) if fp64 else None,
                fp64_one_at_a_time_p50_s=round(float(np.percentile(lat64, 50)), 3) if fp64 else None,
                fp64_one_at_a_time_p99_s=round(float(np.percentile(lat64, 99)), 3) if fp64 else None,
                sigma_rel_err_mix_vs_fp64=max(float(np.max(np.abs(a - b["sigma"])) / np.max(np.abs(b["sigma"])))
                                              for a, b in zip(srv["sigma"], seq64)) if fp64 else None,
                peak_rows=srv["peak_rows"], rows_capacity=srv["rows_capacity"],
                sigma_rel_err_mix_vs_alone=err,
                saturated=dict(solves_per_s=round(cols / sat["makespan"], 2),
                               one_at_a_time_solves_per_s=round(cols / t_seq, 2),
                               note="all requests queued at t = 0; at 75 % load both serve every request as it "
                                    "arrives, so their solves/s above follow the arrival rate"))


# FP64 arithmetic per (point, atom) pair of the probe kernel's point-source
# path: the differences (3), r^2 (5), the reciprocal square root estimate, its
# Newton step and the halving (6), r^-2 and r^-3 (2), the charge's two parts
# times r^-3 (2) and six fused multiply-adds into the complex field (12); a
# dipole adds 3 r^-5 (2), mu . d r^-5 for both parts (12) and twelve fused
# multiply-adds (24).
PROBE_PAIR_FLOP = {0: 30, 1: 68}


def probe_roofline(st, model):
    fl = PROBE_PAIR_FLOP[model] * st["pairs"]
    ach = fl / (st["ms_kernel"] * 1e-3) / 1e12 if st["ms_kernel"] > 0 else 0.0
    return dict(bound="alu", achieved=round(ach, 2), peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                frac=round(ach / FP64_VECTOR_PEAK_TFLOPS, 4), kernel="k_probe (+ k_probe_sum)",
                flop_note=f"{PROBE_PAIR_FLOP[model]} FP64 FLOP per (point, atom) pair of the point-source path; "
                          "pairs within 7 Gaussian widths cost more and count the same")


def probe_extra(pxm):
    """Post-processing rates: the induced density and field of a solved column
    at probe points, for a synthetic 1122-atom Au fcc gap dimer (5 A gap,
    omegaFQFmu, 2.28 eV, x: an 80^3 CUBE grid and a 400 x 400 plane) and the
    20,000-atom Ag sphere (omegaFQ, 3.6 eV) on a 128^3 grid; the probe kernel
    times come from HIP events around its launches."""
    from workloads import configs as C
    from workloads import geometry as G
    from workloads import materials as M
    out = {}
    au = M.load("au_wfqfmu")
    xyz = G.gap_dimer(1122, 5.0)
    s = pxm.Structure(1, xyz, au, pxm.default_stream())
    om = np.array([2.28])
    s.set_frequencies(om, 0b001, 1e-4, M.interband_alpha(au, om))
    s.solve(precision=pxm.PX_MIXED, rel_tol=1e-8)
    lo, hi = xyz.min(0) - 4.0, xyz.max(0) + 4.0
    ax = [np.linspace(lo[a], hi[a], 80) for a in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    cube = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    t0 = time.perf_counter()
    _, rho = s.induced_field(0, 0, cube)
    t_cube = time.perf_counter() - t0
    st_cube = s.probe_stats()
    px_ = np.linspace(lo[0], hi[0], 400)
    py_ = np.linspace(lo[1], hi[1], 400)
    PX, PY = np.meshgrid(px_, py_, indexing="ij")
    plane = np.stack([PX.ravel(), PY.ravel(), np.full(PX.size, xyz[:, 2].mean())], 1)
    t0 = time.perf_counter()
    f, _ = s.induced_field(0, 0, plane)
    t_plane = time.perf_counter() - t0
    st_plane = s.probe_stats()
    s.close()
    out["au_dimer_1122_wfqfmu"] = dict(
        cube_points=len(cube), cube_seconds=round(t_cube, 4), cube_kernel_ms=round(st_cube["ms_kernel"], 3),
        plane_points=len(plane), plane_seconds=round(t_plane, 4), plane_kernel_ms=round(st_plane["ms_kernel"], 3),
        roofline=probe_roofline(st_plane, 1))
    case = C.sphere_20k()
    s = pxm.Structure(0, case["xyz"], case["params"], pxm.default_stream())
    s.set_frequencies(np.array([3.6]), 0b001, case["e0"])
    s.solve(precision=pxm.PX_MIXED, rel_tol=1e-8)
    xyz = case["xyz"]
    lo, hi = xyz.min(0) - 5.0, xyz.max(0) + 5.0
    ax = [np.linspace(lo[a], hi[a], 128) for a in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    grid = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    s.induced_field(0, 0, grid[:65536])   # warm-up
    t0 = time.perf_counter()
    s.induced_field(0, 0, grid)
    t_grid = time.perf_counter() - t0
    st = s.probe_stats()
    s.close()
    out["ag_sphere_20000_wfq_grid128"] = dict(
        points=len(grid), seconds=round(t_grid, 3), kernel_ms=round(st["ms_kernel"], 2),
        points_per_s=round(len(grid) / (st["ms_kernel"] * 1e-3), 1),
        pair_evaluations_per_s=round(st["pairs"] / (st["ms_kernel"] * 1e-3), 1), roofline=probe_roofline(st, 0),
        note="seconds include the host conversion of the points and the copies; kernel_ms the probe kernels")
    return out


def torch_free_bytes():
    import torch
    free, total = torch.cuda.mem_get_info()
    return float(free)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--n-omega", type=int, default=128)
    ap.add_argument("--fp64-sample", type=int, default=6, help="columns of the one-column FP64 baseline")
    ap.add_argument("--no-fp64-blocked", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-lu-n", type=int, default=3000, help="atoms of the oracle's complete LU (CPU baseline)")
    ap.add_argument("--kernel-sample", action="store_true",
                    help="a short solve of the full workload for hardware-counter runs: 8 shared-Krylov steps, or "
                         "with --no-shifted one blocked restart cycle of 4 steps (with --t-apply)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only copy this many GiB device-to-device (scales HBM counters) and exit")
    ap.add_argument("--workload", default="sphere", choices=["sphere", "serving", "serving-full", "serving-wfq-full", "probe", "batch",
                                                           "bem"],
                    help="sphere: the headline line with every config's extra; serving: the serving mix alone; "
                         "serving-wfq-full: the omegaFQ requests of the 1k-100k mix; serving-full: the serving mix at "
                         "1k-100k atoms; probe: the induced-field evaluation; batch: the 64-structure graphene "
                         "batch alone, first and warm call; bem: the BEM sphere in both forms; printed as their own "
                         "JSON lines")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads (rod, batch, serving, BEM)")
    ap.add_argument("--no-blocked", action="store_true", help="skip the blocked mixed-precision comparison step")
    ap.add_argument("--no-shifted", action="store_true",
                    help="time the blocked mixed-precision solver alone (no shared-Krylov phase)")
    ap.add_argument("--t-apply", default="auto", choices=["auto", "on-the-fly", "stored"],
                    help="T-apply method of the timed steps (auto: the autotuner's choice per width)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every box here has a single MI355X and the solver does not shard; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the oracle's host baseline first, in pinned child processes, before this
    # process touches the GPU
    cpu = None
    if not (args.no_cpu_baseline or args.kernel_sample or args.copy_calibration > 0 or args.workload != "sphere"):
        log("[bench] oracle CPU baseline (pinned cores) ...")
        cpu = cpu_baseline(args.n, 3, n_lu=args.cpu_lu_n)
        log(f"[bench] oracle CPU baseline done in {cpu['measured_s']} s")
    bem_cpu = None
    if not (args.no_cpu_baseline or args.kernel_sample or args.copy_calibration > 0 or args.no_extras or
            args.workload not in ("sphere", "bem")):
        log("[bench] oracle CPU baseline, BEM (two pinned cores) ...")
        bem_cpu = bem_cpu_baseline()

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 3}), flush=True)
        return
    ensure_built()
    import paper_2510_12731_amd as pxm
    from workloads import configs as C

    if args.workload == "probe":
        print(json.dumps({"workload": "induced_field", **probe_extra(pxm)}), flush=True)
        return
    if args.workload == "batch":
        from workloads import configs as C2
        cases = C2.graphene_batch()
        import torch
        for label in ("first", "warm"):
            # a small torch sort marks the call's start in a kernel trace
            torch.sort(torch.arange(8, 0, -1, device="cuda"))
            r = batch_run(pxm, cases, pxm.PX_MIXED)
            print(json.dumps({"workload": "graphene_batch_64", "call": label, "seconds": round(r["seconds"], 3),
                              "status": r["status"], "relres_max": r["relres_max"]}), flush=True)
        return
    if args.workload == "bem":
        for form in ("dpcm", "iefpcm"):
            print(json.dumps(bem_extra(pxm, form, bem_cpu)), flush=True)
        return
    if args.workload == "serving":
        out = serving_extra(pxm, 16, 1000, 8000, 5, 0.75)
        print(json.dumps({"workload": "serving_mix", **out}), flush=True)
        return
    if args.workload == "serving-full":
        out = serving_extra(pxm, 40, 1000, 100000, 5, 0.75)
        print(json.dumps({"workload": "serving_mix_full", **out}), flush=True)
        return
    if args.workload == "serving-wfq-full":
        t0 = time.perf_counter()
        out = serving_extra(pxm, 40, 1000, 100000, 5, 0.75, model=0, fp64=False)
        print(json.dumps({"workload": "serving_mix_full_wfq", "seconds": round(time.perf_counter() - t0, 1), **out}),
              flush=True)
        return

    case = C.sphere_20k(args.n, args.n_omega)
    ncol = len(case["omega_ev"]) * bin(case["pol_mask"]).count("1")
    log(f"[bench] workload {case['name']}: N={len(case['xyz'])}, {ncol} columns")
    ta_mode = {"auto": pxm.PX_TAPPLY_AUTO, "on-the-fly": pxm.PX_TAPPLY_ON_THE_FLY,
               "stored": pxm.PX_TAPPLY_STORED}[args.t_apply]
    if args.kernel_sample:
        s = pxm.Structure(case["model"], case["xyz"], case["params"], pxm.default_stream())
        s.set_frequencies(case["omega_ev"], case["pol_mask"], case["e0"])
        if args.no_shifted:
            # one restart cycle of 4 steps of the blocked solver (FP32 T-apply)
            st = s.solve(precision=pxm.PX_MIXED, restart_m=4, max_restart_m=4, max_cycles=1, timings=True,
                         t_apply=ta_mode, shifted=0)
        else:
            # 8 steps of the shared-Krylov phase (narrow FP64 T-apply)
            st = s.solve(precision=pxm.PX_FP64, max_cycles=1, timings=True, t_apply=ta_mode, shifted=1,
                         shifted_max_steps=8)
        tm = s.timings()
        s.close()
        print(json.dumps({"kernel_sample": True, "status": int(st), "tapply_f32_launches": int(tm["n_tapply_f32"]),
                          "cols_f32_padded": int(tm["cols_f32_padded"]),
                          "tapply_f64_launches": int(tm["n_tapply_f64"])}), flush=True)
        return

    shifted = 0 if args.no_shifted else 2
    # the shared-Krylov phase runs in FP64; the blocked solver alone in mixed precision
    head_prec = pxm.PX_FP64 if shifted else pxm.PX_MIXED
    for w in range(args.warmup):
        r = one_step(pxm, case, head_prec, True, t_apply=ta_mode, shifted=shifted)
        log(f"[bench] warmup {w}: status {r['status']} max iters {r['iters'].max()} "
            f"{r['timings']['ms_total'] / 1e3:.2f} s")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    step_s = []
    for k in range(args.steps):
        ta = time.perf_counter()
        runs.append(one_step(pxm, case, head_prec, True, t_apply=ta_mode, shifted=shifted))
        step_s.append(time.perf_counter() - ta)
        log(f"[bench] step {k}: status {runs[-1]['status']} {runs[-1]['timings']['ms_total'] / 1e3:.2f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = ncol * args.steps / (t1 - t0)
    last = runs[-1]
    tm = last["timings"]
    n = len(case["xyz"])
    npol = bin(case["pol_mask"]).count("1")

    # roofline of the dominant T-apply (live HIP-event times of its launches)
    f32_traffic, f32_cols = measured_traffic("paper_2510_12731_amd/csrc/px_tapply.hip",
                                             "tapply_f32_sphere20k_hbm_counters.md")
    n64_traffic, n64_note = measured_traffic_narrow("paper_2510_12731_amd/csrc/px_tapply.hip",
                                                    "tapply_f64_narrow_sphere20k_hbm_counters.md")
    if shifted:
        roof = tapply_roofline(runs, n, npol, n64_traffic, n64_note)
    else:
        roof = blocked_roofline(runs, n, f32_traffic, f32_cols)

    # path roofline: the ideal time of the solve's algorithmic work at the
    # peaks (FP32 and FP64 arithmetic, HBM) over its measured wall time
    wk = last["work"]
    ideal_s = wk["flop_f32"] / (FP32_MFMA_PEAK_TFLOPS * 1e12) + wk["flop_f64"] / (FP64_MFMA_PEAK_TFLOPS * 1e12) + \
        wk["hbm_bytes"] / (HBM_PEAK_GBS * 1e9)
    solve_s = tm["ms_total"] / 1e3
    path = dict(ideal_ms=round(ideal_s * 1e3, 1), solve_ms=round(solve_s * 1e3, 1), frac=round(ideal_s / solve_s, 4),
                flop_f32=wk["flop_f32"], flop_f64=wk["flop_f64"], hbm_bytes=wk["hbm_bytes"],
                peaks="FP32 matrix 157.3 TFLOP/s, FP64 78.6 TFLOP/s, HBM 8 TB/s",
                note="FP64 FLOP counted as 2 N^2 per real column and T-apply (the matrix-vector product alone)")

    med = float(np.median(step_s))
    extra = dict(
        median_step_s=round(med, 3), median_step_freq_solves_per_s=round(ncol / med, 3),
        path_roofline=path,
        iterations_max=int(last["iters"].max()), iterations_mean=round(float(last["iters"].mean()), 1),
        cycles_max=int(last["cycles"].max()), relres_max=float(last["relres"].max()),
        phase_ms=dict(tapply_f32=round(tm["ms_tapply_f32"], 1), tapply_f64=round(tm["ms_tapply_f64_cycles"], 1),
                      sparse=round(tm["ms_spmm"], 1), arnoldi_givens=round(tm["ms_arnoldi"], 1),
                      rest=round(tm["ms_other"], 1)))
    extra["tapply_launches"] = {k: int(v) for k, v in last["tapply"].items() if not k.startswith(("ms_", "flop_"))}

    # error against the oracle: the small spectrum in full, sampled columns of this one
    log("[bench] oracle parity: 249-atom spectrum, sampled columns of the headline ...")
    extra["oracle_parity"] = dict(config1=config1_parity(pxm), headline_sampled_columns=oracle_residuals(pxm, case))

    # the shared-Krylov phase with one Arnoldi process per polarization instead
    if shifted and not args.no_blocked:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rpp = one_step(pxm, case, pxm.PX_FP64, True, t_apply=ta_mode, shifted=1)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        extra["per_polarization_phase"] = dict(
            value=round(ncol / (tb - ta), 3), unit="freq-solves/s", seconds=round(tb - ta, 3),
            status=int(rpp["status"]), steps_max=int(rpp["iters"].max()),
            note="shifted = 1: one Arnoldi process per polarization (the default takes one block process)",
            sigma_rel_err_vs_default=float(np.max(np.abs(rpp["sigma"] - last["sigma"])) /
                                           np.max(np.abs(last["sigma"]))))

    # the blocked mixed-precision solver alone: FP32 MFMA T-apply, FP64 refinement
    if not args.no_blocked:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rbm = one_step(pxm, case, pxm.PX_MIXED, True, t_apply=ta_mode, shifted=0)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        vbm = ncol / (tb - ta)
        extra["blocked_mixed"] = dict(
            value=round(vbm, 3), unit="freq-solves/s", seconds=round(tb - ta, 2), status=int(rbm["status"]),
            iterations_max=int(rbm["iters"].max()), roofline=blocked_roofline([rbm], n, f32_traffic, f32_cols),
            sigma_rel_err_vs_default=float(np.max(np.abs(rbm["sigma"] - last["sigma"])) /
                                           np.max(np.abs(last["sigma"]))))

    # plain FP64 solver, one column at a time, on a sample of the columns
    if args.fp64_sample > 0:
        idx = np.linspace(0, len(case["omega_ev"]) - 1, args.fp64_sample).round().astype(int)
        sub = dict(case)
        sub["omega_ev"] = case["omega_ev"][idx]
        sub["pol_mask"] = 0b001
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r64 = one_step(pxm, sub, pxm.PX_FP64, False, max_block_cols=1, t_apply=pxm.PX_TAPPLY_ON_THE_FLY, shifted=0)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        v64 = len(idx) / (tb - ta)
        extra["fp64_one_column"] = dict(value=round(v64, 4), unit="freq-solves/s",
                                        sample=f"{len(idx)} x-polarized columns spread over the grid; "
                                               "hand-written FP64 kernels (T on the fly), blocked solver one column "
                                               "at a time",
                                        iterations=r64["iters"].tolist(), seconds=round(tb - ta, 2))
        extra["speedup_vs_fp64_one_column"] = round(value / v64, 2)
        if "blocked_mixed" in extra:
            extra["blocked_mixed"]["speedup_vs_fp64_one_column"] = round(extra["blocked_mixed"]["value"] / v64, 2)
        ax = last["alpha"][idx, 0, 0]
        a64 = r64["alpha"][:, 0, 0]
        extra["alpha_xx_vs_fp64_one_column_rel"] = float(np.max(np.abs(ax - a64)) / np.max(np.abs(a64)))
    if not args.no_fp64_blocked:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rb = one_step(pxm, case, pxm.PX_FP64, False, shifted=0)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        extra["fp64_blocked"] = dict(value=round(ncol / (tb - ta), 3), unit="freq-solves/s",
                                     seconds=round(tb - ta, 2), status=int(rb["status"]),
                                     note="all 384 columns in one FP64 block (blocked solver, autotuned T-apply)")
        extra["speedup_vs_fp64_blocked"] = round(value * (tb - ta) / ncol, 2)
        extra["sigma_rel_err_vs_fp64_blocked"] = float(
            np.max(np.abs(last["sigma"] - rb["sigma"])) / np.max(np.abs(rb["sigma"])))
        if "blocked_mixed" in extra:
            extra["blocked_mixed"]["sigma_rel_err_vs_fp64_blocked"] = float(
                np.max(np.abs(rbm["sigma"] - rb["sigma"])) / np.max(np.abs(rb["sigma"])))
            extra["blocked_mixed"]["speedup_vs_fp64_blocked"] = round(extra["blocked_mixed"]["value"] * (tb - ta) / ncol,
                                                                      2)

    if not args.no_extras:
        log("[bench] config 3: 10k-atom Au rod ...")
        extra["rod_10k"] = rod_extra(pxm)
        log("[bench] config 4: 64-structure graphene batch ...")
        extra["batch_full"] = batch_full_extra(pxm)
        log("[bench] config 5: serving mix (1k-8k atoms) ...")
        extra["serving"] = serving_extra(pxm, 16, 1000, 8000, 5, 0.75)
        log("[bench] BEM sphere ...")
        extra["bem"] = bem_extra(pxm, "dpcm", bem_cpu)
        log("[bench] BEM sphere, IEFPCM ...")
        extra["bem_iefpcm"] = bem_extra(pxm, "iefpcm", bem_cpu)

    out = {
        "metric": "omegaFQ freq-solves/s at N=20k (rel res 1e-8)",
        "value": round(value, 3),
        "unit": "freq-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if shifted else "f32/f64",
        "data": "synthetic",
        "config": {"workload": case["name"], "n_atoms": n, "n_omega": int(len(case["omega_ev"])),
                   "polarizations": 3, "columns": ncol, "rel_tol": 1e-8, "t_apply": args.t_apply,
                   "solver": ("shared-Krylov phase (one FP64 block Arnoldi process over the three polarizations for "
                              "all frequencies), blocked GMRES(100) for any column left" if shifted else
                              "blocked GMRES(100), FP32 T-apply, FP64 refinement")},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
