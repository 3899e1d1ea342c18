"""Benchmark: L-sweep GMRES solve time to 1e-6 relative residual, and the sweep (subdomain
apply) bandwidth, on one MI355X.

Workload (default, the largest single-GPU configuration): lens3d, a 95^3 bulk grid + 8-point
PML (111^3 extended points) decomposed into 4x4 beams over all z, Gaussian lens, 8 points per
minimum wavelength, one Gaussian source at (0.5, 0.5, 0.25); complex64 plane-block factors and
sweeps (47.5 GB of factors in full, 25 GB packed) with FP64 GMRES (the mixed form), next to the
plain FP64 form.  `--workload lens2d|const2d|layered2d|fwi2d` selects the 2D configurations.

A step is one complete solve (zero initial guess to ||b - A u|| <= 1e-6 ||b||): every
preconditioner application (stage 1, 4 cardinal and 4 diagonal sweeps), every A x, the
Gram-Schmidt passes and the host least squares.  Setup and factorisation are outside the
timed region.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "L-sweep GMRES solve time to 1e-6 rel. residual; subdomain-apply HBM GB/s"
MEDIA = {"const2d": "c = 1", "lens2d": "lens + 5% smooth noise", "layered2d": "12 dipping layers + 3 faults",
         "fwi2d": "lens + 5% Gaussian blobs", "lens3d": "Gaussian lens"}
HBM_PEAK_GBS = 8000.0
FP32_MATRIX_PEAK_TFLOPS = 157.3   # dense FP32 matrix-core peak of MI355X


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_problem(workload: str, all_sources: bool = False):
    import torch

    from paper_1909_01467_amd import inputs
    from paper_1909_01467_amd.lsweeps import extend_medium

    wl = inputs.workload(workload)
    m_bulk = torch.from_numpy(wl.slowness2).cuda()
    m_ext = extend_medium(m_bulk, wl.n_pml).contiguous()
    src = wl.sources if all_sources else wl.sources[:1]
    f = torch.from_numpy(src).to(torch.complex128).cuda()
    p = wl.n_pml
    b = torch.nn.functional.pad(f, (p, p) * wl.dim).contiguous()   # f extended by zero into the PML
    return wl, m_ext, (b if all_sources else b[0])


def time_solves(solver, b, steps: int, warmup: int):
    import torch

    info = None
    for _ in range(warmup):
        _, info = solver.solve(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u, info = solver.solve(b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return u, info, dt * 1e3


def time_applies(solver, b, reps: int = 20):
    """Device time of one preconditioner application and of each of its kernel families
    (HIP events recorded by the library on its own stream, around the launches of each
    family), median over `reps` applications."""
    keys = ("last_apply_ms", "last_stage1_ms", "last_gemv_ms", "last_final_rhs_ms", "last_final_ms", "last_dom_ms")
    rows = []
    for _ in range(reps):
        solver.apply(b)
        st = solver.stats()
        rows.append([st[k] for k in keys])
    med = {k: sorted(r[i] for r in rows)[len(rows) // 2] for i, k in enumerate(keys)}
    return med, solver.stats()


def kernel_source_sha(path: str, name: str):
    """SHA-256 (first 16 hex digits) of the source text of the __global__ function `name` in `path`:
    from its template/__global__ line to the closing brace at the start of a line."""
    import hashlib

    lines = open(path).read().splitlines(keepends=True)
    for i, line in enumerate(lines):
        if line.startswith("__global__") and f" {name}(" in line:
            start = i - 1 if i > 0 and lines[i - 1].startswith("template") else i
            for j in range(i, len(lines)):
                if lines[j].startswith("}"):
                    return hashlib.sha256("".join(lines[start:j + 1]).encode()).hexdigest()[:16]
    return None


def counter_traffic(kernel: str, workload: str, algorithmic_bytes_per_launch: float | None = None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary of the
    workload (scaled FETCH_SIZE + WRITE_SIZE), or None when there is none, when the kernel's source
    changed since the counters were taken, or when the summary records another amount of work per
    launch than this run's algorithmic bytes (a schedule that launches the kernel differently)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_mixed_hbm_traffic.txt")
    csrc = os.path.join(ROOT, "paper_1909_01467_amd", "csrc")
    try:
        text = open(path).read()
    except OSError:
        return None
    # the summary records the sha of the kernel's own source text
    base = kernel.split("<")[0]
    sha = kernel_source_sha(os.path.join(csrc, "kernels3d.hip" if workload.endswith("3d") else "kernels.hip"), base)
    if sha is None or f"{base} source sha256[:16] = {sha}" not in text:
        return None
    if algorithmic_bytes_per_launch is not None:
        recorded = [float(l.split()[2]) for l in text.splitlines()
                    if len(l.split()) == 3 and l.split()[0] == "algorithmic" and l.split()[1] == kernel]
        if not recorded or abs(recorded[0] - algorithmic_bytes_per_launch) > 0.01 * recorded[0]:
            return None
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic" and parts[1] == kernel:
            return int(parts[2])
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_3d(workload: str):
    """The FP64 oracle (Alg. Scenario3 over beams with SuperLU local solves, inside the oracle's
    FGMRES) on the 3D workload downscaled to 23^3 with 2x2 beams (same medium, PML and points per
    wavelength): at full size one beam's SuperLU factorisation alone takes about 400 s and 9 GB, and
    the banded LU of the whole grid would need 809 GB.  One solve to 1e-6 is timed (setup apart)."""
    from threadpoolctl import threadpool_limits

    from oracle.discretization import GlobalProblem, extend_normal
    from oracle.fgmres import fgmres
    from oracle.lsweep3d import LSweep3D
    from paper_1909_01467_amd import inputs

    wl = inputs.workload(workload, n=23, q=2)
    with threadpool_limits(limits=1):
        m = extend_normal(wl.slowness2, wl.n_pml)
        t0 = time.perf_counter()
        gp = GlobalProblem(m, wl.omega, wl.n, wl.n_pml, wl.C)
        ls = LSweep3D(m, wl.omega, wl.n, wl.n_pml, wl.q, wl.r, wl.C)
        t1 = time.perf_counter()
        res = fgmres(lambda v: gp.A @ v, ls.apply, gp.rhs(wl.sources[0]), tol=1e-6)
        t2 = time.perf_counter()
    return {"value": round((t2 - t1) * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": (f"one solve to 1e-6 of the same recipe downscaled to {wl.n}^3 bulk, {wl.q}x{wl.r} beams "
                       f"({m.shape[0]}^3 extended points; {res.iterations} iterations, {ls.solves} SuperLU beam "
                       f"solves); setup {round((t1 - t0) * 1e3)} ms not included; the full 95^3 workload does not "
                       f"fit the oracle (one beam's SuperLU factorisation takes ~400 s and 9 GB, the global "
                       f"banded LU 809 GB)"),
            "iterations": res.iterations}


def zgbsv_baseline(workload: str = "lens2d"):
    """The oracle's exact solve (LAPACK zgbsv on the band of the global operator, factor + solve)
    of a 2D workload, with BLAS threads = all cores of this process and = 1."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle.direct import solve_banded
    from oracle.discretization import GlobalProblem, extend_normal
    from paper_1909_01467_amd import inputs

    wl = inputs.workload(workload)
    m = extend_normal(wl.slowness2, wl.n_pml)
    gp = GlobalProblem(m, wl.omega, wl.n, wl.n_pml, wl.C)
    b = gp.rhs(wl.sources[0])
    out = {"workload": f"{workload} ({wl.n}^2 bulk + {wl.n_pml}-pt PML, {m.size} unknowns, band {m.shape[1]})"}
    for label, lim in (("all_cores", len(os.sched_getaffinity(0))), ("one_core", 1)):
        with threadpool_limits(limits=lim):
            threads = max((i["num_threads"] for i in threadpool_info() if i.get("user_api") == "blas"), default=lim)
            t0 = time.perf_counter()
            solve_banded(gp.A, b)
            out[label] = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "blas_threads": threads}
    return out


def cpu_baseline(workload: str, windows: bool = False):
    """The FP64 oracle (Alg. Scenario3, or scenario 4 with windows, with SuperLU local solves
    inside FGMRES), timed on the host on the same workload: setup and one solve to 1e-6."""
    from threadpoolctl import threadpool_limits

    from oracle.discretization import GlobalProblem, extend_normal
    from oracle.fgmres import fgmres
    from oracle.lsweep import LSweep2D
    from oracle.scenario4 import Scenario4
    from paper_1909_01467_amd import inputs

    wl = inputs.workload(workload)
    with threadpool_limits(limits=1):
        m = extend_normal(wl.slowness2, wl.n_pml)
        t0 = time.perf_counter()
        gp = GlobalProblem(m, wl.omega, wl.n, wl.n_pml, wl.C)
        ls = (Scenario4 if windows else LSweep2D)(m, wl.omega, wl.n, wl.n_pml, wl.q, wl.r, wl.C)
        t1 = time.perf_counter()
        b = gp.rhs(wl.sources[0])
        res = fgmres(lambda v: gp.A @ v, ls.apply, b, tol=1e-6)
        t2 = time.perf_counter()
    return {"value": round((t2 - t1) * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of the same workload to 1e-6 ({res.iterations} iterations, "
                      f"{ls.solves} SuperLU local solves); setup {round((t1 - t0) * 1e3)} ms not included",
            "iterations": res.iterations}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lens3d")
    ap.add_argument("--no-zgbsv", action="store_true", help="skip the banded-LU oracle timing of lens2d")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--windows", action="store_true",
                    help="scenario 4 (Sec. 2.1): the CDD and three shifted copies with a partition of unity")
    ap.add_argument("--all-sources", action="store_true",
                    help="solve for all of the workload's sources in one batch (nrhs = number of sources)")
    ap.add_argument("--maxit", type=int, default=500)
    ap.add_argument("--restart", type=int, default=50, help="FGMRES restart (the basis holds restart+1 vectors per rhs)")
    ap.add_argument("--apply-reps", type=int, default=20,
                    help="applications timed one by one for the per-kernel times (median)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one device copy of this many MiB (calibrates FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; sharding over several GPUs is "
                                   "not implemented. Use --gpus 1."}))
        sys.exit(2)

    import torch

    from paper_1909_01467_amd.lsweeps import Solver

    torch.cuda.set_device(0)
    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe", args.copy_probe_mb, "MiB read and written once")
        del src, dst
    wl, m_ext, b = make_problem(args.workload, args.all_sources)
    nrhs = b.shape[0] if args.all_sources else 1
    log("workload", wl.name, "n", wl.n, "q", wl.q, "omega", round(wl.omega, 2))
    results = {}
    for precision in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        s = Solver(m_ext, wl.omega, wl.h, wl.n, wl.n_pml, wl.q, wl.r, C=wl.C, precision=precision, tol=1e-6,
                   windows=args.windows, nrhs_max=nrhs, maxit=args.maxit, restart=args.restart)
        st0 = s.stats()
        log(precision, "setup ms", round(st0["t_setup_ms"], 1), "factor ms", round(st0["t_factor_ms"], 1))
        u, info, ms = time_solves(s, b, args.steps, args.warmup)
        med, st = time_applies(s, b, max(1, args.apply_reps))
        conv = all(info["converged"]) and max(info["relres"]) <= 1e-6
        if precision == "mixed" and not conv:   # an unconverged solve time is no measurement
            raise SystemExit(f"the mixed solve did not reach 1e-6: {info}")
        log(precision, "solve ms", round(ms, 3), "iterations", info["iterations"], "relres", info["relres"],
            "apply ms", round(med["last_apply_ms"], 4), "stage1 ms", round(med["last_stage1_ms"], 4),
            "gemv ms", round(med["last_gemv_ms"], 4), "final rhs ms", round(med["last_final_rhs_ms"], 4),
            "final ms", round(med["last_final_ms"], 4), "Q setup ms", round(st["t_q_ms"], 1),
            "sweep items", st["gemv_items"], "max inputs", st["gemv_max_inputs"])
        results[precision] = dict(ms=ms, info=info, med=med, stats=st, converged=conv)
        s.close()
        torch.cuda.synchronize()

    main_r = results["mixed"]
    st = main_r["stats"]
    med = main_r["med"]
    # one entry per kernel symbol launched by an application
    if wl.dim == 3:
        # every front: k_rhs3, then per plane step the factor-reading kernel (timed launch by
        # launch with events on the library's stream) and, on packed blocks, k_red3; then k_epi3
        fronts_ms = med["last_stage1_ms"] + med["last_gemv_ms"]
        if st.get("symmetric_factors"):
            kernels = {
                "k_tile3": dict(desc="3D twisted substitution plane steps on the packed symmetric plane blocks: one "
                                     "64x64 tile of the upper triangle per workgroup, tile v_J and tile^T v_I",
                                launches=st["dom_launches"], bytes=st["dom_bytes"], ms=med["last_dom_ms"]),
                "k_red3+k_rhs3+k_epi3": dict(desc="fixed-order sums of the tile partials per 64-row block; right-hand "
                                                  "sides and epilogues of the fronts", launches=0, bytes=0.0,
                                             ms=fronts_ms - med["last_dom_ms"]),
            }
        else:
            kernels = {
                "k_step3": dict(desc="3D twisted plane-block substitutions of every front (64 rows of G_k per "
                                     "workgroup)", launches=st["dom_launches"], bytes=st["dom_bytes"],
                                ms=med["last_dom_ms"]),
            }
    else:
        # the substitutions: one right-hand side per workgroup on the packed symmetric factors
        # (k_chain_sym, every right-hand side reads every block), or R per workgroup on the full
        # blocks (k_chain_mr, R = 2 or 4; k_chain_mma on matrix cores, R = 16 or 32), each block
        # read once per group of R; the sweeps read Q' once per launch for the whole batch.  With
        # windows every family runs once per CDD (four times).
        sym = bool(st.get("symmetric_factors"))
        ncdd = st["cdd_count"]
        R = st["rhs_per_workgroup"] if nrhs > 1 else 1
        if R == 1:
            chain = "k_chain_sym" if sym else "k_chain"
            layout = ("packed symmetric factors, 4x4 tiles of the upper triangle" if sym else "full factor blocks")
            s1_bytes, fi_bytes = nrhs * st["apply_stage1_bytes"], nrhs * st["apply_final_bytes"]
        else:
            groups = -(-nrhs // R)
            chain = "k_chain_mma" if R >= 16 else "k_chain_mr"
            layout = (f"full factor blocks, {R} right-hand sides per workgroup"
                      + (" as W x W by W x R products on matrix cores" if R >= 16 else ""))
            s1_bytes, fi_bytes = groups * st["apply_stage1_full_bytes"], groups * st["apply_final_full_bytes"]
        gemv_mma = nrhs > 1 and bool(st.get("gemv_mma"))
        gemv = "k_gemv_mma" if gemv_mma else "k_gemv"
        kernels = {
            f"{chain}<CS_STAGE1>": dict(desc=f"stage-1 block substitutions, twisted (forward halves; middle + backward "
                                             f"halves), {layout}",
                                        launches=2 * ncdd, bytes=s1_bytes, ms=med["last_stage1_ms"]),
            gemv: dict(desc=("trace-compressed sweep fronts: out = Q' u~ per solve, " +
                             ("16 or 32 right-hand sides per workgroup on matrix cores" if gemv_mma else
                              "batched GEMV")),
                       launches=st["gemv_launches"], bytes=st["apply_gemv_bytes"], ms=med["last_gemv_ms"]),
            f"{chain}<CS_FINAL>": dict(desc=f"final z block substitutions, twisted (forward halves; middle + backward "
                                            f"halves), {layout}",
                                       launches=2 * ncdd, bytes=fi_bytes, ms=med["last_final_ms"]),
        }
        # matrix-core kernels: 8 real flops per complex entry read and right-hand side (complex64
        # entries of 8 bytes: flops = bytes read per group x right-hand sides)
        if R >= 16:
            kernels[f"{chain}<CS_STAGE1>"]["flops"] = st["apply_stage1_full_bytes"] * nrhs
            kernels[f"{chain}<CS_FINAL>"]["flops"] = st["apply_final_full_bytes"] * nrhs
        if gemv_mma:
            kernels[gemv]["flops"] = st["apply_gemv_bytes"] * nrhs
    for k in kernels.values():
        k["bytes_per_launch"] = k["bytes"] / max(1, k["launches"])
        k["avg_launch_ms"] = k["ms"] / max(1, k["launches"])
        k["gbps"] = k["bytes_per_launch"] / max(1e-12, k["avg_launch_ms"] * 1e-3) / 1e9 if k["launches"] else 0.0
        if k.get("flops"):
            k["tflops"] = k["flops"] / max(1, k["launches"]) / max(1e-12, k["avg_launch_ms"] * 1e-3) / 1e12
    dom_name = max((n for n in kernels if kernels[n]["launches"]), key=lambda n: kernels[n]["ms"])
    dom = kernels[dom_name]
    achieved = dom["gbps"]
    mfma = dom.get("flops", 0) > 0   # a matrix-core kernel: priced against the FP32 matrix peak
    if mfma:
        achieved = dom["flops"] / max(1, dom["launches"]) / max(1e-12, dom["avg_launch_ms"] * 1e-3) / 1e12
    apply_bytes = sum(k["bytes"] for k in kernels.values())   # algorithmic bytes of one application of the batch
    out = {
        "metric": METRIC,
        "value": round(main_r["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": (f"{wl.name}: {wl.n}^2 bulk + {wl.n_pml}-pt PML, {wl.q}x{wl.r} CDD, {MEDIA[wl.name]}, "
                         f"10 ppw (omega={wl.omega:.2f}), {nrhs} Gaussian source{'s' if nrhs > 1 else ''}"
                         f"{' in one batch' if nrhs > 1 else ''}, GMRES tol 1e-6") if wl.dim == 2 else
                        (f"{wl.name}: {wl.n}^3 bulk + {wl.n_pml}-pt PML, {wl.q}x{wl.r} beam CDD (full z), "
                         f"{MEDIA[wl.name]}, 8 ppw (omega={wl.omega:.2f}), 1 Gaussian source, GMRES tol 1e-6"),
            "preconditioner": ("scenario 4: the CDD and three copies shifted by (%d, %d) points, windowed "
                               "right-hand sides (Sec. 2.1)" % tuple(st["window_shift"]) if args.windows else
                               "scenario 3: one CDD (Alg. Scenario3)"),
            "precision": "complex64 factors and sweeps, FP64 FGMRES",
            "iterations": max(main_r["info"]["iterations"]),
            "relres": max(main_r["info"]["relres"]),
            "apply_ms": round(med["last_apply_ms"], 4),
            "apply_GBps_algorithmic": round(apply_bytes / (med["last_apply_ms"] * 1e-3) / 1e9, 1),
            "apply_frac_of_hbm_peak": round(apply_bytes / (med["last_apply_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "final_rhs_ms": round(med["last_final_rhs_ms"], 4),
            "t_setup_ms": round(st["t_setup_ms"], 1),
            "t_factor_ms": round(st["t_factor_ms"], 1),
            "t_Q_ms": round(st["t_q_ms"], 1),
            "kernels": {n: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in k.items()}
                        for n, k in kernels.items()},
        },
        "roofline": {
            "bound": "mfma" if mfma else "hbm",
            "kernel": f"{dom_name}: {dom['desc']}",
            "achieved": round(achieved, 1),
            "peak": FP32_MATRIX_PEAK_TFLOPS if mfma else HBM_PEAK_GBS,
            "unit": "TFLOP/s" if mfma else "GB/s",
            "frac": round(achieved / (FP32_MATRIX_PEAK_TFLOPS if mfma else HBM_PEAK_GBS), 4),
            "traffic": (counter_traffic(dom_name, args.workload, dom["bytes_per_launch"])
                        if not args.windows and not args.all_sources else None),
            "algorithmic_bytes_per_launch": round(dom["bytes_per_launch"]),
            "avg_launch_ms": round(dom["avg_launch_ms"], 5),
        },
    }
    if "fp64" in results:
        f = results["fp64"]
        out["config"]["fp64_ms_per_step"] = round(f["ms"], 3)
        out["config"]["fp64_iterations"] = max(f["info"]["iterations"])
        out["config"]["fp64_relres"] = max(f["info"]["relres"])
        out["config"]["fp64_apply_ms"] = round(f["med"]["last_apply_ms"], 4)
        if f["converged"]:   # both reached 1e-6: the speedup is at equal final residual
            out["config"]["mixed_speedup_vs_fp64"] = round(f["ms"] / main_r["ms"], 3)
        else:
            out["config"]["fp64_note"] = "the FP64 solve did not reach 1e-6; no speedup is reported"
    if not args.no_cpu_baseline and nrhs == 1 and not (wl.dim == 3 and args.windows):
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline_3d(args.workload) if wl.dim == 3 else cpu_baseline(args.workload, args.windows)
        cb["cpu_model"] = cpu_model()
        cb["host_cores"] = len(os.sched_getaffinity(0))
        if not args.no_zgbsv:
            log("cpu baseline: banded LU of lens2d ...")
            cb["zgbsv_lens2d"] = zgbsv_baseline("lens2d")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
