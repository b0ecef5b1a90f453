"""Benchmark: time-to-solution of the nested SAP/SSOR solver on one MI355X.

A step is one full solve of D x = b to a true relative residual of 1e-10 on the
24^3x48 workload: synthetic SU(3) links (eps 0.25, seed 2), c_SW 1.0, kappa 0.125,
SAP blocks 6^3x12 with 16 sub-blocks of 3^3x6, SSOR omega 1.0 x 4 sweeps, N_SAP 4,
FP32 inner BiCGStab inside an FP64 flexible BiCGStab, one complex Gaussian source.
Fields and source are resident in HBM before the timed region starts.

Prints ONE JSON line.  The roofline object describes the dominant kernel (the
fused SAP phase kernel: gather, SSOR sweeps, block hop), timed with HIP events
on the library's stream during the timed solves.  The cpu_baseline object is the
FP64 oracle's own full solve of the same system, timed on the host's threads; the
accuracy object gives the GPU solution's error against the oracle's 1e-12 solve and
its true residual with the oracle's operator.  The learned_stage object is the
NN-augmented FP16 batched solver against the plain FP32 solver at 48^3x96 (12
point sources), with the network trained on the GPU in the same run.
"""
import argparse
import hashlib

import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3         # MI355X vector FP32 (published)
HOP_FLOPS = 168                  # one spin-projected hop: project 12 + 2 SU(3) x half-spinor 132 + rebuild 24
CLOVER_FLOPS = 552               # two hermitian 6x6 complex mat-vecs
AXPY_FLOPS = 48                  # x = v + kappa F h on 12 complex entries

WORKLOADS = {
    "24^3x48": dict(L=(24, 24, 24, 48), B=(6, 6, 6, 12), S=(3, 3, 3, 6), kappa=0.125, csw=1.0, eps=0.25,
                    seed=2, seed_b=1002),
    "8^4": dict(L=(8, 8, 8, 8), B=(4, 4, 4, 4), S=(2, 2, 2, 2), kappa=0.120, csw=1.0, eps=0.25, seed=1,
                seed_b=1001),
    "32^3x64": dict(L=(32, 32, 32, 64), B=(4, 4, 4, 4), S=(2, 2, 2, 2), kappa=0.125, csw=1.0, eps=0.25, seed=3,
                    seed_b=1003),
    "24^3x48/4^4": dict(L=(24, 24, 24, 48), B=(4, 4, 4, 4), S=(2, 2, 2, 2), kappa=0.125, csw=1.0, eps=0.25, seed=2,
                        seed_b=1002),
}


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters of rocprofv3 (run this mode under the profiler), and without the profiler the
    copy and fill rates the box reaches."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        b.fill_(2.0)
    torch.cuda.synchronize()
    df = (time.perf_counter() - t0) / reps
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
                      "launches": reps, "GBps_read_plus_write": 2 * nbytes / dt / 1e9,
                      "fill_GBps": nbytes / df / 1e9}), flush=True)


def make_inputs(w):
    from paper_1210_7398_amd import synth

    t0 = time.time()
    U = synth.gauge_field(w["L"], w["eps"], w["seed"])
    F = synth.clover_inverse(w["L"], U, w["csw"], w["kappa"])
    b = synth.gaussian_spinor(w["L"], w["seed_b"])
    print(f"# inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    return U, F, b


def omp_threads(n=None):
    """Threads the oracle's OpenMP loops use (set to n first if given)."""
    import ctypes

    import oracle

    oracle.lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def oracle_solve_chunked(L, B, S, U, F, kappa, b, tol, label, chunk=2, max_calls=200):
    """The oracle's solve of D x = b to tol in calls of `chunk` outer iterations, each resuming
    from the last iterate and printing its residual, so that a long solve reports progress.
    Returns (x, converged, seconds)."""
    import oracle

    prm = oracle.params(kappa, tol_inner=0.1, maxit_outer=chunk)
    x, t0 = None, time.perf_counter()
    for k in range(max_calls):
        x, st, ok = oracle.solve(L, B, S, U, F, prm, b, tol=tol, x0=x)
        print(f"# oracle {label}: call {k}, relres {st['relres']:.2e} after {time.perf_counter() - t0:.0f} s",
              file=sys.stderr, flush=True)
        if ok:
            return x, True, time.perf_counter() - t0
    return x, False, time.perf_counter() - t0


def oracle_reference(w, U, F, b, x_gpu, tol=1e-10, tol_inner=0.1, one_thread_sample=True):
    """The FP64 CPU oracle beside the GPU solve of the same system (fields, source, blocks,
    sweeps and inner tolerance).  Returns (cpu_baseline, accuracy):
    - cpu_baseline: the oracle's full solve to tol, timed at all the threads OpenMP gives it;
      with one_thread_sample, one DK application (Algorithm 1) and one operator application
      timed at 1 thread, scaled by the solve's counts as a labelled single-thread estimate;
    - accuracy: the oracle's solve continued to 1e-12 (x_oracle), the GPU solution's error
      |x - x_oracle| / |x_oracle|, and its true residual |b - D x| / |b| with the oracle's D."""
    import oracle

    L, B, S, kappa = w["L"], w["B"], w["S"], w["kappa"]
    nthreads = omp_threads()
    prm = oracle.params(kappa, tol_inner=tol_inner)
    t0 = time.perf_counter()
    xo, st, ok = oracle.solve(L, B, S, U, F, prm, b, tol=tol)
    t_solve = time.perf_counter() - t0
    print(f"# oracle solve to {tol:g}: {t_solve:.1f} s on {nthreads} threads, outer {st['outer']} inner "
          f"{st['inner']} relres {st['relres']:.2e}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    xo12, st12, ok12 = oracle.solve(L, B, S, U, F, prm, b, tol=1e-12, x0=xo)
    t12 = time.perf_counter() - t0
    rr = float(np.linalg.norm(b - oracle.dslash(L, U, F, kappa, x_gpu)) / np.linalg.norm(b))
    err = float(np.linalg.norm(x_gpu - xo12) / np.linalg.norm(xo12))
    cpu = dict(value=t_solve, unit="s", cores=nthreads, kind="oracle",
               sample=(f"full FP64 oracle solve of the same system to {tol:g} from x = 0 (nested flexible "
                       f"BiCGStab, M_SAP N_SAP 4, SSOR x4, inner tolerance {tol_inner}), timed on {nthreads} "
                       f"OpenMP threads: {st['outer']} outer and {st['inner']} inner iterations, true relative "
                       f"residual {st['relres']:.2e}"),
               converged=bool(ok))
    if one_thread_sample:
        omp_threads(1)
        v = np.ascontiguousarray(b)
        t0 = time.perf_counter()
        oracle.dk(L, B, S, U, F, prm, v)
        t_dk = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.dslash(L, U, F, kappa, v)
        t_d = time.perf_counter() - t0
        omp_threads(nthreads)
        n_dk = 4 * (2 * st["inner"] + 1)  # N_SAP DKs per M_SAP, about two M_SAP per inner iteration
        cpu["one_thread"] = dict(dk_s=t_dk, dslash_s=t_d, estimate_s=n_dk * t_dk,
                                 note=("timed sample at 1 thread: one DK application and one operator "
                                       "application; estimate_s = the solve's ~4 (2 inner + 1) DK "
                                       "applications times the DK time (an estimate, not a measurement)"))
    acc = dict(err_vs_oracle=err, true_relres_oracle_D=rr, oracle_relres_1e12=st12["relres"],
               oracle_continue_to_1e12_s=t12,
               note=("x_oracle: the oracle's solve continued to 1e-12; err_vs_oracle = |x - x_oracle| / "
                     "|x_oracle|; true_relres_oracle_D = |b - D x| / |b| with the oracle's D"))
    return cpu, acc


def precision_study(args):
    """The precision workload: one lattice solved with FP32, FP16 and BF16 storage for the SAP
    preconditioner and inner solver, FP64 outer iteration, tol 1e-10.  Prints one JSON line
    with time-to-solution, iteration counts, FP64 true residual and the difference of each
    solution from the FP32-storage one."""
    import torch

    from paper_1210_7398_amd import sapq

    wl = "32^3x64" if args.workload == "24^3x48" else args.workload
    w = WORKLOADS[wl]
    U, F, b = make_inputs(w)
    dev = torch.device("cuda:0")
    Ud, Fd, bd = (torch.from_numpy(a).to(dev) for a in (U, F, b))
    res, xref, xs = [], None, []
    for prec in ("fp32", "fp16", "bf16"):
        s = sapq.Solver(w["L"], w["B"], w["S"], w["kappa"], prec=prec, outer=args.outer, maxit_outer=400, device=dev)
        s.load_gauge(Ud)
        s.load_clover(Fd)
        s.solve(bd, tol=1e-10)  # warm-up
        times, st = [], None
        for _ in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = s.solve(bd, tol=1e-10, profile=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        if xref is None:
            xref = x.clone()
        diff = float(torch.linalg.vector_norm(x - xref) / torch.linalg.vector_norm(xref))
        xs.append(x.cpu().numpy())
        ph = st["kernels"].get("phase_E", {}), st["kernels"].get("phase_O", {})
        n_ph = ph[0].get("n", 0) + ph[1].get("n", 0)
        res.append(dict(prec=prec, time_s=sorted(times)[len(times) // 2], outer_its=st["outer_its"],
                        inner_its=st["inner_its"], n_msap=st["n_msap"], true_relres=st["true_relres"],
                        rel_diff_vs_fp32_storage=diff,
                        sap_phase_avg_us=(1e3 * (ph[0].get("ms", 0) + ph[1].get("ms", 0)) / n_ph) if n_ph else None))
        print(f"# {prec}: {res[-1]}", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    # the error of every run against the FP64 oracle's own solve of the system to 1e-12
    import oracle

    del Ud, Fd
    xo, ok, t_or = oracle_solve_chunked(w["L"], w["B"], w["S"], U, F, w["kappa"], b, 1e-12, wl)
    sto = dict(relres=float(np.linalg.norm(b - oracle.dslash(w["L"], U, F, w["kappa"], xo)) / np.linalg.norm(b)))
    for r, x in zip(res, xs):
        r["err_vs_oracle"] = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
        r["true_relres_oracle_D"] = float(np.linalg.norm(b - oracle.dslash(w["L"], U, F, w["kappa"], x))
                                          / np.linalg.norm(b))
    oracle_info = dict(tol=1e-12, converged=bool(ok), relres=sto["relres"], time_s=t_or, threads=omp_threads())
    print(json.dumps({"mode": "precision", "workload": wl, "outer": args.outer, "tol": 1e-10, "results": res,
                      "oracle": oracle_info}), flush=True)


def _solve_stats(s, bd, steps, x_oracle=None):
    """Median time of `steps` solves after one warm-up, with the last solve's statistics; with
    x_oracle (host), the last solution's error against it is added to the statistics."""
    import torch

    s.solve(bd, tol=1e-10)
    times, st = [], None
    for _ in range(max(1, steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = s.solve(bd, tol=1e-10, profile=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    if x_oracle is not None:
        xh = x.cpu().numpy()
        st["err_vs_oracle"] = float(np.linalg.norm(xh - x_oracle) / np.linalg.norm(x_oracle))
    ph = st["kernels"].get("phase_E", {}), st["kernels"].get("phase_O", {})
    n_ph = ph[0].get("n", 0) + ph[1].get("n", 0)
    return sorted(times)[len(times) // 2], st, (1e3 * (ph[0].get("ms", 0) + ph[1].get("ms", 0)) / n_ph) if n_ph else None


def c2_oracle_solution(w, U, F, b):
    """The oracle's solve of the 24^3x48 workload's system to 1e-12 (the reference solution the
    studies state their error against)."""
    x, ok, t = oracle_solve_chunked(w["L"], w["B"], w["S"], U, F, w["kappa"], b, 1e-12, "24^3x48")
    if not ok:
        raise RuntimeError("the oracle's reference solve did not converge")
    return x, t


# (block, sub-block, block solver) of the block study at 24^3x48: sub-block = block is the
# natural-order SSOR, sub-block (0, 0, 0, 0) the even-odd site order; "eomr" replaces the SSOR
# by the even-odd site-preconditioned minimal-residual block solve at the same cost (the block
# solvers the paper measures the ll-ordered SSOR against)
BLOCK_SHAPES = [((6, 6, 6, 12), (3, 3, 3, 6), "ssor"), ((6, 6, 6, 12), (2, 2, 2, 4), "ssor"),
                ((6, 6, 6, 12), (3, 3, 3, 3), "ssor"), ((6, 6, 6, 12), (6, 6, 6, 12), "ssor"),
                ((6, 6, 6, 6), (3, 3, 3, 3), "ssor"), ((6, 6, 6, 6), (2, 2, 2, 2), "ssor"),
                ((6, 6, 6, 6), (6, 6, 6, 6), "ssor"), ((6, 6, 6, 6), (0, 0, 0, 0), "ssor"),
                ((6, 6, 6, 6), (0, 0, 0, 0), "eomr"), ((4, 4, 4, 4), (2, 2, 2, 2), "ssor"),
                ((4, 4, 4, 4), (4, 4, 4, 4), "ssor"), ((4, 4, 4, 4), (0, 0, 0, 0), "ssor"),
                ((4, 4, 4, 4), (0, 0, 0, 0), "eomr")]


def blocks_study(args):
    """Block and sub-block shapes and block solvers at 24^3x48 (the default workload's fields and
    source): M_SAP applications and time to 1e-10 for each, with the phase kernel each runs."""
    import torch

    from paper_1210_7398_amd import sapq

    w = WORKLOADS["24^3x48"]
    U, F, b = make_inputs(w)
    dev = torch.device("cuda:0")
    Ud, Fd, bd = (torch.from_numpy(a).to(dev) for a in (U, F, b))
    xo, t_or = c2_oracle_solution(w, U, F, b)
    del U, F
    res = []
    for B, S, solver in BLOCK_SHAPES:
        s = sapq.Solver(w["L"], B, S, w["kappa"], device=dev, block_solver=solver)
        s.load_gauge(Ud)
        s.load_clover(Fd)
        t, st, ph_us = _solve_stats(s, bd, args.steps, xo)
        res.append(dict(block=list(B), subblock=list(S), block_solver=solver, phase_kernel=s.phase_kernel, time_s=t,
                        n_msap=st["n_msap"],
                        inner_its=st["inner_its"], outer_its=st["outer_its"], true_relres=st["true_relres"],
                        err_vs_oracle=st["err_vs_oracle"], sap_phase_avg_us=ph_us))
        print(f"# {res[-1]}", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "blocks", "lattice": list(w["L"]), "kappa": w["kappa"], "tol": 1e-10, "results": res,
                      "oracle": dict(tol=1e-12, time_s=t_or, threads=omp_threads(),
                                     note="err_vs_oracle = |x - x_oracle| / |x_oracle|, x_oracle the oracle's 1e-12 "
                                          "solve of the same system")}), flush=True)


def nsap_study(args):
    """N_SAP (SAP cycles per M_SAP application, which the paper leaves open) at 24^3x48 with
    the workload's fields, source and blocks: time to 1e-10, M_SAP applications and phase
    launches for N_SAP = 1, 2, 3, 4, 6, 8."""
    import torch

    from paper_1210_7398_amd import sapq

    w = WORKLOADS["24^3x48"]
    U, F, b = make_inputs(w)
    dev = torch.device("cuda:0")
    Ud, Fd, bd = (torch.from_numpy(a).to(dev) for a in (U, F, b))
    xo, t_or = c2_oracle_solution(w, U, F, b)
    del U, F
    res = []
    for n_sap in (1, 2, 3, 4, 6, 8):
        s = sapq.Solver(w["L"], w["B"], w["S"], w["kappa"], n_sap=n_sap, maxit_outer=400, device=dev)
        s.load_gauge(Ud)
        s.load_clover(Fd)
        t, st, ph_us = _solve_stats(s, bd, args.steps, xo)
        res.append(dict(n_sap=n_sap, time_s=t, n_msap=st["n_msap"], phase_launches=2 * n_sap * st["n_msap"],
                        inner_its=st["inner_its"], outer_its=st["outer_its"], true_relres=st["true_relres"],
                        err_vs_oracle=st["err_vs_oracle"], sap_phase_avg_us=ph_us))
        print(f"# {res[-1]}", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "nsap", "lattice": list(w["L"]), "block": list(w["B"]), "subblock": list(w["S"]),
                      "kappa": w["kappa"], "tol": 1e-10, "results": res}), flush=True)


def omega_study(args):
    """SSOR relaxation omega (the paper gives none; the workload uses 1) at 24^3x48 with the
    workload's fields and blocks: time to 1e-10 and M_SAP applications of the workload's source
    for omega from 0.8 to 1.4, and the M_SAP applications of three more Gaussian sources."""
    import torch

    from paper_1210_7398_amd import sapq, synth

    w = WORKLOADS["24^3x48"]
    U, F, b = make_inputs(w)
    dev = torch.device("cuda:0")
    Ud, Fd, bd = (torch.from_numpy(a).to(dev) for a in (U, F, b))
    extra = [torch.from_numpy(synth.gaussian_spinor(w["L"], w["seed_b"] + k)).to(dev) for k in (1, 2, 3)]
    xo, t_or = c2_oracle_solution(w, U, F, b)
    del U, F
    res = []
    for omega in (0.8, 0.9, 1.0, 1.1, 1.2, 1.3, 1.4):
        s = sapq.Solver(w["L"], w["B"], w["S"], w["kappa"], omega=omega, maxit_outer=400, device=dev)
        s.load_gauge(Ud)
        s.load_clover(Fd)
        t, st, ph_us = _solve_stats(s, bd, args.steps, xo)
        n_extra = [s.solve(e, tol=1e-10)[1]["n_msap"] for e in extra]
        res.append(dict(omega=omega, time_s=t, n_msap=st["n_msap"], inner_its=st["inner_its"],
                        outer_its=st["outer_its"], true_relres=st["true_relres"], err_vs_oracle=st["err_vs_oracle"],
                        sap_phase_avg_us=ph_us, n_msap_more_sources=n_extra))
        print(f"# {res[-1]}", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "omega", "lattice": list(w["L"]), "block": list(w["B"]), "subblock": list(w["S"]),
                      "kappa": w["kappa"], "tol": 1e-10, "results": res}), flush=True)


def msap_flops(B, V, n_ssor=4, n_sap=4):
    """Algorithmic flops of one M_SAP application on V sites (phase model, Table 1 counts)."""
    face = sum(2.0 / b for b in B)
    _, ph = phase_model(B, n_ssor, 4)
    return n_sap * V * ph + (V // 2) * (face * HOP_FLOPS + CLOVER_FLOPS + AXPY_FLOPS)


def sustained_study(args):
    """Sustained rate of the solver at three lattice sizes with 6^3x12 blocks: algorithmic flops
    of the M_SAP applications and FP64 operator applications of a solve, divided by its time
    (the BiCGStab vector updates are not counted)."""
    import torch

    from paper_1210_7398_amd import sapq, synth

    dev = torch.device("cuda:0")
    res = []
    for L, seed in (((12, 12, 12, 24), 41), ((24, 24, 24, 48), 2), ((48, 48, 48, 96), 43)):
        B, S, kappa = (6, 6, 6, 12), (3, 3, 3, 6), 0.125
        Ud = synth.gauge_field(L, 0.25, seed, device=dev)
        Fd = synth.clover_inverse(L, Ud, 1.0, kappa, device=dev)
        bd = torch.from_numpy(synth.gaussian_spinor(L, 1000 + seed)).to(dev)
        s = sapq.Solver(L, B, S, kappa, device=dev)
        s.load_gauge(Ud)
        s.load_clover(Fd)
        Uh, Fh, bh = Ud.cpu().numpy(), Fd.cpu().numpy(), bd.cpu().numpy()
        del Ud, Fd
        t, st, ph_us = _solve_stats(s, bd, args.steps)
        # the GPU solution against the oracle: its error against the oracle's 1e-12 solve where
        # that solve is feasible, else (48^3x96) only its residual with the oracle's D
        import oracle

        xg = s.solve(bd, tol=1e-10)[0].cpu().numpy()
        acc = dict(true_relres_oracle_D=float(np.linalg.norm(bh - oracle.dslash(L, Uh, Fh, kappa, xg))
                                              / np.linalg.norm(bh)))
        if L[3] <= 48:
            xo, ok, _ = oracle_solve_chunked(L, B, S, Uh, Fh, kappa, bh, 1e-12, "x".join(map(str, L)))
            acc["err_vs_oracle"] = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
        del Uh, Fh, bh, xg
        V = int(np.prod(L))
        fl = st["n_msap"] * msap_flops(B, V) + st["n_dslash64"] * V * (8 * HOP_FLOPS + CLOVER_FLOPS + AXPY_FLOPS)
        res.append(dict(lattice=list(L), time_s=t, n_msap=st["n_msap"], n_dslash64=st["n_dslash64"],
                        true_relres=st["true_relres"], flops=fl, TFLOPs=fl / t / 1e12,
                        frac_fp32_peak=fl / t / 1e12 / FP32_PEAK_TFLOPS,
                        frac_fp32_unpacked=fl / t / 1e12 / (FP32_PEAK_TFLOPS / 2), sap_phase_avg_us=ph_us, **acc))
        print(f"# {res[-1]}", file=sys.stderr, flush=True)
        s.close()
        del s, bd
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "sustained", "block": [6, 6, 6, 12], "subblock": [3, 3, 3, 6], "tol": 1e-10,
                      "results": res}), flush=True)


BATCH_FIELDS = [((16, 16, 16, 32), 0.2, 11), ((24, 24, 24, 48), 0.25, 12), ((24, 24, 24, 48), 0.3, 13),
                ((32, 32, 32, 64), 0.25, 14)]


def batch_study(args):
    """The batched workload: 12 spin-colour point sources on each of four gauge fields of mixed
    sizes (16^3x32 eps 0.2, 24^3x48 eps 0.25 and 0.3, 32^3x64 eps 0.25), kappa 0.125, 4^4 SAP
    blocks with the sub-block shape chosen by the autotuner, solved together by one
    sapq_solve_batch call (graph-captured inner iterations); compared with solving the same
    48 sources one at a time.  Prints one JSON line."""
    import tempfile

    import torch

    from paper_1210_7398_amd import sapq, synth

    kappa, B = 0.125, (4, 4, 4, 4)
    dev = torch.device("cuda:0")
    t0 = time.time()
    flds, host_fields = [], []
    for L, eps, seed in BATCH_FIELDS:
        U = synth.gauge_field(L, eps, seed, device=dev)
        F = synth.clover_inverse(L, U, 1.0, kappa, device=dev)
        flds.append((L, U, F))
        host_fields.append((L, U.cpu().numpy(), F.cpu().numpy()))
        torch.cuda.synchronize()
        print(f"# field {L} ready after {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    print(f"# fields generated on the GPU in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    cache = os.path.join(tempfile.mkdtemp(), "tune.jsonl")
    L0, U0, F0 = flds[0]
    tuner = sapq.Solver(L0, B, (2, 2, 2, 2), kappa, prec=args.prec, outer="defect", device=dev)
    tuner.load_gauge(U0)
    tuner.load_clover(F0)
    t0 = time.time()
    S = tuner.autotune(cache)
    tune_s = time.time() - t0
    tuner.close()
    print(f"# autotuned sub-block {S} in {tune_s:.1f} s", file=sys.stderr, flush=True)
    solvers, srcs = [], []
    for L, U, F in flds:
        s = sapq.Solver(L, B, S, kappa, prec=args.prec, outer="defect", device=dev)
        s.load_gauge(U)
        s.load_clover(F)
        V = synth.volume(L)
        b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
        for k in range(12):
            b[k, 0, k % 4, k // 4] = 1.0
        solvers.append(s)
        srcs.append(b)
    del flds
    # the batched kernels' sources per workgroup and inner iterations per graph replay, timed
    # on the batch itself (median of 3 solves per candidate, to 1e-6 to keep the tuning short)
    t0 = time.time()
    # a fresh cache file, so that the autotuner times every candidate and records them
    import tempfile

    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "batch_tune.jsonl")
        nr, k_inner = sapq.autotune_batch(solvers, srcs, tol=1e-6, cache_path=cache)
        tune_rec = json.loads(open(cache).read().strip().splitlines()[-1])
    tune_batch_s = time.time() - t0
    print(f"# batch autotune: {nr} sources per workgroup, {k_inner} inner iterations per replay "
          f"({tune_batch_s:.1f} s)", file=sys.stderr, flush=True)
    xs, st = sapq.solve_batch(solvers, srcs, tol=1e-10)  # warm-up
    times = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xs, st = sapq.solve_batch(solvers, srcs, tol=1e-10)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    t_batch = sorted(times)[len(times) // 2]
    print(f"# batched: {t_batch:.3f} s for 48 sources", file=sys.stderr, flush=True)
    # the same 48 sources one at a time with the one-source solver
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seq_stats = []
    for s, b in zip(solvers, srcs):
        for k in range(b.shape[0]):
            _, sk = s.solve(b[k].contiguous(), tol=1e-10)
            seq_stats.append(sk)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    print(f"# one at a time: {t_seq:.3f} s", file=sys.stderr, flush=True)
    out = {
        "mode": "batch", "metric": "time-to-1e-10 residual (s), 48 sources on 4 fields", "prec": args.prec,
        "fields": [dict(lattice=list(L), eps=eps, seed=seed, sources=12) for L, eps, seed in BATCH_FIELDS],
        "kappa": kappa, "block": list(B), "subblock": list(S), "autotune_s": tune_s,
        "batch_sources_per_workgroup": nr, "batch_inner_iterations_per_replay": k_inner,
        "autotune_batch_s": tune_batch_s,
        "autotune_batch_candidates": [dict(sources_per_workgroup=c[0], inner_iterations_per_replay=c[1],
                                           median_s_to_1e6=c[2]) for c in tune_rec.get("candidates", [])],
        "batched_s": t_batch, "one_at_a_time_s": t_seq, "speedup": t_seq / t_batch,
        "batched_max_true_relres": max(x["true_relres"] for x in st),
        "batched_outer_its_max": max(x["outer_its"] for x in st),
        "batched_inner_its_total": sum(x["inner_its"] for x in st),
        "one_at_a_time_max_true_relres": max(x["true_relres"] for x in seq_stats),
    }
    # error against the FP64 oracle's 1e-12 solve for one source per field (spin 0, colour 0);
    # the other 11 are the same arithmetic on other sources and are checked by their residuals
    import oracle

    acc = []
    for (L, U, F), x in zip(host_fields, xs):
        b0 = synth.point_source(L, 0, 0)
        x0 = x[0].cpu().numpy()
        xo, ok, t_or = oracle_solve_chunked(L, B, S, U, F, kappa, b0, 1e-12, "x".join(map(str, L)))
        acc.append(dict(lattice=list(L), err_vs_oracle=float(np.linalg.norm(x0 - xo) / np.linalg.norm(xo)),
                        true_relres_oracle_D=float(np.linalg.norm(b0 - oracle.dslash(L, U, F, kappa, x0))
                                                   / np.linalg.norm(b0)),
                        oracle_converged=bool(ok), oracle_s=t_or))
        print(f"# oracle check {acc[-1]}", file=sys.stderr, flush=True)
    out["accuracy_source0_per_field"] = acc
    out["oracle_threads"] = omp_threads()
    print(json.dumps(out), flush=True)


def nn_study(args):
    """The learned-preconditioner workload: the network is trained on the GPU on 2000
    residual->error pairs from the plain SAP solver on four 16^3x32 fields (eps 0.25, seeds
    21-24), then 12 spin-colour point sources are solved at 48^3x96 (seed 31), kappa 0.125, 4^4
    blocks with the autotuned sub-block shape, with plain SAP and with the learned stage ahead
    of SAP, each with FP32 and FP16 storage inside an FP64 outer iteration.  Prints one JSON
    line."""
    import torch

    from paper_1210_7398_amd import sapq, synth, train_nn

    kappa, B = 0.125, (4, 4, 4, 4)
    dev = torch.device("cuda:0")
    Lt = (16, 16, 16, 32)
    n_src = int(os.environ.get("SAPQ_NN_SOURCES_PER_FIELD", "100"))
    steps = int(os.environ.get("SAPQ_NN_STEPS", "600"))
    # the sub-block shape (or the even-odd site order) that the autotuner picks on the first
    # training field serves the training pairs and every application below
    U = synth.gauge_field(Lt, 0.25, 21, device=dev)
    tuner = sapq.Solver(Lt, B, (2, 2, 2, 2), kappa, device=dev)
    tuner.load_gauge(U)
    tuner.load_clover(synth.clover_inverse(Lt, U, 1.0, kappa, device=dev))
    S = tuner.autotune()
    tuner.close()
    print(f"# autotuned sub-block {S}", file=sys.stderr, flush=True)
    t0 = time.time()
    sets = []
    for seed in (21, 22, 23, 24):
        U = synth.gauge_field(Lt, 0.25, seed, device=dev)
        F = synth.clover_inverse(Lt, U, 1.0, kappa, device=dev)
        s = sapq.Solver(Lt, B, S, kappa, nn=True, device=dev)
        s.load_gauge(U)
        s.load_clover(F)
        srcs = [torch.from_numpy(synth.gaussian_spinor(Lt, 100 * seed + k)).to(dev) for k in range(n_src)]
        sets.append((s, train_nn.make_pairs(s, srcs, n_iter=5)))
        print(f"# training field {seed}: {sets[-1][1].shape[0]} pairs after {time.time() - t0:.1f} s",
              file=sys.stderr, flush=True)
    gen_s = time.time() - t0
    w0 = train_nn.init_weights(0, device=dev)
    for s, _ in sets:
        s.nn_set_weights(w0)
    t0 = time.time()
    losses = train_nn.train(sets, steps=steps, batch=8, lr=2e-3, log=100)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    w = sets[-1][0].nn_get_weights().clone()
    for s, e in sets:
        s.close()
    del sets
    torch.cuda.empty_cache()
    print(f"# trained {steps} steps in {train_s:.1f} s, loss {losses[0]:.3f} -> {np.mean(losses[-20:]):.3f}",
          file=sys.stderr, flush=True)

    La = (48, 48, 48, 96)
    t0 = time.time()
    U = synth.gauge_field(La, 0.25, 31, device=dev)
    F = synth.clover_inverse(La, U, 1.0, kappa, device=dev)
    torch.cuda.synchronize()
    print(f"# 48^3x96 field in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    V = synth.volume(La)
    n_apply = int(os.environ.get("SAPQ_NN_APPLY_SOURCES", "12"))
    results = []
    for prec in ("fp32", "fp16"):
        s = sapq.Solver(La, B, S, kappa, prec=prec, nn=True, device=dev)
        s.load_gauge(U)
        s.load_clover(F)
        s.nn_set_weights(w)
        for use in (False, True):
            s.use_nn(use)
            tot, its, msap, worst = 0.0, 0, 0, 0.0
            for k in range(n_apply):
                b = torch.zeros((V, 4, 3), dtype=torch.complex128, device=dev)
                b[0, k % 4, k // 4 % 3] = 1.0
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                x, st = s.solve(b, tol=1e-10)
                torch.cuda.synchronize()
                tot += time.perf_counter() - t1
                its += st["inner_its"]
                msap += st["n_msap"]
                worst = max(worst, st["true_relres"])
                del x
            results.append(dict(prec=prec, learned_stage=use, sources=n_apply, time_s=tot, inner_its=its,
                                n_msap=msap, max_true_relres=worst))
            print(f"# {results[-1]}", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    # the same sources through the batched solver, in sub-batches of 6 (FP64 defect correction)
    sub = int(os.environ.get("SAPQ_NN_SUB_BATCH", "6"))
    batched = []
    for prec in ("fp32", "fp16"):
        s = sapq.Solver(La, B, S, kappa, prec=prec, outer="defect", nn=True, device=dev)
        s.load_gauge(U)
        s.load_clover(F)
        s.nn_set_weights(w)
        for use in (False, True):
            s.use_nn(use)
            # one untimed batched solve first (the work memory is allocated on the first call)
            bb = point_sources(V, list(range(min(sub, n_apply))), dev)
            sapq.solve_batch([s], [bb], tol=1e-10)
            del bb
            tot, its, worst = 0.0, 0, 0.0
            for k0 in range(0, n_apply, sub):
                ks = list(range(k0, min(k0 + sub, n_apply)))
                bb = torch.zeros((len(ks), V, 4, 3), dtype=torch.complex128, device=dev)
                for j, k in enumerate(ks):
                    bb[j, 0, k % 4, k // 4 % 3] = 1.0
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                xs, sts = sapq.solve_batch([s], [bb], tol=1e-10)
                torch.cuda.synchronize()
                tot += time.perf_counter() - t1
                its += sum(q["inner_its"] for q in sts)
                worst = max(worst, max(q["true_relres"] for q in sts))
                del xs, bb
                torch.cuda.empty_cache()
            batched.append(dict(prec=prec, learned_stage=use, sources=n_apply, sub_batch=sub, time_s=tot,
                                inner_its=its, max_true_relres=worst))
            print(f"# batched {batched[-1]}", file=sys.stderr, flush=True)
        s.close()
        del s
        # the batched solver keeps its work memory between calls: hand it back before the next
        # precision's batch sizes its own
        sapq.release_batch_arena()
        torch.cuda.empty_cache()
    base = results[0]["time_s"]
    for r in results + batched:
        r["speedup_vs_plain_fp32"] = base / r["time_s"]
    print(json.dumps({"mode": "nn", "metric": "time-to-1e-10 residual (s); learned stage + mixed precision vs plain SAP",
                      "train": dict(lattice=list(Lt), fields=[21, 22, 23, 24], pairs=4 * n_src * 5, steps=steps,
                                    batch=8, lr=2e-3, pair_generation_s=gen_s, train_s=train_s,
                                    loss_first=losses[0], loss_last20=float(np.mean(losses[-20:]))),
                      "apply": dict(lattice=list(La), seed=31, kappa=kappa, block=list(B), subblock=list(S)),
                      "results": results, "batched": batched}), flush=True)


def point_sources(V, ks, dev):
    """Spin-colour point sources at the origin, source k = (spin k % 4, colour k // 4 % 3)."""
    import torch

    bb = torch.zeros((len(ks), V, 4, 3), dtype=torch.complex128, device=dev)
    for j, k in enumerate(ks):
        bb[j, 0, k % 4, k // 4 % 3] = 1.0
    return bb


def learned_stage_headline(args):
    """The learned-preconditioner workload, as the default bench line's "learned_stage" object:
    the network is trained on the GPU on 2000 residual -> error pairs of the plain SAP solver on
    four 16^3x32 fields (eps 0.25, seeds 21-24), then the 12 spin-colour point sources of a
    48^3x96 field (seed 31) are solved to 1e-10, kappa 0.125, 4^4 blocks with the autotuned
    ordering: plain FP32 SAP one source at a time (the reference) against the NN-augmented FP16
    batched solver (sub-batches of 6), with plain FP16 batched beside them.  Every solution's
    true residual is checked with the oracle's FP64 D on the host; the error against the oracle
    is stated on the training lattice, where the oracle's solve is feasible."""
    import torch

    import oracle
    from paper_1210_7398_amd import sapq, synth, train_nn

    kappa, B, tol = 0.125, (4, 4, 4, 4), 1e-10
    dev = torch.device("cuda:0")
    Lt, La = (16, 16, 16, 32), (48, 48, 48, 96)
    n_src, steps, sub = 100, args.nn_train_steps, 6
    t_all = time.time()
    U = synth.gauge_field(Lt, 0.25, 21, device=dev)
    F = synth.clover_inverse(Lt, U, 1.0, kappa, device=dev)
    tuner = sapq.Solver(Lt, B, (2, 2, 2, 2), kappa, device=dev)
    tuner.load_gauge(U)
    tuner.load_clover(F)
    t0 = time.time()
    S = tuner.autotune()
    tune_s = time.time() - t0
    tuner.close()
    # the error statement on the training lattice: a Gaussian source on field 21, plain FP32
    s = sapq.Solver(Lt, B, S, kappa, device=dev)
    s.load_gauge(U)
    s.load_clover(F)
    bt = synth.gaussian_spinor(Lt, 2101)
    xt, _ = s.solve(torch.from_numpy(bt).to(dev), tol=tol)
    s.close()
    Uh, Fh = U.cpu().numpy(), F.cpu().numpy()
    xo, sto, _ = oracle.solve(Lt, B, S, Uh, Fh, oracle.params(kappa, tol_inner=0.1), bt, tol=1e-12)
    xt = xt.cpu().numpy()
    train_lattice = dict(lattice=list(Lt), err_vs_oracle=float(np.linalg.norm(xt - xo) / np.linalg.norm(xo)),
                         true_relres_oracle_D=float(np.linalg.norm(bt - oracle.dslash(Lt, Uh, Fh, kappa, xt))
                                                    / np.linalg.norm(bt)))
    del Uh, Fh
    print(f"# learned stage: sub-block {S}; training-lattice check {train_lattice}", file=sys.stderr, flush=True)
    t0 = time.time()
    sets = []
    for seed in (21, 22, 23, 24):
        U = synth.gauge_field(Lt, 0.25, seed, device=dev)
        F = synth.clover_inverse(Lt, U, 1.0, kappa, device=dev)
        s = sapq.Solver(Lt, B, S, kappa, nn=True, device=dev)
        s.load_gauge(U)
        s.load_clover(F)
        srcs = [torch.from_numpy(synth.gaussian_spinor(Lt, 100 * seed + k)).to(dev) for k in range(n_src)]
        sets.append((s, train_nn.make_pairs(s, srcs, n_iter=5)))
    pairs_s = time.time() - t0
    w0 = train_nn.init_weights(0, device=dev)
    for s, _ in sets:
        s.nn_set_weights(w0)
    t0 = time.time()
    losses = train_nn.train(sets, steps=steps, batch=8, lr=2e-3, log=100)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    w = sets[-1][0].nn_get_weights().clone()
    for s, _ in sets:
        s.close()
    del sets
    torch.cuda.empty_cache()
    print(f"# trained {steps} steps in {train_s:.1f} s (pairs {pairs_s:.1f} s), loss {losses[0]:.3f} -> "
          f"{np.mean(losses[-20:]):.3f}", file=sys.stderr, flush=True)

    U = synth.gauge_field(La, 0.25, 31, device=dev)
    F = synth.clover_inverse(La, U, 1.0, kappa, device=dev)
    V = synth.volume(La)
    Uh, Fh = U.cpu().numpy(), F.cpu().numpy()
    ks = list(range(12))
    bh = point_sources(V, ks, "cpu").numpy()

    def oracle_check(xs):
        return max(float(np.linalg.norm(bh[j] - oracle.dslash(La, Uh, Fh, kappa, xs[j])) / np.linalg.norm(bh[j]))
                   for j in range(len(xs)))

    res = {}
    # reference: plain FP32 SAP, one source at a time, FP64 flexible BiCGStab
    s = sapq.Solver(La, B, S, kappa, prec="fp32", device=dev)
    s.load_gauge(U)
    s.load_clover(F)
    tot, msap, its, xs = 0.0, 0, 0, []
    for k in ks:
        bk = point_sources(V, [k], dev)[0]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, st = s.solve(bk, tol=tol)
        torch.cuda.synchronize()
        tot += time.perf_counter() - t1
        msap += st["n_msap"]
        its += st["inner_its"]
        xs.append(x.cpu().numpy())
        del x, bk
    s.close()
    del s
    torch.cuda.empty_cache()
    res["plain_fp32_one_at_a_time"] = dict(time_s=tot, n_msap=msap, inner_its=its,
                                           max_true_relres_oracle_D=oracle_check(xs))
    print(f"# plain fp32: {res['plain_fp32_one_at_a_time']}", file=sys.stderr, flush=True)
    del xs
    # batched FP16 storage, FP64 defect correction, with and without the learned stage
    for key, use in (("nn_fp16_batched", True), ("plain_fp16_batched", False)):
        s = sapq.Solver(La, B, S, kappa, prec="fp16", outer="defect", nn=True, device=dev)
        s.load_gauge(U)
        s.load_clover(F)
        s.nn_set_weights(w)
        s.use_nn(use)
        # one untimed batched solve first: the batched solver's work memory is allocated on its
        # first call (the one-source solver's arena is allocated with the solver, untimed too)
        bb = point_sources(V, ks[:sub], dev)
        sapq.solve_batch([s], [bb], tol=tol)
        del bb
        tot, its, xs = 0.0, 0, []
        for k0 in range(0, len(ks), sub):
            bb = point_sources(V, ks[k0 : k0 + sub], dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            xb, sts = sapq.solve_batch([s], [bb], tol=tol)
            torch.cuda.synchronize()
            tot += time.perf_counter() - t1
            its += sum(q["inner_its"] for q in sts)
            xs.extend(list(xb[0].cpu().numpy()))
            del xb, bb
        s.close()
        del s
        sapq.release_batch_arena()
        torch.cuda.empty_cache()
        res[key] = dict(time_s=tot, inner_its=its, sub_batch=sub, max_true_relres_oracle_D=oracle_check(xs))
        print(f"# {key}: {res[key]}", file=sys.stderr, flush=True)
        del xs
    base = res["plain_fp32_one_at_a_time"]["time_s"]
    return {
        "metric": "time-to-1e-10 residual (s) of 12 point sources; NN + FP16 batched vs plain FP32 SAP",
        "workload": (f"48^3x96 clover-Wilson field (eps 0.25, seed 31), kappa 0.125, c_SW 1.0, SAP blocks 4^4, "
                     f"sub-block {list(S)} (autotuned; 0 = even-odd site order), SSOR x4, N_SAP 4, 12 spin-colour "
                     "point sources, tol 1e-10; network 1->8->8->1 parallel-transport layers, BF16 MFMA, trained "
                     f"on the GPU: {steps} Adam steps on {4 * n_src * 5} pairs of four 16^3x32 fields"),
        "plain_fp32_s": base,
        "nn_fp16_batched_s": res["nn_fp16_batched"]["time_s"],
        "speedup_nn_fp16_batched_vs_plain_fp32": base / res["nn_fp16_batched"]["time_s"],
        "plain_fp16_batched_s": res["plain_fp16_batched"]["time_s"],
        "speedup_plain_fp16_batched_vs_plain_fp32": base / res["plain_fp16_batched"]["time_s"],
        "results": res,
        "train": dict(pair_generation_s=pairs_s, train_s=train_s, steps=steps, loss_first=losses[0],
                      loss_last20=float(np.mean(losses[-20:])), autotune_s=tune_s),
        "training_lattice_accuracy": train_lattice,
        "wall_s": time.time() - t_all,
    }


def nn_apply_study(args):
    """The cost of the learned stage inside the inner preconditioner at 48^3x96 (the learned-stage
    workload's application lattice, 4^4 blocks in the even-odd site order the autotuner picks
    there, FP16 storage): one application of P = N + M_SAP (1 - D N) against one of M_SAP
    alone (sapq_precondition), each timed with CUDA events over 5 applications after one
    warm-up.  The weights are the training's starting point (the time does not depend on them).
    Prints one JSON line; run under rocprofv3 --kernel-trace for the per-layer times."""
    import torch

    from paper_1210_7398_amd import sapq, synth, train_nn

    kappa, B, S, La = 0.125, (4, 4, 4, 4), (0, 0, 0, 0), (48, 48, 48, 96)
    dev = torch.device("cuda:0")
    U = synth.gauge_field(La, 0.25, 31, device=dev)
    F = synth.clover_inverse(La, U, 1.0, kappa, device=dev)
    res = {}
    for prec in ("fp16", "fp32"):
        s = sapq.Solver(La, B, S, kappa, prec=prec, nn=True, device=dev)
        s.load_gauge(U)
        s.load_clover(F)
        s.nn_set_weights(train_nn.init_weights(0, device=dev))
        r = torch.from_numpy(synth.gaussian_spinor(La, 3101)).to(dev)
        for use in (True, False):
            s.use_nn(use)
            s.precondition(r)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(5):
                s.precondition(r)
            e1.record()
            torch.cuda.synchronize()
            key = f"{prec}_{'stage_and_msap' if use else 'msap'}_ms"
            res[key] = e0.elapsed_time(e1) / 5
            print(f"# {key}: {res[key]:.2f}", file=sys.stderr, flush=True)
        s.close()
        del s
        torch.cuda.empty_cache()
    for prec in ("fp16", "fp32"):
        res[f"{prec}_stage_ms"] = res[f"{prec}_stage_and_msap_ms"] - res[f"{prec}_msap_ms"]
        res[f"{prec}_stage_over_msap"] = res[f"{prec}_stage_ms"] / res[f"{prec}_msap_ms"]
    print(json.dumps({"mode": "nn_apply", "lattice": list(La), "block": list(B), "subblock": list(S), **res}), flush=True)


def phase_model(B, n_ssor, prec_bytes):
    """Algorithmic bytes and flops per site of one SAP phase kernel launch (a cycle after the
    first: it gathers the other colour and accumulates y).  Each operand is counted once."""
    face = sum(2.0 / b for b in B)            # hops per site that leave the block
    inner = 8.0 - face                         # hops per site that stay inside it
    S = prec_bytes
    bytes_ = S * (24 + 24 * face + 48 + 12 * face / 2 + 72 + 24 * 3 + 24)
    gather = face * HOP_FLOPS + CLOVER_FLOPS + AXPY_FLOPS
    sweep = inner * HOP_FLOPS + CLOVER_FLOPS + AXPY_FLOPS
    first = 0.5 * inner * HOP_FLOPS + CLOVER_FLOPS + AXPY_FLOPS   # from x = 0 only lower neighbours count
    ssor = (2 * n_ssor - 1) * sweep + first
    final = sweep + 24 + 24
    return bytes_, gather + ssor + final


def phase_stream_model(B, n_ssor, prec_bytes):
    """Bytes per site of one phase launch when the block's links, clover field and v cannot stay
    on chip between sweeps (6^3x12 blocks: one colour's fields exceed the chip's LDS and
    registers): the operands-once bytes plus one re-read of U (4 x 12 reals), F (72 reals) and
    v (24 reals) per sweep, 2 n_ssor sweeps."""
    once, _ = phase_model(B, n_ssor, prec_bytes)
    return once + 2 * n_ssor * prec_bytes * (48 + 72 + 24)


def dslash_model(prec_bytes):
    S = prec_bytes
    return S * (24 + 48 + 72 + 24), 8 * HOP_FLOPS + CLOVER_FLOPS + AXPY_FLOPS


# the sources the SAP phase kernel (k_sap_phase_parts) is built from: its file and the headers
# it includes (counters taken on other sources no longer describe it)
PHASE_KERNEL_SOURCES = ("sap_parts.hip", "twolane.h", "sitecore.h", "sapq_impl.h", "tables.h")


def csrc_sha256(names=PHASE_KERNEL_SOURCES):
    """Hash of the named library sources (in the given order)."""
    d = os.path.join(ROOT, "paper_1210_7398_amd", "csrc")
    h = hashlib.sha256()
    for name in names:
        h.update(name.encode())
        h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def traffic_from_profiles(kernel_name, workload):
    """HBM bytes per launch measured by rocprofv3 counters, if they were taken on the current
    sources and this workload (profiles/counters.json records both)."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        if data.get("csrc_sha256") != csrc_sha256() or data.get("workload") != workload:
            return None
        k = data["kernels"].get(kernel_name)
        return None if k is None else k.get("bytes_per_launch")
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="24^3x48", choices=list(WORKLOADS))
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned-stage", dest="learned_stage", action="store_false",
                    help="leave out the learned-stage headline object (48^3x96, 12 sources)")
    ap.add_argument("--nn-train-steps", type=int, default=300)
    ap.add_argument("--mode", default="solve", choices=["solve", "copy", "precision", "batch", "nn", "blocks",
                                                        "sustained", "nsap", "omega", "nn_apply"])
    ap.add_argument("--outer", default="fbicgstab", choices=["fbicgstab", "defect"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); a domain-decomposed "
              "multi-GPU solver is not built.", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        copy_calibration()
        return
    if args.mode == "precision":
        precision_study(args)
        return
    if args.mode == "batch":
        batch_study(args)
        return
    if args.mode == "nn":
        nn_study(args)
        return
    if args.mode == "blocks":
        blocks_study(args)
        return
    if args.mode == "nsap":
        nsap_study(args)
        return
    if args.mode == "omega":
        omega_study(args)
        return
    if args.mode == "sustained":
        sustained_study(args)
        return
    if args.mode == "nn_apply":
        nn_apply_study(args)
        return

    import numpy as np
    import torch

    from paper_1210_7398_amd import sapq, synth

    w = WORKLOADS[args.workload]
    L, B, S = w["L"], w["B"], w["S"]
    V = int(np.prod(L))
    U, F, b = make_inputs(w)

    dev = torch.device("cuda:0")
    solver = sapq.Solver(L, B, S, w["kappa"], prec=args.prec, outer=args.outer, device=dev)
    solver.load_gauge(torch.from_numpy(U).to(dev))
    solver.load_clover(torch.from_numpy(F).to(dev))
    bd = torch.from_numpy(b).to(dev)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        x, st = solver.solve(bd, tol=1e-10)
        print(f"# warmup {i}: {st['time_s']:.3f} s outer {st['outer_its']} inner {st['inner_its']} "
              f"relres {st['true_relres']:.2e}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        x, st = solver.solve(bd, tol=1e-10, profile=True)
        stats.append(st)
        print(f"# step {i}: {st['time_s']:.3f} s outer {st['outer_its']} inner {st['inner_its']} "
              f"msap {st['n_msap']} relres {st['true_relres']:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    sec_per_solve = elapsed / args.steps
    assert all(s["true_relres"] <= 1e-10 for s in stats), "a timed solve missed the tolerance"

    prec_bytes = 4 if args.prec == "fp32" else 2
    sites_per_phase = V // 2
    ph_bytes, ph_flops = phase_model(B, 4, prec_bytes)
    st_bytes = phase_stream_model(B, 4, prec_bytes) * sites_per_phase
    phase_kernel = solver.phase_kernel
    kname = "k_sap_phase" if phase_kernel == "four-lane" else "k_sap_phase_parts"
    k = {}
    for name in ("phase_E", "phase_O", "face", "dslash64"):
        ms = sum(s["kernels"].get(name, {}).get("ms", 0.0) for s in stats)
        n = sum(s["kernels"].get(name, {}).get("n", 0) for s in stats)
        k[name] = dict(launches=n, avg_us=1e3 * ms / n if n else None, total_ms=ms)
    n_ph = k["phase_E"]["launches"] + k["phase_O"]["launches"]
    avg_ph_s = (k["phase_E"]["total_ms"] + k["phase_O"]["total_ms"]) / n_ph / 1e3
    alg_bytes = ph_bytes * sites_per_phase
    alg_flops = ph_flops * sites_per_phase
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    t_alu = alg_flops / (FP32_PEAK_TFLOPS * 1e12)
    traffic = traffic_from_profiles(kname, args.workload)
    if t_hbm >= t_alu:
        roof = dict(bound="hbm", achieved=alg_bytes / avg_ph_s / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    else:
        roof = dict(bound="alu", achieved=alg_flops / avg_ph_s / 1e12, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic
    roof["kernel"] = kname
    roof["phase_kernel"] = phase_kernel
    roof["avg_launch_us"] = avg_ph_s * 1e6
    roof["alg_bytes_per_launch"] = alg_bytes
    roof["alg_flops_per_launch"] = alg_flops
    # the same launch against the bytes of the implemented form when the block's operands
    # are re-read from HBM on every sweep
    roof["streamed"] = dict(bytes_per_launch=st_bytes, achieved=st_bytes / avg_ph_s / 1e9, unit="GB/s",
                            frac=st_bytes / avg_ph_s / 1e9 / HBM_PEAK_GBS)

    d_bytes, d_flops = dslash_model(8)
    d_avg = k["dslash64"]["avg_us"] * 1e-6 if k["dslash64"]["avg_us"] else None
    kernels = dict(
        sap_phase=dict(avg_us=avg_ph_s * 1e6, launches=n_ph, GBps=alg_bytes / avg_ph_s / 1e9,
                       TFLOPs=alg_flops / avg_ph_s / 1e12),
        dslash_fp64=dict(avg_us=k["dslash64"]["avg_us"], launches=k["dslash64"]["launches"],
                         GBps=(d_bytes * V / d_avg / 1e9) if d_avg else None,
                         frac_hbm=(d_bytes * V / d_avg / 1e9 / HBM_PEAK_GBS) if d_avg else None),
        face=dict(avg_us=k["face"]["avg_us"], launches=k["face"]["launches"]),
    )
    # the operator in the inner storage precision, timed alone (20 launches between HIP events)
    p_in = args.prec
    d_in_bytes, _ = dslash_model(4 if p_in == "fp32" else 2)
    d_us = solver.time_dslash(bd, p_in, 20)
    kernels[f"dslash_{p_in}"] = dict(avg_us=d_us, launches=20, GBps=d_in_bytes * V / (d_us * 1e-6) / 1e9,
                                    frac_hbm=d_in_bytes * V / (d_us * 1e-6) / 1e9 / HBM_PEAK_GBS)

    cpu, accuracy = None, None
    if not args.no_cpu_baseline:
        cpu, accuracy = oracle_reference(w, U, F, b, x.cpu().numpy())
        print(f"# GPU solution vs oracle: {accuracy}", file=sys.stderr, flush=True)

    learned = None
    if args.learned_stage:
        learned = learned_stage_headline(args)

    st0 = stats[-1]
    out = {
        "metric": "time-to-1e-10 residual (s)",
        "value": sec_per_solve,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_solve * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.prec == "fp32" else f"{args.prec}-storage/f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"clover-Wilson solve {args.workload}, kappa {w['kappa']}, c_SW {w['csw']}, "
                         f"SAP blocks {'x'.join(map(str, B))}, sub-blocks {'x'.join(map(str, S))}, "
                         f"SSOR omega 1.0 x4, N_SAP 4, {args.prec} inner BiCGStab, fp64 flexible outer, "
                         "tol 1e-10, 1 Gaussian source"),
            "lattice": list(L), "block": list(B), "subblock": list(S), "kappa": w["kappa"],
            "inner_precision": args.prec, "rhs": 1, "phase_kernel": phase_kernel,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "solver": dict(outer_its=st0["outer_its"], inner_its=st0["inner_its"], n_msap=st0["n_msap"],
                       n_dslash64=st0["n_dslash64"], true_relres=st0["true_relres"]),
        "accuracy": accuracy,
        "kernels": kernels,
        "learned_stage": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
