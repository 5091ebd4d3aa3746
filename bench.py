"""Throughput of the quasi-orthogonal evolution step on one MI355X.

Workload: 3-D unit cube, 96^3 interior grid (Ng = 884,736), 7-point stencil,
Dirichlet, H = -1/2 Lap + V with V = 8 Gaussian wells (seed 0), N = 256
eigenpairs, U0 i.i.d. N(0,1) (seed 1), tau = 0.9 lambda_1 (lambda_1 estimated
on a 32^3 grid of the same potential), PCG tolerance 1e-10, warm starts.
One step = one full pass of the scheme (two inverse-operator solves, two Gram
matrices, the N x N predictor solve, the two block updates and the energy).

value = steps/s of the mixed-precision path (FP32 PCG inside FP64 iterative
refinement, BF16 Gram tiles with FP32 accumulation, FP64 N x N algebra and
energy); the FP64 path is timed beside it.  The inverse operator is applied by
PCG with the fast-Poisson preconditioner (DST-I inverse of kappa(-Lap_h) + vbar
on FP16 matrix cores); the same step with the Jacobi preconditioner is timed
beside it (--jacobi-steps).  The accuracy gate compares the mixed and FP64
Ritz values of the converged pairs after the same number of steps.  The
roofline object describes the dominant streaming kernel of the mixed path,
measured live with HIP events around every launch on the library's stream.
cpu_baseline times the FP64 oracle on a bounded sample of the same workload on
the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "steps/s at 96³,N=256: mixed vs FP64 at 1e-8 eig error; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per (grid point x column) of one launch; s = bytes per value of the
# PCG (8 in FP64, 4 in the mixed path's FP32 iteration); FP16 intermediates are 2 bytes
#   two-sweep form  sweep1: read r, p_old; write p (Jacobi)   -> 3 s
#                           read z (FP32), p_old; write p       -> 2 s + 4 (fast-Poisson,
#                                                                  FP64)
#                           read p (formed by dst_inv)          -> 4 (fast-Poisson, FP32)
#                   sweep2: read p, x, r;  write x, r         -> 5 s
#   one-sweep form  cg:     read r, p_old, x; write r, p, x   -> 6 s
#   fast-Poisson    dst_fwd: read r; write t1 (FP16)          -> s + 2
#                   dst_pencil: read t1, write t2 (FP16)      -> 4
#                   dst_inv: read t2 (FP16); write z (FP32)    -> 6 (FP64 PCG)
#                            read t2, p_old; write p (FP32)    -> 10 (FP32 PCG; the first
#                                                          iteration, without p_old, counts
#                                                          0.6 of a column-iteration)
BYTES_PER_COLPT = {"sweep1_f64": 24, "sweep2_f64": 40, "sweep1_f32": 12, "sweep2_f32": 20,
                   "cg_f64": 48, "cg_f32": 24}
DST_BYTES = {"dst_fwd": lambda s: s + 2, "dst_pencil": lambda s: 4,
             "dst_inv": lambda s: 10 if s == 4 else 6}
KERNEL_SYMBOL = {"sweep1_f64": "k_pcg_sweep1<double>", "sweep2_f64": "k_pcg_sweep2<double>",
                 "sweep1_f32": "k_pcg_sweep1<float>", "sweep2_f32": "k_pcg_sweep2<float>",
                 "cg_f64": "k_cg_step<double>", "cg_f32": "k_cg_step<float>",
                 "dst_pencil": "k_dst_pencil"}


def lambda1_estimate(n_coarse=32, seed=0):
    """Lowest eigenvalue of H on a coarse grid of the same potential (scipy, host)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    from paper_2605_25149_amd import inputs

    n = (n_coarse,) * 3
    V = inputs.gaussian_wells(n, seed=seed)
    h = 1.0 / (n_coarse + 1)
    T = sp.diags([np.full(n_coarse - 1, -1.0), np.full(n_coarse, 2.0),
                  np.full(n_coarse - 1, -1.0)], [-1, 0, 1]) * (0.5 / h**2)
    I = sp.identity(n_coarse)
    H = (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)
         + sp.diags(V)).tocsc()
    vals = spla.eigsh(H, k=1, sigma=0.0, which="LM", return_eigenvectors=False)
    return float(vals[0])


def make_solver(precision, n, N, inner_tol, variant, precond):
    from paper_2605_25149_amd import binding

    # the fast-Poisson solve takes ~10 iterations: poll convergence after every one
    check = 1 if precond == "fast_poisson" else 8
    return binding.Solver(3, n, N, pcg_tol=1e-10, pcg_maxit=5000, pcg_check=check,
                          precision=precision, refine_inner_tol=inner_tol, pcg_variant=variant,
                          precond=precond)


def run_gpu(precision, V, U0, n, N, tau, steps, warmup, inner_tol, log, variant=0,
            precond="fast_poisson", dim_n=None):
    """Two passes over the same trajectory from U0 (same warm-up): first with HIP events
    around every launch (per-kernel times for the roofline), then the timed pass with no
    events; `seconds` is the second pass's wall time over the timed steps."""
    import torch

    s = make_solver(precision, n, N, inner_tol, variant, precond)
    out = {}
    try:
        s.set_potential(V)
        for timed in (False, True):
            tag = f"{precision} {precond}" + ("" if timed else " profiled")
            s.set_state(U0)
            for i in range(warmup):
                st = s.step(tau)
                log(f"[{tag}] warmup step {i + 1}/{warmup}: iters {st['pcg_iters']} "
                    f"rounds {st['refine_rounds']} E {st['energy']:.10f}")
            s.profile(not timed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            stats = []
            for i in range(steps):
                st = s.step(tau)
                stats.append(st)
                log(f"[{tag}] step {i + 1}/{steps}: iters {st['pcg_iters']} "
                    f"rounds {st['refine_rounds']} E {st['energy']:.10f} "
                    f"phases(ms) {[round(x, 1) for x in st['t_phase_ms']]}")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if timed:
                out.update(seconds=t1 - t0, stats=stats)
            else:
                out.update(profile=s.profile_data(), profiled_seconds=t1 - t0)
                s.profile(False)
        return out
    finally:
        s.close()


def kernel_rates(prof, ng, value_bytes):
    """Achieved GB/s of every streaming kernel of a run (algorithmic bytes / time)."""
    bpc = bytes_per_colpt(prof, value_bytes)
    out = {}
    for k, b in bpc.items():
        d = prof[k]
        if d["launches"] and d["ms"] > 0:
            gbs = b * ng * d["work"] / (d["ms"] * 1e-3) / 1e9
            out[k] = {"GB/s": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
                      "bytes_per_point_column": b}
    return out


def run_jacobi_fp64_leg(V64, U064, tau, steps, warmup, log, n=64, N=64):
    """The FP64 Jacobi configuration: 64^3 Gaussian wells, N = 64, Jacobi PCG at tol 1e-10
    (polled every 8 iterations), warm starts: steps/s and per-kernel GB/s."""
    from paper_2605_25149_amd import binding

    grid = (n, n, n)
    r = run_gpu("fp64", V64, binding.as_block(U064), grid, N, tau, steps, warmup, 1e-5, log,
                0, "jacobi")
    ng = n ** 3
    return {
        "workload": f"3-D {n}^3 Dirichlet 7-point grid, 8 Gaussian wells (seed 0), N={N}, "
                    f"random U0 (seed 1), tau={tau:.5f}, Jacobi PCG tol 1e-10, warm starts, FP64",
        "steps": steps, "warmup": warmup,
        "steps_per_s": round(steps / r["seconds"], 4),
        "ms_per_step": round(1e3 * r["seconds"] / steps, 2),
        "pcg_iters_per_step": [st["pcg_iters"] for st in r["stats"]],
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3), "work": v["work"]}
                    for k, v in r["profile"].items() if v["launches"]},
        "kernel_rates": kernel_rates(r["profile"], ng, 8),
    }


def accuracy_gate(V, U0, n, N, tau, K, inner_tol, variant, log, res_tol=1e-5,
                  precond="fast_poisson"):
    """Mixed vs FP64 after the same K-step trajectory: Ritz values of the pairs that the FP64
    run has converged (relative residual ||H u - theta u|| / (|theta| ||u||) <= res_tol)."""
    import torch

    from paper_2605_25149_amd import binding

    out = {}
    for mode in ("fp64", "mixed"):
        s = make_solver(mode, n, N, inner_tol, variant, precond)
        try:
            s.set_potential(V)
            s.set_state(U0)
            t0 = time.perf_counter()
            for i in range(K):
                st = s.step(tau)
                if i % 10 == 0 or i == K - 1:
                    log(f"[accuracy {mode}] step {i + 1}/{K}: iters {st['pcg_iters']} "
                        f"grad {st['grad_norm']:.3e} |O| {st['orth_err_fro']:.3e} "
                        f"E {st['energy']:.12f} ({time.perf_counter() - t0:.1f} s)")
            lam, vec = s.eigenpairs("ritz", vectors=True)
            Hv = s.apply(vec)
            theta = torch.as_tensor(lam, device=vec.device) + s.cfg.sigma
            res = torch.linalg.norm(Hv - theta[:, None] * vec, dim=1) / (
                theta.abs() * torch.linalg.norm(vec, dim=1))
            out[mode] = (np.asarray(lam), res.cpu().numpy(), st)
        finally:
            s.close()
    lam64, res64, st64 = out["fp64"]
    lamm, resm, stm = out["mixed"]
    conv = res64 <= res_tol
    rel = np.abs(lamm - lam64) / np.abs(lam64)
    m = int(conv.sum())
    return {
        "steps": K,
        "converged_pairs": m,
        "pairs": int(len(lam64)),
        "coverage": (f"the 1e-8 gate covers the {m} of {len(lam64)} pairs that the FP64 run has "
                     f"converged (relative residual <= {res_tol:g}) after {K} steps; the others "
                     "are still moving along the trajectory (max_rel_eig_diff_all)"),
        "residual_tol": res_tol,
        "max_rel_eig_diff_converged": float(rel[conv].max()) if m else None,
        "max_rel_eig_diff_all": float(rel.max()),
        "gate_1e-8": bool(m > 0 and rel[conv].max() <= 1e-8),
        "lambda_fp64_first8": [float(x) for x in lam64[:8]],
        "grad_norm_end": {"fp64": st64["grad_norm"], "mixed": stm["grad_norm"]},
    }


def profile_traffic_ratios():
    """traffic_ratio lines of the committed rocprofv3 summaries, kept only while the kernel
    source they were measured on is unchanged (sha256 recorded beside them)."""
    import glob
    import hashlib

    ratios = {}
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        ok, found = True, {}
        for line in open(path, encoding="utf-8"):
            parts = line.split()
            if len(parts) == 3 and parts[0] == "source_sha256":
                src = os.path.join(ROOT, parts[1])
                cur = (hashlib.sha256(open(src, "rb").read()).hexdigest()
                       if os.path.exists(src) else None)
                ok = ok and cur == parts[2]
            elif len(parts) == 3 and parts[0] == "traffic_ratio":
                found[parts[1]] = float(parts[2])
        if ok:
            ratios.update(found)
    return ratios


def bytes_per_colpt(prof, value_bytes):
    out = dict(BYTES_PER_COLPT)
    dst = prof.get("dst_inv", {}).get("launches", 0) > 0
    for k, f in DST_BYTES.items():
        out[k] = f(value_bytes)
    if dst:  # the first sweep reads z (FP64 PCG) or only the finished p (FP32 PCG)
        out["sweep1_f64"] = 2 * 8 + 4
        out["sweep1_f32"] = 4
    return {k: v for k, v in out.items() if k in prof}


def roofline_of(prof, ng, value_bytes):
    """Dominant streaming kernel (PCG sweeps and preconditioner passes, by total time):
    algorithmic bytes per launch / mean launch duration."""
    bpc = bytes_per_colpt(prof, value_bytes)
    best = None
    for k in bpc:
        d = prof[k]
        if d["launches"] == 0 or d["ms"] <= 0:
            continue
        if best is None or d["ms"] > prof[best]["ms"]:
            best = k
    if best is None:
        return None
    d = prof[best]
    bytes_total = bpc[best] * ng * d["work"]
    per_launch_bytes = bytes_total / d["launches"]
    mean_ms = d["ms"] / d["launches"]
    achieved = per_launch_bytes / (mean_ms * 1e-3) / 1e9
    sym = KERNEL_SYMBOL.get(best) or {
        "dst_fwd": "k_dst_plane<%s,false>" % ("float" if value_bytes == 4 else "double"),
        "dst_inv": "k_dst_plane<float,true>"}[best]
    return {
        "kernel": sym,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "traffic_ratio": None,
        "launches": d["launches"],
        "mean_launch_ms": round(mean_ms, 4),
        "algorithmic_bytes_per_launch": round(per_launch_bytes),
    }


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(V, U0, n, N, tau, colits_per_step, log, precond="fast_poisson",
                 jacobi_leg=None):
    """FP64 oracle on the host cores.

    value: the metric's configuration (96^3, N = 256), EXTRAPOLATED from a bounded sample:
    (a) the oracle's PCG (same preconditioner as the GPU run) on a subset of the columns
    for a fixed number of iterations, giving its column-iteration rate (also taken with
    one thread); (b) one pass of the oracle's non-PCG stages (Grams, the 2N x 2N predictor
    solve and the block update, the corrector, the energy) on full-size blocks.
    Steps/s = 1 / (column-iterations per step / rate + time of (b)), column-iterations per
    step from the FP64 GPU run (same algorithm and stop rule).
    Measured in full beside it: the 2-D 32^2, N = 4 trajectory of 200 steps, and one step
    of the 64^3, N = 64 FP64 Jacobi configuration (the GPU leg of the same configuration
    gives the ratio at equal work).  threads: the OpenMP threads of the oracle's C loops;
    its transforms (scipy) run on one thread."""
    from oracle import oracle as orc

    from paper_2605_25149_amd import inputs

    nthreads = orc.threads()
    prob = orc.Problem(3, n, V)
    Uf = np.asfortranarray(U0)

    def pcg_sample(threads):
        orc.threads(threads)
        if precond == "fast_poisson":
            # the oracle's transforms run column by column: a subset of the columns
            ncs = min(N, int(os.environ.get("QO_CPU_COLS", "32")))
            kit = int(os.environ.get("QO_CPU_PCG_ITERS", "2"))
            t0 = time.perf_counter()
            prob.solve_fast_poisson(np.asfortranarray(Uf[:, :ncs]), tol=1e-30, maxit=kit)
        else:
            ncs = N
            kit = int(os.environ.get("QO_CPU_PCG_ITERS", "6"))
            t0 = time.perf_counter()
            prob.solve(Uf, tol=1e-30, maxit=kit)
        return ncs, kit, time.perf_counter() - t0

    ncs, kit, t_pcg = pcg_sample(nthreads)
    rate = ncs * kit / t_pcg
    log(f"[cpu] oracle {precond} PCG {ncs} columns x {kit} iterations: {t_pcg:.2f} s "
        f"({rate:.1f} column-iterations/s, {nthreads} threads)")
    ncs1, kit1, t_pcg1 = pcg_sample(1)
    rate1 = ncs1 * kit1 / t_pcg1
    log(f"[cpu] same sample on 1 thread: {t_pcg1:.2f} s ({rate1:.1f} column-iterations/s)")
    orc.threads(nthreads)
    P = np.asfortranarray(0.1 * Uf)
    t0 = time.perf_counter()
    Uh, Xm, Ym, _ = orc.predictor(prob, Uf, P, tau)
    Unext, _, _, _ = orc.corrector(prob, Uh, P, tau)
    prob.energy(Unext)
    t_rest = time.perf_counter() - t0
    log(f"[cpu] oracle non-PCG stages: {t_rest:.2f} s")
    sec_per_step = colits_per_step / rate + t_rest
    sec_per_step1 = colits_per_step / rate1 + t_rest
    # full runs beside the extrapolation
    n1 = (32, 32)
    p1 = orc.Problem(2, n1, inputs.harmonic(n1, 100.0))
    o1 = orc.Oracle(p1, inputs.random_block(1024, 4, seed=1), tol=1e-12, variant=0)
    t0 = time.perf_counter()
    for _ in range(200):
        o1.step(0.9 * 12.9544687)
    t_cfg1 = time.perf_counter() - t0
    log(f"[cpu] oracle 2-D 32^2 N=4, 200 steps (Jacobi, tol 1e-12): {t_cfg1:.2f} s")
    n2 = (64, 64, 64)
    p2 = orc.Problem(3, n2, inputs.gaussian_wells(n2, seed=0))
    o2 = orc.Oracle(p2, inputs.random_block(64 ** 3, 64, seed=1), tol=1e-10, variant=0)
    t0 = time.perf_counter()
    st2 = o2.step(tau)
    t_cfg2 = time.perf_counter() - t0
    log(f"[cpu] oracle 64^3 N=64 FP64 Jacobi, one step: {t_cfg2:.2f} s "
        f"(iterations {st2.pcg_iters})")
    out = {
        "value": round(1.0 / sec_per_step, 6),
        "unit": "steps/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": (f"EXTRAPOLATED to 96^3 x {N}: oracle {precond} PCG, {kit} iterations on "
                   f"{ncs} of the {N} columns ({t_pcg:.1f} s) + one pass of the non-PCG stages "
                   f"({t_rest:.1f} s), scaled by {colits_per_step:.0f} column-iterations per "
                   "step; full runs in cfg1_full and cfg2_step"),
        "cpu_model": cpu_model(),
        "threads": nthreads,
        "seconds_per_step": round(sec_per_step, 2),
        "value_1thread": round(1.0 / sec_per_step1, 6),
        "cfg1_full": {"workload": "2-D 32^2, N=4, harmonic, 200 steps, Jacobi tol 1e-12",
                      "seconds": round(t_cfg1, 3), "steps_per_s": round(200 / t_cfg1, 2)},
        "cfg2_step": {"workload": "64^3 wells, N=64, FP64 Jacobi tol 1e-10, first step",
                      "seconds": round(t_cfg2, 3), "steps_per_s": round(1 / t_cfg2, 4),
                      "pcg_iters": list(st2.pcg_iters)},
    }
    if jacobi_leg:
        out["cfg2_gpu_over_cpu"] = round(jacobi_leg["steps_per_s"] * t_cfg2, 1)
    return out


def batch_tau(p, kappa=0.5):
    """0.9 x a lower bound of lambda_1(H_sigma) of a 2-D instance: min(V + sigma) plus kappa
    times the smallest eigenvalue of -Lap_h."""
    mu = sum(4.0 * (m + 1) ** 2 * np.sin(np.pi / (2.0 * (m + 1))) ** 2 for m in p["n"])
    return 0.9 * (float(np.min(p["V"])) + p["sigma"] + kappa * mu)


def run_batch(count, steps, log, precisions=("fp64", "mixed")):
    """Aggregate throughput of `count` independent 2-D problems (sides 64..256, N 8..64)
    stepped as one grouped batch (eager launches and graph replay) against the same
    problems stepped one single-instance handle at a time, per precision (mixed: FP32
    PCG in FP64 refinement with FP64 Grams in the batch; the single-instance mixed path
    also uses BF16 Grams)."""
    import torch

    from paper_2605_25149_amd import binding, inputs

    probs = inputs.batch_instances(count, 0)
    taus = [batch_tau(p) for p in probs]
    out = {"instances": count, "columns": sum(p["N"] for p in probs),
           "sides": sorted(set(p["n"][0] for p in probs)), "precond": "fast_poisson",
           "pcg_tol": 1e-10, "steps": steps}
    for prec in precisions:
        res = {}
        cfgs = [dict(dim=2, n=p["n"], N=p["N"], sigma=p["sigma"], pcg_tol=1e-10, pcg_maxit=30,
                     precond="fast_poisson", precision=prec) for p in probs]
        b = binding.Batch(cfgs)
        try:
            for i, p in enumerate(probs):
                b.set_potential(i, p["V"])
                b.set_state(i, inputs.random_block(p["n"][0] * p["n"][1], p["N"], seed=1000 + i))
            out["tiles"] = {str(p["n"][0]): b.tile(i) for i, p in enumerate(probs)}
            for mode in ("eager", "graph"):
                # warm-up: both P/Q parities, and time for the fixed iteration counts to
                # settle (a change re-captures the graphs); the statistics of the last
                # warm-up step give the counts
                st = b.step(taus, nsteps=4, use_graph=mode == "graph")
                res["max_pcg_iters"] = max(max(x["pcg_iters"]) for x in st)
                res["max_refine_rounds"] = max(max(x["refine_rounds"]) for x in st)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                # no per-step statistics: the host waits only at the end (error checks)
                b.step(taus, nsteps=steps, use_graph=mode == "graph", stats=False)
                dt = time.perf_counter() - t0
                res[f"{mode}_instance_steps_per_s"] = round(count * steps / dt, 2)
                log(f"[batch {prec} {mode}] {count} instances, {steps} steps: "
                    f"{dt / steps * 1e3:.1f} ms/step")
        finally:
            b.close()
        sol = []
        try:
            for i, p in enumerate(probs):
                s = binding.Solver(2, p["n"], p["N"], sigma=p["sigma"], pcg_tol=1e-10,
                                   pcg_check=1, precond="fast_poisson", precision=prec)
                s.set_potential(p["V"])
                s.set_state(binding.as_block(inputs.random_block(p["n"][0] * p["n"][1], p["N"],
                                                                 seed=1000 + i)))
                sol.append(s)
            for i, s in enumerate(sol):
                s.step(taus[i])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                for i, s in enumerate(sol):
                    s.step(taus[i])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res["sequential_instance_steps_per_s"] = round(count * steps / dt, 2)
            log(f"[batch {prec} sequential] {count} single-instance handles: "
                f"{dt / steps * 1e3:.1f} ms/round")
        finally:
            for s in sol:
                s.close()
        res["speedup_vs_sequential"] = round(
            max(res["eager_instance_steps_per_s"], res["graph_instance_steps_per_s"]) /
            res["sequential_instance_steps_per_s"], 3)
        # Step roofline of the batch, an UPPER bound of the achieved HBM rate: every column
        # counted for its instance's largest PCG count in both solves (converged columns are
        # frozen on the device and move nothing), at the algorithmic bytes per point-column
        # of one PCG iteration (FP64: 80; mixed FP32 PCG: 40, plus one FP64 residual pass of
        # 32 per round) and 13 FP64 block streams per step for the rest (Grams, updates,
        # corrector, energy).
        colpts = sum(p["n"][0] * p["n"][1] * p["N"] for p in probs)
        per_it = 80 if prec == "fp64" else 40
        rounds = res["max_refine_rounds"] if prec != "fp64" else 0
        bytes_step = colpts * (2 * res["max_pcg_iters"] * per_it + 2 * rounds * 32 + 13 * 8)
        best = max(res["eager_instance_steps_per_s"], res["graph_instance_steps_per_s"])
        gbs = bytes_step * best / count / 1e9
        res["step_roofline_upper"] = {"bytes_per_step": int(bytes_step), "GB/s": round(gbs, 1),
                                      "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
                                      "point_columns": int(colpts)}
        out[prec] = res
    return out


def run_adjoint(K, log, n=64, N=32, tau=6.0):
    """Reverse mode through K taped steps on the 64^3 Gaussian-well grid with N = 32 (the
    Ritz-sum loss, gradients w.r.t. V and U_0): time of the taped forward, of the backward
    and of K plain (warm-started) steps for scale."""
    import torch

    from paper_2605_25149_amd import binding, inputs

    grid = (n, n, n)
    V = inputs.gaussian_wells(grid, seed=0)
    sigma = max(0.0, 1.0 - float(V.min()))
    U0 = inputs.random_block(n ** 3, N, seed=1)
    out = {"workload": f"{n}^3 wells, N={N}, K={K}, loss=ritz_sum, d/dV and d/dU0",
           "precision": "f64", "precond": "fast_poisson", "pcg_tol": 1e-10}
    with binding.Solver(3, grid, N, sigma=sigma, pcg_tol=1e-10, pcg_check=8,
                        precond="fast_poisson") as s:
        s.set_potential(V)
        for rep in range(2):  # the first pass allocates the tape
            s.set_state(U0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L = s.tape_forward(tau, K, "ritz_sum")
            t1 = time.perf_counter()
            gV, gU = s.tape_backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        s.set_state(U0)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        s.step(tau, K)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        # the same tape bounded to about 2 sqrt(K) + 1 state blocks (checkpoints every s-th
        # state, one segment recomputed during the backward pass): same gradients bit for bit
        budget = int(2 * math.isqrt(K) + 1)
        s.tape_budget(budget)
        for rep in range(2):
            s.set_state(U0)
            torch.cuda.synchronize()
            t5 = time.perf_counter()
            Lb = s.tape_forward(tau, K, "ritz_sum")
            t6 = time.perf_counter()
            gVb, gUb = s.tape_backward()
            torch.cuda.synchronize()
            t7 = time.perf_counter()
        s.tape_budget(0)
    out.update(loss=L, forward_s=round(t1 - t0, 4), backward_s=round(t2 - t1, 4),
               plain_steps_s=round(t4 - t3, 4),
               backward_over_forward=round((t2 - t1) / (t1 - t0), 3),
               grad_V_norm=float(torch.linalg.vector_norm(gV)),
               grad_U0_norm=float(torch.linalg.vector_norm(gU)),
               bounded_tape={"state_blocks": budget, "full_tape_blocks": K + 1,
                             "forward_s": round(t6 - t5, 4), "backward_s": round(t7 - t6, 4),
                             "gradients_bit_identical": bool(Lb == L and torch.equal(gVb, gV)
                                                             and torch.equal(gUb, gU))})
    log(f"[adjoint] {out['workload']}: forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s, "
        f"plain {K} steps {t4 - t3:.3f} s; bounded tape ({budget} blocks): forward "
        f"{t6 - t5:.3f} s, backward {t7 - t6:.3f} s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--inner-tol", type=float, default=1e-5)
    ap.add_argument("--modes", default="fp64,mixed")
    ap.add_argument("--pcg-variant", type=int, default=0,
                    help="0: two-sweep Hestenes-Stiefel PCG, 1: one-sweep Chronopoulos-Gear")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precond", default="fast_poisson", choices=["fast_poisson", "jacobi"])
    ap.add_argument("--jacobi-steps", type=int, default=2,
                    help="also time this many steps (after one warm-up step) with the Jacobi "
                         "preconditioner in each mode (0: skip)")
    ap.add_argument("--accuracy-steps", type=int, default=200,
                    help="mixed-vs-FP64 eigenvalue gate over this many steps (0: skip)")
    ap.add_argument("--batch-instances", type=int, default=128,
                    help="also time a grouped batch of this many 2-D problems (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-precisions", default="fp64,mixed")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batch leg and print its JSON (profiling aid)")
    ap.add_argument("--cfg2-steps", type=int, default=20,
                    help="timed steps of the 64^3, N=64 FP64 Jacobi leg (0 skips it)")
    ap.add_argument("--adjoint-steps", type=int, default=50,
                    help="K of the reverse-mode leg (64^3, N=32); 0 skips it")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not an implementation)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2605_25149_amd import binding, inputs

    binding.load_library()
    torch.cuda.set_device(0)
    if args.batch_only:
        print(json.dumps({"batch": run_batch(args.batch_instances, args.batch_steps, log,
                                             tuple(args.batch_precisions.split(",")))}),
              flush=True)
        return
    n = (args.n,) * 3
    N = args.N
    ng = int(np.prod(n))
    t0 = time.perf_counter()
    V = inputs.gaussian_wells(n, seed=0)
    U0 = inputs.random_block(ng, N, seed=1)
    lam1 = lambda1_estimate(32, seed=0)
    tau = 0.9 * lam1
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s; lambda_1(32^3) = {lam1:.6f}, "
        f"tau = {tau:.6f}")
    U0_dev = binding.as_block(U0)
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one copy kernel")
        del a, b

    res = {}
    for mode in args.modes.split(","):
        res[mode] = run_gpu(mode, V, U0_dev, n, N, tau, args.steps, args.warmup,
                            args.inner_tol, log, args.pcg_variant, args.precond)
        r = res[mode]
        log(f"[{mode}] {args.steps} steps in {r['seconds']:.3f} s -> "
            f"{args.steps / r['seconds']:.4f} steps/s")

    head = "mixed" if "mixed" in res else next(iter(res))
    rh = res[head]
    value = args.steps / rh["seconds"]
    out = {
        "metric": METRIC,
        "value": round(value, 6),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * rh["seconds"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"3-D {args.n}^3 Dirichlet 7-point grid (Ng={ng}), 8 Gaussian wells "
                         f"(seed 0), N={N}, random U0 (seed 1), tau=0.9*lambda_1={tau:.5f}, "
                         f"PCG tol 1e-10 ({args.precond} preconditioner), warm starts; "
                         f"{head} precision"),
            "grid": list(n), "N": N, "tau": tau, "pcg_tol": 1e-10,
            "refine_inner_tol": args.inner_tol, "pcg_variant": args.pcg_variant,
            "precond": args.precond,
            "parallelism": "single GPU",
            **({"precond_arithmetic": "DST-I transforms on FP16 MFMA in both the mixed and the "
                                      "FP64 path; the 1e-10 stop test is on an FP64 residual (the "
                                      "PCG's in the FP64 path, the refinement's true residual in "
                                      "the mixed path)"} if args.precond == "fast_poisson" else {}),
        },
    }
    out["timing"] = ("value and ms_per_step: a pass without per-launch events; the kernel times "
                     "come from a first pass over the same trajectory with HIP events around "
                     "every launch (profiled_steps_per_s)")
    for mode, r in res.items():
        its = [st["pcg_iters"] for st in r["stats"]]
        out[f"{mode}_steps_per_s"] = round(args.steps / r["seconds"], 6)
        out[f"{mode}_profiled_steps_per_s"] = round(args.steps / r["profiled_seconds"], 6)
        out[f"{mode}_pcg_iters_per_step"] = its
        out[f"{mode}_kernels"] = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                                      "work": v["work"]}
                                  for k, v in r["profile"].items() if v["launches"]}
        out[f"{mode}_kernel_rates"] = kernel_rates(r["profile"], ng, 4 if mode == "mixed" else 8)
    if "fp64" in res and "mixed" in res:
        out["speedup_mixed_vs_fp64"] = round(res["fp64"]["seconds"] / res["mixed"]["seconds"], 4)
    vbytes = 4 if head == "mixed" else 8
    rf = roofline_of(rh["profile"], ng, vbytes)
    if rf:
        ratio = profile_traffic_ratios().get(rf["kernel"])
        if ratio is not None:
            rf["traffic"] = round(ratio * rf["algorithmic_bytes_per_launch"])
            rf["traffic_ratio"] = ratio
        out["roofline"] = rf
    if "fp64" in res:
        rf64 = roofline_of(res["fp64"]["profile"], ng, 8)
        if rf64:
            out["roofline_fp64"] = rf64
    if args.accuracy_steps > 0:
        out["accuracy"] = accuracy_gate(V, U0_dev, n, N, tau, args.accuracy_steps,
                                        args.inner_tol, args.pcg_variant, log,
                                        precond=args.precond)
        a = out["accuracy"]
        out["config"]["accuracy_gate"] = (
            f"mixed vs FP64 Ritz values after {a['steps']} steps from the same U0, on the "
            f"{a['converged_pairs']}/{a['pairs']} pairs converged in the FP64 run")
    jleg = None
    if args.cfg2_steps > 0:
        n2 = (64, 64, 64)
        jleg = run_jacobi_fp64_leg(inputs.gaussian_wells(n2, seed=0),
                                   inputs.random_block(64 ** 3, 64, seed=1), tau,
                                   args.cfg2_steps, 2, log)
        out["cfg2"] = jleg
        log(f"[cfg2] 64^3 N=64 FP64 Jacobi: {jleg['steps_per_s']} steps/s")
    if args.jacobi_steps > 0 and args.precond != "jacobi":
        jac = {}
        for mode in args.modes.split(","):
            r = run_gpu(mode, V, U0_dev, n, N, tau, args.jacobi_steps, 1, args.inner_tol, log,
                        args.pcg_variant, "jacobi")
            jac[mode] = {"steps_per_s": round(args.jacobi_steps / r["seconds"], 6),
                         "pcg_iters_per_step": [st["pcg_iters"] for st in r["stats"]]}
        out["jacobi_preconditioner"] = jac
    if args.batch_instances > 0:
        out["batch"] = run_batch(args.batch_instances, args.batch_steps, log,
                                 tuple(args.batch_precisions.split(",")))
    if args.adjoint_steps > 0:
        out["adjoint"] = run_adjoint(args.adjoint_steps, log)
    if not args.no_cpu_baseline:
        ref = res["fp64"] if "fp64" in res else rh
        colits = max(ref["profile"][k]["work"] for k in ("sweep2_f64", "sweep2_f32", "cg_f64", "cg_f32"))
        colits_per_step = colits / args.steps
        out["cpu_baseline"] = cpu_baseline(V, U0, n, N, tau, colits_per_step, log, args.precond,
                                           jleg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
