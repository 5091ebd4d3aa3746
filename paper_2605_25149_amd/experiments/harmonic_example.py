"""Finite-difference analogue of the paper's first numerical example (Sec. 5, Example 1).

The 2-D harmonic oscillator -1/2 Lap u + 1/2 |x|^2 u = lambda u on (-5.5, 5.5)^2 with
N = 15 eigenpairs (the first five shells 1, 2, 3, 4, 5 with multiplicities 1..5), run
with Algorithm 1 of Sec. 5 at a fixed time step until ||grad_G E_G(U_n)|| < 1e-5, from a
random start.  The paper uses quadratic finite elements with Ng = 39,601 unknowns; a
199 x 199 interior FD grid has the same Ng.  For each grid and tau this reports the number
of steps of Algorithm 1 (qo_run), tau * steps (the paper reads a roughly constant value as
a time scale independent of tau and of the mesh), ||<U,U> - I|| after the last step and the
relative errors of the Ritz values against the FD operator's exact eigenvalues (sums of
1-D dense eigenvalues, the operator being separable).

Usage:  python -m paper_2605_25149_amd.experiments.harmonic_example --n 49 99 199 --tau 0.1 0.5
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from paper_2605_25149_amd import binding, inputs

HALF = 5.5


def fd_reference(m, N, half=HALF):
    """Lowest N eigenvalues of the FD operator on m x m interior points (separable)."""
    h = 2 * half / (m + 1)
    x = (np.arange(m) + 1) * h - half
    T = (np.diag(np.full(m, 1.0 / h**2) + 0.5 * x**2)
         + np.diag(np.full(m - 1, -0.5 / h**2), 1) + np.diag(np.full(m - 1, -0.5 / h**2), -1))
    mu = np.linalg.eigvalsh(T)
    return np.sort(np.add.outer(mu, mu).ravel())[: N + 1]


def run(m, tau, N=15, max_steps=40000, seed=1, stop=1e-5, variant=0, log=None,
        precond="jacobi"):
    n = (m, m)
    L = (2 * HALF, 2 * HALF)
    V = inputs.harmonic(n, 1.0, centre=(HALF, HALF), L=L)
    U0 = inputs.random_block(m * m, N, seed=seed) / (2 * HALF)  # E<U0,U0> = I
    lam_ref = fd_reference(m, N)
    t0 = time.perf_counter()
    with binding.Solver(2, n, N, L=L, pcg_tol=1e-12, pcg_check=4, pcg_variant=variant,
                        precond=precond) as s:
        s.set_potential(V)
        s.set_state(U0)
        # Algorithm 1 through qo_run (the stop test is taken on U_n before its step), in
        # chunks so that long runs report progress
        steps, conv, st = 0, False, None
        while steps < max_steps and not conv:
            k, _, conv, st_k = s.run(tau, min(2000, max_steps - steps), grad_tol=stop)
            steps += k
            if k:
                st = st_k
            if st is None or not np.isfinite(st["energy"]):
                break
            if log and not conv:
                log(f"  m={m} tau={tau}: step {steps} grad {st['grad_norm']:.3e} "
                    f"|O| {st['orth_err_fro']:.3e}")
        lam = s.eigenpairs("ritz")
        lam_p = s.eigenpairs("paper")
    err = np.abs(lam - lam_ref[:N]) / np.abs(lam_ref[:N])
    err_p = np.abs(lam_p - lam_ref[:N]) / np.abs(lam_ref[:N])
    return {
        "grid": m, "h": 2 * HALF / (m + 1), "tau": tau, "N": N, "steps": steps,
        "converged": bool(conv), "tau_times_steps": tau * steps,
        "orth_err_last_step": float(st["orth_err_fro"]) if st else None,
        "energy_last_step": float(st["energy"]) if st else None,
        "half_sum_lambda": float(0.5 * lam_ref[:N].sum()),
        "ritz": [float(v) for v in lam],
        "max_err_ritz": float(err.max()), "max_err_paper_mode": float(err_p.max()),
        "err_ritz": [float(e) for e in err], "seconds": time.perf_counter() - t0,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[199])
    ap.add_argument("--tau", type=float, nargs="+", default=[0.05, 0.1, 0.5, 0.9, 1.0, 1.5])
    ap.add_argument("--max-steps", type=int, default=40000)
    ap.add_argument("--N", type=int, default=15)
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "fast_poisson"],
                    help="solver of G (the solves are taken to 1e-12 either way)")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    for m in args.n:
        for tau in args.tau:
            r = run(m, tau, N=args.N, max_steps=args.max_steps, log=log,
                    precond=args.precond)
            log(f"m={m} tau={tau}: {r['steps']} steps (converged {r['converged']}), "
                f"tau*steps={r['tau_times_steps']:.1f}, max err {r['max_err_ritz']:.2e}, "
                f"|O| {r['orth_err_last_step']:.1e} ({r['seconds']:.1f} s)")
            r["precond"] = args.precond
            print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
