"""Finite-difference analogue of the paper's first numerical example (Sec. 5, Example 1).

The 2-D harmonic oscillator -1/2 Lap u + 1/2 |x|^2 u = lambda u on (-5.5, 5.5)^2 with
N = 15 eigenpairs (the first five shells 1, 2, 3, 4, 5 with multiplicities 1..5), run
with Algorithm 1 of Sec. 5 at a fixed time step until ||grad_G E_G(U_n)|| < 1e-5, from a
random start.  The paper uses quadratic finite elements with Ng = 39,601 unknowns; a
199 x 199 interior FD grid has the same Ng.  For each tau this reports the number of steps,
tau * steps (the paper reads a roughly constant value as a mesh-independent time scale),
the final ||<U,U> - I|| and the relative errors of the Ritz values against the FD
operator's exact eigenvalues (sums of 1-D dense eigenvalues, the operator being separable).

Usage:  python -m paper_2605_25149_amd.experiments.harmonic_example --n 199 --tau 0.05 0.5
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


def run(m, tau, N=15, max_steps=40000, seed=1, stop=1e-5, variant=0, log=None):
    n = (m, m)
    L = (2 * HALF, 2 * HALF)
    V = inputs.harmonic(n, 1.0, centre=(HALF, HALF), L=L)
    U0 = inputs.random_block(m * m, N, seed=seed) / (2 * HALF)  # E<U0,U0> = I
    lam_ref = fd_reference(m, N)
    t0 = time.perf_counter()
    with binding.Solver(2, n, N, L=L, pcg_tol=1e-12, pcg_check=4, pcg_variant=variant) as s:
        s.set_potential(V)
        s.set_state(U0)
        steps, st = 0, None
        grad = np.inf
        while steps < max_steps:
            st = s.step(tau)
            steps += 1
            grad = st["grad_norm"]
            if not np.isfinite(st["energy"]):
                break
            if log and steps % 2000 == 0:
                log(f"  m={m} tau={tau}: step {steps} grad {grad:.3e} |O| {st['orth_err_fro']:.3e}")
            if grad < stop:
                break
        lam = s.eigenpairs("ritz")
        lam_p = s.eigenpairs("paper")
    err = np.abs(lam - lam_ref[:N]) / np.abs(lam_ref[:N])
    err_p = np.abs(lam_p - lam_ref[:N]) / np.abs(lam_ref[:N])
    return {
        "grid": m, "h": 2 * HALF / (m + 1), "tau": tau, "steps": steps,
        "converged": bool(grad < stop), "tau_times_steps": tau * steps,
        "grad_end": float(grad), "orth_err_end": float(st["orth_err_fro"]),
        "energy_end": float(st["energy"]), "half_sum_lambda": float(0.5 * lam_ref[:N].sum()),
        "max_err_ritz": float(err.max()), "max_err_paper_mode": float(err_p.max()),
        "err_ritz": [float(e) for e in err], "seconds": time.perf_counter() - t0,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[199])
    ap.add_argument("--tau", type=float, nargs="+", default=[0.05, 0.1, 0.5, 0.9, 1.0, 1.5])
    ap.add_argument("--max-steps", type=int, default=40000)
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    for m in args.n:
        for tau in args.tau:
            r = run(m, tau, max_steps=args.max_steps, log=log)
            log(f"m={m} tau={tau}: {r['steps']} steps, tau*steps={r['tau_times_steps']:.1f}, "
                f"max err {r['max_err_ritz']:.2e}, |O| {r['orth_err_end']:.1e} "
                f"({r['seconds']:.1f} s)")
            print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
