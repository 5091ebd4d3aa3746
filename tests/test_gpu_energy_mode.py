"""GPU parity of the propagated energy (qo_energy_mode 1: K = <U, H_sigma U> carried by the
two stages' identities) against the oracle's energy from the stencil and against the GPU's
own stencil energy, and its error paths.

Each step the identities hold up to the solves' tolerance (1e-12 relative residual here),
so after S steps without re-taking K the reported energy stays within about S * 1e-12 *
cond(H) of the true one; the tests allow 1e-9 relative over 30 steps."""
import numpy as np
import pytest

from paper_2605_25149_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def B():
    from paper_2605_25149_amd import binding

    binding.load_library()
    return binding


@pytest.mark.parametrize("precond", ["fast_poisson", "jacobi"])
@pytest.mark.parametrize("anchor", [0, 7])
def test_propagated_energy_matches_oracle(torch, B, oracle_mod, precond, anchor):
    """3-D 24x20x18 wells, N = 8, 30 steps: E and E_sigma per step within 1e-9 relative of
    the oracle's stencil energies (same steps, tol 1e-12) and of the GPU's mode-0 run."""
    n, N, tau = (24, 20, 18), 8, 9.0
    V = inputs.gaussian_wells(n, seed=0)
    U0 = inputs.random_block(int(np.prod(n)), N, seed=1)
    prob = oracle_mod.Problem(3, n, V)
    ref = oracle_mod.Oracle(prob, U0, tol=1e-12, precond=precond)
    runs = {}
    for mode in (0, 1):
        with B.Solver(3, n, N, pcg_tol=1e-12, pcg_check=1, precond=precond) as s:
            s.set_potential(V)
            s.set_state(U0)
            if mode:
                s.energy_mode(1, anchor)
            runs[mode] = [s.step(tau) for _ in range(30)]
    worst = 0.0
    for k in range(30):
        a = ref.step(tau)
        g = runs[1][k]
        for key, val in (("energy", a.energy), ("energy_shifted", a.energy_shifted)):
            rel = abs(g[key] - val) / abs(val)
            worst = max(worst, rel)
            assert rel <= 1e-9, (k, key, rel)
            assert abs(g[key] - runs[0][k][key]) <= 1e-9 * abs(val), (k, key)
    print(f"{precond} anchor {anchor}: worst relative energy difference {worst:.2e}")


def test_energy_mode_errors(torch, B):
    """Mixed precision, an unknown mode and a negative anchor are refused (QO_ERR_ARG)."""
    with B.Solver(2, (16, 16), 2, precision="mixed") as s:
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.energy_mode(1)
    with B.Solver(2, (16, 16), 2) as s:
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.energy_mode(2)
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.energy_mode(1, -1)
        s.energy_mode(1, 3)
        s.energy_mode(0)


def test_propagated_energy_with_adaptive_undo(torch, B):
    """Algorithm 1 with the adaptive step (qo_run with tau_max, which undoes and halves a
    step whose E_sigma rises or whose ||O|| grows): the propagated energy restarts from the
    stencil after every undo, so each accepted step's E_sigma matches the stencil-energy
    run within 1e-10 relative and the run reaches the same eigenvalues."""
    n, N = (32, 32), 4
    V = inputs.harmonic(n, 100.0)
    U0 = inputs.random_block(1024, N, seed=1)
    lam1 = 12.9544687
    out = {}
    for mode in (0, 1):
        with B.Solver(2, n, N, pcg_tol=1e-12) as s:
            s.set_potential(V)
            s.set_state(U0)
            if mode:
                s.energy_mode(1, 0)
            energies, tau, steps, conv = [], 0.3 * lam1, 0, False
            while steps < 2000 and not conv:
                k, tau, conv, st = s.run(tau, 1, grad_tol=1e-6, tau_max=3.0 * lam1)
                steps += k
                if k:
                    energies.append(st["energy_shifted"])
            out[mode] = (np.array(energies), s.eigenpairs("ritz"), conv)
    (e0, l0, c0), (e1, l1, c1) = out[0], out[1]
    assert c0 and c1 and len(e0) == len(e1)
    assert np.max(np.abs(e1 - e0) / np.abs(e0)) <= 1e-10
    np.testing.assert_allclose(l1, l0, rtol=1e-12)
