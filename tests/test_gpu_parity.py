"""GPU parity: the HIP library (through the C ABI) against the oracle on the same
seeded inputs.  Tolerances are stated per test."""
import os

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


def _solver(B, dim, n, N, env=None, **kw):
    old = {}
    for k, v in (env or {}).items():
        old[k] = os.environ.get(k)
        os.environ[k] = str(v)
    try:
        return B.Solver(dim, n, N, **kw)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


CASES_APPLY = [
    # dim, n, N, tiling env (forces several bands and z-chunks with ragged tails)
    (2, (32, 32), 4, None),
    (2, (37, 29), 3, {"QO_TY": 5}),
    (2, (300, 7), 2, None),
    (2, (1000, 3), 2, None),
    (3, (13, 11, 10), 5, {"QO_TY": 3, "QO_ZC": 4}),
    (3, (24, 20, 18), 3, None),
    (3, (64, 64, 64), 2, None),
    # rows wider than a workgroup with several planes per tile: the engine that loops over
    # the halo columns (the one-halo-column-per-thread engine would leave columns >= 256)
    (3, (300, 5, 7), 2, None),
    (3, (520, 3, 4), 3, None),
]


@pytest.mark.parametrize("dim,n,N,env", CASES_APPLY)
def test_apply_matches_oracle(torch, B, oracle_mod, dim, n, N, env):
    """Stencil H_sigma X: max |diff| <= 1e-13 * max|H X| (rounding-order differences only)."""
    V = inputs.gaussian_wells(n, seed=0)
    prob = oracle_mod.Problem(dim, n, V, sigma=0.3)
    X = inputs.random_block(prob.ng, N, seed=2)
    ref = prob.apply(X)
    with _solver(B, dim, n, N, env, sigma=0.3, pcg_variant=0 if n[0] > 256 else 1) as s:
        s.set_potential(V)
        Y = B.to_numpy(s.apply(B.as_block(X)))
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("ncols,ng", [(3, 1000), (37, 4097), (70, 20000), (4, 262144)])
def test_gram_pair_fp64(torch, B, ncols, ng):
    """<Z,Z> = h^d Z^T Z for Z = [X Y]: FP64 MFMA split-K vs NumPy, rel 1e-13 of max entry."""
    n = (ng, 1) if ng <= 1024 else None
    # pick a 2-D grid with Ng = ng (1 row when it fits; else a square-ish factorisation)
    if n is None:
        for a in range(1024, 0, -1):
            if ng % a == 0:
                n = (a, ng // a)
                break
    rng = np.random.default_rng(ncols)
    X = rng.standard_normal((ng, ncols))
    Y = rng.standard_normal((ng, ncols))
    with B.Solver(2, n, min(ncols, ng - 1), pcg_variant=0) as s:
        w = (1.0 / (n[0] + 1)) * (1.0 / (n[1] + 1))
        G = s.gram_pair(B.as_block(X), B.as_block(Y))
    Z = np.hstack([X, Y])
    ref = w * (Z.T @ Z)
    assert np.max(np.abs(G - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.array_equal(G, G.T)


def _bf16_rne(a):
    """Round float64 to bfloat16 (nearest-even on the float64 mantissa), returned as float64."""
    from fractions import Fraction  # noqa: F401  (documentation: exact rounding reference)

    b = np.asarray(a, dtype=np.float64).view(np.uint64)
    lsb = (b >> np.uint64(45)) & np.uint64(1)
    r = (b + np.uint64(0xFFFFFFFFFFF) + lsb) & ~np.uint64((1 << 45) - 1)
    return r.view(np.float64)


def test_gram_pair_bf16(torch, B):
    """Mixed precision Gram: inputs rounded to BF16 (nearest-even), FP32 accumulation per chunk.
    Matches the exact product of the rounded inputs to FP32-accumulation accuracy and the
    FP64 Gram to BF16 accuracy."""
    n = (96, 96)
    ng = n[0] * n[1]
    ncols = 20
    rng = np.random.default_rng(3)
    X = rng.standard_normal((ng, ncols))
    Y = rng.standard_normal((ng, ncols))
    w = (1.0 / 97) ** 2
    with B.Solver(2, n, ncols, precision="mixed") as s:
        G = s.gram_pair(B.as_block(X), B.as_block(Y))
    Z = np.hstack([X, Y])
    Zr = _bf16_rne(Z)
    exact_r = w * (Zr.T @ Zr)
    scale = w * np.sqrt(np.outer((Zr * Zr).sum(0), (Zr * Zr).sum(0)))
    assert np.max(np.abs(G - exact_r) / scale) <= 1e-5
    ref = w * (Z.T @ Z)
    assert np.max(np.abs(G - ref) / scale) <= 2e-3


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("dim,n,N,env,x0", [
    (3, (20, 18, 16), 6, None, False),
    (3, (13, 11, 10), 5, {"QO_TY": 3, "QO_ZC": 4, "QO_CG_TY": 2, "QO_CG_ZC": 3}, True),
    (3, (40, 33, 35), 3, None, True),
    (2, (32, 32), 4, None, True),
])
def test_solve_matches_oracle(torch, B, oracle_mod, dim, n, N, env, x0, variant):
    """Jacobi-PCG in both forms (0: two sweeps, Hestenes-Stiefel; 1: one sweep,
    Chronopoulos-Gear): identical per-column iteration counts and solutions within 1e-11 of
    the oracle's same form (same algorithm and stop rule; differences are rounding order)."""
    # wells in 3-D; the 2-D wells of this family are deep enough to make H indefinite
    V = inputs.gaussian_wells(n, seed=0) if dim == 3 else inputs.harmonic(n, 100.0)
    prob = oracle_mod.Problem(dim, n, V)
    Bm = inputs.random_block(prob.ng, N, seed=4)
    X0 = inputs.random_block(prob.ng, N, seed=5) * 1e-3 if x0 else None
    Xr, itr, st, _ = prob.solve(Bm, X0=X0, tol=1e-10, variant=variant)
    assert st == 0
    with _solver(B, dim, n, N, env, pcg_tol=1e-10, pcg_check=3, pcg_variant=variant) as s:
        s.set_potential(V)
        Xg, itg = s.solve(B.as_block(Bm), None if X0 is None else B.as_block(X0))
        Xg = B.to_numpy(Xg)
    assert list(itg) == list(itr)
    assert np.max(np.abs(Xg - Xr)) <= 1e-11 * np.max(np.abs(Xr))


def test_solve_mixed_refinement(torch, B, oracle_mod):
    """FP32 PCG inside FP64 refinement reaches the FP64 tolerance: true FP64 residual
    ||b - H x|| <= tol ||b|| per column (checked with the oracle's operator)."""
    n = (24, 22, 20)
    V = inputs.gaussian_wells(n, seed=0)
    prob = oracle_mod.Problem(3, n, V)
    Bm = inputs.random_block(prob.ng, 5, seed=4)
    with B.Solver(3, n, 5, pcg_tol=1e-10, precision="mixed", refine_inner_tol=1e-4) as s:
        s.set_potential(V)
        Xg, itg = s.solve(B.as_block(Bm))
        Xg = B.to_numpy(Xg)
    res = np.linalg.norm(Bm - prob.apply(Xg), axis=0) / np.linalg.norm(Bm, axis=0)
    assert np.all(res <= 1e-10)
    Xr = prob.solve_direct(Bm)
    assert np.max(np.abs(Xg - Xr)) <= 1e-8 * np.max(np.abs(Xr))


def iters_agree(gpu, orc):
    """PCG iteration counts are integers decided by a floating-point test (||r|| <= tol ||b||).
    Both sides run the same algorithm in FP64, but in a different summation order, so a solve
    whose residual sits on the threshold can stop one or two iterations apart.  That happens
    late in a trajectory at tol 1e-12, where warm starts begin within a few ulps-worth of the
    tolerance.  Required: at least 90% of the solves equal, none off by more than max(5, 5%)."""
    gpu, orc = np.asarray(gpu).ravel(), np.asarray(orc).ravel()
    same = np.mean(gpu == orc)
    ok = same >= 0.90 and np.all(np.abs(gpu - orc) <= np.maximum(5, 0.05 * orc))
    if not ok:
        bad = np.nonzero(gpu != orc)[0]
        print("iteration mismatches (solve index, gpu, oracle):",
              [(int(i), int(gpu[i]), int(orc[i])) for i in bad[:40]])
    return ok


def _run_pair(B, oracle_mod, dim, n, N, V, U0, tau, nsteps, env=None, tol=1e-12, warm=True,
              variant=1, **kw):
    prob = oracle_mod.Problem(dim, n, V)
    ref = oracle_mod.Oracle(prob, U0, tol=tol, warm_start=warm, variant=variant)
    gpu_stats, ref_stats = [], []
    s = _solver(B, dim, n, N, env, pcg_tol=tol, warm_start=warm, pcg_variant=variant, **kw)
    s.set_potential(V)
    s.set_state(U0)
    for _ in range(nsteps):
        ref_stats.append(ref.step(tau))
        gpu_stats.append(s.step(tau))
    return prob, ref, s, ref_stats, gpu_stats


@pytest.mark.parametrize("warm,variant", [(True, 1), (False, 1), (True, 0)])
def test_step_cfg_small_200(torch, B, oracle_mod, warm, variant):
    """2-D 32x32, V = 50|x-c|^2, N = 4, tau = 0.9 lambda_1, 200 steps from a random start.
    Per step: E and E_sigma within 1e-10 relative, PCG iterations equal (see iters_agree); at
    the end the
    state agrees to 1e-9, Ritz values to 1e-10 and the subspace angle is <= 1e-8."""
    n, N = (32, 32), 4
    V = inputs.harmonic(n, 100.0)
    U0 = inputs.random_block(1024, N, seed=1)
    tau = 0.9 * 12.9544687
    prob, ref, s, rs, gs = _run_pair(B, oracle_mod, 2, n, N, V, U0, tau, 200, warm=warm,
                                     variant=variant)
    try:
        for a, g in zip(rs, gs):
            assert abs(g["energy"] - a.energy) <= 1e-10 * abs(a.energy)
            assert abs(g["energy_shifted"] - a.energy_shifted) <= 1e-10 * abs(a.energy_shifted)
            assert abs(g["orth_err_fro"] - a.orth_err_fro) <= 1e-10 * max(1.0, a.orth_err_fro) + 1e-13
            assert abs(g["grad_norm"] - a.grad_norm) <= 1e-6 * a.grad_norm + 1e-9
        U = B.to_numpy(s.get_state())
        assert np.max(np.abs(U - ref.U)) <= 1e-9 * np.max(np.abs(ref.U))
        lam_ref, _ = oracle_mod.ritz(prob, ref.U)
        lam = s.eigenpairs("ritz")
        np.testing.assert_allclose(lam, lam_ref, rtol=1e-10)
        assert oracle_mod.subspace_sin(U, ref.U) <= 1e-8
        assert iters_agree([g["pcg_iters"] for g in gs], [a.pcg_iters for a in rs])
    finally:
        s.close()


def test_step_matrices_one_step(torch, B, oracle_mod):
    """One step on a 3-D grid with several tiles: the N x N matrices S, M, R, X, Y, O, A, B and
    the blocks P, U_hat, Q, U_1 against the oracle (1e-10 relative to each one's max)."""
    n, N = (13, 11, 10), 5
    V = inputs.gaussian_wells(n, seed=0)
    U0 = inputs.random_block(int(np.prod(n)), N, seed=1)
    prob, ref, s, rs, gs = _run_pair(B, oracle_mod, 3, n, N, V, U0, 9.0, 1,
                                     env={"QO_TY": 3, "QO_ZC": 4, "QO_CG_TY": 2, "QO_CG_ZC": 3})
    try:
        last = ref.last
        for name in ["S", "M", "R", "X", "Y", "O", "A", "B"]:
            g = s.get_matrix(name)
            r = last[name]
            assert np.max(np.abs(g - r)) <= 1e-10 * np.max(np.abs(r)), name
        for name, key in [("P", "P"), ("U_hat", "U_hat"), ("Q", "Q")]:
            g = B.to_numpy(s.get_block(name))
            r = last[key]
            assert np.max(np.abs(g - r)) <= 1e-10 * np.max(np.abs(r)), name
        U = B.to_numpy(s.get_state())
        assert np.max(np.abs(U - ref.U)) <= 1e-10 * np.max(np.abs(ref.U))
    finally:
        s.close()


def test_step_3d_wells(torch, B, oracle_mod):
    """3-D 24x20x18 Gaussian wells, N = 8, 12 steps at tol 1e-10 (warm starts on):
    E within 1e-10, iterations equal, final state within 1e-9."""
    n, N = (24, 20, 18), 8
    V = inputs.gaussian_wells(n, seed=0)
    U0 = inputs.random_block(int(np.prod(n)), N, seed=1)
    prob = oracle_mod.Problem(3, n, V)
    lam1 = 9.0  # below lambda_1 of this family at this size
    prob, ref, s, rs, gs = _run_pair(B, oracle_mod, 3, n, N, V, U0, lam1, 12, tol=1e-10)
    try:
        assert iters_agree([g["pcg_iters"] for g in gs], [a.pcg_iters for a in rs])
        for a, g in zip(rs, gs):
            assert abs(g["energy"] - a.energy) <= 1e-10 * abs(a.energy)
        U = B.to_numpy(s.get_state())
        assert np.max(np.abs(U - ref.U)) <= 1e-9 * np.max(np.abs(ref.U))
    finally:
        s.close()


def test_eigenpairs_modes(torch, B, oracle_mod):
    """After convergence on the 2-D separable case: Ritz values (with vectors) and paper-mode
    values against the oracle and against the closed form (1e-10)."""
    n, N = (32, 32), 4
    V = inputs.harmonic(n, 100.0)
    U0 = inputs.random_block(1024, N, seed=1)
    tau = 0.9 * 12.9544687
    with B.Solver(2, n, N, pcg_tol=1e-12) as s:
        s.set_potential(V)
        s.set_state(U0)
        s.step(tau, 300)
        lam, vec = s.eigenpairs("ritz", vectors=True)
        lamp = s.eigenpairs("paper")
        U = B.to_numpy(s.get_state())
        vec = B.to_numpy(vec)
    prob = oracle_mod.Problem(2, n, V)
    lam_ref, c = oracle_mod.ritz(prob, U)
    np.testing.assert_allclose(lam, lam_ref, rtol=1e-10)
    P = prob.solve_direct(U)
    np.testing.assert_allclose(lamp, oracle_mod.paper_eigenvalues(prob, U, P), rtol=1e-9)
    # Ritz vectors: S-orthonormal and residual small for the converged pairs
    S = prob.inner(vec, vec)
    assert np.max(np.abs(S - np.eye(N))) <= 1e-10
    HV = prob.apply(vec)
    res = np.linalg.norm(HV - vec * lam, axis=0) / np.linalg.norm(vec, axis=0)
    assert np.all(res[:3] <= 1e-4 * lam[:3])


def test_error_paths(torch, B):
    """Status codes: NOT_SPD (indefinite H_sigma or rank-deficient start), PCG_NOCONV with the
    state unchanged (transactional step), NONFINITE for NaN data, ARG for bad tau."""
    n, N = (16, 16), 3
    V = inputs.harmonic(n, 100.0)
    U0 = inputs.random_block(256, N, seed=1)
    with B.Solver(2, n, N, pcg_tol=1e-10, pcg_maxit=3) as s:
        s.set_potential(V)
        s.set_state(U0)
        with pytest.raises(B.QOError) as e:
            s.step(5.0)
        assert e.value.status == B.QO_ERR_PCG_NOCONV
        np.testing.assert_array_equal(B.to_numpy(s.get_state()), U0)
        with pytest.raises(B.QOError) as e:
            s.step(-1.0)
        assert e.value.status == B.QO_ERR_ARG
    # V = 0 makes Jacobi a scalar; with sigma = -2 lambda_1 the lowest sine mode has
    # negative curvature, so PCG on it breaks down at its first iteration
    xs = inputs.grid_coords(n)
    mode = np.sin(np.pi * xs[0]) * np.sin(np.pi * xs[1])
    lam1 = 2 * 4 * 0.5 * 17**2 * np.sin(np.pi / 34) ** 2
    Um = U0.copy()
    Um[:, 0] = mode
    with B.Solver(2, n, N, sigma=-2 * lam1) as s:
        s.set_potential(np.zeros(256))
        s.set_state(Um)
        with pytest.raises(B.QOError) as e:
            s.step(5.0)
        assert e.value.status == B.QO_ERR_NOT_SPD
    with B.Solver(2, n, N, sigma=-1e5) as s:  # negative diagonal: rejected up front
        with pytest.raises(B.QOError) as e:
            s.set_potential(V)
        assert e.value.status == B.QO_ERR_NOT_SPD
    with B.Solver(2, n, N) as s:
        Vb = V.copy()
        Vb[7] = np.nan
        with pytest.raises(B.QOError) as e:
            s.set_potential(Vb)
        assert e.value.status == B.QO_ERR_NONFINITE
        s.set_potential(V)
        Ub = U0.copy()
        Ub[3, 1] = np.inf
        with pytest.raises(B.QOError) as e:
            s.set_state(Ub)
        assert e.value.status == B.QO_ERR_NONFINITE
        Ud = U0.copy()
        Ud[:, 2] = Ud[:, 0]
        s.set_state(Ud)
        with pytest.raises(B.QOError) as e:
            s.step(5.0)
        assert e.value.status == B.QO_ERR_NOT_SPD
    with B.Solver(2, n, N) as s:
        with pytest.raises(B.QOError) as e:
            s.step(5.0)
        assert e.value.status == B.QO_ERR_STATE


def test_algorithm1_fixed_and_adaptive(torch, B, oracle_mod):
    """Algorithm 1 (Sec. 5) through qo_run: with a fixed step the number of steps to
    ||grad|| <= 1e-6 matches the oracle's (within one step: the test compares a floating-point
    norm with a threshold) and the final state agrees; the adaptive step (undo and halve on an
    energy rise, grow up to tau_max) converges to the same eigenvalues and keeps E_sigma
    monotone over accepted steps."""
    n, N = (32, 32), 4
    V = inputs.harmonic(n, 100.0)
    U0 = inputs.random_block(1024, N, seed=1)
    lam1 = 12.9544687
    prob = oracle_mod.Problem(2, n, V)
    ref = oracle_mod.Oracle(prob, U0, tol=1e-12, variant=0)
    kref, _ = ref.algorithm1(0.9 * lam1, 1e-6, 1000)
    with B.Solver(2, n, N, pcg_tol=1e-12, pcg_variant=0) as s:
        s.set_potential(V)
        s.set_state(U0)
        k, tau_end, conv, st = s.run(0.9 * lam1, 1000, grad_tol=1e-6)
        U = B.to_numpy(s.get_state())
        lam_fixed = s.eigenpairs("ritz")
    assert conv and abs(k - kref) <= 1
    if k == kref:
        assert np.max(np.abs(U - ref.U)) <= 1e-9 * np.max(np.abs(ref.U))
    with B.Solver(2, n, N, pcg_tol=1e-12, pcg_variant=0) as s:
        s.set_potential(V)
        s.set_state(U0)
        energies = []
        steps, conv2 = 0, False
        tau = 0.3 * lam1
        while steps < 2000 and not conv2:
            k2, tau, conv2, st = s.run(tau, 1, grad_tol=1e-6, tau_max=3.0 * lam1)
            steps += k2
            if k2:
                energies.append(st["energy_shifted"])
        lam_ad = s.eigenpairs("ritz")
    assert conv2
    assert np.all(np.diff(energies) <= 1e-9 * np.abs(np.array(energies[1:])))
    np.testing.assert_allclose(lam_ad, lam_fixed, rtol=1e-9)


def test_eigsum_gradient(torch, B, oracle_mod):
    """d(sum of Ritz values)/dV = h^d diag(U S^{-1} U^T) on a non-orthogonal 3-D block:
    GPU against the oracle's formula (1e-12 relative to the max entry)."""
    n, N = (13, 11, 10), 5
    V = inputs.gaussian_wells(n, seed=0)
    U0 = inputs.random_block(int(np.prod(n)), N, seed=1)
    prob = oracle_mod.Problem(3, n, V)
    ref = oracle_mod.eigsum_gradient(prob, U0)
    with B.Solver(3, n, N) as s:
        s.set_potential(V)
        s.set_state(U0)
        g = s.eigsum_gradient().cpu().numpy()
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))
