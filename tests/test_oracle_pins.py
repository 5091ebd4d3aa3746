"""Pins of the oracle against facts fixed by the paper and by mathematics (CPU only).

Each test names what it pins.  None of them compares the oracle with itself:
closed forms, brute-force dense linear algebra, the paper's identities and
worked numbers, and invariants of the scheme.
"""
import json
import os

import numpy as np
import pytest

from paper_2605_25149_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_H(dim, n, L, kappa, sigma, V):
    """Dense H_sigma assembled entry by entry from the 5/7-point stencil (independent of the oracle)."""
    n = list(n)
    h = [L[k] / (n[k] + 1) for k in range(dim)]
    ng = int(np.prod(n))
    H = np.zeros((ng, ng))
    strides = [1, n[0], n[0] * (n[1] if dim > 1 else 1)]
    for idx in range(ng):
        coords = []
        rem = idx
        for k in range(dim):
            coords.append(rem % n[k])
            rem //= n[k]
        H[idx, idx] = V[idx] + sigma + sum(2 * kappa / h[k] ** 2 for k in range(dim))
        for k in range(dim):
            if coords[k] > 0:
                H[idx, idx - strides[k]] = -kappa / h[k] ** 2
            if coords[k] < n[k] - 1:
                H[idx, idx + strides[k]] = -kappa / h[k] ** 2
    return H


def sep_1d(n, L, kappa, vfun):
    """1-D dense eigenvalues of -kappa d2/dx2 + v(x) on n interior points."""
    h = L / (n + 1)
    x = (np.arange(n) + 1) * h
    T = (np.diag(np.full(n, 2 * kappa / h**2) + vfun(x))
         + np.diag(np.full(n - 1, -kappa / h**2), 1) + np.diag(np.full(n - 1, -kappa / h**2), -1))
    return np.linalg.eigvalsh(T)


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,L", [(2, (9, 7), (1.0, 1.3)), (3, (6, 5, 7), (1.0, 0.8, 1.2))])
def test_stencil_sine_modes(oracle_mod, dim, n, L):
    """V = 0: the sine modes are eigenvectors of -kappa Lap_h with eigenvalue
    sum_k 4 kappa / h_k^2 sin^2(m_k pi h_k / (2 L_k)) (closed form)."""
    O = oracle_mod
    prob = O.Problem(dim, n, np.zeros(int(np.prod(n))), L=L, kappa=0.5, sigma=0.0)
    xs = inputs.grid_coords(n, L)
    for modes in [(1, 1, 1), (2, 3, 1), (n[0], 1, 2)]:
        u = np.ones(prob.ng)
        lam = 0.0
        for k in range(dim):
            m = modes[k]
            u *= np.sin(m * np.pi * xs[k] / L[k])
            lam += 4 * 0.5 / prob.h[k] ** 2 * np.sin(m * np.pi * prob.h[k] / (2 * L[k])) ** 2
        Hu = prob.apply(u)[:, 0]
        assert np.max(np.abs(Hu - lam * u)) <= 1e-12 * lam


@pytest.mark.parametrize("dim,n", [(2, (5, 4)), (3, (3, 4, 3))])
def test_stencil_dense_bruteforce(oracle_mod, dim, n):
    """H_sigma X equals the dense stencil matrix times X, and the sparse (direct-mode)
    matrix equals the dense one."""
    O = oracle_mod
    rng = np.random.default_rng(5)
    L = (1.0, 1.1, 0.9)[:dim]
    V = rng.standard_normal(int(np.prod(n)))
    prob = O.Problem(dim, n, V, L=L, kappa=0.7, sigma=0.3)
    H = dense_H(dim, n, L, 0.7, 0.3, V)
    X = rng.standard_normal((prob.ng, 3))
    np.testing.assert_allclose(prob.apply(X), H @ X, rtol=0, atol=1e-12 * np.abs(H).max())
    np.testing.assert_allclose(prob.sparse_matrix().toarray(), H, rtol=0, atol=1e-12 * np.abs(H).max())
    q = prob.quad(X)
    np.testing.assert_allclose(q, np.einsum("ij,ij->j", X, H @ X), rtol=1e-12)


# ---------------------------------------------------------------------------
# inverse operator
# ---------------------------------------------------------------------------

def test_pcg_matches_dense_solve(oracle_mod):
    """PCG: true residual <= tol-level and the solution agrees with a dense solve."""
    O = oracle_mod
    n = (7, 6, 5)
    V = inputs.gaussian_wells(n, seed=0)
    prob = O.Problem(3, n, V)
    H = dense_H(3, n, (1, 1, 1), 0.5, 0.0, prob.V)
    B = inputs.random_block(prob.ng, 4, seed=3)
    X, it, st, _ = prob.solve(B, tol=1e-12)
    assert st == O.ORC_OK and np.all(it > 0)
    Xd = np.linalg.solve(H, B)
    assert np.max(np.abs(X - Xd)) <= 1e-9 * np.max(np.abs(Xd))
    res = np.linalg.norm(B - H @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(res <= 1e-11)
    # a warm start at the solution converges in zero iterations
    X2, it2, st2, _ = prob.solve(B, X0=Xd, tol=1e-10)
    assert st2 == O.ORC_OK and np.all(it2 == 0)


def test_pcg_error_paths(oracle_mod):
    O = oracle_mod
    n = (6, 6)
    prob = O.Problem(2, n, np.zeros(36))
    B = inputs.random_block(36, 2, seed=1)
    _, _, st, _ = prob.solve(B, tol=1e-12, maxit=3)
    assert st == O.ORC_NOCONV
    neg = O.Problem(2, n, np.zeros(36), sigma=-1e5)  # indefinite: p.Hp <= 0 appears
    _, _, st, _ = neg.solve(B, tol=1e-12)
    assert st == O.ORC_NOT_SPD
    Bn = B.copy()
    Bn[3, 1] = np.nan
    _, _, st, cst = prob.solve(Bn, tol=1e-12)
    assert st == O.ORC_NONFINITE and cst[1] == O.ORC_NONFINITE and cst[0] == O.ORC_OK


# ---------------------------------------------------------------------------
# Sec. 4.1: the scheme
# ---------------------------------------------------------------------------

def _tiny_problem(O, seed=0, n=(5, 4)):
    V = inputs.harmonic(n, 30.0)
    return O.Problem(len(n), n, V)


def test_predictor_is_cayley_transform(oracle_mod):
    """First stage = Cayley transform (I - tau/2 A)^{-1} (I + tau/2 A) U_n of the skew
    operator A V = P<U,V> - U<P,V>, which is left multiplication by the Ng x Ng matrix
    w (P U^T - U P^T).  Brute force with an arbitrary (non-symmetric <U,P>) P."""
    O = oracle_mod
    prob = _tiny_problem(O)
    rng = np.random.default_rng(11)
    U = rng.standard_normal((prob.ng, 3))
    P = rng.standard_normal((prob.ng, 3)) * 0.1
    tau = 0.7
    U_hat, X, Y, (S, M, R) = O.predictor(prob, U, P, tau)
    K = prob.w * (P @ U.T - U @ P.T)
    I = np.eye(prob.ng)
    ref = np.linalg.solve(I - 0.5 * tau * K, (I + 0.5 * tau * K) @ U)
    assert np.max(np.abs(U_hat - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the implicit equation itself, with A applied from its definition
    Ut = 0.5 * (U_hat + U)
    AUt = P @ prob.inner(U, Ut) - U @ prob.inner(P, Ut)
    assert np.max(np.abs((U_hat - U) / tau - AUt)) <= 1e-12 * np.max(np.abs(AUt))
    # Gram preservation (Sec. 4.1, non-expansion lemma, first stage)
    np.testing.assert_allclose(prob.inner(U_hat, U_hat), S, rtol=0, atol=1e-12 * np.abs(S).max())


def _run(O, prob, U0, tau, nsteps, **kw):
    orc = O.Oracle(prob, U0, **kw)
    stats = []
    mats = []
    for _ in range(nsteps):
        S_before = prob.inner(orc.U, orc.U)
        st = orc.step(tau)
        stats.append(st)
        mats.append((S_before, orc.last, orc.U))
    return orc, stats, mats


def test_gram_recurrence_and_energy_identity(oracle_mod):
    """With exact solves (direct mode):
      O_{n+1} = O_n - tau (A_n O_n + O_n A_n) + tau^2 O_n B_n O_n      (Sec. 4.1)
      E(U_{n+1}) - E(U_hat) = -tau tr(<U_n,U_n> O_n) + tau^2/2 tr(A_n O_n^2)   (Sec. 4.2)
    (energies of the operator whose inverse is G, i.e. the shifted energy)."""
    O = oracle_mod
    prob = _tiny_problem(O, n=(8, 7))
    U0 = inputs.random_block(prob.ng, 3, seed=2)
    tau = 0.5 * 20.0
    orc, stats, mats = _run(O, prob, U0, tau, 4, direct=True)
    for S_before, last, U_next in mats:
        N = S_before.shape[0]
        On = S_before - np.eye(N)
        A, B = last["A"], last["B"]
        lhs = prob.inner(U_next, U_next) - np.eye(N)
        rhs = On - tau * (A @ On + On @ A) + tau**2 * On @ B @ On
        assert np.max(np.abs(lhs - rhs)) <= 1e-10 * max(1.0, np.abs(On).max())
        _, e_next = prob.energy(U_next)
        _, e_hat = prob.energy(last["U_hat"])
        d_ref = -tau * np.trace(S_before @ On) + 0.5 * tau**2 * np.trace(A @ On @ On)
        assert abs((e_next - e_hat) - d_ref) <= 1e-9 * max(1.0, abs(e_hat))


def test_separable_closed_form_cfg_small(oracle_mod):
    """2-D unit square 32x32, V = 50|x - c|^2, N = 4, tau = 0.9 lambda_1, 200 steps from a
    random non-orthogonal start: Ritz values vs the Kronecker sum of 1-D dense spectra."""
    O = oracle_mod
    n = (32, 32)
    V = inputs.harmonic(n, 100.0)
    prob = O.Problem(2, n, V)
    mu = sep_1d(32, 1.0, 0.5, lambda x: 50 * (x - 0.5) ** 2)
    lam = np.sort(np.add.outer(mu, mu).ravel())
    assert abs(lam[0] - 12.9544687) < 1e-6
    U0 = inputs.random_block(prob.ng, 4, seed=1)
    tau = 0.9 * lam[0]
    orc, stats, _ = _run(O, prob, U0, tau, 200, tol=1e-12)
    l, _ = O.ritz(prob, orc.U)
    err = O.err_eigen(l, lam[:4])
    assert np.all(err[:3] <= 1e-10)
    assert err[3] <= 1e-5
    # energy dissipation (shifted energy; sigma = 0 here), quasi-orthogonality reached
    es = np.array([s.energy_shifted for s in stats])
    assert np.all(np.diff(es) <= 1e-9 * np.abs(es[1:]))
    assert stats[-1].orth_err_fro <= 1e-12
    # E -> 1/2 sum lambda at convergence (Sec. 5 reports E(U_end) against 1/2 sum lambda_ref)
    assert abs(stats[-1].energy - 0.5 * lam[:4].sum()) <= 1e-5 * lam[:4].sum()
    # asymptotic rate of the gradient: log-contraction per step ~ tau (1/lam_N - 1/lam_N+1)
    g = np.array([s.grad_norm for s in stats])
    rate = -np.log(g[-1] / g[-41]) / 40
    pred = tau * (1 / lam[3] - 1 / lam[4])
    assert 0.75 * pred <= rate <= 1.25 * pred


def test_dense_eigh_tiny_3d(oracle_mod):
    """3-D 6^3 Gaussian wells, N = 4 (lambda_4 = 25.8 < lambda_5 = 37.6): converged Ritz values equal the lowest dense eigenvalues,
    paper-mode eigenvalues equal them too once <U,U> = I, and the gradient vanishes."""
    O = oracle_mod
    n = (6, 6, 6)
    V = inputs.gaussian_wells(n, seed=0)
    prob = O.Problem(3, n, V)
    H = dense_H(3, n, (1, 1, 1), 0.5, 0.0, prob.V)
    ev = np.linalg.eigvalsh(H)
    U0 = inputs.random_block(prob.ng, 4, seed=1)
    tau = 0.9 * ev[0]
    orc, stats, _ = _run(O, prob, U0, tau, 400, direct=True)
    l, _ = O.ritz(prob, orc.U)
    np.testing.assert_allclose(l, ev[:4], rtol=1e-10)
    P = prob.solve_direct(orc.U)
    np.testing.assert_allclose(O.paper_eigenvalues(prob, orc.U, P), ev[:4], rtol=1e-9)
    assert O.grad_norm(prob, orc.U, P) <= 1e-7


def test_paper_example1_fd(oracle_mod):
    """Paper Example 1 (Sec. 5) on a finite-difference grid: the converged Ritz values approach
    the exact oscillator eigenvalues 1, 2, 2, 3, 3, 3 stated in the paper, with O(h^2) error."""
    O = oracle_mod
    g = json.load(open(os.path.join(GOLDEN, "harmonic_table1.json")))
    a = g["domain_half_width"]
    exact = np.array(g["exact_first_6"])
    errs = []
    for m in (39, 79):
        n = (m, m)
        V = inputs.harmonic(n, 1.0, centre=(a, a), L=(2 * a, 2 * a))
        prob = O.Problem(2, n, V, L=(2 * a, 2 * a))
        mu = sep_1d(m, 2 * a, 0.5, lambda x: 0.5 * (x - a) ** 2)
        lam_fd = np.sort(np.add.outer(mu, mu).ravel())[:7]
        # i.i.d. N(0,1) values scaled by |Omega|^{-1/2} so that E<U0,U0> = I
        U0 = inputs.random_block(prob.ng, 6, seed=1) / (2 * a)
        orc, stats, _ = _run(O, prob, U0, 0.9 * lam_fd[0], 250, direct=True)
        l, _ = O.ritz(prob, orc.U)
        np.testing.assert_allclose(l, lam_fd[:6], rtol=1e-8)
        errs.append(np.max(np.abs(l - exact)))
    h_ratio = (2 * a / 40) / (2 * a / 80)
    assert errs[0] < 0.05 and errs[1] < errs[0] / (0.8 * h_ratio**2)


def test_quasi_stiefel_invariance_and_contraction(oracle_mod):
    """U_0 in M_>= and tau below the bounds of Sec. 4.1 / 4.3: O_n stays positive semidefinite,
    <U_{n+1},U_{n+1}> <= <U_n,U_n>, ||O_{n+1}||^2 <= (1 - tau/E(U_0)) ||O_n||^2."""
    O = oracle_mod
    n = (10, 9)
    V = inputs.harmonic(n, 60.0)
    prob = O.Problem(2, n, V)
    H = dense_H(2, n, (1, 1), 0.5, 0.0, prob.V)
    lam1 = np.linalg.eigvalsh(H)[0]
    rng = np.random.default_rng(7)
    Qb, _ = np.linalg.qr(rng.standard_normal((prob.ng, 3)))
    U0 = Qb / np.sqrt(prob.w) @ np.diag([1.3, 1.1, 1.02])
    S0 = prob.inner(U0, U0)
    E0, _ = prob.energy(U0)
    tau = min(lam1 / (3 * np.linalg.eigvalsh(S0).max()), E0) * 0.99
    orc, stats, mats = _run(O, prob, U0, tau, 30, direct=True)
    prev_norm = np.linalg.norm(S0 - np.eye(3))
    for S_before, last, U_next in mats:
        S_next = prob.inner(U_next, U_next)
        O_next = S_next - np.eye(3)
        assert np.linalg.eigvalsh(O_next).min() >= -1e-12
        assert np.linalg.eigvalsh(S_before - S_next).min() >= -1e-12
        nrm = np.linalg.norm(O_next)
        assert nrm**2 <= (1 - tau / E0) * prev_norm**2 + 1e-24
        prev_norm = nrm
        # Sec. 4.1 matrix bounds: A_n <= S/lambda_1, B_n <= A_n/lambda_1
        A, B = last["A"], last["B"]
        assert np.linalg.eigvalsh(S_before / lam1 - 0.5 * (A + A.T)).min() >= -1e-12
        assert np.linalg.eigvalsh(0.5 * (A + A.T) / lam1 - B).min() >= -1e-12


def test_spectral_bounds_random(oracle_mod):
    """Sec. 3.3 lemma: 1/(2E(U)) <= lambda(<U, G U>) <= lambda_max(<U,U>)/lambda_1."""
    O = oracle_mod
    n = (8, 8)
    prob = O.Problem(2, n, inputs.harmonic(n, 40.0))
    H = dense_H(2, n, (1, 1), 0.5, 0.0, prob.V)
    lam1 = np.linalg.eigvalsh(H)[0]
    U = inputs.random_block(prob.ng, 4, seed=9)
    P = prob.solve_direct(U)
    T = prob.inner(U, P)
    ev = np.linalg.eigvalsh(0.5 * (T + T.T))
    E, _ = prob.energy(U)
    assert ev.min() >= 1 / (2 * E) * (1 - 1e-12)
    assert ev.max() <= np.linalg.eigvalsh(prob.inner(U, U)).max() / lam1 * (1 + 1e-12)


def test_scaling_metamorphic(oracle_mod):
    """H -> 2H (kappa, V, sigma doubled) with tau -> 2 tau gives the same trajectory:
    G halves and tau doubles, so every stage is unchanged."""
    O = oracle_mod
    n = (12, 10)
    V = inputs.harmonic(n, 80.0)
    p1 = O.Problem(2, n, V, kappa=0.5)
    p2 = O.Problem(2, n, 2 * V, kappa=1.0)
    U0 = inputs.random_block(p1.ng, 3, seed=4)
    tau = 10.0
    o1, s1, _ = _run(O, p1, U0, tau, 8, tol=1e-12)
    o2, s2, _ = _run(O, p2, U0, 2 * tau, 8, tol=1e-12)
    assert np.max(np.abs(o1.U - o2.U)) <= 1e-12 * np.max(np.abs(o1.U))
    assert [s.pcg_iters for s in s1] == [s.pcg_iters for s in s2]


def test_right_orthogonal_equivariance(oracle_mod):
    """U_0 -> U_0 Q (Q orthogonal) gives U_n -> U_n Q: A_{UQ} = A_U and O -> Q^T O Q."""
    O = oracle_mod
    n = (9, 8)
    prob = O.Problem(2, n, inputs.harmonic(n, 70.0))
    U0 = inputs.random_block(prob.ng, 3, seed=6)
    Qm, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((3, 3)))
    o1, _, _ = _run(O, prob, U0, 8.0, 6, direct=True)
    o2, _, _ = _run(O, prob, U0 @ Qm, 8.0, 6, direct=True)
    assert np.max(np.abs(o1.U @ Qm - o2.U)) <= 1e-11 * np.max(np.abs(o1.U))


def test_orthonormal_start_stays_orthonormal(oracle_mod):
    """<U_0,U_0> = I implies O_n = 0 for all n (discrete analogue of Sec. 3.1)."""
    O = oracle_mod
    n = (9, 9)
    prob = O.Problem(2, n, inputs.harmonic(n, 50.0))
    rng = np.random.default_rng(3)
    Qb, _ = np.linalg.qr(rng.standard_normal((prob.ng, 3)))
    U0 = Qb / np.sqrt(prob.w)
    orc, stats, _ = _run(O, prob, U0, 9.0, 10, direct=True)
    assert max(s.orth_err_fro for s in stats) <= 1e-13


def test_paper_hydrogen_tables(oracle_mod):
    """The paper's worked numbers (Sec. 5, Tables 2-3): E_ref = 1/2 sum lambda_ref, and the
    printed err_i follow from the printed lambda_i and lambda_ref with the err_i definition."""
    O = oracle_mod
    g = json.load(open(os.path.join(GOLDEN, "hydrogen_tables.json")))
    assert abs(0.5 * sum(g["lambda_ref"]) - g["E_ref"]) <= 1e-15
    err = O.err_eigen(g["lambda_computed"], g["lambda_ref"])
    np.testing.assert_allclose(err, g["err_printed"], rtol=2e-3)
    # E(U_end) - 1/2 sum lambda_i is at the level of the solution accuracy
    assert abs(g["E_end"] - 0.5 * sum(g["lambda_computed"])) <= 1e-9


def test_pcg_one_reduction_form(oracle_mod):
    """The Chronopoulos-Gear form: same solution as a dense solve, iteration counts within a
    couple of the Hestenes-Stiefel form (same iterates in exact arithmetic), error paths."""
    O = oracle_mod
    n = (9, 8, 7)
    V = inputs.gaussian_wells(n, seed=0)
    prob = O.Problem(3, n, V)
    H = dense_H(3, n, (1, 1, 1), 0.5, 0.0, prob.V)
    B = inputs.random_block(prob.ng, 5, seed=3)
    X0 = inputs.random_block(prob.ng, 5, seed=8) * 1e-2
    for x0 in (None, X0):
        X1, it1, st1, _ = prob.solve(B, X0=x0, tol=1e-12, variant=1)
        X0r, it0, st0, _ = prob.solve(B, X0=x0, tol=1e-12, variant=0)
        assert st1 == O.ORC_OK and st0 == O.ORC_OK
        Xd = np.linalg.solve(H, B)
        assert np.max(np.abs(X1 - Xd)) <= 1e-9 * np.max(np.abs(Xd))
        assert np.max(np.abs(it1 - it0)) <= 2
    _, _, st, _ = prob.solve(B, tol=1e-12, maxit=3, variant=1)
    assert st == O.ORC_NOCONV
    p2 = O.Problem(2, (6, 6), np.zeros(36))
    xs = inputs.grid_coords((6, 6))
    mode = np.sin(np.pi * xs[0]) * np.sin(np.pi * xs[1])
    lam1 = 2 * 4 * 0.5 * 7**2 * np.sin(np.pi / 14) ** 2
    neg = O.Problem(2, (6, 6), np.zeros(36), sigma=-2 * lam1)
    _, _, st, _ = neg.solve(mode[:, None], tol=1e-12, variant=1)
    assert st == O.ORC_NOT_SPD


def test_eigsum_gradient_finite_differences(oracle_mod):
    """d(lambda_1 + ... + lambda_N)/dV_j at an exact eigenbasis equals h^d diag(U S^{-1} U^T)_j
    (Hellmann-Feynman): checked by central differences of dense eigenvalues on a 5 x 4 x 3 grid."""
    O = oracle_mod
    n = (5, 4, 3)
    V = inputs.gaussian_wells(n, seed=0)
    prob = O.Problem(3, n, V)
    H = dense_H(3, n, (1, 1, 1), 0.5, 0.0, prob.V)
    ev, vec = np.linalg.eigh(H)
    N = 3
    assert ev[N] - ev[N - 1] > 1.0
    U = vec[:, :N] * 1.7 + vec[:, :N] @ np.array([[1, .2, 0], [0, 1, .3], [0, 0, 1.]])  # any basis
    g = O.eigsum_gradient(prob, U)
    eps = 1e-4
    for j in [0, 7, 23, 41, 59]:
        dV = np.zeros(prob.ng)
        dV[j] = eps
        ep = np.linalg.eigvalsh(dense_H(3, n, (1, 1, 1), 0.5, 0.0, prob.V + dV))[:N].sum()
        em = np.linalg.eigvalsh(dense_H(3, n, (1, 1, 1), 0.5, 0.0, prob.V - dV))[:N].sum()
        # the discrete eigenvalue problem is H u = lambda u with mass h^d: dlambda/dV_j = u_j^2
        # for Euclidean-normalised u; in the grid inner product this is h^d * (grid u_j)^2
        assert abs((ep - em) / (2 * eps) - g[j]) <= 1e-6 * max(1.0, abs(g[j]))


# ---------------------------------------------------------------------------
# fast-Poisson preconditioner of the inverse-operator solve (reading R13)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,L,vshift", [(2, (9, 7), (1.0, 1.3), 3.0),
                                            (3, (6, 5, 7), (1.0, 0.8, 1.2), 0.0),
                                            (3, (4, 4, 4), (1.0, 1.0, 1.0), -5.0)])
def test_fast_poisson_precond_is_exact_inverse(oracle_mod, dim, n, L, vshift):
    """precond_apply equals the dense inverse of kappa (-Lap_h) + vbar assembled
    entry by entry from the stencil, vbar = max(0, mean(V + sigma)); and the 1-D
    eigenvalues it uses are those of the dense second-difference matrix."""
    O = oracle_mod
    ng = int(np.prod(n))
    rng = np.random.default_rng(11)
    V = rng.uniform(-1.0, 1.0, ng) + vshift
    sigma = 0.3
    prob = O.Problem(dim, n, V, L=L, sigma=sigma)
    vbar = max(0.0, float(np.mean(V)) + sigma)
    assert prob.precond_vbar() == pytest.approx(vbar, rel=1e-14, abs=1e-14)
    M = dense_H(dim, n, L, 0.5, vbar, np.zeros(ng))
    R = inputs.random_block(ng, 3, seed=5)
    Z = prob.precond_apply(R)
    Zd = np.linalg.solve(M, R)
    assert np.max(np.abs(Z - Zd)) <= 1e-12 * np.max(np.abs(Zd))
    for k, mu in enumerate(prob.laplace_eigs()):
        ref = sep_1d(n[k], L[k], 1.0, lambda x: 0.0 * x)
        assert np.max(np.abs(np.sort(mu) - ref)) <= 1e-12 * ref.max()


def test_fast_poisson_pcg(oracle_mod):
    """PCG with the fast-Poisson preconditioner reaches the sparse-LU solution, and
    its iteration count stays flat when h halves while Jacobi's grows."""
    O = oracle_mod
    its_fp, its_j = [], []
    for n in [(8, 8, 8), (16, 16, 16)]:
        V = inputs.gaussian_wells(n, seed=0)
        prob = O.Problem(3, n, V)
        B = inputs.random_block(prob.ng, 3, seed=2)
        X, it, st, cst = prob.solve_fast_poisson(B, tol=1e-12)
        assert st == O.ORC_OK and np.all(cst == O.ORC_OK) and np.all(it > 0)
        Xd = prob.solve_direct(B)
        assert np.max(np.abs(X - Xd)) <= 1e-9 * np.max(np.abs(Xd))
        its_fp.append(int(it.max()))
        its_j.append(int(prob.solve(B, tol=1e-12)[1].max()))
        # a warm start at the solution takes no iteration
        _, it0, st0, _ = prob.solve_fast_poisson(B, X0=Xd, tol=1e-10)
        assert st0 == O.ORC_OK and np.all(it0 == 0)
    assert its_fp[1] <= its_fp[0] + 2 and its_fp[1] <= 20
    assert its_j[1] >= 1.5 * its_j[0]


def test_fast_poisson_pcg_error_paths(oracle_mod):
    O = oracle_mod
    n = (6, 6)
    prob = O.Problem(2, n, np.zeros(36))
    B = inputs.random_block(36, 2, seed=1)
    # with V = 0 the preconditioner is H itself: one iteration solves to rounding
    X1, it1, st1, _ = prob.solve_fast_poisson(B, tol=1e-12)
    assert st1 == O.ORC_OK and np.all(it1 == 1)
    well = O.Problem(2, n, inputs.harmonic(n, 400.0))
    _, _, st, _ = well.solve_fast_poisson(B, tol=1e-14, maxit=1)
    assert st == O.ORC_NOCONV
    neg = O.Problem(2, n, np.zeros(36), sigma=-1e5)  # indefinite H, SPD M (vbar = 0)
    _, _, st, _ = neg.solve_fast_poisson(B, tol=1e-12)
    assert st == O.ORC_NOT_SPD
    Bn = B.copy()
    Bn[3, 1] = np.nan
    _, _, st, cst = prob.solve_fast_poisson(Bn, tol=1e-12)
    assert st == O.ORC_NONFINITE and cst[1] == O.ORC_NONFINITE and cst[0] == O.ORC_OK


@pytest.mark.parametrize("loss", ["energy", "ritz_sum"])
@pytest.mark.parametrize("K", [0, 1, 4])
def test_steps_grad_finite_differences(oracle_mod, loss, K):
    """Reading R16: the reverse-mode derivative of K steps + loss against central
    differences of the forward map along random directions of V and of U_0 (FP64,
    eps = 1e-5: truncation and rounding both below 1e-7 relative here)."""
    O = oracle_mod
    n = (12, 10)
    V = inputs.harmonic(n, 100.0) + inputs.gaussian_wells(n, seed=3, depth=(1.0, 4.0))
    U0 = inputs.random_block(120, 3, seed=2)
    prob = O.Problem(2, n, V, sigma=0.3)
    L, gV, gU = O.steps_loss_grad(prob, U0, 8.0, K, loss)
    assert L == pytest.approx(O.steps_loss(prob, U0, 8.0, K, loss)[0], rel=1e-14)
    rng = np.random.default_rng(11)
    eps = 1e-5

    def f(VV, UU):
        return O.steps_loss(O.Problem(2, n, VV, sigma=0.3), UU, 8.0, K, loss)[0]

    for _ in range(2):
        dV = rng.standard_normal(120)
        dU = rng.standard_normal((120, 3))
        fdV = (f(V + eps * dV, U0) - f(V - eps * dV, U0)) / (2 * eps)
        fdU = (f(V, U0 + eps * dU) - f(V, U0 - eps * dU)) / (2 * eps)
        assert gV @ dV == pytest.approx(fdV, rel=1e-6, abs=1e-9 * abs(L))
        assert np.sum(gU * dU) == pytest.approx(fdU, rel=1e-6, abs=1e-9 * abs(L))


def test_steps_grad_ritz_sum_scale_invariance(oracle_mod):
    """The sum of the Ritz values depends on span U only, so at K = 0 its derivative along
    U_0 C vanishes for every C (a dropped term in the S^{-1} K S^{-1} part breaks this)."""
    O = oracle_mod
    n = (9, 8)
    prob = O.Problem(2, n, inputs.harmonic(n, 60.0), sigma=0.0)
    U0 = inputs.random_block(72, 4, seed=6)
    _, _, gU = O.steps_loss_grad(prob, U0, 5.0, 0, "ritz_sum")
    C = np.random.default_rng(2).standard_normal((4, 4))
    assert abs(np.sum(gU * (U0 @ C))) <= 1e-12 * np.linalg.norm(gU) * np.linalg.norm(U0 @ C)


def test_steps_grad_hellmann_feynman_limit(oracle_mod):
    """Reading R16 at convergence: after 80 steps U_K spans the lowest eigenspace of H, so
    the derivative of the sum of the Ritz values w.r.t. V is the Hellmann-Feynman
    gradient sum_i w phi_i(x_j)^2 of lambda_1 + ... + lambda_N (eigenvectors of the dense
    H from numpy's eigh, normalised in the grid inner product), the energy's is half of
    it (E = 1/2 sum lambda_i at an orthonormal eigenbasis) and dL/dU_0 vanishes."""
    O = oracle_mod
    n = (12, 10)
    V = inputs.harmonic(n, 100.0)
    prob = O.Problem(2, n, V, sigma=0.0)
    H = dense_H(2, n, (1.0, 1.0), 0.5, 0.0, V)
    lam, phi = np.linalg.eigh(H)
    hf = np.sum(phi[:, :3] ** 2, axis=1)  # w phi_w^2 with phi_w = phi / sqrt(w)
    U0 = inputs.random_block(120, 3, seed=2)
    L, gV, gU = O.steps_loss_grad(prob, U0, 10.0, 80, "ritz_sum")
    assert L == pytest.approx(lam[:3].sum(), rel=1e-8)
    assert np.max(np.abs(gV - hf)) <= 1e-6 * np.max(hf)
    assert np.max(np.abs(gU)) <= 1e-6
    L, gV, gU = O.steps_loss_grad(prob, U0, 10.0, 80, "energy")
    assert L == pytest.approx(0.5 * lam[:3].sum(), rel=1e-8)
    assert np.max(np.abs(gV - 0.5 * hf)) <= 1e-6 * np.max(hf)


def test_energy_matrix_identities(oracle_mod):
    """The identities behind the propagated energy (Sec. 4.1 stages; the trace of the second
    is the second-stage energy identity of Sec. 4.2), checked with exact solves on a 3-D
    wells grid: K_hat = <U_hat, H U_hat> = X^T K X + X^T S Y + Y^T S X + Y^T M^T Y and
    K_{n+1} = K_hat - tau (S_hat O + O S_hat) + tau^2 O A^T O, each against a direct
    evaluation with the stencil (1e-11 of the largest entry), over three steps."""
    O_ = oracle_mod
    n, N, tau = (9, 8, 7), 4, 6.0
    V = inputs.gaussian_wells(n, seed=2, depth=(1.0, 4.0))
    prob = O_.Problem(3, n, V, sigma=0.5)
    orc = O_.Oracle(prob, inputs.random_block(int(np.prod(n)), N, seed=3), direct=True)
    K = prob.inner(orc.U, prob.apply(orc.U))
    for _ in range(3):
        orc.step(tau)
        L = orc.last
        X, Y, S, M = L["X"], L["Y"], L["S"], L["M"]
        Kh = X.T @ K @ X + X.T @ S @ Y + Y.T @ S @ X + Y.T @ M.T @ Y
        Kh_ref = prob.inner(L["U_hat"], prob.apply(L["U_hat"]))
        assert np.max(np.abs(Kh - Kh_ref)) <= 1e-11 * np.max(np.abs(Kh_ref))
        Sh = prob.inner(L["U_hat"], L["U_hat"])
        Oc = L["O"]
        K = Kh - tau * (Sh @ Oc + Oc @ Sh) + tau ** 2 * Oc @ L["A"].T @ Oc
        K_ref = prob.inner(orc.U, prob.apply(orc.U))
        assert np.max(np.abs(K - K_ref)) <= 1e-11 * np.max(np.abs(K_ref))


def test_block_cg_pins(oracle_mod):
    """Reading R19, O'Leary block PCG (Jacobi) in the oracle:
    * the solution equals sparse LU within 1e-9 and every true residual is <= 5 tol (the
      stop test reads the recursive residual, which drifts from the true one by a few
      units of eps cond(H) over the iterations: ~3e-12 here at tol 1e-12);
    * with one column it is textbook Jacobi-PCG: same iteration count as the oracle's
      column solver and the same iterate (1e-12);
    * finite termination: on a 24-point grid with 4 right-hand sides the block Krylov space
      is full after ceil(24 / 4) = 6 iterations (two more allowed for rounding), where a
      single column needs more;
    * on a 2-D 32^2 grid its block iteration count is at most the largest column count."""
    O_ = oracle_mod
    n = (20, 17)
    V = inputs.harmonic(n, 100.0) + inputs.gaussian_wells(n, seed=3, depth=(1.0, 4.0))
    prob = O_.Problem(2, n, V, sigma=0.3)
    Bm = inputs.random_block(prob.ng, 5, seed=4)
    X, it, st = prob.solve_block_cg(Bm, tol=1e-12)
    assert st == O_.ORC_OK
    Xr = prob.solve_direct(Bm)
    assert np.max(np.abs(X - Xr)) <= 1e-9 * np.max(np.abs(Xr))
    res = np.linalg.norm(Bm - prob.apply(X), axis=0) / np.linalg.norm(Bm, axis=0)
    assert np.all(res <= 5e-12)

    b1 = Bm[:, :1]
    X1, it1, st1 = prob.solve_block_cg(b1, tol=1e-10)
    Xc, itc, stc, _ = prob.solve(b1, tol=1e-10)
    assert st1 == O_.ORC_OK and stc == O_.ORC_OK
    assert int(it1[0]) == int(itc[0])
    assert np.max(np.abs(X1 - Xc)) <= 1e-12 * np.max(np.abs(Xc))

    tiny = O_.Problem(2, (6, 4), inputs.harmonic((6, 4), 30.0), sigma=0.0)
    Bt = inputs.random_block(24, 4, seed=5)
    _, itb, stb = tiny.solve_block_cg(Bt, tol=1e-10)
    _, itcol, _, _ = tiny.solve(Bt, tol=1e-10)
    assert stb == O_.ORC_OK and int(itb.max()) <= 8 < int(itcol.max())

    p32 = O_.Problem(2, (32, 32), inputs.harmonic((32, 32), 100.0))
    B32 = inputs.random_block(1024, 8, seed=6)
    _, itb, _ = p32.solve_block_cg(B32, tol=1e-10)
    _, itcol, _, _ = p32.solve(B32, tol=1e-10)
    assert int(itb.max()) <= int(itcol.max())


# ---------------------------------------------------------------------------
# Sec. 3.1 / Alg. 1: the norm of the Grassmann gradient, and the subspace checker
# ---------------------------------------------------------------------------

def _sine_basis(n, L, modes):
    """Discrete sine modes prod_k sqrt(2/L_k) sin(m_k pi x_k / L_k): orthonormal in the
    grid L2 inner product h^d sum_i u_i v_i (discrete orthogonality of the sine transform),
    eigenvectors of H_sigma = -kappa Lap_h + sigma (V = 0)."""
    xs = inputs.grid_coords(n, L)
    cols = []
    for m in modes:
        u = np.ones_like(xs[0])
        for k in range(len(n)):
            u = u * np.sqrt(2.0 / L[k]) * np.sin(m[k] * np.pi * xs[k] / L[k])
        cols.append(u)
    return np.asfortranarray(np.stack(cols, axis=1))


def _sine_eigs(n, L, kappa, sigma, modes):
    h = [L[k] / (n[k] + 1) for k in range(len(n))]
    return np.array([sigma + sum(4.0 * kappa / h[k] ** 2
                                 * np.sin(m[k] * np.pi * h[k] / (2.0 * L[k])) ** 2
                                 for k in range(len(n))) for m in modes])


@pytest.mark.parametrize("dim,n,L", [(2, (11, 9), (1.0, 1.7)), (3, (7, 6, 5), (1.3, 0.8, 1.1))])
def test_grad_norm_closed_form(oracle_mod, dim, n, L):
    """||grad_G E_G(U)|| = ||G U - U <G U, U>|| (Sec. 3.1; the stop test of Alg. 1) in the
    grid L2 norm.  For U = Phi C with Phi exact orthonormal eigenvectors of H_sigma
    (eigenvalues Lambda): G U = Phi Lambda^{-1} C, <G U, U> = C^T Lambda^{-1} C, so
      ||grad||^2 = ||Lambda^{-1} C - C C^T Lambda^{-1} C||_F^2,
    and for diagonal C = diag(c_i): sum_i c_i^2 (1 - c_i^2)^2 / lambda_i^2.  The box is not
    the unit box, so h^d != 1 and a dropped (or doubled) grid weight changes the value."""
    O = oracle_mod
    ng = int(np.prod(n))
    kappa, sigma = 0.5, 0.7
    prob = O.Problem(dim, n, np.zeros(ng), L=L, kappa=kappa, sigma=sigma)
    assert abs(prob.w - 1.0) > 0.05 and abs(np.sqrt(prob.w) - 1.0) > 0.02
    modes = [(1, 1, 1), (2, 1, 1), (1, 3, 2), (3, 2, 1)]
    Phi = _sine_basis(n, L, modes)
    lam = _sine_eigs(n, L, kappa, sigma, modes)
    np.testing.assert_allclose(prob.w * Phi.T @ Phi, np.eye(len(modes)), atol=1e-13)
    np.testing.assert_allclose(prob.apply(Phi), Phi * lam, atol=1e-11 * lam.max())
    # diagonal coefficients: the verdict's closed form with two scaled eigenvectors
    c = np.array([0.6, 1.3])
    U = np.asfortranarray(Phi[:, :2] * c)
    P = np.asfortranarray(Phi[:, :2] * (c / lam[:2]))
    ref = np.sqrt(np.sum(c**2 * (1 - c**2) ** 2 / lam[:2] ** 2))
    assert abs(O.grad_norm(prob, U, P) - ref) <= 1e-13 * ref
    # a general coefficient matrix mixing four modes into three columns
    rng = np.random.default_rng(7)
    C = rng.standard_normal((4, 3))
    U = np.asfortranarray(Phi @ C)
    Li = np.diag(1.0 / lam)
    P = np.asfortranarray(Phi @ Li @ C)
    ref = np.linalg.norm(Li @ C - C @ (C.T @ Li @ C))
    assert abs(O.grad_norm(prob, U, P) - ref) <= 1e-12 * ref
    # the norm the step reports (P from the oracle's own solve, exact mode)
    orc = O.Oracle(prob, U, direct=True)
    st = orc.step(0.5 * lam[0])
    assert abs(st.grad_norm - ref) <= 1e-10 * ref
    # at an invariant subspace with orthonormal coefficients the gradient vanishes
    Qo, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    U = np.asfortranarray(Phi @ Qo[:, :4])
    P = np.asfortranarray(Phi @ Li @ Qo[:, :4])
    assert O.grad_norm(prob, U, P) <= 1e-13 * np.linalg.norm(Li)


def test_subspace_sin_known_angles(oracle_mod):
    """sin of the largest principal angle.  span{e1, cos a e2 + sin a e3, cos b e4 + sin b e5}
    against span{e1, e2, e4} has principal angles 0, a, b; the checker must return
    max(sin a, sin b) (not a Frobenius sum, not a cosine), for any bases of the two spans
    (non-orthonormal, columns mixed), and 0 for equal spans."""
    O = oracle_mod
    m = 9
    e = np.eye(m)
    rng = np.random.default_rng(11)
    for a, b in [(0.3, 0.1), (0.05, 1.2), (1e-6, 2e-7)]:
        A = np.stack([e[0], np.cos(a) * e[1] + np.sin(a) * e[2],
                      np.cos(b) * e[3] + np.sin(b) * e[4]], axis=1)
        B = np.stack([e[0], e[1], e[3]], axis=1)
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))  # same rotation of both: angles kept
        G1 = rng.standard_normal((3, 3)) + 3 * np.eye(3)  # bases mixed and rescaled
        G2 = rng.standard_normal((3, 3)) + 3 * np.eye(3)
        ref = max(np.sin(a), np.sin(b))
        for AA, BB in [(A, B), (Q @ A @ G1, Q @ B @ G2), (B @ G2, A @ G1)]:
            s = O.subspace_sin(AA, BB)
            assert abs(s - ref) <= 1e-12 + 1e-9 * ref, (a, b, s, ref)
    A = rng.standard_normal((m, 4))
    assert O.subspace_sin(A, A @ (rng.standard_normal((4, 4)) + 4 * np.eye(4))) <= 1e-13
    # a vector outside the span gives sin = 1
    assert abs(O.subspace_sin(e[:, :2], e[:, [0, 5]]) - 1.0) <= 1e-14
