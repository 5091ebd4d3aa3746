"""GPU parity of the reverse mode through K steps (qo_tape_forward / qo_tape_backward of the
C ABI, reading R16) against the oracle's exact derivative, central differences of the
GPU's own forward, the Hellmann-Feynman limit, the autograd bridge and the error paths.

Tolerances: the GPU solves to a relative residual of 1e-13 where the oracle solves
exactly; with cond(H_sigma) of a few hundred on these grids every solve then carries a
relative error near 1e-11, and K steps plus the 2K adjoint solves keep the derivative
within 1e-9 of the oracle's (relative to its largest entry)."""
import ctypes

import numpy as np
import pytest

from paper_2605_25149_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-13


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


def _problem(dim, n, seed=3):
    if dim == 2:
        V = inputs.harmonic(n, 100.0) + inputs.gaussian_wells(n, seed=seed, depth=(1.0, 4.0))
    else:
        V = inputs.harmonic(n, 60.0) + inputs.gaussian_wells(n, seed=seed, depth=(1.0, 4.0))
    return V


CASES = [
    # dim, n, N, tau, K, precond: ragged sides (not multiples of the tile sizes)
    (2, (20, 17), 3, 8.0, 1, "jacobi"),
    (2, (20, 17), 3, 8.0, 5, "fast_poisson"),
    (2, (33, 31), 5, 6.0, 3, "jacobi"),
    (3, (12, 10, 9), 4, 6.0, 3, "fast_poisson"),
]


@pytest.mark.parametrize("loss", ["energy", "ritz_sum"])
@pytest.mark.parametrize("dim,n,N,tau,K,precond", CASES)
def test_tape_matches_oracle(torch, B, oracle_mod, dim, n, N, tau, K, precond, loss):
    """L, dL/dV and dL/dU_0 element by element against the oracle's reverse mode with
    exact solves: L within 1e-11 relative, gradients within 1e-9 of the largest entry."""
    V = _problem(dim, n)
    ng = int(np.prod(n))
    U0 = inputs.random_block(ng, N, seed=2)
    prob = oracle_mod.Problem(dim, n, V, sigma=0.3)
    Lr, gVr, gUr = oracle_mod.steps_loss_grad(prob, U0, tau, K, loss)
    with B.Solver(dim, n, N, sigma=0.3, pcg_tol=TOL, pcg_check=1, precond=precond) as s:
        s.set_potential(V)
        s.set_state(U0)
        L = s.tape_forward(tau, K, loss)
        gV, gU = s.tape_backward()
        gV = gV.cpu().numpy()
        gU = B.to_numpy(gU)
    print(f"L {L:.15e} oracle {Lr:.15e}; |gV| {np.max(np.abs(gVr)):.3e} "
          f"err {np.max(np.abs(gV - gVr)):.3e}; |gU| {np.max(np.abs(gUr)):.3e} "
          f"err {np.max(np.abs(gU - gUr)):.3e}")
    assert abs(L - Lr) <= 1e-11 * abs(Lr)
    assert np.max(np.abs(gV - gVr)) <= 1e-9 * np.max(np.abs(gVr))
    assert np.max(np.abs(gU - gUr)) <= 1e-9 * np.max(np.abs(gUr))


@pytest.mark.parametrize("loss", ["energy", "ritz_sum"])
def test_tape_directional_fd_of_gpu_forward(torch, B, loss):
    """<dL/dV, dV> and <dL/dU_0, dU_0> against central differences of the GPU's own
    forward (eps = 1e-5; solve noise 1e-13 / eps keeps the difference quotient good to
    about 1e-7 relative), two random directions each."""
    dim, n, N, tau, K = 2, (24, 21), 4, 8.0, 4
    V = _problem(dim, n)
    ng = int(np.prod(n))
    U0 = inputs.random_block(ng, N, seed=5)
    rng = np.random.default_rng(9)
    eps = 1e-5
    with B.Solver(dim, n, N, sigma=0.3, pcg_tol=TOL, pcg_check=1,
                  precond="fast_poisson") as s:
        def f(VV, UU):
            s.set_potential(VV)
            s.set_state(UU)
            return s.tape_forward(tau, K, loss)

        L = f(V, U0)
        gV, gU = s.tape_backward()
        gV, gU = gV.cpu().numpy(), B.to_numpy(gU)
        for _ in range(2):
            dV = rng.standard_normal(ng)
            dU = rng.standard_normal((ng, N))
            fdV = (f(V + eps * dV, U0) - f(V - eps * dV, U0)) / (2 * eps)
            fdU = (f(V, U0 + eps * dU) - f(V, U0 - eps * dU)) / (2 * eps)
            print(f"V: {gV @ dV:.12e} fd {fdV:.12e}; U0: {np.sum(gU * dU):.12e} fd {fdU:.12e}")
            assert abs(gV @ dV - fdV) <= 1e-6 * abs(fdV) + 1e-9 * abs(L)
            assert abs(np.sum(gU * dU) - fdU) <= 1e-6 * abs(fdU) + 1e-9 * abs(L)


def test_tape_hellmann_feynman_limit(torch, B, oracle_mod):
    """After 80 steps from a random block the derivative of the Ritz sum w.r.t. V is the
    Hellmann-Feynman gradient sum_i h^d phi_i(x_j)^2 of lambda_1 + ... + lambda_N
    (eigenvectors of the dense H_sigma from numpy's eigh) within 1e-6 of its largest entry,
    and dL/dU_0 has died out.  The frozen-U expression h^d diag(U S^{-1} U^T) at U_K
    (qo_eigsum_gradient) is first order in the subspace error and lags: only 1e-4 there."""
    n, N = (12, 10), 3
    V = inputs.harmonic(n, 100.0)
    U0 = inputs.random_block(120, N, seed=2)
    H = oracle_mod.Problem(2, n, V).sparse_matrix().toarray()
    _, phi = np.linalg.eigh(H)
    hf = np.sum(phi[:, :N] ** 2, axis=1)
    with B.Solver(2, n, N, pcg_tol=TOL, pcg_check=1, precond="fast_poisson") as s:
        s.set_potential(V)
        s.set_state(U0)
        s.tape_forward(10.0, 80, "ritz_sum")
        gV, gU = s.tape_backward()
        hfK = s.eigsum_gradient().cpu().numpy()
        gV, gU = gV.cpu().numpy(), B.to_numpy(gU)
    print(f"total derivative vs HF {np.max(np.abs(gV - hf)):.3e}; "
          f"frozen-U vs HF {np.max(np.abs(hfK - hf)):.3e}; max {np.max(hf):.3e}")
    assert np.max(np.abs(gV - hf)) <= 1e-6 * np.max(hf)
    assert np.max(np.abs(hfK - hf)) <= 1e-4 * np.max(hf)
    assert np.max(np.abs(gU)) <= 1e-6


def test_tape_state_autograd_and_errors(torch, B):
    """The state after qo_tape_backward is U_K bit for bit and stepping continues; the
    autograd bridge returns the ABI's gradients times the incoming seed (to rounding); the
    error paths:
    backward before forward (QO_ERR_STATE), mixed precision and a bad loss id (QO_ERR_ARG)."""
    from paper_2605_25149_amd import autograd

    n, N, tau, K = (20, 17), 3, 8.0, 3
    V = _problem(2, n)
    U0 = inputs.random_block(340, N, seed=2)
    with B.Solver(2, n, N, sigma=0.3, pcg_tol=TOL, pcg_check=1, precond="fast_poisson") as s:
        s.set_potential(V)
        with pytest.raises(B.QOError, match="QO_ERR_STATE"):
            s.tape_backward()
        s.set_state(U0)
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s._chk(s.lib.qo_tape_forward(s.h, 1.0, 1, 7, ctypes.byref(ctypes.c_double())))
        L = s.tape_forward(tau, K, "energy")
        UK = s.get_state().clone()
        gV, gU = s.tape_backward()
        assert torch.equal(s.get_state(), UK)
        s.step(tau)
        Vt = torch.tensor(V, dtype=torch.float64, device="cuda", requires_grad=True)
        Ut = B.as_block(U0).requires_grad_(True)
        Lt = autograd.steps_loss(Vt, Ut, s, tau, K, "energy")
        assert Lt.item() == L
        (2.5 * Lt).backward()
        # the seed enters at the loss gradient, so only the rounding differs
        assert torch.allclose(Vt.grad, 2.5 * gV, rtol=1e-12, atol=1e-12 * gV.abs().max().item())
        assert torch.allclose(Ut.grad, 2.5 * gU, rtol=1e-12, atol=1e-12 * gU.abs().max().item())
        # a float32 potential: FP64 inside, gradient returned as float32
        Vf = torch.tensor(V, dtype=torch.float32, device="cuda", requires_grad=True)
        autograd.steps_loss(Vf, B.as_block(U0), s, tau, K, "energy").backward()
        assert Vf.grad.dtype == torch.float32
        assert torch.allclose(Vf.grad.double(), gV, rtol=1e-4, atol=1e-5 * gV.abs().max().item())
    with B.Solver(2, n, N, precision="mixed") as s:
        s.set_potential(V)
        s.set_state(U0)
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.tape_forward(tau, 1, "energy")


@pytest.mark.parametrize("loss", ["energy", "ritz_sum"])
def test_tape_full_size_directional(torch, B, loss):
    """The differentiation workload: 64^3 grid of Gaussian wells, N = 32, K = 50 taped steps
    with the fast-Poisson solver at tol 1e-13.  16 random directions (8 in V, 8 in U_0):
    the directional derivative against central differences of the GPU forward with step
    1e-4, within 1e-4 relative.  The difference quotient carries the solves' noise: a
    perturbation can move a column's stopping iteration, a jump in L of up to about
    tol * |L| that the quotient divides by 2e-4.  Measured: an absolute floor near 4e-6,
    so 1e-7 relative on most directions and 1e-5 on those whose derivative is small."""
    n, N, tau, K = (64, 64, 64), 32, 6.0, 50
    V = inputs.gaussian_wells(n, seed=0)
    sigma = max(0.0, 1.0 - float(V.min()))
    ng = 64 ** 3
    U0 = inputs.random_block(ng, N, seed=1)
    rng = np.random.default_rng(4)
    h = 1e-4
    with B.Solver(3, n, N, sigma=sigma, pcg_tol=1e-13, pcg_check=1,
                  precond="fast_poisson") as s:
        def f(VV, UU):
            s.set_potential(VV)
            s.set_state(UU)
            return s.tape_forward(tau, K, loss)

        L = f(V, U0)
        gV, gU = s.tape_backward()
        gV, gU = gV.cpu().numpy(), B.to_numpy(gU)
        worst = 0.0
        for _ in range(8):
            dV = rng.standard_normal(ng)
            dU = rng.standard_normal((ng, N))
            fdV = (f(V + h * dV, U0) - f(V - h * dV, U0)) / (2 * h)
            fdU = (f(V, U0 + h * dU) - f(V, U0 - h * dU)) / (2 * h)
            rV = abs(gV @ dV - fdV) / abs(fdV)
            rU = abs(np.sum(gU * dU) - fdU) / abs(fdU)
            print(f"V: {gV @ dV:.10e} fd {fdV:.10e} ({rV:.1e}); "
                  f"U0: {np.sum(gU * dU):.10e} fd {fdU:.10e} ({rU:.1e})")
            worst = max(worst, rV, rU)
    print(f"L {L:.12e}; worst relative difference over 16 directions {worst:.2e}")
    assert worst <= 1e-4


@pytest.mark.parametrize("dim,n,K,budget,loss,precond", [
    (2, (20, 17), 11, 7, "ritz_sum", "fast_poisson"),  # stride 3, a partial last segment
    (3, (10, 9, 8), 9, 6, "energy", "jacobi"),         # stride 3, full segments
])
def test_tape_budget_is_bit_identical(torch, B, dim, n, K, budget, loss, precond):
    """qo_tape_budget: with the tape bounded to `budget` state blocks (checkpoints every
    s-th step plus one recomputed segment) the gradients w.r.t. V and U_0 and the loss are
    bit for bit those of the unbounded tape, and the state afterwards is U_K.  A bound too
    small for K steps is refused by qo_tape_forward, a bound of 1 or 2 by qo_tape_budget."""
    N, tau = 3, 8.0
    V = _problem(dim, n)
    ng = int(np.prod(n))
    U0 = inputs.random_block(ng, N, seed=2)
    out = []
    for b in (0, budget):
        with B.Solver(dim, n, N, sigma=0.3, pcg_tol=TOL, pcg_check=1, precond=precond) as s:
            s.set_potential(V)
            s.set_state(U0)
            s.tape_budget(b)
            L = s.tape_forward(tau, K, loss)
            UK = s.get_state().clone()
            gV, gU = s.tape_backward()
            assert torch.equal(s.get_state(), UK)
            out.append((L, gV.clone(), gU.clone(), UK))
    (L0, gV0, gU0, UK0), (L1, gV1, gU1, UK1) = out
    assert L0 == L1
    assert torch.equal(UK0, UK1)
    assert torch.equal(gV0, gV1)
    assert torch.equal(gU0, gU1)
    with B.Solver(dim, n, N, sigma=0.3, pcg_tol=TOL, pcg_check=1, precond=precond) as s:
        s.set_potential(V)
        s.set_state(U0)
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.tape_budget(2)
        s.tape_budget(3)
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.tape_forward(tau, K, loss)  # 3 blocks hold no stride for K >= 3
