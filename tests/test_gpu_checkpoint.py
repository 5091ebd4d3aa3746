"""Checkpoint and resume through the C ABI (qo_get_checkpoint / qo_set_checkpoint): a run
that is stopped after k steps and resumed on a fresh handle from its checkpoint continues
bit for bit like the uninterrupted run (iterate, energies, gradient norm, orthogonality
error, iteration counts, step index and the energy_rose flag), in FP64 and mixed
precision, with either preconditioner, warm starts on, and in energy mode 1 (carried
K = <U, H_sigma U>).  qo_set_state (cold restart) is the contrast: it drops the warm
start, and in FP64 its next step is not the uninterrupted run's.  Error paths: a checkpoint that claims a
warm block or K without passing it, a negative step index and a non-finite warm block."""
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


CASES = [
    # dim, n, N, precision, precond, energy mode
    (3, (14, 12, 10), 6, "fp64", "fast_poisson", 0),
    (3, (14, 12, 10), 6, "mixed", "fast_poisson", 0),
    (2, (40, 36, 1), 5, "fp64", "jacobi", 1),
    (2, (40, 36, 1), 5, "mixed", "jacobi", 0),
]


def _stats_key(st):
    return (st["energy"], st["energy_shifted"], st["grad_norm"], st["orth_err_fro"],
            st["orth_err_next"], st["pcg_iters"], st["refine_rounds"], st["energy_rose"],
            st["step_index"])


@pytest.mark.parametrize("dim,n,N,precision,precond,emode", CASES)
def test_resume_is_bit_identical(torch, B, dim, n, N, precision, precond, emode):
    nn = n[:dim]
    ng = int(np.prod(nn))
    V = inputs.gaussian_wells(nn, seed=0) if dim == 3 else inputs.harmonic(nn, 100.0)
    U0 = inputs.random_block(ng, N, seed=1)
    tau, k1, k2 = 6.0, 3, 3
    kw = dict(pcg_tol=1e-10, precision=precision, precond=precond)

    with B.Solver(dim, nn, N, **kw) as a:
        a.set_potential(V)
        if emode:
            a.energy_mode(1, 0)
        a.set_state(U0)
        for _ in range(k1):
            a.step(tau)
        U, W, K, info = a.get_checkpoint()
        assert info["step_index"] == k1 and info["has_warm"] == 1 and info["has_energy"] == 1
        assert info["has_K"] == (1 if emode else 0)
        ref = [a.step(tau) for _ in range(k2)]
        Uref = a.get_state().clone()

    with B.Solver(dim, nn, N, **kw) as b:
        b.set_potential(V)
        if emode:
            b.energy_mode(1, 0)
        b.set_checkpoint(U, W, K, info)
        got = [b.step(tau) for _ in range(k2)]
        Ugot = b.get_state()
    assert torch.equal(Ugot, Uref), "resumed iterate differs from the uninterrupted run"
    for s_ref, s_got in zip(ref, got):
        assert _stats_key(s_got) == _stats_key(s_ref)

    # cold restart from the same U_k: the first solve starts from zero, so in FP64 the step
    # is not the uninterrupted run's (the solves agree only to their tolerance).  In mixed
    # precision the solution block enters the step only rounded (BF16 Grams, FP32 block
    # updates), which hides differences at the solve tolerance.
    with B.Solver(dim, nn, N, **kw) as c:
        c.set_potential(V)
        c.set_state(U)
        cold = c.step(tau)
    assert cold["step_index"] == 1
    if precision == "fp64":
        assert _stats_key(cold)[:7] != _stats_key(ref[0])[:7]


def test_checkpoint_errors(torch, B):
    n, N = (24, 20), 3
    V = inputs.harmonic(n, 100.0)
    U0 = inputs.random_block(480, N, seed=1)
    with B.Solver(2, n, N, pcg_tol=1e-10) as s:
        s.set_potential(V)
        with pytest.raises(B.QOError, match="QO_ERR_STATE"):
            s.get_checkpoint()
        s.set_state(U0)
        s.step(8.0, 2)
        U, W, K, info = s.get_checkpoint()
        assert W is not None and K is None
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.set_checkpoint(U, None, None, info)
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.set_checkpoint(U, W, None, dict(info, has_K=1))
        with pytest.raises(B.QOError, match="QO_ERR_ARG"):
            s.set_checkpoint(U, W, None, dict(info, step_index=-1))
        Wbad = W.clone()
        Wbad[1, 7] = float("nan")
        with pytest.raises(B.QOError, match="QO_ERR_NONFINITE"):
            s.set_checkpoint(U, Wbad, None, info)
        with pytest.raises(B.QOError, match="QO_ERR_STATE"):
            s.step(8.0)  # a failed restore leaves no state
        s.set_checkpoint(U, W, None, info)
        st = s.step(8.0)
        assert st["step_index"] == 3
