"""Trajectory parity at the FP64 Jacobi configuration: 3-D 64^3 Gaussian wells
(Ng = 262,144; seed 0), N = 64, random start (seed 1), Jacobi PCG (two-sweep form) at
tol 1e-10 with warm starts, tau = 0.9 x the lowest eigenvalue of the same potential on a
32^3 grid.  The GPU and the oracle take the same 5 steps from the same inputs (the oracle
needs about 10 s per step on 16 host cores).

Per step: E and E_sigma within 1e-10 relative, ||O_n||_F within 1e-10, PCG iteration counts
equal (up to the threshold ties described in iters_agree).  After the last step: the state
within 1e-9 of the largest entry, the Ritz values (Rayleigh-Ritz on span U_5) within 1e-10
relative, and the largest principal angle between the two spans below 1e-8 (sine)."""
import numpy as np
import pytest

from paper_2605_25149_amd import inputs

pytestmark = pytest.mark.gpu

TAU = 0.9 * 10.0685
STEPS = 5


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


def _iters_agree(gpu, orc):
    gpu, orc = np.asarray(gpu).ravel(), np.asarray(orc).ravel()
    same = np.mean(gpu == orc)
    return same >= 0.90 and np.all(np.abs(gpu - orc) <= np.maximum(5, 0.05 * orc))


@pytest.mark.timeout(600)
def test_cfg2_trajectory_fp64_jacobi(torch, B, oracle_mod):
    n, N = (64, 64, 64), 64
    V = inputs.gaussian_wells(n, seed=0)
    U0 = inputs.random_block(int(np.prod(n)), N, seed=1)
    prob = oracle_mod.Problem(3, n, V)
    ref = oracle_mod.Oracle(prob, U0, tol=1e-10, warm_start=True, variant=0)
    with B.Solver(3, n, N, pcg_tol=1e-10, pcg_maxit=5000, pcg_check=8, pcg_variant=0,
                  precond="jacobi", warm_start=True) as s:
        s.set_potential(V)
        s.set_state(U0)
        rs, gs = [], []
        for k in range(STEPS):
            a = ref.step(TAU)
            g = s.step(TAU)
            print(f"cfg2 step {k + 1}: iterations gpu {g['pcg_iters']} oracle {a.pcg_iters}, "
                  f"E gpu {g['energy']:.15e} oracle {a.energy:.15e}", flush=True)
            rs.append(a)
            gs.append(g)
        U = B.to_numpy(s.get_state())
        lam = s.eigenpairs("ritz")
    for a, g in zip(rs, gs):
        assert abs(g["energy"] - a.energy) <= 1e-10 * abs(a.energy)
        assert abs(g["energy_shifted"] - a.energy_shifted) <= 1e-10 * abs(a.energy_shifted)
        assert abs(g["orth_err_fro"] - a.orth_err_fro) <= 1e-10 * max(1.0, a.orth_err_fro)
    assert _iters_agree([g["pcg_iters"] for g in gs], [a.pcg_iters for a in rs])
    assert np.max(np.abs(U - ref.U)) <= 1e-9 * np.max(np.abs(ref.U))
    lam_ref, _ = oracle_mod.ritz(prob, ref.U)
    np.testing.assert_allclose(lam, lam_ref, rtol=1e-10)
    sin = oracle_mod.subspace_sin(U, ref.U)
    print(f"cfg2: max Ritz rel diff {np.max(np.abs(lam - lam_ref) / np.abs(lam_ref)):.3e}, "
          f"subspace sine {sin:.3e}", flush=True)
    assert sin <= 1e-8
