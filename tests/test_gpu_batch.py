"""GPU parity of grouped batches (qo_batch_* of the C ABI): a batch of independent
problems with uneven grids and N against the same problems stepped one by one through
single-instance handles and against the oracle, graph replays against eager execution,
and the error paths."""
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


def _tau(n, V, sigma, kappa=0.5):
    # 0.9 x a lower bound of lambda_1(H_sigma): min(V + sigma) + kappa (mu_x[0] + mu_y[0])
    mu = sum(4.0 * (m + 1) ** 2 * np.sin(np.pi / (2.0 * (m + 1))) ** 2 for m in n)
    return 0.9 * (float(np.min(V)) + sigma + kappa * mu)


def _problems():
    """Two grid groups, uneven N, ragged sizes (not multiples of 32)."""
    probs = []
    spec = [((32, 32), 4, 1), ((32, 32), 6, 2), ((48, 40), 5, 3), ((32, 32), 3, 4),
            ((48, 40), 2, 5)]
    for n, N, seed in spec:
        rng = np.random.default_rng(100 + seed)
        V = inputs.harmonic_wells(n, rng.uniform(50, 150), rng.uniform(0.3, 0.7, 2),
                                  rng.uniform(2, 8, 4), rng.uniform(0.05, 0.15, 4),
                                  rng.uniform(0.1, 0.9, (4, 2)))
        sigma = max(0.0, 1.0 - float(V.min()))
        U0 = inputs.random_block(n[0] * n[1], N, seed=seed)
        probs.append(dict(n=n, N=N, V=V, sigma=sigma, U0=U0, tau=_tau(n, V, sigma)))
    return probs


def _batch(B, probs, precond="fast_poisson", tol=1e-12, maxit=40, precision="fp64"):
    cfgs = [dict(dim=2, n=p["n"], N=p["N"], sigma=p["sigma"], pcg_tol=tol, pcg_maxit=maxit,
                 precond=precond, precision=precision) for p in probs]
    b = B.Batch(cfgs)
    for i, p in enumerate(probs):
        b.set_potential(i, p["V"])
        b.set_state(i, p["U0"])
    return b


@pytest.mark.parametrize("precond,maxit", [("fast_poisson", 40), ("jacobi", 400)])
def test_batch_matches_single_instances(torch, B, precond, maxit):
    """12 steps of a 5-instance batch (two grids, N = 2..6) against the same problems stepped
    by single-instance handles: energies within 1e-10 relative every step, states within
    1e-9 at the end (the two differ only in summation order: band heights and launch
    grouping)."""
    probs = _problems()
    K = 12
    b = _batch(B, probs, precond, maxit=maxit)
    ref = []
    for p in probs:
        s = B.Solver(2, p["n"], p["N"], sigma=p["sigma"], pcg_tol=1e-12, pcg_check=1,
                     precond=precond)
        s.set_potential(p["V"])
        s.set_state(B.as_block(p["U0"]))
        ref.append(s)
    try:
        taus = [p["tau"] for p in probs]
        for k in range(K):
            st = b.step(taus, use_graph=True)
            for i, p in enumerate(probs):
                r = ref[i].step(p["tau"])
                assert abs(st[i]["energy"] - r["energy"]) <= 1e-10 * abs(r["energy"]), (k, i)
                assert abs(st[i]["orth_err_fro"] - r["orth_err_fro"]) <= 1e-9 * max(
                    1.0, r["orth_err_fro"]), (k, i)
        for i in range(len(probs)):
            U = b.get_state(i)
            Ur = B.to_numpy(ref[i].get_state())
            assert np.max(np.abs(U - Ur)) <= 1e-9 * np.max(np.abs(Ur)), i
    finally:
        b.close()
        for s in ref:
            s.close()


def test_batch_graph_replay_equals_eager(torch, B):
    """Steps replayed from the captured graphs (each parity replayed three times, with host
    reads between replays, and re-captured when the iteration count adapts) give
    bit-identical states and statistics to the same steps run eagerly on the same batch
    (same tuned tiles) from the same starting states."""
    probs = _problems()
    taus = [p["tau"] for p in probs]
    b = _batch(B, probs)
    out = {}
    try:
        for mode in (False, True):
            for i, p in enumerate(probs):
                b.set_state(i, p["U0"])
            stats = [b.step(taus, use_graph=mode) for _ in range(6)]
            out[mode] = (stats, [b.get_state(i) for i in range(len(probs))])
    finally:
        b.close()
    (s0, u0), (s1, u1) = out[False], out[True]
    for a, c in zip(s0, s1):
        for i in range(len(probs)):
            assert a[i]["energy"] == c[i]["energy"] and a[i]["grad_norm"] == c[i]["grad_norm"]
            assert a[i]["pcg_iters"] == c[i]["pcg_iters"]
    for a, c in zip(u0, u1):
        assert np.array_equal(a, c)


def test_batch_matches_oracle(torch, B, oracle_mod):
    """One batch instance against the oracle's fast-Poisson step, 8 steps: energies within
    1e-10 relative, final state within 1e-8."""
    probs = _problems()
    p = probs[2]
    ref = oracle_mod.Oracle(oracle_mod.Problem(2, p["n"], p["V"], sigma=p["sigma"]), p["U0"],
                            tol=1e-12, precond="fast_poisson")
    b = _batch(B, probs)
    try:
        taus = [q["tau"] for q in probs]
        for _ in range(8):
            st = b.step(taus)
            a = ref.step(p["tau"])
            assert abs(st[2]["energy"] - a.energy) <= 1e-10 * abs(a.energy)
        U = b.get_state(2)
        assert np.max(np.abs(U - ref.U)) <= 1e-8 * np.max(np.abs(ref.U))
    finally:
        b.close()


def test_batch_tiles_and_errors(torch, B):
    """The tuned band height is a valid one per group; a solve cut short fails with
    QO_ERR_PCG_NOCONV; stepping before the state is set fails with QO_ERR_STATE; the
    one-reduction PCG form is refused."""
    probs = _problems()
    b = _batch(B, probs)
    try:
        for i, p in enumerate(probs):
            ty = b.tile(i)
            assert 1 <= ty <= p["n"][1]
    finally:
        b.close()
    b = _batch(B, probs, tol=1e-14, maxit=1)
    try:
        with pytest.raises(B.QOError, match="QO_ERR_PCG_NOCONV"):
            b.step([p["tau"] for p in probs])
    finally:
        b.close()
    cfgs = [dict(dim=2, n=(16, 16), N=2, precond="fast_poisson", pcg_maxit=30)]
    b = B.Batch(cfgs)
    try:
        b.set_potential(0, np.zeros(256))
        with pytest.raises(B.QOError, match="QO_ERR_STATE"):
            b.step([1.0])
    finally:
        b.close()
    with pytest.raises(B.QOError):
        B.Batch([dict(dim=2, n=(16, 16), N=2, pcg_variant=1)])


@pytest.mark.parametrize("precond,maxit", [("fast_poisson", 40), ("jacobi", 400)])
def test_batch_mixed_matches_fp64(torch, B, precond, maxit):
    """Mixed precision in a batch (FP32 PCG in restarted FP64 refinement rounds, fixed
    counts) against the same problems stepped in FP64 by single-instance handles, 12 steps
    at PCG tol 1e-12 on both sides: each solve meets the same FP64 residual test, so the
    two runs differ by solves that agree to the tolerance: energies within 1e-10 relative
    every step, final states within 1e-8.  Every solve needs at least two rounds (the FP32
    inner tolerance floor is 1e-5)."""
    probs = _problems()
    K = 12
    b = _batch(B, probs, precond, maxit=maxit, precision="mixed")
    ref = []
    for p in probs:
        s = B.Solver(2, p["n"], p["N"], sigma=p["sigma"], pcg_tol=1e-12, pcg_check=1,
                     precond=precond)
        s.set_potential(p["V"])
        s.set_state(B.as_block(p["U0"]))
        ref.append(s)
    try:
        taus = [p["tau"] for p in probs]
        for k in range(K):
            st = b.step(taus, use_graph=True)
            for i, p in enumerate(probs):
                r = ref[i].step(p["tau"])
                assert abs(st[i]["energy"] - r["energy"]) <= 1e-10 * abs(r["energy"]), (k, i)
                assert min(st[i]["refine_rounds"]) >= 2, (k, i)
        for i in range(len(probs)):
            U = b.get_state(i)
            Ur = B.to_numpy(ref[i].get_state())
            assert np.max(np.abs(U - Ur)) <= 1e-8 * np.max(np.abs(Ur)), i
    finally:
        b.close()
        for s in ref:
            s.close()


def test_batch_mixed_graph_equals_eager_and_noconv(torch, B):
    """Mixed precision: graph replays give bit-identical states and statistics to eager
    steps (same tuned tiles, same adapted counts); a solve whose rounds cannot reach the
    tolerance (one FP32 iteration per round, tol 1e-14) fails with QO_ERR_PCG_NOCONV."""
    probs = _problems()
    taus = [p["tau"] for p in probs]
    b = _batch(B, probs, precision="mixed")
    out = {}
    try:
        for mode in (False, True):
            for i, p in enumerate(probs):
                b.set_state(i, p["U0"])
            stats = [b.step(taus, use_graph=mode) for _ in range(6)]
            out[mode] = (stats, [b.get_state(i) for i in range(len(probs))])
    finally:
        b.close()
    (s0, u0), (s1, u1) = out[False], out[True]
    for a, c in zip(s0, s1):
        for i in range(len(probs)):
            assert a[i]["energy"] == c[i]["energy"]
            assert a[i]["pcg_iters"] == c[i]["pcg_iters"]
            assert a[i]["refine_rounds"] == c[i]["refine_rounds"]
    for a, c in zip(u0, u1):
        assert np.array_equal(a, c)
    b = _batch(B, probs, tol=1e-14, maxit=1, precision="mixed")
    try:
        with pytest.raises(B.QOError, match="QO_ERR_PCG_NOCONV"):
            b.step(taus)
    finally:
        b.close()


@pytest.mark.parametrize("what", ["state", "potential"])
def test_batch_reseed_after_warm_steps(torch, B, what):
    """Jacobi-PCG (cold solves need several times the warm-started count), pcg_maxit 400:
    6 graph-replayed steps, then one instance gets a new random state (or a new potential
    and a new state), then 6 more steps.  The cold solve after the re-seed must not run out
    of the adapted fixed count: every step succeeds and matches single-instance handles
    given the same inputs (energies 1e-10 relative, final states 1e-9)."""
    probs = _problems()
    taus = [p["tau"] for p in probs]
    b = _batch(B, probs, "jacobi", maxit=400)
    ref = []
    for p in probs:
        s = B.Solver(2, p["n"], p["N"], sigma=p["sigma"], pcg_tol=1e-12, pcg_check=1,
                     precond="jacobi")
        s.set_potential(p["V"])
        s.set_state(B.as_block(p["U0"]))
        ref.append(s)
    try:
        for _ in range(6):
            b.step(taus, use_graph=True)
            for i, p in enumerate(probs):
                ref[i].step(p["tau"])
        k = 1
        U1 = inputs.random_block(probs[k]["n"][0] * probs[k]["n"][1], probs[k]["N"], seed=77)
        if what == "potential":
            V1 = probs[k]["V"] + 0.5 * inputs.harmonic(probs[k]["n"], 40.0)
            b.set_potential(k, V1)
            ref[k].set_potential(V1)
        b.set_state(k, U1)
        ref[k].set_state(B.as_block(U1))
        for step in range(6):
            st = b.step(taus, use_graph=True)
            for i, p in enumerate(probs):
                r = ref[i].step(p["tau"])
                assert abs(st[i]["energy"] - r["energy"]) <= 1e-10 * abs(r["energy"]), (step, i)
        for i in range(len(probs)):
            U = b.get_state(i)
            Ur = B.to_numpy(ref[i].get_state())
            assert np.max(np.abs(U - Ur)) <= 1e-9 * np.max(np.abs(Ur)), i
    finally:
        b.close()
        for s in ref:
            s.close()


def _mix_subset():
    """From the benchmark's 128-instance mix (sides 64..256, N 8..64): the first instance of
    every side, and the second of side 256, so that the largest grid group holds two
    instances."""
    probs = inputs.batch_instances(128, 0)
    pick, seen = [], {}
    for i, p in enumerate(probs):
        s = p["n"][0]
        if seen.get(s, 0) < (2 if s == 256 else 1):
            seen[s] = seen.get(s, 0) + 1
            pick.append(i)
    assert sorted(seen) == [64, 96, 128, 192, 256] and seen[256] == 2
    out = []
    for i in pick:
        p = dict(probs[i])
        p["U0"] = inputs.random_block(p["n"][0] * p["n"][1], p["N"], seed=1000 + i)
        p["tau"] = _tau(p["n"], p["V"], p["sigma"])
        out.append(p)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_mix_subset_matches_single_instances(torch, B, precision):
    """Six instances of the benchmark's 128-instance mix (every side 64..256, two of side
    256; fast-Poisson, PCG tol 1e-12), 4 steps replayed from the captured graphs, against
    the same problems stepped in FP64 by single-instance handles: energies within 1e-10
    relative every step, final states within 1e-9 (FP64) or 1e-8 (mixed: the FP32 PCG in
    FP64 refinement meets the same residual test, so the runs differ by solves that agree
    to the tolerance)."""
    probs = _mix_subset()
    K = 4
    b = _batch(B, probs, "fast_poisson", maxit=60, precision=precision)
    ref = []
    for p in probs:
        s = B.Solver(2, p["n"], p["N"], sigma=p["sigma"], pcg_tol=1e-12, pcg_check=1,
                     precond="fast_poisson")
        s.set_potential(p["V"])
        s.set_state(B.as_block(p["U0"]))
        ref.append(s)
    try:
        taus = [p["tau"] for p in probs]
        for k in range(K):
            st = b.step(taus, use_graph=True)
            for i, p in enumerate(probs):
                r = ref[i].step(p["tau"])
                assert abs(st[i]["energy"] - r["energy"]) <= 1e-10 * abs(r["energy"]), (k, i)
        tol = 1e-9 if precision == "fp64" else 1e-8
        for i, p in enumerate(probs):
            U = b.get_state(i)
            Ur = B.to_numpy(ref[i].get_state())
            err = np.max(np.abs(U - Ur)) / np.max(np.abs(Ur))
            print(f"[{precision}] side {p['n'][0]} N {p['N']}: state difference {err:.2e}")
            assert err <= tol, i
    finally:
        b.close()
        for s in ref:
            s.close()
