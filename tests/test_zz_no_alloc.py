"""The allocation-free Gram (qo_gram_pair_noalloc) against the allocating entry point
qo_gram_pair (FP64 path) on the same blocks, through the C ABI: two calls in a row, the
second with fewer rows and columns (and a padded leading dimension), both within 1e-13 of
the largest entry of qo_gram_pair's result and of the NumPy product; a size beyond the
maximum is rejected with QO_ERR_ARG and a message."""
import numpy as np
import pytest

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


def _case(torch, B, n, ncols, pad, seed):
    ng = n[0] * n[1]
    w = (1.0 / (n[0] + 1)) * (1.0 / (n[1] + 1))
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((ng, ncols))
    Y = rng.standard_normal((ng, ncols))
    ld = ng + pad
    Xd = torch.zeros((ncols, ld), dtype=torch.float64, device="cuda")
    Yd = torch.zeros((ncols, ld), dtype=torch.float64, device="cuda")
    Xd[:, :ng] = torch.from_numpy(X.T.copy()).cuda()
    Yd[:, :ng] = torch.from_numpy(Y.T.copy()).cuda()
    Xv, Yv = Xd[:, :ng], Yd[:, :ng]
    return X, Y, Xv, Yv, w, ng


def test_noalloc_gram_matches_gram_pair(torch, B):
    G = torch.empty(4 * 200 * 200, dtype=torch.float64, device="cuda")
    for n, ncols, pad, seed in [((512, 512), 200, 0, 1), ((17, 241), 37, 24, 2)]:
        X, Y, Xv, Yv, w, ng = _case(torch, B, n, ncols, pad, seed)
        print(f"noalloc Gram: grid {n}, ncols {ncols}, ld {ng + pad}", flush=True)
        Gv = G[: 4 * ncols * ncols]
        Gv.fill_(np.nan)  # every entry must be written by this call
        B.gram_pair_noalloc(Xv, Yv, w, Gv)
        torch.cuda.synchronize()
        g = Gv.cpu().numpy().reshape(2 * ncols, 2 * ncols).T  # column-major
        with B.Solver(2, n, ncols, pcg_variant=0) as s:
            g_ref = s.gram_pair(Xv, Yv)
        Z = np.hstack([X, Y])
        ref = w * (Z.T @ Z)
        assert np.all(np.isfinite(g))
        assert np.max(np.abs(g - g_ref)) <= 1e-13 * np.max(np.abs(g_ref))
        assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))
        assert np.array_equal(g, g.T)


def test_noalloc_gram_rejects_oversize(torch, B):
    X = torch.zeros((1025, 64), dtype=torch.float64, device="cuda")
    G = torch.zeros(4 * 1025 * 1025, dtype=torch.float64, device="cuda")
    with pytest.raises(B.QOError, match="QO_ERR_ARG.*ncols 1025"):
        B.gram_pair_noalloc(X, X, 1.0, G)
