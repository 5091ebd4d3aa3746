"""Reference (oracle) implementation of the quasi-orthogonal inverse-operator method.

TEST INFRASTRUCTURE ONLY.  A plain, slow, FP64 CPU implementation that the HIP
library is checked against.  It shares no code with the HIP path; only tests,
the smoke check and the benchmark's CPU-baseline leg use it.

Paper: S. Wang and A. Zhou, "A quasi-orthogonal method based on the inverse
operator for Schroedinger eigenvalue problems".  Section / equation references
below are to that paper:

  * Sec. 2.1   inner-product matrices <U,V>, <U,V>_a and the energy E(U)
  * Sec. 3.1   inverse operator G = (-Lap + V)^{-1} and the Grassmann gradient
  * Sec. 4.1   the two-stage scheme (predictor / corrector), the operator A_U,
               its Cayley form, and the auxiliary matrices O_n, A_n, B_n
  * Sec. 5     Algorithm 1 (the driver) and the error measures err_U, err_i

Discretisation (the paper uses quadratic finite elements; this build uses a
finite-difference grid): a grid function is a vector of interior values, the
L2 inner product is the mass-weighted sum (u,v) = h^d * sum_i u_i v_i with
h^d = prod(h_k), and the operator is H_sigma = -kappa*Lap_h + V + sigma.

Readings of the paper taken here (numbered as in the design notes' table of readings):
  R2  G is applied to a block by per-column PCG (``solve``: Jacobi preconditioner,
      Hestenes-Stiefel or Chronopoulos-Gear form; ``solve_fast_poisson``: reading R13);
      a direct sparse factorisation (``solve_direct``) is available for exact tests.
  R3  In A_U V = G U <U,V> - U <U, G V> the second term is evaluated with the
      symmetry of G as U <G U, V> = U <P, V>, P the computed G U, so A_U is
      exactly skew for the computed P and no solve with G V is needed.
  R4  The implicit predictor is solved exactly: since A_U maps into
      span{U, P}, U_hat = U X + P Y and the scheme reduces to a linear system
      for the coefficient matrices (``predictor``).
  R5  O_n in the corrector is the computed <U_hat, U_hat> - I (the literal
      second line of the scheme).
  R11 Warm starts: G U_n starts from the previous G U_hat; G U_hat starts from
      P (X + C Y) with C = <U,U>^{-1} <U,P> (exact when span U is invariant).
  R13 The paper leaves the solver of G open and its concluding section asks for a
      better preconditioner than the diagonal one.  ``solve_fast_poisson`` runs PCG
      with M = kappa*(-Lap_h) + vbar, vbar = max(0, mean(V + sigma)): the operator
      with V replaced by a constant, inverted exactly by the orthonormal type-I
      discrete sine transform, which diagonalises the 1-D Dirichlet second
      difference (``precond_apply``).  Only the iteration count depends on M.
  R19 Block CG (a variant of the solver of G, reading R2): O'Leary's block PCG with the
      Jacobi preconditioner over all N columns at once; converged columns are deflated
      (identity rows/columns in the s x s matrices, zero search directions); when the
      search block loses rank with columns still active (singular P^T H P, or no halving
      of the largest relative residual in 50 iterations) the column solver finishes.
  R20 The stop test of Alg. 1 measures grad_G E_G(U_n) = G U - U <G U, U> in the grid
      L2 norm (``grad_norm``); the algorithm does not name the norm.
  R16 The paper does not differentiate the scheme.  ``steps_loss_grad`` gives the
      exact derivative of the discrete K-step map (solves taken exact) composed
      with a loss of U_K (the energy, or the sum of the Ritz values), with respect
      to the potential V and the starting block U_0.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libqo_oracle.so")
_SRC_PATH = os.path.join(_HERE, "qo_oracle.c")
_lib = None

ORC_OK, ORC_NOT_SPD, ORC_NOCONV, ORC_NONFINITE = 0, 1, 2, 3


def build_lib(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH)
    ):
        import subprocess

        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC_PATH, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_apply.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_double,
                                  dp, dp, dp, ctypes.c_int]
        lib.orc_apply.restype = None
        lib.orc_quad.argtypes = lib.orc_apply.argtypes
        lib.orc_quad.restype = None
        lib.orc_pcg.argtypes = [ctypes.c_int, ip, dp, ctypes.c_double, ctypes.c_double,
                                dp, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, ip, ip]
        lib.orc_pcg.restype = ctypes.c_int
        lib.orc_pcg_variant.argtypes = lib.orc_pcg.argtypes + [ctypes.c_int]
        lib.orc_pcg_variant.restype = ctypes.c_int
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def threads(n=None):
    """OpenMP threads of the C part (set first when n is given); for timing records."""
    lib = _load()
    if n is not None:
        lib.orc_set_threads(int(n))
    return int(lib.orc_threads())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _fcols(X, ng):
    """Column-major (ng, ncols) FP64 view; columns contiguous."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X.reshape(ng, 1)
    return np.asfortranarray(X)


@dataclass
class Problem:
    """Discrete problem: grid, operator H_sigma = -kappa Lap_h + V + sigma (Sec. 2.1/2.2)."""

    dim: int
    n: tuple
    V: np.ndarray
    L: tuple = (1.0, 1.0, 1.0)
    kappa: float = 0.5
    sigma: float = 0.0
    h: np.ndarray = field(init=False)
    w: float = field(init=False)
    ng: int = field(init=False)

    def __post_init__(self):
        n = tuple(int(v) for v in self.n)[: self.dim]
        self.n = n
        self.h = np.array([self.L[k] / (n[k] + 1) for k in range(self.dim)], dtype=np.float64)
        # weight of the discrete L2 inner product (mass matrix of the FD grid)
        self.w = float(np.prod(self.h))
        self.ng = int(np.prod(n))
        self.V = np.ascontiguousarray(np.asarray(self.V, dtype=np.float64).reshape(self.ng))
        self._n3 = np.array(list(n) + [1] * (3 - self.dim), dtype=np.int32)
        self._h3 = np.array(list(self.h) + [1.0] * (3 - self.dim), dtype=np.float64)

    # ---- Sec. 2.1: inner-product matrices --------------------------------
    def inner(self, X, Y):
        """<X, Y> = ((x_i, y_j))_{ij} with the grid L2 inner product."""
        return self.w * (np.asarray(X).T @ np.asarray(Y))

    # ---- the operator and its inverse -----------------------------------
    def apply(self, X):
        """H_sigma X, column by column."""
        X = _fcols(X, self.ng)
        Y = np.empty_like(X, order="F")
        _load().orc_apply(self.dim, _ip(self._n3), _dp(self._h3), self.kappa, self.sigma,
                          _dp(self.V), _dp(X), _dp(Y), X.shape[1])
        return Y

    def quad(self, X):
        """x_j . (H_sigma x_j) per column (unweighted)."""
        X = _fcols(X, self.ng)
        out = np.empty(X.shape[1], dtype=np.float64)
        _load().orc_quad(self.dim, _ip(self._n3), _dp(self._h3), self.kappa, self.sigma,
                         _dp(self.V), _dp(X), _dp(out), X.shape[1])
        return out

    def solve(self, B, X0=None, tol=1e-10, maxit=10000, variant=0):
        """G B = H_sigma^{-1} B by per-column Jacobi-PCG (reading R2).

        variant 0: Hestenes-Stiefel form; 1: Chronopoulos-Gear (one-reduction) form.
        Returns (X, iters, status, col_status)."""
        B = _fcols(B, self.ng)
        if X0 is None:
            X = np.zeros_like(B, order="F")
            use_x0 = 0
        else:
            X = np.array(_fcols(X0, self.ng), order="F", copy=True)
            use_x0 = 1
        iters = np.zeros(B.shape[1], dtype=np.int32)
        cst = np.zeros(B.shape[1], dtype=np.int32)
        st = _load().orc_pcg_variant(self.dim, _ip(self._n3), _dp(self._h3), self.kappa,
                                     self.sigma, _dp(self.V), _dp(B), _dp(X), B.shape[1], tol,
                                     maxit, use_x0, _ip(iters), _ip(cst), int(variant))
        return X, iters, int(st), cst

    def diag(self):
        """Diagonal of H_sigma: V + sigma + sum_k 2 kappa / h_k^2."""
        return self.V + self.sigma + float(np.sum(2.0 * self.kappa / self.h ** 2))

    def solve_block_cg(self, B, X0=None, tol=1e-10, maxit=10000, stall=50):
        """G B by block PCG with the Jacobi preconditioner (O'Leary's block conjugate
        gradients; reading R19): one search block P for all columns, with the s x s
        coefficient matrices
            alpha = (P^T H P)^{-1} (Z^T R),   beta = (Z^T R)_old^{-1} (Z^T R)_new,
        X += P alpha, R -= H P alpha, Z = D^{-1} R, P = Z + P beta.  A column stops at the
        first iteration with ||r|| <= tol ||b|| (recursive residual) and is then deflated:
        its rows and columns of the s x s matrices become those of the identity and its
        Z column zero, so it no longer moves and no longer steers the others.
        The search block can lose rank while columns are still active (P^T H P singular,
        or the largest relative residual not halved in `stall` iterations); the remaining
        columns are then finished by the column solver (``solve``) from the current X.
        Returns (X, iters per column, status); iters of columns finished by the column
        solver add its count to the block iterations."""
        B = _fcols(B, self.ng)
        s = B.shape[1]
        X = np.zeros_like(B, order="F") if X0 is None else np.array(_fcols(X0, self.ng),
                                                                     order="F", copy=True)
        dinv = 1.0 / self.diag()
        bnorm = np.linalg.norm(B, axis=0)
        R = B - self.apply(X) if X0 is not None else B.copy(order="F")
        active = np.linalg.norm(R, axis=0) > tol * bnorm
        iters = np.zeros(s, dtype=np.int32)

        def masked(G, act):
            G = G.copy()
            G[~act, :] = 0.0
            G[:, ~act] = 0.0
            G[~act, ~act] = 1.0
            return G

        Z = R * dinv[:, None]
        Z[:, ~active] = 0.0
        P = Z.copy(order="F")
        rho = masked(Z.T @ R, active)
        k = 0
        best, kbest = np.inf, 0
        while active.any():
            if k >= maxit:
                return X, iters, ORC_NOCONV
            worst = float(np.max(np.linalg.norm(R[:, active], axis=0) / bnorm[active]))
            if worst < 0.5 * best:
                best, kbest = worst, k
            breakdown = k - kbest > stall
            if not breakdown:
                Q = self.apply(P)
                try:
                    alpha = np.linalg.solve(masked(P.T @ Q, active), rho)
                except np.linalg.LinAlgError:
                    breakdown = True
            if breakdown or not np.all(np.isfinite(alpha)):
                Xc, itc, st, _ = self.solve(B, X0=X, tol=tol, maxit=maxit - k)
                iters[active] = k + itc[active]
                return Xc, iters, st
            X += P @ alpha
            R -= Q @ alpha
            k += 1
            now = active & (np.linalg.norm(R, axis=0) > tol * bnorm)
            iters[active & ~now] = k
            if not np.all(np.isfinite(R)):
                return X, iters, ORC_NONFINITE
            Z = R * dinv[:, None]
            Z[:, ~now] = 0.0
            rho_new = masked(Z.T @ R, now)
            try:
                beta = np.linalg.solve(masked(rho, now), rho_new)
            except np.linalg.LinAlgError:
                Xc, itc, st, _ = self.solve(B, X0=X, tol=tol, maxit=maxit - k)
                iters[now] = k + itc[now]
                return Xc, iters, st
            P = Z + P @ beta
            rho = rho_new
            active = now
        return X, iters, ORC_OK

    # ---- fast-Poisson preconditioner (reading R13) ---------------------------
    def laplace_eigs(self):
        """Per axis k: eigenvalues of the 1-D Dirichlet second difference -d^2/dx^2,
        mu_k[j] = (4 / h_k^2) sin^2(pi (j+1) / (2 (n_k + 1))), j = 0..n_k-1; the
        eigenvector of mu_k[j] is sin(pi (j+1) (i+1) / (n_k + 1)) over i."""
        return [4.0 / self.h[k] ** 2 * np.sin(np.pi * np.arange(1, self.n[k] + 1)
                                              / (2.0 * (self.n[k] + 1))) ** 2
                for k in range(self.dim)]

    def precond_vbar(self):
        """vbar = max(0, mean(V + sigma)): keeps M = kappa (-Lap_h) + vbar SPD."""
        return max(0.0, float(np.mean(self.V)) + self.sigma)

    def precond_apply(self, R):
        """M^{-1} R per column, M = kappa (-Lap_h) + vbar: forward DST-I along every
        axis, division by lambda = kappa (mu_x + mu_y (+ mu_z)) + vbar, inverse
        DST-I (the orthonormal DST-I is its own inverse)."""
        import scipy.fft as sfft

        R = _fcols(R, self.ng)
        shape = tuple(reversed(self.n))  # x fastest: C-order (z, y, x)
        mu = self.laplace_eigs()
        lam = np.full(shape, self.precond_vbar())
        for k in range(self.dim):
            ax = self.dim - 1 - k
            sh = [1] * self.dim
            sh[ax] = self.n[k]
            lam = lam + self.kappa * mu[k].reshape(sh)
        Z = np.empty_like(R, order="F")
        for j in range(R.shape[1]):
            r = R[:, j].reshape(shape)
            rh = sfft.dstn(r, type=1, norm="ortho")
            Z[:, j] = sfft.idstn(rh / lam, type=1, norm="ortho").reshape(self.ng)
        return Z

    def solve_fast_poisson(self, B, X0=None, tol=1e-10, maxit=1000):
        """G B by per-column PCG with the fast-Poisson preconditioner (reading R13).

        Hestenes-Stiefel form: r = b - H x0; until ||r|| <= tol ||b||: z = M^{-1} r,
        rho = r.z, p = z + (rho / rho_prev) p, q = H p, alpha = rho / p.q,
        x += alpha p, r -= alpha q.  A column stops at the first iteration whose
        residual passes the test; iters counts the updates it took.
        Returns (X, iters, status, col_status) like ``solve``."""
        B = _fcols(B, self.ng)
        nc = B.shape[1]
        X = np.zeros_like(B, order="F") if X0 is None else np.array(_fcols(X0, self.ng),
                                                                    order="F", copy=True)
        R = B - self.apply(X) if X0 is not None else B.copy(order="F")
        bn = np.linalg.norm(B, axis=0)
        P = np.zeros_like(B, order="F")
        rho_prev = np.ones(nc)
        iters = np.zeros(nc, dtype=np.int32)
        cst = np.zeros(nc, dtype=np.int32)
        active = np.ones(nc, dtype=bool)
        for k in range(maxit + 1):
            rn = np.linalg.norm(R, axis=0)
            bad = active & ~(np.isfinite(rn))
            cst[bad] = ORC_NONFINITE
            active &= ~bad
            done = active & (rn <= tol * bn)
            iters[done] = k
            active &= ~done
            if not active.any():
                break
            if k == maxit:
                cst[active] = ORC_NOCONV
                iters[active] = k
                break
            cols = np.nonzero(active)[0]
            Z = self.precond_apply(R[:, cols])
            rho = np.einsum("ij,ij->j", R[:, cols], Z)
            beta = np.zeros(len(cols)) if k == 0 else rho / rho_prev[cols]
            P[:, cols] = Z + P[:, cols] * beta
            Q = self.apply(P[:, cols])
            gam = np.einsum("ij,ij->j", P[:, cols], Q)
            nspd = gam <= 0
            if nspd.any():
                cst[cols[nspd]] = ORC_NOT_SPD
                active[cols[nspd]] = False
            alpha = np.where(nspd, 0.0, rho / np.where(nspd, 1.0, gam))
            X[:, cols] += P[:, cols] * alpha
            R[:, cols] -= Q * alpha
            rho_prev[cols] = rho
        st = ORC_OK
        if (cst == ORC_NONFINITE).any():
            st = ORC_NONFINITE
        elif (cst == ORC_NOT_SPD).any():
            st = ORC_NOT_SPD
        elif (cst == ORC_NOCONV).any():
            st = ORC_NOCONV
        return X, iters, st, cst

    def sparse_matrix(self):
        """H_sigma as a scipy sparse matrix (Kronecker sum of 1-D second differences)."""
        import scipy.sparse as sp

        mats = []
        for k in range(self.dim):
            m = self.n[k]
            T = sp.diags([np.full(m - 1, -1.0), np.full(m, 2.0), np.full(m - 1, -1.0)],
                         [-1, 0, 1]) * (self.kappa / self.h[k] ** 2)
            mats.append(T.tocsr())
        H = sp.csr_matrix((self.ng, self.ng))
        for k in range(self.dim):
            left = sp.identity(int(np.prod(self.n[k + 1:])) if k + 1 < self.dim else 1)
            right = sp.identity(int(np.prod(self.n[:k])) if k > 0 else 1)
            # x fastest: axis 0 is the innermost Kronecker factor
            H = H + sp.kron(sp.kron(left, mats[k]), right)
        H = H + sp.diags(self.V + self.sigma)
        return H.tocsc()

    def solve_direct(self, B):
        """G B by a sparse LU factorisation (exact up to rounding)."""
        import scipy.sparse.linalg as spla

        if not hasattr(self, "_lu"):
            self._lu = spla.splu(self.sparse_matrix())
        B = _fcols(B, self.ng)
        return np.asfortranarray(self._lu.solve(np.ascontiguousarray(B)))

    # ---- Sec. 2.1 energy ---------------------------------------------------
    def energy(self, U):
        """(E(U), E_sigma(U)): E = 1/2 tr <U,U>_a with a(u,v) = (u, H v); E_sigma with H_sigma."""
        U = _fcols(U, self.ng)
        e_sigma = 0.5 * self.w * float(np.sum(self.quad(U)))
        e = e_sigma - 0.5 * self.sigma * float(np.trace(self.inner(U, U)))
        return e, e_sigma


# ---------------------------------------------------------------------------
# Sec. 4.1: the two stages of the scheme
# ---------------------------------------------------------------------------

def predictor(prob: Problem, U, P, tau):
    """First stage of the scheme: (U_hat - U)/tau = A_U U_tilde, U_tilde = (U_hat + U)/2.

    A_U V = P <U,V> - U <P,V> (reading R3) maps into span{U, P}, so
    U_hat = U X + P Y.  With U_tilde = U (X+I)/2 + P Y/2 the stage reads
        Y = tau <U, U_tilde>,   X = I - tau <P, U_tilde>.
    Writing X = I + tau b, Y = tau a and alpha = tau/2 this is the linear system
        (I - alpha M) a - alpha S b   = S
        alpha R a + (I + alpha M^T) b = -M^T
    with S = <U,U>, M = <U,P>, R = <P,P>.  Returns (U_hat, X, Y, (S, M, R))."""
    N = U.shape[1]
    S = prob.inner(U, U)
    M = prob.inner(U, P)
    R = prob.inner(P, P)
    alpha = 0.5 * tau
    I = np.eye(N)
    K = np.block([[I - alpha * M, -alpha * S], [alpha * R, I + alpha * M.T]])
    rhs = np.vstack([S, -M.T])
    sol = np.linalg.solve(K, rhs)
    a, b = sol[:N], sol[N:]
    X = I + tau * b
    Y = tau * a
    U_hat = np.asfortranarray(U @ X + P @ Y)
    return U_hat, X, Y, (S, M, R)


def corrector(prob: Problem, U_hat, Q, tau):
    """Second stage: U_{n+1} = U_hat - tau G U_hat (<U_hat,U_hat> - I), Q = G U_hat (reading R5).

    Returns (U_next, O, A, B) with O = <U_hat,U_hat> - I, A = <U_hat, Q>, B = <Q, Q>
    (the auxiliary matrices of Sec. 4.1; O equals O_n when the first stage preserves
    the Gram matrix)."""
    N = U_hat.shape[1]
    S_hat = prob.inner(U_hat, U_hat)
    S_hat = 0.5 * (S_hat + S_hat.T)
    O = S_hat - np.eye(N)
    A = prob.inner(U_hat, Q)
    Bm = prob.inner(Q, Q)
    U_next = np.asfortranarray(U_hat - tau * (Q @ O))
    return U_next, O, A, Bm


def grad_norm(prob: Problem, U, P):
    """|| grad_G E_G(U) || = || G U - U <G U, U> || (Sec. 3.1; the stop test of Alg. 1).

    Reading R20: Alg. 1 does not name the norm; it is taken as the grid L2 norm of the
    block, sqrt(h^d sum_{i,c} g_ic^2) -- the weighted Frobenius norm matching the inner
    product of Sec. 2.1 -- with P = G U the computed solve."""
    Mt = prob.inner(P, U)
    Gr = P - U @ Mt
    return float(np.sqrt(prob.w * np.sum(Gr * Gr)))


@dataclass
class StepStats:
    energy: float
    energy_shifted: float
    orth_err_fro: float
    grad_norm: float
    pcg_iters: tuple
    pcg_iters_cols: tuple = ()


class Oracle:
    """Algorithm 1 driver with a fixed time step (Sec. 5)."""

    def __init__(self, prob: Problem, U0, tol=1e-10, maxit=20000, warm_start=True,
                 direct=False, variant=0, precond="jacobi"):
        self.prob = prob
        self.U = np.array(_fcols(U0, prob.ng), order="F", copy=True)
        self.tol = tol
        self.maxit = maxit
        self.warm = warm_start
        self.direct = direct
        self.variant = variant
        self.precond = precond
        self.prevQ = None
        self.n = 0
        self.last = {}

    def _G(self, B, X0):
        if self.direct:
            return self.prob.solve_direct(B), np.zeros(B.shape[1], dtype=np.int32)
        if self.variant == 2:
            X, it, st = self.prob.solve_block_cg(B, X0=X0, tol=self.tol, maxit=self.maxit)
            if st != ORC_OK:
                raise RuntimeError(f"oracle block CG failed with status {st}")
            return X, it
        if self.precond == "fast_poisson":
            X, it, st, _ = self.prob.solve_fast_poisson(B, X0=X0, tol=self.tol,
                                                        maxit=min(self.maxit, 1000))
        else:
            X, it, st, _ = self.prob.solve(B, X0=X0, tol=self.tol, maxit=self.maxit,
                                           variant=self.variant)
        if st != ORC_OK:
            raise RuntimeError(f"oracle PCG failed with status {st}")
        return X, it

    def step(self, tau, grad_stop=None):
        """One step of the scheme; with grad_stop, return None (U_n kept) when
        ||grad_G E_G(U_n)|| <= grad_stop (the test of Alg. 1, taken before the update)."""
        prob, U = self.prob, self.U
        x0 = self.prevQ if (self.warm and self.prevQ is not None) else None
        P, itP = self._G(U, x0)
        gnorm = grad_norm(prob, U, P)
        if grad_stop is not None and gnorm <= grad_stop:
            self.prevQ = P
            return None
        U_hat, X, Y, (S, M, R) = predictor(prob, U, P, tau)
        x0Q = None
        if self.warm:
            C = np.linalg.solve(S, M)
            x0Q = np.asfortranarray(P @ (X + C @ Y))
        Q, itQ = self._G(U_hat, x0Q)
        U_next, O, A, Bm = corrector(prob, U_hat, Q, tau)
        self.last = dict(P=P, U_hat=U_hat, Q=Q, X=X, Y=Y, S=S, M=M, R=R, O=O, A=A, B=Bm,
                         U_prev=U)
        self.U = U_next
        self.prevQ = Q
        self.n += 1
        e, es = prob.energy(U_next)
        return StepStats(e, es, float(np.linalg.norm(O)), gnorm,
                         (int(itP.max(initial=0)), int(itQ.max(initial=0))),
                         (tuple(int(v) for v in itP), tuple(int(v) for v in itQ)))

    def run(self, tau, nsteps):
        return [self.step(tau) for _ in range(nsteps)]

    def algorithm1(self, tau, grad_tol, max_steps):
        """Alg. 1 with a fixed step: iterate while ||grad_G E_G(U_n)|| > grad_tol.
        Returns the number of steps taken and the statistics of the last one."""
        last = None
        for k in range(max_steps):
            st = self.step(tau, grad_stop=grad_tol)
            if st is None:
                return k, last
            last = st
        return max_steps, last


# ---------------------------------------------------------------------------
# Derivatives of K steps (reading R16)
# ---------------------------------------------------------------------------

def steps_loss(prob: Problem, U0, tau, K, loss="energy"):
    """K steps of the scheme (Sec. 4.1) with exact solves, then the loss of U_K:
    "energy": E(U_K) of Sec. 2.2; "ritz_sum": theta_1 + ... + theta_N of span U_K
    (= tr(<U,U>^{-1} <U, H U>)).  Returns (L, U_K, tape) with one record per step."""
    U = np.array(_fcols(U0, prob.ng), order="F", copy=True)
    tape = []
    for _ in range(K):
        P = prob.solve_direct(U)
        U_hat, X, Y, (S, M, R) = predictor(prob, U, P, tau)
        Q = prob.solve_direct(U_hat)
        U_next, O, _, _ = corrector(prob, U_hat, Q, tau)
        tape.append(dict(U=U, P=P, S=S, M=M, R=R, X=X, Y=Y, U_hat=U_hat, Q=Q, O=O))
        U = U_next
    return _loss(prob, U, loss), U, tape


def _loss(prob, U, loss):
    if loss == "energy":
        return prob.energy(U)[0]
    S = prob.inner(U, U)
    Kh = prob.inner(U, prob.apply(U))
    return float(np.trace(np.linalg.solve(S, Kh))) - U.shape[1] * prob.sigma


def _loss_grad(prob, U, loss):
    """(dL/dU, dL/dV) of the loss at fixed U.  With H = H_sigma - sigma:
    energy  L = w/2 tr(U^T H U):  dL/dU = w H U,  dL/dV_j = w/2 sum_c U_jc^2;
    ritz    L = tr(S^{-1} K), S = w U^T U, K = w U^T H_sigma U (minus N sigma):
            dL/dU = 2w (H_sigma U S^{-1} - U S^{-1} K S^{-1}),
            dL/dV_j = w (U S^{-1} U^T)_jj."""
    w = prob.w
    HU = prob.apply(U)
    if loss == "energy":
        return w * (HU - prob.sigma * U), 0.5 * w * np.sum(U * U, axis=1)
    S = prob.inner(U, U)
    Kh = prob.inner(U, HU)
    Si = np.linalg.inv(S)
    gU = 2.0 * w * (HU @ Si - U @ Si @ Kh @ Si)
    gV = w * np.sum((U @ Si) * U, axis=1)
    return gU, gV


def _predictor_adjoint(prob, S, M, R, tau, Xb, Yb):
    """Adjoint of the predictor's coefficient system (see ``predictor``): given dL/dX and
    dL/dY, return dL/dS, dL/dM, dL/dR.  The system is Kmat [a; b] = [S; -M^T] with
    Kmat = [[I - alpha M, -alpha S], [alpha R, I + alpha M^T]], X = I + tau b,
    Y = tau a.  For sol = Kmat^{-1} rhs: rhs_bar = Kmat^{-T} sol_bar and
    Kmat_bar = -rhs_bar sol^T."""
    N = S.shape[0]
    alpha = 0.5 * tau
    I = np.eye(N)
    Kmat = np.block([[I - alpha * M, -alpha * S], [alpha * R, I + alpha * M.T]])
    sol = np.linalg.solve(Kmat, np.vstack([S, -M.T]))
    sol_bar = np.vstack([tau * Yb, tau * Xb])
    rhs_bar = np.linalg.solve(Kmat.T, sol_bar)
    K_bar = -rhs_bar @ sol.T
    K11, K12 = K_bar[:N, :N], K_bar[:N, N:]
    K21, K22 = K_bar[N:, :N], K_bar[N:, N:]
    Sb = -alpha * K12 + rhs_bar[:N]
    Mb = -alpha * K11 + alpha * K22.T - rhs_bar[N:].T
    Rb = alpha * K21
    return Sb, Mb, Rb


def steps_loss_grad(prob: Problem, U0, tau, K, loss="energy"):
    """L of ``steps_loss`` and its exact derivatives dL/dV (Ng,) and dL/dU0 (Ng, N), by
    the chain rule taken backwards through the steps.  Per step, in reverse order:
      corrector U' = U_hat - tau Q O, O = sym<U_hat,U_hat> - I:
          Q_bar = -tau U'_bar O,  O_bar = -tau Q^T U'_bar,
          U_hat_bar = U'_bar + 2w U_hat sym(O_bar);
      Q = G U_hat (G = H_sigma^{-1} symmetric, dG/dV_j = -G e_j e_j^T G):
          U_hat_bar += G Q_bar,  V_bar_j -= sum_c (G Q_bar)_jc Q_jc;
      U_hat = U X + P Y:  U_bar = U_hat_bar X^T, P_bar = U_hat_bar Y^T,
          X_bar = U^T U_hat_bar, Y_bar = P^T U_hat_bar, then the predictor's adjoint;
      S = <U,U>, M = <U,P>, R = <P,P>:
          U_bar += w U (S_bar + S_bar^T) + w P M_bar^T,
          P_bar += w U M_bar + w P (R_bar + R_bar^T);
      P = G U:  U_bar += G P_bar,  V_bar_j -= sum_c (G P_bar)_jc P_jc."""
    L, UK, tape = steps_loss(prob, U0, tau, K, loss)
    w = prob.w
    Ub, Vb = _loss_grad(prob, UK, loss)
    for t in reversed(tape):
        U, P, Q, U_hat, O = t["U"], t["P"], t["Q"], t["U_hat"], t["O"]
        Qb = -tau * Ub @ O
        Ob = -tau * Q.T @ Ub
        Uhb = Ub + 2.0 * w * U_hat @ (0.5 * (Ob + Ob.T))
        W = prob.solve_direct(Qb)
        Uhb = Uhb + W
        Vb = Vb - np.sum(W * Q, axis=1)
        Un = Uhb @ t["X"].T
        Pb = Uhb @ t["Y"].T
        Sb, Mb, Rb = _predictor_adjoint(prob, t["S"], t["M"], t["R"], tau, U.T @ Uhb,
                                        P.T @ Uhb)
        Un = Un + w * U @ (Sb + Sb.T) + w * P @ Mb.T
        Pb = Pb + w * U @ Mb + w * P @ (Rb + Rb.T)
        W = prob.solve_direct(Pb)
        Ub = Un + W
        Vb = Vb - np.sum(W * P, axis=1)
    return L, Vb, np.asfortranarray(Ub)


# ---------------------------------------------------------------------------
# Sec. 5: eigenvalue read-out and error measures
# ---------------------------------------------------------------------------

def ritz(prob: Problem, U):
    """Rayleigh-Ritz on span U: K c = theta S c, K = <U, H_sigma U>, S = <U,U>.

    Returns (lambda ascending, coefficient matrix c); lambda = theta - sigma."""
    import scipy.linalg as sla

    U = _fcols(U, prob.ng)
    K = prob.inner(U, prob.apply(U))
    K = 0.5 * (K + K.T)
    S = prob.inner(U, U)
    S = 0.5 * (S + S.T)
    theta, c = sla.eigh(K, S)
    return theta - prob.sigma, c


def eigsum_gradient(prob: Problem, U):
    """d(theta_1 + ... + theta_N)/dV_j for the Ritz values of span U at fixed U:
    sum theta = tr(S^{-1} K) with K = <U, H U>, dK/dV_j = h^d u_j u_j^T (u_j = row j of U),
    so the derivative is h^d u_j^T S^{-1} u_j.  At an exact eigenbasis it is the
    Hellmann-Feynman derivative of lambda_1 + ... + lambda_N (eigenvalues of Sec. 2.2)."""
    U = np.asarray(U)
    S = prob.inner(U, U)
    Sinv = np.linalg.inv(0.5 * (S + S.T))
    return prob.w * np.einsum("ja,ab,jb->j", U, Sinv, U)


def paper_eigenvalues(prob: Problem, U, P):
    """lambda_i = eigenvalues of <G U, U>^{-1} (Sec. 5 definition of err_i), minus the shift."""
    T = prob.inner(P, U)
    T = 0.5 * (T + T.T)
    mu = np.linalg.eigvalsh(T)
    return np.sort(1.0 / mu) - prob.sigma


def err_eigen(lam, lam_ref):
    """err_i = |lambda_i - lambda_i^*| / |lambda_i^*| (Sec. 5)."""
    lam = np.asarray(lam, dtype=np.float64)
    lam_ref = np.asarray(lam_ref, dtype=np.float64)
    return np.abs(lam - lam_ref) / np.abs(lam_ref)


def err_state(Un, Uend):
    """err_U = ||U_n - U_end|| / ||U_end|| (Sec. 5)."""
    return float(np.linalg.norm(np.asarray(Un) - np.asarray(Uend)) / np.linalg.norm(Uend))


def subspace_sin(A, B):
    """sin of the largest principal angle between span A and span B (Euclidean)."""
    qa, _ = np.linalg.qr(np.asarray(A))
    qb, _ = np.linalg.qr(np.asarray(B))
    r = qb - qa @ (qa.T @ qb)
    return float(np.linalg.norm(r, 2))
