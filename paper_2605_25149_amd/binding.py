"""ctypes binding of libqo_hip.so (argument marshalling only).

Every computation runs in the HIP library; this module converts arguments and
owns nothing but the handle.  PyTorch provides device memory and the stream.

Block convention: a block of ``ncols`` grid functions is a float64 CUDA tensor
of shape ``(ncols, Ng)`` whose rows are contiguous (``stride(1) == 1``); row j
is column j of the column-major Ng x ncols block of the C ABI and
``stride(0)`` is its leading dimension.  ``as_block`` / ``to_numpy`` convert
from / to NumPy ``(Ng, ncols)`` arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqo_hip.so")

QO_OK, QO_ERR_ARG, QO_ERR_ALLOC, QO_ERR_DEVICE, QO_ERR_STATE = 0, 1, 2, 3, 4
QO_ERR_NOT_SPD, QO_ERR_PCG_NOCONV, QO_ERR_NONFINITE = 5, 6, 7
QO_FP64, QO_MIXED = 0, 1
QO_EIG_RITZ, QO_EIG_PAPER = 0, 1
BLOCKS = {"U": 0, "U_hat": 1, "P": 2, "Q": 3}
MATRICES = {"S": 0, "M": 1, "R": 2, "X": 3, "Y": 4, "O": 5, "A": 6, "B": 7}

EXPORTS = [
    "qo_create", "qo_set_potential", "qo_set_state", "qo_get_state", "qo_step", "qo_energy",
    "qo_gram", "qo_eigenpairs", "qo_destroy", "qo_status_string", "qo_last_error", "qo_apply",
    "qo_solve", "qo_gram_pair", "qo_get_block", "qo_get_matrix", "qo_profile", "qo_profile_get",
    "qo_run", "qo_eigsum_gradient", "qo_precond", "qo_tape_forward", "qo_tape_backward",
    "qo_energy_mode",
    "qo_batch_create", "qo_batch_set_potential", "qo_batch_set_state", "qo_batch_get_state",
    "qo_batch_step", "qo_batch_tile", "qo_batch_destroy", "qo_batch_last_error",
    "qo_gram_pair_noalloc", "qo_get_checkpoint", "qo_set_checkpoint", "qo_tape_budget",
]
KERNELS = ["sweep1_f64", "sweep2_f64", "sweep1_f32", "sweep2_f32", "gram", "update", "resid",
           "cg_f64", "cg_f32", "dst_fwd", "dst_pencil", "dst_inv"]
PRECONDS = {"jacobi": 0, "fast_poisson": 1}


class QoConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3),
        ("kinetic", ctypes.c_double), ("N", ctypes.c_int), ("sigma", ctypes.c_double),
        ("pcg_tol", ctypes.c_double), ("pcg_maxit", ctypes.c_int), ("pcg_check", ctypes.c_int),
        ("precision", ctypes.c_int), ("refine_inner_tol", ctypes.c_double),
        ("warm_start", ctypes.c_int), ("pcg_variant", ctypes.c_int),
        ("precond", ctypes.c_int),
    ]


class QoStepStats(ctypes.Structure):
    _fields_ = [
        ("energy", ctypes.c_double), ("energy_shifted", ctypes.c_double),
        ("orth_err_fro", ctypes.c_double), ("grad_norm", ctypes.c_double),
        ("pcg_iters", ctypes.c_int * 2), ("refine_rounds", ctypes.c_int * 2),
        ("energy_rose", ctypes.c_int), ("step_index", ctypes.c_int),
        ("orth_err_next", ctypes.c_double), ("t_phase_ms", ctypes.c_double * 8),
    ]

    def as_dict(self):
        return {
            "energy": self.energy, "energy_shifted": self.energy_shifted,
            "orth_err_fro": self.orth_err_fro, "grad_norm": self.grad_norm,
            "pcg_iters": tuple(self.pcg_iters), "refine_rounds": tuple(self.refine_rounds),
            "energy_rose": bool(self.energy_rose), "step_index": self.step_index,
            "orth_err_next": self.orth_err_next,
            "t_phase_ms": tuple(self.t_phase_ms),
        }


class QoCheckpoint(ctypes.Structure):
    _fields_ = [("step_index", ctypes.c_long), ("has_warm", ctypes.c_int),
                ("has_energy", ctypes.c_int), ("energy_shifted", ctypes.c_double),
                ("has_K", ctypes.c_int)]


class QoProfileData(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_long * 12), ("ms", ctypes.c_double * 12),
                ("work", ctypes.c_double * 12)]


class QOError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqo_hip.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the HIP library is the only compute path)")
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    H = ctypes.c_void_p
    sig = {
        "qo_create": ([ctypes.POINTER(QoConfig), vp, ctypes.POINTER(H)], ctypes.c_int),
        "qo_set_potential": ([H, vp, ctypes.c_int], ctypes.c_int),
        "qo_set_state": ([H, vp, ctypes.c_long, ctypes.c_int], ctypes.c_int),
        "qo_get_state": ([H, vp, ctypes.c_long, ctypes.c_int], ctypes.c_int),
        "qo_get_checkpoint": ([H, vp, vp, ctypes.c_long, vp, ctypes.c_int,
                               ctypes.POINTER(QoCheckpoint)], ctypes.c_int),
        "qo_set_checkpoint": ([H, vp, vp, ctypes.c_long, vp, ctypes.c_int,
                               ctypes.POINTER(QoCheckpoint)], ctypes.c_int),
        "qo_step": ([H, ctypes.c_double, ctypes.c_int, ctypes.POINTER(QoStepStats)], ctypes.c_int),
        "qo_energy": ([H, dp, dp], ctypes.c_int),
        "qo_gram": ([H, vp, vp], ctypes.c_int),
        "qo_eigenpairs": ([H, ctypes.c_int, vp, vp, ctypes.c_long, ctypes.c_int], ctypes.c_int),
        "qo_destroy": ([H], ctypes.c_int),
        "qo_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "qo_last_error": ([H], ctypes.c_char_p),
        "qo_apply": ([H, vp, vp, ctypes.c_long, ctypes.c_int], ctypes.c_int),
        "qo_solve": ([H, vp, vp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ip], ctypes.c_int),
        "qo_gram_pair": ([H, vp, vp, ctypes.c_long, ctypes.c_int, vp], ctypes.c_int),
        "qo_get_block": ([H, ctypes.c_int, vp, ctypes.c_long, ctypes.c_int], ctypes.c_int),
        "qo_get_matrix": ([H, ctypes.c_int, vp], ctypes.c_int),
        "qo_profile": ([H, ctypes.c_int], ctypes.c_int),
        "qo_eigsum_gradient": ([H, vp, ctypes.c_int], ctypes.c_int),
        "qo_run": ([H, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double, ip,
                    dp, ip, ctypes.POINTER(QoStepStats)], ctypes.c_int),
        "qo_profile_get": ([H, ctypes.POINTER(QoProfileData)], ctypes.c_int),
        "qo_precond": ([H, vp, vp, ctypes.c_long, ctypes.c_int, vp], ctypes.c_int),
        "qo_tape_forward": ([H, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp], ctypes.c_int),
        "qo_tape_budget": ([H, ctypes.c_int], ctypes.c_int),
        "qo_energy_mode": ([H, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "qo_tape_backward": ([H, ctypes.c_double, vp, vp, ctypes.c_long, ctypes.c_int],
                             ctypes.c_int),
        "qo_batch_create": ([ctypes.POINTER(QoConfig), ctypes.c_int, vp, ctypes.POINTER(H)],
                            ctypes.c_int),
        "qo_batch_set_potential": ([H, ctypes.c_int, vp, ctypes.c_int], ctypes.c_int),
        "qo_batch_set_state": ([H, ctypes.c_int, vp, ctypes.c_long, ctypes.c_int], ctypes.c_int),
        "qo_batch_get_state": ([H, ctypes.c_int, vp, ctypes.c_long, ctypes.c_int], ctypes.c_int),
        "qo_batch_step": ([H, vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(QoStepStats)],
                          ctypes.c_int),
        "qo_batch_tile": ([H, ctypes.c_int, ip], ctypes.c_int),
        "qo_batch_destroy": ([H], ctypes.c_int),
        "qo_batch_last_error": ([H], ctypes.c_char_p),
        "qo_gram_pair_noalloc": ([vp, vp, ctypes.c_long, ctypes.c_long, ctypes.c_int,
                                  ctypes.c_double, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def gram_pair_noalloc(X, Y, w, G, stream=None):
    """G = w [X | Y]^T [X | Y] through qo_gram_pair_noalloc (no allocation in the library).

    X, Y: blocks (ncols, ng) on the GPU with equal strides; G: a float64 CUDA tensor of
    (2 ncols)^2 elements that receives the column-major Gram matrix (symmetric, so its
    row-major view is the same matrix).  Enqueued on `stream` (default: torch's current
    stream); the call does not wait for the result."""
    import torch

    lib = load_library()
    ncols, ng = X.shape
    ld = _check_block(X, ng)
    if _check_block(Y, ng, ncols) != ld:
        raise ValueError("X and Y need the same shape and leading dimension")
    if G.dtype != torch.float64 or not G.is_cuda or not G.is_contiguous() or \
            G.numel() != 4 * ncols * ncols:
        raise ValueError("G must be a contiguous float64 CUDA tensor of (2 ncols)^2 values")
    st = stream if stream is not None else torch.cuda.current_stream()
    r = lib.qo_gram_pair_noalloc(ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                 ld, ng, ncols, float(w), ctypes.c_void_p(G.data_ptr()),
                                 ctypes.c_void_p(st.cuda_stream))
    if r != QO_OK:
        msg = lib.qo_last_error(None)
        raise QOError(r, msg.decode() if msg else "")
    return G


def _status_name(s):
    names = {0: "QO_OK", 1: "QO_ERR_ARG", 2: "QO_ERR_ALLOC", 3: "QO_ERR_DEVICE",
             4: "QO_ERR_STATE", 5: "QO_ERR_NOT_SPD", 6: "QO_ERR_PCG_NOCONV",
             7: "QO_ERR_NONFINITE"}
    return names.get(int(s), f"status {s}")


def as_block(a, device="cuda"):
    """NumPy (Ng, ncols) -> float64 CUDA tensor (ncols, Ng) in the ABI block layout."""
    import torch

    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device)


def to_numpy(t):
    """Block tensor (ncols, Ng) -> NumPy (Ng, ncols)."""
    return np.asfortranarray(t.detach().to("cpu").numpy().T)


def _check_block(t, ng, ncols=None):
    import torch

    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("blocks are float64 CUDA tensors of shape (ncols, Ng)")
    if t.dim() != 2 or t.shape[1] != ng or t.stride(1) != 1:
        raise ValueError(f"block must have shape (ncols, {ng}) with contiguous rows")
    if ncols is not None and t.shape[0] != ncols:
        raise ValueError(f"block must have {ncols} rows")
    return t.stride(0) if t.shape[0] > 1 else ng


def make_config(dim, n, N, L=(1.0, 1.0, 1.0), kinetic=0.5, sigma=0.0, pcg_tol=1e-10,
                pcg_maxit=20000, pcg_check=8, precision="fp64", refine_inner_tol=1e-5,
                warm_start=True, pcg_variant=0, precond="jacobi"):
    """A qo_config from keyword arguments."""
    cfg = QoConfig()
    cfg.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    LL = list(L) + [1.0] * (3 - len(L))
    for k in range(3):
        cfg.n[k] = int(nn[k])
        cfg.L[k] = float(LL[k])
    cfg.kinetic = kinetic
    cfg.N = N
    cfg.sigma = sigma
    cfg.pcg_tol = pcg_tol
    cfg.pcg_maxit = pcg_maxit
    cfg.pcg_check = pcg_check
    cfg.precision = {"fp64": QO_FP64, "mixed": QO_MIXED}[precision]
    cfg.refine_inner_tol = refine_inner_tol
    cfg.warm_start = 1 if warm_start else 0
    cfg.pcg_variant = int(pcg_variant)
    cfg.precond = PRECONDS[precond] if isinstance(precond, str) else int(precond)
    return cfg


class Solver:
    """One handle of the HIP library: grid, potential, iterate and workspace."""

    def __init__(self, dim, n, N, L=(1.0, 1.0, 1.0), kinetic=0.5, sigma=0.0, pcg_tol=1e-10,
                 pcg_maxit=20000, pcg_check=8, precision="fp64", refine_inner_tol=1e-5,
                 warm_start=True, pcg_variant=0, precond="jacobi", stream=None):
        import torch

        self.lib = load_library()
        nn = list(n) + [1] * (3 - len(n))
        cfg = make_config(dim, n, N, L, kinetic, sigma, pcg_tol, pcg_maxit, pcg_check,
                          precision, refine_inner_tol, warm_start, pcg_variant, precond)
        self.cfg = cfg
        self.dim, self.N = dim, N
        self.ng = int(np.prod(nn[:dim]))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = ctypes.c_void_p()
        st = self.lib.qo_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(self.h))
        if st != QO_OK:
            raise QOError(st, "qo_create failed")

    # -- plumbing
    def _chk(self, st):
        if st != QO_OK:
            msg = self.lib.qo_last_error(self.h)
            raise QOError(st, msg.decode() if msg else "")

    def close(self):
        if self.h:
            self.lib.qo_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- problem data
    def set_potential(self, V):
        import torch

        if isinstance(V, torch.Tensor):
            V = V.detach().to(dtype=torch.float64).contiguous()
            if V.numel() != self.ng:
                raise ValueError("potential must have Ng values")
            if V.is_cuda:
                self._chk(self.lib.qo_set_potential(self.h, ctypes.c_void_p(V.data_ptr()), 1))
                return
            V = V.numpy()
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1))
        if V.size != self.ng:
            raise ValueError("potential must have Ng values")
        self._chk(self.lib.qo_set_potential(self.h, V.ctypes.data_as(ctypes.c_void_p), 0))

    def set_state(self, U):
        """U: block tensor (N, Ng) or NumPy (Ng, N)."""
        if isinstance(U, np.ndarray):
            U = as_block(U)
        ld = _check_block(U, self.ng, self.N)
        self._chk(self.lib.qo_set_state(self.h, ctypes.c_void_p(U.data_ptr()), ld, 1))

    def get_state(self):
        import torch

        out = torch.empty((self.N, self.ng), dtype=torch.float64, device="cuda")
        self._chk(self.lib.qo_get_state(self.h, ctypes.c_void_p(out.data_ptr()), self.ng, 1))
        return out

    def get_checkpoint(self):
        """(U, warm or None, K or None, info dict): everything a resume reads."""
        import torch

        U = torch.empty((self.N, self.ng), dtype=torch.float64, device="cuda")
        W = torch.empty((self.N, self.ng), dtype=torch.float64, device="cuda")
        K = np.zeros((self.N, self.N), dtype=np.float64, order="F")
        ck = QoCheckpoint()
        self._chk(self.lib.qo_get_checkpoint(self.h, ctypes.c_void_p(U.data_ptr()),
                                             ctypes.c_void_p(W.data_ptr()), self.ng,
                                             K.ctypes.data_as(ctypes.c_void_p), 1,
                                             ctypes.byref(ck)))
        info = {"step_index": ck.step_index, "has_warm": ck.has_warm,
                "has_energy": ck.has_energy, "energy_shifted": ck.energy_shifted,
                "has_K": ck.has_K}
        return U, (W if ck.has_warm else None), (K if ck.has_K else None), info

    def set_checkpoint(self, U, warm, K, info):
        ld = _check_block(U, self.ng, self.N)
        wp = None
        if warm is not None:
            _check_block(warm, self.ng, self.N)
            if warm.stride(0) != ld:
                raise ValueError("U and warm must have the same leading dimension")
            wp = ctypes.c_void_p(warm.data_ptr())
        kp = None
        if K is not None:
            K = np.asfortranarray(np.asarray(K, dtype=np.float64))
            kp = K.ctypes.data_as(ctypes.c_void_p)
        ck = QoCheckpoint(int(info["step_index"]), int(info["has_warm"]),
                          int(info["has_energy"]), float(info["energy_shifted"]),
                          int(info["has_K"]))
        self._chk(self.lib.qo_set_checkpoint(self.h, ctypes.c_void_p(U.data_ptr()), wp, ld, kp,
                                             1, ctypes.byref(ck)))

    # -- the method
    def step(self, tau, nsteps=1):
        s = QoStepStats()
        self._chk(self.lib.qo_step(self.h, float(tau), int(nsteps), ctypes.byref(s)))
        return s.as_dict()

    def run(self, tau, max_steps, grad_tol=1e-5, tau_max=None):
        """Algorithm 1: steps until ||grad|| <= grad_tol (adaptive tau when tau_max is given).
        Returns (steps, tau_at_exit, converged, stats_of_last_step)."""
        s = QoStepStats()
        n, c = ctypes.c_int(), ctypes.c_int()
        t = ctypes.c_double()
        self._chk(self.lib.qo_run(self.h, float(tau), float(tau_max or 0.0), int(max_steps),
                                  float(grad_tol), ctypes.byref(n), ctypes.byref(t),
                                  ctypes.byref(c), ctypes.byref(s)))
        return n.value, t.value, bool(c.value), s.as_dict()

    def eigsum_gradient(self):
        """d(sum of the N Ritz values)/dV = h^d diag(U S^{-1} U^T), as a CUDA tensor (Ng,)."""
        import torch

        g = torch.empty(self.ng, dtype=torch.float64, device="cuda")
        self._chk(self.lib.qo_eigsum_gradient(self.h, ctypes.c_void_p(g.data_ptr()), 1))
        return g

    def energy_mode(self, mode, anchor=0):
        """0: stencil energy each step; 1: energy carried by the Gram identities, re-taken
        with the stencil every `anchor` steps (0: only at the start)."""
        self._chk(self.lib.qo_energy_mode(self.h, int(mode), int(anchor)))

    LOSSES = {"energy": 0, "ritz_sum": 1}

    def tape_budget(self, blocks):
        """Bound the tape to `blocks` state blocks (0: keep every state)."""
        self._chk(self.lib.qo_tape_budget(self.h, int(blocks)))

    def tape_forward(self, tau, K, loss="energy"):
        """K taped steps from the current state; returns the loss of U_K (energy, or the
        sum of the Ritz values)."""
        L = ctypes.c_double()
        self._chk(self.lib.qo_tape_forward(self.h, float(tau), int(K), self.LOSSES[loss],
                                           ctypes.byref(L)))
        return L.value

    def tape_backward(self, seed=1.0):
        """(seed dL/dV as a CUDA tensor (Ng,), seed dL/dU_0 as a block (N, Ng))."""
        import torch

        gV = torch.empty(self.ng, dtype=torch.float64, device="cuda")
        gU = torch.empty((self.N, self.ng), dtype=torch.float64, device="cuda")
        self._chk(self.lib.qo_tape_backward(self.h, float(seed), ctypes.c_void_p(gV.data_ptr()),
                                            ctypes.c_void_p(gU.data_ptr()), self.ng, 1))
        return gV, gU

    def energy(self):
        e, es = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.qo_energy(self.h, ctypes.byref(e), ctypes.byref(es)))
        return e.value, es.value

    def gram(self):
        S = np.zeros((self.N, self.N), order="F")
        K = np.zeros((self.N, self.N), order="F")
        self._chk(self.lib.qo_gram(self.h, S.ctypes.data_as(ctypes.c_void_p),
                                   K.ctypes.data_as(ctypes.c_void_p)))
        return S, K

    def eigenpairs(self, mode="ritz", vectors=False):
        import torch

        ev = np.zeros(self.N)
        m = {"ritz": QO_EIG_RITZ, "paper": QO_EIG_PAPER}[mode]
        vec = None
        vp = ctypes.c_void_p()
        if vectors:
            vec = torch.empty((self.N, self.ng), dtype=torch.float64, device="cuda")
            vp = ctypes.c_void_p(vec.data_ptr())
        self._chk(self.lib.qo_eigenpairs(self.h, m, ev.ctypes.data_as(ctypes.c_void_p), vp,
                                         self.ng, 1))
        return (ev, vec) if vectors else ev

    # -- kernel-level calls
    def apply(self, X, Y=None):
        import torch

        ld = _check_block(X, self.ng)
        if Y is None:
            Y = torch.empty_like(X)
        if _check_block(Y, self.ng, X.shape[0]) != ld:
            raise ValueError("X and Y need the same leading dimension")
        self._chk(self.lib.qo_apply(self.h, ctypes.c_void_p(X.data_ptr()),
                                    ctypes.c_void_p(Y.data_ptr()), ld, X.shape[0]))
        return Y

    def solve(self, B, X0=None):
        import torch

        ld = _check_block(B, self.ng)
        ncols = B.shape[0]
        if X0 is None:
            X = torch.zeros_like(B)
            use = 0
        else:
            X = X0.clone()
            use = 1
        if _check_block(X, self.ng, ncols) != ld:
            raise ValueError("B and X need the same leading dimension")
        its = (ctypes.c_int * max(ncols, 1))()
        self._chk(self.lib.qo_solve(self.h, ctypes.c_void_p(B.data_ptr()),
                                    ctypes.c_void_p(X.data_ptr()), ld, ncols, use, its))
        return X, np.array(its[:ncols])

    def precond(self, R):
        """(Z, rz): Z = M^{-1} R with the fast-Poisson preconditioner, rz = r.z per column."""
        import torch

        ld = _check_block(R, self.ng)
        ncols = R.shape[0]
        Z = torch.empty_like(R)
        if _check_block(Z, self.ng, ncols) != ld:
            raise ValueError("R must be a contiguous block")
        rz = np.zeros(ncols)
        self._chk(self.lib.qo_precond(self.h, ctypes.c_void_p(R.data_ptr()),
                                      ctypes.c_void_p(Z.data_ptr()), ld, ncols,
                                      rz.ctypes.data_as(ctypes.c_void_p)))
        return Z, rz

    def gram_pair(self, X, Y):
        ld = _check_block(X, self.ng)
        ncols = X.shape[0]
        if _check_block(Y, self.ng, ncols) != ld:
            raise ValueError("X and Y need the same shape and leading dimension")
        G = np.zeros((2 * ncols, 2 * ncols), order="F")
        self._chk(self.lib.qo_gram_pair(self.h, ctypes.c_void_p(X.data_ptr()),
                                        ctypes.c_void_p(Y.data_ptr()), ld, ncols,
                                        G.ctypes.data_as(ctypes.c_void_p)))
        return G

    def get_block(self, name):
        import torch

        out = torch.empty((self.N, self.ng), dtype=torch.float64, device="cuda")
        self._chk(self.lib.qo_get_block(self.h, BLOCKS[name], ctypes.c_void_p(out.data_ptr()),
                                        self.ng, 1))
        return out

    def profile(self, enable=True):
        """Turn per-kernel event timing on (clearing counters) or off."""
        self._chk(self.lib.qo_profile(self.h, 1 if enable else 0))

    def profile_data(self):
        d = QoProfileData()
        self._chk(self.lib.qo_profile_get(self.h, ctypes.byref(d)))
        return {k: {"launches": d.launches[i], "ms": d.ms[i], "work": d.work[i]}
                for i, k in enumerate(KERNELS)}

    def get_matrix(self, name):
        M = np.zeros((self.N, self.N), order="F")
        self._chk(self.lib.qo_get_matrix(self.h, MATRICES[name], M.ctypes.data_as(ctypes.c_void_p)))
        return M


class Batch:
    """Grouped batch of independent problems stepped together (qo_batch_* of the C ABI).

    ``configs``: a list of keyword dicts for ``make_config`` (one per instance)."""

    def __init__(self, configs, stream=None):
        self.lib = load_library()
        self.count = len(configs)
        arr = (QoConfig * self.count)()
        self.ng, self.N = [], []
        for i, kw in enumerate(configs):
            arr[i] = make_config(**kw)
            n = list(kw["n"])
            self.ng.append(int(np.prod(n[:kw["dim"]])))
            self.N.append(int(kw["N"]))
        self.cfgs = arr
        self.h = ctypes.c_void_p()
        sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else ctypes.c_void_p()
        st = self.lib.qo_batch_create(arr, self.count, sp, ctypes.byref(self.h))
        if st != QO_OK:
            raise QOError(st, "qo_batch_create failed")

    def _chk(self, st):
        if st != QO_OK:
            msg = self.lib.qo_batch_last_error(self.h)
            raise QOError(st, msg.decode() if msg else "")

    def close(self):
        if self.h:
            self.lib.qo_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_potential(self, i, V):
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1))
        if V.size != self.ng[i]:
            raise ValueError("potential size does not match the grid")
        self._chk(self.lib.qo_batch_set_potential(self.h, i, V.ctypes.data_as(ctypes.c_void_p), 0))

    def set_state(self, i, U):
        U = np.asfortranarray(np.asarray(U, dtype=np.float64))
        if U.shape != (self.ng[i], self.N[i]):
            raise ValueError("state must be Ng x N")
        self._chk(self.lib.qo_batch_set_state(self.h, i, U.ctypes.data_as(ctypes.c_void_p),
                                              self.ng[i], 0))

    def get_state(self, i):
        U = np.zeros((self.ng[i], self.N[i]), order="F")
        self._chk(self.lib.qo_batch_get_state(self.h, i, U.ctypes.data_as(ctypes.c_void_p),
                                              self.ng[i], 0))
        return U

    def step(self, taus=None, nsteps=1, use_graph=True, stats=True):
        t = None
        if taus is not None:
            t = np.ascontiguousarray(np.asarray(taus, dtype=np.float64).reshape(self.count))
        out = (QoStepStats * self.count)() if stats else None
        self._chk(self.lib.qo_batch_step(self.h, None if t is None else t.ctypes.data_as(
            ctypes.c_void_p), int(nsteps), 1 if use_graph else 0, out))
        return [o.as_dict() for o in out] if stats else None

    def tile(self, i):
        ty = ctypes.c_int()
        self._chk(self.lib.qo_batch_tile(self.h, i, ctypes.byref(ty)))
        return ty.value
