"""FP64 host steps of Algorithm 1 that the paper assigns to the CPU (Sec. 3).

* reduced SVD of T: LAPACK for small N, the block power method with rank
  determination (Sec. 2.2, Algorithm 3) for large N, whose block products
  T X and T^* Y run on the GPU from the sample grid (prony_toeplitz_mm) while
  the QR factorisations and the small SVD stay on the host;
* eigendecomposition of the random combination C_mu and extraction of the
  nodes z_j, t_j (Algorithm 1, eigenvalue step);
* the m x m solve of the normal equations gram c = rhs formed on the GPU
  (Algorithm 1, coefficient step).

`solve` chains these with the GPU calls of `api` into Algorithm 1.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg
import torch

from . import api


def _orth(X: np.ndarray) -> np.ndarray:
    q, _ = np.linalg.qr(X)
    return q


class DenseToeplitz:
    """The operator interface of power_svd for an explicit matrix."""

    def __init__(self, T: np.ndarray):
        self.T = T

    def matmul(self, X: np.ndarray) -> np.ndarray:
        return self.T @ X

    def rmatmul(self, Y: np.ndarray) -> np.ndarray:
        return self.T.conj().T @ Y

    def fro_norm(self) -> float:
        return float(np.linalg.norm(self.T))


class GpuToeplitz:
    """T of the sample grid f (device tensor) as an operator: T X and T^* Y on the
    GPU without forming T (prony_toeplitz_mm); numpy blocks in and out."""

    def __init__(self, f: torch.Tensor, d: int, n: int, prec: str = "fp64"):
        self.f, self.d, self.n, self.prec = f, d, n, prec

    def _mm(self, X: np.ndarray, adjoint: bool) -> np.ndarray:
        Xd = torch.from_numpy(np.ascontiguousarray(X)).to(self.f.device)
        return api.toeplitz_mm(self.f, self.d, self.n, Xd, adjoint=adjoint, prec=self.prec).cpu().numpy()

    def matmul(self, X: np.ndarray) -> np.ndarray:
        return self._mm(X, False)

    def rmatmul(self, Y: np.ndarray) -> np.ndarray:
        return self._mm(Y, True)

    def fro_norm(self) -> float:
        """||T||_F^2 = sum_p |f(p)|^2 prod_l (n + 1 - |p_l|) over p in {-n..n}^d: every
        difference p = k - h occurs that many times in T."""
        n, d = self.n, self.d
        g = self.f.cpu().numpy().reshape((2 * n + 2,) * d)[(slice(0, 2 * n + 1),) * d]
        w1 = n + 1 - np.abs(np.arange(-n, n + 1))
        w = w1
        for _ in range(d - 1):
            w = np.multiply.outer(w, w1)
        return float(np.sqrt(np.sum(np.abs(g) ** 2 * w)))


def power_svd(T, start_u: np.ndarray, start_v: np.ndarray, tol: float, rank: int | None = None,
              max_sweeps: int = 60):
    """Block power SVD with pivoted-QR rank determination in the first sweep
    (Sec. 2.2, Algorithm 3). T is a matrix or an operator with matmul, rmatmul and
    fro_norm (GpuToeplitz). Returns (U, sigma, V, detected_rank, sweeps)."""
    op = DenseToeplitz(T) if isinstance(T, np.ndarray) else T
    Uk, Vk = _orth(start_u), _orth(start_v)
    norm_t = op.fro_norm()
    TV = op.matmul(Vk)
    Qk = Uk.conj().T @ TV
    sweeps, detected = 0, Vk.shape[1]
    while np.linalg.norm(TV - Uk @ Qk) > tol * norm_t and sweeps < max_sweeps:
        sweeps += 1
        Uk = _orth(op.matmul(Vk))
        W = op.rmatmul(Uk)
        if sweeps == 1:
            Qv, Rv, perm = scipy.linalg.qr(W, mode="economic", pivoting=True)
            tail = np.sqrt(np.cumsum((np.abs(Rv) ** 2).sum(axis=1)[::-1])[::-1])
            cut = np.nonzero(tail <= tol * np.linalg.norm(Rv))[0]
            detected = int(cut[0]) if cut.size else Rv.shape[0]
            r = detected if rank is None else rank
            inv = np.empty_like(perm)
            inv[perm] = np.arange(perm.size)
            Vk = Qv[:, :r]
            Qk = Rv[:r, inv].conj().T
        else:
            Vk, Rv = np.linalg.qr(W)
            Qk = Rv.conj().T
        TV = op.matmul(Vk)
    Uq, s, Vqh = np.linalg.svd(Qk, full_matrices=False)
    r = Vk.shape[1] if rank is None else rank
    return (Uk @ Uq)[:, :r], s[:r], (Vk @ Vqh.conj().T)[:, :r], detected, sweeps


def _project_out(x: np.ndarray, Q: list) -> np.ndarray:
    """Remove the components along the orthonormal vectors Q, twice."""
    if Q:
        M = np.stack(Q, axis=1)
        for _ in range(2):
            x = x - M @ (M.conj().T @ x)
    return x


def lanczos_svd(T, p1: np.ndarray, tol: float, restart_vectors=(), max_steps: int | None = None):
    """Lanczos bidiagonalization (Sec. 2.1, Algorithm 2) with full
    reorthogonalisation and the early-stop check and restart described with it.
    T is a matrix or an operator with matmul, rmatmul and fro_norm (GpuToeplitz:
    every step is one GPU product with T and one with T^*). Coefficients below
    tol ||T||_F count as zero; a zero triggers the check with the next caller-drawn
    vector of `restart_vectors`. Returns (U, sigma, V, rank) from the SVD of the
    bidiagonal factor; the rank counts its singular values above the threshold."""
    op = DenseToeplitz(T) if isinstance(T, np.ndarray) else T
    thr = tol * op.fro_norm()
    vecs = iter(restart_vectors)
    n = p1.shape[0]
    steps = max_steps if max_steps is not None else n

    def mv(x):
        return op.matmul(x[:, None])[:, 0]

    def rmv(x):
        return op.rmatmul(x[:, None])[:, 0]

    us, vs = [], [p1 / np.linalg.norm(p1)]
    diag, sup = [], []
    beta = 0.0
    done = None
    for _ in range(steps):
        r = mv(vs[-1]) - (beta * us[-1] if us else 0.0)
        r = _project_out(r, us)
        alpha = float(np.linalg.norm(r))
        if alpha <= thr:
            y = _project_out(np.asarray(next(vecs), dtype=complex), us)
            if np.linalg.norm(rmv(y)) <= thr * np.linalg.norm(y):
                done = "alpha"
                break
            r, alpha = y, 0.0
        us.append(r / np.linalg.norm(r))
        diag.append(alpha)
        p = _project_out(rmv(us[-1]) - alpha * vs[-1], vs)
        beta = float(np.linalg.norm(p))
        if beta <= thr:
            w = _project_out(np.asarray(next(vecs), dtype=complex), vs)
            if np.linalg.norm(mv(w)) <= thr * np.linalg.norm(w):
                done = "beta"
                break
            p, beta = w, 0.0
        sup.append(beta)
        vs.append(p / np.linalg.norm(p))
    k = len(us)
    cols = k if done == "beta" else k + 1
    B = np.zeros((k, cols))
    B[range(k), range(k)] = diag
    for j, b in enumerate(sup[:cols - 1]):
        B[j, j + 1] = b
    Ub, s, Vbh = np.linalg.svd(B, full_matrices=False)
    U = np.stack(us, axis=1) @ Ub
    V = np.stack(vs[:cols], axis=1) @ Vbh.conj().T
    # a step taken past the rank by rounding leaves a singular value of B at rounding
    # level: the rank counts the singular values above the stopping threshold
    return U, s, V, int(np.count_nonzero(s > thr))


def reduced_svd(T: np.ndarray, m: int, start_blocks=None, tol: float | None = None):
    """Rank-m reduced SVD of T: LAPACK for N <= 1024, Algorithm 3 above."""
    N = T.shape[0]
    if N <= 1024 or start_blocks is None:
        Uf, s, Vh = np.linalg.svd(T)
        return Uf[:, :m], s[:m], Vh[:m].conj().T, s
    tol = N * np.finfo(float).eps if tol is None else tol
    U, s, V, _, _ = power_svd(T, start_blocks[0], start_blocks[1], tol, rank=m)
    return U, s, V, s


def nodes(S: np.ndarray, mu: np.ndarray):
    """z_j(l) = diag(W^{-1} S_l W) with W the eigenvectors of C_mu = sum mu_l S_l;
    t_j(l) = -arg z_j(l) / (2 pi) wrapped to [0, 1)."""
    C = np.einsum("l,lij->ij", mu, S)
    _, W = np.linalg.eig(C)
    lu = scipy.linalg.lu_factor(W)
    z = np.stack([np.diag(scipy.linalg.lu_solve(lu, S[l] @ W)) for l in range(S.shape[0])], axis=1)
    t = np.mod(-np.angle(z) / (2.0 * np.pi), 1.0)
    return z, t


def solve_normal_equations(gram: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """c from gram c = rhs (Hermitian positive definite; Cholesky, LU if that fails)."""
    try:
        return scipy.linalg.cho_solve(scipy.linalg.cho_factor(gram), rhs)
    except np.linalg.LinAlgError:
        return np.linalg.solve(gram, rhs)


@dataclasses.dataclass
class Solution:
    t: np.ndarray
    c: np.ndarray
    z: np.ndarray
    S: np.ndarray
    sigma: np.ndarray
    U: np.ndarray
    V: np.ndarray


def solve(f: torch.Tensor, d: int, n: int, m: int, mu: np.ndarray, prec: str = "fp64",
          start_blocks=None, svd: str = "dense") -> Solution:
    """Algorithm 1 on one GPU plus the host: reduced SVD of T -> S_l (GPU) -> nodes
    (host) -> Vandermonde products (GPU) -> coefficients (host).

    svd="dense": T formed on the GPU and decomposed on the host (LAPACK for
    N <= 1024, else Algorithm 3 on the dense T); svd="gpu": Algorithm 3 with the
    block products on the GPU (start_blocks required), T never formed;
    svd="lanczos": Algorithm 2 with GPU products (start_blocks = (p1, restart
    vectors)), T never formed."""
    dev = f.device
    if svd == "gpu":
        if start_blocks is None:
            raise ValueError("svd='gpu' needs start_blocks (two N x r blocks)")
        N = (n + 1) ** d
        U, s, V, _, _ = power_svd(GpuToeplitz(f, d, n), start_blocks[0], start_blocks[1],
                                  N * np.finfo(float).eps, rank=m)
    elif svd == "lanczos":
        if start_blocks is None:
            raise ValueError("svd='lanczos' needs start_blocks = (p1, restart vectors)")
        N = (n + 1) ** d
        U, s, V, _ = lanczos_svd(GpuToeplitz(f, d, n), start_blocks[0], N * np.finfo(float).eps, start_blocks[1])
        U, s, V = U[:, :m], s[:m], V[:, :m]
    elif svd == "dense":
        T = api.build_T(f, d, n, 0).cpu().numpy()
        U, s, V, _ = reduced_svd(T, m, start_blocks)
        del T
    else:
        raise ValueError("svd must be 'dense', 'gpu' or 'lanczos'")
    Ud = torch.from_numpy(np.ascontiguousarray(U)).to(dev)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).to(dev)
    sd = torch.from_numpy(np.ascontiguousarray(s)).to(dev)
    S = api.build_S(f, d, n, Ud, sd, Vd, prec=prec).cpu().numpy()
    z, t = nodes(S, mu)
    gram, rhs = api.coeffs(torch.from_numpy(np.ascontiguousarray(z)).to(dev), f, d, n)
    c = solve_normal_equations(gram.cpu().numpy(), rhs.cpu().numpy())
    return Solution(t=t, c=c, z=z, S=S, sigma=s, U=U, V=V)
