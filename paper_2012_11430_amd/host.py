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


def pivoted_rank_basis(W: np.ndarray, tol: float, rank: int | None = None):
    """Rank-revealing orthonormal basis of the column space of W (QR with column
    pivoting, W P = Q R). The numerical rank is the first i at which the trailing
    rows R[i:, :] (upper triangular, so the block R[i:, i:]) have Frobenius norm
    at most tol ||R||_F — the rank test of Sec. 2.2; `rank` overrides it.
    Returns (Q[:, :r], Q[:, :r]^* W, detected rank)."""
    Q, R, perm = scipy.linalg.qr(W, mode="economic", pivoting=True)
    tail = np.sqrt(np.cumsum((np.abs(R) ** 2).sum(axis=1)[::-1])[::-1])
    small = np.nonzero(tail <= tol * np.linalg.norm(R))[0]
    detected = int(small[0]) if small.size else R.shape[0]
    r = detected if rank is None else rank
    coords = np.empty_like(R)
    coords[:, perm] = R                        # R P^T: the coordinates of W's columns
    return Q[:, :r], coords[:r], detected


def power_svd(T, start_u: np.ndarray, start_v: np.ndarray, tol: float, rank: int | None = None,
              max_sweeps: int = 60, info: dict | None = None):
    """Dominant singular triplets of T by block power (subspace) iteration with the
    rank determination of Sec. 2.2 (Algorithm 3).

    Orthonormal bases U (left) and V (right) and their coupling B = U^* T V are kept;
    they are accurate when ||T V - U B||_F <= tol ||T||_F. A sweep maps the right
    basis to the left, U = orth(T V), and back: T^* U = V B^* gives the next V and B
    by QR — in the first sweep a pivoted QR whose rank cut (pivoted_rank_basis)
    fixes how many right vectors are kept. The SVD of B yields the triplets.
    T is a matrix or an operator with matmul, rmatmul and fro_norm (GpuToeplitz).
    Returns (U, sigma, V, detected_rank, sweeps); `info`, if given, receives the
    singular values of T^* U in the first sweep ("first_sweep_sigma": estimates of
    sigma_1..sigma_r0, used for sigma_m / sigma_{m+1} when only m are kept)."""
    op = DenseToeplitz(T) if isinstance(T, np.ndarray) else T
    U, V = _orth(start_u), _orth(start_v)
    threshold = tol * op.fro_norm()
    TV = op.matmul(V)
    B = U.conj().T @ TV
    sweeps, detected = 0, V.shape[1]
    while np.linalg.norm(TV - U @ B) > threshold and sweeps < max_sweeps:
        U = _orth(TV)
        TtU = op.rmatmul(U)
        if sweeps == 0:
            if info is not None:
                info["first_sweep_sigma"] = np.linalg.svd(TtU, compute_uv=False)
            V, Bh, detected = pivoted_rank_basis(TtU, tol, rank)
        else:
            V, Bh = np.linalg.qr(TtU)
        B = Bh.conj().T
        sweeps += 1
        TV = op.matmul(V)
    Ub, sigma, Vbh = np.linalg.svd(B, full_matrices=False)
    r = V.shape[1] if rank is None else rank
    return (U @ Ub)[:, :r], sigma[:r], (V @ Vbh.conj().T)[:, :r], detected, sweeps


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


def numerical_rank(sigma: np.ndarray, tol: float) -> int:
    """Number of singular values at or above tol * sigma_1 (the first i with
    sigma_i < tol sigma_1 ends the rank; Sec. 5)."""
    sigma = np.asarray(sigma)
    below = np.nonzero(sigma < tol * sigma[0])[0]
    return int(below[0]) if below.size else int(sigma.size)


def start_blocks_for(N: int, r0: int, seed: int = 0):
    """Two random N x r0 complex Gaussian starting blocks of the block power method
    (Algorithm 3 starts from random bases), from a seeded generator."""
    rng = np.random.Generator(np.random.PCG64(seed))
    def draw():
        return (rng.standard_normal((N, r0)) + 1j * rng.standard_normal((N, r0))) / np.sqrt(2.0)
    return draw(), draw()


def samples_on_index_set(f: np.ndarray, d: int, n: int) -> np.ndarray:
    """f restricted to I_n = {0..n}^d, row-major (the right-hand side of eq. ls_probl):
    grid point p sits at offset p + n along every axis."""
    side = 2 * n + 2
    return np.asarray(f).reshape((side,) * d)[(slice(n, 2 * n + 1),) * d].reshape(-1)


@dataclasses.dataclass
class Solution:
    t: np.ndarray
    c: np.ndarray
    z: np.ndarray
    S: np.ndarray
    sigma: np.ndarray
    U: np.ndarray
    V: np.ndarray
    m: int                    # number of terms used (given, or the detected rank)
    rank: int                 # numerical rank found by the SVD step at tolerance tol
    residual: float           # ||A^T c - f_I|| / ||f_I||: the operational accuracy estimate (Sec. 5)
    sigma_ratio: float | None  # sigma_m / sigma_{m+1} (None when sigma_{m+1} is not known)


def solve(f: torch.Tensor, d: int, n: int, m: int | None, mu: np.ndarray, prec: str = "fp64",
          start_blocks=None, svd: str = "dense", tol: float | None = None, seed: int = 0,
          r0: int | None = None) -> Solution:
    """Algorithm 1 on one GPU plus the host: reduced SVD of T -> S_l (GPU) -> nodes
    (host) -> Vandermonde products (GPU) -> coefficients (host) -> relative LS residual.

    m: number of terms, or None to use the numerical rank the SVD step detects at
    tolerance tol (default N eps, the criterion of Sec. 5; raise it to the noise
    level for noisy samples). The relative residual ||A^T c - f_I|| / ||f_I|| tells
    whether the rank was well determined: a rank below the true number of terms
    leaves a residual far above the noise level (Sec. 5, discussion of Table 1).

    svd="dense": T formed on the GPU and decomposed on the host (LAPACK for
    N <= 1024 or without start blocks, else Algorithm 3 on the dense T); svd="gpu":
    Algorithm 3 with the block products on the GPU, T never formed (start_blocks, or
    seeded random blocks of r0 = 2m columns, 64 when m is None); svd="lanczos":
    Algorithm 2 with GPU products, T never formed (start_blocks = (p1, restart
    vectors), or seeded random ones)."""
    dev = f.device
    N = (n + 1) ** d
    tol = N * np.finfo(float).eps if tol is None else tol
    ratio = None
    if svd == "gpu":
        if start_blocks is None:
            start_blocks = start_blocks_for(N, min(N, r0 or (2 * m if m else 64)), seed)
        info = {}
        U, s, V, rank, _ = power_svd(GpuToeplitz(f, d, n), start_blocks[0], start_blocks[1], tol, rank=m,
                                     info=info)
        m = rank if m is None else m
        est = info.get("first_sweep_sigma")
        if est is not None and est.size > m:
            ratio = float(s[m - 1] / est[m]) if est[m] > 0 else float("inf")
    elif svd == "lanczos":
        if start_blocks is None:
            rng = np.random.Generator(np.random.PCG64(seed))
            draw = lambda: rng.standard_normal(N) + 1j * rng.standard_normal(N)   # noqa: E731
            start_blocks = (draw(), [draw() for _ in range(8)])
        U, s, V, rank = lanczos_svd(GpuToeplitz(f, d, n), start_blocks[0], tol, start_blocks[1])
        m = rank if m is None else m
        if s.size > m:
            ratio = float(s[m - 1] / s[m]) if s[m] > 0 else float("inf")
        U, s, V = U[:, :m], s[:m], V[:, :m]
    elif svd == "dense":
        T = api.build_T(f, d, n, 0).cpu().numpy()
        if N <= 1024 or start_blocks is None:
            Uf, s_all, Vh = np.linalg.svd(T)
            rank = numerical_rank(s_all, tol)
            m = rank if m is None else m
            U, s, V = Uf[:, :m], s_all[:m], Vh[:m].conj().T
            if s_all.size > m:
                ratio = float(s_all[m - 1] / s_all[m]) if s_all[m] > 0 else float("inf")
        else:
            info = {}
            U, s, V, rank, _ = power_svd(T, start_blocks[0], start_blocks[1], tol, rank=m, info=info)
            m = rank if m is None else m
            est = info.get("first_sweep_sigma")
            if est is not None and est.size > m:
                ratio = float(s[m - 1] / est[m]) if est[m] > 0 else float("inf")
        del T
    else:
        raise ValueError("svd must be 'dense', 'gpu' or 'lanczos'")
    if m < 1:
        raise ValueError("the SVD step found no nonzero singular value above the tolerance")
    Ud = torch.from_numpy(np.ascontiguousarray(U)).to(dev)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).to(dev)
    sd = torch.from_numpy(np.ascontiguousarray(s)).to(dev)
    S = api.build_S(f, d, n, Ud, sd, Vd, prec=prec).cpu().numpy()
    z, t = nodes(S, mu)
    gram, rhs, AT = api.coeffs(torch.from_numpy(np.ascontiguousarray(z)).to(dev), f, d, n, want_AT=True)
    c = solve_normal_equations(gram.cpu().numpy(), rhs.cpu().numpy())
    fI = samples_on_index_set(f.cpu().numpy(), d, n)
    residual = float(np.linalg.norm(AT.cpu().numpy() @ c - fI) / np.linalg.norm(fI))
    return Solution(t=t, c=c, z=z, S=S, sigma=s, U=U, V=V, m=m, rank=rank, residual=residual, sigma_ratio=ratio)
