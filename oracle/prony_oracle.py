"""Plain FP64 CPU oracle of the multivariate matrix-pencil Prony method
(N. Bosner, "Parallel Prony's method with multivariate matrix pencil approach
and its numerical aspect", arXiv 2012.11430).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module. The library under
`paper_2012_11430_amd` never imports it and shares no code with it.

Every function follows the paper's definitions literally, with numpy in
complex128 / float64 and library primitives (matmul, SVD, QR, eig, lstsq) as
single steps; nothing is blocked, fused or reordered. Sizes stay small enough
for dense matrices (N <= ~9000).

Conventions (the paper leaves the ordering of I_n free, Sec. 1):
  * I_n = {0..n}^d in row-major order, last coordinate fastest; N = (n+1)^d.
  * The sample grid holds f(p) for p in {-n..n+1}^d, row-major, flat, which
    covers every argument k-h and k-h+e_l of T and T_l.
  * Matrices are numpy arrays; V is the right factor itself (not V^*).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg

# ---------------------------------------------------------------------------
# Index sets
# ---------------------------------------------------------------------------


def index_set(d: int, n: int) -> np.ndarray:
    """I_n = {0..n}^d as an (N, d) integer array in row-major order (Sec. 1)."""
    return np.array(list(itertools.product(range(n + 1), repeat=d)), dtype=np.int64).reshape(-1, d)


def grid_points(d: int, n: int) -> np.ndarray:
    """The sample points {-n..n+1}^d as a ((2n+2)^d, d) array, row-major."""
    return np.array(list(itertools.product(range(-n, n + 2), repeat=d)), dtype=np.int64).reshape(-1, d)


def grid_flat_index(p: np.ndarray, n: int) -> np.ndarray:
    """Flat position of points p (..., d) in the row-major grid {-n..n+1}^d."""
    p = np.asarray(p, dtype=np.int64)
    d = p.shape[-1]
    if np.any(p < -n) or np.any(p > n + 1):
        raise ValueError("point outside the sample grid")
    idx = np.zeros(p.shape[:-1], dtype=np.int64)
    for axis in range(d):
        idx = idx * (2 * n + 2) + (p[..., axis] + n)
    return idx


# ---------------------------------------------------------------------------
# Samples of the exponential sum (Sec. 1, eq. exp_sum; noise model of Sec. 4)
# ---------------------------------------------------------------------------


def samples(t, c, n: int, abs_noise=None, rel_noise=None) -> np.ndarray:
    """f(p) = sum_j c_j exp(-2 pi i <t_j, p>) on the grid {-n..n+1}^d.

    The phase <t_j,p> is reduced to [-1/2, 1/2] by subtracting its nearest
    integer before the exponential (exp(-2 pi i x) has period 1 in x).
    Optional perturbations: relative f(p)(1 + delta_p) (the accuracy test of
    Sec. 5) and additive f(p) + Delta f_p (the noise model of Sec. 4).
    """
    t = np.asarray(t, dtype=float)
    c = np.asarray(c, dtype=complex)
    m, d = t.shape
    p = grid_points(d, n).astype(float)
    phase = p @ t.T                      # (G, m): <t_j, p>
    phase = phase - np.round(phase)
    f = np.exp(-2j * np.pi * phase) @ c
    if rel_noise is not None:
        f = f * (1.0 + np.asarray(rel_noise))
    if abs_noise is not None:
        f = f + np.asarray(abs_noise)
    return f


def restrict_to_index_set(grid: np.ndarray, d: int, n: int) -> np.ndarray:
    """The vector f = [f(k)]_{k in I_n} (Sec. 1, eq. ls_probl)."""
    return grid[grid_flat_index(index_set(d, n), n)]


# ---------------------------------------------------------------------------
# Multilevel Toeplitz matrices (Sec. 1)
# ---------------------------------------------------------------------------


def toeplitz(grid: np.ndarray, d: int, n: int, ell: int) -> np.ndarray:
    """T (ell = 0) or T_ell (ell = 1..d): entry (k, h) is f(k - h + e_ell), k, h in I_n."""
    if not 0 <= ell <= d:
        raise ValueError("ell must be in 0..d")
    I = index_set(d, n)
    e = np.zeros(d, dtype=np.int64)
    if ell > 0:
        e[ell - 1] = 1
    N = I.shape[0]
    out = np.empty((N, N), dtype=complex)
    for row, k in enumerate(I):
        out[row] = grid[grid_flat_index(k[None, :] - I + e[None, :], n)]
    return out


def toeplitz_product(grid: np.ndarray, d: int, n: int, X: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """T X or T^* X with T the multilevel Toeplitz matrix of the grid (the two block
    products of every sweep of Algorithm 3, Sec. 2.2)."""
    T = toeplitz(grid, d, n, 0)
    return (T.conj().T if adjoint else T) @ X


# ---------------------------------------------------------------------------
# Reduced SVD of T (Sec. 1 eq. T_svd; Sec. 2.2 Algorithm 3)
# ---------------------------------------------------------------------------


def reduced_svd(T: np.ndarray, m: int):
    """First m singular triplets of T from a full LAPACK SVD: (U, sigma, V)."""
    Uf, s, Vh = np.linalg.svd(T)
    return Uf[:, :m], s[:m], Vh[:m].conj().T


def numerical_rank(sigma: np.ndarray, tol: float) -> int:
    """Smallest i with sigma_{i+1} < tol * sigma_1 (criterion of Sec. 5)."""
    sigma = np.asarray(sigma)
    below = np.nonzero(sigma < tol * sigma[0])[0]
    return int(below[0]) if below.size else int(sigma.size)


def _orthonormal_columns(X: np.ndarray) -> np.ndarray:
    Q, _ = np.linalg.qr(X)
    return Q


def _reorthogonalize(x: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """x minus its projection on the orthonormal columns of Q, done twice (full
    reorthogonalisation, Sec. 2.1)."""
    for _ in range(2):
        if Q.shape[1]:
            x = x - Q @ (Q.conj().T @ x)
    return x


def lanczos_bidiagonalization(A: np.ndarray, p1: np.ndarray, tol: float, restart_vectors=(),
                              max_steps: int | None = None):
    """Lanczos bidiagonalization with full reorthogonalisation, the early-stop check
    and restart (Sec. 2.1, Algorithm 2 and the text after it); rank from the size of
    the bidiagonal factor.

    A v_i - beta_i u_{i-1} and A^* u_i - alpha_i v_i give alpha_i u_i and
    beta_{i+1} v_{i+1}; a coefficient <= tol ||A||_F counts as zero. Then a random
    vector (taken in order from `restart_vectors`, drawn by the caller) is
    orthogonalised against the current basis: if the operator maps it below the
    tolerance the process has finished, otherwise it becomes the next basis vector
    with a zero coefficient in B.
    Returns (U, sigma, V, rank): the singular triplets of A from the SVD of B
    (left vectors U_i U_B, right V V_B), sorted decreasingly, and the rank.
    """
    rows, cols = A.shape
    thr = tol * np.linalg.norm(A)
    restarts = iter(restart_vectors)
    steps = max_steps if max_steps is not None else min(rows, cols)
    U = np.zeros((rows, 0), dtype=complex)
    beta1 = np.linalg.norm(p1)
    V = (p1 / beta1).astype(complex)[:, None]
    alphas, betas = [], []          # B: alpha_i on the diagonal, beta_{i+1} above it
    beta_i = beta1
    stop = None
    for _ in range(steps):
        r = A @ V[:, -1]
        if U.shape[1]:
            r = r - beta_i * U[:, -1]
        r = _reorthogonalize(r, U)
        alpha = np.linalg.norm(r)
        if alpha <= thr:
            y = _reorthogonalize(np.asarray(next(restarts), dtype=complex), U)
            if np.linalg.norm(A.conj().T @ y) <= thr * np.linalg.norm(y):
                stop = "alpha"      # span{u_1..u_i} = R(A): B is i x (i+1)
                break
            r, alpha = y, 0.0
        u = r / np.linalg.norm(r)
        alphas.append(alpha)
        U = np.hstack([U, u[:, None]])
        p = _reorthogonalize(A.conj().T @ u - alpha * V[:, -1], V)
        beta = np.linalg.norm(p)
        if beta <= thr:
            w = _reorthogonalize(np.asarray(next(restarts), dtype=complex), V)
            if np.linalg.norm(A @ w) <= thr * np.linalg.norm(w):
                stop = "beta"       # span{v_1..v_i} = R(A^*): B is i x i
                break
            p, beta = w, 0.0
        betas.append(beta)
        V = np.hstack([V, (p / np.linalg.norm(p))[:, None]])
        beta_i = beta
    i = U.shape[1]
    ncol = i + 1 if stop == "alpha" or stop is None else i
    B = np.zeros((i, ncol))
    B[np.arange(i), np.arange(i)] = alphas
    sup = betas[:ncol - 1]
    B[np.arange(len(sup)), np.arange(1, len(sup) + 1)] = sup
    UB, s, VBh = np.linalg.svd(B, full_matrices=False)
    # Reading: rounding can let the process take a step past the rank (a v_i with a
    # component just above the threshold); such a step adds a singular value of B
    # at rounding level, so the rank counts the singular values of B above the same
    # threshold instead of the raw size of B.
    rank = int(np.count_nonzero(s > thr))
    return U @ UB, s, V[:, :ncol] @ VBh.conj().T, rank


def pivoted_rank_cut(W: np.ndarray, tol: float):
    """Numerical rank of W from a QR factorisation with column pivoting (Sec. 2.2):
    W Pi = Q R, and the rank is the first i whose trailing block R(i:, i:) has
    Frobenius norm at most tol ||R||_F (all columns when there is none).
    Returns (Q, R Pi^T, rank), so that W = Q (R Pi^T) exactly."""
    Q, R, perm = scipy.linalg.qr(W, mode="economic", pivoting=True)
    Pi = np.eye(W.shape[1])[:, perm]
    total = np.linalg.norm(R)
    rank = R.shape[0]
    for i in range(R.shape[0]):
        if np.linalg.norm(R[i:, i:]) <= tol * total:
            rank = i
            break
    return Q, R @ Pi.T, rank


def block_power_svd(A: np.ndarray, U0: np.ndarray, V0: np.ndarray, tol: float,
                    rank: int | None = None, max_sweeps: int = 60):
    """Block power method for the SVD with rank determination (Sec. 2.2, Algorithm 3),
    written as a subspace iteration.

    The iteration keeps orthonormal bases U (left) and V (right) and their coupling
    C = U^* A V; the pair is converged when the residual A V - U C has Frobenius norm
    at most tol ||A||_F. One sweep maps the right basis to the left one,
    U = orth(A V), and back: A^* U = V C^* is a QR factorisation of A^* U, with
    column pivoting in the first sweep, whose rank cut (pivoted_rank_cut) fixes the
    number of right vectors kept. The singular triplets are those of C in the two
    bases.

    U0, V0: starting blocks with r0 columns (orthonormalised here).
    rank:   if given, the number of right vectors kept after the first sweep (the
            detected rank is still returned as a diagnostic).

    Reading: A^* U = Q (R Pi^T) with Q cut to its first r columns keeps all r0
    columns of U, so C^* = (R Pi^T)(1:r, :) and C is r0 x r in the sweep that cuts
    the rank.
    Returns (U, sigma, V, detected_rank, sweeps).
    """
    U = _orthonormal_columns(U0)
    V = _orthonormal_columns(V0)
    norm_A = np.linalg.norm(A)
    C = U.conj().T @ A @ V
    sweeps = 0
    detected = None
    while np.linalg.norm(A @ V - U @ C) > tol * norm_A and sweeps < max_sweeps:
        U = _orthonormal_columns(A @ V)
        W = A.conj().T @ U                  # = V C^* for the next right basis V
        if detected is None:
            Q, RPt, detected = pivoted_rank_cut(W, tol)
            kept = detected if rank is None else rank
            V = Q[:, :kept]
            C = RPt[:kept, :].conj().T
        else:
            V, RW = np.linalg.qr(W)
            C = RW.conj().T
        sweeps += 1
    if detected is None:
        detected = V.shape[1]
    UC, s, VCh = np.linalg.svd(C, full_matrices=False)
    r = V.shape[1] if rank is None else rank
    return (U @ UC)[:, :r], s[:r], (V @ VCh.conj().T)[:, :r], detected, sweeps


# ---------------------------------------------------------------------------
# Pencil matrices (Sec. 1 eq. generateSl)
# ---------------------------------------------------------------------------


def pencil_matrices(grid: np.ndarray, d: int, n: int, U: np.ndarray, sigma: np.ndarray,
                    V: np.ndarray, with_s0: bool = False) -> np.ndarray:
    """S_ell = U^* T_ell V Sigma^{-1}, ell = 1..d (ell = 0 first when with_s0).

    Returns an array (d or d+1, m, m).
    """
    ells = range(0 if with_s0 else 1, d + 1)
    Sinv = np.diag(1.0 / np.asarray(sigma, dtype=float))
    out = []
    for ell in ells:
        Tl = toeplitz(grid, d, n, ell)
        out.append(U.conj().T @ Tl @ V @ Sinv)
    return np.array(out)


# ---------------------------------------------------------------------------
# Nodes from the pencil (Sec. 1, Algorithm 1, eigenvalue step; Sec. 4 z -> t)
# ---------------------------------------------------------------------------


def combination(S: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """C_mu = sum_ell mu_ell S_ell (Sec. 1)."""
    return np.tensordot(np.asarray(mu), S, axes=(0, 0))


def nodes_from_pencil(S: np.ndarray, mu: np.ndarray):
    """Diagonalise C_mu, read z_j(ell) off diag(W^{-1} S_ell W), t = -arg(z)/(2 pi) mod 1.

    Returns (z (m, d) complex, t (m, d) float, W).
    Reading: the printed arctangent formula loses the quadrant and the sign;
    the principal argument with the sign of Re(log z / (-2 pi i)) is used and
    the result wrapped into [0, 1).
    """
    C = combination(S, mu)
    _, W = np.linalg.eig(C)
    d = S.shape[0]
    z = np.empty((W.shape[0], d), dtype=complex)
    for ell in range(d):
        z[:, ell] = np.diag(np.linalg.solve(W, S[ell] @ W))
    t = np.mod(-np.angle(z) / (2.0 * np.pi), 1.0)
    return z, t, W


# ---------------------------------------------------------------------------
# Coefficients (Sec. 1 eq. ls_probl, Algorithm 1, coefficient step)
# ---------------------------------------------------------------------------


def vandermonde_transpose(z: np.ndarray, d: int, n: int) -> np.ndarray:
    """A^T = [z_j^k]_{k in I_n, j}, z_j^k = prod_ell z_j(ell)^{k_ell} (N x m)."""
    z = np.asarray(z, dtype=complex)
    I = index_set(d, n)
    AT = np.ones((I.shape[0], z.shape[0]), dtype=complex)
    for ell in range(d):
        AT = AT * np.power(z[None, :, ell], I[:, ell:ell + 1])
    return AT


def coefficient_products(z: np.ndarray, grid: np.ndarray, d: int, n: int):
    """Gram (A^T)^* A^T and right-hand side (A^T)^* f of the normal equations."""
    AT = vandermonde_transpose(z, d, n)
    f = restrict_to_index_set(grid, d, n)
    return AT.conj().T @ AT, AT.conj().T @ f


def least_squares_coefficients(z: np.ndarray, grid: np.ndarray, d: int, n: int):
    """c = argmin_c ||A^T c - f||_2 (Householder-QR/SVD least squares)."""
    AT = vandermonde_transpose(z, d, n)
    f = restrict_to_index_set(grid, d, n)
    c, *_ = np.linalg.lstsq(AT, f, rcond=None)
    resid = np.linalg.norm(AT @ c - f) / np.linalg.norm(f)
    return c, resid


# ---------------------------------------------------------------------------
# Algorithm 1 end to end
# ---------------------------------------------------------------------------


def prony(grid: np.ndarray, d: int, n: int, m: int, mu: np.ndarray, svd: str = "full",
          start_blocks=None, tol: float | None = None):
    """Algorithm 1 with rank m: returns dict(t, c, z, sigma, S, U, V, resid, rank).

    svd = 'full' uses LAPACK; 'power' uses Algorithm 3 with the given start
    blocks (N x r0 each) and tolerance.
    """
    T = toeplitz(grid, d, n, 0)
    N = T.shape[0]
    if svd == "full":
        Uf, s_all, Vh = np.linalg.svd(T)
        U, sigma, V = Uf[:, :m], s_all[:m], Vh[:m].conj().T
        detected = numerical_rank(s_all, N * np.finfo(float).eps if tol is None else tol)
    else:
        U0, V0 = start_blocks
        U, sigma, V, detected, _ = block_power_svd(
            T, U0, V0, tol=N * np.finfo(float).eps if tol is None else tol, rank=m)
        s_all = sigma
    S = pencil_matrices(grid, d, n, U, sigma, V)
    z, t, _ = nodes_from_pencil(S, mu)
    c, resid = least_squares_coefficients(z, grid, d, n)
    return dict(t=t, c=c, z=z, sigma=sigma, S=S, U=U, V=V, resid=resid,
                rank=detected, singular_values=s_all)


def match_nodes(t_est: np.ndarray, t_true: np.ndarray):
    """Permutation tau pairing estimated and true nodes by torus distance."""
    from scipy.optimize import linear_sum_assignment
    diff = np.abs(t_est[:, None, :] - t_true[None, :, :]) % 1.0
    dist = np.sqrt(np.sum(np.minimum(diff, 1.0 - diff) ** 2, axis=-1))
    rows, cols = linear_sum_assignment(dist)
    perm = np.empty(t_true.shape[0], dtype=int)
    perm[cols] = rows
    return perm


def recovery_errors(result: dict, t_true: np.ndarray, c_true: np.ndarray):
    """max torus |dt| and ||dc||/||c|| after matching (Sec. 5 Table 1 metrics)."""
    perm = match_nodes(result["t"], t_true)
    t_est = result["t"][perm]
    c_est = result["c"][perm]
    diff = np.abs(t_est - t_true) % 1.0
    dt = float(np.max(np.minimum(diff, 1.0 - diff)))
    dc = float(np.linalg.norm(c_est - c_true) / np.linalg.norm(c_true))
    return dt, dc


# ---------------------------------------------------------------------------
# Adjoint of the pencil map f -> S_ell (for dL/df with U, Sigma, V fixed)
# ---------------------------------------------------------------------------


def pencil_adjoint(gS: np.ndarray, d: int, n: int, U: np.ndarray, sigma: np.ndarray,
                   V: np.ndarray) -> np.ndarray:
    """Gradient on the sample grid of L(f) given gS_ell = dL/dS_ell (ell = 1..d).

    The map f -> U^* T_ell(f) V Sigma^{-1} is complex-linear, so with PyTorch's
    gradient convention the gradient is its conjugate transpose applied to gS:
    X_ell = U gS_ell Sigma^{-1} V^*, and grad(p) = sum_ell sum_{k - h + e_ell = p} X_ell[k, h].
    """
    I = index_set(d, n)
    G = (2 * n + 2) ** d
    grad = np.zeros(G, dtype=complex)
    Sinv = np.diag(1.0 / np.asarray(sigma, dtype=float))
    for ell in range(1, d + 1):
        e = np.zeros(d, dtype=np.int64)
        e[ell - 1] = 1
        X = U @ gS[ell - 1] @ Sinv @ V.conj().T
        for row, k in enumerate(I):
            np.add.at(grad, grid_flat_index(k[None, :] - I + e[None, :], n), X[row])
    return grad


def pencil_loss(grid: np.ndarray, ref: np.ndarray, d: int, n: int, U, sigma, V) -> float:
    """L = sum_ell ||S_ell(f) - ref_ell||_F^2."""
    S = pencil_matrices(grid, d, n, U, sigma, V)
    return float(np.sum(np.abs(S - ref) ** 2))


# ---------------------------------------------------------------------------
# Paper constants used as test bounds
# ---------------------------------------------------------------------------

EPS64 = float(np.finfo(float).eps)           # machine precision epsilon_M
UNIT_ROUNDOFF_F32 = 2.0 ** -24


