"""GPU products with the multilevel Toeplitz matrix (Y = T X, T^* X) for the block
power SVD (Sec. 2.2, Algorithm 3), against the oracle's dense T, and the one-column
products of the Lanczos bidiagonalization (Sec. 2.1, Algorithm 2; the vector kernel),
also at the paper's size on sampled rows; the block power SVD driven by them against
LAPACK; Algorithm 1 end to end without forming T.

Tolerances: 1e-12 (FP64 products), 1e-5 (FP32 products), normwise and entry by
entry; singular values 1e-10 relative."""
import sys

import numpy as np
import pytest
import torch

from oracle import prony_oracle as O
from paper_2012_11430_amd import api, host
from tests._close import assert_close
from workload import config_instances, random_orthonormal

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("d,n,r", [(1, 1, 1), (1, 63, 40), (2, 3, 5), (2, 15, 10), (2, 40, 40), (3, 3, 8),
                                   (3, 7, 33), (2, 5, 64), (1, 200, 17),
                                   # one column (the vector kernel): one and several row tiles and
                                   # chunks, ragged tails
                                   (1, 200, 1), (2, 40, 1), (2, 63, 1), (3, 7, 1), (3, 12, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_products_match_oracle(d, n, r, prec):
    rng = np.random.Generator(np.random.PCG64(3000 + 100 * d + n + r))
    N = (n + 1) ** d
    grid = rng.standard_normal((2 * n + 2) ** d) + 1j * rng.standard_normal((2 * n + 2) ** d)
    X = rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r))
    print(f"toeplitz_mm d={d} n={n} r={r} {prec}", flush=True)
    for adjoint in (False, True):
        ref = O.toeplitz_product(grid, d, n, X, adjoint)
        got = api.toeplitz_mm(_dev(grid), d, n, _dev(X), adjoint=adjoint, prec=prec).cpu().numpy()
        assert_close(got, ref, TOL[prec], f"adjoint={adjoint}")


def test_strided_operands_and_determinism():
    rng = np.random.Generator(np.random.PCG64(31))
    d, n, r = 2, 20, 12
    N = (n + 1) ** d
    grid = rng.standard_normal((2 * n + 2) ** d) + 1j * rng.standard_normal((2 * n + 2) ** d)
    big = _dev(rng.standard_normal((N, 3 * r)) + 1j * rng.standard_normal((N, 3 * r)))
    X = big[:, r:2 * r]                           # leading dimension 3r
    out = torch.zeros((N, 2 * r), dtype=torch.complex128, device=DEV)
    Y = out[:, :r]                                # leading dimension 2r
    api.toeplitz_mm(_dev(grid), d, n, X, out=Y)
    ref = O.toeplitz_product(grid, d, n, X.cpu().numpy())
    assert_close(Y.cpu().numpy(), ref, TOL["fp64"], "strided product")
    assert torch.count_nonzero(out[:, r:]) == 0   # nothing written outside Y
    again = api.toeplitz_mm(_dev(grid), d, n, X)
    assert torch.equal(again, Y)                  # fixed-order sums: bitwise repeatable


def test_gpu_block_power_svd_matches_lapack():
    inst = config_instances("c1", count=1)[0]
    d, n, m = inst.d, 35, inst.m                  # N = 1296: the host LAPACK SVD stays cheap
    grid = O.samples(inst.t, inst.c, n, abs_noise=None)
    N = (n + 1) ** d
    rng = np.random.Generator(np.random.PCG64(7))
    blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
    op = host.GpuToeplitz(_dev(grid), d, n)
    U, s, V, rank, sweeps = host.power_svd(op, blocks[0], blocks[1], N * O.EPS64, rank=m)
    T = O.toeplitz(grid, d, n, 0)
    s_ref = np.linalg.svd(T, compute_uv=False)[:m]
    print(f"gpu power svd: {sweeps} sweeps, detected rank {rank}, sigma rel err "
          f"{np.max(np.abs(s - s_ref) / s_ref):.3e}", flush=True)
    assert np.max(np.abs(s - s_ref) / s_ref) <= 1e-10
    # the singular subspaces: T V = U diag(s)
    assert _rel(T @ V, U * s[None, :]) <= 1e-9
    assert rank == m                                # noise-free: exact rank m


def test_solve_without_forming_T_recovers_c1():
    inst = config_instances("c1", count=1)[0]
    d, n, m = inst.d, inst.n, inst.m
    f = api.samples(_dev(inst.t), _dev(inst.c), n, noise=_dev(inst.noise(inst.noise_levels[0])))
    rng = np.random.Generator(np.random.PCG64(12345))
    N = (n + 1) ** d
    blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
    sol = host.solve(f, d, n, m, inst.mu, prec="fp64", start_blocks=blocks, svd="gpu")
    err_t, err_c = O.recovery_errors(dict(t=sol.t, c=sol.c), inst.t, inst.c)
    print(f"c1 without T: max node error {err_t:.3e}, max coefficient error {err_c:.3e}", flush=True)
    assert err_t <= 1e-6 and err_c <= 1e-4


def test_gpu_lanczos_matches_lapack():
    inst = config_instances("c1", count=1)[0]
    d, n, m = inst.d, 35, inst.m
    grid = O.samples(inst.t, inst.c, n)
    N = (n + 1) ** d
    rng = np.random.Generator(np.random.PCG64(8))
    p1 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    restarts = [rng.standard_normal(N) + 1j * rng.standard_normal(N) for _ in range(8)]
    U, s, V, rank = host.lanczos_svd(host.GpuToeplitz(_dev(grid), d, n), p1, N * O.EPS64, restarts)
    T = O.toeplitz(grid, d, n, 0)
    s_ref = np.linalg.svd(T, compute_uv=False)[:m]
    print(f"gpu lanczos: rank {rank}, sigma rel err {np.max(np.abs(s[:m] - s_ref) / s_ref):.3e}", flush=True)
    assert rank == m
    assert np.max(np.abs(s[:m] - s_ref) / s_ref) <= 1e-10
    assert _rel(T @ V[:, :m], U[:, :m] * s[None, :m]) <= 1e-9


def test_solve_with_gpu_lanczos_recovers_c0():
    inst = config_instances("c0")[0]
    d, n, m = inst.d, inst.n, inst.m
    f = api.samples(_dev(inst.t), _dev(inst.c), n)
    N = (n + 1) ** d
    rng = np.random.Generator(np.random.PCG64(9))
    p1 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    restarts = [rng.standard_normal(N) + 1j * rng.standard_normal(N) for _ in range(8)]
    sol = host.solve(f, d, n, m, inst.mu, prec="fp64", start_blocks=(p1, restarts), svd="lanczos")
    dt, dc = O.recovery_errors(dict(t=sol.t, c=sol.c), inst.t, inst.c)
    assert dt < 1e-12 and dc < 1e-10, (dt, dc)


def test_one_column_strided_and_repeatable():
    # the one-column product reads a strided column and writes only its own column
    rng = np.random.Generator(np.random.PCG64(37))
    d, n = 2, 20
    N = (n + 1) ** d
    grid = rng.standard_normal((2 * n + 2) ** d) + 1j * rng.standard_normal((2 * n + 2) ** d)
    big = _dev(rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3)))
    X = big[:, 1:2]                               # leading dimension 3
    out = torch.zeros((N, 2), dtype=torch.complex128, device=DEV)
    Y = out[:, :1]                                # leading dimension 2
    for adjoint in (False, True):
        api.toeplitz_mm(_dev(grid), d, n, X, adjoint=adjoint, out=Y)
        ref = O.toeplitz_product(grid, d, n, X.cpu().numpy(), adjoint)
        assert_close(Y.cpu().numpy(), ref, TOL["fp64"], f"one column, adjoint={adjoint}")
        assert torch.count_nonzero(out[:, 1:]) == 0
        again = api.toeplitz_mm(_dev(grid), d, n, X, adjoint=adjoint)
        assert torch.equal(again, Y)              # fixed-order sums: bitwise repeatable


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_column_at_the_paper_size_sampled_rows(prec):
    # d = 3, n = 20 (N = 9261, the paper's workload; the products of one Lanczos step):
    # sampled rows of T x and T^* x against rows of T formed one by one from the oracle's
    # index set and grid indexing (T[k, h] = f(k - h); (T^*)[k, h] = conj f(h - k))
    d, n = 3, 20
    rng = np.random.Generator(np.random.PCG64(41))
    N = (n + 1) ** d
    grid = rng.standard_normal((2 * n + 2) ** d) + 1j * rng.standard_normal((2 * n + 2) ** d)
    x = rng.standard_normal((N, 1)) + 1j * rng.standard_normal((N, 1))
    I = O.index_set(d, n)
    rows = np.unique(np.concatenate([[0, N - 1], rng.choice(N, 62, replace=False)]))
    print(f"toeplitz_mm one column d={d} n={n} {prec}", flush=True)
    for adjoint in (False, True):
        got = api.toeplitz_mm(_dev(grid), d, n, _dev(x), adjoint=adjoint, prec=prec).cpu().numpy()[rows, 0]
        ref = np.empty(rows.size, dtype=complex)
        for i, k in enumerate(rows):
            if adjoint:
                trow = grid[O.grid_flat_index(I - I[k][None, :], n)].conj()
            else:
                trow = grid[O.grid_flat_index(I[k][None, :] - I, n)]
            ref[i] = trow @ x[:, 0]
        assert_close(got, ref, TOL[prec], f"sampled rows, adjoint={adjoint}")
