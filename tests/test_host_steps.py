"""Host FP64 steps of Algorithm 1 that need no GPU, on dense matrices: the block
power SVD (Sec. 2.2, Algorithm 3) against LAPACK, its pivoted-QR rank test, the
rank criterion of Sec. 5, the restriction of the sample grid to I_n, and the
seeded start blocks. Pinned against the oracle and LAPACK, not against each other."""
import numpy as np
import pytest

from oracle import prony_oracle as O
from paper_2012_11430_amd import host
from workload import config_instances


def _toeplitz_of(name):
    inst = config_instances(name, count=1)[0]
    grid = O.samples(inst.t, inst.c, inst.n)
    return inst, grid, O.toeplitz(grid, inst.d, inst.n, 0)


def test_power_svd_matches_lapack_on_a_dense_toeplitz_matrix():
    inst, grid, T = _toeplitz_of("c0")
    m, N = inst.m, inst.N
    Uu, Vv = host.start_blocks_for(N, 2 * m, seed=3)
    info = {}
    U, s, V, rank, sweeps = host.power_svd(T, Uu, Vv, N * O.EPS64, info=info)
    ref = np.linalg.svd(T, compute_uv=False)
    assert rank == m and sweeps >= 1
    assert np.max(np.abs(s - ref[:m]) / ref[:m]) < 1e-12
    # singular vectors: T V = U diag(s), U and V orthonormal
    assert np.linalg.norm(T @ V - U * s[None, :]) < 1e-10 * ref[0]
    assert np.linalg.norm(U.conj().T @ U - np.eye(m)) < 1e-12
    # the first sweep's estimates bracket the spectrum's drop after m
    est = info["first_sweep_sigma"]
    assert est[m] < 1e-10 * est[0]


def test_pivoted_rank_basis_finds_the_rank_of_a_low_rank_block():
    rng = np.random.Generator(np.random.PCG64(8))
    A = (rng.standard_normal((60, 3)) + 1j * rng.standard_normal((60, 3))) @ rng.standard_normal((3, 9))
    Q, coords, detected = host.pivoted_rank_basis(A, 1e-12)
    assert detected == 3
    assert np.linalg.norm(Q @ coords - A) < 1e-12 * np.linalg.norm(A)
    _, coords5, _ = host.pivoted_rank_basis(A, 1e-12, rank=5)
    assert coords5.shape == (5, 9)


def test_numerical_rank_matches_the_oracle_criterion():
    s = np.array([10.0, 5.0, 1e-3, 1e-9])
    for tol in (1e-2, 1e-6, 1e-12):
        assert host.numerical_rank(s, tol) == O.numerical_rank(s, tol)


@pytest.mark.parametrize("d,n", [(1, 5), (2, 3), (3, 2)])
def test_samples_on_index_set_matches_the_oracle(d, n):
    rng = np.random.Generator(np.random.PCG64(d + n))
    grid = rng.standard_normal((2 * n + 2) ** d) + 1j * rng.standard_normal((2 * n + 2) ** d)
    assert np.array_equal(host.samples_on_index_set(grid, d, n), O.restrict_to_index_set(grid, d, n))


def test_start_blocks_are_seeded():
    a = host.start_blocks_for(50, 4, seed=1)
    b = host.start_blocks_for(50, 4, seed=1)
    c = host.start_blocks_for(50, 4, seed=2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])
    assert a[0].shape == (50, 4) and a[0].dtype == complex
