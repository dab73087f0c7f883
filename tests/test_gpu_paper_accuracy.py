"""Algorithm 1 on the GPU path, with the block products of the power SVD on the GPU
(T is never formed), on the paper's own accuracy workload: Sec. 5, Table 1 (d=3, n=20,
N=9261, m=5, the deterministic inputs of the efficiency tests, samples f(k)(1 + delta_k)),
and on its rank observations (Sec. 5, d=2, n=20, rank criterion sigma_i < N eps sigma_1).

The recovered nodes, coefficients and the relative LS residual must fall in the decade
band of each printed value (for eps = 0: below ten times the printed rounding level);
the digits themselves are unpinned (the paper does not state the distribution of
delta_k; uniform on [-eps, eps] is the reading used here)."""
import numpy as np
import pytest
import torch

from oracle import prony_oracle as O
from paper_2012_11430_amd import api, host
from workload import paper_efficiency_inputs, paper_relative_noise, random_orthonormal

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
MU = np.array([1.0, 1j, -0.5]) / np.linalg.norm([1.0, 1j, -0.5])


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _rows(golden_dir, name):
    return [line.split() for line in open(f"{golden_dir}/{name}") if line.strip() and not line.startswith("#")]


def _gpu_algorithm1(grid, d, n, m, tol, seed, prec="fp64"):
    N = (n + 1) ** d
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
    f = _dev(grid)
    U, s, V, rank, sweeps = host.power_svd(host.GpuToeplitz(f, d, n), blocks[0], blocks[1], tol, rank=m)
    S = api.build_S(f, d, n, _dev(U), _dev(s), _dev(V), prec=prec).cpu().numpy()
    z, t = host.nodes(S, MU[:d] / np.linalg.norm(MU[:d]))
    gram, rhs, AT = api.coeffs(_dev(z), f, d, n, want_AT=True)
    c = host.solve_normal_equations(gram.cpu().numpy(), rhs.cpu().numpy())
    fI = O.restrict_to_index_set(grid, d, n)
    resid = float(np.linalg.norm(AT.cpu().numpy() @ c - fI) / np.linalg.norm(fI))
    return t, c, resid, rank


@pytest.fixture(scope="module")
def golden_dir():
    import os
    return os.path.join(os.path.dirname(__file__), "golden")


def test_table1_decade_bands_on_gpu_path(golden_dir):
    d, n, m = 3, 20, 5
    N = (n + 1) ** d
    t_true, c_true = paper_efficiency_inputs(d, m)
    clean = O.samples(t_true, c_true, n)
    for eps_s, tol_s, r_res, r_dt, r_dc in _rows(golden_dir, "table1_accuracy.txt"):
        eps = float(eps_s)
        tol = N * O.EPS64 if tol_s == "Neps" else float(tol_s)
        grid = clean * (1.0 + paper_relative_noise(1, d, n, eps)) if eps else clean
        t, c, resid, _ = _gpu_algorithm1(grid, d, n, m, tol, seed=140)
        dt, dc = O.recovery_errors(dict(t=t, c=c), t_true, c_true)
        print(f"Table 1 eps={eps_s}: resid {resid:.3e} ({r_res}), dt {dt:.3e} ({r_dt}), dc {dc:.3e} ({r_dc})",
              flush=True)
        for got, ref in zip((resid, dt, dc), (float(r_res), float(r_dt), float(r_dc))):
            if eps == 0.0:
                assert got < 10 * ref
            else:
                assert ref / 10 < got < 10 * ref


def test_rank_detection_on_gpu_path(golden_dir):
    for d_s, n_s, m_s, rel in _rows(golden_dir, "rank_detection.txt"):
        d, n, m = int(d_s), int(n_s), int(m_s)
        N = (n + 1) ** d
        t_true, c_true = paper_efficiency_inputs(d, m)
        f = _dev(O.samples(t_true, c_true, n))
        rng = np.random.Generator(np.random.PCG64(41))
        blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
        _, _, _, rank, _ = host.power_svd(host.GpuToeplitz(f, d, n), blocks[0], blocks[1], N * O.EPS64)
        print(f"rank d={d} n={n} m={m}: detected {rank} ({rel})", flush=True)
        assert (rank == m) if rel == "eq" else (rank < m)


def test_rank_detection_with_gpu_lanczos(golden_dir):
    # Sec. 5: the Lanczos method found the same ranks as the other SVD algorithms
    for d_s, n_s, m_s, rel in _rows(golden_dir, "rank_detection.txt"):
        d, n, m = int(d_s), int(n_s), int(m_s)
        N = (n + 1) ** d
        t_true, c_true = paper_efficiency_inputs(d, m)
        f = _dev(O.samples(t_true, c_true, n))
        rng = np.random.Generator(np.random.PCG64(42))
        p1 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        restarts = [rng.standard_normal(N) + 1j * rng.standard_normal(N) for _ in range(8)]
        _, _, _, rank = host.lanczos_svd(host.GpuToeplitz(f, d, n), p1, N * O.EPS64, restarts)
        print(f"lanczos rank d={d} n={n} m={m}: detected {rank} ({rel})", flush=True)
        assert (rank == m) if rel == "eq" else (rank < m)


def test_residual_flags_a_wrongly_determined_rank():
    # Sec. 5, after Table 1: at eps = 1e-3 the rank test with tol = eps finds rank 4
    # (sigma_5 / sigma_1 ~ 9e-4) and the errors are large; tol = 1e-4 finds rank 5.
    # The relative LS residual, which needs no knowledge of the true parameters,
    # reveals the difference (the operational accuracy estimate).
    d, n, m, eps = 3, 20, 5, 1e-3
    N = (n + 1) ** d
    t_true, c_true = paper_efficiency_inputs(d, m)
    grid = O.samples(t_true, c_true, n) * (1.0 + paper_relative_noise(1, d, n, eps))
    f = _dev(grid)
    mu = MU / np.linalg.norm(MU)
    blocks = host.start_blocks_for(N, 2 * m, seed=7)
    sols = {tol: host.solve(f, d, n, None, mu, svd="gpu", tol=tol, start_blocks=blocks) for tol in (1e-3, 1e-4)}
    for tol, sol in sols.items():
        dt, dc = O.recovery_errors(dict(t=sol.t, c=sol.c), t_true, c_true) if sol.m == m else (None, None)
        print(f"eps=1e-3 tol={tol:g}: rank {sol.rank}, residual {sol.residual:.3e}, "
              f"sigma_m/sigma_m+1 {sol.sigma_ratio}, dt {dt}, dc {dc}", flush=True)
    wrong, right = sols[1e-3], sols[1e-4]
    assert wrong.rank == 4 and wrong.m == 4
    assert right.rank == 5 and right.m == 5
    # right rank: residual at the noise level (Table 1: 3.0e-4); wrong rank: far above it
    assert 3e-5 < right.residual < 3e-3
    assert wrong.residual > 10 * right.residual
    # the kept singular values are well separated from the next one when the rank is right
    assert right.sigma_ratio is not None and right.sigma_ratio > 10


def test_solve_with_default_start_blocks_and_fixed_m():
    # host.solve(svd="gpu") draws its own seeded start blocks when none are given
    d, n, m = 3, 20, 5
    t_true, c_true = paper_efficiency_inputs(d, m)
    f = _dev(O.samples(t_true, c_true, n))
    sol = host.solve(f, d, n, m, MU, svd="gpu")
    dt, dc = O.recovery_errors(dict(t=sol.t, c=sol.c), t_true, c_true)
    assert sol.m == m and sol.rank == m
    assert dt < 1e-10 and dc < 1e-8 and sol.residual < 1e-10
