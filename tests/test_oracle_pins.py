"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: brute force
in 50-digit arithmetic, closed forms (Vandermonde factorisations, Dirichlet
kernels, Frobenius norms), library routines on special cases (FFT, polynomial
roots), invariants (S_0 = I, eigenvalues of S_l) and the printed results of
Sec. 5 (rank deficiency, Table of accuracy results).
"""
import itertools
import math

import mpmath
import numpy as np
import pytest

from oracle import prony_oracle as O
from workload import config_instances, paper_efficiency_inputs, paper_relative_noise, random_orthonormal

mpmath.mp.dps = 50


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _random_problem(seed, d, m, sep=0.1):
    rng = _rng(seed)
    pts = []
    while len(pts) < m:
        cand = rng.random(d)
        ok = True
        for p in pts:
            diff = np.abs(cand - p) % 1.0
            if np.sqrt(np.sum(np.minimum(diff, 1 - diff) ** 2)) < sep:
                ok = False
        if ok:
            pts.append(cand)
    t = np.array(pts)
    c = rng.uniform(0.5, 1.5, m) * np.exp(2j * np.pi * rng.random(m))
    return t, c


def _vz(t, d, n):
    """Vandermonde factor [exp(-2 pi i <t_j, k>)]_{k in I_n, j}, written out directly."""
    ks = np.array(list(itertools.product(range(n + 1), repeat=d)), dtype=float)
    return np.exp(-2j * np.pi * (ks @ t.T))


# ---------------------------------------------------------------- samples


@pytest.mark.parametrize("d,n,m", [(1, 3, 2), (2, 2, 3), (3, 1, 2), (2, 3, 1)])
def test_samples_match_50_digit_brute_force(d, n, m):
    t, c = _random_problem(10 + d + n, d, m, sep=0.05)
    f = O.samples(t, c, n)
    for pos, p in enumerate(itertools.product(range(-n, n + 2), repeat=d)):
        acc = mpmath.mpc(0)
        for j in range(m):
            arg = sum(mpmath.mpf(float(t[j, a])) * p[a] for a in range(d))
            acc += mpmath.mpc(complex(c[j])) * mpmath.exp(-2j * mpmath.pi * arg)
        assert abs(complex(acc) - f[pos]) <= 1e-14 * np.sum(np.abs(c))


def test_samples_on_rational_nodes_are_an_fft():
    # t_j = q_j / L with L = 2n+2: f(p) = sum_j c_j exp(-2 pi i q_j p / L) = fft(cvec)[p mod L]
    n = 7
    L = 2 * n + 2
    rng = _rng(3)
    q = rng.choice(L, size=5, replace=False)
    c = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    cvec = np.zeros(L, dtype=complex)
    cvec[q] = c
    f = O.samples((q / L).reshape(-1, 1), c, n)
    ref = np.fft.fft(cvec)[np.arange(-n, n + 2) % L]
    assert np.max(np.abs(f - ref)) < 1e-13


def test_samples_two_dimensional_fft():
    n = 3
    L = 2 * n + 2
    rng = _rng(4)
    cells = rng.choice(L * L, size=6, replace=False)
    q = np.stack([cells // L, cells % L], 1)
    c = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    cmat = np.zeros((L, L), dtype=complex)
    cmat[q[:, 0], q[:, 1]] = c
    f = O.samples(q / L, c, n).reshape(L, L)
    ref = np.fft.fft2(cmat)
    idx = np.arange(-n, n + 2) % L
    assert np.max(np.abs(f - ref[np.ix_(idx, idx)])) < 1e-13


def test_sample_noise_models():
    t, c = _random_problem(5, 2, 3)
    n = 2
    clean = O.samples(t, c, n)
    rel = np.linspace(-1e-3, 1e-3, clean.size)
    add = np.linspace(0, 1, clean.size) * (1 + 1j)
    assert np.allclose(O.samples(t, c, n, rel_noise=rel), clean * (1 + rel), rtol=0, atol=1e-15)
    assert np.allclose(O.samples(t, c, n, abs_noise=add), clean + add, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- Toeplitz


@pytest.mark.parametrize("d,n", [(1, 3), (2, 2), (3, 1), (2, 3)])
def test_toeplitz_brute_force(d, n):
    rng = _rng(20 + d)
    G = (2 * n + 2) ** d
    grid = rng.standard_normal(G) + 1j * rng.standard_normal(G)
    table = {p: grid[i] for i, p in enumerate(itertools.product(range(-n, n + 2), repeat=d))}
    ks = list(itertools.product(range(n + 1), repeat=d))
    for ell in range(d + 1):
        T = O.toeplitz(grid, d, n, ell)
        for a, k in enumerate(ks):
            for b, h in enumerate(ks):
                p = tuple(k[i] - h[i] + (1 if i == ell - 1 else 0) for i in range(d))
                assert T[a, b] == table[p]


@pytest.mark.parametrize("d,n,m", [(1, 9, 3), (2, 5, 4), (3, 3, 3)])
def test_toeplitz_vandermonde_factorisation(d, n, m):
    # T = V_z diag(c) V_z^*, T_l = V_z diag(c_j z_j(l)) V_z^* (Sec. 1: f = A^T c)
    t, c = _random_problem(30 + d, d, m)
    grid = O.samples(t, c, n)
    Vz = _vz(t, d, n)
    T = O.toeplitz(grid, d, n, 0)
    assert np.linalg.norm(T - Vz @ np.diag(c) @ Vz.conj().T) <= 1e-13 * np.linalg.norm(T)
    for ell in range(1, d + 1):
        zl = np.exp(-2j * np.pi * t[:, ell - 1])
        Tl = O.toeplitz(grid, d, n, ell)
        assert np.linalg.norm(Tl - Vz @ np.diag(c * zl) @ Vz.conj().T) <= 1e-13 * np.linalg.norm(Tl)
    s = np.linalg.svd(T, compute_uv=False)
    assert s[m] <= T.shape[0] * O.EPS64 * s[0]          # rank m (criterion of Sec. 5)
    assert s[m - 1] > 1e-6 * s[0]


@pytest.mark.parametrize("d,n", [(1, 6), (2, 4), (3, 2)])
def test_toeplitz_frobenius_closed_form(d, n):
    # ||T_l||_F^2 = sum_p |f(p + e_l)|^2 prod_i (n + 1 - |p_i|), p in {-n..n}^d
    rng = _rng(40 + d)
    G = (2 * n + 2) ** d
    grid = rng.standard_normal(G) + 1j * rng.standard_normal(G)
    table = {p: grid[i] for i, p in enumerate(itertools.product(range(-n, n + 2), repeat=d))}
    for ell in range(d + 1):
        ref = 0.0
        for p in itertools.product(range(-n, n + 1), repeat=d):
            q = tuple(p[i] + (1 if i == ell - 1 else 0) for i in range(d))
            ref += abs(table[q]) ** 2 * np.prod([n + 1 - abs(x) for x in p])
        assert math.isclose(np.linalg.norm(O.toeplitz(grid, d, n, ell)) ** 2, ref, rel_tol=1e-12)


def test_toeplitz_hermitian_for_real_coefficients():
    t, _ = _random_problem(50, 2, 4)
    c = np.array([0.7, 1.1, 0.9, 1.3])
    T = O.toeplitz(O.samples(t, c, 4), 2, 4, 0)
    assert np.allclose(T, T.conj().T, atol=1e-13)


# ---------------------------------------------------------------- SVD


def test_block_power_matches_lapack_and_closed_form():
    inst = config_instances("c0")[0]
    d, n, m = inst.d, inst.n, inst.m
    grid = O.samples(inst.t, inst.c, n)
    T = O.toeplitz(grid, d, n, 0)
    U, s, V = O.reduced_svd(T, m)
    rng = _rng(60)
    U0 = random_orthonormal(rng, T.shape[0], 2 * m)
    V0 = random_orthonormal(rng, T.shape[0], 2 * m)
    Up, sp, Vp, rank, sweeps = O.block_power_svd(T, U0, V0, tol=T.shape[0] * O.EPS64)
    assert rank == m and sweeps >= 1
    assert np.allclose(sp, s, rtol=1e-12, atol=0)
    assert np.linalg.norm(Up @ Up.conj().T - U @ U.conj().T) < 1e-11
    assert np.linalg.norm(Vp @ Vp.conj().T - V @ V.conj().T) < 1e-11
    assert np.linalg.norm(Up @ np.diag(sp) @ Vp.conj().T - T) < 1e-12 * np.linalg.norm(T)
    # closed form: V_z = Q R gives T = Q (R diag(c) R^*) Q^*, so sigma(T) = sigma(R diag(c) R^*)
    Q, R = np.linalg.qr(_vz(inst.t, d, n))
    s_closed = np.linalg.svd(R @ np.diag(inst.c) @ R.conj().T, compute_uv=False)
    assert np.allclose(np.sort(s_closed)[::-1], s, rtol=1e-12)


def test_hoffman_wielandt_bound_under_noise():
    # sqrt(sum (sigma~_i - sigma_i)^2) <= ||Delta T||_F (Sec. 4)
    inst = config_instances("c0")[0]
    d, n = inst.d, inst.n
    clean = O.samples(inst.t, inst.c, n)
    noise = 1e-4 * inst.noise_unit
    T = O.toeplitz(clean, d, n, 0)
    Tn = O.toeplitz(clean + noise, d, n, 0)
    s = np.linalg.svd(T, compute_uv=False)
    sn = np.linalg.svd(Tn, compute_uv=False)
    assert np.sqrt(np.sum((sn - s) ** 2)) <= np.linalg.norm(Tn - T)
    # rank criterion sigma~_{m+1} <= ||Delta T||_F (Sec. 4, eq. rank_crit)
    assert sn[inst.m] <= np.linalg.norm(Tn - T)


def test_rank_detection_matches_printed_results(golden_dir):
    rows = [line.split() for line in open(f"{golden_dir}/rank_detection.txt")
            if line.strip() and not line.startswith("#")]
    for d, n, m, rel in rows:
        d, n, m = int(d), int(n), int(m)
        t, c = paper_efficiency_inputs(d, m)
        T = O.toeplitz(O.samples(t, c, n), d, n, 0)
        s = np.linalg.svd(T, compute_uv=False)
        rank = O.numerical_rank(s, T.shape[0] * O.EPS64)
        rng = _rng(70 + m)
        _, _, _, rank_power, _ = O.block_power_svd(
            T, random_orthonormal(rng, T.shape[0], 2 * m), random_orthonormal(rng, T.shape[0], 2 * m),
            tol=T.shape[0] * O.EPS64)
        if rel == "eq":
            assert rank == m and rank_power == m
        else:
            assert rank < m and rank_power < m


# ---------------------------------------------------------------- pencil S_l


def _c0_pencil(with_s0=True):
    inst = config_instances("c0")[0]
    d, n, m = inst.d, inst.n, inst.m
    grid = O.samples(inst.t, inst.c, n)
    U, s, V = O.reduced_svd(O.toeplitz(grid, d, n, 0), m)
    S = O.pencil_matrices(grid, d, n, U, s, V, with_s0=with_s0)
    return inst, grid, U, s, V, S


def test_s0_is_identity_and_eigenvalues_are_nodes():
    inst, grid, U, s, V, S = _c0_pencil()
    assert np.max(np.abs(S[0] - np.eye(inst.m))) < 1e-13
    for ell in range(1, inst.d + 1):
        z_true = np.exp(-2j * np.pi * inst.t[:, ell - 1])
        ev = np.linalg.eigvals(S[ell])
        dist = np.abs(ev[:, None] - z_true[None, :])
        assert np.max(np.min(dist, axis=1)) < 1e-12
        assert abs(np.trace(S[ell]) - np.sum(z_true)) < 1e-12


def test_pencil_factored_closed_form():
    # S_l = (U^* V_z) diag(c_j z_j(l)) (V_z^* V) Sigma^{-1}
    inst, grid, U, s, V, S = _c0_pencil(with_s0=False)
    Vz = _vz(inst.t, inst.d, inst.n)
    for ell in range(1, inst.d + 1):
        zl = np.exp(-2j * np.pi * inst.t[:, ell - 1])
        ref = (U.conj().T @ Vz) @ np.diag(inst.c * zl) @ (Vz.conj().T @ V) @ np.diag(1 / s)
        assert np.linalg.norm(S[ell - 1] - ref) < 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("d,n,m", [(1, 3, 2), (2, 2, 2)])
def test_pencil_50_digit_brute_force(d, n, m):
    rng = _rng(80 + d)
    G = (2 * n + 2) ** d
    N = (n + 1) ** d
    grid = rng.standard_normal(G) + 1j * rng.standard_normal(G)
    U = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
    V = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
    sig = rng.uniform(0.5, 2.0, m)
    S = O.pencil_matrices(grid, d, n, U, sig, V)
    table = {p: grid[i] for i, p in enumerate(itertools.product(range(-n, n + 2), repeat=d))}
    ks = list(itertools.product(range(n + 1), repeat=d))
    for ell in range(1, d + 1):
        for i in range(m):
            for j in range(m):
                acc = mpmath.mpc(0)
                for a, k in enumerate(ks):
                    for b, h in enumerate(ks):
                        p = tuple(k[x] - h[x] + (1 if x == ell - 1 else 0) for x in range(d))
                        acc += (mpmath.mpc(complex(U[a, i])).conjugate() * mpmath.mpc(complex(table[p]))
                                * mpmath.mpc(complex(V[b, j])))
                acc /= mpmath.mpf(float(sig[j]))
                assert abs(complex(acc) - S[ell - 1, i, j]) < 1e-13 * abs(complex(acc)) + 1e-13


def test_pencil_invariant_under_reordering_of_index_set():
    # Any consistent reordering P of I_n: T -> P T P^T, U -> P U, V -> P V leaves S_l unchanged.
    inst, grid, U, s, V, S = _c0_pencil(with_s0=False)
    perm = _rng(90).permutation(U.shape[0])
    for ell in range(1, inst.d + 1):
        Tl = O.toeplitz(grid, inst.d, inst.n, ell)[np.ix_(perm, perm)]
        Sp = U[perm].conj().T @ Tl @ V[perm] @ np.diag(1 / s)
        assert np.allclose(Sp, S[ell - 1], atol=1e-12)


def test_input_perturbation_bound():
    # ||U^* Delta T_l V Sigma^{-1}||_F <= ||Delta T_l||_F / sigma_m (Sec. 4, eq. deltaSl1)
    inst, grid, U, s, V, S = _c0_pencil(with_s0=False)
    noise = 1e-3 * inst.noise_unit
    Sn = O.pencil_matrices(grid + noise, inst.d, inst.n, U, s, V)
    for ell in range(1, inst.d + 1):
        dT = O.toeplitz(noise, inst.d, inst.n, ell)
        assert np.linalg.norm(Sn[ell - 1] - S[ell - 1]) <= np.linalg.norm(dT) / s[-1] * (1 + 1e-12)


# ---------------------------------------------------------------- Vandermonde / LS


def _dirichlet(w, n):
    return np.where(np.abs(w - 1) < 1e-12, n + 1, (1 - w ** (n + 1)) / np.where(np.abs(w - 1) < 1e-12, 1, 1 - w))


@pytest.mark.parametrize("d,n,m", [(1, 12, 4), (2, 6, 5), (3, 3, 4)])
def test_gram_closed_form_and_exact_rhs(d, n, m):
    # G_ij = prod_l D_n(conj(z_i(l)) z_j(l)) with D_n(w) = (1 - w^{n+1})/(1 - w); noise-free rhs = G c
    t, c = _random_problem(100 + d, d, m)
    z = np.exp(-2j * np.pi * t)
    grid = O.samples(t, c, n)
    gram, rhs = O.coefficient_products(z, grid, d, n)
    ref = np.ones((m, m), dtype=complex)
    for ell in range(d):
        ref *= _dirichlet(np.conj(z[:, None, ell]) * z[None, :, ell], n)
    assert np.max(np.abs(gram - ref)) < 1e-11 * (n + 1) ** d
    assert np.max(np.abs(rhs - gram @ c)) < 1e-11 * (n + 1) ** d
    cs, resid = O.least_squares_coefficients(z, grid, d, n)
    assert np.max(np.abs(cs - c)) < 1e-12 and resid < 1e-13


def test_vandermonde_matches_direct_exponentials():
    t, c = _random_problem(110, 3, 4)
    z = np.exp(-2j * np.pi * t)
    assert np.max(np.abs(O.vandermonde_transpose(z, 3, 3) - _vz(t, 3, 3))) < 1e-13


# ---------------------------------------------------------------- end to end


def test_c0_noise_free_exact_recovery():
    inst = config_instances("c0")[0]
    grid = O.samples(inst.t, inst.c, inst.n)
    res = O.prony(grid, inst.d, inst.n, inst.m, inst.mu)
    dt, dc = O.recovery_errors(res, inst.t, inst.c)
    assert res["rank"] == inst.m
    assert dt < 1e-12 and dc < 1e-10 and res["resid"] < 1e-13


def test_c0_power_svd_route_recovers_too():
    inst = config_instances("c0")[0]
    grid = O.samples(inst.t, inst.c, inst.n)
    rng = _rng(120)
    N = inst.N
    blocks = (random_orthonormal(rng, N, 2 * inst.m), random_orthonormal(rng, N, 2 * inst.m))
    res = O.prony(grid, inst.d, inst.n, inst.m, inst.mu, svd="power", start_blocks=blocks)
    dt, dc = O.recovery_errors(res, inst.t, inst.c)
    assert dt < 1e-12 and dc < 1e-10


def test_one_dimensional_case_agrees_with_prony_polynomial_roots():
    # d = 1: the nodes are the roots of the linear-prediction polynomial
    # sum_{i<=m} p_i f(k + i) = 0, p_m = 1, solved from the Hankel system.
    t, c = _random_problem(130, 1, 4)
    n = 11
    grid = O.samples(t, c, n)
    res = O.prony(grid, 1, n, 4, np.array([1.0 + 0j]))
    fk = grid[n:n + n + 1]                      # f(0..n)
    m = 4
    H = np.array([[fk[k + i] for i in range(m)] for k in range(n + 1 - m)])
    rhs = -np.array([fk[k + m] for k in range(n + 1 - m)])
    p = np.linalg.lstsq(H, rhs, rcond=None)[0]
    roots = np.roots(np.concatenate([[1.0], p[::-1]]))
    t_roots = np.mod(-np.angle(roots) / (2 * np.pi), 1.0)
    assert np.max(np.abs(np.sort(t_roots) - np.sort(res["t"][:, 0]))) < 1e-10


def test_error_proportional_to_noise():
    # forward errors of t and c scale with the input error (Sec. 4 conclusion, Sec. 5)
    inst = config_instances("c0")[0]
    clean = O.samples(inst.t, inst.c, inst.n)
    errs = []
    for eps in (1e-9, 1e-6):
        res = O.prony(clean + eps * inst.noise_unit, inst.d, inst.n, inst.m, inst.mu)
        errs.append(O.recovery_errors(res, inst.t, inst.c))
    for k in range(2):
        ratio = errs[1][k] / errs[0][k]
        assert 1e2 < ratio < 1e4


@pytest.mark.slow
def test_table1_orders_of_magnitude(golden_dir):
    rows = [line.split() for line in open(f"{golden_dir}/table1_accuracy.txt")
            if line.strip() and not line.startswith("#")]
    d, n, m = 3, 20, 5
    t, c = paper_efficiency_inputs(d, m)
    clean = O.samples(t, c, n)
    N = (n + 1) ** d
    mu = np.array([1.0, 1j, -0.5]) / np.linalg.norm([1.0, 1j, -0.5])
    rng = _rng(140)
    blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
    for eps_s, _, r_res, r_dt, r_dc in rows:
        eps = float(eps_s)
        if eps not in (0.0, 1e-6):
            continue
        grid = O.samples(t, c, n, rel_noise=paper_relative_noise(1, d, n, eps)) if eps else clean
        res = O.prony(grid, d, n, m, mu, svd="power", start_blocks=blocks)
        dt, dc = O.recovery_errors(res, t, c)
        got = (res["resid"], dt, dc)
        for g, r in zip(got, (float(r_res), float(r_dt), float(r_dc))):
            if eps == 0.0:
                assert g < 10 * r          # rounding level: an upper bound only
            else:
                assert r / 10 < g < 10 * r  # same decade band as the printed value


# ---------------------------------------------------------------- adjoint


def _adjoint_case():
    inst = config_instances("c4", count=1)[0]
    d, m = 2, 4
    n = 5
    rng = _rng(150)
    t, c = _random_problem(151, d, m)
    clean = O.samples(t, c, n)
    noisy = clean + 1e-3 * rng.standard_normal(clean.size)
    U, s, V = O.reduced_svd(O.toeplitz(noisy, d, n, 0), m)
    ref = O.pencil_matrices(clean, d, n, U, s, V)
    del inst
    return d, n, m, clean, noisy, U, s, V, ref


def test_adjoint_dot_product_identity():
    d, n, m, clean, noisy, U, s, V, ref = _adjoint_case()
    rng = _rng(160)
    gS = rng.standard_normal((d, m, m)) + 1j * rng.standard_normal((d, m, m))
    df = rng.standard_normal(clean.size) + 1j * rng.standard_normal(clean.size)
    lhs = np.vdot(gS, O.pencil_matrices(df, d, n, U, s, V)).real
    rhs = np.vdot(O.pencil_adjoint(gS, d, n, U, s, V), df).real
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_adjoint_matches_central_differences():
    d, n, m, clean, noisy, U, s, V, ref = _adjoint_case()
    S = O.pencil_matrices(noisy, d, n, U, s, V)
    grad = O.pencil_adjoint(2 * (S - ref), d, n, U, s, V)
    rng = _rng(170)
    h = 1e-7
    for _ in range(3):
        v = rng.standard_normal(clean.size) + 1j * rng.standard_normal(clean.size)
        # the loss depends on f only through f - f0; evaluating on the difference avoids cancellation
        lp = O.pencil_loss(noisy - clean + h * v, ref * 0, d, n, U, s, V)
        lm = O.pencil_loss(noisy - clean - h * v, ref * 0, d, n, U, s, V)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - np.vdot(grad, v).real) < 1e-6 * abs(fd)


def test_adjoint_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    d, n, m, clean, noisy, U, s, V, ref = _adjoint_case()
    f = torch.tensor(noisy, dtype=torch.complex128, requires_grad=True)
    Ut, Vt = torch.tensor(U), torch.tensor(V)
    st = torch.tensor(s)
    reft = torch.tensor(ref)
    ks = torch.tensor(list(itertools.product(range(n + 1), repeat=d)))
    loss = 0
    for ell in range(1, d + 1):
        e = torch.zeros(d, dtype=torch.long)
        e[ell - 1] = 1
        p = ks[:, None, :] - ks[None, :, :] + e + n
        flat = torch.zeros(p.shape[:2], dtype=torch.long)
        for a in range(d):
            flat = flat * (2 * n + 2) + p[..., a]
        Tl = f[flat]
        Sl = Ut.conj().T @ Tl @ Vt / st
        loss = loss + torch.sum(torch.abs(Sl - reft[ell - 1]) ** 2)
    loss.backward()
    S = O.pencil_matrices(noisy, d, n, U, s, V)
    grad = O.pencil_adjoint(2 * (S - ref), d, n, U, s, V)
    g = f.grad.numpy()
    assert np.linalg.norm(g - grad) < 1e-10 * np.linalg.norm(grad)


# ---------------------------------------------------------------- Lanczos bidiagonalization (Alg. 2)


def _low_rank(rng, rows, cols, sv):
    X = np.linalg.qr(rng.standard_normal((rows, len(sv))) + 1j * rng.standard_normal((rows, len(sv))))[0]
    Y = np.linalg.qr(rng.standard_normal((cols, len(sv))) + 1j * rng.standard_normal((cols, len(sv))))[0]
    return X @ np.diag(sv) @ Y.conj().T, X, Y


def _vectors(rng, n, count):
    return [rng.standard_normal(n) + 1j * rng.standard_normal(n) for _ in range(count)]


@pytest.mark.parametrize("d,n,r", [(1, 5, 3), (2, 3, 2), (3, 2, 2)])
def test_toeplitz_product_is_an_fft_convolution(d, n, r):
    # (T X)[k] = sum_h f(k - h) X[h]: with F[p + n] = f(p), p in {-n..n+1}^d, the linear
    # convolution C = F * X (by zero-padded FFTs) has (T X)[k] = C[k + n]
    rng = _rng(300 + 10 * d + n)
    G = (2 * n + 2) ** d
    grid = rng.standard_normal(G) + 1j * rng.standard_normal(G)
    X = rng.standard_normal(((n + 1) ** d, r)) + 1j * rng.standard_normal(((n + 1) ** d, r))
    L = (2 * n + 2) + (n + 1) - 1
    axes = tuple(range(d))
    F = np.fft.fftn(grid.reshape((2 * n + 2,) * d), s=(L,) * d, axes=axes)
    Y = np.empty_like(X)
    for q in range(r):
        C = np.fft.ifftn(F * np.fft.fftn(X[:, q].reshape((n + 1,) * d), s=(L,) * d, axes=axes), axes=axes)
        Y[:, q] = C[(slice(n, 2 * n + 1),) * d].reshape(-1)
    got = O.toeplitz_product(grid, d, n, X)
    assert np.max(np.abs(got - Y)) < 1e-12 * np.max(np.abs(Y))


def test_toeplitz_product_adjoint_dot_product_identity():
    # <T X, Y> = <X, T^* Y> for random complex X, Y
    rng = _rng(310)
    d, n, r = 2, 4, 3
    G, N = (2 * n + 2) ** d, (n + 1) ** d
    grid = rng.standard_normal(G) + 1j * rng.standard_normal(G)
    X = rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r))
    Y = rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r))
    lhs = np.vdot(O.toeplitz_product(grid, d, n, X), Y)
    rhs = np.vdot(X, O.toeplitz_product(grid, d, n, Y, adjoint=True))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_lanczos_recovers_prescribed_singular_values_and_rank():
    rng = _rng(900)
    sv = np.array([7.0, 3.0, 2.5, 1.0, 0.25, 0.01])
    A, X, Y = _low_rank(rng, 80, 70, sv)
    U, s, V, rank = O.lanczos_bidiagonalization(A, _vectors(rng, 70, 1)[0], 80 * O.EPS64, _vectors(rng, 80, 8))
    assert rank == len(sv)
    assert np.max(np.abs(s[:rank] - sv) / sv) < 1e-12
    # A V = U Sigma and A^* U = V Sigma on the detected triplets; orthonormal bases
    assert np.linalg.norm(A @ V[:, :rank] - U[:, :rank] * s[:rank]) < 1e-12 * sv[0]
    assert np.linalg.norm(A.conj().T @ U[:, :rank] - V[:, :rank] * s[:rank]) < 1e-12 * sv[0]
    assert np.linalg.norm(U[:, :rank].conj().T @ U[:, :rank] - np.eye(rank)) < 1e-12


def test_lanczos_restarts_after_an_early_stop():
    # p1 in the span of two right singular vectors: the plain recurrence stops after
    # two steps; the early-stop check must detect it and restart to the full rank
    rng = _rng(901)
    sv = np.array([5.0, 3.0, 2.0, 1.0, 0.5])
    A, X, Y = _low_rank(rng, 60, 60, sv)
    U, s, V, rank = O.lanczos_bidiagonalization(A, Y[:, 0] + 2 * Y[:, 2], 60 * O.EPS64, _vectors(rng, 60, 8))
    assert rank == len(sv)
    assert np.max(np.abs(s[:rank] - sv) / sv) < 1e-12


def test_lanczos_matches_lapack_on_toeplitz_and_paper_ranks(golden_dir):
    inst = config_instances("c0")[0]
    grid = O.samples(inst.t, inst.c, inst.n)
    T = O.toeplitz(grid, inst.d, inst.n, 0)
    N = T.shape[0]
    rng = _rng(902)
    U, s, V, rank = O.lanczos_bidiagonalization(T, _vectors(rng, N, 1)[0], N * O.EPS64, _vectors(rng, N, 8))
    s_ref = np.linalg.svd(T, compute_uv=False)
    assert rank == inst.m
    assert np.max(np.abs(s[:inst.m] - s_ref[:inst.m]) / s_ref[:inst.m]) < 1e-11
    # Sec. 5: all SVD methods found the same (sometimes deficient) rank at d = 2, n = 20
    rows = [line.split() for line in open(f"{golden_dir}/rank_detection.txt")
            if line.strip() and not line.startswith("#")]
    for d, n, m, rel in rows:
        d, n, m = int(d), int(n), int(m)
        t, c = paper_efficiency_inputs(d, m)
        T = O.toeplitz(O.samples(t, c, n), d, n, 0)
        N = T.shape[0]
        rng = _rng(903 + m)
        _, _, _, rank = O.lanczos_bidiagonalization(T, _vectors(rng, N, 1)[0], N * O.EPS64, _vectors(rng, N, 8))
        assert (rank == m) if rel == "eq" else (rank < m), (d, n, m, rank)
