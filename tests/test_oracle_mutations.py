"""Strength of the oracle pins: plant plausible mistakes in the oracle (on the CPU)
and check that at least one pin of test_oracle_pins fails for each of them."""
import numpy as np
import pytest

import tests.test_oracle_pins as pins
from oracle import prony_oracle as O

_orig = {name: getattr(O, name) for name in
         ("samples", "toeplitz", "pencil_matrices", "vandermonde_transpose", "pencil_adjoint",
          "nodes_from_pencil", "coefficient_products", "toeplitz_product", "lanczos_bidiagonalization",
          "_reorthogonalize")}


def _samples_wrong_sign(t, c, n, abs_noise=None, rel_noise=None):
    return np.conj(_orig["samples"](t, np.conj(c), n, abs_noise, rel_noise))


def _toeplitz_transposed(grid, d, n, ell):
    return _orig["toeplitz"](grid, d, n, ell).T


def _toeplitz_shift_backwards(grid, d, n, ell):
    # f(k - h - e_l) instead of f(k - h + e_l): T_l built from T with the opposite shift
    if ell == 0:
        return _orig["toeplitz"](grid, d, n, 0)
    Q = 2 * n + 2
    g = grid.reshape((Q,) * d)
    g = np.roll(g, 2, axis=ell - 1).reshape(-1)
    return _orig["toeplitz"](g, d, n, ell)


def _pencil_u_transpose(grid, d, n, U, sigma, V, with_s0=False):
    return _orig["pencil_matrices"](grid, d, n, U.conj(), sigma, V, with_s0)


def _pencil_sigma_left(grid, d, n, U, sigma, V, with_s0=False):
    S = _orig["pencil_matrices"](grid, d, n, U, np.ones_like(sigma), V, with_s0)
    return S / np.asarray(sigma)[None, :, None]


def _vandermonde_conj(z, d, n):
    return _orig["vandermonde_transpose"](np.conj(z), d, n)


def _adjoint_missing_conj(gS, d, n, U, sigma, V):
    return _orig["pencil_adjoint"](gS, d, n, U, sigma, V.conj())


def _nodes_wrong_sign(S, mu):
    z, t, W = _orig["nodes_from_pencil"](S, mu)
    return z, np.mod(-t, 1.0), W


def _product_ignores_adjoint(grid, d, n, X, adjoint=False):
    return _orig["toeplitz_product"](grid, d, n, X, adjoint=False)


def _product_transpose_without_conjugate(grid, d, n, X, adjoint=False):
    T = _orig["toeplitz"](grid, d, n, 0)
    return (T.T if adjoint else T) @ X


def _product_reversed_shift(grid, d, n, X, adjoint=False):
    # f(h - k) instead of f(k - h)
    T = _orig["toeplitz"](grid, d, n, 0)
    return (T.conj() if adjoint else T.T) @ X


def _no_reorthogonalization(x, Q):
    return x


def _lanczos_stops_at_first_small_coefficient(A, p1, tol, restart_vectors=(), max_steps=None):
    # the early-stop check skipped: a zero test vector makes every small coefficient end the process
    zeros = [np.zeros(max(A.shape), dtype=complex)[: A.shape[1]] for _ in range(8)]
    return _orig["lanczos_bidiagonalization"](A, p1, tol, zeros, max_steps)


MUTANTS = [
    ("samples", _samples_wrong_sign,
     [pins.test_samples_on_rational_nodes_are_an_fft, pins.test_toeplitz_vandermonde_factorisation]),
    ("toeplitz", _toeplitz_transposed, [pins.test_toeplitz_brute_force]),
    ("toeplitz", _toeplitz_shift_backwards, [pins.test_toeplitz_brute_force]),
    ("pencil_matrices", _pencil_u_transpose, [pins.test_s0_is_identity_and_eigenvalues_are_nodes]),
    ("pencil_matrices", _pencil_sigma_left, [pins.test_pencil_factored_closed_form]),
    ("vandermonde_transpose", _vandermonde_conj, [pins.test_vandermonde_matches_direct_exponentials]),
    ("pencil_adjoint", _adjoint_missing_conj, [pins.test_adjoint_dot_product_identity]),
    ("nodes_from_pencil", _nodes_wrong_sign, [pins.test_c0_noise_free_exact_recovery]),
    ("toeplitz_product", _product_ignores_adjoint, [pins.test_toeplitz_product_adjoint_dot_product_identity]),
    ("toeplitz_product", _product_transpose_without_conjugate,
     [pins.test_toeplitz_product_adjoint_dot_product_identity]),
    ("toeplitz_product", _product_reversed_shift, [pins.test_toeplitz_product_is_an_fft_convolution]),
    ("_reorthogonalize", _no_reorthogonalization,
     [pins.test_lanczos_recovers_prescribed_singular_values_and_rank, pins.test_lanczos_restarts_after_an_early_stop]),
    ("lanczos_bidiagonalization", _lanczos_stops_at_first_small_coefficient,
     [pins.test_lanczos_restarts_after_an_early_stop]),
]


def _run(pin):
    import inspect
    params = inspect.signature(pin).parameters
    kwargs = {}
    if "d" in params:   # parametrised pins: use their first parameter set
        marks = [m for m in getattr(pin, "pytestmark", []) if m.name == "parametrize"]
        names = [n.strip() for n in marks[0].args[0].split(",")]
        kwargs = dict(zip(names, marks[0].args[1][0]))
    if "golden_dir" in params:
        kwargs["golden_dir"] = pins.__file__.rsplit("/", 1)[0] + "/golden"
    pin(**kwargs)


@pytest.mark.parametrize("target,mutant,checks", MUTANTS, ids=[m[1].__name__ for m in MUTANTS])
def test_pins_catch_planted_mistake(monkeypatch, target, mutant, checks):
    monkeypatch.setattr(O, target, mutant)
    caught = 0
    for pin in checks:
        try:
            _run(pin)
        except AssertionError:
            caught += 1
    assert caught > 0, f"no pin caught the mutant {mutant.__name__}"


def test_unmutated_pins_pass():
    for _, _, checks in MUTANTS:
        for pin in checks:
            _run(pin)
