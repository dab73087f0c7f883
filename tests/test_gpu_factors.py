"""Prepared factors (prony_factors_create / prony_build_S_factors): U, sigma and V
packed once, S-builds with several sample grids. The result is bitwise the one
prony_build_S gives under the same plan, it matches the oracle (Sec. 1, eq.
generateSl) to the precision's bound, it does not depend on the caller's copies of
the factors after creation, and a captured build replays to the eager result."""
import gc

import numpy as np
import pytest
import torch

from oracle import prony_oracle as O
from paper_2012_11430_amd import _lib, api
from tests._close import assert_close_per_matrix
from workload import random_orthonormal

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5}


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _problem(d, n, m, seed, grids=2):
    rng = np.random.Generator(np.random.PCG64(seed))
    N, G = (n + 1) ** d, (2 * n + 2) ** d
    fs = [rng.standard_normal(G) + 1j * rng.standard_normal(G) for _ in range(grids)]
    U, V = random_orthonormal(rng, N, m), random_orthonormal(rng, N, m)
    s = rng.uniform(0.5, 2.0, m)
    return fs, U, s, V


_ORACLE = {}


def _oracle(key, grid, d, n, U, s, V, with_s0):
    # one oracle evaluation per (shape, grid), shared by the three precisions
    if key not in _ORACLE:
        _ORACLE[key] = O.pencil_matrices(grid, d, n, U, s, V, with_s0=with_s0)
    return _ORACLE[key]


@pytest.mark.parametrize("d,n,m,with_s0,grids", [(2, 63, 20, False, 2), (3, 7, 5, True, 2), (1, 200, 17, False, 2),
                                                 (3, 19, 30, False, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_factors_match_build_S_bitwise_and_the_oracle(prec, d, n, m, with_s0, grids):
    fs, U, s, V = _problem(d, n, m, seed=31 + d + m, grids=grids)
    Ud, sd, Vd = _dev(U), _dev(s), _dev(V)
    F = api.Factors(d, n, Ud, sd, Vd, prec=prec, with_s0=with_s0)
    try:
        for i, grid in enumerate(fs):
            f = _dev(grid)
            got = F.build_S(f)
            ref = api.build_S(f, d, n, Ud, sd, Vd, prec=prec, with_s0=with_s0)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), f"grid {i}: prepared factors differ from prony_build_S"
            oracle = _oracle((d, n, m, with_s0, i), grid, d, n, U, s, V, with_s0)
            assert_close_per_matrix(got.cpu().numpy(), oracle, TOL[prec], f"{prec} grid {i}")
    finally:
        F.close()


def test_factors_own_their_packed_copy():
    d, n, m = 2, 31, 12
    fs, U, s, V = _problem(d, n, m, seed=41, grids=1)
    f = _dev(fs[0])
    Ud, sd, Vd = _dev(U), _dev(s), _dev(V)
    F = api.Factors(d, n, Ud, sd, Vd, prec="fp32")
    ref = F.build_S(f).clone()
    torch.cuda.synchronize()
    # overwrite and release the caller's tensors; the next allocations may reuse their memory
    Ud.fill_(float("nan"))
    Vd.zero_()
    sd.fill_(-1.0)
    del Ud, Vd, sd
    gc.collect()
    junk = [torch.full((8 << 20,), 7.0, dtype=torch.float64, device=DEV) for _ in range(2)]
    got = F.build_S(f)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    del junk
    F.close()
    with pytest.raises(ValueError):
        F.build_S(f)


def _capture(fn):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream(DEV)
    s.wait_stream(torch.cuda.current_stream(DEV))
    with torch.cuda.stream(s):
        api.synchronize(DEV)
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            fn()
    torch.cuda.current_stream(DEV).wait_stream(s)
    return g


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_captured_factor_build_replays_the_eager_result(prec):
    d, n, m = 3, 19, 30
    fs, U, s, V = _problem(d, n, m, seed=43, grids=1)
    f = _dev(fs[0])
    F = api.Factors(d, n, _dev(U), _dev(s), _dev(V), prec=prec)
    out = torch.empty((d, m, m), dtype=torch.complex128, device=DEV)
    eager = F.build_S(f)            # the first build sizes the handle's workspace
    torch.cuda.synchronize()
    g = _capture(lambda: F.build_S(f, out=out))
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"
        (torch.randn(4096, device=DEV) * 3).sum().item()   # unrelated eager work between replays
    f.mul_(2.0)          # S is linear in f; scaling by 2 is exact in every precision
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, 2.0 * eager)
    del g
    F.close()


def test_factors_info_reports_the_shape():
    import ctypes
    d, n, m = 2, 15, 5
    fs, U, s, V = _problem(d, n, m, seed=47, grids=1)
    F = api.Factors(d, n, _dev(U), _dev(s), _dev(V), prec="bf16x3", with_s0=True)
    vals = [ctypes.c_int() for _ in range(4)]
    flags = ctypes.c_uint()
    lib = _lib.load()
    assert lib.prony_factors_info(F.handle, *[ctypes.byref(v) for v in vals], ctypes.byref(flags)) == _lib.PRONY_OK
    assert [v.value for v in vals] == [d, n, m, _lib.PRONY_BF16X3]
    assert flags.value == _lib.PRONY_WITH_S0
    F.close()
