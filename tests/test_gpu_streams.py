"""Calls through the one library handle on two torch streams: the library orders
the second stream after the first one's queued work (the handle's workspace is
shared), so both results match the oracle whatever the timing.

Also the failure behaviours of the single-instance S-build: NaN samples propagate
to S (no hang, no error), a capture that would need the workspace to grow returns
PRONY_ECAPTURE, and a capture after prony_reserve replays to the eager result.
"""
import numpy as np
import pytest
import torch

from oracle import prony_oracle as O
from paper_2012_11430_amd import _lib, api, autotune
from tests._close import assert_close_per_matrix
from workload import random_orthonormal

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _random_problem(d, n, m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    N, G = (n + 1) ** d, (2 * n + 2) ** d
    grid = rng.standard_normal(G) + 1j * rng.standard_normal(G)
    U, V = random_orthonormal(rng, N, m), random_orthonormal(rng, N, m)
    s = rng.uniform(0.5, 2.0, m)
    return grid, U, s, V


def test_build_S_on_two_streams_back_to_back():
    # a large S-build on stream A, then at once a different one on stream B; the
    # second call's packing would overwrite the first call's operands in the shared
    # workspace if B did not wait for A's queued work
    big = (2, 63, 20)
    small = (3, 9, 12)
    pa = _random_problem(*big, seed=1)
    pb = _random_problem(*small, seed=2)
    da = [_dev(x) for x in pa]
    db = [_dev(x) for x in pb]
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(DEV), torch.cuda.Stream(DEV)
    for prec in ("fp32", "fp64"):
        outs = []
        for _ in range(3):
            with torch.cuda.stream(sa):
                ra = api.build_S(da[0], big[0], big[1], da[1], da[2], da[3], prec=prec)
            with torch.cuda.stream(sb):
                rb = api.build_S(db[0], small[0], small[1], db[1], db[2], db[3], prec=prec)
            outs.append((ra, rb))
        torch.cuda.synchronize()
        tol = 1e-12 if prec == "fp64" else 1e-5
        ref_a = O.pencil_matrices(pa[0], big[0], big[1], pa[1], pa[2], pa[3])
        ref_b = O.pencil_matrices(pb[0], small[0], small[1], pb[1], pb[2], pb[3])
        for ra, rb in outs:
            assert_close_per_matrix(ra.cpu().numpy(), ref_a, tol, f"stream A {prec}")
            assert_close_per_matrix(rb.cpu().numpy(), ref_b, tol, f"stream B {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_nan_samples_propagate(prec):
    # A NaN sample at p = 0 enters every T_l: every entry of every S_l is NaN, as in
    # the oracle, and the call completes. A NaN at the grid's edge enters only some
    # T_l in the definition; the kernels multiply every staged sample, zero-padded
    # factors included, so its NaN reaches at least the oracle's NaN entries.
    d, n, m = 2, 12, 6
    grid, U, s, V = _random_problem(d, n, m, seed=5)
    center = n * (2 * n + 2) + n
    for where in (center, 7):
        g = grid.copy()
        g[where] = np.nan
        S = api.build_S(_dev(g), d, n, _dev(U), _dev(s), _dev(V), prec=prec).cpu().numpy()
        ref = O.pencil_matrices(g, d, n, U, s, V)
        assert np.isnan(ref).any()
        if where == center:
            assert np.isnan(ref).all() and np.isnan(S).all()
        else:
            assert np.all(np.isnan(S)[np.isnan(ref)])


def _capture(fn):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream(DEV)
    s.wait_stream(torch.cuda.current_stream(DEV))
    with torch.cuda.stream(s):
        api.synchronize(DEV)          # the handle now runs on s, outside capture
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            fn()
    torch.cuda.current_stream(DEV).wait_stream(s)
    return g


def test_capture_needing_workspace_growth_returns_ecapture():
    # a fresh handle (no workspace yet) whose first S-build is enqueued under
    # capture: the workspace would have to grow, which is refused (nothing launched)
    import ctypes
    lib = _lib.load()
    d, n, m = 2, 15, 5
    grid, U, s, V = _random_problem(d, n, m, seed=9)
    f, Ud, sd, Vd = _dev(grid), _dev(U), _dev(s), _dev(V)
    out = torch.empty((d, m, m), dtype=torch.complex128, device=DEV)
    h = ctypes.c_void_p()
    assert lib.prony_create(ctypes.byref(h), DEV.index or 0) == _lib.PRONY_OK
    status = []
    try:
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream(DEV)
        cs.wait_stream(torch.cuda.current_stream(DEV))
        torch.cuda.synchronize()
        with torch.cuda.stream(cs):
            with torch.cuda.graph(g, stream=cs, capture_error_mode="thread_local"):
                assert lib.prony_set_stream(h, ctypes.c_void_p(cs.cuda_stream)) == _lib.PRONY_OK
                status.append(lib.prony_build_S(h, d, n, m, ctypes.c_void_p(f.data_ptr()),
                                                ctypes.c_void_p(Ud.data_ptr()), m, 1, ctypes.c_void_p(sd.data_ptr()),
                                                ctypes.c_void_p(Vd.data_ptr()), m, 1, _lib.PRONY_FP32, 0,
                                                ctypes.c_void_p(out.data_ptr())))
                status.append(lib.prony_last_error(h).decode())
        torch.cuda.synchronize()
    finally:
        assert lib.prony_destroy(h) == _lib.PRONY_OK
    assert status[0] == _lib.PRONY_ECAPTURE, status
    assert "prony_reserve" in status[1]


@pytest.mark.parametrize("prec,target_per_cu,with_s0", [("fp32", 8, False), ("bf16x3", 0, True),
                                                        ("fp64", 8, True)])
def test_capture_after_reserve_replays_the_eager_result(prec, target_per_cu, with_s0):
    # prony_reserve sizes the workspace for every plan of the shape (split target
    # registered here, the split-bfloat16 plan, S_0), so the capture allocates nothing
    d, n, m = 3, 19, 30
    cus = torch.cuda.get_device_properties(DEV).multi_processor_count
    grid, U, s, V = _random_problem(d, n, m, seed=11)
    f = _dev(grid)
    args = (f, d, n, _dev(U), _dev(s), _dev(V))
    ells = d + (1 if with_s0 else 0)
    out = torch.empty((ells, m, m), dtype=torch.complex128, device=DEV)
    try:
        autotune.register(DEV, d, n, m, prec, False, target_per_cu * cus)
        api.reserve(DEV, d, n, m)
        torch.cuda.synchronize()
        g = _capture(lambda: api.build_S(*args, prec=prec, with_s0=with_s0, out=out))
        eager = api.build_S(*args, prec=prec, with_s0=with_s0)
        torch.cuda.synchronize()
        for rep in range(3):
            out.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"replay {rep}"
            (torch.randn(4096, device=DEV) * 3).sum().item()   # unrelated eager work between replays
        f.mul_(2.0)      # S is linear in f; scaling by 2 is exact in every precision
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, 2.0 * eager)
    finally:
        autotune.register(DEV, d, n, m, prec, False, 0)
