"""prony_build_S_noalloc (the S-build for callers that cannot allocate device
memory: its scratch is the library's fixed per-device array) against
prony_build_S, through the C ABI, on two calls in a row, the second smaller,
and against the oracle at the bar of the S-build parity tests.
"""
import numpy as np
import pytest
import torch

from oracle import prony_oracle as O
from paper_2012_11430_amd import _lib, api
from tests._close import assert_close_per_matrix
from workload import config_instances, random_orthonormal

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5}


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _inputs(name):
    inst = config_instances(name, count=1)[0]
    level = inst.noise_levels[0]
    grid = O.samples(inst.t, inst.c, inst.n, abs_noise=inst.noise(level) if level > 0 else None)
    rng = np.random.Generator(np.random.PCG64(31 + inst.N))
    U, V = random_orthonormal(rng, inst.N, inst.m), random_orthonormal(rng, inst.N, inst.m)
    s = rng.uniform(0.5, 2.0, inst.m)
    return inst, grid, U, s, V


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
def test_noalloc_matches_build_S_on_two_calls_the_second_smaller(prec):
    for name, with_s0 in (("c1", True), ("c0", False)):   # c1: N = 4096; then c0: N = 256
        inst, grid, U, s, V = _inputs(name)
        print(f"noalloc {prec} {name}", flush=True)
        args = (_dev(grid), inst.d, inst.n, _dev(U), _dev(s), _dev(V))
        ells = inst.d + (1 if with_s0 else 0)
        out = torch.full((ells, inst.m, inst.m), complex("nan"), dtype=torch.complex128, device=DEV)
        got = api.build_S_noalloc(*args, out=out, prec=prec, with_s0=with_s0)
        ref_gpu = api.build_S(*args, prec=prec, with_s0=with_s0)
        torch.cuda.synchronize()
        # the same plan and kernels: the same bits
        assert torch.equal(got, ref_gpu), f"{name} {prec}: differs from prony_build_S"
        ref = O.pencil_matrices(grid, inst.d, inst.n, U, s, V, with_s0=with_s0)
        assert_close_per_matrix(got.cpu().numpy(), ref, TOL[prec], f"noalloc {name} {prec}")


def test_noalloc_rejects_plans_beyond_its_scratch():
    # d=2, n=200 (N = 40401), m=32 in FP64 with S_0 needs far more than 64 MiB of
    # scratch (its partial sums alone): refused on the host before anything is launched
    d, n, m = 2, 200, 32
    N = (n + 1) ** d
    f = torch.zeros((2 * n + 2) ** d, dtype=torch.complex128, device=DEV)
    U = torch.zeros((N, m), dtype=torch.complex128, device=DEV)
    s = torch.ones(m, dtype=torch.float64, device=DEV)
    out = torch.zeros((d + 1, m, m), dtype=torch.complex128, device=DEV)
    with pytest.raises(_lib.PronyError) as err:
        api.build_S_noalloc(f, d, n, U, s, U, out=out, prec="fp64", with_s0=True)
    assert err.value.status == _lib.PRONY_ENOTSUP
    assert "scratch" in str(err.value)
