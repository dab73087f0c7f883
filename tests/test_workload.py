"""The seeded input generator (CPU): the laws, ranges and separations of the
workloads, determinism of the seeds, and the paper's deterministic inputs
(Sec. 5). The generator draws inputs only; nothing here evaluates the method."""
import itertools
import math

import numpy as np
import pytest

from workload import generate as W
from workload import config_instances, paper_efficiency_inputs, paper_relative_noise


def _min_separation(t):
    if len(t) < 2:
        return math.inf
    return min(float(W.torus_distance(a, b)) for a, b in itertools.combinations(t, 2))


@pytest.mark.parametrize("name,d,n,m,sep", [("c0", 2, 15, 5, 0.05), ("c1", 2, 63, 20, 0.05),
                                            ("c2", 3, 19, 30, 0.08)])
def test_single_instance_configs(name, d, n, m, sep):
    (inst,) = config_instances(name)
    assert (inst.d, inst.n, inst.m, inst.N) == (d, n, m, (n + 1) ** d)
    assert inst.t.shape == (m, d) and np.all((inst.t >= 0) & (inst.t < 1))
    assert _min_separation(inst.t) >= sep
    assert inst.c.shape == (m,) and inst.noise_unit.shape == ((2 * n + 2) ** d,)
    assert abs(np.linalg.norm(inst.mu) - 1.0) < 1e-15
    r = np.abs(inst.c)
    if name == "c2":
        assert np.all((r >= 1e-2) & (r <= 1.0))
        assert inst.noise_levels == (0.0, 1e-8, 1e-6, 1e-4, 1e-3)
    else:
        assert np.all((r >= 0.5) & (r <= 1.5))


def test_draws_are_deterministic_and_distinct_across_configs():
    a = config_instances("c1")[0]
    b = config_instances("c1")[0]
    assert np.array_equal(a.t, b.t) and np.array_equal(a.c, b.c)
    assert np.array_equal(a.noise_unit, b.noise_unit) and np.array_equal(a.mu, b.mu)
    c = config_instances("c0")[0]
    assert not np.array_equal(a.t[: c.m], c.t)


def test_noise_scaling_and_circular_law():
    inst = config_instances("c1")[0]
    z = inst.noise_unit
    # CN(0,1): E|z|^2 = 1, real and imaginary parts of equal variance, mean ~ 0
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.03
    assert abs(np.var(z.real) - np.var(z.imag)) < 0.03
    assert abs(np.mean(z)) < 0.02
    scale = 1e-6 * float(np.max(np.abs(inst.c)))
    assert np.array_equal(inst.noise(), scale * z)
    assert np.array_equal(inst.noise(0.0), 0.0 * z)


def test_c3_shapes_ranges_and_separation():
    insts = config_instances("c3")
    assert len(insts) == 512
    ds = [x.d for x in insts]
    assert set(ds) == {1, 2, 3}
    for x in insts:
        assert 64 <= x.N <= 4096 and 2 <= x.m <= 32 and x.m <= x.N
        assert x.noise_levels == (1e-7,)
        assert _min_separation(x.t) >= (min(0.05, 0.5 / x.m) if x.d == 1 else 0.05) - 1e-12
    # the first instances do not depend on how many are drawn
    head = config_instances("c3", count=8)
    assert all(np.array_equal(a.t, b.t) and a.n == b.n for a, b in zip(head, insts[:8]))
    # N* log-uniform: both halves of the log range are populated
    logN = np.log([x.N for x in insts])
    mid = 0.5 * (math.log(64) + math.log(4096))
    assert 0.3 < np.mean(logN < mid) < 0.7


def test_c4_batch_members():
    insts = config_instances("c4")
    assert len(insts) == 64
    assert {(x.d, x.n, x.m) for x in insts} == {(2, 47, 16)}
    assert len({x.t.tobytes() for x in insts}) == 64    # independent draws


def test_paper_efficiency_inputs_follow_the_printed_formula():
    # Sec. 5: t_j(i) = ((i-1) m + j - 1) 10^(-ceil(log10 dm)), c_j = j + i j
    t, c = paper_efficiency_inputs(3, 20)
    assert t.shape == (20, 3)
    assert t[0, 0] == 0.0 and t[1, 0] == 0.01 and t[0, 1] == 0.2 and t[19, 2] == pytest.approx(0.59)
    assert np.array_equal(c, np.arange(1, 21) * (1 + 1j))
    t5, _ = paper_efficiency_inputs(3, 5)    # dm = 15: scale 10^-2
    assert t5[4, 2] == pytest.approx(0.14)
    t1, _ = paper_efficiency_inputs(2, 5)    # dm = 10: scale 10^-1
    assert t1[4, 1] == pytest.approx(0.9)


def test_paper_relative_noise_is_bounded_and_seeded():
    a = paper_relative_noise(3, 3, 4, 1e-6)
    assert a.shape == (10 ** 3,) and np.all(np.abs(a) <= 1e-6) and np.isrealobj(a)
    assert np.array_equal(a, paper_relative_noise(3, 3, 4, 1e-6))
    assert not np.array_equal(a, paper_relative_noise(4, 3, 4, 1e-6))
