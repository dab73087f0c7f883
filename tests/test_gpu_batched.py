"""Batched S-build (many uneven instances in one planned launch sequence) and its
HIP-graph replay, against the CPU oracle.

Inputs per instance: the c3 workload (d ~ U{1,2,3}, N in [64, 4096], m in [2, 32],
noise 1e-7); U, Sigma, V are the exact reduced SVD of the noise-free T obtained
from the QR factorisation of its Vandermonde factor (T = V_z diag(c) V_z^*).
Tolerances as in test_gpu_parity: 1e-12 (FP64), 1e-5 (FP32), normwise and entry by
entry. The full batch is also compared under every per-instance chunk count the
autotuner can register (the configurations the benchmark may time).
"""
import functools
import sys

import numpy as np
import pytest
import torch

from oracle import prony_oracle as O
from paper_2012_11430_amd import api
from tests._close import assert_close, assert_close_per_matrix
from workload import config_instances

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def closed_form_factors(t, c, d, n):
    """Reduced SVD of the noise-free T = V_z diag(c) V_z^* via V_z = Q R."""
    import itertools
    ks = np.array(list(itertools.product(range(n + 1), repeat=d)), dtype=float)
    Vz = np.exp(-2j * np.pi * (ks @ t.T))
    Q, R = np.linalg.qr(Vz)
    Ub, s, Vbh = np.linalg.svd(R @ np.diag(c) @ R.conj().T)
    return Q @ Ub, s, Q @ Vbh.conj().T


@functools.lru_cache(maxsize=None)
def _c3_inputs(count):
    out = []
    for inst in config_instances("c3", count=count):
        grid = O.samples(inst.t, inst.c, inst.n, abs_noise=inst.noise())
        U, s, V = closed_form_factors(inst.t, inst.c, inst.d, inst.n)
        out.append((inst, grid, U, s, V))
    return out


def _device_instances(inputs):
    return [(inst.d, inst.n, _dev(grid), _dev(U), _dev(s), _dev(V)) for inst, grid, U, s, V in inputs]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_matches_oracle_on_sampled_c3_instances(prec):
    inputs = _c3_inputs(512)
    picked = [inputs[i] for i in range(0, 512, 16)]           # 32 instances across the batch
    _say(f"batched {prec}: {len(picked)} instances, d {sorted(set(x[0].d for x in picked))}")
    batch = api.Batch(_device_instances(picked), prec=prec)
    batch.run()
    torch.cuda.synchronize()
    worst = 0.0
    for (inst, grid, U, s, V), S in zip(picked, batch.S):
        ref = O.pencil_matrices(grid, inst.d, inst.n, U, s, V)
        got = S.cpu().numpy()
        norm, entry = assert_close_per_matrix(got, ref, TOL[prec], f"d={inst.d} n={inst.n} m={inst.m}")
        worst = max(worst, norm, entry)
    batch.close()
    _say(f"  worst rel err {worst:.3e}")


def test_full_c3_batch_matches_single_instance_calls():
    inputs = _c3_inputs(512)
    dev_inst = _device_instances(inputs)
    _say("full c3 batch: 512 instances")
    singles = [api.build_S(f, d, n, U, s, V, prec="fp64") for d, n, f, U, s, V in dev_inst]
    for prec in ("fp64", "fp32"):
        batch = api.Batch(dev_inst, prec=prec)
        batch.run()
        torch.cuda.synchronize()
        worst = 0.0
        for i, (a, b) in enumerate(zip(singles, batch.S)):
            worst = max(worst, *assert_close_per_matrix(b.cpu().numpy(), a.cpu().numpy(), TOL[prec],
                                                        f"{prec} instance {i}"))
        _say(f"  {prec}: max rel diff to single FP64 calls {worst:.3e}")
        batch.close()


@pytest.mark.parametrize("chunks", [1, 2, 4])
@pytest.mark.parametrize("fragments", [1, 2])
def test_full_c3_batch_at_every_tuned_tile(chunks, fragments):
    # the FP32 batch the benchmark replays (default class schedule), with each (chunks per
    # instance, fragments per wave) pair the autotuner chooses from registered for
    # every shape bucket, against single FP64 calls (pinned to the oracle above)
    from paper_2012_11430_amd import autotune
    assert chunks in autotune.BATCH_CANDIDATES and fragments in autotune.BATCH_FRAGMENTS
    inputs = _c3_inputs(512)
    dev_inst = _device_instances(inputs)
    shapes = sorted({(inst.d, inst.n, inst.m) for inst, *_r in inputs})
    _say(f"full c3 batch, {chunks} chunk(s) per instance, {fragments} fragment(s) per wave")
    singles = [api.build_S(f, d, n, U, s, V, prec="fp64") for d, n, f, U, s, V in dev_inst]
    try:
        for d, n, m in shapes:
            autotune.register(DEV, d, n, m, "fp32", True, chunks, fragments, bucket=True)
        batch = api.Batch(dev_inst, prec="fp32")
        batch.run()
        torch.cuda.synchronize()
        worst = 0.0
        for i, (a, b) in enumerate(zip(singles, batch.S)):
            worst = max(worst, *assert_close_per_matrix(b.cpu().numpy(), a.cpu().numpy(), TOL["fp32"],
                                                        f"chunks {chunks} fragments {fragments} instance {i}"))
        batch.close()
        _say(f"  worst {worst:.3e}")
    finally:
        for d, n, m in shapes:
            autotune.register(DEV, d, n, m, "fp32", True, 0, 0, bucket=True)


def test_queue_schedule_is_bitwise_equal_to_class_launches():
    # the same tiles and fixed-order sums under both schedules (FP32, full c3 batch)
    dev_inst = _device_instances(_c3_inputs(512))
    batch = api.Batch(dev_inst, prec="fp32")
    _say("queue vs class schedules: 512 instances")
    batch.set_schedule("queue")
    batch.run()
    torch.cuda.synchronize()
    queued = [S.clone() for S in batch.S]
    for S in batch.S:
        S.zero_()
    batch.set_schedule("classes")
    batch.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(queued, batch.S))
    batch.set_schedule("queue")        # and back: a second queue run resets its counter
    for S in batch.S:
        S.zero_()
    batch.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(queued, batch.S))
    batch.close()


def test_queue_schedule_rejected_for_fp64():
    batch = api.Batch(_device_instances(_c3_inputs(512)[:4]), prec="fp64")
    with pytest.raises(api._lib.PronyError):
        batch.set_schedule("queue")
    with pytest.raises(ValueError):
        batch.set_schedule("fifo")
    batch.close()


@pytest.mark.parametrize("schedule", ["queue", "classes"])
def test_graph_replays_match_eager_run(schedule):
    inputs = _c3_inputs(512)[:96]
    dev_inst = _device_instances(inputs)
    batch = api.Batch(dev_inst, prec="fp32")
    batch.set_schedule(schedule)
    batch.run()
    torch.cuda.synchronize()
    eager = [S.clone() for S in batch.S]
    batch.capture()
    for rep in range(3):
        for S in batch.S:
            S.zero_()
        torch.cuda.synchronize()
        batch.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, batch.S):
            assert torch.equal(a, b), f"replay {rep} differs from the eager run"
        # unrelated eager work between replays
        (torch.randn(1024, device=DEV) * 2).sum().item()
    batch.close()


def test_graph_replay_sees_new_sample_values():
    inputs = _c3_inputs(512)[:24]
    dev_inst = _device_instances(inputs)
    batch = api.Batch(dev_inst, prec="fp64")
    batch.capture()
    batch.replay()
    torch.cuda.synchronize()
    for (inst, grid, U, s, V), (d, n, f, *_r) in zip(inputs, dev_inst):
        f.mul_(2.0)      # S is linear in f
    batch.replay()
    torch.cuda.synchronize()
    for (inst, grid, U, s, V), S in zip(inputs, batch.S):
        ref = O.pencil_matrices(2.0 * grid, inst.d, inst.n, U, s, V)
        assert_close_per_matrix(S.cpu().numpy(), ref, 1e-12, "replay after f *= 2")
    batch.close()
