"""Autotuner: candidate tile shapes and split targets are timed (distinct plans
only), the winner is registered and cached, the cache reloads through the Python
and the library's own loader, bucket entries tune batches, and every tuned plan
stays correct against the oracle."""
import json

import numpy as np
import pytest
import torch

from oracle import prony_oracle as O
from paper_2012_11430_amd import api, autotune
from tests._close import assert_close_per_matrix

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_tune_single_registers_caches_and_stays_correct(tmp_path, prec):
    path = str(tmp_path / "tune.json")
    d, n, m = 2, 31, 12
    times = autotune.tune_single(DEV, d, n, m, prec, reps=3, path=path, bucket=True)
    assert 2 <= len(times) <= len(autotune.SINGLE_CANDIDATES) * len(autotune.SINGLE_FRAGMENTS)
    assert all(t > 0 for t in times.values())
    data = json.load(open(path))
    assert data["version"] == 2
    entries = next(iter(data["devices"].values()))
    best = entries[f"{d},{n},{m},{prec},single"]
    assert (best["fragments"], best["target"]) in times
    assert entries[f"bucket:{d},{n},{m},{prec},single"] == best
    # the library's own loader (prony_autotune) reads the same cache
    autotune.register(DEV, d, n, m, prec, False, 0, 0)
    autotune.register(DEV, d, n, m, prec, False, 0, 0, bucket=True)
    assert autotune.registered_tile(DEV, d, n, m, prec, False) == (0, 0)
    autotune.load_cache_native(DEV, path)
    assert autotune.registered_tile(DEV, d, n, m, prec, False) == (best["fragments"], best["target"])
    assert autotune.registered_tile(DEV, d, n, m, prec, False, bucket=True) == (best["fragments"], best["target"])
    assert autotune.load_cache(DEV, path) == 2
    assert autotune.plan(DEV, d, n, m, prec)["fragments"] == best["fragments"]
    autotune.register(DEV, d, n, m, prec, False, 0, 0, bucket=True)
    rng = np.random.Generator(np.random.PCG64(5))
    N = (n + 1) ** d
    grid = rng.standard_normal((2 * n + 2) ** d) + 1j * rng.standard_normal((2 * n + 2) ** d)
    U = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
    V = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
    s = rng.uniform(0.5, 2, m)
    ref = O.pencil_matrices(grid, d, n, U, s, V)
    for frag in autotune.SINGLE_FRAGMENTS:
        for target in (256, 2048):      # plans at both ends of the candidate range
            autotune.register(DEV, d, n, m, prec, False, target, frag)
            got = api.build_S(_dev(grid), d, n, _dev(U), _dev(s), _dev(V), prec=prec).cpu().numpy()
            assert_close_per_matrix(got, ref, 1e-5, f"{prec} fragments {frag} target {target}")
    autotune.register(DEV, d, n, m, prec, False, 0, 0)


def test_tune_batch(tmp_path):
    path = str(tmp_path / "tune.json")
    rng = np.random.Generator(np.random.PCG64(6))
    inst = []
    refs = []
    for d, n, m in [(1, 300, 7), (2, 20, 9), (3, 7, 5), (2, 20, 9)]:
        N = (n + 1) ** d
        grid = rng.standard_normal((2 * n + 2) ** d) + 1j * rng.standard_normal((2 * n + 2) ** d)
        U = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
        V = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
        s = rng.uniform(0.5, 2, m)
        inst.append((d, n, _dev(grid), _dev(U), _dev(s), _dev(V)))
        refs.append(O.pencil_matrices(grid, d, n, U, s, V))
    res = autotune.tune_batch(inst, "fp32", reps=2, path=path)
    assert res["tuned_ms"] <= res["default_ms"] and res["timed_batches"] >= 1
    assert set(res["buckets"]) == {",".join(map(str, autotune.bucket_of(d, n, U.shape[1])))
                                   for d, n, f, U, s, V in inst}
    entries = next(iter(json.load(open(path))["devices"].values()))
    assert all(k.startswith("bucket:") and k.endswith(",fp32,batch") for k in entries)
    # every (chunks, fragments) pair registered for the buckets stays correct
    for chunks in autotune.BATCH_CANDIDATES:
        for frag in autotune.BATCH_FRAGMENTS:
            for d, n, f, U, s, V in inst:
                autotune.register(DEV, d, n, U.shape[1], "fp32", True, chunks, frag, bucket=True)
            b = api.Batch(inst, prec="fp32")
            b.run()
            torch.cuda.synchronize()
            for S, ref in zip(b.S, refs):
                assert_close_per_matrix(S.cpu().numpy(), ref, 1e-5, f"batch chunks {chunks} fragments {frag}")
            b.close()
    for d, n, f, U, s, V in inst:
        autotune.register(DEV, d, n, U.shape[1], "fp32", True, 0, 0, bucket=True)


def test_native_cache_loader_rejects_malformed_entries(tmp_path):
    key = autotune._device_key(DEV)
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps({"devices": {key: {"2,15,5,fp99,single": 3}}, "version": 1}))
    with pytest.raises(api._lib.PronyError):
        autotune.load_cache_native(DEV, str(bad))
    other = tmp_path / "other.json"     # entries of another device only: nothing registered
    other.write_text(json.dumps({"devices": {"gfx000:1": {"2,15,5,fp32,single": 3}}, "version": 1}))
    autotune.load_cache_native(DEV, str(other))
    assert autotune.registered(DEV, 2, 15, 5, "fp32", False) == 0
