"""Autotuner of the S-build's work split, with a JSON cache.

The S-build splits the extended index range of an instance into chunks; the
number of workgroups it aims at trades parallelism against the cost of the
per-workgroup U^* reduction and the partial sums. For single-instance calls the
tuner times candidate targets (multiples of the compute-unit count) on synthetic
inputs of the requested shape; for batches it times uniform per-instance targets
on the batch itself. Winners are registered in the library handle
(prony_tune_set) and stored in a JSON cache keyed by device, shape, precision and
mode, so later processes reuse them (`load_cache`).

Cache file: $PRONY_TUNE_CACHE, else ~/.cache/prony_mi355x_tune.json.
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

from . import _lib, api

CACHE_ENV = "PRONY_TUNE_CACHE"
SINGLE_CANDIDATES = (1, 2, 3, 4, 8)       # x compute units
BATCH_CANDIDATES = (1, 2, 4)              # chunks of the h' range per instance


def cache_path() -> str:
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "prony_mi355x_tune.json"))


def _device_key(device: torch.device) -> str:
    p = torch.cuda.get_device_properties(device)
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}"


def _key(d, n, m, prec, batched):
    return f"{d},{n},{m},{prec},{'batch' if batched else 'single'}"


def _read(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
        if data.get("version") == 1:
            return data
    except (OSError, ValueError):
        pass
    return {"version": 1, "devices": {}}


def _write(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


_PRECS = {"fp64": _lib.PRONY_FP64, "fp32": _lib.PRONY_FP32, "bf16x3": _lib.PRONY_BF16X3}


def register(device: torch.device, d: int, n: int, m: int, prec: str, batched: bool, target: int) -> None:
    api._call("prony_tune_set", device, d, n, m, _PRECS[prec], _lib.PRONY_TUNE_BATCHED if batched else 0,
              int(target))


def registered(device: torch.device, d: int, n: int, m: int, prec: str, batched: bool) -> int:
    """The registered target of a shape (0 when none) — prony_tune_get."""
    out = ctypes.c_int(0)
    api._call("prony_tune_get", device, d, n, m, _PRECS[prec], _lib.PRONY_TUNE_BATCHED if batched else 0,
              ctypes.byref(out))
    return out.value


def load_cache_native(device: torch.device, path: str | None = None) -> None:
    """Register the cached entries of this device through the library's own
    loader (prony_autotune), as a C caller would."""
    api._call("prony_autotune", device, (path or cache_path()).encode())


def load_cache(device: torch.device, path: str | None = None) -> int:
    """Register every cached entry of this device; returns the number registered."""
    data = _read(path or cache_path())
    entries = data["devices"].get(_device_key(device), {})
    for key, target in entries.items():
        d, n, m, prec, mode = key.split(",")
        register(device, int(d), int(n), int(m), prec, mode == "batch", int(target))
    return len(entries)


def _store(device, path, updates):
    path = path or cache_path()
    data = _read(path)
    data["devices"].setdefault(_device_key(device), {}).update(updates)
    _write(path, data)


def _time(fn, reps):
    for _ in range(2):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_single(device: torch.device, d: int, n: int, m: int, prec: str, reps: int = 10,
                path: str | None = None, seed: int = 0) -> dict:
    """Time prony_build_S of shape (d, n, m) for each candidate split target on
    synthetic inputs; register and cache the fastest. Returns {target: ms}."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    N = (n + 1) ** d
    G = (2 * n + 2) ** d
    f = torch.randn(G, dtype=torch.complex128, generator=gen).to(device)
    U = torch.randn(N, m, dtype=torch.complex128, generator=gen).to(device)
    V = torch.randn(N, m, dtype=torch.complex128, generator=gen).to(device)
    s = (torch.rand(m, dtype=torch.float64, generator=gen) + 0.5).to(device)
    cus = torch.cuda.get_device_properties(device).multi_processor_count
    times = {}
    for c in SINGLE_CANDIDATES:
        register(device, d, n, m, prec, False, c * cus)
        times[c * cus] = _time(lambda: api.build_S(f, d, n, U, s, V, prec=prec), reps)
    best = min(times, key=times.get)
    register(device, d, n, m, prec, False, best)
    _store(device, path, {_key(d, n, m, prec, False): best})
    return times


def tune_batch(batch_instances, prec: str, reps: int = 5, path: str | None = None) -> dict:
    """Time a batch (sequence of (d, n, f, U, sigma, V)) under uniform per-instance
    targets; register and cache the fastest for every shape in it."""
    device = batch_instances[0][2].device
    shapes = sorted({(d, n, U.shape[1]) for d, n, f, U, s, V in batch_instances})
    times = {}
    for c in BATCH_CANDIDATES:
        for d, n, m in shapes:
            register(device, d, n, m, prec, True, c)
        b = api.Batch(batch_instances, prec=prec)
        times[c] = _time(b.run, reps)
        b.close()
    best = min(times, key=times.get)
    for d, n, m in shapes:
        register(device, d, n, m, prec, True, best)
    _store(device, path, {_key(d, n, m, prec, True): best for d, n, m in shapes})
    return times
