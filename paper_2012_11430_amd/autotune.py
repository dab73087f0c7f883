"""Autotuner of the S-build's tile shape and work split, with a JSON cache.

The S-build tiles the row-extended product into workgroups of 64 x fragments rows
(16-row fragments per wave) and splits the index range I_n into chunks; the number
of workgroups it aims at trades parallelism against the per-workgroup reduction
with the shifted U and the partial sums, and the fragments per wave trade operand
reuse against registers and row tiles. For single-instance calls the tuner times
every distinct plan among the candidate (fragments, target) pairs (the library's
plan query, prony_build_S_plan, removes duplicates) on synthetic inputs of the
requested shape, then times the three fastest again in three interleaved rounds
and keeps the lowest median. For batches it tunes per shape bucket (same d, floor(log2 N) and
column-block count ceil(m/8)) the chunks per instance and the fragments per wave,
by coordinate descent on the batch itself. Winners are registered in the library
handle (prony_tune_set_tile) and stored in a JSON cache keyed by device, shape (or
bucket), precision and mode, so later processes reuse them (`load_cache`, or the
library's own loader `prony_autotune`).

Cache file: $PRONY_TUNE_CACHE, else ~/.cache/prony_mi355x_tune.json. Format
(version 2): {"version": 2, "devices": {"<arch>:<CUs>": {"d,n,m,prec,mode" or
"bucket:d,n,m,prec,mode": {"target": T, "fragments": F}}}}; version 1 files hold
integer targets and are still read.
"""
from __future__ import annotations

import ctypes
import itertools
import json
import os
import statistics

import torch

from . import _lib, api

CACHE_ENV = "PRONY_TUNE_CACHE"
SINGLE_CANDIDATES = (1, 2, 3, 4, 8)       # split targets, x compute units
SINGLE_FRAGMENTS = (1, 2, 4)              # 16-row fragments per wave
BATCH_CANDIDATES = (1, 2, 4)              # chunks of the h range per instance
BATCH_FRAGMENTS = (1, 2)                  # the batch kernels instantiate these


def cache_path() -> str:
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "prony_mi355x_tune.json"))


def _device_key(device: torch.device) -> str:
    p = torch.cuda.get_device_properties(device)
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}"


def _key(d, n, m, prec, batched, bucket=False):
    return f"{'bucket:' if bucket else ''}{d},{n},{m},{prec},{'batch' if batched else 'single'}"


def bucket_of(d: int, n: int, m: int):
    """The bucket of a shape: (d, floor(log2 N), ceil(m / 8)), as the library keys it."""
    N = (n + 1) ** d
    return d, N.bit_length() - 1, (m + 7) // 8


def _read(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
        if data.get("version") in (1, 2) and isinstance(data.get("devices"), dict):
            data["version"] = 2
            return data
    except (OSError, ValueError):
        pass
    return {"version": 2, "devices": {}}


def _write(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


_PRECS = {"fp64": _lib.PRONY_FP64, "fp32": _lib.PRONY_FP32, "bf16x3": _lib.PRONY_BF16X3}


def _flags(batched, bucket):
    return (_lib.PRONY_TUNE_BATCHED if batched else 0) | (_lib.PRONY_TUNE_BUCKET if bucket else 0)


def register(device: torch.device, d: int, n: int, m: int, prec: str, batched: bool, target: int,
             fragments: int | None = None, bucket: bool = False) -> None:
    """Register a split target (and, if given, fragments per wave) for a shape or its
    bucket (prony_tune_set / prony_tune_set_tile); 0 restores the default."""
    if fragments is None:
        api._call("prony_tune_set", device, d, n, m, _PRECS[prec], _flags(batched, bucket), int(target))
    else:
        api._call("prony_tune_set_tile", device, d, n, m, _PRECS[prec], _flags(batched, bucket), int(fragments),
                  int(target))


def registered(device: torch.device, d: int, n: int, m: int, prec: str, batched: bool) -> int:
    """The registered target of a shape (0 when none) — prony_tune_get."""
    out = ctypes.c_int(0)
    api._call("prony_tune_get", device, d, n, m, _PRECS[prec], _flags(batched, False), ctypes.byref(out))
    return out.value


def registered_tile(device: torch.device, d: int, n: int, m: int, prec: str, batched: bool, bucket: bool = False):
    """(fragments, target) of a shape's entry or of its bucket's (zeros when none)."""
    frag, tgt = ctypes.c_int(0), ctypes.c_int(0)
    api._call("prony_tune_get_tile", device, d, n, m, _PRECS[prec], _flags(batched, bucket), ctypes.byref(frag),
              ctypes.byref(tgt))
    return frag.value, tgt.value


def plan(device: torch.device, d: int, n: int, m: int, prec: str, with_s0: bool = False) -> dict:
    """The plan prony_build_S would use now (prony_build_S_plan): fragments per wave,
    workgroups, h per chunk and workspace bytes."""
    frag, wgs, chunk = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ws = ctypes.c_size_t()
    api._call("prony_build_S_plan", device, d, n, m, _PRECS[prec], _lib.PRONY_WITH_S0 if with_s0 else 0,
              ctypes.byref(frag), ctypes.byref(wgs), ctypes.byref(chunk), ctypes.byref(ws))
    return {"fragments": frag.value, "workgroups": wgs.value, "chunk": chunk.value, "workspace": ws.value}


def load_cache_native(device: torch.device, path: str | None = None) -> None:
    """Register the cached entries of this device through the library's own
    loader (prony_autotune), as a C caller would."""
    api._call("prony_autotune", device, (path or cache_path()).encode())


def load_cache(device: torch.device, path: str | None = None) -> int:
    """Register every cached entry of this device; returns the number registered."""
    data = _read(path or cache_path())
    entries = data["devices"].get(_device_key(device), {})
    for key, value in entries.items():
        bucket = key.startswith("bucket:")
        d, n, m, prec, mode = (key[len("bucket:"):] if bucket else key).split(",")
        if isinstance(value, dict):
            target, fragments = int(value.get("target", 0)), int(value.get("fragments", 0))
        else:
            target, fragments = int(value), 0
        register(device, int(d), int(n), int(m), prec, mode == "batch", target, fragments, bucket)
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
                path: str | None = None, seed: int = 0, fragments=SINGLE_FRAGMENTS,
                targets=SINGLE_CANDIDATES, bucket: bool = False) -> dict:
    """Time prony_build_S of shape (d, n, m) for every distinct plan among the
    candidate (fragments, target x CUs) pairs on synthetic inputs; register and
    cache the fastest (also for the shape's bucket when bucket=True).
    Returns {(fragments, target): ms} of the plans timed."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    N = (n + 1) ** d
    G = (2 * n + 2) ** d
    f = torch.randn(G, dtype=torch.complex128, generator=gen).to(device)
    U = torch.randn(N, m, dtype=torch.complex128, generator=gen).to(device)
    V = torch.randn(N, m, dtype=torch.complex128, generator=gen).to(device)
    s = (torch.rand(m, dtype=torch.float64, generator=gen) + 0.5).to(device)
    cus = torch.cuda.get_device_properties(device).multi_processor_count
    times, seen = {}, set()
    for frag, c in itertools.product(fragments, targets):
        register(device, d, n, m, prec, False, c * cus, frag)
        p = plan(device, d, n, m, prec)
        sig = (p["fragments"], p["workgroups"], p["chunk"])
        if sig in seen:
            continue
        seen.add(sig)
        times[(p["fragments"], c * cus)] = _time(lambda: api.build_S(f, d, n, U, s, V, prec=prec), reps)
    # close candidates swap places from run to run: the three fastest plans are
    # timed again in three interleaved rounds and the lowest median wins
    finalists = sorted(times, key=times.get)[:3]
    rounds = {k: [] for k in finalists}
    if len(finalists) > 1:
        for _ in range(3):
            for frag, target in finalists:
                register(device, d, n, m, prec, False, target, frag)
                rounds[(frag, target)].append(_time(lambda: api.build_S(f, d, n, U, s, V, prec=prec), reps))
    best_frag, best_target = min(finalists, key=lambda k: statistics.median(rounds[k]) if rounds[k] else times[k])
    register(device, d, n, m, prec, False, best_target, best_frag)
    entry = {"target": best_target, "fragments": best_frag}
    updates = {_key(d, n, m, prec, False): entry}
    if bucket:
        register(device, d, n, m, prec, False, best_target, best_frag, bucket=True)
        updates[_key(d, n, m, prec, False, bucket=True)] = entry
    _store(device, path, updates)
    return times


def tune_batch(batch_instances, prec: str, reps: int = 5, path: str | None = None, rounds: int = 1) -> dict:
    """Tune a batch (sequence of (d, n, f, U, sigma, V)) per shape bucket: starting
    from the defaults, every bucket in turn (largest work first) tries each
    (chunks per instance, fragments per wave) pair with the other buckets fixed and
    keeps the fastest whole-batch time (coordinate descent, `rounds` passes).
    Registers and caches the bucket entries; exact-shape batch entries of the
    batch's shapes are removed so that the buckets apply.
    Returns {"default_ms", "tuned_ms", "timed_batches", "buckets": {bucket: (chunks, fragments)}}."""
    device = batch_instances[0][2].device
    shapes = sorted({(d, n, U.shape[1]) for d, n, f, U, s, V in batch_instances})
    for d, n, m in shapes:
        register(device, d, n, m, prec, True, 0, 0)
    groups = {}
    for d, n, m in shapes:
        groups.setdefault(bucket_of(d, n, m), []).append((d, n, m))
    work = {b: 0.0 for b in groups}
    for d, n, f, U, s, V in batch_instances:
        m = U.shape[1]
        work[bucket_of(d, n, m)] += ((n + 2) ** d) * ((n + 1) ** d) * m
    order = sorted(groups, key=lambda b: -work[b])
    choice = {b: (1, 0) for b in groups}

    def apply(b, chunks, frag):
        d, n, m = groups[b][0]
        register(device, d, n, m, prec, True, chunks, frag, bucket=True)

    def time_batch():
        bt = api.Batch(batch_instances, prec=prec)
        t = _time(bt.run, reps)
        bt.close()
        return t

    for b in order:
        apply(b, *choice[b])
    best = default = time_batch()
    timed = 1
    for _ in range(rounds):
        for b in order:
            for chunks, frag in itertools.product(BATCH_CANDIDATES, BATCH_FRAGMENTS):
                if (chunks, frag) == choice[b]:
                    continue
                apply(b, chunks, frag)
                t = time_batch()
                timed += 1
                if t < best:
                    best, choice[b] = t, (chunks, frag)
            apply(b, *choice[b])
    updates = {}
    for b, (chunks, frag) in choice.items():
        d, n, m = groups[b][0]
        updates[_key(d, n, m, prec, True, bucket=True)] = {"target": chunks, "fragments": frag}
    _store(device, path, updates)
    return {"default_ms": default, "tuned_ms": best, "timed_batches": timed,
            "buckets": {f"{b[0]},{b[1]},{b[2]}": list(v) for b, v in choice.items()}}

