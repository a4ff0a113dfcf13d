"""Autotuner for the transform shape (per N) and the batched CG block size.

    import paper_1509_03979_amd.tune as tune
    choice = tune.tune(ns=[2**14, 2**15, 2**16, 2**17, 2**18], dtype="f32")   # times, installs, caches
    tune.load()                                                           # later processes: install cached
    tune.load("f32", tune.SHIPPED)       # the cache shipped for MI355X (all workload sizes)

For every N it times each compiled four-step shape (cs_shape_candidates) on
one H-apply with the library's own timer (cs_time_shape, HIP events), keeps
the fastest and installs it with cs_set_shape.  For the batched call it
times a small representative batch at each CG block size and keeps the
fastest.  Results are cached per device and dtype in a JSON file
(CS_TUNE_CACHE, default ~/.cache/csrecover/tune.json).  Only timing and
bookkeeping happen here; every timed operation runs in the library.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import (CS_F32, CS_F64, Operator, cs_set_shape, cs_shape_candidates, cs_time_shape)

CG_BLOCKS = (128, 256, 512, 1024)


def cache_path() -> str:
    return os.environ.get("CS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "csrecover",
                                                        "tune.json"))


def _device_key(torch) -> str:
    """Architecture (without feature flags) and compute-unit count: the marketing
    name differs between driver versions of the same part."""
    p = torch.cuda.get_device_properties(0)
    arch = str(getattr(p, "gcnArchName", "")).split(":")[0]
    return f"{arch}|cu{p.multi_processor_count}"


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _write(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _probe_operator(n: int, m: int, torch):
    """A seeded operator of size (n, m) for timing (timings do not depend on values)."""
    r = np.random.default_rng([1509, 3979, 99, n, m])
    rows = np.sort(r.choice(n, m, replace=False)).astype(np.int32)
    signs = (r.integers(0, 2, n) * 2 - 1).astype(np.int8)
    return Operator.from_numpy(n, rows, signs)


def tune_shapes(ns, dtype: str = "f32", reps: int = 20, install: bool = True) -> dict:
    """{n: {"shape": (l1, l2, b, e), "ms": t, "all": {shape: ms}}} for each N."""
    import torch
    code = CS_F32 if dtype == "f32" else CS_F64
    out = {}
    for n in ns:
        op = _probe_operator(n, max(1, n // 4), torch)
        timings = {}
        for sh in cs_shape_candidates(code, n):
            cs_time_shape(code, op, sh, 3)                       # first use loads the code object
            timings[sh] = min(cs_time_shape(code, op, sh, reps) for _ in range(3))
        best = min(timings, key=timings.get)
        out[n] = {"shape": best, "ms": timings[best], "default": cs_shape_candidates(code, n)[0],
                  "all": {",".join(map(str, k)): v for k, v in timings.items()}}
        if install:
            cs_set_shape(code, n, best)
    return out


def tune_cg_block(batch_fn, blocks=CG_BLOCKS, reps: int = 2) -> dict:
    """batch_fn(cg_block) runs one batched call; returns {"cg_block": best, "all": {b: s}}."""
    import torch
    times = {}
    for b in blocks:
        batch_fn(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batch_fn(b)
        torch.cuda.synchronize()
        times[b] = (time.perf_counter() - t0) / reps
    best = min(times, key=times.get)
    return {"cg_block": best, "all": times}


def tune(ns, dtype: str = "f32", reps: int = 20, path: str | None = None) -> dict:
    """Times and installs the best shape for each N, and caches the result."""
    import torch
    path = path or cache_path()
    res = tune_shapes(ns, dtype, reps)
    data = _read(path)
    key = f"{_device_key(torch)}|{dtype}"
    ent = data.setdefault(key, {"shapes": {}})
    for n, r in res.items():
        ent["shapes"][str(n)] = {"shape": list(r["shape"]), "ms": r["ms"]}
    _write(path, data)
    return res


def save_cg_block(cg_block: int, dtype: str = "f32", path: str | None = None) -> None:
    import torch
    path = path or cache_path()
    data = _read(path)
    data.setdefault(f"{_device_key(torch)}|{dtype}", {"shapes": {}})["cg_block"] = int(cg_block)
    _write(path, data)


# The sizes the shipped workloads run at, per dtype.
WORKLOAD_SIZES = {"f32": [2 ** 14, 2 ** 15, 2 ** 16, 2 ** 17, 2 ** 18, 2 ** 20, 2 ** 24], "f64": [2 ** 12]}
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_mi355x.json")


def tune_workloads(path: str = SHIPPED, reps: int = 20, cg_block_fn=None) -> dict:
    """Tunes every workload size (and, given cg_block_fn(b) that runs one batched
    call, the batched CG block size) and writes the cache to `path`."""
    import torch
    data = _read(path)
    for dtype, ns in WORKLOAD_SIZES.items():
        res = tune_shapes(ns, dtype, reps)
        ent = data.setdefault(f"{_device_key(torch)}|{dtype}", {"shapes": {}})
        for n, r in res.items():
            ent["shapes"][str(n)] = {"shape": list(r["shape"]), "ms": r["ms"], "default": list(r["default"]),
                                     "all": r["all"]}
    if cg_block_fn is not None:
        data[f"{_device_key(torch)}|f32"]["cg_block"] = int(tune_cg_block(cg_block_fn)["cg_block"])
    _write(path, data)
    return data


def load(dtype: str = "f32", path: str | None = None) -> dict:
    """Installs the cached shapes of this device and dtype; returns the cached entry."""
    import torch
    ent = _read(path or cache_path()).get(f"{_device_key(torch)}|{dtype}", {})
    code = CS_F32 if dtype == "f32" else CS_F64
    for n, r in ent.get("shapes", {}).items():
        cs_set_shape(code, int(n), tuple(r["shape"]))
    return ent
