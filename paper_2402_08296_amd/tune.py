"""Cache of the library's autotuner.

``ddmgnn_autotune`` times capped solves of a problem under candidate launch
schedules (DSS workgroup size per sub-mesh, vector-kernel workgroup count) and
keeps the fastest. ``tuned`` stores that choice in a JSON file keyed by the GPU
architecture and a config class of the problem (sizes, precision, Krylov method,
local solver), and applies a cached choice to later problems of the same class
without tuning again.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

DEFAULT_PATH = os.environ.get("DDMGNN_TUNE_CACHE",
                              os.path.join(os.path.expanduser("~"), ".cache", "ddmgnn_tune.json"))


def config_class(n: int, sub_ptr, opts) -> str:
    """Problems of one class share a schedule: log2 of N and K, the mean sub-mesh size
    in steps of 128 nodes, and the options that select kernels."""
    k = np.diff(np.asarray(sub_ptr, dtype=np.int64))
    return (f"n2^{round(math.log2(max(n, 1)))}-K2^{round(math.log2(max(k.size, 1)))}-"
            f"k{int(k.mean()) // 128 * 128}-prec{opts.precision}-krylov{opts.krylov}-local{opts.local_solver}")


def load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(path: str, cache: dict) -> bool:
    """Writes the cache atomically; False when the location is not writable."""
    try:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
        return True
    except OSError:
        return False


def tuned(prob, hp, opts, arch: str, path: str | None = None, iterations: int = 16) -> dict:
    """Applies the cached schedule of the problem's class, or autotunes and caches it.

    ``prob`` is a ``Problem`` (``set_tuning`` / ``autotune``), ``hp`` its host problem.
    Returns {"key", "tuning", "ms_per_iteration", "cached"}."""
    path = path or DEFAULT_PATH
    key = f"{arch}|{config_class(hp.n, hp.sub_ptr, opts)}"
    cache = load(path)
    hit = cache.get(key)
    if hit is not None:
        prob.set_tuning(**hit["tuning"])
        return {"key": key, "tuning": dict(hit["tuning"]), "ms_per_iteration": hit["ms_per_iteration"],
                "cached": True}
    t, ms = prob.autotune(opts, iterations)
    entry = {"tuning": t.as_dict(), "ms_per_iteration": ms}
    cache[key] = entry
    save(path, cache)
    return {"key": key, "tuning": dict(entry["tuning"]), "ms_per_iteration": ms, "cached": False}
