"""Persistent cache of autotuned launch shapes (split W, register budget, pass budget, and for a
single problem with eigenvectors the overlapped or sequential write).

The library's autotuner (dpr1_autotune / dpr1_batched_autotune) times every
candidate on real data; this module remembers the winner in a JSON file keyed
by GPU architecture, operation and a size bucket, so that later solves of a
similar shape reuse it without timing again.  File: $DPR1_TUNING_CACHE, else
~/.cache/paper_1405_7537_amd/tuning.json.  Entries hold only integers
(split, waves_per_simd, main_passes, vwrite) and the measured time; a corrupt
or unreadable file is treated as empty.
"""
from __future__ import annotations

import json
import math
import os
import tempfile

import numpy as np

VERSION = 4


def cache_path() -> str:
    p = os.environ.get("DPR1_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1405_7537_amd", "tuning.json")


def _bucket(x: float) -> str:
    """Half-octave bucket of a positive size: sizes within a factor sqrt(2) share a key."""
    return f"{round(2.0 * math.log2(max(float(x), 1.0))) / 2.0:.1f}"


def key_single(arch: str, n: int, vectors: bool, root: int) -> str:
    return f"v{VERSION}|{arch}|eig|vec{int(bool(vectors))}|root{int(root)}|n{_bucket(n)}"


def key_batched(arch: str, sizes, vectors: bool, root: int) -> str:
    """A ragged batch is keyed by its problem count, largest size and sum of n^2 (the V volume)."""
    s = np.asarray(sizes, dtype=np.int64)
    return (f"v{VERSION}|{arch}|batched|vec{int(bool(vectors))}|root{int(root)}"
            f"|p{_bucket(s.size)}|max{_bucket(int(s.max()))}|n2{_bucket(float(np.sum(s.astype(np.float64) ** 2)))}")


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: str | None = None) -> bool:
    """Add one entry and rewrite the file atomically (write to a temporary file, then rename).
    Returns False, keeping nothing, when the file cannot be written (the tuned choice is still used)."""
    try:
        _store(key, entry, path or cache_path())
        return True
    except OSError:
        return False


def _store(key: str, entry: dict, path: str) -> None:
    data = load(path)
    data[key] = {"split": int(entry["split"]), "main_passes": int(entry["main_passes"]),
                 "waves_per_simd": int(entry.get("waves_per_simd", 0)), "vwrite": int(entry.get("vwrite", 0)),
                 "ms": float(entry["ms"])}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def arch_of(device) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def tuned_opts(d, z, rho, vectors=True, opts=None, reps=3, device="cuda", path=None):
    """Options for a single problem with the cached (or freshly tuned) split, register and pass budgets.
    Returns (opts, entry, from_cache)."""
    from . import dpr1 as D
    o = D.opts() if opts is None else opts
    n = int(np.asarray(d).size) if not hasattr(d, "numel") else int(d.numel())
    key = key_single(arch_of(device), n, vectors, o.root)
    hit = load(path).get(key)
    if hit is not None:
        o.split = int(hit["split"])
        o.main_passes = int(hit["main_passes"])
        o.waves_per_simd = int(hit.get("waves_per_simd", 0))
        o.vwrite = int(hit.get("vwrite", 0))
        return o, hit, True
    o, ms = D.autotune(d, z, rho, vectors=vectors, opts=o, reps=reps, device=device)
    entry = {"split": o.split, "main_passes": o.main_passes, "waves_per_simd": o.waves_per_simd,
             "vwrite": o.vwrite, "ms": ms}
    store(key, entry, path)
    return o, entry, False


def tuned_batch(offs, d, z, rho, vectors=True, opts=None, reps=3, device="cuda", path=None):
    """A Batch whose plan carries the cached (or freshly tuned) split, register and pass budgets.
    d, z, rho: device tensors of the batch (used only when tuning).  Returns (batch, entry, from_cache)."""
    from . import dpr1 as D
    o = D.opts() if opts is None else opts
    sizes = np.diff(np.asarray(offs, dtype=np.int64))
    key = key_batched(arch_of(device), sizes, vectors, o.root)
    hit = load(path).get(key)
    if hit is not None:
        o.split = int(hit["split"])
        o.main_passes = int(hit["main_passes"])
        o.waves_per_simd = int(hit.get("waves_per_simd", 0))
        return D.Batch(offs, opts=o, vectors=vectors, device=device), hit, True
    b = D.Batch(offs, opts=o, vectors=vectors, device=device)
    ms = b.autotune(d, z, rho, reps=reps)
    entry = {"split": b.plan.split, "main_passes": b.plan.opts.main_passes,
             "waves_per_simd": b.plan.opts.waves_per_simd, "vwrite": b.plan.opts.vwrite, "ms": ms}
    store(key, entry, path)
    return b, entry, False
