"""Launch-shape autotuner for the mfIPM kernels.

A launch shape is (workgroups, team_size, tile):
  * single solves: the number of workgroups of the one team (barrier cost
    grows with it, work per workgroup shrinks with it) and the operator tile
    (partial DCT: log2 of the column-FFT length N1 of the four-step split;
    dense: rows per item of the two-pass path);
  * batched calls: workgroups per team (instances per round vs. bandwidth
    per instance).

`tune()` runs the real call for each candidate shape, times the kernel with
the library's HIP events (`Solver.last_kernel_ms`), keeps the fastest and
stores it in a JSON cache keyed by device architecture, operator kind, the
largest n and m, batch size and operator sharing.  `Solver` looks shapes up
in the user cache, then in the table of shapes measured on MI355X that ships
with the package, and otherwise lets the library choose.
"""
from __future__ import annotations

import json
import math
import os
import time

_PKG = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(_PKG, "tuned_mi355x.json")


def user_cache_path() -> str:
    return os.environ.get("MFIPM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mfipm_autotune.json"))


def make_key(arch: str, op_kind: int, n_max: int, m_max: int, batch: int, shared: bool,
             backward: bool = False) -> str:
    return (f"{arch}|{'bwd' if backward else 'fwd'}|op={op_kind}|n={n_max}|m={m_max}|batch={batch}"
            f"|shared={int(bool(shared))}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


_memo = {}  # path -> (mtime, table): tables are re-read only when the file changes


def _table(path):
    try:
        mtime = os.stat(path).st_mtime_ns
    except OSError:
        return {}
    hit = _memo.get(path)
    if hit is None or hit[0] != mtime:
        hit = (mtime, _load(path))
        _memo[path] = hit
    return hit[1]


def lookup(key: str):
    """Tuned (workgroups, team_size, tile) for `key`, or None."""
    for path in (user_cache_path(), SHIPPED):
        rec = _table(path).get(key)
        if rec:
            return tuple(rec["shape"])
    return None


def store(key: str, shape, ms: float, path: str | None = None):
    path = path or user_cache_path()
    d = _load(path)
    d[key] = {"shape": list(shape), "kernel_ms": ms, "time": time.time()}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(op_kind: int, n_max: int, m_max: int, batch: int, num_cu: int = 256):
    """Candidate shapes for one call."""
    out = []
    if batch == 1:
        if op_kind in (1, 3):  # partial DCT or DST (one kernel)
            lh = int(math.log2(n_max)) - 1
            base = lh // 2
            tiles = sorted({t for t in (base - 2, base - 1, base, base + 1) if 1 <= t <= 9 and 3 <= lh - t <= 11})
            for wg in (0, 32, 64, 96, 128, 192, 256):
                for t in tiles:
                    out.append((wg, 0, t))
        elif op_kind == 2:  # partial Walsh-Hadamard: log2 of the column length
            ln = int(math.log2(n_max))
            base = ln // 2
            tiles = sorted({t for t in (base - 1, base, base + 1) if 2 <= t <= min(13, ln - 2) and ln - t <= 12})
            for wg in (0, 32, 64, 128, 192, 256):
                for t in tiles:
                    out.append((wg, 0, t))
        else:
            for wg in (0, 16, 32, 64, 128, 256):
                out.append((wg, 0, 0))
    else:
        for ts in (1, 2, 4, 8, 16, 32, 64, 128, 256):
            if ts <= num_cu:
                out.append((0, ts, 0))
    return out


def tune(solver, call, key: str, shapes, reps: int = 3, path: str | None = None, verbose: bool = False):
    """Times `call()` (a closure doing one solve on `solver`) for every shape
    and stores the fastest under `key`.  Returns (best_shape, best_ms, table)."""
    table = []
    best = None
    for shape in shapes:
        solver.set_launch(*shape)
        try:
            call()  # warm
            ms = min(_timed(solver, call) for _ in range(reps))
        except Exception as e:  # a shape the device cannot host
            if verbose:
                print("skip", shape, e, flush=True)
            continue
        table.append((shape, ms))
        if verbose:
            print("shape", shape, f"{ms:.3f} ms", flush=True)
        if best is None or ms < best[1]:
            best = (shape, ms)
    solver.set_launch(0, 0, 0)
    if best is not None:
        store(key, best[0], best[1], path)
    return (best[0], best[1], table) if best else (None, None, table)


def _timed(solver, call) -> float:
    call()
    return solver.last_kernel_ms()
