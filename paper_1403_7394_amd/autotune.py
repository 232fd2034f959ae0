"""Launch-shape autotuner for libhap.

Times candidate launch shapes on the actual problem with short runs (HIP events on the
problem's stream) and keeps the fastest; results are cached per device architecture and
size bucket in a JSON file ($HAP_TUNING_CACHE, default ~/.cache/hap_mi355x/tuning.json).

* tune_sweep(h):  threads / chunks / rows per workgroup / streaming of the row pass of a
  single problem (Hap), timed with the library's per-launch event timing.
* tune_batch(bt, X, damping):  threads, workgroup count and row groups of the batched
  persistent kernel (HapBatch), timed over a short run of the whole batch.
"""
from __future__ import annotations

import json
import math
import os

from . import hap

_CACHE_ENV = "HAP_TUNING_CACHE"


def _cache_path() -> str:
    return os.environ.get(_CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "hap_mi355x",
                                                      "tuning.json")


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value) -> None:
    cache = _load_cache()
    cache[key] = value
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _bucket(n: int) -> int:
    return 1 << max(0, math.ceil(math.log2(max(n, 1))))


def sweep_candidates(n: int, elem_size: int):
    vw = 16 // elem_size
    out = []
    for threads, chunks in [(64, 1), (64, 2), (64, 4), (128, 2), (128, 4), (256, 2), (256, 4), (256, 8), (512, 1),
                            (512, 2), (512, 4), (1024, 1), (1024, 2)]:
        if threads * chunks * vw < n or threads * chunks * vw >= 4 * n and threads > 64:
            continue
        for rb in sorted({max(1, n // 256), max(1, n // 512), max(1, n // 1024)}):
            out.append((threads, chunks, rb, False))
    if not out or n > 4096:
        chunks = -(-n // (1024 * vw))
        if chunks <= 16:
            for rb in sorted({max(1, n // 256), max(1, n // 512)}):
                out.append((1024, chunks, rb, True))
        if elem_size == 4 and 16384 < n <= 512 * 16 * 4:
            for rb in sorted({max(1, n // 256), max(1, n // 512)}):
                out.append((512, 16, rb, True))   # the held-row pass
        if elem_size == 4 and 512 * 16 * 4 < n <= 512 * 32 * 4:
            for pairs in (128, 64):
                out.append((512, 32, -(-n // pairs), True))   # the paired pass
    return out


def tune_sweep(h: "hap.Hap", sweeps: int = 3, use_cache: bool = True):
    """Pick the fastest row-pass shape for this problem and set it on h.  Runs sweeps on h,
    so call it on a context whose iteration state may be consumed (or re-create it)."""
    esz = 4 if str(h.dtype).endswith("float32") else 8
    key = f"sweep:{_arch()}:n{_bucket(h.n)}:e{esz}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            try:
                h.set_launch(*hit[:3], streaming=bool(hit[3]))
                return tuple(hit)
            except hap.HapError:
                pass
    best, best_us = None, float("inf")
    for shape in sweep_candidates(h.n, esz):
        try:
            h.set_launch(*shape[:3], streaming=shape[3])
        except hap.HapError:
            continue
        h.iterate(1)
        h.profile(True)
        h.iterate(sweeps)
        row_ms, row_n, col_ms, col_n = h.profile_read()
        h.profile(False)
        us = (row_ms + col_ms) / max(row_n, 1) * 1e3
        if us < best_us:
            best, best_us = shape, us
    if best is not None:
        h.set_launch(*best[:3], streaming=best[3])
        _store(key, list(best) + [best_us])
    return best


def batch_signature(sizes) -> str:
    hist = {}
    for n in sizes:
        b = _bucket(n)
        hist[b] = hist.get(b, 0) + 1
    return ",".join(f"{b}x{hist[b]}" for b in sorted(hist))


def batch_candidates(cus: int, count: int):
    """(threads, workgroups, row_groups) shapes tried for a batch of count problems."""
    out = []
    for threads, groups in ((512, 4), (1024, 4), (512, 2), (256, 1), (512, 1)):
        for per_cu in (1, 2, 4):
            wg = min(cus * per_cu, max(1, count))
            if (threads, wg, groups) not in out:
                out.append((threads, wg, groups))
    return out


def split_candidates():
    """(split_n, max_members) settings tried for the batch's large problems (0: no split)."""
    return [(0, 1), (1448, 2), (1024, 2), (1024, 4), (724, 4), (724, 8)]


def tune_batch(bt: "hap.HapBatch", X, damping: float, iters: int = 50, use_cache: bool = True):
    """Pick threads, workgroup count and row groups of the persistent batched kernel for this
    batch (every shape computes the same bits, so only time decides), then the split of its
    large problems over gangs of workgroups (a split changes the order of the column sums of the
    split problems, so it is chosen with the shape fixed).  Each candidate runs `iters`
    iterations: enough that the sweeps decide, as in a run of a few hundred iterations, rather
    than the build and median of the largest problems, which a split shortens.  Returns
    (threads, workgroups, row_groups, split_n, max_members)."""
    import torch
    key = f"batch3:{_arch()}:d{bt.d}:L{bt.levels}:i{iters}:{batch_signature(bt.sizes)}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit and len(hit) == 6:
            try:
                bt.set_launch(*hit[:3])
                bt.set_split(*hit[3:5])
                return tuple(hit[:5])
            except hap.HapError:
                pass
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = bt.outputs(X.device)

    def time_run():
        bt.run(X, damping, 1, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bt.run(X, damping, iters, out=out)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    bt.set_split(0, 1)
    best, best_ms = None, float("inf")
    for shape in batch_candidates(cus, bt.count):
        bt.set_launch(*shape)
        ms = time_run()
        if ms < best_ms:
            best, best_ms = shape, ms
    bt.set_launch(*best)
    best_split = (0, 1)
    for split in split_candidates()[1:]:
        bt.set_split(*split)
        ms = time_run()
        if ms < best_ms:
            best_split, best_ms = split, ms
    bt.set_split(*best_split)
    result = tuple(best) + tuple(best_split)
    _store(key, list(result) + [best_ms])
    return result
