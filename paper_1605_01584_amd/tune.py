"""Autotuning of tile schedules, with a JSON cache.

* ``best_cfg(n, l, mode)``: the fastest ``TileCfg`` for an all-pairs run of
  that shape, measured by ``pcc_autotune`` (HIP events, median of reps) on a
  synthetic Z of exactly that shape (run time does not depend on the
  values), cached per (device, mode, n, l_pad).
* ``tune_batch(xs, mode)``: the fastest per-dataset tile sizes for one
  uneven batch.  Candidate assignments (all 256, all 128, "128 below a size
  threshold" rules, and 128 where 256-wide tiles would compute a given share
  more pair slots) are built as batch plans and timed as whole graph
  launches, since inside one persistent launch what matters is the sum of
  per-job costs and the balance of the shared job counter, not each
  dataset's stand-alone speed.  Cached per (device, mode, batch signature).

The cache file is ``$PCC_TUNE_CACHE`` or ``~/.cache/pcc_tune.json``.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Sequence

import paper_1605_01584_amd as pcc

_CACHE_ENV = "PCC_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(_CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache",
                                                      "pcc_tune.json")


def _load() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass  # a read-only home is fine: tuning is then redone per process


def _device_key() -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    return f"{getattr(props, 'gcnArchName', props.name)}:{props.multi_processor_count}"


def candidates() -> List[pcc.TileCfg]:
    out = []
    for tile in (256, 128):
        out.append(pcc.TileCfg(tile, 0, 1, 0))
        for band in (2, 4, 8, 16):
            out.append(pcc.TileCfg(tile, 1, band, 0))
    return out


def best_cfg(n: int, l: int, mode="split", reps: int = 3, use_cache: bool = True,
             r=None) -> pcc.TileCfg:
    """Fastest schedule for n profiles of l samples.  Timed at that very
    shape (the tile count and the band balance depend on n, the per-tile
    work on l_pad), on random data; r (nullable) is an n(n-1)/2 float32
    device buffer to time into, e.g. the caller's own output."""
    mode_i = pcc._mode(mode)
    zd = pcc.z_layout(n, l, mode_i)
    key = f"allpairs|{_device_key()}|{mode_i}|n={n}|lpad={zd.l_pad}"
    cache = _load() if use_cache else {}
    if key in cache:
        return pcc.TileCfg(*cache[key]["cfg"])
    import torch
    x = torch.randn(n, l, device="cuda", dtype=torch.float32)
    z, zd = pcc.normalize(x, mode_i)
    del x
    npairs = n * (n - 1) // 2
    if r is None:
        r = torch.empty(npairs, dtype=torch.float32, device="cuda")
    elif r.numel() < npairs or r.dtype != torch.float32 or not r.is_cuda:
        raise ValueError("r must be a device float32 tensor of n(n-1)/2")
    cands = candidates()
    best, times = pcc.autotune(z, zd, r, cands, reps=reps)
    if use_cache:
        cache = _load()
        cache[key] = {"cfg": list(best.as_tuple()), "times_ms": times,
                      "cands": [list(c.as_tuple()) for c in cands]}
        _store(cache)
    return best


def _signature(shapes: Sequence[tuple], mode_i: int) -> str:
    h = hashlib.sha1(repr((mode_i, tuple(shapes))).encode()).hexdigest()[:16]
    return f"batch|{_device_key()}|{mode_i}|{h}"


def _tile_slots(n: int, t: int) -> int:
    """Pair slots the tiles of width t compute for n profiles (whole tiles of
    the inclusive triangle, padding rows included)."""
    m = -(-n // t)
    return m * (m + 1) // 2 * t * t


def _assignments(shapes: Sequence[tuple]) -> Dict[str, List[int]]:
    """Candidate tile widths per dataset: all one width, 128 below a size
    threshold, or 128 where 256-wide tiles would compute a given share more
    pair slots (padding rows and whole diagonal tiles), alone or with the
    size rule."""
    out = {"all256": [256] * len(shapes), "all128": [128] * len(shapes)}
    for thr in (1024, 1536, 2048, 3072, 4096):
        out[f"128_below_{thr}"] = [128 if n < thr else 256 for n, _ in shapes]
    excess = [_tile_slots(n, 256) / _tile_slots(n, 128) - 1.0 for n, _ in shapes]
    for x in (0.1, 0.2, 0.35):
        out[f"128_over_{x:g}_excess"] = [128 if e > x else 256 for e in excess]
        out[f"128_below_2048_or_over_{x:g}_excess"] = [
            128 if (n < 2048 or e > x) else 256 for (n, _), e in zip(shapes, excess)]
    # identical assignments are timed once
    seen, uniq = set(), {}
    for name, tiles in out.items():
        if tuple(tiles) not in seen:
            seen.add(tuple(tiles))
            uniq[name] = tiles
    return uniq


def tune_batch(xs: Sequence, mode="split", reps: int = 3, use_cache: bool = True):
    """Per-dataset tiles for one batch; returns (tiles, {name: ms})."""
    import torch
    mode_i = pcc._mode(mode)
    shapes = [tuple(int(s) for s in x.shape) for x in xs]
    key = _signature(shapes, mode_i)
    cache = _load() if use_cache else {}
    if key in cache:
        return list(cache[key]["tiles"]), cache[key]["times_ms"]
    times, best, best_tiles = {}, None, None
    st = torch.cuda.current_stream()
    for name, tiles in _assignments(shapes).items():
        plan = pcc.BatchPlan(xs, mode, tiles=tiles)
        plan.launch()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(st)
            plan.launch()
            b.record(st)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        plan.close()
        ts.sort()
        times[name] = ts[len(ts) // 2]
        if best is None or times[name] < best:
            best, best_tiles = times[name], tiles
    if use_cache:
        cache = _load()
        cache[key] = {"tiles": best_tiles, "times_ms": times, "shapes": shapes}
        _store(cache)
    return best_tiles, times
