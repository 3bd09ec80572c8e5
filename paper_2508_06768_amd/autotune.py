"""Schedule autotuner for the fused step.

The kernels take a ray-to-wavefront schedule (``dus_schedule``): interfaces
per lane per tile in the forward (0 = chosen per fan table, 4, 8, 16) and the
adjoint (4, 8), the
number of neighbouring rays that share one LDS box in the dL/dZ scatter (2,
4, 8), the number of consecutive rays kept on one XCD (1..64), and the ray
length from which several wavefronts share a ray (``span_samples``: never,
or 1024..8192 samples, tried only up to the plan's longest ray).
``autotune`` times the candidates on the caller's actual plan and inputs
with HIP events (coordinate descent in that order, each candidate over
``reps`` steps), installs the fastest on the plan and remembers it in a JSON
cache keyed by GPU architecture and a shape class of the workload.

Cache file: ``$DUS_AUTOTUNE_CACHE`` or ``~/.cache/diffus_autotune.json``.
"""
from __future__ import annotations

import json
import os

import torch

FWD_CHUNKS = (0, 4, 8, 16)
BWD_CHUNKS = (4, 8)
XCD_GROUPS = (1, 4, 8, 16, 32, 64)
SCATTER_RAYS = (2, 4, 8)
SPAN_SAMPLES = (-1, 1024, 2048, 4096, 8192)


def _cache_path() -> str:
    return os.environ.get("DUS_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                             "diffus_autotune.json"))


def shape_key(geom) -> str:
    """Architecture + coarse workload class (powers of two of the sizes)."""
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    lg = lambda x: max(0, int(x)).bit_length()  # noqa: E731
    rays = sum(int(f.n_rays) for f in geom.fans)
    smax = max((int(f.n_samples) for f in geom.fans), default=0)
    ph = geom.phys
    return (f"{arch}|vol{'x'.join(str(lg(n)) for n in geom.shape)}|poses{lg(geom.n_poses)}|rays{lg(rays)}"
            f"|s{lg(smax)}|spk{int(bool(ph.speckle_on))}|blur{int(bool(ph.blur_on))}|refl{int(ph.refl_mode)}")


def load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def autotune(step, run, reps: int = 10, use_cache: bool = True, verbose: bool = False) -> dict:
    """Pick the fastest schedule for ``step`` (a ``FusedStep``).

    run: zero-argument callable that executes one step with the caller's
    buffers (it is called with each candidate installed).
    Returns {"schedule": ..., "ms": ..., "trials": [...]}.
    """
    key = shape_key(step.geom)
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        step.set_schedule(**cache[key]["schedule"])
        return dict(cache[key], cached=True)
    best = dict(step.get_schedule())
    trials = []

    def trial(cand):
        step.set_schedule(**cand)
        ms = _time(run, reps)
        trials.append({"schedule": dict(cand), "ms": ms})
        if verbose:
            print("autotune", cand, f"{ms:.3f} ms", flush=True)
        return ms

    best_ms = trial(best)
    longest = max((int(f.n_samples) for f in step.geom.fans), default=0)
    spans = tuple(v for v in SPAN_SAMPLES if v <= longest)
    for field, values in (("fwd_chunk", FWD_CHUNKS), ("bwd_chunk", BWD_CHUNKS), ("scatter_rays", SCATTER_RAYS),
                          ("xcd_group", XCD_GROUPS), ("span_samples", spans)):
        for val in values:
            if val == best[field]:
                continue
            cand = dict(best, **{field: val})
            ms = trial(cand)
            if ms < best_ms:
                best, best_ms = cand, ms
    step.set_schedule(**best)
    out = {"schedule": best, "ms": best_ms, "trials": trials}
    if use_cache:
        cache[key] = {"schedule": best, "ms": best_ms}
        save_cache(cache)
    return dict(out, cached=False)
