"""Autotuner for the persistent Monte Carlo launches.

Chooses the launch schedule of the persistent kernels -- workgroup size,
persistent workgroups per compute unit, package ids per grant from the
global counter, lane-refill threshold, deferred scattering threshold and,
for batches, the tile size -- by timing short
calibration runs with HIP events (the library's own per-launch timing) and
keeps the fastest candidate per problem class.  The class key buckets the
grid kind, the number of cells (powers of two), the optical depth of a
cell and the source class, so that one tuning serves every problem of the
same shape.  Only the schedule is tuned: results do not depend on it (a
package's random numbers depend only on its identity), which the GPU tests
check.
"""
from __future__ import annotations

import itertools
import json
import math
import os

DEFAULT_SPACE = {
    "block": (128, 256, 512),
    "blocks_per_cu": (2, 4, 6, 8),
    "chunk": (256, 512),
    "refill_min": (1, 16),
    "scatter_min": (1,),
}
BATCH_TILES = (4096, 16384, 65536)


def class_key(kind: str, ncells: int, tau_cell: float, source: str) -> str:
    """Problem class: grid kind, log2 bucket of the cell count, log10
    bucket of the optical depth of one cell, source class."""
    nb = int(round(math.log2(max(ncells, 1))))
    tb = int(math.floor(math.log10(max(tau_cell, 1e-12))))
    return f"{kind}:n2^{nb}:tau1e{tb}:{source}"


def candidates(space=None):
    space = space or DEFAULT_SPACE
    keys = sorted(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        yield dict(zip(keys, vals))


def pick_best(timings):
    """timings: list of (config, seconds); the fastest, ties to the first."""
    best = None
    for cfg, t in timings:
        if best is None or t < best[1]:
            best = (cfg, t)
    return best


class Autotuner:
    """Times candidates through `measure(config) -> seconds` callables and
    caches the best configuration per class key (optionally in a JSON
    file)."""

    def __init__(self, cache_path: str | None = None):
        self.cache_path = cache_path
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def lookup(self, key):
        return self.cache.get(key)

    def tune(self, key, measure, space=None, repeats=2):
        """Run every candidate `repeats` times (min taken) unless the class
        is cached; returns the best configuration."""
        hit = self.cache.get(key)
        if hit is not None:
            return hit["config"]
        timings = []
        for cfg in candidates(space):
            t = min(measure(cfg) for _ in range(repeats))
            timings.append((cfg, t))
        cfg, t = pick_best(timings)
        self.cache[key] = {"config": cfg, "seconds": t,
                           "tried": [{"config": c, "seconds": s} for c, s in timings]}
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)
        return cfg


def apply(ctx, cfg: dict):
    """Set the library options of a configuration (tile size excluded)."""
    for k, v in cfg.items():
        if k != "tile_packages":
            ctx.set_option(k, int(v))


def event_timer(ctx, run):
    """measure(config) for a context: applies the configuration, runs
    `run()` once as warm-up and once timed, and returns the summed duration
    of the timed MC launches (HIP events around each launch)."""
    def measure(cfg):
        apply(ctx, cfg)
        prev = ctx.get_option("timing")
        ctx.set_option("timing", 1)
        run(cfg)
        ctx.mc_timing(reset=True)
        run(cfg)
        ms, n = ctx.mc_timing(reset=True)
        ctx.set_option("timing", prev)
        return ms / 1e3
    return measure
