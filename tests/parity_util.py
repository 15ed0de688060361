"""Helpers shared by the GPU parity tests (test infrastructure)."""
import math

import numpy as np

TINY = 1e-5   # segments shorter than this (cell units) are tie artefacts: a
              # crossing through an edge or corner is split into a zero-length
              # segment on the GPU (axes taken in x<y<z order) while the oracle,
              # which looks the next leaf up from scratch, goes diagonally.


def _clean(seg):
    return seg[seg["ds"] > TINY]


def compare_trace(gpu_seg, orc_seg, rtol, atol=1e-12):
    """Compare one package's segments.  Returns (match, n_compared,
    max_rel_err, path_rel_err, first_mismatch_index)."""
    g, o = _clean(gpu_seg), _clean(orc_seg)
    n = min(len(g), len(o))
    max_rel = 0.0
    for i in range(n):
        if g["cell"][i] != o["cell"][i] or g["event"][i] != o["event"][i]:
            return False, i, max_rel, float("nan"), i
        d = abs(g["ds"][i] - o["ds"][i])
        if d > atol + rtol * abs(o["ds"][i]):
            return False, i, max(max_rel, d / max(abs(o["ds"][i]), 1e-300)), float("nan"), i
        max_rel = max(max_rel, d / max(abs(o["ds"][i]), 1e-300))
    if len(g) != len(o):
        return False, n, max_rel, float("nan"), n
    pg, po = g["ds"].sum(), o["ds"].sum()
    return True, n, max_rel, abs(pg - po) / max(po, 1e-300), -1


def batch_z(gpu_batches, orc_batches):
    """Per-cell z-scores between two sets of independent batches."""
    g = np.asarray(gpu_batches)
    o = np.asarray(orc_batches)
    mg, mo = g.mean(0), o.mean(0)
    sg = g.std(0, ddof=1) / math.sqrt(g.shape[0])
    so = o.std(0, ddof=1) / math.sqrt(o.shape[0])
    den = np.sqrt(sg * sg + so * so)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = (mg - mo) / den
    return z, mg, mo
