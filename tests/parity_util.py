"""Helpers shared by the GPU parity tests (test infrastructure)."""
import math

import numpy as np

TINY = 1e-5   # segments shorter than this (cell units) are tie artefacts: a
              # crossing through an edge or corner is split into a zero-length
              # segment on the GPU (axes taken in x<y<z order) while the oracle,
              # which looks the next leaf up from scratch, goes diagonally.


def _clean(seg):
    """Segments longer than TINY; the length of each shorter one is added
    to the segment before it, so that a crossing split in two at a tie
    keeps its whole length on both sides."""
    keep = seg["ds"] > TINY
    out = seg[keep].copy()
    if not keep.all() and len(out):
        prev = np.cumsum(keep) - 1           # last kept segment at or before each one
        fold = ~keep & (prev >= 0)
        np.add.at(out["ds"], prev[fold], seg["ds"][fold])
    return out


def compare_trace(gpu_seg, orc_seg, rtol, atol=1e-12):
    """Compare one package's segments.  Returns (match, n_compared,
    max_rel_err, path_rel_err, first_mismatch_index): match requires the
    same cells and events and every length within atol + rtol * ds."""
    same, n, max_abs, path_rel, first = compare_structure(gpu_seg, orc_seg)
    if not same:
        return False, n, float("nan"), float("nan"), first
    g, o = _clean(gpu_seg), _clean(orc_seg)
    d = np.abs(g["ds"] - o["ds"])
    bad = np.nonzero(d > atol + rtol * np.abs(o["ds"]))[0]
    rel = float(np.max(d / np.maximum(np.abs(o["ds"]), 1e-300))) if len(d) else 0.0
    if len(bad):
        return False, int(bad[0]), rel, path_rel, int(bad[0])
    return True, len(g), rel, path_rel, -1


def compare_structure(gpu_seg, orc_seg):
    """Same cell and event sequence?  Returns (same, n, max_abs_ds_err,
    path_rel_err, first_structural_mismatch)."""
    g, o = _clean(gpu_seg), _clean(orc_seg)
    n = min(len(g), len(o))
    cm = np.nonzero((g["cell"][:n] != o["cell"][:n]) | (g["event"][:n] != o["event"][:n]))[0]
    if len(cm):
        return False, n, float("nan"), float("nan"), int(cm[0])
    if len(g) != len(o):
        return False, n, float("nan"), float("nan"), n
    pg, po = g["ds"].sum(), o["ds"].sum()
    max_abs = float(np.max(np.abs(g["ds"] - o["ds"]))) if n else 0.0
    return True, n, max_abs, abs(pg - po) / max(po, 1e-300), -1


def batch_z(gpu_batches, orc_batches):
    """Per-cell z-scores between two sets of B independent batches with the
    pooled batch variance: under the null hypothesis z follows Student's t
    with 2B - 2 degrees of freedom.  Returns (z, mean_gpu, mean_orc, dof)."""
    g = np.asarray(gpu_batches)
    o = np.asarray(orc_batches)
    B = g.shape[0]
    mg, mo = g.mean(0), o.mean(0)
    sp2 = 0.5 * (g.var(0, ddof=1) + o.var(0, ddof=1))
    with np.errstate(divide="ignore", invalid="ignore"):
        z = (mg - mo) / np.sqrt(sp2 * 2.0 / B)
    return z, mg, mo, 2 * B - 2


def check_z(z, mg, mo, dof, label):
    """Parity criteria on selected cells: |mean z| < 0.1, std z within 0.1
    of the Student-t value, KS p > 1e-3 against t(dof), aggregate relative
    bias sum(mg - mo) / sum(mo) below 0.3%."""
    from scipy import stats
    t_std = math.sqrt(dof / (dof - 2.0))
    p = stats.kstest(z, stats.t(dof).cdf).pvalue
    bias = float(np.sum(mg - mo) / np.sum(mo))
    print(f"\n{label}: {z.size} cells, z mean {z.mean():.3f} std {z.std():.3f} (t std {t_std:.3f}) "
          f"KS p {p:.3g} bias {bias:.2e}")
    assert abs(z.mean()) < 0.1
    assert abs(z.std() - t_std) < 0.1
    assert p > 1e-3
    assert abs(bias) < 3e-3
