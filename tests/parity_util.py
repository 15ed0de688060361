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


def relative_bias(gpu_batches, orc_batches, sel):
    """Unweighted mean over the selected cells of the symmetric relative
    difference 2 (mg - mo) / (mg + mo), and its standard error.

    The symmetric form has expectation zero when both sides sample the same
    distribution (dividing by the noisy oracle mean alone would be biased
    upwards by its relative variance).  The standard error comes from the
    batches, which are independent: the per-cell differences are not (one
    package deposits along its whole path), so a per-cell standard error
    would understate it several times on large grids."""
    g = np.asarray(gpu_batches)[:, sel]
    o = np.asarray(orc_batches)[:, sel]
    m = 0.5 * (g.mean(0) + o.mean(0))
    with np.errstate(divide="ignore", invalid="ignore"):
        sg = (g / m).mean(1)
        so = (o / m).mean(1)
    B = g.shape[0]
    return float(sg.mean() - so.mean()), float(math.sqrt(sg.var(ddof=1) / B + so.var(ddof=1) / B))


KS_CELLS = 2000   # cells in the KS test; a random subset when more are selected


def check_z(gpu_batches, orc_batches, hits, label):
    """Parity criteria over the cells with more than 10^3 hits (summed over
    the batches):
      * per-cell z-scores: |mean z| < 0.1, std z within 0.1 of the
        Student-t value, KS p > 1e-3 against t(dof) on at most KS_CELLS
        cells drawn at random (neighbouring cells share packages, so
        their z-scores are correlated and a KS test over tens of
        thousands of cells rejects even the oracle against itself);
      * aggregate relative bias sum(mg - mo) / sum(mo) below 0.3%;
      * unweighted mean relative bias (relative_bias) below 0.3% plus
        three of its standard errors, over these cells and over the cells
        with more than 10^4 hits.  The standard error is printed: where
        it is well below 0.3% (the full-size clouds) the check is a 0.3%
        bound; on small grids a few bright cells make the batch-to-batch
        fluctuations of the mean larger, and the check is what the sample
        can resolve."""
    from scipy import stats
    z, mg, mo, dof = batch_z(gpu_batches, orc_batches)
    B = dof // 2 + 1
    sel = hits * B > 1000
    assert sel.sum() >= 100, f"{label}: only {sel.sum()} well-sampled cells"
    zs = z[sel]
    t_std = math.sqrt(dof / (dof - 2.0))
    rng = np.random.default_rng(12345)
    zk = zs if zs.size <= KS_CELLS else rng.choice(zs, KS_CELLS, replace=False)
    p = stats.kstest(zk, stats.t(dof).cdf).pvalue
    agg = float(np.sum(mg[sel] - mo[sel]) / np.sum(mo[sel]))
    b3, se3 = relative_bias(gpu_batches, orc_batches, sel)
    sel4 = hits * B > 10000
    b4, se4 = relative_bias(gpu_batches, orc_batches, sel4) if sel4.sum() >= 50 else (0.0, 0.0)
    print(f"\n{label}: {zs.size} cells, z mean {zs.mean():.3f} std {zs.std():.3f} (t std {t_std:.3f}) "
          f"KS p {p:.3g} ({zk.size} cells); aggregate bias {agg:.2e}; mean relative bias {b3:.2e} +- {se3:.1e} "
          f"(> 10^3 hits), {b4:.2e} +- {se4:.1e} ({int(sel4.sum())} cells > 10^4 hits)")
    assert abs(zs.mean()) < 0.1
    assert abs(zs.std() - t_std) < 0.1
    assert p > 1e-3
    assert abs(agg) < 3e-3
    assert abs(b3) < 3e-3 + 3.0 * se3
    assert abs(b4) < 3e-3 + 3.0 * se4
