"""Shared checks for GPU-vs-oracle parity.

Tolerance (per unit, component): with M = max(|lo_o|, |hi_o|),
  |lo_g - lo_o| <= 1e-4 M  and  |hi_g - hi_o| <= 1e-4 M      (parity)
  lo_g <= lo_o + 1e-6 M    and  hi_g >= hi_o - 1e-6 M        (never narrower)
M = 0 requires exactly [0, 0]; infinite oracle ends must match exactly.
"""
import numpy as np

REL = 1e-4
NARROW = 1e-6


def check_bounds(lo_g, hi_g, lo_o, hi_o, where=""):
    lo_g, hi_g, lo_o, hi_o = (np.asarray(a, dtype=np.float64) for a in (lo_g, hi_g, lo_o, hi_o))
    assert lo_g.shape == lo_o.shape and hi_g.shape == hi_o.shape, where
    inf_o = ~np.isfinite(lo_o) | ~np.isfinite(hi_o)
    assert np.array_equal(lo_g[inf_o], lo_o[inf_o]) and np.array_equal(hi_g[inf_o], hi_o[inf_o]), \
        "%s: infinite rows differ" % where
    fin = ~inf_o
    assert np.isfinite(lo_g[fin]).all() and np.isfinite(hi_g[fin]).all(), "%s: GPU non-finite" % where
    M = np.maximum(np.abs(lo_o), np.abs(hi_o))[fin]
    lg, hg, lo, ho = lo_g[fin], hi_g[fin], lo_o[fin], hi_o[fin]
    zero = M == 0
    assert (lg[zero] == 0).all() and (hg[zero] == 0).all(), "%s: exact zeros lost" % where
    e_lo = np.abs(lg - lo) / np.where(zero, 1, M)
    e_hi = np.abs(hg - ho) / np.where(zero, 1, M)
    worst = max(e_lo.max(initial=0), e_hi.max(initial=0))
    assert worst <= REL, "%s: relative error %.3e" % (where, worst)
    assert (lg <= lo + NARROW * M).all() and (hg >= ho - NARROW * M).all(), "%s: GPU narrower" % where
    return worst


def sampled_violations(remainder, nom, blo, bhi, lo, hi, per, seed, chunk=64):
    """Violations of [lo, hi] (per unit) by the true remainder at `per`
    sampled points of each unit's box [blo, bhi] (half uniform, a quarter
    vertices, a quarter mixed).  remainder(nom_chunk, pts [U][per][n]) ->
    (r, eps) [U][per][m] with eps bounding the FP64 evaluation error; a
    violation is r > hi + eps or r < lo - eps.  Returns (violations, samples)."""
    import workloads as W
    rng = W.rng_for(seed)
    viol = 0
    count = 0
    for s in range(0, nom.shape[0], chunk):
        e = min(nom.shape[0], s + chunk)
        pts = W.sample_box_points(rng, blo[s:e], bhi[s:e], per)
        r, eps = remainder(nom[s:e], pts)
        viol += int(((r > hi[s:e, None] + eps) | (r < lo[s:e, None] - eps)).sum())
        count += (e - s) * per
    return viol, count
