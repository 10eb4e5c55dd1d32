"""The parity bar of one treecode operator call: device (FP32 arithmetic,
FP64 sums) against the FP64 oracle treecode on the same tree and inputs.

Per target i, with M_i = sum_j |term_ij| the oracle's sum of term
magnitudes:

* |y_gpu - y_oracle| <= TOL * M_i.  Each FP32 term carries a few units of
  2^-24 relative rounding (its inputs, the hardware rsq of about 1 ulp, a
  few products) and the FP64 sums add nothing visible, so the expected
  error is a few times 6e-8 of M_i; TOL = 1e-5 leaves two orders of margin.
* A target may miss that bound only if it is a decision near-tie: one of
  the distances it compared (Alg. 4's |x - x_B| against c * width, or a
  pair distance against the cutoff w of Sec. 4.4) lies within TIE
  (relative) of its threshold in the oracle's FP64 arithmetic.  The device
  forms the same distance in FP32 (relative error a few 1e-7), so such a
  decision can fall the other way; no other target may miss.  The oracle
  reports each target's smallest margins (`Tree.apply(with_margins=True)`).
* At most ceil(EXEMPT_FRAC * n) targets may be exempted that way (99.99 %
  of targets within the bound).
* Relative L2 error over the targets that are not near-ties <= L2_TOL.
* Pair counts: equal when no target is a near-tie; otherwise the
  difference is at most the near-tie targets' own pair counts.
"""
import math

import numpy as np

TOL = 1e-5
TIE = 1e-6
EXEMPT_FRAC = 1e-4
L2_TOL = 1e-5
# Two device walks that make the same decisions and form the same FP32
# terms but group their additions differently (tile shapes, split walks,
# deferred subtrees).  With u = 2^-24 and M_i the sum of the target's term
# magnitudes: the lockstep walk adds a target's terms to FP32 running sums
# of at most 8 sibling nodes (and the points of one leaf, at most 8 with
# the leaf capacities tested) before its FP64 sum, at most about 8 u M_i of
# rounding; a deferred step rounds each term once and adds it in FP64; a
# split walk rounds each part's FP64 sum to FP32 once (u times the part's
# magnitudes).  Two walks then differ by at most about 18 u M_i = 1.1e-6 M_i.
ORDER_TOL = 2e-6


def same_terms(label, a, b, mag, tol=ORDER_TOL):
    """Asserts |a_i - b_i| <= tol * M_i for every target (an exact tie
    where M_i = 0); returns the largest ratio."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    mag = np.asarray(mag, np.float64)
    err = np.abs(a - b)
    if err.ndim == 2:
        err = np.linalg.norm(err, axis=1)
    pos = mag > 0
    assert np.all(err[~pos] == 0.0), label
    rel = err[pos] / mag[pos]
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= tol, f"{label}: summation-order difference {worst:.3e} M_i > {tol:g} M_i"
    return worst


def ties(margins):
    """Targets with a decision within TIE of its threshold (either column)."""
    m = np.asarray(margins, np.float64)
    return np.min(m.reshape(m.shape[0], -1), axis=1) <= TIE


def check(label, got, ref, mag, margins, pairs_gpu=None, pairs_oracle=None, l2=True,
          zero_mag_exact=True):
    """Asserts the bar for one operator call; returns a dict of the measured
    figures (printed by the caller's log line)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    mag = np.asarray(mag, np.float64)
    n = ref.shape[0]
    assert got.shape == ref.shape, (label, got.shape, ref.shape)
    assert np.all(np.isfinite(got)) and np.all(np.isfinite(ref)), label
    err = np.abs(got - ref)
    if err.ndim == 2:
        err = np.linalg.norm(err, axis=1)
    pos = mag > 0
    tie = ties(margins)
    if zero_mag_exact:
        # a target with no terms at all (every pair cut or zero) gets an
        # exact 0, unless one of its decisions is a near-tie
        assert np.all(err[~pos & ~tie] == 0.0), label
    rel = np.where(pos, err / np.where(pos, mag, 1.0), np.where(err > 0, np.inf, 0.0))
    bad = rel > TOL
    unexplained = np.where(bad & ~tie)[0]
    assert unexplained.size == 0, (
        f"{label}: {unexplained.size} targets beyond {TOL:g} of their term magnitudes with no "
        f"decision near-tie; first {unexplained[:5].tolist()} rel {rel[unexplained[:5]].tolist()}")
    n_ex = int(bad.sum())
    cap = math.ceil(EXEMPT_FRAC * n)
    assert n_ex <= cap, f"{label}: {n_ex} near-tie exemptions > {cap}"
    out = dict(n=n, exempt=n_ex, ties=int(tie.sum()), max_rel=float(rel.max()) if n else 0.0,
               max_rel_nontie=float(rel[~tie].max()) if (~tie).any() else 0.0,
               min_margin_exempt=float(np.min(np.asarray(margins)[bad])) if n_ex else None)
    if l2:
        keep = ~tie
        den = np.linalg.norm(ref[keep])
        l2v = float(np.linalg.norm((got - ref)[keep]) / den) if den > 0 else 0.0
        out["rel_l2"] = l2v
        assert l2v <= L2_TOL, f"{label}: relative L2 {l2v:.3e} > {L2_TOL:g} over non-tie targets"
    if pairs_gpu is not None and pairs_oracle is not None:
        po = np.asarray(pairs_oracle, np.int64)
        diff = int(pairs_gpu) - int(po.sum())
        out["pair_diff"] = diff
        if tie.sum() == 0:
            assert diff == 0, f"{label}: pair counts differ by {diff} with no near-tie target"
        else:
            # a turned decision replaces one representative by the terms of
            # one node at the edge of the acceptance sphere (or the reverse);
            # such a node holds far fewer points than the target's whole walk
            # takes pairs, so the tie targets' own counts bound the change
            bound = int(po[tie].sum())
            assert abs(diff) <= bound, f"{label}: pair difference {diff} > {bound}"
    return out


def fmt(r):
    s = (f"exempt={r['exempt']}/{r['n']} ties={r['ties']} max_rel={r['max_rel']:.2e} "
         f"max_rel_nontie={r['max_rel_nontie']:.2e}")
    if r.get("min_margin_exempt") is not None:
        s += f" min_margin_exempt={r['min_margin_exempt']:.1e}"
    if "rel_l2" in r:
        s += f" rel_l2={r['rel_l2']:.2e}"
    if "pair_diff" in r:
        s += f" pair_diff={r['pair_diff']}"
    return s
