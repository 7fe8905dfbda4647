"""Pins of the oracle's finite-tau covering from the rejection side (Sec. 4.1
greedy loop with the local L-Lebesgue test of Sec. 4.2.1, eq. calLstab).

A node j is a candidate of center c when it lies in c's closed retention
ball, is eligible and no earlier center kept it; with owners assigned once,
that is exactly "j in ball(c), owner(j) >= c".  The tests replay the
traversal from the oracle's final owners and check every decision with
weights recomputed one stencil at a time:
  - owner(j) == c  (kept):     j is the center or Lambda_j <= tau Lambda_ref;
  - owner(j) >  c  (rejected): Lambda_j >  tau Lambda_ref.
A covering that rejected every non-center, or kept nodes it should reject,
fails one of the two.

An exact case (tests/golden/lebesgue_rational_case.json) pins the whole
covering, kept and rejected sets included, against a derivation in rational
arithmetic on polynomial-FD stencils (n = M, where eq. rbffd_linsys reduces
to Psi^T w = L psi), with no oracle arithmetic in it.
"""
import json
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

import nodesets
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sqd(a, b):
    # the oracle's order: ((dx*dx) + (dy*dy)) + (dz*dz)
    s = (a[0] - b[0]) * (a[0] - b[0])
    for t in range(1, len(a)):
        s = s + (a[t] - b[t]) * (a[t] - b[t])
    return s


def _reference(P):
    rel = P - P[0]
    cen = np.zeros(P.shape[1])
    for q in range(len(P)):  # summed in stencil order, as the rule states
        cen = cen + rel[q]
    cen = cen / len(P)
    d = ((rel - cen) ** 2).sum(1)
    return int(np.argmin(d))  # first minimum


def _replay(x, idx, rho2, eligible, delta, tau, owner, centers, m, l):
    """Return (kept, rejected) counts; assert every decision."""
    t = 1.0 - delta
    t2 = t * t
    kept = rejected = 0
    for c in centers:
        st = idx[c]
        thr = t2 * rho2[c]
        cand = []
        for q, j in enumerate(st):
            if eligible is not None and not eligible[j]:
                continue
            if owner[j] < c:
                continue  # kept by an earlier center
            if _sqd(x[c], x[j]) <= thr:
                cand.append(q)
        assert cand and cand[0] == 0  # the center is its own candidate
        assert owner[c] == c
        ref = _reference(x[st])
        W = oracle.stencil_weights(x[st], x[st[[ref] + cand]], m, l)
        lam = np.abs(W).sum(1)
        lref = lam[0]
        for i, q in enumerate(cand[1:], start=2):
            j = st[q]
            if owner[j] == c:
                assert lam[i] <= tau * lref, (c, j)
                kept += 1
            else:
                assert owner[j] > c
                assert lam[i] > tau * lref, (c, j, lam[i], tau * lref)
                rejected += 1
        # nodes outside the ball are never kept by c
        inside = set(st[q] for q in cand)
        for j in st:
            if owner[j] == c:
                assert j in inside
    return kept, rejected


@pytest.fixture(scope="module")
def disk4k():
    D = nodesets.disk(4000, 150, 1)
    idx, rho2 = oracle.knn(D["x"], 31)
    return D, idx, rho2


@pytest.fixture(scope="module")
def ball3k():
    x = nodesets.ball(3000, 2)["x"]
    idx, rho2 = oracle.knn(x, 50)
    return x, idx, rho2


# (delta, tau, least number of rejections the case must exercise); at
# tau = 5 these sets reject nothing, so those cases pin the kept side only
CASES = [(0.3, 1.0, 1000), (0.3, 2.0, 1), (0.0, 1.0, 1000), (0.0, 2.0, 100),
         (0.3, 5.0, 0)]


@pytest.mark.parametrize("delta,tau,min_rej", CASES)
def test_disk_every_decision(disk4k, delta, tau, min_rej):
    D, idx, rho2 = disk4k
    el = D["eligible"]
    r = oracle.overlapped_rows(D["x"], idx, rho2, 5, 4, delta, tau, el)
    kept, rej = _replay(D["x"], idx, rho2, el, delta, tau, r["owner"],
                        r["centers"], 5, 4)
    assert kept > 0
    assert rej >= min_rej


@pytest.mark.parametrize("delta,tau,min_rej", CASES)
def test_ball_every_decision(ball3k, delta, tau, min_rej):
    x, idx, rho2 = ball3k
    r = oracle.overlapped_rows(x, idx, rho2, 5, 3, delta, tau, None)
    kept, rej = _replay(x, idx, rho2, None, delta, tau, r["owner"],
                        r["centers"], 5, 3)
    assert kept > 0
    assert rej >= min_rej


def _golden():
    with open(os.path.join(GOLDEN, "lebesgue_rational_case.json")) as f:
        return json.load(f)


def test_rational_case_is_its_derivation():
    """The stored kept/rejected sets are what the exact derivation gives."""
    sys.path.insert(0, GOLDEN)
    try:
        import make_lebesgue_rational as mk
    finally:
        sys.path.remove(GOLDEN)
    g = _golden()
    pts = [tuple(p) for p in g["nodes"]]
    res = mk.derive(pts, Fraction(*g["tau"]))
    assert res["owner"] == g["owner"]
    assert res["centers"] == g["centers"]
    assert sum(len(c["rejected"]) for c in g["centers"]) > 0


def test_oracle_matches_rational_case():
    g = _golden()
    x = np.array(g["nodes"], np.float64) / g["denominator"]
    n = g["n"]
    idx, rho2 = oracle.knn(x, n, "brute")
    tau = g["tau"][0] / g["tau"][1]
    r = oracle.overlapped_rows(x, idx, rho2, g["m"], g["l"], g["delta"], tau)
    assert r["owner"].tolist() == g["owner"]
    assert r["centers"].tolist() == [c["center"] for c in g["centers"]]
    # decisions are far from the threshold, so FP64 rounding cannot flip one
    assert r["min_margin"] > 1e-3


def _replay_prefix(x, idx, rho2, eligible, delta, tau, owner, centers, m, l):
    """Radial prefix: with q* the first eligible ball node (claimed or not,
    center excluded) failing the test, c keeps exactly its unclaimed ball
    nodes before q*.  Returns the number of centers whose ball was cut."""
    t = 1.0 - delta
    t2 = t * t
    cuts = 0
    for c in centers:
        st = idx[c]
        thr = t2 * rho2[c]
        ball = [q for q, j in enumerate(st)
                if (eligible is None or eligible[j])
                and _sqd(x[c], x[j]) <= thr]
        assert ball[0] == 0
        ref = _reference(x[st])
        W = oracle.stencil_weights(x[st], x[st[[ref] + ball]], m, l)
        lam = np.abs(W).sum(1)
        lref = lam[0]
        qstar = len(st)
        for i, q in enumerate(ball[1:], start=2):
            if not lam[i] <= tau * lref:
                qstar = q
                break
        cuts += qstar < len(st)
        want = {st[q] for q in ball if q < qstar and owner[st[q]] >= c}
        got = set(np.nonzero(owner == c)[0].tolist())
        assert got == want, (c, sorted(got ^ want))
    return cuts


@pytest.mark.parametrize("delta,tau", [(0.0, 1.0), (0.0, 2.0), (0.3, 1.0)])
def test_radial_prefix_disk(disk4k, delta, tau):
    D, idx, rho2 = disk4k
    el = D["eligible"]
    r = oracle.overlapped_rows(D["x"], idx, rho2, 5, 4, delta, tau, el,
                               prefix=True)
    assert (r["owner"][el == 1] >= 0).all()
    cuts = _replay_prefix(D["x"], idx, rho2, el, delta, tau, r["owner"],
                          r["centers"], 5, 4)
    assert cuts > 0
    # the same threshold node by node keeps at least as much per stencil,
    # so it never needs more stencils
    nw = oracle.overlapped_rows(D["x"], idx, rho2, 5, 4, delta, tau, el)
    assert len(r["centers"]) >= len(nw["centers"])


@pytest.mark.parametrize("delta,tau", [(0.0, 1.0), (0.3, 2.0)])
def test_radial_prefix_ball(ball3k, delta, tau):
    x, idx, rho2 = ball3k
    r = oracle.overlapped_rows(x, idx, rho2, 5, 3, delta, tau, None,
                               prefix=True)
    cuts = _replay_prefix(x, idx, rho2, None, delta, tau, r["owner"],
                          r["centers"], 5, 3)
    assert cuts > 0


def test_radial_prefix_without_threshold_is_plain_covering(disk4k):
    """tau = infinity cuts nothing: the prefix mode is then the plain greedy
    covering (Sec. 4.1)."""
    D, idx, rho2 = disk4k
    el = D["eligible"]
    a = oracle.overlapped_rows(D["x"], idx, rho2, 5, 4, 0.3, np.inf, el,
                               prefix=True)
    own, cen = oracle.cover(D["x"], idx, rho2, 0.3, el)
    assert np.array_equal(a["owner"], own)
    assert np.array_equal(a["centers"], cen)
