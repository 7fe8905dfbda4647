"""Exact derivation of a small finite-tau covering (Sec. 4.1 greedy loop with
the local L-Lebesgue test of Sec. 4.2.1, eq. calLstab), written to
lebesgue_rational_case.json.

The case is chosen so that everything can be done by hand, in exact rational
arithmetic, without the oracle:
  - 2D, polynomial degree l = 3 (M = 10 monomials) and stencils of n = M = 10
    nodes.  With a square, invertible Psi the constraint block row of eq.
    rbffd_linsys, Psi^T w = L psi(x_e), fixes the weights alone, so the PHS
    part drops out and the weights are polynomial finite-difference weights;
  - node coordinates are multiples of 1/64, so squared distances (and with
    them the stencils and the delta = 0 retention ball) are exact in FP64 as
    well as in rationals;
  - the Laplacian of a cubic is linear, so the weights of different
    evaluation points differ and some of them fail the threshold.

The ratio Lambda_e / Lambda_ref is invariant under translation and scaling,
so the derivation works in physical offsets x_j - x_k.  Rules (the readings
of the paper this repository takes): nodes are visited in ascending index;
a node that no earlier center kept becomes a center; its candidates are
its unclaimed stencil nodes; the reference is the stencil node nearest the
stencil centroid (lowest stencil position on ties); node e is kept iff it is
the center or Lambda_e <= tau * Lambda_ref.

Run from the repository root:  python tests/golden/make_lebesgue_rational.py
It uses only numpy's seeded generator (for the node positions) and Python's
fractions; it imports neither the oracle nor the HIP library.
"""
import json
import os
import sys
from fractions import Fraction as F

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "lebesgue_rational_case.json")

G = 6          # 6 x 6 lattice
DEN = 64       # coordinates are integers / 64
N_STENCIL = 10
EXPONENTS = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2),
             (3, 0), (2, 1), (1, 2), (0, 3)]  # graded lex, degree <= 3


def nodes(seed):
    """Integer numerators (over DEN) of a jittered G x G lattice, spacing
    8/64, jitter uniform in {-2..2}/64 per coordinate, index = G*j + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = []
    for j in range(G):
        for i in range(G):
            jx, jy = rng.integers(-2, 3, size=2)
            pts.append((8 * i + 8 + int(jx), 8 * j + 8 + int(jy)))
    return pts


def sqd(a, b):
    return (a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2


def knn(pts):
    out = []
    for k, p in enumerate(pts):
        order = sorted(range(len(pts)), key=lambda j: (sqd(p, pts[j]), j))
        out.append(order[:N_STENCIL])
    return out


def lap_monomial(e, x, y):
    """Laplacian of x^a y^b at (x, y)."""
    a, b = e
    s = F(0)
    if a >= 2:
        s += a * (a - 1) * x ** (a - 2) * y ** b
    if b >= 2:
        s += b * (b - 1) * x ** a * y ** (b - 2)
    return s


def solve(A, rhs):
    """Gaussian elimination in exact rationals (any nonzero pivot)."""
    n = len(A)
    M = [list(row) + [r] for row, r in zip(A, rhs)]
    for k in range(n):
        p = next(i for i in range(k, n) if M[i][k] != 0)
        M[k], M[p] = M[p], M[k]
        for i in range(n):
            if i != k and M[i][k] != 0:
                f = M[i][k] / M[k][k]
                M[i] = [a - f * b for a, b in zip(M[i], M[k])]
    return [M[i][n] / M[i][i] for i in range(n)]


def lebesgue(pts, st, q_eval):
    """Lambda = sum_j |w_j| of the Laplacian weights at stencil node
    q_eval (positions in st), physical offsets from the center."""
    c = pts[st[0]]
    off = [(F(pts[j][0] - c[0], DEN), F(pts[j][1] - c[1], DEN)) for j in st]
    # Psi^T w = L psi(x_e): row t of Psi^T is monomial t at every node
    PsiT = [[x ** a * y ** b for (x, y) in off] for (a, b) in EXPONENTS]
    xe, ye = off[q_eval]
    rhs = [lap_monomial(e, xe, ye) for e in EXPONENTS]
    w = solve(PsiT, rhs)
    return sum(abs(v) for v in w)


def reference(pts, st):
    c = pts[st[0]]
    off = [(pts[j][0] - c[0], pts[j][1] - c[1]) for j in st]
    n = len(st)
    cx = F(sum(o[0] for o in off), n)
    cy = F(sum(o[1] for o in off), n)
    d = [(o[0] - cx) ** 2 + (o[1] - cy) ** 2 for o in off]
    best = min(d)
    return d.index(best), d


def derive(pts, tau):
    idx = knn(pts)
    N = len(pts)
    owner = [-1] * N
    centers = []
    margin = None
    for k in range(N):
        if owner[k] != -1:
            continue
        st = idx[k]
        ref, _ = reference(pts, st)
        lref = lebesgue(pts, st, ref)
        kept, rejected = [], []
        for q, j in enumerate(st):
            if owner[j] != -1:
                continue
            if q == 0:
                kept.append(j)
                owner[j] = k
                continue
            le = lebesgue(pts, st, q)
            if q != ref:
                mg = abs(le - tau * lref) / (tau * lref)
                margin = mg if margin is None else min(margin, mg)
            if le <= tau * lref:
                kept.append(j)
                owner[j] = k
            else:
                rejected.append(j)
        centers.append(dict(center=k, ref_position=ref, kept=kept,
                            rejected=rejected))
    return dict(owner=owner, centers=centers, min_margin=margin)


SEED = 0
TAU = F(3, 2)


def main():
    pts = nodes(SEED)
    res = derive(pts, TAU)
    doc = {
        "source": "Exact rational derivation (make_lebesgue_rational.py): "
                  "greedy covering of Sec. 4.1 with the L-Lebesgue ratio "
                  "test of Sec. 4.2.1 on polynomial-FD stencils (n = M), "
                  "delta = 0, tau = 3/2; nodes are integers / 64",
        "d": 2, "m": 3, "l": 3, "n": N_STENCIL, "delta": 0.0,
        "tau": [TAU.numerator, TAU.denominator],
        "denominator": DEN,
        "nodes": [list(p) for p in pts],
        "owner": res["owner"],
        "centers": res["centers"],
        "min_margin": float(res["min_margin"]),
    }
    lines = ["{"]
    items = list(doc.items())
    for i, (k, v) in enumerate(items):
        sep = "," if i + 1 < len(items) else ""
        if k == "centers":
            body = ",\n  ".join(json.dumps(c) for c in v)
            lines.append(f' "{k}": [\n  {body}]{sep}')
        else:
            lines.append(f" {json.dumps(k)}: {json.dumps(v)}{sep}")
    lines.append("}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    json.load(open(OUT))  # well-formed
    kept = sum(len(c["kept"]) for c in res["centers"])
    rej = sum(len(c["rejected"]) for c in res["centers"])
    print(f"{OUT}: {len(res['centers'])} centers, {kept} kept, {rej} rejected,"
          f" min margin {float(res['min_margin']):.3g}")


if __name__ == "__main__":
    sys.exit(main())
