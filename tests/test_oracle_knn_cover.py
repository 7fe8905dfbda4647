"""Pins of the oracle's stencils (kNN) and greedy covering.

kNN (Sec. 2 / Sec. 4.1: a stencil is the node and its n-1 nearest
neighbours, the node first) is pinned against a numpy brute force over the
full distance matrix and against itself across two search structures.  The
covering (Sec. 4.1: retention ball of radius (1-delta) rho_k, a row computed
once is never recomputed) is pinned by its invariants and by an independent
characterisation evaluated from the edge list rather than by a sequential
loop: node j is a center iff no earlier center's ball contains j, and its
owner is the smallest such center.
"""
import numpy as np
import pytest

import nodesets
import oracle


def numpy_knn(x, n):
    """Full distance matrix in numpy, same rounding order ((dx*dx)+(dy*dy))
    +(dz*dz), sorted by (d2, index)."""
    N, d = x.shape
    dif = x[:, None, :] - x[None, :, :]
    d2 = dif[..., 0] * dif[..., 0] + dif[..., 1] * dif[..., 1]
    if d == 3:
        d2 = d2 + dif[..., 2] * dif[..., 2]
    idx = np.empty((N, n), np.int32)
    rho2 = np.empty(N)
    cols = np.arange(N)
    for i in range(N):
        o = np.lexsort((cols, d2[i]))[:n]
        idx[i] = o
        rho2[i] = d2[i, o[-1]]
    return idx, rho2


@pytest.mark.parametrize("d,n", [(2, 1), (2, 7), (2, 31), (3, 10), (3, 50)])
def test_knn_matches_numpy_bruteforce(d, n):
    x = np.random.default_rng(100 + d + n).random((400, d))
    got, r = oracle.knn(x, n, "brute")
    ref, rr = numpy_knn(x, n)
    assert np.array_equal(got, ref)
    assert np.array_equal(r, rr)
    assert np.array_equal(got[:, 0], np.arange(len(x)))  # I^k_1 = k


def test_knn_ties_broken_by_index():
    # exact lattice: many equal distances; the order must follow the index
    g = 12
    j, i = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    x = np.stack([i.ravel() * 0.125, j.ravel() * 0.125], 1).astype(float)
    got, _ = oracle.knn(x, 9, "brute")
    ref, _ = numpy_knn(x, 9)
    assert np.array_equal(got, ref)
    c = 5 * g + 5  # interior node: the 4 axis neighbours in index order
    assert list(got[c, 1:5]) == sorted([c - g, c - 1, c + 1, c + g])


@pytest.mark.parametrize("case", ["square", "disk", "ball"])
def test_knn_grid_equals_brute(case):
    if case == "square":
        x, n = nodesets.square(45, 0), 12
    elif case == "disk":
        x, n = nodesets.disk(3000, 120, 1)["x"], 31
    else:
        x, n = nodesets.ball(6000, 2)["x"], 50
    a, ra = oracle.knn(x, n, "brute")
    b, rb = oracle.knn(x, n, "grid")
    assert np.array_equal(a, b) and np.array_equal(ra, rb)
    for q in (0, len(x) // 2, len(x) - 1):
        k1, r1 = oracle.knn_one(x, n, q)
        assert np.array_equal(k1, a[q]) and r1 == ra[q]


def test_knn_errors():
    x = np.random.default_rng(0).random((50, 2))
    with pytest.raises(oracle.OracleError) as e:
        oracle.knn(x, 51)
    assert e.value.code == oracle.EINVAL
    y = x.copy()
    y[7] = y[3]
    with pytest.raises(oracle.OracleError) as e:
        oracle.knn(y, 5)
    assert e.value.code == oracle.EDUPLICATE
    y = x.copy()
    y[2, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.knn(y, 5)
    assert e.value.code == oracle.EINVAL


def _sqdist(x, i, j):
    dif = x[j] - x[i][None, :] if np.ndim(j) else x[j] - x[i]
    dif = np.atleast_2d(dif)
    s = dif[:, 0] * dif[:, 0] + dif[:, 1] * dif[:, 1]
    if x.shape[1] == 3:
        s = s + dif[:, 2] * dif[:, 2]
    return s


def characterise(x, idx, rho2, delta, eligible):
    """Centers and owners from the edge list c -> j (j in ball(c), j > c),
    processed by increasing edge source with vectorised numpy."""
    N, n = idx.shape
    el = np.ones(N, bool) if eligible is None else eligible.astype(bool)
    t = 1.0 - delta
    thr = (t * t) * rho2
    src = np.repeat(np.arange(N), n)
    dst = idx.ravel()
    dif = x[dst] - x[src]
    d2 = dif[:, 0] * dif[:, 0] + dif[:, 1] * dif[:, 1]
    if x.shape[1] == 3:
        d2 = d2 + dif[:, 2] * dif[:, 2]
    keep = (d2 <= thr[src]) & (dst > src) & el[src] & el[dst]
    src, dst = src[keep], dst[keep]
    # predecessors of each node, sorted
    order = np.lexsort((src, dst))
    src, dst = src[order], dst[order]
    ptr = np.searchsorted(dst, np.arange(N + 1))
    is_center = np.zeros(N, bool)
    owner = np.full(N, -1)
    for j in range(N):  # predecessors always have smaller index
        if not el[j]:
            continue
        preds = src[ptr[j]:ptr[j + 1]]
        cp = preds[is_center[preds]]
        if len(cp) == 0:
            is_center[j] = True
            owner[j] = j
        else:
            owner[j] = cp.min()
    return is_center, owner


@pytest.mark.parametrize("case,delta", [("square", 0.2), ("square", 0.5),
                                        ("disk", 0.5), ("disk", 0.2),
                                        ("ball", 0.3), ("ball", 0.0)])
def test_cover_characterisation_and_invariants(case, delta):
    el = None
    if case == "square":
        x, n = nodesets.square(45, 0), 12
    elif case == "disk":
        D = nodesets.disk(3000, 120, 1)
        x, n, el = D["x"], 31, D["eligible"]
    else:
        x, n = nodesets.ball(4000, 2)["x"], 50
    idx, rho2 = oracle.knn(x, n)
    owner, centers = oracle.cover(x, idx, rho2, delta, el)
    is_c, own2 = characterise(x, idx, rho2, delta, el)
    assert np.array_equal(np.nonzero(is_c)[0], centers)
    assert np.array_equal(own2, owner)
    N = len(x)
    elb = np.ones(N, bool) if el is None else el.astype(bool)
    # (i) every eligible node has exactly one owner, ineligible ones none
    assert (owner[elb] >= 0).all() and (owner[~elb] == -1).all()
    # (ii) the owner's stencil contains the node, inside its closed ball
    t = 1.0 - delta
    for j in np.nonzero(elb)[0][::7]:
        c = owner[j]
        assert j in idx[c]
        assert _sqdist(x, c, j)[0] <= (t * t) * rho2[c]
    # (iii) owner(j) <= j; (iv) centers own themselves
    assert (owner[elb] <= np.nonzero(elb)[0]).all()
    assert np.array_equal(owner[centers], centers)
    assert len(centers) < elb.sum() or delta == 1.0  # N_delta < N (Sec. 4.1)


def test_cover_delta_one_is_standard_rbffd():
    x = nodesets.square(45, 0)
    idx, rho2 = oracle.knn(x, 12)
    owner, centers = oracle.cover(x, idx, rho2, 1.0)
    assert np.array_equal(owner, np.arange(len(x)))
    assert np.array_equal(centers, np.arange(len(x)))


def test_cover_delta_zero_keeps_whole_stencil():
    x = nodesets.ball(3000, 2)["x"]
    idx, rho2 = oracle.knn(x, 20)
    owner, centers = oracle.cover(x, idx, rho2, 0.0)
    # replay: each center claims every still-unclaimed node of its stencil
    seen = np.full(len(x), -1)
    for c in centers:
        for j in idx[c]:
            if seen[j] < 0:
                seen[j] = c
    assert np.array_equal(seen, owner)


def test_cover_rejects_bad_delta():
    x = nodesets.square(10, 0)
    idx, rho2 = oracle.knn(x, 12)
    for bad in (-0.1, 1.5, np.nan):
        with pytest.raises(oracle.OracleError):
            oracle.cover(x, idx, rho2, bad)
