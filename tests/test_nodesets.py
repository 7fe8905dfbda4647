"""Seeded input generators: determinism, sizes, no coincident nodes."""
import numpy as np

import nodesets


def test_square_grid():
    a = nodesets.square(45, 0)
    assert a.shape == (2025, 2)
    assert np.array_equal(a, nodesets.square(45, 0))
    h = 1 / 45
    base_i = (np.arange(2025) % 45 + 0.5) * h
    assert np.abs(a[:, 0] - base_i).max() <= 0.25 * h


def test_disk():
    D = nodesets.disk(5000, 200, 1)
    x = D["x"]
    assert x.shape == (5200, 2) and D["eligible"].sum() == 5000
    assert np.array_equal(x, nodesets.disk(5000, 200, 1)["x"])
    r = np.linalg.norm(x, axis=1)
    assert (r[:5000] <= 1 - 0.5 * 2 * np.pi / 200 + 1e-12).all()
    assert np.allclose(r[5000:], 1.0)
    assert np.allclose(np.linalg.norm(D["normals"], axis=1), 1.0)
    assert len(np.unique(x, axis=0)) == len(x)


def test_ball():
    B = nodesets.ball(20000, 2)
    x = B["x"]
    assert x.shape == (20000, 3)
    assert np.array_equal(x, nodesets.ball(20000, 2)["x"])
    r = np.linalg.norm(x, axis=1)
    assert (r <= 1 + 1e-12).all() and np.allclose(r[-B["n_bnd"]:], 1.0)
    assert len(np.unique(x, axis=0)) == len(x)


def test_batch_and_request_specs():
    s = nodesets.batch_specs()
    assert len(s) == 512
    for t in s:
        assert 2 * t["M"] + 1 <= t["n"] <= 3 * t["M"]
        assert t["delta"] in (0.2, 0.5, 1.0)
    r = nodesets.request_specs(100, 10.0)
    assert all(5e3 - 200 <= q["N"] <= 5e5 + 2000 for q in r)
    assert all(b["t"] > a["t"] for a, b in zip(r, r[1:]))


def test_disk_refined():
    """Boundary refinement: interior within 1 - h_b, then one copy of each
    boundary node h_b/2 inside along -n (eligible), then the boundary."""
    import math
    D = nodesets.disk(3000, 150, 4, refine=True)
    x, nb = D["x"], 150
    h_b = 2 * math.pi / nb
    assert D["n_int"] == 3000 + nb and len(x) == 3000 + 2 * nb
    r = np.linalg.norm(x, axis=1)
    assert r[:3000].max() <= 1 - h_b + 1e-12
    copies, bnd = x[3000:3000 + nb], x[D["boundary"]]
    assert np.abs(r[D["boundary"]] - 1).max() < 1e-14
    assert np.abs(copies - (1 - 0.5 * h_b) * bnd).max() < 1e-15
    assert np.array_equal(D["normals"], bnd)
    assert D["eligible"][:3000 + nb].all() and not D["eligible"][3000 + nb:].any()


def test_spectrum_dense_block():
    """Host-side helper of the spectrum diagnostic: the dense block of a
    small CSR, whole and restricted to a node subset."""
    from paper_1606_03135_amd import spectrum as spec
    rp = np.array([0, 2, 3, 5])
    col = np.array([0, 2, 1, 0, 2])
    val = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    B = spec.dense_block(rp, col, val)
    assert np.array_equal(B, [[1, 0, 2], [0, 3, 0], [4, 0, 5]])
    assert np.array_equal(spec.dense_block(rp, col, val, [0, 2]),
                          [[1, 2], [4, 5]])
    # eigenvalues 3 and 3 +- sqrt(12) (the 2 x 2 block [[1, 2], [4, 5]])
    ev, s = spec.spectrum(rp, col, val)
    assert s["n_positive_real"] == 2
    assert abs(s["max_real"] - (3 + 12 ** 0.5)) < 1e-12
