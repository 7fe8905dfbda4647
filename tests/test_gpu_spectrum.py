"""Spectra of small DMs built on the device, with and without the local
L-Lebesgue stabilization (Sec. 6.2, eq. calLstab): a 1,046-node disk with
n = 30, delta = 0.2.  The device's DMs have the oracle's structure bit for
bit and weights within 1e-9, so their interior blocks have the oracle's
spectrum: spurious eigenvalues with positive real part without
stabilization, none with tau = 1, whose rightmost eigenvalue approximates
-j_{0,1}^2, the first Dirichlet eigenvalue of the unit disk's Laplacian."""
import sys

import numpy as np
import pytest

import nodesets
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

J01 = 2.404825557695773


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def orbf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_03135_amd as P
    P.lib()
    return P


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("seed", [1, 2])
def test_spectrum_with_and_without_stabilization(orbf, seed):
    from paper_1606_03135_amd import spectrum as spec
    ctx = orbf.Context(0)
    D = nodesets.disk(946, 100, seed)
    x, el = D["x"], D["eligible"]
    inner = np.nonzero(el)[0]
    res = {}
    for tau in (np.inf, 1.0):
        got = orbf.build_dm(gpu(x), 30, 5, 4, 0.2, tau=tau, eligible=gpu(el),
                            ctx=ctx)
        ref = oracle.build_dm(x, 30, 5, 4, 0.2, tau=tau, eligible=el)
        assert np.array_equal(got["owner"].cpu().numpy(), ref["owner"])
        evg, sg = spec.spectrum(got["row_ptr"], got["col"], got["val"], inner)
        evr, sr = spec.spectrum(ref["row_ptr"], ref["col"], ref["val"], inner)
        nc = int(got["n_centers"].item())
        _say(f"[gpu] spectrum seed {seed} tau {tau}: N_delta={nc} "
             f"max Re {sg['max_real']:.6g} (oracle {sr['max_real']:.6g}), "
             f"{sg['n_positive_real']} with Re > 0")
        scale = np.abs(evr).max()
        assert abs(sg["max_real"] - sr["max_real"]) <= 1e-7 * scale
        assert sg["n_positive_real"] == sr["n_positive_real"]
        res[tau] = (nc, sg)
    assert res[np.inf][1]["n_positive_real"] > 0
    assert res[1.0][1]["n_positive_real"] == 0
    assert res[1.0][0] > res[np.inf][0]
    lam1 = J01 ** 2
    assert abs(res[1.0][1]["max_real"] + lam1) / lam1 < 1e-4
