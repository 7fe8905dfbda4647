"""Spectrum of a small DM (Sec. 4.2.1, Sec. 6.2): the eigenvalues of the
discrete operator restricted to the rows and columns of given nodes (for a
Laplacian with Dirichlet data, the interior block L_ii, whose spectrum
decides the stability of implicit and explicit time stepping).

A host-side diagnostic of a DM already built on the device: the CSR is
copied to the host and the eigenvalues come from a dense eigensolver, so it
is meant for DMs of a few thousand rows, as in the paper's figures.
"""
import numpy as np


def dense_block(row_ptr, col, val, nodes=None):
    """L[nodes][:, nodes] as a dense host array from a CSR (host or device
    tensors / arrays); ``nodes`` None means every row."""
    rp = np.asarray(row_ptr.cpu() if hasattr(row_ptr, "cpu") else row_ptr)
    cl = np.asarray(col.cpu() if hasattr(col, "cpu") else col)
    vl = np.asarray(val.cpu() if hasattr(val, "cpu") else val)
    N = len(rp) - 1
    nodes = np.arange(N) if nodes is None else np.asarray(
        nodes.cpu() if hasattr(nodes, "cpu") else nodes)
    pos = np.full(N, -1, np.int64)
    pos[nodes] = np.arange(len(nodes))
    B = np.zeros((len(nodes), len(nodes)))
    for a, k in enumerate(nodes):
        s0, s1 = int(rp[k]), int(rp[k + 1])
        c = pos[cl[s0:s1]]
        keep = c >= 0
        B[a, c[keep]] = vl[s0:s1][keep]
    return B


def spectrum(row_ptr, col, val, nodes=None):
    """Eigenvalues of L[nodes][:, nodes] and a summary: (eigenvalues,
    dict(max_real, min_real, n_positive_real, max_abs_imag))."""
    ev = np.linalg.eigvals(dense_block(row_ptr, col, val, nodes))
    return ev, dict(max_real=float(ev.real.max()),
                    min_real=float(ev.real.min()),
                    n_positive_real=int((ev.real > 0).sum()),
                    max_abs_imag=float(np.abs(ev.imag).max()))
