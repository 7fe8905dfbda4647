"""Seeded synthetic node sets (inputs only; none of the RBF-FD arithmetic).

These stand in for the paper's node sets (Distmesh disk nodes, Gmsh ball
nodes), which are not available.  Every generator is deterministic given its
seed; the index order it returns is part of the input, because the greedy
covering visits nodes in ascending index (Sec. 4.1).

Workloads:
  square(g=45, seed=0)          jittered g x g cell-centred grid on [0,1]^2
  disk(n_int, n_bnd, seed=1)    Poisson-disk interior + equispaced boundary
  ball(N, seed=2)               scrambled Halton interior + Fibonacci shell
  batch_specs(seed=4)           512 mixed node-set descriptions
  request_specs(...)            Poisson arrival stream of build requests

Both the oracle side and the HIP side consume these arrays; random numbers
are drawn from numpy's PCG64 with the stated seed.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "_bridson.so")
_lib = None


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", _SO,
           os.path.join(HERE, "_bridson.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _SO


def _bridson():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
        _lib.bridson_disk.argtypes = [ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p]
        _lib.bridson_disk.restype = ctypes.c_int
    return _lib


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# 2D unit square: jittered Cartesian grid
# ---------------------------------------------------------------------------
def square(g=45, seed=0):
    """g*g nodes at ((i+1/2)h, (j+1/2)h), h = 1/g, index g*j + i, each
    coordinate jittered by U(-h/4, h/4)."""
    h = 1.0 / g
    j, i = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    base = np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h], axis=1)
    jit = _rng(seed).uniform(-0.25 * h, 0.25 * h, size=base.shape)
    return np.ascontiguousarray(base + jit)


# ---------------------------------------------------------------------------
# 2D unit disk: Poisson-disk interior, equispaced boundary
# ---------------------------------------------------------------------------
def _poisson_disk(R0, r, seed, ntries=30):
    # the stream is long enough for any set this module asks for
    area = math.pi * R0 * R0
    est = int(1.2 * area / (r * r)) + 100
    u = _rng(seed).random(size=est * (2 * ntries + 4) + 1000)
    cap = 2 * est + 1000
    out = np.empty((cap, 2), np.float64)
    cnt = ctypes.c_int64()
    rc = _bridson().bridson_disk(R0, r, ntries, u.ctypes.data, len(u),
                                 out.ctypes.data, cap, ctypes.byref(cnt))
    if rc != 0:
        raise RuntimeError("poisson-disk stream or capacity exhausted")
    return out[: cnt.value].copy()


# Poisson-disk radii (as a fraction of sqrt(area / n_int)) that give at least
# n_int interior points for the sizes used here; found once and checked at
# run time.
_PD_FRACTION = 0.78


def disk(n_int=99400, n_bnd=600, seed=1, order="shuffled", refine=False):
    """Unit disk: ``n_int`` interior Poisson-disk nodes (Bridson, 30 tries,
    PCG64(seed)) inside |x| <= 1 - h_b/2 with h_b = 2*pi/n_bnd, followed by
    ``n_bnd`` boundary nodes (cos 2*pi*b/n_bnd, sin 2*pi*b/n_bnd).

    ``refine``: boundary refinement (Sec. 6, the node sets of Sec. 7): the
    Poisson-disk interior stops at |x| <= 1 - h_b, and a copy of every
    boundary node moved h_b/2 along the inward normal is appended to the
    interior (eligible), so the interior then holds n_int + n_bnd nodes.

    A Poisson-disk run gives slightly more than n_int points; the surplus is
    removed at random (same stream family, seed+1000) so that no region is
    left empty.  ``order``: 'shuffled' (interior indices randomly permuted,
    PCG64(seed+2000)) or 'generation' (Bridson order).

    Returns dict(x, n_int, n_bnd, eligible (uint8: interior), boundary
    (indices), normals (exact outward unit normals of the boundary nodes))."""
    h_b = 2.0 * math.pi / n_bnd
    R0 = 1.0 - (1.0 if refine else 0.5) * h_b
    area = math.pi * R0 * R0
    frac = _PD_FRACTION
    for _ in range(8):
        pts = _poisson_disk(R0, frac * math.sqrt(area / n_int), seed)
        if len(pts) >= n_int:
            break
        frac *= 0.98
    else:
        raise RuntimeError("poisson-disk radius too large")
    if len(pts) > n_int:
        drop = _rng(seed + 1000).choice(len(pts), size=len(pts) - n_int,
                                        replace=False)
        keep = np.ones(len(pts), bool)
        keep[drop] = False
        pts = pts[keep]
    if order == "shuffled":
        pts = pts[_rng(seed + 2000).permutation(n_int)]
    elif order != "generation":
        raise ValueError(order)
    th = 2.0 * math.pi * np.arange(n_bnd) / n_bnd
    bnd = np.stack([np.cos(th), np.sin(th)], axis=1)
    if refine:
        pts = np.concatenate([pts, (1.0 - 0.5 * h_b) * bnd], axis=0)
    ni = len(pts)
    x = np.ascontiguousarray(np.concatenate([pts, bnd], axis=0))
    eligible = np.zeros(ni + n_bnd, np.uint8)
    eligible[:ni] = 1
    return dict(x=x, n_int=ni, n_bnd=n_bnd, eligible=eligible,
                boundary=np.arange(ni, ni + n_bnd, dtype=np.int32),
                normals=np.ascontiguousarray(bnd))


# ---------------------------------------------------------------------------
# 3D unit ball: scrambled Halton interior + Fibonacci-sphere shell
# ---------------------------------------------------------------------------
def _radical_inverse(idx, base):
    idx = idx.astype(np.int64).copy()
    out = np.zeros(idx.shape, np.float64)
    f = 1.0 / base
    while np.any(idx > 0):
        out += f * (idx % base)
        idx //= base
        f /= base
    return out


def halton(count, start=1, bases=(2, 3, 5)):
    idx = np.arange(start, start + count, dtype=np.int64)
    return np.stack([_radical_inverse(idx, b) for b in bases], axis=1)


def fibonacci_sphere(nb):
    i = np.arange(nb, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / nb
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * (math.pi * (3.0 - math.sqrt(5.0)))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def ball(N=1_000_000, seed=2):
    """Unit ball with N nodes: h = (4*pi/(3N))^(1/3); the shell has
    N_b = round(4*pi/h^2) Fibonacci-sphere nodes (indices N-N_b..N-1); the
    interior is the Halton sequence (bases 2,3,5) with a Cranley-Patterson
    shift u ~ PCG64(seed), mapped to [-1,1]^3 and kept where
    |x| <= 1 - h/2, in sequence order.  All nodes are eligible."""
    h = (4.0 * math.pi / (3.0 * N)) ** (1.0 / 3.0)
    nb = int(round(4.0 * math.pi / (h * h)))
    nb = min(nb, N // 2)
    ni = N - nb
    shift = _rng(seed).random(3)
    lim2 = (1.0 - 0.5 * h) ** 2
    chunks, got, start = [], 0, 1
    while got < ni:
        c = int((ni - got) * 2.0) + 1024
        p = 2.0 * np.mod(halton(c, start) + shift, 1.0) - 1.0
        start += c
        p = p[np.einsum("ij,ij->i", p, p) <= lim2]
        chunks.append(p)
        got += len(p)
    interior = np.concatenate(chunks, axis=0)[:ni]
    x = np.ascontiguousarray(np.concatenate([interior, fibonacci_sphere(nb)],
                                            axis=0))
    return dict(x=x, n_int=ni, n_bnd=nb, h=h)


# ---------------------------------------------------------------------------
# batched and served workloads (descriptions; node sets made on demand)
# ---------------------------------------------------------------------------
def phs_exponent(l):
    """PHS exponent used where the workload does not fix one: r^3 for
    degree 2, r^5 for degree 3 and 4."""
    return 3 if l == 2 else 5


def n_monomials(d, l):
    return math.comb(l + d, d)


def make_set(spec):
    """Node set of a batch/request description (2D: jittered square grid with
    g = round(sqrt(N)); 3D: ball generator)."""
    if spec["d"] == 2:
        g = max(4, int(round(math.sqrt(spec["N"]))))
        return square(g, spec["seed"])
    return ball(spec["N"], spec["seed"])["x"]


def batch_specs(nsets=512, seed=4):
    """512 node-set descriptions: N log-uniform in [1e3, 2e5], d in {2,3},
    l in {2,3,4}, n uniform integer in [2M+1, 3M], delta in {0.2,0.5,1.0},
    m = 3 (l = 2) or 5, Laplacian."""
    rng = _rng(seed)
    out = []
    for s in range(nsets):
        N = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        d = int(rng.integers(2, 4))
        l = int(rng.integers(2, 5))
        M = n_monomials(d, l)
        n = int(rng.integers(2 * M + 1, 3 * M + 1))
        delta = float(rng.choice([0.2, 0.5, 1.0]))
        if d == 2:
            N = max(4, int(round(math.sqrt(N)))) ** 2
        out.append(dict(N=N, d=d, l=l, M=M, n=n, delta=delta,
                        m=phs_exponent(l), seed=10_000 + s))
    return out


def request_specs(count, rate_hz, seed=5, median_n=2e4, sigma=1.0):
    """Poisson arrival stream of DM-build requests: exponential gaps at
    ``rate_hz``; N lognormal (median 2e4, sigma 1.0) clipped to [5e3, 5e5];
    d in {2,3}; l in {2,3,4}; delta ~ U[0.2, 1]; n = 2M + 1."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate_hz)
        N = int(min(5e5, max(5e3, math.exp(rng.normal(math.log(median_n),
                                                        sigma)))))
        d = int(rng.integers(2, 4))
        l = int(rng.integers(2, 5))
        M = n_monomials(d, l)
        delta = float(rng.uniform(0.2, 1.0))
        if d == 2:
            N = max(4, int(round(math.sqrt(N)))) ** 2
        out.append(dict(t=t, N=N, d=d, l=l, M=M, n=2 * M + 1, delta=delta,
                        m=phs_exponent(l), seed=20_000 + r))
    return out
