"""The allocation-free CSR entry point (orbf_assemble_csr_noalloc), through
the C ABI: its output equals orbf_assemble_csr's bit for bit on two calls in
a row, the second with a smaller input (the shared scratch array keeps the
first call's contents); it allocates no device memory; and it rejects a size
beyond its fixed scratch with EBUDGET before launching anything."""
import ctypes
import sys

import numpy as np
import pytest

import nodesets

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _outputs(N, n):
    return (torch.empty(N + 1, dtype=torch.int64, device="cuda:0"),
            torch.empty(N * n, dtype=torch.int32, device="cuda:0"),
            torch.empty(N * n, dtype=torch.float64, device="cuda:0"))


def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


def test_noalloc_csr_equals_allocating_csr(orbf):
    ctx = orbf.Context(0)
    cases = [(nodesets.ball(1_000_000, 2)["x"], 50, 5, 3, 0.3),
             (nodesets.disk(20000, 300, 1)["x"], 31, 5, 4, 0.5)]
    for call, (x, n, m, l, delta) in enumerate(cases):
        N = len(x)
        _say(f"[gpu] no-alloc CSR call {call}: N={N} n={n}")
        r = orbf.build_dm(gpu(x), n, m, l, delta, ctx=ctx)
        rp, col, val = _outputs(N, n)
        # poison the outputs so that stale values cannot pass
        rp.fill_(-7)
        col.fill_(-7)
        val.fill_(float("nan"))
        free0 = _free_bytes()
        orbf.assemble_csr_noalloc(ctx, r["knn"], r["owner"], r["W"], rp,
                                  col, val)
        ctx.sync()
        free1 = _free_bytes()
        assert free1 == free0, (free0, free1)  # nothing allocated
        assert torch.equal(rp, r["row_ptr"])
        assert torch.equal(col, r["col"])
        assert torch.equal(val.view(torch.int64), r["val"].view(torch.int64))


def test_noalloc_csr_rejects_oversize(orbf):
    ctx = orbf.Context(0)
    x = gpu(nodesets.ball(2000, 5)["x"])
    r = orbf.build_dm(x, 20, 3, 2, 0.5, ctx=ctx)
    rp, col, val = _outputs(2000, 20)
    L = orbf.lib()
    # 2e6 x 50 bytes of ranks alone exceed the 64 MiB array: refused on the
    # host before anything is launched (the small buffers are never read)
    rc = L.orbf_assemble_csr_noalloc(
        ctx._h, 2_000_000, 50, ctypes.c_void_p(r["knn"].data_ptr()),
        ctypes.c_void_p(r["owner"].data_ptr()),
        ctypes.c_void_p(r["W"].data_ptr()), ctypes.c_void_p(rp.data_ptr()),
        ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(val.data_ptr()))
    assert rc == orbf.EBUDGET
    assert b"64 MiB" in L.orbf_last_error(ctx._h)
    ctx.sync()
    # the context still works, and the next call is right
    orbf.assemble_csr_noalloc(ctx, r["knn"], r["owner"], r["W"], rp, col, val)
    ctx.sync()
    assert torch.equal(rp, r["row_ptr"])
    assert torch.equal(col, r["col"])
