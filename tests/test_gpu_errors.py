"""GPU tests of the error paths: with the library's allocation hook, the k-th allocation of an
entry point is made to fail, for every k until the call needs no more. Each failure must come
back as SELL_ERR_OOM, leave no allocation behind (the library's count of live allocations
returns to where it was), and leave the library usable. No kernel is made to fault: the
failures are forced on the host, before the allocation is issued."""
import numpy as np
import pytest

import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def _drive(sc, op, kmax=80):
    """Runs op with the k-th allocation failing, k = 1, 2, ...; returns how many allocations
    the call makes (the first k at which it succeeds, minus one)."""
    import torch

    op()  # warm-up: per-stream workspaces and caches exist before the counting starts
    torch.cuda.synchronize()
    base = sc.sell_debug_live_allocs()
    for k in range(1, kmax + 1):
        sc.sell_debug_fail_alloc(k)
        failed = False
        try:
            op()
        except sc.SellError as e:
            assert e.code == sc.SELL_ERR_OOM, (k, str(e))
            failed = True
        finally:
            sc.sell_debug_fail_alloc(0)
        torch.cuda.synchronize()
        live = sc.sell_debug_live_allocs()
        assert live == base, (k, live, base)
        if not failed:
            return k - 1
    pytest.fail(f"more than {kmax} allocations")


def _mats():
    return synth.laplacian3d(9), synth.irregular(3000, band=300, max_len=200, seed=3)


def test_matrix_construction_and_drivers(sc):
    import torch

    A, R = _mats()
    n, b = A.nrows, 4
    rp, co, va = (torch.from_numpy(np.ascontiguousarray(A.rowptr)).cuda(),
                  torch.from_numpy(np.ascontiguousarray(A.col)).cuda(), torch.from_numpy(A.val).cuda())
    X = dev(synth.block_vector(n, b, 1))
    Bv = dev(synth.block_vector(n, b, 2))
    M = sc.SellMatrix.from_csr(A)
    Mlo = sc.SellMatrix.from_csr(A, dtype="bf16")

    def build_host():
        sc.SellMatrix.from_csr(R, C=32, sigma=64).close()

    def build_device():
        sc.SellMatrix.from_device_csr(n, n, rp, co, va, C=32, sigma=128).close()

    def transpose_and_update():
        Mt = sc.SellMatrix.from_csr(A)
        try:
            Y = torch.empty_like(X)
            sc.sell_spmmv_T(Mt, X, Y, deterministic=True)  # builds the copy of A^T
            Mt.update_values(va)  # builds the update maps, scatters into A^T
        finally:
            Mt.close()

    def kpm():
        V, W = X.clone(), torch.empty_like(X)
        mu = torch.zeros(21 * b, dtype=torch.float64, device="cuda:0")
        sc.sell_kpm(M, V, W, 10, 14.0, 0.0, mu)

    def cg():
        sc.sell_cg(M, Bv, torch.zeros_like(Bv), tol=1e-8, maxit=50)

    def cg_mixed():
        sc.sell_cg_mixed(M, Mlo, Bv, torch.zeros_like(Bv), tol=1e-8, maxit=50)

    def cheb_filter():
        sc.sell_cheb_filter(M, X, np.linspace(1, 0.1, 12), 14.0)

    def owned_block_vector():
        h = sc.sell_bv_create(n, b, "f64")
        sc.sell_bv_destroy(h)

    counts = {}
    for name, op in [("build_host", build_host), ("build_device", build_device),
                     ("transpose_and_update", transpose_and_update), ("kpm", kpm), ("cg", cg),
                     ("cg_mixed", cg_mixed), ("cheb_filter", cheb_filter), ("owned_block_vector", owned_block_vector)]:
        counts[name] = _drive(sc, op)
    # the constructions and the drivers that keep data on the device do allocate
    assert counts["build_host"] >= 5 and counts["build_device"] >= 5, counts
    assert counts["transpose_and_update"] >= 1 and counts["kpm"] >= 2 and counts["owned_block_vector"] == 1, counts
    M.close()
    Mlo.close()


def test_batches_and_autotuner(sc):
    import torch

    A, R = _mats()
    mats = [A, synth.laplacian3d(6), synth.laplacian3d(11)]
    b = 4
    Ms = [sc.SellMatrix.from_csr(m) for m in mats]
    Mb = [sc.SellMatrix.from_csr(m, dtype="bf16") for m in mats]
    rows = sum(m.nrows for m in mats)
    X = dev(synth.block_vector(rows, b, 5))

    def batch_product():
        Bt = sc.SellBatch(Ms)
        try:
            d = torch.zeros(3 * b * len(mats), dtype=torch.float64, device="cuda:0")
            sc.sell_batch_spmmv_aug(Bt, X, torch.empty_like(X), flags=sc.DOTS, dot=d)
            Bt.set_widths([1, 4, 2])
            nx, ny, nd = Bt.packed_sizes()
            sc.sell_batch_spmmv_aug_packed(Bt, torch.rand(nx, dtype=torch.float64, device="cuda:0"),
                                           torch.empty(ny, dtype=torch.float64, device="cuda:0"), flags=sc.DOTS,
                                           dot=torch.zeros(nd, dtype=torch.float64, device="cuda:0"))
        finally:
            Bt.close()

    def batch_cg():
        B64, Bbf = sc.SellBatch(Ms), sc.SellBatch(Mb)
        try:
            sc.sell_batch_cg(B64, Bbf, X, torch.zeros_like(X), tol=1e-8, maxit=40, graph=True)
        finally:
            B64.close()
            Bbf.close()

    def autotune():
        sc.sell_autotune(R, 2, "f64", cache=False)

    counts = {name: _drive(sc, op) for name, op in [("batch_product", batch_product), ("batch_cg", batch_cg),
                                                    ("autotune", autotune)]}
    assert all(v >= 3 for v in counts.values()), counts
    for M in Ms + Mb:
        M.close()


def test_hook_arguments(sc):
    with pytest.raises(sc.SellError):
        sc.sell_debug_fail_alloc(-1)
    sc.sell_debug_fail_alloc(0)
    assert sc.sell_debug_live_allocs() >= 0
