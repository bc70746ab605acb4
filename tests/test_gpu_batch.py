"""GPU tests of batches: one launch of the augmented product over many matrices against the
oracle (per matrix) and against the single-matrix entry point, and batched CG (FP64 and
FP32 iterations refined in FP64) checked by the oracle's FP64 residual of the returned
solutions; with and without the HIP graph (the graph is replayed many times with eager work
and host synchronisations in between, and must give the eager result bit for bit)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import abs_product, colwise_relerr, dev, host, to_oracle_flags

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def _empty():
    return synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), "empty")


def _square_mats():
    return [synth.laplacian3d(7), _empty(), synth.anderson3d(9, seed=synth.SEED_MATRIX + 1000),
            synth.random_sparse(333, 333, 0.03, 41, empty_rows=17, long_row=333),
            synth.irregular(4000, band=300, max_len=900, seed=42), synth.laplacian2d(5)]


def _stack(parts, b):
    return np.concatenate([p.reshape(-1, b) for p in parts], axis=0) if parts else np.zeros((0, b))


def _value_ref(A, dt):
    if dt == "f64":
        return A
    rnd = oracle.round_f32 if dt == "f32" else oracle.round_bf16
    return synth.CSR(A.nrows, A.ncols, A.rowptr, A.col, rnd(A.val), A.name)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [1, 3, 8, 32])
@pytest.mark.parametrize("flags_name", ["plain", "shift_scale_axpby_dots", "vshift_chain_dots", "cg_dots"])
def test_batch_product_vs_oracle_and_single(sc, dt, b, flags_name):
    import torch

    mats = _square_mats()
    flags = {"plain": 0,
             "shift_scale_axpby_dots": sc.SHIFT | sc.SCALE | sc.AXPBY | sc.DOTS,
             "vshift_chain_dots": sc.VSHIFT | sc.SCALE | sc.AXPBY | sc.DOTS | sc.CHAIN,
             "cg_dots": sc.DOT_YY | sc.DOT_XY}[flags_name]
    kw = dict(alpha=0.5, beta=-1.25, gamma=0.1, delta=0.3, eta=-2.0,
              gamma_v=np.linspace(-1, 1, b) if flags & sc.VSHIFT else None)
    Ms = [sc.SellMatrix.from_csr(A, C=32 if k % 2 == 0 else 8, sigma=[1, 64, 7][k % 3], dtype=dt)
          for k, A in enumerate(mats)]
    Bt = sc.SellBatch(Ms)
    assert Bt.count == len(mats) and Bt.rows == sum(A.nrows for A in mats)
    vt = torch.float64 if dt == "f64" else torch.float32
    Xs = [synth.block_vector(A.ncols, b, synth.SEED_X + 1000 * k) for k, A in enumerate(mats)]
    Ys = [synth.block_vector(A.nrows, b, synth.SEED_Y + 1000 * k) for k, A in enumerate(mats)]
    Zs = [synth.block_vector(A.nrows, b, synth.SEED_Y + 7 + 1000 * k) for k, A in enumerate(mats)]
    if dt != "f64":  # the operands as the FP32 vectors hold them
        Xs, Ys, Zs = [[oracle.round_f32(v) for v in L] for L in (Xs, Ys, Zs)]
    Xd, Yd, Zd = dev(_stack(Xs, b), vt), dev(_stack(Ys, b), vt), dev(_stack(Zs, b), vt)
    dot = torch.full((3 * b * len(mats),), float("nan"), dtype=torch.float64, device="cuda:0")
    sc.sell_batch_spmmv_aug(Bt, Xd, Yd, Zd if flags & sc.CHAIN else None, flags=flags,
                            dot=dot if flags & sc.DOTS else None, **kw)
    Yg, Zg, dg = host(Yd), host(Zd), host(dot)
    if dt == "f64":
        tol = 1e-12
    else:  # FP32 accumulation over a row plus the epilogue: gamma_k with k = longest row + 3
        k = max(int(np.diff(A.rowptr).max()) for A in mats if A.nrows) + 3
        tol = k * 2.0 ** -24 / (1 - k * 2.0 ** -24)
    gmax = 1.0 if flags & sc.VSHIFT else 0.1
    r0 = 0
    for k, A in enumerate(mats):
        Ar = _value_ref(A, dt)
        ofl = to_oracle_flags(flags)
        if flags:
            Yr, Zr, dr = oracle.spmmv_aug(Ar, Xs[k], Ys[k], Zs[k], flags=ofl, **kw)
        else:
            Yr, Zr, dr = oracle.spmmv(Ar, Xs[k]), None, None
        sl = slice(r0, r0 + A.nrows)
        groups = [g for g, bit in enumerate((sc.DOT_YY, sc.DOT_XY, sc.DOT_XX)) if flags & bit]
        if A.nrows == 0:  # an empty matrix: no rows, its dots are zero
            for g in groups:
                assert np.all(dg[3 * b * k + g * b: 3 * b * k + (g + 1) * b] == 0.0)
            continue
        scale = 0.5 * (abs_product(Ar, Xs[k]) + gmax * np.abs(Xs[k])) + 1.25 * np.abs(Ys[k]) if flags else \
            abs_product(Ar, Xs[k])
        assert colwise_relerr(Yg[sl], Yr, scale) <= tol, (k, "y")
        if flags & sc.CHAIN:
            assert colwise_relerr(Zg[sl], Zr, 0.3 * np.abs(Zs[k]) + 2.0 * np.abs(Yr) + 2 * scale) <= tol, (k, "z")
        if flags & sc.DOTS:
            got = dg[3 * b * k: 3 * b * (k + 1)]
            Yq = Yg[sl]
            den = np.concatenate([np.sum(Yq * Yq + 2 * np.abs(Yq) * scale, axis=0),
                                  np.sum(np.abs(Xs[k]) * (np.abs(Yq) + scale), axis=0),
                                  np.sum(Xs[k] * Xs[k], axis=0)])
            for g in groups:
                seg = slice(g * b, (g + 1) * b)
                assert np.all(np.abs(got[seg] - dr[seg]) <= tol * den[seg] + 1e-300), (k, "dots", g)
        r0 += A.nrows
        # the single-matrix entry point computes every row the same way: identical y
        if flags & sc.CHAIN:
            continue
        Y1 = dev(Ys[k], vt)
        if flags:
            d1 = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
            sc.sell_spmmv_aug(Ms[k], dev(Xs[k], vt), Y1, flags=flags, dot=d1, **kw)
        else:
            sc.sell_spmmv(Ms[k], dev(Xs[k], vt), Y1)
        assert np.array_equal(host(Y1), Yg[sl]), k
    Bt.close()
    for M in Ms:
        M.close()


def test_batch_rejects_bad_operands(sc):
    import torch

    A = synth.laplacian2d(6)
    M64 = sc.SellMatrix.from_csr(A)
    M32 = sc.SellMatrix.from_csr(A, dtype="f32")
    with pytest.raises(sc.SellError):
        sc.SellBatch([M64, M32])  # mixed value types
    with pytest.raises(sc.SellError):
        sc.SellBatch([])
    Bt = sc.SellBatch([M64, M64])
    X = torch.zeros((2 * A.ncols, 2), dtype=torch.float64, device="cuda:0")
    Y = torch.zeros((2 * A.nrows - 1, 2), dtype=torch.float64, device="cuda:0")
    with pytest.raises(sc.SellError):
        sc.sell_batch_spmmv_aug(Bt, X, Y)  # wrong stacked size
    Y = torch.zeros((2 * A.nrows, 2), dtype=torch.float32, device="cuda:0")
    with pytest.raises(sc.SellError):
        sc.sell_batch_spmmv_aug(Bt, X, Y)  # wrong vector type
    Bt.close()
    M64.close()
    M32.close()


def test_batch_repeated_calls_reuse_and_replace_tables(sc):
    """Alternating operand sets (more than the device table slots) must each see their own
    arguments."""
    import torch

    mats = [synth.laplacian3d(5), synth.anderson3d(6), synth.laplacian2d(9)]
    Ms = [sc.SellMatrix.from_csr(A) for A in mats]
    Bt = sc.SellBatch(Ms)
    b = 4
    sets = []
    for t in range(6):
        X = _stack([synth.block_vector(A.ncols, b, 500 + 10 * t + k) for k, A in enumerate(mats)], b)
        sets.append((X, dev(X), torch.zeros((Bt.rows, b), dtype=torch.float64, device="cuda:0")))
    for rep in range(3):
        for t, (X, Xd, Yd) in enumerate(sets):
            sc.sell_batch_spmmv_aug(Bt, Xd, Yd, flags=sc.SCALE, alpha=float(t + 1))
    r0 = 0
    c0 = 0
    for k, A in enumerate(mats):
        for t, (X, Xd, Yd) in enumerate(sets):
            ref = (t + 1) * oracle.spmmv(A, X[c0:c0 + A.ncols])
            assert colwise_relerr(host(Yd)[r0:r0 + A.nrows], ref, abs_product(A, X[c0:c0 + A.ncols])) <= 1e-12
        r0 += A.nrows
        c0 += A.ncols
    Bt.close()
    for M in Ms:
        M.close()


# ------------------------------------------------------------------------- batched CG


def _cg_systems():
    edges = [3, 9, 5, 12, 7, 4]
    return [synth.laplacian3d(e) for e in edges]


def _oracle_relres(A, Bm, Xm):
    R = Bm - oracle.spmmv(A, Xm)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(Bm, axis=0)


@pytest.mark.parametrize("mode", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_cg_converges(sc, mode, graph):
    import torch

    mats = _cg_systems()
    b = 4
    M64 = [sc.SellMatrix.from_csr(A, C=32, sigma=1) for A in mats]
    B64 = sc.SellBatch(M64)
    Mlo = Blo = None
    if mode != "f64":
        Mlo = [sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=mode) for A in mats]
        Blo = sc.SellBatch(Mlo)
    Bs = [synth.block_vector(A.nrows, b, synth.SEED_Y + 1000 * k) for k, A in enumerate(mats)]
    Bd = dev(_stack(Bs, b))
    Xd = torch.zeros_like(Bd)
    tol = 1e-10
    st = sc.sell_batch_cg(B64, Blo, Bd, Xd, tol=tol, maxit=4000, graph=graph)
    X = host(Xd)
    r0 = 0
    for k, A in enumerate(mats):
        assert st[k]["converged"] == 1, (k, st[k])
        rel = _oracle_relres(A, Bs[k], X[r0:r0 + A.nrows])
        assert np.all(rel <= 1.05 * tol), (k, rel)
        assert abs(float(rel.max()) - st[k]["relres"]) <= 1e-3 * tol + 1e-2 * st[k]["relres"], k
        assert st[k]["iterations"] > 0
        if mode != "f64":
            assert st[k]["refinements"] >= 1
        r0 += A.nrows
    # smaller systems need fewer iterations (condition number grows with the edge)
    its = {A.nrows: s["iterations"] for A, s in zip(mats, st)}
    assert its[3 ** 3] < its[12 ** 3]
    for obj in [B64, Blo] + M64 + (Mlo or []):
        if obj is not None:
            obj.close()


@pytest.mark.parametrize("mode", ["f64", "f32"])
@pytest.mark.parametrize("b", [2, 8, 12, 16, 32])
def test_batch_cg_every_vector_pass_width(sc, mode, b):
    """The batched vector pass on 16-byte column groups (FP64 vectors: 1, 4, 8 and 16 groups
    per row; FP32 vectors: 2, 4 and 8) and per element (6 FP64 groups or 3 FP32 groups at
    b = 12; FP32 at b = 2, narrower than a group)."""
    import torch

    mats = _cg_systems()[:4]
    M64 = [sc.SellMatrix.from_csr(A, C=32, sigma=1) for A in mats]
    B64 = sc.SellBatch(M64)
    Mlo = [sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=mode) for A in mats] if mode != "f64" else []
    Blo = sc.SellBatch(Mlo) if Mlo else None
    Bs = [synth.block_vector(A.nrows, b, 1500 + 10 * k + b) for k, A in enumerate(mats)]
    Xd = torch.zeros((B64.rows, b), dtype=torch.float64, device="cuda:0")
    st = sc.sell_batch_cg(B64, Blo, dev(_stack(Bs, b)), Xd, tol=1e-10, maxit=4000)
    X = host(Xd)
    r0 = 0
    for k, A in enumerate(mats):
        assert st[k]["converged"] == 1, (k, st[k])
        rel = _oracle_relres(A, Bs[k], X[r0:r0 + A.nrows])
        assert np.all(rel <= 1.05e-10), (k, rel)
        r0 += A.nrows
    for obj in [B64, Blo] + M64 + Mlo:
        if obj is not None:
            obj.close()


@pytest.mark.parametrize("mode", ["f64", "bf16"])
def test_batch_cg_graph_equals_eager(sc, mode):
    import torch

    mats = _cg_systems()
    b = 3
    M64 = [sc.SellMatrix.from_csr(A, C=16, sigma=8) for A in mats]
    B64 = sc.SellBatch(M64)
    Mlo = [sc.SellMatrix.from_csr(A, C=16, sigma=8, dtype=mode) for A in mats] if mode != "f64" else []
    Blo = sc.SellBatch(Mlo) if Mlo else None
    Bs = dev(_stack([synth.block_vector(A.nrows, b, 700 + k) for k, A in enumerate(mats)], b))
    X0 = dev(_stack([synth.block_vector(A.nrows, b, 800 + k) for k, A in enumerate(mats)], b))
    outs = []
    for graph in (False, True, True):
        X = X0.clone()
        st = sc.sell_batch_cg(B64, Blo, Bs, X, tol=1e-9, maxit=3000, graph=graph)
        outs.append((host(X), st))
    for X, st in outs[1:]:
        assert np.array_equal(X, outs[0][0])
        assert st == outs[0][1]
    for obj in [B64, Blo] + M64 + Mlo:
        if obj is not None:
            obj.close()


@pytest.mark.parametrize("mode", ["f64", "bf16"])
def test_batch_cg_graph_equals_eager_equal_systems(sc, mode):
    """Equal systems retire together, so the set of iterating systems stays the same for many
    runs and the graph is captured and replayed many times (unequal systems change that set
    every run or two, and a set is captured only from its third run on)."""
    A = synth.laplacian3d(10)
    K, b = 6, 3
    M64 = [sc.SellMatrix.from_csr(A, C=32, sigma=1) for _ in range(K)]
    B64 = sc.SellBatch(M64)
    Mlo = [sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=mode) for _ in range(K)] if mode != "f64" else []
    Blo = sc.SellBatch(Mlo) if Mlo else None
    Bs = dev(_stack([synth.block_vector(A.nrows, b, 900 + k) for k in range(K)], b))
    outs = []
    for graph in (False, True, True):
        X = dev(np.zeros((K * A.nrows, b)))
        st = sc.sell_batch_cg(B64, Blo, Bs, X, tol=1e-10, maxit=3000, graph=graph)
        assert all(e["converged"] == 1 for e in st), st
        outs.append((host(X), st))
    for X, st in outs[1:]:
        assert np.array_equal(X, outs[0][0])
        assert st == outs[0][1]
    for obj in [B64, Blo] + M64 + Mlo:
        if obj is not None:
            obj.close()


def test_batch_cg_initial_guess_exact_and_maxit(sc):
    import torch

    mats = _cg_systems()[:3]
    b = 2
    M64 = [sc.SellMatrix.from_csr(A) for A in mats]
    B64 = sc.SellBatch(M64)
    Xs = [synth.block_vector(A.nrows, b, 900 + k) for k, A in enumerate(mats)]
    Bs = [oracle.spmmv(A, X) for A, X in zip(mats, Xs)]
    Xd = dev(_stack(Xs, b))
    st = sc.sell_batch_cg(B64, None, dev(_stack(Bs, b)), Xd, tol=1e-10, maxit=100)
    assert all(s["converged"] == 1 and s["iterations"] == 0 for s in st)
    assert np.array_equal(host(Xd), _stack(Xs, b))
    # maxit = 5: stops early, reports the true residual, not converged
    Xd = torch.zeros((B64.rows, b), dtype=torch.float64, device="cuda:0")
    st = sc.sell_batch_cg(B64, None, dev(_stack(Bs, b)), Xd, tol=1e-12, maxit=5)
    X = host(Xd)
    r0 = 0
    for k, A in enumerate(mats):
        assert st[k]["iterations"] <= 5 and st[k]["converged"] == 0
        rel = _oracle_relres(A, Bs[k], X[r0:r0 + A.nrows]).max()
        assert abs(rel - st[k]["relres"]) <= 1e-6 * rel
        r0 += A.nrows
    B64.close()
    for M in M64:
        M.close()


def _pack(blocks):
    return np.concatenate([np.ascontiguousarray(v).ravel() for v in blocks]) if blocks else np.zeros(0)


@pytest.mark.parametrize("dt", ["f64", "bf16"])
@pytest.mark.parametrize("flags_name", ["plain", "shift_scale_axpby_dots", "vshift_chain_dots"])
@pytest.mark.parametrize("widths", [(1, 5, 8, 32, 3, 16), (2, 2, 4, 1, 8, 32)])
def test_batch_packed_widths_vs_oracle(sc, dt, flags_name, widths):
    """Matrices of different block widths in one launch, operands packed per matrix at its own
    width (the second set also puts 2-wide FP64 rows at offsets that break 16-byte alignment,
    which runs the run-time-width body for those matrices)."""
    import torch

    mats = _square_mats()
    flags = {"plain": 0,
             "shift_scale_axpby_dots": sc.SHIFT | sc.SCALE | sc.AXPBY | sc.DOTS,
             "vshift_chain_dots": sc.VSHIFT | sc.SCALE | sc.AXPBY | sc.DOTS | sc.CHAIN}[flags_name]
    wmax = max(widths)
    gv = np.linspace(-1, 1, wmax)
    kw = dict(alpha=0.5, beta=-1.25, gamma=0.1, delta=0.3, eta=-2.0)
    Ms = [sc.SellMatrix.from_csr(A, C=32 if k % 2 == 0 else 8, sigma=[1, 64, 7][k % 3], dtype=dt)
          for k, A in enumerate(mats)]
    Bt = sc.SellBatch(Ms)
    Bt.set_widths(widths)
    nx, ny, nd = Bt.packed_sizes()
    assert nx == sum(A.ncols * w for A, w in zip(mats, widths)) and nd == 3 * sum(widths)
    vt = torch.float64 if dt == "f64" else torch.float32
    Xs = [synth.block_vector(A.ncols, w, synth.SEED_X + 1000 * k) for k, (A, w) in enumerate(zip(mats, widths))]
    Ys = [synth.block_vector(A.nrows, w, synth.SEED_Y + 1000 * k) for k, (A, w) in enumerate(zip(mats, widths))]
    Zs = [synth.block_vector(A.nrows, w, synth.SEED_Y + 7 + 1000 * k) for k, (A, w) in enumerate(zip(mats, widths))]
    if dt != "f64":
        Xs, Ys, Zs = [[oracle.round_f32(v) for v in L] for L in (Xs, Ys, Zs)]
    Xd, Yd, Zd = dev(_pack(Xs), vt), dev(_pack(Ys), vt), dev(_pack(Zs), vt)
    dot = torch.full((nd,), float("nan"), dtype=torch.float64, device="cuda:0")
    sc.sell_batch_spmmv_aug_packed(Bt, Xd, Yd, Zd if flags & sc.CHAIN else None, flags=flags,
                                   dot=dot if flags & sc.DOTS else None,
                                   gamma_v=gv if flags & sc.VSHIFT else None, **kw)
    Yg, Zg, dg = host(Yd), host(Zd), host(dot)
    if dt == "f64":
        tol = 1e-12
    else:
        k = max(int(np.diff(A.rowptr).max()) for A in mats if A.nrows) + 3
        tol = k * 2.0 ** -24 / (1 - k * 2.0 ** -24)
    gmax = 1.0 if flags & sc.VSHIFT else 0.1
    esize = 8 if dt == "f64" else 4
    xo = yo = do = 0
    for k, (A, w) in enumerate(zip(mats, widths)):
        Yk = Yg[yo: yo + A.nrows * w].reshape(A.nrows, w)
        Zk = Zg[yo: yo + A.nrows * w].reshape(A.nrows, w)
        got = dg[3 * do: 3 * (do + w)]
        # the batch runs the body compiled for w when the packed rows allow its vector accesses
        al = min(16, (4 if w >= 4 else w) * esize)
        same_body = w not in (1, 2, 4, 8, 16, 32) or all((o * esize) % al == 0 for o in (xo, yo, w))
        xo += A.ncols * w
        yo += A.nrows * w
        do += w
        if A.nrows == 0:
            if flags & sc.DOTS:
                assert np.all(got == 0.0)
            continue
        Ar = _value_ref(A, dt)
        if flags:
            Yr, Zr, dr = oracle.spmmv_aug(Ar, Xs[k], Ys[k], Zs[k], flags=to_oracle_flags(flags),
                                          gamma_v=gv[:w] if flags & sc.VSHIFT else None, **kw)
        else:
            Yr, Zr, dr = oracle.spmmv(Ar, Xs[k]), None, None
        scale = 0.5 * (abs_product(Ar, Xs[k]) + gmax * np.abs(Xs[k])) + 1.25 * np.abs(Ys[k]) if flags else \
            abs_product(Ar, Xs[k])
        assert colwise_relerr(Yk, Yr, scale) <= tol, (k, "y")
        if flags & sc.CHAIN:
            assert colwise_relerr(Zk, Zr, 0.3 * np.abs(Zs[k]) + 2.0 * np.abs(Yr) + 2 * scale) <= tol, (k, "z")
        if flags & sc.DOTS:
            den = np.concatenate([np.sum(Yk * Yk + 2 * np.abs(Yk) * scale, axis=0),
                                  np.sum(np.abs(Xs[k]) * (np.abs(Yk) + scale), axis=0), np.sum(Xs[k] * Xs[k], axis=0)])
            assert np.all(np.abs(got - dr) <= tol * den + 1e-300), (k, "dots")
        # every row is computed the same way as by the single-matrix entry point (same body)
        if same_body and not flags & sc.CHAIN:
            Y1 = dev(Ys[k], vt)
            d1 = torch.zeros(3 * w, dtype=torch.float64, device="cuda:0")
            sc.sell_spmmv_aug(Ms[k], dev(Xs[k], vt), Y1, flags=flags, dot=d1 if flags & sc.DOTS else None,
                              gamma_v=gv[:w] if flags & sc.VSHIFT else None, **kw)
            assert np.array_equal(host(Y1), Yk), (k, "single")
    Bt.close()
    for M in Ms:
        M.close()


def test_batch_widths_state_and_errors(sc):
    import torch

    mats = _square_mats()
    Ms = [sc.SellMatrix.from_csr(A) for A in mats]
    Bt = sc.SellBatch(Ms)
    b = 8
    Xd = dev(np.concatenate([synth.block_vector(A.ncols, b, 11 + k) for k, A in enumerate(mats)]))
    Y0 = dev(np.concatenate([synth.block_vector(A.nrows, b, 21 + k) for k, A in enumerate(mats)]))
    fl = sc.SHIFT | sc.AXPBY | sc.DOTS
    dot = torch.zeros(3 * b * len(mats), dtype=torch.float64, device="cuda:0")
    Yref = Y0.clone()
    sc.sell_batch_spmmv_aug(Bt, Xd, Yref, flags=fl, beta=0.5, gamma=0.2, dot=dot)
    # packed operands with every width b are the stacked operands: the same rows, bit for bit
    Bt.set_widths([b] * len(mats))
    Yp = Y0.clone().ravel()
    dp = torch.zeros(3 * b * len(mats), dtype=torch.float64, device="cuda:0")
    sc.sell_batch_spmmv_aug_packed(Bt, Xd.ravel(), Yp, flags=fl, beta=0.5, gamma=0.2, dot=dp)
    assert np.array_equal(host(Yp), host(Yref).ravel())
    assert np.allclose(host(dp), host(dot), rtol=1e-13, atol=0)
    # with every width equal to b the stacked entry point still works
    Y2 = Y0.clone()
    sc.sell_batch_spmmv_aug(Bt, Xd, Y2, flags=fl, beta=0.5, gamma=0.2, dot=dot)
    assert np.array_equal(host(Y2), host(Yref))
    with pytest.raises(sc.SellError):
        Bt.set_widths([0] * len(mats))
    with pytest.raises(sc.SellError):
        Bt.set_widths([65] * len(mats))
    Bt.set_widths([1, 2, 3, 4, 5, 6])
    with pytest.raises(sc.SellError):  # stacked operands need one width
        sc.sell_batch_spmmv_aug(Bt, Xd, Y0.clone())
    with pytest.raises(sc.SellError):  # so does the batched solver
        sc.sell_batch_cg(Bt, None, Y0.clone(), torch.zeros_like(Y0), tol=1e-8, maxit=10)
    with pytest.raises(sc.SellError):  # operands of the wrong packed size
        sc.sell_batch_spmmv_aug_packed(Bt, Xd.ravel(), Y0.clone().ravel())
    Bt.set_widths(None)
    with pytest.raises(sc.SellError):  # no widths set
        sc.lib()  # keep the library loaded; the raw call below must fail on the state
        sc._ok(sc.lib().sell_batch_spmmv_aug_packed(Bt.handle, None, None, None, None, None), "packed")
    Y3 = Y0.clone()
    sc.sell_batch_spmmv_aug(Bt, Xd, Y3, flags=fl, beta=0.5, gamma=0.2, dot=dot)
    assert np.array_equal(host(Y3), host(Yref))
    Bt.close()
    for M in Ms:
        M.close()


@pytest.mark.parametrize("dt", ["f64", "bf16"])
def test_batch_index_batch_lengths_bit_identical(sc, dt):
    """A batched launch takes the index batch length its matrices share (set before the batch
    is created; 8 when they differ): every length gives the same outputs and dots bit for bit."""
    import torch

    mats = [synth.laplacian3d(12), synth.laplacian3d(9), synth.anderson3d(10),
            synth.random_sparse(900, 900, 0.01, 76, empty_rows=9, long_row=300)]
    vt = torch.float64 if dt == "f64" else torch.float32
    b = 8
    Xd = dev(_stack([synth.block_vector(A.ncols, b, 77 + k) for k, A in enumerate(mats)], b), vt)
    Y0 = _stack([synth.block_vector(A.nrows, b, 78 + k) for k, A in enumerate(mats)], b)
    fl = sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY | sc.DOT_XY | sc.DOT_XX
    ref = None
    for lens in ((8, 8, 8, 8), (7, 7, 7, 7), (5, 5, 5, 5), (7, 5, 8, 7), (0, 0, 0, 0)):
        Ms = [sc.SellMatrix.from_csr(A, C=32, sigma=64, dtype=dt) for A in mats]
        for M, ln in zip(Ms, lens):
            M.set_batch(ln)
        Bt = sc.SellBatch(Ms)
        Yd = dev(Y0, vt)
        dot = torch.zeros(3 * b * len(mats), dtype=torch.float64, device="cuda:0")
        sc.sell_batch_spmmv_aug(Bt, Xd, Yd, flags=fl, alpha=0.5, gamma=0.25, beta=-1.0, dot=dot)
        got = (host(Yd), host(dot))
        if ref is None:
            ref = got
            # the first matrix alone (single-matrix kernel) gives its rows of the batch
            n0 = mats[0].nrows
            Y1 = dev(Y0[:n0], vt)
            d1 = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
            sc.sell_spmmv_aug(Ms[0], Xd[:mats[0].ncols].contiguous(), Y1, flags=fl, alpha=0.5, gamma=0.25,
                              beta=-1.0, dot=d1)
            assert np.array_equal(host(Y1), got[0][:n0])
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), lens
        Bt.close()
        for M in Ms:
            M.close()
