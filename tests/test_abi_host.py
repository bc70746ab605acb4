"""CPU tests of the C ABI: the library loads and exports what the header declares, and the
host-side SELL-C-sigma construction (integer work) agrees bit for bit with the oracle."""
import ctypes as ct
import json
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module")
def sc():
    import paper_1507_08101_amd as sc

    if not os.path.exists(sc.LIB_PATH):
        from paper_1507_08101_amd import _build

        _build.build()
    sc.lib()
    return sc


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(sell_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(sc):
    names = _declared_functions()
    assert len(names) >= 20, names
    L = ct.CDLL(sc.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) <= set(sc._SIGNATURES), set(names) - set(sc._SIGNATURES)


def test_strerror_and_version(sc):
    for code in range(0, -8, -1):
        assert sc.lib().sell_strerror(code)
    assert sc.lib().sell_version() >= 10000


def _host(sc, A, C, sigma, dt="f64"):
    return sc.SellMatrix.from_csr(A, C=C, sigma=sigma, dtype=dt, host_only=True)


@pytest.mark.parametrize("C,sigma", [(1, 1), (4, 1), (4, 8), (32, 1), (32, 32), (32, 1024), (64, 4096), (7, 5),
                                     (64, 1), (256, 256)])
def test_host_layout_matches_oracle_bit_exact(sc, orc, C, sigma):
    for A in [synth.irregular(3000, band=60, max_len=400, seed=5), synth.random_sparse(90, 70, 0.1, 7, empty_rows=9),
              synth.laplacian2d(20)]:
        M = _host(sc, A, C, sigma)
        perm, cl, cs, col, val = M.export_sell()
        operm, ocl, ocs = orc.sell_layout(A, C, sigma)
        ocol, oval = orc.sell_fill(A, C, operm, ocl, ocs)
        assert np.array_equal(perm, operm) and np.array_equal(cl, ocl) and np.array_equal(cs, ocs)
        assert np.array_equal(col, ocol) and np.array_equal(val.view(np.int64), oval.view(np.int64))
        i = M.info
        assert (i["nrows"], i["ncols"], i["nnz"], i["stored"]) == (A.nrows, A.ncols, A.nnz, int(ocs[-1]))
        assert i["has_perm"] == int(not np.array_equal(operm[:A.nrows], np.arange(A.nrows)))
        M.close()


def test_host_padding_golden(sc):
    g = json.load(open(os.path.join(GOLDEN, "sell_padding_lap2d_64.json")))
    A = synth.laplacian2d(64)
    for case in g["cases"]:
        M = _host(sc, A, case["C"], case["sigma"])
        assert M.info["stored"] == case["stored"], case
        M.close()


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_export_csr_round_trip(sc, orc, dt):
    A = synth.random_sparse(120, 77, 0.08, 9, duplicates=True, empty_rows=11, long_row=77)
    M = _host(sc, A, 8, 32, dt)
    rp, col, val = M.export_csr()
    assert np.array_equal(rp, A.rowptr) and np.array_equal(col, A.col)
    want = {"f64": A.val, "f32": orc.round_f32(A.val), "bf16": orc.round_bf16(A.val)}[dt]
    assert np.array_equal(val.view(np.int64), want.view(np.int64))
    M.close()


def test_bf16_rounding_matches_oracle_on_hard_values(sc, orc):
    e = 2.0 ** -8
    vals = np.array([1 + e, 1 + 3 * e, 1 + e + 2.0 ** -40, -(1 + e + 2.0 ** -40), 3.5e38, -3.5e38, 1e-40, -3e-39,
                     2.0 ** -133, 1.5 * 2.0 ** -133, 2.5 * 2.0 ** -133, 0.0, 6.0, -1.0, 4.0, 1e-300])
    vals = np.concatenate([vals, synth.normal(3, 5000) * np.exp(synth.uniform(4, 5000, -95, 95))])
    n = vals.size
    A = synth.CSR(n, 1, np.arange(n + 1), np.zeros(n, np.int32), vals, "diag-like")
    for dt, ref in [("bf16", orc.round_bf16(vals)), ("f32", orc.round_f32(vals))]:
        M = _host(sc, A, 4, 1, dt)
        _, _, v = M.export_csr()
        assert np.array_equal(v, ref), dt
        M.close()


def test_update_values_host(sc):
    A = synth.random_sparse(50, 50, 0.2, 12)
    M = _host(sc, A, 8, 16)
    newv = synth.uniform(13, A.nnz, -5, 5)
    M.update_values(newv)
    _, col, val = M.export_csr()
    assert np.array_equal(val, newv) and np.array_equal(col, A.col)
    M.close()


def test_empty_and_degenerate_builds(sc):
    E = synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), "empty")
    M = _host(sc, E, 32, 1)
    assert M.info["nchunks"] == 0 and M.info["stored"] == 0
    M.close()
    Z = synth.CSR(10, 10, np.zeros(11, np.int64), np.zeros(0, np.int32), np.zeros(0), "zero")
    M = _host(sc, Z, 4, 8)
    assert M.info["stored"] == 0 and M.info["nchunks"] == 3
    rp, _, _ = M.export_csr()
    assert np.array_equal(rp, Z.rowptr)
    M.close()


def test_build_rejects_bad_input(sc):
    A = synth.random_sparse(10, 10, 0.3, 14)
    ok = dict(nrows=10, ncols=10, rowptr=A.rowptr, col=A.col, val=A.val, C=4, sigma=1)

    def build(**kw):
        d = dict(ok)
        d.update(kw)
        return sc.sell_build(d["nrows"], d["ncols"], d["rowptr"], d["col"], d["val"], d["C"], d["sigma"],
                             host_only=True)

    sc.sell_destroy(build())
    bad_rp = A.rowptr.copy()
    bad_rp[3], bad_rp[4] = bad_rp[4], bad_rp[3] - 1
    col_hi = A.col.copy()
    col_hi[0] = 10
    col_neg = A.col.copy()
    col_neg[-1] = -1
    rp0 = A.rowptr + 1
    for kw in [dict(C=0), dict(sigma=0), dict(rowptr=bad_rp), dict(col=col_hi), dict(col=col_neg),
               dict(rowptr=rp0, col=np.concatenate([A.col, [0]]), val=np.concatenate([A.val, [0.0]])),
               dict(ncols=2 ** 31)]:
        with pytest.raises(sc.SellError) as ei:
            build(**kw)
        assert ei.value.code == sc.SELL_ERR_ARG, kw
    with pytest.raises(sc.SellError) as ei:
        sc.sell_build(10, 10, A.rowptr, A.col, A.val, 4, 1, vdt=7, host_only=True)
    assert ei.value.code == sc.SELL_ERR_DTYPE


def test_host_only_matrix_rejected_by_compute_calls(sc):
    A = synth.laplacian2d(4)
    M = _host(sc, A, 4, 1)
    rc = sc.lib().sell_spmmv(M.handle, None, None, None)
    assert rc == sc.SELL_ERR_STATE
    M.close()


def test_byte_model_matches_paper_figures():
    from paper_1507_08101_amd import model

    g = json.load(open(os.path.join(GOLDEN, "code_balance.json")))
    first = g["items"][0]
    assert model.min_code_balance(first["value_bytes"], first["index_bytes"]) == first["value_bytes_per_flop"]
    for case in g["items"][1]["cases"]:
        red = model.index_width_reduction(case["value_bytes"])
        assert int(100 * red) == case["reduction_percent"]
    ch = json.load(open(os.path.join(GOLDEN, "chunk_height.json")))
    assert model.min_chunk_height(ch["simd_bytes"], ch["element_bytes"]) == ch["C_min"]


@pytest.mark.parametrize("name,make,C,sigma,batch,wide", [
    ("anderson3d_24", lambda: synth.anderson3d(24), 32, 1, 7, 7),      # 7 entries per row
    ("laplacian3d_20", lambda: synth.laplacian3d(20), 32, 1, 7, 7),    # 7, 4..6 at the faces
    ("laplacian2d_64", lambda: synth.laplacian2d(64), 32, 1, 5, 5),    # 5, 3..4 at the edges
    ("laplacian2d_64_C64", lambda: synth.laplacian2d(64), 64, 4096, 5, 5),
    ("irregular_20000", lambda: synth.irregular(20000, band=2000, max_len=300, seed=5), 32, 1, 8, 7),
    ("empty_rows", lambda: synth.CSR(10, 10, np.zeros(11, np.int64), np.zeros(0, np.int32), np.zeros(0), "z"),
     4, 1, 8, 7),
])
def test_batch_length_choice(sc, name, make, C, sigma, batch, wide):
    """The construction picks the index batch length from the chunk lengths: 7 for 7-entry rows,
    5 for 5-entry rows, 8 otherwise (5 or 7 only for the kernels gathering 32 bytes per lane);
    sell_set_batch sets one length for every kernel and 0 restores the choice."""
    M = _host(sc, make(), C, sigma)
    assert (M.info["batch"], M.info["batch_wide"]) == (batch, wide), name
    for b in (5, 7, 8):
        M.set_batch(b)
        assert M.info["batch"] == b and M.info["batch_wide"] == b
    M.set_batch(0)
    assert (M.info["batch"], M.info["batch_wide"]) == (batch, wide)
    for bad in (-1, 1, 4, 6, 9, 16, 32):
        with pytest.raises(sc.SellError):
            M.set_batch(bad)
    assert M.info["batch"] == batch
    M.close()


_LOG_SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1])
import paper_1507_08101_amd as sc, synth
A = synth.laplacian2d(6)
M = sc.SellMatrix.from_csr(A, C=4, sigma=8, host_only=True)
info = M.info
print(info["stored"], info["nchunks"], flush=True)
M.close()
"""


@pytest.mark.parametrize("level", [None, "0", "1", "2"])
def test_log_level_lines(sc, level):
    """SELLCS_LOG: nothing at 0 (or unset) and 1 for a build, which has no performance warning;
    at 2 one INFO line that states what the build made."""
    import subprocess
    import sys

    env = dict(os.environ)
    env.pop("SELLCS_LOG", None)
    if level is not None:
        env["SELLCS_LOG"] = level
    r = subprocess.run([sys.executable, "-c", _LOG_SCRIPT, ROOT], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    stored, nch = (int(v) for v in r.stdout.split())
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("[sellcs]")]
    if level != "2":
        assert lines == []
        return
    assert len(lines) == 1, lines
    # laplacian2d(6): 36 rows, N^2 + 4N(N-1) = 156 nonzeros
    assert lines[0].startswith(f"[sellcs] INFO built SELL-4-8 in host memory only: 36 x 36, 156 nonzeros, "
                               f"{stored} stored ({stored / 156:.4f} per nonzero), {nch} chunks, "), lines[0]
    assert "f64 values" in lines[0]
