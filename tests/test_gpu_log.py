"""GPU test of the SELLCS_LOG performance warnings. The level is read once per process, so
the calls run in a child process with SELLCS_LOG=1: a block width without a fixed-width
kernel, column-major block vectors, a batched product of such a width and the atomic
transpose each print one PERFWARNING line, once however often the call repeats; the
fixed-width row-major product prints none."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1])
import torch
import paper_1507_08101_amd as sc
import synth
A = synth.laplacian2d(8)
M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
n = A.nrows
X8 = torch.rand((n, 8), dtype=torch.float64, device="cuda")
Y8 = torch.empty_like(X8)
sc.sell_spmmv(M, X8, Y8)
torch.cuda.synchronize()
print("STEP fixed", flush=True)
Bt = sc.SellBatch([M, M])
for _ in range(3):
    X3 = torch.rand((n, 3), dtype=torch.float64, device="cuda")
    Y3 = torch.empty_like(X3)
    sc.sell_spmmv(M, X3, Y3)
    Xc = torch.rand((4, n), dtype=torch.float64, device="cuda").T
    Yc = torch.empty((4, n), dtype=torch.float64, device="cuda").T
    sc.sell_spmmv(M, Xc, Yc)
    sc.sell_spmmv_T(M, X3, Y3, deterministic=False)
    Xb = torch.rand((2 * n, 3), dtype=torch.float64, device="cuda")
    Yb = torch.empty_like(Xb)
    sc.sell_batch_spmmv_aug(Bt, Xb, Yb)
torch.cuda.synchronize()
Bt.close()
M.close()
print("STEP done", flush=True)
"""


def test_perfwarnings_once_each():
    env = dict(os.environ, SELLCS_LOG="1")
    r = subprocess.run([sys.executable, "-u", "-c", _SCRIPT, ROOT], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "STEP done" in r.stdout
    # stderr lines in order: nothing before the first odd call (the fixed-width product is silent)
    warn = [ln for ln in r.stderr.splitlines() if ln.startswith("[sellcs]")]
    assert all(ln.startswith("[sellcs] PERFWARNING ") for ln in warn), warn
    assert len(warn) == 4, warn
    assert "block width 3 has no fixed-width product kernel" in warn[0]
    assert "not row-major with 16-byte aligned rows" in warn[1]
    assert "atomic scatter" in warn[2]
    assert "batched product with block width 3" in warn[3]
