"""Benchmark: SELL-C-sigma augmented SpMMV in the kernel polynomial method recurrence.

Workload (one "step"): the Chebyshev/KPM recurrence of M = 200 augmented SpMMVs
    v_{m+1} = (2/s) (A - c I) v_m - v_{m-1},  with fused <v,v> and <v_m, v_{m+1}>,
on the 3D periodic Anderson Hamiltonian of a 128^3 lattice (n = 2,097,152, 7 nonzeros per
row, disorder U[-8.25, 8.25]), FP64, SELL-32-1, row-major block vector of width b = 8
(b = 1 is reported beside it). Inputs are synthetic and seeded and resident in HBM before
the timed region.

Prints ONE JSON line: GFLOP/s (2 flops per true nonzero per vector) of the whole recurrence,
with HBM GB/s against the MI355X's 8 TB/s in "roofline" (algorithmic bytes per launch /
average launch duration from HIP events recorded on the launch stream), measured
achievable bandwidth from streaming probes, the FP64-vs-mixed-precision CG comparison and
the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
W_DISORDER = 16.5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("spmmv_impl.h", "spmmv_f64.hip", "internal.h", "vecops.hip"):
        with open(os.path.join(ROOT, "paper_1507_08101_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str, src_hash: str):
    """HBM traffic per launch measured with rocprofv3 counters (profiles/), or None when the
    kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != src_hash:
        return None
    return d.get("traffic_bytes_per_launch")


# read:write mixes of the streaming probe (name, read streams, write streams)
PROBE_MIXES = (("read", 1, 0), ("write", 0, 1), ("copy", 1, 1), ("triad", 2, 1), ("mix3", 3, 1), ("mix4", 4, 1))
PROBE_GRIDS = (1024, 2048, 4096, 8192, 16384, 65536)
PROBE_UNROLLS = (1, 2, 4, 8)


def probe_bandwidth(sc, torch, nbytes=2 << 30, sweep_reps=2, reps=10):
    """Achievable HBM bandwidth per read:write mix with the library's streaming probe: every
    mix swept over the grid (workgroups of 256), the elements in flight per stream and thread,
    and nontemporal or plain accesses; the three fastest shapes are timed again (best of reps).
    Each stream is nbytes (2 GiB: 8x the infinity cache), so a mix of R reads and W writes
    moves (R + W) nbytes."""
    src = torch.empty(4 * nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    src.fill_(1.0)

    def timed(R, W, u, nt, g, n):
        best = float("inf")
        for _ in range(n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sc.sell_probe_stream(R, W, u, nt, g, dst, src, nbytes)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    out = {}
    for name, R, W in PROBE_MIXES:
        moved = (R + W) * nbytes
        trials = sorted((timed(R, W, u, nt, g, sweep_reps), g, u, nt)
                        for nt in (0, 1) for g in PROBE_GRIDS for u in PROBE_UNROLLS)
        best = min((timed(R, W, u, nt, g, reps), g, u, nt) for _, g, u, nt in trials[:3])
        worst = trials[-1][0]
        out[name] = {"GB/s": round(moved / (best[0] * 1e-3) / 1e9, 1), "grid": best[1], "unroll": best[2],
                     "nontemporal": best[3], "read_bytes": R * nbytes, "write_bytes": W * nbytes,
                     "slowest_shape_GB/s": round(moved / (worst * 1e-3) / 1e9, 1)}
    del src, dst
    torch.cuda.empty_cache()
    return out


def achievable_for_mix(probes, read_bytes, write_bytes):
    """The achievable rate for a kernel's read:write mix: the probe whose mix is nearest (in the
    fraction of bytes written), and the time model that charges reads at the read probe's rate
    and writes at the write probe's rate one after the other."""
    wf = write_bytes / (read_bytes + write_bytes)
    name = min((n for n, R, W in PROBE_MIXES if R > 0 and W > 0), key=lambda n: abs(
        probes[n]["write_bytes"] / (probes[n]["read_bytes"] + probes[n]["write_bytes"]) - wf))
    t = read_bytes / probes["read"]["GB/s"] + write_bytes / probes["write"]["GB/s"]
    return name, probes[name]["GB/s"], (read_bytes + write_bytes) / t

def kpm_run(sc, torch, M_h, V0d, b, M, s, timed_steps, warmup):
    n = V0d.shape[0]
    V = torch.empty((n, b), dtype=torch.float64, device="cuda")
    W = torch.empty_like(V)
    mu = torch.empty((2 * M + 1) * b, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        V.copy_(V0d)
        sc.sell_kpm(M_h, V, W, M, s, 0.0, mu)
    torch.cuda.synchronize()
    step_ms = []
    launch_ms = []
    for _ in range(timed_steps):
        V.copy_(V0d)  # outside the step timing: restore v0
        torch.cuda.synchronize()
        lm = np.zeros(M, dtype=np.float32)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sc.sell_kpm(M_h, V, W, M, s, 0.0, mu, step_ms=lm)
        e1.record()
        e1.synchronize()
        step_ms.append(e0.elapsed_time(e1))
        launch_ms.append(lm)
    return np.array(step_ms), np.concatenate(launch_ms), mu


def cg_compare(sc, torch, synth, edge, nrhs=8, tol=1e-10):
    """Time to ||b - Ax|| <= tol ||b||: FP64 CG vs BF16-value CG with FP64 refinement."""
    A = synth.laplacian3d(edge)
    B = synth.block_vector(A.nrows, nrhs, synth.SEED_Y)
    Bd = torch.from_numpy(B).cuda()
    out = {"matrix": f"3D 7-point Dirichlet Laplacian {edge}^3", "n": A.nrows, "nnz": A.nnz, "nrhs": nrhs}
    A64 = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype="f64")
    for lo in ("bf16", "f32"):
        Alo = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=lo)
        for rep in range(2):
            Xd = torch.zeros_like(Bd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sc.sell_cg_mixed(A64, Alo, Bd, Xd, tol=tol)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
        out[f"mixed_{lo}"] = dict(seconds=t, **st)
        Alo.close()
    for rep in range(2):
        Xd = torch.zeros_like(Bd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sc.sell_cg(A64, Bd, Xd, tol=tol)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
    out["fp64"] = dict(seconds=t, **st)
    A64.close()
    out["speedup_bf16_vs_fp64"] = out["fp64"]["seconds"] / out["mixed_bf16"]["seconds"]
    return out


def cg_reference_row(sc, torch, synth, oracle, edge=50, tol=1e-10):
    """Iteration counts of the GPU's CG drivers beside the oracle's on one right-hand side of a
    3D Laplacian: FP64 CG, and the textbook refinement around a float inner CG on BF16 values
    that restarts at every refinement after a 1e-4 reduction (the GPU's mixed driver instead
    keeps its search direction across reliable updates)."""
    A = synth.laplacian3d(edge)
    b = synth.block_vector(A.nrows, 1, synth.SEED_Y)
    out = {"matrix": f"3D 7-point Dirichlet Laplacian {edge}^3", "n": A.nrows, "nrhs": 1}
    t0 = time.perf_counter()
    _, it64 = oracle.cg(A, b[:, 0], tol=tol)
    _, outer, inner, rr = oracle.cg_refine(A, b[:, 0], val_low=oracle.round_bf16(A.val), tol=tol, inner_rtol=1e-4)
    out["oracle"] = {"fp64_cg_iterations": it64, "refine_bf16_outer": outer, "refine_bf16_inner_total": inner,
                     "refine_relres": rr, "inner_rtol": 1e-4, "seconds": round(time.perf_counter() - t0, 2)}
    A64 = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype="f64")
    Alo = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype="bf16")
    Bd = torch.from_numpy(b).cuda()
    Xd = torch.zeros_like(Bd)
    st64 = sc.sell_cg(A64, Bd, Xd, tol=tol)
    Xd = torch.zeros_like(Bd)
    stm = sc.sell_cg_mixed(A64, Alo, Bd, Xd, tol=tol)
    out["gpu"] = {"fp64_cg_iterations": st64["iterations"], "mixed_bf16_iterations": stm["iterations"],
                  "mixed_bf16_refinements": stm["refinements"], "mixed_relres": stm["relres"]}
    A64.close()
    Alo.close()
    return out


def batch_row(sc, torch, synth, model, nmat=64, b=8, tol=1e-10):
    """Batched workload: nmat 3D Laplacians with edges ~ U{20..100}, b right-hand sides each.
    Formats and launch shapes from the autotuner; one batched product launch (FP64) against
    the same products launched matrix by matrix; CG to tol for the whole batch in FP64 and
    with FP32 iterations on BF16 / FP32 values refined in FP64 (HIP graph on)."""
    t0 = time.perf_counter()
    edges = synth.laplacian3d_batch(nmat)
    mats = [synth.laplacian3d(e) for e in edges]
    gen_s = time.perf_counter() - t0
    n_tot = sum(A.nrows for A in mats)
    nnz_tot = sum(A.nnz for A in mats)
    out = {"matrices": f"{nmat} 3D 7-point Dirichlet Laplacians, edge ~ U{{20..100}}", "n_total": n_tot,
           "nnz_total": nnz_tot, "b": b, "generate_s": round(gen_s, 1)}
    t0 = time.perf_counter()
    tunes = {}
    M = {}
    for dt in ("f64", "bf16", "f32"):
        Ms = []
        for A in mats:
            t = sc.sell_autotune(A, b, "bf16" if dt == "f32" else dt)
            Mk = sc.SellMatrix.from_csr(A, C=t["C"], sigma=t["sigma"], dtype=dt)
            Mk.set_launch(t["vpt"], t["blocks_per_cu"])
            Ms.append(Mk)
            key = (dt, t["C"], t["sigma"], t["vpt"], t["blocks_per_cu"])
            tunes[key] = tunes.get(key, 0) + 1
        M[dt] = Ms
    out["tune_and_build_s"] = round(time.perf_counter() - t0, 1)
    out["tuned_choices"] = [dict(dtype=k[0], C=k[1], sigma=k[2], vpt=k[3], blocks_per_cu=k[4], matrices=v)
                            for k, v in sorted(tunes.items())]
    log(f"[bench] batch: {n_tot} rows, {nnz_tot} nnz, tuned {out['tuned_choices']}")
    B64 = sc.SellBatch(M["f64"])
    Bbf = sc.SellBatch(M["bf16"])
    B32 = sc.SellBatch(M["f32"])
    Xd = torch.rand((n_tot, b), dtype=torch.float64, device="cuda") * 2 - 1
    Yd = torch.empty_like(Xd)
    dots = torch.zeros(3 * b * nmat, dtype=torch.float64, device="cuda")
    alg_bytes = 0
    for A, Mk in zip(mats, M["f64"]):
        alg_bytes += model.bytes_min(A.nnz, A.nrows, A.ncols, b, 8, 8, read_y=False, nchunks=Mk.info["nchunks"])
    us, us_min = time_launches(torch, lambda: sc.sell_batch_spmmv_aug(B64, Xd, Yd, flags=sc.DOT_XY, dot=dots),
                               reps=10, inner=5)
    out["batched_product_f64"] = {"us": round(us, 1), "GB/s": round(alg_bytes / (us * 1e-6) / 1e9, 1),
                                  "GFLOP/s": round(2.0 * nnz_tot * b / (us * 1e-6) / 1e9, 1),
                                  "bytes": int(alg_bytes)}
    offs = np.cumsum([0] + [A.nrows for A in mats])
    dsingle = torch.zeros(3 * b, dtype=torch.float64, device="cuda")

    def one_by_one():
        for k, Mk in enumerate(M["f64"]):
            sc.sell_spmmv_aug(Mk, Xd[offs[k]:offs[k + 1]], Yd[offs[k]:offs[k + 1]], flags=sc.DOT_XY, dot=dsingle)

    us1, _ = time_launches(torch, one_by_one, reps=5)
    out["per_matrix_launches_f64_us"] = round(us1, 1)
    log(f"[bench] batch product: {out['batched_product_f64']}, one by one {us1:.0f} us")
    # block widths 1..32 mixed over the matrices in one launch (operands packed per matrix at its
    # own width), against one launch per matrix and one batch per width
    wlist = [(1, 2, 4, 8, 16, 32)[k % 6] for k in range(nmat)]
    B64.set_widths(wlist)
    nx, ny, nd = B64.packed_sizes()
    Xp = torch.rand(nx, dtype=torch.float64, device="cuda") * 2 - 1
    Yp = torch.empty(ny, dtype=torch.float64, device="cuda")
    dp = torch.zeros(nd, dtype=torch.float64, device="cuda")
    usw, _ = time_launches(torch, lambda: sc.sell_batch_spmmv_aug_packed(B64, Xp, Yp, flags=sc.DOT_XY, dot=dp),
                           reps=4, inner=5)
    B64.set_widths(None)
    xo = np.cumsum([0] + [A.ncols * wlist[k] for k, A in enumerate(mats)])
    yo = np.cumsum([0] + [A.nrows * wlist[k] for k, A in enumerate(mats)])
    views = [(Xp[xo[k]:xo[k + 1]].view(A.ncols, wlist[k]), Yp[yo[k]:yo[k + 1]].view(A.nrows, wlist[k]))
             for k, A in enumerate(mats)]
    dw1 = torch.zeros(3 * max(wlist), dtype=torch.float64, device="cuda")

    def one_by_one_w():
        for k, Mk in enumerate(M["f64"]):
            sc.sell_spmmv_aug(Mk, views[k][0], views[k][1], flags=sc.DOT_XY, dot=dw1)

    usw1, _ = time_launches(torch, one_by_one_w, reps=5)
    classes = []
    for w in sorted(set(wlist)):
        ks = [k for k in range(nmat) if wlist[k] == w]
        Bw = sc.SellBatch([M["f64"][k] for k in ks])
        Xc = torch.cat([views[k][0] for k in ks]).contiguous()
        classes.append((Bw, Xc, torch.empty((Bw.rows, w), dtype=torch.float64, device="cuda"),
                        torch.zeros(3 * w * len(ks), dtype=torch.float64, device="cuda")))

    def per_class():
        for Bw, Xc, Yc, dc in classes:
            sc.sell_batch_spmmv_aug(Bw, Xc, Yc, flags=sc.DOT_XY, dot=dc)

    usc, _ = time_launches(torch, per_class, reps=10)
    for Bw, _, _, _ in classes:
        Bw.close()
    del classes, views, Xp, Yp
    wbytes = sum(model.bytes_min(A.nnz, A.nrows, A.ncols, wlist[k], 8, 8, nchunks=M["f64"][k].info["nchunks"])
                 for k, A in enumerate(mats))
    wflops = sum(2.0 * A.nnz * wlist[k] for k, A in enumerate(mats))
    out["mixed_widths_f64"] = {"widths": "1,2,4,8,16,32 in turn, packed operands", "us": round(usw, 1),
                               "GB/s": round(wbytes / (usw * 1e-6) / 1e9, 1),
                               "GFLOP/s": round(wflops / (usw * 1e-6) / 1e9, 1),
                               "per_matrix_launches_us": round(usw1, 1),
                               "one_batch_per_width_us": round(usc, 1)}
    log(f"[bench] mixed widths: {out['mixed_widths_f64']}")
    Bd = torch.from_numpy(np.concatenate([synth.block_vector(A.nrows, b, synth.SEED_Y + 1000 * k)
                                          for k, A in enumerate(mats)])).cuda()

    def solve(name, lo, graph=True):
        for rep in range(2):  # the first run also warms the kernels and tables
            X = torch.zeros_like(Bd)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = sc.sell_batch_cg(B64, lo, Bd, X, tol=tol, maxit=20000, graph=graph)
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t1
        its = [e["iterations"] for e in st]
        out[name] = {"seconds": round(dt_s, 4), "all_converged": all(e["converged"] for e in st),
                     "max_relres": max(e["relres"] for e in st), "iterations_min": min(its),
                     "iterations_max": max(its), "refinements_max": max(e["refinements"] for e in st)}
        log(f"[bench] batch CG {name}: {out[name]}")

    solve("cg_fp64", None)
    solve("cg_mixed_bf16", Bbf)
    solve("cg_mixed_f32", B32)
    solve("cg_mixed_bf16_no_graph", Bbf, graph=False)
    out["speedup_bf16_vs_fp64"] = round(out["cg_fp64"]["seconds"] / out["cg_mixed_bf16"]["seconds"], 3)
    for Bt in (B64, Bbf, B32):
        Bt.close()
    for Ms in M.values():
        for Mk in Ms:
            Mk.close()
    return out


def time_launches(torch, fn, reps=20, warm=3, inner=1):
    """Mean and best duration (us) of fn() with HIP events on the current stream. With inner > 1
    each event pair spans inner back-to-back calls (throughput: one call's host overhead and the
    idle start after a synchronisation are not counted)."""
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(inner):
            fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3 / inner)
    return float(np.mean(ts)), float(np.min(ts))


def other_rows(sc, torch, model, A, Mh, b, s):
    """The path's other operations on the same matrix: low-precision-value products, the
    transposed product, the values-only update and the build, each timed with HIP events."""
    out = {}
    n = A.nrows
    info = Mh.info
    X32 = torch.rand((n, b), dtype=torch.float32, device="cuda") * 2 - 1
    Y32 = torch.rand((n, b), dtype=torch.float32, device="cuda") * 2 - 1
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda")
    flags = sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY | sc.DOT_XY
    for dt, vb in (("bf16", 2), ("f32", 4)):
        Ml = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=dt)
        mean, best = time_launches(torch, lambda: sc.sell_spmmv_aug(Ml, X32, Y32, flags=flags, alpha=2.0 / s,
                                                                     beta=-1.0, dot=dot), reps=10, inner=5)
        by = model.bytes_min(A.nnz, n, n, b, vb, 4, read_y=True, nchunks=info["nchunks"])
        out[f"aug_{dt}_values_f32_vectors"] = {"us": round(mean, 2), "GB/s": round(by / (mean * 1e-6) / 1e9, 1),
                                               "GFLOP/s": round(model.flops(A.nnz, b) / (mean * 1e-6) / 1e9, 1),
                                               "bytes": by}
        Ml.close()
    X64 = torch.rand((n, b), dtype=torch.float64, device="cuda")
    Y64 = torch.empty_like(X64)
    x1 = X64[:, :1].contiguous()
    y1 = torch.empty_like(x1)
    mean, _ = time_launches(torch, lambda: sc.sell_spmmv(Mh, x1, y1))
    spmv_us = mean
    newv = torch.from_numpy(A.val).cuda()
    upd, _ = time_launches(torch, lambda: Mh.update_values(newv))
    out["update_values_device"] = {"us": round(upd, 2), "spmv_equivalents": round(upd / spmv_us, 2)}
    out["plain_spmv_b1_us"] = round(spmv_us, 2)
    by = model.bytes_min(A.nnz, n, n, b, 8, 8, nchunks=info["nchunks"])
    for det in (False, True):
        mean, best = time_launches(torch, lambda: sc.sell_spmmv_T(Mh, X64, Y64, deterministic=det), reps=4,
                                   inner=5)
        out["transpose_" + ("deterministic" if det else "atomic")] = {
            "us": round(mean, 2), "GB/s": round(by / (mean * 1e-6) / 1e9, 1)}
    upd, _ = time_launches(torch, lambda: Mh.update_values(newv))
    out["update_values_device_with_transpose_copy"] = {"us": round(upd, 2),
                                                        "spmv_equivalents": round(upd / spmv_us, 2)}
    # kernel fusion (Sec. 5.3): one KPM step as the fused augmented product, against the plain
    # product followed by separate passes for scale/shift/axpby and the two dots
    Yf = torch.rand((n, b), dtype=torch.float64, device="cuda")
    T = torch.empty_like(Yf)
    dotf = torch.zeros(3 * b, dtype=torch.float64, device="cuda")
    alpha, gamma = 2.0 / s, 0.1
    fl = sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY | sc.DOT_XY
    fused, _ = time_launches(torch, lambda: sc.sell_spmmv_aug(Mh, X64, Yf, flags=fl, alpha=alpha, gamma=gamma,
                                                               beta=-1.0, dot=dotf), reps=10, inner=5)

    def unfused():
        sc.sell_spmmv(Mh, X64, T)
        Yf.mul_(-1.0).add_(T, alpha=alpha).add_(X64, alpha=-alpha * gamma)
        torch.linalg.vecdot(Yf, Yf, dim=0)
        torch.linalg.vecdot(X64, Yf, dim=0)

    unf, _ = time_launches(torch, unfused, reps=10, inner=5)
    # the same step one vector at a time, unfused: the paper's KPM comparison (block vectors
    # together with the augmented product against single-vector steps with separate passes)
    x1u = X64[:, :1].contiguous()
    y1u = torch.rand((n, 1), dtype=torch.float64, device="cuda")
    t1u = torch.empty_like(y1u)

    def unfused_b1():
        sc.sell_spmmv(Mh, x1u, t1u)
        y1u.mul_(-1.0).add_(t1u, alpha=alpha).add_(x1u, alpha=-alpha * gamma)
        torch.linalg.vecdot(y1u, y1u, dim=0)
        torch.linalg.vecdot(x1u, y1u, dim=0)

    unf1, _ = time_launches(torch, unfused_b1, reps=10, inner=5)
    out["fusion_kpm_step_b8"] = {"fused_us": round(fused, 2), "unfused_us": round(unf, 2),
                                 "speedup": round(unf / fused, 2), "unfused_b1_us": round(unf1, 2),
                                 "block_and_fusion_speedup": round(b * unf1 / fused, 2)}
    # Chebyshev filter of degree 100 (the chained axpby): every step one augmented product that
    # also accumulates z, against the same recurrence with a separate z += c v pass per step
    N = 100
    coef = np.random.default_rng(5).normal(size=N + 1) / np.arange(1, N + 2)
    Zf = torch.empty_like(X64)
    chained, _ = time_launches(torch, lambda: sc.sell_cheb_filter(Mh, X64, coef, s, 0.0, Z=Zf), reps=3, warm=1)
    V0, V1 = torch.empty_like(X64), torch.empty_like(X64)

    def separate():
        V0.copy_(X64)
        torch.mul(X64, coef[0], out=Zf)
        sc.sell_spmmv_aug(Mh, V0, V1, flags=sc.SCALE | sc.SHIFT, alpha=1.0 / s, gamma=0.0)
        Zf.add_(V1, alpha=coef[1])
        a, c2 = V0, V1
        for m in range(1, N):
            sc.sell_spmmv_aug(Mh, c2, a, flags=sc.SCALE | sc.SHIFT | sc.AXPBY, alpha=2.0 / s, gamma=0.0, beta=-1.0)
            a, c2 = c2, a
            Zf.add_(c2, alpha=coef[m + 1])

    sep, _ = time_launches(torch, separate, reps=3, warm=1)
    out["cheb_filter_deg100_b8"] = {"chained_us_per_step": round(chained / N, 2),
                                    "separate_axpy_us_per_step": round(sep / N, 2),
                                    "speedup": round(sep / chained, 2)}
    return out


def latency_row(sc, torch, synth):
    """The 64 x 64 Dirichlet Laplacian (n = 4096, 20,224 nonzeros, b = 1, SELL-32-1): time per
    call of the plain product and of the augmented one (alpha = 0.5, gamma = 0.1, beta = 1, <x,y>
    and <y,y>), back to back (HIP events over 100 calls) and one call at a time (host clock
    around a call and a synchronisation)."""
    A = synth.laplacian2d(64)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    x = torch.tensor(synth.block_vector(A.nrows, 1, synth.SEED_X), device="cuda")
    y = torch.tensor(synth.block_vector(A.nrows, 1, synth.SEED_Y), device="cuda")
    dot = torch.zeros(3, dtype=torch.float64, device="cuda")
    fl = sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_XY | sc.DOT_YY
    # the same calls with block-vector views built once and the stream handle passed explicitly
    # (what a caller of the C ABI pays per call, without the binding's per-call descriptors)
    xv, yv = sc.BlockVector.view(x), sc.BlockVector.view(y)
    st = torch.cuda.current_stream().cuda_stream
    calls = {"plain": lambda: sc.sell_spmmv(M, x, y),
             "augmented": lambda: sc.sell_spmmv_aug(M, x, y, flags=fl, alpha=0.5, gamma=0.1, beta=1.0, dot=dot),
             "plain_prebuilt_views": lambda: sc.sell_spmmv(M, xv, yv, stream=st)}
    out = {"matrix": "2D 5-point Dirichlet Laplacian 64x64", "n": A.nrows, "nnz": A.nnz, "b": 1}
    for name, fn in calls.items():
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(100):
            fn()
        e1.record()
        e1.synchronize()
        back_to_back = e0.elapsed_time(e1) * 1e3 / 100
        ts = []
        for _ in range(100):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out[name] = {"us_back_to_back": round(back_to_back, 2), "us_synchronous_median": round(
            float(np.median(ts)) * 1e6, 1)}
    xv.close()
    yv.close()
    M.close()
    return out


def device_build_row(sc, torch, A, C, sigma, spmv_us):
    """Construction on the GPU from a device-resident CSR (mean of 3 after one warm-up), in
    seconds and in units of one plain SpMV (b = 1)."""
    rp = torch.from_numpy(A.rowptr).cuda()
    co = torch.from_numpy(A.col).cuda()
    va = torch.from_numpy(A.val).cuda()
    ts = []
    for rep in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, co, va, C=C, sigma=sigma)
        ts.append(time.perf_counter() - t0)
        M.close()
    t = float(np.mean(ts[1:]))
    return {"seconds": round(t, 5), "spmv_equivalents": round(t * 1e6 / spmv_us, 1)}


def grad_row(sc, torch, synth):
    """Differentiation workload: loss = sum(T_100(A~(theta)) x)^2 on the 64^3 Anderson
    matrix, checkpoints every 10 steps; forward + backward time with HIP events."""
    from paper_1507_08101_amd.autograd import chebyshev

    A = synth.anderson3d(64)
    s = (6.0 + W_DISORDER / 2) / 0.99
    out = {"matrix": "3D periodic Anderson 64^3", "n": A.nrows, "nnz": A.nnz, "degree": 100, "checkpoint_every": 10}
    for dt, vt in (("f64", torch.float64), ("f32", torch.float32)):
        M = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=dt)
        theta = torch.tensor(A.val, dtype=torch.float64, device="cuda", requires_grad=True)
        X = torch.tensor(synth.block_vector(A.nrows, 1, synth.SEED_X), dtype=vt, device="cuda")

        def step():
            theta.grad = None
            Y = chebyshev(theta, X, M, 100, s, 0.0, 10)
            (Y.double() ** 2).sum().backward()

        mean, _ = time_launches(torch, step, reps=5, warm=2)
        out[dt + "_forward_backward_ms"] = round(mean / 1e3, 3)
        M.close()
    return out


def tsm_row(sc, torch, n=1 << 22, m=8, k=8):
    """Tall-skinny block kernels on n x m / n x k FP64 blocks (the block-Krylov building blocks):
    time with HIP events and the bytes each must move (n (m + k) 8; in place 2 n m 8)."""
    V = torch.rand((n, m), dtype=torch.float64, device="cuda")
    W = torch.rand((n, k), dtype=torch.float64, device="cuda")
    X = torch.rand((m, k), dtype=torch.float64, device="cuda")
    Xs = torch.rand((m, m), dtype=torch.float64, device="cuda")
    out = {"n": n, "m": m, "k": k}
    rows = [("tsmttsm", lambda: sc.sell_tsmttsm(V, W, X), n * (m + k) * 8),
            ("tsmttsm_kahan", lambda: sc.sell_tsmttsm(V, W, X, kahan=True), n * (m + k) * 8),
            ("tsmm", lambda: sc.sell_tsmm(V, X, W, beta=0.5), n * (m + 2 * k) * 8),
            ("tsmm_inplace", lambda: sc.sell_tsmm_inplace(V, Xs, beta=0.5), 2 * n * m * 8)]
    for name, fn, by in rows:
        us, _ = time_launches(torch, fn, reps=10, inner=5)
        out[name] = {"us": round(us, 1), "GB/s": round(by / (us * 1e-6) / 1e9, 1)}
    return out


def irregular_row(sc, torch, synth, model, n=4_000_000, C=32, probes=None):
    """The irregular matrix (lognormal row lengths, mean 15, half banded / half uniform
    columns): plain products y = A X for every sorting window, value type and block width,
    with algorithmic (true nonzeros) and SELL (stored entries, padding included) GB/s.
    SELL-C-sigma is built on the device from a device CSR. At b = 8, FP64, the row-major
    templated kernel is compared with column-major vectors and with rows whose leading
    dimension b + 1 breaks the 16-byte alignment (both run the run-time-width kernel)."""
    t0 = time.perf_counter()
    A = synth.irregular(n)
    out = {"matrix": "irregular, lognormal row lengths (mean 15, clip 1..2000), half +-5000 band, half uniform",
           "n": A.nrows, "nnz": A.nnz, "C": C, "generate_s": round(time.perf_counter() - t0, 1)}
    rp = torch.from_numpy(A.rowptr).cuda()
    co = torch.from_numpy(A.col).cuda()
    va = torch.from_numpy(A.val).cuda()
    widths = (1, 4, 8, 16, 32)
    res = {}
    for dt, vb in (("f64", 8), ("f32", 4), ("bf16", 2)):
        xs = 8 if dt == "f64" else 4
        vt = torch.float64 if dt == "f64" else torch.float32
        res[dt] = {}
        for sg in (1, 32, 1024, A.nrows):
            M = sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, co, va, C=C, sigma=sg, dtype=dt)
            info = M.info
            row = {"stored_over_nnz": round(info["stored"] / A.nnz, 3)}
            for b in widths:
                X = torch.rand((A.ncols, b), dtype=vt, device="cuda")
                Y = torch.empty((A.nrows, b), dtype=vt, device="cuda")
                us, _ = time_launches(torch, lambda: sc.sell_spmmv(M, X, Y), reps=4, inner=5)
                bmin = model.bytes_min(A.nnz, A.nrows, A.ncols, b, vb, xs, nchunks=info["nchunks"],
                                       has_perm=sg > 1)
                bsell = model.bytes_sell(info["stored"], A.nrows, A.ncols, b, vb, xs, nchunks=info["nchunks"],
                                         has_perm=sg > 1)
                row[f"b{b}"] = {"us": round(us, 1), "GFLOP/s": round(model.flops(A.nnz, b) / (us * 1e-6) / 1e9, 1),
                                "GB/s": round(bmin / (us * 1e-6) / 1e9, 1),
                                "GB/s_sell": round(bsell / (us * 1e-6) / 1e9, 1)}
                del X, Y
            if dt == "f64" and sg == 1024:
                b = 8
                bmin = model.bytes_min(A.nnz, A.nrows, A.ncols, b, 8, 8, nchunks=info["nchunks"], has_perm=True)
                lay = {"row_major_templated_us": row["b8"]["us"]}
                Xc = torch.rand((b, A.ncols), dtype=torch.float64, device="cuda").T
                Yc = torch.empty((b, A.nrows), dtype=torch.float64, device="cuda").T
                us, _ = time_launches(torch, lambda: sc.sell_spmmv(M, Xc, Yc), reps=4, inner=5)
                lay["col_major_us"] = round(us, 1)
                lay["col_major_GB/s"] = round(bmin / (us * 1e-6) / 1e9, 1)
                del Xc, Yc
                Xp = torch.rand((A.ncols, b + 1), dtype=torch.float64, device="cuda")[:, :b]
                Yp = torch.empty((A.nrows, b + 1), dtype=torch.float64, device="cuda")[:, :b]
                us, _ = time_launches(torch, lambda: sc.sell_spmmv(M, Xp, Yp), reps=4, inner=5)
                lay["row_major_ld9_runtime_width_us"] = round(us, 1)
                lay["row_major_ld9_runtime_width_GB/s"] = round(bmin / (us * 1e-6) / 1e9, 1)
                del Xp, Yp
                out["layouts_f64_b8_sigma1024"] = lay
            M.close()
            res[dt]["sigma_n" if sg == A.nrows else f"sigma_{sg}"] = row
            log(f"[bench] irregular {dt} sigma={sg}: {row}")
    out["products"] = res
    # achievable rate of scattered row gathers (the library's gather probe): as many uniform
    # random rows as the matrix has uniform columns (half its nonzeros), and as many as nonzeros,
    # for rows of 8 to 256 bytes (b FP64 or FP32 values per row)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_X)
    idx = torch.randint(0, A.ncols, (A.nnz,), dtype=torch.int32, device="cuda", generator=gen)
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    probe = {}
    gather_us = {}
    for rb in (8, 16, 32, 64, 128, 256):
        x = torch.rand((A.ncols, rb // 8), dtype=torch.float64, device="cuda")
        for name, cnt in (("half_nnz", A.nnz // 2), ("nnz", A.nnz)):
            ix = idx[:cnt]
            # five back-to-back launches per timed call (a single call's host overhead would count)
            us, _ = time_launches(torch, lambda: sc.sell_probe_gather(x, ix, sink), reps=4, inner=5)
            probe[f"row{rb}B_{name}"] = {"gathers": cnt, "us": round(us, 1), "Ggathers/s": round(cnt / us / 1e3, 2)}
            if name == "half_nnz":
                gather_us[rb] = us
        del x
    out["gather_probe"] = probe
    log(f"[bench] gather probe: {probe}")
    # floor of each product: the uniform half's gathers at the probe's rate (rows of b x-element
    # bytes, at least 8), the banded half taken as free (L2 hits), plus the matrix stream at
    # the read probe's rate and y at the write probe's rate; ratio = measured / floor
    if probes:
        rd, wr = probes["read"]["GB/s"] * 1e3, probes["write"]["GB/s"] * 1e3  # bytes per us
        for dt, vb in (("f64", 8), ("f32", 4), ("bf16", 2)):
            xs = 8 if dt == "f64" else 4
            for key, row in res[dt].items():
                stored = row["stored_over_nnz"] * A.nnz
                for b in widths:
                    rb = max(8, b * xs)
                    t = gather_us[rb] + (stored * (vb + 4) + 4 * A.nrows) / rd + A.nrows * b * xs / wr
                    row[f"b{b}"]["floor_us"] = round(t, 1)
                    row[f"b{b}"]["over_floor"] = round(row[f"b{b}"]["us"] / t, 2)
    # the autotuner on this matrix at b = 32, FP64: (C, sigma), launch shape and slice width
    t0 = time.perf_counter()
    tune = sc.sell_autotune(A, 32, "f64", cache=False)
    out["autotune_f64_b32"] = {k: (round(v, 1) if isinstance(v, float) else v) for k, v in tune.items()}
    out["autotune_f64_b32"]["seconds"] = round(time.perf_counter() - t0, 1)
    log(f"[bench] irregular autotune b=32: {out['autotune_f64_b32']}")
    del rp, co, va, idx
    torch.cuda.empty_cache()
    return out


def cpu_baseline(oracle, synth, A, b, s, target_s=15.0):
    """The oracle's augmented product (one KPM step) on the host cores, bounded sample; returns
    the baseline and the oracle's output of the first call (for the parity figure)."""
    X = synth.block_vector(A.nrows, b, synth.SEED_X)
    Y = synth.block_vector(A.nrows, b, synth.SEED_Y)
    flags = oracle.SCALE | oracle.SHIFT | oracle.AXPBY | oracle.DOT_YY | oracle.DOT_XY
    calls = 0
    first = None
    t0 = time.perf_counter()
    while True:
        r = oracle.spmmv_aug(A, X, Y=Y, flags=flags, alpha=2.0 / s, beta=-1.0, gamma=0.0)
        if first is None:
            first = r
        calls += 1
        el = time.perf_counter() - t0
        if el >= target_s or calls >= 200:
            break
    gf = calls * 2 * A.nnz * b / el / 1e9
    cores = oracle.num_threads()
    # the oracle's plain product alone (its parallel part), to state how much of the augmented
    # call is the serial epilogue (shift, scale, axpby, Neumaier dots) and the wrapper's copy of y
    cp, tp = 0, time.perf_counter()
    while True:
        oracle.spmmv(A, X)
        cp += 1
        ep = time.perf_counter() - tp
        if ep >= target_s / 3 or cp >= 100:
            break
    # CSR byte model of one call: each nonzero's value and column once, the row pointers,
    # x read, y read and written
    csr_bytes = A.nnz * 12 + 8 * (A.nrows + 1) + 3 * A.nrows * b * 8
    t_aug, t_plain = el / calls, ep / cp
    out = {"value": gf, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"{calls} augmented products (one KPM step each, b={b}) on the full "
                     f"{A.name} matrix, {el:.1f} s",
           "what": "the oracle as it stands, not tuned: an OpenMP CSR product followed by a serial "
                   "epilogue (shift, scale, axpby, Neumaier-compensated dots) and a copy of y in its "
                   "Python wrapper; a large GPU/CPU ratio says nothing about the kernel",
           "plain_product": {"value": round(cp * 2 * A.nnz * b / ep / 1e9, 3), "unit": "GFLOP/s",
                             "sample": f"{cp} plain products (oracle.spmmv, same threads), {ep:.1f} s"},
           "serial_share": round(max(0.0, (t_aug - t_plain) / t_aug), 3),
           "gbs_csr_model": round(calls * csr_bytes / el / 1e9, 2), "cpu": host_cpu_model()}
    # the same on one core (a shorter sample), and the host's STREAM triad on all cores
    oracle.set_num_threads(1)
    try:
        c1, t1 = 0, time.perf_counter()
        while True:
            oracle.spmmv_aug(A, X, Y=Y, flags=flags, alpha=2.0 / s, beta=-1.0, gamma=0.0)
            c1 += 1
            e1 = time.perf_counter() - t1
            if e1 >= target_s / 4 or c1 >= 50:
                break
    finally:
        oracle.set_num_threads(cores)
    out["one_core"] = {"value": round(c1 * 2 * A.nnz * b / e1 / 1e9, 3), "unit": "GFLOP/s",
                       "sample": f"{c1} products, {e1:.1f} s"}
    out["host_triad_gbs"] = round(host_triad_gbs(oracle), 1)
    return out, (X, Y, first)


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_triad_gbs(oracle, n=1 << 27, reps=5):
    """Best STREAM triad rate (3 x 8 bytes per element, 1 GiB arrays) on the oracle's threads."""
    a, b, c = np.zeros(n), np.ones(n), np.full(n, 2.0)
    oracle.triad(a, b, c, 3.0)  # first touch
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.triad(a, b, c, 3.0)
        best = min(best, time.perf_counter() - t0)
    return 3 * 8 * n / best / 1e9


def parity_row(sc, torch, A, Mh, b, s, ref):
    """The timed product (one KPM step: alpha = 2/s, beta = -1, <y,y> and <x,y>) on the full
    matrix against the oracle's result on the same inputs: the largest per-column normwise
    relative error of y and the largest relative error of the dots."""
    X, Y, (Yr, _, dr) = ref
    Yd = torch.from_numpy(Y).cuda()
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda")
    sc.sell_spmmv_aug(Mh, torch.from_numpy(X).cuda(), Yd, flags=sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY
                      | sc.DOT_XY, alpha=2.0 / s, beta=-1.0, gamma=0.0, dot=dot)
    Yg = Yd.cpu().numpy()
    dg = dot.cpu().numpy()
    err = np.linalg.norm(Yg - Yr, axis=0) / np.linalg.norm(Yr, axis=0)
    derr = np.abs(dg[:2 * b] - dr[:2 * b]) / np.abs(dr[:2 * b])
    return {"y_max_colwise_relerr": float(err.max()), "dots_max_relerr": float(derr.max()),
            "what": f"one augmented product of the benchmark, b={b}, full matrix, against the FP64 oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--M", type=int, default=200)
    ap.add_argument("--b", type=int, default=8)
    ap.add_argument("--C", type=int, default=32)
    ap.add_argument("--sigma", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--no-b1", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the low-precision/transpose/update timings")
    ap.add_argument("--cg-edge", type=int, default=100)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched Laplacian workload")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--no-irregular", action="store_true", help="skip the 4M-row irregular matrix sweep")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one copy probe of this many MiB (calibrates HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not offered (the sharded design is "
              f"described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1507_08101_amd as sc
    import synth
    from paper_1507_08101_amd import model

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        sc.sell_probe_bandwidth(0, b, a, nbytes)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes}), flush=True)
        return
    log(f"[bench] device {torch.cuda.get_device_name(0)}")

    t0 = time.perf_counter()
    A = synth.anderson3d(args.L, W=W_DISORDER)
    log(f"[bench] generated {A} in {time.perf_counter() - t0:.1f} s")
    s = (6.0 + W_DISORDER / 2) / 0.99  # Gershgorin bound with 1 % margin
    t0 = time.perf_counter()
    Mh = sc.SellMatrix.from_csr(A, C=args.C, sigma=args.sigma, dtype="f64")
    # index batch length of the timed kernel (FP64 at b >= 4 gathers 32 bytes per lane)
    kern_batch = Mh.info["batch_wide"] if args.b >= 4 else Mh.info["batch"]
    build_s = time.perf_counter() - t0
    info = Mh.info
    log(f"[bench] SELL-{args.C}-{args.sigma} build+upload {build_s:.2f} s, stored {info['stored']}")

    results = {}
    widths = [args.b] + ([] if args.no_b1 or args.b == 1 else [1])
    for b in widths:
        V0 = synth.block_vector(A.nrows, b, synth.SEED_X)
        V0d = torch.from_numpy(V0).cuda()
        steps = args.steps if b == args.b else max(2, args.steps // 2)
        step_ms, launch_ms, mu = kpm_run(sc, torch, Mh, V0d, b, args.M, s, steps, args.warmup)
        flops_step = args.M * model.flops(A.nnz, b)
        # algorithmic bytes: first product writes y only, the others read and write y
        b0 = model.bytes_min(A.nnz, A.nrows, A.ncols, b, 8, 8, read_y=False, nchunks=info["nchunks"])
        b1 = model.bytes_min(A.nnz, A.nrows, A.ncols, b, 8, 8, read_y=True, nchunks=info["nchunks"])
        bytes_launch = (b0 + (args.M - 1) * b1) / args.M
        launch_avg_ms = float(np.mean(launch_ms))
        dos = None
        if b == args.b:
            # density of states from the block moments (Jackson damping) on 2001 energies
            Ed = torch.linspace(-s, s, 2001, dtype=torch.float64, device="cuda")
            us_dos, _ = time_launches(torch, lambda: sc.sell_kpm_dos(mu, b, Ed, s, 0.0), reps=5)
            rho = sc.sell_kpm_dos(mu, b, Ed, s, 0.0).cpu().numpy()
            Eh = Ed.cpu().numpy()
            dos = {"energies": int(Ed.numel()), "moments": 2 * args.M + 1, "kernel": "jackson", "us": round(us_dos, 1),
                   "integral": round(float(np.sum(0.5 * (rho[1:] + rho[:-1]) * np.diff(Eh))), 4),
                   "rho_at_0": round(float(rho[1000]), 5)}
        results[b] = dict(
            dos=dos,
            ms_per_step=float(np.mean(step_ms)),
            gflops=flops_step / (float(np.mean(step_ms)) * 1e-3) / 1e9,
            gflops_pmax=flops_step / (float(np.min(step_ms)) * 1e-3) / 1e9,
            launch_avg_us=launch_avg_ms * 1e3,
            launch_min_us=float(np.min(launch_ms)) * 1e3,
            bytes_per_launch=bytes_launch,
            hbm_gbs=bytes_launch / (launch_avg_ms * 1e-3) / 1e9,
            mu0=float(mu[0].item()), steps=steps)
        log(f"[bench] b={b}: {results[b]['ms_per_step']:.3f} ms/step, {results[b]['gflops']:.1f} GFLOP/s, "
            f"launch {results[b]['launch_avg_us']:.1f} us, {results[b]['hbm_gbs']:.0f} GB/s")
        del V0d

    head = results[args.b]
    extra = None
    if not args.no_other:
        extra = other_rows(sc, torch, model, A, Mh, args.b, s)
        extra["build_spmv_equivalents"] = round(build_s * 1e6 / extra["plain_spmv_b1_us"], 1)
        extra["build_device"] = device_build_row(sc, torch, A, args.C, args.sigma, extra["plain_spmv_b1_us"])
        extra["grad_chebyshev"] = grad_row(sc, torch, synth)
        extra["tall_skinny"] = tsm_row(sc, torch)
        extra["latency_laplacian64"] = latency_row(sc, torch, synth)
        log(f"[bench] other rows: {json.dumps(extra)}")
    probes = None if args.no_probe else probe_bandwidth(sc, torch)
    ach = None
    if probes:
        log(f"[bench] probes GB/s: {probes}")
        # the timed kernel's algorithmic reads and writes (the first product does not read y)
        wr = A.nrows * args.b * 8
        rd = head["bytes_per_launch"] - wr
        pname, pgbs, tmodel = achievable_for_mix(probes, rd, wr)
        ach = {"kernel_read_bytes": int(rd), "kernel_write_bytes": int(wr), "probe": pname,
               "probe_GB/s": pgbs, "time_model_GB/s": round(tmodel, 1),
               "frac_of_time_model": round(head["hbm_gbs"] / tmodel, 4)}
        log(f"[bench] achievable for the kernel's mix: {ach}")
    cg = None
    if not args.no_cg:
        try:
            cg = cg_compare(sc, torch, synth, args.cg_edge)
            log(f"[bench] CG: {json.dumps(cg)}")
        except sc.SellError as e:
            cg = {"error": str(e)}
            log(f"[bench] CG skipped: {e}")
    batch = None
    if not args.no_batch:
        batch = batch_row(sc, torch, synth, model, nmat=args.batch_count)
    irregular = None
    if not args.no_irregular:
        irregular = irregular_row(sc, torch, synth, model, probes=probes)
    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle

        cpu, ref = cpu_baseline(oracle, synth, A, args.b, s)
        log(f"[bench] cpu baseline: {cpu}")
        parity = parity_row(sc, torch, A, Mh, args.b, s, ref)
        log(f"[bench] parity against the oracle: {parity}")
        if not args.no_cg:
            cg_ref = cg_reference_row(sc, torch, synth, oracle)
            log(f"[bench] CG iteration counts beside the oracle's: {cg_ref}")
            if cg is not None and "error" not in cg:
                cg["reference_iterations"] = cg_ref

    src_hash = kernel_source_hash()
    traffic = load_traffic(f"traffic_anderson{args.L}_b{args.b}.json", src_hash)
    frac = head["hbm_gbs"] / HBM_PEAK_GBS
    line = {
        "metric": "SpMMV GFLOP/s and HBM GB/s (% of peak) FP64 vs BF16-value+refine, 1 MI355X",
        "value": round(head["gflops"], 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded 3D Anderson Hamiltonian, block vector U[-1,1])",
        "config": {"workload": f"KPM recurrence, {args.M} augmented SpMMVs with fused dots, 3D periodic "
                               f"Anderson {args.L}^3 (n={A.nrows}, nnz={A.nnz}), SELL-{args.C}-{args.sigma}",
                   "n": A.nrows, "nnz": A.nnz, "b": args.b, "C": args.C, "sigma": args.sigma,
                   "kpm_steps": args.M},
        "kpm_dos": head.get("dos"),
        "roofline": {"bound": "hbm", "achieved": round(head["hbm_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(frac, 4), "traffic": traffic,
                     "kernel": f"prod_kernel (FP64 values and vectors, b={args.b}, augmented, fused dots, "
                               f"{kern_batch}-entry index batches, the KPM step's flags fixed at compile time, "
                               f"the diagonal entry from the row's own x)",
                     "bytes_per_launch": int(head["bytes_per_launch"]),
                     "launch_avg_us": round(head["launch_avg_us"], 2)},
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "hbm_gbs": round(head["hbm_gbs"], 1),
        "pmax_gflops": round(head["gflops_pmax"], 2),
        "b1": None if 1 not in results or args.b == 1 else {k: (round(v, 3) if isinstance(v, float) else v)
                                                            for k, v in results[1].items() if k != "dos"},
        "achievable_gbs": probes,
        "achievable_for_kernel_mix": ach,
        "frac_of_achievable": None if not ach else round(head["hbm_gbs"] / ach["probe_GB/s"], 4),
        "cg_time_to_1e-10": cg,
        "other_rows_b8": extra,
        "batch_laplacians": batch,
        "irregular_4M": irregular,
        "build_s": round(build_s, 3),
        "kernel_source_hash": src_hash,
    }
    print(json.dumps(line), flush=True)
    Mh.close()


if __name__ == "__main__":
    main()
