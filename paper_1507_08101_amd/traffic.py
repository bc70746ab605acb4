"""HBM traffic per launch of a kernel from rocprofv3 counter runs.

Four runs of ``rocprofv3 --pmc <counter> --output-format csv`` are needed: FETCH_SIZE and
WRITE_SIZE over the workload, and the same two counters over the library's copy probe of a
known size (``bench.py --copy-probe-mib N``), whose readings calibrate the counters (bytes per
counted KiB). The result is written as JSON; ``bench.py`` reports it while the kernel sources
still have the hash recorded in it.

    python -m paper_1507_08101_amd.traffic --kernel 'prod_kernel<0, 8, 4, true, 7>' \\
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --copy-mib 1024 \\
        --steps 200 --algorithmic-bytes B --hash H --out profiles/traffic_....json
"""
import argparse
import csv
import glob
import json
import os


def _rows(d, counter):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    out.sort()
    return out


def kernel_kib(d, counter, kernel):
    """Counter values (KiB) of the dispatches of kernels whose name contains ``kernel``."""
    return [v for _, name, v in _rows(d, counter) if kernel in name]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--steps", type=int, default=0,
                    help="products of the recurrence: the first one (y not read) gets weight 1/steps")
    ap.add_argument("--algorithmic-bytes", type=float, required=True)
    ap.add_argument("--hash", required=True, help="kernel source hash of bench.py")
    ap.add_argument("--what", default="")
    ap.add_argument("--commands", nargs="*", default=[])
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    nbytes = a.copy_mib << 20
    cf = kernel_kib(a.copy_fetch, "FETCH_SIZE", "probe")
    cw = kernel_kib(a.copy_write, "WRITE_SIZE", "probe")
    if not cf or not cw:
        raise SystemExit("no probe dispatch in the copy runs")
    fetch_scale = nbytes / (cf[-1] * 1024.0)
    write_scale = nbytes / (cw[-1] * 1024.0)
    f = kernel_kib(a.fetch, "FETCH_SIZE", a.kernel)
    w = kernel_kib(a.write, "WRITE_SIZE", a.kernel)
    if not f or not w:
        raise SystemExit(f"no dispatch of {a.kernel!r}")

    def per_launch(vals):
        # the first dispatch of a recurrence has beta = 0; weight it as the benchmark does
        if a.steps > 1 and len(vals) > 1:
            rest = sum(vals[1:]) / (len(vals) - 1)
            return (vals[0] + (a.steps - 1) * rest) / a.steps, vals[0], rest
        m = sum(vals) / len(vals)
        return m, vals[0], m

    fk, f0, fr = per_launch(f)
    wk, w0, wr = per_launch(w)
    rd = fk * 1024.0 * fetch_scale
    wb = wk * 1024.0 * write_scale
    res = {
        "what": a.what,
        "commands": a.commands,
        "copy_probe": {"bytes_read": nbytes, "bytes_written": nbytes, "FETCH_SIZE_KiB": cf[-1],
                       "WRITE_SIZE_KiB": cw[-1], "fetch_scale": fetch_scale, "write_scale": write_scale},
        "kernel_KiB_per_dispatch": {"FETCH_SIZE_first": f0, "FETCH_SIZE_rest_mean": fr, "WRITE_SIZE_first": w0,
                                    "WRITE_SIZE_rest_mean": wr, "dispatches": len(f)},
        "read_bytes_per_launch": rd,
        "write_bytes_per_launch": wb,
        "traffic_bytes_per_launch": rd + wb,
        "algorithmic_bytes_per_launch": a.algorithmic_bytes,
        "traffic_over_algorithmic": (rd + wb) / a.algorithmic_bytes,
        "kernel_source_hash": a.hash,
    }
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
