"""Short text summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_1505_08115_amd.prof_summary stats KERNEL_STATS_CSV \
        --factorizations F --command "..."
    python -m paper_1505_08115_amd.prof_summary pmc FETCH_CSV WRITE_CSV \
        --factorizations F --command-fetch "..." --command-write "..."

`stats` keeps the library's kernels (namespace rq::) of a
`--kernel-trace --stats` run and reports calls, total and average time per
factorization.  `pmc` reads two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
counter runs (KiB per dispatch), scales each counter by what it reads for the
calibration kernel (the driver's calib_copy_kernel over 2^26 doubles: 2^29
bytes read, 2^29 bytes written), and reports the HBM bytes per W = V^T C
launch (the product kernel and its split-K sum) next to the algorithmic bytes
8 (m_i n_c + b m_i + b n_c) of each launch (n_c = n_i - b).
"""
import argparse
import csv
import hashlib
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEMM_SOURCES = ("paper_1505_08115_amd/csrc/gemm.hip",)   # the file that defines the GEMM kernels
# kernels tagged 2 (W = V^T C): the all-rows or tiled product and the split-K sum
WMAIN = re.compile(r"(gemm_rows_kernel<double, \d+, false, (true|false), 2>|gemm_kernel<double, \d+, \d+, false, false, (true|false), 2>)")
WSUM = re.compile(r"reduce_partials_kernel<double, 2>")
CALIB = "calib_copy_kernel"
CALIB_BYTES = 1 << 29


def gemm_source_hash():
    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short(name, width=96):
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"\(.*\)$", "", name)
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    mine = [r for r in rows if "rq::" in r["Name"]]
    total = sum(float(r["TotalDurationNs"]) for r in mine)
    f = args.factorizations
    out = [f"# rocprofv3 kernel statistics, library kernels only ({f} factorizations profiled)",
           f"command: {args.command}", "",
           f"{'kernel':96s} {'calls/fact':>10s} {'ms/fact':>9s} {'avg us':>10s} {'share':>6s}"]
    for r in sorted(mine, key=lambda r: -float(r["TotalDurationNs"])):
        t = float(r["TotalDurationNs"])
        out.append(f"{short(r['Name']):96s} {int(r['Calls']) / f:10.1f} {t / f / 1e6:9.3f} "
                   f"{float(r['AverageNs']) / 1e3:10.1f} {100 * t / total:5.1f}%")
    out.append(f"{'total (library kernels)':96s} {'':10s} {total / f / 1e6:9.3f}")
    print("\n".join(out))


def _counter_rows(path, counter):
    rows = list(csv.DictReader(open(path)))
    return [r for r in rows if r.get("Counter_Name", "").startswith(counter)]


def pmc(args):
    f = args.factorizations
    res = {}
    for path, counter in ((args.fetch, "FETCH_SIZE"), (args.write, "WRITE_SIZE")):
        rows = _counter_rows(path, counter)
        by = {}
        for r in rows:   # one value per dispatch (summed if split by dimension)
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            by[key] = by.get(key, 0.0) + float(r["Counter_Value"])
        cal = [v for (d, k), v in by.items() if CALIB in k]
        wmain = [v for (d, k), v in by.items() if WMAIN.search(k)]
        wsum = [v for (d, k), v in by.items() if WSUM.search(k)]
        if not cal or not wmain:
            sys.exit(f"{path}: calibration or W-product dispatches missing")
        scale = CALIB_BYTES / (cal[-1] * 1024.0)
        res[counter] = (cal[-1], scale, len(wmain), sum(wmain) + sum(wsum))
    n_tr = res["FETCH_SIZE"][2]
    fetch_b = res["FETCH_SIZE"][3] * 1024.0 * res["FETCH_SIZE"][1]
    write_b = res["WRITE_SIZE"][3] * 1024.0 * res["WRITE_SIZE"][1]
    # algorithmic bytes of the W products of one factorization (m = n = 8192, b = 256)
    m = n = args.n
    b = args.block
    alg = 0.0
    launches = 0
    for i in range((n + b - 1) // b):
        mi, ni = m - i * b, n - i * b
        bi = min(b, ni)
        nc = ni - bi
        if nc <= 0:
            continue
        alg += 8.0 * (mi * nc + mi * bi + bi * nc)
        launches += 1
    per_launch = (fetch_b + write_b) / n_tr
    out = ["# rocprofv3 HBM counters, W = V^T C (product + split-K sum) at the H1 shape (8192^2, b=256, p=10, FP64)",
           f"command (fetch): {args.command_fetch}",
           f"command (write): {args.command_write}",
           f"calibration kernel: {CALIB} over 2^26 doubles ({CALIB_BYTES} B read, {CALIB_BYTES} B written)",
           f"calibration FETCH_SIZE KiB: {res['FETCH_SIZE'][0]:.0f}",
           f"calibration WRITE_SIZE KiB: {res['WRITE_SIZE'][0]:.0f}",
           f"scale_fetch: {res['FETCH_SIZE'][1]:.4f}",
           f"scale_write: {res['WRITE_SIZE'][1]:.4f}",
           f"W launches: {n_tr} ({n_tr / f:.0f} per factorization)",
           f"fetch_bytes_per_launch (scaled): {fetch_b / n_tr:.4e}",
           f"write_bytes_per_launch (scaled): {write_b / n_tr:.4e}",
           f"traffic_bytes_per_launch: {per_launch:.6e}",
           f"algorithmic_bytes_per_launch: {alg / launches:.6e}",
           f"traffic / algorithmic: {per_launch / (alg / launches):.3f}",
           f"gemm_source_sha256: {gemm_source_hash()}"]
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--factorizations", type=int, required=True)
    s.add_argument("--command", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("fetch")
    p.add_argument("write")
    p.add_argument("--factorizations", type=int, required=True)
    p.add_argument("--command-fetch", required=True)
    p.add_argument("--command-write", required=True)
    p.add_argument("--n", type=int, default=8192)
    p.add_argument("--block", type=int, default=256)
    a = ap.parse_args()
    stats(a) if a.mode == "stats" else pmc(a)


if __name__ == "__main__":
    main()
