"""HBM traffic of the product's kernels from rocprofv3 counters.

    run [leaf]
            one FP64 and one FP32 product of the 1M-point mixture with the
            tuned level orders and leaf capacity `leaf` (default 48), stage by
            stage (each kernel alone on the stream), then a device-to-device
            copy of 256 MiB: the calibration, whose bytes are known
    stats   mean duration per (kernel, grid) from a rocprofv3 kernel trace
            (CSV), to read one configuration's launches apart from others
    counters  every counter of the dispatches of one kernel from a --pmc run
    report  from two rocprofv3 --pmc databases of `run` (FETCH_SIZE, then
            WRITE_SIZE; KiB per dispatch) and the leaf capacity of the run, the
            bytes per launch of the near-field, translation, P2M and L2P
            kernels, each counter scaled by what it reads for the copy (2^28
            bytes read, 2^28 written), printed as the table rows the benchmark
            looks up (kernel, workload, leaf, precision, SHA-256 prefix of the
            kernel's source, bytes)

Usage (REPO = the repository root):
    rocprofv3 --pmc FETCH_SIZE -d OUT1 -o run -- python3 REPO/paper_2205_04194_amd/traffic_probe.py run 64
    rocprofv3 --pmc WRITE_SIZE -d OUT2 -o run -- python3 REPO/paper_2205_04194_amd/traffic_probe.py run 64
    python3 REPO/paper_2205_04194_amd/traffic_probe.py report OUT1/.../run_results.db OUT2/.../run_results.db 64
    python3 REPO/paper_2205_04194_amd/traffic_probe.py stats OUT/.../run_kernel_trace.csv
    python3 REPO/paper_2205_04194_amd/traffic_probe.py counters OUT/.../run_results.db 'k_p2p<double'
"""
from __future__ import annotations

import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 28
ORDERS = [11, 11, 11, 11, 11, 11, 8, 6, 6, 4, 4]   # the tuned FP64 orders of the benchmark
LEAF = 48

# kernel key -> (name pattern of the stage-timed launch, source file)
KERNELS = {
    "p2p": (r"k_p2p<{t}, false", "p2p.hip"),
    "m2l": (r"k_m2l_stream<{t},", "m2l.hip"),
    "p2m": (r"k_p2m(_pipe)?<{t},", "fmm.hip"),
    "l2p": (r"k_l2p(_pipe)?<{t},", "fmm.hip"),
}


def run(leaf: int = LEAF) -> None:
    import torch
    sys.path.insert(0, ROOT)
    import workloads as W
    import paper_2205_04194_amd as imq
    d = W.mixture1m()
    dev = torch.device("cuda:0")
    tree = imq.build_tree(torch.tensor(d["xy"], device=dev), d["c"], leaf=leaf, p=max(ORDERS))
    tree.set_level_orders(ORDERS[:tree.info()["nlevels"]])
    tree.set_stage_timing(True)                 # every stage alone, in order, on one stream
    for prec in ("fp64", "fp32"):
        u = torch.tensor(d["u"], device=dev)
        tree.matvec(u, prec)
        torch.cuda.synchronize()
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    tree.close()
    print("traffic probe done", flush=True)


def _dispatches(db: str, counter: str):
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection "
                       "order by dispatch_id").fetchall()
    out = {}
    for did, name, cn, v in rows:
        if cn.startswith(counter):
            e = out.setdefault(did, [name, 0.0])
            e[1] += float(v)
    return [tuple(v) for _, v in sorted(out.items())]


def report(db_fetch: str, db_write: str, leaf: int = LEAF) -> None:
    f = _dispatches(db_fetch, "FETCH_SIZE")
    w = _dispatches(db_write, "WRITE_SIZE")
    # the calibration copy: the last dispatch of each run
    fk, wk = f[-1][1] * 1024.0, w[-1][1] * 1024.0
    sf, sw = COPY_BYTES / fk, COPY_BYTES / wk
    print(f"calibration copy {f[-1][0][:60]}: FETCH {fk / 2**20:.1f} MiB, WRITE {wk / 2**20:.1f} MiB "
          f"for {COPY_BYTES / 2**20:.0f} MiB each way: scale {sf:.4f} / {sw:.4f}")
    for prec, t in (("fp64", "double"), ("fp32", "float")):
        for key, (pat, srcf) in KERNELS.items():
            rx = re.compile(pat.format(t=t))
            fb = [v for n, v in f if rx.search(n)]
            wb = [v for n, v in w if rx.search(n)]
            if not fb or not wb:
                continue
            nb = (sum(fb) * sf + sum(wb) * sw) * 1024.0     # bytes of the product's launches
            with open(os.path.join(HERE, "csrc", srcf), "rb") as fh:
                sha = hashlib.sha256(fh.read()).hexdigest()[:16]
            print(f"| {key} | mixture1m | {leaf} | {prec} | {sha} | {nb:.4g} |   ({len(fb)} launches: "
                  f"fetch {sum(fb) * sf / 1024:.1f} MiB, write {sum(wb) * sw / 1024:.1f} MiB)")


def stats(trace_csv: str) -> None:
    """Mean duration per (kernel, grid) of the product's kernels from a
    rocprofv3 --kernel-trace --output-format csv trace: the launches of one
    configuration share a grid, so its per-launch time can be read apart
    from other trees' launches in the same run."""
    import csv
    groups = {}
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            name = r.get("Kernel_Name", "")
            if not re.search(r"k_(p2p|m2l_stream|gemm_tasks|p2m|l2p|shift)", name):
                continue
            short = re.sub(r"\(.*", "", name.replace("(anonymous namespace)::", "").replace("void ", ""))
            grid = (int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]), int(r["Grid_Size_Z"]))
            g = groups.setdefault((short, grid), [])
            g.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print("| kernel | grid (threads) | launches | mean us | min us | max us |")
    print("|---|---|---|---|---|---|")
    for (k, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        print(f"| {k} | {grid[0]}x{grid[1]}x{grid[2]} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | "
              f"{max(v):.2f} |")


def counters(db: str, pattern: str) -> None:
    """Every counter of each dispatch whose kernel matches `pattern`, from a
    rocprofv3 --pmc database (one line per dispatch)."""
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, grid_size, counter_name, value from counters_collection "
                       "order by dispatch_id").fetchall()
    per = {}
    for did, name, grid, cn, v in rows:
        if re.search(pattern, name):
            e = per.setdefault(did, [name, grid, {}])
            e[2][cn] = e[2].get(cn, 0.0) + float(v)
    for did, (name, grid, cs) in sorted(per.items()):
        short = re.sub(r"\(.*", "", name.replace("(anonymous namespace)::", "").replace("void ", ""))
        print(f"{short} grid {grid}: " + " ".join(f"{k}={v:.4g}" for k, v in sorted(cs.items())))


if __name__ == "__main__":
    if len(sys.argv) in (2, 3) and sys.argv[1] == "run":
        run(int(sys.argv[2]) if len(sys.argv) == 3 else LEAF)
    elif len(sys.argv) in (4, 5) and sys.argv[1] == "report":
        report(sys.argv[2], sys.argv[3], int(sys.argv[4]) if len(sys.argv) == 5 else LEAF)
    elif len(sys.argv) == 3 and sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif len(sys.argv) == 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3])
    else:
        print(__doc__)
        sys.exit(2)
