"""Summaries of rocprofv3 output for the committed profiles (text only, no GPU work).

    python -m paper_1810_09891_amd.profiling stats KERNEL_STATS_CSV --command "..." > summary.txt
    python -m paper_1810_09891_amd.profiling traffic FETCH_CSV WRITE_CSV --copy-mib MIB \\
        --command-fetch "..." --command-write "..." > traffic.json

``stats`` turns the ``*_kernel_stats.csv`` of ``rocprofv3 --kernel-trace --stats
--output-format csv`` into a table of calls and average / total durations per kernel.

    python -m paper_1810_09891_amd.profiling lds-probe     # build _build/lds_bw (no GPU work)

``traffic`` reads two ``--pmc`` runs of the same program (one collecting FETCH_SIZE, one
WRITE_SIZE, both in KiB per dispatch) that begin with one device copy of MIB MiB.  The
copy's readings against its known bytes give the scale factors; every other kernel's
average reading times the factor gives its HBM bytes per launch.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def short_name(name):
    """`void nfft::(anonymous namespace)::k_fold<float, 2>(...)` -> `k_fold<float, 2>`."""
    name = name.strip().strip('"').replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*$", "", name)
    name = re.sub(r"^void\s+", "", name)
    return name.replace("nfft::", "")


def base_name(name):
    return re.sub(r"<.*$", "", short_name(name))


def source_hash():
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1810_09891_amd", "csrc")
    for name in sorted(os.listdir(src)):
        with open(os.path.join(src, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def read_stats(path):
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            calls = int(r.get("Calls", 0))
            total = float(r.get("TotalDurationNs", 0.0))
            avg = float(r.get("AverageNs", total / max(calls, 1)))
            rows.append((short_name(r["Name"]), calls, avg / 1e3, total / 1e3, float(r.get("Percentage", 0.0))))
    rows.sort(key=lambda t: -t[3])
    return rows


def cmd_stats(args):
    rows = read_stats(args.csv)
    print("# rocprofv3 kernel statistics")
    print("# command: %s" % args.command)
    print("#")
    print("%-58s %7s %12s %12s %7s" % ("kernel", "calls", "avg_us", "total_us", "pct"))
    for name, calls, avg, total, pct in rows:
        print("%-58s %7d %12.3f %12.1f %7.2f" % (name[:58], calls, avg, total, pct))


def read_counter(path, counter):
    per = collections.defaultdict(list)
    grid = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            per[name].append(float(r["Counter_Value"]))
            grid[name] = max(grid.get(name, 0), int(r["Grid_Size"]))
    return per, grid


def calibration(per, grid, copy_bytes, counter):
    copies = [k for k in per if "copy" in k.lower()]
    if not copies:
        raise SystemExit("no copy kernel found for %s" % counter)
    # the calibration copy is the largest copy dispatch of the run
    best = max(((max(per[k]), k) for k in copies))
    kib = best[0]
    return copy_bytes / (kib * 1024.0), best[1], kib


def cmd_traffic(args):
    copy_bytes = args.copy_mib * (1 << 20)
    fetch, gf = read_counter(args.fetch_csv, "FETCH_SIZE")
    write, gw = read_counter(args.write_csv, "WRITE_SIZE")
    ff, fk, fkib = calibration(fetch, gf, copy_bytes, "FETCH_SIZE")
    wf, wk, wkib = calibration(write, gw, copy_bytes, "WRITE_SIZE")
    kernels = {}
    for name in sorted(set(fetch) | set(write)):
        if "copy" in name.lower() or "nfft" not in name:
            continue
        f = fetch.get(name, [])
        w = write.get(name, [])
        fb = ff * 1024.0 * (sum(f) / len(f)) if f else None
        wb = wf * 1024.0 * (sum(w) / len(w)) if w else None
        key = base_name(name)
        entry = kernels.setdefault(key, {"instances": []})
        entry["instances"].append({"name": short_name(name), "dispatches": len(f),
                                   "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb})
    for key, entry in kernels.items():
        # one figure per base name only when a single instance ran
        inst = entry["instances"]
        if len(inst) == 1 and inst[0]["fetch_bytes_per_launch"] is not None \
                and inst[0]["write_bytes_per_launch"] is not None:
            entry["bytes_per_launch"] = inst[0]["fetch_bytes_per_launch"] + inst[0]["write_bytes_per_launch"]
    out = {
        "source_hash": source_hash(),
        "calibration": {
            "copy_bytes": copy_bytes,
            "fetch": {"kernel": short_name(fk), "kib": fkib, "factor": ff},
            "write": {"kernel": short_name(wk), "kib": wkib, "factor": wf},
        },
        "commands": {"fetch": args.command_fetch, "write": args.command_write},
        "kernels": kernels,
    }
    json.dump(out, sys.stdout, indent=1)
    print()


def build_lds_probe():
    """Compile the LDS throughput probe (``calib/lds_bw.hip``) into ``_build/lds_bw``.  It is
    measurement tooling, not part of the library: run it on the GPU to obtain the LDS
    ceilings that the window kernels are compared against."""
    import subprocess

    from . import build as hipbuild

    src = os.path.join(ROOT, "paper_1810_09891_amd", "calib", "lds_bw.hip")
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "lds_bw")
    flags = [f for f in hipbuild.CFLAGS if f != "-fPIC"]
    subprocess.run([hipbuild.HIPCC] + flags + [src, "-o", exe], check=True)
    print(exe)
    return exe


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("lds-probe")
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--command-fetch", default="")
    t.add_argument("--command-write", default="")
    args = ap.parse_args(argv)
    if args.cmd == "lds-probe":
        build_lds_probe()
    elif args.cmd == "stats":
        cmd_stats(args)
    else:
        cmd_traffic(args)


if __name__ == "__main__":
    main()
