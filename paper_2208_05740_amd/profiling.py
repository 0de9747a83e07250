"""Summaries of rocprofv3 results for the library's kernels.

  python -m paper_2208_05740_amd.profiling summary --db RUN_results.db --out FILE.md --cmd "..."
      kernel-trace summary: dispatches, average and total duration per kernel,
      with the library's kernel-class name for each gemm_epi instantiation.
  python -m paper_2208_05740_amd.profiling traffic --fetch-db A.db --write-db B.db \\
         --copy-mib 1024 --out profiles/hbm_traffic.json --cmd "..."
      HBM bytes per launch from FETCH_SIZE and WRITE_SIZE counter runs, each
      scaled by that counter's reading for a plain device copy of known size
      (bench.py --copy-probe-mb) so that counter units and sampling drop out.
"""
import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

EPI = {"bound": "BoundEpi", "conc": "ConcEpi", "adj": "AdjEpi", "store": "StoreEpi"}


def class_of(symbol):
    """Library kernel-class name ('adj.bf16.t32x32', ...) of a gemm_epi
    instantiation, from its mangled or demangled symbol; None otherwise."""
    m = re.search(r"gemm_epi_kernelI(DF16b|f)Li(\d+)ELi(\d+)ELi\d+ELi\d+ELi\d+ELb([01])ENS_\d+(\w+?Epi)", symbol)
    if m:
        dt, bm, bn, sg, epi = m.groups()
    else:
        m = re.search(r"gemm_epi_kernel<(float|__bf16), (\d+), (\d+), \d+, \d+, \d+, (true|false), gcp::(\w+Epi)",
                      symbol)
        if not m:
            return None
        dt, bm, bn, sg, epi = m.groups()
        sg = "1" if sg == "true" else "0"
    kind = {v: k for k, v in EPI.items()}.get(epi)
    if kind is None:
        return None
    name = f"{kind}.{'bf16' if dt in ('DF16b', '__bf16') else 'fp32'}"
    if sg == "1":
        name += ".sign"
    return name + f".t{bm}x{bn}"


def kernel_times(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels").fetchall()
    agg = collections.defaultdict(lambda: [0, 0.0])
    for name, s, e in rows:
        agg[name][0] += 1
        agg[name][1] += (e - s)
    return agg


def counters(db):
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
    ci = {c: i for i, c in enumerate(cols)}
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in con.execute("select * from counters_collection"):
        out[r[ci["kernel_name"]]][r[ci["counter_name"]]].append((r[ci["dispatch_id"]], r[ci["value"]]))
    res = {}
    for k, d in out.items():
        res[k] = {}
        for c, vals in d.items():
            per = collections.defaultdict(float)
            for disp, v in vals:
                per[disp] += v
            res[k][c] = (len(per), sum(per.values()) / len(per), max(per.values()))
    return res


def short(name, n=90):
    name = re.sub(r"\(.*", "", name)
    return name if len(name) <= n else name[:n] + "..."


def cmd_summary(a):
    agg = kernel_times(a.db)
    tot = sum(v[1] for v in agg.values())
    lines = [f"# Kernel trace summary: {a.title}", "", f"Command: `{a.cmd}`", "",
             f"Total kernel time {tot / 1e6:.3f} ms over {sum(v[0] for v in agg.values())} dispatches.", "",
             "| kernel class | dispatches | avg us | total ms | share | symbol |", "|---|---:|---:|---:|---:|---|"]
    for name, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:a.top]:
        lines.append(f"| {class_of(name) or '-'} | {n} | {t / n / 1e3:.2f} | {t / 1e6:.3f} | {100 * t / tot:.1f}% "
                     f"| `{short(name)}` |")
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def source_sha():
    """Hash of every device-code source (kernels and the headers they use)."""
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_2208_05740_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()


def cmd_traffic(a):
    fetch = counters(a.fetch_db)
    write = counters(a.write_db)
    copy_bytes = a.copy_mib * 1024 * 1024

    def copy_reading(res, counter):
        best = None
        for k, d in res.items():
            if "copy" in k and counter in d:
                v = d[counter][2]
                best = v if best is None or v > best else best
        return best

    f_copy = copy_reading(fetch, "FETCH_SIZE")
    w_copy = copy_reading(write, "WRITE_SIZE")
    rec = {"source_sha": source_sha(), "command_fetch": a.cmd_fetch, "command_write": a.cmd_write,
           "copy_bytes": copy_bytes, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
           "fetch_scale": copy_bytes / (f_copy * 1024), "write_scale": copy_bytes / (w_copy * 1024), "kernels": {}}
    for k in fetch:
        cls = class_of(k)
        if cls and "FETCH_SIZE" in fetch[k] and k in write and "WRITE_SIZE" in write[k]:
            rec["kernels"][cls] = {"dispatches": fetch[k]["FETCH_SIZE"][0],
                                   "fetch_kib": fetch[k]["FETCH_SIZE"][1], "write_kib": write[k]["WRITE_SIZE"][1]}
    json.dump(rec, open(a.out, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("summary")
    s.add_argument("--db", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--cmd", default="")
    s.add_argument("--title", default="")
    s.add_argument("--top", type=int, default=20)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch-db", required=True)
    t.add_argument("--write-db", required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--cmd-fetch", default="")
    t.add_argument("--cmd-write", default="")
    a = ap.parse_args()
    if a.cmd_name == "summary":
        a.cmd = a.cmd
        cmd_summary(a)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    main()
