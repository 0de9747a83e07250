"""Summaries of rocprofv3 results for the library's kernels.

  python -m paper_2208_05740_amd.profiling summary --db RUN_results.db --out FILE.md --cmd "..."
      kernel-trace summary: dispatches, average and total duration per kernel,
      with the library's kernel-class name for each gemm_epi instantiation.
  python -m paper_2208_05740_amd.profiling traffic --fetch-db A.db --write-db B.db \\
         --copy-mib 1024 --out profiles/hbm_traffic.json --cmd "..."
      HBM bytes per launch from FETCH_SIZE and WRITE_SIZE counter runs, each
      scaled by that counter's reading for a plain device copy of known size
      (bench.py --copy-probe-mb) so that counter units and sampling drop out.
  python -m paper_2208_05740_amd.profiling mfma --db RUN_results.db --out FILE.md --cmd "..."
      MFMA work of each GEMM kernel class from SQ_INSTS_VALU_MFMA_MOPS_BF16 /
      _F32 (units of 512 FLOP): FLOP per dispatch, rate over the dispatch's
      duration in the counter run, fraction of the dense MFMA peak.
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


CONV_EPI = {"BoundEpi": "bound", "ConcEpi": "conc", "StoreEpi": "store", "AdjEpi": "adj", "AhatEpi": "ahat"}


def _explicit_pi(symbol, epi):
    """True for the explicit-pi instantiation of a bound or adjoint epilogue
    (its second template argument, PI, set)."""
    if epi not in ("BoundEpi", "AdjEpi"):
        return False
    return bool(re.search(epi + r"I(DF16b|f)Lb1E", symbol) or re.search(epi + r"<(float|__bf16), true>", symbol))


def conv_class_of(symbol):
    """Kernel-class name ('convT_bound.bf16.w4x1', 'conv_adj.bf16.sign.w4x1',
    'conv_adj_pi.bf16.w8x1', ...) of a conv_slab instantiation (waves x
    column tiles), or None."""
    m = re.search(r"conv_slab_kernelI(DF16b|f)Li(\d+)ELi(\d+)ELb([01])ELb([01])ENS_\d+(\w+?Epi)", symbol)
    if m:
        dt, nw, tn, tr, sg, epi = m.groups()
    else:
        m = re.search(r"conv_slab_kernel<(float|__bf16), (\d+), (\d+), (true|false), (true|false), gcp::(\w+Epi)",
                      symbol)
        if not m:
            return None
        dt, nw, tn, tr, sg, epi = m.groups()
        tr, sg = ("1" if tr == "true" else "0"), ("1" if sg == "true" else "0")
    kind = CONV_EPI.get(epi)
    if kind is None:
        return None
    if _explicit_pi(symbol, epi):
        kind += "_pi"
    name = ("convT_" if tr == "1" else "conv_") + kind + (".bf16" if dt in ("DF16b", "__bf16") else ".fp32")
    return name + (".sign" if sg == "1" else "") + f".w{nw}x{tn}"


def direct_class_of(symbol):
    """Kernel-class name ('convT_conc.fp32.direct.c3k2x2': source channels,
    taps per phase) of a direct transposed-conv instantiation, or None."""
    m = (re.search(r"convT_direct_kernelI(DF16b|f)Li(\d+)ELi(\d+)ELi(\d+)ELi\d+ENS_\d+(\w+?Epi)", symbol) or
         re.search(r"convT_direct_kernel<(float|__bf16), (\d+), (\d+), (\d+), \d+, gcp::(\w+Epi)", symbol))
    if not m:
        return None
    dt, nc, ta, tb, epi = m.groups()
    kind = CONV_EPI.get(epi)
    if kind is None:
        return None
    return f"convT_{kind}.{'bf16' if dt in ('DF16b', '__bf16') else 'fp32'}.direct.c{nc}k{ta}x{tb}"


def class_of(symbol):
    """Library kernel-class name ('adj.bf16.t32x32', 'convT_bound.bf16.w4x1',
    ...) of a gemm_epi, conv_slab or direct transposed-conv instantiation,
    from its mangled or demangled symbol; None otherwise."""
    if "conv_slab_kernel" in symbol:
        return conv_class_of(symbol)
    if "convT_direct_kernel" in symbol:
        return direct_class_of(symbol)
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
    if _explicit_pi(symbol, epi):
        kind += "_pi"
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


PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}


def cmd_mfma(a):
    con = sqlite3.connect(a.db)
    cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
    ci = {c: i for i, c in enumerate(cols)}
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    dur, name = {}, {}
    for r in con.execute("select * from counters_collection"):
        d = r[ci["dispatch_id"]]
        per[d][r[ci["counter_name"]]] += r[ci["value"]]
        dur[d] = r[ci["end"]] - r[ci["start"]]
        name[d] = r[ci["kernel_name"]]
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0, 0.0])
    for d, c in per.items():
        cls = class_of(name[d])
        if not cls:
            continue
        g = agg[cls]
        g[0] += 1
        g[1] += c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) * 512
        g[2] += c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512
        g[3] += dur[d]
    lines = [f"# MFMA work per GEMM kernel class: {a.title}", "", f"Command: `{a.cmd}`", "",
             "FLOP from SQ_INSTS_VALU_MFMA_MOPS_* (512 FLOP units, padding included); rate over the average "
             "dispatch duration of the counter run; peaks: dense bf16 2500, fp32 157.3 TFLOP/s.", "",
             "| kernel class | dispatches | MFMA GFLOP / dispatch | avg us | TFLOP/s | of peak |",
             "|---|---:|---:|---:|---:|---:|"]
    for cls, (n, fb, ff, t) in sorted(agg.items(), key=lambda kv: -kv[1][3]):
        flop = (fb + ff) / n
        us = t / n / 1e3
        dt = "bf16" if fb >= ff else "fp32"
        rate = flop / (us * 1e-6) / 1e12 if us > 0 else 0.0
        lines.append(f"| {cls} | {n} | {flop / 1e9:.2f} | {us:.1f} | {rate:.1f} | {100 * rate / PEAK_TFLOPS[dt]:.1f}% |")
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


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
    m = sub.add_parser("mfma")
    m.add_argument("--db", required=True)
    m.add_argument("--out", required=True)
    m.add_argument("--cmd", default="")
    m.add_argument("--title", default="")
    a = ap.parse_args()
    if a.cmd_name == "mfma":
        cmd_mfma(a)
        return
    if a.cmd_name == "summary":
        a.cmd = a.cmd
        cmd_summary(a)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    main()
