"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2108_12430_amd.profsum summary STATS_CSV FETCH_CSV WRITE_CSV OUT_MD \
        --title TITLE --cmd-trace CMD --cmd-fetch CMD --cmd-write CMD
    python -m paper_2108_12430_amd.profsum traffic FETCH_CSV WRITE_CSV OUT_JSON
    python -m paper_2108_12430_amd.profsum util COUNTER_CSV OUT_MD --title TITLE --cmd CMD
    python -m paper_2108_12430_amd.profsum stats STATS_CSV OUT_MD --title TITLE --cmd CMD \
        [--trace TRACE_CSV --marker NAME]

STATS_CSV is the ``*_kernel_stats.csv`` of a ``--kernel-trace --stats`` run;
FETCH_CSV / WRITE_CSV are the ``*_counter_collection.csv`` files of two
``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` runs of a program that also
copies 1 GiB with a device-to-device copy (``bench.py --copy-calibration
1024``).  The counters read in KiB per dispatch; each is scaled by the
factor that makes the 1 GiB copy read (write) exactly 1 GiB.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_KERNEL = "__amd_rocclr_copyBuffer"
# bench launch name -> (rocprof kernel name, source file), for the kernels
# whose traffic bench.py reports; each entry is valid while its source's
# hash is unchanged
KERNELS = {
    # the serving step's launch: the fused network with the snapshot update
    "dc_fused_bf16": ("void gw::dc_fused<2, false, true>(gw::ConvP, gw::FusedP, int)",
                      "paper_2108_12430_amd/csrc/conv_bf16.hip"),
    "bbh_fused": ("gw::bbh_fused(gw::BbFusedP)", "paper_2108_12430_amd/csrc/bbh_fused.hip"),
    "snapshot": ("gw::snapshot_kernel(char*, gw::Item const*, float const*)",
                 "paper_2108_12430_amd/csrc/misc.hip"),
}


def _per_kernel(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return d


def _factor(d):
    cal = [v for v in d.get(COPY_KERNEL, []) if v > 200000]   # the 1 GiB copy, not small copies
    if not cal:
        raise SystemExit("no 1 GiB calibration copy in the counter file")
    return 1048576.0 / (sum(cal) / len(cal)), sum(cal) / len(cal)


def summary(a):
    rows = list(csv.DictReader(open(a.stats)))
    F, Wr = _per_kernel(a.fetch), _per_kernel(a.write)
    ff, cf = _factor(F)
    fw, cw = _factor(Wr)
    md = [f"# {a.title}", "", "Kernel trace (durations):", "", "```", a.cmd_trace, "```", "",
          "PyTorch kernels (`at::native::*`, the input staging of the set-up) are left out; "
          "`total %` is of the whole trace.", "",
          "| kernel | calls | avg us | total % |", "|---|---|---|---|"]
    for r in [r for r in rows if "at::native" not in r["Name"]][:24]:
        md.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['Percentage']):.2f} |")
    md += ["", "Counters (one rocprofv3 pass per counter; the program also copies 1 GiB for calibration):", "",
           "```", a.cmd_fetch, a.cmd_write, "```", "",
           f"Calibration (1 GiB copy by `{COPY_KERNEL}`): FETCH_SIZE reads {cf:.0f} KiB -> factor {ff:.3f}; "
           f"WRITE_SIZE reads {cw:.0f} KiB -> factor {fw:.3f}.", "",
           "Scaled HBM bytes per launch = (FETCH_SIZE x fetch factor + WRITE_SIZE x write factor) x 1024.", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled HBM MB per launch |",
           "|---|---|---|---|---|"]
    for k in sorted(F, key=lambda k: -sum(F[k]) / len(F[k]))[:16]:
        if k.startswith("__amd") or "at::native" in k:
            continue
        f = sum(F[k]) / len(F[k])
        w = sum(Wr.get(k, [0.0])) / max(len(Wr.get(k, [0.0])), 1)
        md.append(f"| `{k[:110]}` | {len(F[k])} | {f:.0f} | {w:.0f} | {(f * ff + w * fw) * 1024 / 1e6:.2f} |")
    open(a.out, "w").write("\n".join(md) + "\n")
    print("\n".join(md))


def traffic(a):
    F, Wr = _per_kernel(a.fetch), _per_kernel(a.write)
    ff, _ = _factor(F)
    fw, _ = _factor(Wr)
    res = {"_about": "HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE passes, scaled by a 1 GiB "
                     "device copy; an entry is valid only while its kernel source hash matches",
           "fetch_factor": ff, "write_factor": fw, "kernels": {}}
    for name, (rk, source) in KERNELS.items():
        if rk not in F or rk not in Wr:
            continue
        f = sum(F[rk]) / len(F[rk])
        w = sum(Wr[rk]) / len(Wr[rk])
        src = open(os.path.join(ROOT, source), "rb").read()
        res["kernels"][name] = {"rocprof_name": rk, "source": source,
                                "source_sha256": hashlib.sha256(src).hexdigest(), "fetch_kib": f,
                                "write_kib": w, "bytes_per_launch": (f * ff + w * fw) * 1024}
    json.dump(res, open(a.out, "w"), indent=1)
    print(json.dumps(res, indent=1))


N_CU, N_SIMD, N_XCD = 256, 1024, 8  # MI355X


def util(a):
    """Per-kernel utilisation from one pass of SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT, SQ_INSTS_VALU, SQ_INSTS_LDS,
    SQ_INSTS_MFMA, SQ_WAVES and GRBM_GUI_ACTIVE (per-XCD active cycles)."""
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(a.counters)):
        if r["Kernel_Name"].startswith(("__amd", "void at::", "at::")):
            continue
        d[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    md = [f"# {a.title}", "", "```", a.cmd, "```", "",
          f"Per dispatch, averaged over dispatches.  cycles = GRBM_GUI_ACTIVE / {N_XCD} (per-XCD active "
          f"cycles).  MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (cycles x {N_SIMD} SIMDs); LDS busy = "
          f"SQ_LDS_IDX_ACTIVE / (cycles x {N_CU} CUs); conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE; "
          f"VALU issue = SQ_INSTS_VALU x 4 cycles / (cycles x {N_SIMD} SIMDs) (a wave64 VALU instruction "
          "occupies its SIMD for 4 cycles; MFMA instructions are counted in SQ_INSTS_VALU).", "",
          "| kernel | dispatches | cycles | MFMA busy % | LDS busy % | LDS conflict % | VALU issue % | "
          "VALU instr / wave | MFMA instr / wave |", "|---|---|---|---|---|---|---|---|---|"]
    av = lambda v: sum(v) / len(v)
    rows = []
    for k, c in d.items():
        need = ("GRBM_GUI_ACTIVE", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT",
                "SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_WAVES")
        if not all(n in c for n in need):
            continue
        cyc = av(c["GRBM_GUI_ACTIVE"]) / N_XCD
        waves = max(av(c["SQ_WAVES"]), 1.0)
        lds = av(c["SQ_LDS_IDX_ACTIVE"])
        rows.append((cyc, f"| `{k[:100]}` | {len(c['GRBM_GUI_ACTIVE'])} | {cyc:.0f} | "
                          f"{100 * av(c['SQ_VALU_MFMA_BUSY_CYCLES']) / (cyc * N_SIMD):.1f} | "
                          f"{100 * lds / (cyc * N_CU):.1f} | {100 * av(c['SQ_LDS_BANK_CONFLICT']) / max(lds, 1):.1f} | "
                          f"{100 * av(c['SQ_INSTS_VALU']) * 4 / (cyc * N_SIMD):.1f} | "
                          f"{av(c['SQ_INSTS_VALU']) / waves:.0f} | {av(c['SQ_INSTS_MFMA']) / waves:.0f} |"))
    md += [r for _, r in sorted(rows, reverse=True)]
    open(a.out, "w").write("\n".join(md) + "\n")
    print("\n".join(md))


def stats(a):
    """Kernel-trace summary; with --trace, also the per-kernel time of the
    last complete step between two dispatches of the marker kernel."""
    rows = list(csv.DictReader(open(a.stats)))
    md = [f"# {a.title}", "", "```", a.cmd, "```", "",
          "PyTorch kernels (`at::native::*`, input set-up) are left out; `total %` is of the whole trace.", "",
          "| kernel | calls | avg us | min us | max us | total % |", "|---|---|---|---|---|---|"]
    for r in [r for r in rows if "at::native" not in r["Name"]][:a.top]:
        md.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                  f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if a.trace:
        tr = sorted(csv.DictReader(open(a.trace)), key=lambda r: int(r["Start_Timestamp"]))
        idx = [i for i, r in enumerate(tr) if a.marker in r["Kernel_Name"]]
        if len(idx) >= 2:
            seg = tr[idx[-2]:idx[-1]]
            agg = collections.defaultdict(lambda: [0, 0])
            for r in seg:
                agg[r["Kernel_Name"]][0] += 1
                agg[r["Kernel_Name"]][1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            wall = (int(tr[idx[-1]]["Start_Timestamp"]) - int(tr[idx[-2]]["Start_Timestamp"])) / 1e3
            busy = sum(v[1] for v in agg.values()) / 1e3
            md += ["", f"Last complete step (from one `{a.marker}` dispatch to the next): {wall:.1f} us wall, "
                       f"{busy:.1f} us of kernel time, {len(seg)} dispatches.", "",
                   "| kernel | dispatches | us in the step |", "|---|---|---|"]
            for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1]):
                md.append(f"| `{k[:110]}` | {v[0]} | {v[1] / 1e3:.1f} |")
    open(a.out, "w").write("\n".join(md) + "\n")
    print("\n".join(md))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="sub", required=True)
    s = sub.add_parser("summary")
    for n in ("stats", "fetch", "write", "out"):
        s.add_argument(n)
    s.add_argument("--title", required=True)
    s.add_argument("--cmd-trace", required=True)
    s.add_argument("--cmd-fetch", required=True)
    s.add_argument("--cmd-write", required=True)
    t = sub.add_parser("traffic")
    for n in ("fetch", "write", "out"):
        t.add_argument(n)
    u = sub.add_parser("util")
    u.add_argument("counters")
    u.add_argument("out")
    u.add_argument("--title", required=True)
    u.add_argument("--cmd", required=True)
    k = sub.add_parser("stats")
    k.add_argument("stats")
    k.add_argument("out")
    k.add_argument("--title", required=True)
    k.add_argument("--cmd", required=True)
    k.add_argument("--trace")
    k.add_argument("--marker", default="")
    k.add_argument("--top", type=int, default=30)
    a = ap.parse_args()
    {"summary": summary, "traffic": traffic, "util": util, "stats": stats}[a.sub](a)


if __name__ == "__main__":
    main()
