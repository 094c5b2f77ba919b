"""Summaries of rocprofv3 output for the profiles folder (text only).

Two summaries per workload:
  * kernel trace: per-kernel calls and average duration from
    `rocprofv3 --kernel-trace --stats` (kernel_stats.csv), beside the averages
    the sampling profiler of bench.py measured with HIP events in the same run;
  * HBM bytes: FETCH_SIZE and WRITE_SIZE per dispatch (two separate --pmc
    runs), each scaled by what the same counter reads for a plain 1 GiB
    device copy, so that the figures are bytes moved to and from HBM.

The byte summary ends with a JSON block that bench.py reads to fill the
roofline's `traffic`; it carries a hash of the kernel sources so that figures
taken on other kernels are never reported.

Usage:
  python -m paper_2509_10103_amd.profsum trace  <kernel_stats.csv> <bench.log> <out.md> <command>
  python -m paper_2509_10103_amd.profsum bytes  <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv> <out.md> <commands>
  python -m paper_2509_10103_amd.profsum counters <counter_collection.csv> <out.md> <command> <nt> <nz> <shapes>
"""
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_BYTES = 1 << 30


def source_hash():
    """sha256 over the kernel sources of libnpo (sorted by name): the .hip files,
    which hold the kernels and their launchers, and the device header.  The
    bytes a launch moves depend on these and on the launch shapes, which the
    summaries record; host-only changes do not alter them."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") or name == "npo_device.h":
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def short_name(full):
    n = full.split("(")[0]
    for pre in ("void ", "npo::"):
        n = n.replace(pre, "")
    return n


def family_kernels(nt, nz, names=(), shapes=(1, 4, 4), nr=64, rg=16):
    """Kernel name of each bench.py kernel family for transform lengths nt, nz,
    radial size nr, launch shapes (zgroup, azimuthal z-block forward,
    adjoint) and radial block size rg; the generic kernels stand in where
    `names` (the names seen in a profile) holds no compile-time-sized one."""
    zbf, zba = shapes[1], shapes[2]
    nrc = nr if (f"k_solve<1, {nr}, {rg}>" in names or f"k_solve<2, {nr}, {rg}>" in names or not names) else 0
    pz = nz % 12 == 0                       # pruned axial kernels for N_z = 3P,
    # with two m per block for the three-field passes
    zk = "p" if pz else "t"
    mb = (lambda nf: f", {2 if nf <= 3 else 1}") if pz else (lambda nf: "")
    fz = f"k_zinv_{zk}<{nz}, 0, 6{mb(6)}>" in names or not names
    ft = f"k_theta_t<{nt}, 0, {zbf}, false>" in names or f"k_theta_p<{nt}, {zbf}, false>" in names or not names
    zi = (lambda nf: f"k_zinv_{zk}<{nz}, {6 if nf == 3 else 0}, {nf}{mb(nf)}>") if fz else (lambda nf: "k_zinv")
    zf = (lambda nf: f"k_zfwd_{zk}<{nz}, {nf}{mb(nf)}>") if fz else (lambda nf: "k_zfwd")
    def th(a):
        if not a and zbf < 0:
            return f"k_theta_w<{nt}, {-zbf}>"
        if a and zba < 0:
            return f"k_theta_wa<{nt}, {-zba}>"
        if not ft:
            return "k_theta"
        if nt % 12 == 0:
            return f"k_theta_pa<{nt}, {zba}>" if a else f"k_theta_p<{nt}, {zbf}, false>"
        return f"k_theta_t<{nt}, {a}, {zba if a else zbf}, false>"
    return {
        "curl": "k_curl_aux", "zinv_fwd": zi(6), "theta_fwd": th(0), "zfwd_fwd": zf(3),
        "zinv_adj": zi(9), "theta_adj": th(1), "zfwd_adj": zf(6), "zinv_adjy": zi(3),
        "solve_pred": f"k_solve<1, {nrc}, {rg}>", "solve_corr": f"k_solve<2, {nrc}, {rg}>",
        "solve_raw": f"k_solve<0, {nrc}, {rg}>", "solve_adj": f"k_solve_adj<false, {nrc}, {rg}>",
        "solve_adj2": f"k_solve_adj<true, {nrc}, {rg}>", "adj_combine": f"k_final<{rg}>",
        "wdot": "k_wdot_partial", "project": "k_project", "axpby": "k_axpby",
    }


def _counter(path, counter):
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            per[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return per


def trace(stats_csv, bench_log, out_md, command):
    rows = list(csv.DictReader(open(stats_csv)))
    bench = json.loads([ln for ln in open(bench_log).read().splitlines() if ln.startswith('{"metric"')][-1])
    cfg = bench["config"]
    fam = family_kernels(cfg["grid"][1], cfg["grid"][2], {short_name(r["Name"]) for r in rows},
                         cfg.get("launch_shapes") or (1, 4, 4), cfg["grid"][0], cfg.get("radial_block", 16))
    inv = {v: k for k, v in fam.items()}
    lines = [f"# Kernel trace: {cfg['workload']}", "",
             f"Command (repository root, one MI355X): `{command}`", "",
             f"bench.py line of the same run: value {bench['value']:.4g} {bench['unit']}, "
             f"{bench['ms_per_step'] / 1e3:.2f} s per optimisation iteration, launch shapes "
             f"{cfg.get('launch_shapes')}.", "",
             "rocprofv3 `--stats` (all launches) beside the bench.py sampling profiler (HIP events on the "
             "launch stream, every `--stride`-th launch of each family):", "",
             "| kernel | family | calls | rocprof avg us | bench avg us | share of kernel time |",
             "|---|---|---:|---:|---:|---:|"]
    for r in rows:
        n = short_name(r["Name"])
        f = inv.get(n, "")
        b = bench["kernels"].get(f, {}).get("avg_us", "") if f else ""
        lines.append(f"| `{n}` | {f} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {b} | "
                     f"{float(r['Percentage']):.2f}% |")
    rf = bench["roofline"]
    lines += ["", f"Dominant kernel (largest total time): {rf['kernel']} = `{fam.get(rf['kernel'])}`, "
              f"{rf['alg_bytes_per_launch'] / 1e6:.1f} MB algorithmic per launch, "
              f"{rf['avg_launch_us']:.2f} us per launch (bench), {rf['achieved']:.0f} GB/s = "
              f"{100 * rf['frac']:.1f}% of 8 TB/s.", ""]
    open(out_md, "w").write("\n".join(lines))


def bytes_summary(fetch_csv, write_csv, cf_csv, cw_csv, out_md, commands, nt, nz, shapes, nr=64):
    fetch, write = _counter(fetch_csv, "FETCH_SIZE"), _counter(write_csv, "WRITE_SIZE")
    cf = max(_counter(cf_csv, "FETCH_SIZE")["__amd_rocclr_copyBuffer"])
    cw = max(_counter(cw_csv, "WRITE_SIZE")["__amd_rocclr_copyBuffer"])
    ff = COPY_BYTES / (cf * 1024)
    fw = COPY_BYTES / (cw * 1024)
    fam = family_kernels(nt, nz, set(fetch), shapes, nr)
    per = {}
    lines = ["# HBM bytes per launch: workload grid " + f"{nt}x{nz} (theta x z)", "",
             "Commands (repository root, one MI355X, each counter in its own run):", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", f"Copy calibration (1 GiB device copy): FETCH_SIZE reads {cf:.0f} KiB -> factor {ff:.3f}; "
              f"WRITE_SIZE reads {cw:.0f} KiB -> factor {fw:.3f}.", "",
              f"Launch shapes (zgroup, theta z-block forward, adjoint): {shapes}.", "",
              "| family | kernel | dispatches | fetch MB | write MB | traffic MB |", "|---|---|---:|---:|---:|---:|"]
    for f, n in fam.items():
        if n not in fetch or n not in write:
            continue
        fb = sum(fetch[n]) / len(fetch[n]) * 1024 * ff
        wb = sum(write[n]) / len(write[n]) * 1024 * fw
        per[f] = {"fetch": fb, "write": wb}
        lines.append(f"| {f} | `{n}` | {len(fetch[n])} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} |")
    blob = {"source_sha256": source_hash(), "nt": nt, "nz": nz, "launch_shapes": shapes,
            "copy_factors": {"FETCH_SIZE": ff, "WRITE_SIZE": fw}, "bytes_per_launch": per}
    lines += ["", "Machine-readable (read by bench.py; valid only while the kernel sources hash to the value "
              "below):", "", "```json", json.dumps(blob, indent=1), "```", ""]
    open(out_md, "w").write("\n".join(lines))


def counters_summary(csv_path, out_md, command, nt, nz, shapes, nr=64):
    """Per-kernel averages (per dispatch) of the SQ counters of one --pmc run,
    with derived figures: VALU and LDS instructions per wave, the fraction of
    busy cycles with a VALU instruction issued, LDS bank-conflict cycles per
    LDS instruction."""
    rows = list(csv.DictReader(open(csv_path)))
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        per[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    fam = family_kernels(nt, nz, set(per), shapes, nr)
    inv = {v: k for k, v in fam.items()}
    names = sorted({c for k in per.values() for c in k})
    lines = [f"# SQ counters per dispatch: workload grid {nt}x{nz} (theta x z)", "",
             f"Command (repository root, one MI355X): `{command}`", "",
             f"Launch shapes (zgroup, theta z-block forward, adjoint): {shapes}.", "",
             "Derived: VALU/wave = SQ_INSTS_VALU / SQ_WAVES; LDS/wave = SQ_INSTS_LDS / SQ_WAVES; "
             "VALU busy = SQ_ACTIVE_INST_VALU / SQ_BUSY_CYCLES (per SE, summed over SEs, so a ratio of "
             "aggregates); conflict/LDS = SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS; LDS wait = SQ_WAIT_INST_LDS / "
             "SQ_WAVE_CYCLES.", "",
             "| family | kernel | dispatches | waves | VALU/wave | LDS/wave | VALU busy | conflict/LDS | LDS wait |",
             "|---|---|---:|---:|---:|---:|---:|---:|---:|"]
    blob = {}
    for k in sorted(per, key=lambda x: inv.get(x, "~" + x)):
        c = {n: sum(v) / len(v) for n, v in per[k].items()}
        nd = max(len(v) for v in per[k].values())
        w = c.get("SQ_WAVES", 0.0) or 1.0
        valu = c.get("SQ_INSTS_VALU", 0.0) / w
        lds = c.get("SQ_INSTS_LDS", 0.0) / w
        busy = c.get("SQ_ACTIVE_INST_VALU", 0.0) / (c.get("SQ_BUSY_CYCLES", 0.0) or 1.0)
        conf = c.get("SQ_LDS_BANK_CONFLICT", 0.0) / (c.get("SQ_INSTS_LDS", 0.0) or 1.0)
        wait = c.get("SQ_WAIT_INST_LDS", 0.0) / (c.get("SQ_WAVE_CYCLES", 0.0) or 1.0)
        blob[k] = c
        if k not in inv:
            continue
        lines.append(f"| {inv[k]} | `{k}` | {nd} | {w:.0f} | {valu:.0f} | {lds:.0f} | {busy:.3f} | {conf:.3f} | "
                     f"{wait:.3f} |")
    lines += ["", "Raw per-dispatch averages:", "", "```json", json.dumps(blob, indent=1, sort_keys=True), "```", ""]
    open(out_md, "w").write("\n".join(lines))


def load_traffic(path, nt, nz):
    """bytes_per_launch from a byte summary, or None if absent or taken on
    other kernel sources or transform lengths (the launch shapes it records
    are informational: with the XCD-aware placement the z-block size leaves
    the HBM bytes unchanged)."""
    try:
        txt = open(path).read()
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != source_hash() or blob.get("nt") != nt or blob.get("nz") != nz:
        return None
    return blob["bytes_per_launch"]


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(*sys.argv[2:6])
    elif sys.argv[1] == "counters":
        a = sys.argv[2:]
        counters_summary(a[0], a[1], a[2], int(a[3]), int(a[4]), [int(x) for x in a[5].split(",")])
    elif sys.argv[1] == "bytes":
        a = sys.argv[2:]
        bytes_summary(a[0], a[1], a[2], a[3], a[4], a[5].split(" ;; "), int(a[6]), int(a[7]),
                      [int(x) for x in a[8].split(",")])
    else:
        raise SystemExit(__doc__)
