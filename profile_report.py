"""Stage-kernel report on the 4096^2 GL lattice from rocprofv3 output.

Reads the CSV output of the rocprofv3 runs below (each with `--output-format
csv -o run`) and the bench line of the same tree, and writes
  profiles/stage_kernels_gl4096.md  kernel times, HBM traffic, issue counters;
  profiles/traffic.json             per-launch traffic that bench.py reports in
                                    its roofline while the stage-kernel sources
                                    (comments stripped) are unchanged.

    python profile_report.py --stats D1 --fetch D2 --write D3 --valu D4 --lds D5 --bench LOG \
        [--stats D1' --fetch D2' --write D3' --valu D4' --lds D5' --bench LOG' ...]

One set of directories per integrator run of bench.py (`--integrator rk4`, `vv`,
`gf`), given in the same order for every option; kernels of all runs are merged.
D1: `rocprofv3 --kernel-trace --stats` of bench.py; D2, D3: `--pmc FETCH_SIZE`,
`--pmc WRITE_SIZE`; D4: `--pmc SQ_INSTS_VALU SQ_WAVES SQ_WAIT_INST_ANY
SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU`; D5: `--pmc SQ_INSTS_LDS
SQ_LDS_BANK_CONFLICT SQ_INSTS_SALU SQ_WAVE_CYCLES`; LOG: bench.py's output
(its last line is the JSON bench line, whose tile entry names the chosen tile).

Counter scaling comes from a plain device copy of --copy-mib MiB (`python3
bench.py --calibrate-copy-mib 1024` under `--pmc FETCH_SIZE` and `--pmc
WRITE_SIZE`, directories --copy-fetch and --copy-write): each counter's scale is
the copied bytes over what it reads for the copy, rounded to 3 decimals. On
MI355X FETCH_SIZE reads half the bytes read (scale 2) and WRITE_SIZE all the
bytes written (scale 1); those are the defaults without the copy runs.
"""
import argparse
import collections
import csv
import json
import os
import statistics

import bench

ROOT = os.path.dirname(os.path.abspath(__file__))
KIB = 1024
SITES = 4096 * 4096
C, ELEM = 4, 4  # field components, bytes per FP32 element
DEFAULT_SCALE = {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
# field sets read and written per site by each pass (stage passes P1..P4, the
# fused pass of stages 2-4, velocity Verlet in kick-drift-kick form, gradient flow)
ALG_SETS = {"P1": (1, 1), "P234": (3, 2), "P2": (2, 1), "P3": (4, 1), "P4": (5, 2), "VV": (2, 2), "VVA": (3, 3),
            "GF": (1, 1)}
# the kernels' pass template argument (VV: velocity Verlet in kick-drift-kick form,
# VVR: its restart pass, VVA: velocity Verlet with the stored force, GF: gradient
# flow keeping only the field)
PASS_INDEX = {"P1": 0, "P2": 1, "P3": 2, "P4": 3, "VV": 7, "GF": 13, "VVR": 10, "VVA": 12}
# passes each integrator launches every step
INTEG_PASSES = {"rk4": ("P1", "P234"), "vv": ("VV",), "gf": ("GF",)}
TILES = [(64, 16, 2), (64, 8, 2), (64, 16, 4), (64, 32, 4)]  # (TX, TY, rows per thread)
FUSED_TILES = 2  # the fused pass exists for the first two tile shapes


def kernel_name(p, t):
    TX, TY, RY = TILES[t]
    if p == "P234":
        return f"ss::stage_pass_fused<float, 0, {TX}, {TY}, {RY}>"
    return f"ss::stage_pass<float, 0, {PASS_INDEX[p]}, {TX}, {TY}, {RY}>"


def _short(name):
    return name.split("(")[0].replace("void ", "")


def counters(dirs):
    """{kernel: {counter: [values per dispatch]}} of one or more --pmc runs."""
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in [dirs] if isinstance(dirs, str) else dirs:
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                out[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def integrator_of(line):
    """rk4, vv or gf from a bench line's integrator description."""
    text = line.get("config", {}).get("integrator", "RK4")
    return "vv" if "Verlet" in text else "gf" if "gradient flow" in text else "rk4"


def restart_summary(stats_dirs, F, W, fs, ws):
    """Velocity Verlet's restart pass (64 x 16 tiles): it works only after an
    arrest and returns at once otherwise, so its figures are those of the
    dispatches that worked (more than a fifth of the longest duration or of the
    largest counter reading)."""
    k = kernel_name("VVR", 0)
    durs = []
    for d in stats_dirs:
        path = os.path.join(d, "run_kernel_trace.csv")
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            durs += [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in csv.DictReader(fh)
                     if _short(r["Kernel_Name"]) == k]
    if not durs or k not in F or k not in W:
        return None
    work = [x for x in durs if x > 0.2 * max(durs)]
    idle = [x for x in durs if x <= 0.2 * max(durs)]
    fv, wv = F[k]["FETCH_SIZE"], W[k]["WRITE_SIZE"]
    rd = wr = None  # no arrest in the counter runs: no working dispatch to read
    if max(fv) > 0 and max(wv) > 0:
        rd = fs * statistics.median([v for v in fv if v > 0.2 * max(fv)]) * KIB / 1e9
        wr = ws * statistics.median([v for v in wv if v > 0.2 * max(wv)]) * KIB / 1e9
    alg = SITES * C * ELEM / 1e9
    return {"kernel": k, "dispatches": len(durs), "working": len(work), "us_working": statistics.mean(work),
            "us_idle": statistics.mean(idle) if idle else 0.0, "read_GB": rd, "write_GB": wr, "alg_read_GB": alg,
            "alg_write_GB": alg}


def medians(c):
    return {k: {n: statistics.median(v) for n, v in m.items()} for k, m in c.items()}


def copy_scale(d, counter, mib):
    """Copied bytes over the counter's reading (in bytes) for the largest copy dispatch."""
    vals = counters(d)[COPY_KERNEL][counter]
    return round(mib * 2 ** 20 / (max(vals) * KIB), 3), max(vals)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    for a in ("stats", "fetch", "write", "valu", "lds", "bench"):
        ap.add_argument("--" + a, required=True, action="append")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--out-md", default=os.path.join(ROOT, "profiles", "stage_kernels_gl4096.md"))
    ap.add_argument("--out-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args(argv)

    if args.copy_fetch and args.copy_write:
        fs, fk = copy_scale(args.copy_fetch, "FETCH_SIZE", args.copy_mib)
        ws, wk = copy_scale(args.copy_write, "WRITE_SIZE", args.copy_mib)
        scale_text = (f"Counter scaling, from a plain {args.copy_mib} MiB device copy (`{COPY_KERNEL}`): FETCH_SIZE "
                      f"reads {fk:.0f} KiB, so read bytes = {fs:g} x FETCH_SIZE; WRITE_SIZE reads {wk:.0f} KiB, so "
                      f"written bytes = {ws:g} x WRITE_SIZE.")
    else:
        fs, ws = DEFAULT_SCALE["FETCH_SIZE"], DEFAULT_SCALE["WRITE_SIZE"]
        scale_text = (f"Counter scaling (default; no copy runs given): read bytes = {fs:g} x FETCH_SIZE, written "
                      f"bytes = {ws:g} x WRITE_SIZE.")
    F, W = counters(args.fetch), counters(args.write)
    stats = {}
    for d in args.stats:
        with open(os.path.join(d, "run_kernel_stats.csv")) as fh:
            stats.update({_short(r["Name"]): r for r in csv.DictReader(fh)})
    chosen_of, integs = {}, []
    for b in args.bench:
        with open(b) as fh:
            line = json.loads(fh.read().strip().split("\n")[-1])
        ig = integrator_of(line)
        integs.append(ig)
        for p in INTEG_PASSES[ig]:
            chosen_of[p] = line["tile"]["chosen"]
    chosen = chosen_of.get("P1", next(iter(chosen_of.values())))

    rows, traffic = [], {}
    for t in range(len(TILES)):
        for p in ("P1", "P234", "P2", "P3", "P4", "VV", "VVA", "GF"):
            if p == "P234" and t >= FUSED_TILES:
                continue
            k = kernel_name(p, t)
            if k not in F or k not in W or k not in stats:
                continue
            rd = fs * statistics.median(F[k]["FETCH_SIZE"]) * KIB / 1e9
            wr = ws * statistics.median(W[k]["WRITE_SIZE"]) * KIB / 1e9
            nr, nw = ALG_SETS[p]
            ar, aw = SITES * C * ELEM * nr / 1e9, SITES * C * ELEM * nw / 1e9
            us = float(stats[k]["AverageNs"]) / 1e3
            sel = p in chosen_of and list(TILES[t]) == chosen_of[p]
            label = f"{p} (tile {TILES[t][0]}x{TILES[t][1]}, {TILES[t][2]} rows/thread{'; chosen' if sel else ''})"
            rows.append((label, k, int(stats[k]["Calls"]), us, ar, rd, aw, wr, (ar + aw) / (us * 1e-6) / 1e3, sel))
            traffic.setdefault(f"tile{t}", {})[p] = {
                "read_GB": round(rd, 4), "write_GB": round(wr, 4), "total_GB": round(rd + wr, 4),
                "algorithmic_GB": round(ar + aw, 4), "ratio": round((rd + wr) / (ar + aw), 3), "kernel": k}
    rows.sort(key=lambda r: (not r[9], r[0]))

    def bench_args(ig):
        return ("python3 bench.py --steps 3 --warmup 1 --no-cpu --timing-steps 2 --autotune-steps 2"
                + ("" if ig == "rk4" else f" --integrator {ig}"))

    cmd_stats = [f"rocprofv3 --kernel-trace --stats --output-format csv -d {d} -o run -- python3 bench.py --steps 50 "
                 f"--warmup 5 --no-cpu --timing-steps 5" + ("" if ig == "rk4" else f" --integrator {ig}")
                 for d, ig in zip(args.stats, integs)]
    cmd_f = [f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d} -o run -- {bench_args(ig)}"
             for d, ig in zip(args.fetch, integs)]
    cmd_w = [f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d} -o run -- {bench_args(ig)}"
             for d, ig in zip(args.write, integs)]
    cmd_cf = (f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {args.copy_fetch or '<copy_fetch_dir>'} -o run -- "
              f"python3 bench.py --calibrate-copy-mib {args.copy_mib}")
    cmd_cw = (f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {args.copy_write or '<copy_write_dir>'} -o run -- "
              f"python3 bench.py --calibrate-copy-mib {args.copy_mib}")
    cmd_v = [f"rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES SQ_WAIT_INST_ANY SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU "
             f"--output-format csv -d {d} -o run -- {bench_args(ig)}" for d, ig in zip(args.valu, integs)]
    cmd_l = [f"rocprofv3 --pmc SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_INSTS_SALU SQ_WAVE_CYCLES "
             f"--output-format csv -d {d} -o run -- {bench_args(ig)}" for d, ig in zip(args.lds, integs)]
    md = ["# Stage kernels on the 4096^2 GL lattice (FP32 fields): kernel times, HBM traffic, issue counters", "",
          "Workload: `bench.py` default (GL 4096^2, kappa = 1.5, h = 0.2, 256 vortices, FP32 fields, FP64",
          f"reductions), run once per integrator ({', '.join(integs)}). For RK4 the autotuner picked the fused "
          f"plan on {chosen[0]}x{chosen[1]} tiles",
          "(P1 and the fused pass); the kernels each integrator's autotuner chose are marked, the other",
          "plans' and tiles' kernels run during autotuning and are listed for comparison.", "",
          "Commands (repository root, MI355X), summarised by `python profile_report.py` with the same",
          "directories:", "", "```", *cmd_stats, *cmd_f, *cmd_w, cmd_cf, cmd_cw, *cmd_v, *cmd_l, "```", "",
          scale_text, "",
          "| pass | kernel | calls | mean us | algorithmic read GB | measured read GB | algorithmic write GB | "
          "measured write GB | algorithmic TB/s |",
          "|---|---|---|---|---|---|---|---|---|"]
    for label, k, calls, us, ar, rd, aw, wr, tbs, _ in rows:
        md.append(f"| {label} | `{k}` | {calls} | {us:.1f} | {ar:.3f} | {rd:.3f} | {aw:.3f} | {wr:.3f} | {tbs:.2f} |")

    S1, S2 = medians(counters(args.valu)), medians(counters(args.lds))
    md += ["", "Issue counters (medians per dispatch). Lane-instructions per site = wave64 instructions x 64 /",
           "4096^2 sites (SALU: wave instructions per 64 sites). VALU busy = VALU wave instructions over what",
           "1024 SIMDs issue in the kernel's mean time at 2.4 GHz, one wave64 VALU instruction per 4 cycles",
           "(16 lanes per SIMD; packed FP32 is compiled out).", "",
           "| pass | kernel | VALU lane-instr per site | VALU busy | LDS lane-instr per site | "
           "LDS bank-conflict cycles per LDS instr | SALU instr per 64 sites | wait-any / wave cycles |",
           "|---|---|---|---|---|---|---|---|"]
    for label, k, calls, us, *_ in rows:
        if k not in S1 or k not in S2:
            continue
        a, c = S1[k], S2[k]
        busy = a["SQ_INSTS_VALU"] / (1024 * 2.4e9 / 4 * us * 1e-6)
        md.append(f"| {label} | `{k}` | {64 * a['SQ_INSTS_VALU'] / SITES:.0f} | {busy:.2f} | "
                  f"{64 * c['SQ_INSTS_LDS'] / SITES:.0f} | {c['SQ_LDS_BANK_CONFLICT'] / max(c['SQ_INSTS_LDS'], 1):.2f} | "
                  f"{64 * c['SQ_INSTS_SALU'] / SITES:.1f} | {a['SQ_WAIT_INST_ANY'] / a['SQ_WAVE_CYCLES']:.2f} |")

    rs = restart_summary(args.stats, F, W, fs, ws)
    if rs is not None:
        md += ["", f"Velocity Verlet's restart pass `{rs['kernel']}` (reads phi, writes u = dt/2 a after an arrest; "
               "returns at once on", f"the other steps): {rs['working']} of {rs['dispatches']} dispatches in the "
               f"stats run worked, {rs['us_working']:.1f} us each (the others {rs['us_idle']:.1f} us)."]
        if rs["read_GB"] is None:
            md += ["No arrest fired in the counter runs, so its traffic was not counted."]
        else:
            md += [f"A working dispatch reads {rs['read_GB']:.3f} GB (algorithmic {rs['alg_read_GB']:.3f}) and "
                   f"writes {rs['write_GB']:.3f} GB (algorithmic {rs['alg_write_GB']:.3f})."]
    if rs is not None and rs["read_GB"] is not None:
        traffic.setdefault("tile0", {})["VVR"] = {
            "read_GB": round(rs["read_GB"], 4), "write_GB": round(rs["write_GB"], 4),
            "total_GB": round(rs["read_GB"] + rs["write_GB"], 4),
            "algorithmic_GB": round(rs["alg_read_GB"] + rs["alg_write_GB"], 4),
            "ratio": round((rs["read_GB"] + rs["write_GB"]) / (rs["alg_read_GB"] + rs["alg_write_GB"]), 3),
            "kernel": rs["kernel"]}

    fin = stats.get("ss::pass_finalise<0>")
    if fin is not None:
        md += ["", "Each reducing pass is followed by `ss::pass_finalise<PASS>` (one workgroup summing the "
               "workgroup", f"partials and updating the status): {float(fin['AverageNs']) / 1e3:.1f} us per call "
               f"({int(fin['Calls'])} calls of the energy pass in the stats run), included in the P1 time that",
               "`bench.py` reports through `ss_time_passes`."]
    with open(args.out_md, "w") as fh:
        fh.write("\n".join(md) + "\n")
    rec = {"kernel_source": bench.kernel_source_hash(), "scale": {"FETCH_SIZE": fs, "WRITE_SIZE": ws},
           "commands": [*cmd_f, *cmd_w, cmd_cf, cmd_cw], "gl4096": traffic}
    with open(args.out_json, "w") as fh:
        fh.write(json.dumps(rec, indent=1) + "\n")
    print(rec["kernel_source"])


if __name__ == "__main__":
    main()
