"""Benchmark: seconds per additive two-level sweep (Steps 1-4 of Algorithm 2)
on one MI355X, plus the effective-Hamiltonian throughput at chi = 512.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3]

Workload 3 (default): L = 32 spatial orbitals, 32 electrons, Sz = 0, seeded
random integrals (seed 1003, 32 factors), chi = 512, 8 subdomains of lengths
[3,5,4,6,3,4,3,4], FP32 effective-Hamiltonian products with FP64 refinement,
FP64 Rayleigh-Ritz and FP64 coarse eigensolve; every local solve runs to the
workload's residual tolerance 1e-8 with no product cap.  Every step restarts
from the same chi-saturated random QN-consistent TT (seed 1004), so all steps
do the same work.  After the timed steps the same sweep runs once with FP64
products from the same input; its time and energy differences are reported
beside the timed path.

Prints one JSON line (see the repository documentation for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}  # dense MFMA TFLOP/s
HBM_PEAK = 8000.0  # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(idx):
    import seeded_inputs as S

    w = S.WORKLOADS[idx]
    lengths = list(w.lengths)
    return w, lengths


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_a2dmrg_L32_chi512.txt")
# the product kernels whose counters the traffic summary holds are compiled from these two
# files alone (kernels.hip holds the shared GEMM and the Davidson vector kernels)
KERNEL_SOURCES = ("paper_2505_23429_amd/csrc/bsheff.hip", "paper_2505_23429_amd/csrc/bsheff.h")
# timing slots of the product and the kernel symbols they stand for (FP32 products)
KERNEL_SYMBOLS = {
    "gemm_LWx_panels": "lw_gemm_kernel<float, 2, float>",
    "gemm_panels_WR": "panel_mfma_kernel<float, float>",
    "gemm_panels_WR_reduce": "reduce4_kernel<float>",
    "gemm_LWx": "lw_gemm_kernel<float, 1, float>",
    "gemm_Lx": "stage1_mfma_kernel<float>",
    "mix1_gather": "mix_kernel<float, 1, false>",
    "mix1_heavy_scatter": "mix_kernel<float, 1, true>",
    "mix2_gather": "mix_kernel<float, 2, false>",
    "mix2_heavy_scatter": "mix_kernel<float, 2, true>",
    "gemm_R": "stage4_mfma_kernel<float>",
    "gemm_R_reduce": "reduce4_kernel<float>",
}


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """Counter record of `kernel` from the committed traffic summary (HBM bytes per launch
    and their ratio to the algorithmic bytes of the same launches), or None when there is
    none for this kernel or its sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != kernel_source_hash():
        return None
    return t.get("kernels", {}).get(kernel)


# On gfx950 the derived FETCH_SIZE counts a read request as 128 bytes only when it is a
# TCC_BUBBLE; the 128-byte requests of an ordinary streaming read are counted as 64.  The
# raw request counters give the bytes directly: 128 N128 + 64 (N - N128 - N32) + 32 N32.
READ_COUNTERS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_BUBBLE_sum")


def read_bytes_per_dispatch(path):
    """Kernel name -> list of HBM read bytes per dispatch from a rocprofv3 counter file that
    holds either the raw read-request counters (READ_COUNTERS) or FETCH_SIZE (KiB)."""
    import csv
    from collections import defaultdict

    per = defaultdict(dict)
    names = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            per[d][r["Counter_Name"]] = float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
    out = defaultdict(list)
    for d, c in sorted(per.items()):
        if "TCC_EA0_RDREQ_sum" in c:
            n, n32, n128 = c["TCC_EA0_RDREQ_sum"], c["TCC_EA0_RDREQ_32B_sum"], c["TCC_EA0_RDREQ_128B_sum"]
            b = 128.0 * n128 + 32.0 * n32 + 64.0 * (n - n128 - n32)
        elif "FETCH_SIZE" in c:
            b = c["FETCH_SIZE"] * 1024.0
        else:
            continue
        out[names[d]].append(b)
    return out


def traffic_summary(read_csv, write_csv, bench_json, commands):
    """Reduce two rocprofv3 --pmc runs of `bench.py --copy-probe` (read requests, then
    WRITE_SIZE in KiB per dispatch) to HBM bytes per launch of the product kernels.  Each
    direction is scaled by what it reads for the probe, a plain elementwise copy that reads
    1 GiB and writes 1 GiB (a scale near 1 confirms the counter arithmetic); the algorithmic
    bytes per launch come from the same run's JSON line."""
    import csv
    from collections import defaultdict

    reads = read_bytes_per_dispatch(read_csv)
    write = defaultdict(list)
    with open(write_csv) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == "WRITE_SIZE":
                write[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    probe_r = max(v for n, vals in reads.items() if "elementwise" in n for v in vals)
    probe_w = max(v for n, vals in write.items() if "elementwise" in n for v in vals)
    rs, ws = float(1 << 30) / probe_r, float(1 << 30) / probe_w
    with open(read_csv) as f:
        raw = any(r["Counter_Name"] == "TCC_EA0_RDREQ_sum" for r in csv.DictReader(f))
    with open(bench_json) as f:
        run = json.loads([ln for ln in f if ln.startswith("{")][-1])
    out = {"workload": run["config"]["workload"], "source_sha256_16": kernel_source_hash(), "commands": commands,
           "read_counters": list(READ_COUNTERS) if raw else ["FETCH_SIZE"],
           "note": "HBM read bytes (from the read-request counters: 128 N128 + 64 N64 + 32 N32) and WRITE_SIZE per "
                   "dispatch, averaged over the launches of each kernel, each scaled by the value it reads for the "
                   "copy probe; algorithmic bytes per launch from the same run",
           "copy_probe": {"kernel": "torch elementwise x * 1.0, FP32, 1 GiB read + 1 GiB write",
                          "read_bytes_raw": probe_r, "write_bytes_raw": probe_w,
                          "read_scale": round(rs, 4), "write_scale": round(ws, 4)},
           "kernels": {}}
    for slot, sym in KERNEL_SYMBOLS.items():
        rv = [v for n, vals in reads.items() if sym in n for v in vals]
        wv = [v for n, vals in write.items() if sym in n for v in vals]
        k = run["kernels"].get(slot)
        if not rv or not wv or not k or k["launches"] == 0:
            continue
        rd = sum(rv) / len(rv) * rs
        wr = sum(wv) / len(wv) * ws
        alg = k["gbs"] * 1e9 * k["ms"] * 1e-3 / k["launches"]
        out["kernels"][slot] = {"symbol": sym, "launches_counted": len(rv),
                                "hbm_read_bytes_per_launch": int(rd), "hbm_write_bytes_per_launch": int(wr),
                                "hbm_bytes_per_launch": int(rd + wr),
                                "algorithmic_bytes_per_launch": int(alg),
                                "traffic_over_algorithmic": round((rd + wr) / max(alg, 1.0), 3)}
    return out


def mfma_summary(pmc_csv, bench_json, command):
    """Reduce a rocprofv3 --pmc run with the derived counters MfmaUtil (percent of SIMD
    cycles with the matrix cores busy while the GPU is active) and MfmaFlops (matrix-core
    flops, 512 per MOPS) to per-kernel averages for the product kernels, beside the
    algorithmic flops per launch of the same run."""
    import csv
    from collections import defaultdict

    per = defaultdict(dict)
    names = {}
    with open(pmc_csv) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            per[d][r["Counter_Name"]] = float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
    with open(bench_json) as f:
        run = json.loads([ln for ln in f if ln.startswith("{")][-1])
    out = {"workload": run["config"]["workload"], "command": command, "source_sha256_16": kernel_source_hash(),
           "note": "MfmaUtil: matrix-core busy cycles over (GPU active cycles x SIMDs), percent, averaged over "
                   "dispatches; MfmaFlops: counted matrix-core flops per dispatch (including the zero padding of "
                   "partial tiles); algorithmic flops: block-sparse flops per launch from the same run",
           "kernels": {}}
    extra = [("mix1_heavy_gemm", "gemm_grouped_kernel<float"), ("heavy_skinny", "skinny_mfma_kernel<float")]
    for slot, sym in list(KERNEL_SYMBOLS.items()) + extra:
        ds = [d for d, n in names.items() if sym in n and "MfmaUtil" in per[d]]
        heavy = slot in ("mix1_heavy_gemm", "heavy_skinny")
        if not ds or (not heavy and slot not in run["kernels"]):
            continue
        util = sum(per[d]["MfmaUtil"] for d in ds) / len(ds)
        mf = sum(per[d].get("MfmaFlops", 0.0) for d in ds) / len(ds)
        k = run["kernels"].get(slot, {})
        alg = k["tflops"] * 1e12 * k["ms"] * 1e-3 / k["launches"] if k.get("launches") else None
        key = {"mix1_heavy_gemm": "heavy_gemm_grouped (more than 64 rows)",
               "heavy_skinny": "heavy_gemm_skinny (at most 64 rows)"}.get(slot, slot)
        out["kernels"][key] = {
            "symbol": sym, "dispatches": len(ds), "mfma_util_percent": round(util, 2),
            "mfma_flops_per_dispatch": mf, "algorithmic_flops_per_launch": None if heavy else alg}
    return out


def stats_summary(stats_csv, bench_json, command, top=30):
    """Format a `rocprofv3 --kernel-trace --stats` kernel_stats.csv together with the JSON
    line the profiled bench.py run printed: the run's configuration, bench.py's own per-slot
    timing (HIP events) beside the profiler's per-kernel totals, and the kernel sources' hash."""
    import csv

    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    with open(bench_json) as f:
        run = json.loads([ln for ln in f if ln.startswith("{")][-1])
    cfg = run["config"]
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    calls = sum(int(r["Calls"]) for r in rows)
    conc = cfg.get("concurrent_subdomain_solves", 1)
    out = ["rocprofv3 kernel statistics: additive two-level sweep %s (L=%d, chi=%d, %d subdomains), %s products, "
           "%d concurrent subdomain solve%s" % (cfg["workload"], cfg["L"], cfg["chi"], len(cfg["subdomains"]),
                                                cfg["matvec"].upper(), conc, "" if conc == 1 else "s"),
           "command: " + command,
           "product kernel source hash (bsheff.hip + bsheff.h, sha256/16): " + kernel_source_hash(),
           "sweep under the profiler: %.3f s; products %d" % (run["value"], run["matvecs_per_sweep"]),
           "total kernel time %.3f s over %d dispatches%s" % (
               tot / 1e9, calls, "" if conc == 1 else " (summed over streams; kernels of different streams overlap)"),
           "",
           "bench.py timing of the same run (HIP events on each product's stream):"]
    for k, v in run["kernels"].items():
        sym = KERNEL_SYMBOLS.get(k, "")
        prof = [r for r in rows if sym and sym in r["Name"]]
        pavg = ("  rocprofv3 %8.1f us/launch" % (sum(float(r["TotalDurationNs"]) for r in prof) / 1e3 /
                                                max(sum(int(r["Calls"]) for r in prof), 1))) if prof else ""
        out.append("  %-20s %8.1f ms %5d launches %8.1f us/launch%s" % (
            k, v["ms"], v["launches"], v["ms"] * 1e3 / max(v["launches"], 1), pavg))
    rl = run["roofline"]
    out.append("  roofline kernel: %s, %.1f us/launch, %s %.1f of %.1f %s (frac %.4f)" % (
        rl["kernel"], rl["avg_launch_us"], rl["bound"], rl["achieved"], rl["peak"], rl["unit"], rl["frac"]))
    out += ["", " total_s   calls    avg_us   pct  kernel"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        out.append("%8.3f %7s %9.1f %5.1f  %s" % (float(r["TotalDurationNs"]) / 1e9, r["Calls"],
                                                  float(r["AverageNs"]) / 1e3,
                                                  100 * float(r["TotalDurationNs"]) / tot, r["Name"][:100]))
    return "\n".join(out)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, lengths, gpu_flops_heff, budget_s, coarse_k=1, one_site=False):
    """The oracle (oracle.chain with the oracle's own MPO, dense in the bond indices) as
    it stands, timed on the host cores for a bounded sample of this workload: blocks of
    8 output rows of its two-site product at the middle window (the product restricted to
    those bra rows of the left environment is exactly those rows of the full product).
    The measured rate extrapolates, by dense-bond flop counts, to the sweep's products
    (their count from the GPU run) and to the oracle's own environment updates (Step 1,
    the subdomain sweeps, and its coarse step's chains over all sites for every pair of
    states)."""
    import numpy as np

    import seeded_inputs as S
    from oracle import chain as CH
    from oracle import mpo as OM

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:
        threads = os.cpu_count() or 1
    L, r = w.L, w.chi
    # channel counts of the Hamiltonian's MPO at every bond (2 + 4L + 8m^2 - 2m pairs on
    # the smaller side); the sampled window's cores are seeded random sparse cores of
    # those shapes with five entries per output channel (building the oracle's own MPO
    # at L = 32 takes minutes of pure Python, and the sample times arithmetic, not values)
    Rb = [1] + [2 + 4 * L + 8 * min(k, L - k) ** 2 - 2 * min(k, L - k) for k in range(1, L)] + [1]
    b = L // 2 - 3
    RA, RB, RC = Rb[b], Rb[b + 1], Rb[b + 2]
    om = OM.OracleMPO(2, [RA, RB, RC], [S.random_sparse_mpo_core(RA, RB, 5, 11),
                                         S.random_sparse_mpo_core(RB, RC, 5, 12)])
    W1, W2 = CH.site_ops(om, 0), CH.site_ops(om, 1)
    rng = np.random.default_rng(5)
    # one-site: the product of the first site alone (heff1_apply), right environment at bond b+1
    x = rng.standard_normal((r, 4, r) if one_site else (r, 4, 4, r))
    Renv = rng.standard_normal((r, RB if one_site else RC, r))
    rows = 8
    t0 = time.perf_counter()
    nblk = 0
    while True:
        Lrows = rng.standard_normal((rows, RA, r))
        if one_site:
            CH.heff1_apply(Lrows, W1, Renv, x)
        else:
            CH.heff_apply(Lrows, W1, W2, Renv, x)
        nblk += 1
        if time.perf_counter() - t0 > budget_s or nblk * rows >= r:
            break
    t_blk = (time.perf_counter() - t0) / nblk
    t_mv = t_blk * r / rows
    f_mv = (2.0 * 4.0 * r * r * (RA * r + RB * r) if one_site else 2.0 * 16.0 * r * r * (RA * r + RC * r))
    rate = f_mv / t_mv  # the oracle's dense-bond flop rate on this host
    # the oracle's environment updates per sweep, dense-bond flops 4 n R r^3 each (mean R)
    Rm = float(np.mean(Rb[1:-1]))
    f_env = 2.0 * 4 * r * r * (2 * Rm * r)
    n_env = 2 * (L - 1) + sum(max(m - 1, 0) for m in lengths)
    n_states = coarse_k * len(lengths) + 1
    n_env += n_states * (n_states + 1) // 2 * L + L  # coarse sandwiches + final energy chain
    total = gpu_flops_heff / rate + n_env * f_env / rate
    return {
        "value": total, "unit": "s/sweep", "cores": int(threads), "kind": "oracle",
        "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count(),
        "sample": (f"{nblk} blocks of {rows} output rows of the oracle's "
                   f"{'one-site product (oracle.chain.heff1_apply' if one_site else 'two-site product (oracle.chain.heff_apply'}, "
                   f"its own MPO) at window ({b},{b + 1}), RA={RA}, RC={RC}, r={r}: {t_blk:.2f} s per block, "
                   f"{rate / 1e9:.1f} GFLOP/s dense-bond; extrapolated by dense-bond flops to the sweep's "
                   f"products ({gpu_flops_heff:.3e} flop) plus {n_env} oracle environment updates "
                   f"({f_env:.2e} flop each at the mean channel count); SVDs, QR and the oracle's MPO build "
                   f"not included; the sampled window's MPO cores are seeded random sparse cores of the "
                   f"workload's channel counts"),
    }


def breakdown_of(names, stats):
    return {names[i]: {"ms": round(float(stats[i, 0]), 1), "launches": int(stats[i, 1]),
                       "tflops": round(float(stats[i, 2] / max(stats[i, 0], 1e-9) / 1e9), 2),
                       "gbs": round(float(stats[i, 3] / max(stats[i, 0], 1e-9) / 1e6), 1)}
            for i in range(len(names)) if stats[i, 1] > 0}


def roofline_of(names, stats, prec):
    """Roofline of the dominant kernel of the product (largest total time): compute-bound
    if its algorithmic intensity is above the ridge point of its precision, else HBM-bound."""
    import numpy as np

    dom = int(np.argmax(stats[:, 0]))
    ms, launches, flops, nbytes = stats[dom]
    per_launch_s = ms * 1e-3 / max(launches, 1)
    ridge = PEAK[prec] * 1e12 / (HBM_PEAK * 1e9)
    if nbytes > 0 and flops / nbytes > ridge:
        achieved = flops / max(launches, 1) / per_launch_s / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK[prec], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK[prec], 4)}
    else:
        achieved = nbytes / max(launches, 1) / per_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK, 4)}
    roof.update({"traffic": None, "kernel": names[dom], "avg_launch_us": round(per_launch_s * 1e6, 1),
                 "algorithmic_flops_per_launch": flops / max(launches, 1),
                 "algorithmic_bytes_per_launch": nbytes / max(launches, 1)})
    return roof, breakdown_of(names, stats)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dav-maxiter", type=int, default=0)
    ap.add_argument("--chi", type=int, default=0)
    ap.add_argument("--sub-workers", type=int, default=0,
                    help="concurrent subdomain solves (0: the library default of 4; 1: one after another)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the sweep, run a plain elementwise copy of 1 GiB (FP32) three times: the known-size "
                         "kernel that calibrates the HBM byte counters")
    ap.add_argument("--traffic-from", nargs=3, metavar=("READ_CSV", "WRITE_CSV", "RUN_JSON"),
                    help="reduce the counter files of two rocprofv3 --pmc runs (the read-request counters "
                         "TCC_EA0_RDREQ/_32B/_128B/TCC_BUBBLE or FETCH_SIZE; WRITE_SIZE) of "
                         "bench.py --copy-probe, and that run's JSON line, to the traffic summary this script reads; "
                         "prints it and exits (no GPU)")
    ap.add_argument("--traffic-commands", nargs="*", default=[],
                    help="the rocprofv3 commands that produced the counter files (recorded in the summary)")
    ap.add_argument("--stats-from", nargs=2, metavar=("STATS_CSV", "RUN_JSON"),
                    help="format a rocprofv3 --stats kernel_stats.csv and the JSON line of the profiled run; "
                         "prints the summary and exits (no GPU)")
    ap.add_argument("--mfma-from", nargs=2, metavar=("PMC_CSV", "RUN_JSON"),
                    help="reduce a rocprofv3 --pmc MfmaUtil MfmaFlops counter file of the product kernels and the "
                         "run's JSON line to per-kernel matrix-core utilisation; prints it and exits (no GPU)")
    ap.add_argument("--stats-command", default="",
                    help="the rocprofv3 command that produced the kernel statistics (recorded in the summary)")
    ap.add_argument("--capped", action="store_true",
                    help="instead of converged local solves: residual tolerance 1e-5 (FP32) and at most "
                         "--dav-maxiter (default 40) products per local solve, no refinement (fixed work per window)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-product sweep after the timed steps")
    ap.add_argument("--matvec", choices=("f64", "f32", "bf16"), default=None,
                    help="product precision instead of the workload's own")
    ap.add_argument("--linear", action="store_true",
                    help="the linear-system functional 1/2 <X,AX> - <F,X> (A: the workload's Hamiltonian shifted "
                         "to be positive definite, F: a random TT of bond dimension --chi-f; FP64 products)")
    ap.add_argument("--chi-f", type=int, default=64)
    ap.add_argument("--lengths", default="",
                    help="subdomain lengths instead of the workload's: comma-separated, or one integer m for "
                         "subdomains of m sites")
    ap.add_argument("--precontract", type=int, default=2, choices=(0, 1, 2),
                    help="site tensors contracted with their environment once per window: 2 both, 1 left, 0 none")
    ap.add_argument("--graphs", action="store_true",
                    help="replay each local problem's products from a HIP graph of their launches")
    ap.add_argument("--coarse-krylov", action="store_true",
                    help="Step 3 by Lanczos without forming the coarse Hamiltonian matrix")
    ap.add_argument("--one-site", action="store_true",
                    help="one-site micro-steps (Algorithm 2, one-site branch; FP64 products) instead of two-site")
    ap.add_argument("--coarse-k", type=int, default=1,
                    help="local eigenvectors kept per subdomain for the coarse space (Extension One)")
    ap.add_argument("--lowprec-tol", type=float, default=1e-5,
                    help="relative residual at which the low-precision Davidson phase hands over to the "
                         "FP64-anchored refinement")
    args = ap.parse_args()
    if args.stats_from:
        print(stats_summary(*args.stats_from, args.stats_command))
        return
    if args.mfma_from:
        print(json.dumps(mfma_summary(*args.mfma_from, args.stats_command), indent=1))
        return
    if args.traffic_from:
        print(json.dumps(traffic_summary(*args.traffic_from, args.traffic_commands), indent=1))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the additive sweep is measured on a single MI355X "
              "(the multi-GPU distribution of subdomains is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import seeded_inputs as S
    from paper_2505_23429_amd.api import Context
    from paper_2505_23429_amd.mpo import build_mpo

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w, lengths = workload(args.workload)
    if args.lengths:
        parts = [int(x) for x in args.lengths.split(",")]
        if len(parts) == 1:
            m = parts[0]
            lengths = [m] * (w.L // m) + ([w.L % m] if w.L % m else [])
        else:
            lengths = parts
        if sum(lengths) != w.L:
            raise SystemExit(f"--lengths must sum to L = {w.L}")
    chi = args.chi or w.chi
    t0 = time.perf_counter()
    if args.linear:
        h, B, sigma, Fcores, Flabels = S.linear_system(w.L, w.n_elec, w.seed, args.chi_f)
    else:
        h, B = S.integrals(w.L, w.n_factors, w.seed)
    mpo = build_mpo(h, B)
    cores, labels = S.random_mps(w.L, w.n_elec, w.two_sz, chi, w.seed + 1)
    if args.linear:
        cores = S.unit_tt(cores)  # the linear functional depends on the iterate's norm
    log(f"setup: MPO R_mid={mpo.R[w.L // 2]} nnz={sum(mpo.nnz())} in {time.perf_counter() - t0:.1f}s")
    prec = "f64" if (args.one_site or args.linear) else (args.matvec or w.matvec_prec)
    functional = "linear" if args.linear else "eig"
    tol, maxiter, refine = w.dav_tol, args.dav_maxiter or 4000, prec != "f64"
    if args.capped:
        tol, maxiter, refine = (w.dav_tol if prec == "f64" else 1e-5), args.dav_maxiter or 40, False
    ctx = Context(chi=chi, dav_tol=tol, dav_maxiter=maxiter, dav_maxsub=24, matvec_prec=prec,
                  refine_fp64=refine, lowprec_tol=args.lowprec_tol, sub_workers=args.sub_workers,
                  coarse_k=args.coarse_k, one_site=args.one_site, functional=functional,
                  coarse_krylov=args.coarse_krylov, graph_products=args.graphs,
                  precontract=args.precontract)
    workers = min(args.sub_workers or 4, len(lengths))
    ctx.set_mpo(mpo)
    if args.linear:
        ctx.set_rhs(Fcores, Flabels)
    # host -> device hand-over (PCIe) and device left-orthogonalisation: outside the timed region
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.set_mps(cores, labels)
    torch.cuda.synchronize()
    t_upload = time.perf_counter() - t
    ctx.checkpoint()
    log(f"set_mps (host upload + device orthogonalisation): {t_upload:.2f}s")

    def step():
        # every step restarts from the same device-resident iterate
        ctx.checkpoint(restore=True)
        return ctx.sweep(lengths)

    for i in range(args.warmup):
        t = time.perf_counter()
        rep = step()
        log(f"warmup {i}: {time.perf_counter() - t:.2f}s E_after={rep['E_after']:.8f}")
    ctx.kernel_timing(enable=True, reset=True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    reps = []
    for i in range(args.steps):
        t = time.perf_counter()
        reps.append(step())
        log(f"step {i}: {time.perf_counter() - t:.2f}s E_before={reps[-1]['E_before']:.6f} "
            f"lambda={reps[-1]['lambda']:.8f} E_after={reps[-1]['E_after']:.8f} "
            f"matvecs={list(reps[-1]['matvecs'])}")
    torch.cuda.synchronize()
    te = time.perf_counter()
    stats = ctx.kernel_timing(enable=False, reset=True)
    sec = (te - ts) / args.steps
    fl = sum(r["flops_heff"] for r in reps)
    names = (Context.KERNELS_ONE_SITE if args.one_site else
             (Context.KERNELS, Context.KERNELS_LEFT_OPERATOR, Context.KERNELS_PRECONTRACTED)[args.precontract])
    kernels_timed = breakdown_of(names, stats)
    iso_note = "timed region (one solve at a time)"
    if workers > 1:
        # With concurrent solves the kernels of the other workers' streams run alongside
        # each product kernel, so HIP-event durations of the timed region include them.
        # The roofline comes from one more sweep, untimed, with the solves one after
        # another (same input, same kernels): the configuration whose rocprofv3 kernel
        # trace is committed.
        ctx.close()
        ctx1 = Context(chi=chi, dav_tol=tol, dav_maxiter=maxiter, dav_maxsub=24, matvec_prec=prec,
                       refine_fp64=refine, lowprec_tol=args.lowprec_tol, sub_workers=1,
                       coarse_k=args.coarse_k, one_site=args.one_site, functional=functional,
                  coarse_krylov=args.coarse_krylov, graph_products=args.graphs,
                  precontract=args.precontract)
        ctx1.set_mpo(mpo)
        if args.linear:
            ctx1.set_rhs(Fcores, Flabels)
        ctx1.set_mps(cores, labels)
        ctx1.kernel_timing(enable=True, reset=True)
        t = time.perf_counter()
        r1 = ctx1.sweep(lengths)
        torch.cuda.synchronize()
        log(f"one-solve-at-a-time pass: {time.perf_counter() - t:.2f}s E_after={r1['E_after']:.8f}")
        stats = ctx1.kernel_timing(enable=False, reset=True)
        ctx1.close()
        iso_note = "one more sweep after the timed steps with the subdomain solves one after another"
        iso_steps = 1
    else:
        iso_steps = args.steps
    roof, breakdown = roofline_of(names, stats, prec)
    roof["measured"] = iso_note
    # per-sweep product time and block-sparse flops of the pass the stats come from
    heff_s_sweep = float(stats[:, 0].sum()) * 1e-3 / iso_steps
    heff_fl_sweep = float(stats[:, 2].sum()) / iso_steps
    out = {
        "metric": "sec per two-level sweep + H_eff TFLOP/s at chi=512; batched/mixed vs FP64, dE<1e-6",
        "value": round(sec, 4), "unit": "s/sweep", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 2), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": w.name, "L": w.L, "n_elec": w.n_elec, "chi": chi, "subdomains": lengths,
                   "matvec": prec, "rayleigh_ritz": "f64", "coarse": "f64", "dav_tol": tol,
                   "dav_max_products": maxiter, "fp64_refinement": refine,
                   "lowprec_handover": args.lowprec_tol if refine else None,
                   "integrals_seed": w.seed, "mps_seed": w.seed + 1, "parallelism": "single-gpu",
                   "concurrent_subdomain_solves": workers, "coarse_k": args.coarse_k,
                   "micro_step": "one-site" if args.one_site else "two-site",
                   "coarse_solve": "krylov (no coarse matrix)" if args.coarse_krylov else "explicit matrices",
                   "graph_products": bool(args.graphs),
                   "precontracted": ("none (L x, sparse W1 and W2 mixes, R in every product)",
                                     "left (L W1 once per window)",
                                     "left and right (L W1, W2 R once per window)")[args.precontract],
                   "functional": "linear (1/2 <X,AX> - <F,X>)" if args.linear else "eigenvalue (Rayleigh quotient)",
                   **({"chi_f": args.chi_f, "shift_sigma": sigma} if args.linear else {})},
        "heff_tflops_block_sparse": round(heff_fl_sweep / max(heff_s_sweep, 1e-12) / 1e12, 3),
        "heff_block_sparse_flops_per_sweep": heff_fl_sweep,
        "heff_seconds_per_sweep": round(heff_s_sweep, 3),
        "matvecs_per_sweep": int(sum(int(np.sum(r["matvecs"])) for r in reps) / args.steps),
        "fp64_matvecs_per_sweep": int(sum(int(np.sum(r["matvecs_f64"])) for r in reps) / args.steps),
        "E_after": reps[-1]["E_after"], "lambda": reps[-1]["lambda"], "E_before": reps[-1]["E_before"],
        "roofline": roof, "kernels": breakdown, "kernels_timed_region": kernels_timed,
        "phases_s": {k: round(sum(r["phase_seconds"][i] for r in reps) / args.steps, 3) for i, k in enumerate(
            ("lq", "env_step1", "window_setup", "davidson", "split", "env_sweep", "coarse", "compress",
             "step2_wall"))},
    }
    out["set_mps_s"] = round(t_upload, 3)
    out["coarse_matvecs"] = int(reps[-1].get("coarse_matvecs", 0))
    out["statuses"] = sorted({int(r["status"]) for r in reps})
    if not args.no_fp64 and prec != "f64":
        # the same sweep with FP64 products on the same GPU (same input, same solver settings);
        # the measured context's device memory is released first
        ctx.close()
        ctx64 = Context(chi=chi, dav_tol=tol, dav_maxiter=maxiter, dav_maxsub=24,
                        matvec_prec="f64", refine_fp64=False, sub_workers=args.sub_workers,
                        coarse_k=args.coarse_k, precontract=args.precontract)
        ctx64.set_mpo(mpo)
        ctx64.set_mps(cores, labels)
        ctx64.checkpoint()
        r64 = ctx64.sweep(lengths)  # warm-up of the FP64 path (allocator, tables)
        ctx64.checkpoint(restore=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r64 = ctx64.sweep(lengths)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t
        log(f"fp64 sweep: {t64:.2f}s E_after={r64['E_after']:.8f}")
        out["fp64_path"] = {"s_per_sweep": round(t64, 4), "speedup_of_timed_path": round(t64 / sec, 3),
                            "status": int(r64["status"]), "lambda": r64["lambda"],
                            "E_after": r64["E_after"], "dE_after": abs(r64["E_after"] - reps[-1]["E_after"]),
                            "dlambda": abs(r64["lambda"] - reps[-1]["lambda"]),
                            "matvecs": int(np.sum(r64["matvecs"])),
                            "dE_local_max": float(np.abs(np.asarray(r64["E_local"]) -
                                                         np.asarray(reps[-1]["E_local"])).max())}
        ctx64.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, lengths, fl / args.steps, args.cpu_seconds, args.coarse_k, args.one_site)
    if args.copy_probe:
        n = (1 << 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        for _ in range(3):
            dst = src * 1.0  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log(f"copy probe: 3 x (read 1 GiB + write 1 GiB), result {float(dst[0])}")
        del src, dst
    # The counter runs sample the first products of every window (a full sweep under
    # counter collection is too slow), so their per-launch average weights the windows
    # differently from this run: traffic is the measured HBM/algorithmic ratio of the
    # kernel times this run's algorithmic bytes per launch; the sample's own figure is kept.
    rec = measured_traffic(roof["kernel"])
    if rec is not None:
        ratio = rec["traffic_over_algorithmic"]
        roof["traffic"] = round(ratio * roof["algorithmic_bytes_per_launch"])
        roof["traffic_over_algorithmic"] = ratio
        roof["traffic_sample_bytes_per_launch"] = rec["hbm_bytes_per_launch"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
