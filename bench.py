#!/usr/bin/env python3
"""Throughput benchmark of the TPC CA + Kalman track finder on one MI355X.

Workload: the central-Pb-Pb-shaped event (36 sectors, 18,000 primaries +
4,000 displaced secondaries, 5 % noise, 10 % merged-cluster doubling, ~3.8 M
FP32 clusters), resident in HBM.  One step = one tpcca_track call: binning,
neighbour finding, link cleaning, start hits, tracklet construction,
selection and final fit, with the outputs complete on return.

Prints one JSON line: clusters/s, ms per step, the roofline position of the
dominant kernel (its algorithmic bytes per launch over its average duration,
measured with HIP events on the library's stream inside the timed region),
and the CPU oracle timed on a bounded sample of the same event.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cluster of each phase kernel: what the kernel must read and write per cluster.
ALGO_BYTES_PER_CLUSTER = {
    "rows": 52.0,        # read 16 B bucketed (x, y, z, id); write 20 B canonical + 16 B grid entry
    "links": 44.0,       # read 12 B own coordinates + ~2 x 16 B window candidates; write 8 B links
    "tracklets": 44.0,   # chain coords + links, ~2 window candidates of 16 B, 4 B hit slot
    "refit": 16.0,       # 12 B coordinates + 4 B owner check per fitted hit
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--phase-steps", type=int, default=5,
                    help="tracking calls with phase events after the timed ones (per-phase times)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sectors", default="0,13,18",
                    help="sectors of the single-threaded oracle sample")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the multi-threaded oracle sample (0: the usable cores, at most 16)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-event batching leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the calibration-gradient leg")
    ap.add_argument("--no-timeframe", action="store_true", help="skip the time-frame leg")
    ap.add_argument("--no-its", action="store_true", help="skip the ITS leg")
    ap.add_argument("--grad-only", action="store_true",
                    help="only run the calibration-gradient leg (for its kernel trace)")
    ap.add_argument("--its-only", action="store_true", help="only run the ITS leg (for its kernel trace)")
    ap.add_argument("--its-workloads", default="ITS-pp,ITS-mb,ITS-central",
                    help="ITS workloads of the ITS leg (comma-separated)")
    ap.add_argument("--its-no-single", action="store_true",
                    help="ITS leg: time the batches only, not the one-event calls")
    ap.add_argument("--timeframe-only", action="store_true",
                    help="only run the time-frame leg (for its kernel trace)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 64-event batch calls (default tuning, for their kernel trace)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run device copies of this many MiB (calibrates PMC byte counters)")
    ap.add_argument("--pmc-summary", default="",
                    help="only summarise rocprofv3 output under this folder into profiles/")
    args = ap.parse_args()
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.grad_only:
        import torch
        from paper_1712_09434_amd import Tracker
        print(json.dumps({"grad": grad_leg(Tracker, torch.device("cuda:0"))}), flush=True)
        return
    if args.its_only:
        import torch
        print(json.dumps({"its": its_leg(torch.device("cuda:0"), workloads=args.its_workloads.split(","),
                                         single=not args.its_no_single)}), flush=True)
        return
    if args.batch_only:
        import torch
        from paper_1712_09434_amd import Tracker
        print(json.dumps({"batch": batch_trace_leg(args, Tracker, torch.device("cuda:0"))}), flush=True)
        return
    if args.timeframe_only:
        import torch
        import synth
        from paper_1712_09434_amd import Tracker
        trk = Tracker.from_geometry(synth.default_geometry())
        print(json.dumps({"timeframe": timeframe_leg(trk, torch.device("cuda:0"))}), flush=True)
        trk.close()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the tracker shards by event and sector with no exchange, "
              "and this benchmark runs and reports the single-GPU share only (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1712_09434_amd import Tracker

    dev = torch.device("cuda:0")
    log("generating the central-Pb-Pb-shaped event")
    ev = synth.make_config("C3")
    n = ev.n
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    x, y, z, row, sec = t(ev.x), t(ev.y), t(ev.z), t(ev.row), t(ev.sector)
    trk = Tracker.from_geometry(ev.geom)
    log(f"{n} clusters resident; warmup {args.warmup}")
    for _ in range(args.warmup):
        out = trk.track(x, y, z, row, sec)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = trk.track(x, y, z, row, sec)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # per-phase times from separate calls: the library's HIP events between
    # the phases add about 30 us to a call, so they stay out of the timed ones
    trk.set_phase_timing(True)
    for _ in range(args.phase_steps):
        trk.track(x, y, z, row, sec)
    torch.cuda.synchronize()
    phases, calls = trk.phase_times()
    trk.set_phase_timing(False)
    ms = dt / args.steps * 1e3
    value = n / (dt / args.steps)
    n_tracks, n_hits = out.n_tracks, int(out.hit_id.numel())
    log(f"{ms:.3f} ms/step, {value:.3e} clusters/s, {n_tracks} tracks; phases "
        + ", ".join(f"{k}={v:.3f}" for k, v in phases.items()))

    dom = max(ALGO_BYTES_PER_CLUSTER, key=lambda k: phases.get(k, 0.0))
    dom_ms = phases[dom]
    algo_bytes = ALGO_BYTES_PER_CLUSTER[dom] * n
    achieved = algo_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(f"k_{dom}")
    # counted bytes (FETCH_SIZE, which also counts Infinity Cache hits, plus
    # WRITE_SIZE, both scaled by a plain copy) over the same kernel time
    traffic_gbs = None if traffic is None else traffic / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": f"k_{dom}", "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                "traffic": traffic, "kernel_ms": round(dom_ms, 4),
                "traffic_gbs": None if traffic_gbs is None else round(traffic_gbs, 1),
                "traffic_frac": None if traffic_gbs is None else round(traffic_gbs / HBM_PEAK_GBS, 4),
                "sq": measured_valu_issue(f"k_{dom}"),
                "read_bytes_exact": measured_read_bytes(f"k_{dom}"),
                "algo_bytes_per_launch": algo_bytes}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ev, args)

    merge = merge_leg(trk, (x, y, z, row, sec), out, args)
    batch = None if args.no_batch else batch_leg(args, Tracker, dev)
    timeframe = None if args.no_timeframe else timeframe_leg(trk, dev)
    its = None if args.no_its else its_leg(dev)
    grad = None if args.no_grad else grad_leg(Tracker, dev)

    line = {
        "metric": "clusters/sec tracked (central Pb-Pb-shaped event, 1 GPU)",
        "value": value, "unit": "clusters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "C3 central-Pb-Pb-shaped event: 36 sectors, 159 rows, 18000 primaries "
                               "+ 4000 secondaries, 5% noise, 10% doubling, seed 1003",
                   "clusters": n, "tracks": n_tracks, "hits": n_hits},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phase_ms": {k: round(v, 4) for k, v in phases.items()},
        "merge": merge,
        "batch": batch,
        "timeframe": timeframe,
        "its": its,
        "grad": grad,
    }
    trk.close()
    print(json.dumps(line), flush=True)


# every file holding kernels of the profiled workloads (tracking, merger,
# calibration gradient, time frame, ITS)
KERNEL_SOURCES = ("paper_1712_09434_amd/csrc/tpcca_kernels.hip", "paper_1712_09434_amd/csrc/kf_device.hpp",
                  "paper_1712_09434_amd/csrc/internal.hpp", "paper_1712_09434_amd/csrc/kf_c2.hpp",
                  "paper_1712_09434_amd/csrc/calib_device.hpp", "paper_1712_09434_amd/csrc/tpcca_merge.hip",
                  "paper_1712_09434_amd/csrc/merge_internal.hpp", "paper_1712_09434_amd/csrc/tpcca_calib.hip",
                  "paper_1712_09434_amd/csrc/calib_internal.hpp", "paper_1712_09434_amd/csrc/tpcca_timeframe.hip",
                  "paper_1712_09434_amd/csrc/timeframe_internal.hpp", "paper_1712_09434_amd/csrc/tpcca_its.hip")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "tracking_c3_traffic.md")
PMC_BENCH_CMD = ("python3 bench.py --steps 20 --warmup 3 --no-cpu-baseline --no-batch --no-grad --no-timeframe "
                 "--no-its")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = next(json.loads(l[len("record: "):]) for l in f if l.startswith("record: "))
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def measured_read_bytes(kernel: str):
    """Exact L2-miss read bytes per launch of `kernel` (request sizes
    resolved) from the committed counter summary, or None."""
    try:
        with open(os.path.join(ROOT, "profiles", "tracking_c3_read_requests.md")) as f:
            rec = next(json.loads(l[len("record: "):]) for l in f if l.startswith("record: "))
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("read_bytes_per_launch", {}).get(kernel)


def measured_valu_issue(kernel: str):
    """VALU issue time over traced duration of `kernel` from the committed
    SQ-counter summary, or None if there is none or the kernel sources
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "tracking_c3_sq_counters.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    if f"sha256 `{kernel_source_hash()}`" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if cells and cells[0] == kernel and len(cells) >= 10:
            try:
                return {"valu_issue_frac": float(cells[5]), "waves_per_simd": float(cells[6]),
                        "valu_busy": float(cells[7]), "valu_lanes": float(cells[8]), "wait_frac": float(cells[9])}
            except ValueError:
                return None
    return None


def pmc_summary(folder: str):
    """Per-kernel FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the benchmark,
    scaled by what the same counters read for a plain copy of 1 GiB, written
    to profiles/tracking_c3_traffic.md with the kernel-source hash."""
    import csv, glob, re
    from collections import defaultdict

    def load(sub):
        out = defaultdict(list)
        for f in glob.glob(os.path.join(folder, sub, "**", "*counter_collection*.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("tpcca::(anonymous namespace)::", ""))
                name = re.sub(r"^void ", "", name)
                out[name].append(float(r["Counter_Value"]))
        return out

    fetch, write = load("pmc_fetch"), load("pmc_write")
    cf, cw = load("pmc_copy_fetch"), load("pmc_copy_write")
    if fetch and write and cf and cw:
        big = lambda d: max(max(v) for v in d.values())
        kib = 1024 * 1024
        sf, sw = kib / big(cf), kib / big(cw)
        mean = lambda v: sum(v) / len(v)
        rows, rec = [], {}
        for k in sorted(set(fetch) | set(write), key=lambda k: -mean(fetch.get(k, [0]))):
            if not k.startswith("k_"):
                continue
            f, w = mean(fetch.get(k, [0.0])), mean(write.get(k, [0.0]))
            b = (f * sf + w * sw) * 1024
            rec[k] = {"fetch_kib": round(f, 1), "write_kib": round(w, 1), "bytes_per_launch": round(b)}
            rows.append(f"| {k} | {f:,.0f} | {w:,.0f} | {b / 1e6:,.1f} |")
        record = {"workload": "C3", "source_sha256": kernel_source_hash(), "fetch_scale": round(sf, 4),
                  "write_scale": round(sw, 4), "kernels": rec}
        text = f"""# HBM traffic per kernel, central-Pb-Pb-shaped event (3.81 M clusters)

    Commands (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

        rocprofv3 --pmc FETCH_SIZE -f csv -d <out>/pmc_fetch -o fetch -- {PMC_BENCH_CMD}
        rocprofv3 --pmc WRITE_SIZE -f csv -d <out>/pmc_write -o write -- {PMC_BENCH_CMD}
        rocprofv3 --pmc FETCH_SIZE -f csv -d <out>/pmc_copy_fetch -o cfetch -- python3 bench.py --copy-probe-mib 1024
        rocprofv3 --pmc WRITE_SIZE -f csv -d <out>/pmc_copy_write -o cwrite -- python3 bench.py --copy-probe-mib 1024
        python3 bench.py --pmc-summary <out>

    Scale: a plain 1 GiB device copy reads as {big(cf):,.0f} KiB of FETCH_SIZE and {big(cw):,.0f} KiB of
    WRITE_SIZE, so fetch counts are multiplied by {sf:.4f} and write counts by {sw:.4f}.  Values are
    means over the profiled dispatches (28 calls: 3 warm-up, 20 timed, 5 with phase events).

    | Kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | scaled HBM MB/launch |
    |---|---|---|---|
    """ + "\n".join(rows) + f"""

    The record below is read by `bench.py` (roofline `traffic`) only while the kernel sources hash to
    `source_sha256`.

    record: {json.dumps(record)}
    """
        text = "\n".join(l[4:] if l.startswith("    ") else l for l in text.split("\n"))
        os.makedirs(os.path.dirname(TRAFFIC_RECORD), exist_ok=True)
        with open(TRAFFIC_RECORD, "w") as f:
            f.write(text)
        print(text)
    def load_multi(sub):
        vals, calls = defaultdict(lambda: defaultdict(float)), defaultdict(int)
        for fn in glob.glob(os.path.join(folder, sub, "**", "*counter_collection*.csv"), recursive=True):
            for r in csv.DictReader(open(fn)):
                name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("tpcca::(anonymous namespace)::", ""))
                name = re.sub(r"^void ", "", name)
                vals[name][r["Counter_Name"]] += float(r["Counter_Value"])
                if r["Counter_Name"] == "TCC_EA0_RDREQ_sum":
                    calls[name] += 1
        return vals, calls

    rq, rqn = load_multi("pmc_req")
    cq, cqn = load_multi("pmc_req_copy")
    if rq and cq:
        def split(v, c):
            q = {k: x / max(c, 1) for k, x in v.items()}
            n, n32 = q.get("TCC_EA0_RDREQ_sum", 0.0), q.get("TCC_EA0_RDREQ_32B_sum", 0.0)
            n64, n128 = q.get("TCC_EA0_RDREQ_64B_sum", 0.0), q.get("TCC_EA0_RDREQ_128B_sum", 0.0)
            exact = 32 * n32 + 64 * n64 + 128 * n128
            fetch = 32 * n32 + 64 * (n - n32)          # FETCH_SIZE's reading (no 128-byte term seen)
            return n, n32, n64, n128, exact, fetch
        copy_name = max(cq, key=lambda k: cq[k].get("TCC_EA0_RDREQ_sum", 0.0))
        cn, c32, c64, c128, cexact, cfetch = split(cq[copy_name], cqn[copy_name])
        rows_r, rec_r = [], {}
        for k in sorted(rq, key=lambda k: -split(rq[k], rqn[k])[4]):
            if not k.startswith("k_"):
                continue
            n, n32, n64, n128, exact, fetch = split(rq[k], rqn[k])
            if exact < 1e6:
                continue
            rec_r[k] = round(exact)
            rows_r.append(f"| {k} | {n / 1e6:,.2f} | {100 * n32 / max(n, 1):.0f} / {100 * n64 / max(n, 1):.0f} / "
                          f"{100 * n128 / max(n, 1):.0f} | {exact / 1e6:,.1f} | {fetch / 1e6:,.1f} | "
                          f"{2 * fetch / 1e6:,.1f} |")
        record_r = {"workload": "C3", "source_sha256": kernel_source_hash(), "read_bytes_per_launch": rec_r}
        text_r = f"""# L2 read requests by size, central-Pb-Pb-shaped event (3.81 M clusters)

Commands (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

    rocprofv3 --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum -f csv -d <out>/pmc_req -o req -- {PMC_BENCH_CMD}
    rocprofv3 --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum -f csv -d <out>/pmc_req_copy -o reqc -- python3 bench.py --copy-probe-mib 1024
    python3 bench.py --pmc-summary <out>

Read requests from the L2 to the memory side (all XCDs), per dispatch, split by request size.
Exact bytes = 32 n(32 B) + 64 n(64 B) + 128 n(128 B).  FETCH_SIZE's expression counts every
request that is not a 32-byte one as 64 bytes (its 128-byte term reads zero here), so a plain copy,
made of 128-byte requests, reads as half its size and the copy-scaled traffic doubles FETCH_SIZE.
The plain 1 GiB copy: {cn / 1e6:,.2f} M requests, {100 * c32 / max(cn, 1):.0f} / {100 * c64 / max(cn, 1):.0f} /
{100 * c128 / max(cn, 1):.0f} % of 32 / 64 / 128 bytes, {cexact / 2**20:,.0f} MiB exact against
{cfetch / 2**20:,.0f} MiB by FETCH_SIZE's expression.  These are L2 misses: on this chip they are
served by the 256 MB Infinity Cache or by HBM, which the L2 counters do not tell apart.  Kernel
sources sha256 `{kernel_source_hash()}`.

| Kernel | Read requests (M) | 32 / 64 / 128 B (%) | Exact MB | FETCH_SIZE MB | Copy-scaled MB |
|---|---|---|---|---|---|
""" + "\n".join(rows_r) + f"""

record: {json.dumps(record_r)}
"""
        with open(os.path.join(ROOT, "profiles", "tracking_c3_read_requests.md"), "w") as f:
            f.write(text_r)
        print(text_r)
    stats = glob.glob(os.path.join(folder, "prof_c3", "**", "*kernel_stats.csv"), recursive=True)
    if stats:
        lines = []
        tot = 0.0
        for r in csv.DictReader(open(stats[0])):
            name = re.sub(r"\(.*", "", r["Name"].replace("tpcca::(anonymous namespace)::", ""))
            name = re.sub(r"^void ", "", name)
            lines.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
            tot += float(r["TotalDurationNs"])
        body = "\n".join(f"| {n} | {c} | {a:,.1f} | {p:.1f} |" for n, c, a, p in lines[:24])
        text2 = f"""# Kernel trace, central-Pb-Pb-shaped event (3.81 M clusters, one tpcca_track call per step)

Command (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

    rocprofv3 --kernel-trace --stats -f csv -d <out>/prof_c3 -o c3 -- {PMC_BENCH_CMD}
    python3 bench.py --pmc-summary <out>

28 tracking calls (3 warm-up, 20 timed, 5 with phase events); average duration per dispatch.  Kernel sources
sha256 `{kernel_source_hash()}`.

| Kernel | Calls | Average µs | % of GPU time |
|---|---|---|---|
{body}
"""
        with open(os.path.join(ROOT, "profiles", "tracking_c3_kernel_trace.md"), "w") as f:
            f.write(text2)
        print(text2)
        sq = defaultdict(lambda: defaultdict(float))
        ncalls = defaultdict(int)
        grad_stats = glob.glob(os.path.join(folder, "prof_grad", "**", "*kernel_stats.csv"), recursive=True)
        if grad_stats:
            gl = []
            for r in csv.DictReader(open(grad_stats[0])):
                name = re.sub(r"\(.*", "", r["Name"].replace("tpcca::(anonymous namespace)::", ""))
                name = re.sub(r"^void ", "", name)
                gl.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
            body_g = "\n".join(f"| {n} | {c} | {a:,.1f} | {p:.1f} |" for n, c, a, p in gl[:16])
            text_g = f"""# Kernel trace, calibration workload (20 miscalibrated full events, ~82 k tracks, ~10.8 M hits)

Command (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

    rocprofv3 --kernel-trace --stats -f csv -d <out>/prof_grad -o grad -- python3 bench.py --grad-only
    python3 bench.py --pmc-summary <out>

One tpcca_refit_grad over all tracks per call: 11 timed calls, then the 50-step Adam calibration
(132 + 50 calls) and the calibration-map tracking calls; average duration per dispatch.

| Kernel | Calls | Average µs | % of GPU time |
|---|---|---|---|
{body_g}
"""
            with open(os.path.join(ROOT, "profiles", "refit_grad_c5x20_kernel_trace.md"), "w") as f:
                f.write(text_g)
            print(text_g)
        for fn in glob.glob(os.path.join(folder, "pmc_sq", "**", "*counter_collection*.csv"), recursive=True):
            for r in csv.DictReader(open(fn)):
                name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("tpcca::(anonymous namespace)::", ""))
                name = re.sub(r"^void ", "", name)
                sq[name][r["Counter_Name"]] += float(r["Counter_Value"])
                if r["Counter_Name"] == "SQ_WAVES":
                    ncalls[name] += 1
        if sq:
            avg_us = {n: a for n, _, a, _ in lines}
            simds, cus, clock_ghz = 256 * 4, 256, 2.4
            rows3 = []
            for n in sorted(sq, key=lambda k: -avg_us.get(k, 0.0)):
                c = ncalls[n] or 1
                q = {k: v / c for k, v in sq[n].items()}
                valu = q["SQ_INSTS_VALU"]
                issue_us = valu * 4 / simds / (clock_ghz * 1e3)
                d = avg_us.get(n, 0.0)
                if d < 20.0:
                    continue
                cycles = d * clock_ghz * 1e3
                # SQ_WAVE_CYCLES, SQ_ACTIVE_INST_VALU and SQ_WAIT_ANY are quad-cycles summed over
                # the SIMDs: mean resident waves per SIMD, VALU busy per CU (the VALUBusy
                # metric's formula with the traced duration), lane utilisation (VALUUtilization's)
                waves_simd = 4 * q["SQ_WAVE_CYCLES"] / (cycles * simds)
                busy = q["SQ_ACTIVE_INST_VALU"] / (cus * cycles)
                lanes = q["SQ_THREAD_CYCLES_VALU"] / max(q["SQ_ACTIVE_INST_VALU"] * 64, 1.0)
                wait = q["SQ_WAIT_ANY"] / max(q["SQ_WAVE_CYCLES"], 1.0)
                rows3.append(f"| {n} | {q['SQ_WAVES']:,.0f} | {valu / 1e6:,.1f} | {issue_us:,.1f} | {d:,.1f} | "
                             f"{issue_us / d:.2f} | {waves_simd:.2f} | {busy:.2f} | {lanes:.2f} | {wait:.2f} |")
            text3 = f"""# SQ counters per kernel, central-Pb-Pb-shaped event (3.81 M clusters)

Command (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

    rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_WAIT_ANY SQ_INSTS_VALU SQ_INSTS_LDS -f csv -d <out>/pmc_sq -o sq -- {PMC_BENCH_CMD}
    python3 bench.py --pmc-summary <out>

Per dispatch (means over the profiled calls; the tracking call and the sector merger).  VALU issue
time = wave-64 VALU instructions x 4 cycles / (1,024 SIMDs x 2.4 GHz): the time the kernel would
take if every SIMD issued one of its VALU instructions every 4 cycles; its ratio to the traced
duration is the kernel's VALU issue utilisation.  Waves/SIMD = 4 SQ_WAVE_CYCLES (quad-cycles
summed over SIMDs) / (traced cycles x 1,024): the mean number of resident waves per SIMD (the
occupancy; at most 8).  VALU busy = SQ_ACTIVE_INST_VALU / (256 CUs x traced cycles) (the
VALUBusy metric's formula).  Lanes = SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU), the
VALUUtilization metric: the fraction of a wave's 64 lanes active in its VALU instructions.  Wait
= SQ_WAIT_ANY / SQ_WAVE_CYCLES: the fraction of resident wave time spent waiting (memory,
dependencies, barriers).  Traced durations from the kernel trace of the same command.  Kernel
sources sha256 `{kernel_source_hash()}`.

| Kernel | Waves | VALU (M wave-instr.) | VALU issue µs | Traced µs | Issue / traced | Waves/SIMD | VALU busy | Lanes | Wait |
|---|---|---|---|---|---|---|---|---|---|
""" + "\n".join(rows3) + "\n"
            with open(os.path.join(ROOT, "profiles", "tracking_c3_sq_counters.md"), "w") as f:
                f.write(text3)
            print(text3)
    tf_stats = glob.glob(os.path.join(folder, "prof_tf", "**", "*kernel_stats.csv"), recursive=True)
    if tf_stats:
        tl = []
        for r in csv.DictReader(open(tf_stats[0])):
            name = re.sub(r"\(.*", "", r["Name"].replace("tpcca::(anonymous namespace)::", ""))
            name = re.sub(r"^void ", "", name)
            tl.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
        body_t = "\n".join(f"| {n} | {c} | {a:,.1f} | {p:.1f} |" for n, c, a, p in tl[:28])
        text_t = f"""# Kernel trace, continuous-readout time frame (24 collisions over 6 drift lengths, 5.77 M clusters)

Command (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

    rocprofv3 --kernel-trace --stats -f csv -d <out>/prof_tf -o tf -- python3 bench.py --timeframe-only
    python3 bench.py --pmc-summary <out>

tpcca_track_timeframe with 6 slices of one drift length: 2 warm-up calls with the segment
outputs, 5 timed calls; average duration per dispatch (the tracking kernels run once per call
over the batch of 6 slices).

| Kernel | Calls | Average µs | % of GPU time |
|---|---|---|---|
{body_t}
"""
        with open(os.path.join(ROOT, "profiles", "timeframe_tf24_kernel_trace.md"), "w") as f:
            f.write(text_t)
        print(text_t)
    b_stats = glob.glob(os.path.join(folder, "prof_batch", "**", "*kernel_stats.csv"), recursive=True)
    if b_stats:
        bl = []
        for r in csv.DictReader(open(b_stats[0])):
            name = re.sub(r"\(.*", "", r["Name"].replace("tpcca::(anonymous namespace)::", ""))
            name = re.sub(r"^void ", "", name)
            bl.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
        body_b = "\n".join(f"| {n} | {c} | {a:,.1f} | {p:.1f} |" for n, c, a, p in bl[:20])
        text_b = f"""# Kernel trace, batch of 64 events of lognormal multiplicity (12.0 M clusters)

Command (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

    rocprofv3 --kernel-trace --stats -f csv -d <out>/prof_batch -o batch -- python3 bench.py --batch-only
    python3 bench.py --pmc-summary <out>

One tpcca_track_batch call over all 64 events per step (default launch setting): 1 warm-up and
5 timed calls; average duration per dispatch.  Row units: 366,336, of which 321,195 hold at most
64 clusters and 44,470 between 65 and 256.

| Kernel | Calls | Average µs | % of GPU time |
|---|---|---|---|
{body_b}
"""
        with open(os.path.join(ROOT, "profiles", "batch_c4x64_kernel_trace.md"), "w") as f:
            f.write(text_b)
        print(text_b)
    its_stats = glob.glob(os.path.join(folder, "prof_its", "**", "*kernel_stats.csv"), recursive=True)
    if its_stats:
        il = []
        for r in csv.DictReader(open(its_stats[0])):
            name = re.sub(r"\(.*", "", r["Name"].replace("tpcca::(anonymous namespace)::", ""))
            name = re.sub(r"^void ", "", name)
            il.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
        body_i = "\n".join(f"| {n} | {c} | {a:,.1f} | {p:.1f} |" for n, c, a, p in il[:20])
        text_i = f"""# Kernel trace, ITS standalone tracking (pp-like, minimum-bias-like and central-like events)

Command (from the repository root on a machine with the GPU, `TMPDIR=/tmp`):

    rocprofv3 --kernel-trace --stats -f csv -d <out>/prof_its -o its -- python3 bench.py --its-only --its-workloads ITS-central --its-no-single
    python3 bench.py --pmc-summary <out>

One tpcca_its_track_batch call on 20 central-like events (about 18 k clusters and 2.6 k tracks
each): 1 + 1 untimed and 5 timed calls; average duration per dispatch (one dispatch covers all
20 events).

| Kernel | Calls | Average µs | % of GPU time |
|---|---|---|---|
{body_i}
"""
        with open(os.path.join(ROOT, "profiles", "its_central_x20_kernel_trace.md"), "w") as f:
            f.write(text_i)
        print(text_i)


def copy_probe(mib: int, reps: int = 5):
    """A plain device-to-device copy of `mib` MiB, `reps` times: each copy
    reads and writes exactly mib MiB, which scales FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe_mib": mib, "reps": reps, "ms_per_copy": dt * 1e3,
                      "GBps": 2 * mib * (1 << 20) / dt / 1e9}), flush=True)


def _to_dev(ev, dev):
    import numpy as np
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t(ev.x), t(ev.y), t(ev.z), t(ev.row), t(ev.sector)


def batch_trace_leg(args, Tracker, dev, reps=5):
    """The 64-event batch alone: one warm-up and `reps` timed
    tpcca_track_batch calls with the default launch setting."""
    import torch

    import synth
    evs = [synth.make_config("C4", e) for e in range(64)]
    n = sum(e.n for e in evs)
    tens = [_to_dev(e, dev) for e in evs]
    trk = Tracker.from_geometry(evs[0].geom)
    trk.track_batch(tens)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        trk.track_batch(tens)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    trk.close()
    log(f"batch only: {n} clusters in 64 events, {dt * 1e3:.2f} ms per call")
    return {"events": 64, "clusters": n, "ms_per_call": dt * 1e3}


def batch_leg(args, Tracker, dev):
    """64 events of lognormal multiplicity: one tpcca_track_batch call vs 64
    back-to-back tpcca_track calls on the same stream (both with the tuned
    launch setting)."""
    import torch

    import synth
    from paper_1712_09434_amd import autotune

    log("generating the 64-event batch")
    evs = [synth.make_config("C4", e) for e in range(64)]
    n = sum(e.n for e in evs)
    side = torch.cuda.Stream(dev)
    with torch.cuda.stream(side):
        tens = [_to_dev(e, dev) for e in evs]
        trk = Tracker.from_geometry(evs[0].geom)
        tuned = autotune.autotune(trk, tens, reps=2, cache=None, log=log)
        best = tuned["best"]

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        t_batch = timed(lambda: trk.track_batch(tens), args.batch_reps)
        # per-phase times of the batched call (library HIP events between its kernels;
        # timing runs the phases without graph replay)
        trk.set_phase_timing(True)
        for _ in range(args.batch_reps):
            trk.track_batch(tens)
        torch.cuda.synchronize()
        batch_phases = trk.phase_times()[0]
        trk.set_phase_timing(False)

        def seq():
            for e in tens:
                trk.track(*e)

        # the sequential baseline gets its own best setting among the same candidates
        seq_best = None
        for g in sorted({0, best["tracklet_grid"]}):
            for u in (0, 1):
                trk.set_tuning(tracklet_grid=g, use_graph=u)
                t = timed(seq, args.batch_reps)
                if seq_best is None or t < seq_best[0]:
                    seq_best = (t, g, u)
        trk.close()
    t_seq = seq_best[0]
    log(f"batch: {n} clusters in 64 events: batched {t_batch * 1e3:.2f} ms, "
        f"sequential {t_seq * 1e3:.2f} ms, gain {t_seq / t_batch:.2f}; phases "
        + ", ".join(f"{k}={v:.3f}" for k, v in batch_phases.items()))
    return {"events": 64, "clusters": n, "batched_ms": t_batch * 1e3, "sequential_ms": t_seq * 1e3,
            "gain": t_seq / t_batch, "batched_clusters_per_s": n / t_batch,
            "phase_ms": {k: round(v, 4) for k, v in batch_phases.items()},
            "batched_tuning": {"tracklet_grid": best["tracklet_grid"], "use_graph": best["use_graph"]},
            "sequential_tuning": {"tracklet_grid": seq_best[1], "use_graph": seq_best[2]}}


def timeframe_leg(trk, dev, reps=5):
    """One continuous-readout time frame (24 collisions of lognormal
    multiplicity over 6 drift lengths, 5.8 M clusters) sliced per drift
    length, tracked as one batch of slices and merged across slices and
    sectors: tpcca_track_timeframe, inputs resident in HBM."""
    import numpy as np
    import torch

    import synth
    log("generating the time frame")
    tf = synth.make_tf_config("TF")
    D = synth.TF_SLICE
    ns = int(np.ceil(tf.length / D))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    cl = (t(tf.x), t(tf.y), t(tf.tau), t(tf.row), t(tf.sector))
    trk.set_phase_timing(False)
    for _ in range(2):
        merged, seg, sl, lk = trk.track_timeframe(*cl, D, ns, segments=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m = trk.track_timeframe(*cl, D, ns)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    lkn = lk.cpu().numpy()
    s = seg.sector.cpu().numpy()
    links = int((lkn >= 0).sum())
    slice_links = int(sum(1 for a in np.nonzero(lkn >= 0)[0] if s[a] == s[lkn[a]]))
    log(f"time frame: {tf.n} clusters, {ns} slices: {dt * 1e3:.2f} ms, {tf.n / dt:.3e} clusters/s; "
        f"{seg.n_tracks} segments, {links} links ({slice_links} across slices), {m.n_tracks} tracks")
    return {"workload": "24 collisions (lognormal multiplicity, 2% noise) over 6 drift lengths, seed 1006002, "
                        "sliced per drift length", "clusters": tf.n, "slices": ns, "ms_per_frame": dt * 1e3,
            "clusters_per_s": tf.n / dt, "segments": seg.n_tracks, "links": links, "slice_links": slice_links,
            "tracks": m.n_tracks}


def its_leg(dev, n_events=20, reps=5, workloads=("ITS-pp", "ITS-mb", "ITS-central"), single=True):
    """ITS standalone tracking (vertexer, tracklets, following, inward fit,
    vertex fit) of 20 events per workload (inputs resident in HBM, outputs
    marshalled beforehand): one tpcca_its_track_batch call on all 20, and one
    call per event; plus the fitted vertices against the generated ones (the
    luminous-region input)."""
    import numpy as np
    import torch

    import synth
    from paper_1712_09434_amd.its import ItsTracker
    trk = ItsTracker(synth.default_its_geometry())
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    res = {}

    def timed(fns):
        for f in fns:
            f(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for f in fns:
                f(False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / (reps * n_events)

    for name in workloads:
        evs = [synth.make_its_config(name, i) for i in range(n_events)]
        tens = [(t(e.x), t(e.y), t(e.z), t(e.layer), t(e.stave)) for e in evs]
        batch = trk.prepare_batch(tens)
        outs = batch()
        dt_b = timed([batch])
        dt_s = timed([trk.prepare_batch([c]) for c in tens]) if single else float("nan")
        ncl = sum(e.n for e in evs) / n_events
        ntrk = sum(int(o.ok.sum()) for o in outs) / n_events
        dv = np.array([np.array(o.vertex) - e.vertex for o, e in zip(outs, evs)])
        res[name] = {"clusters_per_event": ncl, "tracks_per_event": ntrk, "ms_per_event": dt_b * 1e3,
                     "events_per_s": 1.0 / dt_b, "ms_per_event_single_calls": dt_s * 1e3,
                     "vertex_residual_um": {"mean": [round(v, 2) for v in (dv.mean(0) * 1e4).tolist()],
                                            "rms": [round(v, 2) for v in (dv.std(0) * 1e4).tolist()]}}
        log(f"ITS {name}: {ncl:.0f} clusters, {ntrk:.0f} tracks per event: {dt_b * 1e3:.3f} ms per event in "
            f"batches of {n_events} ({1.0 / dt_b:.0f} events/s), {dt_s * 1e3:.3f} ms in single calls; vertex "
            f"residual rms (x, y, z) {res[name]['vertex_residual_um']['rms']} um")
    trk.close()
    return res


def merge_leg(trk, cl, seg, args, reps=20):
    """tpcca_merge on the segments of the timed event (the step after
    tracking: segments joined across sector boundaries, chains refitted)."""
    import torch
    trk.set_phase_timing(False)
    for _ in range(3):
        m, links = trk.merge(seg, cl, links=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m = trk.merge(seg, cl)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    nl = int((links >= 0).sum())
    log(f"merge: {seg.n_tracks} segments -> {m.n_tracks} tracks ({nl} links) in {dt * 1e3:.3f} ms")
    return {"segments": seg.n_tracks, "tracks": m.n_tracks, "links": nl, "ms_per_call": dt * 1e3,
            "segments_per_s": seg.n_tracks / dt}


def grad_leg(Tracker, dev, n_events=20):
    """The calibration workload: tpcca_refit_grad on the tracks of n_events
    miscalibrated full events (tracks with >= 40 hits, chi2/ndf <= 4 and a
    first hit within the first 11 pad rows; vertex and external tan(lambda)
    terms on), one call over all of them; then the 50-step Adam calibration
    from theta = 0 (prior-scaled Hessian eigen-coordinates: 132 gradient
    calls for the Hessian, then 50 steps), wall time with all work done."""
    import numpy as np
    import torch

    import synth
    from paper_1712_09434_amd import FitTracks, calibrate
    from paper_1712_09434_amd.calib import default_prior_sigma

    log(f"grad: generating {n_events} miscalibrated full events")
    evs = synth.make_configs("C5", range(n_events))
    trk = Tracker.from_geometry(evs[0].geom)
    cols = [[] for _ in range(5)]
    lists, kps, exts = [], [], []
    base = 0
    for ev in evs:
        cl = _to_dev(ev, dev)
        out = trk.track(*cl)
        nh = (out.hit_off[1:] - out.hit_off[:-1]).cpu().numpy()
        q = (out.chi2 / out.ndf).cpu().numpy()
        off = out.hit_off.cpu().numpy()
        ids = out.hit_id.cpu().numpy()
        inner_row = ev.row[ids[off[:-1]]]
        keep = np.nonzero((nh >= 40) & (q <= 4.0) & (inner_row <= 10))[0]
        lists += [ids[off[t]:off[t + 1]].astype(np.int64) + base for t in keep]
        kk = torch.from_numpy(keep).to(dev)
        kps.append(out.k_prior[kk].cpu().numpy())
        exts.append(out.p[kk, 3].cpu().numpy())   # stand-in for the external tan(lambda): timing only
        for L, a in zip(cols, (ev.x, ev.y, ev.z, ev.row, ev.sector)):
            L.append(a)
        base += ev.n
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    clusters = tuple(d(np.concatenate(c)) for c in cols)
    hoff = np.concatenate([[0], np.cumsum([len(l) for l in lists])]).astype(np.int32)
    T = len(lists)
    fit = FitTracks(clusters=clusters, hit_off=d(hoff), hit_id=d(np.concatenate(lists).astype(np.int32)),
                    k_prior=d(np.concatenate(kps).astype(np.float32)),
                    ext_tgl=d(np.concatenate(exts).astype(np.float32)),
                    use_vertex=torch.ones(T, dtype=torch.uint8, device=dev))
    th = torch.zeros(36 * 66, dtype=torch.float32, device=dev)
    trk.refit_grad(fit, th)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        trk.refit_grad(fit, th)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    H = int(hoff[-1])
    log(f"grad: {T} tracks, {H} hits from {n_events} events, {dt * 1e3:.3f} ms per refit_grad")
    sig = default_prior_sigma(36, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, hist, _ = calibrate(trk, fit, steps=50, precondition="eigen", lr_white=0.6, lr_final=1e-3,
                               betas=(0.8, 0.999), prior_sigma=sig)
    torch.cuda.synchronize()
    t_adam = time.perf_counter() - t0
    log(f"grad: 50 Adam steps (after a 132-call Hessian) in {t_adam:.3f} s; objective {hist[0]:.0f} -> {hist[-1]:.0f}")
    # the feedback: the calibration found is installed in front of tracking
    cal_map = calib_map_leg(trk, evs[0], theta, dev)
    trk.close()
    return {"workload": f"{n_events} miscalibrated full events (5000 primaries, 2% noise, seeds 1005000+)",
            "tracks": T, "hits": H, "ms_per_call": dt * 1e3, "tracks_per_s": T / dt, "hits_per_s": H / dt,
            "params": 36 * 66, "adam50_s": t_adam, "adam50_gradient_calls": 132 + 50, "calib_map": cal_map}


def calib_map_leg(trk, ev, theta, dev, reps=20):
    """Tracking of one miscalibrated full event without and with the
    calibration installed in front of binning (tpcca_set_calib): time per
    call and of the binning scatter (where the correction runs)."""
    import torch
    cl = _to_dev(ev, dev)
    res = {}
    for name, th in (("uncorrected", None), ("corrected", theta)):
        trk.set_calib(th)
        for _ in range(3):
            trk.track(*cl)
        trk.set_phase_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            trk.track(*cl)
        torch.cuda.synchronize()
        res[name] = ((time.perf_counter() - t0) / reps * 1e3, trk.phase_times()[0]["scatter"])
        trk.set_phase_timing(False)
    trk.set_calib(None)
    out = {"clusters": int(ev.n), "ms_uncorrected": res["uncorrected"][0], "ms_corrected": res["corrected"][0],
           "scatter_ms_uncorrected": res["uncorrected"][1], "scatter_ms_corrected": res["corrected"][1]}
    log(f"calibration map: {ev.n} clusters, {out['ms_uncorrected']:.3f} ms uncorrected, "
        f"{out['ms_corrected']:.3f} ms with the map (scatter {out['scatter_ms_uncorrected']:.4f} -> "
        f"{out['scatter_ms_corrected']:.4f} ms)")
    return out


def cpu_baseline(ev, args):
    """The oracle as written (FP32 mode), timed on host cores on a bounded
    sample of the same event: (i) single-threaded on a few sectors, (ii) one
    sector per thread on T threads at once (sectors are independent, so the
    event's work splits over them without change).  The reported value is
    the median of three runs of (ii); cores = T."""
    import concurrent.futures
    import numpy as np
    import oracle
    ns = int(ev.geom.n_sectors)

    def one(secs):
        mask = np.zeros(ns, np.uint8)
        mask[list(secs)] = 1
        oracle.track(ev, precision=32, sector_mask=mask)

    secs1 = [int(s) for s in args.cpu_sectors.split(",")]
    n1 = int(np.isin(ev.sector, secs1).sum())
    log(f"oracle (FP32, 1 thread) on sectors {secs1}: {n1} clusters")
    t1 = time.perf_counter()
    one(secs1)
    c1 = time.perf_counter() - t1
    log(f"oracle 1 thread {n1 / c1:.3e} clusters/s")

    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    T = args.cpu_threads or max(1, min(16, avail))
    T = min(T, ns)
    secsT = sorted({int(round(v)) for v in np.linspace(0, ns - 1, T)})
    nT = int(np.isin(ev.sector, secsT).sum())
    log(f"oracle (FP32, {len(secsT)} threads, one sector each) on sectors {secsT}: {nT} clusters, 3 runs")
    walls = []
    for _ in range(3):
        tT = time.perf_counter()
        with concurrent.futures.ThreadPoolExecutor(max_workers=len(secsT)) as pool:
            list(pool.map(lambda s: one([s]), secsT))
        walls.append(time.perf_counter() - tT)
        log(f"oracle {len(secsT)} threads {nT / walls[-1]:.3e} clusters/s")
    cT = sorted(walls)[1]
    return {"value": nT / cT, "unit": "clusters/s", "cores": len(secsT), "kind": "oracle",
            "sample": (f"C3 event: sectors {secsT} ({nT} clusters), one sector per thread on "
                       f"{len(secsT)} threads, median of 3 runs ({', '.join(f'{v:.2f}' for v in walls)} s "
                       f"wall); single-threaded on sectors {secs1} ({n1} clusters) {c1:.1f} s"),
            "runs_s": [round(v, 3) for v in walls],
            "single_thread_value": n1 / c1, "host_cpu": _cpu_model()}

def _cpu_model():
    try:
        for l in open("/proc/cpuinfo"):
            if l.startswith("model name"):
                return l.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
