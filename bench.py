"""Throughput of the NU-FDS reconstruction on one MI355X.

Default workload: the 16384^2, 120 deg full view (pitch lambda / (2 sin 60 deg), lambda = 0.5 um,
1024 seeded points with z ~ U[10, 20] mm, reconstruction at z = 15 mm onto 16384^2 output pixels).
A step is one whole reconstruction (FFT of the hologram, stretch-gather, inverse FFT, Fresnel
transform, remap) of one hologram already resident in HBM.  ``value`` is output Mpixel/s of the
complex64 path (float64 maps and phases); the complex128 path is reported beside it.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# wave64 VALU instructions the chip can issue per second: 256 CUs, each one per clock (four SIMDs of
# 16 lanes, a wave64 instruction taking four clocks on one), at 2.4 GHz; packed FP32 is not used
VALU_ISSUE_PEAK = 256 * 2.4e9
LAM = 0.5e-6

WORKLOADS = {
    # name: (N, fov_deg, z, n_points, z_lo, z_hi, seed)
    "uwa120_16k": (16384, 120.0, 15e-3, 1024, 10e-3, 20e-3, 1003),
    "wa90_4k": (4096, 90.0, 7.5e-3, 4096, 5e-3, 10e-3, 1002),
    "fov60_1k": (1024, 60.0, 3e-3, 64, 2e-3, 4e-3, 1001),
}


PROFILE_JSON = os.path.join(ROOT, "profiles", "counters_uwa120_16k.json")
PROFILE_MD = os.path.join(ROOT, "profiles", "nufds_kernels_uwa120_16k.md")
OUR_KERNELS = ("fft_pass_kernel", "fft_fixed_kernel", "row_chain_kernel", "stretch_gather_kernel", "output_gather_kernel")


def source_hash() -> str:
    """Hash of the kernel and host sources: hardware counters taken on other sources do not apply."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2410_13474_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(role):
    """HBM bytes per launch of a kernel role from the committed counter summary, or None when the
    summary is missing or was taken on different sources."""
    try:
        rec = json.load(open(PROFILE_JSON))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash() or role not in rec.get("roles", {}):
        return None
    r = rec["roles"][role]
    return r["fetch_bytes"] + r["write_bytes"]


def measured_valu(role):
    """VALU wave-instructions per launch of a kernel role (SQ_INSTS_VALU) from the committed counter
    summary, or None when missing or taken on different sources."""
    try:
        rec = json.load(open(PROFILE_JSON))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash() or role not in rec.get("roles", {}):
        return None
    return rec["roles"][role].get("valu_insts")


def summarize_profile(d):
    """rocprofv3 CSVs -> profiles/counters_uwa120_16k.json and the markdown summary."""
    import csv
    import re

    def rows(sub, name):
        import glob
        fs = sorted(glob.glob(os.path.join(d, sub, "*" + name)))
        return list(csv.DictReader(open(fs[0]))) if fs else []

    def short(k):
        k = re.sub(r"\(.*", "", k).replace("void ", "").replace("nufds::", "")
        return k.strip()

    roles = json.load(open(os.path.join(d, "roles.json")))["roles"]
    out = {"source_hash": source_hash(), "workload": "uwa120_16k", "roles": {}, "calibration": {}}
    counters = {}
    for sub, cname in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        rs = [r for r in rows(sub, "counter_collection.csv") if r["Counter_Name"] == cname]
        rs.sort(key=lambda r: int(r.get("Dispatch_Id", r.get("Correlation_Id", 0))))
        copies = [r for r in rs if "copyBuffer" in r["Kernel_Name"]]
        gmax = max((int(r["Grid_Size"]) for r in copies), default=0)
        copy = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == gmax]
        # a 1 GiB device copy reads and writes 1048576 KiB
        factor = 1048576.0 / (sum(copy) / len(copy)) if copy else 1.0
        out["calibration"][cname] = {"copy_kib": sum(copy) / len(copy) if copy else None, "factor": factor}
        ours = [r for r in rs if any(k in r["Kernel_Name"] for k in OUR_KERNELS)]
        n_steps = len(ours) // len(roles)
        ours = ours[len(ours) - n_steps * len(roles):]
        per = {}
        for i, r in enumerate(ours):
            per.setdefault(roles[i % len(roles)], []).append(float(r["Counter_Value"]) * 1024 * factor)
        counters[cname] = {k: sum(v) / len(v) for k, v in per.items()}
    # VALU wave-instructions and waves per launch (no calibration: instruction counts)
    valu = {}
    for cname in ("SQ_INSTS_VALU", "SQ_WAVES"):
        rs = [r for r in rows("valu", "counter_collection.csv") if r["Counter_Name"] == cname]
        rs.sort(key=lambda r: int(r.get("Dispatch_Id", r.get("Correlation_Id", 0))))
        ours = [r for r in rs if any(k in r["Kernel_Name"] for k in OUR_KERNELS)]
        n_steps = len(ours) // len(roles)
        ours = ours[len(ours) - n_steps * len(roles):]
        per = {}
        for i, r in enumerate(ours):
            per.setdefault(roles[i % len(roles)], []).append(float(r["Counter_Value"]))
        valu[cname] = {k: sum(v) / len(v) for k, v in per.items()}
    for role in roles:
        out["roles"][role] = {"fetch_bytes": counters["FETCH_SIZE"].get(role),
                              "write_bytes": counters["WRITE_SIZE"].get(role),
                              "valu_insts": valu["SQ_INSTS_VALU"].get(role), "waves": valu["SQ_WAVES"].get(role)}
    stats = rows("trace", "kernel_stats.csv")
    out["kernel_stats"] = [{"kernel": short(r["Name"]), "calls": int(r["Calls"]),
                            "avg_ms": float(r["AverageNs"]) / 1e6} for r in stats]
    meta = json.load(open(os.path.join(d, "roles.json")))
    out["bench"] = {"ms_per_step": meta.get("ms_per_step"), "avg_ms": meta.get("avg_ms"),
                    "algorithmic_bytes": meta.get("bytes")}
    json.dump(out, open(PROFILE_JSON, "w"), indent=1)
    lines = ["# NU-FDS kernels, 16384^2 120 deg full view (complex64)", "",
             "Workload: 16384^2 hologram, pitch = lambda / (2 sin 60 deg), lambda = 0.5 um, 1024 points "
             "(seed 1003), z = 15 mm, full 16384^2 view, FrT size M = 25600.  One MI355X.", "",
             f"Sources: hash {out['source_hash']} (bench.py's source_hash of paper_2410_13474_amd/csrc); "
             "bench.py reports `roofline.traffic` only while the sources still match.", "",
             "Commands (from /tmp with TMPDIR=/tmp; R = repository root, P = an output folder):", "", "```",
             "rocprofv3 --kernel-trace --stats -d $P/trace -o run --output-format csv -- python3 $R/bench.py "
             "--steps 5 --warmup 1 --no-cpu --no-serving --no-stack --no-oversample --no-paper-model --copy-calibration --roles-out $P/roles.json",
             "rocprofv3 --pmc FETCH_SIZE -d $P/fetch -o run --output-format csv -- python3 $R/bench.py "
             "--steps 2 --warmup 0 --no-cpu --no-fp64 --no-serving --no-stack --no-oversample --no-paper-model --copy-calibration",
             "rocprofv3 --pmc WRITE_SIZE -d $P/write -o run --output-format csv -- python3 $R/bench.py "
             "--steps 2 --warmup 0 --no-cpu --no-fp64 --no-serving --no-stack --no-oversample --no-paper-model --copy-calibration",
             "rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES -d $P/valu -o run --output-format csv -- python3 $R/bench.py "
             "--steps 2 --warmup 0 --no-cpu --no-fp64 --no-serving --no-stack --no-oversample --no-paper-model",
             "python3 $R/bench.py --summarize-profile $P", "```", "",
             "## Kernel statistics (rocprofv3 --stats, complex64 and complex128 steps and plan builds)", "",
             "| kernel | calls | average ms |", "|---|---|---|"]
    for k in out["kernel_stats"]:
        if any(x in k["kernel"] for x in OUR_KERNELS + ("map_table", "tile_bounds", "synth")):
            lines.append(f"| `{k['kernel']}` | {k['calls']} | {k['avg_ms']:.3f} |")
    cal = out["calibration"]
    lines += ["", "## HBM bytes and VALU instructions per launch (complex64 step)", "",
              f"Calibration: a 1 GiB device copy reads FETCH_SIZE = {cal['FETCH_SIZE']['copy_kib']:.0f} KiB "
              f"and WRITE_SIZE = {cal['WRITE_SIZE']['copy_kib']:.0f} KiB, so the counters are scaled by "
              f"{cal['FETCH_SIZE']['factor']:.4f} (fetch) and {cal['WRITE_SIZE']['factor']:.4f} (write).", "",
              "VALU issue: SQ_INSTS_VALU (wave64 instructions) over the launch's duration, against 256 CUs "
              "issuing one per clock at 2.4 GHz (614.4 G/s; packed FP32 is not used).", "",
              "| role | bench avg ms (HIP events) | algorithmic GB | HBM read GB | HBM written GB | traffic / algorithmic "
              "| VALU G instr. | VALU per wave | VALU issue / peak |",
              "|---|---|---|---|---|---|---|---|---|"]
    for role, r in out["roles"].items():
        alg = (meta.get("bytes") or {}).get(role)
        ms_r = (meta.get("avg_ms") or {}).get(role)
        tot = (r["fetch_bytes"] or 0) + (r["write_bytes"] or 0)
        vi, wv = r.get("valu_insts"), r.get("waves")
        vcols = (f" {vi / 1e9:.2f} | {vi / wv:.0f} | {vi / (ms_r * 1e-3) / VALU_ISSUE_PEAK:.2f} |"
                 if vi and wv else " - | - | - |")
        lines.append(f"| {role} | {ms_r:.3f} | {alg / 1e9:.2f} | {r['fetch_bytes'] / 1e9:.2f} | "
                     f"{r['write_bytes'] / 1e9:.2f} | {tot / alg:.2f} |" + vcols)
    open(PROFILE_MD, "w").write("\n".join(lines) + "\n")
    return out


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uwa120_16k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the complex128 path")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (a reference for hardware byte counters)")
    ap.add_argument("--no-serving", action="store_true", help="skip the partial-view latency run")
    ap.add_argument("--roles-out", default=None,
                    help="write the kernel roles of one step, in launch order, to this JSON file")
    ap.add_argument("--summarize-profile", default=None, metavar="DIR",
                    help="no GPU: turn rocprofv3 output under DIR (trace/, fetch/, write/, roles.json) "
                         "into the committed summaries under profiles/")
    ap.add_argument("--no-stack", action="store_true", help="skip the focal-stack run")
    ap.add_argument("--no-oversample", action="store_true", help="skip the oversampled-spectrum run")
    ap.add_argument("--no-paper-model", action="store_true", help="skip the paper's polynomial map model run")
    ap.add_argument("--stack-depths", default="1.0,1.2,1.4",
                    help="focal-stack depths as multiples of the workload's z")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-inflight", type=int, default=4, help="server workspaces (streams)")
    return ap.parse_args()


def time_steps(plan, H, out, steps, warmup, torch):
    for _ in range(warmup):
        plan.execute(H, out)
    torch.cuda.synchronize()
    plan.set_timing(steps)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        plan.execute(H, out)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    launches = plan.timings()
    plan.set_timing(0)
    return ms, launches


def kernel_table(launches, steps):
    agg = {}
    for name, ms, nbytes in launches:
        a = agg.setdefault(name, {"ms": 0.0, "n": 0, "bytes": nbytes})
        a["ms"] += ms
        a["n"] += 1
    table = {}
    for name, a in agg.items():
        avg = a["ms"] / a["n"]
        table[name] = {"avg_ms": avg, "launches_per_step": a["n"] / steps, "bytes": a["bytes"],
                       "gbs": a["bytes"] / (avg * 1e-3) / 1e9}
    return table


def cpu_baseline(torch, N):
    """The float64 oracle on a bounded sample: the 120 deg geometry at 2048^2 (z scaled by 1/8 so
    the aperture-to-distance ratio is that of the 16384^2 workload), 16 points.  The oracle's cost does
    not depend on the hologram's content.  numpy runs it on one thread.  Returns the record and the
    relative L2 error of both GPU paths on the same sample."""
    import numpy as np

    import oracle
    import synth

    n, fov = 2048, 120.0
    scale = n / 16384
    dp = synth.fov_pitch(LAM, fov)
    z = 15e-3 * scale
    pc = synth.draw_points(1003, 16, n, n, dp, LAM, 10e-3 * scale, 20e-3 * scale)
    H = synth.point_hologram(pc, n, n, dp, LAM)
    log(f"cpu baseline: oracle on the {n}^2 sample ...")
    t0 = time.perf_counter()
    ref = oracle.reconstruct(H, LAM, dp, z)
    dt = time.perf_counter() - t0
    rec = {"value": n * n / dt / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
           "sample": (f"float64 oracle, full {n}^2 view of a {n}^2 120 deg hologram (16 points) at "
                      f"z = {z * 1e3:.4f} mm (16384^2 geometry scaled by {n}/16384), one run of {dt:.1f} s on "
                      f"{os.cpu_count()} host cores ({platform.processor() or platform.machine()}); "
                      f"numpy uses one thread")}
    errs = {}
    for prec in ("c64", "c128"):
        plan = N.Plan(LAM, dp, n, n, z, precision=prec)
        host = H.astype(np.complex64) if prec == "c64" else H
        out = plan(torch.from_numpy(host).cuda())
        torch.cuda.synchronize()
        r = oracle.reconstruct(host.astype(np.complex128), LAM, dp, z) if prec == "c64" else ref
        errs[prec] = oracle.rel_l2(out.cpu().numpy().astype(np.complex128), r)
        plan.close()
    return rec, errs


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(math.floor(k))
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def serving(torch, N, n_requests, inflight=4):
    """Partial views of one cached 8192^2 120 deg hologram (2048 points, z ~ U[5, 15] mm): square
    views of side S ~ U{512, 1024, 2048, 4096} at pitch Delta_F, centres uniform over the image,
    reconstruction distance z ~ U[5, 15] mm, seed 2004.  First the closed-loop capacity (8 requests
    outstanding), then Poisson arrivals at 70% of it; latency runs from submit to the completion of
    the request's last kernel."""
    import numpy as np
    import synth

    n, fov = 8192, 120.0
    dp = synth.fov_pitch(LAM, fov)
    pc = synth.draw_points(2004, 2048, n, n, dp, LAM, 5e-3, 15e-3)
    H = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    N.synth_hologram(pc.as_array(), n, n, dp, LAM, H)
    H = H.to(torch.complex64)
    torch.cuda.synchronize()
    spec = N.Spectrum(H, LAM, dp)
    del H
    rng = np.random.default_rng(2004)
    reqs = []
    max_m = 0
    for _ in range(n_requests):
        z = float(rng.uniform(5e-3, 15e-3))
        S = int(rng.choice([512, 1024, 2048, 4096]))
        g = N.plan_geometry(LAM, dp, n, n, z)
        half = g["image_size"] / 2 - S * g["dfx"] / 2
        v = dict(center_x=float(rng.uniform(-half, half)), center_y=float(rng.uniform(-half, half)),
                 pitch_x=0.0, pitch_y=0.0, nx=S, ny=S)
        gv = N.plan_geometry(LAM, dp, n, n, z, view=v)
        max_m = max(max_m, gv["mx"], gv["my"])
        reqs.append((z, v))
    srv = N.Server("c64", max_frt_size=max_m, max_view_size=4096, max_inflight=inflight)
    ring = 32
    outs = [torch.empty((4096, 4096), dtype=torch.complex64, device="cuda") for _ in range(ring)]
    pending = [None] * ring

    def run(order, arrivals=None):
        lat = []
        t_start = time.perf_counter()
        for i, (z, v) in enumerate(order):
            slot = i % ring
            if pending[slot] is not None:
                lat.append(srv.wait(pending[slot]))
            if arrivals is not None:
                while time.perf_counter() - t_start < arrivals[i]:
                    pass
            S = v["nx"]
            o = outs[slot].view(-1)[: S * S].view(S, S)
            pending[slot] = srv.submit(spec, z, o, view=v)
        for slot in range(ring):
            if pending[slot] is not None:
                lat.append(srv.wait(pending[slot]))
                pending[slot] = None
        return lat, time.perf_counter() - t_start

    log(f"serving: {n_requests} requests, FrT sizes up to {max_m}; warm-up pass")
    run(reqs[: min(len(reqs), 400)])
    # closed loop: at most 8 requests outstanding (the ring is deeper, so cap by waiting)
    lat_c, t_closed = [], time.perf_counter()
    window = []
    for i, (z, v) in enumerate(reqs):
        if len(window) == 8:
            lat_c.append(srv.wait(window.pop(0)[0]))
        slot = i % ring
        S = v["nx"]
        o = outs[slot].view(-1)[: S * S].view(S, S)
        window.append((srv.submit(spec, z, o, view=v), slot))
    for t, _ in window:
        lat_c.append(srv.wait(t))
    t_closed = time.perf_counter() - t_closed
    capacity = len(reqs) / t_closed
    pix = sum(v["nx"] * v["ny"] for _, v in reqs)
    log(f"serving closed loop: {capacity:.1f} req/s, {pix / t_closed / 1e6:.0f} Mpix/s")
    rate = 0.7 * capacity
    gaps = np.random.default_rng(20040).exponential(1.0 / rate, size=len(reqs))
    arrivals = np.cumsum(gaps) - gaps[0]
    lat_o, t_open = run(reqs, arrivals)
    p50, p99 = percentile(lat_o, 0.50), percentile(lat_o, 0.99)
    log(f"serving open loop at 70%: p50 {p50:.3f} ms, p99 {p99:.3f} ms")
    srv.close()
    spec.close()
    del outs
    torch.cuda.empty_cache()
    return {"p50": p50, "p99": p99, "requests": len(reqs), "load": 0.7, "rate_per_s": rate,
            "capacity_per_s": capacity, "closed_loop_mpix_s": pix / t_closed / 1e6,
            "closed_loop_p50": percentile(lat_c, 0.5), "closed_loop_p99": percentile(lat_c, 0.99),
            "max_frt_size": max_m, "inflight": inflight,
            "workload": "8192^2 120 deg hologram (2048 points), spectrum cached; square views S in "
                        "{512,1024,2048,4096} at Delta_F, uniform centres, z ~ U[5,15] mm, seed 2004; "
                        "Poisson arrivals at 70% of closed-loop capacity"}


def oversampled(torch, N, H, dp, n, z, steps, warmup, plain_out):
    """The same workload with the spectrum of step 2 sampled twice as finely (complex64)."""
    plan = N.Plan(LAM, dp, n, n, z, precision="c64", oversample=2)
    out = torch.empty((plan.info["sy"], plan.info["sx"]), dtype=torch.complex64, device="cuda")
    ms, launches = time_steps(plan, H, out, steps, warmup, torch)
    kt = kernel_table(launches, steps)
    a = out.to(torch.complex128)
    b = plain_out.to(torch.complex128)
    diff = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    rec = {"ms_per_step": ms, "mpix_s": plan.info["sx"] * plan.info["sy"] / (ms * 1e-3) / 1e6,
           "workspace_gb": plan.info["workspace_bytes"] / 1e9, "rel_l2_vs_plain": diff,
           "kernels": {k: round(v["avg_ms"], 4) for k, v in kt.items()}}
    log(f"oversampled spectrum: {ms:.3f} ms/step, {rec['mpix_s']:.1f} Mpix/s, differs from the plain path by "
        f"{diff:.3e} (rel L2)")
    for name, k in sorted(kt.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["launches_per_step"]):
        log(f"   {name:16s} {k['avg_ms']:8.3f} ms x{k['launches_per_step']:.0f}")
    del plan
    return rec


def paper_model(torch, N, H, dp, n, z, steps, warmup, exact_out):
    """The same workload with the paper's polynomial stand-in for Eq. 16 (complex64): its time, its
    plan build (the map table) and how far its output is from the exact map's."""
    t0 = time.perf_counter()
    plan = N.Plan(LAM, dp, n, n, z, precision="c64", map_model="paper")
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    out = torch.empty((plan.info["sy"], plan.info["sx"]), dtype=torch.complex64, device="cuda")
    ms, _ = time_steps(plan, H, out, steps, warmup, torch)
    a = out.to(torch.complex128)
    b = exact_out.to(torch.complex128)
    diff = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    log(f"paper polynomial map model: {ms:.3f} ms/step, plan {t_plan:.2f} s, differs from the exact map's "
        f"output by {diff:.3e} (rel L2)")
    del plan
    return {"ms_per_step": ms, "plan_s": t_plan, "rel_l2_vs_exact": diff}


def focal_stack(torch, N, H, dp, n, z, factors, steps, warmup, single_ms):
    """Full views at several depths from one hologram, sharing the z-independent stages (complex64)."""
    zs = [z * f for f in factors]
    st = N.Stack(LAM, dp, n, n, zs, precision="c64")
    outs = [torch.empty((i["sy"], i["sx"]), dtype=torch.complex64, device="cuda") for i in st.infos]
    for _ in range(max(1, warmup)):
        st.execute(H, outs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        st.execute(H, outs)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    d = len(zs)
    rec = {"depths_m": zs, "frt_size": st.infos[0]["mx"], "ms_per_execute": ms, "ms_per_depth": ms / d,
           "mpix_s": d * n * n / (ms * 1e-3) / 1e6, "speedup_vs_one_plan_per_depth": d * single_ms / ms}
    log(f"focal stack {d} depths: {ms:.3f} ms ({ms / d:.3f} ms per depth, "
        f"{rec['speedup_vs_one_plan_per_depth']:.2f}x one plan per depth)")
    st.close()
    return rec


def main():
    args = parse()
    if args.summarize_profile:
        rec = summarize_profile(args.summarize_profile)
        print(json.dumps(rec, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(this path runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2410_13474_amd import nufds as N

    N.load()
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.complex64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies done")
        del src, dst
    n, fov, z, npts, zlo, zhi, seed = WORKLOADS[args.workload]
    dp = synth.fov_pitch(LAM, fov)
    log(f"workload {args.workload}: N={n} fov={fov} z={z} points={npts}")
    pc = synth.draw_points(seed, npts, n, n, dp, LAM, zlo, zhi)
    H128 = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    N.synth_hologram(pc.as_array(), n, n, dp, LAM, H128)
    H64 = H128.to(torch.complex64)
    torch.cuda.synchronize()
    log("hologram generated on the GPU (float64 sum, rounded to complex64)")

    results = {}
    outs = {}
    for prec in (("c64",) if args.no_fp64 else ("c64", "c128")):
        t0 = time.perf_counter()
        plan = N.Plan(LAM, dp, n, n, z, precision=prec)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        H = H64 if prec == "c64" else H128
        out = torch.empty((plan.info["sy"], plan.info["sx"]), dtype=plan.dtype, device="cuda")
        ms, launches = time_steps(plan, H, out, args.steps, args.warmup, torch)
        kt = kernel_table(launches, args.steps)
        mpix = plan.info["sx"] * plan.info["sy"] / (ms * 1e-3) / 1e6
        log(f"{prec}: {ms:.3f} ms/step, {mpix:.1f} Mpix/s, plan {t_plan:.2f} s, M={plan.info['mx']}")
        for name, k in sorted(kt.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["launches_per_step"]):
            log(f"   {name:16s} {k['avg_ms']:8.3f} ms x{k['launches_per_step']:.0f}  {k['gbs']:7.0f} GB/s")
        alg_bytes = sum(k["bytes"] * k["launches_per_step"] for k in kt.values())
        results[prec] = {"ms_per_step": ms, "mpix_s": mpix, "plan_s": t_plan, "kernels": kt,
                         "alg_bytes_per_step": alg_bytes, "frac_hbm_end_to_end": alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "info": {k: plan.info[k] for k in ("mx", "my", "kcx", "kcy", "workspace_bytes", "map_bytes")}}
        outs[prec] = out
        if prec == "c64":
            plain64 = out
        if args.roles_out and prec == "c64":
            per_step = len(launches) // args.steps
            with open(args.roles_out, "w") as f:
                json.dump({"roles": [name for name, _, _ in launches[:per_step]],
                           "bytes": {k: v["bytes"] for k, v in kt.items()},
                           "avg_ms": {k: v["avg_ms"] for k, v in kt.items()},
                           "ms_per_step": ms}, f)
        del plan
    rel_fp32_fp64 = None
    if "c128" in outs:
        a = outs["c64"].to(torch.complex128)
        b = outs["c128"]
        rel_fp32_fp64 = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        log(f"rel L2 complex64 vs complex128 GPU paths: {rel_fp32_fp64:.3e}")
    del outs

    main_r = results["c64"]
    kt = main_r["kernels"]
    dom = max(kt, key=lambda k: kt[k]["avg_ms"] * kt[k]["launches_per_step"])
    d = kt[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                "bytes_per_launch": d["bytes"], "avg_ms": d["avg_ms"]}
    # the same kernel's vector-instruction issue (counter summary of the same sources), or null
    vi = measured_valu(dom)
    roofline["valu_issue"] = None if not vi else {
        "insts_per_launch": vi, "achieved_per_s": vi / (d["avg_ms"] * 1e-3), "peak_per_s": VALU_ISSUE_PEAK,
        "frac": vi / (d["avg_ms"] * 1e-3) / VALU_ISSUE_PEAK}

    over = None
    if not args.no_oversample:
        over = oversampled(torch, N, H64, dp, n, z, max(1, min(args.steps, 5)), args.warmup, plain64)
    pmodel = None
    if not args.no_paper_model:
        pmodel = paper_model(torch, N, H64, dp, n, z, max(1, min(args.steps, 5)), args.warmup, plain64)
    del plain64

    stack = None
    if not args.no_stack:
        factors = [float(f) for f in args.stack_depths.split(",")]
        stack = focal_stack(torch, N, H64, dp, n, z, factors, max(1, min(args.steps, 5)), args.warmup,
                            main_r["ms_per_step"])

    serve = None
    if not args.no_serving:
        serve = serving(torch, N, args.serving_requests, args.serving_inflight)

    cpu = None
    errs = {}
    if not args.no_cpu:
        cpu, errs = cpu_baseline(torch, N)
        log(f"cpu baseline {cpu['value']:.4f} Mpix/s; sample rel L2 vs oracle: {errs}")

    line = {
        "metric": "NU-FDS Mpix/s 16K 120° (FP32 vs FP64 @ rel-L2); p50/p99 partial-view ms",
        "value": main_r["mpix_s"],
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": args.workload, "hologram": f"{n}x{n}", "fov_deg": fov, "z_m": z,
                   "points": npts, "seed": seed, "output": f"{n}x{n} full view"},
        "fp64": ({"value": results["c128"]["mpix_s"], "ms_per_step": results["c128"]["ms_per_step"],
                  "dtype": "c128"} if "c128" in results else None),
        "rel_l2": {"fp32_vs_fp64_gpu": rel_fp32_fp64, "sample_vs_oracle": errs or None},
        "roofline": roofline,
        "end_to_end_hbm_frac": main_r["frac_hbm_end_to_end"],
        "kernels": {p: {k: {"avg_ms": round(v["avg_ms"], 4), "gbs": round(v["gbs"], 1),
                            "per_step": v["launches_per_step"]} for k, v in r["kernels"].items()}
                    for p, r in results.items()},
        "partial_view_latency_ms": serve,
        "focal_stack": stack,
        "oversampled": over,
        "paper_map_model": pmodel,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
