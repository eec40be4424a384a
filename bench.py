"""Benchmark of the reconstruction path on one MI355X.

Default workload: 640x480, K = 16 samples per pixel (~4.9M samples), FP16 storage, FP32 arithmetic,
R = 2, 8 px statistics tiles; 64 discs with specular-like highlights over a rotating ramp, samples
stratified over 64 ms (seeded, synthetic: the paper's BART animations are not available).

One step = the whole forward path on one frame's worth of samples already resident in HBM:
afr_build_deep_buffer (stream -> per-pixel deep buffer), then afr_forward (tile statistics and the
adaptive gather in one launch, bit-identical to afr_estimate_gradients + afr_reconstruct). Six
independent copies of the inputs rotate between steps so the ~0.5 GB the steps touch is not served
from the 256 MB Infinity Cache.

Printed: one JSON line. ``value`` is reconstructed Mpixel/s of whole steps, timed with nothing but the
path's launches between two events; extra keys give the per-kernel stage times (from a second pass
over the same steps with HIP events recorded on the launch stream after every stage, the build's four
stages through afr_build_deep_buffer_staged), samples filtered per second by the forward (estimate + gather), the
forward-plus-adjoint time per frame on the 512x512, K = 8, FP32 frame sequence, the plain direct
gather timed on the same data, the roofline of the dominant kernel, a measured device-copy
bandwidth, and the FP64 reference timed on the host as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import subprocess
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (256 CUs x 2.4 GHz; counts packed FP32)
ROTATE = 6


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--radius", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--no-fwdbwd", action="store_true", help="skip the forward+adjoint frames")
    ap.add_argument("--frames", type=int, default=32, help="frames in the forward+adjoint leg")
    ap.add_argument("--reproject-frames", type=int, default=8,
                    help="frames in the reprojection leg (0 skips it)")
    ap.add_argument("--no-crosshair", action="store_true", help="skip the crosshair-estimator leg")
    ap.add_argument("--sampler-frames", type=int, default=10,
                    help="frames of the closed-loop sampling leg (0 skips it)")
    ap.add_argument("--two-stream-frames", type=int, default=None,
                    help="frames of the two-stream leg (default 2 x steps; 0 skips it, as profiled "
                         "runs do, since its kernels overlap and would skew per-kernel averages)")
    ap.add_argument("--graph-steps", type=int, default=1,
                    help="also time the steps replayed from a captured graph (0 skips it)")
    ap.add_argument("--batch", type=int, default=64,
                    help="items in the batched-launch leg (the 64-item uneven batch; 0 skips it)")
    ap.add_argument("--no-scatter", action="store_true", help="skip the scatter-form leg")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain-vs-chosen comparison on FP32 buffers")
    ap.add_argument("--stats-summary", nargs=2, metavar=("KERNEL_STATS_CSV", "COMMAND"),
                    help="print a text summary of a rocprofv3 --stats kernel table and exit")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="print the HBM traffic summary of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV",
                    help="print per-kernel averages of every counter in these rocprofv3 --pmc "
                         "counter_collection.csv files (one pass each) and exit; the command that "
                         "made them goes in --summary-command")
    ap.add_argument("--summary-command", default="", help="command line recorded in a summary")
    ap.add_argument("--summary-workload", default="640x480 K=16 FP16 workload",
                    help="workload named in the first line of a counter summary")
    ap.add_argument("--summary-kernels",
                    default=r"^k_(bin_|scan_|forward<__half,2,|gather<__half,[12],4>|estimate_strip<__half>)",
                    help="regular expression of the kernels a counter summary lists")
    return ap.parse_args()


def _short(name):
    """Kernel name without return type, namespaces and parameter list; template arguments kept,
    without spaces (k_bin_select<__half,16>)."""
    for tok in ("void ", "afr::", "(anonymous namespace)::"):
        name = name.replace(tok, "")
    return name.split("(")[0].replace(" ", "").strip()


def stats_summary(csv_path, command):
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 kernel statistics", "# command: " + command,
           "# kernel | calls | avg us | min us | max us | total %"]
    for r in rows:
        out.append("%-44s %6d %10.2f %10.2f %10.2f %7.2f" % (
            _short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def pmc_summary(fetch_csv, write_csv, command, copy_kib=262144):
    """Per-kernel average FETCH_SIZE and WRITE_SIZE (KiB per dispatch), and the scale of each counter
    from the largest device copies of the run (the 256 MiB copies of copy_bandwidth)."""
    import csv
    import collections

    def per_dispatch(path, counter):
        vals = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return vals

    f = per_dispatch(fetch_csv, "FETCH_SIZE")
    w = per_dispatch(write_csv, "WRITE_SIZE")
    copy = [k for k in w if "copyBuffer" in k]
    wc = sorted(v for k in copy for v in w[k])[-3:]
    fc = sorted(v for k in copy for v in f[k])[-3:]
    f_fetch, f_write = copy_kib / float(np.median(fc)), copy_kib / float(np.median(wc))
    out = ["# HBM traffic per dispatch, 640x480 K=16 FP16 workload (bench.py)",
           "# fetch: " + command.replace("WRITE_SIZE", "FETCH_SIZE"),
           "# write: " + command.replace("FETCH_SIZE", "WRITE_SIZE").replace("/fetch ", "/write "),
           "# scale = %d KiB / counter reading of the 256 MiB device copy (median of the 3 largest)"
           % copy_kib,
           "digest=" + csrc_digest(),
           "scale %.4f %.4f" % (f_fetch, f_write),
           "# kernel <name> <FETCH_SIZE KiB> <WRITE_SIZE KiB>   (raw averages; bytes = KiB*scale*1024)"]
    for k in sorted(set(f) & set(w)):
        name = _short(k)
        if name.startswith("k_"):
            out.append("kernel %s %.3f %.3f" % (name, float(np.mean(f[k])), float(np.mean(w[k]))))
    return "\n".join(out)


def counter_summary(csvs, command, radius=2, kernels=r"^k_", workload="640x480 K=16 FP16 workload"):
    """Per-kernel averages (per dispatch) of every SQ/TCC counter found in the given rocprofv3
    counter-collection CSVs, and for the gather kernels the per-pair and per-cycle ratios the design
    notes quote: VALU wave-instructions per (slot, pixel) pair-wave (a pair-wave is 64 pairs), LDS
    instructions per pair-wave, bank-conflict share of LDS-active cycles and the share of wave
    cycles spent waiting for an instruction to issue. Pairs come from the 640x480 K=16 workload."""
    import csv
    import collections
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in csvs:
        for r in csv.DictReader(open(path)):
            vals[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    import afr_scenes as S
    wl = S.make_workload("c3")
    x, y = wl.stream.arrays()[:2]
    W, H, K = wl.width, wl.height, wl.k
    inside = (x >= 0) & (x < W) & (y >= 0) & (y < H)
    cnt = np.bincount((np.floor(y[inside]).astype(np.int64) * W + np.floor(x[inside]).astype(np.int64)),
                      minlength=W * H)
    count = np.minimum(cnt, K).reshape(H, W)
    pairs = {r: gather_pairs(count, r) for r in (1, 2)}
    out = ["# rocprofv3 counters per dispatch (average over dispatches), " + workload,
           "# command (one rocprofv3 --pmc pass per counter group): " + command,
           "# (slot, pixel) pairs of the gather: R=1 %d, R=2 %d" % (pairs[1], pairs[2]),
           "# kernel | counter | mean per dispatch | dispatches"]
    import re
    for k in sorted(vals):
        if not re.search(kernels, k):
            continue
        for c in sorted(vals[k]):
            v = vals[k][c]
            out.append("%-40s %-24s %16.1f %5d" % (k, c, float(np.mean(v)), len(v)))
        d = {c: float(np.mean(v)) for c, v in vals[k].items()}
        if "gather" in k or "reconstruct_tiled" in k:
            import re
            m = re.search(r"<[^,]+,(\d)", k)
            r = int(m.group(1)) if m else radius
            pw = pairs.get(r, pairs[2]) / 64.0
            if "SQ_INSTS_VALU" in d:
                out.append("%-40s %-24s %16.3f" % (k, "=VALU_per_pair_wave", d["SQ_INSTS_VALU"] / pw))
            if "SQ_INSTS_LDS" in d:
                out.append("%-40s %-24s %16.3f" % (k, "=LDS_per_pair_wave", d["SQ_INSTS_LDS"] / pw))
        if "SQ_WAIT_INST_ANY" in d and d.get("SQ_WAVE_CYCLES"):
            out.append("%-40s %-24s %16.3f" % (k, "=wait_inst_share", d["SQ_WAIT_INST_ANY"] / d["SQ_WAVE_CYCLES"]))
        if "SQ_LDS_BANK_CONFLICT" in d and d.get("SQ_LDS_IDX_ACTIVE"):
            out.append("%-40s %-24s %16.3f" % (k, "=bank_conflict_share",
                                               d["SQ_LDS_BANK_CONFLICT"] / d["SQ_LDS_IDX_ACTIVE"]))
    return "\n".join(out)


STAGES = ("bin_count", "bin_scan", "bin_scatter", "bin_select", "forward")


def kernel_of(stage, k, radius, tpw):
    """The kernel instantiation a stage launches for the FP16 workload (rocprofv3's short name). The
    count and scatter kernels also carry the samples per thread the library picks for the launch
    (from the sample count and the CU count), written here as a trailing '*'."""
    return {"bin_count": "k_bin_count<false,*>", "bin_scan": "k_scan_rows",
            "bin_scatter": "k_bin_scatter<false,*>",
            "bin_select": "k_bin_select<__half,%d>" % (4 if k <= 4 else 8 if k <= 8 else 16 if
                                                       k <= 16 else 32 if k <= 32 else 64),
            "forward": "k_forward<__half,%d,%d>" % (radius, tpw),
            "estimate": "k_estimate_strip<__half>",
            "gather": "k_gather<__half,%d,%d>" % (radius, tpw)}[stage]
SINGLE_KERNEL = ("bin_scatter", "bin_select", "forward")
# Algorithmic bytes of the 640x480 K=16 forward (statistics + gather) as the design target states
# them: every occupied binary16 slot record read once, the image written once.
FORWARD_TARGET_BYTES = 63.0e6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_640x480_k16_fp16.txt")


def csrc_digest():
    """Digest of every kernel source; a traffic figure is valid only for the sources it was taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2510_15876_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def resolve_kernel(kernel, names=None):
    """A name ending in '*>' (any last template argument) resolved against the kernels of the PMC
    summary when exactly one matches; otherwise the name as given."""
    if not kernel.endswith("*>"):
        return kernel
    if names is None:
        names = []
        if os.path.exists(TRAFFIC_FILE):
            names = [l.split()[1] for l in open(TRAFFIC_FILE) if l.startswith("kernel ")]
    hits = [n for n in names if n.startswith(kernel[:-2])]
    return hits[0] if len(hits) == 1 else kernel


def read_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed PMC summary: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) scaled by what the same counters read for a device copy of known size.
    None when there is no summary for it or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals, rows = {}, {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if line.startswith("digest="):
            vals["digest"] = line.split("=", 1)[1]
        elif line.startswith("scale "):
            _, f, w = line.split()
            vals["f_fetch"], vals["f_write"] = float(f), float(w)
        elif line.startswith("kernel "):
            _, name, fk, wk = line.split()
            rows[name] = (float(fk), float(wk))
    kernel = resolve_kernel(kernel, rows)
    if vals.get("digest") != csrc_digest() or kernel not in rows or "f_fetch" not in vals:
        return None
    fk, wk = rows[kernel]
    return int(round((fk * vals["f_fetch"] + wk * vals["f_write"]) * 1024))


_SLEEP_PER_MS = []


def hold_gpu(torch, ms=2.0):
    """Queue a spin kernel of about ``ms`` milliseconds, so that the launches that follow are all
    enqueued while the GPU is still busy and event-timed regions measure GPU time, not the host's
    launch rate. The spin rate is calibrated once."""
    if not _SLEEP_PER_MS:
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda._sleep(1000)
        e[0].record()
        torch.cuda._sleep(1000000)
        e[1].record()
        torch.cuda.synchronize()
        _SLEEP_PER_MS.append(1000000 / max(e[0].elapsed_time(e[1]), 1e-3))
    torch.cuda._sleep(int(_SLEEP_PER_MS[0] * ms))


def copy_bandwidth(torch, dev, mib=256, reps=5):
    """Device-to-device copy of ``mib`` MiB: achieved GB/s (read + write) and the per-copy size,
    the known-size reference for the PMC byte counters."""
    a = torch.empty(mib << 18, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * a.numel() * 4 / (ms * 1e-3) / 1e9


def algorithmic_bytes(stage, n, n_binned, occupied, W, H, K, nt):
    """Bytes a kernel must move by its own inputs and outputs (FP16 storage: 2 B per field). The
    build's (bin, chunk) offset table (< 1% of the scatter's bytes) is left out."""
    e = 2
    if stage == "bin_scatter":   # every field of every sample; one 24 B record per binned sample
        return 24 * n + 24 * n_binned   # (key, x, y) 16 B + binary16 payload 8 B
    if stage == "bin_select":    # every record once; all K slot planes, src and count written
        return 24 * n_binned + K * W * H * (6 * e + 4) + W * H
    if stage == "estimate":      # count, colour and age of every occupied slot; 11 stats planes
        return W * H + occupied * 4 * e + 11 * 4 * nt
    if stage == "gather":        # every occupied slot once, count, 3-channel float image
        return W * H + occupied * 6 * e + 12 * W * H
    if stage == "forward":       # every occupied slot record once, count, image, 11 stats planes
        return W * H + occupied * 6 * e + 12 * W * H + 11 * 4 * nt
    return None


def gather_pairs(count, radius):
    """(slot, output pixel) pairs of the gather: every slot of pixel q counts once for each pixel
    whose (2R+1)^2 block, clipped to the image, holds q."""
    H, W = count.shape
    c = count.astype(np.int64)
    reach_x = np.minimum(np.arange(W) + radius, W - 1) - np.maximum(np.arange(W) - radius, 0) + 1
    reach_y = np.minimum(np.arange(H) + radius, H - 1) - np.maximum(np.arange(H) - radius, 0) + 1
    return int((c * reach_y[:, None] * reach_x[None, :]).sum())


def roofline_entry(stage, kernel, nbytes, ms, traffic, pairs):
    """Roofline of the dominant kernel against HBM bandwidth by its algorithmic bytes; the gather
    alone against vector FP32 arithmetic (per pair one multiply and four fused multiply-adds,
    9 flops). The forward also carries its arithmetic fraction."""
    if stage == "gather":
        flops = 9 * pairs
        tf = flops / (ms * 1e-3) / 1e12
        return {"bound": "alu", "kernel": kernel, "achieved": round(tf, 3),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic,
                "algorithmic_flops": flops, "ms_per_launch": round(ms, 5),
                # packed FP32 is not used: one FMA per lane per cycle is the usable rate
                "frac_of_unpacked_fp32": round(tf / (FP32_VECTOR_PEAK_TFLOPS / 2), 4),
                "hbm_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "kernel": kernel, "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
           "algorithmic_bytes": nbytes, "ms_per_launch": round(ms, 5)}
    if stage == "forward":
        tf = 9 * pairs / (ms * 1e-3) / 1e12
        out["pair_arithmetic_tflops"] = round(tf, 3)
        out["pair_arithmetic_frac_of_unpacked_fp32"] = round(tf / (FP32_VECTOR_PEAK_TFLOPS / 2), 4)
    return out


def main():
    args = _args()
    if args.stats_summary:
        print(stats_summary(*args.stats_summary))
        return
    if args.pmc_summary:
        print(pmc_summary(*args.pmc_summary))
        return
    if args.counter_summary:
        print(counter_summary(args.counter_summary, args.summary_command, args.radius,
                              args.summary_kernels, args.summary_workload))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the multi-GPU layout "
              "is described in the design notes and not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import afr_scenes as S
    import paper_2510_15876_amd as afr

    if not os.path.exists(afr.lib_path()):
        import __graft_entry__
        __graft_entry__.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    wl = S.make_workload("c3")
    W, H, K = wl.width, wl.height, wl.k
    p = afr.Params(t_now=wl.t_now, radius=args.radius)
    streams = []
    base = [torch.from_numpy(a).to(dev) for a in wl.stream.arrays()]
    for r in range(ROTATE):
        streams.append(base if r == 0 else [a.clone() for a in base])
    bufs = [afr.DeepBuffer(W, H, K, "fp16", wl.t_ref, device=dev) for _ in range(ROTATE)]
    stats = [torch.empty((afr.NSTAT,) + afr.tiles_shape(W, H, p.tile), device=dev) for _ in range(ROTATE)]
    rgbs = [torch.empty((3, H, W), device=dev) for _ in range(ROTATE)]
    drop = torch.zeros(1, dtype=torch.int64, device=dev)
    drops2 = [torch.zeros(1, dtype=torch.int64, device=dev) for _ in range(2)]
    nst = afr.build_stage_count()

    def step(r, ev=None, i=0):
        s = streams[r]
        if ev is None:
            afr.build_deep_buffer(*s, W, H, K, "fp16", wl.t_ref, out=bufs[r], dropped=drop)
            afr.forward(bufs[r], p, stats=stats[r], rgb=rgbs[r], want_aux=False)
            return
        ev[0][i].record()
        afr.build_deep_buffer(*s, W, H, K, "fp16", wl.t_ref, out=bufs[r], dropped=drop,
                              stage_events=[ev[1 + j][i] for j in range(nst)])
        afr.forward(bufs[r], p, stats=stats[r], rgb=rgbs[r], want_aux=False)
        ev[nst + 1][i].record()

    # launch shape of the gather: the tuner's choice for this geometry (output is identical for
    # every shape)
    for r in range(ROTATE):
        step(r)
    torch.cuda.synchronize()
    tpw, _ = afr.reconstruct_tune(bufs[0], stats[0], p)
    for i in range(args.warmup):
        step(i % ROTATE)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(args.steps)] for _ in range(nst + 2)]
    for row in ev:  # create every event before the timed regions
        for e in row:
            e.record()
    t_beg, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # the timed steps: nothing but the path's own launches between the two events
    t0 = time.perf_counter()
    hold_gpu(torch)
    t_beg.record()
    for i in range(args.steps):
        step(i % ROTATE)
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = t_beg.elapsed_time(t_end) / args.steps
    # the same steps again with an event after every stage (per-stage times, the roofline's kernel)
    hold_gpu(torch)
    for i in range(args.steps):
        step(i % ROTATE, ev, i)
    torch.cuda.synchronize()
    stage_ms = {}
    for j, name in enumerate(STAGES):
        stage_ms[name] = float(np.mean([ev[j][i].elapsed_time(ev[j + 1][i])
                                        for i in range(args.steps)]))
    build_ms = sum(stage_ms[s] for s in STAGES[:4])
    fwd_ms = stage_ms["forward"]

    occupied = int(bufs[0].count.sum().item())
    n = len(wl.stream)
    xs = wl.stream.arrays()
    n_binned = int(np.count_nonzero((xs[0] >= 0) & (xs[0] < W) & (xs[1] >= 0) & (xs[1] < H)))
    nt = int(np.prod(afr.tiles_shape(W, H, p.tile)))
    dom = max(SINGLE_KERNEL, key=lambda s: stage_ms[s])
    dom_bytes = algorithmic_bytes(dom, n, n_binned, occupied, W, H, K, nt)
    dom_gbs = dom_bytes / (stage_ms[dom] * 1e-3) / 1e9
    pairs = gather_pairs(bufs[0].count.cpu().numpy(), args.radius)
    dom_kernel = resolve_kernel(kernel_of(dom, K, args.radius, tpw))
    traffic = read_traffic(dom_kernel)
    copy_gbs = copy_bandwidth(torch, dev)

    # two streams (default priority), alternate frames: one frame's build (HBM-bound) can run beside
    # another frame's gather (arithmetic- and LDS-bound); frames are independent
    streams2 = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    n2 = 2 * args.steps if args.two_stream_frames is None else args.two_stream_frames

    def two_stream_frames(n):
        e2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        e2[0].record()
        for s2 in streams2:
            s2.wait_event(e2[0])
        for i in range(n):
            r = i % ROTATE
            with torch.cuda.stream(streams2[i % 2]):
                afr.build_deep_buffer(*streams[r], W, H, K, "fp16", wl.t_ref, out=bufs[r],
                                      dropped=drops2[i % 2])
                afr.forward(bufs[r], p, stats=stats[r], rgb=rgbs[r], want_aux=False)
        for s2 in streams2:
            torch.cuda.current_stream().wait_stream(s2)
        e2[1].record()
        torch.cuda.synchronize()
        return e2[0].elapsed_time(e2[1]) / n

    two_streams = None
    if n2 > 0:
        two_stream_frames(2 * max(1, args.warmup))   # each stream's workspaces are allocated here
        two_stream_ms = two_stream_frames(n2)
        two_streams = {"ms_per_frame": round(two_stream_ms, 5),
                       "mpixel_per_s": round(W * H / (two_stream_ms * 1e-3) / 1e6, 3)}

    # the same steps replayed from one captured graph of ROTATE steps (one per input copy): the
    # launches of a frame loop that keeps its buffers, without the host issuing each kernel
    graph_steps = None
    if args.graph_steps:
        gs = torch.cuda.Stream(device=dev)
        gs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(gs):
            for r in range(ROTATE):  # this stream's workspaces are allocated outside the capture
                step(r)
        torch.cuda.current_stream().wait_stream(gs)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            for r in range(ROTATE):
                step(r)
        reps = max(1, args.steps // ROTATE)
        ge = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        graph.replay()
        torch.cuda.synchronize()
        ge[0].record()
        for _ in range(reps):
            graph.replay()
        ge[1].record()
        torch.cuda.synchronize()
        g_ms = ge[0].elapsed_time(ge[1]) / (reps * ROTATE)
        replayed = rgbs[0].clone()
        step(0)  # eager, on the current stream
        torch.cuda.synchronize()
        graph_steps = {"ms_per_step": round(g_ms, 5),
                       "mpixel_per_s": round(W * H / (g_ms * 1e-3) / 1e6, 3),
                       "steps_per_graph": ROTATE, "replays": reps,
                       "replay_equals_eager": bool(torch.equal(replayed, rgbs[0]))}
        del graph

    # the forward's two steps as separate launches on the same buffers (estimate, then gather)
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    n_plain = max(5, args.steps // 5)
    rgb_plain = torch.empty((3, H, W), device=dev)
    ue = [[torch.cuda.Event(enable_timing=True) for _ in range(n_plain)] for _ in range(3)]
    torch.cuda.synchronize()
    hold_gpu(torch)
    for i in range(n_plain):
        r = i % ROTATE
        ue[0][i].record()
        afr.estimate_gradients(bufs[r], p, out=stats[r])
        ue[1][i].record()
        afr.reconstruct(bufs[r], stats[r], p, rgb=rgb_plain, want_aux=False)
        ue[2][i].record()
    torch.cuda.synchronize()
    est_ms = float(np.mean([ue[0][i].elapsed_time(ue[1][i]) for i in range(n_plain)]))
    gat_ms = float(np.mean([ue[1][i].elapsed_time(ue[2][i]) for i in range(n_plain)]))
    fused_equal = bool(torch.equal(rgb_plain, rgbs[(n_plain - 1) % ROTATE]))

    # scatter form on the same buffers: splats of the gather's block size, then the sizes the
    # adaptive rule settles on after a few images of the same buffer
    sp = afr.SplatParams()
    size = afr.splat_sizes(W, H, None, sp, device=dev)
    cov = torch.empty((2, H, W), device=dev)
    scatter_ms = None if args.no_scatter else {}
    for label in (() if args.no_scatter else ("block", "adaptive")):
        if label == "adaptive":
            for _ in range(4):
                afr.reconstruct_scatter(bufs[0], stats[0], p, size, sp.size_max, rgb=rgb_plain,
                                        want_aux=False, coverage=cov)
                afr.splat_sizes(W, H, cov, sp, out=size)
        torch.cuda.synchronize()
        hold_gpu(torch)
        pe[0].record()
        for i in range(n_plain):
            afr.reconstruct_scatter(bufs[i % ROTATE], stats[i % ROTATE], p, size, sp.size_max,
                                    rgb=rgb_plain, want_aux=False, coverage=cov)
        pe[1].record()
        torch.cuda.synchronize()
        scatter_ms[label] = round(pe[0].elapsed_time(pe[1]) / n_plain, 5)
    if scatter_ms is not None:
        scatter_ms["adaptive_mean_size"] = round(float(size.mean().item()), 4)

    # the gather at R = 1 (9 pixels per block instead of 25) on the same buffers: the radius at
    # which the gather is bound by HBM rather than by arithmetic
    p1 = afr.Params(t_now=wl.t_now, radius=1)
    afr.estimate_gradients(bufs[0], p1, out=stats[0])
    afr.reconstruct(bufs[0], stats[0], p1, rgb=rgb_plain, want_aux=False)
    torch.cuda.synchronize()
    hold_gpu(torch)
    pe[0].record()
    for i in range(n_plain):
        afr.reconstruct(bufs[i % ROTATE], stats[i % ROTATE], p1, rgb=rgb_plain, want_aux=False)
    pe[1].record()
    torch.cuda.synchronize()
    r1_ms = pe[0].elapsed_time(pe[1]) / n_plain
    g_bytes = algorithmic_bytes("gather", n, n_binned, occupied, W, H, K, nt)
    gather_r1 = {"ms": round(r1_ms, 5), "hbm_gbs": round(g_bytes / (r1_ms * 1e-3) / 1e9, 1),
                 "hbm_frac": round(g_bytes / (r1_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    for r in range(ROTATE):  # statistics of the R = 2 parameters again
        afr.estimate_gradients(bufs[r], p, out=stats[r])

    # plain against chosen form at FP32 storage (and the images of both forms at both storage
    # precisions, for the precision study below)
    images = {"chosen_fp16": rgbs[0].clone(),
              "plain_fp16": afr.reconstruct_plain(bufs[0], stats[0], p, want_aux=False)[0]}
    plain = None
    if not args.no_plain:
        plain, images32 = plain_vs_chosen(torch, afr, wl, streams, p, dev, n_plain)
        images.update(images32)

    out = {
        "metric": "reconstructed Mpixel/s (build + estimate + gather per frame)",
        "value": round(W * H / (ms_step * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # the paper's own reconstruction rate, other hardware and another workload: context only
        "paper_context": {"mpixel_per_s": 1.31, "samples_splatted_per_s": 8.0e6,
                          "workload": "256x256, 400K-sample deep buffer, about 20 Hz",
                          "hardware": "GeForce 6800 Ultra, 16-bit float buffers",
                          "adaptive_overhead": "under 15% of computation time (simulation)"},
        "dtype": "fp16-storage/f32",
        "data": "synthetic",
        "config": {"workload": "640x480 K=16 FP16-storage, 64 discs + highlights, R=%d, 8px tiles"
                   % args.radius, "width": W, "height": H, "k": K, "radius": args.radius,
                   "samples": n, "occupied_slots": occupied, "gather_tiles_per_wave": tpw},
        "stages_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "build_ms": round(build_ms, 5),
        "forward_ms": round(fwd_ms, 5),
        "forward_mpixel_per_s": round(W * H / (fwd_ms * 1e-3) / 1e6, 3),
        "samples_filtered_per_s": round(occupied / (fwd_ms * 1e-3), 1),
        "build_samples_per_s": round(n / (build_ms * 1e-3), 1),
        "two_streams": two_streams,
        "graph_steps": graph_steps,
        "forward_algorithmic_bytes": algorithmic_bytes("forward", n, n_binned, occupied, W, H, K, nt),
        "forward_hbm_frac": round(FORWARD_TARGET_BYTES / (fwd_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "unfused": {"estimate_ms": round(est_ms, 5), "gather_ms": round(gat_ms, 5),
                    "sum_ms": round(est_ms + gat_ms, 5), "gather_equals_fused": fused_equal,
                    "gather_hbm_frac": round(algorithmic_bytes("gather", n, n_binned, occupied, W, H,
                                                               K, nt) / (gat_ms * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4),
                    "gather_pair_tflops": round(9 * pairs / (gat_ms * 1e-3) / 1e12, 3)},
        "plain_vs_chosen_fp32": plain,
        "gather_r1": gather_r1,
        "scatter_reconstruct_ms": scatter_ms,
        "roofline": roofline_entry(dom, dom_kernel, dom_bytes, stage_ms[dom], traffic, pairs),
        "copy_gbs_measured": round(copy_gbs, 1),
        "wall_s_timed": round(wall, 4),
    }

    # accuracy gate on the rotated buffer 0 against the FP64 reference (same FP16 buffer)
    import oracle as O
    if not args.no_cpu:
        def time_frame(reps):
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                ob, _ = O.build_buffer(wl.stream, W, H, K, "fp16", wl.t_ref)
                o_rgb, _, _ = O.forward(ob, O.Params(t_now=wl.t_now, radius=args.radius))
                times.append(time.perf_counter() - t0)
            return float(np.median(times)), o_rgb
        cores = O.num_threads()
        t_cpu, orgb = time_frame(3)
        O.set_num_threads(1)
        t_one, _ = time_frame(1)
        O.set_num_threads(cores)
        out["cpu_baseline"] = {"value": round(W * H / t_cpu / 1e6, 5), "unit": "Mpixel/s",
                               "cores": cores, "kind": "oracle",
                               "sample": "one full 640x480 K=16 FP16 frame (build+estimate+gather), "
                                         "FP64 C with OpenMP over rows (%d threads), median of 3 "
                                         "runs; single thread: one run" % cores,
                               "seconds_per_frame": round(t_cpu, 3),
                               "single_core_value": round(W * H / t_one / 1e6, 5),
                               "single_core_seconds_per_frame": round(t_one, 3),
                               "host": host_cpu()}
        # rgbs[0] holds the tiled gather of rotation copy 0 (identical inputs in every copy)
        err = float(np.abs(rgbs[0].cpu().numpy() - orgb).max())
        out["max_abs_err_vs_fp64"] = err
        out["accuracy_gate_1e-5"] = bool(err <= 1e-5)
        # the storage error: the FP16-storage image against the FP64 reference on the FP32 buffer
        ob32, _ = O.build_buffer(wl.stream, W, H, K, "fp32", wl.t_ref)
        orgb32, _, _ = O.forward(ob32, O.Params(t_now=wl.t_now, radius=args.radius))
        e16 = np.abs(rgbs[0].cpu().numpy() - orgb32)
        out["fp16_storage_err_vs_fp64_fp32_buffer"] = {
            "max": float(e16.max()), "p99": float(np.quantile(e16, 0.99)),
            "mean": float(e16.mean()), "gate_2e-3": bool(e16.max() <= 2e-3)}
        out["precision"] = precision_study(images, orgb, orgb32)

    if not args.no_fwdbwd:
        out["fwd_bwd"] = fwd_bwd(torch, afr, S, dev, args.frames)
    if args.sampler_frames > 0:
        out["sampler"] = sampler_leg(torch, afr, S, dev, args.sampler_frames)
    if not args.no_crosshair:
        out["crosshair"] = crosshair_leg(torch, afr, S, dev)
    if args.reproject_frames > 0:
        out["reproject"] = reproject_leg(torch, afr, S, dev, args.reproject_frames)
    if args.batch > 0:
        out["batch"] = batch_leg(torch, afr, S, dev, args.batch)
    print(json.dumps(out), flush=True)


def plain_vs_chosen(torch, afr, wl, streams, p, dev, reps):
    """The plain direct gather (one thread per pixel, global loads, an exponential per pair, one
    binary32 running sum per pixel) against the chosen form (the fused statistics + LDS-tiled
    gather) on FP32-storage buffers of the same workload: three copies rotate so that the 354 MB
    they hold is not served from the Infinity Cache. The plain form takes the statistics the
    forward wrote. Returns the timings and both forms' images of copy 0."""
    W, H, K = wl.width, wl.height, wl.k
    bufs = []
    for r in range(3):
        b, _ = afr.build_deep_buffer(*streams[r], W, H, K, "fp32", wl.t_ref)
        bufs.append(b)
    st = [afr.forward(b, p, want_aux=False)[0] for b in bufs]
    out = torch.empty((3, H, W), device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn(0)
        torch.cuda.synchronize()
        hold_gpu(torch)
        ev[0].record()
        for i in range(reps):
            fn(i % 3)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    plain_ms = timed(lambda r: afr.reconstruct_plain(bufs[r], st[r], p, rgb=out, want_aux=False))
    chosen_ms = timed(lambda r: afr.forward(bufs[r], p, stats=st[r], rgb=out, want_aux=False))
    gather_ms = timed(lambda r: afr.reconstruct(bufs[r], st[r], p, rgb=out, want_aux=False))
    images = {"plain_fp32": afr.reconstruct_plain(bufs[0], st[0], p, want_aux=False)[0],
              "chosen_fp32": afr.forward(bufs[0], p, want_aux=False)[1]}
    torch.cuda.synchronize()
    return ({"plain_gather_ms": round(plain_ms, 5), "chosen_forward_ms": round(chosen_ms, 5),
             "chosen_gather_ms": round(gather_ms, 5),
             "plain_over_chosen_forward": round(plain_ms / chosen_ms, 2),
             "note": "FP32 storage; the plain time excludes the statistics it reads, the chosen "
                     "forward includes them"}, images)


def precision_study(images, orgb16, orgb32):
    """Error distributions (max, p99, mean of |C - C_ref| over every pixel and channel) of both
    forms at both storage precisions against the FP64 reference: on the same FP16 buffer (the
    arithmetic's error) and on the FP32 buffer (for FP16, the storage error). The chosen form sums
    each slot plane's terms in binary32 and the planes in binary64; the plain form keeps one
    binary32 running sum per pixel."""
    def dist(a, ref):
        e = np.abs(a.cpu().numpy().astype(np.float64) - ref)
        return {"max": float(e.max()), "p99": float(np.quantile(e, 0.99)), "mean": float(e.mean())}
    out = {"accumulation": {"chosen": "binary32 per slot plane, planes summed in binary64",
                            "plain": "one binary32 running sum per pixel"}}
    for name, img in images.items():
        ref = orgb16 if name.endswith("fp16") else orgb32
        out[name] = dist(img, ref)
        if name.endswith("fp16"):
            out[name + "_vs_fp32_buffer"] = dist(img, orgb32)
    return out


def host_cpu():
    """The host's CPU model (lscpu) and the cores this process may run on."""
    model = None
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def batch_leg(torch, afr, S, dev, n, reps=10):
    """Many uneven reconstructions (sizes from {128x128, 320x240, 640x480, 1024x768}, K from
    {4, 8, 16}, FP16 storage) in one persistent launch replayed from a captured graph: estimate +
    gather of every item per replay, buffers built beforehand (one item's stream at a time)."""
    items, pixels, slots = [], 0, 0
    for i in range(n):
        wl = S.make_c5_batch(n=n, instances=[i])[0]
        arrs = [torch.from_numpy(a).to(dev) for a in wl.stream.arrays()]
        buf, _ = afr.build_deep_buffer(*arrs, wl.width, wl.height, wl.k, "fp16", wl.t_ref)
        del arrs
        items.append((buf, afr.Params(t_now=wl.t_now)))
        pixels += wl.width * wl.height
    torch.cuda.synchronize()
    slots = sum(int(b.count.sum().item()) for b, _ in items)
    batch = afr.Batch(items, want_aux=False)
    tpw, _ = batch.tune()
    batch.run()
    torch.cuda.synchronize()
    # one item against its separate estimate + gather calls (same per-tile code: identical bits)
    b0, p0 = items[0]
    st0 = afr.estimate_gradients(b0, p0)
    rgb0, _ = afr.reconstruct(b0, st0, p0, want_aux=False)
    same = bool(torch.equal(rgb0, batch.rgb[0]))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    batch.close()
    return {"workload": "%d items, sizes {128x128, 320x240, 640x480, 1024x768}, K {4, 8, 16}, "
                        "FP16 storage, R=2" % n,
            "pixels": pixels, "occupied_slots": slots, "ms_per_batch": round(ms, 5),
            "mpixel_per_s": round(pixels / (ms * 1e-3) / 1e6, 3),
            "samples_filtered_per_s": round(slots / (ms * 1e-3), 1),
            "tiles_per_wave": tpw, "graph_replays": reps, "item0_equals_separate_calls": same}


def fwd_bwd(torch, afr, S, dev, frames):
    """Forward + adjoint per frame on the 512x512, K=8, FP32 sequence (60 Hz frames, RMS loss
    against the analytic ground truth): build + forward (statistics and gather in one launch) +
    loss gradient + adjoint."""
    seq = S.make_c4_sequence(n_frames=frames)
    W, H, K = seq.width, seq.height, seq.k
    data = []
    for f in range(frames):
        wl = seq.frame_workload(f)
        gt = torch.from_numpy(S.ground_truth(seq.scene, W, H, wl.t_now, 2)).float().to(dev)
        data.append((wl, [torch.from_numpy(a).to(dev) for a in wl.stream.arrays()], gt))
    buf = afr.DeepBuffer(W, H, K, "fp32", 0.0, device=dev)
    drop = torch.zeros(1, dtype=torch.int64, device=dev)
    sig, tau = torch.tensor(1.0, device=dev), torch.tensor(0.5, device=dev)

    def frame(f):
        wl, s, gt = data[f]
        afr.build_deep_buffer(*s, W, H, K, "fp32", wl.t_ref, out=buf, dropped=drop)
        p = afr.Params(t_now=wl.t_now)
        st, rgb, aux = afr.forward(buf, p)
        _, g = afr.rms_loss(rgb, gt, 1.0 / frames)   # gradient of the mean per-frame RMS error
        return afr.reconstruct_backward(buf, st, p, rgb, aux, g)

    frame(0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for f in range(frames):
        frame(f)
    e1.record()
    torch.cuda.synchronize()
    return {"workload": "512x512 K=8 FP32, %d frames at 60 Hz" % frames,
            "ms_per_frame": round(e0.elapsed_time(e1) / frames, 5)}


def sampler_leg(torch, afr, S, dev, frames, budget=2):
    """Closed-loop sampling on the 256x256 moving-disc scene: the first 64 ms are sampled uniformly,
    then each 60 Hz frame the sampler draws ``budget`` samples per pixel, either uniformly or from
    its feedback (its own depth-4 buffer -> statistics -> tile error -> equal-error tiles -> spots),
    the scene is shaded at those spots on the host, and the reconstructor's K-deep queues (kept
    from frame to frame: a queue only loses samples to newer ones) are rebuilt, estimated and
    gathered at the frame time. Reports the mean RMS error against the analytic ground truth of each
    sampler and the GPU time of the feedback step per frame."""
    wl = S.make_workload("c2")
    scene, W, H, K, B = wl.scene, wl.width, wl.height, wl.k, 8
    ty, tx = afr.tiles_shape(W, H, B)
    sp = afr.SamplerParams()
    gts = {}
    res = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for mode in ("uniform", "feedback"):
        rng = np.random.default_rng(1)
        s = S.stratified_stream(scene, W, H, 8, 64.0, 64.0, rng)
        cur = [torch.from_numpy(a).to(dev) for a in s.arrays()]
        rms, fb_ms, parts = [], [], []
        for f in range(1, frames + 1):
            t_prev = float(np.float32(64.0 + (f - 1) * S.FRAME_MS))
            t_now = float(np.float32(64.0 + f * S.FRAME_MS))
            n = W * H * budget
            r = rng.integers(0, 2 ** 32, 3 * n, dtype=np.uint64).astype(np.uint32)
            rd = torch.from_numpy(r.view(np.int32)).to(dev)
            torch.cuda.synchronize()
            ev[0].record()
            if mode == "feedback":
                p = afr.Params(t_now=t_prev, tile=B)
                sbuf, _ = afr.build_deep_buffer(*cur, W, H, 4, "fp32", t_prev)
                st = afr.estimate_gradients(sbuf, p)
                E, _, g = afr.sampler_stats(sbuf, st, p, sp)
                P = afr.sampler_tile_weights(W, H, B, E, globals_=g)
            else:
                P = afr.sampler_tile_weights(W, H, B, torch.zeros((ty, tx), device=dev), n_parts=1)
            x, y, _ = afr.sampler_select(W, H, B, P, rd, want_tile=False)
            ev[1].record()
            torch.cuda.synchronize()
            if mode == "feedback":
                fb_ms.append(ev[0].elapsed_time(ev[1]))
                parts.append(float(g[7].item()))
            t = (t_prev + (t_now - t_prev) * rng.random(n)).astype(np.float32)
            new = S.shade_samples(scene, x.cpu().numpy(), y.cpu().numpy(), t)
            cur = [torch.cat([a, torch.from_numpy(b).to(dev)]) for a, b in zip(cur, new.arrays())]
            buf, _ = afr.build_deep_buffer(*cur, W, H, K, "fp32", t_now)
            keep = buf.src[buf.src >= 0].long().sort().values
            cur = [a[keep].contiguous() for a in cur]   # what the queues still hold
            buf, _ = afr.build_deep_buffer(*cur, W, H, K, "fp32", t_now)
            pr = afr.Params(t_now=t_now)
            rgb, _ = afr.reconstruct(buf, afr.estimate_gradients(buf, pr), pr)
            if f not in gts:
                gts[f] = torch.from_numpy(S.ground_truth(scene, W, H, t_now, 2)).float().to(dev)
            rms.append(float(torch.sqrt(((rgb - gts[f]) ** 2).mean()).item()))
        res[mode] = (rms, fb_ms, parts)
    return {"workload": "256x256 16 discs over a rotating ramp, %d frames at 60 Hz, %d samples/px "
                        "per frame, K=%d, sampler depth 4, 8 px tiles" % (frames, budget, K),
            "rms_uniform": round(float(np.mean(res["uniform"][0])), 6),
            "rms_feedback": round(float(np.mean(res["feedback"][0])), 6),
            "feedback_ms_per_frame": round(float(np.mean(res["feedback"][1])), 5),
            "mean_target_tiles": round(float(np.mean(res["feedback"][2])), 1)}


def crosshair_leg(torch, afr, S, dev, reps=20):
    """Crosshair gradient estimator on the 256x256 crosshair-sampled workload (static checkerboard
    under moving discs): RMS error against the analytic ground truth of the gather with the
    scattered-sample statistics and with the crosshair statistics, the mean temporal gradient and
    the share of tiles with none, and the time of the crosshair queue build and estimate."""
    cw = S.make_crosshair_workload()
    wl, xh = cw.workload, cw.crosshairs
    W, H, K = wl.width, wl.height, wl.k
    s = [torch.from_numpy(a).to(dev) for a in wl.stream.arrays()]
    ids = [torch.from_numpy(a).to(dev) for a in xh.arrays()]
    p = afr.Params(t_now=wl.t_now)
    buf, _ = afr.build_deep_buffer(*s, W, H, K, "fp32", wl.t_ref)
    xbuf, drop = afr.build_crosshair_buffer(s, ids, W, H, cw.k_xh, p, wl.t_ref)
    st0 = afr.estimate_gradients(buf, p)
    st1 = afr.estimate_gradients_crosshair(buf, xbuf, p)
    gt = torch.from_numpy(S.ground_truth(wl.scene, W, H, wl.t_now, 4)).float().to(dev)
    rms = lambda st: float(torch.sqrt(((afr.reconstruct(buf, st, p)[0] - gt) ** 2).mean()).item())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        afr.build_crosshair_buffer(s, ids, W, H, cw.k_xh, p, wl.t_ref, out=xbuf, dropped=drop)
    ev[1].record()
    for _ in range(reps):
        afr.estimate_gradients_crosshair(buf, xbuf, p, out=st1)
    ev[2].record()
    torch.cuda.synchronize()
    g0, g1 = st0[afr.STAT["gt"]], st1[afr.STAT["gt"]]
    return {"workload": "256x256 crosshair sampling, 4 visits/px over 64 ms (%d samples, %d "
                        "crosshairs), K=%d, crosshair queue depth %d, FP32"
                        % (len(wl.stream), len(xh), K, cw.k_xh),
            "rms_scattered": round(rms(st0), 6), "rms_crosshair": round(rms(st1), 6),
            "mean_gt_scattered": float(g0.mean().item()), "mean_gt_crosshair": float(g1.mean().item()),
            "zero_gt_tiles_scattered": round(float((g0 == 0).float().mean().item()), 4),
            "zero_gt_tiles_crosshair": round(float((g1 == 0).float().mean().item()), 4),
            "crosshair_build_ms": round(ev[0].elapsed_time(ev[1]) / reps, 5),
            "crosshair_estimate_ms": round(ev[1].elapsed_time(ev[2]) / reps, 5)}


def reproject_leg(torch, afr, S, dev, frames, reps=5):
    """Reconstructor reprojection on the 512x512, K=8, FP32 sequence: per frame, the RMS error against
    the analytic ground truth of the full forward with and without advecting samples by their
    surface velocity, and the build time of each; on the reprojected buffers also the scatter form
    with the adaptive splat size carried from frame to frame, and the holes (pixels no sample
    reaches) of each form."""
    seq = S.make_c4_sequence(n_frames=frames)
    W, H, K = seq.width, seq.height, seq.k
    buf = afr.DeepBuffer(W, H, K, "fp32", 0.0, device=dev)
    drop = torch.zeros(1, dtype=torch.int64, device=dev)
    rms = {False: [], True: []}
    build_ms = {False: [], True: []}
    rms_scatter, holes_gather, holes_scatter = [], [], []
    sp = afr.SplatParams()
    cov = None
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for f in range(frames):
        wl = seq.frame_workload(f)
        gt = torch.from_numpy(S.ground_truth(seq.scene, W, H, wl.t_now, 2)).float().to(dev)
        s = [torch.from_numpy(a).to(dev) for a in wl.stream.arrays()]
        vx, vy = (torch.from_numpy(a).to(dev) for a in wl.stream.motion())
        p = afr.Params(t_now=wl.t_now)
        for rep in (False, True):
            vel = dict(vx=vx, vy=vy) if rep else {}
            afr.build_deep_buffer(*s, W, H, K, "fp32", wl.t_ref, out=buf, dropped=drop, **vel)
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(reps):
                afr.build_deep_buffer(*s, W, H, K, "fp32", wl.t_ref, out=buf, dropped=drop, **vel)
            ev[1].record()
            torch.cuda.synchronize()
            build_ms[rep].append(ev[0].elapsed_time(ev[1]) / reps)
            st = afr.estimate_gradients(buf, p)
            rgb, aux = afr.reconstruct(buf, st, p)
            rms[rep].append(float(torch.sqrt(((rgb - gt) ** 2).mean()).item()))
            if rep:  # the scatter form with adaptive splat size on the reprojected buffer
                size = afr.splat_sizes(W, H, cov, sp, device=dev)
                srgb, _, cov = afr.reconstruct_scatter(buf, st, p, size, sp.size_max,
                                                       want_aux=False)
                rms_scatter.append(float(torch.sqrt(((srgb - gt) ** 2).mean()).item()))
                holes_gather.append(int((aux[1] == 0).sum().item()))
                holes_scatter.append(int((cov[0] == 0).sum().item()))
    return {"workload": "512x512 K=8 FP32, %d frames at 60 Hz, 64 discs with analytic velocities"
                        % frames,
            "rms_plain": round(float(np.mean(rms[False])), 6),
            "rms_reprojected": round(float(np.mean(rms[True])), 6),
            "build_ms_plain": round(float(np.mean(build_ms[False])), 5),
            "build_ms_reprojected": round(float(np.mean(build_ms[True])), 5),
            "rms_reprojected_scatter_adaptive": round(float(np.mean(rms_scatter)), 6),
            "holes_per_frame_gather": float(np.mean(holes_gather)),
            "holes_per_frame_scatter_adaptive": float(np.mean(holes_scatter))}


if __name__ == "__main__":
    main()
