"""EvSNet benchmark on one MI355X.

One step = the hot path over one batch of synthetic input with inputs
resident in HBM: the fused forward over the whole 1000-frame 1280x720 clip
(3->16->16->2, FP32), then the event compaction of its output spikes.  The
headline value is 720p event-frames/s; the JSON line also carries the
precision form (3->32->2 in FP32 and BF16 on the same clip), the training
step (4 x 256x256 x 64 crops, forward + EMD loss + BPTT backward) and the
batched persistent launch, each with its own timing.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms ...]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK = 157.3       # TFLOP/s, dense
BF16_MFMA_PEAK = 2500.0      # TFLOP/s, dense
PX720 = 1280 * 720


def conv_flops_per_px(channels):
    return sum(2 * 9 * ci * co for ci, co in zip(channels[:-1], channels[1:]))


def alg_bytes_per_px(channels):
    # x in (float32 per input channel) + int8 spikes out per output channel
    return 4 * channels[0] + channels[-1]


def src_hash(*names):
    h = hashlib.sha1()
    for n in names:
        with open(os.path.join(ROOT, "paper_2508_18071_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Timer:
    """HIP events on the stream the library launches on (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch
        self.s = torch.cuda.Event(enable_timing=True)
        self.e = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.s.record()
        return self

    def __exit__(self, *a):
        self.e.record()

    def ms(self):
        self.e.synchronize()
        return self.s.elapsed_time(self.e)


def make_720p_clip(torch, synth, dev, T):
    wl = synth.WORKLOADS["planes720"]
    x = torch.empty(1, T, 3, wl.H, wl.W, dtype=torch.float32, device=dev)
    synth.make_clip(wl, device=dev, T=T, out=x[0])
    return x


def traffic_from_profile(kernel_key, launches_px):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if
    the kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    ent = d.get(kernel_key)
    if not ent or ent.get("src_hash") != src_hash("evs_forward.hip"):
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(x_host, ws, channels, theta, leak, frames):
    from oracle import evsnet
    try:
        import threadpoolctl
        threads = max(i["num_threads"] for i in threadpoolctl.threadpool_info() if i["user_api"] == "blas")
    except Exception:
        threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    evsnet.forward(x_host[:frames], ws, theta, leak, keep_traces=False)
    dt = time.perf_counter() - t0
    return {"value": frames * x_host.shape[2] * x_host.shape[3] / PX720 / dt, "unit": "720p event-frames/s",
            "cores": int(threads), "kind": "oracle",
            "sample": f"first {frames} frames of the same 1280x720 clip, full frame, FP64 NumPy oracle "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=1000, help="clip length of the headline workload")
    ap.add_argument("--forms", default="fp32,w32")
    ap.add_argument("--cpu-frames", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the EvSNet forward shards over clips and spatial "
              "bands without communication, and this build runs on a single MI355X; "
              "use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2508_18071_amd as evs

    evs.lib()
    dev = torch.device("cuda:0")
    forms = set(args.forms.split(","))
    T = args.frames
    wl = synth.WORKLOADS["planes720"]
    log(f"generating {T} frames of 1280x720x3 on the GPU")
    x = make_720p_clip(torch, synth, dev, T)
    torch.cuda.synchronize()

    # ------------------------------------------------------------ headline: FP32 3->16->16->2
    chans = wl.channels
    net = evs.Net(chans, theta=wl.theta, leak=wl.leak, precision="fp32")
    ws = wl.weights()
    packed = evs.pack_weights(net, [torch.from_numpy(w).to(dev) for w in ws])
    out = torch.empty(1, T, chans[-1], wl.H, wl.W, dtype=torch.int8, device=dev)
    ev_cap = out.numel()
    events = None

    def step():
        tm = Timer(torch)
        with tm:
            evs.forward(net, packed, x, out=out)
        tc = None
        if "compact" in forms:
            tc = Timer(torch)
            with tc:
                evs.compact_events(out[0], capacity=ev_cap)
        return tm, tc

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    fwd_ms, cmp_ms = [], []
    t_all = Timer(torch)
    with t_all:
        timers = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    total_ms = t_all.ms()
    for tm, tc in timers:
        fwd_ms.append(tm.ms())
        if tc is not None:
            cmp_ms.append(tc.ms())
    ms_per_step = total_ms / args.steps
    px_frames = T * wl.H * wl.W
    value = px_frames / PX720 / (ms_per_step / 1e3)
    fwd_avg = float(np.mean(fwd_ms))
    flops = conv_flops_per_px(chans) * px_frames
    achieved = flops / (fwd_avg / 1e3) / 1e12
    spikes_per_px = float(out.abs().float().mean()) if T <= 1000 else None
    rec = {
        "metric": "720p event-frames/s (EvSNet fwd, FP32 vs BF16) + train-step ms; % HBM/MFMA peak",
        "value": round(value, 1),
        "unit": "720p event-frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"planes720: 1 clip x {T} frames x 1280x720x3 textured planes, 1-SPP noise; "
                               f"EvSNet conv3x3 3->16->16->2 + BiLIF, FP32",
                   "frames": T, "height": wl.H, "width": wl.W,
                   "step": "fused forward" + (" + event compaction" if "compact" in forms else "")},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_MFMA_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_MFMA_PEAK, 4),
                     "traffic": traffic_from_profile("fwd_L3_h16_f32", px_frames),
                     "kernel": "fwd_kernel<L3 h16 f32>", "kernel_ms": round(fwd_avg, 3),
                     "alg_flops": flops, "alg_bytes": alg_bytes_per_px(chans) * px_frames},
        "spikes_per_px_frame": spikes_per_px,
        "forms": {},
    }
    if cmp_ms:
        rec["forms"]["compaction_ms"] = round(float(np.mean(cmp_ms)), 3)
    log(f"fp32 3-16-16-2: {ms_per_step:.2f} ms/step, {value:.0f} fps, {achieved:.1f} TFLOP/s")

    # ------------------------------------------------------------ precision form 3->32->2
    if "w32" in forms:
        wl3 = synth.WORKLOADS["planes720_w32"]
        ws3 = wl3.weights()
        o3 = torch.empty(1, T, 2, wl.H, wl.W, dtype=torch.int8, device=dev)
        for prec in ("fp32", "bf16"):
            n3 = evs.Net(wl3.channels, theta=wl3.theta, leak=wl3.leak, precision=prec)
            p3 = evs.pack_weights(n3, [torch.from_numpy(w).to(dev) for w in ws3])
            for _ in range(args.warmup):
                evs.forward(n3, p3, x, out=o3)
            torch.cuda.synchronize()
            ts = []
            for _ in range(max(3, args.steps // 2)):
                tm = Timer(torch)
                with tm:
                    evs.forward(n3, p3, x, out=o3)
                ts.append(tm)
            torch.cuda.synchronize()
            ms = float(np.mean([t.ms() for t in ts]))
            fl = conv_flops_per_px(wl3.channels) * px_frames
            by = alg_bytes_per_px(wl3.channels) * px_frames
            tf = fl / (ms / 1e3) / 1e12
            gbs = by / (ms / 1e3) / 1e9
            peak = FP32_MFMA_PEAK if prec == "fp32" else BF16_MFMA_PEAK
            rec["forms"][f"w32_{prec}"] = {
                "value": round(px_frames / PX720 / (ms / 1e3), 1), "unit": "720p event-frames/s",
                "ms": round(ms, 3), "tflops": round(tf, 2), "mfma_frac": round(tf / peak, 4),
                "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                "workload": f"same clip, conv3x3 3->32->2 + BiLIF, {prec.upper()}"}
            log(f"w32 {prec}: {ms:.2f} ms, {px_frames / PX720 / (ms / 1e3):.0f} fps")
        del o3

    # ------------------------------------------------------------ CPU baseline
    if not args.no_cpu_baseline:
        log(f"CPU oracle on {args.cpu_frames} frames")
        xh = x[0, :args.cpu_frames].cpu().numpy()
        rec["cpu_baseline"] = cpu_baseline(xh, ws, chans, wl.theta, wl.leak, args.cpu_frames)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
