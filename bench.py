"""Throughput of the CoG cascade vs the plain mixture on one MI355X.

One step = the whole hot path over one synthetic 1920x1080 stream already
resident in HBM: the prior-training launch over the first N frames, then the
cascade over the remaining frames in one launch (masks out).  `value` counts
the classified pixel-frames (frames after training) per second of the whole
step, training included; the median of three timed runs of K steps.

Beside it, on the same stream:
  - the plain Stauffer-Grimson mixture (warm-up over N frames, then one
    mixture step per frame) in the same two regimes;
  - the same step with the per-frame level counters and illumination flag;
  - one cog_step per frame (the live-camera regime), GPU time per frame and
    latency from submission to mask ready, for the cascade and the mixture;
  - the speed-up model of the paper's cascade analysis, 1 / sum_i s_i n_i,
    with level costs s_i measured on level-isolating streams;
  - the foreground-occupancy sweep (1, 5, 10, 30 %), the sampling variant,
    the grouping, the 64-stream batched tick and the serving loop;
  - the attainable copy bandwidth and the oracle on the host's cores.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--legs LIST] [--no-cpu]
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel-frames/s CoG vs full-GMM on 1 GPU (% HBM roofline); p99 frame latency"
HEADLINE = "surveil-1920x1080-k5-occ05"
SWEEP = ("surveil-1920x1080-k5-occ01", "surveil-1920x1080-k5-occ05",
         "surveil-1920x1080-k5-occ10", "surveil-1920x1080-k5-occ30")
HBM_PEAK_GBS = 8000.0
# vector ALU operation rate: 256 CU x 4 SIMD x 32 lanes per cycle x 2.4 GHz
# lane operations per second, the rate behind the 157.3 TFLOP/s fp32 vector
# figure (an FMA counts two flops).  (One wave64 instruction per 4 cycles per
# SIMD would be half of it; the cascade's and the mixture's launches issue
# VALU instructions faster than that, by their SQ counters.)
ALU_PEAK_GOPS = 256 * 4 * 32 * 2.4
LEGS = ("stream", "infos", "per_frame", "model", "sweep", "small", "sampling", "grouping", "batch",
        "serve")
# the two smaller configurations: their state fits the 256 MB last-level cache, so
# they are reported labelled cache-resident and carry no roofline claim
SMALL = ("surveil-160x120-k3", "surveil-640x480-k5")
GEN_THREADS = 16


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--runs", type=int, default=3, help="timed runs of K steps (median reported)")
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated subset of " + ",".join(LEGS))
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--serve-budget-gb", type=float, default=150.0)
    return ap.parse_args()


# ---- algorithmic bytes -------------------------------------------------------------

def stream_launch_bytes(P, F, K, dirty_px, C=3):
    """HBM bytes one multi-frame cascade launch over F frames must move.

    Per pixel-frame: the input value (C B) and the mask byte.  Per pixel once
    per launch: the previous value (C B), label bit, running average (16 B)
    and prior record (64 B) read; previous value, label bit and running
    average written.  Mixture records (K(C+2) floats) read and written for
    the pixels whose record the launch changed (counted on the device)."""
    per_frame = P * (C + 1) * F
    dense = P * ((C + 1 / 8 + 16 + 64) + (C + 1 / 8 + 16))
    mix = dirty_px * 2 * K * (C + 2) * 4
    return per_frame + dense + mix


def per_frame_model_bytes(occ, K, C=3):
    """Bytes per pixel-frame of the per-frame byte model (every level's state
    moved each frame): x and x' (2C), label bits (1/4), mask (1), the running
    average read by every pixel S0 passes on and written on an S1 accept, the
    64-byte prior record for S2 and S3, the mixture record read and written
    for S3 and the running average re-seeded on an S3 background match."""
    return (2 * C + 0.25 + 1 + 16 * (1 - occ["n0"]) + 16 * occ["n1"] + 64 * (occ["n2"] + occ["n3"])
            + 2 * K * (C + 2) * 4 * occ["n3"] + 16 * occ["n3_bg"])


def gmm_stream_bytes(P, F, K, C=3):
    """Plain mixture over F frames in one launch: input + mask per
    pixel-frame, the mixture record read and written once, previous value
    and label bits written."""
    return P * (C + 1) * F + P * (2 * K * (C + 2) * 4 + C + 1 / 8)


def train_bytes(P, N, K, C=3):
    """Training launch: N frames of input; writes the mixture, the running
    average, the 64-byte prior record, residue counts, grouping keys, the
    previous value and label bits."""
    return P * (C * N + K * (C + 2) * 4 + 16 + 64 + 8 + 8 + C + 1 / 8)


# ---- committed counter summaries ---------------------------------------------------

def kernel_source_hash() -> str:
    """Hash of the device sources' code: comments and blank lines are left out,
    so a comment edit keeps the committed counters valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1705_09339_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), encoding="utf-8") as fh:
                text = fh.read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
            code = "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())
            h.update(code.encode())
    return h.hexdigest()[:16]


def traffic_name(kernel, grid, workload):
    """File name of a committed traffic summary of one kernel and grid."""
    k = kernel.replace("<", "_").replace(">", "").replace(", ", "_")
    return f"traffic_{k}_g{grid}_{workload}.txt"


def profile_kv(name):
    """key: value lines of a committed profile summary, if it was taken on the
    current kernel sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return kv


def profile_sq(workload, kernel, grid):
    """SQ counters {name: value} of one kernel and grid from the committed
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"sq_{workload}.txt")
    if not os.path.exists(path):
        return None
    sha = None
    for line in open(path):
        if line.startswith("# kernel_source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith(f"{kernel} grid {grid}:"):
            if sha != kernel_source_hash():
                return None
            return {kv.split("=")[0].strip(): float(kv.split("=")[1])
                    for kv in line.split(":", 1)[1].split(",")}
    return None


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def r(x, n=4):
    return None if x is None else round(float(x), n)


# ---- timing helpers ----------------------------------------------------------------

class Runner:
    """One stream's contexts and device buffers; timing of the legs."""

    def __init__(self, C, torch, spec, dev, tile=0):
        self.C, self.torch, self.spec, self.dev = C, torch, spec, dev
        self.P, self.T, self.N, self.K = spec.pixels, spec.frames, spec.n_train, spec.K
        self.F = self.T - self.N
        self.stream = torch.cuda.current_stream()
        self.masks = torch.empty((self.F, self.P), dtype=torch.uint8, device="cuda")
        self.tile = tile

    def params(self, path, **kw):
        p = self.C.cog_default_params(self.spec.width, self.spec.height, 3, self.C.COG_U8, self.K,
                                      path=path, tile_px=self.tile)
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    def ctx(self, path, state=None, **kw):
        return self.C.CogStream(self.params(path, **kw), stream=self.stream, device_state=state)

    def ev(self):
        return self.torch.cuda.Event(enable_timing=True)

    def job(self, ctx, frames=None, ev=None, want_info=False):
        dev = self.dev if frames is None else frames
        ctx.reset()
        if ev:
            ev[0].record(self.stream)
        ctx.train_prior(dev[:self.N])
        if ev:
            ev[1].record(self.stream)
        infos = ctx.step_frames(dev[self.N:], self.masks, want_info=want_info)
        if ev:
            ev[2].record(self.stream)
        return infos

    def stream_runs(self, ctx, steps, warmup, runs, name, frames=None, want_info=False):
        """Median of `runs` timed runs of `steps` whole steps: wall ms per step
        and the live launch times (HIP events on the launch stream)."""
        torch = self.torch
        for _ in range(warmup):
            self.job(ctx, frames, want_info=want_info)
        torch.cuda.synchronize()
        out = []
        for _ in range(runs):
            evs = [[self.ev() for _ in range(3)] for _ in range(steps)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                self.job(ctx, frames, evs[k], want_info=want_info)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / steps * 1e3
            tr = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
            ca = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
            out.append((wall, tr, ca))
        out.sort()
        wall, tr, ca = out[len(out) // 2]
        log(f"{name}: {wall:.3f} ms/step (runs {[round(o[0], 3) for o in out]}), "
            f"train {tr:.3f} ms, frames {ca:.3f} ms")
        return {"ms_per_step": wall, "train_ms": tr, "frames_ms": ca,
                "runs_ms_per_step": [round(o[0], 4) for o in out]}

    def per_frame(self, ctx, runs, name):
        """One cog_step per frame.  GPU time per frame: every step is queued
        behind a GPU sleep so the launches run back to back, with an event
        after each; latency: submission to mask ready, synchronising every
        frame."""
        torch = self.torch
        F, N = self.F, self.N
        out = []
        for _ in range(runs):
            ctx.reset()
            ctx.train_prior(self.dev[:N])
            torch.cuda.synchronize()
            evs = [self.ev() for _ in range(F + 1)]
            torch.cuda._sleep(int(20e6))  # ~10 ms at 2.4 GHz: the host gets ahead
            evs[0].record(self.stream)
            for t in range(F):
                ctx.step(self.dev[N + t], self.masks[t])
                evs[t + 1].record(self.stream)
            torch.cuda.synchronize()
            gaps = [evs[t].elapsed_time(evs[t + 1]) for t in range(F)]
            out.append((evs[0].elapsed_time(evs[F]), gaps))
        out.sort(key=lambda o: o[0])
        total, gaps = out[len(out) // 2]
        ctx.reset()
        ctx.train_prior(self.dev[:N])
        torch.cuda.synchronize()
        wall = []
        for t in range(F):
            ts = time.perf_counter()
            ctx.step(self.dev[N + t], self.masks[t])
            self.stream.synchronize()
            wall.append((time.perf_counter() - ts) * 1e3)
        res = {"us_per_frame": total / F * 1e3, "mpx_s": self.P * F / (total * 1e-3) / 1e6,
               "gpu_frame_p50_us": pct(gaps, 50) * 1e3, "gpu_frame_p99_us": pct(gaps, 99) * 1e3,
               "latency_p50_ms": pct(wall, 50), "latency_p99_ms": pct(wall, 99),
               "runs_us_per_frame": sorted(round(o[0] / F * 1e3, 2) for o in out)}
        log(f"{name} per frame: {res['us_per_frame']:.2f} us/frame ({res['mpx_s']:.0f} Mpx/s), "
            f"latency p50 {res['latency_p50_ms']:.4f} p99 {res['latency_p99_ms']:.4f} ms")
        return res

    def occupancy(self, frames=None, **kw):
        """Level fractions of the stream (summed per-frame counters), taken
        through the 128-pixel tile kernel, whose results equal every other
        tile size's, so the timed kernels' launches are not mixed with it."""
        p = self.params(self.C.COG_PATH_CASCADE, **kw)
        p.tile_px = 128
        ctx = self.C.CogStream(p, stream=self.stream)
        dev = self.dev if frames is None else frames
        ctx.train_prior(dev[:self.N])
        infos = ctx.step_frames(dev[self.N:], self.masks, want_info=True)
        ctx.close()
        tot = {k: int(sum(i[k] for i in infos)) for k in ("n0", "n1", "n2", "n3", "n3_bg", "n_fg")}
        n = self.P * self.F
        occ = {k: v / n for k, v in tot.items()}
        occ["illum_frames"] = int(sum(i["illum_flag"] for i in infos))
        return occ

    def dirty_records(self, steps=1):
        """Pixels whose mixture record one cascade launch over the stream
        changes (the launch's mixture-record traffic), compared on the device
        in a caller-owned state buffer."""
        torch = self.torch
        p = self.params(self.C.COG_PATH_CASCADE)
        buf = torch.zeros(self.C.cog_state_bytes(p), dtype=torch.uint8, device="cuda")
        ctx = self.C.CogStream(p, stream=self.stream, device_state=buf)
        ctx.train_prior(self.dev[:self.N])
        R = ((self.K * 5) + 3) & ~3  # floats per record (C = 3), offset 0 of the state
        rec = buf[:self.P * R * 4].view(torch.float32).view(self.P, R)
        before = rec.clone()
        ctx.step_frames(self.dev[self.N:], self.masks)
        torch.cuda.synchronize()
        n = int((rec.view(torch.int32) != before.view(torch.int32)).any(1).sum().item())
        ctx.close()
        return n


def copy_bandwidth(torch, nbytes=2 << 30, reps=5):
    """Attainable HBM bandwidth of a plain device-to-device copy (bytes read +
    bytes written per second), median of `reps` copies of nbytes."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def level_model(R, C, cog_frames_ms, gmm_frames_ms, occ, steps):
    """The paper's cascade analysis (§3.2): speed-up = 1 / sum_i s_i n_i, with
    n_i the share of pixel-frames decided at level i and s_i the time of a
    pixel decided at level i relative to the full mixture.  The level costs
    are solved (least squares) from launches over level-isolating streams:
    every frame equal (S0), static noisy background (S1), the same with the
    running-average test switched off by a zero threshold (S2), and every
    stage off (S3), plus the workload itself."""
    import torch
    import synth

    P, N, F = R.P, R.N, R.F
    rows, t = [], []

    def add(ctx, frames, name, **kw):
        s = R.stream_runs(ctx, max(2, steps // 2), 1, 1, "model " + name, frames=frames)
        o = R.occupancy(frames=frames, **kw)
        rows.append([o["n0"], o["n1"], o["n2"], o["n3"]])
        t.append(s["frames_ms"] / (P * F))
        return o

    rows.append([occ["n0"], occ["n1"], occ["n2"], occ["n3"]])
    t.append(cog_frames_ms / (P * F))
    rep = torch.cat([R.dev[:N + 1], R.dev[N:N + 1].expand(F - 1, *R.dev.shape[1:])]).contiguous()
    c = R.ctx(C.COG_PATH_CASCADE)
    add(c, rep, "every frame equal")
    del rep
    c3 = R.ctx(C.COG_PATH_CASCADE, stage_mask=0)
    add(c3, None, "every stage off", stage_mask=0)
    c3.close()
    spec = R.spec.with_(ellipse_occ=0.0, dyn_regions=0, frames=R.T)
    st = torch.from_numpy(synth.make_stream(spec, threads=GEN_THREADS)).cuda()
    add(c, st, "static background")
    c2 = R.ctx(C.COG_PATH_CASCADE, lambda_rga=0.0)
    add(c2, st, "static background, no running average accept", lambda_rga=0.0)
    c2.close()
    c.close()
    del st
    torch.cuda.empty_cache()
    A = np.array(rows, dtype=np.float64)
    cost, *_ = np.linalg.lstsq(A, np.array(t), rcond=None)
    c_gmm = gmm_frames_ms / (P * F)
    s = cost / c_gmm
    n = np.array([occ["n0"], occ["n1"], occ["n2"], occ["n3"]])
    pred = 1.0 / float((s * n).sum())
    return {"s": [r(v, 4) for v in s], "n": [r(v, 5) for v in n],
            "predicted_speedup": r(pred, 3),
            "measured_speedup": r(gmm_frames_ms / cog_frames_ms, 3),
            "fit_residual_rel": r(float(np.abs(A @ cost - np.array(t)).max() / np.max(t)), 4),
            "runs": [{"n": [r(v, 4) for v in row], "ns_per_px_frame": r(tt * 1e6, 5)}
                     for row, tt in zip(rows, t)],
            "note": "level costs solved from one-launch runs over the workload, a stream of equal "
                    "frames, a static noisy background (with and without the running-average "
                    "accept) and every stage off; s_i relative to the plain mixture's time per "
                    "pixel-frame in the same one-launch regime"}


def one_workload(args, C, torch, spec, legs, headline):
    """Every leg of one stream; returns (result dict, runner extras)."""
    P, T, N, K = spec.pixels, spec.frames, spec.n_train, spec.K
    F = T - N
    t0 = time.time()
    frames, gt = synth_stream(spec)
    log(f"workload {spec.name}: {spec.width}x{spec.height} x {T} frames, N={N}, K={K}; "
        f"generated in {time.time() - t0:.1f} s")
    dev = torch.from_numpy(frames).cuda()
    torch.cuda.synchronize()
    R = Runner(C, torch, spec, dev, args.tile)
    steps = args.steps if headline else max(2, args.steps // 2)
    runs = args.runs if headline else 1
    out = {"workload": spec.name}
    occ = R.occupancy()
    out["occupancy"] = {k: r(v, 5) if k != "illum_frames" else v for k, v in occ.items()}
    out["early_rejection"] = r(occ["n0"] + occ["n1"] + occ["n2"], 5)
    cog = R.ctx(C.COG_PATH_CASCADE)
    gmm = R.ctx(C.COG_PATH_GMM)
    s_cog = R.stream_runs(cog, steps, args.warmup, runs, "cog")
    acc = {"cascade": accuracy(R.masks, gt[N:])} if headline else None
    s_gmm = R.stream_runs(gmm, steps, args.warmup, runs, "gmm")
    if headline:
        acc["gmm"] = accuracy(R.masks, gt[N:])
    val = P * F / (s_cog["ms_per_step"] * 1e-3) / 1e6
    gval = P * F / (s_gmm["ms_per_step"] * 1e-3) / 1e6
    out["value"] = r(val, 1)
    out["ms_per_step"] = r(s_cog["ms_per_step"])
    out["runs_ms_per_step"] = s_cog["runs_ms_per_step"]
    out["train_ms"] = r(s_cog["train_ms"])
    out["frames_ms"] = r(s_cog["frames_ms"])
    out["gmm"] = {"value": r(gval, 1), "ms_per_step": r(s_gmm["ms_per_step"]),
                  "runs_ms_per_step": s_gmm["runs_ms_per_step"],
                  "train_ms": r(s_gmm["train_ms"]), "frames_ms": r(s_gmm["frames_ms"])}
    out["speedup_vs_gmm"] = r(val / gval, 3)
    out["online"] = {"cog_mpx_s": r(P * F / (s_cog["frames_ms"] * 1e-3) / 1e6, 1),
                     "gmm_mpx_s": r(P * F / (s_gmm["frames_ms"] * 1e-3) / 1e6, 1),
                     "speedup": r(s_gmm["frames_ms"] / s_cog["frames_ms"], 3)}
    if "per_frame" in legs:
        pf = R.per_frame(cog, runs, "cog")
        pg = R.per_frame(gmm, runs, "gmm")
        out["per_frame"] = {"cog": {k: (r(v, 4) if not isinstance(v, list) else v) for k, v in pf.items()},
                            "gmm": {k: (r(v, 4) if not isinstance(v, list) else v) for k, v in pg.items()},
                            "speedup": r(pg["us_per_frame"] / pf["us_per_frame"], 3)}
    extra = {"R": R, "occ": occ, "s_cog": s_cog, "s_gmm": s_gmm, "acc": acc, "cog": cog, "gmm": gmm,
             "gt": gt, "frames": frames}
    return out, extra


def synth_stream(spec):
    import synth
    return synth.make_stream(spec, with_gt=True, threads=GEN_THREADS)


def main():
    args = parse()
    legs = set(x for x in args.legs.split(",") if x)
    bad = legs - set(LEGS)
    if bad:
        raise SystemExit(f"unknown legs {sorted(bad)}; choose from {LEGS}")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: pixels are independent, so the method has no "
              "cross-GPU exchange; one stream would shard by row bands and many streams by "
              "placing whole streams on GPUs, each GPU running the kernels measured here.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_1705_09339_amd import cog as C

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    spec = synth.preset(args.workload)
    P, T, N, K = spec.pixels, spec.frames, spec.n_train, spec.K
    F = T - N
    copy_gbs = copy_bandwidth(torch)
    log(f"copy bandwidth {copy_gbs:.0f} GB/s")
    w, x = one_workload(args, C, torch, spec, legs, headline=True)
    R, occ = x["R"], x["occ"]
    cog, gmm = x["cog"], x["gmm"]
    s_cog, s_gmm = x["s_cog"], x["s_gmm"]

    res = {
        "metric": METRIC,
        "value": w["value"],
        "unit": "Mpixel-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": w["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "width": spec.width, "height": spec.height,
                   "frames": T, "n_train": N, "classified_frames": F, "K": K, "input": "u8 RGB",
                   "tile_px": args.tile or 64,
                   "step": f"prior training over {N} frames + one cascade launch over {F} frames "
                           f"(masks out)",
                   "value_counts": f"classified pixel-frames ({F} per pixel) per second of the "
                                   f"whole step, training included; median of {args.runs} runs"},
    }
    for k in ("runs_ms_per_step", "train_ms", "frames_ms", "gmm", "speedup_vs_gmm", "online",
              "per_frame", "occupancy", "early_rejection"):
        if k in w:
            res[k] = w[k]
    res["copy_bandwidth_gbs"] = r(copy_gbs, 1)

    # the method's per-frame side output: level counters and illumination flag
    if "infos" in legs:
        si = R.stream_runs(cog, args.steps, args.warmup, 1, "cog + per-frame infos", want_info=True)
        res["with_infos"] = {"value": r(P * F / (si["ms_per_step"] * 1e-3) / 1e6, 1),
                             "ms_per_step": r(si["ms_per_step"]), "frames_ms": r(si["frames_ms"]),
                             "overhead": r(si["ms_per_step"] / s_cog["ms_per_step"] - 1.0, 4),
                             "note": "the same step returning every frame's level counters, "
                                     "foreground count and illumination flag to the host"}

    # rooflines
    dirty = R.dirty_records()
    b_stream = stream_launch_bytes(P, F, K, dirty)
    launch_s = s_cog["frames_ms"] * 1e-3
    kname = {64: "k_cascade_d<3, 5, false, true, false>"}.get(args.tile or 64, "cascade")
    hbm = {"alg_bytes_per_launch": int(b_stream), "achieved_gbs": r(b_stream / launch_s / 1e9, 1),
           "frac": r(b_stream / launch_s / 1e9 / HBM_PEAK_GBS, 4),
           "frac_of_copy": r(b_stream / launch_s / 1e9 / copy_gbs, 4),
           "dirty_record_px": dirty}
    grid = P if (args.tile or 64) == 64 else None  # work-items of the 64-pixel launch
    tr = profile_kv(traffic_name(kname, grid, spec.name))
    if tr:
        hbm["traffic"] = int(float(tr["hbm_bytes_per_launch"]))
        hbm["traffic_gbs"] = r(hbm["traffic"] / launch_s / 1e9, 1)
        hbm["amplification"] = r(hbm["traffic"] / b_stream, 3)  # counter bytes / algorithmic
    vl = profile_sq(spec.name, kname, grid)
    dominant = "cascade" if s_cog["frames_ms"] >= s_cog["train_ms"] else "train"
    if dominant == "cascade" and vl and "SQ_INSTS_VALU" in vl:
        valu = int(vl["SQ_INSTS_VALU"])
        ops = valu * 64
        ach = ops / launch_s / 1e9
        roof = {"bound": "alu", "kernel": kname, "achieved": r(ach, 1), "peak": ALU_PEAK_GOPS,
                "unit": "Gop/s", "frac": r(ach / ALU_PEAK_GOPS, 4),
                "traffic": hbm.get("traffic"), "launch_ms": r(s_cog["frames_ms"]),
                "valu_instructions_per_launch": valu,
                "hbm": hbm,
                "note": "achieved = wave64 VALU instructions of the launch (committed SQ counters, "
                        "same kernel, grid and workload) x 64 lanes / live launch time; peak = "
                        "256 CU x 4 SIMD x 32 lanes x 2.4 GHz; the launch's HBM bytes are under hbm"}
    elif dominant == "cascade":
        roof = {"bound": "hbm", "kernel": kname, "achieved": hbm["achieved_gbs"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm["frac"],
                "traffic": hbm.get("traffic"), "launch_ms": r(s_cog["frames_ms"]), "hbm": hbm,
                "note": "no SQ counters of the current kernel sources are committed"}
    else:
        bt = train_bytes(P, N, K)
        ach = bt / (s_cog["train_ms"] * 1e-3) / 1e9
        trt = profile_kv(traffic_name("k_train_prior<3, 5, false>", (P + 127) // 128 * 256, spec.name))
        roof = {"bound": "hbm", "kernel": "k_train_prior<3, 5, false>", "achieved": r(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": r(ach / HBM_PEAK_GBS, 4),
                "traffic": int(float(trt["hbm_bytes_per_launch"])) if trt else None,
                "alg_bytes_per_launch": int(bt), "launch_ms": r(s_cog["train_ms"])}
    roof["state_mb"] = r(C.cog_state_bytes(R.params(C.COG_PATH_CASCADE)) / 1e6, 1)
    res["roofline"] = roof
    if "per_frame" in res:
        bpx = per_frame_model_bytes(occ, K)
        us = res["per_frame"]["cog"]["us_per_frame"]
        ach = bpx * P / (us * 1e-6) / 1e9
        pfr = {"bound": "hbm", "kernel": "cascade, one frame per launch", "achieved": r(ach, 1),
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": r(ach / HBM_PEAK_GBS, 4),
               "frac_of_copy": r(ach / copy_gbs, 4), "bytes_per_px_frame": r(bpx, 3),
               "us_per_frame": us}
        tpf = profile_kv(traffic_name("k_frame<3, 5, false>", (P + 255) // 256 * 64, spec.name))
        if tpf:
            pfr["traffic_per_frame"] = int(float(tpf["hbm_bytes_per_launch"]))
            pfr["traffic_gbs"] = r(pfr["traffic_per_frame"] / (us * 1e-6) / 1e9, 1)
            pfr["traffic_frac"] = r(pfr["traffic_gbs"] / HBM_PEAK_GBS, 4)
            pfr["amplification"] = r(pfr["traffic_per_frame"] / (bpx * P), 3)
            pfr["kernel"] = tpf.get("kernel", pfr["kernel"])
        gb = 3 + 1 + 2 * K * 5 * 4
        gus = res["per_frame"]["gmm"]["us_per_frame"]
        pfr["gmm"] = {"bytes_per_px_frame": gb, "achieved": r(gb * P / (gus * 1e-6) / 1e9, 1),
                      "frac": r(gb * P / (gus * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        res["roofline_per_frame"] = pfr
    bg = gmm_stream_bytes(P, F, K)
    res["gmm"]["launch_hbm_frac"] = r(bg / (s_gmm["frames_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    if "model" in legs:
        res["speedup_model"] = level_model(R, C, s_cog["frames_ms"], s_gmm["frames_ms"], occ,
                                           args.steps)
        log(f"model: {res['speedup_model']}")

    # the sampling variant (§2 "Confidence based temporal sampling")
    if "sampling" in legs and (not args.tile or args.tile == 64):
        R.job(cog)
        cas_masks = R.masks.cpu().numpy()
        s_ctx = R.ctx(C.COG_PATH_CASCADE, stage_mask=C.COG_STAGE_ALL | C.COG_STAGE_SAMPLE)
        ss = R.stream_runs(s_ctx, args.steps, args.warmup, 1, "cog+sampling")
        s_masks = R.masks.cpu().numpy()
        x["acc"]["cascade_sampling"] = accuracy(R.masks, x["gt"][N:])
        s_ctx.reset()
        s_ctx.train_prior(R.dev[:N])
        s_inf = []
        for t0_ in range(0, F, 16):
            s_inf += s_ctx.step_frames(R.dev[N + t0_:N + min(F, t0_ + 16)], None, want_info=True)
        s_ctx.close()
        sp = C.cog_default_params(spec.width, spec.height, 3, C.COG_U8, K)
        sv = P * F / (ss["ms_per_step"] * 1e-3) / 1e6
        res["sampling"] = {"value": r(sv, 1), "ms_per_step": r(ss["ms_per_step"]),
                           "online_mpx_s": r(P * F / (ss["frames_ms"] * 1e-3) / 1e6, 1),
                           "speedup_vs_gmm": r(s_gmm["ms_per_step"] / ss["ms_per_step"], 3),
                           "speedup_vs_gmm_online": r(s_gmm["frames_ms"] / ss["frames_ms"], 3),
                           "halted_frac": r(sum(i["n_skip"] for i in s_inf) / (P * F), 4),
                           "mask_diff_vs_cascade": r(float((s_masks != cas_masks).mean()), 5),
                           "samp_window": sp.samp_window, "samp_period": sp.samp_period,
                           "samp_lambda": r(sp.samp_lambda, 3)}
        log(f"sampling: {res['sampling']}")

    # spatio-temporal grouping of the trained stream (one call, synchronous)
    if "grouping" in legs:
        cog.reset()
        cog.train_prior(R.dev[:N])
        gmap = torch.empty(P, dtype=torch.uint8, device="cuda")
        cog.group(gmap)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ginfo = cog.group(gmap)
        g_ms = (time.perf_counter() - ts) * 1e3
        res["grouping"] = {"ms": r(g_ms, 3), "iterations": ginfo["iterations"],
                           "grouped_frac": r(sum(g["grouped"] for g in ginfo["groups"]) / P, 4),
                           "cluster_sizes": [g["count"] for g in ginfo["groups"]]}
        # one shared running-average variance per group: the fit, then the
        # cascade frames from the shared state (median of 3 launches, each
        # after its own training, grouping and sharing, which are untimed)
        R.job(cog)
        plain = R.masks.clone()
        shared_ms, sh_fit = [], []
        for _ in range(3):
            cog.reset()
            cog.train_prior(R.dev[:N])
            cog.group(gmap)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            gv = cog.share(gmap)
            sh_fit.append((time.perf_counter() - ts) * 1e3)
            e0, e1 = R.ev(), R.ev()
            e0.record(R.stream)
            cog.step_frames(R.dev[N:], R.masks)
            e1.record(R.stream)
            torch.cuda.synchronize()
            shared_ms.append(e0.elapsed_time(e1))
        shared_ms.sort()
        res["grouping"]["shared"] = {
            "fit_ms": r(sorted(sh_fit)[1], 3), "shared_variances": [r(float(v), 3) for v in gv],
            "frames_ms": r(shared_ms[1]), "frames_ms_unshared": r(s_cog["frames_ms"]),
            "online_mpx_s": r(P * F / (shared_ms[1] * 1e-3) / 1e6, 1),
            "mask_diff_vs_unshared": r(float((R.masks != plain).float().mean()), 5),
            "accuracy": accuracy(R.masks, x["gt"][N:]),
            "accuracy_unshared": accuracy(plain, x["gt"][N:])}
        log(f"grouping: {res['grouping']}")
    if x["acc"]:
        res["accuracy_vs_ground_truth"] = x["acc"]
    cog.close()
    gmm.close()
    frames = x["frames"]
    del x, R
    torch.cuda.empty_cache()

    if "sweep" in legs:
        sweep = {}
        for name in SWEEP:
            if name == spec.name:
                sweep[name] = {k: w[k] for k in ("early_rejection", "value", "speedup_vs_gmm", "online",
                                                 "train_ms", "frames_ms") if k in w}
                sweep[name]["gmm_value"] = w["gmm"]["value"]
                if "per_frame" in w:
                    sweep[name]["per_frame_us"] = {"cog": w["per_frame"]["cog"]["us_per_frame"],
                                                   "gmm": w["per_frame"]["gmm"]["us_per_frame"]}
                continue
            sw, sx = one_workload(args, C, torch, synth.preset(name), legs - {"sweep"}, headline=False)
            sweep[name] = {k: sw[k] for k in ("early_rejection", "value", "speedup_vs_gmm", "online",
                                              "train_ms", "frames_ms")}
            sweep[name]["gmm_value"] = sw["gmm"]["value"]
            if "per_frame" in sw:
                sweep[name]["per_frame_us"] = {"cog": sw["per_frame"]["cog"]["us_per_frame"],
                                               "gmm": sw["per_frame"]["gmm"]["us_per_frame"]}
            sx["cog"].close()
            sx["gmm"].close()
            del sx
            torch.cuda.empty_cache()
            log(f"sweep {name}: {sweep[name]}")
        res["occupancy_sweep"] = sweep

    if "small" in legs:
        small = {}
        for name in SMALL:
            sw, sx = one_workload(args, C, torch, synth.preset(name), legs & {"per_frame"},
                                  headline=False)
            small[name] = {k: sw[k] for k in ("early_rejection", "value", "speedup_vs_gmm", "online",
                                              "train_ms", "frames_ms")}
            small[name]["gmm_value"] = sw["gmm"]["value"]
            if "per_frame" in sw:
                small[name]["per_frame_us"] = {"cog": sw["per_frame"]["cog"]["us_per_frame"],
                                               "gmm": sw["per_frame"]["gmm"]["us_per_frame"]}
            sp = sx["R"].params(C.COG_PATH_CASCADE)
            small[name]["state_mb"] = r(C.cog_state_bytes(sp) / 1e6, 1)
            small[name]["cache_resident"] = True
            sx["cog"].close()
            sx["gmm"].close()
            del sx
            torch.cuda.empty_cache()
            log(f"small {name}: {small[name]}")
        res["small_configs"] = small

    if "batch" in legs:
        torch.cuda.empty_cache()
        res["batch"] = batch_leg(args, C)
    if "serve" in legs:
        torch.cuda.empty_cache()
        res["serve"] = serving_leg(args, C)

    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(frames, spec, args.cpu_seconds)

    print(json.dumps(res), flush=True)


# ---- batched tick: 64 streams of mixed sizes --------------------------------------
BATCH_WORKLOAD = "batch-64-mixed"
BATCH_RING = 32    # distinct frames per stream, played forwards then backwards


def batch_streams():
    """16 RGB u8 streams each at 320x240, 640x480 and 1280x720 (K=5), and 16
    latent-map streams (64 channels of 30x40 f32 as single-channel pixels,
    K=3); lengths after training drawn in [300, 2000]."""
    rng = np.random.default_rng(170509339 + 4)
    out = []
    for w, h in ((320, 240), (640, 480), (1280, 720)):
        for i in range(16):
            out.append(dict(kind="u8", w=w, h=h, c=3, K=5, seed=170509339 + 4 + 1000 * len(out),
                            length=int(rng.integers(300, 2001))))
    for i in range(16):
        out.append(dict(kind="latent", w=30 * 40 * 64, h=1, c=1, K=3,
                        seed=170509339 + 4 + 1000 * len(out), length=int(rng.integers(300, 2001))))
    return out


def batch_leg(args, C):
    """The 64-stream batched workload: every stream trained on its first 100
    frames, then ticked until the longest ends; a tick advances every
    unfinished stream by F frames in one graph replay.  Timed with the
    inputs resident in HBM (a ring of distinct frames per stream)."""
    import torch

    import synth
    from synth.device import DeviceScene

    N = 100
    R2 = 2 * BATCH_RING
    specs = batch_streams()
    stream = torch.cuda.Stream()
    t0 = time.time()
    ctxs, rings, masks, trains = [], [], [], []
    with torch.cuda.stream(stream):
        for sp in specs:
            if sp["kind"] == "u8":
                sc = DeviceScene(sp["w"], sp["h"], sp["seed"])
                tr = sc.frames(0, N).view(N, -1)
                ring = sc.frames(N, BATCH_RING).view(BATCH_RING, -1)
                p = C.cog_default_params(sp["w"], sp["h"], 3, C.COG_U8, sp["K"])
            else:
                lat = synth.latent_stream(N + BATCH_RING, seed=sp["seed"])
                tr = torch.from_numpy(lat[:N]).cuda()
                ring = torch.from_numpy(lat[N:]).cuda()
                p = C.cog_default_params(sp["w"], 1, 1, C.COG_F32, sp["K"], in_lo=-5.0, in_hi=5.0)
            rings.append(torch.cat([ring, ring.flip(0)]).contiguous())
            trains.append(tr)
            ctxs.append(C.CogStream(p, stream=stream))
            masks.append(torch.empty((8, sp["w"] * sp["h"]), dtype=torch.uint8, device="cuda"))
    stream.synchronize()
    log(f"batch: {len(specs)} streams generated in {time.time() - t0:.1f} s")
    P = np.array([sp["w"] * sp["h"] for sp in specs], dtype=np.int64)
    L = np.array([sp["length"] for sp in specs], dtype=np.int64)
    fbytes = np.array([r.shape[1] * r.element_size() for r in rings], dtype=np.int64)
    ring_ptr = np.array([r.data_ptr() for r in rings], dtype=np.uint64)
    work = int((P * L).sum())

    def train_all():
        for c, tr in zip(ctxs, trains):
            c.reset()
            c.train_prior(tr)
        stream.synchronize()

    def run_batched(b, F, lat=None):
        table = C.TickTable(len(specs))
        table.view["ctx"] = [c.h for c in ctxs]
        table.view["masks"] = [m.data_ptr() for m in masks]
        done = np.zeros(len(specs), dtype=np.int64)
        n_ticks = int(-(-L.max() // F))
        evs = []
        stream.synchronize()
        ts = time.perf_counter()
        for k in range(n_ticks):
            nf = np.minimum(F, L - done)
            table.view["nframes"] = nf
            table.view["frames"] = ring_ptr + ((done % R2) * fbytes).astype(np.uint64)
            if lat is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                table.tick(b.b)
                e1.record(stream)
                evs.append((e0, e1))
            else:
                table.tick(b.b)
            done += nf
        stream.synchronize()
        wall = time.perf_counter() - ts
        if lat is not None:
            lat.extend(e0.elapsed_time(e1) for e0, e1 in evs)
        return wall, n_ticks

    def run_per_stream(F):
        done = np.zeros(len(specs), dtype=np.int64)
        n_ticks = int(-(-L.max() // F))
        stream.synchronize()
        ts = time.perf_counter()
        for k in range(n_ticks):
            for i, c in enumerate(ctxs):
                n = int(min(F, L[i] - done[i]))
                if n <= 0:
                    continue
                o = int(done[i] % R2)
                c.step_frames(rings[i][o:o + n], masks[i][:n])
                done[i] += n
        stream.synchronize()
        return time.perf_counter() - ts

    res = {"workload": BATCH_WORKLOAD,
           "streams": "16x320x240 + 16x640x480 + 16x1280x720 RGB u8 K=5, "
                      "16x latent 64ch 30x40 f32 (C=1, K=3); lengths 300-2000 after 100 training frames",
           "pixel_frames": work}
    with torch.cuda.stream(stream):
        b = C.CogBatch(stream, max_items=len(specs))
        # training (every stream, one launch each), timed once
        train_all()
        ts = time.perf_counter()
        train_all()
        res["train_ms_all_streams"] = round((time.perf_counter() - ts) * 1e3, 3)
        # autotune on the first F=1 tick, state restored afterwards
        table = C.TickTable(len(specs))
        table.view["ctx"] = [c.h for c in ctxs]
        table.view["masks"] = [m.data_ptr() for m in masks]
        table.view["nframes"] = 1
        table.view["frames"] = ring_ptr
        best = table.autotune(b.b, reps=5)
        res["schedule_u8_k5"] = b.get_schedule(3, 5, C.COG_U8)
        res["schedule_latent"] = b.get_schedule(1, 3, C.COG_F32)
        for F in (1, 8):
            train_all()
            run_batched(b, F)  # warm-up (graph capture)
            train_all()
            lat = []
            wall, n_ticks = run_batched(b, F, lat)
            res[f"f{F}"] = {"mpx_s": round(work / wall / 1e6, 1), "ticks": n_ticks,
                            "ms_per_tick": round(wall / n_ticks * 1e3, 4),
                            "gpu_tick_p50_ms": round(pct(lat, 50), 4),
                            "gpu_tick_p99_ms": round(pct(lat, 99), 4)}
            log(f"batch F={F}: {res[f'f{F}']}")
        # the default schedule (one-frame items in compacting 256-pixel tiles)
        # and the same without compaction (64-pixel one-pixel-per-lane tiles)
        for name, compact in (("default", 1), ("uncompacted", 0)):
            for cls in ((3, 5, C.COG_U8), (1, 3, C.COG_F32)):
                b.set_schedule(*cls, blocks_per_cu=-1, dynamic=0, group=4, use_graph=1,
                               compact=compact)
            train_all()
            run_batched(b, 1)
            train_all()
            wall, n_ticks = run_batched(b, 1)
            res[f"f1_{name}_schedule_mpx_s"] = round(work / wall / 1e6, 1)
        train_all()
        wall = run_per_stream(1)
        res["f1_per_stream_launches_mpx_s"] = round(work / wall / 1e6, 1)
        log(f"batch: default schedule {res['f1_default_schedule_mpx_s']} Mpx/s, uncompacted "
            f"{res['f1_uncompacted_schedule_mpx_s']} Mpx/s, "
            f"per-stream launches {res['f1_per_stream_launches_mpx_s']} Mpx/s")
        b.close()
        for c in ctxs:
            c.close()
    return res


# ---- serving loop: 256 camera streams, Poisson arrivals ---------------------------
SERVE_WORKLOAD = "serve-256-poisson30"


def serving_leg(args, C):
    """256 stream requests over a run of serve_seconds: each asks to join at
    a time in the first 40 % of the run (retrying every 100 ms while the HBM
    budget is full), lives 40-90 % of the run, and submits frames at Poisson
    times with a mean of 30 per second; resolutions cycle over 640x480,
    1920x1080 and 3840x2160 (RGB u8, K=5) and foreground occupancy over 1, 5
    and 10 %.  Streams of one (resolution, occupancy) share a device-resident
    clip (100 training frames, then a ring of 32 frames played back and
    forth).  Reports per-frame latency (submission to completion seen by the
    host) and the aggregate pixel rate."""
    import threading

    import torch

    from synth.device import DeviceScene

    D = args.serve_seconds
    N = 100
    R2 = 2 * BATCH_RING
    sizes = ((640, 480), (1920, 1080), (3840, 2160))
    occs = (0.01, 0.05, 0.10)
    t0 = time.time()
    clips = {}
    for si, (w, h) in enumerate(sizes):
        for oi, occ in enumerate(occs):
            sc = DeviceScene(w, h, 170509339 + 5 + 100 * si + 10 * oi, fg_occ=occ, n_rects=12)
            tr = sc.frames(0, N).view(N, -1)
            ring = sc.frames(N, BATCH_RING).view(BATCH_RING, -1)
            clips[(si, oi)] = (tr, torch.cat([ring, ring.flip(0)]).contiguous())
    torch.cuda.synchronize()
    log(f"serve: clips generated in {time.time() - t0:.1f} s")
    rng = np.random.default_rng(170509339 + 5)
    reqs = []
    for k in range(256):
        si, oi = k % 3, (k // 3) % 3
        start = float(rng.uniform(0.0, 0.4 * D))
        life = float(rng.uniform(0.4 * D, 0.9 * D))
        reqs.append(dict(si=si, oi=oi, start=start, end=min(D, start + life)))
    events = []
    for k, r in enumerate(reqs):
        events.append((r["start"], 0, k))
        t = r["start"]
        while True:
            t += float(rng.exponential(1.0 / 30.0))
            if t >= r["end"]:
                break
            events.append((t, 1, k))
        events.append((r["end"], 2, k))
    events.sort()
    # one mask frame per request (its submissions are in order, one frame each)
    mask_bufs = [torch.empty(sizes[r["si"]][0] * sizes[r["si"]][1], dtype=torch.uint8, device="cuda")
                 for r in reqs]
    torch.cuda.synchronize()
    params = {si: C.cog_default_params(w, h, 3, C.COG_U8, 5) for si, (w, h) in enumerate(sizes)}
    srv = C.CogServer(hbm_budget=int(args.serve_budget_gb * 2**30), max_streams=256, depth=2)
    comps = []
    stop = threading.Event()

    def poller():
        while not stop.is_set():
            comps.extend(srv.poll(max_n=4096, wait_us=5000))

    pt = threading.Thread(target=poller)
    pt.start()
    ids, nsub, last_try = {}, {}, {}
    fbytes = {si: w * h * 3 for si, (w, h) in enumerate(sizes)}
    submitted = 0
    dropped = 0
    ts = time.perf_counter()
    for t, kind, k in events:
        while time.perf_counter() - ts < t:
            pass
        r = reqs[k]
        if kind == 2:
            if k in ids:
                srv.close_stream(ids.pop(k))
            continue
        if k not in ids:
            now = time.perf_counter() - ts
            if kind == 1 and now - last_try.get(k, -1.0) < 0.1:
                dropped += 1
                continue
            last_try[k] = now
            try:
                ids[k] = srv.open(params[r["si"]], clips[(r["si"], r["oi"])][0])
                nsub[k] = 0
            except C.CogError as e:
                if e.status != C.COG_E_OOM:
                    raise
                dropped += kind
                continue
            if kind == 0:
                continue
        si = r["si"]
        ring = clips[(si, r["oi"])][1]
        f = nsub[k] % R2
        srv.submit_ptr(ids[k], ring.data_ptr() + f * fbytes[si], mask_bufs[k].data_ptr(), tag=k)
        nsub[k] += 1
        submitted += 1
    for k in list(ids):
        srv.close_stream(ids.pop(k))
    srv.drain()
    wall = time.perf_counter() - ts
    stop.set()
    pt.join()
    comps.extend(srv.poll(max_n=1 << 16))
    st = srv.stats()
    srv.close()
    lat = np.array([c["t_done_us"] - c["t_submit_us"] for c in comps]) / 1e3
    ok = all(c["status"] == 0 for c in comps)
    res = {"workload": SERVE_WORKLOAD,
           "streams": "256 requests; 640x480 / 1920x1080 / 3840x2160 RGB u8 K=5 cycling, "
                      "foreground 1/5/10 %; Poisson arrivals, mean 30 frames/s per stream",
           "seconds": round(wall, 3), "hbm_budget_gb": args.serve_budget_gb,
           "admitted": st["streams_admitted"], "rejected_attempts": st["streams_rejected"],
           "frames_submitted": submitted, "frames_completed": st["frames"],
           "frames_not_admitted": dropped, "all_ok": ok,
           "ticks": st["ticks"], "frames_per_tick": round(st["frames"] / max(1, st["ticks"]), 2),
           "mpx_s": round(st["pixel_frames"] / wall / 1e6, 1),
           "latency_p50_ms": round(pct(lat, 50), 3), "latency_p99_ms": round(pct(lat, 99), 3),
           "latency_max_ms": round(float(lat.max()), 3)}
    # where the tail is: a stream's first frame (it may wait for the stream's
    # training) against its later frames, and the later frames per frame size
    first = np.zeros(len(comps), dtype=bool)
    seen = set()
    for i, c in enumerate(comps):
        if c["stream_id"] not in seen:
            seen.add(c["stream_id"])
            first[i] = True
    split = {"first_frame": {"n": int(first.sum()), "p50_ms": round(pct(lat[first], 50), 3),
                             "p99_ms": round(pct(lat[first], 99), 3)},
             "later_frames": {"n": int((~first).sum()), "p50_ms": round(pct(lat[~first], 50), 3),
                              "p99_ms": round(pct(lat[~first], 99), 3),
                              "max_ms": round(float(lat[~first].max()), 3)}}
    size_of = np.array([sizes[reqs[c["tag"]]["si"]][0] for c in comps])
    for w, h in sizes:
        sel = (size_of == w) & ~first
        if sel.any():
            split[f"later_{w}x{h}"] = {"n": int(sel.sum()), "p99_ms": round(pct(lat[sel], 99), 3)}
    res["latency_split"] = split
    log(f"serve: {res}")
    return res


def accuracy(masks_dev, gt):
    """Foreground detection against the generator's ground truth (the union
    of the moving objects): per-pixel error rate and F1 of the foreground.
    Context only: the bimodal background regions count as background."""
    m = masks_dev.cpu().numpy().reshape(gt.shape) != 0
    tp = int(np.logical_and(m, gt).sum())
    fp = int(np.logical_and(m, ~gt).sum())
    fn = int(np.logical_and(~m, gt).sum())
    f1 = 2 * tp / max(1, 2 * tp + fp + fn)
    return {"error_rate": round((fp + fn) / gt.size, 5), "f1": round(f1, 4)}


def cpu_model():
    """The host CPU's model name and the cores this process may use."""
    name = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return name, n


def cpu_baseline(frames, spec, budget_s):
    """The oracle on a pixel sample of the same stream (every pixel's
    recurrence is independent, so a sample of pixels over all frames is the
    same work per pixel-frame): once on one thread, then on every core this
    process may use (at most 16), each thread running its own oracle on a
    band of the sample (the oracle's calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    P, T, N, K = spec.pixels, spec.frames, spec.n_train, spec.K
    F = T - N
    flat = frames.reshape(T, P, 3)
    host, ncpu = cpu_model()
    nthr = max(1, min(16, ncpu))

    def sample(stride):
        idx = np.arange(0, P, stride)
        return np.ascontiguousarray(flat[:, idx][:, None])

    def run_one(sub, gmm=False):
        orc = O.Oracle(O.make_params(sub.shape[2], 1, 3, K))
        ts = time.perf_counter()
        orc.train(sub[:N])
        for t in range(N, T):
            if gmm:
                orc.gmm_step(sub[t])
            else:
                orc.step(sub[t])
        el = time.perf_counter() - ts
        orc.close()
        return el

    e0 = run_one(sample(512))
    n0 = len(range(0, P, 512))
    # one-thread run sized to about half the budget, the all-core run to the same
    # wall time with nthr times the pixels
    stride = max(1, int(math.ceil(512 * e0 / (budget_s / 2))))
    sub = sample(stride)
    n1 = sub.shape[2]
    el1 = run_one(sub)
    stride_all = max(1, stride // nthr)
    suball = sample(stride_all)
    na = suball.shape[2]
    bands = [np.ascontiguousarray(b) for b in np.array_split(suball, nthr, axis=2)]
    ts = time.perf_counter()
    with ThreadPoolExecutor(nthr) as ex:
        list(ex.map(run_one, bands))
    ela = time.perf_counter() - ts
    log(f"cpu oracle: 1 thread {n1} px x {T} frames in {el1:.1f} s; {nthr} threads {na} px in {ela:.1f} s")
    one = {"value": r(n1 * F / el1 / 1e6, 3), "cores": 1, "seconds": r(el1, 2), "pixels": n1}
    # the oracle's plain mixture (the comparator) on the same one-thread sample
    elg = run_one(sub, gmm=True)
    one_gmm = {"value": r(n1 * F / elg / 1e6, 3), "cores": 1, "seconds": r(elg, 2), "pixels": n1,
               "cog_speedup": r(elg / el1, 3)}
    return {"value": r(na * F / ela / 1e6, 3), "unit": "Mpixel-frames/s", "cores": nthr,
            "kind": "oracle",
            "sample": f"every {stride_all}th pixel ({na} px) of all {T} frames of {spec.name}: "
                      f"training over {N}, cascade over {F}; value counts the {F} classified "
                      f"frames per second of training + cascade, like the GPU value",
            "seconds": r(ela, 2), "host": host, "host_cores": ncpu,
            "single_core": one, "single_core_gmm": one_gmm}


if __name__ == "__main__":
    main()
