"""Throughput of the CoG cascade vs the plain mixture on one MI355X.

One step = the whole hot path over one synthetic stream already resident in
HBM: the prior-training launch over the first N frames, then the cascade
over the remaining frames.  The plain Stauffer-Grimson baseline processes the
same stream (warm-up over N frames, then a mixture step per frame) in its own
timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
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
HBM_PEAK_GBS = 8000.0
# vector ALU issue rate without packed or fused ops: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="surveil-640x480-k5")
    ap.add_argument("--chunk", type=int, default=0, help="frames per cascade launch (0 = all)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-stream batched tick")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched tick")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving loop")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving loop")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--serve-budget-gb", type=float, default=150.0)
    return ap.parse_args()


def alg_bytes_cascade(occ, P, F, K, C=3):
    """Algorithmic HBM bytes of one multi-frame cascade launch over F frames.

    Per pixel-frame: the input value (C B) and the mask byte; the mixture
    record read and written (K(C+2) floats each way) for every pixel that
    reaches S3.  Per pixel per launch: the 64-byte prior record (staged in
    LDS once), the previous value (C B) and running average (16 B) read and
    written, label bits read and written.
    """
    per_frame = P * (C + 1) * F
    mix = 2 * K * (C + 2) * 4 * occ["n3"]
    per_launch = P * (64 + 2 * C + 2 * 16 + 2 / 8)
    return per_frame + mix + per_launch


def alg_bytes_gmm(P, F, K, C=3):
    """Plain mixture, F frames in one launch: input + mask per pixel-frame,
    the mixture record read and written once per launch, label bits."""
    return P * (C + 1) * F + P * (2 * K * (C + 2) * 4 + C + 2 / 8)


def alg_bytes_train(P, N, K, C=3):
    """Training launch: N frames of input; writes the mixture, the running
    average, the 64-byte prior record, the previous value and label bits."""
    return P * (C * N + K * (C + 2) * 4 + 16 + 64 + C + 1 / 8)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("cog_kernels.hip", "cog_device.h"):
        with open(os.path.join(ROOT, "paper_1705_09339_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        b = int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None
    return {"bytes_per_launch": b, "note": kv.get("note", "")}


def measured_valu(kernel, workload):
    """Wave64 VALU instructions per launch of `kernel` from the committed SQ
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"valu_issue_{workload}.txt")
    if not os.path.exists(path):
        return None
    src = None
    for line in open(path):
        if line.startswith("# kernel_source_sha256:"):
            src = line.split(":", 1)[1].strip()
        elif not line.startswith("#") and line.startswith(kernel + "<3, 5, false, true, false>"):
            if src != kernel_source_hash():
                return None
            return int(line[line.index(">") + 1:].split()[1])  # dur_us, VALU, ...
    return None


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def main():
    args = parse()
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
    if args.batch_only:
        print(json.dumps({"batch": batch_leg(args, C)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serve": serving_leg(args, C)}), flush=True)
        return
    spec = synth.preset(args.workload)
    P, T, N, K = spec.pixels, spec.frames, spec.n_train, spec.K
    F = T - N
    log(f"workload {spec.name}: {spec.width}x{spec.height} x {T} frames, N={N}, K={K}")
    t0 = time.time()
    frames, gt = synth.make_stream(spec, with_gt=True)
    log(f"generated in {time.time() - t0:.1f} s")
    dev = torch.from_numpy(frames).cuda()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    masks = torch.empty((F, P), dtype=torch.uint8, device="cuda")

    def make_params(path, sample=False):
        p = C.cog_default_params(spec.width, spec.height, 3, C.COG_U8, K, path=path,
                                 tile_px=args.tile)
        if sample:
            p.stage_mask = C.COG_STAGE_ALL | C.COG_STAGE_SAMPLE
        return p

    def make(path, sample=False):
        return C.CogStream(make_params(path, sample), stream=stream)

    chunk = args.chunk or F

    def job(ctx, ev=None):
        ctx.reset()
        if ev:
            ev[0].record(stream)
        ctx.train_prior(dev[:N])
        if ev:
            ev[1].record(stream)
        for t0_ in range(0, F, chunk):
            t1_ = min(F, t0_ + chunk)
            ctx.step_frames(dev[N + t0_:N + t1_], masks[t0_:t1_])
        if ev:
            ev[2].record(stream)

    def timed(ctx, name):
        for _ in range(args.warmup):
            job(ctx)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        t_start = time.perf_counter()
        for k in range(args.steps):
            job(ctx, evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        tr = [e[0].elapsed_time(e[1]) for e in evs]
        ca = [e[1].elapsed_time(e[2]) for e in evs]
        log(f"{name}: {wall / args.steps * 1e3:.3f} ms/step, train {np.mean(tr):.3f} ms, "
            f"frames {np.mean(ca):.3f} ms")
        return wall, float(np.mean(tr)), float(np.mean(ca))

    # a plain copy of known size: the reference that scales the HBM byte
    # counters of the profiled runs
    calib = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    calib.copy_(dev.view(-1)[:64 << 20])
    torch.cuda.synchronize()
    del calib

    cog_ctx = make(C.COG_PATH_CASCADE)
    wall, tr_ms, ca_ms = timed(cog_ctx, "cog")
    acc = {"cascade": accuracy(masks, gt[N:])}
    # level occupancy of the same stream, taken through the 128-pixel tile
    # kernel (identical results for every tile size) so that the timed
    # kernel's launches all cover the same frame count
    p_occ = C.cog_default_params(spec.width, spec.height, 3, C.COG_U8, K, tile_px=128)
    occ_ctx = C.CogStream(p_occ, stream=stream)
    occ_ctx.train_prior(dev[:N])
    infos = occ_ctx.step_frames(dev[N:], masks, want_info=True)
    occ_ctx.close()
    occ = {k: int(sum(i[k] for i in infos)) for k in ("n0", "n1", "n2", "n3", "n3_bg", "n_fg")}

    gmm_ctx = make(C.COG_PATH_GMM)
    g_wall, g_tr_ms, g_ca_ms = timed(gmm_ctx, "gmm")
    acc["gmm"] = accuracy(masks, gt[N:])

    # the sampling variant (§2 "Confidence based temporal sampling"), its
    # agreement with the plain cascade and its halted share
    samp = {}
    if not args.tile or args.tile == 64:
        cas_masks = None
        cog_ctx.reset()
        cog_ctx.train_prior(dev[:N])
        cog_ctx.step_frames(dev[N:], masks)
        cas_masks = masks.cpu().numpy()
        s_ctx = make(C.COG_PATH_CASCADE, sample=True)
        s_wall, s_tr_ms, s_ca_ms = timed(s_ctx, "cog+sampling")
        s_masks = masks.cpu().numpy()
        acc["cascade_sampling"] = accuracy(masks, gt[N:])
        s_ctx.reset()
        s_ctx.train_prior(dev[:N])
        s_inf = []
        for t0_ in range(0, F, 16):
            s_inf += s_ctx.step_frames(dev[N + t0_:N + min(F, t0_ + 16)], None, want_info=True)
        s_ctx.close()
        sp = C.cog_default_params(spec.width, spec.height, 3, C.COG_U8, K)
        samp = {"value": round(P * T * args.steps / s_wall / 1e6, 1),
                "ms_per_step": round(s_wall / args.steps * 1e3, 4),
                "online_mpx_s": round(P * F / (s_ca_ms * 1e-3) / 1e6, 1),
                "speedup_vs_gmm": round((P * T * args.steps / s_wall) / (P * T * args.steps / g_wall), 3),
                "speedup_vs_gmm_online": round(g_ca_ms / s_ca_ms, 3),
                "halted_frac": round(sum(i["n_skip"] for i in s_inf) / (P * F), 4),
                "mask_diff_vs_cascade": round(float((s_masks != cas_masks).mean()), 5),
                "samp_window": sp.samp_window, "samp_period": sp.samp_period,
                "samp_lambda": round(sp.samp_lambda, 3)}
        log(f"sampling: {samp}")

    # per-frame streaming: one cog_step per frame, latency submit -> mask ready
    lat = {}
    if not args.no_latency:
        cog_ctx.reset()
        cog_ctx.train_prior(dev[:N])
        torch.cuda.synchronize()
        wall_ms, gpu_ms = [], []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for t in range(F):
            ts = time.perf_counter()
            e0.record(stream)
            cog_ctx.step(dev[N + t], masks[t])
            e1.record(stream)
            e1.synchronize()
            wall_ms.append((time.perf_counter() - ts) * 1e3)
            gpu_ms.append(e0.elapsed_time(e1))
        cog_ctx.reset()
        cog_ctx.train_prior(dev[:N])
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for t in range(F):
            cog_ctx.step(dev[N + t], masks[t])
        torch.cuda.synchronize()
        stream_s = time.perf_counter() - ts
        lat = {"p50_ms": round(pct(wall_ms, 50), 4), "p99_ms": round(pct(wall_ms, 99), 4),
               "kernel_p50_ms": round(pct(gpu_ms, 50), 4), "kernel_p99_ms": round(pct(gpu_ms, 99), 4),
               "per_frame_mpx_s": round(P * F / stream_s / 1e6, 1),
               "note": "one cog_step per frame on device-resident frames, wall time from "
                       "submission to mask ready"}
        log(f"latency p50 {lat['p50_ms']} ms p99 {lat['p99_ms']} ms; per-frame stream "
            f"{lat['per_frame_mpx_s']} Mpx/s")

    # spatio-temporal grouping of the trained stream (one call, synchronous)
    cog_ctx.reset()
    cog_ctx.train_prior(dev[:N])
    gmap = torch.empty(P, dtype=torch.uint8, device="cuda")
    cog_ctx.group(gmap)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ginfo = cog_ctx.group(gmap)
    g_ms = (time.perf_counter() - ts) * 1e3
    grouping = {"ms": round(g_ms, 3), "iterations": ginfo["iterations"],
                "grouped_frac": round(sum(g["grouped"] for g in ginfo["groups"]) / P, 4),
                "cluster_sizes": [g["count"] for g in ginfo["groups"]]}
    log(f"grouping: {grouping}")

    cog_ctx.close()
    gmm_ctx.close()

    value = P * T * args.steps / wall / 1e6
    g_value = P * T * args.steps / g_wall / 1e6
    # dominant kernel of the step and its roofline
    b_casc = alg_bytes_cascade(occ, P, F, K)
    b_train = alg_bytes_train(P, N, K)
    tile = args.tile or 64
    casc_name = "k_cascade_d" if tile == 64 else ("k_cascade_w" if tile == 128 else "k_cascade")
    dominant = casc_name if ca_ms >= tr_ms else "k_train"
    dom_ms = ca_ms if dominant == casc_name else tr_ms
    dom_bytes = b_casc if dominant == casc_name else b_train
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(dominant, spec.name)
    roof = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "alg_bytes_per_launch": int(dom_bytes), "launch_ms": round(dom_ms, 4),
            # the stream's device state, beside the 256 MB last-level cache
            "state_mb": round(C.cog_state_bytes(make_params(C.COG_PATH_CASCADE)) / 1e6, 1)}
    if traffic:
        roof["traffic_note"] = traffic["note"]
    # the kernel is limited by instruction issue rather than HBM: its VALU
    # instructions (committed counters) against one wave64 instruction per 4
    # cycles per SIMD, 1024 SIMDs at 2.4 GHz, over the live launch time
    valu = measured_valu(dominant, spec.name) if K == 5 else None
    if valu:
        roof["valu_instructions"] = valu
        roof["valu_issue_frac"] = round(valu * 4 / (1024 * 2.4e9) / (dom_ms * 1e-3), 4)

    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpixel-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "width": spec.width, "height": spec.height,
                   "frames": T, "n_train": N, "K": K, "input": "u8 RGB",
                   "launches_per_step": 1 + math.ceil(F / chunk), "tile_px": tile},
        "gmm": {"value": round(g_value, 1), "ms_per_step": round(g_wall / args.steps * 1e3, 4),
                "train_ms": round(g_tr_ms, 4), "frames_ms": round(g_ca_ms, 4)},
        "speedup_vs_gmm": round(value / g_value, 3),
        "online": {"cog_mpx_s": round(P * F / (ca_ms * 1e-3) / 1e6, 1),
                   "gmm_mpx_s": round(P * F / (g_ca_ms * 1e-3) / 1e6, 1),
                   "train_ms": round(tr_ms, 4), "frames_ms": round(ca_ms, 4)},
        "occupancy": {k: round(v / (P * F), 5) for k, v in occ.items()},
        "latency": lat,
        "roofline": roof,
        "sampling": samp,
        "grouping": grouping,
        "accuracy_vs_ground_truth": acc,
    }

    if not args.no_batch:
        del dev, masks
        torch.cuda.empty_cache()
        res["batch"] = batch_leg(args, C)
    if not args.no_serve:
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
        for cls in ((3, 5, C.COG_U8), (1, 3, C.COG_F32)):  # the defaults
            b.set_schedule(*cls, blocks_per_cu=-1, dynamic=0, group=4, use_graph=1)
        train_all()
        run_batched(b, 1)
        train_all()
        wall, n_ticks = run_batched(b, 1)
        res["f1_default_schedule_mpx_s"] = round(work / wall / 1e6, 1)
        train_all()
        wall = run_per_stream(1)
        res["f1_per_stream_launches_mpx_s"] = round(work / wall / 1e6, 1)
        log(f"batch: default schedule {res['f1_default_schedule_mpx_s']} Mpx/s, "
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


def cpu_baseline(frames, spec, budget_s):
    """The oracle (single thread) on a pixel sample of the same stream."""
    from oracle import oracle as O

    P, T, N, K = spec.pixels, spec.frames, spec.n_train, spec.K
    flat = frames.reshape(T, P, 3)

    def run(stride):
        idx = np.arange(0, P, stride)
        sub = np.ascontiguousarray(flat[:, idx][:, None])
        orc = O.Oracle(O.make_params(len(idx), 1, 3, K))
        ts = time.perf_counter()
        orc.train(sub[:N])
        for t in range(N, T):
            orc.step(sub[t])
        el = time.perf_counter() - ts
        orc.close()
        return len(idx), el

    n0, e0 = run(256)
    stride = max(1, int(math.ceil(256 * e0 / budget_s)))
    n, el = run(stride)
    log(f"cpu oracle: {n} px x {T} frames in {el:.1f} s")
    return {"value": round(n * T / el / 1e6, 3), "unit": "Mpixel-frames/s", "cores": 1,
            "kind": "oracle",
            "sample": f"every {stride}th pixel ({n} px) of all {T} frames: training over {N}, "
                      f"cascade over {T - N}",
            "host": platform.processor() or platform.machine(), "seconds": round(el, 2)}


if __name__ == "__main__":
    main()
