#!/usr/bin/env python3
"""Throughput of the blob-detection filter bank on one MI355X.

Workload: one 2048 x 2048 uint16 frame (12-bit aerial-like synthetic), 8
scales sigma = 2..64 (geometric).  One step = the whole hot path:
    filter design (host, closed form)
    -> IIR row pass (x) -> IIR column pass (y)        [repeated pole, K = 3]
    -> normalised Laplacian sigma^2 (D20 + D02)
    -> multi-scale strict extrema -> ordered blob list (on the device).
The FIR form of the same step (coloured Savitzky-Golay blur of length
6 sigma + 1, direct convolution; taps designed once) is timed alongside.

Metric: Mpixel*scales/s = H * W * S / (seconds per step); the input is already
resident in HBM.  Per-kernel durations come from HIP events recorded on the
stream the kernels run on.  The FP64 oracle of the same step is timed on the
host (cpu_baseline) and its result is used to check the GPU output of the
timed run.

Prints ONE JSON line on stdout.  Usage:
    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
EV_EVERY = 4   # timed steps per step with unit events (the units' average launch durations)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha(name: str) -> str | None:
    """sha of one kernel source (None if it no longer exists)."""
    path = os.path.join(ROOT, "paper_1912_07133_amd", "csrc", name)
    if not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _oracle_response(job):
    """One scale of the FP64 oracle in a worker process: the IIR (K = 3,
    Table IV) or the coloured SG FIR blur of the frame, then its normalised
    Laplacian.  Returns (blur plane, V plane) as float64."""
    import numpy as np

    from oracle import design, filtering, shape
    frame, sigma, kind = job
    f64 = frame.astype(np.float64)
    if kind == "iir":
        B = filtering.blur_2d(f64, design.table_iv(sigma))
    else:
        B = filtering.blur_2d_matrix(f64, design.colored_sg_taps(sigma))
    return B, shape.laplacian(B, sigma)


def host_cpu():
    """(usable cores, model name) of the host."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def run_batch_leg(P, syn, torch, np, dev, stream, log):
    """64 frames of uneven size (16 each of 512x512, 1920x1080, 4096x3072,
    2048x2048, uint16 12-bit, the full-frame generator with 200 blobs per
    2048^2 pixels, frame f with seed 1000 + f), 12 scales sigma = 1.5..96,
    repeated-pole K = 3, fused Laplacian and extrema.  Timed three ways:
    one frame and one scale per launch sequence, one frame per call, and the
    whole batch in one call over autotuned lanes, captured into a graph."""
    cfg = syn.BATCH
    sig = cfg["sigmas"]
    S = len(sig)
    specs = syn.batch_frames(64, seed=2)
    log(f"batch: generating {len(specs)} frames ...")
    frames = []
    for H, W, seed in specs:
        a = syn.aerial_frame(H, W, seed, nblobs=max(1, int(round(200 * H * W / 2048 ** 2))))
        frames.append(torch.from_numpy(a.view(np.int16)).to(dev))
    torch.cuda.synchronize()
    mpx_scales = sum(H * W for H, W, _ in specs) * S / 1e6
    reps = 5

    def timed_ms(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # (a) per frame and per scale: the fused blur + Laplacian of one scale per
    # call into the frame's V planes, then the frame's detection
    Hm = max(H for H, _, _ in specs)
    Wm = max(W for _, W, _ in specs)
    V = torch.empty(S * Hm * Wm, dtype=torch.float32, device=dev)
    ws1 = torch.empty(P.workspace_bytes(P.OP_IIR_LAPLACIAN, Hm, Wm, 1), dtype=torch.uint8, device=dev)
    wsd = torch.empty(P.workspace_bytes(P.OP_DETECT, Hm, Wm, S), dtype=torch.uint8, device=dev)
    cap = 1 << 16
    blobs = torch.empty(cap * P.BLOB_BYTES, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    filt = P.iir_designs(sig, 3)
    L = P.lib()
    sp = int(stream.cuda_stream)

    def per_frame_per_scale():
        for f in frames:
            H, W = f.shape
            for s in range(S):
                L.fdvm_iir_laplacian(f.data_ptr(), P.U16, H, W, W, V.data_ptr() + 4 * s * H * W, W, H * W,
                                     ctypes.byref(filt[s]), 1, P.BC_REPLICATE, ws1.data_ptr(), ws1.numel(), sp)
            L.fdvm_detect_blobs(V.data_ptr(), H, W, W, H * W, S, cfg["tau"], cfg["border"], blobs.data_ptr(), cap,
                                cnt.data_ptr(), wsd.data_ptr(), wsd.numel(), sp)

    t_pfps = timed_ms(per_frame_per_scale)
    # (b) one frame per call (all scales), one lane
    b1 = P.Batch(frames, sig, cfg["tau"], nlanes=1, cap=cap)
    t_pf = timed_ms(b1.run)
    del b1
    # (c) autotuned lanes and row chunks, whole batch captured in one graph
    nl, chunks, _ = P.autotune_batch(frames, sig, cfg["tau"], lanes=(1, 2, 4, 8), reps=2, cap=cap)
    b = P.Batch(frames, sig, cfg["tau"], nlanes=nl, row_chunks=chunks, cap=cap)
    b.run()
    torch.cuda.synchronize()
    eager_counts = b.counts.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        b.run()
    t_graph = timed_ms(g.replay)
    same = bool(torch.equal(b.counts, eager_counts))
    # algorithmic bytes of the batch: per frame the fused unit (frame read once,
    # S intermediate planes written and read, S planes of V written) and the
    # detection (S planes of V read), H W (2 + 16 S); far above the 256 MB
    # Infinity Cache, so this is the HBM-bound figure
    alg_bytes = sum(H * W for H, W, _ in specs) * (2 + 16 * S)
    gbs = alg_bytes / (t_graph / 1e3) / 1e9
    out = {"workload": cfg["name"], "frames": len(specs), "scales": S, "mpx_scales": round(mpx_scales, 1),
           "per_frame_per_scale": {"ms": round(t_pfps, 3), "value": round(mpx_scales / (t_pfps / 1e3), 1)},
           "per_frame": {"ms": round(t_pf, 3), "value": round(mpx_scales / (t_pf / 1e3), 1)},
           "graph": {"ms": round(t_graph, 3), "value": round(mpx_scales / (t_graph / 1e3), 1), "lanes": nl,
                     "row_chunks": sorted({(int(f.shape[1]), int(c)) for f, c in zip(frames, chunks)}),
                     "replay_counts_match_eager": same, "algorithmic_bytes": alg_bytes,
                     "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)},
           "detections": int(b.counts.sum().item()), "unit": "Mpixel·scales/s"}
    log(f"batch: {mpx_scales:.0f} Mpx*scales; per frame+scale {t_pfps:.2f} ms, per frame {t_pf:.2f} ms, "
        f"graph ({nl} lanes) {t_graph:.2f} ms = {out['graph']['value']:.0f} Mpx*scales/s, "
        f"{gbs:.0f} GB/s algorithmic ({100 * gbs / HBM_PEAK_GBS:.1f} % of 8 TB/s)")
    return out


def run_grad_leg(P, syn, torch, np, dev, stream, log):
    """16 float32 frames of 1024 x 1024 (the full-frame generator / 4095,
    50 blobs each, seeds 500 + f) as one batch, sigma = 3, 6, 12, 24
    learnable: the blur + normalised Laplacian forward (frame after frame) and
    the backward of loss = sum over the detected centres of V^2 in the image
    and sigma, one fdvm_*_laplacian_backward call for the batch; Mpixel*scales/s
    of forward + backward, IIR (the C5 step) and the FIR form beside it."""
    cfg = syn.DIFFERENTIATION
    sig = cfg["sigmas"]
    X = torch.stack([torch.from_numpy(syn.normalised_frame(cfg["H"], cfg["W"], 500 + f, nblobs=cfg["nblobs"])
                                      .astype(np.float32)) for f in range(cfg["frames"])]).to(dev)
    cs = []
    for f in range(cfg["frames"]):
        det = P.detect_blobs(P.iir_laplacian(X[f], sig), 0.02, 1)
        cs += [(f, int(d["scale"]), int(d["y"]), int(d["x"])) for d in det]
    c = torch.tensor(cs, dtype=torch.long, device=dev)

    def make_step(fn):
        def step():
            sig_t = torch.tensor(sig, dtype=torch.float64, device=dev, requires_grad=True)
            xr = X.detach().requires_grad_(True)
            V = fn(xr, sig_t)
            loss = (V[c[:, 0], c[:, 1], c[:, 2], c[:, 3]].double() ** 2).sum()
            loss.backward()
            return sig_t.grad
        return step

    def timed(step, reps=5):
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_wall = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            g = step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, (time.perf_counter() - t_wall) * 1e3 / reps, g

    mpx = cfg["frames"] * cfg["H"] * cfg["W"] * len(sig) / 1e6
    ms, wall_ms, g = timed(make_step(P.iir_laplacian_grad))
    out = {"workload": cfg["name"], "ms_fwd_bwd": round(ms, 3), "value": round(mpx / (ms / 1e3), 1),
           "unit": "Mpixel·scales/s (forward + backward)", "dL_dsigma": [round(float(v), 8) for v in g.cpu()],
           "centres": len(cs), "wall_ms": round(wall_ms, 3), "batch": "one backward call for the 16 frames"}
    fms, fwall, fg = timed(make_step(P.fir_laplacian_grad))
    out["fir"] = {"ms_fwd_bwd": round(fms, 3), "value": round(mpx / (fms / 1e3), 1), "wall_ms": round(fwall, 3),
                  "dL_dsigma": [round(float(v), 8) for v in fg.cpu()],
                  "form": "coloured SG, K = ceil(3 sigma), float64 FIR forward, float32 backward"}
    log(f"grad: 16 x 1024^2 x 4 scales forward + backward IIR {ms:.2f} ms (wall {wall_ms:.2f} ms) = "
        f"{out['value']:.0f} Mpx*scales/s; FIR {fms:.2f} ms = {out['fir']['value']:.0f}")
    return out


def run_precision_leg(P, syn, torch, np, dev, stream, log):
    """One 8192 x 8192 frame (generator seed 3, 3200 blobs, / 4095) stored as
    float16 and as bfloat16; coloured SG FIR of lengths 33, 65, 129, 257
    (sigma = K / 3: direct, Toeplitz on the matrix cores with float32 operands
    and with the frame's half type as operands) and the K = 3 IIR at the same
    sigmas.  Throughput per form; the outputs at 16 sampled pixels are kept
    for the error figures, which the CPU-baseline leg computes against FP64
    references (precision_errors)."""
    cfg = syn.PRECISION
    Ks = [(m - 1) // 2 for m in cfg["fir_lengths"]]
    sig = [k / 3 for k in Ks]
    orig = syn.normalised_frame(cfg["H"], cfg["W"], cfg["seed"], nblobs=cfg["nblobs"])
    rng = np.random.default_rng(5)
    pts = [tuple(int(v) for v in p) for p in rng.integers(0, cfg["H"], (16, 2))]
    mpx = cfg["H"] * cfg["W"] * len(sig) / 1e6
    out = {"workload": cfg["name"], "scales": [round(s, 4) for s in sig], "fir_lengths": cfg["fir_lengths"],
           "error": "max |gpu - fp64| / max |fp64| over 16 sampled pixels, per scale", "forms": {},
           "_pts": pts, "_sig": sig, "_Ks": Ks, "_samples": {}}
    # designs, output planes and workspaces made once, outside the timed calls
    tp = P.fir_taps("sg", sig, Ks)
    outB = torch.empty((len(sig), cfg["H"], cfg["W"]), dtype=torch.float32, device=dev)
    ws_f = torch.empty(P.workspace_bytes(P.OP_BLUR_FIR, cfg["H"], cfg["W"], len(sig), max(Ks)), dtype=torch.uint8,
                       device=dev)
    ws_i = torch.empty(P.workspace_bytes(P.OP_BLUR_IIR, cfg["H"], cfg["W"], len(sig)), dtype=torch.uint8, device=dev)
    for kind, tdt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        x = torch.from_numpy(orig.astype(np.float32)).to(tdt).to(dev)

        def fir_form(algo):
            return lambda: P.blur_fir(x, sig, kind="sg", half_lens=Ks, algo=algo, out=outB, workspace=ws_f, taps=tp)

        runs = {"iir": lambda: P.blur_iir(x, sig, order=3, out=outB, workspace=ws_i),
                "fir_direct": fir_form(P.FIR_DIRECT),
                "fir_mfma": fir_form(P.FIR_TOEPLITZ_MFMA),
                "fir_mfma_half": fir_form(P.FIR_TOEPLITZ_MFMA_HALF)}
        for name, fn in runs.items():
            B = fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                B = fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            idx = torch.tensor([i * cfg["W"] + j for i, j in pts], device=dev)
            Bn = B.reshape(len(sig), -1)[:, idx].cpu().numpy()
            out["_samples"][f"{kind}_{name}"] = [[float(v) for v in Bn[s]] for s in range(len(sig))]
            out["forms"][f"{kind}_{name}"] = {"ms": round(ms, 3), "value": round(mpx / (ms / 1e3), 1)}
            if name == "fir_mfma_half":
                fl = half_mfma_flops(cfg["H"], cfg["W"], Ks)
                out["forms"][f"{kind}_{name}"]["mfma_issued_tflops"] = round(fl / (ms / 1e3) / 1e12, 1)
                out["forms"][f"{kind}_{name}"]["mfma_frac_of_dense_peak"] = round(fl / (ms / 1e3) / 2.5e15, 4)
            del B
        log(f"precision {kind}: " + ", ".join(f"{k.split('_', 1)[1]} {v['ms']:.2f} ms"
                                            for k, v in out["forms"].items() if k.startswith(kind)))
    del outB, ws_f, ws_i
    return out


def half_mfma_flops(H, W, Ks, first_pass_products=2):
    """Matrix-core flops the half-operand Toeplitz FIR issues for one H x W
    frame: per pass and scale, one wavefront per 32 rows x 64 outputs along
    the rows runs 2 K'/16 + 4 groups of 16 samples (K' = K rounded up to 32),
    each meeting one 32 x 32 output block in the first and last two groups and
    both otherwise, with 2 products per block in the first pass (hi and lo
    taps; 3 for uint16 frames, whose samples are split too) and 3 in the
    second (the split intermediate); 32 * 32 * 16 * 2 flops each.  The first
    pass covers the intermediate's padded rows: H rounded up to an odd number
    of 64-sample lines."""
    total = 0
    hp = 64 * ((-(-H // 64)) | 1)
    for K in Ks:
        kp = -(-K // 32) * 32
        blocks = 2 * (2 * kp // 16 + 4) - 4
        for (rows, n), prods in (((hp, W), first_pass_products), ((W, H), 3)):
            waves = -(-rows // 32) * -(-n // 64)
            total += waves * blocks * prods * 32 * 32 * 16 * 2
    return total


def precision_errors(prec, syn, torch, np, log):
    """Per scale, the largest relative error of the sampled GPU outputs of the
    precision leg against float64 direct 2-D sums of the FP64 oracle's taps
    (the IIR's impulse response truncated at 30 sigma), for the stored and for
    the original input.  Part of the CPU-baseline leg."""
    from oracle import design, filtering

    cfg = syn.PRECISION
    pts, sig, Ks = prec["_pts"], prec["_sig"], prec["_Ks"]
    orig = syn.normalised_frame(cfg["H"], cfg["W"], cfg["seed"], nblobs=cfg["nblobs"])

    def sampled(img, h):
        K = (len(h) - 1) // 2
        r = np.arange(-K, K + 1)
        H, W = img.shape
        return np.array([h @ img[np.ix_(np.clip(i - r, 0, H - 1), np.clip(j - r, 0, W - 1))] @ h for i, j in pts])

    taps = {"fir": [design.colored_sg_taps(s, K=K) for s, K in zip(sig, Ks)],
            "iir": [filtering.impulse_response_by_recursion(design.repeated_pole(3, s), int(30 * s) + 8)
                    for s in sig]}
    for kind, tdt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        deq = torch.from_numpy(orig.astype(np.float32)).to(tdt).float().numpy().astype(np.float64)
        for name in ("iir", "fir_direct", "fir_mfma", "fir_mfma_half"):
            key = f"{kind}_{name}"
            if key not in prec["_samples"]:
                continue
            hs = taps["iir" if name == "iir" else "fir"]
            eq, eo = [], []
            for s in range(len(sig)):
                g = np.array(prec["_samples"][key][s], dtype=np.float64)
                rq, ro = sampled(deq, hs[s]), sampled(orig, hs[s])
                eq.append(float(np.max(np.abs(g - rq)) / np.max(np.abs(rq))))
                eo.append(float(np.max(np.abs(g - ro)) / np.max(np.abs(ro))))
            prec["forms"][key]["err_vs_stored"] = [float(f"{v:.3g}") for v in eq]
            prec["forms"][key]["err_vs_original"] = [float(f"{v:.3g}") for v in eo]
        log(f"precision {kind} errors vs original: " +
            ", ".join(f"{k.split('_', 1)[1]} {max(v['err_vs_original']):.2e}"
                      for k, v in prec["forms"].items() if k.startswith(kind) and "err_vs_original" in v))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fir", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-butterworth", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="report the plain 256 MiB device copy in the output (for PMC byte scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(frames and scales are independent and would shard across GPUs without any exchange)",
              file=sys.stderr)
        return 2

    # worker processes for the all-cores oracle baseline, started before
    # anything touches the GPU (they never do); at most 16, the host share of
    # one GPU
    pool = None
    ncores, cpu_model = host_cpu()
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        ncores = max(1, min(16, ncores))
        pool = mp.get_context("spawn").Pool(ncores)

    import numpy as np
    import torch

    import paper_1912_07133_amd as P
    import synthetic as syn

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = P.lib()
    cfg = syn.FULL_FRAME
    H, W, sig = cfg["H"], cfg["W"], cfg["sigmas"]
    S = len(sig)
    tau, border = cfg["tau"], cfg["border"]
    frame = syn.aerial_frame(H, W, cfg["seed"])
    t0 = time.perf_counter()
    x = torch.from_numpy(frame.view(np.int16)).to(dev)
    torch.cuda.synchronize()
    h2d_ms = (time.perf_counter() - t0) * 1e3

    V = torch.empty((S, H, W), dtype=torch.float32, device=dev)   # sigma^2 (D20 + D02)
    B = torch.empty((S, H, W), dtype=torch.float32, device=dev)   # FIR blur planes
    cap = 1 << 20
    blobs = torch.empty(cap * P.BLOB_BYTES, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    ws_det = torch.empty(P.workspace_bytes(P.OP_DETECT, H, W, S), dtype=torch.uint8, device=dev)
    # x-pass intermediate (S fixed-point planes), column states, row exponents
    ws_iir = torch.empty(P.workspace_bytes(P.OP_IIR_LAPLACIAN, H, W, S), dtype=torch.uint8, device=dev)
    sigmas_c = (ctypes.c_double * S)(*sig)
    stream = torch.cuda.current_stream(dev)
    sp = int(stream.cuda_stream)

    # a plain device copy of known size (256 MiB read + 256 MiB written): its
    # rate is the practical HBM ceiling the roofline fraction is read against,
    # and with --calibrate-copy its PMC byte counts scale the counters.  It
    # runs first, 20 timed copies (≈ 2 ms), before any leg.
    src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ncopy = 20
    c0.record(stream)
    for _ in range(ncopy):
        torch.mul(src, 1.0, out=dst)   # elementwise: reads 256 MiB, writes 256 MiB
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = ncopy * 2 * src.numel() * 4 / (c0.elapsed_time(c1) / 1e3) / 1e9
    extra_copy = {"bytes_each_way": src.numel() * 4} if args.calibrate_copy else None
    del src, dst

    def check(st, what):
        if st != P.OK:
            raise P.FdvmError(st, what)

    def designs():
        filt = (P.Filter * S)()
        for i, s in enumerate(sig):
            check(L.fdvm_filter_design(P.IIR_REPEATED_POLE, 3, s, 0, ctypes.byref(filt[i]), None, 0), "design")
        return filt

    def detect_into(ev_det):
        check(L.fdvm_detect_blobs(V.data_ptr(), H, W, W, H * W, S, tau, border, blobs.data_ptr(), cap,
                                  count.data_ptr(), ws_det.data_ptr(), ws_det.numel(), sp), "detect")
        ev_det.record(stream)

    def iir_step(ev):
        filt = designs()
        ev[0].record(stream)
        check(L.fdvm_iir_laplacian(x.data_ptr(), P.U16, H, W, W, V.data_ptr(), W, H * W, filt, S,
                                   P.BC_REPLICATE, ws_iir.data_ptr(), ws_iir.numel(), sp), "iir_laplacian")
        ev[1].record(stream)
        detect_into(ev[2])

    class NoEvent:
        """stands in for the unit events of a step that is not sampled"""
        def record(self, _stream):
            pass

    def timed(step_fn, nev, steps, warmup):
        """K steps between two events (the step rate); the units' durations
        from HIP events around them on every EV_EVERY-th of those steps: a
        timing event costs about 3 us on the stream, so recording three in
        every step would add about 10 us to each step it is meant to measure"""
        for _ in range(warmup):
            step_fn([NoEvent() for _ in range(nev)])
        torch.cuda.synchronize()
        every = EV_EVERY if steps >= 2 * EV_EVERY else 1
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] if i % every == 0
               else [NoEvent() for _ in range(nev)] for i in range(steps)]
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        start.record(stream)
        for e in evs:
            step_fn(e)
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        total_ms = start.elapsed_time(stop)
        sampled = [e for e in evs if not isinstance(e[0], NoEvent)]
        per = [[e[i].elapsed_time(e[i + 1]) for e in sampled] for i in range(nev - 1)]
        return total_ms, wall, [float(np.mean(p)) for p in per]

    # ---------------- IIR path
    log(f"IIR: {H}x{W} u16, {S} scales, warmup {args.warmup}, steps {args.steps}")
    total_ms, wall, per = timed(iir_step, 3, args.steps, args.warmup)
    ms_step = total_ms / args.steps
    n_det = int(count.item())
    mpx = H * W * S / 1e6
    value = mpx / (ms_step / 1e3)
    # algorithmic bytes per call (two-pass schedule): the x pass reads the
    # frame once for all scales and writes S intermediate planes (4 B/px); the
    # y pass with the fused Laplacian reads them and writes S planes of V;
    # detection reads the S planes of V once
    kern = {
        "iir_laplacian": {"ms": per[0], "bytes": H * W * (2 + 12 * S), "kernels": 4},
        "detect": {"ms": per[1], "bytes": H * W * S * 4, "kernels": 3},
    }
    for k in kern.values():
        k["GB/s"] = k["bytes"] / (k["ms"] / 1e3) / 1e9
    dominant = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dominant]
    traffic = None
    if os.path.exists(PMC_FILE):
        with open(PMC_FILE) as f:
            pmc = json.load(f)
        ent = pmc.get("kernels", {}).get(dominant)
        if ent and all(ent.get("source_sha", {}).get(n) == kernel_source_sha(n) for n in ent.get("sources", [])):
            traffic = ent["hbm_bytes_per_launch"]
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(d["GB/s"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(d["GB/s"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": d["bytes"], "avg_launch_ms": round(d["ms"], 5),
                "kernels_in_launch": d["kernels"]}
    log(f"IIR: {ms_step:.4f} ms/step, {value:.0f} Mpx*scales/s, detections {n_det}; "
        + ", ".join(f"{k} {v['ms']:.4f} ms ({v['GB/s']:.0f} GB/s)" for k, v in kern.items()))

    # keep the outputs of the timed IIR run for the parity check
    V_gpu = V.cpu().numpy()
    raw = blobs[: min(n_det, cap) * P.BLOB_BYTES].cpu().numpy()
    det_gpu = raw.view(np.dtype([("y", np.int32), ("x", np.int32), ("scale", np.int32),
                                 ("polarity", np.int32), ("value", np.float32)]))

    # ---------------- FIR path (coloured SG, length 6 sigma + 1)
    # The detection form: fdvm_fir_laplacian (float64 FIR passes, V formed
    # before any rounding of the blur) -> detection, checked against the
    # oracle in the CPU-baseline leg.  The float32 blur alone, direct and on
    # the matrix cores, is timed beside it.
    fir = None
    V_fir = det_fir = V_firm = det_firm = None
    if not args.no_fir:
        taps_d, half, off = P.fir_taps_device("sg", sig, None, dev)
        taps, _, _ = P.fir_taps("sg", sig)
        taps = np.ascontiguousarray(taps)
        ws_fir = torch.empty(P.workspace_bytes(P.OP_BLUR_FIR, H, W, S, int(half.max())), dtype=torch.uint8,
                             device=dev)
        ws_firlap = torch.empty(P.workspace_bytes(P.OP_FIR_LAPLACIAN, H, W, S), dtype=torch.uint8, device=dev)
        ws_firlapm = torch.empty(P.workspace_bytes(P.OP_FIR_LAPLACIAN_MFMA, H, W, S), dtype=torch.uint8,
                                 device=dev)
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)

        sig_from = [(ctypes.c_double * (S - s0))(*sig[s0:]) for s0 in range(S)]

        def fir_fused(ev, s0=0, ns=S):
            ev[0].record(stream)
            check(L.fdvm_fir_laplacian(x.data_ptr(), P.U16, H, W, W, V.data_ptr() + 4 * s0 * H * W, W, H * W,
                                       taps_d.data_ptr(), half[s0:].ctypes.data_as(ip),
                                       off[s0:].ctypes.data_as(ip), sig_from[s0], ns, P.BC_REPLICATE,
                                       ws_firlap.data_ptr(), ws_firlap.numel(), sp), "fir_laplacian")
            ev[1].record(stream)

        def fir_step(ev):
            fir_fused(ev)
            detect_into(ev[2])

        sig_all = (ctypes.c_double * S)(*sig)

        def fir_step_mfma(ev):
            ev[0].record(stream)
            check(L.fdvm_fir_laplacian_mfma(x.data_ptr(), P.U16, H, W, W, V.data_ptr(), W, H * W,
                                            taps.ctypes.data_as(dp), half.ctypes.data_as(ip),
                                            off.ctypes.data_as(ip), sig_all, S, P.BC_REPLICATE,
                                            ws_firlapm.data_ptr(), ws_firlapm.numel(), sp), "fir_laplacian_mfma")
            ev[1].record(stream)
            detect_into(ev[2])

        def fir_blur_for(algo):
            def step(ev):
                ev[0].record(stream)
                check(L.fdvm_blur_fir(x.data_ptr(), P.U16, H, W, W, B.data_ptr(), W, H * W,
                                      taps.ctypes.data_as(dp), half.ctypes.data_as(ip), off.ctypes.data_as(ip), S,
                                      P.BC_REPLICATE, algo, ws_fir.data_ptr(), ws_fir.numel(), sp), "fir")
                ev[1].record(stream)
            return step

        fsteps = max(5, args.steps // 10)
        ntaps = [int(2 * k + 1) for k in half]
        fir = {"kind": "colored_sg", "taps": ntaps, "steps": fsteps}
        # useful flops of the blur: 2 (2K + 1) per pixel per 1-D pass, two passes
        useful = sum(4.0 * t for t in ntaps) * H * W
        ftot, _, fper = timed(fir_step, 3, fsteps, max(1, args.warmup // 5))
        fms = ftot / fsteps
        n_fir = int(count.item())
        V_fir = V.cpu().numpy()
        det_fir = blobs[: min(n_fir, cap) * P.BLOB_BYTES].cpu().numpy().view(P.BLOB_DTYPE).copy()
        fir["fused"] = {"value": round(mpx / (fms / 1e3), 1), "ms_per_step": round(fms, 4),
                        "fir_laplacian_ms": round(fper[0], 4), "detect_ms": round(fper[1], 4),
                        "float64_useful_TFLOPs": round(useful / (fper[0] / 1e3) / 1e12, 2),
                        "detections": n_fir, "step": "fdvm_fir_laplacian (float64 FIR passes) + detection"}
        log(f"FIR fused: {fms:.4f} ms/step, {fir['fused']['value']:.0f} Mpx*scales/s "
            f"(fir_laplacian {fper[0]:.3f} ms), detections {n_fir}")
        # the same detection response on the matrix cores (two-stage band-pass)
        mtot, _, mper = timed(fir_step_mfma, 3, fsteps, max(1, args.warmup // 5))
        mms = mtot / fsteps
        n_firm = int(count.item())
        V_firm = V.cpu().numpy()
        det_firm = blobs[: min(n_firm, cap) * P.BLOB_BYTES].cpu().numpy().view(P.BLOB_DTYPE).copy()
        fir["fused_mfma"] = {"value": round(mpx / (mms / 1e3), 1), "ms_per_step": round(mms, 4),
                             "fir_laplacian_ms": round(mper[0], 4), "detect_ms": round(mper[1], 4),
                             "detections": n_firm,
                             "step": "fdvm_fir_laplacian_mfma (matrix cores, float16 operand pairs, the two-stage "
                                     "band-pass h(y) d(x) + d(y) h(x), d = h * [1, -2, 1]) + detection"}
        log(f"FIR fused (matrix cores): {mms:.4f} ms/step, {fir['fused_mfma']['value']:.0f} Mpx*scales/s "
            f"(fir_laplacian_mfma {mper[0]:.3f} ms), detections {n_firm}")
        fir["blur_only"] = {}
        arith = {"direct": "float32", "mfma": "float32 operands and accumulation",
                 "mfma_half": "float16 operand pairs (exact split of the uint16 samples), float32 accumulation"}
        for name, algo in (("direct", P.FIR_DIRECT), ("mfma", P.FIR_TOEPLITZ_MFMA),
                           ("mfma_half", P.FIR_TOEPLITZ_MFMA_HALF)):
            btot, _, bper = timed(fir_blur_for(algo), 2, fsteps, max(1, args.warmup // 5))
            fir["blur_only"][name] = {"blur_ms": round(bper[0], 4),
                                      "value": round(mpx / (bper[0] / 1e3), 1),
                                      "useful_TFLOPs": round(useful / (bper[0] / 1e3) / 1e12, 2),
                                      "arith": arith[name]}
            if name == "mfma_half":
                fl = half_mfma_flops(H, W, [int(k) for k in half], first_pass_products=3)
                fir["blur_only"][name]["mfma_issued_tflops"] = round(fl / (bper[0] / 1e3) / 1e12, 1)
                fir["blur_only"][name]["mfma_frac_of_dense_peak"] = round(fl / (bper[0] / 1e3) / 2.5e15, 4)
            log(f"FIR blur {name}: {bper[0]:.3f} ms ({fir['blur_only'][name]['useful_TFLOPs']} useful TFLOP/s)")
        # per scale: the IIR and the FIR detection responses of one scale per call
        filt_all = designs()
        per_scale = []
        reps = 5
        for s0 in range(S):
            def iir_one(ev, s0=s0):
                ev[0].record(stream)
                check(L.fdvm_iir_laplacian(x.data_ptr(), P.U16, H, W, W, V.data_ptr() + 4 * s0 * H * W, W, H * W,
                                           ctypes.byref(filt_all[s0]), 1, P.BC_REPLICATE, ws_iir.data_ptr(),
                                           ws_iir.numel(), sp), "iir_laplacian")
                ev[1].record(stream)
            _, _, pi = timed(iir_one, 2, reps, 1)
            _, _, pf = timed(lambda ev, s0=s0: fir_fused(ev, s0, 1), 2, reps, 1)
            per_scale.append({"sigma": round(sig[s0], 3), "fir_taps": ntaps[s0],
                              "iir_ms": round(pi[0], 4), "iir_value": round(H * W / 1e6 / (pi[0] / 1e3), 1),
                              "fir_ms": round(pf[0], 4), "fir_value": round(H * W / 1e6 / (pf[0] / 1e3), 1)})
        fir["per_scale"] = {"unit": "Mpixel/s of one scale's blur + normalised Laplacian (one scale per call)",
                            "scales": per_scale}
        log("per scale (sigma: IIR / FIR Mpx/s): " +
            ", ".join(f"{p['sigma']}: {p['iir_value']:.0f} / {p['fir_value']:.0f}" for p in per_scale))

    # ---------------- Butterworth form of the IIR step (Filter E blur, L_B = 4)
    butterworth = None
    if not args.no_butterworth:
        def designs_bw():
            filt = (P.Filter * S)()
            for i, s in enumerate(sig):
                check(L.fdvm_filter_design(P.IIR_BUTTERWORTH, 4, s, 0, ctypes.byref(filt[i]), None, 0), "design")
            return filt

        def bw_step(ev):
            filt = designs_bw()
            ev[0].record(stream)
            check(L.fdvm_iir_laplacian(x.data_ptr(), P.U16, H, W, W, V.data_ptr(), W, H * W, filt, S,
                                       P.BC_REPLICATE, ws_iir.data_ptr(), ws_iir.numel(), sp), "iir_laplacian")
            ev[1].record(stream)
            detect_into(ev[2])

        steps_bw = max(10, args.steps // 4)
        tot_bw, _, per_bw = timed(bw_step, 3, steps_bw, 3)
        ms_bw = tot_bw / steps_bw
        butterworth = {"blur": "Butterworth L_B = 4 (Filter E), omega_c = sqrt(2 ln 2) / sigma",
                       "steps": steps_bw, "ms_per_step": round(ms_bw, 4), "value": round(mpx / (ms_bw / 1e3), 1),
                       "iir_laplacian_ms": round(per_bw[0], 5), "detect_ms": round(per_bw[1], 5),
                       "detections": int(count.item())}
        log(f"Butterworth: {ms_bw:.4f} ms/step, {butterworth['value']:.0f} Mpx*scales/s, "
            f"iir_laplacian {per_bw[0]:.4f} ms, detections {butterworth['detections']}")

    # ---------------- batch: 64 uneven frames x 12 scales
    batch = None
    if not args.no_batch:
        batch = run_batch_leg(P, syn, torch, np, dev, stream, log)

    # ---------------- differentiation: 16 x 1024^2, forward + backward
    grad = None
    if not args.no_grad:
        grad = run_grad_leg(P, syn, torch, np, dev, stream, log)

    # ---------------- reduced-precision storage: 8192^2 float16 / bfloat16
    precision = None
    if not args.no_precision:
        precision = run_precision_leg(P, syn, torch, np, dev, stream, log)

    # ---------------- CPU baseline: the FP64 oracle on the same frame
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        from oracle import design, filtering, shape
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import compare_detections

        from parity import laplacian_tolerance

        log("cpu baseline: FP64 oracle, whole frame, 8 scales, one thread ...")
        t0 = time.perf_counter()
        B_ref = filtering.blur_bank(frame.astype(np.float64), [design.table_iv(s) for s in sig])
        V_ref = shape.laplacian_bank(B_ref, sig)
        det_ref = shape.detect_extrema(V_ref, tau, border)
        t_cpu = time.perf_counter() - t0
        log(f"cpu baseline: the same on {ncores} worker processes ...")
        t0 = time.perf_counter()
        res = pool.map(_oracle_response, [(frame, s, "iir") for s in sig])
        V_par = np.stack([r[1] for r in res])
        det_par = shape.detect_extrema(V_par, tau, border)
        t_par = time.perf_counter() - t0
        del res
        same_ref = bool(np.array_equal(V_par, V_ref)) and len(det_par) == len(det_ref)
        cpu = {"value": round(mpx / t_par, 3), "unit": "Mpixel·scales/s", "cores": ncores, "kind": "oracle",
               "cpu_model": cpu_model,
               "sample": f"one full {H}x{W} frame x {S} scales (IIR K=3 blur, Laplacian, extrema), numpy float64, "
                         f"one scale per worker process ({ncores} processes), extrema on one thread, "
                         f"{t_par:.1f} s; same result as the one-thread run: {same_ref}",
               "single_thread": {"value": round(mpx / t_cpu, 3), "cores": 1, "seconds": round(t_cpu, 2)}}
        vratio = max(float(np.max(np.abs(V_gpu[s] - V_ref[s]))) / laplacian_tolerance(sig[s], B_ref[s])
                     for s in range(S))
        vb = [laplacian_tolerance(sg, B_ref[s]) for s, sg in enumerate(sig)]
        nfrag, mism = compare_detections(det_gpu, det_ref, V_ref, V_gpu, tau, border, v_bound=vb)
        parity = {"laplacian_err_over_tolerance": round(vratio, 4),
                  "laplacian_tolerance": "8 sigma^2 * 4 ulp(max|B|) per plane", "detections": int(len(det_gpu)),
                  "oracle_detections": int(len(det_ref)), "fragile_excluded": nfrag,
                  "mismatches": len(mism),
                  "rule": "equal outside the fragile set; the GPU list equals the oracle's extremum rule on the "
                          "GPU's own V",
                  "ok": bool(vratio <= 1.0 and not mism and nfrag <= 0.001 * V_gpu.size)}
        log(f"cpu baseline {cpu['value']} Mpx*scales/s on {ncores} cores "
            f"({cpu['single_thread']['value']} on one); parity {parity}")
        del B_ref, V_ref, V_par
        if V_fir is not None:
            # the FIR detection route against the FIR oracle (the separable sum
            # as two matrix products per scale), with the FIR oracle's timing
            log("cpu baseline: FP64 FIR oracle ...")
            t0 = time.perf_counter()
            res = pool.map(_oracle_response, [(frame, s, "fir") for s in sig])
            Bf = np.stack([r[0] for r in res])
            Vf = np.stack([r[1] for r in res])
            det_ref_f = shape.detect_extrema(Vf, tau, border)
            t_fir = time.perf_counter() - t0
            del res
            vratio_f = max(float(np.max(np.abs(V_fir[s] - Vf[s]))) / laplacian_tolerance(sig[s], Bf[s])
                           for s in range(S))
            vbf = [laplacian_tolerance(sg, Bf[s]) for s, sg in enumerate(sig)]
            nfrag_f, mism_f = compare_detections(det_fir, det_ref_f, Vf, V_fir, tau, border, v_bound=vbf)
            fir["parity"] = {"laplacian_err_over_tolerance": round(vratio_f, 4), "detections": int(len(det_fir)),
                             "oracle_detections": int(len(det_ref_f)), "fragile_excluded": nfrag_f,
                             "mismatches": len(mism_f),
                             "ok": bool(vratio_f <= 1.0 and not mism_f and nfrag_f <= 0.001 * V_fir.size)}
            fir["cpu_baseline"] = {"value": round(mpx / t_fir, 3), "unit": "Mpixel·scales/s", "cores": ncores,
                                   "kind": "oracle",
                                   "sample": "the same frame and scales through the FIR oracle (coloured SG, "
                                             "matrix form of the separable sum), one scale per worker process"}
            log(f"FIR parity {fir['parity']}")
            if V_firm is not None:
                # a-priori bound of the matrix-core route: sigma^2 (sum |h|) (sum |d|) max |x|
                # (12 2^-22 + (4 n + 2) 2^-24) plus the float32 rounding of V
                xmax = float(frame.max())
                vbm = []
                for s, sg in enumerate(sig):
                    h_s = np.asarray(taps[off[s]: off[s] + 2 * half[s] + 1], np.float64)
                    hpad = np.concatenate([[0.0, 0.0], h_s, [0.0, 0.0]])
                    d_s = hpad[:-2] - 2 * hpad[1:-1] + hpad[2:]
                    n_s = 2 * int(half[s]) + 3
                    vbm.append(sg * sg * float(np.sum(np.abs(h_s))) * float(np.sum(np.abs(d_s))) * xmax *
                               (12 * 2.0 ** -22 + (4 * n_s + 2) * 2.0 ** -24) +
                               2.0 ** -23 * float(np.max(np.abs(Vf[s]))))
                vratio_m = max(float(np.max(np.abs(V_firm[s] - Vf[s]))) / vbm[s] for s in range(S))
                nfrag_m, mism_m = compare_detections(det_firm, det_ref_f, Vf, V_firm, tau, border, v_bound=vbm)
                fir["parity_mfma"] = {"err_over_bound": round(vratio_m, 4), "detections": int(len(det_firm)),
                                      "oracle_detections": int(len(det_ref_f)), "fragile_excluded": nfrag_m,
                                      "mismatches": len(mism_m),
                                      "ok": bool(vratio_m <= 1.0 and not mism_m and
                                                 nfrag_m <= 0.001 * V_firm.size)}
                log(f"FIR matrix-core parity {fir['parity_mfma']}")
            del Bf, Vf
        if precision is not None:
            precision_errors(precision, syn, torch, np, log)

    roofline["measured_copy_GB/s"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(d["GB/s"] / copy_gbs, 4)

    out = {
        "metric": "Mpixel·scales/s, IIR vs FIR, at <=1e-5 rel err; % HBM roofline",
        "value": round(value, 1),
        "unit": "Mpixel·scales/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 recursion, f32 planes",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "H": H, "W": W, "scales": S, "sigmas": [round(s, 4) for s in sig],
                   "input": "uint16 12-bit", "iir_order": 3, "tau": tau,
                   "step": "design + iir x pass + iir y pass with fused sigma^2 Laplacian + extrema"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fir": fir,
        "batch": batch,
        "grad": grad,
        "butterworth": butterworth,
        "precision": None if precision is None else {k: v for k, v in precision.items() if not k.startswith("_")},
        "kernels": {k: {"ms": round(v["ms"], 5), "GB/s": round(v["GB/s"], 1), "launches": v["kernels"]}
                    for k, v in kern.items()},
        "detections": n_det,
        "parity": parity,
        "h2d_ms_input": round(h2d_ms, 3),
        "wall_s_timed": round(wall, 4),
    }
    if extra_copy:
        out["calibration_copy"] = extra_copy
    if pool is not None:
        pool.terminate()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
