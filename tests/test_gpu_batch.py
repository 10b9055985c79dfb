"""GPU checks of fdvm_batch_detect (many uneven frames in one call).

* Every frame's list equals the single-frame path (fdvm_iir_laplacian +
  fdvm_detect_blobs) exactly: the same kernels on the same data.
* Lane counts 1 .. 8 give identical results.
* Row-pass chunk overrides change only the float64 rounding of the recursion
  (positions, scales and polarities equal; values within 1e-5 relative).
* Frames against the FP64 oracle (fragile-decision rule of parity.py): one
  small frame, and one frame of every size of the 64-frame workload.
* The batch captured into a graph and replayed several times, with eager work
  between the replays, reproduces the eager results each time."""

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering, shape
from parity import compare_detections, laplacian_tolerance, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")

SIG = [1.5, 3.0, 6.5, 14.0]
TAU = 30.0


def make_frames():
    """Uneven frames of all input types, 12-bit aerial-like content."""
    specs = [(257, 300, "u16"), (512, 512, "u16"), (100, 1000, "f32"), (64, 64, "u16"), (333, 129, "bf16"),
             (40, 2100, "f16")]
    out = []
    for i, (H, W, dt) in enumerate(specs):
        a = syn.aerial_frame(H, W, 50 + i, nblobs=max(3, H * W // 20000))
        if dt == "u16":
            t = torch.from_numpy(a.view(np.int16)).cuda()
        elif dt == "f32":
            t = torch.from_numpy(a.astype(np.float32)).cuda()
        elif dt == "bf16":
            t = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).cuda()
        else:
            t = torch.from_numpy(a.astype(np.float32) / 4095).to(torch.float16).cuda()
        out.append(t)
    return out


def single(frame, tau):
    V = P.iir_laplacian(frame, SIG, order=3)
    return P.detect_blobs(V, tau, 1)


def tau_for(frame):
    return TAU / 4095 if frame.dtype == torch.float16 else TAU


def keys(det):
    return [(int(d["scale"]), int(d["y"]), int(d["x"]), int(d["polarity"])) for d in det]


def run_batch(frames, nlanes, row_chunks=None):
    # one tau for all frames of a batch: keep the f16 frame in its own batch
    b = P.Batch(frames, SIG, TAU, nlanes=nlanes, row_chunks=row_chunks)
    b.run()
    return b.results()


def test_batch_equals_single_frame_path_all_lane_counts():
    frames = [f for f in make_frames() if f.dtype != torch.float16]
    ref = [single(f, TAU) for f in frames]
    assert sum(len(r) for r in ref) > 10
    for nl in (1, 2, 3, 8):
        say(f"case: batch of {len(frames)} uneven frames, {nl} lanes")
        got = run_batch(frames, nl)
        for i, (g, r) in enumerate(zip(got, ref)):
            assert len(g) == len(r), (nl, i)
            assert np.array_equal(g, r), (nl, i)


def test_batch_f16_frame_and_threshold():
    frames = [f for f in make_frames() if f.dtype == torch.float16]
    b = P.Batch(frames, SIG, TAU / 4095, nlanes=2)
    b.run()
    got = b.results()
    assert np.array_equal(got[0], single(frames[0], TAU / 4095))


def test_row_chunk_overrides():
    frames = [f for f in make_frames() if f.dtype != torch.float16]
    base = run_batch(frames, 2)
    for c in (8, 16, 32):
        chunks = [c if c in P.row_chunk_choices(int(f.shape[1])) else 0 for f in frames]
        say(f"case: row chunk {c} -> {chunks}")
        got = run_batch(frames, 2, chunks)
        for g, r in zip(got, base):
            assert keys(g) == keys(r)
            np.testing.assert_allclose(g["value"], r["value"], rtol=1e-5, atol=1e-6)


def test_batch_frame_against_oracle():
    say("case: batch frame vs FP64 oracle")
    frames = make_frames()[:2]
    got = run_batch(frames, 2)
    a = frames[0].cpu().numpy().view(np.uint16).astype(np.float64)
    B = filtering.blur_bank(a, [design.repeated_pole(3, s) for s in SIG])
    V_ref = shape.laplacian_bank(B, SIG)
    det_ref = shape.detect_extrema(V_ref, TAU, 1)
    V_gpu = P.iir_laplacian(frames[0], SIG).cpu().numpy()
    nfrag, mism = compare_detections(got[0], det_ref, V_ref, V_gpu, TAU)
    say(f"   detections gpu={len(got[0])} ref={len(det_ref)} fragile={nfrag}")
    assert mism == []
    assert len(det_ref) > 0


def _oracle_check(frame_u16, sig, det_gpu, V_gpu, tau, what):
    a = frame_u16.astype(np.float64)
    B = filtering.blur_bank(a, [design.repeated_pole(3, s) for s in sig])
    V_ref = shape.laplacian_bank(B, sig)
    det_ref = shape.detect_extrema(V_ref, tau, 1)
    vb = [laplacian_tolerance(sg, B[s]) for s, sg in enumerate(sig)]
    nfrag, mism = compare_detections(det_gpu, det_ref, V_ref, V_gpu, tau, 1, v_bound=vb)
    say(f"   {what}: detections gpu={len(det_gpu)} ref={len(det_ref)} fragile={nfrag}")
    assert mism == [], what
    assert len(det_ref) > 0
    assert nfrag <= 0.001 * V_gpu.size, what


def test_batch_workload_sizes_against_oracle():
    """One frame of every size of the 64-frame workload (512 x 512,
    1080 x 1920, 2048 x 2048 with its 12 scales; 3072 x 4096 with 4 of them),
    through the batch call, against the FP64 oracle."""
    cfg = syn.BATCH
    specs = {}
    for (H, W, seed) in syn.batch_frames():
        specs.setdefault((H, W), seed)
    small = [(512, 512), (1080, 1920), (2048, 2048)]
    runs = [(small, cfg["sigmas"]), ([(3072, 4096)], [cfg["sigmas"][i] for i in (0, 4, 8, 11)])]
    for sizes, sig in runs:
        arrays = [syn.aerial_frame(H, W, specs[(H, W)], nblobs=int(round(200 * H * W / 2048 ** 2)))
                  for (H, W) in sizes]
        frames = [torch.from_numpy(a.view(np.int16)).cuda() for a in arrays]
        say(f"case: batch workload sizes {sizes}, {len(sig)} scales")
        b = P.Batch(frames, sig, cfg["tau"], nlanes=2)
        b.run()
        got = b.results()
        for a, f, g, (H, W) in zip(arrays, frames, got, sizes):
            V_gpu = P.iir_laplacian(f, sig).cpu().numpy()
            _oracle_check(a, sig, g, V_gpu, cfg["tau"], f"{H}x{W}")
            del V_gpu


def test_batch_graph_replays():
    frames = [f for f in make_frames() if f.dtype != torch.float16]
    b = P.Batch(frames, SIG, TAU, nlanes=3)
    b.run()
    eager = b.results()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()            # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        say(f"case: graph replay {rep}")
        b.counts.fill_(-1)          # eager work between replays
        _ = single(frames[1], TAU)
        g.replay()
        torch.cuda.synchronize()
        got = b.results()
        for x, y in zip(got, eager):
            assert np.array_equal(x, y), rep


def test_autotune_returns_a_valid_configuration():
    frames = [f for f in make_frames() if f.dtype != torch.float16][:3]
    nl, chunks, timings = P.autotune_batch(frames, SIG, TAU, lanes=(1, 2), reps=1)
    assert nl in (1, 2)
    for f, c in zip(frames, chunks):
        assert c == 0 or c in P.row_chunk_choices(int(f.shape[1]))
    assert all(t > 0 for t in timings.values())
