"""End-to-end GPU parity: blur -> normalised Laplacian -> multi-scale extrema,
against the FP64 oracle run from the same input.

The GPU computes in float32, the oracle in float64, so a few decisions sit
within rounding of a tie or of the threshold.  Those "fragile" decisions are
excluded by the rule in tests/parity.py (an error of at most the measured
per-plane |dV| cannot flip any other decision); everything else must match
exactly.  The noise-free tiny frame must match with no exclusion at all."""

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering, shape
from parity import RTOL_BLUR, assert_planes_close, compare_detections, keys_equal_ok, laplacian_tolerance, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")


def run_oracle(img64, sigmas, order, tau, border=1, fir=None):
    if fir is None:
        filt = [design.repeated_pole(order, s) for s in sigmas]
    else:
        filt = [design.colored_sg_taps(s) for s in sigmas]
    B = filtering.blur_bank(img64, filt)
    V = shape.laplacian_bank(B, sigmas)
    return B, V, shape.detect_extrema(V, tau, border)


def test_tiny_config_end_to_end():
    cfg = syn.TINY
    say("case: tiny end-to-end")
    img = syn.tiny_frame(cfg["seed"])
    B_ref, V_ref, det_ref = run_oracle(img.astype(np.float64), cfg["sigmas"], cfg["iir_order"], cfg["tau"])
    det, V = P.detect(torch.from_numpy(img).cuda(), cfg["sigmas"], cfg["tau"], order=cfg["iir_order"])
    V = V.cpu().numpy()
    nfrag, mism = compare_detections(det, det_ref, V_ref, V, cfg["tau"])
    say(f"   detections gpu={len(det)} ref={len(det_ref)} fragile={nfrag}")
    assert mism == []
    assert len(det_ref) > 0
    # the tiny configuration: blob positions and scales exactly the oracle's
    assert keys_equal_ok(det, det_ref)


def test_tiny_noise_free_exact():
    say("case: tiny noise-free exact")
    img = syn.tiny_frame(0, noise=False)
    tau = 0.3
    _, V_ref, det_ref = run_oracle(img.astype(np.float64), [4.0], 2, tau)
    det, _ = P.detect(torch.from_numpy(img).cuda(), [4.0], tau, order=2)
    assert keys_equal_ok(det, det_ref)
    assert len(det_ref) >= 1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tiny_seeds_multi_scale(seed):
    say(f"case: tiny multi-scale seed {seed}")
    img = syn.tiny_frame(seed)
    sig = [2.0, 3.0, 4.5, 6.5]
    _, V_ref, det_ref = run_oracle(img.astype(np.float64), sig, 3, 0.3)
    det, V = P.detect(torch.from_numpy(img).cuda(), sig, 0.3, order=3)
    nfrag, mism = compare_detections(det, det_ref, V_ref, V.cpu().numpy(), 0.3)
    say(f"   detections gpu={len(det)} ref={len(det_ref)} fragile={nfrag}")
    assert mism == []
    assert keys_equal_ok(det, det_ref)


# Bounds per route on the 2048 x 2048 frame (8 scales, sigma up to 64):
#   fused     -- V formed in float64 from the unrounded blur; the only rounding
#                that reaches it is the fixed-point x-pass intermediate;
#                Measured: max|dV| 0.015 (sigma = 64), 0.014% of the pixels
#                fragile, 3587 detections against 3581.
#   two-step  -- V from float32 blur planes: their rounding is white in x and y
#                and the normalised Laplacian multiplies it by ~8 sigma^2
#                (max|dV| ~2 at sigma = 64), so near-flat plateaus of V at the
#                coarsest scales break up into many spurious extrema (measured
#                6.4% of the pixels fragile, 18480 detections against 3581).
#                Only "no difference outside the fragile set" is asserted.
ROUTE_BOUNDS = {"fused": (0.001, 0.005), "two-step": (0.10, None)}   # fragile fraction, |count| rel. diff


def test_full_frame_end_to_end():
    """2048x2048 uint16, 8 scales, order 3: blur planes everywhere within
    1e-5, and the detection lists of both GPU routes (fused blur + Laplacian,
    and blur then high-pass) equal the oracle's outside the fragile set, which
    must stay a small fraction of the pixels."""
    cfg = syn.FULL_FRAME
    say("case: full frame end-to-end")
    frame = syn.aerial_frame(cfg["H"], cfg["W"], cfg["seed"])
    f64 = frame.astype(np.float64)
    B_ref, V_ref, det_ref = run_oracle(f64, cfg["sigmas"], 3, cfg["tau"])
    x = torch.from_numpy(frame.view(np.int16)).cuda()
    B = P.blur_iir(x, cfg["sigmas"], order=3)
    assert_planes_close(B.cpu().numpy(), B_ref)
    routes = {"fused": P.iir_laplacian(x, cfg["sigmas"], order=3), "two-step": P.highpass(B, cfg["sigmas"])}
    stats = {}
    for name, V in routes.items():
        det = P.detect_blobs(V, cfg["tau"], cfg["border"])
        Vn = V.cpu().numpy()
        dv = max(float(np.max(np.abs(Vn[s] - V_ref[s]))) for s in range(len(cfg["sigmas"])))
        vb = [laplacian_tolerance(sg, B_ref[s]) for s, sg in enumerate(cfg["sigmas"])]
        nfrag, mism = compare_detections(det, det_ref, V_ref, Vn, cfg["tau"], cfg["border"], v_bound=vb)
        stats[name] = (nfrag / Vn.size, abs(len(det) - len(det_ref)) / len(det_ref), mism)
        say(f"   {name}: detections gpu={len(det)} ref={len(det_ref)} fragile={nfrag} max|dV|={dv:.3g}")
    for name, (ffrac, dcount, mism) in stats.items():
        fb, cb = ROUTE_BOUNDS[name]
        assert mism == [], name
        assert ffrac <= fb, (name, ffrac)
        if cb is not None:
            assert dcount <= cb, (name, dcount)
    assert len(det_ref) > 10
