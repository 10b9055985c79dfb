"""GPU parity of fdvm_fir_laplacian (the FIR blur of Eq A5 fused with the
normalised Laplacian sigma^2 (D20 + D02) of Table I's d = 2 taps) against the
FP64 oracle: blur_2d with the oracle's taps, then its Laplacian, then its
multi-scale extrema.

V is compared element by element within the float32 Laplacian tolerance of
tests/parity.py; detections equal the oracle's outside the fragile set, which
must stay below 0.1 % of the pixels on the 2048 x 2048 x 8-scale frame (the
same bound as the IIR's fused route)."""

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering, shape
from parity import compare_detections, keys_equal_ok, laplacian_tolerance, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")


def oracle_v(img64, sigmas, kind="sg", Ks=None, boundary="replicate"):
    Ks = Ks or [None] * len(sigmas)
    if kind == "sg":
        taps = [design.colored_sg_taps(s, K=K) for s, K in zip(sigmas, Ks)]
    else:
        taps = [design.gaussian_taps(s, K if K else design.fir_half_length(s)) for s, K in zip(sigmas, Ks)]
    B = np.stack([filtering.blur_2d_matrix(img64, h, boundary) for h in taps])
    return B, shape.laplacian_bank(B, sigmas)


def check_v(V, B_ref, V_ref, sigmas, what):
    worst = 0.0
    for s, sg in enumerate(sigmas):
        err = float(np.max(np.abs(V[s].astype(np.float64) - V_ref[s])))
        tol = laplacian_tolerance(sg, B_ref[s])
        worst = max(worst, err / tol)
        assert err <= tol, (what, s, err, tol)
    say(f"   {what}: max |dV| / tolerance = {worst:.2e}")
    return worst


@pytest.mark.parametrize("shape_hw", [(1, 1), (2, 7), (5, 300), (77, 131), (129, 65), (300, 1200)])
@pytest.mark.parametrize("kind", ["sg", "gaussian"])
def test_ragged_shapes_both_extensions(shape_hw, kind):
    H, W = shape_hw
    rng = np.random.default_rng(H * 7 + W)
    img = (rng.random((H, W)) * 100).astype(np.float32)
    sig = [1.2, 3.0, 11.0] if kind == "sg" else [0.8, 3.0, 11.0]
    for bc in ("replicate", "zero"):
        say(f"case: fir laplacian {kind} {bc} {H}x{W}")
        V = P.fir_laplacian(torch.from_numpy(img).cuda(), sig, kind=kind, boundary=bc).cpu().numpy()
        B_ref, V_ref = oracle_v(img.astype(np.float64), sig, kind, boundary=bc)
        check_v(V, B_ref, V_ref, sig, f"{kind} {bc} {H}x{W}")


@pytest.mark.parametrize("dtype", ["u16", "f16", "bf16"])
def test_input_types(dtype):
    say(f"case: fir laplacian input {dtype}")
    a = syn.aerial_frame(200, 333, 17, nblobs=6)
    if dtype == "u16":
        x = torch.from_numpy(a.view(np.int16)).cuda()
        x64 = a.astype(np.float64)
    else:
        t = torch.from_numpy(a.astype(np.float32) / 4095).to(torch.float16 if dtype == "f16" else torch.bfloat16)
        x, x64 = t.cuda(), t.float().numpy().astype(np.float64)
    sig = [2.0, 5.0, 9.0]
    V = P.fir_laplacian(x, sig).cpu().numpy()
    B_ref, V_ref = oracle_v(x64, sig)
    check_v(V, B_ref, V_ref, sig, dtype)


def test_long_taps():
    say("case: fir laplacian K = 510 and 300..400")
    rng = np.random.default_rng(5)
    img = (rng.random((260, 1100)) * 50).astype(np.float32)
    for Ks in ([510], [300, 350, 400]):
        sig = [K / 3 for K in Ks]
        V = P.fir_laplacian(torch.from_numpy(img).cuda(), sig, half_lens=Ks).cpu().numpy()
        B_ref, V_ref = oracle_v(img.astype(np.float64), sig, Ks=Ks)
        check_v(V, B_ref, V_ref, sig, f"K={Ks}")


def test_tiny_frames_exact_detections():
    """The tiny configuration's frame (and its noise-free variant) through
    the FIR form: the oracle's blob list exactly."""
    for noise in (True, False):
        say(f"case: fir laplacian tiny noise={noise}")
        img = syn.tiny_frame(0, noise=noise)
        sig, tau = [2.0, 4.0, 6.0], 0.3
        V = P.fir_laplacian(torch.from_numpy(img).cuda(), sig)
        det = P.detect_blobs(V, tau, 1)
        B_ref, V_ref = oracle_v(img.astype(np.float64), sig)
        det_ref = shape.detect_extrema(V_ref, tau, 1)
        nfrag, mism = compare_detections(det, det_ref, V_ref, V.cpu().numpy(), tau)
        say(f"   detections gpu={len(det)} ref={len(det_ref)} fragile={nfrag}")
        assert mism == []
        assert keys_equal_ok(det, det_ref)
        assert len(det_ref) > 0


def test_full_frame_detections_match_oracle():
    """2048 x 2048 u16, 8 scales sigma = 2..64, coloured SG with K = ceil(3 sigma):
    V within tolerance everywhere; detections equal to the oracle's outside a
    fragile set of at most 0.1 % of the pixels, counts within 0.5 %."""
    cfg = syn.FULL_FRAME
    say("case: fir laplacian full frame 2048x2048 u16 8 scales")
    frame = syn.aerial_frame(cfg["H"], cfg["W"], cfg["seed"])
    x = torch.from_numpy(frame.view(np.int16)).cuda()
    V = P.fir_laplacian(x, cfg["sigmas"])
    det = P.detect_blobs(V, cfg["tau"], cfg["border"])
    Vn = V.cpu().numpy()
    del V
    B_ref, V_ref = oracle_v(frame.astype(np.float64), cfg["sigmas"])
    check_v(Vn, B_ref, V_ref, cfg["sigmas"], "full frame")
    det_ref = shape.detect_extrema(V_ref, cfg["tau"], cfg["border"])
    vb = [laplacian_tolerance(sg, B_ref[s]) for s, sg in enumerate(cfg["sigmas"])]
    nfrag, mism = compare_detections(det, det_ref, V_ref, Vn, cfg["tau"], cfg["border"], v_bound=vb)
    say(f"   detections gpu={len(det)} ref={len(det_ref)} fragile={nfrag} ({nfrag / Vn.size:.2e} of the pixels)")
    assert mism == []
    assert nfrag <= 0.001 * Vn.size
    assert abs(len(det) - len(det_ref)) <= 0.005 * len(det_ref)
    assert len(det_ref) > 10
