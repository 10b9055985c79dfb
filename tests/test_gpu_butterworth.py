"""GPU parity of the Butterworth blur (Filter E, Section 4.4: L_B = 4, one
complex-conjugate pole pair per direction) against the FP64 oracle, whose
design is the Eq A17 decomposition of the bilinear prototype and whose
filtering is the three-term DE of Eqs A6-A10 with the Eq A32 steady-state
start.  The scale is tuned by omega_c = sqrt(2 ln 2) / sigma.

* blur planes: normwise per plane within 1e-5 (ragged shapes, both
  boundaries, u16 and f32 input, wide rows that take several wavefronts);
* fused normalised Laplacian: within the float32 Laplacian tolerance;
* detections on an aerial frame: equal to the oracle's outside the fragile
  set (the rule of parity.py);
* the Hessian detector on the ellipse test pattern of Section 5: one
  detection per ellipse whose semi-major axis equals lambda = 2 sigma, at its
  centre (Threshold #1 = 0.06, Threshold #2 = 0.6)."""

import math

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering, shape
from parity import assert_planes_close, compare_detections, laplacian_tolerance, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")

BW = "butterworth"


def coef(sigma):
    return design.butterworth(4, math.sqrt(2.0 * math.log(2.0)) / sigma)


def oracle_bank(x64, sigmas, boundary="replicate"):
    return filtering.blur_bank(x64, [coef(s) for s in sigmas], boundary)


@pytest.mark.parametrize("shape_", [(1, 1), (1, 300), (300, 1), (37, 53), (64, 64), (129, 1000), (70, 2100),
                                    (9, 4100), (520, 17)])
def test_blur_ragged_shapes(shape_):
    H, W = shape_
    say(f"case: butterworth blur {H}x{W}")
    rng = np.random.default_rng(H * 31 + W)
    img = (rng.random((H, W)) * 100 + np.linspace(0, 50, W)[None, :]).astype(np.float32)
    sigmas = [0.6, 3.0, 40.0]
    x = torch.from_numpy(img).cuda()
    for bc in ("replicate", "zero"):
        got = P.blur_iir(x, sigmas, order=BW, boundary=bc).cpu().numpy()
        assert_planes_close(got, oracle_bank(img.astype(np.float64), sigmas, bc))


def test_blur_u16_frame_and_pass_api():
    """u16 input through the fixed-point intermediate, and the one-pass API
    (float32 planes between the passes) against the same oracle."""
    say("case: butterworth u16 600x700 and pass API")
    frame = syn.aerial_frame(600, 700, 11, nblobs=12)
    x = torch.from_numpy(frame.view(np.int16)).cuda()
    sigmas = [1.0, 4.0, 16.0, 64.0]
    ref = oracle_bank(frame.astype(np.float64), sigmas)
    assert_planes_close(P.blur_iir(x, sigmas, order=BW).cpu().numpy(), ref)
    R = P.iir_pass(x, sigmas, 0, order=BW)
    B = P.iir_pass(R, sigmas, 1, order=BW, out=R)
    assert_planes_close(B.cpu().numpy(), ref)


def test_fused_laplacian_and_detection():
    """1024 x 1024 u16 aerial frame, 6 scales: the fused Laplacian within the
    float32 Laplacian tolerance and the detections equal to the oracle's
    outside the fragile set."""
    say("case: butterworth fused laplacian + detection 1024x1024")
    frame = syn.aerial_frame(1024, 1024, 5, nblobs=60)
    sigmas = syn.geometric_scales(2.0, 32.0, 6)
    tau = 40.0
    f64 = frame.astype(np.float64)
    B_ref = oracle_bank(f64, sigmas)
    V_ref = shape.laplacian_bank(B_ref, sigmas)
    det_ref = shape.detect_extrema(V_ref, tau, 1)
    x = torch.from_numpy(frame.view(np.int16)).cuda()
    V = P.iir_laplacian(x, sigmas, order=BW)
    Vn = V.cpu().numpy()
    for s, sg in enumerate(sigmas):
        err = float(np.max(np.abs(Vn[s] - V_ref[s])))
        assert err <= laplacian_tolerance(sg, B_ref[s]), (s, err)
    det = P.detect_blobs(V, tau, 1)
    vb = [laplacian_tolerance(sg, B_ref[s]) for s, sg in enumerate(sigmas)]
    nfrag, mism = compare_detections(det, det_ref, V_ref, Vn, tau, 1, v_bound=vb)
    say(f"   detections gpu={len(det)} ref={len(det_ref)} fragile={nfrag}")
    assert mism == []
    assert len(det_ref) > 10
    assert nfrag <= 0.001 * Vn.size


def test_hessian_ellipse_pattern():
    say("case: butterworth hessian ellipse pattern")
    img, items = syn.ellipse_pattern(2.0)
    sig = [lam / 2 for lam in syn.ELLIPSE_AXES]
    x = torch.from_numpy(img.astype(np.float32)).cuda()
    det, nd = P.iir_hessian(x, sig, 0.06, 0.6, 1, order=BW)
    got = sorted((int(d["scale"]), int(d["y"]), int(d["x"]), int(d["polarity"])) for d in det)
    exp = sorted((s, int(cy), int(cx), -1) for s, lam in enumerate(syn.ELLIPSE_AXES)
                 for (cy, cx, a, b, ang) in items if a == lam)
    assert got == exp
    B = oracle_bank(img.astype(np.float32).astype(np.float64), sig)
    ndn = nd.cpu().numpy().astype(np.float64)
    for s, sg in enumerate(sig):
        ref = shape.detect_hessian(B[s], sg, 0.0, None, 1)[1]
        assert float(np.max(np.abs(ndn[s] - ref))) <= 1e-4 * float(np.max(np.abs(ref))) + 1e-6, s


def test_batch_matches_single_frame_path():
    say("case: butterworth batch")
    frames = [torch.from_numpy(syn.aerial_frame(H, W, 70 + i, nblobs=5).view(np.int16)).cuda()
              for i, (H, W) in enumerate([(300, 400), (129, 2100), (512, 512)])]
    sig = [1.5, 4.0, 12.0]
    b = P.Batch(frames, sig, 40.0, order=BW, nlanes=2)
    b.run()
    got = b.results()
    for f, g in zip(frames, got):
        ref = P.detect_blobs(P.iir_laplacian(f, sig, order=BW), 40.0, 1)
        assert np.array_equal(g, ref)
