"""GPU parity of fdvm_fir_laplacian_mfma: the FIR detection response
sigma^2 (D20 + D02) of the Eq A5 blur (Table I's d = 2 differences, replicate
clamp of the blur at the image edge) on the matrix cores, formed as the
two-stage band-pass of Section 5, sigma^2 (h_y (d_x x) + d_y (h_x x)) with
d = h * [1, -2, 1], with half-precision operand pairs and float32 sums, the
edge rows and columns corrected in float64.

Error model (module doc of test_gpu_fir_half.py for one pass): per product
the taps and samples split into pairs (2^-2p each, p = 11 for float16
operands -- float16 and uint16 frames -- and 8 for bfloat16), the stored
intermediate (2^-2p) and float32 sums of n = 2K + 3 terms; the two products
of V and the float32 partial response between them:
    |V - V_fp64| <= sigma^2 (sum |h|) (sum |d|) max |x| (12 2^-2p + (4 n + 2) 2^-24)
plus the float32 rounding of V.  Every pixel is held to it against the FP64
oracle on the frame as stored; on the full 2048^2 x 8-scale frame the
detections must equal the oracle's outside a fragile set of at most 0.1 % of
the pixels (counts within 0.5 %), as for the float64 route."""

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering, shape
from parity import compare_detections, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")

P_BITS = {"f16": 11, "bf16": 8, "u16": 11}


def oracle_taps(kind, sigma, K):
    return design.colored_sg_taps(sigma, K=K) if kind == "sg" else design.gaussian_taps(sigma, K)


def half_length(sigma):
    return int(np.ceil(3 * sigma - 1e-9))


def bound(h, sigma, xmax, kind):
    """A-priori max |V - V_fp64| (module doc)."""
    hp = np.concatenate([[0.0], h, [0.0]])
    d = hp[:-2] - 2 * hp[1:-1] + hp[2:]
    d = np.concatenate([[hp[1]], d, [hp[-2]]])   # d(-(K+1)) .. d(K+1)
    n = len(h) + 2
    return sigma * sigma * float(np.sum(np.abs(h))) * float(np.sum(np.abs(d))) * xmax * (
        12.0 * 2.0 ** (-2 * P_BITS[kind]) + (4 * n + 2) * 2.0 ** -24)


def stored(kind, H, W, seed, top=4.0):
    """A frame in the kind's storage type and its dequantised float64 copy."""
    rng = np.random.default_rng(seed)
    if kind == "u16":
        a = rng.integers(0, 4096, (H, W)).astype(np.uint16)
        return torch.from_numpy(a.view(np.int16)).cuda(), a.astype(np.float64)
    t = torch.from_numpy((rng.random((H, W)) * top).astype(np.float32))
    t = t.to(torch.float16 if kind == "f16" else torch.bfloat16)
    return t.cuda(), t.float().numpy().astype(np.float64)


def check(V, x64, sigmas, Ks, kind, taps_kind, bc, what):
    worst = 0.0
    xmax = float(np.max(np.abs(x64))) if x64.size else 0.0
    for s, (sg, K) in enumerate(zip(sigmas, Ks)):
        h = oracle_taps(taps_kind, sg, K)
        ref = shape.laplacian(filtering.blur_2d_matrix(x64, h, bc), sg)
        err = float(np.max(np.abs(V[s].astype(np.float64) - ref)))
        b = bound(h, sg, xmax, kind) + 2.0 ** -23 * float(np.max(np.abs(ref)))
        worst = max(worst, err / b)
        assert err <= b, (what, s, err, b)
    say(f"   {what}: max |dV| / bound = {worst:.2e}")


@pytest.mark.parametrize("shape_hw", [(1, 1), (1, 40), (33, 1), (2, 7), (5, 300), (300, 5), (77, 131), (129, 65),
                                      (20, 600)])
@pytest.mark.parametrize("kind", ["f16", "bf16", "u16"])
def test_ragged_shapes_both_extensions(shape_hw, kind):
    """Single rows and columns, ragged tiles, taps longer than the frame
    (K = 33 against 20 rows): the edge corrections on every side."""
    H, W = shape_hw
    x, x64 = stored(kind, H, W, H * 7 + W)
    sig = [1.2, 3.0, 11.0]
    Ks = [half_length(s) for s in sig]
    for bc in ("replicate", "zero"):
        say(f"case: fir laplacian mfma {kind} {bc} {H}x{W}")
        V = P.fir_laplacian(x, sig, half_lens=Ks, boundary=bc, algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
        check(V, x64, sig, Ks, kind, "sg", bc, f"{kind} {bc} {H}x{W}")


def test_gaussian_taps():
    say("case: fir laplacian mfma f16 gaussian")
    x, x64 = stored("f16", 150, 260, 3)
    sig = [0.8, 2.5, 9.0]
    Ks = [design.fir_half_length(s) for s in sig]
    V = P.fir_laplacian(x, sig, kind="gaussian", half_lens=Ks, algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
    check(V, x64, sig, Ks, "f16", "gaussian", "replicate", "gaussian")


def test_long_taps_and_several_launches():
    """The largest half-length, tap sets that need several table-builder
    launches, and more scales than one launch takes."""
    x, x64 = stored("f16", 300, 1100, 11)
    for Ks in ([511], [200, 210, 220, 400], [4, 5, 6, 7, 8, 9, 10, 11, 12, 13]):
        say(f"case: fir laplacian mfma f16 K={Ks}")
        sig = [K / 3 for K in Ks]
        V = P.fir_laplacian(x, sig, half_lens=Ks, algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
        check(V, x64, sig, Ks, "f16", "sg", "replicate", f"K={Ks}")


def test_matches_float64_route():
    """Against fdvm_fir_laplacian (float64 passes) on the same stored frame."""
    say("case: fir laplacian mfma vs float64 route, u16 400x700")
    x, x64 = stored("u16", 400, 700, 21)
    sig = [2.0, 5.4, 14.5, 39.0]
    Ks = [half_length(s) for s in sig]
    Vm = P.fir_laplacian(x, sig, half_lens=Ks, algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy().astype(np.float64)
    Vd = P.fir_laplacian(x, sig, half_lens=Ks).cpu().numpy().astype(np.float64)
    xmax = float(np.max(x64))
    for s, (sg, K) in enumerate(zip(sig, Ks)):
        h = oracle_taps("sg", sg, K)
        b = bound(h, sg, xmax, "u16") + 2.0 ** -22 * float(np.max(np.abs(Vd[s])))
        assert float(np.max(np.abs(Vm[s] - Vd[s]))) <= b, s


def test_full_frame_detections_match_oracle():
    """2048 x 2048 u16, 8 scales sigma = 2..64, coloured SG with K = ceil(3 sigma):
    V within the bound everywhere; detections equal to the oracle's outside a
    fragile set of at most 0.1 % of the pixels, counts within 0.5 %."""
    cfg = syn.FULL_FRAME
    say("case: fir laplacian mfma full frame 2048x2048 u16 8 scales")
    frame = syn.aerial_frame(cfg["H"], cfg["W"], cfg["seed"])
    x = torch.from_numpy(frame.view(np.int16)).cuda()
    sig = cfg["sigmas"]
    Ks = [half_length(s) for s in sig]
    V = P.fir_laplacian(x, sig, half_lens=Ks, algo=P.FIR_TOEPLITZ_MFMA_HALF)
    det = P.detect_blobs(V, cfg["tau"], cfg["border"])
    Vn = V.cpu().numpy()
    del V
    f64 = frame.astype(np.float64)
    xmax = float(np.max(f64))
    V_ref = np.stack([shape.laplacian(filtering.blur_2d_matrix(f64, oracle_taps("sg", sg, K)), sg)
                      for sg, K in zip(sig, Ks)])
    vb = []
    for s, (sg, K) in enumerate(zip(sig, Ks)):
        b = bound(oracle_taps("sg", sg, K), sg, xmax, "u16") + 2.0 ** -23 * float(np.max(np.abs(V_ref[s])))
        d = Vn[s].astype(np.float64) - V_ref[s]
        say(f"   scale {s}: max |dV| {np.max(np.abs(d)):.3e} rms {np.sqrt(np.mean(d * d)):.3e} (bound {b:.3e})")
        vb.append(b)
    det_ref = shape.detect_extrema(V_ref, cfg["tau"], cfg["border"])
    nfrag, mism = compare_detections(det, det_ref, V_ref, Vn, cfg["tau"], cfg["border"], v_bound=vb)
    say(f"   detections gpu={len(det)} ref={len(det_ref)} fragile={nfrag} ({nfrag / Vn.size:.2e} of the pixels)")
    assert mism == []
    assert nfrag <= 0.001 * Vn.size
    assert abs(len(det) - len(det_ref)) <= 0.005 * len(det_ref)
    assert len(det_ref) > 10


def test_rejects_float32():
    say("case: fir laplacian mfma rejects f32")
    with pytest.raises(P.FdvmError):
        P.fir_laplacian(torch.zeros((8, 8), device="cuda"), [2.0], algo=P.FIR_TOEPLITZ_MFMA_HALF)
