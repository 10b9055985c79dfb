"""GPU parity of fdvm_blur_fir with FDVM_FIR_TOEPLITZ_MFMA_HALF: the separable
FIR of Eq A5 as Toeplitz-block products on the matrix cores with half-
precision operands (float16 and bfloat16 frames as stored, uint16 frames
split exactly into float16 pairs) and float32 accumulation.

Error model of one pass, relative to sum |h| * max |x| (x: the pass's input):
the taps are split hi + lo in the operand type (relative error 2^-2p, p the
type's significand bits: 11 for float16, 8 for bfloat16); the intermediate is
stored split the same way (2^-2p) and the lo x lo product is dropped (2^-2p,
2^-2p+1 for the uint16 split, whose lo part is up to one float16 ulp); the
sums are accumulated in float32 (n = 2K + 1 terms, n 2^-24 at worst).  Two
passes: err <= (sum |h|)^2 max |x| * 2 (4 2^-2p + n 2^-24).  Every pixel is
compared against the FP64 oracle on the dequantised stored frame (the uint16
frame itself) to that bound; on the original (unquantised) frame the
per-scale max and rms errors must stay within 2e-3 of max |B|."""

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering
from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")

CFG = syn.PRECISION
KS = [(m - 1) // 2 for m in CFG["fir_lengths"]]
SIGS = [k / 3 for k in KS]
P_BITS = {"f16": 11, "bf16": 8, "u16": 11}


def bound(kind, h, xmax):
    """A-priori max |error| of the two-pass half-operand FIR (module doc)."""
    n = len(h)
    a1 = float(np.sum(np.abs(h)))
    return a1 * a1 * xmax * 2.0 * (4.0 * 2.0 ** (-2 * P_BITS[kind]) + n * 2.0 ** -24)


def torch_type(kind):
    return torch.float16 if kind == "f16" else torch.bfloat16


def stored(frame64, kind):
    t = torch.from_numpy(frame64.astype(np.float32)).to(torch_type(kind))
    return t.cuda(), t.float().numpy().astype(np.float64)


_REF = {}


def references(kind):
    """Oracle planes of the 1024^2 stored (dequantised) and original frames."""
    if kind not in _REF:
        orig = syn.normalised_frame(1024, 1024, CFG["seed"], nblobs=CFG["nblobs"] // 64)
        x, deq = stored(orig, kind)
        hs = [design.colored_sg_taps(sg, K=K) for sg, K in zip(SIGS, KS)]
        _REF[kind] = (x, deq, hs, np.stack([filtering.blur_2d_matrix(deq, h) for h in hs]),
                      np.stack([filtering.blur_2d_matrix(orig, h) for h in hs]))
    return _REF[kind]


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_half_mfma_lengths_every_pixel(kind):
    """FIR lengths 33, 65, 129, 257 (sigma = K/3) on a 1024^2 stored frame."""
    say(f"case: fir mfma_half {kind} 1024x1024 lengths 33..257")
    x, deq, hs, ref_q, ref_o = references(kind)
    got = P.blur_fir(x, SIGS, kind="sg", half_lens=KS, algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
    got = got.astype(np.float64)
    xmax = float(np.max(np.abs(deq)))
    for s, K in enumerate(KS):
        dq, do = got[s] - ref_q[s], got[s] - ref_o[s]
        sq, so = float(np.max(np.abs(ref_q[s]))), float(np.max(np.abs(ref_o[s])))
        b = bound(kind, hs[s], xmax)
        say(f"   length {2 * K + 1}: vs dequantised max {np.max(np.abs(dq)) / sq:.2e} "
            f"rms {np.sqrt(np.mean(dq * dq)) / sq:.2e} (bound {b / sq:.2e}); "
            f"vs original max {np.max(np.abs(do)) / so:.2e} rms {np.sqrt(np.mean(do * do)) / so:.2e}")
        assert float(np.max(np.abs(dq))) <= b
        assert float(np.max(np.abs(do))) <= 2e-3 * so
        assert float(np.sqrt(np.mean(do * do))) <= 2e-3 * so


@pytest.mark.parametrize("shape", [(1, 1), (5, 300), (300, 5), (77, 131), (129, 65), (256, 2500)])
@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_half_mfma_ragged(shape, kind):
    H, W = shape
    say(f"case: fir mfma_half {kind} {H}x{W}")
    rng = np.random.default_rng(H + 7 * W)
    x, deq = stored(rng.random((H, W)) * 4.0, kind)
    sig = [1.2, 2.5, 11.0]
    hs = [design.colored_sg_taps(s) for s in sig]
    xmax = float(np.max(np.abs(deq)))
    for bc in ("replicate", "zero"):
        got = P.blur_fir(x, sig, kind="sg", boundary=bc, algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
        for s, h in enumerate(hs):
            ref = filtering.blur_2d(deq, h, bc)
            err = float(np.max(np.abs(got[s].astype(np.float64) - ref)))
            assert err <= bound(kind, h, xmax), f"{bc} scale {s}: {err:.3e}"


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_half_mfma_long_taps(kind):
    """Half-lengths near the 512 limit, and a tap set too long for one launch's
    table (the form then runs scale by scale)."""
    rng = np.random.default_rng(23)
    x, deq = stored(rng.random((300, 1200)) * 8.0, kind)
    xmax = float(np.max(np.abs(deq)))
    for Ks in ([510], [300, 350, 400]):
        say(f"case: fir mfma_half {kind} long taps K={Ks} 300x1200")
        sig = [K / 3 for K in Ks]
        got = P.blur_fir(x, sig, kind="sg", half_lens=Ks, algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
        for s, (sg, K) in enumerate(zip(sig, Ks)):
            h = design.colored_sg_taps(sg, K=K)
            ref = filtering.blur_2d_matrix(deq, h)
            err = float(np.max(np.abs(got[s].astype(np.float64) - ref)))
            assert err <= bound(kind, h, xmax), f"K={K}: {err:.3e}"


def test_half_mfma_gaussian_and_large_values():
    """Sampled Gaussian taps and float16 values near its largest finite
    magnitude (the first pass multiplies them unrounded; the taps are scaled to
    [0.5, 1), so no product overflows)."""
    say("case: fir mfma_half f16 gaussian, values to 6e4")
    rng = np.random.default_rng(5)
    x, deq = stored(rng.random((200, 333)) * 6.0e4, "f16")
    sig = [0.9, 4.0, 20.0]
    got = P.blur_fir(x, sig, kind="gaussian", algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
    assert np.all(np.isfinite(got))
    xmax = float(np.max(np.abs(deq)))
    for s, sg in enumerate(sig):
        h = design.gaussian_taps(sg, design.fir_half_length(sg))
        ref = filtering.blur_2d(deq, h)
        assert float(np.max(np.abs(got[s].astype(np.float64) - ref))) <= bound("f16", h, xmax)


def test_half_mfma_u16_frames():
    """uint16 frames (split exactly into float16 pairs), ragged and to 65535."""
    rng = np.random.default_rng(9)
    sig = [1.2, 5.0, 21.0]
    hs = [design.colored_sg_taps(s) for s in sig]
    for (H, W), top in (((77, 131), 4096), ((300, 517), 65536), ((1, 1), 65536)):
        say(f"case: fir mfma_half u16 {H}x{W} values < {top}")
        a = rng.integers(0, top, (H, W)).astype(np.uint16)
        a.flat[0] = top - 1
        x = torch.from_numpy(a.view(np.int16)).cuda()
        x64 = a.astype(np.float64)
        got = P.blur_fir(x, sig, kind="sg", algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
        assert np.all(np.isfinite(got))
        for s, h in enumerate(hs):
            err = float(np.max(np.abs(got[s].astype(np.float64) - filtering.blur_2d(x64, h))))
            assert err <= bound("u16", h, float(np.max(x64))), f"scale {s}: {err:.3e}"


def test_half_mfma_full_frame_u16_every_pixel():
    """The 2048^2 uint16 frame with the 8 scales of 2..64 (coloured SG,
    K = ceil(3 sigma)): every pixel within the bound; normwise max printed."""
    cfg = syn.FULL_FRAME
    say("case: fir mfma_half u16 full frame 2048x2048 8 scales (every pixel)")
    frame = syn.aerial_frame(cfg["H"], cfg["W"], cfg["seed"])
    f64 = frame.astype(np.float64)
    got = P.blur_fir(torch.from_numpy(frame.view(np.int16)).cuda(), cfg["sigmas"], kind="sg",
                     algo=P.FIR_TOEPLITZ_MFMA_HALF).cpu().numpy()
    xmax = float(np.max(f64))
    for s, sg in enumerate(cfg["sigmas"]):
        h = design.colored_sg_taps(sg)
        ref = filtering.blur_2d_matrix(f64, h)
        d = got[s].astype(np.float64) - ref
        sc = float(np.max(np.abs(ref)))
        say(f"   scale {s}: max {np.max(np.abs(d)) / sc:.2e} rms {np.sqrt(np.mean(d * d)) / sc:.2e} "
            f"(bound {bound('u16', h, xmax) / sc:.2e})")
        assert float(np.max(np.abs(d))) <= bound("u16", h, xmax)


def test_half_mfma_unaligned_views():
    """Frames whose rows do not start 16-byte aligned take the element-wise
    load path; output planes with an odd pitch take element-wise stores."""
    say("case: fir mfma_half f16 unaligned input view and odd output pitch")
    rng = np.random.default_rng(31)
    big = torch.from_numpy(rng.random((130, 403)).astype(np.float32)).to(torch.float16).cuda()
    x = big[1:, 3:]   # pitch 403, offset 406 elements
    deq = x.float().cpu().numpy().astype(np.float64)
    sig = [2.0, 9.0]
    out = torch.empty((2, 129, 401), dtype=torch.float32, device="cuda")
    out_view = out[:, :, :400]
    got = P.blur_fir(x, sig, kind="sg", algo=P.FIR_TOEPLITZ_MFMA_HALF, out=out_view).cpu().numpy()
    for s, sg in enumerate(sig):
        h = design.colored_sg_taps(sg)
        err = float(np.max(np.abs(got[s].astype(np.float64) - filtering.blur_2d(deq, h))))
        assert err <= bound("f16", h, float(np.max(deq)))


def test_half_mfma_rejects_float32():
    say("case: fir mfma_half rejects f32")
    with pytest.raises(P.FdvmError):
        P.blur_fir(torch.zeros((8, 8), device="cuda"), [2.0], algo=P.FIR_TOEPLITZ_MFMA_HALF)
