"""GPU parity of fdvm_blur_fir (Eq A5, separable) against the oracle, for both
algorithms: direct LDS-staged convolution and the Toeplitz-block products on
the matrix cores (float32 operands and accumulation).

Every output pixel is compared, also on the 2048x2048 x 8-scale frame (the
benchmark's FIR configuration, coloured SG of length 6 sigma + 1), whose
oracle planes are the separable sum written as two matrix products."""

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering
from parity import assert_planes_close, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")


def oracle_taps(kind, sigma, K=None):
    if kind == "sg":
        return design.colored_sg_taps(sigma, K=K)
    return design.gaussian_taps(sigma, K if K else design.fir_half_length(sigma))


ALGOS = {"direct": P.FIR_DIRECT, "mfma": P.FIR_TOEPLITZ_MFMA}


@pytest.mark.parametrize("shape", [(1, 1), (5, 300), (300, 5), (77, 131), (256, 2500), (129, 65)])
@pytest.mark.parametrize("kind", ["sg", "gaussian"])
@pytest.mark.parametrize("algo", list(ALGOS))
def test_fir_ragged(shape, kind, algo):
    H, W = shape
    say(f"case: fir {algo} {kind} {H}x{W}")
    rng = np.random.default_rng(H + 3 * W)
    img = (rng.random((H, W)) * 10).astype(np.float32)
    # the coloured SG needs omega_c = 3/sigma < pi (a non-empty stopband)
    sigmas = [1.2, 2.5, 11.0] if kind == "sg" else [0.7, 2.5, 11.0]
    for bc in ("replicate", "zero"):
        got = P.blur_fir(torch.from_numpy(img).cuda(), sigmas, kind=kind, boundary=bc,
                         algo=ALGOS[algo]).cpu().numpy()
        ref = np.stack([filtering.blur_2d(img.astype(np.float64), oracle_taps(kind, s), bc) for s in sigmas])
        assert_planes_close(got, ref, what=f"{bc} scale")


@pytest.mark.parametrize("algo", list(ALGOS))
def test_fir_explicit_lengths_precision_config(algo):
    """FIR lengths 33, 65, 129, 257 (sigma = K/3) on a normalised frame."""
    say(f"case: fir {algo} lengths 33..257")
    frame = syn.normalised_frame(700, 900, 3, nblobs=30).astype(np.float32)
    Ks = [16, 32, 64, 128]
    sig = [K / 3 for K in Ks]
    got = P.blur_fir(torch.from_numpy(frame).cuda(), sig, kind="sg", half_lens=Ks,
                     algo=ALGOS[algo]).cpu().numpy()
    ref = np.stack([filtering.blur_2d(frame.astype(np.float64), design.colored_sg_taps(s, K=K))
                    for s, K in zip(sig, Ks)])
    assert_planes_close(got, ref)


_FULL_REF = {}


def full_frame_reference():
    """The oracle's FIR planes of the 2048 x 2048 u16 frame, 8 scales (coloured
    SG, K = ceil(3 sigma)), computed once for both algorithms."""
    if not _FULL_REF:
        cfg = syn.FULL_FRAME
        frame = syn.aerial_frame(cfg["H"], cfg["W"], cfg["seed"])
        f64 = frame.astype(np.float64)
        _FULL_REF["frame"] = frame
        _FULL_REF["B"] = np.stack([filtering.blur_2d_matrix(f64, design.colored_sg_taps(s)) for s in cfg["sigmas"]])
    return _FULL_REF["frame"], _FULL_REF["B"]


@pytest.mark.parametrize("algo", list(ALGOS))
def test_full_frame_fir_every_pixel(algo):
    """The benchmark's FIR configuration compared element by element: every
    plane within 1e-5 of its maximum (normwise); per-scale max and rms printed."""
    cfg = syn.FULL_FRAME
    say(f"case: fir {algo} full frame 2048x2048 u16 8 scales (every pixel)")
    frame, ref = full_frame_reference()
    x = torch.from_numpy(frame.view(np.int16)).cuda()
    got = P.blur_fir(x, cfg["sigmas"], kind="sg", algo=ALGOS[algo]).cpu().numpy().astype(np.float64)
    for s in range(len(cfg["sigmas"])):
        d = got[s] - ref[s]
        scale = float(np.max(np.abs(ref[s])))
        say(f"   scale {s}: max {np.max(np.abs(d)) / scale:.2e} rms {np.sqrt(np.mean(d * d)) / scale:.2e} (of max |B|)")
    assert_planes_close(got, ref)


@pytest.mark.parametrize("algo", list(ALGOS))
def test_fir_long_taps(algo):
    """Half-lengths near the 512 limit, and a tap set too long for the matrix
    cores' one-launch table (sum of K + 1 over the scales > 880: the Toeplitz
    form then runs scale by scale)."""
    rng = np.random.default_rng(21)
    img = (rng.random((300, 1200)) * 100).astype(np.float32)
    for Ks in ([510], [300, 350, 400]):
        say(f"case: fir {algo} long taps K={Ks} 300x1200")
        sig = [K / 3 for K in Ks]
        got = P.blur_fir(torch.from_numpy(img).cuda(), sig, kind="sg", half_lens=Ks,
                         algo=ALGOS[algo]).cpu().numpy()
        ref = np.stack([filtering.blur_2d_matrix(img.astype(np.float64), design.colored_sg_taps(sg, K=K))
                        for sg, K in zip(sig, Ks)])
        assert_planes_close(got, ref)


@pytest.mark.parametrize("dtype", ["f16", "bf16", "u16"])
def test_fir_mfma_input_dtypes(dtype):
    say(f"case: fir mfma dtype {dtype} 150x333")
    rng = np.random.default_rng(11)
    if dtype == "u16":
        a = rng.integers(0, 4096, (150, 333)).astype(np.uint16)
        x = torch.from_numpy(a.view(np.int16)).cuda()
        x64 = a.astype(np.float64)
    else:
        t = torch.from_numpy(rng.random((150, 333)).astype(np.float32))
        t = t.to(torch.float16 if dtype == "f16" else torch.bfloat16)
        x = t.cuda()
        x64 = t.float().numpy().astype(np.float64)
    sig = [1.5, 6.0, 30.0]
    got = P.blur_fir(x, sig, kind="sg", algo=P.FIR_TOEPLITZ_MFMA).cpu().numpy()
    ref = np.stack([filtering.blur_2d(x64, design.colored_sg_taps(s)) for s in sig])
    assert_planes_close(got, ref)
