"""GPU parity of fdvm_blur_fir (Eq A5, separable) against the oracle, for both
algorithms: direct LDS-staged convolution and the Toeplitz-block products on
the matrix cores (float32 operands and accumulation).

Small frames are compared everywhere; the 2048x2048 x 8-scale frame (the
benchmark's FIR configuration, coloured SG of length 6 sigma + 1) is compared
on sampled pixels, each computed by the oracle as a direct 2-D sum."""

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


def sampled_2d(img64, h, points):
    """Direct 2-D sums B(i, j) = sum_ab h(a) h(b) X(clamp(i - a), clamp(j - b))."""
    H, W = img64.shape
    K = (len(h) - 1) // 2
    r = np.arange(-K, K + 1)
    out = []
    for i, j in points:
        rows = np.clip(i - r, 0, H - 1)
        cols = np.clip(j - r, 0, W - 1)
        out.append(h @ img64[np.ix_(rows, cols)] @ h)
    return np.array(out)


@pytest.mark.parametrize("algo", list(ALGOS))
def test_full_frame_fir_sampled(algo):
    cfg = syn.FULL_FRAME
    say(f"case: fir {algo} full frame 2048x2048 u16 8 scales (sampled)")
    frame = syn.aerial_frame(cfg["H"], cfg["W"], cfg["seed"])
    x = torch.from_numpy(frame.view(np.int16)).cuda()
    got = P.blur_fir(x, cfg["sigmas"], kind="sg", algo=ALGOS[algo]).cpu().numpy()
    rng = np.random.default_rng(0)
    pts = [(0, 0), (2047, 2047), (0, 2047), (5, 1000), (1024, 3)] + \
          [tuple(p) for p in rng.integers(0, 2048, (60, 2))]
    f64 = frame.astype(np.float64)
    for s, sigma in enumerate(cfg["sigmas"]):
        ref = sampled_2d(f64, design.colored_sg_taps(sigma), pts)
        g = np.array([got[s, i, j] for i, j in pts])
        assert np.max(np.abs(g - ref)) <= 1e-5 * np.max(np.abs(f64)), s


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
