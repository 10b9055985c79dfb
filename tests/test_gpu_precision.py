"""Reduced-precision storage: frames stored as float16 and bfloat16 (RNE) of the
normalised aerial generator, blurred by the IIR (K = 3) and by the coloured SG
FIR of lengths 33, 65, 129, 257 (sigma = K/3) on both FIR algorithms.

Errors against the FP64 oracle, per scale, normwise (max |err| / max |ref|):
  * on the dequantised stored input: the float32 / float64 arithmetic of the
    kernels only, <= 1e-5;
  * on the original (unquantised) input: storage rounding included, <= 2e-3.
The FIR is checked on sampled pixels (direct 2-D sums), the IIR everywhere."""

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


def stored(frame64, kind):
    t = torch.from_numpy(frame64.astype(np.float32)).to(torch.float16 if kind == "f16" else torch.bfloat16)
    return t.cuda(), t.float().numpy().astype(np.float64)


def sampled_2d(img64, h, points):
    H, W = img64.shape
    K = (len(h) - 1) // 2
    r = np.arange(-K, K + 1)
    return np.array([h @ img64[np.ix_(np.clip(i - r, 0, H - 1), np.clip(j - r, 0, W - 1))] @ h for i, j in points])


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_iir_on_stored_frames(kind):
    say(f"case: precision iir {kind} 1024x1024")
    orig = syn.normalised_frame(1024, 1024, CFG["seed"], nblobs=CFG["nblobs"] // 64)
    x, deq = stored(orig, kind)
    got = P.blur_iir(x, SIGS, order=3).cpu().numpy().astype(np.float64)
    for s, sg in enumerate(SIGS):
        f = design.repeated_pole(3, sg)
        ref_q = filtering.blur_2d(deq, f)
        ref_o = filtering.blur_2d(orig, f)
        eq = float(np.max(np.abs(got[s] - ref_q))) / float(np.max(np.abs(ref_q)))
        eo = float(np.max(np.abs(got[s] - ref_o))) / float(np.max(np.abs(ref_o)))
        say(f"   sigma {sg:.2f}: vs dequantised {eq:.2e}, vs original {eo:.2e}")
        assert eq <= 1e-5
        assert eo <= 2e-3


@pytest.mark.parametrize("kind", ["f16", "bf16"])
@pytest.mark.parametrize("algo", ["direct", "mfma"])
def test_fir_lengths_on_stored_frames(kind, algo):
    say(f"case: precision fir {algo} {kind} 1024x1024")
    orig = syn.normalised_frame(1024, 1024, CFG["seed"], nblobs=CFG["nblobs"] // 64)
    x, deq = stored(orig, kind)
    a = P.FIR_DIRECT if algo == "direct" else P.FIR_TOEPLITZ_MFMA
    got = P.blur_fir(x, SIGS, kind="sg", half_lens=KS, algo=a).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(1)
    pts = [(0, 0), (1023, 1023), (5, 700)] + [tuple(p) for p in rng.integers(0, 1024, (40, 2))]
    for s, (sg, K) in enumerate(zip(SIGS, KS)):
        h = design.colored_sg_taps(sg, K=K)
        ref_q = sampled_2d(deq, h, pts)
        ref_o = sampled_2d(orig, h, pts)
        g = np.array([got[s, i, j] for i, j in pts])
        eq = float(np.max(np.abs(g - ref_q))) / float(np.max(np.abs(ref_q)))
        eo = float(np.max(np.abs(g - ref_o))) / float(np.max(np.abs(ref_o)))
        say(f"   length {2 * K + 1}: vs dequantised {eq:.2e}, vs original {eo:.2e}")
        assert eq <= 1e-5
        assert eo <= 2e-3
