"""Reduced-precision storage: frames stored as float16 and bfloat16 (RNE) of the
normalised aerial generator, blurred by the IIR (K = 3) and by the coloured SG
FIR of lengths 33, 65, 129, 257 (sigma = K/3) on both FIR algorithms.

Errors against the FP64 oracle, per scale, normwise (max |err| / max |ref|):
  * on the dequantised stored input: the float32 / float64 arithmetic of the
    kernels only, <= 1e-5;
  * on the original (unquantised) input: storage rounding included, <= 2e-3.
Every pixel is compared (the FIR oracle planes as two matrix products of the
separable sum)."""

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


_REF = {}


def fir_references(kind):
    """Oracle FIR planes of the stored (dequantised) and the original frame."""
    if kind not in _REF:
        orig = syn.normalised_frame(1024, 1024, CFG["seed"], nblobs=CFG["nblobs"] // 64)
        x, deq = stored(orig, kind)
        hs = [design.colored_sg_taps(sg, K=K) for sg, K in zip(SIGS, KS)]
        _REF[kind] = (x, np.stack([filtering.blur_2d_matrix(deq, h) for h in hs]),
                      np.stack([filtering.blur_2d_matrix(orig, h) for h in hs]))
    return _REF[kind]


@pytest.mark.parametrize("kind", ["f16", "bf16"])
@pytest.mark.parametrize("algo", ["direct", "mfma"])
def test_fir_lengths_on_stored_frames(kind, algo):
    """Every pixel; per-scale max and rms errors printed."""
    say(f"case: precision fir {algo} {kind} 1024x1024")
    x, ref_q, ref_o = fir_references(kind)
    a = P.FIR_DIRECT if algo == "direct" else P.FIR_TOEPLITZ_MFMA
    got = P.blur_fir(x, SIGS, kind="sg", half_lens=KS, algo=a).cpu().numpy().astype(np.float64)
    for s, K in enumerate(KS):
        dq, do = got[s] - ref_q[s], got[s] - ref_o[s]
        sq, so = float(np.max(np.abs(ref_q[s]))), float(np.max(np.abs(ref_o[s])))
        eq, eo = float(np.max(np.abs(dq))) / sq, float(np.max(np.abs(do))) / so
        say(f"   length {2 * K + 1}: vs dequantised max {eq:.2e} rms {np.sqrt(np.mean(dq * dq)) / sq:.2e}; "
            f"vs original max {eo:.2e} rms {np.sqrt(np.mean(do * do)) / so:.2e}")
        assert eq <= 1e-5
        assert eo <= 2e-3
