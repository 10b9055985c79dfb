"""GPU parity of fdvm_highpass (Table I differences) and fdvm_detect_blobs
(multi-scale strict extrema) against the oracle, on identical float32 inputs.
Detection on identical inputs is compared exactly (same fp32 values, same
decisions)."""

import numpy as np
import pytest

from oracle import shape
from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")


@pytest.mark.parametrize("shape_hw", [(1, 1), (2, 3), (45, 67), (256, 300)])
def test_highpass_all_outputs(shape_hw):
    H, W = shape_hw
    say(f"case: highpass {H}x{W}")
    rng = np.random.default_rng(H + W)
    B = rng.standard_normal((3, H, W)).astype(np.float32)
    sig = [1.5, 4.0, 20.0]
    what = P.HP_LAPLACIAN | P.HP_D20 | P.HP_D02 | P.HP_D11 | P.HP_D10 | P.HP_D01
    got = P.highpass(torch.from_numpy(B).cuda(), sig, what, True).cpu().numpy()
    for s in range(3):
        b = B[s].astype(np.float64)
        refs = [shape.laplacian(b, sig[s]), shape.derivative(b, 2, 0), shape.derivative(b, 0, 2),
                shape.derivative(b, 1, 1), shape.derivative(b, 1, 0), shape.derivative(b, 0, 1)]
        for j, ref in enumerate(refs):
            scale = max(1.0, np.max(np.abs(ref)))
            assert np.max(np.abs(got[s, j] - ref)) <= 2e-6 * scale, (s, j)


def test_highpass_unnormalised_laplacian():
    say("case: highpass unnormalised")
    rng = np.random.default_rng(3)
    B = rng.random((2, 30, 40)).astype(np.float32)
    got = P.highpass(torch.from_numpy(B).cuda(), [3.0, 5.0], P.HP_LAPLACIAN, False).cpu().numpy()
    for s in range(2):
        ref = shape.laplacian(B[s].astype(np.float64), 1.0)
        assert np.max(np.abs(got[s] - ref)) < 1e-6


def keys(bl):
    return [(int(b["scale"]), int(b["y"]), int(b["x"]), int(b["polarity"])) for b in bl]


@pytest.mark.parametrize("S,H,W,border,tau", [(1, 40, 50, 1, 0.5), (3, 64, 130, 1, 0.3), (4, 33, 70, 0, 0.0),
                                              (2, 100, 65, 3, 1.0), (5, 7, 9, 1, 0.2)])
def test_detect_matches_oracle_exactly(S, H, W, border, tau):
    say(f"case: detect S={S} {H}x{W} border={border} tau={tau}")
    rng = np.random.default_rng(S * 100 + H)
    V = np.round(rng.standard_normal((S, H, W)), 1).astype(np.float32)  # ties included
    got = P.detect_blobs(torch.from_numpy(V).cuda(), tau, border)
    ref = shape.detect_extrema(V.astype(np.float64), tau, border)
    assert keys(got) == keys(ref)
    assert np.array_equal(got["value"], ref["value"].astype(np.float32))


def test_detect_overflow_reports_true_count():
    say("case: detect overflow")
    rng = np.random.default_rng(8)
    V = rng.standard_normal((2, 128, 256)).astype(np.float32)
    ref = shape.detect_extrema(V.astype(np.float64), 0.0, 1)
    assert len(ref) > 50
    n = P.detect_blobs(torch.from_numpy(V).cuda(), 0.0, 1, count_only=True)
    assert n == len(ref)
    with pytest.raises(P.FdvmError) as ei:
        P.detect_blobs(torch.from_numpy(V).cuda(), 0.0, 1, cap=50)
    assert ei.value.status == P.EOVERFLOW


def test_detect_nothing_and_large_tau():
    say("case: detect empty")
    V = torch.zeros((3, 50, 60), device="cuda")
    assert len(P.detect_blobs(V, 0.0, 1)) == 0
    V2 = torch.randn((2, 50, 60), device="cuda")
    assert len(P.detect_blobs(V2, 1e9, 1)) == 0


def planted(S, H, W, n, seed):
    """Zero planes with n isolated +-1 values (no two within one step in
    scale, y and x; none on the one-pixel border): each is a strict extremum
    with |V| = 1, and no other pixel is."""
    rng = np.random.default_rng(seed)
    taken = set()
    pts = []
    while len(pts) < n:
        s, y, x = int(rng.integers(0, S)), int(rng.integers(1, H - 1)), int(rng.integers(1, W - 1))
        if any((s + a, y + b, x + c) in taken for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)):
            continue
        taken.add((s, y, x))
        pts.append((s, y, x, 1 if rng.random() < 0.5 else -1))
    return sorted(pts)


@pytest.mark.parametrize("S,H,W", [(4, 2048, 1024), (16, 16384, 1024)])
@pytest.mark.parametrize("tau", [0.5, 0.0])
def test_detect_planted_extrema_both_compaction_routes(S, H, W, tau):
    """Planted isolated extrema: the list is exactly the planted pixels in
    (scale, y, x) order, polarity +1 for the minima.  The first stack has few
    word blocks (the emit kernel forms its block offsets), the second more
    than 4096 (a separate scan forms them); tau = 0 takes the key path."""
    say(f"case: planted extrema S={S} {H}x{W} tau={tau}")
    pts = planted(S, H, W, 3000, S * 7 + H)
    V = torch.zeros((S, H, W), dtype=torch.float32, device="cuda")
    idx = torch.tensor([[s, y, x] for s, y, x, _ in pts], dtype=torch.long, device="cuda")
    val = torch.tensor([-1.0 if pol > 0 else 1.0 for *_, pol in pts], dtype=torch.float32, device="cuda")
    V[idx[:, 0], idx[:, 1], idx[:, 2]] = val
    det = P.detect_blobs(V, tau, 1)
    got = [(int(d["scale"]), int(d["y"]), int(d["x"]), int(d["polarity"])) for d in det]
    assert got == pts
    del V
