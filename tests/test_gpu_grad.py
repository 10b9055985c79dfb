"""GPU checks of the gradient path (adjoint kernels behind
paper_1912_07133_amd.iir_laplacian_grad).

* Dot-product tests of the transposed operators against the FP64 oracle's
  forward operators: <G x, y> = <x, G^T y> and <Lap B, g> = <B, Lap^T g>.
* d B / d sigma from the sigma-derivative recursions against an FP64 central
  difference of the oracle blur.
* Plane inner products against numpy.
* End to end: loss = sum over the detected blob centres of V^2 (the set held
  fixed), gradients in the image and in sigma against the FP64 reference
  gradient (central differences of the oracle, h = 1e-3) on a small frame, and
  against central differences of the GPU forward (h = 1e-3) on a 1024 x 1024
  frame with the scales sigma = 3, 6, 12, 24."""

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering, shape
from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")

SIGMAS_GRAD = syn.DIFFERENTIATION["sigmas"]


def oracle_blur(x64, sigmas, bc="replicate"):
    return filtering.blur_bank(x64, [design.repeated_pole(3, s) for s in sigmas], bc)


@pytest.mark.parametrize("bc", ["replicate", "zero"])
@pytest.mark.parametrize("shape_", [(70, 90), (1, 40), (33, 1), (130, 257), (20, 2100), (1100, 7)])
def test_blur_adjoint_dot_product(bc, shape_):
    # the last two put more than 1024 samples of the folded tail (sigma = 40)
    # along x and along y: the tail table is scanned in several blocks
    H, W = shape_
    say(f"case: blur adjoint {H}x{W} {bc}")
    rng = np.random.default_rng(H * 13 + W)
    sig = [0.8, 3.0, 12.0, 40.0]
    x = rng.standard_normal((H, W))
    y = rng.standard_normal((len(sig), H, W))
    Gx = oracle_blur(x, sig, bc)
    gty = P.blur_iir_adjoint(torch.from_numpy(y.astype(np.float32)).cuda(), sig, boundary=bc).cpu().numpy()
    y32 = y.astype(np.float32).astype(np.float64)   # the GPU saw y rounded to float32
    for s in range(len(sig)):
        lhs = float(np.sum(Gx[s] * y32[s]))
        rhs = float(np.sum(x * gty[s].astype(np.float64)))
        scale = float(np.sum(np.abs(Gx[s] * y32[s]))) + 1e-30
        assert abs(lhs - rhs) <= 1e-5 * scale, (s, lhs, rhs)


def test_laplacian_adjoint_dot_product():
    rng = np.random.default_rng(3)
    sig = [1.0, 2.5, 7.0]
    for H, W in [(1, 1), (1, 9), (8, 1), (2, 2), (45, 61)]:
        say(f"case: laplacian adjoint {H}x{W}")
        B = rng.standard_normal((len(sig), H, W))
        g = rng.standard_normal((len(sig), H, W)).astype(np.float32)
        LtG = P.laplacian_adjoint(torch.from_numpy(g).cuda(), sig).cpu().numpy().astype(np.float64)
        for s, sg in enumerate(sig):
            lhs = float(np.sum(shape.laplacian(B[s], sg) * g[s]))
            rhs = float(np.sum(B[s] * LtG[s]))
            # float32 rounding of the transposed stencil: relative to its l1 norm
            scale = 8.0 * sg * sg * float(np.sum(np.abs(B[s]) * np.abs(g[s])))
            assert abs(lhs - rhs) <= 1e-6 * scale, (H, W, s, lhs, rhs)


@pytest.mark.parametrize("bc", ["replicate", "zero"])
def test_sigma_derivative_against_fp64_central_difference(bc):
    say(f"case: dB/dsigma {bc}")
    frame = syn.aerial_frame(96, 140, 21, nblobs=6).astype(np.float64)
    sig = [1.2, 3.0, 9.0, 30.0]
    D1, D2 = P.dblur_dsigma_parts(torch.from_numpy(frame.astype(np.float32)).cuda(), sig, boundary=bc)
    got = (D1 + D2).cpu().numpy().astype(np.float64)
    for s, sg in enumerate(sig):
        d = 1e-4 * sg
        ref = (oracle_blur(frame, [sg + d], bc)[0] - oracle_blur(frame, [sg - d], bc)[0]) / (2 * d)
        err = float(np.max(np.abs(got[s] - ref)))
        assert err <= 1e-4 * float(np.max(np.abs(ref))) + 1e-3, (s, err, float(np.max(np.abs(ref))))


def test_plane_dots():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((3, 37, 1001)).astype(np.float32)
    b = rng.standard_normal((3, 37, 1001)).astype(np.float32)
    got = P.plane_dots(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()).cpu().numpy()
    ref = np.einsum("shw,shw->s", a.astype(np.float64), b.astype(np.float64))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)
    again = P.plane_dots(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()).cpu().numpy()
    assert np.array_equal(got, again)   # fixed summation order


def centres_of(V, tau):
    det = P.detect_blobs(V.detach(), tau, 1)
    return [(int(d["scale"]), int(d["y"]), int(d["x"])) for d in det]


def gpu_loss(x, sig_t, centres):
    V = P.iir_laplacian_grad(x, sig_t)
    idx = torch.tensor(centres, dtype=torch.long, device=V.device)
    return (V[idx[:, 0], idx[:, 1], idx[:, 2]].double() ** 2).sum()


def oracle_loss(x64, sig, centres):
    V = shape.laplacian_bank(oracle_blur(x64, sig), sig)
    return float(sum(V[s, y, x] ** 2 for s, y, x in centres))


def test_gradients_against_fp64_reference():
    """128 x 128 frame, sigma = 3, 6, 12, 24: autograd gradients against
    central differences (h = 1e-3) of the FP64 oracle loss."""
    say("case: gradients vs FP64 reference")
    frame = (syn.normalised_frame(128, 128, 500, nblobs=8)).astype(np.float32)
    x = torch.from_numpy(frame).cuda().requires_grad_(True)
    sig_t = torch.tensor(SIGMAS_GRAD, dtype=torch.float64, device="cuda", requires_grad=True)
    with torch.no_grad():
        V0 = P.iir_laplacian(x, SIGMAS_GRAD)
    centres = centres_of(V0, 0.02)
    assert len(centres) >= 4
    L = gpu_loss(x, sig_t, centres)
    L.backward()
    gx, gs = x.grad.cpu().numpy(), sig_t.grad.cpu().numpy()
    x64 = frame.astype(np.float64)
    h = 1e-3
    for s in range(len(SIGMAS_GRAD)):
        sp = list(SIGMAS_GRAD); sm = list(SIGMAS_GRAD)
        sp[s] += h; sm[s] -= h
        ref = (oracle_loss(x64, sp, centres) - oracle_loss(x64, sm, centres)) / (2 * h)
        say(f"   dL/dsigma[{s}] gpu={gs[s]:.6g} ref={ref:.6g}")
        assert abs(gs[s] - ref) <= 1e-3 * abs(ref) + 1e-9, (s, gs[s], ref)
    rng = np.random.default_rng(0)
    pts = [(y, x_) for _, y, x_ in centres[:6]] + [tuple(p) for p in rng.integers(0, 128, (6, 2))]
    refs, gots = [], []
    for (py, px) in pts:
        xp = x64.copy(); xp[py, px] += h
        xm = x64.copy(); xm[py, px] -= h
        refs.append((oracle_loss(xp, SIGMAS_GRAD, centres) - oracle_loss(xm, SIGMAS_GRAD, centres)) / (2 * h))
        gots.append(gx[py, px])
    refs, gots = np.array(refs), np.array(gots)
    say(f"   dL/dx max|ref|={np.max(np.abs(refs)):.4g} max|diff|={np.max(np.abs(refs - gots)):.3g}")
    assert np.max(np.abs(refs - gots)) <= 1e-3 * np.max(np.abs(refs))


def test_gradients_full_size_against_gpu_central_differences():
    """One 1024 x 1024 float32 frame of the differentiation configuration:
    autograd gradients against central differences (h = 1e-3) of the GPU
    forward."""
    cfg = syn.DIFFERENTIATION
    say("case: gradients 1024x1024 vs GPU central differences")
    frame = syn.normalised_frame(cfg["H"], cfg["W"], 500, nblobs=cfg["nblobs"]).astype(np.float32)
    x = torch.from_numpy(frame).cuda().requires_grad_(True)
    sig_t = torch.tensor(cfg["sigmas"], dtype=torch.float64, device="cuda", requires_grad=True)
    with torch.no_grad():
        V0 = P.iir_laplacian(x, cfg["sigmas"])
    centres = centres_of(V0, 0.02)
    assert len(centres) >= 10
    L = gpu_loss(x, sig_t, centres)
    L.backward()
    gs = sig_t.grad.cpu().numpy()
    h = 1e-3
    with torch.no_grad():
        for s in range(len(cfg["sigmas"])):
            sp = sig_t.detach().clone(); sp[s] += h
            sm = sig_t.detach().clone(); sm[s] -= h
            ref = float(gpu_loss(x.detach(), sp, centres) - gpu_loss(x.detach(), sm, centres)) / (2 * h)
            say(f"   dL/dsigma[{s}] autograd={gs[s]:.6g} fd={ref:.6g}")
            assert abs(gs[s] - ref) <= 1e-2 * abs(ref) + 1e-6
        gx = x.grad
        for (s_, py, px) in centres[:5]:
            xp = x.detach().clone(); xp[py, px] += h
            xm = x.detach().clone(); xm[py, px] -= h
            ref = float(gpu_loss(xp, sig_t.detach(), centres) - gpu_loss(xm, sig_t.detach(), centres)) / (2 * h)
            got = float(gx[py, px])
            say(f"   dL/dx[{py},{px}] autograd={got:.6g} fd={ref:.6g}")
            assert abs(got - ref) <= 5e-2 * abs(ref) + 1e-3
