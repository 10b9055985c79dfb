"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, its host-only filter design matches the oracle, and the
host-side argument validation rejects bad calls before touching a device."""

import ctypes
import math

import numpy as np
import pytest

import paper_1912_07133_amd as P
from oracle import design

pytestmark = pytest.mark.skipif(not P.library_available(), reason="libfdvm.so not built")


def test_every_header_symbol_is_exported():
    syms = P.header_symbols()
    assert set(syms) >= {"fdvm_filter_design", "fdvm_blur_iir", "fdvm_blur_fir", "fdvm_highpass",
                         "fdvm_detect_blobs", "fdvm_workspace_bytes", "fdvm_status_string"}
    L = P.lib()
    for name in syms:
        assert hasattr(L, name), name


def test_struct_layouts_match_header():
    assert ctypes.sizeof(P.Blob) == 20
    assert ctypes.sizeof(P.Filter) == 8 + 8 * 3 + 8 * 4 * 2 + 8 * 2 + 8


@pytest.mark.parametrize("sigma", [0.3, 1.0, 2.0, 8.0, 23.8, 64.0, 96.0, 1000.0])
def test_iir_design_matches_table_iv(sigma):
    d = P.filter_design("iir", sigma, order=3)
    t = design.table_iv(sigma)
    assert d["p"] == pytest.approx(math.exp(-1 / sigma), rel=1e-15)
    assert d["b0"] == pytest.approx(t.b0, rel=1e-9, abs=1e-16)
    for m in range(4):
        assert d["bp"][m] == pytest.approx(t.bp[m], rel=1e-7 if sigma > 500 else 1e-10, abs=1e-16)
        assert d["ap"][m] == pytest.approx(t.ap[m], rel=1e-14)
    assert d["side_gain"] == pytest.approx((1 - t.b0) / 2, rel=1e-12)


@pytest.mark.parametrize("sigma", [0.5, 1.5, 4.0, 12.0, 64.0])
def test_iir_order2_design_matches_general_procedure(sigma):
    d = P.filter_design("iir", sigma, order=2)
    g = design.repeated_pole(2, sigma)
    assert d["b0"] == pytest.approx(g.b0, rel=1e-10)
    for m in range(3):
        assert d["bp"][m] == pytest.approx(g.bp[m], rel=1e-9, abs=1e-16)
        assert d["ap"][m] == pytest.approx(g.ap[m], rel=1e-14)


@pytest.mark.parametrize("sigma", [2.0, 3.28, 8.83, 23.8, 64.0, 96.0])
def test_colored_sg_taps_match_oracle(sigma):
    got = P.filter_design("sg", sigma)["taps"]
    ref = design.colored_sg_taps(sigma)
    assert len(got) == len(ref) == 2 * math.ceil(3 * sigma - 1e-9) + 1
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_fir_length_override_and_gaussian():
    d = P.filter_design("sg", 10.0, fir_half_len=64)
    assert d["ntaps"] == 129
    # K = 6.4 sigma: S of Eq 22 has condition number ~2e15, so two float64
    # solves agree only to ~1e-7 relative; both meet the constraints exactly
    ref = design.colored_sg_taps(10.0, K=64)
    assert np.max(np.abs(d["taps"] - ref)) < 1e-6 * np.max(np.abs(ref))
    m = np.arange(-64, 65)
    assert abs(d["taps"].sum() - 1) < 1e-14 and abs((m * m * d["taps"]).sum()) < 1e-9
    g = P.filter_design("gaussian", 4.0, fir_half_len=20)["taps"]
    assert np.max(np.abs(g - design.gaussian_taps(4.0, 20))) < 1e-15


@pytest.mark.parametrize("sigma,K", [(2.0, 0), (5.4, 0), (23.8, 0), (64.0, 0), (10.0, 40)])
def test_fir_dsigma_designs_match_oracle(sigma, K):
    """d h / d sigma of the coloured SG (Lagrange system of Eq 20
    differentiated) and of the sampled Gaussian, at fixed K."""
    Kk = K if K else math.ceil(3 * sigma - 1e-9)
    got = P.filter_design(P.FIR_COLORED_SG_DSIGMA, sigma, fir_half_len=K)
    ref = design.colored_sg_taps_dsigma(sigma, Kk)
    assert got["ntaps"] == 2 * Kk + 1
    assert np.max(np.abs(got["taps"] - ref)) <= 1e-7 * np.max(np.abs(ref))
    assert got["b0"] == got["taps"][Kk]
    g = P.filter_design(P.FIR_GAUSSIAN_DSIGMA, sigma, fir_half_len=K)["taps"]
    assert np.max(np.abs(g - design.gaussian_taps_dsigma(sigma, Kk))) <= 1e-12 * np.max(np.abs(g))


def test_design_errors():
    L = P.lib()
    f = P.Filter()
    buf = (ctypes.c_double * 10)()
    assert L.fdvm_filter_design(0, 3, 8.0, 0, None, None, 0) == P.EINVAL
    assert L.fdvm_filter_design(0, 4, 8.0, 0, ctypes.byref(f), None, 0) == P.EINVAL
    assert L.fdvm_filter_design(0, 3, 0.1, 0, ctypes.byref(f), None, 0) == P.ERANGE
    assert L.fdvm_filter_design(0, 3, float("nan"), 0, ctypes.byref(f), None, 0) == P.ERANGE
    assert L.fdvm_filter_design(1, 0, 8.0, 0, ctypes.byref(f), buf, 10) == P.ENOMEM
    assert L.fdvm_filter_design(1, 0, 8.0, 0, ctypes.byref(f), None, 0) == P.EINVAL
    assert L.fdvm_filter_design(1, 0, 8.0, 600, ctypes.byref(f), buf, 10) == P.ERANGE
    assert L.fdvm_filter_design(7, 3, 8.0, 0, ctypes.byref(f), None, 0) == P.EINVAL
    assert P.status_string(P.EOVERFLOW) == "detection list overflow"


def test_device_calls_validate_on_the_host():
    """Bad arguments are rejected before any HIP call (no GPU in this test)."""
    L = P.lib()
    f = P.Filter()
    assert L.fdvm_filter_design(0, 3, 4.0, 0, ctypes.byref(f), None, 0) == P.OK
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    filt = (P.Filter * 1)(f)
    assert L.fdvm_blur_iir(None, P.F32, 8, 8, 8, fake, 8, 64, filt, 1, 0, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, P.F32, 0, 8, 8, fake, 8, 64, filt, 1, 0, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 4, fake, 8, 64, filt, 1, 0, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 8, fake, 8, 64, filt, 0, 0, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 8, fake, 8, 64, filt, 17, 0, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, 9, 8, 8, 8, fake, 8, 64, filt, 1, 0, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 8, fake, 8, 64, filt, 1, 5, fake, 1 << 30, None) == P.EINVAL
    two = (P.Filter * 2)(f, f)
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 8, fake, 8, 10, two, 2, 0, fake, 1 << 30, None) == P.EINVAL  # stride
    f2 = P.Filter()
    assert L.fdvm_filter_design(0, 2, 4.0, 0, ctypes.byref(f2), None, 0) == P.OK
    mixed = (P.Filter * 2)(f, f2)
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 8, fake, 8, 64, mixed, 2, 0, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 8, fake, 8, 64, filt, 1, 0, None, 0, None) == P.EINVAL
    assert L.fdvm_blur_iir(fake, P.F32, 8, 8, 8, fake, 8, 64, filt, 1, 0, fake, 16, None) == P.ENOMEM
    assert L.fdvm_iir_laplacian(fake, P.F32, 8, 8, 8, fake, 8, 64, filt, 1, 0, fake, 16, None) == P.ENOMEM
    assert L.fdvm_iir_pass(fake, P.U16, 8, 8, 8, 64, fake, 8, 64, filt, 1, 0, 1, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_iir_pass(fake, P.F32, 8, 8, 8, 64, fake, 8, 64, filt, 1, 0, 2, fake, 1 << 30, None) == P.EINVAL
    assert L.fdvm_iir_pass(fake, P.F32, 8, 8, 8, 64, fake, 8, 64, filt, 1, 0, 3, fake, 1 << 30, None) == P.EINVAL
    sig = (ctypes.c_double * 1)(2.0)
    assert L.fdvm_highpass(fake, 8, 8, 8, 64, 1, sig, 0, 1, fake, 64, None) == P.EINVAL
    assert L.fdvm_highpass(fake, 8, 8, 8, 64, 1, sig, 64, 1, fake, 64, None) == P.EINVAL
    assert L.fdvm_highpass(fake, 8, 8, 8, 64, 1, sig, 3, 1, fake, 10, None) == P.EINVAL
    assert L.fdvm_detect_blobs(fake, 8, 8, 8, 64, 1, -1.0, 1, fake, 10, fake, fake, 1 << 20, None) == P.EINVAL
    assert L.fdvm_detect_blobs(fake, 8, 8, 8, 64, 1, 0.5, 1, fake, 10, fake, fake, 1, None) == P.ENOMEM
    half = (ctypes.c_int32 * 1)(2)
    off = (ctypes.c_int32 * 1)(0)
    asym = (ctypes.c_double * 5)(0.1, 0.2, 0.4, 0.2, 0.11)
    assert L.fdvm_blur_fir(fake, P.F32, 8, 8, 8, fake, 8, 64, asym, half, off, 1, 0, 0, fake, 1 << 20,
                           None) == P.EINVAL
    sym = (ctypes.c_double * 5)(0.1, 0.2, 0.4, 0.2, 0.1)
    assert L.fdvm_blur_fir(fake, P.F32, 8, 8, 8, fake, 8, 64, sym, half, off, 1, 0, 0, fake, 4, None) == P.ENOMEM
    # half-precision matrix-core operands: float16, bfloat16 and uint16 frames
    assert L.fdvm_blur_fir(fake, P.F32, 8, 8, 8, fake, 8, 64, sym, half, off, 1, 0, P.FIR_TOEPLITZ_MFMA_HALF,
                           fake, 1 << 20, None) == P.EINVAL
    assert L.fdvm_blur_fir(fake, P.F16, 8, 8, 8, fake, 8, 64, sym, half, off, 1, 0, 3, fake, 1 << 20,
                           None) == P.EINVAL


def test_fir_laplacian_mfma_validation():
    """fdvm_fir_laplacian_mfma rejects, on the host, float32 frames,
    asymmetric taps, half-lengths beyond FDVM_MAX_FIR_LAP_MFMA_HALF, bad sigmas
    and short workspaces (fake device pointers, nothing is launched)."""
    L = P.lib()
    fake = ctypes.c_void_p(0x1000)
    half = (ctypes.c_int32 * 1)(2)
    off = (ctypes.c_int32 * 1)(0)
    sym = (ctypes.c_double * 5)(0.1, 0.2, 0.4, 0.2, 0.1)
    asym = (ctypes.c_double * 5)(0.1, 0.2, 0.4, 0.2, 0.11)
    sig = (ctypes.c_double * 1)(2.0)
    big = 1 << 30

    def call(dt, taps=sym, hl=half, sg=sig, ws_bytes=big, bc=0):
        return L.fdvm_fir_laplacian_mfma(fake, dt, 8, 8, 8, fake, 8, 64, taps, hl, off, sg, 1, bc, fake, ws_bytes,
                                         None)

    assert call(P.F32) == P.EINVAL
    assert call(P.F16, taps=asym) == P.EINVAL
    assert call(P.F16, hl=(ctypes.c_int32 * 1)(P.MAX_FIR_LAP_MFMA_HALF + 1)) == P.ERANGE
    assert call(P.F16, hl=(ctypes.c_int32 * 1)(0)) == P.ERANGE
    assert call(P.U16, sg=(ctypes.c_double * 1)(-1.0)) == P.ERANGE
    assert call(P.BF16, bc=7) == P.EINVAL
    need = P.workspace_bytes(P.OP_FIR_LAPLACIAN_MFMA, 8, 8, 1)
    assert need > 0
    assert call(P.F16, ws_bytes=need - 1) == P.ENOMEM


def test_workspace_sizes():
    assert P.workspace_bytes(P.OP_BLUR_IIR, 2048, 2048, 8) >= 8 * 32 * 6 * 2048 * 4
    assert P.workspace_bytes(P.OP_IIR_LAPLACIAN, 2048, 2048, 8) >= 8 * 2048 * 2048 * 4
    assert P.workspace_bytes(P.OP_BLUR_FIR, 2048, 2048, 8, 192) >= 2048 * 2048 * 4
    assert P.workspace_bytes(P.OP_DETECT, 2048, 2048, 8) >= 8 * 2048 * (2048 // 64) * 8


def test_batch_layout_and_validation():
    """fdvm_frame layout, batch workspace sizing, and host-side rejection of bad
    batches (fake device pointers, nothing is launched)."""
    assert ctypes.sizeof(P.Frame) == 56
    L = P.lib()
    f = P.Filter()
    assert L.fdvm_filter_design(0, 3, 4.0, 0, ctypes.byref(f), None, 0) == P.OK
    filt = (P.Filter * 2)(f, f)
    fake = 0x1000

    def frames(*shapes, chunk=0, dtype=P.U16):
        fr = (P.Frame * len(shapes))()
        for i, (H, W) in enumerate(shapes):
            fr[i] = P.Frame(fake, dtype, H, W, chunk, W, fake, fake, 16, 0)
        return fr

    two = frames((300, 500), (64, 2048))
    per_lane = L.fdvm_batch_workspace_bytes(two, 2, 2, 1)
    # the largest frame term by term: x-pass planes + V planes of the 300 x 500
    # frame, states and words of the wider one
    assert per_lane >= 2 * (300 * 500 * 4) * 2
    assert L.fdvm_batch_workspace_bytes(two, 2, 2, 2) == 2 * per_lane
    assert L.fdvm_batch_workspace_bytes(two, 2, 2, 8) == 2 * per_lane   # lanes capped at the frame count
    assert L.fdvm_batch_workspace_bytes(two, 2, 17, 1) == 0
    ws = ctypes.c_void_p(fake)
    big = 1 << 40
    ok = lambda fr, n=2, lanes=2, tau=1.0: L.fdvm_batch_detect(fr, n, filt, 2, 0, tau, 1, lanes, ws, big, None)
    assert ok(frames((0, 5), (4, 4))) == P.EINVAL
    assert ok(frames((5, 5), (4, 4), chunk=12)) == P.EINVAL
    assert ok(frames((5, 5), (4, 4), dtype=9)) == P.EINVAL
    assert ok(frames((5, 5), (4, 16384), chunk=8)) == P.EUNSUPPORTED   # 64 * 8 * 8 < 16384
    assert ok(frames((5, 5), (4, 4)), lanes=0) == P.EINVAL
    assert ok(frames((5, 5), (4, 4)), lanes=17) == P.EINVAL
    assert ok(frames((5, 5), (4, 4)), tau=-1.0) == P.EINVAL
    bad = frames((5, 5), (4, 4))
    bad[1].pitch = 3
    assert ok(bad) == P.EINVAL
    assert L.fdvm_batch_detect(two, 2, filt, 2, 0, 1.0, 1, 2, ws, 16, None) == P.ENOMEM


def test_adjoint_entry_points_validate_on_the_host():
    L = P.lib()
    f = P.Filter()
    assert L.fdvm_filter_design(0, 3, 4.0, 0, ctypes.byref(f), None, 0) == P.OK
    d = P.Filter()
    assert L.fdvm_filter_design(3, 3, 4.0, 0, ctypes.byref(d), None, 0) == P.OK
    assert d.kind == 3 and d.order == 3
    filt = (P.Filter * 1)(f)
    dfilt = (P.Filter * 1)(d)
    a, b, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    big = 1 << 40
    assert L.fdvm_blur_iir_adjoint(a, 8, 8, 8, 64, a, 8, 64, filt, 1, 0, ws, big, None) == P.EINVAL   # aliasing
    assert L.fdvm_blur_iir_adjoint(a, 8, 8, 8, 64, b, 8, 64, dfilt, 1, 0, ws, big, None) == P.EINVAL  # kind
    assert L.fdvm_blur_iir_adjoint(a, 8, 8, 8, 64, b, 8, 64, filt, 1, 0, ws, 16, None) == P.ENOMEM
    # the sigma derivative is a per-pass filter: not accepted by the 2-D calls
    assert L.fdvm_blur_iir(a, P.F32, 8, 8, 8, b, 8, 64, dfilt, 1, 0, ws, big, None) == P.EINVAL
    assert L.fdvm_iir_laplacian(a, P.F32, 8, 8, 8, b, 8, 64, dfilt, 1, 0, ws, big, None) == P.EINVAL
    assert L.fdvm_iir_pass(a, P.F32, 8, 8, 8, 64, b, 8, 64, dfilt, 1, 0, 2, ws, big, None) == P.EINVAL
    sig = (ctypes.c_double * 1)(2.0)
    bad = (ctypes.c_double * 1)(-1.0)
    assert L.fdvm_laplacian_adjoint(a, 8, 8, 8, 64, 1, sig, a, 8, 64, None) == P.EINVAL
    assert L.fdvm_laplacian_adjoint(a, 8, 8, 8, 64, 1, bad, b, 8, 64, None) == P.ERANGE
    assert L.fdvm_plane_dots(a, b, 8, 8, 8, 64, 1, ws, ws, 1, None) == P.ENOMEM
    assert L.fdvm_plane_dots(a, None, 8, 8, 8, 64, 1, ws, ws, big, None) == P.EINVAL
    assert P.workspace_bytes(P.OP_BLUR_IIR_ADJOINT, 64, 64, 2) >= 2 * 64 * 64 * 4


def test_sigma_derivative_design_matches_difference_of_designs():
    """d b0 / d sigma of the derivative design against a central difference of
    the blur designs (host only)."""
    L = P.lib()
    for order in (2, 3):
        for s in (0.7, 2.0, 8.0, 40.0, 300.0):
            d = P.Filter()
            assert L.fdvm_filter_design(3, order, s, 0, ctypes.byref(d), None, 0) == P.OK
            h = 1e-5 * s
            num = (P.filter_design("iir", s + h, order)["b0"] - P.filter_design("iir", s - h, order)["b0"]) / (2 * h)
            assert abs(d.b0 - num) <= 1e-6 * abs(num) + 1e-12, (order, s)


# ------------------------------------------------- Butterworth (Filter E)

def _wc(sigma):
    return math.sqrt(2.0 * math.log(2.0)) / sigma   # Section 4.4 scale tuning


def test_butterworth_design_matches_filter_e():
    """The library's closed-form design (poles of the bilinear prototype and
    residues) at the Filter E cutoff reproduces the printed coefficients and
    the oracle's Eq A17 decomposition of the same transfer function."""
    wc = 0.1472
    d = P.filter_design("butterworth", math.sqrt(2.0 * math.log(2.0)) / wc, order=4)
    assert d["order"] == 4 and d["omega_c"] == pytest.approx(wc, rel=1e-15)
    printed = {"b0": 0.0518, "bp": [0.0, 0.0513, -0.0420], "ap": [1.0, -1.7929, 0.8124]}   # Section 5, Filter E
    tol = 0.5e-4 + 1e-4   # 4 printed decimals; the printed cutoff is itself rounded
    assert abs(d["b0"] - printed["b0"]) <= tol
    for m in range(3):
        assert abs(d["bp"][m] - printed["bp"][m]) <= tol
        assert abs(d["ap"][m] - printed["ap"][m]) <= tol
    ref = design.butterworth(4, wc)
    assert d["b0"] == pytest.approx(ref.b0, rel=1e-12)
    for m in range(3):
        assert d["bp"][m] == pytest.approx(ref.bp[m], rel=1e-12, abs=1e-15)
        assert d["ap"][m] == pytest.approx(ref.ap[m], rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("sigma", [0.5, 1.3, 4.0, 20.0, 150.0, 2000.0])
def test_butterworth_design_across_scales(sigma):
    """Against the oracle's decomposition at every scale of the supported
    range, and unit dc gain of the three-term DE: b0 + 2 B+(1)/A+(1) = 1."""
    d = P.filter_design("butterworth", sigma, order=4)
    ref = design.butterworth(4, _wc(sigma))
    assert d["b0"] == pytest.approx(ref.b0, rel=1e-9)
    for m in (1, 2):
        assert d["ap"][m] == pytest.approx(ref.ap[m], rel=1e-12)
        assert d["bp"][m] == pytest.approx(ref.bp[m], rel=1e-8, abs=1e-14)
    den = 1.0 + d["ap"][1] + d["ap"][2]   # A+(1) = |1 - p|^2, small at coarse scales
    side = (d["bp"][1] + d["bp"][2]) / den
    assert d["b0"] + 2.0 * side == pytest.approx(1.0, abs=1e-13 / den)
    assert d["side_gain"] == pytest.approx(side, rel=1e-7)


def test_butterworth_design_errors_and_unsupported_calls():
    L = P.lib()
    f = P.Filter()
    assert L.fdvm_filter_design(P.IIR_BUTTERWORTH, 3, 4.0, 0, ctypes.byref(f), None, 0) == P.EINVAL
    assert L.fdvm_filter_design(P.IIR_BUTTERWORTH, 4, 0.4, 0, ctypes.byref(f), None, 0) == P.ERANGE
    assert L.fdvm_filter_design(P.IIR_BUTTERWORTH, 4, 4.0, 0, ctypes.byref(f), None, 0) == P.OK
    g = P.Filter()
    assert L.fdvm_filter_design(P.IIR_REPEATED_POLE, 3, 4.0, 0, ctypes.byref(g), None, 0) == P.OK
    a, b, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    big = 1 << 40
    mixed = (P.Filter * 2)(f, g)
    assert L.fdvm_blur_iir(a, P.F32, 8, 8, 8, b, 8, 64, mixed, 2, 0, ws, big, None) == P.EINVAL
    one = (P.Filter * 1)(f)
    assert L.fdvm_blur_iir_adjoint(a, 8, 8, 8, 64, b, 8, 64, one, 1, 0, ws, big, None) == P.EUNSUPPORTED
    with pytest.raises(P.FdvmError):
        P.iir_designs([2.0], P.BUTTERWORTH, dsigma=True)


def test_noalloc_detect_rejects_sizes_beyond_its_scratch():
    # host-side checks only: nothing reaches a device
    L = P.lib()
    cap_bytes = L.fdvm_noalloc_scratch_bytes()
    assert cap_bytes == 32 << 20
    fake = ctypes.c_void_p(4096)   # never dereferenced: the call fails validation first
    H, W, S = 65535, 16384, 16
    assert P.workspace_bytes(P.OP_DETECT, H, W, S) > cap_bytes
    st = L.fdvm_detect_blobs_noalloc(fake, H, W, W, H * W, S, 0.1, 1, fake, 10, fake, None)
    assert st == P.ERANGE
    # the ordinary argument checks come first
    assert L.fdvm_detect_blobs_noalloc(None, 10, 10, 10, 100, 1, 0.1, 1, fake, 10, fake, None) == P.EINVAL
    assert L.fdvm_detect_blobs_noalloc(fake, 10, 10, 10, 100, 1, -1.0, 1, fake, 10, fake, None) == P.EINVAL
    assert L.fdvm_detect_blobs_noalloc(fake, 10, 10, 10, 100, 0, 0.1, 1, fake, 10, fake, None) == P.EINVAL


def test_batch_validates_every_frame_before_enqueueing():
    # a bad descriptor after good ones: EINVAL on the host, nothing forked
    L = P.lib()
    frames = (P.Frame * 3)()
    for f in frames:
        f.data, f.dtype, f.H, f.W, f.row_chunk, f.pitch = 4096, P.U16, 64, 64, 0, 64
        f.out, f.count, f.cap = 8192, 12288, 10
    frames[2].pitch = 10   # pitch < W
    filt = P.iir_designs([2.0, 4.0])
    st = L.fdvm_batch_detect(frames, 3, filt, 2, P.BC_REPLICATE, 1.0, 1, 2, ctypes.c_void_p(4096), 1 << 40, None)
    assert st == P.EINVAL


def test_backward_validation():
    """Argument checks of the two backward calls, before any device work."""
    L = P.lib()
    fake = ctypes.c_void_p(4096)
    f = (P.Filter * 2)()
    for i, sg in enumerate((2.0, 4.0)):
        assert L.fdvm_filter_design(P.IIR_REPEATED_POLE, 3, sg, 0, ctypes.byref(f[i]), None, 0) == P.OK
    bw = (P.Filter * 1)()
    assert L.fdvm_filter_design(P.IIR_BUTTERWORTH, 4, 4.0, 0, ctypes.byref(bw[0]), None, 0) == P.OK
    big = 1 << 40
    other = ctypes.c_void_p(1 << 20)   # gx must not be gV

    def iir(what=P.GRAD_X, nframes=1, filt=f, S=2, ws=fake, wsb=big, gx=other, gs=fake):
        return L.fdvm_iir_laplacian_backward(fake, P.F32, 16, 16, 16, 256, fake, fake, 16, 256, 512, nframes, filt,
                                             S, 0, what, gx, 16, 256, gs, ws, wsb, None)

    assert iir(what=0) == P.EINVAL
    assert iir(what=4) == P.EINVAL
    assert iir(nframes=0) == P.EINVAL
    assert iir(ws=None) == P.EINVAL
    assert iir(gx=None) == P.EINVAL
    assert iir(gx=fake) == P.EINVAL      # gx overlapping gV
    assert iir(what=P.GRAD_SIGMA, gs=None) == P.EINVAL
    assert iir(filt=bw, S=1) == P.EUNSUPPORTED
    assert iir(wsb=16) == P.ENOMEM
    half = (ctypes.c_int32 * 1)(2)
    off = (ctypes.c_int32 * 1)(0)
    sig = (ctypes.c_double * 1)(1.0)
    sym = (ctypes.c_double * 5)(0.1, 0.2, 0.4, 0.2, 0.1)
    asym = (ctypes.c_double * 5)(0.1, 0.2, 0.4, 0.2, 0.11)

    def fir(taps=sym, dtaps=sym, what=P.GRAD_X, wsb=big, s=sig):
        return L.fdvm_fir_laplacian_backward(fake, P.F32, 16, 16, 16, 256, fake, fake, 16, 256, 256, 1, taps, dtaps,
                                             half, off, s, 1, 0, what, other, 16, 256, fake, fake, wsb, None)

    assert fir(taps=asym) == P.EINVAL
    assert fir(what=P.GRAD_SIGMA, dtaps=None) == P.EINVAL
    assert fir(s=(ctypes.c_double * 1)(-1.0)) == P.ERANGE
    assert fir(wsb=16) == P.ENOMEM
    assert P.workspace_bytes(P.OP_IIR_LAPLACIAN_BACKWARD, 1024, 1024, 4) >= 3 * 4 * 1024 * 1024 * 4
    assert P.workspace_bytes(P.OP_FIR_LAPLACIAN_BACKWARD, 1024, 1024, 4) >= 7 * 1024 * 1024 * 4
