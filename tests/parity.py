"""Helpers shared by the parity tests: tolerances, the fragile-decision rule
for detection sets, and torch/device plumbing.  No filter arithmetic here:
expected values always come from the oracle."""

from __future__ import annotations

import sys

import numpy as np

# Float32 tolerance of the blur planes: max |B_gpu - B_ref| <= RTOL_BLUR * max |B_ref|
# (normwise per plane; 1e-5 relative in float32).
RTOL_BLUR = 1e-5

# Laplacian planes V = sigma^2 (D20 + D02): the 5-point stencil has gain 8, so
# a float32 blur correct to a few units in the last place perturbs V by up to
# 8 sigma^2 * (a few ulp of max |B|).  Tolerance: 4 ulps (2^-22 relative).
ULPS_V = 4 * 2.0 ** -24


def laplacian_tolerance(sigma, B_ref_plane):
    return 8.0 * sigma * sigma * ULPS_V * float(np.max(np.abs(B_ref_plane)))


def say(*args):
    """Print and flush: names the case before each GPU step."""
    print(*args, flush=True)
    sys.stdout.flush()


def normwise_error(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(np.max(np.abs(ref)), 1e-300)
    return float(np.max(np.abs(got - ref)) / scale)


def assert_planes_close(got, ref, rtol=RTOL_BLUR, what="plane"):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    if got.ndim == 2:
        got, ref = got[None], ref[None]
    for s in range(got.shape[0]):
        err = normwise_error(got[s], ref[s])
        assert err <= rtol, f"{what} {s}: normwise error {err:.3e} > {rtol:.1e}"


def neighbour_extremes(V):
    """min and max of the existing 3x3x3 neighbours (excluding the centre)."""
    V = np.asarray(V, dtype=np.float64)
    S, H, W = V.shape
    lo = np.full(V.shape, np.inf)
    hi = np.full(V.shape, -np.inf)
    for ds in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if ds == dy == dx == 0:
                    continue
                sh = np.full(V.shape, np.nan)
                s0, s1 = max(0, -ds), min(S, S - ds)
                y0, y1 = max(0, -dy), min(H, H - dy)
                x0, x1 = max(0, -dx), min(W, W - dx)
                sh[s0:s1, y0:y1, x0:x1] = V[s0 + ds:s1 + ds, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
                ok = ~np.isnan(sh)
                lo = np.where(ok, np.minimum(lo, sh), lo)
                hi = np.where(ok, np.maximum(hi, sh), hi)
    return lo, hi


def fragile_mask(V_ref, errs, tau):
    """Decisions that an error of at most errs[s] per plane could flip: the
    threshold test (||v| - tau| <= e) or the strict-extremum comparison (gap to
    the nearest competing neighbour <= 2 max(e_s, e_s-1, e_s+1))."""
    V = np.asarray(V_ref, dtype=np.float64)
    S = V.shape[0]
    e = np.asarray(errs, dtype=np.float64)
    e_nb = np.array([max(e[max(s - 1, 0):s + 2]) for s in range(S)])[:, None, None]
    e_s = e[:, None, None]
    lo, hi = neighbour_extremes(V)
    thr = (np.abs(np.abs(V) - tau) <= e_s)
    # a pixel that fails the threshold by more than e in both results can
    # never be a detection, whatever its neighbours do
    cand = np.abs(V) >= tau - e_s
    ext = (np.abs(lo - V) <= 2 * e_nb) | (np.abs(V - hi) <= 2 * e_nb)
    return thr | (cand & ext)


def blob_keys(blobs):
    return [(int(b["scale"]), int(b["y"]), int(b["x"]), int(b["polarity"])) for b in blobs]


def compare_detections(got, ref, V_ref, V_got, tau, border=1, v_bound=None):
    """Compares a GPU detection list `got` (from the planes V_got) with the
    oracle's list `ref` (from V_ref).  Returns (number of fragile decisions,
    mismatches); the caller asserts that the mismatches are [].

    * Outside the fragile set (decisions that an error of at most the measured
      max |V_got - V_ref| of each plane could flip) the two lists must agree
      exactly: (scale, y, x, polarity).
    * Inside it neither list is held to the other's decisions, but the GPU list
      must still be valid for its own planes: the whole GPU list must equal
      the oracle's extremum rule applied to V_got (in float64, tau rounded to
      float32 as the kernels compare it).  Entries that break this are
      reported as ("invalid", s, y, x, polarity) or ("missing", ...).
    * v_bound (optional, per plane): an a-priori bound on |V_got - V_ref|.  The
      measured errors size the fragile set, so they must not exceed it
      (reported as ("bound", s, error, bound)).
    Ordering of `got` must already be (scale, y, x)."""
    S = V_ref.shape[0]
    errs = [float(np.max(np.abs(np.asarray(V_got[s], np.float64) - V_ref[s]))) for s in range(S)]
    frag = fragile_mask(V_ref, errs, tau)
    g = set(blob_keys(got))
    r = set(blob_keys(ref))
    keep = lambda k: not frag[k[0], k[1], k[2]]  # noqa: E731
    g2 = {k for k in g if keep(k)}
    r2 = {k for k in r if keep(k)}
    mism = sorted(g2 ^ r2)
    from oracle import shape
    own = set(blob_keys(shape.detect_extrema(np.asarray(V_got, np.float64), float(np.float32(tau)), border)))
    mism += [("invalid",) + k for k in sorted(g - own)] + [("missing",) + k for k in sorted(own - g)]
    if v_bound is not None:
        mism += [("bound", s, errs[s], float(v_bound[s])) for s in range(S) if not errs[s] <= v_bound[s]]
    return int(frag.sum()), mism


def torch_cuda():
    import torch
    return torch


def keys_equal_ok(got, ref) -> bool:
    """Exact equality of the (scale, y, x, polarity) lists, in order."""
    return blob_keys(got) == blob_keys(ref)
