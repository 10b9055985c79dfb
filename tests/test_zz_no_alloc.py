"""fdvm_detect_blobs_noalloc against fdvm_detect_blobs, through the C ABI: the
same records and counts from the fixed scratch array as from a caller
workspace, over consecutive calls whose sizes shrink (the array keeps the
previous call's words)."""

import ctypes

import numpy as np
import pytest

from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1912_07133_amd")


def _planes(S, H, W, seed):
    # smooth-ish random planes: many strict extrema of both signs
    g = torch.Generator(device="cuda").manual_seed(seed)
    v = torch.randn((S, H, W), generator=g, device="cuda", dtype=torch.float32)
    return torch.nn.functional.avg_pool2d(v[:, None], 3, stride=1, padding=1)[:, 0].contiguous()


def _run(V, tau, border, cap, noalloc):
    S, H, W = V.shape
    L = P.lib()
    out = torch.zeros(max(cap, 1) * P.BLOB_BYTES, dtype=torch.uint8, device=V.device)
    cnt = torch.full((1,), -7, dtype=torch.int32, device=V.device)
    stream = P._stream_ptr(V.device)
    if noalloc:
        st = L.fdvm_detect_blobs_noalloc(V.data_ptr(), H, W, V.stride(1), V.stride(0), S, float(tau), border,
                                         out.data_ptr(), cap, cnt.data_ptr(), stream)
    else:
        need = P.workspace_bytes(P.OP_DETECT, H, W, S)
        ws = torch.empty(need, dtype=torch.uint8, device=V.device)
        st = L.fdvm_detect_blobs(V.data_ptr(), H, W, V.stride(1), V.stride(0), S, float(tau), border,
                                 out.data_ptr(), cap, cnt.data_ptr(), ws.data_ptr(), need, stream)
    assert st == P.OK, P.status_string(st)
    torch.cuda.synchronize()
    n = int(cnt.item())
    return n, out[: min(n, cap) * P.BLOB_BYTES].cpu().numpy().tobytes()


def test_noalloc_matches_workspace_call_over_shrinking_sizes():
    # largest first (close to the biggest batch frame: 3072 rows x 4096 columns
    # x 12 scales, 19.8 MB of scratch), then smaller inputs that reuse the array
    cases = [(12, 3072, 4096, 0.05, 1, 1 << 22), (8, 700, 900, 0.05, 2, 1 << 20), (1, 256, 256, 0.1, 1, 1 << 16),
             (3, 5, 70, 0.0, 0, 64)]
    for (S, H, W, tau, border, cap) in cases:
        say(f"case: noalloc detect S={S} H={H} W={W} tau={tau} border={border}")
        need = P.workspace_bytes(P.OP_DETECT, H, W, S)
        assert need <= P.lib().fdvm_noalloc_scratch_bytes()
        V = _planes(S, H, W, seed=S * 1000 + H)
        n_ref, rec_ref = _run(V, tau, border, cap, noalloc=False)
        n_got, rec_got = _run(V, tau, border, cap, noalloc=True)
        assert n_got == n_ref
        assert rec_got == rec_ref
        assert n_ref > 0 or (S, H, W) == (3, 5, 70)


def test_noalloc_overflow_count_and_repeat():
    # a capacity below the count: both calls write the true count and the first cap records
    V = _planes(4, 300, 333, seed=5)
    say("case: noalloc overflow 4x300x333")
    n_ref, rec_ref = _run(V, 0.02, 1, 17, noalloc=False)
    for _ in range(2):
        n_got, rec_got = _run(V, 0.02, 1, 17, noalloc=True)
        assert n_ref > 17 and n_got == n_ref and rec_got == rec_ref
