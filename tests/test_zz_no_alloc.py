"""ws_watershed_noalloc (through the C ABI) against ws_watershed: the
allocation-free entry point gives the same labels on two calls in a row, the
second with a smaller input of another dimensionality, allocates nothing, and
rejects an image whose scratch exceeds its fixed area."""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_noalloc_matches_watershed():
    import torch

    import paper_2410_08946_amd as ws
    big = oracle.gradient(gen.blobs2d(700, 913, seed=21), 0.0, "u8")                     # 2D, 8-connected
    small = oracle.gradient(gen.synth.blobs3d_device((40, 50, 61), seed=22, device="cpu").numpy(), 0.0, "u8")
    ref_ctx = ws.Context(0)
    ctx = ws.Context(0)   # fresh: it has allocated nothing
    try:
        for grad, conn in ((big, 8), (small, 6)):
            g = _dev(grad)
            want = ref_ctx.watershed(g, conn)
            out = torch.full(g.shape, -7, dtype=torch.int32, device="cuda:0")
            ctx.watershed_noalloc(g, conn, out)
            torch.cuda.synchronize()
            print("  noalloc", grad.shape, "conn", conn, flush=True)
            assert torch.equal(out, want)
            assert np.array_equal(out.cpu().numpy(), oracle.watershed(grad, conn))
        assert ctx.stats()["allocations"] == 0
        # a second context shares the same fixed area; the result stays the same
        ctx2 = ws.Context(0)
        try:
            g = _dev(big)
            out = torch.empty(g.shape, dtype=torch.int32, device="cuda:0")
            ctx2.watershed_noalloc(g, 8, out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref_ctx.watershed(g, 8))
            assert ctx2.stats()["allocations"] == 0
        finally:
            ctx2.close()
        # scratch beyond the fixed area: rejected before any launch
        huge = torch.zeros((6000, 6000), dtype=torch.uint8, device="cuda:0")
        lab = torch.full((6000, 6000), -7, dtype=torch.int32, device="cuda:0")
        with pytest.raises(ws.WSError) as ei:
            ctx.watershed_noalloc(huge, 8, lab)
        assert ei.value.code == ws.binding.WS_EINVAL and "fixed area" in str(ei.value)
        torch.cuda.synchronize()
        assert int((lab != -7).sum()) == 0
        assert ctx.stats()["allocations"] == 0
    finally:
        ctx.close()
        ref_ctx.close()
