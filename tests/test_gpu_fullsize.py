"""The 928^3 uint8, 6-connected, NL = 6 configuration at full size.

The volume is generated and its gradient quantised on the device; the HIP path
then runs in the launch configuration the benchmark times. Two kinds of check:

* oracle parity: the device's gradient bytes go to the host, where the CPU
  oracle computes the watershed and the NL - 1 waterfall levels, and every
  layer is compared element by element. The whole volume takes the oracle
  about four minutes of one host core (and some 30 GB of host memory), so
  that comparison runs when WS_FULLSIZE_ORACLE=1 is set; by default a
  32-plane slab of the same gradient (27.6 Mvoxel, several thousand tiles)
  is compared instead;
* at full size, with torch operations that share nothing with the library,
  the properties the paper's definitions fix at any size:
  * gradient: the float64 3D Sobel magnitude of the same float volume, quantised
    to 0..255 by its maximum, equals the library's bytes except by one level where
    the unrounded value lies within 2e-5*Q of a rounding boundary;
  * watershed (Alg. 1): every label is canonical (the smallest index of its
    basin: L[p] <= p and L[L[p]] == L[p]), and every voxel with a strictly lower
    neighbour carries the label of its Eq. (1) target (the last of its lowest
    neighbours in index order);
  * Step II (Section 3.3): the distances are the fixpoint of the relaxation,
    checked locally on the stage output: every resolved plateau voxel (balanced
    state -d) has d - 1 as the smallest distance among its equal-grey
    neighbours, and no unresolved voxel (state 2/3, a minimal plateau) has an
    equal-grey neighbour with a finite distance;
  * waterfall (Section 4): every layer is canonical and nested in the previous
    one (L_k[p] == L_k[L_{k-1}[p]]), the returned counts equal the number of
    voxels carrying their own label, and a layer has at most half the regions of
    the previous one while that one has more than one.
"""
from __future__ import annotations

import os
import time

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

SLAB = 48  # z-planes per checking slab


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def blobs928():
    import torch

    import paper_2410_08946_amd as ws

    cfg = gen.CONFIGS["blobs928"]
    shape = tuple(cfg["shape"])
    say("blobs928: generating", shape)
    img = gen.synth.blobs3d_device(shape, seed=cfg["seed"], device="cuda:0")
    ctx = ws.Context(0)
    say("blobs928: gradient")
    mag = torch.empty(shape, dtype=torch.float32, device="cuda:0")
    grad = ctx.gradient(img, 0.0, "u8", mag=mag)
    say("blobs928: watershed")
    lab = ctx.watershed(grad, cfg["conn"])
    say("blobs928: waterfall NL", cfg["NL"])
    out, nreg = ctx.waterfall(lab, grad, cfg["conn"], cfg["NL"])
    torch.cuda.synchronize()
    say("blobs928: regions per layer", nreg.cpu().tolist())
    yield dict(img=img, mag=mag, grad=grad, lab=lab, out=out, nreg=nreg.cpu().tolist(), shape=shape)
    ctx.close()


def _sobel64(img, z0, z1):
    """float64 3D Sobel magnitude of planes [z0, z1) (replicated border)."""
    import torch
    nz = img.shape[0]
    lo = max(0, z0 - 1)
    zi = torch.arange(z0 - 1, z1 + 1, device=img.device).clamp(0, nz - 1) - lo
    a = img[lo:min(nz, z1 + 1)].double()[zi]  # replicated border in z
    a = torch.cat([a[:, :1], a, a[:, -1:]], 1)
    a = torch.cat([a[:, :, :1], a, a[:, :, -1:]], 2)
    w = torch.tensor([1.0, 2.0, 1.0], dtype=torch.float64, device=img.device)

    def sm(x, axis):  # [1, 2, 1] along axis (valid)
        n = x.shape[axis]
        return (w[0] * x.narrow(axis, 0, n - 2) + w[1] * x.narrow(axis, 1, n - 2) + w[2] * x.narrow(axis, 2, n - 2))

    def df(x, axis):  # [-1, 0, 1] along axis (valid)
        n = x.shape[axis]
        return x.narrow(axis, 2, n - 2) - x.narrow(axis, 0, n - 2)

    gx = sm(sm(df(a, 2), 1), 0)
    gy = sm(sm(df(a, 1), 2), 0)
    gz = sm(sm(df(a, 0), 2), 1)
    return torch.sqrt(gx * gx + gy * gy + gz * gz)


def test_blobs928_gradient(blobs928):
    import torch
    img, grad = blobs928["img"], blobs928["grad"]
    nz = img.shape[0]
    mx = 0.0
    for z0 in range(0, nz, SLAB):
        mx = max(mx, float(_sobel64(img, z0, min(nz, z0 + SLAB)).max()))
    assert mx > 0
    Q = 255.0
    bad = 0
    for z0 in range(0, nz, SLAB):
        z1 = min(nz, z0 + SLAB)
        v = _sobel64(img, z0, z1) * Q / mx
        ref = torch.round(v)  # ties to even
        got = grad[z0:z1].double()
        d = (got - ref).abs()
        near = ((v - torch.floor(v)) - 0.5).abs() <= 2e-5 * Q
        bad += int(((d > 1) | ((d == 1) & ~near)).sum())
    assert bad == 0, "%d gradient bytes differ beyond the rounding allowance" % bad
    # the kernel's own rule, exactly: rint(fp32(mag * 255) / max(mag)) in float32
    mag = blobs928["mag"]
    mx32 = np.float32(float(mag.max()))
    off = 0
    for z0 in range(0, nz, SLAB):
        z1 = min(nz, z0 + SLAB)
        m = mag[z0:z1].cpu().numpy()
        rule = np.clip(np.rint((m * np.float32(255.0)) / mx32), 0, 255).astype(np.uint8)
        off += int((rule != grad[z0:z1].cpu().numpy()).sum())
    assert off == 0, "%d bytes do not follow rint(mag*Q/max)" % off


def _canonical(lab_flat, n, chunk=1 << 26):
    import torch
    for p0 in range(0, n, chunk):
        p1 = min(n, p0 + chunk)
        idx = torch.arange(p0, p1, device=lab_flat.device, dtype=torch.int64)
        l = lab_flat[p0:p1].long()
        if not bool((l >= 0).all()) or not bool((l <= idx).all()):
            return False
        if not bool((lab_flat[l].long() == l).all()):
            return False
    return True


def test_blobs928_watershed(blobs928):
    import torch
    lab, grad = blobs928["lab"], blobs928["grad"]
    nz, ny, nx = blobs928["shape"]
    n = nz * ny * nx
    flat = lab.reshape(-1)
    assert _canonical(flat, n)
    # Eq. (1): the last of the lowest neighbours (6-connectivity, index order
    # z-1, y-1, x-1, x+1, y+1, z+1); out-of-image neighbours do not exist
    plane = ny * nx
    offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    big = torch.iinfo(torch.int32).max
    bad = 0
    for z0 in range(0, nz, SLAB):
        z1 = min(nz, z0 + SLAB)
        Z = z1 - z0
        gp = torch.full((Z + 2, ny + 2, nx + 2), big, dtype=torch.int32, device=grad.device)
        lo, hi = max(0, z0 - 1), min(nz, z1 + 1)
        gp[lo - (z0 - 1):hi - (z0 - 1), 1:-1, 1:-1] = grad[lo:hi].int()
        m = torch.full((Z, ny, nx), big, dtype=torch.int32, device=grad.device)
        q = torch.zeros((Z, ny, nx), dtype=torch.int64, device=grad.device)
        p = (torch.arange(z0, z1, device=grad.device).view(-1, 1, 1) * plane +
             torch.arange(ny, device=grad.device).view(1, -1, 1) * nx +
             torch.arange(nx, device=grad.device).view(1, 1, -1))
        for dz, dy, dx in offs:
            v = gp[1 + dz:1 + dz + Z, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
            take = (v <= m) & (v < big)
            m = torch.where(take, v, m)
            q = torch.where(take, p + (dz * plane + dy * nx + dx), q)
        slope = m < grad[z0:z1].int()
        lp = lab[z0:z1][slope].long()
        lq = flat[q[slope]].long()
        bad += int((lp != lq).sum())
        del gp, m, q, p, slope, lp, lq
    assert bad == 0, "%d slope voxels do not share the label of their Eq. (1) target" % bad


def test_blobs928_waterfall(blobs928):
    import torch
    out, nreg = blobs928["out"], blobs928["nreg"]
    nz, ny, nx = blobs928["shape"]
    n = nz * ny * nx
    assert torch.equal(out[0], blobs928["lab"])
    for k in range(out.shape[0]):
        flat = out[k].reshape(-1)
        assert _canonical(flat, n), "layer %d not canonical" % k
        own = 0
        for p0 in range(0, n, 1 << 26):
            p1 = min(n, p0 + (1 << 26))
            own += int((flat[p0:p1].long() == torch.arange(p0, p1, device=flat.device)).sum())
        assert own == nreg[k], "layer %d: %d own labels, %d reported" % (k, own, nreg[k])
        if k > 0:
            prev = out[k - 1].reshape(-1)
            for p0 in range(0, n, 1 << 26):
                p1 = min(n, p0 + (1 << 26))
                assert torch.equal(flat[p0:p1], flat[prev[p0:p1].long()]), "layer %d not nested" % k
            if nreg[k - 1] > 1:
                assert nreg[k] <= nreg[k - 1] // 2


def test_blobs928_step2_fixpoint(blobs928):
    """Step II converged: the local fixpoint conditions on the balanced states."""
    import torch
    import paper_2410_08946_amd as ws
    grad = blobs928["grad"]
    nz, ny, nx = blobs928["shape"]
    ctx = ws.Context(0)
    try:
        bal, _ = ctx.watershed_stages(grad, 6)
        torch.cuda.synchronize()
    finally:
        ctx.close()
    BIG = 1 << 30
    offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    bad_res = bad_min = 0
    for z0 in range(0, nz, SLAB):
        z1 = min(nz, z0 + SLAB)
        Z = z1 - z0
        lo, hi = max(0, z0 - 1), min(nz, z1 + 1)
        gp = torch.full((Z + 2, ny + 2, nx + 2), -1, dtype=torch.int32, device=grad.device)
        dp = torch.full((Z + 2, ny + 2, nx + 2), BIG, dtype=torch.int32, device=grad.device)
        b = bal[lo:hi]
        dist = torch.where(b < 0, -b, torch.where(b == 0, torch.zeros_like(b), torch.full_like(b, BIG)))
        gp[lo - (z0 - 1):hi - (z0 - 1), 1:-1, 1:-1] = grad[lo:hi].int()
        dp[lo - (z0 - 1):hi - (z0 - 1), 1:-1, 1:-1] = dist
        g0 = grad[z0:z1].int()
        b0 = bal[z0:z1]
        m = torch.full((Z, ny, nx), BIG, dtype=torch.int32, device=grad.device)
        for dz, dy, dx in offs:
            gv = gp[1 + dz:1 + dz + Z, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
            dv = dp[1 + dz:1 + dz + Z, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
            m = torch.minimum(m, torch.where(gv == g0, dv, torch.full_like(dv, BIG)))
        res = b0 < 0
        bad_res += int((res & (m != -b0 - 1)).sum())
        unres = (b0 == 2) | (b0 == 3)
        bad_min += int((unres & (m < BIG)).sum())
        del gp, dp, m, dist, b, g0, b0
    assert bad_res == 0 and bad_min == 0, \
        "%d resolved voxels off the fixpoint, %d unresolved voxels next to a finite distance" % (bad_res, bad_min)


def _compare_with_oracle(grad, out, nreg, conn, tag):
    """Layer 0 and every waterfall layer of the HIP path against the oracle on
    the same gradient bytes; the oracle's levels run one at a time (a level
    reads only the previous layer and the gradient)."""
    g = grad.cpu().numpy()
    NL = out.shape[0]
    t = time.time()
    prev = oracle.watershed(g, conn)
    say("%s: oracle watershed %.1f s" % (tag, time.time() - t))
    got = out[0].cpu().numpy()
    bad = int((got != prev).sum())
    assert bad == 0, "%s: layer 0 differs from the oracle at %d voxels" % (tag, bad)
    assert int((prev.reshape(-1) == np.arange(prev.size)).sum()) == nreg[0]
    del got
    for k in range(1, NL):
        t = time.time()
        lay, n = oracle.waterfall_g1(prev, g, conn, 2)
        got = out[k].cpu().numpy()
        bad = int((got != lay[1]).sum())
        say("%s: oracle level %d %.1f s, %d regions, %d voxels differ" % (tag, k, time.time() - t, int(n[1]), bad))
        assert bad == 0, "%s: layer %d differs from the oracle at %d voxels" % (tag, k, bad)
        assert int(n[1]) == nreg[k]
        prev = np.ascontiguousarray(lay[1])
        del lay, got


def test_blobs928_slab_oracle(blobs928):
    """A 32-plane slab of the full volume's gradient (same recipe, same
    bytes): watershed and NL = 6 layers equal the oracle's element by
    element."""
    import torch

    import paper_2410_08946_amd as ws
    z0, z1 = 448, 480
    sub = blobs928["grad"][z0:z1].contiguous()
    ctx = ws.Context(0)
    try:
        lab = ctx.watershed(sub, 6)
        out, nreg = ctx.waterfall(lab, sub, 6, gen.CONFIGS["blobs928"]["NL"])
        torch.cuda.synchronize()
        _compare_with_oracle(sub, out, nreg.cpu().tolist(), 6, "blobs928 slab %d:%d" % (z0, z1))
    finally:
        ctx.close()


@pytest.mark.skipif(os.environ.get("WS_FULLSIZE_ORACLE") != "1",
                    reason="the full 928^3 oracle comparison takes about four minutes of host time "
                           "(set WS_FULLSIZE_ORACLE=1)")
def test_blobs928_full_oracle(blobs928):
    """The whole 928^3 volume: labels of the watershed and of all six layers,
    as the benchmark computes them, equal the oracle's element by element."""
    oracle.set_progress(True)
    try:
        _compare_with_oracle(blobs928["grad"], blobs928["out"], blobs928["nreg"], gen.CONFIGS["blobs928"]["conn"],
                             "blobs928 full")
    finally:
        oracle.set_progress(False)
