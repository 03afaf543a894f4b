"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer stages must match bit for bit on the same quantised bytes; the float32
gradient must stay within 1e-5 of max|oracle| (the oracle is float64), and its
quantised bytes may differ by one level only where the oracle's unrounded
value lies within that tolerance of a rounding boundary.
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
from tests import brute

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_08946_amd as ws
    c = ws.Context(0)
    yield c
    c.close()


def to_dev(a):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).to("cuda:0").view(torch.uint16)
    return torch.from_numpy(a).to("cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


def gpu_ws(ctx, grad, conn):
    say("  watershed", grad.shape, grad.dtype, "conn", conn)
    return to_host(ctx.watershed(to_dev(grad), conn))


def check_ws(ctx, grad, conn):
    got = gpu_ws(ctx, grad, conn)
    ref = oracle.watershed(grad, conn)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError("labels differ at %d pixels, first %s: gpu %s oracle %s" %
                             (len(bad), bad[0].tolist(), got[tuple(bad[0])], ref[tuple(bad[0])]))
    return got


def check_stages(ctx, grad, conn):
    say("  stages", grad.shape, "conn", conn)
    bal, arrow = ctx.watershed_stages(to_dev(grad), conn)
    _, st = oracle.watershed(grad, conn, full=True)
    assert np.array_equal(to_host(bal), st["bal"])
    assert np.array_equal(to_host(arrow), st["arrow"])


def check_wf(ctx, grad, conn, NL):
    import torch
    g = to_dev(grad)
    say("  waterfall", grad.shape, "conn", conn, "NL", NL)
    lab = ctx.watershed(g, conn)
    out, nreg = ctx.waterfall(lab, g, conn, NL)
    ref0 = oracle.watershed(grad, conn)
    ref, refn = oracle.waterfall_g1(ref0, grad, conn, NL)
    assert np.array_equal(to_host(out), ref)
    assert to_host(nreg).tolist() == refn.tolist()
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
def test_tiny_images(ctx):
    for img, conn in [(np.array([[7]], np.uint8), 4), (np.array([[3, 1, 4, 1, 5]], np.uint8), 4),
                      (np.array([[3], [1], [4], [1], [5]], np.uint8), 8), (np.array([[2, 2], [2, 2]], np.uint8), 8),
                      (np.array([[[1]], [[0]]], np.uint8), 6)]:
        check_ws(ctx, img, conn)


@pytest.mark.parametrize("n", [2, 5, 33, 100, 2000])
def test_paper_rows(ctx, n):
    row = gen.paper_row(n)
    lab = check_ws(ctx, row, 4)
    assert lab[0].tolist() == [0] * (n + 1) + [n + 1] * (n + 1)
    check_stages(ctx, row, 4)
    check_ws(ctx, np.ascontiguousarray(row.T), 8)


def test_paper_bal14(ctx):
    row = np.array([[75] + [89] * 12 + [81]], np.uint8)
    bal, arrow = ctx.watershed_stages(to_dev(row), 4)
    assert to_host(bal)[0].tolist() == [1, 0, -1, -2, -3, -4, -5, -5, -4, -3, -2, -1, 0, 1]


@pytest.mark.parametrize("shape", [(7, 9), (32, 64), (33, 65), (64, 130), (100, 37), (1, 300), (300, 1), (97, 203)])
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_random_2d(ctx, shape, conn, dtype):
    rng = np.random.default_rng(hash((shape, conn)) % (2 ** 32))
    for levels in (2, 4, 50):
        img = rng.integers(0, levels, size=shape).astype(dtype)
        check_ws(ctx, img, conn)
        check_stages(ctx, img, conn)


@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 8, 32), (9, 17, 33), (20, 10, 70), (1, 9, 40)])
@pytest.mark.parametrize("conn", [6, 26])
def test_random_3d(ctx, shape, conn):
    if shape[0] == 1:
        conn = 4 if conn == 6 else 8
        shape = shape[1:]
    rng = np.random.default_rng(7)
    for levels in (2, 4, 50):
        img = rng.integers(0, levels, size=shape).astype(np.uint8)
        check_ws(ctx, img, conn)
        check_stages(ctx, img, conn)


def test_volume_recipe_many_tiles(ctx):
    """The 928^3 recipe (blob density, sigma, noise) at 160^3: about 2000
    watershed tiles with the plateau structure of the full volume (a few per
    cent of the voxels on plateaux touching and crossing tile borders), whole
    labels, Step II stages and waterfall against the oracle."""
    import torch
    f = gen.synth.blobs3d_device((160, 160, 160), seed=7, device="cpu").numpy()
    grad = oracle.gradient(f, 0.0, "u8")
    check_ws(ctx, grad, 6)
    check_stages(ctx, grad, 6)
    check_wf(ctx, grad, 6, 4)
    g2 = oracle.gradient(gen.synth.blobs3d_device((72, 96, 120), seed=8, device="cpu").numpy(), 0.0, "u8")
    check_ws(ctx, g2, 26)
    check_stages(ctx, g2, 26)


def test_plateau_structures(ctx):
    check_ws(ctx, gen.serpentine(70, 150), 4)
    check_stages(ctx, gen.serpentine(70, 150), 8)
    check_ws(ctx, np.full((300, 200), 5, np.uint8), 8)
    check_ws(ctx, np.full((20, 40, 70), 9, np.uint16), 6)
    yy, xx = np.mgrid[0:200, 0:300]
    check_ws(ctx, ((yy // 37 + xx // 53) % 3).astype(np.uint8), 4)   # large flat blocks
    zz, yy, xx = np.mgrid[0:24, 0:40, 0:70]
    check_ws(ctx, ((zz // 7 + yy // 9 + xx // 11) % 4).astype(np.uint8), 26)


def test_blob_images_and_waterfall(ctx):
    img = gen.blobs2d(256, 256, seed=0)
    grad = oracle.gradient(img, 0.0, "u8")
    check_ws(ctx, grad, 4)
    check_wf(ctx, grad, 4, 3)
    check_wf(ctx, grad, 8, 8)
    vol = gen.blobs3d(40, 48, 56, seed=2, n_blobs=12, sigma=(3.0, 8.0))
    g3 = oracle.gradient(vol, 0.0, "u8")
    check_ws(ctx, g3, 6)
    check_wf(ctx, g3, 6, 6)
    check_wf(ctx, g3, 26, 4)


@pytest.mark.parametrize("shape,conn", [((45, 61), 4), ((45, 61), 8), ((9, 11, 13), 6), ((9, 11, 13), 26)])
def test_waterfall_random(ctx, shape, conn):
    rng = np.random.default_rng(41)
    for levels in (3, 40, 1000):
        img = rng.integers(0, levels, size=shape).astype(np.uint16)
        check_wf(ctx, img, conn, 12)
    check_wf(ctx, np.full(shape, 4, np.uint8), conn, 3)


def test_waterfall_hash_overflow(ctx):
    """Inputs whose waterfall tiles hold more distinct region pairs and
    regions than the pixel pass's LDS hashes have slots, so that inserts fall
    back to direct slab entries and global keys (Alg. 4 Step V: the lowest
    pass value per pair of adjacent regions must not depend on where a pair
    was recorded; the level passes use the same fallback). A checkerboard of
    zeros and random heights makes every other voxel a minimum: its 16 x 8 x 8
    waterfall tiles hold up to 2560 distinct pairs (1024 edge slots) and 748
    regions (512 region slots), and a 2D one's 64 x 16 tiles up to 1536 pairs
    and 585 regions (counted on the oracle's layer 0); the random heights keep
    hundreds of regions in the later layers. Sizes span several tiles with a
    ragged tail; the batched call takes the same path."""
    import torch
    rng = np.random.default_rng(11)
    zz, yy, xx = np.mgrid[0:20, 0:19, 0:37]
    cb3 = np.where((xx + yy + zz) % 2 == 0, 0, rng.integers(1, 256, xx.shape)).astype(np.uint8)
    yy, xx = np.mgrid[0:37, 0:150]
    cb2 = np.where((xx + yy) % 2 == 0, 0, rng.integers(1, 65536, xx.shape)).astype(np.uint16)
    check_wf(ctx, cb3, 6, 5)
    check_wf(ctx, cb2, 4, 5)
    outs, nreg = ctx.batch([to_dev(cb3), to_dev(cb3[:9])], [6, 6], 4)
    torch.cuda.synchronize()
    for grad, o, n in zip((cb3, cb3[:9]), outs, nreg):
        wf, wn = oracle.waterfall_g1(oracle.watershed(grad, 6), grad, 6, 4)
        assert np.array_equal(to_host(o), wf) and to_host(n).tolist() == wn.tolist()


def test_schedule_invariance(ctx):
    img = gen.blobs2d(300, 280, seed=5)
    grad = oracle.gradient(img, 0.0, "u8")
    ref = oracle.watershed(grad, 8)
    serp = gen.serpentine(66, 130)
    ref_s = oracle.watershed(serp, 4)
    try:
        for step3 in (0, 1):
            for rr in (1, 2, 6):
                for batch in (1, 3, 32):
                    ctx.set_option("step3", step3)
                    ctx.set_option("rr", rr)
                    ctx.set_option("sweep_batch", batch)
                    assert np.array_equal(gpu_ws(ctx, grad, 8), ref)
                    assert np.array_equal(gpu_ws(ctx, serp, 4), ref_s)
    finally:
        ctx.set_option("step3", 0)
        ctx.set_option("rr", 6)
        ctx.set_option("sweep_batch", 4)


def _check_gradient(ctx, img, sigma, dtype, offset=0):
    """offset > 0 places the magnitude and the output `offset` elements into
    their allocations (buffers not aligned for vector accesses)."""
    import torch
    say("  gradient", img.shape, "sigma", sigma, dtype, "offset", offset)
    q_ref, mag_ref = oracle.gradient(img, sigma, dtype, return_mag=True)
    d_img = torch.from_numpy(img).to("cuda:0")
    n = img.size
    mag = torch.empty(n + offset, dtype=torch.float32, device="cuda:0")[offset:].view(img.shape)
    qt = torch.uint8 if dtype == "u8" else torch.uint16
    out = torch.empty(n + offset, dtype=qt, device="cuda:0")[offset:].view(img.shape)
    q = ctx.gradient(d_img, sigma, dtype, out=out, mag=mag)
    m = to_host(mag).astype(np.float64)
    mx = mag_ref.max()
    assert np.abs(m - mag_ref).max() <= GRAD_RTOL * mx
    Q = 255 if dtype == "u8" else 65535
    qh = to_host(q).astype(np.int64)
    # the kernel's rounding rule, exactly, on the magnitude it returned:
    # rint(fp32(mag * Q) / max(mag)) in float32, ties to even
    m32 = to_host(mag).astype(np.float32)
    mx32 = m32.max()
    if mx32 > 0:
        rule = np.rint((m32 * np.float32(Q)) / mx32).astype(np.int64)
    else:
        rule = np.zeros(m32.shape, np.int64)
    assert np.array_equal(qh, np.clip(rule, 0, Q)), "quantised bytes do not follow rint(mag*Q/max)"
    # against the oracle: the magnitudes agree to GRAD_RTOL * max, so a byte
    # may differ by one level only where the oracle's unrounded value lies
    # within GRAD_RTOL * Q (plus float32 rounding) of a .5 boundary
    exact = mag_ref * Q / mx if mx > 0 else np.zeros_like(mag_ref)
    dq = np.abs(qh - q_ref.astype(np.int64))
    near = np.abs(exact - np.floor(exact) - 0.5) <= GRAD_RTOL * Q + 1e-6 * Q
    assert dq.max() <= 1
    assert (dq[~near] == 0).all()
    say("  gradient bytes differing from the oracle: %d of %d (near a boundary: %d)" %
        (int((dq != 0).sum()), dq.size, int(near.sum())))
    return to_host(q)


@pytest.mark.parametrize("Q,dtype", [(255, "u8"), (65535, "u16")])
def test_gradient_quantisation_ties(ctx, Q, dtype):
    """Magnitudes that scale exactly onto k + 1/2 (the fixture's Sobel values
    are exact in float32) are rounded half to even by the quantisation kernel."""
    import torch
    from tests.quant_fixture import tie_image
    img, mag_exact, expect = tie_image(Q)
    mag = torch.empty(img.shape, dtype=torch.float32, device="cuda:0")
    q = ctx.gradient(torch.from_numpy(img).to("cuda:0"), 0.0, dtype, mag=mag)
    assert np.array_equal(to_host(mag).astype(np.float64), mag_exact)
    assert np.array_equal(to_host(q).astype(np.int64), expect)


def test_gradient(ctx):
    rng = np.random.default_rng(13)
    _check_gradient(ctx, gen.blobs2d(256, 256, seed=0), 0.0, "u8")
    _check_gradient(ctx, (rng.normal(0, 100, (61, 77)) + 500).astype(np.float32), 1.0, "u16")
    _check_gradient(ctx, (rng.normal(0, 100, (61, 77)) + 500).astype(np.float32), 2.5, "u8")
    _check_gradient(ctx, gen.blobs3d(30, 34, 38, seed=4, n_blobs=8, sigma=(3.0, 6.0)), 0.0, "u8")
    _check_gradient(ctx, (rng.normal(0, 10, (17, 19, 23))).astype(np.float32), 1.0, "u16")
    _check_gradient(ctx, (rng.normal(0, 10, (1, 300))).astype(np.float32), 1.0, "u16")
    _check_gradient(ctx, np.full((20, 30), 3.0, np.float32), 1.0, "u8")
    # 3D Sobel slabs of 16 planes and 64 x 4 columns: several slabs, partial
    # columns, a single row, a thin volume; unaligned magnitudes and outputs
    for shape, dt, off in [((33, 9, 70), "u8", 0), ((40, 13, 130), "u16", 0), ((2, 5, 7), "u8", 0),
                           ((17, 1, 65), "u16", 0), ((20, 6, 67), "u8", 1), ((19, 5, 33), "u16", 3)]:
        _check_gradient(ctx, (rng.normal(0, 10, shape) + 40).astype(np.float32), 0.0, dt, offset=off)
    _check_gradient(ctx, (rng.normal(0, 100, (61, 77)) + 500).astype(np.float32), 1.0, "u8", offset=1)


def test_argument_errors(ctx):
    import torch
    import paper_2410_08946_amd as ws
    g = torch.zeros((16, 16), dtype=torch.uint8, device="cuda:0")
    for conn in (0, 5, 6, 26):
        with pytest.raises(ws.WSError) as e:
            ctx.watershed(g, conn)
        assert e.value.code == ws.binding.WS_EINVAL
    g3 = torch.zeros((4, 16, 16), dtype=torch.uint8, device="cuda:0")
    for conn in (4, 8):
        with pytest.raises(ws.WSError):
            ctx.watershed(g3, conn)
    lab = ctx.watershed(g, 4)
    with pytest.raises(ws.WSError):
        ctx.waterfall(lab, g, 4, 0)
    with pytest.raises(ws.WSError):
        ctx.set_option("no_such_option", 1)
    # the Step II sweep cap surfaces as WS_ENOCONV (a plateau crossing tiles)
    ctx.set_option("max_sweeps", 1)
    try:
        with pytest.raises(ws.WSError) as e:
            ctx.watershed(to_dev(gen.serpentine(70, 150)), 4)
        assert e.value.code == ws.binding.WS_ENOCONV
    finally:
        ctx.set_option("max_sweeps", 2 ** 31 - 1)
    check_ws(ctx, gen.serpentine(70, 150), 4)


def test_ellipses4096_full_size(ctx):
    """4096 x 4096 u16, blur sigma 1 + Sobel, 8-conn, NL = 6: every stage
    compared in full with the oracle, in the launch configuration of the
    benchmark."""
    import torch
    img = gen.config_image("ellipses4096")
    q = _check_gradient(ctx, img, 1.0, "u16")
    grad = oracle.gradient(img, 1.0, "u16")
    say("  ellipses4096 watershed + waterfall")
    g = to_dev(grad)
    lab = ctx.watershed(g, 8)
    out, nreg = ctx.waterfall(lab, g, 8, 6)
    ref0 = oracle.watershed(grad, 8)
    ref, refn = oracle.waterfall_g1(ref0, grad, 8, 6)
    assert np.array_equal(to_host(lab), ref0)
    assert np.array_equal(to_host(out), ref)
    assert to_host(nreg).tolist() == refn.tolist()
    # the bench feeds the GPU's own quantised gradient forward: its labels are
    # those of the oracle on the same bytes
    g2 = to_dev(q)
    lab2 = ctx.watershed(g2, 8)
    assert np.array_equal(to_host(lab2), oracle.watershed(q, 8))
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
# Batched path: every image of an uneven batch equals the oracle (and the
# single-image calls) bit for bit.
# --------------------------------------------------------------------------

def _batch_case(ctx, grads, conn, NL):
    say("  batch", len(grads), "images conn", conn, "NL", NL)
    outs, nregs = ctx.batch([to_dev(g) for g in grads], conn, NL)
    for g, o, n in zip(grads, outs, nregs):
        ref0 = oracle.watershed(g, conn)
        ref, refn = oracle.waterfall_g1(ref0, g, conn, NL)
        assert np.array_equal(to_host(o), ref)
        assert to_host(n).tolist() == refn.tolist()
    return outs


def test_batch_2d_uneven(ctx):
    rng = np.random.default_rng(77)
    grads = []
    for i in range(24):
        ny, nx = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        if i % 3 == 0:
            img = gen.blobs2d(max(ny, 8), max(nx, 8), seed=100 + i)
            grads.append(oracle.gradient(img, 0.0, "u8"))
        else:
            grads.append(rng.integers(0, 1 + i % 7, size=(ny, nx)).astype(np.uint8))
    _batch_case(ctx, grads, 8, 4)
    _batch_case(ctx, grads, 4, 3)


def test_batch_with_largest_batch_image(ctx):
    """An image at the largest side of the uneven batch (2048^2, the blob
    recipe) batched with small ones equals the oracle."""
    grads = [oracle.gradient(gen.blobs2d(2048, 2048, seed=3777), 0.0, "u8"),
             oracle.gradient(gen.blobs2d(130, 1900, seed=3778), 0.0, "u8"),
             oracle.gradient(gen.blobs2d(128, 128, seed=3779), 0.0, "u8")]
    _batch_case(ctx, grads, 8, 4)


def test_batch_matches_single_calls(ctx):
    rng = np.random.default_rng(5)
    grads = [rng.integers(0, 30, size=(int(rng.integers(20, 200)), int(rng.integers(20, 200)))).astype(np.uint16)
             for _ in range(9)]
    outs = _batch_case(ctx, grads, 8, 5)
    for g, o in zip(grads, outs):
        d = to_dev(g)
        lab = ctx.watershed(d, 8)
        single, _ = ctx.waterfall(lab, d, 8, 5)
        assert np.array_equal(to_host(single), to_host(o))


def test_batch_3d_and_plateaux(ctx):
    rng = np.random.default_rng(9)
    grads = [rng.integers(0, 4, size=(int(rng.integers(2, 20)), int(rng.integers(2, 20)), int(rng.integers(2, 40))))
             .astype(np.uint8) for _ in range(7)]
    grads.append(np.full((9, 10, 70), 3, np.uint8))
    _batch_case(ctx, grads, 6, 4)
    _batch_case(ctx, grads, 26, 3)
    serp = [gen.serpentine(66, 130), gen.serpentine(9, 12), np.full((40, 70), 2, np.uint16)]
    _batch_case(ctx, serp, 4, 3)


def test_batch_mixed_connectivities(ctx):
    """One ws_batch call over 2D 4- and 8-connected and 3D 6- and 26-connected
    images, interleaved: every image equals the oracle."""
    import torch
    rng = np.random.default_rng(41)
    items = []
    for i in range(14):
        kind = i % 4
        if kind == 0:
            g = oracle.gradient(gen.blobs2d(int(rng.integers(30, 200)), int(rng.integers(30, 200)), seed=900 + i),
                                0.0, "u8")
            items.append((g, 8))
        elif kind == 1:
            s3 = tuple(int(v) for v in rng.integers(3, 40, size=3))
            items.append((rng.integers(0, 5, size=s3).astype(np.uint8), 6))
        elif kind == 2:
            items.append((rng.integers(0, 4, size=(int(rng.integers(1, 90)), int(rng.integers(1, 90))))
                          .astype(np.uint8), 4))
        else:
            s3 = tuple(int(v) for v in rng.integers(2, 25, size=3))
            items.append((rng.integers(0, 6, size=s3).astype(np.uint8), 26))
    items.append((oracle.gradient(gen.blobs3d(128, 128, 128, seed=4_100_777, n_blobs=13), 0.0, "u8"), 6))
    items.append((oracle.gradient(gen.blobs2d(512, 512, seed=4_000_777), 0.0, "u8"), 8))
    NL = 4
    say("  mixed batch", len(items), "images")
    outs, nregs = ctx.batch([to_dev(g) for g, _ in items], [c for _, c in items], NL)
    for (g, c), o, n in zip(items, outs, nregs):
        ref, refn = oracle.waterfall_g1(oracle.watershed(g, c), g, c, NL)
        assert np.array_equal(to_host(o), ref), (g.shape, c)
        assert to_host(n).tolist() == refn.tolist()
    torch.cuda.synchronize()


def test_scratch_budget():
    """ws_create's scratch budget: a call whose scratch exceeds it returns
    WS_ENOMEM and writes nothing; calls that fit still run and equal the
    oracle."""
    import torch

    import paper_2410_08946_amd as ws
    small = oracle.gradient(gen.blobs2d(64, 80, seed=3), 0.0, "u8")
    big = np.zeros((1500, 1500), np.uint8)
    c = ws.Context(0, scratch_budget=4 << 20)
    try:
        g = to_dev(big)
        lab = torch.full(big.shape, -7, dtype=torch.int32, device="cuda:0")
        with pytest.raises(ws.WSError) as e:
            c.watershed(g, 4, out=lab)
        assert e.value.code == ws.binding.WS_ENOMEM
        torch.cuda.synchronize()
        assert bool((lab == -7).all())  # nothing was launched
        with pytest.raises(ws.WSError) as e:
            c.batch([g, to_dev(small)], 8, 3)
        assert e.value.code == ws.binding.WS_ENOMEM
        d = to_dev(small)
        lab = c.watershed(d, 8)
        out, n = c.waterfall(lab, d, 8, 3)
        ref, refn = oracle.waterfall_g1(oracle.watershed(small, 8), small, 8, 3)
        assert np.array_equal(to_host(out), ref) and to_host(n).tolist() == refn.tolist()
    finally:
        c.close()


def test_batch_errors(ctx):
    import torch
    import paper_2410_08946_amd as ws
    g = torch.zeros((16, 16), dtype=torch.uint8, device="cuda:0")
    g3 = torch.zeros((4, 16, 16), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ws.WSError):
        ctx.batch([g, g3], 8, 3)          # 8-connectivity on a volume
    with pytest.raises(ws.WSError):
        ctx.batch([g, g3], [8, 4], 3)
    with pytest.raises(ws.WSError):
        ctx.batch([g], 8, 0)
    with pytest.raises(ValueError):
        ctx.batch([g, g3], [8], 3)        # one connectivity per image
    with pytest.raises(ValueError):
        ctx.batch([], 8, 3)


# --------------------------------------------------------------------------
# Serving: jobs admitted while others run, micro-batched across slots; every
# result equals the job run alone.
# --------------------------------------------------------------------------

def test_serving_mix_identity(ctx):
    """Jobs of the serving mix (2D 8-connected and 3D 6-connected, including
    the smallest sizes of the served workload, 512^2 and 128^3) give the
    oracle's layers when served in a mix, and the same as when run alone."""
    import torch
    from paper_2410_08946_amd import serve
    rng = np.random.default_rng(21)
    jobs_in = []
    for i in range(40):
        if i % 3 == 2:
            s = int(rng.integers(8, 40))
            g = rng.integers(0, 5, size=(int(rng.integers(2, 12)), s, s + 3)).astype(np.uint8)
            jobs_in.append((g, 6))
        else:
            ny, nx = int(rng.integers(16, 300)), int(rng.integers(16, 300))
            g = oracle.gradient(gen.blobs2d(ny, nx, seed=500 + i), 0.0, "u8")
            jobs_in.append((g, 8))
    # the served workload's content at its smallest sizes: the 2D blob recipe
    # (32 blobs, 1 % salt) at 512^2 and the volume recipe's blob density at 128^3
    jobs_in.insert(7, (oracle.gradient(gen.blobs2d(512, 512, seed=4_000_123), 0.0, "u8"), 8))
    jobs_in.insert(20, (oracle.gradient(gen.blobs3d(128, 128, 128, seed=4_100_123, n_blobs=13), 0.0, "u8"), 6))
    say("  serving mix: %d jobs, %d voxels" % (len(jobs_in), sum(g.size for g, _ in jobs_in)))
    devs = [(to_dev(g), c) for g, c in jobs_in]
    solo = []
    for (g, c), (d, _) in zip(jobs_in, devs):
        lab = ctx.watershed(d, c)
        out, n = ctx.waterfall(lab, d, c, 4)
        solo.append((to_host(out), to_host(n)))
        ref, refn = oracle.waterfall_g1(oracle.watershed(g, c), g, c, 4)
        assert np.array_equal(solo[-1][0], ref) and solo[-1][1].tolist() == refn.tolist()
    srv = serve.Server(slots=3, budget_bytes=1 << 30, max_batch_jobs=6)
    try:
        jobs = [srv.submit(serve.Job(grad=d, conn=c, NL=4, jid=k)) for k, (d, c) in enumerate(devs)]
        assert srv.drain(timeout=120)
    finally:
        srv.close()
    for j, (o, n) in zip(jobs, solo):
        assert j.error is None, j.error
        assert np.array_equal(to_host(j.out), o)
        assert to_host(j.nregions).tolist() == n.tolist()
    assert srv.batches >= 2
    # a job larger than the whole budget is rejected without harming the rest
    srv2 = serve.Server(slots=2, budget_bytes=8 << 20)
    try:
        big = srv2.submit(serve.Job(grad=to_dev(np.zeros((1000, 1000), np.uint8)), conn=8))
        small = srv2.submit(serve.Job(grad=devs[0][0], conn=devs[0][1]))
        assert srv2.drain(timeout=60)
    finally:
        srv2.close()
    assert big.error is not None and small.error is None
    assert np.array_equal(to_host(small.out), solo[0][0])


def test_reserve_covers_padded_and_ragged_batches():
    """reserve_pixels(n): later ws_batch calls of up to n pixels allocate
    nothing, also when the images' 64-pixel alignment pads the batch past n
    (a lone image of n - 5 pixels) and for a ragged mix of 2D and 3D batches;
    the results equal those of a context that allocates as it goes."""
    import torch

    import paper_2410_08946_amd as ws
    rng = np.random.default_rng(33)
    n = 2053 * 2043 + 5  # the lone image pads to 2^22 > n
    res, ref = ws.Context(0), ws.Context(0)
    try:
        res.set_option("reserve_pixels", n)
        a0 = res.stats()["allocations"]
        say("  reserved", n, "pixels with", a0, "allocations")
        batches = [[(gen.blobs2d(2043, 2053, seed=61), 8)]]
        sides = []
        while sum(a * b for a, b in sides) < n - 400 * 400:
            sides.append((int(rng.integers(300, 500)), int(rng.integers(300, 500))))
        batches.append([(gen.blobs2d(a, b, seed=70 + k), 8) for k, (a, b) in enumerate(sides[:-1])])
        vols, tot = [], 0
        while True:
            s = tuple(int(v) for v in rng.integers(100, 140, size=3))
            if tot + s[0] * s[1] * s[2] > n:
                break
            tot += s[0] * s[1] * s[2]
            vols.append(s)
        batches.append([(rng.integers(0, 60, size=s).astype(np.uint8), 6) for s in vols])
        for bi, items in enumerate(batches):
            grads = []
            for g, conn in items:
                if g.dtype != np.uint8:
                    g = oracle.gradient(g, 0.0, "u8")
                grads.append(to_dev(g))
            conn = items[0][1]
            say("  batch", bi, "images", len(grads), "pixels", sum(int(g.numel()) for g in grads))
            outs = [torch.empty((4,) + tuple(g.shape), dtype=torch.int32, device="cuda:0") for g in grads]
            nregs = [torch.zeros(4, dtype=torch.int64, device="cuda:0") for _ in grads]
            res.batch(grads, conn, 4, outs=outs, nregions=nregs)
            torch.cuda.synchronize()
            assert res.stats()["allocations"] == a0, "batch %d allocated" % bi
            for k in (0, len(grads) - 1):
                lab = ref.watershed(grads[k], conn)
                o, nr = ref.waterfall(lab, grads[k], conn, 4)
                assert np.array_equal(to_host(outs[k]), to_host(o))
                assert to_host(nregs[k]).tolist() == to_host(nr).tolist()
    finally:
        res.close()
        ref.close()


def test_graph_replay_matches_direct():
    """Launch graphs (option "graph"): the same calls on the same buffers, with
    the buffers' contents changed between calls and eager work between the
    replays, give exactly the direct path's results on every replay."""
    import torch

    import paper_2410_08946_amd as ws
    gctx, dctx = ws.Context(0), ws.Context(0)
    gctx.set_option("graph", 1)
    ny, nx, conn, NL = 300, 280, 8, 4
    dev = "cuda:0"
    bufs = {}
    for name, c in (("g", gctx), ("d", dctx)):
        bufs[name] = dict(img=torch.empty((ny, nx), dtype=torch.float32, device=dev),
                          grad=torch.empty((ny, nx), dtype=torch.uint8, device=dev),
                          out=torch.empty((NL, ny, nx), dtype=torch.int32, device=dev),
                          nreg=torch.zeros(NL, dtype=torch.int64, device=dev))
    imgs = [gen.blobs2d(ny, nx, seed=s) for s in (5, 6, 7)]
    try:
        for rep in range(6):
            im = torch.from_numpy(imgs[rep % 3]).to(dev)
            res = {}
            for name, c in (("g", gctx), ("d", dctx)):
                b = bufs[name]
                b["img"].copy_(im)
                c.gradient(b["img"], 0.0, "u8", out=b["grad"])
                c.watershed(b["grad"], conn, out=b["out"][0])
                c.waterfall(b["out"][0], b["grad"], conn, NL, out=b["out"], nregions=b["nreg"])
                torch.cuda.synchronize()
                res[name] = (b["grad"].cpu().numpy(), b["out"].cpu().numpy(), b["nreg"].cpu().numpy())
            say("  graph replay round", rep, "replays so far", gctx.stats().get("graph_replays"))
            for a, d in zip(res["g"], res["d"]):
                assert np.array_equal(a, d)
            float((im * 2).sum())  # eager work between replays
            torch.cuda.synchronize()
        assert gctx.stats()["graph_replays"] >= 6  # gradient + waterfall replayed from the third round on
        lab = oracle.watershed(res["d"][0], conn)
        wf, n = oracle.waterfall_g1(lab, res["d"][0], conn, NL)
        assert np.array_equal(res["g"][1], wf) and np.array_equal(res["g"][2], n)
    finally:
        gctx.close()
        dctx.close()


def _long_plateau(ny, nx, dtype=np.uint8):
    """One non-minimal plateau covering the image, drained through its corner
    pixel: Step II needs about one sweep per tile along the longest geodesic."""
    g = np.full((ny, nx), 9, dtype=dtype)
    g[0, 0] = 8
    return g


def test_graph_watershed_sweep_fallback():
    """ws_watershed under the graph option: replays of the captured call (a
    fixed number of Step II sweeps) equal the direct path; when the buffer's
    new contents need more sweeps than the graph holds, the call runs directly
    and the next identical call is captured again."""
    import torch

    import paper_2410_08946_amd as ws
    gctx = ws.Context(0)
    gctx.set_option("graph", 1)
    ny, nx, conn = 257, 700, 8
    grad = torch.empty((ny, nx), dtype=torch.uint8, device="cuda:0")
    lab = torch.empty((ny, nx), dtype=torch.int32, device="cuda:0")
    blob = oracle.gradient(gen.blobs2d(ny, nx, seed=11), 0.0, "u8")
    flat = _long_plateau(ny, nx)
    refs = {"blob": oracle.watershed(blob, conn), "flat": oracle.watershed(flat, conn)}
    try:
        for rep, name in enumerate(["blob"] * 4 + ["flat"] * 4 + ["blob", "flat"]):
            grad.copy_(to_dev(blob if name == "blob" else flat))
            gctx.watershed(grad, conn, out=lab)
            got = to_host(lab)
            st = gctx.stats()
            say("  round", rep, name, "replays", st["graph_replays"], "sweeps", st["sweeps_launched"])
            assert np.array_equal(got, refs[name]), "round %d (%s) differs from the oracle" % (rep, name)
            float(grad.float().sum())  # eager work between replays
            torch.cuda.synchronize()
        assert gctx.stats()["graph_replays"] >= 4
    finally:
        gctx.close()


def test_batch_graph_replay():
    """ws_batch under the graph option (one graph launch per call once
    captured): mixed 4/8-connected images whose contents change between calls,
    one change needing more Step II sweeps than the graph holds; every call
    equals the direct context's output, and the last one the oracle's."""
    import torch

    import paper_2410_08946_amd as ws
    gctx, dctx = ws.Context(0), ws.Context(0)
    gctx.set_option("graph", 1)
    dev = "cuda:0"
    shapes, conns, NL = [(200, 310), (130, 129), (257, 640)], [8, 4, 8], 4
    blobs = [[oracle.gradient(gen.blobs2d(ny, nx, seed=100 * r + i), 0.0, "u8") for i, (ny, nx) in enumerate(shapes)]
             for r in range(2)]
    flat = _long_plateau(*shapes[2])
    grads = [torch.empty(s, dtype=torch.uint8, device=dev) for s in shapes]
    outs = {k: [torch.empty((NL,) + s, dtype=torch.int32, device=dev) for s in shapes] for k in "gd"}
    nreg = {k: [torch.zeros(NL, dtype=torch.int64, device=dev) for _ in shapes] for k in "gd"}
    try:
        plan = [0, 1, 0, 1, "flat", "flat", "flat", 0]
        for rep, what in enumerate(plan):
            host = list(blobs[0 if what == "flat" else what])
            if what == "flat":
                host[2] = flat
            for g, h in zip(grads, host):
                g.copy_(to_dev(h))
            gctx.batch(grads, conns, NL, outs=outs["g"], nregions=nreg["g"])
            dctx.batch(grads, conns, NL, outs=outs["d"], nregions=nreg["d"])
            torch.cuda.synchronize()
            st = gctx.stats()
            say("  batch round", rep, what, "replays", st["graph_replays"], "sweeps", st["sweeps_launched"])
            for i in range(len(shapes)):
                assert torch.equal(outs["g"][i], outs["d"][i]), "round %d image %d differs" % (rep, i)
                assert torch.equal(nreg["g"][i], nreg["d"][i])
            float(grads[0].float().sum())  # eager work between replays
            torch.cuda.synchronize()
        assert gctx.stats()["graph_replays"] >= 4
        for i, h in enumerate(host):
            lab = oracle.watershed(h, conns[i])
            ref, refn = oracle.waterfall_g1(lab, h, conns[i], NL)
            assert np.array_equal(to_host(outs["g"][i]), ref)
            assert to_host(nreg["g"][i]).tolist() == refn.tolist()
    finally:
        gctx.close()
        dctx.close()


def check_recon(ctx, grad, conn, NL):
    import torch
    say("  recon", grad.shape, grad.dtype, "conn", conn, "NL", NL)
    ref, nref = oracle.waterfall_recon(grad, conn, NL)
    g = to_dev(grad)
    lab = ctx.watershed(g, conn)
    out, n = ctx.waterfall_recon(lab, g, conn, NL)
    got = to_host(out)
    for k in range(NL):
        if not np.array_equal(got[k], ref[k]):
            bad = np.argwhere(got[k] != ref[k])
            raise AssertionError("recon layer %d differs at %d pixels, first %s" % (k, len(bad), bad[0].tolist()))
    assert np.array_equal(to_host(n), nref)
    torch.cuda.synchronize()


def test_recon_fixture(ctx):
    # the 1x8 row where the reconstruction splits old region 4 (not nested)
    row = np.array([[0, 4, 0, 2, 9, 1, 6, 3]], np.uint8)
    import torch
    g = to_dev(row)
    lab = ctx.watershed(g, 4)
    out, n = ctx.waterfall_recon(lab, g, 4, 3)
    got = to_host(out)
    assert got[0].tolist() == [[0, 1, 1, 1, 4, 4, 4, 7]]
    assert got[1].tolist() == [[0, 0, 0, 0, 0, 5, 5, 5]]
    check_recon(ctx, row, 4, 3)


@pytest.mark.parametrize("conn", [4, 8])
def test_recon_blobs_2d(ctx, conn):
    img = gen.blobs2d(200, 230, seed=11)
    check_recon(ctx, oracle.gradient(img, 0.0, "u8"), conn, 5)
    check_recon(ctx, oracle.gradient(gen.ellipses2d(160, 170, seed=3, n_ellipses=40), 1.0, "u16"), conn, 4)


def test_recon_random_and_3d(ctx):
    rng = np.random.default_rng(12)
    check_recon(ctx, rng.integers(0, 6, size=(90, 110)).astype(np.uint8), 8, 6)
    vol = oracle.gradient(gen.blobs3d(40, 44, 48, seed=4, n_blobs=12), 0.0, "u8")
    check_recon(ctx, vol, 6, 4)
    check_recon(ctx, vol, 26, 4)
    check_recon(ctx, np.full((33, 40), 7, np.uint8), 4, 3)


def check_rag(ctx, labels, grad, conn):
    import torch
    say("  rag", labels.shape, "conn", conn)
    a, b, h = ctx.rag(to_dev(np.ascontiguousarray(labels, np.int32)), to_dev(grad), conn)
    got = list(zip(to_host(a).tolist(), to_host(b).tolist(), to_host(h).tolist()))
    ref = sorted((x, y, w) for (x, y), w in brute.rag(labels, grad, conn).items())
    assert got == ref, "rag differs: %d vs %d edges" % (len(got), len(ref))
    torch.cuda.synchronize()


def test_rag_export(ctx):
    img = gen.blobs2d(64, 70, seed=21)
    grad = oracle.gradient(img, 0.0, "u8")
    for conn in (4, 8):
        lab = oracle.watershed(grad, conn)
        check_rag(ctx, lab, grad, conn)
        wf, _ = oracle.waterfall_g1(lab, grad, conn, 4)
        for k in (1, 3):
            check_rag(ctx, wf[k], grad, conn)
    vol = oracle.gradient(gen.blobs3d(14, 15, 16, seed=6, n_blobs=6), 0.0, "u8")
    for conn in (6, 26):
        check_rag(ctx, oracle.watershed(vol, conn), vol, conn)
    const = np.full((20, 30), 3, np.uint8)
    check_rag(ctx, oracle.watershed(const, 4), const, 4)  # one region, no edge
