"""Tile shapes and the autotuner against the CPU oracle.

Block size and the reduction rate change only the time of the method, never
its result (Section 3.4, last paragraph; Section 5, parameters paragraph).
Every watershed tile shape of the library (options "tile2d" / "tile3d") and
every setting the autotuner may choose must therefore give the oracle's
labels bit for bit, on inputs that span several tiles of each shape with a
ragged tail, need many Step II sweeps, or overflow a tile's plateau list.
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


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


def _cases_2d():
    rng = np.random.default_rng(5)
    flat = np.full((130, 700), 9, np.uint8)
    flat[0, 0] = 8                                          # one plateau, many sweeps, whole-tile relaxation
    yy, xx = np.mgrid[0:150, 0:260]
    return [
        (oracle.gradient(gen.blobs2d(300, 281, seed=3), 0.0, "u8"), 8),
        (rng.integers(0, 3, size=(200, 333)).astype(np.uint16), 4),   # plateau-heavy: long lists
        (rng.integers(0, 40, size=(97, 203)).astype(np.uint8), 8),
        (flat, 8),
        (((yy // 37 + xx // 53) % 3).astype(np.uint8), 4),            # large flat blocks
        (np.full((70, 90), 4, np.uint8), 8),                          # one minimal plateau
    ]


def _cases_3d():
    rng = np.random.default_rng(6)
    zz, yy, xx = np.mgrid[0:24, 0:40, 0:70]
    vol = gen.synth.blobs3d_device((72, 60, 90), seed=9, device="cpu").numpy()
    return [
        (oracle.gradient(vol, 0.0, "u8"), 6),
        (oracle.gradient(vol, 0.0, "u8"), 26),
        (rng.integers(0, 3, size=(20, 37, 45)).astype(np.uint8), 6),
        (((zz // 7 + yy // 9 + xx // 11) % 4).astype(np.uint8), 26),
        (np.full((18, 33, 40), 7, np.uint16), 6),
    ]


def _check_shape(opt, shape, cases, NL=4):
    import torch

    import paper_2410_08946_amd as ws
    ctx = ws.Context(0)
    ctx.set_option(opt, shape)
    try:
        for i, (grad, conn) in enumerate(cases):
            say("  %s=%d case %d %s conn %d" % (opt, shape, i, grad.shape, conn))
            g = to_dev(grad)
            lab = ctx.watershed(g, conn)
            ref = oracle.watershed(grad, conn)
            got = to_host(lab)
            assert np.array_equal(got, ref), "case %d: %d labels differ" % (i, int((got != ref).sum()))
            bal, arrow = ctx.watershed_stages(g, conn)
            _, st = oracle.watershed(grad, conn, full=True)
            assert np.array_equal(to_host(bal), st["bal"]) and np.array_equal(to_host(arrow), st["arrow"])
            if i < 2:
                out, n = ctx.waterfall(lab, g, conn, NL)
                wf, wn = oracle.waterfall_g1(ref, grad, conn, NL)
                assert np.array_equal(to_host(out), wf) and to_host(n).tolist() == wn.tolist()
        # one batched call over the cases of one grey type
        grey = cases[0][0].dtype
        sel = [(g, c) for g, c in cases if g.dtype == grey]
        outs, nreg = ctx.batch([to_dev(g) for g, _ in sel], [c for _, c in sel], NL)
        torch.cuda.synchronize()
        for (grad, conn), o, n in zip(sel, outs, nreg):
            wf, wn = oracle.waterfall_g1(oracle.watershed(grad, conn), grad, conn, NL)
            assert np.array_equal(to_host(o), wf) and to_host(n).tolist() == wn.tolist()
    finally:
        ctx.close()


@pytest.mark.parametrize("shape", [2, 12, 22, 32])
def test_tile_shapes_2d(shape):
    _check_shape("tile2d", shape, _cases_2d())


@pytest.mark.parametrize("shape", [3, 13, 23, 33])
def test_tile_shapes_3d(shape):
    _check_shape("tile3d", shape, _cases_3d())


def test_tile_shape_option_errors():
    import paper_2410_08946_amd as ws
    ctx = ws.Context(0)
    try:
        for opt, bad in (("tile2d", 3), ("tile2d", 0), ("tile3d", 2), ("tile3d", 43)):
            with pytest.raises(ws.WSError):
                ctx.set_option(opt, bad)
    finally:
        ctx.close()


def test_autotune_choices_match_oracle(tmp_path):
    """The autotuner times candidate settings, checks each candidate's labels
    against the default setting's, caches its choice by (dimensionality, grey
    type, connectivity, size class) and applies a cached choice without
    timing; the chosen settings give the oracle's labels."""
    import torch

    import paper_2410_08946_amd as ws
    from paper_2410_08946_amd import autotune
    cache = str(tmp_path / "tune.json")
    ctx = ws.Context(0)
    try:
        g2 = oracle.gradient(gen.blobs2d(512, 512, seed=4), 0.0, "u8")
        g3 = oracle.gradient(gen.synth.blobs3d_device((64, 80, 96), seed=5, device="cpu").numpy(), 0.0, "u8")
        for grad, conn in ((g2, 8), (g3, 6)):
            r = autotune.tune_watershed(ctx, to_dev(grad), conn, reps=2, cache=cache)
            say("  tuned", r["key"], r["options"], r["ms"], "ms,", len(r["candidates"]), "candidates")
            assert not r["cached"] and len(r["candidates"]) >= 6
            assert np.array_equal(to_host(ctx.watershed(to_dev(grad), conn)), oracle.watershed(grad, conn))
            r2 = autotune.tune_watershed(ctx, to_dev(grad), conn, cache=cache)
            assert r2["cached"] and r2["options"] == r["options"]
        imgs = [oracle.gradient(gen.synth.batch_image(i), 0.0, "u8") for i in range(6)]
        rb = autotune.tune_batch(ctx, [to_dev(g) for g in imgs], 8, 4, reps=1, cache=cache)
        say("  tuned", rb["key"], rb["options"])
        outs, nreg = ctx.batch([to_dev(g) for g in imgs], 8, 4)
        torch.cuda.synchronize()
        for g, o, n in zip(imgs, outs, nreg):
            wf, wn = oracle.waterfall_g1(oracle.watershed(g, 8), g, 8, 4)
            assert np.array_equal(to_host(o), wf) and to_host(n).tolist() == wn.tolist()
    finally:
        ctx.close()


_TILE = {2: (64, 32, 1), 12: (128, 16, 1), 22: (32, 32, 1), 32: (64, 64, 1),
         3: (32, 8, 8), 13: (16, 16, 8), 23: (32, 16, 8), 33: (16, 16, 16)}


def _peaks(shape_zyx, tile_xyz, shift):
    """Grey values that fall with the L1 distance from the centre of every
    tile-sized cell of a grid offset by `shift` (shift 0: the cells are the
    tiles, so the lowest values lie on the tile seams)."""
    nz, ny, nx = shape_zyx
    tx, ty, tz = tile_xyz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.abs((x + shift) % tx - (tx - 1) / 2.0) + np.abs((y + shift) % ty - (ty - 1) / 2.0)
    if nz > 1:
        d = d + np.abs((z + shift) % tz - (tz - 1) / 2.0)
    return np.clip(np.rint(200.0 - 4.0 * d), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("shape", [2, 32, 3, 33])
def test_tile_scale_structure(shape):
    """Tile-scale structure: peaks at the tile centres (minimal plateaux
    where the tiles' corners meet, arrows along the faces) and on a shifted
    grid (valleys and exits inside and across tiles), at every tile shape's
    own size, with both connectivities. Every crossing a tile records must
    reach the global merge: labels equal the oracle's (Sections 3.1-3.2)."""
    import paper_2410_08946_amd as ws
    tx, ty, tz = _TILE[shape]
    ndim = 3 if tz > 1 else 2
    dims = (2 * tz + 3, 2 * ty + 1, 2 * tx + 5) if ndim == 3 else (1, 3 * ty + 1, 2 * tx + 5)
    ctx = ws.Context(0)
    ctx.set_option("tile3d" if ndim == 3 else "tile2d", shape)
    try:
        for shift in (0, 3):
            grad = _peaks(dims, (tx, ty, tz), shift)
            if ndim == 2:
                grad = grad[0]
            for conn in ((6, 26) if ndim == 3 else (4, 8)):
                say("  shape %d shift %d conn %d %s" % (shape, shift, conn, grad.shape))
                got = to_host(ctx.watershed(to_dev(grad), conn))
                ref = oracle.watershed(grad, conn)
                assert np.array_equal(got, ref), "%d labels differ" % int((got != ref).sum())
    finally:
        ctx.close()
