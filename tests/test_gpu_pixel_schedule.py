"""The per-pixel synchronous schedule (Section 3.3, with the PRUF / APRUF Step
III of Section 3.2 and the PRW Step IV of Alg. 2) against the CPU oracle.

Every variant must give the oracle's labels and Step II stage arrays bit for
bit; the Step II sweep count on the paper's (2n+2)-pixel row must be the n
iterations Section 3.3 derives for the synchronous implementation.
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
from tests.test_gpu_parity import say, to_dev, to_host

pytestmark = pytest.mark.gpu

# (step3, step4): APRUF_sync, PRUF_sync, PRW_sync (PRUF Step III + Alg. 2), APRUF + Alg. 2
VARIANTS = [(0, 0), (1, 0), (1, 1), (0, 1)]


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_08946_amd as ws
    c = ws.Context(0)
    c.set_option("schedule", 1)
    yield c
    c.close()


@pytest.fixture(params=VARIANTS, ids=["aprufsync", "prufsync", "prwsync", "apruf_prw"])
def px(ctx, request):
    step3, step4 = request.param
    ctx.set_option("step3", step3)
    ctx.set_option("step4", step4)
    yield ctx
    ctx.set_option("step3", 0)
    ctx.set_option("step4", 0)


def check(ctx, grad, conn, stages=False):
    say("  per-pixel watershed", grad.shape, grad.dtype, "conn", conn)
    got = to_host(ctx.watershed(to_dev(grad), conn))
    ref, st = oracle.watershed(grad, conn, full=True)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError("labels differ at %d pixels, first %s: gpu %s oracle %s" %
                             (len(bad), bad[0].tolist(), got[tuple(bad[0])], ref[tuple(bad[0])]))
    if stages:
        bal, arrow = ctx.watershed_stages(to_dev(grad), conn)
        assert np.array_equal(to_host(bal), st["bal"])
        assert np.array_equal(to_host(arrow), st["arrow"])
    return got


def test_tiny_and_rows(px):
    for img, conn in [(np.array([[7]], np.uint8), 4), (np.array([[3, 1, 4, 1, 5]], np.uint8), 4),
                      (np.array([[3], [1], [4], [1], [5]], np.uint8), 8), (np.array([[2, 2], [2, 2]], np.uint8), 8),
                      (np.array([[[1]], [[0]]], np.uint8), 6)]:
        check(px, img, conn, stages=True)
    for n in (2, 5, 33, 100):
        row = gen.paper_row(n)
        lab = check(px, row, 4, stages=True)
        assert lab[0].tolist() == [0] * (n + 1) + [n + 1] * (n + 1)
        check(px, np.ascontiguousarray(row.T), 8)


@pytest.mark.parametrize("shape", [(7, 9), (33, 65), (100, 37), (1, 300), (97, 203)])
@pytest.mark.parametrize("conn", [4, 8])
def test_random_2d(px, shape, conn):
    rng = np.random.default_rng(1000 * shape[0] + shape[1] + conn)
    for levels, dtype in ((3, np.uint8), (40, np.uint16), (256, np.uint8)):
        check(px, rng.integers(0, levels, size=shape).astype(dtype), conn, stages=levels == 3)


@pytest.mark.parametrize("conn", [6, 26])
def test_random_3d(px, conn):
    rng = np.random.default_rng(conn)
    for shape in ((5, 6, 7), (9, 17, 33), (2, 9, 40)):
        for levels in (2, 5, 300):
            check(px, rng.integers(0, levels, size=shape).astype(np.uint16), conn, stages=levels == 2)


def test_plateaux_and_blobs(px):
    check(px, gen.serpentine(30, 60), 4, stages=True)
    check(px, np.full((50, 70), 5, np.uint8), 8)
    check(px, np.full((8, 10, 12), 9, np.uint16), 6)
    yy, xx = np.mgrid[0:120, 0:150]
    check(px, ((yy // 37 + xx // 53) % 3).astype(np.uint8), 4)
    zz, yy, xx = np.mgrid[0:16, 0:30, 0:40]
    check(px, ((zz // 7 + yy // 9 + xx // 11) % 4).astype(np.uint8), 26)
    grad = oracle.gradient(gen.blobs2d(256, 256, seed=0), 0.0, "u8")
    check(px, grad, 8, stages=True)
    g3 = oracle.gradient(gen.blobs3d(40, 48, 56, seed=2, n_blobs=12, sigma=(3.0, 8.0)), 0.0, "u8")
    check(px, g3, 6)
    check(px, g3, 26)


@pytest.mark.parametrize("n", [2, 5, 12, 40])
def test_paper_row_sweep_count(ctx, n):
    """Section 3.3: the (2n+2)-pixel row needs n synchronous iterations of Step
    II, the last of which changes nothing."""
    ctx.set_option("sweep_batch", 1)
    try:
        check(ctx, gen.paper_row(n), 4)
        st = ctx.stats()
        assert st["sweeps_launched"] - 1 == n      # minus the Step I pass
        assert st["sweeps_changing"] == n - 1
    finally:
        ctx.set_option("sweep_batch", 4)


def test_prw_passes_and_caps(ctx):
    import paper_2410_08946_amd as ws
    # a comb-shaped minimal plateau: every tooth ends in a state-3 pixel, so
    # Step III leaves one label per tooth and the PRW passes must merge them
    comb = np.full((40, 64), 5, np.uint8)
    comb[0, :] = 1
    comb[:, ::7] = 1
    ctx.set_option("step3", 1)
    ctx.set_option("step4", 1)
    try:
        check(ctx, comb, 4)
        assert ctx.stats()["step4_passes"] >= 1
        ctx.set_option("max_sweeps", 3)
        with pytest.raises(ws.WSError):
            ctx.watershed(to_dev(gen.paper_row(20)), 4)
    finally:
        ctx.set_option("max_sweeps", 2**31 - 1)
        ctx.set_option("step3", 0)
        ctx.set_option("step4", 0)


def test_prw_needs_per_pixel_schedule():
    import paper_2410_08946_amd as ws
    c = ws.Context(0)
    try:
        c.set_option("step4", 1)
        with pytest.raises(ws.WSError):
            c.watershed(to_dev(np.zeros((4, 4), np.uint8)), 4)
        c.set_option("schedule", 1)
        assert to_host(c.watershed(to_dev(np.zeros((4, 4), np.uint8)), 4)).max() == 0
    finally:
        c.close()


def test_recipe_images(ctx):
    """The 256^2 recipe and a 96^3 cube at the volume recipe's blob density,
    every variant against the oracle."""
    cases = [(oracle.gradient(gen.blobs2d(256, 256, seed=0), 0.0, "u8"), 4),
             (oracle.gradient(gen.blobs3d(96, 96, 96, seed=2, n_blobs=6), 0.0, "u8"), 6)]
    try:
        for grad, conn in cases:
            ref = oracle.watershed(grad, conn)
            for step3, step4 in VARIANTS:
                ctx.set_option("step3", step3)
                ctx.set_option("step4", step4)
                say("  recipe", grad.shape, conn, step3, step4)
                assert np.array_equal(to_host(ctx.watershed(to_dev(grad), conn)), ref)
    finally:
        ctx.set_option("step3", 0)
        ctx.set_option("step4", 0)
