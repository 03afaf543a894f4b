"""Pins of the CPU oracle against the paper and against independent definitions.

The oracle is checked here against: the worked examples the paper prints
(tests/golden/), brute-force re-definitions on exhaustive tiny inputs
(tests/brute.py), Meyer priority flooding on distinct-valued images, and
invariants on random inputs dominated by plateaux.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
import pytest

import oracle
from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=", 1)
            vals[k] = [int(t) for t in v.split()]
    return vals


# --------------------------------------------------------------------------
# Worked examples printed in the paper
# --------------------------------------------------------------------------

def test_paper_row_sync_example():
    """Section 3.3: states, sweep count and fair split of the (2n+2)x1 row."""
    g = _golden("paper_row_sync.txt")
    row = np.array([g["row"]], np.uint16)
    n = g["n"][0]
    lab, st = oracle.watershed(row, 4, full=True)
    assert st["state1"][0].tolist() == g["state1"]
    assert st["sweeps"] == g["sweeps"][0] == n
    assert st["arrow"][0].tolist() == g["arrows"]
    _, st2 = oracle.watershed(row, 4, max_step2_sweeps=n - 2, full=True)
    states = np.where(st2["bal"][0] < 0, 0, st2["bal"][0])
    assert states.tolist() == g["state_after_n_minus_2"]
    assert lab[0].tolist() == [0] * (n + 1) + [n + 1] * (n + 1)


@pytest.mark.parametrize("n", [2, 3, 4, 7, 10, 33])
def test_paper_row_sync_general_n(n):
    """Same example for other n: n sweeps, 1 0 2..2 0 1, half/half split."""
    from gen import paper_row
    row = paper_row(n)
    lab, st = oracle.watershed(row, 4, full=True)
    assert st["state1"][0].tolist() == [1, 0] + [2] * (2 * n - 2) + [0, 1]
    assert st["sweeps"] == n
    _, st2 = oracle.watershed(row, 4, max_step2_sweeps=n - 2, full=True)
    states = np.where(st2["bal"][0] < 0, 0, st2["bal"][0]).tolist()
    assert states == [1] + [0] * (n - 1) + [2, 2] + [0] * (n - 1) + [1]
    assert lab[0].tolist() == [0] * (n + 1) + [n + 1] * (n + 1)


def test_paper_row_bal14_example():
    """Section 3.4: the converged balanced (negative-distance) states."""
    g = _golden("paper_row_bal14.txt")
    row = np.array([g["row"]], np.uint16)
    lab, st = oracle.watershed(row, 4, full=True)
    assert st["bal"][0].tolist() == g["bal"]
    assert lab[0].tolist() == [0] * 7 + [7] * 7


def test_path_reduction_iterations():
    """Figure on path reduction: length 22, RR = 2 -> 3 iterations."""
    g = _golden("path_reduction.txt")
    L, RR = g["length"][0], g["RR"][0]
    row = np.arange(L + 1, dtype=np.uint16)[None, :]
    lab, st = oracle.watershed(row, 4, RR=RR, full=True)
    assert st["syncs"] == g["iterations"][0] == math.ceil(math.log(L, RR + 1))
    assert (lab == 0).all()


@pytest.mark.parametrize("RR", [1, 2, 3, 6])
def test_path_reduction_log_bound(RR):
    """Step III: ceil(log_{RR+1} Len) synchronisations for a path of Len arrows."""
    for L in list(range(1, 60)) + [100, 343, 344, 1000]:
        row = np.arange(L + 1, dtype=np.uint16)[None, :]
        _, st = oracle.watershed(row, 4, RR=RR, full=True)
        k = 0
        while (RR + 1) ** k < L:
            k += 1
        assert st["syncs"] == k, (L, RR)


def test_one_dimensional_minimal_plateaux_have_one_state3_pixel():
    """Section 3.1 (1D remark): in 1D every minimal plateau has exactly one
    state-3 pixel, its rightmost one, so Steps I-III already give the result."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        row = rng.integers(0, 4, size=(1, n)).astype(np.uint16)
        lab, st = oracle.watershed(row, 4, full=True)
        I = row[0].astype(int)
        bal = st["bal"][0]
        # minimal plateaux = maximal runs of equal value with no lower neighbour
        i = 0
        while i < n:
            j = i
            while j + 1 < n and I[j + 1] == I[i]:
                j += 1
            lower = (i > 0 and I[i - 1] < I[i]) or (j + 1 < n and I[j + 1] < I[i])
            if not lower and j > i:
                s = bal[i:j + 1].tolist()
                assert s.count(3) == 1 and s[-1] == 3 and all(v == 2 for v in s[:-1])
            i = j + 1


# --------------------------------------------------------------------------
# Exhaustive tiny inputs against the brute-force drop walk
# --------------------------------------------------------------------------

def _exhaustive(shape, values):
    n = int(np.prod(shape))
    for t in itertools.product(values, repeat=n):
        yield np.array(t, np.uint16).reshape(shape)


@pytest.mark.parametrize("shape,values,conns", [
    ((1, 7), range(4), (4, 8)),
    ((3, 3), range(3), (4, 8)),
    ((2, 4), range(3), (4, 8)),
    ((3, 4), range(2), (4, 8)),
    ((2, 2, 2), range(3), (6, 26)),
])
def test_exhaustive_vs_drop_walk(shape, values, conns):
    for img in _exhaustive(shape, values):
        for conn in conns:
            got = oracle.watershed(img, conn)
            ref = brute.drop_watershed(img, conn)
            if not np.array_equal(got, ref):
                raise AssertionError("mismatch conn=%d img=%s\n%s\n%s" % (conn, img.tolist(), got, ref))


@pytest.mark.parametrize("shape,conn", [((9, 11), 4), ((9, 11), 8), ((5, 4, 6), 6), ((5, 4, 6), 26)])
def test_random_plateaux_vs_drop_walk(shape, conn):
    rng = np.random.default_rng(11)
    for trial in range(40):
        img = rng.integers(0, 3 + trial % 3, size=shape).astype(np.uint16)
        assert np.array_equal(oracle.watershed(img, conn), brute.drop_watershed(img, conn))


@pytest.mark.parametrize("shape,conn", [((8, 8), 4), ((8, 8), 8), ((4, 4, 4), 6), ((4, 4, 4), 26),
                                        ((1, 40), 4), ((13, 7), 8)])
def test_distinct_values_vs_meyer_flooding(shape, conn):
    rng = np.random.default_rng(3)
    n = int(np.prod(shape))
    for _ in range(30):
        img = rng.permutation(n).astype(np.uint16).reshape(shape)
        assert np.array_equal(oracle.watershed(img, conn), brute.meyer_flood(img, conn))


# --------------------------------------------------------------------------
# Invariants on larger random inputs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,conn", [((48, 40), 4), ((48, 40), 8), ((12, 10, 9), 6), ((12, 10, 9), 26)])
def test_watershed_invariants(shape, conn):
    rng = np.random.default_rng(17)
    img = rng.integers(0, 4, size=shape).astype(np.uint16)
    lab, st = oracle.watershed(img, conn, full=True)
    L = lab.reshape(-1)
    I = img.reshape(-1).astype(int)
    nb = brute.nbrs(shape, conn)
    n = L.size
    # canonical: label = smallest index of its class, every pixel labelled
    assert (L >= 0).all() and (L < n).all()
    for lbl in np.unique(L):
        assert np.flatnonzero(L == lbl).min() == lbl
    # one regional minimum per basin, as many basins as regional minima
    zone = brute.flat_zones(list(I), nb)
    minimal = brute.regional_minima(list(I), nb, zone)
    assert len(np.unique(L)) == len(minimal) == st["nbasins"]
    per_basin = {}
    for p in range(n):
        if zone[p] in minimal:
            per_basin.setdefault(int(L[p]), set()).add(zone[p])
    assert all(len(v) == 1 for v in per_basin.values()) and len(per_basin) == len(minimal)
    # each basin connected
    for lbl in np.unique(L):
        members = set(np.flatnonzero(L == lbl).tolist())
        start = next(iter(members))
        seen, stack = {start}, [start]
        while stack:
            p = stack.pop()
            for q in nb[p]:
                if q in members and q not in seen:
                    seen.add(q)
                    stack.append(q)
        assert seen == members
    # steepest descent consistency on slope pixels (Eq. (1))
    for p in range(n):
        low = min(I[q] for q in nb[p]) if nb[p] else None
        if low is not None and low < I[p]:
            q = max(q for q in nb[p] if I[q] == low)
            assert L[p] == L[q]
    # plateau distances equal breadth-first-search distances
    d = brute.plateau_distance(list(I), nb, zone, minimal)
    bal = st["bal"].reshape(-1)
    for p in range(n):
        if d[p] is not None and d[p] > 0:
            assert bal[p] == -d[p]


def test_special_cases():
    one = np.array([[7]], np.uint16)
    assert oracle.watershed(one, 4).tolist() == [[0]]
    const = np.full((17, 23), 5, np.uint16)
    assert (oracle.watershed(const, 8) == 0).all()
    const3 = np.full((4, 5, 6), 2, np.uint16)
    assert (oracle.watershed(const3, 6) == 0).all()
    # a single pit: everything drains into it
    yy, xx = np.mgrid[0:21, 0:21]
    pit = ((yy - 10) ** 2 + (xx - 10) ** 2).astype(np.uint16)
    lab = oracle.watershed(pit, 8)
    assert (lab == 0).all()
    # Eq. (1) tie rule: of two equally low neighbours the later one is taken
    col = np.array([[3], [1], [4], [1], [5]], np.uint16)
    assert oracle.watershed(col, 4).reshape(-1).tolist() == [0, 0, 2, 2, 2]


def test_serpentine_plateau_distance():
    from gen import serpentine
    img = serpentine(9, 12)
    lab, st = oracle.watershed(img, 4, full=True)
    assert (lab == 0).all()
    assert -st["bal"].min() >= 30


# --------------------------------------------------------------------------
# Graph waterfall
# --------------------------------------------------------------------------

def test_waterfall_fixture_1x8():
    """Hand-derived fixture: I = 0 4 0 2 9 1 6 3 (neighbours +-x).
    Watershed basins {0} {1,2,3} {4,5,6} {7}; lowest passes 0:(4, via 1),
    1:(4, via 0), 4:(6, via 7), 7:(6, via 4); so layer 1 joins {0,1} and
    {4,7}; layer 2 joins the two (pass height 9 between 3 and 4 being the
    only boundary)."""
    I = np.array([[0, 4, 0, 2, 9, 1, 6, 3]], np.uint16)
    lab = oracle.watershed(I, 4)
    assert lab[0].tolist() == [0, 1, 1, 1, 4, 4, 4, 7]
    out, nr = oracle.waterfall_g1(lab, I, 4, 3)
    assert out[1, 0].tolist() == [0, 0, 0, 0, 4, 4, 4, 4]
    assert out[2, 0].tolist() == [0] * 8
    assert nr.tolist() == [4, 2, 1]
    # the reconstruction form (Alg. 4 + re-watershed) splits old region 4
    rec, nr2 = oracle.waterfall_recon(I, 4, 2)
    assert rec[1, 0].tolist() == [0, 0, 0, 0, 0, 5, 5, 5]


def _waterfall_by_rag(lab0, img, conn, NL):
    """Independent graph waterfall: per level, contract the level-0 region
    adjacency graph by the previous layer, take each region's lowest edge
    (ties: smaller neighbour label), join along those edges with scipy's
    connected components, relabel by the smallest label."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    w = brute.rag(lab0, img, conn)
    layers = [lab0.reshape(-1).copy()]
    chosen_total = []
    cur_of = {int(l): int(l) for l in np.unique(lab0)}
    for _ in range(1, NL):
        best = {}
        for (a, b), h in w.items():
            A, B = cur_of[a], cur_of[b]
            if A == B:
                continue
            for X, Y in ((A, B), (B, A)):
                if X not in best or (h, Y) < best[X]:
                    best[X] = (h, Y)
        regs = sorted(set(cur_of.values()))
        pos = {r: i for i, r in enumerate(regs)}
        rows = [pos[x] for x in best]
        cols = [pos[best[x][1]] for x in best]
        g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(len(regs), len(regs)))
        ncomp, comp = connected_components(g, directed=True, connection="weak")
        newlab = {}
        for r in regs:
            c = comp[pos[r]]
            newlab[c] = min(newlab.get(c, r), r)
        edges = {(min(x, best[x][1]), max(x, best[x][1])): best[x][0] for x in best}
        chosen_total.append(sum(edges.values()))
        cur_of = {a: newlab[comp[pos[cur_of[a]]]] for a in cur_of}
        layers.append(np.array([cur_of[int(v)] for v in lab0.reshape(-1)], np.int32))
    return np.stack(layers).reshape((NL,) + lab0.shape), chosen_total, w


@pytest.mark.parametrize("shape,conn,vals", [((20, 24), 4, 6), ((20, 24), 8, 50), ((6, 7, 5), 6, 10),
                                             ((6, 7, 5), 26, 5)])
def test_waterfall_vs_rag_and_kruskal(shape, conn, vals):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    rng = np.random.default_rng(23)
    for trial in range(4):
        img = rng.integers(0, vals, size=shape).astype(np.uint16)
        lab = oracle.watershed(img, conn)
        NL = 12
        out, nr = oracle.waterfall_g1(lab, img, conn, NL)
        ref, chosen, w = _waterfall_by_rag(lab, img, conn, NL)
        assert np.array_equal(out, ref)
        # nesting, halving, canonical labels
        for k in range(1, NL):
            prev, cur = out[k - 1].reshape(-1), out[k].reshape(-1)
            for lbl in np.unique(prev):
                assert len(np.unique(cur[prev == lbl])) == 1
            if nr[k - 1] > 1:
                assert nr[k] <= nr[k - 1] // 2
            for lbl in np.unique(cur):
                assert np.flatnonzero(cur == lbl).min() == lbl
            assert nr[k] == len(np.unique(cur))
        assert nr[-1] == 1
        # Borůvka edges over all levels form a minimum spanning tree (weight)
        if w:
            regs = sorted(np.unique(lab).tolist())
            pos = {r: i for i, r in enumerate(regs)}
            rows = [pos[a] for a, b in w]
            cols = [pos[b] for a, b in w]
            g = coo_matrix(([h + 1 for h in w.values()], (rows, cols)), shape=(len(regs), len(regs)))
            mst = minimum_spanning_tree(g).sum() - (len(regs) - 1)
            assert sum(chosen) == int(round(mst))


def test_waterfall_single_region_and_nl1():
    img = np.full((5, 6), 3, np.uint16)
    lab = oracle.watershed(img, 4)
    out, nr = oracle.waterfall_g1(lab, img, 4, 4)
    assert (out == 0).all() and nr.tolist() == [1, 1, 1, 1]
    I = np.array([[0, 4, 0, 2, 9, 1, 6, 3]], np.uint16)
    out, nr = oracle.waterfall_g1(oracle.watershed(I, 4), I, 4, 1)
    assert out.shape == (1, 1, 8) and nr.tolist() == [4]


def test_recon_counts_decrease():
    rng = np.random.default_rng(29)
    img = rng.integers(0, 40, size=(24, 24)).astype(np.uint16)
    out, nr = oracle.waterfall_recon(img, 4, 8)
    for k in range(1, 8):
        if nr[k - 1] > 1:
            assert nr[k] < nr[k - 1]


# --------------------------------------------------------------------------
# Gradient pre-processing (double precision)
# --------------------------------------------------------------------------

def _scipy_grad(f, sigma):
    from scipy import ndimage
    g = f.astype(np.float64)
    if sigma > 0:
        g = ndimage.gaussian_filter(g, sigma, mode="reflect", truncate=4.0)
    comps = [ndimage.sobel(g, axis=a, mode="reflect") for a in range(g.ndim)]
    return np.sqrt(sum(c * c for c in comps))


@pytest.mark.parametrize("shape,sigma", [((37, 53), 0.0), ((37, 53), 1.0), ((40, 31), 2.3),
                                         ((9, 11, 13), 0.0), ((9, 11, 13), 1.0), ((3, 40), 1.5)])
def test_gradient_vs_scipy(shape, sigma):
    rng = np.random.default_rng(31)
    f = (rng.normal(0, 100, size=shape) + 1000).astype(np.float32)
    q, mag = oracle.gradient(f, sigma, "u16", return_mag=True)
    ref = _scipy_grad(f, sigma)
    assert np.allclose(mag, ref, rtol=0, atol=1e-12 * ref.max())
    # quantisation: rint(mag * Q / max) ties to even, exactly, except where the
    # scaled value lies within the float64 disagreement of the two magnitudes
    # (1e-12 * Q) of a .5 boundary, where one level either way is allowed
    exact = ref * 65535.0 / ref.max()
    near = np.abs(exact - np.floor(exact) - 0.5) <= 1e-12 * 65535.0
    assert near.mean() < 0.01  # the allowance covers almost nothing
    d = np.abs(q.astype(np.int64) - np.rint(exact).astype(np.int64))
    assert (d[~near] == 0).all() and d.max() <= 1
    assert q.max() == 65535


@pytest.mark.parametrize("Q,dtype", [(255, "u8"), (65535, "u16")])
def test_gradient_quantisation_ties(Q, dtype):
    """Magnitudes that scale exactly onto k + 1/2 are rounded half to even: a
    flooring, truncating or round-half-up quantiser fails here."""
    from tests.quant_fixture import tie_image
    img, mag_exact, expect = tie_image(Q)
    q, mag = oracle.gradient(img, 0.0, dtype, return_mag=True)
    assert np.array_equal(mag, mag_exact)
    ties = (mag_exact * Q / mag_exact.max()) % 1.0 == 0.5
    assert ties.mean() > 0.9
    assert np.array_equal(q.astype(np.int64), expect)


def test_gradient_closed_forms():
    yy, xx = np.mgrid[0:30, 0:40].astype(np.float64)
    a, b = 3.0, -2.0
    ramp = (a * xx + b * yy).astype(np.float32)
    _, mag = oracle.gradient(ramp, 0.0, "u16", return_mag=True)
    assert np.allclose(mag[1:-1, 1:-1], 8.0 * math.hypot(a, b))
    _, magb = oracle.gradient(ramp, 1.0, "u16", return_mag=True)
    assert np.allclose(magb[5:-5, 5:-5], 8.0 * math.hypot(a, b))  # blur keeps a ramp
    zz, yy, xx = np.mgrid[0:12, 0:12, 0:12].astype(np.float64)
    ramp3 = (1.0 * xx + 2.0 * yy - 2.0 * zz).astype(np.float32)
    _, mag3 = oracle.gradient(ramp3, 0.0, "u8", return_mag=True)
    assert np.allclose(mag3[1:-1, 1:-1, 1:-1], 32.0 * 3.0)
    const = np.full((10, 12), 7.5, np.float32)
    q, magc = oracle.gradient(const, 1.0, "u8", return_mag=True)
    assert (magc == 0).all() and (q == 0).all()
