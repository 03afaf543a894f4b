"""Independent brute-force definitions used to pin the CPU oracle.

Nothing here calls the oracle or the HIP library. Each function restates a
definition from the paper (or a textbook equivalent) in the most direct way,
for tiny inputs only.
"""
from __future__ import annotations

import heapq
import itertools
from collections import deque

import numpy as np


def nbrs(shape, conn):
    """Neighbour lists by linear index (x fastest), in-image pixels only."""
    if len(shape) == 1:
        shape = (1, shape[0])
    nd = len(shape)
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    out = [[] for _ in range(idx.size)]
    for coord in itertools.product(*[range(s) for s in shape]):
        p = idx[coord]
        for d in itertools.product((-1, 0, 1), repeat=nd):
            m = sum(abs(v) for v in d)
            if m == 0:
                continue
            if conn in (4, 6) and m != 1:
                continue
            c = tuple(a + b for a, b in zip(coord, d))
            if all(0 <= c[i] < shape[i] for i in range(nd)):
                out[p].append(int(idx[c]))
        out[p].sort()
    return out


def flat_zones(I, nb):
    """Zone id per pixel: maximal connected sets of equal grey value."""
    n = len(I)
    zone = [-1] * n
    z = 0
    for s in range(n):
        if zone[s] >= 0:
            continue
        zone[s] = z
        st = [s]
        while st:
            p = st.pop()
            for q in nb[p]:
                if zone[q] < 0 and I[q] == I[s]:
                    zone[q] = z
                    st.append(q)
        z += 1
    return zone


def regional_minima(I, nb, zone):
    """Set of zone ids none of whose pixels has a strictly lower neighbour."""
    nz = max(zone) + 1
    has_lower = [False] * nz
    for p in range(len(I)):
        if any(I[q] < I[p] for q in nb[p]):
            has_lower[zone[p]] = True
    return {z for z in range(nz) if not has_lower[z]}


def plateau_distance(I, nb, zone, minimal):
    """Geodesic distance inside each non-minimal flat zone to its pixels that
    have a lower neighbour (0 there), by breadth-first search per pixel."""
    n = len(I)
    d = [None] * n
    for p in range(n):
        if zone[p] in minimal:
            continue
        if any(I[q] < I[p] for q in nb[p]):
            d[p] = 0
            continue
        seen = {p}
        frontier = deque([(p, 0)])
        while frontier:
            u, k = frontier.popleft()
            if any(I[q] < I[u] for q in nb[u]):
                d[p] = k
                break
            for q in nb[u]:
                if q not in seen and I[q] == I[u]:
                    seen.add(q)
                    frontier.append((q, k + 1))
    return d


def drop_watershed(img, conn):
    """Per-pixel 'drop' walk. Each step recomputes the arrow from scratch:
    the steepest descent arrow (largest index among the lowest neighbours) when
    a lower neighbour exists, otherwise on a non-minimal plateau the equal
    neighbour with the smallest index one geodesic step closer to the lower
    border. The walk stops in a regional minimum, which names the basin; the
    basin's label is its smallest pixel index."""
    shape = img.shape
    I = [int(v) for v in np.asarray(img).reshape(-1)]
    nb = nbrs(shape, conn)
    zone = flat_zones(I, nb)
    minimal = regional_minima(I, nb, zone)
    d = plateau_distance(I, nb, zone, minimal)
    n = len(I)
    basin = [None] * n
    for p in range(n):
        u = p
        steps = 0
        while zone[u] not in minimal:
            lowest = min(I[q] for q in nb[u])
            if lowest < I[u]:
                u = max(q for q in nb[u] if I[q] == lowest)
            else:
                u = min(q for q in nb[u] if I[q] == I[u] and d[q] is not None and d[q] == d[u] - 1)
            steps += 1
            assert steps <= n
        basin[p] = zone[u]
    lab = {}
    for p in range(n):
        lab.setdefault(basin[p], p)
    return np.array([lab[basin[p]] for p in range(n)], np.int32).reshape(shape)


def meyer_flood(img, conn):
    """Meyer's priority flooding from the regional minima (distinct values)."""
    shape = img.shape
    I = [int(v) for v in np.asarray(img).reshape(-1)]
    nb = nbrs(shape, conn)
    n = len(I)
    lab = [-1] * n
    heap = []
    for p in range(n):
        if all(I[q] > I[p] for q in nb[p]):
            lab[p] = p
            heapq.heappush(heap, (I[p], p))
    while heap:
        _, p = heapq.heappop(heap)
        for q in nb[p]:
            if lab[q] < 0:
                lab[q] = lab[p]
                heapq.heappush(heap, (I[q], q))
    canon = {}
    for p in range(n):
        canon[lab[p]] = min(canon.get(lab[p], p), p)
    return np.array([canon[lab[p]] for p in range(n)], np.int32).reshape(shape)


def rag(labels, img, conn):
    """Region adjacency graph: {(a, b): min over adjacent pixel pairs of
    max(I(p), I(q))} for labels a < b."""
    L = np.asarray(labels).reshape(-1)
    I = np.asarray(img).reshape(-1).astype(np.int64)
    nb = nbrs(labels.shape, conn)
    w = {}
    for p in range(L.size):
        for q in nb[p]:
            if L[p] != L[q]:
                a, b = (int(L[p]), int(L[q])) if L[p] < L[q] else (int(L[q]), int(L[p]))
                h = int(max(I[p], I[q]))
                if (a, b) not in w or h < w[(a, b)]:
                    w[(a, b)] = h
    return w
