"""Independent brute-force checkers used to pin the oracle.

Nothing here is shared with the oracle or with the HIP path: each routine
restates a definition in the most direct (and slowest) way -- exact
rational ray casting per pixel centre, pixel-by-pixel polygon clipping
of summation areas, direct double sums.
"""
from fractions import Fraction

import numpy as np


def snapped(x: float, N: int) -> int:
    # x * 256N is exact in binary floating point; round() is half-to-even
    return int(round(x * 256 * N))


def brute_labels(xy, ring_off, ring_idx, ring_reg, N):
    """Labels by exact rational ray casting from each pixel centre.

    A centre (xc, yc) is inside a region when the number of its ring edges
    crossing the horizontal line y = yc (exactly one endpoint with Y <= yc)
    at an exact abscissa <= xc is odd; the label is the highest region id
    among the regions that contain the centre (0 when none)."""
    X = [snapped(float(v), N) for v in xy[:, 0]]
    Y = [snapped(float(v), N) for v in xy[:, 1]]
    regs = sorted(set(int(r) for r in ring_reg))
    edges = {r: [] for r in regs}
    for k in range(len(ring_reg)):
        ids = [int(v) for v in ring_idx[ring_off[k]:ring_off[k + 1]]]
        for t in range(len(ids)):
            edges[int(ring_reg[k])].append((ids[t], ids[(t + 1) % len(ids)]))
    lab = np.zeros((N, N), dtype=np.int64)
    for q in range(N):
        yc = 256 * q + 128
        xk = {r: [] for r in regs}
        for r in regs:
            for a, b in edges[r]:
                if (Y[a] <= yc) != (Y[b] <= yc):
                    xk[r].append(Fraction(X[a]) + Fraction((yc - Y[a]) * (X[b] - X[a]), Y[b] - Y[a]))
        for p in range(N):
            xc = 256 * p + 128
            inside = [r for r in regs if sum(1 for v in xk[r] if v <= xc) % 2 == 1]
            lab[q, p] = max(inside) if inside else 0
    return lab


def _clip(poly, a, b, c):
    """Part of polygon `poly` with a*x + b*y <= c (Sutherland-Hodgman)."""
    out = []
    n = len(poly)
    for k in range(n):
        P, Q = poly[k], poly[(k + 1) % n]
        fp = a * P[0] + b * P[1] - c
        fq = a * Q[0] + b * Q[1] - c
        if fp <= 0:
            out.append(P)
        if (fp < 0 < fq) or (fq < 0 < fp):
            t = fp / (fp - fq)
            out.append((P[0] + t * (Q[0] - P[0]), P[1] + t * (Q[1] - P[1])))
    return out


def _area(poly):
    s = 0.0
    for k in range(len(poly)):
        x1, y1 = poly[k]
        x2, y2 = poly[(k + 1) % len(poly)]
        s += x1 * y2 - x2 * y1
    return abs(s) / 2.0


def wedge_mass(d, i, j, which):
    """Integral of the piecewise-constant density d ([q][p]) over a
    45-degree wedge with apex at node (i, j), by clipping every pixel
    square.  which: 'top' y' <= j - |x'-i|, 'left' x' <= i - |y'-j|,
    'bottom' y' >= j + |x'-i|, 'right' x' >= i + |y'-j|."""
    N = d.shape[0]
    tot = 0.0
    for q in range(N):
        for p in range(N):
            sq = [(p, q), (p + 1, q), (p + 1, q + 1), (p, q + 1)]
            if which == 'top':      # y'-y <= x'-x and y'-y <= x-x'
                h = [(-1, 1, j - i), (1, 1, i + j)]
            elif which == 'left':   # x'-x <= y'-y and x'-x <= y-y'
                h = [(1, -1, i - j), (1, 1, i + j)]
            elif which == 'bottom':  # y'-y >= |x'-x|
                h = [(1, -1, i - j), (-1, -1, -(i + j))]
            else:                   # right: x'-x >= |y'-y|
                h = [(-1, 1, j - i), (-1, -1, -(i + j))]
            poly = sq
            for a, b, c in h:
                poly = _clip(poly, a, b, c)
                if not poly:
                    break
            if poly:
                tot += d[q, p] * _area(poly)
    return tot


def rect_mass(d, x0, x1, y0, y1):
    """Direct double sum of d over pixels p in [x0, x1), q in [y0, y1)."""
    s = 0.0
    for q in range(y0, y1):
        for p in range(x0, x1):
            s += d[q, p]
    return s


def segments_cross(xy, ring_off, ring_idx):
    """Number of pairs of map edges that properly cross (shared vertices
    excluded), by brute force with bounding-box pruning."""
    es = set()
    for k in range(len(ring_off) - 1):
        ids = [int(v) for v in ring_idx[ring_off[k]:ring_off[k + 1]]]
        for t in range(len(ids)):
            a, b = ids[t], ids[(t + 1) % len(ids)]
            es.add((min(a, b), max(a, b)))
    es = sorted(es)
    A = np.array([xy[a] for a, _ in es])
    B = np.array([xy[b] for _, b in es])
    lo = np.minimum(A, B)
    hi = np.maximum(A, B)

    def orient(p, q, r):
        return np.sign((q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0]))

    n = 0
    for u in range(len(es)):
        cand = np.nonzero((lo[:, 0] <= hi[u, 0]) & (hi[:, 0] >= lo[u, 0])
                          & (lo[:, 1] <= hi[u, 1]) & (hi[:, 1] >= lo[u, 1]))[0]
        for v in cand:
            if v <= u or len({*es[u], *es[v]}) < 4:
                continue
            if (orient(A[u], B[u], A[v]) * orient(A[u], B[u], B[v]) < 0
                    and orient(A[v], B[v], A[u]) * orient(A[v], B[v], B[u]) < 0):
                n += 1
    return n
