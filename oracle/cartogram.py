"""FP64 CPU oracle of the integral-image contiguous-cartogram method.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that
the HIP path is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does,
and this module imports nothing from the product package.

Conventions (paper: Background, "Integral Images", and the coordinate
remark under eq.(1)):
  * texture of N x N pixels, N = 2^k; pixel (p, q) covers
    [p, p+1] x [q, q+1] in pixel units, p = column (x), q = row (y);
    the y axis points down;
  * nodes (i, j), 0 <= i, j <= N, sit at (x, y) = (i/N, j/N); node tables
    are indexed [j][i];
  * integral images are the exact integrals of the piecewise-constant
    density over the summation areas with the node as corner or apex.

Readings where the paper is silent:
  R1 integral images are node-based exact integrals (see above);
  R2 tilted areas: alpha_t = top wedge, beta_t = left, gamma_t = bottom,
     delta_t = right (pairing of the Fig. 2 caption with eq.(2));
  R3 pixel membership: pixel centre sampling with coordinates snapped to
     1/256 pixel (round half to even), half-open rows, a centre on an edge
     belongs to the region on the edge's +x side; a centre claimed by
     several regions of a folded map goes to the highest region id;
  R4 d0 = sum s(v) / sum o(v) over map regions with o(v) > 0, BDV = b*d0
     with b the shape parameter (default 1);
  R5 desired areas w(v) = s(v) * (sum of current map-region areas)/sum s;
  R6 stopping: xi_k < tol, or no new minimum of xi in the last
     `patience` iterations, or max_iters; the final (not the best) state
     is returned;
  R7 no step-size damping; points are clamped to [0, 1]^2.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SUB = 256  # fixed-point subdivisions per pixel used for rasterisation

STATUS_CONVERGED = 0
STATUS_STALLED = 1
STATUS_MAXITER = 2


# ----------------------------------------------------------------------------
# Step 2: labels by pixel-centre membership (reading R3)


def snap(xy: np.ndarray, N: int):
    """Fixed-point coordinates X = rint(x * 256 N), round half to even."""
    X = np.rint(xy[:, 0] * (SUB * N)).astype(np.int64)
    Y = np.rint(xy[:, 1] * (SUB * N)).astype(np.int64)
    return X, Y


def ring_edges(ring_off, ring_idx, ring_reg):
    """Directed edges (a -> b, region) of every ring, closing each ring."""
    a_list, b_list, r_list = [], [], []
    for k in range(len(ring_reg)):
        ids = ring_idx[ring_off[k]:ring_off[k + 1]]
        a_list.append(ids)
        b_list.append(np.roll(ids, -1))
        r_list.append(np.full(len(ids), ring_reg[k], dtype=np.int64))
    return (np.concatenate(a_list).astype(np.int64),
            np.concatenate(b_list).astype(np.int64),
            np.concatenate(r_list))


def rasterize(xy, ring_off, ring_idx, ring_reg, n_regions: int, N: int):
    """Label map (uint16 [N][N], 0 = background), pixel counts o(v)
    (int64 [R+1]) and the number of pixels claimed by two or more regions
    (possible only once the subdivision has folded; such a pixel takes the
    highest claiming region id, reading R3).

    Region v contains the centre of pixel (p, q) iff the number of
    crossings of v's ring edges with row q whose first pixel p0 is <= p
    is odd (even-odd rule).  An edge a->b crosses row q iff
    (a.Y <= yc) != (b.Y <= yc) with yc = 256 q + 128; its p0 is the
    smallest p in [0, N] whose centre is at or right of the crossing,
    decided by the exact sign of the orientation determinant.
    """
    X, Y = snap(xy, N)
    ea, eb, ereg = ring_edges(ring_off, ring_idx, ring_reg)
    aX, aY, bX, bY = X[ea], Y[ea], X[eb], Y[eb]
    lo = np.minimum(aY, bY)
    hi = np.maximum(aY, bY)
    # rows with lo <= 256 q + 128 < hi
    q_first = np.clip(-((-(lo - SUB // 2)) // SUB), 0, N)
    q_end = np.clip(-((-(hi - SUB // 2)) // SUB), 0, N)
    cnt = np.maximum(q_end - q_first, 0)
    e = np.repeat(np.arange(len(ea)), cnt)
    starts = np.repeat(q_first, cnt)
    within = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    q = starts + within
    yc = SUB * q + SUB // 2
    ax, ay, bx, by = aX[e], aY[e], bX[e], bY[e]
    assert np.all((ay <= yc) != (by <= yc))
    sgn = np.sign(by - ay)

    def at_or_right(p):
        xc = SUB * p + SUB // 2
        det = (xc - ax) * (by - ay) - (yc - ay) * (bx - ax)
        return det * sgn >= 0

    # binary search for the smallest p in [0, N] with the predicate true
    # (p = N stands for "no centre of the row is at or right of it")
    plo = np.zeros(len(e), dtype=np.int64)
    phi = np.full(len(e), N, dtype=np.int64)
    while True:
        act = plo < phi
        if not act.any():
            break
        mid = (plo + phi) // 2
        ok = at_or_right(mid)
        phi = np.where(act & ok, mid, phi)
        plo = np.where(act & ~ok, mid + 1, plo)
    p0 = plo
    reg = ereg[e]

    # even-odd fill per (region, row): sorted crossings pair up
    order = np.lexsort((p0, q, reg))
    reg_s, q_s, p_s = reg[order], q[order], p0[order]
    key = reg_s * (N + 1) + q_s
    if len(key):
        _, first, sizes = np.unique(key, return_index=True, return_counts=True)
        assert np.all(sizes % 2 == 0) and np.all(first % 2 == 0)
    start = p_s[0::2]
    end = p_s[1::2]
    rows = q_s[0::2]
    regs = reg_s[0::2]
    claim = np.zeros((N, N + 1), dtype=np.int64)
    lsum = np.zeros((N, N + 1), dtype=np.int64)
    np.add.at(claim, (rows, start), 1)
    np.add.at(claim, (rows, end), -1)
    np.add.at(lsum, (rows, start), regs)
    np.add.at(lsum, (rows, end), -regs)
    claim = np.cumsum(claim, axis=1)[:, :N]
    lsum = np.cumsum(lsum, axis=1)[:, :N]
    labels = np.where(claim == 1, lsum, 0)
    # a centre claimed by several regions (the subdivision has folded)
    # goes to the highest claiming region id
    cq, cp = np.nonzero(claim > 1)
    for qq, pp in zip(cq, cp):
        cover = (rows == qq) & (start <= pp) & (pp < end)
        labels[qq, pp] = regs[cover].max()
    conflicts = int(len(cq))
    labels = labels.astype(np.uint16)
    counts = np.bincount(labels.ravel().astype(np.int64),
                         minlength=n_regions + 1)[: n_regions + 1].astype(np.int64)
    return labels, counts, conflicts


# ----------------------------------------------------------------------------
# Step 3: density texture (reading R4)


def density_lut(counts, values, b: float = 1.0, areas=None, bg_mass=None):
    """LUT [R+1] of densities: lut[v] = s(v)/o(v), lut[0] = BDV = b*d0.

    With `areas` (polygon areas in pixel units) the density uses them in
    place of the pixel counts (the POLYGON area source).  With `bg_mass`
    M_b (the background's share of the mass, eq.(4)) the BDV is
    b * M_b / (background pixel count) instead, so that the background
    holds the mass M_b (b * d0 when the raster has no background pixel)."""
    o = (np.asarray(counts, np.float64) if areas is None else np.asarray(areas, np.float64))[1:]
    s = np.asarray(values, np.float64)
    have = o > 0
    d0 = s[have].sum() / o.sum() if o.sum() > 0 else 1.0   # an empty raster: unit density
    lut = np.zeros(len(s) + 1)
    lut[1:][have] = s[have] / o[have]
    o_bg = float(counts[0])
    lut[0] = b * (bg_mass / o_bg if (bg_mass is not None and o_bg > 0) else d0)
    return lut, d0


def background_masses(series, area_min: float, area_max: float, t0: int = 0, t1: int | None = None, at=None):
    """Background mass M_b(t) of every step of a value series [T][R] (the
    time-varying section, eq.(4)): the map's total M_i(t) = sum_v s_t(v);
    with M_min / M_max the extremes of M_i over the steps t0..t1,
    w = (M_i(t) - M_min) / (M_max - M_min) (clamped to [0, 1] for steps
    outside that range; 1 when M_max = M_min), the map's area fraction
    A_i(t) = (1 - w) A_min + w A_max, and M_i / (M_i + M_b) = A_i gives
    M_b(t) = M_i(t) (1 - A_i(t)) / A_i(t).  `at` evaluates the same rule
    at other totals (the in-between frames of a series) with the extremes
    still taken over the series' steps.  Returns (M_b, A_i)."""
    S = np.asarray(series, np.float64)
    t1 = S.shape[0] - 1 if t1 is None else t1
    lo, hi = S.sum(axis=1)[t0:t1 + 1].min(), S.sum(axis=1)[t0:t1 + 1].max()
    Mi = S.sum(axis=1) if at is None else np.asarray(at, np.float64)
    w = np.ones_like(Mi) if hi == lo else np.clip((Mi - lo) / (hi - lo), 0.0, 1.0)
    A = (1.0 - w) * area_min + w * area_max
    return Mi * (1.0 - A) / A, A


def density_texture(labels, lut):
    return lut[labels.astype(np.int64)]


def log_density(labels, counts, values, b: float = 1.0):
    """Input of the learned warm start: log of the Step-3 density over its
    mean over the texture."""
    lut, _ = density_lut(counts, values, b)
    d = density_texture(labels, lut)
    return np.log(d / d.mean())


# ----------------------------------------------------------------------------
# Step 4: integral images (reading R1, R2; eq.(1))


@dataclasses.dataclass
class InIm:
    S: np.ndarray    # [N+1][N+1]  S[j][i] = sum_{p<i, q<j} d
    T: np.ndarray    # [N+1][N+1]  mass of the top wedge with apex at node (i, j)
    HA: np.ndarray   # [2N+1]      HA[s] = mass with x'+y' <= s (pixel units)
    HB: np.ndarray   # [2N+1]      HB[r+N] = mass with y'-x' <= r
    C: float


def integral_images(d: np.ndarray) -> InIm:
    """Node integral images of density d ([N][N], indexed [q][p]).

    Axis-aligned: S is the exact integral over [0, x] x [0, y].
    Tilted: in the rotated coordinates u = x+y, r = y-x the top wedge of
    node (i, j) is the quadrant u <= i+j, r <= j-i.  A pixel is the
    diamond |u-U| + |r-V| <= 1 around U = p+q+1, V = q-p, so with P the
    inclusive prefix sum of the pixels over (U, V) the wedge mass is
    P(s, r-1) fully covered pixels plus one half of the pixels that the
    lines u = s and r = r cut in two: T = (P(s, r-1) + P(s-1, r)) / 2.
    The same argument gives the diagonal marginals HA and HB.
    """
    N = d.shape[0]
    S = np.zeros((N + 1, N + 1))
    S[1:, 1:] = np.cumsum(np.cumsum(d, axis=0), axis=1)
    q, p = np.mgrid[0:N, 0:N]
    U = p + q + 1
    V = q - p
    L = np.zeros((2 * N + 2, 2 * N + 2))
    L[U + 1, V + N + 1] = d           # L[a+1][b+N+1] holds the pixel at (U, V) = (a, b)
    P = np.cumsum(np.cumsum(L, axis=0), axis=1)
    jj, ii = np.mgrid[0:N + 1, 0:N + 1]
    s = ii + jj
    r = jj - ii
    T = 0.5 * (P[s + 1, r + N] + P[s, r + N + 1])
    sv = np.arange(2 * N + 1)
    HA = 0.5 * (P[sv + 1, -1] + P[sv, -1])
    rv = np.arange(-N, N + 1)
    HB = 0.5 * (P[-1, rv + N + 1] + P[-1, rv + N])
    return InIm(S=S, T=T, HA=HA, HB=HB, C=float(S[N, N]))


def eight_inims(im: InIm):
    """The eight integral images at every node (Background, "Integral
    Images"): quadrants top-left, bottom-left, bottom-right, top-right and
    the top, left, bottom, right wedges (reading R2)."""
    N = im.S.shape[0] - 1
    S, T, C = im.S, im.T, im.C
    colN = S[N, :][None, :]       # S(i, N): everything left of x
    rowN = S[:, N][:, None]       # S(N, j): everything above y
    a = S
    b = colN - S
    dl = rowN - S
    g = C - colN - rowN + S
    jj, ii = np.mgrid[0:N + 1, 0:N + 1]
    HA = im.HA[ii + jj]
    HB = im.HB[jj - ii + N]
    at = T
    bt = HA - T
    dt = HB - T
    gt = C - HA - HB + T
    return a, b, g, dl, at, bt, gt, dt


# ----------------------------------------------------------------------------
# Step 5: the eight-anchor map, eq.(2), and the DET, eq.(3)


def anchors(x, y):
    """Anchor points q1..q4 of the two diagonals through (x, y); y down."""
    lowx = y < x
    q1 = np.where(lowx, 1.0, 1.0 - y + x), np.where(lowx, 1.0 + y - x, 1.0)
    q3 = np.where(lowx, x - y, 0.0), np.where(lowx, 0.0, y - x)
    low = x + y < 1.0
    q2 = np.where(low, x + y, 1.0), np.where(low, 0.0, x + y - 1.0)
    q4 = np.where(low, 0.0, x + y - 1.0), np.where(low, x + y, 1.0)
    return q1, q2, q3, q4


def eight_anchor_map(im: InIm):
    """t(x, y; d) of eq.(2) at every node, returned as (tx, ty) [N+1][N+1]."""
    N = im.S.shape[0] - 1
    a, b, g, dl, at, bt, gt, dt = eight_inims(im)
    jj, ii = np.mgrid[0:N + 1, 0:N + 1]
    x = ii / N
    y = jj / N
    q1, q2, q3, q4 = anchors(x, y)
    tx = a * q1[0] + b * q2[0] + g * q3[0] + dl * q4[0] + at * x + bt * 1.0 + gt * x + dt * 0.0
    ty = a * q1[1] + b * q2[1] + g * q3[1] + dl * q4[1] + at * 1.0 + bt * y + gt * 0.0 + dt * y
    return tx / (2.0 * im.C), ty / (2.0 * im.C)


_T0_CACHE: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def t_uniform(N: int):
    """t(x, y; d0) for a constant density (Step 1: computed once per N)."""
    if N not in _T0_CACHE:
        _T0_CACHE[N] = eight_anchor_map(integral_images(np.ones((N, N))))
    return _T0_CACHE[N]


def displacement(im: InIm):
    """Node displacement D = t(.; d) - t(.; d0), eq.(3)."""
    N = im.S.shape[0] - 1
    tx, ty = eight_anchor_map(im)
    ux, uy = t_uniform(N)
    return tx - ux, ty - uy


# ----------------------------------------------------------------------------
# Warm start (not in the paper): a displacement field at the pixel centres
# of a G x G grid moves the starting positions before the iteration.


def warm_start_move(xy: np.ndarray, field: np.ndarray) -> np.ndarray:
    """Bilinear interpolation of field[j][i] = (dx, dy) given at
    ((i + 1/2)/G, (j + 1/2)/G), constant beyond the outermost centres,
    then clamp to the unit square."""
    G = field.shape[0]
    if G == 1:
        d = np.broadcast_to(field[0, 0], xy.shape)
    else:
        u = np.clip(xy[:, 0] * G - 0.5, 0.0, G - 1.0)
        v = np.clip(xy[:, 1] * G - 0.5, 0.0, G - 1.0)
        i0 = np.minimum(np.floor(u).astype(np.int64), G - 2)
        j0 = np.minimum(np.floor(v).astype(np.int64), G - 2)
        fx = (u - i0)[:, None]
        fy = (v - j0)[:, None]
        d = ((1 - fx) * (1 - fy) * field[j0, i0] + fx * (1 - fy) * field[j0, i0 + 1]
             + (1 - fx) * fy * field[j0 + 1, i0] + fx * fy * field[j0 + 1, i0 + 1])
    return np.clip(xy + d, 0.0, 1.0)


WARM_STEPS = (1.0, 0.75, 0.5, 0.25)


def warm_start_choose(m, values, N: int, xy0: np.ndarray, field: np.ndarray):
    """Graded warm start: among the trial steps alpha * field, keep the one
    whose moved map has no pixel claimed by two regions and whose max area
    error is lowest, if that error is below the plain start's.  Returns
    (alpha, starting positions); alpha = 0 is the plain start."""
    A = region_areas(xy0, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
    best = cartographic_errors(A, values)[1]
    pick = 0.0
    for a in WARM_STEPS:
        xy = warm_start_move(xy0, a * field)
        _, _, conflicts = rasterize(xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
        if conflicts > 0:
            continue
        xi = cartographic_errors(region_areas(xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions), values)[1]
        if xi < best:
            best, pick = xi, a
    return pick, (warm_start_move(xy0, pick * field) if pick else xy0.copy())


def tracer_grid(G: int) -> np.ndarray:
    """Pixel centres ((i + 1/2)/G, (j + 1/2)/G), row-major over j, [G*G][2]."""
    c = (np.arange(G) + 0.5) / G
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


# ----------------------------------------------------------------------------
# Step 6: bilinear advection of points (reading R7)


def move_points(xy: np.ndarray, Dx: np.ndarray, Dy: np.ndarray) -> np.ndarray:
    N = Dx.shape[0] - 1
    u = np.clip(xy[:, 0] * N, 0.0, N)
    v = np.clip(xy[:, 1] * N, 0.0, N)
    i0 = np.minimum(np.floor(u).astype(np.int64), N - 1)
    j0 = np.minimum(np.floor(v).astype(np.int64), N - 1)
    fx = u - i0
    fy = v - j0

    def bil(F):
        return ((1 - fx) * (1 - fy) * F[j0, i0] + fx * (1 - fy) * F[j0, i0 + 1]
                + (1 - fx) * fy * F[j0 + 1, i0] + fx * fy * F[j0 + 1, i0 + 1])

    out = np.empty_like(xy, dtype=np.float64)
    out[:, 0] = np.clip(xy[:, 0] + bil(Dx), 0.0, 1.0)
    out[:, 1] = np.clip(xy[:, 1] + bil(Dy), 0.0, 1.0)
    return out


# ----------------------------------------------------------------------------
# Step 7 and the quality measures: areas and cartographic errors


def ring_areas(xy, ring_off, ring_idx):
    """Signed shoelace area of every ring."""
    out = np.zeros(len(ring_off) - 1)
    for k in range(len(out)):
        ids = ring_idx[ring_off[k]:ring_off[k + 1]]
        p = xy[ids]
        q = np.roll(p, -1, axis=0)
        out[k] = 0.5 * np.sum(p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1])
    return out


def region_areas(xy, ring_off, ring_idx, ring_reg, n_regions: int):
    """A(v) for v = 1..R (index 0: the background, 1 - sum of the map)."""
    ra = ring_areas(xy, ring_off, ring_idx)
    A = np.zeros(n_regions + 1)
    np.add.at(A, np.asarray(ring_reg, np.int64), ra)
    A[0] = 1.0 - A[1:].sum()
    return A


def cartographic_errors(A, values):
    """(eps, xi): mean and max of |A - w| / max(A, w) over map regions,
    w(v) = s(v) * (sum_u A(u)) / sum_u s(u) (reading R5)."""
    a = np.asarray(A, np.float64)[1:]
    s = np.asarray(values, np.float64)
    w = s * a.sum() / s.sum()
    e = np.abs(a - w) / np.maximum(a, w)
    return float(e.mean()), float(e.max())


# ----------------------------------------------------------------------------
# the iteration (Steps 2-7) and its stopping rule (reading R6)


@dataclasses.dataclass
class RunResult:
    xy: np.ndarray
    iters: int
    status: int
    eps: float
    xi: float
    xi_history: list
    extra: np.ndarray | None = None


def iterate_once(xy, m, values, N, b=1.0, area_source="pixel", extra=None, bg_mass=None):
    """One pass of Steps 2-6 on positions xy; returns the moved points and
    the intermediate products (labels, counts, lut, InIm, D, and the moved
    tracer points `extra` when given)."""
    labels, counts, conflicts = rasterize(xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    areas = None
    if area_source == "polygon":
        areas = region_areas(xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions) * (N * N)
    lut, _ = density_lut(counts, values, b, areas, bg_mass)
    d = density_texture(labels, lut)
    im = integral_images(d)
    Dx, Dy = displacement(im)
    new = move_points(xy, Dx, Dy)
    moved_extra = None if extra is None else move_points(extra, Dx, Dy)
    return new, dict(labels=labels, counts=counts, conflicts=conflicts, lut=lut, im=im, Dx=Dx, Dy=Dy,
                     extra=moved_extra)


def run(m, values, N, xy0=None, b=1.0, tol=0.01, patience=32, max_iters=512,
        area_source="pixel", fixed_iters=None, state_dtype=np.float64, extra=None, bg_mass=None,
        progress=None) -> RunResult:
    """Iterate until xi < tol, no new minimum in `patience` iterations, or
    max_iters (or exactly `fixed_iters` iterations when given).

    `state_dtype` is the precision the positions are kept in between
    iterations (float64 by default; float32 reproduces a float32 state,
    whose snapping to the raster grid is then decided in the same
    precision as a float32 implementation).  `progress(k, xi)`, when
    given, is called after every iteration (reporting only)."""
    xy = np.asarray(m.xy if xy0 is None else xy0, np.float64).astype(state_dtype).astype(np.float64)
    if extra is not None:
        extra = np.asarray(extra, np.float64).astype(state_dtype).astype(np.float64)
    A = region_areas(xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
    eps, xi = cartographic_errors(A, values)
    hist = [xi]
    best, best_k, k = xi, 0, 0
    status = STATUS_MAXITER
    while True:
        if fixed_iters is not None:
            if k >= fixed_iters:
                status = STATUS_MAXITER
                break
        else:
            if xi < tol:
                status = STATUS_CONVERGED
                break
            if k - best_k >= patience:
                status = STATUS_STALLED
                break
            if k >= max_iters:
                status = STATUS_MAXITER
                break
        xy, info = iterate_once(xy, m, values, N, b, area_source, extra, bg_mass)
        xy = xy.astype(state_dtype).astype(np.float64)
        if extra is not None:
            extra = info["extra"].astype(state_dtype).astype(np.float64)
        k += 1
        A = region_areas(xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
        eps, xi = cartographic_errors(A, values)
        hist.append(xi)
        if progress is not None:
            progress(k, xi)
        if xi < best:
            best, best_k = xi, k
    return RunResult(xy=xy, iters=k, status=status, eps=eps, xi=xi, xi_history=hist, extra=extra)


# ----------------------------------------------------------------------------
# time series (Method section, "Coherence of Dynamic Cartograms")


def run_series(m, series, N, mode="direct", frames_per_step=0, frame_mode="positions", area_fraction=None, **kw):
    """Cartograms for every row of `series` [T][R].  Direct: every step
    deforms the original map; cumulative: every step starts from the
    previous step's cartogram.  With frames_per_step = K > 0 each
    transition gets K-1 in-between frames: frame_mode "positions" lerps
    the vertex positions of consecutive steps; "values" computes a
    cartogram of the lerped values (1 - k/K) s_t + (k/K) s_{t+1} for each
    frame (from the original map in direct mode, from the previous frame
    in cumulative mode, so that the chain runs step, frames, next step).
    With area_fraction = (A_min, A_max[, t0, t1]) every step and frame
    gets the background mass of eq.(4), the extremes of the map total
    taken over the steps t0..t1 (all steps by default)."""
    S = np.asarray(series, np.float64)
    T = S.shape[0]
    K = frames_per_step
    by_values = K > 1 and frame_mode == "values"
    if by_values:   # expanded series: step t at row t*K, frame k of transition t at row t*K + k
        rows = [S[0]]
        for t in range(1, T):
            rows += [(1 - k / K) * S[t - 1] + (k / K) * S[t] for k in range(1, K)] + [S[t]]
        E = np.stack(rows, 0)
    else:
        E = S
    masses = [None] * E.shape[0]
    if area_fraction is not None:
        t0 = area_fraction[2] if len(area_fraction) > 2 else 0
        t1 = area_fraction[3] if len(area_fraction) > 3 else T - 1
        masses = list(background_masses(S, area_fraction[0], area_fraction[1], t0, t1, at=E.sum(axis=1))[0])
    res_all = []
    prev = np.asarray(m.xy, np.float64)
    for e in range(E.shape[0]):
        start = m.xy if mode == "direct" else prev
        r = run(m, E[e], N, xy0=start, bg_mass=masses[e], **kw)
        res_all.append(r)
        prev = r.xy
    if by_values:
        out = [res_all[t * K] for t in range(T)]
        frames = [np.stack([res_all[(t - 1) * K + k].xy for k in range(1, K)], 0) for t in range(1, T)]
        return out, frames
    out = res_all
    frames = []
    if K > 0:
        for t in range(1, len(out)):
            a, bq = out[t - 1].xy, out[t].xy
            frames.append(np.stack([a + (k / K) * (bq - a) for k in range(1, K)], 0))
    return out, frames
