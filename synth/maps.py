"""Seeded synthetic planar maps and region values.

This module only builds inputs: polygons that tile a square, shared
boundaries, and lognormal values.  It holds none of the cartogram
method's arithmetic (no rasterisation, integral images, displacement or
area error), so both the FP64 oracle and the HIP path can take their
inputs from it.

A map is a planar subdivision of the square [0.05, 0.95]^2 (the unit
square scaled isotropically by 0.9 and centred, the placement rule of
the paper's method section) into R polygonal regions.  The rest of the
unit domain is the background.  Region ids run 1..R; id 0 is the
background.

Representation (`PlanarMap`):
  xy        float64 [n][2]  unique vertices; every coordinate is exactly
                            representable in float32
  ring_off  int32 [nr+1]    CSR offsets into ring_idx
  ring_idx  int32 [sum]     vertex ids of each ring, without repeating
                            the first vertex at the end
  ring_reg  int32 [nr]      region id (1..R) owning each ring
  rings have positive signed area, 0.5*sum(x_k*y_{k+1} - x_{k+1}*y_k) > 0

Recipe (the workloads stand in for the paper's go-cart / Natural Earth
maps, which are not available):
  * sites ~ U[0,1]^2 from numpy PCG64(seed); Voronoi cells built by FP64
    half-plane clipping of the unit square; vertices merged within 1e-9;
  * each shared Voronoi edge a-b is replaced by a chain of K_e segments,
    sum_e (K_e - 1) ~= n_target - n_voronoi, K_e proportional to length;
  * straight mode: chain points evenly spaced on a-b;
    fractal mode: chain points at t_k = k/K_e on a-b displaced along the
    edge normal by a recursive midpoint-displacement function
    (amplitude `amp` * sub-interval length), clamped to 80% of the
    "kite" formed by the two fan triangles (a, b, site) of the cells on
    either side.  The fan triangles of different edges have disjoint
    interiors and the chain is a graph over a-b, so the refined map is
    a valid planar subdivision by construction;
  * outline edges (on the square border) use the fan triangle of the
    cell inside and its mirror image across the border outside, the
    outward excursion capped at 0.04/0.9 of the unit square;
  * values s(v) = exp(mu + sigma*Z), Z ~ N(0,1).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "PlanarMap", "voronoi_map", "square_grid_map", "lognormal_values",
    "random_walk_series", "uneven_batch_specs", "rng_for",
]


@dataclasses.dataclass
class PlanarMap:
    xy: np.ndarray          # float64 [n][2], float32-representable
    ring_off: np.ndarray    # int32 [nr+1]
    ring_idx: np.ndarray    # int32 [sum]
    ring_reg: np.ndarray    # int32 [nr]
    n_regions: int

    @property
    def n_vertices(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_rings(self) -> int:
        return int(self.ring_reg.shape[0])

    def xy32(self) -> np.ndarray:
        return self.xy.astype(np.float32)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ----------------------------------------------------------------------------
# Voronoi cells by half-plane clipping


def _clip(poly: np.ndarray, nrm: np.ndarray, off: float) -> np.ndarray:
    """Keep the part of convex polygon `poly` with nrm.X <= off."""
    if len(poly) == 0:
        return poly
    val = poly @ nrm - off
    out = []
    n = len(poly)
    for k in range(n):
        p, q = poly[k], poly[(k + 1) % n]
        vp, vq = val[k], val[(k + 1) % n]
        if vp <= 0.0:
            out.append(p)
        if (vp < 0.0 < vq) or (vq < 0.0 < vp):
            t = vp / (vp - vq)
            out.append(p + t * (q - p))
    return np.array(out) if out else np.zeros((0, 2))


def _voronoi_cells(sites: np.ndarray) -> list[np.ndarray]:
    square = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    cells = []
    for i, s in enumerate(sites):
        order = np.argsort(((sites - s) ** 2).sum(1))
        poly = square.copy()
        for j in order:
            if j == i:
                continue
            dj = np.sqrt(((sites[j] - s) ** 2).sum())
            rmax = np.sqrt(((poly - s) ** 2).sum(1)).max() if len(poly) else 0.0
            if dj > 2.0 * rmax + 1e-12:
                break   # no farther site can cut the cell
            nrm = 2.0 * (sites[j] - s)
            off = float(sites[j] @ sites[j] - s @ s)
            poly = _clip(poly, nrm, off)
        cells.append(poly)
    return cells


def _merge_vertices(cells: list[np.ndarray], tol: float = 1e-9):
    pts = np.concatenate(cells, axis=0)
    key = np.round(pts / tol).astype(np.int64)
    # union points whose rounded keys are within one cell of each other
    order = np.lexsort((key[:, 1], key[:, 0]))
    parent = np.arange(len(pts))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    from scipy.spatial import cKDTree  # geometry helper only
    tree = cKDTree(pts)
    for a, b in tree.query_pairs(2.0 * tol):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(a) for a in range(len(pts))])
    uniq, inv = np.unique(roots, return_inverse=True)
    verts = pts[uniq]
    rings = []
    k = 0
    for c in cells:
        ids = inv[k:k + len(c)]
        k += len(c)
        ring = []
        for v in ids:
            if not ring or ring[-1] != v:
                ring.append(int(v))
        while len(ring) > 1 and ring[0] == ring[-1]:
            ring.pop()
        rings.append(ring)
    del order
    return verts, rings


# ----------------------------------------------------------------------------
# boundary refinement


def _fan_height(a, b, s, t):
    """Cross-section height of triangle (a, b, s) above segment a-b, at
    parameters t in [0, 1], measured along the normal towards s."""
    ab = b - a
    L2 = ab @ ab
    ts = ((s - a) @ ab) / L2
    hs = abs(ab[0] * (s - a)[1] - ab[1] * (s - a)[0]) / np.sqrt(L2)
    h = np.full_like(t, np.inf)
    if ts > 0:
        h = np.minimum(h, hs * t / ts)
    if ts < 1:
        h = np.minimum(h, hs * (1.0 - t) / (1.0 - ts))
    return np.maximum(h, 0.0)


def _midpoint_fractal(K: int, rng: np.random.Generator, amp: float) -> np.ndarray:
    f = np.zeros(K + 1)
    stack = [(0, K)]
    while stack:
        lo, hi = stack.pop()
        if hi - lo < 2:
            continue
        m = (lo + hi) // 2
        w = (m - lo) / (hi - lo)
        f[m] = (1 - w) * f[lo] + w * f[hi] + amp * (hi - lo) / K * rng.uniform(-1.0, 1.0)
        stack.append((lo, m))
        stack.append((m, hi))
    return f


def _border_mirror(a, b, s):
    """Mirror site s across the square side that contains edge a-b."""
    for d in (0, 1):
        for val in (0.0, 1.0):
            if abs(a[d] - val) < 1e-9 and abs(b[d] - val) < 1e-9:
                m = s.copy()
                m[d] = 2 * val - s[d]
                return m
    return None


def _refine(verts, rings, sites, n_target, fractal, rng, amp):
    # unique edges with owning cells
    owners: dict[tuple[int, int], list[int]] = {}
    for c, ring in enumerate(rings):
        for k in range(len(ring)):
            a, b = ring[k], ring[(k + 1) % len(ring)]
            owners.setdefault((min(a, b), max(a, b)), []).append(c)
    for key, own in owners.items():
        if len(own) > 2:
            raise ValueError("non-manifold Voronoi edge")
    keys = sorted(owners)
    lens = np.array([np.linalg.norm(verts[b] - verts[a]) for a, b in keys])
    extra = max(0, n_target - len(verts))
    share = lens / lens.sum() * extra
    K = np.maximum(1, np.floor(share + 1.0).astype(int))
    chains: dict[tuple[int, int], np.ndarray] = {}
    new_pts = [verts]
    nxt = len(verts)
    for e, (a, b) in enumerate(keys):
        k = int(K[e])
        if k <= 1:
            chains[(a, b)] = np.zeros(0, dtype=np.int64)
            continue
        pa, pb = verts[a], verts[b]
        t = np.arange(1, k) / k
        pts = pa[None, :] + t[:, None] * (pb - pa)[None, :]
        if fractal:
            ab = pb - pa
            nrm = np.array([-ab[1], ab[0]]) / np.linalg.norm(ab)
            f = _midpoint_fractal(k, rng, amp * np.linalg.norm(ab))[1:k]
            own = owners[(a, b)]
            hpos = np.zeros(k - 1)
            hneg = np.zeros(k - 1)
            sides = [sites[c] for c in own]
            if len(own) == 1:
                mir = _border_mirror(pa, pb, sites[own[0]])
                if mir is not None:
                    sides.append(mir)
            for sc in sides:
                h = _fan_height(pa, pb, sc, t)
                if len(own) == 1 and sc is not sides[0]:
                    h = np.minimum(h, 0.04 / 0.9)
                if (sc - pa) @ nrm > 0:
                    hpos = np.maximum(hpos, h)
                else:
                    hneg = np.maximum(hneg, h)
            f = np.clip(f, -0.8 * hneg, 0.8 * hpos)
            pts = pts + f[:, None] * nrm[None, :]
        ids = np.arange(nxt, nxt + k - 1)
        nxt += k - 1
        new_pts.append(pts)
        chains[(a, b)] = ids
    allv = np.concatenate(new_pts, axis=0)
    out_rings = []
    for ring in rings:
        r = []
        for k in range(len(ring)):
            a, b = ring[k], ring[(k + 1) % len(ring)]
            r.append(a)
            ch = chains[(min(a, b), max(a, b))]
            r.extend(ch.tolist() if a < b else ch[::-1].tolist())
        out_rings.append(r)
    return allv, out_rings


def _signed_area(xy, ring):
    p = xy[ring]
    q = np.roll(p, -1, axis=0)
    return 0.5 * float((p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1]).sum())


def _finish(verts, rings, regs, R, scale=0.9) -> PlanarMap:
    xy = (0.5 - scale / 2) + scale * verts
    xy = xy.astype(np.float32).astype(np.float64)
    fixed = []
    for ring in rings:
        if _signed_area(xy, ring) < 0:
            ring = ring[::-1]
        fixed.append(ring)
    off = np.zeros(len(fixed) + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(r) for r in fixed])
    idx = np.array([v for r in fixed for v in r], dtype=np.int32)
    return PlanarMap(xy=xy, ring_off=off, ring_idx=idx,
                     ring_reg=np.asarray(regs, dtype=np.int32), n_regions=int(R))


def voronoi_map(seed: int, R: int, n_target: int, fractal: bool = True,
                amp: float = 0.35, scale: float = 0.9) -> PlanarMap:
    """R Voronoi regions from seeded uniform sites, boundaries refined to
    about n_target unique vertices (straight or fractal)."""
    rng = rng_for(seed)
    sites = rng.random((R, 2))
    cells = _voronoi_cells(sites)
    verts, rings = _merge_vertices(cells)
    verts, rings = _refine(verts, rings, sites, n_target, fractal, rng, amp)
    return _finish(verts, rings, list(range(1, R + 1)), R, scale)


def square_grid_map(k: int = 3, seg: int = 8, lo: float = 0.25, hi: float = 0.75) -> PlanarMap:
    """k x k axis-aligned square regions tiling [lo, hi]^2 with shared
    vertices, each side subdivided into `seg` segments."""
    m = k * seg
    g = np.linspace(lo, hi, m + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel()], 1)   # id = row*(m+1) + col
    vid = lambda r, c: r * (m + 1) + c
    rings, regs = [], []
    used = set()
    for a in range(k):
        for b in range(k):
            r0, c0 = a * seg, b * seg
            ring = [vid(r0, c0 + t) for t in range(seg)]
            ring += [vid(r0 + t, c0 + seg) for t in range(seg)]
            ring += [vid(r0 + seg, c0 + seg - t) for t in range(seg)]
            ring += [vid(r0 + seg - t, c0) for t in range(seg)]
            rings.append(ring)
            regs.append(a * k + b + 1)
            used.update(ring)
    keep = sorted(used)
    remap = {v: i for i, v in enumerate(keep)}
    verts = verts[keep]
    rings = [[remap[v] for v in r] for r in rings]
    xy = verts.astype(np.float32).astype(np.float64)
    fixed = []
    for ring in rings:
        if _signed_area(xy, ring) < 0:
            ring = ring[::-1]
        fixed.append(ring)
    off = np.zeros(len(fixed) + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(r) for r in fixed])
    idx = np.array([v for r in fixed for v in r], dtype=np.int32)
    return PlanarMap(xy=xy, ring_off=off, ring_idx=idx,
                     ring_reg=np.asarray(regs, dtype=np.int32), n_regions=k * k)


def lognormal_values(seed: int, R: int, sigma: float = 1.0, mu: float = 0.0) -> np.ndarray:
    rng = rng_for(seed + 7_777_777)
    return np.exp(mu + sigma * rng.standard_normal(R))


def random_walk_series(seed: int, R: int, T: int, sigma0: float = 1.0,
                       step_sigma: float = 0.1) -> np.ndarray:
    """[T][R] values: s_0 lognormal(0, sigma0), s_{t+1} = s_t exp(step_sigma Z)."""
    rng = rng_for(seed + 9_999_999)
    s = np.exp(sigma0 * rng.standard_normal(R))
    out = [s]
    for _ in range(T - 1):
        s = s * np.exp(step_sigma * rng.standard_normal(R))
        out.append(s)
    return np.stack(out, 0)


def uneven_batch_specs(seed: int, count: int):
    """Specs of an uneven batch of independent cartograms: texture sides
    from {256, 512, 1024, 2048}, 16-300 regions, value sigma in
    [0.5, 2], about 500*R*N/1024 vertices."""
    rng = rng_for(seed)
    specs = []
    for k in range(count):
        N = int(rng.choice([256, 512, 1024, 2048]))
        R = int(rng.integers(16, 301))
        sigma = float(rng.uniform(0.5, 2.0))
        specs.append(dict(seed=int(seed * 1000 + k), N=N, R=R, sigma=sigma,
                          n_target=int(500 * R * N / 1024)))
    return specs
