"""Geographic-distortion quality measures of a cartogram against its
original map (paper: Background, "Quality Measures"): topology distortion
tau, shape distortion (normalised symmetric difference, minimised over
translations by whole pixels) and relative position error R.

TEST INFRASTRUCTURE ONLY.  Plain reference for the HIP path; only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it.
It imports nothing from the product package.

Readings where the paper is silent:
  Q1 both the original map and the cartogram are rasterised at the same
     texture size N with the Step-2 label rule; two regions are
     neighbours when a pixel of one and a pixel of the other share a
     pixel side (4-neighbourhood); the background is not a region;
  Q2 a region's polygon is its pixel set in that raster; the shape
     distortion of region v is min over integer translations t of
     |P_m (sym. difference) (P_c + t)| / |P_m union (P_c + t)| (no
     scaling); 0 when both sets are empty, 1 when exactly one is;
     reported per region, as the mean over regions and as the maximum;
  Q3 barycentres are the area centroids of the regions' polygons (all
     rings of a region together, shoelace moments); the angle between
     two vectors is atan2(cross, dot); R sums |angle| over ordered pairs
     u != v and divides by pi |V| (|V| - 1).
"""
from __future__ import annotations

import numpy as np

from . import cartogram as oc


# ----------------------------------------------------------------------------
# topology distortion tau


def adjacency(labels: np.ndarray) -> set:
    """Unordered pairs (u, v), 1 <= u < v, of regions with pixels sharing
    a pixel side (reading Q1)."""
    lab = labels.astype(np.int64)
    pairs = set()
    for a, b in ((lab[:, :-1], lab[:, 1:]), (lab[:-1, :], lab[1:, :])):
        m = (a != b) & (a > 0) & (b > 0)
        u = np.minimum(a[m], b[m])
        v = np.maximum(a[m], b[m])
        pairs.update(zip(u.tolist(), v.tolist()))
    return pairs


def topology_distortion(lab_map: np.ndarray, lab_cart: np.ndarray):
    """tau = 1 - |E_c intersect E_m| / |E_c union E_m| (0 when both are
    empty), with the sizes |E_m|, |E_c| and |E_c intersect E_m|."""
    em, ec = adjacency(lab_map), adjacency(lab_cart)
    union = len(em | ec)
    common = len(em & ec)
    tau = 0.0 if union == 0 else 1.0 - common / union
    return tau, len(em), len(ec), common


# ----------------------------------------------------------------------------
# shape distortion


def _crop(mask: np.ndarray):
    ys, xs = np.nonzero(mask)
    return mask[ys.min():ys.max() + 1, xs.min():xs.max() + 1]


def best_overlap_bruteforce(A: np.ndarray, B: np.ndarray) -> int:
    """max over integer translations t of |A intersect (B + t)| for boolean
    images, by trying every translation under which the two can meet."""
    if not A.any() or not B.any():
        return 0
    a, b = _crop(A), _crop(B)
    ha, wa = a.shape
    hb, wb = b.shape
    best = 0
    for dy in range(-(hb - 1), ha):
        for dx in range(-(wb - 1), wa):
            ya0, ya1 = max(0, dy), min(ha, hb + dy)
            xa0, xa1 = max(0, dx), min(wa, wb + dx)
            o = int(np.sum(a[ya0:ya1, xa0:xa1] & b[ya0 - dy:ya1 - dy, xa0 - dx:xa1 - dx]))
            best = max(best, o)
    return best


def overlap_all(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """|a intersect (b + t)| for every translation t = (dy, dx) with
    -(hb-1) <= dy < ha, -(wb-1) <= dx < wa: the full 2-D
    cross-correlation of the indicator images by FFT, rounded to the
    integers it counts (exact: the float error is far below 1/2)."""
    ha, wa = a.shape
    hb, wb = b.shape
    H, W = ha + hb - 1, wa + wb - 1
    fa = np.fft.rfft2(a.astype(np.float64), (H, W))
    fb = np.fft.rfft2(b[::-1, ::-1].astype(np.float64), (H, W))
    c = np.fft.irfft2(fa * fb, (H, W))
    return np.rint(c).astype(np.int64)     # index (dy + hb - 1, dx + wb - 1)


def best_overlap(A: np.ndarray, B: np.ndarray) -> int:
    if not A.any() or not B.any():
        return 0
    return int(overlap_all(_crop(A), _crop(B)).max())


def shape_ratio(na: int, nb: int, o: int) -> float:
    """|A sym. diff. B| / |A union B| from the set sizes and their overlap."""
    u = na + nb - o
    return 0.0 if u == 0 else (na + nb - 2 * o) / u


def shape_distortion(lab_map: np.ndarray, lab_cart: np.ndarray, R: int, brute: bool = False):
    """Per-region shape distortion [R+1] (index 0 unused, 0), its mean and
    max over regions 1..R, and the best overlaps (reading Q2)."""
    H = np.zeros(R + 1)
    best = np.zeros(R + 1, dtype=np.int64)
    for v in range(1, R + 1):
        A = lab_map == v
        B = lab_cart == v
        o = best_overlap_bruteforce(A, B) if brute else best_overlap(A, B)
        best[v] = o
        H[v] = shape_ratio(int(A.sum()), int(B.sum()), o)
    return H, float(H[1:].mean()) if R else 0.0, float(H[1:].max()) if R else 0.0, best


# ----------------------------------------------------------------------------
# relative position error R


def barycenters(xy, ring_off, ring_idx, ring_reg, R: int) -> np.ndarray:
    """Area centroid of every region [R+1][2] (row 0 unused): the first
    moments of its rings over their total signed area (reading Q3)."""
    A = np.zeros(R + 1)
    Mx = np.zeros(R + 1)
    My = np.zeros(R + 1)
    for k in range(len(ring_reg)):
        ids = ring_idx[ring_off[k]:ring_off[k + 1]]
        p = xy[ids]
        q = np.roll(p, -1, axis=0)
        c = p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1]
        v = ring_reg[k]
        A[v] += 0.5 * c.sum()
        Mx[v] += np.sum((p[:, 0] + q[:, 0]) * c) / 6.0
        My[v] += np.sum((p[:, 1] + q[:, 1]) * c) / 6.0
    out = np.zeros((R + 1, 2))
    out[1:, 0] = Mx[1:] / A[1:]
    out[1:, 1] = My[1:] / A[1:]
    return out


def relative_position_error(b_map: np.ndarray, b_cart: np.ndarray) -> float:
    """R = sum over ordered pairs u != v of |angle(b_c(u,v), b_m(u,v))|
    / (pi |V| (|V| - 1)), with b(u,v) = b(v) - b(u) (rows 1.. of the
    barycentre arrays)."""
    bm = b_map[1:]
    bc = b_cart[1:]
    n = len(bm)
    if n < 2:
        return 0.0
    vm = bm[None, :, :] - bm[:, None, :]
    vc = bc[None, :, :] - bc[:, None, :]
    cross = vm[..., 0] * vc[..., 1] - vm[..., 1] * vc[..., 0]
    dot = vm[..., 0] * vc[..., 0] + vm[..., 1] * vc[..., 1]
    ang = np.abs(np.arctan2(cross, dot))
    np.fill_diagonal(ang, 0.0)
    return float(ang.sum() / (np.pi * n * (n - 1)))


# ----------------------------------------------------------------------------


def quality(m, xy_map, xy_cart, N: int, values=None) -> dict:
    """All measures of the cartogram xy_cart against the map xy_map at
    texture size N (and eps, xi when the region values are given)."""
    lm, _, _ = oc.rasterize(xy_map, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    lc, _, _ = oc.rasterize(xy_cart, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    tau, nm, nc, common = topology_distortion(lm, lc)
    H, hmean, hmax, best = shape_distortion(lm, lc, m.n_regions)
    bm = barycenters(xy_map, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
    bc = barycenters(xy_cart, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
    out = dict(tau=tau, adj_map=nm, adj_cart=nc, adj_common=common, shape=H, shape_mean=hmean, shape_max=hmax,
               best_overlap=best, rel_pos=relative_position_error(bm, bc), bary_map=bm, bary_cart=bc)
    if values is not None:
        A = oc.region_areas(xy_cart, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
        out["eps"], out["xi"] = oc.cartographic_errors(A, values)
    return out
