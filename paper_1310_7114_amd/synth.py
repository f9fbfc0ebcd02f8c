"""Seeded synthetic inputs: lattice weight images and initial codebooks.

This module only draws and rasterises inputs. It holds none of the clustering
arithmetic (no kernels, no maps, no updates), so the FP64 oracle and the HIP
path can both be fed from it without sharing computation.

The paper's data model (Section 3.2): a binary image is a set of lattice points
[u, v] with u the row and v the column; pixel centres sit at integer
coordinates. Gray images carry a per-pixel weight h(x) = g/255 (Section 5).
The paper timed on the MPEG-7 shape set, which is not available here; the
silhouette generators below stand in for it with shapes of similar size and
structure. Nothing from that set is reproduced.

Every image i of workload c is drawn from ``SeedSequence([c, i])``; the initial
codebook of that image from ``SeedSequence([c, i, 1])`` (Algorithm 1 draws the
initial codevectors from the foreground pixels; the draw happens here and the
result is passed to both sides).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "rng_for", "fill_ellipse", "fill_star_polygon", "star_polygon_vertices",
    "ellipses_union", "shapes_union", "star_silhouette", "gray_gaussians",
    "sample_init", "LatticeCase", "config1_case", "config2_case", "config3_cases",
    "config3_spec", "config3_specs", "config4_case", "config5_cases",
]


def rng_for(*key: int) -> np.random.Generator:
    """Counter-keyed PCG64 generator; the key names (workload, image[, stream])."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


# ----------------------------------------------------------------------------
# rasterisation (pixel centres at integer (u, v))
# ----------------------------------------------------------------------------

def fill_ellipse(mask: np.ndarray, cu: float, cv: float, a: float, b: float,
                 angle: float) -> None:
    """OR a filled ellipse (semi-axes a, b, rotated by ``angle``) into ``mask``."""
    H, W = mask.shape
    r = max(a, b) + 1.0
    u0, u1 = max(0, int(math.floor(cu - r))), min(H, int(math.ceil(cu + r)) + 1)
    v0, v1 = max(0, int(math.floor(cv - r))), min(W, int(math.ceil(cv + r)) + 1)
    if u0 >= u1 or v0 >= v1:
        return
    uu, vv = np.meshgrid(np.arange(u0, u1, dtype=np.float64) - cu,
                         np.arange(v0, v1, dtype=np.float64) - cv, indexing="ij")
    ca, sa = math.cos(angle), math.sin(angle)
    p = (uu * ca + vv * sa) / a
    q = (-uu * sa + vv * ca) / b
    mask[u0:u1, v0:v1] |= (p * p + q * q) <= 1.0


def star_polygon_vertices(rng: np.random.Generator, cu: float, cv: float,
                          rmax: float, kmin: int = 5, kmax: int = 24) -> np.ndarray:
    """Vertices (K, 2) of a star-shaped polygon: sorted angles, radii U[0.3,1]*rmax."""
    K = int(rng.integers(kmin, kmax + 1))
    ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=K))
    rad = rng.uniform(0.3, 1.0, size=K) * rmax
    return np.stack([cu + rad * np.cos(ang), cv + rad * np.sin(ang)], axis=1)


def fill_star_polygon(mask: np.ndarray, verts: np.ndarray) -> None:
    """OR a polygon into ``mask`` by the even-odd rule at pixel centres.

    Scanline form: on row u, an edge (a, b) crosses when exactly one endpoint
    lies on or below u (half-open in u, so shared vertices count once); pixel v
    is inside when an odd number of crossings lie strictly to its right, i.e.
    for sorted crossings c0 < c1 < ..., inside iff c_{2m} <= v < c_{2m+1}.
    """
    H, W = mask.shape
    ua, va = verts[:, 0], verts[:, 1]
    ub, vb = np.roll(ua, -1), np.roll(va, -1)
    lo = max(0, int(math.ceil(ua.min())))
    hi = min(H - 1, int(math.floor(ua.max())))
    if lo > hi:
        return
    rows = np.arange(lo, hi + 1, dtype=np.float64)[:, None]           # (nr, 1)
    cond = ((ua[None, :] <= rows) & (ub[None, :] > rows)) | \
           ((ub[None, :] <= rows) & (ua[None, :] > rows))
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (rows - ua[None, :]) / (ub - ua)[None, :]
        vc = va[None, :] + t * (vb - va)[None, :]
    vc = np.where(cond, vc, np.inf)
    vc.sort(axis=1)
    ncross = cond.sum(axis=1)
    diff = np.zeros((hi - lo + 1, W + 1), dtype=np.int32)
    for m in range(0, vc.shape[1] - 1, 2):
        ok = ncross > m + 1
        if not ok.any():
            break
        r_idx = np.nonzero(ok)[0]
        s = np.clip(np.ceil(vc[r_idx, m]), 0, W).astype(np.int64)
        e = np.clip(np.ceil(vc[r_idx, m + 1]), 0, W).astype(np.int64)
        np.add.at(diff, (r_idx, s), 1)
        np.add.at(diff, (r_idx, e), -1)
    mask[lo:hi + 1, :] |= np.cumsum(diff, axis=1)[:, :W] > 0


def _interior(H: int, W: int, margin: int) -> np.ndarray:
    keep = np.zeros((H, W), dtype=bool)
    keep[margin:H - margin, margin:W - margin] = True
    return keep


# ----------------------------------------------------------------------------
# image generators
# ----------------------------------------------------------------------------

def ellipses_union(seed_key, H: int = 64, W: int = 64, n: int = 3,
                   centre=(18.0, 46.0), semi=(10.0, 20.0), margin: int = 7,
                   count=(1300, 1700)) -> np.ndarray:
    """Binary union of ``n`` filled ellipses, clipped to a border margin.

    Redrawn until the on-pixel count lies in ``count``. The margin keeps every
    datum at least R+1 pixels from the lattice edge for R = margin - 1.
    """
    rng = rng_for(*seed_key)
    keep = _interior(H, W, margin)
    for _ in range(10000):
        m = np.zeros((H, W), dtype=bool)
        for _ in range(n):
            cu, cv = rng.uniform(*centre, size=2)
            a, b = rng.uniform(*semi, size=2)
            fill_ellipse(m, cu, cv, a, b, rng.uniform(0.0, math.pi))
        m &= keep
        if count[0] <= int(m.sum()) <= count[1]:
            return m.astype(np.uint8)
    raise RuntimeError("ellipses_union: no draw met the on-pixel count")


def shapes_union(seed_key, H: int = 512, W: int = 512, n: int = 20, margin: int = 13,
                 cover=(0.25, 0.35)) -> np.ndarray:
    """Binary union of ``n`` shapes (ellipse or star polygon, p = 1/2 each).

    Centres are uniform at least ``margin`` from the edge; each shape's mean
    area is about 4.7k px so that 20 of them cover roughly 30% of 512x512.
    Redrawn until the covered fraction lies in ``cover``.
    """
    rng = rng_for(*seed_key)
    keep = _interior(H, W, margin)
    for _ in range(1000):
        m = np.zeros((H, W), dtype=bool)
        for _ in range(n):
            cu = rng.uniform(margin, H - 1 - margin)
            cv = rng.uniform(margin, W - 1 - margin)
            if rng.uniform() < 0.5:
                a, b = rng.uniform(25.0, 55.0, size=2)
                fill_ellipse(m, cu, cv, a, b, rng.uniform(0.0, math.pi))
            else:
                fill_star_polygon(m, star_polygon_vertices(rng, cu, cv, rng.uniform(45.0, 75.0)))
        m &= keep
        f = m.mean()
        if cover[0] <= f <= cover[1]:
            return m.astype(np.uint8)
    raise RuntimeError("shapes_union: no draw met the coverage band")


def star_silhouette(seed_key, H: int, W: int, R: int) -> np.ndarray:
    """One centred star-shaped polygon filling most of an H x W frame.

    Radii are U[0.3, 1] * (min(H, W)/2 - R - 2), so every on-pixel keeps at least
    R + 1 pixels to the edge.
    """
    rng = rng_for(*seed_key)
    m = np.zeros((H, W), dtype=bool)
    rmax = min(H, W) / 2.0 - R - 2.0
    fill_star_polygon(m, star_polygon_vertices(rng, (H - 1) / 2.0, (W - 1) / 2.0, rmax))
    return m.astype(np.uint8)


def gray_gaussians(seed_key, H: int = 2048, W: int = 2048, n: int = 50,
                   amp=(30.0, 120.0), major=(20.0, 200.0), noise: int = 8) -> np.ndarray:
    """uint8 field: sum of ``n`` anisotropic Gaussian bumps plus integer noise.

    Bump: amplitude U[amp], major std U[major], minor std = major * U[0.2, 1],
    orientation U[0, pi), centre U[0, H) x U[0, W). Each bump is evaluated on the
    box of +-4 major stds around its centre (beyond it the bump is < 0.04 gray
    levels). Noise is U{-noise..noise}; the sum is rounded and clipped to 0..255.
    """
    rng = rng_for(*seed_key)
    f = np.zeros((H, W), dtype=np.float32)
    for _ in range(n):
        A = rng.uniform(*amp)
        s1 = rng.uniform(*major)
        s2 = s1 * rng.uniform(0.2, 1.0)
        th = rng.uniform(0.0, math.pi)
        cu, cv = rng.uniform(0.0, H), rng.uniform(0.0, W)
        r = 4.0 * s1
        u0, u1 = max(0, int(cu - r)), min(H, int(cu + r) + 1)
        v0, v1 = max(0, int(cv - r)), min(W, int(cv + r) + 1)
        if u0 >= u1 or v0 >= v1:
            continue
        du = (np.arange(u0, u1, dtype=np.float32) - np.float32(cu))[:, None]
        dv = (np.arange(v0, v1, dtype=np.float32) - np.float32(cv))[None, :]
        c, s = np.float32(math.cos(th)), np.float32(math.sin(th))
        p = (du * c + dv * s) / np.float32(s1)
        q = (-du * s + dv * c) / np.float32(s2)
        f[u0:u1, v0:v1] += np.float32(A) * np.exp(np.float32(-0.5) * (p * p + q * q))
    f += rng.integers(-noise, noise + 1, size=(H, W)).astype(np.float32)
    return np.clip(np.rint(f), 0, 255).astype(np.uint8)


def sample_init(img: np.ndarray, M: int, seed_key, jitter=None) -> np.ndarray:
    """M distinct lattice points with img > 0, uniform without replacement.

    Returns an (M, 2) float64 array of (u, v). With ``jitter=(lo, hi)`` each
    coordinate gets a U[lo, hi) offset (keeps codevectors off integer cells).
    """
    rng = rng_for(*seed_key)
    on = np.flatnonzero(img.reshape(-1) > 0)
    if on.size < M:
        raise ValueError(f"sample_init: {on.size} on-pixels < M={M}")
    pick = rng.choice(on, size=M, replace=False)
    W = img.shape[1]
    w = np.stack([pick // W, pick % W], axis=1).astype(np.float64)
    if jitter is not None:
        w += rng.uniform(jitter[0], jitter[1], size=w.shape)
    return w


def ellipsoids_volume(seed_key, D: int, H: int, W: int, n: int = 4, margin: int = 7,
                      semi=(0.12, 0.3), cover=(0.04, 0.25)) -> np.ndarray:
    """Binary union of ``n`` axis-rotated filled ellipsoids in a D x H x W volume.

    Centres uniform in the interior, semi-axes U[semi] times the smallest
    extent, each ellipsoid rotated about the slice axis by U[0, pi); voxels
    within ``margin`` of a face are cleared. Redrawn until the on-voxel
    fraction lies in ``cover``.
    """
    rng = rng_for(*seed_key)
    s, u, v = np.meshgrid(np.arange(D, dtype=np.float64), np.arange(H, dtype=np.float64),
                          np.arange(W, dtype=np.float64), indexing="ij")
    keep = ((s >= margin) & (s < D - margin) & (u >= margin) & (u < H - margin) & (v >= margin)
            & (v < W - margin))
    ext = float(min(D, H, W))
    for _ in range(1000):
        m = np.zeros((D, H, W), dtype=bool)
        for _ in range(n):
            c = [rng.uniform(margin, n_ - margin) for n_ in (D, H, W)]
            a, b, cax = rng.uniform(semi[0] * ext, semi[1] * ext, size=3)
            th = rng.uniform(0.0, math.pi)
            du, dv = u - c[1], v - c[2]
            pu = math.cos(th) * du + math.sin(th) * dv
            pv = -math.sin(th) * du + math.cos(th) * dv
            m |= ((s - c[0]) / a) ** 2 + (pu / b) ** 2 + (pv / cax) ** 2 <= 1.0
        m &= keep
        if cover[0] <= float(m.mean()) <= cover[1]:
            return m.astype(np.uint8)
    raise RuntimeError("ellipsoids_volume: no draw met the coverage")


def sample_init_volume(vol: np.ndarray, M: int, seed_key) -> np.ndarray:
    """M distinct voxels with vol > 0, uniform without replacement: (M, 3) float64 of (s, u, v)."""
    rng = rng_for(*seed_key)
    on = np.flatnonzero(vol.reshape(-1) > 0)
    if on.size < M:
        raise ValueError(f"sample_init_volume: {on.size} on-voxels < M={M}")
    pick = rng.choice(on, size=M, replace=False)
    D, H, W = vol.shape
    return np.stack([pick // (H * W), (pick // W) % H, pick % W], axis=1).astype(np.float64)


@dataclass
class VolumeCase:
    """One clustering problem on a 3-D lattice: weights = scale * vol."""
    vol: np.ndarray            # (D, H, W) uint8 stored weights
    scale: float
    w0: np.ndarray             # (M, 3) float64 initial codebook (s, u, v)
    sigma: float
    R: int
    iters: int
    name: str = ""

    @property
    def weights(self) -> np.ndarray:
        return self.vol.astype(np.float64) * self.scale

    @property
    def M(self) -> int:
        return int(self.w0.shape[0])


def volume_case(seed: int = 0, D: int = 48, H: int = 56, W: int = 64, M: int = 24, sigma: float = 2.0,
                iters: int = 30) -> VolumeCase:
    """Ellipsoids in a D x H x W volume, M codevectors on on-voxels."""
    vol = ellipsoids_volume((6, seed), D, H, W)
    return VolumeCase(vol, 1.0, sample_init_volume(vol, M, (6, seed, 1)), sigma, radius_for(sigma), iters,
                      name=f"ellipsoids{D}x{H}x{W}-s{seed}")


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

@dataclass
class LatticeCase:
    """One clustering problem: weights = scale * img, codebook init, kernel width."""
    img: np.ndarray            # (H, W) uint8 stored weights
    scale: float               # h = scale * img
    w0: np.ndarray             # (M, 2) float64 initial codebook (u, v)
    sigma: float
    R: int
    iters: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def weights(self) -> np.ndarray:
        return self.img.astype(np.float64) * self.scale

    @property
    def M(self) -> int:
        return int(self.w0.shape[0])


def radius_for(sigma: float) -> int:
    """Truncation radius of the Gaussian window: ceil(3 sigma)."""
    return int(math.ceil(3.0 * sigma - 1e-12))


def config1_case(seed: int = 1) -> LatticeCase:
    """64x64 binary, union of 3 ellipses (~1.5k on-pixels), M=16, sigma=2, 50 iters."""
    img = ellipses_union((1, seed))
    return LatticeCase(img, 1.0, sample_init(img, 16, (1, seed, 1)), 2.0, 6, 50,
                       name=f"ellipses64-s{seed}")


def config2_case(seed: int = 0) -> LatticeCase:
    """512x512 binary, union of 20 ellipses/star polygons (~30%), M=100, sigma=4."""
    img = shapes_union((2, seed))
    return LatticeCase(img, 1.0, sample_init(img, 100, (2, seed, 1)), 4.0, 12, 100,
                       name=f"shapes512-s{seed}")


def config3_spec(i: int):
    """(H, W, M, sigma) of silhouette i: W in 128..1024, H in 128..768, M in 10..200."""
    rng = rng_for(3, i)
    Wd = int(rng.integers(128, 1025))
    Hd = int(rng.integers(128, 769))
    M = int(rng.integers(10, 201))
    sigma = float(rng.choice([2.0, 4.0, 8.0]))
    return Hd, Wd, M, sigma


def config3_specs(n: int = 1400):
    """Per-image (H, W, M, sigma) of the silhouette batch, drawn before rasterising."""
    return [config3_spec(i) for i in range(n)]


def config3_cases(n: int = 1400, indices=None) -> list:
    """The batch of star silhouettes (sizes 128..768 x 128..1024), 100 iters each."""
    idx = range(n) if indices is None else indices
    out = []
    for i in idx:
        Hd, Wd, M, sigma = config3_spec(i)
        R = radius_for(sigma)
        img = star_silhouette((3, i, 2), Hd, Wd, R)
        out.append(LatticeCase(img, 1.0, sample_init(img, M, (3, i, 1)), sigma, R, 100,
                               name=f"silhouette-{i}", meta={"index": i}))
    return out


def config4_case(seed: int = 0) -> LatticeCase:
    """2048x2048 gray field (50 bumps + noise), weight g/255, M=500, sigma=6, 200 iters."""
    img = gray_gaussians((4, seed))
    return LatticeCase(img, 1.0 / 255.0, sample_init(img, 500, (4, seed, 1)), 6.0, 18, 200,
                       name=f"gray2048-s{seed}")


def config5_cases(n: int = 64, indices=None, H: int = 1024, W: int = 1024) -> list:
    """Batch of 1024x1024 gray fields (bump stds halved), M=256, sigma=4, jittered init."""
    idx = range(n) if indices is None else indices
    out = []
    for i in idx:
        img = gray_gaussians((5, i), H=H, W=W, major=(10.0, 100.0))
        w0 = sample_init(img, 256, (5, i, 1), jitter=(0.05, 0.95))
        out.append(LatticeCase(img, 1.0 / 255.0, w0, 4.0, 12, 0, name=f"gray1024-{i}",
                               meta={"index": i}))
    return out
