"""Seeded synthetic point clouds shared by the tests, the smoke check and the bench.

Holds none of the method's arithmetic: only random inputs and the parameter
sets of the workloads.  The paper measures on three scanned clouds (a NEON
aerial LiDAR tile, the Great Hall and Oplontis architectural scans) that are
not available here; these generators stand in for them with the same kinds of
structure: aerial terrain with dense clusters, architectural planes, and a
uniform cube as the easy case.

All generators use numpy's PCG64 with an explicit seed, produce float32 SoA
coordinates (x, y, z) in input ("scan") order and uint8 colours, and are exact
functions of (seed, n): the same call gives the same bytes on every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cloud:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    rgb: np.ndarray | None = None
    kind: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _split_exact(weights: np.ndarray, n: int) -> np.ndarray:
    """Largest-remainder rounding of n * weights / sum(weights) to integers summing to n."""
    w = np.asarray(weights, dtype=np.float64)
    q = n * w / w.sum()
    base = np.floor(q).astype(np.int64)
    rem = n - int(base.sum())
    if rem > 0:
        order = np.argsort(-(q - base), kind="stable")
        base[order[:rem]] += 1
    return base


def uniform(n: int, seed: int = 1, lo: float = 0.0, hi: float = 1.0, colors: bool = True) -> Cloud:
    """x, y, z ~ U[lo, hi) as float32; rgb ~ U{0..255}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = rng.random((3, n), dtype=np.float32)
    if lo != 0.0 or hi != 1.0:
        xyz = (np.float32(lo) + xyz * np.float32(hi - lo)).astype(np.float32)
    rgb = rng.integers(0, 256, size=(n, 3), dtype=np.uint8) if colors else None
    return Cloud(np.ascontiguousarray(xyz[0]), np.ascontiguousarray(xyz[1]),
                 np.ascontiguousarray(xyz[2]), rgb, "uniform")


def planes(n: int, seed: int = 2, num_planes: int = 200, box: float = 50.0,
           side_lo: float = 1.0, side_hi: float = 20.0, sigma: float = 0.005,
           colors: bool = True) -> Cloud:
    """Points on random rectangles (an architectural scan).

    Rectangle centre ~ U[0, box]^3, normal uniform on the sphere, side lengths
    ~ U[side_lo, side_hi] each; points per rectangle proportional to its area
    (exact total n); each point uniform on its rectangle plus isotropic
    Gaussian noise of standard deviation sigma.  Emitted rectangle by
    rectangle, the way a scanner sweeps surfaces.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centre = rng.uniform(0.0, box, size=(num_planes, 3))
    normal = rng.normal(size=(num_planes, 3))
    normal /= np.linalg.norm(normal, axis=1, keepdims=True)
    sides = rng.uniform(side_lo, side_hi, size=(num_planes, 2))
    helper = np.where(np.abs(normal[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    e1 = np.cross(normal, helper)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(normal, e1)
    counts = _split_exact(sides[:, 0] * sides[:, 1], n)
    x = np.empty(n, dtype=np.float32)
    y = np.empty(n, dtype=np.float32)
    z = np.empty(n, dtype=np.float32)
    pos = 0
    step = 4_000_000
    for k in range(num_planes):
        m = int(counts[k])
        done = 0
        while done < m:
            b = min(step, m - done)
            a = rng.uniform(-0.5, 0.5, size=(b, 1)) * sides[k, 0]
            c = rng.uniform(-0.5, 0.5, size=(b, 1)) * sides[k, 1]
            p = centre[k] + a * e1[k] + c * e2[k] + rng.normal(scale=sigma, size=(b, 3))
            x[pos:pos + b] = p[:, 0]
            y[pos:pos + b] = p[:, 1]
            z[pos:pos + b] = p[:, 2]
            pos += b
            done += b
    rgb = rng.integers(0, 256, size=(n, 3), dtype=np.uint8) if colors else None
    return Cloud(x, y, z, rgb, "planes", {"num_planes": num_planes})


def _value_noise_params(rng, octaves, base_wavelength, extent):
    grids = []
    for o in range(octaves):
        lam = base_wavelength / (2 ** o)
        cells = int(math.ceil(extent / lam)) + 2
        grids.append((lam, rng.random((cells, cells))))
    return grids


def _fbm(grids, px, py, gain=0.5):
    """fBm of value noise at (px, py): octaves of bilinear-smoothstep
    interpolated lattice values, amplitudes gain^o, normalised to [0, 1]."""
    h = np.zeros(px.shape[0], dtype=np.float32)
    amp = 1.0
    norm = 0.0
    for lam, g in grids:
        cells = g.shape[1]
        flat = g.astype(np.float32).ravel()
        fx = px * np.float32(1.0 / lam)
        fy = py * np.float32(1.0 / lam)
        ix = fx.astype(np.int32)          # px, py >= 0: truncation is floor
        iy = fy.astype(np.int32)
        tx = fx - ix
        ty = fy - iy
        tx = tx * tx * (3 - 2 * tx)
        ty = ty * ty * (3 - 2 * ty)
        i00 = ix * cells + iy
        v00 = flat.take(i00)
        v01 = flat.take(i00 + 1)
        v10 = flat.take(i00 + cells)
        v11 = flat.take(i00 + cells + 1)
        h += np.float32(amp) * ((v00 + (v10 - v00) * tx) * (1 - ty) + (v01 + (v11 - v01) * tx) * ty)
        norm += amp
        amp *= gain
    return h / np.float32(norm)


def terrain_clusters(n: int, seed: int = 3, extent: float = 1000.0, relief: float = 100.0,
                     cluster_fraction: float = 0.2, cluster_size: int = 8000,
                     cluster_sigma: float = 0.5, octaves: int = 8, base_wavelength: float = 250.0,
                     colors: bool = True, rgba: bool = True, block: int = 4_000_000, workers: int = 8) -> Cloud:
    """Aerial terrain (an fBm value-noise heightfield over [0, extent)^2 with the
    given relief) plus dense Gaussian clusters (vegetation, buildings) holding
    cluster_fraction of the points, each cluster_size points of standard
    deviation cluster_sigma, centred on the terrain plus U[0, 20] m of height.
    Terrain points come first (blocks of `block` points, block k drawn from
    PCG64([seed, 1, k]), so the result does not depend on `workers`), then
    the clusters one after another."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.Generator(np.random.PCG64([seed, 0]))
    grids = _value_noise_params(rng, octaves, base_wavelength, extent)
    n_cl_pts = int(round(n * cluster_fraction))
    num_clusters = max(1, int(round(n_cl_pts / cluster_size))) if n_cl_pts > 0 else 0
    n_terrain = n - n_cl_pts
    x = np.empty(n, dtype=np.float32)
    y = np.empty(n, dtype=np.float32)
    z = np.empty(n, dtype=np.float32)

    def terrain_block(k):
        lo = k * block
        b = min(block, n_terrain - lo)
        r = np.random.Generator(np.random.PCG64([seed, 1, k]))
        px = r.random(b, dtype=np.float32) * np.float32(extent)
        py = r.random(b, dtype=np.float32) * np.float32(extent)
        x[lo:lo + b] = px
        y[lo:lo + b] = py
        z[lo:lo + b] = _fbm(grids, px, py) * np.float32(relief)

    nblocks = (n_terrain + block - 1) // block
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        list(ex.map(terrain_block, range(nblocks)))
    if num_clusters:
        per = _split_exact(np.ones(num_clusters), n_cl_pts).astype(np.int64)
        cx = rng.uniform(0.0, extent, size=num_clusters).astype(np.float32)
        cy = rng.uniform(0.0, extent, size=num_clusters).astype(np.float32)
        cz = (_fbm(grids, cx, cy) * np.float32(relief)
              + rng.uniform(0.0, 20.0, size=num_clusters).astype(np.float32))
        noise = rng.normal(scale=cluster_sigma, size=(n_cl_pts, 3)).astype(np.float32)
        x[n_terrain:] = np.repeat(cx, per) + noise[:, 0]
        y[n_terrain:] = np.repeat(cy, per) + noise[:, 1]
        z[n_terrain:] = np.repeat(cz, per) + noise[:, 2]
    rgb = rng.integers(0, 256, size=(n, 4 if rgba else 3), dtype=np.uint8) if colors else None
    return Cloud(x, y, z, rgb, "terrain_clusters", {"num_clusters": num_clusters})


def clusters(n: int, seed: int, num_clusters: int, box: float = 50.0, sigma_frac: float = 0.01,
             colors: bool = True) -> Cloud:
    """Gaussian blobs of standard deviation sigma_frac * box, centres ~ U[0, box]^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per = _split_exact(np.ones(num_clusters), n)
    c = rng.uniform(0.0, box, size=(num_clusters, 3))
    x = np.empty(n, dtype=np.float32)
    y = np.empty(n, dtype=np.float32)
    z = np.empty(n, dtype=np.float32)
    pos = 0
    for k in range(num_clusters):
        m = int(per[k])
        p = c[k] + rng.normal(scale=sigma_frac * box, size=(m, 3))
        x[pos:pos + m] = p[:, 0]
        y[pos:pos + m] = p[:, 1]
        z[pos:pos + m] = p[:, 2]
        pos += m
    rgb = rng.integers(0, 256, size=(n, 3), dtype=np.uint8) if colors else None
    return Cloud(x, y, z, rgb, "clusters", {"num_clusters": num_clusters})


# ---- workload parameter sets -------------------------------------------------

@dataclass(frozen=True)
class BuildParams:
    count_grid: int
    max_points_per_chunk: int
    subsample_grid: int
    leaf_capacity: int = 10_000
    preview_modulus: int = 64


def params_for_size(n: int) -> BuildParams:
    """Per-cloud parameters for the batched and served mixes, by cloud size."""
    g = 64 if n < 1_000_000 else 128 if n < 3_000_000 else 256 if n < 16_000_000 else 512
    c = 100_000 if n < 4_000_000 else 1_000_000 if n < 32_000_000 else 2_000_000
    s = 32 if n < 4_000_000 else 128
    return BuildParams(g, c, s)


UNIFORM_1M = BuildParams(count_grid=64, max_points_per_chunk=100_000, subsample_grid=32)
PLANES_20M = BuildParams(count_grid=128, max_points_per_chunk=1_000_000, subsample_grid=128)
TERRAIN_200M = BuildParams(count_grid=512, max_points_per_chunk=2_000_000, subsample_grid=128)


def uniform_1m(n: int = 1_000_000) -> Cloud:
    """Plain build, uniform cube (1M points at full size)."""
    return uniform(n, seed=1)


def planes_20m(n: int = 20_000_000) -> Cloud:
    """Plain build, 200 random planes with 5 mm noise (20M points at full size)."""
    return planes(n, seed=2)


def terrain_200m(n: int = 200_000_000) -> Cloud:
    """Out-of-core build: terrain plus clusters (200M points at full size)."""
    return terrain_clusters(n, seed=3, colors=False)


def batch_mix(num_clouds: int = 256, seed: int = 4, lo: int = 10_000, hi: int = 4_000_000,
              scale: float = 1.0):
    """The batched workload: cloud sizes log-uniform in [lo, hi] (times scale),
    generator kind uniform over {uniform cube, planes (5-200), clusters (10-500)}.
    Returns a list of (Cloud, BuildParams)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=num_clouds))
    out = []
    for k in range(num_clouds):
        n = max(1, int(round(sizes[k] * scale)))
        kind = int(rng.integers(0, 3))
        sub = int(rng.integers(0, 2**31 - 1))
        if kind == 0:
            c = uniform(n, seed=sub, lo=0.0, hi=float(rng.uniform(1.0, 100.0)))
        elif kind == 1:
            c = planes(n, seed=sub, num_planes=int(rng.integers(5, 201)))
        else:
            c = clusters(n, seed=sub, num_clusters=int(rng.integers(10, 501)))
        out.append((c, params_for_size(int(round(sizes[k])))))
    return out


@dataclass(frozen=True)
class Request:
    """One served build request: the first n points of pool cloud `kind`,
    arriving `arrival` seconds after the first request (before scaling by the
    offered load)."""
    kind: int
    n: int
    arrival: float


def serve_trace(num_requests: int = 2000, seed: int = 5, lo: int = 100_000, hi: int = 50_000_000,
                pool_size: int = 0, mean_gap: float = 1.0):
    """The served workload: request sizes log-uniform in [lo, hi], generator
    kind uniform over {uniform cube, planes, clusters}, Poisson arrivals with
    mean gap `mean_gap` (rescaled by the caller to the offered load).  To keep
    host generation bounded, every request is a prefix (its first n points)
    of one pool cloud per kind of pool_size points (default hi); a prefix of
    a seeded cloud is itself a valid cloud.  Returns (pool, requests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = pool_size or hi
    pool = [uniform(m, seed=seed * 10 + 1, lo=0.0, hi=80.0, colors=False),
            planes(m, seed=seed * 10 + 2, num_planes=120, colors=False),
            clusters(m, seed=seed * 10 + 3, num_clusters=300, colors=False)]
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=num_requests))
    kinds = rng.integers(0, 3, size=num_requests)
    gaps = rng.exponential(mean_gap, size=num_requests)
    t = np.cumsum(gaps) - gaps[0]
    reqs = [Request(int(k), min(m, max(1, int(round(v)))), float(a)) for k, v, a in zip(kinds, sizes, t)]
    return pool, reqs

