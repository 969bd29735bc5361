"""Seeded synthetic 3D+time microscopy-like images and centre tracks.

The paper's data (zebrafish hind-brain windows of 30^3 x 23 frames and the
pectoral fin at 567x577x147 x 70 frames, Sec. 4) are not available; these
generators stand in for them with the same shapes and structure: bright
nuclei (spheres or randomly oriented ellipsoids) on a dark background,
moving between frames, with Gaussian or Poisson noise.

Every array is x-fastest with shape (t, z, y, x).  Centres are voxel
coordinates (x, y, z) of the voxel grid X = (i-1, j-1, k-1) plus a 0-based
frame index.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import os

import numpy as np

CENTRE_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("frame", "<i4")])


@dataclass
class Image4D:
    n: tuple                      # (N1, N2, N3, N4) = (x, y, z, t) interior sizes
    image: np.ndarray             # shape (N4, N3, N2, N1); float64 or uint8
    centres: np.ndarray           # CENTRE_DTYPE: ball centres (threshold / rescale)
    seeds: np.ndarray             # CENTRE_DTYPE: seeds of the initial function
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        n1, n2, n3, n4 = self.n
        return n1 * n2 * n3 * n4


def _tracks_to_centres(tracks: np.ndarray) -> np.ndarray:
    """tracks: (n_tracks, n_frames, 3) xyz -> flat CENTRE_DTYPE array, frame-major."""
    nt, nf, _ = tracks.shape
    out = np.zeros(nt * nf, dtype=CENTRE_DTYPE)
    t = np.asarray(tracks, dtype=np.float32).transpose(1, 0, 2).reshape(nt * nf, 3)
    out["x"], out["y"], out["z"] = t[:, 0], t[:, 1], t[:, 2]
    out["frame"] = np.repeat(np.arange(nf, dtype=np.int32), nt)
    return out


def _grid(n1, n2, n3):
    z, y, x = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


# ------------------------------------------------------------------ config 1


def spheres_cfg1(n=(24, 24, 24, 8), radius=5.0, n_spheres=3, noise_sigma=0.1,
                 geom_seed=1, noise_seed=2) -> Image4D:
    """Three spheres of radius 5 moving one voxel per frame along random unit
    directions, intensity 1.0 on 0.0, plus N(0, 0.1^2) noise.

    Starts uniform in [3, N-4]^3, directions uniform on the sphere; redrawn
    until every position lies in [3, N-4]^3 (a sphere may touch the border) and
    the spheres keep a distance >= 11 in every frame.  Ball centres and seeds
    follow sphere 0.
    """
    n1, n2, n3, n4 = n
    rng = np.random.default_rng(geom_seed)
    lo, hi = 3.0, min(n1, n2, n3) - 4.0
    for _ in range(200000):
        c0 = rng.uniform(lo, hi, size=(n_spheres, 3))
        d = rng.normal(size=(n_spheres, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        tr = c0[:, None, :] + np.arange(n4)[None, :, None] * d[:, None, :]
        if tr.min() < lo or tr.max() > hi:
            continue
        ok = True
        for a in range(n_spheres):
            for b in range(a + 1, n_spheres):
                if np.linalg.norm(tr[a] - tr[b], axis=1).min() < 11.0:
                    ok = False
        if ok:
            break
    else:
        raise RuntimeError("could not place the spheres")
    x, y, z = _grid(n1, n2, n3)
    img = np.zeros((n4, n3, n2, n1), dtype=np.float64)
    for f in range(n4):
        for m in range(n_spheres):
            c = tr[m, f]
            inside = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= radius * radius
            img[f][inside] = 1.0
    img += np.random.default_rng(noise_seed).normal(0.0, noise_sigma, size=img.shape)
    cen = _tracks_to_centres(tr[:1].astype(np.float32))
    return Image4D(n=tuple(n), image=img, centres=cen, seeds=cen.copy(),
                   meta=dict(config=1, tracks=tr, geom_seed=geom_seed, noise_seed=noise_seed))


# ----------------------------------------------------------- nuclei images


def _rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def _brownian(rng, c0, n_frames, sigma, lo, hi):
    tr = np.empty((n_frames, 3))
    tr[0] = c0
    for f in range(1, n_frames):
        c = tr[f - 1] + rng.normal(0.0, sigma, size=3)
        c = np.where(c < lo, 2 * lo - c, c)
        c = np.where(c > hi, 2 * hi - c, c)
        tr[f] = np.clip(c, lo, hi)
    return tr


def _paint(frame: np.ndarray, c, axes, rot, inten):
    """max-paint one ellipsoid (centre c xyz, semi-axes, rotation) into frame[z,y,x]."""
    n3, n2, n1 = frame.shape
    rr = int(np.ceil(max(axes))) + 1
    x0, x1 = max(0, int(np.floor(c[0])) - rr), min(n1, int(np.floor(c[0])) + rr + 2)
    y0, y1 = max(0, int(np.floor(c[1])) - rr), min(n2, int(np.floor(c[1])) + rr + 2)
    z0, z1 = max(0, int(np.floor(c[2])) - rr), min(n3, int(np.floor(c[2])) + rr + 2)
    if x0 >= x1 or y0 >= y1 or z0 >= z1:
        return
    z, y, x = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    p = np.stack([x - c[0], y - c[1], z - c[2]], axis=-1) @ rot
    inside = ((p / np.asarray(axes)) ** 2).sum(-1) <= 1.0
    sub = frame[z0:z1, y0:y1, x0:x1]
    np.maximum(sub, np.where(inside, inten, 0.0), out=sub)


def _paint_all(frame: np.ndarray, cs, axes, rots, intens, chunk=512):
    """max-paint many ellipsoids at once (same result as _paint for each)."""
    n3, n2, n1 = frame.shape
    rr = int(np.ceil(np.max(axes))) + 1
    o = np.arange(-rr, rr + 2)
    oz, oy, ox = np.meshgrid(o, o, o, indexing="ij")
    off = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=-1)          # (B, 3) xyz
    flat = frame.reshape(-1)
    for a in range(0, cs.shape[0], chunk):
        c = cs[a:a + chunk]
        X = np.floor(c)[:, None, :].astype(np.int64) + off[None, :, :]    # (M, B, 3)
        ok = ((X[..., 0] >= 0) & (X[..., 0] < n1) & (X[..., 1] >= 0) & (X[..., 1] < n2)
              & (X[..., 2] >= 0) & (X[..., 2] < n3))
        p = np.einsum("mbi,mij->mbj", X - c[:, None, :], rots[a:a + chunk])
        inside = ok & (((p / axes[a:a + chunk, None, :]) ** 2).sum(-1) <= 1.0)
        idx = (X[..., 2] * n2 + X[..., 1]) * n1 + X[..., 0]
        val = np.broadcast_to(intens[a:a + chunk, None], inside.shape)
        np.maximum.at(flat, idx[inside], val[inside])


def _nuclei_image(n, tracks, axes, rots, intens, background, noise_seed):
    """Paint every frame, then draw Poisson noise with one generator per frame
    (spawned from `noise_seed`, so the result does not depend on the number of
    worker threads)."""
    n1, n2, n3, n4 = n
    img = np.empty((n4, n3, n2, n1), dtype=np.uint8)
    seeds = np.random.SeedSequence(noise_seed).spawn(n4)

    def one(f):
        fr = np.full((n3, n2, n1), float(background), dtype=np.float64)
        _paint_all(fr, tracks[:, f, :], axes, rots, intens)
        rng = np.random.default_rng(seeds[f])
        img[f] = np.minimum(rng.poisson(fr), 255).astype(np.uint8)

    if n1 * n2 * n3 * n4 < (1 << 22):
        for f in range(n4):
            one(f)
    else:
        from concurrent.futures import ThreadPoolExecutor
        import os
        with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1, n4))) as ex:
            list(ex.map(one, range(n4)))
    return img


def nuclei_cfg2(n=(512, 512, 96, 16), n_nuclei=2000, geom_seed=11, noise_seed=12,
                sigma=1.5, background=20.0) -> Image4D:
    """~2000 ellipsoidal nuclei (semi-axes U[3,6], random orientation, intensity
    U[120,220]) on background 20, Brownian motion sigma=1.5 voxel/frame
    reflected at the margins, Poisson noise, uint8 (one GPU's share of the
    pectoral-fin shape of Sec. 4).  Every track is a ball centre and a seed."""
    n1, n2, n3, n4 = n
    rng = np.random.default_rng(geom_seed)
    lo = np.array([6.0, 6.0, 6.0])
    hi = np.array([n1 - 7.0, n2 - 7.0, n3 - 7.0])
    c0 = rng.uniform(lo, hi, size=(n_nuclei, 3))
    axes = rng.uniform(3.0, 6.0, size=(n_nuclei, 3))
    rots = np.stack([_rotation(rng) for _ in range(n_nuclei)])
    intens = rng.uniform(120.0, 220.0, size=n_nuclei)
    tracks = np.stack([_brownian(rng, c0[m], n4, sigma, lo, hi) for m in range(n_nuclei)])
    img = _nuclei_image(n, tracks, axes, rots, intens, background, noise_seed)
    cen = _tracks_to_centres(tracks.astype(np.float32))
    return Image4D(n=tuple(n), image=img, centres=cen, seeds=cen.copy(),
                   meta=dict(config=2, geom_seed=geom_seed, noise_seed=noise_seed))


def window_job(n, geom_seed, noise_seed, sigma=1.5, background=20.0, extra_rate=2.0) -> Image4D:
    """One per-nucleus window (the paper cuts 30^3 windows around nuclei, Sec. 4):
    a central ellipsoidal nucleus with Brownian drift plus Poisson(2) extra
    nuclei at uniform positions, background 20, Poisson noise, uint8.  The
    ball centre and seed follow the central nucleus."""
    n1, n2, n3, n4 = n
    rng = np.random.default_rng(geom_seed)
    mid = np.array([(n1 - 1) / 2.0, (n2 - 1) / 2.0, (n3 - 1) / 2.0])
    lo = np.maximum(mid - 4.0, 0.0)
    hi = mid + 4.0
    k = 1 + int(rng.poisson(extra_rate))
    c0 = np.empty((k, 3))
    c0[0] = mid
    c0[1:] = rng.uniform([0, 0, 0], [n1 - 1, n2 - 1, n3 - 1], size=(k - 1, 3))
    axes = rng.uniform(3.0, 6.0, size=(k, 3))
    rots = np.stack([_rotation(rng) for _ in range(k)])
    intens = rng.uniform(120.0, 220.0, size=k)
    tracks = np.empty((k, n4, 3))
    tracks[0] = _brownian(rng, c0[0], n4, sigma, lo, hi)
    big = np.array([n1 - 1.0, n2 - 1.0, n3 - 1.0])
    for m in range(1, k):
        tracks[m] = _brownian(rng, c0[m], n4, sigma, np.zeros(3), big)
    img = _nuclei_image(n, tracks, axes, rots, intens, background, noise_seed)
    cen = _tracks_to_centres(tracks[:1].astype(np.float32))
    return Image4D(n=tuple(n), image=img, centres=cen, seeds=cen.copy(),
                   meta=dict(geom_seed=geom_seed, noise_seed=noise_seed))


def _pool_map(fn, items):
    """map over a thread pool: windows are independent and seeded per job, so
    the output does not depend on the number of threads"""
    from concurrent.futures import ThreadPoolExecutor

    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, items))


def _cfg4_window(j):
    r = np.random.default_rng(1000 + j)
    n = (int(r.integers(24, 65)), int(r.integers(24, 65)), int(r.integers(24, 65)), int(r.integers(3, 10)))
    return window_job(n, 1000 + j, 100000 + j)


def windows_cfg4(count=2048, first=0):
    """Batched workload: window j has x,y,z ~ U{24..64}, t ~ U{3..9} (seed 1000+j),
    content seeds 1000+j (geometry) and 100000+j (noise)."""
    return _pool_map(_cfg4_window, range(first, first + count))


def serving_windows(sizes, first_job=0):
    """Images of serving jobs first_job, first_job+1, ... with the given sizes
    (content seeds 200000+j and 300000+j)."""
    return _pool_map(lambda q: window_job(sizes[q], 200000 + first_job + q, 300000 + first_job + q),
                     range(len(sizes)))


def serving_stream(rate, count, seed=7, median=(40, 40, 40, 5), log_sigma=0.4,
                   lo=(17, 17, 17, 2), hi=(96, 96, 96, 12), first_job=0):
    """Serving workload: Poisson arrivals at `rate` jobs/s (seed 7), window sizes
    lognormal around `median` (log-sigma 0.4) clamped to [lo, hi]; job j has
    content seeds 200000+j.  Returns (arrival_times_s, list of sizes); images are
    drawn lazily with `window_job(size, 200000+j, 300000+j)`."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    sizes = []
    for _ in range(count):
        s = tuple(int(np.clip(np.rint(m * np.exp(rng.normal(0.0, log_sigma))), a, b))
                  for m, a, b in zip(median, lo, hi))
        sizes.append(s)
    return t, sizes
