"""Seeded synthetic particle sets standing in for the paper's datasets.

Pure input generation: this module holds none of the compressor's arithmetic
and is shared by the tests, the benchmark and the CPU oracle checks.  Every
generator draws with numpy's PCG64 in float64 and rounds to float32 once, in
fixed-size chunks (``CHUNK`` particles, one spawned stream per chunk), so a
given (seed, size) always yields the same arrays on any machine.

The paper's datasets (HACC cosmology, LAMMPS molecular dynamics, USGS 3DEP
LiDAR, ...) are not available; these sets have their shapes, value
distributions and storage order instead:

* ``clusters``  -- Gaussian clusters plus a uniform background in the unit
  cube (small parity workload, and the batched-form snapshots);
* ``cosmology`` -- halos in a periodic box with per-halo bulk velocities;
* ``md``        -- a jittered FCC lattice with Gaussian velocities;
* ``lidar``     -- a fractal-Brownian terrain tile with sensor noise.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from typing import List

import numpy as np

CHUNK = 1 << 22  # particles per generator chunk


def _chunks(n: int):
    for start in range(0, n, CHUNK):
        yield start, min(CHUNK, n - start)


def _workers() -> int:
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return max(1, min(16, cores))


def _run_chunks(body, n: int):
    """Calls body(ci, start, count) for every chunk, on a pool of host
    threads.  Each chunk draws from its own spawned stream and writes its own
    slice of the outputs, so the arrays do not depend on the thread count or
    on the order in which chunks finish."""
    chunks = list(enumerate(_chunks(n)))
    if len(chunks) <= 1:
        for ci, (s, m) in chunks:
            body(ci, s, m)
        return
    with ThreadPoolExecutor(min(_workers(), len(chunks))) as ex:
        list(ex.map(lambda c: body(c[0], *c[1]), chunks))


def _streams(seed: int, count: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in
            np.random.SeedSequence(seed).spawn(count + 1)]


def clusters(n: int = 1_000_000, seed: int = 0, n_clusters: int = 64, sigma: float = 0.01,
             background: float = 0.2, extra_fields: int = 0, labels: np.ndarray | None = None
             ) -> List[np.ndarray]:
    """Positions in [0,1)^3: a mixture of ``n_clusters`` isotropic Gaussians
    (equal weights, centres uniform in the cube) plus a ``background``
    fraction of uniform points; coordinates wrap periodically.  Particles
    appear in draw order (labels i.i.d. per particle).  ``extra_fields``
    standard-normal attribute fields follow x, y, z.  ``labels`` (n int32,
    optional) receives each particle's cluster, ``n_clusters`` for the
    background."""
    nch = (n + CHUNK - 1) // CHUNK
    rs = _streams(seed, nch)
    centres = rs[0].random((n_clusters, 3))
    out = [np.empty(n, np.float32) for _ in range(3 + extra_fields)]

    def body(ci, s, m):
        r = rs[ci + 1]
        lab = r.integers(0, n_clusters, m)
        bg = r.random(m) < background
        if labels is not None:
            labels[s:s + m] = np.where(bg, n_clusters, lab)
        p = centres[lab] + sigma * r.standard_normal((m, 3))
        p[bg] = r.random((int(bg.sum()), 3))
        p = np.mod(p, 1.0)
        p32 = p.astype(np.float32)
        p32[p32 >= np.float32(1.0)] = np.float32(0.0)
        for a in range(3):
            out[a][s:s + m] = p32[:, a]
        for e in range(extra_fields):
            out[3 + e][s:s + m] = r.standard_normal(m).astype(np.float32)
    _run_chunks(body, n)
    return out


def cosmology(n: int = 64_000_000, seed: int = 1, box: float = 256.0, n_halos: int = 4096,
              background: float = 0.3, vsig: float = 300.0, labels: np.ndarray | None = None
              ) -> List[np.ndarray]:
    """x, y, z, vx, vy, vz of a HACC-like snapshot: halo centres uniform in a
    periodic box, halo widths log-uniform in [0.1, 2], 30 % uniform
    background; velocities = per-halo bulk velocity ~ N(0, vsig^2) per axis
    (zero for the background) plus N(0, vsig^2) dispersion.  ``labels`` (n
    int32, optional) receives each particle's halo, ``n_halos`` for the
    background."""
    nch = (n + CHUNK - 1) // CHUNK
    rs = _streams(seed, nch)
    cen = rs[0].random((n_halos, 3)) * box
    sig = np.exp(rs[0].uniform(np.log(0.1), np.log(2.0), n_halos))
    bulk = rs[0].standard_normal((n_halos, 3)) * vsig
    out = [np.empty(n, np.float32) for _ in range(6)]

    def body(ci, s, m):
        r = rs[ci + 1]
        lab = r.integers(0, n_halos, m)
        bg = r.random(m) < background
        if labels is not None:
            labels[s:s + m] = np.where(bg, n_halos, lab)
        p = cen[lab] + sig[lab, None] * r.standard_normal((m, 3))
        p[bg] = r.random((int(bg.sum()), 3)) * box
        p = np.mod(p, box)
        v = bulk[lab] + vsig * r.standard_normal((m, 3))
        v[bg] -= bulk[lab[bg]]
        p32 = p.astype(np.float32)
        p32[p32 >= np.float32(box)] = np.float32(0.0)
        for a in range(3):
            out[a][s:s + m] = p32[:, a]
            out[3 + a][s:s + m] = v[:, a].astype(np.float32)
    _run_chunks(body, n)
    return out


def md(cells: int = 200, seed: int = 2, a: float = 1.0, jitter: float = 0.05,
       n: int | None = None) -> List[np.ndarray]:
    """x, y, z, vx, vy, vz of a LAMMPS-like crystal: 4*cells^3 atoms on an
    FCC lattice of constant ``a`` with N(0, jitter^2) displacements, stored
    in lattice order (z, y, x, then basis atom fastest); velocities N(0,1).
    ``n`` truncates to the first n atoms."""
    total = 4 * cells ** 3
    n = total if n is None else min(n, total)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    nch = (n + CHUNK - 1) // CHUNK
    rs = _streams(seed, nch)
    out = [np.empty(n, np.float32) for _ in range(6)]

    def body(ci, s, m):
        r = rs[ci + 1]
        i = np.arange(s, s + m, dtype=np.int64)
        b = i % 4
        cell = i // 4
        ix = cell % cells
        iy = (cell // cells) % cells
        iz = cell // (cells * cells)
        p = (np.stack([ix, iy, iz], 1) + basis[b]) * a + jitter * r.standard_normal((m, 3))
        v = r.standard_normal((m, 3))
        for k in range(3):
            out[k][s:s + m] = p[:, k].astype(np.float32)
            out[3 + k][s:s + m] = v[:, k].astype(np.float32)
    _run_chunks(body, n)
    return out


def _value_noise(rng, x, y, wavelength, extent):
    cells = int(np.ceil(extent / wavelength)) + 2
    lat = rng.random((cells + 1, cells + 1)) * 2.0 - 1.0
    gx, gy = x / wavelength, y / wavelength
    ix, iy = np.floor(gx).astype(np.int64), np.floor(gy).astype(np.int64)
    fx, fy = gx - ix, gy - iy
    sx, sy = fx * fx * (3 - 2 * fx), fy * fy * (3 - 2 * fy)
    v00, v10 = lat[ix, iy], lat[ix + 1, iy]
    v01, v11 = lat[ix, iy + 1], lat[ix + 1, iy + 1]
    return (v00 * (1 - sx) + v10 * sx) * (1 - sy) + (v01 * (1 - sx) + v11 * sx) * sy


def lidar(n: int = 100_000_000, seed: int = 3, extent: float = 10_000.0, octaves: int = 8,
          amplitude: float = 200.0, base_wavelength: float = 2500.0, noise: float = 0.05
          ) -> List[np.ndarray]:
    """x, y uniform over an extent x extent tile; z = fractal Brownian height
    (``octaves`` octaves of seeded value noise, lacunarity 2, gain 0.5,
    octave amplitudes summing to ``amplitude``) + N(0, noise^2)."""
    nch = (n + CHUNK - 1) // CHUNK
    rs = _streams(seed, nch)
    lat_rngs = [np.random.Generator(np.random.PCG64(s)) for s in
                np.random.SeedSequence(seed + 1000).spawn(octaves)]
    amps = np.array([0.5 ** o for o in range(octaves)])
    amps *= amplitude / amps.sum()
    # lattice values are drawn once per octave and reused for every chunk
    lat_states = [r.bit_generator.state for r in lat_rngs]
    out = [np.empty(n, np.float32) for _ in range(3)]

    def body(ci, s, m):
        r = rs[ci + 1]
        x = r.random(m) * extent
        y = r.random(m) * extent
        z = np.zeros(m)
        for o in range(octaves):
            lr = np.random.Generator(np.random.PCG64())
            lr.bit_generator.state = lat_states[o]
            z += amps[o] * _value_noise(lr, x, y, base_wavelength / 2 ** o, extent)
        z += noise * r.standard_normal(m)
        out[0][s:s + m] = x.astype(np.float32)
        out[1][s:s + m] = y.astype(np.float32)
        out[2][s:s + m] = z.astype(np.float32)
    _run_chunks(body, n)
    return out


def request_stream(count: int = 20_000, seed: int = 5, rate: float = 2000.0, n_min: int = 100_000,
                   n_max: int = 32_000_000, scale: float = 1.0):
    """Serving-form arrivals: Poisson process of ``rate`` requests/s; each
    request has a size log-uniform in [n_min, n_max] (times ``scale``), a
    generator kind in {clusters, cosmology, md, lidar}, a relative bound in
    {1e-2, 1e-3, 1e-4} and an operation (compress or decompress, 50/50)."""
    r = np.random.Generator(np.random.PCG64(seed))
    gaps = r.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    ns = np.maximum(1, np.floor(np.exp(r.uniform(np.log(n_min), np.log(n_max), count)) * scale)
                    ).astype(np.int64)
    kinds = r.integers(0, 4, count)
    rels = np.array([1e-2, 1e-3, 1e-4])[r.integers(0, 3, count)]
    ops = r.integers(0, 2, count)
    return [dict(t=float(t[i]), n=int(ns[i]), kind=("clusters", "cosmology", "md", "lidar")[kinds[i]],
                 rel=float(rels[i]), op=("compress", "decompress")[ops[i]]) for i in range(count)]


KINDS = ("clusters", "cosmology", "md", "lidar")


def make(kind: str, n: int, seed: int, order: str = "drawn") -> List[np.ndarray]:
    """A particle set of ``kind`` with about ``n`` particles, in the order the
    generator draws it (``order="drawn"``), in the file-like order of
    ``local_order`` (``order="local"``; for md the drawn lattice order is
    already local), or seeded-shuffled (``order="shuffled"``)."""
    labels = np.empty(n, np.int32) if order == "local" and kind in ("clusters", "cosmology") \
        else None
    if kind == "clusters":
        out = clusters(n, seed, labels=labels)
    elif kind == "cosmology":
        out = cosmology(n, seed, n_halos=max(16, min(4096, n // 16_000)), labels=labels)
    elif kind == "md":
        cells = max(1, int(np.ceil((n / 4) ** (1 / 3))))
        out = md(cells, seed, n=n)
    elif kind == "lidar":
        out = lidar(n, seed)
    else:
        raise ValueError(kind)
    if order == "drawn" or (order == "local" and kind == "md"):
        return out
    if order == "shuffled":
        perm = np.random.Generator(np.random.PCG64(seed + 7)).permutation(out[0].size)
    elif order == "local":
        perm = local_order(kind, out, labels)
    else:
        raise ValueError(order)
    return [f[perm] for f in out]


def local_order(kind: str, fields: List[np.ndarray], labels: np.ndarray | None = None
                ) -> np.ndarray:
    """Permutation to a file-like storage order, the particles stored near
    their spatial neighbours as the paper's blocks assume of real files:
    clusters and cosmology cluster- (halo-) major with the background last,
    each group in draw order; LiDAR in 10-unit strips of y, serpentine in x
    (as a scanner sweeps)."""
    if kind in ("clusters", "cosmology"):
        if labels is None:
            raise ValueError("labels required")
        return np.argsort(labels, kind="stable")
    if kind == "lidar":
        x, y = fields[0], fields[1]
        strip = np.floor(y.astype(np.float64) / 10.0).astype(np.int64)
        xk = np.where(strip % 2 == 0, x, -x)
        return np.lexsort((xk, strip))
    raise ValueError(kind)


def clusters_device(n: int, seed: int, n_clusters: int = 64, sigma: float = 0.01,
                    background: float = 0.2, extra_fields: int = 0, device="cuda"):
    """`clusters` drawn on the GPU with torch's seeded generator (same
    distribution, different random stream); for large benchmark batches whose
    host generation would dominate.  Returns float32 CUDA tensors."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    centres = torch.rand((n_clusters, 3), generator=g, dtype=torch.float64, device=device)
    lab = torch.randint(0, n_clusters, (n,), generator=g, device=device)
    bg = torch.rand(n, generator=g, dtype=torch.float64, device=device) < background
    p = centres[lab] + sigma * torch.randn((n, 3), generator=g, dtype=torch.float64, device=device)
    u = torch.rand((n, 3), generator=g, dtype=torch.float64, device=device)
    p = torch.where(bg[:, None], u, p)
    p = torch.remainder(p, 1.0).to(torch.float32)
    p = torch.where(p >= 1.0, torch.zeros_like(p), p)
    out = [p[:, a].contiguous() for a in range(3)]
    for _ in range(extra_fields):
        out.append(torch.randn(n, generator=g, dtype=torch.float32, device=device))
    return out


def batch_specs(count: int = 256, seed: int = 4, n_min: int = 10_000, n_max: int = 8_000_000):
    """Shapes of the batched-form snapshots: particle counts log-uniform in
    [n_min, n_max], 3-6 fields, cluster counts uniform in [8, 1024], absolute
    bounds log-uniform in [1e-5, 1e-2].  List of dicts with n, fields,
    clusters, eb, seed (the snapshot's generator seed)."""
    r = np.random.Generator(np.random.PCG64(seed))
    ns = np.maximum(1, np.floor(np.exp(r.uniform(np.log(n_min), np.log(n_max), count)))).astype(np.int64)
    Fs = r.integers(3, 7, count)
    ks = r.integers(8, 1025, count)
    ebs = np.exp(r.uniform(np.log(1e-5), np.log(1e-2), count)).astype(np.float32)
    seeds = r.integers(0, 2 ** 31, count)
    return [dict(n=int(ns[i]), fields=int(Fs[i]), clusters=int(ks[i]), eb=float(ebs[i]),
                 seed=int(seeds[i])) for i in range(count)]
