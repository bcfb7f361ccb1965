"""Seeded particle-position generators (numpy PCG64).

Every generator returns a C-contiguous array of shape (n, dims) in the
requested floating type, in shuffled storage order (particle data carries no
spatial coherence in its storage order, Section 2 of the paper).  The
recipes stand in for the paper's benchmark sets (Table 2): a uniform cube,
a cosmology-shaped set (uniform background plus Gaussian halos, Nyx/HACC
style), a fluid-shaped set (jittered lattice displaced by a smooth vortex
field, SPH/FPM style) and a fusion-shaped 2-D set (Poincare-plot-like flux
surfaces and island chains, XGC style).  Nothing here knows about quantization, trees or bit
packing.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, (tuple, list)):
        return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    return np.random.Generator(np.random.PCG64(seed))


def sha256_of(arr: np.ndarray) -> str:
    """SHA-256 of the raw bytes of a fixed-seed array (guards against RNG drift)."""
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


def uniform_cube(n: int, seed: int = 1, dims: int = 3, dtype=np.float32) -> np.ndarray:
    """i.i.d. uniform positions in [0, 1)^dims (the plain single-set workload)."""
    rng = _rng(seed)
    dt = np.dtype(dtype)
    return np.ascontiguousarray(rng.random((n, dims), dtype=np.float64 if dt == np.float64 else np.float32))


def cosmology(n: int, seed: int = 2, box: float = 256.0, n_halos: int = 2000,
              background: float = 0.3, dims: int = 3, dtype=np.float32,
              halo_seed=None) -> np.ndarray:
    """Cosmology-shaped set: a uniform background plus Gaussian halos.

    round(background * n) particles are uniform in [0, box)^dims; the rest
    pick one of ``n_halos`` halos uniformly, whose centres are uniform in the
    box and whose isotropic Gaussian radius is lognormal(mu=ln 0.5,
    sigma=0.7).  Positions wrap periodically into the box, are cast to the
    output type and clamped below ``box``; the storage order is shuffled.
    ``halo_seed`` (default: ``seed``) fixes the halo catalogue separately, so
    that many small sets can share the same halos.
    """
    dt = np.dtype(dtype)
    rng = _rng(seed)
    hrng = rng if halo_seed is None else _rng(halo_seed)
    centres = hrng.random((n_halos, dims)) * box
    radii = hrng.lognormal(mean=math.log(0.5), sigma=0.7, size=n_halos)
    n_bg = int(round(background * n))
    bg = rng.random((n_bg, dims)) * box
    member = rng.integers(0, n_halos, size=n - n_bg)
    halo = centres[member] + rng.standard_normal((n - n_bg, dims)) * radii[member][:, None]
    pos = np.concatenate([bg, halo], axis=0)
    del bg, halo, member
    np.mod(pos, box, out=pos)
    out = pos.astype(dt)
    del pos
    np.minimum(out, np.nextafter(dt.type(box), dt.type(0)), out=out)
    perm = rng.permutation(n)
    return np.ascontiguousarray(out[perm])


def fluid_lattice_dims(n: int) -> tuple[int, int, int]:
    """Lattice shape used for a fluid set of n = 2^k particles (x >= y >= z)."""
    k = int(n).bit_length() - 1
    if n <= 0 or (1 << k) != n:
        raise ValueError("fluid sets use power-of-two particle counts")
    a = [k // 3 + (1 if i < k % 3 else 0) for i in range(3)]
    return (1 << a[0], 1 << a[1], 1 << a[2])


def fluid(nx: int, ny: int, nz: int, seed: int = 4, amp: float = 2.0,
          jitter: float = 0.3, dtype=np.float32) -> np.ndarray:
    """Fluid-shaped set on an nx*ny*nz lattice (3D only).

    Cell centres (i + 1/2, j + 1/2, k + 1/2) get a U(-jitter, jitter) offset
    per coordinate and are then displaced by a divergence-free sinusoidal
    vortex of amplitude ``amp`` cells, each component depending only on the
    other axes: (amp sin(2 pi y/ny), amp sin(2 pi z/nz), amp sin(2 pi x/nx)).
    No wrapping; storage order is shuffled.
    """
    dt = np.dtype(dtype)
    rng = _rng(seed)
    n = nx * ny * nz
    out = np.empty((n, 3), dtype=dt)
    ii = np.arange(nx, dtype=np.float64) + 0.5
    jj = np.arange(ny, dtype=np.float64) + 0.5
    slab = nx * ny
    base_x = np.tile(ii, ny)
    base_y = np.repeat(jj, nx)
    two_pi = 2.0 * math.pi
    for k in range(nz):
        p = np.empty((slab, 3), dtype=np.float64)
        p[:, 0] = base_x
        p[:, 1] = base_y
        p[:, 2] = k + 0.5
        p += rng.uniform(-jitter, jitter, size=(slab, 3))
        d0 = amp * np.sin(two_pi * p[:, 1] / ny)
        d1 = amp * np.sin(two_pi * p[:, 2] / nz)
        d2 = amp * np.sin(two_pi * p[:, 0] / nx)
        p[:, 0] += d0
        p[:, 1] += d1
        p[:, 2] += d2
        out[k * slab:(k + 1) * slab] = p
    perm = rng.permutation(n)
    return np.ascontiguousarray(out[perm])


def poincare(n: int, seed: int = 8, dtype=np.float32) -> np.ndarray:
    """Fusion-shaped 2-D set (R, Z): a Poincare-plot-like cross-section of a
    tokamak plasma, standing in for the XGC Poincare data of Table 2.

    Points lie on curves rather than filling the plane, with very uneven
    density: 70% on 600 nested flux surfaces (minor radius rho = 0.57 sqrt(u),
    u uniform; poloidal angle uniform), 20% on three island chains (m = 3, 4,
    5 islands around the surfaces rho = 0.33, 0.45, 0.54; each point on a
    closed loop of relative size s ~ U(0.2, 1) around an island's O-point) and
    10% in a chaotic edge band rho ~ U(0.576, 0.624).  (rho, theta) map to an
    elongated, triangular, egg-shaped section R = 1.7 + rho cos(theta +
    0.35 sin theta) + 0.1 rho sin^2 theta, Z = 1.7 rho sin theta, plus
    N(0, 1e-4) jitter; storage order is shuffled.
    """
    dt = np.dtype(dtype)
    rng = _rng(seed)
    a = 0.6
    n_isl = int(round(0.2 * n))
    n_edge = int(round(0.1 * n))
    n_surf = n - n_isl - n_edge
    two_pi = 2.0 * math.pi
    surfaces = 0.95 * a * np.sqrt(rng.random(600))
    rho_s = surfaces[rng.integers(0, 600, size=n_surf)]
    th_s = rng.random(n_surf) * two_pi
    chains = np.array([[0.55 * a, 3, 0.030 * a], [0.75 * a, 4, 0.025 * a], [0.90 * a, 5, 0.020 * a]])
    c = chains[rng.integers(0, 3, size=n_isl)]
    r_c, m_c, w_c = c[:, 0], c[:, 1], c[:, 2]
    k = np.floor(rng.random(n_isl) * m_c)
    t = rng.random(n_isl) * two_pi
    sz = rng.uniform(0.2, 1.0, size=n_isl)
    rho_i = r_c + w_c * sz * np.sin(t)
    th_i = two_pi * (k + 0.25) / m_c + (w_c / r_c) * 2.0 * sz * np.cos(t)
    rho_e = a * rng.uniform(0.96, 1.04, size=n_edge)
    th_e = rng.random(n_edge) * two_pi
    rho = np.concatenate([rho_s, rho_i, rho_e])
    th = np.concatenate([th_s, th_i, th_e])
    del rho_s, th_s, rho_i, th_i, rho_e, th_e, c, k, t, sz
    pos = np.empty((n, 2), dtype=np.float64)
    pos[:, 0] = 1.7 + rho * np.cos(th + 0.35 * np.sin(th)) + 0.1 * rho * np.sin(th) ** 2
    pos[:, 1] = 1.7 * rho * np.sin(th)
    del rho, th
    pos += rng.normal(0.0, 1e-4, size=(n, 2))
    out = pos.astype(dt)
    del pos
    perm = rng.permutation(n)
    return np.ascontiguousarray(out[perm])


def batch_plan(nsets: int, seed0: int = 5, lo_exp: float = 3.0, hi_exp: float = 6.0):
    """Sizes (log-uniform 10^lo_exp..10^hi_exp), kinds and relative bounds
    of the sets of ``batch_sets``: (sizes int64[nsets], kinds list, ebs list)."""
    master = _rng((seed0, 0x5E75))
    sizes = np.rint(10.0 ** master.uniform(lo_exp, hi_exp, size=nsets)).astype(np.int64)
    kinds = master.integers(0, 2, size=nsets)
    ebs = np.where(master.integers(0, 2, size=nsets) == 0, 1e-3, 1e-4)
    return (sizes, ["uniform" if k == 0 else "cosmology" for k in kinds],
            [float(e) for e in ebs])


def batch_set(s: int, n: int, kind: str, seed0: int = 5, dtype=np.float32):
    """Positions of set s of ``batch_sets`` (independent of the other sets)."""
    if kind == "uniform":
        return uniform_cube(n, seed=(seed0, s), dtype=dtype)
    return cosmology(n, seed=(seed0, s), dtype=dtype, halo_seed=(seed0, 0xC0DE))


def batch_sets(nsets: int, seed0: int = 5, lo_exp: float = 3.0, hi_exp: float = 6.0,
               dtype=np.float32):
    """Many independent sets of log-uniform sizes 10^lo_exp..10^hi_exp.

    Set s draws with seed (seed0, s); it is uniform-cube or cosmology-shaped
    (shared halo catalogue) with probability 1/2 each, and carries a relative
    error bound of 1e-3 or 1e-4 with probability 1/2 each.  Yields
    (positions, rel_eb, kind) tuples lazily.
    """
    sizes, kinds, ebs = batch_plan(nsets, seed0, lo_exp, hi_exp)
    for s in range(nsets):
        yield batch_set(s, int(sizes[s]), kinds[s], seed0, dtype), ebs[s], kinds[s]


def served_requests(nreq: int, seed0: int = 6, lo_exp: float = 4.0, hi_exp: float = 7.0):
    """Request mix for a served stream: (size, kind, is_compress) per request.

    Sizes are log-uniform 10^lo_exp..10^hi_exp; kind is uniform-cube or
    cosmology with probability 1/2; half the requests compress, half
    decompress.  A request of size n and kind k takes the first n particles
    of ``request_pool(k, ...)`` (a shuffled set, so every prefix is a uniform
    random subset of it).
    """
    rng = _rng((seed0, 0x5E7E))
    sizes = np.rint(10.0 ** rng.uniform(lo_exp, hi_exp, size=nreq)).astype(np.int64)
    kinds = rng.integers(0, 2, size=nreq)
    comp = rng.integers(0, 2, size=nreq) == 0
    return [(int(sizes[i]), "uniform" if kinds[i] == 0 else "cosmology", bool(comp[i]))
            for i in range(nreq)]


def request_pool(kind: str, nmax: int, seed0: int = 6, dtype=np.float32):
    """The positions that served requests of one kind take prefixes of."""
    if kind == "uniform":
        return uniform_cube(nmax, seed=(seed0, 0x900), dtype=dtype)
    return cosmology(nmax, seed=(seed0, 0x901), dtype=dtype)


def poisson_arrivals(nreq: int, qps: float, seed: int = 7):
    """Arrival times (seconds from 0) of a Poisson process of rate qps."""
    rng = _rng((seed, 0xA77))
    return np.cumsum(rng.exponential(1.0 / qps, size=nreq))
