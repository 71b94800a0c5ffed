"""Seeded synthetic inputs for the Voronoi hot path.

This module only draws random particle sets; it holds none of the
tessellation's arithmetic and is the one piece of code shared by the oracle
tests and the GPU path.  The paper's own data (LambdaCDM N-body snapshots of
about 3.5M and 27.5M particles, a halo catalogue and an SDSS-like mock, paper
sections 2-3) are not available; these generators stand in for them with the
clustering the workloads prescribe: a uniform background plus NFW-like halos.

Workloads (seeds in SEEDS):
  uniform4096       4096 points, i.i.d. uniform in the periodic unit cube, FP64, unit masses.
  clustered2m       2,097,152 points in a periodic box of side 100, FP32: half uniform, half in
     200 NFW-like halos (concentration 5-15, radius 0.5-3, masses log-uniform
     over two decades), unit masses; density deposited on a 256^3 grid.
  lattice_halos16m  16,777,216 points: 256^3 lattice in the periodic unit box with Gaussian
     displacements (sigma = 0.3 spacing), 20% of points replaced by 1000 NFW-like
     halos of mean overdensity 1e2-1e4, FP32, unit masses.
  batched64         64 cuboid sub-volumes of 1e4-1e6 owned points (log-uniform), clustered-2M
     density and mix, each with a ghost buffer of 3 mean spacings.
  diff262k          262,144 points, the clustered mix scaled to the periodic unit cube, plus a
     smooth sinusoidal target density for a density-matching loss.
  survey_slab       262,144 points, the clustered mix in a bounded 10 x 1 x 1 box (an elongated
     survey-like volume for the slab decomposition), FP32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20160126
# one seed per workload (kept stable so that stored results stay comparable)
SEEDS = {"uniform4096": SEED_BASE + 1, "clustered2m": SEED_BASE + 2, "lattice_halos16m": SEED_BASE + 3,
         "batched64": SEED_BASE + 4, "diff262k": SEED_BASE + 5, "survey_slab": SEED_BASE + 6}


def rng_for(name: str) -> np.random.Generator:
    return np.random.default_rng(SEEDS[name])


# --------------------------------------------------------------------------
# building blocks


def _nfw_mu(y):
    return np.log1p(y) - y / (1.0 + y)


def nfw_radii(rng, n, conc, r_vir):
    """Radii in [0, r_vir] drawn from an NFW enclosed-mass profile.

    The enclosed fraction at x = r / r_vir is mu(c x) / mu(c) with
    mu(y) = ln(1 + y) - y / (1 + y); it is inverted by bisection in FP64.
    """
    u = rng.random(n)
    target = u * _nfw_mu(conc)
    lo = np.zeros(n)
    hi = np.ones(n)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        below = _nfw_mu(conc * mid) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi) * r_vir


def isotropic(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def largest_remainder(weights, total):
    w = np.asarray(weights, np.float64)
    q = w / w.sum() * total
    base = np.floor(q).astype(np.int64)
    rest = int(total - base.sum())
    if rest > 0:
        order = np.argsort(-(q - base), kind="stable")
        base[order[:rest]] += 1
    return base


def halo_points(rng, counts, centres, radii, conc):
    """Concatenated NFW-like halos, one per (count, centre, radius, concentration)."""
    out = np.empty((int(np.sum(counts)), 3))
    k = 0
    for n_h, c_h, r_h, cc in zip(counts, centres, radii, conc):
        n_h = int(n_h)
        if n_h == 0:
            continue
        r = nfw_radii(rng, n_h, cc, r_h)
        out[k:k + n_h] = c_h + r[:, None] * isotropic(rng, n_h)
        k += n_h
    return out


def wrap(pos, lo, length):
    return lo + np.mod(pos - lo, length)


def to_dtype_wrapped(pos, length, dtype):
    """Cast to dtype; a coordinate that rounds up to the box length maps to 0."""
    p = pos.astype(dtype)
    L = np.asarray(length, dtype=dtype)
    p = np.where(p >= L, p - L, p).astype(dtype)
    p = np.where(p < 0, p + L, p).astype(dtype)
    return p


def duplicate_rows(p):
    """Indices of rows that exactly repeat an earlier row."""
    a = np.ascontiguousarray(p)
    if a.dtype == np.float32:
        cols = a.view(np.uint32).reshape(-1, 3)
    else:
        cols = a.view(np.uint64).reshape(-1, 3)
    order = np.lexsort((cols[:, 2], cols[:, 1], cols[:, 0]))
    s = cols[order]
    same = np.all(s[1:] == s[:-1], axis=1)
    return np.sort(order[1:][same])


def redraw_duplicates(rng, p, lo, length, dtype):
    """Replace exact duplicates by fresh uniform points (repeat until none)."""
    for _ in range(100):
        dup = duplicate_rows(p)
        if dup.size == 0:
            return p
        fresh = lo + rng.random((dup.size, 3)) * length
        p[dup] = to_dtype_wrapped(fresh, length, dtype) if np.isscalar(length) else fresh.astype(dtype)
    raise RuntimeError("could not remove duplicate points")


# --------------------------------------------------------------------------
# workloads


@dataclass
class Workload:
    name: str
    pos: np.ndarray            # n x 3, FP32 or FP64
    mass: np.ndarray           # n
    box_lo: np.ndarray         # 3
    box_hi: np.ndarray         # 3
    periodic: bool = True
    grid: tuple | None = None  # deposit grid dims
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def box_len(self) -> np.ndarray:
        return self.box_hi - self.box_lo

    @property
    def spacing(self) -> float:
        return float(np.prod(self.box_len) / self.n) ** (1.0 / 3.0)


def uniform_box(n, length=1.0, seed=0, dtype=np.float64, name="uniform"):
    rng = np.random.default_rng(seed)
    L = float(length)
    p = to_dtype_wrapped(rng.random((n, 3)) * L, L, dtype)
    p = redraw_duplicates(rng, p, 0.0, L, dtype)
    return Workload(name, p, np.ones(n, dtype=np.float64), np.zeros(3), np.full(3, L))


def uniform4096():
    rng = rng_for("uniform4096")
    n = 4096
    p = rng.random((n, 3))
    p = redraw_duplicates(rng, p, 0.0, 1.0, np.float64)
    return Workload("uniform-4096-fp64", p, np.ones(n), np.zeros(3), np.ones(3), True, (32, 32, 32))


def clustered_box(rng, n, length, n_halo, r_range, conc_range=(5.0, 15.0), dtype=np.float32, halo_frac=0.5):
    """Uniform background plus NFW-like halos in a periodic cube of side `length`."""
    L = float(length)
    n_halo_pts = int(round(n * halo_frac))
    n_bg = n - n_halo_pts
    bg = rng.random((n_bg, 3)) * L
    masses = 10.0 ** rng.uniform(0.0, 2.0, n_halo)
    counts = largest_remainder(masses, n_halo_pts)
    centres = rng.random((n_halo, 3)) * L
    radii = rng.uniform(r_range[0], r_range[1], n_halo)
    conc = rng.uniform(conc_range[0], conc_range[1], n_halo)
    halos = halo_points(rng, counts, centres, radii, conc)
    p = np.concatenate([bg, halos])
    p = wrap(p, 0.0, L)
    p = to_dtype_wrapped(p, L, dtype)
    p = redraw_duplicates(rng, p, 0.0, L, dtype)
    p = p[rng.permutation(n)]
    info = {"halo_counts": counts, "halo_centres": centres, "halo_radii": radii, "halo_conc": conc}
    return p, info


def clustered2m(n=2_097_152):
    rng = rng_for("clustered2m")
    L = 100.0
    p, info = clustered_box(rng, n, L, 200, (0.5, 3.0))
    return Workload("clustered-2M-fp32", p, np.ones(n), np.zeros(3), np.full(3, L), True, (256, 256, 256), info)


def lattice_halos16m(side=256):
    rng = rng_for("lattice_halos16m")
    n = side ** 3
    g = (np.arange(side, dtype=np.float64) + 0.5) / side
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p += rng.normal(scale=0.3 / side, size=p.shape)
    n_rep = int(round(0.2 * n))
    keep = np.ones(n, bool)
    keep[rng.choice(n, n_rep, replace=False)] = False
    p = p[keep]
    n_halo = 1000
    masses = 10.0 ** rng.uniform(0.0, 2.0, n_halo)
    counts = largest_remainder(masses, n_rep)
    delta = 10.0 ** rng.uniform(2.0, 4.0, n_halo)
    radii = (3.0 * counts / (4.0 * math.pi * delta * n)) ** (1.0 / 3.0)
    centres = rng.random((n_halo, 3))
    conc = rng.uniform(5.0, 15.0, n_halo)
    halos = halo_points(rng, counts, centres, radii, conc)
    p = wrap(np.concatenate([p, halos]), 0.0, 1.0)
    p = to_dtype_wrapped(p, 1.0, np.float32)
    p = redraw_duplicates(rng, p, 0.0, 1.0, np.float32)
    p = p[rng.permutation(n)]
    info = {"halo_counts": counts, "halo_centres": centres, "halo_radii": radii, "halo_overdensity": delta}
    return Workload("lattice-halos-16M-fp32", p, np.ones(n), np.zeros(3), np.ones(3), True, None, info)


@dataclass
class Item:
    """One sub-volume: owned box [lo, hi] with a ghost buffer of width `ghost`."""
    lo: np.ndarray
    hi: np.ndarray
    ghost: float
    owned: np.ndarray   # n_owned x 3 (FP32)
    ghosts: np.ndarray  # n_ghost x 3 (FP32)

    @property
    def buffered_lo(self):
        return self.lo - self.ghost

    @property
    def buffered_hi(self):
        return self.hi + self.ghost


def ghost_width(border_factor, spacing):
    """Buffer thickness = BORDERFACTOR x mean inter-particle distance (section 2)."""
    return float(border_factor) * float(spacing)


def batched64(n_items=64, n_range=(1e4, 1e6), border_factor=3.0, seed_offset=0):
    rng = np.random.default_rng(SEEDS["batched64"] + seed_offset)
    s = 100.0 / 2_097_152 ** (1.0 / 3.0)   # mean spacing of the clustered 2M box, 0.78125
    nbar = 1.0 / s ** 3
    w = ghost_width(border_factor, s)
    items = []
    for _ in range(n_items):
        n_b = int(round(10.0 ** rng.uniform(math.log10(n_range[0]), math.log10(n_range[1]))))
        ratios = np.exp(rng.uniform(-math.log(2.0), math.log(2.0), 3))
        vol = n_b / nbar
        side = ratios * (vol / np.prod(ratios)) ** (1.0 / 3.0)
        lo = np.zeros(3)
        hi = side
        blo, bhi = lo - w, hi + w
        bvol = float(np.prod(bhi - blo))
        n_tot = int(round(bvol * nbar))
        n_h = max(1, int(round(200 * bvol / 1e6)))
        n_halo_pts = n_tot // 2
        bg = blo + rng.random((n_tot - n_halo_pts, 3)) * (bhi - blo)
        masses = 10.0 ** rng.uniform(0.0, 2.0, n_h)
        counts = largest_remainder(masses, n_halo_pts)
        centres = blo + rng.random((n_h, 3)) * (bhi - blo)
        radii = rng.uniform(0.5, 3.0, n_h)
        conc = rng.uniform(5.0, 15.0, n_h)
        halos = halo_points(rng, counts, centres, radii, conc)
        p = np.concatenate([bg, halos]).astype(np.float32)
        inside = np.all((p >= blo) & (p < bhi), axis=1)
        p = p[inside]
        p = redraw_duplicates(rng, p, blo, bhi - blo, np.float32)
        own = np.all((p >= lo) & (p < hi), axis=1)
        items.append(Item(lo, hi, w, p[own], p[~own]))
    return items


def diff262k(n=262_144):
    rng = rng_for("diff262k")
    s2 = 100.0 / 2_097_152 ** (1.0 / 3.0)
    s5 = 1.0 / n ** (1.0 / 3.0)
    scale = s5 / s2
    n_halo = max(1, int(round(200 * n / 2_097_152)))
    p, info = clustered_box(rng, n, 1.0, n_halo, (0.5 * scale, 3.0 * scale), dtype=np.float32)
    lam = rng.choice(np.array([1.0, 0.5, 1.0 / 3.0, 0.25]), size=3)
    phi = rng.uniform(0.0, 2.0 * math.pi, 3)
    info.update({"target_lambda": lam, "target_phase": phi, "target_amplitude": 0.5, "fd_rows":
                 np.sort(rng.choice(n, 512, replace=False))})
    return Workload("diff-262k-fp32", p, np.ones(n), np.zeros(3), np.ones(3), True, None, info)


def survey_slab(n=262_144, sides=(10.0, 1.0, 1.0)):
    """A bounded, elongated world (the survey slices and cones the paper's slab decomposition is
    meant for): the clustered mix (half uniform background, half NFW-like halos with radii scaled to
    the mean spacing like diff262k) in the non-periodic box [0, sides], FP32.  Halo points that fall
    outside the box are replaced by background points, so the set holds exactly n points."""
    rng = rng_for("survey_slab")
    hi = np.asarray(sides, np.float64)
    s = float(np.cbrt(np.prod(hi) / n))
    scale = s / (100.0 / 2_097_152 ** (1.0 / 3.0))
    n_halo = max(1, int(round(200 * n / 2_097_152)))
    n_halo_pts = n // 2
    masses = 10.0 ** rng.uniform(0.0, 2.0, n_halo)
    counts = largest_remainder(masses, n_halo_pts)
    centres = rng.random((n_halo, 3)) * hi
    radii = rng.uniform(0.5 * scale, 3.0 * scale, n_halo)
    conc = rng.uniform(5.0, 15.0, n_halo)
    halos = halo_points(rng, counts, centres, radii, conc).astype(np.float32)
    halos = halos[np.all((halos >= 0) & (halos < hi), axis=1)]
    bg = (rng.random((n - len(halos), 3)) * hi).astype(np.float32)
    p = np.concatenate([bg, halos])
    p = np.minimum(p, np.nextafter(hi.astype(np.float32), np.float32(0)))
    p = redraw_duplicates(rng, p, np.zeros(3), hi, np.float32)
    p = p[rng.permutation(n)]
    return Workload("survey-slab-262k-fp32", p, np.ones(n), np.zeros(3), hi, False, None,
                    {"halo_counts": counts, "halo_centres": centres, "halo_radii": radii})


def target_density(x, lam, phi, amplitude, mean_density):
    """Smooth periodic target rho_t(x) = mean * (1 + A * prod_a sin(2 pi x_a / lam_a + phi_a))."""
    x = np.asarray(x, np.float64)
    s = np.prod(np.sin(2.0 * math.pi * x / lam + phi), axis=-1)
    return mean_density * (1.0 + amplitude * s)


def lattice(kind, n_side, length=1.0):
    """Simple-cubic, body-centred or face-centred cubic lattice with n_side cubes per axis."""
    a = length / n_side
    g = (np.arange(n_side) + 0.5) * a
    base = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    if kind == "sc":
        offs = [(0, 0, 0)]
    elif kind == "bcc":
        offs = [(0, 0, 0), (0.5, 0.5, 0.5)]
    elif kind == "fcc":
        offs = [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)]
    else:
        raise ValueError(kind)
    p = np.concatenate([base + a * np.asarray(o) for o in offs])
    return np.mod(p, length)
