"""Seeded primary photon sets (inputs only).

Like the paper's benchmark (Alg. 2, phases 2-3), primaries are generated on
the host and handed to the navigation code as arrays.  All randomness here
comes from numpy's counter-based Philox generator with a stated key, so a
workload is reproducible from (config, seed).  Units: mm, MeV.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np


@dataclass
class Primaries:
    event: np.ndarray      # int32 [n]  event id of each primary
    prim_id: np.ndarray    # int32 [n]  index of the primary inside its event
    pos: np.ndarray        # float64 [n, 3]
    dir: np.ndarray        # float64 [n, 3] unit vectors
    energy: np.ndarray     # float64 [n]
    n_events: int

    @property
    def n(self):
        return int(self.energy.shape[0])

    def subset(self, idx):
        idx = np.asarray(idx)
        return Primaries(self.event[idx].copy(), self.prim_id[idx].copy(), self.pos[idx].copy(),
                         self.dir[idx].copy(), self.energy[idx].copy(), self.n_events)


def _rng(seed):
    return np.random.Generator(np.random.Philox(key=seed))


def isotropic(rng, n):
    """Unit vectors uniform on the sphere: cos(theta) = 1 - 2u, phi = 2 pi u'."""
    u1 = rng.uniform(size=n)
    u2 = rng.uniform(size=n)
    ct = 1.0 - 2.0 * u1
    st = np.sqrt(np.maximum(0.0, (1.0 - ct) * (1.0 + ct)))
    ph = 2.0 * math.pi * u2
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def log_uniform(rng, n, lo, hi):
    return lo * np.power(hi / lo, rng.uniform(size=n))


def one_per_event(pos, dirs, energy):
    n = energy.shape[0]
    return Primaries(np.arange(n, dtype=np.int32), np.zeros(n, dtype=np.int32),
                     np.ascontiguousarray(pos, dtype=np.float64),
                     np.ascontiguousarray(dirs, dtype=np.float64),
                     np.ascontiguousarray(energy, dtype=np.float64), n)


def tiny_source(n=10_000, seed=0, energy=1.0):
    """Point source at the origin, isotropic, mono-energetic (1 MeV)."""
    rng = _rng(seed)
    d = isotropic(rng, n)
    return one_per_event(np.zeros((n, 3)), d, np.full(n, energy))


def calorimeter_beam(n=1_000_000, seed=0, z0=-999.0, sigma=10.0, e_lo=0.1, e_hi=10.0):
    """Pencil beam along +z with Gaussian transverse spread, log-uniform energy."""
    rng = _rng(seed)
    xy = rng.normal(0.0, sigma, size=(n, 2))
    pos = np.column_stack([xy, np.full(n, z0)])
    d = np.zeros((n, 3))
    d[:, 2] = 1.0
    e = log_uniform(rng, n, e_lo, e_hi)
    return one_per_event(pos, d, e)


def barrel_source(n=10_000_000, seed=0, half_z=2000.0, e_lo=0.05, e_hi=20.0):
    """Points on the beam axis, z uniform in the barrel, isotropic, log-uniform energy."""
    rng = _rng(seed)
    z = rng.uniform(-half_z, half_z, size=n)
    pos = np.column_stack([np.zeros(n), np.zeros(n), z])
    d = isotropic(rng, n)
    e = log_uniform(rng, n, e_lo, e_hi)
    return one_per_event(pos, d, e)


def origin_iso(n=20_000, seed=0, e_lo=0.05, e_hi=20.0):
    """Point source at the origin, isotropic, log-uniform energy."""
    rng = _rng(seed)
    d = isotropic(rng, n)
    e = log_uniform(rng, n, e_lo, e_hi)
    return one_per_event(np.zeros((n, 3)), d, e)


def pencil(n, pos, direction, energy):
    pos = np.broadcast_to(np.asarray(pos, dtype=np.float64), (n, 3)).copy()
    d = np.broadcast_to(np.asarray(direction, dtype=np.float64), (n, 3)).copy()
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return one_per_event(pos, d, np.full(n, float(energy)))


def batched_events(n_events=4096, n_geoms=8, seed=0, median=2000.0, sigma_ln=1.0,
                   lo=10, hi=50_000, sources=None, e_lo=0.05, e_hi=20.0):
    """Uneven events: lognormal primary counts, a geometry drawn per event.

    ``sources[g](rng, n) -> (pos[n,3], dir[n,3])`` gives each geometry's source
    law.  Returns (Primaries, event_geom[int32 n_events]).
    """
    rng = _rng(seed)
    geom = rng.integers(0, n_geoms, size=n_events).astype(np.int32)
    z = rng.normal(size=n_events)
    counts = np.clip(np.floor(median * np.exp(sigma_ln * z)), lo, hi).astype(np.int64)
    ev, pid, pos, dirs = [], [], [], []
    for e in range(n_events):
        c = int(counts[e])
        p, d = sources[int(geom[e])](rng, c)
        ev.append(np.full(c, e, dtype=np.int32))
        pid.append(np.arange(c, dtype=np.int32))
        pos.append(p)
        dirs.append(d)
    n = int(counts.sum())
    energy = log_uniform(rng, n, e_lo, e_hi)
    prim = Primaries(np.concatenate(ev), np.concatenate(pid),
                     np.ascontiguousarray(np.concatenate(pos)),
                     np.ascontiguousarray(np.concatenate(dirs)), energy, n_events)
    return prim, geom


def source_origin_iso(rng, n):
    return np.zeros((n, 3)), isotropic(rng, n)


def source_beam(rng, n, z0=-999.0, sigma=10.0):
    xy = rng.normal(0.0, sigma, size=(n, 2))
    d = np.zeros((n, 3))
    d[:, 2] = 1.0
    return np.column_stack([xy, np.full(n, z0)]), d


def source_axis_iso(rng, n, half_z=2000.0):
    z = rng.uniform(-half_z, half_z, size=n)
    return np.column_stack([np.zeros(n), np.zeros(n), z]), isotropic(rng, n)


# ---------------------------------------------------------------------------
# The paper's particle sets for the free-path benchmark (Sec. 3.5): every
# particle starts at the centre of the geometry.
# ---------------------------------------------------------------------------

def paper_random(n=100_000, seed=0):
    """Random set: isotropic directions, Exp(1) lifetimes; (pos, dir, life)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    d = isotropic(rng, n)
    u = 1.0 - rng.uniform(size=n)  # (0, 1]
    return np.zeros((n, 3)), d, -np.log(u)


def paper_regular(nx=400, ny=250, half_w=1.0):
    """Regular set: rays from the centre through the pixel centres of an
    nx x ny grid on the plane z = 1 (x in [-half_w, half_w], square pixels),
    listed column by column (column-major), all with lifetime 1."""
    px = 2.0 * half_w / nx
    col = np.repeat(np.arange(nx), ny)
    row = np.tile(np.arange(ny), nx)
    x = -half_w + (col + 0.5) * px
    y = -0.5 * ny * px + (row + 0.5) * px
    d = np.column_stack([x, y, np.ones(nx * ny)])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.zeros((nx * ny, 3)), d, np.ones(nx * ny)
