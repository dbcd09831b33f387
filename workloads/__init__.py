"""Seeded synthetic workloads shared by the CPU oracle tests and the GPU path.

This package holds inputs only (geometry descriptions, primary photon sets and
their seeds); it contains none of the navigation or transport arithmetic.
"""
from . import geometry, primaries
from .geometry import GeometryDesc, BOX, TUBS, CONS, ORB
from .primaries import Primaries

# Workload registry: name -> (geometry builders, primary generator, defaults).
#   tiny:        1 m vacuum cube, 8 water/lead cubes, 1e4 photons of 1 MeV from the origin
#   calorimeter: Pb/Si sampling calorimeter (50 layers x 20 x 20 cells), 1e6 photons along +z
#   barrel:      64 tube layers x 128 phi segments, cone endcaps, 32 orbs, 1e7 photons
#   batched:     4096 lognormal-sized events over 8 resident geometries


def tiny(n=10_000, seed=0):
    return [geometry.tiny()], primaries.tiny_source(n, seed), None


def calorimeter(n=1_000_000, seed=0):
    return [geometry.calorimeter()], primaries.calorimeter_beam(n, seed), None


def barrel(n=10_000_000, seed=0, geom_seed=1):
    return [geometry.barrel(seed=geom_seed)], primaries.barrel_source(n, seed), None


def batched(n_events=4096, seed=0, plan_seed=2):
    """Three named geometries plus five seeded barrel variants, uneven events."""
    geoms = [geometry.tiny(), geometry.calorimeter(), geometry.barrel(seed=1)]
    geoms += [geometry.barrel_variant(101 + i) for i in range(5)]
    sources = [primaries.source_origin_iso, primaries.source_beam] + \
              [primaries.source_axis_iso] * 6
    prim, event_geom = primaries.batched_events(n_events, len(geoms), seed=plan_seed,
                                                sources=sources)
    return geoms, prim, event_geom


def endcap(n=20_000, seed=0):
    """Trapezoid endcaps around a tube: photons from the origin, isotropic,
    log-uniform 0.05-20 MeV."""
    return [geometry.endcap()], primaries.origin_iso(n, seed), None


WORKLOADS = {"tiny": tiny, "calorimeter": calorimeter, "barrel": barrel, "batched": batched, "endcap": endcap}
