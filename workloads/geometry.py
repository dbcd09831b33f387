"""Seeded synthetic geometry descriptions (inputs only, no navigation arithmetic).

A geometry is a Geant4-style placement hierarchy: logical volumes (LV: a solid,
a material and an ordered list of daughter placements) and physical placements
(PV: a child LV put into its mother with x_mother = R x_local + t).  The paper
states the navigation problem on such a hierarchy (Sec. 3.2) and names boxes,
tubes, cones and balls as its solids (Sec. 3.5); the concrete detectors built
here are the synthetic workloads the project measures on.

Everything here is plain data: solid parameters, material composition and the
rotation matrices of the placements (computed once, so that both the oracle and
the GPU library read the same numbers).  Units: mm, rad, g/cm3.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Solid type codes shared by the flat description.
BOX, TUBS, CONS, ORB, TRD, SPHERE = 0, 1, 2, 3, 4, 5
NPAR = 8

# Material composition table: name -> (density g/cm3, [(Z, A g/mol, mass fraction)]).
MATERIALS = {
    "vacuum": (0.0, []),
    "water": (1.0, [(1, 1.008, 0.111894), (8, 15.999, 0.888106)]),
    "lead": (11.35, [(82, 207.2, 1.0)]),
    "silicon": (2.33, [(14, 28.085, 1.0)]),
    "aluminium": (2.699, [(13, 26.9815385, 1.0)]),
}


@dataclass
class GeometryDesc:
    """Flat, index-based description of a placement hierarchy."""

    name: str
    solid_type: np.ndarray
    solid_par: np.ndarray
    mat_names: list
    mat_density: np.ndarray
    mat_el_off: np.ndarray
    el_Z: np.ndarray
    el_A: np.ndarray
    el_wfrac: np.ndarray
    lv_solid: np.ndarray
    lv_mat: np.ndarray
    lv_dau_off: np.ndarray
    lv_dau_cnt: np.ndarray
    lv_voxelize: np.ndarray
    pv_lv: np.ndarray
    pv_rot: np.ndarray
    pv_trans: np.ndarray
    world_lv: int = 0
    lv_names: list = field(default_factory=list)

    @property
    def n_solids(self):
        return int(self.solid_type.shape[0])

    @property
    def n_mats(self):
        return int(self.mat_density.shape[0])

    @property
    def n_lv(self):
        return int(self.lv_solid.shape[0])

    @property
    def n_pv(self):
        return int(self.pv_lv.shape[0])

    def n_touchables(self):
        """Number of distinct placement paths (world included)."""
        cnt = [0] * self.n_lv

        def rec(lv):
            if cnt[lv]:
                return cnt[lv]
            total = 1
            o, n = int(self.lv_dau_off[lv]), int(self.lv_dau_cnt[lv])
            for k in range(o, o + n):
                total += rec(int(self.pv_lv[k]))
            cnt[lv] = total
            return total

        return rec(self.world_lv)


def rot_identity():
    return np.eye(3)


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_x_pi():
    """Exact rotation by pi about x (no rounding residue in the matrix)."""
    return np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, -1.0]])


class Builder:
    """Accumulates solids, materials, LVs and daughter lists, then flattens."""

    def __init__(self, name):
        self.name = name
        self.solids = []  # (type, params)
        self.mats = []
        self.mat_index = {}
        self.lvs = []  # dict(solid, mat, daughters=[(lv, R, t)], voxelize, name)

    def solid(self, stype, *par):
        p = np.zeros(NPAR)
        p[: len(par)] = par
        self.solids.append((stype, p))
        return len(self.solids) - 1

    def material(self, name):
        if name not in self.mat_index:
            self.mat_index[name] = len(self.mats)
            self.mats.append(name)
        return self.mat_index[name]

    def lv(self, solid, mat, name="", voxelize=True):
        self.lvs.append(dict(solid=solid, mat=self.material(mat), daughters=[],
                             voxelize=voxelize, name=name))
        return len(self.lvs) - 1

    def place(self, mother, child, R=None, t=(0.0, 0.0, 0.0)):
        R = rot_identity() if R is None else np.asarray(R, dtype=np.float64)
        self.lvs[mother]["daughters"].append((child, R, np.asarray(t, dtype=np.float64)))

    def build(self, world_lv=0) -> GeometryDesc:
        solid_type = np.array([s[0] for s in self.solids], dtype=np.int32)
        solid_par = np.stack([s[1] for s in self.solids]).astype(np.float64)
        dens, off, Z, A, W = [], [0], [], [], []
        for m in self.mats:
            d, els = MATERIALS[m]
            dens.append(d)
            for z, a, w in els:
                Z.append(z)
                A.append(a)
                W.append(w)
            off.append(len(Z))
        lv_solid, lv_mat, lv_off, lv_cnt, lv_vox = [], [], [], [], []
        pv_lv, pv_rot, pv_trans = [], [], []
        for lv in self.lvs:
            lv_solid.append(lv["solid"])
            lv_mat.append(lv["mat"])
            lv_off.append(len(pv_lv))
            lv_cnt.append(len(lv["daughters"]))
            lv_vox.append(1 if lv["voxelize"] else 0)
            for child, R, t in lv["daughters"]:
                pv_lv.append(child)
                pv_rot.append(R.reshape(9))
                pv_trans.append(t)
        npv = len(pv_lv)
        return GeometryDesc(
            name=self.name,
            solid_type=solid_type,
            solid_par=solid_par,
            mat_names=list(self.mats),
            mat_density=np.array(dens, dtype=np.float64),
            mat_el_off=np.array(off, dtype=np.int32),
            el_Z=np.array(Z, dtype=np.int32),
            el_A=np.array(A, dtype=np.float64),
            el_wfrac=np.array(W, dtype=np.float64),
            lv_solid=np.array(lv_solid, dtype=np.int32),
            lv_mat=np.array(lv_mat, dtype=np.int32),
            lv_dau_off=np.array(lv_off, dtype=np.int32),
            lv_dau_cnt=np.array(lv_cnt, dtype=np.int32),
            lv_voxelize=np.array(lv_vox, dtype=np.uint8),
            pv_lv=np.array(pv_lv, dtype=np.int32).reshape(npv),
            pv_rot=np.array(pv_rot, dtype=np.float64).reshape(npv, 9),
            pv_trans=np.array(pv_trans, dtype=np.float64).reshape(npv, 3),
            world_lv=world_lv,
            lv_names=[lv["name"] for lv in self.lvs],
        )


# ---------------------------------------------------------------------------
# Workload geometries
# ---------------------------------------------------------------------------

def tiny(rotated=False, seed=0):
    """1 m vacuum cube with eight 20 cm cubes at the octant centres (+-25 cm).

    Cube material alternates: water when the number of negative centre
    coordinates is even, lead when it is odd.  With ``rotated`` each cube gets
    a seeded random rotation (it still fits inside its octant).
    """
    b = Builder("tiny" + ("_rot" if rotated else ""))
    s_world = b.solid(BOX, 500.0, 500.0, 500.0)
    s_cube = b.solid(BOX, 100.0, 100.0, 100.0)
    world = b.lv(s_world, "vacuum", "world", voxelize=False)
    water = b.lv(s_cube, "water", "cube_water")
    lead = b.lv(s_cube, "lead", "cube_lead")
    rng = np.random.Generator(np.random.Philox(key=seed + 7))
    for i in range(8):
        c = [250.0 if (i >> k) & 1 else -250.0 for k in range(3)]
        nneg = sum(1 for x in c if x < 0)
        R = None
        if rotated:
            q = rng.normal(size=4)
            q /= np.linalg.norm(q)
            w, x, y, z = q
            R = np.array([
                [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
            ])
        b.place(world, water if nneg % 2 == 0 else lead, R, c)
    return b.build(world)


def calorimeter(n_layers=50, n_cells=20, pb_mm=5.0, si_mm=10.0, cell_mm=20.0):
    """Sampling calorimeter: world -> calo box -> layers -> cells (3 levels).

    Layers alternate lead / silicon starting with lead, stacked along z; each
    layer is tiled by n_cells x n_cells cell boxes of the layer's material.
    """
    b = Builder("calorimeter")
    half_xy = 0.5 * n_cells * cell_mm
    npair = n_layers // 2
    depth = npair * (pb_mm + si_mm) + (n_layers % 2) * pb_mm
    s_world = b.solid(BOX, 1000.0, 1000.0, 1000.0)
    s_calo = b.solid(BOX, half_xy, half_xy, 0.5 * depth)
    s_lpb = b.solid(BOX, half_xy, half_xy, 0.5 * pb_mm)
    s_lsi = b.solid(BOX, half_xy, half_xy, 0.5 * si_mm)
    s_cpb = b.solid(BOX, 0.5 * cell_mm, 0.5 * cell_mm, 0.5 * pb_mm)
    s_csi = b.solid(BOX, 0.5 * cell_mm, 0.5 * cell_mm, 0.5 * si_mm)
    world = b.lv(s_world, "vacuum", "world", voxelize=False)
    calo = b.lv(s_calo, "vacuum", "calo")
    lpb = b.lv(s_lpb, "lead", "layer_pb")
    lsi = b.lv(s_lsi, "silicon", "layer_si")
    cpb = b.lv(s_cpb, "lead", "cell_pb")
    csi = b.lv(s_csi, "silicon", "cell_si")
    b.place(world, calo)
    z = -0.5 * depth
    for i in range(n_layers):
        t = pb_mm if i % 2 == 0 else si_mm
        b.place(calo, lpb if i % 2 == 0 else lsi, None, (0.0, 0.0, z + 0.5 * t))
        z += t
    for layer, cell in ((lpb, cpb), (lsi, csi)):
        for ix in range(n_cells):
            for iy in range(n_cells):
                x = -half_xy + (ix + 0.5) * cell_mm
                y = -half_xy + (iy + 0.5) * cell_mm
                b.place(layer, cell, None, (x, y, 0.0))
    return b.build(world)


def barrel(seed=1, n_layers=64, n_seg=128, n_rings=16, n_orbs=32, name="barrel"):
    """Mixed-solid barrel: tube layers of phi segments, cone endcaps, orbs in the bore.

    An envelope tube (r 100-1500, half-length 2000) holds ``n_layers``
    concentric layers of pitch 1400/n_layers and half-pitch thickness; each
    layer is tiled by ``n_seg`` rotated phi segments.  Each side carries
    ``n_rings`` full-phi cone rings; the -z side reuses the +z logical volumes
    placed with a rotation by pi about x.  ``n_orbs`` balls of radius 50 sit in
    the bore at seeded positions.  Materials cycle water / lead / silicon.
    """
    rng = np.random.Generator(np.random.Philox(key=seed))
    cyc = ["water", "lead", "silicon"]
    b = Builder(name)
    s_world = b.solid(BOX, 1600.0, 1600.0, 3000.0)
    s_env = b.solid(TUBS, 100.0, 1500.0, 2000.0, 0.0, 2 * math.pi)
    world = b.lv(s_world, "vacuum", "world")
    env = b.lv(s_env, "vacuum", "envelope")
    b.place(world, env)
    pitch = 1400.0 / n_layers
    thick = 0.5 * pitch
    dphi = 2 * math.pi / n_seg
    layer_lvs = []
    for i in range(n_layers):
        r0 = 100.0 + pitch * i
        mat = cyc[i % 3]
        s_layer = b.solid(TUBS, r0, r0 + thick, 2000.0, 0.0, 2 * math.pi)
        s_seg = b.solid(TUBS, r0, r0 + thick, 2000.0, -0.5 * dphi, dphi)
        lv_layer = b.lv(s_layer, mat, f"layer{i}")
        lv_seg = b.lv(s_seg, mat, f"seg{i}")
        layer_lvs.append(lv_layer)
        for k in range(n_seg):
            b.place(lv_layer, lv_seg, rot_z((k + 0.5) * dphi))
    for lv_layer in layer_lvs:
        b.place(env, lv_layer)
    ring_lvs = []
    for j in range(n_rings):
        s_ring = b.solid(CONS, 100.0 - 5 * j, 1500.0 - 20 * j, 95.0 - 5 * j, 1480.0 - 20 * j,
                         25.0, 0.0, 2 * math.pi)
        ring_lvs.append(b.lv(s_ring, cyc[j % 3], f"ring{j}"))
    for j in range(n_rings):
        b.place(world, ring_lvs[j], None, (0.0, 0.0, 2025.0 + 50.0 * j))
    for j in range(n_rings):
        b.place(world, ring_lvs[j], rot_x_pi(), (0.0, 0.0, -(2025.0 + 50.0 * j)))
    s_orb = b.solid(ORB, 50.0)
    lv_orb = b.lv(s_orb, "silicon", "orb")
    span = 3880.0 / n_orbs
    for k in range(n_orbs):
        zk = -1940.0 + (k + 0.5) * span + rng.uniform(-10.0, 10.0)
        rho = 45.0 * math.sqrt(rng.uniform())
        ph = 2 * math.pi * rng.uniform()
        b.place(world, lv_orb, None, (rho * math.cos(ph), rho * math.sin(ph), zk))
    return b.build(world)


def barrel_variant(seed):
    """Barrel with seeded layer count (8..64) and segment count (16..256)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    n_layers = int(rng.integers(8, 65))
    n_seg = int(rng.integers(16, 257))
    return barrel(seed=seed, n_layers=n_layers, n_seg=n_seg, name=f"barrel_v{seed}")


def slab(material="water", thickness=50.0, half_xy=500.0):
    """A single slab (normal along z) in a vacuum world: the Beer-Lambert case."""
    b = Builder(f"slab_{material}")
    s_world = b.solid(BOX, 1000.0, 1000.0, 1000.0)
    s_slab = b.solid(BOX, half_xy, half_xy, 0.5 * thickness)
    world = b.lv(s_world, "vacuum", "world", voxelize=False)
    sl = b.lv(s_slab, material, "slab")
    b.place(world, sl)
    return b.build(world)


def foil_stack(n_foils=400, half_thickness=4.5e-10, half_xy=10.0, material="vacuum"):
    """Vacuum foils thinner than the surface tolerance (1e-9 mm), stacked
    along z without gaps and centred on the origin, in a vacuum world.

    Every step through such a foil is shorter than the tolerance, so tracks
    crossing the stack take runs of zero-length steps: the case of the
    zero-step push and kill rule.
    """
    b = Builder("foil_stack")
    s_world = b.solid(BOX, 100.0, 100.0, 100.0)
    s_foil = b.solid(BOX, half_xy, half_xy, half_thickness)
    world = b.lv(s_world, "vacuum", "world")
    foil = b.lv(s_foil, material, "foil")
    z0 = -n_foils * half_thickness
    for k in range(n_foils):
        b.place(world, foil, t=(0.0, 0.0, z0 + (2 * k + 1) * half_thickness))
    return b.build(world)


def solids_zoo(seed=5):
    """One daughter of every solid family (rotated and translated) in a box world.

    Used by unit tests of the per-solid distances under transforms.
    """
    rng = np.random.Generator(np.random.Philox(key=seed))
    b = Builder("zoo")
    s_world = b.solid(BOX, 1000.0, 1000.0, 1000.0)
    world = b.lv(s_world, "vacuum", "world")
    shapes = [
        (BOX, (120.0, 80.0, 60.0)),
        (TUBS, (40.0, 110.0, 90.0, 0.0, 2 * math.pi)),
        (TUBS, (30.0, 120.0, 70.0, 0.3, 1.9)),
        (CONS, (20.0, 90.0, 50.0, 130.0, 80.0, 0.0, 2 * math.pi)),
        (CONS, (0.0, 100.0, 30.0, 60.0, 70.0, -0.5, 2.4)),
        (ORB, (100.0,)),
        (TUBS, (0.0, 90.0, 60.0, 0.0, 2 * math.pi)),
        (CONS, (60.0, 110.0, 0.0, 40.0, 60.0, 0.0, 2 * math.pi)),
    ]
    centres = [(-500.0, -500.0, -500.0), (500.0, -500.0, -500.0), (-500.0, 500.0, -500.0),
               (500.0, 500.0, -500.0), (-500.0, -500.0, 500.0), (500.0, -500.0, 500.0),
               (-500.0, 500.0, 500.0), (500.0, 500.0, 500.0)]
    mats = ["water", "lead", "silicon"]
    for i, ((st, par), c) in enumerate(zip(shapes, centres)):
        s = b.solid(st, *par)
        lv = b.lv(s, mats[i % 3], f"zoo{i}")
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ])
        off = rng.uniform(-60.0, 60.0, size=3)
        b.place(world, lv, R, tuple(np.array(c) + off))
    return b.build(world)


def solids_zoo_more(seed=6):
    """The solid families beyond the paper's boxes, tubes, cones and balls, one
    rotated and translated daughter each, in a box world: trapezoids of both
    tapers and a near-box; sphere sections (full shell, phi wedge, theta bands
    above, across and below the equator, the upper hemisphere, a band with a
    phi wedge), for the per-solid tests of those families."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    b = Builder("zoo_more")
    s_world = b.solid(BOX, 1000.0, 1000.0, 1000.0)
    world = b.lv(s_world, "vacuum", "world")
    shapes = [
        (TRD, (60.0, 120.0, 90.0, 40.0, 80.0)),
        (TRD, (100.0, 30.0, 70.0, 70.0, 50.0)),
        (TRD, (80.0, 80.0, 80.0, 80.0, 80.0)),
        (TRD, (20.0, 140.0, 120.0, 10.0, 110.0)),
        # sphere sections: rmin, rmax, sphi, dphi, stheta, dtheta
        (SPHERE, (40.0, 120.0, 0.0, 2 * math.pi, 0.0, math.pi)),
        (SPHERE, (0.0, 110.0, 0.4, 2.2, 0.0, math.pi)),
        (SPHERE, (30.0, 130.0, 0.0, 2 * math.pi, 0.3, 0.9)),
        (SPHERE, (50.0, 120.0, -0.7, 1.9, 0.8, 1.4)),
        (SPHERE, (0.0, 100.0, 0.0, 2 * math.pi, 0.0, 0.5 * math.pi)),
        (SPHERE, (20.0, 115.0, 1.0, 3.0, 1.9, 1.0)),
    ]
    centres = [(-500.0, -500.0, -500.0), (500.0, -500.0, 500.0), (-500.0, 500.0, 500.0),
               (500.0, 500.0, -500.0), (0.0, 0.0, 0.0), (-500.0, -500.0, 500.0),
               (500.0, 500.0, 500.0), (-500.0, 500.0, -500.0), (500.0, -500.0, -500.0),
               (0.0, 500.0, 0.0)]
    mats = ["water", "lead", "silicon"]
    for i, ((st, par), c) in enumerate(zip(shapes, centres)):
        s = b.solid(st, *par)
        lv = b.lv(s, mats[i % 3], f"more{i}")
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ])
        off = rng.uniform(-60.0, 60.0, size=3)
        b.place(world, lv, R, tuple(np.array(c) + off))
    return b.build(world)


def endcap(n_wedges=36, n_crystals=4, r_in=400.0, r_out=800.0, half_t=60.0, z_c=900.0):
    """Two endcap discs of trapezoid wedges (the tapered modules of a CMS-like
    endcap, Sec. 3.5's CMS case) around a central tube, in a vacuum world.

    Each disc at z = +-z_c holds ``n_wedges`` trapezoid wedges around the z
    axis, their local z pointing radially outward (x half width growing from
    the inner to the outer radius, y half width = disc half thickness); each
    wedge holds ``n_crystals`` trapezoid crystals stacked radially.  Materials
    alternate lead / silicon wedge by wedge, crystals lead.  A silicon tube
    layer (r 300-320, half length 700) sits between the discs, and a spherical
    shell section (r 100-150, polar angles 0.5-2.6 rad, four phi quarters of
    lead and water) around the origin.
    """
    b = Builder("endcap")
    s_world = b.solid(BOX, 1200.0, 1200.0, 1200.0)
    world = b.lv(s_world, "vacuum", "world")
    s_tube = b.solid(TUBS, 300.0, 320.0, 700.0, 0.0, 2 * math.pi)
    b.place(world, b.lv(s_tube, "silicon", "tube"))
    # a spherical shell section around the source: polar band 0.5-2.6 rad, open
    # at the poles, in four phi quarters of lead and water
    for k in range(4):
        s_sh = b.solid(SPHERE, 100.0, 150.0, 0.5 * math.pi * k, 0.5 * math.pi, 0.5, 2.1)
        b.place(world, b.lv(s_sh, "lead" if k % 2 == 0 else "water", f"shell{k}"))
    half_phi = math.pi / n_wedges
    dz = 0.5 * (r_out - r_in)
    # wedge half widths at the inner and outer radius, kept inside the phi slice
    dx1 = 0.98 * r_in * math.tan(half_phi)
    dx2 = 0.98 * r_out * math.tan(half_phi)
    wedges = []
    for m, mat in enumerate(("lead", "silicon")):
        s_w = b.solid(TRD, dx1, dx2, half_t, half_t, dz)
        lv_w = b.lv(s_w, mat, f"wedge_{mat}")
        # crystals: radial slices of the wedge, shrunk by 0.5 mm on every side
        pitch = 2 * dz / n_crystals
        for k in range(n_crystals):
            z0 = -dz + k * pitch + 0.5
            z1 = -dz + (k + 1) * pitch - 0.5
            w0 = dx1 + (dx2 - dx1) * (z0 + dz) / (2 * dz) - 0.5
            w1 = dx1 + (dx2 - dx1) * (z1 + dz) / (2 * dz) - 0.5
            s_c = b.solid(TRD, w0, w1, half_t - 0.5, half_t - 0.5, 0.5 * (z1 - z0))
            lv_c = b.lv(s_c, "lead", f"crystal_{mat}_{k}")
            b.place(lv_w, lv_c, None, (0.0, 0.0, 0.5 * (z0 + z1)))
        wedges.append(lv_w)
    rc = 0.5 * (r_in + r_out)
    for side in (1.0, -1.0):
        for j in range(n_wedges):
            ph = (j + 0.5) * 2 * half_phi
            c, s_ = math.cos(ph), math.sin(ph)
            # local x tangential, local y along the global z axis, local z radial
            R = np.array([[-s_, 0.0, c], [c, 0.0, s_], [0.0, 1.0, 0.0]])
            b.place(world, wedges[j % 2], R, (rc * c, rc * s_, side * z_c))
    return b.build(world)


def spheres(n_per_axis=20, radius=100.0, half=2500.0):
    """The paper's Spheres geometry: aluminium balls on a regular grid in a vacuum cube.

    Sec. 3.5 gives 8000 balls in a 5 m cube but not the radius; the pitch of a
    20^3 grid is 250 mm and the radius is a free parameter here.
    """
    b = Builder("spheres")
    s_world = b.solid(BOX, half, half, half)
    s_ball = b.solid(ORB, radius)
    world = b.lv(s_world, "vacuum", "world")
    ball = b.lv(s_ball, "aluminium", "ball")
    pitch = 2 * half / n_per_axis
    for ix in range(n_per_axis):
        for iy in range(n_per_axis):
            for iz in range(n_per_axis):
                c = (-half + (ix + 0.5) * pitch, -half + (iy + 0.5) * pitch,
                     -half + (iz + 0.5) * pitch)
                b.place(world, ball, None, c)
    return b.build(world)
