"""GPU: ComputeStep and ComputeSafety at scale, against the oracle.

ComputeStep: a million random queries per geometry plus the cases where the
voxel walk and the tie rule are most exposed -- rays lying in planes shared
by neighbouring volumes (layer faces of the calorimeter, which are also its
voxel slice planes; the phi faces between barrel segments) and rays running
along or crossing edges shared by four cells or by segments and layer
surfaces.  Limiter and next touchable exact, step within 1e-9 relative.

ComputeSafety: without voxels (the tiny geometry) the GPU safety is the
oracle's brute-force isotropic safety.  With voxels the two are different
lower bounds of the distance to the nearest boundary (the start node's faces
bound the GPU's, while a daughter outside the node, which the GPU does not
consult, may have an isotropic bound below its true distance and below the
node faces' distance), so neither bounds the other; element by element the
GPU safety must not exceed an upper bound of the true distance, the shortest
oracle ComputeStep over 8 directions from the point, and zero safeties must
be rare where the oracle's is clearly positive.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import ATOL, RTOL, ctx, geom, print_case, sample_points, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _unit(a):
    return a / np.linalg.norm(a, axis=1)[:, None]


def _calorimeter_special(rng, m):
    """Points on layer faces with in-plane directions, and points on the
    edges shared by four cells with directions along the edge or random."""
    thick = np.array([5.0 if i % 2 == 0 else 10.0 for i in range(50)])
    faces = -187.5 + np.concatenate([[0.0], np.cumsum(thick)])
    z = faces[rng.integers(0, len(faces), m)]
    p1 = np.column_stack([rng.uniform(-200, 200, m), rng.uniform(-200, 200, m), z])
    ph = rng.uniform(0, 2 * np.pi, m)
    d1 = np.column_stack([np.cos(ph), np.sin(ph), np.zeros(m)])
    # some in-plane rays exactly along a cell row boundary too
    k = m // 4
    p1[:k, 1] = -200 + 20 * rng.integers(0, 21, k)
    d1[:k] = np.column_stack([np.sign(rng.uniform(-1, 1, k)), np.zeros(k), np.zeros(k)])
    ex = -200 + 20 * rng.integers(1, 20, m)
    ey = -200 + 20 * rng.integers(1, 20, m)
    p2 = np.column_stack([ex.astype(float), ey.astype(float), rng.uniform(-187.4, 187.4, m)])
    d2 = W.primaries.isotropic(rng, m)
    d2[: m // 3] = np.column_stack([np.zeros(m // 3), np.zeros(m // 3), np.sign(rng.uniform(-1, 1, m // 3))])
    # diagonal rays through edges in the xy plane
    j = slice(m // 3, 2 * (m // 3))
    s = np.sign(rng.uniform(-1, 1, (m // 3, 2)))
    d2[j] = _unit(np.column_stack([s[:, 0], s[:, 1], np.zeros(m // 3)]))
    return np.concatenate([p1, p2]), np.concatenate([d1, d2])


def _barrel_special(rng, m):
    """Points on the phi faces between segments with directions in that plane,
    and points on the edges where a phi face meets a layer's inner or outer
    surface, with random directions."""
    pitch = 1400.0 / 64
    dphi = 2 * np.pi / 128
    layer = rng.integers(0, 64, m)
    r0 = 100.0 + pitch * layer
    rho = r0 + rng.uniform(0.0, 0.5 * pitch, m)
    phib = dphi * rng.integers(0, 128, m)
    z = rng.uniform(-1990, 1990, m)
    p1 = np.column_stack([rho * np.cos(phib), rho * np.sin(phib), z])
    a = rng.uniform(-1, 1, m)
    b = np.sqrt(1 - a * a) * np.sign(rng.uniform(-1, 1, m))
    d1 = np.column_stack([a * np.cos(phib), a * np.sin(phib), b])
    edge_r = np.where(rng.uniform(size=m) < 0.5, r0, r0 + 0.5 * pitch)
    p2 = np.column_stack([edge_r * np.cos(phib), edge_r * np.sin(phib), z])
    d2 = W.primaries.isotropic(rng, m)
    return np.concatenate([p1, p2]), np.concatenate([d1, d2])


SPECIAL = {"calorimeter": _calorimeter_special, "barrel": _barrel_special}


@pytest.mark.parametrize("name", ["calorimeter", "barrel", "zoo", "endcap"])
def test_compute_step_million_queries(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("step_1e6", name)
    rng = np.random.Generator(np.random.Philox(key=2002))
    n = 1_000_000
    pts = sample_points(desc, rng, n)
    dirs = W.primaries.isotropic(rng, n)
    if name in SPECIAL:
        sp, sd = SPECIAL[name](rng, 100_000)
        pts = np.concatenate([pts, sp])
        dirs = np.concatenate([dirs, sd])
    T = og.locate(pts, dirs)
    ok = T >= 0
    pts, dirs, T = pts[ok], dirs[ok], T[ok]
    s_ref, l_ref, n_ref = og.compute_step(pts, dirs, T)
    s, l, nx = ctx.compute_step(gid, torch.from_numpy(pts).cuda(), torch.from_numpy(dirs).cuda(),
                                torch.from_numpy(T.astype(np.int32)).cuda())
    s, l, nx = s.cpu().numpy(), l.cpu().numpy(), nx.cpu().numpy()
    bad = np.nonzero(l != l_ref)[0]
    assert len(bad) == 0, (len(bad), bad[:5], pts[bad[:3]], dirs[bad[:3]], l[bad[:3]], l_ref[bad[:3]])
    fin = np.isfinite(s_ref)
    assert np.array_equal(np.isfinite(s), fin)
    assert np.allclose(s[fin], s_ref[fin], rtol=RTOL, atol=ATOL)
    assert np.array_equal(nx, n_ref)
    print(name, "queries", len(pts), "zero steps", int((s_ref == 0).sum()), flush=True)


@pytest.mark.parametrize("name", ["tiny", "tiny_rot", "calorimeter", "barrel", "zoo", "zoo_more", "endcap"])
def test_safety_against_brute_force(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("safety_brute", name)
    rng = np.random.Generator(np.random.Philox(key=2003))
    pts = sample_points(desc, rng, 200_000)
    T = og.locate(pts)
    ok = T >= 0
    pts, T = pts[ok], T[ok]
    ref = og.compute_safety(pts, T)
    got = ctx.compute_safety(gid, torch.from_numpy(pts).cuda(),
                             torch.from_numpy(T.astype(np.int32)).cuda()).cpu().numpy()
    assert np.all(got >= 0)
    if name.startswith("tiny"):
        # no voxel grid: the same isotropic lower bound over every daughter
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    else:
        m = min(len(pts), 50_000)
        dirs = W.primaries.isotropic(rng, 8 * m)
        s, _, _ = og.compute_step(np.repeat(pts[:m], 8, axis=0), dirs, np.repeat(T[:m], 8), with_next=False)
        upper = s.reshape(m, 8).min(axis=1)
        over = got[:m] > upper * (1 + 1e-12) + 1e-12
        assert not over.any(), (int(over.sum()), np.nonzero(over)[0][:5])
        clear = ref > 1e-6
        assert np.mean(got[clear] == 0) < 1e-3
        assert np.median(got[clear] / ref[clear]) > 0.01
    print(name, "points", len(pts), "median ratio", float(np.median(got[ref > 0] / ref[ref > 0])), flush=True)
