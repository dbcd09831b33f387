"""GPU: the exit normal of gnav_compute_step_ex against the oracle.

On random and on-surface queries over six geometries (boxes, rotated boxes,
rotated tube/cone/orb sections, the calorimeter and the barrel): the validity
code must match exactly, and where the end point lies on a single face the
normal must match within 1e-12 per component (frames are composed differently
on the two sides, in long double on the GPU and level by level in the
oracle).  On edges and corners the face whose signed value is largest may
differ by rounding between the two sides, so there only unit length is
required.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import (ATOL, GEOMS, RTOL, ctx, geom, print_case, sample_points,  # noqa: F401
                              surface_points, torch_dev)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(GEOMS))
def test_exit_normal_parity(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("normal", name)
    rng = np.random.Generator(np.random.Philox(key=1010))
    pts = sample_points(desc, rng, 30000)
    dirs = W.primaries.isotropic(rng, len(pts))
    end, d2, nxt = surface_points(desc, og, rng, 10000)
    keep = nxt >= 0
    pts = np.concatenate([pts, end[keep]])
    dirs = np.concatenate([dirs, d2[keep]])
    T = og.locate(pts, dirs)
    ok = T >= 0
    pts, dirs, T = pts[ok], dirs[ok], T[ok]
    s_ref, l_ref, n_ref, nrm_ref, val_ref = og.compute_step_normal(pts, dirs, T)
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    s, l, nx, nrm, val = (a.cpu().numpy() for a in ctx.compute_step(gid, tt(pts), tt(dirs),
                                                                     tt(T.astype(np.int32)),
                                                                     with_normal=True))
    assert np.array_equal(l, l_ref) and np.array_equal(nx, n_ref)
    assert np.allclose(s, s_ref, rtol=RTOL, atol=ATOL)
    assert np.array_equal(val, val_ref), np.argwhere(val != val_ref)[:5]
    face = val == 1
    assert face.sum() > 0.5 * len(val)
    assert np.allclose(nrm[face], nrm_ref[face], rtol=0, atol=1e-12)
    edge = val == 2
    assert np.allclose(np.linalg.norm(nrm[edge], axis=1), 1, atol=1e-12)
    none = val == 0
    assert np.array_equal(none, ~np.isfinite(s_ref))
    assert not nrm[none].any()
    # exit normals point along the direction of travel
    assert np.all(np.sum(nrm[face] * dirs[face], 1) >= -1e-12)
