"""GPU: the free path of Alg. 1 alone (the paper's Table 1 phase) against the oracle,
on the tiny geometry and on Spheres with the paper's Random and Regular particle sets."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import ctx, print_case, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

MU_AL = 0.06146  # cm2/g, aluminium at 1 MeV (Sec. 3.4)


def _check(ctx, torch, oracle_lib, desc, pos, dirs, life, mu_mass, energy=1.0):
    gid, _ = ctx.upload_geometry(desc)
    og = oracle_lib.Geometry(desc)
    if mu_mass > 0:
        og.set_paper_mode(True, mu_mass)
    t, nb = ctx.free_path(gid, torch.from_numpy(pos).cuda(), torch.from_numpy(dirs).cuda(),
                          torch.from_numpy(life).cuda(), energy=energy, mu_mass=mu_mass)
    t, nb = t.cpu().numpy(), nb.cpu().numpy()
    ref = [og.free_path(p, d, energy, y) for p, d, y in zip(pos, dirs, life)]
    t_ref = np.array([r[0] for r in ref])
    nb_ref = np.array([r[1] for r in ref])
    assert np.array_equal(nb, nb_ref)
    fin = np.isfinite(t_ref)
    assert np.array_equal(np.isfinite(t), fin)
    assert np.allclose(t[fin], t_ref[fin], rtol=1e-9, atol=1e-12)
    return t, nb


def test_free_path_tiny_tables_and_paper_mu(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    print_case("free_path_tiny")
    pos, dirs, life = W.primaries.paper_random(3000, seed=5)
    desc = W.geometry.tiny(rotated=True)
    _check(ctx, torch, oracle_lib, desc, pos, dirs, life, 0.0, energy=1.0)
    _check(ctx, torch, oracle_lib, desc, pos, dirs, life * 3.0, MU_AL)


def test_free_path_spheres_random(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    print_case("free_path_spheres_random")
    pos, dirs, life = W.primaries.paper_random(1500, seed=0)
    t, nb = _check(ctx, torch, oracle_lib, W.geometry.spheres(), pos, dirs, life, MU_AL)
    assert nb.max() > 2


def test_free_path_spheres_regular_subgrid(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    print_case("free_path_spheres_regular")
    pos, dirs, life = W.primaries.paper_regular()
    keep = np.arange(0, len(life), 97)
    _check(ctx, torch, oracle_lib, W.geometry.spheres(), pos[keep], dirs[keep], life[keep], MU_AL)
