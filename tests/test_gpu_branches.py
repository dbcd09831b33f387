"""GPU: per-track parity on the rarely taken branches of the transport loop.

* energy cut raised until it fires (the configs' 1 keV cut never does): the
  cut tracks, their deposits and every other track against the oracle;
* zero-length steps on a stack of foils thinner than the tolerance: every
  photon is pushed twice and killed, on the axis-aligned box build (block 64)
  and on the general build (block 128);
* pair conversions overflowing the block stack are in test_gpu_parity.py.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import (EXACT, RTOL, compare_logs, ctx, geom, print_case,  # noqa: F401
                              run_transport, torch_dev)

pytestmark = pytest.mark.gpu


def _check(got, ref, cap):
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, cap)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["escaped_event"], ref["escaped_event"], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["edep_touchable"], ref["edep_touchable"], rtol=RTOL, atol=1e-12)


@pytest.mark.parametrize("name,n,ecut,block", [("tiny", 6000, 0.3, 0), ("calorimeter", 4000, 0.5, 0),
                                               ("calorimeter", 4000, 0.5, 128), ("barrel", 2000, 0.2, 0)])
def test_energy_cut_parity(ctx, torch_dev, oracle_lib, name, n, ecut, block):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("ecut", name, ecut, block)
    _, prim, _ = W.WORKLOADS[name](n=n)
    cap = 512
    got = run_transport(ctx, torch, gid, prim, cap, e_cut=ecut, block=block)
    ref = og.transport(prim, seed=0, ecut=ecut, log_cap=cap)
    assert ref["counters"]["cutoff"] > 100
    _check(got, ref, cap)


@pytest.mark.parametrize("block", [64, 128])
def test_zero_step_push_and_kill_parity(ctx, torch_dev, oracle_lib, block):
    torch = torch_dev
    from tests.gpu_common import GEOMS
    GEOMS.setdefault("foil_stack", lambda: W.geometry.foil_stack())
    desc, gid, nt, og = geom(ctx, "foil_stack", oracle_lib)
    print_case("zero_steps", block)
    n = 3000
    rng = np.random.default_rng(9)
    pos = np.stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), np.full(n, -50.0)], 1)
    d = np.tile([0.0, 0.0, 1.0], (n, 1))
    # a third of the photons slightly oblique: longer steps through the foils, still
    # below the tolerance
    d[: n // 3, 0] = rng.uniform(-0.2, 0.2, n // 3)
    d /= np.linalg.norm(d, axis=1)[:, None]
    prim = W.primaries.one_per_event(pos, d, np.full(n, 1.0))
    cap = 64
    got = run_transport(ctx, torch, gid, prim, cap, block=block)
    ref = og.transport(prim, seed=0, log_cap=cap)
    assert ref["counters"]["stuck"] > n // 2 and ref["counters"]["pushes"] > n
    _check(got, ref, cap)
