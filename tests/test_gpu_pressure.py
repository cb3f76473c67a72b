"""Stokes pressure (pfmm_eval_pressure) against the oracle's periodic
pressure, doubly and singly periodic, both precisions, sources as targets
and separate targets. Bars as in tests/parity.py."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


@pytest.mark.parametrize("cell,periodic", [(((1.0, 0.0), (0.0, 1.0)), 2), (((2.0, 0.0), (0.4, 1.0)), 2),
                                           (((1.0, 0.0), (0.5, np.sqrt(3) / 2)), 2), (((100.0, 0.0), (0.0, 1.0)), 2),
                                           (((1.3, 0.4), (0.2, 2.0)), 1)])
@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-10), ("mixed", 1e-6, 1e-6)])
@pytest.mark.parametrize("self_trg", [True, False])
def test_pressure_matches_oracle(env, cell, periodic, prec, tol, bar, self_trg):
    P, torch, dev = env
    e1, e2 = cell
    rng = np.random.default_rng(71)
    n = 900
    if periodic == 1:
        from test_gpu_p1 import strip_points
        src = strip_points(rng, e1, e2, n)
        trg = None if self_trg else strip_points(rng, e1, e2, 300)
    else:
        src = W.cell_points(rng, e1, e2, n)
        trg = None if self_trg else W.cell_points(rng, e1, e2, 300)
    f = W.neutral_forces(rng, n)
    print(f"case pressure {cell} P{periodic} {prec} self={self_trg}", flush=True)
    plan = P.Plan("stokes", e1, e2, tol, precision=prec, self_exclude=self_trg, periodic=periodic)
    p = P.pfmm_eval_pressure(plan, torch.tensor(src, device=dev), torch.tensor(f, device=dev),
                             None if trg is None else torch.tensor(trg, device=dev))
    po = oracle.stokes_pressure(e1, e2, src, f, trg, periodic=periodic)
    check(bar, (p.cpu().numpy(), po), label=f"pressure {cell} P{periodic} {prec} self={self_trg}")


def test_pressure_several_densities_and_errors(env):
    P, torch, dev = env
    e1, e2 = (1.0, 0.0), (0.3, 1.1)
    rng = np.random.default_rng(72)
    src = W.cell_points(rng, e1, e2, 500)
    f = W.neutral_forces(rng, 500, 3)
    plan = P.Plan("stokes", e1, e2, 1e-6, precision="mixed", self_exclude=True, n_dens=3)
    p = P.pfmm_eval_pressure(plan, torch.tensor(src, device=dev), torch.tensor(f, device=dev)).cpu().numpy()
    for v in range(3):
        check(1e-6, (p[v], oracle.stokes_pressure(e1, e2, src, f[v])), label=f"pressure nd=3 v={v}")
    lap = P.Plan("laplace", e1, e2, 1e-6, self_exclude=True)
    with pytest.raises(ValueError):
        P.pfmm_eval_pressure(lap, torch.tensor(src, device=dev), torch.tensor(f[0], device=dev))
    from paper_2111_01083_amd import _lib as L
    rc = L.load().pfmm_eval_pressure(lap.handle, 500, None, None, 500, None, None, None, 0, None)
    assert rc == -1    # not a Stokes plan
