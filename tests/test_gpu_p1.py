"""Singly periodic plans (periodic in e1 only, the operator P1 of Sec. 3,
eq. ksplitting1) on the GPU against the FP64 oracle's P1 sums: the cell and
its two neighbours directly, the west/east columns through the planner's
rule. Points lie anywhere along e1 (wrapped) and within the strip's height
across it. Bars as in tests/parity.py."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check

pytestmark = pytest.mark.gpu

STRIPS = {"square": ((1.0, 0.0), (0.0, 1.0)), "tilted": ((1.3, 0.4), (0.2, 2.0)),
          "tall": ((1.0, 0.0), (0.0, 8.0)), "wide": ((6.0, 0.0), (0.0, 1.0))}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


def strip_points(rng, e1, e2, n):
    e1a = np.array(e1, float)
    d = np.hypot(*e1a)
    along = e1a / d
    perp = np.array([-along[1], along[0]])
    H = abs(np.dot(np.array(e2, float), perp))
    # anywhere along e1 (shifted by whole periods to exercise the wrapping)
    return np.outer(along, d * (rng.random(n) - 0.5 + rng.integers(-2, 3, n))) + np.outer(perp, H * (rng.random(n) - 0.5))


@pytest.mark.parametrize("strip", list(STRIPS))
@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 2.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-10), ("mixed", 1e-6, 1e-6)])
@pytest.mark.parametrize("self_trg", [True, False])
def test_p1_matches_oracle(env, strip, kernel, beta, prec, tol, bar, self_trg):
    P, torch, dev = env
    e1, e2 = STRIPS[strip]
    rng = np.random.default_rng(51)
    n = 1100
    src = strip_points(rng, e1, e2, n)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    trg = None if self_trg else strip_points(rng, e1, e2, 400)
    print(f"case p1 {kernel} {strip} {prec} self={self_trg}", flush=True)
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, self_exclude=self_trg, periodic=1)
    assert plan.info["n_images"] == 3
    pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev),
                     None if trg is None else torch.tensor(trg, device=dev))
    po, go = oracle.singly_periodic(kernel, e1, src, dens, trg, beta=beta)
    check(bar, (pot.cpu().numpy(), po), (grad.cpu().numpy(), go), label=f"p1 {kernel} {strip} {prec} self={self_trg}")


def test_p1_periodic_along_e1_only(env):
    # shifting every point by a period leaves the result; the field is not
    # periodic across the strip (no images in that direction)
    P, torch, dev = env
    e1, e2 = STRIPS["tilted"]
    rng = np.random.default_rng(52)
    src = strip_points(rng, e1, e2, 500)
    q = W.neutral_charges(rng, 500)
    trg = strip_points(rng, e1, e2, 200)
    plan = P.Plan("laplace", e1, e2, 1e-10, periodic=1)
    p0, g0 = plan(torch.tensor(src, device=dev), torch.tensor(q, device=dev), torch.tensor(trg, device=dev))
    sh = 2 * np.array(e1)[:, None]
    p1, g1 = plan(torch.tensor(src + sh, device=dev), torch.tensor(q, device=dev), torch.tensor(trg - sh, device=dev))
    check(1e-12, (p1.cpu().numpy(), p0.cpu().numpy()), (g1.cpu().numpy(), g0.cpu().numpy()), label="p1 shift")


def test_p1_energy_gradient_matches_oracle_forces(env):
    # the adjoint (kernel symmetry) holds for the singly periodic sum too
    P, torch, dev = env
    e1, e2 = STRIPS["square"]
    rng = np.random.default_rng(53)
    n = 600
    src = strip_points(rng, e1, e2, n)
    q = W.neutral_charges(rng, n)
    plan = P.Plan("laplace", e1, e2, 1e-10, self_exclude=True, periodic=1)
    x = torch.tensor(src, device=dev, requires_grad=True)
    qt = torch.tensor(q, device=dev, requires_grad=True)
    E = 0.5 * (qt * P.periodic_potential(plan, x, qt)).sum()
    E.backward()
    pot, grad = oracle.singly_periodic("laplace", e1, src, q, None)
    check(1e-9, (x.grad.cpu().numpy(), q * grad), label="p1 forces")


def test_p1_plans_are_not_batched_and_have_no_nufft(env):
    P, torch, dev = env
    with pytest.raises(P.PfmmError):
        P.Plan("laplace", (1.0, 0.0), (0.0, 1.0), 1e-6, far_mode="nufft", periodic=1)
    plan = P.Plan("laplace", (1.0, 0.0), (0.0, 1.0), 1e-6, self_exclude=True, periodic=1)
    with pytest.raises(P.PfmmError):
        P.Batch([plan], [0, 10])
