"""Symmetric near field (targets == sources, one density vector): every pair
(i, j, l) and its mirror (j, i, -l) are evaluated once for both points (the
free-space kernels are even, Sec. 1 eq. psum). Parity with the FP64 oracle
and with the one-sided near field on the same inputs, over sizes that leave
ragged target tiles and source sub-tiles."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check, golden, rel

pytestmark = pytest.mark.gpu

CELLS = {"square": ((1.0, 0.0), (0.0, 1.0)), "sheared": ((2.0, 0.0), (0.9, 1.3)),
         "long": ((10.0, 0.0), (0.0, 1.0))}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


def run(env, kernel, e1, e2, src, dens, prec, tol, beta, mode):
    P, torch, dev = env
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, self_exclude=True, near_mode=mode)
    pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev))
    torch.cuda.synchronize()
    return pot.cpu().numpy(), grad.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 63, 256, 257, 700, 1537])
@pytest.mark.parametrize("cell", list(CELLS))
@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 3.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-10), ("mixed", 1e-6, 1e-6)])
def test_mutual_matches_oracle_and_one_sided(env, n, cell, kernel, beta, prec, tol, bar):
    e1, e2 = CELLS[cell]
    rng = np.random.default_rng(n)
    src = W.cell_points(rng, e1, e2, n)
    if kernel == "yukawa":
        dens = rng.standard_normal(n)          # Yukawa needs no neutrality
    else:
        dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    if n == 1 and kernel != "yukawa":
        pytest.skip("a single neutral charge is zero")
    print(f"case mutual {kernel} {cell} n={n} {prec}", flush=True)
    pm, gm = run(env, kernel, e1, e2, src, dens, prec, tol, beta, "mutual")
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, None, beta=beta)
    p1, g1 = run(env, kernel, e1, e2, src, dens, prec, tol, beta, "one_sided")
    agree = 1e-12 if prec == "fp64" else 1e-6
    if n == 1:
        # one charge and its images: the field at the charge vanishes by symmetry
        check(bar, (pm, po), label=f"mutual {kernel} {cell} n=1 {prec}")
        assert np.abs(gm).max() < 1e-2 * bar * np.abs(pm).max()
        return
    check(bar, (pm, po), (gm, go), label=f"mutual {kernel} {cell} n={n} {prec}")
    assert rel(pm, p1) < agree and rel(gm, g1) < agree, (rel(pm, p1), rel(gm, g1))


def test_symmetric_path_at_full_size_is_accurate(env):
    # square cell, N = 2e5 uniform, Yukawa beta = 10, mixed, tol 1e-6: the
    # symmetric direct sum (AUTO takes the FMM at this size); sampled outputs
    # against the oracle
    P, torch, dev = env
    e1, e2, src, q = W.square_uniform("yukawa")
    print("mutual full size", flush=True)
    pm, gm = run(env, "yukawa", e1, e2, src, q, "mixed", 1e-6, 10.0, "mutual")
    ref = golden("square_n200k_yukawa", src, q)
    idx = ref["idx"]
    check(1e-6, (pm[idx], ref["pot"]), (gm[:, idx], ref["grad"]), label="mutual full size")


@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 10.0), ("stokes", 0.0)])
def test_repeated_evaluations_agree_to_fp64_rounding(env, kernel, beta):
    # the binned order is stable (ascending index within a bin), so two runs
    # differ only through the order of the FP64 atomic adds
    P, torch, dev = env
    n = 20000
    rng = np.random.default_rng(5)
    e1, e2 = CELLS["sheared"]
    src = torch.tensor(W.cell_points(rng, e1, e2, n), device=dev)
    dens = torch.tensor(W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n), device=dev)
    plan = P.Plan(kernel, e1, e2, 1e-6, beta=beta, precision="mixed", self_exclude=True)
    a = [t.cpu().numpy() for t in plan(src, dens)]
    b = [t.cpu().numpy() for t in plan(src, dens)]
    assert rel(a[0], b[0]) < 1e-13 and rel(a[1], b[1]) < 1e-13


@pytest.mark.parametrize("a_ratio,groups", [(2000.0, 1), (4000.0, 3)])
@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
def test_thin_cells_share_logs_across_images(env, a_ratio, groups, kernel):
    # the mixed symmetric kernel takes one log2 of the FP32 product of r^2 over
    # a group of images; in very thin cells the y-images are close together, so
    # the product starts at 2^e0 > 1 (A = 2000) or the groups are the rows of
    # images one period apart (A = 4000)
    P, torch, dev = env
    n = 1537
    e1, e2 = (a_ratio, 0.0), (0.0, 1.0)
    rng = np.random.default_rng(11)
    src = W.cell_points(rng, e1, e2, n)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    plan = P.Plan(kernel, e1, e2, 1e-6, precision="mixed", self_exclude=True)
    assert plan.info["n_log_groups"] == groups
    print(f"case thin {kernel} A={a_ratio}", flush=True)
    pm, gm = run(env, kernel, e1, e2, src, dens, "mixed", 1e-6, 0.0, "mutual")
    p1, g1 = run(env, kernel, e1, e2, src, dens, "mixed", 1e-6, 0.0, "one_sided")
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, None)
    check(1e-6, (pm, po), (gm, go), label=f"thin {kernel} A={a_ratio}")
    assert rel(pm, p1) < 1e-6 and rel(gm, g1) < 1e-6, (rel(pm, p1), rel(gm, g1))


@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
def test_near_coincident_points(env, kernel):
    # pairs 1e-6, 1e-9 and 1e-11 apart (r^2 down to 1e-22): exact in the
    # diagonal tiles (the self-pair guard 2^-100 is far below their r^2) and in
    # the images' FP32 r^2 product of the symmetric kernel (no underflow)
    P, torch, dev = env
    n = 600
    e1, e2 = CELLS["square"]
    rng = np.random.default_rng(12)
    src = W.cell_points(rng, e1, e2, n)
    for k, sep in enumerate([1e-6, 1e-9, 1e-11]):
        ang = rng.uniform(0, 2 * np.pi)
        src[:, 2 * k + 1] = src[:, 2 * k] + sep * np.array([np.cos(ang), np.sin(ang)])
    # pairs 1e-9 apart through an edge and through a corner of the cell: close
    # only under a nonzero image shift, and far apart in the binned order
    src[:, 6], src[:, 7] = (0.5 - 5e-10, 0.1), (-0.5 + 5e-10, 0.1)
    src[:, 8], src[:, 9] = (0.5 - 3e-10, 0.5 - 4e-10), (-0.5 + 3e-10, -0.5 + 4e-10)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    print(f"case coincident {kernel}", flush=True)
    pm, gm = run(env, kernel, e1, e2, src, dens, "mixed", 1e-6, 0.0, "mutual")
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, None)
    assert np.isfinite(pm).all() and np.isfinite(gm).all()
    check(1e-6, (pm, po), (gm, go), label=f"coincident {kernel}")


@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 3.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-10), ("mixed", 1e-6, 1e-6)])
def test_widest_near_region(env, kernel, beta, prec, tol, bar):
    # m0 = 3: 21 images, the most the plan allows (image masks and log groups
    # at their widest); symmetric and one-sided paths against the oracle
    P, torch, dev = env
    n = 700
    e1, e2 = (1.0, 0.0), (0.3, 1.0)
    rng = np.random.default_rng(21)
    src = W.cell_points(rng, e1, e2, n)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    print(f"case m0=3 {kernel} {prec}", flush=True)
    outs = []
    for mode in ("mutual", "one_sided"):
        plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, self_exclude=True, near_mode=mode, m0=3)
        assert plan.info["n_images"] == 21
        pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev))
        outs.append((pot.cpu().numpy(), grad.cpu().numpy()))
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, None, beta=beta)
    for mode, (pm, gm) in zip(("mutual", "one_sided"), outs):
        check(bar, (pm, po), (gm, go), label=f"m0=3 {kernel} {prec} {mode}")
