"""Autotuner and tunings: every tuning keeps the plan's accuracy (the NUFFT
doubled grid with its narrower kernel included), the autotuner leaves a
valid result and a plan that reproduces it, and the batched autotuner
likewise."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-10), ("mixed", 1e-6, 1e-6)])
def test_nufft_doubled_grid_keeps_accuracy(env, kernel, prec, tol, bar):
    P, torch, dev = env
    e1, e2 = (100.0, 0.0), (0.0, 1.0)
    rng = np.random.default_rng(8)
    n = 3000
    src = W.blob_points(rng, e1, e2, n)
    trg = W.cell_points(rng, e1, e2, 500)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, trg)
    plan = P.Plan(kernel, e1, e2, tol, precision=prec, far_mode="nufft")
    nf0 = plan.info["nufft_nf"]
    plan.set_tuning(nufft_grid=1)
    assert plan.info["nufft_nf"] == 2 * nf0
    print(f"case doubled grid {kernel} {prec}", flush=True)
    pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev), torch.tensor(trg, device=dev))
    check(bar, (pot.cpu().numpy(), po), (grad.cpu().numpy(), go), label=f"doubled grid {kernel} {prec}")


@pytest.mark.parametrize("cell,kernel,beta,far,near,n", [
    (((1.0, 0.0), (0.0, 1.0)), "yukawa", 10.0, "auto", "auto", 20000),
    (((100.0, 0.0), (0.0, 1.0)), "laplace", 0.0, "nufft", "auto", 20000),
    (((1.0, 0.0), (0.3, 1.0)), "yukawa", 10.0, "auto", "fmm", 100000)])
def test_autotune_result_and_reuse(env, cell, kernel, beta, far, near, n):
    # the FMM plan: the candidates are the leaf levels next to the cost
    # model's and the other leaf form (symmetric / one-sided)
    P, torch, dev = env
    e1, e2 = cell
    rng = np.random.default_rng(2)
    src = W.blob_points(rng, e1, e2, n) if far == "nufft" else W.cell_points(rng, e1, e2, n)
    q = W.neutral_charges(rng, n)
    plan = P.Plan(kernel, e1, e2, 1e-6, beta=beta, precision="mixed", far_mode=far, self_exclude=True,
                  near_mode=near)
    ds, dq = torch.tensor(src, device=dev), torch.tensor(q, device=dev)
    print(f"case autotune {kernel} {far} {near}", flush=True)
    rep, pot, grad = P.pfmm_autotune(plan, ds, dq)
    assert rep["n_tried"] >= 3 and rep["best_ms"] > 0
    assert rep["best_ms"] <= 1.10 * rep["default_ms"]
    assert rep["near_blocks"] in (4096, 8192, 16384, 0)
    assert 0 <= rep["fmm_level"] <= 11 and (near == "fmm" or rep["fmm_level"] == 0)
    assert rep["fmm_leaves"] in (0, 1, 2) and (near == "fmm" or rep["fmm_leaves"] == 0)
    if near == "fmm":
        assert rep["n_tried"] >= 4   # the reference, two leaf levels, the other leaf form
    pot = pot[0].cpu().numpy(); grad = grad[0].cpu().numpy()
    p2, g2 = plan(ds, dq)
    assert rel(p2.cpu().numpy(), pot) < 1e-12 and rel(g2.cpu().numpy(), grad) < 1e-12
    idx = np.sort(rng.choice(n, 12, replace=False))
    po, go = oracle.evaluate(kernel, e1, e2, src, q, src[:, idx], beta=beta, tol=1e-10, self_idx=idx)
    check(1e-6, (pot[idx], po), (grad[:, idx], go), label=f"autotune {kernel} {far}")


def test_batch_autotune(env):
    P, torch, dev = env
    from test_gpu_batch import small_cells
    cells = small_cells(13)
    nd = 4
    plans, srcs, dens, offs = [], [], [], [0]
    for c in cells:
        beta = 10.0 if c["kernel"] == "yukawa" else 0.0
        plans.append(P.Plan(c["kernel"], c["e1"], c["e2"], 1e-6, beta=beta, precision="mixed", n_dens=nd,
                            self_exclude=True))
        srcs.append(W.cell_points(c["rng"], c["e1"], c["e2"], c["n"]))
        dens.append(W.neutral_charges(c["rng"], c["n"], nd).reshape(nd, c["n"]))
        offs.append(offs[-1] + c["n"])
    batch = P.Batch(plans, offs, use_graph=True)
    ds = torch.tensor(np.concatenate(srcs, 1), device=dev); dq = torch.tensor(np.concatenate(dens, 1), device=dev)
    print("case batch autotune", flush=True)
    rep, pot, grad = batch.autotune(ds, dq)
    assert rep["n_tried"] >= 2
    p2, g2 = batch(ds, dq)                 # graph captured with the chosen task shape
    assert torch.allclose(p2, pot, rtol=1e-12, atol=1e-12 * float(pot.abs().max()))
    pot = pot.cpu().numpy(); grad = grad.cpu().numpy()
    for c, cell in enumerate(cells):
        beta = 10.0 if cell["kernel"] == "yukawa" else 0.0
        po, go = oracle.evaluate(cell["kernel"], cell["e1"], cell["e2"], srcs[c], dens[c][nd - 1], None, beta=beta)
        sl = slice(offs[c], offs[c + 1])
        check(1e-6, (pot[nd - 1, sl], po), (grad[nd - 1, :, sl], go), label=f"batch autotune cell {c}")
