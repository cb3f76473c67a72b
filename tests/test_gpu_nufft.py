"""NUFFT-accelerated south/north factors on high-aspect cells: parity with
the FP64 oracle and with the direct plane-wave path on the same inputs.

Inputs follow the clustered high-aspect workload: sources in 50 Gaussian
blobs (sigma = 0.02 |e2|) wrapped into the cell, neutral densities."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

HIGH = {"A100": ((100.0, 0.0), (0.0, 1.0)), "sheared20": ((20.0, 0.0), (3.0, 1.0))}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


def rel(a, b):
    return np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel())


def run(env, kernel, e1, e2, src, dens, trg, far, prec, tol, beta=0.0, **kw):
    P, torch, dev = env
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, far_mode=far, self_exclude=trg is None, **kw)
    t = None if trg is None else torch.tensor(trg, device=dev)
    pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev), t)
    torch.cuda.synchronize()
    return pot.cpu().numpy(), grad.cpu().numpy(), plan.info


def blob_inputs(kernel, e1, e2, ns, nt, seed):
    rng = np.random.default_rng(seed)
    src = W.blob_points(rng, e1, e2, ns)
    trg = W.cell_points(rng, e1, e2, nt)
    dens = W.neutral_forces(rng, ns) if kernel == "stokes" else W.neutral_charges(rng, ns)
    return src, dens, trg


@pytest.mark.parametrize("cell", list(HIGH))
@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("stokes", 0.0), ("yukawa", 0.5)])
@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-10), ("mixed", 1e-6, 1e-6)])
def test_nufft_matches_oracle_and_direct(env, cell, kernel, beta, prec, tol, bar):
    e1, e2 = HIGH[cell]
    src, dens, trg = blob_inputs(kernel, e1, e2, 3000, 700, seed=21)
    print(f"case nufft {kernel} {cell} {prec}", flush=True)
    pn, gn, info = run(env, kernel, e1, e2, src, dens, trg, "nufft", prec, tol, beta)
    assert info["far_mode_used"] == 2
    pd, gd, _ = run(env, kernel, e1, e2, src, dens, trg, "direct", prec, tol, beta)
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, trg, beta=beta)
    assert rel(pn, po) < bar and rel(gn, go) < bar, (rel(pn, po), rel(gn, go))
    # the two far paths differ only by NUFFT/interpolation error (<< bar)
    assert rel(pn, pd) < bar and rel(gn, gd) < bar


def test_nufft_self_targets_and_several_densities(env):
    e1, e2 = HIGH["sheared20"]
    rng = np.random.default_rng(4)
    src = W.blob_points(rng, e1, e2, 2000)
    q = W.neutral_charges(rng, 2000, 3)
    P, torch, dev = env
    plan = P.Plan("laplace", e1, e2, 1e-6, precision="mixed", far_mode="nufft", self_exclude=True, n_dens=3)
    pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(q, device=dev))
    pot = pot.cpu().numpy(); grad = grad.cpu().numpy()
    for v in range(3):
        po, go = oracle.laplace(e1, e2, src, q[v], None)
        assert rel(pot[v], po) < 1e-6 and rel(grad[v], go) < 1e-6


def test_auto_mode_picks_nufft_at_high_aspect(env):
    P, torch, dev = env
    assert P.Plan("laplace", (100.0, 0.0), (0.0, 1.0), 1e-6).info["far_mode_used"] == 2
    assert P.Plan("laplace", (1.0, 0.0), (0.0, 1.0), 1e-6).info["far_mode_used"] == 1


@pytest.mark.parametrize("cell", list(HIGH))
@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
def test_full_size_blobs_n200k_sampled(env, cell, kernel):
    # N = 2e5 sources in 50 Gaussian blobs (sigma = 0.02 |e2|), mixed FP32/FP64,
    # far part via NUFFT, tol 1e-6; potential + gradient at all sources.
    e1, e2 = HIGH[cell]
    n = 200_000
    rng = np.random.default_rng(0)
    src = W.blob_points(rng, e1, e2, n)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    print(f"full-size blobs {kernel} {cell}", flush=True)
    pot, grad, info = run(env, kernel, e1, e2, src, dens, None, "nufft", "mixed", 1e-6)
    assert info["far_mode_used"] == 2
    idx = np.sort(np.random.default_rng(1).choice(n, 16, replace=False))
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, src[:, idx], tol=1e-10, self_idx=idx)
    assert rel(pot[..., idx], po) < 1e-6 and rel(grad[:, idx], go) < 1e-6
