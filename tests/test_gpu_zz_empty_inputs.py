"""GPU edge cases of empty inputs through the C ABI: no sources (the field is
exactly zero at every target), no targets, and a self-target plan over no
points (nothing is evaluated; outputs have empty shapes)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


@pytest.mark.parametrize("kernel,e1,e2,beta", [
    ("laplace", (1.1, 0.35), (-0.2, 0.9), 0.0),
    ("yukawa", (2.0, 0.0), (0.4, 1.0), 3.0),
    ("stokes", (100.0, 0.0), (0.0, 1.0), 0.0),      # far field through the NUFFT
])
def test_empty_inputs(env, kernel, e1, e2, beta):
    P, torch, dev = env
    stokes = kernel == "stokes"
    rng = np.random.default_rng(12)
    trg = torch.tensor(W.cell_points(rng, e1, e2, 37), device=dev)
    src = torch.tensor(W.cell_points(rng, e1, e2, 50), device=dev)
    dens = torch.tensor(W.neutral_forces(rng, 50) if stokes else W.neutral_charges(rng, 50), device=dev)
    src0 = torch.zeros((2, 0), dtype=torch.float64, device=dev)
    dens0 = torch.zeros((2, 0) if stokes else (0,), dtype=torch.float64, device=dev)
    for prec in ("fp64", "mixed"):
        print(f"empty inputs: {kernel} {prec}", flush=True)
        plan = P.Plan(kernel, e1, e2, 1e-6, beta=beta, precision=prec)
        pot, grad = plan(src0, dens0, trg)
        torch.cuda.synchronize()
        assert pot.shape == ((2, 37) if stokes else (37,)) and grad.shape == ((4 if stokes else 2), 37)
        assert float(pot.abs().max()) == 0.0 and float(grad.abs().max()) == 0.0
        pot, grad = plan(src, dens, trg[:, :0])
        assert pot.shape[-1] == 0 and grad.shape[-1] == 0
        pot, grad = P.Plan(kernel, e1, e2, 1e-6, beta=beta, precision=prec, self_exclude=True)(src0, dens0)
        torch.cuda.synchronize()
        assert pot.shape[-1] == 0 and grad.shape[-1] == 0
