"""Adjoint / autograd: energy gradients of the periodic potential against
central finite differences of the oracle energy and the oracle's forces,
and a general loss against finite differences of the GPU forward pass."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check, golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


def energy_grads(env, kernel, e1, e2, src, dens, prec, tol, beta=0.0):
    P, torch, dev = env
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, self_exclude=True)
    x = torch.tensor(src, device=dev, requires_grad=True)
    q = torch.tensor(dens, device=dev, requires_grad=True)
    pot = P.periodic_potential(plan, x, q)
    E = 0.5 * (q * pot).sum()
    E.backward()
    return E.item(), x.grad.cpu().numpy(), q.grad.cpu().numpy()


def oracle_energy(kernel, e1, e2, src, dens, beta=0.0):
    pot, _ = oracle.evaluate(kernel, e1, e2, src, dens, None, beta=beta)
    return 0.5 * np.sum(dens * pot)


CELL = ((2.0, 0.0), (0.3, 1.0))


@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 2.0), ("stokes", 0.0)])
def test_energy_gradient_vs_finite_differences_of_oracle(env, kernel, beta):
    rng = np.random.default_rng(3)
    n = 150
    src = W.cell_points(rng, *CELL, n)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    E, dx, dq = energy_grads(env, kernel, *CELL, src, dens, "fp64", 1e-12, beta)
    assert abs(E - oracle_energy(kernel, *CELL, src, dens, beta)) < 1e-10 * abs(E)
    h = 1e-5
    for j in rng.choice(n, 6, replace=False):
        for c in range(2):
            sp = src.copy(); sp[c, j] += h
            sm = src.copy(); sm[c, j] -= h
            fd = (oracle_energy(kernel, *CELL, sp, dens, beta) - oracle_energy(kernel, *CELL, sm, dens, beta)) / (2 * h)
            assert abs(dx[c, j] - fd) < 1e-6 * (abs(fd) + 1e-3), (j, c, dx[c, j], fd)
    # densities: central differences along neutral directions e_j - e_k (per component for Stokes)
    for _ in range(4):
        j, k = rng.choice(n, 2, replace=False)
        comp = rng.integers(2) if kernel == "stokes" else None
        dd = np.zeros_like(dens)
        if comp is None:
            dd[j], dd[k] = 1.0, -1.0
            an = dq[j] - dq[k]
        else:
            dd[comp, j], dd[comp, k] = 1.0, -1.0
            an = dq[comp, j] - dq[comp, k]
        fd = (oracle_energy(kernel, *CELL, src, dens + h * dd, beta)
              - oracle_energy(kernel, *CELL, src, dens - h * dd, beta)) / (2 * h)
        assert abs(an - fd) < 1e-6 * (abs(fd) + 1e-3), (an, fd)


@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
@pytest.mark.parametrize("prec,bar", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_forces_match_oracle(env, kernel, prec, bar):
    rng = np.random.default_rng(5)
    n = 700
    src = W.cell_points(rng, *CELL, n)
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    _, dx, dq = energy_grads(env, kernel, *CELL, src, dens, prec, 1e-10 if prec == "fp64" else 1e-6)
    pot, grad = oracle.evaluate(kernel, *CELL, src, dens, None)
    if kernel == "stokes":
        ref_dx = np.stack([dens[0] * grad[c] + dens[1] * grad[2 + c] for c in range(2)])
        ref_dq = pot - pot.mean(axis=1, keepdims=True)
        dq = dq - dq.mean(axis=1, keepdims=True)
    else:
        ref_dx = dens * grad
        ref_dq = pot - pot.mean()
        dq = dq - dq.mean()
    check(bar, (dx, ref_dx), (dq, ref_dq), label=f"forces {kernel} {prec}")


def test_general_loss_vs_gpu_finite_differences(env):
    # L = sum w_i pot_i^2 for Yukawa (no neutrality needed): adjoint vs FD of the FP64 forward
    P, torch, dev = env
    rng = np.random.default_rng(7)
    n = 300
    e1, e2 = (1.0, 0.0), (0.2, 1.1)
    src = W.cell_points(rng, e1, e2, n)
    q = rng.standard_normal(n)
    w = rng.random(n)
    plan = P.Plan("yukawa", e1, e2, 1e-12, beta=3.0, self_exclude=True)
    x = torch.tensor(src, device=dev, requires_grad=True)
    qt = torch.tensor(q, device=dev, requires_grad=True)
    wt = torch.tensor(w, device=dev)
    loss = (wt * P.periodic_potential(plan, x, qt) ** 2).sum()
    loss.backward()

    def L(s, qq):
        pot, _ = plan(torch.tensor(s, device=dev), torch.tensor(qq, device=dev))
        return float((wt * pot ** 2).sum())
    h = 1e-5

    def fd4(f, base, idx):
        # fourth-order central difference (truncation O(h^4))
        def at(t):
            v = base.copy(); v[idx] += t
            return f(v)
        return (8 * (at(h) - at(-h)) - (at(2 * h) - at(-2 * h))) / (12 * h)
    # rounding of L (~1e-16 |L| per evaluation) divided by h bounds how well
    # a difference quotient can resolve one component: compare against the
    # gradient's own scale
    gx_scale = float(x.grad.abs().max()); gq_scale = float(qt.grad.abs().max())
    for j in (3, 77, 250):
        for c in range(2):
            fd = fd4(lambda s_: L(s_, q), src, (c, j))
            assert abs(x.grad[c, j].item() - fd) < 1e-6 * max(abs(fd), gx_scale), (j, c, fd)
        fd = fd4(lambda q_: L(src, q_), q, j)
        assert abs(qt.grad[j].item() - fd) < 1e-6 * max(abs(fd), gq_scale), (j, fd)


@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
def test_differentiation_workload_n50k(env, kernel):
    # cell e1 = (10, 0), e2 = (0, 1); N = 5e4 uniform sources, neutral N(0,1)
    # densities; forward in mixed precision, adjoint backward. Against stored
    # oracle values: forces dE/dx and dE/dq (on the neutral subspace) at 1024
    # particles, and differences of the energy in x at 64 particles.
    e1, e2, src, dens = W.energy_uniform(kernel)
    ref = golden(f"energy_n50k_{kernel}", src, dens)
    print(f"energy n50k {kernel}", flush=True)
    _, dx, dq = energy_grads(env, kernel, e1, e2, src, dens, "mixed", 1e-6)
    idx = ref["idx"]
    pot, grad = ref["pot"], ref["grad"]
    if kernel == "stokes":
        ref_dx = np.stack([dens[0, idx] * grad[c] + dens[1, idx] * grad[2 + c] for c in range(2)])
    else:
        ref_dx = dens[idx] * grad
    # dE/dq = pot; compare differences between particles (the neutral
    # directions e_j - e_k: a central difference of the quadratic energy along
    # them is exactly pot_j - pot_k)
    sel = np.arange(0, len(idx) - 1, 2)
    dq_s = dq[..., idx]
    check(1e-6, (dx[:, idx], ref_dx), (dq_s[..., sel] - dq_s[..., sel + 1], pot[..., sel] - pot[..., sel + 1]),
          label=f"energy n50k {kernel}")
    # fourth-order difference quotient of the energy in x_j from the stored
    # potentials at x_j + t e_c, t = h, -h, 2h, -2h
    fd_idx, fp, h = ref["fd_idx"], ref["fd_pot"], float(ref["fd_steps"][0])
    fd = np.empty((2, len(fd_idx)))
    for c in range(2):
        up, um, u2p, u2m = fp[c]
        dphi = (8 * (up - um) - (u2p - u2m)) / (12 * h)
        fd[c] = (dens[:, fd_idx] * dphi).sum(axis=0) if kernel == "stokes" else dens[fd_idx] * dphi
    check(1e-6, (dx[:, fd_idx], fd), label=f"energy n50k {kernel} differences")
