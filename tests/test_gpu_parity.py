"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars per output (pot and grad separately), see tests/parity.py: relative l2
error below the bar and largest elementwise error below 10x the bar relative
to the rms of the reference, with
  FP64 mode:  bar = tol = 1e-10
  mixed mode: bar = tol = 1e-6
Sizes span several near-field tiles (256 targets/sources) plus a ragged tail.
The full-size workloads compare with oracle values stored under
tests/golden/ (written by tests/golden/make_oracle_samples.py).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check, golden, rel

pytestmark = pytest.mark.gpu

CELLS = {
    "square": ((1.0, 0.0), (0.0, 1.0)),
    "sheared": ((2.0, 0.0), (0.4, 1.0)),
    "rotated_general": ((1.1, 0.35), (-0.2, 0.9)),
    "hexagonal": ((1.0, 0.0), (0.5, np.sqrt(3) / 2)),
    # |xi| > d/4 after reduction: west/east waves along e2-perp, 9 near images
    "shear04": ((1.0, 0.0), (0.4, 1.0)),
    "long_shear": ((3.0, 0.0), (1.2, 1.0)),
}
BAR = {"fp64": (1e-10, 1e-10), "mixed": (1e-6, 1e-6)}   # (tol requested, error bar)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


def run(env, kernel, e1, e2, src, dens, trg, beta=0.0, prec="fp64", tol=None, **kw):
    P, torch, dev = env
    tol = BAR[prec][0] if tol is None else tol
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, self_exclude=trg is None, **kw)
    t = None if trg is None else torch.tensor(trg, device=dev)
    pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev), t)
    torch.cuda.synchronize()
    return pot.cpu().numpy(), grad.cpu().numpy(), plan


def inputs(kernel, e1, e2, ns, nt, seed):
    rng = np.random.default_rng(seed)
    src = W.cell_points(rng, e1, e2, ns)
    trg = W.cell_points(rng, e1, e2, nt)
    dens = W.neutral_forces(rng, ns) if kernel == "stokes" else W.neutral_charges(rng, ns)
    return src, dens, trg


@pytest.mark.parametrize("cell", list(CELLS))
@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 3.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("self_trg", [True, False])
def test_parity_small(env, cell, kernel, beta, prec, self_trg):
    e1, e2 = CELLS[cell]
    src, dens, trg = inputs(kernel, e1, e2, 700, 300, seed=11)
    trg = None if self_trg else trg
    print(f"case {kernel} {cell} {prec} self={self_trg}", flush=True)
    pot, grad, _ = run(env, kernel, e1, e2, src, dens, trg, beta, prec)
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, trg, beta=beta)
    check(BAR[prec][1], (pot, po), (grad, go), label=f"{kernel} {cell} {prec} self={self_trg}")


def test_config1_laplace_square_n1000(env):
    # Plain FP64, square cell, N = 1000 uniform, neutral N(0,1) charges,
    # targets = sources, tol 1e-10, seed 0.
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    rng = np.random.default_rng(0)
    src = W.cell_points(rng, e1, e2, 1000)
    q = W.neutral_charges(rng, 1000)
    pot, grad, _ = run(env, "laplace", e1, e2, src, q, None, prec="fp64", tol=1e-10)
    po, go = oracle.laplace(e1, e2, src, q, None)
    check(1e-10, (pot, po), (grad, go), label="config 1")


@pytest.mark.parametrize("kernel", ["laplace", "stokes", "yukawa"])
@pytest.mark.parametrize("nd", [3, 4, 6])
def test_multiple_density_vectors(env, kernel, nd):
    e1, e2 = CELLS["sheared"]
    rng = np.random.default_rng(5)
    src = W.cell_points(rng, e1, e2, 500)
    dens = W.neutral_forces(rng, 500, nd) if kernel == "stokes" else W.neutral_charges(rng, 500, nd)
    pot, grad, _ = run(env, kernel, e1, e2, src, dens, None, beta=2.0, prec="mixed", n_dens=nd)
    for v in range(nd):
        po, go = oracle.evaluate(kernel, e1, e2, src, dens[v], None, beta=2.0)
        check(1e-6, (pot[v], po), (grad[v], go), label=f"{kernel} nd={nd} v={v}")


@pytest.mark.parametrize("ns,nt", [(2, 1), (3, 257), (255, 7), (256, 256), (513, 1)])
def test_ragged_and_tiny_sizes(env, ns, nt):
    e1, e2 = CELLS["rotated_general"]
    src, q, trg = inputs("laplace", e1, e2, ns, nt, seed=ns + nt)
    for prec in ("fp64", "mixed"):
        pot, grad, _ = run(env, "laplace", e1, e2, src, q, trg, prec=prec)
        po, go = oracle.laplace(e1, e2, src, q, trg)
        check(BAR[prec][1], (pot, po), (grad, go), label=f"ragged {ns} {nt} {prec}")


def test_points_outside_the_cell_are_wrapped(env):
    # the sum is periodic: moving sources and targets by lattice vectors
    # must not change anything
    e1, e2 = CELLS["sheared"]
    src, f, trg = inputs("stokes", e1, e2, 400, 200, seed=3)
    rng = np.random.default_rng(4)
    L = np.array([e1, e2]).T
    src_m = src + L @ rng.integers(-3, 4, (2, 400))
    trg_m = trg + L @ rng.integers(-3, 4, (2, 200))
    p1, g1, _ = run(env, "stokes", e1, e2, src, f, trg)
    p2, g2, _ = run(env, "stokes", e1, e2, src_m, f, trg_m)
    assert rel(p2, p1) < 1e-12 and rel(g2, g1) < 1e-12


PERIODIC_CELLS = {"sheared3": ((3.0, 0.0), (0.5, 1.0)), "a100": ((100.0, 0.0), (0.0, 1.0))}


@pytest.mark.parametrize("cell", list(PERIODIC_CELLS))
@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 2.0), ("stokes", 0.0)])
def test_periodicity_error_on_cell_boundary(env, cell, kernel, beta):
    # the paper's check (Sec. 7): equispaced targets on opposite sides of the
    # cell must see the same potential and gradient; the error is the l2
    # difference between the two sides relative to the field's l2 norm, for
    # the potential (Stokes: velocity) and the gradient separately
    e1, e2 = (np.array(v) for v in PERIODIC_CELLS[cell])
    src, dens, _ = inputs(kernel, e1, e2, 600, 1, seed=8)
    n = 101
    s = np.linspace(-0.5, 0.5, n)
    left = -0.5 * e1[:, None] + np.outer(e2, s)
    bottom = -0.5 * e2[:, None] + np.outer(e1, s)
    trg = np.concatenate([left, left + e1[:, None], bottom, bottom + e2[:, None]], axis=1)
    pot, grad, _ = run(env, kernel, e1, e2, src, dens, trg, beta=beta)
    for out in (pot, grad):
        f = out.reshape(-1, 4 * n)
        err = (np.linalg.norm(f[:, n:2 * n] - f[:, :n]) + np.linalg.norm(f[:, 3 * n:] - f[:, 2 * n:3 * n])) \
            / np.linalg.norm(f)
        assert err < 1e-11, (cell, kernel, err)


def test_translation_invariance(env):
    e1, e2 = CELLS["square"]
    src, q, trg = inputs("yukawa", e1, e2, 500, 300, seed=9)
    shift = np.array([[0.3217], [-0.1409]])
    p1, g1, _ = run(env, "yukawa", e1, e2, src, q, trg, beta=5.0)
    p2, g2, _ = run(env, "yukawa", e1, e2, src + shift, q, trg + shift, beta=5.0)
    assert rel(p2, p1) < 1e-12 and rel(g2, g1) < 1e-12


def test_neutrality_check_and_workspace_errors(env):
    P, torch, dev = env
    e1, e2 = CELLS["square"]
    src, q, trg = inputs("laplace", e1, e2, 64, 8, seed=2)
    q = q + 0.1
    plan = P.Plan("laplace", e1, e2, 1e-6, check_neutral=True)
    with pytest.raises(P.PfmmError) as e:
        plan(torch.tensor(src, device=dev), torch.tensor(q, device=dev), torch.tensor(trg, device=dev))
    assert e.value.code == -6
    plan = P.Plan("laplace", e1, e2, 1e-6)
    small = torch.empty(512, dtype=torch.uint8, device=dev)
    with pytest.raises(P.PfmmError) as e:
        plan(torch.tensor(src, device=dev), torch.tensor(q, device=dev), torch.tensor(trg, device=dev),
             workspace=small)
    assert e.value.code == -4


# --- full-size configuration (N = 200000) ----------------------------------

@pytest.mark.parametrize("kernel,beta", [("yukawa", 10.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_square_n200k_sampled(env, kernel, beta, prec):
    # Square cell, N = 2e5 uniform sources, neutral N(0,1) densities (Stokes:
    # zero net force), potential + gradient at all sources, tol 1e-6; checked
    # at 512 sampled sources against stored oracle values
    e1, e2, src, dens = W.square_uniform(kernel)
    ref = golden(f"square_n200k_{kernel}", src, dens)
    print(f"full-size {kernel} {prec}", flush=True)
    pot, grad, _ = run(env, kernel, e1, e2, src, dens, None, beta, prec, tol=1e-6)
    idx = ref["idx"]
    check(1e-6, (pot[..., idx], ref["pot"]), (grad[:, idx], ref["grad"]), label=f"square n200k {kernel} {prec}")


@pytest.mark.parametrize("kernel,beta", [("yukawa", 10.0), ("stokes", 0.0)])
def test_full_size_mixed_against_fp64_every_output(env, kernel, beta):
    # the same workload in both precisions: every output of the mixed path
    # (tol 1e-6) against the FP64 path at tol 1e-10
    e1, e2, src, dens = W.square_uniform(kernel)
    print(f"full-size mixed vs fp64 {kernel}", flush=True)
    pm, gm, _ = run(env, kernel, e1, e2, src, dens, None, beta, "mixed", tol=1e-6)
    pd, gd, _ = run(env, kernel, e1, e2, src, dens, None, beta, "fp64", tol=1e-10)
    check(1e-6, (pm, pd), (gm, gd), label=f"mixed vs fp64 n200k {kernel}")
