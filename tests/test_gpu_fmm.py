"""GPU parity of the near part by the interpolation FMM (near_mode "fmm"):
the whole result against the FP64 oracle at the plan's bar, on trees forced
deep enough to have several levels of interaction lists, with ragged and
empty leaf boxes, separate targets, several density vectors and points on
the cell's edges; and the FMM against the direct near sum on the same plan
at larger N, where the tree comes from the cost model."""
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
    "shear04": ((1.0, 0.0), (0.4, 1.0)),
    "long_shear": ((3.0, 0.0), (1.2, 1.0)),
    "a10": ((10.0, 0.0), (0.0, 1.0)),
}
BAR = {"fp64": (1e-10, 1e-10), "mixed": (1e-6, 1e-6)}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


def run(env, kernel, e1, e2, src, dens, trg, beta, prec, tol=None, mode="fmm", level=0, n_dens=1):
    P, torch, dev = env
    tol = BAR[prec][0] if tol is None else tol
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, self_exclude=trg is None, near_mode=mode,
                  n_dens=n_dens)
    if level:
        plan.set_tuning(fmm_level=level)
    t = None if trg is None else torch.tensor(trg, device=dev)
    pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev), t)
    torch.cuda.synchronize()
    return pot.cpu().numpy(), grad.cpu().numpy(), plan


def inputs(kernel, e1, e2, ns, nt, seed, nd=1):
    rng = np.random.default_rng(seed)
    src = W.cell_points(rng, e1, e2, ns)
    trg = W.cell_points(rng, e1, e2, nt)
    dens = W.neutral_forces(rng, ns, nd) if kernel == "stokes" else W.neutral_charges(rng, ns, nd)
    return src, dens, trg


@pytest.mark.parametrize("cell", list(CELLS))
@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 6.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("self_trg", [True, False])
def test_fmm_matches_oracle(env, cell, kernel, beta, prec, self_trg):
    # 1500 sources (700 separate targets); leaf level 3 (64 k1 k2 leaves of
    # about 23 points): interaction lists on levels 1..3, plus level 0 for
    # the cells with several top boxes
    e1, e2 = CELLS[cell]
    src, dens, trg = inputs(kernel, e1, e2, 1500, 700, seed=31)
    trg = None if self_trg else trg
    print(f"case fmm {kernel} {cell} {prec} self={self_trg}", flush=True)
    pot, grad, plan = run(env, kernel, e1, e2, src, dens, trg, beta, prec, level=3)
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, trg, beta=beta)
    check(BAR[prec][1], (pot, po), (grad, go), label=f"fmm {kernel} {cell} {prec} self={self_trg}")


@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 10.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fmm_every_leaf_level_matches_the_direct_sum(env, kernel, beta, prec):
    # N = 20000 in the sheared cell: leaf levels 1 (a few large leaves) to 6
    # (4096 leaves of about 5 points, some empty) against the direct near
    # sum of the same plan; the cost model's own level too
    e1, e2 = CELLS["sheared"]
    src, dens, _ = inputs(kernel, e1, e2, 20000, 1, seed=32)
    pd, gd, _ = run(env, kernel, e1, e2, src, dens, None, beta, "fp64", tol=BAR[prec][0], mode="one_sided")
    for level in (0, 1, 2, 4, 6):
        print(f"case levels {kernel} {prec} L={level}", flush=True)
        pf, gf, _ = run(env, kernel, e1, e2, src, dens, None, beta, prec, level=level)
        check(BAR[prec][1], (pf, pd), (gf, gd), label=f"fmm levels {kernel} {prec} L={level}")


@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 10.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fmm_clustered_points_leave_boxes_empty(env, kernel, beta, prec):
    # 20 Gaussian blobs (sigma 0.01) in the square cell, N = 6000, leaf level
    # 5: most leaves and many boxes of every level hold no source; oracle at
    # 400 sampled sources
    e1, e2 = CELLS["square"]
    rng = np.random.default_rng(33)
    c = rng.uniform(-0.5, 0.5, (2, 20))
    src = np.repeat(c, 300, axis=1) + 0.01 * rng.standard_normal((2, 6000))
    src -= np.rint(src)
    dens = W.neutral_forces(rng, 6000) if kernel == "stokes" else W.neutral_charges(rng, 6000)
    print(f"case blobs {kernel} {prec}", flush=True)
    pot, grad, _ = run(env, kernel, e1, e2, src, dens, None, beta, prec, level=5)
    idx = W.sample_indices(6000, 400, seed=4)
    po, go = oracle.evaluate(kernel, e1, e2, src, dens, src[:, idx], beta=beta, self_idx=idx)
    check(BAR[prec][1], (pot[..., idx], po), (grad[:, idx], go), label=f"fmm blobs {kernel} {prec}")


@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
def test_fmm_points_on_the_cell_edges_and_tiny_sizes(env, kernel):
    # sources on the edges and a corner of the cell (lattice coordinates
    # +-1/2: the first and last leaf boxes, and the images' boxes next to
    # them; an edge point and its copy across the cell are distinct points
    # only when their other coordinates differ, as here); then 2, 3 and 7
    # points
    e1, e2 = CELLS["shear04"]
    rng = np.random.default_rng(34)
    u = rng.uniform(-0.5, 0.5, (2, 900))
    u[0, :100] = -0.5; u[0, 100:200] = 0.5; u[1, 200:300] = -0.5; u[1, 300:400] = 0.5
    u[:, 400] = (-0.5, -0.5)   # one corner: the other three are its periodic copies
    L = np.array([e1, e2]).T
    src = L @ u
    dens = W.neutral_forces(rng, 900) if kernel == "stokes" else W.neutral_charges(rng, 900)
    for prec in ("fp64", "mixed"):
        print(f"case edges {kernel} {prec}", flush=True)
        pot, grad, _ = run(env, kernel, e1, e2, src, dens, None, 0.0, prec, level=3)
        po, go = oracle.evaluate(kernel, e1, e2, src, dens, None)
        check(BAR[prec][1], (pot, po), (grad, go), label=f"fmm edges {kernel} {prec}")
    for n in (2, 3, 7):
        s, d, _ = inputs(kernel, e1, e2, n, 1, seed=n)
        for prec in ("fp64", "mixed"):
            pot, grad, _ = run(env, kernel, e1, e2, s, d, None, 0.0, prec, level=2)
            po, go = oracle.evaluate(kernel, e1, e2, s, d, None)
            check(BAR[prec][1], (pot, po), (grad, go), label=f"fmm tiny {kernel} n={n} {prec}")


@pytest.mark.parametrize("kernel", ["laplace", "yukawa", "stokes"])
def test_fmm_multiple_density_vectors(env, kernel):
    e1, e2 = CELLS["hexagonal"]
    src, dens, trg = inputs(kernel, e1, e2, 2000, 300, seed=35, nd=3)
    print(f"case nd=3 {kernel}", flush=True)
    pot, grad, _ = run(env, kernel, e1, e2, src, dens, trg, 6.0, "mixed", level=3, n_dens=3)
    for v in range(3):
        po, go = oracle.evaluate(kernel, e1, e2, src, dens[v], trg, beta=6.0)
        check(1e-6, (pot[v], po), (grad[v], go), label=f"fmm {kernel} nd=3 v={v}")


@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 10.0), ("stokes", 0.0)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_symmetric_leaves_match_one_sided_leaves(env, kernel, beta, prec):
    # targets = sources: each forward pair of leaf boxes evaluated once for
    # both against the same plan and tree with one-sided leaves; equal up to
    # the order of the sums (FP64) and the grouping of the FP32 partial sums
    # (mixed); three density vectors. First the square cell with 100 points:
    # the cost model's tree is the single leaf of the 1 x 1 top grid, which is
    # its own forward neighbour four times (shifted); its 3 x 3 super-grid
    # has no interaction list, so the FMM near part is the direct near sum.
    # Then the sheared cell at leaf levels 1 (thousands of points per box:
    # the stream is visited once per chunk of a block's points), 2, 5 and 7
    # (about one point per box, most neighbours empty).
    P, torch, dev = env
    tol = 2e-14 if prec == "fp64" else 3e-7

    def run3(cell, src, dens, mode, level=0, leaves=0):
        e1, e2 = CELLS[cell]
        plan = P.Plan(kernel, e1, e2, BAR[prec][0], beta=beta, precision=prec, self_exclude=True,
                      near_mode=mode, n_dens=3)
        if mode == "fmm":
            plan.set_tuning(fmm_level=level, fmm_leaves=leaves)
            assert plan.fmm_symmetric == (leaves == 2)
        tree = plan.fmm_tree(src.shape[1])
        pot, grad = plan(torch.tensor(src, device=dev), torch.tensor(dens, device=dev), None)
        torch.cuda.synchronize()
        return pot.cpu().numpy(), grad.cpu().numpy(), tree

    def same(a, b, label, bar=None):
        for v in range(3):
            ep, eg = rel(a[0][v], b[0][v]), rel(a[1][v], b[1][v])
            assert ep < (bar or tol) and eg < (bar or tol), (label, v, ep, eg)

    e1, e2 = CELLS["square"]
    src, dens, _ = inputs(kernel, e1, e2, 100, 1, seed=37, nd=3)
    print(f"case symmetric leaves {kernel} {prec} square n=100", flush=True)
    sym = run3("square", src, dens, "fmm", 0, 2)
    assert sym[2]["level"] == 0 and sym[2]["k1"] * sym[2]["k2"] == 1
    # (the direct sum drops screened pairs beyond its cutoff and groups its
    # FP32 sums its own way: agreement to a tenth of the plan's bar in FP64,
    # to the bar in mixed precision, where each path is within about 1e-7)
    same(sym, run3("square", src, dens, "one_sided"), "square L=0",
         BAR[prec][0] if prec == "mixed" else 0.1 * BAR[prec][0])
    e1, e2 = CELLS["sheared"]
    src, dens, _ = inputs(kernel, e1, e2, 20000, 1, seed=38, nd=3)
    for level in (1, 2, 5, 7):
        print(f"case symmetric leaves {kernel} {prec} sheared n=20000 L={level}", flush=True)
        sym = run3("sheared", src, dens, "fmm", level, 2)
        one = run3("sheared", src, dens, "fmm", level, 1)
        assert sym[2] == one[2] and sym[2]["level"] == level
        same(sym, one, f"sheared L={level}")


def test_fmm_repeated_evaluations_are_identical(env):
    # no atomics: the FMM near part is deterministic
    e1, e2 = CELLS["sheared"]
    src, dens, _ = inputs("stokes", e1, e2, 30000, 1, seed=36)
    a = run(env, "stokes", e1, e2, src, dens, None, 0.0, "mixed")
    b = run(env, "stokes", e1, e2, src, dens, None, 0.0, "mixed")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("kernel,beta", [("yukawa", 10.0), ("stokes", 0.0)])
def test_auto_takes_the_fmm_at_full_size(env, kernel, beta):
    # square cell, N = 2e5: AUTO evaluates the near part by the FMM (the
    # same numbers as near_mode "fmm"), within the bar of the stored oracle
    # values, for both precisions
    e1, e2, src, dens = W.square_uniform(kernel)
    ref = golden(f"square_n200k_{kernel}", src, dens)
    idx = ref["idx"]
    for prec in ("mixed", "fp64"):
        print(f"case auto full {kernel} {prec}", flush=True)
        pa, ga, plan = run(env, kernel, e1, e2, src, dens, None, beta, prec, tol=1e-6, mode="auto")
        pf, gf, _ = run(env, kernel, e1, e2, src, dens, None, beta, prec, tol=1e-6, mode="fmm")
        assert np.array_equal(pa, pf) and np.array_equal(ga, gf)
        check(1e-6, (pa[..., idx], ref["pot"]), (ga[:, idx], ref["grad"]), label=f"auto fmm n200k {kernel} {prec}")
