"""pfmm_eval_static (no allocation, fixed device workspace) against pfmm_eval.

Two calls in a row on one plan, the second with fewer points, each compared
with pfmm_eval on the same inputs (same kernels, so the results agree to
FP64 rounding of the atomic sums) and with the oracle at the plan's bar.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_01083_amd as P
    return P, torch, torch.device("cuda:0")


def maxrms(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.sqrt(np.mean(b ** 2)))


def rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


CASES = [
    # kernel, beta, e1, e2, precision, self targets, far mode, sizes
    ("laplace", 0.0, (1.0, 0.0), (0.0, 1.0), "mixed", True, "auto", (3000, 1100)),
    ("yukawa", 10.0, (1.0, 0.0), (0.3, 1.0), "fp64", False, "auto", (2500, 700)),
    ("stokes", 0.0, (100.0, 0.0), (0.0, 1.0), "mixed", True, "nufft", (4000, 1500)),
    ("stokes", 0.0, (1.0, 0.0), (0.4, 1.0), "mixed", False, "fmm", (6000, 2500)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] + "-" + c[4] + "-" + c[6] for c in CASES])
def test_static_matches_eval_twice(env, case):
    P, torch, dev = env
    kernel, beta, e1, e2, prec, self_trg, far, sizes = case
    tol = 1e-10 if prec == "fp64" else 1e-6
    near = "fmm" if far == "fmm" else "auto"   # the last case: near part by the FMM
    far = "auto" if far == "fmm" else far
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, precision=prec, self_exclude=self_trg, far_mode=far,
                  near_mode=near)
    P.pfmm_plan_upload(plan)
    for call, n in enumerate(sizes):
        print(f"static {kernel} {prec} call {call} n={n}", flush=True)
        rng = np.random.default_rng(100 + call)
        src = W.cell_points(rng, e1, e2, n)
        dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
        trg = None if self_trg else W.cell_points(rng, e1, e2, n // 2 + 3)
        s_t = torch.tensor(src, device=dev)
        d_t = torch.tensor(dens, device=dev)
        t_t = None if trg is None else torch.tensor(trg, device=dev)
        p_ref, g_ref = plan(s_t, d_t, t_t)
        p_st, g_st = P.pfmm_eval_static(plan, s_t, d_t, t_t)
        torch.cuda.synchronize()
        p_ref = p_ref.cpu().numpy(); g_ref = g_ref.cpu().numpy()
        p_st = p_st.cpu().numpy().reshape(p_ref.shape); g_st = g_st.cpu().numpy().reshape(g_ref.shape)
        assert maxrms(p_st, p_ref) < 1e-12 and maxrms(g_st, g_ref) < 1e-12, (maxrms(p_st, p_ref),
                                                                               maxrms(g_st, g_ref))
        po, go = oracle.evaluate(kernel, e1, e2, src, dens, trg, beta=beta)
        assert rel(p_st, po) < tol and rel(g_st, go) < tol, (rel(p_st, po), rel(g_st, go))


def test_static_argument_errors(env):
    P, torch, dev = env
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    rng = np.random.default_rng(7)
    src = torch.tensor(W.cell_points(rng, e1, e2, 64), device=dev)
    q = torch.tensor(W.neutral_charges(rng, 64), device=dev)
    plan = P.Plan("laplace", e1, e2, 1e-6, self_exclude=True)
    # tables not uploaded: the entry point does not upload them itself
    with pytest.raises(P.PfmmError) as e:
        P.pfmm_eval_static(plan, src, q)
    assert e.value.code == -1
    P.pfmm_plan_upload(plan)
    # sizes whose workspace exceeds the fixed array
    from paper_2111_01083_amd import _lib as L
    big = 1
    while P.pfmm_workspace_bytes(plan, big, big) <= L.PFMM_STATIC_WORKSPACE_BYTES:
        big *= 2
    rc = L.load().pfmm_eval_static(plan.handle, big, src.data_ptr(), q.data_ptr(), big, None,
                                   None, None, None)
    assert rc == -4
