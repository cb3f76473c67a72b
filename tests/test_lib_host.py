"""Host-side checks of libpfmm that need no GPU: the library loads and
exports every function include/pfmm.h declares, and the planner's
canonical lattice, truncation sizes, west/east quadrature and argument
validation are right."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.special as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    from paper_2111_01083_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2111_01083_amd import build
        build.build()
    import paper_2111_01083_amd as P
    return P


def test_library_exports_every_declared_function(P):
    from paper_2111_01083_amd import _lib
    header = open(os.path.join(ROOT, "include", "pfmm.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = sorted(set(re.findall(r"\b(pfmm_[a-z_0-9]+)\s*\(", header)))
    assert declared == sorted(_lib.EXPORTS)
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def test_header_is_c99_and_the_abi_works_from_c(P, tmp_path):
    # a plain C program built against include/pfmm.h with warnings as errors,
    # linked with libpfmm, runs the host-only entry points; the struct sizes it
    # prints must match the Python binding's ctypes layouts
    import shutil
    import subprocess
    from paper_2111_01083_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    libdir = os.path.dirname(_lib.LIB_PATH)
    exe = str(tmp_path / "c_abi_check")
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_check.c"),
                    "-o", exe, "-L", libdir, "-lpfmm", "-Wl,-rpath," + libdir], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=60).stdout.split("\n")
    assert out[-2] == "ok", out
    sizes = dict(line.split()[1:] for line in out if line.startswith("sizeof "))
    for name, ct in (("pfmm_opts", _lib.pfmm_opts), ("pfmm_plan_info_t", _lib.pfmm_plan_info_t),
                     ("pfmm_tuning_t", _lib.pfmm_tuning_t), ("pfmm_tune_report_t", _lib.pfmm_tune_report_t)):
        assert int(sizes[name]) == ctypes.sizeof(ct), name


def test_binding_fails_loudly_without_the_library(tmp_path):
    # with libpfmm.so absent the binding raises; there is no other path
    import subprocess
    import sys
    code = ("import paper_2111_01083_amd._lib as L; L.LIB_PATH = %r\n"
            "import paper_2111_01083_amd as P\n"
            "try:\n    P.Plan('laplace', (1.0, 0.0), (0.0, 1.0), 1e-6)\n"
            "except RuntimeError as e:\n    print('raised:', e)\n") % str(tmp_path / "missing.so")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert res.returncode == 0 and "raised:" in res.stdout and "no fallback" in res.stdout, res.stdout + res.stderr


def test_binding_rejects_host_tensors_before_calling_the_library(P):
    import torch
    plan = P.Plan("laplace", (1.0, 0.0), (0.0, 1.0), 1e-6, self_exclude=True)
    src = torch.zeros((2, 4), dtype=torch.float64)
    q = torch.zeros(4, dtype=torch.float64)
    with pytest.raises(TypeError):
        plan(src, q)


def test_canonical_lattice_of_rotated_unreduced_basis(P):
    # lattice of (3, 0), (0.6, 1), given rotated and as an unreduced basis
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    a, b = R @ np.array([3.0, 0.0]), R @ np.array([0.6, 1.0])
    plan = P.Plan("laplace", a + 2 * b, b, 1e-8)     # (a + 2b, b) spans the same lattice
    inf = plan.info
    d, xi, eta = inf["d"], inf["xi"], inf["eta"]
    # Sec. 1 conventions: e1 = (d, 0) longest, eta > 0, |xi| <= d/2, same cell area
    assert d >= np.hypot(xi, eta) - 1e-12 and eta > 0 and abs(xi) <= d / 2 + 1e-12
    assert abs(d * eta - 3.0) < 1e-12
    # the canonical basis spans the user's lattice: the user vectors, rotated
    # into the canonical frame, have integer lattice coordinates
    c, s = inf["rot_cos"], inf["rot_sin"]
    Rc = np.array([[c, -s], [s, c]])
    B = np.array([[d, xi], [0.0, eta]])
    for v in (a + 2 * b, b, a):
        u = np.linalg.solve(B, Rc @ v)
        assert np.allclose(u, np.round(u), atol=1e-12)
    # reduced: here the shortest lattice vector is (0.6, 1) and the next (2.4, -1)
    assert abs(np.hypot(xi, eta) - np.hypot(0.6, 1.0)) < 1e-12 and abs(d - 2.6) < 1e-12
    assert inf["m0"] == 1 and inf["n_images"] == 9


def test_hexagonal_cell_keeps_nine_images_with_rotated_west_east_waves(P):
    # with the west/east waves along the x axis the hexagonal cell needs m0 = 2
    # (Sec. 7 uses it for theta = pi/3); taken along e2-perp instead (Appendix
    # A) the closest west/east image is a full column away and m0 = 1 holds
    plan = P.Plan("stokes", (1.0, 0.0), (0.5, np.sqrt(3) / 2), 1e-6)
    inf = plan.info
    assert inf["m0"] == 1 and inf["n_images"] == 9 and inf["ew_rotated"] == 1
    c, s = inf["ew_cos"], inf["ew_sin"]
    assert abs(c * c + s * s - 1) < 1e-15
    assert abs(c * inf["xi"] - s * inf["eta"]) < 1e-14        # e2 on the frame's y axis
    assert s * inf["xi"] + c * inf["eta"] > 0
    # an explicit m0 = 2 keeps the canonical frame (15 images)
    inf2 = P.Plan("stokes", (1.0, 0.0), (0.5, np.sqrt(3) / 2), 1e-6, m0=2).info
    assert inf2["m0"] == 2 and inf2["n_images"] == 15 and inf2["ew_rotated"] == 0
    assert inf2["ew_cos"] == 1.0 and inf2["ew_sin"] == 0.0


@pytest.mark.parametrize("cell", [((1.0, 0.0), (0.5, np.sqrt(3) / 2)), ((3.0, 0.0), (1.2, 1.0)),
                                  ((40.0, 0.0), (17.0, 1.0))])
@pytest.mark.parametrize("beta,tol", [(0.3, 1e-6), (3.0, 1e-10), (0.3, 1e-10)])
def test_rotated_west_east_rule_sums_the_columns(P, cell, beta, tol):
    # eq. k0west2: in the rotated frame the west columns p >= 2 of rows
    # n = -1, 0, 1 sum to Re int_0^inf e^{-kappa X} e^{i lam Y} R B / kappa,
    # R = sum_p e^{-p (kappa dx - i lam dy)}, B = sum_n e^{-i n lam eta'};
    # against the direct sum of K0 over those images
    plan = P.Plan("yukawa", *cell, tol, beta=beta)
    inf = plan.info
    assert inf["ew_rotated"] == 1 and inf["m0"] == 1
    lam, w = plan.quadrature()
    c, s = inf["ew_cos"], inf["ew_sin"]
    dx, dy = c * inf["d"], s * inf["d"]
    eta2 = s * inf["xi"] + c * inf["eta"]
    kap = np.sqrt(lam ** 2 + beta ** 2)
    a = kap * dx - 1j * lam * dy
    R = np.exp(-2 * a) / (1 - np.exp(-a))
    B = 1 + 2 * np.cos(lam * eta2)
    pmax = int(np.ceil(60.0 / (beta * dx))) + 3
    for X in np.linspace(-0.99 * dx, 0.99 * dx, 5):
        for Y in np.linspace(-(abs(dy) + eta2), abs(dy) + eta2, 7):
            approx = np.sum(w * (np.exp(-kap * X + 1j * lam * Y) * R * B).real / kap)
            exact = sum(sp.k0(beta * np.hypot(X + p * dx, Y + p * dy - n * eta2))
                        for p in range(2, pmax) for n in (-1, 0, 1))
            scale = sp.k0(beta * dx)
            assert abs(approx - exact) < 10 * inf["eps"] * scale + 1e-13, (X, Y, approx, exact)


@pytest.mark.parametrize("d,eta,tol", [(1.0, 1.0, 1e-10), (100.0, 1.0, 1e-6), (20.0, 1.0, 1e-6), (10.0, 1.0, 1e-6)])
def test_mode_count_follows_truncation_formula(P, d, eta, tol):
    # eq. mpk0s with the internal tolerance eps = tol/10
    plan = P.Plan("laplace", (d, 0.0), (0.0, eta), tol)
    eps = plan.info["eps"]
    M = int(np.ceil(d / (2 * np.pi * eta) * np.log(1 / ((1 - np.exp(-2 * np.pi * eta / d)) * eps))))
    assert plan.info["n_modes"] == M
    # and the bound of eq. esbound1 on the dropped modes is below eps
    q = np.exp(-2 * np.pi * (M + 1) * eta / d)
    Es = q / (2 * np.pi * (M + 1) * (1 - q) * (1 - np.exp(-2 * np.pi * eta / d)))
    assert Es < eps


@pytest.mark.parametrize("cell", [((1.0, 0.0), (0.0, 1.0)), ((2.0, 0.0), (0.4, 1.0)),
                                  ((10.0, 0.0), (1.5, 1.0)), ((100.0, 0.0), (0.0, 1.0))])
@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_west_east_rule_integrates_laplace_plane_waves(P, cell, tol):
    # (canonical west/east frame; the rotated one is checked below)
    # int_0^inf e^{-lam X} e^{i lam Y} dlam = 1/(X - iY) over the X, Y range
    # the rule is used on (closest west/east image and beyond, |Y| <= 2 eta)
    plan = P.Plan("laplace", *cell, tol)
    inf = plan.info
    lam, w = plan.quadrature()
    d, xi, eta, m0 = inf["d"], inf["xi"], inf["eta"], inf["m0"]
    Xmin = m0 * d - 2 * abs(xi)
    for X in np.linspace(Xmin, Xmin + 3 * d, 7):
        for Y in np.linspace(-2 * eta, 2 * eta, 9):
            approx = np.sum(w * np.exp(-lam * X + 1j * lam * Y))
            exact = 1.0 / (X - 1j * Y)
            assert abs(approx - exact) < 2 * inf["eps"] * abs(exact) + 1e-15, (X, Y)


@pytest.mark.parametrize("beta", [0.3, 3.0, 10.0])
def test_west_east_rule_integrates_sommerfeld_k0(P, beta):
    # eq. k0planewave: K0(beta r) = int_0^inf e^{-kappa X} cos(lam Y)/kappa dlam
    plan = P.Plan("yukawa", (2.0, 0.0), (0.3, 1.0), 1e-10, beta=beta)
    inf = plan.info
    lam, w = plan.quadrature()
    kap = np.sqrt(lam ** 2 + beta ** 2)
    d, xi, eta, m0 = inf["d"], inf["xi"], inf["eta"], inf["m0"]
    Xmin = m0 * d - 2 * abs(xi)
    scale = sp.k0(beta * Xmin)
    for X in np.linspace(Xmin, Xmin + 2 * d, 5):
        for Y in np.linspace(-2 * eta, 2 * eta, 7):
            approx = np.sum(w * np.exp(-kap * X) * np.cos(lam * Y) / kap)
            exact = sp.k0(beta * np.hypot(X, Y))
            assert abs(approx - exact) < 10 * inf["eps"] * max(scale, 1e-300) + 1e-13, (X, Y)


def test_yukawa_west_east_dropped_when_negligible(P):
    plan = P.Plan("yukawa", (1.0, 0.0), (0.0, 1.0), 1e-6, beta=40.0)
    assert plan.info["n_quad"] == 0


@pytest.mark.parametrize("kw,code", [
    (dict(kernel="laplace", e1=(1.0, 0.0), e2=(2.0, 0.0), tol=1e-6), "PFMM_EINVAL_LATTICE"),
    (dict(kernel="laplace", e1=(1.0, 0.0), e2=(np.nan, 1.0), tol=1e-6), "PFMM_EINVAL_LATTICE"),
    (dict(kernel="laplace", e1=(1.0, 0.0), e2=(0.0, 1.0), tol=1e-16), "PFMM_EINVAL_TOL"),
    (dict(kernel="laplace", e1=(1.0, 0.0), e2=(0.0, 1.0), tol=0.5), "PFMM_EINVAL_TOL"),
    (dict(kernel="yukawa", e1=(1.0, 0.0), e2=(0.0, 1.0), tol=1e-6), "PFMM_EINVAL"),
    (dict(kernel="laplace", e1=(1.0, 0.0), e2=(0.0, 1.0), tol=1e-6, n_dens=0), "PFMM_EINVAL"),
    # symmetric pair evaluation needs targets == sources
    (dict(kernel="laplace", e1=(1.0, 0.0), e2=(0.0, 1.0), tol=1e-6, near_mode="mutual"), "PFMM_EINVAL"),
])
def test_plan_rejects_bad_arguments(P, kw, code):
    with pytest.raises(P.PfmmError) as e:
        P.Plan(**kw)
    from paper_2111_01083_amd import _lib
    assert _lib.ERRORS[e.value.code] == code


def test_south_terms_at_double_precision_match_the_papers_estimate(P):
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "south_terms_double_precision.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for A, per_a, band in ((float(a), float(b), float(c)) for a, b, c in rows):
        for kernel, beta in (("laplace", 0.0), ("yukawa", 1.0)):
            M = P.Plan(kernel, (A, 0.0), (0.0, 1.0), 1e-14, beta=beta).info["n_modes"]
            assert abs(M / A - per_a) <= band * per_a, (kernel, A, M)


def test_west_east_rule_size_against_the_papers_node_counts(P):
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "ggq_node_counts.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for kernel, beta, digits, paper, ratio in rows:
        # `digits` correct digits = internal eps 10^-digits = tol 10^(1 - digits)
        plan = P.Plan(kernel, (1.0, 0.0), (0.0, 1.0), 10.0 ** (1 - int(digits)), beta=float(beta))
        n = plan.info["n_quad"]
        assert 0 < n <= float(ratio) * int(paper), (kernel, beta, digits, n)


def test_workspace_size_grows_with_problem(P):
    plan = P.Plan("stokes", (1.0, 0.0), (0.0, 1.0), 1e-6, precision="mixed")
    a = P.pfmm_workspace_bytes(plan, 1000, 500)
    b = P.pfmm_workspace_bytes(plan, 100000, 50000)
    assert 0 < a < b and a % 256 == 0


@pytest.mark.parametrize("kernel", ["laplace", "yukawa", "stokes"])
@pytest.mark.parametrize("near_mode", ["one_sided", "mutual"])
@pytest.mark.parametrize("cell", [((1.1, 0.35), (-0.2, 0.9)), ((100.0, 0.0), (0.0, 1.0))])
def test_workspace_sizes_of_empty_inputs(P, kernel, near_mode, cell):
    # sizing for no sources, no targets, or neither is host-only work and must
    # not fail for any plan shape (symmetric near field, NUFFT far field, adjoint)
    for prec in ("fp64", "mixed"):
        kw = dict(beta=3.0 if kernel == "yukawa" else 0.0, precision=prec)
        plan = P.Plan(kernel, *cell, 1e-6, **kw)
        for ns, nt in ((0, 37), (50, 0), (0, 0)):
            assert P.pfmm_workspace_bytes(plan, ns, nt) > 0
        splan = P.Plan(kernel, *cell, 1e-6, self_exclude=True, near_mode=near_mode, **kw)
        assert P.pfmm_workspace_bytes(splan, 0, 0) > 0
        assert P.pfmm_workspace_bytes_adjoint(splan, 0) > 0


def test_eval_without_workspace_is_rejected_before_any_launch(P):
    from paper_2111_01083_amd import _lib
    lib = _lib.load()
    plan = P.Plan("laplace", (1.0, 0.0), (0.0, 1.0), 1e-6)
    dummy = ctypes.c_void_p(256)   # never dereferenced: the size check fails first
    rc = lib.pfmm_eval(plan.handle, 10, dummy, dummy, 10, dummy, dummy, dummy, None, 0, None)
    assert _lib.ERRORS[rc] == "PFMM_EWORKSPACE"
    rc = lib.pfmm_eval(plan.handle, -1, dummy, dummy, 10, dummy, dummy, dummy, None, 0, None)
    assert _lib.ERRORS[rc] == "PFMM_EINVAL"


def test_sizes_beyond_the_point_limit_are_rejected_before_any_launch(P):
    from paper_2111_01083_amd import _lib
    lib = _lib.load()
    big = _lib.PFMM_MAX_POINTS + 1
    plan = P.Plan("laplace", (1.0, 0.0), (0.0, 1.0), 1e-6)
    assert P.pfmm_workspace_bytes(plan, _lib.PFMM_MAX_POINTS, 10) > 0
    assert P.pfmm_workspace_bytes(plan, big, 10) == 0 and P.pfmm_workspace_bytes(plan, 10, big) == 0
    dummy = ctypes.c_void_p(256)   # never dereferenced: the size check fails first
    for ns, nt in ((big, 10), (10, big)):
        rc = lib.pfmm_eval(plan.handle, ns, dummy, dummy, nt, dummy, dummy, dummy, dummy, 1 << 62, None)
        assert _lib.ERRORS[rc] == "PFMM_EINVAL"
    splan = P.Plan("laplace", (1.0, 0.0), (0.0, 1.0), 1e-6, self_exclude=True)
    assert P.pfmm_workspace_bytes_adjoint(splan, big) == 0
    rc = lib.pfmm_eval_adjoint(splan.handle, big, dummy, dummy, dummy, dummy, dummy, dummy, 1 << 62, None)
    assert _lib.ERRORS[rc] == "PFMM_EINVAL"
    plans = (ctypes.c_void_p * 2)(splan.handle.value, splan.handle.value)
    off = (ctypes.c_int64 * 3)(0, 10, 10 + big)
    out = ctypes.c_void_p()
    rc = lib.pfmm_batch_create(2, plans, off, None, 0, ctypes.byref(out))
    assert _lib.ERRORS[rc] == "PFMM_EINVAL" and not out.value


def test_tuning_get_set_and_nufft_grid(P):
    plan = P.Plan("laplace", (100.0, 0.0), (0.0, 1.0), 1e-6, far_mode="nufft")
    nf0, w0 = plan.info["nufft_nf"], plan.info["nufft_w"]
    assert plan.tuning == {"near_blocks": 0, "nufft_grid": 0, "fmm_level": 0, "fmm_leaves": 0}
    assert nf0 >= 2 * (2 * plan.info["n_modes"] + 1) and nf0 & (nf0 - 1) == 0
    plan.set_tuning(near_blocks=4096, nufft_grid=1)
    assert plan.tuning == {"near_blocks": 4096, "nufft_grid": 1, "fmm_level": 0, "fmm_leaves": 0}
    assert plan.info["nufft_nf"] == 2 * nf0 and plan.info["nufft_w"] == max(4, w0 - 1)
    plan.set_tuning(nufft_grid=0)
    assert plan.info["nufft_nf"] == nf0 and plan.info["nufft_w"] == w0
    # a doubled grid beyond the largest line (2^20 points) is refused and nothing changes
    big = P.Plan("laplace", (60000.0, 0.0), (0.0, 1.0), 1e-6, far_mode="nufft")
    assert big.info["nufft_nf"] == 1 << 20
    with pytest.raises(P.PfmmError):
        big.set_tuning(nufft_grid=1)
    assert big.tuning["nufft_grid"] == 0 and big.info["nufft_nf"] == 1 << 20
    with pytest.raises(P.PfmmError):
        plan.set_tuning(near_blocks=-1)


def _tables():
    import re
    txt = open(os.path.join(ROOT, "paper_2111_01083_amd", "csrc", "bessel_tables.h")).read()
    tabs = {}
    for name, body in re.findall(r"(\w+)\[\d+\] = \{([^}]*)\}", txt):
        tabs[name] = np.array([float(v) for v in body.split(",") if v.strip()])
    for name, val in re.findall(r"(\w+) = ([0-9.eE+-]+);", txt):
        tabs[name] = np.array([float(val)])
    return tabs


@pytest.mark.parametrize("tag,bar", [("F32", 1e-7), ("F64", 1e-14)])
def test_device_bessel_tables_against_scipy(tag, bar):
    # the K0/K1 forms the device evaluates (ascending series for x <= 2, scaled
    # large-argument fit for x > 2), in FP64 here, against scipy.special
    import scipy.special as sp
    from numpy.polynomial import chebyshev as C
    t = _tables()
    xs = np.linspace(2e-3, 2.0, 2001)
    tt = 0.25 * xs * xs
    lt = np.log(tt)
    hz = lambda c, v: np.polyval(c[::-1], v)
    k0 = hz(t[f"KS_P0_{tag}"], tt) - 0.5 * lt * hz(t[f"KS_I0_{tag}"], tt)
    k1x = (1 + tt * (lt * hz(t[f"KS_J1_{tag}"], tt) - hz(t[f"KS_P1_{tag}"], tt))) / xs ** 2
    assert np.max(np.abs(k0 / sp.k0(xs) - 1)) < bar
    assert np.max(np.abs(k1x * xs / sp.k1(xs) - 1)) < bar
    xl = np.linspace(2.0, 80.0, 4001)
    if tag == "F32":
        rx = 1.0 / xl
        k0l = hz(t["KL0_F32"], rx)
        k1l = hz(t["KL1_F32"], rx)
    else:
        s = 2 * (2.0 / xl) - 1
        k0l = C.chebval(s, t["KL0_F64"])
        k1l = C.chebval(s, t["KL1_F64"])
    assert np.max(np.abs(k0l / (sp.k0e(xl) * np.sqrt(xl)) - 1)) < bar
    assert np.max(np.abs(k1l / (sp.k1e(xl) * np.sqrt(xl)) - 1)) < bar
    if tag == "F32":
        # the shorter fits used where every argument is known to be >= KF_X
        xf = np.linspace(t["KF_X"][0], 200.0, 4001)
        assert np.max(np.abs(hz(t["KF0_F32"], 1.0 / xf) / (sp.k0e(xf) * np.sqrt(xf)) - 1)) < bar
        assert np.max(np.abs(hz(t["KF1_F32"], 1.0 / xf) / (sp.k1e(xf) * np.sqrt(xf)) - 1)) < bar


@pytest.mark.parametrize("e1,e2,m0,groups", [((1.0, 0.0), (0.0, 1.0), 0, 1), ((1.0, 0.0), (0.5, 0.866), 0, 1),
                                             ((1.0, 0.0), (0.5, 0.866), 2, 3), ((100.0, 0.0), (0.0, 1.0), 0, 1),
                                             ((4000.0, 0.0), (0.0, 1.0), 0, 3)])
def test_log_groups_of_the_symmetric_mixed_near_field(P, e1, e2, m0, groups):
    # 9 images: one group unless the cell is so thin that the product could
    # leave the FP32 range; 15 images (the hexagonal cell with m0 = 2) or such
    # thin cells: one group per row of images (one period apart)
    inf = P.Plan("laplace", e1, e2, 1e-6, precision="mixed", self_exclude=True, m0=m0).info
    assert inf["n_log_groups"] == groups and inf["n_images"] % groups == 0


@pytest.mark.parametrize("e1,e2,m0", [((1.0, 0.0), (0.0, 1.0), 0), ((1.0, 0.0), (0.5, 0.866), 0),
                                      ((1.0, 0.0), (0.3, 1.0), 3), ((10.0, 0.0), (0.0, 1.0), 0),
                                      ((2000.0, 0.0), (0.0, 1.0), 0), ((4000.0, 0.0), (0.0, 1.0), 0)])
def test_log_group_products_stay_in_the_fp32_range(P, e1, e2, m0):
    # FP32 emulation of the symmetric kernel's image products: for pair
    # differences across the cell, and for pairs as close as r^2 = 2^-100
    # under any one image, every partial product of a group (started at
    # 2^e0) stays a normal FP32 number; in cells of aspect <= 10 the typical
    # product is also near 1 (in thinner cells the range bound keeps e0 from
    # centring it: products of 2^80..2^100 there)
    f32 = np.float32
    pl = P.Plan("laplace", e1, e2, 1e-6, precision="mixed", self_exclude=True, m0=m0)
    inf = pl.info
    ends, e0 = pl.log_groups()
    assert ends[-1] == inf["n_images"] and len(ends) == inf["n_log_groups"]
    d, xi, eta, mm = inf["d"], inf["xi"], inf["eta"], (inf["n_images"] // 3 - 1) // 2
    sg = 2.0 ** round(-0.5 * np.log2(d * eta))
    imgs = np.array([(sg * (m * d + n * xi), sg * n * eta) for n in (-1, 0, 1) for m in range(-mm, mm + 1)])
    rng = np.random.default_rng(4)
    u, v = rng.uniform(-1, 1, (2, 4000))
    d0 = np.stack([sg * (u * d + v * xi), sg * v * eta], 1)
    # near-coincident pairs: 2^-50 from a random image, or a few FP64 ulps of
    # the shift where 2^-50 is not representable next to it (a pair any closer
    # is coincident in FP64, a singularity on every path)
    k = rng.integers(0, len(imgs), 400)
    ang = rng.uniform(0, 2 * np.pi, 400)
    off = np.maximum(2.0 ** -50, 8 * np.spacing(np.abs(imgs[k]).max(1)))
    close = imgs[k] + off[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    d0 = np.concatenate([d0, close])
    g0, logs = 0, []
    for end, e in zip(ends, e0):
        p = np.full(len(d0), f32(2.0 ** e))
        for i in range(g0, end):
            r2 = ((d0[:, 0] - imgs[i, 0]) ** 2 + (d0[:, 1] - imgs[i, 1]) ** 2).astype(f32)
            p = (p * r2).astype(f32)
            assert np.all(np.isfinite(p)) and np.all(p >= np.finfo(f32).tiny), (end, e, i)
        logs.append(np.log2(p[:4000].astype(np.float64)))
        g0 = end
    if max(abs(e1[0]), abs(e2[1])) <= 10:
        assert np.median(np.abs(np.concatenate(logs))) < 16


@pytest.mark.parametrize("cell,tol,grid", [(((100.0, 0.0), (0.0, 1.0)), 1e-6, 0), (((100.0, 0.0), (0.0, 1.0)), 1e-6, 1),
                                           (((100.0, 0.0), (0.0, 1.0)), 1e-10, 0), (((30.0, 0.0), (0.0, 1.0)), 1e-12, 0)])
def test_spread_kernel_polynomials_match_the_kernel(P, cell, tol, grid):
    # the device evaluates the w + 1 taps of the exponential-of-semicircle
    # kernel (Sec. 6.1) as the planner's polynomials in the grid offset; they
    # must reproduce exp(b (sqrt(1 - z^2) - 1)) on |z| < 1 (0 outside) to a
    # fraction of eps at every offset
    plan = P.Plan("laplace", *cell, tol, far_mode="nufft")
    if grid:
        plan.set_tuning(nufft_grid=1)
    coef, deg, b = plan.spread_kernel()
    w, eps = plan.info["nufft_w"], plan.info["eps"]
    assert deg == min(20, w + 4) and np.all(coef[w + 1:] == 0) and np.all(coef[:, deg:] == 0)
    f = np.linspace(0.0, 1.0, 4001, endpoint=False)
    u = 2 * f - 1
    for t in range(w + 1):
        z = (t + f - w / 2) / (w / 2)
        exact = np.where(np.abs(z) < 1, np.exp(b * (np.sqrt(np.clip(1 - z * z, 0, None)) - 1)), 0.0)
        approx = np.polynomial.polynomial.polyval(u, coef[t, :deg])
        assert np.abs(approx - exact).max() < 0.5 * eps, (t, np.abs(approx - exact).max())


def test_fmm_plan_options_and_workspace(P):
    # the FMM near part: Chebyshev order from the kernel and tolerance, only
    # for doubly periodic plans, leaf level as a tuning with its workspace
    cell = ((1.0, 0.0), (0.3, 1.0))
    orders = {}
    for k in ("laplace", "yukawa", "stokes"):
        for tol in (1e-3, 1e-6, 1e-10):
            orders[k, tol] = P.Plan(k, *cell, tol, beta=2.0, near_mode="fmm").info["fmm_order"]
    for k in ("laplace", "yukawa", "stokes"):
        assert 4 <= orders[k, 1e-3] < orders[k, 1e-6] < orders[k, 1e-10] <= 20
    assert orders["stokes", 1e-6] > orders["laplace", 1e-6] == orders["yukawa", 1e-6]
    assert P.Plan("laplace", *cell, 1e-6, near_mode="one_sided").info["fmm_order"] == 0
    with pytest.raises(P.PfmmError):
        P.Plan("laplace", *cell, 1e-6, near_mode="fmm", periodic=1)
    plan = P.Plan("stokes", *cell, 1e-6, near_mode="fmm", self_exclude=True, precision="mixed")
    n = 50000
    ws = {}
    for lv in (2, 4, 6):
        plan.set_tuning(fmm_level=lv)
        assert plan.tuning["fmm_level"] == lv
        ws[lv] = P.pfmm_workspace_bytes(plan, n, n)
    # expansions: P^2 (2 + 6) doubles per box, (4^(L+1) - 1) / 3 boxes
    P2 = plan.info["fmm_order"] ** 2
    assert ws[6] - ws[4] >= 8 * P2 * 8 * ((4 ** 7 - 4 ** 5) // 3)
    assert ws[2] < ws[4] < ws[6]
    with pytest.raises(P.PfmmError):
        plan.set_tuning(fmm_level=12)
    # symmetric leaves (targets are the sources) keep 4 slots of the 6
    # Stokes outputs per point; one-sided leaves need none; by default
    # mixed Stokes is one-sided, FP64 Stokes symmetric
    plan.set_tuning(fmm_level=4)
    one = P.pfmm_workspace_bytes(plan, n, n)
    plan.set_tuning(fmm_leaves=2)
    assert plan.tuning["fmm_leaves"] == 2
    assert P.pfmm_workspace_bytes(plan, n, n) - one == 8 * 4 * 6 * n
    plan.set_tuning(fmm_leaves=1)
    assert P.pfmm_workspace_bytes(plan, n, n) == one
    with pytest.raises(P.PfmmError):
        plan.set_tuning(fmm_leaves=3)
    plan.set_tuning(fmm_leaves=0)
    f64 = P.Plan("stokes", *cell, 1e-10, near_mode="fmm", self_exclude=True)
    f64.set_tuning(fmm_level=4)
    sym = P.pfmm_workspace_bytes(f64, n, n)
    f64.set_tuning(fmm_leaves=1)
    assert sym - P.pfmm_workspace_bytes(f64, n, n) == 8 * 4 * 6 * n
    other = P.Plan("stokes", *cell, 1e-6, near_mode="fmm", precision="mixed")
    other.set_tuning(fmm_level=4)
    one = P.pfmm_workspace_bytes(other, n, n)
    other.set_tuning(fmm_leaves=2)
    assert P.pfmm_workspace_bytes(other, n, n) == one
    plan.set_tuning(fmm_level=0)
    # forced levels deeper than the cap (4e6 leaves) are cut back, not refused
    plan.set_tuning(fmm_level=11)
    assert P.pfmm_workspace_bytes(plan, 10, 10) > 0
    assert plan.fmm_tree(10)["level"] <= 10
    plan.set_tuning(fmm_level=0)
    # the cost model deepens the tree with N; AUTO takes the FMM from
    # N_S N_T >= 2^32 on cells with at most 16 top boxes, never for P1
    t1, t2 = plan.fmm_tree(20000), plan.fmm_tree(2000000)
    assert t2["level"] > t1["level"] and t1["order"] == plan.info["fmm_order"]
    auto = P.Plan("laplace", *cell, 1e-6, self_exclude=True)
    assert auto.fmm_tree(60000) is None and auto.fmm_tree(70000) is not None
    assert P.Plan("laplace", (100.0, 0.0), (0.0, 1.0), 1e-6, self_exclude=True).fmm_tree(200000) is None
    assert P.Plan("laplace", (10.0, 0.0), (0.0, 1.0), 1e-6, self_exclude=True).fmm_tree(200000)["k1"] == 10
    assert P.Plan("laplace", *cell, 1e-6, self_exclude=True, periodic=1).fmm_tree(200000) is None
    assert P.Plan("laplace", *cell, 1e-6, self_exclude=True, near_mode="mutual").fmm_tree(200000) is None
    # top grid: boxes within 10 % of square where 128 top boxes allow it
    for e1, e2 in (((3.0, 0.0), (1.2, 1.0)), ((1.0, 0.0), (0.5, 0.8660254)), ((7.3, 0.0), (0.2, 1.0))):
        p = P.Plan("stokes", e1, e2, 1e-6, near_mode="fmm")
        t = p.fmm_tree(100000, 100000)
        inf = p.info
        r = inf["d"] / np.hypot(inf["xi"], inf["eta"])
        assert abs(np.log(r * t["k2"] / t["k1"])) <= np.log(1.1) + 1e-12, (e1, e2, t)
