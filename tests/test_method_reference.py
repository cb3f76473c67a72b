"""CPU restatement of the periodic scheme for the modified Helmholtz, Laplace and Stokes kernels,
written from the paper's formulas with numpy/scipy, fed with the planner's
host outputs only (canonical lattice and rotation, near-region width m0,
south/north truncation M, west/east quadrature nodes and weights), and
compared with the FP64 oracle (a plain truncated lattice sum).

It checks the host side of the plan end to end, without a GPU: if the
planner's canonical frame, m0, M or quadrature were wrong, or a reading of
the paper's theorems were, the scheme would miss the oracle.

  near part:  the 3 (2 m0 + 1) images of Def. 1 (eq. nearfarsplit), summed directly;
  south/north: Thm. south_thm and its corollary (rows n <= -2 and n >= 2);
  west/east:   Thm. west_thm (columns |m| > m0 of rows n = -1, 0, 1), through
               K0(beta r) = int_0^inf cos(lam y) e^{-kappa |x|} / kappa dlam,
               kappa = sqrt(lam^2 + beta^2).
The Laplace version takes the beta -> 0 limits (Thm. south_thm_lap): modes
m != 0 with |alpha_m|, the m = 0 term -y P_y / (d eta) plus the constant
sum_j q_j y_j^2 / (2 d eta) of the zero-mean convention, and west and east
together, each image's constant removed (neutral charges), so that the
integrand stays regular at lam = 0. The Stokes version is derived here from
the Stokeslet symbol (I - k k^T / k^2) / k^2 rather than transcribed from
Thms. south_thm_s and west_thm_s: south/north by Poisson summation along the
rows with a geometric sum over them, the m = 0 term on u1 only, west/east
from the 1D transforms of the symbol in x. Last, the NUFFT form of the
Laplace south/north sums (Sec. 6.1) with the planner's grid, width and line
count must reproduce the direct sums to well below tol.
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle
import workloads as W


@pytest.fixture(scope="module")
def P():
    import os
    from paper_2111_01083_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2111_01083_amd import build
        build.build()
    import paper_2111_01083_amd as P
    return P


def _canonical(info, pts):
    """User frame -> canonical frame (e1 = (d, 0), e2 = (xi, eta)), wrapped
    into the cell u1 e1 + u2 e2, u in [-1/2, 1/2)^2."""
    c, s = info["rot_cos"], info["rot_sin"]
    R = np.array([[c, -s], [s, c]])
    p = R @ pts
    B = np.array([[info["d"], info["xi"]], [0.0, info["eta"]]])
    u = np.linalg.solve(B, p)
    u -= np.floor(u + 0.5)
    return B @ u, R


# the last four have |xi| > d/4 after reduction: their west/east waves run
# along e2-perp (Appendix A) with m0 = 1
SCHEME_CELLS = [((1.0, 0.0), (0.0, 1.0)), ((2.0, 0.0), (0.4, 1.0)), ((1.1, 0.35), (-0.2, 0.9)),
                ((10.0, 0.0), (1.5, 1.0)), ((1.0, 0.0), (0.5, np.sqrt(3) / 2)), ((1.0, 0.0), (0.4, 1.0)),
                ((3.0, 0.0), (1.2, 1.0)), ((40.0, 0.0), (17.0, 1.0))]


def _ew_frame(info, s, t):
    """West/east frame of the plan (Appendix A; the identity unless the waves
    run along e2-perp): pair differences X, Y in it, e1 = (dx, dy) and
    e2 = (xi2, eta2) there, and the rotation (c, sn) from the canonical frame."""
    c, sn = info["ew_cos"], info["ew_sin"]
    Rb = np.array([[c, -sn], [sn, c]])
    sb, tb = Rb @ s, Rb @ t
    e1 = Rb @ np.array([info["d"], 0.0])
    e2 = Rb @ np.array([info["xi"], info["eta"]])
    X = tb[0][:, None] - sb[0][None, :]
    Y = tb[1][:, None] - sb[1][None, :]
    return X, Y, e1[0], e1[1], e2[0], e2[1], Rb


def _columns(kap, lam, dx, dy, p):
    """sum_{q >= p} e^{-q a} and sum_{q >= p} q e^{-q a}, a = kappa dx - i lambda dy
    (the west columns; the east ones are the conjugates)."""
    a = kap * dx - 1j * lam * dy
    ea = np.exp(-a)
    T0 = np.exp(-p * a) / (1 - ea)
    T1 = np.exp(-p * a) * (p - (p - 1) * ea) / (1 - ea) ** 2
    return T0, T1


def _scalar_ew(info, lam, wq, kap, s, t, q, laplace):
    """West + east columns (|m| >= m0 + 1 of rows -1, 0, 1) of a scalar kernel
    in the plan's west/east frame; returns pot and the canonical gradient.
    Laplace drops each image's pair-independent constant (neutral charges)."""
    X, Y, dx, dy, xi2, eta2, Rb = _ew_frame(info, s, t)
    T0, _ = _columns(kap, lam, dx, dy, info["m0"] + 1)
    base = wq / kap / (2 * np.pi)
    pot = np.zeros(t.shape[1]); gx = np.zeros_like(pot); gy = np.zeros_like(pot)
    for n in ((0,) if info["periodic"] == 1 else (-1, 0, 1)):
        Xn = (X - n * xi2)[..., None]; Yn = (Y - n * eta2)[..., None]
        ph = np.exp(1j * lam * Yn)
        west = np.exp(-kap * Xn) * T0
        east = np.exp(kap * Xn) * np.conj(T0)
        tot = ph * (west + east)
        if laplace:
            tot = tot - 2 * T0.real
        pot += ((tot.real * base).sum(-1)) @ q
        gx += (((ph * kap * (east - west)).real * base).sum(-1)) @ q
        gy += (((1j * lam * ph * (west + east)).real * base).sum(-1)) @ q
    return pot, Rb.T @ np.vstack([gx, gy])


def yukawa_scheme(info, lam, wq, beta, src, q, trg):
    d, xi, eta, m0, M = info["d"], info["xi"], info["eta"], info["m0"], info["n_modes"]
    s, R = _canonical(info, src)
    t, _ = _canonical(info, trg)
    X = t[0][:, None] - s[0][None, :]           # [nt, ns]
    Y = t[1][:, None] - s[1][None, :]
    pot = np.zeros(t.shape[1]); gx = np.zeros_like(pot); gy = np.zeros_like(pot)
    # near images
    for n in (-1, 0, 1):
        for m in range(-m0, m0 + 1):
            dx = X - m * d - n * xi
            dy = Y - n * eta
            r = np.hypot(dx, dy)
            pot += (sp.k0(beta * r) @ q) / (2 * np.pi)
            k1r = beta * sp.k1(beta * r) / r
            gx -= ((k1r * dx) @ q) / (2 * np.pi)
            gy -= ((k1r * dy) @ q) / (2 * np.pi)
    # south / north: rows n <= -2 and n >= 2, a geometric sum over the row index
    m = np.arange(-M, M + 1)
    al = 2 * np.pi * m / d
    chi = np.sqrt(al * al + beta * beta)
    Q = chi * eta - 1j * al * xi
    DS = np.exp(-2 * Q) / (2 * d * chi * (1 - np.exp(-Q)))
    Qn = chi * eta + 1j * al * xi
    DN = np.exp(-2 * Qn) / (2 * d * chi * (1 - np.exp(-Qn)))
    cS = (np.exp(chi[:, None] * s[1][None, :] - 1j * al[:, None] * s[0][None, :]) * q[None, :]).sum(1)
    cN = (np.exp(-chi[:, None] * s[1][None, :] - 1j * al[:, None] * s[0][None, :]) * q[None, :]).sum(1)
    eS = np.exp(-chi[None, :] * t[1][:, None] + 1j * al[None, :] * t[0][:, None]) * (DS * cS)[None, :]
    eN = np.exp(chi[None, :] * t[1][:, None] + 1j * al[None, :] * t[0][:, None]) * (DN * cN)[None, :]
    pot += (eS + eN).sum(1).real
    gx += ((eS + eN) * (1j * al)[None, :]).sum(1).real
    gy += ((-eS + eN) * chi[None, :]).sum(1).real
    # west / east: columns m >= m0 + 1 (east) and m <= -(m0 + 1) (west) of rows -1, 0, 1
    kap = np.sqrt(lam * lam + beta * beta)
    pe, ge = _scalar_ew(info, lam, wq, kap, s, t, q, laplace=False)
    grad = R.T @ (np.vstack([gx, gy]) + ge)
    return pot + pe, grad


def laplace_scheme(info, lam, wq, src, q, trg):
    d, xi, eta, m0, M = info["d"], info["xi"], info["eta"], info["m0"], info["n_modes"]
    s, R = _canonical(info, src)
    t, _ = _canonical(info, trg)
    X = t[0][:, None] - s[0][None, :]
    Y = t[1][:, None] - s[1][None, :]
    pot = np.zeros(t.shape[1]); gx = np.zeros_like(pot); gy = np.zeros_like(pot)
    # near images
    for n in (-1, 0, 1):
        for m in range(-m0, m0 + 1):
            dx = X - m * d - n * xi; dy = Y - n * eta
            r2 = dx * dx + dy * dy
            pot += (-0.5 * np.log(r2) @ q) / (2 * np.pi)
            gx -= ((dx / r2) @ q) / (2 * np.pi)
            gy -= ((dy / r2) @ q) / (2 * np.pi)
    # south / north, modes m != 0
    m = np.concatenate([np.arange(-M, 0), np.arange(1, M + 1)])
    al = 2 * np.pi * m / d
    chi = np.abs(al)
    Q = chi * eta - 1j * al * xi
    DS = np.exp(-2 * Q) / (4 * np.pi * np.abs(m) * (1 - np.exp(-Q)))
    Qn = chi * eta + 1j * al * xi
    DN = np.exp(-2 * Qn) / (4 * np.pi * np.abs(m) * (1 - np.exp(-Qn)))
    cS = (np.exp(chi[:, None] * s[1][None, :] - 1j * al[:, None] * s[0][None, :]) * q[None, :]).sum(1)
    cN = (np.exp(-chi[:, None] * s[1][None, :] - 1j * al[:, None] * s[0][None, :]) * q[None, :]).sum(1)
    eS = np.exp(-chi[None, :] * t[1][:, None] + 1j * al[None, :] * t[0][:, None]) * (DS * cS)[None, :]
    eN = np.exp(chi[None, :] * t[1][:, None] + 1j * al[None, :] * t[0][:, None]) * (DN * cN)[None, :]
    pot += (eS + eN).sum(1).real
    gx += ((eS + eN) * (1j * al)[None, :]).sum(1).real
    gy += ((-eS + eN) * chi[None, :]).sum(1).real
    # m = 0 south + north and the zero-mean constant
    Py = (q * s[1]).sum()
    pot += -t[1] * Py / (d * eta) + (q * s[1] ** 2).sum() / (2 * d * eta)
    gy += -Py / (d * eta)
    # west + east together (regular at lam = 0 after removing the constant of each image)
    pe, ge = _scalar_ew(info, lam, wq, lam, s, t, q, laplace=True)
    return pot + pe, R.T @ (np.vstack([gx, gy]) + ge)


def _stokes_ew(info, lam, wq, s, t, f1, f2):
    """West + east columns of the Stokeslet in the plan's west/east frame
    (canonical force components f1, f2; canonical velocity and gradient out)."""
    nt = t.shape[1]
    m0 = info["m0"]
    u = np.zeros((2, nt))
    g = np.zeros((2, 2, nt))
    Xb, Yb, dxb, dyb, xi2, eta2, Rb = _ew_frame(info, s, t)
    fb1, fb2 = Rb @ np.vstack([f1, f2])
    ub = np.zeros((2, nt))
    gb = np.zeros((2, 2, nt))

    def applyb(txx, txy, tyy):
        return np.array([txx @ fb1 + txy @ fb2, txy @ fb1 + tyy @ fb2])

    T0, T1 = _columns(lam, lam, dxb, dyb, m0 + 1)
    w = wq / np.pi
    xx_ref = (2 * T0.real + 2 * lam * dxb * T1.real) / (4 * lam)
    yy_ref = (2 * T0.real - 2 * lam * dxb * T1.real) / (4 * lam)
    for n in ((0,) if info["periodic"] == 1 else (-1, 0, 1)):
        X0 = (Xb - n * xi2)[..., None]
        Yn = (Yb - n * eta2)[..., None]
        ph = np.exp(1j * lam * Yn)
        AE, AW = np.exp(lam * X0) * np.conj(T0), np.exp(-lam * X0) * T0
        BE = np.exp(lam * X0) * (dxb * np.conj(T1) - X0 * np.conj(T0))
        BW = np.exp(-lam * X0) * (X0 * T0 + dxb * T1)
        A, B = AE + AW, BE + BW
        ub += applyb((((ph * (A + lam * B)).real / (4 * lam) - xx_ref) * w).sum(-1),
                     ((0.25 * (ph * (BW - BE)).imag) * w).sum(-1),
                     (((ph * (A - lam * B)).real / (4 * lam) - yy_ref) * w).sum(-1))
        dA = lam * (AE - AW)
        dB = lam * (BE - BW) - AE + AW
        gb[:, 0] += applyb(((ph * (dA + lam * dB)).real / (4 * lam) * w).sum(-1),
                           (0.25 * (ph * (AW + AE - lam * (BW + BE))).imag * w).sum(-1),
                           ((ph * (dA - lam * dB)).real / (4 * lam) * w).sum(-1))
        gb[:, 1] += applyb((-(ph * (A + lam * B)).imag / 4 * w).sum(-1),
                           (0.25 * (ph * (BW - BE)).real * lam * w).sum(-1),
                           (-(ph * (A - lam * B)).imag / 4 * w).sum(-1))
    u += Rb.T @ ub
    g += np.einsum("ji,jkt,kl->ilt", Rb, gb, Rb)
    return u, g


def stokes_scheme(info, lam, wq, src, f, trg):
    d, xi, eta, m0, M = info["d"], info["xi"], info["eta"], info["m0"], info["n_modes"]
    s, R = _canonical(info, src)
    t, _ = _canonical(info, trg)
    f1, f2 = R @ f                               # forces in the canonical frame
    X = t[0][:, None] - s[0][None, :]
    Y = t[1][:, None] - s[1][None, :]
    nt = t.shape[1]
    u = np.zeros((2, nt))
    g = np.zeros((2, 2, nt))                     # g[i, k] = d u_i / d x_k

    def apply(txx, txy, tyy):                    # sum_j T_j f_j for a symmetric 2x2 T
        return np.array([txx @ f1 + txy @ f2, txy @ f1 + tyy @ f2])

    # near images: G = (1/4pi)(-log r I + r r^T / r^2)
    c4 = 1 / (4 * np.pi)
    for n in (-1, 0, 1):
        for m in range(-m0, m0 + 1):
            r = (X - m * d - n * xi, Y - n * eta)
            r2 = r[0] ** 2 + r[1] ** 2
            L = -0.5 * np.log(r2)
            u += c4 * apply(L + r[0] ** 2 / r2, r[0] * r[1] / r2, L + r[1] ** 2 / r2)
            for k in range(2):
                def dG(i, j):
                    return c4 * (-(i == j) * r[k] / r2 + ((k == i) * r[j] + (k == j) * r[i]) / r2
                                 - 2 * r[i] * r[j] * r[k] / (r2 * r2))
                g[:, k] += apply(dG(0, 0), dG(0, 1), dG(1, 1))
    # south (rows n <= -2) and north (n >= 2), modes m != 0: Poisson summation
    # in x turns a row at offset Y_n into (1/d) sum_m T(alpha_m, Y_n) e^{i alpha_m X_n},
    # with, for a = |alpha|, |Y_n| = y:  T_xx = (1 - a y) e^{-a y} / (4a),
    # T_yy = (1 + a y) e^{-a y} / (4a), T_xy = -i alpha Y_n e^{-a y} / (4a);
    # the rows then sum geometrically (S0 = sum_{p>=2} e^{-pQ}, S1 = sum p e^{-pQ})
    for mm in list(range(-M, 0)) + list(range(1, M + 1)):
        al = 2 * np.pi * mm / d
        a = abs(al)
        for side in (-1, 1):
            E = np.exp(-(a * eta + side * 1j * al * xi))
            S0 = E * E / (1 - E)
            S1 = E * E * (2 - E) / (1 - E) ** 2
            c = np.exp(side * a * Y + 1j * al * X) / (4 * a * d)
            xx = c * ((1 + side * a * Y) * S0 - a * eta * S1)
            yy = c * ((1 - side * a * Y) * S0 + a * eta * S1)
            xy = c * (1j * al) * (side * eta * S1 - Y * S0)
            dxx = side * a * xx + side * c * a * S0
            dyy = side * a * yy - side * c * a * S0
            dxy = side * a * xy - c * (1j * al) * S0
            u += apply(xx, xy, yy).real
            g[:, 0] += apply(1j * al * xx, 1j * al * xy, 1j * al * yy).real
            g[:, 1] += apply(dxx, dxy, dyy).real
    # m = 0: u1 only (T_xx(0, k_y) = 1/k_y^2, the Laplace symbol), plus the zero-mean constant
    P1 = (f1 * s[1]).sum()
    u[0] += -t[1] * P1 / (d * eta) + (f1 * s[1] ** 2).sum() / (2 * d * eta)
    g[0, 1] += -P1 / (d * eta)
    # west + east (rows -1, 0, 1; columns |m| >= p = m0 + 1) from
    #   G_xx = (1/pi) int cos(lam Y) (1 + lam|X|) e^{-lam|X|} / (4 lam),
    #   G_yy = (1/pi) int cos(lam Y) (1 - lam|X|) e^{-lam|X|} / (4 lam),
    #   G_xy = (1/pi) int sin(lam Y) X e^{-lam|X|} / 4,
    # in the plan's west/east frame (forces rotated into it, results rotated
    # back), summed over the columns (A = sum e^{-lam|X|}, B = sum |X| e^{-lam|X|},
    # complex geometric sums when e1 is not along the frame's x axis; cos and
    # sin become real and imaginary parts of e^{i lam Y}); the part of G_xx,
    # G_yy that does not depend on the pair is removed (zero net force)
    ue, ge = _stokes_ew(info, lam, wq, s, t, f1, f2)
    u += ue
    g += ge
    # back to the caller's frame: u -> R^T u, grad u -> R^T (grad u) R
    return R.T @ u, np.einsum("ji,jkt,kl->ilt", R, g, R).reshape(4, nt)


@pytest.mark.parametrize("cell", SCHEME_CELLS)
@pytest.mark.parametrize("beta", [0.5, 3.0, 10.0])
def test_yukawa_scheme_from_plan_matches_oracle(P, cell, beta):
    # beta = 10 on the square cell: the planner drops the west/east part and
    # all but a few south/north modes as negligible (their whole factor is
    # below eps); the scheme must still meet tol
    e1, e2 = cell
    rng = np.random.default_rng(31)
    src = W.cell_points(rng, e1, e2, 40)
    trg = W.cell_points(rng, e1, e2, 25)
    q = rng.standard_normal(40)
    po, go = oracle.yukawa(e1, e2, beta, src, q, trg)
    for tol in (1e-6, 1e-10):
        plan = P.Plan("yukawa", e1, e2, tol, beta=beta)
        info = plan.info
        lam, wq = plan.quadrature()
        pot, grad = yukawa_scheme(info, lam, wq, beta, src, q, trg)
        ep = np.linalg.norm(pot - po) / np.linalg.norm(po)
        eg = np.linalg.norm(grad - go) / np.linalg.norm(go)
        assert ep < tol and eg < tol, (tol, ep, eg, info["m0"], info["n_modes"], len(lam))


@pytest.mark.parametrize("cell", SCHEME_CELLS)
def test_laplace_scheme_from_plan_matches_oracle(P, cell):
    e1, e2 = cell
    rng = np.random.default_rng(31)
    src = W.cell_points(rng, e1, e2, 40)
    trg = W.cell_points(rng, e1, e2, 25)
    q = W.neutral_charges(rng, 40)
    po, go = oracle.laplace(e1, e2, src, q, trg)
    for tol in (1e-6, 1e-10):
        plan = P.Plan("laplace", e1, e2, tol)
        info = plan.info
        lam, wq = plan.quadrature()
        pot, grad = laplace_scheme(info, lam, wq, src, q, trg)
        ep = np.linalg.norm(pot - po) / np.linalg.norm(po)
        eg = np.linalg.norm(grad - go) / np.linalg.norm(go)
        assert ep < tol and eg < tol, (tol, ep, eg, info["m0"], info["n_modes"], len(lam))


@pytest.mark.parametrize("cell", SCHEME_CELLS)
def test_stokes_scheme_from_plan_matches_oracle(P, cell):
    e1, e2 = cell
    rng = np.random.default_rng(31)
    src = W.cell_points(rng, e1, e2, 40)
    trg = W.cell_points(rng, e1, e2, 25)
    f = W.neutral_forces(rng, 40)
    uo, go = oracle.stokes(e1, e2, src, f, trg)
    for tol in (1e-6, 1e-10):
        plan = P.Plan("stokes", e1, e2, tol)
        info = plan.info
        lam, wq = plan.quadrature()
        u, grad = stokes_scheme(info, lam, wq, src, f, trg)
        eu = np.linalg.norm(u - uo) / np.linalg.norm(uo)
        eg = np.linalg.norm(grad - go) / np.linalg.norm(go)
        assert eu < tol and eg < tol, (tol, eu, eg, info["m0"], info["n_modes"], len(lam))


# --- NUFFT form of the south/north sums (Sec. 6.1) --------------------------
# Sources and targets are interpolated in y onto M_GL Gauss-Legendre lines
# (Lagrange basis at the lines), and the x sums along each line are type-1 /
# type-2 NUFFTs with the exponential-of-semicircle kernel
# phi(z) = exp(b (sqrt(1 - z^2) - 1)), b = 0.97 pi (1 - 1/(2 sigma)) w, on the
# planner's grid n_f (oversampling sigma = 2, or 4 on the doubled grid) and
# width w, deconvolved by phi's Fourier transform.

def _es(info, grid):
    w, nf, d = info["nufft_w"], info["nufft_nf"], info["d"]
    b = 0.97 * np.pi * (1 - 1 / (2 * (4.0 if grid else 2.0))) * w
    h = d / nf
    s = w * h / 2

    def phi(z):
        return np.where(np.abs(z) <= 1, np.exp(b * (np.sqrt(np.maximum(0.0, 1 - z * z)) - 1)), 0.0)

    z, wz = np.polynomial.legendre.leggauss(4 * w + 60)

    def phihat(al):                              # int phi(x / s) e^{-i al x} dx
        return s * (wz[None, :] * phi(z)[None, :] * np.cos(np.outer(al, s * z))).sum(1)
    return phi, phihat, h, s, nf, w


def _type1(es, d, x, c, al):
    """F_m = sum_j c_j e^{-i al_m x_j} (period d): spread, FFT, deconvolve."""
    phi, phihat, h, s, nf, w = es
    g = np.zeros(nf)
    for xj, cj in zip(x, c):
        ls = np.arange(int(np.floor((xj - s) / h)), int(np.floor((xj - s) / h)) + w + 3)
        np.add.at(g, np.mod(ls, nf), cj * phi((xj - ls * h) / s))
    m = np.rint(al * d / (2 * np.pi)).astype(int)
    return np.fft.fft(g)[np.mod(m, nf)] * h / phihat(al)


def _type2(es, d, G, al, x):
    """v(x) = sum_m G_m e^{i al_m x}: deconvolve, inverse FFT, interpolate."""
    phi, phihat, h, s, nf, w = es
    spec = np.zeros(nf, complex)
    np.add.at(spec, np.mod(np.rint(al * d / (2 * np.pi)).astype(int), nf), G / phihat(al))
    grid = np.fft.ifft(spec) * nf
    out = np.zeros(len(x), complex)
    for i, xt in enumerate(x):
        ls = np.arange(int(np.floor((xt - s) / h)), int(np.floor((xt - s) / h)) + w + 3)
        out[i] = (grid[np.mod(ls, nf)] * phi((xt - ls * h) / s)).sum() * h
    return out


def _lagrange(nodes, y):
    L = np.ones((len(nodes), len(y)))
    for k in range(len(nodes)):
        for i in range(len(nodes)):
            if i != k:
                L[k] *= (y - nodes[i]) / (nodes[k] - nodes[i])
    return L


def south_north(info, beta, src, q, trg, grid=None):
    """The south/north field of the scheme (beta = 0: Laplace, modes m != 0;
    else Yukawa, all modes), directly (grid None) or through the NUFFT form
    on the given grid."""
    d, xi, eta, M = info["d"], info["xi"], info["eta"], info["n_modes"]
    s, _ = _canonical(info, src)
    t, _ = _canonical(info, trg)
    m = np.concatenate([np.arange(-M, 0), np.arange(1, M + 1)]) if beta == 0 else np.arange(-M, M + 1)
    al = 2 * np.pi * m / d
    chi = np.sqrt(al * al + beta * beta)
    Q, Qn = chi * eta - 1j * al * xi, chi * eta + 1j * al * xi
    DS = np.exp(-2 * Q) / (2 * d * chi * (1 - np.exp(-Q)))      # 1 / (2 d chi) = 1 / (4 pi |m|) for Laplace
    DN = np.exp(-2 * Qn) / (2 * d * chi * (1 - np.exp(-Qn)))
    if grid is None:
        cS = (np.exp(chi[:, None] * s[1][None, :] - 1j * al[:, None] * s[0][None, :]) * q[None, :]).sum(1)
        cN = (np.exp(-chi[:, None] * s[1][None, :] - 1j * al[:, None] * s[0][None, :]) * q[None, :]).sum(1)
        eS = np.exp(-chi[None, :] * t[1][:, None] + 1j * al[None, :] * t[0][:, None]) * (DS * cS)[None, :]
        eN = np.exp(chi[None, :] * t[1][:, None] + 1j * al[None, :] * t[0][:, None]) * (DN * cN)[None, :]
        return (eS + eN).sum(1).real
    es = _es(info, grid)
    yb = 0.5 * eta * np.polynomial.legendre.leggauss(info["m_gl"])[0]
    gs, gt = _lagrange(yb, s[1]), _lagrange(yb, t[1])
    F = np.array([_type1(es, d, s[0], q * gs[k], al) for k in range(len(yb))])
    wS = DS * (np.exp(chi[None, :] * yb[:, None]) * F).sum(0)
    wN = DN * (np.exp(-chi[None, :] * yb[:, None]) * F).sum(0)
    out = np.zeros(t.shape[1])
    for k in range(len(yb)):
        out += (gt[k] * _type2(es, d, wS * np.exp(-chi * yb[k]) + wN * np.exp(chi * yb[k]), al, t[0])).real
    return out


@pytest.mark.parametrize("cell", [((100.0, 0.0), (0.0, 1.0)), ((20.0, 0.0), (3.0, 1.0)),
                                  ((30.0, 0.0), (7.0, 1.0))])
@pytest.mark.parametrize("kernel,beta,share", [("laplace", 0.0, 0.1), ("yukawa", 0.5, 0.1), ("yukawa", 5.0, 0.5)])
@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_nufft_parameters_from_plan_reach_tol(P, cell, kernel, beta, share, tol):
    # clustered sources (the high-aspect workload's blobs); the NUFFT form with
    # the planner's n_f, w and M_GL must reproduce the direct south/north
    # field to below share * tol of the whole potential, on both grids (with
    # beta = 5 the factors e^{chi y} interpolated across the lines are steeper)
    e1, e2 = cell
    rng = np.random.default_rng(5)
    src = W.blob_points(rng, e1, e2, 300)
    trg = W.cell_points(rng, e1, e2, 60)
    if kernel == "laplace":
        q = W.neutral_charges(rng, 300)
        po, _ = oracle.laplace(e1, e2, src, q, trg)
    else:
        q = rng.standard_normal(300)
        po, _ = oracle.yukawa(e1, e2, beta, src, q, trg, tol=1e-13)
    plan = P.Plan(kernel, e1, e2, tol, beta=beta, far_mode="nufft")
    direct = south_north(plan.info, beta, src, q, trg)
    for grid in (0, 1):
        if grid:
            plan.set_tuning(nufft_grid=1)
        info = plan.info
        err = np.linalg.norm(south_north(info, beta, src, q, trg, grid) - direct) / np.linalg.norm(po)
        assert err < share * tol, (grid, err, info["nufft_nf"], info["nufft_w"], info["m_gl"])


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_yukawa_near_cutoff_drops_less_than_eps(P, tol):
    # the screened near field leaves out pairs farther apart than r_c with
    # e^{-beta r_c} = eps / 30; on uniform sources (the benchmark's
    # distribution, square cell, beta = 10) what is left out stays below eps
    # of the potential and of the gradient
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    beta = 10.0
    plan = P.Plan("yukawa", e1, e2, tol, beta=beta)
    eps = plan.info["eps"]
    rc = np.log(30.0 / eps) / beta
    rng = np.random.default_rng(17)
    n = 1500
    src = W.cell_points(rng, e1, e2, n)
    q = W.neutral_charges(rng, n)
    trg = src[:, :300]
    pot = np.zeros(300); gx = np.zeros(300); gy = np.zeros(300)
    dpot = np.zeros(300); dgx = np.zeros(300); dgy = np.zeros(300)
    for n_ in (-1, 0, 1):
        for m in (-1, 0, 1):
            dx = trg[0][:, None] - src[0][None, :] - m
            dy = trg[1][:, None] - src[1][None, :] - n_
            r = np.hypot(dx, dy)
            r = np.where(r == 0, np.inf, r)        # the self pair
            k0 = sp.k0(beta * r) / (2 * np.pi)
            k1r = beta * sp.k1(beta * r) / r / (2 * np.pi)
            far = r > rc
            pot += k0 @ q; gx -= (k1r * dx) @ q; gy -= (k1r * dy) @ q
            dpot += (k0 * far) @ q; dgx -= (k1r * dx * far) @ q; dgy -= (k1r * dy * far) @ q
    assert np.linalg.norm(dpot) < eps * np.linalg.norm(pot)
    assert np.hypot(np.linalg.norm(dgx), np.linalg.norm(dgy)) < eps * np.hypot(np.linalg.norm(gx), np.linalg.norm(gy))


@pytest.mark.parametrize("kernel", ["laplace", "yukawa", "stokes"])
def test_wider_near_region_m0_3(P, kernel):
    # the paper's thin parallelograms use m0 = 3 (21 near images); with the
    # override the west/east sums start at column p = 4, which the scheme's
    # geometric factors must follow (for Stokes (p - (p-1) e^{-a}) / (1 - e^{-a})^2)
    e1, e2 = (1.0, 0.0), (0.3, 1.0)
    rng = np.random.default_rng(41)
    src = W.cell_points(rng, e1, e2, 30)
    trg = W.cell_points(rng, e1, e2, 20)
    tol = 1e-10
    plan = P.Plan(kernel, e1, e2, tol, beta=2.0 if kernel == "yukawa" else 0.0, m0=3)
    info = plan.info
    assert info["m0"] == 3 and info["n_images"] == 21
    lam, wq = plan.quadrature()
    if kernel == "stokes":
        f = W.neutral_forces(rng, 30)
        ref, gref = oracle.stokes(e1, e2, src, f, trg)
        u, g = stokes_scheme(info, lam, wq, src, f, trg)
    elif kernel == "laplace":
        q = W.neutral_charges(rng, 30)
        ref, gref = oracle.laplace(e1, e2, src, q, trg)
        u, g = laplace_scheme(info, lam, wq, src, q, trg)
    else:
        q = rng.standard_normal(30)
        ref, gref = oracle.yukawa(e1, e2, 2.0, src, q, trg)
        u, g = yukawa_scheme(info, lam, wq, 2.0, src, q, trg)
    eu = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    eg = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    assert eu < tol and eg < tol, (eu, eg)


# --- singly periodic plans (P1, Sec. 3 eq. ksplitting1) ----------------------
# Near part: the cell and its two neighbours along e1 (direct sums); far
# part: the west/east columns |m| >= 2 of the single row, from the planner's
# nodes and weights (Thm. west_thm with B = 1 and its Laplace/Stokes forms).

def p1_scheme(info, lam, wq, kernel, beta, src, dens, trg):
    c, s_ = info["rot_cos"], info["rot_sin"]
    R = np.array([[c, -s_], [s_, c]])
    d = info["d"]

    def canon(p):
        q = R @ p
        q[0] -= d * np.round(q[0] / d)
        return q
    sc, tc = canon(src), canon(trg)
    dc = R @ dens if kernel == "stokes" else dens
    s_img = np.concatenate([sc + np.array([[m * d], [0.0]]) for m in (-1, 0, 1)], axis=1)
    d_img = np.concatenate([dc] * 3, axis=-1)
    pot, grad = oracle.free_space(kernel, s_img, d_img, tc, beta=beta)
    if kernel == "stokes":
        ue, ge = _stokes_ew(info, lam, wq, sc, tc, dc[0], dc[1])
        u = pot + ue
        J = grad.reshape(2, 2, -1) + ge
        return R.T @ u, np.einsum("ji,jkt,kl->ilt", R, J, R).reshape(4, -1)
    kap = np.sqrt(lam * lam + beta * beta) if kernel == "yukawa" else lam
    pe, ge = _scalar_ew(info, lam, wq, kap, sc, tc, dc, laplace=kernel == "laplace")
    return pot + pe, R.T @ (grad + ge)


@pytest.mark.parametrize("e1,e2", [((1.0, 0.0), (0.0, 1.0)), ((1.3, 0.4), (0.2, 2.0)), ((1.0, 0.0), (0.0, 8.0)),
                                   ((6.0, 0.0), (0.0, 1.0))])
@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 0.5), ("yukawa", 4.0), ("stokes", 0.0)])
def test_p1_scheme_from_plan_matches_oracle(P, e1, e2, kernel, beta):
    rng = np.random.default_rng(37)
    n, nt = 40, 25
    # points in the strip: anywhere along e1, within half the height across it
    e1a = np.array(e1); dd = np.hypot(*e1a); along = e1a / dd; perp = np.array([-along[1], along[0]])
    H = abs(np.dot(np.array(e2), perp))
    src = np.outer(along, dd * (rng.random(n) - 0.5) + 3 * dd) + np.outer(perp, H * (rng.random(n) - 0.5))
    trg = np.outer(along, dd * (rng.random(nt) - 0.5)) + np.outer(perp, H * (rng.random(nt) - 0.5))
    dens = W.neutral_forces(rng, n) if kernel == "stokes" else W.neutral_charges(rng, n)
    po, go = oracle.singly_periodic(kernel, e1, src, dens, trg, beta=beta)
    for tol in (1e-6, 1e-10):
        plan = P.Plan(kernel, e1, e2, tol, beta=beta, periodic=1)
        info = plan.info
        assert info["periodic"] == 1 and info["n_images"] == 3 and info["n_modes"] == 0
        lam, wq = plan.quadrature()
        pot, grad = p1_scheme(info, lam, wq, kernel, beta, src, dens, trg)
        ep = np.linalg.norm(pot - po) / np.linalg.norm(po)
        eg = np.linalg.norm(grad - go) / np.linalg.norm(go)
        assert ep < tol and eg < tol, (tol, ep, eg, len(lam))
