"""Pins for the FP64 oracle: each check compares it with something other
than itself (a second independent formula, a library routine, a limit, an
invariant of the periodic problem), so that a dropped term, a wrong sign
or a wrong normalisation in any of its functions fails at least one test.
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle
import workloads as W

SHEARED = ((2.0, 0.0), (0.4, 1.0))          # d = 2, xi = 0.4, eta = 1
GENERAL = ((1.1, 0.35), (-0.2, 0.9))        # not canonical, rotated basis


def _setup(e1, e2, ns=12, nt=9, seed=1, stokes=False):
    rng = np.random.default_rng(seed)
    src = W.cell_points(rng, e1, e2, ns)
    trg = W.cell_points(rng, e1, e2, nt)
    dens = W.neutral_forces(rng, ns) if stokes else W.neutral_charges(rng, ns)
    return src, dens, trg


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


# --- library special functions the oracle calls -----------------------------

def test_free_space_yukawa_matches_scipy_bessel():
    rng = np.random.default_rng(3)
    src = rng.random((2, 7)); trg = rng.random((2, 5)) + 0.01
    q = rng.standard_normal(7)
    beta = 2.7
    pot, grad = oracle.free_space("yukawa", src, q, trg, beta=beta)
    r = trg[:, :, None] - src[:, None, :]
    rr = np.hypot(r[0], r[1])
    ref = (sp.k0(beta * rr) @ q) / (2 * np.pi)
    gref = -(beta / (2 * np.pi)) * np.einsum("tj,ktj->kt", sp.k1(beta * rr) / rr * q, r)
    assert rel(pot, ref) < 1e-14 and rel(grad, gref) < 1e-14


def test_free_space_laplace_and_stokes_match_numpy():
    rng = np.random.default_rng(4)
    src = rng.random((2, 6)); trg = rng.random((2, 4)) + 0.02
    q = rng.standard_normal(6); f = rng.standard_normal((2, 6))
    r = trg[:, :, None] - src[:, None, :]
    r2 = r[0] ** 2 + r[1] ** 2
    pot, grad = oracle.free_space("laplace", src, q, trg)
    assert rel(pot, -(np.log(np.sqrt(r2)) @ q) / (2 * np.pi)) < 1e-14
    assert rel(grad, -np.einsum("ktj,j->kt", r / r2, q) / (2 * np.pi)) < 1e-14
    vel, _ = oracle.free_space("stokes", src, f, trg)
    rf = np.einsum("ktj,kj->tj", r, f)
    u = (-np.log(np.sqrt(r2))[None] * f[:, None, :] + rf[None] * r / r2[None]).sum(-1) / (4 * np.pi)
    assert rel(vel, u) < 1e-14


# --- Laplace ------------------------------------------------------------------

@pytest.mark.parametrize("e1,e2", [SHEARED, GENERAL])
@pytest.mark.parametrize("self_trg", [False, True])
def test_laplace_ewald_independent_of_split(e1, e2, self_trg):
    src, q, trg = _setup(e1, e2)
    trg = None if self_trg else trg
    base = oracle.laplace(e1, e2, src, q, trg, alpha=2.0)
    for a in (1.2, 3.5, 7.0):
        p, g = oracle.laplace(e1, e2, src, q, trg, alpha=a)
        assert rel(p, base[0]) < 1e-12 and rel(g, base[1]) < 1e-12


@pytest.mark.parametrize("self_trg", [False, True])
def test_laplace_ewald_equals_row_sum_formula(self_trg):
    (d, _), (xi, eta) = SHEARED
    src, q, trg = _setup(*SHEARED, ns=15, nt=11)
    trg = None if self_trg else trg
    p1, g1 = oracle.laplace(*SHEARED, src, q, trg)
    p2, g2 = oracle.laplace_rowsum(d, xi, eta, src, q, trg)
    assert rel(p1, p2) < 1e-12 and rel(g1, g2) < 1e-12


def test_laplace_row_sum_high_aspect_matches_ewald():
    e1, e2 = (20.0, 0.0), (3.0, 1.0)
    src, q, trg = _setup(e1, e2, ns=10, nt=6, seed=5)
    p1, g1 = oracle.laplace(e1, e2, src, q, trg)
    p2, g2 = oracle.laplace_rowsum(20.0, 3.0, 1.0, src, q, trg)
    assert rel(p1, p2) < 1e-11 and rel(g1, g2) < 1e-11


def test_laplace_periodic_across_both_lattice_vectors():
    # Row-sum formula on targets of the bottom edge and the same targets
    # moved by e2 (top edge), and left/right edges: the periodicity
    # requirement (Sec. 1 eq. pbc).
    (d, _), (xi, eta) = SHEARED
    src, q, _ = _setup(*SHEARED, ns=10)
    s = np.linspace(-0.5, 0.5, 13)
    bottom = np.stack([s * d - 0.5 * xi, np.full_like(s, -0.5 * eta)])
    top = bottom + np.array([[xi], [eta]])
    pb, gb = oracle.laplace_rowsum(d, xi, eta, src, q, bottom)
    pt, gt = oracle.laplace_rowsum(d, xi, eta, src, q, top)
    assert rel(pt, pb) < 1e-12 and rel(gt, gb) < 1e-12
    left = np.stack([-0.5 * d + s * xi, s * eta])
    right = left + np.array([[d], [0.0]])
    pl, gl = oracle.laplace_rowsum(d, xi, eta, src, q, left)
    pr, gr = oracle.laplace_rowsum(d, xi, eta, src, q, right)
    assert rel(pr, pl) < 1e-12 and rel(gr, gl) < 1e-12


def test_laplace_cell_mean_is_zero():
    # midpoint rule over the cell (sources kept off the grid points); the
    # log singularities limit this to a few digits.
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    src = np.array([[0.1037, -0.2519, 0.3311], [0.2203, -0.1107, -0.3391]])
    q = np.array([1.0, -0.4, -0.6])
    n = 160
    g = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(g, g)
    p, _ = oracle.laplace(e1, e2, src, q, np.stack([X.ravel(), Y.ravel()]), tol=1e-10)
    assert abs(p.mean()) < 2e-3 * np.abs(p).mean()


def test_laplace_gradient_is_derivative_of_potential():
    src, q, trg = _setup(*GENERAL, ns=8, nt=4)
    _, g = oracle.laplace(*GENERAL, src, q, trg)
    h = 1e-5
    for k in range(2):
        dp = np.zeros((2, 1)); dp[k] = h
        fd = (oracle.laplace(*GENERAL, src, q, trg + dp)[0] - oracle.laplace(*GENERAL, src, q, trg - dp)[0]) / (2 * h)
        assert rel(g[k], fd) < 1e-6


def test_laplace_tight_dipole_reduces_to_free_space():
    # A +-q pair of separation delta in a unit cell: near the pair the
    # images add a field of relative size O(delta).
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    delta = 1e-4
    src = np.array([[0.0, delta], [0.0, 0.0]])
    q = np.array([1.0, -1.0])
    trg = np.array([[0.5 * delta, 2 * delta, -delta], [delta, -delta, 0.5 * delta]])
    p, g = oracle.laplace(e1, e2, src, q, trg)
    pf, gf = oracle.free_space("laplace", src, q, trg)
    assert np.max(np.abs(p - pf)) < 10 * delta and rel(g, gf) < 10 * delta


# --- Yukawa -------------------------------------------------------------------

def test_yukawa_lattice_sum_converged_in_truncation():
    src, q, trg = _setup(*SHEARED)
    p1, g1 = oracle.yukawa(*SHEARED, 1.5, src, q, trg, tol=1e-9)
    p2, g2 = oracle.yukawa(*SHEARED, 1.5, src, q, trg, tol=1e-16)
    assert rel(p1, p2) < 1e-7 and rel(g1, g2) < 1e-7


def test_yukawa_large_beta_is_free_space():
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    rng = np.random.default_rng(6)
    src = 0.2 * (rng.random((2, 6)) - 0.5)      # well inside the cell
    trg = 0.2 * (rng.random((2, 4)) - 0.5)
    q = rng.standard_normal(6)
    beta = 60.0      # nearest image >= 0.8 away: K0(48) ~ 1e-22
    p, g = oracle.yukawa(e1, e2, beta, src, q, trg)
    pf, gf = oracle.free_space("yukawa", src, q, trg, beta=beta)
    assert rel(p, pf) < 1e-13 and rel(g, gf) < 1e-13


def test_yukawa_tends_to_laplace_quadratically_in_beta():
    # neutral charges: the periodic symbols 1/(k^2+beta^2) and 1/k^2 differ by O(beta^2)
    src, q, trg = _setup(*SHEARED, ns=6, nt=4, seed=7)
    pl, gl = oracle.laplace(*SHEARED, src, q, trg)
    errs = []
    for beta in (0.4, 0.2):
        p, g = oracle.yukawa(*SHEARED, beta, src, q, trg, tol=1e-13)
        errs.append(np.linalg.norm(p - pl) + np.linalg.norm(g - gl))
    ratio = errs[0] / errs[1]
    assert 3.3 < ratio < 4.7, ratio
    assert errs[1] < 0.05 * (np.linalg.norm(pl) + np.linalg.norm(gl))


def _yukawa_row_spectral(d, e2, beta, src, q, trg, nrow=40, nk=300):
    """Periodic Yukawa field for e1 = (d, 0) by Poisson summation along each
    row of images: the 1D Fourier transform of K0(beta sqrt(x^2 + Y^2)) / (2 pi)
    is exp(-|Y| s) / (2 s) with s = sqrt(k^2 + beta^2), so a row of images
    offset by Y sums to (1/d) sum_k exp(-|Y| s_k) cos(k X) / (2 s_k),
    k = 2 pi j / d. Converges exponentially when every row offset is away
    from zero; no Bessel function and no image cut-off of the oracle's."""
    xi, eta = e2
    pot = np.zeros(trg.shape[1]); grad = np.zeros((2, trg.shape[1]))
    k = 2 * np.pi * np.arange(-nk, nk + 1) / d
    s = np.sqrt(k * k + beta * beta)
    for n in range(-nrow, nrow + 1):
        X = trg[0][:, None] - src[0][None, :] + n * xi
        Y = trg[1][:, None] - src[1][None, :] + n * eta
        e = np.exp(-np.abs(Y)[..., None] * s) / (2 * s * d)
        ph = k * X[..., None]
        pot += (np.cos(ph) * e).sum(-1) @ q
        grad[0] += (-k * np.sin(ph) * e).sum(-1) @ q
        grad[1] += (-np.sign(Y)[..., None] * s * np.cos(ph) * e).sum(-1) @ q
    return pot, grad


@pytest.mark.parametrize("e1,e2", [SHEARED, GENERAL])
@pytest.mark.parametrize("beta", [1.5, 4.0])
def test_yukawa_equals_row_spectral_sum(e1, e2, beta):
    # Work in the frame where e1 lies on the x axis; sources and targets sit
    # in separate horizontal bands so that no row offset comes near zero.
    th = np.arctan2(e1[1], e1[0])
    R = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]])   # rotates e1 onto +x
    d = np.hypot(*e1)
    e2r = R @ np.asarray(e2)
    eta = e2r[1]
    rng = np.random.default_rng(11)
    ns, nt = 12, 9
    src_r = np.vstack([rng.uniform(-d / 2, d / 2, ns), rng.uniform(-0.45, -0.25, ns) * eta])
    trg_r = np.vstack([rng.uniform(-d / 2, d / 2, nt), rng.uniform(0.05, 0.25, nt) * eta])
    q = rng.standard_normal(ns)
    p, g = oracle.yukawa(e1, e2, beta, R.T @ src_r, q, R.T @ trg_r)
    ps, gs = _yukawa_row_spectral(d, e2r, beta, src_r, q, trg_r)
    assert np.abs(p - ps).max() < 1e-12 * np.abs(ps).max()
    assert np.abs(R @ g - gs).max() < 1e-12 * np.abs(gs).max()


# --- Stokes -------------------------------------------------------------------

def _stokes_row_spectral(d, e2, src, f, trg, nrow=40, nk=300):
    """Zero-mean periodic Stokeslet velocity and gradient for e1 = (d, 0),
    from the Fourier symbol T(k) = (I - k k^T / k^2) / k^2 summed over the
    reciprocal lattice with k = 0 left out. Reciprocal vectors with
    k_x = 2 pi j / d != 0 are summed over k_y by Poisson summation, which
    turns them into rows of images offset by n e2 with the 1D transforms
      int e^{i k_y Y} / k^2   dk_y / 2pi = e^{-a|Y|} / (2a)
      int e^{i k_y Y} / k^4   dk_y / 2pi = (1 + a|Y|) e^{-a|Y|} / (4a^3),  a = |k_x|;
    those with k_x = 0 are k = (0, 2 pi l / eta), where T = diag(1/k_y^2, 0)
    sums to (eta / 2d) B2(t) with B2(t) = t^2 - t + 1/6, t = Y/eta mod 1.
    No Ewald split, no exponential integral, no real-space image sum."""
    xi, eta = e2
    nt = trg.shape[1]
    u = np.zeros((2, nt)); g = np.zeros((4, nt))     # g: du1/dx, du1/dy, du2/dx, du2/dy
    a = 2 * np.pi * np.arange(1, nk + 1) / d          # k_x > 0; -k_x is folded in (factor 2)
    fx = f[0][None, :]; fy = f[1][None, :]

    def add(out, kxx, kxy, kyy):                      # out += sum_src [[xx, xy], [xy, yy]] f
        out[0] += (kxx.sum(-1) * fx + kxy.sum(-1) * fy).sum(1) / d
        out[1] += (kxy.sum(-1) * fx + kyy.sum(-1) * fy).sum(1) / d

    for n in range(-nrow, nrow + 1):
        X = (trg[0][:, None] - src[0][None, :] + n * xi)[..., None]
        Y = (trg[1][:, None] - src[1][None, :] + n * eta)[..., None]
        y = np.abs(Y); s = np.sign(Y); E = np.exp(-a * y)
        F1, dF1 = E / (2 * a), -s * E / 2                                  # 1/k^2 and d/dY
        G0, dG0 = (1 + a * y) * E / (4 * a), -a * Y * E / 4                # k_x^2 / k^4 and d/dY
        G1, dG1 = -Y * E / (4 * a), -(1 - a * y) * E / (4 * a)             # d/dY of 1/k^4, and next
        dG2 = s * (2 - a * y) * E / 4                                      # third derivative of 1/k^4
        Txx, Tyy, dTxx, dTyy = F1 - G0, F1 + dG1, dF1 - dG0, dF1 + dG2
        c = np.cos(a * X); sn = np.sin(a * X)
        vel = np.zeros((2, nt)); gx = np.zeros((2, nt)); gy = np.zeros((2, nt))
        add(vel, 2 * c * Txx, -2 * a * G1 * sn, 2 * c * Tyy)
        add(gx, -2 * a * sn * Txx, -2 * a * a * G1 * c, -2 * a * sn * Tyy)
        add(gy, 2 * c * dTxx, -2 * a * dG1 * sn, 2 * c * dTyy)
        u += vel; g[0] += gx[0]; g[2] += gx[1]; g[1] += gy[0]; g[3] += gy[1]
    t = np.mod((trg[1][:, None] - src[1][None, :]) / eta, 1.0)
    u[0] += ((eta / (2 * d)) * (t * t - t + 1.0 / 6.0) * fx).sum(1)
    g[1] += (((2 * t - 1) / (2 * d)) * fx).sum(1)
    return u, g


@pytest.mark.parametrize("e1,e2", [SHEARED, GENERAL, ((1.0, 0.0), (0.0, 1.0))])
def test_stokes_equals_spectral_row_sum(e1, e2):
    # also fixes the additive constant: the oracle's velocity has zero cell mean
    th = np.arctan2(e1[1], e1[0])
    R = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]])   # rotates e1 onto +x
    d = np.hypot(*e1)
    e2r = R @ np.asarray(e2)
    eta = e2r[1]
    rng = np.random.default_rng(11)
    ns, nt = 12, 9
    src_r = np.vstack([rng.uniform(-d / 2, d / 2, ns), rng.uniform(-0.45, -0.25, ns) * eta])
    trg_r = np.vstack([rng.uniform(-d / 2, d / 2, nt), rng.uniform(0.05, 0.25, nt) * eta])
    f_r = rng.standard_normal((2, ns))
    f_r -= f_r.mean(1, keepdims=True)
    u, g = oracle.stokes(e1, e2, R.T @ src_r, R.T @ f_r, R.T @ trg_r)
    us, gs = _stokes_row_spectral(d, e2r, src_r, f_r, trg_r)
    gr = np.einsum("ij,jkt,lk->ilt", R, g.reshape(2, 2, nt), R).reshape(4, nt)
    assert np.abs(R @ u - us).max() < 1e-12 * np.abs(us).max()
    assert np.abs(gr - gs).max() < 1e-12 * np.abs(gs).max()


@pytest.mark.parametrize("self_trg", [False, True])
def test_stokes_ewald_independent_of_split(self_trg):
    src, f, trg = _setup(*GENERAL, stokes=True)
    trg = None if self_trg else trg
    u0, g0 = oracle.stokes(*GENERAL, src, f, trg, alpha=2.0)
    for a in (1.3, 4.0, 7.5):
        u, g = oracle.stokes(*GENERAL, src, f, trg, alpha=a)
        assert rel(u, u0) < 1e-12 and rel(g, g0) < 1e-12


def test_stokes_trace_is_laplace():
    # tr G_stokeslet = -(1/2pi) log r + const, and the periodic symbols obey
    # tr (I - k k^T/k^2)/k^2 = 1/k^2: u1[f=(q,0)] + u2[f=(0,q)] = Laplace[q].
    src, q, trg = _setup(*SHEARED, ns=10, nt=7, seed=8)
    z = np.zeros_like(q)
    ua, ga = oracle.stokes(*SHEARED, src, np.stack([q, z]), trg)
    ub, gb = oracle.stokes(*SHEARED, src, np.stack([z, q]), trg)
    pl, gl = oracle.laplace(*SHEARED, src, q, trg)
    assert rel(ua[0] + ub[1], pl) < 1e-12
    assert rel(np.stack([ga[0] + gb[2], ga[1] + gb[3]]), gl) < 1e-12


@pytest.mark.parametrize("e1,e2", [SHEARED, GENERAL])
def test_stokes_trace_is_laplace_at_the_sources(e1, e2):
    # the self-excluded sums: tr G_stokeslet(r) = G_laplace(r) + 1/(4 pi), so
    # with the (j = i, zero shift) term left out on both sides the traces
    # differ by the left-out constant, -q_i/(4 pi). The velocity gradient
    # has no such constant. An error in the alpha-independent part of the
    # Stokes self term (Sec. 5.2 eq. stokeslet at r -> 0) fails this.
    rng = np.random.default_rng(31)
    n = 11
    src = W.cell_points(rng, e1, e2, n)
    q = W.neutral_charges(rng, n)
    z = np.zeros_like(q)
    ua, ga = oracle.stokes(e1, e2, src, np.stack([q, z]), None)
    ub, gb = oracle.stokes(e1, e2, src, np.stack([z, q]), None)
    pl, gl = oracle.laplace(e1, e2, src, q, None)
    assert np.abs(ua[0] + ub[1] - (pl - q / (4 * np.pi))).max() < 1e-12 * np.abs(pl).max()
    assert rel(np.stack([ga[0] + gb[2], ga[1] + gb[3]]), gl) < 1e-12


def test_stokes_self_term_is_the_limit_at_the_source():
    # u_self(x_i) = lim_{h -> 0} [u(x_i + h) - G_stokeslet(h) f_i]: the
    # oracle's self term against its own sums at nearby non-self targets
    # (which never use the self constant). Averaging over +-h along x and
    # along y cancels the O(h) gradient term, leaving O(h^2).
    rng = np.random.default_rng(32)
    n = 9
    src = W.cell_points(rng, *SHEARED, n)
    f = W.neutral_forces(rng, n)
    i = 4
    u_self, _ = oracle.stokes(*SHEARED, src, f, None)
    for h in (1e-4, 1e-5, 1e-6):
        acc = np.zeros(2)
        for dv in ((h, 0.0), (-h, 0.0), (0.0, h), (0.0, -h)):
            t = src[:, [i]] + np.array(dv)[:, None]
            u, _ = oracle.stokes(*SHEARED, src, f, t)
            r2 = dv[0] ** 2 + dv[1] ** 2
            G = (-0.5 * np.log(r2) * np.eye(2) + np.outer(dv, dv) / r2) / (4 * np.pi)
            acc += u[:, 0] - G @ f[:, i]
        acc /= 4
        assert np.abs(acc - u_self[:, i]).max() < 1e-9 * np.abs(u_self).max() + 50 * h * h, (h, acc, u_self[:, i])


def test_stokes_divergence_free_and_gradient_consistent():
    src, f, trg = _setup(*SHEARED, ns=9, nt=5, seed=9, stokes=True)
    u, g = oracle.stokes(*SHEARED, src, f, trg)
    assert np.max(np.abs(g[0] + g[3])) < 1e-12 * np.max(np.abs(g))
    h = 1e-5
    for k in range(2):
        dp = np.zeros((2, 1)); dp[k] = h
        fd = (oracle.stokes(*SHEARED, src, f, trg + dp)[0] - oracle.stokes(*SHEARED, src, f, trg - dp)[0]) / (2 * h)
        assert rel(np.stack([g[k], g[2 + k]]), fd) < 1e-6


def test_stokes_periodic_and_tight_pair_free_space():
    src, f, _ = _setup(*SHEARED, ns=8, seed=10, stokes=True)
    t = np.array([[0.13, -0.61], [0.27, 0.05]])
    u0, g0 = oracle.stokes(*SHEARED, src, f, t)
    for sh in (SHEARED[0], SHEARED[1]):
        u1, g1 = oracle.stokes(*SHEARED, src, f, t + np.array(sh)[:, None])
        assert rel(u1, u0) < 1e-12 and rel(g1, g0) < 1e-12
    delta = 1e-4
    src = np.array([[0.0, delta], [0.0, 0.0]])
    f = np.array([[1.0, -1.0], [0.5, -0.5]])
    trg = np.array([[0.5 * delta, 2 * delta], [delta, -delta]])
    u, g = oracle.stokes((1.0, 0.0), (0.0, 1.0), src, f, trg)
    uf, gf = oracle.free_space("stokes", src, f, trg)
    assert np.max(np.abs(u - uf)) < 10 * delta and rel(g, gf) < 10 * delta


# --- reciprocity (self targets) ---------------------------------------------

@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 2.5), ("stokes", 0.0)])
def test_reciprocity_at_the_sources(kernel, beta):
    # the periodic kernel is symmetric, G(x_i - x_j) = G(x_j - x_i), so with
    # targets = sources sum_i g_i . u[q](x_i) = sum_j q_j . u[g](x_j); an image
    # set or reciprocal-space sum that is not symmetric under l -> -l breaks
    # it (the self term is diagonal and is pinned by the split independence)
    rng = np.random.default_rng(23)
    n = 14
    src = W.cell_points(rng, *GENERAL, n)
    if kernel == "stokes":
        q, g = W.neutral_forces(rng, n), W.neutral_forces(rng, n)
    else:
        q, g = W.neutral_charges(rng, n), W.neutral_charges(rng, n)
    uq, _ = oracle.evaluate(kernel, *GENERAL, src, q, None, beta=beta)
    ug, _ = oracle.evaluate(kernel, *GENERAL, src, g, None, beta=beta)
    a, b = np.sum(g * uq), np.sum(q * ug)
    assert abs(a - b) < 1e-12 * (abs(a) + abs(b)), (a, b)


# --- singly periodic sums (P1, periodic in e1 only) --------------------------

P1_E1 = (1.3, 0.4)          # period vector, not along x


def _p1_points(n, nt, seed, stokes=False, height=2.0):
    rng = np.random.default_rng(seed)
    e1 = np.array(P1_E1)
    d = np.hypot(*e1)
    perp = np.array([-e1[1], e1[0]]) / d
    u = rng.random(n) - 0.5; v = (rng.random(n) - 0.5) * height
    src = np.outer(e1, u) + np.outer(perp, v)
    ut = rng.random(nt) - 0.5; vt = (rng.random(nt) - 0.5) * height
    trg = np.outer(e1, ut) + np.outer(perp, vt)
    dens = W.neutral_forces(rng, n) if stokes else W.neutral_charges(rng, n)
    return src, dens, trg


def _p1_brute(kernel, src, dens, trg, beta=0.0, M0=64, levels=5):
    """Symmetric partial sums over |m| <= M of the free-space kernel over the
    images s_j + m e1, for M = M0 2^k, extrapolated to M -> infinity by fitting
    a polynomial in 1/M through all levels (the neutral sums' tails have an
    expansion in powers of 1/M); Yukawa needs no extrapolation."""
    e1 = np.array(P1_E1)
    vals = []
    Ms = [M0 * 2 ** k for k in range(levels)]
    for M in Ms:
        m = np.arange(-M, M + 1)
        s_img = (src[:, None, :] + np.outer(e1, m)[:, :, None]).reshape(2, -1)
        d_img = np.repeat(dens[..., None, :], len(m), axis=-2).reshape(dens.shape[:-1] + (-1,))
        p, g = oracle.free_space(kernel, s_img, d_img, trg, beta=beta)
        vals.append(np.concatenate([np.ravel(p), np.ravel(g)]))
        if kernel == "yukawa":
            return vals[-1]
    h = 1.0 / np.array(Ms, float)
    V = np.vander(h, levels, increasing=True)
    coef = np.linalg.solve(V, np.array(vals))
    return coef[0]


@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
def test_p1_closed_forms_equal_extrapolated_direct_sums(kernel):
    # the sine-product (Laplace) and complex cotangent (Stokes) forms of the
    # symmetric image sums against brute force over up to 2 x 1024 images
    src, dens, trg = _p1_points(7, 5, seed=41, stokes=kernel == "stokes")
    p, g = oracle.singly_periodic(kernel, P1_E1, src, dens, trg)
    ref = _p1_brute(kernel, src, dens, trg)
    got = np.concatenate([np.ravel(p), np.ravel(g)])
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max(), np.abs(got - ref).max()


def test_p1_yukawa_equals_direct_sum_and_row_spectral_sum():
    beta = 1.7
    src, q, trg = _p1_points(8, 6, seed=42)
    p, g = oracle.singly_periodic("yukawa", P1_E1, src, q, trg, beta=beta)
    ref = _p1_brute("yukawa", src, q, trg, beta=beta, M0=80, levels=1)
    got = np.concatenate([p, np.ravel(g)])
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    # one row of the Poisson-summation form (no Bessel function), in the frame
    # where the period lies along x
    e1 = np.array(P1_E1); d = np.hypot(*e1)
    R = np.array([[e1[0], e1[1]], [-e1[1], e1[0]]]) / d
    ps, gs = _yukawa_row_spectral(d, (0.0, 1e6), beta, R @ src, q, R @ trg, nrow=0, nk=600)
    assert rel(p, ps) < 1e-12 and rel(g, R.T @ gs) < 1e-12


def test_p1_stokes_trace_is_laplace_and_divergence_free():
    src, q, trg = _p1_points(9, 7, seed=43)
    lp, lg = oracle.singly_periodic("laplace", P1_E1, src, q, trg)
    ua, ga = oracle.singly_periodic("stokes", P1_E1, src, np.stack([q, 0 * q]), trg)
    ub, gb = oracle.singly_periodic("stokes", P1_E1, src, np.stack([0 * q, q]), trg)
    # trace of the Stokeslet = Laplace kernel + 1/(4 pi); the constant drops for neutral q
    assert rel(ua[0] + ub[1], lp) < 1e-13
    assert rel(ga[0:2] + gb[2:4], lg) < 1e-13
    src, f, trg = _p1_points(9, 7, seed=44, stokes=True)
    u, g = oracle.singly_periodic("stokes", P1_E1, src, f, trg)
    assert np.abs(g[0] + g[3]).max() < 1e-12 * np.abs(g).max()


@pytest.mark.parametrize("kernel,beta", [("laplace", 0.0), ("yukawa", 2.0), ("stokes", 0.0)])
def test_p1_periodic_along_e1_and_gradient_is_derivative(kernel, beta):
    src, dens, trg = _p1_points(8, 5, seed=45, stokes=kernel == "stokes")
    e1 = np.array(P1_E1)[:, None]
    p0, g0 = oracle.singly_periodic(kernel, P1_E1, src, dens, trg, beta=beta)
    p1, g1 = oracle.singly_periodic(kernel, P1_E1, src, dens, trg + 3 * e1, beta=beta)
    assert rel(p1, p0) < 1e-12 and rel(g1, g0) < 1e-12
    h = 1e-6
    for c in range(2):
        dv = np.zeros((2, 1)); dv[c] = h
        pp, _ = oracle.singly_periodic(kernel, P1_E1, src, dens, trg + dv, beta=beta)
        pm, _ = oracle.singly_periodic(kernel, P1_E1, src, dens, trg - dv, beta=beta)
        fd = (pp - pm) / (2 * h)
        an = g0[c::2] if kernel == "stokes" else g0[c]
        assert rel(an, fd) < 1e-7, (c, rel(an, fd))


@pytest.mark.parametrize("kernel", ["laplace", "stokes"])
def test_p1_self_term_is_the_limit_at_the_source(kernel):
    # value at a source with its own m = 0 term left out = lim_{h->0} of the
    # full sum at x_i + h minus the free-space kernel at h
    src, dens, _ = _p1_points(7, 1, seed=46, stokes=kernel == "stokes")
    i = 3
    u_self, _ = oracle.singly_periodic(kernel, P1_E1, src, dens, None)
    for h in (1e-4, 1e-5):
        acc = 0
        for dv in ((h, 0.0), (-h, 0.0), (0.0, h), (0.0, -h)):
            t = src[:, [i]] + np.array(dv)[:, None]
            u, _ = oracle.singly_periodic(kernel, P1_E1, src, dens, t)
            r2 = dv[0] ** 2 + dv[1] ** 2
            if kernel == "stokes":
                G = (-0.5 * np.log(r2) * np.eye(2) + np.outer(dv, dv) / r2) / (4 * np.pi)
                acc = acc + (u[:, 0] - G @ dens[:, i])
            else:
                acc = acc + (u[0] + 0.25 * np.log(r2) / np.pi * dens[i])
        acc = acc / 4
        ref = u_self[:, i] if kernel == "stokes" else u_self[i]
        assert np.abs(acc - ref).max() < 1e-8 * np.abs(u_self).max() + 50 * h * h, (h, acc, ref)


def test_p1_yukawa_tends_to_laplace():
    # neutral charges: the row sum of K0(beta r)/(2 pi) differs from the
    # Laplace one by O(beta) (its zero mode is (1/(2 beta d)) e^{-beta |y|})
    src, q, trg = _p1_points(8, 6, seed=47)
    lp, lg = oracle.singly_periodic("laplace", P1_E1, src, q, trg)
    errs = []
    for beta in (1e-2, 5e-3):
        yp, yg = oracle.singly_periodic("yukawa", P1_E1, src, q, trg, beta=beta, tol=1e-15)
        errs.append(rel(yp, lp))
    assert errs[0] < 0.05 and 1.6 < errs[0] / errs[1] < 2.4, errs


# --- Stokes pressure ----------------------------------------------------------

@pytest.mark.parametrize("periodic", [2, 1])
def test_stokes_pressure_satisfies_the_momentum_equation(periodic):
    # away from the forces the Stokes equations (mu = 1) give grad p = lap u;
    # the velocity comes from the Stokes oracle (Ewald, or the singly periodic
    # closed form), the pressure from the Laplace one: central differences
    # of the analytic velocity gradient against differences of the pressure
    rng = np.random.default_rng(61)
    if periodic == 2:
        e1, e2 = SHEARED
        src, f, trg = _setup(e1, e2, ns=10, nt=6, seed=62, stokes=True)
        vel = lambda t: oracle.stokes(e1, e2, src, f, t)
    else:
        e1, e2 = P1_E1, None
        src, f, trg = _p1_points(10, 6, seed=62, stokes=True)
        vel = lambda t: oracle.singly_periodic("stokes", e1, src, f, t)
    pres = lambda t: oracle.stokes_pressure(e1, e2, src, f, t, periodic=periodic)
    h = 2e-4

    def d4(fun, k):
        # fourth-order central difference along x_k
        dv = np.zeros((2, 1)); dv[k] = h
        return (8 * (fun(trg + dv) - fun(trg - dv)) - (fun(trg + 2 * dv) - fun(trg - 2 * dv))) / (12 * h)
    lap_u = np.zeros((2, trg.shape[1])); grad_p = np.zeros((2, trg.shape[1]))
    for k in range(2):
        dj = d4(lambda t: vel(t)[1], k)
        # d/dx_k of du_i/dx_k (gradient rows: du1/dx, du1/dy, du2/dx, du2/dy)
        lap_u[0] += dj[k]
        lap_u[1] += dj[2 + k]
        grad_p[k] = d4(pres, k)
    assert rel(grad_p, lap_u) < 1e-7, rel(grad_p, lap_u)


def test_stokes_pressure_of_a_tight_pair_is_free_space():
    # a force dipole much smaller than the cell: the periodic pressure near it
    # is the free-space pressurelet sum (1/2pi) r.f/r^2 up to the images' smooth part
    e1, e2 = SHEARED
    c = np.array([[0.1], [0.05]])
    src = c + 1e-3 * np.array([[1.0, -1.0], [0.5, -0.5]])
    f = np.array([[1.0, -1.0], [-0.3, 0.3]])
    trg = c + np.array([[0.02, -0.015, 0.0], [0.01, 0.02, -0.025]])
    p = oracle.stokes_pressure(e1, e2, src, f, trg)
    r = trg[:, :, None] - src[:, None, :]
    ref = (np.einsum("ktj,kj->tj", r, f) / (r[0] ** 2 + r[1] ** 2)).sum(1) / (2 * np.pi)
    assert rel(p, ref) < 1e-3


# --- modified Stokeslet (Sec. 5, eq. msgreen) --------------------------------

def _g_mb(beta, x, y):
    # G_MB = -(K0(beta r) + log r)/(2 pi beta^2), the paper's modified
    # biharmonic Green's function, from scipy
    r = np.hypot(x, y)
    return -(sp.k0(beta * r) + np.log(r)) / (2 * np.pi * beta ** 2)


def test_free_space_mstokes_is_the_operator_on_g_mb():
    # the oracle's free-space modified Stokeslet against the operator
    # [[-d_yy, d_xy], [d_xy, -d_xx]] applied to G_MB by fourth-order differences
    rng = np.random.default_rng(40)
    beta = 2.5
    src = rng.uniform(-0.5, 0.5, (2, 3))
    f = rng.standard_normal((2, 3))
    trg = rng.uniform(-0.5, 0.5, (2, 4)) + np.array([[1.5], [0.0]])
    u, g = oracle.free_space("mstokes", src, f, trg, beta=beta)
    h = 2e-3
    w = {-2: 1 / 12, -1: -2 / 3, 1: 2 / 3, 2: -1 / 12}

    def d(fun, kx, ky):
        # fourth-order difference: kx, ky derivative orders (0..2 in sum)
        if kx == 2 or ky == 2:
            c = {-2: -1 / 12, -1: 4 / 3, 0: -5 / 2, 1: 4 / 3, 2: -1 / 12}
            return lambda x, y: sum(c[a] * (fun(x + a * h, y) if kx == 2 else fun(x, y + a * h))
                                    for a in c) / h ** 2
        if kx == 1 and ky == 1:
            return lambda x, y: sum(w[a] * w[b] * fun(x + a * h, y + b * h) for a in w for b in w) / h ** 2
        raise ValueError

    ref = np.zeros((2, trg.shape[1]))
    for j in range(3):
        x = trg[0] - src[0, j]; y = trg[1] - src[1, j]
        gm = lambda x, y: _g_mb(beta, x, y)
        gxx, gyy, gxy = d(gm, 2, 0)(x, y), d(gm, 0, 2)(x, y), d(gm, 1, 1)(x, y)
        ref[0] += -gyy * f[0, j] + gxy * f[1, j]
        ref[1] += gxy * f[0, j] - gxx * f[1, j]
    assert rel(u, ref) < 1e-7
    # gradient of the free-space velocity by differences
    for k in range(2):
        dp = np.zeros((2, 1)); dp[k] = 1e-5
        fd = (oracle.free_space("mstokes", src, f, trg + dp, beta=beta)[0]
              - oracle.free_space("mstokes", src, f, trg - dp, beta=beta)[0]) / 2e-5
        assert rel(np.stack([g[k], g[2 + k]]), fd) < 1e-7


@pytest.mark.parametrize("self_trg", [False, True])
def test_mstokes_independent_of_split(self_trg):
    rng = np.random.default_rng(41)
    src = W.cell_points(rng, *GENERAL, 8)
    trg = None if self_trg else W.cell_points(rng, *GENERAL, 6)
    f = rng.standard_normal((2, 8))          # net force allowed
    a = oracle.mstokes(*GENERAL, 3.0, src, f, trg, alpha=2.5)
    b = oracle.mstokes(*GENERAL, 3.0, src, f, trg, alpha=8.0)
    assert rel(a[0], b[0]) < 1e-12 and rel(a[1], b[1]) < 1e-12


def test_mstokes_periodic_divergence_free_and_gradient_is_derivative():
    rng = np.random.default_rng(42)
    src = W.cell_points(rng, *SHEARED, 7)
    trg = W.cell_points(rng, *SHEARED, 5)
    f = rng.standard_normal((2, 7))
    u, g = oracle.mstokes(*SHEARED, 1.7, src, f, trg)
    for sh in SHEARED:
        u1, g1 = oracle.mstokes(*SHEARED, 1.7, src, f, trg + np.array(sh)[:, None])
        assert rel(u1, u) < 1e-12 and rel(g1, g) < 1e-12
    assert np.max(np.abs(g[0] + g[3])) < 1e-12 * np.max(np.abs(g))
    h = 1e-5
    for k in range(2):
        dp = np.zeros((2, 1)); dp[k] = h
        fd = (oracle.mstokes(*SHEARED, 1.7, src, f, trg + dp)[0]
              - oracle.mstokes(*SHEARED, 1.7, src, f, trg - dp)[0]) / (2 * h)
        assert rel(np.stack([g[k], g[2 + k]]), fd) < 1e-6


def test_mstokes_tends_to_stokes_quadratically_in_beta():
    # zero net force: the symbol (I - k k^T/k^2)/(beta^2 + k^2) differs from
    # the Stokes one by O(beta^2) summably, so the error falls by 4 when beta halves
    src, f, trg = _setup(*SHEARED, ns=7, nt=5, seed=43, stokes=True)
    us, gs = oracle.stokes(*SHEARED, src, f, trg)
    err = []
    for beta in (0.5, 0.25):
        u, g = oracle.mstokes(*SHEARED, beta, src, f, trg)
        err.append((rel(u, us), rel(g, gs)))
    for c in range(2):
        assert 3.5 < err[0][c] / err[1][c] < 4.5, err
    assert max(err[1]) < 1e-2, err


def test_mstokes_large_beta_is_the_laplace_hessian():
    # away from the sources beta^2 u -> Hess(G_L^per) f: the screened part
    # dies like K0(beta r); Hess by differences of the Laplace oracle's gradient
    rng = np.random.default_rng(44)
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    src = np.array([[-0.3, 0.2, 0.1], [0.25, -0.2, 0.3]])
    f = W.neutral_forces(rng, 3)
    trg = np.array([[0.45, -0.4], [-0.3, -0.45]])      # >= 0.25 from every source image
    beta = 160.0
    u, _ = oracle.mstokes(e1, e2, beta, src, f, trg)
    h = 1e-4
    ref = np.zeros((2, 2))
    for j in range(2):
        dp = np.zeros((2, 1)); dp[j] = h
        gp = oracle.laplace(e1, e2, src, f[j], trg + dp)[1]
        gm = oracle.laplace(e1, e2, src, f[j], trg - dp)[1]
        gp2 = oracle.laplace(e1, e2, src, f[j], trg + 2 * dp)[1]
        gm2 = oracle.laplace(e1, e2, src, f[j], trg - 2 * dp)[1]
        ref += (8 * (gp - gm) - (gp2 - gm2)) / (12 * h)   # d_j grad_i phi[f_j]
    assert rel(beta ** 2 * u, ref) < 1e-8


def test_mstokes_cell_mean_is_net_force_over_beta2_area():
    # integrating (beta^2 - Lap) u + grad p = f over the cell: beta^2 |C| mean(u) = F
    # (periodic u and p); midpoint rule over the cell in lattice coordinates
    rng = np.random.default_rng(45)
    e1, e2 = (1.0, 0.0), (0.35, 0.9)
    src = W.cell_points(rng, e1, e2, 3)
    f = rng.standard_normal((2, 3))
    beta, n = 3.0, 128
    g = (np.arange(n) + 0.5) / n - 0.5
    a, b = np.meshgrid(g, g, indexing="ij")
    trg = np.array([a.ravel() * e1[0] + b.ravel() * e2[0], a.ravel() * e1[1] + b.ravel() * e2[1]])
    u, _ = oracle.mstokes(e1, e2, beta, src, f, trg, tol=1e-12)
    mean = f.sum(axis=1) / (beta ** 2 * 0.9)
    assert np.max(np.abs(u.mean(axis=1) - mean)) < 1e-4 * np.max(np.abs(mean))


def test_mstokes_tight_pair_is_free_space():
    # a force pair 1e-3 apart seen from 3e-3: the images add O((r/L)^3)
    delta = 1e-3
    src = np.array([[0.0, delta], [0.0, 0.0]])
    f = np.array([[1.0, -1.0], [0.5, -0.5]])
    trg = np.array([[0.5 * delta, 3 * delta, -2 * delta], [2 * delta, -delta, 2 * delta]])
    u, g = oracle.mstokes((1.0, 0.0), (0.0, 1.0), 20.0, src, f, trg)
    uf, gf = oracle.free_space("mstokes", src, f, trg, beta=20.0)
    assert rel(u, uf) < 1e-6 and rel(g, gf) < 1e-6


def test_mstokes_self_term_is_the_limit_at_the_source():
    # u_self(x_i) = lim_{h -> 0} [u(x_i + h) - G_MS(h) f_i], with G_MS from
    # the free-space operator form; the +-h average cancels the O(h) term.
    # Both sides cancel 1/r^2 terms near r = 0, so h stays >= 1e-4
    rng = np.random.default_rng(46)
    n = 7
    src = W.cell_points(rng, *SHEARED, n)
    f = rng.standard_normal((2, n))
    i, beta = 3, 2.0
    u_self, _ = oracle.mstokes(*SHEARED, beta, src, f, None)
    for h in (1e-3, 3e-4, 1e-4):
        acc = np.zeros(2)
        for dv in ((h, 0.0), (-h, 0.0), (0.0, h), (0.0, -h)):
            t = src[:, [i]] + np.array(dv)[:, None]
            u, _ = oracle.mstokes(*SHEARED, beta, src, f, t)
            G, _ = oracle.free_space("mstokes", src[:, [i]], f[:, [i]], t, beta=beta)
            acc += u[:, 0] - G[:, 0]
        acc /= 4
        assert np.abs(acc - u_self[:, i]).max() < 1e-8 * np.abs(u_self).max() + 2 * h * h, (h, acc, u_self[:, i])
