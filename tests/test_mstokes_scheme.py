"""CPU restatement of the paper's periodizing scheme for the modified
Stokeslet (Sec. 5), written from its formulas with numpy/scipy and compared
with the FP64 oracle. No GPU kernel exists for this kernel yet; the test
fixes how the paper's factors are read before one is written.

  near part:   the 3 (2 m0 + 1) images (Def. 1), free-space kernel summed directly;
  south/north: eq. pmss1 (Thm. south_thm_ms): for every mode alpha_m the
               chi_m family with [[chi, i a], [i a, -a^2/chi]] and the
               |alpha_m| family with [[-|a|, -i a], [-i a, |a|]], each times its
               geometric sum over the rows, e^{-2Q}/(1 - e^{-Q}); north by the
               kernel's evenness (off-diagonals change sign);
  west/east:   eq. mspwexpeast (x > 0; x < 0 by evenness) summed in closed
               form over the columns |m| > m0 of rows n = -1, 0, 1, then
               integrated over lambda numerically.
The |alpha_m| family's m = 0 term is 0 x infinity. With it set to zero the
scheme sums the lattice row by row and its mean velocity is
diag(1, 0) F / (beta^2 |C|) in this frame (F the net force); read as the
constant n n^T F / (beta^2 |C|), n the unit normal to e1, the mean becomes
F / (beta^2 |C|), the cell average of (beta^2 - Laplacian) u + grad p = f,
which is the oracle's value and does not depend on which lattice vector
is e1.
"""
import numpy as np
import pytest
from scipy.integrate import quad_vec

import oracle

C_OFF = [(0, 0), (0, 1), (1, 0), (1, 1)]


def _south_north(d, xi, eta, beta, src, f, trg, M):
    nt = trg.shape[1]
    u = np.zeros((2, nt), complex); g = np.zeros((2, 2, nt), complex)
    al = 2 * np.pi * np.arange(-M, M + 1) / d
    chi = np.sqrt(al ** 2 + beta ** 2)
    c = 1 / (2 * d * beta ** 2)
    for sg in (1.0, -1.0):            # +1: sources to the south (rows n <= -2), -1: north
        Qb = chi * eta - sg * 1j * al * xi
        Ql = np.abs(al) * eta - sg * 1j * al * xi
        wb = np.exp(-2 * Qb) / (1 - np.exp(-Qb))
        wl = np.zeros_like(Ql)
        nz = al != 0
        wl[nz] = np.exp(-2 * Ql[nz]) / (1 - np.exp(-Ql[nz]))
        Bb = np.array([[chi, sg * 1j * al], [sg * 1j * al, -al ** 2 / chi]]) * wb
        Bl = np.array([[-np.abs(al), -sg * 1j * al], [-sg * 1j * al, np.abs(al)]]) * wl
        for j in range(src.shape[1]):
            X = trg[0] - src[0, j]; Y = trg[1] - src[1, j]
            ph = np.exp(1j * np.outer(X, al))
            eb = ph * np.exp(-sg * np.outer(Y, chi)); el = ph * np.exp(-sg * np.outer(Y, np.abs(al)))
            for a, b in C_OFF:
                t = eb * Bb[a, b] + el * Bl[a, b]
                u[a] += c * t.sum(1) * f[b, j]
                g[a, 0] += c * (1j * al * t).sum(1) * f[b, j]
                g[a, 1] += c * (-sg * (chi * eb * Bb[a, b] + np.abs(al) * el * Bl[a, b])).sum(1) * f[b, j]
    return u, g


def _west_east(d, xi, eta, beta, m0, src, f, trg):
    nt = trg.shape[1]
    u = np.zeros((2, nt), complex); g = np.zeros((2, 2, nt), complex)
    cc = 1 / (4 * np.pi * beta ** 2)
    for n in (-1, 0, 1):
        for j in range(src.shape[1]):
            X = trg[0] - src[0, j] - n * xi; Y = trg[1] - src[1, j] - n * eta

            def integrand(lam):
                out = np.zeros((2, 2, 3, nt), complex)       # [a][b][value, d/dx, d/dy]
                for lm in (lam, -lam):
                    s = np.sqrt(beta ** 2 + lm ** 2); al = abs(lm)
                    M1 = np.array([[-lm ** 2, 1j * lm * s], [1j * lm * s, s * s]]) / s
                    M2 = np.array([[al, -1j * lm], [-1j * lm, -al]])
                    # west columns: x = X + |m| d > 0 as written; east: x < 0, G(t) = G(-t)
                    for west in (True, False):
                        xs = X + (m0 + 1) * d if west else (m0 + 1) * d - X
                        gb = np.exp(-s * xs) / -np.expm1(-s * d)
                        gl = np.exp(-al * xs) / -np.expm1(-al * d)
                        py = np.exp((1j if west else -1j) * lm * Y)
                        sx = -1.0 if west else 1.0
                        dy = (1j if west else -1j) * lm
                        for a, b in C_OFF:
                            tb = M1[a, b] * gb * py; tl = M2[a, b] * gl * py
                            out[a, b, 0] += tb + tl
                            out[a, b, 1] += sx * (s * tb + al * tl)
                            out[a, b, 2] += dy * (tb + tl)
                return out.ravel()

            val = quad_vec(integrand, 1e-300, np.inf, epsabs=1e-15, epsrel=1e-13)[0]
            val = val.reshape(2, 2, 3, nt) * cc
            for a, b in C_OFF:
                u[a] += val[a, b, 0] * f[b, j]
                g[a, 0] += val[a, b, 1] * f[b, j]
                g[a, 1] += val[a, b, 2] * f[b, j]
    return u, g


def mstokes_scheme(d, xi, eta, beta, m0, src, f, trg, M=40):
    """Velocity [2, nt] and gradient [4, nt] (du1/dx, du1/dy, du2/dx, du2/dy)
    in the canonical frame e1 = (d, 0), e2 = (xi, eta)."""
    e1 = np.array([d, 0.0]); e2 = np.array([xi, eta])
    u = np.zeros((2, trg.shape[1])); g = np.zeros((4, trg.shape[1]))
    for m in range(-m0, m0 + 1):
        for n in (-1, 0, 1):
            v, gg = oracle.free_space("mstokes", src + (m * e1 + n * e2)[:, None], f, trg, beta=beta)
            u += v; g += gg
    for part in (_south_north(d, xi, eta, beta, src, f, trg, M), _west_east(d, xi, eta, beta, m0, src, f, trg)):
        pu, pg = part
        assert np.abs(pu.imag).max() < 1e-12 and np.abs(pg.imag).max() < 1e-12
        u += pu.real; g += pg.reshape(4, -1).real
    # the m = 0 term of the |alpha| family: n n^T F / (beta^2 |C|), n = (0, 1)
    u[1] += f[1].sum() / (beta ** 2 * d * eta)
    return u, g


@pytest.mark.parametrize("d,xi,eta,beta", [(1.0, 0.3, 1.0, 2.0), (2.0, -0.5, 0.8, 0.7), (1.0, 0.0, 1.5, 6.0)])
@pytest.mark.parametrize("net_force", [False, True])
def test_mstokes_scheme_matches_oracle(d, xi, eta, beta, net_force):
    rng = np.random.default_rng(int(100 * beta) + net_force)
    B = np.array([[d, xi], [0.0, eta]])
    src = B @ rng.uniform(-0.5, 0.5, (2, 4))
    trg = B @ rng.uniform(-0.5, 0.5, (2, 3))
    f = rng.standard_normal((2, 4))
    if not net_force:
        f -= f.mean(axis=1, keepdims=True)
    u, g = mstokes_scheme(d, xi, eta, beta, 1, src, f, trg)
    uo, go = oracle.mstokes((d, 0.0), (xi, eta), beta, src, f, trg)
    assert np.abs(u - uo).max() < 1e-11 * np.abs(uo).max()
    assert np.abs(g - go).max() < 1e-11 * np.abs(go).max()
