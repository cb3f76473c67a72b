"""FP64 CPU oracle for doubly periodic Laplace, Yukawa and Stokes sums.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers. The product library
never imports, links or runs anything here, and nothing here comes from
the product library: the C++ source (``oracle.cpp``) is compiled on its
own with g++ and loaded through ctypes.

Every function evaluates the plain definition of the periodic sum
(Sec. 1, eq. psum) -- see the header of ``oracle.cpp`` for the methods
(Ewald splits, closed-form row sums, truncated lattice sums). Coordinates
are arrays of shape (2, n) (row 0 = x, row 1 = y) in float64.

Parity status: every function here is pinned by ``tests/test_oracle.py``
(split-parameter independence, agreement of two independent Laplace
formulas, Yukawa and Stokes against spectral sums by Poisson summation over
rows of images -- no Ewald split, no Bessel function; the Stokes one also
fixes the zero-mean constant -- free-space limits, lattice periodicity,
Yukawa -> Laplace limit, divergence-free Stokes velocity, library special
functions).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build(force=False):
    """Compile oracle.cpp into liboracle.so (g++, OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        common = [i64, _dp, _dp, _dp, i64, _dp, _dp, ctypes.POINTER(ctypes.c_int64), _dp, _dp]
        lib.oracle_laplace_ewald.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double] + common
        lib.oracle_laplace_rowsum.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int] + common
        lib.oracle_yukawa_lattice.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double] + common
        lib.oracle_stokes_ewald.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double] + common
        lib.oracle_mstokes.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double] + common
        lib.oracle_free_space.argtypes = [ctypes.c_int, ctypes.c_double] + common
        lib.oracle_laplace_p1.argtypes = [ctypes.c_double] + common
        lib.oracle_yukawa_p1.argtypes = [ctypes.c_double] * 3 + common
        lib.oracle_stokes_p1.argtypes = [ctypes.c_double] + common
        for f in (lib.oracle_laplace_ewald, lib.oracle_laplace_rowsum, lib.oracle_yukawa_lattice,
                  lib.oracle_stokes_ewald, lib.oracle_mstokes, lib.oracle_free_space, lib.oracle_laplace_p1,
                  lib.oracle_yukawa_p1, lib.oracle_stokes_p1):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arr(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _p(a):
    if a is None:
        return None
    if a.dtype == np.int64:
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    return a.ctypes.data_as(_dp)


def _prep(src, dens, trg, ncomp, self_idx=None):
    """trg None: targets are all sources (self terms left out). Otherwise
    self_idx[i] = j marks target i as sitting on source j (-1: none)."""
    src = _arr(src)
    assert src.ndim == 2 and src.shape[0] == 2
    ns = src.shape[1]
    if trg is None:
        trg = src
        self_idx = np.arange(ns, dtype=np.int64)
    else:
        trg = _arr(trg)
    assert trg.ndim == 2 and trg.shape[0] == 2
    if self_idx is not None:
        self_idx = np.ascontiguousarray(self_idx, dtype=np.int64)
        assert self_idx.shape == (trg.shape[1],)
        ok = self_idx >= 0
        assert np.array_equal(trg[:, ok], src[:, self_idx[ok]]), "self_idx targets must equal their sources"
    dens = _arr(dens, (ncomp, ns) if ncomp > 1 else (ns,))
    return src, dens, trg, ns, trg.shape[1], self_idx


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} failed with code {rc}")


def laplace(e1, e2, src, q, trg=None, tol=1e-14, alpha=0.0, self_idx=None):
    """Zero-mean periodic Laplace potential and gradient (Ewald split).

    trg=None means the targets are the sources, self term excluded; with
    explicit targets, self_idx[i] = j says target i is source j (term excluded).
    Returns (pot[nt], grad[2, nt]).
    """
    lib = _load()
    src, q, trg, ns, nt, se = _prep(src, q, trg, 1, self_idx)
    e1 = _arr(e1); e2 = _arr(e2)
    pot = np.empty(nt); grad = np.empty((2, nt))
    _check(lib.oracle_laplace_ewald(_p(e1), _p(e2), alpha, tol, ns, _p(src[0]), _p(src[1]), _p(q),
                                    nt, _p(trg[0]), _p(trg[1]), _p(se), _p(pot), _p(grad)),
           "oracle_laplace_ewald")
    return pot, grad


def laplace_rowsum(d, xi, eta, src, q, trg=None, nrows=None, self_idx=None):
    """Same quantity as laplace() from closed-form row sums (canonical lattice
    e1=(d,0), e2=(xi,eta), all points with |y| <= eta/2)."""
    lib = _load()
    src, q, trg, ns, nt, se = _prep(src, q, trg, 1, self_idx)
    if nrows is None:
        # terms decay like exp(-2 pi n eta/d); 40 digits of margin
        nrows = int(np.ceil(40.0 * d / (2 * np.pi * eta))) + 2
    pot = np.empty(nt); grad = np.empty((2, nt))
    _check(lib.oracle_laplace_rowsum(d, xi, eta, nrows, ns, _p(src[0]), _p(src[1]), _p(q),
                                     nt, _p(trg[0]), _p(trg[1]), _p(se), _p(pot), _p(grad)),
           "oracle_laplace_rowsum")
    return pot, grad


def yukawa(e1, e2, beta, src, q, trg=None, tol=1e-15, self_idx=None):
    """Periodic modified-Helmholtz sum with G = K0(beta r)/(2 pi) (truncated lattice sum)."""
    lib = _load()
    src, q, trg, ns, nt, se = _prep(src, q, trg, 1, self_idx)
    e1 = _arr(e1); e2 = _arr(e2)
    pot = np.empty(nt); grad = np.empty((2, nt))
    _check(lib.oracle_yukawa_lattice(_p(e1), _p(e2), beta, tol, ns, _p(src[0]), _p(src[1]), _p(q),
                                     nt, _p(trg[0]), _p(trg[1]), _p(se), _p(pot), _p(grad)),
           "oracle_yukawa_lattice")
    return pot, grad


def stokes(e1, e2, src, f, trg=None, tol=1e-14, alpha=0.0, self_idx=None):
    """Zero-mean periodic Stokeslet velocity u[2, nt] and gradient g[4, nt]
    (du1/dx, du1/dy, du2/dx, du2/dy); f has shape (2, ns) with zero sum."""
    lib = _load()
    src, f, trg, ns, nt, se = _prep(src, f, trg, 2, self_idx)
    e1 = _arr(e1); e2 = _arr(e2)
    vel = np.empty((2, nt)); grad = np.empty((4, nt))
    _check(lib.oracle_stokes_ewald(_p(e1), _p(e2), alpha, tol, ns, _p(src[0]), _p(src[1]), _p(f),
                                   nt, _p(trg[0]), _p(trg[1]), _p(se), _p(vel), _p(grad)),
           "oracle_stokes_ewald")
    return vel, grad


def mstokes(e1, e2, beta, src, f, trg=None, tol=1e-14, alpha=0.0, self_idx=None):
    """Periodic modified Stokeslet (Sec. 5, eq. msgreen) velocity u[2, nt]
    and gradient g[4, nt] (du1/dx, du1/dy, du2/dx, du2/dy); f has shape
    (2, ns), any net force: the cell mean of u is sum(f)/(beta^2 |C|)."""
    lib = _load()
    src, f, trg, ns, nt, se = _prep(src, f, trg, 2, self_idx)
    e1 = _arr(e1); e2 = _arr(e2)
    vel = np.empty((2, nt)); grad = np.empty((4, nt))
    _check(lib.oracle_mstokes(_p(e1), _p(e2), beta, alpha, tol, ns, _p(src[0]), _p(src[1]), _p(f),
                              nt, _p(trg[0]), _p(trg[1]), _p(se), _p(vel), _p(grad)),
           "oracle_mstokes")
    return vel, grad


def free_space(kernel, src, dens, trg=None, beta=0.0, self_idx=None):
    """Non-periodic direct sums ('laplace' | 'yukawa' | 'stokes' | 'mstokes'),
    same layouts."""
    lib = _load()
    k = {"laplace": 0, "yukawa": 1, "stokes": 2, "mstokes": 3}[kernel]
    src, dens, trg, ns, nt, se = _prep(src, dens, trg, 2 if k >= 2 else 1, self_idx)
    pot = np.empty((2, nt)) if k >= 2 else np.empty(nt)
    grad = np.empty((4, nt)) if k >= 2 else np.empty((2, nt))
    _check(lib.oracle_free_space(k, beta, ns, _p(src[0]), _p(src[1]), _p(dens), nt,
                                 _p(trg[0]), _p(trg[1]), _p(se), _p(pot), _p(grad)), "oracle_free_space")
    return pot, grad


def _p1_frame(e1, pts):
    """Rotate points so that the period e1 lies along +x: (canonical points, R, d)."""
    e1 = np.asarray(e1, float)
    d = float(np.hypot(*e1))
    c, s = e1[0] / d, e1[1] / d
    R = np.array([[c, s], [-s, c]])          # canonical = R user
    return R @ pts, R, d


def singly_periodic(kernel, e1, src, dens, trg=None, beta=0.0, tol=1e-15, self_idx=None):
    """Sums periodic in e1 only (the operator P1, Sec. 3 eq. ksplitting1):
    u(t) = sum_j sum_{m in Z} G(t - s_j - m e1) dens_j, symmetric in m for
    Laplace and Stokes (neutral densities). Same layouts as evaluate();
    gradients and Stokes velocities in the caller's frame."""
    lib = _load()
    nc = 2 if kernel == "stokes" else 1
    src, dens, trg, ns, nt, se = _prep(src, dens, trg, nc, self_idx)
    sc, R, d = _p1_frame(e1, src)
    tc = R @ trg
    dc = R @ dens if kernel == "stokes" else dens
    sc = np.ascontiguousarray(sc); tc = np.ascontiguousarray(tc); dc = np.ascontiguousarray(dc)
    if kernel == "stokes":
        pot = np.empty((2, nt)); grad = np.empty((4, nt))
        _check(lib.oracle_stokes_p1(d, ns, _p(sc[0]), _p(sc[1]), _p(dc), nt, _p(tc[0]), _p(tc[1]), _p(se),
                                    _p(pot), _p(grad)), "oracle_stokes_p1")
        J = grad.reshape(2, 2, nt)
        return R.T @ pot, np.einsum("ji,jkt,kl->ilt", R, J, R).reshape(4, nt)
    pot = np.empty(nt); grad = np.empty((2, nt))
    if kernel == "laplace":
        _check(lib.oracle_laplace_p1(d, ns, _p(sc[0]), _p(sc[1]), _p(dc), nt, _p(tc[0]), _p(tc[1]), _p(se),
                                     _p(pot), _p(grad)), "oracle_laplace_p1")
    elif kernel == "yukawa":
        _check(lib.oracle_yukawa_p1(d, beta, max(tol, 1e-16), ns, _p(sc[0]), _p(sc[1]), _p(dc), nt, _p(tc[0]),
                                    _p(tc[1]), _p(se), _p(pot), _p(grad)), "oracle_yukawa_p1")
    else:
        raise ValueError(kernel)
    return pot, R.T @ grad


def stokes_pressure(e1, e2, src, f, trg=None, tol=1e-14, self_idx=None, periodic=2):
    """Pressure of the periodic Stokeslet sum: the Stokeslet's pressure is
    (1/2pi) r.f/r^2 = -f . grad G_L (G_L = -(1/2pi) log r), so the periodic
    pressure is -(d/dx u_L[f1] + d/dy u_L[f2]) with u_L the periodic Laplace
    sum of the force components as charges (zero cell mean for the doubly
    periodic sum; the symmetric limit along e1 for periodic=1)."""
    f = _arr(f)
    if periodic == 1:
        _, g1 = singly_periodic("laplace", e1, src, f[0], trg, self_idx=self_idx)
        _, g2 = singly_periodic("laplace", e1, src, f[1], trg, self_idx=self_idx)
    else:
        _, g1 = laplace(e1, e2, src, f[0], trg, tol=tol, self_idx=self_idx)
        _, g2 = laplace(e1, e2, src, f[1], trg, tol=tol, self_idx=self_idx)
    return -(g1[0] + g2[1])


def evaluate(kernel, e1, e2, src, dens, trg=None, beta=0.0, tol=1e-14, self_idx=None):
    """Dispatch by kernel name; dens is q[ns] (scalar kernels) or f[2, ns] (Stokes).
    trg None: targets are the sources; self_idx marks sampled sources as targets."""
    if kernel == "laplace":
        return laplace(e1, e2, src, dens, trg, tol=tol, self_idx=self_idx)
    if kernel == "yukawa":
        return yukawa(e1, e2, beta, src, dens, trg, tol=max(tol, 1e-16), self_idx=self_idx)
    if kernel == "stokes":
        return stokes(e1, e2, src, dens, trg, tol=tol, self_idx=self_idx)
    raise ValueError(kernel)
