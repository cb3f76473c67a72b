"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module only draws numbers: it holds none of the periodic-sum
arithmetic, so the oracle and the GPU path can both consume its output
without sharing any of the method. The paper's experiments use uniform
random sources in the unit cell (Sec. 7); the clustered, batched and
multi-density workloads follow the same recipe with the shapes listed in
each function. All draws use numpy's PCG64 generator.
"""
import numpy as np


def cell_points(rng, e1, e2, n):
    """n points uniform in the cell {u1 e1 + u2 e2 : u in [-1/2, 1/2)^2}, shape (2, n)."""
    u = rng.random((2, n)) - 0.5
    e1 = np.asarray(e1, float); e2 = np.asarray(e2, float)
    return np.stack([u[0] * e1[0] + u[1] * e2[0], u[0] * e1[1] + u[1] * e2[1]])


def wrap_to_cell(p, e1, e2):
    """Map points to the cell centred at 0 through lattice coordinates u <- u - round(u)."""
    e1 = np.asarray(e1, float); e2 = np.asarray(e2, float)
    B = np.array([[e1[0], e2[0]], [e1[1], e2[1]]])
    u = np.linalg.solve(B, p)
    u = u - np.round(u)
    return B @ u


def blob_points(rng, e1, e2, n, nblobs=50, sigma=None):
    """n points in nblobs Gaussian clusters (centres uniform in the cell,
    std sigma, default 0.02*|e2|), wrapped into the cell."""
    e2n = float(np.hypot(*e2))
    sigma = 0.02 * e2n if sigma is None else sigma
    c = cell_points(rng, e1, e2, nblobs)
    per = np.full(nblobs, n // nblobs)
    per[: n - per.sum()] += 1
    pts = np.concatenate([c[:, [b]] + sigma * rng.standard_normal((2, per[b])) for b in range(nblobs)],
                         axis=1)
    return wrap_to_cell(pts, e1, e2)


def neutral_charges(rng, n, ndens=1):
    """N(0,1) charges with the mean removed, shape (ndens, n) (or (n,) if ndens == 1)."""
    q = rng.standard_normal((ndens, n))
    q -= q.mean(axis=1, keepdims=True)
    return q[0] if ndens == 1 else q


def neutral_forces(rng, n, ndens=1):
    """N(0,1) 2-vector forces with zero net force, shape (ndens, 2, n) (or (2, n))."""
    f = rng.standard_normal((ndens, 2, n))
    f -= f.mean(axis=2, keepdims=True)
    return f[0] if ndens == 1 else f


def batched_cells(seed=0, ncells=64, nmin=1000, nmax=50000, amax=50.0, smax=0.5):
    """The batched workload: per cell N log-uniform in [nmin, nmax], aspect
    ratio A log-uniform in [1, amax], shear s uniform in [0, smax]; cell
    e1 = (A, 0), e2 = (s*A, 1). Even cells Laplace, odd cells Yukawa.
    Returns a list of dicts (e1, e2, n, kernel, rng)."""
    ss = np.random.SeedSequence(seed)
    out = []
    for c, child in enumerate(ss.spawn(ncells)):
        rng = np.random.default_rng(child)
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        A = float(np.exp(rng.uniform(0.0, np.log(amax))))
        s = float(rng.uniform(0.0, smax))
        out.append(dict(e1=(A, 0.0), e2=(s * A, 1.0), n=n,
                        kernel="laplace" if c % 2 == 0 else "yukawa", rng=rng))
    return out


# --- full-size workloads, as the tests and the stored oracle samples draw them ---

SQUARE = ((1.0, 0.0), (0.0, 1.0))
HIGH_ASPECT = {"a100": ((100.0, 0.0), (0.0, 1.0)), "sheared20": ((20.0, 0.0), (3.0, 1.0))}
ENERGY_CELL = ((10.0, 0.0), (0.0, 1.0))


def densities(rng, kernel, n, ndens=1):
    """Neutral N(0,1) densities for a kernel: forces (2, n) for Stokes, charges (n,) otherwise."""
    return neutral_forces(rng, n, ndens) if kernel == "stokes" else neutral_charges(rng, n, ndens)


def square_uniform(kernel, n=200_000, seed=0):
    """Square cell, n uniform sources, neutral densities: (e1, e2, src, dens)."""
    rng = np.random.default_rng(seed)
    src = cell_points(rng, *SQUARE, n)
    return SQUARE[0], SQUARE[1], src, densities(rng, kernel, n)


def high_aspect_blobs(cell, kernel, n=200_000, seed=0):
    """Cell (100,0),(0,1) or (20,0),(3,1), n sources in 50 Gaussian blobs: (e1, e2, src, dens)."""
    e1, e2 = HIGH_ASPECT[cell]
    rng = np.random.default_rng(seed)
    src = blob_points(rng, e1, e2, n)
    return e1, e2, src, densities(rng, kernel, n)


def energy_uniform(kernel, n=50_000, seed=0):
    """Cell (10,0),(0,1), n uniform sources, neutral densities: (e1, e2, src, dens)."""
    rng = np.random.default_rng(seed)
    src = cell_points(rng, *ENERGY_CELL, n)
    return ENERGY_CELL[0], ENERGY_CELL[1], src, densities(rng, kernel, n)


def batched_inputs(nd=16, seed=0):
    """The 64-cell workload with nd neutral charge vectors per cell: a list of
    dicts (e1, e2, n, kernel, beta, src (2, n), dens (nd, n))."""
    out = []
    for c in batched_cells(seed=seed):
        src = cell_points(c["rng"], c["e1"], c["e2"], c["n"])
        dens = neutral_charges(c["rng"], c["n"], nd).reshape(nd, c["n"])
        out.append(dict(e1=c["e1"], e2=c["e2"], n=c["n"], kernel=c["kernel"],
                        beta=10.0 if c["kernel"] == "yukawa" else 0.0, src=src, dens=dens))
    return out


def sample_indices(n, k, seed=1):
    """k distinct indices out of n, sorted (the sampled targets of a full-size check)."""
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def checksum(*arrays):
    """sha256 (hex, 16 digits) of the float64 bytes of the arrays, in order."""
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()[:16]
