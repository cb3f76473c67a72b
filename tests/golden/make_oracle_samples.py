"""Write the oracle's values at sampled targets of the full-size workloads.

The GPU tests of those workloads compare against these stored values, so the
slow FP64 oracle does not run on the GPU machine's clock. Only `oracle/` and
the seeded generators of `workloads.py` are called here; each file records
a checksum of the generated inputs, which the tests recompute before using
the values.

    python tests/golden/make_oracle_samples.py            # every workload
    python tests/golden/make_oracle_samples.py square_n200k_yukawa ...

Files (numpy .npz, no pickled objects), one per workload:
  square_n200k_{yukawa,stokes}       square cell, N = 2e5 uniform, 512 targets
  {a100,sheared20}_blobs_n200k_{laplace,stokes}
                                     high-aspect / sheared cell, N = 2e5 in 50
                                     Gaussian blobs, 512 targets
  batch64_nd16                       64 cells, 16 charge vectors each, 32
                                     targets per cell, every density vector
  energy_n50k_{laplace,stokes}       cell (10,0),(0,1), N = 5e4: potential and
                                     gradient at 1024 particles, and the
                                     potential at x_j +- h e_c, x_j +- 2h e_c
                                     (h = 1e-5) for 64 of them (differences)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

ORACLE_TOL = 1e-12      # truncation of the oracle's own sums
N_SAMPLE = 512
N_BATCH_SAMPLE = 32
N_FORCE = 1024
N_FD = 64
FD_H = 1e-5


def _save(name, **arrays):
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **arrays)
    print(f"wrote {path}", flush=True)


def full_size(name, kernel, beta, e1, e2, src, dens):
    idx = W.sample_indices(src.shape[1], N_SAMPLE)
    pot, grad = oracle.evaluate(kernel, e1, e2, src, dens, src[:, idx], beta=beta, tol=ORACLE_TOL, self_idx=idx)
    _save(name, idx=idx, pot=pot, grad=grad, inputs=np.array(W.checksum(src, dens)), beta=np.array(beta))


def batch(name):
    cells = W.batched_inputs(nd=16)
    arrays = {}
    for c, cell in enumerate(cells):
        idx = W.sample_indices(cell["n"], N_BATCH_SAMPLE, seed=100 + c)
        pots, grads = [], []
        for v in range(cell["dens"].shape[0]):
            p, g = oracle.evaluate(cell["kernel"], cell["e1"], cell["e2"], cell["src"], cell["dens"][v],
                                   cell["src"][:, idx], beta=cell["beta"], tol=ORACLE_TOL, self_idx=idx)
            pots.append(p); grads.append(g)
        arrays[f"c{c}_idx"] = idx
        arrays[f"c{c}_pot"] = np.stack(pots)
        arrays[f"c{c}_grad"] = np.stack(grads)
    srcs = [c["src"] for c in cells] + [c["dens"] for c in cells]
    _save(name, inputs=np.array(W.checksum(*srcs)), **arrays)


def energy(name, kernel):
    e1, e2, src, dens = W.energy_uniform(kernel)
    n = src.shape[1]
    idx = W.sample_indices(n, N_FORCE)
    pot, grad = oracle.evaluate(kernel, e1, e2, src, dens, src[:, idx], tol=ORACLE_TOL, self_idx=idx)
    # differences of the energy in x_j: only the pair terms of particle j
    # move, and its own periodic images enter through an even function of the
    # displacement, so a central difference of E equals (density_j) . (u(x_j +
    # t e_c) - u(x_j - t e_c)) / 2t with u the whole periodic field. Stored at
    # t = +-h and +-2h (fourth-order quotient: near neighbours make the
    # second-order one too coarse)
    fd = W.sample_indices(n, N_FD, seed=2)
    shifted = []
    for c in range(2):
        for s in (1.0, -1.0, 2.0, -2.0):
            t = src[:, fd].copy()
            t[c] += s * FD_H
            p, _ = oracle.evaluate(kernel, e1, e2, src, dens, t, tol=ORACLE_TOL)
            shifted.append(p)
    shape = (2, 4) + shifted[0].shape
    _save(name, idx=idx, pot=pot, grad=grad, fd_idx=fd, fd_pot=np.stack(shifted).reshape(shape),
          fd_steps=np.array([1.0, -1.0, 2.0, -2.0]) * FD_H, inputs=np.array(W.checksum(src, dens)))


def jobs():
    out = {}
    for k, beta in (("yukawa", 10.0), ("stokes", 0.0)):
        out[f"square_n200k_{k}"] = (lambda k=k, beta=beta: full_size(f"square_n200k_{k}", k, beta,
                                                                     *W.square_uniform(k)))
    for cell in W.HIGH_ASPECT:
        for k in ("laplace", "stokes"):
            nm = f"{cell}_blobs_n200k_{k}"
            out[nm] = (lambda nm=nm, cell=cell, k=k: full_size(nm, k, 0.0, *W.high_aspect_blobs(cell, k)))
    out["batch64_nd16"] = lambda: batch("batch64_nd16")
    for k in ("laplace", "stokes"):
        out[f"energy_n50k_{k}"] = (lambda k=k: energy(f"energy_n50k_{k}", k))
    return out


if __name__ == "__main__":
    todo = jobs()
    names = sys.argv[1:] or list(todo)
    for nm in names:
        t0 = time.perf_counter()
        todo[nm]()
        print(f"{nm}: {time.perf_counter() - t0:.1f} s", flush=True)
