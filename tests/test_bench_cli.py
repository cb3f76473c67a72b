"""bench.py checked without a GPU: the options the driver passes exist, a
multi-GPU request ends with a message and a non-zero status before anything
touches a device, and the FMM work counts behind its rooflines agree with a
brute-force count."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_options_exist():
    res = _run("--help")
    assert res.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup"):
        assert opt in res.stdout


def test_more_than_one_gpu_is_refused_with_a_message():
    res = _run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert res.returncode != 0 and res.stdout == ""
    assert "one GPU" in res.stderr


def test_fmm_work_counts_match_a_brute_force_count():
    # the algorithmic work behind the bench's FMM rooflines, recounted pair by
    # pair and box by box: leaf pairs between neighbouring leaves (periodic),
    # the split of those pairs into own-box and forward pairs of the
    # symmetric leaves, and the interaction lists (children of the parent's
    # neighbours that are not neighbours; the super-grid of image cells at
    # level 0)
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    from paper_2111_01083_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2111_01083_amd import build
        build.build()
    import paper_2111_01083_amd as P
    rng = np.random.default_rng(7)
    e1, e2 = (1.0, 0.0), (0.3, 1.0)
    # three blobs, so that some boxes stay empty, in the user frame
    c = rng.uniform(-0.5, 0.5, (3, 2))
    u = (c[rng.integers(0, 3, 400)] + 0.06 * rng.standard_normal((400, 2))).T
    src = np.array([u[0] * e1[0] + u[1] * e2[0], u[0] * e1[1] + u[1] * e2[1]])
    n = src.shape[1]
    plan = P.Plan("laplace", e1, e2, 1e-6, near_mode="fmm", self_exclude=True)
    plan.set_tuning(fmm_level=3, fmm_leaves=2)
    w = bench.fmm_work(plan, src, n)
    inf = plan.info
    assert (w["level"], w["k1"], w["k2"]) == (3, 1, 1) and w["symmetric_leaves"]
    # lattice coordinates in [-1/2, 1/2) from the canonical basis
    rc, rs = inf["rot_cos"], inf["rot_sin"]
    B = np.array([[inf["d"], inf["xi"]], [0.0, inf["eta"]]])
    xy = np.array([[rc, -rs], [rs, rc]]) @ src
    lat = np.linalg.solve(B, xy)
    lat -= np.rint(lat)
    m = 8
    box = np.minimum(np.floor((lat + 0.5) * m).astype(int), m - 1)
    d = (box[:, :, None] - box[:, None, :]) % m
    near = np.all((d == 0) | (d == 1) | (d == m - 1), axis=0)
    same = np.all(d == 0, axis=0)
    assert w["p2p_pairs"] == near.sum() - n
    assert w["p2p_own_pairs"] == same.sum() - n
    assert 2 * w["p2p_forward_pairs"] == near.sum() - same.sum()
    # interaction lists of levels 1..3 (level 3 = 64 boxes is tabulated)
    P4 = w["order"] ** 4
    visits = {}
    for lev in (1, 2, 3):
        k = 1 << lev
        full = np.zeros((k, k), bool)
        full[box[0] >> (3 - lev), box[1] >> (3 - lev)] = True
        v = 0
        for a in range(k):
            for b in range(k):
                for pa in range(a // 2 - 1, a // 2 + 2):
                    for pb in range(b // 2 - 1, b // 2 + 2):
                        for ca in (2 * pa, 2 * pa + 1):
                            for cb in (2 * pb, 2 * pb + 1):
                                if max(abs(ca - a), abs(cb - b)) > 1 and full[ca % k, cb % k]:
                                    v += 1
        visits[lev] = v
    # level 0: the one box against the super-grid of (2 m0 + 1) x 3 images
    lev0 = 3 * (2 * inf["m0"] + 1) - 9
    assert w["tabulated_levels"] == [3]
    assert w["m2l_table_pairs_fp64"] == visits[3] * P4
    assert w["m2l_node_pairs_fp64"] == (visits[1] + visits[2] + lev0) * P4
    assert w["m2l_node_pairs_fp32"] == 0 and w["m2l_table_pairs_fp32"] == 0
