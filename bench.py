#!/usr/bin/env python
"""Throughput of the periodic evaluation on one MI355X.

Workload: square cell e1 = (1, 0), e2 = (0, 1); N = 200000 sources uniform
in the cell (seed 0); modified Helmholtz with beta = 10 (neutral N(0,1)
charges) and Stokes (N(0,1) forces with zero net force); potential +
gradient (Stokes: velocity + velocity gradient) at every source, tol 1e-6.
One step = one evaluation of each kernel, i.e. 2N targets. The headline
value is the mixed-precision path; the plain FP64 GPU path is timed on the
same inputs, and the FP64 CPU oracle on a bounded sample of targets.

Prints one JSON line (rank 0). Only one GPU is supported.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "targets/sec (pot+grad) at 1e-6 rel err, mixed vs FP64 GPU path; % FP32/HBM roofline"
# algorithmic flops of one kernel sample (a target-source pair of the
# leaves' direct sums, or a node pair of an interaction list) in the FMM
# kernels: add/mul = 1, fma = 2, transcendental = 1 (a divide, and every FP64
# log, exp, sqrt or Bessel sequence, counts as its one transcendental plus
# its polynomial arithmetic), counted from the kernel source;
# FP64/FP32 conversions, the r = 0 guards and the log-shift bookkeeping are
# not counted. FP32 Yukawa: the large-argument K0/K1 branch. FP64 Yukawa:
# coordinate differences 2, r^2 3, sqrt and beta r 2, 2/x, exp(-x)/sqrt(x) 4,
# 2u - 1 2, two 21-term Clenshaw sums 128, scaling 3, accumulation 7.
FLOPS_PER_PAIR = {"laplace": 14, "yukawa": 51, "stokes": 30}
FLOPS_FP64_PER_PAIR = {"laplace": 14, "yukawa": 155, "stokes": 30}
# symmetric leaves: the terms at the source end of a pair (same kernel values,
# the target's density as weight)
FLOPS_REVERSE_PER_PAIR = {"laplace": 7, "yukawa": 7, "stokes": 19}
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6


# HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
# summary (scaled by a plain-copy calibration); used only while the kernel
# sources still hash to the value recorded with the counters
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters_square_n200k.md")
HASHED = ["paper_2111_01083_amd/csrc/fmm.hip", "paper_2111_01083_amd/csrc/fmm.h",
          "paper_2111_01083_amd/csrc/kernels.hip", "paper_2111_01083_amd/csrc/kernels.h",
          "paper_2111_01083_amd/csrc/device_math.h", "paper_2111_01083_amd/csrc/bessel_tables.h"]


def code_only(text):
    """Source text without // comments and blank lines (the hash follows code, not comments)."""
    return "\n".join(ln.split("//", 1)[0].rstrip() for ln in text.splitlines() if ln.split("//", 1)[0].strip())


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in HASHED:
        with open(os.path.join(ROOT, f)) as fh:
            h.update(code_only(fh.read()).encode())
    try:
        lines = open(COUNTERS).read().splitlines()
    except OSError:
        return {}
    rec = [l.split(":", 1)[1].strip() for l in lines if l.startswith("sources_hash:")]
    if not rec or rec[0] != h.hexdigest()[:16]:
        return {}
    out = {}
    for l in lines:
        if l.startswith("traffic:"):
            name, val = l[len("traffic:"):].strip().rsplit(" ", 1)
            out[name] = float(val)
    return out


def fmm_work(plan, src, n_trg):
    """Algorithmic work of the FMM near part of one evaluation with targets =
    sources src (user frame, [2][n]): the leaves' direct pairs and the
    interaction lists' kernel samples (node pairs) on the FP32 and FP64
    levels, counted on the host from the same tree (the plan's lattice, leaf
    boxes in lattice coordinates, empty boxes and the screened cutoff as in
    the kernels). None if the evaluation's near part is direct."""
    import numpy as np
    t = plan.fmm_tree(src.shape[1], n_trg)
    if t is None:
        return None
    inf = plan.info
    d, xi, eta, rc, rs = inf["d"], inf["xi"], inf["eta"], inf["rot_cos"], inf["rot_sin"]
    x = rc * src[0] - rs * src[1]
    y = rs * src[0] + rc * src[1]
    u2 = y / eta
    u2 -= np.rint(u2)
    u1 = (x - xi * (y / eta)) / d
    u1 -= np.rint(u1)
    L, k1, k2, P = t["level"], t["k1"], t["k2"], t["order"]
    n1, n2 = k1 << L, k2 << L
    i = np.clip(np.floor((u1 + 0.5) * n1).astype(np.int64), 0, n1 - 1)
    j = np.clip(np.floor((u2 + 0.5) * n2).astype(np.int64), 0, n2 - 1)
    leaf = np.zeros((n2, n1))
    np.add.at(leaf, (j, i), 1.0)
    # leaves: every target against the 3 x 3 neighbouring leaves (periodic
    # neighbours are the images' boxes), less the self pairs
    nb = sum(np.roll(np.roll(leaf, a, 0), b, 1) for a in (-1, 0, 1) for b in (-1, 0, 1))
    p2p = float((leaf * nb).sum()) - src.shape[1]
    # symmetric leaves (targets are the sources): the own box one-sided, the
    # forward boxes (the row above, the box to the right) once per pair
    sym = plan.fmm_symmetric
    own = float((leaf * leaf).sum()) - src.shape[1]
    fwd = sum(np.roll(np.roll(leaf, -dj, 0), -di, 1) for di, dj in ((-1, 1), (0, 1), (1, 1), (1, 0)))
    fwd = float((leaf * fwd).sum())
    m0 = inf["m0"]
    beta = plan.beta if plan.kernel == 1 else 0.0
    rcut = np.log(30.0 / inf["eps"]) / beta if beta > 0 else np.inf
    # mixed: FP32 kernel samples on the two finest levels (every level for Yukawa)
    f32_from = (0 if plan.kernel == 1 else max(0, L - 1)) if plan.precision == 1 else L + 1
    # tabulated levels (FP64 tables and products): from the finest down (for
    # mixed Stokes from the finest level it samples in FP64) while a level has
    # >= 64 boxes and the tables fit 1 GiB (49 classes x nc NOUT P^4 entries)
    tab = set()
    nc, no = (2, 6) if plan.kernel == 2 else (1, 3)
    total = 0
    top = min(L, f32_from - 1) if (plan.kernel == 2 and plan.precision == 1) else L
    for lev in range(top, 0, -1):
        if (k1 << lev) * (k2 << lev) < 64:
            break
        b = 49 * nc * no * P ** 4 * 8
        if total + b > 1 << 30:
            break
        total += b
        tab.add(lev)
    pairs = {"fp32": 0.0, "fp64": 0.0, "tab_fp32": 0.0, "tab_fp64": 0.0}
    cnt = leaf
    for lev in range(L, -1, -1):
        m1, m2 = k1 << lev, k2 << lev
        h1, h2 = 0.5 / m1, 0.5 / m2
        rad = 0.5 * max(np.hypot(2 * d * h1 + 2 * xi * h2, 2 * eta * h2), np.hypot(-2 * d * h1 + 2 * xi * h2, 2 * eta * h2))
        ne = cnt > 0
        visits = 0.0
        if lev == 0:
            offs = [(I, J) for J in range(-m2, 2 * m2) for I in range(-m0 * m1, (m0 + 1) * m1)]
            for jj in range(m2):
                for ii in range(m1):
                    for I, J in offs:
                        if abs(I - ii) <= 1 and abs(J - jj) <= 1:
                            continue
                        Dx = d * (ii - I) / m1 + xi * (jj - J) / m2
                        Dy = eta * (jj - J) / m2
                        if np.hypot(Dx, Dy) - 2 * rad > rcut or not ne[J % m2, I % m1]:
                            continue
                        visits += 1
        else:
            # offsets of the interaction list by the target's position in its parent
            for pj in (0, 1):
                for pi in (0, 1):
                    tj, ti = np.meshgrid(np.arange(pj, m2, 2), np.arange(pi, m1, 2), indexing="ij")
                    for dJ in range(-3, 4):
                        for dI in range(-3, 4):
                            if abs(dI) <= 1 and abs(dJ) <= 1:
                                continue
                            # children of the parent's neighbours: offsets from the target
                            if not (-2 - pi <= dI <= 3 - pi and -2 - pj <= dJ <= 3 - pj):
                                continue
                            Dx = -(d * dI / m1 + xi * dJ / m2)
                            Dy = -(eta * dJ / m2)
                            if np.hypot(Dx, Dy) - 2 * rad > rcut:
                                continue
                            visits += float(ne[(tj + dJ) % m2, (ti + dI) % m1].sum())
        pairs["tab_fp64" if lev in tab else ("fp32" if lev >= f32_from else "fp64")] += visits * P ** 4
        if lev > 0:
            cnt = cnt.reshape(m2 // 2, 2, m1 // 2, 2).sum(axis=(1, 3))
    return {"level": L, "k1": k1, "k2": k2, "order": P, "p2p_pairs": p2p, "symmetric_leaves": bool(sym),
            "p2p_own_pairs": own, "p2p_forward_pairs": fwd, "tabulated_levels": sorted(tab),
            "m2l_node_pairs_fp32": pairs["fp32"], "m2l_node_pairs_fp64": pairs["fp64"],
            "m2l_table_pairs_fp32": pairs["tab_fp32"], "m2l_table_pairs_fp64": pairs["tab_fp64"]}


def rel(a, b):
    import numpy as np
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def batch_workload(P, W, torch, dev, np):
    """The batched form: 64 cells (N log-uniform in [1e3, 5e4], aspect ratio
    log-uniform in [1, 50], shear in [0, 0.5]|e1|, even cells Laplace, odd
    Yukawa beta = 10), 16 neutral density vectors per cell, pot + grad at all
    sources, one hipGraph per batch, tol 1e-6; mixed (autotuned task shape)
    against the plain FP64 path, each checked on the stored oracle samples
    (32 targets of every cell, all 16 densities)."""
    cells = W.batched_inputs(nd=16)
    offs = [0]
    for c in cells:
        offs.append(offs[-1] + c["n"])
    src = torch.tensor(np.concatenate([c["src"] for c in cells], axis=1), device=dev)
    q = torch.tensor(np.concatenate([c["dens"] for c in cells], axis=1), device=dev)
    ref = None
    gpath = os.path.join(ROOT, "tests", "golden", "batch64_nd16.npz")
    if os.path.exists(gpath):
        z = np.load(gpath)
        if str(z["inputs"]) == W.checksum(*([c["src"] for c in cells] + [c["dens"] for c in cells])):
            ref = {k: z[k] for k in z.files}
    res = {"workload": "64 cells, 16 density vectors each, sum N = %d, tol 1e-6, hipGraph" % offs[-1]}
    for prec in ("mixed", "fp64"):
        plans = [P.Plan(c["kernel"], c["e1"], c["e2"], 1e-6, beta=c["beta"], precision=prec, n_dens=16,
                        self_exclude=True) for c in cells]
        batch = P.Batch(plans, offs, use_graph=True)
        if prec == "mixed":
            batch.autotune(src, q)
        ws = torch.empty(batch.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        pot = torch.empty((16, offs[-1]), dtype=torch.float64, device=dev)
        grad = torch.empty((16, 2, offs[-1]), dtype=torch.float64, device=dev)
        batch(src, q, out_pot=pot, out_grad=grad, workspace=ws)      # captures the graph
        torch.cuda.synchronize()
        steps = 3 if prec == "mixed" else 2
        t0 = time.perf_counter()
        for _ in range(steps):
            batch(src, q, out_pot=pot, out_grad=grad, workspace=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        entry = {"ms_per_eval": round(ms, 3), "target_densities_per_s": round(16 * offs[-1] / (ms * 1e-3), 1),
                 "steps": steps}
        if ref is not None:
            p_h = pot.cpu().numpy(); g_h = grad.cpu().numpy()
            worst = 0.0
            for c in range(len(cells)):
                sl = offs[c] + ref[f"c{c}_idx"]
                worst = max(worst, rel(p_h[:, sl], ref[f"c{c}_pot"]), rel(g_h[:, :, sl], ref[f"c{c}_grad"]))
            entry["max_rel_err_vs_oracle_per_cell"] = worst
        res[prec] = entry
        del batch, plans, ws
    res["speedup_mixed_vs_fp64"] = round(res["fp64"]["ms_per_eval"] / res["mixed"]["ms_per_eval"], 2)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=200000, help="sources (= targets) per cell")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--sample", type=int, default=16, help="oracle targets per kernel")
    ap.add_argument("--streams", type=int, default=2, choices=(1, 2),
                    help="HIP streams of a step: 2 = the Yukawa and Stokes evaluations run concurrently")
    ap.add_argument("--no-one-stream", action="store_true",
                    help="skip the comparison pass with both evaluations on one stream")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the one-step context run of the direct near-image sum")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-cell batched workload (mixed and FP64) reported beside the headline")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB elementwise copy (to calibrate HBM byte counters)")
    ap.add_argument("--nufft-sweep", default="",
                    help="comma-separated N: instead of the benchmark, time the far part alone (NUFFT "
                         "spread/FFT/interp) on the A = 100 blob workload at each N, one JSON line each")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the benchmark evaluates on one GPU only; multi-GPU runs are not supported "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calib:
        n = 1 << 27                      # float64 elements = 1 GiB
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # elementwise kernel: reads and writes 1 GiB
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 3}), flush=True)
        return

    import workloads as W
    import paper_2111_01083_amd as P

    dev = torch.device("cuda:0")
    if args.nufft_sweep:
        # far part only (near_mode none): the periodizing operator through the
        # NUFFT, Laplace, mixed, tol 1e-6, targets = sources
        for n in [int(float(v)) for v in args.nufft_sweep.split(",")]:
            e1, e2, src, q = W.high_aspect_blobs("a100", "laplace", n)
            d_src, d_q = torch.tensor(src, device=dev), torch.tensor(q, device=dev)
            p = P.Plan("laplace", e1, e2, 1e-6, precision="mixed", far_mode="nufft", near_mode="none",
                       self_exclude=True, profile=True)
            ws = torch.empty(P.pfmm_workspace_bytes(p, n, n) + 256, dtype=torch.uint8, device=dev)
            pot = torch.empty((1, n), dtype=torch.float64, device=dev)
            grad = torch.empty((1, 2, n), dtype=torch.float64, device=dev)
            for _ in range(max(args.warmup, 1)):
                P.pfmm_eval(p, d_src, d_q, None, out_pot=pot, out_grad=grad, workspace=ws)
            torch.cuda.synchronize()
            p.stage_times()
            for _ in range(args.steps):
                P.pfmm_eval(p, d_src, d_q, None, out_pot=pot, out_grad=grad, workspace=ws)
            torch.cuda.synchronize()
            _, total_ms, cnt = p.stage_times()
            ms = total_ms / max(cnt, 1)
            print(json.dumps({"sweep": "far part alone, A=100 blobs, Laplace mixed tol 1e-6, NUFFT", "n": n,
                              "eval_ms": round(ms, 4), "targets_per_s": round(n / (ms * 1e-3), 1),
                              "nufft_nf": p.info["nufft_nf"], "nufft_w": p.info["nufft_w"],
                              "m_gl": p.info["m_gl"], "steps": args.steps}), flush=True)
            del ws, pot, grad, d_src, d_q
        return
    n = args.n
    e1, e2 = (1.0, 0.0), (0.0, 1.0)
    rng = np.random.default_rng(0)
    src = W.cell_points(rng, e1, e2, n)
    q = W.neutral_charges(rng, n)
    f = W.neutral_forces(rng, n)
    d_src = torch.tensor(src, device=dev)
    d_q = torch.tensor(q, device=dev)
    d_f = torch.tensor(f, device=dev)
    cases = [("yukawa", 10.0, d_q), ("stokes", 0.0, d_f)]

    def make(prec):
        plans, outs, wss = [], [], []
        for kern, beta, dens in cases:
            p = P.Plan(kern, e1, e2, 1e-6, beta=beta, precision=prec, self_exclude=True, profile=True)
            ws = torch.empty(P.pfmm_workspace_bytes(p, n, n) + 256, dtype=torch.uint8, device=dev)
            npot, ngrad = (2, 4) if kern == "stokes" else (1, 2)
            pot = torch.empty((1, npot, n) if kern == "stokes" else (1, n), dtype=torch.float64, device=dev)
            grad = torch.empty((1, ngrad, n), dtype=torch.float64, device=dev)
            plans.append(p); outs.append((pot, grad)); wss.append(ws)
        return plans, outs, wss

    # two streams (default priority): the step's two evaluations are
    # independent, and each has phases that do not fill the GPU (binning,
    # the coarse levels of the tree, the far part), which the other's
    # kernels fill; the step starts after, and ends with, the main stream
    side = [torch.cuda.Stream(), torch.cuda.Stream()]

    def step(plans, outs, wss, nstreams=1):
        if nstreams == 1:
            for (kern, beta, dens), p, (pot, grad), ws in zip(cases, plans, outs, wss):
                P.pfmm_eval(p, d_src, dens, None, out_pot=pot, out_grad=grad, workspace=ws)
            return
        main = torch.cuda.current_stream()
        ev = torch.cuda.Event()
        ev.record(main)
        for (kern, beta, dens), p, (pot, grad), ws, st in zip(cases, plans, outs, wss, side):
            st.wait_event(ev)
            with torch.cuda.stream(st):
                P.pfmm_eval(p, d_src, dens, None, out_pot=pot, out_grad=grad, workspace=ws, stream=st)
        for st in side:
            main.wait_stream(st)

    def timed(prec, steps, warmup, nstreams=1):
        plans, outs, wss = make(prec)
        for _ in range(warmup):
            step(plans, outs, wss, nstreams)
        torch.cuda.synchronize()
        for p in plans:
            p.stage_times()      # drop warm-up events
        t0 = time.perf_counter()
        for _ in range(steps):
            step(plans, outs, wss, nstreams)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stages = [p.stage_times() + p.fmm_stage_times() for p in plans]
        res = [(o[0].cpu().numpy()[0], o[1].cpu().numpy()[0]) for o in outs]
        works = [fmm_work(p, src, n) for p in plans]
        return (t1 - t0) / steps, stages, res, works

    print(f"bench: N={n} mixed steps={args.steps} warmup={args.warmup} streams={args.streams}", file=sys.stderr,
          flush=True)
    ms_mixed_s, st_mixed, res_mixed, work_mixed = timed("mixed", args.steps, args.warmup, args.streams)
    print(f"bench: mixed {ms_mixed_s * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    ms64_s, st64, res64, work64 = timed("fp64", args.fp64_steps, 1, args.streams)
    print(f"bench: fp64 {ms64_s * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    one = one64 = None
    if args.streams == 2 and not args.no_one_stream:
        # the same steps with both evaluations on one stream: every kernel
        # alone on the GPU, so that the HIP events between its launches time
        # the kernels themselves (with two streams they also hold the waits
        # for the other stream's kernels); the rooflines come from these
        one = timed("mixed", args.steps, args.warmup, 1)
        print(f"bench: mixed, one stream {one[0] * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
        one64 = timed("fp64", args.fp64_steps, 1, 1)

    targets_per_step = 2 * n
    value = targets_per_step / ms_mixed_s
    fp64_value = targets_per_step / ms64_s

    # rooflines of the FMM near part's kernels (HIP events on the evaluation
    # stream between its launches) against the algorithmic work of the same
    # tree counted on the host
    traffic = measured_traffic()

    def stage_roofs(prec, stages, works):
        peak = FP32_VECTOR_PEAK_TFLOPS if prec == "mixed" else FP64_VECTOR_PEAK_TFLOPS
        pair32, pair64 = FLOPS_PER_PAIR, FLOPS_FP64_PER_PAIR
        out_k = {}
        for (kern, _, _), st, w in zip(cases, stages, works):
            near_ms, total_ms, cnt, fst, fcnt = st
            per = {k: v / max(fcnt, 1) for k, v in fst.items()}
            pw = pair32 if prec == "mixed" else pair64
            nout = 6 if kern == "stokes" else 3
            # leaves: direct pairs, plus per target the interpolation of NOUT
            # fields (P^2 fma each) and the two 1D bases (about 6 P)
            if w["symmetric_leaves"]:
                pairs_fl = pw[kern] * w["p2p_own_pairs"] + (pw[kern] + FLOPS_REVERSE_PER_PAIR[kern]) * w["p2p_forward_pairs"]
            else:
                pairs_fl = pw[kern] * w["p2p_pairs"]
            leaf_flops = pairs_fl + n * (2 * nout * w["order"] ** 2 + 6 * w["order"])
            kname = f"{kern}, {'mixed' if prec == 'mixed' else 'fp64'}"
            # list stages: sampled point pairs at the sample's flops, tabulated
            # ones at 2 nc NOUT flops (one fma per table entry); the kernel
            # named is the one with the most flops in the stage
            tabf = 2 * nout * (2 if kern == "stokes" else 1)
            f32s, f32t = FLOPS_PER_PAIR[kern] * w["m2l_node_pairs_fp32"], tabf * w["m2l_table_pairs_fp32"]
            f64s, f64t = FLOPS_FP64_PER_PAIR[kern] * w["m2l_node_pairs_fp64"], tabf * w["m2l_table_pairs_fp64"]
            rows = {"m2l_fp32": (f32s + f32t, FP32_VECTOR_PEAK_TFLOPS,
                                 f"fmm_m2l_kernel<{kern}, mixed>"),
                    "m2l_fp64": (f64s + f64t, FP64_VECTOR_PEAK_TFLOPS,
                                 f"fmm_m2l_mfma_kernel<{kern}>" if f64t > f64s else f"fmm_m2l_kernel<{kern}, fp64>"),
                    "leaves": (leaf_flops, peak,
                               f"fmm_leaf_sym_kernel<{kname}>" if w["symmetric_leaves"] else f"fmm_leaf_kernel<{kname}>")}
            ent = {}
            for stg, (fl, pk, kn) in rows.items():
                ms = per[stg]
                if fl <= 0 or ms <= 0:
                    continue
                tf = fl / (ms * 1e-3) / 1e12
                ent[stg] = {"bound": "alu", "achieved": round(tf, 3), "peak": pk, "unit": "TFLOP/s",
                            "frac": round(tf / pk, 4), "traffic": traffic.get(kn), "ms_per_launch": round(ms, 4),
                            "flops_per_launch": fl, "kernel": kn}
            out_k[kern] = {"stages_ms_per_eval": {k: round(v, 4) for k, v in per.items()},
                           "near_ms_per_eval": round(near_ms / max(cnt, 1), 3),
                           "eval_ms": round(total_ms / max(cnt, 1), 3), "tree": w, "rooflines": ent}
        return out_k

    roof_main = stage_roofs("mixed", st_mixed, work_mixed)
    roof64_main = stage_roofs("fp64", st64, work64)
    # rooflines from the one-stream passes when the timed steps overlap
    roof_all = stage_roofs("mixed", one[1], one[3]) if one is not None else roof_main
    roof64 = stage_roofs("fp64", one64[1], one64[3]) if one64 is not None else roof64_main
    # the dominant kernel: the longest FMM stage over both kernels of a step
    dom_k, dom_s = max(((k, s_) for k in roof_all for s_ in roof_all[k]["rooflines"]),
                       key=lambda ks: roof_all[ks[0]]["rooflines"][ks[1]]["ms_per_launch"])
    roofline = dict(roof_all[dom_k]["rooflines"][dom_s])
    d64_k, d64_s = max(((k, s_) for k in roof64 for s_ in roof64[k]["rooflines"]),
                       key=lambda ks: roof64[ks[0]]["rooflines"][ks[1]]["ms_per_launch"])
    roofline64 = dict(roof64[d64_k]["rooflines"][d64_s])
    one_stream = None
    if one is not None:
        # context: the step on one stream, and the stage times of the timed
        # (overlapped) steps, which include the waits for the other stream
        one_stream = {"value": round(targets_per_step / one[0], 1), "ms_per_step": round(one[0] * 1e3, 3),
                      "fp64_value": round(targets_per_step / one64[0], 1),
                      "fp64_ms_per_step": round(one64[0] * 1e3, 3),
                      "rooflines_from": "these one-stream passes (roofline, roofline_all, fp64_gpu.roofline)"}
        one_stream["stages_two_streams"] = {k: v["stages_ms_per_eval"] for k, v in roof_main.items()}
        one_stream["fp64_stages_two_streams"] = {k: v["stages_ms_per_eval"] for k, v in roof64_main.items()}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "targets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_mixed_s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "square cell, N=200000 uniform sources = targets, modified Helmholtz "
                               "beta=10 + Stokes, pot+grad, tol 1e-6",
                   "n": n, "tol": 1e-6, "precision": "mixed (FP32 pairs, FP64 accumulation and far field)",
                   "targets_per_step": targets_per_step, "streams": args.streams},
        "fp64_gpu": {"value": round(fp64_value, 1), "unit": "targets/s", "ms_per_step": round(ms64_s * 1e3, 3),
                     "steps": args.fp64_steps, "roofline": roofline64, "kernels": roof64},
        "speedup_mixed_vs_fp64": round(value / fp64_value, 2),
        "roofline": roofline,
        "roofline_all": roof_all,
    }
    if one_stream is not None:
        out["one_stream"] = one_stream
    if not args.no_direct:
        # context: the same mixed step with the near part as the direct sum
        # over the near images (symmetric pair evaluation), one step
        plans_d = [P.Plan(kern, e1, e2, 1e-6, beta=beta, precision="mixed", self_exclude=True, near_mode="mutual")
                   for kern, beta, _ in cases]
        outs_d = [o for o in make("mixed")[1]]
        wss_d = [torch.empty(P.pfmm_workspace_bytes(p_, n, n) + 256, dtype=torch.uint8, device=dev) for p_ in plans_d]
        step(plans_d, outs_d, wss_d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(plans_d, outs_d, wss_d)
        torch.cuda.synchronize()
        ms_d = (time.perf_counter() - t0) * 1e3
        out["direct_near_mixed"] = {"ms_per_step": round(ms_d, 3), "value": round(targets_per_step / (ms_d * 1e-3), 1),
                                    "speedup_fmm_vs_direct": round(ms_d / (ms_mixed_s * 1e3), 2)}
        del plans_d, wss_d

    if not args.no_batch:
        out["batch"] = batch_workload(P, W, torch, dev, np)

    if not args.no_cpu_baseline:
        import oracle
        idx = np.sort(np.random.default_rng(1).choice(n, args.sample, replace=False))
        refs, parts = [], {}
        cpu_total = 0.0
        for kern, beta, _ in cases:
            dens = f if kern == "stokes" else q
            # one target first (the per-source setup -- Ewald structure factors
            # for Stokes, none for the Yukawa lattice sum -- plus one target),
            # then the whole sample; their difference gives the per-target cost
            t0 = time.perf_counter()
            oracle.evaluate(kern, e1, e2, src, dens, src[:, idx[:1]], beta=beta, tol=1e-10, self_idx=idx[:1])
            t1 = time.perf_counter()
            refs.append(oracle.evaluate(kern, e1, e2, src, dens, src[:, idx], beta=beta, tol=1e-10, self_idx=idx))
            t2 = time.perf_counter()
            per_target = max((t2 - t1) - (t1 - t0), 0.0) / max(args.sample - 1, 1)
            setup = max((t1 - t0) - per_target, 0.0)
            parts[kern] = {"setup_s": round(setup, 3), "per_target_s": round(per_target, 5),
                           "sample_s": round(t2 - t1, 3), "full_workload_s_est": round(setup + n * per_target, 1)}
            cpu_total += setup + n * per_target
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        model = ""
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
        except OSError:
            pass
        out["cpu_baseline"] = {"value": round(targets_per_step / cpu_total, 3), "unit": "targets/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{args.sample} sampled targets per kernel (of the {n}) with all {n} "
                                         f"sources, FP64 Ewald (Stokes) / truncated lattice sum (Yukawa); "
                                         f"value = 2N targets over the per-source setup plus N times the "
                                         f"per-target time of each kernel, both measured on the sample",
                               "per_kernel": parts, "nproc": os.cpu_count(),
                               "affinity_cpus": len(os.sched_getaffinity(0)), "omp_threads": threads,
                               "cpu_model": model}
        acc = {}
        for (kern, _, _), (po, go), (pm, gm), (p6, g6) in zip(cases, refs, res_mixed, res64):
            acc[kern] = {"mixed_pot": rel(pm[..., idx], po), "mixed_grad": rel(gm[:, idx], go),
                         "fp64_pot": rel(p6[..., idx], po), "fp64_grad": rel(g6[:, idx], go)}
        out["rel_err_vs_oracle_on_sample"] = acc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
