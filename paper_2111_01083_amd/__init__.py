"""MI355X periodic field evaluator: Python binding of libpfmm (include/pfmm.h).

Functions carry the C ABI's names and only marshal arguments (torch device
tensors -> raw pointers, the current HIP stream); every step of an
evaluation runs in the HIP library, and nothing here falls back to a CPU
path. A `Plan` wraps a pfmm_plan_t handle.

Shapes (torch float64 tensors on the HIP device):
  src (2, ns); trg (2, nt) or None when targets are the sources
  dens (ns,) | (n_dens, ns); Stokes (2, ns) | (n_dens, 2, ns)
  returns pot (nt,) | (n_dens, nt) [Stokes (2, nt) | (n_dens, 2, nt)] and
          grad (2, nt) | (n_dens, 2, nt) [Stokes (4, nt) | (n_dens, 4, nt)]
"""
import ctypes

import numpy as np

from . import _lib as L

KERNELS = {"laplace": L.PFMM_LAPLACE, "yukawa": L.PFMM_YUKAWA, "stokes": L.PFMM_STOKES}
PRECISIONS = {"fp64": L.PFMM_FP64, "mixed": L.PFMM_MIXED}
FAR_MODES = {"auto": L.PFMM_FAR_AUTO, "direct": L.PFMM_FAR_DIRECT, "nufft": L.PFMM_FAR_NUFFT}
NEAR_MODES = {"auto": L.PFMM_NEAR_AUTO, "one_sided": L.PFMM_NEAR_ONE_SIDED, "mutual": L.PFMM_NEAR_MUTUAL,
              "none": L.PFMM_NEAR_NONE, "fmm": L.PFMM_NEAR_FMM}


class PfmmError(RuntimeError):
    def __init__(self, code, where):
        lib = L.load()
        super().__init__(f"{where}: {L.ERRORS.get(code, code)} ({lib.pfmm_strerror(code).decode()})")
        self.code = code


def _check(rc, where):
    if rc != 0:
        raise PfmmError(rc, where)


def _dp(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Plan:
    """Owner of a pfmm_plan_t (see pfmm_plan)."""

    def __init__(self, kernel, e1, e2, tol, beta=0.0, precision="fp64", far_mode="auto", m0=0,
                 n_dens=1, self_exclude=False, m_gl=0, check_neutral=False, profile=False, near_mode="auto",
                 periodic=2, ew_rule="compressed"):
        lib = L.load()
        self.kernel_name = kernel
        self.kernel = KERNELS[kernel]
        opts = L.pfmm_opts(float(beta), PRECISIONS[precision], FAR_MODES[far_mode], int(m0), int(n_dens),
                           int(bool(self_exclude)), int(m_gl), int(bool(check_neutral)), int(bool(profile)),
                           NEAR_MODES[near_mode], int(periodic), {"compressed": 0, "panels": 1}[ew_rule])
        e1 = np.ascontiguousarray(e1, dtype=np.float64)
        e2 = np.ascontiguousarray(e2, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib.pfmm_plan(self.kernel, _dp(e1), _dp(e2), float(tol), ctypes.byref(opts), ctypes.byref(h)),
               "pfmm_plan")
        self.handle = h
        self.n_dens = int(n_dens)
        self.self_exclude = bool(self_exclude)
        self.beta = float(beta)
        self.precision = PRECISIONS[precision]
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and L is not None and L._lib is not None:
            L._lib.pfmm_destroy(h)
            self.handle = None

    @property
    def info(self):
        inf = L.pfmm_plan_info_t()
        _check(L.load().pfmm_plan_get_info(self.handle, ctypes.byref(inf)), "pfmm_plan_get_info")
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    @property
    def fmm_symmetric(self):
        """True if an FMM near part of this plan takes symmetric leaves."""
        return bool(self.info["fmm_symmetric"])

    def quadrature(self):
        n = self.info["n_quad"]
        x = np.zeros(n); w = np.zeros(n)
        _check(L.load().pfmm_plan_get_quadrature(self.handle, _dp(x), _dp(w)), "pfmm_plan_get_quadrature")
        return x, w

    def log_groups(self):
        """(ends, e0): image groups of the mixed symmetric near field (pfmm_plan_get_log_groups)."""
        n = self.info["n_log_groups"]
        ends = (ctypes.c_int * max(n, 1))(); e0 = (ctypes.c_int * max(n, 1))()
        _check(L.load().pfmm_plan_get_log_groups(self.handle, ends, e0), "pfmm_plan_get_log_groups")
        return list(ends)[:n], list(e0)[:n]

    def spread_kernel(self):
        """(coef (17, 20), deg, beta_es): the NUFFT kernel's tap polynomials (pfmm_plan_get_spread_kernel)."""
        coef = np.zeros(17 * 20)
        deg, b = ctypes.c_int(), ctypes.c_double()
        _check(L.load().pfmm_plan_get_spread_kernel(self.handle, _dp(coef), ctypes.byref(deg), ctypes.byref(b)),
               "pfmm_plan_get_spread_kernel")
        return coef.reshape(17, 20), deg.value, b.value

    def stage_times(self):
        """(near-field ms, whole-evaluation ms, evaluations) since the last call
        (profiling plans; waits for the recorded HIP events)."""
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(L.load().pfmm_plan_stage_times(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)),
               "pfmm_plan_stage_times")
        return a.value, b.value, n.value

    def fmm_stage_times(self):
        """FMM near part of the evaluations since the last call (profiling
        plans): ({stage: ms summed}, evaluations) for the stages upward,
        m2l_fp64, m2l_fp32, downward, leaves."""
        ms = (ctypes.c_double * 5)()
        n = ctypes.c_int()
        _check(L.load().pfmm_plan_fmm_stage_times(self.handle, ms, ctypes.byref(n)), "pfmm_plan_fmm_stage_times")
        return dict(zip(("upward", "m2l_fp64", "m2l_fp32", "downward", "leaves"), list(ms))), n.value

    def fmm_tree(self, n_src, n_trg=None):
        """The FMM tree an evaluation with these sizes takes, or None if its
        near part is direct: dict(level, k1, k2, order)."""
        out = (ctypes.c_int * 5)()
        _check(L.load().pfmm_fmm_tree(self.handle, int(n_src), int(n_src if n_trg is None else n_trg), out),
               "pfmm_fmm_tree")
        return dict(level=out[1], k1=out[2], k2=out[3], order=out[4]) if out[0] else None

    @property
    def tuning(self):
        return pfmm_plan_get_tuning(self)

    def set_tuning(self, near_blocks=None, nufft_grid=None, fmm_level=None, fmm_leaves=None):
        pfmm_plan_set_tuning(self, near_blocks, nufft_grid, fmm_level, fmm_leaves)

    def __call__(self, src, dens, trg=None, **kw):
        return pfmm_eval(self, src, dens, trg, **kw)


def pfmm_plan(kernel, e1, e2, tol, **opts):
    return Plan(kernel, e1, e2, tol, **opts)


def pfmm_plan_upload(plan):
    _check(L.load().pfmm_plan_upload(plan.handle), "pfmm_plan_upload")


def pfmm_workspace_bytes(plan, n_src, n_trg):
    return int(L.load().pfmm_workspace_bytes(plan.handle, int(n_src), int(n_trg)))


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes, device, workspace):
    torch = _torch()
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = workspace.data_ptr()
    aligned = (ptr + 255) & ~255
    avail = workspace.numel() - (aligned - ptr)
    return workspace, aligned, avail


def _as_dev(t, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 tensor on the HIP device")
    return t.contiguous()


def _as_points(t, name):
    t = _as_dev(t, name)
    if t.dim() != 2 or t.shape[0] != 2:
        raise ValueError(f"{name} must have shape (2, n) (x row, then y row), got {tuple(t.shape)}")
    return t


def pfmm_eval(plan, src, dens, trg=None, out_pot=None, out_grad=None, workspace=None, stream=None,
              want_pot=True, want_grad=True):
    """Potentials and gradients at the targets (trg None: targets = sources)."""
    torch = _torch()
    lib = L.load()
    src = _as_points(src, "src")
    dens = _as_dev(dens, "dens")
    ns = src.shape[1]
    stokes = plan.kernel == L.PFMM_STOKES
    squeeze = dens.dim() == (2 if stokes else 1)
    nd = plan.n_dens
    if dens.numel() != nd * (2 if stokes else 1) * ns:
        raise ValueError("dens has the wrong size for this plan")
    if plan.self_exclude:
        if trg is not None and trg.data_ptr() != src.data_ptr():
            raise ValueError("self_exclude plan: targets are the sources (pass trg=None)")
        trg_t, nt = None, ns
    else:
        if trg is None:
            raise ValueError("plan without self_exclude needs targets")
        trg_t = _as_points(trg, "trg")
        nt = trg_t.shape[1]
    npot = 2 if stokes else 1
    ngrad = 4 if stokes else 2
    if want_pot and out_pot is None:
        out_pot = torch.empty((nd, npot, nt) if stokes else (nd, nt), dtype=torch.float64, device=src.device)
    if want_grad and out_grad is None:
        out_grad = torch.empty((nd, ngrad, nt), dtype=torch.float64, device=src.device)
    nbytes = pfmm_workspace_bytes(plan, ns, nt)
    ws, wptr, avail = _workspace(nbytes, src.device, workspace)
    rc = lib.pfmm_eval(plan.handle, ns, src.data_ptr(), dens.data_ptr(), nt,
                       None if trg_t is None else trg_t.data_ptr(),
                       None if out_pot is None else out_pot.data_ptr(),
                       None if out_grad is None else out_grad.data_ptr(),
                       wptr, avail, _stream_ptr(stream))
    _check(rc, "pfmm_eval")
    if squeeze:
        out_pot = None if out_pot is None else out_pot[0]
        out_grad = None if out_grad is None else out_grad[0]
    return out_pot, out_grad


def pfmm_eval_static(plan, src, dens, trg=None, out_pot=None, out_grad=None, stream=None):
    """pfmm_eval without a workspace: the library's fixed device array is
    used instead (see pfmm.h; the plan must have been uploaded with
    pfmm_plan_upload). Output tensors are allocated here unless passed."""
    torch = _torch()
    lib = L.load()
    src = _as_points(src, "src")
    dens = _as_dev(dens, "dens")
    ns = src.shape[1]
    stokes = plan.kernel == L.PFMM_STOKES
    nd = plan.n_dens
    if dens.numel() != nd * (2 if stokes else 1) * ns:
        raise ValueError("dens has the wrong size for this plan")
    trg_t = None if plan.self_exclude else _as_points(trg, "trg")
    nt = ns if trg_t is None else trg_t.shape[1]
    if out_pot is None:
        out_pot = torch.empty((nd, 2, nt) if stokes else (nd, nt), dtype=torch.float64, device=src.device)
    if out_grad is None:
        out_grad = torch.empty((nd, 4 if stokes else 2, nt), dtype=torch.float64, device=src.device)
    _check(lib.pfmm_eval_static(plan.handle, ns, src.data_ptr(), dens.data_ptr(), nt,
                                None if trg_t is None else trg_t.data_ptr(), out_pot.data_ptr(),
                                out_grad.data_ptr(), _stream_ptr(stream)), "pfmm_eval_static")
    return out_pot, out_grad


def pfmm_plan_get_log_groups(plan):
    return plan.log_groups()


def pfmm_plan_get_tuning(plan):
    t = L.pfmm_tuning_t()
    _check(L.load().pfmm_plan_get_tuning(plan.handle, ctypes.byref(t)), "pfmm_plan_get_tuning")
    return {"near_blocks": int(t.near_blocks), "nufft_grid": int(t.nufft_grid), "fmm_level": int(t.fmm_level),
            "fmm_leaves": int(t.fmm_leaves)}


def pfmm_plan_set_tuning(plan, near_blocks=None, nufft_grid=None, fmm_level=None, fmm_leaves=None):
    cur = pfmm_plan_get_tuning(plan)
    t = L.pfmm_tuning_t(int(cur["near_blocks"] if near_blocks is None else near_blocks),
                        int(cur["nufft_grid"] if nufft_grid is None else nufft_grid),
                        int(cur["fmm_level"] if fmm_level is None else fmm_level),
                        int(cur["fmm_leaves"] if fmm_leaves is None else fmm_leaves))
    _check(L.load().pfmm_plan_set_tuning(plan.handle, ctypes.byref(t)), "pfmm_plan_set_tuning")


def _tuning_workspace_bytes(plan, ns, nt):
    # the largest workspace over the autotuner's candidates
    start = pfmm_plan_get_tuning(plan)
    best = pfmm_workspace_bytes(plan, ns, nt)
    try:
        for nb in (4096, 16384):
            for g in (0, 1):
                for lv in range(0, 12):   # FMM leaf levels (only the tree's neighbours are tried)
                    for leaves in (0, 1, 2):
                        try:
                            pfmm_plan_set_tuning(plan, nb, g, lv, leaves)
                        except PfmmError:
                            continue
                        best = max(best, pfmm_workspace_bytes(plan, ns, nt))
    finally:
        pfmm_plan_set_tuning(plan, start["near_blocks"], start["nufft_grid"], start["fmm_level"], start["fmm_leaves"])
    return best


def pfmm_autotune(plan, src, dens, trg=None, out_pot=None, out_grad=None, workspace=None, stream=None):
    """Time the tuning candidates on these inputs and keep the fastest in the
    plan (see pfmm.h); returns (report dict, pot, grad) with the outputs of
    an evaluation with the chosen tuning."""
    torch = _torch()
    lib = L.load()
    src = _as_points(src, "src"); dens = _as_dev(dens, "dens")
    ns = src.shape[1]
    stokes = plan.kernel == L.PFMM_STOKES
    nd = plan.n_dens
    trg_t = None if plan.self_exclude else _as_points(trg, "trg")
    nt = ns if trg_t is None else trg_t.shape[1]
    if out_pot is None:
        out_pot = torch.empty((nd, 2, nt) if stokes else (nd, nt), dtype=torch.float64, device=src.device)
    if out_grad is None:
        out_grad = torch.empty((nd, 4 if stokes else 2, nt), dtype=torch.float64, device=src.device)
    ws, wptr, avail = _workspace(_tuning_workspace_bytes(plan, ns, nt), src.device, workspace)
    rep = L.pfmm_tune_report_t()
    _check(lib.pfmm_autotune(plan.handle, ns, src.data_ptr(), dens.data_ptr(), nt,
                             None if trg_t is None else trg_t.data_ptr(), out_pot.data_ptr(), out_grad.data_ptr(),
                             wptr, avail, _stream_ptr(stream), ctypes.byref(rep)), "pfmm_autotune")
    report = {"n_tried": rep.n_tried, "default_ms": rep.default_ms, "best_ms": rep.best_ms,
              **pfmm_plan_get_tuning(plan)}
    return report, out_pot, out_grad


def pfmm_workspace_bytes_pressure(plan, n_src, n_trg):
    return int(L.load().pfmm_workspace_bytes_pressure(plan.handle, int(n_src), int(n_trg)))


def pfmm_eval_pressure(plan, src, dens, trg=None, out_pres=None, workspace=None, stream=None):
    """Stokes pressure at the targets (trg None: targets = sources), shape
    (n_trg,) or (n_dens, n_trg) like the potential of a scalar plan."""
    torch = _torch()
    lib = L.load()
    src = _as_points(src, "src")
    dens = _as_dev(dens, "dens")
    ns = src.shape[1]
    nd = plan.n_dens
    if plan.kernel != L.PFMM_STOKES:
        raise ValueError("pfmm_eval_pressure needs a Stokes plan")
    if dens.numel() != nd * 2 * ns:
        raise ValueError("dens has the wrong size for this plan")
    squeeze = dens.dim() == 2
    trg_t = None if plan.self_exclude else _as_points(trg, "trg")
    nt = ns if trg_t is None else trg_t.shape[1]
    if out_pres is None:
        out_pres = torch.empty((nd, nt), dtype=torch.float64, device=src.device)
    ws, wptr, avail = _workspace(pfmm_workspace_bytes_pressure(plan, ns, nt), src.device, workspace)
    _check(lib.pfmm_eval_pressure(plan.handle, ns, src.data_ptr(), dens.data_ptr(), nt,
                                  None if trg_t is None else trg_t.data_ptr(), out_pres.data_ptr(), wptr, avail,
                                  _stream_ptr(stream)), "pfmm_eval_pressure")
    return out_pres[0] if squeeze else out_pres


def pfmm_workspace_bytes_adjoint(plan, n_src):
    return int(L.load().pfmm_workspace_bytes_adjoint(plan.handle, int(n_src)))


def pfmm_eval_adjoint(plan, src, dens, g_pot, workspace=None, stream=None):
    """dL/dq and dL/dx (2, ns) for a loss of the potentials at the sources,
    given g_pot = dL/dpot (see pfmm.h)."""
    torch = _torch()
    lib = L.load()
    src = _as_points(src, "src"); dens = _as_dev(dens, "dens"); g_pot = _as_dev(g_pot, "g_pot")
    ns = src.shape[1]
    if g_pot.numel() != dens.numel():
        raise ValueError("g_pot must have the shape of the potential (= shape of dens)")
    dq = torch.empty_like(dens)
    dxy = torch.empty((2, ns), dtype=torch.float64, device=src.device)
    ws, wptr, avail = _workspace(pfmm_workspace_bytes_adjoint(plan, ns), src.device, workspace)
    _check(lib.pfmm_eval_adjoint(plan.handle, ns, src.data_ptr(), dens.data_ptr(), g_pot.data_ptr(),
                                 dq.data_ptr(), dxy.data_ptr(), wptr, avail, _stream_ptr(stream)),
           "pfmm_eval_adjoint")
    return dq, dxy


def _autograd():
    torch = _torch()

    class PeriodicPotential(torch.autograd.Function):
        """pot = periodic potential at the sources (self terms excluded), with
        a backward pass through pfmm_eval_adjoint (dL/dx and dL/dq)."""

        @staticmethod
        def forward(ctx, src, dens, plan):
            pot, _ = pfmm_eval(plan, src, dens, None, want_grad=False)
            ctx.plan = plan
            ctx.save_for_backward(src, dens)
            return pot

        @staticmethod
        def backward(ctx, g_pot):
            src, dens = ctx.saved_tensors
            dq, dxy = pfmm_eval_adjoint(ctx.plan, src, dens, g_pot.contiguous())
            return dxy, dq, None

    return PeriodicPotential


_PP = None


def periodic_potential(plan, src, dens):
    """Differentiable periodic potential at the sources (plan: self_exclude=True,
    n_dens=1). E.g. the energy is 0.5 * (dens * periodic_potential(...)).sum()."""
    global _PP
    if _PP is None:
        _PP = _autograd()
    return _PP.apply(src, dens, plan)


class Batch:
    """Owner of a pfmm_batch_t: many cells evaluated together (see pfmm.h).

    plans: list of Plan (same precision, n_dens, self_exclude); src_off /
    trg_off: int sequences of length n_cells + 1 into concatenated arrays."""

    def __init__(self, plans, src_off, trg_off=None, use_graph=False):
        lib = L.load()
        n = len(plans)
        self.plans = list(plans)               # keep the plans alive
        self.src_off = np.ascontiguousarray(src_off, dtype=np.int64)
        self.trg_off = None if trg_off is None else np.ascontiguousarray(trg_off, dtype=np.int64)
        arr = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
        i64p = ctypes.POINTER(ctypes.c_int64)
        h = ctypes.c_void_p()
        _check(lib.pfmm_batch_create(n, arr, self.src_off.ctypes.data_as(i64p),
                                     None if self.trg_off is None else self.trg_off.ctypes.data_as(i64p),
                                     int(bool(use_graph)), ctypes.byref(h)), "pfmm_batch_create")
        self.handle = h
        self.stokes = plans[0].kernel == L.PFMM_STOKES
        self.n_dens = plans[0].n_dens
        self.self_exclude = plans[0].self_exclude
        self.workspace_bytes = int(lib.pfmm_batch_workspace_bytes(h))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and L is not None and L._lib is not None:
            L._lib.pfmm_batch_destroy(h)
            self.handle = None

    def __call__(self, src, dens, trg=None, out_pot=None, out_grad=None, workspace=None, stream=None):
        return pfmm_eval_batch(self, src, dens, trg, out_pot, out_grad, workspace, stream)

    def autotune(self, src, dens, trg=None, stream=None):
        return pfmm_batch_autotune(self, src, dens, trg, stream=stream)


def pfmm_eval_batch(batch, src, dens, trg=None, out_pot=None, out_grad=None, workspace=None, stream=None):
    """Evaluate every cell of a Batch; arrays are concatenated over cells.
    Returns pot (n_dens, T) [Stokes (n_dens, 2, T)] and grad (n_dens, 2|4, T)."""
    torch = _torch()
    lib = L.load()
    src = _as_points(src, "src"); dens = _as_dev(dens, "dens")
    T = int(batch.src_off[-1] if batch.self_exclude else batch.trg_off[-1])
    trg_t = None if batch.self_exclude else _as_points(trg, "trg")
    nd = batch.n_dens
    if out_pot is None:
        out_pot = torch.empty((nd, 2, T) if batch.stokes else (nd, T), dtype=torch.float64, device=src.device)
    if out_grad is None:
        out_grad = torch.empty((nd, 4 if batch.stokes else 2, T), dtype=torch.float64, device=src.device)
    # re-read: retuning a plan of the batch can change the size
    batch.workspace_bytes = int(lib.pfmm_batch_workspace_bytes(batch.handle))
    ws, wptr, avail = _workspace(batch.workspace_bytes, src.device, workspace)
    batch._ws_keep = ws
    _check(lib.pfmm_eval_batch(batch.handle, src.data_ptr(), dens.data_ptr(),
                               None if trg_t is None else trg_t.data_ptr(), out_pot.data_ptr(),
                               out_grad.data_ptr(), wptr, avail, _stream_ptr(stream)), "pfmm_eval_batch")
    return out_pot, out_grad


def pfmm_batch_autotune(batch, src, dens, trg=None, out_pot=None, out_grad=None, workspace=None, stream=None):
    """Time task lengths and persistent grid sizes on these inputs and keep
    the fastest in the batch; returns (report dict, pot, grad)."""
    torch = _torch()
    lib = L.load()
    src = _as_points(src, "src"); dens = _as_dev(dens, "dens")
    T = int(batch.src_off[-1] if batch.self_exclude else batch.trg_off[-1])
    trg_t = None if batch.self_exclude else _as_points(trg, "trg")
    nd = batch.n_dens
    if out_pot is None:
        out_pot = torch.empty((nd, 2, T) if batch.stokes else (nd, T), dtype=torch.float64, device=src.device)
    if out_grad is None:
        out_grad = torch.empty((nd, 4 if batch.stokes else 2, T), dtype=torch.float64, device=src.device)
    # room for candidates with more source splits than the current one
    ws, wptr, avail = _workspace(2 * batch.workspace_bytes, src.device, workspace)
    rep = L.pfmm_tune_report_t()
    _check(lib.pfmm_batch_autotune(batch.handle, src.data_ptr(), dens.data_ptr(),
                                   None if trg_t is None else trg_t.data_ptr(), out_pot.data_ptr(),
                                   out_grad.data_ptr(), wptr, avail, _stream_ptr(stream), ctypes.byref(rep)),
           "pfmm_batch_autotune")
    batch.workspace_bytes = int(lib.pfmm_batch_workspace_bytes(batch.handle))
    return {"n_tried": rep.n_tried, "default_ms": rep.default_ms, "best_ms": rep.best_ms}, out_pot, out_grad


def pfmm_strerror(code):
    return L.load().pfmm_strerror(int(code)).decode()


def pfmm_destroy(plan):
    plan.__del__()
