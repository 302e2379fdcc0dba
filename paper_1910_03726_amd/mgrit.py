"""Python binding of libmgrit (include/mgrit.h): argument marshalling only.

Every computation runs in libmgrit.so: the host setup of the coarse
operators in its C++ code, every step of a solve in its gfx950 kernels.
PyTorch supplies device memory (float64 CUDA tensors, passed by pointer)
and the HIP stream.  There is no fallback: if the library is missing,
``lib()`` raises.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgrit.so")
_lib = None

SCHEMES = {"ERK1": 1, "ERK2": 2, "ERK3": 3, "ERK4": 4, "ERK5": 5,
           "SDIRK1": 11, "SDIRK2": 12, "SDIRK3": 13, "SDIRK4": 14}
CYCLES = {"V": 0, "F": 1}
RELAX = {"FCF": 0, "F": 1}
PRECISION = {"fp64": 0, "fp32": 1, "fp32_ir": 2}
PSI_RULES = {"auto": 0, "window": 1, "eta": 2, "redisc": 3}
OUT = {"none": 0, "final": 1, "cpoints": 2, "all": 3}

OK, EINVAL, EUNSTABLE, ENOMEM, EHIP, ENOTCONV, EDIVERGED, EIMAG, ENODEV, \
    ECAPACITY, EBUSY, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11
STATIC_BYTES = 64 << 20  # MGRIT_STATIC_BYTES
COARSE = {"auto": 0, "sweep": 1, "spectral": 2}
PROF_CLASSES = ("relax_fine", "relax_coarse", "coarsest", "norm", "other")


class MgritError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().mgrit_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class Taps(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int), ("offset", ctypes.POINTER(ctypes.c_int)),
                ("weight", ctypes.POINTER(ctypes.c_double))]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("fine_passes_fp64", ctypes.c_int), ("fine_passes_fp32", ctypes.c_int),
                ("final_residual", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("batched_launches", ctypes.c_longlong)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 5), ("launches", ctypes.c_longlong * 5),
                ("fine_dof_steps", ctypes.c_double)]


class ProfEntry(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("pass_", ctypes.c_int), ("precision", ctypes.c_int),
                ("launches", ctypes.c_longlong), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


PASSES = ("fc", "res", "f", "sweep", "spectral", "norm", "copy")


class Request(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("nt", ctypes.c_int), ("scheme", ctypes.c_int),
                ("m", ctypes.c_int), ("levels", ctypes.c_int), ("cycle", ctypes.c_int),
                ("relax", ctypes.c_int), ("precision", ctypes.c_int),
                ("alpha", ctypes.c_double), ("cfl", ctypes.c_double),
                ("tol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("seed", ctypes.c_ulonglong), ("u0", ctypes.POINTER(ctypes.c_double))]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_longlong), ("status", ctypes.c_int),
                ("iterations", ctypes.c_int), ("levels", ctypes.c_int),
                ("final_residual", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("hbm_bytes", ctypes.c_size_t), ("admit_seq", ctypes.c_longlong)]


def solve_batch(plans, u0s, tol=1e-10, maxit=100, out="final"):
    """mgrit_solve_batch: the solves of `plans` (same stream) stepped together,
    launches of equal shape merged.  u0s: one device tensor of n_x values per
    plan.  Returns one SolveResult per plan, in order."""
    import torch
    n = len(plans)
    if n == 0 or len(u0s) != n:
        raise ValueError("one u0 per plan")
    hs = (_P * n)(*[p._h for p in plans])
    u0p = (_P * n)(*[_ptr(u, "u0", p.nx) for p, u in zip(plans, u0s)])
    tols = (_D * n)(*([float(tol)] * n if not hasattr(tol, "__len__") else tol))
    mx = [int(maxit)] * n if not hasattr(maxit, "__len__") else [int(x) for x in maxit]
    maxits = (_I * n)(*mx)
    outs, outp = [], (_P * n)()
    for i, p in enumerate(plans):
        rows = {"none": 0, "final": 1, "cpoints": p.nc + 1, "all": p.nt + 1}[out]
        t = None
        if out != "none":
            t = torch.empty((rows, p.nx), dtype=torch.float64, device=u0s[i].device)
            outp[i] = t.data_ptr()
        outs.append(t)
    kinds = (_I * n)(*([OUT[out]] * n))
    hists = [(_D * (mx[i] + 1))() for i in range(n)]
    histp = (_P * n)(*[ctypes.cast(h, _P) for h in hists])
    its = (_I * n)()
    sts = (_I * n)()
    rc = lib().mgrit_solve_batch(n, hs, u0p, None, tols, maxits,
                                 outp if out != "none" else None, kinds, histp, its, sts)
    _check(rc, "mgrit_solve_batch")
    res = []
    for i, p in enumerate(plans):
        if sts[i] not in (OK, ENOTCONV, EDIVERGED):
            raise MgritError(sts[i], "mgrit_solve_batch")
        res.append(p._result(sts[i], its[i], hists[i], outs[i]))
    return res


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong),
                ("active", ctypes.c_longlong), ("waiting", ctypes.c_longlong),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("hbm_budget", ctypes.c_size_t), ("psi_cache_hits", ctypes.c_longlong),
                ("psi_cache_misses", ctypes.c_longlong), ("batches", ctypes.c_longlong),
                ("batched_requests", ctypes.c_longlong)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "mgrit_version": (_I, []),
    "mgrit_strerror": (ctypes.c_char_p, [_I]),
    "mgrit_max_amplification": (_I, [_I, _D, ctypes.POINTER(_D)]),
    "mgrit_phi_taps": (_I, [_I, _D, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_D),
                            ctypes.POINTER(_I)]),
    "mgrit_psi_optimize": (_I, [_I, _D, _I, _I, _I, _I, ctypes.POINTER(_I), _D,
                                ctypes.POINTER(Taps), ctypes.POINTER(_D)]),
    "mgrit_psi_optimize_bound": (_I, [_I, _D, _I, _I, _I, _I, _D, ctypes.POINTER(Taps),
                                      ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "mgrit_plan_create": (_I, [ctypes.POINTER(_P), _I, _I, _D, _D, _I, _I, _I,
                               ctypes.POINTER(Taps), _I, _I, _I, _P]),
    "mgrit_plan_create_inflow": (_I, [ctypes.POINTER(_P), _I, _I, _D, _D, _I, _I, _I,
                                      ctypes.POINTER(Taps), _I, _I, ctypes.POINTER(_D), _I,
                                      _P]),
    "mgrit_inflow_operator": (_I, [_I, _D, _D, _I, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                   ctypes.POINTER(_I)]),
    "mgrit_solve": (_I, [_P, _P, _P, _D, _I, _P, _I, ctypes.POINTER(_D),
                         ctypes.POINTER(_I)]),
    "mgrit_solve_batch": (_I, [_I, ctypes.POINTER(_P), ctypes.POINTER(_P),
                               ctypes.POINTER(_P), ctypes.POINTER(_D), ctypes.POINTER(_I),
                               ctypes.POINTER(_P), ctypes.POINTER(_I), ctypes.POINTER(_P),
                               ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "phi_apply_batch": (_I, [_P, _P, _P, _I, _I]),
    "mgrit_plan_bytes": (_I, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "mgrit_plan_set_seed": (_I, [_P, ctypes.c_ulonglong]),
    "mgrit_plan_set_coarse_solver": (_I, [_P, _I]),
    "mgrit_get_stats": (_I, [_P, ctypes.POINTER(Stats)]),
    "mgrit_set_profiling": (_I, [_P, _I]),
    "mgrit_get_profile": (_I, [_P, ctypes.POINTER(Profile)]),
    "mgrit_operator_complexity": (_I, [_P, ctypes.POINTER(_D)]),
    "mgrit_get_profile_detail": (_I, [_P, ctypes.POINTER(ProfEntry), _I,
                                      ctypes.POINTER(_I)]),
    "mgrit_plan_describe": (ctypes.c_char_p, [_P]),
    "mgrit_destroy": (None, [_P]),
    "mgrit_solve_static": (_I, [_I, _I, _D, _D, _I, _I, _I, ctypes.POINTER(Taps), _I, _I,
                                _I, _P, _P, _P, _D, _I, _P, _I, ctypes.POINTER(_D),
                                ctypes.POINTER(_I)]),
    "mgrit_plan_estimate_bytes": (_I, [_I, _I, _I, _I, _I,
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "mgrit_server_create": (_I, [ctypes.POINTER(_P), ctypes.c_size_t, _I, _I, _I, _I]),
    "mgrit_server_submit": (_I, [_P, ctypes.POINTER(Request),
                                 ctypes.POINTER(ctypes.c_longlong)]),
    "mgrit_server_wait": (_I, [_P, ctypes.c_longlong, _I, ctypes.POINTER(Result),
                               ctypes.POINTER(_D)]),
    "mgrit_server_get_stats": (_I, [_P, ctypes.POINTER(ServerStats)]),
    "mgrit_server_destroy": (None, [_P]),
}


def lib():
    """The loaded libmgrit.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # PyTorch-ROCm ships its own HIP runtime with the same soname
        # (libamdhip64.so.7).  Loading torch first makes libmgrit bind to that
        # runtime, so the process has one HIP runtime and torch's streams and
        # allocations are the library's.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1910_03726_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != OK:
        raise MgritError(rc, what)


def _scheme(s):
    return SCHEMES[s] if isinstance(s, str) else int(s)


def max_amplification(scheme, cfl):
    v = _D()
    _check(lib().mgrit_max_amplification(_scheme(scheme), cfl, ctypes.byref(v)),
           "mgrit_max_amplification")
    return v.value


def phi_taps(scheme, cfl, nx):
    """Collapsed ERK stepper (offsets in [0, nx), weights)."""
    cap = 256
    off = (_I * cap)()
    w = (_D * cap)()
    n = _I()
    _check(lib().mgrit_phi_taps(_scheme(scheme), cfl, nx, cap, off, w, ctypes.byref(n)),
           "mgrit_phi_taps")
    return np.array(off[:n.value]), np.array(w[:n.value])


def psi_optimize(scheme, cfl, nx, m, levels, rule="auto", widths=None, eta=0.0,
                 capacity=None, allow_imag=False):
    """Coarse operators Psi_2..Psi_L: list of (offsets, weights), max_imag."""
    cap = capacity or max(64, nx)
    bufs = []
    arr = (Taps * (levels - 1))()
    for i in range(levels - 1):
        o = (_I * cap)()
        w = (_D * cap)()
        bufs.append((o, w))
        arr[i].nnz = cap
        arr[i].offset = o
        arr[i].weight = w
    wd = None
    if widths is not None:
        wd = (_I * len(widths))(*[int(x) for x in widths])
    mi = _D()
    rc = lib().mgrit_psi_optimize(_scheme(scheme), cfl, nx, m, levels, PSI_RULES[rule],
                                  wd, eta, arr, ctypes.byref(mi))
    if not (rc == OK or (rc == EIMAG and allow_imag)):
        raise MgritError(rc, "mgrit_psi_optimize")
    out = []
    for i in range(levels - 1):
        n = arr[i].nnz
        out.append((np.array(bufs[i][0][:n]), np.array(bufs[i][1][:n])))
    return out, mi.value


def psi_optimize_bound(scheme, cfl, nx, nt, m, levels, target=1e-3):
    """Coarse operators with bound-driven window widths
    (mgrit_psi_optimize_bound): list of (offsets, weights), the bound of
    each level's choice, max_imag."""
    cap = 64
    bufs = []
    arr = (Taps * (levels - 1))()
    for i in range(levels - 1):
        o = (_I * cap)()
        w = (_D * cap)()
        bufs.append((o, w))
        arr[i].nnz = cap
        arr[i].offset = o
        arr[i].weight = w
    bounds = (_D * (levels - 1))()
    mi = _D()
    rc = lib().mgrit_psi_optimize_bound(_scheme(scheme), cfl, nx, nt, m, levels, target, arr,
                                        bounds, ctypes.byref(mi))
    _check(rc, "mgrit_psi_optimize_bound")
    out = []
    for i in range(levels - 1):
        n = arr[i].nnz
        out.append((np.array(bufs[i][0][:n]), np.array(bufs[i][1][:n])))
    return out, list(bounds), mi.value


def inflow_operator(scheme, cfl, nx, alpha=1.0):
    """(Phi, B) of the inflow/outflow fine step (mgrit_inflow_operator):
    u^{n+1} = Phi u^n + B (g^(d)(t_n))_d, dense, host only."""
    nd = _I()
    _check(lib().mgrit_inflow_operator(_scheme(scheme), cfl, alpha, nx, None, None,
                                       ctypes.byref(nd)), "mgrit_inflow_operator")
    phi = np.empty((nx, nx))
    B = np.empty((nx, nd.value))
    _check(lib().mgrit_inflow_operator(_scheme(scheme), cfl, alpha, nx,
                                       phi.ctypes.data_as(ctypes.POINTER(_D)),
                                       B.ctypes.data_as(ctypes.POINTER(_D)), ctypes.byref(nd)),
           "mgrit_inflow_operator")
    return phi, B


def workload_psi(w):
    """The coarse operators of a workload description (inputs.WORKLOADS):
    (list of (offsets, weights), max_imag)."""
    if w["psi_rule"] == "bound":
        psi, _, mi = psi_optimize_bound(w["scheme"], w["cfl"], w["nx"], w["nt"], w["m"],
                                        w["levels"], w["psi_target"])
        return psi, mi
    return psi_optimize(w["scheme"], w["cfl"], w["nx"], w["m"], w["levels"],
                        rule=w["psi_rule"], widths=w["psi_widths"])


def _ptr(t, name, numel=None):
    import torch
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} values, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class SolveResult:
    def __init__(self, status, iters, hist, out, stats):
        self.status = status
        self.iters = iters
        self.hist = hist
        self.out = out
        self.stats = stats

    @property
    def converged(self):
        return self.status == OK


class Plan:
    """An MGRIT plan on the current HIP device (see mgrit_plan_create).

    ``inflow``: for the inflow/outflow problem (mgrit_plan_create_inflow),
    an (n_t, >= p+1) array of the inflow data's derivatives g^(d)(n dt).
    """

    def __init__(self, nx, nt, cfl, scheme, m, levels, psi, alpha=1.0, cycle="V",
                 relax="FCF", precision="fp64", stream=None, coarse="auto", inflow=None):
        import torch
        self.nx, self.nt, self.m, self.levels = int(nx), int(nt), int(m), int(levels)
        self.scheme = scheme
        self.precision = precision
        self.relax = relax
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        arr = (Taps * max(1, levels - 1))()
        keep = []
        for i, (o, w) in enumerate(psi):
            oa = (_I * len(o))(*[int(x) for x in o])
            wa = (_D * len(w))(*[float(x) for x in w])
            keep.append((oa, wa))
            arr[i].nnz = len(o)
            arr[i].offset = oa
            arr[i].weight = wa
        h = _P()
        if inflow is None:
            rc = lib().mgrit_plan_create(ctypes.byref(h), self.nx, self.nt, alpha, cfl,
                                         _scheme(scheme), self.m, self.levels, arr,
                                         CYCLES[cycle], RELAX[relax], PRECISION[precision],
                                         ctypes.c_void_p(stream))
            _check(rc, "mgrit_plan_create")
        else:
            if precision != "fp64":
                raise MgritError(EINVAL, "inflow plans are FP64")
            g = np.ascontiguousarray(inflow, dtype=np.float64)
            if g.ndim != 2 or g.shape[0] != self.nt:
                raise ValueError("inflow must be an (n_t, n_derivs) array")
            rc = lib().mgrit_plan_create_inflow(
                ctypes.byref(h), self.nx, self.nt, alpha, cfl, _scheme(scheme), self.m,
                self.levels, arr, CYCLES[cycle], RELAX[relax],
                g.ctypes.data_as(ctypes.POINTER(_D)), g.shape[1], ctypes.c_void_p(stream))
            _check(rc, "mgrit_plan_create_inflow")
        self._h = h
        if coarse != "auto":
            self.set_coarse_solver(coarse)

    def set_coarse_solver(self, mode):
        """'auto', 'sweep' or 'spectral' (mgrit_plan_set_coarse_solver)."""
        _check(lib().mgrit_plan_set_coarse_solver(self._h, COARSE[mode]),
               "mgrit_plan_set_coarse_solver")

    @property
    def nc(self):
        return self.nt // self.m

    def close(self):
        if getattr(self, "_h", None):
            lib().mgrit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def solve(self, u0, uinit=None, tol=1e-10, maxit=100, out="final", u_out=None):
        import torch
        nx, nc = self.nx, self.nc
        rows = {"none": 0, "final": 1, "cpoints": nc + 1, "all": self.nt + 1}[out]
        if out != "none" and u_out is None:
            u_out = torch.empty((rows, nx), dtype=torch.float64, device=u0.device)
        hist = (_D * (maxit + 1))()
        it = _I()
        rc = lib().mgrit_solve(self._h, _ptr(u0, "u0", nx),
                               _ptr(uinit, "uinit", (nc + 1) * nx), tol, maxit,
                               _ptr(u_out, "u_out", rows * nx) if out != "none" else None,
                               OUT[out], hist, ctypes.byref(it))
        if rc not in (OK, ENOTCONV, EDIVERGED):
            raise MgritError(rc, "mgrit_solve")
        return self._result(rc, it.value, hist, u_out)

    def _result(self, rc, iters, hist, u_out):
        st = self.stats()
        # one norm per correction; FP32 iterative refinement (asked for, or
        # FP32 Parareal) records one per FP64 refinement step instead
        refine = self.precision == "fp32_ir" or (self.precision == "fp32" and self.relax == "F")
        nh = (st.outer_iterations if refine else iters) + 1
        return SolveResult(rc, iters, list(hist[:nh]), u_out, st)

    def phi_apply_batch(self, inp, out, ksteps):
        b = inp.numel() // self.nx
        _ptr(inp, "in", b * self.nx)
        _ptr(out, "out", b * self.nx)
        _check(lib().phi_apply_batch(self._h, ctypes.c_void_p(inp.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), b, ksteps),
               "phi_apply_batch")

    def bytes(self):
        v = ctypes.c_size_t()
        _check(lib().mgrit_plan_bytes(self._h, ctypes.byref(v)), "mgrit_plan_bytes")
        return v.value

    def set_seed(self, seed):
        _check(lib().mgrit_plan_set_seed(self._h, seed), "mgrit_plan_set_seed")

    def stats(self):
        s = Stats()
        _check(lib().mgrit_get_stats(self._h, ctypes.byref(s)), "mgrit_get_stats")
        return s

    def set_profiling(self, on):
        _check(lib().mgrit_set_profiling(self._h, 1 if on else 0), "mgrit_set_profiling")

    def profile(self):
        p = Profile()
        _check(lib().mgrit_get_profile(self._h, ctypes.byref(p)), "mgrit_get_profile")
        return {"ms": dict(zip(PROF_CLASSES, list(p.ms))),
                "launches": dict(zip(PROF_CLASSES, list(p.launches))),
                "fine_dof_steps": p.fine_dof_steps}

    def profile_detail(self):
        """Per (level, pass, precision): launches, ms and the algorithmic
        HBM bytes and flops of the profiled launches
        (mgrit_get_profile_detail)."""
        n = _I()
        _check(lib().mgrit_get_profile_detail(self._h, None, 0, ctypes.byref(n)),
               "mgrit_get_profile_detail")
        arr = (ProfEntry * max(1, n.value))()
        _check(lib().mgrit_get_profile_detail(self._h, arr, n.value, ctypes.byref(n)),
               "mgrit_get_profile_detail")
        return [{"level": e.level, "pass": PASSES[e.pass_],
                 "precision": ("fp64", "fp32")[e.precision], "launches": e.launches,
                 "ms": e.ms, "bytes": e.bytes, "flops": e.flops} for e in arr[:n.value]]

    def operator_complexity(self):
        v = _D()
        _check(lib().mgrit_operator_complexity(self._h, ctypes.byref(v)),
               "mgrit_operator_complexity")
        return v.value

    def describe(self):
        return lib().mgrit_plan_describe(self._h).decode()


def _taps_array(psi, levels):
    arr = (Taps * max(1, levels - 1))()
    keep = []
    for i, (o, w) in enumerate(psi):
        oa = (_I * len(o))(*[int(x) for x in o])
        wa = (_D * len(w))(*[float(x) for x in w])
        keep.append((oa, wa))
        arr[i].nnz = len(o)
        arr[i].offset = oa
        arr[i].weight = wa
    return arr, keep


def solve_static(nx, nt, cfl, scheme, m, levels, psi, u0, uinit=None, tol=1e-10, maxit=100,
                 out="final", u_out=None, alpha=1.0, cycle="V", relax="FCF",
                 precision="fp64", stream=None):
    """mgrit_solve_static: a plan's solve without device allocation in the
    library (its arrays live in the static per-device workspace).  Returns
    (status, iterations, residual history, u_out)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    nc = nt // m
    rows = {"none": 0, "final": 1, "cpoints": nc + 1, "all": nt + 1}[out]
    if out != "none" and u_out is None:
        u_out = torch.empty((rows, nx), dtype=torch.float64, device=u0.device)
    arr, keep = _taps_array(psi, levels)
    hist = (_D * (maxit + 1))()
    it = _I()
    rc = lib().mgrit_solve_static(
        nx, nt, alpha, cfl, _scheme(scheme), m, levels, arr, CYCLES[cycle], RELAX[relax],
        PRECISION[precision], ctypes.c_void_p(stream), _ptr(u0, "u0", nx),
        _ptr(uinit, "uinit", (nc + 1) * nx), tol, maxit,
        _ptr(u_out, "u_out", rows * nx) if out != "none" else None, OUT[out], hist,
        ctypes.byref(it))
    del keep
    if rc not in (OK, ENOTCONV, EDIVERGED):
        raise MgritError(rc, "mgrit_solve_static")
    return rc, it.value, list(hist[:it.value + 1]), u_out


def estimate_bytes(nx, nt, m, levels, precision="fp64"):
    v = ctypes.c_size_t()
    _check(lib().mgrit_plan_estimate_bytes(nx, nt, m, levels, PRECISION[precision],
                                           ctypes.byref(v)), "mgrit_plan_estimate_bytes")
    return v.value


class Server:
    """Continuous-batching server (include/mgrit_serve.h)."""

    def __init__(self, hbm_budget, slots=8, setup_threads=8, max_bypass=4, max_batch=8):
        h = _P()
        _check(lib().mgrit_server_create(ctypes.byref(h), int(hbm_budget), slots,
                                         setup_threads, max_bypass, max_batch),
               "mgrit_server_create")
        self._h = h

    def submit(self, nx, nt, scheme, cfl, m, u0, levels=0, cycle="V", relax="FCF",
               precision="fp64", tol=1e-10, maxit=100, seed=1, alpha=1.0):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        if u0.size != nx:
            raise ValueError("u0 must hold nx values")
        r = Request(nx, nt, _scheme(scheme), m, levels, CYCLES[cycle], RELAX[relax],
                    PRECISION[precision], alpha, cfl, tol, maxit, seed,
                    u0.ctypes.data_as(ctypes.POINTER(_D)))
        i = ctypes.c_longlong()
        _check(lib().mgrit_server_submit(self._h, ctypes.byref(r), ctypes.byref(i)),
               "mgrit_server_submit")
        return i.value

    def wait(self, rid, nx, timeout_ms=-1):
        """(Result, u_final ndarray) or None on timeout."""
        res = Result()
        u = np.empty(nx)
        rc = lib().mgrit_server_wait(self._h, rid, timeout_ms, ctypes.byref(res),
                                     u.ctypes.data_as(ctypes.POINTER(_D)))
        if rc == EBUSY:
            return None
        _check(rc, "mgrit_server_wait")
        return res, u

    def stats(self):
        st = ServerStats()
        _check(lib().mgrit_server_get_stats(self._h, ctypes.byref(st)),
               "mgrit_server_get_stats")
        return st

    def close(self):
        if getattr(self, "_h", None):
            lib().mgrit_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
