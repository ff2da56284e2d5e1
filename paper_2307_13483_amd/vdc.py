"""ctypes binding of libvdc (include/vdc.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
values to the C structs, hands torch device buffers (PyTorch is used for
device memory and streams only) to the entry points of the same names, and
turns status codes into exceptions.  Loading fails loudly when the library
has not been built: there is no fallback.
"""
import ctypes
import logging
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_log = logging.getLogger("vdc")
LIB_PATH = os.path.join(_HERE, "libvdc.so")

VDC_OK, VDC_ERR_INVALID_ARG, VDC_ERR_WORKSPACE, VDC_ERR_HIP, VDC_ERR_UNSUPPORTED = range(5)
CONVERGED, NOT_CONVERGED, BREAKDOWN, NONFINITE = range(4)
PREC_NONE, PREC_JACOBI, PREC_BLOCK, PREC_ROWS = 0, 1, 2, 3
FP64, FP32_INNER = 0, 1
GMRES, COCG = 0, 1
STATUS_NAMES = {CONVERGED: "converged", NOT_CONVERGED: "not_converged",
                BREAKDOWN: "breakdown", NONFINITE: "nonfinite"}


class VdcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vdc error {code}: {msg}")
        self.code = code


class ModelDesc(ctypes.Structure):
    _fields_ = [("omega_g", ctypes.c_double), ("omega_u", ctypes.c_double),
                ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double),
                ("lam", ctypes.c_double), ("lam1", ctypes.c_double), ("lam2", ctypes.c_double),
                ("E1", ctypes.c_double), ("gap", ctypes.c_double),
                ("A", (ctypes.c_double * 2) * 2), ("B", (ctypes.c_double * 2) * 2),
                ("l", ctypes.c_int * 2), ("Ng", ctypes.c_int), ("Nu", ctypes.c_int),
                ("hilbert_nodes", ctypes.c_int), ("hilbert_xmax", ctypes.c_double)]


class Job(ctypes.Structure):
    _fields_ = [("eps_i", ctypes.c_double), ("vi_g", ctypes.c_int), ("vi_u", ctypes.c_int),
                ("mu_i", ctypes.c_int), ("model", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_iter", ctypes.c_int), ("tol", ctypes.c_double),
                ("precond", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_restart", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("outer_restart", ctypes.c_int), ("tile_rows", ctypes.c_int),
                ("method", ctypes.c_int), ("check_optical", ctypes.c_int)]


class JobInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("outer_iters", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("retried", ctypes.c_int),
                ("reserved", ctypes.c_int), ("optical_defect", ctypes.c_double)]


class Co2Desc(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in (
        "omega_s", "omega_b", "omega_a", "E_sigma", "E_pi", "k_sigma", "k_pi", "gs_sigma",
        "gb_sigma", "ga_sigma", "gs_pi", "gb_pi", "ga_pi", "c_rt", "c_sp", "c_sp2", "l_sigma",
        "l_pi", "h_sigma", "h_pi")] + [
        ("A", (ctypes.c_double * 2) * 2), ("B", (ctypes.c_double * 2) * 2),
        ("Ns", ctypes.c_int), ("Nx", ctypes.c_int), ("Ny", ctypes.c_int), ("Na", ctypes.c_int),
        ("hilbert_nodes", ctypes.c_int), ("hilbert_xmax", ctypes.c_double)]


class Co2Job(ctypes.Structure):
    _fields_ = [("eps_i", ctypes.c_double), ("v", ctypes.c_int * 4), ("mu_i", ctypes.c_int)]


MAX_MODES = 8


class Term(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("e", ctypes.c_int), ("coeff", ctypes.c_double),
                ("pow", ctypes.c_int * MAX_MODES)]


class Width(ctypes.Structure):
    _fields_ = [("A", ctypes.c_double), ("B", ctypes.c_double), ("l", ctypes.c_int)]


class TermDesc(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int), ("n_modes", ctypes.c_int), ("n_pw", ctypes.c_int),
                ("omega", ctypes.POINTER(ctypes.c_double)), ("nbasis", ctypes.POINTER(ctypes.c_int)),
                ("e_state", ctypes.POINTER(ctypes.c_double)),
                ("n_uterms", ctypes.c_int), ("uterms", ctypes.POINTER(Term)),
                ("n_vterms", ctypes.c_int), ("vterms", ctypes.POINTER(Term)),
                ("width", ctypes.POINTER(Width)), ("hilbert_nodes", ctypes.c_int),
                ("hilbert_xmax", ctypes.c_double), ("dispatch", ctypes.c_int)]


class MJob(ctypes.Structure):
    _fields_ = [("eps_i", ctypes.c_double), ("v", ctypes.c_int * MAX_MODES), ("mu_i", ctypes.c_int),
                ("model", ctypes.c_int)]


_lib = None


def lib():
    """Load libvdc.so (raises if it is missing: no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libvdc.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sigs = {
        "vdc_model2d_create": (I, [ctypes.POINTER(ModelDesc), ctypes.POINTER(P)]),
        "vdc_model_destroy": (I, [P]),
        "vdc_workspace_size": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                   ctypes.POINTER(Job), ctypes.POINTER(S)]),
        "vdc_solve": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I, ctypes.POINTER(Job),
                          I, ctypes.POINTER(ctypes.c_int), P, S, P, P, P,
                          ctypes.POINTER(JobInfo), P]),
        "vdc_solve_history": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                  ctypes.POINTER(Job), I, ctypes.POINTER(ctypes.c_int), P, S, P, P,
                                  P, ctypes.POINTER(JobInfo), P, I, P]),
        "vdc_solve_noalloc": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                  ctypes.POINTER(Job), I, ctypes.POINTER(ctypes.c_int), P, P, P,
                                  ctypes.POINTER(JobInfo), P]),
        "vdc_solve_plain": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                ctypes.POINTER(Job), I, ctypes.POINTER(ctypes.c_int), P, S, P, P,
                                P, ctypes.POINTER(JobInfo), P]),
        "vdc_batch_create": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                 ctypes.POINTER(Job), I, ctypes.POINTER(ctypes.c_int), P, S, P, P,
                                 P, P, ctypes.POINTER(P)]),
        "vdc_batch_launch": (I, [P, P]),
        "vdc_batch_capture": (I, [P, P]),
        "vdc_batch_replay": (I, [P, P]),
        "vdc_batch_info": (I, [P, ctypes.POINTER(JobInfo), P]),
        "vdc_batch_kernel_times": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "vdc_batch_destroy": (I, [P]),
        "vdc_adjoint_workspace_size": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                           ctypes.POINTER(Job), ctypes.POINTER(S)]),
        "vdc_solve_adjoint": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                  ctypes.POINTER(Job), I, ctypes.POINTER(ctypes.c_int), P, P, P,
                                  P, S, P, ctypes.POINTER(D), ctypes.POINTER(JobInfo), P]),
        "vdc_level_shift": (I, [P, I, P, P, P]),
        "vdc_matvec_workspace_size": (I, [P, I, ctypes.POINTER(S)]),
        "vdc_matvec": (I, [P, D, I, ctypes.POINTER(ctypes.c_int), P, P, P, S, P]),
        "vdc_matvec_block_workspace_size": (I, [P, I, ctypes.POINTER(S)]),
        "vdc_matvec_block": (I, [P, D, I, ctypes.POINTER(ctypes.c_int), P, P, P, S, P]),
        "vdc_last_kernel_times": (I, [ctypes.POINTER(D), ctypes.POINTER(D)]),
        "vdc_co2_create": (I, [ctypes.POINTER(Co2Desc), ctypes.POINTER(P)]),
        "vdc_co2_destroy": (I, [P]),
        "vdc_co2_workspace_size": (I, [P, ctypes.POINTER(SolveOpts), I, ctypes.POINTER(Co2Job),
                                       ctypes.POINTER(S)]),
        "vdc_co2_solve": (I, [P, ctypes.POINTER(SolveOpts), I, ctypes.POINTER(Co2Job), I,
                              ctypes.POINTER(ctypes.c_int), P, P, P, ctypes.POINTER(JobInfo), P, S,
                              P]),
        "vdc_co2_ops_workspace_size": (I, [P, I, I, ctypes.POINTER(S)]),
        "vdc_co2_apply": (I, [P, D, I, I, ctypes.POINTER(ctypes.c_int), P, P, P, S, P]),
        "vdc_eels_workspace_size": (I, [P, I, ctypes.POINTER(S)]),
        "vdc_eels": (I, [P, I, ctypes.POINTER(Job), P, S, I, D, D, D, P, P, S, P]),
        "vdc_model_create": (I, [ctypes.POINTER(TermDesc), ctypes.POINTER(P)]),
        "vdc_model_kind": (I, [P, ctypes.POINTER(ctypes.c_int)]),
        "vdc_model_workspace_size": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                         ctypes.POINTER(MJob), ctypes.POINTER(S)]),
        "vdc_model_solve": (I, [I, ctypes.POINTER(P), ctypes.POINTER(SolveOpts), I,
                                ctypes.POINTER(MJob), I, ctypes.POINTER(ctypes.c_int), P, S, P, P,
                                P, ctypes.POINTER(JobInfo), P]),
        "vdc_model_apply_workspace_size": (I, [P, I, ctypes.POINTER(S)]),
        "vdc_model_apply": (I, [P, D, I, P, P, P, S, P]),
        "vdc_sum_partial_waves": (I, [I, P, I, I, P, P, P]),
        "vdc_last_error": (ctypes.c_char_p, []),
        "vdc_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code):
    if code != VDC_OK:
        raise VdcError(code, lib().vdc_last_error().decode())


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _aligned_workspace(nbytes, device):
    raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw[off:off + int(nbytes)]


class Model2D:
    """The generalized two-state model (vdc_model2d_create).  ``params`` uses
    the names of paper_2307_13483_amd.inputs (omega_g ... B2o, E1, l_e, l_o, K, X)."""

    def __init__(self, params, Ng, Nu):
        p = params
        d = ModelDesc()
        d.omega_g, d.omega_u = p["omega_g"], p["omega_u"]
        d.kappa1, d.kappa2, d.lam = p["kappa1"], p["kappa2"], p["lam"]
        d.lam1, d.lam2 = p["lam1"], p["lam2"]
        d.E1, d.gap = p["E1"], p["gap"]
        for s, st in enumerate(("1", "2")):
            for m, mu in enumerate(("e", "o")):
                d.A[s][m] = p["A" + st + mu]
                d.B[s][m] = p["B" + st + mu]
        d.l[0], d.l[1] = int(p["l_e"]), int(p["l_o"])
        d.Ng, d.Nu = int(Ng), int(Nu)
        d.hilbert_nodes, d.hilbert_xmax = int(p.get("K", 4096)), float(p.get("X", 40.0))
        self.desc = d
        self.params = dict(p)
        self.Ng, self.Nu = int(Ng), int(Nu)
        h = ctypes.c_void_p()
        _check(lib().vdc_model2d_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    @property
    def N(self):
        return 2 * self.Ng * self.Nu

    def close(self):
        if self.handle:
            lib().vdc_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Opts:
    restart: int = 50
    max_iter: int = 20000
    tol: float = 1e-10
    precond: int = PREC_BLOCK
    precision: int = FP64
    inner_restart: int = 8
    inner_tol: float = 1e-3
    outer_restart: int = 16
    tile_rows: int = 0
    method: int = GMRES
    check_optical: int = 0   # 1: every job's optical-theorem defect (JobInfo.optical_defect)

    def c(self):
        return SolveOpts(self.restart, self.max_iter, self.tol, self.precond, self.precision,
                         self.inner_restart, self.inner_tol, self.outer_restart, self.tile_rows,
                         self.method, int(self.check_optical))


def level_shift(model, eps):
    """vdc_level_shift: eps (1-D) -> complex128 [n, 6] on the GPU."""
    eps = torch.as_tensor(eps, dtype=torch.float64, device="cuda").contiguous()
    out = torch.empty((eps.numel(), 6), dtype=torch.complex128, device="cuda")
    _check(lib().vdc_level_shift(model.handle, eps.numel(), _ptr(eps), _ptr(out), _stream_ptr()))
    return out


def matvec(model, E, x, parity):
    """vdc_matvec: y = A(E) x for full-layout vectors x [n_vec, N] (complex128)."""
    x = torch.as_tensor(x, dtype=torch.complex128, device="cuda").contiguous()
    if x.dim() == 1:
        x = x[None]
    n_vec = x.shape[0]
    par = (ctypes.c_int * n_vec)(*[int(p) for p in parity])
    nb = ctypes.c_size_t()
    _check(lib().vdc_matvec_workspace_size(model.handle, n_vec, ctypes.byref(nb)))
    raw, ws = _aligned_workspace(nb.value, x.device)
    y = torch.empty_like(x)
    _check(lib().vdc_matvec(model.handle, float(E), n_vec, par, _ptr(x), _ptr(y), _ptr(ws),
                            nb.value, _stream_ptr()))
    return y


PARAM_NAMES = ("omega_g", "omega_u", "kappa1", "kappa2", "lam", "lam1", "lam2", "gap",
               "A1e", "A2e", "A1o", "A2o", "B1e", "B2e", "B1o", "B2o")


def matvec_block(model, E, x, parity, ws_cache=None):
    """vdc_matvec_block: y = A(E) x for block vectors x [n_vec, Ng*Nu] (complex128)."""
    x = torch.as_tensor(x, dtype=torch.complex128, device="cuda").contiguous()
    if x.dim() == 1:
        x = x[None]
    n_vec = x.shape[0]
    par = (ctypes.c_int * n_vec)(*[int(p) for p in parity])
    nb = ctypes.c_size_t()
    _check(lib().vdc_matvec_block_workspace_size(model.handle, n_vec, ctypes.byref(nb)))
    if ws_cache is not None and ws_cache.get("bytes", 0) >= nb.value:
        ws = ws_cache["ws"]
    else:
        raw, ws = _aligned_workspace(nb.value, x.device)
        if ws_cache is not None:
            ws_cache.update(bytes=nb.value, ws=ws, raw=raw)
    y = torch.empty_like(x)
    _check(lib().vdc_matvec_block(model.handle, float(E), n_vec, par, _ptr(x), _ptr(y), _ptr(ws),
                                  nb.value, _stream_ptr()))
    return y


def eels(model, jobs, psi, loss0, dloss, n_grid, fwhm=0.010):
    """vdc_eels: the 2D energy-loss spectrum (Eq. (17)) of each solved
    right-hand side.  jobs: tuples (eps_i, (n_g, n_u), mu_i) of one model;
    psi: device complex [n_jobs, 2 Ng Nu] full-layout solutions (e.g.
    Solver(..., want_psi=True).psi).  Returns S, device float64 [n_jobs, n_grid]
    on loss0 + j dloss; sum the rows of mu_i = e and o for the total."""
    n = len(jobs)
    arr = (Job * max(1, n))()
    for k, jb in enumerate(jobs):
        arr[k] = Job(float(jb[0]), int(jb[1][0]), int(jb[1][1]), int(jb[2]), 0)
    psi = psi.contiguous()
    S = torch.zeros((n, n_grid), dtype=torch.float64, device="cuda")
    nb = ctypes.c_size_t()
    _check(lib().vdc_eels_workspace_size(model.handle, n, ctypes.byref(nb)))
    raw, ws = _aligned_workspace(nb.value, "cuda")
    _check(lib().vdc_eels(model.handle, n, arr, _ptr(psi), psi.shape[1], int(n_grid), float(loss0),
                          float(dloss), float(fwhm), _ptr(S), _ptr(ws), nb.value, _stream_ptr()))
    return S


class Solver:
    """Holds a job list and a workspace; ``run`` calls vdc_solve (batched
    persistent launch) or vdc_solve_plain.  ``jobs`` are tuples
    (eps_i, (n_g, n_u), mu_i[, model index]); ``finals`` are (n_g, n_u)."""

    def __init__(self, models, jobs, finals, opts=None, want_psi=False):
        self.models = list(models) if isinstance(models, (list, tuple)) else [models]
        self.opts = opts or Opts()
        self.n_jobs = len(jobs)
        self.jobs = (Job * max(1, self.n_jobs))()
        for k, jb in enumerate(jobs):
            e, v, mu = jb[0], jb[1], jb[2]
            mi = jb[3] if len(jb) > 3 else 0
            self.jobs[k] = Job(float(e), int(v[0]), int(v[1]), int(mu), int(mi))
        self.n_final = len(finals)
        self.finals = (ctypes.c_int * max(2, 2 * self.n_final))(*[int(c) for f in finals for c in f])
        self.handles = (ctypes.c_void_p * len(self.models))(*[m.handle.value for m in self.models])
        self.copts = self.opts.c()
        nb = ctypes.c_size_t()
        _check(lib().vdc_workspace_size(len(self.models), self.handles, ctypes.byref(self.copts),
                                        self.n_jobs, self.jobs, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self._raw, self.ws = _aligned_workspace(self.ws_bytes, "cuda")
        nmax = max(m.N for m in self.models)
        self.T = torch.zeros((self.n_jobs, self.n_final, 2), dtype=torch.complex128, device="cuda")
        self.sigma = torch.zeros((self.n_jobs, self.n_final), dtype=torch.float64, device="cuda")
        self.psi = (torch.zeros((self.n_jobs, nmax), dtype=torch.complex128, device="cuda")
                    if want_psi else None)
        self.info = (JobInfo * max(1, self.n_jobs))()
        self.adj_ws = None

    def adjoint(self, dL_dsigma, stream=None):
        """vdc_solve_adjoint after run() with want_psi: dL_dsigma [n_jobs, n_final]
        (device) -> (grad over jobs as a numpy array [16], per-job [n_jobs, 16])."""
        if self.psi is None:
            raise ValueError("the adjoint needs the forward solutions: build with want_psi=True")
        if self.adj_ws is None:
            nb = ctypes.c_size_t()
            _check(lib().vdc_adjoint_workspace_size(len(self.models), self.handles,
                                                    ctypes.byref(self.copts), self.n_jobs,
                                                    self.jobs, ctypes.byref(nb)))
            self.adj_bytes = nb.value
            self._adj_raw, self.adj_ws = _aligned_workspace(nb.value, "cuda")
            self.grad_jobs = torch.zeros((self.n_jobs, 16), dtype=torch.float64, device="cuda")
            self.adj_info = (JobInfo * max(1, self.n_jobs))()
        dsig = torch.as_tensor(dL_dsigma, dtype=torch.float64, device="cuda").contiguous()
        g = (ctypes.c_double * 16)()
        _check(lib().vdc_solve_adjoint(len(self.models), self.handles, ctypes.byref(self.copts),
                                       self.n_jobs, self.jobs, self.n_final, self.finals,
                                       _ptr(self.psi), _ptr(self.T), _ptr(dsig), _ptr(self.adj_ws),
                                       self.adj_bytes, _ptr(self.grad_jobs), g, self.adj_info,
                                       _stream_ptr(stream)))
        return np.array(list(g)), self.grad_jobs

    def run_history(self, hist_len, stream=None):
        """vdc_solve_history: the solve with every job's relative residual after
        each step; returns the history [n_jobs, hist_len] (NaN past the end)."""
        hist = torch.full((self.n_jobs, int(hist_len)), float("nan"), dtype=torch.float64,
                          device="cuda")
        _check(lib().vdc_solve_history(len(self.models), self.handles, ctypes.byref(self.copts),
                                       self.n_jobs, self.jobs, self.n_final, self.finals,
                                       _ptr(self.ws), self.ws_bytes, _ptr(self.T), _ptr(self.sigma),
                                       _ptr(self.psi), self.info, _ptr(hist), int(hist_len),
                                       _stream_ptr(stream)))
        return hist

    def run_noalloc(self, stream=None):
        """vdc_solve_noalloc: the same solve in the library's static device
        scratch (this object's workspace is not used)."""
        _check(lib().vdc_solve_noalloc(len(self.models), self.handles, ctypes.byref(self.copts),
                                       self.n_jobs, self.jobs, self.n_final, self.finals,
                                       _ptr(self.T), _ptr(self.sigma), _ptr(self.psi), self.info,
                                       _stream_ptr(stream)))
        return self

    def run(self, plain=False, stream=None):
        f = lib().vdc_solve_plain if plain else lib().vdc_solve
        _check(f(len(self.models), self.handles, ctypes.byref(self.copts), self.n_jobs, self.jobs,
                 self.n_final, self.finals, _ptr(self.ws), self.ws_bytes, _ptr(self.T),
                 _ptr(self.sigma), _ptr(self.psi), self.info, _stream_ptr(stream)))
        return self

    def infos(self):
        out = [dict(status=self.info[k].status, iters=self.info[k].iters,
                    restarts=self.info[k].restarts, outer_iters=self.info[k].outer_iters,
                    rel_res=self.info[k].rel_res, alg_bytes=self.info[k].alg_bytes,
                    retried=self.info[k].retried, optical_defect=self.info[k].optical_defect)
               for k in range(self.n_jobs)]
        n_retry = sum(1 for i in out if i["retried"])
        if n_retry:
            _log.warning("%d of %d FP32-inner solves did not converge and were solved again "
                         "in FP64", n_retry, self.n_jobs)
        return out


class Batch(Solver):
    """vdc_batch_*: the Solver's jobs prepared once; ``launch`` enqueues the
    whole solve (kernels only), ``capture`` records that into a HIP graph on
    a stream of its own and ``replay`` launches the graph.  ``infos`` reads
    the per-job results of the last completed launch or replay."""

    def __init__(self, models, jobs, finals, opts=None, want_psi=False, stream=None):
        super().__init__(models, jobs, finals, opts, want_psi)
        self.handle = ctypes.c_void_p()
        _check(lib().vdc_batch_create(len(self.models), self.handles, ctypes.byref(self.copts),
                                      self.n_jobs, self.jobs, self.n_final, self.finals,
                                      _ptr(self.ws), self.ws_bytes, _ptr(self.T), _ptr(self.sigma),
                                      _ptr(self.psi), _stream_ptr(stream), ctypes.byref(self.handle)))

    def launch(self, stream=None):
        _check(lib().vdc_batch_launch(self.handle, _stream_ptr(stream)))
        return self

    def capture(self, stream):
        """Capture on ``stream`` (a torch.cuda.Stream, not the default one)."""
        _check(lib().vdc_batch_capture(self.handle, _stream_ptr(stream)))
        return self

    def replay(self, stream=None):
        _check(lib().vdc_batch_replay(self.handle, _stream_ptr(stream)))
        return self

    def infos(self, stream=None):
        _check(lib().vdc_batch_info(self.handle, self.info, _stream_ptr(stream)))
        return super().infos()

    def kernel_times(self):
        """(ms of the table kernels, ms of the solver) of the last launch."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().vdc_batch_kernel_times(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.vdc_batch_destroy(h)
            self.handle = None


def solve(models, jobs, finals, opts=None, plain=False, want_psi=False):
    """One-shot helper: returns (T, sigma, psi, infos) as torch/python objects."""
    s = Solver(models, jobs, finals, opts, want_psi).run(plain=plain)
    return s.T, s.sigma, s.psi, s.infos()


def last_kernel_times():
    """(ms of the table kernel, ms of the solver) of the last solve call."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().vdc_last_kernel_times(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


class CrossSections(torch.autograd.Function):
    """sigma_{v_f <- v_i}(eps_i) (Eq. (16), summed over mu_i and mu_f) as a
    differentiable function of the 16 model parameters (PARAM_NAMES order).

    forward(params [16] float64, spec) -> sigma [n_energies, n_final] on the GPU,
    where spec = dict(base=params dict, Ng, Nu, eps (list), v_i, finals, opts).
    backward: one adjoint solve per right-hand side (vdc_solve_adjoint).
    """

    @staticmethod
    def forward(ctx, params, spec):
        p = dict(spec["base"])
        for name, v in zip(PARAM_NAMES, params.detach().cpu().tolist()):
            p[name] = float(v)
        model = Model2D(p, spec["Ng"], spec["Nu"])
        jobs = [(e, spec["v_i"], mu) for e in spec["eps"] for mu in (0, 1)]
        s = Solver(model, jobs, spec["finals"], spec.get("opts"), want_psi=True).run()
        ctx.solver, ctx.model = s, model
        ctx.n_e, ctx.n_f = len(spec["eps"]), len(spec["finals"])
        # Eq. (16): the two mu_i shares of each energy, added by the library
        return sum_partial_waves([k // 2 for k in range(len(jobs))], ctx.n_e, s.sigma)

    @staticmethod
    def backward(ctx, grad_sigma):
        dsig = grad_sigma.to(torch.float64).contiguous()[:, None, :].expand(ctx.n_e, 2, ctx.n_f)
        g, _ = ctx.solver.adjoint(dsig.reshape(ctx.n_e * 2, ctx.n_f).contiguous())
        return torch.tensor(g, dtype=torch.float64), None


def version():
    return lib().vdc_version().decode()



# ---------------------------------------------------------------- CO2-like model

CO2_PARAMS = ("omega_s", "omega_b", "omega_a", "E_sigma", "E_pi", "k_sigma", "k_pi", "gs_sigma",
              "gb_sigma", "ga_sigma", "gs_pi", "gb_pi", "ga_pi", "c_rt", "c_sp", "c_sp2",
              "l_sigma", "l_pi", "h_sigma", "h_pi")


class Co2Model:
    """The CO2-like three-state, four-mode model (vdc_co2_create); ``params``
    uses the names of inputs.co2like_params, ``sizes`` the keys s, x, y, a."""

    def __init__(self, params, sizes):
        d = Co2Desc()
        for k in CO2_PARAMS:
            setattr(d, k, float(params[k]))
        for c, cn in enumerate(("sigma", "pi")):
            for w, wn in enumerate(("s", "p")):
                d.A[c][w] = float(params["A_%s_%s" % (cn, wn)])
                d.B[c][w] = float(params["B_%s_%s" % (cn, wn)])
        d.Ns, d.Nx, d.Ny, d.Na = (int(sizes[k]) for k in ("s", "x", "y", "a"))
        d.hilbert_nodes = int(params.get("K", 4096))
        d.hilbert_xmax = float(params.get("X", 40.0))
        self.sizes = dict(s=d.Ns, x=d.Nx, y=d.Ny, a=d.Na)
        self.npts = d.Ns * d.Nx * d.Ny * d.Na
        h = ctypes.c_void_p()
        _check(lib().vdc_co2_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vdc_co2_destroy(self.handle)
            self.handle = None


def co2_sector(v, mu):
    """Sector bits (px, py) of the right-hand side Phi^{v mu} (mu 0 s, 1 p_x, 2 p_y)."""
    return ((v[1] + (mu == 1)) & 1, (v[2] + (mu == 2)) & 1)


def co2_solve(model, jobs, finals, opts=None, want_psi=False, stream=None):
    """vdc_co2_solve.  jobs: (eps_i, (n_s, n_x, n_y, n_a), mu_i); finals: 4-tuples.
    Returns (T [n_jobs, n_final, 3], sigma [n_jobs, n_final], psi or None, infos)."""
    opts = opts or Opts(restart=20, precision=FP64)
    n = len(jobs)
    cj = (Co2Job * max(1, n))()
    for k, (e, v, mu) in enumerate(jobs):
        cj[k].eps_i = float(e)
        for q in range(4):
            cj[k].v[q] = int(v[q])
        cj[k].mu_i = int(mu)
    so = opts.c()
    ws = ctypes.c_size_t()
    _check(lib().vdc_co2_workspace_size(model.handle, ctypes.byref(so), n, cj, ctypes.byref(ws)))
    nf = len(finals)
    fin = (ctypes.c_int * max(1, 4 * nf))(*[int(c) for f in finals for c in f])
    T = torch.zeros((n, nf, 3), dtype=torch.complex128, device="cuda")
    sigma = torch.zeros((n, nf), dtype=torch.float64, device="cuda")
    psi = torch.zeros((n, model.npts), dtype=torch.complex128, device="cuda") if want_psi else None
    info = (JobInfo * max(1, n))()
    raw, w = _aligned_workspace(ws.value, "cuda")
    _check(lib().vdc_co2_solve(model.handle, ctypes.byref(so), n, cj, nf, fin, _ptr(T),
                               _ptr(sigma), _ptr(psi), info, _ptr(w), ws.value,
                               _stream_ptr(stream)))
    infos = [dict(status=info[k].status, iters=info[k].iters, restarts=info[k].restarts,
                  rel_res=info[k].rel_res, alg_bytes=info[k].alg_bytes) for k in range(n)]
    return T, sigma, psi, infos


def co2_apply(model, E, x, sectors, which=0, stream=None):
    """vdc_co2_apply: y = A(E) x (which 0) or the block preconditioner's
    M^{-1} x (which 1) for sector vectors x [n_vec, npts]."""
    x = torch.as_tensor(x, dtype=torch.complex128, device="cuda").contiguous()
    if x.dim() == 1:
        x = x[None]
    n = x.shape[0]
    sec = (ctypes.c_int * max(1, 2 * n))(*[int(b) for s_ in sectors for b in s_])
    ws = ctypes.c_size_t()
    _check(lib().vdc_co2_ops_workspace_size(model.handle, n, int(which), ctypes.byref(ws)))
    y = torch.empty_like(x)
    raw, w = _aligned_workspace(ws.value, "cuda")
    _check(lib().vdc_co2_apply(model.handle, float(E), int(which), n, sec, _ptr(x), _ptr(y),
                               _ptr(w), ws.value, _stream_ptr(stream)))
    return y


# ---------------------------------------------------------------- term-list models

class TermModel:
    """A model given by polynomial term lists (vdc_model_create).  ``desc``:
    dict with omega [M], nbasis [M], e_state [D], uterms / vterms as lists of
    (d, d' or mu, coeff, powers), width {(d, mu): (A, B)}, l [P], K, X (as
    paper_2307_13483_amd.inputs builds them).  dispatch: let the two-state
    kernels solve it when its terms are those of the two-state model."""

    def __init__(self, desc, dispatch=False):
        D, M, P = len(desc["e_state"]), len(desc["nbasis"]), len(desc["l"])
        self.D, self.M, self.P = D, M, P
        self.nbasis = [int(n) for n in desc["nbasis"]]
        self.npts = int(np.prod(self.nbasis))
        self._omega = (ctypes.c_double * M)(*[float(w) for w in desc["omega"]])
        self._nbasis = (ctypes.c_int * M)(*self.nbasis)
        self._estate = (ctypes.c_double * D)(*[float(e) for e in desc["e_state"]])

        def terms(lst):
            arr = (Term * max(1, len(lst)))()
            for k, (d, e, c, pw) in enumerate(lst):
                arr[k].d, arr[k].e, arr[k].coeff = int(d), int(e), float(c)
                for q, pq in enumerate(pw):
                    arr[k].pow[q] = int(pq)
            return arr
        self._u, self._v = terms(desc["uterms"]), terms(desc["vterms"])
        self._w = (Width * (D * P))()
        for dd in range(D):
            for mu in range(P):
                A, B = desc["width"].get((dd, mu), (0.0, 1.0))
                self._w[dd * P + mu] = Width(float(A), float(B), int(desc["l"][mu]))
        d = TermDesc(D, M, P, self._omega, self._nbasis, self._estate, len(desc["uterms"]),
                     self._u, len(desc["vterms"]), self._v, self._w, int(desc.get("K", 4096)),
                     float(desc.get("X", 40.0)), 1 if dispatch else 0)
        h = ctypes.c_void_p()
        _check(lib().vdc_model_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    @property
    def N(self):
        return self.D * self.npts

    def kind(self):
        k = ctypes.c_int()
        _check(lib().vdc_model_kind(self.handle, ctypes.byref(k)))
        return k.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vdc_model_destroy(self.handle)
            self.handle = None


def _mjobs(jobs):
    arr = (MJob * max(1, len(jobs)))()
    for k, jb in enumerate(jobs):
        arr[k].eps_i = float(jb[0])
        for q, vq in enumerate(jb[1]):
            arr[k].v[q] = int(vq)
        arr[k].mu_i = int(jb[2])
        arr[k].model = int(jb[3]) if len(jb) > 3 else 0
    return arr


def model_solve(models, jobs, finals, opts=None, want_psi=False, stream=None):
    """vdc_model_solve.  jobs: (eps_i, v (multi-index), mu_i[, model index]);
    finals: multi-indices.  Returns (T [n_jobs, n_final, P], sigma shares
    [n_jobs, n_final], psi [n_jobs, max N] or None, infos)."""
    models = list(models) if isinstance(models, (list, tuple)) else [models]
    opts = opts or Opts(precond=PREC_JACOBI)
    n = len(jobs)
    cj = _mjobs(jobs)
    hs = (ctypes.c_void_p * len(models))(*[m.handle.value for m in models])
    so = opts.c()
    nb = ctypes.c_size_t()
    _check(lib().vdc_model_workspace_size(len(models), hs, ctypes.byref(so), n, cj, ctypes.byref(nb)))
    nf = len(finals)
    fin = (ctypes.c_int * max(1, MAX_MODES * nf))()
    for f, vf in enumerate(finals):
        for q, vq in enumerate(vf):
            fin[f * MAX_MODES + q] = int(vq)
    two_state = all(m.kind() == 0 for m in models)
    P = 2 if two_state else max(m.P for m in models)
    T = torch.zeros((n, nf, P), dtype=torch.complex128, device="cuda")
    sigma = torch.zeros((n, nf), dtype=torch.float64, device="cuda")
    psi = (torch.zeros((n, max(m.N for m in models)), dtype=torch.complex128, device="cuda")
           if want_psi else None)
    info = (JobInfo * max(1, n))()
    raw, ws = _aligned_workspace(nb.value, "cuda")
    _check(lib().vdc_model_solve(len(models), hs, ctypes.byref(so), n, cj, nf, fin, _ptr(ws),
                                 nb.value, _ptr(T), _ptr(sigma), _ptr(psi), info,
                                 _stream_ptr(stream)))
    infos = [dict(status=info[k].status, iters=info[k].iters, restarts=info[k].restarts,
                  rel_res=info[k].rel_res, alg_bytes=info[k].alg_bytes, retried=info[k].retried,
                  optical_defect=info[k].optical_defect)
             for k in range(n)]
    return T, sigma, psi, infos


def model_apply(model, E, x, stream=None):
    """vdc_model_apply: y = A(E) x for full-layout vectors x [n_vec, N]."""
    x = torch.as_tensor(x, dtype=torch.complex128, device="cuda").contiguous()
    if x.dim() == 1:
        x = x[None]
    n = x.shape[0]
    nb = ctypes.c_size_t()
    _check(lib().vdc_model_apply_workspace_size(model.handle, n, ctypes.byref(nb)))
    raw, ws = _aligned_workspace(nb.value, "cuda")
    y = torch.empty_like(x)
    _check(lib().vdc_model_apply(model.handle, float(E), n, _ptr(x), _ptr(y), _ptr(ws), nb.value,
                                 _stream_ptr(stream)))
    return y


def sum_partial_waves(collision, n_coll, share, stream=None):
    """vdc_sum_partial_waves: sigma [n_coll, n_final] of Eq. (16) from the
    per-job shares [n_jobs, n_final] (device) and each job's collision index."""
    share = share.contiguous()
    coll = torch.as_tensor(list(collision), dtype=torch.int32, device=share.device)
    sig = torch.zeros((int(n_coll), share.shape[1]), dtype=torch.float64, device=share.device)
    _check(lib().vdc_sum_partial_waves(share.shape[0], _ptr(coll), int(n_coll), share.shape[1],
                                       _ptr(share), _ptr(sig), _stream_ptr(stream)))
    return sig
