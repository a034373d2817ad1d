"""ctypes binding of libhsrom.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts torch
tensors (float64 / int32 / uint8, contiguous, on the context's device) into
pointers and checks status codes.  Importing it without a built library
raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhsrom.so")

HS_OK = 0
STATUS = {0: "HS_OK", -1: "HS_ERR_INVALID_ARG", -2: "HS_ERR_SHAPE", -3: "HS_ERR_NOT_CONVERGED",
          -4: "HS_ERR_RANK", -5: "HS_ERR_NONFINITE", -6: "HS_ERR_HIP", -7: "HS_ERR_OOM"}
HS_ERR_NOT_CONVERGED = -3
HS_ERR_RANK = -4

BURGERS_1D, BURGERS_2D, EULER_2D = 0, 1, 2
RULE_FRACTION, RULE_RRE = 0, 1
TAPE_RECORD, TAPE_REPLAY = 0, 1
FP64, MIXED_FP32 = 0, 1


class HsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dt", ctypes.c_double), ("gamma", ctypes.c_double), ("inflow", ctypes.c_double),
                ("newton_rtol", ctypes.c_double), ("newton_maxit", ctypes.c_int32),
                ("lin_rtol", ctypes.c_double), ("lin_maxit", ctypes.c_int32),
                ("m_max", ctypes.c_int32), ("w_max", ctypes.c_int32)]


class StepInfo(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("lin_sweeps", ctypes.c_int32),
                ("subiters", ctypes.c_int32), ("filter_passes", ctypes.c_int32),
                ("filter_kept", ctypes.c_int32), ("n_s", ctypes.c_int32), ("l", ctypes.c_int32),
                ("fit_rank", ctypes.c_int32), ("residual_inf", ctypes.c_double),
                ("dy_last", ctypes.c_double), ("fit_cond", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SampleParams(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("fraction", ctypes.c_double),
                ("delta", ctypes.c_double), ("halo", ctypes.c_int32)]


class HybridParams(ctypes.Structure):
    _fields_ = [("eps_y", ctypes.c_double), ("jmax", ctypes.c_int32), ("n_orders", ctypes.c_int32),
                ("filter_orders", ctypes.c_int32 * 4), ("eps_f", ctypes.c_double),
                ("jfmax", ctypes.c_int32), ("rcond_fit", ctypes.c_double),
                ("floor_rel", ctypes.c_double), ("precision", ctypes.c_int32)]


class TrajParams(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32), ("w", ctypes.c_int32),
                ("m", ctypes.c_int32), ("z", ctypes.c_int32), ("tau_pod", ctypes.c_double),
                ("sample", SampleParams), ("hybrid", HybridParams), ("psi_adjoint", ctypes.c_int32)]


PAPER_BC_FIXED, PAPER_BC_WALL = 0, 1   # HS_PAPER_BC_*


class PaperHDM(ctypes.Structure):
    _fields_ = [("bc", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ghost", (ctypes.c_double * 4) * 4)]


def paper_hdm(bc=PAPER_BC_FIXED, ghost=()) -> PaperHDM:
    """Boundary data of the paper's scheme: ghost = up to four conservative
    4-vectors (left, right, bottom, top) for PAPER_BC_FIXED."""
    h = PaperHDM()
    h.bc = bc
    for s, g in enumerate(ghost):
        for a in range(4):
            h.ghost[s][a] = float(g[a])
    return h


def hybrid_params(eps_y=1e-4, jmax=10, filter_orders=(1, 2, 3), eps_f=1e-2, jfmax=10,
                  rcond_fit=1e-8, floor_rel=1e-14, precision=FP64) -> HybridParams:
    hp = HybridParams()
    hp.eps_y, hp.jmax, hp.eps_f, hp.jfmax = eps_y, jmax, eps_f, jfmax
    hp.rcond_fit, hp.floor_rel, hp.precision = rcond_fit, floor_rel, precision
    hp.n_orders = len(filter_orders)
    for i, o in enumerate(filter_orders):
        hp.filter_orders[i] = o
    return hp


_lib = None
P = ctypes.c_void_p
I32 = ctypes.c_int32
D = ctypes.c_double

_SIGS = {
    "hs_create": [ctypes.POINTER(Problem), P, ctypes.POINTER(P)],
    "hs_destroy": [P],
    "hs_sync": [P],
    "hs_status_string": [I32],
    "hs_last_error": [P],
    "hs_residual": [P, P, P, P],
    "hs_stream_add": [P, P, P, P, ctypes.c_int64],
    "hs_jvp": [P, P, P, P],
    "hdm_step": [P, P, P, ctypes.POINTER(StepInfo)],
    "hs_paper_residual": [P, ctypes.POINTER(PaperHDM), P, P, P, P],
    "hdm_step_bdf2": [P, ctypes.POINTER(PaperHDM), P, P, P, ctypes.POINTER(StepInfo)],
    "rom_hybrid_step_bdf2": [P, ctypes.POINTER(PaperHDM), P, P, P, P, I32, P, P, I32, ctypes.POINTER(HybridParams),
                             P, P, P, ctypes.POINTER(StepInfo)],
    "hs_odeim": [P, P, I32, I32, P],
    "rom_hybrid_step_fit": [P, P, P, P, I32, P, P, I32, ctypes.POINTER(HybridParams), P, P, P,
                            ctypes.POINTER(StepInfo)],
    "rom_hybrid_step_gn": [P, P, P, P, I32, P, ctypes.POINTER(HybridParams), P, P, P, P, ctypes.POINTER(StepInfo)],
    "hs_samples_add_points": [P, P, P, I32],
    "hs_samples_create": [P, ctypes.POINTER(P)],
    "hs_samples_destroy": [P],
    "sample_select": [P, P, ctypes.POINTER(SampleParams), P],
    "hs_samples_set": [P, P, P, I32],
    "hs_samples_counts": [P, ctypes.POINTER(I32)],
    "hs_samples_export": [P, P, P, P, P],
    "hs_indicator_full": [P, P, P, P, I32, D, I32, P, P],
    "hs_indicator_full_noalloc": [P, I32, I32, P, P, P, I32, D, I32, P, P],
    "basis_update": [P, ctypes.POINTER(P), I32, I32, I32, D, I32, P, P, P, ctypes.POINTER(I32)],
    "basis_update_async": [P, ctypes.POINTER(P), I32, I32, I32, D, I32, P, P, P],
    "basis_update_finish": [P, ctypes.POINTER(I32)],
    "hs_basis_m_eff": [P, ctypes.POINTER(I32)],
    "rom_hybrid_step": [P, P, P, P, I32, P, ctypes.POINTER(HybridParams), P, P, P,
                        ctypes.POINTER(StepInfo)],
    "hs_filter": [P, P, P, ctypes.POINTER(HybridParams), P, ctypes.POINTER(StepInfo)],
    "hs_htape_create": [P, ctypes.POINTER(P)],
    "hs_htape_destroy": [P],
    "hs_htape_info": [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32), P],
    "hs_htape_samples": [P, ctypes.POINTER(P)],
    "rom_hybrid_step_taped": [P, P, P, P, I32, P, ctypes.POINTER(HybridParams), P, P,
                              ctypes.POINTER(StepInfo), P, I32],
    "hdm_step_adjoint": [P, P, P, P, ctypes.POINTER(StepInfo)],
    "rom_hybrid_step_adjoint": [P, P, I32, P, P, P, ctypes.POINTER(StepInfo)],
    "rom_hybrid_step_adjoint_psi": [P, P, I32, P, P, P, P, ctypes.POINTER(StepInfo)],
    "hs_tape_create": [P, ctypes.POINTER(P)],
    "hs_tape_destroy": [P],
    "hs_traj_forward": [P, P, ctypes.POINTER(TrajParams), P, P],
    "hs_traj_backward": [P, P, P, P],
    "hs_tape_step": [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(P)],
    "hs_tape_basis": [P, P, I32, P, P, ctypes.POINTER(I32)],
    "hs_tape_checkpoint": [P, P, I32, P],
    "hs_set_option": [P, I32, ctypes.c_int64],
    "hs_prof_enable": [P, I32],
    "hs_prof_read": [P, ctypes.POINTER(D), ctypes.POINTER(I32), ctypes.POINTER(D)],
}

BASIS_PENDING = -1   # rom_hybrid_step's m for a basis still being formed (HS_BASIS_PENDING)

PROF_CLASSES = {"basis_gram": 1, "basis_form": 2, "recon": 3, "resjac": 4, "sweep": 5, "cellres": 6, "basis_pgram": 9,
                "filter": 7, "residual": 8, "stream": 10}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2301_01718_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name in ("hs_status_string", "hs_last_error") else I32
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def indicator_full_noalloc(gamma, Phi, psi, m, ncell, ncomp, eps, y=None, floor_rel=1e-14, stream=None):
    """hs_indicator_full_noalloc: the indicator of a full snapshot with no
    context and no allocation (the library's own device scratch array), on
    ``stream`` (default: torch's current stream).  ``eps`` (ncell doubles)
    and ``y`` (m doubles, optional) are caller-owned outputs."""
    import torch
    prec = basis_precision(Phi)
    if stream is None:
        stream = torch.cuda.current_stream(gamma.device).cuda_stream
    st = lib().hs_indicator_full_noalloc(ctypes.c_void_p(stream), ncell, ncomp, _ptr(gamma), _ptr(Phi), _ptr(psi),
                                         m, floor_rel, prec, _ptr(eps), _ptr(y))
    if st != 0:
        raise HsError(st, f"hs_indicator_full_noalloc: {lib().hs_status_string(st).decode()}")


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def basis_precision(Phi):
    """FP64 for a float64 basis, MIXED_FP32 for its float32 master copy."""
    if Phi.dtype == torch.float64:
        return FP64
    if Phi.dtype == torch.float32:
        return MIXED_FP32
    raise ValueError(f"basis must be float64 or float32, got {Phi.dtype}")


def _with_precision(params, prec):
    if params.precision == prec:
        return params
    hp = HybridParams()
    ctypes.pointer(hp)[0] = params
    hp.precision = prec
    return hp


class SnapshotTable:
    """Device addresses of a fixed list of snapshots of one context (checked
    when built; the tensors are kept alive with it)."""

    __slots__ = ("ctx", "arr", "count", "_keep")

    def __init__(self, ctx, snaps):
        self.ctx = ctx
        self._keep = list(snaps)
        self.arr = (P * len(self._keep))(*[P(ctx._in(t).data_ptr()) for t in self._keep])
        self.count = len(self._keep)


class Context:
    """One problem on one device and stream.  Tensors are float64 (states),
    int32 (cell lists) or uint8 (masks), contiguous, on ``device``."""

    def __init__(self, prob, m_max=64, w_max=64, device="cuda", stream=None,
                 newton_rtol=0.0, newton_maxit=0, lin_rtol=0.0, lin_maxit=0):
        d = torch.device(device)
        if d.type == "cuda" and d.index is None:
            d = torch.device("cuda", torch.cuda.current_device())
        self.device = d
        self.prob = prob
        p = Problem(kind=prob.kind, nx=prob.nx, ny=prob.ny, bc=prob.bc, dx=prob.dx, dy=prob.dy,
                    dt=prob.dt, gamma=prob.gamma, inflow=prob.inflow, newton_rtol=newton_rtol,
                    newton_maxit=newton_maxit, lin_rtol=lin_rtol, lin_maxit=lin_maxit,
                    m_max=m_max, w_max=w_max)
        self.m_max, self.w_max = m_max, w_max
        self.ncomp = 4 if prob.kind == EULER_2D else 1
        self.ncell = prob.nx * prob.ny
        self.n = self.ncomp * self.ncell
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            h = P()
            self._check(lib().hs_create(ctypes.byref(p), P(s.cuda_stream), ctypes.byref(h)), None)
            self.h = h

    def _check(self, st, h=None):
        if st != HS_OK:
            msg = lib().hs_last_error(h if h is not None else self.h)
            raise HsError(st, (msg or b"").decode())

    def close(self):
        if getattr(self, "h", None):
            lib().hs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, n=None, dtype=torch.float64):
        return torch.empty(self.n if n is None else n, dtype=dtype, device=self.device)

    def _in(self, t, n=None, dtype=torch.float64):
        n = self.n if n is None else n
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != n or t.device != self.device:
            raise ValueError(f"expected contiguous {dtype} tensor of {n} elements on {self.device}")
        return t

    def sync(self):
        self._check(lib().hs_sync(self.h))

    def set_tiled_sweeps(self, mode):
        """Relaxation sweeps: False = one sweep per launch over the cell list;
        True = LDS tiles where they pay (default); "always" = tiles wherever
        they fit.  The iterates are the same bit for bit."""
        v = 2 if mode == "always" else (1 if mode else 0)
        self._check(lib().hs_set_option(self.h, 1, v))

    def set_small_pinv(self, on):
        """The fit's pseudo-inverse for m <= 8: True = one wavefront with the
        matrix in registers (default); False = the general LDS routine.  The
        results are the same bit for bit."""
        self._check(lib().hs_set_option(self.h, 2, 1 if on else 0))

    def set_fit_cholesky(self, on):
        """The fit's pseudo-inverse for m > 8: True = the Cholesky inverse when
        a condition bound shows nothing is cut (default); False = always the
        Jacobi eigendecomposition."""
        self._check(lib().hs_set_option(self.h, 3, 1 if on else 0))

    # ---------------------------------------------------------- measurement
    def prof_enable(self, kernel_class):
        cls = PROF_CLASSES[kernel_class] if isinstance(kernel_class, str) else kernel_class
        self._check(lib().hs_prof_enable(self.h, cls))

    def prof_read(self):
        ms, n, b = D(0), I32(0), D(0)
        self._check(lib().hs_prof_read(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    # ----------------------------------------------------------- kernels
    def residual(self, q, q_prev, out=None):
        out = self.empty() if out is None else out
        self._check(lib().hs_residual(self.h, _ptr(self._in(q)), _ptr(self._in(q_prev)), _ptr(self._in(out))))
        return out

    def stream_add(self, a, b, out):
        """hs_stream_add: out = a + b (float64, equal sizes; the streaming reference)."""
        n = a.numel()
        self._check(lib().hs_stream_add(self.h, _ptr(self._in(a, n)), _ptr(self._in(b, n)),
                                        _ptr(self._in(out, n)), n))
        return out

    def jvp(self, q, v, out=None):
        out = self.empty() if out is None else out
        self._check(lib().hs_jvp(self.h, _ptr(self._in(q)), _ptr(self._in(v)), _ptr(self._in(out))))
        return out

    def hdm_step(self, q_prev, out=None):
        out = self.empty() if out is None else out
        info = StepInfo()
        self._check(lib().hdm_step(self.h, _ptr(self._in(q_prev)), _ptr(self._in(out)), ctypes.byref(info)))
        return out, info.as_dict()

    def paper_residual(self, hdm, q, q_prev, q_prev2=None, out=None):
        """The paper's BDF2 residual (BDF1 without q_prev2); hdm: PaperHDM."""
        out = self.empty() if out is None else out
        p2 = None if q_prev2 is None else _ptr(self._in(q_prev2))
        self._check(lib().hs_paper_residual(self.h, ctypes.byref(hdm), _ptr(self._in(q)), _ptr(self._in(q_prev)),
                                            p2, _ptr(self._in(out))))
        return out

    def hdm_step_bdf2(self, hdm, q_prev, q_prev2=None, out=None):
        """One step of the paper's scheme; returns (q, info)."""
        out = self.empty() if out is None else out
        info = StepInfo()
        p2 = None if q_prev2 is None else _ptr(self._in(q_prev2))
        self._check(lib().hdm_step_bdf2(self.h, ctypes.byref(hdm), _ptr(self._in(q_prev)), p2,
                                        _ptr(self._in(out)), ctypes.byref(info)))
        return out, info.as_dict()

    # ----------------------------------------------------------- sampling
    def samples(self):
        return Samples(self)

    def sample_select(self, eps, fraction, halo=2, samples=None, rule=RULE_FRACTION, delta=0.9):
        s = samples or Samples(self)
        sp = SampleParams(rule=rule, fraction=fraction, delta=delta, halo=halo)
        self._check(lib().sample_select(self.h, _ptr(self._in(eps, self.ncell)), ctypes.byref(sp), s.h))
        return s

    def samples_set(self, hat, samples=None):
        s = samples or Samples(self)
        hat = self._in(hat, hat.numel(), torch.int32)
        self._check(lib().hs_samples_set(self.h, s.h, _ptr(hat) if hat.numel() else None, hat.numel()))
        return s

    def _basis(self, Phi, m):
        # m = BASIS_PENDING: the basis an asynchronous update is forming (up to m_max modes)
        m = self.m_max if m == BASIS_PENDING else m
        if not Phi.is_contiguous() or Phi.numel() < m * self.n or Phi.device != self.device:
            raise ValueError(f"basis must be a contiguous tensor of at least {m} x {self.n} entries on {self.device}")
        return basis_precision(Phi)

    def indicator_full(self, gamma, Phi, psi, m, floor_rel=1e-14, eps=None, y=None):
        prec = self._basis(Phi, m)
        eps = self.empty(self.ncell) if eps is None else self._in(eps, self.ncell)
        y = self.empty(m) if y is None else y
        self._check(lib().hs_indicator_full(self.h, _ptr(self._in(gamma)), _ptr(Phi), _ptr(self._in(psi)), m,
                                            floor_rel, prec, _ptr(eps), _ptr(y)))
        return eps, y

    # ------------------------------------------------------------- basis
    def snapshot_table(self, snaps):
        """The device addresses of a list of snapshots, checked once; pass it
        to basis_update(_async) in place of the list while the tensors live."""
        return SnapshotTable(self, snaps)

    def _snap_array(self, snaps):
        if isinstance(snaps, SnapshotTable):
            if snaps.ctx is not self:
                raise ValueError("snapshot table of another context")
            return snaps.arr, snaps.count
        return (P * len(snaps))(*[P(self._in(s).data_ptr()) for s in snaps]), len(snaps)

    def basis_update(self, snaps, w, m, Phi_out, psi_out, sigma_out, tau_pod=1e-8):
        """Phi_out float64: FP64 basis; float32: the FP32 master copy (HS_MIXED_FP32)."""
        precision = self._basis(Phi_out, m)
        arr, count = self._snap_array(snaps)
        me = I32(0)
        self._check(lib().basis_update(self.h, arr, count, w, m, tau_pod, precision, _ptr(Phi_out),
                                       _ptr(self._in(psi_out)), _ptr(sigma_out), ctypes.byref(me)))
        return me.value

    def basis_update_async(self, snaps, w, m, Phi_out, psi_out, sigma_out, tau_pod=1e-8):
        """Enqueue the update on the context's own stream; finish with basis_update_finish."""
        precision = self._basis(Phi_out, m)
        arr, count = self._snap_array(snaps)
        self._check(lib().basis_update_async(self.h, arr, count, w, m, tau_pod, precision, _ptr(Phi_out),
                                             _ptr(self._in(psi_out)), _ptr(sigma_out)))
        self._pending = True

    def basis_pending(self):
        """Whether an asynchronous basis update is in flight."""
        return getattr(self, "_pending", False)

    def basis_m_eff(self):
        """m_eff of the last completed basis update."""
        me = I32(0)
        self._check(lib().hs_basis_m_eff(self.h, ctypes.byref(me)))
        return me.value

    def basis_update_finish(self):
        me = I32(0)
        self._pending = False
        self._check(lib().basis_update_finish(self.h, ctypes.byref(me)))
        return me.value

    # -------------------------------------------------------------- hybrid
    def rom_hybrid_step(self, q_prev, Phi, psi, m, samples, params=None, out=None, eps=None, y=None,
                        fit_points=None):
        """One hybrid step; fit_points (int32 state entries): the fit's rows
        (rom_hybrid_step_fit), else every entry of the sampled cells."""
        params = _with_precision(params or hybrid_params(), self._basis(Phi, m))
        out = self.empty() if out is None else out
        info = StepInfo()
        try:
            if fit_points is not None:
                nf = fit_points.numel()
                self._check(lib().rom_hybrid_step_fit(self.h, _ptr(self._in(q_prev)), _ptr(Phi), _ptr(self._in(psi)),
                                                      m, samples.h, _ptr(self._in(fit_points, nf, torch.int32)), nf,
                                                      ctypes.byref(params), _ptr(self._in(out)), _ptr(eps), _ptr(y),
                                                      ctypes.byref(info)))
            else:
                self._check(lib().rom_hybrid_step(self.h, _ptr(self._in(q_prev)), _ptr(Phi), _ptr(self._in(psi)),
                                                  m, samples.h, ctypes.byref(params), _ptr(self._in(out)),
                                                  _ptr(eps), _ptr(y), ctypes.byref(info)))
        finally:
            if m == BASIS_PENDING:
                self._pending = False        # the step completes the update on every path
        return out, info.as_dict()

    def rom_hybrid_step_bdf2(self, hdm, q_prev, q_prev2, Phi, psi, m, samples, params=None, out=None, eps=None,
                             y=None, fit_points=None):
        """rom_hybrid_step with the paper's scheme (hdm: PaperHDM; q_prev2 may
        be None; fit_points: int32 state entries for the fit, or None)."""
        params = _with_precision(params or hybrid_params(), self._basis(Phi, m))
        out = self.empty() if out is None else out
        info = StepInfo()
        p2 = None if q_prev2 is None else _ptr(self._in(q_prev2))
        nf = 0 if fit_points is None else fit_points.numel()
        fp = None if fit_points is None else _ptr(self._in(fit_points, nf, torch.int32))
        self._check(lib().rom_hybrid_step_bdf2(self.h, ctypes.byref(hdm), _ptr(self._in(q_prev)), p2, _ptr(Phi),
                                               _ptr(self._in(psi)), m, samples.h, fp, nf, ctypes.byref(params),
                                               _ptr(self._in(out)), _ptr(eps), _ptr(y), ctypes.byref(info)))
        return out, info.as_dict()

    def rom_hybrid_step_gn(self, q_prev, Phi, psi, m, samples, params=None, out=None, eps=None, y=None, work=None):
        """The hybrid step with Gauss-Newton subiterations (FP64 basis)."""
        params = _with_precision(params or hybrid_params(), FP64)
        if Phi.dtype != torch.float64 or not Phi.is_contiguous() or Phi.numel() < m * self.n:
            raise ValueError("Gauss-Newton subiterations need a contiguous float64 basis of at least m x N entries")
        out = self.empty() if out is None else out
        work = self.empty(m * self.n) if work is None else work[: m * self.n]   # at least m N doubles
        info = StepInfo()
        self._check(lib().rom_hybrid_step_gn(self.h, _ptr(self._in(q_prev)), _ptr(Phi), _ptr(self._in(psi)), m,
                                             samples.h, ctypes.byref(params), _ptr(self._in(work, m * self.n)),
                                             _ptr(self._in(out)), _ptr(eps), _ptr(y), ctypes.byref(info)))
        return out, info.as_dict()

    def odeim(self, Phi, m, n_p, out=None):
        """hs_odeim: n_p ODEIM points (int32 state entries, in the order taken)."""
        if Phi.dtype != torch.float64 or not Phi.is_contiguous() or Phi.numel() < m * self.n:
            raise ValueError("ODEIM needs a contiguous float64 basis of at least m x N entries")
        out = torch.empty(n_p, dtype=torch.int32, device=self.device) if out is None else out
        self._check(lib().hs_odeim(self.h, _ptr(Phi), m, n_p, _ptr(self._in(out, n_p, torch.int32))))
        return out

    def samples_add_points(self, samples, points):
        self._check(lib().hs_samples_add_points(self.h, samples.h, _ptr(self._in(points, points.numel(), torch.int32)),
                                                points.numel()))
        return samples

    def filter(self, gamma, q_prev, params=None, out=None):
        params = params or hybrid_params()
        out = self.empty() if out is None else out
        info = StepInfo()
        self._check(lib().hs_filter(self.h, _ptr(self._in(gamma)), _ptr(self._in(q_prev)), ctypes.byref(params),
                                    _ptr(self._in(out)), ctypes.byref(info)))
        return out, info.as_dict()


    # ------------------------------------------------------------- adjoint
    def tape(self):
        return Tape(self)

    def rom_hybrid_step_taped(self, q_prev, Phi, psi, m, tape, mode, samples=None, params=None, out=None,
                              eps=None):
        params = _with_precision(params or hybrid_params(), self._basis(Phi, m))
        out = self.empty() if out is None else out
        info = StepInfo()
        try:
            self._check(lib().rom_hybrid_step_taped(self.h, _ptr(self._in(q_prev)), _ptr(Phi), _ptr(self._in(psi)),
                                                    m, samples.h if samples is not None else None,
                                                    ctypes.byref(params), _ptr(self._in(out)), _ptr(eps),
                                                    ctypes.byref(info), tape.h, mode))
        finally:
            if m == BASIS_PENDING:
                self._pending = False
        return out, info.as_dict()

    def hdm_step_adjoint(self, q_out, lam, out=None):
        out = self.empty() if out is None else out
        info = StepInfo()
        self._check(lib().hdm_step_adjoint(self.h, _ptr(self._in(q_out)), _ptr(self._in(lam)), _ptr(self._in(out)),
                                           ctypes.byref(info)))
        return out, info.as_dict()

    def rom_hybrid_step_adjoint(self, Phi, m, tape, lam, out=None):
        out = self.empty() if out is None else out
        info = StepInfo()
        self._check(lib().rom_hybrid_step_adjoint(self.h, _ptr(Phi), m, tape.h, _ptr(self._in(lam)),
                                                  _ptr(self._in(out)), ctypes.byref(info)))
        return out, info.as_dict()

    def rom_hybrid_step_adjoint_psi(self, Phi, m, tape, lam, out=None, lam_psi=None):
        """(lambda_{k-1}, lambda_psi, info): the step adjoint and its part with
        respect to the step's reference state psi."""
        out = self.empty() if out is None else out
        lam_psi = self.empty() if lam_psi is None else lam_psi
        info = StepInfo()
        self._check(lib().rom_hybrid_step_adjoint_psi(self.h, _ptr(Phi), m, tape.h, _ptr(self._in(lam)),
                                                      _ptr(self._in(out)), _ptr(self._in(lam_psi)),
                                                      ctypes.byref(info)))
        return out, lam_psi, info.as_dict()


class Tape:
    """Library-owned record of one hybrid step's frozen decisions (``handle``:
    a tape borrowed from a trajectory tape, which owns and frees it)."""

    def __init__(self, ctx: Context, handle=None, owner=None):
        self.ctx = ctx
        self.owner = owner
        if handle is not None:
            self.h = handle
            self.borrowed = True
            return
        self.borrowed = False
        h = P()
        ctx._check(lib().hs_htape_create(ctx.h, ctypes.byref(h)))
        self.h = h

    def info(self):
        """(J, [(n, kept-cell mask tensor), ...]) of the recorded step."""
        J, npass = I32(0), I32(0)
        passes = (I32 * 64)()
        self.ctx._check(lib().hs_htape_info(self.h, ctypes.byref(J), ctypes.byref(npass), passes, None))
        masks = torch.empty(max(npass.value, 1) * self.ctx.ncell, dtype=torch.uint8, device=self.ctx.device)
        self.ctx._check(lib().hs_htape_info(self.h, None, None, None, _ptr(masks)))
        nc = self.ctx.ncell
        return J.value, [(passes[k], masks[k * nc:(k + 1) * nc]) for k in range(npass.value)]

    def samples(self):
        """The sampled set the tape holds (owned by the tape)."""
        h = P()
        self.ctx._check(lib().hs_htape_samples(self.h, ctypes.byref(h)))
        return Samples(self.ctx, handle=h, owner=self)

    def close(self):
        if getattr(self, "h", None):
            if not getattr(self, "borrowed", False):
                lib().hs_htape_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Samples:
    """Library-owned sampled sets (hat-S, tilde-S, mask)."""

    def __init__(self, ctx: Context, handle=None, owner=None):
        self.ctx = ctx
        self.owner = owner          # set for a set borrowed from another object
        if handle is None:
            handle = P()
            ctx._check(lib().hs_samples_create(ctx.h, ctypes.byref(handle)))
        self.h = handle

    def counts(self):
        c = (I32 * 3)()
        self.ctx._check(lib().hs_samples_counts(self.h, c))
        return {"n_g": c[0], "n_s": c[1], "l": c[2]}

    def export(self):
        c = self.counts()
        hat = torch.empty(max(c["n_s"], 1), dtype=torch.int32, device=self.ctx.device)
        tilde = torch.empty(max(c["l"], 1), dtype=torch.int32, device=self.ctx.device)
        mask = torch.empty(self.ctx.ncell, dtype=torch.uint8, device=self.ctx.device)
        self.ctx._check(lib().hs_samples_export(self.ctx.h, self.h, _ptr(hat), _ptr(tilde), _ptr(mask)))
        return hat[:c["n_s"]], tilde[:c["l"]], mask

    def close(self):
        if getattr(self, "h", None):
            if self.owner is None:
                lib().hs_samples_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TrajTape:
    """Library-owned record of one run of hs_traj_forward (hs_tape)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        h = P()
        ctx._check(lib().hs_tape_create(ctx.h, ctypes.byref(h)))
        self.h = h

    def step(self, k):
        """(kind, basis index, borrowed Tape or None) of step k."""
        kind, ver, ht = I32(0), I32(0), P()
        self.ctx._check(lib().hs_tape_step(self.h, k, ctypes.byref(kind), ctypes.byref(ver), ctypes.byref(ht)))
        tape = Tape(self.ctx, handle=ht, owner=self) if kind.value == 1 else None
        return kind.value, ver.value, tape

    def basis(self, version, m_max):
        """Copies of basis `version`: (Phi, flat m x N), psi, m."""
        m = I32(0)
        self.ctx._check(lib().hs_tape_basis(self.ctx.h, self.h, version, None, None, ctypes.byref(m)))
        Phi = self.ctx.empty(max(m.value, 1) * self.ctx.n)
        psi = self.ctx.empty()
        self.ctx._check(lib().hs_tape_basis(self.ctx.h, self.h, version, _ptr(Phi), _ptr(psi), None))
        return Phi[: m.value * self.ctx.n], psi, m.value

    def checkpoint(self, k):
        q = self.ctx.empty()
        self.ctx._check(lib().hs_tape_checkpoint(self.ctx.h, self.h, k, _ptr(q)))
        return q

    def close(self):
        if getattr(self, "h", None):
            lib().hs_tape_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

