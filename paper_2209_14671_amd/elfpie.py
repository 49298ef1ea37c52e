"""Python binding of the gfx950 Elfpie library on torch device memory and streams.

Every computation runs in the HIP library (``lib/libelfpie.so``); this module only
allocates torch tensors, checks their shapes and dtypes, and passes pointers and
the current stream through the C ABI of ``include/elfpie.h``.  There is no CPU or
torch fallback: if the library is missing, importing ``Plan`` works but creating
one raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import (F32, F32_MFMA_BF16X3, F64, FID_AMPLITUDE, FID_GAMMA, FID_INTENSITY, FID_LOG, LEARN_PUPIL, NORM_ANISO, NORM_ISO,  # noqa: F401
                   OPT_ADABELIEF, OPT_ELFPIE, OPT_NADAM, OPT_SGD, PUPIL_FILTER, PUPIL_SUPPORT, ElfpieError)


@dataclasses.dataclass
class Problem:
    """Problem statement (mirrors ``elfpie_problem``)."""
    n_lo: int
    upsample: int
    led_k: np.ndarray               # (K, 2) (kx, ky) in 1/um
    wavelength_um: float
    na: float
    dx_lo_um: float
    alpha: float = 1e-3
    beta: float = 1e-3
    lr: float = 1e-2
    gamma1: float = 0.9
    gamma2: float = 0.999
    eta_opt: float = 1e-8
    eta_h: float = 1e-6
    l1_eps: float = 0.0
    fidelity: int = FID_INTENSITY
    norm: int = NORM_ANISO
    precision: int = F32
    flags: int = PUPIL_SUPPORT
    fid_gamma: float = 0.5          # exponent of FID_GAMMA
    optimizer: int = OPT_ELFPIE     # update rule (Eq. 19 or a Sec. 6.2 alternative)
    mux: int = 1                    # LEDs lit together per image (Eq. 1's M)

    def to_c(self):
        k = np.ascontiguousarray(np.asarray(self.led_k, dtype=np.float64).reshape(-1, 2))
        p = _lib.ProblemC()
        p.n_lo, p.upsample, p.K = int(self.n_lo), int(self.upsample), int(k.shape[0])
        p.wavelength_um, p.na, p.dx_lo_um = float(self.wavelength_um), float(self.na), float(self.dx_lo_um)
        p.led_k = k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.alpha, p.beta, p.lr = float(self.alpha), float(self.beta), float(self.lr)
        p.gamma1, p.gamma2, p.eta_opt = float(self.gamma1), float(self.gamma2), float(self.eta_opt)
        p.eta_h, p.l1_eps = float(self.eta_h), float(self.l1_eps)
        p.fidelity, p.norm, p.precision, p.flags = int(self.fidelity), int(self.norm), int(self.precision), int(self.flags)
        p.fid_gamma = float(self.fid_gamma)
        p.optimizer = int(self.optimizer)
        p.mux = int(self.mux)
        return p, k  # keep k alive while p is used


def problem_from_optics(optics, led_k, **kw) -> Problem:
    """Problem from a ``synth.Optics`` description and LED wave-vectors."""
    return Problem(n_lo=optics.n_lo, upsample=optics.upsample, led_k=np.asarray(led_k, float),
                   wavelength_um=optics.wavelength_um, na=optics.na, dx_lo_um=optics.dx_lo_um, **kw)


def workspace_bytes(problem: Problem) -> int:
    lib = _lib.load()
    p, _keep = problem.to_c()
    n = ctypes.c_size_t(0)
    _lib.check(lib.elfpie_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return int(n.value)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclasses.dataclass
class State:
    """Optimiser state of Eq. (19) on the device; saving these tensors is a checkpoint."""
    psi: torch.Tensor
    P: torch.Tensor
    mu_psi: torch.Tensor
    v_psi: torch.Tensor
    delta_psi: torch.Tensor
    mu_P: torch.Tensor
    v_P: torch.Tensor
    delta_P: torch.Tensor
    t: torch.Tensor

    def to_c(self):
        return _lib.StateC(*(getattr(self, f).data_ptr() for f in _STATE_FIELDS))

    def clone(self) -> "State":
        return State(*(getattr(self, f.name).clone() for f in dataclasses.fields(self)))

    def state_dict(self):
        return {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}


_STATE_FIELDS = tuple(f.name for f in dataclasses.fields(State))


class Plan:
    """A validated problem with its device workspace (owned here, as a torch tensor)."""

    def __init__(self, problem: Problem, device=None):
        self.lib = _lib.load()
        self.problem = problem
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        p, _keep = problem.to_c()
        n = ctypes.c_size_t(0)
        _lib.check(self.lib.elfpie_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            handle = ctypes.c_void_p(0)
            _lib.check(self.lib.elfpie_plan_create(ctypes.byref(p), ctypes.c_void_p(base + off),
                                                   ctypes.c_size_t(int(n.value)), ctypes.byref(handle)))
        self.handle = handle
        info = (ctypes.c_int32 * 5)()
        _lib.check(self.lib.elfpie_plan_info(self.handle, info), self.handle)
        self.n_hi, self.S, self.K, self.n_lo, self.kc = (int(v) for v in info)
        self.mux = int(problem.mux)
        self.n_img = self.K // self.mux
        f32 = problem.precision != F64  # ELFPIE_F32 and the split-BF16 GEMM form keep FP32 arrays
        self.rdtype = torch.float32 if f32 else torch.float64
        self.cdtype = torch.complex64 if f32 else torch.complex128

    def close(self):
        if getattr(self, "handle", None):
            self.lib.elfpie_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks ------------------------------------------------------------
    def _need(self, t, shape, dtype, name):
        # one combined test on the common path (a run call checks nine state tensors)
        if (isinstance(t, torch.Tensor) and t.dtype == dtype and t.shape == shape and t.device == self.device
                and t.is_contiguous()):
            return t
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, plan is on {self.device}")
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")

    def _check(self, status):
        _lib.check(status, self.handle)

    @property
    def spec_shape(self):
        return (self.n_hi, self.n_hi)

    @property
    def pupil_shape(self):
        return (self.n_lo, self.n_lo)

    @property
    def stack_shape(self):
        """Measured (and predicted) images: K / mux of n_lo x n_lo."""
        return (self.n_img, self.n_lo, self.n_lo)

    @property
    def fields_shape(self):
        """Low-resolution fields: one n_lo x n_lo per LED."""
        return (self.K, self.n_lo, self.n_lo)

    # -- state ----------------------------------------------------------------------
    def new_state(self, psi0: torch.Tensor, P0: torch.Tensor) -> State:
        """Fresh Eq. (19) state (mu = v = 0, delta = lr^2, t = 0) around copies of psi0, P0."""
        A, B = self.spec_shape, self.pupil_shape
        kw = dict(device=self.device)
        d0 = self.problem.lr ** 2
        return State(
            psi=self._need(psi0, A, self.cdtype, "psi0").clone(), P=self._need(P0, B, self.cdtype, "P0").clone(),
            mu_psi=torch.zeros(A, dtype=self.cdtype, **kw), v_psi=torch.zeros(A, dtype=torch.float64, **kw),
            delta_psi=torch.full(A, d0, dtype=self.rdtype, **kw),
            mu_P=torch.zeros(B, dtype=self.cdtype, **kw), v_P=torch.zeros(B, dtype=torch.float64, **kw),
            delta_P=torch.full(B, d0, dtype=self.rdtype, **kw),
            t=torch.zeros(1, dtype=torch.int64, **kw))

    def init_state(self, meas: torch.Tensor) -> State:
        """Initial guess from the on-axis image (library kernel), all moments reset."""
        self._need(meas, self.stack_shape, self.rdtype, "meas")
        A, B = self.spec_shape, self.pupil_shape
        kw = dict(device=self.device)
        st = State(psi=torch.empty(A, dtype=self.cdtype, **kw), P=torch.empty(B, dtype=self.cdtype, **kw),
                   mu_psi=torch.empty(A, dtype=self.cdtype, **kw), v_psi=torch.empty(A, dtype=torch.float64, **kw),
                   delta_psi=torch.empty(A, dtype=self.rdtype, **kw),
                   mu_P=torch.empty(B, dtype=self.cdtype, **kw), v_P=torch.empty(B, dtype=torch.float64, **kw),
                   delta_P=torch.empty(B, dtype=self.rdtype, **kw), t=torch.empty(1, dtype=torch.int64, **kw))
        sc = st.to_c()
        self._check(self.lib.elfpie_init_state(self.handle, _ptr(meas), ctypes.byref(sc), _stream()))
        return st

    def _state_c(self, st: State):
        A, B = self.spec_shape, self.pupil_shape
        self._need(st.psi, A, self.cdtype, "psi")
        self._need(st.P, B, self.cdtype, "P")
        self._need(st.mu_psi, A, self.cdtype, "mu_psi")
        self._need(st.v_psi, A, torch.float64, "v_psi")
        self._need(st.delta_psi, A, self.rdtype, "delta_psi")
        self._need(st.mu_P, B, self.cdtype, "mu_P")
        self._need(st.v_P, B, torch.float64, "v_P")
        self._need(st.delta_P, B, self.rdtype, "delta_P")
        self._need(st.t, (1,), torch.int64, "t")
        return st.to_c()

    # -- entry points ---------------------------------------------------------------
    def forward(self, psi, P, meas=None, fields=False, intens=False, loss=False):
        """Returns dict with optional 'fields', 'intens', 'loss4' (Eq. 1, Eq. 8)."""
        self._need(psi, self.spec_shape, self.cdtype, "psi")
        self._need(P, self.pupil_shape, self.cdtype, "P")
        if meas is not None:
            self._need(meas, self.stack_shape, self.rdtype, "meas")
        out = {}
        kw = dict(device=self.device)
        f = torch.empty(self.fields_shape, dtype=self.cdtype, **kw) if fields else None
        i = torch.empty(self.stack_shape, dtype=self.rdtype, **kw) if intens else None
        l4 = torch.empty(4, dtype=torch.float64, **kw) if loss else None
        if loss and meas is None:
            raise ValueError("loss needs meas")
        self._check(self.lib.elfpie_forward(self.handle, _ptr(psi), _ptr(P), _ptr(meas), _ptr(f), _ptr(i),
                                            _ptr(l4), _stream()))
        if fields:
            out["fields"] = f
        if intens:
            out["intens"] = i
        if loss:
            out["loss4"] = l4
        return out

    def grad(self, psi, P, meas, want_gP=True, fields=None):
        """(loss4, dL/d conj(psi), dL_fid/d conj(P) or None) at (psi, P) (Eq. 8, 15, 18).
        With `fields` (the K x n_lo x n_lo complex fields of forward at the same psi, P)
        the per-LED fields are read instead of recomputed."""
        self._need(psi, self.spec_shape, self.cdtype, "psi")
        self._need(P, self.pupil_shape, self.cdtype, "P")
        self._need(meas, self.stack_shape, self.rdtype, "meas")
        kw = dict(device=self.device)
        g = torch.empty(self.spec_shape, dtype=self.cdtype, **kw)
        gP = torch.empty(self.pupil_shape, dtype=self.cdtype, **kw) if want_gP else None
        l4 = torch.empty(4, dtype=torch.float64, **kw)
        if fields is None:
            self._check(self.lib.elfpie_grad(self.handle, _ptr(psi), _ptr(P), _ptr(meas), _ptr(g), _ptr(gP),
                                             _ptr(l4), _stream()))
        else:
            self._need(fields, self.fields_shape, self.cdtype, "fields")
            self._check(self.lib.elfpie_grad_fields(self.handle, _ptr(psi), _ptr(P), _ptr(meas), _ptr(fields),
                                                    _ptr(g), _ptr(gP), _ptr(l4), _stream()))
        return l4, g, gP

    def step(self, st: State, meas, want_loss=True):
        sc = self._state_c(st)
        self._need(meas, self.stack_shape, self.rdtype, "meas")
        l4 = torch.empty(4, dtype=torch.float64, device=self.device) if want_loss else None
        self._check(self.lib.elfpie_step(self.handle, ctypes.byref(sc), _ptr(meas), _ptr(l4), _stream()))
        return l4

    def run(self, st: State, meas, n_iter: int, history=True, checked=False):
        """n_iter iterations replayed from captured graphs.  `history`: True (a new
        n_iter x 4 FP64 tensor of loss terms), False (none), or a caller-owned contiguous
        FP64 tensor of at least n_iter x 4, which is filled from its first row.  The graphs
        are keyed on the state, stack and history pointers, so passing the same history
        buffer to repeated calls keeps them replay-only."""
        sc = self._state_c(st)
        self._need(meas, self.stack_shape, self.rdtype, "meas")
        if isinstance(history, torch.Tensor):
            h = history
            if (h.device != self.device or h.dtype != torch.float64 or not h.is_contiguous() or h.dim() != 2
                    or h.shape[1] != 4 or h.shape[0] < n_iter):
                raise ValueError(f"history must be a contiguous float64 tensor of at least ({n_iter}, 4) "
                                 f"on {self.device}")
        else:
            h = torch.empty((max(n_iter, 1), 4), dtype=torch.float64, device=self.device) if history else None
        self._check(self.lib.elfpie_run(self.handle, ctypes.byref(sc), _ptr(meas), int(n_iter), _ptr(h),
                                        1 if checked else 0, _stream()))
        return h[:n_iter] if h is not None else None

    def stats(self):
        """{'captures': graphs captured so far, 'replays': run-graph launches so far}."""
        out = (ctypes.c_int64 * 2)()
        self._check(self.lib.elfpie_plan_stats(self.handle, out))
        return {"captures": int(out[0]), "replays": int(out[1])}

    def object_from_spectrum(self, psi):
        self._need(psi, self.spec_shape, self.cdtype, "psi")
        o = torch.empty_like(psi)
        self._check(self.lib.elfpie_object_from_spectrum(self.handle, _ptr(psi), _ptr(o), _stream()))
        return o

    def spectrum_from_object(self, obj):
        self._need(obj, self.spec_shape, self.cdtype, "obj")
        p = torch.empty_like(obj)
        self._check(self.lib.elfpie_spectrum_from_object(self.handle, _ptr(obj), _ptr(p), _stream()))
        return p

    def auto_penalty(self, meas) -> float:
        """alpha = beta of Eq. 16 / 17 from the measured stack (computed on the device)."""
        self._need(meas, self.stack_shape, self.rdtype, "meas")
        out = ctypes.c_double(0.0)
        self._check(self.lib.elfpie_auto_penalty(self.handle, _ptr(meas), ctypes.byref(out), _stream()))
        return float(out.value)

    def set_penalty(self, alpha: float, beta: float):
        """New Eq. 8 weights for later calls."""
        self._check(self.lib.elfpie_plan_set_penalty(self.handle, float(alpha), float(beta)))

    def stage_timing(self, st: State, meas, n_rep: int = 20):
        """Mean ms per launch of each stage in isolation (see elfpie_stage_timing)."""
        sc = self._state_c(st)
        self._need(meas, self.stack_shape, self.rdtype, "meas")
        ms = (ctypes.c_float * 8)()
        self._check(self.lib.elfpie_stage_timing(self.handle, ctypes.byref(sc), _ptr(meas), int(n_rep), ms,
                                                 _stream()))
        names = ["led", "object", "update", "tail"]
        out = {n: float(ms[i]) for i, n in enumerate(names)}
        out["object_in_led_launch"] = bool(ms[4] > 0.5)
        return out


def grad_noalloc(problem: Problem, psi, P, meas, want_gP=True):
    """elfpie_grad_noalloc: the loss terms and gradients of elfpie_grad with no plan and no
    device workspace (the library's static scratch).  Returns (loss4, g_psi, g_P or None);
    the outputs are allocated here, by torch, as for every other call of this binding."""
    lib = _lib.load()
    p, _keep = problem.to_c()
    f32 = problem.precision != F64
    cdt = torch.complex64 if f32 else torch.complex128
    n_hi, n_lo = problem.n_lo * problem.upsample, problem.n_lo
    for t, shape, name in ((psi, (n_hi, n_hi), "psi"), (P, (n_lo, n_lo), "P")):
        if t.dtype != cdt or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {cdt} tensor of shape {shape}")
    g = torch.empty((n_hi, n_hi), dtype=cdt, device=psi.device)
    gP = torch.empty((n_lo, n_lo), dtype=cdt, device=psi.device) if want_gP else None
    l4 = torch.empty(4, dtype=torch.float64, device=psi.device)
    _lib.check(lib.elfpie_grad_noalloc(ctypes.byref(p), _ptr(psi), _ptr(P), _ptr(meas.contiguous()), _ptr(g),
                                       _ptr(gP), _ptr(l4), _stream()))
    return l4, g, gP


class Batch:
    """Independent fields of view (tiles) run together: one replay of the batch graph is
    one iteration of every tile, the tiles spread over parallel graph branches.
    `tiles` is a list of (Plan, State, measured stack); all of them must stay alive and
    in place while the batch exists (the batch keeps references)."""

    def __init__(self, tiles, n_branches: int = 4):
        self.lib = _lib.load()
        self.tiles = list(tiles)
        n = len(self.tiles)
        for plan, st, meas in self.tiles:
            plan._need(meas, plan.stack_shape, plan.rdtype, "meas")
        self._plans = (ctypes.c_void_p * n)(*[plan.handle.value for plan, _, _ in self.tiles])
        self._states = (_lib.StateC * n)(*[plan._state_c(st) for plan, st, _ in self.tiles])
        self._meas = (ctypes.c_void_p * n)(*[m.data_ptr() for _, _, m in self.tiles])
        handle = ctypes.c_void_p(0)
        st = self.lib.elfpie_batch_create(self._plans, self._states, self._meas, n, int(n_branches),
                                          ctypes.byref(handle))
        self._check(st, None)
        self.handle = handle
        self.n_branches = min(int(n_branches), n)

    def _check(self, status, handle=True):
        if status != _lib.OK:
            h = self.handle if handle else None
            msg = self.lib.elfpie_batch_last_error(h)
            raise ElfpieError(status, msg.decode() if msg else "")

    def tune(self, n_rep: int = 5):
        """Time 1, 2, 4 and 8 branches on gradient evaluations; keep the fastest.
        Returns {branches: ms per replay}."""
        ms = (ctypes.c_float * 4)()
        nb = ctypes.c_int32(0)
        self._check(self.lib.elfpie_batch_tune(self.handle, int(n_rep), ms, ctypes.byref(nb), _stream()))
        self.n_branches = int(nb.value)
        return {c: float(ms[i]) for i, c in enumerate((1, 2, 4, 8)) if ms[i] > 0}

    def run(self, n_iter: int, history: bool = True):
        """n_iter iterations of every tile; returns the per-tile loss histories."""
        hist = [torch.empty((max(n_iter, 1), 4), dtype=torch.float64, device=p.device) if history else None
                for p, _, _ in self.tiles]
        arr = (ctypes.c_void_p * len(hist))(*[h.data_ptr() if h is not None else None for h in hist])
        self._check(self.lib.elfpie_batch_run(self.handle, int(n_iter), arr if history else None, _stream()))
        return [h[:n_iter] for h in hist] if history else None

    def close(self):
        if getattr(self, "handle", None):
            self.lib.elfpie_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ElfpieLoss(torch.autograd.Function):
    """L(psi, P) of Eq. (8) as an autograd function whose backward is the library's
    closed-form gradient (Eq. 15, 18).  With store_fields=False the backward
    recomputes the per-LED fields; with True the forward keeps them (K n_lo^2
    complex) and the backward reads them.  torch's gradient of a real loss with
    respect to a complex tensor z is 2 dL/d(conj z)."""

    @staticmethod
    def forward(ctx, psi, P, plan: Plan, meas, store_fields=False):
        psi_c, P_c = psi.detach().contiguous(), P.detach().contiguous()
        out = plan.forward(psi_c, P_c, meas, fields=store_fields, loss=True)
        ctx.plan = plan
        saved = [psi_c, P_c, meas] + ([out["fields"]] if store_fields else [])
        ctx.save_for_backward(*saved)
        return out["loss4"][3].clone()

    @staticmethod
    def backward(ctx, g_out):
        psi, P, meas, *kept = ctx.saved_tensors
        _, g, gP = ctx.plan.grad(psi, P, meas, want_gP=ctx.needs_input_grad[1], fields=kept[0] if kept else None)
        s = (2.0 * g_out).to(ctx.plan.rdtype)
        gpsi = g * s if ctx.needs_input_grad[0] else None
        gp = gP * s if (gP is not None and ctx.needs_input_grad[1]) else None
        return gpsi, gp, None, None, None


class SpectrumFromObject(torch.autograd.Function):
    """Psi = fftshift(fft2(O)) / n_hi on the library's transform.  The map is
    unitary, so its backward is the inverse transform."""

    @staticmethod
    def forward(ctx, obj, plan: Plan):
        ctx.plan = plan
        return plan.spectrum_from_object(obj.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.object_from_spectrum(g.contiguous()), None


def elfpie_loss(psi, P, plan: Plan, meas, store_fields=False):
    """L(psi, P), differentiable in psi and P."""
    return ElfpieLoss.apply(psi, P, plan, meas, store_fields)


def elfpie_loss_object(obj, P, plan: Plan, meas, store_fields=False):
    """L as a function of the object O (Psi = fftshift(fft2 O) / n_hi) and P."""
    return ElfpieLoss.apply(SpectrumFromObject.apply(obj, plan), P, plan, meas, store_fields)
