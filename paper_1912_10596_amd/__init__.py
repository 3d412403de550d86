"""Python binding of libnubulb (the MI355X bulb-model radial stepper).

Argument marshalling only: every step of the path runs in the HIP kernels behind the
C-ABI of include/nubulb.h.  PyTorch provides device memory (the workspace and outputs)
and the current HIP stream.  There is no fallback: if the shared library is missing or
no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnubulb.so")

NB_OK, NB_EINVAL, NB_EUNBOUND, NB_EWORKSPACE, NB_EHIP, NB_ENUMERIC, NB_ETIMEOUT, NB_ESTEP, NB_EIO = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
NB_FP64, NB_FP32_STATE = 0, 1

EXPORTS = [
    "nb_model_create", "nb_batch_create", "nb_model_destroy", "nb_n_beams", "nb_n_models",
    "nb_state_comps", "nb_pee_offsets", "nb_workspace_bytes", "nb_bind", "nb_reset",
    "nb_step", "nb_run", "nb_step_index", "nb_read_pee", "nb_get_state", "nb_set_state",
    "nb_adjoint", "nb_host_tables", "nb_last_error", "nb_graph_capture", "nb_graph_launch",
    "nb_autotune", "nb_set_tuning", "nb_get_tuning", "nb_cancel", "nb_mixed_fp32_step",
    "nb_run_adaptive", "nb_step_static",
]


class Params(C.Structure):
    _fields_ = [
        ("n_flavor", C.c_int32), ("n_energy", C.c_int32), ("n_u", C.c_int32),
        ("ne_power", C.c_int32), ("precision", C.c_int32), ("renorm", C.c_int32),
        ("adjoint_ckpt", C.c_int32), ("max_blocks", C.c_int32), ("n_steps", C.c_int64),
        ("e_min_mev", C.c_double), ("e_max_mev", C.c_double), ("r_nu_km", C.c_double),
        ("r_start_km", C.c_double), ("r_end_km", C.c_double),
        ("lum_erg_s", C.c_double * 3), ("temp_mev", C.c_double * 3),
        ("dm2_ev2", C.c_double * 2), ("theta", C.c_double * 3), ("delta_cp", C.c_double),
        ("n0_cm3", C.c_double), ("adaptive", C.c_int32), ("n_phi", C.c_int32),
        ("track_all", C.c_int32), ("reserved", C.c_int32), ("lum_xbar_erg_s", C.c_double),
        ("temp_xbar_mev", C.c_double),
    ]


class AdaptiveStats(C.Structure):
    _fields_ = [("accepted", C.c_int64), ("rejected", C.c_int64), ("attempts", C.c_int64),
                ("h_last_km", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("blocks", C.c_int32), ("row_cost", C.c_double),
                ("ms", C.c_double), ("from_cache", C.c_int32), ("candidates", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class NubulbError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


_lib = None


def lib():
    """Load libnubulb.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        # the library works on torch's device memory and streams, so it must bind to the HIP
        # runtime torch loads: import torch first (loading the library first would bring in
        # a second runtime, which then finds no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
        L.nb_model_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.nb_batch_create.argtypes = [C.POINTER(Params), C.c_int32, C.POINTER(vp)]
        L.nb_model_destroy.argtypes = [vp]
        L.nb_model_destroy.restype = None
        L.nb_n_beams.argtypes = [vp]
        L.nb_n_beams.restype = i64
        L.nb_n_models.argtypes = [vp]
        L.nb_state_comps.argtypes = [vp]
        L.nb_pee_offsets.argtypes = [vp, C.POINTER(i64)]
        L.nb_workspace_bytes.argtypes = [vp]
        L.nb_workspace_bytes.restype = C.c_size_t
        L.nb_bind.argtypes = [vp, vp, C.c_size_t, vp]
        L.nb_reset.argtypes = [vp]
        L.nb_step.argtypes = [vp, i64]
        L.nb_step_static.argtypes = [vp, i64]
        L.nb_run.argtypes = [vp]
        L.nb_step_index.argtypes = [vp]
        L.nb_step_index.restype = i64
        L.nb_mixed_fp32_step.argtypes = [vp]
        L.nb_mixed_fp32_step.restype = i64
        L.nb_read_pee.argtypes = [vp, vp]
        L.nb_get_state.argtypes = [vp, vp, C.c_int]
        L.nb_set_state.argtypes = [vp, vp, i64, C.c_int]
        L.nb_adjoint.argtypes = [vp, vp, dp, C.c_int32, vp]
        L.nb_host_tables.argtypes = [vp, dp, i64]
        L.nb_last_error.restype = C.c_char_p
        L.nb_graph_capture.argtypes = [vp, i64]
        L.nb_graph_launch.argtypes = [vp]
        L.nb_autotune.argtypes = [vp, C.c_int32, C.c_char_p, C.POINTER(Tuning)]
        L.nb_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.nb_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.nb_cancel.argtypes = [vp, C.c_int32]
        L.nb_run_adaptive.argtypes = [vp, C.c_double, C.c_double, i64, C.POINTER(AdaptiveStats)]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != NB_OK:
        raise NubulbError(rc, what, lib().nb_last_error().decode(errors="replace"))


def make_params(d: dict, precision: int | None = None, adjoint_ckpt: int = 0,
                max_blocks: int = 0, adaptive: bool = False) -> Params:
    p = Params()
    p.max_blocks = int(d.get("max_blocks", max_blocks))
    p.adaptive = int(bool(adaptive))
    p.n_phi = int(d.get("n_phi", 0))
    p.track_all = int(d.get("track_all", 0))
    p.lum_xbar_erg_s = float(d.get("lum_xbar_erg_s", 0.0))
    p.temp_xbar_mev = float(d.get("temp_xbar_mev", 0.0))
    for k in ("n_flavor", "n_energy", "n_u", "ne_power", "renorm", "n_steps"):
        setattr(p, k, int(d[k]))
    p.precision = int(d.get("precision", 0) if precision is None else precision)
    p.adjoint_ckpt = int(adjoint_ckpt)
    for k in ("e_min_mev", "e_max_mev", "r_nu_km", "r_start_km", "r_end_km", "delta_cp",
              "n0_cm3"):
        setattr(p, k, float(d[k]))
    p.lum_erg_s[:] = [float(x) for x in d["lum_erg_s"]]
    p.temp_mev[:] = [float(x) for x in d["temp_mev"]]
    p.dm2_ev2[:] = [float(x) for x in d["dm2_ev2"]]
    p.theta[:] = [float(x) for x in d["theta"]]
    return p


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class HostModel:
    """A model (or, given a list of parameter dicts, a batch of two-flavour models)
    created on the host only: parameter validation and tables, no device work."""

    def __init__(self, d, precision: int | None = None, adjoint_ckpt: int = 0,
                 adaptive: bool = False):
        h = C.c_void_p()
        if isinstance(d, (list, tuple)):
            self.ds = [dict(x) for x in d]
            arr = (Params * len(d))(*[make_params(x, precision, adjoint_ckpt) for x in d])
            self.params = arr
            _check(lib().nb_batch_create(arr, len(d), C.byref(h)), "nb_batch_create")
            d = d[0]
        else:
            self.ds = [dict(d)]
            self.params = make_params(d, precision, adjoint_ckpt, adaptive=adaptive)
            _check(lib().nb_model_create(C.byref(self.params), C.byref(h)), "nb_model_create")
        self.d = dict(d)
        self.h = h
        self.nb = int(lib().nb_n_beams(h))
        self.nsc = int(lib().nb_state_comps(h))
        self.nf = int(d["n_flavor"])
        self.n_models = int(lib().nb_n_models(h))

    def mixed_fp32_step(self) -> int:
        """First step advanced with FP32 stage arithmetic (mixed precision), or -1."""
        return int(lib().nb_mixed_fp32_step(self.h))

    def offsets(self):
        off = (C.c_int64 * (self.n_models + 1))()
        _check(lib().nb_pee_offsets(self.h, off), "nb_pee_offsets")
        return [int(x) for x in off]

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.nb_model_destroy(self.h)
            self.h = None

    def workspace_bytes(self) -> int:
        return int(lib().nb_workspace_bytes(self.h))

    def tables(self) -> dict:
        import numpy as np
        ne = int(self.d["n_energy"])
        nv = 2 if self.nf == 2 else 6
        ns = 2 * self.nf if self.d.get("track_all", 0) else 2
        n = ne + ns * ne + nv * ne + 7
        out = np.empty(n, np.float64)
        _check(lib().nb_host_tables(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n),
               "nb_host_tables")
        o = 0
        E = out[o:o + ne]; o += ne
        w = out[o:o + ns * ne].reshape(ns, ne); o += ns * ne
        bv = out[o:o + nv * ne].reshape(ne, nv); o += nv * ne
        lam0, kappa0, h, p2e1, p2e0, e1, e0 = out[o:o + 7]
        return dict(E=E, w=w, bv=bv, lam0=lam0, kappa0=kappa0, h=h, p2e1=p2e1, p2e0=p2e0,
                    e1=int(e1), e0=int(e0))


class Model(HostModel):
    """A bulb model bound to device memory on the current torch device and stream."""

    def __init__(self, d: dict, precision: int | None = None, adjoint_ckpt: int = 0,
                 device="cuda", stream=None, adaptive: bool = False):
        super().__init__(d, precision, adjoint_ckpt, adaptive)
        torch = _torch()
        nbytes = self.workspace_bytes()
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = stream
        _check(lib().nb_bind(self.h, C.c_void_p(base + off), nbytes, _stream_ptr(stream)),
               "nb_bind")

    def reset(self):
        _check(lib().nb_reset(self.h), "nb_reset")

    def step(self, n: int):
        _check(lib().nb_step(self.h, int(n)), "nb_step")

    def run(self):
        _check(lib().nb_run(self.h), "nb_run")

    def step_static(self, n: int):
        """nb_step with the launch scratch in the library's static device array."""
        _check(lib().nb_step_static(self.h, int(n)), "nb_step_static")

    def step_index(self) -> int:
        return int(lib().nb_step_index(self.h))

    def run_adaptive(self, tol: float, h_max: float = 0.0, max_attempts: int = 10**7) -> dict:
        """Adaptive step-size control from step 0 to r_end (nb_run_adaptive); the model must
        have been created with adaptive=True."""
        st = AdaptiveStats()
        _check(lib().nb_run_adaptive(self.h, float(tol), float(h_max), int(max_attempts),
                                     C.byref(st)), "nb_run_adaptive")
        return dict(accepted=int(st.accepted), rejected=int(st.rejected),
                    attempts=int(st.attempts), h_last=float(st.h_last_km))

    def pee(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.nb, dtype=torch.float64, device=self.ws.device)
        _check(lib().nb_read_pee(self.h, C.c_void_p(out.data_ptr())), "nb_read_pee")
        return out

    def get_state(self):
        torch = _torch()
        out = torch.empty(self.nsc, self.nb, dtype=torch.float64, device=self.ws.device)
        _check(lib().nb_get_state(self.h, C.c_void_p(out.data_ptr()), 1), "nb_get_state")
        return out

    def graph_capture(self, n_steps: int):
        _check(lib().nb_graph_capture(self.h, int(n_steps)), "nb_graph_capture")

    def graph_launch(self):
        _check(lib().nb_graph_launch(self.h), "nb_graph_launch")

    def autotune(self, trial_steps: int = 10, cache: str | None = None) -> dict:
        """nb_autotune; returns the chosen shape (block_threads, blocks, row_cost, ms,
        from_cache, candidates)."""
        t = Tuning()
        path = None if cache is None else os.fsencode(cache)
        _check(lib().nb_autotune(self.h, int(trial_steps), path, C.byref(t)), "nb_autotune")
        return t.as_dict()

    def set_tuning(self, block_threads: int, blocks: int = 0, row_cost: float = 1.0):
        t = Tuning(block_threads=int(block_threads), blocks=int(blocks), row_cost=float(row_cost))
        _check(lib().nb_set_tuning(self.h, C.byref(t)), "nb_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().nb_get_tuning(self.h, C.byref(t)), "nb_get_tuning")
        return t.as_dict()

    def cancel(self, on: bool = True):
        """nb_cancel: make the model's launches give up (on) or run again (off)."""
        _check(lib().nb_cancel(self.h, int(bool(on))), "nb_cancel")

    def get_state_host(self):
        """State planes [nsc][nb] as a float64 numpy array (host path of nb_get_state)."""
        import numpy as np
        out = np.empty((self.nsc, self.nb), np.float64)
        _check(lib().nb_get_state(self.h, out.ctypes.data_as(C.c_void_p), 0), "nb_get_state")
        return out

    def set_state_host(self, x, step: int):
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size == self.nsc * self.nb
        _check(lib().nb_set_state(self.h, x.ctypes.data_as(C.c_void_p), int(step), 0),
               "nb_set_state")

    def set_state(self, x, step: int):
        torch = _torch()
        x = x.to(device=self.ws.device, dtype=torch.float64).contiguous()
        assert x.numel() == self.nsc * self.nb
        _check(lib().nb_set_state(self.h, C.c_void_p(x.data_ptr()), int(step), 1),
               "nb_set_state")

    def adjoint(self, dl_dpee=None, ckpt: int = 0, want_state_bar: bool = False):
        """Reverse-mode gradients of L = sum_b dl_dpee[b] Pee_b at r_end (default
        cotangent dE/N_u) with respect to (L_e, L_ebar, L_x, theta_v, n0), from the current
        state; the model ends at r_end.  Returns a float64 numpy array of 5, or
        (grad, state_bar) with state_bar = dL/d(state at the start) as [3][nb] planes."""
        import numpy as np
        torch = _torch()
        c = None
        if dl_dpee is not None:
            c = dl_dpee.to(device=self.ws.device, dtype=torch.float64).contiguous()
            assert c.numel() == self.nb
        sb = None
        if want_state_bar:
            sb = torch.empty(3, self.nb, dtype=torch.float64, device=self.ws.device)
        g = np.empty(5, np.float64)
        _check(lib().nb_adjoint(self.h, None if c is None else _ptr(c),
                                g.ctypes.data_as(C.POINTER(C.c_double)), int(ckpt),
                                None if sb is None else _ptr(sb)), "nb_adjoint")
        return (g, sb) if want_state_bar else g


PARAM_NAMES = ("L_e", "L_ebar", "L_x", "theta_v", "n0")


def _with_params(d: dict, x) -> dict:
    q = {k: (list(v) if isinstance(v, list) else v) for k, v in d.items()}
    q["lum_erg_s"] = [float(x[0]), float(x[1]), float(x[2])]
    q["theta"] = [float(x[3])] + list(d["theta"][1:])
    q["n0_cm3"] = float(x[4])
    return q


def _bulb_fn():
    torch = _torch()

    class BulbPee(torch.autograd.Function):
        """Final P_ee of every beam of a two-flavour bulb model as a differentiable
        function of x = (L_e, L_ebar, L_x, theta_v, n0); backward runs the library's
        reverse-mode adjoint with the given checkpoint period."""

        @staticmethod
        def forward(ctx, x, d, ckpt):
            m = Model(_with_params(d, x.detach().cpu().tolist()), adjoint_ckpt=int(ckpt))
            m.run()
            ctx.model = m
            return m.pee()

        @staticmethod
        def backward(ctx, g):
            m = ctx.model
            m.reset()
            grad = m.adjoint(g.detach())
            return torch.as_tensor(grad, dtype=torch.float64), None, None

    return BulbPee


def bulb_pee(x, d: dict, ckpt: int = 64):
    """Differentiable final P_ee (device tensor [nb]) of the two-flavour model d with its
    luminosities, theta_v and n0 replaced by the float64 tensor x (5 entries, CPU)."""
    return _bulb_fn().apply(x, d, ckpt)
