"""ctypes wrapper of the CPU oracle (oracle/nbo.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU-baseline
leg of bench.py.  The product path (paper_1912_10596_amd) never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Params(C.Structure):
    _fields_ = [
        ("n_flavor", C.c_int32), ("n_energy", C.c_int32), ("n_u", C.c_int32),
        ("ne_power", C.c_int32), ("renorm", C.c_int32), ("integrator", C.c_int32),
        ("species4", C.c_int32), ("n_phi", C.c_int32), ("n_steps", C.c_int64),
        ("e_min_mev", C.c_double), ("e_max_mev", C.c_double), ("r_nu_km", C.c_double),
        ("r_start_km", C.c_double), ("r_end_km", C.c_double),
        ("lum_erg_s", C.c_double * 3), ("temp_mev", C.c_double * 3),
        ("dm2_ev2", C.c_double * 2), ("theta", C.c_double * 3), ("delta_cp", C.c_double),
        ("n0_cm3", C.c_double), ("lum_xbar_erg_s", C.c_double), ("temp_xbar_mev", C.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        vp = C.c_void_p
        L.nbo_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.nbo_destroy.argtypes = [vp]
        L.nbo_destroy.restype = None
        L.nbo_set_threads.argtypes = [C.c_int]
        L.nbo_get_threads.argtypes = []
        L.nbo_n_beams.argtypes = [vp]
        L.nbo_n_beams.restype = C.c_int64
        L.nbo_n_species.argtypes = [vp]
        L.nbo_state_comps.argtypes = [vp]
        L.nbo_reset.argtypes = [vp]
        L.nbo_step.argtypes = [vp, C.c_int64]
        L.nbo_step_index.argtypes = [vp]
        L.nbo_step_index.restype = C.c_int64
        L.nbo_read_pee.argtypes = [vp, dp]
        L.nbo_get_state.argtypes = [vp, dp]
        L.nbo_set_state.argtypes = [vp, dp, C.c_int64]
        L.nbo_tables.argtypes = [vp, dp, C.c_int64]
        L.nbo_moments.argtypes = [vp, C.c_double, dp, dp]
        L.nbo_hamiltonian.argtypes = [vp, C.c_double, dp, dp, dp]
        L.nbo_cos_theta.argtypes = [vp, C.c_double, dp]
        L.nbo_sincos.argtypes = [dp, C.c_int64, dp, dp]
        L.nbo_sincos.restype = None
        L.nbo_exp3_apply.argtypes = [dp, dp, dp]
        L.nbo_exp3_apply.restype = None
        L.nbo_rotate.argtypes = [dp, dp, dp]
        L.nbo_rotate.restype = None
        L.nbo_fixed_sum.argtypes = [dp, C.c_int64, C.c_int]
        L.nbo_fixed_sum.restype = C.c_double
        L.nbo_fix_round.argtypes = [dp, dp, C.c_int64, C.POINTER(C.c_int64)]
        L.nbo_fix_round.restype = None
        L.nbo_single_angle_run.argtypes = [C.POINTER(Params), dp]
        L.nbo_adjoint.argtypes = [vp, C.c_int32, vp, dp, dp, vp]
        L.nbo_run_adaptive.argtypes = [vp, C.c_double, C.c_double, C.c_int64,
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64), dp]
        L.nbo_step_error.argtypes = [vp, C.c_double, dp]
        L.nbo_moments4.argtypes = [vp, C.c_double, dp]
        L.nbo_hamiltonian4.argtypes = [vp, C.c_double, dp, dp]
        L.nbo_phi_table.argtypes = [vp, dp]
        L.nbp_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.nbp_destroy.argtypes = [vp]
        L.nbp_destroy.restype = None
        L.nbp_n_beams.argtypes = [vp]
        L.nbp_n_beams.restype = C.c_int64
        L.nbp_step_index.argtypes = [vp]
        L.nbp_step_index.restype = C.c_int64
        L.nbp_reset.argtypes = [vp]
        L.nbp_step.argtypes = [vp, C.c_int64]
        L.nbp_read_pee.argtypes = [vp, dp]
        L.nbp_get_rho.argtypes = [vp, dp]
        L.nbp_set_rho.argtypes = [vp, dp, C.c_int64]
        L.nbp_moments.argtypes = [vp, C.c_double, dp]
        L.nbp_hamiltonian.argtypes = [vp, C.c_double, dp]
        L.nbp_expm.argtypes = [C.c_int, dp, dp]
        L.nbp_expm.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(d: dict, integrator: int = 0, species4: int = 0) -> Params:
    p = Params()
    for k in ("n_flavor", "n_energy", "n_u", "ne_power", "renorm", "n_steps"):
        setattr(p, k, int(d[k]))
    for k in ("e_min_mev", "e_max_mev", "r_nu_km", "r_start_km", "r_end_km", "delta_cp",
              "n0_cm3"):
        setattr(p, k, float(d[k]))
    p.lum_erg_s[:] = [float(x) for x in d["lum_erg_s"]]
    p.temp_mev[:] = [float(x) for x in d["temp_mev"]]
    p.dm2_ev2[:] = [float(x) for x in d["dm2_ev2"]]
    p.theta[:] = [float(x) for x in d["theta"]]
    p.integrator = integrator
    p.species4 = species4
    p.n_phi = int(d.get("n_phi", 0))
    p.lum_xbar_erg_s = float(d.get("lum_xbar_erg_s", 0.0))
    p.temp_xbar_mev = float(d.get("temp_xbar_mev", 0.0))
    return p


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


class Model:
    """One bulb model held by the oracle."""

    def __init__(self, d: dict, integrator: int = 0, species4: int = 0):
        self.d = dict(d)
        self.params = make_params(d, integrator, species4)
        h = C.c_void_p()
        _check(lib().nbo_create(C.byref(self.params), C.byref(h)), "nbo_create")
        self.h = h
        self.nb = lib().nbo_n_beams(h)
        self.ns = lib().nbo_n_species(h)
        self.nsc = lib().nbo_state_comps(h)
        self.nf = int(d["n_flavor"])
        self.ncomp = 3 if self.nf == 2 else 8

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.nbo_destroy(self.h)
            self.h = None

    def reset(self):
        _check(lib().nbo_reset(self.h), "nbo_reset")

    def step(self, n: int):
        _check(lib().nbo_step(self.h, int(n)), "nbo_step")

    def run(self):
        self.step(int(self.d["n_steps"]) - self.step_index())

    def step_index(self) -> int:
        return int(lib().nbo_step_index(self.h))

    def step_error(self, h: float) -> float:
        """Error estimate of one step of length h from the current state (no state change)."""
        e = C.c_double()
        _check(lib().nbo_step_error(self.h, float(h), C.byref(e)), "nbo_step_error")
        return float(e.value)

    def run_adaptive(self, tol: float, h_max: float = 0.0, max_attempts: int = 10**7) -> dict:
        """Adaptive step-size control from step 0 to r_end (nbo_run_adaptive)."""
        acc, rej, hl = C.c_int64(), C.c_int64(), C.c_double()
        _check(lib().nbo_run_adaptive(self.h, float(tol), float(h_max), int(max_attempts),
                                      C.byref(acc), C.byref(rej), C.byref(hl)),
               "nbo_run_adaptive")
        return dict(accepted=int(acc.value), rejected=int(rej.value), h_last=float(hl.value))

    def pee(self) -> np.ndarray:
        """P_ee as [species][n_u][n_energy] (bulb) or [species][n_u][n_phi][n_energy]."""
        out = np.empty(self.nb, np.float64)
        _check(lib().nbo_read_pee(self.h, _dp(out)), "nbo_read_pee")
        nphi = int(self.d.get("n_phi", 0))
        shape = (self.ns, int(self.d["n_u"])) + ((nphi,) if nphi else ()) + (int(self.d["n_energy"]),)
        return out.reshape(shape)

    def get_state(self) -> np.ndarray:
        out = np.empty(self.nb * self.nsc, np.float64)
        _check(lib().nbo_get_state(self.h, _dp(out)), "nbo_get_state")
        return out.reshape(self.nsc, self.nb)

    def set_state(self, x: np.ndarray, step: int):
        x = np.ascontiguousarray(x, np.float64).reshape(-1)
        assert x.size == self.nb * self.nsc
        _check(lib().nbo_set_state(self.h, _dp(x), int(step)), "nbo_set_state")

    def tables(self) -> dict:
        ne = int(self.d["n_energy"])
        nv = 2 if self.nf == 2 else 6
        n = ne + ne * self.ns + ne * nv + 7
        out = np.empty(n, np.float64)
        _check(lib().nbo_tables(self.h, _dp(out), n), "nbo_tables")
        o = 0
        E = out[o:o + ne]; o += ne
        w = out[o:o + ne * self.ns].reshape(self.ns, ne); o += ne * self.ns
        bv = out[o:o + ne * nv].reshape(ne, nv); o += ne * nv
        lam0, kappa0, h, p2e1, p2e0, e1, e0 = out[o:o + 7]
        return dict(E=E, w=w, bv=bv, lam0=lam0, kappa0=kappa0, h=h, p2e1=p2e1, p2e0=p2e0,
                    e1=int(e1), e0=int(e0))

    def moments(self, r: float):
        j0 = np.empty(8, np.float64); j1 = np.empty(8, np.float64)
        _check(lib().nbo_moments(self.h, float(r), _dp(j0), _dp(j1)), "nbo_moments")
        return j0[:self.ncomp].copy(), j1[:self.ncomp].copy()

    def hamiltonian(self, r: float, j0, j1) -> np.ndarray:
        a0 = np.zeros(8); a1 = np.zeros(8)
        a0[:self.ncomp] = j0; a1[:self.ncomp] = j1
        per = 3 if self.nf == 2 else 9
        out = np.empty(self.nb * per, np.float64)
        _check(lib().nbo_hamiltonian(self.h, float(r), _dp(a0), _dp(a1), _dp(out)),
               "nbo_hamiltonian")
        return out.reshape(self.nb, per)

    def moments4(self, r: float) -> np.ndarray:
        """[4][ncomp]: J0, J1 and (extended model) J_sc, J_ss."""
        out = np.zeros(4 * self.ncomp, np.float64)
        _check(lib().nbo_moments4(self.h, float(r), _dp(out)), "nbo_moments4")
        return out.reshape(4, self.ncomp)

    def hamiltonian4(self, r: float, jm) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(jm, np.float64).reshape(4 * self.ncomp))
        per = 3 if self.nf == 2 else 9
        out = np.empty(self.nb * per, np.float64)
        _check(lib().nbo_hamiltonian4(self.h, float(r), _dp(a), _dp(out)), "nbo_hamiltonian4")
        return out.reshape(self.nb, per)

    def phi_table(self) -> np.ndarray:
        n = int(self.d["n_phi"])
        out = np.empty(2 * n, np.float64)
        _check(lib().nbo_phi_table(self.h, _dp(out)), "nbo_phi_table")
        return out.reshape(2, n)

    def cos_theta(self, r: float) -> np.ndarray:
        out = np.empty(int(self.d["n_u"]), np.float64)
        _check(lib().nbo_cos_theta(self.h, float(r), _dp(out)), "nbo_cos_theta")
        return out

    def adjoint(self, ckpt: int = 64, dl_dpee=None, want_state_bar: bool = False):
        """Reverse-mode gradients of L = sum_b dl_dpee[b] Pee_b at r_end (default weights
        dE/N_u) with respect to (L_e, L_ebar, L_x, theta_v, n0).  Returns (L, grad) or
        (L, grad, state_bar) with state_bar = dL/d(initial state) as planes [3][nb]."""
        g = np.empty(5, np.float64)
        loss = C.c_double()
        c = None
        if dl_dpee is not None:
            c = np.ascontiguousarray(dl_dpee, dtype=np.float64).reshape(-1)
            assert c.size == self.nb
        sb = np.empty((self.nb, 3), np.float64) if want_state_bar else None
        _check(lib().nbo_adjoint(self.h, int(ckpt), None if c is None else _dp(c), _dp(g),
                                 C.byref(loss), None if sb is None else _dp(sb)), "nbo_adjoint")
        if want_state_bar:
            return float(loss.value), g, np.ascontiguousarray(sb.T)
        return float(loss.value), g


def rho_from_planes(x: np.ndarray, nf: int) -> np.ndarray:
    """Density matrices [nb][n][n] of state planes (2f: Bloch vectors [3][nb], rho =
    (1 + P.sigma)/2; 3f: wavefunctions [6][nb] as Re/Im pairs, rho = psi psi^+)."""
    x = np.asarray(x, np.float64)
    if nf == 2:
        P = x.reshape(3, -1)
        rho = np.empty((P.shape[1], 2, 2), complex)
        rho[:, 0, 0] = 0.5 * (1 + P[2]); rho[:, 1, 1] = 0.5 * (1 - P[2])
        rho[:, 0, 1] = 0.5 * (P[0] - 1j * P[1]); rho[:, 1, 0] = 0.5 * (P[0] + 1j * P[1])
        return rho
    pv = (x.reshape(6, -1)[0::2] + 1j * x.reshape(6, -1)[1::2]).T
    return np.einsum("bi,bj->bij", pv, pv.conj())


class PlainModel:
    """The oracle's plain mode (oracle/plain.c): density matrices, dense per-beam
    generators, Jacobi exponentials, plain FP64 sums.  Same parameters and beam order as
    Model; fixed-step RKMK4 only."""

    def __init__(self, d: dict, species4: int = 0):
        self.d = dict(d)
        self.params = make_params(d, 0, species4)
        h = C.c_void_p()
        _check(lib().nbp_create(C.byref(self.params), C.byref(h)), "nbp_create")
        self.h = h
        self.nb = int(lib().nbp_n_beams(h))
        self.nf = int(d["n_flavor"])
        self.ns = 2 * self.nf if species4 else 2

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.nbp_destroy(self.h)
            self.h = None

    def reset(self):
        _check(lib().nbp_reset(self.h), "nbp_reset")

    def step(self, n: int):
        _check(lib().nbp_step(self.h, int(n)), "nbp_step")

    def run(self):
        self.step(int(self.d["n_steps"]) - self.step_index())

    def step_index(self) -> int:
        return int(lib().nbp_step_index(self.h))

    def pee(self) -> np.ndarray:
        out = np.empty(self.nb, np.float64)
        _check(lib().nbp_read_pee(self.h, _dp(out)), "nbp_read_pee")
        nphi = int(self.d.get("n_phi", 0))
        shape = (self.ns, int(self.d["n_u"])) + ((nphi,) if nphi else ()) + (int(self.d["n_energy"]),)
        return out.reshape(shape)

    def get_rho(self) -> np.ndarray:
        n = self.nf
        out = np.empty(self.nb * n * n * 2, np.float64)
        _check(lib().nbp_get_rho(self.h, _dp(out)), "nbp_get_rho")
        return out.view(np.complex128).reshape(self.nb, n, n)

    def set_rho(self, rho: np.ndarray, step: int):
        a = np.ascontiguousarray(np.asarray(rho, np.complex128).reshape(self.nb, self.nf, self.nf))
        _check(lib().nbp_set_rho(self.h, _dp(a.view(np.float64).reshape(-1)), int(step)),
               "nbp_set_rho")

    def set_state(self, x: np.ndarray, step: int):
        """From state planes as Model.set_state takes them."""
        self.set_rho(rho_from_planes(x, self.nf), step)

    def moments(self, r: float) -> np.ndarray:
        n = self.nf
        out = np.empty(4 * n * n * 2, np.float64)
        _check(lib().nbp_moments(self.h, float(r), _dp(out)), "nbp_moments")
        return out.view(np.complex128).reshape(4, n, n)

    def hamiltonian(self, r: float) -> np.ndarray:
        n = self.nf
        out = np.empty(self.nb * n * n * 2, np.float64)
        _check(lib().nbp_hamiltonian(self.h, float(r), _dp(out)), "nbp_hamiltonian")
        return out.view(np.complex128).reshape(self.nb, n, n)


def plain_expm(K: np.ndarray) -> np.ndarray:
    """exp(-i K) of a Hermitian 2x2 or 3x3 K by the plain mode's Jacobi exponential."""
    K = np.ascontiguousarray(np.asarray(K, np.complex128))
    n = K.shape[0]
    out = np.empty((n, n), np.complex128)
    lib().nbp_expm(n, _dp(K.view(np.float64).reshape(-1)), _dp(out.view(np.float64).reshape(-1)))
    return out


def set_threads(n: int):
    lib().nbo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().nbo_get_threads())


def sincos(x: np.ndarray):
    x = np.ascontiguousarray(x, np.float64)
    s = np.empty_like(x); c = np.empty_like(x)
    lib().nbo_sincos(_dp(x), x.size, _dp(s), _dp(c))
    return s, c


def exp3_apply(k9, psi6) -> np.ndarray:
    k9 = np.ascontiguousarray(k9, np.float64); psi6 = np.ascontiguousarray(psi6, np.float64)
    out = np.empty(6, np.float64)
    lib().nbo_exp3_apply(_dp(k9), _dp(psi6), _dp(out))
    return out


def rotate(x3, p3) -> np.ndarray:
    x3 = np.ascontiguousarray(x3, np.float64); p3 = np.ascontiguousarray(p3, np.float64)
    out = np.empty(3, np.float64)
    lib().nbo_rotate(_dp(x3), _dp(p3), _dp(out))
    return out


def fixed_sum(v, e: int) -> float:
    v = np.ascontiguousarray(v, np.float64)
    return float(lib().nbo_fixed_sum(_dp(v), v.size, int(e)))


def fix_round(v, ws) -> np.ndarray:
    """The fixed-point integers of beam contributions v * ws (round to nearest, ties even)."""
    v = np.ascontiguousarray(v, np.float64); ws = np.ascontiguousarray(ws, np.float64)
    assert v.shape == ws.shape
    out = np.empty(v.size, np.int64)
    lib().nbo_fix_round(_dp(v), _dp(ws), v.size, out.ctypes.data_as(C.POINTER(C.c_int64)))
    return out


def single_angle_run(d: dict) -> np.ndarray:
    p = make_params(d)
    out = np.empty(2 * int(d["n_energy"]), np.float64)
    _check(lib().nbo_single_angle_run(C.byref(p), _dp(out)), "nbo_single_angle_run")
    return out.reshape(2, int(d["n_energy"]))
