"""Two-flavour bulb model in Bloch-vector form, in numpy, for forward-mode derivatives.

TEST INFRASTRUCTURE ONLY: used by tests/ to check reverse-mode adjoints against
directional derivatives.  The product path never imports it.

The same method as the oracle's plain mode (oracle/plain.c), restated for two flavours
with every quantity real: a density matrix rho = (I + P.sigma)/2 is its Bloch vector P;
a Hamiltonian H = h0 I + (w.sigma)/2 acts through w alone (its trace only adds a global
phase); the generator F = -i (h/c) H of a stage (Eq. U) is the rotation vector f = (h/c) w;
the commutator [F_a, F_b] is the vector f_a x f_b; exp(F) rho exp(-F) is the rotation of
P by the angle |f| about f (Rodrigues).  The pieces, with the paper's equations:

  beams b = (s, j, k) with energy innermost; species s = 0 (nu, born nu_e), s = 1 (anti-nu,
  born anti-nu_e); u_j = (j + 1/2)/N_u, E_k midpoints of N_E equal bins      (Sec. 3.2)
  rho~ = rho (nu), -conj(rhobar) (anti-nu)                                   (Eq. F)
     vector part: P/2, and (-Pbar_x, Pbar_y, -Pbar_z)/2
  J0 = sum_b g_b v_b / c_b(r), J1 = sum_b g_b v_b (vector parts), with
     c_b(r) = sqrt(1 - u_j R^2/r^2) and g_b = kappa0 du dE (N_e f_e - N_x f_x) for nu,
     (N_ebar f_ebar - N_x f_x) for anti-nu                         (Eqs. Hnu, F, int-v)
  w_vac = 2 (dm^2/4E) (sin 2t, 0, -cos 2t);  matter: lam(r) z, lam = sqrt2 G_F n0 (R/r)^p
  nu:      w = w_vac + lam z + 2 mu (J0 - c J1)
  anti-nu: w = w_vac - lam z - 2 mu conj_vec(J0 - c J1), conj_vec(x, y, z) = (x, -y, z)
     with mu(r) = R^2 / (2 r^2)                                      (Eqs. eom, Hnu)
  one step r_n -> r_{n+1}: the classical RK4 tableau on the rotation group
     Y1 = P_n; Y2 = R(f1/2) P_n; Y3 = R(f2/2 - f1 x f2 / 8) P_n; Y4 = R(f3) P_n;
     P_{n+1} = R(Theta) P_n, Theta = (f1 + 2 f2 + 2 f3 + f4)/6 - f1 x f4 / 12,
     f_i = (h / c(r_i)) w(r_i, J(Y_i)), radii r_n, r_n + h/2, r_n + h/2, r_{n+1}
  renormalisation: P <- P / sqrt(P.P)

Every operation is analytic (no abs, conj or branches on values), so running it with
complex inputs x + i eps v gives the directional derivative Im(out)/eps exactly to
rounding (complex-step differentiation, Squire and Trapp 1998); eps = 1e-30 leaves no
truncation error.  Pinned in tests/test_oracle_bloch2.py against the plain mode.
"""
from __future__ import annotations

import numpy as np

# constants (the same physical values as oracle/nbo.h)
GF_GEV2 = 1.1663787e-5
HBARC_GEV_CM = 1.973269804e-14
HBARC_EV_KM = 1.973269804e-10
C_CM_S = 2.99792458e10
ERG_MEV = 6.241509074460763e5
F2 = 1.5 * 1.2020569031595942854          # int x^2/(e^x+1) dx = 3 zeta(3)/2
F3 = 7.0 * np.pi ** 4 / 120.0             # int x^3/(e^x+1) dx


def sqrt2gf_km() -> float:
    """sqrt(2) G_F n_e as a wavenumber in km^-1 per cm^-3."""
    hc3 = HBARC_GEV_CM ** 3
    return np.sqrt(2.0) * GF_GEV2 * hc3 / (HBARC_GEV_CM * 1.0e-5)


PARAMS = ("L_e", "L_ebar", "L_x", "theta_v", "n0")


def default_x(d: dict) -> np.ndarray:
    """The differentiated parameters (L_e, L_ebar, L_x, theta_v, n0) of a parameter dict."""
    L = d["lum_erg_s"]
    return np.array([L[0], L[1], L[2], d["theta"][0], d["n0_cm3"]], dtype=np.float64)


class Bloch2:
    """The model's fixed tables (geometry, energies, spectra shapes)."""

    def __init__(self, d: dict):
        assert d["n_flavor"] == 2 and not d.get("n_phi") and not d.get("track_all")
        assert not d.get("temp_xbar_mev"), "anti-nu_x = nu_x"
        self.d = dict(d)
        self.NE, self.NU = int(d["n_energy"]), int(d["n_u"])
        self.nb = 2 * self.NU * self.NE
        self.R = float(d["r_nu_km"])
        self.h = (d["r_end_km"] - d["r_start_km"]) / d["n_steps"]
        self.dE = (d["e_max_mev"] - d["e_min_mev"]) / self.NE
        self.E = d["e_min_mev"] + (np.arange(self.NE) + 0.5) * self.dE
        self.u = (np.arange(self.NU) + 0.5) / self.NU
        rcm = self.R * 1.0e5
        self.kappa0 = sqrt2gf_km() / (2.0 * np.pi * rcm * rcm * C_CM_S)
        T = d["temp_mev"]
        self.T = (float(T[0]), float(T[1]), float(T[2]))
        # per beam: species, emission bin, energy bin
        b = np.arange(self.nb)
        self.k = b % self.NE
        self.j = (b // self.NE) % self.NU
        self.s = b // (self.NE * self.NU)
        self.anti = self.s == 1

    def fermi_dirac(self, T):
        return self.E ** 2 / (F2 * T ** 3 * (np.exp(self.E / T) + 1.0))

    def weights(self, x):
        """g_b for the parameters x (luminosities enter as number luminosities L/<E>)."""
        N = [x[i] * ERG_MEV / (self.T[i] * F3 / F2) for i in range(3)]
        fe, feb, fx = (self.fermi_dirac(t) for t in self.T)
        pref = self.kappa0 * (1.0 / self.NU) * self.dE
        g_nu = pref * (N[0] * fe - N[2] * fx)
        g_an = pref * (N[1] * feb - N[2] * fx)
        return np.concatenate([np.tile(g_nu, self.NU), np.tile(g_an, self.NU)])

    def cos_theta(self, r):
        return np.sqrt(1.0 - self.u[self.j] * (self.R / r) ** 2)

    def w_vac(self, x):
        om = self.d["dm2_ev2"][0] / (4.0 * self.E * 1.0e6) / HBARC_EV_KM
        c2, s2 = np.cos(2.0 * x[3]), np.sin(2.0 * x[3])
        om = om[self.k]
        return np.stack([2.0 * om * s2, np.zeros_like(om) * s2, -2.0 * om * c2])

    def moments(self, P, g, r):
        """Vector parts of J0 and J1 (Eqs. Hnu, F)."""
        v = 0.5 * P
        v = np.where(self.anti, np.stack([-v[0], v[1], -v[2]]), v)
        c = self.cos_theta(r)
        j1 = (g * v).sum(axis=1)
        j0 = (g * v / c).sum(axis=1)
        return j0, j1

    def omega(self, wv, lam, J, r):
        j0, j1 = J
        c = self.cos_theta(r)
        mu = 0.5 * (self.R / r) ** 2
        dd = j0[:, None] - c[None, :] * j1[:, None]
        dd_conj = np.stack([dd[0], -dd[1], dd[2]])
        nn = np.where(self.anti, -2.0 * mu * dd_conj, 2.0 * mu * dd)
        z = np.where(self.anti, -lam, lam)
        w = wv + nn
        w = np.stack([w[0], w[1], w[2] + z])
        return w

    @staticmethod
    def rotate(f, P):
        """P rotated by the angle |f| about f (Rodrigues), analytic in f."""
        th2 = (f * f).sum(axis=0)
        th = np.sqrt(th2)
        sinc = np.sin(th) / th
        half = np.sin(0.5 * th) / th
        omc = 2.0 * half * half                   # (1 - cos th) / th^2
        cr = np.cross(f, P, axis=0)
        fp = (f * P).sum(axis=0)
        return P * np.cos(th) + cr * sinc + f * (fp * omc)

    def run(self, steps: int, x=None, state0=None, start_step: int = 0):
        """Bloch planes [3][nb] after `steps` steps from start_step, for parameters x (5
        values, complex allowed) and the start state (default: flavour eigenstates)."""
        d = self.d
        if x is None:
            x = default_x(d)
        dt = np.result_type(np.asarray(x), np.float64 if state0 is None else np.asarray(state0))
        P = np.zeros((3, self.nb), dtype=dt)
        if state0 is None:
            P[2] = 1.0
        else:
            P[:] = state0
        g = self.weights(x)
        wv = self.w_vac(x)
        lam0 = sqrt2gf_km() * x[4]
        p = int(d["ne_power"])
        h = self.h
        for n in range(start_step, start_step + steps):
            r0 = d["r_start_km"] + n * h
            rm = r0 + 0.5 * h
            r1 = d["r_start_km"] + (n + 1) * h
            lam = lambda r: lam0 * (self.R / r) ** p

            def f_of(Y, r):
                w = self.omega(wv, lam(r), self.moments(Y, g, r), r)
                return (h / self.cos_theta(r)) * w

            f1 = f_of(P, r0)
            f2 = f_of(self.rotate(0.5 * f1, P), rm)
            f3 = f_of(self.rotate(0.5 * f2 - 0.125 * np.cross(f1, f2, axis=0), P), rm)
            f4 = f_of(self.rotate(f3, P), r1)
            th = (f1 + 2.0 * f2 + 2.0 * f3 + f4) / 6.0 - np.cross(f1, f4, axis=0) / 12.0
            P = self.rotate(th, P)
            if d["renorm"]:
                P = P / np.sqrt((P * P).sum(axis=0))
        return P

    def pee(self, P):
        return 0.5 * (1.0 + P[2])

    def jvp(self, steps: int, dx=None, dstate=None, state0=None, eps: float = 1e-30):
        """Directional derivative of the final P_ee of every beam along the parameter
        direction dx (absolute units, 5 values) and the start-state direction dstate
        ([3][nb]), by complex-step differentiation."""
        x = default_x(self.d).astype(np.complex128)
        if dx is not None:
            x = x + 1j * eps * np.asarray(dx, dtype=np.float64)
        s0 = np.zeros((3, self.nb), np.complex128)
        if state0 is None:
            s0[2] = 1.0
        else:
            s0[:] = state0
        if dstate is not None:
            s0 = s0 + 1j * eps * np.asarray(dstate, dtype=np.float64)
        P = self.run(steps, x=x, state0=s0)
        return self.pee(P).imag / eps, self.pee(P.real)
