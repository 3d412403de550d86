"""Independent NumPy/SciPy references used to pin the oracle (tests only).

Everything here is written directly from the paper's formulas and from textbook results,
with its own constants and its own quadrature of the spectra; it shares nothing with the
oracle's C code.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, linalg

HBARC_GEV_CM = 1.973269804e-14
HBARC_EV_KM = 1.973269804e-10
GF_GEV2 = 1.1663787e-5
C_CM_S = 2.99792458e10
ERG_MEV = 6.241509074460763e5


def sqrt2gf_km_cm3() -> float:
    """sqrt(2) G_F (hbar c)^3 / (hbar c) in km^-1 cm^3: potential per unit number density."""
    return np.sqrt(2.0) * GF_GEV2 * HBARC_GEV_CM ** 3 / (HBARC_GEV_CM * 1e-5)


def fd_moments():
    """Integrals int x^n/(e^x+1) dx for n = 2, 3 by adaptive quadrature."""
    f2 = integrate.quad(lambda x: x * x / (np.exp(x) + 1.0), 0, 200, epsabs=1e-14, limit=200)[0]
    f3 = integrate.quad(lambda x: x ** 3 / (np.exp(x) + 1.0), 0, 200, epsabs=1e-14, limit=200)[0]
    return f2, f3


def spectrum(E, T):
    """Normalised Fermi-Dirac energy distribution (zero chemical potential)."""
    f2, _ = fd_moments()
    return E ** 2 / (f2 * T ** 3 * (np.exp(E / T) + 1.0))


def mean_energy(T):
    f2, f3 = fd_moments()
    return T * f3 / f2


def omega_km(dm2_ev2, E_mev):
    """dm^2 / (4E) in km^-1."""
    return dm2_ev2 / (4.0 * E_mev * 1e6) / HBARC_EV_KM


def pmns(t12, t13, t23):
    c12, s12, c13, s13, c23, s23 = (np.cos(t12), np.sin(t12), np.cos(t13), np.sin(t13),
                                    np.cos(t23), np.sin(t23))
    R23 = np.array([[1, 0, 0], [0, c23, s23], [0, -s23, c23]])
    U13 = np.array([[c13, 0, s13], [0, 1, 0], [-s13, 0, c13]])
    R12 = np.array([[c12, s12, 0], [-s12, c12, 0], [0, 0, 1]])
    return R23 @ U13 @ R12


def hvac3(d, E):
    U = pmns(*d["theta"])
    m = np.diag([0.0, d["dm2_ev2"][0], d["dm2_ev2"][1]]) / (2.0 * E * 1e6) / HBARC_EV_KM
    return U @ m @ U.T


def hvac2(d, E):
    w = omega_km(d["dm2_ev2"][0], E)
    t = d["theta"][0]
    return w * np.array([[-np.cos(2 * t), np.sin(2 * t)], [np.sin(2 * t), np.cos(2 * t)]])


def path_length(r, rs, R, u):
    """Length travelled from radius rs to r by a beam emitted at sin^2(theta_R) = u."""
    return np.sqrt(r * r - u * R * R) - np.sqrt(rs * rs - u * R * R)


def bins(d):
    NE, NU = d["n_energy"], d["n_u"]
    dE = (d["e_max_mev"] - d["e_min_mev"]) / NE
    E = d["e_min_mev"] + (np.arange(NE) + 0.5) * dE
    u = (np.arange(NU) + 0.5) / NU
    return E, dE, u, 1.0 / NU


def _n_f_xbar(d, E):
    """Number luminosity and spectrum of anti-nu_x: its own (lum_xbar_erg_s, temp_xbar_mev)
    when temp_xbar_mev is set, else those of nu_x."""
    T = d.get("temp_xbar_mev", 0.0) or d["temp_mev"][2]
    L = d["lum_xbar_erg_s"] if d.get("temp_xbar_mev", 0.0) else d["lum_erg_s"][2]
    return L * ERG_MEV / mean_energy(T), spectrum(E, T)


def brute_h_nunu(d, r, rho_e, rho_ebar):
    """H_nunu for every (species, angle, energy) beam by the direct pair sum of Eq. Hnu.

    rho_e, rho_ebar: [NU, NE, n, n] density matrices of the nu_e-born and anti-nu_e-born
    beams.  All four (six) initial flavours are summed explicitly: heavy-flavour-born
    states are obtained from unitarity (they started orthogonal to the electron state and
    evolve with the same Hamiltonian), i.e. sum over the other flavours = I - rho_e.
    Returns [2, NU, NE, n, n] (neutrino and antineutrino Hamiltonians' nu-nu parts as
    they enter each equation: +H_nunu for neutrinos, -H_nunu^* for antineutrinos).
    """
    n = rho_e.shape[-1]
    E, dE, u, du = bins(d)
    R = d["r_nu_km"]
    L = d["lum_erg_s"]; T = d["temp_mev"]
    Nnum = [L[a] * ERG_MEV / mean_energy(T[a]) for a in range(3)]
    fe, fb, fx = spectrum(E, T[0]), spectrum(E, T[1]), spectrum(E, T[2])
    Nxb, fxb = _n_f_xbar(d, E)
    I = np.eye(n)
    cth = np.sqrt(1.0 - u * (R / r) ** 2)
    # number density of the emitted flux per d cos(theta'): L_N/(2 pi R^2 c) at the
    # neutrinosphere; at radius r, d cos(theta') = (R^2 / 2 r^2) du / cos(theta')
    pref = sqrt2gf_km_cm3() / (2.0 * np.pi * (R * 1e5) ** 2 * C_CM_S)
    Hnn = np.zeros((2, len(u), len(E), n, n), complex)
    for j in range(len(u)):
        for jp in range(len(u)):
            geo = (1.0 - cth[j] * cth[jp]) * (R * R / (2 * r * r)) * du / cth[jp]
            F = np.zeros((n, n), complex)
            for kp in range(len(E)):
                w = dE
                Fe = Nnum[0] * fe[kp] * rho_e[jp, kp]
                Fx = Nnum[2] * fx[kp] * (I - rho_e[jp, kp])          # nu_mu + nu_tau (or nu_x)
                Fb = Nnum[1] * fb[kp] * rho_ebar[jp, kp]
                Fbx = Nxb * fxb[kp] * (I - rho_ebar[jp, kp])       # anti-nu_mu + anti-nu_tau
                F += w * (Fe + Fx - np.conj(Fb + Fbx))
            Hnn[0, j] += pref * geo * F
    Hnn[1] = -np.conj(Hnn[0])
    return Hnn


def bvec(H):
    """B vector of a 2x2 Hermitian matrix: H = B.sigma/2 + trace."""
    return np.array([2 * H[0, 1].real, -2 * H[0, 1].imag, (H[0, 0] - H[1, 1]).real])


def expm_apply(H, L, psi):
    return linalg.expm(-1j * H * L) @ psi


def brute_h_nunu_ext(d, r, rho_e, rho_ebar):
    """H_nunu of the extended bulb model by the direct pair sum of Eq. Hnu with the
    azimuthal replacements of Eq. int-v: 1 - v.v' = 1 - [c c' + s s' cos(phi - phi')] and
    the average (1/2 pi) int dphi' taken over n_phi equal bins.

    rho_e, rho_ebar: [NU, NP, NE, n, n].  Returns [2, NU, NP, NE, n, n] as brute_h_nunu.
    """
    n = rho_e.shape[-1]
    E, dE, u, du = bins(d)
    NP = d["n_phi"]
    phi = 2.0 * np.pi * (np.arange(NP) + 0.5) / NP
    R = d["r_nu_km"]
    L = d["lum_erg_s"]; T = d["temp_mev"]
    Nnum = [L[a] * ERG_MEV / mean_energy(T[a]) for a in range(3)]
    fe, fb, fx = spectrum(E, T[0]), spectrum(E, T[1]), spectrum(E, T[2])
    I = np.eye(n)
    cth = np.sqrt(1.0 - u * (R / r) ** 2)
    sth = np.sqrt(u) * (R / r)
    pref = sqrt2gf_km_cm3() / (2.0 * np.pi * (R * 1e5) ** 2 * C_CM_S)
    F = np.zeros((len(u), NP, n, n), complex)          # energy-integrated source per bin
    for jp in range(len(u)):
        for pp in range(NP):
            for kp in range(len(E)):
                Fe = Nnum[0] * fe[kp] * rho_e[jp, pp, kp]
                Fx = Nnum[2] * fx[kp] * (I - rho_e[jp, pp, kp])
                Fb = Nnum[1] * fb[kp] * rho_ebar[jp, pp, kp]
                Fbx = Nnum[2] * fx[kp] * (I - rho_ebar[jp, pp, kp])
                F[jp, pp] += dE * (Fe + Fx - np.conj(Fb + Fbx))
    Hnn = np.zeros((2, len(u), NP, len(E), n, n), complex)
    for j in range(len(u)):
        for p in range(NP):
            acc = np.zeros((n, n), complex)
            for jp in range(len(u)):
                for pp in range(NP):
                    vv = cth[j] * cth[jp] + sth[j] * sth[jp] * np.cos(phi[p] - phi[pp])
                    geo = (1.0 - vv) * (R * R / (2 * r * r)) * du / cth[jp] / NP
                    acc += geo * F[jp, pp]
            Hnn[0, j, p] = pref * acc
    Hnn[1] = -np.conj(Hnn[0])
    return Hnn
