"""Seeded synthetic workloads for the bulb-model radial stepper.

This module only *draws and names* inputs: physical parameters, bin counts and step
counts.  It contains none of the method's arithmetic, so both the CPU oracle (tests)
and the HIP path (binding, bench) may import it.

Random draws use SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) with a uniform double U = (x >> 11) * 2**-53.  The draw order
for each workload is fixed below; changing it changes every seeded value.

The physics values follow the bulb model of the paper (Sec. 2: neutrinosphere radius R,
Fermi-Dirac spectra, luminosities, two- or three-flavour mixing, n_e(r) = n0 (R/r)^3).
"""
from __future__ import annotations

import copy

SEED = 0x1912105960
MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 counter-based generator (Steele et al. 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


# Common physics (Sec. 2 of the paper; numbers as in the benchmark definitions).
TEMPS_MEV = (2.76, 4.01, 6.26)          # nu_e, anti-nu_e, nu_x (= anti-nu_x)
LUM_ERG_S = (1e51, 1e51, 1e51)
R_NU_KM = 10.0
E_MIN_MEV, E_MAX_MEV = 1.0, 50.0


def base_params(**kw) -> dict:
    """Parameter dict understood by both the oracle wrapper and the HIP binding."""
    p = dict(
        n_flavor=2, n_energy=32, n_u=16,
        e_min_mev=E_MIN_MEV, e_max_mev=E_MAX_MEV,
        r_nu_km=R_NU_KM, r_start_km=R_NU_KM, r_end_km=200.0, n_steps=2000,
        lum_erg_s=list(LUM_ERG_S), temp_mev=list(TEMPS_MEV),
        dm2_ev2=[-2.4e-3, 0.0], theta=[0.1, 0.0, 0.0], delta_cp=0.0,
        n0_cm3=1e33, ne_power=3, renorm=1, precision=0,
    )
    p.update(kw)
    return p


def draw_n0() -> float:
    """n0 of the single-model workloads: the first draw of the seeded stream."""
    g = SplitMix64(SEED)
    return 1e33 + 9e33 * g.uniform()


def two_flavor_small() -> dict:
    """2 flavours, 32 E x 16 u x 2 species = 1024 beams, 10 -> 200 km in 2000 steps."""
    return base_params(n_flavor=2, n_energy=32, n_u=16, r_end_km=200.0, n_steps=2000,
                       n0_cm3=draw_n0())


THREE_FLAVOR_MIX = dict(dm2_ev2=[7.5e-5, -2.4e-3], theta=[0.59, 0.15, 0.78], delta_cp=0.0)


def three_flavor_800k() -> dict:
    """3 flavours, 400 E x 1000 u x 2 species = 800k beams, 10 -> 1000 km in 20000 steps."""
    return base_params(n_flavor=3, n_energy=400, n_u=1000, r_end_km=1000.0, n_steps=20000,
                       n0_cm3=draw_n0(), **copy.deepcopy(THREE_FLAVOR_MIX))


def adjoint_200k() -> dict:
    """2 flavours, 200 E x 500 u x 2 = 200k beams, 10 -> 300 km in 5000 steps."""
    return base_params(n_flavor=2, n_energy=200, n_u=500, r_end_km=300.0, n_steps=5000,
                       n0_cm3=draw_n0())


# Start radius of the resolved adjoint variant: with the 200k workload's step length
# (0.058 km) every beam's per-step rotation angle is below one radian from here on (matter
# term included); nearer the neutrinosphere the step does not resolve the Hamiltonian and
# the linearised dynamics, hence the gradients, overflow.
ADJOINT_RESOLVED_START_KM = 500.0


def adjoint_200k_resolved() -> dict:
    """The 200k adjoint workload with its step length and step count kept and the start
    moved out to ADJOINT_RESOLVED_START_KM (500 -> 790 km)."""
    return resolved(adjoint_200k(), ADJOINT_RESOLVED_START_KM)


# Start radius of the resolved mixed-precision variant of the 6M-beam workload: with its
# step length (0.049 km) every beam's per-step rotation angle is below one radian from
# here on, so the FP32 stage arithmetic applies to every step.
MIXED_RESOLVED_START_KM = 600.0


def three_flavor_6m_resolved() -> dict:
    """The 6M-beam workload with its step length and step count kept and the start moved
    out to MIXED_RESOLVED_START_KM (600 -> 1090 km)."""
    return resolved(three_flavor_6m(), MIXED_RESOLVED_START_KM)


def three_flavor_6m() -> dict:
    """3 flavours, 1000 E x 3000 u x 2 = 6M beams, 10 -> 500 km in 10000 steps."""
    return base_params(n_flavor=3, n_energy=1000, n_u=3000, r_end_km=500.0, n_steps=10000,
                       n0_cm3=draw_n0(), **copy.deepcopy(THREE_FLAVOR_MIX))


def extended_paper(n_u: int = 10000) -> dict:
    """The extended bulb model in the shape of the paper's multi-node benchmark: 10
    azimuthal x 100 energy bins x n_u polar bins (10k-30k there) x 2 species, two flavours;
    radial grid and physics of the 1024-beam model (10 -> 200 km, 2000 steps)."""
    return base_params(n_flavor=2, n_energy=100, n_u=n_u, n_phi=10, n0_cm3=draw_n0())


def batch_256(n_models: int = 256) -> list[dict]:
    """256 independent 2-flavour models of uneven size, 10 -> 300 km in 5000 steps.

    Draw order per model: N_E, N_u, L_e, L_ebar, L_x, theta_v, n0.
    """
    g = SplitMix64(SEED)
    out = []
    for _ in range(n_models):
        ne = 50 + int(351 * g.uniform())
        nu = 100 + int(901 * g.uniform())
        le = (0.5 + 4.5 * g.uniform()) * 1e51
        leb = (0.5 + 4.5 * g.uniform()) * 1e51
        lx = (0.5 + 4.5 * g.uniform()) * 1e51
        th = 1e-3 + 0.599 * g.uniform()
        n0 = 1e33 + 9e33 * g.uniform()
        out.append(base_params(n_flavor=2, n_energy=ne, n_u=nu, r_end_km=300.0,
                               n_steps=5000, lum_erg_s=[le, leb, lx], theta=[th, 0.0, 0.0],
                               n0_cm3=n0))
    return out


def resolved(p: dict, r_start_km: float = 60.0) -> dict:
    """Same shapes and parameters with the start radius moved out to where the
    neutrino-neutrino term is resolved by the step (initial flavour states at r_start).
    The step length h is kept: the end radius moves out by the same amount."""
    q = copy.deepcopy(p)
    h = (p["r_end_km"] - p["r_start_km"]) / p["n_steps"]
    q["r_start_km"] = r_start_km
    q["r_end_km"] = r_start_km + h * p["n_steps"]
    return q


def small_params(n_flavor: int = 2, n_energy: int = 37, n_u: int = 5, n_steps: int = 40,
                 r_start_km: float = 60.0, r_end_km: float = 62.0, **kw) -> dict:
    """Small seeded cases used by the parity tests (ragged sizes on purpose)."""
    mix = THREE_FLAVOR_MIX if n_flavor == 3 else {}
    d = dict(n_flavor=n_flavor, n_energy=n_energy, n_u=n_u, n_steps=n_steps,
             r_start_km=r_start_km, r_end_km=r_end_km, n0_cm3=draw_n0())
    d.update(copy.deepcopy(mix))
    d.update(kw)
    return base_params(**d)
