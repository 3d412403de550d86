"""The HIP FP64 path against the oracle's plain mode (oracle/plain.c): an evaluation of the
step straight from its definitions (density matrices, dense per-beam generators and
commutators, Jacobi exponentials, plain FP64 sums, exact renormalisation) that shares no
algorithm with the kernels.

Bar: max |dP_ee| <= 1e-10 over every beam (the FP64 target).  The cases are resolved runs,
where the step resolves every beam's Hamiltonian and two FP64 evaluations of the method
with different rounding agree to a few 1e-14; on the literal configurations near the
neutrinosphere the discrete evolution amplifies rounding to O(1) and the kernels are held
to the specification oracle bit for bit instead (tests/test_gpu_parity.py).
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nb():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_1912_10596_amd as nb
    nb.lib()
    return nb


def _case(name):
    if name == "2f_1024_60_1000km":      # the 1024-beam shape from 60 km, h = 0.235 km
        return dict(workloads.resolved(workloads.two_flavor_small(), 60.0), r_end_km=1000.0,
                    n_steps=4000), None
    if name == "3f_37x5_600_1000km":
        return workloads.small_params(n_flavor=3, n_energy=37, n_u=5, n_steps=800,
                                      r_start_km=600.0, r_end_km=1000.0), None
    if name == "3f_130x7_two_chunks":    # 3 lane passes per row, ragged tail
        return workloads.small_params(n_flavor=3, n_energy=130, n_u=7, n_steps=400,
                                      r_start_km=600.0, r_end_km=800.0), None
    if name == "3f_800k_600km_30st":     # benchmark shape and launch, its step length
        return workloads.resolved(workloads.three_flavor_800k(), 600.0), 30
    if name == "2f_200k_500km_200st":    # adjoint workload shape, resolved variant
        return workloads.adjoint_200k_resolved(), 200
    if name == "3f_6m_shape_600km_200st":  # the 6M workload's energy grid and step, 30 angles
        return dict(workloads.three_flavor_6m_resolved(), n_u=30), 200
    if name == "3f_ext_5phi":
        return workloads.small_params(n_flavor=3, n_energy=11, n_u=4, n_phi=5, n_steps=800,
                                      r_start_km=600.0, r_end_km=1000.0), None
    if name == "3f_track_all":
        return dict(workloads.small_params(n_flavor=3, n_energy=9, n_u=3, n_steps=300,
                                           r_start_km=600.0, r_end_km=900.0), track_all=1), None
    if name == "2f_track_all_xbar":
        return dict(workloads.small_params(n_flavor=2, n_energy=40, n_u=6, n_steps=2000,
                                           r_start_km=60.0, r_end_km=530.0,
                                           lum_xbar_erg_s=1.7e51, temp_xbar_mev=5.3),
                    track_all=1), None
    raise KeyError(name)


CASES = ["2f_1024_60_1000km", "3f_37x5_600_1000km", "3f_130x7_two_chunks", "3f_ext_5phi",
         "3f_track_all", "2f_track_all_xbar", "2f_200k_500km_200st", "3f_800k_600km_30st",
         "3f_6m_shape_600km_200st"]


@pytest.mark.parametrize("name", CASES)
def test_fp64_path_against_plain_oracle(nb, oracle, name):
    d, steps = _case(name)
    _say(f"case {name}: {d['n_flavor']}f {d['n_energy']}x{d['n_u']} n_phi={d.get('n_phi', 0)} "
         f"track_all={d.get('track_all', 0)} steps={steps or d['n_steps']}")
    g = nb.Model(d)
    o = oracle.PlainModel(d, species4=int(d.get("track_all", 0)))
    if steps is None:
        g.run(); o.run()
    else:
        g.step(steps); o.step(steps)
    pg = g.pee().cpu().numpy()
    po = o.pee().reshape(-1)
    dp = float(np.abs(pg - po).max())
    _say(f"  max |dP_ee| = {dp:.3e}, min P_ee = {po.min():.4f}")
    assert np.abs(po - 1.0).max() > 1e-4        # the run does convert flavour
    assert dp <= TOL
