"""Constant-energy dynamics with the oracle's SASA forces (CPU).

Velocity Verlet conserves E = kinetic + potential up to O(dt^2) when the
force is the exact derivative of the potential, so halving the step must cut
the largest energy excursion about four-fold; a force that is not the
derivative (the oracle's gradient scaled by 0.8, a planted mistake) must show
as a far larger excursion.  This pins the oracle's gradient against its own
area along a trajectory, and calibrates the same check run with the library.
The surface tension is 0.5 kcal/(mol A^2), a hundred times the paper's, so
that the surface forces are as large as the thermal bond forces.
"""
import numpy as np
import torch

from synth.globule import globule
from paper_2401_10462_amd.gbsa_md import bonds_by_distance, masses_from_radii, thermal_velocities, velocity_verlet
from tests._oracle_md import OracleModel


def _system():
    xyz, rad = globule(30, 3, hydrogens=True)  # 60 atoms
    bonds, r0 = bonds_by_distance(xyz)
    m = masses_from_radii(rad)
    v0 = thermal_velocities(m, 300.0, torch.Generator().manual_seed(5))
    return torch.tensor(xyz), rad, bonds, r0, m, v0


def _max_excursion(model, x0, v0, m, dt, steps):
    _, _, tr = velocity_verlet(model, x0, v0, m, dt, steps)
    e = np.array([t[2] for t in tr])
    return np.abs(e - e[0]).max()


def test_energy_conservation_oracle_forces():
    x0, rad, bonds, r0, m, v0 = _system()
    ok1 = _max_excursion(OracleModel(rad, bonds, r0, 0.5), x0, v0, m, 1.0, 150)
    ok2 = _max_excursion(OracleModel(rad, bonds, r0, 0.5), x0, v0, m, 0.5, 300)
    bad = _max_excursion(OracleModel(rad, bonds, r0, 0.5, grad_scale=0.8), x0, v0, m, 1.0, 150)
    print(f"max |E - E0|: dt 1 fs {ok1:.4f}, dt 0.5 fs {ok2:.4f}, planted 0.8 x gradient {bad:.4f} kcal/mol")
    assert ok2 < 0.4 * ok1          # second order in dt
    assert bad > 5.0 * ok1           # a wrong gradient shows
