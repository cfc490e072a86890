"""The MD harness with the library's SASA forces (SASAFunction forward + VJP kernel).

Constant-energy runs of the 60-atom system of test_md_energy_oracle: the
largest energy excursion must fall about four-fold when the step is halved
(forces that are the energy's derivative) and stay within twice what the same
run with the oracle's forces gives.  A Langevin run at the paper's surface
tension must hold its temperature.
"""
import numpy as np
import pytest
import torch

from synth.globule import globule
from paper_2401_10462_amd.gbsa_md import (NonpolarBondedModel, bonds_by_distance, langevin_baoab, masses_from_radii,
                                          temperature_of, thermal_velocities, velocity_verlet)
from tests._oracle_md import OracleModel

pytestmark = pytest.mark.gpu


def _excursion(model, x0, v0, m, dt, steps):
    _, _, tr = velocity_verlet(model, x0, v0, m, dt, steps)
    e = np.array([t[2] for t in tr])
    assert np.isfinite(e).all()
    return np.abs(e - e[0]).max()


@pytest.fixture(scope="module")
def system():
    xyz, rad = globule(30, 3, hydrogens=True)
    bonds, r0 = bonds_by_distance(xyz)
    m = masses_from_radii(rad)
    v0 = thermal_velocities(m, 300.0, torch.Generator().manual_seed(5))
    ref = _excursion(OracleModel(rad, bonds, r0, 0.5), torch.tensor(xyz), v0, m, 1.0, 150)
    return xyz, rad, bonds, r0, m, v0, ref


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_energy_conservation_library_forces(system, prec):
    xyz, rad, bonds, r0, m, v0, ref = system
    dev = torch.device("cuda:0")
    print(f"NVE 60 atoms {prec}", flush=True)
    model = NonpolarBondedModel(torch.tensor(rad, device=dev), bonds.to(dev), r0.to(dev), gamma=0.5, precision=prec)
    x0 = torch.tensor(xyz, device=dev)
    e1 = _excursion(model, x0, v0.to(dev), m.to(dev), 1.0, 150)
    e2 = _excursion(model, x0, v0.to(dev), m.to(dev), 0.5, 300)
    print(f"max |E - E0|: dt 1 fs {e1:.4f}, dt 0.5 fs {e2:.4f}, oracle forces at 1 fs {ref:.4f} kcal/mol", flush=True)
    assert e2 < 0.4 * e1
    assert e1 < 2.0 * ref


def test_langevin_holds_temperature():
    xyz, rad = globule(1000, 8, hydrogens=True)  # 2,000 atoms
    dev = torch.device("cuda:0")
    print("Langevin 2000 atoms, gamma 0.007, 300 K, 300 steps of 1 fs", flush=True)
    bonds, r0 = bonds_by_distance(xyz)
    m = masses_from_radii(rad).to(dev)
    g = torch.Generator().manual_seed(9)
    v0 = thermal_velocities(m.cpu(), 300.0, g).to(dev)
    model = NonpolarBondedModel(torch.tensor(rad, device=dev), bonds.to(dev), r0.to(dev), gamma=0.007,
                                precision="mixed")
    _, _, tr = langevin_baoab(model, torch.tensor(xyz, device=dev), v0, m, 1.0, 300, 300.0, 5.0, g)
    temps = np.array([temperature_of(k, len(rad)) for _, k, _ in tr])
    e_np = np.array([t[2] for t in tr])
    assert np.isfinite(temps).all() and np.isfinite(e_np).all()
    assert 240.0 < temps[-100:].mean() < 360.0
    assert (e_np > 0).all()
