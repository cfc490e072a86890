"""Nonpolar solvation forces coupled to a small MD integrator (torch tensors).

The nonpolar term of a GB/SA model is one surface tension times the molecular
SASA (Introduction and Methods, nonpolar solvation energy): E_np = gamma * sum_i
A_i, gamma 5 or 7 cal/(mol A^2) in the paper's simulations (0.005 / 0.007
kcal/(mol A^2)).  Its forces -gamma dA/dx come from the library through
``SASAFunction``: the forward computes the areas, the backward is the
library's VJP kernel (Eq. 2), so every step runs one forward and one backward
on the GPU.  The polar (GB) term needs a force field that is not part of this
package; harmonic bonds stand in for the bonded terms so that a molecule keeps
its shape.

Units: kcal/mol, Angstrom, amu, femtoseconds.

``velocity_verlet`` integrates at constant energy, so the drift and the
fluctuation of E = kinetic + potential check that the forces are the exact
derivative of the energy (the paper's supporting information checked energy
conservation with the method inside Amber).  ``langevin_baoab`` samples at a
temperature (the BAOAB splitting: half kick, half drift, Ornstein-Uhlenbeck
step, half drift, half kick).
"""
import math

import torch

ACC = 4.184e-4          # 1 kcal/(mol A amu) in A/fs^2
KE_UNIT = 1.0 / ACC     # 1 amu A^2/fs^2 in kcal/mol
KB = 0.0019872041       # Boltzmann constant, kcal/(mol K)


def bonds_by_distance(xyz, cutoff=1.6):
    """Index pairs (a < b) closer than ``cutoff`` and their lengths (harmonic bond rest lengths)."""
    x = torch.as_tensor(xyz, dtype=torch.float64)
    d = torch.cdist(x, x)
    a, b = torch.nonzero(torch.triu(d < cutoff, diagonal=1), as_tuple=True)
    return torch.stack([a, b], 1), d[a, b]


def masses_from_radii(radii, h_radius=1.2):
    """12 amu for heavy atoms, 1.008 amu for atoms with the hydrogen radius."""
    r = torch.as_tensor(radii, dtype=torch.float64)
    return torch.where(torch.isclose(r, torch.tensor(h_radius, dtype=torch.float64)),
                       torch.tensor(1.008, dtype=torch.float64), torch.tensor(12.0, dtype=torch.float64))


def bond_energy(x, bonds, r0, k_bond):
    d = x[bonds[:, 1]] - x[bonds[:, 0]]
    return (k_bond * (torch.linalg.norm(d, dim=1) - r0) ** 2).sum()


class NonpolarBondedModel:
    """U(x) = gamma * sum_i A_i(x) + sum over bonds k (|x_a - x_b| - r0)^2.

    The areas and their gradient come from the HIP library (``SASAFunction``);
    ``x`` must be a HIP tensor.
    """

    def __init__(self, radii, bonds, r0, gamma=0.005, k_bond=300.0, probe=1.4, precision="fp64"):
        self.radii = radii
        self.bonds = bonds
        self.r0 = r0
        self.gamma = gamma
        self.k_bond = k_bond
        self.probe = probe
        self.precision = precision

    def __call__(self, x):
        """Potential energy (float, kcal/mol), its parts, and the forces (tensor like x)."""
        from .autograd import sasa
        xr = x.detach().requires_grad_(True)
        area = sasa(xr, self.radii, self.probe, precision=self.precision)
        e_np = self.gamma * area.sum()
        e_b = bond_energy(xr, self.bonds, self.r0, self.k_bond)
        (e_np + e_b).backward()
        e_np, e_b = e_np.item(), e_b.item()
        return e_np + e_b, {"nonpolar": e_np, "bonds": e_b, "sasa": e_np / self.gamma if self.gamma else 0.0}, -xr.grad


def kinetic(v, m):
    return 0.5 * KE_UNIT * float((m[:, None] * v * v).sum())


def thermal_velocities(m, temperature, generator):
    """Maxwell-Boltzmann velocities (A/fs) with the centre-of-mass motion removed."""
    sd = torch.sqrt(KB * temperature * ACC / m)[:, None]
    v = torch.randn(m.shape[0], 3, dtype=torch.float64, generator=generator).to(m.device) * sd
    return v - (m[:, None] * v).sum(0) / m.sum()


def velocity_verlet(model, x, v, m, dt, steps):
    """Constant-energy run; returns x, v and per-step totals (potential, kinetic, total)."""
    x, v = x.clone(), v.clone()
    inv_m = (ACC / m)[:, None]
    u, _, f = model(x)
    trace = [(u, kinetic(v, m), u + kinetic(v, m))]
    for _ in range(steps):
        v = v + 0.5 * dt * f * inv_m
        x = x + dt * v
        u, _, f = model(x)
        v = v + 0.5 * dt * f * inv_m
        k = kinetic(v, m)
        trace.append((u, k, u + k))
    return x, v, trace


def langevin_baoab(model, x, v, m, dt, steps, temperature, friction_per_ps, generator):
    """Langevin dynamics (BAOAB); returns x, v, per-step (potential, kinetic, nonpolar energy)."""
    x, v = x.clone(), v.clone()
    inv_m = (ACC / m)[:, None]
    c1 = math.exp(-friction_per_ps * 1e-3 * dt)
    c2 = torch.sqrt((1.0 - c1 * c1) * KB * temperature * ACC / m)[:, None]
    u, parts, f = model(x)
    trace = []
    for _ in range(steps):
        v = v + 0.5 * dt * f * inv_m
        x = x + 0.5 * dt * v
        noise = torch.randn(v.shape, dtype=torch.float64, generator=generator).to(v.device)
        v = c1 * v + c2 * noise
        x = x + 0.5 * dt * v
        u, parts, f = model(x)
        v = v + 0.5 * dt * f * inv_m
        trace.append((u, kinetic(v, m), parts["nonpolar"]))
    return x, v, trace


def temperature_of(kinetic_energy, n_atoms):
    """Instantaneous temperature (K) for 3n - 3 degrees of freedom."""
    return 2.0 * kinetic_energy / ((3 * n_atoms - 3) * KB)
