"""Force provider for the MD harness tests built on the FP64 oracle (CPU)."""
import torch

import oracle
from paper_2401_10462_amd.gbsa_md import bond_energy


class OracleModel:
    """gamma * sum_i A_i + harmonic bonds, areas and gradient from the oracle.

    grad_scale != 1 plants a force that is not the energy's derivative (used
    only to show that the energy check catches such a mistake).
    """

    def __init__(self, rad, bonds, r0, gamma, k_bond=300.0, grad_scale=1.0):
        self.rad, self.bonds, self.r0 = rad, bonds, r0
        self.gamma, self.k_bond, self.grad_scale = gamma, k_bond, grad_scale

    def __call__(self, x):
        ref = oracle.run(x.detach().cpu().numpy(), self.rad, 1.4)
        xr = x.detach().cpu().requires_grad_(True)
        eb = bond_energy(xr, self.bonds, self.r0, self.k_bond)
        eb.backward()
        f = -self.gamma * self.grad_scale * torch.from_numpy(ref.dadx) - xr.grad
        e_np = self.gamma * float(ref.area.sum())
        return e_np + eb.item(), {"nonpolar": e_np, "bonds": eb.item()}, f.to(x.device)
