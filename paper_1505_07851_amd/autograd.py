"""Differentiable solvation energy (Sec. 2, Eqs. 1, 13, 14) as a torch.autograd.Function.

E = PCMEnergy.apply(P, R_nuc, r_surf, mol, opts) places the nuclei at R_nuc and the kept
surface points at r_surf (independent inputs), forms c = L P and Bz, solves A q = -f(Bz + c)
and returns the Eq. 13 energy.  Because E is stationary in q at the solution, backward needs
no adjoint solve: dE/dP = sum_k q_k L^k (the pcm_fock output, returned unchanged when the
incoming gradient is 1), dE/dR_nuc = g_nuc and dE/dr_surf = g_surf of pcm_grad.

To move the points with their atoms, build r_surf from R_nuc with torch operations
(r_surf = R_nuc[owner] + radius[owner, None] * u) and autograd composes the two gradients.
The molecule keeps the geometry of the last forward call: call backward before the next
forward on the same molecule.
"""
from __future__ import annotations

import torch

from .api import Molecule


class PCMEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, R_nuc, r_surf, mol: Molecule, opts=None):
        opts = dict(opts or {})
        xyz = R_nuc.detach().to("cpu", torch.float64).numpy()
        rs = None if r_surf is None else r_surf.detach().to("cpu", torch.float64).numpy()
        mol.update_geometry(xyz, rs)
        Pd = P.detach().contiguous()
        c, bz = mol.esp(Pd)
        q, info = mol.solve(bz + c, **opts)
        ctx.mol = mol
        ctx.has_surf = r_surf is not None
        ctx.dev_R = R_nuc.device
        ctx.dev_r = None if r_surf is None else r_surf.device
        ctx.save_for_backward(Pd, q)
        ctx.info = info
        return torch.tensor(info["energy"], dtype=torch.float64, device=P.device)

    @staticmethod
    def backward(ctx, gE):
        Pd, q = ctx.saved_tensors
        mol = ctx.mol
        g = gE.to(torch.float64)
        dP = dR = dr = None
        if ctx.needs_input_grad[0]:
            F = mol.fock(q)
            dP = F if bool(g == 1.0) else F * g
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            gn, gs = mol.grad(Pd, q)
            if ctx.needs_input_grad[1]:
                dR = (gn if bool(g == 1.0) else gn * g).to(ctx.dev_R)
            if ctx.needs_input_grad[2] and ctx.has_surf:
                dr = (gs if bool(g == 1.0) else gs * g).to(ctx.dev_r)
        return dP, dR, dr, None, None


def pcm_energy(P, R_nuc, r_surf, mol: Molecule, **opts):
    """Functional form of PCMEnergy.apply."""
    return PCMEnergy.apply(P, R_nuc, r_surf, mol, opts)
