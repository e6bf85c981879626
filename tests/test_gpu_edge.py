"""Degenerate inputs through the C ABI.

* Empty surface: with a switching cut above 1 every point is pruned (S_k <= 1); building
  such a surface is refused with PCM_E_ARG.
* A single hydrogen atom: M = 50 points in one ragged tile, two basis functions; c, q, E
  and the gradient against the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def test_empty_surface(torch_cuda):
    """A cavity with no kept points is refused when the surface is built (PCM_E_ARG), before
    any integral or solve could run on it; the context stays usable."""
    from paper_1505_07851_amd import Context, Molecule, PCMError
    print("\n[case empty surface]", flush=True)
    s = I.water_tiny()
    ctx = Context(switch_thresh=2.0)
    with pytest.raises(PCMError) as e:
        Molecule.from_system(ctx, s)
    assert e.value.status == 1 and "buried" in str(e.value)
    ok = Molecule.from_system(Context(), s)
    assert ok.M > 0


def test_single_atom(torch_cuda):
    from paper_1505_07851_amd import Context, Molecule
    torch = torch_cuda
    print("\n[case single H atom]", flush=True)
    s = I.small_protein(1, 50, seed=9)
    om = O.mol_from_system(s)
    ref = O.full_solution(om, s.P)
    ctx = Context()
    mol = Molecule.from_system(ctx, s)
    assert mol.M == om.M == 50
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    c, bz = mol.esp(P)
    assert np.linalg.norm(c.cpu().numpy() - ref["c"]) <= 1e-10 * np.linalg.norm(ref["c"])
    for precond in ("none", "jacobi", "rbj"):
        q, info = mol.solve(bz + c, precond=precond, block=7, seed=1, tol=1e-11)
        assert np.abs(q.cpu().numpy() - ref["q"]).max() <= 1e-7 * np.abs(ref["q"]).max()
        assert abs(info["energy"] - ref["E"]) <= 1e-9
    gn, gs = mol.grad(P, q)
    g = om.grad_terms(s.P, ref["q"])
    assert np.abs(gn.cpu().numpy() - g["g_nuc"]).max() <= 1e-8 * max(1.0, np.abs(g["g_nuc"]).max())
    assert np.abs(gs.cpu().numpy() - g["g_surf"]).max() <= 1e-8 * max(1.0, np.abs(g["g_surf"]).max())
