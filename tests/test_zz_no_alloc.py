"""The allocation-free share of the product (pcm_matvec_share_noalloc) against the entry
point it mirrors (pcm_matvec_share): same kernels and summation order, so the two must agree
bit for bit.  Two calls in a row on one context, the second on a smaller molecule, so the
second call reuses scratch that still holds the first call's larger partial slots."""
import ctypes

import numpy as np
import pytest

from synth import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def _mol(ctx, s):
    from paper_1505_07851_amd import Molecule
    return Molecule.from_system(ctx, s)


def test_noalloc_share_equals_share(torch_cuda):
    torch = torch_cuda
    from paper_1505_07851_amd import Context
    ctx = Context()
    big = _mol(ctx, I.small_protein(30, 110, seed=11))  # M = 1,230
    small = _mol(ctx, I.water_tiny())
    assert big.M > 4 * 256 and big.M % 256 != 0, big.M  # several tiles and a ragged tail
    assert small.M < big.M
    g = torch.Generator(device="cpu").manual_seed(2024)
    for mol, rank, nranks in [(big, 0, 1), (small, 0, 1), (big, 2, 3), (small, 1, 2)]:
        print(f"[noalloc] M={mol.M} rank={rank}/{nranks}", flush=True)
        x = torch.randn(mol.M, generator=g, dtype=torch.float64).cuda()
        y_ref = mol.matvec_share(x, rank, nranks)
        y = torch.full((mol.M,), float("nan"), dtype=torch.float64, device="cuda")
        mol.matvec_share_noalloc(x, y, rank, nranks)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        scale = y_ref.abs().max().item()
        assert (y - y_ref).abs().max().item() <= 1e-13 * scale
        assert torch.equal(y, y_ref), "same kernels and order: expected identical bits"


def test_noalloc_full_product_sums_shares(torch_cuda):
    torch = torch_cuda
    from paper_1505_07851_amd import Context
    ctx = Context()
    mol = _mol(ctx, I.small_protein(12, 110, seed=5))
    x = torch.randn(mol.M, generator=torch.Generator(device="cpu").manual_seed(7), dtype=torch.float64).cuda()
    full = torch.empty(mol.M, dtype=torch.float64, device="cuda")
    mol.matvec_share_noalloc(x, full, 0, 1)
    parts = []
    for r in range(3):
        y = torch.empty(mol.M, dtype=torch.float64, device="cuda")
        mol.matvec_share_noalloc(x, y, r, 3)
        parts.append(y.clone())
    torch.cuda.synchronize()
    tot = parts[0] + parts[1] + parts[2]
    assert (tot - full).abs().max().item() <= 1e-12 * full.abs().max().item()


def test_noalloc_rejects_before_any_work(torch_cuda):
    torch = torch_cuda
    from paper_1505_07851_amd import Context, Molecule
    from paper_1505_07851_amd import _lib as C
    ctx = Context()
    # 1,000 isolated atoms with a 50-point rule keep every point: M = 50,000, too many
    n, nsph = 1000, 50
    xyz = np.zeros((n, 3))
    xyz[:, 0] = np.arange(n) * 20.0
    dirs, w = I.sphere_rule(nsph)
    basis = I.Basis(shell_atom=np.zeros(1, np.int32), shell_l=np.zeros(1, np.int32),
                    shell_nprim=np.ones(1, np.int32), shell_off=np.zeros(1, np.int32),
                    prim_exp=np.ones(1), prim_coef=np.ones(1))
    mol = Molecule(ctx, xyz, np.ones(n), np.full(n, 2.0), dirs, w, basis)
    assert mol.M == n * nsph
    x = torch.zeros(mol.M, dtype=torch.float64, device="cuda")
    y = torch.zeros(mol.M, dtype=torch.float64, device="cuda")
    L = ctx.lib
    st = L.pcm_matvec_share_noalloc(ctx.h, mol.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 0, 1)
    assert st == C.PCM_E_ARG
    assert b"scratch" in L.pcm_last_error(ctx.h)
    small = _mol(ctx, I.water_tiny())
    xs = torch.zeros(small.M + 1, dtype=torch.float64, device="cuda")
    ys = torch.zeros(small.M + 1, dtype=torch.float64, device="cuda")
    bad = ctypes.c_void_p(xs.data_ptr() + 4)  # misaligned
    assert L.pcm_matvec_share_noalloc(ctx.h, small.h, bad, ctypes.c_void_p(ys.data_ptr()), 0, 1) == C.PCM_E_ARG
    assert L.pcm_matvec_share_noalloc(ctx.h, small.h, ctypes.c_void_p(xs.data_ptr()),
                                      ctypes.c_void_p(ys.data_ptr()), 3, 3) == C.PCM_E_ARG
