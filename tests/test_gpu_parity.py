"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element by element,
on seeded inputs small enough for the oracle: the water of the tiny configuration and
protein-shaped fragments with s, p and d shells whose sizes span several 256-lane tiles
with ragged tails.

Tolerances (FP64 path): surface and screening lists bit-exact; c, Bz and the Fock
correction within 1e-10 relative in norm; q within 1e-7 relative (max norm); energies within
1e-8 hartree; gradients within 1e-8 hartree/bohr times max(1, |g|max).
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import inputs as I

pytestmark = pytest.mark.gpu

CASES = {
    "water": lambda: I.water_tiny(),
    "frag6": lambda: I.small_protein(6, 50, seed=3),
    "frag12": lambda: I.small_protein(12, 110, seed=5),
}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module", params=list(CASES))
def case(request, torch_cuda):
    from paper_1505_07851_amd import Context, Molecule
    name = request.param
    print(f"\n[case {name}]", flush=True)
    s = CASES[name]()
    om = O.mol_from_system(s)
    ref = O.full_solution(om, s.P)
    ctx = Context()
    mol = Molecule.from_system(ctx, s)
    P = torch_cuda.tensor(s.P, dtype=torch_cuda.float64, device="cuda")
    return {"name": name, "s": s, "om": om, "ref": ref, "ctx": ctx, "mol": mol, "P": P}


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_surface_bit_exact(case):
    mol, om = case["mol"], case["om"]
    assert mol.M == om.M
    sf = mol.surface()
    raw = sf["owner"].cpu().numpy().astype(np.int64) * om.nsph + sf["sph"].cpu().numpy()
    assert np.array_equal(raw, om.keep_idx)
    assert np.abs(sf["r"].cpu().numpy() - om.r).max() <= 1e-13
    assert np.abs(sf["zeta"].cpu().numpy() - om.zeta).max() <= 1e-14 * om.zeta.max()
    S = sf["S"].cpu().numpy()
    assert np.all(np.abs(S - om.S) <= 1e-13 * np.maximum(om.S, 1e-8))
    assert np.all(np.abs(sf["Akk"].cpu().numpy() - om.Akk) <= 1e-12 * om.Akk)


def test_fock_pair_list_bit_exact(case):
    mol, om = case["mol"], case["om"]
    got = mol.pair_list(0)
    ref = om.pairs()
    for k in ("cls", "a", "b", "i", "j"):
        assert np.array_equal(got[k], ref[k]), k


def test_esp_and_bz(case, torch_cuda):
    mol, om, ref = case["mol"], case["om"], case["ref"]
    c, bz = mol.esp(case["P"])
    torch_cuda.cuda.synchronize()
    assert rel(c.cpu().numpy(), ref["c"]) <= 1e-10
    assert rel(bz.cpu().numpy(), ref["bz"]) <= 1e-13
    got = mol.pair_list(1)
    pr = om.pairs(case["s"].P)
    for k in ("cls", "a", "b", "i", "j"):
        assert np.array_equal(got[k], pr[k]), k


def test_fock(case, torch_cuda):
    mol, om = case["mol"], case["om"]
    rng = np.random.default_rng(17)
    qh = rng.normal(size=om.M)
    q = torch_cuda.tensor(qh, dtype=torch_cuda.float64, device="cuda")
    F0 = torch_cuda.tensor(rng.normal(size=(om.nbf, om.nbf)), dtype=torch_cuda.float64, device="cuda")
    F = mol.fock(q, F0.clone())
    Fr = om.fock(qh)
    d = F.cpu().numpy() - F0.cpu().numpy()
    assert rel(d, Fr) <= 1e-10
    assert np.abs(d - d.T).max() <= 1e-10 * np.abs(Fr).max()


@pytest.mark.parametrize("precond", ["none", "jacobi", "rbj", "octree"])
def test_solve_fp64(case, torch_cuda, precond):
    mol, om, ref = case["mol"], case["om"], case["ref"]
    v = torch_cuda.tensor(ref["bz"] + ref["c"], dtype=torch_cuda.float64, device="cuda")
    q, info = mol.solve(v, precond=precond, block=32, seed=104, tol=1e-10, max_iter=100000)
    qh = q.cpu().numpy()
    assert info["resid"] < 1e-10
    assert np.abs(qh - ref["q"]).max() <= 1e-7 * np.abs(ref["q"]).max()
    assert abs(info["energy"] - ref["E"]) <= 1e-8
    b = -om.f * (ref["bz"] + ref["c"])
    _, it = om.pcg(b, 1e-10, precond=precond, block=32, seed=104, A=ref["A"], max_iter=100000)
    # same algorithm, different rounding order: preconditioned counts agree to +-2; the long
    # unpreconditioned runs on the ill-conditioned A (diagonal spread 1e7-1e8, Sec. 4b) drift
    # with rounding, so they are held to 10%
    allow = 2 if precond != "none" else max(2, 0.10 * it)
    assert abs(info["iters"] - it) <= allow, (info["iters"], it)


@pytest.mark.parametrize("precond", ["jacobi", "rbj", "octree"])
def test_solve_mixed_refinement(case, torch_cuda, precond):
    mol, ref = case["mol"], case["ref"]
    v = torch_cuda.tensor(ref["bz"] + ref["c"], dtype=torch_cuda.float64, device="cuda")
    q, info = mol.solve(v, precond=precond, block=32, seed=104, tol=1e-10, precision="mixed")
    assert info["resid"] < 1e-10
    assert np.abs(q.cpu().numpy() - ref["q"]).max() <= 1e-7 * np.abs(ref["q"]).max()
    assert abs(info["energy"] - ref["E"]) <= 1e-8


def test_energy_eq13(case, torch_cuda):
    mol, ref = case["mol"], case["ref"]
    t = lambda a: torch_cuda.tensor(a, dtype=torch_cuda.float64, device="cuda")
    E = mol.energy(t(ref["bz"]), t(ref["c"]), t(ref["q"]))
    assert abs(E - ref["E"]) <= 1e-10 * max(1.0, abs(ref["E"]))


def test_gradient(case, torch_cuda):
    mol, om, ref, s = case["mol"], case["om"], case["ref"], case["s"]
    q = torch_cuda.tensor(ref["q"], dtype=torch_cuda.float64, device="cuda")
    gn, gs = mol.grad(case["P"], q)
    g = om.grad_terms(s.P, ref["q"])
    gnh, gsh = gn.cpu().numpy(), gs.cpu().numpy()
    scale = max(1.0, np.abs(g["g_nuc"]).max(), np.abs(g["g_surf"]).max())
    assert np.abs(gnh - g["g_nuc"]).max() <= 1e-8 * scale
    assert np.abs(gsh - g["g_surf"]).max() <= 1e-8 * scale
    tot = gnh.sum(0) + gsh.sum(0)
    assert np.abs(tot).max() <= 1e-10 * (np.abs(gnh).sum() + np.abs(gsh).sum())


def test_bitwise_reproducible(case, torch_cuda):
    mol = case["mol"]
    c1, _ = mol.esp(case["P"])
    c2, _ = mol.esp(case["P"])
    assert torch_cuda.equal(c1, c2)
    q1, _ = mol.solve(c1, tol=1e-9)
    q2, _ = mol.solve(c2, tol=1e-9)
    assert torch_cuda.equal(q1, q2)
    F1 = mol.fock(q1)
    F2 = mol.fock(q1)
    assert torch_cuda.equal(F1, F2)
    g1 = mol.grad(case["P"], q1)
    g2 = mol.grad(case["P"], q1)
    assert torch_cuda.equal(g1[0], g2[0]) and torch_cuda.equal(g1[1], g2[1])


def test_mixed_integrals_error_statement(case, torch_cuda):
    """FP32 Hermite/Boys evaluation with FP64 accumulation: stated error vs the FP64 oracle."""
    from paper_1505_07851_amd import Context, Molecule
    s, ref, om = case["s"], case["ref"], case["om"]
    ctx = Context(precision="mixed")
    mol = Molecule.from_system(ctx, s)
    c, bz = mol.esp(case["P"])
    q, info = mol.solve(bz + c, tol=1e-10, precision="mixed")
    rng = np.random.default_rng(2)
    qh = rng.normal(size=om.M)
    F = mol.fock(torch_cuda.tensor(qh, dtype=torch_cuda.float64, device="cuda"))
    gn, gs = mol.grad(case["P"], torch_cuda.tensor(ref["q"], dtype=torch_cuda.float64, device="cuda"))
    g = om.grad_terms(s.P, ref["q"])
    err = {"c_rel": rel(c.cpu().numpy(), ref["c"]), "E_abs": abs(info["energy"] - ref["E"]),
           "q_rel_max": np.abs(q.cpu().numpy() - ref["q"]).max() / np.abs(ref["q"]).max(),
           "F_rel": rel(F.cpu().numpy(), om.fock(qh)),
           "g_nuc_abs": np.abs(gn.cpu().numpy() - g["g_nuc"]).max(),
           "g_surf_abs": np.abs(gs.cpu().numpy() - g["g_surf"]).max()}
    print("mixed-precision errors vs FP64 oracle:", {k: f"{v:.2e}" for k, v in err.items()}, flush=True)
    # stated bounds of the mixed form (measured errors are printed above); q carries the
    # condition number of A times the relative error of c, so it is held to a looser bound
    # (measured: c 3e-9 to 9e-9, F 2e-8 to 2e-7 for these random charges of both signs)
    assert err["c_rel"] <= 3e-8 and err["F_rel"] <= 1e-6
    assert err["E_abs"] <= 1e-6
    assert err["q_rel_max"] <= 1e-3
    assert err["g_nuc_abs"] <= 1e-6 and err["g_surf_abs"] <= 1e-6


def test_matvec_shares_add_up(case, torch_cuda):
    """The per-rank shares of the sharded product add up to A x (dense oracle A), for rank counts
    below, at and above the number of tile pairs."""
    mol, ref = case["mol"], case["ref"]
    rng = np.random.default_rng(23)
    xh = rng.normal(size=mol.M)
    x = torch_cuda.tensor(xh, dtype=torch_cuda.float64, device="cuda")
    Ax = ref["A"] @ xh
    for nranks in (1, 2, 3, 7, 40):
        y = sum(mol.matvec_share(x, r, nranks).cpu().numpy() for r in range(nranks))
        assert rel(y, Ax) <= 1e-12, nranks
