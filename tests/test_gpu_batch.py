"""Batched solves through the C ABI (pcm_batch_create / pcm_solve_batched).

Several molecules with uneven surface sizes share one launch over a work table; groups of
PCG iterations are replayed from a captured hipGraph.  A molecule's kernels, partial-sum
slots and reduction orders do not depend on the rest of the batch or on the launch grid, so
the batched result must equal, bitwise, the molecule solved alone, with the same iteration
count.  The batch is also compared with the oracle's dense solution (Eq. 1).
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import inputs as I

pytestmark = pytest.mark.gpu

SYSTEMS = [
    ("water", lambda: I.water_tiny()),
    ("frag6", lambda: I.small_protein(6, 50, seed=3)),
    ("frag12", lambda: I.small_protein(12, 110, seed=5)),
    ("frag9", lambda: I.small_protein(9, 74, seed=8)),
]


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1505_07851_amd import Context, Molecule
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    print("\n[case batch of 4: water, frag6, frag12, frag9]", flush=True)
    ctx = Context()
    systems = [f() for _, f in SYSTEMS]
    mols = [Molecule.from_system(ctx, s) for s in systems]
    vs = []
    for s, m in zip(systems, mols):
        P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
        c, bz = m.esp(P)
        vs.append(bz + c)
    return torch, ctx, systems, mols, vs


@pytest.mark.parametrize("precond,precision", [("none", "fp64"), ("jacobi", "fp64"), ("rbj", "fp64"),
                                                ("octree", "fp64"), ("jacobi", "mixed"), ("rbj", "mixed"),
                                                ("octree", "mixed")])
def test_batch_equals_single(setup, precond, precision):
    # Unpreconditioned refinement is left out: points near the switching cut have
    # A_kk ~ 1/S_k up to ~1e8, cond(A) ~ 1e10, and restarted FP32 CG does not reduce the
    # FP64 residual to 1e-9 (plain FP64 CG needs tens of thousands of iterations there).
    from paper_1505_07851_amd import Batch
    torch, ctx, systems, mols, vs = setup
    kw = dict(precond=precond, block=40, seed=17, tol=1e-9, max_iter=100000, precision=precision)
    single = [m.solve(v, **kw) for m, v in zip(mols, vs)]
    b = Batch(ctx, mols)
    qs, infos = b.solve(vs, **kw)
    for (q1, i1), q2, i2, (name, _) in zip(single, qs, infos, SYSTEMS):
        assert i1["iters"] == i2["iters"], (name, i1["iters"], i2["iters"])
        assert i1["refinements"] == i2["refinements"], name
        assert torch.equal(q1, q2), name
        assert i1["energy"] == i2["energy"], name
        assert i2["resid"] < 1e-9
    b.close()


def test_batch_vs_oracle_and_replay(setup):
    from paper_1505_07851_amd import Batch
    torch, ctx, systems, mols, vs = setup
    b = Batch(ctx, mols)
    kw = dict(precond="rbj", block=40, seed=5, tol=1e-10, max_iter=10000)
    qs, infos = b.solve(vs, **kw)
    for s, q, info, v in zip(systems, qs, infos, vs):
        om = O.mol_from_system(s)
        ref = om.solve_dense(v.cpu().numpy())
        qh = q.cpu().numpy()
        assert np.abs(qh - ref).max() <= 1e-7 * np.abs(ref).max()
        E = 0.5 * float(v.cpu().numpy() @ ref)
        assert abs(info["energy"] - E) <= 1e-8
    # replays of the captured groups give the same bits; a looser tolerance stops earlier
    qs2, infos2 = b.solve(vs, **kw)
    for q, q2 in zip(qs, qs2):
        assert torch.equal(q, q2)
    qs3, infos3 = b.solve(vs, **dict(kw, tol=1e-6))
    for i, i3 in zip(infos, infos3):
        assert i3["iters"] < i["iters"] and i3["resid"] < 1e-6
    b.close()


def test_batch_warm_start_and_noconv(setup):
    from paper_1505_07851_amd import Batch
    torch, ctx, systems, mols, vs = setup
    b = Batch(ctx, mols)
    qs, infos = b.solve(vs, precond="jacobi", tol=1e-9)
    # warm start at the solution: nothing to do
    qw, iw = b.solve(vs, precond="jacobi", tol=1e-9, q0s=[q.clone() for q in qs])
    for q, q2, i in zip(qs, qw, iw):
        assert i["iters"] <= 2 and i["resid"] < 2e-9
        if i["iters"] == 0:
            assert torch.equal(q, q2)
        assert (q2 - q).abs().max().item() <= 1e-8 * q.abs().max().item()
    # max_iter reached: every molecule stops at the bound, status NOCONV, best iterate kept
    qn, inn = b.solve(vs, precond="none", tol=1e-14, max_iter=3, raise_noconv=False)
    for i in inn:
        assert i["status"] == 4 and i["iters"] == 3
        assert np.isfinite(i["resid"]) and np.isfinite(i["energy"])
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_esp_fock_equal_single(precision):
    """Batched c = L P and F += L^T q: one launch per class over all molecules; each molecule
    must get bitwise what the single-molecule call gives on the same context."""
    import torch
    from paper_1505_07851_amd import Batch, Context, Molecule
    print(f"\n[case batched esp/fock {precision}]", flush=True)
    ctx = Context(precision=precision)
    systems = [f() for _, f in SYSTEMS]
    mols = [Molecule.from_system(ctx, s) for s in systems]
    Ps = [torch.tensor(s.P, dtype=torch.float64, device="cuda") for s in systems]
    rng = np.random.default_rng(31)
    qs = [torch.tensor(rng.normal(size=m.M) * 1e-2, dtype=torch.float64, device="cuda") for m in mols]
    single_c = [m.esp(P) for m, P in zip(mols, Ps)]
    single_F = [m.fock(q) for m, q in zip(mols, qs)]
    b = Batch(ctx, mols)
    cs, bzs = b.esp(Ps)
    Fs = b.fock(qs)
    for (c1, bz1), c2, bz2, F1, F2, (name, _) in zip(single_c, cs, bzs, single_F, Fs, SYSTEMS):
        assert torch.equal(c1, c2), name
        assert torch.equal(bz1, bz2), name
        assert torch.equal(F1, F2), name
    # and against the oracle (FP64 tolerance of the single path; mixed: its error statement)
    tol = 1e-10 if precision == "fp64" else 1e-5
    for s, c, F, q in zip(systems, cs, Fs, qs):
        om = O.mol_from_system(s)
        cr = om.esp(s.P)
        assert np.linalg.norm(c.cpu().numpy() - cr) <= tol * np.linalg.norm(cr)
        Fr = om.fock(q.cpu().numpy())
        assert np.abs(F.cpu().numpy() - Fr).max() <= tol * max(np.abs(Fr).max(), 1e-12)
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "dynamic"])
def test_batch_grad_equal_single(precision):
    """Batched Eq. 14 gradient (pcm_grad_batched): one launch per class for the point side and
    one for the pair side over all molecules; each molecule gets bitwise what pcm_grad gives,
    and the FP64 form matches the oracle."""
    import torch
    from paper_1505_07851_amd import Batch, Context, Molecule
    print(f"\n[case batched gradient {precision}]", flush=True)
    ctx = Context(precision=precision)
    systems = [f() for _, f in SYSTEMS]
    mols = [Molecule.from_system(ctx, s) for s in systems]
    Ps = [torch.tensor(s.P, dtype=torch.float64, device="cuda") for s in systems]
    rng = np.random.default_rng(47)
    qs = [torch.tensor(rng.normal(size=m.M) * 1e-2, dtype=torch.float64, device="cuda") for m in mols]
    single = [m.grad(P, q) for m, P, q in zip(mols, Ps, qs)]
    b = Batch(ctx, mols)
    batched = b.grad(Ps, qs)
    for (gn1, gs1), (gn2, gs2), (name, _) in zip(single, batched, SYSTEMS):
        assert torch.equal(gn1, gn2), name
        assert torch.equal(gs1, gs2), name
    if precision == "fp64":
        for s, (gn, gs), q in zip(systems, batched, qs):
            om = O.mol_from_system(s)
            g = om.grad_terms(s.P, q.cpu().numpy())
            assert np.abs(gn.cpu().numpy() - g["g_nuc"]).max() <= 1e-8 * max(1.0, np.abs(g["g_nuc"]).max())
            assert np.abs(gs.cpu().numpy() - g["g_surf"]).max() <= 1e-8 * max(1.0, np.abs(g["g_surf"]).max())
    b.close()
