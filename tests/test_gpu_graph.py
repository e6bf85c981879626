"""The batched pass captured as one hipGraph (pcm_graph_capture / pcm_graph_launch) against the
same pass run eagerly (pcm_esp_batched, pcm_solve_batched, pcm_fock_batched) on a batch of
molecules with uneven surfaces: the same kernels in the same order, so c, Bz, q, the energy and
F must agree bit for bit on every replay (several replays, with other GPU work and host
synchronisation between them), and q against the oracle's dense solution."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import inputs as I

pytestmark = pytest.mark.gpu

SYSTEMS = [lambda: I.water_tiny(), lambda: I.small_protein(6, 50, seed=3), lambda: I.small_protein(12, 110, seed=5),
           lambda: I.small_protein(20, 110, seed=9)]
KW = dict(precond="rbj", block=32, seed=104, tol=1e-9)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def test_graph_replays_equal_eager(torch_cuda):
    torch = torch_cuda
    from paper_1505_07851_amd import Batch, Context, Molecule, PCMError
    systems = [f() for f in SYSTEMS]
    ctx = Context()
    mols = [Molecule.from_system(ctx, s) for s in systems]
    print("\n[graph] M =", [m.M for m in mols], flush=True)
    Ps = [torch.tensor(s.P, dtype=torch.float64, device="cuda") for s in systems]
    b = Batch(ctx, mols)
    cs, bzs = b.esp(Ps)
    qs, infos = b.solve([bz + c for c, bz in zip(cs, bzs)], max_iter=600, **KW)
    Fs = b.fock(qs)
    torch.cuda.synchronize()
    g = b.capture(Ps, max_iter=600, **KW)
    other = Molecule.from_system(Context(), I.small_protein(8, 50, seed=21))  # not in the batch
    Po = torch.tensor(I.small_protein(8, 50, seed=21).P, dtype=torch.float64, device="cuda")
    for rep in range(3):
        for F in g.Fs:
            F.zero_()
        g.replay()
        ginfo, nodes = g.info()
        print(f"[graph] replay {rep}: nodes {nodes}, iters {[d['iters'] for d in ginfo]}", flush=True)
        for i in range(len(mols)):
            assert torch.equal(g.cs[i], cs[i]), (rep, i)
            assert torch.equal(g.bzs[i], bzs[i]), (rep, i)
            assert ginfo[i]["iters"] == infos[i]["iters"], (rep, i)
            assert torch.equal(g.qs[i], qs[i]), (rep, i)
            # the energy of a replay is formed on the device, the eager one on the host
            assert abs(g.E[i].item() - infos[i]["energy"]) <= 1e-14 * abs(infos[i]["energy"]), (rep, i)
            assert torch.equal(g.Fs[i], Fs[i]), (rep, i)
            assert ginfo[i]["converged"]
        # other work on the device and the host between replays
        other.esp(Po)
        torch.cuda.synchronize()
    # the batch and its molecules refuse other calls while the graph holds their buffers
    with pytest.raises(PCMError):
        mols[0].esp(Ps[0])
    with pytest.raises(PCMError):
        b.esp(Ps)
    # the oracle's dense solution for one molecule
    om = O.mol_from_system(systems[2])
    ref = O.full_solution(om, systems[2].P)
    qh = g.qs[2].cpu().numpy()
    assert np.abs(qh - ref["q"]).max() <= 1e-7 * np.abs(ref["q"]).max()
    assert abs(g.E[2].item() - ref["E"]) <= 1e-8
    g.close()
    c0, _ = mols[0].esp(Ps[0])  # usable again
    assert torch.equal(c0, cs[0])
    b.close()


def test_graph_reads_current_density(torch_cuda):
    torch = torch_cuda
    from paper_1505_07851_amd import Batch, Context, Molecule
    systems = [f() for f in SYSTEMS[1:3]]
    ctx = Context()
    mols = [Molecule.from_system(ctx, s) for s in systems]
    Ps = [torch.tensor(s.P, dtype=torch.float64, device="cuda") for s in systems]
    b = Batch(ctx, mols)
    g = b.capture(Ps, max_iter=600, **KW)
    g.replay()
    torch.cuda.synchronize()
    c1 = [c.clone() for c in g.cs]
    for P in g.Ps:
        P.mul_(1.25)  # same screening (every weight grows), new coefficients at the next replay
    g.replay()
    torch.cuda.synchronize()
    for a, b_ in zip(g.cs, c1):
        assert ((a - 1.25 * b_).norm() / a.norm()).item() <= 1e-14
    g.close()
    b.close()


def test_graph_refuses_mixed_solve(torch_cuda):
    torch = torch_cuda
    import ctypes
    from paper_1505_07851_amd import Batch, Context, Molecule
    from paper_1505_07851_amd import _lib as C
    from paper_1505_07851_amd.api import _solve_opts
    s = I.water_tiny()
    ctx = Context()
    m = Molecule.from_system(ctx, s)
    b = Batch(ctx, [m])
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    bufs = [m._zeros(m.M) for _ in range(3)] + [m._zeros(m.nbf, m.nbf)]
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    o = _solve_opts(ctx.lib, "jacobi", 1, 0, 1e-8, 100, "mixed", 1e-4)
    p = b._ptrs
    h = ctypes.c_void_p()
    st = ctx.lib.pcm_graph_capture(ctx.h, b.h, p([P]), p([bufs[0]]), p([bufs[1]]), p([bufs[2]]), p([bufs[3]]),
                                   ctypes.c_void_p(E.data_ptr()), ctypes.byref(o), ctypes.byref(h))
    assert st == C.PCM_E_UNSUPPORTED
    b.close()


def test_graph_budget_too_small_reports_noconv(torch_cuda):
    torch = torch_cuda
    from paper_1505_07851_amd import Batch, Context, Molecule
    from paper_1505_07851_amd import _lib as C
    systems = [f() for f in SYSTEMS[1:3]]
    ctx = Context()
    mols = [Molecule.from_system(ctx, s) for s in systems]
    Ps = [torch.tensor(s.P, dtype=torch.float64, device="cuda") for s in systems]
    b = Batch(ctx, mols)
    g = b.capture(Ps, max_iter=3, **KW)  # three iterations cannot reach 1e-9
    g.replay()
    torch.cuda.synchronize()
    infos, _ = g.info()
    for d in infos:
        assert d["status"] == C.PCM_E_NOCONV
        assert not d["converged"] and 1 <= d["iters"] <= 3
        assert np.isfinite(d["resid"]) and d["resid"] > KW["tol"]
    g.close()
    b.close()
