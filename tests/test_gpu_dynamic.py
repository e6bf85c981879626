"""Per-pair dynamic precision of the integrals (PCM_DYNAMIC): pairs whose screening bound reaches
dp_thresh are evaluated in FP64, the others in FP32 with FP64 accumulation.

* The two parts together are the FP64 lists exactly (merged entries and sizes).
* dp_thresh = 0 puts every pair in the FP64 part: c, F and the gradient equal the FP64 form bit
  for bit.  A threshold above every bound puts every pair in the FP32 part (FP32 records, Boys
  interpolation and far field, FP64 accumulation): the results then carry FP32 evaluation
  errors, within 1e-6 of the FP64 form, and differ from the mixed form (FP64 records, FP32
  Boys interpolation only).
* At the default 1e-6 the results stay within 1e-10 (c, F) and 1e-9 (gradient) of the oracle.
* Batched calls equal single calls bit for bit.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import inputs as I

pytestmark = pytest.mark.gpu

CASES = {
    "frag12": lambda: I.small_protein(12, 110, seed=5),
    "frag30": lambda: I.small_protein(30, 110, seed=8),
}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module", params=list(CASES))
def case(request, torch_cuda):
    name = request.param
    print(f"\n[case dynamic {name}]", flush=True)
    s = CASES[name]()
    om = O.mol_from_system(s)
    ref = O.full_solution(om, s.P)
    P = torch_cuda.tensor(s.P, dtype=torch_cuda.float64, device="cuda")
    q = torch_cuda.tensor(ref["q"], dtype=torch_cuda.float64, device="cuda")
    return {"s": s, "om": om, "ref": ref, "P": P, "q": q}


def _run(case, torch, **kw):
    from paper_1505_07851_amd import Context, Molecule
    mol = Molecule.from_system(Context(**kw), case["s"])
    c, bz = mol.esp(case["P"])
    F = mol.fock(case["q"])
    gn, gs = mol.grad(case["P"], case["q"])
    return mol, {"c": c, "F": F, "gn": gn, "gs": gs}


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_limits_are_the_fixed_precisions(case, torch_cuda):
    # fixed chunk shapes: separately autotuned contexts may choose different partial-sum orders
    torch = torch_cuda
    _, r64 = _run(case, torch, precision="fp64", autotune=False)
    _, r32 = _run(case, torch, precision="mixed", autotune=False)
    _, d0 = _run(case, torch, precision="dynamic", dp_thresh=0.0, autotune=False)
    _, dinf = _run(case, torch, precision="dynamic", dp_thresh=1e30, autotune=False)
    for k in r64:
        assert torch.equal(d0[k], r64[k]), k
        scale = r64[k].abs().max().item()
        assert (dinf[k] - r64[k]).abs().max().item() <= 1e-6 * max(1.0, scale), k
        assert (r32[k] - r64[k]).abs().max().item() <= 1e-7 * max(1.0, scale), k
    assert not torch.equal(dinf["c"], r32["c"])


def test_split_lists_cover_the_fp64_lists(case, torch_cuda):
    m64, _ = _run(case, torch_cuda, precision="fp64")
    md, _ = _run(case, torch_cuda, precision="dynamic", dp_thresh=1e-6)
    s64, sd = m64.sizes(), md.sizes()
    for k in ("pairs_fock", "pairs_esp", "sp_fock", "sp_esp"):
        assert list(s64[k]) == list(sd[k]), k
    for which in (0, 1):  # Fock list, esp list
        a, b = m64.pair_list(which), md.pair_list(which)
        for k in a:
            assert np.array_equal(a[k], b[k]), (which, k)


def test_default_threshold_against_oracle(case, torch_cuda):
    om, ref, s = case["om"], case["ref"], case["s"]
    _, r = _run(case, torch_cuda, precision="dynamic")
    assert rel(r["c"].cpu().numpy(), ref["c"]) <= 1e-10
    qh = ref["q"]
    Fr = om.fock(qh)
    assert rel(r["F"].cpu().numpy(), Fr) <= 1e-10
    g = om.grad_terms(s.P, qh)
    scale = max(1.0, np.abs(g["g_nuc"]).max(), np.abs(g["g_surf"]).max())
    assert np.abs(r["gn"].cpu().numpy() - g["g_nuc"]).max() <= 1e-9 * scale
    assert np.abs(r["gs"].cpu().numpy() - g["g_surf"]).max() <= 1e-9 * scale


def test_batched_dynamic_equals_single(torch_cuda):
    from paper_1505_07851_amd import Batch, Context, Molecule
    torch = torch_cuda
    systems = [I.small_protein(n, 74, seed=40 + n) for n in (6, 10, 14)]
    ctx = Context(precision="dynamic", dp_thresh=1e-7)
    mols = [Molecule.from_system(ctx, s) for s in systems]
    Ps = [torch.tensor(s.P, dtype=torch.float64, device="cuda") for s in systems]
    single = [m.esp(P) for m, P in zip(mols, Ps)]
    rng = np.random.default_rng(3)
    qs = [torch.tensor(rng.normal(size=m.M) * 1e-2, dtype=torch.float64, device="cuda") for m in mols]
    Fs = [m.fock(q) for m, q in zip(mols, qs)]
    b = Batch(ctx, mols)
    cb, bzb = b.esp(Ps)
    Fb = b.fock(qs)
    for (c1, bz1), c2, bz2, F1, F2 in zip(single, cb, bzb, Fs, Fb):
        assert torch.equal(c1, c2) and torch.equal(bz1, bz2) and torch.equal(F1, F2)
    b.close()
