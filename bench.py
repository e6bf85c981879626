#!/usr/bin/env python
"""Benchmark of the C-PCM solvation hot path on one MI355X.

One step = one pass of the whole path over the 600-atom protein-shaped solute
(6-31G*-shaped basis, ~50 kept surface points per atom, M ~ 30k):
  geometry update (surface switching values, A_kk, pair geometry), c = L P with its point
  derivative dc and Bz (one point-side integral pass), the randomized block-Jacobi PCG solve of
  A q = -f (Bz + c) from q = 0 (blocks of 512 points), the Eq. 13 energy, then F += L^T q with the
  Eq. 14 gradient (one pair-side pass over the Eq. 18 list and a Fock pass over the rest of the
  Eq. 15 list).
The value is shell-pair x point integrals per second over the whole step (c, the gradient and
F counted), with the PCG solve time and its residual reported beside it.  The FP64 path gives
the line's value; beside it the mixed form (FP32 Boys-table interpolation, FP32 matvec inside
FP64 refinement), the per-pair dynamic form (FP64 or FP32 integral evaluation by screening
bound, FP32 matvec inside FP64 refinement) and the solve-only mixed form, each compared with
the FP64 state solved to 1e-10.  Inputs are synthetic and seeded (see synth/inputs.py).

Second workload (--workload conformers64): 64 seeded conformers of a 150-atom peptide
(6-31G-shaped basis, nbf 825, 3.9k-9k kept points each).  One step = c = L P with Bz,
the RBJ-100 PCG solve, the Eq. 13 energy and F += L^T q for all 64, batched (one launch per
class for the integrals, hipGraph-replayed PCG iteration groups over all conformers), and the
same pass captured whole as one hipGraph (pcm_graph_capture: one launch per step, FP64 PCG
with a fixed iteration budget), against the same 64 done one after another with the plain FP64
single-molecule calls.
The geometries are fixed, so surfaces, pair lists and RBJ blocks are built before timing.

Third workload (--workload stress2000): the 2,000-atom solute (M ~ 150k).  Fifteen
SCF-like outer iterations t = 1..15, each with its own density P_t = 2 C_t C_t^T,
C_t = orth(C_{t-1} + e_t G_t), and its own c_t = L P_t evaluated on the GPU (timed
separately), solve A q = -f (Bz + c_t) with the threshold tightening as
delta_t = 10^(-3 - 4(t-1)/14) (the Eq. 21 range), each solve warm-started from the previous q;
unpreconditioned and RBJ with blocks of 1,024 points, FP64 and mixed (FP32 matvec in FP64
refinement).

One GPU's share of the sharded matvec (--workload shard8): the 2,000-atom solute's product split
over 8 ranks as a multi-GPU solve would split it; each rank's kernel time at its real shape,
the balance, and the reduce-scatter volume per CG iteration.

Studies (--workload scf_policies, eq21_fit): the synthetic analogues of the solver-policy
and threshold experiments of Sec. 4b (CG steps per SCF iteration under fixed, 2-delta and
dynamic thresholds; RBJ against the octree partition over seeds; the power-law fit of the
energy error against the CG threshold).  They print one JSON line each, with the counts.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
                       [--workload protein600|conformers64|stress2000|scf_policies|eq21_fit|shard8]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shell-pair×point integrals/s + PCG solve ms at stated error, mixed vs FP64"
PEAK_F64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop/FMA x 2.4 GHz (FP64 and unpacked FP32)
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ntuv(L):
    return (L + 1) * (L + 2) * (L + 3) // 6


def hermite_flops():
    """FP64 flops (FMA = 2) of the straight-line R_tuv build for L = 0..5, counted from the
    generated source the kernels compile."""
    txt = open(os.path.join(ROOT, "paper_1505_07851_amd", "csrc", "hermite_gen.h")).read()
    out = {}
    for L in range(6):
        body = re.search(r"void md_R%d\(.*?\n}\n" % L, txt, re.S).group(0)
        n = 0
        for line in body.splitlines():
            if "const T r" not in line:
                continue
            if "fma(" in line:
                n += 3 if "T(" in line.split("fma(")[1] else 2
            else:
                n += 1
        out[L] = n
    return out


# FP64 flops (FMA = 2, 1/sqrt = 1) per (primitive pair x point) evaluation of the kernels that
# contract the auxiliary R^(n) in factored form, counted from the far-field branch of
# their source.  Point side: the common part 13 + 2N (P - C 3, r^2 5, far test 2, 1/sqrt 1,
# r^-2 1, R^(0) 1, R^(n) 2 each up to N) plus the contraction and accumulation.  Pair side with
# FP64 records (V up to order N >= 1): the far-field factored sums, 12 (P - C 3, r^2 5, far
# test 2, 1/sqrt 1, r^-2 1) + s_0 .. s_N (N + 1) + the sums: 7 (N = 1), 23 (N = 2), 53 (N = 3),
# 106 (N = 4).
#   point side, c only (N = L):               esp_L          15  24  45  87
#   point side, dc (N = L + 1):               grad_pts_L     22  37  75 156
#   point side, c and dc:                     esp_grad_pts_L 24  41  81 164
#   pair side, V up to L (N = L):             fock_v_L       15  21  38  69 123
#   pair side, V' up to L + 1 (N = L + 1):    grad_v_L       21  38  69 123
#                                             fock_grad_v_L  21  38  69 123
FACTORED = {"esp": (15, 24, 45, 87), "grad_pts": (22, 37, 75, 156), "esp_grad_pts": (24, 41, 81, 164),
            "fock_v": (15, 21, 38, 69, 123), "grad_v": (21, 38, 69, 123), "fock_grad_v": (21, 38, 69, 123)}


def flop_model():
    """Algorithmic FP64 flops per (primitive pair x point) evaluation, far-field branch.  The
    kernels that contract R^(n) in factored form (FACTORED) are counted from their own source;
    the others form every R_tuv and contract it (table form): P - C (3), r^2 (5), far test (1),
    1/sqrt (1), 1/r^2 (1), R^(0) (1), R^(n) (2 per n), Hermite recursion H(L), contraction (2 per
    coefficient), accumulation (1)."""
    H = hermite_flops()
    m = {}
    for L in range(5):
        base = 12 + 2 * L + H[L]
        m[f"esp_L{L}"] = base + 2 * ntuv(L) + 1
        m[f"fock_v_L{L}"] = base + 2 * ntuv(L)
        b1 = 12 + 2 * (L + 1) + H[L + 1]
        m[f"grad_pts_L{L}"] = b1 + 3 * 2 * ntuv(L) + 3
        m[f"grad_v_L{L}"] = b1 + 2 * ntuv(L + 1)
        m[f"esp_grad_pts_L{L}"] = m[f"grad_pts_L{L}"] + 2 * ntuv(L)  # the potential beside its derivative
        m[f"fock_grad_v_L{L}"] = m[f"grad_v_L{L}"]
    for fam, counts in FACTORED.items():
        for L, n in enumerate(counts):
            m[f"{fam}_L{L}"] = n
    # per unordered point pair (A is symmetric and each pair is evaluated once): d (3), r^2 (5),
    # far test (1), 1/sqrt (1), row FMA (2), column product (1), column sum (1)
    m["matvec"] = 14
    m["grad_aoff"] = 23
    return m


def family_rooflines(prof, model, n_prof):
    """Model TFLOP/s and fraction of the FP64 peak per kernel family of the FP64 step, over all its
    classes: the point side (c with dc), the pair side over the Eq. 18 list (F and the gradient),
    the Fock-only pass over the rest of the Eq. 15 list, and the product; and the HBM rate of the
    block-Jacobi apply against the 8 TB/s peak."""
    fams = {"point_side": r"esp_grad_pts_L\d_f64", "pair_side": r"fock_grad_v_L\d_f64", "fock_only": r"fock_v_L\d_f64",
            "matvec": r"matvec_f64"}
    out = {}
    for fam, pat in fams.items():
        ks = [k for k in prof if re.fullmatch(pat, k)]
        ms = sum(prof[k]["ms"] for k in ks)
        if not ks or ms <= 0:
            continue
        tf = sum(kernel_flops(k, prof[k]["work"], model) for k in ks) / (ms * 1e-3) / 1e12
        out[fam] = {"ms_per_step": round(ms / n_prof, 3), "model_tflops": round(tf, 3),
                    "frac": round(tf / PEAK_F64_TFLOPS, 4)}
    # the block-Jacobi apply is bound by HBM: every inverse entry of every block is read once per
    # application (8 bytes each; the gathered residual and the written z add under 1%)
    ra = prof.get("rbj_apply")
    if ra and ra["ms"] > 0:
        gbs = 8.0 * ra["work"] / (ra["ms"] * 1e-3) / 1e9
        out["rbj_apply"] = {"ms_per_step": round(ra["ms"] / n_prof, 3), "bound": "hbm",
                            "bytes_per_launch": round(8.0 * ra["work"] / ra["launches"]),
                            "GB_per_s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}
    return out


def kernel_flops(name, work, model):
    key = re.sub(r"_(f64|f32|mix)$", "", name)
    key = "matvec" if key.startswith("matvec") else key
    return model.get(key, 0) * work


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--tol-ref", type=float, default=1e-10,
                    help="solve tolerance of the untimed accuracy pass that every form is compared on")
    ap.add_argument("--prof-steps", type=int, default=3, help="steps of the profiled (per-kernel) pass")
    ap.add_argument("--nearfar-points", type=int, default=2048, help="nearfar: sampled surface points")
    ap.add_argument("--block", type=int, default=None,
                    help="RBJ block size of the solves; default 512 for the 600-atom system (the fastest expected "
                         "solve + setup of --workload rbj_blocks) and the paper's 100 for the conformers")
    ap.add_argument("--workload", default="protein600",
                    choices=["protein600", "conformers64", "stress2000", "scf_policies", "eq21_fit", "shard8", "copy",
                             "oracle1t", "nearfar", "rbj_blocks"],
                    help="copy: a plain device copy of known size, to calibrate rocprofv3 byte counters")
    ap.add_argument("--max-iter-none", type=int, default=300,
                    help="stress2000: matvec budget of each unpreconditioned outer solve")
    ap.add_argument("--seeds", type=int, default=20,
                    help="scf_policies, and rbj_blocks on protein2000: RBJ seeds per block size")
    ap.add_argument("--scf-system", default="protein600", choices=["protein600", "protein2000"],
                    help="scf_policies and rbj_blocks: the 600-atom solute (M ~ 30k) or the 2,000-atom one (M ~ 150k)")
    args = ap.parse_args()
    if args.block is None:
        args.block = 100 if args.workload == "conformers64" else 512
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the collectives of a multi-GPU run are "
                                   "not implemented (--workload shard8 times one GPU's share of the sharded "
                                   "product)", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "conformers64":
        return bench_conformers(args)
    if args.workload == "stress2000":
        return bench_stress(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "scf_policies":
        return bench_scf_policies(args)
    if args.workload == "eq21_fit":
        return bench_eq21_fit(args)
    if args.workload == "shard8":
        return bench_shard(args)
    if args.workload == "oracle1t":
        return bench_oracle1t(args)
    if args.workload == "nearfar":
        return bench_nearfar(args)
    if args.workload == "rbj_blocks":
        return bench_rbj_blocks(args)

    import numpy as np
    import torch

    from paper_1505_07851_amd import Context, Molecule
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    s = I.protein_single_solve()
    log(f"[bench] inputs ready in {time.time() - t0:.1f}s: {s.n_atoms} atoms, nbf={s.basis.nbf}")
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    model = flop_model()

    n_prof = max(1, min(args.steps, args.prof_steps))

    def run_form(prec, solve_prec=None, label=None):
        solve_prec = solve_prec or ("mixed" if prec == "mixed" else "fp64")
        label = label or prec
        ctx = Context(precision=prec)
        t = time.time()
        mol = Molecule.from_system(ctx, s)
        torch.cuda.synchronize()
        log(f"[bench] {label}: surface + pair lists built in {time.time() - t:.2f}s, M={mol.M}")
        state = {}

        def step(tol=args.tol):
            # one pass of the path: geometry, c and dc_k = dc_k/dr_k with Bz (one integral pass), the
            # RBJ-preconditioned solve, then F += L^T q and the Eq. 14 gradient (one integral pass)
            mol.update_geometry(s.xyz)
            c, bz, dc = mol.esp_deriv(P)
            q, info = mol.solve(bz + c, precond="rbj", block=args.block, seed=s.seeds["rbj"], tol=tol,
                                precision=solve_prec, q0=state.get("q"))
            F, gn, gs = mol.fock_grad(P, q, dc)
            state.update(c=c, bz=bz, q=q, info=info, F=F, gn=gn, gs=gs)
            return info

        for w in range(args.warmup):
            info = step()
            torch.cuda.synchronize()
            log(f"[bench] {label}: warmup {w} done, solve {info['solve_ms']:.1f} ms, iters {info['iters']}")
        # production pass: no per-kernel events, PCG iteration groups replayed from the captured graph
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = []
        for k in range(args.steps):
            state.pop("q", None)  # every step solves from scratch
            infos.append(step())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        log(f"[bench] {label}: {args.steps} steps, {dt * 1e3:.1f} ms/step")
        # profiled pass: HIP events around every heavy launch on the library's stream; the PCG then
        # steps one iteration at a time with the states read back, so only the kernel table and the
        # launch durations come from it
        ctx.profile(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(n_prof):
            state.pop("q", None)
            step()
        torch.cuda.synchronize()
        dt_prof = (time.perf_counter() - t) / n_prof
        prof = ctx.profile_read()
        ctx.profile(False)
        log(f"[bench] {label}: {n_prof} profiled steps, {dt_prof * 1e3:.1f} ms/step")
        # accuracy pass at a tight solve tolerance (untimed): the state compared across forms
        state.pop("q", None)
        info_t = step(tol=args.tol_ref)
        torch.cuda.synchronize()
        tight = {k: v for k, v in state.items()}
        sz = mol.sizes()
        return {"ctx": ctx, "mol": mol, "ms": dt * 1e3, "ms_prof": dt_prof * 1e3, "prof": prof, "sizes": sz,
                "infos": infos, "state": state, "tight": tight, "info_tight": info_t, "label": label}

    r64 = run_form("fp64")
    mol = r64["mol"]
    sz = r64["sizes"]
    M = mol.M
    sp_esp, sp_fock = sum(sz["sp_esp"]), sum(sz["sp_fock"])
    integrals = (2 * sp_esp + sp_fock) * M   # c, gradient (esp list) and F (Eq. 15 list)
    value = integrals / (r64["ms"] * 1e-3)

    # dominant kernel and its roofline (launch durations from the profiled pass)
    prof = r64["prof"]
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    avg_ms = d["ms"] / d["launches"]
    flops = kernel_flops(dom, d["work"] / d["launches"], model)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": PEAK_F64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_TFLOPS, 4), "traffic": measured_traffic(dom),
            "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops}
    # the dominant integral kernel on the factored flop model (ALU bound, FP64 peak)
    ints = {k: v for k, v in prof.items() if re.match(r"(esp|fock|grad)", k) and kernel_flops(k, 1.0, model) > 0}
    dom_i = max(ints, key=lambda k: ints[k]["ms"])
    di = ints[dom_i]
    avg_i = di["ms"] / di["launches"]
    flops_i = kernel_flops(dom_i, di["work"] / di["launches"], model)
    ach_i = flops_i / (avg_i * 1e-3) / 1e12
    roof_int = {"bound": "alu", "kernel": dom_i, "achieved": round(ach_i, 3), "peak": PEAK_F64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach_i / PEAK_F64_TFLOPS, 4), "avg_launch_ms": round(avg_i, 4),
                "flops_per_launch": flops_i, "flops_per_evaluation": kernel_flops(dom_i, 1.0, model),
                "evaluations_per_launch": di["work"] / di["launches"]}
    kernels = {k: {"ms_per_step": round(v["ms"] / n_prof, 3), "launches": v["launches"],
                   "tflops": round(kernel_flops(k, v["work"], model) / (v["ms"] * 1e-3) / 1e12, 3)
                   if v["ms"] > 0 else None,
                   "work_units_per_s": round(v["work"] / (v["ms"] * 1e-3), 1) if v["ms"] > 0 else None}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    info64 = r64["infos"][-1]
    ref = r64["tight"]
    E_ref = r64["info_tight"]["energy"]
    # shell-pair x point integrals/s per total angular momentum L = l_a + l_b (classes ss, sp, sd, pp,
    # pd, dd have L = 0, 1, 2, 2, 3, 4): the c, F and gradient integrals of the L classes over the time
    # of their two kernels (point side with c, pair side with F)
    cls_L = [0, 1, 2, 2, 3, 4]
    by_L = {}
    for L in range(5):
        spe = sum(n for n, l in zip(sz["sp_esp"], cls_L) if l == L)
        spf = sum(n for n, l in zip(sz["sp_fock"], cls_L) if l == L)
        t_p = prof.get(f"esp_grad_pts_L{L}_f64", {}).get("ms", 0.0)
        # the pair side: F and the gradient over the Eq. 18 list, F alone over the rest of Eq. 15
        t_v = prof.get(f"fock_grad_v_L{L}_f64", {}).get("ms", 0.0) + prof.get(f"fock_v_L{L}_f64", {}).get("ms", 0.0)
        rate = lambda n, t: round(n * M * n_prof / (t * 1e-3), 1) if t > 0 else None
        by_L[f"L{L}"] = {"shell_pairs_esp": spe, "shell_pairs_fock": spf, "point_side": rate(spe, t_p),
                         "pair_side": rate(spf, t_v), "c_F_grad": rate(2 * spe + spf, t_p + t_v)}

    out = {"metric": METRIC, "value": value, "unit": "shell-pair×point integrals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r64["ms"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "protein600_631gs", "atoms": s.n_atoms, "nbf": mol.nbf, "surface_points": M,
                      "raw_points_per_atom": int(s.sph_w.shape[0]), "shell_pairs_esp": sp_esp,
                      "shell_pairs_fock": sp_fock, "prim_pairs_esp": sum(sz["pairs_esp"]),
                      "prim_pairs_fock": sum(sz["pairs_fock"]), "precond": f"rbj{args.block}", "tol": args.tol},
           "pcg_solve_ms": round(info64["solve_ms"], 3), "pcg_setup_ms": round(info64["setup_ms"], 3),
           "pcg_iters": info64["iters"], "pcg_resid": info64["resid"], "energy": info64["energy"],
           "profiled_ms_per_step": round(r64["ms_prof"], 3), "profiled_steps": n_prof,
           "roofline": roof, "roofline_integrals": roof_int,
           "roofline_by_family": family_rooflines(prof, model, n_prof), "integrals_per_s_by_L": by_L,
           "kernels": kernels,
           "reference": {"solve_tol": args.tol_ref, "energy": E_ref, "resid": r64["info_tight"]["resid"]}}

    def errors(st, info_t, info_prod):
        rel = lambda a, b: (a - b).norm().item() / b.norm().item()
        return {"E_abs": abs(info_t["energy"] - E_ref), "E_abs_at_tol": abs(info_prod["energy"] - E_ref),
                "q_rel_max": (st["q"] - ref["q"]).abs().max().item() / ref["q"].abs().max().item(),
                "q_rel_norm": rel(st["q"], ref["q"]),
                "c_rel": rel(st["c"], ref["c"]), "F_rel": rel(st["F"], ref["F"]),
                "g_nuc_abs_max": (st["gn"] - ref["gn"]).abs().max().item(),
                "g_surf_abs_max": (st["gs"] - ref["gs"]).abs().max().item()}

    out["err_fp64_at_tol"] = {"E_abs": abs(info64["energy"] - E_ref)}
    # the mixed form (FP32 Boys-table interpolation in the integrals, FP32 matvec in FP64 refinement),
    # the per-pair dynamic form (FP64 or FP32 integrals by screening bound, FP32 matvec in FP64
    # refinement) and the solve-only mixed form (FP64 integrals, FP32 matvec in FP64 refinement), each
    # compared with the FP64 path's state at the tight tolerance
    forms = {}
    form_list = [("mixed", "mixed", "mixed"), ("dynamic", "mixed", "dynamic"), ("fp64", "mixed", "solve_mixed")]
    for form, sprec, label in ([] if args.no_mixed else form_list):
        rmx = run_form(form, sprec, label)
        key = rmx["label"]
        forms[key] = rmx
        infm = rmx["infos"][-1]
        sm = rmx["sizes"]
        integ_m = (2 * sum(sm["sp_esp"]) + sum(sm["sp_fock"])) * rmx["mol"].M
        out[key] = {"value": integ_m / (rmx["ms"] * 1e-3), "ms_per_step": round(rmx["ms"], 3),
                    "speedup_vs_fp64": round(r64["ms"] / rmx["ms"], 3),
                    "pcg_solve_ms": round(infm["solve_ms"], 3),
                    "solve_speedup_vs_fp64": round(info64["solve_ms"] / infm["solve_ms"], 3),
                    "pcg_iters": infm["iters"], "pcg_refinements": infm["refinements"], "pcg_resid": infm["resid"],
                    "err_vs_fp64_ref": errors(rmx["tight"], rmx["info_tight"], infm),
                    "kernels": {k: round(v["ms"] / n_prof, 3) for k, v in
                                sorted(rmx["prof"].items(), key=lambda kv: -kv[1]["ms"])[:8]}}
        if form == "dynamic":
            out[key]["dp_thresh"] = 1e-6
        e = out[key]["err_vs_fp64_ref"]
        # the FP64 path's own tolerances, and the targets stated for the mixed-integral form
        out[key]["meets_fp64_tolerances"] = bool(e["E_abs"] <= 1e-8 and e["q_rel_max"] <= 1e-7 and
                                                 e["c_rel"] <= 1e-10 and e["F_rel"] <= 1e-10)
        out[key]["meets_mixed_targets"] = bool(e["E_abs"] <= 1e-6 and e["q_rel_norm"] <= 1e-6)
        del rmx["ctx"], rmx["mol"]
    # the fastest form at the FP64 path's own accuracy (the equal-accuracy comparison)
    eq = [k for k in ("mixed", "dynamic", "solve_mixed") if k in out and out[k]["meets_fp64_tolerances"]]
    if eq:
        k = max(eq, key=lambda k: out[k]["speedup_vs_fp64"])
        out["equal_accuracy"] = {"form": k, "ms_per_step": out[k]["ms_per_step"],
                                 "speedup_vs_fp64": out[k]["speedup_vs_fp64"],
                                 "criterion": "vs the FP64 path solved to 1e-10: E <= 1e-8, q <= 1e-7 (max rel), "
                                              "c and F <= 1e-10 (rel)"}

    if not args.no_cpu_baseline:
        base = oracle_baseline(s, r64, forms, sp_esp, sp_fock)
        for form, err in base.pop("form_c_err").items():
            out[form]["c_sample_rel_err_vs_oracle"] = err
        out.update(base)
    print(json.dumps(out))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_baseline(s, r64, forms, sp_esp, sp_fock):
    """The FP64 oracle timed on the host cores as it stands (a baseline, not a target), on bounded
    samples of the same workload, in the units the GPU kernels are timed in: c (the line's value),
    F on sampled shell pairs, one matvec on sampled rows, g_surf on sampled points, dense Cholesky
    solves of the water and of one 64-conformer member, and 1-thread numbers in a child process.
    Sampled figures are scaled linearly to the full workload and labelled as extrapolated."""
    import subprocess
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    res = {}
    t = time.time()
    om = O.mol_from_system(s)
    pr = om.pairs(s.P)
    pr15 = om.pairs()
    log(f"[bench] oracle setup {time.time() - t:.1f}s, esp list {pr['a'].shape[0]} prim pairs")
    M = om.M
    rng = np.random.default_rng(s.seeds["pert"])
    order = rng.permutation(M)
    # c: sample sized to ~12 s of oracle work from a probe of one point per thread
    t = time.time()
    om.esp(s.P, kidx=np.sort(order[:threads]), pairs=pr)
    t_probe = max(time.time() - t, 1e-3)
    n_sample = int(min(M, max(threads, threads * 12.0 / t_probe)))
    kidx = np.sort(order[:n_sample])
    t = time.time()
    c_or = om.esp(s.P, kidx=kidx, pairs=pr)
    t_c = time.time() - t
    st64 = r64["state"]
    c_gpu = st64["c"].cpu().numpy()[kidx]
    res["cpu_baseline"] = {"value": sp_esp * n_sample / t_c, "unit": "shell-pair×point integrals/s",
                           "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
                           "sample": f"c_k = sum P L^k for {n_sample} seeded surface points over the full "
                                     f"Eq. 18 pair list ({t_c:.1f} s)"}
    res["c_sample_rel_err_fp64"] = float(np.abs(c_gpu - c_or).max() / np.abs(c_or).max())
    res["form_c_err"] = {form: float(np.abs(rf["state"]["c"].cpu().numpy()[kidx] - c_or).max() / np.abs(c_or).max())
                         for form, rf in forms.items()}
    units = {}
    units["c"] = {"extrapolated_full_ms": round(M / n_sample * t_c * 1e3, 1), "sample_points": n_sample,
                  "sample_s": round(t_c, 2)}
    # F on sampled shell pairs of the Eq. 15 list
    qh = st64["q"].cpu().numpy()
    sps = sorted(set(zip(pr15["a"].tolist(), pr15["b"].tolist())))
    pick = rng.choice(len(sps), size=min(len(sps), 400), replace=False)
    t = time.time()
    om.fock(qh, shell_pairs=[sps[i] for i in pick], pairs=pr15)
    t_f = time.time() - t
    n_f = len(pick)
    units["F"] = {"extrapolated_full_ms": round(sp_fock / n_f * t_f * 1e3, 1), "sample_shell_pairs": n_f,
                  "sample_s": round(t_f, 2), "shell_pair_x_point_per_s": round(n_f * M / t_f, 1)}
    # one A x on sampled rows (the oracle evaluates whole rows: M evaluations each)
    rows = np.sort(order[:min(M, 4 * threads * 64)])
    x = rng.normal(size=M)
    t = time.time()
    om.matvec(x, kidx=rows)
    t_m = time.time() - t
    units["matvec"] = {"extrapolated_full_ms": round(M / rows.shape[0] * t_m * 1e3, 2),
                       "sample_rows": int(rows.shape[0]), "sample_s": round(t_m, 3)}
    # g_surf on sampled points (c term over the Eq. 18 list, the A and B terms of each point)
    kg = np.sort(order[:max(threads, 2 * threads)])
    t = time.time()
    om.grad_surface_points(s.P, qh, kg, pairs=pr)
    t_g = time.time() - t
    units["g_surf"] = {"extrapolated_full_ms": round(M / kg.shape[0] * t_g * 1e3, 1),
                       "sample_points": int(kg.shape[0]), "sample_s": round(t_g, 2)}
    # dense solves (Cholesky of A, Eq. 1) at the water and at one member of the 64 conformers
    from synth import inputs as I
    for name, sysobj in (("water", I.water_tiny()), ("conformer0", I.conformer(0))):
        omx = O.mol_from_system(sysobj)
        t = time.time()
        v = omx.bz() + (omx.esp(sysobj.P) if name == "water" else 0.0)
        A = omx.amat()
        omx.solve_dense(v, A)
        units[f"dense_solve_{name}"] = {"ms": round((time.time() - t) * 1e3, 2), "M": int(omx.M),
                                        "note": "A built and Cholesky-solved" +
                                                ("" if name == "water" else "; v = Bz only")}
    res["cpu_baseline"]["units"] = units
    # 1-thread numbers in a child process (OpenMP and BLAS read their thread counts at start)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--workload", "oracle1t"], env=env,
                           capture_output=True, text=True, timeout=300)
        res["cpu_baseline"]["one_thread"] = json.loads(r.stdout.strip().splitlines()[-1])
    except Exception as e:  # reported, not fatal: the baseline is context only
        res["cpu_baseline"]["one_thread"] = {"error": str(e)[:200]}
    return res


def bench_nearfar(args):
    """Share of (primitive pair, point) evaluations in the near field (T = p z^2/(p + z^2) r^2 below
    40, the FP64 Boys-table range) per class, for the Eq. 18 and Eq. 15 lists of the 600-atom
    protein, counted over a seeded sample of surface points (all pairs each).  The far field is the
    asymptotic branch of the integral kernels.  A wave of 64 lanes takes the near branch when any
    lane needs it, so for the Eq. 18 list the share of wave evaluations that do is reported too:
    pair side (64 pairs x one sampled point) with the pairs in list order and in the kernels' order
    (exponent octave, then a Morton curve of the product centre), point side (64 points x one pair,
    48 sampled point waves) with the points in surface order and in the kernels' Morton order."""
    import numpy as np
    import torch

    from paper_1505_07851_amd import Context, Molecule
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    s = I.protein_single_solve()
    ctx = Context()
    mol = Molecule.from_system(ctx, s)
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    mol.esp(P)
    sf = mol.surface()
    rng = np.random.default_rng(s.seeds["pert"])
    kidx = torch.tensor(np.sort(rng.choice(mol.M, min(mol.M, args.nearfar_points), replace=False)), device="cuda")
    r = sf["r"][kidx]
    z2 = sf["zeta"][kidx] ** 2
    b = s.basis
    exps = torch.tensor(b.prim_exp, dtype=torch.float64, device="cuda")
    soff = torch.tensor(b.shell_off, dtype=torch.int64, device="cuda")
    satom = torch.tensor(b.shell_atom, dtype=torch.int64, device="cuda")
    xyz = torch.tensor(s.xyz, dtype=torch.float64, device="cuda")
    names = ["ss", "sp", "sd", "pp", "pd", "dd"]
    out = {"workload": "nearfar_protein600", "sample_points": int(kidx.numel()), "M": mol.M, "T_far": 40.0}

    def morton(g, bits):
        code = torch.zeros(g.shape[0], dtype=torch.int64, device="cuda")
        for bit in range(bits):
            for ax in range(3):
                code |= ((g[:, ax] >> bit) & 1) << (3 * bit + ax)
        return code

    def near_of(Pc, p, rr, zz):
        d2 = ((Pc[:, None, :] - rr[None, :, :]) ** 2).sum(-1)
        return p[:, None] * zz[None, :] / (p[:, None] + zz[None, :]) * d2 < 40.0

    def pair_wave_share(Pc, p):
        n = Pc.shape[0]
        nw = (n + 63) // 64
        hit = 0
        for k0 in range(0, r.shape[0], 64):
            nr = near_of(Pc, p, r[k0:k0 + 64], z2[k0:k0 + 64])
            nr = torch.cat([nr, torch.zeros(nw * 64 - n, nr.shape[1], dtype=torch.bool, device="cuda")])
            hit += int(nr.view(nw, 64, -1).any(1).sum().item())
        return hit / (nw * r.shape[0])

    # the kernels' orders (the same keys as the library's device sorts)
    lo = xyz.min(0).values
    ext = max(float((xyz.max(0).values - lo).max()), 1.0)
    rad = torch.tensor(s.radius, dtype=torch.float64, device="cuda")
    plo = lo - (2.0 * float(rad.max()) + 1.0)
    pext = ext + 2.0 * (2.0 * float(rad.max()) + 1.0)
    rall, zall = sf["r"], sf["zeta"] ** 2
    gp = ((rall - plo) * (1023.999 / pext)).long().clamp(0, 1023)
    porder = torch.argsort(morton(gp, 10), stable=True)
    wsel = np.sort(rng.choice(mol.M // 64, min(48, mol.M // 64), replace=False))

    def point_wave_share(Pc, p, order):
        hit = 0
        for w in wsel:
            kk = order[int(w) * 64:int(w) * 64 + 64]
            hit += int(near_of(Pc, p, rall[kk], zall[kk]).any(1).sum().item())
        return hit / (Pc.shape[0] * len(wsel))

    for which, label in ((1, "eq18_list"), (0, "eq15_list")):
        pl = mol.pair_list(which)
        cls = torch.tensor(pl["cls"], device="cuda")
        a = torch.tensor(pl["a"], dtype=torch.int64, device="cuda")
        bb = torch.tensor(pl["b"], dtype=torch.int64, device="cuda")
        ea = exps[soff[a] + torch.tensor(pl["i"], dtype=torch.int64, device="cuda")]
        eb = exps[soff[bb] + torch.tensor(pl["j"], dtype=torch.int64, device="cuda")]
        p = ea + eb
        Pc = (ea[:, None] * xyz[satom[a]] + eb[:, None] * xyz[satom[bb]]) / p[:, None]
        res = {}
        for c in range(6):
            sel = cls == c
            n = int(sel.sum().item())
            if not n:
                continue
            near = 0
            for k0 in range(0, r.shape[0], 64):
                near += int(near_of(Pc[sel], p[sel], r[k0:k0 + 64], z2[k0:k0 + 64]).sum().item())
            res[names[c]] = {"prim_pairs": n, "near_fraction": round(near / (n * r.shape[0]), 5)}
            if which == 1:
                Pcs, ps = Pc[sel], p[sel]
                g = ((Pcs - lo) * (255.999 / ext)).long().clamp(0, 255)
                octv = (torch.floor(torch.log2(ps)).long() + 2).clamp(0, 15)
                o = torch.argsort((octv << 24) | morton(g, 8), stable=True)
                res[names[c]].update({
                    "pair_side_wave_near_list_order": round(pair_wave_share(Pcs, ps), 4),
                    "pair_side_wave_near_kernel_order": round(pair_wave_share(Pcs[o], ps[o]), 4),
                    "point_side_wave_near_surface_order": round(point_wave_share(Pcs, ps, torch.arange(
                        mol.M, device="cuda")), 4),
                    "point_side_wave_near_kernel_order": round(point_wave_share(Pcs, ps, porder), 4)})
            log(f"[bench] nearfar {label} {names[c]}: {res[names[c]]}")
        out[label] = res
    print(json.dumps(out))


def bench_rbj_blocks(args):
    """Randomized block-Jacobi block size (Sec. 4b-ii).  600-atom solute (default): for block sizes
    100 ... 1024 and twelve partition seeds each, the solve of a benchmark step.  As in a step, the
    geometry update starts the partition on a host thread, c is evaluated meanwhile, and the solve
    (FP64, from q = 0 to 1e-8) then fills and inverts the blocks on the GPU.  With --scf-system
    protein2000 (M ~ 150k): block sizes 100 ... 1024 and --seeds partition seeds each, one FP64
    solve from q = 0 to 1e-8 of the same right-hand side per seed, the partition not overlapped.
    Reported per size: PCG iterations (each seed's, mean, spread), solve ms and setup ms."""
    import numpy as np
    import torch

    from paper_1505_07851_amd import Context, Molecule
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    big = args.scf_system == "protein2000"
    s = I.linear_solve_stress() if big else I.protein_single_solve()
    mol = Molecule.from_system(Context(), s)
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    n_seeds = args.seeds if big else 12
    blocks = (100, 256, 512, 768, 1024) if big else (100, 192, 256, 320, 384, 512, 768, 1024)
    if big:
        c, bz = mol.esp(P)
        v = bz + c
    sizes = {}
    for blk in blocks:
        rows = []
        for k in range(n_seeds):
            seed = s.seeds["rbj"] + k
            if big:
                _, info = mol.solve(v, precond="rbj", block=blk, seed=seed, tol=args.tol)
            else:
                c, bz = mol.esp(P)
                mol.solve(bz + c, precond="rbj", block=blk, seed=seed, tol=args.tol)  # last partition = this one
                mol.update_geometry(s.xyz)  # starts the partition for it on a host thread
                c, bz = mol.esp(P)
                _, info = mol.solve(bz + c, precond="rbj", block=blk, seed=seed, tol=args.tol)
            torch.cuda.synchronize()
            rows.append(info)
        it = [i["iters"] for i in rows]
        solve = [i["solve_ms"] for i in rows]
        setup = [i["setup_ms"] for i in rows]
        sizes[str(blk)] = {"iters": it, "iters_mean": float(np.mean(it)), "iters_std": float(np.std(it)),
                           "iters_min": int(np.min(it)), "iters_max": int(np.max(it)),
                           "solve_ms_mean": round(float(np.mean(solve)), 3),
                           "setup_ms_mean": round(float(np.mean(setup)), 3),
                           "solve_plus_setup_ms_mean": round(float(np.mean(solve) + np.mean(setup)), 3)}
        log(f"[bench] rbj block {blk}: {sizes[str(blk)]}")
    best = min(sizes, key=lambda b: sizes[b]["solve_plus_setup_ms_mean"])
    label = "a cold solve" if big else "a benchmark step"
    out = {"metric": f"PCG solve + setup ms of {label} against the RBJ block size ({n_seeds} partition seeds each)",
           "value": sizes[best]["solve_plus_setup_ms_mean"], "unit": "ms", "n_gpus": 1, "steps": n_seeds,
           "warmup": 0, "ms_per_step": sizes[best]["solve_plus_setup_ms_mean"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": ("protein2000" if big else "protein600") + "_631gs_rbj_blocks", "atoms": s.n_atoms,
                      "surface_points": mol.M, "tol": args.tol, "first_seed": s.seeds["rbj"]},
           "block_sizes": sizes, "fastest_block": int(best)}
    print(json.dumps(out))


def bench_oracle1t(args):
    """1-thread oracle figures (run by oracle_baseline in a child process): the whole water case
    (Bz, c, A, Cholesky, energy) and c on 64 points of one member of the 64 conformers."""
    import numpy as np
    from oracle import oracle as O
    from synth import inputs as I
    out = {"threads": int(os.environ.get("OMP_NUM_THREADS", "0"))}
    s = I.water_tiny()
    om = O.mol_from_system(s)
    t = time.time()
    O.full_solution(om, s.P)
    out["water_full_path_ms"] = round((time.time() - t) * 1e3, 2)
    s = I.conformer(0)
    om = O.mol_from_system(s)
    pr = om.pairs(s.P)
    kidx = np.sort(np.random.default_rng(7).permutation(om.M)[:64])
    t = time.time()
    om.esp(s.P, kidx=kidx, pairs=pr)
    dt = time.time() - t
    n_sp = len(set(zip(pr["a"].tolist(), pr["b"].tolist())))
    out["conformer0_c"] = {"M": int(om.M), "sample_points": 64, "sample_s": round(dt, 2),
                           "extrapolated_full_ms": round(om.M / 64 * dt * 1e3, 1),
                           "shell_pair_x_point_per_s": round(n_sp * 64 / dt, 1)}
    print(json.dumps(out))


# translation units of the kernels whose HBM counters are committed (profiles/traffic_protein600.txt)
TRAFFIC_SOURCES = {"solver": ("pcm_internal.h", "solve.hip"),
                   "integrals": ("pcm_internal.h", "low_order.h", "contract.h", "integrals.hip", "grad.hip")}


def source_digest(kernel="matvec_f64"):
    """Digest of the sources of a counted kernel (its translation units and the shared headers):
    counter figures are reported only for the code they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1505_07851_amd", "csrc")
    for name in TRAFFIC_SOURCES["solver" if kernel.startswith(("matvec", "rbj")) else "integrals"]:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (profiles/), scaled by
    the plain-copy calibration recorded there; None if absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", "traffic_protein600.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("#") or "=" not in line:
            continue
        k, v = line.split("=", 1)
        vals[k.strip()] = v.strip()
    if vals.get(f"{kernel}.source_digest") != source_digest(kernel):
        return None
    key = f"{kernel}.hbm_bytes_per_launch"
    return float(vals[key]) if key in vals else None


def bench_copy(args):
    """Plain device-to-device copy of 1 GiB (read 1 GiB, write 1 GiB), timed; under rocprofv3
    --pmc its FETCH_SIZE / WRITE_SIZE give the counter-to-byte factor."""
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = 1 << 27  # doubles
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    print(json.dumps({"workload": "copy", "bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n,
                      "ms_per_copy": round(dt * 1e3, 4), "GBps": round(16 * n / dt / 1e9, 1)}))


def bench_stress(args):
    import numpy as np
    import torch

    from paper_1505_07851_amd import Context, Molecule, dynamic_threshold
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t = time.time()
    s = I.linear_solve_stress()
    log(f"[bench] inputs in {time.time() - t:.1f}s: {s.n_atoms} atoms, nbf {s.basis.nbf}")
    nbf = s.basis.nbf
    n_out = 15
    # thresholds from Eq. 21 (pcm_dynamic_threshold) fed the synthetic DIIS error sequence of the
    # schedule, which tightens geometrically from 1e-3 to 1e-7
    diis_err, target = I.stress_outer_errors(n_out)
    deltas = [dynamic_threshold(e) for e in diis_err]
    assert all(abs(d / t - 1.0) < 1e-9 for d, t in zip(deltas, target)), (deltas, target)
    # the outer densities P_t = 2 C_t C_t^T, C_t = orth(C_{t-1} + e_t G_t) (block-diagonal C)
    t = time.time()
    seq = I.stress_density_sequence(s, n_out)
    log(f"[bench] {n_out} perturbed occupied blocks in {time.time() - t:.1f}s")
    runs = {}
    ctx = Context(precision="fp64")  # integrals in FP64: this workload measures the solver
    t = time.time()
    mol = Molecule.from_system(ctx, s)
    torch.cuda.synchronize()
    log(f"[bench] surface + lists in {time.time() - t:.1f}s, M = {mol.M}")
    P = torch.zeros((nbf, nbf), dtype=torch.float64, device="cuda")

    def density_on_gpu(windows):
        # input synthesis (untimed): the block-diagonal P_t assembled in HBM from its windows
        P.zero_()
        for s0, C in windows:
            Cg = torch.tensor(C, dtype=torch.float64, device="cuda")
            B = 2.0 * torch.mm(Cg, Cg.t().contiguous())
            P[s0:s0 + C.shape[0], s0:s0 + C.shape[0]] = 0.5 * (B + B.t())

    vs, esp_ms, esp_pairs = [], [], []
    # untimed c with the unperturbed and the first perturbed density first: chunk shapes are tuned
    # on first use of a (class, size bucket), and the density-screened class sizes can cross a bucket
    P.copy_(torch.tensor(s.P, dtype=torch.float64))
    c_t, bz = mol.esp(P)
    density_on_gpu(seq[0])
    mol.esp(P, want_bz=False)
    torch.cuda.synchronize()
    for t_ in range(n_out):
        density_on_gpu(seq[t_])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c_t = mol.esp(P, want_bz=False)
        torch.cuda.synchronize()
        esp_ms.append(round((time.perf_counter() - t0) * 1e3, 1))
        esp_pairs.append(int(sum(mol.sizes()["pairs_esp"])))
        vs.append(bz + c_t)
    del P
    torch.cuda.synchronize()
    log(f"[bench] c_t = L P_t for the {n_out} outer densities: {esp_ms} ms")
    for prec in ("fp64", "mixed"):
        for pc, blk, cap in (("rbj", 1024, 10000), ("none", 0, args.max_iter_none)):
            q = None
            per = []
            t0 = time.perf_counter()
            for t_, (v, d) in enumerate(zip(vs, deltas)):
                q, info = mol.solve(v, precond=pc, block=max(blk, 1), seed=s.seeds["rbj"], tol=d, q0=q,
                                    max_iter=cap, precision=prec, raise_noconv=False)
                per.append(info)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            key = f"{prec}_{pc}{blk if blk else ''}"
            runs[key] = {"wall_ms": round(wall, 1), "solve_ms": round(sum(i["solve_ms"] for i in per), 1),
                         "setup_ms": round(sum(i["setup_ms"] for i in per), 1),
                         "iters": [i["iters"] for i in per], "converged": sum(i["status"] == 0 for i in per),
                         "final_resid": per[-1]["resid"], "final_energy": per[-1]["energy"],
                         "energies": [i["energy"] for i in per]}
            log(f"[bench] {key}: {wall:.0f} ms, iters {runs[key]['iters']}, converged {runs[key]['converged']}/15")
    ref = runs["fp64_rbj1024"]["energies"]
    for k, r in runs.items():
        r["E_abs_err_vs_fp64_rbj_max"] = max(abs(a - b) for a, b in zip(r.pop("energies"), ref))
    # one profiled cold solve of the last outer system per precision (untimed above): per-kernel
    # launch means, the product's rate on the 14-flop model and the RBJ apply's bandwidth, whose
    # algorithmic bytes are the inverse blocks (8 sum l_b^2) plus the residual read and z written
    prof_solve = {}
    for prec in ("fp64", "mixed"):
        ctx.profile(True)
        _, info = mol.solve(vs[-1], precond="rbj", block=1024, seed=s.seeds["rbj"], tol=deltas[-1], max_iter=10000,
                            precision=prec, raise_noconv=False)
        prof = ctx.profile_read()
        ctx.profile(False)
        ent = {"iters": info["iters"], "kernels": {}}
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
            if v["launches"] == 0 or v["ms"] <= 0:
                continue
            e = {"ms_per_launch": round(v["ms"] / v["launches"], 4), "launches": v["launches"]}
            if k.startswith("matvec"):
                e["tflops"] = round(14.0 * v["work"] / (v["ms"] * 1e-3) / 1e12, 3)
                e["frac"] = round(e["tflops"] / PEAK_F64_TFLOPS, 4)
            if k == "rbj_apply":
                nbytes = 8.0 * v["work"] + 2 * 8.0 * mol.M * v["launches"]
                e["bytes_per_launch"] = nbytes / v["launches"]
                e["GB_per_s"] = round(nbytes / (v["ms"] * 1e-3) / 1e9, 1)
                e["frac_hbm"] = round(e["GB_per_s"] / 8000.0, 4)
            ent["kernels"][k] = e
        prof_solve[prec] = ent
        rb = ent["kernels"].get("rbj_apply", {})
        log(f"[bench] profiled {prec} solve: {info['iters']} iters, rbj_apply {rb.get('ms_per_launch')} ms "
            f"= {rb.get('GB_per_s')} GB/s")
    out = {"metric": "PCG solve ms over 15 outer iterations at the Eq. 21 thresholds (1e-3 -> 1e-7)",
           "value": runs["mixed_rbj1024"]["wall_ms"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": runs["mixed_rbj1024"]["wall_ms"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64/f32-matvec", "data": "synthetic",
           "config": {"workload": "protein2000_631gs_stress", "atoms": s.n_atoms, "nbf": nbf, "surface_points": mol.M,
                      "outer_iterations": n_out, "deltas": deltas, "rbj_block": 1024,
                      "max_iter_unpreconditioned": args.max_iter_none},
           "esp_ms_per_outer": esp_ms, "esp_prim_pairs_per_outer": esp_pairs,
           "esp_ms_total": round(sum(esp_ms), 1), "runs": runs, "profiled_solve": prof_solve}
    print(json.dumps(out))


def bench_conformers(args):
    import numpy as np
    import torch

    from paper_1505_07851_amd import Batch, Context, Molecule
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n_conf = 64
    t = time.time()
    systems = [I.conformer(j) for j in range(n_conf)]
    log(f"[bench] {n_conf} conformers generated in {time.time() - t:.1f}s")
    Ps = [torch.tensor(s.P, dtype=torch.float64, device="cuda") for s in systems]
    kw = dict(precond="rbj", block=args.block, seed=7, tol=args.tol, max_iter=10000)

    def setup(prec):
        ctx = Context(precision=prec)
        mols = [Molecule.from_system(ctx, s) for s in systems]
        return ctx, mols

    def seq_step(mols):
        out = []
        for m, P in zip(mols, Ps):
            c, bz = m.esp(P)
            q, info = m.solve(bz + c, **kw)
            F = m.fock(q)
            out.append((q, info, F))
        return out

    def batch_step(b, prec):
        cs, bzs = b.esp(Ps)
        qs, infos = b.solve([bz + c for c, bz in zip(cs, bzs)], precision=prec, **kw)
        Fs = b.fock(qs)
        return list(zip(qs, infos, Fs))

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps * 1e3, res

    ctx64, mols64 = setup("fp64")
    M = [m.M for m in mols64]
    log(f"[bench] surfaces built: M min {min(M)} max {max(M)} mean {np.mean(M):.0f}, nbf {mols64[0].nbf}")
    ms_seq, r_seq = timed(lambda: seq_step(mols64))
    log(f"[bench] sequential FP64: {ms_seq:.1f} ms per step")
    b64 = Batch(ctx64, mols64)
    ms_b64, r_b64 = timed(lambda: batch_step(b64, "fp64"))
    log(f"[bench] batched FP64: {ms_b64:.1f} ms per step")
    # Eq. 14 gradient of every conformer at its solved q: 64 pcm_grad calls against one
    # pcm_grad_batched (not part of the step above)
    qs64 = [r[0] for r in r_b64]
    ms_gseq, g_seq = timed(lambda: [m.grad(P, q) for m, P, q in zip(mols64, Ps, qs64)])
    ms_gb, g_b = timed(lambda: b64.grad(Ps, qs64))
    g_bitwise = all(torch.equal(a[0], c[0]) and torch.equal(a[1], c[1]) for a, c in zip(g_seq, g_b))
    log(f"[bench] gradient FP64: sequential {ms_gseq:.1f} ms, batched {ms_gb:.1f} ms, bitwise equal {g_bitwise}")
    # the same pass captured as one hipGraph (c, Bz, FP64 PCG with an iteration budget, E, F); the
    # budget is the largest count of the eager batched solve plus a margin
    it_b = [r[1]["iters"] for r in r_b64]
    budget = int(max(it_b) * 1.25) + 8
    t = time.time()
    g = b64.capture(Ps, precond="rbj", block=args.block, seed=7, tol=args.tol, max_iter=budget)
    t_cap = time.time() - t

    def graph_step():
        for F in g.Fs:
            F.zero_()
        g.replay()
        return g

    ms_g, _ = timed(graph_step)
    ginfo, nodes = g.info()
    r_g = [(q, {"iters": d["iters"], "energy": d["energy"]}, F) for q, d, F in zip(g.qs, ginfo, g.Fs)]
    log(f"[bench] captured graph ({nodes} nodes, budget {budget}, capture {t_cap:.1f}s): {ms_g:.1f} ms per step")
    ctxm, molsm = setup("mixed")
    bm = Batch(ctxm, molsm)
    ms_bm, r_bm = timed(lambda: batch_step(bm, "mixed"))
    log(f"[bench] batched mixed: {ms_bm:.1f} ms per step")
    # per-pair dynamic precision of the integrals (the equal-accuracy form) with the FP32-product solve
    ctxd, molsd = setup("dynamic")
    bd = Batch(ctxd, molsd)
    ms_bd, r_bd = timed(lambda: batch_step(bd, "mixed"))
    log(f"[bench] batched dynamic: {ms_bd:.1f} ms per step")

    def errs(res):
        dE = max(abs(r[1]["energy"] - s[1]["energy"]) for r, s in zip(res, r_seq))
        dq = max((r[0] - s[0]).abs().max().item() / s[0].abs().max().item() for r, s in zip(res, r_seq))
        dF = max((r[2] - s[2]).abs().max().item() / s[2].abs().max().item() for r, s in zip(res, r_seq))
        bitwise = all(torch.equal(r[0], s[0]) and torch.equal(r[2], s[2]) for r, s in zip(res, r_seq))
        return {"E_abs_max": dE, "q_rel_max": dq, "F_rel_max": dF, "bitwise_equal": bitwise}

    iters = [r[1]["iters"] for r in r_seq]
    out = {"metric": "conformers/s (64-conformer batch: c = L P, PCG solve, energy, F += L^T q)",
           "value": n_conf / (ms_b64 * 1e-3), "unit": "conformers/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_b64, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "conformers64_peptide150_631g", "conformers": n_conf, "atoms": 150,
                      "nbf": mols64[0].nbf, "M_min": min(M), "M_max": max(M), "M_mean": round(float(np.mean(M)), 1),
                      "precond": f"rbj{args.block}", "tol": args.tol},
           "sequential_fp64": {"ms_per_step": round(ms_seq, 3), "ms_per_conformer": round(ms_seq / n_conf, 3),
                               "pcg_iters_min": min(iters), "pcg_iters_max": max(iters)},
           "batched_fp64": {"ms_per_step": round(ms_b64, 3), "ms_per_conformer": round(ms_b64 / n_conf, 3),
                            "speedup_vs_sequential": round(ms_seq / ms_b64, 3), "err_vs_sequential": errs(r_b64)},
           "batched_mixed": {"ms_per_step": round(ms_bm, 3), "ms_per_conformer": round(ms_bm / n_conf, 3),
                             "speedup_vs_sequential": round(ms_seq / ms_bm, 3), "err_vs_sequential": errs(r_bm)},
           "batched_dynamic": {"ms_per_step": round(ms_bd, 3), "ms_per_conformer": round(ms_bd / n_conf, 3),
                               "speedup_vs_sequential": round(ms_seq / ms_bd, 3), "err_vs_sequential": errs(r_bd)},
           "gradient_fp64": {"sequential_ms": round(ms_gseq, 3), "batched_ms": round(ms_gb, 3),
                             "speedup": round(ms_gseq / ms_gb, 3), "bitwise_equal": g_bitwise},
           "graph_fp64": {"ms_per_step": round(ms_g, 3), "ms_per_conformer": round(ms_g / n_conf, 3),
                          "speedup_vs_sequential": round(ms_seq / ms_g, 3),
                          "speedup_vs_batched": round(ms_b64 / ms_g, 3), "graph_nodes": nodes,
                          "iteration_budget": budget, "capture_s": round(t_cap, 2),
                          "all_converged": all(d["converged"] for d in ginfo),
                          "err_vs_sequential": errs(r_g)}}
    g.close()
    print(json.dumps(out))


def scf_trajectory(n_steps=16, e_first=1e-1, e_last=1e-6):
    """Synthetic SCF: DIIS errors falling geometrically from e_first to e_last; the density
    of step t is P* + (e_t / e_first) D, i.e. its error is proportional to the DIIS error."""
    return [e_first * (e_last / e_first) ** (t / (n_steps - 1)) for t in range(n_steps)]


def bench_scf_policies(args):
    """Sec. 4b-i/4b-ii solver policies over a 16-step synthetic SCF on the 600-atom solute
    (default) or the 2,000-atom one (--scf-system protein2000; no unpreconditioned run there,
    Jacobi capped at 2,000 products per solve, RBJ blocks of 100 and 1,024).

    Step t solves A q = -f (Bz + L P_t) warm-started from the previous step's q, at the
    threshold the policy gives from the previous step's DIIS error.  Reported per run: CG
    matrix-vector products per step and in total, wall time of the solves (preconditioner
    setup included), and the Eq. 13 energy error against a 1e-10 solve at the same density,
    also as a ratio to 1e-3 times the previous step's DIIS error (the target of Sec. 4b-i)."""
    import numpy as np
    import torch

    from paper_1505_07851_amd import Context, Molecule, ThresholdPolicy, octree_partition
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    big = args.scf_system == "protein2000"
    s = I.linear_solve_stress() if big else I.protein_single_solve()
    nbf = s.basis.nbf
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    n_occ = min(int(s.Z.sum()) // 2, nbf)
    D = (I.density_matrix_blocked if big else I.density_matrix)(nbf, n_occ, s.seeds["pert"]) - s.P
    D = torch.tensor(D, dtype=torch.float64, device="cuda")
    ctx = Context(precision="fp64")
    mol = Molecule.from_system(ctx, s)
    c0, bz = mol.esp(P)
    cD = mol.esp(D, want_bz=False)
    errs = scf_trajectory()
    vs = [bz + c0 + (e / errs[0]) * cD for e in errs]
    torch.cuda.synchronize()
    log(f"[bench] scf_policies: M = {mol.M}, nbf = {nbf}, trajectory ready in {time.time() - t0:.1f}s")
    E_ref = []
    ref_block, ref_tol = (1024, 1e-9) if big else (100, 1e-10)
    for v in vs:
        _, info = mol.solve(v, precond="rbj", block=ref_block, seed=s.seeds["rbj"], tol=ref_tol)
        E_ref.append(info["energy"])
    log(f"[bench] reference energies at {ref_tol:g} done in {time.time() - t0:.1f}s")

    def run(policy, precond, block=100, seed=0, max_iter=10000):
        pol = ThresholdPolicy(policy, delta=1e-6, scale=1e4, switch_at=1e-3)
        q, iters, dE, deltas, conv = None, [], [], [], 0
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k, v in enumerate(vs):
            d = pol(errs[k - 1] if k else None)
            q, info = mol.solve(v, precond=precond, block=block, seed=seed, tol=d, q0=q, max_iter=max_iter,
                                raise_noconv=False)
            iters.append(info["iters"])
            deltas.append(d)
            conv += info["status"] == 0
            dE.append(abs(info["energy"] - E_ref[k]))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) * 1e3
        # Sec. 4b-i aims the CG error of step t at 1e-3 times the DIIS error of step t-1
        return {"iters": iters, "total_iters": sum(iters), "wall_ms": round(wall, 1), "converged": conv,
                "deltas": deltas, "E_err": dE,
                "E_err_over_target_max": max(dE[k] / (1e-3 * errs[k - 1]) for k in range(1, len(dE))),
                "E_err_final": dE[-1]}

    runs = {}
    if big:
        plan = [("fixed", "jacobi", 0), ("fixed", "rbj", 100), ("fixed", "rbj", 1024), ("fixed", "octree", 800),
                ("two_delta", "rbj", 100), ("dynamic", "jacobi", 0), ("dynamic", "rbj", 100), ("dynamic", "rbj", 1024),
                ("dynamic", "octree", 800)]
        seed_blocks = (100, 1024)
    else:
        plan = [("fixed", "none", 0), ("fixed", "jacobi", 0), ("fixed", "rbj", 100), ("fixed", "octree", 800),
                ("two_delta", "jacobi", 0), ("two_delta", "rbj", 100), ("dynamic", "jacobi", 0), ("dynamic", "rbj", 100),
                ("dynamic", "octree", 800)]
        seed_blocks = (100, 800)
    for policy, precond, block in plan:
        key = f"{policy}+{precond}{block if block else ''}"
        cap = 3000 if precond == "none" else (2000 if big and precond == "jacobi" else 10000)
        runs[key] = run(policy, precond, max(block, 1), s.seeds["rbj"], cap)
        log(f"[bench] {key}: total {runs[key]['total_iters']} matvecs, {runs[key]['wall_ms']:.0f} ms, "
            f"per step {runs[key]['iters']}")
    # randomized partition over seeds against the deterministic octree (fixed delta)
    seeds = {}
    for block in seed_blocks:
        tot = [run("fixed", "rbj", block, 1000 + j)["total_iters"] for j in range(args.seeds)]
        seeds[f"rbj{block}"] = {"mean": float(np.mean(tot)), "std": float(np.std(tot)), "min": int(min(tot)),
                                "max": int(max(tot)), "n_seeds": args.seeds}
        log(f"[bench] fixed+rbj{block} over {args.seeds} seeds: {seeds[f'rbj{block}']}")
    r = mol.surface()["r"].cpu().numpy()
    _, off = octree_partition(r, 800)
    sizes = np.diff(off)
    out = {"metric": "CG matrix-vector products over a 16-step synthetic SCF (DIIS error 1e-1 -> 1e-6)",
           "value": runs["dynamic+rbj100"]["total_iters"], "unit": "matvecs", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": runs["dynamic+rbj100"]["wall_ms"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{s.name}_scf16", "atoms": s.n_atoms, "nbf": nbf, "surface_points": mol.M,
                      "diis_errors": errs, "reference_tol": ref_tol, "fixed_delta": 1e-6,
                      "two_delta": {"delta2": 1e-6, "s": 1e4, "switch_at": 1e-3}},
           "runs": runs, "rbj_seeds": seeds,
           "octree800_blocks": {"n": int(sizes.size), "mean": float(sizes.mean()), "min": int(sizes.min()),
                                "max": int(sizes.max())}}
    print(json.dumps(out))


def bench_eq21_fit(args):
    """Sec. 4b-i, Eq. 21 re-derived on synthetic solutes: six sizes, each at its generated
    geometry and with seeded displacements (0.1 A rms), 6-31G-shaped basis.  The first solve
    (q from zero) at thresholds 10^-9 .. 1 is compared with a 1e-10 solve: the error of the
    Eq. 13 energy and the largest element of the Fock-matrix error sum_k dq_k L^k.  Both are
    averaged over the twelve structures and fitted with a power law err = a delta^b."""
    import numpy as np
    import torch

    from paper_1505_07851_amd import Context, Molecule
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    deltas = [10.0 ** (-9 + 0.5 * i) for i in range(19)]
    sizes = (16, 24, 36, 50, 70, 96)
    ctx = Context(precision="fp64")
    e_rows, f_rows, meta = [], [], []
    for n in sizes:
        base = I.small_protein(n, 110, seed=300 + n, polarized=False)
        for distorted in (False, True):
            s = base
            if distorted:
                rng = np.random.default_rng(700 + n)
                shift = rng.normal(scale=0.1 / 0.52917721092 / np.sqrt(3), size=base.xyz.shape)
                s = dataclasses.replace(base, xyz=base.xyz + shift)
            mol = Molecule.from_system(ctx, s)
            P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
            c, bz = mol.esp(P)
            v = bz + c
            q_ref, info = mol.solve(v, precond="jacobi", tol=1e-10)
            E_ref = info["energy"]
            er, fr = [], []
            for d in deltas:
                q, info = mol.solve(v, precond="jacobi", tol=d)
                er.append(abs(info["energy"] - E_ref))
                fr.append(mol.fock(q - q_ref).abs().max().item())
            e_rows.append(er)
            f_rows.append(fr)
            meta.append({"atoms": n, "distorted": distorted, "M": mol.M, "E": E_ref})
            log(f"[bench] eq21: {n} atoms{' distorted' if distorted else ''}, M = {mol.M}")
            mol.close()
    e_mean = np.mean(e_rows, axis=0)
    f_mean = np.mean(f_rows, axis=0)

    def fit(y):
        keep = [i for i, v in enumerate(y) if v > 1e-13]
        b, la = np.polyfit(np.log10(np.array(deltas)[keep]), np.log10(np.array(y)[keep]), 1)
        return {"a": float(10.0 ** la), "b": float(b), "points": len(keep)}

    bound = [0.01 * d ** 1.07 for d in deltas]
    out = {"metric": "power-law fit of the energy error against the CG threshold (Eq. 21 re-derived)",
           "value": fit(e_mean)["b"], "unit": "exponent b", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": None, "higher_is_better": None, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "six_solutes_x2_geometries_631g", "structures": meta, "deltas": deltas,
                      "precond": "jacobi", "reference_delta": 1e-10},
           "energy_error": {"mean": e_mean.tolist(), "fit": fit(e_mean),
                            "below_eq21_all": bool(np.all(np.max(e_rows, axis=0) <= bound))},
           "fock_error_max": {"mean": f_mean.tolist(), "fit": fit(f_mean)},
           "eq21": {"a": 0.01, "b": 1.07}}
    print(json.dumps(out))


def bench_shard(args):
    """Sec. 5 / Table 3 scale-out, one GPU's part: the FP64 product of the 2,000-atom solute
    (M ~ 150k) computed whole and as the 8 shares of an 8-GPU run (tile pairs dealt out round
    robin), each share timed on this GPU at its real shape; the shares must add up to A x."""
    import numpy as np
    import torch

    from paper_1505_07851_amd import Context, Molecule
    from synth import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    s = I.linear_solve_stress()
    ctx = Context(precision="fp64")
    mol = Molecule.from_system(ctx, s)
    rng = np.random.default_rng(s.seeds["pert"])
    x = torch.tensor(rng.normal(size=mol.M), dtype=torch.float64, device="cuda")
    n_ranks = 8
    mol.matvec_share(x, 0, 1)
    mol.matvec_share(x, 0, n_ranks)
    torch.cuda.synchronize()

    def timed_share(r, n):
        ms = []
        for _ in range(max(args.steps, 1)):
            ctx.profile(True)
            y = mol.matvec_share(x, r, n)
            prof = ctx.profile_read()
            ctx.profile(False)
            ms.append(prof["matvec_share_f64"]["ms"] if "matvec_share_f64" in prof else 0.0)
            work = prof["matvec_share_f64"]["work"] if "matvec_share_f64" in prof else 0.0
        return min(ms), work, y

    full_ms, full_pairs, y_full = timed_share(0, 1)
    shares = [timed_share(r, n_ranks) for r in range(n_ranks)]
    y_sum = sum(sh[2] for sh in shares)
    rel = ((y_sum - y_full).norm() / y_full.norm()).item()
    per = [sh[0] for sh in shares]
    log(f"[bench] shard8: full product {full_ms:.3f} ms; shares {['%.3f' % t for t in per]} ms; "
        f"sum of shares vs whole {rel:.1e}")
    flops = 14.0 * full_pairs
    rs_bytes = mol.M * 8 * (n_ranks - 1) / n_ranks
    out = {"metric": "one rank's share of the FP64 product, 8-way sharded (ms per CG iteration)",
           "value": max(per), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": max(per), "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "protein2000_631gs_matvec_shard8", "atoms": s.n_atoms, "surface_points": mol.M,
                      "ranks": n_ranks, "tile": 256},
           "whole_product_ms": full_ms, "whole_product_tflops": flops / (full_ms * 1e-3) / 1e12,
           "share_ms": per, "share_max_over_mean": max(per) / (sum(per) / len(per)),
           "speedup_whole_over_max_share": full_ms / max(per),
           "sum_of_shares_rel_err": rel,
           "reduce_scatter_bytes_per_rank_per_iteration": rs_bytes,
           "reduce_scatter_us_at_153GBps": rs_bytes / 153e9 * 1e6}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
