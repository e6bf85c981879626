"""Host-side checks of the benchmark's command line and measurement helpers (no GPU).

* ``--gpus N`` with N != 1 exits with status 2 and one JSON line saying why (the collectives of a
  multi-GPU run are not implemented), before touching a GPU;
* the flop model counts the factored kernels from their far-field code and the others (L = 4)
  from the generated Hermite recursion and the fixed per-evaluation terms; the matvec is 14 flops
  per unordered pair;
* the committed traffic summary parses, and its figure is reported only for the digest it states;
* the per-family roofline sums the model flops of a family's FP64 classes over their time.
"""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_multi_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_flop_model():
    import bench
    m = bench.flop_model()
    assert m["matvec"] == 14
    # factored kernels: the common far-field part 13 + 2N, then the contraction as written
    assert m["esp_L0"] == 13 + 0 + 2            # one FMA D_0 R^(0)
    # pair side, far-field factored sums: 12 + s_0, s_1, then S_0 and three S_1i by FMA
    assert m["fock_v_L1"] == 12 + 2 + 1 + 6
    assert m["fock_grad_v_L1"] == 12 + 3 + 1 + 6 + 1 + 3 + 12  # + S_1, three s_2 X_i, six S_2ij by FMA
    assert m["esp_grad_pts_L0"] == m["grad_pts_L0"] + 2  # the potential's FMA beside the derivative
    for fam, counts in bench.FACTORED.items():
        assert [m[f"{fam}_L{L}"] for L in range(len(counts))] == list(counts), fam
    # order-4 pair-side sums: 12 + s_0 .. s_4 + 53 (to order 3) + 53 for order 4
    assert m["fock_grad_v_L3"] == m["fock_v_L4"] == 12 + 5 + 53 + 53
    # the other L = 4 kernels form every R_tuv: table form with the generated Hermite recursion
    H = bench.hermite_flops()
    assert m["esp_L4"] == 12 + 2 * 4 + H[4] + 2 * bench.ntuv(4) + 1
    # every model grows with L
    for k in ("esp", "fock_v", "grad_pts", "grad_v", "esp_grad_pts", "fock_grad_v"):
        vals = [m[f"{k}_L{L}"] for L in range(5)]
        assert all(a < b for a, b in zip(vals, vals[1:])), k
    assert bench.kernel_flops("matvec_f32", 10.0, m) == 140.0
    assert bench.kernel_flops("esp_L2_f64", 1.0, m) == m["esp_L2"]
    assert bench.kernel_flops("fock_grad_v_L1_mix", 1.0, m) == m["fock_grad_v_L1"]


def test_traffic_summary_digest(tmp_path, monkeypatch):
    import bench
    path = os.path.join(ROOT, "profiles", "traffic_protein600.txt")
    vals = dict(l.split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    vals = {k.strip(): v.strip() for k, v in vals.items()}
    kernels = [k[: -len(".hbm_bytes_per_launch")] for k in vals if k.endswith(".hbm_bytes_per_launch")]
    assert "matvec_f64" in kernels and len(kernels) >= 2
    for kern in kernels:
        assert float(vals[f"{kern}.hbm_bytes_per_launch"]) > 0
        got = bench.measured_traffic(kern)
        if vals[f"{kern}.source_digest"] == bench.source_digest(kern):
            assert got == float(vals[f"{kern}.hbm_bytes_per_launch"])
        else:
            assert got is None
    # the matvec and the integral kernels are digested over their own sources
    assert bench.source_digest("matvec_f64") != bench.source_digest("fock_grad_v_L1_f64")
    assert bench.source_digest("rbj_apply") == bench.source_digest("matvec_f64")  # both in solve.hip
    monkeypatch.setattr(bench, "source_digest", lambda kernel="matvec_f64": "0" * 16)
    assert bench.measured_traffic("matvec_f64") is None


def test_family_rooflines():
    import bench
    m = bench.flop_model()
    prof = {"esp_grad_pts_L0_f64": {"ms": 10.0, "work": 1e9, "launches": 1},
            "esp_grad_pts_L1_f64": {"ms": 10.0, "work": 1e9, "launches": 1},
            "fock_v_L0_f64": {"ms": 2.0, "work": 1e8, "launches": 1},
            "matvec_f64": {"ms": 3.0, "work": 4.5e8, "launches": 10},
            "esp_grad_pts_L0_f32": {"ms": 99.0, "work": 1.0, "launches": 1},
            "rbj_apply": {"ms": 0.5, "work": 2.5e8, "launches": 20}}
    fam = bench.family_rooflines(prof, m, 2)
    pts = (m["esp_grad_pts_L0"] + m["esp_grad_pts_L1"]) * 1e9 / 20e-3 / 1e12
    assert abs(fam["point_side"]["model_tflops"] - round(pts, 3)) < 1e-9
    assert fam["point_side"]["ms_per_step"] == 10.0  # 20 ms over 2 profiled steps; FP32 entries excluded
    assert abs(fam["matvec"]["frac"] - round(14 * 4.5e8 / 3e-3 / 1e12 / bench.PEAK_F64_TFLOPS, 4)) < 1e-12
    assert "pair_side" not in fam
    # RBJ apply: 8 bytes per inverse entry, 2e9 bytes in 0.5 ms = 4000 GB/s, half the HBM peak
    ra = fam["rbj_apply"]
    assert ra["bound"] == "hbm" and ra["GB_per_s"] == 4000.0 and ra["frac"] == 0.5
    assert ra["bytes_per_launch"] == 1e8 and ra["ms_per_step"] == 0.25

