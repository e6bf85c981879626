"""Write tests/golden/water_tiny.json from the FP64 oracle (and the seeded generators only).

Run from the repository root:  python tests/golden/make_golden.py
The stored values pin the oracle against later unintended changes; they are not
the paper's numbers (the paper prints none for a reproducible input).
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from synth import inputs as I  # noqa: E402


def main():
    s = I.water_tiny()
    om = O.mol_from_system(s)
    sol = O.full_solution(om, s.P)
    pr = om.pairs()
    pe = om.pairs(s.P)
    out = {
        "_made_by": "tests/golden/make_golden.py (oracle only)",
        "M": int(om.M), "nbf": int(om.nbf),
        "n_pairs_fock": int(pr["a"].shape[0]), "n_pairs_esp": int(pe["a"].shape[0]),
        "keep_idx_head": om.keep_idx[:20].tolist(),
        "E": sol["E"], "sum_q": float(sol["q"].sum()),
        "c_head": sol["c"][:8].tolist(), "bz_head": sol["bz"][:8].tolist(), "q_head": sol["q"][:8].tolist(),
    }
    with open(os.path.join(ROOT, "tests", "golden", "water_tiny.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
