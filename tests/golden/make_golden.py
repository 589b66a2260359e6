"""Write the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
Every value here is computed by ``oracle/`` from the seeded inputs; none comes
from the GPU path.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import seeded_inputs as S  # noqa: E402
from oracle import fock as F  # noqa: E402


def main():
    out = {}
    # ground-state energy of the L=6 workload (400-dim N=6, Sz=0 sector)
    h, B = S.workload_integrals(1)
    E, _, st = F.ed_ground(h, B, 6, 0)
    out["ed_L6_N6_seed1001"] = {"E0": float(E), "sector_dim": int(len(st))}
    # L=8 sector used by the small additive-sweep parity cases
    h, B = S.integrals(8, 8, 1008)
    E, _, st = F.ed_ground(h, B, 8, 0)
    out["ed_L8_N8_seed1008"] = {"E0": float(E), "sector_dim": int(len(st))}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ed_energies.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=2, sort_keys=True)
        f.write("\n")
    print(json.dumps(out, indent=2))


if __name__ == "__main__":
    main()
