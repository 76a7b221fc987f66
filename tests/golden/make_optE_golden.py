"""Write tests/golden/<workload>_optE.json: the CPU oracle's simplex skills and optE of the
library series of a seeded workload (E = 1..20, leave-one-out, Tp = 1, tau = 1; Sec. II-B
and Alg. 1 phase 1) -- all 1,024 series of the rate-network workload, or the 512 libraries
of the 101,729-series block.  Only the oracle and the seeded input generator are called.
The whole-matrix and full-size GPU parity tests read these files instead of spending up to
an hour of CPU time on the box.

    python tests/golden/make_optE_golden.py <workload> [processes]
"""
import hashlib
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

E_MIN, E_MAX, TAU, TP = 1, 20, 1, 1


def panel_sha256(ts) -> str:
    return hashlib.sha256(np.ascontiguousarray(ts, dtype=np.float32).tobytes()).hexdigest()


def _chunk(args):
    workload, ids = args
    ts = synth.make(workload).panel
    optE, rho, _ = O.simplex_optE(ts, ids, E_MIN, E_MAX, TAU, TP, O.MODE_LOO)
    return ids, optE, rho


def main(workload: str, procs: int) -> None:
    wl = synth.make(workload)
    ts = wl.panel
    lib = [int(v) for v in wl.lib_ids]
    chunks = [lib[a: a + 16] for a in range(0, len(lib), 16)]
    optE = {}
    rho = {}
    with ProcessPoolExecutor(max_workers=procs) as ex:
        for ids, e, r in ex.map(_chunk, [(workload, c) for c in chunks]):
            for q, sid in enumerate(ids):
                optE[sid], rho[sid] = int(e[q]), r[q]
            print(f"series {ids[0]}..{ids[-1]} done", flush=True)
    out = {
        "workload": workload,
        "panel_sha256": panel_sha256(ts),
        "E_min": E_MIN, "E_max": E_MAX, "tau": TAU, "Tp": TP, "mode": "leave-one-out",
        "series": lib,
        "optE": [optE[s] for s in lib],
        # skills rho_E [series][E - E_min] (FP64 oracle, 12 significant digits; NaN as null)
        "rho_E": [[None if np.isnan(v) else float(f"{v:.12g}") for v in rho[s]] for s in lib],
    }
    with open(os.path.join(HERE, f"{workload}_optE.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1))
