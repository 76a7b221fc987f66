"""Write tests/golden/ratenet1024_optE.json: the CPU oracle's simplex skills and optE of all
1,024 series of the 1,024-series rate-network workload (E = 1..20, leave-one-out, Tp = 1,
tau = 1; Sec. II-B and Alg. 1 phase 1).  Only the oracle and the seeded input generator are
called.  The full-matrix GPU parity test reads this file instead of spending about an hour
of CPU time on the box.

    python tests/golden/make_ratenet1024_optE.py [processes]
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


def _chunk(ids):
    ts = synth.make("ratenet1024").panel
    optE, rho, _ = O.simplex_optE(ts, ids, E_MIN, E_MAX, TAU, TP, O.MODE_LOO)
    return ids, optE, rho


def main(procs: int) -> None:
    ts = synth.make("ratenet1024").panel
    N = ts.shape[1]
    chunks = [list(range(a, min(N, a + 16))) for a in range(0, N, 16)]
    optE = np.zeros(N, dtype=np.int32)
    rho = np.zeros((N, E_MAX - E_MIN + 1))
    with ProcessPoolExecutor(max_workers=procs) as ex:
        for ids, e, r in ex.map(_chunk, chunks):
            optE[ids] = e
            rho[ids] = r
            print(f"series {ids[0]}..{ids[-1]} done", flush=True)
    out = {
        "workload": "ratenet1024",
        "panel_sha256": panel_sha256(ts),
        "E_min": E_MIN, "E_max": E_MAX, "tau": TAU, "Tp": TP, "mode": "leave-one-out",
        "optE": optE.tolist(),
        # skills rho_E [series][E - E_min] (FP64 oracle, 12 significant digits; NaN as null)
        "rho_E": [[None if np.isnan(v) else float(f"{v:.12g}") for v in row] for row in rho],
    }
    with open(os.path.join(HERE, "ratenet1024_optE.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1))
