"""One process of the CPU oracle's timing sample -- test infrastructure only.

Run as ``python -m oracle.sample_worker <sample.npz> <column> <out.npz>`` by the
benchmark's ``cpu_baseline`` leg, one process per library on its own core.  The sample
file holds the library series (``lib`` [L][n]) and the sampled targets (``tgt`` [L][m]).
For library column ``column`` it runs the oracle's optE (E = 1..20, leave-one-out,
Tp = 1; Alg. 1 phase 1), the table at that E (Tp = 0; Alg. 2) and the cross-map of every
sampled target (Alg. 5 plus Pearson), and writes E, the table indices, rho and the two
timings (seconds per library for optE + table, seconds per library-target pair).
"""
import sys
import time

import numpy as np

from . import ccm_oracle as O


def main(argv):
    path, col, out = argv[0], int(argv[1]), argv[2]
    with np.load(path, allow_pickle=False) as z:
        lib = np.ascontiguousarray(z["lib"])
        tgt = np.ascontiguousarray(z["tgt"])
    a = time.perf_counter()
    oE, _, _ = O.simplex_optE(lib, [col], 1, 20, 1, 1)
    E = int(oE[0])
    idx, w, _ = O.knn(lib, [col], [E], 1, 0, 21)
    b = time.perf_counter()
    rho = O.crossmap_rho(tgt, idx, w, [E], 1, 0, tgt.shape[1])
    c = time.perf_counter()
    np.savez(out, E=E, idx=idx[0], rho=rho[0], t_lib=b - a, t_pair=(c - b) / tgt.shape[1])


if __name__ == "__main__":
    main(sys.argv[1:])
