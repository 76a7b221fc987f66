"""One process of a fanned-out oracle run over a block of libraries -- test infrastructure
only.

Run as ``python -m oracle.block_worker <in.npz> <out.npz> [panel.npy]`` by the full-size
parity tests, one process per chunk of libraries.  The input holds the panel (``ts``
[L][N], or read from ``panel.npy`` when that is given, so several workers share one file),
the library columns (``lib``) with their E (``E``), ``tau`` and ``k_max``.  A library
whose E is 0 first gets the oracle's optE (E = 1..20, leave-one-out, Tp = 1; Sec. II-B,
Alg. 1 phase 1), written with its skills (``optE`` [m], ``rho_E`` [m][20]).  For each
library it builds the oracle's neighbour table (Tp = 0; Sec. III-B, Alg. 2) and
cross-maps every column of the panel (Alg. 5 plus Pearson), then writes the SHA-256 of
each table's indices and of its FP32 squared distances (``idx_sha``, ``d2_sha``: uint8
[m][32], over the [L][k_max] rows in the library layout) and the rho rows (``rho`` [m][N],
FP64).
"""
import hashlib
import sys

import numpy as np

from . import ccm_oracle as O


def table_digests(idx, d2):
    """SHA-256 of one library's [L][k_max] indices (int32) and d^2 (float32), row-major."""
    a = hashlib.sha256(np.ascontiguousarray(idx, dtype=np.int32).tobytes()).digest()
    b = hashlib.sha256(np.ascontiguousarray(d2, dtype=np.float32).tobytes()).digest()
    return a, b


def main(argv):
    src, out = argv[0], argv[1]
    with np.load(src, allow_pickle=False) as z:
        ts = np.ascontiguousarray(np.load(argv[2], allow_pickle=False) if len(argv) > 2 else z["ts"])
        lib = z["lib"].astype(np.int64)
        E = z["E"].astype(np.int64)
        tau = int(z["tau"])
        k_max = int(z["k_max"])
    m, N = len(lib), ts.shape[1]
    idx_sha = np.zeros((m, 32), dtype=np.uint8)
    d2_sha = np.zeros((m, 32), dtype=np.uint8)
    rho = np.zeros((m, N))
    rho_E = np.full((m, 20), np.nan)
    for r in range(m):
        if E[r] == 0:
            oE, rE, _ = O.simplex_optE(ts, [int(lib[r])], 1, 20, tau, 1, O.MODE_LOO)
            E[r], rho_E[r] = int(oE[0]), rE[0]
        idx, w, d2 = O.knn(ts, [int(lib[r])], [int(E[r])], tau, 0, k_max)
        a, b = table_digests(idx[0], d2[0])
        idx_sha[r] = np.frombuffer(a, dtype=np.uint8)
        d2_sha[r] = np.frombuffer(b, dtype=np.uint8)
        rho[r] = O.crossmap_rho(ts, idx, w, [int(E[r])], tau, 0, N)[0]
    np.savez(out, idx_sha=idx_sha, d2_sha=d2_sha, rho=rho, optE=E.astype(np.int32), rho_E=rho_E)


if __name__ == "__main__":
    main(sys.argv[1:])
