"""Whole-matrix parity on the 1,024-series rate-network workload (L = 1,450): every output
of the N x N map of Alg. 2 (Sec. III-B) against the oracle, nothing sampled.

  * optE of all 1,024 series (E = 1..20, leave-one-out, Tp = 1; Alg. 1 phase 1) against the
    oracle's, stored in tests/golden/ratenet1024_optE.json by a script that calls only the
    oracle (about an hour of CPU time); where they differ, the oracle's two best skills must
    be closer than 1e-6.  The skills themselves agree within 1e-5.
  * all 1,024 tables at the oracle's optE bit-identical (indices and FP32 d^2) to the
    oracle's, which the test computes itself, fanned out over the host's cores;
  * the whole 1,024 x 1,024 rho within 1e-5 (FP32 gather) and 5e-3 (BF16 form) of the FP64
    oracle, and the N x N driver (ccm_matrix) equal to the direct calls."""
import hashlib
import json
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "ratenet1024_optE.json")
RHO_TOL = 1e-5
BF16_TOL = 5e-3
SKILL_TOL = 1e-5


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ccm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_11082_amd as m

    m.load_library()
    return m


def _oracle_block(ts, lib_E, k_max):
    """The oracle's table digests and rho rows of every library (column i at E lib_E[i]),
    one worker process per chunk of libraries on at most 16 cores."""
    N = ts.shape[1]
    P = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                   else (os.cpu_count() or 1)))
    chunks = np.array_split(np.arange(N), P)
    tmp = tempfile.mkdtemp(prefix="ccm_full_oracle_")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    try:
        procs = []
        for c, ids in enumerate(chunks):
            src = os.path.join(tmp, f"in{c}.npz")
            np.savez(src, ts=ts, lib=ids.astype(np.int32), E=lib_E[ids].astype(np.int32),
                     tau=1, k_max=k_max)
            procs.append(subprocess.Popen([sys.executable, "-m", "oracle.block_worker", src,
                                           os.path.join(tmp, f"out{c}.npz")], cwd=ROOT, env=env))
        rcs = [p.wait() for p in procs]
        assert not any(rcs), f"oracle workers failed: {rcs}"
        idx_sha = np.zeros((N, 32), dtype=np.uint8)
        d2_sha = np.zeros((N, 32), dtype=np.uint8)
        rho = np.zeros((N, N))
        for c, ids in enumerate(chunks):
            with np.load(os.path.join(tmp, f"out{c}.npz"), allow_pickle=False) as z:
                idx_sha[ids], d2_sha[ids], rho[ids] = z["idx_sha"], z["d2_sha"], z["rho"]
        return idx_sha, d2_sha, rho, P
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def _stats(d):
    return (f"max {d.max():.3e} p99 {np.quantile(d, 0.99):.3e} median {np.median(d):.3e} "
            f"over {d.size} values")


def test_ratenet1024_whole_matrix(ccm):
    import torch

    from oracle.block_worker import table_digests

    with open(GOLDEN) as f:
        gold = json.load(f)
    ts = synth.make("ratenet1024").panel
    L, N = ts.shape
    sha = hashlib.sha256(np.ascontiguousarray(ts, dtype=np.float32).tobytes()).hexdigest()
    assert sha == gold["panel_sha256"], ("the 1,024-series input generator changed: rerun "
                                         "tests/golden/make_optE_golden.py ratenet1024")
    oE = np.asarray(gold["optE"], dtype=np.int32)
    oR = np.array([[np.nan if v is None else v for v in row] for row in gold["rho_E"]])
    d = torch.as_tensor(ts).cuda()
    ids = torch.arange(N, dtype=torch.int32, device="cuda")

    _say("ratenet1024: optE of all 1,024 series")
    gE, gR = (a.cpu().numpy() for a in ccm.simplex_optE(d, ids, 1, 20, 1, 1, ccm.MODE_LOO))
    assert np.array_equal(np.isnan(gR), np.isnan(oR))
    dskill = np.abs(gR.astype(np.float64) - oR)[~np.isnan(oR)]
    print("skills:", _stats(dskill))
    assert dskill.max() < SKILL_TOL
    ties = []
    for i in np.nonzero(gE != oE)[0]:
        s_ = np.sort(oR[i][~np.isnan(oR[i])])[::-1]
        assert s_[0] - s_[1] < 1e-6, f"series {i}: GPU optE {gE[i]}, oracle {oE[i]}"
        ties.append(int(i))
    print(f"optE: {N - len(ties)} of {N} equal; near-ties (< 1e-6) {ties}")

    _say("ratenet1024: 1,024 tables at the oracle's optE and the 1,024 x 1,024 rho")
    k_max = 21
    idx, w, d2 = ccm.knn(d, ids, torch.as_tensor(oE).cuda(), k_max=k_max)
    rho32 = ccm.crossmap_rho(d, idx, w, torch.as_tensor(oE).cuda()).cpu().numpy()
    rho16 = ccm.crossmap_rho(d, idx, w, torch.as_tensor(oE).cuda(),
                             precision=ccm.PRECISION_BF16).cpu().numpy()
    idx, d2 = idx.cpu().numpy(), d2.cpu().numpy()

    _say("ratenet1024: the oracle over all 1,024 libraries (host processes)")
    o_idx_sha, o_d2_sha, rho_o, P = _oracle_block(ts, oE, k_max)
    print(f"oracle fanned out over {P} processes")
    bad = []
    for i in range(N):
        a, b = table_digests(idx[i], d2[i])
        if a != o_idx_sha[i].tobytes() or b != o_d2_sha[i].tobytes():
            bad.append(i)
    assert not bad, f"{len(bad)} tables differ from the oracle's, first libraries {bad[:8]}"

    assert np.array_equal(np.isnan(rho32), np.isnan(rho_o)), "FP32: NaN pattern differs"
    valid = ~np.isnan(rho_o)
    d32 = np.abs(rho32.astype(np.float64) - rho_o)[valid]
    d16 = np.abs(rho16.astype(np.float64) - rho_o)[valid]
    print("FP32 rho:", _stats(d32))
    print("BF16 rho:", _stats(d16))
    assert d32.max() < RHO_TOL
    assert d16.max() < BF16_TOL

    _say("ratenet1024: ccm_matrix against the direct calls")
    rho_m, optE_m = ccm.ccm_matrix(d)
    rho_m, optE_m = rho_m.cpu().numpy(), optE_m.cpu().numpy()
    assert np.array_equal(optE_m, gE)
    same = gE == oE   # libraries whose table is the one compared above
    assert np.array_equal(rho_m[same], rho32[same], equal_nan=True)
