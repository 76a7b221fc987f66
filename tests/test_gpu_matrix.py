"""The whole N x N causal matrix through ccm_matrix (phase 1, then blocks of libraries, each
a table call and a cross-map call against every series), against the oracle on the 64-map
coupled logistic network: optE as the oracle's (near-ties aside), every row whose library
E matches within 1e-5 (5e-3 in the BF16 form), in the library-E and the per-target-E forms,
and the same matrix bit for bit whatever the block size; and with phase 1 by the paper's half
split."""
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5


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


def test_matrix_logistic64_both_forms(ccm):
    import torch

    w = synth.make("logistic64")
    ts = w.panel
    N = ts.shape[1]
    Y = torch.as_tensor(ts).cuda()
    _say("ccm_matrix logistic64, E=1..10, blocks of 24 and 64")
    rho24, optE = ccm.ccm_matrix(Y, 1, 10, block=24)
    rho64, optE64 = ccm.ccm_matrix(Y, 1, 10, block=64)
    assert torch.equal(optE, optE64)
    assert torch.equal(rho24, rho64)          # a row does not depend on its block
    oE, oR, _ = O.simplex_optE(ts, np.arange(N), 1, 10, 1, 1)
    g = optE.cpu().numpy()
    same = g == oE
    for i in np.nonzero(~same)[0]:            # only near-ties may differ
        r = np.sort(oR[i][~np.isnan(oR[i])])[::-1]
        assert len(r) > 1 and r[0] - r[1] < 1e-6, f"optE differs at series {i}"
    rows = np.nonzero(same)[0]
    rho_o, _, _, _ = O.ccm_block(ts, rows, oE[rows], 1, 0, N, k_max=11)
    rg = rho24.cpu().numpy()[rows].astype(np.float64)
    assert np.array_equal(np.isnan(rg), np.isnan(rho_o))
    d = np.nanmax(np.abs(rg - rho_o))
    print(f"matrix library-E: |drho| max {d:.3e} over {len(rows)} rows")
    assert d < RHO_TOL
    _say("ccm_matrix logistic64, per-target E")
    rt, optE_t = ccm.ccm_matrix(Y, 1, 10, block=40, per_target_E=True)
    assert torch.equal(optE_t, optE)
    cols = np.nonzero(same)[0]
    rho_t = O.crossmap_rho_target_E(ts, np.arange(N), oE, 1, 0, N, k_max=11)
    rtg = rt.cpu().numpy().astype(np.float64)[:, cols]
    assert np.array_equal(np.isnan(rtg), np.isnan(rho_t[:, cols]))
    d = np.nanmax(np.abs(rtg - rho_t[:, cols]))
    print(f"matrix per-target E: |drho| max {d:.3e} over {len(cols)} columns")
    assert d < RHO_TOL
    _say("ccm_matrix logistic64, BF16 form")
    rb, _ = ccm.ccm_matrix(Y, 1, 10, block=64, precision=ccm.PRECISION_BF16)
    rbg = rb.cpu().numpy()[rows].astype(np.float64)
    assert np.array_equal(np.isnan(rbg), np.isnan(rho_o))
    d = np.nanmax(np.abs(rbg - rho_o))
    print(f"matrix BF16: |drho| max {d:.3e}")
    assert d < 5e-3


def test_matrix_logistic64_half_split(ccm):
    # phase 1 by the paper's half split (library half, target half) inside ccm_matrix; the
    # cross-map rows then use each library's half-split E
    import torch

    w = synth.make("logistic64")
    ts = w.panel
    N = ts.shape[1]
    Y = torch.as_tensor(ts).cuda()
    _say("ccm_matrix logistic64, half-split phase 1, E=1..8")
    rho, optE = ccm.ccm_matrix(Y, 1, 8, block=32, mode=ccm.MODE_HALF)
    oE, oR, _ = O.simplex_optE(ts, np.arange(N), 1, 8, 1, 1, mode=O.MODE_HALF)
    g = optE.cpu().numpy()
    same = g == oE
    for i in np.nonzero(~same)[0]:
        r = np.sort(oR[i][~np.isnan(oR[i])])[::-1]
        assert len(r) > 1 and r[0] - r[1] < 1e-6, f"optE differs at series {i}"
    rows = np.nonzero(same)[0]
    rho_o, _, _, _ = O.ccm_block(ts, rows, oE[rows], 1, 0, N, k_max=9)
    rg = rho.cpu().numpy()[rows].astype(np.float64)
    assert np.array_equal(np.isnan(rg), np.isnan(rho_o))
    d = np.nanmax(np.abs(rg - rho_o))
    print(f"matrix half split: |drho| max {d:.3e} over {len(rows)} rows")
    assert d < RHO_TOL
