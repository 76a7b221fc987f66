"""Parity at the benchmark's sizes, in its launch configuration, on outputs the oracle can
compute one by one: the 8192-series precision workload (FP32 and BF16 forms against FP64)
and the 512-library x 101,729-target block (optE, tables and rho on sampled libraries and
targets)."""
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


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


def _stats(d):
    d = d[~np.isnan(d)]
    return f"max {d.max():.2e} p99 {np.quantile(d, 0.99):.2e} median {np.median(d):.2e}"


def test_poisson8192_fp32_and_bf16_sampled(ccm):
    import torch

    w = synth.make("poisson8192")
    ts = w.panel
    Y = torch.as_tensor(ts).cuda()
    lib_ids = np.arange(0, 8192, 1024, dtype=np.int32)  # 8 libraries
    _say("poisson8192: optE, tables, FP32 and BF16 cross-maps over all 8192 targets")
    optE, rho_E = ccm.simplex_optE(Y, lib_ids, 1, 20, 1, 1)
    idx, wt, _ = ccm.knn(Y, lib_ids, optE, k_max=21)
    r32 = ccm.crossmap_rho(Y, idx, wt, optE).cpu().numpy()
    r16 = ccm.crossmap_rho(Y, idx, wt, optE, precision=ccm.PRECISION_BF16).cpu().numpy()
    lib_E = optE.cpu().numpy()
    idx_o, w_o, _ = O.knn(ts, lib_ids, lib_E, 1, 0, 21)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    tg = np.arange(0, 8192, 7)
    r_o = O.crossmap_rho(np.ascontiguousarray(ts[:, tg]), idx_o, w_o, lib_E, 1, 0, len(tg))
    d32 = np.abs(r32[:, tg] - r_o)
    d16 = np.abs(r16[:, tg] - r_o)
    print(f"poisson8192 |drho| FP32: {_stats(d32)}; BF16: {_stats(d16)}")
    assert np.nanmax(d32) < 1e-5 and np.nanmax(d16) < 5e-3
    # optE of two libraries against the oracle
    oE, oR, _ = O.simplex_optE(ts, lib_ids[:2], 1, 20, 1, 1)
    assert np.nanmax(np.abs(rho_E.cpu().numpy()[:2] - oR)) < 1e-5
    for a, b, r in zip(lib_E[:2], oE, oR):
        if a != b:
            s = np.sort(r[~np.isnan(r)])[::-1]
            assert s[0] - s[1] < 1e-6


def test_brain101729_block_sampled(ccm):
    import torch

    w = synth.make("brain101729")
    ts = w.panel
    L, N = ts.shape
    Y = torch.as_tensor(ts).cuda()
    lib_ids = torch.as_tensor(w.lib_ids).cuda()
    _say("brain101729: optE -> tables -> FP32 and BF16 cross-maps, 512 x 101729")
    optE, rho_E = ccm.simplex_optE(Y, lib_ids, 1, 20, 1, 1)
    idx, wt, _ = ccm.knn(Y, lib_ids, optE, 1, 0, 21)
    r32 = ccm.crossmap_rho(Y, idx, wt, optE, 1, 0, N)
    r16 = ccm.crossmap_rho(Y, idx, wt, optE, 1, 0, N, ccm.PRECISION_BF16)
    torch.cuda.synchronize()
    lib_E = optE.cpu().numpy()
    samp = [0, 137, 300, 511]
    tg = np.unique(np.concatenate([np.arange(0, N, 997), [N - 1]]))
    sub = np.ascontiguousarray(ts[:, tg])
    r32s = r32.cpu().numpy()[samp][:, tg]
    r16s = r16.cpu().numpy()[samp][:, tg]
    # optE of two sampled libraries
    oE, oR, _ = O.simplex_optE(ts, [0, 300], 1, 20, 1, 1)
    assert np.nanmax(np.abs(rho_E.cpu().numpy()[[0, 300]] - oR)) < 1e-5
    idx_np = idx.cpu().numpy()
    worst32 = worst16 = 0.0
    for li in samp:
        E = int(lib_E[li])
        oi, ow, _ = O.knn(ts, [li], [E], 1, 0, 21)
        assert np.array_equal(idx_np[li], oi[0]), f"library {li}: table differs"
        ro = O.crossmap_rho(sub, oi, ow, [E], 1, 0, len(tg))[0]
        k = samp.index(li)
        worst32 = max(worst32, float(np.nanmax(np.abs(r32s[k] - ro))))
        worst16 = max(worst16, float(np.nanmax(np.abs(r16s[k] - ro))))
    print(f"brain101729 sampled |drho|: FP32 {worst32:.2e}, BF16 {worst16:.2e}")
    assert worst32 < 1e-5 and worst16 < 5e-3
    # properties at full size: finite rho in [-1, 1] everywhere, diagonal near 1
    r = r32.cpu().numpy()
    assert np.all(np.isfinite(r)) and np.all(np.abs(r) <= 1.0 + 1e-6)
    assert np.all(r[np.arange(512), np.arange(512)] > 0.9)
