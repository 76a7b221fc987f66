"""GPU-vs-oracle parity of the HIP path, called through the C ABI.

kNN indices (and canonical FP32 d^2) must be bit-identical to the oracle's; rho must be
within 1e-5 of the FP64 oracle using the same neighbour sets; optE must agree except where
the oracle's two best skills are closer than 1e-6 (listed)."""
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


def _cuda(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _check_tables(ts, lib_ids, lib_E, tau, Tp, k_max, idx_g, w_g, d2_g, label):
    idx_o, w_o, d2_o = O.knn(ts, lib_ids, lib_E, tau, Tp, k_max)
    bad = np.argwhere(idx_g != idx_o)
    assert bad.size == 0, f"{label}: {len(bad)} index mismatches, first {bad[:3].tolist()}"
    valid = idx_o >= 0
    assert np.array_equal(d2_g[valid], d2_o[valid]), f"{label}: d2 not bit-identical"
    assert np.all(np.isinf(d2_g[~valid])) and np.all(w_g[~valid] == 0)
    err = np.abs(w_g.astype(np.float64) - w_o)
    assert err.max() < 2e-6, f"{label}: weight error {err.max()}"


# ---------------------------------------------------------------------------------------
def test_knn_bit_exact_adversarial(ccm):
    rng = np.random.default_rng(123)
    L = 150
    cols = [
        rng.integers(0, 4, size=L).astype(np.float32),            # many exact ties
        np.repeat(rng.integers(-3, 4, size=L // 5), 5)[:L].astype(np.float32),  # runs
        synth.periodic(6, L, rng),                                # exact repeats, d1 = 0
        (rng.standard_normal(L) * 1e-30).astype(np.float32),     # tiny values (subnormal d^2)
        rng.standard_normal(L).astype(np.float32),
        np.round(rng.standard_normal(L), 1).astype(np.float32),
    ]
    ts = np.stack(cols, axis=1)
    for tau in (1, 2):
        for Tp in (0, 1):
            lib_ids = np.array([0, 1, 2, 3, 4, 5, 0, 4, 2], dtype=np.int32)
            lib_E = np.array([1, 2, 3, 4, 5, 7, 6, 20, 2], dtype=np.int32)
            _say("knn adversarial", tau, Tp)
            idx, w, d2 = ccm.knn(_cuda(ts), lib_ids, lib_E, tau=tau, Tp=Tp, k_max=21)
            _check_tables(ts, lib_ids, lib_E, tau, Tp, 21, idx.cpu().numpy(), w.cpu().numpy(),
                          d2.cpu().numpy(), f"adv tau={tau} Tp={Tp}")


def test_knn_invalid_library_gets_padding(ccm):
    rng = np.random.default_rng(5)
    ts = rng.standard_normal((30, 2)).astype(np.float32)
    _say("knn invalid E")
    idx, w, d2 = ccm.knn(_cuda(ts), [0, 1, 0], [0, 25, 20], k_max=21)
    # E = 0, E = 25: out of range; E = 20 on 30 points leaves 10 points < k + 1 = 22
    assert np.all(idx.cpu().numpy() == -1) and np.all(w.cpu().numpy() == 0)


def test_series_ids_outside_the_panel(ccm):
    # ids outside [0, ld) are never read: padding tables, NaN skills (optE = E_min), NaN
    # embeddings; the valid ids of the same call are unaffected
    rng = np.random.default_rng(6)
    ts = rng.standard_normal((80, 2)).astype(np.float32)
    _say("series ids outside the panel: knn, simplex, embed")
    idx, w, d2 = ccm.knn(_cuda(ts), [1, -1, 2, 0], [3, 3, 3, 3], k_max=4)
    idx, w = idx.cpu().numpy(), w.cpu().numpy()
    assert np.all(idx[1:3] == -1) and np.all(w[1:3] == 0)
    ref_idx, ref_w, _ = ccm.knn(_cuda(ts), [1, 0], [3, 3], k_max=4)
    assert np.array_equal(idx[[0, 3]], ref_idx.cpu().numpy())
    assert np.array_equal(w[[0, 3]], ref_w.cpu().numpy())
    optE, rho = ccm.simplex_optE(_cuda(ts), [1, 7, -3], 2, 12, 1, 1)
    optE, rho = optE.cpu().numpy(), rho.cpu().numpy()
    assert list(optE[1:]) == [2, 2] and np.all(np.isnan(rho[1:]))
    ref_optE, ref_rho = ccm.simplex_optE(_cuda(ts), [1], 2, 12, 1, 1)
    assert optE[0] == ref_optE.item() and np.array_equal(rho[0], ref_rho.cpu().numpy()[0])
    emb = ccm.embed(_cuda(ts), [0, 2, -1], 4, 1).cpu().numpy()
    assert np.array_equal(emb[0], O.embed(ts[:, 0], 4, 1)) and np.all(np.isnan(emb[1:]))


def test_debug_mode_rejects_non_finite_inputs(ccm):
    # with the finiteness check on, a NaN or infinity in a series, target or weight that the
    # call reads makes it fail with CCM_EINVAL before any work; values it does not read
    # (other columns) are ignored
    import torch

    rng = np.random.default_rng(8)
    ts = rng.standard_normal((100, 6)).astype(np.float32)
    ts[40, 3] = np.nan
    Y = _cuda(ts)
    _say("debug mode: non-finite inputs")
    ccm.set_check_finite(True)
    try:
        def rejected(fn, *a, **kw):
            with pytest.raises(ccm.CCMError) as ei:
                fn(*a, **kw)
            assert ei.value.status == ccm.CCM_EINVAL and "non-finite" in str(ei.value)

        idx, wt, _ = ccm.knn(Y, [0, 1], [2, 2], k_max=3)
        rejected(ccm.knn, Y, [0, 3], [2, 2], k_max=3)
        rejected(ccm.simplex_optE, Y, [3], 1, 3, 1, 1)
        rejected(ccm.embed, Y, [1, 3], 2, 1)
        ccm.crossmap_rho(Y, idx, wt, [2, 2], tgt0=4, n_tgt=2)
        rejected(ccm.crossmap_rho, Y, idx, wt, [2, 2], tgt0=2, n_tgt=3)
        rejected(ccm.crossmap_rho, Y, idx, wt, [2, 2], tgt0=2, n_tgt=3,
                 precision=ccm.PRECISION_BF16)
        wbad = wt.clone()
        wbad[1, 10, 0] = float("inf")
        rejected(ccm.crossmap_rho, Y, idx, wbad, [2, 2], tgt0=4, n_tgt=2)
        X = torch.as_tensor(np.ascontiguousarray(ts[:, [0, 1]].T)).cuda()
        ccm.crossmap_rho_backward(Y, X, idx, wt, [2, 2], [0], [5], torch.ones(1))
        rejected(ccm.crossmap_rho_backward, Y, X, idx, wt, [2, 2], [0], [3], torch.ones(1))
        rejected(ccm.crossmap_rho_backward, Y, X, idx, wt, [2, 2], [0], [5],
                 torch.full((1,), float("nan")))
    finally:
        ccm.set_check_finite(False)
    idx2, wt2, _ = ccm.knn(Y, [0, 1], [2, 2], k_max=3)
    assert torch.equal(idx, idx2) and torch.equal(wt, wt2)


def test_knn_bit_exact_logistic64(ccm):
    w = synth.make("logistic64")
    ts = w.panel
    lib_E = (np.arange(64) % 10 + 1).astype(np.int32)
    _say("knn logistic64 all libraries, E = 1..10 mixed")
    idx, wt, d2 = ccm.knn(_cuda(ts), np.arange(64), lib_E, k_max=11)
    _check_tables(ts, np.arange(64), lib_E, 1, 0, 11, idx.cpu().numpy(), wt.cpu().numpy(),
                  d2.cpu().numpy(), "logistic64")


def test_knn_bit_exact_ratenet_sample(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    lib_ids = np.arange(0, 1024, 97, dtype=np.int32)  # 11 libraries
    lib_E = np.array([20, 1, 2, 5, 9, 13, 17, 19, 3, 7, 11], dtype=np.int32)
    _say("knn ratenet1024 sample")
    idx, wt, d2 = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=21)
    _check_tables(ts, lib_ids, lib_E, 1, 0, 21, idx.cpu().numpy(), wt.cpu().numpy(),
                  d2.cpu().numpy(), "ratenet1024")


# ---------------------------------------------------------------------------------------
def _check_optE(optE_g, rho_g, optE_o, rho_o, label):
    rho_o = np.asarray(rho_o)
    err = np.nanmax(np.abs(rho_g.astype(np.float64) - rho_o))
    assert np.array_equal(np.isnan(rho_g), np.isnan(rho_o)), label
    assert err < RHO_TOL, f"{label}: rho_E error {err}"
    near = []
    for i in range(len(optE_o)):
        if optE_g[i] != optE_o[i]:
            r = np.sort(rho_o[i][~np.isnan(rho_o[i])])[::-1]
            assert len(r) > 1 and r[0] - r[1] < 1e-6, f"{label}: optE differs at series {i}"
            near.append(i)
    if near:
        print(f"{label}: optE near-ties {near}")


def test_optE_logistic64(ccm):
    w = synth.make("logistic64")
    ts = w.panel
    ids = np.arange(64)
    _say("simplex logistic64 E=1..10")
    optE, rho = ccm.simplex_optE(_cuda(ts), ids, 1, 10, 1, 1, ccm.MODE_LOO)
    oE, oR, _ = O.simplex_optE(ts, ids, 1, 10, 1, 1)
    _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR, "logistic64")


def test_longer_horizons(ccm):
    # Tp > 1: candidates need s + Tp <= L - 1 and predict Tp steps ahead, in the tables and
    # in both phase-1 protocols
    w = synth.make("logistic64")
    ts = w.panel
    ids = np.arange(8)
    _say("knn Tp=3, logistic64 sample")
    lib_E = np.array([1, 2, 3, 5, 8, 10, 13, 20], dtype=np.int32)
    idx, wt, d2 = ccm.knn(_cuda(ts), ids, lib_E, Tp=3, k_max=21)
    _check_tables(ts, ids, lib_E, 1, 3, 21, idx.cpu().numpy(), wt.cpu().numpy(),
                  d2.cpu().numpy(), "Tp=3")
    _say("simplex Tp=3 LOO E=1..10, Tp=2 HALF tau=2 E=2..6")
    optE, rho = ccm.simplex_optE(_cuda(ts), ids, 1, 10, 1, 3, ccm.MODE_LOO)
    oE, oR, _ = O.simplex_optE(ts, ids, 1, 10, 1, 3)
    _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR, "Tp=3 LOO")
    optE, rho = ccm.simplex_optE(_cuda(ts), ids, 2, 6, 2, 2, ccm.MODE_HALF)
    oE, oR, _ = O.simplex_optE(ts, ids, 2, 6, 2, 2, O.MODE_HALF)
    _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR, "Tp=2 HALF tau=2")


def test_optE_lags_and_clipped_E_ranges(ccm):
    # tau > 1 with E ranges that start and end inside the kernel's E groups: lists seeded
    # from neighbouring E must respect each E's own first admissible candidate (E - 1) tau,
    # and lists of clipped-off E must neither be scored nor feed their neighbours' seeds
    w = synth.make("logistic64")
    ts = w.panel
    ids = np.arange(6)
    for E_min, E_max, tau in ((3, 17, 2), (5, 14, 3), (2, 2, 2), (19, 20, 1)):
        _say(f"simplex LOO E={E_min}..{E_max} tau={tau}, logistic64 sample")
        optE, rho = ccm.simplex_optE(_cuda(ts), ids, E_min, E_max, tau, 1, ccm.MODE_LOO)
        oE, oR, _ = O.simplex_optE(ts, ids, E_min, E_max, tau, 1)
        _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR,
                    f"LOO E={E_min}..{E_max} tau={tau}")


def test_optE_horizon_zero_ragged_last_chunk(ccm):
    # Tp = 0: the last candidate is the series' last point, so the final chunk of 64
    # candidates reaches furthest past the series (its extra lanes read the zero tail and are
    # never admitted); lengths that leave 1, 63 and 37 candidates in that chunk for the lists
    # of E = 1..4, whose candidates start at 0
    w = synth.make("logistic64")
    ids = np.arange(4)
    for L in (65, 127, 165):
        ts = np.ascontiguousarray(w.panel[:L])
        for mode, omode in ((ccm.MODE_LOO, O.MODE_LOO), (ccm.MODE_HALF, O.MODE_HALF)):
            E_max = 20 if mode == ccm.MODE_LOO else 8
            _say(f"simplex Tp=0 L={L} mode={mode} E=1..{E_max}")
            optE, rho = ccm.simplex_optE(_cuda(ts), ids, 1, E_max, 1, 0, mode)
            oE, oR, _ = O.simplex_optE(ts, ids, 1, E_max, 1, 0, mode=omode)
            _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR, f"Tp=0 L={L} mode={mode}")


def test_optE_ratenet_sample_and_half_mode(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    ids = np.array([3, 500, 1021], dtype=np.int32)
    _say("simplex ratenet1024 sample E=1..20")
    optE, rho = ccm.simplex_optE(_cuda(ts), ids, 1, 20, 1, 1, ccm.MODE_LOO)
    oE, oR, _ = O.simplex_optE(ts, ids, 1, 20, 1, 1)
    _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR, "ratenet LOO")
    _say("simplex HALF / tau=2 / E=3..8")
    optE, rho = ccm.simplex_optE(_cuda(ts), ids, 3, 8, 2, 1, ccm.MODE_HALF)
    oE, oR, _ = O.simplex_optE(ts, ids, 3, 8, 2, 1, O.MODE_HALF)
    _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR, "ratenet HALF")


def test_optE_half_split_full_E_range_brain_sample(ccm):
    # the paper's phase-1 protocol over E = 1..20 at tau = 1 on filtered-Poisson rates
    w = synth.make("brain101729")
    ids = np.array([0, 1, 77, 511, 4096, 50000, 101728], dtype=np.int32)
    ts = np.ascontiguousarray(w.panel[:, ids])
    _say("simplex HALF E=1..20, 7 brain101729 series")
    optE, rho = ccm.simplex_optE(_cuda(ts), np.arange(len(ids), dtype=np.int32), 1, 20, 1, 1,
                                 ccm.MODE_HALF)
    oE, oR, _ = O.simplex_optE(ts, list(range(len(ids))), 1, 20, 1, 1, O.MODE_HALF)
    _check_optE(optE.cpu().numpy(), rho.cpu().numpy(), oE, oR, "brain HALF")


def test_optE_degenerate_constant(ccm):
    ts = np.ones((60, 2), dtype=np.float32)
    ts[:, 1] = np.arange(60) % 2
    _say("simplex constant series")
    optE, rho = ccm.simplex_optE(_cuda(ts), [0], 2, 5, 1, 1)
    assert optE.item() == 2 and np.all(np.isnan(rho.cpu().numpy()))


# ---------------------------------------------------------------------------------------
def _check_rho(rho_g, rho_o, label, tol=RHO_TOL):
    assert np.array_equal(np.isnan(rho_g), np.isnan(rho_o)), f"{label}: NaN pattern differs"
    d = np.abs(rho_g.astype(np.float64) - rho_o)[~np.isnan(rho_o)]
    print(f"{label}: |drho| max {d.max():.3e} p99 {np.quantile(d, 0.99):.3e} "
          f"median {np.median(d):.3e}")
    assert d.max() < tol, f"{label}: max |drho| {d.max()}"


def test_crossmap_logistic64_full_block(ccm):
    w = synth.make("logistic64")
    ts = w.panel
    oE, _, _ = O.simplex_optE(ts, np.arange(64), 1, 10, 1, 1)
    _say("crossmap logistic64 64x64")
    idx, wt, _ = ccm.knn(_cuda(ts), np.arange(64), oE, k_max=11)
    rho = ccm.crossmap_rho(_cuda(ts), idx, wt, oE).cpu().numpy()
    rho_o, idx_o, _, _ = O.ccm_block(ts, np.arange(64), oE, 1, 0, 64, k_max=11)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    _check_rho(rho, rho_o, "logistic64")


def test_crossmap_ratenet_ragged_targets(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    lib_ids = np.arange(5, 1024, 41, dtype=np.int32)  # 25 libraries
    lib_E = (np.arange(25) * 7 % 20 + 1).astype(np.int32)
    tgt0, n_tgt = 7, 1001  # ragged last tile
    _say("crossmap ratenet1024 25 libs x 1001 targets")
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=21)
    rho, mom = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tgt0=tgt0, n_tgt=n_tgt,
                                want_moments=True)
    idx_o, w_o, _ = O.knn(ts, lib_ids, lib_E, 1, 0, 21)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    rho_o = O.crossmap_rho(ts, idx_o, w_o, lib_E, 1, tgt0, n_tgt)
    _check_rho(rho.cpu().numpy(), rho_o, "ratenet1024")
    # moments: sum(yhat) against the oracle prediction for one pair
    i, j = 3, 500
    E = int(lib_E[i])
    Q = np.arange(E - 1, ts.shape[0])
    y = ts[:, tgt0 + j].astype(np.float64)
    yhat = np.sum(w_o[i][Q, : E + 1] * y[idx_o[i][Q, : E + 1]], axis=1)
    m = mom.cpu().numpy()[i, j]
    np.testing.assert_allclose(m, [yhat.sum(), (yhat * yhat).sum(), (y[Q] * yhat).sum()],
                               rtol=1e-5, atol=1e-3)


def test_crossmap_nan_for_constant_target_and_bad_library(ccm):
    rng = np.random.default_rng(9)
    ts = rng.standard_normal((120, 20)).astype(np.float32)
    ts[:, 4] = 2.0
    lib_E = np.array([3, 2, 0], dtype=np.int32)  # third library unusable
    _say("crossmap NaN cases")
    idx, wt, _ = ccm.knn(_cuda(ts), [0, 1, 2], lib_E, k_max=4)
    rho = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E).cpu().numpy()
    assert np.all(np.isnan(rho[:, 4])) and np.all(np.isnan(rho[2]))
    idx_o, w_o, _ = O.knn(ts, [0, 1], lib_E[:2], 1, 0, 4)
    rho_o = O.crossmap_rho(ts, idx_o, w_o, lib_E[:2], 1, 0, 20)
    _check_rho(rho[:2], rho_o, "small")


# ---------------------------------------------------------------------------------------
BF16_TOL = 5e-3


def test_crossmap_bf16_logistic64(ccm):
    w = synth.make("logistic64")
    ts = w.panel
    oE = (np.arange(64) % 7 + 2).astype(np.int32)
    _say("crossmap BF16 logistic64 64x64")
    idx, wt, _ = ccm.knn(_cuda(ts), np.arange(64), oE, k_max=11)
    rho = ccm.crossmap_rho(_cuda(ts), idx, wt, oE, precision=ccm.PRECISION_BF16).cpu().numpy()
    rho_o, _, _, _ = O.ccm_block(ts, np.arange(64), oE, 1, 0, 64, k_max=11)
    _check_rho(rho, rho_o, "logistic64 BF16", tol=BF16_TOL)


def test_crossmap_bf16_ratenet_ragged(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    lib_ids = np.arange(3, 1024, 51, dtype=np.int32)  # 21 libraries (odd count)
    lib_E = (np.arange(21) * 3 % 20 + 1).astype(np.int32)
    tgt0, n_tgt = 5, 1000  # ragged last 128-target tile
    _say("crossmap BF16 ratenet1024 21 libs x 1000 targets")
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=21)
    rho, mom = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tgt0=tgt0, n_tgt=n_tgt,
                                precision=ccm.PRECISION_BF16, want_moments=True)
    idx_o, w_o, _ = O.knn(ts, lib_ids, lib_E, 1, 0, 21)
    rho_o = O.crossmap_rho(ts, idx_o, w_o, lib_E, 1, tgt0, n_tgt)
    _check_rho(rho.cpu().numpy(), rho_o, "ratenet1024 BF16", tol=BF16_TOL)
    rho32 = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tgt0=tgt0, n_tgt=n_tgt).cpu().numpy()
    _check_rho(rho32, rho_o, "ratenet1024 FP32 (same tables)")


def test_crossmap_bf16_nan_cases(ccm):
    rng = np.random.default_rng(9)
    ts = rng.standard_normal((120, 20)).astype(np.float32)
    ts[:, 4] = 2.0
    lib_E = np.array([3, 2, 0], dtype=np.int32)
    _say("crossmap BF16 NaN cases")
    idx, wt, _ = ccm.knn(_cuda(ts), [0, 1, 2], lib_E, k_max=4)
    rho = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, precision=ccm.PRECISION_BF16).cpu().numpy()
    assert np.all(np.isnan(rho[:, 4])) and np.all(np.isnan(rho[2]))
    assert not np.any(np.isnan(np.delete(rho[:2], 4, 1)))
