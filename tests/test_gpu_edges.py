"""Edge cases of the HIP path against the oracle, through the C ABI: the delay embedding
(bit-exact, every E and several lags), lag tau = 2 in the cross-map (both precisions), the
largest series the 16-target FP32 LDS tile holds (L = 2475) and series beyond it (L = 3000:
8-target LDS tiles; L = 6000: the 32-target global copy), each also through every other tile
width the testing switch can force (the 4-target LDS tile included), in both the library-E and
the per-target-E forms; long series in
the table and optE kernels (sampled query rows), the largest length the ABI accepts in the
tables, both cross-map forms and the adjoint, and empty inputs."""
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


def _cuda(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _check_rho(rho_g, rho_o, label, tol):
    assert np.array_equal(np.isnan(rho_g), np.isnan(rho_o)), f"{label}: NaN pattern differs"
    d = np.abs(rho_g.astype(np.float64) - rho_o)[~np.isnan(rho_o)]
    print(f"{label}: |drho| max {d.max():.3e}")
    assert d.max() < tol, f"{label}: max |drho| {d.max()}"


def test_embed_bit_exact(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    ids = np.array([0, 5, 1023, 512, 77], dtype=np.int32)
    for E, tau in [(1, 1), (2, 1), (7, 1), (20, 1), (3, 2), (5, 3), (20, 4)]:
        _say(f"embed E={E} tau={tau}, 5 series of L={ts.shape[0]}")
        emb = ccm.embed(_cuda(ts), ids, E, tau).cpu().numpy()
        assert emb.shape == (len(ids), ts.shape[0] - (E - 1) * tau, E)
        for r, c in enumerate(ids):
            assert np.array_equal(emb[r], O.embed(ts[:, c], E, tau)), (E, tau, c)
    # the shortest series that still has a point, and one that has none (an error)
    short = np.ascontiguousarray(ts[:11])
    emb = ccm.embed(_cuda(short), ids[:2], 6, 2).cpu().numpy()
    assert emb.shape == (2, 1, 6)
    assert np.array_equal(emb[1], O.embed(short[:, ids[1]], 6, 2))
    with pytest.raises(ccm.CCMError) as ei:
        ccm.embed(_cuda(short[:10]), ids[:2], 6, 2)
    assert ei.value.status == ccm.CCM_ERANGE


def test_crossmap_tau2_both_precisions(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    lib_ids = np.array([2, 90, 333, 700, 1001, 512], dtype=np.int32)
    lib_E = np.array([1, 3, 8, 12, 20, 5], dtype=np.int32)
    tgt0, n_tgt = 3, 77
    _say("crossmap tau=2, 6 libraries x 77 targets")
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, tau=2, k_max=21)
    idx_o, w_o, _ = O.knn(ts, lib_ids, lib_E, 2, 0, 21)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    rho_o = O.crossmap_rho(ts, idx_o, w_o, lib_E, 2, tgt0, n_tgt)
    r32 = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tau=2, tgt0=tgt0, n_tgt=n_tgt)
    _check_rho(r32.cpu().numpy(), rho_o, "tau=2 FP32", 1e-5)
    r16 = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tau=2, tgt0=tgt0, n_tgt=n_tgt,
                           precision=ccm.PRECISION_BF16)
    _check_rho(r16.cpu().numpy(), rho_o, "tau=2 BF16", 5e-3)
    # the narrower tiles and the global copy at tau = 2 (the tables' first rows and the
    # column sums start at (E - 1) tau)
    try:
        for tj in (8, 4, 32):
            _say(f"crossmap tau=2, tile {tj}")
            ccm.set_gather_tile(tj)
            r = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tau=2, tgt0=tgt0, n_tgt=n_tgt)
            _check_rho(r.cpu().numpy(), rho_o, f"tau=2 FP32 tile {tj}", 1e-5)
    finally:
        ccm.set_gather_tile(0)


def test_crossmap_at_the_largest_fp32_tile(ccm):
    L = 2475                                  # L * 64 B + the column sums fill the 160 KB LDS
    rng = np.random.default_rng(41)
    ts = np.cumsum(rng.standard_normal((L, 40)), axis=0).astype(np.float32)
    ts = (ts - ts.mean(0)) / ts.std(0)
    lib_ids, lib_E = [0, 7, 33], np.array([2, 5, 9], dtype=np.int32)
    _say("crossmap L=2475, 3 libraries x 40 targets")
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=10)
    rho_o, idx_o, _, _ = O.ccm_block(ts, lib_ids, lib_E, 1, 0, 40, k_max=10)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    try:
        for tj in (0, 8, 4, 32):             # 0: the 16-target LDS tile
            _say(f"crossmap L=2475, tile {tj or 16}")
            ccm.set_gather_tile(tj)
            rho = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E).cpu().numpy()
            _check_rho(rho, rho_o, f"L=2475 tile {tj or 16}", 1e-5)
    finally:
        ccm.set_gather_tile(0)


def test_crossmap_beyond_the_lds_tile(ccm):
    L = 3000                                  # past 2475: 8-target tiles in LDS
    rng = np.random.default_rng(47)
    ts = np.cumsum(rng.standard_normal((L, 40)), axis=0).astype(np.float32)
    ts = ((ts - ts.mean(0)) / ts.std(0)).astype(np.float32)
    lib_ids, lib_E = [0, 7, 33], np.array([2, 7, 20], dtype=np.int32)
    tgt0, n_tgt = 3, 37                       # three tiles, the last one ragged
    _say("crossmap L=3000, 3 libraries x 37 targets")
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=21)
    rho_o, idx_o, _, _ = O.ccm_block(ts, lib_ids, lib_E, 1, tgt0, n_tgt, k_max=21)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    try:
        for tj in (0, 4, 32):                # 0: the 8-target LDS tile
            _say(f"crossmap L=3000, tile {tj or 8}")
            ccm.set_gather_tile(tj)
            rho, mom = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tgt0=tgt0, n_tgt=n_tgt,
                                        want_moments=True)
            _check_rho(rho.cpu().numpy(), rho_o, f"L=3000 tile {tj or 8}", 1e-5)
            assert np.all(np.isfinite(mom.cpu().numpy()))
    finally:
        ccm.set_gather_tile(0)
    r16 = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tgt0=tgt0, n_tgt=n_tgt,
                           precision=ccm.PRECISION_BF16)
    _check_rho(r16.cpu().numpy(), rho_o, "L=3000 BF16", 5e-3)
    tgt_E = rng.integers(3, 5, size=n_tgt).astype(np.int32)
    idx, wt, _ = ccm.knn_all_E(_cuda(ts), lib_ids[:2], 3, 2, k_max=21)
    rho_o = O.crossmap_rho_target_E(ts, lib_ids[:2], tgt_E, 1, tgt0, n_tgt, k_max=21)
    try:
        for tj in (0, 32):                   # 0: the 8-target LDS tile
            _say(f"crossmap per-target E, L=3000, tile {tj or 8}, 2 libraries x 37 targets")
            ccm.set_gather_tile(tj)
            rho = ccm.crossmap_rho_target_E(_cuda(ts), idx, wt, 2, tgt_E, E_lo=3, tgt0=tgt0,
                                            n_tgt=n_tgt).cpu().numpy()
            _check_rho(rho, rho_o, f"L=3000 per-target E tile {tj or 8}", 1e-5)
    finally:
        ccm.set_gather_tile(0)


def test_crossmap_global_and_four_target_tiles(ccm):
    L = 6000                                  # past 5035: the global copy, or 4-target tiles
    rng = np.random.default_rng(53)
    ts = np.cumsum(rng.standard_normal((L, 24)), axis=0).astype(np.float32)
    ts = ((ts - ts.mean(0)) / ts.std(0)).astype(np.float32)
    lib_ids, lib_E = [0, 11], np.array([3, 12], dtype=np.int32)
    tgt0, n_tgt = 2, 21                       # six tiles, the last one ragged
    _say("crossmap L=6000, 2 libraries x 21 targets")
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=13)
    rho_o, idx_o, _, _ = O.ccm_block(ts, lib_ids, lib_E, 1, tgt0, n_tgt, k_max=13)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    try:
        for tj in (0, 4):                    # 0: the 32-target global copy
            _say(f"crossmap L=6000, tile {tj or 32}")
            ccm.set_gather_tile(tj)
            rho = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tgt0=tgt0, n_tgt=n_tgt)
            _check_rho(rho.cpu().numpy(), rho_o, f"L=6000 tile {tj or 32}", 1e-5)
    finally:
        ccm.set_gather_tile(0)


def test_long_series_tables_and_optE(ccm):
    L = 16384                                  # the largest L the ABI accepts
    rng = np.random.default_rng(42)
    x = np.sin(0.05 * np.arange(L)) + 0.3 * rng.standard_normal(L)
    ts = np.stack([x, np.roll(x, 7)], axis=1).astype(np.float32)
    E = 3
    _say("knn L=16384 E=3, sampled rows")
    idx, wt, d2 = ccm.knn(_cuda(ts), [0], [E], k_max=4)
    idx, wt, d2 = idx.cpu().numpy()[0], wt.cpu().numpy()[0], d2.cpu().numpy()[0]
    Q, C, _ = O.point_sets(L, E, 1, 0)
    q = Q[::331]
    D2 = O.sqdist_fp32(ts[:, 0], q, C, E, 1)
    idx_o, d2_o = O.select_knn(D2, q, C, E + 1, True)
    w_o = O.weights_rows_fp64(ts[:, 0], q, idx_o, E, 1)
    assert np.array_equal(idx[q], idx_o)
    assert np.array_equal(d2[q], d2_o)
    assert np.abs(wt[q].astype(np.float64) - w_o).max() < 2e-6
    assert np.all(idx[: E - 1] == -1)
    # optE at L = 16384 on an exactly periodic series with distinct phase values: every
    # query has exact repeats as neighbours (d_1 = 0), so each prediction is exact and every
    # skill is 1 (which E wins is then decided by rounding: all skills tie within 1e-6)
    _say("optE L=16384 periodic, E=1..6")
    per = np.stack([synth.periodic(37, L, rng), synth.periodic(53, L, rng)], axis=1)
    optE, rho_E = ccm.simplex_optE(_cuda(per), [0, 1], 1, 6, 1, 1)
    assert np.abs(rho_E.cpu().numpy() - 1.0).max() < 1e-6
    assert np.all((optE.cpu().numpy() >= 1) & (optE.cpu().numpy() <= 6))
    # and the oracle on a 3,000-step prefix of the noisy pair, every skill
    _say("optE L=3000 E=1..4")
    ts3 = np.ascontiguousarray(ts[:3000])
    optE, rho_E = ccm.simplex_optE(_cuda(ts3), [0, 1], 1, 4, 1, 1)
    oE, oR, _ = O.simplex_optE(ts3, [0, 1], 1, 4, 1, 1)
    assert np.array_equal(optE.cpu().numpy(), oE)
    assert np.abs(rho_E.cpu().numpy() - oR).max() < 1e-5


def test_maximum_length_crossmap_and_adjoint(ccm):
    # L = 16384, the largest the ABI accepts: tables at E = 3 and E = 20 on sampled rows
    # against the oracle; the cross-map (FP32 from the global 32-target tile, and BF16) of
    # an exactly periodic library with distinct phase states, whose targets of the same
    # period are predicted exactly (every neighbour has d = 0 and the same phase, so
    # rho = 1) and whose constant target gives NaN; and the adjoint's invariances
    # (rho unchanged by y -> a y + b and x -> a x + b) on the noisy library's tables.
    import torch

    L = 16384
    rng = np.random.default_rng(47)
    x = (np.sin(0.031 * np.arange(L)) + 0.3 * rng.standard_normal(L)).astype(np.float32)
    P = 37
    cols = [x, synth.periodic(P, L, rng)]
    cols += [synth.periodic(P, L, rng) for _ in range(38)]      # targets 2..39
    cols += [np.full(L, 0.5, np.float32), np.roll(x, 5)]        # 40: constant, 41: noisy
    ts = np.stack(cols, axis=1).astype(np.float32)
    Y = _cuda(ts)
    libs, lib_E = [0, 0, 1], [3, 20, 3]
    _say("knn L=16384 E=3 and E=20, sampled rows")
    idx, wt, d2 = ccm.knn(Y, libs, lib_E, k_max=21)
    idx_h, wt_h, d2_h = idx.cpu().numpy(), wt.cpu().numpy(), d2.cpu().numpy()
    for r in (0, 1):
        E = lib_E[r]
        Q, C, _ = O.point_sets(L, E, 1, 0)
        q = np.concatenate([Q[:3], Q[::523], Q[-3:]])
        D2 = O.sqdist_fp32(x, q, C, E, 1)
        idx_o, d2_o = O.select_knn(D2, q, C, E + 1, True)
        w_o = O.weights_rows_fp64(x, q, idx_o, E, 1)
        assert np.array_equal(idx_h[r][q][:, : E + 1], idx_o), f"E={E} indices"
        assert np.array_equal(d2_h[r][q][:, : E + 1], d2_o), f"E={E} d2"
        assert np.abs(wt_h[r][q][:, : E + 1].astype(np.float64) - w_o).max() < 2e-6
        assert np.all(idx_h[r][q][:, E + 1:] == -1) and np.all(idx_h[r][: E - 1] == -1)
    _say("crossmap L=16384 periodic library, 40 targets (FP32 global tile, BF16)")
    sub = (idx[2:3].contiguous(), wt[2:3].contiguous())
    for prec, tol in ((ccm.PRECISION_FP32, 1e-6), (ccm.PRECISION_BF16, 5e-3)):
        rho = ccm.crossmap_rho(Y, sub[0], sub[1], [3], tgt0=2, n_tgt=39,
                               precision=prec).cpu().numpy()[0]
        assert np.abs(rho[:38] - 1.0).max() < tol, (prec, np.abs(rho[:38] - 1.0).max())
        assert np.isnan(rho[38])
    _say("adjoint L=16384, 2 pairs")
    X = torch.as_tensor(np.ascontiguousarray(ts[:, libs].T)).cuda()
    y = ts[:, 41].astype(np.float64)
    for r in (0, 1):
        gt, gl = ccm.crossmap_rho_backward(Y, X, idx, wt, lib_E, [r], [41], torch.ones(1))
        gy = gt[:, 41].double().cpu().numpy()
        gx = gl[r].double().cpu().numpy()
        assert np.all(np.isfinite(gy)) and np.all(np.isfinite(gx))
        assert np.abs(gy).sum() > 0 and np.abs(gx).sum() > 0
        for g, v in ((gy, y), (gx, x.astype(np.float64))):
            r1 = abs(g.sum()) / np.abs(g).sum()
            r2 = abs((v * g).sum()) / np.abs(v * g).sum()
            print(f"E={lib_E[r]}: invariance residuals {r1:.2e} {r2:.2e}")
            assert r1 <= 2e-5 and r2 <= 2e-5


def test_empty_inputs(ccm):
    import torch

    ts = _cuda(synth.make("logistic64").panel)
    _say("empty inputs")
    idx, wt, d2 = ccm.knn(ts, np.zeros(0, np.int32), np.zeros(0, np.int32), k_max=4)
    assert idx.shape == (0, ts.shape[0], 4)
    optE, rho_E = ccm.simplex_optE(ts, np.zeros(0, np.int32), 1, 5, 1, 1)
    assert optE.numel() == 0
    idx, wt, _ = ccm.knn(ts, [0, 1], [2, 3], k_max=4)
    rho = ccm.crossmap_rho(ts, idx, wt, [2, 3], tgt0=10, n_tgt=0)
    assert rho.shape == (2, 0)
    rho = ccm.crossmap_rho(ts, idx, wt, [2, 3], tgt0=10, n_tgt=0, precision=ccm.PRECISION_BF16)
    assert rho.shape == (2, 0)
    torch.cuda.synchronize()
