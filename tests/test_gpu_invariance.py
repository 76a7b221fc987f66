"""Invariances of the cross-map on the HIP path (the corrcoef of Sec. III-A / III-B).

Pearson's rho is unchanged when a target is replaced by a*y + b (a != 0: the prediction
becomes a*yhat + b because the weights sum to one), so the GPU's rho on a shifted and scaled
target panel must match the FP64 oracle on that same panel to the usual tolerances, however
large the offset b.  Negating a library, or scaling it by a power of two, changes every
distance by an exact factor, so the GPU's neighbour tables must stay bit-identical.
Duplicate target columns give identical rho columns, and permuting the targets permutes the
columns."""
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5
BF16_TOL = 5e-3


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
    print(f"{label}: |drho| max {d.max():.3e} p99 {np.quantile(d, 0.99):.3e} "
          f"median {np.median(d):.3e}")
    assert d.max() < tol, f"{label}: max |drho| {d.max()}"


def _affine(ts, n_tgt, a, b):
    """Targets 0..n_tgt-1 replaced by a*y + b, computed and rounded in FP32."""
    out = ts.copy()
    out[:, :n_tgt] = np.float32(a) * ts[:, :n_tgt] + np.float32(b)
    return out


def test_target_shift_and_scale(ccm):
    w = synth.make("ratenet1024")           # z-scored: sigma = 1 for every series
    ts = w.panel
    lib_ids = np.arange(0, 1024, 64, dtype=np.int32)          # 16 libraries
    lib_E = (np.arange(16) * 7 % 20 + 1).astype(np.int32)     # E = 1..20 mixed
    n_tgt = 300                                                # ragged last tile
    _say("invariance: tables of 16 ratenet1024 libraries")
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=21)
    idx_o, w_o, _ = O.knn(ts, lib_ids, lib_E, 1, 0, 21)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    for b in (100.0, 1000.0):
        Yb = _affine(ts, n_tgt, -2.5, b)
        rho_o = O.crossmap_rho(Yb, idx_o, w_o, lib_E, 1, 0, n_tgt)
        _say(f"invariance: targets -2.5 y + {b:g}, FP32 and BF16")
        rho, mom = ccm.crossmap_rho(_cuda(Yb), idx, wt, lib_E, tgt0=0, n_tgt=n_tgt,
                                    want_moments=True)
        _check_rho(rho.cpu().numpy(), rho_o, f"FP32 b={b:g}", RHO_TOL)
        r16 = ccm.crossmap_rho(_cuda(Yb), idx, wt, lib_E, tgt0=0, n_tgt=n_tgt,
                               precision=ccm.PRECISION_BF16)
        _check_rho(r16.cpu().numpy(), rho_o, f"BF16 b={b:g}", BF16_TOL)
        # the moments stay those of the unshifted values
        i, j = 5, 123
        E = int(lib_E[i])
        Q = np.arange(E - 1, ts.shape[0])
        y = Yb[:, j].astype(np.float64)
        yhat = np.sum(w_o[i][Q, : E + 1] * y[idx_o[i][Q, : E + 1]], axis=1)
        np.testing.assert_allclose(mom.cpu().numpy()[i, j],
                                   [yhat.sum(), (yhat * yhat).sum(), (y[Q] * yhat).sum()],
                                   rtol=1e-6)


def test_target_shift_per_target_E_and_long_series(ccm):
    rng = np.random.default_rng(61)
    # per-target-E form (tables at E = 3..5) on a shifted panel
    w = synth.make("ratenet1024")
    ts = w.panel
    lib_ids = np.array([11, 400, 901], dtype=np.int32)
    n_tgt = 200
    tgt_E = rng.integers(3, 6, size=n_tgt).astype(np.int32)
    Yb = _affine(ts, n_tgt, 3.0, -1000.0)
    _say("invariance: per-target-E form, targets 3 y - 1000")
    idx, wt, _ = ccm.knn_all_E(_cuda(ts), lib_ids, 3, 3, k_max=21)
    rho = ccm.crossmap_rho_target_E(_cuda(Yb), idx, wt, 3, tgt_E, E_lo=3, tgt0=0,
                                    n_tgt=n_tgt).cpu().numpy()
    # the oracle builds its tables from the panel it is given: give it the libraries'
    # original columns beside the shifted targets
    panel = np.concatenate([Yb[:, :n_tgt], ts[:, lib_ids]], axis=1)
    lib_cols = np.arange(n_tgt, n_tgt + 3, dtype=np.int32)
    rho_o = O.crossmap_rho_target_E(panel, lib_cols, tgt_E, 1, 0, n_tgt, k_max=21)
    _check_rho(rho, rho_o, "per-target E, 3 y - 1000", RHO_TOL)

    # series longer than the 16-target LDS tile: the 8-target LDS tile and the global tile
    # copy are centred the same way
    L = 3000
    x = np.cumsum(rng.standard_normal((L, 40)), axis=0)
    x = ((x - x.mean(0)) / x.std(0)).astype(np.float32)
    lib_ids, lib_E = [0, 7, 33], np.array([2, 7, 20], dtype=np.int32)
    Xb = _affine(x, 40, -2.5, 1000.0)
    _say("invariance: L = 3000 (8-target and global tiles), targets -2.5 y + 1000")
    idx, wt, _ = ccm.knn(_cuda(x), lib_ids, lib_E, k_max=21)
    idx_o, w_o, _ = O.knn(x, lib_ids, lib_E, 1, 0, 21)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    rho_o = O.crossmap_rho(Xb, idx_o, w_o, lib_E, 1, 3, 37)
    try:
        for tj in (0, 32):
            ccm.set_gather_tile(tj)
            rho = ccm.crossmap_rho(_cuda(Xb), idx, wt, lib_E, tgt0=3, n_tgt=37).cpu().numpy()
            _check_rho(rho, rho_o, f"L=3000 FP32 tile {tj or 8}, -2.5 y + 1000", RHO_TOL)
    finally:
        ccm.set_gather_tile(0)
    r16 = ccm.crossmap_rho(_cuda(Xb), idx, wt, lib_E, tgt0=3, n_tgt=37,
                           precision=ccm.PRECISION_BF16).cpu().numpy()
    _check_rho(r16, rho_o, "L=3000 BF16, -2.5 y + 1000", BF16_TOL)


def test_library_sign_and_power_of_two_scale(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    lib_ids = np.arange(3, 1024, 97, dtype=np.int32)          # 11 libraries
    lib_E = (np.arange(11) * 3 % 20 + 1).astype(np.int32)
    _say("invariance: library tables under x -> -x and x -> 8 x")
    idx, wt, d2 = (a.cpu().numpy() for a in ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=21))
    for f, s2 in ((-1.0, 1.0), (8.0, 64.0), (0.25, 0.0625)):
        t2 = (np.float32(f) * ts).astype(np.float32)
        i2, w2, d22 = (a.cpu().numpy() for a in ccm.knn(_cuda(t2), lib_ids, lib_E, k_max=21))
        assert np.array_equal(i2, idx), f"indices change under x -> {f} x"
        assert np.array_equal(w2, wt), f"weights change under x -> {f} x"
        valid = idx >= 0
        assert np.array_equal(d22[valid], (d2[valid] * np.float32(s2)).astype(np.float32))
    _say("invariance: optE under x -> -x and x -> 8 x")
    ids = np.arange(0, 1024, 128, dtype=np.int32)
    e0, r0 = (a.cpu().numpy() for a in ccm.simplex_optE(_cuda(ts), ids, 1, 20, 1, 1))
    for f in (-1.0, 8.0):
        t2 = (np.float32(f) * ts).astype(np.float32)
        e2, r2 = (a.cpu().numpy() for a in ccm.simplex_optE(_cuda(t2), ids, 1, 20, 1, 1))
        assert np.array_equal(e2, e0)
        assert np.nanmax(np.abs(r2.astype(np.float64) - r0)) < 1e-6


def test_duplicate_and_permuted_targets(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    rng = np.random.default_rng(77)
    lib_ids = np.arange(1, 1024, 113, dtype=np.int32)         # 10 libraries
    lib_E = (np.arange(10) * 9 % 20 + 1).astype(np.int32)
    idx, wt, _ = ccm.knn(_cuda(ts), lib_ids, lib_E, k_max=21)
    n_tgt = 250
    cols = rng.integers(0, n_tgt, size=n_tgt)                  # a permutation with repeats
    assert len(np.unique(cols)) < n_tgt
    _say("invariance: duplicated and permuted target columns")
    for prec, exact in ((ccm.PRECISION_FP32, True), (ccm.PRECISION_BF16, False)):
        base = ccm.crossmap_rho(_cuda(ts), idx, wt, lib_E, tgt0=0, n_tgt=n_tgt,
                                precision=prec).cpu().numpy()
        perm = ccm.crossmap_rho(_cuda(ts[:, cols]), idx, wt, lib_E, tgt0=0, n_tgt=n_tgt,
                                precision=prec).cpu().numpy()
        if exact:
            assert np.array_equal(perm, base[:, cols])
        else:
            assert np.nanmax(np.abs(perm - base[:, cols])) < 1e-6
