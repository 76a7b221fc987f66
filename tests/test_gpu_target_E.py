"""GPU-vs-oracle parity of the per-target-E cross-map (the paper's Alg. 2 as printed: every
target is read through the libraries' tables at the target's own E), through the C ABI.

The target E values are seeded inputs (any E per target is a valid input); rho must be
within 1e-5 of the FP64 oracle, and a target whose E has no table gets NaN."""
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


def _check_rho(rho_g, rho_o, label, tol=RHO_TOL):
    assert np.array_equal(np.isnan(rho_g), np.isnan(rho_o)), f"{label}: NaN pattern differs"
    d = np.abs(rho_g.astype(np.float64) - rho_o)[~np.isnan(rho_o)]
    print(f"{label}: |drho| max {d.max():.3e} median {np.median(d):.3e}")
    assert d.max() < tol, f"{label}: max |drho| {d.max()}"


def test_target_E_logistic64(ccm):
    w = synth.make("logistic64")
    ts = w.panel
    lib_ids = np.arange(0, 64, 4, dtype=np.int32)          # 16 libraries
    tgt_E = np.random.default_rng(31).integers(1, 11, size=64).astype(np.int32)
    _say("target-E logistic64 16 libs x 64 targets, E 1..10")
    idx, wt, _ = ccm.knn_all_E(_cuda(ts), lib_ids, 1, 10, k_max=11)
    rho = ccm.crossmap_rho_target_E(_cuda(ts), idx, wt, len(lib_ids), tgt_E, E_lo=1).cpu().numpy()
    rho_o = O.crossmap_rho_target_E(ts, lib_ids, tgt_E, 1, 0, 64, k_max=11)
    _check_rho(rho, rho_o, "target-E logistic64")


def test_target_E_tau2(ccm):
    # lag tau = 2: each (library, E) table embeds with lags 0, 2, .., 2(E-1), and target j's
    # prediction rows start at (E_j - 1) * 2
    w = synth.make("logistic64")
    ts = w.panel
    lib_ids = np.array([1, 9, 30, 57], dtype=np.int32)
    tgt_E = np.random.default_rng(32).integers(2, 9, size=40).astype(np.int32)
    _say("target-E logistic64 tau=2, 4 libs x 40 targets, E 2..8")
    idx, wt, _ = ccm.knn_all_E(_cuda(ts), lib_ids, 2, 7, tau=2, k_max=9)
    rho = ccm.crossmap_rho_target_E(_cuda(ts), idx, wt, len(lib_ids), tgt_E, E_lo=2, tau=2,
                                    tgt0=5, n_tgt=40).cpu().numpy()
    rho_o = O.crossmap_rho_target_E(ts, lib_ids, tgt_E, 2, 5, 40, k_max=9)
    _check_rho(rho, rho_o, "target-E tau=2")


def test_target_E_ratenet_ragged_and_missing_E(ccm):
    w = synth.make("ratenet1024")
    ts = w.panel
    lib_ids = np.array([3, 200, 517, 1000], dtype=np.int32)
    tgt0, n_tgt = 37, 203                                     # ragged tiles in every bucket
    rng = np.random.default_rng(32)
    tgt_E = rng.integers(3, 11, size=n_tgt).astype(np.int32)
    tgt_E[[5, 77, 150]] = [1, 15, 0]                          # no table at these E: NaN
    _say("target-E ratenet1024 4 libs x 203 targets, tables E 3..10")
    idx, wt, _ = ccm.knn_all_E(_cuda(ts), lib_ids, 3, 8, k_max=11)
    rho, mom = ccm.crossmap_rho_target_E(_cuda(ts), idx, wt, len(lib_ids), tgt_E, E_lo=3,
                                         tgt0=tgt0, n_tgt=n_tgt, want_moments=True)
    rho = rho.cpu().numpy()
    ok = (tgt_E >= 3) & (tgt_E <= 10)
    assert np.all(np.isnan(rho[:, ~ok]))
    assert np.all(np.isnan(mom.cpu().numpy()[:, ~ok]))
    cols = np.nonzero(ok)[0]
    sub = np.ascontiguousarray(ts[:, tgt0 + cols])
    # the oracle reads the libraries from the same panel as the targets: give it both
    panel = np.concatenate([ts[:, lib_ids], sub], axis=1)
    rho_o = O.crossmap_rho_target_E(panel, list(range(len(lib_ids))), tgt_E[cols], 1,
                                    len(lib_ids), len(cols), k_max=11)
    _check_rho(rho[:, cols], rho_o, "target-E ratenet1024")


def test_target_E_single_E_equals_library_E_form(ccm):
    w = synth.make("ratenet1024")
    ts = _cuda(w.panel)
    lib_ids = np.arange(10, 1024, 97, dtype=np.int32)        # 11 libraries
    E = 7
    _say("target-E single E vs library-E form, ratenet1024")
    idx, wt, _ = ccm.knn_all_E(ts, lib_ids, E, 1, k_max=21)
    rho_t = ccm.crossmap_rho_target_E(ts, idx, wt, len(lib_ids), np.full(300, E, np.int32),
                                      E_lo=E, tgt0=100, n_tgt=300)
    rho_l = ccm.crossmap_rho(ts, idx, wt, np.full(len(lib_ids), E, np.int32), tgt0=100,
                             n_tgt=300)
    # same tables, same kernel, same column order: identical bits
    assert np.array_equal(rho_t.cpu().numpy(), rho_l.cpu().numpy(), equal_nan=True)
