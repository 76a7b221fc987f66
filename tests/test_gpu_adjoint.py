"""GPU adjoint (ccm_crossmap_rho_backward through torch.autograd) against the FP64 oracle
gradient, on the 2048-series coupled logistic network with 256 random pairs, plus the exact
invariances of the gradients on subsampled and padded tables."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_adjoint_matches_fp64_oracle_logistic2048(ccm):
    import torch

    w = synth.make("logistic2048")
    ts = w.panel
    L, N = ts.shape
    pairs = w.pairs
    libs, lib_row = np.unique(pairs[:, 0], return_inverse=True)
    lib_row = lib_row.astype(np.int32)
    # any E per library is a valid input of the adjoint: a seeded draw feeds both sides
    lib_E = np.random.default_rng(44).integers(2, 9, size=len(libs)).astype(np.int32)
    optE = torch.as_tensor(lib_E).cuda()
    Y = torch.as_tensor(ts).cuda()
    X = torch.as_tensor(np.ascontiguousarray(ts[:, libs].T)).cuda().requires_grad_(True)
    Yg = Y.clone().requires_grad_(True)
    _say("adjoint: forward + backward")
    rho = ccm.crossmap_rho_autograd(X, Yg, optE)
    sel = torch.zeros_like(rho)
    sel[torch.as_tensor(lib_row).long().cuda(), torch.as_tensor(pairs[:, 1]).long().cuda()] = 1.0
    loss = (rho * sel).sum()
    loss.backward()
    gX = X.grad.cpu().numpy().astype(np.float64)
    gY = Yg.grad.cpu().numpy().astype(np.float64)
    # oracle: same tables (bit-exact), FP64 gradient
    idx_o, w_o, _ = O.knn(ts, libs, lib_E, 1, 0, int(lib_E.max()) + 1)
    opairs = np.stack([lib_row, pairs[:, 1]], axis=1)
    g_tgt, g_lib = O.crossmap_rho_grad(ts, libs, lib_E, idx_o, 1, opairs, np.ones(len(pairs)))
    rt, rl = _rel(gY, g_tgt), _rel(gX, g_lib)
    print(f"adjoint rel L2 error: targets {rt:.2e}, libraries {rl:.2e}")
    assert rt < 1e-3 and rl < 1e-3
    # invariants: rho is unchanged by y -> a y + b and by x -> a x + b
    cols = np.unique(pairs[:, 1])
    scale_t = np.abs(gY[:, cols]).sum(axis=0) + 1e-30
    assert np.max(np.abs(gY[:, cols].sum(axis=0)) / scale_t) < 1e-4
    scale_l = np.abs(gX).sum(axis=1) + 1e-30
    assert np.max(np.abs(gX.sum(axis=1)) / scale_l) < 1e-4


def test_adjoint_zero_and_nan_pairs(ccm):
    import torch

    rng = np.random.default_rng(3)
    ts = rng.standard_normal((200, 6)).astype(np.float32)
    ts[:, 5] = 1.0  # constant target: rho NaN, contributes no gradient
    X = torch.as_tensor(np.ascontiguousarray(ts[:, :2].T)).cuda().requires_grad_(True)
    Y = torch.as_tensor(ts).cuda().requires_grad_(True)
    _say("adjoint: NaN pair")
    rho = ccm.crossmap_rho_autograd(X, Y, [3, 2])
    assert torch.isnan(rho[:, 5]).all()
    g = torch.zeros_like(rho)
    g[0, 5] = 1.0
    g[1, 2] = 1.0
    rho.backward(g)
    assert torch.all(Y.grad[:, 5] == 0)
    assert torch.isfinite(Y.grad).all() and torch.isfinite(X.grad).all()
    assert Y.grad[:, 2].abs().sum() > 0 and X.grad[1].abs().sum() > 0 and X.grad[0].abs().sum() == 0


def _check_invariances(gy, gx, y, x):
    assert np.all(np.isfinite(gy)) and np.all(np.isfinite(gx))
    assert abs(gy.sum()) <= 1e-5 * np.abs(gy).sum()
    assert abs((y * gy).sum()) <= 1e-5 * np.abs(y * gy).sum()
    if np.abs(gx).sum() > 0:
        assert abs(gx.sum()) <= 1e-5 * np.abs(gx).sum()
        assert abs((x * gx).sum()) <= 1e-5 * np.abs(x * gx).sum()


def test_adjoint_subsampled_and_padded_tables(ccm):
    # Whatever the table, rho is invariant to y -> a y + b and, through d / d_1, to
    # x -> a x + b, so each pair's gradients obey sum_s g(s) = 0 and sum_s v(s) g(s) = 0
    # exactly (P11, P12).  Checked on tables of library subsamples (one library with too
    # few marked points is unusable: NaN and no gradient) and on a table whose rows lose
    # their farthest entry to padding (-1, weight 0, the rest renormalised), which both
    # directions treat as absent.
    import torch

    w = synth.make("logistic64")
    ts = w.panel
    L = ts.shape[0]
    libs = np.array([3, 17, 40], dtype=np.int32)
    lib_E = np.array([3, 2, 4], dtype=np.int32)
    rng = np.random.default_rng(46)
    mask = np.zeros((len(libs), L), dtype=np.uint8)
    for r, n_keep in enumerate([4, 60, 9]):     # library 0: 4 points < k + 1 = 5
        mask[r, rng.choice(L, size=n_keep, replace=False)] = 1
    Y = torch.as_tensor(ts).cuda()
    X = torch.as_tensor(np.ascontiguousarray(ts[:, libs].T)).cuda()
    _say("adjoint on subsampled tables")
    idx, wt, _ = ccm.knn(Y, libs, lib_E, k_max=5, cand_mask=torch.as_tensor(mask).cuda())
    assert bool((idx[0] < 0).all())
    rho = ccm.crossmap_rho(Y, idx, wt, lib_E).cpu().numpy()
    assert np.all(np.isnan(rho[0]))
    for r in range(len(libs)):
        for j in (5, 33):
            gt, gl = ccm.crossmap_rho_backward(Y, X, idx, wt, lib_E, [r], [j], torch.ones(1))
            gy = gt[:, j].double().cpu().numpy()
            gx = gl[r].double().cpu().numpy()
            if r == 0:
                assert not gy.any() and not gx.any()
                continue
            _check_invariances(gy, gx, ts[:, j].astype(np.float64),
                               ts[:, libs[r]].astype(np.float64))
    _say("adjoint on a table with padding entries")
    idx, wt, _ = ccm.knn(Y, libs, lib_E, k_max=5)
    rows = torch.arange(10, L, 7, device="cuda")
    for r in range(len(libs)):
        idx[r, rows, int(lib_E[r])] = -1                # the k-th (farthest) entry
        wt[r, rows, int(lib_E[r])] = 0.0
        # weights of the remaining entries sum to 1 again, so y -> a y + b stays exact
        wt[r, rows] = wt[r, rows] / wt[r, rows].sum(dim=1, keepdim=True)
    for r in range(len(libs)):
        gt, gl = ccm.crossmap_rho_backward(Y, X, idx, wt, lib_E, [r], [21], torch.ones(1))
        _check_invariances(gt[:, 21].double().cpu().numpy(), gl[r].double().cpu().numpy(),
                           ts[:, 21].astype(np.float64), ts[:, libs[r]].astype(np.float64))


def test_adjoint_tau2_against_oracle(ccm):
    # lag tau = 2 through the whole adjoint (distances over lags 0, 2, .., the scatter of a
    # point's lag coordinates back to the series), against the FP64 oracle gradient
    import torch

    w = synth.make("logistic64")
    ts = w.panel
    L, N = ts.shape
    libs = np.array([2, 11, 40, 63], dtype=np.int32)
    lib_E = np.array([2, 3, 4, 5], dtype=np.int32)
    rng = np.random.default_rng(48)
    pairs = np.stack([rng.integers(0, 4, 12), rng.integers(0, N, 12)], axis=1).astype(np.int32)
    Y = torch.as_tensor(ts).cuda()
    X = torch.as_tensor(np.ascontiguousarray(ts[:, libs].T)).cuda()
    _say("adjoint tau=2, 4 libraries, 12 pairs")
    idx, wt, _ = ccm.knn(Y, libs, lib_E, tau=2, k_max=6)
    gt, gl = ccm.crossmap_rho_backward(Y, X, idx, wt, lib_E, pairs[:, 0], pairs[:, 1],
                                       torch.ones(len(pairs)), tau=2)
    idx_o, _, _ = O.knn(ts, libs, lib_E, 2, 0, 6)
    assert np.array_equal(idx.cpu().numpy(), idx_o)
    g_tgt, g_lib = O.crossmap_rho_grad(ts, libs, lib_E, idx_o, 2, pairs, np.ones(len(pairs)))
    rt = _rel(gt.cpu().numpy().astype(np.float64), g_tgt)
    rl = _rel(gl.cpu().numpy().astype(np.float64), g_lib)
    print(f"adjoint tau=2 rel L2 error: targets {rt:.2e}, libraries {rl:.2e}")
    assert rt < 1e-3 and rl < 1e-3


def test_adjoint_through_a_column_slice_of_a_wider_panel(ccm):
    # Y is an [L][N] view of an [L][N + 16] panel (row stride > N, storage offset 5): the
    # backward must write the target gradient at Y's strides, inside Y's columns only
    import torch

    w = synth.make("logistic64")
    ts = w.panel
    L, N = ts.shape
    libs = np.array([3, 17, 40], dtype=np.int32)
    lib_E = np.array([3, 2, 4], dtype=np.int32)
    wide_np = np.full((L, N + 16), 7.0, dtype=np.float32)
    wide_np[:, 5:5 + N] = ts
    wide = torch.as_tensor(wide_np).cuda().requires_grad_(True)
    Y = wide[:, 5:5 + N]
    assert Y.stride(0) == N + 16 and not Y.is_contiguous()
    X = torch.as_tensor(np.ascontiguousarray(ts[:, libs].T)).cuda().requires_grad_(True)
    _say("adjoint through a strided target view")
    rho = ccm.crossmap_rho_autograd(X, Y, lib_E)
    rng = np.random.default_rng(52)
    g = np.zeros((len(libs), N), dtype=np.float32)
    pick = rng.choice(len(libs) * N, 10, replace=False)
    g.flat[pick] = rng.standard_normal(10).astype(np.float32)
    (rho * torch.as_tensor(g).cuda()).sum().backward()
    gw = wide.grad.cpu().numpy().astype(np.float64)
    assert not gw[:, :5].any() and not gw[:, 5 + N:].any()
    idx_o, _, _ = O.knn(ts, libs, lib_E, 1, 0, int(lib_E.max()) + 1)
    r_i, r_j = np.nonzero(g)
    pairs = np.stack([r_i, r_j], axis=1).astype(np.int32)
    g_tgt, g_lib = O.crossmap_rho_grad(ts, libs, lib_E, idx_o, 1, pairs, g[r_i, r_j])
    rt = _rel(gw[:, 5:5 + N], g_tgt)
    rl = _rel(X.grad.cpu().numpy().astype(np.float64), g_lib)
    print(f"strided view: rel L2 error targets {rt:.2e}, libraries {rl:.2e}")
    assert rt < 1e-3 and rl < 1e-3
    # a caller's gradient buffer must carry the panel's strides
    idx, wt, _ = ccm.knn(Y.detach(), libs, lib_E, k_max=5)
    with pytest.raises(ValueError):
        ccm.crossmap_rho_backward(Y.detach(), X.detach(), idx, wt, lib_E, [0], [1], torch.ones(1),
                                  grad_ts=torch.zeros((L, N), device="cuda"))
    with pytest.raises(ValueError):
        ccm.crossmap_rho_backward(Y.detach(), X.detach(), idx, wt, lib_E, [0], [N], torch.ones(1))
