"""Pins for the CPU oracle: each test checks it against something other than itself --
hand-derived values, exact arithmetic, brute force, closed forms, invariants, a library
routine, or a finite difference -- so that a dropped term, a wrong sign, a wrong lag or a
transposed operand fails at least one of them."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- embedding (Sec. II-B) --------------------------------------------------------------
def test_embed_closed_form():
    x = np.arange(10, 17, dtype=np.float32)  # x(t) = 10 + t, L = 7
    got = O.embed(x, E=3, tau=2)
    # points t = 4, 5, 6; coordinates x(t), x(t-2), x(t-4)
    want = np.array([[14, 12, 10], [15, 13, 11], [16, 14, 12]], dtype=np.float32)
    assert np.array_equal(got, want)
    assert O.embed(x, E=1, tau=1).ravel().tolist() == x.tolist()
    assert O.embed(x, E=8, tau=1).shape == (0, 8)


# --- canonical FP32 squared distance -------------------------------------------------
def test_sqdist_exact_on_small_integers():
    # Small integers: every FP32 operation is exact, so d^2 must equal the exact sum.
    rng = np.random.default_rng(0)
    x = rng.integers(-20, 21, size=40).astype(np.float32)
    for E, tau in [(1, 1), (3, 1), (4, 2), (7, 3)]:
        Q, C, _ = O.point_sets(40, E, tau, 0)
        D2 = O.sqdist_fp32(x, Q, C, E, tau)
        xi = [int(v) for v in x]
        for a, t in enumerate(Q[::3]):
            for b, s in enumerate(C[::5]):
                exact = sum((xi[t - e * tau] - xi[s - e * tau]) ** 2 for e in range(E))
                assert D2[3 * a, 5 * b] == exact


def test_sqdist_order_lag0_first_no_fma():
    # delta_0 = 1, delta_1 = delta_2 = 2^-12.  Lag 0 first: fl(1 + 2^-24) = 1 twice -> 1.
    # (Lag E-1 first would give 1 + 2^-23; a fused multiply-add would keep 2^-24 terms.)
    h = np.float32(2.0 ** -12)
    x_t = np.array([0.0, 0.0, 0.0], dtype=np.float32)  # x(t-2), x(t-1), x(t)
    x_s = np.array([-h, -h, -1.0], dtype=np.float32)   # x(s-2), x(s-1), x(s)
    x = np.concatenate([x_s, x_t])                     # s = 2, t = 5
    D2 = O.sqdist_fp32(x, [5], [2], E=3, tau=1)
    assert D2[0, 0] == np.float32(1.0)


def test_sqdist_within_rounding_bound():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(60).astype(np.float32)
    E = 6
    Q, C, _ = O.point_sets(60, E, 1, 0)
    D2 = O.sqdist_fp32(x, Q, C, E, 1)
    u = 2.0 ** -24
    for a in range(0, len(Q), 7):
        for b in range(0, len(C), 5):
            t, s = Q[a], C[b]
            ex = sum((Fraction(float(x[t - e])) - Fraction(float(x[s - e]))) ** 2 for e in range(E))
            # each of E subtractions, E products, E-1 additions rounds once
            assert abs(Fraction(float(D2[a, b])) - ex) <= Fraction((3 * E + 1) * u) * ex + Fraction(0)


# --- neighbour selection (Alg. 3 / Alg. 4) ----------------------------------------------
def _brute_knn(xi, E, tau, Tp, k):
    """Pure-Python exact brute force on integer series: sort (d^2, s) tuples."""
    L = len(xi)
    lo = (E - 1) * tau
    Q = list(range(lo, L - Tp))
    out = {}
    for t in Q:
        cand = []
        for s in Q:
            if s == t:
                continue
            d2 = sum((xi[t - e * tau] - xi[s - e * tau]) ** 2 for e in range(E))
            cand.append((d2, s))
        cand.sort()
        out[t] = [s for _, s in cand[:k]]
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_knn_matches_brute_force_with_ties(seed):
    rng = np.random.default_rng(seed)
    L = 48
    # a few distinct small integers: many exact ties and zero distances
    xi = rng.integers(0, 4, size=L).tolist()
    x = np.array(xi, dtype=np.float32)
    for E in (1, 2, 3, 5):
        for tau in (1, 2):
            for Tp in (0, 1):
                Q, idx, w, d2 = O.knn_table(x, E, tau, Tp)
                bf = _brute_knn(xi, E, tau, Tp, E + 1)
                for r, t in enumerate(Q):
                    assert idx[r].tolist() == bf[int(t)], (E, tau, Tp, t)


def test_knn_sets_match_kdtree_away_from_near_ties():
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(7)
    x = rng.standard_normal(300).astype(np.float32)
    for E in (2, 4, 7):
        Q, idx, w, d2 = O.knn_table(x, E, 1, 0)
        V = O.embed(x.astype(np.float64), E, 1)
        tree = cKDTree(V)
        dist, nb = tree.query(V, k=E + 3)
        checked = 0
        for r in range(len(Q)):
            nbr = [int(n) for n in nb[r] if n != r][: E + 2]
            dd = [float(dv) for n, dv in zip(nb[r], dist[r]) if n != r][: E + 2]
            if dd[E + 1] - dd[E] < 1e-5 * max(dd[E], 1e-30):
                continue  # k-th and (k+1)-th too close to call in FP32
            assert set((np.array(nbr[: E + 1]) + E - 1).tolist()) == set(idx[r].tolist())
            checked += 1
        assert checked > 0.9 * len(Q)


def test_knn_rejects_k_beyond_candidates():
    x = np.arange(6, dtype=np.float32)
    with pytest.raises(ValueError):
        O.knn_table(x, 5, 1, 0)  # 2 points, k = 6


def test_knn_invariant_under_exact_transforms():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(200).astype(np.float32)
    for E in (1, 3, 6):
        _, i0, _, _ = O.knn_table(x, E, 1, 0)
        _, i1, _, _ = O.knn_table(-x, E, 1, 0)
        _, i2, _, _ = O.knn_table(x * np.float32(8.0), E, 1, 0)
        _, i3, _, _ = O.knn_table(x * np.float32(2.0 ** -5), E, 1, 0)
        assert np.array_equal(i0, i1) and np.array_equal(i0, i2) and np.array_equal(i0, i3)


# --- weights (Sec. III-A "normalize") --------------------------------------------------
def test_weights_hand_worked():
    with open(os.path.join(GOLDEN, "hand_worked_L5.json")) as f:
        g = json.load(f)
    x = np.array(g["x"], dtype=np.float32)
    Q, idx, w, d2 = O.knn_table(x, g["E"], g["tau"], g["Tp"])
    for row in g["rows"]:
        r = list(Q).index(row["t"])
        assert idx[r].tolist() == row["nbr"]
        want = [eval(expr, {"exp": math.exp}) for expr in row["w"]]
        np.testing.assert_allclose(w[r], want, rtol=0, atol=1e-15)


def test_weights_equal_distances_uniform():
    x = np.array([0, 1, -1, 2, -2, 1, -1], dtype=np.float32)
    w = O.weights_fp64(x, 0, [1, 2, 5], 1, 1)
    np.testing.assert_allclose(w, [1 / 3, 1 / 3, 1 / 3], atol=1e-15)


def test_weights_zero_distance_limit():
    x = np.array([0, 5, 0, 5, 1, 0], dtype=np.float32)
    w = O.weights_fp64(x, 0, [2, 5, 4], 1, 1)  # d = 0, 0, 1
    np.testing.assert_array_equal(w, [0.5, 0.5, 0.0])
    assert np.all(np.isfinite(w))


# --- Pearson --------------------------------------------------------------------------
def test_pearson_closed_forms_and_library():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(500)
    b = 0.3 * a + rng.standard_normal(500)
    assert abs(O.pearson(a, b) - np.corrcoef(a, b)[0, 1]) < 1e-13
    assert abs(O.pearson(a, 2 * a + 1) - 1.0) < 1e-14
    assert abs(O.pearson(a, -a) + 1.0) < 1e-14
    assert math.isnan(O.pearson(a, np.full(500, 3.0)))
    assert math.isnan(O.pearson(np.ones(4), a[:4]))


# --- whole cross-map ------------------------------------------------------------------
def test_periodic_series_cross_map_exactly():
    rng = np.random.default_rng(11)
    L, P = 140, 7
    x = synth.periodic(P, L, rng)
    tab2 = rng.standard_normal(P).astype(np.float32)
    y = tab2[np.arange(L) % P]                        # any function of phase
    ts = np.stack([x, y, rng.standard_normal(L).astype(np.float32)], axis=1)
    rho, idx, w, d2 = O.ccm_block(ts, [0], [2], 1, 0, 3)
    assert abs(rho[0, 0] - 1.0) < 1e-12
    assert abs(rho[0, 1] - 1.0) < 1e-12
    assert rho[0, 2] < 0.9


def test_target_affine_invariance_and_columns():
    w = synth.make("logistic64", cache=False)
    ts = w.panel
    lib = [0, 5, 9]
    E = [3, 4, 2]
    rho, idx, wt, d2 = O.ccm_block(ts, lib, E, 1, 0, 8)
    ts2 = ts.astype(np.float64).copy()
    ts2[:, 3] = -2.5 * ts2[:, 3] + 7.0
    rho2 = O.crossmap_rho(ts2, idx, wt, E, 1, 0, 8)
    # both the observed y and the prediction (weights sum to 1) map through a y + b
    np.testing.assert_allclose(rho2[:, 3], rho[:, 3], atol=1e-12)
    np.testing.assert_allclose(np.delete(rho2, 3, 1), np.delete(rho, 3, 1), atol=0)
    # duplicate and permuted targets
    perm = [4, 4, 0, 7, 1]
    ts3 = ts[:, perm]
    rho3 = O.crossmap_rho(ts3, idx, wt, E, 1, 0, 5)
    np.testing.assert_array_equal(rho3, rho[:, perm])


def test_reuse_equals_per_pair_recompute():
    """Alg. 2's one-table-per-library reuse gives exactly Alg. 1's per-pair result."""
    w = synth.make("logistic64", cache=False)
    ts = w.panel[:200, :6]
    lib_E = [2, 3, 4, 3, 5, 2]
    rho, idx, wt, d2 = O.ccm_block(ts, list(range(6)), lib_E, 1, 0, 6)
    for i in range(6):
        for j in range(6):
            Q, ii, ww, _ = O.knn_table(ts[:, i], lib_E[i], 1, 0)  # rebuilt for this pair
            y = ts[:, j].astype(np.float64)
            r = O.pearson(y[Q], np.sum(ww * y[ii], axis=1))
            assert r == rho[i, j]


def test_self_cross_map_is_simplex_at_tp0():
    w = synth.make("logistic64", cache=False)
    ts = w.panel[:, :4]
    lib_E = [2, 3, 5, 1]
    rho, *_ = O.ccm_block(ts, list(range(4)), lib_E, 1, 0, 4)
    for i in range(4):
        assert abs(O.simplex_rho(ts[:, i], lib_E[i], 1, 0) - rho[i, i]) < 1e-14


def test_optE_argmax_and_ties():
    w = synth.make("logistic64", cache=False)
    ts = w.panel[:300, :3]
    optE, rho, nanf = O.simplex_optE(ts, [0, 1, 2], 1, 6, 1, 1)
    for i in range(3):
        best = np.nanmax(rho[i])
        assert optE[i] == 1 + int(np.nonzero(rho[i] == best)[0][0])
        assert not nanf[i]
    # constant series: every skill is NaN -> E_min, flagged
    c = np.ones((50, 1), dtype=np.float32)
    o, r, f = O.simplex_optE(c, [0], 2, 4, 1, 1)
    assert o[0] == 2 and f[0] and np.all(np.isnan(r))


def test_half_mode_sets():
    Q, C, excl = O.point_sets(20, 3, 1, 1, O.MODE_HALF)
    assert C.tolist() == list(range(2, 9)) and Q.tolist() == list(range(12, 19)) and not excl


def test_coupled_logistic_direction():
    """CCM direction (Sec. II-B): if j drives i, i's manifold recovers j, so
    rho[lib=i, tgt=j] exceeds rho[lib=j, tgt=i] on most one-way edges."""
    from scipy.stats import binomtest

    wins = 0
    total = 0
    for trial in (0, 1):
        w = synth.make("logistic64", trial, cache=False)
        ts = w.panel
        b = w.beta
        optE = np.full(64, 3, dtype=np.int32)
        rho, *_ = O.ccm_block(ts, np.arange(64), optE, 1, 0, 64)
        i, j = np.nonzero((b > 0.05) & (b.T == 0))
        wins += int(np.sum(rho[i, j] > rho[j, i]))
        total += len(i)
    assert binomtest(wins, total, 0.5, alternative="greater").pvalue < 0.01


# --- gradients --------------------------------------------------------------------------
def _rho_fixed(ts64, lib_col, j, idx, E, tau, x_override=None):
    """rho of one pair from oracle pieces with the neighbour sets held fixed."""
    L = ts64.shape[0]
    Q = np.arange((E - 1) * tau, L)
    x = ts64[:, lib_col] if x_override is None else x_override
    w = O.weights_rows_fp64(x, Q, idx, E, tau)
    y = ts64[:, j]
    return O.pearson(y[Q], np.sum(w * y[idx], axis=1))


def test_gradient_invariants_and_finite_differences():
    w = synth.make("logistic64", cache=False)
    ts64 = w.panel[:160, :6].astype(np.float64)
    lib_ids = [1, 4]
    lib_E = [3, 2]
    pairs = np.array([[0, 2], [1, 5], [0, 1]], dtype=np.int32)
    gw = np.array([1.0, -0.5, 2.0])
    idx, wt, d2 = O.knn(ts64.astype(np.float32), lib_ids, lib_E, 1, 0, 4)
    g_tgt, g_lib = O.crossmap_rho_grad(ts64, lib_ids, lib_E, idx, 1, pairs, gw)
    L = ts64.shape[0]
    # target invariants: rho is invariant under y -> a y + b
    for j in (1, 2, 5):
        assert abs(g_tgt[:, j].sum()) < 1e-10
        assert abs(np.dot(g_tgt[:, j], ts64[:, j])) < 1e-10
    # library invariants: weights depend on x only through d_k / d_1
    for i in range(2):
        assert abs(g_lib[i].sum()) < 1e-10
        assert abs(np.dot(g_lib[i], ts64[:, lib_ids[i]])) < 1e-10

    def loss(ts_t, xs):
        tot = 0.0
        for (i, j), g in zip(pairs, gw):
            E = lib_E[i]
            Q = np.arange(E - 1, L)
            tot += g * _rho_fixed(ts_t, lib_ids[i], j, idx[i][Q, : E + 1], E, 1, x_override=xs[i])
        return tot

    xs0 = [ts64[:, c].copy() for c in lib_ids]
    h = 1e-6
    rng = np.random.default_rng(0)
    for s in rng.choice(L, 12, replace=False):
        for j in (2, 5):
            tp = ts64.copy(); tp[s, j] += h
            tm = ts64.copy(); tm[s, j] -= h
            fd = (loss(tp, xs0) - loss(tm, xs0)) / (2 * h)
            assert abs(fd - g_tgt[s, j]) < 1e-6 * max(1.0, abs(g_tgt[s, j]))
        for i in range(2):
            xp = [v.copy() for v in xs0]; xp[i][s] += h
            xm = [v.copy() for v in xs0]; xm[i][s] -= h
            # the perturbation is far too small to change any neighbour set
            for xv in (xp[i], xm[i]):
                E = lib_E[i]
                Q, ii, _, _ = O.knn_table(xv, E, 1, 0)
                assert np.array_equal(ii, idx[i][Q, : E + 1])
            fd = (loss(ts64, xp) - loss(ts64, xm)) / (2 * h)
            assert abs(fd - g_lib[i, s]) < 1e-6 * max(1.0, abs(g_lib[i, s]))


# --- the paper's per-target-E cross-map (Alg. 2 as printed) -------------------------------
def _brute_rho_target_E(xs, lib_cols, tgt_cols, tgt_E):
    """Pure-Python brute force on integer series: for target j, library i's points at E_j
    (Tp = 0, self excluded), the E_j + 1 nearest by exact integer d^2 then time index,
    weights exp(-d/d1) normalised (zero-distance rule when d1 = 0), two-pass Pearson."""
    L = len(xs[0])
    out = []
    for i in lib_cols:
        x = xs[i]
        row = []
        for j, E in zip(tgt_cols, tgt_E):
            y = xs[j]
            Q = list(range(E - 1, L))
            obs, pred = [], []
            for t in Q:
                cand = sorted((sum((x[t - e] - x[s - e]) ** 2 for e in range(E)), s)
                              for s in Q if s != t)[:E + 1]
                d = [math.sqrt(c[0]) for c in cand]
                if d[0] > 0:
                    u = [math.exp(-dk / d[0]) for dk in d]
                else:
                    u = [1.0 if dk == 0 else 0.0 for dk in d]
                pred.append(sum(uk * y[c[1]] for uk, c in zip(u, cand)) / sum(u))
                obs.append(float(y[t]))
            mo, mp = sum(obs) / len(obs), sum(pred) / len(pred)
            so = sum((a - mo) ** 2 for a in obs)
            sp = sum((b - mp) ** 2 for b in pred)
            sop = sum((a - mo) * (b - mp) for a, b in zip(obs, pred))
            row.append(sop / math.sqrt(so * sp) if so > 0 and sp > 0 else float("nan"))
        out.append(row)
    return np.array(out)


def test_target_E_cross_map_matches_brute_force():
    rng = np.random.default_rng(21)
    L, N = 22, 6
    xs = rng.integers(0, 9, size=(N, L)).tolist()
    ts = np.array(xs, dtype=np.float32).T.copy()
    lib = [0, 2, 5]
    tgt_E = [3, 1, 2, 3, 4, 1]          # one E per target column 0..5
    rho = O.crossmap_rho_target_E(ts, lib, tgt_E, 1, 0, N, k_max=5)
    bf = _brute_rho_target_E(xs, lib, list(range(N)), tgt_E)
    np.testing.assert_allclose(rho, bf, rtol=0, atol=1e-12)


def test_target_E_cross_map_periodic_and_columns():
    rng = np.random.default_rng(12)
    L, P = 150, 5
    x = synth.periodic(P, L, rng)
    tab = rng.standard_normal((3, P)).astype(np.float32)
    ph = np.arange(L) % P
    noise = rng.standard_normal(L).astype(np.float32)
    # library 0 is P-periodic; targets 1..3 are functions of its phase, 4 is noise
    ts = np.stack([x, tab[0][ph], tab[1][ph], tab[2][ph], noise], axis=1)
    tgt_E = [2, 4, 1, 3, 2]
    rho = O.crossmap_rho_target_E(ts, [0], tgt_E, 1, 0, 5, k_max=6)
    np.testing.assert_allclose(rho[0, :4], 1.0, atol=1e-12)
    assert rho[0, 4] < 0.9
    # targets permuted together with their E permute the columns; a constant E reduces to
    # the library-E form at that E
    perm = [4, 2, 0, 3, 1]
    ts_p = np.concatenate([ts[:, :1], ts[:, perm]], axis=1)     # library stays column 0
    rho_p = O.crossmap_rho_target_E(ts_p, [0], [tgt_E[c] for c in perm], 1, 1, 5, k_max=6)
    np.testing.assert_array_equal(rho_p, rho[:, perm])
    for E in (1, 3):
        r_const = O.crossmap_rho_target_E(ts, [0, 4], [E] * 5, 1, 0, 5, k_max=6)
        r_lib, _, _, _ = O.ccm_block(ts, [0, 4], [E, E], 1, 0, 5, k_max=6)
        np.testing.assert_array_equal(r_const, r_lib)


# --- the CCM convergence test: tables over random library subsamples ----------------------
def _brute_knn_subset(xi, E, allowed, k):
    """Pure-Python brute force: every point is a query; neighbours come only from the
    allowed time indices (self excluded); exact integer d^2, ties to the lower index."""
    L = len(xi)
    out = {}
    for t in range(E - 1, L):
        cand = sorted((sum((xi[t - e] - xi[s - e]) ** 2 for e in range(E)), s)
                      for s in allowed if s != t and s >= E - 1)
        out[t] = [s for _, s in cand[:k]]
    return out


@pytest.mark.parametrize("seed", [3, 4])
def test_subsampled_knn_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    L = 60
    xi = rng.integers(0, 5, size=L).tolist()
    x = np.array(xi, dtype=np.float32)
    for E in (1, 2, 4):
        for m in (E + 2, 15, 40):
            mask = synth.library_samples(L, E, [m], 1, seed)[0]
            Q, idx, w, d2 = O.knn_table(x, E, 1, 0, cand=mask)
            bf = _brute_knn_subset(xi, E, np.nonzero(mask)[0].tolist(), E + 1)
            assert len(Q) == L - (E - 1)                     # every point is a query
            for r, t in enumerate(Q):
                assert idx[r].tolist() == bf[int(t)], (E, m, t)
                assert all(mask[s] for s in idx[r])


def test_subsample_masks_and_full_library_reduction():
    masks = synth.library_samples(200, 3, [5, 50, 198], 4, 0)
    assert masks.shape == (12, 200)
    assert masks[:, :2].sum() == 0                            # only embedded points
    np.testing.assert_array_equal(masks.sum(axis=1), [5] * 4 + [50] * 4 + [198] * 4)
    assert len({m.tobytes() for m in masks[:4]}) == 4           # distinct draws
    # a mask with every embedded point is the ordinary table and the ordinary rho
    ts = synth.make("logistic64", cache=False).panel[:200]
    full = np.ones((1, 1, 200), dtype=bool)
    r_conv = O.ccm_convergence(ts, [2], [3], full, 1, 0, 10, k_max=4)
    r_blk, _, _, _ = O.ccm_block(ts, [2], [3], 1, 0, 10, k_max=4)
    np.testing.assert_array_equal(r_conv[:, 0, :], r_blk)


def test_convergence_on_two_species():
    """Skill of the driven series' library at recovering its driver rises with library
    size and ends high (the behaviour the CCM convergence test looks for)."""
    ts = synth.two_species(1000, 0)
    sizes = [12, 50, 200, 800]
    masks = synth.library_samples(1000, 2, sizes, 8, 1)
    rho = O.ccm_convergence(ts, [1], [2], masks[None], 1, 0, 1, k_max=3)[0, :, 0]
    curve = rho.reshape(len(sizes), 8).mean(axis=1)
    assert np.all(np.diff(curve) > 0), curve
    assert curve[-1] > 0.9 and curve[-1] - curve[0] > 0.1, curve
    # the driver's library recovers the weakly coupled direction less well at every size
    back = O.ccm_convergence(ts, [0], [2], masks[None], 1, 1, 1, k_max=3)[0, :, 0]
    assert np.all(back.reshape(len(sizes), 8).mean(axis=1) < curve)


# --- simplex skill at horizons Tp >= 1 (Sec. II-B; Alg. 1 phase 1) ------------------------
def _brute_simplex_rho(xi, E, tau, Tp, half):
    """Pure-Python simplex skill on an integer series, from the definition: embed, pick the
    E + 1 nearest library points by exact integer d^2 then time index, forecast x(t + Tp) as
    the weighted mean of the neighbours' own values Tp steps later, and correlate the
    forecasts with what was observed (two-pass Pearson, NaN on a zero variance).
    Leave-one-out: every point with a future is both query and candidate, the query itself
    excluded.  Half split: candidates from the first half, queries from the second, each
    point's window and future inside its own half."""
    L = len(xi)
    span = (E - 1) * tau
    if half:
        h = L // 2
        lib = [s for s in range(L) if s - span >= 0 and s + Tp <= h - 1]
        qry = [t for t in range(L) if t - span >= h and t + Tp <= L - 1]
    else:
        lib = [s for s in range(L) if s - span >= 0 and s + Tp <= L - 1]
        qry = list(lib)
    obs, pred = [], []
    for t in qry:
        near = sorted((sum((xi[t - e * tau] - xi[s - e * tau]) ** 2 for e in range(E)), s)
                      for s in lib if half or s != t)[:E + 1]
        d = [math.sqrt(c[0]) for c in near]
        u = ([math.exp(-dk / d[0]) for dk in d] if d[0] > 0 else
             [1.0 if dk == 0 else 0.0 for dk in d])
        pred.append(sum(uk * xi[c[1] + Tp] for uk, c in zip(u, near)) / sum(u))
        obs.append(float(xi[t + Tp]))
    mo, mp = sum(obs) / len(obs), sum(pred) / len(pred)
    so = sum((a - mo) ** 2 for a in obs)
    sp = sum((b - mp) ** 2 for b in pred)
    if so == 0 or sp == 0:
        return float("nan")
    return sum((a - mo) * (b - mp) for a, b in zip(obs, pred)) / math.sqrt(so * sp)


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("half", [False, True])
def test_simplex_rho_matches_brute_force(seed, half):
    rng = np.random.default_rng(100 + seed)
    L = 44
    # few distinct values: exact ties and zero distances in every list
    xi = rng.integers(0, 6, size=L).tolist()
    x = np.array(xi, dtype=np.float32)
    mode = O.MODE_HALF if half else O.MODE_LOO
    checked = 0
    for Tp in (1, 2, 3):
        for tau in (1, 2):
            for E in (1, 2, 3, 4):
                want = _brute_simplex_rho(xi, E, tau, Tp, half)
                got = O.simplex_rho(x, E, tau, Tp, mode)
                if math.isnan(want):
                    assert math.isnan(got), (E, tau, Tp)
                else:
                    assert abs(got - want) < 1e-12, (E, tau, Tp, got, want)
                    checked += 1
    assert checked >= 20


def test_simplex_rho_sees_the_horizon():
    """Forecasting x(t+Tp) is not forecasting x(t): on a random integer series the skills
    at Tp = 0, 1, 2 all differ, so a dropped or doubled +Tp cannot pass the brute force."""
    rng = np.random.default_rng(7)
    xi = rng.integers(0, 9, size=40).tolist()
    x = np.array(xi, dtype=np.float32)
    r = [O.simplex_rho(x, 2, 1, Tp) for Tp in (0, 1, 2)]
    assert len({round(v, 9) for v in r}) == 3
    for Tp, v in zip((1, 2), r[1:]):
        assert abs(v - _brute_simplex_rho(xi, 2, 1, Tp, False)) < 1e-12


def test_simplex_hand_worked_tp1():
    with open(os.path.join(GOLDEN, "hand_worked_simplex_Tp1.json")) as f:
        g = json.load(f)
    env = {"exp": math.exp}
    for name, mode in (("loo", O.MODE_LOO), ("half", O.MODE_HALF)):
        blk = g[name]
        x = np.array(blk["x"], dtype=np.float32)
        Q, idx, w, d2 = O.knn_table(x, g["E"], g["tau"], g["Tp"], mode)
        assert Q.tolist() == [row["t"] for row in blk["rows"]]
        pred, obs = [], []
        for r, row in enumerate(blk["rows"]):
            assert idx[r].tolist() == row["nbr"], (name, row["t"])
            want = [eval(expr, env) for expr in row["w"]]
            np.testing.assert_allclose(w[r], want, rtol=0, atol=1e-15)
            pred.append(eval(row["pred"], env))
            obs.append(float(row["obs"]))
        want_rho = np.corrcoef(obs, pred)[0, 1]
        assert abs(O.simplex_rho(x, g["E"], g["tau"], g["Tp"], mode) - want_rho) < 1e-14, name


def test_simplex_periodic_closed_form():
    """x(t) = tab[t mod 5] with tab = (0, 1, 0, 2, 3): one lag cannot tell phase 0 from
    phase 2 (both read 0; one step later they read 1 and 2, two steps later 0 and 3), two
    lags can.  Once E resolves the phase the
    nearest neighbours sit at distance 0 in the same phase and the zero-distance rule gives
    an exact forecast at any horizon: rho_E = 1.  At E = 1 the forecast is not exact, so
    optE >= 2 (which of the E >= 2, all 1 up to rounding, wins is left to rounding).  A
    forecast of x(t) instead of x(t+Tp) would be exact at E = 1 already."""
    tab = [0.0, 1.0, 0.0, 2.0, 3.0]
    L = 120
    x = np.array([tab[t % 5] for t in range(L)], dtype=np.float32)
    for mode in (O.MODE_LOO, O.MODE_HALF):
        for Tp in (1, 2):
            assert O.simplex_rho(x, 1, 1, Tp, mode) < 0.99, (mode, Tp)
            for E in (2, 3, 5):
                assert abs(O.simplex_rho(x, E, 1, Tp, mode) - 1.0) < 1e-12, (mode, Tp, E)
        optE, rho, nanf = O.simplex_optE(x[:, None], [0], 1, 6, 1, 1, mode)
        assert optE[0] >= 2 and not nanf[0] and rho[0, 0] < 0.99
        np.testing.assert_allclose(rho[0, 1:], 1.0, rtol=0, atol=1e-12)
    # at Tp = 0 the one-lag forecast of x(t) itself is exact (the degenerate protocol)
    assert abs(O.simplex_rho(x, 1, 1, 0) - 1.0) < 1e-12


# --- the Pearson zero-variance rule -------------------------------------------------------
def test_pearson_nan_threshold_boundary():
    """A centred sum of squares counts as zero when it is at most 1e-10 of the raw sum of
    squares.  a = 1 + delta * s with s = (+1, -1, ...) over n = 10 points has centred sum
    n delta^2 and raw sum n (1 + delta^2): the boundary is delta^2 = 1e-10 / (1 - 1e-10),
    delta ~ 1e-5.  Just above it rho(a, s) is 1 (a is affine in s); just below it is NaN.
    A threshold slipped by a factor n (mean instead of sum on one side) moves the boundary
    by sqrt(10) and fails one side."""
    n = 10
    s = np.array([1.0, -1.0] * (n // 2))
    for delta, is_nan in ((1.01e-5, False), (0.99e-5, True), (3.2e-5, False), (3.1e-6, True)):
        a = 1.0 + delta * s
        for r in (O.pearson(a, s), O.pearson(s, a)):
            if is_nan:
                assert math.isnan(r), delta
            else:
                assert abs(r - 1.0) < 1e-9, (delta, r)
    # a large offset with a healthy spread is not mistaken for a constant
    a = 1e4 + 0.5 * s
    assert abs(O.pearson(a, -s) + 1.0) < 1e-12
