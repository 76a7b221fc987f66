"""CPU oracle for the all-pairs Convergent Cross Mapping (CCM) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this module: only the tests, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the GPU library; both are fed by the seeded input
generators in ``synth``.

It is the plain, slow definition of what the GPU path computes, written from the
paper (Watanakeesuntorn et al., "Massively Parallel Causal Inference of Whole Brain
Dynamics at Single Neuron Resolution", IEEE eScience 2020):

  * delay embedding            -- Sec. II-B (shadow manifold from lags x(t), x(t-tau), ...)
  * k nearest neighbours       -- Sec. III-B, Alg. 3 / Alg. 4 (all-pairs distances, then
                                  the E+1 smallest per query row)
  * distance -> weight         -- Sec. III-A, Alg. 1 "normalize": exponential scale, each
                                  row normalised
  * lookup (prediction)        -- Sec. III-B, Alg. 5: weighted sum of the neighbours' values
  * corrcoef (Pearson rho)     -- Sec. III-A, Alg. 1 / Alg. 2
  * simplex projection / optE  -- Sec. II-B and Sec. III-A, Alg. 1 phase 1 (argmax over E)
  * table reuse across targets -- Sec. III-B, Alg. 2 (one table per library, every target)
  * convergence test           -- Sec. III-A (skill against library size over random
                                  library subsamples; the paper skips it)

Readings where the paper is silent or garbled (each is listed with its reason in the
design notes):
  * a point is labelled by its newest coordinate: row t holds (x(t), x(t-tau), ...,
    x(t-(E-1)tau)); queries and candidates are the library's own points;
  * neighbours are selected on a canonical FP32 squared distance (lag 0 first, one
    rounding per subtraction, multiplication and addition, no fused multiply-add), sorted
    ascending by (d^2, time index) -- ties go to the lower time index; the query itself is
    excluded; k = E + 1;
  * weights: d_k = Euclidean distance recomputed in FP64 from the inputs,
    u_k = exp(-d_k / d_1), w_k = u_k / sum(u); when d_1 = 0, u_k = 1 where d_k = 0 and 0
    elsewhere (the limit d_1 -> 0+);
  * everything after the selection is FP64; Pearson is the two-pass centred formula and is
    NaN when either centred sum of squares vanishes (<= 1e-10 of the raw sum of squares);
  * optE is scored by leave-one-out simplex at Tp = 1 (query = candidate set, self
    excluded); the paper's half split is kept as ``mode = HALF``; the smallest E reaching
    the largest non-NaN rho wins;
  * the cross-map uses the library's own E and Tp = 0; row = library, column = target;
    ``crossmap_rho_target_E`` is the paper's own form, where each target picks the
    libraries' tables at the target's E.

Parity pins for every function live in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import numpy as np

MODE_LOO = 0
MODE_HALF = 1

__all__ = [
    "MODE_LOO", "MODE_HALF", "embed", "point_sets", "sqdist_fp32", "select_knn",
    "weights_fp64", "weights_rows_fp64", "pearson", "knn_table", "knn", "simplex_rho", "simplex_optE",
    "crossmap_rho", "ccm_block", "crossmap_rho_target_E", "ccm_convergence", "crossmap_rho_grad",
]


# ---------------------------------------------------------------------------
# Embedding (Sec. II-B)
# ---------------------------------------------------------------------------
def embed(x, E: int, tau: int) -> np.ndarray:
    """Delay embedding of one series.

    Row r is the point labelled t = r + (E-1)*tau; column e is x(t - e*tau).
    Shape [L - (E-1)*tau][E].
    """
    x = np.asarray(x)
    L = x.shape[0]
    n = L - (E - 1) * tau
    if n <= 0:
        return np.zeros((0, E), dtype=x.dtype)
    out = np.empty((n, E), dtype=x.dtype)
    for r in range(n):
        t = r + (E - 1) * tau
        for e in range(E):
            out[r, e] = x[t - e * tau]
    return out


def point_sets(L: int, E: int, tau: int, Tp: int, mode: int = MODE_LOO):
    """Query set Q and candidate set C (time indices) for one E.

    LOO (and the cross-map, Tp = 0): Q = C = {t : (E-1)tau <= t <= L-1-Tp}; the query
    itself is excluded from its own candidates.
    HALF (the paper's phase 1, Alg. 1): library half [0, L//2), target half [L//2, L),
    each embedded on its own; C = library points whose lags and future stay in the
    library half, Q = target points whose lags and future stay in the target half; no
    self-exclusion is needed.
    """
    lo = (E - 1) * tau
    if mode == MODE_LOO:
        Q = np.arange(lo, L - Tp, dtype=np.int64)
        return Q, Q.copy(), True
    h = L // 2
    C = np.arange(lo, h - Tp, dtype=np.int64)
    Q = np.arange(h + lo, L - Tp, dtype=np.int64)
    return Q, C, False


# ---------------------------------------------------------------------------
# Neighbour search (Sec. III-B, Alg. 3 / Alg. 4)
# ---------------------------------------------------------------------------
def sqdist_fp32(x32, Q, C, E: int, tau: int) -> np.ndarray:
    """Canonical FP32 squared distances between the points labelled Q and C.

    acc = 0; for e = 0..E-1: d = fl32(x[t-e tau] - x[s-e tau]); acc = fl32(acc + fl32(d*d)).
    Element-wise float32 NumPy arithmetic (no BLAS, no fused multiply-add).
    """
    x32 = np.asarray(x32, dtype=np.float32)
    Q = np.asarray(Q, dtype=np.int64)
    C = np.asarray(C, dtype=np.int64)
    acc = np.zeros((Q.size, C.size), dtype=np.float32)
    for e in range(E):
        a = x32[Q - e * tau][:, None]
        b = x32[C - e * tau][None, :]
        d = np.subtract(a, b, dtype=np.float32)
        sq = np.multiply(d, d, dtype=np.float32)
        acc = np.add(acc, sq, dtype=np.float32)
    return acc


def select_knn(D2: np.ndarray, Q, C, k: int, exclude_self: bool):
    """The k smallest candidates of each query row, sorted by (d^2, time index).

    Returns (idx [|Q|][k] int64 time indices, d2 [|Q|][k] float32).  Raises ValueError
    if a query has fewer than k admissible candidates.
    """
    Q = np.asarray(Q, dtype=np.int64)
    C = np.asarray(C, dtype=np.int64)
    D2 = np.array(D2, dtype=np.float32, copy=True)
    avail = C.size - (1 if exclude_self else 0)
    if k > avail or k < 1:
        raise ValueError(f"k={k} exceeds the {avail} admissible candidates")
    if exclude_self:
        pos = np.searchsorted(C, Q)
        hit = (pos < C.size) & (C[np.minimum(pos, C.size - 1)] == Q)
        rows = np.nonzero(hit)[0]
        D2[rows, pos[rows]] = np.inf
    # Columns are in ascending time order, so a stable sort on d^2 breaks ties toward
    # the lower time index.
    order = np.argsort(D2, axis=1, kind="stable")[:, :k]
    idx = C[order]
    d2 = np.take_along_axis(D2, order, axis=1)
    return idx, d2


def weights_fp64(x, t, nbr, E: int, tau: int) -> np.ndarray:
    """Simplex weights of one query t with neighbours nbr (Sec. III-A "normalize").

    d_k = sqrt(sum_e (x(t-e tau) - x(n_k-e tau))^2) in FP64, u_k = exp(-d_k/d_1),
    w = u / sum(u); if d_1 == 0: u_k = 1 where d_k == 0, else 0.
    """
    x64 = np.asarray(x, dtype=np.float64)
    nbr = np.asarray(nbr, dtype=np.int64)
    lags = np.arange(E) * tau
    diff = x64[t - lags][None, :] - x64[nbr[:, None] - lags[None, :]]
    d = np.sqrt(np.sum(diff * diff, axis=1))
    d1 = d[0]
    if d1 > 0:
        u = np.exp(-d / d1)
    else:
        u = (d == 0).astype(np.float64)
    return u / u.sum()


def weights_rows_fp64(x, Q, idx, E: int, tau: int) -> np.ndarray:
    """``weights_fp64`` applied to every query row at once (same formulas, row-wise)."""
    x64 = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    lags = np.arange(E) * tau
    diff = x64[Q[:, None, None] - lags[None, None, :]] - x64[idx[:, :, None] - lags[None, None, :]]
    d = np.sqrt(np.sum(diff * diff, axis=2))
    d1 = d[:, :1]
    pos = d1 > 0
    u = np.where(pos, np.exp(-d / np.where(pos, d1, 1.0)), (d == 0).astype(np.float64))
    return u / u.sum(axis=1, keepdims=True)


def pearson(a, b) -> float:
    """Two-pass centred Pearson correlation in FP64.

    NaN if either centred sum of squares vanishes, read as: is at most 1e-10 of the raw
    sum of squares (a variance below the rounding level of the data is indistinguishable
    from zero; an exactly constant series always lands here)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return float("nan")
    da = a - a.mean()
    db = b - b.mean()
    saa = float(np.sum(da * da))
    sbb = float(np.sum(db * db))
    if saa <= 1e-10 * float(np.sum(a * a)) or sbb <= 1e-10 * float(np.sum(b * b)):
        return float("nan")
    return float(np.sum(da * db) / np.sqrt(saa * sbb))


def knn_table(x, E: int, tau: int, Tp: int, mode: int = MODE_LOO, cand=None):
    """Neighbour table of one series at one E: (Q, idx [|Q|][E+1], w [|Q|][E+1] FP64,
    d2 [|Q|][E+1] FP32).  k = E + 1 (Sec. III-A: the E+1 nearest points).

    cand (optional bool [L]): only time indices marked True may be neighbours (a library
    subsample of the CCM convergence test); every point is still a query.
    """
    x32 = np.asarray(x, dtype=np.float32)
    L = x32.shape[0]
    Q, C, excl = point_sets(L, E, tau, Tp, mode)
    if cand is not None:
        C = C[np.asarray(cand, dtype=bool)[C]]
    k = E + 1
    D2 = sqdist_fp32(x32, Q, C, E, tau)
    idx, d2 = select_knn(D2, Q, C, k, excl)
    w = weights_rows_fp64(x32, Q, idx, E, tau)
    return Q, idx, w, d2


def knn(ts, lib_ids, lib_E, tau: int, Tp: int, k_max: int, cand_masks=None):
    """Tables of many libraries in the library's layout [n_lib][L][k_max].

    Row t holds the table row of query t; rows outside Q and slots beyond E_i + 1 are
    padding (idx = -1, w = 0, d2 = +inf).  cand_masks (optional bool [n_lib][L]) restricts
    each library's neighbours to its marked time indices.
    """
    ts = np.asarray(ts, dtype=np.float32)
    L = ts.shape[0]
    n = len(lib_ids)
    idx_out = np.full((n, L, k_max), -1, dtype=np.int32)
    w_out = np.zeros((n, L, k_max), dtype=np.float64)
    d2_out = np.full((n, L, k_max), np.inf, dtype=np.float32)
    for i, (sid, E) in enumerate(zip(lib_ids, lib_E)):
        E = int(E)
        if E + 1 > k_max:
            raise ValueError("E + 1 > k_max")
        Q, idx, w, d2 = knn_table(ts[:, sid], E, tau, Tp,
                                  cand=None if cand_masks is None else cand_masks[i])
        idx_out[i, Q, : E + 1] = idx
        w_out[i, Q, : E + 1] = w
        d2_out[i, Q, : E + 1] = d2
    return idx_out, w_out, d2_out


# ---------------------------------------------------------------------------
# Simplex projection and optimal E (Sec. II-B; Sec. III-A, Alg. 1 phase 1)
# ---------------------------------------------------------------------------
def simplex_rho(x, E: int, tau: int, Tp: int, mode: int = MODE_LOO) -> float:
    """Forecast skill of one series at one E: predict x(t+Tp) from the neighbours'
    futures x(n_k+Tp) (Sec. II-B) and correlate with the observed x(t+Tp)."""
    x64 = np.asarray(x, dtype=np.float32).astype(np.float64)
    Q, idx, w, _ = knn_table(x, E, tau, Tp, mode)
    pred = np.sum(w * x64[idx + Tp], axis=1)
    obs = x64[Q + Tp]
    return pearson(obs, pred)


def simplex_optE(ts, ids, E_min: int, E_max: int, tau: int, Tp: int = 1, mode: int = MODE_LOO):
    """optE per series: argmax over E of the simplex skill (Alg. 1, phase 1).

    Returns (optE int32 [n], rho_E float64 [n][E_max-E_min+1], all_nan bool [n]).
    NaN skills are skipped; ties go to the smaller E; a series whose skills are all NaN
    gets E_min and is flagged.
    """
    ts = np.asarray(ts, dtype=np.float32)
    n = len(ids)
    nE = E_max - E_min + 1
    rho = np.full((n, nE), np.nan)
    optE = np.full(n, E_min, dtype=np.int32)
    all_nan = np.zeros(n, dtype=bool)
    for i, sid in enumerate(ids):
        for E in range(E_min, E_max + 1):
            rho[i, E - E_min] = simplex_rho(ts[:, sid], E, tau, Tp, mode)
        best = None
        for E in range(E_min, E_max + 1):
            r = rho[i, E - E_min]
            if np.isnan(r):
                continue
            if best is None or r > best:
                best = r
                optE[i] = E
        all_nan[i] = best is None
    return optE, rho, all_nan


# ---------------------------------------------------------------------------
# Cross-map (Sec. III-B, Alg. 2 with Alg. 5 lookup and corrcoef)
# ---------------------------------------------------------------------------
def crossmap_rho(ts, nbr_idx, nbr_w, lib_E, tau: int, tgt0: int, n_tgt: int):
    """rho[i, j] = Pearson(Y[Q_i, j], yhat_ij[Q_i]), yhat_ij(t) = sum_k w_i[t,k] Y[n_ik(t), j].

    One table per library is reused for every target (Alg. 2).  Q_i = rows
    (E_i-1)tau .. L-1 (Tp = 0).  FP64 throughout.
    """
    Y = np.asarray(ts, dtype=np.float64)[:, tgt0: tgt0 + n_tgt]
    L = Y.shape[0]
    n_lib = len(lib_E)
    rho = np.full((n_lib, n_tgt), np.nan)
    for i in range(n_lib):
        E = int(lib_E[i])
        k = E + 1
        Q = np.arange((E - 1) * tau, L)
        idx = np.asarray(nbr_idx[i][Q, :k], dtype=np.int64)
        w = np.asarray(nbr_w[i][Q, :k], dtype=np.float64)
        for j in range(n_tgt):
            yhat = np.sum(w * Y[idx, j], axis=1)
            rho[i, j] = pearson(Y[Q, j], yhat)
    return rho


def ccm_block(ts, lib_ids, lib_E, tau: int, tgt0: int, n_tgt: int, k_max=None):
    """Tables at each library's E (Tp = 0), then the n_lib x n_tgt block of rho."""
    k_max = int(max(lib_E)) + 1 if k_max is None else k_max
    idx, w, d2 = knn(ts, lib_ids, lib_E, tau, 0, k_max)
    return crossmap_rho(ts, idx, w, lib_E, tau, tgt0, n_tgt), idx, w, d2


def crossmap_rho_target_E(ts, lib_ids, tgt_E, tau: int, tgt0: int, n_tgt: int, k_max: int = 21):
    """Alg. 2 as the paper prints it: target j is cross-mapped with every library's table at
    the target's own optimal E, E_j = tgt_E[j] (Sec. III-B, phase 2 of Alg. 1).  One table
    per (library, E) is shared by all targets of that E.

    rho[i, j] = Pearson(Y[Q_i(E_j), j], yhat_ij) with yhat_ij(t) = sum_k w[t,k] Y[n_k(t), j]
    over library i's table at E_j (Tp = 0).  FP64 after selection.
    """
    ts = np.asarray(ts, dtype=np.float32)
    tgt_E = np.asarray(tgt_E, dtype=np.int64)
    if tgt_E.shape != (n_tgt,):
        raise ValueError("tgt_E needs one E per target")
    n_lib = len(lib_ids)
    rho = np.full((n_lib, n_tgt), np.nan)
    for E in sorted(set(tgt_E.tolist())):
        cols = np.nonzero(tgt_E == E)[0]
        idx, w, _ = knn(ts, lib_ids, [E] * n_lib, tau, 0, k_max)
        Y = ts[:, tgt0 + cols]
        rho[:, cols] = crossmap_rho(Y, idx, w, [E] * n_lib, tau, 0, len(cols))
    return rho


def ccm_convergence(ts, lib_ids, lib_E, masks, tau: int, tgt0: int, n_tgt: int,
                    k_max: int = 21):
    """CCM convergence test (Sec. III-A recalls it as part of the original CCM definition --
    predictions repeated over random library subsamples of growing size -- and leaves it
    out of Alg. 1): for library i and each candidate mask r (a random library subsample),
    library i's table at E_i with neighbours drawn only from the subsample (every point
    is a query, self excluded), then the cross-map rho of each target.

    masks: bool [n_lib][n_samp][L].  Returns rho [n_lib][n_samp][n_tgt].
    """
    masks = np.asarray(masks, dtype=bool)
    n_lib, n_samp = masks.shape[0], masks.shape[1]
    rho = np.full((n_lib, n_samp, n_tgt), np.nan)
    for i in range(n_lib):
        E = int(lib_E[i])
        idx, w, _ = knn(ts, [lib_ids[i]] * n_samp, [E] * n_samp, tau, 0, k_max,
                        cand_masks=masks[i])
        rho[i] = crossmap_rho(ts, idx, w, [E] * n_samp, tau, tgt0, n_tgt)
    return rho


# ---------------------------------------------------------------------------
# Gradients of a weighted sum of rho entries (differentiable form of the cross-map)
# ---------------------------------------------------------------------------
def crossmap_rho_grad(ts, lib_ids, lib_E, nbr_idx, tau: int, pairs, gw):
    """FP64 gradient of loss = sum_p gw[p] * rho[lib p, tgt p] with the neighbour sets fixed.

    pairs[p] = (library row i, target column j) into ts; the library series is
    ts[:, lib_ids[i]].  Returns (g_tgt [L][N] w.r.t. ts read as targets,
    g_lib [n_lib][L] w.r.t. each library series).  The two are kept apart: the same
    series read as a library and as a target gets two separate gradients.

    Derivation (all FP64, neighbour sets n_k(t) fixed):
      rho = c / sqrt(a b), a = sum (y-ybar)^2, b = sum (p-pbar)^2, c = sum (y-ybar)(p-pbar)
      drho/dy_t = (p_t-pbar)/sqrt(ab) - rho (y_t-ybar)/a           (observed term)
      drho/dp_t = (y_t-ybar)/sqrt(ab) - rho (p_t-pbar)/b =: H_t     (prediction term)
      p_t = sum_k w_tk Y[n_k(t)]  ->  dL/dY[s] += sum_{(t,k): n_k(t)=s} w_tk H_t
      dL/dw_tk = H_t Y[n_k(t)];  w = u / sum(u), u_k = exp(-d_k/d_1)
      du_k/dd_k = -u_k/d_1 (k > 1), du_k/dd_1 = u_k d_k/d_1^2 (k > 1); u_1 = e^-1 is constant
      d_k = ||v_t - v_{n_k}||: dd_k/dx(t-e tau) = (x(t-e tau) - x(n_k-e tau))/d_k and the
      opposite sign on x(n_k-e tau).
    The gradient is taken as 0 through any d_k == 0 or d_1 == 0 (non-differentiable).
    """
    ts64 = np.asarray(ts, dtype=np.float64)
    L, N = ts64.shape
    n_lib = len(lib_E)
    g_tgt = np.zeros((L, N))
    g_lib = np.zeros((n_lib, L))
    for (i, j), g in zip(np.asarray(pairs), np.asarray(gw, dtype=np.float64)):
        i = int(i)
        j = int(j)
        E = int(lib_E[i])
        k = E + 1
        x = ts64[:, int(lib_ids[i])]
        Q = np.arange((E - 1) * tau, L)
        idx = np.asarray(nbr_idx[i][Q, :k], dtype=np.int64)
        lags = np.arange(E) * tau
        # distances, weights
        V = x[Q[:, None] - lags[None, :]]                    # [n][E]
        Vn = x[idx[:, :, None] - lags[None, None, :]]        # [n][k][E]
        diff = V[:, None, :] - Vn                            # [n][k][E]
        d = np.sqrt(np.sum(diff * diff, axis=2))             # [n][k]
        d1 = d[:, :1]
        pos = d1[:, 0] > 0
        u = np.where(pos[:, None], np.exp(-d / np.where(pos[:, None], d1, 1.0)),
                     (d == 0).astype(np.float64))
        S = u.sum(axis=1, keepdims=True)
        w = u / S
        y = ts64[:, j]
        Yn = y[idx]
        p = np.sum(w * Yn, axis=1)
        yo = y[Q]
        dy = yo - yo.mean()
        dp = p - p.mean()
        a = np.sum(dy * dy)
        b = np.sum(dp * dp)
        if a == 0 or b == 0:
            continue
        sab = np.sqrt(a * b)
        r = np.sum(dy * dp) / sab
        H = dy / sab - r * dp / b                            # drho/dp_t
        Gy = dp / sab - r * dy / a                           # drho/dy_t (observed)
        # target gradient
        np.add.at(g_tgt[:, j], Q, g * Gy)
        np.add.at(g_tgt[:, j], idx.ravel(), (g * w * H[:, None]).ravel())
        # library gradient
        wbar = g * H[:, None] * Yn                           # dL/dw [n][k]
        ubar = (wbar - np.sum(wbar * w, axis=1, keepdims=True)) / S   # dL/du
        dbar = np.zeros_like(d)
        ok = pos[:, None] & (d > 0)
        safe_d1 = np.where(pos, d1[:, 0], 1.0)[:, None]
        # k >= 2: u_k = exp(-d_k/d_1)
        dbar[:, 1:] += np.where(ok[:, 1:], -ubar[:, 1:] * u[:, 1:] / safe_d1, 0.0)
        dd1 = np.sum(np.where(ok[:, 1:], ubar[:, 1:] * u[:, 1:] * d[:, 1:] / safe_d1 ** 2, 0.0),
                     axis=1)
        dbar[:, 0] += np.where(pos, dd1, 0.0)
        safe_d = np.where(d > 0, d, 1.0)
        coef = np.where(d > 0, dbar / safe_d, 0.0)           # [n][k]
        contrib = coef[:, :, None] * diff                    # d/dV_t (+), d/dVn (-)
        gl = g_lib[i]
        np.add.at(gl, (Q[:, None] - lags[None, :]).ravel(),
                  np.broadcast_to(contrib.sum(axis=1), V.shape).ravel())
        np.add.at(gl, (idx[:, :, None] - lags[None, None, :]).ravel(), (-contrib).ravel())
    return g_tgt, g_lib
