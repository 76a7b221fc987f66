"""Seeded synthetic workloads for the all-pairs CCM hot path.

This module only draws inputs.  It holds none of the method's arithmetic
(no embedding, no neighbour search, no prediction, no correlation), so the
CPU oracle and the GPU library can both be fed from it without sharing any
code that computes a result.

The paper evaluates on zebrafish calcium-imaging recordings (Table I: Fish1_Normo
1,450 steps x 53,053 series, Subject6 3,780 x 92,538, Subject11 8,528 x 101,729);
those recordings are not available, so the workloads below stand in for them with
the same shapes (series length, series count) and the same kind of signal
(nonlinear coupled dynamics, neuron-like firing rates).

Every workload is drawn from ``numpy.random.default_rng([config_id, trial])``,
with the draws made in the order listed in each function.  Panels are time-major
float32 arrays ``[L][N]`` (series are columns), the layout the kernels read.
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "coupled_logistic",
    "rate_network",
    "zscore",
    "make",
    "CONFIGS",
]

GENERATOR_VERSION = 1


@dataclasses.dataclass
class Workload:
    """One synthetic input: a time-major panel plus what a run needs around it."""

    name: str
    panel: np.ndarray  # [L][N] float32, time-major
    E_min: int
    E_max: int
    lib_ids: np.ndarray  # int32 series used as libraries
    tgt0: int
    n_tgt: int
    beta: Optional[np.ndarray] = None  # coupling matrix (logistic networks), beta[i, j]: effect of j on i
    flagged: Optional[np.ndarray] = None  # series whose z-score was undefined (constant)
    pairs: Optional[np.ndarray] = None  # [P][2] (lib row, target col) for the loss of the gradient workload
    pair_weights: Optional[np.ndarray] = None


def zscore(panel: np.ndarray):
    """Per-series z-score with the population standard deviation (ddof = 0).

    A constant series has no defined z-score: it is set to all zeros and flagged.
    """
    p = np.asarray(panel, dtype=np.float64)
    mu = p.mean(axis=0)
    sd = p.std(axis=0)
    flagged = sd == 0
    sd_safe = np.where(flagged, 1.0, sd)
    z = (p - mu) / sd_safe
    z[:, flagged] = 0.0
    return z, flagged


def coupled_logistic(rng: np.random.Generator, N: int, T: int, *, r_lo=3.7, r_hi=3.9,
                     beta_hi=0.1, density=0.1, burn=200, noise_sd=0.01, beta_scale=1.0):
    """Coupled logistic maps x_i(t+1) = x_i(t) (r_i - r_i x_i(t) - sum_j beta_ij x_j(t)).

    Draw order: r (N), directed edge mask (N x N, no self-loops), beta values (N x N),
    x0 (N), observation noise (T x N).  The noise is added to the recorded series only
    (it is not fed back into the dynamics).  Returns (panel float32 [T][N], beta).
    """
    r = rng.uniform(r_lo, r_hi, size=N)
    mask = rng.random((N, N)) < density
    np.fill_diagonal(mask, False)
    bvals = rng.uniform(0.0, beta_hi, size=(N, N))
    beta = np.where(mask, bvals, 0.0) * beta_scale
    x = rng.uniform(0.1, 0.9, size=N)
    noise = rng.normal(0.0, noise_sd, size=(T, N))
    out = np.empty((T, N), dtype=np.float64)
    for step in range(burn + T):
        x = x * (r - r * x - beta @ x)
        if step >= burn:
            out[step - burn] = x
    out += noise
    return out.astype(np.float32), beta


def _sparse_gaussian(rng: np.random.Generator, N: int, p: float):
    """Sparse N x N matrix: each row has Binomial(N, p) entries at uniform columns,
    values N(0, 1/(pN)).  Repeated columns in a row are summed (rare at the sizes used).
    Draw order: row counts (N), column indices (nnz), values (nnz)."""
    import scipy.sparse as sp

    counts = rng.binomial(N, p, size=N)
    nnz = int(counts.sum())
    cols = rng.integers(0, N, size=nnz)
    vals = rng.standard_normal(nnz) / np.sqrt(p * N)
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    J = sp.csr_matrix((vals, cols, indptr), shape=(N, N))
    J.sum_duplicates()
    return J


def _row_split_matvec(J, min_rows: int = 16384):
    """J @ v computed over row blocks in threads (each row's dot product is the same
    arithmetic as the unsplit product, so the result is bitwise identical)."""
    N = J.shape[0]
    nt = min(16, os.cpu_count() or 1)
    if N < min_rows or nt < 2:
        return lambda v: J @ v
    from concurrent.futures import ThreadPoolExecutor

    bounds = np.linspace(0, N, nt + 1).astype(int)
    parts = [J[bounds[i]: bounds[i + 1]] for i in range(nt)]
    pool = ThreadPoolExecutor(nt)
    return lambda v: np.concatenate(list(pool.map(lambda P: P @ v, parts)))


def rate_network(rng: np.random.Generator, N: int, T: int, *, p=0.01, g=1.5, dt=0.1,
                 sigma=0.05, burn=1000, poisson=False, lam_max=1.0, tau_f=5.0):
    """Sparse random recurrent rate network of tanh units.

    x <- x + dt (-x + g J tanh(x)) + sigma xi, xi ~ N(0, 1) each step.
    Without ``poisson`` the recorded signal is tanh(x).  With ``poisson`` each unit
    fires Poisson(lam_max (1 + tanh x) / 2) spikes per step, filtered as
    f(t) = exp(-1/tau_f) f(t-1) + s(t) from the start of the burn-in, and f is recorded.

    Draw order: J (see _sparse_gaussian), x0 ~ N(0, 1) (N), then per step the drive
    xi (N) followed, with ``poisson``, by the spike counts (N).
    Returns the raw (not z-scored) float64 panel [T][N].
    """
    J = _sparse_gaussian(rng, N, p)
    matvec = _row_split_matvec(J)
    x = rng.standard_normal(N)
    decay = np.exp(-1.0 / tau_f)
    f = np.zeros(N)
    out = np.empty((T, N), dtype=np.float64)
    for step in range(burn + T):
        r = np.tanh(x)
        x = x + dt * (-x + g * matvec(r)) + sigma * rng.standard_normal(N)
        r = np.tanh(x)
        if poisson:
            s = rng.poisson(lam_max * 0.5 * (1.0 + r))
            f = decay * f + s
            rec = f
        else:
            rec = r
        if step >= burn:
            out[step - burn] = rec
    return out


# Config table.  Names describe the workload; ids seed the generator.
CONFIGS = {
    # 64 coupled logistic maps, T = 500, optE over E = 1..10, full 64 x 64 block.
    "logistic64": dict(id=1, kind="logistic", N=64, T=500, E_max=10),
    # 1024-unit sparse tanh rate network, T = 1450 (Fish1_Normo's length), E = 1..20.
    "ratenet1024": dict(id=2, kind="rate", N=1024, T=1450, E_max=20, p=0.01),
    # 8192 neuron-like filtered-Poisson rates, T = 1600, E = 1..20.
    "poisson8192": dict(id=3, kind="poisson", N=8192, T=1600, E_max=20, p=0.01),
    # 2048 coupled logistic maps, T = 1000, for the gradient checks.
    "logistic2048": dict(id=4, kind="logistic", N=2048, T=1000, E_max=20),
    # 512 libraries x 101,729 targets (Subject11's series count), T = 1600.
    "brain101729": dict(id=5, kind="poisson", N=101729, T=1600, E_max=20, p=0.001, n_lib=512),
}


def _cache_path(name: str, trial: int, overrides: dict) -> Optional[str]:
    root = os.environ.get("CCM_INPUT_CACHE", "/tmp/ccm_input_cache")
    if not root:
        return None
    key = f"{name}|{trial}|{sorted(overrides.items())}|v{GENERATOR_VERSION}"
    h = hashlib.sha1(key.encode()).hexdigest()[:16]
    return os.path.join(root, f"{name}_{trial}_{h}.npz")


def make(name: str, trial: int = 0, *, cache: bool = True, **overrides) -> Workload:
    """Build workload ``name`` (a key of CONFIGS) for seed trial ``trial``.

    ``overrides`` may shrink a workload for quick tests (e.g. N=..., T=...); the
    seed stays ``[config id, trial]`` so a shrunk workload is still reproducible.
    """
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    cid = cfg["id"]
    N, T = int(cfg["N"]), int(cfg["T"])
    path = _cache_path(name, trial, overrides) if cache else None
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Workload(
            name=name, panel=z["panel"], E_min=int(z["E_min"]), E_max=int(z["E_max"]),
            lib_ids=z["lib_ids"], tgt0=int(z["tgt0"]), n_tgt=int(z["n_tgt"]),
            beta=z["beta"] if z["beta"].size else None,
            flagged=z["flagged"] if z["flagged"].size else None,
            pairs=z["pairs"] if z["pairs"].size else None,
            pair_weights=z["pair_weights"] if z["pair_weights"].size else None,
        )
    rng = np.random.default_rng([cid, trial])
    beta = None
    flagged = None
    pairs = None
    pair_weights = None
    kind = cfg["kind"]
    if kind == "logistic":
        if name == "logistic2048":
            density = 0.02
            beta_hi = 0.05
            # The map diverges with these couplings as stated; the expected in-degree is
            # normalised to the 64-map network's (0.1 * 63 = 6.3 inputs per unit).
            scale = 6.3 / (density * (N - 1))
        else:
            density, beta_hi, scale = 0.1, 0.1, 1.0
        panel, beta = coupled_logistic(rng, N, T, beta_hi=beta_hi, density=density,
                                       beta_scale=scale)
        if name == "logistic2048":
            P = int(cfg.get("n_pairs", 256))
            prng = np.random.default_rng([cid, trial, 1])
            i = prng.integers(0, N, size=4 * P)
            j = prng.integers(0, N, size=4 * P)
            keep = i != j
            pairs = np.stack([i[keep], j[keep]], axis=1)[:P].astype(np.int32)
            pair_weights = np.ones(P, dtype=np.float32)
    elif kind in ("rate", "poisson"):
        raw = rate_network(rng, N, T, p=cfg.get("p", 0.01), burn=int(cfg.get("burn", 1000)),
                           poisson=(kind == "poisson"))
        z, flagged = zscore(raw)
        panel = z.astype(np.float32)
    else:
        raise ValueError(kind)
    n_lib = int(cfg.get("n_lib", N))
    wl = Workload(
        name=name, panel=np.ascontiguousarray(panel, dtype=np.float32), E_min=1,
        E_max=int(cfg["E_max"]), lib_ids=np.arange(n_lib, dtype=np.int32), tgt0=0, n_tgt=N,
        beta=beta, flagged=flagged, pairs=pairs, pair_weights=pair_weights,
    )
    if path:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        e = np.zeros(0)
        np.savez(tmp, panel=wl.panel, E_min=wl.E_min, E_max=wl.E_max, lib_ids=wl.lib_ids,
                 tgt0=wl.tgt0, n_tgt=wl.n_tgt,
                 beta=beta if beta is not None else e,
                 flagged=flagged if flagged is not None else e,
                 pairs=pairs if pairs is not None else e,
                 pair_weights=pair_weights if pair_weights is not None else e)
        os.replace(tmp, path)
    return wl


def periodic(P: int, L: int, rng: np.random.Generator) -> np.ndarray:
    """A series that repeats exactly with period P (x(t) = tab[t mod P])."""
    tab = rng.standard_normal(P).astype(np.float32)
    return tab[np.arange(L) % P]


def library_samples(L: int, E: int, sizes, n_samples: int, seed: int, tau: int = 1) -> np.ndarray:
    """Random library subsamples for the CCM convergence test: for each size m in `sizes`
    and each of `n_samples` draws, a boolean mask over time indices [L] marking m points
    drawn without replacement from the embedded points {(E-1) tau, ..., L-1}.

    Draw order: sizes in the given order, samples in order, one `rng.choice` each, from
    `default_rng([7, seed, E])`.  Returns bool [len(sizes) * n_samples][L].
    """
    rng = np.random.default_rng([7, seed, E])
    lo = (E - 1) * tau
    pts = np.arange(lo, L)
    out = np.zeros((len(sizes) * n_samples, L), dtype=bool)
    r = 0
    for m in sizes:
        if m > pts.size:
            raise ValueError(f"library size {m} exceeds the {pts.size} embedded points")
        for _ in range(n_samples):
            out[r, rng.choice(pts, size=m, replace=False)] = True
            r += 1
    return out


def two_species(T: int, seed: int, *, rx=3.8, ry=3.5, bxy=0.02, byx=0.1, burn=300) -> np.ndarray:
    """Two coupled logistic maps (x drives y more strongly than y drives x):
    x(t+1) = x(t) (rx - rx x(t) - bxy y(t)),  y(t+1) = y(t) (ry - ry y(t) - byx x(t)).
    Draw order: x0, y0 ~ U(0.2, 0.8) from `default_rng([8, seed])`.  Returns float32 [T][2]
    with columns (x, y)."""
    rng = np.random.default_rng([8, seed])
    x, y = rng.uniform(0.2, 0.8, size=2)
    out = np.empty((T, 2), dtype=np.float64)
    for t in range(burn + T):
        if t >= burn:
            out[t - burn] = (x, y)
        x, y = x * (rx - rx * x - bxy * y), y * (ry - ry * y - byx * x)
    return out.astype(np.float32)
