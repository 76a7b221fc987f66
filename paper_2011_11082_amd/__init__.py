"""MI355X (gfx950) all-pairs Convergent Cross Mapping hot path.

Thin ctypes binding over the C ABI of ``libccm.so`` (declared in include/ccm.h).  It only
marshals arguments: tensors become device pointers, the current torch stream becomes the
HIP stream, and a caller-owned workspace is allocated through torch's caching allocator.
Every step of the computation runs in the library's HIP kernels; there is no fallback.

Entry points (same names as the C ABI, minus the ``ccm_`` prefix):
  embed, knn, simplex_optE, crossmap_rho, crossmap_rho_backward, workspace_size
and the differentiable wrapper ``CrossMapRho`` / ``crossmap_rho_autograd``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch  # loaded first: the library then binds to torch's HIP runtime

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libccm.so")

CCM_OK, CCM_EINVAL, CCM_ERANGE, CCM_EDEVICE, CCM_ENOTSUP, CCM_EWORKSPACE = range(6)
E_MAX = 20
K_MAX = 21
MODE_LOO, MODE_HALF = 0, 1
PRECISION_FP32, PRECISION_BF16 = 0, 1
(OP_EMBED, OP_KNN, OP_SIMPLEX, OP_CROSSMAP_FP32, OP_CROSSMAP_BF16, OP_CROSSMAP_BACKWARD,
 OP_CROSSMAP_TARGET_E) = range(7)

EXPORTED = (
    "ccm_embed", "ccm_knn", "ccm_knn_subset", "ccm_simplex_optE", "ccm_simplex_optE_noalloc",
    "ccm_crossmap_rho",
    "ccm_crossmap_rho_backward", "ccm_crossmap_rho_target_E", "ccm_workspace_size",
    "ccm_set_check_finite", "ccm_set_gather_tile", "ccm_status_string", "ccm_last_error",
    "ccm_version",
)


class CCMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[status {status}] {msg}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libccm.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with __graft_entry__.build() "
                           "(the CCM kernels have no CPU fallback)")
    lib = ctypes.CDLL(p)
    sig = {
        "ccm_embed": [_P, _I64, _I32, _P, _I32, _I32, _I32, _P, _P],
        "ccm_knn": [_P, _I64, _I32, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _SZ, _P],
        "ccm_knn_subset": [_P, _I64, _I32, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _P, _P,
                           _SZ, _P],
        "ccm_simplex_optE": [_P, _I64, _I32, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P,
                             _SZ, _P],
        "ccm_simplex_optE_noalloc": [_P, _I64, _I32, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P,
                                     _P, _P],
        "ccm_crossmap_rho": [_P, _I64, _I32, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _I32, _P,
                             _P, _P, _SZ, _P],
        "ccm_crossmap_rho_backward": [_P, _I64, _I32, _P, _P, _P, _P, _I32, _I32, _I32, _P, _P,
                                      _P, _I32, _P, _P, _P, _SZ, _P],
        "ccm_crossmap_rho_target_E": [_P, _I64, _I32, _P, _P, _I32, _I32, _I32, _I32, _I32, _P,
                                      _I32, _I32, _P, _P, _P, _SZ, _P],
        "ccm_workspace_size": [_I32, _I32, _I32, _I32, _I32, ctypes.POINTER(_SZ)],
        "ccm_set_check_finite": [_I32],
        "ccm_set_gather_tile": [_I32],
        "ccm_status_string": [_I32],
        "ccm_last_error": [],
        "ccm_version": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("ccm_status_string", "ccm_last_error",
                                                "ccm_version") else _I32
    if path is None:
        _lib = lib
    return lib


def _check(status: int):
    if status != CCM_OK:
        lib = load_library()
        raise CCMError(status, (lib.ccm_last_error() or b"").decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t


def _panel(ts: torch.Tensor):
    """(tensor, ld, L) of a time-major [L][N] float32 panel with unit column stride."""
    _dev(ts, "ts", torch.float32)
    if ts.dim() != 2 or ts.stride(1) != 1:
        raise ValueError("ts must be a 2-D [L][N] panel with unit stride along N")
    if ts.device.index is not None and ts.device.index != torch.cuda.current_device():
        # kernels launch on the current device and its current stream
        raise ValueError(f"ts is on {ts.device}, the current device is cuda:"
                         f"{torch.cuda.current_device()} (use torch.cuda.device(...))")
    return ts, int(ts.stride(0)), int(ts.shape[0])


def _i32(t, device) -> torch.Tensor:
    if isinstance(t, torch.Tensor):
        t = t.to(device=device, dtype=torch.int32)
    else:
        t = torch.as_tensor(t, dtype=torch.int32, device=device)
    return t.contiguous()


def set_check_finite(on: bool) -> None:
    """Debug mode (process-wide): every call first checks that the values it reads are
    finite, synchronising its stream, and raises CCMError (CCM_EINVAL) if one is not."""
    _check(load_library().ccm_set_check_finite(1 if on else 0))


def set_gather_tile(targets: int) -> None:
    """Testing switch (process-wide) for the FP32 cross-map's target tile: 0 chooses it from
    L; 4, 8 or 16 force that LDS tile where it fits; 32 forces the global tile copy."""
    _check(load_library().ccm_set_gather_tile(int(targets)))


def workspace_size(op: int, L: int, n_lib: int, n_tgt: int, k_max: int) -> int:
    lib = load_library()
    out = _SZ(0)
    _check(lib.ccm_workspace_size(op, L, n_lib, n_tgt, k_max, ctypes.byref(out)))
    return int(out.value)


def _workspace(op, L, n_lib, n_tgt, k_max, device, ws=None):
    need = workspace_size(op, L, n_lib, n_tgt, k_max)
    if ws is not None:
        return ws, need
    if need == 0:
        return None, 0
    return torch.empty(need, dtype=torch.uint8, device=device), need


def embed(ts: torch.Tensor, ids, E: int, tau: int = 1) -> torch.Tensor:
    """Delay embedding [n][L-(E-1)tau][E] of series ``ids`` (columns of ts)."""
    lib = load_library()
    ts, ld, L = _panel(ts)
    ids = _i32(ids, ts.device)
    n = ids.numel()
    emb = torch.empty((n, max(L - (E - 1) * tau, 0), E), dtype=torch.float32, device=ts.device)
    _check(lib.ccm_embed(_ptr(ts), ld, L, _ptr(ids), n, E, tau, _ptr(emb), _stream()))
    return emb


def knn(ts: torch.Tensor, lib_ids, lib_E, tau: int = 1, Tp: int = 0, k_max: int = K_MAX,
        want_d2: bool = True, cand_mask: Optional[torch.Tensor] = None):
    """Neighbour tables (idx int32, w float32, d2 float32 or None), each [n_lib][L][k_max].
    cand_mask (bool or uint8 [n_lib][L], optional): library subsample per row
    (ccm_knn_subset)."""
    lib = load_library()
    ts, ld, L = _panel(ts)
    lib_ids = _i32(lib_ids, ts.device)
    lib_E = _i32(lib_E, ts.device)
    n = lib_ids.numel()
    if lib_E.numel() != n:
        raise ValueError("lib_E and lib_ids differ in length")
    idx = torch.empty((n, L, k_max), dtype=torch.int32, device=ts.device)
    w = torch.empty((n, L, k_max), dtype=torch.float32, device=ts.device)
    d2 = torch.empty((n, L, k_max), dtype=torch.float32, device=ts.device) if want_d2 else None
    if cand_mask is None:
        _check(lib.ccm_knn(_ptr(ts), ld, L, _ptr(lib_ids), _ptr(lib_E), n, tau, Tp, k_max,
                           _ptr(idx), _ptr(w), _ptr(d2), None, 0, _stream()))
    else:
        m = torch.as_tensor(cand_mask, device=ts.device).to(torch.uint8).contiguous()
        if m.shape != (n, L):
            raise ValueError("cand_mask must be [n_lib][L]")
        _check(lib.ccm_knn_subset(_ptr(ts), ld, L, _ptr(lib_ids), _ptr(lib_E), n, tau, Tp, k_max,
                                  _ptr(m), _ptr(idx), _ptr(w), _ptr(d2), None, 0, _stream()))
    return idx, w, d2


def simplex_optE(ts: torch.Tensor, ids, E_min: int = 1, E_max: int = E_MAX, tau: int = 1,
                 Tp: int = 1, mode: int = MODE_LOO):
    """(optE int32 [n], rho_E float32 [n][E_max-E_min+1])."""
    lib = load_library()
    ts, ld, L = _panel(ts)
    ids = _i32(ids, ts.device)
    n = ids.numel()
    optE = torch.empty(n, dtype=torch.int32, device=ts.device)
    rho_E = torch.empty((n, E_max - E_min + 1), dtype=torch.float32, device=ts.device)
    ws, need = _workspace(OP_SIMPLEX, L, n, 0, 0, ts.device)
    _check(lib.ccm_simplex_optE(_ptr(ts), ld, L, _ptr(ids), n, E_min, E_max, tau, Tp, mode,
                                _ptr(optE), _ptr(rho_E), _ptr(ws), need, _stream()))
    return optE, rho_E


NOALLOC_MAX_SERIES = 104857


def simplex_optE_noalloc(ts: torch.Tensor, ids, optE: torch.Tensor, rho_E: torch.Tensor,
                         E_min: int = 1, E_max: int = E_MAX, tau: int = 1, Tp: int = 1,
                         mode: int = MODE_LOO) -> None:
    """ccm_simplex_optE_noalloc into the caller's optE (int32 [n]) and rho_E (float32
    [n][E_max-E_min+1]) on ts's device: no workspace, nothing allocated by the call.  ids
    must already be an int32 device tensor."""
    lib = load_library()
    ts, ld, L = _panel(ts)
    for t, name, dt in ((ids, "ids", torch.int32), (optE, "optE", torch.int32),
                        (rho_E, "rho_E", torch.float32)):
        _dev(t, name, dt)
        if t.device != ts.device or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous on the panel's device")
    n = ids.numel()
    if optE.numel() != n or tuple(rho_E.shape) != (n, E_max - E_min + 1):
        raise ValueError("optE must be [n] and rho_E [n][E_max-E_min+1]")
    _check(lib.ccm_simplex_optE_noalloc(_ptr(ts), ld, L, _ptr(ids), n, E_min, E_max, tau, Tp,
                                        mode, _ptr(optE), _ptr(rho_E), _stream()))


def crossmap_rho(ts: torch.Tensor, nbr_idx: torch.Tensor, nbr_w: torch.Tensor, lib_E,
                 tau: int = 1, tgt0: int = 0, n_tgt: Optional[int] = None,
                 precision: int = PRECISION_FP32, want_moments: bool = False,
                 ws: Optional[torch.Tensor] = None):
    """rho [n_lib][n_tgt] (and FP64 moments [n_lib][n_tgt][3] if asked)."""
    lib = load_library()
    ts, ld, L = _panel(ts)
    _dev(nbr_idx, "nbr_idx", torch.int32)
    _dev(nbr_w, "nbr_w", torch.float32)
    if not (nbr_idx.is_contiguous() and nbr_w.is_contiguous()):
        raise ValueError("tables must be contiguous")
    n_lib, L2, k_max = nbr_idx.shape
    if L2 != L or nbr_w.shape != nbr_idx.shape:
        raise ValueError("table shape does not match the panel")
    lib_E = _i32(lib_E, ts.device)
    if n_tgt is None:
        n_tgt = int(ts.shape[1]) - tgt0
    rho = torch.empty((n_lib, n_tgt), dtype=torch.float32, device=ts.device)
    mom = (torch.empty((n_lib, n_tgt, 3), dtype=torch.float64, device=ts.device)
           if want_moments else None)
    op = OP_CROSSMAP_FP32 if precision == PRECISION_FP32 else OP_CROSSMAP_BF16
    ws, need = _workspace(op, L, n_lib, n_tgt, k_max, ts.device, ws)
    nbytes = ws.numel() if ws is not None else 0
    _check(lib.ccm_crossmap_rho(_ptr(ts), ld, L, _ptr(nbr_idx), _ptr(nbr_w), _ptr(lib_E), n_lib,
                                k_max, tau, tgt0, n_tgt, precision, _ptr(rho), _ptr(mom), _ptr(ws),
                                nbytes, _stream()))
    return (rho, mom) if want_moments else rho


def knn_all_E(ts: torch.Tensor, lib_ids, E_lo: int = 1, n_E: int = E_MAX, tau: int = 1,
              k_max: int = K_MAX, want_d2: bool = False):
    """Tables of every library at every E in E_lo .. E_lo + n_E - 1 (Tp = 0), E-major:
    [n_E * n_lib][L][k_max], table e * n_lib + i = library i at E_lo + e.  One ccm_knn call
    over the (E, library) pairs."""
    ts, _, _ = _panel(ts)
    ids = _i32(lib_ids, ts.device)
    pair_ids = ids.repeat(n_E)
    pair_E = torch.arange(E_lo, E_lo + n_E, dtype=torch.int32,
                          device=ts.device).repeat_interleave(ids.numel())
    return knn(ts, pair_ids, pair_E, tau, 0, k_max, want_d2=want_d2)


def crossmap_rho_target_E(ts: torch.Tensor, nbr_idx: torch.Tensor, nbr_w: torch.Tensor,
                          n_lib: int, tgt_E, E_lo: int = 1, tau: int = 1, tgt0: int = 0,
                          n_tgt: Optional[int] = None, want_moments: bool = False,
                          ws: Optional[torch.Tensor] = None):
    """The paper's per-target-E cross-map: rho [n_lib][n_tgt], target j read through every
    library's table at E = tgt_E[j] (tables from knn_all_E)."""
    lib = load_library()
    ts, ld, L = _panel(ts)
    _dev(nbr_idx, "nbr_idx", torch.int32)
    _dev(nbr_w, "nbr_w", torch.float32)
    if not (nbr_idx.is_contiguous() and nbr_w.is_contiguous()):
        raise ValueError("tables must be contiguous")
    n_tab, L2, k_max = nbr_idx.shape
    if L2 != L or nbr_w.shape != nbr_idx.shape or n_lib <= 0 or n_tab % n_lib:
        raise ValueError("table shape does not match the panel or n_lib")
    n_E = n_tab // n_lib
    if n_tgt is None:
        n_tgt = int(ts.shape[1]) - tgt0
    tgt_E = _i32(tgt_E, ts.device)
    if tgt_E.numel() != n_tgt:
        raise ValueError("tgt_E needs one E per target")
    rho = torch.empty((n_lib, n_tgt), dtype=torch.float32, device=ts.device)
    mom = (torch.empty((n_lib, n_tgt, 3), dtype=torch.float64, device=ts.device)
           if want_moments else None)
    ws, need = _workspace(OP_CROSSMAP_TARGET_E, L, n_tab, n_tgt, k_max, ts.device, ws)
    nbytes = ws.numel() if ws is not None else 0
    _check(lib.ccm_crossmap_rho_target_E(_ptr(ts), ld, L, _ptr(nbr_idx), _ptr(nbr_w), n_lib,
                                         E_lo, n_E, k_max, tau, _ptr(tgt_E), tgt0, n_tgt,
                                         _ptr(rho), _ptr(mom), _ptr(ws), nbytes, _stream()))
    return (rho, mom) if want_moments else rho


def ccm_convergence(ts: torch.Tensor, lib_ids, lib_E, masks, tau: int = 1, tgt0: int = 0,
                    n_tgt: Optional[int] = None, k_max: int = K_MAX):
    """CCM convergence test: rho [n_lib][n_samp][n_tgt], library i's table at E_i built over
    each candidate mask masks[i][r] (a random library subsample; every point is a query),
    then the cross-map of every target.  One ccm_knn_subset call over the (library, sample)
    rows and one ccm_crossmap_rho call."""
    ts, _, L = _panel(ts)
    masks = torch.as_tensor(masks, device=ts.device)
    n_lib, n_samp = int(masks.shape[0]), int(masks.shape[1])
    ids = _i32(lib_ids, ts.device).repeat_interleave(n_samp)
    Es = _i32(lib_E, ts.device).repeat_interleave(n_samp)
    idx, w, _ = knn(ts, ids, Es, tau, 0, k_max, want_d2=False,
                    cand_mask=masks.reshape(n_lib * n_samp, L))
    rho = crossmap_rho(ts, idx, w, Es, tau, tgt0, n_tgt)
    return rho.reshape(n_lib, n_samp, -1)


def ccm_matrix(ts: torch.Tensor, E_min: int = 1, E_max: int = E_MAX, tau: int = 1,
               block: int = 512, precision: int = PRECISION_FP32, per_target_E: bool = False,
               mode: int = MODE_LOO, out: Optional[torch.Tensor] = None):
    """The whole N x N causal matrix of an L x N panel (Sec. III-B, Alg. 1 and Alg. 2):
    phase 1 (optE of every series, E_min..E_max, Tp = 1, leave-one-out or the half split),
    then blocks of `block` libraries, each a table call and a cross-map call against every
    series.  rho[i][j] = cross-map skill of library i for target j (row = library).  With
    per_target_E, target j is read through every library's table at j's own optE (the
    paper's form; FP32 only); otherwise at the library's optE.  Returns (rho [N][N], optE)."""
    if per_target_E and precision != PRECISION_FP32:
        raise ValueError("the per-target-E form is FP32")
    if block < 1:
        raise ValueError("block must be >= 1")
    ts, _, L = _panel(ts)
    N = int(ts.shape[1])
    if out is not None and (tuple(out.shape) != (N, N) or out.dtype != torch.float32
                            or not out.is_contiguous() or out.device != ts.device):
        raise ValueError("out must be a contiguous float32 [N][N] tensor on the panel's device")
    ids = torch.arange(N, dtype=torch.int32, device=ts.device)
    optE, _ = simplex_optE(ts, ids, E_min, E_max, tau, 1, mode)
    if out is None:
        out = torch.empty((N, N), dtype=torch.float32, device=ts.device)
    k_max = E_max + 1
    for b0 in range(0, N, block):
        b1 = min(N, b0 + block)
        if per_target_E:
            idx, w, _ = knn_all_E(ts, ids[b0:b1], E_min, E_max - E_min + 1, tau, k_max)
            out[b0:b1] = crossmap_rho_target_E(ts, idx, w, b1 - b0, optE, E_lo=E_min, tau=tau)
        else:
            idx, w, _ = knn(ts, ids[b0:b1], optE[b0:b1], tau, 0, k_max, want_d2=False)
            out[b0:b1] = crossmap_rho(ts, idx, w, optE[b0:b1], tau, precision=precision)
        del idx, w
    return out, optE


def storage_span_ok(t: torch.Tensor, first: int, last: int) -> bool:
    """True when element offsets first .. last (counted from t's data pointer, in elements
    of t's dtype) all lie inside t's storage.  A host-side check of the memory a kernel is
    about to read or write through a raw pointer."""
    if last < first:
        return True   # an empty range
    total = t.untyped_storage().nbytes() // t.element_size()
    off = t.storage_offset()
    return off + first >= 0 and off + last < total


def crossmap_rho_backward(ts, lib_ts, nbr_idx, nbr_w, lib_E, pair_lib, pair_tgt, grad_rho,
                          tau: int = 1, grad_ts=None, grad_lib=None):
    """Adjoint of sum_p grad_rho[p] * rho[pair_lib[p], pair_tgt[p]] with fixed neighbour sets.

    ts is the [L][N] target panel (row stride ld >= N); pair_tgt are columns of it, in
    [0, N), and pair_lib rows of the tables, in [0, n_lib).  Accumulates into (and returns)
    grad_ts, an [L][N] view with ts's row stride (allocated as [L][ld] zeros when None), and
    grad_lib [n_lib][L] (float32, zeros when None).  The kernels write grad_ts at
    row * ld + column, so a caller's grad_ts must have ts's strides."""
    lib = load_library()
    ts, ld, L = _panel(ts)
    N = int(ts.shape[1])
    _dev(nbr_idx, "nbr_idx", torch.int32)
    _dev(nbr_w, "nbr_w", torch.float32)
    if nbr_idx.dim() != 3 or nbr_w.shape != nbr_idx.shape or int(nbr_idx.shape[1]) != L:
        raise ValueError("tables must be [n_lib][L][k_max] with the panel's L")
    if not (nbr_idx.is_contiguous() and nbr_w.is_contiguous()):
        raise ValueError("tables must be contiguous")
    n_lib, _, k_max = nbr_idx.shape
    lib_E = _i32(lib_E, ts.device)
    if lib_E.numel() != n_lib:
        raise ValueError("lib_E needs one E per table")
    pair_lib = _i32(pair_lib, ts.device)
    pair_tgt = _i32(pair_tgt, ts.device)
    grad_rho = grad_rho.to(device=ts.device, dtype=torch.float32).contiguous()
    n_pairs = pair_lib.numel()
    if pair_tgt.numel() != n_pairs or grad_rho.numel() != n_pairs:
        raise ValueError("pair_lib, pair_tgt and grad_rho differ in length")
    if n_pairs:
        # the pair ids index the panel view and the tables: keep them inside both
        lo_t, hi_t = int(pair_tgt.min()), int(pair_tgt.max())
        lo_l, hi_l = int(pair_lib.min()), int(pair_lib.max())
        if lo_t < 0 or hi_t >= N or lo_l < 0 or hi_l >= n_lib:
            raise ValueError(f"pair ids out of range: targets in [{lo_t}, {hi_t}] for N = {N}, "
                             f"libraries in [{lo_l}, {hi_l}] for n_lib = {n_lib}")
    if not isinstance(lib_ts, torch.Tensor) or lib_ts.device != ts.device:
        raise TypeError("lib_ts must be a tensor on the panel's device")
    lib_ts = lib_ts.to(torch.float32).contiguous()
    if tuple(lib_ts.shape) != (n_lib, L):
        raise ValueError(f"lib_ts must be [n_lib][L] = [{n_lib}][{L}], got {tuple(lib_ts.shape)}")
    if grad_ts is None:
        grad_ts = torch.zeros((L, ld), dtype=torch.float32, device=ts.device)[:, :N]
    else:
        _dev(grad_ts, "grad_ts", torch.float32)
        if (grad_ts.device != ts.device or tuple(grad_ts.shape) != (L, N)
                or grad_ts.stride() != (ld, 1)):
            raise ValueError(f"grad_ts must be a float32 [L][N] = [{L}][{N}] tensor on the "
                             f"panel's device with strides ({ld}, 1)")
    if grad_lib is None:
        grad_lib = torch.zeros((n_lib, L), dtype=torch.float32, device=ts.device)
    else:
        _dev(grad_lib, "grad_lib", torch.float32)
        if (grad_lib.device != ts.device or tuple(grad_lib.shape) != (n_lib, L)
                or not grad_lib.is_contiguous()):
            raise ValueError(f"grad_lib must be a contiguous float32 [{n_lib}][{L}] tensor on "
                             "the panel's device")
    # every element the kernels touch: rows 0..L-1, columns 0..N-1 at stride ld
    if not (storage_span_ok(ts, 0, (L - 1) * ld + N - 1)
            and storage_span_ok(grad_ts, 0, (L - 1) * ld + N - 1)):
        raise ValueError("panel or grad_ts storage is smaller than its [L][N] view")
    ws, need = _workspace(OP_CROSSMAP_BACKWARD, L, n_lib, n_pairs, k_max, ts.device)
    _check(lib.ccm_crossmap_rho_backward(_ptr(ts), ld, L, _ptr(lib_ts), _ptr(nbr_idx), _ptr(nbr_w),
                                         _ptr(lib_E), n_lib, k_max, tau, _ptr(pair_lib),
                                         _ptr(pair_tgt), _ptr(grad_rho), n_pairs, _ptr(grad_ts),
                                         _ptr(grad_lib), _ptr(ws), need, _stream()))
    return grad_ts, grad_lib


class CrossMapRho(torch.autograd.Function):
    """rho[i][j] = cross-map skill of library series X[i] for target column Y[:, j].

    X: [n_lib][L] library series; Y: [L][N] time-major target panel; lib_E: E of each
    library.  Forward builds one table per library (ccm_knn, Tp = 0) and runs
    ccm_crossmap_rho.  Backward runs the hand-written adjoint (ccm_crossmap_rho_backward)
    with the neighbour sets held fixed: d rho / d Y through the observed and looked-up
    target values, d rho / d X through the distances and weights.  The adjoint is that of
    the FP32 form, whichever precision the forward used.
    """

    @staticmethod
    def forward(ctx, X, Y, lib_E, tau=1, precision=PRECISION_FP32):
        Xd = X.detach().contiguous()
        Yd = Y.detach()
        lib_E = _i32(lib_E, Xd.device)
        n_lib, L = Xd.shape
        k_max = int(lib_E.max().item()) + 1 if n_lib else 2
        panel = Xd.t().contiguous()
        ids = torch.arange(n_lib, dtype=torch.int32, device=Xd.device)
        idx, w, _ = knn(panel, ids, lib_E, tau, 0, max(k_max, 2), want_d2=False)
        rho = crossmap_rho(Yd, idx, w, lib_E, tau, 0, int(Yd.shape[1]), precision)
        ctx.save_for_backward(Xd, Yd, idx, w, lib_E)
        ctx.tau = tau
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        X, Y, idx, w, lib_E = ctx.saved_tensors
        g = grad_rho.to(torch.float32)
        nz = torch.nonzero(g != 0)
        pair_lib = nz[:, 0].to(torch.int32)
        pair_tgt = nz[:, 1].to(torch.int32)
        gvals = g[nz[:, 0], nz[:, 1]].contiguous()
        # Y may be a view of a wider panel (row stride > N): the target gradient is written at
        # Y's strides, into an [L][ld] buffer whose [L][N] view is returned
        gts, glib = crossmap_rho_backward(Y, X, idx, w, lib_E, pair_lib, pair_tgt, gvals,
                                          ctx.tau)
        return glib, gts, None, None, None


def crossmap_rho_autograd(X, Y, lib_E, tau: int = 1, precision: int = PRECISION_FP32):
    """Differentiable rho block: see ``CrossMapRho``."""
    return CrossMapRho.apply(X, Y, lib_E, tau, precision)
