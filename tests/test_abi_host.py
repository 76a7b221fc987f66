"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and
rejects bad arguments before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest
import torch

import paper_2011_11082_amd as ccm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccm.h")

pytestmark = pytest.mark.skipif(not os.path.exists(ccm.LIB_PATH), reason="libccm.so not built")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:ccm_status|const char\*)\s+(ccm_\w+)\(", text, re.M)))


def test_header_declares_the_abi():
    syms = declared_symbols()
    for name in ("ccm_embed", "ccm_knn", "ccm_simplex_optE", "ccm_crossmap_rho",
                 "ccm_crossmap_rho_backward", "ccm_workspace_size"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ccm.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) <= set(ccm.EXPORTED)


def test_status_strings_and_version():
    lib = ccm.load_library()
    assert lib.ccm_status_string(0) == b"CCM_OK"
    assert b"workspace" in lib.ccm_status_string(5)
    assert lib.ccm_version().startswith(b"ccm-gfx950")


def test_check_finite_switch_is_host_only():
    lib = ccm.load_library()
    assert lib.ccm_set_check_finite(1) == ccm.CCM_OK
    assert lib.ccm_set_check_finite(0) == ccm.CCM_OK


def test_workspace_size_host_only():
    n = ccm.workspace_size(ccm.OP_CROSSMAP_FP32, 1600, 512, 101729, 21)
    # blocked tables: 512 libraries x 100 blocks x 6 slots x 64 lanes x (4 + 4) bytes
    assert n >= 512 * 100 * 6 * 64 * 8
    assert ccm.workspace_size(ccm.OP_KNN, 1600, 512, 0, 21) == 0
    with pytest.raises(ccm.CCMError) as e:
        ccm.workspace_size(99, 10, 1, 1, 2)
    assert e.value.status == ccm.CCM_EINVAL


def _null():
    return ctypes.c_void_p(0)


def test_argument_errors_return_status_before_device_work():
    lib = ccm.load_library()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation
    # NULL panel
    assert lib.ccm_knn(_null(), 8, 100, fake, fake, 1, 1, 0, 21, fake, fake, _null(), _null(), 0,
                       _null()) == ccm.CCM_EINVAL
    assert b"ts is NULL" in lib.ccm_last_error()
    # k_max out of range
    assert lib.ccm_knn(fake, 8, 100, fake, fake, 1, 1, 0, 22, fake, fake, _null(), _null(), 0,
                       _null()) == ccm.CCM_EINVAL
    # E range of simplex
    assert lib.ccm_simplex_optE(fake, 8, 100, fake, 1, 0, 5, 1, 1, 0, fake, _null(), _null(), 0,
                                _null()) == ccm.CCM_ERANGE
    assert lib.ccm_simplex_optE(fake, 8, 100, fake, 1, 1, 21, 1, 1, 0, fake, _null(), _null(), 0,
                                _null()) == ccm.CCM_ERANGE
    # too few points for E_max
    assert lib.ccm_simplex_optE(fake, 8, 20, fake, 1, 1, 20, 1, 1, 0, fake, _null(), _null(), 0,
                                _null()) == ccm.CCM_ERANGE
    # bad mode
    assert lib.ccm_simplex_optE(fake, 8, 100, fake, 1, 1, 5, 1, 1, 7, fake, _null(), _null(), 0,
                                _null()) == ccm.CCM_EINVAL
    # tau < 1, L too large
    assert lib.ccm_embed(fake, 8, 100, fake, 1, 2, 0, fake, _null()) == ccm.CCM_ERANGE
    assert lib.ccm_embed(fake, 8, 20000, fake, 1, 2, 1, fake, _null()) == ccm.CCM_ERANGE
    # no embedded point ((E-1) tau >= L) is a range error even when the (empty) output is
    # NULL; a NULL output with points to write is EINVAL
    assert lib.ccm_embed(fake, 8, 10, fake, 2, 6, 2, _null(), _null()) == ccm.CCM_ERANGE
    assert lib.ccm_embed(fake, 8, 11, fake, 2, 6, 2, _null(), _null()) == ccm.CCM_EINVAL
    # crossmap: workspace missing, targets past the panel, unknown precision
    assert lib.ccm_crossmap_rho(fake, 64, 100, fake, fake, fake, 4, 21, 1, 0, 64, 0, fake, _null(),
                                _null(), 0, _null()) == ccm.CCM_EWORKSPACE
    assert lib.ccm_crossmap_rho(fake, 64, 100, fake, fake, fake, 4, 21, 1, 10, 64, 0, fake,
                                _null(), _null(), 0, _null()) == ccm.CCM_EINVAL
    assert lib.ccm_crossmap_rho(fake, 64, 100, fake, fake, fake, 4, 21, 1, 0, 64, 9, fake, _null(),
                                _null(), 0, _null()) == ccm.CCM_EINVAL
    assert lib.ccm_crossmap_rho(fake, 64, 4000, fake, fake, fake, 4, 21, 1, 0, 64, 0, fake,
                                _null(), _null(), 0, _null()) == ccm.CCM_EWORKSPACE
    # the target tile sits in LDS up to L = 5035 (16, then 8 targets); beyond it the FP32
    # form keeps a global copy of every 32-target tile in the workspace
    short = ccm.workspace_size(ccm.OP_CROSSMAP_FP32, 5035, 4, 64, 21)
    long = ccm.workspace_size(ccm.OP_CROSSMAP_FP32, 5036, 4, 64, 21)
    assert long - short >= 2 * 5036 * 32 * 4 + 2 * 2 * 21 * 32 * 8
    # the testing switch: a forced global copy shows in the workspace (none at L = 2476 or
    # 1600 otherwise, nor with a forced LDS width); bad values are refused
    try:
        for L in (1600, 2476):
            auto = ccm.workspace_size(ccm.OP_CROSSMAP_FP32, L, 4, 64, 21)
            ccm.set_gather_tile(32)
            forced = ccm.workspace_size(ccm.OP_CROSSMAP_FP32, L, 4, 64, 21)
            ccm.set_gather_tile(8)
            assert ccm.workspace_size(ccm.OP_CROSSMAP_FP32, L, 4, 64, 21) == auto
            ccm.set_gather_tile(0)
            assert forced - auto >= 2 * L * 32 * 4 + 2 * 2 * 21 * 32 * 8
    finally:
        ccm.set_gather_tile(0)
    assert lib.ccm_set_gather_tile(12) == ccm.CCM_EINVAL
    assert lib.ccm_set_gather_tile(0) == ccm.CCM_OK


def test_backward_argument_errors():
    lib = ccm.load_library()
    fake = ctypes.c_void_p(0x1000)
    # both gradients NULL
    assert lib.ccm_crossmap_rho_backward(fake, 8, 100, fake, fake, fake, fake, 2, 4, 1, fake, fake,
                                         fake, 3, _null(), _null(), fake, 1 << 20,
                                         _null()) == ccm.CCM_EINVAL
    # workspace too small
    assert lib.ccm_crossmap_rho_backward(fake, 8, 100, fake, fake, fake, fake, 2, 4, 1, fake, fake,
                                         fake, 3, fake, fake, fake, 16, _null()) == ccm.CCM_EWORKSPACE
    # zero pairs: nothing to do
    assert lib.ccm_crossmap_rho_backward(fake, 8, 100, fake, fake, fake, fake, 2, 4, 1, fake, fake,
                                         fake, 0, fake, fake, _null(), 0, _null()) == ccm.CCM_OK
    n = ccm.workspace_size(ccm.OP_CROSSMAP_BACKWARD, 1000, 2048, 256, 21)
    assert n >= 256 * 1000 * 21 * 4


def test_target_E_argument_errors_and_workspace():
    lib = ccm.load_library()
    fake = ctypes.c_void_p(0x1000)
    f = lib.ccm_crossmap_rho_target_E
    # args: ts, ld, L, idx, w, n_lib, E_lo, n_E, k_max, tau, tgt_E, tgt0, n_tgt, rho, mom, ws,
    #       ws_bytes, stream
    assert f(fake, 64, 100, fake, fake, 4, 0, 5, 21, 1, fake, 0, 64, fake, _null(), fake, 1 << 30,
             _null()) == ccm.CCM_ERANGE                      # E_lo < 1
    assert f(fake, 64, 100, fake, fake, 4, 15, 8, 21, 1, fake, 0, 64, fake, _null(), fake, 1 << 30,
             _null()) == ccm.CCM_ERANGE                      # largest E 22 > CCM_E_MAX
    assert f(fake, 64, 100, fake, fake, 4, 1, 10, 8, 1, fake, 0, 64, fake, _null(), fake, 1 << 30,
             _null()) == ccm.CCM_ERANGE                      # k_max < largest E + 1
    assert f(fake, 64, 100, fake, fake, 4, 1, 5, 21, 1, _null(), 0, 64, fake, _null(), fake,
             1 << 30, _null()) == ccm.CCM_EINVAL             # tgt_E NULL
    assert f(fake, 64, 100, fake, fake, 4, 1, 5, 21, 1, fake, 8, 64, fake, _null(), fake, 1 << 30,
             _null()) == ccm.CCM_EINVAL                      # targets past the panel
    assert f(fake, 64, 100, fake, fake, 4, 1, 5, 21, 1, fake, 0, 64, fake, _null(), fake, 64,
             _null()) == ccm.CCM_EWORKSPACE
    need = ccm.workspace_size(ccm.OP_CROSSMAP_TARGET_E, 2476, 20, 64, 21)
    assert f(fake, 64, 2476, fake, fake, 4, 1, 5, 21, 1, fake, 0, 64, fake, _null(), fake,
             need - 1, _null()) == ccm.CCM_EWORKSPACE       # long series: tile copies
    # workspace grows with the number of (E, library) tables and covers the tile list
    a = ccm.workspace_size(ccm.OP_CROSSMAP_TARGET_E, 1600, 20 * 512, 101729, 21)
    b = ccm.workspace_size(ccm.OP_CROSSMAP_FP32, 1600, 20 * 512, 101729, 21)
    assert a >= b + 101729 * 4 + ((101729 + 15) // 16 + 21) * 12


def test_knn_subset_requires_a_mask():
    lib = ccm.load_library()
    fake = ctypes.c_void_p(0x1000)
    assert lib.ccm_knn_subset(fake, 8, 100, fake, fake, 2, 1, 0, 21, _null(), fake, fake, _null(),
                              _null(), 0, _null()) == ccm.CCM_EINVAL
    assert b"cand_mask" in lib.ccm_last_error()
    # no libraries: nothing to do
    assert lib.ccm_knn_subset(fake, 8, 100, fake, fake, 0, 1, 0, 21, _null(), fake, fake, _null(),
                              _null(), 0, _null()) == ccm.CCM_OK


def test_matrix_argument_errors_before_device_work():
    # rejected before any device call (a CPU tensor never reaches the library)
    x = torch.zeros((100, 8), dtype=torch.float32)
    with pytest.raises(ValueError):
        ccm.ccm_matrix(x, per_target_E=True, precision=ccm.PRECISION_BF16)
    with pytest.raises(ValueError):
        ccm.ccm_matrix(x, block=0)


def test_backward_workspace_is_bounded_by_chunks():
    # pairs run in chunks: the workspace stops growing once a chunk is full, and a chunk
    # never exceeds 65,535 pairs or 4 GiB of per-pair buffers
    lib = ccm.load_library()
    lib.ccm_backward_chunk_pairs.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.ccm_backward_chunk_pairs.restype = ctypes.c_int32
    for L, k_max in ((1600, 21), (100, 3), (16384, 21), (8, 2)):
        c = lib.ccm_backward_chunk_pairs(L, k_max)
        per = 6 * L * 4 + 2 * L * k_max * 4 + 21 * L * 8 + 8
        assert 1 <= c <= 65535 and c * per <= 4 << 30
        at_chunk = ccm.workspace_size(ccm.OP_CROSSMAP_BACKWARD, L, 64, c, k_max)
        assert ccm.workspace_size(ccm.OP_CROSSMAP_BACKWARD, L, 64, 2_000_000_000, k_max) == at_chunk
        assert ccm.workspace_size(ccm.OP_CROSSMAP_BACKWARD, L, 64, max(c - 1, 0), k_max) <= at_chunk
    # 52 M pairs (a dense rho.sum() over a 512 x 101,729 block) at L = 1600: about 4 GiB plus
    # the per-library lists
    n = ccm.workspace_size(ccm.OP_CROSSMAP_BACKWARD, 1600, 512, 512 * 101729, 21)
    assert n < (4 << 30) + 16 * 512 * 1601 * 21 + 4 * 512 * 1601 + (1 << 20)


def test_storage_span_check():
    # the host-side bound the backward applies before handing raw pointers to the kernels:
    # an [L][N] view of a wider panel covers (L-1) ld + N elements from its first element
    wide = torch.zeros((10, 12))
    v = wide[:, 3:8]                         # L = 10, N = 5, ld = 12, storage offset 3
    L, N, ld = 10, 5, v.stride(0)
    assert ccm.storage_span_ok(v, 0, (L - 1) * ld + N - 1)
    assert ccm.storage_span_ok(v, 0, (L - 1) * ld + 8)          # up to the storage's last element
    assert not ccm.storage_span_ok(v, 0, (L - 1) * ld + 9)      # one past it
    # a contiguous [L][N] buffer written with the wider row stride would overflow: the bug a
    # backward through a column slice of a panel had when its gradient was allocated [L][N]
    tight = torch.zeros((L, N))
    assert not ccm.storage_span_ok(tight, 0, (L - 1) * ld + N - 1)
    assert ccm.storage_span_ok(torch.zeros((L, ld))[:, :N], 0, (L - 1) * ld + N - 1)
    assert ccm.storage_span_ok(tight, 5, 4)                      # empty range


def test_noalloc_optE_argument_errors_before_device_work():
    # the allocation-free optE checks its arguments and its size limit on the host, before
    # it looks up its static scratch or launches anything
    lib = ccm.load_library()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    assert lib.ccm_simplex_optE_noalloc(fake, 8, 100, fake, ccm.NOALLOC_MAX_SERIES + 1, 1, 10,
                                        1, 1, 0, fake, _null(), _null()) == ccm.CCM_ERANGE
    assert b"CCM_NOALLOC_MAX_SERIES" in lib.ccm_last_error()
    assert lib.ccm_simplex_optE_noalloc(fake, 8, 100, fake, 1, 0, 5, 1, 1, 0, fake, _null(),
                                        _null()) == ccm.CCM_ERANGE
    assert lib.ccm_simplex_optE_noalloc(_null(), 8, 100, fake, 1, 1, 5, 1, 1, 0, fake, _null(),
                                        _null()) == ccm.CCM_EINVAL
    assert lib.ccm_simplex_optE_noalloc(fake, 8, 100, fake, 1, 1, 5, 1, 1, 7, fake, _null(),
                                        _null()) == ccm.CCM_EINVAL
    assert lib.ccm_simplex_optE_noalloc(fake, 8, 100, fake, 0, 1, 5, 1, 1, 0, fake, _null(),
                                        _null()) == ccm.CCM_OK
    # the limit in the header and in the binding agree with the library's
    text = open(HEADER).read()
    assert f"#define CCM_NOALLOC_MAX_SERIES {ccm.NOALLOC_MAX_SERIES}" in text
