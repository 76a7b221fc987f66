"""The allocation-free optE entry point, ccm_simplex_optE_noalloc, called through the C ABI,
against the workspace form ccm_simplex_optE on the same inputs: optE equal and every skill
bit-identical (the two share their kernels), over two calls in a row where the second is
smaller (the static scratch keeps the first call's values), plus its size limit."""
import sys

import numpy as np
import pytest

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


def _same(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return a.shape == b.shape and np.array_equal(a, b, equal_nan=True)


def test_noalloc_optE_matches_workspace_form(ccm):
    import torch

    ts = synth.make("ratenet1024").panel
    d = torch.as_tensor(ts).cuda()
    cases = [
        # (first series, n, E_min, E_max, mode): the second call is smaller
        (0, 700, 1, 20, ccm.MODE_LOO),
        (301, 45, 2, 9, ccm.MODE_HALF),
    ]
    for s0, n, E_min, E_max, mode in cases:
        _say(f"noalloc optE: {n} series from {s0}, E {E_min}..{E_max}, mode {mode}")
        ids = torch.arange(s0, s0 + n, dtype=torch.int32, device="cuda")
        ref_E, ref_rho = ccm.simplex_optE(d, ids, E_min, E_max, 1, 1, mode)
        optE = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        rho = torch.full((n, E_max - E_min + 1), -3.0, dtype=torch.float32, device="cuda")
        ccm.simplex_optE_noalloc(d, ids, optE, rho, E_min, E_max, 1, 1, mode)
        torch.cuda.synchronize()
        assert _same(optE, ref_E), "optE differs from ccm_simplex_optE"
        assert _same(rho, ref_rho), "skills differ from ccm_simplex_optE"


def test_noalloc_optE_size_limit(ccm):
    import torch

    ts = synth.make("logistic64").panel
    d = torch.as_tensor(ts).cuda()
    n = ccm.NOALLOC_MAX_SERIES + 1
    _say(f"noalloc optE: {n} series is refused on the host")
    ids = torch.zeros(n, dtype=torch.int32, device="cuda")
    optE = torch.zeros(n, dtype=torch.int32, device="cuda")
    rho = torch.zeros((n, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(ccm.CCMError) as ei:
        ccm.simplex_optE_noalloc(d, ids, optE, rho, 1, 10, 1, 1)
    assert ei.value.status == ccm.CCM_ERANGE
    assert "CCM_NOALLOC_MAX_SERIES" in str(ei.value)
