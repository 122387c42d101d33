"""kifmm_nn_max_abs_noalloc (the entry point that allocates nothing: its partial maxima live in
a static device array) against kifmm_nn_max_abs with a caller's workspace, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2006_03515_amd import kifmm
    return kifmm


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _with_workspace(K, x, batch, per, recip):
    out = torch.empty(batch, dtype=torch.float32, device="cuda")
    work = torch.empty(batch * 256, dtype=torch.float32, device="cuda")
    rc = K._lib.kifmm_nn_max_abs(batch, per, _p(x), _p(out), recip, _p(work), work.numel(), _stream())
    assert rc == K.OK, K._lib.kifmm_last_error()
    return out


def _no_alloc(K, x, batch, per, recip):
    out = torch.full((batch,), -7.0, dtype=torch.float32, device="cuda")
    rc = K._lib.kifmm_nn_max_abs_noalloc(batch, per, _p(x), _p(out), recip, _stream())
    assert rc == K.OK, K._lib.kifmm_last_error()
    return out


def test_no_alloc_max_abs_equals_the_workspace_entry_point(K):
    rng = np.random.default_rng(7)
    # two calls in a row, the second smaller: the second must not see the first's partials
    for batch, per, recip in ((6, 64 ** 3, 0), (3, 5000, 1)):
        x = torch.from_numpy(rng.standard_normal(batch * per).astype(np.float32) *
                             np.repeat(10.0 ** rng.uniform(-3, 3, batch), per).astype(np.float32)).cuda()
        a = _no_alloc(K, x, batch, per, recip)
        b = _with_workspace(K, x, batch, per, recip)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (batch, per)
        ref = np.abs(x.cpu().numpy().reshape(batch, per)).max(axis=1)
        if recip:
            np.testing.assert_allclose(a.cpu().numpy(), 1.0 / ref.astype(np.float64), rtol=2e-7)
        else:
            np.testing.assert_array_equal(a.cpu().numpy(), ref.astype(np.float32))
    # a zero field: max 0, reciprocal 1
    z = torch.zeros(2 * 300, dtype=torch.float32, device="cuda")
    assert torch.equal(_no_alloc(K, z, 2, 300, 1), torch.ones(2, device="cuda"))


def test_no_alloc_rejects_sizes_beyond_its_scratch(K):
    # batch * min(256, ceil(per / 256)) > 262144 floats: refused on the host, before any launch
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    out = torch.zeros(2048, dtype=torch.float32, device="cuda")
    rc = K._lib.kifmm_nn_max_abs_noalloc(2048, 1 << 20, _p(x), _p(out), 0, _stream())
    assert rc == K.EINVAL
    assert b"scratch" in K._lib.kifmm_last_error()
    assert int(torch.count_nonzero(out)) == 0
