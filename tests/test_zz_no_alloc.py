"""The allocation-free forward (project_fwd_noalloc) against project_fwd,
through the C ABI: two calls in a row, the second with a smaller batch (the
scratch keeps the first call's contents), list-mode rows, and the size and
mode checks."""
import ctypes as C

import numpy as np
import pytest

from paper_1607_06170_amd import _lib
from paper_1607_06170_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _call(sc, t, x, y, events=None, n_events=0):
    import torch
    o = sc.opts()
    tc = t.c()
    ev = C.c_void_p(events.data_ptr()) if events is not None else C.c_void_p(0)
    r = sc.L.project_fwd_noalloc(sc.h, C.byref(tc), C.byref(o), C.c_void_p(x.data_ptr()), x.shape[0], ev,
                                 n_events, C.c_void_p(y.data_ptr()),
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return r


def test_noalloc_forward_matches_workspace_forward(torch):
    from paper_1607_06170_amd import Scanner
    sc = Scanner(S.CFG_2D)
    t = sc.build_table(61, 4, 1.0)
    for batch, seed in ((9, 41), (2, 42)):
        x = torch.tensor(S.phantom_uniform(S.CFG_2D, seed=seed, batch=batch), dtype=torch.float32, device="cuda")
        ref = sc.project_fwd(t, x)
        y = torch.full((batch, sc.n_bins), float("nan"), device="cuda")
        assert _call(sc, t, x, y) == _lib.PSF_OK
        np.testing.assert_allclose(y.cpu().numpy(), ref.cpu().numpy(), rtol=1e-6, atol=0)
        # list-mode rows of some events
        rng = np.random.default_rng(seed)
        bins = rng.integers(0, sc.n_bins, 500)
        i, j = S.bin_to_pair(bins, sc.n_crystals)
        ev = torch.tensor(np.stack([i, j], 1), dtype=torch.int32, device="cuda").contiguous()
        q_ref = sc.project_fwd(t, x, events=ev)
        q = torch.full((batch, 500), float("nan"), device="cuda")
        assert _call(sc, t, x, q, ev, 500) == _lib.PSF_OK
        np.testing.assert_allclose(q.cpu().numpy(), q_ref.cpu().numpy(), rtol=1e-6, atol=0)


def test_noalloc_forward_limits(torch):
    from paper_1607_06170_amd import Scanner
    sc = Scanner(S.CFG_2D)
    t = sc.build_table(61, 4, 1.0)
    x = torch.zeros(259, sc.n_voxels, device="cuda")
    y = torch.zeros(259, sc.n_bins, device="cuda")
    assert _call(sc, t, x, y) == _lib.PSF_ESIZE            # 259 images exceed the 16 MiB scratch
    assert _call(sc, t, x[:258], y[:258]) == _lib.PSF_OK    # 258 fit
    sc3 = Scanner(S.CFG_3D_SMALL, mode3d=True)
    t3 = sc3.build_table(91, 4, 1.0)
    x3 = torch.zeros(1, sc3.n_voxels, device="cuda")
    y3 = torch.zeros(1, sc3.n_bins, device="cuda")
    assert _call(sc3, t3, x3, y3) == _lib.PSF_EUNSUPPORTED
