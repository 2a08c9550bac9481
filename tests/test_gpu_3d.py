"""GPU parity of the 3D-scanner path against the FP64 oracle, through the C ABI.

Bar: bins and the CSR sparsity pattern bit-exact (voxels whose decisions the
oracle flags as within a hair of a boundary are excused from the pattern
check only); values within 1e-5 relative (FP32 plain form); projections
within 1e-5 relative to the largest entry.
"""
import numpy as np
import pytest

from paper_1607_06170_amd import synth as S

pytestmark = pytest.mark.gpu

SMALL = S.CFG_3D_SMALL
CFG3 = S.CFG_3D
RTOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _scanner(cfg):
    from paper_1607_06170_amd import Scanner
    return Scanner(cfg, mode3d=True)


def _progress(msg):
    """A progress line for the long full-volume tests (seen with pytest -s)."""
    import sys
    import time
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _unbin3(b, cfg):
    Nc = cfg["n_blocks"] * cfg["n_ct"]
    NR = cfg["n_cz"] * cfg["n_brings"]
    tb, rest = b // (NR * NR), b % (NR * NR)
    gi, gj = S.bin_to_pair(tb, Nc)
    return gi.astype(np.int64), rest // NR, gj.astype(np.int64), rest % NR


@pytest.fixture(scope="module")
def small_ref(oracle):
    nr = SMALL["n_rows"]
    td = S.random_table((nr, nr, 4, 4, 5, 5), seed=12)
    tab = oracle.TableRef(td, nr, 4, 1.0)
    n = SMALL["nx"] * SMALL["ny"] * SMALL["nz"]
    cols, flags = oracle.columns_3d(SMALL, tab, np.arange(n), cap=1 << 16)
    return td, cols, flags


def _sparse(cols, nbins):
    import scipy.sparse as sp
    rows = np.concatenate([np.full(len(b), k) for k, (b, _) in enumerate(cols)])
    cidx = np.concatenate([b for b, _ in cols])
    vals = np.concatenate([v for _, v in cols])
    return sp.csr_matrix((vals, (rows, cidx)), shape=(len(cols), nbins))


def test_table3_parity(torch, oracle):
    sc = _scanner(CFG3)
    t = sc.build_table(61, 4, 1.0)
    got = t.data.cpu().numpy().reshape(61, 61, 4, 4, 5, 5).astype(np.float64)
    rt, rz = np.meshgrid(np.arange(61), np.arange(61), indexing="ij")   # every one of the 3721 row pairs
    ref = oracle.table3_rows(CFG3, rt.ravel(), rz.ravel(), 4, 1.0, 16).reshape(61, 61, 4, 4, 5, 5)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-9)


def _check_rows(oracle, rp, col, val, cols, flags, vox):
    rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    exact = 0
    for r, v in enumerate(vox):
        g = col[rp[r]:rp[r + 1]].astype(np.int64)
        gv = val[rp[r]:rp[r + 1]]
        ob, ov = cols[v]
        if flags[v] & oracle.F_TIES == 0:
            assert np.array_equal(g, ob), f"voxel {v}: pattern differs ({len(g)} vs {len(ob)})"
            np.testing.assert_allclose(gv, ov, rtol=RTOL, atol=0, err_msg=f"voxel {v}")
            exact += 1
        else:
            m = dict(zip(ob.tolist(), ov.tolist()))
            common = [k for k in range(len(g)) if int(g[k]) in m]
            np.testing.assert_allclose(gv[common], [m[int(g[k])] for k in common], rtol=RTOL)
    assert exact >= 0.95 * len(vox)


def test_sysmat_small_scanner(torch, oracle, small_ref):
    td, cols, flags = small_ref
    nr = SMALL["n_rows"]
    sc = _scanner(SMALL)
    t = sc.table_from(td, nr, 4, 1.0)
    rp, col, val = sc.build_psf_sysmat(t, threshold=0.0)
    _check_rows(oracle, rp, col, val, cols, flags, np.arange(len(cols)))


@pytest.mark.parametrize("vb,ve", [(0, 1), (17, 50), (583, 600)])
def test_sysmat_small_ranges(torch, oracle, small_ref, vb, ve):
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    rp, col, val = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=vb, vox_end=ve)
    _check_rows(oracle, rp, col, val, cols, flags, np.arange(vb, ve))


def test_sysmat_class_order(torch, oracle, small_ref):
    """Ranges of the library's voxel order (voxels sharing tiles side by side):
    the order lists every voxel once, and two ranges that cut a group of
    sharing voxels build each voxel's row as the oracle does."""
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    order = sc.voxel_order()
    n = sc.n_voxels
    assert np.array_equal(np.sort(order), np.arange(n))
    for vb, ve in ((0, 301), (301, n), (17, 19)):
        rp, col, val = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=vb, vox_end=ve, class_order=True)
        _check_rows(oracle, rp, col, val, cols, flags, order[vb:ve])


def test_sysmat_staging_paths(torch, oracle, small_ref):
    """The fill phase copies what the count phase staged; without staging, or
    when another call used the workspace in between, it recomputes: the three
    give the same matrix."""
    import ctypes as C
    from paper_1607_06170_amd import _lib
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    vb, ve = 40, 230
    ref = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=vb, vox_end=ve, stage=False)
    got = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=vb, vox_end=ve, stage=True)
    # same pattern; values equal up to the order of the FP32 atomic sums
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    np.testing.assert_allclose(got[2].cpu().numpy(), ref[2].cpu().numpy(), rtol=1e-6)
    # count phase, then a projection on the same workspace, then the fill phase
    o = sc.opts(0, 0.0, vb, ve, flags=_lib.PSF_OPT_STAGE_CSR)
    ws = sc.workspace(t, 1, 0, o)
    tc = t.c()
    n = ve - vb
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    csr = _lib.psf_csr(n, 0, row_ptr.data_ptr(), None, None)
    ptr = lambda x: C.c_void_p(x.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(sc.L.build_psf_sysmat(sc.h, C.byref(tc), C.byref(o), ptr(ws), ws.numel(), C.byref(csr), stream), "count")
    sc.project_fwd(t, torch.ones(1, sc.n_voxels, device="cuda"))
    col = torch.empty(csr.nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(csr.nnz, dtype=torch.float32, device="cuda")
    csr.col, csr.val = col.data_ptr(), val.data_ptr()
    _lib.check(sc.L.build_psf_sysmat(sc.h, C.byref(tc), C.byref(o), ptr(ws), ws.numel(), C.byref(csr), stream), "fill")
    assert torch.equal(row_ptr, ref[0]) and torch.equal(col, ref[1])
    np.testing.assert_allclose(val.cpu().numpy(), ref[2].cpu().numpy(), rtol=1e-6)
    _check_rows(oracle, row_ptr, col, val, cols, flags, np.arange(vb, ve))


def test_sysmat_clean_workspace_flag(torch, oracle, small_ref):
    """PSF_OPT_WS_CLEAN skips clearing the build's accumulators only when the
    workspace header records a completed build of this handle and layout: on a
    workspace of arbitrary bytes the build still clears them, and a build after
    a projection on the same workspace (the Scanner sets the flag) gives the
    same matrix."""
    import ctypes as C
    from paper_1607_06170_amd import _lib
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    vb, ve = 0, 200
    ref = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=vb, vox_end=ve, stage=False)
    # a foreign workspace full of ones, with the flag: the header does not match, so the build clears
    o = sc.opts(0, 0.0, vb, ve, flags=_lib.PSF_OPT_WS_CLEAN)
    n_ws = C.c_size_t()
    tc = t.c()
    _lib.check(sc.L.psf_workspace_size(sc.h, C.byref(tc), C.byref(o), 1, 0, C.byref(n_ws)), "size")
    ws = torch.ones(n_ws.value, dtype=torch.uint8, device="cuda")
    n = ve - vb
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    csr = _lib.psf_csr(n, 0, row_ptr.data_ptr(), None, None)
    ptr = lambda x: C.c_void_p(x.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(sc.L.build_psf_sysmat(sc.h, C.byref(tc), C.byref(o), ptr(ws), ws.numel(), C.byref(csr), stream), "count")
    col = torch.empty(csr.nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(csr.nnz, dtype=torch.float32, device="cuda")
    csr.col, csr.val = col.data_ptr(), val.data_ptr()
    _lib.check(sc.L.build_psf_sysmat(sc.h, C.byref(tc), C.byref(o), ptr(ws), ws.numel(), C.byref(csr), stream), "fill")
    assert torch.equal(row_ptr, ref[0]) and torch.equal(col, ref[1])
    np.testing.assert_allclose(val.cpu().numpy(), ref[2].cpu().numpy(), rtol=1e-6)
    del ws
    # the Scanner's own workspace: a projection, then a build that trusts the accumulators
    sc.project_fwd(t, torch.ones(1, sc.n_voxels, device="cuda"))
    assert sc._ws_clean
    got = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=vb, vox_end=ve, stage=False)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    np.testing.assert_allclose(got[2].cpu().numpy(), ref[2].cpu().numpy(), rtol=1e-6)
    _check_rows(oracle, got[0], got[1], got[2], cols, flags, np.arange(vb, ve))


# offsets chosen so that no voxel's angle-row decision sits on a rounding tie
@pytest.mark.parametrize("shift", [dict(nx=9, cx=0.137), dict(nx=9, cx=0.137, cz=0.291)],
                         ids=["axial-mirror-only", "no-symmetry"])
def test_sysmat_and_projections_off_centre(torch, oracle, small_ref, shift):
    """Images the square's symmetry does not map onto themselves (non-square,
    off-centre): classes keep one column, and join their axial mirror run only
    when the image is centred axially (first case).  Every row and both
    projections against the oracle."""
    cfg = dict(SMALL, **shift)
    td = small_ref[0]
    nr = cfg["n_rows"]
    tab = oracle.TableRef(td, nr, 4, 1.0)
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    cols, flags = oracle.columns_3d(cfg, tab, np.arange(n), cap=1 << 16)
    sc = _scanner(cfg)
    t = sc.table_from(td, nr, 4, 1.0)
    rp, col, val = sc.build_psf_sysmat(t, threshold=0.0)
    _check_rows(oracle, rp, col, val, cols, flags, np.arange(n))
    A_T = _sparse(cols, sc.n_bins)
    x = S.phantom_uniform(cfg, seed=9, batch=1)
    xf = x.astype(np.float32).astype(np.float64)
    y = sc.project_fwd(t, torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    yo = (A_T.T @ xf.T).T
    np.testing.assert_allclose(y, yo, rtol=RTOL, atol=RTOL * 1e-2 * np.abs(yo).max())
    xb = sc.project_adj(t, torch.tensor(yo, dtype=torch.float32, device="cuda")).cpu().numpy()
    xbo = (A_T @ yo.astype(np.float32).astype(np.float64).T).T
    np.testing.assert_allclose(xb, xbo, rtol=RTOL, atol=RTOL * 1e-2 * np.abs(xbo).max())
    sc.check()


def test_projections_small_scanner(torch, oracle, small_ref):
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    A_T = _sparse(cols, sc.n_bins)          # voxels x bins
    x = S.phantom_uniform(SMALL, seed=7, batch=2)
    xf = x.astype(np.float32).astype(np.float64)
    y = sc.project_fwd(t, torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    yo = (A_T.T @ xf.T).T
    np.testing.assert_allclose(y, yo, rtol=RTOL, atol=RTOL * 1e-2 * np.abs(yo).max())
    rng = np.random.default_rng(8)
    yc = rng.poisson(50.0 * yo / yo.max()).astype(np.float64)
    xb = sc.project_adj(t, torch.tensor(yc, dtype=torch.float32, device="cuda")).cpu().numpy()
    xbo = (A_T @ yc.T).T
    np.testing.assert_allclose(xb, xbo, rtol=RTOL, atol=RTOL * 1e-2 * np.abs(xbo).max())
    s = sc.sensitivity(t).cpu().numpy()
    np.testing.assert_allclose(s, np.asarray(A_T.sum(axis=1)).ravel(), rtol=RTOL)
    sc.check()


def test_precision_forms_small_scanner(torch, oracle, small_ref):
    """BF16 operands (U and X = W V rounded) with FP32 accumulation, and the
    hi/lo split: error against FP64, per element and per projection entry.
    The bounds are 1e-2 per element and 1e-3 per projection entry (entries
    above 1e-3 of the largest): the hi/lo form meets both; plain BF16 meets the
    element bound and, per projection entry, only 1e-2 (its rounding of U and
    X leaves each product up to about 2^-8 off, and an entry sums few of them)."""
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    A_T = _sparse(cols, sc.n_bins)
    x = S.phantom_uniform(SMALL, seed=7)
    yo = (A_T.T @ x[0])
    big = yo > 1e-3 * yo.max()
    for prec, e_tol, p_tol in [(1, 1e-2, 1e-2), (2, 1e-4, 1e-4)]:   # hi/lo: within the 1e-3 projection bound tenfold
        rp, col, val = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=100, vox_end=140, precision=prec)
        rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
        for r in range(40):
            b, v = cols[100 + r]
            g = col[rp[r]:rp[r + 1]]
            assert np.array_equal(g, b)
            assert (np.abs(val[rp[r]:rp[r + 1]] - v) / v).max() <= e_tol
        y = sc.project_fwd(t, torch.tensor(x, dtype=torch.float32, device="cuda"), precision=prec).cpu().numpy()[0]
        assert (np.abs(y - yo)[big] / yo[big]).max() <= p_tol
        ya = yo.astype(np.float32)
        xo = A_T @ ya.astype(np.float64)
        xa = sc.project_adj(t, torch.tensor(ya[None], device="cuda"), precision=prec).cpu().numpy()[0]
        bigx = xo > 1e-3 * xo.max()
        assert (np.abs(xa - xo)[bigx] / xo[bigx]).max() <= p_tol


def _events3(oracle, cfg, A_T, x, n_true, n_rand, seed):
    yo = A_T.T @ x
    bins = S.sample_events(yo, n_true, n_rand, seed=seed)
    gi, ri, gj, rj = _unbin3(bins, cfg)
    Nc = cfg["n_blocks"] * cfg["n_ct"]
    i, j = ri * Nc + gi, rj * Nc + gj
    rng = np.random.default_rng(seed + 1)
    sw = rng.random(len(bins)) < 0.5
    return bins, np.stack([np.where(sw, j, i), np.where(sw, i, j)], 1).astype(np.int32)


def test_listmode_small_scanner(torch, oracle, small_ref):
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    A_T = _sparse(cols, sc.n_bins)
    x = S.phantom_uniform(SMALL, seed=9)[0]
    bins, ev = _events3(oracle, SMALL, A_T, x, 20_000, 2_000, 300)
    evd = torch.tensor(ev, device="cuda")
    q = sc.project_fwd(t, torch.tensor(x[None], dtype=torch.float32, device="cuda"), events=evd).cpu().numpy()[0]
    qo = A_T[:, bins].T @ x.astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(q, qo, rtol=RTOL, atol=RTOL * 1e-2 * qo.max())
    sens = sc.sensitivity(t)
    M, r = 10, 0.1 * float((A_T.T @ x).mean())
    x0 = np.ones(sc.n_voxels)
    sub = slice(0, 5_000)
    xg = sc.lm_osem_update(t, evd[sub], torch.tensor(x0, dtype=torch.float32, device="cuda"), sens, M, r)
    sc.check()
    s_o = np.asarray(A_T.sum(axis=1)).ravel()
    q0 = A_T[:, bins[sub]].T @ x0 + r
    back = A_T[:, bins[sub]] @ (1.0 / q0)
    xo = np.where(s_o > 0, x0 / (s_o / M) * back, 0.0)
    np.testing.assert_allclose(xg.cpu().numpy(), xo, rtol=2e-5, atol=2e-5 * xo.max())


def test_table_gradient_zero_entries(torch, oracle):
    """A table with zero entries (the analytic table's one-sided neighbours are
    zero): the gradient at a zero entry is not zero, since the bin it would
    feed still carries a weight; every entry's gradient against the oracle's."""
    nr = SMALL["n_rows"]
    td = S.random_table((nr, nr, 4, 4, 5, 5), seed=13)
    rng = np.random.default_rng(78)
    td[rng.random(td.shape) < 0.4] = 0.0
    td[..., :2, :] = 0.0  # whole transaxial neighbour columns empty
    sc = _scanner(SMALL)
    t = sc.table_from(td, nr, 4, 1.0)
    n = sc.n_voxels
    vox = np.sort(rng.choice(n, 40, replace=False))
    xt = np.zeros((1, n))
    xt[0, vox] = rng.random(40)
    gy = rng.random((1, sc.n_bins))
    xf = xt.astype(np.float32).astype(np.float64)
    gf = gy.astype(np.float32).astype(np.float64)
    ref = oracle.table_grad_3d(SMALL, oracle.TableRef(td, nr, 4, 1.0), vox, xf[0, vox], np.arange(sc.n_bins), gf[0])
    _, grad = sc.project_adj(t, torch.tensor(gy, dtype=torch.float32, device="cuda"),
                             xt=torch.tensor(xt, dtype=torch.float32, device="cuda"), want_table_grad=True)
    sc.check()
    grad = grad.cpu().numpy().reshape(ref.shape)
    at_zero = (td == 0) & (ref != 0)
    assert at_zero.sum() > 1000
    np.testing.assert_allclose(grad, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())


def test_deterministic_build_small_scanner(torch, oracle, small_ref):
    """PSF_OPT_DETERMINISTIC: integer sums of the tile entries.  Two builds
    give the same CSR bit for bit; each entry meets the oracle within 1e-5
    relative plus the integer sums' rounding (2^-63 per tile entry); the
    default build (FP32 atomics, summed in arrival order) meets the
    deterministic one within its own FP32 rounding, entry by entry."""
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    runs = [[a.cpu().numpy() for a in sc.build_psf_sysmat(t, threshold=0.0, deterministic=True)] for _ in range(2)]
    for a, b in zip(*runs):
        assert a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))
    rp, col, val = runs[0]
    floor = 2.0 ** -56  # 128 tile entries' rounding
    exact = 0
    for v in range(len(cols)):
        g = col[rp[v]:rp[v + 1]].astype(np.int64)
        gv = val[rp[v]:rp[v + 1]].astype(np.float64)
        ob, ov = cols[v]
        m = dict(zip(ob.tolist(), ov.tolist()))
        assert all(int(b) in m for b in g), f"voxel {v}: a bin the oracle does not have"
        if flags[v] & oracle.F_TIES == 0:
            big = ob[ov > floor]
            assert np.isin(big, g).all(), f"voxel {v}: an oracle entry above 2^-56 missing"
            exact += 1
        ref = np.array([m[int(b)] for b in g])
        assert np.all(np.abs(gv - ref) <= RTOL * ref + floor), f"voxel {v}"
    assert exact >= 0.95 * len(cols)
    rpf, colf, valf = (a.cpu().numpy() for a in sc.build_psf_sysmat(t, threshold=0.0))
    for v in range(len(cols)):
        gd, vd = col[rp[v]:rp[v + 1]], val[rp[v]:rp[v + 1]].astype(np.float64)
        gf, vf = colf[rpf[v]:rpf[v + 1]], valf[rpf[v]:rpf[v + 1]].astype(np.float64)
        both, id_, if_ = np.intersect1d(gd, gf, return_indices=True)
        assert np.all(np.abs(vd[id_] - vf[if_]) <= 1e-6 * vf[if_] + floor), f"voxel {v}"
        only = np.setxor1d(gd, gf)
        assert np.all(np.concatenate([vd[np.isin(gd, only)], vf[np.isin(gf, only)]]) <= floor), f"voxel {v}"


def test_deterministic_build_errors(torch, small_ref):
    """A tile entry outside [0, 1) cannot be summed as a 2^-62 integer: the
    deterministic build says so (PSF_ERANGE); projections refuse the flag."""
    import ctypes as C
    from paper_1607_06170_amd import PsfError, _lib
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td * 1e4, SMALL["n_rows"], 4, 1.0)
    with pytest.raises(PsfError) as e:
        sc.build_psf_sysmat(t, threshold=0.0, deterministic=True)
    assert e.value.code == _lib.PSF_ERANGE
    o = sc.opts(flags=_lib.PSF_OPT_DETERMINISTIC)
    x = torch.zeros(1, sc.n_voxels, device="cuda")
    y = torch.empty(1, sc.n_bins, device="cuda")
    ws = sc.workspace(t, 1, 0, o)
    tc = t.c()
    code = sc.L.project_fwd(sc.h, C.byref(tc), C.byref(o), C.c_void_p(x.data_ptr()), 1, None, 0,
                            C.c_void_p(y.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert code == _lib.PSF_EUNSUPPORTED


def test_table_gradient_small_scanner(torch, oracle, small_ref):
    """d <y, A xt> / d table (two images, all bins weighted) against the
    oracle's, and the autograd wrapper against the direct call."""
    from paper_1607_06170_amd import PsfProject
    td, cols, flags = small_ref
    nr = SMALL["n_rows"]
    sc = _scanner(SMALL)
    t = sc.table_from(td, nr, 4, 1.0)
    n = sc.n_voxels
    rng = np.random.default_rng(77)
    xt = np.zeros((2, n))
    vox = [np.sort(rng.choice(n, 30, replace=False)) for _ in range(2)]
    for b in range(2):
        xt[b, vox[b]] = rng.random(30)
    gy = rng.random((2, sc.n_bins))
    xf = xt.astype(np.float32).astype(np.float64)
    gf = gy.astype(np.float32).astype(np.float64)
    tab_o = oracle.TableRef(td, nr, 4, 1.0)
    allb = np.arange(sc.n_bins)
    ref = sum(oracle.table_grad_3d(SMALL, tab_o, vox[b], xf[b, vox[b]], allb, gf[b]) for b in range(2))
    xd = torch.tensor(xt, dtype=torch.float32, device="cuda")
    gyd = torch.tensor(gy, dtype=torch.float32, device="cuda")
    xb, grad = sc.project_adj(t, gyd, xt=xd, want_table_grad=True)
    sc.check()
    grad = grad.cpu().numpy().reshape(ref.shape)
    assert np.count_nonzero(ref) > 1000
    np.testing.assert_allclose(grad, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())
    # the adjoint returned with it is the plain one
    A_T = _sparse(cols, sc.n_bins)
    np.testing.assert_allclose(xb.cpu().numpy(), (A_T @ gf.T).T, rtol=RTOL, atol=RTOL * 1e-2 * np.abs(xb.cpu().numpy()).max())
    # autograd: backward of <gy, y(xt, table)>
    tdat = t.data.clone().requires_grad_(True)
    xr = xd.clone().requires_grad_(True)
    y = PsfProject.apply(xr, tdat, sc, (nr, 4, 1.0))
    (y * gyd).sum().backward()
    np.testing.assert_allclose(tdat.grad.cpu().numpy().reshape(ref.shape), ref, rtol=1e-5,
                               atol=1e-6 * np.abs(ref).max())
    np.testing.assert_allclose(xr.grad.cpu().numpy(), xb.cpu().numpy(), rtol=1e-6)


@pytest.mark.parametrize("ijk", [(64, 64, 48), (20, 100, 3)])
def test_sysmat_full_scanner_sampled(torch, oracle, ijk):
    """The 128 x 128 x 96 configuration: single voxels' rows against the oracle."""
    ix, iy, iz = ijk
    v = (iz * 128 + iy) * 128 + ix
    td = S.random_table((61, 61, 4, 4, 5, 5), seed=13, scale=0.3)
    tab = oracle.TableRef(td, 61, 4, 1.0)
    cols, flags = oracle.columns_3d(CFG3, tab, [v], cap=1 << 22)
    sc = _scanner(CFG3)
    t = sc.table_from(td, 61, 4, 1.0)
    rp, col, val = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=v, vox_end=v + 1)
    _check_rows(oracle, rp, col, val, {v: cols[0]}, {v: flags[0]}, [v])


def test_bench_workload_sampled(torch, oracle):
    """The configuration the benchmark times: full scanner, central 16^3 voxels,
    analytic table, every class (z-runs, square-symmetry images, axial mirrors)
    in one call.  Sampled voxels' matrix rows, their adjoint and sensitivity
    entries, and the forward projection of those voxels alone against the
    oracle; <A x, y> = <x, A^T y> on dense seeded inputs."""
    cfg = dict(CFG3, nx=16, ny=16, nz=16)
    nr, P, step = cfg["n_rows"], cfg["n_sub"], cfg["step_deg"]
    rt, rz = np.meshgrid(np.arange(nr), np.arange(nr), indexing="ij")
    # the oracle's table, rounded to FP32 so that both sides read the same entries
    td = oracle.table3_rows(cfg, rt.ravel(), rz.ravel(), P, step, 16).astype(np.float32).astype(np.float64)
    samp = [(7, 8, 5), (8, 7, 10), (1, 4, 2), (13, 6, 9), (10, 2, 14), (5, 11, 1)]
    vox = [(iz * 16 + iy) * 16 + ix for ix, iy, iz in samp]
    cols, flags = oracle.columns_3d(cfg, oracle.TableRef(td, nr, P, step), vox, cap=1 << 21)
    sc = _scanner(cfg)
    t = sc.table_from(td, nr, P, step)
    rp, col, val = sc.build_psf_sysmat(t, threshold=cfg["threshold"])
    rpc = rp.cpu().numpy()
    exact = []
    for v, (ob, ov), fl in zip(vox, cols, flags):
        g = col[rpc[v]:rpc[v + 1]].cpu().numpy().astype(np.int64)
        gv = val[rpc[v]:rpc[v + 1]].cpu().numpy()
        if fl & oracle.F_TIES == 0:
            assert np.array_equal(g, ob), f"voxel {v}: pattern differs ({len(g)} vs {len(ob)})"
            np.testing.assert_allclose(gv, ov, rtol=RTOL, atol=0, err_msg=f"voxel {v}")
            exact.append((v, ob, ov))
        else:
            m = dict(zip(ob.tolist(), ov.tolist()))
            common = [k for k in range(len(g)) if int(g[k]) in m]
            assert len(common) >= 0.99 * len(ob)
            np.testing.assert_allclose(gv[common], [m[int(g[k])] for k in common], rtol=RTOL)
    assert len(exact) >= 3
    del col, val
    # sensitivity and adjoint entries of the exact voxels: their columns summed, and against y
    s = sc.sensitivity(t).cpu().numpy()
    rng = np.random.default_rng(5)
    yd = rng.random(sc.n_bins, dtype=np.float32)
    xa = sc.project_adj(t, torch.from_numpy(yd[None]).cuda()).cpu().numpy()[0]
    for v, ob, ov in exact:
        np.testing.assert_allclose(s[v], ov.sum(), rtol=RTOL)
        np.testing.assert_allclose(xa[v], ov @ yd[ob].astype(np.float64), rtol=RTOL)
    # the forward projection of the exact voxels alone, bin by bin
    xs = np.zeros(sc.n_voxels, np.float32)
    ye = {}
    for k, (v, ob, ov) in enumerate(exact):
        xs[v] = 1.0 + 0.5 * k
        for b, a in zip(ob.tolist(), ov.tolist()):
            ye[b] = ye.get(b, 0.0) + float(xs[v]) * a
    y = sc.project_fwd(t, torch.from_numpy(xs[None]).cuda())[0]
    bins = np.fromiter(ye.keys(), np.int64)
    ref = np.fromiter(ye.values(), np.float64)
    got = y[torch.from_numpy(bins).cuda()].cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=RTOL, atol=0)
    assert int((y != 0).sum().item()) == int(np.count_nonzero(ref))
    # the adjoint identity at full size, dense seeded images
    xd = torch.from_numpy(rng.random((1, sc.n_voxels), dtype=np.float32)).cuda()
    yt = torch.from_numpy(yd[None]).cuda()
    lhs = torch.dot(sc.project_fwd(t, xd)[0].double(), yt[0].double()).item()
    rhs = torch.dot(xd[0].double(), torch.from_numpy(xa).cuda().double()).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_bench_workload_table_grad_and_listmode(torch):
    """Properties that hold at any size, on the benchmark's configuration:
    f(table) = <y, A(table) x> is homogeneous of degree 2 in the table (each
    tile is linear in U and in V, both linear in the table entries, the
    block-edge remap included), so <grad f, table> = 2 f; list-mode rows
    (per event, either photon order) equal the full forward projection at the
    events' bins, and their back projection equals the adjoint of the events'
    histogram."""
    cfg = dict(CFG3, nx=16, ny=16, nz=16)
    sc = _scanner(cfg)
    t = sc.build_table(cfg["n_rows"], cfg["n_sub"], cfg["step_deg"])
    rng = np.random.default_rng(9)
    xt = torch.from_numpy(rng.random((1, sc.n_voxels), dtype=np.float32)).cuda()
    yd = torch.from_numpy(rng.random((1, sc.n_bins), dtype=np.float32)).cuda()
    yf = sc.project_fwd(t, xt)
    f = torch.dot(yf[0].double(), yd[0].double()).item()
    xb, grad = sc.project_adj(t, yd, xt=xt, want_table_grad=True)
    g = torch.dot(grad.double(), t.data.double()).item()
    assert abs(g - 2.0 * f) <= 1e-5 * abs(2.0 * f)
    # list mode: 1e5 events on bins the phantom reaches
    live = torch.nonzero(yf[0] > 0).reshape(-1).cpu().numpy()
    bins = np.sort(rng.choice(live, 100_000))
    gi, ri, gj, rj = _unbin3(bins, cfg)
    Nc = cfg["n_blocks"] * cfg["n_ct"]
    ci, cj = ri * Nc + gi, rj * Nc + gj
    sw = rng.random(len(bins)) < 0.5
    ev = torch.from_numpy(np.stack([np.where(sw, cj, ci), np.where(sw, ci, cj)], 1).astype(np.int32)).cuda()
    q = sc.project_fwd(t, xt, events=ev)[0]
    bt = torch.from_numpy(bins).cuda()
    np.testing.assert_allclose(q.cpu().numpy(), yf[0][bt].cpu().numpy(), rtol=RTOL)
    w = torch.from_numpy(rng.random(len(bins), dtype=np.float32)).cuda()
    xl = sc.project_adj(t, w[None], events=ev)[0]
    hist = torch.zeros(sc.n_bins, dtype=torch.float64, device="cuda").index_add_(0, bt, w.double())
    xh = sc.project_adj(t, hist.float()[None])[0]
    np.testing.assert_allclose(xl.cpu().numpy(), xh.cpu().numpy(), rtol=RTOL, atol=RTOL * 1e-2 * float(xh.abs().max()))


def test_degenerate_inputs(torch, oracle, small_ref):
    """An empty voxel range, an all-zero image, a batch of 10 images (a chunk of
    8 and one of 2), and an empty event list."""
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    rp, col, val = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=5, vox_end=5)
    assert rp.cpu().tolist() == [0] and col.numel() == 0 and val.numel() == 0
    z = torch.zeros(2, sc.n_voxels, device="cuda")
    assert int((sc.project_fwd(t, z) != 0).sum().item()) == 0
    A_T = _sparse(cols, sc.n_bins)
    x = S.phantom_uniform(SMALL, seed=21, batch=10)
    xf = x.astype(np.float32).astype(np.float64)
    y = sc.project_fwd(t, torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    yo = (A_T.T @ xf.T).T
    np.testing.assert_allclose(y, yo, rtol=RTOL, atol=RTOL * 1e-2 * np.abs(yo).max())
    yc = yo.astype(np.float32)
    xb = sc.project_adj(t, torch.tensor(yc, device="cuda")).cpu().numpy()
    xbo = (A_T @ yc.astype(np.float64).T).T
    np.testing.assert_allclose(xb, xbo, rtol=RTOL, atol=RTOL * 1e-2 * np.abs(xbo).max())
    ev = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    q = sc.project_fwd(t, torch.tensor(x[:2], dtype=torch.float32, device="cuda"), events=ev)
    assert tuple(q.shape) == (2, 0)
    xe = sc.project_adj(t, torch.zeros(2, 0, device="cuda"), events=ev)
    assert tuple(xe.shape) == (2, sc.n_voxels) and int((xe != 0).sum().item()) == 0


def test_capacity_exceeded_is_an_error(torch):
    """A ring of 1280 crystals (80 blocks of 16, nearly no gaps) shows a voxel
    more than 4096 transaxial sub-segment pairs and 1024 crystal pairs, beyond
    the per-class scratch of the 3D kernels.  The kernels drop that class and
    exit normally with the capacity flag set; every 3D entry point must then
    return PSF_ECAPACITY instead of an incomplete result."""
    import math

    from paper_1607_06170_amd import PsfError, _lib
    cfg = dict(CFG3, n_blocks=80, n_ct=16, n_cz=1, n_brings=2, r_face=16.0 / math.tan(math.pi / 80) + 0.5,
               nx=2, ny=2, nz=2, n_rows=61)
    sc = _scanner(cfg)
    t = sc.build_table(61, 4, 1.0)
    x = torch.ones(1, sc.n_voxels, device="cuda")
    for call in (lambda: sc.project_fwd(t, x), lambda: sc.project_adj(t, torch.ones(1, sc.n_bins, device="cuda")),
                 lambda: sc.sensitivity(t), lambda: sc.build_psf_sysmat(t)):
        with pytest.raises(PsfError) as ei:
            call()
        assert ei.value.code == _lib.PSF_ECAPACITY
    # the same scanner with 40 blocks stays within the scratch and runs
    ok = dict(cfg, n_blocks=40, r_face=16.0 / math.tan(math.pi / 40) + 0.5)
    sc2 = _scanner(ok)
    t2 = sc2.build_table(61, 4, 1.0)
    y = sc2.project_fwd(t2, torch.ones(1, sc2.n_voxels, device="cuda"))
    assert float(y.sum()) > 0


def test_osem_subset_update_small_scanner(torch, oracle, small_ref):
    """Histogram OSEM in 3D (subsets by the transaxial pair's sinogram angle):
    subset sensitivity and one update against the oracle on the small scanner."""
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    A_T = _sparse(cols, sc.n_bins)
    Nc = SMALL["n_blocks"] * SMALL["n_ct"]
    NR = SMALL["n_cz"] * SMALL["n_brings"]
    x_true = S.phantom_uniform(SMALL, seed=5)[0]
    y = S.poisson_counts(1e3 * (A_T.T @ x_true), seed=201).astype(np.float32)
    x0 = np.ones(sc.n_voxels, np.float32)
    for k in (0, 2):
        m = oracle.subset_mask(sc.n_bins, Nc, NR, 4, k)
        s_gpu = sc.subset_sensitivity(t, 4, k).cpu().numpy()
        s_ref = A_T @ m
        np.testing.assert_allclose(s_gpu, s_ref, rtol=RTOL, atol=RTOL * 1e-2 * float(s_ref.max()))
        xk = sc.osem_update(t, torch.tensor(y, device="cuda"), torch.tensor(x0, device="cuda"),
                            torch.tensor(s_gpu, device="cuda"), 4, k).cpu().numpy()
        yhat = A_T.T @ x0.astype(np.float64)
        ratio = np.where((m > 0) & (yhat > 0), y / np.where(yhat > 0, yhat, 1.0), 0.0)
        xo = np.where(s_ref > 0, x0 * (A_T @ ratio) / np.where(s_ref > 0, s_ref, 1.0), 0.0)
        np.testing.assert_allclose(xk, xo, rtol=2e-5, atol=2e-5 * float(xo.max()))


@pytest.fixture(scope="module")
def full_cfg(oracle):
    """The benchmark's configuration: the whole 128 x 128 x 96 image, the
    oracle's analytic table rounded to FP32 as the input of both sides."""
    cfg = dict(CFG3)
    nr, P, step = cfg["n_rows"], cfg["n_sub"], cfg["step_deg"]
    rt, rz = np.meshgrid(np.arange(nr), np.arange(nr), indexing="ij")
    td = oracle.table3_rows(cfg, rt.ravel(), rz.ravel(), P, step, 16).astype(np.float32).astype(np.float64)
    return cfg, td


def test_full_volume_sampled(torch, oracle, full_cfg):
    """The whole image as the benchmark builds it: ranges of the voxel order
    (two of them, one cutting groups), sampled rows from several slabs (the
    axial ends, the corners, off-axis) against the oracle; the forward
    projection of a sparse image made of those voxels, bin by bin; their
    adjoint entries; and <A x, y> = <x, A^T y> on dense seeded inputs."""
    cfg, td = full_cfg
    nr, P, step = cfg["n_rows"], cfg["n_sub"], cfg["step_deg"]
    nx, ny = cfg["nx"], cfg["ny"]
    samp = [(3, 60, 0), (124, 8, 95), (64, 64, 47), (100, 30, 20), (10, 117, 70), (70, 5, 2)]
    vox = [(iz * ny + iy) * nx + ix for ix, iy, iz in samp]
    cols, flags = oracle.columns_3d(cfg, oracle.TableRef(td, nr, P, step), vox, cap=1 << 21, nthreads=16)
    sc = _scanner(cfg)
    t = sc.table_from(td, nr, P, step)
    order = sc.voxel_order()
    pos = np.empty_like(order)
    pos[order] = np.arange(len(order))
    exact = []
    for v, (ob, ov), fl in zip(vox, cols, flags):
        p = int(pos[v])
        vb = max(0, p - 700)   # a range holding the voxel, cut at an arbitrary place
        rp, col, val = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=vb, vox_end=min(vb + 2048, sc.n_voxels),
                                           class_order=True)
        r = p - vb
        rpc = rp[r:r + 2].cpu().numpy()
        g = col[rpc[0]:rpc[1]].cpu().numpy().astype(np.int64)
        gv = val[rpc[0]:rpc[1]].cpu().numpy()
        del rp, col, val
        if fl & oracle.F_TIES == 0:
            assert np.array_equal(g, ob), f"voxel {v}: pattern differs ({len(g)} vs {len(ob)})"
            np.testing.assert_allclose(gv, ov, rtol=RTOL, atol=0, err_msg=f"voxel {v}")
            exact.append((v, ob, ov))
        else:
            _, ia, ib = np.intersect1d(g, ob, assume_unique=True, return_indices=True)
            assert len(ia) >= 0.99 * len(np.union1d(g, ob))
            np.testing.assert_allclose(gv[ia], ov[ib], rtol=RTOL)
    assert len(exact) >= 3
    # the sparse image of the sampled voxels: forward bin by bin, adjoint entries
    xs = np.zeros(sc.n_voxels, np.float32)
    ye = {}
    for k, (v, ob, ov) in enumerate(exact):
        xs[v] = 1.0 + 0.5 * k
        for b, a in zip(ob.tolist(), ov.tolist()):
            ye[b] = ye.get(b, 0.0) + float(xs[v]) * a
    y = sc.project_fwd(t, torch.from_numpy(xs[None]).cuda())[0]
    bins = np.fromiter(ye.keys(), np.int64)
    ref = np.fromiter(ye.values(), np.float64)
    got = y[torch.from_numpy(bins).cuda()].cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=RTOL, atol=0)
    assert int((y != 0).sum().item()) == int(np.count_nonzero(ref))
    del y
    rng = np.random.default_rng(15)
    yd = torch.rand(1, sc.n_bins, device="cuda", generator=torch.Generator(device="cuda").manual_seed(15))
    xa = sc.project_adj(t, yd)[0]
    for v, ob, ov in exact:
        np.testing.assert_allclose(float(xa[v]), ov @ yd[0][torch.from_numpy(ob).cuda()].double().cpu().numpy(),
                                   rtol=RTOL)
    xd = torch.from_numpy(rng.random((1, sc.n_voxels), dtype=np.float32)).cuda()
    lhs = torch.dot(sc.project_fwd(t, xd)[0].double(), yd[0].double()).item()
    rhs = torch.dot(xd[0].double(), xa.double()).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_config4_batch8_autograd_full_volume(torch, oracle, full_cfg):
    """Differentiation at its stated size, 128 x 128 x 96.  A batch of 8
    seeded phantoms through PsfProject: backward gives A^T g, with
    <A x_b, g_b> = <x_b, A^T g_b> per image on seeded Poisson counts g and
    A^T g against the oracle's columns at sampled voxels.  The table
    gradient through PsfProject for a sparse image of those voxels: every
    entry against the oracle's, the degree-2 identity <grad, table> = 2 f,
    and central differences (h = 1e-3; f is exactly quadratic in the
    table).  The table gradient of the dense batch is left out: with the
    analytic table (two thirds of its entries zero) it reads about nine
    times the adjoint's sinogram entries (see the adjoint's gradient form)."""
    from paper_1607_06170_amd import PsfProject
    cfg, td = full_cfg
    nr, P, step = cfg["n_rows"], cfg["n_sub"], cfg["step_deg"]
    sc = _scanner(cfg)
    xs = np.stack([S.phantom_blobs(cfg, seed=100 + b) for b in range(8)]).astype(np.float32)
    x = torch.from_numpy(xs).cuda().requires_grad_(True)
    tab = torch.from_numpy(td.astype(np.float32)).cuda()
    _progress("config 4: forward of 8 images")
    y = PsfProject.apply(x, tab, sc, (nr, P, step))
    # seeded Poisson counts (mean uniform in [0, 10) per bin)
    gen = torch.Generator(device="cuda").manual_seed(200)
    g = torch.poisson(10.0 * torch.rand(y.shape, generator=gen, device="cuda"), generator=gen)
    _progress("config 4: backward of 8 images")
    (y * g).sum().backward()
    torch.cuda.synchronize()
    gx = x.grad
    for b in range(8):
        lhs = torch.dot(y.detach()[b].double(), g[b].double()).item()
        rhs = torch.dot(x.detach()[b].double(), gx[b].double()).item()
        assert abs(lhs - rhs) <= 1e-5 * abs(rhs), b
    # A^T g at sampled voxels of image 0 against the oracle's columns
    rng = np.random.default_rng(201)
    vox = [int(v) for v in rng.choice(sc.n_voxels, 4, replace=False)]
    _progress("config 4: oracle columns")
    cols, flags = oracle.columns_3d(cfg, oracle.TableRef(td, nr, P, step), vox, cap=1 << 21, nthreads=16)
    g0 = g[0]
    for v, (ob, ov), fl in zip(vox, cols, flags):
        if fl & oracle.F_TIES:
            continue
        ref = ov @ g0[torch.from_numpy(ob).cuda()].double().cpu().numpy()
        np.testing.assert_allclose(float(gx[0, v]), ref, rtol=RTOL)
    del y, g, x, gx
    # the table gradient of a sparse image through autograd
    xsp = np.zeros(sc.n_voxels, np.float32)
    xsp[vox] = xs[0][vox]
    bins = np.unique(np.concatenate([b for b, _ in cols]))
    gv = rng.random(len(bins))
    gsp = torch.zeros(1, sc.n_bins, device="cuda")
    gsp[0, torch.from_numpy(bins).cuda()] = torch.from_numpy(gv.astype(np.float32)).cuda()
    xt = torch.from_numpy(xsp[None]).cuda()
    tab_g = tab.clone().requires_grad_(True)
    _progress("config 4: table gradient of a sparse image")
    ysp = PsfProject.apply(xt, tab_g, sc, (nr, P, step))
    fsp = (ysp * gsp).sum()
    fsp.backward()
    torch.cuda.synchronize()
    f = torch.dot(ysp.detach()[0].double(), gsp[0].double()).item()
    grad = tab_g.grad.double().reshape(-1)
    g2 = torch.dot(grad, tab.double().reshape(-1)).item()
    assert abs(g2 - 2.0 * f) <= 1e-4 * abs(2.0 * f)
    _progress("config 4: oracle table gradient")
    ref = oracle.table_grad_3d(cfg, oracle.TableRef(td, nr, P, step), vox, xsp[vox].astype(np.float64), bins,
                               gv.astype(np.float32).astype(np.float64), nthreads=16).reshape(-1)
    grad = grad.cpu().numpy()
    np.testing.assert_allclose(grad, ref, rtol=1e-4, atol=1e-6 * np.abs(ref).max())
    assert np.count_nonzero(ref[td.reshape(-1) == 0]) > 1000   # zero table entries carry gradient
    # central differences of f through the FP32 forward projection: entries
    # among the largest gradients, so that the forward's rounding (about 1e-11
    # of f) stays far below the tolerance
    h = 1e-3
    _progress("config 4: central differences")
    for e in rng.choice(np.argsort(-np.abs(ref))[:100], 3, replace=False):
        fs = []
        for sgn in (1.0, -1.0):
            tp = td.astype(np.float32).copy().reshape(-1)
            tp[e] += sgn * h
            yp = sc.project_fwd(sc.table_from(tp, nr, P, step), xt)[0]
            fs.append(torch.dot(yp.double(), gsp[0].double()).item())
        fd = (fs[0] - fs[1]) / (2 * h)
        assert abs(fd - ref[e]) <= 1e-3 * abs(ref[e]) + 1e-6 * np.abs(ref).max(), (e, fd, ref[e])


def test_config5_listmode_1e7_events(torch, full_cfg):
    """List mode at its stated size: 1e7 seeded events (9e6 drawn from the
    forward projection of the phantom, 1e6 uniform randoms over the LORs,
    shuffled); one LM-OSEM subset update of the first 1e6 (M = 10) at
    128 x 128 x 96 in the FP32 and BF16 forms.  Each update keeps
    sum_j (s_j / M) x_new_j = sum_e q_e / (q_e + r) (q_e the events' forward
    rows, FP64 sums), and the BF16 form stays within its bounds of the FP32 one."""
    cfg, td = full_cfg
    nr, P, step = cfg["n_rows"], cfg["n_sub"], cfg["step_deg"]
    sc = _scanner(cfg)
    t = sc.table_from(td, nr, P, step)
    x = torch.from_numpy(S.phantom_blobs(cfg, seed=2).astype(np.float32)[None]).cuda()
    w = sc.project_fwd(t, x)[0].double()
    gen = torch.Generator(device="cuda").manual_seed(300)
    cdf = torch.cumsum(w, 0)
    trues = torch.searchsorted(cdf, torch.rand(9_000_000, generator=gen, device="cuda", dtype=torch.float64) * cdf[-1])
    lors = torch.nonzero(w > 0).reshape(-1)
    rnd = lors[torch.randint(0, lors.numel(), (1_000_000,), generator=gen, device="cuda")]
    bins = torch.cat([trues.clamp_max(w.numel() - 1), rnd])
    bins = bins[torch.randperm(bins.numel(), generator=gen, device="cuda")]
    n_lor = int(lors.numel())
    del cdf, trues, rnd, lors
    Nc = cfg["n_blocks"] * cfg["n_ct"]
    NR = cfg["n_cz"] * cfg["n_brings"]
    tb, rr = bins // (NR * NR), bins % (NR * NR)
    starts = torch.tensor([i * Nc - i * (i + 1) // 2 for i in range(Nc)], device="cuda", dtype=torch.int64)
    gi = torch.searchsorted(starts, tb, right=True) - 1
    gj = tb - starts[gi] + gi + 1
    events = torch.stack([(rr // NR) * Nc + gi, (rr % NR) * Nc + gj], 1).to(torch.int32).contiguous()
    assert events.shape[0] == 10_000_000
    sub = events[:1_000_000].contiguous()
    s = sc.sensitivity(t)
    x0 = torch.full_like(x[0], 9e6 / float(s.double().sum()))
    r = 1e6 / n_lor
    q = sc.project_fwd(t, x0[None].contiguous(), events=sub)[0].double()
    expect = float((q / (q + r)).sum())
    outs = {}
    for prec in (0, 1):
        xn = sc.lm_osem_update(t, sub, x0, s, 10, r, precision=prec)
        lhs = float((s.double() / 10 * xn.double()).sum())
        assert abs(lhs - expect) <= (1e-4 if prec == 0 else 1e-2) * expect, (prec, lhs, expect)
        outs[prec] = xn.double()
    d = outs[1] - outs[0]
    assert float(d.norm() / outs[0].norm()) <= 1e-2
