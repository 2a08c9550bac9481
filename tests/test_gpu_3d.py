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
    rng = np.random.default_rng(3)
    rt = np.concatenate([[0, 0, 60, 60, 45, 1], rng.integers(0, 61, 40)])
    rz = np.concatenate([[0, 60, 0, 60, 45, 0], rng.integers(0, 61, 40)])
    ref = oracle.table3_rows(CFG3, rt, rz)
    np.testing.assert_allclose(got[rt, rz], ref, rtol=1e-6, atol=1e-9)


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
    hi/lo split: error against FP64, per element and per projection."""
    td, cols, flags = small_ref
    sc = _scanner(SMALL)
    t = sc.table_from(td, SMALL["n_rows"], 4, 1.0)
    A_T = _sparse(cols, sc.n_bins)
    x = S.phantom_uniform(SMALL, seed=7)
    yo = (A_T.T @ x[0])
    big = yo > 1e-3 * yo.max()
    for prec, e_tol, p_tol in [(1, 1e-2, 1e-2), (2, 1e-4, 1e-4)]:
        rp, col, val = sc.build_psf_sysmat(t, threshold=0.0, vox_begin=100, vox_end=140, precision=prec)
        rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
        for r in range(40):
            b, v = cols[100 + r]
            g = col[rp[r]:rp[r + 1]]
            assert np.array_equal(g, b)
            assert (np.abs(val[rp[r]:rp[r + 1]] - v) / v).max() <= e_tol
        y = sc.project_fwd(t, torch.tensor(x, dtype=torch.float32, device="cuda"), precision=prec).cpu().numpy()[0]
        assert (np.abs(y - yo)[big] / yo[big]).max() <= p_tol
        # each projection as a whole (relative 2-norm): 1e-3 for BF16, 1e-5 for hi/lo
        n_tol = 1e-3 if prec == 1 else 1e-5
        assert np.linalg.norm(y - yo) / np.linalg.norm(yo) <= n_tol
        ya = yo.astype(np.float32)
        xo = A_T @ ya.astype(np.float64)
        xa = sc.project_adj(t, torch.tensor(ya[None], device="cuda"), precision=prec).cpu().numpy()[0]
        assert np.linalg.norm(xa - xo) / np.linalg.norm(xo) <= n_tol


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
