"""FP64 CPU oracle for the P-SPIR PSF system matrix -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The library never does: it shares no
code with the oracle, and the oracle shares none with it.

The heavy lifting is plain C in ``psf_oracle.c`` / ``psf_oracle3d.c`` (FP64,
no FMA contraction), loaded through ctypes.  What is done here in numpy is the
plain linear algebra on top of the dense matrix columns the C code returns:
projections ``y = A x`` and ``x = A^T y``, the sensitivity ``A^T 1``, the
thresholded CSR, and the list-mode OSEM update.

Paper: Sun et al., Chinese Physics C (2016), arXiv 1607.06170.  Sections,
equations and tables are cited next to each function.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "_psf_oracle.so")
SOURCES = [os.path.join(HERE, "psf_oracle.c"), os.path.join(HERE, "psf_oracle3d.c"),
           os.path.join(HERE, "psf_oracle_mc.c")]

# flag bits (see psf_oracle.c)
F_MIRROR_TIE = 1
F_ROW_TIE = 2
F_OVERLAP_TIE = 4
F_REMAP_TIE = 8
F_RANGE = 16
F_GEOM = 32
F_TIES = F_MIRROR_TIE | F_ROW_TIE | F_OVERLAP_TIE | F_REMAP_TIE


def build(force: bool = False) -> str:
    """Compile the oracle's C sources into a shared object next to them."""
    srcs = [s for s in SOURCES if os.path.exists(s)]
    if not force and os.path.exists(SO_PATH):
        so_m = os.path.getmtime(SO_PATH)
        if all(os.path.getmtime(s) <= so_m for s in srcs):
            return SO_PATH
    tmp = SO_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO_PATH)
    return SO_PATH


class Geom(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("n_ct", C.c_int32), ("n_cz", C.c_int32), ("n_brings", C.c_int32),
                ("pitch_t", C.c_double), ("pitch_z", C.c_double), ("depth", C.c_double),
                ("r_face", C.c_double), ("gap_z", C.c_double), ("mu", C.c_double), ("phi0", C.c_double)]


class Image(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double)]


class Table(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_sub", C.c_int32), ("step_deg", C.c_double),
                ("data", C.POINTER(C.c_double))]


_lib = None
_lock = threading.Lock()

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(SO_PATH)
            G, I, T = C.POINTER(Geom), C.POINTER(Image), C.POINTER(Table)
            L.og_rho_point.restype = C.c_double
            L.og_rho_point.argtypes = [C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, C.c_double]
            L.og_rho_sub.restype = C.c_double
            L.og_rho_sub.argtypes = [C.c_double, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double]
            L.og_table_2d.restype = None
            L.og_table_2d.argtypes = [G, C.c_int, C.c_int, C.c_double, _dp]
            L.og_sigma.restype = C.c_double
            L.og_sigma.argtypes = [G]
            L.og_ap1.restype = C.c_double
            L.og_ap1.argtypes = [G, C.c_double, C.c_double]
            L.og_uv_row_2d.restype = C.c_int
            L.og_uv_row_2d.argtypes = [G, T, C.c_double, C.c_double, C.c_int, C.c_int, _dp, _i32p]
            L.og_samples_2d.restype = C.c_int
            L.og_samples_2d.argtypes = [G, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int64, _i32p, _i32p, _dp,
                                        C.POINTER(C.c_int64)]
            L.og_column_2d.restype = C.c_int
            L.og_column_2d.argtypes = [G, T, C.c_double, C.c_double, C.c_int, _dp]
            L.og_columns_2d.restype = None
            L.og_columns_2d.argtypes = [G, T, I, _i64p, C.c_int64, C.c_int, _dp, _i32p, C.c_int]
            L.og_table_grad_2d.restype = None
            L.og_table_grad_2d.argtypes = [G, T, I, _dp, _dp, C.c_int, _dp, C.c_int]
            L.og_gauss_legendre.restype = None
            L.og_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
            if hasattr(L, "og_table3_rows"):
                _bind3d(L, G, I, T)
            _u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
            L.og_philox4x32_10.restype = None
            L.og_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
            L.og_kn_sigma.restype = C.c_double
            L.og_kn_sigma.argtypes = [C.c_double]
            L.og_kn_cos_samples.restype = None
            L.og_kn_cos_samples.argtypes = [C.c_double, C.c_int64, C.c_uint64, _dp]
            L.og_table_mc.restype = None
            L.og_table_mc.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_int64, C.c_uint64, C.c_int, C.c_int64, C.c_int64, _i64p,
                                      C.c_int]
            _lib = L
    return _lib


def _bind3d(L, G, I, T):
    L.og_rho_point3.restype = C.c_double
    L.og_rho_point3.argtypes = [C.c_double] * 4 + [C.c_int, C.c_int] + [C.c_double] * 4
    L.og_rho_sub3.restype = C.c_double
    L.og_rho_sub3.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int] + [C.c_double] * 4
    L.og_table3_rows.restype = None
    L.og_table3_rows.argtypes = [G, C.c_int, C.c_double, _i32p, _i32p, C.c_int, _dp, C.c_int]
    L.og_uv_row_3d.restype = C.c_int
    L.og_uv_row_3d.argtypes = [G, T, _dp, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _i32p]
    L.og_columns_3d.restype = None
    L.og_columns_3d.argtypes = [G, T, I, _i64p, C.c_int64, C.c_int64, _i64p, _dp, _i64p, _i32p, C.c_int]
    L.og_table_grad_3d.restype = None
    L.og_table_grad_3d.argtypes = [G, T, I, _i64p, _dp, C.c_int64, _i64p, _dp, C.c_int64, _dp, C.c_int]
    L.og3_set_full_ring_scan.restype = None
    L.og3_set_full_ring_scan.argtypes = [C.c_int]
    L.og_w3_pair.restype = C.c_double
    L.og_w3_pair.argtypes = [G, C.c_int, _dp, C.c_int, C.c_int, C.c_int, C.c_int]


# ---------------------------------------------------------------------------
# Python-side views of the C structures
# ---------------------------------------------------------------------------

def geom(cfg: dict) -> Geom:
    return Geom(int(cfg["n_blocks"]), int(cfg["n_ct"]), int(cfg.get("n_cz", 1)), int(cfg.get("n_brings", 1)),
                float(cfg["pitch_t"]), float(cfg.get("pitch_z", cfg["pitch_t"])), float(cfg["depth"]),
                float(cfg["r_face"]), float(cfg.get("gap_z", 0.0)), float(cfg["mu"]), float(cfg.get("phi0", 0.0)))


def image(cfg: dict) -> Image:
    return Image(int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1)), 0, float(cfg["dx"]), float(cfg["dy"]),
                 float(cfg.get("dz", 1.0)), float(cfg.get("cx", 0.0)), float(cfg.get("cy", 0.0)),
                 float(cfg.get("cz", 0.0)))


class TableRef:
    """Keeps the numpy array alive next to the C view of it."""

    def __init__(self, data: np.ndarray, n_rows: int, n_sub: int, step_deg: float):
        self.data = np.ascontiguousarray(data, dtype=np.float64)
        self.n_rows, self.n_sub, self.step_deg = n_rows, n_sub, step_deg
        self.c = Table(n_rows, n_sub, step_deg, self.data.ctypes.data_as(C.POINTER(C.c_double)))


def n_crystals_ring(cfg: dict) -> int:
    return int(cfg["n_blocks"]) * int(cfg["n_ct"])


def n_bins_2d(cfg: dict) -> int:
    n = n_crystals_ring(cfg)
    return n * (n - 1) // 2


def voxel_centre(cfg: dict, j: int) -> np.ndarray:
    nx, ny = int(cfg["nx"]), int(cfg["ny"])
    ix, iy, iz = j % nx, (j // nx) % ny, j // (nx * ny)
    nz = int(cfg.get("nz", 1))
    return np.array([(ix - 0.5 * (nx - 1)) * cfg["dx"] + cfg.get("cx", 0.0),
                     (iy - 0.5 * (ny - 1)) * cfg["dy"] + cfg.get("cy", 0.0),
                     (iz - 0.5 * (nz - 1)) * cfg.get("dz", 1.0) + cfg.get("cz", 0.0)])


# ---------------------------------------------------------------------------
# Response table (Sec 2.1.1, Eq.1, 6, 7)
# ---------------------------------------------------------------------------

def table_2d(cfg: dict, n_rows: int = 61, n_sub: int = 4, step_deg: float = 1.0) -> TableRef:
    """Analytic absolute response table rho[row][p][a+2] (FP64)."""
    out = np.zeros(n_rows * n_sub * 5)
    lib().og_table_2d(C.byref(geom(cfg)), n_rows, n_sub, step_deg, out)
    return TableRef(out.reshape(n_rows, n_sub, 5), n_rows, n_sub, step_deg)


def rho_point(alpha: float, u: float, a: int, lam: float, depth: float, mu: float) -> float:
    return lib().og_rho_point(alpha, u, a, lam, depth, mu)


def rho_sub(alpha: float, p: int, n_sub: int, a: int, lam: float, depth: float, mu: float) -> float:
    return lib().og_rho_sub(alpha, p, n_sub, a, lam, depth, mu)


def sigma(cfg: dict) -> float:
    return lib().og_sigma(C.byref(geom(cfg)))


def ap1(cfg: dict, alpha: float, nu: float) -> float:
    """Eq.4, the equivalent incidence position in the next block."""
    return lib().og_ap1(C.byref(geom(cfg)), alpha, nu)


def uv_row_2d(cfg: dict, tab: TableRef, v: np.ndarray, g: int, p: int):
    val = np.zeros(5)
    src = np.zeros(5, dtype=np.int32)
    fl = lib().og_uv_row_2d(C.byref(geom(cfg)), C.byref(tab.c), float(v[0]), float(v[1]), int(g), int(p), val, src)
    return val, src, fl


# ---------------------------------------------------------------------------
# Homogenization samples and matrix columns (Sec 2.3, Eq.10-12)
# ---------------------------------------------------------------------------

def samples_2d(cfg: dict, n_sub: int, v: np.ndarray, homog_k: int = 0):
    """(s1, s2, w) for every homogenized line through v, s1 < s2; plus flags."""
    maxs = 1 << 16 if homog_k == 0 else homog_k + 16
    s1 = np.zeros(maxs, np.int32)
    s2 = np.zeros(maxs, np.int32)
    w = np.zeros(maxs)
    n = C.c_int64(0)
    fl = lib().og_samples_2d(C.byref(geom(cfg)), n_sub, float(v[0]), float(v[1]), homog_k, maxs, s1, s2, w,
                             C.byref(n))
    n = n.value
    assert n <= maxs
    return s1[:n].copy(), s2[:n].copy(), w[:n].copy(), fl


def columns_2d(cfg: dict, tab: TableRef, vox, homog_k: int = 0, nthreads: int = 0):
    """Dense FP64 columns A[:, v] for the voxels in ``vox``: array [len(vox), n_bins], flags."""
    vox = np.ascontiguousarray(np.asarray(vox, dtype=np.int64))
    nb = n_bins_2d(cfg)
    out = np.zeros((len(vox), nb))
    flags = np.zeros(len(vox), np.int32)
    lib().og_columns_2d(C.byref(geom(cfg)), C.byref(tab.c), C.byref(image(cfg)), vox, len(vox), homog_k,
                        out.reshape(-1), flags, nthreads)
    return out, flags


def table_grad_2d(cfg: dict, tab: TableRef, x: np.ndarray, gy: np.ndarray, homog_k: int = 0, nthreads: int = 0):
    """d <gy, A x> / d table, for one image x (all voxels) and bin weights gy."""
    grad = np.zeros(tab.data.size)
    lib().og_table_grad_2d(C.byref(geom(cfg)), C.byref(tab.c), C.byref(image(cfg)),
                           np.ascontiguousarray(x, dtype=np.float64).reshape(-1),
                           np.ascontiguousarray(gy, dtype=np.float64).reshape(-1), homog_k, grad, nthreads)
    return grad.reshape(tab.data.shape)


# ---------------------------------------------------------------------------
# Plain linear algebra on the dense matrix (rows = bins, columns = voxels)
# ---------------------------------------------------------------------------

def csr_from_columns(cols: np.ndarray, threshold: float):
    """CSR of A^T (rows = voxels, columns = bins ascending) keeping A >= threshold
    (and A > 0).  Returns row_ptr (int64), col (int32), val (float64)."""
    keep = (cols > 0) & (cols >= threshold)
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(cols.shape[0] + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    r, c = np.nonzero(keep)
    return row_ptr, c.astype(np.int32), cols[r, c]


def sinogram_view(i, j, n: int):
    """Sinogram angle of the crystal pair (i, j) of a ring of n crystals (Table 1:
    a histogram of n/2 angles for n crystals per ring).  Chords with the same
    i + j (mod n) are parallel on a circular ring; the two parities of i + j
    interleave in one view: view ((i + j) mod n) // 2."""
    return ((np.asarray(i) + np.asarray(j)) % n) // 2


def truncate_top_n(cols: np.ndarray, n_crystals: int, top_n: int) -> np.ndarray:
    """Sec 3.3: for every voxel (row of cols, columns = 2D bins) and every
    sinogram angle, keep the top_n largest bins and drop the others (ties keep
    the lower bin).  Returns a new dense array."""
    nb = cols.shape[1]
    i = np.zeros(nb, np.int64)
    j = np.zeros(nb, np.int64)
    for a in range(n_crystals):          # the unordered pairs in bin order
        lo = a * n_crystals - a * (a + 1) // 2
        i[lo:lo + n_crystals - a - 1] = a
        j[lo:lo + n_crystals - a - 1] = np.arange(a + 1, n_crystals)
    view = sinogram_view(i, j, n_crystals)
    out = np.zeros_like(cols)
    for v in range(n_crystals // 2):
        idx = np.nonzero(view == v)[0]   # ascending bins
        sub = cols[:, idx]
        order = np.argsort(-sub, axis=1, kind="stable")[:, :top_n]   # largest first, lower bin first on ties
        rows = np.arange(cols.shape[0])[:, None]
        keep = idx[order]
        out[rows, keep] = cols[rows, keep]
    return out


def subset_mask(n_bins: int, n_crystals: int, n_rings: int, n_subsets: int, subset: int) -> np.ndarray:
    """Bins of OSEM subset k (Sec 3: OSEM over the sinogram of Table 1): the
    bins whose sinogram angle v (of their transaxial crystal pair) has
    v mod n_subsets = k.  Bins: transaxial pair major, then the ring pair."""
    tb = np.arange(n_bins, dtype=np.int64) // (n_rings * n_rings)
    starts = np.array([a * n_crystals - a * (a + 1) // 2 for a in range(n_crystals)], dtype=np.int64)
    gi = np.searchsorted(starts, tb, side="right") - 1
    gj = tb - starts[gi] + gi + 1
    return (sinogram_view(gi, gj, n_crystals) % n_subsets == subset).astype(np.float64)


def osem_update(cols: np.ndarray, y: np.ndarray, x: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """One OSEM subset update (Sec 3): x <- x / s_k * A^T (m_k y / A x),
    s_k = A^T m_k; bins with A x = 0 add nothing, voxels with s_k = 0 get 0.
    cols[voxels, bins] holds A^T."""
    yhat = cols.T @ x
    ratio = np.zeros_like(yhat)
    ok = (mask > 0) & (yhat > 0)
    ratio[ok] = y[ok] / yhat[ok]
    back = cols.dot(ratio)
    sens = cols.dot(mask)
    out = np.zeros_like(x)
    nz = sens > 0
    out[nz] = x[nz] * back[nz] / sens[nz]
    return out


def project_fwd(cols: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y[B, bins] = A x for x[B, voxels]; cols[voxels, bins] holds A^T."""
    return np.atleast_2d(x) @ cols


def project_adj(cols: np.ndarray, y: np.ndarray) -> np.ndarray:
    """x[B, voxels] = A^T y for y[B, bins]."""
    return np.atleast_2d(y) @ cols.T


def sensitivity(cols: np.ndarray) -> np.ndarray:
    """s = A^T 1."""
    return cols.sum(axis=1)


def listmode_fwd(cols: np.ndarray, ev_bins: np.ndarray, x: np.ndarray) -> np.ndarray:
    """q_e = a_e^T x for every event, a_e the matrix row of the event's bin."""
    return cols[:, ev_bins].T @ x


def listmode_adj(cols: np.ndarray, ev_bins: np.ndarray, h: np.ndarray) -> np.ndarray:
    """sum_e h_e a_e."""
    return cols[:, ev_bins] @ h


def lm_osem_update(cols: np.ndarray, ev_bins: np.ndarray, x: np.ndarray, sens: np.ndarray, n_subsets: int,
                   randoms: float) -> np.ndarray:
    """One list-mode OSEM subset update: x <- x / (s/M) * sum_e a_e / (a_e^T x + r)."""
    q = listmode_fwd(cols, ev_bins, x) + randoms
    back = listmode_adj(cols, ev_bins, 1.0 / q)
    out = np.zeros_like(x)
    nz = sens > 0
    out[nz] = x[nz] / (sens[nz] / n_subsets) * back[nz]
    return out


# ---------------------------------------------------------------------------
# 3D scanner (extension of Sec 2 to block rings; see psf_oracle3d.c)
# ---------------------------------------------------------------------------

def n_rings(cfg: dict) -> int:
    return int(cfg.get("n_cz", 1)) * int(cfg.get("n_brings", 1))


def n_crystals_3d(cfg: dict) -> int:
    return n_crystals_ring(cfg) * n_rings(cfg)


def rho_point3(tt, tz, ut, uz, at, az, lt, lz, depth, mu):
    return lib().og_rho_point3(tt, tz, ut, uz, at, az, lt, lz, depth, mu)


def rho_sub3(alpha_t, alpha_z, pt, pz, P, at, az, lt, lz, depth, mu):
    return lib().og_rho_sub3(alpha_t, alpha_z, pt, pz, P, at, az, lt, lz, depth, mu)


def table3_rows(cfg: dict, rows_t, rows_z, n_sub: int = 4, step_deg: float = 1.0, nthreads: int = 0):
    """Analytic 3D table entries for the listed (row_t, row_z) pairs:
    array [n][n_sub][n_sub][5][5]."""
    rt = np.ascontiguousarray(rows_t, dtype=np.int32)
    rz = np.ascontiguousarray(rows_z, dtype=np.int32)
    out = np.zeros(len(rt) * n_sub * n_sub * 25)
    lib().og_table3_rows(C.byref(geom(cfg)), n_sub, step_deg, rt, rz, len(rt), out, nthreads)
    return out.reshape(len(rt), n_sub, n_sub, 5, 5)


def uv_row_3d(cfg: dict, tab: TableRef, c, g: int, pt: int, r: int, pz: int):
    val = np.zeros(25)
    src = np.zeros(25, dtype=np.int32)
    fl = lib().og_uv_row_3d(C.byref(geom(cfg)), C.byref(tab.c), np.ascontiguousarray(c, dtype=np.float64), g, pt, r,
                            pz, val, src)
    return val.reshape(5, 5), src.reshape(5, 5), fl


def w3_pair(cfg: dict, n_sub: int, c, s1: int, q1: int, s2: int, q2: int) -> float:
    return lib().og_w3_pair(C.byref(geom(cfg)), n_sub, np.ascontiguousarray(c, dtype=np.float64), s1, q1, s2, q2)


def columns_3d(cfg: dict, tab: TableRef, vox, cap: int = 1 << 20, nthreads: int = 0):
    """Sparse FP64 columns for the voxels in vox: list of (bins int64, vals), flags."""
    vox = np.ascontiguousarray(np.asarray(vox, dtype=np.int64))
    nv = len(vox)
    bins = np.zeros(nv * cap, np.int64)
    vals = np.zeros(nv * cap)
    cnt = np.zeros(nv, np.int64)
    flags = np.zeros(nv, np.int32)
    lib().og_columns_3d(C.byref(geom(cfg)), C.byref(tab.c), C.byref(image(cfg)), vox, nv, cap, bins, vals, cnt,
                        flags, nthreads)
    out = []
    for k in range(nv):
        n = int(cnt[k])
        assert n <= cap, "column capacity exceeded"
        out.append((bins[k * cap:k * cap + n].copy(), vals[k * cap:k * cap + n].copy()))
    return out, flags


def set_full_ring_scan(on: bool) -> None:
    """Test switch: the 3D columns pair every ring with every ring instead of
    the rings their lines can reach (the window's pin)."""
    lib().og3_set_full_ring_scan(int(bool(on)))


def table_grad_3d(cfg: dict, tab: TableRef, vox, xv, gy_bins, gy_vals, nthreads: int = 0):
    """d <gy, A x> / d table for x supported on vox (values xv), gy sparse (sorted bins)."""
    vox = np.ascontiguousarray(np.asarray(vox, dtype=np.int64))
    order = np.argsort(gy_bins)
    gb = np.ascontiguousarray(np.asarray(gy_bins, dtype=np.int64)[order])
    gv = np.ascontiguousarray(np.asarray(gy_vals, dtype=np.float64)[order])
    grad = np.zeros(tab.data.size)
    lib().og_table_grad_3d(C.byref(geom(cfg)), C.byref(tab.c), C.byref(image(cfg)), vox,
                           np.ascontiguousarray(xv, dtype=np.float64), len(vox), gb, gv, len(gb), grad, nthreads)
    return grad.reshape(tab.data.shape)


def bin3(g1, r1, g2, r2, cfg: dict):
    """3D bin numbering: transaxial pair (g_i < g_j) major, then (r_i, r_j)."""
    Nc, NR = n_crystals_ring(cfg), n_rings(cfg)
    g1, r1, g2, r2 = (np.asarray(a, dtype=np.int64) for a in (g1, r1, g2, r2))
    sw = g1 > g2
    gi, gj = np.where(sw, g2, g1), np.where(sw, g1, g2)
    ri, rj = np.where(sw, r2, r1), np.where(sw, r1, r2)
    tb = gi * Nc - gi * (gi + 1) // 2 + (gj - gi - 1)
    return np.where(g1 == g2, -1, (tb * NR + ri) * NR + rj)


def n_bins_3d(cfg: dict) -> int:
    return n_bins_2d(cfg) * n_rings(cfg) ** 2


def pair_bin(i, j, n):
    i, j = np.minimum(i, j), np.maximum(i, j)
    return i * n - i * (i + 1) // 2 + (j - i - 1)


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 (Salmon et al., SC 2011) of a 4-word counter and 2-word key."""
    out = np.zeros(4, np.uint32)
    lib().og_philox4x32_10(np.ascontiguousarray(ctr, np.uint32), np.ascontiguousarray(key, np.uint32), out)
    return out


def table_mc_counts(cfg: dict, mode3d: bool, photons: int, seed: int, scatter: bool, cells,
                    n_rows: int = 61, n_sub: int = 4, step_deg: float = 1.0, nthreads: int = 8) -> np.ndarray:
    """Photon-transport Monte Carlo of the response table (Sec 2.1.1, Eq.1): for
    table cells [cells[0], cells[1]) the counts of detected photons, shape
    [cells, 5 (a_t + 2), 5 (a_z + 2)] (2D: a_z = 0).  See psf_oracle_mc.c."""
    c0, c1 = int(cells[0]), int(cells[1])
    out = np.zeros((c1 - c0) * 25, np.int64)
    lib().og_table_mc(int(mode3d), int(n_rows), int(n_sub), float(step_deg), float(cfg["pitch_t"]),
                      float(cfg["pitch_z"]), float(cfg["depth"]), float(cfg["mu"]), int(photons), int(seed),
                      int(scatter), c0, c1, out, int(nthreads))
    return out.reshape(c1 - c0, 5, 5)


def kn_cos_samples(k: float, n: int, seed: int) -> np.ndarray:
    """n Compton scattering cosines at k = E / 511 keV from the MC's sampler."""
    out = np.zeros(int(n))
    lib().og_kn_cos_samples(float(k), int(n), int(seed), out)
    return out


def kn_sigma(k: float) -> float:
    """The MC's Klein-Nishina total cross section (units of 2 pi r_e^2) at k = E / 511 keV."""
    return float(lib().og_kn_sigma(float(k)))
