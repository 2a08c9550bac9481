"""P-SPIR PSF-contained PET system matrix on AMD MI355X (gfx950).

Thin Python binding over the C ABI of ``libpsf.so`` (include/psf.h).  PyTorch
provides device memory and the current HIP stream; every step of the method
runs in the library's HIP kernels.  There is no CPU fallback: without the
built library or a GPU every call raises.

Method: Sun et al., "Fast and accurate generation method of PSF-based system
matrix for PET reconstruction", Chinese Physics C (2016), arXiv 1607.06170.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import _lib
from ._lib import PSF_BF16, PSF_BF16X2, PSF_FP32, PsfError, check

__all__ = ["Scanner", "Table", "PsfProject", "PSF_FP32", "PSF_BF16", "PSF_BF16X2", "PsfError"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1607_06170_amd needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _events_ptr(events):
    """The event list's address: NULL means "every bin" to the library, so an
    empty list (whose tensor has no storage) is passed as a non-NULL address
    that is never read."""
    if events is None:
        return C.c_void_p(0)
    if events.numel() == 0:
        return C.c_void_p(C.addressof(_EMPTY_EVENTS))
    return C.c_void_p(events.data_ptr())


_EMPTY_EVENTS = C.c_int64(0)  # host storage whose address stands for an empty list


def _dev_f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return t.contiguous()


@dataclass
class Table:
    """Response table on the device (layout of psf_table in include/psf.h)."""
    data: "object"  # torch.Tensor float32 on the GPU
    n_rows: int
    n_sub: int
    step_deg: float

    def c(self) -> _lib.psf_table:
        return _lib.psf_table(self.n_rows, self.n_sub, self.step_deg, self.data.data_ptr())


class Scanner:
    """A scanner geometry plus image grid, i.e. one library handle.

    ``cfg`` is a dict with the keys of ``synth.CFG_2D`` (geometry in mm,
    image shape and voxel size)."""

    def __init__(self, cfg: dict, mode3d: bool = False):
        torch = _torch()
        self.L = _lib.load()
        self.cfg = dict(cfg)
        self.mode3d = bool(mode3d)
        self.geom = _lib.psf_geometry(int(cfg["n_blocks"]), int(cfg["n_ct"]), int(cfg.get("n_cz", 1)),
                                      int(cfg.get("n_brings", 1)), float(cfg["pitch_t"]),
                                      float(cfg.get("pitch_z", cfg["pitch_t"])), float(cfg["depth"]),
                                      float(cfg["r_face"]), float(cfg.get("gap_z", 0.0)), float(cfg["mu"]),
                                      float(cfg.get("phi0", 0.0)))
        self.img = _lib.psf_image(int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1)), 0, float(cfg["dx"]),
                                  float(cfg["dy"]), float(cfg.get("dz", 1.0)), float(cfg.get("cx", 0.0)),
                                  float(cfg.get("cy", 0.0)), float(cfg.get("cz", 0.0)))
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = C.c_void_p(0)
        check(self.L.psf_create(C.byref(self.geom), C.byref(self.img), int(self.mode3d), C.byref(h)), "psf_create")
        self.h = h
        nc, nb, nv = C.c_int64(), C.c_int64(), C.c_int64()
        check(self.L.psf_sizes(self.h, C.byref(nc), C.byref(nb), C.byref(nv)), "psf_sizes")
        self.n_crystals, self.n_bins, self.n_voxels = nc.value, nb.value, nv.value
        self._ws = None
        self._ws_clean = False  # a 3D build completed on self._ws since it was allocated

    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                self.L.psf_destroy(self.h)
                self.h = C.c_void_p(0)
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def opts(self, precision=PSF_FP32, threshold=0.0, vox_begin=0, vox_end=-1, accumulate=0, homog_k=0, flags=0,
             top_n=0):
        return _lib.psf_opts(int(precision), int(homog_k), float(threshold), int(vox_begin), int(vox_end),
                             int(accumulate), int(flags), int(top_n), 0)

    def workspace(self, table: Table, batch: int = 1, n_events: int = 0, opts=None):
        torch = _torch()
        o = opts or self.opts()
        n = C.c_size_t()
        tc = table.c()
        check(self.L.psf_workspace_size(self.h, C.byref(tc), C.byref(o), int(batch), int(n_events), C.byref(n)),
              "psf_workspace_size")
        if self._ws is None or self._ws.numel() < n.value:
            self._ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
            self._ws_clean = False
        return self._ws

    # -- entry points --------------------------------------------------------
    def build_table(self, n_rows: int = 61, n_sub: int = 4, step_deg: float = 1.0) -> Table:
        """Analytic response table computed on the device (psf_build_table)."""
        torch = _torch()
        if self.mode3d:
            numel = n_rows * n_rows * n_sub * n_sub * 25
        else:
            numel = n_rows * n_sub * 5
        data = torch.empty(numel, dtype=torch.float32, device=self.device)
        check(self.L.psf_build_table(self.h, int(n_rows), int(n_sub), float(step_deg), _ptr(data), _stream()),
              "psf_build_table")
        return Table(data, n_rows, n_sub, step_deg)

    def build_table_host(self, n_rows: int = 61, n_sub: int = 4, step_deg: float = 1.0):
        """The same analytic table in FP64 on the host (psf_build_table_host):
        numpy float64 in the layout of psf_table."""
        import numpy as np
        numel = n_rows * n_rows * n_sub * n_sub * 25 if self.mode3d else n_rows * n_sub * 5
        out = np.zeros(numel, dtype=np.float64)
        check(self.L.psf_build_table_host(C.byref(self.geom), int(self.mode3d), int(n_rows), int(n_sub),
                                          float(step_deg), C.c_void_p(out.ctypes.data)), "psf_build_table_host")
        return out

    def build_table_mc(self, n_rows: int = 61, n_sub: int = 4, step_deg: float = 1.0, photons: int = 100_000,
                       seed: int = 1, scatter: bool = False, counts: bool = False):
        """Response table by photon-transport Monte Carlo on the device
        (psf_build_table_mc): a Table, and with counts=True also the int64
        detected-photon counts [cells, 5, 5]."""
        torch = _torch()
        cells = n_rows * n_rows * n_sub * n_sub if self.mode3d else n_rows * n_sub
        data = torch.empty(cells * (25 if self.mode3d else 5), dtype=torch.float32, device=self.device)
        cnt = torch.empty(cells * 25, dtype=torch.int64, device=self.device) if counts else None
        check(self.L.psf_build_table_mc(self.h, int(n_rows), int(n_sub), float(step_deg), int(photons), int(seed),
                                        int(bool(scatter)), _ptr(data), _ptr(cnt), _stream()), "psf_build_table_mc")
        t = Table(data, n_rows, n_sub, step_deg)
        return (t, cnt.reshape(cells, 5, 5)) if counts else t

    def table_from(self, data, n_rows: int, n_sub: int, step_deg: float = 1.0) -> Table:
        """Wrap a caller-provided table (any shape with the right number of entries)."""
        torch = _torch()
        t = torch.as_tensor(data, dtype=torch.float32).reshape(-1).to(self.device).contiguous()
        return Table(t, n_rows, n_sub, step_deg)

    def voxel_order(self):
        """Linear voxel index of each position of the library's voxel order
        (psf_voxel_order): numpy int64 [n_voxels]."""
        import numpy as np
        out = np.zeros(self.n_voxels, dtype=np.int64)
        check(self.L.psf_voxel_order(self.h, C.c_void_p(out.ctypes.data)), "psf_voxel_order")
        return out

    def build_psf_sysmat(self, table: Table, threshold: float = 0.0, vox_begin: int = 0, vox_end: int = -1,
                         precision: int = PSF_FP32, stage: bool = True, counters: list | None = None,
                         class_order: bool = False, homog_k: int = 0, top_n: int = 0, deterministic: bool = False):
        """CSR of A^T for voxels [vox_begin, vox_end): (row_ptr int64, col int32, val float32).
        stage: the count phase keeps its rows in the workspace for the fill phase (3D).
        counters: if a list, each phase appends its header_counters() snapshot (3D).
        class_order: the range counts positions of voxel_order() (row k is voxel
        voxel_order()[vox_begin + k]).
        homog_k: 0 for the k -> infinity homogenization weights, k > 0 for k lines (2D).
        top_n: n > 0 keeps each voxel's n largest bins per sinogram angle (2D).
        deterministic: integer sums of the tile entries (PSF_OPT_DETERMINISTIC): the
        same CSR, bit for bit, on every run."""
        torch = _torch()
        flags = (_lib.PSF_OPT_STAGE_CSR if stage else 0) | (_lib.PSF_OPT_CLASS_ORDER if class_order else 0)
        flags |= _lib.PSF_OPT_DETERMINISTIC if deterministic else 0
        o = self.opts(precision, threshold, vox_begin, vox_end, flags=flags, homog_k=homog_k, top_n=top_n)
        ve = self.n_voxels if vox_end is None or vox_end < 0 else vox_end
        n = ve - vox_begin
        row_ptr = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        ws = self.workspace(table, 1, 0, o)
        if self._ws_clean:  # only this object's calls used the workspace since a build completed on it
            o.flags |= _lib.PSF_OPT_WS_CLEAN
        self._ws_clean = False
        tc = table.c()
        csr = _lib.psf_csr(n, 0, row_ptr.data_ptr(), None, None)
        check(self.L.build_psf_sysmat(self.h, C.byref(tc), C.byref(o), _ptr(ws), ws.numel(), C.byref(csr),
                                      _stream()), "build_psf_sysmat (count)")
        if counters is not None:
            counters.append(self.header_counters())
        nnz = csr.nnz
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(nnz, 1), dtype=torch.float32, device=self.device)
        csr.col, csr.val = col.data_ptr(), val.data_ptr()
        check(self.L.build_psf_sysmat(self.h, C.byref(tc), C.byref(o), _ptr(ws), ws.numel(), C.byref(csr),
                                      _stream()), "build_psf_sysmat (fill)")
        self._ws_clean = True
        if counters is not None:
            counters.append(self.header_counters())
        return row_ptr, col[:nnz], val[:nnz]

    def project_fwd(self, table: Table, x, events=None, precision: int = PSF_FP32, y=None, accumulate: int = 0,
                    homog_k: int = 0, top_n: int = 0):
        """y = A x (x: [batch, n_voxels] float32); with ``events`` (int32 [n, 2]
        crystal pairs) the list-mode rows y[batch, n]."""
        torch = _torch()
        x = _dev_f32(x, "x")
        x2 = x.reshape(-1, self.n_voxels)
        batch = x2.shape[0]
        ne = 0 if events is None else int(events.shape[0])
        nout = self.n_bins if events is None else ne
        if y is None:
            y = torch.empty(batch, nout, dtype=torch.float32, device=self.device)
        o = self.opts(precision, accumulate=accumulate, homog_k=homog_k, top_n=top_n)
        ws = self.workspace(table, batch, ne, o)
        tc = table.c()
        check(self.L.project_fwd(self.h, C.byref(tc), C.byref(o), _ptr(x2), batch, _events_ptr(events), ne, _ptr(y),
                                 _ptr(ws), ws.numel(), _stream()), "project_fwd")
        return y

    def project_adj(self, table: Table, y, events=None, xt=None, want_table_grad=False, precision: int = PSF_FP32,
                    x=None, accumulate: int = 0, top_n: int = 0):
        """x = A^T y; optionally also d<y, A xt>/d table.  Returns x or (x, grad)."""
        torch = _torch()
        y = _dev_f32(y, "y")
        ne = 0 if events is None else int(events.shape[0])
        nin = self.n_bins if events is None else ne
        y2 = y.reshape(-1, nin) if nin > 0 else y.reshape(y.shape[0] if y.dim() > 1 else 1, 0)
        batch = y2.shape[0]
        if x is None:
            x = torch.empty(batch, self.n_voxels, dtype=torch.float32, device=self.device)
        grad = None
        if want_table_grad:
            xt = _dev_f32(xt, "xt").reshape(batch, self.n_voxels)
            grad = torch.zeros_like(table.data)
        o = self.opts(precision, accumulate=accumulate, flags=_lib.PSF_OPT_TABLE_GRAD if want_table_grad else 0,
                      top_n=top_n)
        ws = self.workspace(table, batch, ne, o)
        tc = table.c()
        check(self.L.project_adj(self.h, C.byref(tc), C.byref(o), _ptr(y2), batch, _events_ptr(events), ne, _ptr(x),
                                 _ptr(xt if want_table_grad else None), _ptr(grad), _ptr(ws), ws.numel(),
                                 _stream()), "project_adj")
        return (x, grad) if want_table_grad else x

    def sensitivity(self, table: Table, precision: int = PSF_FP32, top_n: int = 0):
        torch = _torch()
        s = torch.empty(self.n_voxels, dtype=torch.float32, device=self.device)
        o = self.opts(precision, top_n=top_n)
        ws = self.workspace(table, 1, 0, o)
        tc = table.c()
        check(self.L.psf_sensitivity(self.h, C.byref(tc), C.byref(o), _ptr(s), _ptr(ws), ws.numel(), _stream()),
              "psf_sensitivity")
        return s

    def lm_osem_update(self, table: Table, events, x, sens, n_subsets: int, randoms: float,
                       precision: int = PSF_FP32):
        torch = _torch()
        x = _dev_f32(x, "x")
        sens = _dev_f32(sens, "sens")
        out = torch.empty_like(x)
        ne = int(events.shape[0])
        o = self.opts(precision)
        ws = self.workspace(table, 1, ne, o)
        tc = table.c()
        check(self.L.psf_lm_osem_update(self.h, C.byref(tc), C.byref(o), _ptr(events), ne, float(randoms),
                                        _ptr(sens), int(n_subsets), _ptr(x), _ptr(out), _ptr(ws), ws.numel(),
                                        _stream()), "psf_lm_osem_update")
        return out

    def subset_sensitivity(self, table: Table, n_subsets: int, subset: int, precision: int = PSF_FP32,
                           top_n: int = 0):
        """s_k = A^T m_k for OSEM subset k of n_subsets (psf_subset_sensitivity)."""
        torch = _torch()
        s = torch.empty(self.n_voxels, dtype=torch.float32, device=self.device)
        o = self.opts(precision, flags=_lib.PSF_OPT_OSEM, top_n=top_n)
        ws = self.workspace(table, 1, 0, o)
        tc = table.c()
        check(self.L.psf_subset_sensitivity(self.h, C.byref(tc), C.byref(o), int(n_subsets), int(subset), _ptr(s),
                                            _ptr(ws), ws.numel(), _stream()), "psf_subset_sensitivity")
        return s

    def osem_update(self, table: Table, y, x, sens_k, n_subsets: int, subset: int, precision: int = PSF_FP32,
                    top_n: int = 0):
        """One histogram OSEM subset update (psf_osem_update); returns x_out."""
        torch = _torch()
        y = _dev_f32(y, "y").reshape(-1)
        x = _dev_f32(x, "x").reshape(-1)
        sens_k = _dev_f32(sens_k, "sens_k").reshape(-1)
        out = torch.empty_like(x)
        o = self.opts(precision, flags=_lib.PSF_OPT_OSEM, top_n=top_n)
        ws = self.workspace(table, 1, 0, o)
        tc = table.c()
        check(self.L.psf_osem_update(self.h, C.byref(tc), C.byref(o), _ptr(y), int(n_subsets), int(subset),
                                     _ptr(sens_k), _ptr(x), _ptr(out), _ptr(ws), ws.numel(), _stream()),
              "psf_osem_update")
        return out

    def profile_start(self):
        """Start timing the contraction kernels with HIP events (psf_profile)."""
        check(self.L.psf_profile(self.h, 1, None, None), "psf_profile")

    def profile_stop(self):
        """{'contraction': (ms, launches), 'geometry': (ms, launches)} summed over recorded launches."""
        ms, n = (C.c_double * 2)(), (C.c_int64 * 2)()
        check(self.L.psf_profile(self.h, 0, C.cast(ms, C.c_void_p), C.cast(n, C.c_void_p)), "psf_profile")
        return {"contraction": (ms[0], n[0]), "geometry": (ms[1], n[1])}

    def tiles_last_call(self) -> int:
        """Tiles contracted by the last 3D call (from the workspace header)."""
        _torch().cuda.synchronize()
        return int(self._ws[64:72].cpu().view(__import__("torch").int64).item()) if self._ws is not None else 0

    def header_counters(self):
        """Device copy (stream-ordered, no synchronisation) of the last 3D call's tile counters."""
        return self._ws[64:80].clone() if self._ws is not None else None

    @staticmethod
    def read_counters(snap):
        """(tiles, voxel tiles) from a header_counters() snapshot."""
        if snap is None:
            return 0, 0
        t, v = snap.cpu().view(__import__("torch").int64).tolist()
        return int(t), int(v)

    def voxel_tiles_last_call(self) -> int:
        """(voxel, tile) pairs the last 3D call's tiles served (from the workspace header)."""
        _torch().cuda.synchronize()
        return int(self._ws[72:80].cpu().view(__import__("torch").int64).item()) if self._ws is not None else 0

    def check(self):
        """Synchronise and raise if a kernel flagged an error (e.g. angle range)."""
        ws = self._ws
        if ws is None:
            return
        check(self.L.psf_check(self.h, _ptr(ws), _stream()), "psf_check")


def _make_autograd():
    import torch

    class PsfProject(torch.autograd.Function):
        """y = A(table) x with a hand-written adjoint: backward returns
        A^T g for x and d<g, A x>/d table for the table entries."""

        @staticmethod
        def forward(ctx, x, table_data, scanner, meta, precision=PSF_FP32):
            n_rows, n_sub, step = meta
            tab = Table(table_data.contiguous(), n_rows, n_sub, step)
            y = scanner.project_fwd(tab, x, precision=precision)
            ctx.save_for_backward(x, table_data)
            ctx.scanner, ctx.meta, ctx.precision = scanner, meta, precision
            return y

        @staticmethod
        def backward(ctx, gy):
            x, table_data = ctx.saved_tensors
            n_rows, n_sub, step = ctx.meta
            tab = Table(table_data.contiguous(), n_rows, n_sub, step)
            need_t = ctx.needs_input_grad[1]
            gy = gy.contiguous()
            if need_t:
                gx, gt = ctx.scanner.project_adj(tab, gy, xt=x.reshape(gy.shape[0], -1).contiguous(),
                                                 want_table_grad=True, precision=ctx.precision)
                gt = gt.reshape(table_data.shape)
            else:
                gx, gt = ctx.scanner.project_adj(tab, gy, precision=ctx.precision), None
            return gx.reshape(x.shape), gt, None, None, None

    return PsfProject


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _make_autograd()
        return getattr(_Lazy._cls, name)


PsfProject = _Lazy()
