// C ABI of the library (declared in include/psf.h): argument checks, handle,
// workspace carving and kernel launches.  No exception crosses this boundary.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "api_internal.hpp"

using namespace psf;

namespace psf {
thread_local int g_last_hip = 0;
}

// Scratch of project_fwd_noalloc: the status word and the FP64 bin accumulator
// of one call, in device memory the library owns.  Each GPU the library runs
// on holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress gives for the device (the array's
// name is a host-side stand-in).
constexpr size_t kNoAllocScratch = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

// once per device, with that device current
static int scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return PSF_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev]) return PSF_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        psf::g_last_hip = (int)e;
        return PSF_EHIP;
    }
    g_scratch_dev[dev] = p;
    return PSF_OK;
}


static int check_geometry(const psf_geometry* g, const psf_image* im, int mode3d) {
    if (g->n_blocks < 3 || g->n_cryst_t < 1 || g->n_cryst_z < 1 || g->n_block_rings < 1) return PSF_EINVAL;
    if (!(g->pitch_t > 0) || !(g->pitch_z > 0) || !(g->depth > 0) || !(g->radius_face > 0) || !(g->mu > 0))
        return PSF_EINVAL;
    if (g->gap_z != 0.0) return PSF_EUNSUPPORTED;
    if (im->nx < 1 || im->ny < 1 || im->nz < 1 || !(im->dx > 0) || !(im->dy > 0) || !(im->dz > 0)) return PSF_EINVAL;
    if (mode3d == 0 && (g->n_cryst_z != 1 || g->n_block_rings != 1 || im->nz != 1)) return PSF_EINVAL;
    // blocks must not overlap on the polygon of face lines
    const double half_w = 0.5 * g->n_cryst_t * g->pitch_t;
    if (g->radius_face * tan(M_PI / g->n_blocks) - half_w < 0.0) return PSF_EGEOM;
    // every voxel centre strictly inside every face line (corners suffice: convex)
    for (int b = 0; b < g->n_blocks; ++b) {
        const double phi = g->phi0 + 2.0 * M_PI * b / g->n_blocks;
        const double c = cos(phi), s = sin(phi);
        for (int cxs = 0; cxs < 2; ++cxs)
            for (int cys = 0; cys < 2; ++cys) {
                const double x = (cxs ? 0.5 : -0.5) * (im->nx - 1) * im->dx + im->cx;
                const double y = (cys ? 0.5 : -0.5) * (im->ny - 1) * im->dy + im->cy;
                if (!(c * x + s * y < g->radius_face)) return PSF_EGEOM;
            }
    }
    return PSF_OK;
}

extern "C" {

int psf_create(const psf_geometry* geom, const psf_image* img, int32_t mode3d, psf_handle** out) {
    if (!geom || !img || !out) return PSF_EINVAL;
    *out = nullptr;
    if (mode3d != 0 && mode3d != 1) return PSF_EINVAL;
    const int st = check_geometry(geom, img, mode3d);
    if (st != PSF_OK) return st;
    psf_handle* h = new (std::nothrow) psf_handle();
    if (!h) return PSF_EINVAL;
    h->prof_on = false;
    h->frames_dev = nullptr;
    h->g = *geom;
    h->im = *img;
    h->mode3d = mode3d;
    const int64_t Nc = (int64_t)geom->n_blocks * geom->n_cryst_t;
    const int64_t rings = (int64_t)geom->n_cryst_z * geom->n_block_rings;
    h->n_crystals = mode3d ? Nc * rings : Nc;
    // 2D: unordered crystal pairs; 3D: transaxial pair major, then the ring pair
    h->n_bins = mode3d ? Nc * (Nc - 1) / 2 * rings * rings : h->n_crystals * (h->n_crystals - 1) / 2;
    h->n_vox = (int64_t)img->nx * img->ny * img->nz;
    h->sigma = geom->radius_face * tan(M_PI / geom->n_blocks) - 0.5 * geom->n_cryst_t * geom->pitch_t;
    double* fr = (double*)malloc(sizeof(double) * 2 * geom->n_blocks);
    for (int b = 0; b < geom->n_blocks; ++b) {
        const double phi = geom->phi0 + 2.0 * M_PI * b / geom->n_blocks;
        fr[2 * b] = cos(phi);
        fr[2 * b + 1] = sin(phi);
    }
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess && scratch_init(h->device) != PSF_OK) e = (hipError_t)psf::g_last_hip;
    if (e == hipSuccess) e = hipMalloc((void**)&h->frames_dev, sizeof(double) * 2 * geom->n_blocks);
    if (e == hipSuccess) e = hipMemcpy(h->frames_dev, fr, sizeof(double) * 2 * geom->n_blocks, hipMemcpyHostToDevice);
    free(fr);
    if (e != hipSuccess) {
        psf::g_last_hip = (int)e;
        if (h->frames_dev) (void)hipFree(h->frames_dev);
        delete h;
        return PSF_EHIP;
    }
    *out = h;
    return PSF_OK;
}

void psf_destroy(psf_handle* h) {
    if (!h) return;
    for (auto& e : h->prof_ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (h->frames_dev) (void)hipFree(h->frames_dev);
    if (h->aux) {  // the streams are the device's and stay; this handle's events go
        for (int i = 0; i < kAuxEvents; ++i) {
            (void)hipEventSynchronize(h->aux_ev[i]);
            (void)hipEventDestroy(h->aux_ev[i]);
        }
    }
    delete h;
}

int psf_sizes(const psf_handle* h, int64_t* n_crystals, int64_t* n_bins, int64_t* n_voxels) {
    if (!h) return PSF_EINVAL;
    if (n_crystals) *n_crystals = h->n_crystals;
    if (n_bins) *n_bins = h->n_bins;
    if (n_voxels) *n_voxels = h->n_vox;
    return PSF_OK;
}

const char* psf_status_string(int s) {
    switch (s) {
        case PSF_OK: return "ok";
        case PSF_EINVAL: return "invalid argument";
        case PSF_EGEOM: return "inconsistent geometry";
        case PSF_ERANGE: return "incidence angle beyond the response table";
        case PSF_ESIZE: return "buffer too small";
        case PSF_EHIP: return "HIP runtime error";
        case PSF_EOVERFLOW: return "fill phase exceeded the counted row sizes";
        case PSF_EUNSUPPORTED: return "unsupported geometry or options";
        case PSF_ECAPACITY: return "a fixed scratch capacity was exceeded (output incomplete)";
        default: return "unknown status";
    }
}

int psf_last_hip_error(void) { return psf::g_last_hip; }

}  // extern "C"

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

int64_t table_elems(const psf_handle* h, const psf_table* t) {
    if (h->mode3d) return (int64_t)t->n_rows * t->n_rows * t->n_sub * t->n_sub * kNb * kNb;
    return (int64_t)t->n_rows * t->n_sub * kNb;
}

int check_table(const psf_handle* h, const psf_table* t) {
    if (!t || !t->data) return PSF_EINVAL;
    if (t->n_rows < 1 || t->n_sub < 1 || !(t->step_deg > 0)) return PSF_EINVAL;
    return PSF_OK;
}

static Ring2D make_ring2d(const psf_handle* h, const psf_table* t, const psf_opts* o) {
    Ring2D G;
    G.R = h->g.n_blocks;
    G.nc = h->g.n_cryst_t;
    G.P = t->n_sub;
    G.Nc = G.R * G.nc;
    G.nseg = G.Nc * G.P;
    G.n_rows = t->n_rows;
    G.nx = h->im.nx;
    G.ny = h->im.ny;
    G.nbins = h->n_bins;
    G.nvox = h->n_vox;
    G.lam = h->g.pitch_t;
    G.half_w = 0.5 * h->g.n_cryst_t * h->g.pitch_t;
    G.rf = h->g.radius_face;
    G.sigma = h->sigma;
    G.step_deg = t->step_deg;
    G.two_pi_R = 2.0 * M_PI / h->g.n_blocks;
    G.dx = h->im.dx;
    G.dy = h->im.dy;
    G.cx = h->im.cx;
    G.cy = h->im.cy;
    G.frames = h->frames_dev;
    G.table = t->data;
    G.precision = o ? o->precision : PSF_FP32;
    G.homog_k = o ? o->homog_k : 0;
    G.top_n = o ? o->top_n : 0;
    G.det = 0;  // set by the matrix build
    return G;
}

static int check_2d_support(const psf_handle* h, const Ring2D& G, int mode) {
    if (G.top_n > 0 && (G.Nc % 2 != 0 || mode == kModeAdjGrad)) return PSF_EUNSUPPORTED;
    int dev = 0, maxsm = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSF_EHIP;
    if (hipDeviceGetAttribute(&maxsm, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return PSF_EHIP;
    if (voxel2d_smem_bytes(G, mode) > (size_t)maxsm) return PSF_EUNSUPPORTED;
    return PSF_OK;
}

int check_opts(const psf_opts* o, bool build) {
    if (!o) return PSF_EINVAL;
    if (o->precision < PSF_FP32 || o->precision > PSF_BF16X2) return PSF_EINVAL;
    if (o->homog_k < 0) return PSF_EINVAL;
    if (o->top_n < 0 || o->top_n > kTopNMax) return PSF_EINVAL;
    if (!build && (o->flags & PSF_OPT_DETERMINISTIC)) return PSF_EUNSUPPORTED;  // matrix builds only
    return PSF_OK;
}

// status word: zero at the start of a call, read back by psf_check
__global__ void k_zero_header(int* p) {
    if (threadIdx.x < kWsDense / sizeof(int)) p[threadIdx.x] = 0;
}

int zero_header(void* ws, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, st, (int*)ws);
    HIP_TRY(hipGetLastError());
    return PSF_OK;
}

int read_status(void* ws, hipStream_t st) {
    int s = 0;
    HIP_TRY(hipMemcpyAsync(&s, ws, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (s & kStatOverflow) return PSF_EOVERFLOW;
    if (s & kStatScratch) return PSF_ECAPACITY;
    if (s & kStatRange) return PSF_ERANGE;
    if (s & kStatGeom) return PSF_EGEOM;
    if (s & kStatEventBad) return PSF_EINVAL;
    return PSF_OK;
}

// Workspace layout, all regions 256-byte aligned:
//   header   status word (+ spare)
//   y64      FP64 bin accumulator [batch][n_bins]   (forward; list-mode rows)
//   g64      FP64 table-gradient accumulator [table entries]
//   h64      FP64 bin histogram [batch][n_bins]      (list-mode only)
//   h32      FP32 copy of h64                        (list-mode only)
//   back     FP32 back projection [n_voxels]         (LM-OSEM only)
struct WsLayout {
    size_t y64, g64, h64, h32, back, total;
};

static WsLayout ws_layout(const psf_handle* h, const psf_table* t, int batch, int64_t n_events) {
    WsLayout L;
    const size_t b = (size_t)(batch > 0 ? batch : 1);
    size_t off = kWsHeader;
    L.y64 = off;
    off += align256(sizeof(double) * b * (size_t)h->n_bins);
    L.g64 = off;
    off += align256(sizeof(double) * (size_t)table_elems(h, t));
    L.h64 = L.h32 = L.back = off;
    if (n_events > 0) {
        L.h64 = off;
        off += align256(sizeof(double) * b * (size_t)h->n_bins);
        L.h32 = off;
        off += align256(sizeof(float) * b * (size_t)h->n_bins);
        L.back = off;
        off += align256(sizeof(float) * (size_t)h->n_vox);
    }
    L.total = off;
    return L;
}

template <class T>
static T* at(void* ws, size_t off) {
    return (T*)((char*)ws + off);
}

extern "C" {

int psf_workspace_size(const psf_handle* h, const psf_table* table, const psf_opts* opts, int32_t batch,
                       int64_t n_events, size_t* bytes) {
    if (!h || !table || !bytes || batch < 0 || n_events < 0) return PSF_EINVAL;
    if (opts && (opts->flags & PSF_OPT_OSEM) && n_events == 0) n_events = 1;  // the OSEM sinogram buffers
    *bytes = h->mode3d ? ws3_total(h, table, batch, n_events, opts) : ws_layout(h, table, batch, n_events).total;
    return PSF_OK;
}

int psf_build_table(psf_handle* h, int32_t n_rows, int32_t n_sub, double step_deg, float* table_dev, void* stream) {
    if (!h || !table_dev || n_rows < 1 || n_sub < 1 || !(step_deg > 0)) return PSF_EINVAL;
    if (h->mode3d) {
        HIP_TRY(launch_table_3d(h->g, n_rows, n_sub, step_deg, table_dev, (hipStream_t)stream));
        return PSF_OK;
    }
    HIP_TRY(launch_table_2d(h->g, n_rows, n_sub, step_deg, table_dev, (hipStream_t)stream));
    return PSF_OK;
}

int psf_build_table_mc(psf_handle* h, int32_t n_rows, int32_t n_sub, double step_deg, int64_t photons, uint64_t seed,
                       int32_t scatter, float* table_dev, int64_t* counts_dev, void* stream) {
    if (!h || !table_dev || n_rows < 1 || n_sub < 1 || !(step_deg > 0)) return PSF_EINVAL;
    if (photons < 1 || photons >= ((int64_t)1 << 32) || (scatter != 0 && scatter != 1)) return PSF_EINVAL;
    const int64_t cells = h->mode3d ? (int64_t)n_rows * n_rows * n_sub * n_sub : (int64_t)n_rows * n_sub;
    if (cells >= ((int64_t)1 << 31)) return PSF_ESIZE;
    HIP_TRY(launch_table_mc(h->g, h->mode3d, n_rows, n_sub, step_deg, photons, seed, scatter, table_dev,
                            (long long*)counts_dev, (hipStream_t)stream));
    return PSF_OK;
}

int psf_build_table_host(const psf_geometry* geom, int32_t mode3d, int32_t n_rows, int32_t n_sub, double step_deg,
                         double* out) {
    if (!geom || !out || n_rows < 1 || n_sub < 1 || !(step_deg > 0) || (mode3d != 0 && mode3d != 1)) return PSF_EINVAL;
    if (!(geom->pitch_t > 0) || !(geom->pitch_z > 0) || !(geom->depth > 0) || !(geom->mu > 0)) return PSF_EINVAL;
    if (mode3d)
        table_3d_host(*geom, n_rows, n_sub, step_deg, out);
    else
        table_2d_host(*geom, n_rows, n_sub, step_deg, out);
    return PSF_OK;
}

int build_psf_sysmat(psf_handle* h, const psf_table* table, const psf_opts* opts, void* ws, size_t ws_bytes,
                     psf_csr* csr, void* stream) {
    if (!h || !csr || !ws) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts, true))) return st;
    if (h->mode3d) return build_sysmat_3d(h, table, opts, ws, ws_bytes, csr, (hipStream_t)stream);
    if (ws_bytes < kWsHeader) return PSF_ESIZE;
    const int64_t vb = opts->vox_begin, ve = opts->vox_end > 0 ? opts->vox_end : h->n_vox;
    if (vb < 0 || ve > h->n_vox || ve < vb) return PSF_EINVAL;
    if (!csr->row_ptr) return PSF_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    Ring2D G = make_ring2d(h, table, opts);
    G.det = (opts->flags & PSF_OPT_DETERMINISTIC) != 0;
    VoxArgs2D a;
    memset(&a, 0, sizeof(a));
    a.vox_begin = vb;
    a.n_vox_range = ve - vb;
    a.batch = 1;
    a.threshold = opts->threshold;
    a.row_ptr = csr->row_ptr;
    a.col = csr->col;
    a.val = csr->val;
    a.status = (int*)ws;
    csr->n_rows = ve - vb;
    const int mode = csr->col ? kModeFill : kModeCount;
    if ((st = check_2d_support(h, G, mode))) return st;
    if ((st = zero_header(ws, s))) return st;
    if (!csr->col) {
        {
            ProfScope ps_(h, s);
            HIP_TRY(launch_voxel2d(kModeCount, G, a, s));
        }
        HIP_TRY(launch_scan_rowptr(csr->row_ptr, ve - vb, s));
        int64_t nnz = 0;
        HIP_TRY(hipMemcpyAsync(&nnz, csr->row_ptr + (ve - vb), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        st = read_status(ws, s);  // synchronises
        csr->nnz = nnz;
        return st;
    }
    if (!csr->val) return PSF_EINVAL;
    int64_t need = 0;
    HIP_TRY(hipMemcpyAsync(&need, csr->row_ptr + (ve - vb), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (csr->nnz < need) {
        csr->nnz = need;
        return PSF_ESIZE;
    }
    {
        ProfScope ps_(h, s);
        HIP_TRY(launch_voxel2d(kModeFill, G, a, s));
    }
    return read_status(ws, s);
}

}  // extern "C"

// y64[batch][n_bins] = A x (FP64 accumulation), on the fly
static int fwd_bins(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* x, int batch,
                    double* y64, void* ws, hipStream_t s, bool prof = true) {
    Ring2D G = make_ring2d(h, table, opts);
    int st = check_2d_support(h, G, kModeFwd);
    if (st) return st;
    VoxArgs2D a;
    memset(&a, 0, sizeof(a));
    a.vox_begin = 0;
    a.n_vox_range = h->n_vox;
    a.batch = batch;
    a.x = x;
    a.y64 = y64;
    a.status = (int*)ws;
    HIP_TRY(launch_zero_f64(y64, (int64_t)batch * h->n_bins, s));
    if (!prof) {  // no timing events (they are created per launch)
        HIP_TRY(launch_voxel2d(kModeFwd, G, a, s));
        return PSF_OK;
    }
    {
        ProfScope ps_(h, s);
        HIP_TRY(launch_voxel2d(kModeFwd, G, a, s));
    }
    return PSF_OK;
}

// x[batch][n_voxels] = A^T y (y FP32 [batch][n_bins], or all ones), optionally
// with the table gradient accumulated into g64
static int adj_bins(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* y, int ones,
                    int batch, float* x, const float* xt, double* g64, int accumulate, void* ws, hipStream_t s) {
    Ring2D G = make_ring2d(h, table, opts);
    const int mode = g64 ? kModeAdjGrad : kModeAdj;
    int st = check_2d_support(h, G, mode);
    if (st) return st;
    // the table-gradient kernel keeps up to 8 images' voxel values in registers
    const int chunk = g64 ? 8 : batch;
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = batch - b0 < chunk ? batch - b0 : chunk;
        VoxArgs2D a;
        memset(&a, 0, sizeof(a));
        a.vox_begin = 0;
        a.n_vox_range = h->n_vox;
        a.batch = nb;
        a.y = ones ? nullptr : y + (int64_t)b0 * h->n_bins;
        a.ones = ones;
        a.xout = x + (int64_t)b0 * h->n_vox;
        a.x = xt ? xt + (int64_t)b0 * h->n_vox : nullptr;
        a.grad64 = g64;
        a.status = (int*)ws;
        a.accumulate = accumulate;
        {
            ProfScope ps_(h, s);
            HIP_TRY(launch_voxel2d(mode, G, a, s));
        }
    }
    return PSF_OK;
}

extern "C" {

int project_fwd(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* x, int32_t batch,
                const int32_t* events, int64_t n_events, float* y, void* ws, size_t ws_bytes, void* stream) {
    if (!h || !x || batch < 1 || n_events < 0) return PSF_EINVAL;
    if (events && n_events == 0) return PSF_OK;  // an empty event list: y has no entries
    if (!y || !ws) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if (h->mode3d)
        return project_fwd_3d(h, table, opts, x, batch, events, n_events, y, ws, ws_bytes, (hipStream_t)stream);
    const WsLayout L = ws_layout(h, table, batch, events ? n_events : 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const hipStream_t s = (hipStream_t)stream;
    if ((st = zero_header(ws, s))) return st;
    double* y64 = at<double>(ws, L.y64);
    if ((st = fwd_bins(h, table, opts, x, batch, y64, ws, s))) return st;
    if (events) {
        HIP_TRY(launch_lm_gather(y64, nullptr, h->n_bins, events, n_events, batch, h->n_crystals, 1, y,
                                 opts->accumulate, (int*)ws, s));
    } else {
        HIP_TRY(launch_finalize(y64, y, (int64_t)batch * h->n_bins, opts->accumulate, s));
    }
    return PSF_OK;
}

int project_fwd_noalloc(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* x, int32_t batch,
                        const int32_t* events, int64_t n_events, float* y, void* stream) {
    if (!h || !x || batch < 1 || n_events < 0) return PSF_EINVAL;
    if (events && n_events == 0) return PSF_OK;
    if (!y) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if (h->mode3d) return PSF_EUNSUPPORTED;
    const WsLayout L = ws_layout(h, table, batch, 0);  // header and the FP64 bin accumulator only
    if (L.g64 > kNoAllocScratch) return PSF_ESIZE;
    void* ws = (h->device >= 0 && h->device < kMaxDevices) ? g_scratch_dev[h->device] : nullptr;
    if (!ws) return PSF_EHIP;
    const hipStream_t s = (hipStream_t)stream;
    if ((st = zero_header(ws, s))) return st;
    double* y64 = at<double>(ws, L.y64);
    if ((st = fwd_bins(h, table, opts, x, batch, y64, ws, s, false))) return st;
    if (events) {
        HIP_TRY(launch_lm_gather(y64, nullptr, h->n_bins, events, n_events, batch, h->n_crystals, 1, y,
                                 opts->accumulate, (int*)ws, s));
    } else {
        HIP_TRY(launch_finalize(y64, y, (int64_t)batch * h->n_bins, opts->accumulate, s));
    }
    return PSF_OK;
}

int project_adj(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* y, int32_t batch,
                const int32_t* events, int64_t n_events, float* x, const float* xt, float* grad, void* ws,
                size_t ws_bytes, void* stream) {
    if (!h || !x || batch < 1 || n_events < 0) return PSF_EINVAL;
    if (grad && !xt) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if (events && n_events == 0) {  // an empty event list: x = 0 (kept when accumulating), nothing added to grad
        if (!opts->accumulate) HIP_TRY(launch_zero_f32(x, (int64_t)batch * h->n_vox, (hipStream_t)stream));
        return PSF_OK;
    }
    if (!y || !ws) return PSF_EINVAL;
    if (h->mode3d)
        return project_adj_3d(h, table, opts, y, 0, batch, events, n_events, x, grad ? xt : nullptr, grad, ws,
                              ws_bytes, (hipStream_t)stream);
    const WsLayout L = ws_layout(h, table, batch, events ? n_events : 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const hipStream_t s = (hipStream_t)stream;
    if ((st = zero_header(ws, s))) return st;
    const float* ybins = y;
    if (events) {
        double* h64 = at<double>(ws, L.h64);
        float* h32 = at<float>(ws, L.h32);
        const int64_t n = (int64_t)batch * h->n_bins;
        HIP_TRY(launch_zero_f64(h64, n, s));
        HIP_TRY(launch_lm_scatter(y, n_events, events, batch, h->n_crystals, 1, h->n_bins, h64, (int*)ws, s));
        HIP_TRY(launch_finalize(h64, h32, n, 0, s));
        ybins = h32;
    }
    double* g64 = grad ? at<double>(ws, L.g64) : nullptr;
    const int64_t tsize = table_elems(h, table);
    if (grad) HIP_TRY(launch_zero_f64(g64, tsize, s));
    if ((st = adj_bins(h, table, opts, ybins, 0, batch, x, xt, g64, opts->accumulate, ws, s))) return st;
    if (grad) HIP_TRY(launch_finalize(g64, grad, tsize, 1, s));
    return PSF_OK;
}

int psf_sensitivity(psf_handle* h, const psf_table* table, const psf_opts* opts, float* s_dev, void* ws,
                    size_t ws_bytes, void* stream) {
    if (!h || !s_dev || !ws) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if (h->mode3d)
        return project_adj_3d(h, table, opts, nullptr, 1, 1, nullptr, 0, s_dev, nullptr, nullptr, ws, ws_bytes,
                              (hipStream_t)stream);
    if (ws_bytes < ws_layout(h, table, 1, 0).total) return PSF_ESIZE;
    const hipStream_t s = (hipStream_t)stream;
    if ((st = zero_header(ws, s))) return st;
    return adj_bins(h, table, opts, nullptr, 1, 1, s_dev, nullptr, nullptr, 0, ws, s);
}

int psf_lm_osem_update(psf_handle* h, const psf_table* table, const psf_opts* opts, const int32_t* events,
                       int64_t n_events, float randoms, const float* sens, int32_t n_subsets, const float* x_in,
                       float* x_out, void* ws, size_t ws_bytes, void* stream) {
    if (!h || !events || !sens || !x_in || !x_out || !ws || n_events < 1 || n_subsets < 1) return PSF_EINVAL;
    if (!(randoms >= 0.0f)) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if (h->mode3d)
        return lm_osem_3d(h, table, opts, events, n_events, randoms, sens, n_subsets, x_in, x_out, ws, ws_bytes,
                          (hipStream_t)stream);
    const WsLayout L = ws_layout(h, table, 1, n_events);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const hipStream_t s = (hipStream_t)stream;
    if ((st = zero_header(ws, s))) return st;
    double* y64 = at<double>(ws, L.y64);
    double* h64 = at<double>(ws, L.h64);
    float* h32 = at<float>(ws, L.h32);
    float* back = at<float>(ws, L.back);
    // q_e = a_e^T x + r  ->  h[bin] += 1 / q_e  ->  back = A^T h  ->  update
    if ((st = fwd_bins(h, table, opts, x_in, 1, y64, ws, s))) return st;
    HIP_TRY(launch_zero_f64(h64, h->n_bins, s));
    HIP_TRY(launch_lm_ratio(y64, nullptr, events, n_events, h->n_crystals, 1, (double)randoms, h64, (int*)ws, s));
    HIP_TRY(launch_finalize(h64, h32, h->n_bins, 0, s));
    if ((st = adj_bins(h, table, opts, h32, 0, 1, back, nullptr, nullptr, 0, ws, s))) return st;
    HIP_TRY(launch_lm_update(x_in, back, sens, n_subsets, h->n_vox, x_out, s));
    return PSF_OK;
}

static int check_subsets(const psf_handle* h, int n_subsets, int subset) {
    const int64_t Nc = (int64_t)h->g.n_blocks * h->g.n_cryst_t;
    if (n_subsets < 1 || subset < 0 || subset >= n_subsets || n_subsets > Nc / 2) return PSF_EINVAL;
    return PSF_OK;
}

int psf_osem_update(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* y, int32_t n_subsets,
                    int32_t subset, const float* sens, const float* x_in, float* x_out, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!h || !y || !sens || !x_in || !x_out || !ws) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if ((st = check_subsets(h, n_subsets, subset))) return st;
    if (h->mode3d)
        return osem_3d(h, table, opts, y, n_subsets, subset, sens, x_in, x_out, ws, ws_bytes, (hipStream_t)stream);
    const WsLayout L = ws_layout(h, table, 1, 1);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const hipStream_t s = (hipStream_t)stream;
    if ((st = zero_header(ws, s))) return st;
    double* y64 = at<double>(ws, L.y64);
    float* r = at<float>(ws, L.h32);
    float* back = at<float>(ws, L.back);
    const int64_t Nc = h->n_crystals;
    if ((st = fwd_bins(h, table, opts, x_in, 1, y64, ws, s))) return st;
    HIP_TRY(launch_osem_ratio(y64, nullptr, y, h->n_bins, Nc, 1, n_subsets, subset, r, s));
    if ((st = adj_bins(h, table, opts, r, 0, 1, back, nullptr, nullptr, 0, ws, s))) return st;
    HIP_TRY(launch_osem_update(x_in, back, sens, h->n_vox, x_out, s));
    return PSF_OK;
}

int psf_subset_sensitivity(psf_handle* h, const psf_table* table, const psf_opts* opts, int32_t n_subsets,
                           int32_t subset, float* s_dev, void* ws, size_t ws_bytes, void* stream) {
    if (!h || !s_dev || !ws) return PSF_EINVAL;
    int st = check_table(h, table);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if ((st = check_subsets(h, n_subsets, subset))) return st;
    if (h->mode3d)
        return subset_sensitivity_3d(h, table, opts, n_subsets, subset, s_dev, ws, ws_bytes, (hipStream_t)stream);
    const WsLayout L = ws_layout(h, table, 1, 1);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const hipStream_t s = (hipStream_t)stream;
    if ((st = zero_header(ws, s))) return st;
    float* m = at<float>(ws, L.h32);
    HIP_TRY(launch_subset_mask(h->n_bins, h->n_crystals, 1, n_subsets, subset, m, s));
    return adj_bins(h, table, opts, m, 0, 1, s_dev, nullptr, nullptr, 0, ws, s);
}

int psf_profile(psf_handle* h, int32_t enable, double* ms, int64_t* launches) {
    if (!h) return PSF_EINVAL;
    auto clear = [h]() {
        for (auto& e : h->prof_ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        h->prof_ev.clear();
        h->prof_kind.clear();
    };
    if (enable) {
        clear();
        h->prof_on = true;
        return PSF_OK;
    }
    double tot[2] = {0.0, 0.0};
    int64_t cnt[2] = {0, 0};
    int st = PSF_OK;
    for (size_t i = 0; i < h->prof_ev.size(); ++i) {
        float t = 0.0f;
        hipError_t r = hipEventSynchronize(h->prof_ev[i].second);
        if (r == hipSuccess) r = hipEventElapsedTime(&t, h->prof_ev[i].first, h->prof_ev[i].second);
        if (r != hipSuccess) {
            psf::g_last_hip = (int)r;
            st = PSF_EHIP;
        }
        const int k = h->prof_kind[i] ? 1 : 0;
        tot[k] += t;
        cnt[k] += 1;
    }
    if (ms) {
        ms[0] = tot[0];
        ms[1] = tot[1];
    }
    if (launches) {
        launches[0] = cnt[0];
        launches[1] = cnt[1];
    }
    clear();
    h->prof_on = false;
    return st;
}

int psf_voxel_order(psf_handle* h, int64_t* order) {
    if (!h || !order) return PSF_EINVAL;
    if (!h->mode3d) {
        for (int64_t k = 0; k < h->n_vox; ++k) order[k] = k;
        return PSF_OK;
    }
    return voxel_order_3d(h, order);
}

int psf_check(psf_handle* h, void* ws, void* stream) {
    if (!h || !ws) return PSF_EINVAL;
    return read_status(ws, (hipStream_t)stream);
}

}  // extern "C"
