// 3D-scanner halves of the C-ABI entry points: argument checks, workspace
// carving and the batched launches of the cyl3d.hip kernels.
#include <math.h>
#include <stddef.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "api_internal.hpp"

using namespace psf;

namespace {

constexpr int kBatchCsr = 1024;   // voxels per batch of the matrix build (dense accumulators, FP32: about 67 GB)
constexpr int kShareCsr = 16;     // voxels of one column in a class of the matrix build (interleaved accumulators)
constexpr int kBatchProj = 4096;  // voxels per batch of the projections (fewer, fuller launches)
constexpr int kClsBatch = 2047;   // classes per batch: a tile record's header holds the class index in 11 bits
constexpr int kMaxMemProj = 256;  // voxels of a projection class with images or the axial mirror (16 z-shifts x 8 images x 2)
constexpr int kCapSamples = 4096;
constexpr int kCapPairs = 1024;
constexpr int kCapSlots = 4096;
constexpr int64_t kRecsPerVoxel = 65536;   // tile records allowed for one voxel
constexpr int64_t kRecBudget = 1 << 21;    // tile records per batch (1.1 KB each)
constexpr int kUvRings = 16;               // response-row table: rings per batch beyond the members, in NR
constexpr int64_t kStagePerVoxel = 262144;  // staged cells (8 B; non-zeros and the band's zeros) per voxel of the range
constexpr int64_t kStageMax = (int64_t)1 << 32;  // at most 32 GB of staged entries

// the count phase's record of what it staged (workspace header, kWsStage)
struct StageState {
    int full;                // device: a row did not fit
    int batches;             // device: batches fully staged
    unsigned long long magic;
    const void* table;
    int64_t vb, ve;
    double threshold;
    int32_t precision, n_rows, n_sub, n_batches;
};
static_assert(kWsStage + sizeof(StageState) <= kWsDense, "stage state fits the header");
constexpr unsigned long long kStageMagic = 0x5053465354414745ull;

Cyl3D make_cyl3d(const psf_handle* h, const psf_table* t, const psf_opts* o) {
    Cyl3D G;
    G.R = h->g.n_blocks;
    G.nc = h->g.n_cryst_t;
    G.P = t->n_sub;
    G.Nc = G.R * G.nc;
    G.nseg = G.Nc * G.P;
    G.n_rows = t->n_rows;
    G.NR = h->g.n_cryst_z * h->g.n_block_rings;
    G.nx = h->im.nx;
    G.ny = h->im.ny;
    G.nz = h->im.nz;
    G.nvox = h->n_vox;
    G.ntbins = (int64_t)G.Nc * (G.Nc - 1) / 2;
    G.nbins = h->n_bins;
    G.lam = h->g.pitch_t;
    G.half_w = 0.5 * h->g.n_cryst_t * h->g.pitch_t;
    G.rf = h->g.radius_face;
    G.sigma = h->sigma;
    G.step_deg = t->step_deg;
    G.two_pi_R = 2.0 * M_PI / h->g.n_blocks;
    G.sin_two_pi_R = sin(2.0 * M_PI / h->g.n_blocks);
    G.lz = h->g.pitch_z;
    G.z0 = -0.5 * G.NR * G.lz;
    G.dx = h->im.dx;
    G.dy = h->im.dy;
    G.dz = h->im.dz;
    G.cx = h->im.cx;
    G.cy = h->im.cy;
    G.cz = h->im.cz;
    G.frames = h->frames_dev;
    G.table = t->data;
    G.precision = o ? o->precision : PSF_FP32;
    return G;
}

int check3d(const psf_handle* h, const psf_table* t, const psf_opts* o) {
    if (o && o->homog_k > 0) return PSF_EUNSUPPORTED;  // the 3D weights are the k -> infinity solid angles
    if (o && o->top_n > 0) return PSF_EUNSUPPORTED;    // the truncation per sinogram angle is built for the 2D ring
    if (t->n_sub > 4) return PSF_EUNSUPPORTED;  // tiles hold P^2 <= 16 sub-patches
    const int64_t nseg = (int64_t)h->g.n_blocks * h->g.n_cryst_t * t->n_sub;
    if (nseg >= 32768) return PSF_EUNSUPPORTED;
    if (h->n_bins >= ((int64_t)1 << 31)) return PSF_EUNSUPPORTED;  // bins are int32 CSR columns
    // tile records hold rings offset by 512 in 10 bits, and voxel ids are int32 in the batch plans
    if ((int64_t)h->g.n_cryst_z * h->g.n_block_rings > 255) return PSF_EUNSUPPORTED;
    if (h->n_vox >= ((int64_t)1 << 31)) return PSF_EUNSUPPORTED;
    return PSF_OK;
}

struct Ws3 {
    size_t counts, sidx, sth, pairs, slotmap, slot_tbin, slot_order, dense, band, bandc, chunks, recs, reccount, uvtab, uvmask, xrep, xm, uvgrad,
        g64, plan, stage_cb, stage_cn, stage_nch, stage_cnt, stage_col, stage_val, x64, ydiag, y32, h64, h32, back, total;
    int64_t table_elems, cap_stage, stage_rows;  // stage: entries; rows with a region of kStagePerVoxel
    int bmax, bcsr, cap_slots, band_rows;
    int64_t dense_slab;  // cells of one member's share of the build accumulators
    int det;             // deterministic build: 64-bit integer cells (fix62) instead of FP32
    int64_t max_chunks;
    int64_t cap_recs, per_vox;
    int64_t cap_uv_rings, cap_uv;  // response-row table: (relative ring) slots per crystal, and in all
    // staged builds: a second set of the per-batch slot and band arrays (and the
    // counters), so that one batch's compaction overlaps the next batch's geometry
    size_t counts2, slotmap2, slot_tbin2, slot_order2, band2, bandc2;
    int set2;
    // the projections (no staging): a second set of the geometry's outputs, so
    // that one batch's geometry overlaps the previous batch's contraction
    size_t sidx2, sth2, pairs2, recs2, reccount2, uvtab2, uvmask2;
    int geo2;
};

Ws3 ws3_layout(const psf_handle* h, const psf_table* t, int batch, int64_t n_events, int grad, int64_t stage_rows,
               int det = 0) {
    Ws3 L;
    L.det = det;
    const int64_t Nc = (int64_t)h->g.n_blocks * h->g.n_cryst_t;
    const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
    const int64_t ntbins = Nc * (Nc - 1) / 2;
    const size_t b = (size_t)(batch > 0 ? batch : 1);
    L.bmax = (int)(h->n_vox < kBatchProj ? h->n_vox : kBatchProj);
    L.bcsr = (int)(h->n_vox < kBatchCsr ? h->n_vox : kBatchCsr);
    L.cap_slots = (int)(ntbins < kCapSlots ? ntbins : kCapSlots);
    size_t off = kWsHeader;
    L.counts = off;
    off += align256(sizeof(int) * 3 * (size_t)L.bmax);
    L.sidx = off;
    off += align256(sizeof(int) * (size_t)L.bmax * kCapSamples);
    L.sth = off;
    off += align256(sizeof(double) * 2 * (size_t)L.bmax * kCapSamples);
    L.pairs = off;
    off += align256(sizeof(int4) * (size_t)L.bmax * kCapPairs);
    L.slotmap = off;
    off += align256(sizeof(int) * (size_t)L.bcsr * ntbins);
    L.slot_tbin = off;
    off += align256(sizeof(int) * (size_t)L.bcsr * L.cap_slots);
    L.slot_order = off;
    off += align256(sizeof(int) * (size_t)L.bcsr * L.cap_slots);
    L.dense = off;  // a class of n members takes n slabs: [slot][NR + n - 1][NR + n - 1][n]
    L.dense_slab = (int64_t)L.cap_slots * (NR + kShareCsr - 1) * (NR + kShareCsr - 1);
    off += align256((det ? sizeof(unsigned long long) : sizeof(float)) * (size_t)L.bcsr * L.dense_slab);
    L.band = off;  // a build class's s_max is below kShareCsr
    L.band_rows = (int)NR + kShareCsr + 3;
    off += align256(sizeof(int2) * (size_t)L.bcsr * L.cap_slots * L.band_rows);
    L.bandc = off;
    off += align256(sizeof(int2) * (size_t)L.bcsr * L.cap_slots * L.band_rows);
    L.chunks = off;
    // chunks of a row: over member rows (slot, r_i), or over a column group's
    // accumulator rows (slot, i < NR + s_max), whichever are more
    L.max_chunks = cyl3d_max_chunks(L.cap_slots, (int)NR + kShareCsr - 1);
    off += align256(sizeof(int) * (size_t)L.bcsr * L.max_chunks);
    {
        L.per_vox = Nc * NR * 2 < kRecsPerVoxel ? (Nc * NR * 2 > 1024 ? Nc * NR * 2 : 1024) : kRecsPerVoxel;
        L.cap_recs = L.per_vox * L.bmax < kRecBudget ? L.per_vox * L.bmax : kRecBudget;
        if (L.cap_recs < L.per_vox) L.cap_recs = L.per_vox;
    }
    L.recs = off;
    off += align256(sizeof(float) * (size_t)L.cap_recs * kRecFloats);
    L.reccount = off;
    off += align256(sizeof(unsigned int));
    // a batch's classes need NR + s_max ring slots each, s_max + 1 their members
    L.cap_uv_rings = kUvRings * NR + (L.bmax > L.bcsr ? L.bmax : L.bcsr);
    L.cap_uv = Nc * L.cap_uv_rings;
    L.uvtab = off;
    off += align256(sizeof(float) * 400 * (size_t)L.cap_uv);
    L.uvmask = off;
    off += align256(sizeof(int) * (size_t)L.cap_uv);
    L.xrep = off;  // cleared at carving and by every fold
    off += align256(sizeof(double) * kXRep * 8 * (size_t)(L.bmax > L.bcsr ? L.bmax : L.bcsr));
    L.xm = off;
    off += align256(sizeof(float) * 8 * (size_t)(L.bmax > L.bcsr ? L.bmax : L.bcsr));
    // table gradient: per-slot accumulator (cleared by the fold into the table) and the FP64 table
    L.table_elems = (int64_t)t->n_rows * t->n_rows * t->n_sub * t->n_sub * 25;
    L.uvgrad = L.g64 = 0;
    if (grad) {
        L.uvgrad = off;
        off += align256(sizeof(double) * 400 * (size_t)L.cap_uv);
        L.g64 = off;
        off += align256(sizeof(double) * kGradRep * (size_t)L.table_elems);
    }
    L.plan = off;  // classes, members, row-table offsets and images of every batch: at most 2 int4 + 2 int per voxel
    off += align256((2 * sizeof(int4) + 2 * sizeof(int)) * (size_t)h->n_vox);
    // matrix build staging (count phase -> fill phase)
    L.cap_stage = stage_rows > 0 ? (stage_rows * kStagePerVoxel < kStageMax ? stage_rows * kStagePerVoxel : kStageMax)
                                 : 0;
    L.stage_rows = L.cap_stage / kStagePerVoxel;
    L.stage_cb = L.stage_cn = L.stage_nch = L.stage_cnt = L.stage_col = L.stage_val = 0;
    if (L.cap_stage > 0) {
        L.stage_cb = off;
        off += align256(sizeof(int64_t) * (size_t)stage_rows * L.max_chunks);
        L.stage_cn = off;
        off += align256(sizeof(int) * (size_t)stage_rows * L.max_chunks);
        L.stage_nch = off;
        off += align256(sizeof(int) * (size_t)stage_rows);
        L.stage_cnt = off;
        off += align256(sizeof(int) * (size_t)stage_rows);
        L.stage_col = off;
        off += align256(sizeof(int32_t) * (size_t)L.cap_stage);
        L.stage_val = off;
        off += align256(sizeof(float) * (size_t)L.cap_stage);
    }
    L.set2 = L.cap_stage > 0;
    L.geo2 = 1;
    L.counts2 = L.slotmap2 = L.slot_tbin2 = L.slot_order2 = L.band2 = L.bandc2 = 0;
    L.sidx2 = L.sth2 = L.pairs2 = L.recs2 = L.reccount2 = L.uvtab2 = L.uvmask2 = 0;
    L.counts2 = off;
    off += align256(sizeof(int) * 3 * (size_t)L.bmax);
    if (L.geo2) {
        L.sidx2 = off;
        off += align256(sizeof(int) * (size_t)L.bmax * kCapSamples);
        L.sth2 = off;
        off += align256(sizeof(double) * 2 * (size_t)L.bmax * kCapSamples);
        L.pairs2 = off;
        off += align256(sizeof(int4) * (size_t)L.bmax * kCapPairs);
        L.recs2 = off;
        off += align256(sizeof(float) * (size_t)L.cap_recs * kRecFloats);
        L.reccount2 = off;
        off += align256(2 * sizeof(unsigned int));
        L.uvtab2 = off;
        off += align256(sizeof(float) * 400 * (size_t)L.cap_uv);
        L.uvmask2 = off;
        off += align256(sizeof(int) * (size_t)L.cap_uv);
    }
    if (L.set2) {
        L.slotmap2 = off;
        off += align256(sizeof(int) * (size_t)L.bcsr * ntbins);
        L.slot_tbin2 = off;
        off += align256(sizeof(int) * (size_t)L.bcsr * L.cap_slots);
        L.slot_order2 = off;
        off += align256(sizeof(int) * (size_t)L.bcsr * L.cap_slots);
        L.band2 = off;
        off += align256(sizeof(int2) * (size_t)L.bcsr * L.cap_slots * L.band_rows);
        L.bandc2 = off;
        off += align256(sizeof(int2) * (size_t)L.bcsr * L.cap_slots * L.band_rows);
    }
    L.x64 = off;
    off += align256(sizeof(double) * b * (size_t)h->n_vox);
    L.ydiag = off;  // up to 8 sinograms in the diagonal ring-pair layout
    off += align256(sizeof(float) * (b < 8 ? b : 8) * (size_t)h->n_bins);
    L.y32 = L.h64 = L.h32 = L.back = off;
    if (n_events > 0) {
        L.y32 = off;
        off += align256(sizeof(float) * b * (size_t)h->n_bins);
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
T* at3(void* ws, size_t off) {
    return (T*)((char*)ws + off);
}

Scratch3D make_scratch(void* ws, const Ws3& L) {
    Scratch3D S;
    S.cap_samples = kCapSamples;
    S.cap_pairs = kCapPairs;
    S.cap_slots = L.cap_slots;
    int* c = at3<int>(ws, L.counts);
    S.n_samples = c;
    S.n_pairs = c + L.bmax;
    S.n_slots = c + 2 * L.bmax;
    S.sidx = at3<int>(ws, L.sidx);
    S.sth = at3<double>(ws, L.sth);
    S.pairs = at3<int4>(ws, L.pairs);
    S.slotmap = at3<int>(ws, L.slotmap);
    S.slot_tbin = at3<int>(ws, L.slot_tbin);
    S.slot_order = at3<int>(ws, L.slot_order);
    S.dense = at3<float>(ws, L.dense);
    S.dense_slab = L.dense_slab;
    S.det = L.det;
    S.chunk_counts = at3<int>(ws, L.chunks);
    S.max_chunks = L.max_chunks;
    S.recs = at3<float>(ws, L.recs);
    S.rec_count = at3<unsigned int>(ws, L.reccount);
    S.cap_recs = L.cap_recs;
    S.uvtab = at3<float>(ws, L.uvtab);
    S.uvmask = at3<int>(ws, L.uvmask);
    S.cap_uv = L.cap_uv;
    S.xrep = at3<double>(ws, L.xrep);
    S.cap_mem = L.bmax > L.bcsr ? L.bmax : L.bcsr;
    S.uvgrad = L.uvgrad ? at3<double>(ws, L.uvgrad) : nullptr;
    S.xm = at3<float>(ws, L.xm);
    S.band = at3<int2>(ws, L.band);
    S.bandc = at3<int2>(ws, L.bandc);
    S.band_rows = L.band_rows;
    return S;
}

// the scratch of odd batches of the projections: the second set of the
// geometry's outputs (bundles, pairs, counters, response rows, tile records),
// everything else shared
Scratch3D make_scratch_geo_odd(void* ws, const Ws3& L) {
    Scratch3D S = make_scratch(ws, L);
    if (!L.geo2) return S;
    int* c = at3<int>(ws, L.counts2);
    S.n_samples = c;
    S.n_pairs = c + L.bmax;
    S.n_slots = c + 2 * L.bmax;
    S.sidx = at3<int>(ws, L.sidx2);
    S.sth = at3<double>(ws, L.sth2);
    S.pairs = at3<int4>(ws, L.pairs2);
    S.recs = at3<float>(ws, L.recs2);
    S.rec_count = at3<unsigned int>(ws, L.reccount2);
    S.uvtab = at3<float>(ws, L.uvtab2);
    S.uvmask = at3<int>(ws, L.uvmask2);
    return S;
}

// the scratch of odd batches of a staged build: the second sets of the
// geometry's outputs and of the slots and bands, everything else shared
Scratch3D make_scratch_odd(void* ws, const Ws3& L) {
    Scratch3D S = make_scratch_geo_odd(ws, L);
    if (!L.set2) return S;
    int* c = at3<int>(ws, L.counts2);
    S.n_samples = c;
    S.n_pairs = c + L.bmax;
    S.n_slots = c + 2 * L.bmax;
    S.slotmap = at3<int>(ws, L.slotmap2);
    S.slot_tbin = at3<int>(ws, L.slot_tbin2);
    S.slot_order = at3<int>(ws, L.slot_order2);
    S.band = at3<int2>(ws, L.band2);
    S.bandc = at3<int2>(ws, L.bandc2);
    return S;
}

// The second and third streams (the build's compaction and geometry; the
// forward's geometry), one pair per device for the process, and the handle's
// events that order them against the caller's stream: created on first use,
// at the default priority.  False when they cannot be had (another device is
// current, or creation failed): the work then runs on the caller's stream.
bool aux_stream(psf_handle* h) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device || dev < 0 || dev >= kAuxDevices) return false;
    if (h->aux) return true;
    // the streams: two per device for the process, shared by every handle, so
    // that handles do not multiply the streams the hardware queues serve
    static std::mutex mu;
    static hipStream_t dev_streams[kAuxDevices][2];
    {
        std::lock_guard<std::mutex> lock(mu);
        if (!dev_streams[dev][0]) {
            hipStream_t st = nullptr, st2 = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return false;
            if (hipStreamCreateWithFlags(&st2, hipStreamNonBlocking) != hipSuccess) {
                (void)hipStreamDestroy(st);
                return false;
            }
            dev_streams[dev][0] = st;
            dev_streams[dev][1] = st2;
        }
    }
    hipEvent_t ev[kAuxEvents] = {};
    for (int i = 0; i < kAuxEvents; ++i) {
        if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
            for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
            return false;
        }
    }
    h->aux = dev_streams[dev][0];
    h->aux2 = dev_streams[dev][1];
    for (int i = 0; i < kAuxEvents; ++i) h->aux_ev[i] = ev[i];
    return true;
}

// ---------------------------------------------------------------------------
// classes of voxels and batches
// ---------------------------------------------------------------------------
// A class is a run of voxels of one z-column, iz = iz0 + m s for s = 0, 1, ...,
// where m dz is the ring pitch: the scanner seen from member s is the one seen
// from the reference (s = 0) moved by s rings.  When the pitch is not a whole
// number of voxels every voxel is its own class.  Classes are cut to at most
// `cmax` members and packed into batches of at most `bmax` members whose tile
// record estimates fit the record buffer and whose response rows fit the table.

struct Batch3 {
    int cls0, ncls, mem0, nmem;
    int64_t uv_slots;  // response-row slots of the batch
};

struct Plan3 {
    std::vector<int4> cls, mem;  // cls: reference voxel, first member (batch-relative), count, largest shift
    std::vector<int> uvoff;      // mem: voxel, shift, class (batch-relative), CSR row
    std::vector<int> sym;        // uvoff: first response-row slot of the class (batch-relative)
    std::vector<Batch3> batches; // sym: voxels per column | axial mirror << 8 | image codes of columns 1..7
                                 //      << 9 (3 bits each)
};

int64_t class_recs(const Ws3& L, int64_t NR, int n) {
    return (L.per_vox * (NR + n - 1) + NR - 1) / NR;
}

// The image is symmetric under the scanner's quarter turns and its mirror
// y -> -y when it is square, centred on the axis and the block layout starts on
// the x axis: image `code` (bit 2: mirror first; bits 0-1: quarter turns
// counter-clockwise) of column (ix, iy).
static bool square_symmetry(const psf_handle* h) {
    return h->im.nx == h->im.ny && h->im.dx == h->im.dy && h->im.cx == 0.0 && h->im.cy == 0.0 &&
           h->g.n_blocks % 4 == 0 && h->g.phi0 == 0.0;
}

static int64_t column_image(int code, int64_t n, int64_t ixy) {
    int64_t ix = ixy % n, iy = ixy / n;
    if (code & 4) iy = n - 1 - iy;
    for (int k = 0; k < (code & 3); ++k) {
        const int64_t t = ix;
        ix = n - 1 - iy;
        iy = t;
    }
    return iy * n + ix;
}

// sym: classes may join the images of a column under the square's symmetry.
// zmir: a class may also take the axial mirror image of its z-run (z -> -z
// about the scanner's centre), when the image grid is centred axially.
// share: most voxels of one column in a class.
Plan3 plan3(const psf_handle* h, const Ws3& L, int64_t vb, int64_t ve, int bmax, bool sym, int share, bool zmir,
            int max_mem = 128) {
    Plan3 pl;
    const int64_t nx = h->im.nx, ny = h->im.ny, nz = h->im.nz, nxy = nx * ny;
    const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
    int64_t m = 0;
    const double q = nearbyint(h->g.pitch_z / h->im.dz);
    if (q >= 1.0 && q < 1e6 && fabs(q * h->im.dz - h->g.pitch_z) <= 1e-12 * h->g.pitch_z) m = (int64_t)q;
    const int64_t Nc = (int64_t)h->g.n_blocks * h->g.n_cryst_t;
    sym = sym && square_symmetry(h);
    zmir = zmir && h->im.cz == 0.0;
    int cmax = bmax < share ? bmax : share;
    while (cmax > 1 && (class_recs(L, NR, cmax) > L.cap_recs || NR + cmax - 1 > L.cap_uv_rings)) --cmax;
    Batch3 cur = {0, 0, 0, 0, 0};
    int64_t cur_recs = 0;
    // a class: reference voxel v0, nz voxels step `step` apart in z, in the
    // columns images[0..ni) (image 0 the reference's own column), and with
    // `mir` also the axial mirror images of those voxels (listed in z order)
    auto add_class = [&](int64_t v0, int64_t step, int nzc, const int64_t* cols, const int* codes, int ni, int mir) {
        const int n = nzc * ni * (mir ? 2 : 1);
        const int64_t need = class_recs(L, NR, nzc), uv = Nc * (NR + nzc - 1);
        if (cur.nmem > 0 && (cur.nmem + n > bmax || cur.ncls + 1 > kClsBatch || cur_recs + need > L.cap_recs ||
                             cur.uv_slots + uv > L.cap_uv)) {
            pl.batches.push_back(cur);
            cur = {(int)pl.cls.size(), 0, (int)pl.mem.size(), 0, 0};
            cur_recs = 0;
        }
        pl.cls.push_back(make_int4((int)v0, cur.nmem, n, nzc - 1));
        pl.uvoff.push_back((int)cur.uv_slots);
        int sc = nzc | (mir ? 1 << 8 : 0);
        for (int i = 1; i < ni; ++i) sc |= codes[i] << (3 * i + 6);
        pl.sym.push_back(sc);
        cur.uv_slots += uv;
        const int64_t z0 = v0 / nxy, zm = nz - 1 - (z0 + (int64_t)(nzc - 1) * (step / nxy));
        for (int i = 0; i < ni; ++i)
            for (int h2 = 0; h2 < (mir ? 2 : 1); ++h2)
                for (int k = 0; k < nzc; ++k) {
                    const int64_t v = cols[i] + ((h2 ? zm : z0) * nxy + k * step);
                    pl.mem.push_back(make_int4((int)v, k, cur.ncls, (int)(v - vb)));
                }
        cur.ncls += 1;
        cur.nmem += n;
        cur_recs += need;
    };
    auto zrange = [&](int64_t ixy, int64_t* zlo, int64_t* zhi) {
        *zlo = vb - ixy <= 0 ? 0 : (vb - ixy + nxy - 1) / nxy;
        *zhi = ve - 1 - ixy < 0 ? -1 : (ve - 1 - ixy) / nxy;
        if (*zhi > nz - 1) *zhi = nz - 1;
    };
    // the columns of one class group, all with the z range [zlo, zhi]
    auto add_columns = [&](const int64_t* cols, const int* codes, int ni, int64_t zlo, int64_t zhi) {
        if (zlo > zhi) return;
        if (m == 0) {
            for (int64_t iz = zlo; iz <= zhi; ++iz) add_class(cols[0] + iz * nxy, 0, 1, cols, codes, ni, 0);
            return;
        }
        // classes with images or the axial mirror hold at most max_mem members
        // (the contraction's emission keeps a class's member values in LDS): half
        // of them in the reference half
        int run = cmax;
        if (ni > 1 && run * ni > max_mem / 2) run = max_mem / 2 / ni;
        std::vector<int64_t> rs, rn;  // runs: first z, voxels
        for (int64_t c = 0; c < m && zlo + c <= zhi; ++c) {
            const int64_t n_all = (zhi - (zlo + c)) / m + 1;
            for (int64_t k0 = 0; k0 < n_all; k0 += run) {
                rs.push_back(zlo + c + k0 * m);
                rn.push_back(n_all - k0 < run ? n_all - k0 : run);
            }
        }
        std::vector<char> used(rs.size(), 0);
        for (size_t i = 0; i < rs.size(); ++i) {
            if (used[i]) continue;
            used[i] = 1;
            int mir = 0;
            if (zmir && rn[i] * ni * 2 <= max_mem) {  // the run whose voxels are this run's mirror images, if it is one
                const int64_t s2 = nz - 1 - (rs[i] + (rn[i] - 1) * m);
                for (size_t j = i + 1; j < rs.size(); ++j)
                    if (!used[j] && rs[j] == s2 && rn[j] == rn[i]) {
                        used[j] = 1;
                        mir = 1;
                        break;
                    }
            }
            add_class(cols[0] + rs[i] * nxy, m * nxy, (int)rn[i], cols, codes, ni, mir);
        }
    };
    for (int64_t ixy = 0; ixy < nxy; ++ixy) {
        int64_t zlo, zhi;
        zrange(ixy, &zlo, &zhi);
        if (!sym) {
            const int code0 = 0;
            add_columns(&ixy, &code0, 1, zlo, zhi);
            continue;
        }
        // only the orbit's first column (smallest index) builds its classes
        int64_t img[8];
        bool first = true;
        for (int c = 0; c < 8; ++c) {
            img[c] = column_image(c, nx, ixy);
            if (img[c] < ixy) first = false;
        }
        if (!first) continue;
        // images with the reference's z range join its classes; others stand alone
        int64_t cols[8];
        int codes[8], ni = 0;
        for (int c = 0; c < 8; ++c) {
            bool seen = false;
            for (int i = 0; i < c; ++i) seen = seen || img[i] == img[c];
            if (seen) continue;
            int64_t zl, zh;
            zrange(img[c], &zl, &zh);
            if (zl == zlo && zh == zhi) {
                cols[ni] = img[c];
                codes[ni++] = c;
            } else {
                const int code0 = 0;
                add_columns(&img[c], &code0, 1, zl, zh);
            }
        }
        add_columns(cols, codes, ni, zlo, zhi);
    }
    if (cur.nmem > 0) pl.batches.push_back(cur);
    return pl;
}

// The classes of a whole-image build plan, in order (cached in the handle):
// position k of the class order is voxel order.mem[k].x.
const ClassOrderCache& class_order(psf_handle* h, const Ws3& L) {
    ClassOrderCache& C = h->order;
    const int64_t key[3] = {L.bcsr, L.cap_recs, L.cap_uv_rings};
    if (C.valid && C.key[0] == key[0] && C.key[1] == key[1] && C.key[2] == key[2]) return C;
    const Plan3 all = plan3(h, L, 0, h->n_vox, L.bcsr, true, kShareCsr, true, kMaxMemProj);
    C.cls.clear();
    C.sym.clear();
    C.first.clear();
    C.mem.clear();
    C.mem.reserve(all.mem.size());
    for (const Batch3& b : all.batches)
        for (int c = 0; c < b.ncls; ++c) {
            const int4 cl = all.cls[b.cls0 + c];
            C.cls.push_back(cl);
            C.sym.push_back(all.sym[b.cls0 + c]);
            C.first.push_back((int64_t)C.mem.size());
            for (int i = 0; i < cl.z; ++i) {
                const int4 m = all.mem[b.mem0 + cl.y + i];
                C.mem.push_back(make_int2(m.x, m.y));
            }
        }
    for (int i = 0; i < 3; ++i) C.key[i] = key[i];
    C.valid = true;
    return C;
}

// Build plan for positions [vb, ve) of the class order: classes inside the
// range whole, and the members of a class the range cuts as classes of one
// voxel each.  CSR row = position - vb.
Plan3 plan3_order(psf_handle* h, const Ws3& L, int64_t vb, int64_t ve, int bmax) {
    const ClassOrderCache& C = class_order(h, L);
    const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
    const int64_t Nc = (int64_t)h->g.n_blocks * h->g.n_cryst_t;
    Plan3 pl;
    Batch3 cur = {0, 0, 0, 0, 0};
    int64_t cur_recs = 0;
    // a class of n members (voxel, shift) at positions p0.. (rows p - vb); nzc voxels per column
    auto push = [&](int v0, int n, int nzc, int sym, const int2* mm, int64_t p0) {
        const int64_t need = class_recs(L, NR, nzc), uv = Nc * (NR + nzc - 1);
        if (cur.nmem > 0 && (cur.nmem + n > bmax || cur.ncls + 1 > kClsBatch || cur_recs + need > L.cap_recs ||
                             cur.uv_slots + uv > L.cap_uv)) {
            pl.batches.push_back(cur);
            cur = {(int)pl.cls.size(), 0, (int)pl.mem.size(), 0, 0};
            cur_recs = 0;
        }
        pl.cls.push_back(make_int4(v0, cur.nmem, n, nzc - 1));
        pl.uvoff.push_back((int)cur.uv_slots);
        pl.sym.push_back(sym);
        for (int i = 0; i < n; ++i) pl.mem.push_back(make_int4(mm[i].x, mm[i].y, cur.ncls, (int)(p0 + i - vb)));
        cur.uv_slots += uv;
        cur.ncls += 1;
        cur.nmem += n;
        cur_recs += need;
    };
    // the first class that reaches past vb
    int64_t lo = 0, hi = (int64_t)C.first.size();
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (C.first[mid] + C.cls[mid].z <= vb) lo = mid + 1;
        else hi = mid;
    }
    for (int64_t c = lo; c < (int64_t)C.first.size() && C.first[c] < ve; ++c) {
        const int64_t f = C.first[c], n = C.cls[c].z;
        if (f >= vb && f + n <= ve) {
            push(C.cls[c].x, (int)n, C.sym[c] & 0xff, C.sym[c], &C.mem[f], f);
        } else {
            for (int64_t k = f > vb ? f : vb; k < f + n && k < ve; ++k) {
                const int2 one = make_int2(C.mem[k].x, 0);
                push(one.x, 1, 1, 1, &one, k);
            }
        }
    }
    if (cur.nmem > 0) pl.batches.push_back(cur);
    return pl;
}

struct PlanDev {
    const int4 *cls, *mem;
    const int *uvoff, *sym;
};

// copies the plan into the workspace; returns the device arrays
int upload_plan(const Plan3& pl, void* ws, const Ws3& L, hipStream_t s, PlanDev* d) {
    int4* c = at3<int4>(ws, L.plan);
    int4* mm = c + pl.cls.size();
    int* uo = (int*)(mm + pl.mem.size());
    int* sy = uo + pl.uvoff.size();
    if (!pl.cls.empty()) {
        HIP_TRY(hipMemcpyAsync(c, pl.cls.data(), sizeof(int4) * pl.cls.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(mm, pl.mem.data(), sizeof(int4) * pl.mem.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(uo, pl.uvoff.data(), sizeof(int) * pl.uvoff.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(sy, pl.sym.data(), sizeof(int) * pl.sym.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // the host vectors go out of scope after the call
    }
    d->cls = c;
    d->mem = mm;
    d->uvoff = uo;
    d->sym = sy;
    return PSF_OK;
}

void set_batch(Args3D& a, const Batch3& b, const PlanDev& d) {
    a.cls = d.cls + b.cls0;
    a.mem = d.mem + b.mem0;
    a.uvoff = d.uvoff + b.cls0;
    a.sym = d.sym + b.cls0;
    a.n_cls = b.ncls;
    a.n_mem = b.nmem;
}

// K1, K1b and K2a of one batch: line bundles, response rows, tile records
int batch_geometry(psf_handle* h, const Cyl3D& G, const Scratch3D& S, const Args3D& a, const Batch3& b,
                   int want_slots, hipStream_t s) {
    HIP_TRY(launch_cyl3d_transaxial(G, S, a, want_slots, s));
    if (want_slots) {
        HIP_TRY(launch_image_slots(G, S, a, s));
        HIP_TRY(launch_band_init(S, a, s));
    }
    HIP_TRY(launch_cyl3d_uvtab(G, S, a, b.uv_slots, s));
    ProfScope pg_(h, s, 1);
    HIP_TRY(launch_cyl3d_geom(G, S, a, s));
    return PSF_OK;
}

// the caller's stream s waits for the handle's second stream when the work
// that uses it ends, also on an early return
struct AuxJoin {
    bool on;
    hipStream_t s, aux;
    hipEvent_t ev;
    hipError_t now() {
        if (!on) return hipSuccess;
        on = false;
        hipError_t e = hipEventRecord(ev, aux);
        return e == hipSuccess ? hipStreamWaitEvent(s, ev, 0) : e;
    }
    ~AuxJoin() { (void)now(); }
};

// The forward projection runs each batch's geometry (K1, K1b, K2a) on the
// handle's second stream, one batch ahead of the contractions on the caller's
// stream (its atomics leave room for it: 4.49 s against 4.75 s on the whole
// image):
// odd batches take the second set of the geometry's outputs, a contraction
// waits for its batch's geometry, and the geometry of batch b waits for the
// caller's-stream work of batch b - 2, the last to read its set.
struct GeoPipe {
    psf_handle* h;
    hipStream_t s, g;  // the caller's stream; the geometry's
    bool two;
    int n = 0;         // batches issued
    AuxJoin join;
    GeoPipe(psf_handle* h_, const Ws3& L, hipStream_t s_, bool want)
        : h(h_), s(s_), g(s_), two(want && L.geo2 && aux_stream(h_)), join{false, s_, s_, nullptr} {
        if (two) {
            g = h->aux;
            join.on = true;
            join.aux = g;
            join.ev = h->aux_ev[3];
        }
    }
    hipError_t start() {  // the geometry stream after everything queued on s so far
        if (!two) return hipSuccess;
        hipError_t e = hipEventRecord(h->aux_ev[5], s);
        return e == hipSuccess ? hipStreamWaitEvent(g, h->aux_ev[5], 0) : e;
    }
    // before batch n's geometry, on g
    hipError_t before_geometry() {
        return two && n >= 2 ? hipStreamWaitEvent(g, h->aux_ev[1 + (n & 1)], 0) : hipSuccess;
    }
    // after batch n's geometry: s waits for it
    hipError_t after_geometry() {
        if (!two) return hipSuccess;
        hipError_t e = hipEventRecord(h->aux_ev[4], g);
        return e == hipSuccess ? hipStreamWaitEvent(s, h->aux_ev[4], 0) : e;
    }
    // after batch n's last kernel on s
    hipError_t after_batch() {
        hipError_t e = two ? hipEventRecord(h->aux_ev[1 + (n & 1)], s) : hipSuccess;
        ++n;
        return e;
    }
};

// y[batch][n_bins] = A x (accumulate: +=) over every voxel; the kernels add
// into a diagonal-layout copy (FP32 atomics), permuted into y at the end
int fwd3_all(psf_handle* h, const Cyl3D& G, const Scratch3D& S, const Ws3& L, const float* x, int batch, float* y,
             int accumulate, void* ws, hipStream_t s) {
    const Plan3 pl = plan3(h, L, 0, h->n_vox, L.bmax, true, L.bmax, true, kMaxMemProj);
    PlanDev pd;
    int st = upload_plan(pl, ws, L, s, &pd);
    if (st) return st;
    float* yd = at3<float>(ws, L.ydiag);
    GeoPipe gp(h, L, s, true);
    const Scratch3D S_odd = gp.two ? make_scratch_geo_odd(ws, L) : S;
    HIP_TRY(gp.start());
    for (int b0 = 0; b0 < batch; b0 += 8) {
        const int nb = batch - b0 < 8 ? batch - b0 : 8;
        HIP_TRY(launch_zero_f32(yd, (int64_t)nb * h->n_bins, s));
        for (const Batch3& bt : pl.batches) {
            const Scratch3D& Sb = (gp.n & 1) ? S_odd : S;
            Args3D a;
            memset(&a, 0, sizeof(a));
            set_batch(a, bt, pd);
            a.batch = nb;
            a.x = x + (int64_t)b0 * h->n_vox;
            a.y = yd;
            a.status = (int*)ws;
            a.tiles = (unsigned long long*)((char*)ws + kWsTileCounter);
            a.vtiles = (unsigned long long*)((char*)ws + kWsVoxTileCounter);
            HIP_TRY(gp.before_geometry());
            if ((st = batch_geometry(h, G, Sb, a, bt, 0, gp.g))) return st;
            HIP_TRY(gp.after_geometry());
            HIP_TRY(launch_gather_members(Sb, a, a.x, h->n_vox, s));
            {
                ProfScope pm_(h, s, 0);
                HIP_TRY(launch_cyl3d_mma(kModeFwd, G, Sb, a, s));
            }
            HIP_TRY(gp.after_batch());
        }
        HIP_TRY(launch_diag_perm(yd, y + (int64_t)b0 * h->n_bins, h->n_bins, G.NR, nb, 1, accumulate, s));
    }
    HIP_TRY(gp.join.now());
    return PSF_OK;
}

// x64[batch][n_voxels] += A^T y (y FP32 [batch][n_bins], or all ones); with
// g64, also d <y, A xt> / d table summed over the batch
int adj3_all(psf_handle* h, const Cyl3D& G, const Scratch3D& S, const Ws3& L, const float* y, int ones, int batch,
             double* x64, const float* xt, double* g64, void* ws, hipStream_t s) {
    const Plan3 pl = plan3(h, L, 0, h->n_vox, L.bmax, true, L.bmax, true, kMaxMemProj);
    PlanDev pd;
    int st = upload_plan(pl, ws, L, s, &pd);
    if (st) return st;
    float* yd = at3<float>(ws, L.ydiag);
    HIP_TRY(launch_zero_f64(S.xrep, (int64_t)kXRep * 8 * S.cap_mem, s));
    // the adjoint's gathers lose more to the geometry beside them than the
    // geometry saves (measured: 3.15 s against 2.92 s on the whole image)
    GeoPipe gp(h, L, s, false);
    const Scratch3D S_odd = gp.two ? make_scratch_geo_odd(ws, L) : S;
    HIP_TRY(gp.start());
    for (int b0 = 0; b0 < batch; b0 += 8) {
        const int nb = batch - b0 < 8 ? batch - b0 : 8;
        if (!ones) HIP_TRY(launch_diag_perm(y + (int64_t)b0 * h->n_bins, yd, h->n_bins, G.NR, nb, 0, 0, s));
        for (const Batch3& bt : pl.batches) {
            const Scratch3D& Sb = (gp.n & 1) ? S_odd : S;
            Args3D a;
            memset(&a, 0, sizeof(a));
            set_batch(a, bt, pd);
            a.batch = nb;
            a.yin = ones ? nullptr : yd;
            a.xt = xt ? xt + (int64_t)b0 * h->n_vox : nullptr;
            a.g64 = g64;
            a.g64_n = L.table_elems;
            a.ones = ones;
            a.x64 = x64 + (int64_t)b0 * h->n_vox;
            a.status = (int*)ws;
            a.tiles = (unsigned long long*)((char*)ws + kWsTileCounter);
            a.vtiles = (unsigned long long*)((char*)ws + kWsVoxTileCounter);
            HIP_TRY(gp.before_geometry());
            if ((st = batch_geometry(h, G, Sb, a, bt, 0, gp.g))) return st;
            HIP_TRY(gp.after_geometry());
            if (a.xt) HIP_TRY(launch_gather_members(Sb, a, a.xt, h->n_vox, s));
            {
                ProfScope pm_(h, s, 0);
                HIP_TRY(launch_cyl3d_mma(g64 ? kModeAdjGrad : kModeAdj, G, Sb, a, s));
            }
            HIP_TRY(launch_xrep_fold(Sb, a, h->n_vox, s));
            if (g64) HIP_TRY(launch_cyl3d_uvgrad(G, Sb, a, bt.uv_slots, s));
            HIP_TRY(gp.after_batch());
        }
    }
    HIP_TRY(gp.join.now());
    return PSF_OK;
}

}  // namespace

// rows of the build's range when its count phase stages them, else 0
static int64_t stage_rows(const psf_handle* h, const psf_opts* o) {
    if (!o || !(o->flags & PSF_OPT_STAGE_CSR)) return 0;
    const int64_t vb = o->vox_begin, ve = o->vox_end > 0 ? o->vox_end : h->n_vox;
    return ve > vb && vb >= 0 && ve <= h->n_vox ? ve - vb : 0;
}

size_t ws3_total(const psf_handle* h, const psf_table* t, int batch, int64_t n_events, const psf_opts* o) {
    return ws3_layout(h, t, batch, n_events, o && (o->flags & PSF_OPT_TABLE_GRAD), stage_rows(h, o),
                      o && (o->flags & PSF_OPT_DETERMINISTIC)).total;
}

int build_sysmat_3d(psf_handle* h, const psf_table* t, const psf_opts* o, void* ws, size_t ws_bytes, psf_csr* csr,
                    hipStream_t s) {
    int st = check3d(h, t, o);
    if (st) return st;
    const Ws3 L = ws3_layout(h, t, 1, 0, o->flags & PSF_OPT_TABLE_GRAD, stage_rows(h, o),
                             (o->flags & PSF_OPT_DETERMINISTIC) != 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    if (L.dense_slab * kShareCsr >= ((int64_t)1 << 31)) return PSF_EUNSUPPORTED;  // a group's cells index in 32 bits
    const int64_t vb = o->vox_begin, ve = o->vox_end > 0 ? o->vox_end : h->n_vox;
    if (vb < 0 || ve > h->n_vox || ve < vb) return PSF_EINVAL;
    if (!csr->row_ptr) return PSF_EINVAL;
    const Cyl3D G = make_cyl3d(h, t, o);
    const Scratch3D S = make_scratch(ws, L);
    const int phase_fill = csr->col != nullptr;
    const int stage = L.cap_stage > 0;
    csr->n_rows = ve - vb;
    const Plan3 pl = (o->flags & PSF_OPT_CLASS_ORDER) ? plan3_order(h, L, vb, ve, L.bcsr)
                                                       : plan3(h, L, vb, ve, L.bcsr, true, kShareCsr, true, kMaxMemProj);
    // what a count phase on this workspace staged for us (read before the header is cleared)
    int staged = 0;
    StageState ss;
    if (phase_fill && stage) {
        HIP_TRY(hipMemcpyAsync(&ss, (char*)ws + kWsStage, sizeof(ss), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (ss.magic == kStageMagic && ss.table == (const void*)t->data && ss.vb == vb && ss.ve == ve &&
            ss.threshold == o->threshold && ss.precision == o->precision && ss.n_rows == t->n_rows &&
            ss.n_sub == t->n_sub && ss.n_batches == (int32_t)pl.batches.size())
            staged = ss.batches < (int)pl.batches.size() ? ss.batches : (int)pl.batches.size();
    }
    if ((st = zero_header(ws, s))) return st;
    if (phase_fill) {
        if (!csr->val) return PSF_EINVAL;
        int64_t need = 0;
        HIP_TRY(hipMemcpyAsync(&need, csr->row_ptr + (ve - vb), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (csr->nnz < need) {
            csr->nnz = need;
            return PSF_ESIZE;
        }
    }
    // the accumulators start clean (cleared, or known clean from the last build
    // on this workspace); the compaction leaves them clean
    const bool use_dense = !(phase_fill && staged == (int)pl.batches.size());
    const int64_t dense_floats = L.bcsr * L.dense_slab * (L.det ? 2 : 1);  // FP32 cells, or 64-bit integer ones
    const unsigned long long dsig[3] = {(unsigned long long)(uintptr_t)h, (unsigned long long)L.dense,
                                        (unsigned long long)dense_floats};
    unsigned long long* dstate = (unsigned long long*)((char*)ws + kWsDense);
    if (use_dense)
        HIP_TRY(launch_dense_clear(S.dense, dense_floats, dstate, dsig, (o->flags & PSF_OPT_WS_CLEAN) != 0, s));
    // the count phase writes each row's count into row_ptr[row + 1]
    if (!phase_fill) HIP_TRY(launch_zero_f64((double*)csr->row_ptr, ve - vb + 1, s));
    PlanDev pd;
    if ((st = upload_plan(pl, ws, L, s, &pd))) return st;
    Args3D a0;
    memset(&a0, 0, sizeof(a0));
    a0.batch = 1;
    a0.threshold = o->threshold;
    a0.row_ptr = csr->row_ptr;
    a0.col = csr->col;
    a0.val = csr->val;
    a0.status = (int*)ws;
    a0.tiles = (unsigned long long*)((char*)ws + kWsTileCounter);
    a0.vtiles = (unsigned long long*)((char*)ws + kWsVoxTileCounter);
    if (stage) {
        a0.stage_cb = at3<int64_t>(ws, L.stage_cb);  // indexed by row (voxel - vox_begin) and chunk
        a0.stage_cn = at3<int>(ws, L.stage_cn);
        a0.stage_nch = at3<int>(ws, L.stage_nch);
        a0.stage_col = at3<int32_t>(ws, L.stage_col);
        a0.stage_val = at3<float>(ws, L.stage_val);
        a0.stage_cnt = at3<int>(ws, L.stage_cnt);
        a0.stage_rows = L.stage_rows;
        a0.stage_per_row = kStagePerVoxel;
        if (!phase_fill) HIP_TRY(launch_zero_f32((float*)a0.stage_cnt, stage_rows(h, o), s));
        StageState* dss = (StageState*)((char*)ws + kWsStage);
        a0.stage_full = &dss->full;
        a0.stage_batches = &dss->batches;
    }
    // fill phase: rows the count phase staged are copied
    if (staged > 0) {
        Args3D a = a0;
        set_batch(a, pl.batches[0], pd);
        const int n_rows = staged < (int)pl.batches.size() ? pl.batches[staged].mem0 : (int)pl.mem.size();
        HIP_TRY(launch_stage_copy(a, n_rows, L.max_chunks, s));
    }
    // A staged count phase runs three streams: the geometry of a batch on the
    // third one, during the previous batch's contraction; the contraction on
    // the caller's stream; the compaction on the second one.  Odd batches take
    // the second sets of the geometry's outputs and of the slots and bands.
    // Batch b's geometry waits for batch b - 2's compaction (the last user of
    // its sets); its contraction waits for its geometry and for batch b - 1's
    // compaction (the accumulators are shared); its compaction for its
    // contraction.
    const bool two = L.set2 && L.geo2 && stage && !phase_fill && aux_stream(h);
    const Scratch3D S_odd = two ? make_scratch_odd(ws, L) : S;
    hipStream_t sc = two ? h->aux : s;   // the compaction's stream
    hipStream_t sg = two ? h->aux2 : s;  // the geometry's stream
    // the caller's stream waits for the other two when the loop ends, also on
    // an early return
    struct Join {
        bool on;
        hipStream_t s, sc, sg;
        hipEvent_t ev;
        hipError_t now() {
            if (!on) return hipSuccess;
            on = false;
            hipError_t e = hipEventRecord(ev, sc);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
            if (e == hipSuccess) e = hipEventRecord(ev, sg);
            return e == hipSuccess ? hipStreamWaitEvent(s, ev, 0) : e;
        }
        ~Join() { (void)now(); }
    } join{two, s, sc, sg, two ? h->aux_ev[3] : nullptr};
    if (two) {  // the geometry stream after everything queued on s so far
        HIP_TRY(hipEventRecord(h->aux_ev[5], s));
        HIP_TRY(hipStreamWaitEvent(sg, h->aux_ev[5], 0));
    }
    for (int bi = staged; bi < (int)pl.batches.size(); ++bi) {
        const Batch3& bt = pl.batches[bi];
        Args3D a = a0;
        set_batch(a, bt, pd);
        a.stage = stage && !phase_fill;
        const Scratch3D& Sb = (bi & 1) ? S_odd : S;
        if (two && bi >= staged + 2) HIP_TRY(hipStreamWaitEvent(sg, h->aux_ev[1 + (bi & 1)], 0));
        if ((st = batch_geometry(h, G, Sb, a, bt, 1, sg))) return st;
        if (two) {
            HIP_TRY(hipEventRecord(h->aux_ev[4], sg));
            HIP_TRY(hipStreamWaitEvent(s, h->aux_ev[4], 0));
            if (bi > staged) HIP_TRY(hipStreamWaitEvent(s, h->aux_ev[1 + ((bi - 1) & 1)], 0));
        }
        {
            ProfScope pm_(h, s, 0);
            HIP_TRY(launch_cyl3d_mma(kModeCount, G, Sb, a, s));
        }
        if (two) {
            HIP_TRY(hipEventRecord(h->aux_ev[0], s));
            HIP_TRY(hipStreamWaitEvent(sc, h->aux_ev[0], 0));
        }
        HIP_TRY(launch_cyl3d_compact(phase_fill ? kModeFill : kModeCount, G, Sb, a, sc));
        if (two) HIP_TRY(hipEventRecord(h->aux_ev[1 + (bi & 1)], sc));
    }
    HIP_TRY(join.now());
    if (use_dense) HIP_TRY(launch_dense_mark(dstate, dsig, 1, s));  // every batch compacted: clear again
    if (!phase_fill) {
        HIP_TRY(launch_scan_rowptr(csr->row_ptr, ve - vb, s));
        int64_t nnz = 0;
        HIP_TRY(hipMemcpyAsync(&nnz, csr->row_ptr + (ve - vb), sizeof(int64_t), hipMemcpyDeviceToHost, s));
        if (stage) {  // sign what was staged for the fill phase
            StageState host;
            memset(&host, 0, sizeof(host));
            host.magic = kStageMagic;
            host.table = (const void*)t->data;
            host.vb = vb;
            host.ve = ve;
            host.threshold = o->threshold;
            host.precision = o->precision;
            host.n_rows = t->n_rows;
            host.n_sub = t->n_sub;
            host.n_batches = (int32_t)pl.batches.size();
            const size_t head = offsetof(StageState, magic);
            HIP_TRY(hipMemcpyAsync((char*)ws + kWsStage + head, (const char*)&host + head, sizeof(host) - head,
                                   hipMemcpyHostToDevice, s));
        }
        st = read_status(ws, s);
        csr->nnz = nnz;
        return st;
    }
    return read_status(ws, s);
}

int project_fwd_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const float* x, int batch,
                   const int32_t* events, int64_t n_events, float* y, void* ws, size_t ws_bytes, hipStream_t s) {
    int st = check3d(h, t, o);
    if (st) return st;
    const Ws3 L = ws3_layout(h, t, batch, events ? n_events : 0, 0, 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const Cyl3D G = make_cyl3d(h, t, o);
    const Scratch3D S = make_scratch(ws, L);
    if ((st = zero_header(ws, s))) return st;
    if (events) {
        float* y32 = at3<float>(ws, L.y32);
        if ((st = fwd3_all(h, G, S, L, x, batch, y32, 0, ws, s))) return st;
        const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
        HIP_TRY(launch_lm_gather(nullptr, y32, h->n_bins, events, n_events, batch, G.Nc, NR, y, o->accumulate,
                                 (int*)ws, s));
        return read_status(ws, s);
    }
    if ((st = fwd3_all(h, G, S, L, x, batch, y, o->accumulate, ws, s))) return st;
    return read_status(ws, s);  // blocks: a capacity or range flag means y is incomplete
}

int project_adj_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const float* y, int ones, int batch,
                   const int32_t* events, int64_t n_events, float* x, const float* xt, float* grad, void* ws,
                   size_t ws_bytes, hipStream_t s) {
    int st = check3d(h, t, o);
    if (st) return st;
    const Ws3 L = ws3_layout(h, t, batch, events ? n_events : 0, grad != nullptr, 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const Cyl3D G = make_cyl3d(h, t, o);
    const Scratch3D S = make_scratch(ws, L);
    if ((st = zero_header(ws, s))) return st;
    const float* ybins = y;
    const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
    if (events) {
        double* h64 = at3<double>(ws, L.h64);
        float* h32 = at3<float>(ws, L.h32);
        const int64_t n = (int64_t)batch * h->n_bins;
        HIP_TRY(launch_zero_f64(h64, n, s));
        HIP_TRY(launch_lm_scatter(y, n_events, events, batch, G.Nc, NR, h->n_bins, h64, (int*)ws, s));
        HIP_TRY(launch_finalize(h64, h32, n, 0, s));
        ybins = h32;
    }
    double* x64 = at3<double>(ws, L.x64);
    HIP_TRY(launch_zero_f64(x64, (int64_t)batch * h->n_vox, s));
    double* g64 = grad ? at3<double>(ws, L.g64) : nullptr;
    if (grad) {
        HIP_TRY(launch_zero_f64(g64, kGradRep * L.table_elems, s));
        HIP_TRY(launch_zero_f64(S.uvgrad, 400 * L.cap_uv, s));
    }
    if ((st = adj3_all(h, G, S, L, ybins, ones, batch, x64, xt, g64, ws, s))) return st;
    HIP_TRY(launch_finalize(x64, x, (int64_t)batch * h->n_vox, ones ? 0 : o->accumulate, s));
    if (grad) {
        HIP_TRY(launch_sum_copies(g64, L.table_elems, kGradRep, s));  // the copies into the first
        HIP_TRY(launch_finalize(g64, grad, L.table_elems, 1, s));
    }
    return read_status(ws, s);  // blocks: a capacity or range flag means x is incomplete
}

int lm_osem_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const int32_t* events, int64_t n_events,
               float randoms, const float* sens, int n_subsets, const float* x_in, float* x_out, void* ws,
               size_t ws_bytes, hipStream_t s) {
    int st = check3d(h, t, o);
    if (st) return st;
    const Ws3 L = ws3_layout(h, t, 1, n_events, 0, 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const Cyl3D G = make_cyl3d(h, t, o);
    const Scratch3D S = make_scratch(ws, L);
    if ((st = zero_header(ws, s))) return st;
    const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
    float* y32 = at3<float>(ws, L.y32);
    double* h64 = at3<double>(ws, L.h64);
    float* h32 = at3<float>(ws, L.h32);
    float* back = at3<float>(ws, L.back);
    double* x64 = at3<double>(ws, L.x64);
    // q_e = a_e^T x + r  ->  h[bin] += 1 / q_e  ->  back = A^T h  ->  update
    if ((st = fwd3_all(h, G, S, L, x_in, 1, y32, 0, ws, s))) return st;
    HIP_TRY(launch_zero_f64(h64, h->n_bins, s));
    HIP_TRY(launch_lm_ratio(nullptr, y32, events, n_events, G.Nc, NR, (double)randoms, h64, (int*)ws, s));
    HIP_TRY(launch_finalize(h64, h32, h->n_bins, 0, s));
    HIP_TRY(launch_zero_f64(x64, h->n_vox, s));
    if ((st = adj3_all(h, G, S, L, h32, 0, 1, x64, nullptr, nullptr, ws, s))) return st;
    HIP_TRY(launch_finalize(x64, back, h->n_vox, 0, s));
    HIP_TRY(launch_lm_update(x_in, back, sens, n_subsets, h->n_vox, x_out, s));
    return read_status(ws, s);
}

int voxel_order_3d(psf_handle* h, int64_t* order) {
    // the plan's limits do not depend on the table beyond its presence
    psf_table t;
    memset(&t, 0, sizeof(t));
    t.n_rows = 1;
    t.n_sub = 4;
    const Ws3 L = ws3_layout(h, &t, 1, 0, 0, 0);
    const ClassOrderCache& C = class_order(h, L);
    if ((int64_t)C.mem.size() != h->n_vox) return PSF_EINVAL;
    for (int64_t k = 0; k < h->n_vox; ++k) order[k] = C.mem[k].x;
    return PSF_OK;
}

int osem_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const float* y, int n_subsets, int subset,
            const float* sens, const float* x_in, float* x_out, void* ws, size_t ws_bytes, hipStream_t s) {
    int st = check3d(h, t, o);
    if (st) return st;
    const Ws3 L = ws3_layout(h, t, 1, 1, 0, 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const Cyl3D G = make_cyl3d(h, t, o);
    const Scratch3D S = make_scratch(ws, L);
    if ((st = zero_header(ws, s))) return st;
    const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
    float* yh = at3<float>(ws, L.y32);
    float* r = at3<float>(ws, L.h32);
    float* back = at3<float>(ws, L.back);
    double* x64 = at3<double>(ws, L.x64);
    // yhat = A x -> r = m_k y / yhat -> back = A^T r -> update
    if ((st = fwd3_all(h, G, S, L, x_in, 1, yh, 0, ws, s))) return st;
    HIP_TRY(launch_osem_ratio(nullptr, yh, y, h->n_bins, G.Nc, NR, n_subsets, subset, r, s));
    HIP_TRY(launch_zero_f64(x64, h->n_vox, s));
    if ((st = adj3_all(h, G, S, L, r, 0, 1, x64, nullptr, nullptr, ws, s))) return st;
    HIP_TRY(launch_finalize(x64, back, h->n_vox, 0, s));
    HIP_TRY(launch_osem_update(x_in, back, sens, h->n_vox, x_out, s));
    return read_status(ws, s);
}

int subset_sensitivity_3d(psf_handle* h, const psf_table* t, const psf_opts* o, int n_subsets, int subset, float* s_dev,
                          void* ws, size_t ws_bytes, hipStream_t s) {
    int st = check3d(h, t, o);
    if (st) return st;
    const Ws3 L = ws3_layout(h, t, 1, 1, 0, 0);
    if (ws_bytes < L.total) return PSF_ESIZE;
    const Cyl3D G = make_cyl3d(h, t, o);
    const Scratch3D S = make_scratch(ws, L);
    if ((st = zero_header(ws, s))) return st;
    const int64_t NR = (int64_t)h->g.n_cryst_z * h->g.n_block_rings;
    float* m = at3<float>(ws, L.h32);
    double* x64 = at3<double>(ws, L.x64);
    HIP_TRY(launch_subset_mask(h->n_bins, G.Nc, NR, n_subsets, subset, m, s));
    HIP_TRY(launch_zero_f64(x64, h->n_vox, s));
    if ((st = adj3_all(h, G, S, L, m, 0, 1, x64, nullptr, nullptr, ws, s))) return st;
    HIP_TRY(launch_finalize(x64, s_dev, h->n_vox, 0, s));
    return read_status(ws, s);
}
