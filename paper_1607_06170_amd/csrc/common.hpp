// Internal declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psf.h"

namespace psf {

constexpr double kPi = 3.14159265358979323846;
// Direction overlaps at or below this many radians are empty: a set of lines
// of zero measure (it guards exact antipodal coincidences against rounding).
constexpr double kEpsOverlap = 1e-12;
constexpr int kNb = 5;  // neighbour crystals per axis: offsets -2..2
constexpr int kTopNMax = 16;  // largest top_n (bins kept per voxel and sinogram view)

// status bits kept in the first word of the workspace
constexpr int kStatRange = 1;     // an incidence angle beyond the last table row was used
constexpr int kStatOverflow = 2;  // fill phase wanted more entries than allotted
constexpr int kStatGeom = 4;
constexpr int kStatEventBad = 8;  // an event names a crystal out of range, or the same crystal twice

// Workspace header: status word at byte 0, tile counter (uint64) at byte 64,
// voxel-tile counter (uint64: tiles times the voxels they serve) at byte 72,
// padding to 256 bytes.
constexpr size_t kWsHeader = 256;
constexpr size_t kWsTileCounter = 64;
constexpr size_t kWsVoxTileCounter = 72;
// Bytes 128..223: the matrix build's staging state (full flag, staged batches,
// then the signature of the count phase that filled it).
constexpr size_t kWsStage = 128;
// Bytes 224..255 survive the header clear of every call: the handle and the
// accumulator layout of the last build that completed (left its accumulators
// clear), or zeros.
constexpr size_t kWsDense = 224;

// Everything a 2D-ring kernel needs, passed by value.
struct Ring2D {
    int R, nc, P, Nc, nseg, n_rows, nx, ny;
    int64_t nbins, nvox;
    double lam, half_w, rf, sigma, step_deg, two_pi_R;
    double dx, dy, cx, cy;
    const double* frames;  // [R][2]: cos, sin of the block's outward normal
    const float* table;    // [n_rows][P][5]
    int precision;
    int homog_k;           // 0: the k -> infinity sweep; k > 0: k lines at theta_i = pi i / k (Eq.11)
    int top_n;             // 0: every bin; n > 0: each sinogram view keeps its n largest bins
    int det;               // matrix build: integer sums of the tile entries (fix62)
};

// Everything a 3D-scanner kernel needs, passed by value.  Crystal (g, r):
// transaxial index g = b * nc + c, ring r; axial sub-position q = r * P + pz.
struct Cyl3D {
    int R, nc, P, Nc, nseg, n_rows, NR, nx, ny, nz;
    int64_t nvox, ntbins, nbins;
    double lam, half_w, rf, sigma, step_deg, two_pi_R, sin_two_pi_R, lz, z0;
    double dx, dy, dz, cx, cy, cz;
    const double* frames;
    const float* table;  // [n_rows][n_rows][P][P][5][5]
    int precision;
};

// Per-voxel scratch of the 3D kernels (a batch of B voxels at a time).
struct Scratch3D {
    int cap_samples, cap_pairs, cap_slots;
    // per class of the batch (index cb)
    int* n_samples;    // [B_cls]
    int* n_pairs;      // [B_cls]
    int* n_slots;      // [B_cls]
    int* sidx;         // [B_cls][cap_samples]  s1 << 16 | s2
    double* sth;       // [B_cls][cap_samples][2]  direction interval of the sample
    int4* pairs;       // [B_cls][cap_pairs]  g1, g2, first sample, sample count
    // matrix build, per column (index: the member index of its first voxel)
    int* slotmap;      // [B_mem][ntbins]  transaxial bin -> slot (-1: none), reference columns
    int* slot_tbin;    // [B_mem][cap_slots]  the column's bins in ascending order
    int* slot_order;   // [B_mem][cap_slots]  their reference slots (bit 30: photons swapped)
    // matrix build: FP32 sums of the FP32 tile entries (deterministic builds:
    // exact integer sums in units of 2^-62, see fix62).  A column of n members
    // (s_max = n - 1) from batch member mi0 on holds [slot][i][j][s] from slab
    // mi0: member s's ring pair (r_i, r_j) at i = r_i - s + s_max, j = r_j - s +
    // s_max (both < NR + s_max), so an entry's members lie side by side
    float* dense;      // [B_mem][dense_slab] (deterministic builds: 64-bit integer cells, fix62)
    int64_t dense_slab;
    int det;
    int* chunk_counts; // [B_mem][max_chunks]  kept entries per compaction chunk
    int64_t max_chunks;
    float* recs;       // [cap_recs][kRecFloats]  tile records (header, sample blocks of W)
    unsigned int* rec_count;  // [0] records appended, [1] the geometry's next work unit (both reset by K1)
    int64_t cap_recs;
    // response rows of every (crystal g, relative ring r) of each class: slot
    // uvoff[class] + g * (NR + s_max) + (r + s_max) holds P^2 rows of 25
    float* uvtab;      // [cap_uv][16][25]
    int* uvmask;       // [cap_uv]  rows whose angle row was clamped (bit per row)
    int64_t cap_uv;
    // adjoint sums of the batch's members, in kXRep copies taken by wavefront
    // index so that concurrent records do not queue on one address
    double* xrep;      // [kXRep][B_mem][8]
    int cap_mem;
    // table gradient: d loss / d response-row entries of the batch's slots
    // (layout of uvtab), folded into the table entries after each batch
    double* uvgrad;    // [cap_uv][16][25], or null
    float* xm;         // [B_mem][8]  the batch members' image values (forward input, or the gradient's image)
    // matrix build: for each class (at its first member), reference slot and ring
    // r_i relative to the reference voxel (offset s_max + 2), the range of r_j
    // its tiles touched; bandc the same by column: for each r_j, the r_i range
    int2* band;        // [B_mem][cap_slots][band_rows]
    int2* bandc;       // [B_mem][cap_slots][band_rows]
    int band_rows;
};
constexpr int kXRep = 64;
// copies of the FP64 table-gradient accumulator, taken by workgroup: many response
// rows feed the same table entries, and one copy would serialise their atomics
constexpr int kGradRep = 32;

// tile record (ints and floats in one array):
//   [0] g1  [1] g2  [2] (r1 + 512) | (r2 + 512) << 10 | class << 20  [3] n samples
//   [4] row-table slot of U (g1, r1)  [5] of V (g2, r2)
//   [6] the class's first member | member count << 16
//   [7] the class's voxels per column | image codes << 8 (3 bits per column)
//   [8 + k]        pt1 | pt2 << 8 of sample k (the transaxial sub-segments of the bundle)
//   [24 + 16k + q] W of sample k between axial sub-positions pz1 = q / P and pz2 = q % P
// rings are relative to the class's reference member
constexpr int kRecPts = 8;
constexpr int kRecHead = 24;
constexpr int kRecFloats = kRecHead + 16 * 16;

// Voxels are processed in classes: voxels of one z-column whose z differ by a
// whole number of ring pitches see the scanner identically up to a shift of
// whole rings, so the class computes its line bundles, weights and response
// rows once, for the ring offsets of its reference member (shift 0), and each
// member takes the tiles shifted by its own ring shift.
struct Args3D {
    const int4* cls;    // [n_cls]: reference voxel, first member, member count, largest shift
    const int4* mem;    // [n_mem]: voxel, ring shift, class, CSR row
    const int* uvoff;   // [n_cls]: first response-row slot of the class
    const int* sym;     // [n_cls]: voxels per column | image codes << 8 (3 bits per column of the class)
    int n_cls;          // classes in this batch
    int n_mem;          // members (voxels) in this batch
    int batch;
    double threshold;
    const float* x;     // [batch][nvox]  forward input
    float* y;           // [batch][nbins] forward output (FP32 atomics), diagonal ring-pair layout
    const float* yin;   // [batch][nbins] adjoint input, diagonal ring-pair layout
    double* x64;        // [batch][nvox]  adjoint accumulator
    int64_t* row_ptr;
    int32_t* col;
    float* val;
    int* status;
    int ones;           // adjoint with y == 1 (sensitivity)
    const float* xt;    // [batch][nvox] image of the table gradient (adjoint with gradient)
    double* g64;        // table-gradient accumulator [kGradRep][table entries]
    int64_t g64_n;      // table entries (the stride of g64's copies)
    // matrix build, count phase with staging: rows compacted into the stage, in
    // pieces of one compaction chunk each
    int stage;
    int64_t* stage_cb;          // [rows of the range][max_chunks]  stage offset of a chunk's entries, -1 if none
    int* stage_cn;              // [rows of the range][max_chunks]  its kept entries
    int* stage_nch;             // [rows of the range]  the row's chunks
    int32_t* stage_col;         // [cap_stage]
    float* stage_val;           // [cap_stage]
    int64_t stage_rows;             // rows of the range with a stage region (the first ones)
    int64_t stage_per_row;          // entries of a row's region
    int* stage_cnt;                 // [stage_rows]  entries a row's chunks reserved
    int* stage_full;                // workspace header: a row did not fit (sticky)
    int* stage_batches;             // workspace header: batches fully staged
    unsigned long long* tiles;   // count of tiles contracted (workspace header)
    unsigned long long* vtiles;  // count of (voxel, tile) pairs emitted (workspace header)
};

// Device view of the handle (host struct defined in api.cpp).
struct HandleView {
    psf_geometry g;
    psf_image im;
    int mode3d;
    int64_t n_crystals, n_bins, n_vox;
    double sigma;
    const double* frames;
};

// Per-call arguments of the voxel-stationary 2D kernels.
struct VoxArgs2D {
    int64_t vox_begin, n_vox_range;
    int batch;
    double threshold;
    const float* x;       // [batch][nvox]       fwd input / table-gradient image
    const float* y;       // [batch][nbins]      adj input
    double* y64;          // [batch][nbins]      fwd FP64 accumulator
    float* xout;          // [batch][nvox]       adj output
    int64_t* row_ptr;     // CSR row pointers (count: slot v+1 gets the count)
    int32_t* col;
    float* val;
    double* grad64;       // table-gradient FP64 accumulator (table size)
    int* status;
    int accumulate;
    int ones;             // adj with y == 1 (sensitivity)
};

// host launchers (ring2d.hip / table.hip)
hipError_t launch_table_2d(const psf_geometry& g, int n_rows, int P, double step_deg, float* out,
                           hipStream_t st);
hipError_t launch_voxel2d(int mode, const Ring2D& G, const VoxArgs2D& a, hipStream_t st);
hipError_t launch_scan_rowptr(int64_t* row_ptr, int64_t n, hipStream_t st);
hipError_t launch_finalize(const double* src, float* dst, int64_t n, int accumulate, hipStream_t st);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st);
size_t voxel2d_smem_bytes(const Ring2D& G, int mode);
hipError_t launch_lm_gather(const double* y64, const float* y32, int64_t nbins, const int32_t* ev, int64_t ne,
                            int batch, int64_t Nc, int64_t NR, float* out, int accumulate, int* status,
                            hipStream_t st);
hipError_t launch_lm_scatter(const float* h, int64_t ne, const int32_t* ev, int batch, int64_t Nc, int64_t NR,
                             int64_t nbins, double* hist, int* status, hipStream_t st);
hipError_t launch_lm_ratio(const double* y64, const float* y32, const int32_t* ev, int64_t ne, int64_t Nc, int64_t NR,
                           double randoms, double* hist, int* status, hipStream_t st);
hipError_t launch_lm_update(const float* x_in, const float* back, const float* sens, int n_subsets, int64_t nvox,
                            float* x_out, hipStream_t st);

hipError_t launch_osem_ratio(const double* yh64, const float* yh32, const float* y, int64_t nbins, int64_t Nc,
                             int64_t NR, int n_subsets, int subset, float* r, hipStream_t st);
hipError_t launch_subset_mask(int64_t nbins, int64_t Nc, int64_t NR, int n_subsets, int subset, float* m,
                              hipStream_t st);
hipError_t launch_osem_update(const float* x_in, const float* back, const float* sens, int64_t nvox, float* x_out,
                              hipStream_t st);

enum { kModeCount = 0, kModeFill = 1, kModeFwd = 2, kModeAdj = 3, kModeAdjGrad = 4 };

// 3D launchers (cyl3d.hip, table3d.hip)
hipError_t launch_table_3d(const psf_geometry& g, int n_rows, int P, double step_deg, float* out, hipStream_t st);
hipError_t launch_table_mc(const psf_geometry& g, int mode3d, int n_rows, int P, double step_deg, long long photons,
                           unsigned long long seed, int scatter, float* table, long long* counts, hipStream_t st);
void table_2d_host(const psf_geometry& g, int n_rows, int P, double step_deg, double* out);
void table_3d_host(const psf_geometry& g, int n_rows, int P, double step_deg, double* out);
hipError_t launch_cyl3d_transaxial(const Cyl3D& G, const Scratch3D& S, const Args3D& a, int want_slots,
                                   hipStream_t st);
hipError_t launch_cyl3d_uvtab(const Cyl3D& G, const Scratch3D& S, const Args3D& a, int64_t n_slots, hipStream_t st);
hipError_t launch_cyl3d_uvgrad(const Cyl3D& G, const Scratch3D& S, const Args3D& a, int64_t n_slots, hipStream_t st);
hipError_t launch_sum_copies(double* p, int64_t n, int reps, hipStream_t st);
hipError_t launch_cyl3d_geom(const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st);
hipError_t launch_cyl3d_mma(int mode, const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st);
hipError_t launch_cyl3d_compact(int mode, const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st);
hipError_t launch_stage_copy(const Args3D& a, int n_rows, int64_t max_chunks, hipStream_t st);
hipError_t launch_band_init(const Scratch3D& S, const Args3D& a, hipStream_t st);
hipError_t launch_image_slots(const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st);
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st);
// the build's accumulators: cleared unless `trust` and the header words at
// `state` (magic, handle, offset, size) match `sig`; then marked in use
hipError_t launch_dense_clear(float* p, int64_t n, unsigned long long* state, const unsigned long long* sig, bool trust,
                              hipStream_t st);
// marks the accumulators clean (`clean`, with the signature) or in use
hipError_t launch_dense_mark(unsigned long long* state, const unsigned long long* sig, int clean, hipStream_t st);
hipError_t launch_xrep_fold(const Scratch3D& S, const Args3D& a, int64_t nvox, hipStream_t st);
hipError_t launch_gather_members(const Scratch3D& S, const Args3D& a, const float* x, int64_t nvox, hipStream_t st);
hipError_t launch_diag_perm(const float* src, float* dst, int64_t nbins, int NR, int nb, int to_user, int accumulate,
                            hipStream_t st);
int64_t cyl3d_max_chunks(int cap_slots, int NR);
constexpr int kStatScratch = 16;  // a per-voxel scratch capacity was exceeded

// Deterministic matrix builds: a tile entry t in [0, 1) is rounded once to the
// nearest multiple of 2^-62 and summed as a 64-bit integer.  Integer sums are
// exact, so a bin's sum does not depend on the order in which its entries
// arrive; an element (below 2) is read back as q * 2^-62, rounded to FP64.
__device__ __forceinline__ bool fix62_ok(float t) { return t >= 0.0f && t < 1.0f; }
__device__ __forceinline__ unsigned long long fix62(float t) {
    return fix62_ok(t) ? (unsigned long long)__builtin_rint((double)t * 0x1p62) : 0ull;
}
__host__ __device__ inline double unfix62(unsigned long long q) { return (double)q * 0x1p-62; }

}  // namespace psf
