/*
 * psf.h -- C ABI of the P-SPIR PSF system-matrix library for AMD MI355X (gfx950).
 *
 * Method: Sun et al., "Fast and accurate generation method of PSF-based system
 * matrix for PET reconstruction", Chinese Physics C (2016), arXiv 1607.06170.
 *
 * Conventions shared by every entry point
 *   - Return value: PSF_OK (0) on success, a negative PSF_E* code otherwise.
 *     No exception ever crosses this interface.
 *   - Pointers named *_dev, and the data fields of psf_table / psf_csr, are
 *     device (HBM) pointers; everything else is host memory.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = the default stream)
 *     and runs asynchronously unless the description says the call blocks.
 *     Some 3D calls (the count phase of a staged build, the forward
 *     projection and what runs it) also use a second and a third stream that
 *     the library keeps for each device (shared by the process's handles,
 *     created on first use, at the default priority), ordered against
 *     `stream` by the handle's events both ways: `stream` waits for them
 *     before the call returns, on error returns too.
 *     Calls on one handle are not thread-safe.
 *   - The caller owns every buffer passed in.  The library never frees caller
 *     memory; its own device state lives in the handle (geometry constants)
 *     and in the caller-provided workspace (sized by psf_workspace_size).
 *   - Outputs are overwritten unless psf_opts.accumulate is 1.
 *
 * Geometry (paper Sec 2.1.2 symbols in brackets): n_blocks flat blocks [R]
 * per ring; block b has outward normal at angle phi0 + 2 pi b / R and its front
 * face at distance radius_face from the axis; along the face, n_cryst_t
 * crystals of width pitch_t [lambda]; crystal depth `depth`; attenuation `mu`.
 * Global transaxial crystal index g = b * n_cryst_t + c increases
 * counter-clockwise.  3D scanners stack n_block_rings rings of blocks of
 * n_cryst_z crystals axially (pitch_z), with crystal id = ring * N_c + g.
 *
 * Image: voxel (ix, iy, iz) has centre ((ix - (nx-1)/2) dx + cx, ...), linear
 * index (iz * ny + iy) * nx + ix.
 *
 * Bins: a bin is an unordered crystal pair (i < j), numbered
 *   bin(i, j) = i * N - i (i + 1) / 2 + (j - i - 1),   N crystals in total.
 */
#ifndef PSF_H
#define PSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PSF_OK = 0,
    PSF_EINVAL = -1,       /* a NULL pointer, a negative size or a bad option */
    PSF_EGEOM = -2,        /* inconsistent geometry (e.g. a voxel outside the ring) */
    PSF_ERANGE = -3,       /* an incidence angle beyond the table's last row, a table shape mismatch, or
                            * (PSF_OPT_DETERMINISTIC) a tile entry outside [0, 1) */
    PSF_ESIZE = -4,        /* a buffer is too small; the required size is written back */
    PSF_EHIP = -5,         /* a HIP runtime error (see psf_last_hip_error) */
    PSF_EOVERFLOW = -6,    /* fill phase produced more entries than the count phase allotted */
    PSF_EUNSUPPORTED = -7, /* geometry or option combination this library does not handle */
    PSF_ECAPACITY = -8     /* 3D: a voxel's lines exceeded a fixed scratch capacity (more than 4096
                            * sub-segment pairs or 1024 crystal pairs seen from one voxel, more than
                            * 16 sub-segment pairs per crystal pair, more than 4096 transaxial bins
                            * under one image column, or a batch's tile records beyond the record
                            * buffer); the output is incomplete and must not be used */
};

/* precision of the tile contraction T = U^T W V (paper Sec 2.2-2.3, Eq.10, 12) */
enum {
    PSF_FP32 = 0,   /* FP32 products, FP64 bin accumulation */
    PSF_BF16 = 1,   /* X = W V in FP32; U and X rounded to BF16 for T = U^T X, FP32 accumulation */
    PSF_BF16X2 = 2  /* as PSF_BF16 with a hi/lo BF16 split of U and X (three products) */
};

typedef struct {
    int32_t n_blocks;       /* R: blocks per ring (Eq.2) */
    int32_t n_cryst_t;      /* crystals per block along the face (transaxial) */
    int32_t n_cryst_z;      /* crystals per block axially (1 for a 2D ring) */
    int32_t n_block_rings;  /* block rings along z (1 for a 2D ring) */
    double pitch_t;         /* lambda: crystal width transaxially, mm (Eq.5) */
    double pitch_z;         /* crystal width axially, mm */
    double depth;           /* crystal length, mm */
    double radius_face;     /* axis-to-front-face distance, mm */
    double gap_z;           /* axial gap between block rings, mm (must be 0) */
    double mu;              /* linear attenuation, 1/mm (table builder only) */
    double phi0;            /* angle of block 0's outward normal, rad */
} psf_geometry;

typedef struct {
    int32_t nx, ny, nz, pad;
    double dx, dy, dz;      /* voxel size, mm */
    double cx, cy, cz;      /* image centre, mm */
} psf_image;

/* Response table (paper Sec 2.1.1, Eq.1, 6-7): absolute first-interaction
 * probability for a photon entering sub-position p of a crystal at incidence
 * angle row * step_deg, tilted towards larger crystal offsets; entry a+2 is
 * the crystal at offset a in -2..2.
 *   2D: data[n_rows][n_sub][5]
 *   3D: data[n_rows][n_rows][n_sub][n_sub][5][5]  (transaxial angle row,
 *       axial angle row, transaxial sub-position, axial sub-position,
 *       transaxial offset, axial offset) */
typedef struct {
    int32_t n_rows;
    int32_t n_sub;
    double step_deg;
    const float* data;      /* device */
} psf_table;

typedef struct {
    int32_t precision;      /* PSF_FP32 / PSF_BF16 / PSF_BF16X2 */
    int32_t homog_k;        /* 0: homogenization in the k -> infinity limit; k > 0: Eq.11 with k lines */
    double threshold;       /* build_psf_sysmat keeps entries with A >= threshold (and A > 0) */
    int64_t vox_begin;      /* voxel range of build_psf_sysmat: [vox_begin, vox_end) */
    int64_t vox_end;        /* vox_end <= 0 means all voxels */
    int32_t accumulate;     /* 1: add into the output instead of overwriting */
    int32_t flags;          /* PSF_OPT_* bits */
    int32_t top_n;          /* 0: every bin; n > 0 (2D, n <= 16): the matrix keeps, for each voxel and
                             * each sinogram angle, only its n largest bins (paper Sec 3.3, Table 3).
                             * The angle of crystal pair (i, j) of an N-crystal ring is view
                             * ((i + j) mod N) / 2 of N / 2: pairs of one view are parallel chords
                             * of a circular ring, the two parities interleaved (Table 1: 192 angles
                             * for 384 crystals per ring).  Ties keep the lower bin.  Applies to every
                             * 2D call (matrix, projections, sensitivity, list mode); not with the
                             * table gradient, nor in 3D (PSF_EUNSUPPORTED). */
    int32_t reserved;       /* 0 */
} psf_opts;

/* psf_opts.flags: project_adj will be asked for the table gradient (3D: the
 * workspace then holds its per-batch accumulator). */
#define PSF_OPT_TABLE_GRAD 1
/* psf_opts.flags: build_psf_sysmat's count phase keeps the rows it compacts in
 * the workspace (psf_workspace_size adds room for them, about 1 MB per voxel
 * of the range, at most 32 GB), and a fill phase that follows on the same
 * workspace with the same table and options copies them instead of
 * recomputing; rows that did not fit are recomputed. */
#define PSF_OPT_STAGE_CSR 2
/* psf_opts.flags (3D build_psf_sysmat): the caller asserts that since a build
 * on this handle last completed on this workspace, the workspace was passed
 * only to calls on this handle and not otherwise written.  The build then
 * skips clearing its accumulators (every build leaves them clear; the last
 * 32 bytes of the workspace header record the handle and layout that did, and
 * the clear is skipped only when they match).  A wrong assertion gives wrong
 * matrices; without the flag every build clears them (about 67 GB, twice that
 * for deterministic builds). */
#define PSF_OPT_WS_CLEAN 4
/* psf_opts.flags (build_psf_sysmat): [vox_begin, vox_end) counts positions in
 * the library's voxel order (psf_voxel_order) instead of linear voxel indices;
 * CSR row k is then voxel order[vox_begin + k].  In that order the voxels that
 * share their line bundles and tiles (Sec 2.3 computes each voxel's bundle
 * separately; a ring shift along z, the square's quarter turns and mirrors and
 * the axial mirror leave a bundle's tiles unchanged up to a relabelling of the
 * crystals) lie side by side, so a range of it builds at the rate of a whole
 * image.  A range may cut a group; its voxels inside the range are then built
 * one by one.  2D: the order is the linear one. */
#define PSF_OPT_CLASS_ORDER 8
/* psf_opts.flags: the workspace will serve psf_osem_update and
 * psf_subset_sensitivity (psf_workspace_size adds their sinogram buffers). */
#define PSF_OPT_OSEM 16
/* psf_opts.flags (build_psf_sysmat): a deterministic build.  Each voxel's
 * entries are summed as 64-bit integers in units of 2^-62 (each tile entry
 * rounded to that unit once) instead of FP32 / FP64 floating-point atomics,
 * whose order of arrival varies; integer sums do not depend on that order, so
 * the CSR (pattern and values) is bitwise the same from run to run, on any
 * GPU of the same architecture.  An element's error against the exact sum of
 * its tile entries is at most (number of entries) x 2^-63 in absolute value,
 * so elements far below 1e-12 lose relative precision and those below about
 * 1e-19 may round to zero.  Tile entries must lie in [0, 1) and elements
 * below 2 (true for response tables of probabilities); a tile entry outside
 * that range returns PSF_ERANGE.  3D: the accumulators take 8 bytes per cell
 * instead of 4 (psf_workspace_size must be asked with the flag).  Projections
 * refuse the flag (PSF_EUNSUPPORTED). */
#define PSF_OPT_DETERMINISTIC 32

/* CSR of A^T: one row per voxel of the range, columns are bins, ascending. */
typedef struct {
    int64_t n_rows;         /* out: vox_end - vox_begin */
    int64_t nnz;            /* out (phase 1), in (phase 2): capacity of col/val */
    int64_t* row_ptr;       /* device [n_rows + 1] */
    int32_t* col;           /* device [nnz]; NULL selects phase 1 */
    float* val;             /* device [nnz] */
} psf_csr;

typedef struct psf_handle psf_handle;

/* Validate the geometry and image and upload geometry constants to the
 * current device.  mode3d = 0: a single 2D ring (n_cryst_z = n_block_rings = 1,
 * nz = 1, lines in the transaxial plane); mode3d = 1: the 3D scanner.
 * PSF_EGEOM if any voxel centre lies outside the ring of face lines. */
int psf_create(const psf_geometry* geom, const psf_image* img, int32_t mode3d, psf_handle** out);
/* Release the handle: waits for the work it ordered on its extra streams,
 * then frees its events and device constants.  The extra streams themselves
 * belong to the device and serve every handle until the process ends. */
void psf_destroy(psf_handle* h);

/* Number of crystals N and of bins N (N - 1) / 2; number of voxels. */
int psf_sizes(const psf_handle* h, int64_t* n_crystals, int64_t* n_bins, int64_t* n_voxels);

/* Analytic response table (stands in for the paper's GATE simulation, Sec
 * 2.1.1 Eq.1, normalised as Eq.6-7): first-interaction probability with
 * attenuation `mu` in a laterally unbounded crystal array, averaged over each
 * sub-position; computed in FP64 on the device, stored as FP32 into
 * table_dev (layout of psf_table, 2D or 3D by the handle's mode). */
int psf_build_table(psf_handle* h, int32_t n_rows, int32_t n_sub, double step_deg, float* table_dev,
                    void* stream);

/* The same analytic table computed in FP64 on the host (the table builder
 * of Sec 2.1.1 and Eq.6-7 as the device call above, kept in double precision
 * and written to host memory, layout of psf_table for mode3d 0 or 1).  Needs no
 * handle and no GPU; runs on the calling thread (the 3D table of 61 x 61 rows
 * and 4 x 4 sub-positions takes a few seconds). */
int psf_build_table_host(const psf_geometry* geom, int32_t mode3d, int32_t n_rows, int32_t n_sub, double step_deg,
                         double* table_host);

/* Response table by photon-transport Monte Carlo (paper Sec 2.1.1, Eq.1:
 * the response of the crystal array to photons entering at each sub-position
 * and incidence angle is simulated; indexed as Sec 2.1.3, Eq.6-7), in the
 * layout of psf_build_table, for this handle's crystals (pitches, depth,
 * attenuation mu) and its mode (2D or 3D).  Each of the table's cells (2D:
 * n_rows x n_sub; 3D: n_rows^2 x n_sub^2) follows `photons` photons entering
 * uniformly over its sub-position; an entry is the fraction detected in that
 * neighbour crystal.
 *   scatter 0: first interaction only (the path length is exponential with
 *     attenuation mu); its expectation is psf_build_table's analytic table.
 *   scatter 1: photoelectric absorption (0.32 of mu at 511 keV, scaled by
 *     (511/E)^3) and Compton scatter (Klein-Nishina cross section and angles);
 *     a photon counts when 350 keV or more is deposited, in the crystal of the
 *     energy-weighted centroid of its deposits.
 * Photon k of cell c draws from Philox4x32-10 with counter (k, c, draw) and
 * key `seed`, so results do not depend on the launch and are reproducible.
 * counts_dev (optional, may be NULL): int64 [cells][5][5] detected photons
 * (2D: entries [a + 2][2]).  photons in [1, 2^32).  Asynchronous. */
int psf_build_table_mc(psf_handle* h, int32_t n_rows, int32_t n_sub, double step_deg, int64_t photons,
                       uint64_t seed, int32_t scatter, float* table_dev, int64_t* counts_dev, void* stream);

/* Device workspace in bytes needed by the calls below for these options,
 * batch size and number of events. */
int psf_workspace_size(const psf_handle* h, const psf_table* table, const psf_opts* opts, int32_t batch,
                       int64_t n_events, size_t* bytes);

/* System matrix, voxel by voxel (paper Sec 2.3): for each voxel of
 * [vox_begin, vox_end), every homogenized line through its centre (Eq.11)
 * spreads, through the response rows of its two end crystals (Eq.2-7), into
 * the crystal-pair bins with probability w U[a] V[b] (Eq.10, summed as Eq.12).
 * Two phases on the same options:
 *   phase 1 (csr->col == NULL): writes row_ptr and sets csr->nnz; BLOCKS.
 *   phase 2: fills col/val (capacity csr->nnz); BLOCKS; PSF_EOVERFLOW if a
 *   row would exceed what phase 1 allotted.
 * 3D: PSF_EUNSUPPORTED when a class's accumulator cells (4096 transaxial
 * slots x (NR + 15)^2 ring pairs x 16 voxels) would not index in 32 bits, that
 * is for more than about 165 crystal rings.  A 3D phase 1 with
 * PSF_OPT_STAGE_CSR also uses the handle's extra streams (see the conventions
 * above). */
int build_psf_sysmat(psf_handle* h, const psf_table* table, const psf_opts* opts, void* workspace_dev,
                     size_t workspace_bytes, psf_csr* csr, void* stream);

/* The voxel order of PSF_OPT_CLASS_ORDER: order_host[k] (host memory,
 * n_voxels entries) is the linear index of the voxel at position k.  Every
 * voxel appears once.  The first call on a 3D handle plans the whole image
 * (tens of milliseconds on the host); the plan is kept in the handle. */
int psf_voxel_order(psf_handle* h, int64_t* order_host);

/* Forward projection y = A x on the fly, without storing A (paper Table 2's
 * projector).  x_dev: [batch][n_voxels]; y_dev: [batch][n_bins] when
 * events_dev is NULL, else [batch][n_events] with events_dev an int32
 * [n_events][2] list of crystal pairs (list-mode rows).  An empty list
 * (events_dev not NULL, n_events 0) writes nothing (y_dev may be NULL). */
int project_fwd(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* x_dev, int32_t batch,
                const int32_t* events_dev, int64_t n_events, float* y_dev, void* workspace_dev,
                size_t workspace_bytes, void* stream);

/* project_fwd for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation on a 2D handle, with its scratch (a status word and the
 * FP64 bin accumulator, 256 + 8 * batch * n_bins bytes) in a 16 MiB device
 * array the library owns instead of a workspace; the caller passes inputs and
 * outputs only.  No hipMalloc, hipFree or other allocation happens in the call.
 * PSF_ESIZE if the scratch would exceed 16 MiB (at most 258 images of the
 * 128-crystal ring); PSF_EUNSUPPORTED on a 3D handle.  Each GPU has one such
 * array, shared by every call on it: calls that overlap on one GPU (other
 * streams, other threads, other handles) race and must be serialised by the
 * caller.  Status flags of the call (psf_check) are not kept. */
int project_fwd_noalloc(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* x_dev,
                        int32_t batch, const int32_t* events_dev, int64_t n_events, float* y_dev, void* stream);

/* Back projection x = A^T y (layouts as project_fwd; an empty event list
 * gives x = 0, or leaves x as it is with opts->accumulate, and y_dev may then
 * be NULL).  If grad_table_dev is
 * not NULL, also accumulates d <y, A xt> / d table into it (FP32, table
 * layout, summed over the batch) with xt = xt_dev [batch][n_voxels]: each
 * response entry U[p][a] (Eq.6-7, with its mirror and two-block remap) is a
 * table entry, so the gradient collects, over the tiles T = U^T W V (Eq.10,
 * 12), (W V G^T) for the rows of photon 1 and (W^T U G) for those of photon 2,
 * G the bins' y times the voxel's xt.  In 3D the workspace must have been
 * sized with PSF_OPT_TABLE_GRAD in opts->flags (else PSF_ESIZE). */
int project_adj(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* y_dev, int32_t batch,
                const int32_t* events_dev, int64_t n_events, float* x_dev, const float* xt_dev,
                float* grad_table_dev, void* workspace_dev, size_t workspace_bytes, void* stream);

/* Sensitivity s = A^T 1 over all bins, FP32 [n_voxels] (summed in FP64). */
int psf_sensitivity(psf_handle* h, const psf_table* table, const psf_opts* opts, float* s_dev,
                    void* workspace_dev, size_t workspace_bytes, void* stream);

/* One list-mode OSEM subset update (the list-mode use the paper names as
 * its next step, Sec 4):
 *   x_out = x_in / (s / n_subsets) * sum_e a_e / (a_e^T x_in + randoms)
 * over the n_events crystal pairs of events_dev; voxels with s = 0 get 0. */
int psf_lm_osem_update(psf_handle* h, const psf_table* table, const psf_opts* opts, const int32_t* events_dev,
                       int64_t n_events, float randoms, const float* sens_dev, int32_t n_subsets,
                       const float* x_in_dev, float* x_out_dev, void* workspace_dev, size_t workspace_bytes,
                       void* stream);

/* One histogram-mode OSEM subset update (paper Sec 3: the reconstructions of
 * Fig. 9-12 and Table 2-3 run OSEM, 24 subsets of a 192-angle sinogram):
 *   x_out = x_in / s_k * A^T (m_k y / A x_in),
 * with y_dev the measured sinogram [n_bins] (FP32, bin layout of project_fwd),
 * m_k the bins whose sinogram angle lies in subset k (angle of crystal pair
 * (g_i, g_j) on an Nc-crystal ring: view ((g_i + g_j) mod Nc) / 2 of Nc / 2;
 * subset k: the views v with v mod n_subsets = k; in 3D the transaxial pair
 * decides), and s_k = A^T m_k from psf_subset_sensitivity.  Bins whose
 * estimate A x_in is 0 contribute 0; voxels with s_k = 0 get 0.  One image;
 * the workspace is sized with PSF_OPT_OSEM.  2D: asynchronous; 3D: blocks
 * (see project_fwd). */
int psf_osem_update(psf_handle* h, const psf_table* table, const psf_opts* opts, const float* y_dev,
                    int32_t n_subsets, int32_t subset, const float* sens_dev, const float* x_in_dev, float* x_out_dev,
                    void* workspace_dev, size_t workspace_bytes, void* stream);

/* s_k = A^T m_k: the sensitivity of subset k of psf_osem_update, FP32 [n_voxels]. */
int psf_subset_sensitivity(psf_handle* h, const psf_table* table, const psf_opts* opts, int32_t n_subsets,
                           int32_t subset, float* s_dev, void* workspace_dev, size_t workspace_bytes, void* stream);

/* Wait for `stream` and report the status word the kernels keep in the
 * workspace (PSF_ERANGE if an incidence angle fell beyond the table). */
int psf_check(psf_handle* h, void* workspace_dev, void* stream);

/* Timing of the kernels, for measurement.  enable = 1 clears and starts
 * recording a pair of HIP events around each launch of the contraction
 * kernels (the 2D per-voxel sweep, the 3D matrix-core tile contraction) and of
 * the 3D tile-geometry kernel, on the stream they run on; enable = 0 waits for
 * them and writes ms[0], launches[0] (contraction) and ms[1], launches[1]
 * (3D geometry): summed elapsed milliseconds and launch counts.  ms and
 * launches point to two entries each (either may be NULL).  In 3D the
 * workspace holds at byte 64 a uint64 count of the tiles contracted by the
 * last call, and at byte 72 the count of (voxel, tile) pairs they served
 * (a tile serves every voxel of its z-column class that sees both its rings). */
int psf_profile(psf_handle* h, int32_t enable, double* ms, int64_t* launches);

const char* psf_status_string(int status);
int psf_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PSF_H */
