// Host-side internals shared by the C-ABI translation units (not part of the ABI).
#pragma once

#include <math.h>

#include <utility>
#include <vector>

#include "common.hpp"

// The 3D build's voxels in class order (voxels that share tiles side by side):
// the classes of a whole-image plan, each with its first position and its
// members (voxel, ring shift), in order.  Computed once per handle.
struct ClassOrderCache {
    bool valid = false;
    int64_t key[3] = {0, 0, 0};     // the plan's limits it was made with
    std::vector<int4> cls;          // reference voxel, -, member count, largest shift
    std::vector<int> sym;           // the class's symmetry word
    std::vector<int64_t> first;     // position of the class's first member
    std::vector<int2> mem;          // by position: voxel, ring shift
};

// the extra streams' events: after a contraction (build); after an even / odd
// batch (build: its compaction; projections: its last kernel); the join; a
// batch's geometry; the start
constexpr int kAuxEvents = 6;
constexpr int kAuxDevices = 64;  // devices with the extra streams

struct psf_handle {
    ClassOrderCache order;
    psf_geometry g;
    psf_image im;
    int mode3d;
    int device;
    int64_t n_crystals, n_bins, n_vox;
    double sigma;
    double* frames_dev;  // [R][2] cos, sin of each block's outward normal
    // HIP-event timing of the contraction (kind 0) and 3D geometry (kind 1) kernels (psf_profile)
    bool prof_on;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
    std::vector<int> prof_kind;
    // the 3D calls' second and third streams (the device's, shared by the
    // process's handles) and this handle's events (created on first use)
    hipStream_t aux = nullptr, aux2 = nullptr;
    hipEvent_t aux_ev[kAuxEvents] = {};
};

// bracket one launch of the contraction kernel with events when profiling
struct ProfScope {
    psf_handle* h;
    hipStream_t s;
    hipEvent_t e1;
    ProfScope(psf_handle* h_, hipStream_t s_, int kind = 0) : h(h_), s(s_), e1(nullptr) {
        if (h->prof_on) {
            hipEvent_t e0;
            if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
                hipEventRecord(e0, s) == hipSuccess) {
                h->prof_ev.emplace_back(e0, e1);
                h->prof_kind.push_back(kind);
            } else {
                e1 = nullptr;
            }
        }
    }
    ~ProfScope() {
        if (e1) (void)hipEventRecord(e1, s);
    }
};

namespace psf {
extern thread_local int g_last_hip;
}

#define HIP_TRY(expr)                         \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) {               \
            psf::g_last_hip = (int)e_;        \
            return PSF_EHIP;                  \
        }                                     \
    } while (0)

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t table_elems(const psf_handle* h, const psf_table* t);
int check_table(const psf_handle* h, const psf_table* t);
int check_opts(const psf_opts* o, bool build = false);  // build: a matrix build (the only call taking PSF_OPT_DETERMINISTIC)
int zero_header(void* ws, hipStream_t st);
int read_status(void* ws, hipStream_t st);

// 3D entry points (api3d.hip)
size_t ws3_total(const psf_handle* h, const psf_table* t, int batch, int64_t n_events, const psf_opts* o);
int build_sysmat_3d(psf_handle* h, const psf_table* t, const psf_opts* o, void* ws, size_t ws_bytes, psf_csr* csr,
                    hipStream_t s);
int project_fwd_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const float* x, int batch,
                   const int32_t* events, int64_t n_events, float* y, void* ws, size_t ws_bytes, hipStream_t s);
int project_adj_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const float* y, int ones, int batch,
                   const int32_t* events, int64_t n_events, float* x, const float* xt, float* grad, void* ws,
                   size_t ws_bytes, hipStream_t s);
int voxel_order_3d(psf_handle* h, int64_t* order);
int osem_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const float* y, int n_subsets, int subset,
            const float* sens, const float* x_in, float* x_out, void* ws, size_t ws_bytes, hipStream_t s);
int subset_sensitivity_3d(psf_handle* h, const psf_table* t, const psf_opts* o, int n_subsets, int subset, float* s_dev,
                          void* ws, size_t ws_bytes, hipStream_t s);
int lm_osem_3d(psf_handle* h, const psf_table* t, const psf_opts* o, const int32_t* events, int64_t n_events,
               float randoms, const float* sens, int n_subsets, const float* x_in, float* x_out, void* ws,
               size_t ws_bytes, hipStream_t s);
