// List-mode helpers (the list-mode use of the matrix is the paper's stated
// next step, Sec 4).  An event is a crystal pair (i, j); its matrix row is the
// row of bin(i, j).  The rows come from the on-the-fly projector, which runs
// voxel by voxel over every bin whatever the number of events: a voxel's tiles
// are computed once and serve every event whose bins they reach, while rows
// evaluated event by event would recompute a voxel's tiles for each event
// through it (the projector's cost does not fall with fewer events, but stays
// far below per-event rows for a subset of 1e6 events on 1.7e8 bins).  These
// kernels move between event space and bin space:
//   gather   q_e = y[bin_e]                        (forward rows)
//   scatter  h[bin] += v_e over events in the bin  (adjoint rows)
//   ratio    h[bin] += 1 / (y[bin_e] + r)          (the LM-OSEM weights)
//   update   x_out = x_in * back / (s / M)         (one subset update)
#include "common.hpp"

namespace psf {

constexpr int kStatEvent = kStatEventBad;

// Crystal ids: id = ring * Nc + g.  2D (NR == 1): bin of the unordered pair;
// 3D: transaxial pair (g_i < g_j) major, then the rings (r_i, r_j).
struct EvGeo {
    int64_t Nc, NR;
};

__device__ __forceinline__ bool event_bin(const int32_t* ev, int64_t e, EvGeo g, int64_t& bin) {
    const int64_t N = g.Nc * g.NR;
    int64_t i = ev[2 * e], j = ev[2 * e + 1];
    if (i < 0 || j < 0 || i >= N || j >= N || i == j) return false;
    int64_t gi = i % g.Nc, ri = i / g.Nc, gj = j % g.Nc, rj = j / g.Nc;
    if (g.NR == 1) {
        if (i > j) { const int64_t t = i; i = j; j = t; }
        bin = i * N - i * (i + 1) / 2 + (j - i - 1);
        return true;
    }
    if (gi == gj) return false;  // no line through the inside joins them
    if (gi > gj) {
        int64_t t = gi; gi = gj; gj = t;
        t = ri; ri = rj; rj = t;
    }
    bin = ((gi * g.Nc - gi * (gi + 1) / 2 + (gj - gi - 1)) * g.NR + ri) * g.NR + rj;
    return true;
}

__global__ void k_lm_gather(const double* y64, const float* y32, int64_t nbins, const int32_t* ev, int64_t ne, int batch, EvGeo N,
                            float* out, int accumulate, int* status) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t bin = 0;
        const bool ok = event_bin(ev, e, N, bin);
        if (!ok) atomicOr(status, kStatEvent);
        for (int bb = 0; bb < batch; ++bb) {
            const int64_t k = (int64_t)bb * nbins + bin;
            const float v = ok ? (y64 ? (float)y64[k] : y32[k]) : 0.0f;
            float* o = out + (int64_t)bb * ne + e;
            *o = accumulate ? *o + v : v;
        }
    }
}

__global__ void k_lm_scatter(const float* h, int64_t ne, const int32_t* ev, int batch, EvGeo N, int64_t nbins,
                             double* hist, int* status) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t bin = 0;
        if (!event_bin(ev, e, N, bin)) {
            atomicOr(status, kStatEvent);
            continue;
        }
        for (int bb = 0; bb < batch; ++bb) {
            const double v = (double)h[(int64_t)bb * ne + e];
            if (v != 0.0) atomicAdd(&hist[(int64_t)bb * nbins + bin], v);
        }
    }
}

__global__ void k_lm_ratio(const double* y64, const float* y32, const int32_t* ev, int64_t ne, EvGeo N, double randoms, double* hist,
                           int* status) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t bin = 0;
        if (!event_bin(ev, e, N, bin)) {
            atomicOr(status, kStatEvent);
            continue;
        }
        const double q = (y64 ? y64[bin] : (double)y32[bin]) + randoms;
        if (q > 0.0) atomicAdd(&hist[bin], 1.0 / q);
    }
}

__global__ void k_lm_update(const float* x_in, const float* back, const float* sens, double n_subsets,
                            int64_t nvox, float* x_out) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x) {
        const double s = (double)sens[v];
        x_out[v] = s > 0.0 ? (float)((double)x_in[v] * (double)back[v] * n_subsets / s) : 0.0f;
    }
}

static unsigned grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b < 65536 ? b : 65536));
}

hipError_t launch_lm_gather(const double* y64, const float* y32, int64_t nbins, const int32_t* ev, int64_t ne,
                            int batch, int64_t Nc, int64_t NR, float* out, int accumulate, int* status,
                            hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lm_gather, dim3(grid_for(ne)), dim3(256), 0, st, y64, y32, nbins, ev, ne, batch,
                       EvGeo{Nc, NR}, out, accumulate, status);
    return hipGetLastError();
}

hipError_t launch_lm_scatter(const float* h, int64_t ne, const int32_t* ev, int batch, int64_t Nc, int64_t NR,
                             int64_t nbins, double* hist, int* status, hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lm_scatter, dim3(grid_for(ne)), dim3(256), 0, st, h, ne, ev, batch, EvGeo{Nc, NR}, nbins,
                       hist, status);
    return hipGetLastError();
}

hipError_t launch_lm_ratio(const double* y64, const float* y32, const int32_t* ev, int64_t ne, int64_t Nc, int64_t NR,
                           double randoms, double* hist, int* status, hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lm_ratio, dim3(grid_for(ne)), dim3(256), 0, st, y64, y32, ev, ne, EvGeo{Nc, NR}, randoms,
                       hist, status);
    return hipGetLastError();
}

hipError_t launch_lm_update(const float* x_in, const float* back, const float* sens, int n_subsets, int64_t nvox,
                            float* x_out, hipStream_t st) {
    hipLaunchKernelGGL(k_lm_update, dim3(grid_for(nvox)), dim3(256), 0, st, x_in, back, sens, (double)n_subsets,
                       nvox, x_out);
    return hipGetLastError();
}

}  // namespace psf
