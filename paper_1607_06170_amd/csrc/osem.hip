// Histogram-mode OSEM (paper Sec 3: the reconstructions of Fig. 9-12 and
// Table 2-3 run OSEM over a sinogram of angles x radial bins, Table 1).  One
// subset update:
//   x_out = x_in / s_k * A^T (m_k y / A x_in),   s_k = A^T m_k,
// where m_k selects the bins whose sinogram angle belongs to subset k.  The
// angle of the crystal pair (g_i, g_j) of an Nc-crystal ring is view
// ((g_i + g_j) mod Nc) / 2 of Nc / 2; subset k holds the views v with
// v mod n_subsets = k.  These kernels are the elementwise steps between the
// projections.
#include "common.hpp"

namespace psf {

// transaxial pair (gi < gj) of a transaxial bin: the largest gi whose first bin
// is at most tb (bisection on gi Nc - gi (gi + 1) / 2)
__device__ __forceinline__ void tbin_pair(int64_t tb, int64_t Nc, int64_t& gi, int64_t& gj) {
    int64_t lo = 0, hi = Nc - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (mid * Nc - mid * (mid + 1) / 2 <= tb) lo = mid;
        else hi = mid - 1;
    }
    gi = lo;
    gj = tb - (lo * Nc - lo * (lo + 1) / 2) + lo + 1;
}

__device__ __forceinline__ bool in_subset(int64_t bin, int64_t Nc, int64_t NR, int n_subsets, int subset) {
    int64_t gi, gj;
    tbin_pair(bin / (NR * NR), Nc, gi, gj);
    const int64_t view = ((gi + gj) % Nc) >> 1;
    return view % n_subsets == subset;
}

// r[b] = m_k(b) y[b] / yhat[b] (0 where yhat is 0); yhat FP64 (2D) or FP32 (3D)
__global__ void k_osem_ratio(const double* yh64, const float* yh32, const float* y, int64_t nbins, int64_t Nc,
                             int64_t NR, int n_subsets, int subset, float* r) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nbins; b += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.0f;
        if (in_subset(b, Nc, NR, n_subsets, subset)) {
            const double q = yh64 ? yh64[b] : (double)yh32[b];
            if (q > 0.0) v = (float)((double)y[b] / q);
        }
        r[b] = v;
    }
}

__global__ void k_subset_mask(int64_t nbins, int64_t Nc, int64_t NR, int n_subsets, int subset, float* m) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nbins; b += (int64_t)gridDim.x * blockDim.x)
        m[b] = in_subset(b, Nc, NR, n_subsets, subset) ? 1.0f : 0.0f;
}

__global__ void k_osem_update(const float* x_in, const float* back, const float* sens, int64_t nvox, float* x_out) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x) {
        const double s = (double)sens[v];
        x_out[v] = s > 0.0 ? (float)((double)x_in[v] * (double)back[v] / s) : 0.0f;
    }
}

static unsigned grid_of(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b < 65536 ? b : 65536));
}

hipError_t launch_osem_ratio(const double* yh64, const float* yh32, const float* y, int64_t nbins, int64_t Nc,
                             int64_t NR, int n_subsets, int subset, float* r, hipStream_t st) {
    hipLaunchKernelGGL(k_osem_ratio, dim3(grid_of(nbins)), dim3(256), 0, st, yh64, yh32, y, nbins, Nc, NR, n_subsets,
                       subset, r);
    return hipGetLastError();
}

hipError_t launch_subset_mask(int64_t nbins, int64_t Nc, int64_t NR, int n_subsets, int subset, float* m,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_subset_mask, dim3(grid_of(nbins)), dim3(256), 0, st, nbins, Nc, NR, n_subsets, subset, m);
    return hipGetLastError();
}

hipError_t launch_osem_update(const float* x_in, const float* back, const float* sens, int64_t nvox, float* x_out,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_osem_update, dim3(grid_of(nvox)), dim3(256), 0, st, x_in, back, sens, nvox, x_out);
    return hipGetLastError();
}

}  // namespace psf
