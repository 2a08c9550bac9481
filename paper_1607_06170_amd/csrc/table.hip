// Analytic response tables (stand-in for the GATE simulation of Sec 2.1.1,
// Eq.1, normalised as Eq.6-7), computed on the device in FP64.
//
// A photon enters the front face of a laterally unbounded row of crystals
// (width lambda, depth L, attenuation mu) at offset u from the entry crystal's
// lower edge, tilted by alpha >= 0 towards higher offsets.  Its first
// interaction lies in crystal a with probability
//     exp(-mu s_in) - exp(-mu s_out),
// s_in / s_out the path lengths at which it enters / leaves crystal a's column
// (both capped at the back face, L / cos alpha).  Each table entry is the mean
// over a sub-position u in [p lambda/P, (p+1) lambda/P), integrated here in
// closed form: exp(-mu * clip((c - u) / sin alpha, 0, smax)) has an elementary
// antiderivative on each of its three pieces.
#include "common.hpp"

namespace psf {

// integral over [u0, u1] of exp(-mu * clip((c - u) / sa, 0, smax)) du
__host__ __device__ static double edge_integral(double c, double u0, double u1, double sa, double smax, double mu) {
    const double reach = smax * sa;  // lateral travel over the full depth
    double tot = 0.0;
    double lo = fmax(u0, c), hi = u1;  // photon already past the edge c: factor 1
    if (hi > lo) tot += hi - lo;
    lo = fmax(u0, c - reach);
    hi = fmin(u1, c);                  // reaches the edge c inside the crystal depth
    if (hi > lo) tot += (sa / mu) * (exp(-mu * (c - hi) / sa) - exp(-mu * (c - lo) / sa));
    lo = u0;
    hi = fmin(u1, c - reach);          // leaves through the back face first
    if (hi > lo) tot += (hi - lo) * exp(-mu * smax);
    return tot;
}

// mean first-interaction probability in crystal a over sub-position [u0, u1)
__host__ __device__ static double sub_response(double alpha, double u0, double u1, int a, double lam, double L, double mu) {
    if (a < 0) return 0.0;
    if (alpha == 0.0) return a == 0 ? 1.0 - exp(-mu * L) : 0.0;
    const double sa = sin(alpha), smax = L / cos(alpha);
    const double in = edge_integral(a * lam, u0, u1, sa, smax, mu);
    const double out = edge_integral((a + 1) * lam, u0, u1, sa, smax, mu);
    return (in - out) / (u1 - u0);
}

__global__ void k_table_2d(int n_rows, int P, double step_deg, double lam, double L, double mu, float* out) {
    const int n = n_rows * P * kNb;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int a = i % kNb - 2;
        const int p = (i / kNb) % P;
        const int row = i / (kNb * P);
        const double alpha = row * step_deg * kPi / 180.0;
        const double u0 = p * lam / P, u1 = (p + 1) * lam / P;
        out[i] = (float)sub_response(alpha, u0, u1, a, lam, L, mu);
    }
}

// the same entries in FP64 on the host, one after the other
void table_2d_host(const psf_geometry& g, int n_rows, int P, double step_deg, double* out) {
    const int n = n_rows * P * kNb;
    for (int i = 0; i < n; ++i) {
        const int a = i % kNb - 2;
        const int p = (i / kNb) % P;
        const int row = i / (kNb * P);
        const double alpha = row * step_deg * kPi / 180.0;
        out[i] = sub_response(alpha, p * g.pitch_t / P, (p + 1) * g.pitch_t / P, a, g.pitch_t, g.depth, g.mu);
    }
}

hipError_t launch_table_2d(const psf_geometry& g, int n_rows, int P, double step_deg, float* out, hipStream_t st) {
    const int n = n_rows * P * kNb;
    const int threads = 256, blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(k_table_2d, dim3(blocks), dim3(threads), 0, st, n_rows, P, step_deg, g.pitch_t, g.depth, g.mu,
                       out);
    return hipGetLastError();
}

}  // namespace psf
