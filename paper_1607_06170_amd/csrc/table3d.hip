// Analytic 3D response table (the 3D form of Sec 2.1.1 Eq.1, normalised as
// Eq.6-7), FP64 on the device, stored FP32 as
//   table[row_t][row_z][pt][pz][a_t+2][a_z+2].
//
// A photon enters at (ut, uz) from the entry crystal's lower edges with
// lateral slopes tt = tan(alpha_t), tz = tan(alpha_z) >= 0 per unit depth;
// the path length to depth d is d * k, k = sqrt(1 + tt^2 + tz^2).  Column
// (a_t, a_z) holds the photon for the depths inside both lateral crystal
// ranges, [max(ta, za), min(tb, zb)], so its first-interaction probability is
// exp(-mu k max(ta, za)) - exp(-mu k min(tb, zb)).  For a fixed ut the
// integral over uz is elementary (za, zb are linear in uz); the integral over
// ut is 16-point Gauss-Legendre between the points where that closed form
// changes shape, so each piece is smooth.
#include "common.hpp"

namespace psf {

struct GL16 {
    double x[16], w[16];
};

// integral over uz in [uz0, uz1] at fixed ut
__host__ __device__ static double inner_uz3(double tt, double tz, double ut, double uz0, double uz1, int at, int az,
                                   double lt, double lz, double L, double mu) {
    double ta, tb;
    if (tt == 0.0) {
        if (at != 0) return 0.0;
        ta = 0.0;
        tb = L;
    } else {
        ta = fmax(0.0, (at * lt - ut) / tt);
        tb = fmin(L, ((at + 1) * lt - ut) / tt);
        if (!(tb > ta)) return 0.0;
    }
    const double m = mu * sqrt(1.0 + tt * tt + tz * tz);
    if (tz == 0.0) {
        if (az != 0) return 0.0;
        return (uz1 - uz0) * (exp(-m * ta) - exp(-m * tb));
    }
    // za(uz) = (az lz - uz)/tz, zb = za + lz/tz; the column is crossed iff za < tb and zb > ta
    const double lo = fmax(uz0, az * lz - tz * tb), hi = fmin(uz1, (az + 1) * lz - tz * ta);
    if (!(hi > lo)) return 0.0;
    const double e0 = az * lz, e1 = (az + 1) * lz;
    // entry depth max(ta, za): za > ta below u1
    const double u1 = e0 - tz * ta;
    double i1 = 0.0, a, b;
    a = lo;
    b = fmin(hi, u1);
    if (b > a) i1 += (tz / m) * (exp(-m * (e0 - b) / tz) - exp(-m * (e0 - a) / tz));
    a = fmax(lo, u1);
    b = hi;
    if (b > a) i1 += (b - a) * exp(-m * ta);
    // exit depth min(tb, zb): zb >= tb below u2
    const double u2 = e1 - tz * tb;
    double i2 = 0.0;
    a = lo;
    b = fmin(hi, u2);
    if (b > a) i2 += (b - a) * exp(-m * tb);
    a = fmax(lo, u2);
    b = hi;
    if (b > a) i2 += (tz / m) * (exp(-m * (e1 - b) / tz) - exp(-m * (e1 - a) / tz));
    return i1 - i2;
}

// entry i of the table (layout of psf_table, 3D), FP64
__host__ __device__ static double table3_entry(int64_t i, int n_rows, int P, double step_deg, double lt, double lz,
                                               double L, double mu, const GL16& gl) {
    {
        const int az = (int)(i % kNb) - 2;
        const int at = (int)((i / kNb) % kNb) - 2;
        const int pz = (int)((i / (kNb * kNb)) % P);
        const int pt = (int)((i / (kNb * kNb * P)) % P);
        const int rz = (int)((i / ((int64_t)kNb * kNb * P * P)) % n_rows);
        const int rt = (int)(i / ((int64_t)kNb * kNb * P * P * n_rows));
        if (at < 0 || az < 0) return 0.0;
        const double alt = rt * step_deg * kPi / 180.0, alz = rz * step_deg * kPi / 180.0;
        const double tt = rt == 0 ? 0.0 : tan(alt), tz = rz == 0 ? 0.0 : tan(alz);
        const double ut0 = pt * lt / P, ut1 = (pt + 1) * lt / P;
        const double uz0 = pz * lz / P, uz1 = (pz + 1) * lz / P;
        double cut[16];
        int nc = 0;
        cut[nc++] = ut0;
        if (tt > 0.0) {
            double dep[6];
            int nd = 0;
            dep[nd++] = 0.0;
            dep[nd++] = L;
            if (tz > 0.0) {
                dep[nd++] = (az * lz - uz0) / tz;
                dep[nd++] = (az * lz - uz1) / tz;
                dep[nd++] = ((az + 1) * lz - uz0) / tz;
                dep[nd++] = ((az + 1) * lz - uz1) / tz;
            }
            for (int k = 0; k < nd; ++k) {
                const double c1 = at * lt - tt * dep[k], c2 = (at + 1) * lt - tt * dep[k];
                if (c1 > ut0 && c1 < ut1) cut[nc++] = c1;
                if (c2 > ut0 && c2 < ut1) cut[nc++] = c2;
            }
        }
        cut[nc++] = ut1;
        for (int a = 1; a < nc; ++a) {
            const double v = cut[a];
            int b = a - 1;
            while (b >= 0 && cut[b] > v) {
                cut[b + 1] = cut[b];
                --b;
            }
            cut[b + 1] = v;
        }
        double tot = 0.0;
        for (int k = 0; k + 1 < nc; ++k) {
            const double a = cut[k], b = cut[k + 1];
            if (!(b > a)) continue;
            const double h = 0.5 * (b - a), m = 0.5 * (a + b);
            double s = 0.0;
            for (int q = 0; q < 16; ++q) s += gl.w[q] * inner_uz3(tt, tz, m + h * gl.x[q], uz0, uz1, at, az, lt, lz, L, mu);
            tot += h * s;
        }
        return tot / ((ut1 - ut0) * (uz1 - uz0));
    }
}

__global__ void k_table_3d(int n_rows, int P, double step_deg, double lt, double lz, double L, double mu, GL16 gl,
                           float* out) {
    const int64_t n = (int64_t)n_rows * n_rows * P * P * kNb * kNb;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)table3_entry(i, n_rows, P, step_deg, lt, lz, L, mu, gl);
}

// Gauss-Legendre nodes on [-1, 1]: Newton's method on the Legendre recurrence
static GL16 gauss_legendre16() {
    GL16 g;
    const int n = 16;
    for (int i = 0; i < n; ++i) {
        double z = cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
            const double p2 = p1;
            p1 = p0;
            p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        g.x[i] = z;
        g.w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return g;
}

void table_3d_host(const psf_geometry& g, int n_rows, int P, double step_deg, double* out) {
    const int64_t n = (int64_t)n_rows * n_rows * P * P * kNb * kNb;
    const GL16 gl = gauss_legendre16();
    for (int64_t i = 0; i < n; ++i) out[i] = table3_entry(i, n_rows, P, step_deg, g.pitch_t, g.pitch_z, g.depth, g.mu, gl);
}

hipError_t launch_table_3d(const psf_geometry& g, int n_rows, int P, double step_deg, float* out, hipStream_t st) {
    const int64_t n = (int64_t)n_rows * n_rows * P * P * kNb * kNb;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(k_table_3d, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(threads), 0, st, n_rows,
                       P, step_deg, g.pitch_t, g.pitch_z, g.depth, g.mu, gauss_legendre16(), out);
    return hipGetLastError();
}

}  // namespace psf
