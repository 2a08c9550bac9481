// Response table by photon-transport Monte Carlo (Sec 2.1.1 Eq.1 obtains the
// table by simulating photons entering a crystal array; Sec 2.1.3 Eq.6-7
// indexes it by angle row and sub-position).  Same layout as the analytic
// table: 2D [row][p][a+2], 3D [row_t][row_z][pt][pz][a_t+2][a_z+2], each
// entry the fraction of the cell's photons detected in that crystal.
//
// One workgroup per table cell; its threads take the cell's photons in turn
// and count detections in LDS.  Photon k of cell c draws from a
// counter-based generator, Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC
// 2011), with counter (k low, k high, c, draw) and key (seed low, seed high),
// so a photon's path does not depend on which thread runs it; each draw
// gives two FP64 uniforms in (0, 1) from 53 bits of two output words.
//
// Transport (FP64), in a crystal array unbounded laterally, depth L, front
// face at depth 0; the photon enters uniformly over the sub-position of
// crystal 0 with direction (tan a_t, tan a_z, 1) normalised (2D: a_z = 0, no
// axial bound):
//   - first interaction (scatter = 0): depth -ln(u) / (mu k), k the path per
//     unit depth; detected in the crystal holding that point if inside L;
//   - with Compton scatter (scatter = 1): attenuation mu at 511 keV of which
//     0.32 photoelectric; at energy E the photoelectric part scales by
//     (511 / E)^3, the Compton part by the Klein-Nishina cross section.  Each
//     Compton event leaves E - E' at its point and turns the photon by a
//     Klein-Nishina angle (a uniform cosine kept with probability f / 2, at
//     most 64 tries) and a uniform azimuth; photons crossing either face are
//     lost; energy below 1 keV is absorbed in place.  A photon counts when 350
//     keV or more was deposited, in the crystal of the energy-weighted
//     centroid.
#include "common.hpp"

namespace psf {

namespace {

struct Philox {
    unsigned int c0, c1, c2, c3, k0, k1;
    // two uniforms from the next draw of this photon's stream
    __device__ void next(double& a, double& b) {
        unsigned int x0 = c0, x1 = c1, x2 = c2, x3 = c3, y0 = k0, y1 = k1;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const unsigned int lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
            const unsigned int lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
            const unsigned int n0 = hi1 ^ x1 ^ y0, n2 = hi0 ^ x3 ^ y1;
            x0 = n0;
            x1 = lo1;
            x2 = n2;
            x3 = lo0;
            y0 += 0x9E3779B9u;
            y1 += 0xBB67AE85u;
        }
        c3 += 1;
        a = ((double)((((unsigned long long)x0 << 32) | x1) >> 11) + 0.5) * 0x1p-53;
        b = ((double)((((unsigned long long)x2 << 32) | x3) >> 11) + 0.5) * 0x1p-53;
    }
};

// Klein-Nishina total cross section (units of 2 pi r_e^2) at k = E / 511 keV
__device__ double kn_total(double k) {
    const double q = 1.0 + 2.0 * k, lq = log(q);
    return (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / q - lq / k) + lq / (2.0 * k) - (1.0 + 3.0 * k) / (q * q);
}

struct McCell {
    double lt, lz, L, mu, tt, tz;
    int P, pt, pz, mode3d;
};

// the detected crystal offsets of one photon; false if it is not detected
template <bool SCATTER>
__device__ bool track(const McCell& m, Philox& rng, int& at, int& az) {
    double a, b;
    rng.next(a, b);
    const double x0 = (m.pt + a) / m.P * m.lt;
    const double y0 = m.mode3d ? (m.pz + b) / m.P * m.lz : 0.0;
    const double kk = sqrt(1.0 + m.tt * m.tt + m.tz * m.tz);
    if constexpr (!SCATTER) {
        double s, unused;
        rng.next(s, unused);
        const double d = -log(s) / m.mu / kk;
        if (!(d < m.L)) return false;
        at = (int)floor((x0 + d * m.tt) / m.lt);
        az = m.mode3d ? (int)floor((y0 + d * m.tz) / m.lz) : 0;
        return true;
    } else {
        const double k511 = kn_total(1.0);
        double px = x0, py = y0, pz = 0.0;
        double dx = m.tt / kk, dy = m.tz / kk, dz = 1.0 / kk;
        double e = 511.0, esum = 0.0, wx = 0.0, wy = 0.0;
        for (int it = 0; it < 64; ++it) {
            const double kr = e / 511.0, ir = 511.0 / e;
            const double mpe = 0.32 * m.mu * ir * ir * ir;
            const double mtot = mpe + (1.0 - 0.32) * m.mu * kn_total(kr) / k511;
            double us, ut;
            rng.next(us, ut);
            const double step = -log(us) / mtot;
            px += step * dx;
            py += step * dy;
            pz += step * dz;
            if (pz < 0.0 || pz > m.L) break;
            if (ut * mtot < mpe) {  // photoelectric: all of it stays here
                esum += e;
                wx += e * px;
                wy += e * py;
                break;
            }
            double cth = 1.0, ratio = 1.0;
            for (int t = 0; t < 64; ++t) {
                double ua, ub;
                rng.next(ua, ub);
                cth = 2.0 * ua - 1.0;
                ratio = 1.0 / (1.0 + kr * (1.0 - cth));
                const double shape = ratio * ratio * (ratio + 1.0 / ratio - (1.0 - cth * cth));
                if (ub * 2.0 < shape) break;
            }
            double uphi, unused;
            rng.next(uphi, unused);
            const double phi = 2.0 * kPi * uphi;
            const double eout = e * ratio, dep = e - eout;
            esum += dep;
            wx += dep * px;
            wy += dep * py;
            e = eout;
            const double sth = sqrt(fmax(0.0, 1.0 - cth * cth)), cp = cos(phi), sp = sin(phi);
            double nx, ny, nz;
            if (fabs(dz) > 0.99999) {
                nx = sth * cp;
                ny = sth * sp;
                nz = dz > 0.0 ? cth : -cth;
            } else {
                const double r = sqrt(1.0 - dz * dz);
                nx = sth * (dx * dz * cp - dy * sp) / r + dx * cth;
                ny = sth * (dy * dz * cp + dx * sp) / r + dy * cth;
                nz = -sth * cp * r + dz * cth;
            }
            dx = nx;
            dy = ny;
            dz = nz;
            if (e < 1.0) {
                esum += e;
                wx += e * px;
                wy += e * py;
                break;
            }
        }
        if (!(esum >= 350.0)) return false;
        at = (int)floor(wx / esum / m.lt);
        az = m.mode3d ? (int)floor(wy / esum / m.lz) : 0;
        return true;
    }
}

constexpr int kMcBlock = 256;

template <bool SCATTER>
__global__ void __launch_bounds__(kMcBlock) k_table_mc(psf_geometry g, int mode3d, int n_rows, int P, double step_deg,
                                                       long long photons, unsigned long long seed, float* table,
                                                       long long* counts) {
    __shared__ unsigned int cnt[25];
    const long long cell = blockIdx.x;
    if (threadIdx.x < 25) cnt[threadIdx.x] = 0u;
    __syncthreads();
    McCell m;
    m.lt = g.pitch_t;
    m.lz = g.pitch_z;
    m.L = g.depth;
    m.mu = g.mu;
    m.P = P;
    m.mode3d = mode3d;
    int rt, rz;
    if (mode3d) {
        m.pz = (int)(cell % P);
        m.pt = (int)((cell / P) % P);
        rz = (int)((cell / ((long long)P * P)) % n_rows);
        rt = (int)(cell / ((long long)P * P * n_rows));
    } else {
        m.pt = (int)(cell % P);
        m.pz = 0;
        rt = (int)(cell / P);
        rz = 0;
    }
    m.tt = tan(rt * step_deg * kPi / 180.0);
    m.tz = mode3d ? tan(rz * step_deg * kPi / 180.0) : 0.0;
    for (long long k = threadIdx.x; k < photons; k += kMcBlock) {
        Philox rng{(unsigned int)k, (unsigned int)((unsigned long long)k >> 32), (unsigned int)cell, 0u,
                   (unsigned int)seed, (unsigned int)(seed >> 32)};
        int at = 0, az = 0;
        if (!track<SCATTER>(m, rng, at, az)) continue;
        if (at < -2 || at > 2 || az < -2 || az > 2) continue;
        atomicAdd(&cnt[(at + 2) * 5 + az + 2], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 25) {
        const int j = threadIdx.x;
        if (counts) counts[cell * 25 + j] = cnt[j];
        const double f = (double)cnt[j] / (double)photons;
        if (mode3d) table[cell * 25 + j] = (float)f;
        else if (j % 5 == 2) table[cell * 5 + j / 5] = (float)f;  // 2D: the transaxial offsets (a_z = 0)
    }
}

}  // namespace

hipError_t launch_table_mc(const psf_geometry& g, int mode3d, int n_rows, int P, double step_deg, long long photons,
                           unsigned long long seed, int scatter, float* table, long long* counts, hipStream_t st) {
    const long long cells = mode3d ? (long long)n_rows * n_rows * P * P : (long long)n_rows * P;
    if (cells <= 0) return hipSuccess;
    if (scatter)
        hipLaunchKernelGGL(k_table_mc<true>, dim3((unsigned)cells), dim3(kMcBlock), 0, st, g, mode3d, n_rows, P,
                           step_deg, photons, seed, table, counts);
    else
        hipLaunchKernelGGL(k_table_mc<false>, dim3((unsigned)cells), dim3(kMcBlock), 0, st, g, mode3d, n_rows, P,
                           step_deg, photons, seed, table, counts);
    return hipGetLastError();
}

}  // namespace psf
