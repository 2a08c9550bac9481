// 3D scanner (block rings): system matrix and on-the-fly projections.
//
// The paper builds the 2D matrix and names the 3D one as its next step
// (Sec 4); this is that extension of Sec 2.  Voxels go in classes: the voxels
// of one z-column whose z differ by whole ring pitches.  Everything below
// depends on z only through z - z_voxel, so a class computes its tiles once,
// for its reference voxel and ring offsets that reach every member, and each
// member takes them shifted by its own number of rings.
//   K1 transaxial  one workgroup per class.  The 2D homogenization sweep of
//                  Sec 2.3 over the transaxial sub-segments (Eq.11) gives the
//                  line bundles (s1, s2, direction interval), grouped into
//                  crystal pairs (g1, g2).  For the matrix build it also lists
//                  the class's transaxial bins (sorted) and maps each to a slot.
//   K1b rows       the response rows (P^2 x 25 per crystal and relative ring,
//                  Eq.2-7 with the transaxial two-block remap) of every crystal
//                  the class can see, into a table.
//   K2a geometry   one wavefront per (crystal pair, relative ring r1) task.  For
//                  each ring r2 the lines reach: the P^2 x P^2 weights W3
//                  between sub-patches (solid angle of the lines, in closed
//                  form), appended as a tile record (its non-zero blocks).
//   K2b contract   the tile T = U^T (W V) (Eq.10, 12) on matrix cores, U and V
//                  from the table, then
//                  emission for every member: forward atomics, adjoint
//                  gathers, or FP32 atomics into the build's slot x ring-pair
//                  accumulators (a class's members interleaved).
//   K3 compact     ordered compaction of each member's accumulator into CSR rows.
//
// Bins: bin = tbin(g_i, g_j) * NR^2 + r_i * NR + r_j with g_i < g_j (r_i the
// ring of crystal g_i): the transaxial pair major, then the ring pair.
//
// The homogenization weight of the lines from sub-patch (s1, q1) to (s2, q2)
// is (1/2pi) * integral over theta of [S(T_hi) - S(T_lo)]^+, S(T) = T/sqrt(1+T^2)
// the sine of the elevation.  Every slope limit has the form A cos(theta - psi),
// and S(A cos u) has the antiderivative asin(A sin u / sqrt(1 + A^2)); the
// integral is exact once the interval is cut where the binding limits switch
// (roots of p cos theta + q sin theta = 0).
#include <atomic>

#include "common.hpp"

namespace psf {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr double kEpsW3 = 1e-14;  // weights at or below this fraction of the sphere are empty
constexpr int kMaxK = 16;         // P^2 sub-patches per crystal face (P <= 4)

__device__ __forceinline__ double wrap2pi3(double a) {
    while (a >= 2.0 * kPi) a -= 2.0 * kPi;
    while (a < 0.0) a += 2.0 * kPi;
    return a;
}

__device__ __forceinline__ double wrappm3(double a) {
    while (a > kPi) a -= 2.0 * kPi;
    while (a <= -kPi) a += 2.0 * kPi;
    return a;
}

__device__ __forceinline__ double bangle3(const Cyl3D& G, int b, int k, double vx, double vy) {
    const double c = G.frames[2 * b], s = G.frames[2 * b + 1];
    const double xi = -G.half_w + k * (G.lam / G.P);
    return atan2(G.rf * s + xi * c - vy, G.rf * c - xi * s - vx);
}

__device__ __forceinline__ int64_t tbin_of(int64_t gi, int64_t gj, int64_t Nc) {
    return gi * Nc - gi * (gi + 1) / 2 + (gj - gi - 1);
}

// crystal g of a column seen from its image `code` under the square's symmetry
// (bit 2: the mirror y -> -y, c -> nc - 1 - c; bits 0-1: quarter turns, a
// quarter of the ring's crystals each)
// A class's symmetry word: voxels per column and half (bits 0-7), the axial
// mirror half (bit 8), the image codes of columns 1..7 (3 bits each from bit 9;
// column 0 is the reference).  Members go by column, then half, then z: member
// m is voxel s2 = m % nzc of group g = m / nzc, column g (g / 2 with the
// mirror half), half g % 2.  A mirror-half voxel is the axial image (rings
// r -> NR - 1 - r) of reference-half voxel nzc - 1 - s2.
__device__ __forceinline__ int sym_code(int sy, int ci) { return ci ? (sy >> (3 * ci + 6)) & 7 : 0; }

__device__ __forceinline__ int image_crystal(int code, int g, int Nc, int nc) {
    if (code & 4) {
        g = nc - 1 - g;
        if (g < 0) g += Nc;
    }
    g += (code & 3) * (Nc >> 2);
    return g >= Nc ? g - Nc : g;
}

__device__ __forceinline__ void voxel_xyz(const Cyl3D& G, int64_t v, double& x, double& y, double& z) {
    const int64_t ix = v % G.nx, iy = (v / G.nx) % G.ny, iz = v / ((int64_t)G.nx * G.ny);
    x = (ix - 0.5 * (G.nx - 1)) * G.dx + G.cx;
    y = (iy - 0.5 * (G.ny - 1)) * G.dy + G.cy;
    z = (iz - 0.5 * (G.nz - 1)) * G.dz + G.cz;
}

// Sinograms inside the projections are stored ring pair by diagonal: within a
// transaxial bin, (r_i, r_j) goes to the diagonal r_j - r_i (ascending), then
// r_i.  Voxels of a class differ by whole rings, so one tile entry lands on
// consecutive floats for consecutive members.
// 32-bit forms for the emission (bins < 2^31, checked at the entry points)
__device__ __forceinline__ int tbin32(int gi, int gj, int Nc) { return gi * Nc - ((gi * (gi + 1)) >> 1) + (gj - gi - 1); }
__device__ __forceinline__ int diag32(int ri, int rj, int NR) {
    const int d = rj - ri + NR - 1;
    if (d < NR - 1) return ((d * (d + 1)) >> 1) + (ri - (NR - 1 - d));
    const int k = d - (NR - 1);
    return ((NR * (NR - 1)) >> 1) + k * NR - ((k * (k - 1)) >> 1) + ri;
}

// the matrix build's accumulator cell i (an index into S.dense counted in
// cells): add a tile entry, or take the sum (read it, and clear the cell)
__device__ __forceinline__ void acc_add(const Scratch3D& S, int64_t i, float v, int& flag) {
    if (S.det) {
        if (!fix62_ok(v)) flag |= kStatRange;
        atomicAdd((unsigned long long*)S.dense + i, fix62(v));
    } else {
        atomicAdd(S.dense + i, v);
    }
}
__device__ __forceinline__ float acc_take(const Scratch3D& S, int64_t i, bool clear) {
    if (S.det) {
        unsigned long long* p = (unsigned long long*)S.dense + i;
        const unsigned long long q = *p;
        if (clear) *p = 0ull;
        return (float)unfix62(q);
    }
    const float a = S.dense[i];
    if (clear) S.dense[i] = 0.0f;
    return a;
}

__device__ __forceinline__ int64_t diag_index(int ri, int rj, int NR) {
    const int d = rj - ri + NR - 1;
    if (d < NR - 1) return (int64_t)d * (d + 1) / 2 + (ri - (NR - 1 - d));
    const int k = d - (NR - 1);
    return (int64_t)NR * (NR - 1) / 2 + (int64_t)k * NR - (int64_t)k * (k - 1) / 2 + ri;
}

// to_user: user[b] (+)= diag[...]; else diag[...] = user[b].  One workgroup per
// (image, transaxial bin): its NR^2 ring pairs, user order r_i NR + r_j on one
// side, the diagonal order on the other, both inside the bin's NR^2 floats.
__global__ void __launch_bounds__(256) k_diag_perm(const float* src, float* dst, int NR, int to_user, int accumulate) {
    const int nrr = NR * NR;
    const int64_t base = (int64_t)blockIdx.x * nrr;  // blockIdx.x = image * transaxial bins + bin
    for (int rr = threadIdx.x; rr < nrr; rr += blockDim.x) {
        const int ri = rr / NR, rj = rr - ri * NR;
        const int64_t u = base + rr, d = base + diag32(ri, rj, NR);
        if (to_user) dst[u] = accumulate ? dst[u] + src[d] : src[d];
        else dst[d] = src[u];
    }
}

hipError_t launch_diag_perm(const float* src, float* dst, int64_t nbins, int NR, int nb, int to_user, int accumulate,
                            hipStream_t st) {
    const int64_t nrr = (int64_t)NR * NR;
    const int64_t blocks = nbins / nrr * nb;  // the sinogram holds whole transaxial bins of NR^2 ring pairs
    if (blocks <= 0) return hipSuccess;
    if (blocks * nrr != nbins * nb || blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_diag_perm, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, NR, to_user, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// homogenization weight on the sphere, closed form
// ---------------------------------------------------------------------------

struct W3Geo {
    double c1, s1, D1;  // photon 1's face: normal (c1, s1), distance D1 from the voxel
    double c2, s2, D2;  // photon 2's face
};

__host__ __device__ __forceinline__ void cswap(double& a, double& b) {
    const double lo = fmin(a, b), hi = fmax(a, b);
    a = lo;
    b = hi;
}

// one cut of the bundle: where A_i cos(theta - psi_i) = A_j cos(theta - psi_j),
// i.e. p cos(theta) + q sin(theta) = 0, if that falls strictly inside (ta, tb);
// otherwise tb (an empty piece)
__host__ __device__ __forceinline__ double w3_cut(double Ai, double Ci, double Si, double Aj, double Cj, double Sj, double ta,
                                         double tb) {
    const double p = Ai * Ci - Aj * Cj, q = Ai * Si - Aj * Sj;
    if (p == 0.0 && q == 0.0) return tb;
    const double th0 = atan2(-p, q);
    const double r = th0 + rint((0.5 * (ta + tb) - th0) / kPi) * kPi;
    return (r > ta && r < tb) ? r : tb;
}

// asin(A sin(theta - psi) / sqrt(1 + A^2)) at (cos theta, sin theta)
__host__ __device__ __forceinline__ double w3_F(double A, double C, double S, double inv, double ct, double st) {
    return asin(A * (st * C - ct * S) * inv);
}

__host__ __device__ double w3_closed(const W3Geo& g, double zv, double z1lo, double z1hi, double z2lo, double z2hi,
                                     double ta, double tb) {
    // slope limits T_k(theta) = A_k cos(theta - psi_k): 0 T1lo, 1 T1hi (photon 1, psi = its face normal),
    // 2 T2lo, 3 T2hi (photon 2 travels along theta + pi: psi = its face normal + pi)
    const double A0 = (z1lo - zv) / g.D1, A1 = (z1hi - zv) / g.D1;
    const double A2 = (zv - z2hi) / g.D2, A3 = (zv - z2lo) / g.D2;
    const double C1 = g.c1, S1 = g.s1, C2 = -g.c2, S2 = -g.s2;
    // the binding limits switch where T1hi = T2hi, T1lo = T2lo, T1hi = T2lo or T2hi = T1lo
    double r0 = w3_cut(A1, C1, S1, A3, C2, S2, ta, tb);
    double r1 = w3_cut(A0, C1, S1, A2, C2, S2, ta, tb);
    double r2 = w3_cut(A1, C1, S1, A2, C2, S2, ta, tb);
    double r3 = w3_cut(A3, C2, S2, A0, C1, S1, ta, tb);
    cswap(r0, r1);
    cswap(r2, r3);
    cswap(r0, r2);
    cswap(r1, r3);
    cswap(r1, r2);
    const double i0 = 1.0 / sqrt(1.0 + A0 * A0), i1 = 1.0 / sqrt(1.0 + A1 * A1);
    const double i2 = 1.0 / sqrt(1.0 + A2 * A2), i3 = 1.0 / sqrt(1.0 + A3 * A3);
    double sum = 0.0;
    double a = ta, ca = cos(ta), sa = sin(ta);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double b = k == 0 ? r0 : (k == 1 ? r1 : (k == 2 ? r2 : (k == 3 ? r3 : tb)));
        if (b > a) {
            const double m = 0.5 * (a + b), cm = cos(m), sm = sin(m);
            const double T0 = A0 * (cm * C1 + sm * S1), T1 = A1 * (cm * C1 + sm * S1);
            const double T2 = A2 * (cm * C2 + sm * S2), T3 = A3 * (cm * C2 + sm * S2);
            const bool h1 = T1 < T3, l0 = T0 > T2;
            const double Th = h1 ? T1 : T3, Tl = l0 ? T0 : T2;
            const double cb = cos(b), sb = sin(b);
            if (Th > Tl) {
                const double Ah = h1 ? A1 : A3, Ch = h1 ? C1 : C2, Sh = h1 ? S1 : S2, ih = h1 ? i1 : i3;
                const double Al = l0 ? A0 : A2, Cl = l0 ? C1 : C2, Sl = l0 ? S1 : S2, il = l0 ? i0 : i2;
                sum += (w3_F(Ah, Ch, Sh, ih, cb, sb) - w3_F(Ah, Ch, Sh, ih, ca, sa)) -
                       (w3_F(Al, Cl, Sl, il, cb, sb) - w3_F(Al, Cl, Sl, il, ca, sa));
            }
            a = b;
            ca = cb;
            sa = sb;
        }
    }
    return sum / (2.0 * kPi);
}

// The same integral without trigonometric calls, from the unit vectors of the
// bundle's ends.  A point of the bundle (width below a half turn) is the unit
// vector u; its place along the bundle is the key
//   key(u) = sin(theta_u - theta_a)       while cos(theta_u - theta_a) >= 0,
//            2 - sin(theta_u - theta_a)   beyond a quarter turn,
// which grows with the angle from the start.  A switch of the binding limits
// (a root of p cos + q sin, Th = Tl or a swap of the binding limit) lies inside
// when p cos + q sin changes sign strictly between the ends; the root is then
// +-(q, -p)/|(p, q)|, the sign taken so that it lies ahead of the start.  On
// each piece the binding limits are read at the (unnormalised) midpoint
// u_i + u_{i+1}, and each asin difference is taken in one call:
//   asin x_b - asin x_a = asin(x_b y_a - x_a y_b)   when y_a y_b + x_a x_b >= 0,
// with x = A sin(theta - psi)/sqrt(1 + A^2) and y = sqrt(1 - x^2) =
// sqrt(1 + T^2)/sqrt(1 + A^2) (T = A cos(theta - psi), the limit itself).

__host__ __device__ __forceinline__ double w3_key(double ca, double sa, double c, double s) {
    const double sn = ca * s - sa * c, cs = ca * c + sa * s;
    return cs >= 0.0 ? sn : 2.0 - sn;
}

// p, q of switch i: 0 T1hi = T2hi, 1 T1lo = T2lo, 2 T1hi = T2lo, 3 T2hi = T1lo
struct W3Lim {
    double A0, A1, A2, A3, C1, S1, C2, S2;
    __host__ __device__ __forceinline__ void pq(int i, double& p, double& q) const {
        const double Ai = i == 1 ? A0 : (i == 3 ? A3 : A1);
        const double Aj = i == 0 ? A3 : (i == 3 ? A0 : A2);
        const double Ci = i == 3 ? C2 : C1, Si = i == 3 ? S2 : S1;
        const double Cj = i == 3 ? C1 : C2, Sj = i == 3 ? S1 : S2;
        p = Ai * Ci - Aj * Cj;
        q = Ai * Si - Aj * Sj;
    }
};

// the root of p cos + q sin inside the bundle when the sign changes strictly
// between the ends (else key 4: beyond the end)
__host__ __device__ __forceinline__ double w3_cut_key(double p, double q, double ca, double sa, double cb, double sb) {
    const double fa = p * ca + q * sa, fb = p * cb + q * sb;
    if (!((fa < 0.0 && fb > 0.0) || (fa > 0.0 && fb < 0.0))) return 4.0;
    double uc = q, us = -p;  // unnormalised: the key needs the unit vector
    const double inv = 1.0 / sqrt(p * p + q * q);
    uc *= inv;
    us *= inv;
    if (ca * us - sa * uc < 0.0) {
        uc = -uc;
        us = -us;
    }
    return w3_key(ca, sa, uc, us);
}

__host__ __device__ __forceinline__ void w3_cut_uv(double p, double q, double ca, double sa, double& uc, double& us) {
    const double inv = 1.0 / sqrt(p * p + q * q);
    uc = q * inv;
    us = -p * inv;
    if (ca * us - sa * uc < 0.0) {
        uc = -uc;
        us = -us;
    }
}

__host__ __device__ __forceinline__ void kswap(double& ka, int& ia, double& kb, int& ib) {
    const bool sw = kb < ka;
    const double k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const int i0 = sw ? ib : ia, i1 = sw ? ia : ib;
    ka = k0;
    kb = k1;
    ia = i0;
    ib = i1;
}

// asin(x_b) - asin(x_a) for the limit A cos(theta - psi) between the unit vectors a and b
__host__ __device__ __forceinline__ double w3_dF(double A, double C, double S, double inv, double ac, double as_,
                                                 double bc, double bs) {
    const double xa = A * (as_ * C - ac * S) * inv, xb = A * (bs * C - bc * S) * inv;
    const double Ta = A * (ac * C + as_ * S), Tb = A * (bc * C + bs * S);
    const double ya = sqrt(1.0 + Ta * Ta) * inv, yb = sqrt(1.0 + Tb * Tb) * inv;
    const double sd = xb * ya - xa * yb, cd = ya * yb + xa * xb;
    const double r = asin(fmin(1.0, fmax(-1.0, sd)));
    return cd >= 0.0 ? r : (sd >= 0.0 ? kPi - r : -kPi - r);
}

__host__ __device__ double w3_closed_uv(const W3Geo& g, double zv, double z1lo, double z1hi, double z2lo, double z2hi,
                                        double ca, double sa, double cb, double sb) {
    W3Lim L;
    L.A0 = (z1lo - zv) / g.D1;
    L.A1 = (z1hi - zv) / g.D1;
    L.A2 = (zv - z2hi) / g.D2;
    L.A3 = (zv - z2lo) / g.D2;
    L.C1 = g.c1;
    L.S1 = g.s1;
    L.C2 = -g.c2;
    L.S2 = -g.s2;
    double k0, k1, k2, k3;
    {
        double p, q;
        L.pq(0, p, q);
        k0 = w3_cut_key(p, q, ca, sa, cb, sb);
        L.pq(1, p, q);
        k1 = w3_cut_key(p, q, ca, sa, cb, sb);
        L.pq(2, p, q);
        k2 = w3_cut_key(p, q, ca, sa, cb, sb);
        L.pq(3, p, q);
        k3 = w3_cut_key(p, q, ca, sa, cb, sb);
    }
    int j0 = 0, j1 = 1, j2 = 2, j3 = 3;
    kswap(k0, j0, k1, j1);
    kswap(k2, j2, k3, j3);
    kswap(k0, j0, k2, j2);
    kswap(k1, j1, k3, j3);
    kswap(k1, j1, k2, j2);
    const double kend = w3_key(ca, sa, cb, sb);
    const double i0 = 1.0 / sqrt(1.0 + L.A0 * L.A0), i1 = 1.0 / sqrt(1.0 + L.A1 * L.A1);
    const double i2 = 1.0 / sqrt(1.0 + L.A2 * L.A2), i3 = 1.0 / sqrt(1.0 + L.A3 * L.A3);
    double sum = 0.0;
    double akey = 0.0, ac = ca, as_ = sa;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double bkey = k == 0 ? k0 : (k == 1 ? k1 : (k == 2 ? k2 : (k == 3 ? k3 : kend)));
        const int bj = k == 0 ? j0 : (k == 1 ? j1 : (k == 2 ? j2 : j3));
        if (bkey > kend) bkey = kend;
        if (bkey > akey) {
            double bc = cb, bs = sb;
            if (k < 4 && bkey < kend) {
                double p, q;
                L.pq(bj, p, q);
                w3_cut_uv(p, q, ca, sa, bc, bs);
            }
            const double cm = ac + bc, sm = as_ + bs;
            const double T0 = L.A0 * (cm * L.C1 + sm * L.S1), T1 = L.A1 * (cm * L.C1 + sm * L.S1);
            const double T2 = L.A2 * (cm * L.C2 + sm * L.S2), T3 = L.A3 * (cm * L.C2 + sm * L.S2);
            const bool h1 = T1 < T3, l0 = T0 > T2;
            if ((h1 ? T1 : T3) > (l0 ? T0 : T2)) {
                const double Ah = h1 ? L.A1 : L.A3, Ch = h1 ? L.C1 : L.C2, Sh = h1 ? L.S1 : L.S2, ih = h1 ? i1 : i3;
                const double Al = l0 ? L.A0 : L.A2, Cl = l0 ? L.C1 : L.C2, Sl = l0 ? L.S1 : L.S2, il = l0 ? i0 : i2;
                sum += w3_dF(Ah, Ch, Sh, ih, ac, as_, bc, bs) - w3_dF(Al, Cl, Sl, il, ac, as_, bc, bs);
            }
            akey = bkey;
            ac = bc;
            as_ = bs;
        }
    }
    return sum / (2.0 * kPi);
}

// ---------------------------------------------------------------------------
// response row of a sub-patch (3D form of Eq.2-7)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t tab3_idx(int nr, int P, int rt, int rz, int pt, int pz, int at, int az) {
    return (((((int64_t)rt * nr + rz) * P + pt) * P + pz) * kNb + (at + 2)) * kNb + (az + 2);
}

// out[(a_t+2)*5 + (a_z+2)]: response of the crystal at transaxial offset a_t
// and ring r + a_z to a photon entering sub-patch (g, pt; r, pz) from (cx, cy, cz)
// (IDX: the table entry it comes from, -1 for none).  Rings outside the
// scanner are kept here (r may be a relative ring of a class); the emission
// drops them.  Returns 1 when an angle row beyond the table had to be clamped.
template <bool IDX>
__device__ int uv_row3(const Cyl3D& G, double cx, double cy, double cz, int g, int pt, int r, int pz, void* out) {
    int range = 0;
    const int b = g / G.nc, c = g - b * G.nc, P = G.P, nr = G.n_rows;
    const double cs = G.frames[2 * b], sn = G.frames[2 * b + 1];
    const double xi_m = -G.half_w + (c + (pt + 0.5) / P) * G.lam;
    const double z_m = G.z0 + (r + (pz + 0.5) / P) * G.lz;
    const double D = G.rf - (cs * cx + sn * cy);
    const double tan_t = (xi_m - (-sn * cx + cs * cy)) / D;
    const double tan_z = (z_m - cz) / D;
    const double at = atan(tan_t), az = atan(tan_z);
    const bool mt = at < 0.0, mz = az < 0.0;
    const double aat = fabs(at), aaz = fabs(az);
    int row_t = (int)floor(aat * 180.0 / kPi / G.step_deg + 0.5);
    int row_z = (int)floor(aaz * 180.0 / kPi / G.step_deg + 0.5);
    if (row_t > nr - 1) { range = 1; row_t = nr - 1; }
    if (row_z > nr - 1) { range = 1; row_z = nr - 1; }
    const int cm = mt ? G.nc - 1 - c : c;
    const int ptm = mt ? P - 1 - pt : pt;
    const int pzm = mz ? P - 1 - pz : pz;
    const double nu = mt ? xi_m + G.half_w : G.half_w - xi_m;
    bool remap = false;
    int kv = 0, pt1 = 0, pz1 = 0, dr = 0, row_bt = 0, row_bz = 0;
    const double beta = aat - G.two_pi_R;
    if (beta > 0.0 && cm + 2 >= G.nc) {
        const double ca = cos(aat), cb = cos(beta);
        const double ap1 = G.sigma + ca / cb * (G.sigma + nu);
        const double n = ap1 / G.lam;
        kv = (int)ceil(n) - 1;
        pt1 = (int)floor(((kv + 1) - n) * P);
        const double atz = fabs(tan_z);
        const double tzb = atz * ca / cb;
        const double ell = (G.sigma + nu) * G.sin_two_pi_R / cb;
        const double u = (pzm + 0.5) * G.lz / P + ell * atz * ca;
        dr = (int)floor(u / G.lz);
        const double uz1 = u - dr * G.lz;
        pz1 = (int)floor(uz1 * P / G.lz);
        if (pz1 > P - 1) pz1 = P - 1;
        row_bt = (int)floor(beta * 180.0 / kPi / G.step_deg + 0.5);
        row_bz = (int)floor(atan(tzb) * 180.0 / kPi / G.step_deg + 0.5);
        if (row_bt > nr - 1) { range = 1; row_bt = nr - 1; }
        if (row_bz > nr - 1) { range = 1; row_bz = nr - 1; }
        remap = true;
    }
    for (int amt = -2; amt <= 2; ++amt) {
        const int a_t = mt ? -amt : amt, cc = cm + amt;
        for (int amz = -2; amz <= 2; ++amz) {
            const int a_z = mz ? -amz : amz;
            int64_t ti = -1;
            if (cc >= 0 && cc < G.nc) {
                ti = tab3_idx(nr, P, row_t, row_z, ptm, pzm, amt, amz);
            } else if (cc >= G.nc && remap) {
                const int idx = kv + 1 + (cc - G.nc), az1 = amz - dr;
                if (idx <= 2 && az1 >= -2 && az1 <= 2) ti = tab3_idx(nr, P, row_bt, row_bz, pt1, pz1, idx, az1);
            }
            const int pos = (a_t + 2) * kNb + (a_z + 2);
            if (IDX) ((int*)out)[pos] = (int)ti;
            else ((float*)out)[pos] = ti >= 0 ? G.table[ti] : 0.0f;
        }
    }
    return range;
}

// ---------------------------------------------------------------------------
// K1: transaxial sweep, crystal pairs, transaxial bins
// ---------------------------------------------------------------------------

constexpr int kBlockT = 512;

// a class that gives up: none of its columns has slots
__device__ void clear_slot_counts(const Scratch3D& S, const Args3D& A, int cb) {
    if (!S.n_slots) return;
    const int4 c = A.cls[cb];
    const int nzc = A.sym[cb] & 0xff;
    for (int i = 0; i < c.z; i += nzc) S.n_slots[c.y + i] = 0;
}

// The build's slot numbering keeps a bitmap of the transaxial bins and a word
// prefix in the kernel's dynamic LDS (over the spent sweep arrays) when they
// fit in kSlotBitsMax bytes; else it scans the slot map in global memory.
constexpr size_t kSlotBitsMax = 48 * 1024;
__host__ __device__ inline size_t slot_bitmap_bytes(const Cyl3D& G) {
    const size_t b = 2 * sizeof(unsigned int) * (size_t)((G.ntbins + 31) / 32);
    return b <= kSlotBitsMax ? b : 0;
}

__global__ void __launch_bounds__(kBlockT) k_cyl3d_transaxial(Cyl3D G, Scratch3D S, Args3D A, int want_slots) {
    extern __shared__ __align__(16) unsigned char smem3[];
    const int tid = threadIdx.x, bs = blockDim.x;
    const int vb = blockIdx.x;  // class of the batch
    const int64_t v = A.cls[vb].x;
    const int M1 = G.nc * G.P + 1, spb = G.nc * G.P;
    if (vb == 0 && tid == 0) {  // the batch's tile records start empty, and so does the geometry's unit queue
        S.rec_count[0] = 0u;
        S.rec_count[1] = 0u;
    }
    double* th = (double*)smem3;                    // [R * M1]
    double* unw = th + G.R * M1;                    // [nseg]
    int* cnt = (int*)(unw + G.nseg);                // [nseg + 1]
    __shared__ int red[kBlockT / 64 + 1];
    __shared__ int s_total;
    double vx, vy, vz;
    voxel_xyz(G, v, vx, vy, vz);
    for (int i = tid; i < G.R * M1; i += bs) {
        const int b = i / M1, k = i - b * M1;
        th[i] = bangle3(G, b, k, vx, vy);
    }
    __syncthreads();
    const double lo0 = th[0];
    for (int s = tid; s < G.nseg; s += bs) {
        const int b = s / spb, k = s - b * spb;
        unw[s] = lo0 + wrap2pi3(th[b * M1 + k] - lo0);
    }
    __syncthreads();
    int* sidx = S.sidx + (int64_t)vb * S.cap_samples;
    double* sth = S.sth + (int64_t)vb * S.cap_samples * 2;
    // two passes over the sweep: count the bundles of each s1, then write them
    // in (s1, s2) order at the scanned offsets
    for (int pass = 0; pass < 2; ++pass) {
        for (int s1 = tid; s1 < G.nseg; s1 += bs) {
            const int b1 = s1 / spb, k1 = s1 - b1 * spb;
            const double lo1 = th[b1 * M1 + k1];
            const double len1 = wrap2pi3(th[b1 * M1 + k1 + 1] - lo1);
            double x = unw[s1] + kPi;
            if (x >= lo0 + 2.0 * kPi) x -= 2.0 * kPi;
            int lo = 0, hi = G.nseg;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (unw[mid] <= x) lo = mid + 1;
                else hi = mid;
            }
            const int j0 = lo > 0 ? lo - 1 : 0;
            int n = 0, out = pass ? cnt[s1] : 0;
            for (int c = 0; c < G.nseg; ++c) {
                const int jj = j0 + c;
                const int s2 = jj >= G.nseg ? jj - G.nseg : jj;
                const double base = unw[s2] + (jj >= G.nseg ? 2.0 * kPi : 0.0);
                if (c > 0 && base >= x + len1) break;
                if (s2 <= s1) continue;
                const int b2 = s2 / spb, k2 = s2 - b2 * spb;
                const double lo2 = th[b2 * M1 + k2];
                const double len2 = wrap2pi3(th[b2 * M1 + k2 + 1] - lo2);
                const double d = wrappm3(lo2 + kPi - lo1);
                const double ov = fmin(len1, d + len2) - fmax(0.0, d);
                if (!(ov > kEpsOverlap)) continue;
                if (pass && out < S.cap_samples) {
                    sidx[out] = (s1 << 16) | s2;
                    sth[2 * out] = lo1 + fmax(0.0, d);
                    sth[2 * out + 1] = lo1 + fmin(len1, d + len2);
                }
                ++n;
                ++out;
            }
            if (!pass) cnt[s1] = n;
        }
        __syncthreads();
        if (!pass) {  // exclusive scan of cnt (serial over chunks of the block)
            if (tid == 0) {
                int run = 0;
                for (int s = 0; s < G.nseg; ++s) {
                    const int c = cnt[s];
                    cnt[s] = run;
                    run += c;
                }
                cnt[G.nseg] = run;
                s_total = run;
            }
            __syncthreads();
        }
    }
    const int ns = s_total;
    if (ns > S.cap_samples) {
        if (tid == 0) atomicOr(A.status, kStatScratch);
        if (tid == 0) { S.n_samples[vb] = 0; S.n_pairs[vb] = 0; clear_slot_counts(S, A, vb); }
        return;
    }
    // group each g1's bundles by g2 (insertion sort of <= P * few entries)
    for (int g1 = tid; g1 < G.Nc; g1 += bs) {
        const int a = cnt[g1 * G.P], e = cnt[g1 * G.P + G.P];
        for (int i = a + 1; i < e; ++i) {
            const int key = sidx[i];
            const double t0 = sth[2 * i], t1 = sth[2 * i + 1];
            const int k2 = (key & 0xffff) / G.P;
            int j = i - 1;
            while (j >= a && (sidx[j] & 0xffff) / G.P > k2) {
                sidx[j + 1] = sidx[j];
                sth[2 * (j + 1)] = sth[2 * j];
                sth[2 * (j + 1) + 1] = sth[2 * j + 1];
                --j;
            }
            sidx[j + 1] = key;
            sth[2 * (j + 1)] = t0;
            sth[2 * (j + 1) + 1] = t1;
        }
    }
    __syncthreads();
    // pairs: runs of equal (g1, g2).  Count per g1, scan, write.
    int4* pairs = S.pairs + (int64_t)vb * S.cap_pairs;
    int* pc = cnt;  // reuse: per-g1 pair counts live past the sample offsets
    __syncthreads();
    __shared__ int s_np;
    // count
    int* gcnt = (int*)(unw);  // unw is free now: [Nc] ints
    for (int g1 = tid; g1 < G.Nc; g1 += bs) {
        const int a = pc[g1 * G.P], e = pc[g1 * G.P + G.P];
        int n = 0, last = -1;
        for (int i = a; i < e; ++i) {
            const int g2 = (sidx[i] & 0xffff) / G.P;
            if (g2 != last) { ++n; last = g2; }
        }
        gcnt[g1] = n;
    }
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int g = 0; g < G.Nc; ++g) {
            const int c = gcnt[g];
            gcnt[g] = run;
            run += c;
        }
        s_np = run;
    }
    __syncthreads();
    const int np = s_np;
    if (np > S.cap_pairs) {
        if (tid == 0) { atomicOr(A.status, kStatScratch); S.n_samples[vb] = 0; S.n_pairs[vb] = 0; clear_slot_counts(S, A, vb); }
        return;
    }
    for (int g1 = tid; g1 < G.Nc; g1 += bs) {
        const int a = pc[g1 * G.P], e = pc[g1 * G.P + G.P];
        int o = gcnt[g1], last = -1, first = a;
        for (int i = a; i <= e; ++i) {
            const int g2 = i < e ? (sidx[i] & 0xffff) / G.P : -2;
            if (g2 != last) {
                if (last >= 0) pairs[o++] = make_int4(g1, last, first, i - first);
                last = g2;
                first = i;
            }
        }
    }
    if (tid == 0) {
        S.n_samples[vb] = ns;
        S.n_pairs[vb] = np;
    }
    if (!want_slots) return;
    // the reference column's transaxial bins: mark, then scan in bin order into
    // slots (group cl.y, the member index of its first voxel).  The class's other
    // columns take their bins from these (k_image_slots).
    const int grp = A.cls[vb].y;
    __shared__ int s_run;
    const int lane = tid & 63, wid = tid >> 6, nw = bs >> 6;
    int* smap = S.slotmap + (int64_t)grp * G.ntbins;
    if (slot_bitmap_bytes(G) > 0) {
        // marks as bits in LDS (the sweep arrays are spent), a prefix count per
        // word, then every bin's slot (or -1) written with consecutive threads
        // on consecutive bins
        const int nwd = (int)((G.ntbins + 31) / 32);
        unsigned int* bits = (unsigned int*)smem3;
        int* wpre = (int*)(bits + nwd);
        __syncthreads();
        for (int w = tid; w < nwd; w += bs) bits[w] = 0u;
        __syncthreads();
        for (int p = tid; p < np; p += bs) {
            const int4 pr = pairs[p];
            for (int at = -2; at <= 2; ++at)
                for (int bt = -2; bt <= 2; ++bt) {
                    int gi = pr.x + at, gj = pr.y + bt;
                    gi = gi < 0 ? gi + G.Nc : (gi >= G.Nc ? gi - G.Nc : gi);
                    gj = gj < 0 ? gj + G.Nc : (gj >= G.Nc ? gj - G.Nc : gj);
                    if (gi == gj) continue;
                    const int64_t tb = tbin_of(gi < gj ? gi : gj, gi < gj ? gj : gi, G.Nc);
                    atomicOr(&bits[tb >> 5], 1u << (tb & 31));
                }
        }
        __syncthreads();
        // words in contiguous runs per thread: counts, one block scan, prefixes
        const int per = (nwd + bs - 1) / bs, w0 = tid * per, w1 = w0 + per < nwd ? w0 + per : nwd;
        int mine = 0;
        for (int w = w0; w < w1; ++w) mine += __popc(bits[w]);
        int inc = mine;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) red[wid] = inc;
        __syncthreads();
        int run = inc - mine;
        for (int w = 0; w < wid; ++w) run += red[w];
        if (tid == 0) {
            int all = 0;
            for (int w = 0; w < nw; ++w) all += red[w];
            s_run = all;
        }
        for (int w = w0; w < w1; ++w) {
            wpre[w] = run;
            run += __popc(bits[w]);
        }
        __syncthreads();
        int* stb = S.slot_tbin + (int64_t)grp * S.cap_slots;
        for (int64_t i = tid; i < G.ntbins; i += bs) {
            const unsigned int word = bits[i >> 5], bit = 1u << (i & 31);
            int sl = -1;
            if (word & bit) {
                const int k = wpre[i >> 5] + __popc(word & (bit - 1u));
                if (k < S.cap_slots) {
                    sl = k;
                    stb[k] = (int)i;
                }
            }
            smap[i] = sl;
        }
        __syncthreads();
        if (tid == 0) {
            const int nsl = s_run;
            if (nsl > S.cap_slots) atomicOr(A.status, kStatScratch);
            S.n_slots[grp] = nsl < S.cap_slots ? nsl : S.cap_slots;
        }
        return;
    }
    for (int64_t i = tid; i < G.ntbins; i += bs) smap[i] = 0;
    __syncthreads();
    for (int p = tid; p < np; p += bs) {
        const int4 pr = pairs[p];
        for (int at = -2; at <= 2; ++at)
            for (int bt = -2; bt <= 2; ++bt) {
                int gi = pr.x + at, gj = pr.y + bt;
                gi = gi < 0 ? gi + G.Nc : (gi >= G.Nc ? gi - G.Nc : gi);
                gj = gj < 0 ? gj + G.Nc : (gj >= G.Nc ? gj - G.Nc : gj);
                if (gi == gj) continue;
                const int lo_ = gi < gj ? gi : gj, hi_ = gi < gj ? gj : gi;
                smap[tbin_of(lo_, hi_, G.Nc)] = 1;
            }
    }
    __syncthreads();
    // the marks numbered in bin order: each thread counts a contiguous range,
    // one block-wide exclusive scan of the counts, then each thread numbers its range
    int* stb = S.slot_tbin + (int64_t)grp * S.cap_slots;
    const int64_t per = (G.ntbins + bs - 1) / bs, i0 = tid * per, i1 = i0 + per < G.ntbins ? i0 + per : G.ntbins;
    int mine = 0;
    for (int64_t i = i0; i < i1; ++i) mine += smap[i] != 0;
    int inc = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) red[wid] = inc;
    __syncthreads();
    int slot = inc - mine;
    for (int w = 0; w < wid; ++w) slot += red[w];
    if (tid == 0) {
        int all = 0;
        for (int w = 0; w < nw; ++w) all += red[w];
        s_run = all;
    }
    for (int64_t i = i0; i < i1; ++i) {
        if (smap[i]) {
            smap[i] = slot < S.cap_slots ? slot : -1;
            if (slot < S.cap_slots) stb[slot] = (int)i;
            ++slot;
        } else {
            smap[i] = -1;
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int nsl = s_run;
        if (nsl > S.cap_slots) atomicOr(A.status, kStatScratch);
        S.n_slots[grp] = nsl < S.cap_slots ? nsl : S.cap_slots;
    }
}

// The build's slots of each group (column and half) of a class: the reference
// column's bins (in K1's order) seen through the column's image code, sorted.
// slot_order of the group lists, in bin order, the reference slot of each bin,
// with bit 30 set when the image swaps the photon order (then its ring pair is
// the reference's transposed); slot_tbin the bins.  One workgroup per group
// (member blocks of index 0); the reference column's groups get the identity.
constexpr int kSortSlots = 4096;  // the build's slot capacity at most
__global__ void __launch_bounds__(512) k_image_slots(Cyl3D G, Scratch3D S, Args3D A) {
    __shared__ unsigned long long kv[kSortSlots];
    const int grp = blockIdx.x, tid = threadIdx.x, bs = blockDim.x;
    const int4 me = A.mem[grp];
    if (me.y != 0) return;
    const int4 cl = A.cls[me.z];
    const int sy = A.sym[me.z], nzc = sy & 0xff, g = (grp - cl.y) / nzc;
    const int ci = (sy & 0x100) ? g >> 1 : g, code = sym_code(sy, ci);
    const int n = S.n_slots[cl.y];
    int* order = S.slot_order + (int64_t)grp * S.cap_slots;
    const int* rtb = S.slot_tbin + (int64_t)cl.y * S.cap_slots;
    if (ci == 0) {  // the reference column (its mirror half takes its bins too)
        int* stb = S.slot_tbin + (int64_t)grp * S.cap_slots;
        for (int k = tid; k < n; k += bs) {
            order[k] = k;
            if (g != 0) stb[k] = rtb[k];
        }
        if (tid == 0 && g != 0) S.n_slots[grp] = n;
        return;
    }
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int k = tid; k < np2; k += bs) {
        unsigned long long v = ~0ull;
        if (k < n) {
            // the crystals of bin t: g_i = the last row start <= t, g_j from the offset
            const int64_t t = rtb[k], N2 = 2 * (int64_t)G.Nc - 1;
            int64_t gi = (int64_t)floor(0.5 * ((double)N2 - sqrt((double)(N2 * N2 - 8 * t))));
            gi = gi < 0 ? 0 : (gi > G.Nc - 2 ? G.Nc - 2 : gi);
            while (gi > 0 && tbin_of(gi, gi + 1, G.Nc) > t) --gi;
            while (gi < G.Nc - 2 && tbin_of(gi + 1, gi + 2, G.Nc) <= t) ++gi;
            const int gj = (int)(t - tbin_of(gi, gi + 1, G.Nc)) + (int)gi + 1;
            const int a = image_crystal(code, (int)gi, G.Nc, G.nc), b = image_crystal(code, gj, G.Nc, G.nc);
            const int64_t t2 = a < b ? tbin_of(a, b, G.Nc) : tbin_of(b, a, G.Nc);
            v = ((unsigned long long)t2 << 32) | (unsigned)(k | (a > b ? 0x40000000 : 0));
        }
        kv[k] = v;
    }
    __syncthreads();
    // bitonic sort, ascending
    for (int k2 = 2; k2 <= np2; k2 <<= 1)
        for (int j = k2 >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < np2; i += bs) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long x = kv[i], y = kv[l];
                    if ((x > y) == ((i & k2) == 0)) {
                        kv[i] = y;
                        kv[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    int* stb = S.slot_tbin + (int64_t)grp * S.cap_slots;
    for (int k = tid; k < n; k += bs) {
        order[k] = (int)(kv[k] & 0xffffffffu);
        stb[k] = (int)(kv[k] >> 32);
    }
    if (tid == 0) S.n_slots[grp] = n;
}

hipError_t launch_image_slots(const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st) {
    if (a.n_mem <= 0) return hipSuccess;
    if (S.cap_slots > kSortSlots) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_image_slots, dim3(a.n_mem), dim3(512), 0, st, G, S, a);
    return hipGetLastError();
}

size_t cyl3d_transaxial_smem(const Cyl3D& G) {
    const size_t sweep = sizeof(double) * (size_t)(G.R * (G.nc * G.P + 1) + G.nseg) + sizeof(int) * (size_t)(G.nseg + 1) + 64;
    const size_t bits = slot_bitmap_bytes(G);
    return bits > sweep ? bits : sweep;
}

hipError_t launch_cyl3d_transaxial(const Cyl3D& G, const Scratch3D& S, const Args3D& a, int want_slots,
                                   hipStream_t st) {
    if (a.n_cls <= 0) return hipSuccess;
    const size_t smem = cyl3d_transaxial_smem(G);
    hipFuncSetAttribute((const void*)k_cyl3d_transaxial, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    hipLaunchKernelGGL(k_cyl3d_transaxial, dim3(a.n_cls), dim3(kBlockT), smem, st, G, S, a, want_slots);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K1b: response-row table
// ---------------------------------------------------------------------------
// One thread per row (crystal g, relative ring r, sub-patch pt * P + pz) from
// the class's reference voxel; rows are staged in LDS and stored coalesced.
// Rows beyond P^2 are zero.  uvmask gets a bit for every row whose angle row
// had to be clamped.

constexpr int kUvBlock = 256;  // rows per workgroup: 16 (crystal, ring) slots

__global__ void __launch_bounds__(kUvBlock) k_cyl3d_uvtab(Cyl3D G, Scratch3D S, Args3D A, int64_t n_slots) {
    __shared__ float rows[kUvBlock * 25];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t slot0 = (int64_t)blockIdx.x * (kUvBlock / 16);
    const int64_t slot = slot0 + tid / 16;
    const int row = tid & 15;
    float* out = rows + tid * 25;
    int rng = 0;
    if (slot < n_slots) {
        // the class whose slots hold this one
        int lo = 0, hi = A.n_cls - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.uvoff[mid] <= slot) lo = mid;
            else hi = mid - 1;
        }
        const int4 cl = A.cls[lo];
        const int nr1 = G.NR + cl.w;
        const int64_t rel = slot - A.uvoff[lo];
        const int g = (int)(rel / nr1), r = (int)(rel - (int64_t)g * nr1) - cl.w;
        if (row < G.P * G.P) {
            double vx, vy, vz;
            voxel_xyz(G, cl.x, vx, vy, vz);
            rng = uv_row3<false>(G, vx, vy, vz, g, row / G.P, r, row % G.P, out);
        } else {
            for (int q = 0; q < 25; ++q) out[q] = 0.0f;
        }
    }
    const unsigned long long b = __ballot(rng != 0);
    if (row == 0 && slot < n_slots) S.uvmask[slot] = (int)((b >> (lane & 48)) & 0xffffull);
    __syncthreads();
    const int64_t left = (n_slots - slot0) * 400;
    const int nflt = (int)(left < (int64_t)kUvBlock * 25 ? left : (int64_t)kUvBlock * 25);
    float* dst = S.uvtab + slot0 * 400;
    for (int e = tid; e < nflt; e += kUvBlock) dst[e] = rows[e];
}

hipError_t launch_cyl3d_uvtab(const Cyl3D& G, const Scratch3D& S, const Args3D& a, int64_t n_slots, hipStream_t st) {
    if (a.n_cls <= 0 || n_slots <= 0) return hipSuccess;
    if (n_slots > S.cap_uv) return hipErrorInvalidValue;
    const int64_t blocks = (n_slots + kUvBlock / 16 - 1) / (kUvBlock / 16);
    hipLaunchKernelGGL(k_cyl3d_uvtab, dim3((unsigned)blocks), dim3(kUvBlock), 0, st, G, S, a, n_slots);
    return hipGetLastError();
}

// Table gradient: each (slot, row) recomputes the table entries its 25 values
// came from and adds the row's accumulated gradient into them (FP64 atomics),
// then clears the accumulator for the next batch.
__global__ void __launch_bounds__(kUvBlock) k_cyl3d_uvgrad(Cyl3D G, Scratch3D S, Args3D A, int64_t n_slots) {
    __shared__ int idx[kUvBlock * 25];
    const int tid = threadIdx.x;
    const int64_t slot = (int64_t)blockIdx.x * (kUvBlock / 16) + tid / 16;
    const int row = tid & 15;
    int* out = idx + tid * 25;
    if (slot >= n_slots) return;
    double* gr = S.uvgrad + (slot * 16 + row) * 25;
    if (row >= G.P * G.P) return;
    bool any = false;
    for (int c = 0; c < 25; ++c) any |= gr[c] != 0.0;
    if (!any) return;  // no tile of the batch reached this row
    int lo = 0, hi = A.n_cls - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.uvoff[mid] <= slot) lo = mid;
        else hi = mid - 1;
    }
    const int4 cl = A.cls[lo];
    const int nr1 = G.NR + cl.w;
    const int64_t rel = slot - A.uvoff[lo];
    const int g = (int)(rel / nr1), r = (int)(rel - (int64_t)g * nr1) - cl.w;
    double vx, vy, vz;
    voxel_xyz(G, cl.x, vx, vy, vz);
    uv_row3<true>(G, vx, vy, vz, g, row / G.P, r, row % G.P, out);
    for (int c = 0; c < 25; ++c) {
        const double v = gr[c];
        if (v == 0.0) continue;
        if (out[c] >= 0) atomicAdd(&A.g64[(int64_t)(blockIdx.x % kGradRep) * A.g64_n + out[c]], v);
        gr[c] = 0.0;
    }
}

// p[i] += p[r * n + i] for r = 1 .. reps - 1
__global__ void k_sum_copies(double* p, int64_t n, int reps) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = p[i];
        for (int r = 1; r < reps; ++r) v += p[r * n + i];
        p[i] = v;
    }
}

hipError_t launch_sum_copies(double* p, int64_t n, int reps, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_sum_copies, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, p, n, reps);
    return hipGetLastError();
}

hipError_t launch_cyl3d_uvgrad(const Cyl3D& G, const Scratch3D& S, const Args3D& a, int64_t n_slots, hipStream_t st) {
    if (a.n_cls <= 0 || n_slots <= 0) return hipSuccess;
    if (n_slots > S.cap_uv || !S.uvgrad || !a.g64) return hipErrorInvalidValue;
    const int64_t blocks = (n_slots + kUvBlock / 16 - 1) / (kUvBlock / 16);
    hipLaunchKernelGGL(k_cyl3d_uvgrad, dim3((unsigned)blocks), dim3(kUvBlock), 0, st, G, S, a, n_slots);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K2a: tile geometry (FP64) -> tile records
// ---------------------------------------------------------------------------
// One wavefront per (crystal pair, run of rings r1) unit, r1 relative to the class's
// reference voxel and ranging over [-s_max, NR - 1] (s_max the largest member
// shift), so that every member's rings are covered.  For every ring r2 the
// lines reach, and that some member sees with both rings inside the scanner,
// it computes the P^2 x P^2 weights W, one P x P block per line bundle
// (sample), and when any is non-zero appends the record (header and the
// blocks) for the contraction kernel.  The units come from one queue: each
// wavefront takes the batch's next unit (classes in order) from a device
// counter until none is left, so that classes and units of unequal cost even
// out over the kGeomWG workgroups.
// Each wavefront takes record slots kSlotChunk at a time from the shared
// counter and marks the ones it leaves unused empty (no samples).

constexpr int kWavesT = 4;
constexpr int kGeomWG = 1024;
constexpr unsigned int kSlotChunk = 16;
constexpr int kR2Chunk = 8;  // rings r2 handled together
constexpr int kR1Run = 16;   // consecutive rings r1 of one crystal pair per work unit
constexpr int kQueue = 128;  // candidate queue (a power of two >= 127)

// Most candidates (r2, sample, pz1, pz2) fail the quick test; the survivors
// are queued in LDS and the closed form runs on full wavefronts.
struct WaveLds {
    float Wr[kR2Chunk][kMaxK][16];  // ring r2c + j, sample k: weights between pz1 * P + pz2
    int q[kQueue];
    unsigned char cks[kR2Chunk * kMaxK];  // (ring, sample) pairs that pass the whole-face test
    unsigned char alive[kR2Chunk * kMaxK];  // by j * nsmp + k: whether the pair passed
    double ta[kMaxK], tb[kMaxK];
    double ca[kMaxK], sa[kMaxK], cb[kMaxK], sb[kMaxK];  // unit vectors of the bundle's ends
    double c1lo[kMaxK], c1hi[kMaxK], c2lo[kMaxK], c2hi[kMaxK];  // cos(theta - psi) ranges over the bundle
    int pt1[kMaxK], pt2[kMaxK];
};

__device__ __forceinline__ float bf16r(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// two waves per SIMD: the FP64 geometry needs ~256 registers
template <int P>
__global__ void __launch_bounds__(64 * kWavesT) __attribute__((amdgpu_waves_per_eu(2)))
k_cyl3d_geom(Cyl3D G, Scratch3D S, Args3D A) {
    constexpr int K = P * P;
    __shared__ WaveLds wl[kWavesT];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    WaveLds& L = wl[wid];
    int flag = 0;
    unsigned int slot_next = 0, slot_end = 0;  // this wave's reserved record slots
    unsigned long long n_tiles = 0;
    for (;;) {
        // the next unit of the batch: classes in order, each np * nrun units
        unsigned int next = 0;
        if (lane == 0) next = atomicAdd(S.rec_count + 1, 1u);
        int u = __builtin_amdgcn_readfirstlane(__shfl(next, 0, 64));
        int vb = 0;
        for (; vb < A.n_cls; ++vb) {
            const int nu = S.n_pairs[vb] * ((G.NR + A.cls[vb].w + kR1Run - 1) / kR1Run);
            if (u < nu) break;
            u -= nu;
        }
        if (vb >= A.n_cls) break;  // every unit is taken
        const int4 cl = A.cls[vb];
        const int smax = cl.w;
        const int nr1 = G.NR + smax;
        const int nrun = (nr1 + kR1Run - 1) / kR1Run;
        const int4* pairs = S.pairs + (int64_t)vb * S.cap_pairs;
        const int* sidx = S.sidx + (int64_t)vb * S.cap_samples;
        const double* sth = S.sth + (int64_t)vb * S.cap_samples * 2;
        const int* umask = S.uvmask + A.uvoff[vb];
        double vx, vy, vz;
        voxel_xyz(G, cl.x, vx, vy, vz);
        const int pi = u / nrun;
        const int r1a = (u - pi * nrun) * kR1Run - smax, r1e = min(r1a + kR1Run, G.NR);
        const int4 pr = pairs[pi];
        const int g1 = pr.x, g2 = pr.y, nsmp = pr.w;
        if (nsmp > kMaxK) { flag |= kStatScratch; continue; }
        if (lane < nsmp) {
            const int key = sidx[pr.z + lane];
            L.pt1[lane] = (key >> 16) - g1 * P;
            L.pt2[lane] = (key & 0xffff) - g2 * P;
            L.ta[lane] = sth[2 * (pr.z + lane)];
            L.tb[lane] = sth[2 * (pr.z + lane) + 1];
        }
        __builtin_amdgcn_wave_barrier();
        const int b1 = g1 / G.nc, b2 = g2 / G.nc;
        W3Geo wg;
        wg.c1 = G.frames[2 * b1];
        wg.s1 = G.frames[2 * b1 + 1];
        wg.c2 = G.frames[2 * b2];
        wg.s2 = G.frames[2 * b2 + 1];
        wg.D1 = G.rf - (wg.c1 * vx + wg.s1 * vy);
        wg.D2 = G.rf - (wg.c2 * vx + wg.s2 * vy);
        // range of cos(theta - psi) over each bundle, for both faces: the slope
        // limits A cos(theta - psi) then lie within A times that range
        if (lane < nsmp) {
            const double ca = cos(L.ta[lane]), sa = sin(L.ta[lane]), cb = cos(L.tb[lane]), sb = sin(L.tb[lane]);
            L.ca[lane] = ca;
            L.sa[lane] = sa;
            L.cb[lane] = cb;
            L.sb[lane] = sb;
            const double u1a = ca * wg.c1 + sa * wg.s1, u1b = cb * wg.c1 + sb * wg.s1;
            const double u2a = -(ca * wg.c2 + sa * wg.s2), u2b = -(cb * wg.c2 + sb * wg.s2);
            // the maximum 1 is reached inside when the face normal direction lies in the bundle
            const double m1 = wrap2pi3(atan2(wg.s1, wg.c1) - L.ta[lane]);
            const double m2 = wrap2pi3(atan2(-wg.s2, -wg.c2) - L.ta[lane]);
            const double wdt = L.tb[lane] - L.ta[lane];
            L.c1lo[lane] = fmin(u1a, u1b);
            L.c1hi[lane] = m1 <= wdt ? 1.0 : fmax(u1a, u1b);
            L.c2lo[lane] = fmin(u2a, u2b);
            L.c2hi[lane] = m2 <= wdt ? 1.0 : fmax(u2a, u2b);
        }
        // photon 2 lands at zv - ratio (z1 - zv): the range of the ratio over the
        // bundles' ends (lanes < nsmp), then over the lanes
        double rmin = 1e300, rmax = -1e300;
        if (lane < nsmp) {
            for (int e = 0; e < 2; ++e) {
                const double ct = e ? L.cb[lane] : L.ca[lane], st = e ? L.sb[lane] : L.sa[lane];
                const double ratio = (wg.D2 / wg.D1) * (ct * wg.c1 + st * wg.s1) / -(ct * wg.c2 + st * wg.s2);
                rmin = fmin(rmin, ratio);
                rmax = fmax(rmax, ratio);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rmin = fmin(rmin, __shfl_xor(rmin, off, 64));
            rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
        }
        const double invD1 = 1.0 / wg.D1, invD2 = 1.0 / wg.D2;
        const int smag = (65536 + nsmp - 1) / nsmp;  // c / nsmp == (c * smag) >> 16 for c < 4096
        __builtin_amdgcn_wave_barrier();
        for (int r1 = r1a; r1 < r1e; ++r1) {
        // rings r2 reached from ring r1
        double zmin = 1e300, zmax = -1e300;
        for (int f = 0; f < 2; ++f) {
            const double z1 = G.z0 + (r1 + f) * G.lz;
            for (int e = 0; e < 2; ++e) {
                const double z2 = vz - (e ? rmax : rmin) * (z1 - vz);
                zmin = fmin(zmin, z2);
                zmax = fmax(zmax, z2);
            }
        }
        int r2a = (int)floor((zmin - G.z0) / G.lz) - 1, r2b = (int)floor((zmax - G.z0) / G.lz) + 1;
        r2a = r2a < -smax ? -smax : r2a;
        r2b = r2b > G.NR - 1 ? G.NR - 1 : r2b;
        for (int r2c = r2a; r2c <= r2b; r2c += kR2Chunk) {
            const int nj = min(kR2Chunk, r2b - r2c + 1);
            // rings of the chunk that some member sees with both rings inside the scanner
            unsigned int jok = 0u;
            for (int j = 0; j < nj; ++j) {
                const int r2 = r2c + j;
                const int slo = max(0, max(-r1, -r2)), shi = min(smax, min(G.NR - 1 - r1, G.NR - 1 - r2));
                if (slo <= shi) jok |= 1u << j;
            }
            if (!jok) continue;
            unsigned int jm = 0u;  // rings whose tile got a weight (this lane's share)
            int head = 0, tail = 0;
            // The quick test below, on the whole crystal faces of ring r1 and r2
            // (the extreme sub-patches' own bounds, so the same rounding): its
            // slope bounds grow with the face's z range when the direction cosines
            // are positive, so a (ring, sample) pair that fails it fails for every
            // pair of sub-patches and is dropped at once.
            int nsurv = 0;
            for (int c0 = 0; c0 < nj * nsmp; c0 += 64) {
                const int c = c0 + lane;
                bool pass = false;
                if (c < nj * nsmp) {
                    const int j = (c * smag) >> 16, k = c - j * nsmp;
                    if ((jok >> j) & 1u) {
                        pass = true;
                        if (L.c1lo[k] > 0.0 && L.c2lo[k] > 0.0) {
                            const int r2 = r2c + j;
                            const double z1lo = G.z0 + (r1 + 0.0) * G.lz, z1hi = G.z0 + (r1 + 1.0) * G.lz;
                            const double z2lo = G.z0 + (r2 + 0.0) * G.lz, z2hi = G.z0 + (r2 + 1.0) * G.lz;
                            const double a1lo = (z1lo - vz) * invD1, a1hi = (z1hi - vz) * invD1;
                            const double a2lo = (vz - z2hi) * invD2, a2hi = (vz - z2lo) * invD2;
                            const double t1hi_max = a1hi * (a1hi >= 0.0 ? L.c1hi[k] : L.c1lo[k]);
                            const double t1lo_min = a1lo * (a1lo >= 0.0 ? L.c1lo[k] : L.c1hi[k]);
                            const double t2hi_max = a2hi * (a2hi >= 0.0 ? L.c2hi[k] : L.c2lo[k]);
                            const double t2lo_min = a2lo * (a2lo >= 0.0 ? L.c2lo[k] : L.c2hi[k]);
                            pass = !(t1hi_max <= t2lo_min || t2hi_max <= t1lo_min);
                        }
                    }
                }
                const unsigned long long bal = __ballot(pass);
                if (pass) L.cks[nsurv + __popcll(bal & ((1ull << lane) - 1ull))] = (unsigned char)c;
                nsurv += __popcll(bal);
                if (c < nj * nsmp) L.alive[c] = pass;
            }
            __builtin_amdgcn_wave_barrier();
            // only the passing pairs' weight rows are cleared, read and written back
            auto is_alive = [&](int j, int k) -> bool { return L.alive[j * nsmp + k] != 0; };
            for (int e = lane; e < nsurv * 16; e += 64) {
                const int ck = L.cks[e >> 4], j = (ck * smag) >> 16;
                L.Wr[j][ck - j * nsmp][e & 15] = 0.0f;
            }
            __builtin_amdgcn_wave_barrier();
            const int ncand = nsurv * K;
            // W3 of queue entry head + lane, when it exists
            auto eval = [&](int count) {
                if (lane < count) {
                    const int item = L.q[(head + lane) & (kQueue - 1)];
                    const int j = item >> 8, k = (item >> 4) & 15, q = item & 15;
                    const int pz1 = q / P, pz2 = q - pz1 * P, r2 = r2c + j;
                    const double z1lo = G.z0 + (r1 + (double)pz1 / P) * G.lz;
                    const double z1hi = G.z0 + (r1 + (double)(pz1 + 1) / P) * G.lz;
                    const double z2lo = G.z0 + (r2 + (double)pz2 / P) * G.lz;
                    const double z2hi = G.z0 + (r2 + (double)(pz2 + 1) / P) * G.lz;
                    const double w = w3_closed_uv(wg, vz, z1lo, z1hi, z2lo, z2hi, L.ca[k], L.sa[k], L.cb[k], L.sb[k]);
                    if (w > kEpsW3) {
                        L.Wr[j][k][q] = (float)w;
                        jm |= 1u << j;
                    }
                }
                head += count < 64 ? count : 64;
            };
#pragma unroll 1
            for (int c0 = 0; c0 < ncand; c0 += 64) {
                const int c = c0 + lane;
                bool pass = false;
                int item = 0;
                if (c < ncand) {
                    const int sv = c / K, q = c - sv * K, ck = L.cks[sv];
                    const int j = (ck * smag) >> 16, k = ck - j * nsmp;
                    const int pz1 = q / P, pz2 = q - pz1 * P;
                    if ((jok >> j) & 1u) {
                        const int r2 = r2c + j;
                        const double z1lo = G.z0 + (r1 + (double)pz1 / P) * G.lz;
                        const double z1hi = G.z0 + (r1 + (double)(pz1 + 1) / P) * G.lz;
                        const double z2lo = G.z0 + (r2 + (double)pz2 / P) * G.lz;
                        const double z2hi = G.z0 + (r2 + (double)(pz2 + 1) / P) * G.lz;
                        // pairs whose slope windows cannot meet anywhere in the bundle
                        // have weight exactly 0
                        const double a1lo = (z1lo - vz) * invD1, a1hi = (z1hi - vz) * invD1;
                        const double a2lo = (vz - z2hi) * invD2, a2hi = (vz - z2lo) * invD2;
                        const double t1hi_max = a1hi * (a1hi >= 0.0 ? L.c1hi[k] : L.c1lo[k]);
                        const double t1lo_min = a1lo * (a1lo >= 0.0 ? L.c1lo[k] : L.c1hi[k]);
                        const double t2hi_max = a2hi * (a2hi >= 0.0 ? L.c2hi[k] : L.c2lo[k]);
                        const double t2lo_min = a2lo * (a2lo >= 0.0 ? L.c2lo[k] : L.c2hi[k]);
                        pass = !(t1hi_max <= t2lo_min || t2hi_max <= t1lo_min);
                        item = (j << 8) | (k << 4) | (pz1 * P + pz2);
                    }
                }
                const unsigned long long bal = __ballot(pass);
                if (pass) L.q[(tail + __popcll(bal & ((1ull << lane) - 1ull))) & (kQueue - 1)] = item;
                tail += __popcll(bal);
                __builtin_amdgcn_wave_barrier();
                while (tail - head >= 64) eval(64);
            }
            if (tail > head) eval(tail - head);
            __builtin_amdgcn_wave_barrier();
            // rings with a non-zero tile: OR over the lanes
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) jm |= __shfl_xor(jm, off, 64);
            for (int j = 0; j < nj; ++j) {
                if (!((jm >> j) & 1u)) continue;
                const int r2 = r2c + j;
                // range errors count only for response rows that carry weight
                if (lane < 2 * K) {
                    const int l = lane < K ? lane : lane - K;
                    const int m = lane < K ? umask[g1 * nr1 + r1 + smax] : umask[g2 * nr1 + r2 + smax];
                    if ((m >> l) & 1) {  // a row out of the table's range: an error if it carries weight
                        const int pt = l / P, pz = l % P;
                        float sum = 0.0f;
                        for (int k = 0; k < nsmp; ++k) {
                            if ((lane < K ? L.pt1[k] : L.pt2[k]) != pt || !is_alive(j, k)) continue;
                            for (int q = 0; q < P; ++q) sum += lane < K ? L.Wr[j][k][pz * P + q] : L.Wr[j][k][q * P + pz];
                        }
                        if (sum != 0.0f) flag |= kStatRange;
                    }
                }
                // append the tile record: header, sample sub-segments, weight blocks
                if (slot_next == slot_end) {
                    unsigned int base = 0;
                    if (lane == 0) base = atomicAdd(S.rec_count, kSlotChunk);
                    slot_next = __shfl(base, 0, 64);
                    slot_end = slot_next + kSlotChunk;
                }
                const unsigned int slot = slot_next++;
                if (slot >= (unsigned int)S.cap_recs) {
                    flag |= kStatScratch;
                    continue;
                }
                ++n_tiles;
                float* rec = S.recs + (int64_t)slot * kRecFloats;
                int* h = (int*)rec;
                if (lane == 0) {
                    h[0] = g1;
                    h[1] = g2;
                    h[2] = (r1 + 512) | ((r2 + 512) << 10) | (vb << 20);
                    h[3] = nsmp;
                    h[4] = A.uvoff[vb] + g1 * nr1 + r1 + smax;
                    h[5] = A.uvoff[vb] + g2 * nr1 + r2 + smax;
                    h[6] = cl.y | (cl.z << 16);
                    h[7] = A.sym[vb];
                }
                if (lane < nsmp) h[kRecPts + lane] = L.pt1[lane] | (L.pt2[lane] << 8);
                for (int e = lane; e < nsmp * 16; e += 64) rec[kRecHead + e] = is_alive(j, e >> 4) ? L.Wr[j][e >> 4][e & 15] : 0.0f;
            }
            __builtin_amdgcn_wave_barrier();
        }
        }
    }
    // reserved slots left unused hold no samples
    for (unsigned int sl = slot_next + lane; sl < slot_end && sl < (unsigned int)S.cap_recs; sl += 64)
        ((int*)(S.recs + (int64_t)sl * kRecFloats))[3] = 0;
    if (lane == 0 && A.tiles && n_tiles) atomicAdd(A.tiles, n_tiles);
    if (flag) atomicOr(A.status, flag);
}

// ---------------------------------------------------------------------------
// K2b: tile contraction on matrix cores, and emission
// ---------------------------------------------------------------------------
// Persistent wavefronts walk the record buffer.  Per tile:
//   X = W V      (16 x 32, FP32 matrix cores: v_mfma_f32_16x16x4_f32, two column blocks)
//   T = U^T X    (32 x 32 padded from 25 x 25): FP32 form v_mfma_f32_32x32x2_f32 (8 steps);
//                BF16 form one v_mfma_f32_32x32x16_bf16 with U and X rounded to BF16;
//                hi/lo form adds U_hi X_lo and U_lo X_hi (three bf16 MFMAs).
// Lane l holds T[8(j/4) + 4(l/32) + j%4][l%32] in accumulator j: its column
// b = l%32 fixes the photon-2 crystal, its 16 rows the photon-1 crystals.
// The transaxial part of each entry's bin is the same for every member of the
// class.  A tile has few non-zero entries (those whose crystals see the
// bundle), so they are first compacted into a list in LDS (over the operands,
// which are spent by then); the emission then walks the members, each with its
// rings shifted, the lanes spread over the list.

constexpr int kGE = 8;  // adjoint list entries whose sinogram loads are in flight together

struct MmaOps {
    float W[16][17];
    float U[16][25];
    float V[16][25];
    float X[16][32];
};

struct MmaList {
    float t[640];           // entry value
    int key[640];           // transaxial bin (projections) or the class's slot for it (matrix build)
    unsigned char m[640];   // (a_z + 2) | (b_z + 2) << 3 | (photon 2 first) << 6
    unsigned short ab[640]; // a | b << 8: the entry's place in the tile
};

// The forward's emission by runs: a tile's entries grouped by transaxial
// neighbour pair p and axial diagonal bz - az.  Along such a group the bins of
// consecutive az lie on one ring-pair diagonal, one ring apart, and so do the
// class's z-members of one column and half (one ring shift apart), so the
// group reaches, for each column and half, one run of consecutive floats of
// the diagonal sinogram: float u = s + az sums the products of the entries
// with the member of shift s.  The runs of a chunk of (group, column-half)
// pairs are laid out one float per lane, and each float is added once.
constexpr int kFwdGroups = 225;   // 25 transaxial pairs x 9 axial diagonals
constexpr int kXsPad = 4;         // zero guards on both sides of a column-half's member values
constexpr int kFwdSlots = 1536;   // floats of the runs of one chunk of pairs
struct MmaFwdRuns {
    float gt[1152];                     // [group][az + 2]: the tile's entries (1125 used; cleared as float4)
    float xs[384];                      // [column-half][kXsPad + ring shift]: the members' values, 0 if the tile misses them
    unsigned short gl[kFwdGroups + 3];  // groups present in the tile
    unsigned int gmask[8];
    int mpos[64];                       // per pair of the chunk: the bin of its run's first valid float
    int minfo[64];                      // group | column-half << 8 | (u + 2) << 12 | mirror << 22
    int mstart[65];                     // exclusive prefix of the runs' valid lengths
    unsigned char mmap[kFwdSlots];      // float slot -> pair of the chunk
};

// classes with images: for each transaxial neighbour pair p = a_t * 5 + b_t
// of the tile and column ci of the class, entry p * 8 + ci holds the pair's
// transaxial bin seen from the column times NR^2 (the bin's first ring pair),
// with bit 31 set when the column's image puts photon 2's crystal first.
// The projections also keep, per list entry, the start of its ring-pair
// diagonal for both photon orders (see the emission).
struct MmaLds {
    union {
        MmaOps o;
        MmaList e;
    };
    int ptab[200];
    unsigned int dd[640];
};

// the forward: the runs over the spent operands (the list and its diagonal
// starts serve classes too large for the runs)
struct MmaLdsFwd {
    union {
        MmaOps o;
        struct {
            MmaList e;
            unsigned int dd[640];
        };
        MmaFwdRuns f;
    };
    int ptab[200];
};

// the adjoint with the table gradient keeps the operands past the emission
struct MmaLdsGrad {
    MmaOps o;
    MmaList e;
    union {
        int ptab[200];     // during the emission
        float Gm[32][33];  // after it: d loss / d T
    };
    float Gl[640];  // the same, by list entry
};

// the matrix build also gathers each tile's band contribution: for every
// transaxial neighbour pair (a_t, b_t) and row of the tile, the r_j range of its
// live entries (and for every column the r_i range), and the pair's slot (with
// the photon order in bit 30)
struct MmaLdsBuild {
    union {
        MmaOps o;
        MmaList e;
    };
    int2 bnd[125];   // by row: the r_j range
    int2 bndc[125];  // by column: the r_i range (classes with images)
    int bslot[25];
    int ptab[200];
    // the emission: per (entry, column-half) pair of a chunk, its accumulator
    // cell, group, valid ring shifts and value
    int mcell[64];
    int minfo[64];   // group | mirror << 5 | first valid shift << 8 | end << 16
    float mt[64];
};

template <int MODE>
struct MmaLdsOf {
    typedef MmaLds type;
};
template <>
struct MmaLdsOf<kModeAdjGrad> {
    typedef MmaLdsGrad type;
};
template <>
struct MmaLdsOf<kModeFwd> {
    typedef MmaLdsFwd type;
};
template <>
struct MmaLdsOf<kModeCount> {
    typedef MmaLdsBuild type;
};
template <>
struct MmaLdsOf<kModeFill> {
    typedef MmaLdsBuild type;
};

constexpr int kWavesM = 4;

template <int MODE>
__global__ void __launch_bounds__(64 * kWavesM) __attribute__((amdgpu_waves_per_eu(MODE == kModeAdjGrad ? 2 : 3)))
k_cyl3d_mma(Cyl3D G, Scratch3D S, Args3D A) {
    typedef typename MmaLdsOf<MODE>::type Lds;
    constexpr bool kAdj = MODE == kModeAdj || MODE == kModeAdjGrad;
    constexpr bool kGrad = MODE == kModeAdjGrad;
    __shared__ Lds ml[kWavesM];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int P = G.P;
    Lds& L = ml[wid];
    const unsigned int nrec = min(*S.rec_count, (unsigned int)S.cap_recs);
    const unsigned int wave0 = blockIdx.x * kWavesM + wid, nwaves = gridDim.x * kWavesM;
    // consecutive records run side by side: their emissions meet in the caches
    const int nb = A.batch < 8 ? A.batch : 8;
    int flag = 0;
    unsigned long long n_vt = 0;  // (voxel, tile) pairs
    const int m = lane & 31, hk = lane >> 5;
    // Software pipeline: while a record is processed, the next one's header
    // (one word per lane 0..23), weight blocks (4 per lane) and response rows
    // (7 + 7 per lane) are in flight, and the header after it too.
    int hA = 0, hB = 0;  // headers of the next two records, word = lane
    float pw[4], pu[7], pv[7];
    auto load_head = [&](unsigned int j) -> int {
        return lane < kRecHead ? ((const int*)(S.recs + (int64_t)j * kRecFloats))[lane] : 0;
    };
    auto load_data = [&](unsigned int j, int hd) {
        const float* r = S.recs + (int64_t)j * kRecFloats;
        const int ns = __shfl(hd, 3, 64);
        const float* ur = S.uvtab + (int64_t)__shfl(hd, 4, 64) * 400;
        const float* vr = S.uvtab + (int64_t)__shfl(hd, 5, 64) * 400;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = lane + 64 * i;
            pw[i] = e < ns * 16 ? r[kRecHead + e] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const int e = lane + 64 * i;
            pu[i] = e < 400 && ns > 0 ? ur[e] : 0.0f;
            pv[i] = e < 400 && ns > 0 ? vr[e] : 0.0f;
        }
    };
    if (wave0 < nrec) {
        hA = load_head(wave0);
        load_data(wave0, hA);
        if (wave0 + nwaves < nrec) hB = load_head(wave0 + nwaves);
    }
    for (unsigned int idx = wave0; idx < nrec; idx += nwaves) {
        const int hcur = hA;
        const int nsmp = __builtin_amdgcn_readfirstlane(__shfl(hcur, 3, 64));
        if (nsmp > 0) {
            // the record's operands into LDS
            for (int e = lane; e < 256; e += 64) L.o.W[e >> 4][e & 15] = 0.0f;
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                const int e = lane + 64 * i;
                if (e < 400) {
                    L.o.U[e / 25][e % 25] = pu[i];
                    L.o.V[e / 25][e % 25] = pv[i];
                }
            }
            __builtin_amdgcn_wave_barrier();
            // scatter the weight blocks: sample k couples (pt1, pz1) with (pt2, pz2)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = lane + 64 * i, k = e >> 4, q = e & 15;
                const int pts = __shfl(hcur, kRecPts + (k & 15), 64);
                if (e < nsmp * 16 && q < P * P) {
                    const int pt1 = pts & 0xff, pt2 = pts >> 8;
                    L.o.W[pt1 * P + q / P][pt2 * P + q % P] = pw[i];
                }
            }
        }
        // next record's data, and the header after it
        hA = hB;
        if (idx + nwaves < nrec) load_data(idx + nwaves, hA);
        if (idx + 2 * nwaves < nrec) hB = load_head(idx + 2 * nwaves);
        if (nsmp == 0) continue;  // a reserved slot left unused
        const int g1 = __builtin_amdgcn_readfirstlane(__shfl(hcur, 0, 64));
        const int g2 = __builtin_amdgcn_readfirstlane(__shfl(hcur, 1, 64));
        const int hv = __builtin_amdgcn_readfirstlane(__shfl(hcur, 2, 64));
        const int r1 = (hv & 1023) - 512, r2 = ((hv >> 10) & 1023) - 512;
        const int64_t su = __builtin_amdgcn_readfirstlane(__shfl(hcur, 4, 64));
        const int64_t sv = __builtin_amdgcn_readfirstlane(__shfl(hcur, 5, 64));
        const int h6 = __builtin_amdgcn_readfirstlane(__shfl(hcur, 6, 64));
        const int h7 = __builtin_amdgcn_readfirstlane(__shfl(hcur, 7, 64));
        // the class's members: first (batch index) and count; h7 its symmetry word
        const int4 cl = make_int4(0, h6 & 0xffff, h6 >> 16, 0);
        const int nzc = h7 & 0xff;
        const bool mir = h7 & 0x100, imgs = (h7 >> 9) != 0;
        __builtin_amdgcn_wave_barrier();
        // X = W V: lane l supplies W[l%16][k + l/16] and V[k + l/16][n0 + l%16]
#pragma unroll
        for (int n0 = 0; n0 < 32; n0 += 16) {
            v4f cx = {0.0f, 0.0f, 0.0f, 0.0f};
            const int col = n0 + (lane & 15);
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const int k = kk + (lane >> 4);
                const float a = L.o.W[lane & 15][k];
                const float b = col < 25 ? L.o.V[k][col] : 0.0f;
                cx = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, cx, 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) L.o.X[4 * (lane >> 4) + j][col] = cx[j];
        }
        __builtin_amdgcn_wave_barrier();
        v16f ct;
#pragma unroll
        for (int j = 0; j < 16; ++j) ct[j] = 0.0f;
        if (G.precision == PSF_FP32) {
#pragma unroll
            for (int kk = 0; kk < 16; kk += 2) {
                const float a = m < 25 ? L.o.U[kk + hk][m] : 0.0f;
                ct = __builtin_amdgcn_mfma_f32_32x32x2f32(a, L.o.X[kk + hk][m], ct, 0, 0, 0);
            }
        } else {
            v8bf ah, bh, al, bl;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float u = m < 25 ? L.o.U[8 * hk + i][m] : 0.0f;
                const float x = L.o.X[8 * hk + i][m];
                const float uh = bf16r(u), xh = bf16r(x);
                ah[i] = (__bf16)uh;
                bh[i] = (__bf16)xh;
                al[i] = (__bf16)bf16r(u - uh);
                bl[i] = (__bf16)bf16r(x - xh);
            }
            ct = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, ct, 0, 0, 0);
            if (G.precision == PSF_BF16X2) {
                ct = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, ct, 0, 0, 0);
                ct = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, ct, 0, 0, 0);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if constexpr (MODE == kModeFwd) {
          if (cl.z <= 256 && cl.z / nzc <= 16) {
            // the forward: emission by runs (see MmaFwdRuns); the operands are spent
            const int nhg = cl.z / nzc;          // columns x halves
            const int XS = nzc + 2 * kXsPad;     // a column-half's row of member values
            float4* g4 = (float4*)L.f.gt;
            for (int i = lane; i < 288; i += 64) g4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (lane < 8) L.f.gmask[lane] = 0u;
            if (imgs) {  // the neighbour pairs seen from every column of the class
                const int ni = cl.z / (nzc * (mir ? 2 : 1));
                for (int it = lane; it < 200; it += 64) {
                    const int pp = it >> 3, ci = it & 7;
                    if (ci >= ni) continue;
                    int ga = g1 + pp / 5 - 2, gb = g2 + pp % 5 - 2;
                    ga = ga < 0 ? ga + G.Nc : (ga >= G.Nc ? ga - G.Nc : ga);
                    gb = gb < 0 ? gb + G.Nc : (gb >= G.Nc ? gb - G.Nc : gb);
                    int v = 0;
                    if (ga != gb) {
                        const int code = sym_code(h7, ci);
                        const int a = image_crystal(code, ga, G.Nc, G.nc), b = image_crystal(code, gb, G.Nc, G.nc);
                        v = (a < b ? tbin32(a, b, G.Nc) : tbin32(b, a, G.Nc)) * (G.NR * G.NR) | (a > b ? (int)0x80000000 : 0);
                    }
                    L.ptab[it] = v;
                }
            }
            __builtin_amdgcn_wave_barrier();
            {  // the tile's live entries into their groups
                const int bt_ = m / 5, bz_ = m % 5 - 2;
                int gbb = g2 + bt_ - 2;
                gbb = gbb < 0 ? gbb + G.Nc : (gbb >= G.Nc ? gbb - G.Nc : gbb);
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int a = 8 * (j >> 2) + 4 * hk + (j & 3);
                    if (m >= 25 || a >= 25 || ct[j] == 0.0f) continue;
                    int ga = g1 + a / 5 - 2;
                    ga = ga < 0 ? ga + G.Nc : (ga >= G.Nc ? ga - G.Nc : ga);
                    if (ga == gbb) continue;
                    const int az_ = a % 5 - 2;
                    const int gi = ((a / 5) * 5 + bt_) * 9 + (bz_ - az_ + 4);
                    L.f.gt[gi * 5 + az_ + 2] = ct[j];
                    atomicOr(&L.f.gmask[gi >> 5], 1u << (gi & 31));
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < 8) {  // list the present groups
                const unsigned int w = L.f.gmask[lane];
                const int pre = __popc(w);
                int incl = pre;
                for (int off = 1; off < 8; off <<= 1) {
                    const int o = __shfl_up(incl, off, 8);
                    if (lane >= off) incl += o;
                }
                int at = incl - pre;
                for (unsigned int b = w; b; b &= b - 1) L.f.gl[at++] = (unsigned short)(lane * 32 + __ffs(b) - 1);
            }
            __builtin_amdgcn_wave_barrier();
            const int ngr = __builtin_amdgcn_readfirstlane(__popc(L.f.gmask[0]) + __popc(L.f.gmask[1]) + __popc(L.f.gmask[2]) +
                                                           __popc(L.f.gmask[3]) + __popc(L.f.gmask[4]) + __popc(L.f.gmask[5]) +
                                                           __popc(L.f.gmask[6]) + __popc(L.f.gmask[7]));
            const int npair = ngr * nhg;
            const int NR = G.NR;
            // pairs per chunk: their runs (at most nzc + 4 floats each) fit the slot map
            const int cp = kFwdSlots / (nzc + 4) < 64 ? kFwdSlots / (nzc + 4) : 64;
            for (int bb = 0; bb < nb; ++bb) {
                // the members' values by (column-half, ring shift), zero guards around
                for (int i = lane; i < nhg * XS; i += 64) L.f.xs[i] = 0.0f;
                __builtin_amdgcn_wave_barrier();
                for (int sm0 = 0; sm0 < cl.z; sm0 += 64) {
                    const int sm = sm0 + lane;
                    bool ok = false;
                    if (sm < cl.z) {
                        const int hg = sm / nzc, s2 = sm - hg * nzc;
                        const int sh = (mir && (hg & 1)) ? nzc - 1 - s2 : s2;
                        ok = r1 + sh >= 0 && r1 + sh < NR && r2 + sh >= 0 && r2 + sh < NR;
                        if (ok) L.f.xs[hg * XS + kXsPad + sh] = S.xm[(int64_t)(cl.y + sm) * 8 + bb];
                    }
                    if (bb == 0) n_vt += __popcll(__ballot(ok)) * (lane == 0);
                }
                float* ob = A.y + (int64_t)bb * G.nbins;
                for (int c0 = 0; c0 < npair; c0 += cp) {
                    __builtin_amdgcn_wave_barrier();
                    // one lane per pair of the chunk: its run's valid part, first bin and direction
                    int cnt = 0;
                    if (lane < cp && c0 + lane < npair) {
                        const int pi = c0 + lane;
                        const int gq = pi / nhg, hg = pi - gq * nhg;
                        const int g = L.f.gl[gq];
                        const int p = g / 9, dz = g - p * 9 - 4;
                        const int azlo = dz > 0 ? -2 : -2 - dz;
                        const int len = nzc + 4 - (dz < 0 ? -dz : dz);
                        // float o of the run is u = o + azlo = shift + az: rings r1 + u and r2 + dz + u
                        int ulo = -r1 > -r2 - dz ? -r1 : -r2 - dz;
                        int uhi = NR - r1 < NR - r2 - dz ? NR - r1 : NR - r2 - dz;
                        ulo = ulo > azlo ? ulo : azlo;
                        uhi = uhi < azlo + len ? uhi : azlo + len;
                        cnt = uhi > ulo ? uhi - ulo : 0;
                        const bool mh = mir && (hg & 1);
                        int tb;
                        bool sw;
                        if (imgs) {
                            const int v = L.ptab[(p << 3) + (mir ? hg >> 1 : hg)];
                            sw = v < 0;
                            tb = v & 0x7fffffff;
                        } else {
                            int ga = g1 + p / 5 - 2, gb = g2 + p % 5 - 2;
                            ga = ga < 0 ? ga + G.Nc : (ga >= G.Nc ? ga - G.Nc : ga);
                            gb = gb < 0 ? gb + G.Nc : (gb >= G.Nc ? gb - G.Nc : gb);
                            sw = ga > gb;
                            tb = (sw ? tbin32(gb, ga, G.Nc) : tbin32(ga, gb, G.Nc)) * (NR * NR);
                        }
                        const int ri = r1 + ulo, rj = r2 + dz + ulo;
                        int rb = sw ? rj : ri, rc = sw ? ri : rj;  // the bin's rings, photon order of the bin
                        if (mh) {
                            rb = NR - 1 - rb;
                            rc = NR - 1 - rc;
                        }
                        L.f.mpos[lane] = cnt > 0 ? tb + diag32(rb, rc, NR) : 0;
                        L.f.minfo[lane] = g | (hg << 8) | ((ulo + 2) << 12) | (mh ? 1 << 22 : 0);
                    }
                    int incl = cnt;
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        const int o = __shfl_up(incl, off, 64);
                        if (lane >= off) incl += o;
                    }
                    const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
                    const int st0 = incl - cnt;
                    L.f.mstart[lane] = st0;
                    for (int t = 0; t < cnt; ++t) L.f.mmap[st0 + t] = (unsigned char)lane;
                    __builtin_amdgcn_wave_barrier();
                    for (int k = lane; k < total; k += 64) {
                        const int j = L.f.mmap[k];
                        const int info = L.f.minfo[j];
                        const int t = k - L.f.mstart[j];
                        const int g = info & 0xff, hg = (info >> 8) & 0xf;
                        const int u = ((info >> 12) & 0x3ff) - 2 + t;
                        const float* gv = &L.f.gt[g * 5];
                        const float* xv = &L.f.xs[hg * XS + kXsPad + u + 2];   // shift u - az at az = a - 2
                        float val = 0.0f;
#pragma unroll
                        for (int a = 0; a < 5; ++a) val += gv[a] * xv[-a];
                        if (val != 0.0f) atomicAdd(&ob[L.f.mpos[j] + ((info >> 22) ? -t : t)], val);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
            continue;
          }
        }
        // live entries (crystals distinct, inside the 25 x 25 tile, non-zero) and
        // the transaxial part of their bins.  The table gradient also needs the
        // zero entries in a row a of a non-zero column of U or a column b of a
        // non-zero column of X: dU = X dT^T and dV = W^T U dT read d loss / d T
        // there (a zero table entry still has a gradient).
        unsigned int uzm = 0u, xzm = 0u;
        if constexpr (kGrad) {
            bool nu = false, nx = false;
            if (lane < 25)
                for (int p = 0; p < 16; ++p) {
                    nu |= L.o.U[p][lane] != 0.0f;
                    nx |= L.o.X[p][lane] != 0.0f;
                }
            uzm = (unsigned int)__ballot(nu);
            xzm = (unsigned int)__ballot(nx);
        }
        const int bq = m;
        const int bt = bq / 5 - 2, bz = bq % 5 - 2;
        int gb = g2 + bt;
        gb = gb < 0 ? gb + G.Nc : (gb >= G.Nc ? gb - G.Nc : gb);
        // the build keys entries by the reference column's slot (group cl.y); the
        // projections by transaxial bin, or by crystals in classes with images
        const int* smap = (MODE == kModeCount || MODE == kModeFill) ? S.slotmap + (int64_t)cl.y * G.ntbins : nullptr;
        int key[16];
        unsigned int live = 0u, swap = 0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int a = 8 * (j >> 2) + 4 * hk + (j & 3);
            key[j] = 0;
            int ga = g1 + a / 5 - 2;
            ga = ga < 0 ? ga + G.Nc : (ga >= G.Nc ? ga - G.Nc : ga);
            if (bq >= 25 || a >= 25 || ga == gb) continue;
            if (ct[j] == 0.0f && !(kGrad && (((uzm >> a) | (xzm >> bq)) & 1u))) continue;
            const bool sw = ga > gb;
            const int tb_ = (int)tbin_of(sw ? gb : ga, sw ? ga : gb, G.Nc);
            if (MODE == kModeCount || MODE == kModeFill) {
                key[j] = smap[tb_];
                if (key[j] < 0) {
                    flag |= kStatScratch;
                    continue;
                }
            } else {
                key[j] = imgs ? 0 : tb_ * (G.NR * G.NR);  // with images the pair table gives the bin
            }
            live |= 1u << j;
            swap |= sw ? 1u << j : 0u;
        }
        // compaction: wave prefix sum of the per-lane counts
        const int nl = __popc(live);
        int pre = nl;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(pre, off, 64);
            if (lane >= off) pre += o;
        }
        const int total = __shfl(pre, 63, 64);
        int pos = pre - nl;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (!((live >> j) & 1u)) continue;
            const int a = 8 * (j >> 2) + 4 * hk + (j & 3);
            L.e.t[pos] = ct[j];
            L.e.key[pos] = key[j];
            L.e.m[pos] = (unsigned char)(a % 5 | ((bz + 2) << 3) | (((swap >> j) & 1u) << 6));
            L.e.ab[pos] = (unsigned short)(a | (bq << 8));
            ++pos;
        }
        if constexpr (MODE == kModeFwd || MODE == kModeAdj) {
            // the projections: ab packs the rings, the photon order and the pair's
            // row of the pair table, (a_z + 2) | (b_z + 2) << 3 | swap << 6 | p << 7,
            // and dd the start of the entry's ring-pair diagonal offset by NR (ring
            // pair (r_i, r_j) sits at diag32(r_i, r_j) = start(r_j - r_i) + r_i), with
            // photon 1 first (low half) and photon 2 first (high half): r_j - r_i is
            // the same for every member up to that order and the axial mirror.
            // Rings are below 256 (checked at the entry points), so starts fit 16 bits.
            __builtin_amdgcn_wave_barrier();
            const int NR = G.NR;
            auto start = [&](int d) -> int {  // diag32(r_i, r_j) - r_i + NR, d = r_j - r_i + NR - 1
                if (d < NR - 1) return ((d * (d + 1)) >> 1) - (NR - 1 - d) + NR;
                const int k = d - (NR - 1);
                return ((NR * (NR - 1)) >> 1) + k * NR - ((k * (k - 1)) >> 1) + NR;
            };
            for (int e = lane; e < total; e += 64) {
                const int mm = L.e.m[e], ab = L.e.ab[e], a = ab & 0xff, b = ab >> 8;
                const int dl = ((mm >> 3) & 7) - (mm & 7) + r2 - r1;  // r_j - r_i, photon 1 first
                // (an entry whose difference leaves the scanner reaches no member: masked)
                L.dd[e] = (unsigned int)(start(NR - 1 + dl) & 0xffff) | ((unsigned int)(start(NR - 1 - dl) & 0xffff) << 16);
                L.e.ab[e] = (unsigned short)(mm | ((a / 5 * 5 + b / 5) << 7));
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (imgs) {  // the neighbour pairs seen from every column of the class
            const int ni = cl.z / (nzc * (mir ? 2 : 1));
            for (int it = lane; it < 200; it += 64) {
                const int pp = it >> 3, ci = it & 7;
                if (ci >= ni) continue;
                int ga = g1 + pp / 5 - 2, gb = g2 + pp % 5 - 2;
                ga = ga < 0 ? ga + G.Nc : (ga >= G.Nc ? ga - G.Nc : ga);
                gb = gb < 0 ? gb + G.Nc : (gb >= G.Nc ? gb - G.Nc : gb);
                int v = 0;
                if (ga != gb) {
                    const int code = sym_code(h7, ci);
                    const int a = image_crystal(code, ga, G.Nc, G.nc), b = image_crystal(code, gb, G.Nc, G.nc);
                    v = (a < b ? tbin32(a, b, G.Nc) : tbin32(b, a, G.Nc)) * (G.NR * G.NR) | (a > b ? (int)0x80000000 : 0);
                }
                L.ptab[it] = v;
            }
            __builtin_amdgcn_wave_barrier();
        }
        if constexpr (MODE == kModeCount) {
            // the reference column's band, in the reference's photon order: the
            // r_j range each (slot, relative r_i) row receives, and with images
            // also the r_i range of each (slot, relative r_j) column (a column
            // whose image swaps the photons reads its rows there).  The tile's
            // entries first meet in LDS, cell (a_t, b_t, row or column), where
            // the row is a_z (b_z when photon 2 is first: the slot is ordered so).
            const int brow0 = nzc + 1;  // s_max + 2
            for (int c = lane; c < 125; c += 64) {
                L.bnd[c] = make_int2(0x7fffffff, -0x7fffffff);
                L.bndc[c] = make_int2(0x7fffffff, -0x7fffffff);
            }
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < total; e += 64) {
                const int mm = L.e.m[e], ab = L.e.ab[e];
                const int az = mm & 7, bze = (mm >> 3) & 7;
                const bool sw = (mm >> 6) & 1;
                const int p = ((ab & 0xff) / 5) * 5 + (ab >> 8) / 5;
                const int cr = p * 5 + (sw ? bze : az), cc = p * 5 + (sw ? az : bze);
                const int ai = sw ? r2 + bze - 2 : r1 + az - 2, bj = sw ? r1 + az - 2 : r2 + bze - 2;
                atomicMin(&L.bnd[cr].x, bj);
                atomicMax(&L.bnd[cr].y, bj);
                if (imgs) {
                    atomicMin(&L.bndc[cc].x, ai);
                    atomicMax(&L.bndc[cc].y, ai);
                }
                L.bslot[p] = L.e.key[e] | (sw ? 0x40000000 : 0);
            }
            __builtin_amdgcn_wave_barrier();
            const int64_t bbase = (int64_t)cl.y * S.cap_slots * S.band_rows;
            for (int c = lane; c < 125; c += 64) {
                const int p = c / 5, ks = L.bslot[p];
                const bool sw = ks & 0x40000000;
                const int64_t brow = bbase + (int64_t)(ks & 0x3fffffff) * S.band_rows + c - 5 * p - 2 + brow0;
                const int2 v = L.bnd[c];
                if (v.x <= v.y) {
                    int2* b = S.band + brow + (sw ? r2 : r1);
                    atomicMin(&b->x, v.x);
                    atomicMax(&b->y, v.y);
                }
                const int2 w = L.bndc[c];
                if (imgs && w.x <= w.y) {
                    int2* b = S.bandc + brow + (sw ? r1 : r2);
                    atomicMin(&b->x, w.x);
                    atomicMax(&b->y, w.y);
                }
            }
        }
        if constexpr (MODE == kModeCount || MODE == kModeFill) {
          if (cl.z <= 256 && nzc <= 16) {
            // the build: each (entry, column-half) pair reaches one accumulator
            // cell, whose nzc members (one per ring shift) are adjacent floats.
            // Chunks of 64 pairs: one lane per pair finds the cell and the ring
            // shifts for which the entry's rings exist; then eight (nzc <= 8) or
            // sixteen lanes per pair add the entry to its members' floats.
            const int ngrp = cl.z / nzc;
            const int NRr = G.NR + nzc - 1, NR = G.NR;
            const int npair = total * ngrp;
            // members' shifts whose central rings exist: counted (voxel, tile) pairs
            {
                const int lo = (-r1 > -r2 ? -r1 : -r2) > 0 ? (-r1 > -r2 ? -r1 : -r2) : 0;
                const int hi = (NR - r1 < NR - r2 ? NR - r1 : NR - r2) < nzc ? (NR - r1 < NR - r2 ? NR - r1 : NR - r2) : nzc;
                n_vt += (unsigned long long)(hi > lo ? (hi - lo) * ngrp : 0) * (lane == 0);
            }
            for (int c0 = 0; c0 < npair; c0 += 64) {
                __builtin_amdgcn_wave_barrier();
                const int pi = c0 + lane;
                if (pi < npair) {
                    const int e = pi / ngrp, g = pi - e * ngrp;
                    const int mm = L.e.m[e], key = L.e.key[e];
                    const bool mh = mir && (g & 1);
                    const int ai = r1 + (mm & 7) - 2, bj = r2 + ((mm >> 3) & 7) - 2;
                    bool sw = (mm >> 6) & 1;
                    if (imgs) {  // the pair's photon order seen from the group's column
                        const int ab = L.e.ab[e];
                        const int v = L.ptab[((ab & 0xff) * 13 >> 6) * 40 + ((ab >> 8) * 13 >> 6) * 8 + (mir ? g >> 1 : g)];
                        sw = v < 0;
                    }
                    const int u = sw ? bj : ai, w = sw ? ai : bj;  // (r_i, r_j) for the reference voxel
                    const int i = mh ? NR - 1 - u : u + nzc - 1, j = mh ? NR - 1 - w : w + nzc - 1;
                    // shifts s with r1 + s, r2 + s, ai + s, bj + s inside the scanner
                    int lo = -r1 > -r2 ? -r1 : -r2;
                    lo = lo > -ai ? lo : -ai;
                    lo = lo > -bj ? lo : -bj;
                    lo = lo > 0 ? lo : 0;
                    int hi = NR - r1 < NR - r2 ? NR - r1 : NR - r2;
                    hi = hi < NR - ai ? hi : NR - ai;
                    hi = hi < NR - bj ? hi : NR - bj;
                    hi = hi < nzc ? hi : nzc;
                    L.mcell[lane] = (key * NRr + i) * NRr + j;
                    L.minfo[lane] = g | (mh ? 32 : 0) | ((lo > hi ? hi : lo) << 8) | (hi << 16);
                    L.mt[lane] = L.e.t[e];
                }
                __builtin_amdgcn_wave_barrier();
                const int nq = npair - c0 < 64 ? npair - c0 : 64;
                const int lsh = nzc <= 8 ? 3 : 4;  // lanes per pair: 8 or 16
                for (int q0 = 0; q0 < nq; q0 += 64 >> lsh) {
                    const int q = q0 + (lane >> lsh), s2 = lane & ((1 << lsh) - 1);
                    if (q >= nq || s2 >= nzc) continue;
                    const int info = L.minfo[q];
                    const int g = info & 31;
                    const int sh = (info & 32) ? nzc - 1 - s2 : s2;  // the reference-half voxel's shift
                    if (sh < ((info >> 8) & 0xff) || sh >= (info >> 16)) continue;
                    acc_add(S, (int64_t)(cl.y + g * nzc) * S.dense_slab + L.mcell[q] * nzc + s2, L.mt[q], flag);
                }
            }
            __builtin_amdgcn_wave_barrier();
            continue;
          }
        }
        // emission.  With at most 256 members, in passes of up to 64: lane =
        // (entry, member), the member fixed per lane (lane mod the pass's member
        // count rounded up to a power of two); projection sinograms in the
        // diagonal layout, so a lane group touches consecutive floats.
        // Otherwise member by member.
        const int npass = (cl.z + 63) >> 6;
        if (npass <= 4) {
            int lg = 0;
            while ((1 << lg) < (cl.z < 64 ? cl.z : 64)) ++lg;
            const int msk = (1 << lg) - 1;
            for (int mp = 0; mp < npass; ++mp) {
            const int sm = (mp << 6) + (lane & msk);  // the lane's member
            int R1 = -1, R2 = -1;
            double xv[8], acc[8];
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) {
                xv[bb] = 0.0;
                acc[bb] = 0.0;
            }
            bool mok = false, mh = false;
            int g = 0, s2 = 0;
            if (sm < cl.z) {
                g = sm / nzc;  // group (column and half) and index in it
                s2 = sm - g * nzc;
                mh = mir && (g & 1);
                const int s = mh ? nzc - 1 - s2 : s2;  // the reference-half voxel: its ring shift
                R1 = r1 + s;
                R2 = r2 + s;
                mok = R1 >= 0 && R1 < G.NR && R2 >= 0 && R2 < G.NR;
                if (kGrad && mok) {
                    const float* xs = S.xm + (int64_t)(cl.y + sm) * 8;
#pragma unroll
                    for (int bb = 0; bb < 8; ++bb)
                        if (bb < nb) xv[bb] = (double)xs[bb];
                }
            }
            bool mx = false;  // the member's xt is non-zero in some image
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) mx |= xv[bb] != 0.0;
            n_vt += __popcll(__ballot(mok && lane <= msk));
            // build: the lane's group's accumulators, [slot][i][j][s2] (members interleaved)
            const int64_t dbase = (int64_t)(cl.y + g * nzc) * S.dense_slab;
            const int NRr = G.NR + nzc - 1;
            // one list entry (code, value, key, place): forward atomics, or the
            // adjoint (and gradient) products
            auto ld = [&](int e, int& mm, float& t, int& key, int& ab) {
                mm = L.e.m[e];
                t = L.e.t[e];
                key = L.e.key[e];
                ab = imgs ? L.e.ab[e] : 0;
            };
            const int s_ref = R1 - r1;  // the reference-half voxel's ring shift
            // the entry's cell for the lane's member: the accumulator cell (build) or
            // the sinogram bin (projections); -1 when a ring leaves the scanner
            auto locate = [&](int mm, int key, int ab) -> int {
                // the entry's rings for the reference voxel; the member's are s_ref rings on
                const int ai = r1 + (mm & 7) - 2, bj = r2 + ((mm >> 3) & 7) - 2;
                if ((unsigned)(ai + s_ref) >= (unsigned)G.NR || (unsigned)(bj + s_ref) >= (unsigned)G.NR) return -1;
                bool sw = (mm >> 6) & 1;
                int tb = key;
                if (imgs) {  // the pair seen from the member's column: p * 8 + ci, p = (a / 5) * 5 + b / 5
                    const int v = L.ptab[((ab & 0xff) * 13 >> 6) * 40 + ((ab >> 8) * 13 >> 6) * 8 + (mir ? g >> 1 : g)];
                    sw = v < 0;
                    tb = v & 0x7fffffff;
                }
                const int u = sw ? bj : ai, w = sw ? ai : bj;  // (r_i, r_j) for the reference voxel
                if (MODE == kModeCount || MODE == kModeFill) {
                    // the group's cell: the same for all its members (key: the reference slot)
                    const int i = mh ? G.NR - 1 - u : u + nzc - 1, j = mh ? G.NR - 1 - w : w + nzc - 1;
                    return ((key * NRr + i) * NRr + j) * nzc + s2;
                }
                int ri = u + s_ref, rj = w + s_ref;
                if (mh) {  // the axial mirror image
                    ri = G.NR - 1 - ri;
                    rj = G.NR - 1 - rj;
                }
                return tb + diag32(ri, rj, G.NR);
            };
            const int step = 64 >> lg;
            if constexpr (MODE == kModeFwd || MODE == kModeAdj) {
                // the lane's member: its column's row in the pair table, the axial
                // mirror, and the rings of a list entry: offsets from r1s, r2s
                const int ci = mir ? g >> 1 : g;
                const int r1s = R1 - 2, r2s = R2 - 2, NR = G.NR;
                auto cell = [&](int e, float& t) -> int {  // the entry's sinogram bin, or -1
                    const int ab = L.e.ab[e];
                    t = L.e.t[e];
                    const int ai = r1s + (ab & 7), bj = r2s + ((ab >> 3) & 7);
                    if ((unsigned)ai >= (unsigned)NR || (unsigned)bj >= (unsigned)NR) return -1;
                    int tb;
                    bool sw;
                    if (imgs) {
                        const int v = L.ptab[((ab >> 7) << 3) + ci];
                        sw = v < 0;
                        tb = v & 0x7fffffff;
                    } else {
                        sw = ab & 64;
                        tb = L.e.key[e];
                    }
                    const unsigned int dd = L.dd[e];
                    const int st = (int)(sw != mh ? dd >> 16 : dd & 0xffff) - NR;
                    const int ri = sw ? bj : ai;
                    return tb + st + (mh ? NR - 1 - ri : ri);
                };
                // image by image; kGE entries at a time: their bins first, then their
                // atomics, or their sinogram loads (all in flight together) and the
                // products in entry order
                for (int bb = 0; bb < nb; ++bb) {
                    const float* yb = A.yin + (int64_t)bb * G.nbins;
                    float* ob = A.y + (int64_t)bb * G.nbins;
                    // (float)(x * t) in FP32 equals the FP64 product rounded once (both are FP32 values)
                    const float xb = MODE == kModeFwd && mok ? S.xm[(int64_t)(cl.y + sm) * 8 + bb] : 0.0f;
                    double acc1 = 0.0;
                    if (mok && (MODE == kModeAdj || xb != 0.0f)) {
                        for (int e0 = lane >> lg; e0 < total; e0 += kGE * step) {
                            int c[kGE];
                            float tv[kGE];
#pragma unroll
                            for (int u = 0; u < kGE; ++u) {
                                const int e = e0 + u * step;
                                c[u] = -1;
                                tv[u] = 0.0f;
                                if (e < total) c[u] = cell(e, tv[u]);
                            }
                            if constexpr (MODE == kModeFwd) {
#pragma unroll
                                for (int u = 0; u < kGE; ++u)
                                    if (c[u] >= 0) atomicAdd(&ob[c[u]], xb * tv[u]);
                            } else {
                                float yv[kGE];
#pragma unroll
                                for (int u = 0; u < kGE; ++u) yv[u] = c[u] < 0 ? 0.0f : (A.ones ? 1.0f : yb[c[u]]);
                                float part = 0.0f;
#pragma unroll
                                for (int u = 0; u < kGE; ++u)
                                    if (c[u] >= 0) part += tv[u] * yv[u];
                                acc1 += (double)part;
                            }
                        }
                    }
                    if constexpr (MODE == kModeAdj) {  // the member's sum over its lanes
                        for (int off = 1 << lg; off < 64; off <<= 1) acc1 += __shfl_xor(acc1, off, 64);
                        if (lane <= msk && mok && acc1 != 0.0)
                            atomicAdd(&S.xrep[((int64_t)(wave0 % kXRep) * S.cap_mem + cl.y + sm) * 8 + bb], acc1);
                    }
                }
            } else if constexpr (kGrad) {
                // kGE entries at a time: their bins first, then all their sinogram
                // loads in flight together, then the products in entry order.  With the
                // table gradient every lane runs the same trip count: an entry's
                // gradient sums across its member lanes.
                for (int e0 = lane >> lg; e0 - (lane >> lg) < total; e0 += kGE * step) {
                    int c[kGE];
                    float tv[kGE];
#pragma unroll
                    for (int u = 0; u < kGE; ++u) {
                        const int e = e0 + u * step;
                        c[u] = -1;
                        tv[u] = 0.0f;
                        if (mok && e < total) {
                            int mm, key, ab;
                            ld(e, mm, tv[u], key, ab);
                            // a zero entry serves only the gradient: members with xt = 0 skip it
                            if (tv[u] != 0.0f || mx) c[u] = locate(mm, key, ab);
                        }
                    }
                    double gv[kGE];
#pragma unroll
                    for (int u = 0; u < kGE; ++u) gv[u] = 0.0;
#pragma unroll
                    for (int bb = 0; bb < 8; ++bb) {
                        if (bb >= nb) continue;
                        float yv[kGE];
#pragma unroll
                        for (int u = 0; u < kGE; ++u)
                            yv[u] = c[u] < 0 ? 0.0f : (A.ones ? 1.0f : A.yin[(int64_t)bb * G.nbins + c[u]]);
#pragma unroll
                        for (int u = 0; u < kGE; ++u) {
                            if (c[u] < 0) continue;
                            acc[bb] += (double)tv[u] * (double)yv[u];
                            if constexpr (kGrad) gv[u] += xv[bb] * (double)yv[u];
                        }
                    }
                    if constexpr (kGrad) {
#pragma unroll
                        for (int u = 0; u < kGE; ++u) {
                            double g = gv[u];
                            for (int off = 1; off <= msk; off <<= 1) g += __shfl_xor(g, off, 64);
                            const int e = e0 + u * step;
                            if ((lane & msk) == 0 && e < total) L.Gl[e] = mp ? L.Gl[e] + (float)g : (float)g;
                        }
                    }
                }
            } else if (mok) {
                // the build: the next entry's loads are in flight while one is emitted
                int e = lane >> lg, mm = 0, key = 0, ab = 0;
                float t = 0.0f;
                if (e < total) ld(e, mm, t, key, ab);
                for (; e < total; e += step) {
                    const int cm = mm, ck = key, ca = ab;
                    const float cv = t;
                    if (e + step < total) ld(e + step, mm, t, key, ab);
                    const int c = locate(cm, ck, ca);
                    if (c >= 0) acc_add(S, dbase + c, cv, flag);
                }
            }
            if constexpr (kGrad) {
#pragma unroll
                for (int bb = 0; bb < 8; ++bb) {
                    if (bb >= nb) break;
                    double sacc = acc[bb];
                    for (int off = 1 << lg; off < 64; off <<= 1) sacc += __shfl_xor(sacc, off, 64);
                    if (lane <= msk && mok && sacc != 0.0)
                        atomicAdd(&S.xrep[((int64_t)(wave0 % kXRep) * S.cap_mem + cl.y + sm) * 8 + bb], sacc);
                }
            }
            }
        } else if (imgs || mir) {
            flag |= kStatGeom;  // classes with images have at most 256 members (the plan keeps them so)
        } else {
        if constexpr (kGrad)
            for (int e = lane; e < total; e += 64) L.Gl[e] = 0.0f;
        for (int mi = cl.y; mi < cl.y + cl.z; ++mi) {
            const int4 me = A.mem[mi];
            const int R1 = r1 + me.y, R2 = r2 + me.y;
            if (R1 < 0 || R1 >= G.NR || R2 < 0 || R2 >= G.NR) continue;
            ++n_vt;
            const int64_t v = me.x;
            double xv[8], acc[8];
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) {
                acc[bb] = 0.0;
                xv[bb] = ((MODE == kModeFwd || kGrad) && bb < nb) ? (double)(kGrad ? A.xt : A.x)[(int64_t)bb * G.nvox + v] : 0.0;
            }
            const int64_t dbase = (int64_t)cl.y * S.dense_slab;
            const int NRr = G.NR + nzc - 1;
            for (int e = lane; e < total; e += 64) {
                const int mm = L.e.m[e];
                const int ra = R1 + (mm & 7) - 2, rb = R2 + ((mm >> 3) & 7) - 2;
                if (ra < 0 || ra >= G.NR || rb < 0 || rb >= G.NR) continue;
                const float t = L.e.t[e];
                const bool sw = (mm >> 6) & 1;
                const int ri = sw ? rb : ra, rj = sw ? ra : rb;
                if (MODE == kModeFwd || kAdj) {
                    const int64_t idx = (int64_t)L.e.key[e] + diag_index(ri, rj, G.NR);
                    if (MODE == kModeFwd) {
#pragma unroll
                        for (int bb = 0; bb < 8; ++bb)
                            if (bb < nb && xv[bb] != 0.0) atomicAdd(&A.y[(int64_t)bb * G.nbins + idx], (float)(xv[bb] * t));
                    } else {
                        double gv = 0.0;
#pragma unroll
                        for (int bb = 0; bb < 8; ++bb) {
                            if (bb >= nb) continue;
                            const double yv = A.ones ? 1.0 : (double)A.yin[(int64_t)bb * G.nbins + idx];
                            acc[bb] += (double)t * yv;
                            if constexpr (kGrad) gv += xv[bb] * yv;
                        }
                        if constexpr (kGrad) L.Gl[e] += (float)gv;
                    }
                } else {
                    acc_add(S,
                            dbase + (((int64_t)L.e.key[e] * NRr + ri - me.y + nzc - 1) * NRr + rj - me.y + nzc - 1) * nzc +
                                me.y,
                            t, flag);
                }
            }
            if (kAdj) {
#pragma unroll
                for (int bb = 0; bb < 8; ++bb) {
                    if (bb >= nb) break;
                    double sacc = acc[bb];
                    for (int off = 32; off > 0; off >>= 1) sacc += __shfl_down(sacc, off, 64);
                    if (lane == 0 && sacc != 0.0)
                        atomicAdd(&S.xrep[((int64_t)(wave0 % kXRep) * S.cap_mem + mi) * 8 + bb], sacc);
                }
            }
        }
        }
        if constexpr (kGrad) {
            // d loss / d T as a 25 x 25 matrix, then dU = X dT^T and dV = W^T (U dT)
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < 32 * 33; e += 64) (&L.Gm[0][0])[e] = 0.0f;
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < total; e += 64) {
                const int ab = L.e.ab[e];
                L.Gm[ab & 0xff][ab >> 8] = L.Gl[e];
            }
            __builtin_amdgcn_wave_barrier();
            const int K = P * P;
            for (int o = lane; o < K * 25; o += 64) {
                const int p = o / 25, a = o - p * 25;
                double d = 0.0;
                for (int b = 0; b < 25; ++b) d += (double)L.o.X[p][b] * (double)L.Gm[a][b];
                if (d != 0.0) atomicAdd(&S.uvgrad[(su * 16 + p) * 25 + a], d);
            }
            __builtin_amdgcn_wave_barrier();
            // Y = U dT over the spent X
            for (int o = lane; o < K * 25; o += 64) {
                const int p = o / 25, b = o - p * 25;
                double d = 0.0;
                for (int a = 0; a < 25; ++a) d += (double)L.o.U[p][a] * (double)L.Gm[a][b];
                L.o.X[p][b] = (float)d;
            }
            __builtin_amdgcn_wave_barrier();
            for (int o = lane; o < K * 25; o += 64) {
                const int q = o / 25, b = o - q * 25;
                double d = 0.0;
                for (int p = 0; p < K; ++p) d += (double)L.o.W[p][q] * (double)L.o.X[p][b];
                if (d != 0.0) atomicAdd(&S.uvgrad[(sv * 16 + q) * 25 + b], d);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0 && A.vtiles && n_vt) atomicAdd(A.vtiles, n_vt);
    if (flag) atomicOr(A.status, flag);
}

hipError_t launch_cyl3d_geom(const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st) {
    if (a.n_cls <= 0) return hipSuccess;
    const dim3 grid(kGeomWG), block(64 * kWavesT);
    switch (G.P) {
        case 1: hipLaunchKernelGGL(k_cyl3d_geom<1>, grid, block, 0, st, G, S, a); break;
        case 2: hipLaunchKernelGGL(k_cyl3d_geom<2>, grid, block, 0, st, G, S, a); break;
        case 3: hipLaunchKernelGGL(k_cyl3d_geom<3>, grid, block, 0, st, G, S, a); break;
        case 4: hipLaunchKernelGGL(k_cyl3d_geom<4>, grid, block, 0, st, G, S, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Blocks of a k_cyl3d_mma launch: twice as many as the GPU holds at once (the
// kernel's blocks per compute unit times the compute units), so that every
// block runs in one of two full rounds.  Each block's share of the records is
// fixed at launch; a partial last round would leave compute units idle.
template <int MODE>
dim3 mma_grid() {
    constexpr int kDevs = 64;
    static std::atomic<int> cached[kDevs];  // per device; 0 until queried (host threads may race: same value)
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kDevs) {
        int n = cached[dev].load(std::memory_order_relaxed);
        if (n <= 0) {
            int cus = 0, per = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cyl3d_mma<MODE>, 64 * kWavesM, 0) == hipSuccess &&
                cus > 0 && per > 0) {
                n = 2 * cus * per;
                cached[dev].store(n, std::memory_order_relaxed);
            }
        }
        if (n > 0) return dim3((unsigned)n);
    }
    return dim3(2048);
}

hipError_t launch_cyl3d_mma(int mode, const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st) {
    if (a.n_cls <= 0) return hipSuccess;
    const dim3 block(64 * kWavesM);
    switch (mode) {
        case kModeCount:
        case kModeFill:
            hipLaunchKernelGGL(k_cyl3d_mma<kModeCount>, mma_grid<kModeCount>(), block, 0, st, G, S, a);
            break;
        case kModeFwd:
            hipLaunchKernelGGL(k_cyl3d_mma<kModeFwd>, mma_grid<kModeFwd>(), block, 0, st, G, S, a);
            break;
        case kModeAdj:
            hipLaunchKernelGGL(k_cyl3d_mma<kModeAdj>, mma_grid<kModeAdj>(), block, 0, st, G, S, a);
            break;
        case kModeAdjGrad:
            if (!S.uvgrad || !a.xt) return hipErrorInvalidValue;
            hipLaunchKernelGGL(k_cyl3d_mma<kModeAdjGrad>, mma_grid<kModeAdjGrad>(), block, 0, st, G, S, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// the batch members' image values: xm[member][image] (one gather per batch,
// so the contraction reads them with the member's index)
__global__ void k_gather_members(Scratch3D S, Args3D A, const float* x, int64_t nvox) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // member * 8 + image
    if (i >= A.n_mem * 8) return;
    const int mi = i >> 3, bb = i & 7;
    S.xm[i] = bb < A.batch ? x[(int64_t)bb * nvox + A.mem[mi].x] : 0.0f;
}

hipError_t launch_gather_members(const Scratch3D& S, const Args3D& a, const float* x, int64_t nvox, hipStream_t st) {
    if (a.n_mem <= 0) return hipSuccess;
    if (a.n_mem > S.cap_mem) return hipErrorInvalidValue;
    const int n = a.n_mem * 8;
    hipLaunchKernelGGL(k_gather_members, dim3((n + 255) / 256), dim3(256), 0, st, S, a, x, nvox);
    return hipGetLastError();
}

// adjoint: fold the member sums' copies into x64 (each voxel is one member of
// the batch) and clear them for the next batch
__global__ void k_xrep_fold(Scratch3D S, Args3D A, int64_t nvox) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // member * 8 + image
    if (i >= A.n_mem * 8) return;
    const int mi = i >> 3, bb = i & 7;
    double sum = 0.0;
    for (int c = 0; c < kXRep; ++c) {
        double* p = &S.xrep[((int64_t)c * S.cap_mem + mi) * 8 + bb];
        sum += *p;
        *p = 0.0;
    }
    if (bb < A.batch && sum != 0.0) A.x64[(int64_t)bb * nvox + A.mem[mi].x] += sum;
}

hipError_t launch_xrep_fold(const Scratch3D& S, const Args3D& a, int64_t nvox, hipStream_t st) {
    if (a.n_mem <= 0) return hipSuccess;
    if (a.n_mem > S.cap_mem) return hipErrorInvalidValue;
    const int n = a.n_mem * 8;
    hipLaunchKernelGGL(k_xrep_fold, dim3((n + 255) / 256), dim3(256), 0, st, S, a, nvox);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K3: compaction of the dense accumulator into CSR rows (ascending bins)
// ---------------------------------------------------------------------------
// A member's accumulator rows (slot, r_i) are cut into chunks of kRowsC rows,
// one workgroup each; of each row only the columns in the class's band (moved
// by the member's shift) can be non-zero, and only those are read.  Count
// phase: each chunk adds its number of kept entries to the row count.  Fill
// phase: a first pass stores the per-chunk counts, the second writes each
// chunk at its offset (row start + counts of the chunks before it), in order.
// The last pass over a chunk clears what it read for the next batch.  Count
// phase with staging: one pass per column group (k_cyl3d_compact_group
// below); the fill phase copies each row's chunks in order (k_stage_copy).

constexpr int kBlockC = 256;
constexpr int kRowsC = 256;  // rows per chunk (one per thread for the row scan)
constexpr int kMapC = 8192;  // flat entries of a chunk mapped to their rows in LDS

enum { kCompactCount = 0, kCompactChunks = 1, kCompactFill = 2 };

__global__ void k_band_init(Scratch3D S, Args3D A) {
    const int grp = blockIdx.y;  // a member; the first voxel of each class holds the class's bands
    if (A.cls[A.mem[grp].z].y != grp) return;
    const int64_t n = (int64_t)S.n_slots[grp] * S.band_rows;
    int2* band = S.band + (int64_t)grp * S.cap_slots * S.band_rows;
    int2* bandc = S.bandc + (int64_t)grp * S.cap_slots * S.band_rows;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        band[i] = make_int2(0x7fffffff, -0x7fffffff);
        bandc[i] = make_int2(0x7fffffff, -0x7fffffff);
    }
}

hipError_t launch_band_init(const Scratch3D& S, const Args3D& a, hipStream_t st) {
    if (a.n_mem <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_init, dim3(64, a.n_mem), dim3(256), 0, st, S, a);
    return hipGetLastError();
}

template <int MODE>
__global__ void __launch_bounds__(kBlockC) k_cyl3d_compact(Cyl3D G, Scratch3D S, Args3D A) {
    __shared__ int wave_tot[kBlockC / 64];
    __shared__ int64_t s_run;
    __shared__ int rlo[kRowsC], rpre[kRowsC + 1];
    __shared__ int rbase[kRowsC], rbin[kRowsC];  // a row's cells: dense[rbase + col * nzc], bin rbin + col
    __shared__ unsigned short rowof[kMapC];      // the row of each flat entry, when the chunk has at most kMapC
    const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = bs >> 6;
    const int mi = blockIdx.y;  // member of the batch
    const int4 me = A.mem[mi];
    const int vb = me.z, sh = me.y;  // its class and ring shift
    const int grp = mi - sh;         // its column's group (the member index of the column's first voxel)
    const int64_t chunk = blockIdx.x;
    const int64_t row = me.w;
    const int NR = G.NR;
    const int nsl = S.n_slots[grp];
    const int64_t nrows = (int64_t)nsl * NR;
    const int64_t q0 = chunk * kRowsC;
    if (q0 >= nrows) return;
    const int nq = nrows - q0 < kRowsC ? (int)(nrows - q0) : kRowsC;
    const int64_t nrr = (int64_t)NR * NR;
    const int nzc = A.cls[vb].w + 1, NRr = NR + nzc - 1;  // the group's members, interleaved
    const int64_t dbase = (int64_t)grp * S.dense_slab;   // the group's cells in S.dense
    const int* stb = S.slot_tbin + (int64_t)grp * S.cap_slots;
    // the column's slots in its bin order: the reference slot, and whether the
    // image swaps the photons (the ring pair then reads the reference transposed)
    const int* order = S.slot_order + (int64_t)grp * S.cap_slots;
    int* ccount = S.chunk_counts + (int64_t)mi * S.max_chunks;
    const int brow0 = A.cls[vb].w + 2 - sh;  // band row of r_i is r_i - shift + s_max + 2
    const int64_t bref = (int64_t)A.cls[vb].y * S.cap_slots * S.band_rows;  // the class's bands
    // a mirror-half member reads the band of its reference-half voxel, rings
    // reflected: relative row C - (r_i - shift), columns C + shift - [hi, lo]
    const bool mh = (A.sym[vb] & 0x100) && (((grp - A.cls[vb].y) / nzc) & 1);
    const int C = NR - 1 - A.cls[vb].w;
    // the chunk's rows: first column and length (band moved by the shift, cut to the scanner)
    {
        const int r = tid;  // kRowsC == kBlockC
        int lo = 0, len = 0;
        if (r < nq) {
            const int q = (int)(q0 + r);  // rows of a member: below 4096 slots x NR
            const int slot = q / NR, ri = q - slot * NR;
            const int ov = order[slot];
            rbase[r] = (((ov & 0x3fffffff) * NRr + ri - sh + nzc - 1) * NRr - sh + nzc - 1) * nzc + sh;
            rbin[r] = stb[slot] * (NR * NR) + ri * NR;
            const int brow = mh ? NR + 1 - ri + sh : ri + brow0;
            const int2 b = ((ov & 0x40000000) ? S.bandc : S.band)[bref + (int64_t)(ov & 0x3fffffff) * S.band_rows + brow];
            if (b.x <= b.y) {  // else the row was never reached (and holds the empty sentinel)
                const int l = max(mh ? C + sh - b.y : b.x + sh, 0), h = min(mh ? C + sh - b.x : b.y + sh, NR - 1);
                if (l <= h) {
                    lo = l;
                    len = h - l + 1;
                }
            }
        }
        // block exclusive scan of the lengths
        int inc = len;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wave_tot[wid] = inc;
        __syncthreads();
        int base = 0, all = 0;
        for (int w = 0; w < nw; ++w) {
            base += w < wid ? wave_tot[w] : 0;
            all += wave_tot[w];
        }
        rlo[r] = lo;
        rpre[r] = base + inc - len;
        if (tid == 0) rpre[kRowsC] = all;
        __syncthreads();
    }
    const int T = rpre[kRowsC];
    if (T <= kMapC) {
        for (int i = rpre[tid]; i < rpre[tid + 1]; ++i) rowof[i] = (unsigned short)tid;  // kRowsC == kBlockC
        __syncthreads();
    }
    int64_t start = 0, cap = 0;
    if (MODE == kCompactFill) {
        // kept entries of the chunks before this one
        int64_t part = 0;
        for (int64_t c = tid; c < chunk; c += bs) part += ccount[c];
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
        __syncthreads();
        if (lane == 0) wave_tot[wid] = (int)part;
        __syncthreads();
        if (tid == 0) {
            int64_t off = 0;
            for (int w = 0; w < nw; ++w) off += wave_tot[w];
            s_run = off;
        }
        start = A.row_ptr[row];
        cap = A.row_ptr[row + 1] - start;
    } else {
        if (tid == 0) s_run = 0;
    }
    __syncthreads();
    const int64_t run0 = s_run;
    for (int f0 = 0; f0 < T; f0 += bs) {
        const int f = f0 + tid;
        float a = 0.0f;
        int lo = 0, col = 0;
        if (f < T) {
            if (T <= kMapC) {  // the row holding flat entry f
                lo = rowof[f];
            } else {  // last r with rpre[r] <= f
                int hi = nq - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (rpre[mid] <= f) lo = mid;
                    else hi = mid - 1;
                }
            }
            col = rlo[lo] + (f - rpre[lo]);
            const int di = rbase[lo] + col * nzc;
            a = acc_take(S, dbase + di, MODE != kCompactChunks);  // leave the accumulator clean
        }
        const bool keep = a > 0.0f && (double)a >= A.threshold;
        const unsigned long long m = __ballot(keep);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wid] = __popcll(m);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < nw; ++w) {
            off += w < wid ? wave_tot[w] : 0;
            tot += wave_tot[w];
        }
        const int64_t run = s_run;
        if (MODE == kCompactFill && keep) {
            const int64_t pos = run + off + pre;
            const int32_t b = rbin[lo] + col;
            if (pos < cap) {
                A.col[start + pos] = b;
                A.val[start + pos] = a;
            } else {
                atomicOr(A.status, kStatOverflow);
            }
        }
        __syncthreads();
        if (tid == 0) s_run = run + tot;
        __syncthreads();
    }
    if (tid == 0) {
        const int64_t n = s_run - run0;
        if (MODE == kCompactCount) atomicAdd((unsigned long long*)&A.row_ptr[row + 1], (unsigned long long)n);
        if (MODE == kCompactChunks) {
            ccount[chunk] = (int)n;
        } else if (MODE == kCompactFill && q0 + nq == nrows && s_run != cap) {
            atomicOr(A.status, kStatOverflow);
        }
    }
}

// The count phase with staging, one workgroup per (chunk, column group): the
// group's n members (n <= 8) are interleaved in the accumulators, member s of
// cell (slot k, i, j) at ((k (NR + n - 1) + i)(NR + n - 1) + j) n + s, so the
// workgroup reads and clears each cell's n floats together.  A cell's band row
// and column range are the same for every member (the bands are kept relative
// to the reference voxel); member s owns cell (i, j) as ring pair
// (i + s - n + 1, j + s - n + 1) when both rings are inside the scanner, and its
// bin is the cell's plus s (NR + 1).  Each member's entries come out in its
// bin order, as in the member-by-member kernel, into its own stage region.
// Chunks are kRowsC accumulator rows (slot, i) of the group.
static_assert(kBlockC == 256, "the group compaction's pass totals hold four waves");
__global__ void __launch_bounds__(kBlockC) k_cyl3d_compact_group(Cyl3D G, Scratch3D S, Args3D A) {
    __shared__ int wave_tot[8][kBlockC / 64];
    __shared__ __align__(16) int pass_tot[2][8][4];  // a pass's kept entries per member and wave (two passes alternate)
    __shared__ int64_t s_base[8];
    __shared__ int rlo[kRowsC], rpre[kRowsC + 1], wave_len[kBlockC / 64];
    __shared__ int rcell[kRowsC], rbin[kRowsC];  // a row's cell (j = 0), its bin for member 0 at j = n - 1
    __shared__ unsigned short rowof[kMapC];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = kBlockC / 64;
    // a column group of up to 16 members is compacted in halves of up to 8:
    // the block of its member 0 takes members 0-7, that of member 8 takes 8-15
    const int grp = blockIdx.y;  // the member index of the half's first voxel
    const int4 me = A.mem[grp];
    if (me.y & 7) return;  // not the first voxel of a half of its column group
    const int vb = me.z;
    const int NR = G.NR;
    const int nzc = A.cls[vb].w + 1, c = nzc - 1, NRr = NR + c;
    const int s0 = me.y, g0 = grp - s0;        // the half's first member; the group's first voxel
    const int nh = nzc - s0 < 8 ? nzc - s0 : 8;  // the half's members
    const int nsl = S.n_slots[g0];
    const int64_t nrows = (int64_t)nsl * NRr;
    const int64_t chunk = blockIdx.x;
    const int64_t q0 = chunk * kRowsC;
    if (chunk == 0 && tid < nh) A.stage_nch[A.mem[grp + tid].w] = (int)((nrows + kRowsC - 1) / kRowsC);
    if (q0 >= nrows) return;
    const int nq = nrows - q0 < kRowsC ? (int)(nrows - q0) : kRowsC;
    const int64_t dbase = (int64_t)g0 * S.dense_slab;  // the group's cells in S.dense
    const int* stb = S.slot_tbin + (int64_t)g0 * S.cap_slots;
    const int* order = S.slot_order + (int64_t)g0 * S.cap_slots;
    const int64_t bref = (int64_t)A.cls[vb].y * S.cap_slots * S.band_rows;
    const bool mh = (A.sym[vb] & 0x100) && (((g0 - A.cls[vb].y) / nzc) & 1);
    const int C = NR - 1 - c;
    int tot_s[8];  // the chunk's cells of each member (its stage reservation)
    {
        const int r = tid;  // kRowsC == kBlockC
        int lo = 0, len = 0;
        int ls[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) ls[s] = 0;
        if (r < nq) {
            const int q = (int)(q0 + r);
            const int slot = q / NRr, i = q - slot * NRr;
            const int ov = order[slot];
            rcell[r] = ((ov & 0x3fffffff) * NRr + i) * NRr * nzc;
            rbin[r] = stb[slot] * (NR * NR) + (i - c) * NR - c;
            const int brow = mh ? NR + nzc - i : i + 2;
            const int2 b = ((ov & 0x40000000) ? S.bandc : S.band)[bref + (int64_t)(ov & 0x3fffffff) * S.band_rows + brow];
            if (b.x <= b.y) {  // else the row was never reached
                const int l = max(mh ? C - b.y + c : b.x + c, 0), h = min(mh ? C - b.x + c : b.y + c, NRr - 1);
                if (l <= h) {
                    lo = l;
                    len = h - l + 1;
#pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        // member sg = s0 + s: rows and columns c - sg .. NR - 1 + c - sg
                        const int sg = s0 + s;
                        if (s < nh && i >= c - sg && i <= NR - 1 + c - sg) {
                            const int l2 = max(l, c - sg), h2 = min(h, NR - 1 + c - sg);
                            ls[s] = h2 >= l2 ? h2 - l2 + 1 : 0;
                        }
                    }
                }
            }
        }
        // block exclusive scan of the lengths, and each member's total
        int inc = len;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            int v = ls[s];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) wave_tot[s][wid] = v;
        }
        if (lane == 63) wave_len[wid] = inc;
        __syncthreads();
        int base = 0, all = 0;
        for (int w = 0; w < nw; ++w) {
            base += w < wid ? wave_len[w] : 0;
            all += wave_len[w];
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            int t = 0;
            for (int w = 0; w < nw; ++w) t += wave_tot[s][w];
            tot_s[s] = t;
        }
        rlo[r] = lo;
        rpre[r] = base + inc - len;
        __syncthreads();
        if (tid == 0) rpre[kRowsC] = all;
        __syncthreads();
    }
    const int T = rpre[kRowsC];
    if (T <= kMapC) {
        for (int i = rpre[tid]; i < rpre[tid + 1]; ++i) rowof[i] = (unsigned short)tid;
        __syncthreads();
    }
    // each member's reservation in its stage region
    if (tid < nh) {
        const int s = tid;
        int64_t b = -1;
        int ts = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u == s) ts = tot_s[u];
        const int64_t row = A.mem[grp + s].w;
        if (ts > 0) {
            if (row < A.stage_rows) {
                const int cnt = atomicAdd(&A.stage_cnt[row], ts);
                if ((int64_t)cnt + ts <= A.stage_per_row) b = row * A.stage_per_row + cnt;
            }
            if (b < 0) atomicOr(A.stage_full, 1);
        }
        s_base[s] = b;
    }
    __syncthreads();
    int run[8];  // each member's kept entries so far (the same in every thread)
#pragma unroll
    for (int s = 0; s < 8; ++s) run[s] = 0;
    for (int f0 = 0; f0 < T; f0 += kBlockC) {
        const int f = f0 + tid;
        float a[8];
        unsigned int keep = 0u;
        int lo = 0, j = 0;
        if (f < T) {
            if (T <= kMapC) {
                lo = rowof[f];
            } else {
                int hi = nq - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (rpre[mid] <= f) lo = mid;
                    else hi = mid - 1;
                }
            }
            j = rlo[lo] + (f - rpre[lo]);
            const int i = (int)((q0 + lo) % NRr);
            const int64_t cell = dbase + rcell[lo] + j * nzc;
            if (!S.det && nh == 8 && ((uintptr_t)(S.dense + cell + s0) & 15) == 0) {
                // the half's eight floats: two 16-byte loads and stores
                float4* q = (float4*)(S.dense + cell + s0);
                const float4 v0 = q[0], v1 = q[1];
                q[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                q[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                a[0] = v0.x; a[1] = v0.y; a[2] = v0.z; a[3] = v0.w;
                a[4] = v1.x; a[5] = v1.y; a[6] = v1.z; a[7] = v1.w;
            } else {
#pragma unroll
                for (int s = 0; s < 8; ++s) a[s] = s < nh ? acc_take(S, cell + s0 + s, true) : 0.0f;
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (s < nh) {
                    const int sg = s0 + s;
                    const bool ok = i >= c - sg && i <= NR - 1 + c - sg && j >= c - sg && j <= NR - 1 + c - sg;
                    if (ok && a[s] > 0.0f && (double)a[s] >= A.threshold) keep |= 1u << s;
                }
            }
        }
        int pre[8];
        const int pb = (f0 / kBlockC) & 1;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const unsigned long long m = __ballot((keep >> s) & 1u);
            pre[s] = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) pass_tot[pb][s][wid] = __popcll(m);
        }
        // one barrier a pass: the totals written two passes on are behind the next one
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int4 wt = *(const int4*)pass_tot[pb][s];
            const int off = (wid > 0 ? wt.x : 0) + (wid > 1 ? wt.y : 0) + (wid > 2 ? wt.z : 0);
            if ((keep >> s) & 1u) {
                const int64_t start = s_base[s];
                if (start >= 0) {
                    const int64_t pos = run[s] + off + pre[s];  // below the member's reservation
                    A.stage_col[start + pos] = rbin[lo] + j + (s0 + s) * (NR + 1);
                    A.stage_val[start + pos] = a[s];
                }
            }
            run[s] += wt.x + wt.y + wt.z + wt.w;
        }
    }
    if (tid < nh) {
        const int64_t row = A.mem[grp + tid].w;
        int n = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) n = s == tid ? run[s] : n;
        atomicAdd((unsigned long long*)&A.row_ptr[row + 1], (unsigned long long)n);
        A.stage_cb[row * S.max_chunks + chunk] = s_base[tid];
        A.stage_cn[row * S.max_chunks + chunk] = n;
    }
}

int64_t cyl3d_max_chunks(int cap_slots, int NR) {
    return ((int64_t)cap_slots * NR + kRowsC - 1) / kRowsC;
}

// after a batch's staged compaction: the batch counts as staged if no chunk
// so far lacked room
__global__ void k_stage_batch(Args3D A) {
    if (threadIdx.x == 0 && !*A.stage_full) *A.stage_batches += 1;
}

// fill phase: staged rows of the members [0, n) copied to their CSR place,
// chunk by chunk
// One workgroup per row. The row's chunk records are read kCopyTile at a time
// (one per thread), their counts prefix-summed into output offsets, and the
// chunks copied by the workgroup's wavefronts side by side.
constexpr int kCopyTile = 512;

__global__ void __launch_bounds__(kCopyTile) k_stage_copy(Args3D A, int64_t max_chunks) {
    __shared__ int64_t csrc[kCopyTile];
    __shared__ int64_t cdst[kCopyTile];
    __shared__ int ccnt[kCopyTile];
    __shared__ int wsum[kCopyTile / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = kCopyTile / 64;
    const int64_t row = A.mem[blockIdx.x].w;
    int64_t dst = A.row_ptr[row];
    const int nch = A.stage_nch[row];
    for (int c0 = 0; c0 < nch; c0 += kCopyTile) {
        const int c = c0 + tid;
        const int n = c < nch ? A.stage_cn[row * max_chunks + c] : 0;
        const int64_t src = c < nch ? A.stage_cb[row * max_chunks + c] : -1;
        // exclusive prefix sum of the counts over the workgroup
        int inc = n;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        int base = 0, all = 0;
        for (int w = 0; w < nw; ++w) {
            base += w < wid ? wsum[w] : 0;
            all += wsum[w];
        }
        csrc[tid] = src;
        cdst[tid] = dst + base + inc - n;
        ccnt[tid] = n;
        __syncthreads();
        const int nt = nch - c0 < kCopyTile ? nch - c0 : kCopyTile;
        for (int k = wid; k < nt; k += nw) {
            const int64_t s = csrc[k], d = cdst[k];
            const int m = ccnt[k];
            if (s >= 0)
                for (int i = lane; i < m; i += 64) {
                    A.col[d + i] = A.stage_col[s + i];
                    A.val[d + i] = A.stage_val[s + i];
                }
        }
        dst += all;
        __syncthreads();  // before the next tile's records overwrite these
    }
}

hipError_t launch_stage_copy(const Args3D& a, int n_rows, int64_t max_chunks, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage_copy, dim3(n_rows), dim3(kCopyTile), 0, st, a, max_chunks);
    return hipGetLastError();
}

hipError_t launch_cyl3d_compact(int mode, const Cyl3D& G, const Scratch3D& S, const Args3D& a, hipStream_t st) {
    if (a.n_mem <= 0) return hipSuccess;
    const dim3 grid((unsigned)S.max_chunks, a.n_mem), block(kBlockC);
    if (mode == kModeCount && a.stage) {
        hipLaunchKernelGGL(k_cyl3d_compact_group, grid, block, 0, st, G, S, a);
        hipLaunchKernelGGL(k_stage_batch, dim3(1), dim3(64), 0, st, a);
    } else if (mode == kModeCount) {
        hipLaunchKernelGGL(k_cyl3d_compact<kCompactCount>, grid, block, 0, st, G, S, a);
    } else {
        hipLaunchKernelGGL(k_cyl3d_compact<kCompactChunks>, grid, block, 0, st, G, S, a);
        hipLaunchKernelGGL(k_cyl3d_compact<kCompactFill>, grid, block, 0, st, G, S, a);
    }
    return hipGetLastError();
}

__global__ void k_zero_f32(float* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

constexpr unsigned long long kDenseMagic = 0x50534644454e5345ull;

__global__ void k_dense_clear(float* p, int64_t n, const unsigned long long* state, unsigned long long s0,
                              unsigned long long s1, unsigned long long s2, int trust) {
    if (trust && state[0] == kDenseMagic && state[1] == s0 && state[2] == s1 && state[3] == s2) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_dense_mark(unsigned long long* state, unsigned long long s0, unsigned long long s1,
                             unsigned long long s2, int clean) {
    if (threadIdx.x == 0) {
        state[0] = clean ? kDenseMagic : 0ull;
        state[1] = s0;
        state[2] = s1;
        state[3] = s2;
    }
}

hipError_t launch_dense_clear(float* p, int64_t n, unsigned long long* state, const unsigned long long* sig, bool trust,
                              hipStream_t st) {
    if (n > 0) {
        const int64_t blocks = (n + 255) / 256;
        hipLaunchKernelGGL(k_dense_clear, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, p, n,
                           state, sig[0], sig[1], sig[2], trust ? 1 : 0);
    }
    return launch_dense_mark(state, sig, 0, st);
}

hipError_t launch_dense_mark(unsigned long long* state, const unsigned long long* sig, int clean, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_mark, dim3(1), dim3(64), 0, st, state, sig[0], sig[1], sig[2], clean);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace psf
