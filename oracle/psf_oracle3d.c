/*
 * psf_oracle3d.c -- FP64 CPU oracle, 3D scanner.  TEST INFRASTRUCTURE ONLY
 * (see psf_oracle.c: only the tests, the smoke check and the CPU baseline of
 * the benchmark may load it; it shares no code with the library).
 *
 * The paper builds the matrix for a 2D ring and names the 3D matrix as future
 * work (Sec 4).  This file extends each step of Sec 2 to a cylinder of block
 * rings, with these readings:
 *   - Response table indexed by the two projected incidence angles: alpha_t in
 *     the transaxial plane and alpha_z, whose tangents are the lateral slopes
 *     of the ray per unit depth along the face normal.  Entry (a_t, a_z) is
 *     the first-interaction probability in the crystal column at those offsets
 *     (the 3D form of Eq.1, 6-7: attenuation along the slanted path, averaged
 *     over the sub-patch of entry points).
 *   - Each crystal face is split into P x P sub-patches (P per axis, Sec 2.1.1).
 *   - Homogenization (Eq.11 in the k -> infinity limit, now on the sphere):
 *     an unordered line through the voxel centre with transaxial direction
 *     theta and elevation slope T has weight dOmega / 2pi, so the weight of the
 *     lines from sub-patch (s1, q1) to (s2, q2) is
 *         W3 = 1/(2 pi) * integral over theta of [S(T_hi) - S(T_lo)]^+ ,
 *     S(T) = T / sqrt(1 + T^2), theta over the transaxial overlap of s1 and s2
 *     (the 2D sweep) and [T_lo, T_hi] the slopes that land in both axial
 *     sub-positions.  Sets below OG3_EPS_W (a fraction of the sphere) are empty.
 *   - Two-block penetration (Eq.2, 4, 5) acts transaxially, as in 2D; the ray
 *     keeps its axial slope through the gap: the axial slope in the next
 *     block's frame is tan(alpha_z) cos(alpha_t) / cos(beta), and its axial
 *     entry point is advanced by the axial travel between P^0 and P^1.
 *   - Block rings meet without an axial gap, so the axial neighbours need no
 *     remap; crystals beyond the axial ends do not exist.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_PI 3.14159265358979323846
#define OG_NB 5
#define OG_EPS_OV 1e-12
#define OG3_EPS_W 1e-14

#define OGF_MIRROR_TIE 1
#define OGF_ROW_TIE 2
#define OGF_OVERLAP_TIE 4
#define OGF_REMAP_TIE 8
#define OGF_RANGE 16
#define OGF_GEOM 32

typedef struct {
    int32_t n_blocks, n_ct, n_cz, n_brings;
    double pitch_t, pitch_z, depth, r_face, gap_z, mu, phi0;
} og_geom;

typedef struct {
    int32_t nx, ny, nz, pad;
    double dx, dy, dz, cx, cy, cz;
} og_image;

typedef struct {
    int32_t n_rows, n_sub;
    double step_deg;
    const double* data;
} og_table;

/* from psf_oracle.c */
void og_gauss_legendre(int n, double* x, double* w);
void og_seg_intervals(const og_geom* G, int P, double vx, double vy, double* lo, double* len);
double og_overlap_opposite(double lo1, double len1, double lo2, double len2);
int og_inside_ring(const og_geom* G, double vx, double vy);
void og_voxel_centre(const og_image* I, int64_t j, double* c);

static double g3x[16], g3w[16];
static int g3_ready = 0;
static void gl3_init(void) {
    if (!g3_ready) {
        og_gauss_legendre(16, g3x, g3w);
        g3_ready = 1;
    }
}

static int near_half_int(double f) {
    double r = f - floor(f);
    return fabs(r - 0.5) < 1e-9;
}
static int near_int(double f) { return fabs(f - nearbyint(f)) < 1e-9; }

static int cmp_double(const void* x, const void* y) {
    double a = *(const double*)x, b = *(const double*)y;
    return (a > b) - (a < b);
}

/* ------------------------------------------------------------------ */
/* 3D response table                                                   */
/* ------------------------------------------------------------------ */

/*
 * First-interaction probability in the crystal column at offsets (at, az) for
 * a photon entering at (ut, uz) from the entry crystal's lower edges, with
 * lateral slopes tt, tz >= 0 per unit depth.  It occupies column (at, az) for
 * the depths where both lateral positions lie in that column; the path length
 * to depth d is d * sqrt(1 + tt^2 + tz^2).
 */
double og_rho_point3(double tt, double tz, double ut, double uz, int at, int az, double lt, double lz, double L,
                     double mu) {
    double din = 0.0, dout = L;
    if (tt == 0.0) {
        if (at != 0) return 0.0;
    } else {
        din = fmax(din, (at * lt - ut) / tt);
        dout = fmin(dout, ((at + 1) * lt - ut) / tt);
    }
    if (tz == 0.0) {
        if (az != 0) return 0.0;
    } else {
        din = fmax(din, (az * lz - uz) / tz);
        dout = fmin(dout, ((az + 1) * lz - uz) / tz);
    }
    if (!(dout > din)) return 0.0;
    double k = sqrt(1.0 + tt * tt + tz * tz);
    return exp(-mu * k * din) - exp(-mu * k * dout);
}

/* integral over uz in [uz0, uz1] at fixed ut, split where a depth limit switches */
static double inner_uz(double tt, double tz, double ut, double uz0, double uz1, int at, int az, double lt, double lz,
                       double L, double mu) {
    gl3_init();
    double cuts[16];
    int nc = 0;
    cuts[nc++] = uz0;
    if (tz > 0.0) {
        double c[4] = {0.0, L, tt > 0.0 ? (at * lt - ut) / tt : 0.0, tt > 0.0 ? ((at + 1) * lt - ut) / tt : L};
        for (int i = 0; i < 4; i++) {
            double u1 = az * lz - tz * c[i], u2 = (az + 1) * lz - tz * c[i];
            if (u1 > uz0 && u1 < uz1) cuts[nc++] = u1;
            if (u2 > uz0 && u2 < uz1) cuts[nc++] = u2;
        }
    }
    cuts[nc++] = uz1;
    qsort(cuts, nc, sizeof(double), cmp_double);
    double tot = 0.0;
    for (int k = 0; k + 1 < nc; k++) {
        double lo = cuts[k], hi = cuts[k + 1];
        if (!(hi > lo)) continue;
        double h = 0.5 * (hi - lo), m = 0.5 * (hi + lo), s = 0.0;
        for (int i = 0; i < 16; i++) s += g3w[i] * og_rho_point3(tt, tz, ut, m + h * g3x[i], at, az, lt, lz, L, mu);
        tot += h * s;
    }
    return tot;
}

typedef struct {
    double tt, tz, uz0, uz1, lt, lz, L, mu;
    int at, az;
} outer_ctx;

static double gl16_outer(const outer_ctx* c, double a, double b) {
    double h = 0.5 * (b - a), m = 0.5 * (a + b), s = 0.0;
    for (int i = 0; i < 16; i++)
        s += g3w[i] * inner_uz(c->tt, c->tz, m + h * g3x[i], c->uz0, c->uz1, c->at, c->az, c->lt, c->lz, c->L, c->mu);
    return h * s;
}

/* adaptive bisection: accept when one 16-point rule agrees with two halves */
static double adapt_outer(const outer_ctx* c, double a, double b, double whole, int depth) {
    double m = 0.5 * (a + b);
    double l = gl16_outer(c, a, m), r = gl16_outer(c, m, b);
    if (depth >= 30 || fabs(l + r - whole) <= 1e-14 * fabs(l + r) + 1e-17) return l + r;
    return adapt_outer(c, a, m, l, depth + 1) + adapt_outer(c, m, b, r, depth + 1);
}

/* mean over sub-patch (pt, pz) of P x P, angles alpha_t, alpha_z >= 0.
 * The outer integral over ut is split where the inner integrand's pieces can
 * change (a transaxial depth limit meeting 0, L, an axial limit at a corner of
 * the sub-patch, or an axial limit shifted by one crystal), then each piece is
 * integrated adaptively (bisection until one 16-point rule agrees with two). */
double og_rho_sub3(double alpha_t, double alpha_z, int pt, int pz, int P, int at, int az, double lt, double lz,
                   double L, double mu) {
    gl3_init();
    outer_ctx c;
    c.tt = alpha_t == 0.0 ? 0.0 : tan(alpha_t);
    c.tz = alpha_z == 0.0 ? 0.0 : tan(alpha_z);
    c.uz0 = pz * lz / P;
    c.uz1 = (pz + 1) * lz / P;
    c.lt = lt; c.lz = lz; c.L = L; c.mu = mu; c.at = at; c.az = az;
    double ut0 = pt * lt / P, ut1 = (pt + 1) * lt / P;
    double cuts[64];
    int nc = 0;
    cuts[nc++] = ut0;
    if (c.tt > 0.0) {
        double dep[16];
        int nd = 0;
        dep[nd++] = 0.0;
        dep[nd++] = L;
        if (c.tz > 0.0) {
            const double zc[4] = {(az * lz - c.uz0) / c.tz, (az * lz - c.uz1) / c.tz, ((az + 1) * lz - c.uz0) / c.tz,
                                  ((az + 1) * lz - c.uz1) / c.tz};
            for (int i = 0; i < 4; i++) dep[nd++] = zc[i];
            dep[nd++] = lz / c.tz;
            dep[nd++] = -lz / c.tz;
            dep[nd++] = L + lz / c.tz;
            dep[nd++] = L - lz / c.tz;
        }
        for (int i = 0; i < nd; i++) {
            const double u1 = at * lt - c.tt * dep[i], u2 = (at + 1) * lt - c.tt * dep[i];
            if (u1 > ut0 && u1 < ut1) cuts[nc++] = u1;
            if (u2 > ut0 && u2 < ut1) cuts[nc++] = u2;
        }
    }
    cuts[nc++] = ut1;
    qsort(cuts, nc, sizeof(double), cmp_double);
    double v = 0.0;
    for (int k = 0; k + 1 < nc; k++) {
        if (!(cuts[k + 1] > cuts[k])) continue;
        const double whole = gl16_outer(&c, cuts[k], cuts[k + 1]);
        v += adapt_outer(&c, cuts[k], cuts[k + 1], whole, 0);
    }
    return v / ((ut1 - ut0) * (c.uz1 - c.uz0));
}

/* table entries for a list of angle-row pairs: out[k][pt][pz][at+2][az+2] */
void og_table3_rows(const og_geom* G, int P, double step_deg, const int32_t* rows_t, const int32_t* rows_z,
                    int nlist, double* out, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
#endif
    for (int k = 0; k < nlist; k++) {
        for (int pt = 0; pt < P; pt++) {
            double at_ = rows_t[k] * step_deg * OG_PI / 180.0, az_ = rows_z[k] * step_deg * OG_PI / 180.0;
            for (int pz = 0; pz < P; pz++)
                for (int a = -2; a <= 2; a++)
                    for (int b = -2; b <= 2; b++)
                        out[((((int64_t)k * P + pt) * P + pz) * OG_NB + (a + 2)) * OG_NB + (b + 2)] =
                            og_rho_sub3(at_, az_, pt, pz, P, a, b, G->pitch_t, G->pitch_z, G->depth, G->mu);
        }
    }
}

/* ------------------------------------------------------------------ */
/* 3D geometry and response rows                                       */
/* ------------------------------------------------------------------ */

static int n_rings(const og_geom* G) { return G->n_cz * G->n_brings; }

/* 1: column3 pairs every ring r1 with every ring r2 (no window); for tests */
static int g_full_ring_scan = 0;
void og3_set_full_ring_scan(int on) { g_full_ring_scan = on ? 1 : 0; }
static double z_first(const og_geom* G) { return -0.5 * n_rings(G) * G->pitch_z; }

static int64_t tab3_index(int nr, int P, int rt, int rz, int pt, int pz, int at, int az) {
    return (((((int64_t)rt * nr + rz) * P + pt) * P + pz) * OG_NB + (at + 2)) * OG_NB + (az + 2);
}

/*
 * Response row of sub-patch (g, pt; ring r, pz) seen from c: val[(a_t+2)*5 +
 * (a_z+2)] for the crystal at transaxial offset a_t and ring r + a_z; src the
 * table entry used (-1: zero by construction).  Returns flag bits.
 */
int og_uv_row_3d(const og_geom* G, const og_table* T, const double* c, int g, int pt, int r, int pz, double* val,
                 int32_t* src) {
    int flags = 0;
    const int nc = G->n_ct, R = G->n_blocks, P = T->n_sub, NR = n_rings(G), nr = T->n_rows;
    const double lt = G->pitch_t, lz = G->pitch_z, W = nc * lt;
    const int b = g / nc, cr = g % nc;
    const double phi = G->phi0 + 2.0 * OG_PI * b / R;
    const double nx = cos(phi), ny = sin(phi), tx = -ny, ty = nx;
    const double xi_m = -0.5 * W + (cr + (pt + 0.5) / P) * lt;
    const double z_m = z_first(G) + (r + (pz + 0.5) / P) * lz;
    const double D = G->r_face - (nx * c[0] + ny * c[1]);
    const double tan_t = (xi_m - (tx * c[0] + ty * c[1])) / D;
    const double tan_z = (z_m - c[2]) / D;
    const double alpha_t = atan(tan_t), alpha_z = atan(tan_z);
    if (fabs(tan_t) < 1e-12 || fabs(tan_z) < 1e-12) flags |= OGF_MIRROR_TIE;
    const int mt = alpha_t < 0.0, mz = alpha_z < 0.0;
    const double aat = fabs(alpha_t), aaz = fabs(alpha_z);
    double ft = aat * 180.0 / OG_PI / T->step_deg, fz = aaz * 180.0 / OG_PI / T->step_deg;
    if (near_half_int(ft) || near_half_int(fz)) flags |= OGF_ROW_TIE;
    int row_t = (int)floor(ft + 0.5), row_z = (int)floor(fz + 0.5);
    if (row_t > nr - 1) { flags |= OGF_RANGE; row_t = nr - 1; }
    if (row_z > nr - 1) { flags |= OGF_RANGE; row_z = nr - 1; }
    const int cm = mt ? nc - 1 - cr : cr;
    const int ptm = mt ? P - 1 - pt : pt;
    const int pzm = mz ? P - 1 - pz : pz;
    const double nu = mt ? xi_m + 0.5 * W : 0.5 * W - xi_m;

    /* two-block penetration: where the ray meets the next block's face line */
    int have_remap = 0, k = 0, pt1 = 0, pz1 = 0, dr = 0, row_bt = 0, row_bz = 0;
    const double beta = aat - 2.0 * OG_PI / R; /* Eq.2 */
    if (fabs(beta) < 1e-12) flags |= OGF_REMAP_TIE;
    if (beta > 0.0 && cm + 2 >= nc) {
        const double sigma = G->r_face * tan(OG_PI / R) - 0.5 * W;
        const double ap1 = sigma + sin(OG_PI / 2 - aat) / sin(OG_PI / 2 + beta) * (sigma + nu); /* Eq.4 */
        const double n = ap1 / lt;                                                            /* Eq.5 */
        if (near_int(n)) flags |= OGF_REMAP_TIE;
        k = (int)ceil(n) - 1;
        const double up = (k + 1) - n;
        if (near_int(up * P)) flags |= OGF_REMAP_TIE;
        pt1 = (int)floor(up * P);
        /* axial: slope in the next block's frame and axial travel from P^0 to P^1 */
        const double tzb = fabs(tan_z) * cos(aat) / cos(beta);
        const double ell = (sigma + nu) * sin(2.0 * OG_PI / R) / cos(beta);
        const double dz = ell * fabs(tan_z) * cos(aat);
        const double u = (pzm + 0.5) * lz / P + dz; /* axial entry offset from ring r's lower edge (leaning) */
        dr = (int)floor(u / lz);
        const double uz1 = u - dr * lz;
        if (near_int(u / lz) || near_int(uz1 * P / lz)) flags |= OGF_REMAP_TIE;
        pz1 = (int)floor(uz1 * P / lz);
        if (pz1 > P - 1) pz1 = P - 1;
        double fbt = beta * 180.0 / OG_PI / T->step_deg, fbz = atan(tzb) * 180.0 / OG_PI / T->step_deg;
        if (near_half_int(fbt) || near_half_int(fbz)) flags |= OGF_ROW_TIE;
        row_bt = (int)floor(fbt + 0.5);
        row_bz = (int)floor(fbz + 0.5);
        if (row_bt > nr - 1) { flags |= OGF_RANGE; row_bt = nr - 1; }
        if (row_bz > nr - 1) { flags |= OGF_RANGE; row_bz = nr - 1; }
        have_remap = 1;
    }
    for (int amt = -2; amt <= 2; amt++) {
        for (int amz = -2; amz <= 2; amz++) {
            const int a_t = mt ? -amt : amt, a_z = mz ? -amz : amz;
            const int ring = r + a_z, cc = cm + amt;
            double v = 0.0;
            int32_t s = -1;
            if (ring >= 0 && ring < NR) {
                if (cc >= 0 && cc < nc) {
                    s = (int32_t)tab3_index(nr, P, row_t, row_z, ptm, pzm, amt, amz);
                    v = T->data[s];
                } else if (cc >= nc && have_remap) {
                    const int idx = k + 1 + (cc - nc), az1 = amz - dr;
                    if (idx <= 2 && az1 >= -2 && az1 <= 2) {
                        s = (int32_t)tab3_index(nr, P, row_bt, row_bz, pt1, pz1, idx, az1);
                        v = T->data[s];
                    }
                }
            }
            val[(a_t + 2) * OG_NB + (a_z + 2)] = v;
            src[(a_t + 2) * OG_NB + (a_z + 2)] = s;
        }
    }
    return flags;
}

/* ------------------------------------------------------------------ */
/* Homogenization weights on the sphere                                */
/* ------------------------------------------------------------------ */

typedef struct {
    double D1, phi1, D2, phi2;   /* distances of the voxel to the two face lines, their normal angles */
    double z1lo, z1hi, z2lo, z2hi, zv;
} w3_ctx;

static double S_of(double t) { return t / sqrt(1.0 + t * t); }

/* slopes at direction theta: photon 1 towards theta, photon 2 towards theta + pi */
static void w3_slopes(const w3_ctx* c, double th, double* t1lo, double* t1hi, double* t2lo, double* t2hi) {
    const double d1 = c->D1 / cos(th - c->phi1);
    const double d2 = c->D2 / -cos(th - c->phi2);
    *t1lo = (c->z1lo - c->zv) / d1;
    *t1hi = (c->z1hi - c->zv) / d1;
    *t2lo = (c->zv - c->z2hi) / d2;
    *t2hi = (c->zv - c->z2lo) / d2;
}

static double w3_f(const w3_ctx* c, double th) {
    double a, b, p, q;
    w3_slopes(c, th, &a, &b, &p, &q);
    const double lo = fmax(a, p), hi = fmin(b, q);
    return hi > lo ? S_of(hi) - S_of(lo) : 0.0;
}

/* the four differences whose sign changes are the kinks of w3_f */
static double w3_g(const w3_ctx* c, double th, int which) {
    double a, b, p, q;
    w3_slopes(c, th, &a, &b, &p, &q);
    switch (which) {
        case 0: return b - q;
        case 1: return a - p;
        case 2: return b - p;
        default: return q - a;
    }
}

/*
 * W3 = 1/(2 pi) * integral over [th_a, th_b] of w3_f: the kinks (where the
 * binding slope limit switches, or the slope window closes) are located by
 * bisection on sign changes, and each smooth piece is integrated with 16-point
 * Gauss-Legendre.
 */
double og_w3(const w3_ctx* c, double th_a, double th_b) {
    gl3_init();
    double cuts[40];
    int nc = 0;
    cuts[nc++] = th_a;
    const int NSUB = 4;
    for (int which = 0; which < 4; which++) {
        for (int k = 0; k < NSUB; k++) {
            double a = th_a + (th_b - th_a) * k / NSUB, b = th_a + (th_b - th_a) * (k + 1) / NSUB;
            double ga = w3_g(c, a, which), gb = w3_g(c, b, which);
            /* a kink exactly on an interior subdivision point is a cut too */
            if (k > 0 && ga == 0.0) cuts[nc++] = a;
            if ((ga < 0.0 && gb > 0.0) || (ga > 0.0 && gb < 0.0)) {
                for (int it = 0; it < 200 && b - a > 1e-17; it++) {
                    double m = 0.5 * (a + b), gm = w3_g(c, m, which);
                    if ((gm < 0.0) == (ga < 0.0)) { a = m; ga = gm; }
                    else b = m;
                }
                cuts[nc++] = 0.5 * (a + b);
            }
        }
    }
    cuts[nc++] = th_b;
    qsort(cuts, nc, sizeof(double), cmp_double);
    double tot = 0.0;
    for (int k = 0; k + 1 < nc; k++) {
        double lo = cuts[k], hi = cuts[k + 1];
        if (!(hi > lo)) continue;
        double h = 0.5 * (hi - lo), m = 0.5 * (hi + lo), s = 0.0;
        for (int i = 0; i < 16; i++) s += g3w[i] * w3_f(c, m + h * g3x[i]);
        tot += h * s;
    }
    return tot / (2.0 * OG_PI);
}

/* ------------------------------------------------------------------ */
/* Sparse per-voxel column                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t* key;
    double* val;
    int64_t cap, n;
} hmap;

static void hm_init(hmap* h, int64_t cap) {
    h->cap = cap;
    h->n = 0;
    h->key = (int64_t*)malloc(sizeof(int64_t) * cap);
    h->val = (double*)calloc(cap, sizeof(double));
    for (int64_t i = 0; i < cap; i++) h->key[i] = -1;
}
static void hm_free(hmap* h) {
    free(h->key);
    free(h->val);
}
static void hm_add(hmap* h, int64_t k, double v);
static void hm_grow(hmap* h) {
    hmap n2;
    hm_init(&n2, h->cap * 2);
    for (int64_t i = 0; i < h->cap; i++)
        if (h->key[i] >= 0) hm_add(&n2, h->key[i], h->val[i]);
    hm_free(h);
    *h = n2;
}
static void hm_add(hmap* h, int64_t k, double v) {
    if (2 * (h->n + 1) > h->cap) hm_grow(h);
    uint64_t x = (uint64_t)k * 0x9E3779B97F4A7C15ull;
    int64_t i = (int64_t)(x >> 20) & (h->cap - 1);
    while (h->key[i] >= 0 && h->key[i] != k) i = (i + 1) & (h->cap - 1);
    if (h->key[i] < 0) {
        h->key[i] = k;
        h->n++;
    }
    h->val[i] += v;
}

/*
 * 3D bin of the crystal pair (g1, r1), (g2, r2): the transaxial pair, ordered
 * (g_i < g_j), then the rings in that order:
 *     bin = tbin(g_i, g_j) * NR^2 + r_i * NR + r_j,
 * tbin the 2D numbering of unordered transaxial pairs.  Pairs with g1 == g2
 * (never joined by a line through the inside of the ring) have no bin: -1.
 */
static int64_t bin3(int64_t g1, int64_t r1, int64_t g2, int64_t r2, int64_t Nc, int64_t NR) {
    if (g1 == g2) return -1;
    if (g1 > g2) {
        int64_t t = g1; g1 = g2; g2 = t;
        t = r1; r1 = r2; r2 = t;
    }
    const int64_t tb = g1 * Nc - g1 * (g1 + 1) / 2 + (g2 - g1 - 1);
    return (tb * NR + r1) * NR + r2;
}

typedef struct {
    int32_t s1, s2;
    double ta, tb;
} tsample;

static int cmp_tsample(const void* x, const void* y) {
    const tsample *a = (const tsample*)x, *b = (const tsample*)y;
    if (a->s1 != b->s1) return (a->s1 > b->s1) - (a->s1 < b->s1);
    return (a->s2 > b->s2) - (a->s2 < b->s2);
}

static int cmp_i64(const void* x, const void* y) {
    int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
    return (a > b) - (a < b);
}

/*
 * Column A[:, v] for the voxel centred at c (3D), accumulated tile by tile:
 * for each pair of crystals (g1, r1), (g2, r2) joined by lines through c, the
 * P^2 x P^2 weights W3 between their sub-patches spread through the response
 * rows into the 5x5 x 5x5 crystal pairs around them (Eq.10, 12).  Returns
 * flags; writes up to cap (bin, value) pairs sorted by bin, *n = count.
 * If grad is given, accumulates d<gy, A x>/d table with voxel value xv
 * instead (gy indexed by bin through gy_bins/gy_vals sorted by bin).
 */
static int column3(const og_geom* G, const og_table* T, const double* c, int64_t cap, int64_t* bins, double* vals,
                   int64_t* n_out, const int64_t* gy_bins, const double* gy_vals, int64_t n_gy, double xv,
                   double* grad) {
    int flags = 0;
    const int P = T->n_sub, nc = G->n_ct, R = G->n_blocks, Nc = R * nc, NR = n_rings(G), NZ = NR * P;
    const int nseg = Nc * P;
    const double lz = G->pitch_z, z0 = z_first(G);
    if (!og_inside_ring(G, c[0], c[1])) flags |= OGF_GEOM;
    double* lo = (double*)malloc(sizeof(double) * nseg);
    double* len = (double*)malloc(sizeof(double) * nseg);
    og_seg_intervals(G, P, c[0], c[1], lo, len);
    /* transaxial samples: the 2D sweep */
    int64_t nts = 0, capts = 1024;
    tsample* ts = (tsample*)malloc(sizeof(tsample) * capts);
    for (int s1 = 0; s1 < nseg; s1++)
        for (int s2 = s1 + 1; s2 < nseg; s2++) {
            double ov = og_overlap_opposite(lo[s1], len[s1], lo[s2], len[s2]);
            if (fabs(ov - OG_EPS_OV) < 1e-13) flags |= OGF_OVERLAP_TIE;
            if (!(ov > OG_EPS_OV)) continue;
            double d = lo[s2] + OG_PI - lo[s1];
            while (d > OG_PI) d -= 2 * OG_PI;
            while (d <= -OG_PI) d += 2 * OG_PI;
            if (nts == capts) {
                capts *= 2;
                ts = (tsample*)realloc(ts, sizeof(tsample) * capts);
            }
            ts[nts].s1 = s1;
            ts[nts].s2 = s2;
            ts[nts].ta = lo[s1] + fmax(0.0, d);
            ts[nts].tb = lo[s1] + fmin(len[s1], d + len[s2]);
            nts++;
        }
    qsort(ts, nts, sizeof(tsample), cmp_tsample);
    /* response rows, computed once per sub-patch when first needed */
    const int64_t nsp = (int64_t)nseg * NZ;
    double* U = (double*)malloc(sizeof(double) * nsp * 25);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * nsp * 25);
    int* uf = (int*)malloc(sizeof(int) * nsp);
    for (int64_t i = 0; i < nsp; i++) uf[i] = -1;
    hmap hm;
    hm_init(&hm, 1 << 20);
    double tile[625];
    /* group transaxial samples by crystal pair (g1, g2) */
    int64_t i0 = 0;
    while (i0 < nts) {
        const int g1 = ts[i0].s1 / P;
        int64_t i1 = i0;
        while (i1 < nts && ts[i1].s1 / P == g1) i1++;
        /* within g1, the distinct g2 */
        for (int64_t a = i0; a < i1; a++) {
            const int g2 = ts[a].s2 / P;
            int seen = 0;
            for (int64_t b = i0; b < a; b++)
                if (ts[b].s2 / P == g2) seen = 1;
            if (seen) continue;
            const int b1 = g1 / nc, b2 = g2 / nc;
            const double ph1 = G->phi0 + 2.0 * OG_PI * b1 / R, ph2 = G->phi0 + 2.0 * OG_PI * b2 / R;
            w3_ctx wc;
            wc.D1 = G->r_face - (cos(ph1) * c[0] + sin(ph1) * c[1]);
            wc.D2 = G->r_face - (cos(ph2) * c[0] + sin(ph2) * c[1]);
            wc.phi1 = ph1;
            wc.phi2 = ph2;
            wc.zv = c[2];
            /* slope range over the pair's directions (conservative) -> ring ranges */
            for (int r1 = 0; r1 < NR; r1++) {
                /* candidate rings r2: photon 2 lands at zv - d2 T for T of ring r1 */
                double zmin = 1e300, zmax = -1e300;
                for (int64_t t = i0; t < i1; t++) {
                    if (ts[t].s2 / P != g2) continue;
                    for (int e = 0; e < 3; e++) {
                        double th = e == 0 ? ts[t].ta : (e == 1 ? ts[t].tb : 0.5 * (ts[t].ta + ts[t].tb));
                        double d1 = wc.D1 / cos(th - ph1), d2 = wc.D2 / -cos(th - ph2);
                        for (int f = 0; f < 2; f++) {
                            double z1 = z0 + (r1 + f) * lz;
                            double z2 = c[2] - d2 * (z1 - c[2]) / d1;
                            zmin = fmin(zmin, z2);
                            zmax = fmax(zmax, z2);
                        }
                    }
                }
                /* z2 is linear in z1, and monotone in theta over a bundle
                 * (d2/d1 is proportional to cos(th - phi1) / cos(th - phi2 - pi),
                 * whose derivative has the sign of sin(phi1 - phi2 - pi) for
                 * every th), so its extremes are at the sampled ends; one ring
                 * more each way absorbs rounding.  og3_set_full_ring_scan(1)
                 * scans every ring instead (the pin of this window). */
                int r2a = (int)floor((zmin - z0) / lz) - 1, r2b = (int)floor((zmax - z0) / lz) + 1;
                if (r2a < 0 || g_full_ring_scan) r2a = 0;
                if (r2b > NR - 1 || g_full_ring_scan) r2b = NR - 1;
                for (int r2 = r2a; r2 <= r2b; r2++) {
                    int any = 0;
                    memset(tile, 0, sizeof(tile));
                    for (int64_t t = i0; t < i1; t++) {
                        if (ts[t].s2 / P != g2) continue;
                        const int pt1 = ts[t].s1 % P, pt2 = ts[t].s2 % P;
                        for (int pz1 = 0; pz1 < P; pz1++) {
                            for (int pz2 = 0; pz2 < P; pz2++) {
                                wc.z1lo = z0 + (r1 + (double)pz1 / P) * lz;
                                wc.z1hi = z0 + (r1 + (double)(pz1 + 1) / P) * lz;
                                wc.z2lo = z0 + (r2 + (double)pz2 / P) * lz;
                                wc.z2hi = z0 + (r2 + (double)(pz2 + 1) / P) * lz;
                                const double w = og_w3(&wc, ts[t].ta, ts[t].tb);
                                if (fabs(w - OG3_EPS_W) < 0.9 * OG3_EPS_W) flags |= OGF_OVERLAP_TIE;
                                if (!(w > OG3_EPS_W)) continue;
                                const int64_t q1 = ((int64_t)(g1 * P + pt1)) * NZ + (r1 * P + pz1);
                                const int64_t q2 = ((int64_t)(g2 * P + pt2)) * NZ + (r2 * P + pz2);
                                if (uf[q1] < 0) uf[q1] = og_uv_row_3d(G, T, c, g1, pt1, r1, pz1, U + q1 * 25, S + q1 * 25);
                                if (uf[q2] < 0) uf[q2] = og_uv_row_3d(G, T, c, g2, pt2, r2, pz2, U + q2 * 25, S + q2 * 25);
                                flags |= uf[q1] | uf[q2];
                                const double* u = U + q1 * 25;
                                const double* v = U + q2 * 25;
                                if (grad) {
                                    const int32_t* su = S + q1 * 25;
                                    const int32_t* sv = S + q2 * 25;
                                    for (int ia = 0; ia < 25; ia++) {
                                        const int ct1 = ((g1 + ia / 5 - 2) % Nc + Nc) % Nc, rr1 = r1 + ia % 5 - 2;
                                        if (rr1 < 0 || rr1 >= NR) continue;
                                        for (int ib = 0; ib < 25; ib++) {
                                            const int ct2 = ((g2 + ib / 5 - 2) % Nc + Nc) % Nc, rr2 = r2 + ib % 5 - 2;
                                            if (rr2 < 0 || rr2 >= NR) continue;
                                            const int64_t bin = bin3(ct1, rr1, ct2, rr2, Nc, NR);
                                            if (bin < 0) continue;
                                            const int64_t* f = (const int64_t*)bsearch(&bin, gy_bins, n_gy,
                                                                                       sizeof(int64_t), cmp_i64);
                                            if (!f) continue;
                                            const double gg = gy_vals[f - gy_bins] * w * xv;
                                            if (su[ia] >= 0) grad[su[ia]] += gg * v[ib];
                                            if (sv[ib] >= 0) grad[sv[ib]] += gg * u[ia];
                                        }
                                    }
                                } else {
                                    for (int ia = 0; ia < 25; ia++) {
                                        if (u[ia] == 0.0) continue;
                                        const double wu = w * u[ia];
                                        for (int ib = 0; ib < 25; ib++) tile[ia * 25 + ib] += wu * v[ib];
                                    }
                                    any = 1;
                                }
                            }
                        }
                    }
                    if (!any) continue;
                    for (int ia = 0; ia < 25; ia++) {
                        const int ct1 = ((g1 + ia / 5 - 2) % Nc + Nc) % Nc, rr1 = r1 + ia % 5 - 2;
                        if (rr1 < 0 || rr1 >= NR) continue;
                        for (int ib = 0; ib < 25; ib++) {
                            const double t = tile[ia * 25 + ib];
                            if (t == 0.0) continue;
                            const int ct2 = ((g2 + ib / 5 - 2) % Nc + Nc) % Nc, rr2 = r2 + ib % 5 - 2;
                            if (rr2 < 0 || rr2 >= NR) continue;
                            const int64_t bin = bin3(ct1, rr1, ct2, rr2, Nc, NR);
                            if (bin < 0) continue;
                            hm_add(&hm, bin, t);
                        }
                    }
                }
            }
        }
        i0 = i1;
    }
    /* sorted output */
    int64_t n = 0;
    if (!grad) {
        int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (hm.n + 1));
        for (int64_t i = 0; i < hm.cap; i++)
            if (hm.key[i] >= 0) keys[n++] = hm.key[i];
        qsort(keys, n, sizeof(int64_t), cmp_i64);
        for (int64_t i = 0; i < n && i < cap; i++) {
            bins[i] = keys[i];
            uint64_t x = (uint64_t)keys[i] * 0x9E3779B97F4A7C15ull;
            int64_t h = (int64_t)(x >> 20) & (hm.cap - 1);
            while (hm.key[h] != keys[i]) h = (h + 1) & (hm.cap - 1);
            vals[i] = hm.val[h];
        }
        free(keys);
    }
    *n_out = n;
    hm_free(&hm);
    free(U); free(S); free(uf); free(ts); free(lo); free(len);
    return flags;
}

/* Columns for a list of voxels: bins[k][cap], vals[k][cap], counts[k], flags[k]. */
void og_columns_3d(const og_geom* G, const og_table* T, const og_image* I, const int64_t* vox, int64_t nvox,
                   int64_t cap, int64_t* bins, double* vals, int64_t* counts, int32_t* flags, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < nvox; k++) {
        double c[3];
        og_voxel_centre(I, vox[k], c);
        flags[k] = column3(G, T, c, cap, bins + k * cap, vals + k * cap, counts + k, NULL, NULL, 0, 0.0, NULL);
    }
}

/* d <gy, A x> / d table over the voxels with x != 0 (gy sparse, sorted bins) */
void og_table_grad_3d(const og_geom* G, const og_table* T, const og_image* I, const int64_t* vox, const double* xv,
                      int64_t nvox, const int64_t* gy_bins, const double* gy_vals, int64_t n_gy, double* grad,
                      int nthreads) {
    const int64_t tsize = (int64_t)T->n_rows * T->n_rows * T->n_sub * T->n_sub * 25;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double* part = (double*)calloc(tsize, sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t k = 0; k < nvox; k++) {
            double c[3];
            int64_t n = 0;
            og_voxel_centre(I, vox[k], c);
            column3(G, T, c, 0, NULL, NULL, &n, gy_bins, gy_vals, n_gy, xv[k], part);
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        for (int64_t e = 0; e < tsize; e++) grad[e] += part[e];
        free(part);
    }
}

/* W3 for one pair of sub-patches seen from c (for tests) */
double og_w3_pair(const og_geom* G, int P, const double* c, int s1, int q1, int s2, int q2) {
    const int nc = G->n_ct, R = G->n_blocks, nseg = R * nc * P;
    const double lz = G->pitch_z, z0 = z_first(G);
    double* lo = (double*)malloc(sizeof(double) * nseg);
    double* len = (double*)malloc(sizeof(double) * nseg);
    og_seg_intervals(G, P, c[0], c[1], lo, len);
    double ov = og_overlap_opposite(lo[s1], len[s1], lo[s2], len[s2]);
    double out = 0.0;
    if (ov > OG_EPS_OV) {
        double d = lo[s2] + OG_PI - lo[s1];
        while (d > OG_PI) d -= 2 * OG_PI;
        while (d <= -OG_PI) d += 2 * OG_PI;
        const int b1 = (s1 / P) / nc, b2 = (s2 / P) / nc;
        w3_ctx wc;
        wc.phi1 = G->phi0 + 2.0 * OG_PI * b1 / R;
        wc.phi2 = G->phi0 + 2.0 * OG_PI * b2 / R;
        wc.D1 = G->r_face - (cos(wc.phi1) * c[0] + sin(wc.phi1) * c[1]);
        wc.D2 = G->r_face - (cos(wc.phi2) * c[0] + sin(wc.phi2) * c[1]);
        wc.zv = c[2];
        wc.z1lo = z0 + (double)q1 * lz / P;
        wc.z1hi = z0 + (double)(q1 + 1) * lz / P;
        wc.z2lo = z0 + (double)q2 * lz / P;
        wc.z2hi = z0 + (double)(q2 + 1) * lz / P;
        out = og_w3(&wc, lo[s1] + fmax(0.0, d), lo[s1] + fmin(len[s1], d + len[s2]));
    }
    free(lo);
    free(len);
    return out;
}
