/*
 * psf_oracle.c -- FP64 CPU oracle for the P-SPIR PSF system matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load it; the library never includes, links or
 * calls it, and it shares no code with the library.
 *
 * Paper: Sun et al., "Fast and accurate generation method of PSF-based system
 * matrix for PET reconstruction" (Chinese Physics C, 2016; arXiv 1607.06170).
 *
 * What is computed, in the paper's order (2D single ring; the 3D extension is
 * in psf_oracle3d.c):
 *   - response table rho[angle][sub-position][neighbour]   Sec 2.1.1, Eq.1, 6, 7
 *   - two-block penetration remap (beta, AP^1, n)          Sec 2.1.2, Eq.2, 4, 5
 *   - LOR probability as product of single responses       Sec 2.2, Eq.10
 *   - homogenization weights (k -> infinity, or finite k)  Sec 2.3, Eq.11
 *   - spread of each homogenized LOR into crystal pairs    Sec 2.3, Eq.12
 * Every floating-point quantity is FP64.  Compile with -ffp-contract=off.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - The table is the analytic first-interaction probability in a laterally
 *     unbounded crystal array (attenuation only), averaged over each
 *     sub-position; it stands in for the GATE simulation of Eq.1.
 *   - Neighbours beyond +-2 crystals are dropped, not renormalised.
 *   - The incidence angle and position of a sub-segment are those of the line
 *     from the voxel centre to the sub-segment centre.
 *   - Angle rows: nearest row, floor(|alpha|/step + 1/2).
 *   - A line counts for a pair of sub-segments only where both ends land on a
 *     crystal front face; lines through a gap contribute nothing.
 *   - Overlaps of at most OG_EPS_OV radians are treated as empty (a line set
 *     of zero measure).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_PI 3.14159265358979323846
#define OG_NB 5          /* neighbours per axis: offsets -2..2 */
#define OG_EPS_OV 1e-12  /* overlaps at or below this (rad) are empty */

/* flag bits returned with every result: decisions taken within a hair of a
 * boundary (where a second FP64 implementation may legitimately decide the
 * other way), and range errors */
#define OGF_MIRROR_TIE 1
#define OGF_ROW_TIE 2
#define OGF_OVERLAP_TIE 4
#define OGF_REMAP_TIE 8
#define OGF_RANGE 16
#define OGF_GEOM 32

typedef struct {
    int32_t n_blocks;  /* R, blocks per ring (Eq.2) */
    int32_t n_ct;      /* crystals per block, transaxial */
    int32_t n_cz;      /* crystals per block, axial */
    int32_t n_brings;  /* block rings along z */
    double pitch_t;    /* lambda, crystal width transaxially (Eq.5) */
    double pitch_z;    /* crystal width axially */
    double depth;      /* crystal length L */
    double r_face;     /* distance from the ring centre to each block front face */
    double gap_z;      /* axial gap between block rings */
    double mu;         /* linear attenuation coefficient (1/mm) */
    double phi0;       /* angle of block 0's outward normal */
} og_geom;

typedef struct {
    int32_t nx, ny, nz, pad;
    double dx, dy, dz, cx, cy, cz;
} og_image;

typedef struct {
    int32_t n_rows;   /* angle rows (per axis in 3D) */
    int32_t n_sub;    /* sub-positions per crystal (per axis in 3D) */
    double step_deg;  /* angle step between rows */
    const double* data;
} og_table;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* angle wrapped into (-pi, pi] */
static double wrap_pm_pi(double a) {
    while (a > OG_PI) a -= 2.0 * OG_PI;
    while (a <= -OG_PI) a += 2.0 * OG_PI;
    return a;
}

/* angle wrapped into [0, 2 pi) */
static double wrap_2pi(double a) {
    while (a >= 2.0 * OG_PI) a -= 2.0 * OG_PI;
    while (a < 0.0) a += 2.0 * OG_PI;
    return a;
}

static int near_half_int(double f) { /* f within 1e-9 of k + 1/2 */
    double r = f - floor(f);
    return fabs(r - 0.5) < 1e-9;
}
static int near_int(double f) { return fabs(f - nearbyint(f)) < 1e-9; }

/* Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n. */
void og_gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; i++) {
        double z = cos(OG_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; k++) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            double dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) {
                /* recompute the derivative at the converged node */
                p0 = 1.0; p1 = 0.0;
                for (int k = 1; k <= n; k++) {
                    double p2 = p1;
                    p1 = p0;
                    p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
                }
                dp = n * (z * p0 - p1) / (z * z - 1.0);
                break;
            }
        }
        x[i] = z;
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; k++) {
            double p2 = p1;
            p1 = p0;
            p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        double dp = n * (z * p0 - p1) / (z * z - 1.0);
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

#define OG_GL_N 16
static double g_glx[OG_GL_N], g_glw[OG_GL_N];
static int g_gl_ready = 0;
static void gl_init(void) {
    if (!g_gl_ready) {
        og_gauss_legendre(OG_GL_N, g_glx, g_glw);
        g_gl_ready = 1;
    }
}

/* ------------------------------------------------------------------ */
/* Response model (Sec 2.1.1, Eq.1; normalisation Eq.6-7)              */
/* ------------------------------------------------------------------ */

/*
 * Probability that a photon entering the front face of an unbounded row of
 * crystals (width lam, depth L, attenuation mu) makes its first interaction in
 * the crystal at offset a from the entry crystal.  It enters at lateral offset
 * u in [0, lam) from the entry crystal's lower edge, tilted by alpha >= 0
 * towards increasing offsets.  Along the path s the lateral position is
 * u + s sin(alpha) and the depth s cos(alpha); the path leaves the array at
 * depth L.  The probability is absolute (Eq.6-7: already multiplied by the
 * detection efficiency), so summed over all offsets it is 1 - exp(-mu L/cos a).
 */
double og_rho_point(double alpha, double u, int a, double lam, double L, double mu) {
    if (a < 0) return 0.0;
    if (alpha == 0.0) return a == 0 ? 1.0 - exp(-mu * L) : 0.0;
    double sa = sin(alpha);
    double smax = L / cos(alpha);
    double s_in = clampd((a * lam - u) / sa, 0.0, smax);
    double s_out = clampd(((a + 1) * lam - u) / sa, 0.0, smax);
    if (!(s_out > s_in)) return 0.0;
    return exp(-mu * s_in) - exp(-mu * s_out);
}

static int cmp_double(const void* x, const void* y) {
    double a = *(const double*)x, b = *(const double*)y;
    return (a > b) - (a < b);
}

/*
 * Average of og_rho_point over the sub-position p of P equal parts of the entry
 * crystal (u in [p lam/P, (p+1) lam/P)).  The integrand is smooth between the
 * points where the path starts or stops touching crystal a, so the interval is
 * split there and each piece integrated with 16-point Gauss-Legendre.
 */
double og_rho_sub(double alpha, int p, int P, int a, double lam, double L, double mu) {
    gl_init();
    double u0 = p * lam / P, u1 = (p + 1) * lam / P;
    double cuts[8];
    int nc = 0;
    cuts[nc++] = u0;
    if (alpha > 0.0) {
        double reach = L * tan(alpha); /* lateral travel across the full depth */
        double cand[4] = {a * lam, a * lam - reach, (a + 1) * lam, (a + 1) * lam - reach};
        for (int i = 0; i < 4; i++)
            if (cand[i] > u0 && cand[i] < u1) cuts[nc++] = cand[i];
    }
    cuts[nc++] = u1;
    qsort(cuts, nc, sizeof(double), cmp_double);
    double total = 0.0;
    for (int k = 0; k + 1 < nc; k++) {
        double lo = cuts[k], hi = cuts[k + 1];
        if (!(hi > lo)) continue;
        double h = 0.5 * (hi - lo), m = 0.5 * (hi + lo);
        double s = 0.0;
        for (int i = 0; i < OG_GL_N; i++) s += g_glw[i] * og_rho_point(alpha, m + h * g_glx[i], a, lam, L, mu);
        total += h * s;
    }
    return total / (u1 - u0);
}

/* Table rho[row][p][a+2], row angle = row * step_deg degrees, a in -2..2. */
void og_table_2d(const og_geom* G, int n_rows, int P, double step_deg, double* out) {
    for (int r = 0; r < n_rows; r++) {
        double alpha = r * step_deg * OG_PI / 180.0;
        for (int p = 0; p < P; p++)
            for (int a = -2; a <= 2; a++)
                out[(r * P + p) * OG_NB + (a + 2)] = og_rho_sub(alpha, p, P, a, G->pitch_t, G->depth, G->mu);
    }
}

/* ------------------------------------------------------------------ */
/* Gap process (Sec 2.1.2, Eq.2, 4, 5)                                 */
/* ------------------------------------------------------------------ */

/* sigma: the gap half-length AB = BC, from the corner C of block 0 to the
 * vertex B where the face lines of two neighbouring blocks meet. */
double og_sigma(const og_geom* G) {
    return G->r_face * tan(OG_PI / G->n_blocks) - 0.5 * G->n_ct * G->pitch_t;
}

/* Eq.4: AP^1 for a ray entering block 0 at distance nu from its edge with
 * incidence angle alpha (towards the edge), beta from Eq.2. */
double og_ap1(const og_geom* G, double alpha, double nu) {
    double beta = alpha - 2.0 * OG_PI / G->n_blocks; /* Eq.2 */
    double sigma = og_sigma(G);
    return sigma + sin(OG_PI / 2 - alpha) / sin(OG_PI / 2 + beta) * (sigma + nu);
}

/* ------------------------------------------------------------------ */
/* Geometry of the 2D ring                                             */
/* ------------------------------------------------------------------ */

/* point on block b's front face line at lateral coordinate xi */
static void face_point(const og_geom* G, int b, double xi, double* px, double* py) {
    double phi = G->phi0 + 2.0 * OG_PI * b / G->n_blocks;
    double nx = cos(phi), ny = sin(phi);
    double tx = -ny, ty = nx;
    *px = G->r_face * nx + xi * tx;
    *py = G->r_face * ny + xi * ty;
}

/* lateral coordinate of boundary k (0..n_ct*P) on a block face */
static double boundary_xi(const og_geom* G, int P, int k) {
    double W = G->n_ct * G->pitch_t;
    return -0.5 * W + k * (G->pitch_t / P);
}

/* true when (vx, vy) lies strictly inside every block's front-face line */
int og_inside_ring(const og_geom* G, double vx, double vy) {
    for (int b = 0; b < G->n_blocks; b++) {
        double phi = G->phi0 + 2.0 * OG_PI * b / G->n_blocks;
        if (!(cos(phi) * vx + sin(phi) * vy < G->r_face)) return 0;
    }
    return 1;
}

/*
 * Response row of sub-segment (g, p) seen from (vx, vy): val[a+2] is the
 * response of crystal g+a (global numbering, a in -2..2) and src[a+2] the
 * table entry it came from (-1 when the response is zero by construction).
 * Returns flag bits.
 */
int og_uv_row_2d(const og_geom* G, const og_table* T, double vx, double vy, int g, int p, double* val,
                 int32_t* src) {
    int flags = 0;
    int nc = G->n_ct, R = G->n_blocks, P = T->n_sub;
    double lam = G->pitch_t, W = nc * lam;
    int b = g / nc, c = g % nc;
    double phi = G->phi0 + 2.0 * OG_PI * b / R;
    double nx = cos(phi), ny = sin(phi), tx = -ny, ty = nx;
    double xi_m = -0.5 * W + (c + (p + 0.5) / P) * lam; /* incidence position: sub-segment centre */
    double D = G->r_face - (nx * vx + ny * vy);           /* distance from the voxel to the face line */
    double tan_a = (xi_m - (tx * vx + ty * vy)) / D;
    double alpha = atan(tan_a);
    if (fabs(tan_a) < 1e-12) flags |= OGF_MIRROR_TIE;
    int mirror = alpha < 0.0;
    double aa = fabs(alpha);
    double frow = aa * 180.0 / OG_PI / T->step_deg;
    if (near_half_int(frow)) flags |= OGF_ROW_TIE;
    int row = (int)floor(frow + 0.5);
    if (row > T->n_rows - 1) {
        flags |= OGF_RANGE;
        row = T->n_rows - 1;
    }
    /* frame in which the photon leans towards increasing crystal index */
    int cm = mirror ? nc - 1 - c : c;
    int pm = mirror ? P - 1 - p : p;
    double nu = mirror ? xi_m + 0.5 * W : 0.5 * W - xi_m; /* distance to the approached edge */
    for (int am = -2; am <= 2; am++) {
        int a = mirror ? -am : am;
        int cc = cm + am;
        double v = 0.0;
        int32_t s = -1;
        if (cc >= 0 && cc < nc) {
            s = (row * P + pm) * OG_NB + (am + 2);
            v = T->data[s];
        } else if (cc >= nc) {
            /* crystal of the next block: equivalent incidence (Eq.2, 4, 5) */
            double beta = aa - 2.0 * OG_PI / R;
            if (fabs(beta) < 1e-12) flags |= OGF_REMAP_TIE;
            if (beta > 0.0) {
                double ap1 = og_ap1(G, aa, nu);
                double n = ap1 / lam;
                if (near_int(n)) flags |= OGF_REMAP_TIE;
                int k = (int)ceil(n) - 1;      /* virtual crystals before the block's first crystal */
                double up = (k + 1) - n;       /* entry offset in the virtual crystal, in crystal widths */
                if (near_int(up * P)) flags |= OGF_REMAP_TIE;
                int p1 = (int)floor(up * P);
                int m = cc - nc;               /* crystal of the next block, counted from its near edge */
                int idx = k + 1 + m;           /* offset from the virtual entry crystal */
                double fb = beta * 180.0 / OG_PI / T->step_deg;
                if (near_half_int(fb)) flags |= OGF_ROW_TIE;
                int rowb = (int)floor(fb + 0.5);
                if (rowb > T->n_rows - 1) {
                    flags |= OGF_RANGE;
                    rowb = T->n_rows - 1;
                }
                if (idx <= 2) {
                    s = (rowb * P + p1) * OG_NB + (idx + 2);
                    v = T->data[s];
                }
            }
        }
        /* cc < 0: crystals behind the receding edge, across a gap: no response */
        val[a + 2] = v;
        src[a + 2] = s;
    }
    return flags;
}

/* canonical index of the unordered crystal pair (i, j), i != j, among
 * n*(n-1)/2 pairs ordered by (min, max) */
static int64_t pair_bin(int64_t i, int64_t j, int64_t n) {
    if (i > j) {
        int64_t t = i;
        i = j;
        j = t;
    }
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}

/* direction interval [lo, lo + len) of every sub-segment seen from (vx, vy) */
void og_seg_intervals(const og_geom* G, int P, double vx, double vy, double* lo, double* len) {
    int nc = G->n_ct, R = G->n_blocks;
    for (int b = 0; b < R; b++) {
        for (int c = 0; c < nc; c++) {
            for (int p = 0; p < P; p++) {
                int k = c * P + p;
                double x0, y0, x1, y1;
                face_point(G, b, boundary_xi(G, P, k), &x0, &y0);
                face_point(G, b, boundary_xi(G, P, k + 1), &x1, &y1);
                double t0 = atan2(y0 - vy, x0 - vx);
                double t1 = atan2(y1 - vy, x1 - vx);
                int s = (b * nc + c) * P + p;
                lo[s] = t0;
                len[s] = wrap_2pi(t1 - t0);
            }
        }
    }
}

/* measure of the directions in I1 whose opposite direction lies in I2 */
double og_overlap_opposite(double lo1, double len1, double lo2, double len2) {
    double d = wrap_pm_pi(lo2 + OG_PI - lo1);
    double hi = fmin(len1, d + len2);
    double lo = fmax(0.0, d);
    return hi - lo;
}

/*
 * Homogenization model (Sec 2.3, Eq.11).  Lines through the voxel centre are
 * spread uniformly in direction; a line hitting sub-segments s1 and s2 at its
 * two ends carries weight (its share of the half-turn of directions).
 *   homog_k == 0: the k -> infinity limit, W[s1,s2] = |I(s1) n (I(s2)+pi)| / pi
 *   homog_k  > 0: Eq.11 literally, k lines at theta_i = pi i / k, weight 1/k each
 * Each unordered line is counted once; pairs are reported with s1 < s2.
 * Returns flag bits; *n_out is the number of (s1, s2, w) triples written (at
 * most max_out; the count is still returned in full).
 */
int og_samples_2d(const og_geom* G, int P, double vx, double vy, int homog_k, int64_t max_out, int32_t* s1o,
                  int32_t* s2o, double* wo, int64_t* n_out) {
    int flags = 0;
    int nseg = G->n_blocks * G->n_ct * P;
    double* lo = (double*)malloc(sizeof(double) * nseg);
    double* len = (double*)malloc(sizeof(double) * nseg);
    if (!og_inside_ring(G, vx, vy)) flags |= OGF_GEOM;
    og_seg_intervals(G, P, vx, vy, lo, len);
    int64_t n = 0;
    if (homog_k == 0) {
        for (int s1 = 0; s1 < nseg; s1++) {
            for (int s2 = s1 + 1; s2 < nseg; s2++) {
                double ov = og_overlap_opposite(lo[s1], len[s1], lo[s2], len[s2]);
                if (fabs(ov - OG_EPS_OV) < 1e-13) flags |= OGF_OVERLAP_TIE;
                if (!(ov > OG_EPS_OV)) continue;
                if (n < max_out) {
                    s1o[n] = s1;
                    s2o[n] = s2;
                    wo[n] = ov / OG_PI;
                }
                n++;
            }
        }
    } else {
        for (int i = 0; i < homog_k; i++) {
            double th = OG_PI * i / homog_k;
            int h1 = -1, h2 = -1;
            for (int s = 0; s < nseg; s++) {
                double d1 = wrap_2pi(th - lo[s]);
                double d2 = wrap_2pi(th + OG_PI - lo[s]);
                if (d1 < len[s]) h1 = s;
                if (d2 < len[s]) h2 = s;
            }
            if (h1 < 0 || h2 < 0) continue; /* the line ends in a gap */
            if (n < max_out) {
                s1o[n] = h1 < h2 ? h1 : h2;
                s2o[n] = h1 < h2 ? h2 : h1;
                wo[n] = 1.0 / homog_k;
            }
            n++;
        }
    }
    free(lo);
    free(len);
    *n_out = n;
    return flags;
}

/*
 * Column A[:, v] of the 2D system matrix for a voxel centred at (vx, vy):
 * every homogenized line (s1, s2, w) spreads into the crystal pairs
 * (g1 + a, g2 + b) with probability w * U[s1][a] * U[s2][b] (Eq.10 for each
 * pair of detecting crystals, summed as in Eq.12).  col has n(n-1)/2 entries
 * for n crystals in the ring and is accumulated into (not cleared).
 * If grad != NULL, instead of filling col this accumulates
 * d<gy, A x>/d table into grad with voxel value xv.
 */
static int column_or_grad_2d(const og_geom* G, const og_table* T, double vx, double vy, int homog_k, double* col,
                             const double* gy, double xv, double* grad) {
    int P = T->n_sub;
    int Nc = G->n_blocks * G->n_ct;
    int nseg = Nc * P;
    int64_t maxs = (int64_t)nseg * 8 + (homog_k > 0 ? homog_k : 0);
    int32_t* s1 = (int32_t*)malloc(sizeof(int32_t) * maxs);
    int32_t* s2 = (int32_t*)malloc(sizeof(int32_t) * maxs);
    double* w = (double*)malloc(sizeof(double) * maxs);
    int64_t ns = 0;
    int flags = og_samples_2d(G, P, vx, vy, homog_k, maxs, s1, s2, w, &ns);
    if (ns > maxs) { /* more lines than the generous first guess: redo with room */
        free(s1); free(s2); free(w);
        maxs = ns;
        s1 = (int32_t*)malloc(sizeof(int32_t) * maxs);
        s2 = (int32_t*)malloc(sizeof(int32_t) * maxs);
        w = (double*)malloc(sizeof(double) * maxs);
        flags = og_samples_2d(G, P, vx, vy, homog_k, maxs, s1, s2, w, &ns);
    }
    double* U = (double*)malloc(sizeof(double) * nseg * OG_NB);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * nseg * OG_NB);
    int* rf = (int*)malloc(sizeof(int) * nseg);
    for (int s = 0; s < nseg; s++) rf[s] = og_uv_row_2d(G, T, vx, vy, s / P, s % P, U + s * OG_NB, S + s * OG_NB);
    for (int64_t k = 0; k < ns; k++) {
        int a1 = s1[k], a2 = s2[k];
        flags |= rf[a1] | rf[a2];
        int g1 = a1 / P, g2 = a2 / P;
        for (int a = -2; a <= 2; a++) {
            for (int b = -2; b <= 2; b++) {
                int i = ((g1 + a) % Nc + Nc) % Nc;
                int j = ((g2 + b) % Nc + Nc) % Nc;
                if (i == j) continue;
                int64_t bin = pair_bin(i, j, Nc);
                double u = U[a1 * OG_NB + a + 2], v = U[a2 * OG_NB + b + 2];
                if (grad == NULL) {
                    col[bin] += w[k] * u * v;
                } else {
                    double gg = gy[bin] * w[k] * xv;
                    int32_t su = S[a1 * OG_NB + a + 2], sv = S[a2 * OG_NB + b + 2];
                    if (su >= 0) grad[su] += gg * v;
                    if (sv >= 0) grad[sv] += gg * u;
                }
            }
        }
    }
    free(s1); free(s2); free(w); free(U); free(S); free(rf);
    return flags;
}

int og_column_2d(const og_geom* G, const og_table* T, double vx, double vy, int homog_k, double* col) {
    return column_or_grad_2d(G, T, vx, vy, homog_k, col, NULL, 0.0, NULL);
}

/* voxel centre of linear index j (x fastest, then y, then z) */
void og_voxel_centre(const og_image* I, int64_t j, double* c) {
    int64_t ix = j % I->nx, iy = (j / I->nx) % I->ny, iz = j / ((int64_t)I->nx * I->ny);
    c[0] = (ix - 0.5 * (I->nx - 1)) * I->dx + I->cx;
    c[1] = (iy - 0.5 * (I->ny - 1)) * I->dy + I->cy;
    c[2] = (iz - 0.5 * (I->nz - 1)) * I->dz + I->cz;
}

/* Dense columns for a list of voxels: out[k][bin] (FP64), flags[k]. */
void og_columns_2d(const og_geom* G, const og_table* T, const og_image* I, const int64_t* vox, int64_t nvox,
                   int homog_k, double* out, int32_t* flags, int nthreads) {
    int64_t Nc = (int64_t)G->n_blocks * G->n_ct;
    int64_t nbins = Nc * (Nc - 1) / 2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < nvox; k++) {
        double c[3];
        og_voxel_centre(I, vox[k], c);
        double* col = out + k * nbins;
        memset(col, 0, sizeof(double) * nbins);
        flags[k] = og_column_2d(G, T, c[0], c[1], homog_k, col);
    }
}

/*
 * Gradient of <gy, A x> with respect to every table entry (the table enters
 * A through U and V only; each U or V entry is one table entry or zero).
 * grad has the table's size and is accumulated into.  x covers all voxels.
 */
void og_table_grad_2d(const og_geom* G, const og_table* T, const og_image* I, const double* x, const double* gy,
                      int homog_k, double* grad, int nthreads) {
    int64_t nvox = (int64_t)I->nx * I->ny;
    int64_t tsize = (int64_t)T->n_rows * T->n_sub * OG_NB;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double* part = (double*)calloc(tsize, sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int64_t j = 0; j < nvox; j++) {
            if (x[j] == 0.0) continue;
            double c[3];
            og_voxel_centre(I, j, c);
            column_or_grad_2d(G, T, c[0], c[1], homog_k, NULL, gy, x[j], part);
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        for (int64_t e = 0; e < tsize; e++) grad[e] += part[e];
        free(part);
    }
}
