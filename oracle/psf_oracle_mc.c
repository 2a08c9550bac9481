/*
 * psf_oracle_mc.c -- FP64 CPU oracle of the photon-transport Monte Carlo that
 * estimates the single-photon response table.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load it; the library never includes, links or
 * calls it, and it shares no code with the library.
 *
 * Paper: Sun et al., "Fast and accurate generation method of PSF-based system
 * matrix for PET reconstruction" (Chinese Physics C, 2016; arXiv 1607.06170).
 * Sec 2.1.1 (Eq.1) obtains the response of a crystal array to a photon
 * entering at sub-position p with incidence angle alpha by Monte Carlo
 * simulation (GATE in the paper, with a biased source); Sec 2.1.3 (Eq.6-7)
 * indexes the result by angle row and sub-position.  This oracle estimates
 * the same table with an in-house photon transport:
 *
 *   - geometry: a crystal array unbounded laterally (pitch pitch_t across,
 *     pitch_z along the axis in 3D; unbounded along the axis in 2D), depth
 *     `depth`, front face z = 0; the photon enters uniformly over the
 *     sub-position of crystal 0 (p / n_sub .. (p + 1) / n_sub of the pitch)
 *     with direction (tan alpha_t, tan alpha_z, 1) normalised; in 2D
 *     alpha_z = 0.  Angle row r is the angle r * step_deg.
 *   - mode 0 (first interaction): the path length to the first interaction
 *     is exponential with attenuation mu; the photon counts for the crystal
 *     that holds that point if it lies inside the depth.  Its expectation is
 *     the analytic table of psf_oracle.c / psf_oracle3d.c.
 *   - mode 1 (with Compton scatter): at 511 keV the attenuation splits into
 *     photoelectric absorption (a fraction f_pe = 0.32 of mu) and Compton
 *     scatter.  At lower energy E the photoelectric part scales as
 *     (511 / E)^3 and the Compton part as the Klein-Nishina cross section;
 *     Rayleigh scatter, fluorescence and electron range are neglected.  A
 *     Compton event deposits E - E' where it happens and turns the photon by
 *     an angle drawn from the Klein-Nishina distribution (rejection against
 *     its value 2 at theta = 0) and a uniform azimuth; a photon leaving
 *     through the front or back face is lost.  The event counts when the
 *     energy deposited reaches 350 keV (the lower energy threshold), in the
 *     crystal that holds the energy-weighted centroid of the deposits (the
 *     block detector's positioning).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC 2011), counter {photon index low,
 * photon index high, table cell, draw}, key {seed low, seed high}; each draw
 * gives two uniforms in (0, 1) from 53 bits of two output words.  The GPU
 * library implements the same generator from the same definition, so the two
 * sides can follow the same photons.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static const double kPiMc = 3.14159265358979323846;

/* one Philox4x32 round and the key schedule (the published constants) */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void og_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

/* a uniform in (0, 1): the top 53 bits of (hi, lo), centred in their cell */
static double u01(uint32_t hi, uint32_t lo) {
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return ((double)v + 0.5) * 0x1p-53;
}

typedef struct {
    uint32_t ctr[4], key[2];
} Stream;

static void draw2(Stream* s, double* a, double* b) {
    uint32_t o[4];
    og_philox4x32_10(s->ctr, s->key, o);
    s->ctr[3] += 1;
    *a = u01(o[0], o[1]);
    *b = u01(o[2], o[3]);
}

/* Klein-Nishina total cross section, up to a constant, at k = E / 511 keV */
static double kn_sigma(double k) {
    const double l = log(1.0 + 2.0 * k);
    return (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k) + l / (2.0 * k) -
           (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
}

double og_kn_sigma(double k) { return kn_sigma(k); }

/* cos(theta) of a Compton scatter at k = E / 511 keV: a candidate uniform in
 * [-1, 1] is kept with probability f / 2, f = eps^2 (eps + 1 / eps - sin^2)
 * the Klein-Nishina shape (2 at theta = 0, its largest); at most 64 trials */
static double kn_cos(double k, Stream* s, double* eps_out) {
    double c = 1.0, eps = 1.0;
    for (int t = 0; t < 64; ++t) {
        double ua, ub;
        draw2(s, &ua, &ub);
        c = 2.0 * ua - 1.0;
        eps = 1.0 / (1.0 + k * (1.0 - c));
        const double f = eps * eps * (eps + 1.0 / eps - (1.0 - c * c));
        if (ub * 2.0 < f) break;
    }
    *eps_out = eps;
    return c;
}

/* n samples of cos(theta) at k, photon i on counter {i, 0, 0, draw} */
void og_kn_cos_samples(double k, int64_t n, uint64_t seed, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        Stream s = {{(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u}, {(uint32_t)seed, (uint32_t)(seed >> 32)}};
        double eps;
        out[i] = kn_cos(k, &s, &eps);
    }
}

/* the detected offset (at, az) of one photon, or 0 when it is not detected */
static int one_photon(int mode3d, int scatter, int pt, int pz, int n_sub, double tt, double tz, double pitch_t,
                      double pitch_z, double depth, double mu, Stream* s, int* at, int* az) {
    double u0, u1, u2, u3;
    draw2(s, &u0, &u1);
    const double x0 = (pt + u0) / n_sub * pitch_t;
    const double y0 = mode3d ? (pz + u1) / n_sub * pitch_z : 0.0;
    const double kk = sqrt(1.0 + tt * tt + tz * tz);
    if (!scatter) {
        draw2(s, &u2, &u3);
        const double d = -log(u2) / mu / kk;  /* depth of the first interaction */
        if (!(d < depth)) return 0;
        *at = (int)floor((x0 + d * tt) / pitch_t);
        *az = mode3d ? (int)floor((y0 + d * tz) / pitch_z) : 0;
        return 1;
    }
    const double f_pe = 0.32, e_thr = 350.0, s511 = kn_sigma(1.0);
    double x = x0, y = y0, z = 0.0, u = tt / kk, v = tz / kk, w = 1.0 / kk, e = 511.0;
    double ed = 0.0, ex = 0.0, ey = 0.0;
    for (int it = 0; it < 64; ++it) {
        const double k = e / 511.0;
        const double r = 511.0 / e;
        const double m_pe = f_pe * mu * r * r * r, m_c = (1.0 - f_pe) * mu * kn_sigma(k) / s511;
        draw2(s, &u2, &u3);
        const double step = -log(u2) / (m_pe + m_c);
        x += step * u;
        y += step * v;
        z += step * w;
        if (z < 0.0 || z > depth) break;  /* leaves the array */
        if (u3 * (m_pe + m_c) < m_pe) {   /* photoelectric absorption */
            ed += e;
            ex += e * x;
            ey += e * y;
            break;
        }
        double eps;
        const double c = kn_cos(k, s, &eps);  /* Compton: the scattering angle */
        double uf, unused;
        draw2(s, &uf, &unused);
        const double phi = 2.0 * kPiMc * uf;
        const double e2 = e * eps;
        ed += e - e2;
        ex += (e - e2) * x;
        ey += (e - e2) * y;
        e = e2;
        const double sn = sqrt(fmax(0.0, 1.0 - c * c)), cp = cos(phi), sp = sin(phi);
        double nu, nv, nw;
        if (fabs(w) > 0.99999) {
            nu = sn * cp;
            nv = sn * sp;
            nw = (w > 0.0 ? c : -c);
        } else {
            const double q = sqrt(1.0 - w * w);
            nu = sn * (u * w * cp - v * sp) / q + u * c;
            nv = sn * (v * w * cp + u * sp) / q + v * c;
            nw = -sn * cp * q + w * c;
        }
        u = nu;
        v = nv;
        w = nw;
        if (e < 1.0) {  /* the rest is absorbed where it is */
            ed += e;
            ex += e * x;
            ey += e * y;
            break;
        }
    }
    if (!(ed >= e_thr)) return 0;
    *at = (int)floor(ex / ed / pitch_t);
    *az = mode3d ? (int)floor(ey / ed / pitch_z) : 0;
    return 1;
}

/* Detected-photon counts of table cells [cell_begin, cell_end): counts has
 * (cell_end - cell_begin) x 25 entries, [a_t + 2][a_z + 2] (2D: a_z = 0, so
 * entries [a_t + 2][2]).  Cell numbering: 2D row * n_sub + p; 3D
 * ((row_t * n_rows + row_z) * n_sub + p_t) * n_sub + p_z. */
void og_table_mc(int mode3d, int n_rows, int n_sub, double step_deg, double pitch_t, double pitch_z, double depth,
                 double mu, int64_t photons, uint64_t seed, int scatter, int64_t cell_begin, int64_t cell_end,
                 int64_t* counts, int nthreads) {
    (void)nthreads;
    const int64_t nc = cell_end - cell_begin;
    memset(counts, 0, sizeof(int64_t) * 25 * (size_t)(nc > 0 ? nc : 0));
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t ci = 0; ci < nc; ++ci) {
        const int64_t cell = cell_begin + ci;
        int rt, rz, pt, pz;
        if (mode3d) {
            pz = (int)(cell % n_sub);
            pt = (int)((cell / n_sub) % n_sub);
            rz = (int)((cell / ((int64_t)n_sub * n_sub)) % n_rows);
            rt = (int)(cell / ((int64_t)n_sub * n_sub * n_rows));
        } else {
            pt = (int)(cell % n_sub);
            rt = (int)(cell / n_sub);
            rz = 0;
            pz = 0;
        }
        const double tt = tan(rt * step_deg * kPiMc / 180.0), tz = mode3d ? tan(rz * step_deg * kPiMc / 180.0) : 0.0;
        int64_t* out = counts + 25 * ci;
        for (int64_t k = 0; k < photons; ++k) {
            Stream s;
            s.ctr[0] = (uint32_t)k;
            s.ctr[1] = (uint32_t)((uint64_t)k >> 32);
            s.ctr[2] = (uint32_t)cell;
            s.ctr[3] = 0;
            s.key[0] = (uint32_t)seed;
            s.key[1] = (uint32_t)(seed >> 32);
            int at = 0, az = 0;
            if (!one_photon(mode3d, scatter, pt, pz, n_sub, tt, tz, pitch_t, pitch_z, depth, mu, &s, &at, &az)) continue;
            if (at < -2 || at > 2 || az < -2 || az > 2) continue;
            out[(at + 2) * 5 + (az + 2)] += 1;
        }
    }
}
