/*
 * orc_core.c -- oracle: random numbers, derived constants and the collision
 * sampling formulas.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include "oracle.h"

#include <math.h>

/* CODATA 2018 */
#define ORC_E    1.602176634e-19
#define ORC_ME   9.1093837015e-31
#define ORC_EPS0 8.8541878128e-12
#define ORC_KB   1.380649e-23
#define ORC_AMU  1.66053906660e-27

/*
 * Philox4x32-10 counter-based generator, from its definition in Salmon, Moraes,
 * Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11), Sec. 3:
 * ten rounds, each multiplying counter words 0 and 2 by the two fixed 32-bit
 * multipliers (keeping both halves of the 64-bit products), mixing in the key,
 * and bumping the key by the two Weyl constants between rounds.
 */
static void orc_mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint32_t hi0, lo0, hi1, lo1;
        orc_mulhilo(M0, x0, &hi0, &lo0);
        orc_mulhilo(M1, x2, &hi1, &lo1);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Open-interval uniform from two words: the top 52 bits of hi:lo, centred. */
double orc_u52(uint32_t hi, uint32_t lo) {
    uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

/*
 * Derived constants.  Gas density from pressure and temperature (Sec. II.A:
 * uniform, constant neutral density is an input), null-collision frequency
 * bound nu' = n_n (sigma_el + max sigma_iz) v_cap (null-collision method of
 * the MCC reference cited in Sec. II.A), per-step candidate probability
 * P_null = 1 - exp(-nu' dt).
 */
void orc_derive(const orc_cfg* c, orc_derived* d) {
    d->dr = (c->b - c->a) / (double)c->nr;
    d->dz = c->L / (double)c->nz;
    d->inv_dr = 1.0 / d->dr;
    d->inv_dz = 1.0 / d->dz;
    double qm = -ORC_E / ORC_ME;
    d->h = (0.5 * qm) * c->dt;
    d->n_n = (100.0 * c->p_mbar) / (ORC_KB * c->T_gas_K);
    d->v_cap = sqrt(((2.0 * c->E_cap_eV) * ORC_E) / ORC_ME);
    /* ln(E/I)/(E I) peaks at E = e I (e = Euler's number): max = 1/(e I^2). */
    d->sig_iz_max = (c->lotz_a * c->lotz_q) / ((exp(1.0) * c->iz_I_eV) * c->iz_I_eV);
    d->nu_prime = (d->n_n * (c->sigma_el + d->sig_iz_max)) * d->v_cap;
    d->P_null = -expm1(-(d->nu_prime * c->dt));
    d->nsig_el = d->n_n * c->sigma_el;
    d->lotz_aq = c->lotz_a * c->lotz_q;
    d->half_me_over_e = (0.5 * ORC_ME) / ORC_E;
    d->two_e_over_me = (2.0 * ORC_E) / ORC_ME;
    d->mass_ratio2 = (2.0 * ORC_ME) / (c->M_gas_amu * ORC_AMU);
    d->two_S = ldexp(1.0, c->fx_shift);
    d->inv_two_S = ldexp(1.0, -c->fx_shift);
    d->bscale = ((-ORC_E) * d->inv_two_S) / ((2.0 * M_PI) * ORC_EPS0);
}

/* Largest S with w_max * 2^S <= 2^31, so per-particle charge fits 31 bits and
 * up to 2^31 particles per instance fit an int64 grid. */
int orc_auto_shift(double w_max) {
    int S = 0;
    while (ldexp(w_max, S + 1) <= 2147483648.0) ++S;
    while (ldexp(w_max, S) > 2147483648.0) --S;
    return S;
}

/*
 * Okhrimovskyy et al. (2002) analytic differential cross section,
 * dsigma/dOmega ~ (1 - xi^2) / (1 - xi cos chi)^2.  Its CDF in mu = cos chi is
 * F(mu) = (1-xi^2)/(2 xi) [1/(1 - xi mu) - 1/(1 + xi)]; inverting F(mu) = u:
 */
double orc_okh_cos(double xi, double u) {
    return ((2.0 * u + xi) - 1.0) / ((1.0 - xi) + (2.0 * xi) * u);
}

/*
 * Opal et al. (1971) secondary-electron energy spectrum,
 * sigma(E_s) ~ 1 / (1 + (E_s / Ebar)^2) on [0, E_av/2]; its CDF is
 * atan(E_s/Ebar) / atan(E_av/(2 Ebar)); inverting at u:
 */
double orc_opal_split(double Ebar, double E_av, double u) {
    return Ebar * tan(u * atan(E_av / (2.0 * Ebar)));
}

/*
 * Rotate unit vector u by polar angle chi (given cos chi) and azimuth phi
 * about itself.  Frame: e1 = unit(z_hat x u) unless u is within ~8 degrees of
 * z_hat, then e1 = unit(r_hat x u); e2 = u x e1.
 */
void orc_scatter(double ur, double ut, double uz, double cosx, double phi, double out[3]) {
    double e1r, e1t, e1z;
    if (fabs(uz) < 0.99) {
        double n = sqrt(ur * ur + ut * ut);
        e1r = -ut / n; e1t = ur / n; e1z = 0.0;
    } else {
        double n = sqrt(uz * uz + ut * ut);
        e1r = 0.0; e1t = -uz / n; e1z = ut / n;
    }
    double e2r = ut * e1z - uz * e1t;
    double e2t = uz * e1r - ur * e1z;
    double e2z = ur * e1t - ut * e1r;
    double sinx = sqrt(fmax(0.0, 1.0 - cosx * cosx));
    double cp = cos(phi), sp = sin(phi);
    out[0] = cosx * ur + sinx * (cp * e1r + sp * e2r);
    out[1] = cosx * ut + sinx * (cp * e1t + sp * e2t);
    out[2] = cosx * uz + sinx * (cp * e1z + sp * e2z);
}

/*
 * Tabulated cross sections (energy / cross-section pairs as in LXCat files):
 * linear interpolation in E between the tabulated points, the end values held
 * outside the table.  Ionisation is zero at or below the threshold.
 */
double orc_xs_at(int n, const double* E, const double* s, double x) {
    if (x <= E[0]) return s[0];
    if (x >= E[n - 1]) return s[n - 1];
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (E[mid] <= x) lo = mid;
        else hi = mid;
    }
    return s[lo] + (s[lo + 1] - s[lo]) * ((x - E[lo]) / (E[lo + 1] - E[lo]));
}

static double xs_total(const orc_cfg* c, int n, const double* E, const double* el, const double* iz, double x,
                       int above) {
    double t = orc_xs_at(n, E, el, x);
    if (x > c->iz_I_eV || (above && x == c->iz_I_eV)) t += orc_xs_at(n, E, iz, x);
    return t;
}

/* max over 0 <= E <= E_cap of (sigma_el + sigma_iz)(E) v(E): the pieces
 * between table points, the threshold and E_cap are linear in E, so
 * (alpha + beta E) sqrt(E) peaks at an end or at E = -alpha / (3 beta). */
double orc_xs_sigv_max(const orc_cfg* c, int n, const double* E, const double* el, const double* iz) {
    const double two_e_over_me = (2.0 * 1.602176634e-19) / 9.1093837015e-31;
    const double Ecap = c->E_cap_eV;
    double cut[4096 + 3];
    int m = 0;
    cut[m++] = 0.0;
    for (int k = 0; k < n && m < 4096 + 1; ++k)
        if (E[k] > 0.0 && E[k] < Ecap) cut[m++] = E[k];
    if (c->iz_I_eV > 0.0 && c->iz_I_eV < Ecap) cut[m++] = c->iz_I_eV;
    cut[m++] = Ecap;
    /* sort the cut points (insertion; the table is already increasing) */
    for (int i = 1; i < m; ++i)
        for (int j = i; j > 0 && cut[j - 1] > cut[j]; --j) {
            double t = cut[j]; cut[j] = cut[j - 1]; cut[j - 1] = t;
        }
    double best = 0.0;
    for (int i = 0; i + 1 < m; ++i) {
        const double p = cut[i], q = cut[i + 1];
        if (!(q > p)) continue;
        const double sp = xs_total(c, n, E, el, iz, p, 1), sq = xs_total(c, n, E, el, iz, q, 0);
        double f = sp * sqrt(p * two_e_over_me);
        if (f > best) best = f;
        f = sq * sqrt(q * two_e_over_me);
        if (f > best) best = f;
        const double beta = (sq - sp) / (q - p), alpha = sp - beta * p;
        if (beta < 0.0 && alpha > 0.0) {
            const double x = -alpha / (3.0 * beta);
            if (x > p && x < q) {
                f = (alpha + beta * x) * sqrt(x * two_e_over_me);
                if (f > best) best = f;
            }
        }
    }
    return best;
}

/* The null-collision bound of a table in use: the maximum of sigma v widened
 * by 2^-20, then rounded up to 12 significant bits, so the bound does not
 * depend on how the maximum's own rounding came out. */
double orc_xs_bound(double sigv_max) {
    int e;
    const double m = frexp(sigv_max * (1.0 + 0x1p-20), &e);
    return ldexp(ceil(ldexp(m, 12)), e - 12);
}

/* Single-shell Lotz ionisation cross section (m^2) at energy E (eV). */
double orc_sigma_iz(const orc_cfg* c, double E_eV) {
    if (!(E_eV > c->iz_I_eV)) return 0.0;
    return ((c->lotz_a * c->lotz_q) * log(E_eV / c->iz_I_eV)) / (E_eV * c->iz_I_eV);
}
