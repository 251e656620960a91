/*
 * orc_sim.c -- oracle: the particle loop (load, gather, Boris push with the
 * cylindrical remap, absorption, null-collision MCC, deposit) and the step
 * sequence with its diagnostics.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Step n (the paper leaves the ordering to a later publication; this is the
 * standard explicit PIC-MCC cycle):
 *   1. every live particle: gather E^n,B at x^n, Boris v^{n-1/2} -> v^{n+1/2},
 *      move to x^{n+1} in the local Cartesian frame and rotate back to (r,z),
 *      remove it if it reached an electrode or an end;
 *   2. null-collision test for every survivor, elastic or ionising event;
 *   2b. the volumetric seed source adds its electrons (when switched on);
 *   3. deposit survivors and newly created electrons at x^{n+1};
 *   4. field solve for E^{n+1} (unless the field is frozen);
 *   5. every D steps: density and current samples.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_E 1.602176634e-19

struct orc_sim {
    orc_cfg c;
    orc_derived d;
    int64_t n, cap;
    double *r, *z, *vr, *vt, *vz, *w;
    uint64_t* key;
    int nodes;
    int64_t* Q;
    int64_t* Qw;               /* insert: deposit of q (w(x_p) - 1) (else NULL) */
    int64_t* Qx;               /* cubic shapes: ghosted cubic deposit (else NULL) */
    double* cx;                /* cubic shapes: ghosted space-charge coefficients */
    orc_s3* s3;                /* cubic shapes: factorised Galerkin system      */
    orc_is3* is3;              /* cubic shapes with the insert: web-spline system */
    int64_t* Qxw;              /* cubic shapes with the insert: band deposit    */
    int xs_n;                  /* tabulated cross sections (0: constant / Lotz) */
    double *xs_E, *xs_el, *xs_iz;
    int xi_n;                  /* tabulated anisotropy xi(E) (0: the constant okh_xi) */
    double *xi_E, *xi_v;
    orc_ins* ins;              /* insert: factorised web-spline system          */
    double *phi_vac, *phi, *Er, *Ez, *Br, *Bz, *V, *avg_acc;
    int frozen;
    int64_t step;
    orc_diag dg;
    int64_t absorbed_W_last[4];
};

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static void sim_reserve(orc_sim* s, int64_t need) {
    if (need <= s->cap) return;
    int64_t cap = s->cap > 0 ? s->cap : 1024;
    while (cap < need) cap *= 2;
    s->r = (double*)realloc(s->r, sizeof(double) * cap);
    s->z = (double*)realloc(s->z, sizeof(double) * cap);
    s->vr = (double*)realloc(s->vr, sizeof(double) * cap);
    s->vt = (double*)realloc(s->vt, sizeof(double) * cap);
    s->vz = (double*)realloc(s->vz, sizeof(double) * cap);
    s->w = (double*)realloc(s->w, sizeof(double) * cap);
    s->key = (uint64_t*)realloc(s->key, sizeof(uint64_t) * cap);
    s->cap = cap;
}

/* ---- shape function (bilinear, order-1 spline) ---- */
typedef struct { int i, j; double w00, w10, w01, w11; } orc_shape;

static inline orc_shape shape_at(const orc_cfg* c, const orc_derived* d, double r, double z) {
    orc_shape sh;
    double s = (r - c->a) * d->inv_dr;
    int i = (int)floor(s);
    if (i < 0) i = 0;
    if (i > c->nr - 1) i = c->nr - 1;
    double fr = s - (double)i;
    double t = z * d->inv_dz;
    int j = (int)floor(t);
    if (j < 0) j = 0;
    if (j > c->nz - 1) j = c->nz - 1;
    double fz = t - (double)j;
    sh.i = i; sh.j = j;
    sh.w00 = (1.0 - fr) * (1.0 - fz);
    sh.w10 = fr * (1.0 - fz);
    sh.w01 = (1.0 - fr) * fz;
    sh.w11 = fr * fz;
    return sh;
}

static inline double gather(const orc_shape* sh, const double* F, int W) {
    size_t n00 = (size_t)sh->i * W + sh->j;
    size_t n10 = n00 + W, n01 = n00 + 1, n11 = n00 + W + 1;
    return ((sh->w00 * F[n00] + sh->w10 * F[n10]) + sh->w01 * F[n01]) + sh->w11 * F[n11];
}

/* Fixed-point deposit of one particle: the four node charges round
 * W * (node weight) to the nearest integer, and the last node takes the
 * remainder so the particle's charge is conserved exactly. */
static inline void deposit_shape(const orc_shape* sh, int64_t Wq, int64_t* Q, int W) {
    double Wd = (double)Wq;
    int64_t q00 = (int64_t)rint(Wd * sh->w00);
    int64_t q10 = (int64_t)rint(Wd * sh->w10);
    int64_t q01 = (int64_t)rint(Wd * sh->w01);
    int64_t q11 = Wq - q00 - q10 - q01;
    size_t n00 = (size_t)sh->i * W + sh->j;
    Q[n00] += q00;
    Q[n00 + W] += q10;
    Q[n00 + 1] += q01;
    Q[n00 + W + 1] += q11;
}

void orc_deposit_one(const orc_cfg* c, double r, double z, double w, int64_t* Q) {
    orc_derived d;
    orc_derive(c, &d);
    orc_shape sh = shape_at(c, &d, r, z);
    deposit_shape(&sh, (int64_t)rint(w * d.two_S), Q, c->nz + 1);
}

/* ---- push: Boris in the local (r,theta,z) frame, then the remap ---- */
/* returns -1 if the particle survives, the wall index 0..3 if an electrode
 * or an end absorbs it, 4 if its new position is not finite */
static inline int push_one(const orc_sim* s, int64_t p, double* rr, double* zz,
                           double* vrr, double* vtt, double* vzz) {
    const orc_cfg* c = &s->c;
    const orc_derived* d = &s->d;
    const int W = c->nz + 1;
    double r = rr[p], z = zz[p], vr = vrr[p], vt = vtt[p], vz = vzz[p];
    orc_shape sh = shape_at(c, d, r, z);
    double Er = gather(&sh, s->Er, W), Ez = gather(&sh, s->Ez, W);
    if (s->s3 || s->is3) {
        /* cubic shapes: the nodal arrays hold the vacuum field; the space
         * charge's comes from the spline coefficients at the particle */
        double er, ez;
        if (s->is3) orc_is3_field(c, s->cx, r, z, &er, &ez);
        else orc_s3_field(c, s->cx, r, z, &er, &ez);
        Er += er;
        Ez += ez;
    }
    double Br = gather(&sh, s->Br, W), Bz = gather(&sh, s->Bz, W);
    const double h = d->h;
    /* half electric kick */
    double hEr = h * Er, hEz = h * Ez;
    double mr = vr + hEr, mt = vt, mz = vz + hEz;
    /* magnetic rotation: t = h B, s = 2 t / (1 + t.t) */
    double tr = h * Br, tz = h * Bz;
    double tt = tr * tr + tz * tz;
    double f = 2.0 / (1.0 + tt);
    double sr = f * tr, sz = f * tz;
    double pr = mr + mt * tz;              /* v' = v- + v- x t */
    double pt = mt + (mz * tr - mr * tz);
    double pz = mz - mt * tr;
    double qr = mr + pt * sz;              /* v+ = v- + v' x s */
    double qt = mt + (pz * sr - pr * sz);
    double qz = mz - pt * sr;
    /* second half electric kick */
    vr = qr + hEr; vt = qt; vz = qz + hEz;
    /* move in the Cartesian frame whose x axis is the particle's radius */
    double x = r + vr * c->dt;
    double y = vt * c->dt;
    double zn = z + vz * c->dt;
    double rr2 = x * x + y * y;
    double rn = sqrt(rr2);
    int wall = -1;
    /* a new position that is not finite (from a non-finite field value or
     * velocity) removes the particle; it is counted apart, not as charge
     * absorbed by an electrode */
    if (!(isfinite(rr2) && isfinite(zn))) return 4;
    if (rn <= c->a) wall = 0;
    else if (rn >= c->b) wall = 1;
    else if (s->ins && orc_ins_g(c, rn, zn) <= 0.0) wall = 1;   /* the insert is part of the outer electrode */
    else if (zn <= 0.0) wall = 2;
    else if (zn >= c->L) wall = 3;
    if (wall >= 0) return wall;
    /* rotate the velocity into the new (r,theta) frame */
    double cs = x / rn, sn = y / rn;
    double vrn = cs * vr + sn * vt;
    double vtn = cs * vt - sn * vr;
    rr[p] = rn; zz[p] = zn; vrr[p] = vrn; vtt[p] = vtn; vzz[p] = vz;
    return -1;
}

/* ---- MCC ---- */
typedef struct { double r, z, vr, vt, vz, w; uint64_t key; } orc_part;

static inline void philox_blk(const orc_sim* s, uint64_t key, uint32_t step, uint32_t blk, uint32_t o[4]) {
    uint32_t ctr[4] = {(uint32_t)key, (uint32_t)(key >> 32), step, blk};
    uint32_t k[2] = {(uint32_t)s->c.seed, (uint32_t)(s->c.seed >> 32)};
    orc_philox4x32_10(ctr, k, o);
}

/* Anisotropy of the scattering of an electron of energy E (eV): the table
 * xi(E), linear in E and held at its ends; else, with okh_E0_eV > 0, the
 * screened-Coulomb parameter of Okhrimovskyy et al. (2002),
 * xi = 4 e / (1 + 4 e) with e = E / E0 (E0 their atomic energy unit); else
 * the constant okh_xi. */
double orc_xi_sc(double E0, double E) {
    const double e4 = 4.0 * (E * (1.0 / E0));
    return e4 / (1.0 + e4);
}

static inline double xi_at(const orc_sim* s, double E) {
    if (s->xi_n > 0) return orc_xs_at(s->xi_n, s->xi_E, s->xi_v, E);
    return s->c.okh_E0_eV > 0.0 ? orc_xi_sc(s->c.okh_E0_eV, E) : s->c.okh_xi;
}

/* event: 0 none, 1 elastic, 2 ionisation (child filled), 3 candidate rejected.
 * The elastically scattered electron takes xi at its incoming energy; after
 * an ionisation the primary and the freed electron are scattered with xi at
 * their own energies after the split. */
static inline int mcc_one(const orc_sim* s, int64_t p, orc_part* child) {
    const orc_cfg* c = &s->c;
    const orc_derived* d = &s->d;
    uint32_t step = (uint32_t)s->step;
    uint32_t b0[4];
    philox_blk(s, s->key[p], step, 0u, b0);
    double u_null = orc_u52(b0[0], b0[1]);
    if (!(u_null < d->P_null)) return 0;
    double u_proc = orc_u52(b0[2], b0[3]);
    double vr = s->vr[p], vt = s->vt[p], vz = s->vz[p];
    double v2 = (vr * vr + vt * vt) + vz * vz;
    double v = sqrt(v2);
    double E = v2 * d->half_me_over_e;
    double nu_el, sig_iz = 0.0;
    if (s->xs_n > 0) {
        nu_el = (d->n_n * orc_xs_at(s->xs_n, s->xs_E, s->xs_el, E)) * v;
        if (E > c->iz_I_eV) sig_iz = orc_xs_at(s->xs_n, s->xs_E, s->xs_iz, E);
    } else {
        nu_el = d->nsig_el * v;
        if (E > c->iz_I_eV) sig_iz = (d->lotz_aq * log(E / c->iz_I_eV)) / (E * c->iz_I_eV);
    }
    double nu_iz = (d->n_n * sig_iz) * v;
    double R = u_proc * d->nu_prime;
    int ev;
    if (R < nu_el) ev = 1;
    else if (R < nu_el + nu_iz) ev = 2;
    else return 3;
    double ur = vr / v, ut = vt / v, uz = vz / v;
    uint32_t b1[4];
    philox_blk(s, s->key[p], step, 1u, b1);
    double phi1 = (2.0 * M_PI) * orc_u52(b1[2], b1[3]);
    double dir[3];
    if (ev == 1) {
        double cos1 = orc_okh_cos(xi_at(s, E), orc_u52(b1[0], b1[1]));
        double En = E * (1.0 - d->mass_ratio2 * (1.0 - cos1));
        double vn = sqrt(En * d->two_e_over_me);
        orc_scatter(ur, ut, uz, cos1, phi1, dir);
        s->vr[p] = vn * dir[0]; s->vt[p] = vn * dir[1]; s->vz[p] = vn * dir[2];
        return 1;
    }
    uint32_t b2[4], b3[4];
    philox_blk(s, s->key[p], step, 2u, b2);
    philox_blk(s, s->key[p], step, 3u, b3);
    double E_av = E - c->iz_I_eV;
    double E_s = orc_opal_split(c->opal_Ebar_eV, E_av, orc_u52(b2[0], b2[1]));
    double E_p = E_av - E_s;
    double cos1 = orc_okh_cos(xi_at(s, E_p), orc_u52(b1[0], b1[1]));
    double cos2 = orc_okh_cos(xi_at(s, E_s), orc_u52(b2[2], b2[3]));
    double phi2 = (2.0 * M_PI) * orc_u52(b3[0], b3[1]);
    double vp = sqrt(E_p * d->two_e_over_me);
    double vs = sqrt(E_s * d->two_e_over_me);
    orc_scatter(ur, ut, uz, cos1, phi1, dir);
    s->vr[p] = vp * dir[0]; s->vt[p] = vp * dir[1]; s->vz[p] = vp * dir[2];
    orc_scatter(ur, ut, uz, cos2, phi2, dir);
    child->r = s->r[p]; child->z = s->z[p];
    child->vr = vs * dir[0]; child->vt = vs * dir[1]; child->vz = vs * dir[2];
    child->w = s->w[p];
    child->key = ((((uint64_t)b3[2]) << 32) | (uint64_t)b3[3]) | (1ull << 63);
    return 2;
}

/* Which of n electrons (by key) are null-collision candidates at step
 * `step` of an instance with the analytic cross sections: the first uniform
 * of Philox block 0 below P_null (the test mcc_one starts with). */
void orc_null_candidates(const orc_cfg* c, uint32_t step, int64_t n, const uint64_t* key, uint8_t* out) {
    orc_derived d;
    orc_derive(c, &d);
    const uint32_t k[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        const uint32_t ctr[4] = {(uint32_t)key[p], (uint32_t)(key[p] >> 32), step, 0u};
        uint32_t o[4];
        orc_philox4x32_10(ctr, k, o);
        out[p] = orc_u52(o[0], o[1]) < d.P_null ? 1 : 0;
    }
}

/* ---- deposit of all particles into s->Q (per-thread grids, exact sums) ---- */
/* With the insert, a particle inside the weight function's band also
 * deposits rint(Wq (w(x_p) - 1)) into Qw by the same exact-sum rule. */
static void deposit_all(orc_sim* s) {
    const int W = s->c.nz + 1;
    const int N = s->nodes;
    const double gam = s->ins ? orc_ins_gamma(&s->c) : 0.0;
    const int NX = s->Qx ? orc_s3_ext(&s->c) : 0;
    memset(s->Q, 0, sizeof(int64_t) * N);
    if (s->Qw) memset(s->Qw, 0, sizeof(int64_t) * N);
    if (s->Qx) memset(s->Qx, 0, sizeof(int64_t) * NX);
    if (s->Qxw) memset(s->Qxw, 0, sizeof(int64_t) * NX);
#pragma omp parallel
    {
        int64_t* loc = (int64_t*)calloc(N, sizeof(int64_t));
        int64_t* locw = s->Qw ? (int64_t*)calloc(N, sizeof(int64_t)) : NULL;
        int64_t* locx = s->Qx ? (int64_t*)calloc(NX, sizeof(int64_t)) : NULL;
        int64_t* locxw = s->Qxw ? (int64_t*)calloc(NX, sizeof(int64_t)) : NULL;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < s->n; ++p) {
            orc_shape sh = shape_at(&s->c, &s->d, s->r[p], s->z[p]);
            int64_t Wq = (int64_t)rint(s->w[p] * s->d.two_S);
            deposit_shape(&sh, Wq, loc, W);
            if (locw && orc_ins_g(&s->c, s->r[p], s->z[p]) < gam) {
                double wp = orc_ins_wp(&s->c, s->r[p], s->z[p]);
                deposit_shape(&sh, (int64_t)rint((double)Wq * (wp - 1.0)), locw, W);
            }
            if (locx) orc_s3_deposit(&s->c, s->r[p], s->z[p], Wq, locx);
            if (locxw && orc_ins_g(&s->c, s->r[p], s->z[p]) < gam) {
                double wp = orc_ins_wp(&s->c, s->r[p], s->z[p]);
                orc_s3_deposit(&s->c, s->r[p], s->z[p], (int64_t)rint((double)Wq * (wp - 1.0)), locxw);
            }
        }
#pragma omp critical
        {
            for (int k = 0; k < N; ++k) s->Q[k] += loc[k];
            if (locw)
                for (int k = 0; k < N; ++k) s->Qw[k] += locw[k];
            if (locx)
                for (int k = 0; k < NX; ++k) s->Qx[k] += locx[k];
            if (locxw)
                for (int k = 0; k < NX; ++k) s->Qxw[k] += locxw[k];
        }
        free(loc);
        free(locw);
        free(locx);
        free(locxw);
    }
}

static void solve_fields(orc_sim* s) {
    if (s->frozen) return;
    if (s->is3) {
        /* cubic shapes with the insert: the nodal E stays the vacuum field */
        orc_is3_solve(s->is3, &s->c, s->Qx, s->Qxw, s->cx, s->phi);
        for (int k = 0; k < s->nodes; ++k) s->phi[k] += s->phi_vac[k];
        return;
    }
    if (s->s3) {
        /* cubic shapes: the nodal E stays the vacuum field */
        orc_s3_solve(s->s3, &s->c, s->Qx, s->cx, s->phi);
        for (int k = 0; k < s->nodes; ++k) s->phi[k] += s->phi_vac[k];
        return;
    }
    if (s->ins) orc_ins_poisson_charge(s->ins, &s->c, s->Q, s->Qw, s->phi);
    else orc_poisson_charge(&s->c, s->Q, s->phi);
    for (int k = 0; k < s->nodes; ++k) s->phi[k] += s->phi_vac[k];
    orc_efield(&s->c, s->phi, s->Er, s->Ez);
}

/* ---- public sim API ---- */
orc_sim* orc_create(const orc_cfg* c, int64_t capacity) {
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->c = *c;
    if (s->c.diag_interval <= 0) s->c.diag_interval = 1;
    orc_derive(&s->c, &s->d);
    s->nodes = (c->nr + 1) * (c->nz + 1);
    sim_reserve(s, capacity > 0 ? capacity : 1024);
    s->Q = (int64_t*)calloc(s->nodes, sizeof(int64_t));
    s->phi_vac = (double*)calloc(s->nodes, sizeof(double));
    s->phi = (double*)calloc(s->nodes, sizeof(double));
    s->Er = (double*)calloc(s->nodes, sizeof(double));
    s->Ez = (double*)calloc(s->nodes, sizeof(double));
    s->Br = (double*)calloc(s->nodes, sizeof(double));
    s->Bz = (double*)calloc(s->nodes, sizeof(double));
    s->V = (double*)calloc(s->nodes, sizeof(double));
    s->avg_acc = (double*)calloc(s->nodes, sizeof(double));
    if (s->c.spline_order == 3) {
        if (orc_has_insert(&s->c)) {
            s->is3 = orc_is3_create(&s->c);
            s->Qxw = (int64_t*)calloc((size_t)orc_s3_ext(&s->c), sizeof(int64_t));
        } else {
            s->s3 = orc_s3_create(&s->c);
        }
        if (!s->s3 && !s->is3) {
            orc_destroy(s);
            return NULL;
        }
        s->Qx = (int64_t*)calloc((size_t)orc_s3_ext(&s->c), sizeof(int64_t));
        s->cx = (double*)calloc((size_t)orc_s3_ext(&s->c), sizeof(double));
    } else if (s->c.spline_order != 0 && s->c.spline_order != 1) {
        orc_destroy(s);
        return NULL;
    }
    if (orc_has_insert(&s->c)) {
        s->ins = orc_ins_create(&s->c);
        if (!s->ins) {
            orc_destroy(s);
            return NULL;
        }
        if (!s->is3) s->Qw = (int64_t*)calloc(s->nodes, sizeof(int64_t));
    }
    orc_bfield(&s->c, s->Br, s->Bz);
    orc_vacuum(&s->c, s->phi_vac);
    memcpy(s->phi, s->phi_vac, sizeof(double) * s->nodes);
    orc_efield(&s->c, s->phi, s->Er, s->Ez);
    orc_node_volume(&s->c, s->V);
    return s;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    free(s->r); free(s->z); free(s->vr); free(s->vt); free(s->vz); free(s->w); free(s->key);
    free(s->Q); free(s->phi_vac); free(s->phi); free(s->Er); free(s->Ez);
    free(s->Br); free(s->Bz); free(s->V); free(s->avg_acc);
    free(s->Qw);
    free(s->Qx); free(s->cx);
    orc_s3_destroy(s->s3);
    orc_is3_destroy(s->is3);
    free(s->Qxw);
    free(s->xs_E); free(s->xs_el); free(s->xs_iz);
    free(s->xi_E); free(s->xi_v);
    orc_ins_destroy(s->ins);
    free(s);
}

/*
 * Initial load (Sec. III.A: homogeneous Maxwellian cloud; Sec. II.A seed
 * source: uniform in space, Maxwellian in velocity).  Particle p draws from
 * Philox counter {p, 0xFFFFFFFF, block}; positions uniform in volume
 * (load_mode 0) or in r (load_mode 1); velocity components by Box-Muller.
 */
int orc_load(orc_sim* s) {
    const orc_cfg* c = &s->c;
    int64_t n = c->n_init;
    if (s->ins && n > 0 && orc_ins_box_hits(c, c->r_lo, c->r_hi, c->z_lo, c->z_hi)) return -1;
    sim_reserve(s, n);
    double sv = sqrt((c->T_init_eV * ORC_E) / 9.1093837015e-31);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        uint32_t b0[4], b1[4], b2[4];
        philox_blk(s, (uint64_t)p, 0xFFFFFFFFu, 0u, b0);
        philox_blk(s, (uint64_t)p, 0xFFFFFFFFu, 1u, b1);
        philox_blk(s, (uint64_t)p, 0xFFFFFFFFu, 2u, b2);
        double ur = orc_u52(b0[0], b0[1]), uz = orc_u52(b0[2], b0[3]);
        double r;
        if (c->load_mode == 1) r = c->r_lo + ur * (c->r_hi - c->r_lo);
        else r = sqrt(c->r_lo * c->r_lo + ur * (c->r_hi * c->r_hi - c->r_lo * c->r_lo));
        double z = c->z_lo + uz * (c->z_hi - c->z_lo);
        double u1 = orc_u52(b1[0], b1[1]), u2 = orc_u52(b1[2], b1[3]);
        double u3 = orc_u52(b2[0], b2[1]), u4 = orc_u52(b2[2], b2[3]);
        double m1 = sqrt(-2.0 * log(u1)), m3 = sqrt(-2.0 * log(u3));
        s->r[p] = r; s->z[p] = z;
        s->vr[p] = sv * (m1 * cos((2.0 * M_PI) * u2));
        s->vt[p] = sv * (m1 * sin((2.0 * M_PI) * u2));
        s->vz[p] = sv * (m3 * cos((2.0 * M_PI) * u4));
        s->w[p] = c->weight;
        s->key[p] = (uint64_t)p;
    }
    s->n = n;
    deposit_all(s);
    solve_fields(s);
    return 0;
}

int orc_set_particles(orc_sim* s, int64_t n, const double* r, const double* z,
                      const double* vr, const double* vt, const double* vz,
                      const double* w, const uint64_t* key) {
    sim_reserve(s, n);
    memcpy(s->r, r, sizeof(double) * n);
    memcpy(s->z, z, sizeof(double) * n);
    memcpy(s->vr, vr, sizeof(double) * n);
    memcpy(s->vt, vt, sizeof(double) * n);
    memcpy(s->vz, vz, sizeof(double) * n);
    memcpy(s->w, w, sizeof(double) * n);
    memcpy(s->key, key, sizeof(uint64_t) * n);
    s->n = n;
    deposit_all(s);
    solve_fields(s);
    return 0;
}

int64_t orc_get_particles(const orc_sim* s, int64_t cap, double* r, double* z,
                          double* vr, double* vt, double* vz, double* w, uint64_t* key) {
    int64_t n = s->n < cap ? s->n : cap;
    memcpy(r, s->r, sizeof(double) * n);
    memcpy(z, s->z, sizeof(double) * n);
    memcpy(vr, s->vr, sizeof(double) * n);
    memcpy(vt, s->vt, sizeof(double) * n);
    memcpy(vz, s->vz, sizeof(double) * n);
    memcpy(w, s->w, sizeof(double) * n);
    memcpy(key, s->key, sizeof(uint64_t) * n);
    return s->n;
}

void orc_set_fields(orc_sim* s, const double* Er, const double* Ez,
                    const double* Br, const double* Bz, int frozen) {
    size_t b = sizeof(double) * s->nodes;
    if (Er) memcpy(s->Er, Er, b);
    if (Ez) memcpy(s->Ez, Ez, b);
    if (Br) memcpy(s->Br, Br, b);
    if (Bz) memcpy(s->Bz, Bz, b);
    s->frozen = frozen;
    if (s->s3 || s->is3) {
        /* cubic shapes: a frozen field is the given nodal one alone; back to
         * the self-consistent field, the nodal arrays hold the vacuum field */
        memset(s->cx, 0, sizeof(double) * (size_t)orc_s3_ext(&s->c));
        if (!frozen) {
            orc_efield(&s->c, s->phi_vac, s->Er, s->Ez);
            solve_fields(s);
        }
    }
}

void orc_get_fields(const orc_sim* s, double* Er, double* Ez, double* Br, double* Bz) {
    size_t b = sizeof(double) * s->nodes;
    if (Er) memcpy(Er, s->Er, b);
    if (Ez) memcpy(Ez, s->Ez, b);
    if (Br) memcpy(Br, s->Br, b);
    if (Bz) memcpy(Bz, s->Bz, b);
}

void orc_set_step(orc_sim* s, int64_t step) { s->step = step; }

void orc_sim_derived(const orc_sim* s, orc_derived* d) { *d = s->d; }

int orc_set_cross_sections(orc_sim* s, int n, const double* E, const double* el, const double* iz) {
    if (n != 0 && (n < 2 || n > 4096)) return -1;
    for (int k = 0; k < n; ++k) {
        if (!(E[k] >= 0.0) || !(el[k] >= 0.0) || !(iz[k] >= 0.0)) return -1;
        if (k > 0 && !(E[k] > E[k - 1])) return -1;
    }
    free(s->xs_E); free(s->xs_el); free(s->xs_iz);
    s->xs_E = s->xs_el = s->xs_iz = NULL;
    s->xs_n = n;
    orc_derive(&s->c, &s->d);
    if (n == 0) return 0;
    s->xs_E = (double*)malloc(sizeof(double) * n);
    s->xs_el = (double*)malloc(sizeof(double) * n);
    s->xs_iz = (double*)malloc(sizeof(double) * n);
    memcpy(s->xs_E, E, sizeof(double) * n);
    memcpy(s->xs_el, el, sizeof(double) * n);
    memcpy(s->xs_iz, iz, sizeof(double) * n);
    /* the bound, widened and rounded up (orc_xs_bound) */
    s->d.nu_prime = s->d.n_n * orc_xs_bound(orc_xs_sigv_max(&s->c, n, E, el, iz));
    s->d.P_null = -expm1(-(s->d.nu_prime * s->c.dt));
    return 0;
}

int orc_set_anisotropy(orc_sim* s, int n, const double* E, const double* xi) {
    if (n != 0 && (n < 2 || n > 4096)) return -1;
    for (int k = 0; k < n; ++k) {
        if (!(E[k] >= 0.0) || !(xi[k] > -1.0 && xi[k] < 1.0)) return -1;
        if (k > 0 && !(E[k] > E[k - 1])) return -1;
    }
    free(s->xi_E); free(s->xi_v);
    s->xi_E = s->xi_v = NULL;
    s->xi_n = n;
    if (n == 0) return 0;
    s->xi_E = (double*)malloc(sizeof(double) * n);
    s->xi_v = (double*)malloc(sizeof(double) * n);
    memcpy(s->xi_E, E, sizeof(double) * n);
    memcpy(s->xi_v, xi, sizeof(double) * n);
    return 0;
}

static void sample_diag(orc_sim* s) {
    const int D = s->c.diag_interval;
    double peak = 0.0;
    for (int k = 0; k < s->nodes; ++k) {
        double dens = ((double)s->Q[k] * s->d.inv_two_S) / s->V[k];
        if (dens > peak) peak = dens;
        s->avg_acc[k] += (double)s->Q[k];
    }
    if (peak > s->dg.peak_density) s->dg.peak_density = peak;
    s->dg.n_samples += 1;
    double span = (double)D * s->c.dt;
    for (int wl = 0; wl < 4; ++wl) {
        int64_t dW = s->dg.absorbed_W[wl] - s->absorbed_W_last[wl];
        s->dg.I_wall[wl] = (((double)dW * ORC_E) * s->d.inv_two_S) / span;
        s->absorbed_W_last[wl] = s->dg.absorbed_W[wl];
    }
    if (s->dg.I_wall[1] > s->dg.peak_I_outer) s->dg.peak_I_outer = s->dg.I_wall[1];
    if (s->dg.I_wall[0] > s->dg.peak_I_inner) s->dg.peak_I_inner = s->dg.I_wall[0];
}

/*
 * Volumetric seed source (Sec. II.A: a weak source over the whole domain,
 * uniform in space, Maxwellian in velocity).  With R = src_rate electrons per
 * step, step n creates floor((n+1) R) - floor(n R) of them, so that
 * floor(n R) exist after n steps; the j-th of step n has key
 * 2^62 + floor(n R) + j.  Each draws three Philox blocks of its key at the
 * step word 0xFFFFFFFE: r uniform in volume over (a, b), z uniform over
 * (0, L), Box-Muller velocity components at src_T_eV (T_init_eV if 0).  An
 * electron drawn inside the elliptic insert lies outside the domain and is
 * not created (its key is skipped).
 */
static void seed_source(orc_sim* s) {
    const orc_cfg* c = &s->c;
    if (!(c->src_rate > 0.0)) return;
    const double n0 = floor((double)s->step * c->src_rate);
    const double n1 = floor((double)(s->step + 1) * c->src_rate);
    const int64_t count = (int64_t)(n1 - n0), first = (int64_t)n0;
    if (count <= 0) return;
    const double T = c->src_T_eV > 0.0 ? c->src_T_eV : c->T_init_eV;
    const double sv = sqrt((T * ORC_E) / 9.1093837015e-31);
    sim_reserve(s, s->n + count);
    int64_t made = 0;
    for (int64_t j = 0; j < count; ++j) {
        const uint64_t key = (UINT64_C(1) << 62) + (uint64_t)(first + j);
        uint32_t b0[4], b1[4], b2[4];
        philox_blk(s, key, 0xFFFFFFFEu, 0u, b0);
        philox_blk(s, key, 0xFFFFFFFEu, 1u, b1);
        philox_blk(s, key, 0xFFFFFFFEu, 2u, b2);
        const double ur = orc_u52(b0[0], b0[1]), uz = orc_u52(b0[2], b0[3]);
        const double u1 = orc_u52(b1[0], b1[1]), u2 = orc_u52(b1[2], b1[3]);
        const double u3 = orc_u52(b2[0], b2[1]), u4 = orc_u52(b2[2], b2[3]);
        const double m1 = sqrt(-2.0 * log(u1)), m3 = sqrt(-2.0 * log(u3));
        const double r = sqrt(c->a * c->a + ur * (c->b * c->b - c->a * c->a)), z = uz * c->L;
        if (s->ins && orc_ins_g(c, r, z) <= 0.0) continue;   /* inside the insert: not in the domain */
        const int64_t q = s->n + made;
        s->r[q] = r;
        s->z[q] = z;
        s->vr[q] = sv * (m1 * cos((2.0 * M_PI) * u2));
        s->vt[q] = sv * (m1 * sin((2.0 * M_PI) * u2));
        s->vz[q] = sv * (m3 * cos((2.0 * M_PI) * u4));
        s->w[q] = c->weight;
        s->key[q] = key;
        ++made;
    }
    s->n += made;
    s->dg.n_source += made;
}

int orc_step(orc_sim* s, int n_steps) {
    const double vcap2 = s->d.v_cap * s->d.v_cap;
    for (int it = 0; it < n_steps; ++it) {
        const int64_t n = s->n;
        int* wall = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
        /* 1. push and absorb */
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p) wall[p] = push_one(s, p, s->r, s->z, s->vr, s->vt, s->vz);
        int64_t m = 0;
        for (int64_t p = 0; p < n; ++p) {
            if (wall[p] == 4) {
                s->dg.n_nonfinite += 1;
                continue;
            }
            if (wall[p] >= 0) {
                s->dg.n_absorbed[wall[p]] += 1;
                s->dg.absorbed_W[wall[p]] += (int64_t)rint(s->w[p] * s->d.two_S);
                continue;
            }
            s->r[m] = s->r[p]; s->z[m] = s->z[p]; s->vr[m] = s->vr[p];
            s->vt[m] = s->vt[p]; s->vz[m] = s->vz[p]; s->w[m] = s->w[p]; s->key[m] = s->key[p];
            ++m;
        }
        s->n = m;
        free(wall);
        /* 2. MCC on the survivors */
        int64_t cap_over = 0;
        for (int64_t p = 0; p < m; ++p) {
            double v2 = (s->vr[p] * s->vr[p] + s->vt[p] * s->vt[p]) + s->vz[p] * s->vz[p];
            if (v2 > vcap2) ++cap_over;
        }
        s->dg.n_cap_overflow += cap_over;
        if (s->c.collisions) {
            int nt = orc_num_threads();
            orc_part** kids = (orc_part**)calloc(nt, sizeof(orc_part*));
            int64_t* nk = (int64_t*)calloc(nt, sizeof(int64_t));
            int64_t* ck = (int64_t*)calloc(nt, sizeof(int64_t));
            int64_t n_el = 0, n_iz = 0, n_cand = 0;
#pragma omp parallel reduction(+ : n_el, n_iz, n_cand)
            {
#ifdef _OPENMP
                int t = omp_get_thread_num();
#else
                int t = 0;
#endif
#pragma omp for schedule(static)
                for (int64_t p = 0; p < m; ++p) {
                    orc_part ch;
                    int ev = mcc_one(s, p, &ch);
                    if (ev != 0) ++n_cand;
                    if (ev == 1) ++n_el;
                    if (ev == 2) {
                        ++n_iz;
                        if (nk[t] == ck[t]) {
                            ck[t] = ck[t] ? 2 * ck[t] : 64;
                            kids[t] = (orc_part*)realloc(kids[t], sizeof(orc_part) * ck[t]);
                        }
                        kids[t][nk[t]++] = ch;
                    }
                }
            }
            s->dg.n_elastic += n_el;
            s->dg.n_ioniz += n_iz;
            s->dg.n_null_cand += n_cand;
            int64_t tot = 0;
            for (int t = 0; t < nt; ++t) tot += nk[t];
            sim_reserve(s, m + tot);
            int64_t q = m;
            for (int t = 0; t < nt; ++t) {
                for (int64_t k = 0; k < nk[t]; ++k, ++q) {
                    s->r[q] = kids[t][k].r; s->z[q] = kids[t][k].z;
                    s->vr[q] = kids[t][k].vr; s->vt[q] = kids[t][k].vt; s->vz[q] = kids[t][k].vz;
                    s->w[q] = kids[t][k].w; s->key[q] = kids[t][k].key;
                }
                free(kids[t]);
            }
            s->n = q;
            free(kids); free(nk); free(ck);
        }
        seed_source(s);
        /* 3. deposit, 4. field */
        deposit_all(s);
        solve_fields(s);
        /* 5. diagnostics */
        s->step += 1;
        s->dg.step = s->step;
        if (s->step % s->c.diag_interval == 0) sample_diag(s);
    }
    return 0;
}

/* Fluid moments of the particle distribution on the nodes (Sec. IV "Prevalent
 * force terms" evaluates its force terms from these): each particle adds
 * w * N_i(x) * {1, v_r, v_t, v_z, v_a v_b, nu_m(v)} to node i; the sums are
 * divided by the node volume.  Plain sequential loop. */
void orc_moments(const orc_sim* s, double* out) {
    const int W = s->c.nz + 1, N = s->nodes;
    memset(out, 0, sizeof(double) * (size_t)ORC_NMOM * N);
    for (int64_t p = 0; p < s->n; ++p) {
        orc_shape sh = shape_at(&s->c, &s->d, s->r[p], s->z[p]);
        const double vr = s->vr[p], vt = s->vt[p], vz = s->vz[p], w = s->w[p];
        const double v2 = (vr * vr + vt * vt) + vz * vz, v = sqrt(v2);
        const double E = v2 * s->d.half_me_over_e;
        double nu;
        if (s->xs_n > 0) {
            const double siz = E > s->c.iz_I_eV ? orc_xs_at(s->xs_n, s->xs_E, s->xs_iz, E) : 0.0;
            nu = (s->d.n_n * orc_xs_at(s->xs_n, s->xs_E, s->xs_el, E) + s->d.n_n * siz) * v;
        } else {
            nu = (s->d.nsig_el + s->d.n_n * orc_sigma_iz(&s->c, E)) * v;
        }
        const double q[ORC_NMOM] = {1.0, vr, vt, vz, vr * vr, vr * vt, vr * vz, vt * vt, vt * vz, vz * vz, nu};
        const size_t n00 = (size_t)sh.i * W + sh.j;
        const size_t node[4] = {n00, n00 + W, n00 + 1, n00 + W + 1};
        const double sw[4] = {sh.w00, sh.w10, sh.w01, sh.w11};
        for (int c = 0; c < ORC_NMOM; ++c)
            for (int k = 0; k < 4; ++k) out[(size_t)c * N + node[k]] += (w * sw[k]) * q[c];
    }
    for (int c = 0; c < ORC_NMOM; ++c)
        for (int k = 0; k < N; ++k) out[(size_t)c * N + k] /= s->V[k];
}

void orc_get_charge(const orc_sim* s, int64_t* Q) { memcpy(Q, s->Q, sizeof(int64_t) * s->nodes); }
void orc_get_charge3(const orc_sim* s, int64_t* Qx) {
    if (s->Qx) memcpy(Qx, s->Qx, sizeof(int64_t) * (size_t)orc_s3_ext(&s->c));
    else memset(Qx, 0, sizeof(int64_t) * (size_t)orc_s3_ext(&s->c));
}
void orc_get_coef3(const orc_sim* s, double* cx) {
    if (s->cx) memcpy(cx, s->cx, sizeof(double) * (size_t)orc_s3_ext(&s->c));
    else memset(cx, 0, sizeof(double) * (size_t)orc_s3_ext(&s->c));
}
void orc_get_charge3w(const orc_sim* s, int64_t* Qxw) {
    if (s->Qxw) memcpy(Qxw, s->Qxw, sizeof(int64_t) * (size_t)orc_s3_ext(&s->c));
    else memset(Qxw, 0, sizeof(int64_t) * (size_t)orc_s3_ext(&s->c));
}
void orc_get_charge_w(const orc_sim* s, int64_t* Qw) {
    if (s->Qw) memcpy(Qw, s->Qw, sizeof(int64_t) * s->nodes);
    else memset(Qw, 0, sizeof(int64_t) * s->nodes);
}
void orc_get_phi(const orc_sim* s, double* phi) { memcpy(phi, s->phi, sizeof(double) * s->nodes); }

void orc_get_diag(const orc_sim* s, orc_diag* d) {
    *d = s->dg;
    d->step = s->step;
    d->n_live = s->n;
    int64_t tq = 0;
    for (int k = 0; k < s->nodes; ++k) tq += s->Q[k];
    d->total_Q = tq;
}

void orc_get_time_avg_density(const orc_sim* s, double* n_avg) {
    for (int k = 0; k < s->nodes; ++k) {
        if (s->dg.n_samples == 0) { n_avg[k] = 0.0; continue; }
        n_avg[k] = ((s->avg_acc[k] * s->d.inv_two_S) / (double)s->dg.n_samples) / s->V[k];
    }
}
