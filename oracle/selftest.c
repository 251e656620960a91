/*
 * selftest.c -- a stand-alone driver of the oracle for sanitizer builds
 * (address and undefined-behaviour checks of the host C code).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/.  It runs every stage
 * of the oracle on small meshes -- the load, the push, both collision
 * processes, the deposit, the Poisson solves (Dirichlet and open ends, the
 * elliptic insert at orders 1 and 3, cubic shapes), the seed source, the
 * cross-section and anisotropy tables, the moments, the well depth and the
 * diagnostics -- and checks the bookkeeping that holds exactly for any run:
 * every electron is live, absorbed or removed, and the deposited grid sums to
 * the live electrons' fixed-point weights.  Exit status 0: all checks held.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static orc_cfg coax(void) {
    orc_cfg c;
    memset(&c, 0, sizeof c);
    c.a = 1.0e-3; c.b = 10.0e-3; c.L = 60.0e-3; c.nr = 16; c.nz = 32;
    c.V_inner = -20000.0; c.V_outer = 0.0; c.V_end = -2000.0; c.end_mode = 0;
    c.B0 = 0.28; c.mirror_k = 0.3;
    c.p_mbar = 1.0; c.T_gas_K = 300.0; c.M_gas_amu = 2.016;
    c.sigma_el = 1.0e-19; c.iz_I_eV = 15.4; c.lotz_a = 4.5e-18; c.lotz_q = 2.0;
    c.opal_Ebar_eV = 10.0; c.okh_xi = 0.5; c.E_cap_eV = 3000.0;
    /* loaded up to the walls, so that the runs absorb electrons on every wall */
    c.n_init = 3000; c.r_lo = 1.05e-3; c.r_hi = 9.95e-3; c.z_lo = 0.5e-3; c.z_hi = 59.5e-3;
    c.T_init_eV = 50.0; c.weight = 1.0e5; c.load_mode = 1;
    c.seed = 11; c.dt = 1.0e-12; c.fx_shift = 0; c.diag_interval = 5; c.collisions = 1;
    c.spline_order = 1;
    return c;
}

static orc_cfg gun(int order) {
    orc_cfg c = coax();
    c.a = 63.75e-3; c.b = 81.0e-3; c.L = 44.0e-3; c.nr = 32; c.nz = 64;
    c.V_inner = -30000.0; c.V_end = 0.0; c.end_mode = 2; c.mirror_k = 0.0;
    c.p_mbar = 0.1; c.E_cap_eV = 33000.0;
    /* the load box must stay clear of the insert; hot enough to reach it */
    c.r_lo = 64.0e-3; c.r_hi = 76.0e-3; c.z_lo = 0.5e-3; c.z_hi = 43.5e-3; c.load_mode = 0;
    c.T_init_eV = 2000.0; c.weight = 3.6e6;
    c.ins_r0 = 81.0e-3; c.ins_z0 = 22.0e-3; c.ins_er = 3.0e-3; c.ins_ez = 14.0e-3;
    c.spline_order = order;
    return c;
}

static int failures = 0;

#define CHECK(cond, ...)                       \
    do {                                       \
        if (!(cond)) {                         \
            fprintf(stderr, __VA_ARGS__);      \
            fputc('\n', stderr);               \
            ++failures;                        \
        }                                      \
    } while (0)

/* Run one configuration for `steps` steps and check its bookkeeping. */
static void run(const char* name, orc_cfg c, int steps, int tables) {
    orc_sim* s = orc_create(&c, 4 * c.n_init + 4096);
    CHECK(s != NULL, "%s: orc_create failed", name);
    if (!s) return;
    CHECK(orc_load(s) == 0, "%s: orc_load failed", name);
    if (tables) {
        enum { N = 40 };
        double E[N], el[N], iz[N], xi[N];
        for (int k = 0; k < N; ++k) {
            E[k] = 0.01 * pow(10.0, 7.0 * k / (N - 1));
            el[k] = 2.0e-19 / pow(1.0 + E[k] / 50.0, 0.75);
            const double t = E[k] > c.iz_I_eV ? (E[k] - c.iz_I_eV) / 100.0 : 0.0;
            iz[k] = 4.0e-20 * t / ((1.0 + t) * (1.0 + t));
            xi[k] = 0.9 * E[k] / (E[k] + 20.0);
        }
        CHECK(orc_set_cross_sections(s, N, E, el, iz) == 0, "%s: cross sections refused", name);
        CHECK(orc_set_anisotropy(s, N, E, xi) == 0, "%s: anisotropy refused", name);
    }
    CHECK(orc_step(s, steps) == 0, "%s: orc_step failed", name);
    orc_diag d;
    orc_get_diag(s, &d);
    int64_t absorbed = 0;
    for (int w = 0; w < 4; ++w) absorbed += d.n_absorbed[w];
    CHECK(d.n_live + absorbed + d.n_nonfinite == c.n_init + d.n_ioniz + d.n_source,
          "%s: electrons not conserved (%lld live, %lld absorbed, %lld removed, %lld ionisations, %lld sourced)",
          name, (long long)d.n_live, (long long)absorbed, (long long)d.n_nonfinite, (long long)d.n_ioniz,
          (long long)d.n_source);
    const int64_t n = d.n_live;
    double* buf = (double*)malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1));
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    orc_get_particles(s, n, buf, buf + n, buf + 2 * n, buf + 3 * n, buf + 4 * n, buf + 5 * n, key);
    orc_derived dv;
    orc_sim_derived(s, &dv);
    int64_t want = 0;
    for (int64_t p = 0; p < n; ++p) want += (int64_t)llrint(buf[5 * n + p] * dv.two_S);
    CHECK(d.total_Q == want, "%s: deposited %lld, live weights %lld", name, (long long)d.total_Q, (long long)want);
    const int nodes = (c.nr + 1) * (c.nz + 1);
    int64_t* Q = (int64_t*)malloc(sizeof(int64_t) * (size_t)nodes);
    orc_get_charge(s, Q);
    int64_t sumQ = 0;
    for (int k = 0; k < nodes; ++k) sumQ += Q[k];
    CHECK(sumQ == d.total_Q, "%s: grid sums to %lld, total %lld", name, (long long)sumQ, (long long)d.total_Q);
    double* m = (double*)malloc(sizeof(double) * ORC_NMOM * (size_t)nodes);
    orc_moments(s, m);
    double* phi = (double*)malloc(sizeof(double) * (size_t)nodes);
    orc_get_phi(s, phi);
    double rmid[3] = {0.25 * (3 * c.a + c.b), 0.5 * (c.a + c.b), 0.25 * (c.a + 3 * c.b)}, depth[3], zmax[3];
    if (c.mirror_k == 0.0 && !orc_has_insert(&c)) orc_well_depth(&c, phi, 3, rmid, depth, zmax);
    double* navg = (double*)malloc(sizeof(double) * (size_t)nodes);
    orc_get_time_avg_density(s, navg);
    for (int k = 0; k < nodes; ++k) CHECK(isfinite(phi[k]) && isfinite(navg[k]), "%s: non-finite field", name);
    printf("%s: %d steps, %lld live, %lld elastic, %lld ionisations, %lld absorbed\n", name, steps,
           (long long)d.n_live, (long long)d.n_elastic, (long long)d.n_ioniz, (long long)absorbed);
    free(navg); free(phi); free(m); free(Q); free(key); free(buf);
    orc_destroy(s);
}

int main(void) {
    orc_cfg c = coax();
    run("coax, mirror field", c, 100, 0);
    c.mirror_k = 0.0;
    c.src_rate = 7.5;
    run("coax, seed source, tables", c, 100, 1);
    c = coax();
    c.end_mode = 2;
    c.V_end = 0.0;
    c.spline_order = 3;
    run("coax, open ends, cubic shapes", c, 60, 0);
    run("gun, insert, order 1", gun(1), 120, 0);
    run("gun, insert, order 3", gun(3), 60, 0);
    if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
    return failures ? 1 : 0;
}
