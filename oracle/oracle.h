/*
 * oracle.h -- plain, slow, FP64 CPU oracle of the axisymmetric 2D3V (r,z)
 * PIC-MCC particle loop (Le Bars et al., "Self-consistent formation and
 * steady-state characterisation of trapped high energy electron clouds in the
 * presence of a neutral gas background", Sec. II.A "Numerical model").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product path never
 * links, imports or calls it, and it shares no source with the HIP library.
 *
 * What each part follows:
 *   - Boris push in (r,theta,z) with d/dtheta = 0 (Sec. II.A; Boris as in
 *     Birdsall & Langdon, cited there), written in the local Cartesian frame
 *     and rotated back to the (r,z) plane (angular-momentum conserving remap).
 *   - Bilinear (order-1 spline) gather and deposit on the rectangular (r,z)
 *     grid (Sec. II.A: rectangular grid, spline FEM).
 *   - Perfectly absorbing particle boundaries (Sec. II.A).
 *   - Monte-Carlo electron-neutral collisions with a uniform, constant neutral
 *     background of one species (Sec. II.A), null-collision form:
 *     elastic scattering with the Okhrimovskyy analytic DCS, ionisation with
 *     the binding energy removed, the remainder split by the Opal energy
 *     differential cross section, both electrons scattered; ions not followed.
 *   - Poisson by order-1 FEM with Dirichlet electrodes (Sec. II.A).
 * The paper defers the numerical details to a later publication; every reading
 * taken where it is silent is listed in the design notes of the repository.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One simulation instance: coaxial trap, fields, gas, cross sections, load. */
typedef struct {
    double a, b, L;            /* inner radius, outer radius, length (m)        */
    int nr, nz;                /* cells in r and z                              */
    double V_inner, V_outer;   /* electrode potentials at r=a and r=b (V)       */
    double V_end;              /* end-electrode potential offset (V)            */
    int end_mode;              /* 0: phi_end(r)=phi_coax(r)+V_end; 1: V_end     */
    double B0, mirror_k;       /* Bz = B0 (1 + k zeta^2), zeta=(z-L/2)/(L/2)    */
    double p_mbar, T_gas_K, M_gas_amu;
    double sigma_el;           /* constant elastic cross section (m^2)          */
    double iz_I_eV;            /* ionisation threshold / binding energy (eV)   */
    double lotz_a, lotz_q;     /* Lotz sigma = a q ln(E/I)/(E I), a in m^2 eV^2 */
    double opal_Ebar_eV;       /* Opal energy-split parameter (eV)              */
    double okh_xi;             /* Okhrimovskyy screening parameter, 0 isotropic */
    double E_cap_eV;           /* energy bound used for the null collision rate */
    int64_t n_init;            /* initial macro-electrons                       */
    double r_lo, r_hi, z_lo, z_hi, T_init_eV, weight;
    int load_mode;             /* 0: uniform in volume, 1: uniform in r         */
    uint64_t seed;             /* Philox key of this instance                   */
    double dt;                 /* time step (s)                                 */
    int fx_shift;              /* S: fixed-point charge scale 2^S               */
    int diag_interval;         /* D: steps per density / current sample         */
    int collisions;            /* 0 switches the MCC stage off                  */
    double src_rate;           /* seed source: macro-electrons per step (0 off)  */
    double src_T_eV;           /* its Maxwellian temperature (0: T_init_eV)     */
    /* elliptic insert on the outer electrode (metal, at V_outer) where
     * ((r-ins_r0)/ins_er)^2 + ((z-ins_z0)/ins_ez)^2 <= 1; ins_er = 0: none */
    double ins_r0, ins_z0, ins_er, ins_ez;
    double ins_band;           /* weight-function band in cells (0: 3)          */
    int spline_order;          /* space-charge shapes and FEM: 1 (0) bilinear/Q1, 3 cubic */
    double okh_E0_eV;          /* > 0: xi(E) = 4e/(1+4e), e = E/okh_E0_eV (screened Coulomb) */
} orc_cfg;

/* Host-derived constants (all FP64). */
typedef struct {
    double dr, dz, inv_dr, inv_dz;
    double h;                  /* 0.5 * (q/m) * dt, q = -e                      */
    double n_n;                /* neutral density (m^-3)                        */
    double v_cap, sig_iz_max, nu_prime, P_null;
    double nsig_el;            /* n_n * sigma_el                                */
    double lotz_aq;            /* lotz_a * lotz_q                               */
    double half_me_over_e;     /* E[eV] = v^2 * half_me_over_e                  */
    double two_e_over_me;      /* v = sqrt(E[eV] * two_e_over_me)               */
    double mass_ratio2;        /* 2 m_e / M                                     */
    double two_S, inv_two_S;
    double bscale;             /* Q -> FEM right-hand side incl. 1/(2 pi eps0)  */
} orc_derived;

typedef struct {
    int64_t step;
    int64_t n_live;
    int64_t n_elastic, n_ioniz, n_null_cand, n_cap_overflow;
    int64_t n_absorbed[4];     /* inner, outer, left, right                     */
    int64_t absorbed_W[4];     /* absorbed fixed-point weight per wall          */
    int64_t total_Q;           /* sum of the deposited grid                     */
    int64_t n_samples;         /* density samples in the time average           */
    double I_wall[4];          /* last window currents (A), electron flux >0    */
    double peak_density;       /* time max of the spatial max (m^-3)            */
    double peak_I_outer, peak_I_inner;
    int64_t n_source;          /* electrons created by the seed source          */
    int64_t n_nonfinite;       /* removed with a non-finite new position        */
} orc_diag;

typedef struct orc_sim orc_sim;

/* ---- unit-level functions (for pins) ---- */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u52(uint32_t hi, uint32_t lo);
void   orc_derive(const orc_cfg* c, orc_derived* d);
int    orc_auto_shift(double w_max);
double orc_okh_cos(double xi, double u);
double orc_opal_split(double Ebar, double E_av, double u);
void   orc_scatter(double ur, double ut, double uz, double cosx, double phi, double out[3]);
double orc_sigma_iz(const orc_cfg* c, double E_eV);
double orc_xs_at(int n, const double* E, const double* s, double x);
double orc_xs_sigv_max(const orc_cfg* c, int n, const double* E, const double* el, const double* iz);
double orc_xs_bound(double sigv_max);   /* widened by 2^-20, rounded up to 12 bits */
double orc_xi_sc(double E0_eV, double E_eV);   /* screened-Coulomb anisotropy 4e/(1+4e), e = E/E0 */

/* Node arrays are r-major: node (i,j) at i*(nz+1)+j, i in [0,nr], j in [0,nz]. */
void orc_bfield(const orc_cfg* c, double* Br, double* Bz);
void orc_vacuum(const orc_cfg* c, double* phi_vac);
void orc_solve(const orc_cfg* c, const double* rhs_interior_full, double* phi);
void orc_poisson_charge(const orc_cfg* c, const int64_t* Q, double* phi_sc);
void orc_efield(const orc_cfg* c, const double* phi, double* Er, double* Ez);
void orc_node_volume(const orc_cfg* c, double* V);
void orc_deposit_one(const orc_cfg* c, double r, double z, double w, int64_t* Q);
/* The same deposit of n particles into a zeroed node array Q, evaluated in
 * single precision from the FP32 values of r, z and w (orc_fp32.c). */
void orc_deposit_f32(const orc_cfg* c, int64_t n, const double* r, const double* z, const double* w,
                     int64_t* Q);
/* Potential-well depth along the configured magnetic field lines (Sec. II.B):
 * line l passes r_mid[l] at z = L/2 and keeps r^2 Bz(z) constant; phi is
 * sampled (bilinearly) at every node column inside a < r < b; depth[l] =
 * max phi - max(min phi left of it, min phi right of it) in volts (eV for an
 * electron), z_max[l] the position of the maximum (-1 and 0 when the line
 * leaves the domain at the midplane). */
void orc_well_depth(const orc_cfg* c, const double* phi, int n_lines, const double* r_mid, double* depth,
                    double* z_max);

/* Fluid moments (Sec. IV: force terms from moments of the distribution):
 * number of channels and their order in orc_moments' output. */
#define ORC_NMOM 11
/* n, n u_r, n u_t, n u_z, then sum w v_a v_b / V for (rr, rt, rz, tt, tz, zz),
 * then sum w nu_m(v) / V with nu_m = n_n (sigma_el + sigma_iz(E)) |v|. */

/* ---- elliptic insert (web-splines of degree 1), orc_insert.c ---- */
typedef struct orc_ins orc_ins;
int      orc_has_insert(const orc_cfg* c);
double   orc_ins_g(const orc_cfg* c, double r, double z);
double   orc_ins_gamma(const orc_cfg* c);
double   orc_ins_wp(const orc_cfg* c, double r, double z);
double   orc_ins_weight(const orc_cfg* c, double r, double z, double* wr, double* wz);
int      orc_ins_box_hits(const orc_cfg* c, double rl, double rh, double zl, double zh);
int      orc_ins_check(const orc_cfg* c);
orc_ins* orc_ins_create(const orc_cfg* c);
void     orc_ins_destroy(orc_ins* I);
void     orc_ins_solve_loads(const orc_ins* I, const orc_cfg* c, const double* load, double* phi);
void     orc_ins_solve_rows(const orc_ins* I, const orc_cfg* c, const double* rhs, double* phi);
void     orc_ins_poisson_charge(const orc_ins* I, const orc_cfg* c, const int64_t* Q, const int64_t* Qw,
                                double* phi_sc);
int      orc_ins_poisson_fn(const orc_cfg* c, double (*f)(double, double, void*), void* user, double* phi);
int      orc_ins_classify(const orc_cfg* c, int* cls);
int      orc_ins_info(const orc_cfg* c, int* n_unknowns, int* bandwidth, int counts[4]);

/* ---- cubic B-spline shapes and space charge, orc_spline3.c ---- */
typedef struct orc_s3 orc_s3;
void     orc_s3_weights(double f, double w[4], double dw[4]);
int      orc_s3_ext(const orc_cfg* c);              /* (nr+3)(nz+3): ghosted grid */
void     orc_s3_deposit(const orc_cfg* c, double r, double z, int64_t Wq, int64_t* Qx);
orc_s3*  orc_s3_create(const orc_cfg* c);
void     orc_s3_destroy(orc_s3* S);
void     orc_s3_solve(const orc_s3* S, const orc_cfg* c, const int64_t* Qx, double* cx, double* phi_sc);
void     orc_s3_field(const orc_cfg* c, const double* cx, double r, double z, double* Er, double* Ez);
double   orc_s3_phi_at(const orc_cfg* c, const double* cx, double r, double z);
int      orc_s3_poisson_fn(const orc_cfg* c, double (*f)(double, double, void*), void* user, double* cx);

/* null-collision candidates among n electrons at a step (analytic model) */
void orc_null_candidates(const orc_cfg* c, uint32_t step, int64_t n, const uint64_t* key, uint8_t* out);

/* ---- elliptic insert with cubic shapes (web-splines of degree 3), orc_insert3.c ---- */
typedef struct orc_is3 orc_is3;
orc_is3* orc_is3_create(const orc_cfg* c);
void     orc_is3_destroy(orc_is3* S);
/* load Qx + Qxw (ghosted, fixed point) -> ghosted expanded coefficients cx and
 * the nodal space-charge potential (NULL skips it) */
void     orc_is3_solve(const orc_is3* S, const orc_cfg* c, const int64_t* Qx, const int64_t* Qxw, double* cx,
                       double* phi_sc);
void     orc_is3_field(const orc_cfg* c, const double* cx, double r, double z, double* Er, double* Ez);
double   orc_is3_phi_at(const orc_cfg* c, const double* cx, double r, double z);
int      orc_is3_poisson_fn(const orc_cfg* c, double (*f)(double, double, void*), void* user, double* cx);
int      orc_is3_info(const orc_cfg* c, int* n_inner, int* bandwidth, int counts[4]);

/* ---- simulation object ---- */
orc_sim* orc_create(const orc_cfg* c, int64_t capacity);
void     orc_destroy(orc_sim* s);
int      orc_load(orc_sim* s);      /* initial Maxwellian load from Philox  */
int      orc_set_particles(orc_sim* s, int64_t n, const double* r, const double* z,
                           const double* vr, const double* vt, const double* vz,
                           const double* w, const uint64_t* key);
int64_t  orc_get_particles(const orc_sim* s, int64_t cap, double* r, double* z,
                           double* vr, double* vt, double* vz, double* w, uint64_t* key);
/* ORC_NMOM channel-major node arrays (channel c at out + c * nodes): the
 * bilinear (hat-function) sums of w times each quantity, divided by the node
 * volume, i.e. densities in m^-3 times the quantity's unit. */
void     orc_moments(const orc_sim* s, double* out);
void     orc_set_fields(orc_sim* s, const double* Er, const double* Ez,
                        const double* Br, const double* Bz, int frozen);
void     orc_get_fields(const orc_sim* s, double* Er, double* Ez, double* Br, double* Bz);
void     orc_set_step(orc_sim* s, int64_t step);
/* Tabulated elastic and ionisation cross sections (m^2) at n >= 2 strictly
 * increasing energies (eV), linear in E between them; n = 0 returns to the
 * constant elastic and Lotz ionisation cross sections.  The null-collision
 * bound becomes n_n max (sigma_el + sigma_iz) v over 0 <= E <= E_cap. */
int      orc_set_cross_sections(orc_sim* s, int n, const double* E, const double* el, const double* iz);
/* xi(E) of the Okhrimovskyy scattering law at n increasing energies (eV),
 * linear in E and held at the ends; n = 0 returns to the constant okh_xi.
 * Returns -1 for a refused table (n, order, xi outside (-1, 1)). */
int      orc_set_anisotropy(orc_sim* s, int n, const double* E, const double* xi);
void     orc_sim_derived(const orc_sim* s, orc_derived* d);   /* the constants in use */
int      orc_step(orc_sim* s, int n_steps);
void     orc_get_charge(const orc_sim* s, int64_t* Q);
void     orc_get_charge_w(const orc_sim* s, int64_t* Qw);   /* insert: band charges (else 0) */
/* cubic shapes: the ghosted cubic deposit and the space-charge coefficients
 * ((nr+3)(nz+3) arrays, ghost layer included; zeros for order 1) */
void     orc_get_charge3(const orc_sim* s, int64_t* Qx);
void     orc_get_coef3(const orc_sim* s, double* cx);
void     orc_get_charge3w(const orc_sim* s, int64_t* Qxw);  /* cubic + insert: band charges (else 0) */
void     orc_get_phi(const orc_sim* s, double* phi);
void     orc_get_diag(const orc_sim* s, orc_diag* d);
void     orc_get_time_avg_density(const orc_sim* s, double* n_avg);
int      orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
