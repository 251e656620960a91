/*
 * pic.h -- C ABI of the MI355X (gfx950) particle loop of an axisymmetric
 * 2D3V (r,z) particle-in-cell code with Monte-Carlo electron-neutral
 * collisions (Le Bars et al., arXiv 2206.14662, Sec. II.A "Numerical model"
 * and Sec. II.B "Geometry and numerical parameters").
 *
 * The problem the calls describe (Sec. II.A-B): electrons between two coaxial
 * electrodes with an applied bias, an external (possibly non-uniform) axial
 * magnetic field, perfectly absorbing walls, a uniform constant neutral gas
 * given by its pressure and temperature, elastic and ionising collisions
 * given by their cross sections; ions are not followed.  One step advances
 * every instance by dt: gather + Boris push + cylindrical remap + absorb,
 * null-collision MCC (elastic, ionisation with a new electron), charge
 * deposit, FP64 Poisson solve.
 *
 * Conventions
 *   - Units are SI unless a name says otherwise (_eV, _mbar, _amu).
 *   - Node arrays are r-major: node (i,j), i in [0,nr], j in [0,nz], sits at
 *     index i*(nz+1)+j; r_i = a + i (b-a)/nr, z_j = j L/nz.
 *   - Every call returns a pic_status; nothing throws or aborts across the
 *     ABI.  pic_last_error() gives a message for the last failing call.
 *   - Host buffers passed in are owned by the caller and only read or
 *     written during the call.  Device memory is owned by the context and
 *     released by pic_destroy(); it comes from the caller's allocator when
 *     one is given in pic_run_cfg, else from hipMalloc.
 *   - pic_step() is asynchronous on the context's stream.  Device-side error
 *     flags (spawn overflow, fixed-point overflow, a non-finite particle) are
 *     sticky and reported by the next call that synchronises (pic_diag,
 *     pic_get_*, pic_sync); pic_diag still fills its output then.
 *   - One context must not be used from two host threads at once.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,     /* bad argument or configuration                        */
    PIC_ENOMEM = -2,     /* device or host allocation failed                     */
    PIC_EDEVICE = -3,    /* HIP runtime error (message in pic_last_error)        */
    PIC_ECAPACITY = -4,  /* particle storage full: new electrons were dropped    */
    PIC_EOVERFLOW = -5,  /* a weight does not fit the fixed-point charge scale   */
    PIC_ESTATE = -6,     /* call not valid in the current state                  */
    PIC_ENONFINITE = -7  /* a particle's new position was not finite (NaN or inf,
                            e.g. from a non-finite field value): it was removed
                            and counted in n_nonfinite, not as absorbed charge   */
} pic_status;

typedef enum {
    PIC_MODE_FP64_PLAIN = 0,   /* FP64 particles, one kernel per stage, no sort  */
    PIC_MODE_FP32_BATCHED = 1  /* FP32 particles, tile-sorted, fused, persistent */
} pic_mode;

/* Device memory provider.  alloc returns a device pointer of at least
 * `bytes` bytes (256-byte aligned) or NULL; free releases it. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} pic_allocator;

/* One simulation instance (one coaxial trap). */
typedef struct {
    double a, b, L;            /* inner radius, outer radius, length (m); 0<a<b  */
    int nr, nz;                /* cells in r and z; nz a multiple of 4 in [4, 4096]
                                  with no prime factor above 5 (2 nz-point FFTs) */
    double V_inner, V_outer;   /* electrode potentials at r=a, r=b (V)           */
    double V_end;              /* end electrodes at z=0,L (V), see end_mode      */
    int end_mode;              /* 0: phi_end(r) = phi_coax(r) + V_end; 1: V_end;
                                  2: open ends, d(phi)/dz = 0 (Sec. II.A)        */
    double B0, mirror_k;       /* Bz = B0 (1 + k zeta^2), zeta = (z-L/2)/(L/2),
                                  Br = -(r/2) dBz/dz                             */
    double p_mbar, T_gas_K;    /* neutral pressure and temperature: n = p/(kT)   */
    double M_gas_amu;          /* neutral mass (elastic recoil loss)             */
    double sigma_el;           /* elastic momentum-transfer cross section (m^2)  */
    double iz_I_eV;            /* ionisation threshold = binding energy (eV)     */
    double lotz_a, lotz_q;     /* Lotz sigma_iz = a q ln(E/I)/(E I), a [m^2 eV^2] */
    double opal_Ebar_eV;       /* Opal energy-split parameter (eV)               */
    double okh_xi;             /* Okhrimovskyy DCS parameter in [0,1), 0 isotropic */
    double E_cap_eV;           /* energy bound of the null-collision frequency   */
    long long n_init;          /* initial macro-electrons                        */
    double r_lo, r_hi, z_lo, z_hi; /* initial load box (m)                       */
    double T_init_eV;          /* Maxwellian temperature of the load (eV)        */
    double weight;             /* electrons per macro-electron                   */
    int load_mode;             /* 0: uniform in volume, 1: uniform in r          */
    unsigned long long seed;   /* Philox key of the instance                     */
    double dt;                 /* time step (s)                                  */
    int fx_shift;              /* S of the 2^S fixed-point charge; 0 = automatic */
    int diag_interval;         /* D: steps between density/current samples      */
    int collisions;            /* 0 switches the MCC stage off                   */
    /* Volumetric seed source (Sec. II.A): a weak source over the whole domain,
     * uniform in volume over a<r<b, 0<z<L, Maxwellian in velocity.  Step n
     * creates floor((n+1) src_rate) - floor(n src_rate) electrons after the
     * collisions (keys 2^62 + running index, Philox step word 0xFFFFFFFE). */
    double src_rate;           /* macro-electrons per step, >= 0 (0: off)        */
    double src_T_eV;           /* source temperature (eV); 0 takes T_init_eV     */
    /* Elliptic insert on the outer electrode (Sec. III: the gun geometry, a
     * filled ellipse on the outer cylinder): metal at V_outer where
     * ((r-ins_r0)/ins_er)^2 + ((z-ins_z0)/ins_ez)^2 <= 1.  The space-charge
     * potential uses weighted extended B-splines (Sec. II.A) of the degree of
     * the particle shapes (1 or 3, spline_order): B-splines times a weight
     * function that vanishes on the ellipse and is 1 beyond a band of about
     * ins_band cells; the vacuum potential uses those of degree 1.  Particles entering it are
     * absorbed as at r = b; seed-source electrons drawn inside it are not
     * created.  The band must keep 3 cells from r = a and from end plates,
     * and the load box must lie outside the ellipse (PIC_EINVAL otherwise).
     * ins_er = ins_ez = 0: no insert. */
    double ins_r0, ins_z0;     /* centre (m)                                     */
    double ins_er, ins_ez;     /* semi-axes in r and z (m), > 0 with an insert   */
    double ins_band;           /* weight band in cells, 0 takes 3; at most 64    */
    /* Order of the space-charge splines (Sec. II.A: B-spline FEM of any
     * order): 1 (or 0) bilinear shapes and Q1 FEM; 3 cubic B-spline particle
     * shapes (16 nodes), cubic FEM for the space-charge potential with the
     * walls' Dirichlet conditions built in by odd reflection, and the
     * space-charge field -grad phi_sc evaluated at each particle from the
     * spline coefficients (the vacuum field stays the order-1 nodal field).
     * With open ends (end_mode 2) the coefficients are reflected evenly at
     * z = 0 and z = L instead, so the space-charge potential has zero
     * z-derivative there.  With the elliptic insert the space-charge basis
     * is the cubic web-spline one, the field at a particle -grad(w u) =
     * w (-grad u) - u grad w.  Order 3 runs in both forms (the batched FP32
     * form gathers from an FP32 copy of the coefficients) and needs the same
     * order for every instance of the context. */
    int spline_order;
    /* Energy-dependent anisotropy of elastic and ionisation scattering
     * (Sec. II.A, Okhrimovskyy's differential cross section): okh_E0_eV > 0
     * takes the screened-Coulomb parameter xi(E) = 4 e / (1 + 4 e) with
     * e = E / okh_E0_eV (E the electron's energy; okh_E0_eV = 27.211386 eV,
     * the atomic unit of energy, in Okhrimovskyy et al.) instead of the
     * constant okh_xi; a table from pic_set_anisotropy takes precedence over
     * both.  0: the constant okh_xi. */
    double okh_E0_eV;
} pic_instance_cfg;

typedef struct {
    int mode;                  /* pic_mode                                       */
    int n_instances;           /* >= 1; PIC_MODE_FP64_PLAIN loops over them      */
    int tile_r, tile_z;        /* sort tile in cells (FP32 form); 0 = default    */
    int halo;                  /* LDS deposit-window halo in cells; 0 = default  */
    int sort_interval;         /* steps between tile sorts; 0 = default          */
    int chunk;                 /* max particles per work item; 0 = default       */
    int use_graph;             /* 0: plain launches; 1: each sort cycle (and    */
                               /* step kind) replayed as a captured HIP graph;  */
                               /* 2: graphs until pic_autotune, which times     */
                               /* both modes on its choice and keeps the faster */
    int device;                /* HIP device ordinal                             */
    void* stream;              /* hipStream_t to run on; NULL = a library stream */
    pic_allocator alloc;       /* alloc == NULL: hipMalloc/hipFree               */
    double capacity_factor;    /* particle slots = factor * n_init; 0 = 2.0      */
    long long capacity_min;    /* lower bound on slots per instance; 0 = 4096    */
    /* FP32 form: particles per lane and pass of the bilinear particle kernel.
     * 0 or 1: one, at 64 registers, two workgroups per CU; 2: two, whose
     * loads are in flight together, at up to 128 registers, one workgroup per
     * CU.  Results are bit-identical either way; pic_autotune times both and
     * keeps the faster.  Cubic shapes always take one. */
    int lanes;
} pic_run_cfg;

/* Per-instance diagnostics (Sec. III.A: peak density and boundary currents). */
typedef struct {
    long long step;            /* steps taken                                    */
    long long n_live;          /* live macro-electrons                           */
    long long n_elastic, n_ioniz;   /* real collision events so far              */
    long long n_null_cand;     /* null-collision candidates (u < P_null)         */
    long long n_cap_overflow;  /* particle-steps with |v| > v_cap                */
    long long n_spawn_dropped; /* new electrons lost to a full buffer (must be 0) */
    long long n_absorbed[4];   /* absorbed macro-electrons: inner, outer, left, right */
    long long absorbed_W[4];   /* absorbed charge per wall, units 2^-S electrons */
    long long total_Q;         /* sum of the deposited grid, units 2^-S electrons */
    long long n_samples;       /* density samples in the time average            */
    int S;                     /* fixed-point shift                              */
    double total_charge_C;     /* -e 2^-S total_Q                                */
    double I_wall[4];          /* last-window electron current into each wall (A) */
    double peak_density;       /* time max of the spatial max density (m^-3)    */
    double peak_time_avg_density; /* spatial max of the time-averaged density    */
    double peak_I_outer, peak_I_inner; /* max over windows of I_wall[1], I_wall[0] */
    long long particle_steps;  /* live macro-electrons pushed, summed over steps */
    long long n_far_deposit;   /* FP32 form: deposits that missed the LDS window */
    long long n_source;        /* electrons created by the seed source           */
    long long n_nonfinite;     /* particles removed because their new position was
                                  not finite; > 0 makes every synchronising call
                                  return PIC_ENONFINITE (sticky)                  */
} pic_diag_t;

/* Host-derived constants of an instance (FP64); see pic_derive. */
typedef struct {
    double dr, dz, inv_dr, inv_dz;
    double h;                  /* (q/m) dt / 2 with q = -e                       */
    double n_n;                /* neutral density 100 p_mbar / (k_B T) (m^-3)    */
    double v_cap, sig_iz_max, nu_prime, P_null;
    double nsig_el, lotz_aq, half_me_over_e, two_e_over_me, mass_ratio2;
    double two_S, inv_two_S;
    double bscale;             /* Q -> FEM load / eps0: -e 2^-S / (2 pi eps0)    */
} pic_derived_t;

/*
 * pic_init -- create a context: validate every instance, derive constants,
 * allocate device storage, build the static B and the vacuum potential
 * (discrete Laplace solution with the electrode data), load n_init
 * Maxwellian electrons per instance from the instance's Philox stream
 * (Sec. III.A initial homogeneous Maxwellian cloud), deposit them and solve
 * for the first field.  run->n_instances entries of inst are read.
 * Errors: PIC_EINVAL (bad configuration; nz must be a multiple of 4 with no
 * prime factor above 5),
 * PIC_ENOMEM, PIC_EDEVICE, PIC_EOVERFLOW (weight 2^S above 2^31 for an
 * explicit fx_shift; checked before any device call).  On error *out is
 * NULL and nothing is leaked.
 */
pic_status pic_init(const pic_run_cfg* run, const pic_instance_cfg* inst, pic_ctx** out);

/*
 * pic_step -- advance every instance by n_steps steps (Sec. II.A particle
 * loop: Boris push, absorbing walls, Monte-Carlo collisions, deposit,
 * Poisson).  Asynchronous on the context's stream.  Errors: PIC_EINVAL
 * (n_steps < 0), PIC_EDEVICE, PIC_ECAPACITY (reported when a capacity check
 * between sort intervals finds dropped electrons).
 */
pic_status pic_step(pic_ctx* ctx, int n_steps);

/*
 * pic_diag -- synchronise and copy instance `inst`'s diagnostics to *out.
 * density and time_avg_density are optional host arrays of (nr+1)(nz+1)
 * doubles receiving the current density Q 2^-S / V_i and the time average
 * over the samples taken every diag_interval steps, where V_i is the FEM
 * node volume (integral of the hat function over 2 pi r dr dz).
 */
pic_status pic_diag(pic_ctx* ctx, int inst, pic_diag_t* out, double* density,
                    double* time_avg_density);

/* pic_destroy -- release all device memory, streams and graphs of ctx. */
pic_status pic_destroy(pic_ctx* ctx);

/* pic_last_error -- message of the last failing call on ctx (or of the last
 * failing pic_init when ctx is NULL); valid until the next call. */
const char* pic_last_error(const pic_ctx* ctx);

/* pic_sync -- wait for the context's stream and report sticky device errors. */
pic_status pic_sync(pic_ctx* ctx);

/*
 * pic_get_particles -- copy instance `inst`'s live particles to host FP64
 * arrays of `cap` entries (storage order, FP32 values widened), set *n to
 * the live count.  Keys identify particles across steps: loaded electrons
 * have keys 0..n_init-1, electrons created by ionisation have the top bit
 * set.  If cap < *n only cap entries are written and PIC_EINVAL is returned.
 * After a sticky device error (PIC_ECAPACITY, PIC_ENONFINITE) the arrays
 * are still filled and that status is returned.
 */
pic_status pic_get_particles(pic_ctx* ctx, int inst, double* r, double* z, double* vr,
                             double* vt, double* vz, double* w, unsigned long long* key,
                             long long cap, long long* n);

/*
 * pic_set_particles -- replace instance `inst`'s particles with n host FP64
 * particles (velocities are v^{n-1/2}), redeposit and, unless the field is
 * frozen, solve for the field.  Every particle must lie in a<r<b, 0<z<L
 * with finite velocity components and a weight > 0.
 * Errors: PIC_EINVAL, PIC_ECAPACITY (n above the slots), PIC_EOVERFLOW
 * (a weight with w 2^S > 2^31).
 */
pic_status pic_set_particles(pic_ctx* ctx, int inst, long long n, const double* r,
                             const double* z, const double* vr, const double* vt,
                             const double* vz, const double* w,
                             const unsigned long long* key);

/*
 * pic_set_fields -- overwrite instance `inst`'s nodal fields with host FP64
 * node arrays (NULL leaves a component unchanged).  frozen = 1 keeps E fixed
 * (the Poisson stage is skipped; charge is still deposited), frozen = 0
 * returns to the self-consistent field at the next solve.  Values are not
 * checked: a particle that gathers a non-finite value gets a non-finite
 * position, is removed and makes later synchronising calls return
 * PIC_ENONFINITE.
 */
pic_status pic_set_fields(pic_ctx* ctx, int inst, const double* Er, const double* Ez,
                          const double* Br, const double* Bz, int frozen);

/* pic_get_fields -- copy the nodal fields the next push will gather (FP64
 * node arrays; NULL skips a component). */
pic_status pic_get_fields(pic_ctx* ctx, int inst, double* Er, double* Ez, double* Br,
                          double* Bz);

/* pic_get_charge -- copy the last deposited fixed-point grid (units 2^-S
 * electrons, FEM-weighted node charge) of instance `inst`. */
pic_status pic_get_charge(pic_ctx* ctx, int inst, long long* Q);

/* pic_set_cross_sections -- tabulated electron-neutral cross sections for
 * instance `inst` (Sec. II.A: the MCC module reads the gas's cross sections;
 * LXCat-style energy / cross-section pairs): n >= 2 strictly increasing
 * energies E_eV (eV) with the elastic momentum-transfer and ionisation cross
 * sections (m^2), linear in E between the points, the end values held outside
 * the table, ionisation zero at or below iz_I_eV.  The null-collision bound
 * becomes n_n max (sigma_el + sigma_iz)(E) v(E) over 0 <= E <= E_cap_eV
 * (widened by 2^-20).  n = 0 returns to the constant sigma_el and the Lotz
 * formula.  The arrays are copied (host pointers); at most 4096 points;
 * PIC_EINVAL for a bad table.  Call between steps. */
pic_status pic_set_cross_sections(pic_ctx* ctx, int inst, int n, const double* E_eV, const double* sigma_el,
                                  const double* sigma_iz);

/* pic_set_anisotropy -- energy-dependent anisotropy of the scattering law
 * for instance `inst` (Sec. II.A: the scattering angle follows the analytic
 * differential cross section of Okhrimovskyy et al., whose parameter xi
 * depends on the electron's energy): n >= 2 strictly increasing energies
 * E_eV (eV) with xi in (-1, 1), linear in E between the points and held
 * outside.  An elastically scattered electron takes xi at its incoming
 * energy; after an ionisation the primary and the freed electron take xi at
 * their own energies after the split.  n = 0 returns to the constant okh_xi.
 * The arrays are copied (host pointers); at most 4096 points; PIC_EINVAL for
 * a bad table.  Call between steps. */
pic_status pic_set_anisotropy(pic_ctx* ctx, int inst, int n, const double* E_eV, const double* xi);

/* pic_get_band_charge -- with the elliptic insert (Sec. II.A web-splines):
 * copy the fixed-point charges of q (w(x_p) - 1) that the particles inside
 * the weight function's band deposit next to the plain charges (units 2^-S
 * electrons; all zero without an insert): a node array ((nr+1) x (nz+1))
 * with bilinear shapes, the ghosted cubic layout of pic_get_spline3
 * ((nr+3) x (nz+3)) with cubic shapes.  The load of the Poisson system is
 * the plain grid plus this one carried through the web-spline extension. */
pic_status pic_get_band_charge(pic_ctx* ctx, int inst, long long* Qw);

/* pic_get_spline3 -- with cubic shapes: copy the ghosted cubic deposit Qx
 * (fixed point, node (i, j) for -1 <= i <= nr+1, -1 <= j <= nz+1 at
 * (i+1)(nz+3) + (j+1)) and the space-charge coefficients cx of the last
 * solve in the same layout (reflections filled).  Either pointer may be NULL.
 * PIC_EINVAL when the instance does not use cubic shapes. */
pic_status pic_get_spline3(pic_ctx* ctx, int inst, long long* Qx, double* cx);

/* pic_insert_layout -- host-only check of an instance's elliptic insert
 * (no device work): node counts by class (counts[0] not an unknown, [1]
 * inner, [2] outer, [3] inside the metal), the m nodes whose rows differ
 * from the plain grid's, and the entries of that difference; for the
 * space-charge system of the instance's shapes (the cubic B-spline unknowns
 * with spline_order 3).  PIC_EINVAL when the instance is invalid or has no
 * insert. */
pic_status pic_insert_layout(const pic_instance_cfg* inst, int counts[4], int* m, long long* entries);

/* pic_get_phi -- copy the last solved potential (V) of instance `inst`. */
pic_status pic_get_phi(pic_ctx* ctx, int inst, double* phi);

/* pic_set_step -- set the step counter that keys the Philox streams
 * (checkpoint/resume: a resumed run draws the same numbers). */
pic_status pic_set_step(pic_ctx* ctx, long long step);

/*
 * pic_derive -- host-only: the FP64 constants one instance derives (mesh
 * spacings, (q/m)dt/2, neutral density, null-collision bound and P_null,
 * fixed-point scale).  S is the fixed-point shift; S = 0 picks it
 * automatically (pic_auto_shift).  Needs no GPU.
 */
pic_status pic_derive(const pic_instance_cfg* inst, int S, pic_derived_t* out);

/* pic_auto_shift -- host-only: largest S with w_max 2^S <= 2^31. */
int pic_auto_shift(double w_max);

/*
 * pic_timing -- event timing of the dominant particle kernel.  enable = 1
 * records HIP events around every particle-kernel launch on the context's
 * stream in later pic_step calls (steps then run as plain launches, not a
 * graph); the call resets the accumulators.  With enable = 0 it returns the
 * number of timed launches and their summed duration (ms) since the last
 * reset, synchronising first.
 */
pic_status pic_timing(pic_ctx* ctx, int enable, long long* launches, double* total_ms);

/* pic_tuning -- the tile shape, halo, sort interval, chunk, particles per
 * lane and pass (1 or 2, see pic_run_cfg.lanes) and launch mode (1: captured
 * graphs, 0: plain launches) in use; any pointer may be NULL; zeros in the
 * FP64 form. */
pic_status pic_tuning(pic_ctx* ctx, int* tile_r, int* tile_z, int* halo, int* sort_interval,
                      int* chunk, int* lanes, int* use_graph);

/*
 * pic_retune -- FP32 form only: switch to tile_r x tile_z cell tiles, a
 * halo-cell LDS window and a sort every sort_interval steps (a value <= 0,
 * or < 0 for halo, keeps the current one), then re-sort every particle.
 * Synchronises.  No result of the method depends on these choices.
 * Errors: PIC_EINVAL (out of range, a window above the LDS of the launch shape --
 * 64 KiB with one particle per lane, 144 KiB with two -- or the FP64
 * form; the context is unchanged), PIC_ENOMEM/PIC_EDEVICE (the context must
 * then be destroyed).
 */
pic_status pic_retune(pic_ctx* ctx, int tile_r, int tile_z, int halo, int sort_interval);

/*
 * pic_autotune -- FP32 form only: time the context's own workload under
 * candidate tile shapes, halos and sort intervals, for one and for two
 * particles per lane and pass (pic_run_cfg.lanes; about 20 trials each of
 * max(trial_steps, 2 sort intervals) steps each, after two intervals of
 * warm-up) and keep the fastest; with pic_run_cfg.use_graph = 2 it then
 * times captured graphs against plain launches on that choice (twice each)
 * and keeps the faster mode.  The trial steps advance the simulation like
 * any other steps.  cache_path (or NULL) names a text file of one JSON
 * object per line keyed by a signature of the device and the workload
 * (meshes, live counts to a power of two): a hit applies the stored choice
 * without trials (*trials = 0), a miss appends the new result.  Outputs may
 * be NULL; *ms_per_step is the winning trial's time.  Errors as pic_retune.
 */
pic_status pic_autotune(pic_ctx* ctx, int trial_steps, const char* cache_path, int* tile_r,
                        int* tile_z, int* halo, int* sort_interval, double* ms_per_step,
                        int* trials);

/*
 * pic_reserve -- grow instance `inst`'s particle storage to at least `slots`
 * slots (new device stores from the allocator, live particles copied, the
 * FP32 form re-sorted and its step graphs re-captured).  pic_step grows
 * storage by itself: an instance found more than 3/4 full at one of the
 * checks taken every 64 steps gets twice its used slots.  Synchronises.
 * Errors: PIC_EINVAL, PIC_ENOMEM (the context must then be destroyed).
 */
pic_status pic_reserve(pic_ctx* ctx, int inst, long long slots);

/*
 * pic_moments -- fluid moments of instance `inst`'s electrons on the nodes
 * (Sec. IV evaluates its force terms from moments of the distribution):
 * 11 channel-major node arrays of (nr+1)(nz+1) doubles written to the host
 * array out (channel c at out + c (nr+1)(nz+1)): n; n u_r, n u_theta, n u_z;
 * the second moments sum w v_a v_b / V for (rr, r theta, rz, theta theta,
 * theta z, zz); and sum w nu_m / V with nu_m = n_n (sigma_el + sigma_iz(E)) |v|
 * (collisional drag weight).  Each is the bilinear (hat-function) node sum of
 * the particles' weight times the quantity, divided by the node volume V;
 * the pressure tensor is m_e (second moments - n u u), the radial current
 * density -e n u_r.  Synchronises; allocates a temporary device buffer.
 * Errors: PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE.
 */
pic_status pic_moments(pic_ctx* ctx, int inst, double* out);

/*
 * pic_well_depth -- depth (V; eV for an electron) of the potential well along
 * n_lines magnetic field lines of instance `inst` (Sec. II.B defines the well
 * along field lines): line l passes radius r_mid[l] at z = L/2 and follows the
 * configured field (r^2 Bz conserved); phi is interpolated at every node
 * column the line crosses inside a < r < b.  depth[l] = max phi - max(lowest
 * phi before it, lowest phi after it); z_max[l] = position of the maximum,
 * -1 (and depth 0) if the line is outside the domain at mid-length.  Host
 * arrays of n_lines doubles; synchronises.  Errors: PIC_EINVAL, PIC_EDEVICE.
 */
pic_status pic_well_depth(pic_ctx* ctx, int inst, int n_lines, const double* r_mid, double* depth,
                          double* z_max);

/*
 * pic_moments_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the moments of pic_moments, written to the caller's DEVICE
 * array out (11 channel-major node arrays of (nr+1)(nz+1) doubles, same
 * layout and values up to the order of the floating-point sums), queued on
 * the context's stream without synchronising and without any allocation.
 * The partial sums live in a fixed device scratch array of 32 MiB per GPU
 * (held until the process ends), so the instance's mesh may have at most
 * 381300 nodes (PIC_EINVAL beyond).  All contexts on one GPU share that
 * array: calls whose work overlaps on one GPU (different streams at once)
 * race and must be ordered by the caller.  Errors: PIC_EINVAL, PIC_ESTATE,
 * PIC_EDEVICE.
 */
pic_status pic_moments_noalloc(pic_ctx* ctx, int inst, double* out);

/* pic_capacity -- the slots of instance `inst` and the number of storage
 * regrowths so far (per context). */
pic_status pic_capacity(pic_ctx* ctx, int inst, long long* slots, long long* grow_events);

#ifdef __cplusplus
}
#endif
#endif
