// api.hip -- host side of the C ABI declared in include/pic.h: validation,
// derived constants, device storage, the vacuum potential, the step
// sequence of both forms, checkpoint hooks and diagnostics.
#include <math.h>
#include <string.h>

#include <cmath>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "pic_internal.h"
#include "fp32.h"

using namespace pic;

struct Inst {
    pic_instance_cfg c;
    pic_derived_t d;
    DevInst I;
    int S = 0;
    long long cap = 0;
    long long nodes = 0;
    bool frozen = false;
    P64 p64[2];
    int cur = 0;
    long long* Q = nullptr;
    double *rhs = nullptr, *phi = nullptr, *phi_vac = nullptr, *phiB = nullptr;
    double *Er = nullptr, *Ez = nullptr, *Br = nullptr, *Bz = nullptr, *V = nullptr;
    double *avg_acc = nullptr, *th_cp = nullptr, *th_im = nullptr, *th_lo = nullptr;
    double *th_G = nullptr, *th_H = nullptr;
    float4* EB = nullptr;
    long long* cnt = nullptr;
    std::vector<double> V_host;
    // elliptic insert
    bool has_ins = false;
    InsHost ih;
    InsDev idev;              // device pointers of the corrected solve
    int h_owner = -1;         // an earlier instance with the same corrected system: its H is used
    long long* Qw = nullptr;
    // cubic shapes with the insert: the web-spline system of degree 3 (the
    // bilinear one above still gives the vacuum potential)
    Ins3Host ih3;
    InsDev idev3;             // its corrected solve (M, H and the buffers of insert.hip's kernels)
    Ins3Dev xdev3;            // its load map and rebuilt coefficients
    int h3_owner = -1;
    // cubic shapes
    long long* Qx = nullptr;
    double *cx = nullptr, *cbuf = nullptr, *zeros = nullptr;
    float* cxf = nullptr;     // FP32 copy of cx (batched form)
    double *s3_L1 = nullptr, *s3_L2 = nullptr, *s3_L3 = nullptr, *s3_Dinv = nullptr;
};

struct pic_ctx {
    pic_run_cfg run;
    int mode = 0;
    std::vector<Inst> in;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::vector<void*> allocs;
    long long grow_events = 0;  // FP64 store regrowths
    DevInst* dI = nullptr;
    FieldDev* dF = nullptr;
    FieldDev* dFvac = nullptr;
    double* dbscale = nullptr;
    // elliptic insert: the instances that have one, their corrected-solve
    // tables and the field tables of the two fast solves
    std::vector<int> ins_list;
    int max_m = 0;
    InsDev* dIns = nullptr;
    DevInst* dIins = nullptr;     // DevInst of the insert instances, in ins_list order
    int n_grp = 0;                // groups of insert instances sharing one H
    std::vector<int> h_goff, h_gmem;
    int *dGoff = nullptr, *dGmem = nullptr;  // group g: dIns entries dGmem[dGoff[g] .. dGoff[g+1])
    FieldDev *dF1 = nullptr, *dF1v = nullptr;   // first solve (step / vacuum): phi -> ybuf
    FieldDev *dF2 = nullptr, *dF2v = nullptr;   // second solve, insert instances only
    // cubic shapes (every instance of the context)
    bool s3 = false;
    long long max_ext = 0;
    FieldDev* dF3 = nullptr;                    // coefficient solve: rhs, phi -> cbuf, phi_vac -> zeros
    // cubic shapes with the insert: the corrected solve's tables (insert
    // instances in ins_list order) and the two fast solves' field tables
    int max_m3 = 0, max_nx3 = 0;
    InsDev* dIns3 = nullptr;
    Ins3Dev* dX3 = nullptr;
    int n_grp3 = 0;
    std::vector<int> h_goff3, h_gmem3;
    int *dGoff3 = nullptr, *dGmem3 = nullptr;
    FieldDev *dF3a = nullptr, *dF3b = nullptr;  // first solve (phi -> ybuf of the insert instances), second
    long long* dcnt = nullptr;
    long long* prep_ctl = nullptr;  // FP32 step plan the end-of-step kernel refreshes
    long long* dtmp = nullptr;
    double2* tw = nullptr;
    int tw_n = 0;
    int max_nr = 0, max_nz = 0;
    long long max_nodes = 0;
    long long host_step = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;      // pairs (start, stop)
    size_t ev_used = 0;
    long long timed_launches = 0;
    double timed_ms = 0.0;
    F32State* f32 = nullptr;
};

static std::string g_init_error;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

#define CK(call)                                                                     \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) return fail(ctx, PIC_EDEVICE, std::string(#call) + ": " + \
                                          hipGetErrorString(e_));                    \
    } while (0)

static pic_status fail(pic_ctx* ctx, pic_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    else g_init_error = msg;
    return st;
}

void* pic_dev_alloc(pic_ctx* ctx, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (ctx->run.alloc.alloc) {
        p = ctx->run.alloc.alloc(bytes, ctx->run.alloc.user);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
    if (p) ctx->allocs.push_back(p);
    return p;
}

void pic_dev_free(pic_ctx* ctx, void* p) {
    if (!p) return;
    auto it = std::find(ctx->allocs.begin(), ctx->allocs.end(), p);
    if (it == ctx->allocs.end()) return;  // not ours
    ctx->allocs.erase(it);
    if (ctx->run.alloc.alloc) {
        if (ctx->run.alloc.free) ctx->run.alloc.free(p, ctx->run.alloc.user);
    } else {
        (void)hipFree(p);
    }
}

hipStream_t pic_stream(pic_ctx* ctx) { return ctx->stream; }
int pic_device(pic_ctx* ctx) { return ctx->run.device; }

template <class T>
static T* dalloc(pic_ctx* ctx, long long count) {
    return (T*)pic_dev_alloc(ctx, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

// ---------------------------------------------------------------------------
// host-only: derived constants (same expressions and order as documented for
// the FP64 form; evaluated once per instance)
// ---------------------------------------------------------------------------

extern "C" int pic_auto_shift(double w_max) {
    int S = 0;
    while (ldexp(w_max, S + 1) <= 2147483648.0) ++S;
    while (ldexp(w_max, S) > 2147483648.0) --S;
    return S;
}

extern "C" pic_status pic_derive(const pic_instance_cfg* c, int S, pic_derived_t* d) {
    if (!c || !d) return PIC_EINVAL;
    if (S == 0) S = c->fx_shift != 0 ? c->fx_shift : pic_auto_shift(c->weight);
    d->dr = (c->b - c->a) / (double)c->nr;
    d->dz = c->L / (double)c->nz;
    d->inv_dr = 1.0 / d->dr;
    d->inv_dz = 1.0 / d->dz;
    double qm = -kE / kMe;
    d->h = (0.5 * qm) * c->dt;
    d->n_n = (100.0 * c->p_mbar) / (kKb * c->T_gas_K);
    d->v_cap = sqrt(((2.0 * c->E_cap_eV) * kE) / kMe);
    d->sig_iz_max = (c->lotz_a * c->lotz_q) / ((exp(1.0) * c->iz_I_eV) * c->iz_I_eV);
    d->nu_prime = (d->n_n * (c->sigma_el + d->sig_iz_max)) * d->v_cap;
    d->P_null = -expm1(-(d->nu_prime * c->dt));
    d->nsig_el = d->n_n * c->sigma_el;
    d->lotz_aq = c->lotz_a * c->lotz_q;
    d->half_me_over_e = (0.5 * kMe) / kE;
    d->two_e_over_me = (2.0 * kE) / kMe;
    d->mass_ratio2 = (2.0 * kMe) / (c->M_gas_amu * kAmu);
    d->two_S = ldexp(1.0, S);
    d->inv_two_S = ldexp(1.0, -S);
    d->bscale = ((-kE) * d->inv_two_S) / ((2.0 * kPi) * kEps0);
    return PIC_OK;
}

// Integer form of the null test: u52(x) < P  <=>  (x >> 12) < k.
static unsigned long long null_threshold(double P) {
    if (!(P > 0.0)) return 0ull;
    double lim = 4503599627370496.0;  // 2^52
    double x = P * lim;
    unsigned long long k = x >= lim ? (1ull << 52) : (unsigned long long)x;
    while (k > 0 && (((double)(k - 1) + 0.5) * 0x1p-52) >= P) --k;
    while (k < (1ull << 52) && (((double)k + 0.5) * 0x1p-52) < P) ++k;
    return k;
}

// nz for the z transforms: 2 nz points, a multiple of 8 with no prime factor
// beyond 5
static bool fft_size_ok(int nz) {
    if (nz < 4 || nz % 4 != 0) return false;
    int m = nz;
    for (int p : {2, 3, 5})
        while (m % p == 0) m /= p;
    return m == 1;
}

static std::string validate(const pic_instance_cfg& c) {
    if (!(c.a > 0.0 && c.b > c.a && c.L > 0.0)) return "need 0 < a < b and L > 0";
    if (c.nr < 4 || c.nr > 16384) return "nr must be in [4, 16384]";
    if (!fft_size_ok(c.nz) || c.nz > 4096)
        return "nz must be a multiple of 4 in [4, 4096] with no prime factor above 5";
    if (!(c.dt > 0.0)) return "dt must be > 0";
    if (!(c.T_gas_K > 0.0) || !(c.p_mbar >= 0.0)) return "need T_gas_K > 0 and p_mbar >= 0";
    if (!(c.M_gas_amu > 0.0)) return "M_gas_amu must be > 0";
    if (!(c.sigma_el >= 0.0) || !(c.lotz_a >= 0.0) || !(c.lotz_q >= 0.0)) return "cross sections must be >= 0";
    if (!(c.iz_I_eV > 0.0) || !(c.opal_Ebar_eV > 0.0)) return "iz_I_eV and opal_Ebar_eV must be > 0";
    if (!(c.okh_xi > -1.0 && c.okh_xi < 1.0)) return "okh_xi must be in (-1, 1)";
    if (!(c.okh_E0_eV >= 0.0 && c.okh_E0_eV < 1e30)) return "okh_E0_eV must be >= 0 and finite";
    if (!(c.E_cap_eV > 0.0)) return "E_cap_eV must be > 0";
    if (c.n_init < 0) return "n_init must be >= 0";
    if (c.n_init > 0) {
        if (!(c.r_lo >= c.a && c.r_hi <= c.b && c.r_lo < c.r_hi)) return "load box must satisfy a <= r_lo < r_hi <= b";
        if (!(c.z_lo >= 0.0 && c.z_hi <= c.L && c.z_lo < c.z_hi)) return "load box must satisfy 0 <= z_lo < z_hi <= L";
        if (!(c.T_init_eV >= 0.0) || !(c.weight > 0.0)) return "need T_init_eV >= 0 and weight > 0";
    }
    if (!(c.src_rate >= 0.0 && c.src_rate <= 1e9) || !(c.src_T_eV >= 0.0))
        return "need 0 <= src_rate <= 1e9 per step and src_T_eV >= 0";
    if (c.load_mode != 0 && c.load_mode != 1) return "load_mode must be 0 or 1";
    if (c.end_mode < 0 || c.end_mode > 2) return "end_mode must be 0, 1 or 2";
    if (c.diag_interval < 0) return "diag_interval must be >= 0";
    if (c.spline_order != 0 && c.spline_order != 1 && c.spline_order != 3) return "spline_order must be 1 or 3";
    if (c.ins_er != 0.0 || c.ins_ez != 0.0) {
        if (!(c.ins_er > 0.0 && c.ins_ez > 0.0 && std::isfinite(c.ins_r0) && std::isfinite(c.ins_z0)))
            return "insert: need ins_er > 0, ins_ez > 0 and a finite centre";
        if (!(c.ins_band >= 0.0 && c.ins_band <= 64.0)) return "insert: ins_band must be in [0, 64] cells";
        const double dr = (c.b - c.a) / (double)c.nr, dz = c.L / (double)c.nz;
        const double band = c.ins_band > 0.0 ? c.ins_band : 3.0;
        const double sg = sqrt(1.0 + 2.0 * band * std::max(dr / c.ins_er, dz / c.ins_ez));
        if (c.ins_r0 - c.ins_er * sg < c.a + 3.0 * dr) return "insert: its weight band reaches the inner electrode";
        if (c.end_mode != 2 && (c.ins_z0 - c.ins_ez * sg < 3.0 * dz || c.ins_z0 + c.ins_ez * sg > c.L - 3.0 * dz))
            return "insert: its weight band reaches an end electrode";
        if (c.n_init > 0) {
            // the load box must lie outside the metal: the least g over the box
            const double rc = std::min(std::max(c.ins_r0, c.r_lo), c.r_hi);
            const double zc = std::min(std::max(c.ins_z0, c.z_lo), c.z_hi);
            const double u = (rc - c.ins_r0) / c.ins_er, v = (zc - c.ins_z0) / c.ins_ez;
            if ((u * u + v * v) - 1.0 <= 0.0) return "insert: the load box reaches into the insert";
        }
    }
    return "";
}

// ---------------------------------------------------------------------------
// host-side static arrays of an instance
// ---------------------------------------------------------------------------

static double r_at(const pic_instance_cfg& c, double dr, double i) { return c.a + i * dr; }

static void host_bfield(const pic_instance_cfg& c, std::vector<double>& Br, std::vector<double>& Bz) {
    const int W = c.nz + 1;
    const double dr = (c.b - c.a) / (double)c.nr, dz = c.L / (double)c.nz;
    const double halfL = 0.5 * c.L;
    Br.assign((size_t)(c.nr + 1) * W, 0.0);
    Bz.assign((size_t)(c.nr + 1) * W, 0.0);
    for (int i = 0; i <= c.nr; ++i) {
        double r = r_at(c, dr, (double)i);
        for (int j = 0; j <= c.nz; ++j) {
            double z = (double)j * dz;
            double zeta = (z - halfL) / halfL;
            size_t n = (size_t)i * W + j;
            Bz[n] = c.B0 * (1.0 + c.mirror_k * (zeta * zeta));
            Br[n] = -(r * ((c.B0 * c.mirror_k) * zeta)) / halfL;
        }
    }
}

// 1D assembled FEM entries between node i and i+di (r with weight r, z plain).
static double kr(const pic_instance_cfg& c, double dr, int i, int di) {
    double rm = r_at(c, dr, i - 0.5), rp = r_at(c, dr, i + 0.5);
    if (di == 0) return (i > 0 ? rm / dr : 0.0) + (i < c.nr ? rp / dr : 0.0);
    return di < 0 ? -rm / dr : -rp / dr;
}
static double mr(const pic_instance_cfg& c, double dr, int i, int di) {
    double rm = r_at(c, dr, i - 1), r0 = r_at(c, dr, i), rp = r_at(c, dr, i + 1);
    if (di == 0)
        return (i > 0 ? dr * (rm + 3.0 * r0) / 12.0 : 0.0) + (i < c.nr ? dr * (3.0 * r0 + rp) / 12.0 : 0.0);
    return di < 0 ? dr * (rm + r0) / 12.0 : dr * (r0 + rp) / 12.0;
}
// z entries at node j; with open ends (end_mode 2) the end nodes carry one element
static double kz(const pic_instance_cfg& c, double dz, int j, int dj) {
    if (dj != 0) return -1.0 / dz;
    return (c.end_mode == 2 && (j == 0 || j == c.nz)) ? 1.0 / dz : 2.0 / dz;
}
static double mz(const pic_instance_cfg& c, double dz, int j, int dj) {
    if (dj != 0) return dz / 6.0;
    return (c.end_mode == 2 && (j == 0 || j == c.nz)) ? 2.0 * dz / 6.0 : 4.0 * dz / 6.0;
}

static double edge_value(const pic_instance_cfg& c, double dr, int i) {
    if (i == 0) return c.V_inner;
    if (i == c.nr) return c.V_outer;
    if (c.end_mode == 1) return c.V_end;
    double r = r_at(c, dr, (double)i);
    return c.V_inner + (c.V_outer - c.V_inner) * (log(r / c.a) / log(c.b / c.a)) + c.V_end;
}

// Vacuum right-hand side from the electrode data, taken relative to `shift`
// (V_outer with the elliptic insert: the insert's potential, so that the
// weighted basis, which vanishes on the insert, holds the solution).  phiB
// gets the data on the electrode nodes and `shift` elsewhere: the base the
// solution is added to.
static void host_vacuum_rhs(const pic_instance_cfg& c, double shift, std::vector<double>& phiB,
                            std::vector<double>& rhs) {
    const int nr = c.nr, nz = c.nz, W = nz + 1;
    const double dr = (c.b - c.a) / (double)nr, dz = c.L / (double)nz;
    phiB.assign((size_t)(nr + 1) * W, 0.0);
    rhs.assign((size_t)(nr + 1) * W, 0.0);
    // Dirichlet nodes: the radial electrodes, and the end plates unless the ends are open
    const bool open_ends = c.end_mode == 2;
    auto edge = [&](int i, int j) { return i == 0 || i == nr || (!open_ends && (j == 0 || j == nz)); };
    for (int i = 0; i <= nr; ++i)
        for (int j = 0; j <= nz; ++j)
            if (edge(i, j)) phiB[(size_t)i * W + j] = edge_value(c, dr, i) - shift;
    const int j0 = open_ends ? 0 : 1, j1 = open_ends ? nz : nz - 1;
    for (int i = 1; i < nr; ++i)
        for (int j = j0; j <= j1; ++j) {
            double s = 0.0;
            for (int di = -1; di <= 1; ++di)
                for (int dj = -1; dj <= 1; ++dj) {
                    if (j + dj < 0 || j + dj > nz || !edge(i + di, j + dj)) continue;
                    double A = kr(c, dr, i, di) * mz(c, dz, j, dj) + mr(c, dr, i, di) * kz(c, dz, j, dj);
                    s -= A * phiB[(size_t)(i + di) * W + (j + dj)];
                }
            rhs[(size_t)i * W + j] = s;
        }
    for (size_t n = 0; n < phiB.size(); ++n) phiB[n] += shift;
}

static void host_thomas(const pic_instance_cfg& c, int nseg, std::vector<double>& cp, std::vector<double>& im,
                        std::vector<double>& lo, std::vector<double>& G, std::vector<double>& H) {
    const int nr = c.nr, nz = c.nz, W = nz + 1;
    const double dr = (c.b - c.a) / (double)nr, dz = c.L / (double)nz;
    size_t N = (size_t)(nr + 1) * W;
    cp.assign(N, 0.0); im.assign(N, 0.0); lo.assign(N, 0.0);
    // sine modes 1..nz-1 with Dirichlet ends, cosine modes 0..nz with open ends
    const int k0 = c.end_mode == 2 ? 0 : 1, k1 = c.end_mode == 2 ? nz : nz - 1;
    for (int k = k0; k <= k1; ++k) {
        double ck = cos(kPi * (double)k / (double)nz);
        double mu = (dz / 3.0) * (2.0 + ck), lam = (2.0 / dz) * (1.0 - ck);
        double cprev = 0.0;
        for (int i = 1; i < nr; ++i) {
            double dg = mu * kr(c, dr, i, 0) + lam * mr(c, dr, i, 0);
            double up = mu * kr(c, dr, i, +1) + lam * mr(c, dr, i, +1);
            double lw = i > 1 ? mu * kr(c, dr, i, -1) + lam * mr(c, dr, i, -1) : 0.0;
            double m = dg - lw * cprev;
            size_t n = (size_t)i * W + k;
            lo[n] = lw;
            im[n] = 1.0 / m;
            cp[n] = up / m;
            cprev = cp[n];
        }
    }
    // homogeneous factors of the partitioned sweeps (same segments as the kernel)
    G.assign(N, 0.0);
    H.assign(N, 0.0);
    const int nri = nr - 1, seg = (nri + nseg - 1) / nseg;
    for (int k = k0; k <= k1; ++k)
        for (int sg = 0; sg < nseg; ++sg) {
            const int r0 = 1 + sg * seg, r1 = std::min(r0 + seg, nri + 1);
            double g = 1.0;
            for (int i = r0; i < r1; ++i) {
                size_t n = (size_t)i * W + k;
                g *= -(lo[n] * im[n]);
                G[n] = g;
            }
            double hh = 1.0;
            for (int i = r1 - 1; i >= r0; --i) {
                size_t n = (size_t)i * W + k;
                hh *= -cp[n];
                H[n] = hh;
            }
        }
}

// Cubic shapes: per z mode k the 7-band r system (mu_k Kr + kappa_k Mr),
// Kr = int r psi_i' psi_i'' dr, Mr = int r psi_i psi_i' dr over the
// odd-reflected cubic B-splines of the unknowns 1 .. nr-1 (4-point Gauss per
// cell, exact), mu_k and kappa_k the eigenvalues of the reflected cubic mass
// and stiffness in z (autocorrelations of the cubic B-spline and of its
// derivative) for the sine modes 1 .. nz-1 (odd reflection, electrode ends)
// or the cosine modes 0 .. nz (even reflection, open ends: the Galerkin end
// rows are half the periodic operator's, which the cosine transform of the
// loads accounts for); factored as L D L^T, stored [i][k].
static void host_spline3(const pic_instance_cfg& c, std::vector<double>& L1, std::vector<double>& L2,
                         std::vector<double>& L3, std::vector<double>& Dinv) {
    const int nr = c.nr, nz = c.nz, W = nz + 1, m = nr - 1;
    const double dr = (c.b - c.a) / (double)nr, dz = c.L / (double)nz;
    const size_t N = (size_t)(nr + 1) * W;
    L1.assign(N, 0.0); L2.assign(N, 0.0); L3.assign(N, 0.0); Dinv.assign(N, 0.0);
    const double gx[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                          0.86113631159405257522};
    const double gw[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                          0.34785484513745385737};
    // band storage [i][d] for (i, i - d), i = 1 .. m
    std::vector<double> K((size_t)(m + 1) * 4, 0.0), M((size_t)(m + 1) * 4, 0.0);
    auto fold = [&](int i, int& u) {
        if (i >= 1 && i <= nr - 1) { u = i; return 1; }
        if (i == -1) { u = 1; return -1; }
        if (i == nr + 1) { u = nr - 1; return -1; }
        return 0;
    };
    for (int cell = 0; cell < nr; ++cell)
        for (int q = 0; q < 4; ++q) {
            const double f = 0.5 * (1.0 + gx[q]);
            const double r = c.a + ((double)cell + f) * dr, wt = 0.5 * dr * gw[q] * r;
            double w[4], dw[4];
            bspline3(f, w, dw);
            for (int p1 = 0; p1 < 4; ++p1)
                for (int p2 = 0; p2 < 4; ++p2) {
                    int u1, u2;
                    const int s1 = fold(cell - 1 + p1, u1), s2 = fold(cell - 1 + p2, u2);
                    if (!s1 || !s2 || u2 > u1) continue;
                    const double sg = (double)(s1 * s2);
                    K[(size_t)u1 * 4 + (u1 - u2)] += sg * ((dw[p1] / dr) * (dw[p2] / dr)) * wt;
                    M[(size_t)u1 * 4 + (u1 - u2)] += sg * (w[p1] * w[p2]) * wt;
                }
        }
    const double mm[4] = {151.0 / 315.0, 397.0 / 1680.0, 1.0 / 42.0, 1.0 / 5040.0};
    const double kk[4] = {2.0 / 3.0, -1.0 / 8.0, -1.0 / 5.0, -1.0 / 120.0};
    std::vector<double> A((size_t)(m + 1) * 4), Lr((size_t)(m + 1) * 4, 0.0), D(m + 1, 0.0);
    const bool open = c.end_mode == 2;
    for (int k = open ? 0 : 1; k <= (open ? nz : nz - 1); ++k) {
        const double th = kPi * (double)k / (double)nz;
        double mu = mm[0], ka = kk[0];
        for (int l = 1; l <= 3; ++l) {
            mu += 2.0 * mm[l] * cos((double)l * th);
            ka += 2.0 * kk[l] * cos((double)l * th);
        }
        mu *= dz;
        ka /= dz;
        for (size_t t = 0; t < A.size(); ++t) A[t] = mu * K[t] + ka * M[t];
        for (int i = 1; i <= m; ++i) {
            for (int d = 3; d >= 1; --d) {
                const int j = i - d;
                if (j < 1) continue;
                double v = A[(size_t)i * 4 + d];
                for (int t = std::max(1, i - 3); t < j; ++t)
                    v -= Lr[(size_t)i * 4 + (i - t)] * Lr[(size_t)j * 4 + (j - t)] * D[t];
                Lr[(size_t)i * 4 + d] = v / D[j];
            }
            double dd = A[(size_t)i * 4];
            for (int t = std::max(1, i - 3); t < i; ++t) dd -= Lr[(size_t)i * 4 + (i - t)] * Lr[(size_t)i * 4 + (i - t)] * D[t];
            D[i] = dd;
            const size_t n = (size_t)i * W + k;
            L1[n] = Lr[(size_t)i * 4 + 1];
            L2[n] = Lr[(size_t)i * 4 + 2];
            L3[n] = Lr[(size_t)i * 4 + 3];
            Dinv[n] = 1.0 / dd;
        }
    }
}

static void host_volume(const pic_instance_cfg& c, std::vector<double>& V) {
    const int nr = c.nr, nz = c.nz, W = nz + 1;
    const double dr = (c.b - c.a) / (double)nr, dz = c.L / (double)nz;
    V.assign((size_t)(nr + 1) * W, 0.0);
    for (int i = 0; i <= nr; ++i) {
        double lr = i == 0 ? dr * (c.a / 2.0 + dr / 6.0)
                  : (i == nr ? dr * (c.b / 2.0 - dr / 6.0) : r_at(c, dr, (double)i) * dr);
        for (int j = 0; j <= nz; ++j) {
            double lz = (j == 0 || j == nz) ? dz / 2.0 : dz;
            V[(size_t)i * W + j] = 2.0 * kPi * lr * lz;
        }
    }
}

static void fill_devinst(Inst& in) {
    const pic_instance_cfg& c = in.c;
    const pic_derived_t& d = in.d;
    DevInst& I = in.I;
    memset(&I, 0, sizeof(I));
    I.a = c.a; I.b = c.b; I.L = c.L; I.dr = d.dr; I.dz = d.dz; I.inv_dr = d.inv_dr; I.inv_dz = d.inv_dz;
    I.nr = c.nr; I.nz = c.nz; I.W = c.nz + 1; I.nodes = (c.nr + 1) * (c.nz + 1);
    I.h = d.h; I.dt = c.dt;
    I.P_null = d.P_null; I.nu_prime = d.nu_prime; I.nsig_el = d.nsig_el; I.n_n = d.n_n;
    I.lotz_aq = d.lotz_aq; I.iz_I = c.iz_I_eV; I.opal_Ebar = c.opal_Ebar_eV; I.okh_xi = c.okh_xi;
    I.half_me_over_e = d.half_me_over_e; I.two_e_over_me = d.two_e_over_me;
    I.mass_ratio2 = d.mass_ratio2; I.v_cap2 = d.v_cap * d.v_cap;
    I.null_k = null_threshold(d.P_null);
    I.seed_lo = (unsigned int)c.seed; I.seed_hi = (unsigned int)(c.seed >> 32);
    I.collisions = c.collisions;
    I.frozen = in.frozen ? 1 : 0;
    I.two_S = d.two_S; I.inv_two_S = d.inv_two_S;
    I.p_cap = in.cap;
    I.a_f = (float)c.a; I.b_f = (float)c.b; I.L_f = (float)c.L;
    I.inv_dr_f = (float)d.inv_dr; I.inv_dz_f = (float)d.inv_dz; I.h_f = (float)d.h; I.dt_f = (float)c.dt;
    I.nu_prime_f = (float)d.nu_prime; I.nsig_el_f = (float)d.nsig_el; I.n_n_f = (float)d.n_n;
    I.lotz_aq_f = (float)d.lotz_aq; I.iz_I_f = (float)c.iz_I_eV; I.opal_Ebar_f = (float)c.opal_Ebar_eV;
    I.okh_xi_f = (float)c.okh_xi; I.half_me_over_e_f = (float)d.half_me_over_e;
    I.okh_inv_E0 = c.okh_E0_eV > 0.0 ? 1.0 / c.okh_E0_eV : 0.0;
    I.okh_inv_E0_f = (float)I.okh_inv_E0;
    I.two_e_over_me_f = (float)d.two_e_over_me; I.mass_ratio2_f = (float)d.mass_ratio2;
    I.v_cap2_f = (float)(d.v_cap * d.v_cap);
    I.diag_D = c.diag_interval > 0 ? c.diag_interval : 1;
    I.open_ends = c.end_mode == 2 ? 1 : 0;
    I.src_rate = c.src_rate;
    I.src_sv = sqrt(((c.src_T_eV > 0.0 ? c.src_T_eV : c.T_init_eV) * kE) / kMe);
    I.weight = c.weight;
    I.w_uni = (float)c.weight;
    I.has_ins = (c.ins_er > 0.0 && c.ins_ez > 0.0) ? 1 : 0;
    I.spline3 = c.spline_order == 3 ? 1 : 0;
    if (I.has_ins) {
        ins_fill(c, d.dr, d.dz, I);
        I.ins_r0_f = (float)c.ins_r0; I.ins_z0_f = (float)c.ins_z0;
        I.ins_inv_er_f = (float)(1.0 / c.ins_er); I.ins_inv_ez_f = (float)(1.0 / c.ins_ez);
        I.ins_gam_f = (float)I.ins_gam;
    }
}

static pic_status upload_insert_inst(pic_ctx* ctx) {
    if (ctx->ins_list.empty()) return PIC_OK;
    std::vector<DevInst> Ii;
    for (int k : ctx->ins_list) Ii.push_back(ctx->in[k].I);
    CK(hipMemcpyAsync(ctx->dIins, Ii.data(), sizeof(DevInst) * Ii.size(), hipMemcpyHostToDevice, ctx->stream));
    return PIC_OK;
}

// Groups of insert instances sharing one H: group g holds the entries
// gmem[goff[g] .. goff[g+1]) of D.
static void h_groups(const std::vector<InsDev>& D, std::vector<int>& goff, std::vector<int>& gmem, int& n_grp) {
    std::vector<const double*> hs;
    std::vector<std::vector<int>> mem;
    for (size_t t = 0; t < D.size(); ++t) {
        size_t g = std::find(hs.begin(), hs.end(), D[t].H) - hs.begin();
        if (g == hs.size()) {
            hs.push_back(D[t].H);
            mem.emplace_back();
        }
        mem[g].push_back((int)t);
    }
    goff.assign(1, 0);
    gmem.clear();
    for (auto& v : mem) {
        gmem.insert(gmem.end(), v.begin(), v.end());
        goff.push_back((int)gmem.size());
    }
    n_grp = (int)mem.size();
}

static pic_status upload_tables(pic_ctx* ctx) {
    std::vector<DevInst> I;
    std::vector<FieldDev> F, Fv, F1, F1v, F2, F2v, F3, F3a, F3b;
    std::vector<InsDev> D, D3;
    std::vector<Ins3Dev> X3;
    std::vector<double> bs;
    for (auto& in : ctx->in) {
        in.I.frozen = in.frozen ? 1 : 0;
        I.push_back(in.I);
        FieldDev f;
        memset(&f, 0, sizeof(f));
        f.Q = in.Q; f.rhs = in.rhs; f.phi = in.phi; f.phi_vac = in.phi_vac;
        f.th_cp = in.th_cp; f.th_im = in.th_im; f.th_lo = in.th_lo;
        f.th_G = in.th_G; f.th_H = in.th_H;
        f.Er = in.Er; f.Ez = in.Ez; f.Br = in.Br; f.Bz = in.Bz; f.EB = in.EB;
        f.V = in.V; f.avg_acc = in.avg_acc;
        f.Qw = in.Qw;
        f.Qx = in.Qx;
        f.cx = in.cx;
        f.cxf = in.cxf;
        F.push_back(f);
        FieldDev v = f;  // vacuum solve: boundary data in, phi_vac out
        v.phi_vac = in.phiB;
        v.phi = in.phi_vac;
        Fv.push_back(v);
        // first of the two solves of an insert instance: phi goes to ybuf
        FieldDev f1 = f, f1v = v;
        if (in.has_ins) {
            f1.phi = in.idev.ybuf;
            f1v.phi = in.idev.ybuf;
            FieldDev f2 = f, f2v = v;  // second: the correction's modes, on top of ybuf
            f2.rhs = in.idev.rhs2;
            f2.phi_vac = in.idev.ybuf;
            f2v.rhs = in.idev.rhs2;
            f2v.phi_vac = in.idev.ybuf;
            F2.push_back(f2);
            F2v.push_back(f2v);
            D.push_back(in.idev);
        }
        F1.push_back(f1);
        F1v.push_back(f1v);
        bs.push_back(in.d.bscale);
        if (ctx->s3) {
            FieldDev f3 = f;
            f3.phi = in.cbuf;
            f3.phi_vac = in.zeros;
            f3.s3_L1 = in.s3_L1; f3.s3_L2 = in.s3_L2; f3.s3_L3 = in.s3_L3; f3.s3_Dinv = in.s3_Dinv;
            F3.push_back(f3);
            // with the insert: the first solve into ybuf, the second (the
            // correction's load on top of ybuf) into the coefficient buffer
            FieldDev f3a = f3;
            if (in.has_ins) {
                f3a.phi = in.idev3.ybuf;
                FieldDev f3b = f3;
                f3b.rhs = in.idev3.rhs2;
                f3b.phi_vac = in.idev3.ybuf;
                F3b.push_back(f3b);
                D3.push_back(in.idev3);
                X3.push_back(in.xdev3);
            }
            F3a.push_back(f3a);
        }
    }
    hipStream_t s = ctx->stream;
    CK(hipMemcpyAsync(ctx->dI, I.data(), sizeof(DevInst) * I.size(), hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(ctx->dF, F.data(), sizeof(FieldDev) * F.size(), hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(ctx->dFvac, Fv.data(), sizeof(FieldDev) * Fv.size(), hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(ctx->dbscale, bs.data(), sizeof(double) * bs.size(), hipMemcpyHostToDevice, s));
    if (ctx->s3) CK(hipMemcpyAsync(ctx->dF3, F3.data(), sizeof(FieldDev) * F3.size(), hipMemcpyHostToDevice, s));
    if (!ctx->ins_list.empty()) {
        CK(hipMemcpyAsync(ctx->dF1, F1.data(), sizeof(FieldDev) * F1.size(), hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(ctx->dF1v, F1v.data(), sizeof(FieldDev) * F1v.size(), hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(ctx->dF2, F2.data(), sizeof(FieldDev) * F2.size(), hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(ctx->dF2v, F2v.data(), sizeof(FieldDev) * F2v.size(), hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(ctx->dIns, D.data(), sizeof(InsDev) * D.size(), hipMemcpyHostToDevice, s));
        // groups of insert instances by their H (shared between equal corrected systems)
        h_groups(D, ctx->h_goff, ctx->h_gmem, ctx->n_grp);
        CK(hipMemcpyAsync(ctx->dGoff, ctx->h_goff.data(), sizeof(int) * ctx->h_goff.size(), hipMemcpyHostToDevice,
                          s));
        CK(hipMemcpyAsync(ctx->dGmem, ctx->h_gmem.data(), sizeof(int) * ctx->h_gmem.size(), hipMemcpyHostToDevice,
                          s));
        if (ctx->s3) {
            CK(hipMemcpyAsync(ctx->dF3a, F3a.data(), sizeof(FieldDev) * F3a.size(), hipMemcpyHostToDevice, s));
            CK(hipMemcpyAsync(ctx->dF3b, F3b.data(), sizeof(FieldDev) * F3b.size(), hipMemcpyHostToDevice, s));
            CK(hipMemcpyAsync(ctx->dIns3, D3.data(), sizeof(InsDev) * D3.size(), hipMemcpyHostToDevice, s));
            CK(hipMemcpyAsync(ctx->dX3, X3.data(), sizeof(Ins3Dev) * X3.size(), hipMemcpyHostToDevice, s));
            h_groups(D3, ctx->h_goff3, ctx->h_gmem3, ctx->n_grp3);
            CK(hipMemcpyAsync(ctx->dGoff3, ctx->h_goff3.data(), sizeof(int) * ctx->h_goff3.size(),
                              hipMemcpyHostToDevice, s));
            CK(hipMemcpyAsync(ctx->dGmem3, ctx->h_gmem3.data(), sizeof(int) * ctx->h_gmem3.size(),
                              hipMemcpyHostToDevice, s));
        }
        pic_status st = upload_insert_inst(ctx);
        if (st != PIC_OK) return st;
    }
    CK(hipStreamSynchronize(s));
    return PIC_OK;
}

// One Poisson solve of every instance into the field table `fin` (the main
// table, or the vacuum table).  Instances with the elliptic insert take the
// corrected two-solve path: first into ybuf, the M correction, the second
// solve on top of ybuf, then the basis evaluated at the nodes of M.
static pic_status solve_tables(pic_ctx* ctx, bool vac, bool from_q, bool edges, hipStream_t s) {
    const int n = (int)ctx->in.size(), ni = (int)ctx->ins_list.size();
    FieldDev* fin = vac ? ctx->dFvac : ctx->dF;
    if (ni == 0) {
        CK(launch_solve_tab(ctx->dI, fin, 0, n, ctx->max_nr, ctx->max_nz, ctx->tw, ctx->tw_n, from_q ? 0 : 1,
                            ctx->dbscale, edges, s));
        return PIC_OK;
    }
    FieldDev* f1 = vac ? ctx->dF1v : ctx->dF1;
    FieldDev* f2 = vac ? ctx->dF2v : ctx->dF2;
    if (from_q) CK(launch_ins_rhs(ctx->dI, ctx->dIns, ni, ctx->max_nodes, ctx->dF, ctx->dbscale, s));
    CK(launch_solve_tab(ctx->dI, f1, 0, n, ctx->max_nr, ctx->max_nz, ctx->tw, ctx->tw_n, from_q ? 0 : 1,
                        ctx->dbscale, edges, s));
    CK(launch_ins_correct(ctx->dI, ctx->dIns, ni, ctx->dGoff, ctx->dGmem, ctx->n_grp, ctx->max_m, ctx->max_nodes,
                          f1, s));
    CK(launch_solve_tab(ctx->dIins, f2, 0, ni, ctx->max_nr, ctx->max_nz, ctx->tw, ctx->tw_n, 1, ctx->dbscale,
                        edges, s));
    CK(launch_ins_fix(ctx->dI, ctx->dIns, ni, ctx->max_m, fin, s));
    return PIC_OK;
}

// Cubic space-charge solve of every non-frozen instance from Qx (and the
// band charges Qw of the insert instances): the plain fast solve, or for a
// context with inserts the load of M over the folded load, the first fast
// solve (insert instances into ybuf), the correction through H, the second
// fast solve of the insert instances on top of ybuf, the ghosted
// coefficients and nodal potential, rebuilt where the insert changes them.
static pic_status solve3_tables(pic_ctx* ctx, hipStream_t s) {
    const int n = (int)ctx->in.size(), ni = (int)ctx->ins_list.size();
    if (ni == 0) {
        CK(launch_solve3_tab(ctx->dI, ctx->dF, ctx->dF3, n, ctx->max_nr, ctx->max_nz, ctx->max_ext, ctx->tw,
                             ctx->tw_n, ctx->dbscale, s));
        return PIC_OK;
    }
    CK(launch_s3_fold(ctx->dI, ctx->dF3, n, ctx->max_nodes, ctx->dbscale, s));
    CK(launch_ins3_rhs(ctx->dI, ctx->dX3, ni, ctx->max_m3, ctx->dF3, ctx->dbscale, s));
    CK(launch_s3_rect(ctx->dI, ctx->dF3a, n, ctx->max_nr, ctx->max_nz, ctx->tw, ctx->tw_n, ctx->dbscale, s));
    CK(launch_ins_correct(ctx->dI, ctx->dIns3, ni, ctx->dGoff3, ctx->dGmem3, ctx->n_grp3, ctx->max_m3,
                          ctx->max_nodes, ctx->dF3, s));
    CK(launch_s3_rect(ctx->dIins, ctx->dF3b, ni, ctx->max_nr, ctx->max_nz, ctx->tw, ctx->tw_n, ctx->dbscale, s));
    CK(launch_s3_post(ctx->dI, ctx->dF, ctx->dF3, n, ctx->max_ext, s));
    CK(launch_ins3_post(ctx->dI, ctx->dX3, ni, ctx->max_nx3, ctx->max_nodes, ctx->dF, ctx->dF3, s));
    return PIC_OK;
}

// Field of every non-frozen instance from its current Q.
pic_status pic_solve_all(pic_ctx* ctx) {
    int n = (int)ctx->in.size();
    hipStream_t s = ctx->stream;
    if (ctx->s3) return solve3_tables(ctx, s);  // the nodal E arrays keep the vacuum field
    pic_status st = solve_tables(ctx, false, true, true, s);
    if (st != PIC_OK) return st;
    CK(launch_efield_tab(ctx->dI, ctx->dF, 0, n, ctx->max_nodes, true, s));
    return PIC_OK;
}

pic_status pic_field_stage(pic_ctx* ctx, hipStream_t s) {
    int n = (int)ctx->in.size();
    // per step: the electrode rows of phi and the static B half of EB keep
    // the values the initial solve (or pic_set_fields) gave them
    if (ctx->s3) {
        pic_status st = solve3_tables(ctx, s);
        if (st != PIC_OK) return st;
        CK(launch_sample_tab(ctx->dI, ctx->dF, n, ctx->dcnt, ctx->prep_ctl, s));
        return PIC_OK;
    }
    pic_status st = solve_tables(ctx, false, true, false, s);
    if (st != PIC_OK) return st;
    CK(launch_efield_tab(ctx->dI, ctx->dF, 0, n, ctx->max_nodes, false, s, ctx->dcnt));
    CK(launch_commit(ctx->dI, ctx->dcnt, ctx->prep_ctl, n, s));
    return PIC_OK;
}

FieldDev* pic_field_table(pic_ctx* ctx) { return ctx->dF; }

void pic_set_prep_ctl(pic_ctx* ctx, long long* ctl) { ctx->prep_ctl = ctl; }

// Accessors used by the FP32 form (fp32.hip).
int pic_n_inst(pic_ctx* ctx) { return (int)ctx->in.size(); }
DevInst& pic_inst_dev(pic_ctx* ctx, int k) { return ctx->in[k].I; }
const pic_instance_cfg& pic_inst_cfg(pic_ctx* ctx, int k) { return ctx->in[k].c; }
long long* pic_counters(pic_ctx* ctx) { return ctx->dcnt; }
long long* pic_inst_Q(pic_ctx* ctx, int k) { return ctx->in[k].Q; }
long long pic_inst_nodes(pic_ctx* ctx, int k) { return ctx->in[k].nodes; }
const double* pic_inst_volume(pic_ctx* ctx, int k) { return ctx->in[k].V; }
long long* pic_inst_Qw(pic_ctx* ctx, int k) { return ctx->in[k].Qw; }
long long* pic_inst_Qx(pic_ctx* ctx, int k) { return ctx->in[k].Qx; }
float4* pic_inst_EB(pic_ctx* ctx, int k) { return ctx->in[k].EB; }
DevInst* pic_dev_table(pic_ctx* ctx) { return ctx->dI; }
long long& pic_inst_cap(pic_ctx* ctx, int k) { return ctx->in[k].cap; }

pic_status pic_upload_inst(pic_ctx* ctx) {
    std::vector<DevInst> I;
    for (auto& in : ctx->in) {
        in.I.frozen = in.frozen ? 1 : 0;
        in.I.p_cap = ctx->mode == PIC_MODE_FP64_PLAIN ? in.cap : in.I.p_cap;
        I.push_back(in.I);
    }
    CK(hipMemcpyAsync(ctx->dI, I.data(), sizeof(DevInst) * I.size(), hipMemcpyHostToDevice, ctx->stream));
    pic_status st = upload_insert_inst(ctx);
    if (st != PIC_OK) return st;
    CK(hipStreamSynchronize(ctx->stream));
    return PIC_OK;
}
const pic_run_cfg& pic_run(pic_ctx* ctx) { return ctx->run; }
void pic_set_error(pic_ctx* ctx, const std::string& m) { ctx->err = m; }
bool pic_timing_on(pic_ctx* ctx) { return ctx->timing; }

// Record a timed launch: returns the start event to record before the launch
// and stores the stop event in *stop.
hipEvent_t pic_timing_begin(pic_ctx* ctx, hipEvent_t* stop) {
    if (ctx->ev_used + 2 > ctx->ev.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            // timing only (read after a stream synchronisation): no system-scope
            // fence, whose cache writeback and invalidation would be timed too
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            ctx->ev.push_back(e);
        }
    }
    hipEvent_t a = ctx->ev[ctx->ev_used], b = ctx->ev[ctx->ev_used + 1];
    ctx->ev_used += 2;
    *stop = b;
    return a;
}

static pic_status timing_collect(pic_ctx* ctx) {
    if (ctx->ev_used == 0) return PIC_OK;
    CK(hipStreamSynchronize(ctx->stream));
    for (size_t k = 0; k + 1 < ctx->ev_used; k += 2) {
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
        ctx->timed_ms += ms;
        ctx->timed_launches += 1;
    }
    ctx->ev_used = 0;
    return PIC_OK;
}

// ---------------------------------------------------------------------------
// init / destroy
// ---------------------------------------------------------------------------

template <typename T>
static T* upload_vec(pic_ctx* ctx, const std::vector<T>& v, hipStream_t s, bool& ok) {
    T* p = dalloc<T>(ctx, std::max<long long>(1, (long long)v.size()));
    if (!p) {
        ok = false;
        return nullptr;
    }
    if (!v.empty() && hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        ok = false;
    return p;
}

// Whether two insert instances have the same corrected system (mesh, end
// conditions, node set M and correction entries D), so that one H serves both.
static bool same_insert_system(const Inst& x, const Inst& y) {
    const pic_instance_cfg &a = x.c, &b = y.c;
    return a.nr == b.nr && a.nz == b.nz && a.a == b.a && a.b == b.b && a.L == b.L && a.end_mode == b.end_mode &&
           x.ih.m == y.ih.m && x.ih.Mnode == y.ih.Mnode && x.ih.Dr == y.ih.Dr && x.ih.Dc == y.ih.Dc &&
           x.ih.Dv == y.ih.Dv;
}

// Entries of the band-charge grid Qw: one per node with bilinear shapes, the
// ghosted (nr+3) x (nz+3) grid with cubic shapes.
static long long band_cells(const Inst& in) {
    return in.I.spline3 ? (long long)(in.c.nr + 3) * (in.c.nz + 3) : in.nodes;
}

// Device arrays of an instance's insert.  H is filled by setup_insert, or is
// that of an earlier instance with the same corrected system.
static pic_status init_insert_storage(pic_ctx* ctx, Inst& in) {
    const InsHost& h = in.ih;
    InsDev& D = in.idev;
    hipStream_t s = ctx->stream;
    bool ok = true;
    const long long N = in.nodes, m = std::max(1, h.m);
    D.m = h.m;
    D.nodes = N;
    D.Mnode = upload_vec(ctx, h.Mnode, s, ok);
    D.map = upload_vec(ctx, h.map, s, ok);
    D.rp = upload_vec(ctx, h.rp, s, ok);
    D.rk = upload_vec(ctx, h.rk, s, ok);
    D.rf = upload_vec(ctx, h.rf, s, ok);
    D.typ = upload_vec(ctx, h.typ, s, ok);
    D.wn = upload_vec(ctx, h.wn, s, ok);
    D.ek = upload_vec(ctx, h.ek, s, ok);
    D.ef = upload_vec(ctx, h.ef, s, ok);
    in.h_owner = -1;
    for (size_t k = 0; k < ctx->in.size() && &ctx->in[k] != &in; ++k) {
        const Inst& o = ctx->in[k];
        if (o.has_ins && o.h_owner < 0 && o.idev.H && same_insert_system(o, in)) {
            in.h_owner = (int)k;
            break;
        }
    }
    double* H = in.h_owner >= 0 ? const_cast<double*>(ctx->in[in.h_owner].idev.H) : dalloc<double>(ctx, m * m);
    D.H = H;
    D.ybuf = dalloc<double>(ctx, N);
    D.rhs2 = dalloc<double>(ctx, N);
    D.yM = dalloc<double>(ctx, m);
    D.sM = dalloc<double>(ctx, m);
    D.val = dalloc<double>(ctx, m);
    const long long nQw = band_cells(in);
    in.Qw = dalloc<long long>(ctx, nQw);
    if (!ok || !H || !D.ybuf || !D.rhs2 || !D.yM || !D.sM || !D.val || !in.Qw)
        return fail(ctx, PIC_ENOMEM, "device allocation of the insert arrays failed");
    if (in.h_owner < 0) CK(hipMemsetAsync(H, 0, sizeof(double) * m * m, s));
    CK(hipMemsetAsync(D.ybuf, 0, sizeof(double) * N, s));
    CK(hipMemsetAsync(D.rhs2, 0, sizeof(double) * N, s));
    CK(hipMemsetAsync(in.Qw, 0, sizeof(long long) * nQw, s));
    CK(hipStreamSynchronize(s));
    return PIC_OK;
}

// H = (I + D G)^-1 D with G = (A_rect^-1)_MM from m unit solves of the
// rectangle system (batched as copies of the instance; the cubic one when
// cubic), Gauss-Jordan on the device.
static pic_status build_H(pic_ctx* ctx, Inst& in, int m, const int* Mnode, const std::vector<int>& Dr,
                          const std::vector<int>& Dc, const std::vector<double>& Dv, double* Hout, bool cubic) {
    hipStream_t s = ctx->stream;
    const long long N = in.nodes;
    const int B = std::min(64, m);
    double* rhsT = dalloc<double>(ctx, (long long)B * N);
    double* phiT = dalloc<double>(ctx, (long long)B * N);
    double* zeros = dalloc<double>(ctx, N);
    DevInst* It = dalloc<DevInst>(ctx, B);
    FieldDev* Ftab = dalloc<FieldDev>(ctx, B);
    double* Gd = dalloc<double>(ctx, (long long)m * m);
    double* CDd = dalloc<double>(ctx, (long long)m * 2 * m);
    double* fcol = dalloc<double>(ctx, m);
    double* pval = dalloc<double>(ctx, m);
    int* piv = dalloc<int>(ctx, 1);
    auto release = [&]() {
        void* ps[] = {rhsT, phiT, zeros, It, Ftab, Gd, CDd, fcol, pval, piv};
        for (void* p : ps)
            if (p) pic_dev_free(ctx, p);
    };
    if (!rhsT || !phiT || !zeros || !It || !Ftab || !Gd || !CDd || !fcol || !pval || !piv) {
        release();
        return fail(ctx, PIC_ENOMEM, "device allocation for the insert set-up failed");
    }
    DevInst I = in.I;
    I.frozen = 0;
    I.has_ins = 0;
    std::vector<DevInst> Iv(B, I);
    std::vector<FieldDev> Fv(B);
    for (int t = 0; t < B; ++t) {
        FieldDev f;
        memset(&f, 0, sizeof(f));
        f.Q = in.Q;
        f.rhs = rhsT + (long long)t * N;
        f.phi = phiT + (long long)t * N;
        f.phi_vac = zeros;
        f.th_cp = in.th_cp; f.th_im = in.th_im; f.th_lo = in.th_lo; f.th_G = in.th_G; f.th_H = in.th_H;
        f.s3_L1 = in.s3_L1; f.s3_L2 = in.s3_L2; f.s3_L3 = in.s3_L3; f.s3_Dinv = in.s3_Dinv;
        Fv[t] = f;
    }
    hipError_t e = hipMemsetAsync(zeros, 0, sizeof(double) * N, s);
    if (e == hipSuccess) e = hipMemsetAsync(phiT, 0, sizeof(double) * B * N, s);
    if (e == hipSuccess) e = hipMemcpyAsync(It, Iv.data(), sizeof(DevInst) * B, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(Ftab, Fv.data(), sizeof(FieldDev) * B, hipMemcpyHostToDevice, s);
    for (int b0 = 0; b0 < m && e == hipSuccess; b0 += B) {
        const int cnt = std::min(B, m - b0);
        e = launch_ins_units(rhsT, N, N, Mnode, b0, cnt, s);
        if (e == hipSuccess)
            e = cubic ? launch_s3_rect(It, Ftab, cnt, ctx->max_nr, ctx->max_nz, ctx->tw, ctx->tw_n, ctx->dbscale, s)
                      : launch_solve_tab(It, Ftab, 0, cnt, ctx->max_nr, ctx->max_nz, ctx->tw, ctx->tw_n, 1,
                                         ctx->dbscale, false, s);
        if (e == hipSuccess) e = launch_ins_collect(phiT, N, Mnode, m, b0, cnt, Gd, s);
    }
    std::vector<double> G((size_t)m * m);
    if (e == hipSuccess) e = hipMemcpyAsync(G.data(), Gd, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release();
        return fail(ctx, PIC_EDEVICE, std::string("insert set-up solves: ") + hipGetErrorString(e));
    }
    // [C | D] with C = I + D G
    std::vector<double> CD((size_t)m * 2 * m, 0.0);
    for (int a = 0; a < m; ++a) CD[(size_t)a * 2 * m + a] = 1.0;
    for (size_t t = 0; t < Dv.size(); ++t) {
        const int a = Dr[t], c = Dc[t];
        const double v = Dv[t];
        double* row = &CD[(size_t)a * 2 * m];
        const double* gr = &G[(size_t)c * m];
        for (int j = 0; j < m; ++j) row[j] += v * gr[j];
        row[m + c] += v;
    }
    e = hipMemcpyAsync(CDd, CD.data(), sizeof(double) * CD.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_ins_gauss_jordan(CDd, m, fcol, piv, pval, s);
    std::vector<double> pv(m);
    if (e == hipSuccess) e = hipMemcpyAsync(pv.data(), pval, sizeof(double) * m, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync((void*)Hout, sizeof(double) * m, CDd + m, sizeof(double) * 2 * m, sizeof(double) * m, m,
                             hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) return fail(ctx, PIC_EDEVICE, std::string("insert set-up: ") + hipGetErrorString(e));
    for (int a = 0; a < m; ++a)
        if (!(std::fabs(pv[a]) > 0.0) || !std::isfinite(pv[a]))
            return fail(ctx, PIC_EINVAL, "insert: the corrected system is singular");
    return PIC_OK;
}

static pic_status setup_insert(pic_ctx* ctx, Inst& in) {
    if (in.ih.m > 0 && in.h_owner < 0) {
        pic_status st = build_H(ctx, in, in.ih.m, in.idev.Mnode, in.ih.Dr, in.ih.Dc, in.ih.Dv,
                                const_cast<double*>(in.idev.H), false);
        if (st != PIC_OK) return st;
    }
    if (in.I.spline3 && in.ih3.m > 0 && in.h3_owner < 0)
        return build_H(ctx, in, in.ih3.m, in.idev3.Mnode, in.ih3.Dr, in.ih3.Dc, in.ih3.Dv,
                       const_cast<double*>(in.idev3.H), true);
    return PIC_OK;
}

// Whether two cubic insert instances have the same corrected system.
static bool same_insert3_system(const Inst& x, const Inst& y) {
    const pic_instance_cfg &a = x.c, &b = y.c;
    return a.nr == b.nr && a.nz == b.nz && a.a == b.a && a.b == b.b && a.L == b.L && a.end_mode == b.end_mode &&
           x.ih3.m == y.ih3.m && x.ih3.Mnode == y.ih3.Mnode && x.ih3.Dr == y.ih3.Dr && x.ih3.Dc == y.ih3.Dc &&
           x.ih3.Dv == y.ih3.Dv;
}

// Device arrays of an instance's cubic web-spline system.
static pic_status init_insert3_storage(pic_ctx* ctx, Inst& in) {
    const Ins3Host& h = in.ih3;
    InsDev& D = in.idev3;
    Ins3Dev& X = in.xdev3;
    hipStream_t s = ctx->stream;
    bool ok = true;
    const long long N = in.nodes, m = std::max(1, h.m);
    D.m = h.m;
    D.nodes = N;
    D.Mnode = upload_vec(ctx, h.Mnode, s, ok);
    D.map = upload_vec(ctx, h.map, s, ok);
    X.m = h.m;
    X.nx = h.nx;
    X.Mnode = D.Mnode;
    X.typ = upload_vec(ctx, h.typ, s, ok);
    X.rp = upload_vec(ctx, h.rp, s, ok);
    X.rk = upload_vec(ctx, h.rk, s, ok);
    X.rf = upload_vec(ctx, h.rf, s, ok);
    X.xk = upload_vec(ctx, h.xk, s, ok);
    X.xn = upload_vec(ctx, h.xn, s, ok);
    X.xf = upload_vec(ctx, h.xf, s, ok);
    in.h3_owner = -1;
    for (size_t k = 0; k < ctx->in.size() && &ctx->in[k] != &in; ++k) {
        const Inst& o = ctx->in[k];
        if (o.has_ins && o.h3_owner < 0 && o.idev3.H && same_insert3_system(o, in)) {
            in.h3_owner = (int)k;
            break;
        }
    }
    double* H = in.h3_owner >= 0 ? const_cast<double*>(ctx->in[in.h3_owner].idev3.H) : dalloc<double>(ctx, m * m);
    D.H = H;
    D.ybuf = dalloc<double>(ctx, N);
    D.rhs2 = dalloc<double>(ctx, N);
    D.yM = dalloc<double>(ctx, m);
    D.sM = dalloc<double>(ctx, m);
    if (!ok || !H || !D.ybuf || !D.rhs2 || !D.yM || !D.sM)
        return fail(ctx, PIC_ENOMEM, "device allocation of the cubic insert arrays failed");
    if (in.h3_owner < 0) CK(hipMemsetAsync(H, 0, sizeof(double) * m * m, s));
    CK(hipMemsetAsync(D.ybuf, 0, sizeof(double) * N, s));
    CK(hipMemsetAsync(D.rhs2, 0, sizeof(double) * N, s));
    CK(hipStreamSynchronize(s));
    return PIC_OK;
}

static pic_status init_instance_storage(pic_ctx* ctx, Inst& in) {
    const long long N = in.nodes;
    in.Q = dalloc<long long>(ctx, N);
    in.rhs = dalloc<double>(ctx, N);
    in.phi = dalloc<double>(ctx, N);
    in.phi_vac = dalloc<double>(ctx, N);
    in.phiB = dalloc<double>(ctx, N);
    in.Br = dalloc<double>(ctx, N);
    in.Bz = dalloc<double>(ctx, N);
    in.V = dalloc<double>(ctx, N);
    in.avg_acc = dalloc<double>(ctx, N);
    // The r-direction factors depend only on the mesh and the end condition:
    // instances that agree on these share one copy (read-only after set-up),
    // so a batched solve streams them once from the cache for all of them.
    const Inst* twin = nullptr;
    for (const Inst& o : ctx->in) {
        if (&o == &in) break;
        if (o.th_cp && o.c.nr == in.c.nr && o.c.nz == in.c.nz && o.c.a == in.c.a && o.c.b == in.c.b &&
            o.c.L == in.c.L && o.c.end_mode == in.c.end_mode) {
            twin = &o;
            break;
        }
    }
    if (twin) {
        in.th_cp = twin->th_cp; in.th_im = twin->th_im; in.th_lo = twin->th_lo;
        in.th_G = twin->th_G; in.th_H = twin->th_H;
    } else {
        in.th_cp = dalloc<double>(ctx, N);
        in.th_im = dalloc<double>(ctx, N);
        in.th_lo = dalloc<double>(ctx, N);
        in.th_G = dalloc<double>(ctx, N);
        in.th_H = dalloc<double>(ctx, N);
    }
    if (!in.Q || !in.rhs || !in.phi || !in.phi_vac || !in.phiB || !in.Br || !in.Bz || !in.V ||
        !in.avg_acc || !in.th_cp || !in.th_im || !in.th_lo || !in.th_G || !in.th_H)
        return fail(ctx, PIC_ENOMEM, "device allocation of node arrays failed");
    if (ctx->mode == PIC_MODE_FP64_PLAIN) {
        in.Er = dalloc<double>(ctx, N);
        in.Ez = dalloc<double>(ctx, N);
        if (!in.Er || !in.Ez) return fail(ctx, PIC_ENOMEM, "device allocation of E failed");
        for (int b = 0; b < 2; ++b) {
            P64& p = in.p64[b];
            p.r = dalloc<double>(ctx, in.cap);
            p.z = dalloc<double>(ctx, in.cap);
            p.vr = dalloc<double>(ctx, in.cap);
            p.vt = dalloc<double>(ctx, in.cap);
            p.vz = dalloc<double>(ctx, in.cap);
            p.w = dalloc<double>(ctx, in.cap);
            p.key = dalloc<unsigned long long>(ctx, in.cap);
            if (!p.r || !p.z || !p.vr || !p.vt || !p.vz || !p.w || !p.key)
                return fail(ctx, PIC_ENOMEM, "device allocation of FP64 particles failed");
        }
    } else {
        in.EB = dalloc<float4>(ctx, N);
        if (!in.EB) return fail(ctx, PIC_ENOMEM, "device allocation of EB failed");
    }
    hipStream_t s = ctx->stream;
    std::vector<double> a, b, cc;
    host_bfield(in.c, a, b);
    CK(hipMemcpyAsync(in.Br, a.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(in.Bz, b.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));
    host_volume(in.c, in.V_host);
    CK(hipMemcpyAsync(in.V, in.V_host.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    if (!twin) {
        std::vector<double> gg, hh;
        host_thomas(in.c, thomas_segments(ctx->max_nr), a, b, cc, gg, hh);
        CK(hipMemcpyAsync(in.th_cp, a.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(in.th_im, b.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(in.th_lo, cc.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(in.th_G, gg.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(in.th_H, hh.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipStreamSynchronize(s));
    }
    if (in.I.spline3) {
        const long long X = (long long)(in.c.nr + 3) * (in.c.nz + 3);
        in.Qx = dalloc<long long>(ctx, X);
        in.cx = dalloc<double>(ctx, X);
        in.cbuf = dalloc<double>(ctx, N);
        in.zeros = dalloc<double>(ctx, N);
        in.s3_L1 = dalloc<double>(ctx, N);
        in.s3_L2 = dalloc<double>(ctx, N);
        in.s3_L3 = dalloc<double>(ctx, N);
        in.s3_Dinv = dalloc<double>(ctx, N);
        if (ctx->mode == PIC_MODE_FP32_BATCHED) {
            in.cxf = dalloc<float>(ctx, X);
            if (!in.cxf) return fail(ctx, PIC_ENOMEM, "device allocation of the cubic-shape arrays failed");
            CK(hipMemsetAsync(in.cxf, 0, sizeof(float) * X, s));
        }
        if (!in.Qx || !in.cx || !in.cbuf || !in.zeros || !in.s3_L1 || !in.s3_L2 || !in.s3_L3 || !in.s3_Dinv)
            return fail(ctx, PIC_ENOMEM, "device allocation of the cubic-shape arrays failed");
        std::vector<double> l1, l2, l3, di;
        host_spline3(in.c, l1, l2, l3, di);
        CK(hipMemcpyAsync(in.s3_L1, l1.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(in.s3_L2, l2.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(in.s3_L3, l3.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemcpyAsync(in.s3_Dinv, di.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
        CK(hipMemsetAsync(in.Qx, 0, sizeof(long long) * X, s));
        CK(hipMemsetAsync(in.cx, 0, sizeof(double) * X, s));
        CK(hipMemsetAsync(in.cbuf, 0, sizeof(double) * N, s));
        CK(hipMemsetAsync(in.zeros, 0, sizeof(double) * N, s));
        CK(hipStreamSynchronize(s));
    }
    if (in.has_ins) {
        std::string m = ins_build(in.c, in.ih);
        if (!m.empty()) return fail(ctx, PIC_EINVAL, "insert: " + m);
        pic_status st = init_insert_storage(ctx, in);
        if (st != PIC_OK) return st;
        if (in.I.spline3) {
            m = ins3_build(in.c, in.ih3);
            if (!m.empty()) return fail(ctx, PIC_EINVAL, "insert: " + m);
            st = init_insert3_storage(ctx, in);
            if (st != PIC_OK) return st;
        }
    }
    host_vacuum_rhs(in.c, in.has_ins ? in.c.V_outer : 0.0, a, b);
    if (in.has_ins)
        for (int t = 0; t < in.ih.m; ++t)
            if (in.ih.typ[t] != 1) b[in.ih.Mnode[t]] = 0.0;  // outer and metal rows hold no load
    CK(hipMemcpyAsync(in.phiB, a.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(in.rhs, b.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    CK(hipMemsetAsync(in.avg_acc, 0, sizeof(double) * N, s));
    CK(hipMemsetAsync(in.Q, 0, sizeof(long long) * N, s));
    CK(hipStreamSynchronize(s));
    return PIC_OK;
}

static void destroy_ctx(pic_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->f32) f32_destroy(ctx);
    for (auto e : ctx->ev) (void)hipEventDestroy(e);
    std::vector<void*> all = ctx->allocs;
    for (void* p : all) pic_dev_free(ctx, p);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

void pic_set_f32(pic_ctx* ctx, F32State* s) { ctx->f32 = s; }
F32State* pic_get_f32(pic_ctx* ctx) { return ctx->f32; }

static pic_status deposit_and_solve(pic_ctx* ctx, int k_only);

extern "C" pic_status pic_init(const pic_run_cfg* run, const pic_instance_cfg* inst, pic_ctx** out) {
    g_init_error.clear();
    if (!out) return fail(nullptr, PIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!run || !inst) return fail(nullptr, PIC_EINVAL, "run or inst is NULL");
    if (run->n_instances < 1 || run->n_instances > 4096) return fail(nullptr, PIC_EINVAL, "n_instances must be in [1, 4096]");
    if (run->mode != PIC_MODE_FP64_PLAIN && run->mode != PIC_MODE_FP32_BATCHED)
        return fail(nullptr, PIC_EINVAL, "unknown mode");
    if (run->capacity_factor < 0.0 || (run->capacity_factor > 0.0 && run->capacity_factor < 1.0))
        return fail(nullptr, PIC_EINVAL, "capacity_factor must be 0 or >= 1");
    if (run->lanes < 0 || run->lanes > 2) return fail(nullptr, PIC_EINVAL, "lanes must be 0, 1 or 2");
    if (run->use_graph < 0 || run->use_graph > 2) return fail(nullptr, PIC_EINVAL, "use_graph must be 0, 1 or 2");
    for (int k = 0; k < run->n_instances; ++k) {
        std::string m = validate(inst[k]);
        if (!m.empty()) return fail(nullptr, PIC_EINVAL, "instance " + std::to_string(k) + ": " + m);
        const double w = inst[k].weight > 0.0 ? inst[k].weight : 1.0;
        const int S = inst[k].fx_shift != 0 ? inst[k].fx_shift : pic_auto_shift(w);
        if (ldexp(w, S) > 2147483648.0)
            return fail(nullptr, PIC_EOVERFLOW, "instance " + std::to_string(k) + ": weight * 2^S exceeds 2^31");
    }
    pic_ctx* ctx = new pic_ctx();
    ctx->run = *run;
    ctx->mode = run->mode;
    hipError_t e = hipSetDevice(run->device);
    if (e == hipSuccess) e = noalloc_setup(run->device);
    if (e != hipSuccess) {
        std::string m = std::string("device set-up: ") + hipGetErrorString(e);
        delete ctx;
        return fail(nullptr, PIC_EDEVICE, m);
    }
    if (run->stream) {
        ctx->stream = (hipStream_t)run->stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return fail(nullptr, PIC_EDEVICE, "hipStreamCreate failed");
        }
        ctx->own_stream = true;
    }
    double cf = run->capacity_factor > 0.0 ? run->capacity_factor : 2.0;
    long long cmin = run->capacity_min > 0 ? run->capacity_min : 4096;
    ctx->in.resize(run->n_instances);
    pic_status st = PIC_OK;
    for (int k = 0; k < run->n_instances && st == PIC_OK; ++k) {
        Inst& in = ctx->in[k];
        in.c = inst[k];
        if (in.c.diag_interval <= 0) in.c.diag_interval = 1;
        in.S = in.c.fx_shift != 0 ? in.c.fx_shift : pic_auto_shift(in.c.weight > 0.0 ? in.c.weight : 1.0);
        in.c.fx_shift = in.S;
        pic_derive(&in.c, in.S, &in.d);
        if (in.c.weight > 0.0 && ldexp(in.c.weight, in.S) > 2147483648.0)
            st = fail(ctx, PIC_EOVERFLOW, "weight * 2^S exceeds 2^31");
        in.cap = std::max<long long>(cmin, (long long)ceil(cf * (double)in.c.n_init));
        in.nodes = (long long)(in.c.nr + 1) * (in.c.nz + 1);
        fill_devinst(in);
        in.has_ins = in.I.has_ins != 0;
        in.idev.inst = k;
        in.idev3.inst = k;
        in.xdev3.inst = k;
        if (in.has_ins) ctx->ins_list.push_back(k);
        ctx->max_nr = std::max(ctx->max_nr, in.c.nr);
        ctx->max_nz = std::max(ctx->max_nz, in.c.nz);
        ctx->max_nodes = std::max(ctx->max_nodes, in.nodes);
    }
    int n = run->n_instances;
    ctx->s3 = n > 0 && ctx->in[0].I.spline3 != 0;
    for (int k = 0; k < n && st == PIC_OK; ++k) {
        if ((ctx->in[k].I.spline3 != 0) != ctx->s3)
            st = fail(ctx, PIC_EINVAL, "every instance of a context needs the same spline_order");
        ctx->max_ext = std::max<long long>(ctx->max_ext, (long long)(ctx->in[k].c.nr + 3) * (ctx->in[k].c.nz + 3));
    }
    if (st == PIC_OK) {
        ctx->dI = dalloc<DevInst>(ctx, n);
        ctx->dF = dalloc<FieldDev>(ctx, n);
        ctx->dFvac = dalloc<FieldDev>(ctx, n);
        ctx->dbscale = dalloc<double>(ctx, n);
        ctx->dcnt = dalloc<long long>(ctx, (long long)n * C_NCOUNT);
        ctx->dtmp = dalloc<long long>(ctx, 64);
        // one twiddle table for every instance: the full circle at a
        // resolution that every transform length 2 nz divides
        long long tw = 1;
        for (const Inst& x : ctx->in) tw = std::lcm(tw, 2ll * x.c.nz);
        if (tw > (1ll << 22)) st = fail(ctx, PIC_EINVAL, "the instances' nz values have too large a common multiple");
        ctx->tw_n = (int)std::min(tw, 1ll << 22);
        ctx->tw = dalloc<double2>(ctx, ctx->tw_n);
        if (!ctx->dI || !ctx->dF || !ctx->dFvac || !ctx->dbscale || !ctx->dcnt || !ctx->dtmp || !ctx->tw)
            st = fail(ctx, PIC_ENOMEM, "device allocation of tables failed");
        const int ni = (int)ctx->ins_list.size();
        if (st == PIC_OK && ni > 0) {
            ctx->dIns = dalloc<InsDev>(ctx, ni);
            ctx->dIins = dalloc<DevInst>(ctx, ni);
            ctx->dF1 = dalloc<FieldDev>(ctx, n);
            ctx->dF1v = dalloc<FieldDev>(ctx, n);
            ctx->dF2 = dalloc<FieldDev>(ctx, ni);
            ctx->dF2v = dalloc<FieldDev>(ctx, ni);
            ctx->dGoff = dalloc<int>(ctx, ni + 1);
            ctx->dGmem = dalloc<int>(ctx, ni);
            if (!ctx->dIns || !ctx->dIins || !ctx->dF1 || !ctx->dF1v || !ctx->dF2 || !ctx->dF2v || !ctx->dGoff ||
                !ctx->dGmem)
                st = fail(ctx, PIC_ENOMEM, "device allocation of insert tables failed");
        }
        if (st == PIC_OK && ctx->s3) {
            ctx->dF3 = dalloc<FieldDev>(ctx, n);
            if (!ctx->dF3) st = fail(ctx, PIC_ENOMEM, "device allocation of the cubic table failed");
        }
        if (st == PIC_OK && ctx->s3 && ni > 0) {
            ctx->dIns3 = dalloc<InsDev>(ctx, ni);
            ctx->dX3 = dalloc<Ins3Dev>(ctx, ni);
            ctx->dF3a = dalloc<FieldDev>(ctx, n);
            ctx->dF3b = dalloc<FieldDev>(ctx, ni);
            ctx->dGoff3 = dalloc<int>(ctx, ni + 1);
            ctx->dGmem3 = dalloc<int>(ctx, ni);
            if (!ctx->dIns3 || !ctx->dX3 || !ctx->dF3a || !ctx->dF3b || !ctx->dGoff3 || !ctx->dGmem3)
                st = fail(ctx, PIC_ENOMEM, "device allocation of the cubic insert tables failed");
        }
    }
    if (st == PIC_OK) {
        std::vector<double2> tw(ctx->tw_n);  // the full circle
        for (int k = 0; k < ctx->tw_n; ++k) {
            double a = 2.0 * kPi * (double)k / (double)ctx->tw_n;
            tw[k] = make_double2(cos(a), -sin(a));
        }
        e = hipMemcpy(ctx->tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) st = fail(ctx, PIC_EDEVICE, "twiddle upload failed");
        e = set_field_kernel_attrs(ctx->max_nz);
        if (e != hipSuccess && st == PIC_OK) st = fail(ctx, PIC_EDEVICE, "LDS attribute failed");
    }
    for (int k = 0; k < n && st == PIC_OK; ++k) st = init_instance_storage(ctx, ctx->in[k]);
    for (int k : ctx->ins_list) {
        ctx->max_m = std::max(ctx->max_m, ctx->in[k].ih.m);
        ctx->max_m3 = std::max(ctx->max_m3, ctx->in[k].ih3.m);
        ctx->max_nx3 = std::max(ctx->max_nx3, ctx->in[k].ih3.nx);
    }
    if (st == PIC_OK && ctx->mode == PIC_MODE_FP32_BATCHED) st = f32_init(ctx);
    if (st == PIC_OK) {
        std::vector<long long> cnt((size_t)n * C_NCOUNT, 0);
        for (int k = 0; k < n; ++k) cnt[(size_t)k * C_NCOUNT + C_SLOTS] = ctx->in[k].c.n_init;
        e = hipMemcpy(ctx->dcnt, cnt.data(), sizeof(long long) * cnt.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) st = fail(ctx, PIC_EDEVICE, "counter upload failed");
        for (int k = 0; k < n; ++k) ctx->in[k].cnt = ctx->dcnt + (long long)k * C_NCOUNT;
    }
    if (st == PIC_OK) st = upload_tables(ctx);
    for (size_t t = 0; t < ctx->ins_list.size() && st == PIC_OK; ++t) st = setup_insert(ctx, ctx->in[ctx->ins_list[t]]);
    // vacuum potential
    if (st == PIC_OK) st = solve_tables(ctx, true, false, true, ctx->stream);
    if (st == PIC_OK && ctx->s3) {
        // cubic shapes: the nodal E arrays hold the vacuum field for good
        e = launch_efield_tab(ctx->dI, ctx->dFvac, 0, n, ctx->max_nodes, true, ctx->stream);
        if (e != hipSuccess) st = fail(ctx, PIC_EDEVICE, "vacuum field");
    }
    if (st == PIC_OK) {
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = fail(ctx, PIC_EDEVICE, std::string("vacuum solve: ") + hipGetErrorString(e));
    }
    // initial load
    for (int k = 0; k < n && st == PIC_OK; ++k) {
        Inst& in = ctx->in[k];
        if (ctx->mode == PIC_MODE_FP64_PLAIN) {
            e = launch_load64(in.I, in.c, in.p64[0], in.c.n_init, ctx->stream);
            if (e != hipSuccess) st = fail(ctx, PIC_EDEVICE, "load kernel failed");
        } else {
            st = f32_load(ctx, k);
        }
    }
    if (st == PIC_OK) st = deposit_and_solve(ctx, -1);
    if (st == PIC_OK && ctx->mode == PIC_MODE_FP32_BATCHED) st = f32_sort_now(ctx);
    if (st == PIC_OK) {
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = fail(ctx, PIC_EDEVICE, std::string("init: ") + hipGetErrorString(e));
    }
    if (st != PIC_OK) {
        g_init_error = ctx->err;
        destroy_ctx(ctx);
        return st;
    }
    *out = ctx;
    return PIC_OK;
}

extern "C" pic_status pic_destroy(pic_ctx* ctx) {
    if (!ctx) return PIC_EINVAL;
    destroy_ctx(ctx);
    return PIC_OK;
}

extern "C" const char* pic_last_error(const pic_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

// ---------------------------------------------------------------------------
// deposit + field (used at init and after set_particles); k_only < 0: all
// ---------------------------------------------------------------------------

static pic_status deposit_and_solve(pic_ctx* ctx, int k_only) {
    hipStream_t s = ctx->stream;
    for (int k = 0; k < (int)ctx->in.size(); ++k) {
        if (k_only >= 0 && k != k_only) continue;
        Inst& in = ctx->in[k];
        CK(launch_zero_i64(in.Q, in.nodes, s));
        if (in.Qw) CK(launch_zero_i64(in.Qw, band_cells(in), s));
        if (in.Qx) CK(launch_zero_i64(in.Qx, (long long)(in.c.nr + 3) * (in.c.nz + 3), s));
        if (ctx->mode == PIC_MODE_FP64_PLAIN) {
            CK(launch_deposit64(in.I, in.p64[in.cur], in.Q, in.Qw, in.Qx, in.cnt, in.cap, s));
        } else {
            pic_status st = f32_deposit_only(ctx, k);
            if (st != PIC_OK) return st;
        }
    }
    return pic_solve_all(ctx);
}

// ---------------------------------------------------------------------------
// FP64 plain step
// ---------------------------------------------------------------------------

static pic_status check_counts(pic_ctx* ctx, std::vector<long long>& cnt) {
    cnt.resize(ctx->in.size() * C_NCOUNT);
    CK(hipMemcpyAsync(cnt.data(), ctx->dcnt, sizeof(long long) * cnt.size(), hipMemcpyDeviceToHost,
                      ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    for (size_t k = 0; k < ctx->in.size(); ++k) {
        if (cnt[k * C_NCOUNT + C_DROPPED] > 0)
            return fail(ctx, PIC_ECAPACITY, "instance " + std::to_string(k) + ": new electrons dropped (storage full)");
        if (cnt[k * C_NCOUNT + C_OVERFLOW] > 0)
            return fail(ctx, PIC_EOVERFLOW, "instance " + std::to_string(k) + ": fixed-point overflow");
        if (cnt[k * C_NCOUNT + C_NONFIN] > 0)
            return fail(ctx, PIC_ENONFINITE, "instance " + std::to_string(k) + ": " +
                                                 std::to_string(cnt[k * C_NCOUNT + C_NONFIN]) +
                                                 " particles with a non-finite position removed");
    }
    if (ctx->mode == PIC_MODE_FP32_BATCHED) return f32_check(ctx);
    return PIC_OK;
}

// New FP64 stores of `cap` slots for instance k holding its used slots.
static pic_status grow64(pic_ctx* ctx, int k, long long cap) {
    Inst& in = ctx->in[k];
    hipStream_t s = ctx->stream;
    long long slots = 0;
    CK(hipStreamSynchronize(s));
    CK(hipMemcpy(&slots, in.cnt + C_SLOTS, sizeof(long long), hipMemcpyDeviceToHost));
    if (cap <= in.cap) return PIC_OK;
    P64 np[2];
    bool ok = true;
    for (int b = 0; b < 2; ++b) {
        P64& p = np[b];
        p.r = dalloc<double>(ctx, cap);
        p.z = dalloc<double>(ctx, cap);
        p.vr = dalloc<double>(ctx, cap);
        p.vt = dalloc<double>(ctx, cap);
        p.vz = dalloc<double>(ctx, cap);
        p.w = dalloc<double>(ctx, cap);
        p.key = dalloc<unsigned long long>(ctx, cap);
        ok = ok && p.r && p.z && p.vr && p.vt && p.vz && p.w && p.key;
    }
    if (!ok) {
        for (int b = 0; b < 2; ++b) {
            void* a[] = {np[b].r, np[b].z, np[b].vr, np[b].vt, np[b].vz, np[b].w, np[b].key};
            for (void* q : a) pic_dev_free(ctx, q);
        }
        return fail(ctx, PIC_ENOMEM, "growing FP64 particle stores");
    }
    const P64& o = in.p64[in.cur];
    if (slots > 0) {
        double* src[6] = {o.r, o.z, o.vr, o.vt, o.vz, o.w};
        double* dst[6] = {np[0].r, np[0].z, np[0].vr, np[0].vt, np[0].vz, np[0].w};
        for (int a = 0; a < 6; ++a)
            CK(hipMemcpyAsync(dst[a], src[a], sizeof(double) * slots, hipMemcpyDeviceToDevice, s));
        CK(hipMemcpyAsync(np[0].key, o.key, sizeof(unsigned long long) * slots, hipMemcpyDeviceToDevice, s));
        CK(hipStreamSynchronize(s));
    }
    for (int b = 0; b < 2; ++b) {
        void* a[] = {in.p64[b].r, in.p64[b].z, in.p64[b].vr, in.p64[b].vt, in.p64[b].vz, in.p64[b].w,
                     in.p64[b].key};
        for (void* q : a) pic_dev_free(ctx, q);
        in.p64[b] = np[b];
    }
    in.cur = 0;
    in.cap = cap;
    in.I.p_cap = cap;
    ctx->grow_events += 1;
    return pic_upload_inst(ctx);
}

static pic_status compact64(pic_ctx* ctx, int k) {
    Inst& in = ctx->in[k];
    hipStream_t s = ctx->stream;
    CK(hipMemsetAsync(ctx->dtmp, 0, sizeof(long long), s));
    CK(launch_compact64(in.I, in.p64[in.cur], in.p64[1 - in.cur], in.cnt, ctx->dtmp, in.cap, s));
    long long live = 0;
    CK(hipMemcpyAsync(&live, ctx->dtmp, sizeof(long long), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    in.cur = 1 - in.cur;
    long long upd[3] = {live, 0, 0};  // slots, spawn, dead
    CK(hipMemcpyAsync(in.cnt + C_SLOTS, upd, sizeof(upd), hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));
    return PIC_OK;
}

static pic_status step64(pic_ctx* ctx, int n_steps) {
    hipStream_t s = ctx->stream;
    const int check_every = 64;
    std::vector<long long> cnt;
    for (int done = 0; done < n_steps;) {
        pic_status st = check_counts(ctx, cnt);
        if (st != PIC_OK) return st;
        for (size_t k = 0; k < ctx->in.size(); ++k) {
            long long slots = cnt[k * C_NCOUNT + C_SLOTS], dead = cnt[k * C_NCOUNT + C_DEAD];
            const long long cap = ctx->in[k].cap;
            if (slots > (cap * 3) / 4 && dead > 0) {
                st = compact64(ctx, (int)k);
                if (st != PIC_OK) return st;
                slots -= dead;
            }
            // still 3/4 full once the dead are gone (counting what the seed
            // source adds before the next check): twice that
            const long long need = slots + (long long)ceil(ctx->in[k].c.src_rate) * check_every;
            if (need > (cap * 3) / 4) {
                st = grow64(ctx, (int)k, std::max<long long>(2 * need, cap + cap / 2));
                if (st != PIC_OK) return st;
            }
        }
        int batch = std::min(check_every, n_steps - done);
        for (int it = 0; it < batch; ++it) {
            for (size_t k = 0; k < ctx->in.size(); ++k) {
                Inst& in = ctx->in[k];
                P64 p = in.p64[in.cur];
                CK(launch_zero_i64(in.Q, in.nodes, s));
                if (in.Qw) CK(launch_zero_i64(in.Qw, band_cells(in), s));
                if (in.Qx) CK(launch_zero_i64(in.Qx, (long long)(in.c.nr + 3) * (in.c.nz + 3), s));
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (ctx->timing) {
                    e0 = pic_timing_begin(ctx, &e1);
                    CK(hipEventRecord(e0, s));
                }
                CK(launch_push64(in.I, p, in.Er, in.Ez, in.Br, in.Bz, in.cx, in.cnt, in.cap, s));
                if (ctx->timing) CK(hipEventRecord(e1, s));
                CK(launch_mcc64(in.I, p, in.cnt, in.cap, s));
                if (in.c.src_rate > 0.0) CK(launch_source64(in.I, p, in.cnt, s));
                CK(launch_deposit64(in.I, p, in.Q, in.Qw, in.Qx, in.cnt, in.cap, s));
            }
            st = pic_field_stage(ctx, s);
            if (st != PIC_OK) return st;
            ctx->host_step += 1;
        }
        done += batch;
        if (ctx->timing && ctx->ev_used > 4096) {
            st = timing_collect(ctx);
            if (st != PIC_OK) return st;
        }
    }
    return PIC_OK;
}

extern "C" pic_status pic_step(pic_ctx* ctx, int n_steps) {
    if (!ctx) return PIC_EINVAL;
    if (n_steps < 0) return fail(ctx, PIC_EINVAL, "n_steps < 0");
    if (n_steps == 0) return PIC_OK;
    if (ctx->mode == PIC_MODE_FP64_PLAIN) return step64(ctx, n_steps);
    return f32_step(ctx, n_steps);
}

extern "C" pic_status pic_sync(pic_ctx* ctx) {
    if (!ctx) return PIC_EINVAL;
    std::vector<long long> cnt;
    return check_counts(ctx, cnt);
}

// ---------------------------------------------------------------------------
// hooks
// ---------------------------------------------------------------------------

static pic_status check_inst(pic_ctx* ctx, int k) {
    if (!ctx) return PIC_EINVAL;
    if (k < 0 || k >= (int)ctx->in.size()) return fail(ctx, PIC_EINVAL, "instance index out of range");
    return PIC_OK;
}

pic_status pic_check_instance(pic_ctx* ctx, int k) { return check_inst(ctx, k); }
pic_status pic_fail(pic_ctx* ctx, pic_status st, const std::string& msg) { return fail(ctx, st, msg); }

extern "C" pic_status pic_set_particles(pic_ctx* ctx, int k, long long n, const double* r,
                                        const double* z, const double* vr, const double* vt,
                                        const double* vz, const double* w,
                                        const unsigned long long* key) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    Inst& in = ctx->in[k];
    if (n < 0 || (n > 0 && (!r || !z || !vr || !vt || !vz || !w || !key)))
        return fail(ctx, PIC_EINVAL, "bad particle arrays");
    if (n > in.cap / 2 && ctx->mode == PIC_MODE_FP32_BATCHED)
        return fail(ctx, PIC_ECAPACITY, "more particles than half the slots");
    if (n > in.cap) return fail(ctx, PIC_ECAPACITY, "more particles than slots");
    for (long long q = 0; q < n; ++q) {
        if (!(r[q] > in.c.a && r[q] < in.c.b && z[q] > 0.0 && z[q] < in.c.L))
            return fail(ctx, PIC_EINVAL, "particle " + std::to_string(q) + " outside a<r<b, 0<z<L");
        if (!(std::isfinite(vr[q]) && std::isfinite(vt[q]) && std::isfinite(vz[q])))
            return fail(ctx, PIC_EINVAL, "particle " + std::to_string(q) + ": non-finite velocity");
        if (!(w[q] > 0.0)) return fail(ctx, PIC_EINVAL, "weights must be > 0");
        if (w[q] * in.d.two_S > 2147483648.0) return fail(ctx, PIC_EOVERFLOW, "weight * 2^S exceeds 2^31");
    }
    hipStream_t s = ctx->stream;
    CK(hipStreamSynchronize(s));
    if (ctx->mode == PIC_MODE_FP64_PLAIN) {
        P64 p = in.p64[in.cur];
        size_t b = sizeof(double) * (size_t)n;
        if (n > 0) {
            CK(hipMemcpy(p.r, r, b, hipMemcpyHostToDevice));
            CK(hipMemcpy(p.z, z, b, hipMemcpyHostToDevice));
            CK(hipMemcpy(p.vr, vr, b, hipMemcpyHostToDevice));
            CK(hipMemcpy(p.vt, vt, b, hipMemcpyHostToDevice));
            CK(hipMemcpy(p.vz, vz, b, hipMemcpyHostToDevice));
            CK(hipMemcpy(p.w, w, b, hipMemcpyHostToDevice));
            CK(hipMemcpy(p.key, key, sizeof(unsigned long long) * n, hipMemcpyHostToDevice));
        }
    } else {
        st = f32_set_particles(ctx, k, n, r, z, vr, vt, vz, w, key);
        if (st != PIC_OK) return st;
    }
    long long upd[3] = {n, 0, 0};
    CK(hipMemcpy(in.cnt + C_SLOTS, upd, sizeof(upd), hipMemcpyHostToDevice));
    long long zero = 0;
    CK(hipMemcpy(in.cnt + C_LIVE_SORTED, &zero, sizeof(zero), hipMemcpyHostToDevice));
    st = deposit_and_solve(ctx, k);
    if (st != PIC_OK) return st;
    if (ctx->mode == PIC_MODE_FP32_BATCHED) {
        st = f32_sort_now(ctx);
        if (st != PIC_OK) return st;
    }
    CK(hipStreamSynchronize(s));
    return PIC_OK;
}

extern "C" pic_status pic_get_particles(pic_ctx* ctx, int k, double* r, double* z, double* vr,
                                        double* vt, double* vz, double* w, unsigned long long* key,
                                        long long cap, long long* n_out) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    std::vector<long long> cnt;
    st = check_counts(ctx, cnt);
    if (st != PIC_OK && st != PIC_ECAPACITY && st != PIC_ENONFINITE) return st;
    Inst& in = ctx->in[k];
    if (ctx->mode != PIC_MODE_FP64_PLAIN) {
        const pic_status g = f32_get_particles(ctx, k, r, z, vr, vt, vz, w, key, cap, n_out);
        return g != PIC_OK ? g : st;
    }
    long long slots = cnt[(size_t)k * C_NCOUNT + C_SLOTS];
    P64 p = in.p64[in.cur];
    std::vector<double> hr(slots), hz(slots), hvr(slots), hvt(slots), hvz(slots), hw(slots);
    std::vector<unsigned long long> hk(slots);
    size_t b = sizeof(double) * (size_t)slots;
    if (slots > 0) {
        CK(hipMemcpy(hr.data(), p.r, b, hipMemcpyDeviceToHost));
        CK(hipMemcpy(hz.data(), p.z, b, hipMemcpyDeviceToHost));
        CK(hipMemcpy(hvr.data(), p.vr, b, hipMemcpyDeviceToHost));
        CK(hipMemcpy(hvt.data(), p.vt, b, hipMemcpyDeviceToHost));
        CK(hipMemcpy(hvz.data(), p.vz, b, hipMemcpyDeviceToHost));
        CK(hipMemcpy(hw.data(), p.w, b, hipMemcpyDeviceToHost));
        CK(hipMemcpy(hk.data(), p.key, sizeof(unsigned long long) * slots, hipMemcpyDeviceToHost));
    }
    long long m = 0;
    for (long long q = 0; q < slots; ++q) {
        if (hr[q] < 0.0) continue;
        if (m < cap) {
            if (r) r[m] = hr[q];
            if (z) z[m] = hz[q];
            if (vr) vr[m] = hvr[q];
            if (vt) vt[m] = hvt[q];
            if (vz) vz[m] = hvz[q];
            if (w) w[m] = hw[q];
            if (key) key[m] = hk[q];
        }
        ++m;
    }
    if (n_out) *n_out = m;
    if (m > cap) return fail(ctx, PIC_EINVAL, "cap smaller than the live count");
    return st;
}

extern "C" pic_status pic_set_fields(pic_ctx* ctx, int k, const double* Er, const double* Ez,
                                     const double* Br, const double* Bz, int frozen) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    Inst& in = ctx->in[k];
    size_t N = (size_t)in.nodes, b = sizeof(double) * N;
    CK(hipStreamSynchronize(ctx->stream));
    if (Br) CK(hipMemcpy(in.Br, Br, b, hipMemcpyHostToDevice));
    if (Bz) CK(hipMemcpy(in.Bz, Bz, b, hipMemcpyHostToDevice));
    if (ctx->mode == PIC_MODE_FP64_PLAIN) {
        if (Er) CK(hipMemcpy(in.Er, Er, b, hipMemcpyHostToDevice));
        if (Ez) CK(hipMemcpy(in.Ez, Ez, b, hipMemcpyHostToDevice));
    } else {
        std::vector<float4> eb(N);
        CK(hipMemcpy(eb.data(), in.EB, sizeof(float4) * N, hipMemcpyDeviceToHost));
        for (size_t n = 0; n < N; ++n) {
            if (Er) eb[n].x = (float)Er[n];
            if (Ez) eb[n].y = (float)Ez[n];
            if (Br) eb[n].z = (float)Br[n];
            if (Bz) eb[n].w = (float)Bz[n];
        }
        CK(hipMemcpy(in.EB, eb.data(), sizeof(float4) * N, hipMemcpyHostToDevice));
    }
    in.frozen = frozen != 0;
    st = upload_tables(ctx);
    if (st != PIC_OK || !ctx->s3) return st;
    // cubic shapes: a frozen field is the given nodal one alone; back to the
    // self-consistent field, the nodal arrays hold the vacuum field again
    CK(hipMemsetAsync(in.cx, 0, sizeof(double) * (size_t)(in.c.nr + 3) * (in.c.nz + 3), ctx->stream));
    if (in.cxf) CK(hipMemsetAsync(in.cxf, 0, sizeof(float) * (size_t)(in.c.nr + 3) * (in.c.nz + 3), ctx->stream));
    if (!in.frozen) {
        CK(launch_efield_tab(ctx->dI, ctx->dFvac, k, 1, in.nodes, false, ctx->stream));
        st = pic_solve_all(ctx);
    }
    CK(hipStreamSynchronize(ctx->stream));
    return st;
}

extern "C" pic_status pic_get_fields(pic_ctx* ctx, int k, double* Er, double* Ez, double* Br,
                                     double* Bz) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    Inst& in = ctx->in[k];
    size_t N = (size_t)in.nodes, b = sizeof(double) * N;
    CK(hipStreamSynchronize(ctx->stream));
    if (ctx->mode == PIC_MODE_FP64_PLAIN) {
        if (Er) CK(hipMemcpy(Er, in.Er, b, hipMemcpyDeviceToHost));
        if (Ez) CK(hipMemcpy(Ez, in.Ez, b, hipMemcpyDeviceToHost));
        if (Br) CK(hipMemcpy(Br, in.Br, b, hipMemcpyDeviceToHost));
        if (Bz) CK(hipMemcpy(Bz, in.Bz, b, hipMemcpyDeviceToHost));
    } else {
        std::vector<float4> eb(N);
        CK(hipMemcpy(eb.data(), in.EB, sizeof(float4) * N, hipMemcpyDeviceToHost));
        for (size_t n = 0; n < N; ++n) {
            if (Er) Er[n] = eb[n].x;
            if (Ez) Ez[n] = eb[n].y;
            if (Br) Br[n] = eb[n].z;
            if (Bz) Bz[n] = eb[n].w;
        }
    }
    return PIC_OK;
}

extern "C" pic_status pic_get_charge(pic_ctx* ctx, int k, long long* Q) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (!Q) return fail(ctx, PIC_EINVAL, "Q is NULL");
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(Q, ctx->in[k].Q, sizeof(long long) * ctx->in[k].nodes, hipMemcpyDeviceToHost));
    return PIC_OK;
}

extern "C" pic_status pic_get_spline3(pic_ctx* ctx, int k, long long* Qx, double* cx) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    Inst& in = ctx->in[k];
    if (!in.Qx) return fail(ctx, PIC_EINVAL, "the instance does not use cubic shapes");
    const size_t X = (size_t)(in.c.nr + 3) * (in.c.nz + 3);
    CK(hipStreamSynchronize(ctx->stream));
    if (Qx) CK(hipMemcpy(Qx, in.Qx, sizeof(long long) * X, hipMemcpyDeviceToHost));
    if (cx) CK(hipMemcpy(cx, in.cx, sizeof(double) * X, hipMemcpyDeviceToHost));
    return PIC_OK;
}

extern "C" pic_status pic_get_band_charge(pic_ctx* ctx, int k, long long* Qw) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (!Qw) return fail(ctx, PIC_EINVAL, "Qw is NULL");
    CK(hipStreamSynchronize(ctx->stream));
    const Inst& in = ctx->in[k];
    if (!in.Qw) {
        memset(Qw, 0, sizeof(long long) * band_cells(in));
        return PIC_OK;
    }
    CK(hipMemcpy(Qw, in.Qw, sizeof(long long) * band_cells(in), hipMemcpyDeviceToHost));
    return PIC_OK;
}

// Null-collision bound of a cross-section table (Sec. II.A null-collision
// method): the largest sigma_total(E) v(E) over 0 <= E <= E_cap.  Between
// consecutive knots (table energies, the ionisation threshold, 0 and E_cap)
// the total is linear in E, s(E) = s0 + m (E - e0), so s(E) sqrt(E) can
// only peak at the knots or where m E + s(E) / 2 = 0.  The threshold is a
// knot on both sides: ionisation is off just below it and on from it.
static double table_sigv_max(const pic_instance_cfg& c, int n, const double* E, const double* el,
                             const double* iz) {
    const double v2_per_eV = (2.0 * kE) / kMe;
    const double top = c.E_cap_eV, thr = c.iz_I_eV;
    std::vector<double> knot{0.0, top};
    for (int t = 0; t < n; ++t)
        if (E[t] > 0.0 && E[t] < top) knot.push_back(E[t]);
    if (thr > 0.0 && thr < top) knot.push_back(thr);
    std::sort(knot.begin(), knot.end());
    knot.erase(std::unique(knot.begin(), knot.end()), knot.end());
    // the total cross section at x, approached from above (up) or below
    auto sigma = [&](double x, bool up) {
        const bool ion = up ? x >= thr : x > thr;
        return xs_interp(n, E, el, x) + (ion ? xs_interp(n, E, iz, x) : 0.0);
    };
    auto sv = [&](double s, double x) { return s * sqrt(x * v2_per_eV); };
    double peak = 0.0;
    for (size_t t = 1; t < knot.size(); ++t) {
        const double e0 = knot[t - 1], e1 = knot[t];
        const double s0 = sigma(e0, true), s1 = sigma(e1, false);
        peak = std::max({peak, sv(s0, e0), sv(s1, e1)});
        const double m = (s1 - s0) / (e1 - e0);
        if (m < 0.0) {
            const double x = (m * e0 - s0) / (3.0 * m);
            if (x > e0 && x < e1) peak = std::max(peak, sv(s0 + m * (x - e0), x));
        }
    }
    return peak;
}

// The bound in use: the maximum widened by 2^-20 and rounded up to 12
// significant bits, so it does not depend on the maximum's own rounding.
static double table_bound(double sigv_max) {
    int ex;
    const double frac = frexp(sigv_max * (1.0 + 0x1p-20), &ex);
    return ldexp(ceil(frac * 4096.0), ex - 12);
}

extern "C" pic_status pic_set_cross_sections(pic_ctx* ctx, int k, int n, const double* E_eV,
                                             const double* sigma_el, const double* sigma_iz) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (n != 0 && (n < 2 || n > 4096)) return fail(ctx, PIC_EINVAL, "need 2 <= n <= 4096 table points (or 0)");
    if (n > 0 && (!E_eV || !sigma_el || !sigma_iz)) return fail(ctx, PIC_EINVAL, "table arrays are NULL");
    for (int t = 0; t < n; ++t) {
        if (!(E_eV[t] >= 0.0) || !(sigma_el[t] >= 0.0) || !(sigma_iz[t] >= 0.0))
            return fail(ctx, PIC_EINVAL, "energies and cross sections must be >= 0");
        if (t > 0 && !(E_eV[t] > E_eV[t - 1])) return fail(ctx, PIC_EINVAL, "energies must increase strictly");
    }
    CK(hipStreamSynchronize(ctx->stream));
    Inst& in = ctx->in[k];
    DevInst& I = in.I;
    const void* old[6] = {I.xs_E, I.xs_el, I.xs_iz, I.xs_Ef, I.xs_elf, I.xs_izf};
    for (const void* p : old)
        if (p) pic_dev_free(ctx, const_cast<void*>(p));
    I.xs_n = 0;
    I.xs_E = I.xs_el = I.xs_iz = nullptr;
    I.xs_Ef = I.xs_elf = I.xs_izf = nullptr;
    pic_derived_t d;
    pic_derive(&in.c, in.S, &d);
    if (n > 0) {
        bool ok = true;
        std::vector<double> vE(E_eV, E_eV + n), vel(sigma_el, sigma_el + n), viz(sigma_iz, sigma_iz + n);
        std::vector<float> fE(n), fel(n), fiz(n);
        for (int t = 0; t < n; ++t) {
            fE[t] = (float)E_eV[t];
            fel[t] = (float)sigma_el[t];
            fiz[t] = (float)sigma_iz[t];
        }
        I.xs_E = upload_vec(ctx, vE, ctx->stream, ok);
        I.xs_el = upload_vec(ctx, vel, ctx->stream, ok);
        I.xs_iz = upload_vec(ctx, viz, ctx->stream, ok);
        I.xs_Ef = upload_vec(ctx, fE, ctx->stream, ok);
        I.xs_elf = upload_vec(ctx, fel, ctx->stream, ok);
        I.xs_izf = upload_vec(ctx, fiz, ctx->stream, ok);
        CK(hipStreamSynchronize(ctx->stream));
        if (!ok) return fail(ctx, PIC_ENOMEM, "device allocation of the cross-section table failed");
        I.xs_n = n;
        d.nu_prime = d.n_n * table_bound(table_sigv_max(in.c, n, E_eV, sigma_el, sigma_iz));
        d.P_null = -expm1(-(d.nu_prime * in.c.dt));
    }
    in.d.nu_prime = d.nu_prime;
    in.d.P_null = d.P_null;
    I.nu_prime = d.nu_prime;
    I.P_null = d.P_null;
    I.null_k = null_threshold(d.P_null);
    I.nu_prime_f = (float)d.nu_prime;
    st = pic_upload_inst(ctx);
    if (st != PIC_OK) return st;
    if (ctx->mode == PIC_MODE_FP32_BATCHED) return f32_rates_changed(ctx);
    return PIC_OK;
}

extern "C" pic_status pic_set_anisotropy(pic_ctx* ctx, int k, int n, const double* E_eV, const double* xi) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (n != 0 && (n < 2 || n > 4096)) return fail(ctx, PIC_EINVAL, "need 2 <= n <= 4096 table points (or 0)");
    if (n > 0 && (!E_eV || !xi)) return fail(ctx, PIC_EINVAL, "table arrays are NULL");
    for (int t = 0; t < n; ++t) {
        if (!(E_eV[t] >= 0.0)) return fail(ctx, PIC_EINVAL, "energies must be >= 0");
        if (!(xi[t] > -1.0 && xi[t] < 1.0)) return fail(ctx, PIC_EINVAL, "xi must be in (-1, 1)");
        if (t > 0 && !(E_eV[t] > E_eV[t - 1])) return fail(ctx, PIC_EINVAL, "energies must increase strictly");
    }
    CK(hipStreamSynchronize(ctx->stream));
    DevInst& I = ctx->in[k].I;
    const void* old[4] = {I.xi_E, I.xi_v, I.xi_Ef, I.xi_vf};
    for (const void* p : old)
        if (p) pic_dev_free(ctx, const_cast<void*>(p));
    I.xi_n = 0;
    I.xi_E = I.xi_v = nullptr;
    I.xi_Ef = I.xi_vf = nullptr;
    if (n > 0) {
        bool ok = true;
        std::vector<double> vE(E_eV, E_eV + n), vx(xi, xi + n);
        std::vector<float> fE(n), fx(n);
        for (int t = 0; t < n; ++t) {
            fE[t] = (float)E_eV[t];
            fx[t] = (float)xi[t];
        }
        I.xi_E = upload_vec(ctx, vE, ctx->stream, ok);
        I.xi_v = upload_vec(ctx, vx, ctx->stream, ok);
        I.xi_Ef = upload_vec(ctx, fE, ctx->stream, ok);
        I.xi_vf = upload_vec(ctx, fx, ctx->stream, ok);
        CK(hipStreamSynchronize(ctx->stream));
        if (!ok) return fail(ctx, PIC_ENOMEM, "device allocation of the anisotropy table failed");
        I.xi_n = n;
    }
    return pic_upload_inst(ctx);
}

extern "C" pic_status pic_insert_layout(const pic_instance_cfg* inst, int counts[4], int* m, long long* entries) {
    if (!inst) return fail(nullptr, PIC_EINVAL, "inst is NULL");
    std::string msg = validate(*inst);
    if (!msg.empty()) return fail(nullptr, PIC_EINVAL, msg);
    if (!(inst->ins_er > 0.0 && inst->ins_ez > 0.0)) return fail(nullptr, PIC_EINVAL, "no insert");
    if (inst->spline_order == 3) {
        Ins3Host h3;
        msg = ins3_build(*inst, h3);
        if (!msg.empty()) return fail(nullptr, PIC_EINVAL, "insert: " + msg);
        if (counts)
            for (int t = 0; t < 4; ++t) counts[t] = h3.counts[t];
        if (m) *m = h3.m;
        if (entries) *entries = (long long)h3.Dv.size();
        return PIC_OK;
    }
    InsHost h;
    msg = ins_build(*inst, h);
    if (!msg.empty()) return fail(nullptr, PIC_EINVAL, "insert: " + msg);
    if (counts)
        for (int t = 0; t < 4; ++t) counts[t] = h.counts[t];
    if (m) *m = h.m;
    if (entries) *entries = (long long)h.Dv.size();
    return PIC_OK;
}

extern "C" pic_status pic_get_phi(pic_ctx* ctx, int k, double* phi) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (!phi) return fail(ctx, PIC_EINVAL, "phi is NULL");
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(phi, ctx->in[k].phi, sizeof(double) * ctx->in[k].nodes, hipMemcpyDeviceToHost));
    return PIC_OK;
}

extern "C" pic_status pic_set_step(pic_ctx* ctx, long long step) {
    if (!ctx || step < 0) return PIC_EINVAL;
    CK(hipStreamSynchronize(ctx->stream));
    for (auto& in : ctx->in) CK(hipMemcpy(in.cnt + C_STEP, &step, sizeof(long long), hipMemcpyHostToDevice));
    ctx->host_step = step;
    return PIC_OK;
}

extern "C" pic_status pic_diag(pic_ctx* ctx, int k, pic_diag_t* out, double* density,
                               double* time_avg_density) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (!out) return fail(ctx, PIC_EINVAL, "out is NULL");
    std::vector<long long> all;
    pic_status cs = check_counts(ctx, all);
    if (cs != PIC_OK && cs != PIC_ECAPACITY && cs != PIC_EOVERFLOW && cs != PIC_ENONFINITE) return cs;
    Inst& in = ctx->in[k];
    const long long* c = all.data() + (size_t)k * C_NCOUNT;
    memset(out, 0, sizeof(*out));
    out->step = c[C_STEP];
    out->n_elastic = c[C_ELASTIC];
    out->n_ioniz = c[C_IONIZ];
    out->n_null_cand = c[C_CAND];
    out->n_cap_overflow = c[C_CAPOVER];
    out->n_spawn_dropped = c[C_DROPPED];
    for (int w = 0; w < 4; ++w) {
        out->n_absorbed[w] = c[C_ABS_N + w];
        out->absorbed_W[w] = c[C_ABS_W + w];
        long long bits = c[C_IWALL + w];
        memcpy(&out->I_wall[w], &bits, 8);
    }
    memcpy(&out->peak_density, &c[C_PEAK], 8);
    memcpy(&out->peak_I_outer, &c[C_PEAKI_OUT], 8);
    memcpy(&out->peak_I_inner, &c[C_PEAKI_IN], 8);
    out->n_samples = c[C_NSAMP];
    out->particle_steps = c[C_PSTEPS];
    out->n_far_deposit = c[C_FARDEP];
    out->n_source = c[C_SOURCE];
    out->n_nonfinite = c[C_NONFIN];
    out->S = in.S;
    if (ctx->mode == PIC_MODE_FP64_PLAIN) out->n_live = c[C_SLOTS] - c[C_DEAD];
    else out->n_live = f32_live_count(ctx, k, c);
    size_t N = (size_t)in.nodes;
    std::vector<long long> Q(N);
    std::vector<double> acc(N);
    CK(hipMemcpy(Q.data(), in.Q, sizeof(long long) * N, hipMemcpyDeviceToHost));
    CK(hipMemcpy(acc.data(), in.avg_acc, sizeof(double) * N, hipMemcpyDeviceToHost));
    long long tq = 0;
    double pk = 0.0;
    for (size_t n = 0; n < N; ++n) {
        tq += Q[n];
        if (density) density[n] = ((double)Q[n] * in.d.inv_two_S) / in.V_host[n];
        double avg = out->n_samples > 0
                         ? ((acc[n] * in.d.inv_two_S) / (double)out->n_samples) / in.V_host[n]
                         : 0.0;
        if (time_avg_density) time_avg_density[n] = avg;
        if (avg > pk) pk = avg;
    }
    out->total_Q = tq;
    out->total_charge_C = -kE * ((double)tq * in.d.inv_two_S);
    out->peak_time_avg_density = pk;
    return cs;
}

extern "C" pic_status pic_timing(pic_ctx* ctx, int enable, long long* launches, double* total_ms) {
    if (!ctx) return PIC_EINVAL;
    pic_status st = timing_collect(ctx);
    if (st != PIC_OK) return st;
    if (launches) *launches = ctx->timed_launches;
    if (total_ms) *total_ms = ctx->timed_ms;
    if (enable) {
        ctx->timed_launches = 0;
        ctx->timed_ms = 0.0;
    }
    ctx->timing = enable != 0;
    return PIC_OK;
}

extern "C" pic_status pic_tuning(pic_ctx* ctx, int* tile_r, int* tile_z, int* halo,
                                 int* sort_interval, int* chunk, int* lanes, int* use_graph) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->mode != PIC_MODE_FP32_BATCHED) {
        if (tile_r) *tile_r = 0;
        if (tile_z) *tile_z = 0;
        if (halo) *halo = 0;
        if (sort_interval) *sort_interval = 0;
        if (chunk) *chunk = 0;
        if (lanes) *lanes = 0;
        if (use_graph) *use_graph = 0;
        return PIC_OK;
    }
    return f32_tuning(ctx, tile_r, tile_z, halo, sort_interval, chunk, lanes, use_graph);
}

extern "C" pic_status pic_retune(pic_ctx* ctx, int tile_r, int tile_z, int halo, int sort_interval) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->mode != PIC_MODE_FP32_BATCHED) return fail(ctx, PIC_EINVAL, "tiles exist in the FP32 form only");
    return f32_retune(ctx, tile_r, tile_z, halo, sort_interval);
}

extern "C" pic_status pic_autotune(pic_ctx* ctx, int trial_steps, const char* cache_path, int* tile_r,
                                   int* tile_z, int* halo, int* sort_interval, double* ms_per_step,
                                   int* trials) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->mode != PIC_MODE_FP32_BATCHED) return fail(ctx, PIC_EINVAL, "the autotuner serves the FP32 form");
    if (trial_steps < 1) return fail(ctx, PIC_EINVAL, "trial_steps >= 1");
    int v[4] = {0, 0, 0, 0};
    pic_status st = f32_autotune(ctx, trial_steps, cache_path, v, ms_per_step, trials);
    if (st != PIC_OK) return st;
    if (tile_r) *tile_r = v[0];
    if (tile_z) *tile_z = v[1];
    if (halo) *halo = v[2];
    if (sort_interval) *sort_interval = v[3];
    return PIC_OK;
}

extern "C" pic_status pic_reserve(pic_ctx* ctx, int k, long long slots) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (slots < 0) return fail(ctx, PIC_EINVAL, "slots < 0");
    if (slots <= ctx->in[k].cap) return PIC_OK;
    if (ctx->mode == PIC_MODE_FP64_PLAIN) return grow64(ctx, k, slots);
    return f32_reserve(ctx, k, slots);
}

extern "C" pic_status pic_capacity(pic_ctx* ctx, int k, long long* slots, long long* grow_events) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (slots) *slots = ctx->in[k].cap;
    if (grow_events) *grow_events = ctx->mode == PIC_MODE_FP64_PLAIN ? ctx->grow_events : f32_grow_events(ctx);
    return PIC_OK;
}

pic_status pic_moments_accumulate(pic_ctx* ctx, int k, double* acc) {
    Inst& in = ctx->in[k];
    if (ctx->mode != PIC_MODE_FP64_PLAIN) return f32_moments(ctx, k, acc);
    const hipError_t e = launch_moments64(in.I, in.p64[in.cur], in.cnt, acc, ctx->stream);
    if (e != hipSuccess) return fail(ctx, PIC_EDEVICE, std::string("moments: ") + hipGetErrorString(e));
    return PIC_OK;
}

extern "C" pic_status pic_moments(pic_ctx* ctx, int k, double* out) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (!out) return fail(ctx, PIC_EINVAL, "out is NULL");
    Inst& in = ctx->in[k];
    const long long N = in.nodes;
    hipStream_t s = ctx->stream;
    CK(hipStreamSynchronize(s));
    double* acc = dalloc<double>(ctx, kMoments * N);
    if (!acc) return fail(ctx, PIC_ENOMEM, "moment accumulators");
    hipError_t e = hipMemsetAsync(acc, 0, sizeof(double) * kMoments * N, s);
    if (e == hipSuccess) st = pic_moments_accumulate(ctx, k, acc);
    if (e == hipSuccess && st == PIC_OK) e = hipMemcpyAsync(out, acc, sizeof(double) * kMoments * N, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && st == PIC_OK) e = hipStreamSynchronize(s);
    pic_dev_free(ctx, acc);
    if (st != PIC_OK) return st;
    if (e != hipSuccess) return fail(ctx, PIC_EDEVICE, std::string("moments: ") + hipGetErrorString(e));
    for (int c = 0; c < kMoments; ++c)
        for (long long n = 0; n < N; ++n) out[c * N + n] /= in.V_host[n];
    return PIC_OK;
}

// Potential-well depth along the configured field lines (Sec. II.B): the
// trap of an electron on a line is a maximum of phi; its depth is that
// maximum less the higher of the lowest values on its two sides.  Lines of
// Bz = B0 (1 + k zeta^2), Br = -(r/2) Bz' keep r^2 Bz fixed.  Host work on a
// copy of the solved potential.
extern "C" pic_status pic_well_depth(pic_ctx* ctx, int k, int n_lines, const double* r_mid, double* depth,
                                     double* z_max) {
    pic_status st = check_inst(ctx, k);
    if (st != PIC_OK) return st;
    if (n_lines < 0 || (n_lines > 0 && (!r_mid || !depth || !z_max))) return fail(ctx, PIC_EINVAL, "bad line arrays");
    Inst& in = ctx->in[k];
    const pic_instance_cfg& c = in.c;
    const int nr = c.nr, nz = c.nz, W = nz + 1;
    std::vector<double> phi((size_t)in.nodes);
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(phi.data(), in.phi, sizeof(double) * phi.size(), hipMemcpyDeviceToHost));
    const double dr = (c.b - c.a) / (double)nr, dz = c.L / (double)nz, halfL = 0.5 * c.L;
    std::vector<double> U((size_t)W);
    std::vector<char> inside((size_t)W);
    for (int l = 0; l < n_lines; ++l) {
        for (int j = 0; j <= nz; ++j) {
            const double z = (double)j * dz, zeta = (z - halfL) / halfL;
            const double r = r_mid[l] * sqrt(c.B0 / (c.B0 * (1.0 + c.mirror_k * (zeta * zeta))));
            inside[j] = r > c.a && r < c.b;
            U[j] = 0.0;
            if (!inside[j]) continue;
            const double s = (r - c.a) / dr;
            const int i = std::min((int)floor(s), nr - 1);
            const double fr = s - (double)i;
            const int jc = std::min(j, nz - 1);
            const double fz = (z - (double)jc * dz) / dz;
            const double* P = phi.data() + (size_t)i * W + jc;
            U[j] = ((1.0 - fr) * (1.0 - fz) * P[0] + fr * (1.0 - fz) * P[W]) +
                   ((1.0 - fr) * fz * P[1] + fr * fz * P[W + 1]);
        }
        depth[l] = 0.0;
        z_max[l] = -1.0;
        const int mid = nz / 2;
        if (!inside[mid]) continue;
        int lo = mid, hi = mid;
        while (lo > 0 && inside[lo - 1]) --lo;
        while (hi < nz && inside[hi + 1]) ++hi;
        const int top = (int)(std::max_element(U.begin() + lo, U.begin() + hi + 1) - U.begin());
        const double left = *std::min_element(U.begin() + lo, U.begin() + top + 1);
        const double right = *std::min_element(U.begin() + top, U.begin() + hi + 1);
        depth[l] = U[top] - std::max(left, right);
        z_max[l] = (double)top * dz;
    }
    return PIC_OK;
}
