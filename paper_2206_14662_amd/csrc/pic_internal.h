// pic_internal.h -- shared declarations of the gfx950 PIC-MCC library:
// the per-instance parameter block the kernels read, the device counter
// layout, the Philox4x32-10 generator and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pic.h"

namespace pic {

// CODATA 2018
constexpr double kE = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kKb = 1.380649e-23;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kPi = 3.14159265358979323846;

// Per-instance constants read by the kernels (plain old data, passed by
// value to the per-instance FP64 kernels and stored as a device table for the
// batched FP32 kernels).
struct DevInst {
    // mesh
    double a, b, L, dr, dz, inv_dr, inv_dz;
    int nr, nz, W, nodes;           // W = nz + 1, nodes = (nr+1) W
    long long node_off;             // offset of this instance in batched node arrays
    // push
    double h, dt;
    // collisions
    double P_null, nu_prime, nsig_el, n_n, lotz_aq, iz_I, opal_Ebar, okh_xi;
    double okh_inv_E0;          // 1 / okh_E0_eV, 0: no screened-Coulomb xi(E)
    double half_me_over_e, two_e_over_me, mass_ratio2, v_cap2;
    unsigned long long null_k;      // u52 < P_null  <=>  (x >> 12) < null_k
    unsigned int seed_lo, seed_hi;
    int collisions;
    int frozen;
    // fixed point
    double two_S, inv_two_S;
    // particle segment (batched form)
    long long p_off, p_cap;
    // single-precision copies for the FP32 form
    float a_f, b_f, L_f, inv_dr_f, inv_dz_f, h_f, dt_f;
    float nu_prime_f, nsig_el_f, n_n_f, lotz_aq_f, iz_I_f, opal_Ebar_f, okh_xi_f, okh_inv_E0_f;
    float half_me_over_e_f, two_e_over_me_f, mass_ratio2_f, v_cap2_f;
    // sort tiles (FP32 form)
    int ntr, ntz;                   // tiles in r and z
    int tile_off;                   // first global tile id of this instance
    int diag_D;                     // steps between diagnostic samples
    int open_ends;                  // 1: d(phi)/dz = 0 at z = 0, L (cosine modes)
    // volumetric seed source
    double src_rate;                // macro-electrons per step (0: off)
    double src_sv;                  // its thermal speed sqrt(T e / m)
    double weight;                  // electrons per macro-electron of new source electrons
    // FP32 form: the weight every particle of the instance carries, so the
    // per-particle weight array is neither read nor kept up to date; 0 when
    // weights differ between particles (the array is then authoritative)
    float w_uni;
    // elliptic insert on the outer electrode (has_ins = 0: none): metal where
    // ins_g <= 0; web-spline weight band up to g = ins_gam
    int has_ins;
    double ins_r0, ins_z0, ins_er, ins_ez, ins_gam;
    float ins_r0_f, ins_z0_f, ins_inv_er_f, ins_inv_ez_f, ins_gam_f;
    // cubic space-charge shapes (0: bilinear / Q1)
    int spline3;
    // tabulated cross sections (xs_n = 0: constant elastic, Lotz ionisation)
    int xs_n;
    const double *xs_E, *xs_el, *xs_iz;
    const float *xs_Ef, *xs_elf, *xs_izf;
    // tabulated anisotropy xi(E) of the scattering law (xi_n = 0: okh_xi)
    int xi_n;
    const double *xi_E, *xi_v;
    const float *xi_Ef, *xi_vf;
};

// Tabulated cross section at energy x: linear in E between the tabulated
// points, the end values held outside the table (LXCat-style pairs).
template <typename T>
__host__ __device__ inline T xs_interp(int n, const T* E, const T* s, T x) {
#pragma clang fp contract(off)
    if (x <= E[0]) return s[0];
    if (x >= E[n - 1]) return s[n - 1];
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (E[mid] <= x) lo = mid;
        else hi = mid;
    }
    return s[lo] + (s[lo + 1] - s[lo]) * ((x - E[lo]) / (E[lo + 1] - E[lo]));
}

// Elliptic insert (Sec. III gun geometry): g = ((r-r0)/er)^2 + ((z-z0)/ez)^2 - 1,
// g <= 0 inside the metal.  Web-spline weight function of the space-charge
// basis: 0 in the metal, 1 - (1 - g/gam)^3 in the band 0 < g < gam, 1 beyond.
__host__ __device__ inline double ins_g(const DevInst& I, double r, double z) {
#pragma clang fp contract(off)
    const double u = (r - I.ins_r0) / I.ins_er, v = (z - I.ins_z0) / I.ins_ez;
    return (u * u + v * v) - 1.0;
}
__host__ __device__ inline double ins_w(const DevInst& I, double g) {
#pragma clang fp contract(off)
    if (g <= 0.0) return 0.0;
    if (g >= I.ins_gam) return 1.0;
    const double s = 1.0 - g / I.ins_gam;
    return 1.0 - s * s * s;
}

// Device counter block per instance (long long entries).
enum Counter {
    C_SLOTS = 0,      // used particle slots (live + dead), at step start
    C_SPAWN,          // electrons created in the current step
    C_DEAD,           // dead slots among C_SLOTS
    C_STEP,           // step counter (Philox counter word 2)
    C_ELASTIC,
    C_IONIZ,
    C_CAND,
    C_CAPOVER,
    C_DROPPED,
    C_ABS_N,          // 4 entries
    C_ABS_W = C_ABS_N + 4,   // 4 entries
    C_WLAST = C_ABS_W + 4,   // 4 entries: absorbed_W at the last sample
    C_IWALL = C_WLAST + 4,   // 4 entries: double bits, last window current
    C_PEAK = C_IWALL + 4,    // double bits: time max of spatial max density
    C_PEAKI_OUT,             // double bits
    C_PEAKI_IN,              // double bits
    C_NSAMP,
    C_OVERFLOW,              // fixed-point overflow flag
    C_LIVE_SORTED,           // live particles in the sorted region (FP32 form)
    C_PSTEPS,                // particle-steps pushed so far
    C_FARDEP,                // deposits outside the LDS window (FP32 form)
    C_SOURCE,                // electrons created by the seed source
    C_NONFIN,                // particles removed with a non-finite position (sticky error)
    C_NCOUNT = 40
};

// Control words of the batched FP32 step (device array, FP32 form only):
// work units handed out in a plain step, particles pushed this step, of
// which tile-sorted, real collision events queued, queue overflow flag, then
// per-instance exclusive prefix of the tail counts (electrons created since
// the last sort).
enum { CTL_WORK = 0, CTL_TOTAL = 1, CTL_SORTED = 2, CTL_QCOUNT = 3, CTL_QOVER = 4, CTL_TAIL = 5 };

// Plan of the coming step from the committed counters: tail prefix, total,
// an empty collision queue, no work units handed out.  Every thread of one block (at most 256
// threads) calls it; the prefix is an LDS scan over up to blockDim
// instances at a time.
__device__ inline void prep_tails_block(long long* ctl, const long long* cnt, int n_inst) {
    __shared__ long long s_v[256];
    __shared__ long long s_carry;
    long long* tb = ctl + CTL_TAIL;
    const int t = threadIdx.x, nt = blockDim.x;
    if (t == 0) {
        tb[0] = 0;
        ctl[CTL_QCOUNT] = 0;
        ctl[CTL_WORK] = 0;
        s_carry = 0;
    }
    for (int k0 = 0; k0 < n_inst; k0 += nt) {
        const int k = k0 + t;
        long long v = 0;
        if (k < n_inst) {
            const long long* c = cnt + (long long)k * C_NCOUNT;
            const long long tail = c[C_SLOTS] - c[C_LIVE_SORTED];
            v = tail > 0 ? tail : 0;
        }
        s_v[t] = v;
        __syncthreads();
        for (int off = 1; off < nt; off <<= 1) {  // inclusive scan
            const long long add = t >= off ? s_v[t - off] : 0;
            __syncthreads();
            s_v[t] += add;
            __syncthreads();
        }
        const long long carry = s_carry;
        if (k < n_inst) tb[k + 1] = carry + s_v[t];
        __syncthreads();
        if (t == nt - 1) s_carry = carry + s_v[t];
        __syncthreads();
    }
    if (t == 0) ctl[CTL_TOTAL] = ctl[CTL_SORTED] + s_carry;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// of counter words 0 and 2 by fixed multipliers, xor-mixed with the key,
// with the key advanced by two Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, unsigned int k0, unsigned int k1) {
    const unsigned int M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const unsigned int W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const unsigned long long p0 = (unsigned long long)M0 * c.x;
        const unsigned long long p1 = (unsigned long long)M1 * c.z;
        c = make_uint4((unsigned int)(p1 >> 32) ^ c.y ^ k0, (unsigned int)p1,
                       (unsigned int)(p0 >> 32) ^ c.w ^ k1, (unsigned int)p0);
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Open-interval uniform from the top 52 bits of hi:lo (exact in FP64).
__device__ __forceinline__ double u52(unsigned int hi, unsigned int lo) {
    unsigned long long x = ((unsigned long long)hi << 32) | (unsigned long long)lo;
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

// Fluid moments: channels n, n u (r, t, z), sum w v_a v_b (rr, rt, rz, tt,
// tz, zz) and sum w nu_m with nu_m = n_n (sigma_el + sigma_iz(E)) |v|, each as
// a bilinear (hat-function) node sum; divided by the node volume afterwards.
constexpr int kMoments = 11;

__device__ inline void moments_add(const DevInst& I, double r, double z, double vr, double vt, double vz, double w,
                                   double* __restrict__ acc) {
#pragma clang fp contract(off)
    double s = (r - I.a) * I.inv_dr;
    int i = (int)floor(s);
    i = i < 0 ? 0 : (i > I.nr - 1 ? I.nr - 1 : i);
    const double fr = s - (double)i;
    double t = z * I.inv_dz;
    int j = (int)floor(t);
    j = j < 0 ? 0 : (j > I.nz - 1 ? I.nz - 1 : j);
    const double fz = t - (double)j;
    const double sw[4] = {(1.0 - fr) * (1.0 - fz), fr * (1.0 - fz), (1.0 - fr) * fz, fr * fz};
    const long long n00 = (long long)i * I.W + j;
    const long long node[4] = {n00, n00 + I.W, n00 + 1, n00 + I.W + 1};
    const double v2 = (vr * vr + vt * vt) + vz * vz, v = sqrt(v2);
    const double E = v2 * I.half_me_over_e;
    double nu;
    if (I.xs_n > 0) {
        const double siz = E > I.iz_I ? xs_interp(I.xs_n, I.xs_E, I.xs_iz, E) : 0.0;
        nu = (I.n_n * xs_interp(I.xs_n, I.xs_E, I.xs_el, E) + I.n_n * siz) * v;
    } else {
        const double sig_iz = E > I.iz_I ? (I.lotz_aq * log(E / I.iz_I)) / (E * I.iz_I) : 0.0;
        nu = (I.nsig_el + I.n_n * sig_iz) * v;
    }
    const double q[kMoments] = {1.0, vr, vt, vz, vr * vr, vr * vt, vr * vz, vt * vt, vt * vz, vz * vz, nu};
    const long long N = I.nodes;
    for (int c = 0; c < kMoments; ++c)
        for (int k = 0; k < 4; ++k) atomicAdd(&acc[c * N + node[k]], (w * sw[k]) * q[c]);
}

// Seed source of step `step`: how many electrons it creates and the running
// index of the first (floor((n+1) R) - floor(n R) and floor(n R), R per step).
__device__ __forceinline__ void source_count(const DevInst& I, long long step, long long& first, long long& count) {
#pragma clang fp contract(off)
    const double n0 = floor((double)step * I.src_rate);
    const double n1 = floor((double)(step + 1) * I.src_rate);
    first = (long long)n0;
    count = (long long)(n1 - n0);
}

// The state of the seed-source electron with running index idx: key
// 2^62 + idx, three Philox blocks at step word 0xFFFFFFFE, r uniform in volume
// over (a, b), z uniform over (0, L), Box-Muller velocities (FP64).
__device__ inline void source_draw(const DevInst& I, long long idx, unsigned long long& key, double& r, double& z,
                                   double& vr, double& vt, double& vz) {
#pragma clang fp contract(off)
    key = (1ull << 62) + (unsigned long long)idx;
    const uint4 c0 = make_uint4((unsigned int)key, (unsigned int)(key >> 32), 0xFFFFFFFEu, 0u);
    const uint4 b0 = philox4x32_10(c0, I.seed_lo, I.seed_hi);
    const uint4 b1 = philox4x32_10(make_uint4(c0.x, c0.y, c0.z, 1u), I.seed_lo, I.seed_hi);
    const uint4 b2 = philox4x32_10(make_uint4(c0.x, c0.y, c0.z, 2u), I.seed_lo, I.seed_hi);
    const double ur = u52(b0.x, b0.y), uz = u52(b0.z, b0.w);
    const double u1 = u52(b1.x, b1.y), u2 = u52(b1.z, b1.w);
    const double u3 = u52(b2.x, b2.y), u4 = u52(b2.z, b2.w);
    const double m1 = sqrt(-2.0 * log(u1)), m3 = sqrt(-2.0 * log(u3));
    r = sqrt(I.a * I.a + ur * (I.b * I.b - I.a * I.a));
    z = uz * I.L;
    vr = I.src_sv * (m1 * cos((2.0 * kPi) * u2));
    vt = I.src_sv * (m1 * sin((2.0 * kPi) * u2));
    vz = I.src_sv * (m3 * cos((2.0 * kPi) * u4));
}
// Open-interval uniform from the top 23 bits of a word (exact in FP32).
__device__ __forceinline__ float u23(unsigned int w) {
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

// Positive doubles order like their bit patterns.
__device__ __forceinline__ void atomic_max_pos_double(long long* slot, double v) {
    atomicMax((unsigned long long*)slot, (unsigned long long)__double_as_longlong(v));
}

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
// ---------------------------------------------------------------------------

// FP64 plain form (k_fp64.hip)
struct P64 {
    double *r, *z, *vr, *vt, *vz, *w;
    unsigned long long* key;
};
hipError_t launch_load64(const DevInst& I, const pic_instance_cfg& c, P64 p, long long n,
                         hipStream_t s);
// cx: cubic shapes' ghosted space-charge coefficients (else null)
hipError_t launch_push64(const DevInst& I, P64 p, const double* Er, const double* Ez,
                         const double* Br, const double* Bz, const double* cx, long long* cnt, long long grid_cap,
                         hipStream_t s);
// Seed-source electrons of the step appended after the slots (FP64 form).
hipError_t launch_source64(const DevInst& I, P64 p, long long* cnt, hipStream_t s);
// Fluid-moment node sums of the FP64 store into acc (kMoments x nodes, zeroed).
hipError_t launch_moments64(const DevInst& I, P64 p, const long long* cnt, double* acc, hipStream_t s);
hipError_t launch_mcc64(const DevInst& I, P64 p, long long* cnt, long long grid_cap,
                        hipStream_t s);
// Qw (insert instances, else null): the band particles' q (w(x_p) - 1)
// Qx (cubic shapes, else null): the ghosted cubic deposit
hipError_t launch_deposit64(const DevInst& I, P64 p, long long* Q, long long* Qw, long long* Qx, long long* cnt,
                            long long grid_cap, hipStream_t s);
hipError_t launch_compact64(const DevInst& I, P64 src, P64 dst, long long* cnt,
                            long long* tmp_count, long long grid_cap, hipStream_t s);

// Field solve and diagnostics (k_field.hip), FP64.
// The tridiagonal solve in r splits the interior rows into segments solved
// concurrently: 32 register-held segments (two per wave, 32 modes per
// workgroup, so that a batch fills the chip) of at most kThomasRegRows rows,
// else kThomasSeg segments streamed through memory.  Host factors and kernels
// take the count from thomas_segments(largest nr of the context).
constexpr int kThomasSeg = 8;
constexpr int kThomasSegReg = 16;
constexpr int kThomasRegRows = 16;
inline int thomas_segments(int max_nr) {
    const int rows = max_nr - 1;
    if ((rows + 2 * kThomasSegReg - 1) / (2 * kThomasSegReg) <= kThomasRegRows) return 2 * kThomasSegReg;
    return kThomasSeg;
}
struct FieldDev {
    long long* Q;          // fixed-point charge (nodes)
    double* rhs;           // scratch node array: transformed rows / modes
    double* phi;           // potential (nodes)
    const double* phi_vac; // vacuum potential (nodes), boundary data on the edges
    const double* th_cp;   // Thomas factors, [i][k] with row length W
    const double* th_im;
    const double* th_lo;
    const double* th_G;    // forward and backward homogeneous factors within
    const double* th_H;    // the kThomasSeg row segments of the partitioned solve
    double *Er, *Ez;       // FP64 plain form outputs (or null)
    const double *Br, *Bz;
    float4* EB;            // FP32 form output (or null)
    const double* V;       // node volumes
    double* avg_acc;       // time-average accumulator
    long long* Qw;         // insert: charges of q (w(x_p) - 1) of the particles in the weight band, a node
                           // array with bilinear shapes, ghosted like Qx with cubic shapes
    // cubic shapes: ghosted deposit and coefficients ((nr+3) x (nz+3)), the
    // per-mode LDL^T factors of the 7-band r systems ([i][k], row length W)
    long long* Qx;
    double* cx;
    float* cxf;            // FP32 copy of cx for the batched form (else NULL)
    const double *s3_L1, *s3_L2, *s3_L3, *s3_Dinv;
};

// Cubic B-spline weights of the nodes i0-1 .. i0+2 at offset f in [0, 1)
// from i0, and their derivatives.
__host__ __device__ inline void bspline3(double f, double w[4], double dw[4]) {
#pragma clang fp contract(off)
    const double g = 1.0 - f;
    w[0] = (g * g * g) / 6.0;
    w[1] = ((3.0 * f - 6.0) * f * f + 4.0) / 6.0;
    w[2] = (((-3.0 * f + 3.0) * f + 3.0) * f + 1.0) / 6.0;
    w[3] = (f * f * f) / 6.0;
    dw[0] = -(g * g) / 2.0;
    dw[1] = ((3.0 * f - 4.0) * f) / 2.0;
    dw[2] = ((-3.0 * f + 2.0) * f + 1.0) / 2.0;
    dw[3] = (f * f) / 2.0;
}

// Elliptic insert, device side of the corrected solve (insert.hip).  The
// instance's Galerkin system differs from the rectangle's only in the rows
// and columns of the m nodes of M (next to the insert): A = A_rect + E D E^T.
// A step solves y = A_rect^-1 b, s = H y_M with H = (I + D G)^-1 D and
// G = (A_rect^-1)_MM, then x = y - A_rect^-1 E s, and evaluates the basis at
// the nodes of M.
struct InsDev {
    int inst;              // instance in the main tables
    int m;                 // nodes in M
    long long nodes;
    const int* Mnode;      // [m] node index of each M entry
    const int* map;        // [nodes] index in M or -1
    const int* rp;         // [m+1] load of M entry a: sum_t rf[t] (Q + Qw)[rk[t]]
    const int* rk;
    const double* rf;
    const double* H;       // [m x m] row-major
    const int* typ;        // [m] basis at the node: 1 w c, 2 w * extension, 0 zero
    const double* wn;      // [m] weight function at the node
    const int* ek;         // [4m] extension block of an outer node
    const double* ef;      // [4m] its factors
    double* ybuf;          // [nodes] phi_base + A_rect^-1 b
    double* rhs2;          // [nodes] load of the correction, then its modes
    double* yM;            // [m]
    double* sM;            // [m]
    double* val;           // [m]
};

// Cubic shapes with the insert (insert3.hip): the load of the unknowns of M
// and the ghosted coefficients rebuilt after the corrected solve.
struct Ins3Dev {
    int inst;              // instance in the main tables
    int m;                 // unknowns in M
    int nx;                // ghosted coefficients rebuilt after a solve
    const int* Mnode;      // [m] node of each unknown of M
    const int* typ;        // [m] 1: inner (takes its load), 0: load 0
    const int* rp;         // [m+1] load of M entry a: sum_t rf[t] (Qx + Qw)[rk[t]] (ghosted)
    const int* rk;
    const double* rf;
    const int* xk;         // [nx] ghosted index of a rebuilt coefficient
    const int* xn;         // [16 nx] nodes of the block's coefficients (-1: none)
    const double* xf;      // [16 nx] their factors (reflection sign times extension weight)
};

// Host set-up of one instance's cubic web-spline system (insert3.hip).
struct Ins3Host {
    int m = 0, nx = 0;
    std::vector<int> Mnode, map, typ, rp, rk, xk, xn;
    std::vector<double> rf, xf;
    std::vector<int> Dr, Dc;          // correction matrix D (entries by M index)
    std::vector<double> Dv;
    int counts[4] = {0, 0, 0, 0};     // nodes: not an unknown, inner, outer, exterior
};

// Host set-up of one instance's insert (independent of the device).
struct InsHost {
    int m = 0;
    std::vector<int> Mnode, map, rp, rk, typ, ek;
    std::vector<double> rf, wn, ef;
    std::vector<int> Dr, Dc;          // correction matrix D (entries by M index)
    std::vector<double> Dv;
    int counts[4] = {0, 0, 0, 0};     // nodes: not unknown, inner, outer, exterior
};
hipError_t launch_zero_i64(long long* p, long long n, hipStream_t s);
// Poisson solve of instances [inst_base, inst_base+n_inst) of the device
// tables: mode 0 from Q (scaled by bscale[inst]), mode 1 from rhs.
hipError_t launch_solve_tab(const DevInst* It, const FieldDev* Ft, int inst_base, int n_inst,
                            int max_nr, int max_nz, const double2* tw, int tw_n, int mode,
                            const double* bscale, bool edges, hipStream_t s);
// cnt: the instances' counters (from instance 0) when the step's diagnostics
// sample rides on the same launch, else NULL
hipError_t launch_efield_tab(const DevInst* It, const FieldDev* Ft, int inst_base, int n_inst,
                             long long max_nodes, bool with_B, hipStream_t s, long long* cnt = nullptr);
// Diagnostics sample (every D steps), then the end of the step: counters
// committed (slots += spawned, step += 1) and, when ctl is given, the next
// FP32 step planned.
hipError_t launch_sample_tab(const DevInst* It, const FieldDev* Ft, int n_inst, long long* cnt, long long* ctl,
                             hipStream_t s);
hipError_t set_field_kernel_attrs(int max_nz);
// the end of the step alone (after a sample taken by launch_efield_tab)
hipError_t launch_commit(const DevInst* It, long long* cnt, long long* ctl, int n_inst, hipStream_t s);

// Elliptic insert (insert.hip).  ins_build classifies the nodes, attaches
// the outer hats, and assembles D on the host; an empty string means success.
std::string ins_build(const pic_instance_cfg& c, InsHost& h);
// The allocation-free entry points' scratch on the current device
// (noalloc.hip): look up its address once per device.
hipError_t noalloc_setup(int device);
// The insert fields of DevInst (centre, semi-axes, weight band gam) of an
// instance with mesh spacings dr, dz.
void ins_fill(const pic_instance_cfg& c, double dr, double dz, DevInst& I);
// Cubic shapes (k_field.hip): load folded from Qx, sine transform, the
// 7-band solves, inverse transform into the coefficient buffer (the table's
// phi), then the ghosted coefficients and phi = phi_vac + nodal value.
hipError_t launch_solve3_tab(const DevInst* It, const FieldDev* Ft, const FieldDev* F3, int n_inst, int max_nr,
                             int max_nz, long long max_ext, const double2* tw, int tw_n, const double* bscale,
                             hipStream_t s);
// ... and its three parts: the folded load into the table's rhs; the
// rectangle solve of rhs (phi = phi_vac + A_rect^-1 rhs); the ghosted
// coefficients and the nodal potential.
hipError_t launch_s3_fold(const DevInst* It, const FieldDev* F3, int n_inst, long long max_nodes,
                          const double* bscale, hipStream_t s);
hipError_t launch_s3_rect(const DevInst* It, const FieldDev* F3, int n_inst, int max_nr, int max_nz,
                          const double2* tw, int tw_n, const double* bscale, hipStream_t s);
hipError_t launch_s3_post(const DevInst* It, const FieldDev* Ft, const FieldDev* F3, int n_inst, long long max_ext,
                          hipStream_t s);
// Cubic web-splines with the insert (insert3.hip): host set-up (an empty
// string means success), the load of M over the plain folded load, and after
// the corrected solve the rebuilt ghosted coefficients and the nodal
// potential phi_vac + w (coefficient sum).
std::string ins3_build(const pic_instance_cfg& c, Ins3Host& h);
hipError_t launch_ins3_rhs(const DevInst* It, const Ins3Dev* X, int n_ins, int max_m, const FieldDev* Ft,
                           const double* bscale, hipStream_t s);
hipError_t launch_ins3_post(const DevInst* It, const Ins3Dev* X, int n_ins, int max_nx, long long max_nodes,
                            const FieldDev* Ft, const FieldDev* F3, hipStream_t s);
// per step (or for the vacuum): the load of every insert instance's nodes
// from Q and Qw (scaled by bscale) into rhs
hipError_t launch_ins_rhs(const DevInst* It, const InsDev* D, int n_ins, long long max_nodes, const FieldDev* Ft,
                          const double* bscale, hipStream_t s);
// y_M = ybuf - base at M, s = H y_M, rhs2 = -E s (every node written); the
// instances sharing one H form the n_grp groups goff / gmem (entries of D)
hipError_t launch_ins_correct(const DevInst* It, const InsDev* D, int n_ins, const int* goff, const int* gmem,
                              int n_grp, int max_m, long long max_nodes, const FieldDev* Fbase, hipStream_t s);
// the basis evaluated at the nodes of M: phi = base + (w c | w ext c | 0)
hipError_t launch_ins_fix(const DevInst* It, const InsDev* D, int n_ins, int max_m, const FieldDev* Fout,
                          hipStream_t s);
// set-up: unit right-hand sides e_{Mnode[b0+t]} in rhs + t * stride, and the
// M entries of the solutions into G[:, b0+t]
hipError_t launch_ins_units(double* rhs, long long stride, long long nodes, const int* Mnode, int b0, int cnt,
                            hipStream_t s);
hipError_t launch_ins_collect(const double* phi, long long stride, const int* Mnode, int m, int b0, int cnt,
                              double* G, hipStream_t s);
// set-up: Gauss-Jordan elimination with partial pivoting of [C | D] (m x 2m,
// row-major) into [I | C^-1 D]; *singular set when a pivot vanishes
hipError_t launch_ins_gauss_jordan(double* CD, int m, double* fcol, int* piv, double* pval, hipStream_t s);

}  // namespace pic
