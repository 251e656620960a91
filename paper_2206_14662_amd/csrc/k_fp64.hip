// k_fp64.hip -- the plain FP64 form of the particle loop: one kernel per
// stage (push, collisions, deposit), SoA FP64 particles, no sort, no LDS,
// direct global int64 atomics.  Built with floating-point contraction off so
// every operation rounds exactly as written; the CPU oracle of the test-suite
// evaluates the same expressions in the same order.
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint4 blk(const DevInst& I, unsigned long long key, unsigned int step,
                                     unsigned int b) {
    return philox4x32_10(make_uint4((unsigned int)key, (unsigned int)(key >> 32), step, b),
                         I.seed_lo, I.seed_hi);
}

// Bilinear shape (order-1 spline) of a position; cell (i,j) and fractions.
struct Shape {
    int i, j;
    double w00, w10, w01, w11;
};

__device__ __forceinline__ Shape shape64(const DevInst& I, double r, double z) {
    Shape sh;
    double s = (r - I.a) * I.inv_dr;
    int i = (int)floor(s);
    i = i < 0 ? 0 : (i > I.nr - 1 ? I.nr - 1 : i);
    double fr = s - (double)i;
    double t = z * I.inv_dz;
    int j = (int)floor(t);
    j = j < 0 ? 0 : (j > I.nz - 1 ? I.nz - 1 : j);
    double fz = t - (double)j;
    sh.i = i;
    sh.j = j;
    sh.w00 = (1.0 - fr) * (1.0 - fz);
    sh.w10 = fr * (1.0 - fz);
    sh.w01 = (1.0 - fr) * fz;
    sh.w11 = fr * fz;
    return sh;
}

// Cubic shapes: base node i0 (clamped) and offset of a coordinate.
__device__ __forceinline__ void base3(double s, int n, int& i0, double& f) {
    int i = (int)floor(s);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    i0 = i;
    f = s - (double)i;
}

// Space-charge field -grad phi_sc at (r, z) from the ghosted cubic
// coefficients (nodes i0-1 .. i0+2 at ghosted rows i0 .. i0+3).  With the
// insert phi_sc = w u (web-splines, u the cubic expansion), so inside the
// weight band E = w (-grad u) - u grad w.
__device__ __forceinline__ void field3(const DevInst& I, const double* cx, double r, double z, double& er,
                                       double& ez) {
    int i0, j0;
    double fr, fz, wr[4], dwr[4], wz[4], dwz[4];
    base3((r - I.a) / I.dr, I.nr, i0, fr);
    base3(z / I.dz, I.nz, j0, fz);
    bspline3(fr, wr, dwr);
    bspline3(fz, wz, dwz);
    const int WX = I.nz + 3;
    double gr = 0.0, gz = 0.0, u = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const double v = cx[(long long)(i0 + a) * WX + (j0 + b)];
            gr += v * (dwr[a] * wz[b]);
            gz += v * (wr[a] * dwz[b]);
            u += v * (wr[a] * wz[b]);
        }
    er = -(gr / I.dr);
    ez = -(gz / I.dz);
    if (I.has_ins) {
        const double g = ins_g(I, r, z);
        if (g < I.ins_gam) {
            const double w = ins_w(I, g);
            double gwr = 0.0, gwz = 0.0;
            if (g > 0.0) {
                const double s = 1.0 - g / I.ins_gam, d = 3.0 * s * s / I.ins_gam;
                gwr = d * (2.0 * (r - I.ins_r0) / (I.ins_er * I.ins_er));
                gwz = d * (2.0 * (z - I.ins_z0) / (I.ins_ez * I.ins_ez));
            }
            er = w * er - u * gwr;
            ez = w * ez - u * gwz;
        }
    }
}

__device__ __forceinline__ double gather64(const Shape& sh, const double* F, int W) {
    long long n00 = (long long)sh.i * W + sh.j;
    return ((sh.w00 * F[n00] + sh.w10 * F[n00 + W]) + sh.w01 * F[n00 + 1]) + sh.w11 * F[n00 + W + 1];
}

// Initial Maxwellian load: Philox counter {p, 0xFFFFFFFF, block}, Box-Muller.
__global__ void k_load64(DevInst I, double r_lo, double r_hi, double z_lo, double z_hi, double sv,
                         double w0, int load_mode, P64 p, long long n) {
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        unsigned long long key = (unsigned long long)q;
        uint4 b0 = blk(I, key, 0xFFFFFFFFu, 0u);
        uint4 b1 = blk(I, key, 0xFFFFFFFFu, 1u);
        uint4 b2 = blk(I, key, 0xFFFFFFFFu, 2u);
        double ur = u52(b0.x, b0.y), uz = u52(b0.z, b0.w);
        double r;
        if (load_mode == 1) r = r_lo + ur * (r_hi - r_lo);
        else r = sqrt(r_lo * r_lo + ur * (r_hi * r_hi - r_lo * r_lo));
        double z = z_lo + uz * (z_hi - z_lo);
        double u1 = u52(b1.x, b1.y), u2 = u52(b1.z, b1.w);
        double u3 = u52(b2.x, b2.y), u4 = u52(b2.z, b2.w);
        double m1 = sqrt(-2.0 * log(u1)), m3 = sqrt(-2.0 * log(u3));
        p.r[q] = r;
        p.z[q] = z;
        p.vr[q] = sv * (m1 * cos((2.0 * kPi) * u2));
        p.vt[q] = sv * (m1 * sin((2.0 * kPi) * u2));
        p.vz[q] = sv * (m3 * cos((2.0 * kPi) * u4));
        p.w[q] = w0;
        p.key[q] = key;
    }
}

// Gather + Boris + remap + absorb over the slots present at step start.
__global__ void __launch_bounds__(kBlock) k_push64(DevInst I, P64 p, const double* __restrict__ Er,
                                                  const double* __restrict__ Ez,
                                                  const double* __restrict__ Br,
                                                  const double* __restrict__ Bz,
                                                  const double* __restrict__ cx, long long* cnt) {
    const long long n = cnt[C_SLOTS];
    const double h = I.h, dt = I.dt;
    unsigned long long pushed = 0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        double r = p.r[q];
        if (r < 0.0) continue;
        ++pushed;
        double z = p.z[q], vr = p.vr[q], vt = p.vt[q], vz = p.vz[q];
        Shape sh = shape64(I, r, z);
        double er = gather64(sh, Er, I.W), ez = gather64(sh, Ez, I.W);
        double br = gather64(sh, Br, I.W), bz = gather64(sh, Bz, I.W);
        if (cx) {
            // cubic shapes: the nodal arrays hold the vacuum field; the space
            // charge's comes from the spline coefficients at the particle
            double e3r, e3z;
            field3(I, cx, r, z, e3r, e3z);
            er += e3r;
            ez += e3z;
        }
        double hEr = h * er, hEz = h * ez;
        double mr = vr + hEr, mt = vt, mz = vz + hEz;
        double tr = h * br, tz = h * bz;
        double tt = tr * tr + tz * tz;
        double f = 2.0 / (1.0 + tt);
        double sr = f * tr, sz = f * tz;
        double pr = mr + mt * tz;
        double pt = mt + (mz * tr - mr * tz);
        double pz = mz - mt * tr;
        double qr = mr + pt * sz;
        double qt = mt + (pz * sr - pr * sz);
        double qz = mz - pt * sr;
        vr = qr + hEr;
        vt = qt;
        vz = qz + hEz;
        double x = r + vr * dt;
        double y = vt * dt;
        double zn = z + vz * dt;
        double rr2 = x * x + y * y;
        double rn = sqrt(rr2);
        int wall = -1;
        // a non-finite new position (a non-finite field or velocity) removes
        // the particle without counting it as absorbed charge
        if (!(rr2 < HUGE_VAL && fabs(zn) < HUGE_VAL)) wall = 4;
        else if (rn <= I.a) wall = 0;
        else if (rn >= I.b) wall = 1;
        else if (I.has_ins && ins_g(I, rn, zn) <= 0.0) wall = 1;  // the insert is outer-electrode metal
        else if (zn <= 0.0) wall = 2;
        else if (zn >= I.L) wall = 3;
        if (wall >= 0) {
            if (wall == 4) {
                atomicAdd((unsigned long long*)&cnt[C_NONFIN], 1ull);
            } else {
                long long Wq = (long long)rint(p.w[q] * I.two_S);
                atomicAdd((unsigned long long*)&cnt[C_ABS_N + wall], 1ull);
                atomicAdd((unsigned long long*)&cnt[C_ABS_W + wall], (unsigned long long)Wq);
            }
            atomicAdd((unsigned long long*)&cnt[C_DEAD], 1ull);
            p.r[q] = -1.0;
            continue;
        }
        double cs = x / rn, sn = y / rn;
        p.r[q] = rn;
        p.z[q] = zn;
        p.vr[q] = cs * vr + sn * vt;
        p.vt[q] = cs * vt - sn * vr;
        p.vz[q] = vz;
    }
    if (pushed) atomicAdd((unsigned long long*)&cnt[C_PSTEPS], pushed);
}

// Anisotropy of the scattering law for an electron of energy E (eV): the
// table xi(E) when the instance has one, else the constant okh_xi.
__device__ __forceinline__ double xi_at(const DevInst& I, double E) {
    if (I.xi_n > 0) return xs_interp(I.xi_n, I.xi_E, I.xi_v, E);
    if (I.okh_inv_E0 > 0.0) {
        // screened-Coulomb xi(E) = 4 e / (1 + 4 e), e = E / E0
        const double e4 = 4.0 * (E * I.okh_inv_E0);
        return e4 / (1.0 + e4);
    }
    return I.okh_xi;
}

__device__ __forceinline__ double okh_cos(double xi, double u) {
    return ((2.0 * u + xi) - 1.0) / ((1.0 - xi) + (2.0 * xi) * u);
}

__device__ __forceinline__ void scatter64(double ur, double ut, double uz, double cosx, double phi,
                                          double* o) {
    double e1r, e1t, e1z;
    if (fabs(uz) < 0.99) {
        double nn = sqrt(ur * ur + ut * ut);
        e1r = -ut / nn; e1t = ur / nn; e1z = 0.0;
    } else {
        double nn = sqrt(uz * uz + ut * ut);
        e1r = 0.0; e1t = -uz / nn; e1z = ut / nn;
    }
    double e2r = ut * e1z - uz * e1t;
    double e2t = uz * e1r - ur * e1z;
    double e2z = ur * e1t - ut * e1r;
    double sinx = sqrt(fmax(0.0, 1.0 - cosx * cosx));
    double cp = cos(phi), sp = sin(phi);
    o[0] = cosx * ur + sinx * (cp * e1r + sp * e2r);
    o[1] = cosx * ut + sinx * (cp * e1t + sp * e2t);
    o[2] = cosx * uz + sinx * (cp * e1z + sp * e2z);
}

// Null-collision MCC over the slots present at step start; new electrons are
// appended after them and are not collided in their first step.
__global__ void __launch_bounds__(kBlock) k_mcc64(DevInst I, P64 p, long long* cnt) {
    const long long n = cnt[C_SLOTS];
    const unsigned int step = (unsigned int)cnt[C_STEP];
    unsigned long long n_el = 0, n_iz = 0, n_cand = 0, n_cap = 0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        double r = p.r[q];
        if (r < 0.0) continue;
        double vr = p.vr[q], vt = p.vt[q], vz = p.vz[q];
        double v2 = (vr * vr + vt * vt) + vz * vz;
        if (v2 > I.v_cap2) ++n_cap;
        if (!I.collisions) continue;
        unsigned long long key = p.key[q];
        uint4 b0 = blk(I, key, step, 0u);
        if (!(u52(b0.x, b0.y) < I.P_null)) continue;
        ++n_cand;
        double u_proc = u52(b0.z, b0.w);
        double v = sqrt(v2);
        double E = v2 * I.half_me_over_e;
        double nu_el, sig_iz = 0.0;
        if (I.xs_n > 0) {
            nu_el = (I.n_n * xs_interp(I.xs_n, I.xs_E, I.xs_el, E)) * v;
            if (E > I.iz_I) sig_iz = xs_interp(I.xs_n, I.xs_E, I.xs_iz, E);
        } else {
            nu_el = I.nsig_el * v;
            if (E > I.iz_I) sig_iz = (I.lotz_aq * log(E / I.iz_I)) / (E * I.iz_I);
        }
        double nu_iz = (I.n_n * sig_iz) * v;
        double R = u_proc * I.nu_prime;
        int ev;
        if (R < nu_el) ev = 1;
        else if (R < nu_el + nu_iz) ev = 2;
        else continue;
        double ur = vr / v, ut = vt / v, uz = vz / v;
        uint4 b1 = blk(I, key, step, 1u);
        double phi1 = (2.0 * kPi) * u52(b1.z, b1.w);
        double dir[3];
        if (ev == 1) {
            const double cos1 = okh_cos(xi_at(I, E), u52(b1.x, b1.y));
            ++n_el;
            double En = E * (1.0 - I.mass_ratio2 * (1.0 - cos1));
            double vn = sqrt(En * I.two_e_over_me);
            scatter64(ur, ut, uz, cos1, phi1, dir);
            p.vr[q] = vn * dir[0];
            p.vt[q] = vn * dir[1];
            p.vz[q] = vn * dir[2];
            continue;
        }
        ++n_iz;
        uint4 b2 = blk(I, key, step, 2u);
        uint4 b3 = blk(I, key, step, 3u);
        double E_av = E - I.iz_I;
        double E_s = I.opal_Ebar * tan(u52(b2.x, b2.y) * atan(E_av / (2.0 * I.opal_Ebar)));
        double E_p = E_av - E_s;
        const double cos1 = okh_cos(xi_at(I, E_p), u52(b1.x, b1.y));
        double cos2 = okh_cos(xi_at(I, E_s), u52(b2.z, b2.w));
        double phi2 = (2.0 * kPi) * u52(b3.x, b3.y);
        double vp = sqrt(E_p * I.two_e_over_me);
        double vs = sqrt(E_s * I.two_e_over_me);
        scatter64(ur, ut, uz, cos1, phi1, dir);
        p.vr[q] = vp * dir[0];
        p.vt[q] = vp * dir[1];
        p.vz[q] = vp * dir[2];
        scatter64(ur, ut, uz, cos2, phi2, dir);
        long long slot = n + (long long)atomicAdd((unsigned long long*)&cnt[C_SPAWN], 1ull);
        if (slot >= I.p_cap) {
            atomicAdd((unsigned long long*)&cnt[C_DROPPED], 1ull);
            continue;
        }
        p.r[slot] = r;
        p.z[slot] = p.z[q];
        p.vr[slot] = vs * dir[0];
        p.vt[slot] = vs * dir[1];
        p.vz[slot] = vs * dir[2];
        p.w[slot] = p.w[q];
        p.key[slot] = ((((unsigned long long)b3.z) << 32) | (unsigned long long)b3.w) | (1ull << 63);
    }
    if (n_el) atomicAdd((unsigned long long*)&cnt[C_ELASTIC], n_el);
    if (n_iz) atomicAdd((unsigned long long*)&cnt[C_IONIZ], n_iz);
    if (n_cand) atomicAdd((unsigned long long*)&cnt[C_CAND], n_cand);
    if (n_cap) atomicAdd((unsigned long long*)&cnt[C_CAPOVER], n_cap);
}

// Volumetric seed source (Sec. II.A): this step's new electrons, appended
// after the slots like the ionisation products; deposited with them.
__global__ void __launch_bounds__(kBlock) k_source64(DevInst I, P64 p, long long* cnt) {
    long long first, count;
    source_count(I, cnt[C_STEP], first, count);
    const long long n = cnt[C_SLOTS];
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < count;
         j += (long long)gridDim.x * blockDim.x) {
        unsigned long long key;
        double r, z, vr, vt, vz;
        source_draw(I, first + j, key, r, z, vr, vt, vz);
        if (I.has_ins && ins_g(I, r, z) <= 0.0) continue;  // inside the insert: outside the domain
        atomicAdd((unsigned long long*)&cnt[C_SOURCE], 1ull);
        const long long slot = n + (long long)atomicAdd((unsigned long long*)&cnt[C_SPAWN], 1ull);
        if (slot >= I.p_cap) {
            atomicAdd((unsigned long long*)&cnt[C_DROPPED], 1ull);
            continue;
        }
        p.r[slot] = r;
        p.z[slot] = z;
        p.vr[slot] = vr;
        p.vt[slot] = vt;
        p.vz[slot] = vz;
        p.w[slot] = I.weight;
        p.key[slot] = key;
    }
}

// Fluid-moment node sums of every live particle (diagnostic).
__global__ void __launch_bounds__(kBlock) k_moments64(DevInst I, P64 p, const long long* cnt, double* acc) {
    const long long n = cnt[C_SLOTS];
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const double r = p.r[q];
        if (r < 0.0) continue;
        moments_add(I, r, p.z[q], p.vr[q], p.vt[q], p.vz[q], p.w[q], acc);
    }
}

// Fixed-point deposit: node charges rint(W w_k) for three nodes, the fourth
// takes the remainder so every particle adds exactly W.  With the insert, a
// particle in the weight function's band also deposits rint(W (w(x_p) - 1))
// into Qw by the same rule (by the 16-node rule into the ghosted Qw with
// cubic shapes).
__device__ __forceinline__ void deposit4(long long* Q, const Shape& sh, int W, long long Wq) {
    const double Wd = (double)Wq;
    const long long q00 = (long long)rint(Wd * sh.w00);
    const long long q10 = (long long)rint(Wd * sh.w10);
    const long long q01 = (long long)rint(Wd * sh.w01);
    const long long q11 = Wq - q00 - q10 - q01;
    const long long n00 = (long long)sh.i * W + sh.j;
    atomicAdd((unsigned long long*)&Q[n00], (unsigned long long)q00);
    atomicAdd((unsigned long long*)&Q[n00 + W], (unsigned long long)q10);
    atomicAdd((unsigned long long*)&Q[n00 + 1], (unsigned long long)q01);
    atomicAdd((unsigned long long*)&Q[n00 + W + 1], (unsigned long long)q11);
}

// Cubic shapes: the 16 node charges of one particle (rint(W w) for 15, the
// last the remainder) into the ghosted grid Qx.
__device__ __forceinline__ void deposit16(const DevInst& I, long long* Qx, double r, double z, long long Wq) {
    int i0, j0;
    double fr, fz, wr[4], dwr[4], wz[4], dwz[4];
    base3((r - I.a) / I.dr, I.nr, i0, fr);
    base3(z / I.dz, I.nz, j0, fz);
    bspline3(fr, wr, dwr);
    bspline3(fz, wz, dwz);
    const int WX = I.nz + 3;
    const double Wd = (double)Wq;
    long long sum = 0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const long long q = (a == 3 && b == 3) ? Wq - sum : (long long)rint(Wd * (wr[a] * wz[b]));
            sum += q;
            atomicAdd((unsigned long long*)&Qx[(long long)(i0 + a) * WX + (j0 + b)], (unsigned long long)q);
        }
}

__global__ void __launch_bounds__(kBlock) k_deposit64(DevInst I, P64 p, long long* __restrict__ Q,
                                                     long long* __restrict__ Qw, long long* __restrict__ Qx,
                                                     long long* cnt) {
    long long n = cnt[C_SLOTS] + cnt[C_SPAWN];
    if (n > I.p_cap) n = I.p_cap;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        double r = p.r[q];
        if (r < 0.0) continue;
        Shape sh = shape64(I, r, p.z[q]);
        double wq = p.w[q] * I.two_S;
        long long Wq = (long long)rint(wq);
        if (wq > 2147483648.0) atomicMax((unsigned long long*)&cnt[C_OVERFLOW], 1ull);
        deposit4(Q, sh, I.W, Wq);
        if (Qw) {
            // the band charge, on the particle's own shape grid
            const double g = ins_g(I, r, p.z[q]);
            if (g < I.ins_gam) {
                const long long Wb = (long long)rint((double)Wq * (ins_w(I, g) - 1.0));
                if (Qx) deposit16(I, Qw, r, p.z[q], Wb);
                else deposit4(Qw, sh, I.W, Wb);
            }
        }
        if (Qx) deposit16(I, Qx, r, p.z[q], Wq);
    }
}

// Out-of-place removal of dead slots (order not kept; results do not depend
// on particle order).
__global__ void k_compact64(P64 src, P64 dst, const long long* cnt, unsigned long long* out_n) {
    const long long n = cnt[C_SLOTS];
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        double r = src.r[q];
        if (r < 0.0) continue;
        unsigned long long d = atomicAdd(out_n, 1ull);
        dst.r[d] = r;
        dst.z[d] = src.z[q];
        dst.vr[d] = src.vr[q];
        dst.vt[d] = src.vt[q];
        dst.vz[d] = src.vz[q];
        dst.w[d] = src.w[q];
        dst.key[d] = src.key[q];
    }
}

unsigned int grid_for(long long cap) {
    long long g = (cap + kBlock - 1) / kBlock;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return (unsigned int)g;
}

}  // namespace

hipError_t launch_load64(const DevInst& I, const pic_instance_cfg& c, P64 p, long long n,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    double sv = sqrt((c.T_init_eV * kE) / kMe);
    hipLaunchKernelGGL(k_load64, dim3(grid_for(n)), dim3(kBlock), 0, s, I, c.r_lo, c.r_hi, c.z_lo,
                       c.z_hi, sv, c.weight, c.load_mode, p, n);
    return hipGetLastError();
}

hipError_t launch_push64(const DevInst& I, P64 p, const double* Er, const double* Ez,
                         const double* Br, const double* Bz, const double* cx, long long* cnt, long long grid_cap,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_push64, dim3(grid_for(grid_cap)), dim3(kBlock), 0, s, I, p, Er, Ez, Br, Bz,
                       I.spline3 ? cx : nullptr, cnt);
    return hipGetLastError();
}

hipError_t launch_mcc64(const DevInst& I, P64 p, long long* cnt, long long grid_cap,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_mcc64, dim3(grid_for(grid_cap)), dim3(kBlock), 0, s, I, p, cnt);
    return hipGetLastError();
}

hipError_t launch_source64(const DevInst& I, P64 p, long long* cnt, hipStream_t s) {
    const long long most = (long long)ceil(I.src_rate) + 1;
    hipLaunchKernelGGL(k_source64, dim3(grid_for(most)), dim3(kBlock), 0, s, I, p, cnt);
    return hipGetLastError();
}

hipError_t launch_moments64(const DevInst& I, P64 p, const long long* cnt, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(k_moments64, dim3(grid_for(I.p_cap)), dim3(kBlock), 0, s, I, p, cnt, acc);
    return hipGetLastError();
}

hipError_t launch_deposit64(const DevInst& I, P64 p, long long* Q, long long* Qw, long long* Qx, long long* cnt,
                            long long grid_cap, hipStream_t s) {
    hipLaunchKernelGGL(k_deposit64, dim3(grid_for(grid_cap)), dim3(kBlock), 0, s, I, p, Q, I.has_ins ? Qw : nullptr,
                       I.spline3 ? Qx : nullptr, cnt);
    return hipGetLastError();
}


hipError_t launch_compact64(const DevInst& I, P64 src, P64 dst, long long* cnt,
                            long long* tmp_count, long long grid_cap, hipStream_t s) {
    (void)I;
    hipLaunchKernelGGL(k_compact64, dim3(grid_for(grid_cap)), dim3(kBlock), 0, s, src, dst, cnt,
                       (unsigned long long*)tmp_count);
    return hipGetLastError();
}

}  // namespace pic
