// fp32.hip -- the batched FP32 form of the particle loop.
//
// Layout: all instances share one SoA FP32 particle store (r, z, vr, vt, vz,
// w as float, key as uint64); instance k owns slots [p_off, p_off + p_cap).
// Two such stores are kept; the tile sort scatters from one to the other.
// After a sort an instance's slots hold its live particles grouped by tile
// (a TR x TZ block of cells); electrons created since the sort sit after them
// (the tail).
//
// One step is a fixed launch sequence (captured once as a HIP graph):
//   zero Q -> plan tail work -> particle kernel -> FP64 field solve -> sample
//   -> commit
// and every K steps the tile sort (count -> plan -> scatter -> commit).
//
// The particle kernel is persistent and statically balanced: workgroup w
// takes the w-th of gridDim.x equal ranges of the step's tile-sorted
// particles of all instances and walks the tile segments the range covers,
// then the w-th of gridDim.x equal ranges of the instances' tails.  For a tile segment it stages the tile's field
// window (tile plus `halo` cells, float4 {Er, Ez, Br, Bz} per node) in LDS,
// accumulates the segment's charge in an LDS int64 window, then flushes
// non-zero window nodes to the global grid with int64 atomics.  Integer sums do not depend on
// order, so the deposited grid is the same for any schedule.  Per particle:
// coalesced SoA loads, bilinear gather, Boris, cylindrical remap, absorbing
// walls, one Philox4x32-10 block for the null-collision test (an integer
// compare on the top 52 bits, the same decision the FP64 form takes), rarely
// an elastic or ionising collision, fixed-point deposit, coalesced stores.
#include <string.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fp32.h"

// Contraction is off in this file and fused multiply-adds are written out:
// every instantiation of the particle kernel then evaluates each particle's
// update with the same operations, so results do not depend on which kernel
// variant (plain, counting, scattering) advanced a particle.
#pragma clang fp contract(off)

using namespace pic;

namespace {

constexpr int kWG = 256;
// workgroup of the particle kernel: 16 waves share one LDS window, so large
// windows (wide halos) still leave room for 8 waves per SIMD
constexpr int kPWG = 1024;

// LDS-qualified pointers: loads and atomics through them compile to ds_*
// instructions even where a global fallback path sits next to them.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4f lds_float4;
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(1))) const float gbl_f32;

__device__ __forceinline__ void lds_add(lds_u64* p, unsigned long long v) {
    __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}

// Global-qualified views of device pointers read from tables.
typedef __attribute__((address_space(1))) const v4f gbl_v4f;
typedef __attribute__((address_space(1))) unsigned long long gbl_u64;

__device__ __forceinline__ gbl_v4f* as_gbl(const float4* p) { return (gbl_v4f*)(const v4f*)p; }
__device__ __forceinline__ gbl_u64* as_gbl(long long* p) { return (gbl_u64*)(unsigned long long*)p; }
__device__ __forceinline__ void gbl_add(gbl_u64* p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One particle store.  Slots come in blocks of 64 (an instance's slots start
// on a block boundary); a block holds its 64 slots' values field by field:
// 64 floats each of r, z, vr, vt and vz, then the 64 keys, 1792 bytes in all.
// The values a wave reads and writes for 64 consecutive slots thus lie in
// one block instead of six arrays far apart, which streams at a markedly
// higher HBM rate on this GPU (5.5 against 4.9 TB/s for the same bytes).
// Per-particle weights, read only by instances without a common weight,
// keep an array of their own.
constexpr long long kBlkSlots = 64;
constexpr long long kBlkWords = 448;   // 4-byte words per block
constexpr long long kDynUnit = 32768;  // particles per unit of a plain step's shared last part
constexpr long long kBlkBytes = 4 * kBlkWords;
struct PSet {
    unsigned int* b = nullptr;
    float* wt = nullptr;
    // first word of the block holding slot p (block indices fit 32 bits)
    __device__ __forceinline__ unsigned int* blk(long long p) const {
        return b + (unsigned long long)(unsigned int)(p >> 6) * (unsigned int)kBlkWords;
    }
    __device__ __forceinline__ float& col(long long p, int f) const {
        return *reinterpret_cast<float*>(blk(p) + (f << 6) + ((int)p & 63));
    }
    __device__ __forceinline__ float& r(long long p) const { return col(p, 0); }
    __device__ __forceinline__ float& z(long long p) const { return col(p, 1); }
    __device__ __forceinline__ float& vr(long long p) const { return col(p, 2); }
    __device__ __forceinline__ float& vt(long long p) const { return col(p, 3); }
    __device__ __forceinline__ float& vz(long long p) const { return col(p, 4); }
    __device__ __forceinline__ float& w(long long p) const { return wt[p]; }
    __device__ __forceinline__ unsigned long long& key(long long p) const {
        return *reinterpret_cast<unsigned long long*>(blk(p) + 320 + (((int)p & 63) << 1));
    }
};


// control block: [0] units of the shared last part handed out this step
// (plain steps), [1] particles to push this step (sorted + tails), [2] sorted
// particles over all instances, [3] collision events queued this step,
// [4] queue overflow flag, [5 .. 5+n_inst] prefix of the instances' tail counts

struct KArgs {
    const DevInst* It;
    const FieldDev* Ft;
    long long* cnt;
    PSet p;                        // input store
    PSet out;                      // output store of a scatter step
    const long long* vtile;        // prefix of sorted particles over all tiles (n_tiles + 1)
    const int4* tile_info;         // instance, tile row, tile column
    long long* ctl;
    unsigned int* cnt_out;         // per-tile totals being counted (COUNT)
    unsigned int* tile_fill;       // per-tile ranks handed out (SCATTER)
    const long long* tile_start;   // first slot of each tile in the input store
    const long long* tile_dst;     // first slot of each tile in the output store (SCATTER)
    const long long* new_base;     // per instance: slots of the sorted output
    unsigned long long* queue;     // real collision events: (instance << 40) | slot
    long long qcap;
    unsigned int* crec;            // per (workgroup, chunk): survivors per neighbouring tile, from COUNT
    int crec_max;                  // chunks per workgroup with a record
    int n_inst, n_tiles, TR, TZ, halo, C, win_max;
    int win3_max;                  // ghosted cubic window nodes (even; 0 without cubic shapes)
};

// ---- shared device helpers ------------------------------------------------

// Weight of the particle in slot p: the instance's common weight when it has
// one, else the per-particle array.
__device__ __forceinline__ float weight_at(const DevInst& I, const PSet& P, long long p) {
    return I.w_uni != 0.0f ? I.w_uni : P.w(p);
}

__device__ __forceinline__ void cell_of(const DevInst& I, float r, float z, int& i, int& j, float& fr,
                                        float& fz) {
    float s = (r - I.a_f) * I.inv_dr_f;
    float t = z * I.inv_dz_f;
    float si = floorf(s), tj = floorf(t);
    i = (int)si;
    j = (int)tj;
    i = i < 0 ? 0 : (i > I.nr - 1 ? I.nr - 1 : i);
    j = j < 0 ? 0 : (j > I.nz - 1 ? I.nz - 1 : j);
    fr = s - (float)i;
    fz = t - (float)j;
}

// The collision constants of an instance the event decision reads (FP32),
// copied once per chunk in the particle kernel.
struct EvConst {
    float half_me_over_e, nsig_el, iz_I, lotz_aq, n_n, nu_prime;
    int xs_n;
};

__device__ __forceinline__ EvConst ev_const(const DevInst& I) {
    EvConst c;
    c.half_me_over_e = I.half_me_over_e_f; c.nsig_el = I.nsig_el_f; c.iz_I = I.iz_I_f;
    c.lotz_aq = I.lotz_aq_f; c.n_n = I.n_n_f; c.nu_prime = I.nu_prime_f; c.xs_n = I.xs_n;
    return c;
}

// Per-chunk copy of the instance constants the particle loop reads, kept in
// registers so stores to the particle arrays never force them to be reloaded.
struct LocalInst {
    float a, b, L, inv_dr, inv_dz, h, dt, v_cap2, two_S, w_uni;
    float ins_r0, ins_z0, ins_inv_er, ins_inv_ez, ins_gam;
    int nr, nz, W, ntz, tile_off, collisions, has_ins;
    unsigned int seed_lo, seed_hi;
    unsigned long long null_k;
};

// The instance table seen through the constant address space: a field read
// with a wave-uniform index becomes a scalar load, so rare paths can fetch
// instance constants when they need them instead of holding them in
// registers across the particle loop.
// The empty asm keeps the index (and so the load) where it is written: the
// compiler would otherwise hoist the invariant load out of the loop and hold
// its value in a register for the whole chunk.
typedef __attribute__((address_space(4))) const DevInst cDevInst;
__device__ __forceinline__ cDevInst* const_inst(const DevInst* It, int k) {
    asm volatile("" : "+s"(k));
    return (cDevInst*)(const __attribute__((address_space(1))) DevInst*)It + k;
}
typedef __attribute__((address_space(4))) const FieldDev cFieldDev;
__device__ __forceinline__ cFieldDev* const_field(const FieldDev* Ft, int k) {
    asm volatile("" : "+s"(k));
    return (cFieldDev*)(const __attribute__((address_space(1))) FieldDev*)Ft + k;
}

__device__ __forceinline__ float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ __forceinline__ LocalInst local_inst(const DevInst& I) {
    LocalInst L;
    L.a = uniform_f(I.a_f); L.b = uniform_f(I.b_f); L.L = uniform_f(I.L_f);
    L.inv_dr = uniform_f(I.inv_dr_f); L.inv_dz = uniform_f(I.inv_dz_f);
    L.h = uniform_f(I.h_f); L.dt = uniform_f(I.dt_f); L.v_cap2 = uniform_f(I.v_cap2_f);
    L.two_S = uniform_f((float)I.two_S);
    L.w_uni = uniform_f(I.w_uni);
    L.ins_r0 = uniform_f(I.ins_r0_f); L.ins_z0 = uniform_f(I.ins_z0_f);
    L.ins_inv_er = uniform_f(I.ins_inv_er_f); L.ins_inv_ez = uniform_f(I.ins_inv_ez_f);
    L.ins_gam = uniform_f(I.ins_gam_f);
    L.has_ins = __builtin_amdgcn_readfirstlane(I.has_ins);
    L.nr = __builtin_amdgcn_readfirstlane(I.nr); L.nz = __builtin_amdgcn_readfirstlane(I.nz);
    L.W = __builtin_amdgcn_readfirstlane(I.W); L.ntz = __builtin_amdgcn_readfirstlane(I.ntz);
    L.tile_off = __builtin_amdgcn_readfirstlane(I.tile_off);
    L.collisions = __builtin_amdgcn_readfirstlane(I.collisions);
    L.seed_lo = __builtin_amdgcn_readfirstlane(I.seed_lo);
    L.seed_hi = __builtin_amdgcn_readfirstlane(I.seed_hi);
    const unsigned long long k = I.null_k;
    L.null_k = ((unsigned long long)(unsigned int)__builtin_amdgcn_readfirstlane((int)(k >> 32)) << 32) |
               (unsigned long long)(unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)k);
    return L;
}

__device__ __forceinline__ void cell_of(const LocalInst& I, float r, float z, int& i, int& j, float& fr,
                                        float& fz) {
    float s = (r - I.a) * I.inv_dr;
    float t = z * I.inv_dz;
    i = (int)floorf(s);
    j = (int)floorf(t);
    i = i < 0 ? 0 : (i > I.nr - 1 ? I.nr - 1 : i);
    j = j < 0 ? 0 : (j > I.nz - 1 ? I.nz - 1 : j);
    fr = s - (float)i;
    fz = t - (float)j;
}

// Philox4x32-10 for the particle loop: the same rounds as philox4x32_10, but
// the key schedule (the Weyl sequence k + r W) is stepped on the scalar unit
// inside the loop instead of being held as twenty loop-invariant registers,
// which the particle kernel cannot afford next to its other uniform values.
// k0, k1 must be wave-uniform.
__device__ __forceinline__ uint4 philox_hot(uint4 c, unsigned int k0, unsigned int k1) {
    const unsigned int M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const unsigned int W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        asm volatile("" : "+s"(k0), "+s"(k1));
        const unsigned long long p0 = (unsigned long long)M0 * c.x;
        const unsigned long long p1 = (unsigned long long)M1 * c.z;
        c = make_uint4((unsigned int)(p1 >> 32) ^ c.y ^ k0, (unsigned int)p1,
                       (unsigned int)(p0 >> 32) ^ c.w ^ k1, (unsigned int)p0);
        k0 += W0;
        k1 += W1;
    }
    return c;
}

__device__ __forceinline__ uint4 philox_step(const DevInst& I, unsigned long long key, unsigned int step,
                                             unsigned int b) {
    return philox4x32_10(make_uint4((unsigned int)key, (unsigned int)(key >> 32), step, b), I.seed_lo,
                         I.seed_hi);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ void flush_counter(long long* slot, unsigned long long v) {
    if (__ballot(v != 0ull) == 0ull) return;
    v = wave_sum(v);
    if (__lane_id() == 0) atomicAdd((unsigned long long*)slot, v);
}

// Anisotropy of the scattering law for an electron of energy E (eV), FP32:
// the table xi(E) when the instance has one, else the constant okh_xi.
__device__ __forceinline__ float xi_at_f(const DevInst& I, float E) {
    if (I.xi_n > 0) return xs_interp(I.xi_n, I.xi_Ef, I.xi_vf, E);
    if (I.okh_inv_E0_f > 0.0f) {
        // screened-Coulomb xi(E) = 4 e / (1 + 4 e), e = E / E0
        const float e4 = 4.0f * (E * I.okh_inv_E0_f);
        return e4 / (1.0f + e4);
    }
    return I.okh_xi_f;
}

__device__ __forceinline__ float okh_cos_f(float xi, float u) {
    return ((2.0f * u + xi) - 1.0f) / ((1.0f - xi) + (2.0f * xi) * u);
}

__device__ __forceinline__ void scatter_f(float ur, float ut, float uz, float cosx, float phi, float* o) {
    float e1r, e1t, e1z;
    if (fabsf(uz) < 0.99f) {
        float nn = rsqrtf(ur * ur + ut * ut);
        e1r = -ut * nn; e1t = ur * nn; e1z = 0.0f;
    } else {
        float nn = rsqrtf(uz * uz + ut * ut);
        e1r = 0.0f; e1t = -uz * nn; e1z = ut * nn;
    }
    float e2r = ut * e1z - uz * e1t;
    float e2t = uz * e1r - ur * e1z;
    float e2z = ur * e1t - ut * e1r;
    float sinx = sqrtf(fmaxf(0.0f, 1.0f - cosx * cosx));
    float sp, cp;
    sincosf(phi, &sp, &cp);
    o[0] = cosx * ur + sinx * (cp * e1r + sp * e2r);
    o[1] = cosx * ut + sinx * (cp * e1t + sp * e2t);
    o[2] = cosx * uz + sinx * (cp * e1z + sp * e2z);
}

// Which process a null-collision candidate undergoes at its post-push
// velocity (FP32): the process uniform scaled by nu' against nu_el and
// nu_el + nu_iz.  Returns 0 null, 1 elastic, 2 ionisation, with the speed and
// energy it used.  The particle kernel calls it to queue only real events;
// the collision kernel calls it again on the same stored velocity, so both
// take the same decision.  I supplies the cross-section tables only.
template <class INST>
__device__ __forceinline__ int event_kind_f(const EvConst& c, const INST& I, unsigned int bits, float vr,
                                            float vt, float vz, float& v, float& E) {
    const float u_proc = u23(bits);
    const float v2 = (vr * vr + vt * vt) + vz * vz;
    v = sqrtf(v2);
    E = v2 * c.half_me_over_e;
    float nu_el, sig = 0.0f;
    if (c.xs_n > 0) {
        nu_el = (c.n_n * xs_interp(c.xs_n, I.xs_Ef, I.xs_elf, E)) * v;
        if (E > c.iz_I) sig = xs_interp(c.xs_n, I.xs_Ef, I.xs_izf, E);
    } else {
        nu_el = c.nsig_el * v;
        if (E > c.iz_I) sig = (c.lotz_aq * logf(E / c.iz_I)) / (E * c.iz_I);
    }
    const float nu_iz = (c.n_n * sig) * v;
    const float R = u_proc * c.nu_prime;
    if (R < nu_el) return 1;
    if (R < nu_el + nu_iz) return 2;
    return 0;
}

// The event of a queued candidate.  Returns 0 null, 1 elastic, 2
// ionisation; sets the parent's new velocity and, for an ionisation, the new
// electron's velocity and key.
__device__ __forceinline__ int collide_f(const DevInst& I, unsigned long long key, unsigned int step, uint4 b0,
                                      float& vr, float& vt, float& vz, float& cvr, float& cvt, float& cvz,
                                      unsigned long long& ckey) {
    float v, E;
    const int ev = event_kind_f(ev_const(I), I, b0.z, vr, vt, vz, v, E);
    if (ev == 0) return 0;
    float inv_v = 1.0f / v;
    float ur = vr * inv_v, ut = vt * inv_v, uz = vz * inv_v;
    uint4 b1 = philox_step(I, key, step, 1u);
    float phi1 = 6.28318530717958648f * u23(b1.z);
    float dir[3];
    if (ev == 1) {
        const float cos1 = okh_cos_f(xi_at_f(I, E), u23(b1.x));
        float En = E * (1.0f - I.mass_ratio2_f * (1.0f - cos1));
        float vn = sqrtf(En * I.two_e_over_me_f);
        scatter_f(ur, ut, uz, cos1, phi1, dir);
        vr = vn * dir[0]; vt = vn * dir[1]; vz = vn * dir[2];
        return 1;
    }
    uint4 b2 = philox_step(I, key, step, 2u);
    uint4 b3 = philox_step(I, key, step, 3u);
    float E_av = E - I.iz_I_f;
    float E_s = I.opal_Ebar_f * tanf(u23(b2.x) * atanf(E_av / (2.0f * I.opal_Ebar_f)));
    float E_p = E_av - E_s;
    const float cos1 = okh_cos_f(xi_at_f(I, E_p), u23(b1.x));
    float cos2 = okh_cos_f(xi_at_f(I, E_s), u23(b2.z));
    float phi2 = 6.28318530717958648f * u23(b3.x);
    float vp = sqrtf(fmaxf(E_p, 0.0f) * I.two_e_over_me_f);
    float vs = sqrtf(fmaxf(E_s, 0.0f) * I.two_e_over_me_f);
    scatter_f(ur, ut, uz, cos1, phi1, dir);
    vr = vp * dir[0]; vt = vp * dir[1]; vz = vp * dir[2];
    scatter_f(ur, ut, uz, cos2, phi2, dir);
    cvr = vs * dir[0]; cvt = vs * dir[1]; cvz = vs * dir[2];
    ckey = ((((unsigned long long)b3.z) << 32) | (unsigned long long)b3.w) | (1ull << 63);
    return 2;
}

// Fixed-point charges of one particle with bilinear weights from (fr, fz):
// W = rint(w 2^S) (exact: a power-of-two scaling of w), three nodes take
// rint(W w_k) (FP32 product), the fourth the remainder, so every particle
// adds exactly W.
__device__ __forceinline__ void node_charges(float w, float two_S, float fr, float fz, long long& q00,
                                             long long& q10, long long& q01, long long& q11) {
    const float Wf = rintf(w * two_S);
    const float gr = 1.0f - fr, gz = 1.0f - fz;
    const unsigned int Wu = (unsigned int)Wf;
    const unsigned int a = (unsigned int)rintf(Wf * (gr * gz));
    const unsigned int b = (unsigned int)rintf(Wf * (fr * gz));
    const unsigned int c = (unsigned int)rintf(Wf * (gr * fz));
    q00 = (long long)a;
    q10 = (long long)b;
    q01 = (long long)c;
    q11 = (long long)Wu - (long long)a - (long long)b - (long long)c;
}

// Elliptic insert in FP32: g <= 0 in the metal; in the weight function's
// band (0 < g < gam) a particle adds its charge times (w(x_p) - 1) to Qw,
// rint(W (w - 1)) split over the four nodes by the same exact-sum rule (over
// the sixteen nodes of the ghosted grid with cubic shapes).
__device__ __forceinline__ float ins_g_f(const DevInst& I, float r, float z) {
    const float u = (r - I.ins_r0_f) * I.ins_inv_er_f, v = (z - I.ins_z0_f) * I.ins_inv_ez_f;
    return fmaf(u, u, v * v) - 1.0f;
}

__device__ __forceinline__ void bspline3_f(float f, float w[4], float dw[4]);
__device__ __forceinline__ void band_cubic_gbl(long long* Qx, int WX, int i, int j, float Wt, float fr, float fz);

__device__ __forceinline__ void deposit_qw(const DevInst& I, long long* Qw, float w, float r, float z) {
    const float g = ins_g_f(I, r, z);
    if (!(g < I.ins_gam_f)) return;
    float s = 1.0f - g / I.ins_gam_f;
    s = g <= 0.0f ? 1.0f : s;
    const float wp = 1.0f - s * s * s;
    const float Wt = rintf(rintf(w * (float)I.two_S) * (wp - 1.0f));
    int i, j;
    float fr, fz;
    cell_of(I, r, z, i, j, fr, fz);
    if (I.spline3) {
        band_cubic_gbl(Qw, I.nz + 3, i, j, Wt, fr, fz);
        return;
    }
    const float gr = 1.0f - fr, gz = 1.0f - fz;
    const long long a = (long long)rintf(Wt * (gr * gz));
    const long long b = (long long)rintf(Wt * (fr * gz));
    const long long c = (long long)rintf(Wt * (gr * fz));
    const long long d = (long long)Wt - a - b - c;
    unsigned long long* Q = (unsigned long long*)Qw;
    const long long n00 = (long long)i * I.W + j;
    atomicAdd(&Q[n00], (unsigned long long)a);
    atomicAdd(&Q[n00 + I.W], (unsigned long long)b);
    atomicAdd(&Q[n00 + 1], (unsigned long long)c);
    atomicAdd(&Q[n00 + I.W + 1], (unsigned long long)d);
}

// One atomic per distinct key among the active lanes of the wave (the key's
// lanes add their count at once); with RET each lane gets its rank: the
// returned base plus its position among the lanes sharing the key.  Every
// lane of the wave must call it.
template <bool RET, typename F>
__device__ __forceinline__ unsigned int wave_aggregate(bool act, int key, F&& add) {
    const int lane = __lane_id();
    unsigned long long todo = __ballot(act);
    unsigned int rank = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int k = __shfl(key, leader);
        const unsigned long long m = __ballot(act && key == k) & todo;
        unsigned int base = 0;
        if (lane == leader) base = add(k, (unsigned int)__popcll(m));
        if (RET) {
            base = __shfl(base, leader);
            if ((m >> lane) & 1ull) rank = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
        }
        todo &= ~m;
    }
    return rank;
}

// LDS queue of the real collision events per workgroup and chunk
constexpr int kLQ = 512;

// chunk-level event counters kept in LDS and their device counter slots
enum {
    SC_ABS_N = 0, SC_ABS_W = 4, SC_DEAD = 8, SC_CAND = 9, SC_CAP = 10, SC_FAR = 11, SC_EL = 12, SC_IZ = 13,
    SC_NONFIN = 14, SC_N = 15
};
__constant__ int kCounterOf[SC_N] = {C_ABS_N,     C_ABS_N + 1, C_ABS_N + 2, C_ABS_N + 3, C_ABS_W,   C_ABS_W + 1,
                                     C_ABS_W + 2, C_ABS_W + 3, C_DEAD,      C_CAND,      C_CAPOVER, C_FARDEP,
                                     C_ELASTIC,   C_IONIZ,     C_NONFIN};


// Cubic B-spline weights of the nodes i-1 .. i+2 at offset f in [0, 1) from
// i, and their derivatives in units of the cell (FP32).
__device__ __forceinline__ void bspline3_f(float f, float w[4], float dw[4]) {
    const float g = 1.0f - f;
    w[0] = (g * g * g) / 6.0f;
    w[1] = fmaf(fmaf(3.0f, f, -6.0f) * f, f, 4.0f) / 6.0f;
    w[2] = fmaf(fmaf(fmaf(-3.0f, f, 3.0f), f, 3.0f), f, 1.0f) / 6.0f;
    w[3] = (f * f * f) / 6.0f;
    dw[0] = -(g * g) / 2.0f;
    dw[1] = (fmaf(3.0f, f, -4.0f) * f) / 2.0f;
    dw[2] = fmaf(fmaf(-3.0f, f, 2.0f), f, 1.0f) / 2.0f;
    dw[3] = (f * f) / 2.0f;
}

// Fixed-point cubic charges of one particle whose cell is (i, j) with
// offsets (fr, fz): the node (i-1+a, j-1+b) takes rint(W w_a w_b) for fifteen
// nodes and the remainder for the last, so the particle adds exactly W.
// add(a, b, q) receives them.
template <typename F>
__device__ __forceinline__ void cubic_charges(float w, float two_S, float fr, float fz, F&& add) {
    float wr[4], dwr[4], wz[4], dwz[4];
    bspline3_f(fr, wr, dwr);
    bspline3_f(fz, wz, dwz);
    const float Wf = rintf(w * two_S);
    long long sum = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const long long q = (a == 3 && b == 3) ? (long long)(unsigned int)Wf - sum
                                                   : (long long)(unsigned int)rintf(Wf * (wr[a] * wz[b]));
            sum += q;
            add(a, b, q);
        }
}

// The same charges into the ghosted grid of the device (new electrons and
// particles outside the LDS window).
__device__ __forceinline__ void deposit_cubic_gbl(long long* Qx, int WX, int i, int j, float w, float two_S,
                                                  float fr, float fz) {
    gbl_u64* Q = as_gbl(Qx);
    cubic_charges(w, two_S, fr, fz, [&](int a, int b, long long q) {
        gbl_add(&Q[(long long)(i + a) * WX + (j + b)], (unsigned long long)q);
    });
}

// The band charge Wt = rint(W (w - 1)) (negative) of a particle whose cell
// is (i, j) with offsets (fr, fz) into the ghosted grid: rint(Wt w_a w_b) for
// fifteen nodes, the remainder for the last.
__device__ __forceinline__ void band_cubic_gbl(long long* Qx, int WX, int i, int j, float Wt, float fr, float fz) {
    float wr[4], dwr[4], wz[4], dwz[4];
    bspline3_f(fr, wr, dwr);
    bspline3_f(fz, wz, dwz);
    gbl_u64* Q = as_gbl(Qx);
    const long long total = (long long)Wt;
    long long sum = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const long long q = (a == 3 && b == 3) ? total - sum : (long long)rintf(Wt * (wr[a] * wz[b]));
            sum += q;
            gbl_add(&Q[(long long)(i + a) * WX + (j + b)], (unsigned long long)q);
        }
}

// Everything the particle loop needs about the current chunk.
struct ChunkCtx {
    LocalInst L;
    lds_float4* sEB;
    lds_u64* sQ;
    unsigned long long* s_ctr;
    unsigned int* s_bcnt;
    const unsigned int* s_bbase;
    unsigned int* s_ccnt;
    unsigned int* s_qn;
    unsigned long long* s_q;
    PSet out;
    const float4* EB;
    long long* Q;
    long long* Qw;
    int inst, ti_c, tj_c, i0, i1, j0, j1, ww;
    bool win;
    unsigned int step;
    // cubic shapes: the ghosted coefficient and charge windows (rows of ww + 2
    // nodes from ghosted node (i0, j0)) and the device arrays (rows of WX)
    lds_f32* sC;
    lds_u64* sQx;
    const float* cxf;
    long long* Qx;
    int WX;
};

// One particle: (optional) sort destination, gather, Boris, remap, walls,
// null-collision test, store, deposit, (optional) destination-tile count.
// Every lane of the wave calls it (collectives inside).
template <bool COUNT, bool SCATTER, bool INS, bool CUB>
__device__ __forceinline__ void push_particle(const KArgs& A, const ChunkCtx& X, long long p, bool inr, float r,
                                              float z, float vr, float vt, float vz, float w,
                                              unsigned long long key, unsigned int& c_push) {
    const LocalInst& L = X.L;
    const float h = L.h, dt = L.dt;
    const bool live = inr && r >= 0.0f;
    // The arithmetic runs on every lane (cell indices are clamped, so every
    // address stays inside the mesh); only side effects depend on `live`.
    // Every loaded field thus has an unconditional use and the loads issue
    // together instead of waiting on the liveness test.
    int i, j;
    float fr, fz;
    cell_of(L, r, z, i, j, fr, fz);
    long long dst = p;
    if (SCATTER) {
        const int dti = i / A.TR, dtj = j / A.TZ;
        const int dr = dti - X.ti_c, dz = dtj - X.tj_c;
        const bool near = X.win && dr >= -1 && dr <= 1 && dz >= -1 && dz <= 1;
        const int bkt = near ? (dr + 1) * 3 + (dz + 1) : -1;
        const int tile = L.tile_off + dti * L.ntz + dtj;
        unsigned int* s_bcnt = X.s_bcnt;
        const unsigned int rn = wave_aggregate<true>(live && near, bkt, [&](int k, unsigned int n) {
            return atomicAdd(&s_bcnt[k], n);
        });
        const unsigned int rf = wave_aggregate<true>(live && !near, tile, [&](int k, unsigned int n) {
            return atomicAdd(&A.tile_fill[k], n);
        });
        if (live) dst = A.tile_dst[tile] + (long long)(near ? X.s_bbase[bkt] + rn : rf);
    }
    // gather (LDS window when the cell is inside it)
    const bool inwin = X.win && i >= X.i0 && i + 1 <= X.i1 && j >= X.j0 && j + 1 <= X.j1;
    v4f f00, f10, f01, f11;
    if (inwin) {
        const int li = (i - X.i0) * X.ww + (j - X.j0);
        f00 = X.sEB[li]; f01 = X.sEB[li + 1]; f10 = X.sEB[li + X.ww]; f11 = X.sEB[li + X.ww + 1];
    } else {
        gbl_v4f* G = as_gbl(const_field(A.Ft, X.inst)->EB);
        const long long n00 = (long long)i * L.W + j;
        f00 = G[n00]; f01 = G[n00 + 1]; f10 = G[n00 + L.W]; f11 = G[n00 + L.W + 1];
    }
    const float gr = 1.0f - fr, gz = 1.0f - fz;
    const float w00 = gr * gz, w10 = fr * gz, w01 = gr * fz, w11 = fr * fz;
    float er = fmaf(w11, f11.x, fmaf(w01, f01.x, fmaf(w10, f10.x, w00 * f00.x)));
    float ez = fmaf(w11, f11.y, fmaf(w01, f01.y, fmaf(w10, f10.y, w00 * f00.y)));
    if (CUB) {
        // cubic shapes: the nodal field is the vacuum field; add the space
        // charge's -grad of the cubic expansion at the particle
        float wr[4], dwr[4], wz[4], dwz[4];
        bspline3_f(fr, wr, dwr);
        bspline3_f(fz, wz, dwz);
        float gr3 = 0.0f, gz3 = 0.0f, u3 = 0.0f;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            float c[4];
            if (inwin) {
                const int l = (i - X.i0 + a) * (X.ww + 2) + (j - X.j0);
#pragma unroll
                for (int b = 0; b < 4; ++b) c[b] = X.sC[l + b];
            } else {
                gbl_f32* C = (gbl_f32*)X.cxf;
                const long long n = (long long)(i + a) * X.WX + j;
#pragma unroll
                for (int b = 0; b < 4; ++b) c[b] = C[n + b];
            }
            const float sz = fmaf(c[3], wz[3], fmaf(c[2], wz[2], fmaf(c[1], wz[1], c[0] * wz[0])));
            const float dz = fmaf(c[3], dwz[3], fmaf(c[2], dwz[2], fmaf(c[1], dwz[1], c[0] * dwz[0])));
            gr3 = fmaf(dwr[a], sz, gr3);
            gz3 = fmaf(wr[a], dz, gz3);
            if (INS) u3 = fmaf(wr[a], sz, u3);
        }
        if (INS && L.has_ins) {
            // web-splines: phi_sc = w u, so E = w (-grad u) - u grad w, with
            // w = 1 - (1 - g/gam)^3 and its gradient inside the band
            float e3r = -gr3 * L.inv_dr, e3z = -gz3 * L.inv_dz;
            const float gu = (r - L.ins_r0) * L.ins_inv_er, gv = (z - L.ins_z0) * L.ins_inv_ez;
            const float g = fmaf(gu, gu, gv * gv) - 1.0f;
            if (g < L.ins_gam) {
                const float s = 1.0f - g / L.ins_gam;
                const bool in = g > 0.0f;
                const float wv = in ? 1.0f - s * s * s : 0.0f;
                const float d = in ? 3.0f * s * s / L.ins_gam : 0.0f;
                const float gwr = d * (2.0f * gu * L.ins_inv_er), gwz = d * (2.0f * gv * L.ins_inv_ez);
                e3r = fmaf(wv, e3r, -u3 * gwr);
                e3z = fmaf(wv, e3z, -u3 * gwz);
            }
            er += e3r;
            ez += e3z;
        } else {
            er = fmaf(-gr3, L.inv_dr, er);
            ez = fmaf(-gz3, L.inv_dz, ez);
        }
    }
    const float br = fmaf(w11, f11.z, fmaf(w01, f01.z, fmaf(w10, f10.z, w00 * f00.z)));
    const float bz = fmaf(w11, f11.w, fmaf(w01, f01.w, fmaf(w10, f10.w, w00 * f00.w)));
    // Boris: half kick, rotation, half kick
    const float mr = fmaf(h, er, vr), mt = vt, mz = fmaf(h, ez, vz);
    const float tr = h * br, tz = h * bz;
    const float f = 2.0f * __builtin_amdgcn_rcpf(fmaf(tr, tr, fmaf(tz, tz, 1.0f)));
    const float sr = f * tr, sz = f * tz;
    const float pr = fmaf(mt, tz, mr);
    const float pt = mt + fmaf(mz, tr, -(mr * tz));
    const float pz = fmaf(-mt, tr, mz);
    vr = fmaf(h, er, fmaf(pt, sz, mr));
    vt = mt + fmaf(pz, sr, -(pr * sz));
    vz = fmaf(h, ez, fmaf(-pt, sr, mz));
    // move in the Cartesian frame, rotate back to (r, z)
    const float x = fmaf(vr, dt, r), y = vt * dt;
    const float zn = fmaf(vz, dt, z);
    const float rr2 = fmaf(x, x, y * y);
    const float inv = __builtin_amdgcn_rsqf(rr2);
    const float rn = rr2 * inv;
    // The wall that absorbs the particle, by priority: a non-finite new
    // position (a non-finite field or velocity; removed, not counted as
    // absorbed charge) before the inner electrode (x = y = 0 gives rn NaN
    // from 0 * inf: inner), the outer one, the insert (outer-electrode
    // metal), then the ends.  Written as selects, lowest priority first.
    int wall = -1;
    wall = zn >= L.L ? 3 : wall;
    wall = zn <= 0.0f ? 2 : wall;
    if (INS && L.has_ins)
        wall = fmaf((rn - L.ins_r0) * L.ins_inv_er, (rn - L.ins_r0) * L.ins_inv_er,
                    ((zn - L.ins_z0) * L.ins_inv_ez) * ((zn - L.ins_z0) * L.ins_inv_ez)) - 1.0f <= 0.0f
                   ? 1
                   : wall;
    wall = rn >= L.b ? 1 : wall;
    wall = !(rn > L.a) ? 0 : wall;
    wall = !(rr2 < __builtin_inff() && fabsf(zn) < __builtin_inff()) ? 4 : wall;
    const float cs = x * inv, sn = y * inv;
    const float vrn = fmaf(cs, vr, sn * vt);
    const float vtn = fmaf(cs, vt, -(sn * vr));
    // null-collision test: one Philox block per particle-step
    const uint4 b0 = philox_hot(make_uint4((unsigned int)key, (unsigned int)(key >> 32), X.step, 0u),
                                L.seed_lo, L.seed_hi);
    const unsigned long long x52 = ((((unsigned long long)b0.x) << 32) | (unsigned long long)b0.y) >> 12;
    const PSet out = X.out;
    const bool alive = live && wall < 0;
    if (live) {
        ++c_push;
        if (wall >= 0) {
            if (wall == 4) {
                atomicAdd(&X.s_ctr[SC_NONFIN], 1ull);
            } else {
                const unsigned long long Wq = (unsigned long long)(unsigned int)rintf(w * L.two_S);
                atomicAdd(&X.s_ctr[SC_ABS_N + wall], 1ull);
                atomicAdd(&X.s_ctr[SC_ABS_W + wall], Wq);
            }
            atomicAdd(&X.s_ctr[SC_DEAD], 1ull);
            out.r(dst) = -1.0f;
        }
    }
    int ni = 0, nj = 0;
    if (alive) {
        if (fmaf(vz, vz, fmaf(vtn, vtn, vrn * vrn)) > L.v_cap2) atomicAdd(&X.s_ctr[SC_CAP], 1ull);
        if (L.collisions && x52 < L.null_k) {
            // a null-collision candidate; a real event is resolved by
            // k_collide after this kernel: into the workgroup's LDS queue
            // (flushed to the device queue once per chunk), beyond its size
            // straight to the device
            atomicAdd(&X.s_ctr[SC_CAND], 1ull);
            float sp, en;
            cDevInst* Ic = const_inst(A.It, X.inst);
            EvConst ev;
            ev.half_me_over_e = Ic->half_me_over_e_f; ev.nsig_el = Ic->nsig_el_f; ev.iz_I = Ic->iz_I_f;
            ev.lotz_aq = Ic->lotz_aq_f; ev.n_n = Ic->n_n_f; ev.nu_prime = Ic->nu_prime_f; ev.xs_n = Ic->xs_n;
            const int kind = event_kind_f(ev, *Ic, b0.z, vrn, vtn, vz, sp, en);
            if (kind != 0) {
                atomicAdd(&X.s_ctr[kind == 1 ? SC_EL : SC_IZ], 1ull);
                const unsigned int qr = atomicAdd(X.s_qn, 1u);
                const unsigned long long e = ((unsigned long long)X.inst << 40) | (unsigned long long)dst;
                if (qr < (unsigned int)kLQ) {
                    X.s_q[qr] = e;
                } else {
                    const long long qi = (long long)atomicAdd((unsigned long long*)&A.ctl[CTL_QCOUNT], 1ull);
                    if (qi < A.qcap) A.queue[qi] = e;
                    else A.ctl[CTL_QOVER] = 1;
                }
            }
        }
        out.r(dst) = rn;
        out.z(dst) = zn;
        out.vr(dst) = vrn;
        out.vt(dst) = vtn;
        out.vz(dst) = vz;
        if (SCATTER) {
            if (L.w_uni == 0.0f) out.w(dst) = w;
            out.key(dst) = key;
        }
        // deposit at the new position
        float nfr, nfz;
        cell_of(L, rn, zn, ni, nj, nfr, nfz);
        long long q00, q10, q01, q11;
        node_charges(w, L.two_S, nfr, nfz, q00, q10, q01, q11);
        if (X.win && ni >= X.i0 && ni + 1 <= X.i1 && nj >= X.j0 && nj + 1 <= X.j1) {
            const int l = (ni - X.i0) * X.ww + (nj - X.j0);
            lds_add(&X.sQ[l], (unsigned long long)q00);
            lds_add(&X.sQ[l + X.ww], (unsigned long long)q10);
            lds_add(&X.sQ[l + 1], (unsigned long long)q01);
            lds_add(&X.sQ[l + X.ww + 1], (unsigned long long)q11);
        } else {
            atomicAdd(&X.s_ctr[SC_FAR], 1ull);
            gbl_u64* Qg = as_gbl(const_field(A.Ft, X.inst)->Q);
            const long long n00 = (long long)ni * L.W + nj;
            gbl_add(&Qg[n00], (unsigned long long)q00);
            gbl_add(&Qg[n00 + L.W], (unsigned long long)q10);
            gbl_add(&Qg[n00 + 1], (unsigned long long)q01);
            gbl_add(&Qg[n00 + L.W + 1], (unsigned long long)q11);
        }
        if (CUB) {
            if (X.win && ni >= X.i0 && ni + 1 <= X.i1 && nj >= X.j0 && nj + 1 <= X.j1) {
                const int l = (ni - X.i0) * (X.ww + 2) + (nj - X.j0);
                cubic_charges(w, L.two_S, nfr, nfz, [&](int a, int b, long long q) {
                    lds_add(&X.sQx[l + a * (X.ww + 2) + b], (unsigned long long)q);
                });
            } else {
                deposit_cubic_gbl(X.Qx, X.WX, ni, nj, w, L.two_S, nfr, nfz);
            }
        }
        if (INS && L.has_ins) {
            // the band test from the chunk's copy of the insert constants (the
            // same arithmetic as ins_g_f): the instance table is read only in
            // the band
            const float gu = (rn - L.ins_r0) * L.ins_inv_er, gv = (zn - L.ins_z0) * L.ins_inv_ez;
            if (fmaf(gu, gu, gv * gv) - 1.0f < L.ins_gam) deposit_qw(A.It[X.inst], X.Qw, w, rn, zn);
        }
    }
    if (COUNT) {
        // survivors, by the tile of the new position: tiles next to the
        // chunk's own are counted in LDS and flushed once per chunk
        const int ti = ni / A.TR, tj = nj / A.TZ;
        const int dr = ti - X.ti_c, dz = tj - X.tj_c;
        const bool near = X.win && dr >= -1 && dr <= 1 && dz >= -1 && dz <= 1;
        unsigned int* s_ccnt = X.s_ccnt;
        wave_aggregate<false>(alive && near, (dr + 1) * 3 + (dz + 1), [&](int k, unsigned int n) {
            atomicAdd(&s_ccnt[k], n);
            return 0u;
        });
        wave_aggregate<false>(alive && !near, L.tile_off + ti * L.ntz + tj, [&](int k, unsigned int n) {
            atomicAdd(&A.cnt_out[k], n);
            return 0u;
        });
    }
}

// Largest t in [0, n) with a[t] <= v for a nondecreasing a with a[0] <= v,
// by one full wave: 64 probes per round narrow the range 64-fold.
__device__ __forceinline__ int wave_search(const long long* a, int n, long long v) {
    const int lane = __lane_id();
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int idx = lo + lane * step;
        const bool ok = idx < hi && a[idx] <= v;
        const unsigned long long m = __ballot(ok);
        const int last = 63 - __clzll((long long)m);
        lo = lo + last * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// ---- the particle kernel --------------------------------------------------
//
// MODE bit 0 (COUNT): after the push, count every survivor (and new
// electron) in the tile of its new position; these totals size the next
// sort.  MODE bit 1 (SCATTER): each particle's destination in the other
// store is fixed by the tile of its position at step start (the totals of
// the previous COUNT give each tile's first slot); a tile chunk reserves
// room for its particles per neighbouring destination tile with one atomic
// each, particles outside the 3x3 neighbourhood and tail particles take
// single ranks.  The updated particle (or a dead marker if it was absorbed)
// is written there instead of in place.  MODE bit 2: a context with the
// elliptic insert (absorption on it and the band charges compiled in).
// MODE bit 3: cubic shapes (the space-charge field from the cubic
// coefficients, the cubic deposit into the ghosted grid beside Q).
template <int MODE, int U>
__device__ __forceinline__ void particles_body(const KArgs& A) {
    constexpr bool COUNT = (MODE & 1) != 0;
    constexpr bool SCATTER = (MODE & 2) != 0;
    constexpr bool INS = (MODE & 4) != 0;
    constexpr bool CUB = (MODE & 8) != 0;
    extern __shared__ __align__(16) unsigned char smem[];
    lds_float4* sEB = (lds_float4*)(v4f*)smem;
    lds_u64* sQ = (lds_u64*)(unsigned long long*)(smem + sizeof(float4) * (size_t)A.win_max);
    // cubic shapes: coefficient and charge windows after them
    lds_f32* sC = (lds_f32*)(float*)(smem + 24 * (size_t)A.win_max);
    lds_u64* sQx = (lds_u64*)(unsigned long long*)(smem + 24 * (size_t)A.win_max + 4 * (size_t)A.win3_max);
    __shared__ long long s_start;
    __shared__ int s_count, s_inst, s_tr0, s_tz0;
    __shared__ unsigned int s_bcnt[9], s_bbase[9], s_ccnt[9];
    __shared__ unsigned long long s_ctr[SC_N];
    __shared__ unsigned long long s_q[kLQ];
    __shared__ unsigned int s_qn;
    __shared__ long long s_qbase;
    const int tid = threadIdx.x;
    // Static balance: workgroup w pushes the w-th of gridDim.x equal ranges of
    // the step's tile-sorted particles, walking the tile segments its range
    // covers, then the w-th of gridDim.x equal ranges of the tails.  The
    // tails (electrons created since the sort) have no LDS window and deposit
    // with device atomics, so they are spread over every workgroup rather
    // than left to the last ones.
    const long long total = A.ctl[CTL_TOTAL], nsorted = A.ctl[CTL_SORTED];
    const long long G = gridDim.x, wg = blockIdx.x;
    // The sorted part is cut into the same chunks in every step between two
    // sorts, so the counting step records each chunk's survivors per
    // neighbouring tile and the sorting step reserves its destinations from
    // that record instead of reading the positions a second time.
    int kc = 0;
    // Plain steps hand out the last twelfth of the sorted particles in units
    // of kDynUnit from a device counter (ctl[CTL_WORK], cleared at every step
    // end) once a workgroup's own ranges are done, so the workgroups that run
    // faster take more of it and all finish together; the counting and
    // sorting steps keep the static cut their records depend on.
    // (Only when a workgroup's share holds at least two units: on small
    // workloads a unit would outweigh the static shares.)
    constexpr bool DYN = !COUNT && !SCATTER;
    const long long n_dyn = DYN && nsorted >= 2 * kDynUnit * G ? nsorted / 12 : 0;
    __shared__ long long s_unit;
    for (int part = 0; part < (DYN ? 3 : 2); ++part) {
        for (;;) {
            long long v, vend;
            if (part < 2) {
                const long long n_part = part ? total - nsorted : nsorted - n_dyn;
                const long long per = n_part / G, rmd = n_part % G;
                v = (part ? nsorted : 0ll) + wg * per + min(wg, rmd);
                vend = v + per + (wg < rmd ? 1 : 0);
            } else {
                if (tid == 0) s_unit = (long long)atomicAdd((unsigned long long*)&A.ctl[CTL_WORK], 1ull);
                __syncthreads();
                const long long a = nsorted - n_dyn + s_unit * kDynUnit;
                __syncthreads();
                if (a >= nsorted) break;
                v = a;
                vend = min(a + kDynUnit, nsorted);
            }
            while (v < vend) {
                if (tid < 64) {
                    if (v < nsorted) {
                        const int t = wave_search(A.vtile, A.n_tiles, v);
                        if (tid == 0) {
                            const long long tv = A.vtile[t], tv1 = A.vtile[t + 1];
                            const int4 ti = A.tile_info[t];
                            s_start = A.tile_start[t] + (v - tv);
                            s_count = (int)min(min(vend, tv1) - v, (long long)A.C);
                            s_inst = ti.x;
                            s_tr0 = ti.y * A.TR;
                            s_tz0 = ti.z * A.TZ;
                        }
                    } else {
                        const long long u = v - nsorted;
                        const long long* tb = A.ctl + CTL_TAIL;
                        const int k = wave_search(tb, A.n_inst, u);
                        if (tid == 0) {
                            const long long* cj = A.cnt + (long long)k * C_NCOUNT;
                            s_start = A.It[k].p_off + cj[C_LIVE_SORTED] + (u - tb[k]);
                            s_count = (int)min(min(vend - v, tb[k + 1] - u), (long long)A.C);
                            s_inst = k;
                            s_tr0 = -1;
                            s_tz0 = -1;
                        }
                    }
                }
                if (SCATTER && tid < 9) s_bcnt[tid] = 0u;
                if (COUNT && tid < 9) s_ccnt[tid] = 0u;
                if (tid < SC_N) s_ctr[tid] = 0ull;
                if (tid == SC_N) s_qn = 0u;
                __syncthreads();
                const int count = __builtin_amdgcn_readfirstlane(s_count);
                v += count;
                const long long start = s_start;
                const int inst = __builtin_amdgcn_readfirstlane(s_inst);
                const int tr0 = __builtin_amdgcn_readfirstlane(s_tr0), tz0 = __builtin_amdgcn_readfirstlane(s_tz0);
                const DevInst& I = A.It[inst];
                const FieldDev& F = A.Ft[inst];
                long long* cnt = A.cnt + (long long)inst * C_NCOUNT;
                const unsigned int step = (unsigned int)cnt[C_STEP];
                const PSet out = SCATTER ? A.out : A.p;
                const int W = I.W;
                const bool win = tr0 >= 0;
                const bool rec = win && kc < A.crec_max;
                const long long rbase = (wg * A.crec_max + kc) * 9;
                if (win) ++kc;
                const int ti_c = win ? tr0 / A.TR : 0, tj_c = win ? tz0 / A.TZ : 0;
                int i0 = 0, i1 = -1, j0 = 0, j1 = -1, ww = 1;
                if (win) {
                    i0 = max(tr0 - A.halo, 0);
                    i1 = min(tr0 + A.TR + A.halo, I.nr);
                    j0 = max(tz0 - A.halo, 0);
                    j1 = min(tz0 + A.TZ + A.halo, I.nz);
                    ww = j1 - j0 + 1;
                    const int nwin = (i1 - i0 + 1) * ww;
                    for (int t = tid; t < nwin; t += kPWG) {
                        int a = t / ww, b = t - a * ww;
                        sEB[t] = as_gbl(F.EB)[(long long)(i0 + a) * W + (j0 + b)];
                        sQ[t] = 0ull;
                    }
                    if (CUB) {
                        // ghosted nodes i0 .. i1 + 2, j0 .. j1 + 2 (physical i - 1)
                        const int w3 = ww + 2, nwin3 = (i1 - i0 + 3) * w3, WX = I.nz + 3;
                        for (int t = tid; t < nwin3; t += kPWG) {
                            int a = t / w3, b = t - a * w3;
                            sC[t] = ((gbl_f32*)F.cxf)[(long long)(i0 + a) * WX + (j0 + b)];
                            sQx[t] = 0ull;
                        }
                    }
                }
                if (SCATTER && win) {
                    // pass 1: destinations of this chunk's particles per neighbouring
                    // tile, unless the counting step recorded them
                    const bool from_rec = !COUNT && rec;
                    const LocalInst L1 = local_inst(I);
                    const int lead = (int)(start & 63);
                    for (int base = from_rec ? count : -lead; base < count; base += kPWG) {
                        const int q = base + tid;
                        const bool in = q >= 0 && q < count;
                        const long long p = start + (in ? q : 0);
                        const float r = A.p.r(p), z = A.p.z(p);
                        int bkt = -1;
                        if (in && r >= 0.0f) {
                            int i, j;
                            float fr, fz;
                            cell_of(L1, r, z, i, j, fr, fz);
                            int dr = i / A.TR - ti_c, dz = j / A.TZ - tj_c;
                            if (dr >= -1 && dr <= 1 && dz >= -1 && dz <= 1) bkt = (dr + 1) * 3 + (dz + 1);
                        }
                        wave_aggregate<false>(bkt >= 0, bkt, [&](int k, unsigned int n) {
                            atomicAdd(&s_bcnt[k], n);
                            return 0u;
                        });
                    }
                    if (!from_rec) __syncthreads();
                    if (tid < 9) {
                        unsigned int n = from_rec ? A.crec[rbase + tid] : s_bcnt[tid];
                        if (n) {
                            int t = I.tile_off + (ti_c + tid / 3 - 1) * I.ntz + (tj_c + tid % 3 - 1);
                            s_bbase[tid] = atomicAdd(&A.tile_fill[t], n);
                        }
                        s_bcnt[tid] = 0u;
                    }
                }
                __syncthreads();
                unsigned int c_push = 0;
                ChunkCtx X;
                X.L = local_inst(I);
                X.sEB = sEB; X.sQ = sQ; X.s_ctr = s_ctr; X.s_bcnt = s_bcnt; X.s_bbase = s_bbase; X.s_ccnt = s_ccnt;
                X.s_qn = &s_qn; X.s_q = s_q;
                X.out = out; X.EB = F.EB; X.Q = F.Q; X.Qw = F.Qw;
                X.inst = inst; X.ti_c = ti_c; X.tj_c = tj_c; X.i0 = i0; X.i1 = i1; X.j0 = j0; X.j1 = j1; X.ww = ww;
                X.win = win; X.step = step;
                X.sC = sC; X.sQx = sQx; X.cxf = F.cxf; X.Qx = F.Qx; X.WX = I.nz + 3;
                // U particles per lane per pass (their loads are all in flight before
                // any is processed, and their arithmetic interleaves).  Passes start
                // on a 64-slot boundary so that every wave's loads and stores cover
                // whole aligned lines; lanes before the chunk idle.
                const int lead = (int)(start & 63);
                const float wu = X.L.w_uni;
                for (int base = -lead; base < count; base += U * kPWG) {
                    long long pp[U];
                    bool inr[U];
                    float r[U], z[U], vr[U], vt[U], vz[U], w[U];
                    unsigned long long key[U];
                    // A pass issues its loads at a raised wave priority, so the
                    // SIMD's arbiter puts them (and their address arithmetic)
                    // ahead of other waves' push arithmetic and more of the
                    // particle stream is in flight: plain step -0.25%, scan32's
                    // launch -0.5%, the gun's -0.2%.
                    __builtin_amdgcn_sched_barrier(0);
                    __builtin_amdgcn_s_setprio(1);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int q = base + u * kPWG + tid;
                        inr[u] = q >= 0 && q < count;
                        pp[u] = start + (inr[u] ? q : 0);
                        r[u] = A.p.r(pp[u]);
                        z[u] = A.p.z(pp[u]);
                        vr[u] = A.p.vr(pp[u]);
                        vt[u] = A.p.vt(pp[u]);
                        vz[u] = A.p.vz(pp[u]);
                        w[u] = wu != 0.0f ? wu : A.p.w(pp[u]);
                        key[u] = A.p.key(pp[u]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    __builtin_amdgcn_s_setprio(0);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        push_particle<COUNT, SCATTER, INS, CUB>(A, X, pp[u], inr[u], r[u], z[u], vr[u], vt[u], vz[u], w[u], key[u],
                                                      c_push);
                }
                flush_counter(&cnt[C_PSTEPS], (unsigned long long)c_push);
                __syncthreads();
                if (tid < SC_N) {
                    const unsigned long long v = s_ctr[tid];
                    if (v) atomicAdd((unsigned long long*)&cnt[kCounterOf[tid]], v);
                }
                // the chunk's queued events: one device reservation
                const unsigned int q_all = s_qn;
                const unsigned int q_lds = min(q_all, (unsigned int)kLQ);
                if (tid == SC_N) {
                    s_qbase = q_lds ? (long long)atomicAdd((unsigned long long*)&A.ctl[CTL_QCOUNT], (unsigned long long)q_lds)
                                    : 0ll;
                }
                if (COUNT && win && tid < 9) {
                    const unsigned int v = s_ccnt[tid];
                    if (v) atomicAdd(&A.cnt_out[I.tile_off + (ti_c + tid / 3 - 1) * I.ntz + (tj_c + tid % 3 - 1)], v);
                    if (!SCATTER && rec) A.crec[rbase + tid] = v;
                }
                __syncthreads();
                for (unsigned int t = tid; t < q_lds; t += kPWG) {
                    const long long qi = s_qbase + t;
                    if (qi < A.qcap) A.queue[qi] = s_q[t];
                    else A.ctl[CTL_QOVER] = 1;
                }
                if (win) {
                    const int nwin = (i1 - i0 + 1) * ww;
                    gbl_u64* Qg = as_gbl(F.Q);
                    for (int t = tid; t < nwin; t += kPWG) {
                        const unsigned long long v = sQ[t];
                        if (v != 0ull) {
                            int a = t / ww, b = t - a * ww;
                            gbl_add(&Qg[(long long)(i0 + a) * W + (j0 + b)], v);
                        }
                    }
                    if (CUB) {
                        const int w3 = ww + 2, nwin3 = (i1 - i0 + 3) * w3, WX = I.nz + 3;
                        gbl_u64* Qx = as_gbl(F.Qx);
                        for (int t = tid; t < nwin3; t += kPWG) {
                            const unsigned long long v = sQx[t];
                            if (v != 0ull) {
                                int a = t / w3, b = t - a * w3;
                                gbl_add(&Qx[(long long)(i0 + a) * WX + (j0 + b)], v);
                            }
                        }
                    }
                }
            }
            if (part < 2) break;
        }
    }
}

// Two launch shapes of the bilinear forms, both timed by the autotuner: one
// particle per lane and pass at 64 registers, so two workgroups share a CU
// (8 waves per SIMD); or two particles per lane and pass at up to 128
// registers, one workgroup per CU (4 waves per SIMD), whose two particles'
// loads are in flight together and whose arithmetic interleaves.
template <int MODE>
__global__ void __launch_bounds__(kPWG) __attribute__((amdgpu_waves_per_eu(8, 8))) k_particles(KArgs A) {
    particles_body<MODE, 1>(A);
}

template <int MODE>
__global__ void __launch_bounds__(kPWG) __attribute__((amdgpu_waves_per_eu(4, 4))) k_particles2(KArgs A) {
    particles_body<MODE, 2>(A);
}

// The elliptic insert's plain step with one particle per lane: its band
// test and band deposit spill 11 registers at 64, so it takes up to 128
// registers and one workgroup per CU; its counting and sorting steps keep
// two workgroups per CU (their spills cost less than half the workgroups).
template <int MODE>
__global__ void __launch_bounds__(kPWG) k_particles_ins(KArgs A) {
    particles_body<MODE, 1>(A);
}

// Cubic shapes: the 16-node gather and deposit keep their values in up to
// 128 registers (one workgroup per CU) instead of spilling.
template <int MODE>
__global__ void __launch_bounds__(kPWG) k_particles3(KArgs A) {
    particles_body<MODE | 8, 1>(A);
}

// Resolve the collision events queued by the particle kernel (which took
// the null-or-real decision and counted the events): the parent's new
// velocity (FP32) and, for an ionisation, a new electron appended after the
// instance's slots, deposited at the parent's position and counted for the
// next sort.  The new electrons' slots are reserved per workgroup pass and
// instance: LDS ranks, then one device atomic per instance present.
__global__ void __launch_bounds__(kWG) k_collide(KArgs A, PSet P, int scatter) {
    extern __shared__ unsigned int s_coll[];
    unsigned int* s_niz = s_coll;             // [n_inst] ionisations in this pass
    unsigned int* s_base = s_coll + A.n_inst;  // [n_inst] their first spawn rank
    const long long nq = min(A.ctl[CTL_QCOUNT], A.qcap);
    for (long long b0q = (long long)blockIdx.x * kWG; b0q < nq; b0q += (long long)gridDim.x * kWG) {
        for (int k = threadIdx.x; k < A.n_inst; k += kWG) s_niz[k] = 0u;
        __syncthreads();
        const long long qi = b0q + threadIdx.x;
        int inst = 0, ev = 0;
        unsigned int local = 0u;
        float r = 0.0f, z = 0.0f, w = 0.0f, cvr = 0.0f, cvt = 0.0f, cvz = 0.0f;
        unsigned long long ckey = 0ull;
        if (qi < nq) {
            const unsigned long long e = A.queue[qi];
            inst = (int)(e >> 40);
            const long long p = (long long)(e & ((1ull << 40) - 1ull));
            const DevInst& I = A.It[inst];
            const unsigned int step = (unsigned int)A.cnt[(long long)inst * C_NCOUNT + C_STEP];
            const unsigned long long key = P.key(p);
            const uint4 b0 = philox_step(I, key, step, 0u);
            float vr = P.vr(p), vt = P.vt(p), vz = P.vz(p);
            r = P.r(p);
            z = P.z(p);
            w = weight_at(I, P, p);
            ev = collide_f(I, key, step, b0, vr, vt, vz, cvr, cvt, cvz, ckey);
            if (ev != 0) {
                P.vr(p) = vr;
                P.vt(p) = vt;
                P.vz(p) = vz;
            }
            if (ev == 2) local = atomicAdd(&s_niz[inst], 1u);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < A.n_inst; k += kWG) {
            const unsigned int n = s_niz[k];
            if (n)
                s_base[k] = (unsigned int)atomicAdd((unsigned long long*)&A.cnt[(long long)k * C_NCOUNT + C_SPAWN],
                                                    (unsigned long long)n);
        }
        __syncthreads();
        if (ev != 2) continue;
        const DevInst& I = A.It[inst];
        long long* cnt = A.cnt + (long long)inst * C_NCOUNT;
        const long long rel = (scatter ? A.new_base[inst] : cnt[C_SLOTS]) + (long long)(s_base[inst] + local);
        if (rel >= I.p_cap) {
            atomicAdd((unsigned long long*)&cnt[C_DROPPED], 1ull);
            continue;
        }
        const long long d = I.p_off + rel;
        P.r(d) = r; P.z(d) = z;
        P.vr(d) = cvr; P.vt(d) = cvt; P.vz(d) = cvz;
        P.w(d) = w;
        P.key(d) = ckey;
        int i, j;
        float fr, fz;
        cell_of(I, r, z, i, j, fr, fz);
        long long q00, q10, q01, q11;
        node_charges(w, (float)I.two_S, fr, fz, q00, q10, q01, q11);
        unsigned long long* Qg = (unsigned long long*)A.Ft[inst].Q;
        const long long n00 = (long long)i * I.W + j;
        atomicAdd(&Qg[n00], (unsigned long long)q00);
        atomicAdd(&Qg[n00 + I.W], (unsigned long long)q10);
        atomicAdd(&Qg[n00 + 1], (unsigned long long)q01);
        atomicAdd(&Qg[n00 + I.W + 1], (unsigned long long)q11);
        if (I.has_ins) deposit_qw(I, A.Ft[inst].Qw, w, r, z);
        if (I.spline3) deposit_cubic_gbl(A.Ft[inst].Qx, I.nz + 3, i, j, w, (float)I.two_S, fr, fz);
        if (A.cnt_out) atomicAdd(&A.cnt_out[I.tile_off + (i / A.TR) * I.ntz + (j / A.TZ)], 1u);
    }
}

// Volumetric seed source (Sec. II.A): this step's new electrons of every
// instance (blockIdx.y), appended to the tail like the ionisation products
// (after the sorted block of the output store in a sorting step), deposited
// with global atomics and, in a counting step, counted in their tiles.
__global__ void __launch_bounds__(kWG) k_source32(KArgs A, PSet P, int scatter) {
    const int inst = blockIdx.y;
    const DevInst& I = A.It[inst];
    if (!(I.src_rate > 0.0)) return;
    long long* cnt = A.cnt + (long long)inst * C_NCOUNT;
    long long first, count;
    source_count(I, cnt[C_STEP], first, count);
    const long long base = scatter ? A.new_base[inst] : cnt[C_SLOTS];
    unsigned long long* Qg = (unsigned long long*)A.Ft[inst].Q;
    const float wf = (float)I.weight;
    for (long long j = (long long)blockIdx.x * kWG + threadIdx.x; j < count; j += (long long)gridDim.x * kWG) {
        unsigned long long key;
        double rd, zd, vr, vt, vz;
        source_draw(I, first + j, key, rd, zd, vr, vt, vz);
        if (I.has_ins && ins_g(I, rd, zd) <= 0.0) continue;  // inside the insert: outside the domain
        atomicAdd((unsigned long long*)&cnt[C_SOURCE], 1ull);
        const long long rel = base + (long long)atomicAdd((unsigned long long*)&cnt[C_SPAWN], 1ull);
        if (rel >= I.p_cap) {
            atomicAdd((unsigned long long*)&cnt[C_DROPPED], 1ull);
            continue;
        }
        const long long d = I.p_off + rel;
        const float r = (float)rd, z = (float)zd;
        P.r(d) = r;
        P.z(d) = z;
        P.vr(d) = (float)vr;
        P.vt(d) = (float)vt;
        P.vz(d) = (float)vz;
        P.w(d) = wf;
        P.key(d) = key;
        int i, jj;
        float fr, fz;
        cell_of(I, r, z, i, jj, fr, fz);
        long long q00, q10, q01, q11;
        node_charges(wf, (float)I.two_S, fr, fz, q00, q10, q01, q11);
        const long long n00 = (long long)i * I.W + jj;
        atomicAdd(&Qg[n00], (unsigned long long)q00);
        atomicAdd(&Qg[n00 + I.W], (unsigned long long)q10);
        atomicAdd(&Qg[n00 + 1], (unsigned long long)q01);
        atomicAdd(&Qg[n00 + I.W + 1], (unsigned long long)q11);
        if (I.has_ins) deposit_qw(I, A.Ft[inst].Qw, wf, r, z);
        if (I.spline3) deposit_cubic_gbl(A.Ft[inst].Qx, I.nz + 3, i, jj, wf, (float)I.two_S, fr, fz);
        if (A.cnt_out) atomicAdd(&A.cnt_out[I.tile_off + (i / A.TR) * I.ntz + (jj / A.TZ)], 1u);
    }
}

// Fluid-moment node sums of one instance's live particles (diagnostic),
// from the FP32 state widened to FP64.
__global__ void __launch_bounds__(kWG) k_moments32(DevInst I, PSet P, const long long* cnt, double* acc) {
    const long long slots = cnt[C_SLOTS];
    for (long long q = (long long)blockIdx.x * kWG + threadIdx.x; q < slots; q += (long long)gridDim.x * kWG) {
        const long long p = I.p_off + q;
        const float r = P.r(p);
        if (r < 0.0f) continue;
        moments_add(I, (double)r, (double)P.z(p), (double)P.vr(p), (double)P.vt(p), (double)P.vz(p),
                    (double)weight_at(I, P, p), acc);
    }
}

// Tail plan of the coming step (see prep_tails_block) when no field stage ran
// since the counters changed (after a full sort).
__global__ void k_prep(long long* ctl, const long long* cnt, int n_inst) {
    if (blockIdx.x != 0) return;
    prep_tails_block(ctl, cnt, n_inst);
}

__global__ void k_zero_q(const DevInst* It, const FieldDev* Ft) {
    const DevInst& I = It[blockIdx.y];
    long long* Q = Ft[blockIdx.y].Q;
    long long* Qw = I.spline3 ? nullptr : Ft[blockIdx.y].Qw;  // node array with bilinear shapes
    // pairs of nodes as 16-byte stores (the arrays are 256-byte aligned), then an odd last node
    const int pairs = I.nodes / 2;
    const longlong2 z2 = make_longlong2(0, 0);
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < pairs; n += gridDim.x * blockDim.x) {
        reinterpret_cast<longlong2*>(Q)[n] = z2;
        if (Qw) reinterpret_cast<longlong2*>(Qw)[n] = z2;
    }
    if ((I.nodes & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        Q[I.nodes - 1] = 0;
        if (Qw) Qw[I.nodes - 1] = 0;
    }
    if (I.spline3) {  // the ghosted cubic grids
        long long* Qx = Ft[blockIdx.y].Qx;
        long long* Qxw = Ft[blockIdx.y].Qw;
        const int ext = (I.nr + 3) * (I.nz + 3);
        for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < ext; n += gridDim.x * blockDim.x) {
            Qx[n] = 0;
            if (Qxw) Qxw[n] = 0;
        }
    }
}

// ---- tile sort ------------------------------------------------------------

__device__ __forceinline__ int tile_of(const DevInst& I, float r, float z, int TR, int TZ) {
    int i, j;
    float fr, fz;
    cell_of(I, r, z, i, j, fr, fz);
    return I.tile_off + (i / TR) * I.ntz + (j / TZ);
}

__global__ void __launch_bounds__(kWG) k_sort_count(KArgs A, unsigned long long* sortkey,
                                                    unsigned int* tile_count) {
    const int inst = blockIdx.y;
    const DevInst& I = A.It[inst];
    const long long slots = A.cnt[(long long)inst * C_NCOUNT + C_SLOTS];
    const long long stride = (long long)gridDim.x * kWG;
    const int lane = __lane_id();
    for (long long b = (long long)blockIdx.x * kWG; b < slots; b += stride) {
        long long q = b + threadIdx.x;
        bool valid = false;
        int tile = 0;
        long long p = I.p_off + q;
        if (q < slots) {
            float r = A.p.r(p);
            if (r >= 0.0f) {
                valid = true;
                tile = tile_of(I, r, A.p.z(p), A.TR, A.TZ);
            }
        }
        unsigned long long active = __ballot(valid);
        unsigned int rank = 0;
        while (active) {
            int leader = __ffsll((long long)active) - 1;
            int t = __shfl(tile, leader);
            unsigned long long m = __ballot(valid && tile == t) & active;
            unsigned int base = 0;
            if (lane == leader) base = atomicAdd(&tile_count[t], (unsigned int)__popcll(m));
            base = __shfl(base, leader);
            if ((m >> lane) & 1ull) rank = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
            active &= ~m;
        }
        if (q < slots) sortkey[p] = valid ? ((((unsigned long long)tile) << 32) | rank) : ~0ull;
    }
}

// Inclusive prefix sum of v over the 64 lanes of the wave (Hillis-Steele:
// six cross-lane shifts).
__device__ __forceinline__ long long wave_inclusive_scan(long long v) {
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive prefix sum of v over the kScanWG threads of the block (every
// thread calls it): each wave scans its lanes, the first wave scans the wave
// totals, each thread adds its wave's offset.  *total gets the block's sum.
// s_wave is kScanWG / 64 + 1 entries of LDS; the call ends with a barrier,
// so it can be called again.
constexpr int kScanWG = 1024;
__device__ __forceinline__ long long block_exclusive_scan(long long v, long long* s_wave, long long* total) {
    constexpr int NW = kScanWG / 64;
    const int lane = __lane_id(), wave = (int)(threadIdx.x >> 6);
    const long long inc = wave_inclusive_scan(v);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        const long long t = lane < NW ? s_wave[lane] : 0;
        const long long ti = wave_inclusive_scan(t);
        if (lane < NW) s_wave[lane] = ti - t;
        if (lane == NW - 1) s_wave[NW] = ti;
    }
    __syncthreads();
    const long long ex = s_wave[wave] + (inc - v);
    *total = s_wave[NW];
    __syncthreads();
    return ex;
}

// Per instance: exclusive scan of the tile totals -> each tile's first slot
// in the destination store (absolute) and its offset among the instance's
// sorted particles; the instance's sorted total.  Each thread sums a
// contiguous run of tiles, the block scans the run totals.
__global__ void __launch_bounds__(kScanWG) k_sort_plan1(const DevInst* It, const unsigned int* tile_count,
                                                        long long* tile_start, long long* tile_lpre,
                                                        long long* inst_live) {
    __shared__ long long s_wave[kScanWG / 64 + 1];
    const DevInst& I = It[blockIdx.x];
    const int nt = I.ntr * I.ntz, base = I.tile_off;
    const int seg = (nt + kScanWG - 1) / kScanWG;
    const int t0 = min((int)threadIdx.x * seg, nt), t1 = min(t0 + seg, nt);
    long long sc = 0;
    for (int t = t0; t < t1; ++t) sc += tile_count[base + t];
    long long total;
    long long a = block_exclusive_scan(sc, s_wave, &total);
    if (threadIdx.x == 0) inst_live[blockIdx.x] = total;
    for (int t = t0; t < t1; ++t) {
        tile_start[base + t] = I.p_off + a;
        tile_lpre[base + t] = a;
        a += tile_count[base + t];
    }
}

// Instances' offsets in the step's particle order; total sorted particles.
// One block scans the instance totals kScanWG at a time with a carry.
__global__ void __launch_bounds__(kScanWG) k_sort_plan2(const long long* inst_live, long long* inst_voff,
                                                        long long* ctl, long long* vtile, int n_inst,
                                                        int n_tiles) {
    __shared__ long long s_wave[kScanWG / 64 + 1];
    long long carry = 0;
    for (int k0 = 0; k0 < n_inst; k0 += kScanWG) {
        const int k = k0 + (int)threadIdx.x;
        const long long v = k < n_inst ? inst_live[k] : 0;
        long long total;
        const long long ex = block_exclusive_scan(v, s_wave, &total);
        if (k < n_inst) inst_voff[k] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        ctl[CTL_SORTED] = carry;
        vtile[n_tiles] = carry;
    }
}

// Global prefix of sorted particles over all tiles.
__global__ void k_sort_plan3(const int4* tile_info, int n_tiles, const long long* tile_lpre,
                             const long long* inst_voff, long long* vtile) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    vtile[t] = inst_voff[tile_info[t].x] + tile_lpre[t];
}

__global__ void __launch_bounds__(kWG) k_sort_scatter(KArgs A, PSet dst, const unsigned long long* sortkey,
                                                      const long long* tile_start) {
    const int inst = blockIdx.y;
    const DevInst& I = A.It[inst];
    const long long slots = A.cnt[(long long)inst * C_NCOUNT + C_SLOTS];
    for (long long q = (long long)blockIdx.x * kWG + threadIdx.x; q < slots; q += (long long)gridDim.x * kWG) {
        long long p = I.p_off + q;
        unsigned long long k = sortkey[p];
        if (k == ~0ull) continue;
        long long d = tile_start[k >> 32] + (long long)(k & 0xffffffffull);
        dst.r(d) = A.p.r(p);
        dst.z(d) = A.p.z(p);
        dst.vr(d) = A.p.vr(p);
        dst.vt(d) = A.p.vt(p);
        dst.vz(d) = A.p.vz(p);
        if (I.w_uni == 0.0f) dst.w(d) = A.p.w(p);
        dst.key(d) = A.p.key(p);
    }
}

__global__ void k_sort_commit(long long* cnt, const long long* inst_live, int n_inst) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    long long* c = cnt + (long long)k * C_NCOUNT;
    c[C_SLOTS] = inst_live[k];
    c[C_LIVE_SORTED] = inst_live[k];
    c[C_DEAD] = 0;
}

// Scatter step: before the particle kernel the old holes are dropped from
// the dead count; after it the sorted output becomes the slot range.
__global__ void k_scatter_pre(long long* cnt, int n_inst) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_inst) cnt[(long long)k * C_NCOUNT + C_DEAD] = 0;
}

__global__ void k_scatter_commit(long long* cnt, const long long* inst_live, int n_inst) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    long long* c = cnt + (long long)k * C_NCOUNT;
    c[C_SLOTS] = inst_live[k];
    c[C_LIVE_SORTED] = inst_live[k];
}

__global__ void k_zero_u32(unsigned int* p, int n) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}

// ---- load and standalone deposit ------------------------------------------

__global__ void k_load32(DevInst I, double r_lo, double r_hi, double z_lo, double z_hi, double sv, float w0,
                         int load_mode, PSet p, long long n) {
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        unsigned long long key = (unsigned long long)q;
        uint4 b0 = philox_step(I, key, 0xFFFFFFFFu, 0u);
        uint4 b1 = philox_step(I, key, 0xFFFFFFFFu, 1u);
        uint4 b2 = philox_step(I, key, 0xFFFFFFFFu, 2u);
        double ur = u52(b0.x, b0.y), uz = u52(b0.z, b0.w);
        double r = load_mode == 1 ? r_lo + ur * (r_hi - r_lo)
                                  : sqrt(r_lo * r_lo + ur * (r_hi * r_hi - r_lo * r_lo));
        double z = z_lo + uz * (z_hi - z_lo);
        double u1 = u52(b1.x, b1.y), u2 = u52(b1.z, b1.w);
        double u3 = u52(b2.x, b2.y), u4 = u52(b2.z, b2.w);
        double m1 = sqrt(-2.0 * log(u1)), m3 = sqrt(-2.0 * log(u3));
        long long d = I.p_off + q;
        p.r(d) = (float)r;
        p.z(d) = (float)z;
        p.vr(d) = (float)(sv * (m1 * cos((2.0 * kPi) * u2)));
        p.vt(d) = (float)(sv * (m1 * sin((2.0 * kPi) * u2)));
        p.vz(d) = (float)(sv * (m3 * cos((2.0 * kPi) * u4)));
        p.w(d) = w0;
        p.key(d) = key;
    }
}

__global__ void k_deposit32(DevInst I, PSet P, long long* Q, long long* Qw, long long* Qx, const long long* cnt) {
    const long long slots = cnt[C_SLOTS];
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < slots;
         q += (long long)gridDim.x * blockDim.x) {
        long long p = I.p_off + q;
        float r = P.r(p);
        if (r < 0.0f) continue;
        int i, j;
        float fr, fz;
        cell_of(I, r, P.z(p), i, j, fr, fz);
        long long q00, q10, q01, q11;
        node_charges(weight_at(I, P, p), (float)I.two_S, fr, fz, q00, q10, q01, q11);
        unsigned long long* Qg = (unsigned long long*)Q;
        long long n00 = (long long)i * I.W + j;
        atomicAdd(&Qg[n00], (unsigned long long)q00);
        atomicAdd(&Qg[n00 + I.W], (unsigned long long)q10);
        atomicAdd(&Qg[n00 + 1], (unsigned long long)q01);
        atomicAdd(&Qg[n00 + I.W + 1], (unsigned long long)q11);
        if (Qw) deposit_qw(I, Qw, weight_at(I, P, p), r, P.z(p));
        if (Qx) deposit_cubic_gbl(Qx, I.nz + 3, i, j, weight_at(I, P, p), (float)I.two_S, fr, fz);
    }
}

typedef void (*ParticleKernel)(KArgs);
// Variant v = step kind (bits 0-1) | insert (4) | cubic shapes (8); lanes =
// particles per lane and pass of the bilinear forms (1 or 2).
ParticleKernel particle_kernel(int v, int lanes) {
    if (lanes == 2 && v < 8) {
        switch (v) {
            case 0: return k_particles2<0>;
            case 1: return k_particles2<1>;
            case 2: return k_particles2<2>;
            case 3: return k_particles2<3>;
            case 4: return k_particles2<4>;
            case 5: return k_particles2<5>;
            case 6: return k_particles2<6>;
            default: return k_particles2<7>;
        }
    }
    switch (v) {
        case 0: return k_particles<0>;
        case 1: return k_particles<1>;
        case 2: return k_particles<2>;
        case 3: return k_particles<3>;
        case 4: return k_particles_ins<4>;
        case 5: return k_particles<5>;
        case 6: return k_particles<6>;
        case 7: return k_particles<7>;
        case 8: return k_particles3<0>;
        case 9: return k_particles3<1>;
        case 10: return k_particles3<2>;
        case 11: return k_particles3<3>;
        case 12: return k_particles3<4>;
        case 13: return k_particles3<5>;
        case 14: return k_particles3<6>;
        default: return k_particles3<7>;
    }
}

// LDS bytes of the particle kernel's windows: fields and charge per window
// node, with cubic shapes the ghosted coefficient and charge windows.
size_t particle_lds(int win, int win3) { return (size_t)win * 24 + (size_t)win3 * 12; }

unsigned int grid_for(long long n, long long cap = 16384) {
    long long g = (n + kWG - 1) / kWG;
    return (unsigned int)std::max(1ll, std::min(g, cap));
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Chunks per workgroup whose neighbouring-tile counts the counting step
// records for the sorting step (later chunks count again).
constexpr int kRecMax = 64;

struct F32State {
    int TR = 8, TZ = 32, halo = 8, K = 16, C = 1 << 22, win_max = 0, win3_max = 0;
    bool ins = false;  // some instance has the elliptic insert
    bool cub = false;  // the instances use cubic shapes
    int coll_grid = 64;   // workgroups of k_collide
    int cu = 256, wg_per_cu = 4;  // resident workgroups per CU of the counting and sorting steps
    int wg_per_cu_plain = 4;      // and of the plain step
    int lanes = 1;        // particles per lane and pass of the bilinear particle kernel (1 or 2)
    PSet set[2];
    int cur = 0;
    long long total_cap = 0;
    unsigned long long* sortkey = nullptr;
    unsigned int* tile_count = nullptr;
    long long* tstart[2] = {nullptr, nullptr};  // tile starts of the layout held in set[k]
    long long *tile_lpre = nullptr, *vtile = nullptr;
    long long *inst_live = nullptr, *inst_voff = nullptr;
    int4* tile_info = nullptr;
    int n_tiles = 0;
    long long* ctl = nullptr;
    unsigned int* cbuf[2] = {nullptr, nullptr};  // per-tile totals counted for the next sort
    unsigned int* tile_fill = nullptr;
    unsigned int* crec = nullptr;         // chunk records of the counting step (kRecMax per workgroup)
    unsigned long long* queue = nullptr;  // real collision events of one step
    long long qcap = 0;
    FieldDev* dF = nullptr;  // field table (owned by the context)
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipEvent_t ev_snap = nullptr;  // counter snapshot for the capacity check
    long long* h_cnt = nullptr;    // pinned copy of the counters
    bool snap_pending = false;
    int since_check = 0;
    long long grow_events = 0;
    bool checked_once = false;
    std::vector<long long> prev_used;  // used slots at the previous inspected copy
    hipGraphExec_t g_step[4][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
    hipGraphExec_t g_cycle[2] = {nullptr, nullptr};  // K steps from a sort to the next, per store
    bool graphs = false;
    bool graph_auto = false;  // the autotuner chooses between graphs and plain launches
    int phase = 0;        // steps since the last sort
    bool counted = false; // the last step counted tile totals for a scatter
};

static pic_status f32_fail(pic_ctx* ctx, pic_status st, const std::string& m) {
    pic_set_error(ctx, m);
    return st;
}

#define CK32(call)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return f32_fail(ctx, PIC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

static KArgs kargs(pic_ctx* ctx, F32State* S, int set) {
    KArgs A;
    A.It = pic_dev_table(ctx);
    A.Ft = S->dF;
    A.cnt = pic_counters(ctx);
    A.p = S->set[set];
    A.out = S->set[1 - set];
    A.vtile = S->vtile;
    A.tile_info = S->tile_info;
    A.ctl = S->ctl;
    A.cnt_out = nullptr;
    A.tile_fill = S->tile_fill;
    A.crec = S->crec;
    A.crec_max = kRecMax;
    A.tile_start = S->tstart[set];
    A.tile_dst = S->tstart[1 - set];
    A.new_base = S->inst_live;
    A.queue = S->queue;
    A.qcap = S->qcap;
    A.n_inst = pic_n_inst(ctx);
    A.n_tiles = S->n_tiles;
    A.TR = S->TR;
    A.TZ = S->TZ;
    A.halo = S->halo;
    A.C = S->C;
    A.win_max = S->win_max;
    A.win3_max = S->win3_max;
    return A;
}

// A store of n slots (n a multiple of the block).
static PSet alloc_set(pic_ctx* ctx, long long n) {
    PSet p;
    p.b = (unsigned int*)pic_dev_alloc(ctx, (size_t)(n / kBlkSlots) * kBlkBytes);
    p.wt = (float*)pic_dev_alloc(ctx, sizeof(float) * (size_t)n);
    return p;
}

static bool set_ok(const PSet& p) { return p.b != nullptr && p.wt != nullptr; }

static void free_set(pic_ctx* ctx, PSet& p) {
    pic_dev_free(ctx, p.b);
    pic_dev_free(ctx, p.wt);
    p = PSet{};
}

// Host address arithmetic of a store: the block holding slot p and the
// number of blocks covering `slots` slots from a block-aligned offset.
static unsigned int* block_of(const PSet& P, long long p) { return P.b + (p / kBlkSlots) * kBlkWords; }
static long long blocks_for(long long slots) { return (slots + kBlkSlots - 1) / kBlkSlots; }

// Tile tables for S->TR x S->TZ tiles with an S->halo window (the particle
// stores are untouched): per-instance tile counts and offsets, the device
// arrays indexed by tile, the LDS window size and the persistent grid.
static pic_status build_tiles(pic_ctx* ctx, F32State* S) {
    if (S->TR < 1 || S->TZ < 1 || S->TR > 256 || S->TZ > 256 || S->halo < 0 || S->halo > 32 || S->K < 1 ||
        S->C < 1 || S->C > (1 << 30))
        return f32_fail(ctx, PIC_EINVAL, "1 <= tile_r, tile_z <= 256, 0 <= halo <= 32, sort_interval >= 1, "
                                         "1 <= chunk <= 2^30");
    const int win = (S->TR + 2 * S->halo + 1) * (S->TZ + 2 * S->halo + 1);
    const int win3 = S->cub ? ((S->TR + 2 * S->halo + 3) * (S->TZ + 2 * S->halo + 3) + 1) / 2 * 2 : 0;
    // two workgroups per CU share its 160 KiB of LDS with one particle per
    // lane; with two, one workgroup has it to itself
    const size_t lds_cap = S->lanes == 2 ? 144 * 1024 : 64 * 1024;
    if (particle_lds(win, win3) > lds_cap)
        return f32_fail(ctx, PIC_EINVAL, "tile window exceeds the LDS of the launch shape (64 or 144 KiB)");
    const int n = pic_n_inst(ctx);
    long long tsum = 0;
    for (int k = 0; k < n; ++k) {
        const DevInst& I = pic_inst_dev(ctx, k);
        tsum += (long long)((I.nr + S->TR - 1) / S->TR) * ((I.nz + S->TZ - 1) / S->TZ);
    }
    if (tsum > (1 << 26)) return f32_fail(ctx, PIC_EINVAL, "too many tiles");
    // nothing is changed before this point: PIC_EINVAL leaves the tables as they were
    S->win_max = win;
    S->win3_max = win3;
    void* old[] = {S->tile_count, S->tstart[0], S->tstart[1], S->tile_lpre, S->vtile,
                   S->tile_info, S->cbuf[0],   S->cbuf[1],   S->tile_fill, S->crec};
    for (void* q : old) pic_dev_free(ctx, q);
    int toff = 0;
    std::vector<int4> tinfo;
    for (int k = 0; k < n; ++k) {
        DevInst& I = pic_inst_dev(ctx, k);
        I.ntr = (I.nr + S->TR - 1) / S->TR;
        I.ntz = (I.nz + S->TZ - 1) / S->TZ;
        I.tile_off = toff;
        for (int a = 0; a < I.ntr; ++a)
            for (int b = 0; b < I.ntz; ++b) tinfo.push_back(make_int4(k, a, b, 0));
        toff += I.ntr * I.ntz;
    }
    S->n_tiles = toff;
    S->tile_count = (unsigned int*)pic_dev_alloc(ctx, sizeof(unsigned int) * toff);
    S->tstart[0] = (long long*)pic_dev_alloc(ctx, sizeof(long long) * toff);
    S->tstart[1] = (long long*)pic_dev_alloc(ctx, sizeof(long long) * toff);
    S->tile_lpre = (long long*)pic_dev_alloc(ctx, sizeof(long long) * toff);
    S->vtile = (long long*)pic_dev_alloc(ctx, sizeof(long long) * (toff + 1));
    S->tile_info = (int4*)pic_dev_alloc(ctx, sizeof(int4) * toff);
    S->cbuf[0] = (unsigned int*)pic_dev_alloc(ctx, sizeof(unsigned int) * toff);
    S->cbuf[1] = (unsigned int*)pic_dev_alloc(ctx, sizeof(unsigned int) * toff);
    S->tile_fill = (unsigned int*)pic_dev_alloc(ctx, sizeof(unsigned int) * toff);
    if (!S->tile_count || !S->tstart[0] || !S->tstart[1] || !S->tile_lpre || !S->vtile || !S->tile_info ||
        !S->cbuf[0] || !S->cbuf[1] || !S->tile_fill)
        return f32_fail(ctx, PIC_ENOMEM, "FP32 tile tables");
    hipStream_t s = pic_stream(ctx);
    CK32(hipMemcpyAsync(S->tile_info, tinfo.data(), sizeof(int4) * toff, hipMemcpyHostToDevice, s));
    CK32(hipStreamSynchronize(s));
    const size_t lds = particle_lds(S->win_max, S->win3_max);
    // every workgroup of the statically balanced grid must be resident at
    // once; the counting and sorting steps share one grid (the sorting step
    // reads the counting step's records per workgroup), the plain step may
    // hold another number per CU
    int omin = 1 << 30, oplain = 1;
    for (int q = 0; q < 4; ++q) {  // the context's variants
        const void* f = (const void*)particle_kernel(q | (S->ins ? 4 : 0) | (S->cub ? 8 : 0), S->lanes);
        CK32(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int occ = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, kPWG, lds);
        if (q == 0) oplain = occ;
        else omin = std::min(omin, occ);
    }
    S->wg_per_cu = omin > 0 ? omin : 1;
    S->wg_per_cu_plain = oplain > 0 ? oplain : 1;
    S->crec = (unsigned int*)pic_dev_alloc(ctx, sizeof(unsigned int) * 9 * kRecMax * (size_t)S->cu * S->wg_per_cu);
    if (!S->crec) return f32_fail(ctx, PIC_ENOMEM, "FP32 chunk records");
    return PIC_OK;
}

// Particle stores for per-instance capacities caps (segments 64-slot aligned).
// With copy, the used slots of every instance move from the current store to
// the new one; the tile layout must then be rebuilt by a full sort.
static pic_status build_store(pic_ctx* ctx, F32State* S, const std::vector<long long>& caps, bool copy) {
    const int n = pic_n_inst(ctx);
    std::vector<long long> slots(n, 0), old_off(n, 0);
    if (copy) {
        std::vector<long long> cnt((size_t)n * C_NCOUNT);
        CK32(hipMemcpy(cnt.data(), pic_counters(ctx), sizeof(long long) * cnt.size(), hipMemcpyDeviceToHost));
        for (int k = 0; k < n; ++k) {
            slots[k] = cnt[(size_t)k * C_NCOUNT + C_SLOTS];
            old_off[k] = pic_inst_dev(ctx, k).p_off;
            if (slots[k] > caps[k]) return f32_fail(ctx, PIC_EINVAL, "capacity below the used slots");
        }
    }
    long long off = 0;
    std::vector<long long> new_off(n);
    for (int k = 0; k < n; ++k) {
        new_off[k] = off;
        off += (caps[k] + 63) / 64 * 64;
    }
    PSet ns[2] = {alloc_set(ctx, off), alloc_set(ctx, off)};
    unsigned long long* nkey = (unsigned long long*)pic_dev_alloc(ctx, sizeof(unsigned long long) * off);
    // collision candidates per step are binomial(N, P_null) and the real
    // events a part of them: size the queue far above the candidates' mean
    // (an overflow is reported, never ignored)
    double pmax = 0.0;
    for (int k = 0; k < n; ++k) pmax = std::max(pmax, pic_inst_dev(ctx, k).P_null);
    const long long qcap = std::min<long long>(off, std::max<long long>(1 << 16, (long long)(64.0 * pmax * (double)off)));
    // collision kernel grid: at most four expected candidates per thread
    S->coll_grid = (int)std::min<double>(4096.0, std::max(64.0, std::ceil(pmax * (double)off / (4.0 * kWG))));
    unsigned long long* nq = (unsigned long long*)pic_dev_alloc(ctx, sizeof(unsigned long long) * qcap);
    if (!set_ok(ns[0]) || !set_ok(ns[1]) || !nkey || !nq) {
        for (int b = 0; b < 2; ++b) free_set(ctx, ns[b]);
        pic_dev_free(ctx, nkey);
        pic_dev_free(ctx, nq);
        return f32_fail(ctx, PIC_ENOMEM, "FP32 particle stores");
    }
    hipStream_t s = pic_stream(ctx);
    if (copy) {
        // instances start on block boundaries, so whole blocks move
        const PSet& P = S->set[S->cur];
        for (int k = 0; k < n; ++k) {
            if (slots[k] <= 0) continue;
            CK32(hipMemcpyAsync(block_of(ns[0], new_off[k]), block_of(P, old_off[k]),
                                (size_t)blocks_for(slots[k]) * kBlkBytes, hipMemcpyDeviceToDevice, s));
            CK32(hipMemcpyAsync(ns[0].wt + new_off[k], P.wt + old_off[k], sizeof(float) * slots[k],
                                hipMemcpyDeviceToDevice, s));
        }
        CK32(hipStreamSynchronize(s));
    }
    for (int b = 0; b < 2; ++b) free_set(ctx, S->set[b]);
    pic_dev_free(ctx, S->sortkey);
    pic_dev_free(ctx, S->queue);
    S->set[0] = ns[0];
    S->set[1] = ns[1];
    S->cur = 0;
    S->sortkey = nkey;
    S->queue = nq;
    S->qcap = qcap;
    S->total_cap = off;
    for (int k = 0; k < n; ++k) {
        DevInst& I = pic_inst_dev(ctx, k);
        I.p_off = new_off[k];
        I.p_cap = caps[k];
    }
    return PIC_OK;
}

pic_status f32_init(pic_ctx* ctx) {
    F32State* S = new F32State();
    pic_set_f32(ctx, S);
    const pic_run_cfg& run = pic_run(ctx);
    if (run.tile_r > 0) S->TR = run.tile_r;
    if (run.tile_z > 0) S->TZ = run.tile_z;
    if (run.halo > 0) S->halo = run.halo;
    if (run.sort_interval > 0) S->K = run.sort_interval;
    if (run.chunk > 0) S->C = run.chunk;
    for (int k = 0; k < pic_n_inst(ctx); ++k) S->ins = S->ins || pic_inst_dev(ctx, k).has_ins != 0;
    S->cub = pic_inst_dev(ctx, 0).spline3 != 0;  // every instance of a context has the same shapes
    S->lanes = (run.lanes == 2 && !S->cub) ? 2 : 1;
    pic_status st = build_tiles(ctx, S);
    if (st != PIC_OK) return st;
    const int n = pic_n_inst(ctx);
    std::vector<long long> caps(n);
    for (int k = 0; k < n; ++k) caps[k] = pic_inst_dev(ctx, k).p_cap;
    st = build_store(ctx, S, caps, false);
    if (st != PIC_OK) return st;
    S->ctl = (long long*)pic_dev_alloc(ctx, sizeof(long long) * (CTL_TAIL + n + 1));
    pic_set_prep_ctl(ctx, S->ctl);
    S->inst_live = (long long*)pic_dev_alloc(ctx, sizeof(long long) * n);
    S->inst_voff = (long long*)pic_dev_alloc(ctx, sizeof(long long) * n);
    CK32(hipHostMalloc((void**)&S->h_cnt, sizeof(long long) * (size_t)n * C_NCOUNT, hipHostMallocDefault));
    if (!S->ctl || !S->inst_live || !S->inst_voff) return f32_fail(ctx, PIC_ENOMEM, "FP32 sort buffers");
    hipStream_t s = pic_stream(ctx);
    CK32(hipMemsetAsync(S->ctl, 0, sizeof(long long) * (CTL_TAIL + n + 1), s));
    CK32(hipStreamSynchronize(s));
    CK32(hipStreamCreateWithFlags(&S->gstream, hipStreamNonBlocking));
    CK32(hipEventCreateWithFlags(&S->ev_in, hipEventDisableTiming));
    CK32(hipEventCreateWithFlags(&S->ev_out, hipEventDisableTiming));
    CK32(hipEventCreateWithFlags(&S->ev_snap, hipEventDisableTiming));
    S->graphs = run.use_graph != 0;
    S->graph_auto = run.use_graph == 2;
    S->dF = pic_field_table(ctx);
    return PIC_OK;
}

static void drop_graphs(F32State* S) {
    for (int k = 0; k < 2; ++k) {
        for (int m = 0; m < 4; ++m) {
            if (S->g_step[m][k]) (void)hipGraphExecDestroy(S->g_step[m][k]);
            S->g_step[m][k] = nullptr;
        }
        if (S->g_cycle[k]) (void)hipGraphExecDestroy(S->g_cycle[k]);
        S->g_cycle[k] = nullptr;
    }
}

void f32_destroy(pic_ctx* ctx) {
    F32State* S = pic_get_f32(ctx);
    if (!S) return;
    drop_graphs(S);
    if (S->gstream) {
        (void)hipStreamSynchronize(S->gstream);
        (void)hipStreamDestroy(S->gstream);
    }
    if (S->ev_in) (void)hipEventDestroy(S->ev_in);
    if (S->ev_out) (void)hipEventDestroy(S->ev_out);
    if (S->ev_snap) {
        (void)hipEventSynchronize(S->ev_snap);
        (void)hipEventDestroy(S->ev_snap);
    }
    if (S->h_cnt) (void)hipHostFree(S->h_cnt);
    delete S;
    pic_set_f32(ctx, nullptr);
}

static long long max_slots(pic_ctx* ctx) {
    long long m = 0;
    for (int k = 0; k < pic_n_inst(ctx); ++k) m = std::max(m, pic_inst_dev(ctx, k).p_cap);
    return m;
}

// the launch sequences -------------------------------------------------------

static pic_status launch_step(pic_ctx* ctx, F32State* S, hipStream_t s, bool timed, int mode) {
    const int n = pic_n_inst(ctx);
    KArgs A = kargs(ctx, S, S->cur);
    long long max_nodes = 0;
    for (int k = 0; k < n; ++k) max_nodes = std::max<long long>(max_nodes, pic_inst_dev(ctx, k).nodes);
    hipLaunchKernelGGL(k_zero_q, dim3(grid_for(max_nodes / 8, 128), n), dim3(kWG), 0, s, A.It, A.Ft);
    CK32(hipGetLastError());
    const unsigned int tgrid = (unsigned int)((S->n_tiles + 255) / 256);
    if (mode & 2) {
        hipLaunchKernelGGL(k_zero_u32, dim3(tgrid), dim3(256), 0, s, S->tile_fill, S->n_tiles);
        CK32(hipGetLastError());
        hipLaunchKernelGGL(k_sort_plan1, dim3(n), dim3(kScanWG), 0, s, A.It, S->cbuf[S->cur], S->tstart[1 - S->cur],
                           S->tile_lpre, S->inst_live);
        CK32(hipGetLastError());
        hipLaunchKernelGGL(k_scatter_pre, dim3((n + 63) / 64), dim3(64), 0, s, A.cnt, n);
        CK32(hipGetLastError());
    }
    if (mode & 1) {
        const int oset = (mode & 2) ? 1 - S->cur : S->cur;
        A.cnt_out = S->cbuf[oset];
        hipLaunchKernelGGL(k_zero_u32, dim3(tgrid), dim3(256), 0, s, A.cnt_out, S->n_tiles);
        CK32(hipGetLastError());
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        e0 = pic_timing_begin(ctx, &e1);
        if (!e0) return f32_fail(ctx, PIC_EDEVICE, "event pool");
        CK32(hipEventRecord(e0, s));
    }
    const size_t lds = particle_lds(S->win_max, S->win3_max);
    const dim3 grid(S->cu * ((mode & 3) ? S->wg_per_cu : S->wg_per_cu_plain));
    hipLaunchKernelGGL(particle_kernel((mode & 3) | (S->ins ? 4 : 0) | (S->cub ? 8 : 0), S->lanes), grid, dim3(kPWG),
                       lds, s,
                       A);
    CK32(hipGetLastError());
    if (timed) CK32(hipEventRecord(e1, s));
    hipLaunchKernelGGL(k_collide, dim3(S->coll_grid), dim3(kWG), sizeof(unsigned int) * 2 * (size_t)n, s, A,
                       (mode & 2) ? S->set[1 - S->cur] : S->set[S->cur], (mode & 2) ? 1 : 0);
    CK32(hipGetLastError());
    double src_max = 0.0;
    for (int k = 0; k < n; ++k) src_max = std::max(src_max, pic_inst_dev(ctx, k).src_rate);
    if (src_max > 0.0) {
        hipLaunchKernelGGL(k_source32, dim3(grid_for((long long)ceil(src_max) + 1, 256), n), dim3(kWG), 0, s, A,
                           (mode & 2) ? S->set[1 - S->cur] : S->set[S->cur], (mode & 2) ? 1 : 0);
        CK32(hipGetLastError());
    }
    if (mode & 2) {
        hipLaunchKernelGGL(k_sort_plan2, dim3(1), dim3(kScanWG), 0, s, S->inst_live, S->inst_voff, S->ctl, S->vtile, n,
                           S->n_tiles);
        CK32(hipGetLastError());
        hipLaunchKernelGGL(k_sort_plan3, dim3(tgrid), dim3(256), 0, s, S->tile_info, S->n_tiles, S->tile_lpre,
                           S->inst_voff, S->vtile);
        CK32(hipGetLastError());
        hipLaunchKernelGGL(k_scatter_commit, dim3((n + 63) / 64), dim3(64), 0, s, A.cnt, S->inst_live, n);
        CK32(hipGetLastError());
    }
    return PIC_OK;
}

static pic_status launch_sort(pic_ctx* ctx, F32State* S, hipStream_t s) {
    const int n = pic_n_inst(ctx);
    KArgs A = kargs(ctx, S, S->cur);
    hipLaunchKernelGGL(k_zero_u32, dim3((S->n_tiles + 255) / 256), dim3(256), 0, s, S->tile_count, S->n_tiles);
    CK32(hipGetLastError());
    unsigned int gx = grid_for(max_slots(ctx), 2048);
    hipLaunchKernelGGL(k_sort_count, dim3(gx, n), dim3(kWG), 0, s, A, S->sortkey, S->tile_count);
    CK32(hipGetLastError());
    hipLaunchKernelGGL(k_sort_plan1, dim3(n), dim3(kScanWG), 0, s, A.It, S->tile_count, S->tstart[1 - S->cur],
                       S->tile_lpre, S->inst_live);
    CK32(hipGetLastError());
    hipLaunchKernelGGL(k_sort_plan2, dim3(1), dim3(kScanWG), 0, s, S->inst_live, S->inst_voff, S->ctl, S->vtile, n,
                       S->n_tiles);
    CK32(hipGetLastError());
    hipLaunchKernelGGL(k_sort_plan3, dim3((S->n_tiles + 255) / 256), dim3(256), 0, s, S->tile_info, S->n_tiles,
                       S->tile_lpre, S->inst_voff, S->vtile);
    CK32(hipGetLastError());
    hipLaunchKernelGGL(k_sort_scatter, dim3(gx, n), dim3(kWG), 0, s, A, S->set[1 - S->cur], S->sortkey,
                       S->tstart[1 - S->cur]);
    CK32(hipGetLastError());
    hipLaunchKernelGGL(k_sort_commit, dim3((n + 63) / 64), dim3(64), 0, s, A.cnt, S->inst_live, n);
    CK32(hipGetLastError());
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(64), 0, s, S->ctl, A.cnt, n);
    CK32(hipGetLastError());
    return PIC_OK;
}

static pic_status run_step_direct(pic_ctx* ctx, F32State* S, hipStream_t s, bool timed, int mode) {
    pic_status st = launch_step(ctx, S, s, timed, mode);
    if (st != PIC_OK) return st;
    return pic_field_stage(ctx, s);
}

static pic_status run_sort_direct(pic_ctx* ctx, F32State* S, hipStream_t s) {
    pic_status st = launch_sort(ctx, S, s);
    if (st != PIC_OK) return st;
    S->cur = 1 - S->cur;
    S->phase = 0;
    S->counted = false;
    return PIC_OK;
}

static pic_status capture_step(pic_ctx* ctx, F32State* S, int mode, int cur) {
    const int cur0 = S->cur;
    S->cur = cur;
    hipGraph_t g = nullptr;
    CK32(hipStreamBeginCapture(S->gstream, hipStreamCaptureModeThreadLocal));
    pic_status st = run_step_direct(ctx, S, S->gstream, false, mode);
    hipError_t e = hipStreamEndCapture(S->gstream, &g);
    S->cur = cur0;
    if (st != PIC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    CK32(e);
    e = hipGraphInstantiate(&S->g_step[mode][cur], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CK32(e);
    return PIC_OK;
}

// One graph for a whole sort cycle (K >= 2 steps starting right after a
// sort): K-2 plain steps, the counting step and the sorting step, so the
// host launches one graph per K steps.
static pic_status capture_cycle(pic_ctx* ctx, F32State* S, int cur) {
    const int cur0 = S->cur;
    S->cur = cur;
    hipGraph_t g = nullptr;
    CK32(hipStreamBeginCapture(S->gstream, hipStreamCaptureModeThreadLocal));
    pic_status st = PIC_OK;
    for (int p = 0; p < S->K && st == PIC_OK; ++p) {
        const int mode = p < S->K - 2 ? 0 : (p == S->K - 2 ? 1 : 2);
        st = run_step_direct(ctx, S, S->gstream, false, mode);
    }
    hipError_t e = hipStreamEndCapture(S->gstream, &g);
    S->cur = cur0;
    if (st != PIC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    CK32(e);
    e = hipGraphInstantiate(&S->g_cycle[cur], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CK32(e);
    return PIC_OK;
}

pic_status f32_sort_now(pic_ctx* ctx) {
    F32State* S = pic_get_f32(ctx);
    return run_sort_direct(ctx, S, pic_stream(ctx));
}

// Step kind from the sort schedule: every K steps a scatter (mode bit 2),
// preceded by a step that counts the tile totals it needs (mode bit 1).
static int next_mode(const F32State* S) {
    if (S->K == 1) return S->counted ? 3 : 1;
    if (S->phase >= S->K - 1) return S->counted ? 2 : 1;
    if (S->phase == S->K - 2) return 1;
    return 0;
}

// Every particle counts as unsorted again and one full sort rebuilds the
// layout (after the tiles or the stores changed).
static pic_status resort_all(pic_ctx* ctx, F32State* S) {
    hipStream_t s = pic_stream(ctx);
    const int n = pic_n_inst(ctx);
    CK32(hipStreamSynchronize(s));
    for (int k = 0; k < n; ++k) {
        long long zero = 0;
        CK32(hipMemcpy(pic_counters(ctx) + (long long)k * C_NCOUNT + C_LIVE_SORTED, &zero, sizeof(zero),
                       hipMemcpyHostToDevice));
    }
    pic_status st = pic_upload_inst(ctx);
    if (st != PIC_OK) return st;
    st = run_sort_direct(ctx, S, s);
    if (st != PIC_OK) return st;
    CK32(hipStreamSynchronize(s));
    return PIC_OK;
}

static pic_status quiesce(pic_ctx* ctx, F32State* S) {
    CK32(hipStreamSynchronize(pic_stream(ctx)));
    if (S->gstream) CK32(hipStreamSynchronize(S->gstream));
    if (S->snap_pending) CK32(hipEventSynchronize(S->ev_snap));  // the copy stays valid
    drop_graphs(S);
    return PIC_OK;
}

// The null-collision probability of an instance changed (tabulated cross
// sections): size the candidate queue and the collision grid again.
pic_status f32_rates_changed(pic_ctx* ctx) {
    F32State* S = pic_get_f32(ctx);
    pic_status st = quiesce(ctx, S);
    if (st != PIC_OK) return st;
    double pmax = 0.0;
    for (int k = 0; k < pic_n_inst(ctx); ++k) pmax = std::max(pmax, pic_inst_dev(ctx, k).P_null);
    const long long off = S->total_cap;
    const long long qcap = std::min<long long>(off, std::max<long long>(1 << 16, (long long)(64.0 * pmax * (double)off)));
    if (qcap > S->qcap) {
        unsigned long long* nq = (unsigned long long*)pic_dev_alloc(ctx, sizeof(unsigned long long) * qcap);
        if (!nq) return f32_fail(ctx, PIC_ENOMEM, "collision queue");
        pic_dev_free(ctx, S->queue);
        S->queue = nq;
        S->qcap = qcap;
    }
    S->coll_grid = (int)std::min<double>(4096.0, std::max(64.0, std::ceil(pmax * (double)off / (4.0 * kWG))));
    return PIC_OK;
}


// New tiles, halo, sort interval and launch shape (lanes 1 or 2; 0 keeps
// it): the tile tables rebuilt and every particle re-sorted.  PIC_EINVAL
// leaves the context as it was.
static pic_status reconfigure(pic_ctx* ctx, int lanes, int tile_r, int tile_z, int halo, int sort_interval) {
    F32State* S = pic_get_f32(ctx);
    pic_status st = quiesce(ctx, S);
    if (st != PIC_OK) return st;
    const int old[5] = {S->TR, S->TZ, S->halo, S->K, S->lanes};
    if (tile_r > 0) S->TR = tile_r;
    if (tile_z > 0) S->TZ = tile_z;
    if (halo >= 0) S->halo = halo;
    if (sort_interval > 0) S->K = sort_interval;
    if (lanes > 0 && !S->cub) S->lanes = lanes;
    st = build_tiles(ctx, S);
    if (st == PIC_EINVAL) {  // rejected before anything changed
        S->TR = old[0]; S->TZ = old[1]; S->halo = old[2]; S->K = old[3]; S->lanes = old[4];
        return st;
    }
    if (st != PIC_OK) return st;
    return resort_all(ctx, S);
}

pic_status f32_retune(pic_ctx* ctx, int tile_r, int tile_z, int halo, int sort_interval) {
    return reconfigure(ctx, 0, tile_r, tile_z, halo, sort_interval);
}

pic_status f32_reserve(pic_ctx* ctx, int k, long long slots) {
    F32State* S = pic_get_f32(ctx);
    const int n = pic_n_inst(ctx);
    std::vector<long long> caps(n);
    for (int j = 0; j < n; ++j) caps[j] = pic_inst_dev(ctx, j).p_cap;
    if (slots <= caps[k]) return PIC_OK;
    caps[k] = slots;
    pic_status st = quiesce(ctx, S);
    if (st != PIC_OK) return st;
    st = build_store(ctx, S, caps, true);
    if (st != PIC_OK) return st;
    for (int j = 0; j < n; ++j) pic_inst_cap(ctx, j) = caps[j];
    return resort_all(ctx, S);
}

// Capacity check, a lagged one so the stream never drains: the counters are
// copied to pinned memory every kCheckEvery steps and the previous copy is
// inspected.  Its used slots, grown for two check periods at the rate seen
// since the copy before (and by the seed source), must stay under 3/4 of the
// segment, else the instance is grown to twice that projection (new stores,
// copy, full sort, graphs re-captured).  The first check of a context looks
// at the current counters.  Dropped electrons or a fixed-point overflow in
// the copy end the step call with an error.
constexpr int kCheckEvery = 64;

static pic_status capacity_check(pic_ctx* ctx, F32State* S, hipStream_t work) {
    const int n = pic_n_inst(ctx);
    if (!S->checked_once) {
        // the first check of a context inspects the current counters at once
        S->checked_once = true;
        CK32(hipMemcpyAsync(S->h_cnt, pic_counters(ctx), sizeof(long long) * (size_t)n * C_NCOUNT,
                            hipMemcpyDeviceToHost, work));
        CK32(hipEventRecord(S->ev_snap, work));
        S->snap_pending = true;
    }
    if (S->snap_pending) {
        CK32(hipEventSynchronize(S->ev_snap));
        S->snap_pending = false;
        if ((int)S->prev_used.size() != n) S->prev_used.assign(n, -1);
        std::vector<long long> caps(n);
        bool grow = false;
        for (int k = 0; k < n; ++k) {
            const long long* c = S->h_cnt + (size_t)k * C_NCOUNT;
            if (c[C_DROPPED] > 0)
                return f32_fail(ctx, PIC_ECAPACITY, "instance " + std::to_string(k) + ": new electrons dropped");
            if (c[C_OVERFLOW] > 0)
                return f32_fail(ctx, PIC_EOVERFLOW, "instance " + std::to_string(k) + ": fixed-point overflow");
            if (c[C_NONFIN] > 0)
                return f32_fail(ctx, PIC_ENONFINITE,
                                "instance " + std::to_string(k) + ": particles with a non-finite position removed");
            const long long cap = pic_inst_dev(ctx, k).p_cap;
            const long long used = c[C_SLOTS];
            // the lag spans up to two check periods: growth at the rate seen
            // between the last two copies (compounded), at least the seed source's
            const double f = S->prev_used[k] > 0 ? std::min(4.0, std::max(1.0, (double)used / S->prev_used[k])) : 1.0;
            const long long proj =
                std::max((long long)((double)used * f * f),
                         used + 2 * (long long)ceil(pic_inst_dev(ctx, k).src_rate) * kCheckEvery);
            S->prev_used[k] = used;
            caps[k] = cap;
            if (proj > cap - cap / 4) {
                caps[k] = std::max<long long>(2 * proj, cap + cap / 2);
                grow = true;
            }
        }
        if (grow) {
            pic_status st = quiesce(ctx, S);
            if (st != PIC_OK) return st;
            st = build_store(ctx, S, caps, true);
            if (st != PIC_OK) return st;
            for (int k = 0; k < n; ++k) pic_inst_cap(ctx, k) = caps[k];
            st = resort_all(ctx, S);
            if (st != PIC_OK) return st;
            S->grow_events += 1;
        }
    }
    CK32(hipMemcpyAsync(S->h_cnt, pic_counters(ctx), sizeof(long long) * (size_t)n * C_NCOUNT,
                        hipMemcpyDeviceToHost, work));
    CK32(hipEventRecord(S->ev_snap, work));
    S->snap_pending = true;
    return PIC_OK;
}

pic_status f32_step(pic_ctx* ctx, int n_steps) {
    F32State* S = pic_get_f32(ctx);
    hipStream_t s = pic_stream(ctx);
    const bool timed = pic_timing_on(ctx);
    const bool use_graph = S->graphs && !timed;
    bool waited = false;
    for (int it = 0; it < n_steps;) {
        if (!S->checked_once || S->since_check >= kCheckEvery) {
            if (use_graph && waited) {
                // bring the caller's stream up to date before a possible regrowth
                CK32(hipEventRecord(S->ev_out, S->gstream));
                CK32(hipStreamWaitEvent(s, S->ev_out, 0));
                waited = false;
            }
            pic_status st = capacity_check(ctx, S, s);
            if (st != PIC_OK) return st;
            S->since_check = 0;
        }
        // a whole sort cycle as one graph when the schedule is at its start
        const bool cycle = use_graph && S->K >= 2 && S->phase == 0 && !S->counted && n_steps - it >= S->K;
        if (cycle || use_graph) {
            hipGraphExec_t* g = cycle ? &S->g_cycle[S->cur] : &S->g_step[next_mode(S)][S->cur];
            if (!*g) {
                CK32(hipStreamSynchronize(s));
                CK32(hipStreamSynchronize(S->gstream));
                pic_status st = cycle ? capture_cycle(ctx, S, S->cur) : capture_step(ctx, S, next_mode(S), S->cur);
                if (st != PIC_OK) return st;
            }
            if (!waited) {
                CK32(hipEventRecord(S->ev_in, s));
                CK32(hipStreamWaitEvent(S->gstream, S->ev_in, 0));
                waited = true;
            }
            CK32(hipGraphLaunch(*g, S->gstream));
        }
        if (cycle) {
            S->cur = 1 - S->cur;
            S->phase = 0;
            S->counted = false;
            it += S->K;
            S->since_check += S->K;
            continue;
        }
        const int mode = next_mode(S);
        if (!use_graph) {
            pic_status st = run_step_direct(ctx, S, s, timed, mode);
            if (st != PIC_OK) return st;
        }
        S->counted = (mode & 1) != 0;
        if (mode & 2) {
            S->cur = 1 - S->cur;
            S->phase = 0;
        } else {
            S->phase += 1;
        }
        it += 1;
        S->since_check += 1;
    }
    if (use_graph && waited) {
        CK32(hipEventRecord(S->ev_out, S->gstream));
        CK32(hipStreamWaitEvent(s, S->ev_out, 0));
    }
    return PIC_OK;
}

// ---- autotuner ---------------------------------------------------------------
// Times the real workload under candidate tile shapes, halos and sort
// intervals (coordinate search: tile shape, then halo, then interval), for
// each launch shape of the particle kernel (one or two particles per lane
// and pass), and keeps the fastest.  Every result of the method is independent of these
// choices (bit-identical), so the trial steps are ordinary steps of the run.
// A cache file holds one JSON object per line keyed by a workload signature.

static std::string tune_signature(pic_ctx* ctx) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    const int n = pic_n_inst(ctx);
    std::vector<long long> cnt((size_t)n * C_NCOUNT);
    (void)hipStreamSynchronize(pic_stream(ctx));
    (void)hipMemcpy(cnt.data(), pic_counters(ctx), sizeof(long long) * cnt.size(), hipMemcpyDeviceToHost);
    std::string sig = arch + ";" + std::to_string(n);
    for (int k = 0; k < n; ++k) {
        const DevInst& I = pic_inst_dev(ctx, k);
        const long long live = cnt[(size_t)k * C_NCOUNT + C_SLOTS] - cnt[(size_t)k * C_NCOUNT + C_DEAD];
        int lb = 0;
        while ((1ll << (lb + 1)) <= std::max(live, 1ll)) ++lb;
        sig += ";" + std::to_string(I.nr) + "x" + std::to_string(I.nz) + ":" + std::to_string(lb);
    }
    return sig;
}

static bool tune_lookup(const char* path, const std::string& sig, int v[4], int* lanes, int* graphs) {
    FILE* f = path ? fopen(path, "r") : nullptr;
    if (!f) return false;
    char line[4096];
    const std::string key = "\"sig\": \"" + sig + "\"";
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        std::string l(line);
        if (l.find(key) == std::string::npos) continue;
        const char* names[4] = {"\"tile_r\": ", "\"tile_z\": ", "\"halo\": ", "\"sort_interval\": "};
        bool ok = true;
        for (int i = 0; i < 4; ++i) {
            size_t at = l.find(names[i]);
            if (at == std::string::npos) { ok = false; break; }
            v[i] = atoi(l.c_str() + at + strlen(names[i]));
        }
        if (ok) {
            found = true;
            const char* lk = "\"lanes\": ";
            const size_t at = l.find(lk);
            *lanes = at == std::string::npos ? 1 : atoi(l.c_str() + at + strlen(lk));
            const char* gk = "\"graphs\": ";
            const size_t ag = l.find(gk);
            *graphs = ag == std::string::npos ? -1 : atoi(l.c_str() + ag + strlen(gk));
        }
    }
    fclose(f);
    return found;
}

pic_status f32_autotune(pic_ctx* ctx, int trial_steps, const char* cache, int out[4], double* ms_out,
                        int* trials_out) {
    F32State* S = pic_get_f32(ctx);
    const std::string sig = tune_signature(ctx);
    int v[4], lanes = 1, graphs = -1;
    if (tune_lookup(cache, sig, v, &lanes, &graphs)) {
        pic_status st = reconfigure(ctx, lanes == 2 ? 2 : 1, v[0], v[1], v[2], v[3]);
        if (st != PIC_OK) return st;
        if (S->graph_auto && graphs >= 0) S->graphs = graphs != 0;
        for (int i = 0; i < 4; ++i) out[i] = v[i];
        if (ms_out) *ms_out = 0.0;
        if (trials_out) *trials_out = 0;
        return PIC_OK;
    }
    hipStream_t s = pic_stream(ctx);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EventPair {  // destroyed on every way out
        hipEvent_t* a;
        hipEvent_t* b;
        ~EventPair() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } guard{&e0, &e1};
    CK32(hipEventCreate(&e0));
    CK32(hipEventCreate(&e1));
    int trials = 0;
    const int n = pic_n_inst(ctx);
    std::vector<long long> cnt((size_t)n * C_NCOUNT);
    auto psteps = [&]() -> long long {
        // the steps ran on the library's graph stream, joined to the context stream
        if (hipStreamSynchronize(pic_stream(ctx)) != hipSuccess) return 0;
        if (hipMemcpy(cnt.data(), pic_counters(ctx), sizeof(long long) * cnt.size(), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return 0;
        long long t = 0;
        for (int k = 0; k < n; ++k) t += cnt[(size_t)k * C_NCOUNT + C_PSTEPS];
        return t;
    };
    // one candidate: particles per lane and pass, tile shape, halo, sort interval
    typedef std::array<int, 5> Cand;
    auto trial = [&](const Cand& c, double& ms) -> pic_status {
        ms = 1e30;
        pic_status st = reconfigure(ctx, c[0], c[1], c[2], c[3], c[4]);
        if (st == PIC_EINVAL) return PIC_OK;  // does not fit: skipped
        if (st != PIC_OK) return st;
        const int K = c[4];
        st = f32_step(ctx, 2 * K);  // every step kind captured and warm
        if (st != PIC_OK) return st;
        const int T = ((std::max(trial_steps, 2 * K) + K - 1) / K) * K;
        const long long ps0 = psteps();
        CK32(hipEventRecord(e0, s));
        st = f32_step(ctx, T);
        if (st != PIC_OK) return st;
        CK32(hipEventRecord(e1, s));
        CK32(hipEventSynchronize(e1));
        float t = 0.0f;
        CK32(hipEventElapsedTime(&t, e0, e1));
        // per particle-step, so a population that changes between trials
        // does not bias the comparison; reported per step at the final count
        const long long ps = std::max(1ll, psteps() - ps0);
        ms = (double)t / (double)ps;
        ++trials;
        return PIC_OK;
    };
    Cand best = {S->lanes, S->TR, S->TZ, S->halo, S->K};
    double best_ms = 1e30;
    pic_status st = PIC_OK;
    const bool verbose = getenv("PICMCC_TUNE_LOG") != nullptr;  // trial log on stderr
    std::vector<Cand> tried;
    std::vector<double> tried_ms;
    auto consider = [&](const Cand& c) {
        if (st != PIC_OK || std::find(tried.begin(), tried.end(), c) != tried.end()) return;
        double ms;
        st = trial(c, ms);
        tried.push_back(c);
        tried_ms.push_back(ms);
        if (verbose)
            fprintf(stderr, "autotune: %d per lane, tile %dx%d halo %d sort %d: %.4g ps per particle-step%s\n", c[0],
                    c[1], c[2], c[3], c[4], ms * 1e9, ms >= 1e29 ? " (does not fit)" : "");
        if (st == PIC_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    };
    // (the last three fit the LDS with two particles per lane only)
    const int shapes[][2] = {{8, 32}, {8, 8}, {8, 16}, {16, 8}, {16, 16}, {32, 8}, {16, 32},
                             {32, 16}, {32, 32}, {8, 64}, {16, 64}, {4, 64}, {4, 32},
                             {32, 64}, {16, 128}, {64, 32}};
    const int halos[] = {2, 4, 8, 12};
    const int Ks[] = {4, 8, 16, 32};
    // coordinate search, twice, for each launch shape of the particle kernel
    // (cubic shapes have one), each starting from the best found so far
    for (int lanes = 1; lanes <= (S->cub ? 1 : 2); ++lanes)
        for (int round = 0; round < 2; ++round) {
            for (auto& sh : shapes) consider({lanes, sh[0], sh[1], best[3], best[4]});
            for (int h : halos) consider({lanes, best[1], best[2], h, best[4]});
            for (int K : Ks) consider({lanes, best[1], best[2], best[3], K});
        }
    // The run evolves while the trials go on, which biases trials far apart
    // in time: the four best are timed again, interleaved, twice each, and
    // the lowest mean of those repeats wins.
    if (st == PIC_OK && tried.size() > 1) {
        std::vector<int> order(tried.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return tried_ms[a] < tried_ms[b]; });
        const int top = std::min<int>(4, (int)order.size());
        std::vector<double> sum(top, 0.0);
        for (int rep = 0; rep < 2 && st == PIC_OK; ++rep)
            for (int c = 0; c < top && st == PIC_OK; ++c) {
                const Cand& v = tried[order[c]];
                double ms;
                st = trial(v, ms);
                sum[c] += ms;
                if (verbose)
                    fprintf(stderr, "autotune: repeat %d per lane, tile %dx%d halo %d sort %d: %.4g ps per particle-step\n",
                            v[0], v[1], v[2], v[3], v[4], ms * 1e9);
            }
        if (st == PIC_OK) {
            int bc = 0;
            for (int c = 1; c < top; ++c)
                if (sum[c] < sum[bc]) bc = c;
            best = tried[order[bc]];
            best_ms = sum[bc] / 2.0;
        }
    }
    if (st != PIC_OK) return st;
    st = reconfigure(ctx, best[0], best[1], best[2], best[3], best[4]);
    if (st != PIC_OK) return st;
    if (S->graph_auto) {
        // the launch mode on the chosen tiles: captured graphs against plain
        // launches, interleaved, twice each, per particle-step; the lower sum wins
        const int K = best[4];
        const int T = ((std::max(trial_steps, 2 * K) + K - 1) / K) * K;
        double sum[2] = {0.0, 0.0};
        for (int rep = 0; rep < 2; ++rep)
            for (int g = 1; g >= 0; --g) {
                S->graphs = g != 0;
                st = f32_step(ctx, 2 * K);
                if (st != PIC_OK) return st;
                const long long ps0 = psteps();
                CK32(hipEventRecord(e0, s));
                st = f32_step(ctx, T);
                if (st != PIC_OK) return st;
                CK32(hipEventRecord(e1, s));
                CK32(hipEventSynchronize(e1));
                float t = 0.0f;
                CK32(hipEventElapsedTime(&t, e0, e1));
                sum[g] += (double)t / (double)std::max(1ll, psteps() - ps0);
                ++trials;
            }
        S->graphs = sum[1] <= sum[0];
        if (verbose)
            fprintf(stderr, "autotune: graphs %.4g, plain launches %.4g ps per particle-step\n", sum[1] * 0.5e9,
                    sum[0] * 0.5e9);
    }
    for (int i = 0; i < 4; ++i) out[i] = best[i + 1];
    long long live = 0;
    (void)psteps();
    for (int k = 0; k < n; ++k) live += cnt[(size_t)k * C_NCOUNT + C_SLOTS] - cnt[(size_t)k * C_NCOUNT + C_DEAD];
    best_ms *= (double)std::max(1ll, live);
    if (ms_out) *ms_out = best_ms;
    if (trials_out) *trials_out = trials;
    if (cache) {
        FILE* f = fopen(cache, "a");
        if (f) {
            fprintf(f, "{\"sig\": \"%s\", \"tile_r\": %d, \"tile_z\": %d, \"halo\": %d, \"sort_interval\": %d, "
                       "\"lanes\": %d, \"graphs\": %d, \"ms_per_step\": %.6f, \"trials\": %d}\n",
                    sig.c_str(), best[1], best[2], best[3], best[4], best[0], S->graphs ? 1 : 0, best_ms, trials);
            fclose(f);
        }
    }
    return PIC_OK;
}

long long f32_grow_events(pic_ctx* ctx) { return pic_get_f32(ctx)->grow_events; }

pic_status f32_load(pic_ctx* ctx, int k) {
    F32State* S = pic_get_f32(ctx);
    const pic_instance_cfg& c = pic_inst_cfg(ctx, k);
    const DevInst& I = pic_inst_dev(ctx, k);
    if (c.n_init <= 0) return PIC_OK;
    double sv = sqrt((c.T_init_eV * kE) / kMe);
    hipLaunchKernelGGL(k_load32, dim3(grid_for(c.n_init)), dim3(kWG), 0, pic_stream(ctx), I, c.r_lo, c.r_hi,
                       c.z_lo, c.z_hi, sv, (float)c.weight, c.load_mode, S->set[S->cur], (long long)c.n_init);
    CK32(hipGetLastError());
    return PIC_OK;
}

pic_status f32_deposit_only(pic_ctx* ctx, int k) {
    F32State* S = pic_get_f32(ctx);
    const DevInst& I = pic_inst_dev(ctx, k);
    hipLaunchKernelGGL(k_deposit32, dim3(grid_for(I.p_cap)), dim3(kWG), 0, pic_stream(ctx), I, S->set[S->cur],
                       pic_inst_Q(ctx, k), I.has_ins ? pic_inst_Qw(ctx, k) : nullptr,
                       I.spline3 ? pic_inst_Qx(ctx, k) : nullptr, pic_counters(ctx) + (long long)k * C_NCOUNT);
    CK32(hipGetLastError());
    return PIC_OK;
}

pic_status f32_set_particles(pic_ctx* ctx, int k, long long n, const double* r, const double* z,
                             const double* vr, const double* vt, const double* vz, const double* w,
                             const unsigned long long* key) {
    F32State* S = pic_get_f32(ctx);
    const DevInst& I = pic_inst_dev(ctx, k);
    if (n <= 0) {
        pic_inst_dev(ctx, k).w_uni = (float)I.weight;
        return pic_upload_inst(ctx);
    }
    // the instance's first blocks, built on the host (slots past n in the
    // last block are marked dead and never read)
    const PSet& P = S->set[S->cur];
    const long long nb = blocks_for(n);
    std::vector<unsigned int> blk((size_t)(nb * kBlkWords), 0u);
    const double* src[5] = {r, z, vr, vt, vz};
    for (long long q = 0; q < nb * kBlkSlots; ++q) {
        unsigned int* b = blk.data() + (q / kBlkSlots) * kBlkWords;
        const int l = (int)(q % kBlkSlots);
        for (int c = 0; c < 5; ++c) {
            const float v = q < n ? (float)src[c][q] : (c == 0 ? -1.0f : 0.0f);
            memcpy(b + c * kBlkSlots + l, &v, 4);
        }
        const unsigned long long kq = q < n ? key[q] : 0ull;
        memcpy(b + 5 * kBlkSlots + 2 * l, &kq, 8);
    }
    CK32(hipMemcpy(block_of(P, I.p_off), blk.data(), (size_t)nb * kBlkBytes, hipMemcpyHostToDevice));
    std::vector<float> wf((size_t)n);
    for (long long q = 0; q < n; ++q) wf[q] = (float)w[q];
    CK32(hipMemcpy(P.wt + I.p_off, wf.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    // a common weight lets the particle loop skip the weight array; the seed
    // source adds electrons of the configured weight, so with the source on
    // the common weight must be that one
    const float w0 = (float)w[0];
    bool uni = !(I.src_rate > 0.0) || w0 == (float)I.weight;
    for (long long q = 1; q < n && uni; ++q) uni = (float)w[q] == w0;
    pic_inst_dev(ctx, k).w_uni = uni ? w0 : 0.0f;
    return pic_upload_inst(ctx);
}

pic_status f32_get_particles(pic_ctx* ctx, int k, double* r, double* z, double* vr, double* vt, double* vz,
                             double* w, unsigned long long* key, long long cap, long long* n_out) {
    F32State* S = pic_get_f32(ctx);
    const DevInst& I = pic_inst_dev(ctx, k);
    long long slots = 0;
    CK32(hipMemcpy(&slots, pic_counters(ctx) + (long long)k * C_NCOUNT + C_SLOTS, sizeof(long long),
                   hipMemcpyDeviceToHost));
    const PSet& P = S->set[S->cur];
    const long long nb = blocks_for(slots);
    std::vector<unsigned int> blk((size_t)std::max(nb * kBlkWords, 1ll));
    std::vector<float> wf((size_t)std::max(slots, 1ll), I.w_uni);
    if (slots > 0) {
        CK32(hipMemcpy(blk.data(), block_of(P, I.p_off), (size_t)nb * kBlkBytes, hipMemcpyDeviceToHost));
        if (I.w_uni == 0.0f)
            CK32(hipMemcpy(wf.data(), P.wt + I.p_off, sizeof(float) * slots, hipMemcpyDeviceToHost));
    }
    double* out[5] = {r, z, vr, vt, vz};
    long long m = 0;
    for (long long q = 0; q < slots; ++q) {
        const unsigned int* b = blk.data() + (q / kBlkSlots) * kBlkWords;
        const int l = (int)(q % kBlkSlots);
        float v[5];
        for (int c = 0; c < 5; ++c) memcpy(&v[c], b + c * kBlkSlots + l, 4);
        if (v[0] < 0.0f) continue;
        if (m < cap) {
            for (int c = 0; c < 5; ++c)
                if (out[c]) out[c][m] = (double)v[c];
            if (w) w[m] = (double)wf[q];
            if (key) memcpy(&key[m], b + 5 * kBlkSlots + 2 * l, 8);
        }
        ++m;
    }
    if (n_out) *n_out = m;
    if (m > cap) return f32_fail(ctx, PIC_EINVAL, "cap smaller than the live count");
    return PIC_OK;
}

long long f32_live_count(pic_ctx*, int, const long long* c) { return c[C_SLOTS] - c[C_DEAD]; }

pic_status f32_check(pic_ctx* ctx) {
    F32State* S = pic_get_f32(ctx);
    long long over = 0;
    CK32(hipMemcpy(&over, S->ctl + CTL_QOVER, sizeof(long long), hipMemcpyDeviceToHost));
    if (over) return f32_fail(ctx, PIC_ECAPACITY, "collision event queue overflowed");
    return PIC_OK;
}

pic_status f32_tuning(pic_ctx* ctx, int* tile_r, int* tile_z, int* halo, int* sort_interval, int* chunk,
                      int* lanes, int* use_graph) {
    F32State* S = pic_get_f32(ctx);
    if (lanes) *lanes = S->lanes;
    if (use_graph) *use_graph = S->graphs ? 1 : 0;
    if (tile_r) *tile_r = S->TR;
    if (tile_z) *tile_z = S->TZ;
    if (halo) *halo = S->halo;
    if (sort_interval) *sort_interval = S->K;
    if (chunk) *chunk = S->C;
    return PIC_OK;
}

pic_status f32_moments(pic_ctx* ctx, int k, double* acc) {
    F32State* S = pic_get_f32(ctx);
    const DevInst& I = pic_inst_dev(ctx, k);
    hipLaunchKernelGGL(k_moments32, dim3(grid_for(I.p_cap)), dim3(kWG), 0, pic_stream(ctx), I, S->set[S->cur],
                       pic_counters(ctx) + (long long)k * C_NCOUNT, acc);
    CK32(hipGetLastError());
    return PIC_OK;
}
