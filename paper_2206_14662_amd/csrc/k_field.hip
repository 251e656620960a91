// k_field.hip -- FP64 field stage shared by both forms: fixed-point charge
// -> order-1 FEM load -> Poisson solve -> nodal E, and the diagnostics
// sampling.  Instances are batched along gridDim.y through device tables.
//
// The interior FEM system (Kr (x) Mz + Mr (x) Kz) phi = b / eps0 with
// homogeneous Dirichlet data is diagonalised in z by the discrete sine
// transform (the eigenvectors of Kz and Mz on a uniform mesh), leaving one
// tridiagonal system in r per sine mode.  The sine transform of two rows at
// once is one complex FFT of length 2 nz of their odd extensions, done in LDS.
#include "pic_internal.h"

namespace pic {
namespace {

// The FFT block has N/8 threads for the largest N = 2 nz of the batch (at
// least 64): every thread holds 8 points per pass.
constexpr int kFftMaxBlock = 1024;
inline int fft_block(int max_nz) { return 2 * max_nz / 8 > 64 ? 2 * max_nz / 8 : 64; }
// Nodes per thread and row in the load and store phases of the z transform:
// the block holds at least nz / 4 threads, so for nz >= 4 one round covers
// the nz + 1 nodes of a row.
constexpr int kRowPer = 5;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }  // times -i

// Forward DFTs of 2, 4 and 8 points in registers (natural order in and out,
// kernel exp(-2 pi i r m / R)).
__device__ __forceinline__ void dft2(double2* v) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}
__device__ __forceinline__ void dft8(double2* v) {
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const double c = 0.70710678118654752440;  // sqrt(1/2)
    o1 = make_double2(c * (o1.x + o1.y), c * (o1.y - o1.x));    // times (1 - i)/sqrt 2
    o2 = mul_mi(o2);                                            // times -i
    o3 = make_double2(c * (o3.y - o3.x), -c * (o3.x + o3.y));   // times (-1 - i)/sqrt 2
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// Forward DFTs of 3 and 5 points (kernel exp(-2 pi i r m / R)): with
// c_l = cos(2 pi l / R), s_l = sin(2 pi l / R), pairs of inputs r and R - r
// enter as their sum (times c) and difference (times -i s).
__device__ __forceinline__ void dft3(double2* v) {
    const double s1 = 0.86602540378443864676;  // sin(2 pi / 3)
    const double2 t = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const double2 b = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    const double2 e = make_double2(s1 * d.y, -s1 * d.x);  // -i s1 d
    v[0] = cadd(v[0], t);
    v[1] = cadd(b, e);
    v[2] = csub(b, e);
}
__device__ __forceinline__ void dft5(double2* v) {
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;  // cos(2 pi / 5), cos(4 pi / 5)
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;   // sin(2 pi / 5), sin(4 pi / 5)
    const double2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const double2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const double2 b1 = make_double2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    const double2 b2 = make_double2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    const double2 d1 = make_double2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    const double2 d2 = make_double2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = make_double2(b1.x + d1.y, b1.y - d1.x);  // b1 - i d1
    v[4] = make_double2(b1.x - d1.y, b1.y + d1.x);  // b1 + i d1
    v[2] = make_double2(b2.x + d2.y, b2.y - d2.x);
    v[3] = make_double2(b2.x - d2.y, b2.y + d2.x);
}

// LDS slot of FFT point i: one spare slot after every 8 points, so that the
// first pass's writes (8 consecutive points per thread, threads 128 bytes
// apart) spread over the banks instead of falling on the same four.
__device__ __forceinline__ int lp(int i) { return i + (i >> 3); }
inline size_t fft_lds_bytes(int max_nz) { return sizeof(double2) * (size_t)(2 * max_nz + (2 * max_nz) / 8); }

// One Stockham pass of radix R over N points in LDS (in place: every
// thread reads its butterflies' inputs -- at most ceil(8 / R) of them, the
// block holding at least N / 8 threads -- barrier, writes).  Butterfly j of
// span Ns reads y[j + r N/R], twiddles input r by exp(-2 pi i r k / (Ns R))
// with k = j mod Ns, and writes output m to y[(j/Ns) Ns R + k + m Ns].
// tw[t] = exp(-2 pi i t / tw_n) over the full circle, tw_n a multiple of N.
// Only the first twiddle of a butterfly is read from the table; the others
// are its powers, so a pass waits on one table read instead of R - 1 (the
// powers round within a few ulp).
template <int R>
__device__ __forceinline__ void fft_pass(double2* y, int N, int Ns, const double2* __restrict__ tw, int tw_n) {
    constexpr int PER = (8 + R - 1) / R;
    const int nb = N / R;
    double2 v[PER * R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = threadIdx.x + q * blockDim.x;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q * R + r] = y[lp(j + r * nb)];
        }
    }
    __syncthreads();
    const int tscale = (tw_n / N) * (N / (Ns * R));
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = threadIdx.x + q * blockDim.x;
        if (j < nb) {
            const int k = j - (j / Ns) * Ns;
            double2* w = v + q * R;
            const double2 w1 = tw[k * tscale];
            double2 wp = w1;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                w[r] = cmul(w[r], wp);
                wp = cmul(wp, w1);
            }
            if (R == 8) dft8(w);
            else if (R == 5) dft5(w);
            else if (R == 4) dft4(w[0], w[1], w[2], w[3]);
            else if (R == 3) dft3(w);
            else dft2(w);
            const int d = (j - k) * R + k;
#pragma unroll
            for (int m = 0; m < R; ++m) y[lp(d + m * Ns)] = w[m];
        }
    }
    __syncthreads();
}

// Forward FFT of N = 2^a 3^b 5^c points (N a multiple of 8) in natural
// order in LDS: radix-8 passes while 8 divides what is left, then radix 4
// or 2, then the radix-3 and radix-5 passes.
__device__ void fft_lds(double2* y, int N, const double2* __restrict__ tw, int tw_n) {
    int Ns = 1;
    while ((N / Ns) % 8 == 0) {
        fft_pass<8>(y, N, Ns, tw, tw_n);
        Ns *= 8;
    }
    if ((N / Ns) % 4 == 0) {
        fft_pass<4>(y, N, Ns, tw, tw_n);
        Ns *= 4;
    } else if ((N / Ns) % 2 == 0) {
        fft_pass<2>(y, N, Ns, tw, tw_n);
        Ns *= 2;
    }
    while ((N / Ns) % 3 == 0) {
        fft_pass<3>(y, N, Ns, tw, tw_n);
        Ns *= 3;
    }
    while ((N / Ns) % 5 == 0) {
        fft_pass<5>(y, N, Ns, tw, tw_n);
        Ns *= 5;
    }
}

// z transform of interior rows, two per block.  Dirichlet ends: sine
// transform of the interior nodes through the FFT of the odd extension;
// open ends: cosine sums over all nodes 0..nz through the FFT of the even
// extension, S_k = (Y_k + x_0 + (-1)^k x_nz) / 2.
//   mode 0: rows of Q * bscale            -> rhs (modes; divided by c_k when open)
//   mode 1: rows of rhs (already scaled)  -> rhs (modes; divided by c_k when open)
//   mode 2: rows of rhs (solved modes)    -> phi = phi_vac + (2/nz) DST, or + S
__global__ void __launch_bounds__(kFftMaxBlock) kf_dst(const DevInst* __restrict__ It,
                                                    const FieldDev* __restrict__ Ft, int inst_base,
                                                    const double2* __restrict__ tw, int tw_n,
                                                    int mode, const double* __restrict__ bscale) {
    extern __shared__ double2 y[];
    __shared__ double2 ends[2];  // (A, B) at j = 0 and j = nz, open ends
    const int inst = inst_base + blockIdx.y;
    const DevInst& I = It[inst];
    const FieldDev& F = Ft[inst];
    const int nz = I.nz, W = I.W;
    const int iA = 1 + 2 * blockIdx.x, iB = iA + 1;
    if (I.frozen || iA > I.nr - 1) return;
    const bool hasB = iB <= I.nr - 1;
    const bool open = I.open_ends != 0;
    const int N = 2 * nz;
    // an instance with the elliptic insert has its load in rhs already
    const bool from_q = mode == 0 && !I.has_ins;
    const double bs = from_q ? bscale[inst] : 1.0;
    // Each node of the two rows is read once, a thread's loads all issued
    // before the first is used, and stored to its slot jj and (interior
    // nodes) to the mirror slot N - jj of the odd (even) extension.
    const unsigned long long* src =
        from_q ? reinterpret_cast<const unsigned long long*>(F.Q) : reinterpret_cast<const unsigned long long*>(F.rhs);
    for (int j0 = 0; j0 <= nz; j0 += kRowPer * blockDim.x) {
        unsigned long long ba[kRowPer], bb[kRowPer];
#pragma unroll
        for (int q = 0; q < kRowPer; ++q) {
            const int jj = j0 + threadIdx.x + q * blockDim.x;
            const bool ld = jj <= nz && (open || (jj >= 1 && jj <= nz - 1));
            ba[q] = ld ? src[(long long)iA * W + jj] : 0ull;
            bb[q] = ld && hasB ? src[(long long)iB * W + jj] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < kRowPer; ++q) {
            const int jj = j0 + threadIdx.x + q * blockDim.x;
            if (jj > nz) continue;
            const bool ld = open || (jj >= 1 && jj <= nz - 1);
            double va = 0.0, vb = 0.0;
            if (ld) {
                va = from_q ? (double)(long long)ba[q] * bs : __longlong_as_double((long long)ba[q]);
                if (hasB) vb = from_q ? (double)(long long)bb[q] * bs : __longlong_as_double((long long)bb[q]);
            }
            y[lp(jj)] = make_double2(va, vb);
            if (jj >= 1 && jj <= nz - 1) {
                const double sg = open ? 1.0 : -1.0;
                y[lp(N - jj)] = make_double2(sg * va, sg * vb);
            }
            if (open && jj == 0) ends[0] = make_double2(va, vb);
            if (open && jj == nz) ends[1] = make_double2(va, vb);
        }
    }
    __syncthreads();
    fft_lds(y, N, tw, tw_n);
    if (open) {
        const double2 e0 = ends[0], e1 = ends[1];
        for (int k0 = 0; k0 <= nz; k0 += kRowPer * blockDim.x) {
            double pa[kRowPer], pb[kRowPer];
#pragma unroll
            for (int q = 0; q < kRowPer; ++q) {
                const int k = k0 + threadIdx.x + q * blockDim.x;
                const bool ld = mode == 2 && k <= nz;
                pa[q] = ld ? F.phi_vac[(long long)iA * W + k] : 0.0;
                pb[q] = ld && hasB ? F.phi_vac[(long long)iB * W + k] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < kRowPer; ++q) {
                const int k = k0 + threadIdx.x + q * blockDim.x;
                if (k > nz) continue;
                const double sgn = (k & 1) ? -1.0 : 1.0;
                const double2 yk = y[lp(k)];
                double SA = 0.5 * (yk.x + (e0.x + sgn * e1.x));
                double SB = 0.5 * (yk.y + (e0.y + sgn * e1.y));
                const long long nA = (long long)iA * W + k, nB = (long long)iB * W + k;
                if (mode == 2) {
                    F.phi[nA] = pa[q] + SA;
                    if (hasB) F.phi[nB] = pb[q] + SB;
                } else {
                    const double ck = (k == 0 || k == nz) ? (double)nz : 0.5 * (double)nz;
                    F.rhs[nA] = SA / ck;
                    if (hasB) F.rhs[nB] = SB / ck;
                }
            }
        }
        return;
    }
    // y = -2i X_A + 2 X_B for odd real inputs A (real part) and B (imag part)
    const double sc = 2.0 / (double)nz;
    for (int k0 = 1; k0 <= nz - 1; k0 += kRowPer * blockDim.x) {
        double pa[kRowPer], pb[kRowPer];
#pragma unroll
        for (int q = 0; q < kRowPer; ++q) {
            const int k = k0 + threadIdx.x + q * blockDim.x;
            const bool ld = mode == 2 && k <= nz - 1;
            pa[q] = ld ? F.phi_vac[(long long)iA * W + k] : 0.0;
            pb[q] = ld && hasB ? F.phi_vac[(long long)iB * W + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kRowPer; ++q) {
            const int k = k0 + threadIdx.x + q * blockDim.x;
            if (k > nz - 1) continue;
            const double2 yk = y[lp(k)];
            double XA = -0.5 * yk.y, XB = 0.5 * yk.x;
            long long nA = (long long)iA * W + k, nB = (long long)iB * W + k;
            if (mode == 2) {
                F.phi[nA] = pa[q] + sc * XA;
                if (hasB) F.phi[nB] = pb[q] + sc * XB;
            } else {
                F.rhs[nA] = XA;
                if (hasB) F.rhs[nB] = XB;
            }
        }
    }
}

// Tridiagonal solve in r for every sine mode k with the LU factors of the
// matrix precomputed on the host: forward d_i = (b_i - lo_i d_{i-1}) im_i,
// backward x_i = d_i - cp_i x_{i+1}.  The interior rows are cut into
// kThomasSeg segments handled by different waves: each sweeps its segment
// with a zero incoming value, the segment-end values are propagated through
// LDS, and each row is corrected by its precomputed homogeneous factor
// (G_i = prod(-lo im) from the segment start, H_i = prod(-cp) to its end).
// A block covers 64 modes; lane = mode, threadIdx.y = segment.
constexpr int kTB = 8;

__global__ void __launch_bounds__(64 * kThomasSeg) kf_thomas(const DevInst* __restrict__ It,
                                                             const FieldDev* __restrict__ Ft, int inst_base) {
    __shared__ double s_val[kThomasSeg][64], s_fac[kThomasSeg][64];
    const int inst = inst_base + blockIdx.y;
    const DevInst& I = It[inst];
    const FieldDev& F = Ft[inst];
    if (I.frozen) return;
    const int lane = threadIdx.x, sg = __builtin_amdgcn_readfirstlane(threadIdx.y);  // one wave per segment
    // modes 1..nz-1 (sine, Dirichlet ends) or 0..nz (cosine, open ends)
    const int kfirst = I.open_ends ? 0 : 1, klast = I.open_ends ? I.nz : I.nz - 1;
    const int k = kfirst + blockIdx.x * 64 + lane;
    if (kfirst + (int)blockIdx.x * 64 > klast) return;  // whole block past the modes
    const bool valid = k <= klast;
    const int kk = valid ? k : kfirst;
    const long long W = I.W;
    const int nri = I.nr - 1;
    const int m = (nri + kThomasSeg - 1) / kThomasSeg;
    const int r0 = 1 + sg * m, r1 = min(r0 + m, nri + 1);
    double* __restrict__ rhs = F.rhs;
    const double* __restrict__ lo = F.th_lo;
    const double* __restrict__ im = F.th_im;
    const double* __restrict__ cp = F.th_cp;
    const double* __restrict__ G = F.th_G;
    const double* __restrict__ H = F.th_H;
    // forward sweep of the segment from zero
    double d = 0.0;
    int i = r0;
    for (; i + kTB <= r1; i += kTB) {
        double bb[kTB], ll[kTB], mm[kTB];
#pragma unroll
        for (int u = 0; u < kTB; ++u) {
            const long long n = (long long)(i + u) * W + kk;
            bb[u] = rhs[n]; ll[u] = lo[n]; mm[u] = im[n];
        }
#pragma unroll
        for (int u = 0; u < kTB; ++u) {
            d = (bb[u] - ll[u] * d) * mm[u];
            if (valid) rhs[(long long)(i + u) * W + kk] = d;
        }
    }
    for (; i < r1; ++i) {
        const long long n = (long long)i * W + kk;
        d = (rhs[n] - lo[n] * d) * im[n];
        if (valid) rhs[n] = d;
    }
    s_val[sg][lane] = r1 > r0 ? d : 0.0;
    s_fac[sg][lane] = r1 > r0 ? G[(long long)(r1 - 1) * W + kk] : 1.0;
    __syncthreads();
    double din = 0.0;
    for (int s2 = 0; s2 < sg; ++s2) din = s_val[s2][lane] + s_fac[s2][lane] * din;
    __syncthreads();
    // correct the forward values and sweep the segment backward from zero
    double x = 0.0;
    i = r1 - 1;
    for (; i - kTB + 1 >= r0; i -= kTB) {
        double dd[kTB], gg[kTB], cc[kTB];
#pragma unroll
        for (int u = 0; u < kTB; ++u) {
            const long long n = (long long)(i - u) * W + kk;
            dd[u] = rhs[n]; gg[u] = G[n]; cc[u] = cp[n];
        }
#pragma unroll
        for (int u = 0; u < kTB; ++u) {
            x = (dd[u] + gg[u] * din) - cc[u] * x;
            if (valid) rhs[(long long)(i - u) * W + kk] = x;
        }
    }
    for (; i >= r0; --i) {
        const long long n = (long long)i * W + kk;
        x = (rhs[n] + G[n] * din) - cp[n] * x;
        if (valid) rhs[n] = x;
    }
    s_val[sg][lane] = r1 > r0 ? x : 0.0;
    s_fac[sg][lane] = r1 > r0 ? H[(long long)r0 * W + kk] : 1.0;
    __syncthreads();
    double xin = 0.0;
    for (int s2 = kThomasSeg - 1; s2 > sg; --s2) xin = s_val[s2][lane] + s_fac[s2][lane] * xin;
    if (!valid || xin == 0.0) return;
    for (i = r0; i + kTB <= r1; i += kTB) {
        double xx[kTB], hh[kTB];
#pragma unroll
        for (int u = 0; u < kTB; ++u) {
            const long long n = (long long)(i + u) * W + kk;
            xx[u] = rhs[n]; hh[u] = H[n];
        }
#pragma unroll
        for (int u = 0; u < kTB; ++u) rhs[(long long)(i + u) * W + kk] = xx[u] + hh[u] * xin;
    }
    for (; i < r1; ++i) {
        const long long n = (long long)i * W + kk;
        rhs[n] = rhs[n] + H[n] * xin;
    }
}

// The same partitioned solve with segments of at most R rows whose values
// stay in registers between the sweeps: the right-hand side is read once and
// the solution written once.  With SPLIT = 2 (the form launched) each half
// wave takes a segment: 32 modes per block and 2 kThomasSegReg segments;
// SPLIT = 1 takes one segment per wave and 64 modes per block.
template <int R, int SPLIT>
__global__ void __launch_bounds__(64 * kThomasSegReg) kf_thomas_reg(const DevInst* __restrict__ It,
                                                                    const FieldDev* __restrict__ Ft,
                                                                    int inst_base) {
    constexpr int P = kThomasSegReg * SPLIT;
    constexpr int MB = 64 / SPLIT;  // modes per block
    constexpr int B = R < 8 ? R : 8;  // rows whose loads are issued together
    __shared__ double s_val[P][MB], s_fac[P][MB];
    const int inst = inst_base + blockIdx.y;
    const DevInst& I = It[inst];
    const FieldDev& F = Ft[inst];
    if (I.frozen) return;
    // SPLIT = 1: the segment index and the row offsets are wave-uniform
    const int lane = threadIdx.x % MB;
    const int sg = SPLIT == 1 ? __builtin_amdgcn_readfirstlane(threadIdx.y) : threadIdx.y * SPLIT + threadIdx.x / MB;
    // modes 1..nz-1 (sine, Dirichlet ends) or 0..nz (cosine, open ends)
    const int kfirst = I.open_ends ? 0 : 1, klast = I.open_ends ? I.nz : I.nz - 1;
    const int k = kfirst + blockIdx.x * MB + lane;
    if (kfirst + (int)blockIdx.x * MB > klast) return;  // whole block past the modes
    const bool valid = k <= klast;
    const int kk = valid ? k : kfirst;
    const int W = I.W;  // node offsets fit 32 bits ((nr+1)(nz+1) < 2^31)
    const int nri = I.nr - 1;
    const int m = (nri + P - 1) / P;  // <= R (checked by the launcher)
    const int r0 = 1 + sg * m;
    const int cnt = max(0, min(m, nri + 1 - r0));
    double* __restrict__ rhs = F.rhs;
    const double* __restrict__ lo = F.th_lo;
    const double* __restrict__ im = F.th_im;
    const double* __restrict__ cp = F.th_cp;
    const double* __restrict__ G = F.th_G;
    const double* __restrict__ H = F.th_H;
    // rows past the segment read a valid row (clamped) and are not used
    auto node = [&](int u) { return min(r0 + u, nri) * W + kk; };
    double v[R];
    double d = 0.0;
#pragma unroll
    for (int b = 0; b < R; b += B) {
        double bb[B], ll[B], mm[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int n = node(b + u);
            bb[u] = rhs[n]; ll[u] = lo[n]; mm[u] = im[n];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const double dn = (bb[u] - ll[u] * d) * mm[u];
            d = b + u < cnt ? dn : d;
            v[b + u] = d;
        }
    }
    s_val[sg][lane] = cnt > 0 ? d : 0.0;
    s_fac[sg][lane] = cnt > 0 ? G[node(cnt - 1)] : 1.0;
    __syncthreads();
    double din = 0.0;
    for (int s2 = 0; s2 < sg; ++s2) din = s_val[s2][lane] + s_fac[s2][lane] * din;
    __syncthreads();
    double x = 0.0;
#pragma unroll
    for (int b = R - B; b >= 0; b -= B) {
        double gg[B], cc[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int n = node(b + u);
            gg[u] = G[n]; cc[u] = cp[n];
        }
#pragma unroll
        for (int u = B - 1; u >= 0; --u) {
            const double xn = (v[b + u] + gg[u] * din) - cc[u] * x;
            x = b + u < cnt ? xn : x;
            v[b + u] = x;
        }
    }
    s_val[sg][lane] = cnt > 0 ? x : 0.0;
    s_fac[sg][lane] = cnt > 0 ? H[node(0)] : 1.0;
    __syncthreads();
    double xin = 0.0;
    for (int s2 = P - 1; s2 > sg; --s2) xin = s_val[s2][lane] + s_fac[s2][lane] * xin;
    if (!valid) return;
#pragma unroll
    for (int b = 0; b < R; b += B) {
        double hh[B];
#pragma unroll
        for (int u = 0; u < B; ++u) hh[u] = H[node(b + u)];
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (b + u < cnt) rhs[node(b + u)] = v[b + u] + hh[u] * xin;
    }
}

// Boundary rows of phi are the electrode data (the solve covers interior rows).
__global__ void kf_phi_edges(const DevInst* __restrict__ It, const FieldDev* __restrict__ Ft,
                             int inst_base) {
    const int inst = inst_base + blockIdx.y;
    const DevInst& I = It[inst];
    const FieldDev& F = Ft[inst];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int W = I.W;
    if (I.frozen) return;
    // rows i=0 and i=nr (W entries each), columns j=0 and j=nz (nr+1 entries
    // each; with open ends the columns are solved, not given)
    if (t < W) {
        F.phi[t] = F.phi_vac[t];
        long long n = (long long)I.nr * W + t;
        F.phi[n] = F.phi_vac[n];
    } else if (!I.open_ends && t < W + I.nr + 1) {
        long long i = t - W;
        F.phi[i * W] = F.phi_vac[i * W];
        F.phi[i * W + I.nz] = F.phi_vac[i * W + I.nz];
    }
}

// E = -grad phi at node n (central inside, second-order one-sided on the
// edges); writes FP64 arrays and/or the packed FP32 {Er, Ez, Br, Bz} (the
// static B half only with with_B).
__device__ __forceinline__ void efield_node(const DevInst& I, const FieldDev& F, int n, bool with_B) {
    const int W = I.W, i = n / W, j = n - i * W;
    const double hr = 0.5 / I.dr, hz = 0.5 / I.dz;
    const double* P = F.phi;
    // every stencil value is read unconditionally (unused ones at n), then
    // the edge or interior difference is selected
    const bool r0 = i == 0, r1 = i == I.nr, z0 = j == 0, z1 = j == I.nz;
    const double a0 = P[r0 ? j : (r1 ? n : n + W)];
    const double a1 = P[r0 ? W + j : n - W];
    const double a2 = P[r0 ? 2 * W + j : (r1 ? n - 2 * W : n)];
    const double b0 = P[(z0 || z1) ? n : n + 1];
    const double b1 = P[z0 ? n + 1 : n - 1];
    const double b2 = P[z0 ? n + 2 : (z1 ? n - 2 : n)];
    const double gr = r0 ? (-3.0 * a0 + 4.0 * a1 - a2) * hr : (r1 ? (3.0 * a0 - 4.0 * a1 + a2) * hr : (a0 - a1) * hr);
    const double gz = z0 ? (-3.0 * b0 + 4.0 * b1 - b2) * hz : (z1 ? (3.0 * b0 - 4.0 * b1 + b2) * hz : (b0 - b1) * hz);
    if (F.Er) {
        F.Er[n] = -gr;
        F.Ez[n] = -gz;
    }
    if (F.EB) {
        if (with_B) F.EB[n] = make_float4((float)(-gr), (float)(-gz), (float)F.Br[n], (float)F.Bz[n]);
        else *reinterpret_cast<float2*>(&F.EB[n]) = make_float2((float)(-gr), (float)(-gz));
    }
}

// Diagnostics sample (every D steps): the density at node n into the
// running spatial max mx and its charge into the time-average accumulator.
__device__ __forceinline__ void sample_node(const DevInst& I, const FieldDev& F, int n, double& mx) {
    double q = (double)F.Q[n];
    double dens = (q * I.inv_two_S) / F.V[n];
    mx = dens > mx ? dens : mx;
    F.avg_acc[n] += q;
}

// The rest of a sample in a 256-thread block (every thread calls it): the
// block's max density into the time max (one device atomic, and only when
// it exceeds the max seen so far); in the instance's first block the
// windowed wall currents and their peaks.
__device__ void sample_block(const DevInst& I, long long* cnt, double mx, bool first_block) {
    __shared__ double red[256];
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] > 0.0 && red[0] > __longlong_as_double(cnt[C_PEAK]))
        atomic_max_pos_double(&cnt[C_PEAK], red[0]);
    if (first_block && threadIdx.x == 0) {
        const int D = I.diag_D;
        cnt[C_NSAMP] += 1;
        double span = (double)D * I.dt;
        for (int w = 0; w < 4; ++w) {
            long long dW = cnt[C_ABS_W + w] - cnt[C_WLAST + w];
            double cur = (((double)dW * kE) * I.inv_two_S) / span;
            cnt[C_IWALL + w] = __double_as_longlong(cur);
            cnt[C_WLAST + w] = cnt[C_ABS_W + w];
        }
        double io = __longlong_as_double(cnt[C_IWALL + 1]);
        double ii = __longlong_as_double(cnt[C_IWALL + 0]);
        if (io > __longlong_as_double(cnt[C_PEAKI_OUT])) cnt[C_PEAKI_OUT] = __double_as_longlong(io);
        if (ii > __longlong_as_double(cnt[C_PEAKI_IN])) cnt[C_PEAKI_IN] = __double_as_longlong(ii);
    }
}

// Nodal E of every instance (blockIdx.y), one node per thread; with
// cnt_base, also the diagnostics sample of the step on the same nodes (the
// per-step form of ks_sample, saving its launch).
__global__ void __launch_bounds__(256) kf_efield(const DevInst* __restrict__ It, const FieldDev* __restrict__ Ft,
                                                 int inst_base, int with_B, long long* cnt_base) {
    const int inst = inst_base + blockIdx.y;
    const DevInst& I = It[inst];
    const FieldDev& F = Ft[inst];
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (!I.frozen && n < I.nodes) efield_node(I, F, n, with_B != 0);
    if (!cnt_base) return;
    long long* cnt = cnt_base + (long long)inst * C_NCOUNT;
    if ((cnt[C_STEP] + 1) % I.diag_D != 0) return;  // the same for the whole block
    double mx = 0.0;
    if (n < I.nodes) sample_node(I, F, n, mx);
    sample_block(I, cnt, mx, blockIdx.x == 0);
}

__global__ void kz_zero(long long* p, long long n) {
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = 0;
}

// Every D steps: spatial-max density into the running time max, the
// time-average accumulator, and windowed wall currents.
__global__ void ks_sample(const DevInst* __restrict__ It, const FieldDev* __restrict__ Ft, long long* cnt_base) {
    const int inst = blockIdx.y;
    const DevInst& I = It[inst];
    const FieldDev& F = Ft[inst];
    long long* cnt = cnt_base + (long long)inst * C_NCOUNT;
    if ((cnt[C_STEP] + 1) % I.diag_D != 0) return;
    double mx = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < I.nodes; n += gridDim.x * blockDim.x)
        sample_node(I, F, n, mx);
    sample_block(I, cnt, mx, blockIdx.x == 0);
}

// End of step, one block: fold each instance's new electrons into its slot
// count and advance its step counter, then (FP32 form, ctl != NULL) plan
// the next step.
__global__ void ks_commit(const DevInst* __restrict__ It, long long* cnt_base, long long* ctl, int n_inst) {
    for (int k = threadIdx.x; k < n_inst; k += blockDim.x) {
        long long* c = cnt_base + (long long)k * C_NCOUNT;
        const long long sl = c[C_SLOTS] + c[C_SPAWN];
        c[C_SLOTS] = sl < It[k].p_cap ? sl : It[k].p_cap;
        c[C_SPAWN] = 0;
        c[C_STEP] += 1;
    }
    __syncthreads();
    if (ctl) prep_tails_block(ctl, cnt_base, n_inst);
}

// ---- cubic B-spline space charge ------------------------------------------
// Unknown coefficients at 1 <= i <= nr-1, 1 <= j <= nz-1; the ghost nodes
// -1 and nr+1 (nz+1) hold minus the reflected coefficient, the wall nodes 0.
// Open ends reflect evenly in z instead: j = 0 .. nz are unknowns and the
// ghosts j = -1, nz+1 hold the coefficients at 1, nz-1.

// raw index in [-1, n+1] -> unknown index and sign (0: fixed at 0)
__device__ __forceinline__ int fold3(int i, int n, int& u) {
    if (i >= 1 && i <= n - 1) {
        u = i;
        return 1;
    }
    u = i < 0 ? 1 : n - 1;
    return (i == -1 || i == n + 1) ? -1 : 0;
}

// the z fold: odd (electrode ends) or even (open ends)
__device__ __forceinline__ int fold3z(int j, int n, bool open, int& u) {
    if (!open) return fold3(j, n, u);
    u = j < 0 ? -j : (j > n ? 2 * n - j : j);
    return 1;
}

// load of the unknowns: the ghosted deposit folded with the reflection signs
__global__ void k3_fold(const DevInst* __restrict__ It, const FieldDev* __restrict__ F3,
                        const double* __restrict__ bscale) {
    const DevInst& I = It[blockIdx.y];
    const FieldDev& F = F3[blockIdx.y];
    if (I.frozen) return;
    const int W = I.W, WX = I.nz + 3;
    const double bs = bscale[blockIdx.y];
    const bool open = I.open_ends != 0;
    const double sz = open ? 1.0 : -1.0;  // sign of the z ghosts
    const int jlo = open ? 0 : 1, jhi = open ? I.nz : I.nz - 1;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < I.nodes; n += gridDim.x * blockDim.x) {
        const int i = n / W, j = n - i * W;
        if (i < 1 || i > I.nr - 1 || j < jlo || j > jhi) continue;
        const int ri[2] = {i, i == 1 ? -1 : (i == I.nr - 1 ? I.nr + 1 : -100)};
        const int rj[2] = {j, j == 1 ? -1 : (j == I.nz - 1 ? I.nz + 1 : -100)};
        double v = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                if (ri[a] == -100 || rj[b] == -100) continue;
                const double sg = (a == 0 ? 1.0 : -1.0) * (b == 0 ? 1.0 : sz);
                v += sg * (double)F.Qx[(long long)(ri[a] + 1) * WX + (rj[b] + 1)];
            }
        F.rhs[n] = v * bs;
    }
}

// per sine mode k (one lane each): the 7-band r system, L D L^T factors
// precomputed on the host; in place in rhs.  The sweeps are sequential in r,
// so the rows' operands are loaded kB3 rows at a time (their loads in flight
// together) before the recurrence consumes them.
constexpr int kB3 = 16;

__global__ void __launch_bounds__(64) k3_band(const DevInst* __restrict__ It, const FieldDev* __restrict__ F3) {
    const DevInst& I = It[blockIdx.y];
    const FieldDev& F = F3[blockIdx.y];
    const int k = blockIdx.x * 64 + threadIdx.x;
    const bool open = I.open_ends != 0;
    if (I.frozen || k < (open ? 0 : 1) || k > (open ? I.nz : I.nz - 1)) return;
    const int W = I.W, m = I.nr - 1;
    double* __restrict__ x = F.rhs;
    const double* __restrict__ L1 = F.s3_L1;
    const double* __restrict__ L2 = F.s3_L2;
    const double* __restrict__ L3 = F.s3_L3;
    const double* __restrict__ Dinv = F.s3_Dinv;
    // forward: y_i = x_i - L1_i y_{i-1} - L2_i y_{i-2} - L3_i y_{i-3}
    double y1 = 0.0, y2 = 0.0, y3 = 0.0;  // y at rows i-1, i-2, i-3
    for (int ib = 1; ib <= m; ib += kB3) {
        double xb[kB3], l1[kB3], l2[kB3], l3[kB3];
#pragma unroll
        for (int u = 0; u < kB3; ++u) {
            const long long n = (long long)min(ib + u, m) * W + k;
            xb[u] = x[n]; l1[u] = L1[n]; l2[u] = L2[n]; l3[u] = L3[n];
        }
#pragma unroll
        for (int u = 0; u < kB3; ++u) {
            if (ib + u > m) break;
            const double y = ((xb[u] - l1[u] * y1) - l2[u] * y2) - l3[u] * y3;
            x[(long long)(ib + u) * W + k] = y;
            y3 = y2;
            y2 = y1;
            y1 = y;
        }
    }
    // backward: v_i = y_i Dinv_i - L1_{i+1} v_{i+1} - L2_{i+2} v_{i+2} - L3_{i+3} v_{i+3}
    double x1 = 0.0, x2 = 0.0, x3 = 0.0;  // x at rows i+1, i+2, i+3
    for (int ib = m; ib >= 1; ib -= kB3) {
        double yb[kB3], di[kB3], l1[kB3], l2[kB3], l3[kB3];
#pragma unroll
        for (int u = 0; u < kB3; ++u) {
            const int i = max(ib - u, 1);
            const long long n = (long long)i * W + k;
            yb[u] = x[n];
            di[u] = Dinv[n];
            l1[u] = i + 1 <= m ? L1[n + W] : 0.0;
            l2[u] = i + 2 <= m ? L2[n + 2 * W] : 0.0;
            l3[u] = i + 3 <= m ? L3[n + 3 * W] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kB3; ++u) {
            if (ib - u < 1) break;
            const double v = ((yb[u] * di[u] - l1[u] * x1) - l2[u] * x2) - l3[u] * x3;
            x[(long long)(ib - u) * W + k] = v;
            x3 = x2;
            x2 = x1;
            x1 = v;
        }
    }
}

// ghosted coefficients from the solved ones (the table's phi), and the
// potential phi = phi_vac + sum of the 3x3 neighbouring coefficients with
// B(0) = 4/6, B(+-1) = 1/6
__global__ void k3_post(const DevInst* __restrict__ It, const FieldDev* __restrict__ Ft,
                        const FieldDev* __restrict__ F3) {
    const DevInst& I = It[blockIdx.y];
    const FieldDev& F = Ft[blockIdx.y];
    if (I.frozen) return;
    const double* c = F3[blockIdx.y].phi;
    const int W = I.W, WX = I.nz + 3;
    const long long ext = (long long)(I.nr + 3) * WX;
    const bool open = I.open_ends != 0;
    auto coef = [&](int ri, int rj) {
        int ui, uj;
        const int si = fold3(ri, I.nr, ui), sj = fold3z(rj, I.nz, open, uj);
        return (si && sj) ? (double)(si * sj) * c[(long long)ui * W + uj] : 0.0;
    };
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ext;
         t += (long long)gridDim.x * blockDim.x) {
        const int gi = (int)(t / WX), gj = (int)(t - (long long)gi * WX);
        const double ct = coef(gi - 1, gj - 1);
        F.cx[t] = ct;
        if (F.cxf) F.cxf[t] = (float)ct;
        if (gi > I.nr || gj > I.nz) continue;
        // node (gi, gj)
        const double nb[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
        double v = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) v += (nb[a] * nb[b]) * coef(gi - 1 + a, gj - 1 + b);
        const long long n = (long long)gi * W + gj;
        F.phi[n] = F.phi_vac[n] + v;
    }
}

}  // namespace

hipError_t launch_s3_fold(const DevInst* It, const FieldDev* F3, int n_inst, long long max_nodes,
                          const double* bscale, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k3_fold, dim3((unsigned)((max_nodes + 255) / 256), n_inst), dim3(256), 0, s, It, F3, bscale);
    return hipGetLastError();
}

hipError_t launch_s3_rect(const DevInst* It, const FieldDev* F3, int n_inst, int max_nr, int max_nz,
                          const double2* tw, int tw_n, const double* bscale, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    size_t lds = fft_lds_bytes(max_nz);
    dim3 gdst((unsigned)(max_nr / 2), (unsigned)n_inst);
    const dim3 fb((unsigned)fft_block(max_nz));
    hipLaunchKernelGGL(kf_dst, gdst, fb, lds, s, It, F3, 0, tw, tw_n, 1, bscale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // modes 0 .. nz (open ends) or 1 .. nz-1: nz + 1 lanes
    hipLaunchKernelGGL(k3_band, dim3((unsigned)((max_nz + 1 + 63) / 64), n_inst), dim3(64), 0, s, It, F3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(kf_dst, gdst, fb, lds, s, It, F3, 0, tw, tw_n, 2, bscale);
    return hipGetLastError();
}

hipError_t launch_s3_post(const DevInst* It, const FieldDev* Ft, const FieldDev* F3, int n_inst, long long max_ext,
                          hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k3_post, dim3((unsigned)((max_ext + 255) / 256), n_inst), dim3(256), 0, s, It, Ft, F3);
    return hipGetLastError();
}

hipError_t launch_solve3_tab(const DevInst* It, const FieldDev* Ft, const FieldDev* F3, int n_inst, int max_nr,
                             int max_nz, long long max_ext, const double2* tw, int tw_n, const double* bscale,
                             hipStream_t s) {
    const long long max_nodes = (long long)(max_nr + 1) * (max_nz + 1);
    hipError_t e = launch_s3_fold(It, F3, n_inst, max_nodes, bscale, s);
    if (e == hipSuccess) e = launch_s3_rect(It, F3, n_inst, max_nr, max_nz, tw, tw_n, bscale, s);
    if (e == hipSuccess) e = launch_s3_post(It, Ft, F3, n_inst, max_ext, s);
    return e;
}

hipError_t launch_zero_i64(long long* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(kz_zero, dim3((unsigned)g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_solve_tab(const DevInst* It, const FieldDev* Ft, int inst_base, int n_inst,
                            int max_nr, int max_nz, const double2* tw, int tw_n, int mode,
                            const double* bscale, bool edges, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    size_t lds = fft_lds_bytes(max_nz);
    dim3 gdst((unsigned)(max_nr / 2), (unsigned)n_inst);
    const dim3 fb((unsigned)fft_block(max_nz));
    hipLaunchKernelGGL(kf_dst, gdst, fb, lds, s, It, Ft, inst_base, tw, tw_n, mode, bscale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 gth((unsigned)((max_nz + 1 + 63) / 64), (unsigned)n_inst);  // up to nz + 1 modes
    const int nseg = thomas_segments(max_nr);
    if (nseg == 2 * kThomasSegReg) {
        const int rows = (max_nr - 1 + nseg - 1) / nseg;
        const dim3 blk(64, kThomasSegReg);
        const dim3 g2((unsigned)((max_nz + 1 + 31) / 32), (unsigned)n_inst);
        if (rows <= 4)  // meshes up to 129 cells in r: half the loads of R = 8
            hipLaunchKernelGGL((kf_thomas_reg<4, 2>), g2, blk, 0, s, It, Ft, inst_base);
        else if (rows <= 8)
            hipLaunchKernelGGL((kf_thomas_reg<8, 2>), g2, blk, 0, s, It, Ft, inst_base);
        else
            hipLaunchKernelGGL((kf_thomas_reg<16, 2>), g2, blk, 0, s, It, Ft, inst_base);
    } else {
        hipLaunchKernelGGL(kf_thomas, gth, dim3(64, kThomasSeg), 0, s, It, Ft, inst_base);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(kf_dst, gdst, fb, lds, s, It, Ft, inst_base, tw, tw_n, 2, bscale);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!edges) return hipSuccess;  // the electrode rows of phi keep their values
    dim3 ged((unsigned)((max_nz + 1 + max_nr + 1 + 255) / 256), (unsigned)n_inst);
    hipLaunchKernelGGL(kf_phi_edges, ged, dim3(256), 0, s, It, Ft, inst_base);
    return hipGetLastError();
}

hipError_t launch_efield_tab(const DevInst* It, const FieldDev* Ft, int inst_base, int n_inst,
                             long long max_nodes, bool with_B, hipStream_t s, long long* cnt) {
    if (n_inst <= 0) return hipSuccess;
    dim3 g((unsigned)((max_nodes + 255) / 256), (unsigned)n_inst);
    hipLaunchKernelGGL(kf_efield, g, dim3(256), 0, s, It, Ft, inst_base, with_B ? 1 : 0, cnt);
    return hipGetLastError();
}

hipError_t launch_commit(const DevInst* It, long long* cnt, long long* ctl, int n_inst, hipStream_t s) {
    hipLaunchKernelGGL(ks_commit, dim3(1), dim3(256), 0, s, It, cnt, ctl, n_inst);
    return hipGetLastError();
}

hipError_t launch_sample_tab(const DevInst* It, const FieldDev* Ft, int n_inst, long long* cnt, long long* ctl,
                             hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(ks_sample, dim3(64, (unsigned)n_inst), dim3(256), 0, s, It, Ft, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ks_commit, dim3(1), dim3(256), 0, s, It, cnt, ctl, n_inst);
    return hipGetLastError();
}

hipError_t set_field_kernel_attrs(int max_nz) {
    size_t lds = fft_lds_bytes(max_nz);
    if (lds > 65536)
        return hipFuncSetAttribute((const void*)kf_dst, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    return hipSuccess;
}

}  // namespace pic
