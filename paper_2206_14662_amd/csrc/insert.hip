// insert.hip -- the elliptic insert on the outer electrode (the gun geometry
// of Sec. III): web-spline set-up on the host and the kernels of the
// corrected Poisson solve.
//
// Space of the space-charge potential (Sec. II.A: weighted extended
// B-splines, degree 1): B_i = w (b_i + sum_{k outer} e_ik b_k) over the inner
// hats i, with b the bilinear hats of the grid and w the weight function of
// DevInst (0 in the metal, 1 - (1 - g/gam)^3 in the band, 1 beyond).  A hat is
// inner when a cell of its support lies outside the metal, outer when its
// support meets the domain without such a cell, exterior otherwise; an outer
// hat joins the nearest 2x2 block of inner hats with bilinear Lagrange
// weights in index space.  The Galerkin matrix A = int r grad B . grad B uses
// the exact Q1 element matrix on cells with w = 1 and a 3x3 Gauss rule on 2x2
// boxes elsewhere, boxes cut by the insert being split into four down to
// kQDepth levels (points in the metal dropped at the finest one).  Outer and
// exterior nodes keep the rectangle's rows among themselves, decoupled from
// the inner ones.
//
// A differs from the rectangle's matrix A_rect only in the rows and columns
// of M, the unknown corners of the cells that meet the band (cells inside
// the metal count only with an inner corner) and the block nodes of the
// outer hats: A = A_rect + E D E^T.  So A x = b is solved with the
// fast rectangle solver twice (Woodbury):
//     y = A_rect^-1 b,  s = H y_M,  x = y - A_rect^-1 E s,
// with H = (I + D G)^-1 D, G = (A_rect^-1)_MM set up once from m unit solves.
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "pic_internal.h"

namespace pic {

// ---------------------------------------------------------------------------
// host set-up
// ---------------------------------------------------------------------------
namespace {

constexpr int kQDepth = 6;
constexpr int kExtRadius = 4;
const double kGX[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
const double kGW[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};

struct Geo {
    const pic_instance_cfg* c;
    DevInst I;  // only the insert fields are used
    int nr, nz, W, j0, j1;
    double dr, dz, gam;
};

// exact range of g over a box (sum of convex parabolas: minimum at the
// clamped centre, maximum at the farthest corner)
void box_range(const Geo& G, double rl, double rh, double zl, double zh, double& gmin, double& gmax) {
    const double r0 = G.I.ins_r0, z0 = G.I.ins_z0;
    const double rc = std::min(std::max(r0, rl), rh), zc = std::min(std::max(z0, zl), zh);
    const double rf = std::fabs(rl - r0) > std::fabs(rh - r0) ? rl : rh;
    const double zf = std::fabs(zl - z0) > std::fabs(zh - z0) ? zl : zh;
    gmin = ins_g(G.I, rc, zc);
    gmax = ins_g(G.I, rf, zf);
}

void cell_range(const Geo& G, int ci, int cj, double& gmin, double& gmax) {
    const double rl = G.c->a + (double)ci * G.dr, zl = (double)cj * G.dz;
    box_range(G, rl, rl + G.dr, zl, zl + G.dz, gmin, gmax);
}

// weight function gradient (the value is ins_w)
void w_grad(const Geo& G, double r, double z, double g, double& wr, double& wz) {
    wr = wz = 0.0;
    if (g <= 0.0 || g >= G.gam) return;
    const double s = 1.0 - g / G.gam;
    const double dw = 3.0 * s * s / G.gam;
    wr = dw * (2.0 * (r - G.I.ins_r0) / (G.I.ins_er * G.I.ins_er));
    wz = dw * (2.0 * (z - G.I.ins_z0) / (G.I.ins_ez * G.I.ins_ez));
}

// r-major corners of a cell: (0,0), (1,0), (0,1), (1,1)
const int kCR[4] = {0, 1, 0, 1}, kCZ[4] = {0, 0, 1, 1};

void q1_element(const Geo& G, int ci, double E[4][4]) {
    const double rl = G.c->a + (double)ci * G.dr, rh = rl + G.dr, rm = 0.5 * (rl + rh);
    const double kr2[2][2] = {{rm / G.dr, -rm / G.dr}, {-rm / G.dr, rm / G.dr}};
    const double mr2[2][2] = {{G.dr * (3.0 * rl + rh) / 12.0, G.dr * (rl + rh) / 12.0},
                              {G.dr * (rl + rh) / 12.0, G.dr * (rl + 3.0 * rh) / 12.0}};
    const double kz2[2][2] = {{1.0 / G.dz, -1.0 / G.dz}, {-1.0 / G.dz, 1.0 / G.dz}};
    const double mz2[2][2] = {{2.0 * G.dz / 6.0, G.dz / 6.0}, {G.dz / 6.0, 2.0 * G.dz / 6.0}};
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q)
            E[p][q] = kr2[kCR[p]][kCR[q]] * mz2[kCZ[p]][kCZ[q]] + mr2[kCR[p]][kCR[q]] * kz2[kCZ[p]][kCZ[q]];
}

struct WeightedAcc {
    double rl, zl;
    double E[4][4];
};

void add_point(const Geo& G, WeightedAcc& A, double r, double z, double g, double wq) {
    const double w = ins_w(G.I, g);
    double wr, wz;
    w_grad(G, r, z, g, wr, wz);
    const double fr = (r - A.rl) / G.dr, fz = (z - A.zl) / G.dz;
    const double N[4] = {(1.0 - fr) * (1.0 - fz), fr * (1.0 - fz), (1.0 - fr) * fz, fr * fz};
    const double Nr[4] = {-(1.0 - fz) / G.dr, (1.0 - fz) / G.dr, -fz / G.dr, fz / G.dr};
    const double Nz[4] = {-(1.0 - fr) / G.dz, -fr / G.dz, (1.0 - fr) / G.dz, fr / G.dz};
    double gr[4], gz[4];
    for (int p = 0; p < 4; ++p) {
        gr[p] = wr * N[p] + w * Nr[p];
        gz[p] = wz * N[p] + w * Nz[p];
    }
    const double f = r * wq;
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) A.E[p][q] += f * (gr[p] * gr[q] + gz[p] * gz[q]);
}

void weighted_box(const Geo& G, WeightedAcc& A, double rl, double rh, double zl, double zh, int depth) {
    double gmin, gmax;
    box_range(G, rl, rh, zl, zh, gmin, gmax);
    if (gmax <= 0.0) return;
    if (gmin <= 0.0 && depth < kQDepth) {
        const double rm = 0.5 * (rl + rh), zm = 0.5 * (zl + zh);
        weighted_box(G, A, rl, rm, zl, zm, depth + 1);
        weighted_box(G, A, rm, rh, zl, zm, depth + 1);
        weighted_box(G, A, rl, rm, zm, zh, depth + 1);
        weighted_box(G, A, rm, rh, zm, zh, depth + 1);
        return;
    }
    const double hr = rh - rl, hz = zh - zl;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double r = rl + 0.5 * hr * (1.0 + kGX[a]);
            const double z = zl + 0.5 * hz * (1.0 + kGX[b]);
            const double g = ins_g(G.I, r, z);
            if (g <= 0.0) continue;
            add_point(G, A, r, z, g, (0.25 * hr * hz) * kGW[a] * kGW[b]);
        }
}

void weighted_element(const Geo& G, int ci, int cj, double E[4][4]) {
    WeightedAcc A;
    A.rl = G.c->a + (double)ci * G.dr;
    A.zl = (double)cj * G.dz;
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) A.E[p][q] = 0.0;
    const double hr = 0.5 * G.dr, hz = 0.5 * G.dz;
    for (int sr = 0; sr < 2; ++sr)
        for (int sz = 0; sz < 2; ++sz)
            weighted_box(G, A, A.rl + hr * sr, A.rl + hr * (sr + 1), A.zl + hz * sz, A.zl + hz * (sz + 1), 0);
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) E[p][q] = A.E[p][q];
}

}  // namespace

std::string ins_build(const pic_instance_cfg& c, InsHost& h) {
    Geo G;
    G.c = &c;
    G.nr = c.nr;
    G.nz = c.nz;
    G.W = c.nz + 1;
    G.j0 = c.end_mode == 2 ? 0 : 1;
    G.j1 = c.end_mode == 2 ? c.nz : c.nz - 1;
    G.dr = (c.b - c.a) / (double)c.nr;
    G.dz = c.L / (double)c.nz;
    const double band = c.ins_band > 0.0 ? c.ins_band : 3.0;
    G.gam = 2.0 * band * std::max(G.dr / c.ins_er, G.dz / c.ins_ez);
    G.I = DevInst();
    G.I.ins_r0 = c.ins_r0;
    G.I.ins_z0 = c.ins_z0;
    G.I.ins_er = c.ins_er;
    G.I.ins_ez = c.ins_ez;
    G.I.ins_gam = G.gam;
    const int W = G.W, NN = (c.nr + 1) * W;
    auto unknown = [&](int i, int j) { return i >= 1 && i <= c.nr - 1 && j >= G.j0 && j <= G.j1; };

    // node classes
    std::vector<int> cls(NN, 0);
    for (int i = 1; i <= c.nr - 1; ++i)
        for (int j = G.j0; j <= G.j1; ++j) {
            bool any_in = false, any_cut = false;
            for (int ci = i - 1; ci <= i; ++ci)
                for (int cj = j - 1; cj <= j; ++cj) {
                    if (ci < 0 || ci >= c.nr || cj < 0 || cj >= c.nz) continue;
                    double gmin, gmax;
                    cell_range(G, ci, cj, gmin, gmax);
                    if (gmin > 0.0) any_in = true;
                    else if (gmax > 0.0) any_cut = true;
                }
            cls[i * W + j] = any_in ? 1 : (any_cut ? 2 : 3);
        }
    for (int n = 0; n < NN; ++n) h.counts[cls[n]] += 1;

    // extension blocks of the outer hats
    std::vector<int> blk(NN, -1);
    std::vector<double> e4((size_t)NN * 4, 0.0);
    for (int k1 = 1; k1 <= c.nr - 1; ++k1)
        for (int k2 = G.j0; k2 <= G.j1; ++k2) {
            const int n = k1 * W + k2;
            if (cls[n] != 2) continue;
            double best = -1.0;
            int b1 = 0, b2 = 0;
            for (int l1 = k1 - kExtRadius; l1 <= k1 + kExtRadius - 1; ++l1)
                for (int l2 = k2 - kExtRadius; l2 <= k2 + kExtRadius - 1; ++l2) {
                    if (!unknown(l1, l2) || !unknown(l1 + 1, l2 + 1)) continue;
                    if (cls[l1 * W + l2] != 1 || cls[(l1 + 1) * W + l2] != 1 || cls[l1 * W + l2 + 1] != 1 ||
                        cls[(l1 + 1) * W + l2 + 1] != 1)
                        continue;
                    const double du = ((double)l1 + 0.5 - (double)k1) * G.dr;
                    const double dv = ((double)l2 + 0.5 - (double)k2) * G.dz;
                    const double d2 = du * du + dv * dv;
                    if (best < 0.0 || d2 < best) {
                        best = d2;
                        b1 = l1;
                        b2 = l2;
                    }
                }
            if (best < 0.0) return "no 2x2 block of inner nodes near an outer node: refine the mesh";
            const double x = (double)(k1 - b1), y = (double)(k2 - b2);
            blk[n] = b1 * W + b2;
            e4[(size_t)n * 4 + 0] = (1.0 - x) * (1.0 - y);
            e4[(size_t)n * 4 + 1] = x * (1.0 - y);
            e4[(size_t)n * 4 + 2] = (1.0 - x) * y;
            e4[(size_t)n * 4 + 3] = x * y;
        }
    // the nodes a hat feeds, with factors (nodes, not M indices)
    auto feeds = [&](int n, int* u, double* f) -> int {
        if (n < 0 || n >= NN || cls[n] == 0) return 0;
        if (cls[n] == 1) {
            u[0] = n;
            f[0] = 1.0;
            return 1;
        }
        if (cls[n] != 2) return 0;
        const int b = blk[n];
        const int nd[4] = {b, b + W, b + 1, b + W + 1};
        for (int q = 0; q < 4; ++q) {
            u[q] = nd[q];
            f[q] = e4[(size_t)n * 4 + q];
        }
        return 4;
    };

    // M: unknown corners of the cells that meet the band, and the blocks
    // (a cell inside the metal adds nothing unless it has an inner corner)
    std::vector<char> inM(NN, 0);
    auto meets = [&](int ci, int cj) {
        double gmin, gmax;
        cell_range(G, ci, cj, gmin, gmax);
        if (gmin >= G.gam) return false;
        if (gmax > 0.0) return true;
        for (int p = 0; p < 4; ++p)
            if (cls[(ci + kCR[p]) * W + cj + kCZ[p]] == 1) return true;
        return false;
    };
    for (int ci = 0; ci < c.nr; ++ci)
        for (int cj = 0; cj < c.nz; ++cj) {
            if (!meets(ci, cj)) continue;
            for (int p = 0; p < 4; ++p) {
                const int i = ci + kCR[p], j = cj + kCZ[p];
                if (unknown(i, j)) inM[i * W + j] = 1;
            }
        }
    for (int n = 0; n < NN; ++n)
        if (cls[n] == 2) {
            const int b = blk[n];
            inM[b] = inM[b + W] = inM[b + 1] = inM[b + W + 1] = 1;
        }
    h.map.assign(NN, -1);
    h.Mnode.clear();
    for (int n = 0; n < NN; ++n)
        if (inM[n]) {
            h.map[n] = (int)h.Mnode.size();
            h.Mnode.push_back(n);
        }
    h.m = (int)h.Mnode.size();

    // D = A - A_rect on M x M, from the cells that meet the band
    std::map<long long, double> D;
    auto addD = [&](int nu, int nv, double v) {
        const int a = h.map[nu], b = h.map[nv];
        D[(long long)a * h.m + b] += v;
    };
    for (int ci = 0; ci < c.nr; ++ci)
        for (int cj = 0; cj < c.nz; ++cj) {
            if (!meets(ci, cj)) continue;
            double gmin, gmax;
            cell_range(G, ci, cj, gmin, gmax);
            double Ex[4][4];
            q1_element(G, ci, Ex);
            int nd[4];
            for (int p = 0; p < 4; ++p) nd[p] = (ci + kCR[p]) * W + cj + kCZ[p];
            if (gmax > 0.0) {
                double Eq[4][4];
                weighted_element(G, ci, cj, Eq);
                for (int p = 0; p < 4; ++p) {
                    int up[4];
                    double fp[4];
                    const int mp = feeds(nd[p], up, fp);
                    for (int q = 0; q < 4; ++q) {
                        int uq[4];
                        double fq[4];
                        const int mq = feeds(nd[q], uq, fq);
                        for (int s = 0; s < mp; ++s)
                            for (int t = 0; t < mq; ++t) addD(up[s], uq[t], fp[s] * fq[t] * Eq[p][q]);
                    }
                }
            }
            // the rectangle's entries, kept between outer/exterior pairs
            for (int p = 0; p < 4; ++p)
                for (int q = 0; q < 4; ++q) {
                    const int np = nd[p], nq = nd[q];
                    if (cls[np] == 0 || cls[nq] == 0) continue;
                    if (cls[np] >= 2 && cls[nq] >= 2) continue;
                    addD(np, nq, -Ex[p][q]);
                }
        }
    h.Dr.clear();
    h.Dc.clear();
    h.Dv.clear();
    for (const auto& kv : D) {
        h.Dr.push_back((int)(kv.first / h.m));
        h.Dc.push_back((int)(kv.first % h.m));
        h.Dv.push_back(kv.second);
    }

    // load of each M node: inner nodes gather their own charge and that of
    // the outer hats whose block holds them; the others take none
    std::vector<std::vector<std::pair<int, double>>> load(h.m);
    for (int n = 0; n < NN; ++n) {
        if (cls[n] != 1 && cls[n] != 2) continue;
        int u[4];
        double f[4];
        const int k = feeds(n, u, f);
        for (int q = 0; q < k; ++q) {
            const int a = h.map[u[q]];
            if (a >= 0) load[a].push_back({n, f[q]});
        }
    }
    h.rp.assign(h.m + 1, 0);
    h.rk.clear();
    h.rf.clear();
    for (int a = 0; a < h.m; ++a) {
        for (const auto& e : load[a]) {
            h.rk.push_back(e.first);
            h.rf.push_back(e.second);
        }
        h.rp[a + 1] = (int)h.rk.size();
    }

    // the basis at the nodes of M
    h.typ.assign(h.m, 0);
    h.wn.assign(h.m, 0.0);
    h.ek.assign((size_t)h.m * 4, 0);
    h.ef.assign((size_t)h.m * 4, 0.0);
    for (int a = 0; a < h.m; ++a) {
        const int n = h.Mnode[a], i = n / W, j = n % W;
        const double r = c.a + (double)i * G.dr, z = (double)j * G.dz;
        const double g = ins_g(G.I, r, z);
        h.wn[a] = ins_w(G.I, g);
        if (cls[n] == 1) {
            h.typ[a] = 1;
        } else if (cls[n] == 2 && g > 0.0) {
            h.typ[a] = 2;
            const int b = blk[n];
            const int nd[4] = {b, b + W, b + 1, b + W + 1};
            for (int q = 0; q < 4; ++q) {
                h.ek[(size_t)a * 4 + q] = nd[q];
                h.ef[(size_t)a * 4 + q] = e4[(size_t)n * 4 + q];
            }
        }
    }
    return "";
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
namespace {

// rhs of every node of an insert instance: bscale Q off M, the folded load
// on M (0 for nodes that are not inner)
__global__ void ki_rhs(const DevInst* It, const InsDev* Dt, const FieldDev* Ft, const double* bscale) {
    const InsDev& D = Dt[blockIdx.y];
    if (It[D.inst].frozen) return;
    const FieldDev& F = Ft[D.inst];
    const double bs = bscale[D.inst];
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < D.nodes;
         n += (long long)gridDim.x * blockDim.x) {
        const int a = D.map[n];
        double v;
        if (a < 0) {
            v = (double)F.Q[n] * bs;
        } else {
            double s = 0.0;
            for (int t = D.rp[a]; t < D.rp[a + 1]; ++t) {
                const int k = D.rk[t];
                s += D.rf[t] * (double)(F.Q[k] + F.Qw[k]);
            }
            v = s * bs;
        }
        F.rhs[n] = v;
    }
}

// y_M = ybuf - base at the nodes of M
__global__ void ki_gather(const DevInst* It, const InsDev* Dt, const FieldDev* Fb) {
    const InsDev& D = Dt[blockIdx.y];
    if (It[D.inst].frozen) return;
    const double* base = Fb[D.inst].phi_vac;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < D.m; a += gridDim.x * blockDim.x) {
        const int n = D.Mnode[a];
        D.yM[a] = D.ybuf[n] - base[n];
    }
}

// s = H y_M for NC instances sharing H, rows a0 .. a0 + kRows - 1: the
// workgroup's 256 threads over the columns, each column's y values loaded
// once for all the rows, then the four waves' sums added in a fixed order.
// Every (row, instance) sum has the same order for any NC.
// (The operands are read through global-address-space pointers: generic
// pointers taken from a table make every load wait for the previous one.)
typedef __attribute__((address_space(1))) const double gbl_f64;
constexpr int kGrp = 8, kRows = 4;

template <int NC>
__device__ __forceinline__ void matvec_rows(const DevInst* It, const InsDev* Dt, const int* mem, gbl_f64* H, int m,
                                            int a0, double (*s_part)[kRows][kGrp]) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    gbl_f64* y[NC];
    gbl_f64* row[kRows];
    double s[kRows][NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) y[t] = (gbl_f64*)Dt[mem[t]].yM;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        row[r] = H + (size_t)min(a0 + r, m - 1) * m;
#pragma unroll
        for (int t = 0; t < NC; ++t) s[r][t] = 0.0;
    }
    for (int b = tid; b < m; b += 256) {
        double yv[NC], h[kRows];
#pragma unroll
        for (int t = 0; t < NC; ++t) yv[t] = y[t][b];
#pragma unroll
        for (int r = 0; r < kRows; ++r) h[r] = row[r][b];
#pragma unroll
        for (int r = 0; r < kRows; ++r)
#pragma unroll
            for (int t = 0; t < NC; ++t) s[r][t] += h[r] * yv[t];
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            double v = s[r][t];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) s_part[wv][r][t] = v;
        }
    __syncthreads();
    if (tid < kRows * NC) {
        const int r = tid / NC, t = tid - r * NC;
        const double v = ((s_part[0][r][t] + s_part[1][r][t]) + s_part[2][r][t]) + s_part[3][r][t];
        const InsDev& D = Dt[mem[t]];
        if (a0 + r < m && !It[D.inst].frozen) D.sM[a0 + r] = v;
    }
    __syncthreads();
}

// s = H y_M for every instance of a group sharing H (blockIdx.y): kRows rows
// per workgroup pass; each row is read once for up to kGrp instances.
__global__ void __launch_bounds__(256) ki_matvec(const DevInst* It, const InsDev* Dt, const int* goff,
                                                 const int* gmem) {
    __shared__ double s_part[4][kRows][kGrp];
    const int g0 = goff[blockIdx.y], g1 = goff[blockIdx.y + 1];
    const InsDev& D0 = Dt[gmem[g0]];
    const int m = D0.m;
    gbl_f64* H = (gbl_f64*)D0.H;
    for (int a0 = blockIdx.x * kRows; a0 < m; a0 += gridDim.x * kRows) {
        for (int c0 = g0; c0 < g1; c0 += kGrp) {
            const int* mem = gmem + c0;
            switch (min(kGrp, g1 - c0)) {
                case 1: matvec_rows<1>(It, Dt, mem, H, m, a0, s_part); break;
                case 2: matvec_rows<2>(It, Dt, mem, H, m, a0, s_part); break;
                case 3: matvec_rows<3>(It, Dt, mem, H, m, a0, s_part); break;
                case 4: matvec_rows<4>(It, Dt, mem, H, m, a0, s_part); break;
                case 5: matvec_rows<5>(It, Dt, mem, H, m, a0, s_part); break;
                case 6: matvec_rows<6>(It, Dt, mem, H, m, a0, s_part); break;
                case 7: matvec_rows<7>(It, Dt, mem, H, m, a0, s_part); break;
                default: matvec_rows<8>(It, Dt, mem, H, m, a0, s_part); break;
            }
        }
    }
}

// load of the correction: -s on M, 0 elsewhere (every node written)
__global__ void ki_scatter(const DevInst* It, const InsDev* Dt) {
    const InsDev& D = Dt[blockIdx.y];
    if (It[D.inst].frozen) return;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < D.nodes;
         n += (long long)gridDim.x * blockDim.x) {
        const int a = D.map[n];
        D.rhs2[n] = a < 0 ? 0.0 : -D.sM[a];
    }
}

// the basis at the nodes of M, from the coefficients c = phi - base
__global__ void ki_fix_eval(const DevInst* It, const InsDev* Dt, const FieldDev* Fo) {
    const InsDev& D = Dt[blockIdx.y];
    if (It[D.inst].frozen) return;
    const FieldDev& F = Fo[D.inst];
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < D.m; a += gridDim.x * blockDim.x) {
        const int n = D.Mnode[a];
        double v = 0.0;
        if (D.typ[a] == 1) {
            v = D.wn[a] * (F.phi[n] - F.phi_vac[n]);
        } else if (D.typ[a] == 2) {
            double s = 0.0;
            for (int q = 0; q < 4; ++q) {
                const int k = D.ek[a * 4 + q];
                s += D.ef[a * 4 + q] * (F.phi[k] - F.phi_vac[k]);
            }
            v = D.wn[a] * s;
        }
        D.val[a] = v;
    }
}

__global__ void ki_fix_store(const DevInst* It, const InsDev* Dt, const FieldDev* Fo) {
    const InsDev& D = Dt[blockIdx.y];
    if (It[D.inst].frozen) return;
    const FieldDev& F = Fo[D.inst];
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < D.m; a += gridDim.x * blockDim.x) {
        const int n = D.Mnode[a];
        F.phi[n] = F.phi_vac[n] + D.val[a];
    }
}

__global__ void ki_units(double* rhs, long long stride, long long nodes, const int* Mnode, int b0) {
    const int t = blockIdx.y;
    double* R = rhs + (long long)t * stride;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < nodes;
         n += (long long)gridDim.x * blockDim.x)
        R[n] = n == (long long)Mnode[b0 + t] ? 1.0 : 0.0;
}

__global__ void ki_collect(const double* phi, long long stride, const int* Mnode, int m, int b0, double* G) {
    const int t = blockIdx.y;
    const double* P = phi + (long long)t * stride;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < m; a += gridDim.x * blockDim.x)
        G[(size_t)a * m + (b0 + t)] = P[Mnode[a]];
}

// Gauss-Jordan step k on [C | D] (m x 2m): pivot row, swap and scale, the
// column of factors, elimination of column k from the other rows.
__global__ void __launch_bounds__(1024) ki_gj_pivot(const double* M, int m, int k, int* piv, double* pval) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    const int t = threadIdx.x;
    double best = -1.0;
    int bi = k;
    for (int i = k + t; i < m; i += 1024) {
        const double v = fabs(M[(size_t)i * 2 * m + k]);
        if (v > best) {
            best = v;
            bi = i;
        }
    }
    sv[t] = best;
    si[t] = bi;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (t < off) {
            const double o = sv[t + off];
            const int oi = si[t + off];
            if (o > sv[t] || (o == sv[t] && oi < si[t])) {
                sv[t] = o;
                si[t] = oi;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        piv[0] = si[0];
        pval[k] = M[(size_t)si[0] * 2 * m + k];
    }
}

__global__ void ki_gj_swap(double* M, int m, int k, const int* piv, const double* pval) {
    const int p = piv[0];
    const double inv = 1.0 / pval[k];
    for (int j = k + blockIdx.x * blockDim.x + threadIdx.x; j < 2 * m; j += gridDim.x * blockDim.x) {
        const double a = M[(size_t)k * 2 * m + j], b = M[(size_t)p * 2 * m + j];
        M[(size_t)p * 2 * m + j] = a;
        M[(size_t)k * 2 * m + j] = b * inv;
    }
}

__global__ void ki_gj_col(const double* M, int m, int k, double* f) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        f[i] = i == k ? 0.0 : M[(size_t)i * 2 * m + k];
}

__global__ void ki_gj_elim(double* M, int m, int k, const double* f) {
    const int i = blockIdx.y;
    const double fi = f[i];
    if (fi == 0.0) return;
    for (int j = k + blockIdx.x * blockDim.x + threadIdx.x; j < 2 * m; j += gridDim.x * blockDim.x)
        M[(size_t)i * 2 * m + j] -= fi * M[(size_t)k * 2 * m + j];
}

unsigned blocks_for(long long n, long long cap = 1024) {
    return (unsigned)std::max(1ll, std::min((n + 255) / 256, cap));
}

}  // namespace

hipError_t launch_ins_rhs(const DevInst* It, const InsDev* D, int n_ins, long long max_nodes, const FieldDev* Ft,
                          const double* bscale, hipStream_t s) {
    if (n_ins <= 0) return hipSuccess;
    hipLaunchKernelGGL(ki_rhs, dim3(blocks_for(max_nodes), n_ins), dim3(256), 0, s, It, D, Ft, bscale);
    return hipGetLastError();
}

hipError_t launch_ins_correct(const DevInst* It, const InsDev* D, int n_ins, const int* goff, const int* gmem,
                              int n_grp, int max_m, long long max_nodes, const FieldDev* Fbase, hipStream_t s) {
    if (n_ins <= 0) return hipSuccess;
    hipLaunchKernelGGL(ki_gather, dim3(blocks_for(max_m), n_ins), dim3(256), 0, s, It, D, Fbase);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ki_matvec, dim3((unsigned)std::max(1, std::min((max_m + 3) / 4, 4096)), n_grp), dim3(256), 0,
                       s, It, D, goff, gmem);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(ki_scatter, dim3(blocks_for(max_nodes), n_ins), dim3(256), 0, s, It, D);
    return hipGetLastError();
}

hipError_t launch_ins_fix(const DevInst* It, const InsDev* D, int n_ins, int max_m, const FieldDev* Fout,
                          hipStream_t s) {
    if (n_ins <= 0) return hipSuccess;
    hipLaunchKernelGGL(ki_fix_eval, dim3(blocks_for(max_m), n_ins), dim3(256), 0, s, It, D, Fout);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ki_fix_store, dim3(blocks_for(max_m), n_ins), dim3(256), 0, s, It, D, Fout);
    return hipGetLastError();
}

hipError_t launch_ins_units(double* rhs, long long stride, long long nodes, const int* Mnode, int b0, int cnt,
                            hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(ki_units, dim3(blocks_for(nodes), cnt), dim3(256), 0, s, rhs, stride, nodes, Mnode, b0);
    return hipGetLastError();
}

hipError_t launch_ins_collect(const double* phi, long long stride, const int* Mnode, int m, int b0, int cnt,
                              double* G, hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(ki_collect, dim3(blocks_for(m), cnt), dim3(256), 0, s, phi, stride, Mnode, m, b0, G);
    return hipGetLastError();
}

hipError_t launch_ins_gauss_jordan(double* CD, int m, double* fcol, int* piv, double* pval, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int k = 0; k < m; ++k) {
        hipLaunchKernelGGL(ki_gj_pivot, dim3(1), dim3(1024), 0, s, CD, m, k, piv, pval);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(ki_gj_swap, dim3(blocks_for(2ll * m - k)), dim3(256), 0, s, CD, m, k, piv, pval);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(ki_gj_col, dim3(blocks_for(m)), dim3(256), 0, s, CD, m, k, fcol);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(ki_gj_elim, dim3(blocks_for(2ll * m - k, 64), m), dim3(256), 0, s, CD, m, k, fcol);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return e;
}

}  // namespace pic
