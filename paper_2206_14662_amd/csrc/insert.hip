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
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "pic_internal.h"

namespace pic {

// ---------------------------------------------------------------------------
// host set-up
// ---------------------------------------------------------------------------

void ins_fill(const pic_instance_cfg& c, double dr, double dz, DevInst& I) {
    const double band = c.ins_band > 0.0 ? c.ins_band : 3.0;
    I.ins_r0 = c.ins_r0;
    I.ins_z0 = c.ins_z0;
    I.ins_er = c.ins_er;
    I.ins_ez = c.ins_ez;
    I.ins_gam = 2.0 * band * std::max(dr / c.ins_er, dz / c.ins_ez);
}

namespace {

// Cut boxes are split into four down to this many levels; an outer hat looks
// for its block of inner hats within this many nodes in each direction.
constexpr int kCutLevels = 6;
constexpr int kBlockReach = 4;

// Three-point Gauss-Legendre rule on [-1, 1].
constexpr double kGaussX[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
constexpr double kGaussW[3] = {0.55555555555555555556, 0.88888888888888888889, 0.55555555555555555556};

// How a cell or a box sits against the insert: g > 0 everywhere (free), g
// changes sign inside (cut), g <= 0 everywhere (metal).
enum Where { kFree, kCut, kMetal };

// Node roles (pic_insert_layout's counts): 0 not an unknown of the solve,
// 1 inner hat, 2 outer hat, 3 exterior (all its cells in the metal).
enum Role { kFixed = 0, kInner = 1, kOuter = 2, kExterior = 3 };

class InsertMesh {
public:
    InsertMesh(const pic_instance_cfg& c) : c_(c) {
        dr_ = (c.b - c.a) / (double)c.nr;
        dz_ = c.L / (double)c.nz;
        ins_fill(c, dr_, dz_, I_);
        W_ = c.nz + 1;
        jlo_ = c.end_mode == 2 ? 0 : 1;
        jhi_ = c.end_mode == 2 ? c.nz : c.nz - 1;
    }
    int W() const { return W_; }
    int nodes() const { return (c_.nr + 1) * W_; }
    double dr() const { return dr_; }
    double dz() const { return dz_; }
    double gam() const { return I_.ins_gam; }
    double r_of(int i) const { return c_.a + (double)i * dr_; }
    double z_of(int j) const { return (double)j * dz_; }
    bool unknown(int i, int j) const { return i >= 1 && i <= c_.nr - 1 && j >= jlo_ && j <= jhi_; }
    double g(double r, double z) const { return ins_g(I_, r, z); }
    double w(double g) const { return ins_w(I_, g); }

    // Lowest and highest g over the box [rl, rh] x [zl, zh]: g is a sum of one
    // square in r and one in z, each monotone away from the centre.
    void g_range(double rl, double rh, double zl, double zh, double& lo, double& hi) const {
        double ulo, uhi, vlo, vhi;
        sq_range((rl - I_.ins_r0) / I_.ins_er, (rh - I_.ins_r0) / I_.ins_er, ulo, uhi);
        sq_range((zl - I_.ins_z0) / I_.ins_ez, (zh - I_.ins_z0) / I_.ins_ez, vlo, vhi);
        lo = (ulo + vlo) - 1.0;
        hi = (uhi + vhi) - 1.0;
    }
    Where where(double rl, double rh, double zl, double zh) const {
        double lo, hi;
        g_range(rl, rh, zl, zh, lo, hi);
        return lo > 0.0 ? kFree : (hi > 0.0 ? kCut : kMetal);
    }
    void cell_g(int ci, int cj, double& lo, double& hi) const {
        g_range(r_of(ci), r_of(ci + 1), z_of(cj), z_of(cj + 1), lo, hi);
    }

    // Gradient of the weight function at (r, z) where g = g(r, z).
    void w_grad(double r, double z, double g, double& gr, double& gz) const {
        if (!(g > 0.0 && g < I_.ins_gam)) {
            gr = gz = 0.0;
            return;
        }
        const double t = 1.0 - g / I_.ins_gam;
        const double dwdg = 3.0 * t * t / I_.ins_gam;
        gr = dwdg * (2.0 * (r - I_.ins_r0) / (I_.ins_er * I_.ins_er));
        gz = dwdg * (2.0 * (z - I_.ins_z0) / (I_.ins_ez * I_.ins_ez));
    }

private:
    // range of x^2 for x in [a, b]
    static void sq_range(double a, double b, double& lo, double& hi) {
        const double qa = a * a, qb = b * b;
        hi = std::max(qa, qb);
        lo = (a <= 0.0 && b >= 0.0) ? 0.0 : std::min(qa, qb);
    }
    const pic_instance_cfg& c_;
    DevInst I_;
    double dr_, dz_;
    int W_, jlo_, jhi_;
};

// Cell corners in r-major order: (i, j), (i+1, j), (i, j+1), (i+1, j+1).
inline int corner(const InsertMesh& M, int ci, int cj, int p) { return (ci + (p & 1)) * M.W() + cj + (p >> 1); }

// The Q1 stiffness of one cell in the r-weighted form (the rectangle's
// element matrix): K_r (x) M_z + M_r (x) K_z with the 1-D matrices of the
// cell [r_i, r_i+1] x [z_j, z_j+1].
void rect_element(const InsertMesh& M, int ci, double E[4][4]) {
    const double h = M.dr(), k = M.dz();
    const double r0 = M.r_of(ci), r1 = r0 + h;
    const double Kr[2][2] = {{0.5 * (r0 + r1) / h, -0.5 * (r0 + r1) / h}, {-0.5 * (r0 + r1) / h, 0.5 * (r0 + r1) / h}};
    const double off = h * (r0 + r1) / 12.0;
    const double Mr[2][2] = {{h * (3.0 * r0 + r1) / 12.0, off}, {off, h * (r0 + 3.0 * r1) / 12.0}};
    const double Kz[2][2] = {{1.0 / k, -1.0 / k}, {-1.0 / k, 1.0 / k}};
    const double Mz[2][2] = {{k / 3.0, k / 6.0}, {k / 6.0, k / 3.0}};
    for (int p = 0; p < 4; ++p) {
        const int pr = p & 1, pz = p >> 1;
        for (int q = 0; q < 4; ++q) {
            const int qr = q & 1, qz = q >> 1;
            E[p][q] = Kr[pr][qr] * Mz[pz][qz] + Mr[pr][qr] * Kz[pz][qz];
        }
    }
}

// The weighted element: integral over the cell of r grad(w N_p) . grad(w N_q)
// for the cell's four hats N.  The cell is cut into 2x2 boxes; a box that
// the insert cuts is split into four, level by level, down to kCutLevels;
// other boxes (and cut ones at the last level, without their points in the
// metal) take the 3x3 Gauss rule; boxes wholly in the metal add nothing.
void weighted_element(const InsertMesh& M, int ci, int cj, double E[4][4]) {
    struct Box {
        double rl, rh, zl, zh;
        int level;
    };
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) E[p][q] = 0.0;
    const double r0 = M.r_of(ci), z0 = M.z_of(cj), h = M.dr(), k = M.dz();
    std::vector<Box> todo;
    for (int b = 0; b < 4; ++b) {
        const double rl = r0 + 0.5 * h * (b & 1), zl = z0 + 0.5 * k * (b >> 1);
        todo.push_back({rl, rl + 0.5 * h, zl, zl + 0.5 * k, 0});
    }
    while (!todo.empty()) {
        const Box bx = todo.back();
        todo.pop_back();
        const Where at = M.where(bx.rl, bx.rh, bx.zl, bx.zh);
        if (at == kMetal) continue;
        if (at == kCut && bx.level < kCutLevels) {
            const double rm = 0.5 * (bx.rl + bx.rh), zm = 0.5 * (bx.zl + bx.zh);
            todo.push_back({bx.rl, rm, bx.zl, zm, bx.level + 1});
            todo.push_back({rm, bx.rh, bx.zl, zm, bx.level + 1});
            todo.push_back({bx.rl, rm, zm, bx.zh, bx.level + 1});
            todo.push_back({rm, bx.rh, zm, bx.zh, bx.level + 1});
            continue;
        }
        const double hr = bx.rh - bx.rl, hz = bx.zh - bx.zl;
        for (int a = 0; a < 3; ++a) {
            const double r = bx.rl + 0.5 * hr * (1.0 + kGaussX[a]);
            for (int b = 0; b < 3; ++b) {
                const double z = bx.zl + 0.5 * hz * (1.0 + kGaussX[b]);
                const double g = M.g(r, z);
                if (!(g > 0.0)) continue;
                const double wv = M.w(g);
                double wr, wz;
                M.w_grad(r, z, g, wr, wz);
                // hats of the cell and their derivatives at the point
                const double s = (r - r0) / h, t = (z - z0) / k;
                const double hs[2] = {1.0 - s, s}, ht[2] = {1.0 - t, t};
                const double ds[2] = {-1.0 / h, 1.0 / h}, dt[2] = {-1.0 / k, 1.0 / k};
                double gr[4], gz[4];
                for (int p = 0; p < 4; ++p) {
                    const double N = hs[p & 1] * ht[p >> 1];
                    gr[p] = wr * N + wv * (ds[p & 1] * ht[p >> 1]);
                    gz[p] = wz * N + wv * (hs[p & 1] * dt[p >> 1]);
                }
                const double f = r * ((0.25 * hr * hz) * (kGaussW[a] * kGaussW[b]));
                for (int p = 0; p < 4; ++p)
                    for (int q = 0; q < 4; ++q) E[p][q] += f * (gr[p] * gr[q] + gz[p] * gz[q]);
            }
        }
    }
}

}  // namespace

// Web-spline set-up of an instance's insert (readings of Sec. II.A for the
// gun geometry of Sec. III): node roles, the outer hats' extension blocks,
// the node set M and the correction D = A - A_rect on it, the load map and
// the basis at the nodes of M.
std::string ins_build(const pic_instance_cfg& c, InsHost& h) {
    const InsertMesh M(c);
    const int W = M.W(), NN = M.nodes(), nr = c.nr, nz = c.nz;

    // where each cell sits against the insert
    std::vector<Where> cell((size_t)nr * nz);
    std::vector<double> cell_lo((size_t)nr * nz), cell_hi((size_t)nr * nz);
    for (int ci = 0; ci < nr; ++ci)
        for (int cj = 0; cj < nz; ++cj) {
            const size_t x = (size_t)ci * nz + cj;
            M.cell_g(ci, cj, cell_lo[x], cell_hi[x]);
            cell[x] = cell_lo[x] > 0.0 ? kFree : (cell_hi[x] > 0.0 ? kCut : kMetal);
        }

    // node roles from the cells of each unknown's support: inner if one of
    // them is free, outer if none is free but one is cut, else exterior
    std::vector<int> role(NN, kFixed);
    for (int i = 0; i <= nr; ++i)
        for (int j = 0; j <= nz; ++j) {
            if (!M.unknown(i, j)) continue;
            bool free_cell = false, cut_cell = false;
            for (int di = -1; di <= 0; ++di)
                for (int dj = -1; dj <= 0; ++dj) {
                    const int ci = i + di, cj = j + dj;
                    if (ci < 0 || ci >= nr || cj < 0 || cj >= nz) continue;
                    const Where at = cell[(size_t)ci * nz + cj];
                    free_cell |= at == kFree;
                    cut_cell |= at == kCut;
                }
            role[i * W + j] = free_cell ? kInner : (cut_cell ? kOuter : kExterior);
        }
    for (int n = 0; n < NN; ++n) h.counts[role[n]] += 1;

    // blocks: lower-left corners of 2x2 squares of inner unknowns
    auto inner = [&](int i, int j) { return M.unknown(i, j) && role[i * W + j] == kInner; };
    auto block_ok = [&](int i, int j) { return inner(i, j) && inner(i + 1, j) && inner(i, j + 1) && inner(i + 1, j + 1); };

    // each outer hat joins the block whose centre is nearest (the distance
    // in units of half a cell: (2 di + 1) dr, (2 dj + 1) dz), ties to the
    // lower index in r, then in z, with the bilinear Lagrange weights of its
    // index offsets from the block's lower-left node
    std::vector<int> base(NN, -1);
    std::vector<std::array<double, 4>> ext(NN);
    for (int i = 1; i < nr; ++i)
        for (int j = 0; j <= nz; ++j) {
            const int n = i * W + j;
            if (role[n] != kOuter) continue;
            bool found = false;
            double best_d = 0.0;
            int bi = 0, bj = 0;
            for (int li = i - kBlockReach; li < i + kBlockReach; ++li)
                for (int lj = j - kBlockReach; lj < j + kBlockReach; ++lj) {
                    if (!block_ok(li, lj)) continue;
                    const double er = (double)(2 * (li - i) + 1) * M.dr();
                    const double ez = (double)(2 * (lj - j) + 1) * M.dz();
                    const double d = er * er + ez * ez;
                    if (!found || d < best_d || (d == best_d && (li < bi || (li == bi && lj < bj)))) {
                        found = true;
                        best_d = d;
                        bi = li;
                        bj = lj;
                    }
                }
            if (!found) return "no 2x2 block of inner nodes near an outer node: refine the mesh";
            const double x = (double)(i - bi), y = (double)(j - bj);
            base[n] = bi * W + bj;
            ext[n] = {(1.0 - x) * (1.0 - y), x * (1.0 - y), (1.0 - x) * y, x * y};
        }

    // the inner unknowns a node's hat contributes to, with their factors
    struct Feed {
        int n;
        double f;
    };
    auto feed = [&](int n, Feed* out) -> int {
        if (role[n] == kInner) {
            out[0] = {n, 1.0};
            return 1;
        }
        if (role[n] != kOuter) return 0;
        const int b = base[n];
        const int to[4] = {b, b + W, b + 1, b + W + 1};
        for (int q = 0; q < 4; ++q) out[q] = {to[q], ext[n][q]};
        return 4;
    };

    // cells whose matrix differs from the rectangle's: they meet the weight
    // band and are not wholly in the metal, or are in the metal with an
    // inner corner
    auto band_cell = [&](int ci, int cj) {
        const size_t x = (size_t)ci * nz + cj;
        if (!(cell_lo[x] < M.gam())) return false;
        if (cell[x] != kMetal) return true;
        for (int p = 0; p < 4; ++p)
            if (role[corner(M, ci, cj, p)] == kInner) return true;
        return false;
    };
    std::vector<char> inM(NN, 0);
    for (int ci = 0; ci < nr; ++ci)
        for (int cj = 0; cj < nz; ++cj)
            if (band_cell(ci, cj))
                for (int p = 0; p < 4; ++p) {
                    const int n = corner(M, ci, cj, p);
                    if (role[n] != kFixed) inM[n] = 1;
                }
    for (int n = 0; n < NN; ++n)
        if (role[n] == kOuter)
            for (int q = 0; q < 4; ++q) inM[base[n] + (q & 1) * W + (q >> 1)] = 1;
    h.map.assign(NN, -1);
    h.Mnode.clear();
    for (int n = 0; n < NN; ++n)
        if (inM[n]) {
            h.map[n] = (int)h.Mnode.size();
            h.Mnode.push_back(n);
        }
    h.m = (int)h.Mnode.size();

    // D on M x M as (row, column, value) triplets, summed per entry below:
    // the weighted element through the extension, minus the rectangle's
    // entries that the web-spline space replaces (pairs with an inner node;
    // outer and exterior nodes keep the rectangle's rows among themselves)
    struct Trip {
        long long rc;
        double v;
    };
    std::vector<Trip> trips;
    for (int ci = 0; ci < nr; ++ci)
        for (int cj = 0; cj < nz; ++cj) {
            if (!band_cell(ci, cj)) continue;
            int nd[4];
            for (int p = 0; p < 4; ++p) nd[p] = corner(M, ci, cj, p);
            if (cell[(size_t)ci * nz + cj] != kMetal) {
                double Ew[4][4];
                weighted_element(M, ci, cj, Ew);
                Feed fp[4], fq[4];
                for (int p = 0; p < 4; ++p) {
                    const int mp = feed(nd[p], fp);
                    for (int q = 0; q < 4; ++q) {
                        const int mq = feed(nd[q], fq);
                        for (int s = 0; s < mp; ++s)
                            for (int t = 0; t < mq; ++t)
                                trips.push_back({(long long)h.map[fp[s].n] * h.m + h.map[fq[t].n],
                                                 fp[s].f * fq[t].f * Ew[p][q]});
                    }
                }
            }
            double Er[4][4];
            rect_element(M, ci, Er);
            for (int p = 0; p < 4; ++p)
                for (int q = 0; q < 4; ++q) {
                    const int rp = role[nd[p]], rq = role[nd[q]];
                    if (rp == kFixed || rq == kFixed) continue;
                    if (rp != kInner && rq != kInner) continue;
                    trips.push_back({(long long)h.map[nd[p]] * h.m + h.map[nd[q]], -Er[p][q]});
                }
        }
    std::stable_sort(trips.begin(), trips.end(), [](const Trip& x, const Trip& y) { return x.rc < y.rc; });
    h.Dr.clear();
    h.Dc.clear();
    h.Dv.clear();
    for (size_t t = 0; t < trips.size();) {
        const long long rc = trips[t].rc;
        double v = 0.0;
        for (; t < trips.size() && trips[t].rc == rc; ++t) v += trips[t].v;
        h.Dr.push_back((int)(rc / h.m));
        h.Dc.push_back((int)(rc % h.m));
        h.Dv.push_back(v);
    }

    // load of each node of M: the charges of the hats that feed it (an inner
    // node its own, plus the outer hats whose block holds it); outer and
    // metal nodes of M take none
    std::vector<std::vector<Feed>> load(h.m);
    for (int n = 0; n < NN; ++n) {
        Feed f[4];
        const int k = feed(n, f);
        for (int q = 0; q < k; ++q)
            if (h.map[f[q].n] >= 0) load[h.map[f[q].n]].push_back({n, f[q].f});
    }
    h.rp.assign(h.m + 1, 0);
    h.rk.clear();
    h.rf.clear();
    for (int a = 0; a < h.m; ++a) {
        for (const Feed& e : load[a]) {
            h.rk.push_back(e.n);
            h.rf.push_back(e.f);
        }
        h.rp[a + 1] = (int)h.rk.size();
    }

    // the basis at the nodes of M: an inner node is its own coefficient times
    // w, an outer node inside the domain w times its block's extension, a
    // node in the metal 0
    h.typ.assign(h.m, 0);
    h.wn.assign(h.m, 0.0);
    h.ek.assign((size_t)h.m * 4, 0);
    h.ef.assign((size_t)h.m * 4, 0.0);
    for (int a = 0; a < h.m; ++a) {
        const int n = h.Mnode[a];
        const double g = M.g(M.r_of(n / W), M.z_of(n % W));
        h.wn[a] = M.w(g);
        if (role[n] == kInner) {
            h.typ[a] = 1;
        } else if (role[n] == kOuter && g > 0.0) {
            h.typ[a] = 2;
            Feed f[4];
            feed(n, f);
            for (int q = 0; q < 4; ++q) {
                h.ek[(size_t)a * 4 + q] = f[q].n;
                h.ef[(size_t)a * 4 + q] = f[q].f;
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
