// insert3.hip -- the elliptic insert with cubic shapes: weighted extended
// B-splines of degree 3 (Sec. II.A, web-splines of any degree) for the
// space-charge potential of the gun geometry (Sec. III).
//
// The rectangle's cubic system (k_field.hip) has one unknown coefficient per
// node u = (i, j), 1 <= i <= nr-1 and j over the z unknowns (1 .. nz-1
// between electrode ends, 0 .. nz with open ends); psi_u is the cubic
// B-spline of node u together with its reflections at the walls.  With the
// insert the space is
//     B_u = w (psi_u + sum_{k outer} e_ku psi_k)   over the inner u,
// w the weight function of DevInst.  An unknown is inner when a cell of its
// support (the 4 x 4 cells around its node, clipped to the rectangle) lies
// wholly outside the metal, outer when none does but one is cut by the
// ellipse, exterior otherwise.  An outer unknown joins the 4 x 4 block of
// inner unknowns whose centre is nearest to its node (ties to the lower r
// index, then z) with the tensor cubic Lagrange weights of its index offsets
// from the block's first node.  The Galerkin matrix A = int r grad B . grad B
// takes the 4 x 4 Gauss rule per cell; a cell that meets the band integrates
// on 2 x 2 boxes, boxes cut by the ellipse split into four down to kCut3
// levels (points in the metal dropped at the finest).
//
// As with bilinear shapes (insert.hip) the web-spline system keeps the
// rectangle's rows among the unknowns that are not inner, decoupled from the
// inner ones, so it differs from the rectangle's matrix only on the set M of
// the unknowns of the cells that meet the band (or lie in the metal with an
// inner B-spline alive on them) and of the extension blocks:
// A = A_rect + E D E^T, solved with two fast cubic solves and the m x m
// matrix H = (I + D G)^-1 D (the device kernels of insert.hip).  The load of
// an unknown of M is its share of Qx + Qxw through the reflections and the
// extension; the others keep the plain reflected load of Qx.  After the
// second solve the ghosted coefficients of the outer B-splines are rebuilt
// from their blocks (the exterior ones set to 0) and the nodal potential is
// phi_vac + w(node) (B-spline sum of the 3 x 3 neighbouring coefficients).
#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "pic_internal.h"

namespace pic {
namespace {

// Cut boxes are split into four down to this many levels; an outer unknown
// looks for its block within this many nodes of its own.
constexpr int kCut3 = 6;
constexpr int kReach3 = 8;

// Four-point Gauss-Legendre rule on [-1, 1] (exact to degree 7: the products
// of two cubic B-splines times r on a cell).
constexpr double kX4[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                           0.86113631159405257522};
constexpr double kW4[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                           0.34785484513745385737};

enum Role3 { kNot3 = 0, kInner3 = 1, kOuter3 = 2, kExterior3 = 3 };

struct Feed3 {
    int n;      // node of an inner unknown
    double f;   // its factor
};

// Mesh, reflections and weight function of one instance.
class Cubic3 {
public:
    explicit Cubic3(const pic_instance_cfg& c)
        : nr(c.nr), nz(c.nz), W(c.nz + 1), WX(c.nz + 3), open(c.end_mode == 2) {
        a = c.a;
        dr = (c.b - c.a) / (double)c.nr;
        dz = c.L / (double)c.nz;
        ins_fill(c, dr, dz, I);
        jlo = open ? 0 : 1;
        jhi = open ? nz : nz - 1;
    }
    const int nr, nz, W, WX;
    const bool open;
    int jlo = 0, jhi = 0;
    double a = 0.0, dr = 0.0, dz = 0.0;
    DevInst I{};

    bool unknown(int i, int j) const { return i >= 1 && i <= nr - 1 && j >= jlo && j <= jhi; }
    double r_of(int i) const { return a + (double)i * dr; }
    double z_of(int j) const { return (double)j * dz; }
    long long ghost(int gi, int gj) const { return (long long)(gi + 1) * WX + (gj + 1); }

    // a ghosted row / column onto the unknowns: the sign of the reflection,
    // 0 for a wall row (a fixed zero)
    int fold_r(int gi, int& i) const { return fold_odd(gi, nr, i); }
    int fold_z(int gj, int& j) const {
        if (!open) return fold_odd(gj, nz, j);
        j = gj < 0 ? -gj : (gj > nz ? 2 * nz - gj : gj);
        return 1;
    }

    // lowest and highest g over a box (g is one square in r plus one in z)
    void g_range(double rl, double rh, double zl, double zh, double& lo, double& hi) const {
        double ulo, uhi, vlo, vhi;
        sq_range((rl - I.ins_r0) / I.ins_er, (rh - I.ins_r0) / I.ins_er, ulo, uhi);
        sq_range((zl - I.ins_z0) / I.ins_ez, (zh - I.ins_z0) / I.ins_ez, vlo, vhi);
        lo = (ulo + vlo) - 1.0;
        hi = (uhi + vhi) - 1.0;
    }

    // weight function and its gradient at (r, z)
    void weight(double r, double z, double& w, double& wr, double& wz) const {
        const double g = ins_g(I, r, z);
        w = ins_w(I, g);
        wr = wz = 0.0;
        if (g > 0.0 && g < I.ins_gam) {
            const double s = 1.0 - g / I.ins_gam, d = 3.0 * s * s / I.ins_gam;
            wr = d * (2.0 * (r - I.ins_r0) / (I.ins_er * I.ins_er));
            wz = d * (2.0 * (z - I.ins_z0) / (I.ins_ez * I.ins_ez));
        }
    }

private:
    static int fold_odd(int g, int n, int& u) {
        if (g >= 1 && g <= n - 1) {
            u = g;
            return 1;
        }
        if (g == -1) {
            u = 1;
            return -1;
        }
        if (g == n + 1) {
            u = n - 1;
            return -1;
        }
        return 0;
    }
    static void sq_range(double x0, double x1, double& lo, double& hi) {
        const double q0 = x0 * x0, q1 = x1 * x1;
        hi = std::max(q0, q1);
        lo = (x0 <= 0.0 && x1 >= 0.0) ? 0.0 : std::min(q0, q1);
    }
};

// cubic Lagrange basis function k of the nodes 0, 1, 2, 3 at x
double lagrange3(int k, double x) {
    double v = 1.0;
    for (int m = 0; m < 4; ++m)
        if (m != k) v *= (x - (double)m) / (double)(k - m);
    return v;
}

// 1-D matrices of the four B-splines alive on the cell [x0, x0 + h]:
// stiffness K and mass Mm, weighted by x when radial.
void cell_1d(double x0, double h, bool radial, double K[4][4], double Mm[4][4]) {
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) K[p][q] = Mm[p][q] = 0.0;
    for (int t = 0; t < 4; ++t) {
        const double f = 0.5 * (1.0 + kX4[t]);
        const double wt = 0.5 * h * kW4[t] * (radial ? x0 + f * h : 1.0);
        double b[4], db[4];
        bspline3(f, b, db);
        for (int p = 0; p < 4; ++p)
            for (int q = 0; q < 4; ++q) {
                K[p][q] += wt * ((db[p] / h) * (db[q] / h));
                Mm[p][q] += wt * (b[p] * b[q]);
            }
    }
}

// The rectangle's element of a cell in column ci: Kr (x) Mz + Mr (x) Kz over
// its 16 B-splines (p = 4 a + b: the one of ghosted node (ci-1+a, cj-1+b)).
void rect_element3(const Cubic3& M, int ci, double E[16][16]) {
    double Kr[4][4], Mr[4][4], Kz[4][4], Mz[4][4];
    cell_1d(M.r_of(ci), M.dr, true, Kr, Mr);
    cell_1d(0.0, M.dz, false, Kz, Mz);
    for (int p = 0; p < 16; ++p)
        for (int q = 0; q < 16; ++q)
            E[p][q] = Kr[p / 4][q / 4] * Mz[p % 4][q % 4] + Mr[p / 4][q / 4] * Kz[p % 4][q % 4];
}

// 4 x 4 Gauss points of the box [rl, rh] x [zl, zh] inside the cell with
// origin (r0, z0), added to E = int r grad(w b_p) . grad(w b_q) (w = 1 when
// not weighted; points in the metal skipped when drop).
void box_points(const Cubic3& M, double r0, double z0, double rl, double rh, double zl, double zh, bool weighted,
                bool drop, double E[16][16]) {
    const double hr = rh - rl, hz = zh - zl;
    for (int s = 0; s < 4; ++s)
        for (int t = 0; t < 4; ++t) {
            const double r = rl + 0.5 * hr * (1.0 + kX4[s]), z = zl + 0.5 * hz * (1.0 + kX4[t]);
            if (drop && !(ins_g(M.I, r, z) > 0.0)) continue;
            double w = 1.0, wr = 0.0, wz = 0.0;
            if (weighted) M.weight(r, z, w, wr, wz);
            double br[4], dbr[4], bz[4], dbz[4];
            bspline3((r - r0) / M.dr, br, dbr);
            bspline3((z - z0) / M.dz, bz, dbz);
            double gr[16], gz[16];
            for (int p = 0; p < 16; ++p) {
                const double v = br[p / 4] * bz[p % 4];
                gr[p] = wr * v + w * ((dbr[p / 4] / M.dr) * bz[p % 4]);
                gz[p] = wz * v + w * (br[p / 4] * (dbz[p % 4] / M.dz));
            }
            const double q = r * ((0.25 * hr * hz) * (kW4[s] * kW4[t]));
            for (int p = 0; p < 16; ++p)
                for (int k = 0; k < 16; ++k) E[p][k] += q * (gr[p] * gr[k] + gz[p] * gz[k]);
        }
}

// The web-spline element of cell (ci, cj) on its 16 B-splines: the plain
// rule when w = 1 on the whole cell (cell_lo >= gam), else the weighted rule
// on 2 x 2 boxes refined where the ellipse cuts them.
void web_element3(const Cubic3& M, int ci, int cj, double cell_lo, double E[16][16]) {
    for (int p = 0; p < 16; ++p)
        for (int q = 0; q < 16; ++q) E[p][q] = 0.0;
    const double r0 = M.r_of(ci), z0 = M.z_of(cj);
    if (cell_lo >= M.I.ins_gam) {
        box_points(M, r0, z0, r0, r0 + M.dr, z0, z0 + M.dz, false, false, E);
        return;
    }
    struct Box {
        double rl, rh, zl, zh;
        int level;
    };
    std::vector<Box> todo;
    for (int b = 0; b < 4; ++b) {
        const double rl = r0 + 0.5 * M.dr * (b & 1), zl = z0 + 0.5 * M.dz * (b >> 1);
        todo.push_back({rl, rl + 0.5 * M.dr, zl, zl + 0.5 * M.dz, 0});
    }
    while (!todo.empty()) {
        const Box bx = todo.back();
        todo.pop_back();
        double lo, hi;
        M.g_range(bx.rl, bx.rh, bx.zl, bx.zh, lo, hi);
        if (!(hi > 0.0)) continue;
        if (!(lo > 0.0) && bx.level < kCut3) {
            const double rm = 0.5 * (bx.rl + bx.rh), zm = 0.5 * (bx.zl + bx.zh);
            todo.push_back({bx.rl, rm, bx.zl, zm, bx.level + 1});
            todo.push_back({rm, bx.rh, bx.zl, zm, bx.level + 1});
            todo.push_back({bx.rl, rm, zm, bx.zh, bx.level + 1});
            todo.push_back({rm, bx.rh, zm, bx.zh, bx.level + 1});
            continue;
        }
        box_points(M, r0, z0, bx.rl, bx.rh, bx.zl, bx.zh, true, true, E);
    }
}

}  // namespace

// Web-spline set-up of degree 3 for an instance's insert (readings of
// Sec. II.A for the gun geometry of Sec. III): unknown roles, the outer
// unknowns' extension blocks, the set M and the correction D = A - A_rect on
// it, the load map of M and the ghosted coefficients rebuilt after a solve.
std::string ins3_build(const pic_instance_cfg& c, Ins3Host& h) {
    const Cubic3 M(c);
    const int nr = c.nr, nz = c.nz, W = M.W, NN = (nr + 1) * W;
    h = Ins3Host();

    // where each cell sits against the insert
    std::vector<double> clo((size_t)nr * nz), chi((size_t)nr * nz);
    for (int ci = 0; ci < nr; ++ci)
        for (int cj = 0; cj < nz; ++cj)
            M.g_range(M.r_of(ci), M.r_of(ci) + M.dr, M.z_of(cj), M.z_of(cj) + M.dz, clo[(size_t)ci * nz + cj],
                      chi[(size_t)ci * nz + cj]);

    // roles from the cells of each unknown's support
    std::vector<int> role(NN, kNot3);
    for (int i = 1; i <= nr - 1; ++i)
        for (int j = M.jlo; j <= M.jhi; ++j) {
            bool free_cell = false, cut_cell = false;
            for (int ci = std::max(0, i - 2); ci <= std::min(nr - 1, i + 1); ++ci)
                for (int cj = std::max(0, j - 2); cj <= std::min(nz - 1, j + 1); ++cj) {
                    const size_t x = (size_t)ci * nz + cj;
                    if (clo[x] > 0.0) free_cell = true;
                    else if (chi[x] > 0.0) cut_cell = true;
                }
            role[i * W + j] = free_cell ? kInner3 : (cut_cell ? kOuter3 : kExterior3);
        }
    for (int n = 0; n < NN; ++n) h.counts[role[n]] += 1;

    // extension blocks: 4 x 4 squares of inner unknowns, the nearest centre
    auto inner = [&](int i, int j) { return M.unknown(i, j) && role[i * W + j] == kInner3; };
    auto block_ok = [&](int li, int lj) {
        for (int x = 0; x < 4; ++x)
            for (int y = 0; y < 4; ++y)
                if (!inner(li + x, lj + y)) return false;
        return true;
    };
    std::vector<int> blk(NN, -1);
    std::vector<std::array<double, 16>> ext(NN);
    for (int i = 1; i <= nr - 1; ++i)
        for (int j = M.jlo; j <= M.jhi; ++j) {
            const int n = i * W + j;
            if (role[n] != kOuter3) continue;
            bool found = false;
            double best = 0.0;
            int bi = 0, bj = 0;
            for (int li = i - kReach3; li <= i + kReach3 - 3; ++li)
                for (int lj = j - kReach3; lj <= j + kReach3 - 3; ++lj) {
                    if (!block_ok(li, lj)) continue;
                    const double du = ((double)li + 1.5 - (double)i) * M.dr;
                    const double dv = ((double)lj + 1.5 - (double)j) * M.dz;
                    const double d2 = du * du + dv * dv;
                    if (!found || d2 < best || (d2 == best && (li < bi || (li == bi && lj < bj)))) {
                        found = true;
                        best = d2;
                        bi = li;
                        bj = lj;
                    }
                }
            if (!found) return "no 4x4 block of inner unknowns near an outer unknown: refine the mesh";
            blk[n] = bi * W + bj;
            for (int x = 0; x < 4; ++x)
                for (int y = 0; y < 4; ++y)
                    ext[n][x * 4 + y] = lagrange3(x, (double)(i - bi)) * lagrange3(y, (double)(j - bj));
        }

    // the unknown a ghosted B-spline reflects onto (node, sign; sign 0: none)
    auto fold = [&](int gi, int gj, int& node) {
        int ui, uj;
        const int si = M.fold_r(gi, ui), sj = M.fold_z(gj, uj);
        node = (si && sj) ? ui * W + uj : -1;
        return si * sj;
    };
    // the inner unknowns a ghosted B-spline feeds, with their factors
    auto feeds = [&](int gi, int gj, Feed3* out) -> int {
        int u;
        const int s = fold(gi, gj, u);
        if (!s) return 0;
        if (role[u] == kInner3) {
            out[0] = {u, (double)s};
            return 1;
        }
        if (role[u] != kOuter3) return 0;
        for (int q = 0; q < 16; ++q) out[q] = {blk[u] + (q / 4) * W + (q % 4), (double)s * ext[u][q]};
        return 16;
    };

    // D = A - A_rect, cell by cell where they differ: cells that meet the
    // band, and any cell with a B-spline that is not an inner one alive on it
    struct Trip {
        long long key;   // row node * NN + column node
        double v;
    };
    std::vector<Trip> trips;
    std::vector<int> loc(NN, -1);
    std::vector<int> lnodes;
    std::vector<double> acc;
    for (int ci = 0; ci < nr; ++ci)
        for (int cj = 0; cj < nz; ++cj) {
            const size_t x = (size_t)ci * nz + cj;
            Feed3 fd[16][16];
            int nf[16], un[16], sg[16];
            bool differs = clo[x] < M.I.ins_gam;
            for (int p = 0; p < 16; ++p) {
                const int gi = ci - 1 + p / 4, gj = cj - 1 + p % 4;
                sg[p] = fold(gi, gj, un[p]);
                nf[p] = feeds(gi, gj, fd[p]);
                if (sg[p] && role[un[p]] != kInner3) differs = true;
            }
            if (!differs) continue;
            bool any_inner = false;
            for (int p = 0; p < 16; ++p) any_inner = any_inner || (sg[p] && role[un[p]] == kInner3);
            if (!any_inner && !(chi[x] > 0.0)) continue;  // metal, nothing to replace
            // the unknowns the cell couples, numbered locally
            lnodes.clear();
            auto local = [&](int n) {
                if (loc[n] < 0) {
                    loc[n] = (int)lnodes.size();
                    lnodes.push_back(n);
                }
                return loc[n];
            };
            for (int p = 0; p < 16; ++p) {
                if (sg[p]) local(un[p]);
                for (int t = 0; t < nf[p]; ++t) local(fd[p][t].n);
            }
            const int nl = (int)lnodes.size();
            acc.assign((size_t)nl * nl, 0.0);
            if (chi[x] > 0.0) {
                double Ew[16][16];
                web_element3(M, ci, cj, clo[x], Ew);
                for (int p = 0; p < 16; ++p)
                    for (int q = 0; q < 16; ++q)
                        for (int s = 0; s < nf[p]; ++s)
                            for (int t = 0; t < nf[q]; ++t)
                                acc[(size_t)loc[fd[p][s].n] * nl + loc[fd[q][t].n]] +=
                                    (fd[p][s].f * fd[q][t].f) * Ew[p][q];
            }
            double Er[16][16];
            rect_element3(M, ci, Er);
            for (int p = 0; p < 16; ++p)
                for (int q = 0; q < 16; ++q) {
                    if (!sg[p] || !sg[q]) continue;
                    if (role[un[p]] != kInner3 && role[un[q]] != kInner3) continue;
                    acc[(size_t)loc[un[p]] * nl + loc[un[q]]] -= (double)(sg[p] * sg[q]) * Er[p][q];
                }
            for (int s = 0; s < nl; ++s)
                for (int t = 0; t < nl; ++t) {
                    const double v = acc[(size_t)s * nl + t];
                    if (v != 0.0) trips.push_back({(long long)lnodes[s] * NN + lnodes[t], v});
                }
            for (int n : lnodes) loc[n] = -1;
        }
    std::stable_sort(trips.begin(), trips.end(), [](const Trip& p, const Trip& q) { return p.key < q.key; });

    // M: the unknowns of D and of the extension blocks
    std::vector<char> inM(NN, 0);
    for (const Trip& t : trips) {
        inM[t.key / NN] = 1;
        inM[t.key % NN] = 1;
    }
    for (int n = 0; n < NN; ++n)
        if (role[n] == kOuter3)
            for (int q = 0; q < 16; ++q) inM[blk[n] + (q / 4) * W + (q % 4)] = 1;
    h.map.assign(NN, -1);
    for (int n = 0; n < NN; ++n)
        if (inM[n]) {
            h.map[n] = (int)h.Mnode.size();
            h.Mnode.push_back(n);
        }
    h.m = (int)h.Mnode.size();
    for (size_t t = 0; t < trips.size();) {
        const long long key = trips[t].key;
        double v = 0.0;
        for (; t < trips.size() && trips[t].key == key; ++t) v += trips[t].v;
        h.Dr.push_back(h.map[key / NN]);
        h.Dc.push_back(h.map[key % NN]);
        h.Dv.push_back(v);
    }

    // load of M: every ghosted B-spline's charge carried to the inner
    // unknowns it feeds (the unknowns of M that are not inner take none)
    std::vector<std::vector<std::pair<int, double>>> load(h.m);
    for (int gi = -1; gi <= nr + 1; ++gi)
        for (int gj = -1; gj <= nz + 1; ++gj) {
            Feed3 f[16];
            const int k = feeds(gi, gj, f);
            for (int t = 0; t < k; ++t)
                if (h.map[f[t].n] >= 0) load[h.map[f[t].n]].push_back({(int)M.ghost(gi, gj), f[t].f});
        }
    h.rp.assign(h.m + 1, 0);
    h.typ.assign(h.m, 0);
    for (int a = 0; a < h.m; ++a) {
        h.typ[a] = role[h.Mnode[a]] == kInner3 ? 1 : 0;
        if (h.typ[a])
            for (const auto& e : load[a]) {
                h.rk.push_back(e.first);
                h.rf.push_back(e.second);
            }
        h.rp[a + 1] = (int)h.rk.size();
    }

    // ghosted coefficients that a solve's reflected values do not give: the
    // outer B-splines' (from their blocks) and the exterior ones' (zero)
    for (int gi = -1; gi <= nr + 1; ++gi)
        for (int gj = -1; gj <= nz + 1; ++gj) {
            int u;
            const int s = fold(gi, gj, u);
            if (!s || role[u] == kInner3) continue;
            h.xk.push_back((int)M.ghost(gi, gj));
            for (int q = 0; q < 16; ++q) {
                const bool outer = role[u] == kOuter3;
                h.xn.push_back(outer ? blk[u] + (q / 4) * W + (q % 4) : -1);
                h.xf.push_back(outer ? (double)s * ext[u][q] : 0.0);
            }
        }
    h.nx = (int)h.xk.size();
    return "";
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
namespace {

// load of the unknowns of M, after the plain reflected load of every unknown
__global__ void ki3_rhs(const DevInst* It, const Ins3Dev* Xt, const FieldDev* Ft, const double* bscale) {
    const Ins3Dev& X = Xt[blockIdx.y];
    if (It[X.inst].frozen) return;
    const FieldDev& F = Ft[X.inst];
    const double bs = bscale[X.inst];
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < X.m; a += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (X.typ[a]) {
            double s = 0.0;
            for (int t = X.rp[a]; t < X.rp[a + 1]; ++t) {
                const int k = X.rk[t];
                s += X.rf[t] * (double)(F.Qx[k] + F.Qw[k]);
            }
            v = s * bs;
        }
        F.rhs[X.Mnode[a]] = v;
    }
}

// the ghosted coefficients of the outer and exterior B-splines from the
// solved coefficients c (the cubic table's phi)
__global__ void ki3_fix_cx(const DevInst* It, const Ins3Dev* Xt, const FieldDev* Ft, const FieldDev* F3) {
    const Ins3Dev& X = Xt[blockIdx.y];
    if (It[X.inst].frozen) return;
    const FieldDev& F = Ft[X.inst];
    const double* c = F3[X.inst].phi;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < X.nx; e += gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int q = 0; q < 16; ++q) {
            const int n = X.xn[(size_t)e * 16 + q];
            if (n >= 0) v += X.xf[(size_t)e * 16 + q] * c[n];
        }
        F.cx[X.xk[e]] = v;
        if (F.cxf) F.cxf[X.xk[e]] = (float)v;
    }
}

// nodal potential phi_vac + w (B-spline sum of the 3 x 3 coefficients
// around the node, B(0) = 4/6, B(+-1) = 1/6)
__global__ void ki3_phi(const DevInst* It, const Ins3Dev* Xt, const FieldDev* Ft) {
    const Ins3Dev& X = Xt[blockIdx.y];
    const DevInst& I = It[X.inst];
    if (I.frozen) return;
    const FieldDev& F = Ft[X.inst];
    const int W = I.W, WX = I.nz + 3;
    const double nb[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < I.nodes; n += gridDim.x * blockDim.x) {
        const int i = n / W, j = n - i * W;
        double v = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) v += (nb[a] * nb[b]) * F.cx[(long long)(i + a) * WX + (j + b)];
        const double w = ins_w(I, ins_g(I, I.a + (double)i * I.dr, (double)j * I.dz));
        F.phi[n] = F.phi_vac[n] + w * v;
    }
}

unsigned blocks3(long long n, long long cap = 1024) {
    return (unsigned)std::max(1ll, std::min((n + 255) / 256, cap));
}

}  // namespace

hipError_t launch_ins3_rhs(const DevInst* It, const Ins3Dev* X, int n_ins, int max_m, const FieldDev* Ft,
                           const double* bscale, hipStream_t s) {
    if (n_ins <= 0) return hipSuccess;
    hipLaunchKernelGGL(ki3_rhs, dim3(blocks3(max_m), n_ins), dim3(256), 0, s, It, X, Ft, bscale);
    return hipGetLastError();
}

hipError_t launch_ins3_post(const DevInst* It, const Ins3Dev* X, int n_ins, int max_nx, long long max_nodes,
                            const FieldDev* Ft, const FieldDev* F3, hipStream_t s) {
    if (n_ins <= 0) return hipSuccess;
    hipLaunchKernelGGL(ki3_fix_cx, dim3(blocks3(max_nx), n_ins), dim3(256), 0, s, It, X, Ft, F3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ki3_phi, dim3(blocks3(max_nodes), n_ins), dim3(256), 0, s, It, X, Ft);
    return hipGetLastError();
}

}  // namespace pic
