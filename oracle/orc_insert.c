/*
 * orc_insert.c -- oracle: the elliptic insert on the outer electrode, with
 * weighted extended B-splines (web-splines) of degree 1.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Geometry (Sec. III, the gun geometry: a filled ellipse on the outer
 * cylinder): metal where
 *     g(r,z) = ((r - r0)/er)^2 + ((z - z0)/ez)^2 - 1 <= 0,
 * held at V_outer.
 *
 * Web-spline FEM (Sec. II.A, after Hollig): the space-charge potential, which
 * vanishes on every electrode, is sought in the span of
 *     B_i = w (b_i + sum_{k outer} e_ik b_k)          (i inner)
 * with b the bilinear hat functions of the rectangular grid and a weight
 * function that vanishes on the insert:
 *     w = 0 (g <= 0),  1 - (1 - g/gam)^3 (0 < g < gam),  1 (g >= gam),
 * gam = 2 band max(dr/er, dz/ez), a band about `band` cells wide.
 * A hat is inner if some grid cell of its support lies entirely outside the
 * metal; outer if its support meets the domain but holds no such cell;
 * exterior if its support lies in the metal.  An outer hat k is attached to
 * the 2x2 block of inner hats nearest to it (distance from k to the block
 * centre; ties to the lower indices) with the bilinear Lagrange weights of
 * the block evaluated at k's indices (e = (1-x)(1-y), x(1-y), (1-x)y, xy with
 * x, y the index offsets of k from the block's first node).
 *
 * Galerkin matrix A_ij = int r grad B_i . grad B_j dr dz, assembled per cell:
 * cells with w = 1 throughout (g >= gam) take the exact Q1 element matrix;
 * the others a 3x3 Gauss-Legendre rule on 2x2 boxes, boxes cut by the insert
 * being split into four again down to QDEPTH levels (points in the metal
 * dropped at the finest level).  Load of a macro-particle of charge q: q B_i(x_p), i.e. the node
 * charges of the plain bilinear deposit (Q) plus those of q (w(x_p) - 1)
 * (Qw), carried through the extension.  Nodes that are not inner keep the
 * plain grid rows among themselves and are decoupled from the inner ones, so
 * their coefficients are 0.  The system is solved by a banded Cholesky
 * factorisation.  The potential at a node is sum_i c_i B_i(node): w c at inner
 * nodes, w times the extension at outer nodes outside the metal, 0 inside.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_ins {
    int nr, nz, W, j0, j1;
    double a, dr, dz, gam;
    int* cls;        /* per node: 0 not an unknown (Dirichlet row), 1 inner, 2 outer, 3 exterior */
    int* blk;        /* per outer node: node index of its block's first node (l1, l2) */
    double* e4;      /* per outer node: weights of (l1,l2), (l1+1,l2), (l1,l2+1), (l1+1,l2+1) */
    int* uidx;       /* per node: unknown index or -1 */
    int N, bw;
    double* Lb;      /* Cholesky factor, row u holds L[u][u-d] at Lb[u*(bw+1)+d] */
};

int orc_has_insert(const orc_cfg* c) { return c->ins_er > 0.0 && c->ins_ez > 0.0; }

double orc_ins_g(const orc_cfg* c, double r, double z) {
    double u = (r - c->ins_r0) / c->ins_er;
    double v = (z - c->ins_z0) / c->ins_ez;
    return (u * u + v * v) - 1.0;
}

double orc_ins_gamma(const orc_cfg* c) {
    double dr = (c->b - c->a) / (double)c->nr, dz = c->L / (double)c->nz;
    double band = c->ins_band > 0.0 ? c->ins_band : 3.0;
    return 2.0 * band * fmax(dr / c->ins_er, dz / c->ins_ez);
}

/* weight at a particle position (value only) */
double orc_ins_wp(const orc_cfg* c, double r, double z) {
    double g = orc_ins_g(c, r, z), gam = orc_ins_gamma(c);
    if (g <= 0.0) return 0.0;
    if (g >= gam) return 1.0;
    double s = 1.0 - g / gam;
    return 1.0 - s * s * s;
}

/* weight and its gradient */
double orc_ins_weight(const orc_cfg* c, double r, double z, double* wr, double* wz) {
    double g = orc_ins_g(c, r, z), gam = orc_ins_gamma(c);
    if (g <= 0.0 || g >= gam) {
        *wr = 0.0;
        *wz = 0.0;
        return g <= 0.0 ? 0.0 : 1.0;
    }
    double s = 1.0 - g / gam;
    double dw = 3.0 * s * s / gam;
    *wr = dw * (2.0 * (r - c->ins_r0) / (c->ins_er * c->ins_er));
    *wz = dw * (2.0 * (z - c->ins_z0) / (c->ins_ez * c->ins_ez));
    return 1.0 - s * s * s;
}

/* Exact range of g over a box: g is a sum of convex parabolas in r and z, so
 * its minimum sits at the clamped centre and its maximum at a corner. */
static void box_g(const orc_cfg* c, double rl, double rh, double zl, double zh, double* gmin, double* gmax) {
    double rc = c->ins_r0 < rl ? rl : (c->ins_r0 > rh ? rh : c->ins_r0);
    double zc = c->ins_z0 < zl ? zl : (c->ins_z0 > zh ? zh : c->ins_z0);
    double rf = fabs(rl - c->ins_r0) > fabs(rh - c->ins_r0) ? rl : rh;
    double zf = fabs(zl - c->ins_z0) > fabs(zh - c->ins_z0) ? zl : zh;
    *gmin = orc_ins_g(c, rc, zc);
    *gmax = orc_ins_g(c, rf, zf);
}

int orc_ins_box_hits(const orc_cfg* c, double rl, double rh, double zl, double zh) {
    double gmin, gmax;
    box_g(c, rl, rh, zl, zh, &gmin, &gmax);
    return gmin <= 0.0;
}

static void cell_g(const orc_ins* I, const orc_cfg* c, int ci, int cj, double* gmin, double* gmax) {
    double rl = I->a + (double)ci * I->dr, zl = (double)cj * I->dz;
    box_g(c, rl, rl + I->dr, zl, zl + I->dz, gmin, gmax);
}

/* 0 when the insert keeps its band clear of the inner electrode and of
 * Dirichlet ends, else a negative code */
int orc_ins_check(const orc_cfg* c) {
    if (!orc_has_insert(c)) return 0;
    double dr = (c->b - c->a) / (double)c->nr, dz = c->L / (double)c->nz;
    double s = sqrt(1.0 + orc_ins_gamma(c));
    if (c->ins_r0 - c->ins_er * s < c->a + 3.0 * dr) return -1;
    if (c->end_mode != 2 && (c->ins_z0 - c->ins_ez * s < 3.0 * dz || c->ins_z0 + c->ins_ez * s > c->L - 3.0 * dz))
        return -2;
    return 0;
}

/* unknowns (i, j) -> index: rows i = 1..nr-1, columns j = j0..j1, the
 * shorter direction running fastest (keeps the band narrow) */
static int unk_of(const orc_ins* I, int i, int j) {
    int nri = I->nr - 1, nzu = I->j1 - I->j0 + 1;
    if (nri <= nzu) return (j - I->j0) * nri + (i - 1);
    return (i - 1) * nzu + (j - I->j0);
}

/* the unknowns that hat n feeds, with their factors (inner: itself; outer:
 * its block) */
static int factors(const orc_ins* I, int n, int* u, double* f) {
    if (n < 0 || I->uidx[n] < 0) return 0;
    if (I->cls[n] == 1) {
        u[0] = I->uidx[n];
        f[0] = 1.0;
        return 1;
    }
    if (I->cls[n] != 2) return 0;
    int b = I->blk[n];
    int nodes[4] = {b, b + I->W, b + 1, b + I->W + 1};
    for (int q = 0; q < 4; ++q) {
        u[q] = I->uidx[nodes[q]];
        f[q] = I->e4[(size_t)n * 4 + q];
    }
    return 4;
}

/* corners of cell (ci, cj): (0,0), (1,0), (0,1), (1,1) in (r, z) */
static const int CR[4] = {0, 1, 0, 1}, CZ[4] = {0, 0, 1, 1};

static void exact_q1(const orc_ins* I, int ci, double E[4][4]) {
    double rl = I->a + (double)ci * I->dr, rh = rl + I->dr, rm = 0.5 * (rl + rh);
    double kr[2][2] = {{rm / I->dr, -rm / I->dr}, {-rm / I->dr, rm / I->dr}};
    double mr[2][2] = {{I->dr * (3.0 * rl + rh) / 12.0, I->dr * (rl + rh) / 12.0},
                       {I->dr * (rl + rh) / 12.0, I->dr * (rl + 3.0 * rh) / 12.0}};
    double kz[2][2] = {{1.0 / I->dz, -1.0 / I->dz}, {-1.0 / I->dz, 1.0 / I->dz}};
    double mz[2][2] = {{2.0 * I->dz / 6.0, I->dz / 6.0}, {I->dz / 6.0, 2.0 * I->dz / 6.0}};
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q)
            E[p][q] = kr[CR[p]][CR[q]] * mz[CZ[p]][CZ[q]] + mr[CR[p]][CR[q]] * kz[CZ[p]][CZ[q]];
}

static const double GX[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
static const double GW[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
#define QDEPTH 6   /* finest box: a cell / 2^(QDEPTH+1) per side */

/* Integration rule for a cell that meets the weight function's band: the
 * cell is split into 2x2 boxes; a box inside the domain (g > 0 throughout)
 * takes the 3x3 Gauss-Legendre rule, a box in the metal is dropped, a box cut
 * by the insert is split into four again, down to QDEPTH levels, where the
 * Gauss points inside the metal are dropped.  `visit` receives every point
 * (r, z) with its weight. */
typedef void (*qvisit)(double r, double z, double wq, void* ctx);

static void quad_box(const orc_cfg* c, double rl, double rh, double zl, double zh, int depth, qvisit visit,
                     void* ctx) {
    double gmin, gmax;
    box_g(c, rl, rh, zl, zh, &gmin, &gmax);
    if (gmax <= 0.0) return;
    if (gmin <= 0.0 && depth < QDEPTH) {
        double rm = 0.5 * (rl + rh), zm = 0.5 * (zl + zh);
        quad_box(c, rl, rm, zl, zm, depth + 1, visit, ctx);
        quad_box(c, rm, rh, zl, zm, depth + 1, visit, ctx);
        quad_box(c, rl, rm, zm, zh, depth + 1, visit, ctx);
        quad_box(c, rm, rh, zm, zh, depth + 1, visit, ctx);
        return;
    }
    double hr = rh - rl, hz = zh - zl;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double r = rl + 0.5 * hr * (1.0 + GX[a]);
            double z = zl + 0.5 * hz * (1.0 + GX[b]);
            if (gmin <= 0.0 && orc_ins_g(c, r, z) <= 0.0) continue;
            visit(r, z, (0.25 * hr * hz) * GW[a] * GW[b], ctx);
        }
}

static void quad_cell(const orc_ins* I, const orc_cfg* c, int ci, int cj, qvisit visit, void* ctx) {
    double rl = I->a + (double)ci * I->dr, zl = (double)cj * I->dz;
    double hr = 0.5 * I->dr, hz = 0.5 * I->dz;
    for (int sr = 0; sr < 2; ++sr)
        for (int sz = 0; sz < 2; ++sz)
            quad_box(c, rl + hr * sr, rl + hr * (sr + 1), zl + hz * sz, zl + hz * (sz + 1), 0, visit, ctx);
}

typedef struct {
    const orc_cfg* c;
    double rl, zl, dr, dz;
    double E[4][4];
} wq_ctx;

static void wq_visit(double r, double z, double wq, void* vctx) {
    wq_ctx* X = (wq_ctx*)vctx;
    double wr, wz, w = orc_ins_weight(X->c, r, z, &wr, &wz);
    double fr = (r - X->rl) / X->dr, fz = (z - X->zl) / X->dz;
    double N[4] = {(1.0 - fr) * (1.0 - fz), fr * (1.0 - fz), (1.0 - fr) * fz, fr * fz};
    double Nr[4] = {-(1.0 - fz) / X->dr, (1.0 - fz) / X->dr, -fz / X->dr, fz / X->dr};
    double Nz[4] = {-(1.0 - fr) / X->dz, -fr / X->dz, (1.0 - fr) / X->dz, fr / X->dz};
    double gr[4], gz[4];
    for (int p = 0; p < 4; ++p) {
        gr[p] = wr * N[p] + w * Nr[p];
        gz[p] = wz * N[p] + w * Nz[p];
    }
    double qw = r * wq;
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) X->E[p][q] += qw * (gr[p] * gr[q] + gz[p] * gz[q]);
}

/* weighted element matrix int r grad(w b_p) . grad(w b_q) over the part of
 * the cell outside the metal */
static void weighted_q1(const orc_ins* I, const orc_cfg* c, int ci, int cj, double E[4][4]) {
    wq_ctx X;
    memset(&X, 0, sizeof(X));
    X.c = c;
    X.rl = I->a + (double)ci * I->dr;
    X.zl = (double)cj * I->dz;
    X.dr = I->dr;
    X.dz = I->dz;
    quad_cell(I, c, ci, cj, wq_visit, &X);
    memcpy(E, X.E, sizeof(X.E));
}

void orc_ins_destroy(orc_ins* I) {
    if (!I) return;
    free(I->cls); free(I->blk); free(I->e4); free(I->uidx); free(I->Lb);
    free(I);
}

int orc_ins_classify(const orc_cfg* c, int* cls_out) {
    orc_ins* I = orc_ins_create(c);
    if (!I) return -1;
    memcpy(cls_out, I->cls, sizeof(int) * (size_t)(I->nr + 1) * I->W);
    orc_ins_destroy(I);
    return 0;
}

orc_ins* orc_ins_create(const orc_cfg* c) {
    if (!orc_has_insert(c) || orc_ins_check(c) != 0) return NULL;
    orc_ins* I = (orc_ins*)calloc(1, sizeof(orc_ins));
    I->nr = c->nr; I->nz = c->nz; I->W = c->nz + 1;
    I->j0 = c->end_mode == 2 ? 0 : 1;
    I->j1 = c->end_mode == 2 ? c->nz : c->nz - 1;
    I->a = c->a;
    I->dr = (c->b - c->a) / (double)c->nr;
    I->dz = c->L / (double)c->nz;
    I->gam = orc_ins_gamma(c);
    const int W = I->W, NN = (c->nr + 1) * W;
    I->cls = (int*)calloc(NN, sizeof(int));
    I->blk = (int*)calloc(NN, sizeof(int));
    I->e4 = (double*)calloc((size_t)NN * 4, sizeof(double));
    I->uidx = (int*)malloc(sizeof(int) * NN);
    for (int n = 0; n < NN; ++n) I->uidx[n] = -1;
    /* node classes */
    for (int i = 1; i <= c->nr - 1; ++i)
        for (int j = I->j0; j <= I->j1; ++j) {
            int any_in = 0, any_cut = 0;
            for (int ci = i - 1; ci <= i; ++ci)
                for (int cj = j - 1; cj <= j; ++cj) {
                    if (ci < 0 || ci >= c->nr || cj < 0 || cj >= c->nz) continue;
                    double gmin, gmax;
                    cell_g(I, c, ci, cj, &gmin, &gmax);
                    if (gmin > 0.0) any_in = 1;
                    else if (gmax > 0.0) any_cut = 1;
                }
            int n = i * W + j;
            I->cls[n] = any_in ? 1 : (any_cut ? 2 : 3);
            I->uidx[n] = unk_of(I, i, j);
        }
    I->N = (c->nr - 1) * (I->j1 - I->j0 + 1);
    /* extension blocks of the outer nodes */
    const int R = 4;
    for (int k1 = 1; k1 <= c->nr - 1; ++k1)
        for (int k2 = I->j0; k2 <= I->j1; ++k2) {
            int n = k1 * W + k2;
            if (I->cls[n] != 2) continue;
            double best = -1.0;
            int bl1 = 0, bl2 = 0;
            for (int l1 = k1 - R; l1 <= k1 + R - 1; ++l1)
                for (int l2 = k2 - R; l2 <= k2 + R - 1; ++l2) {
                    if (l1 < 1 || l1 + 1 > c->nr - 1 || l2 < I->j0 || l2 + 1 > I->j1) continue;
                    if (I->cls[l1 * W + l2] != 1 || I->cls[(l1 + 1) * W + l2] != 1 ||
                        I->cls[l1 * W + l2 + 1] != 1 || I->cls[(l1 + 1) * W + l2 + 1] != 1)
                        continue;
                    double du = ((double)l1 + 0.5 - (double)k1) * I->dr;
                    double dv = ((double)l2 + 0.5 - (double)k2) * I->dz;
                    double d2 = du * du + dv * dv;
                    if (best < 0.0 || d2 < best) {
                        best = d2;
                        bl1 = l1;
                        bl2 = l2;
                    }
                }
            if (best < 0.0) {
                orc_ins_destroy(I);
                return NULL;
            }
            double x = (double)(k1 - bl1), y = (double)(k2 - bl2);
            I->blk[n] = bl1 * W + bl2;
            I->e4[(size_t)n * 4 + 0] = (1.0 - x) * (1.0 - y);
            I->e4[(size_t)n * 4 + 1] = x * (1.0 - y);
            I->e4[(size_t)n * 4 + 2] = (1.0 - x) * y;
            I->e4[(size_t)n * 4 + 3] = x * y;
        }
    /* bandwidth from the couplings of every cell */
    int bw = 0;
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj) {
            int us[20], nu = 0;
            for (int p = 0; p < 4; ++p) {
                int n = (ci + CR[p]) * W + cj + CZ[p];
                int u[4];
                double f[4];
                int m = factors(I, n, u, f);
                for (int q = 0; q < m; ++q) us[nu++] = u[q];
                if (I->uidx[n] >= 0) us[nu++] = I->uidx[n];
            }
            for (int p = 0; p < nu; ++p)
                for (int q = 0; q < nu; ++q) {
                    int d = us[p] - us[q];
                    if (d > bw) bw = d;
                }
        }
    I->bw = bw;
    const int B1 = bw + 1;
    double* A = (double*)calloc((size_t)I->N * B1, sizeof(double));
#define ADD(u, v, val)                                            \
    do {                                                          \
        if ((u) >= (v)) A[(size_t)(u) * B1 + ((u) - (v))] += (val); \
    } while (0)
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj) {
            double gmin, gmax, Ex[4][4], Eq[4][4];
            cell_g(I, c, ci, cj, &gmin, &gmax);
            exact_q1(I, ci, Ex);
            int nodes[4];
            for (int p = 0; p < 4; ++p) nodes[p] = (ci + CR[p]) * W + cj + CZ[p];
            /* weighted basis part */
            if (gmax > 0.0) {
                double (*E)[4] = Ex;
                if (gmin < I->gam) {
                    weighted_q1(I, c, ci, cj, Eq);
                    E = Eq;
                }
                for (int p = 0; p < 4; ++p) {
                    int up[4];
                    double fp[4];
                    int mp = factors(I, nodes[p], up, fp);
                    for (int q = 0; q < 4; ++q) {
                        int uq[4];
                        double fq[4];
                        int mq = factors(I, nodes[q], uq, fq);
                        for (int s = 0; s < mp; ++s)
                            for (int t = 0; t < mq; ++t) ADD(up[s], uq[t], fp[s] * fq[t] * E[p][q]);
                    }
                }
            }
            /* the plain grid rows of outer and exterior nodes among themselves */
            for (int p = 0; p < 4; ++p) {
                int np = nodes[p];
                if (I->uidx[np] < 0 || I->cls[np] < 2) continue;
                for (int q = 0; q < 4; ++q) {
                    int nq = nodes[q];
                    if (I->uidx[nq] < 0 || I->cls[nq] < 2) continue;
                    ADD(I->uidx[np], I->uidx[nq], Ex[p][q]);
                }
            }
        }
#undef ADD
    /* banded Cholesky in place */
    for (int u = 0; u < I->N; ++u) {
        int v0 = u - bw < 0 ? 0 : u - bw;
        for (int v = v0; v <= u; ++v) {
            double s = A[(size_t)u * B1 + (u - v)];
            int k0 = v0 > v - bw ? v0 : v - bw;
            for (int k = k0; k < v; ++k) s -= A[(size_t)u * B1 + (u - k)] * A[(size_t)v * B1 + (v - k)];
            if (v == u) {
                if (!(s > 0.0)) {
                    free(A);
                    orc_ins_destroy(I);
                    return NULL;
                }
                A[(size_t)u * B1] = sqrt(s);
            } else {
                A[(size_t)u * B1 + (u - v)] = s / A[(size_t)v * B1];
            }
        }
    }
    I->Lb = A;
    return I;
}

static void chol_solve(const orc_ins* I, double* x) {
    const int B1 = I->bw + 1;
    for (int u = 0; u < I->N; ++u) {
        double s = x[u];
        int k0 = u - I->bw < 0 ? 0 : u - I->bw;
        for (int k = k0; k < u; ++k) s -= I->Lb[(size_t)u * B1 + (u - k)] * x[k];
        x[u] = s / I->Lb[(size_t)u * B1];
    }
    for (int u = I->N - 1; u >= 0; --u) {
        double s = x[u];
        int k1 = u + I->bw > I->N - 1 ? I->N - 1 : u + I->bw;
        for (int k = u + 1; k <= k1; ++k) s -= I->Lb[(size_t)k * B1 + (k - u)] * x[k];
        x[u] = s / I->Lb[(size_t)u * B1];
    }
}

/* coefficients x (per unknown) -> potential at every node */
static void nodal(const orc_ins* I, const orc_cfg* c, const double* x, double* phi) {
    const int W = I->W;
    for (int i = 0; i <= c->nr; ++i)
        for (int j = 0; j <= c->nz; ++j) {
            int n = i * W + j;
            double r = c->a + (double)i * I->dr, z = (double)j * I->dz, v = 0.0;
            if (I->cls[n] == 1) {
                v = orc_ins_wp(c, r, z) * x[I->uidx[n]];
            } else if (I->cls[n] == 2 && orc_ins_g(c, r, z) > 0.0) {
                int u[4];
                double f[4], s = 0.0;
                int m = factors(I, n, u, f);
                for (int q = 0; q < m; ++q) s += f[q] * x[u[q]];
                v = orc_ins_wp(c, r, z) * s;
            }
            phi[n] = v;
        }
}

/* Solve with a right-hand side given per hat (raw node loads, b_k for every
 * node; only inner and outer hats count) and return the nodal potential. */
void orc_ins_solve_loads(const orc_ins* I, const orc_cfg* c, const double* load, double* phi) {
    double* x = (double*)calloc(I->N, sizeof(double));
    const int NN = (c->nr + 1) * I->W;
    for (int n = 0; n < NN; ++n) {
        int u[4];
        double f[4];
        int m = factors(I, n, u, f);
        for (int q = 0; q < m; ++q) x[u[q]] += f[q] * load[n];
    }
    chol_solve(I, x);
    nodal(I, c, x, phi);
    free(x);
}

/* Solve with right-hand side values given directly per unknown node (only
 * inner nodes keep theirs) and return the nodal potential. */
void orc_ins_solve_rows(const orc_ins* I, const orc_cfg* c, const double* rhs, double* phi) {
    double* x = (double*)calloc(I->N, sizeof(double));
    const int NN = (c->nr + 1) * I->W;
    for (int n = 0; n < NN; ++n)
        if (I->cls[n] == 1) x[I->uidx[n]] = rhs[n];
    chol_solve(I, x);
    nodal(I, c, x, phi);
    free(x);
}

/* Space-charge potential of the node charges Q (plain deposit) and Qw (the
 * deposit of q (w - 1)): loads bscale (Q + Qw). */
void orc_ins_poisson_charge(const orc_ins* I, const orc_cfg* c, const int64_t* Q, const int64_t* Qw,
                            double* phi_sc) {
    orc_derived d;
    orc_derive(c, &d);
    const int NN = (c->nr + 1) * I->W;
    double* load = (double*)malloc(sizeof(double) * NN);
    for (int n = 0; n < NN; ++n) load[n] = (double)(Q[n] + (Qw ? Qw[n] : 0)) * d.bscale;
    orc_ins_solve_loads(I, c, load, phi_sc);
    free(load);
}

/* Manufactured-solution hook: hat loads int r f w b_k dr dz over the domain
 * (3x3 Gauss per cell where w = 1, the band rule elsewhere), solved. */
typedef struct {
    const orc_cfg* c;
    double (*f)(double, double, void*);
    void* user;
    double rl, zl, dr, dz;
    double F[4];
} fn_ctx;

static void fn_visit(double r, double z, double wq, void* vctx) {
    fn_ctx* X = (fn_ctx*)vctx;
    double w = orc_ins_wp(X->c, r, z);
    double fr = (r - X->rl) / X->dr, fz = (z - X->zl) / X->dz;
    double N[4] = {(1.0 - fr) * (1.0 - fz), fr * (1.0 - fz), (1.0 - fr) * fz, fr * fz};
    double val = X->f(r, z, X->user) * r * w * wq;
    for (int p = 0; p < 4; ++p) X->F[p] += val * N[p];
}

int orc_ins_poisson_fn(const orc_cfg* c, double (*f)(double, double, void*), void* user, double* phi) {
    orc_ins* I = orc_ins_create(c);
    if (!I) return -1;
    const int W = I->W, NN = (c->nr + 1) * W;
    double* load = (double*)calloc(NN, sizeof(double));
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj) {
            double gmin, gmax;
            cell_g(I, c, ci, cj, &gmin, &gmax);
            if (gmax <= 0.0) continue;
            fn_ctx X;
            memset(&X, 0, sizeof(X));
            X.c = c; X.f = f; X.user = user;
            X.rl = c->a + (double)ci * I->dr; X.zl = (double)cj * I->dz;
            X.dr = I->dr; X.dz = I->dz;
            if (gmin < I->gam) {
                quad_cell(I, c, ci, cj, fn_visit, &X);
            } else {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        fn_visit(X.rl + 0.5 * I->dr * (1.0 + GX[a]), X.zl + 0.5 * I->dz * (1.0 + GX[b]),
                                 (0.25 * I->dr * I->dz) * GW[a] * GW[b], &X);
            }
            for (int p = 0; p < 4; ++p) load[(ci + CR[p]) * W + cj + CZ[p]] += X.F[p];
        }
    orc_ins_solve_loads(I, c, load, phi);
    free(load);
    orc_ins_destroy(I);
    return 0;
}

int orc_ins_info(const orc_cfg* c, int* n_unknowns, int* bandwidth, int counts[4]) {
    orc_ins* I = orc_ins_create(c);
    if (!I) return -1;
    if (n_unknowns) *n_unknowns = I->N;
    if (bandwidth) *bandwidth = I->bw;
    if (counts) {
        counts[0] = counts[1] = counts[2] = counts[3] = 0;
        for (int n = 0; n < (c->nr + 1) * I->W; ++n) counts[I->cls[n]] += 1;
    }
    orc_ins_destroy(I);
    return 0;
}
