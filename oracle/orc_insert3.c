/*
 * orc_insert3.c -- oracle: the elliptic insert with cubic shapes, i.e.
 * weighted extended B-splines (web-splines) of degree 3 for the space-charge
 * potential.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Space (Sec. II.A, web-splines of any order; Sec. III, the gun's insert):
 *     phi_sc = sum_i c_i B_i,   B_i = w (psi_i + sum_{k outer} e_ki psi_k)
 * over the inner i, with psi_u the cubic B-spline of the rectangle's unknown
 * u reflected at the walls as in orc_spline3.c (odd at r = a, b; odd at
 * z = 0, L, or even there with open ends), and w the insert's weight function
 * of orc_insert.c (0 in the metal, 1 - (1 - g/gam)^3 in the band, 1 beyond).
 * Roles: an unknown is inner if a cell of its support (the 4 x 4 cells around
 * its node, clipped to the rectangle) lies wholly outside the metal, outer if
 * its support holds no such cell but meets the domain, exterior otherwise.
 * Extension: an outer unknown k is attached to the 4 x 4 block of inner
 * unknowns whose centre is nearest to it (ties to the lower indices in r,
 * then z) with the cubic Lagrange weights of the block's index offsets,
 * e = L_alpha(k_r - l_r) L_beta(k_z - l_z), L the cubic Lagrange basis on the
 * nodes 0, 1, 2, 3.
 * Galerkin matrix A_ij = int r grad B_i . grad B_j dr dz over the domain,
 * assembled per rectangle cell from the 16 B-splines alive on it, carried to
 * the inner unknowns through the reflection signs and the extension: cells
 * with w = 1 throughout take the 4 x 4 Gauss rule over the cell; the others
 * that rule on 2 x 2 boxes, boxes cut by the insert split into four down to
 * QDEPTH3 levels (points in the metal dropped at the finest).  Banded Cholesky.
 * Load of a macro-particle of charge q: q B_i(x_p), i.e. the cubic deposit
 * (Qx) plus the cubic deposit of q (w(x_p) - 1) for particles in the band
 * (Qxw), carried through the reflection and the extension.  The space-charge
 * field at a particle is -grad(w u), u = sum_k c~_k b_k with c~ the
 * coefficients expanded onto every ghosted B-spline.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QDEPTH3 6
#define REACH3 8

struct orc_is3 {
    int nr, nz, open, j0, j1, nzu, nu;
    double a, dr, dz, gam;
    int* role;       /* per rectangle unknown: 1 inner, 2 outer, 3 exterior */
    int* id;         /* per rectangle unknown: inner index or -1 */
    int* blk;        /* per outer unknown: rectangle index of its block's first unknown */
    double* ext;     /* per outer unknown: 16 weights, (alpha, beta) alpha-major */
    int N, bw;
    double* Lb;      /* Cholesky factor, row u holds L[u][u-d] at Lb[u*(bw+1)+d] */
};

static const double G4X3[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                               0.86113631159405257522};
static const double G4W3[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                               0.34785484513745385737};

/* rectangle unknown index of (i, j), r-major; -1 outside the unknowns */
static int ridx(const orc_is3* S, int i, int j) {
    if (i < 1 || i > S->nr - 1 || j < S->j0 || j > S->j1) return -1;
    return (i - 1) * S->nzu + (j - S->j0);
}

/* ghosted index -> rectangle unknown and reflection sign (0: a fixed zero) */
static int fold_r3(int i, int n, int* u) {
    if (i >= 1 && i <= n - 1) {
        *u = i;
        return 1;
    }
    if (i == -1) {
        *u = 1;
        return -1;
    }
    if (i == n + 1) {
        *u = n - 1;
        return -1;
    }
    return 0;
}

static int fold_z3(const orc_is3* S, int j, int* u) {
    if (S->open) {
        *u = j < 0 ? -j : (j > S->nz ? 2 * S->nz - j : j);
        return 1;
    }
    return fold_r3(j, S->nz, u);
}

/* range of g over a box (a sum of convex parabolas in r and in z) */
static void g_range(const orc_cfg* c, double rl, double rh, double zl, double zh, double* lo, double* hi) {
    double rc = c->ins_r0 < rl ? rl : (c->ins_r0 > rh ? rh : c->ins_r0);
    double zc = c->ins_z0 < zl ? zl : (c->ins_z0 > zh ? zh : c->ins_z0);
    double rf = fabs(rl - c->ins_r0) > fabs(rh - c->ins_r0) ? rl : rh;
    double zf = fabs(zl - c->ins_z0) > fabs(zh - c->ins_z0) ? zl : zh;
    *lo = orc_ins_g(c, rc, zc);
    *hi = orc_ins_g(c, rf, zf);
}

static void cell_range(const orc_is3* S, const orc_cfg* c, int ci, int cj, double* lo, double* hi) {
    double rl = S->a + (double)ci * S->dr, zl = (double)cj * S->dz;
    g_range(c, rl, rl + S->dr, zl, zl + S->dz, lo, hi);
}

/* cubic Lagrange basis on the nodes 0..3 at x */
static double lag3(int m, double x) {
    switch (m) {
        case 0: return -((x - 1.0) * (x - 2.0) * (x - 3.0)) / 6.0;
        case 1: return (x * (x - 2.0) * (x - 3.0)) / 2.0;
        case 2: return -(x * (x - 1.0) * (x - 3.0)) / 2.0;
        default: return (x * (x - 1.0) * (x - 2.0)) / 6.0;
    }
}

/* the inner unknowns (with factors) that the ghosted B-spline (gi, gj) feeds */
static int feeds3(const orc_is3* S, int gi, int gj, int* id, double* f) {
    int ui, uj;
    const int si = fold_r3(gi, S->nr, &ui), sj = fold_z3(S, gj, &uj);
    if (!si || !sj) return 0;
    const int u = ridx(S, ui, uj);
    const double s = (double)(si * sj);
    if (S->role[u] == 1) {
        id[0] = S->id[u];
        f[0] = s;
        return 1;
    }
    if (S->role[u] != 2) return 0;
    int n = 0;
    const int b = S->blk[u];
    for (int al = 0; al < 4; ++al)
        for (int be = 0; be < 4; ++be) {
            id[n] = S->id[b + al * S->nzu + be];
            f[n] = s * S->ext[(size_t)u * 16 + al * 4 + be];
            ++n;
        }
    return n;
}

/* inner index ordering: the shorter direction runs fastest */
static int order_key(const orc_is3* S, int u) {
    const int i = u / S->nzu + 1, j = u % S->nzu + S->j0;
    const int nri = S->nr - 1;
    if (nri <= S->nzu) return (j - S->j0) * nri + (i - 1);
    return (i - 1) * S->nzu + (j - S->j0);
}

/* ---- element matrices ---- */
typedef struct {
    const orc_cfg* c;
    const orc_is3* S;
    double r0, z0;  /* cell origin */
    double E[16][16];
} el3;

static void add_point3(el3* A, double r, double z, double wq, int weighted) {
    const orc_is3* S = A->S;
    double w = 1.0, wr = 0.0, wz = 0.0;
    if (weighted) w = orc_ins_weight(A->c, r, z, &wr, &wz);
    double fr = (r - A->r0) / S->dr, fz = (z - A->z0) / S->dz;
    double br[4], dbr[4], bz[4], dbz[4];
    orc_s3_weights(fr, br, dbr);
    orc_s3_weights(fz, bz, dbz);
    double gr[16], gz[16];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const double v = br[a] * bz[b];
            const double vr = (dbr[a] / S->dr) * bz[b], vz = br[a] * (dbz[b] / S->dz);
            gr[a * 4 + b] = wr * v + w * vr;
            gz[a * 4 + b] = wz * v + w * vz;
        }
    const double q = r * wq;
    for (int p = 0; p < 16; ++p)
        for (int k = 0; k < 16; ++k) A->E[p][k] += q * (gr[p] * gr[k] + gz[p] * gz[k]);
}

static void gauss_box3(el3* A, double rl, double rh, double zl, double zh, int drop_metal) {
    const double hr = rh - rl, hz = zh - zl;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const double r = rl + 0.5 * hr * (1.0 + G4X3[a]), z = zl + 0.5 * hz * (1.0 + G4X3[b]);
            if (drop_metal && !(orc_ins_g(A->c, r, z) > 0.0)) continue;
            add_point3(A, r, z, (0.25 * hr * hz) * G4W3[a] * G4W3[b], 1);
        }
}

static void weighted_box3(el3* A, double rl, double rh, double zl, double zh, int depth) {
    double lo, hi;
    g_range(A->c, rl, rh, zl, zh, &lo, &hi);
    if (!(hi > 0.0)) return;
    if (!(lo > 0.0) && depth < QDEPTH3) {
        const double rm = 0.5 * (rl + rh), zm = 0.5 * (zl + zh);
        weighted_box3(A, rl, rm, zl, zm, depth + 1);
        weighted_box3(A, rm, rh, zl, zm, depth + 1);
        weighted_box3(A, rl, rm, zm, zh, depth + 1);
        weighted_box3(A, rm, rh, zm, zh, depth + 1);
        return;
    }
    gauss_box3(A, rl, rh, zl, zh, 1);
}

static void element3(const orc_is3* S, const orc_cfg* c, int ci, int cj, el3* A) {
    A->c = c;
    A->S = S;
    A->r0 = S->a + (double)ci * S->dr;
    A->z0 = (double)cj * S->dz;
    memset(A->E, 0, sizeof(A->E));
    double lo, hi;
    cell_range(S, c, ci, cj, &lo, &hi);
    if (lo >= S->gam) {
        /* w = 1 on the whole cell: the plain rule */
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const double r = A->r0 + 0.5 * S->dr * (1.0 + G4X3[a]);
                const double z = A->z0 + 0.5 * S->dz * (1.0 + G4X3[b]);
                add_point3(A, r, z, (0.25 * S->dr * S->dz) * G4W3[a] * G4W3[b], 0);
            }
        return;
    }
    const double hr = 0.5 * S->dr, hz = 0.5 * S->dz;
    for (int sr = 0; sr < 2; ++sr)
        for (int sz = 0; sz < 2; ++sz)
            weighted_box3(A, A->r0 + hr * sr, A->r0 + hr * (sr + 1), A->z0 + hz * sz, A->z0 + hz * (sz + 1), 0);
}

/* ---- set-up ---- */
void orc_is3_destroy(orc_is3* S) {
    if (!S) return;
    free(S->role);
    free(S->id);
    free(S->blk);
    free(S->ext);
    free(S->Lb);
    free(S);
}

orc_is3* orc_is3_create(const orc_cfg* c) {
    if (!orc_has_insert(c) || orc_ins_check(c) != 0 || c->nr < 8 || c->nz < 8) return NULL;
    orc_is3* S = (orc_is3*)calloc(1, sizeof(orc_is3));
    S->nr = c->nr;
    S->nz = c->nz;
    S->open = c->end_mode == 2;
    S->j0 = S->open ? 0 : 1;
    S->j1 = S->open ? c->nz : c->nz - 1;
    S->nzu = S->j1 - S->j0 + 1;
    S->nu = (c->nr - 1) * S->nzu;
    S->a = c->a;
    S->dr = (c->b - c->a) / (double)c->nr;
    S->dz = c->L / (double)c->nz;
    S->gam = orc_ins_gamma(c);
    S->role = (int*)calloc((size_t)S->nu, sizeof(int));
    S->id = (int*)malloc(sizeof(int) * (size_t)S->nu);
    S->blk = (int*)malloc(sizeof(int) * (size_t)S->nu);
    S->ext = (double*)calloc((size_t)S->nu * 16, sizeof(double));
    /* roles from the cells of each unknown's support */
    for (int i = 1; i <= c->nr - 1; ++i)
        for (int j = S->j0; j <= S->j1; ++j) {
            int any_free = 0, any_cut = 0;
            for (int ci = i - 2; ci <= i + 1; ++ci)
                for (int cj = j - 2; cj <= j + 1; ++cj) {
                    if (ci < 0 || ci >= c->nr || cj < 0 || cj >= c->nz) continue;
                    double lo, hi;
                    cell_range(S, c, ci, cj, &lo, &hi);
                    if (lo > 0.0) any_free = 1;
                    else if (hi > 0.0) any_cut = 1;
                }
            S->role[ridx(S, i, j)] = any_free ? 1 : (any_cut ? 2 : 3);
        }
    /* inner indices in band order */
    int* keys = (int*)malloc(sizeof(int) * (size_t)S->nu);
    int* pos = (int*)malloc(sizeof(int) * (size_t)S->nu);
    for (int u = 0; u < S->nu; ++u) pos[order_key(S, u)] = u;
    S->N = 0;
    for (int k = 0; k < S->nu; ++k) {
        const int u = pos[k];
        S->id[u] = S->role[u] == 1 ? S->N++ : -1;
    }
    free(keys);
    free(pos);
    /* extension blocks of the outer unknowns */
    for (int i = 1; i <= c->nr - 1; ++i)
        for (int j = S->j0; j <= S->j1; ++j) {
            const int u = ridx(S, i, j);
            S->blk[u] = -1;
            if (S->role[u] != 2) continue;
            double best = -1.0;
            int bi = 0, bj = 0;
            for (int li = i - REACH3; li <= i + REACH3 - 3; ++li)
                for (int lj = j - REACH3; lj <= j + REACH3 - 3; ++lj) {
                    int ok = 1;
                    for (int al = 0; al < 4 && ok; ++al)
                        for (int be = 0; be < 4 && ok; ++be) {
                            const int v = ridx(S, li + al, lj + be);
                            ok = v >= 0 && S->role[v] == 1;
                        }
                    if (!ok) continue;
                    const double du = ((double)li + 1.5 - (double)i) * S->dr;
                    const double dv = ((double)lj + 1.5 - (double)j) * S->dz;
                    const double d2 = du * du + dv * dv;
                    if (best < 0.0 || d2 < best) {
                        best = d2;
                        bi = li;
                        bj = lj;
                    }
                }
            if (best < 0.0) {
                orc_is3_destroy(S);
                return NULL;
            }
            S->blk[u] = ridx(S, bi, bj);
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be)
                    S->ext[(size_t)u * 16 + al * 4 + be] = lag3(al, (double)(i - bi)) * lag3(be, (double)(j - bj));
        }
    /* bandwidth from the couplings of every cell */
    S->bw = 0;
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj) {
            int lo = S->N, hi = -1;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    int id[16];
                    double f[16];
                    const int n = feeds3(S, ci - 1 + a, cj - 1 + b, id, f);
                    for (int t = 0; t < n; ++t) {
                        if (id[t] < lo) lo = id[t];
                        if (id[t] > hi) hi = id[t];
                    }
                }
            if (hi >= lo && hi - lo > S->bw) S->bw = hi - lo;
        }
    const int B1 = S->bw + 1;
    double* A = (double*)calloc((size_t)S->N * B1, sizeof(double));
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj) {
            double lo, hi;
            cell_range(S, c, ci, cj, &lo, &hi);
            if (!(hi > 0.0)) continue;  /* wholly in the metal: w = 0 */
            el3 E;
            element3(S, c, ci, cj, &E);
            int idp[16][16], np[16];
            double fp[16][16];
            for (int p = 0; p < 16; ++p) np[p] = feeds3(S, ci - 1 + p / 4, cj - 1 + p % 4, idp[p], fp[p]);
            for (int p = 0; p < 16; ++p)
                for (int q = 0; q < 16; ++q)
                    for (int s = 0; s < np[p]; ++s)
                        for (int t = 0; t < np[q]; ++t) {
                            const int x = idp[p][s], y = idp[q][t];
                            if (y > x) continue;
                            A[(size_t)x * B1 + (x - y)] += (fp[p][s] * fp[q][t]) * E.E[p][q];
                        }
        }
    for (int u = 0; u < S->N; ++u) {
        const int v0 = u - S->bw < 0 ? 0 : u - S->bw;
        for (int v = v0; v <= u; ++v) {
            double s = A[(size_t)u * B1 + (u - v)];
            const int k0 = v0 > v - S->bw ? v0 : v - S->bw;
            for (int k = k0; k < v; ++k) s -= A[(size_t)u * B1 + (u - k)] * A[(size_t)v * B1 + (v - k)];
            if (v == u) {
                if (!(s > 0.0)) {
                    free(A);
                    orc_is3_destroy(S);
                    return NULL;
                }
                A[(size_t)u * B1] = sqrt(s);
            } else {
                A[(size_t)u * B1 + (u - v)] = s / A[(size_t)v * B1];
            }
        }
    }
    S->Lb = A;
    return S;
}

static void chol3(const orc_is3* S, double* x) {
    const int B1 = S->bw + 1;
    for (int u = 0; u < S->N; ++u) {
        double s = x[u];
        const int k0 = u - S->bw < 0 ? 0 : u - S->bw;
        for (int k = k0; k < u; ++k) s -= S->Lb[(size_t)u * B1 + (u - k)] * x[k];
        x[u] = s / S->Lb[(size_t)u * B1];
    }
    for (int u = S->N - 1; u >= 0; --u) {
        double s = x[u];
        const int k1 = u + S->bw > S->N - 1 ? S->N - 1 : u + S->bw;
        for (int k = u + 1; k <= k1; ++k) s -= S->Lb[(size_t)k * B1 + (k - u)] * x[k];
        x[u] = s / S->Lb[(size_t)u * B1];
    }
}

/* inner coefficients -> ghosted expanded coefficients cx and the nodal
 * space-charge potential w u at the nodes */
static void expand3(const orc_is3* S, const orc_cfg* c, const double* x, double* cx, double* phi_sc) {
    const int WX = c->nz + 3, W = c->nz + 1;
    for (int gi = -1; gi <= c->nr + 1; ++gi)
        for (int gj = -1; gj <= c->nz + 1; ++gj) {
            int id[16];
            double f[16];
            const int n = feeds3(S, gi, gj, id, f);
            double v = 0.0;
            for (int t = 0; t < n; ++t) v += f[t] * x[id[t]];
            cx[(size_t)(gi + 1) * WX + (size_t)(gj + 1)] = v;
        }
    if (!phi_sc) return;
    const double nb[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    for (int i = 0; i <= c->nr; ++i)
        for (int j = 0; j <= c->nz; ++j) {
            double v = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) v += (nb[a] * nb[b]) * cx[(size_t)(i + a) * WX + (size_t)(j + b)];
            const double r = S->a + (double)i * S->dr, z = (double)j * S->dz;
            phi_sc[(size_t)i * W + j] = orc_ins_wp(c, r, z) * v;
        }
}

void orc_is3_solve(const orc_is3* S, const orc_cfg* c, const int64_t* Qx, const int64_t* Qxw, double* cx,
                   double* phi_sc) {
    orc_derived d;
    orc_derive(c, &d);
    const int WX = c->nz + 3;
    double* x = (double*)calloc((size_t)S->N + 1, sizeof(double));
    for (int gi = -1; gi <= c->nr + 1; ++gi)
        for (int gj = -1; gj <= c->nz + 1; ++gj) {
            const size_t g = (size_t)(gi + 1) * WX + (size_t)(gj + 1);
            const double q = (double)(Qx[g] + (Qxw ? Qxw[g] : 0));
            if (q == 0.0) continue;
            int id[16];
            double f[16];
            const int n = feeds3(S, gi, gj, id, f);
            for (int t = 0; t < n; ++t) x[id[t]] += f[t] * q;
        }
    for (int u = 0; u < S->N; ++u) x[u] *= d.bscale;
    chol3(S, x);
    expand3(S, c, x, cx, phi_sc);
    free(x);
}

/* space-charge field -grad(w u) at (r, z) from the ghosted coefficients */
void orc_is3_field(const orc_cfg* c, const double* cx, double r, double z, double* Er, double* Ez) {
    double ur, uz;
    orc_s3_field(c, cx, r, z, &ur, &uz);   /* -grad u */
    const double u = orc_s3_phi_at(c, cx, r, z);
    double wr, wz;
    const double w = orc_ins_weight(c, r, z, &wr, &wz);
    *Er = w * ur - u * wr;
    *Ez = w * uz - u * wz;
}

double orc_is3_phi_at(const orc_cfg* c, const double* cx, double r, double z) {
    return orc_ins_wp(c, r, z) * orc_s3_phi_at(c, cx, r, z);
}

/* Manufactured-solution hook: loads int r f B_i over the domain (the cells'
 * quadrature of the Galerkin matrix), solved; returns the ghosted
 * coefficients. */
int orc_is3_poisson_fn(const orc_cfg* c, double (*f)(double, double, void*), void* user, double* cx) {
    orc_is3* S = orc_is3_create(c);
    if (!S) return -1;
    double* x = (double*)calloc((size_t)S->N + 1, sizeof(double));
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj) {
            double lo, hi;
            cell_range(S, c, ci, cj, &lo, &hi);
            if (!(hi > 0.0)) continue;
            /* quadrature points of the cell: the plain rule, or 4x4 Gauss on
             * the refined boxes of the cut cell, points in the metal dropped */
            const double r0 = S->a + (double)ci * S->dr, z0 = (double)cj * S->dz;
            double bl[16];
            memset(bl, 0, sizeof(bl));
            int stack_n = 0;
            double st[256][4];
            int sd[256];
            if (lo >= S->gam) {
                st[0][0] = r0; st[0][1] = r0 + S->dr; st[0][2] = z0; st[0][3] = z0 + S->dz;
                sd[0] = QDEPTH3;
                stack_n = 1;
            } else {
                for (int sr = 0; sr < 2; ++sr)
                    for (int sz = 0; sz < 2; ++sz) {
                        st[stack_n][0] = r0 + 0.5 * S->dr * sr;
                        st[stack_n][1] = r0 + 0.5 * S->dr * (sr + 1);
                        st[stack_n][2] = z0 + 0.5 * S->dz * sz;
                        st[stack_n][3] = z0 + 0.5 * S->dz * (sz + 1);
                        sd[stack_n] = 0;
                        ++stack_n;
                    }
            }
            while (stack_n > 0) {
                --stack_n;
                const double rl = st[stack_n][0], rh = st[stack_n][1], zl = st[stack_n][2], zh = st[stack_n][3];
                const int dep = sd[stack_n];
                double blo, bhi;
                g_range(c, rl, rh, zl, zh, &blo, &bhi);
                if (!(bhi > 0.0)) continue;
                if (!(blo > 0.0) && dep < QDEPTH3) {
                    const double rm = 0.5 * (rl + rh), zm = 0.5 * (zl + zh);
                    const double bx[4][4] = {{rl, rm, zl, zm}, {rm, rh, zl, zm}, {rl, rm, zm, zh}, {rm, rh, zm, zh}};
                    for (int t = 0; t < 4; ++t) {
                        memcpy(st[stack_n], bx[t], sizeof(bx[t]));
                        sd[stack_n] = dep + 1;
                        ++stack_n;
                    }
                    continue;
                }
                const double hr = rh - rl, hz = zh - zl;
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        const double r = rl + 0.5 * hr * (1.0 + G4X3[a]), z = zl + 0.5 * hz * (1.0 + G4X3[b]);
                        if (!(orc_ins_g(c, r, z) > 0.0)) continue;
                        const double wq = (0.25 * hr * hz) * G4W3[a] * G4W3[b] * r * f(r, z, user) *
                                          orc_ins_wp(c, r, z);
                        double br[4], dbr[4], bz[4], dbz[4];
                        orc_s3_weights((r - r0) / S->dr, br, dbr);
                        orc_s3_weights((z - z0) / S->dz, bz, dbz);
                        for (int p = 0; p < 16; ++p) bl[p] += wq * br[p / 4] * bz[p % 4];
                    }
            }
            for (int p = 0; p < 16; ++p) {
                int id[16];
                double fc[16];
                const int n = feeds3(S, ci - 1 + p / 4, cj - 1 + p % 4, id, fc);
                for (int t = 0; t < n; ++t) x[id[t]] += fc[t] * bl[p];
            }
        }
    chol3(S, x);
    expand3(S, c, x, cx, NULL);
    free(x);
    orc_is3_destroy(S);
    return 0;
}

int orc_is3_info(const orc_cfg* c, int* n_inner, int* bandwidth, int counts[4]) {
    orc_is3* S = orc_is3_create(c);
    if (!S) return -1;
    if (n_inner) *n_inner = S->N;
    if (bandwidth) *bandwidth = S->bw;
    if (counts) {
        counts[0] = counts[1] = counts[2] = counts[3] = 0;
        for (int u = 0; u < S->nu; ++u) counts[S->role[u]] += 1;
    }
    orc_is3_destroy(S);
    return 0;
}
