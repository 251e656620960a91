/*
 * orc_spline3.c -- oracle: cubic B-spline particle shapes and space-charge
 * Poisson solve (the paper's spline FEM of higher order, Sec. II.A).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The space-charge potential is phi_sc = sum_ij c_ij B(s - i) B(t - j) with
 * s = (r - a)/dr, t = z/dz and B the centred cubic B-spline (support
 * |x| < 2).  Homogeneous Dirichlet conditions on r = a, r = b, z = 0, z = L
 * are built into the coefficients by odd reflection: c at i = 0 and i = nr is
 * 0, c at i = -1 is -c at i = 1, c at i = nr+1 is -c at i = nr-1 (the same
 * in z), so every basis function of an unknown vanishes on the walls.  The
 * unknowns are c_ij, 1 <= i <= nr-1, 1 <= j <= nz-1.
 * Galerkin system: sum_(i'j') c_i'j' int r grad psi_ij . grad psi_i'j' dr dz
 * = sum_p q_p psi_ij(x_p) / (2 pi eps0) (the measure's 2 pi r cancels the
 * ring's), psi the reflected basis.  The matrix is assembled cell by cell
 * with the 4x4 Gauss-Legendre rule (exact: the integrand is a polynomial of
 * degree <= 7 in each direction) and solved by a banded Cholesky
 * factorisation.  A particle's load is its charge times the 16 products of
 * its cubic weights: the fixed-point rule of the bilinear deposit (15 nodes
 * rint(W w), the last the remainder) on a grid with one ghost layer, folded
 * onto the unknowns with the reflection signs.
 * The external (vacuum) field stays the order-1 nodal field of orc_field.c;
 * the space-charge field at a particle is -grad phi_sc from the cubic
 * derivatives.
 * Open ends (end_mode 2, Sec. II.A: d phi / dz = 0 at z = 0 and z = L): the
 * coefficients are reflected evenly in z instead (c at j = -1 is c at j = 1,
 * c at j = nz+1 is c at j = nz-1, and c at j = 0 and j = nz are unknowns),
 * so every basis function has zero z-derivative on the ends; the unknowns in
 * z are then 0 <= j <= nz.  The r direction keeps the odd reflection.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_s3 {
    int nr, nz, N, bw;
    int open;          /* even reflection in z (open ends) */
    double a, dr, dz;
    double* Lb;  /* banded Cholesky factor */
};

/* Cubic weights of the four nodes i0-1 .. i0+2 at offset f in [0, 1) from
 * i0, and their derivatives in s. */
void orc_s3_weights(double f, double w[4], double dw[4]) {
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

/* base node and offset of a coordinate (clamped to the mesh) */
static void base_of(double s, int n, int* i0, double* f) {
    int i = (int)floor(s);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    *i0 = i;
    *f = s - (double)i;
}

int orc_s3_ext(const orc_cfg* c) { return (c->nr + 3) * (c->nz + 3); }

/* fixed-point deposit of one particle into the ghosted grid Qx */
void orc_s3_deposit(const orc_cfg* c, double r, double z, int64_t Wq, int64_t* Qx) {
    const double dr = (c->b - c->a) / (double)c->nr, dz = c->L / (double)c->nz;
    int i0, j0;
    double fr, fz, wr[4], dwr[4], wz[4], dwz[4];
    base_of((r - c->a) / dr, c->nr, &i0, &fr);
    base_of(z / dz, c->nz, &j0, &fz);
    orc_s3_weights(fr, wr, dwr);
    orc_s3_weights(fz, wz, dwz);
    const int WX = c->nz + 3;
    const double Wd = (double)Wq;
    int64_t sum = 0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            int64_t q;
            if (a == 3 && b == 3) q = Wq - sum;
            else q = (int64_t)rint(Wd * (wr[a] * wz[b]));
            sum += q;
            /* node (i0-1+a, j0-1+b) at ghosted index (i0+a, j0+b) */
            Qx[(size_t)(i0 + a) * WX + (size_t)(j0 + b)] += q;
        }
}

/* raw index in [-1, n+1] -> unknown index in [0, n] with its sign under the
 * even reflection of open ends (every index maps to an unknown) */
static int fold_even(int i, int n, int* u) {
    *u = i < 0 ? -i : (i > n ? 2 * n - i : i);
    return 1;
}

/* raw index in [-1, n+1] -> unknown index in [1, n-1] with its sign; 0 if the
 * coefficient is fixed at 0 (on the wall) */
static int fold(int i, int n, int* u) {
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

/* z fold of the configuration: odd (Dirichlet ends) or even (open ends) */
static int fold_z(int open, int j, int nz, int* u) { return open ? fold_even(j, nz, u) : fold(j, nz, u); }

/* first unknown index in z and the number of unknowns in z */
static int zfirst(const orc_s3* S) { return S->open ? 0 : 1; }
static int nz_unk(const orc_s3* S) { return S->open ? S->nz + 1 : S->nz - 1; }

static int unk(const orc_s3* S, int i, int j) {
    const int nri = S->nr - 1, nzi = nz_unk(S), jj = j - zfirst(S);
    if (nri <= nzi) return jj * nri + (i - 1);
    return (i - 1) * nzi + jj;
}

static const double G4X[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                              0.86113631159405257522};
static const double G4W[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                              0.34785484513745385737};

void orc_s3_destroy(orc_s3* S) {
    if (!S) return;
    free(S->Lb);
    free(S);
}

orc_s3* orc_s3_create(const orc_cfg* c) {
    if (c->nr < 4 || c->nz < 4) return NULL;
    orc_s3* S = (orc_s3*)calloc(1, sizeof(orc_s3));
    S->nr = c->nr;
    S->nz = c->nz;
    S->open = c->end_mode == 2;
    S->a = c->a;
    S->dr = (c->b - c->a) / (double)c->nr;
    S->dz = c->L / (double)c->nz;
    S->N = (c->nr - 1) * nz_unk(S);
    /* couplings reach 3 nodes in each direction (the fold keeps them there) */
    const int nri = c->nr - 1, nzi = nz_unk(S);
    S->bw = nri <= nzi ? 3 * nri + 3 : 3 * nzi + 3;
    const int B1 = S->bw + 1;
    double* A = (double*)calloc((size_t)S->N * B1, sizeof(double));
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj) {
            /* element matrix over the 16 splines alive on the cell */
            double E[16][16];
            memset(E, 0, sizeof(E));
            for (int qa = 0; qa < 4; ++qa)
                for (int qb = 0; qb < 4; ++qb) {
                    const double fr = 0.5 * (1.0 + G4X[qa]), fz = 0.5 * (1.0 + G4X[qb]);
                    const double r = c->a + ((double)ci + fr) * S->dr;
                    const double wq = (0.25 * S->dr * S->dz) * G4W[qa] * G4W[qb] * r;
                    double wr[4], dwr[4], wz[4], dwz[4];
                    orc_s3_weights(fr, wr, dwr);
                    orc_s3_weights(fz, wz, dwz);
                    double gr[16], gz[16];
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b) {
                            gr[a * 4 + b] = (dwr[a] / S->dr) * wz[b];
                            gz[a * 4 + b] = wr[a] * (dwz[b] / S->dz);
                        }
                    for (int p = 0; p < 16; ++p)
                        for (int q = 0; q < 16; ++q) E[p][q] += wq * (gr[p] * gr[q] + gz[p] * gz[q]);
                }
            /* splines (ci-1+a, cj-1+b) folded onto the unknowns */
            int up[16], sp[16];
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    int ui = 0, uj = 0;
                    const int si = fold(ci - 1 + a, c->nr, &ui), sj = fold_z(S->open, cj - 1 + b, c->nz, &uj);
                    sp[a * 4 + b] = si * sj;
                    up[a * 4 + b] = (si && sj) ? unk(S, ui, uj) : -1;
                }
            for (int p = 0; p < 16; ++p) {
                if (up[p] < 0) continue;
                for (int q = 0; q < 16; ++q) {
                    if (up[q] < 0 || up[q] > up[p]) continue;
                    A[(size_t)up[p] * B1 + (up[p] - up[q])] += (double)(sp[p] * sp[q]) * E[p][q];
                }
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
                    free(S);
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

/* Solve for the coefficients of the load bscale (folded Qx); returns them in
 * the ghosted array cx (reflections filled) and the nodal space-charge
 * potential (sum of the 3x3 neighbouring coefficients with B(0) = 4/6,
 * B(+-1) = 1/6). */
void orc_s3_solve(const orc_s3* S, const orc_cfg* c, const int64_t* Qx, double* cx, double* phi_sc) {
    orc_derived d;
    orc_derive(c, &d);
    const int WX = c->nz + 3, W = c->nz + 1, B1 = S->bw + 1;
    double* x = (double*)calloc(S->N, sizeof(double));
    for (int i = -1; i <= c->nr + 1; ++i)
        for (int j = -1; j <= c->nz + 1; ++j) {
            int ui = 0, uj = 0;
            const int si = fold(i, c->nr, &ui), sj = fold_z(S->open, j, c->nz, &uj);
            if (!si || !sj) continue;
            x[unk(S, ui, uj)] += (double)(si * sj) * (double)Qx[(size_t)(i + 1) * WX + (size_t)(j + 1)];
        }
    for (int u = 0; u < S->N; ++u) x[u] *= d.bscale;
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
    for (int i = -1; i <= c->nr + 1; ++i)
        for (int j = -1; j <= c->nz + 1; ++j) {
            int ui = 0, uj = 0;
            const int si = fold(i, c->nr, &ui), sj = fold_z(S->open, j, c->nz, &uj);
            cx[(size_t)(i + 1) * WX + (size_t)(j + 1)] = (si && sj) ? (double)(si * sj) * x[unk(S, ui, uj)] : 0.0;
        }
    const double nb[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    for (int i = 0; i <= c->nr; ++i)
        for (int j = 0; j <= c->nz; ++j) {
            double v = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) v += (nb[a] * nb[b]) * cx[(size_t)(i + a) * WX + (size_t)(j + b)];
            phi_sc[(size_t)i * W + j] = v;
        }
    free(x);
}

/* space-charge field -grad phi_sc at (r, z) from the ghosted coefficients */
void orc_s3_field(const orc_cfg* c, const double* cx, double r, double z, double* Er, double* Ez) {
    const double dr = (c->b - c->a) / (double)c->nr, dz = c->L / (double)c->nz;
    int i0, j0;
    double fr, fz, wr[4], dwr[4], wz[4], dwz[4];
    base_of((r - c->a) / dr, c->nr, &i0, &fr);
    base_of(z / dz, c->nz, &j0, &fz);
    orc_s3_weights(fr, wr, dwr);
    orc_s3_weights(fz, wz, dwz);
    const int WX = c->nz + 3;
    double gr = 0.0, gz = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const double v = cx[(size_t)(i0 + a) * WX + (size_t)(j0 + b)];
            gr += v * (dwr[a] * wz[b]);
            gz += v * (wr[a] * dwz[b]);
        }
    *Er = -(gr / dr);
    *Ez = -(gz / dz);
}

/* space-charge potential at (r, z) (for pins) */
double orc_s3_phi_at(const orc_cfg* c, const double* cx, double r, double z) {
    const double dr = (c->b - c->a) / (double)c->nr, dz = c->L / (double)c->nz;
    int i0, j0;
    double fr, fz, wr[4], dwr[4], wz[4], dwz[4];
    base_of((r - c->a) / dr, c->nr, &i0, &fr);
    base_of(z / dz, c->nz, &j0, &fz);
    orc_s3_weights(fr, wr, dwr);
    orc_s3_weights(fz, wz, dwz);
    const int WX = c->nz + 3;
    double v = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) v += cx[(size_t)(i0 + a) * WX + (size_t)(j0 + b)] * (wr[a] * wz[b]);
    return v;
}

/* Manufactured-solution hook: loads int r f psi_ij over every cell (4x4 Gauss
 * per cell), solved; returns the ghosted coefficients. */
int orc_s3_poisson_fn(const orc_cfg* c, double (*f)(double, double, void*), void* user, double* cx) {
    orc_s3* S = orc_s3_create(c);
    if (!S) return -1;
    const int WX = c->nz + 3;
    double* load = (double*)calloc((size_t)orc_s3_ext(c), sizeof(double));
    const double dr = S->dr, dz = S->dz;
    for (int ci = 0; ci < c->nr; ++ci)
        for (int cj = 0; cj < c->nz; ++cj)
            for (int qa = 0; qa < 4; ++qa)
                for (int qb = 0; qb < 4; ++qb) {
                    const double fr = 0.5 * (1.0 + G4X[qa]), fz = 0.5 * (1.0 + G4X[qb]);
                    const double r = c->a + ((double)ci + fr) * dr, z = ((double)cj + fz) * dz;
                    const double wq = (0.25 * dr * dz) * G4W[qa] * G4W[qb] * r * f(r, z, user);
                    double wr[4], dwr[4], wz[4], dwz[4];
                    orc_s3_weights(fr, wr, dwr);
                    orc_s3_weights(fz, wz, dwz);
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b) load[(size_t)(ci + a) * WX + (size_t)(cj + b)] += wq * wr[a] * wz[b];
                }
    /* fold and solve as in orc_s3_solve, without the charge scaling */
    const int B1 = S->bw + 1;
    double* x = (double*)calloc(S->N, sizeof(double));
    for (int i = -1; i <= c->nr + 1; ++i)
        for (int j = -1; j <= c->nz + 1; ++j) {
            int ui = 0, uj = 0;
            const int si = fold(i, c->nr, &ui), sj = fold_z(S->open, j, c->nz, &uj);
            if (!si || !sj) continue;
            x[unk(S, ui, uj)] += (double)(si * sj) * load[(size_t)(i + 1) * WX + (size_t)(j + 1)];
        }
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
    for (int i = -1; i <= c->nr + 1; ++i)
        for (int j = -1; j <= c->nz + 1; ++j) {
            int ui = 0, uj = 0;
            const int si = fold(i, c->nr, &ui), sj = fold_z(S->open, j, c->nz, &uj);
            cx[(size_t)(i + 1) * WX + (size_t)(j + 1)] = (si && sj) ? (double)(si * sj) * x[unk(S, ui, uj)] : 0.0;
        }
    free(x);
    free(load);
    orc_s3_destroy(S);
    return 0;
}
