/*
 * orc_field.c -- oracle: static B on the nodes, order-1 FEM Poisson solve in
 * (r,z) with Dirichlet electrodes, nodal E.  TEST INFRASTRUCTURE ONLY.
 *
 * Weak form of the axisymmetric Poisson equation (Sec. II.A, FEM on a
 * rectangular grid): with dV = 2 pi r dr dz and macro-particles as charged
 * rings, the 2 pi r of the measure cancels the ring's 1/(2 pi r), so
 *     sum_j phi_j  int grad N_j . grad N_i  r dr dz = sum_p q_p N_i(x_p) / (2 pi eps0).
 * With tensor-product hat functions the matrix is Kr (x) Mz + Mr (x) Kz where
 *     Kr = int r N_a' N_b' dr,  Mr = int r N_a N_b dr,  Kz = int N' N' dz,
 *     Mz = int N N dz   (1D element integrals, exact).
 * The interior system (homogeneous Dirichlet on all four sides) is solved by
 * a discrete sine transform in z, which diagonalises Kz and Mz, followed by a
 * tridiagonal solve in r per sine mode.  The sine transform is written as the
 * plain sum with a table; no fast transform.
 *
 * Open ends (end_mode 2, the Neumann condition d(phi)/dz = 0 of Sec. II.A):
 * the end nodes z = 0, L are unknowns and the natural boundary condition
 * halves the end rows of Kz and Mz; with D = diag(1/2, 1, ..., 1, 1/2) both
 * satisfy A v_k = eig_k D v_k for the cosine vectors v_k(j) = cos(pi j k / nz),
 * k = 0..nz (same eigenvalues as the sine modes), and v_m^T D v_k = c_k
 * delta_mk with c_k = nz for k = 0, nz and nz/2 otherwise.  So each mode k
 * solves (mu_k Kr + lam_k Mr) x_k = (sum_j b_j v_k(j)) / c_k and
 * phi_j = sum_k x_k v_k(j).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline double r_node(const orc_cfg* c, double dr, double i) { return c->a + i * dr; }

/* External magnetic field on the nodes.  Bz = B0 (1 + k zeta^2) with
 * zeta = (z - L/2)/(L/2); Br = -(r/2) dBz/dz keeps div B = 0 to first order
 * in r (paraxial form). */
void orc_bfield(const orc_cfg* c, double* Br, double* Bz) {
    double dr = (c->b - c->a) / (double)c->nr;
    double dz = c->L / (double)c->nz;
    double halfL = 0.5 * c->L;
    for (int i = 0; i <= c->nr; ++i) {
        double r = r_node(c, dr, (double)i);
        for (int j = 0; j <= c->nz; ++j) {
            double z = (double)j * dz;
            double zeta = (z - halfL) / halfL;
            int n = i * (c->nz + 1) + j;
            Bz[n] = c->B0 * (1.0 + c->mirror_k * (zeta * zeta));
            Br[n] = -(r * ((c->B0 * c->mirror_k) * zeta)) / halfL;
        }
    }
}

/* 1D matrix entries (full, assembled) between node i and node i+di. */
static double Kr_ent(const orc_cfg* c, double dr, int i, int di) {
    double rm = r_node(c, dr, (double)i - 0.5), rp = r_node(c, dr, (double)i + 0.5);
    if (di == 0) {
        double s = 0.0;
        if (i > 0) s += rm / dr;
        if (i < c->nr) s += rp / dr;
        return s;
    }
    return di < 0 ? -rm / dr : -rp / dr;
}
static double Mr_ent(const orc_cfg* c, double dr, int i, int di) {
    double rim = r_node(c, dr, (double)(i - 1)), ri = r_node(c, dr, (double)i),
           rip = r_node(c, dr, (double)(i + 1));
    if (di == 0) {
        double s = 0.0;
        if (i > 0) s += dr * (rim + 3.0 * ri) / 12.0;
        if (i < c->nr) s += dr * (3.0 * ri + rip) / 12.0;
        return s;
    }
    return di < 0 ? dr * (rim + ri) / 12.0 : dr * (ri + rip) / 12.0;
}
static double Kz_ent(double dz, int di) { return di == 0 ? 2.0 / dz : -1.0 / dz; }
static double Mz_ent(double dz, int di) { return di == 0 ? 4.0 * dz / 6.0 : dz / 6.0; }
/* the same at node j of an open-ended column: one element on the end nodes */
static double Kz_at(const orc_cfg* c, double dz, int j, int dj) {
    if (c->end_mode == 2 && dj == 0 && (j == 0 || j == c->nz)) return 1.0 / dz;
    return Kz_ent(dz, dj);
}
static double Mz_at(const orc_cfg* c, double dz, int j, int dj) {
    if (c->end_mode == 2 && dj == 0 && (j == 0 || j == c->nz)) return 2.0 * dz / 6.0;
    return Mz_ent(dz, dj);
}

/*
 * Solve (Kr (x) Mz + Mr (x) Kz) x = rhs on the interior nodes with x = 0 on
 * the boundary.  rhs and phi are full node arrays; boundary entries of rhs are
 * ignored and boundary entries of phi are set to 0.
 */
static void solve_neumann(const orc_cfg* c, const double* rhs, double* phi);

void orc_solve(const orc_cfg* c, const double* rhs, double* phi) {
    if (c->end_mode == 2) {
        solve_neumann(c, rhs, phi);
        return;
    }
    const int nr = c->nr, nz = c->nz, W = nz + 1;
    const double dr = (c->b - c->a) / (double)nr, dz = c->L / (double)nz;
    const int nri = nr - 1, nzi = nz - 1;
    /* sine table S[j][k] = sin(pi j k / nz), j,k in [0,nz] */
    double* S = (double*)malloc(sizeof(double) * (size_t)W * W);
    for (int j = 0; j <= nz; ++j)
        for (int k = 0; k <= nz; ++k)
            S[(size_t)j * W + k] = sin(M_PI * (double)((j * k) % (2 * nz)) / (double)nz);
    double* bh = (double*)calloc((size_t)(nr + 1) * W, sizeof(double));
    /* forward transform of each interior row: bh[i][k] = sum_j rhs[i][j] S[j][k] */
#pragma omp parallel for schedule(static)
    for (int i = 1; i <= nri; ++i) {
        double* out = bh + (size_t)i * W;
        for (int j = 1; j <= nzi; ++j) {
            double v = rhs[(size_t)i * W + j];
            const double* Sj = S + (size_t)j * W;
            for (int k = 1; k <= nzi; ++k) out[k] += v * Sj[k];
        }
    }
    /* tridiagonal solve in r for each sine mode k */
    double* xh = (double*)calloc((size_t)(nr + 1) * W, sizeof(double));
#pragma omp parallel
    {
        double* cp = (double*)malloc(sizeof(double) * (size_t)(nr + 1));
        double* dp = (double*)malloc(sizeof(double) * (size_t)(nr + 1));
#pragma omp for schedule(static)
        for (int k = 1; k <= nzi; ++k) {
            double ck = cos(M_PI * (double)k / (double)nz);
            double mu = (dz / 3.0) * (2.0 + ck);       /* eigenvalue of Mz */
            double lam = (2.0 / dz) * (1.0 - ck);      /* eigenvalue of Kz */
            for (int i = 1; i <= nri; ++i) {
                double diag = mu * Kr_ent(c, dr, i, 0) + lam * Mr_ent(c, dr, i, 0);
                double up = mu * Kr_ent(c, dr, i, +1) + lam * Mr_ent(c, dr, i, +1);
                double lo = mu * Kr_ent(c, dr, i, -1) + lam * Mr_ent(c, dr, i, -1);
                double b = bh[(size_t)i * W + k];
                if (i == 1) {
                    cp[i] = up / diag;
                    dp[i] = b / diag;
                } else {
                    double m = diag - lo * cp[i - 1];
                    cp[i] = up / m;
                    dp[i] = (b - lo * dp[i - 1]) / m;
                }
            }
            xh[(size_t)nri * W + k] = dp[nri];
            for (int i = nri - 1; i >= 1; --i)
                xh[(size_t)i * W + k] = dp[i] - cp[i] * xh[(size_t)(i + 1) * W + k];
        }
        free(cp); free(dp);
    }
    /* inverse transform: phi[i][j] = (2/nz) sum_k xh[i][k] S[j][k] */
    memset(phi, 0, sizeof(double) * (size_t)(nr + 1) * W);
#pragma omp parallel for schedule(static)
    for (int i = 1; i <= nri; ++i) {
        double* out = phi + (size_t)i * W;
        for (int k = 1; k <= nzi; ++k) {
            double v = xh[(size_t)i * W + k];
            const double* Sk = S + (size_t)k * W;  /* S is symmetric */
            for (int j = 1; j <= nzi; ++j) out[j] += v * Sk[j];
        }
        for (int j = 1; j <= nzi; ++j) out[j] *= 2.0 / (double)nz;
    }
    free(S); free(bh); free(xh);
}

/* The open-ended system: interior rows in r, all nodes j = 0..nz in z,
 * solved by the cosine modes (plain sums with a table). */
static void solve_neumann(const orc_cfg* c, const double* rhs, double* phi) {
    const int nr = c->nr, nz = c->nz, W = nz + 1;
    const double dr = (c->b - c->a) / (double)nr, dz = c->L / (double)nz;
    const int nri = nr - 1;
    double* Ct = (double*)malloc(sizeof(double) * (size_t)W * W);  /* cos(pi j k / nz) */
    for (int j = 0; j <= nz; ++j)
        for (int k = 0; k <= nz; ++k)
            Ct[(size_t)j * W + k] = cos(M_PI * (double)((j * k) % (2 * nz)) / (double)nz);
    double* bh = (double*)calloc((size_t)(nr + 1) * W, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 1; i <= nri; ++i) {
        double* out = bh + (size_t)i * W;
        for (int j = 0; j <= nz; ++j) {
            double v = rhs[(size_t)i * W + j];
            const double* Cj = Ct + (size_t)j * W;
            for (int k = 0; k <= nz; ++k) out[k] += v * Cj[k];
        }
        for (int k = 0; k <= nz; ++k) out[k] /= (k == 0 || k == nz) ? (double)nz : 0.5 * (double)nz;
    }
    double* xh = (double*)calloc((size_t)(nr + 1) * W, sizeof(double));
#pragma omp parallel
    {
        double* cp = (double*)malloc(sizeof(double) * (size_t)(nr + 1));
        double* dp = (double*)malloc(sizeof(double) * (size_t)(nr + 1));
#pragma omp for schedule(static)
        for (int k = 0; k <= nz; ++k) {
            double ck = cos(M_PI * (double)k / (double)nz);
            double mu = (dz / 3.0) * (2.0 + ck);
            double lam = (2.0 / dz) * (1.0 - ck);
            for (int i = 1; i <= nri; ++i) {
                double diag = mu * Kr_ent(c, dr, i, 0) + lam * Mr_ent(c, dr, i, 0);
                double up = mu * Kr_ent(c, dr, i, +1) + lam * Mr_ent(c, dr, i, +1);
                double lo = mu * Kr_ent(c, dr, i, -1) + lam * Mr_ent(c, dr, i, -1);
                double b = bh[(size_t)i * W + k];
                if (i == 1) {
                    cp[i] = up / diag;
                    dp[i] = b / diag;
                } else {
                    double m = diag - lo * cp[i - 1];
                    cp[i] = up / m;
                    dp[i] = (b - lo * dp[i - 1]) / m;
                }
            }
            xh[(size_t)nri * W + k] = dp[nri];
            for (int i = nri - 1; i >= 1; --i)
                xh[(size_t)i * W + k] = dp[i] - cp[i] * xh[(size_t)(i + 1) * W + k];
        }
        free(cp); free(dp);
    }
    memset(phi, 0, sizeof(double) * (size_t)(nr + 1) * W);
#pragma omp parallel for schedule(static)
    for (int i = 1; i <= nri; ++i) {
        double* out = phi + (size_t)i * W;
        for (int k = 0; k <= nz; ++k) {
            double v = xh[(size_t)i * W + k];
            const double* Ck = Ct + (size_t)k * W;
            for (int j = 0; j <= nz; ++j) out[j] += v * Ck[j];
        }
    }
    free(Ct); free(bh); free(xh);
}

/* Dirichlet data on the electrodes.  r=a: V_inner; r=b: V_outer (corners
 * belong to the radial electrodes); ends z=0,L: end_mode 0 gives the coaxial
 * vacuum profile shifted by V_end, end_mode 1 a flat V_end. */
static double boundary_value(const orc_cfg* c, double dr, int i, int j) {
    (void)j;
    if (i == 0) return c->V_inner;
    if (i == c->nr) return c->V_outer;
    double r = r_node(c, dr, (double)i);
    if (c->end_mode == 1) return c->V_end;
    double coax = c->V_inner + (c->V_outer - c->V_inner) * (log(r / c->a) / log(c->b / c->a));
    return coax + c->V_end;
}

static int is_boundary(const orc_cfg* c, int i, int j) {
    if (c->end_mode == 2) return i == 0 || i == c->nr;  /* open ends: z nodes are unknowns */
    return i == 0 || i == c->nr || j == 0 || j == c->nz;
}

/* Vacuum potential: discrete Laplace solution with the electrode data.  With
 * the elliptic insert the data are taken relative to V_outer (the insert's
 * potential), so that the weighted basis, which vanishes on the insert, holds
 * the solution; the lift of the remaining data lives on the hats next to the
 * inner electrode and the ends, away from the insert. */
void orc_vacuum(const orc_cfg* c, double* phi_vac) {
    const int nr = c->nr, nz = c->nz, W = nz + 1;
    const double dr = (c->b - c->a) / (double)nr, dz = c->L / (double)nz;
    size_t N = (size_t)(nr + 1) * W;
    const int ins = orc_has_insert(c);
    const double shift = ins ? c->V_outer : 0.0;
    double* rhs = (double*)calloc(N, sizeof(double));
    double* x = (double*)calloc(N, sizeof(double));
    const int j0 = c->end_mode == 2 ? 0 : 1, j1 = c->end_mode == 2 ? nz : nz - 1;
    for (int i = 1; i < nr; ++i)
        for (int j = j0; j <= j1; ++j) {
            double s = 0.0;
            for (int di = -1; di <= 1; ++di)
                for (int dj = -1; dj <= 1; ++dj) {
                    int ii = i + di, jj = j + dj;
                    if (jj < 0 || jj > nz || !is_boundary(c, ii, jj)) continue;
                    double A = Kr_ent(c, dr, i, di) * Mz_at(c, dz, j, dj) +
                               Mr_ent(c, dr, i, di) * Kz_at(c, dz, j, dj);
                    s -= A * (boundary_value(c, dr, ii, jj) - shift);
                }
            rhs[(size_t)i * W + j] = s;
        }
    if (ins) {
        orc_ins* I = orc_ins_create(c);
        if (I) {
            orc_ins_solve_rows(I, c, rhs, x);
            orc_ins_destroy(I);
        }
    } else {
        orc_solve(c, rhs, x);
    }
    for (int i = 0; i <= nr; ++i)
        for (int j = 0; j <= nz; ++j) {
            size_t n = (size_t)i * W + j;
            phi_vac[n] = is_boundary(c, i, j) ? boundary_value(c, dr, i, j) : x[n] + shift;
        }
    free(rhs); free(x);
}

/* Self-consistent part: rhs_i = -e 2^-S Q_i / (2 pi eps0), homogeneous Dirichlet. */
void orc_poisson_charge(const orc_cfg* c, const int64_t* Q, double* phi_sc) {
    orc_derived d;
    orc_derive(c, &d);
    size_t N = (size_t)(c->nr + 1) * (c->nz + 1);
    double* rhs = (double*)malloc(sizeof(double) * N);
    for (size_t n = 0; n < N; ++n) rhs[n] = (double)Q[n] * d.bscale;
    orc_solve(c, rhs, phi_sc);
    free(rhs);
}

/* E = -grad phi at the nodes: central differences inside, second-order
 * one-sided differences on the boundary rows and columns. */
void orc_efield(const orc_cfg* c, const double* phi, double* Er, double* Ez) {
    const int nr = c->nr, nz = c->nz, W = nz + 1;
    const double dr = (c->b - c->a) / (double)nr, dz = c->L / (double)nz;
    const double hr = 0.5 / dr, hz = 0.5 / dz;
#define P(i, j) phi[(size_t)(i) * W + (j)]
    for (int i = 0; i <= nr; ++i)
        for (int j = 0; j <= nz; ++j) {
            double gr, gz;
            if (i == 0) gr = (-3.0 * P(0, j) + 4.0 * P(1, j) - P(2, j)) * hr;
            else if (i == nr) gr = (3.0 * P(nr, j) - 4.0 * P(nr - 1, j) + P(nr - 2, j)) * hr;
            else gr = (P(i + 1, j) - P(i - 1, j)) * hr;
            if (j == 0) gz = (-3.0 * P(i, 0) + 4.0 * P(i, 1) - P(i, 2)) * hz;
            else if (j == nz) gz = (3.0 * P(i, nz) - 4.0 * P(i, nz - 1) + P(i, nz - 2)) * hz;
            else gz = (P(i, j + 1) - P(i, j - 1)) * hz;
            Er[(size_t)i * W + j] = -gr;
            Ez[(size_t)i * W + j] = -gz;
        }
#undef P
}

/* Lumped node volume V_i = int N_i dV = 2 pi (int r N_a dr)(int N_b dz). */
void orc_node_volume(const orc_cfg* c, double* V) {
    const int nr = c->nr, nz = c->nz, W = nz + 1;
    const double dr = (c->b - c->a) / (double)nr, dz = c->L / (double)nz;
    for (int i = 0; i <= nr; ++i) {
        double lr;
        if (i == 0) lr = dr * (c->a / 2.0 + dr / 6.0);
        else if (i == nr) lr = dr * (c->b / 2.0 - dr / 6.0);
        else lr = r_node(c, dr, (double)i) * dr;
        for (int j = 0; j <= nz; ++j) {
            double lz = (j == 0 || j == nz) ? dz / 2.0 : dz;
            V[(size_t)i * W + j] = 2.0 * M_PI * lr * lz;
        }
    }
}

/*
 * Potential-well depth along magnetic field lines, as the paper defines it
 * after Pagonakis et al. (Sec. II.B): along a field line the electrons'
 * trap is a local maximum of phi (a minimum of their potential energy); its
 * depth is that maximum less the higher of the lowest values on either side.
 * Field lines of Bz = B0 (1 + k zeta^2), Br = -(r/2) dBz/dz conserve r^2 Bz.
 */
void orc_well_depth(const orc_cfg* c, const double* phi, int n_lines, const double* r_mid, double* depth,
                    double* z_max) {
    const int nr = c->nr, nz = c->nz, W = nz + 1;
    const double dr = (c->b - c->a) / (double)nr, dz = c->L / (double)nz, halfL = 0.5 * c->L;
    double* U = (double*)malloc(sizeof(double) * (size_t)W);
    int* in = (int*)malloc(sizeof(int) * (size_t)W);
    for (int l = 0; l < n_lines; ++l) {
        const double Bmid = c->B0;  /* zeta = 0 */
        for (int j = 0; j <= nz; ++j) {
            const double z = (double)j * dz, zeta = (z - halfL) / halfL;
            const double Bz = c->B0 * (1.0 + c->mirror_k * (zeta * zeta));
            const double r = r_mid[l] * sqrt(Bmid / Bz);
            in[j] = r > c->a && r < c->b;
            U[j] = 0.0;
            if (!in[j]) continue;
            double s = (r - c->a) / dr;
            int i = (int)floor(s);
            if (i > nr - 1) i = nr - 1;
            const double fr = s - (double)i;
            int jj = j < nz ? j : nz - 1;
            const double fz = (z - (double)jj * dz) / dz;
            const double* P = phi + (size_t)i * W + jj;
            U[j] = ((1.0 - fr) * (1.0 - fz) * P[0] + fr * (1.0 - fz) * P[W]) + ((1.0 - fr) * fz * P[1] + fr * fz * P[W + 1]);
        }
        const int jm = nz / 2;
        depth[l] = 0.0;
        z_max[l] = -1.0;
        if (!in[jm]) continue;
        int lo = jm, hi = jm;
        while (lo > 0 && in[lo - 1]) --lo;
        while (hi < nz && in[hi + 1]) ++hi;
        int jx = lo;
        for (int j = lo; j <= hi; ++j)
            if (U[j] > U[jx]) jx = j;
        double left = U[jx], right = U[jx];
        for (int j = lo; j <= jx; ++j) left = U[j] < left ? U[j] : left;
        for (int j = jx; j <= hi; ++j) right = U[j] < right ? U[j] : right;
        depth[l] = U[jx] - (left > right ? left : right);
        z_max[l] = (double)jx * dz;
    }
    free(U);
    free(in);
}
