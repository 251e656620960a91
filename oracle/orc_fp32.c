/*
 * orc_fp32.c -- oracle: the charge deposit (Sec. II.A: order-1 spline
 * weights of the particle's position, the particle's charge shared over the
 * four nodes of its cell) evaluated in single precision.  TEST
 * INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The batched FP32 form of the library keeps positions and weights in FP32
 * and rounds the node charges from FP32 products.  Where floating point
 * decides an integer (here the fixed-point node charges), both sides must
 * take that decision in the same precision, so this is the definition of
 * orc_deposit_one written out in float: cell index and offsets from the
 * FP32 position and the FP32 constants (a, 1/dr, 1/dz rounded once from
 * their FP64 values), W = rint(w 2^S) of the FP32 weight, three nodes
 * rint(W w_k) of the FP32 products, the fourth node the remainder.
 * Contraction is off (the build passes -ffp-contract=off), so every product
 * and difference rounds to float as written.
 */
#include "oracle.h"

#include <math.h>
#include <string.h>

void orc_deposit_f32(const orc_cfg* c, int64_t n, const double* r, const double* z, const double* w,
                     int64_t* Q) {
    orc_derived d;
    orc_derive(c, &d);
    const int W = c->nz + 1;
    const float a = (float)c->a;
    const float inv_dr = (float)d.inv_dr, inv_dz = (float)d.inv_dz;
    const float two_S = (float)d.two_S;
    memset(Q, 0, sizeof(int64_t) * (size_t)(c->nr + 1) * (size_t)W);
    for (int64_t p = 0; p < n; ++p) {
        const float rf = (float)r[p], zf = (float)z[p], wf = (float)w[p];
        const float s = (rf - a) * inv_dr;
        const float t = zf * inv_dz;
        int i = (int)floorf(s), j = (int)floorf(t);
        if (i < 0) i = 0;
        if (i > c->nr - 1) i = c->nr - 1;
        if (j < 0) j = 0;
        if (j > c->nz - 1) j = c->nz - 1;
        const float fr = s - (float)i, fz = t - (float)j;
        const float gr = 1.0f - fr, gz = 1.0f - fz;
        const float Wf = rintf(wf * two_S);
        const int64_t Wq = (int64_t)Wf;
        const int64_t q00 = (int64_t)rintf(Wf * (gr * gz));
        const int64_t q10 = (int64_t)rintf(Wf * (fr * gz));
        const int64_t q01 = (int64_t)rintf(Wf * (gr * fz));
        const int64_t q11 = Wq - q00 - q10 - q01;
        const size_t n00 = (size_t)i * (size_t)W + (size_t)j;
        Q[n00] += q00;
        Q[n00 + W] += q10;
        Q[n00 + 1] += q01;
        Q[n00 + W + 1] += q11;
    }
}
