/*
 * or_math.c -- oracle math: exp, SH basis, fp16/bf16 rounding.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * or_vm_exp is the one exp definition the splat decisions use (alpha >= 1/255,
 * transmittance stop).  It is Cody and Waite's argument reduction (1980):
 * n = rint(x log2 e), r = x - n ln2 with ln2 split into a 15-bit head and a
 * tail, then the degree-7 Taylor polynomial of e^r in Horner form with fused
 * multiply-adds, then scaling by 2^n.  The HIP kernels implement the same
 * definition independently.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include "oracle.h"

float or_vm_exp(float x)
{
    if (!(x >= -87.0f)) return 0.0f;          /* e^-87 is still a normal float */
    if (x > 88.0f) return INFINITY;
    const float log2e = (float)(1.0 / log(2.0));
    const float ln2_hi = (float)(22713.0 / 32768.0);      /* ln 2 to 15 bits: n*ln2_hi is exact */
    const float ln2_lo = (float)(log(2.0) - 22713.0 / 32768.0);
    float n = rintf(x * log2e);
    float r = fmaf(-n, ln2_hi, x);
    r = fmaf(-n, ln2_lo, r);
    /* Taylor coefficients 1/k!, k = 7 .. 0 */
    float p = (float)(1.0 / 5040.0);
    p = fmaf(p, r, (float)(1.0 / 720.0));
    p = fmaf(p, r, (float)(1.0 / 120.0));
    p = fmaf(p, r, (float)(1.0 / 24.0));
    p = fmaf(p, r, (float)(1.0 / 6.0));
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)n);
}

/*
 * Real spherical harmonics up to degree 3 on the unit sphere, written as
 * polynomials in (x, y, z) with the normalisation sqrt((2l+1)/(4 pi) *
 * (l-m)!/(l+m)!) (times sqrt 2 for m != 0).  Index k = l*l + l + m.
 * The sign of each function is a fixed convention; the basis is orthonormal.
 */
static double sh_const(int k)
{
    const double pi = 3.14159265358979323846;
    switch (k) {
    case 0: return 0.5 * sqrt(1.0 / pi);
    case 1: return -sqrt(3.0 / (4.0 * pi));
    case 2: return sqrt(3.0 / (4.0 * pi));
    case 3: return -sqrt(3.0 / (4.0 * pi));
    case 4: return 0.5 * sqrt(15.0 / pi);
    case 5: return -0.5 * sqrt(15.0 / pi);
    case 6: return 0.25 * sqrt(5.0 / pi);
    case 7: return -0.5 * sqrt(15.0 / pi);
    case 8: return 0.25 * sqrt(15.0 / pi);
    case 9: return -0.25 * sqrt(35.0 / (2.0 * pi));
    case 10: return 0.5 * sqrt(105.0 / pi);
    case 11: return -0.25 * sqrt(21.0 / (2.0 * pi));
    case 12: return 0.25 * sqrt(7.0 / pi);
    case 13: return -0.25 * sqrt(21.0 / (2.0 * pi));
    case 14: return 0.25 * sqrt(105.0 / pi);
    case 15: return -0.25 * sqrt(35.0 / (2.0 * pi));
    }
    return 0.0;
}

/* polynomial part of basis function k at a unit direction (double) */
static double sh_poly(int k, double x, double y, double z)
{
    double xx = x * x, yy = y * y, zz = z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return y;
    case 2: return z;
    case 3: return x;
    case 4: return x * y;
    case 5: return y * z;
    case 6: return 2.0 * zz - xx - yy;
    case 7: return x * z;
    case 8: return xx - yy;
    case 9: return y * (3.0 * xx - yy);
    case 10: return x * y * z;
    case 11: return y * (4.0 * zz - xx - yy);
    case 12: return z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    case 13: return x * (4.0 * zz - xx - yy);
    case 14: return z * (xx - yy);
    case 15: return x * (xx - 3.0 * yy);
    }
    return 0.0;
}

double or_sh_basis(int k, double x, double y, double z)
{
    return sh_const(k) * sh_poly(k, x, y, z);
}

/*
 * Float evaluation used by the splat (colour is continuous, so its rounding
 * only needs to match within tolerance; it is kept in one fixed order):
 * b_k = (float)const_k * poly_k evaluated in float, acc summed k = 0..15.
 */
void or_sh_color_f32(const float* sh /*[16][3]*/, float x, float y, float z, float out[3])
{
    float xx = x * x, yy = y * y, zz = z * z;
    float xy = x * y, yz = y * z, xz = x * z;
    float b[16];
    b[0] = (float)sh_const(0);
    b[1] = (float)sh_const(1) * y;
    b[2] = (float)sh_const(2) * z;
    b[3] = (float)sh_const(3) * x;
    b[4] = (float)sh_const(4) * xy;
    b[5] = (float)sh_const(5) * yz;
    b[6] = (float)sh_const(6) * ((2.0f * zz - xx) - yy);
    b[7] = (float)sh_const(7) * xz;
    b[8] = (float)sh_const(8) * (xx - yy);
    b[9] = ((float)sh_const(9) * y) * (3.0f * xx - yy);
    b[10] = ((float)sh_const(10) * xy) * z;
    b[11] = ((float)sh_const(11) * y) * ((4.0f * zz - xx) - yy);
    b[12] = ((float)sh_const(12) * z) * ((2.0f * zz - 3.0f * xx) - 3.0f * yy);
    b[13] = ((float)sh_const(13) * x) * ((4.0f * zz - xx) - yy);
    b[14] = ((float)sh_const(14) * z) * (xx - yy);
    b[15] = ((float)sh_const(15) * x) * (xx - 3.0f * yy);
    for (int c = 0; c < 3; c++) {
        float acc = b[0] * sh[c];
        for (int k = 1; k < 16; k++) acc = acc + b[k] * sh[k * 3 + c];
        acc = acc + 0.5f;
        out[c] = acc > 0.0f ? acc : 0.0f;
    }
}

/* nearest fp16 value, ties to even (IEEE binary16: 11-bit significand,
 * exponents -14..15, subnormal spacing 2^-24) */
float or_round_f16(float x)
{
    if (x != x) return x;
    float ax = fabsf(x);
    if (ax >= 65520.0f) return copysignf(INFINITY, x);
    if (ax == 0.0f) return x;
    int e;
    frexpf(ax, &e);                     /* ax in [2^(e-1), 2^e) */
    int ue = e - 11;
    if (ue < -24) ue = -24;
    float ulp = ldexpf(1.0f, ue);
    float q = nearbyintf(ax / ulp);
    return copysignf(q * ulp, x);
}

/* nearest bfloat16 value, ties to even (8-bit significand, float exponents) */
float or_round_bf16(float x)
{
    if (x != x) return x;
    float ax = fabsf(x);
    if (ax == 0.0f) return x;
    if (ax >= 3.3961514e38f) return copysignf(INFINITY, x);  /* halfway to 2^128 */
    int e;
    frexpf(ax, &e);
    int ue = e - 8;
    if (ue < -133) ue = -133;
    double ulp = ldexp(1.0, ue);
    double q = nearbyint((double)ax / ulp);
    return copysignf((float)(q * ulp), x);
}

/* array forms for sweeps in the tests */
void or_vm_exp_n(const float* x, float* y, int64_t n)
{
    for (int64_t i = 0; i < n; i++) y[i] = or_vm_exp(x[i]);
}

void or_round_f16_n(const float* x, float* y, int64_t n)
{
    for (int64_t i = 0; i < n; i++) y[i] = or_round_f16(x[i]);
}

void or_round_bf16_n(const float* x, float* y, int64_t n)
{
    for (int64_t i = 0; i < n; i++) y[i] = or_round_bf16(x[i]);
}
