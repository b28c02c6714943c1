/*
 * or_create.c -- oracle create-time data (paper Sec. 3).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 *  - storage transform (Sec. 3 "Scene Storage"): unit quaternion, activated
 *    scale/opacity, 59 floats per Gaussian;
 *  - page assignment (Sec. 3 "Page Assignment"): Gaussians in Morton order
 *    (the locality order the paper recommends in Sec. 5.3), consecutive
 *    blocks of P per page, the last page padded with all-zero Gaussians;
 *  - proxy for the page-ID buffer (Sec. 3 "Mesh Extraction" samples the
 *    scene on a uniform grid): one box per occupied grid cell, the bounding
 *    box of the means in the cell, tagged with the page that has most means
 *    in it (ties to the lower page id);
 *  - page links (Sec. 3 "Page Linking"): a Gaussian of page p whose mean
 *    lies in, or whose link_sigma ellipsoid contains the centre of, a box
 *    tagged q != p makes the link q -> p (load p whenever q is seen);
 *  - page bounding spheres for the frustum test: the box of mu +- 3 sigma
 *    over the page's Gaussians joined with its proxy boxes;
 *  - LOD levels (Sec. 3 "Level of Detail"): parents of 8 consecutive
 *    children by opacity-weighted moment matching.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

struct or_scene {
    int64_t n_in;
    int P, L, n_pg, attr_format;
    double cell, link_sigma;
    double lo[3];                 /* min corner of the means */
    int64_t* perm;                /* [n_pg*P] input index, -1 = padding */
    float* attr[3];               /* level l: [n_pg * (P >> 3l)][59] */
    float* spheres;               /* [n_pg][4] */
    int64_t n_cells;
    float* cell_box;              /* [n_cells][6] lo xyz, hi xyz */
    int32_t* cell_page;           /* [n_cells] */
    int64_t* cell_key;            /* [n_cells] */
    int32_t* cell_start;          /* [n_pg+1] */
    int64_t n_links;
    int32_t* link_start;          /* [n_pg+1] */
    int32_t* link_dst;            /* [n_links] */
};

/* ------------------------------------------------------------------------ */
/* rotation matrix of a unit quaternion (w, x, y, z), double */
static void quat_rot_d(const float* q, double R[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* standard deviation of a Gaussian along each world axis: sqrt(Sigma_aa) */
static void axis_sigma(const float* rec, double sig[3])
{
    double R[3][3];
    quat_rot_d(rec + 6, R);
    for (int a = 0; a < 3; a++) {
        double v0 = R[a][0] * rec[3], v1 = R[a][1] * rec[4], v2 = R[a][2] * rec[5];
        sig[a] = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    }
}

/* ------------------------------------------------------------------------ */
typedef struct { uint64_t code; int64_t idx; } mkey;

static int cmp_mkey(const void* a, const void* b)
{
    const mkey* x = a; const mkey* y = b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* interleave: bit b of axis a goes to bit 3b + a */
static uint64_t morton3(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t c = 0;
    for (int b = 0; b < 21; b++) {
        c |= (uint64_t)((qx >> b) & 1u) << (3 * b);
        c |= (uint64_t)((qy >> b) & 1u) << (3 * b + 1);
        c |= (uint64_t)((qz >> b) & 1u) << (3 * b + 2);
    }
    return c;
}

static uint32_t morton_q(double x, double lo, double side)
{
    double t = floor((x - lo) / side * 2097152.0);
    if (t < 0.0) t = 0.0;
    if (t > 2097151.0) t = 2097151.0;
    return (uint32_t)t;
}

/* ------------------------------------------------------------------------ */
typedef struct { int64_t key; int32_t page; int32_t pad; float m[3]; } cellrec;

static int cmp_cellrec(const void* a, const void* b)
{
    const cellrec* x = a; const cellrec* y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->page > y->page) - (x->page < y->page);
}

static int64_t cell_key_of(int64_t ix, int64_t iy, int64_t iz)
{
    return ((ix + 1048576) << 42) | ((iy + 1048576) << 21) | (iz + 1048576);
}

typedef struct { int32_t page; int64_t key; int64_t src; } cellsort;

static int cmp_cellsort(const void* a, const void* b)
{
    const cellsort* x = a; const cellsort* y = b;
    if (x->page != y->page) return x->page < y->page ? -1 : 1;
    return (x->key > y->key) - (x->key < y->key);
}

typedef struct { int32_t q, p; } linkrec;

static int cmp_link(const void* a, const void* b)
{
    const linkrec* x = a; const linkrec* y = b;
    if (x->q != y->q) return x->q < y->q ? -1 : 1;
    return (x->p > y->p) - (x->p < y->p);
}

static int64_t find_cell(const int64_t* keys, int64_t n, int64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && keys[lo] == key) ? lo : -1;
}

/* ------------------------------------------------------------------------ */
/* symmetric 3x3 eigen-decomposition in closed form (Smith 1961): eigenvalues
 * from the trigonometric solution of the characteristic cubic, eigenvectors
 * from cross products of rows of A - lambda I.  Values descending. */
static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void eig_sym3(const double A[3][3], double lam[3], double V[3][3] /* columns */)
{
    const double pi = 3.14159265358979323846;
    double p1 = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double q = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    double d0 = A[0][0] - q, d1 = A[1][1] - q, d2 = A[2][2] - q;
    double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
    double p = sqrt(p2 / 6.0);
    if (p == 0.0) {
        lam[0] = lam[1] = lam[2] = q;
        for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) V[i][j] = (i == j);
        return;
    }
    double B[3][3];
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) B[i][j] = (A[i][j] - (i == j ? q : 0.0)) / p;
    double detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1])
                - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0])
                + B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    double r = detB / 2.0;
    if (r < -1.0) r = -1.0;
    if (r > 1.0) r = 1.0;
    double phi = acos(r) / 3.0;
    lam[0] = q + 2.0 * p * cos(phi);
    lam[2] = q + 2.0 * p * cos(phi + 2.0 * pi / 3.0);
    lam[1] = 3.0 * q - lam[0] - lam[2];
    /* eigenvectors of the two outer eigenvalues, the middle one by cross product */
    double vec[3][3];
    for (int e = 0; e < 3; e += 2) {
        double M[3][3];
        for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) M[i][j] = A[i][j] - (i == j ? lam[e] : 0.0);
        double c[3][3];
        cross3(M[0], M[1], c[0]);
        cross3(M[0], M[2], c[1]);
        cross3(M[1], M[2], c[2]);
        int best = 0; double bn = dot3(c[0], c[0]);
        for (int k = 1; k < 3; k++) { double nk = dot3(c[k], c[k]); if (nk > bn) { bn = nk; best = k; } }
        if (bn <= 0.0) { vec[e][0] = (e == 0); vec[e][1] = 0.0; vec[e][2] = (e == 2); continue; }
        double inv = 1.0 / sqrt(bn);
        for (int i = 0; i < 3; i++) vec[e][i] = c[best][i] * inv;
    }
    /* make the third orthogonal to the first if the two outer ones are degenerate */
    double d = dot3(vec[0], vec[2]);
    if (fabs(d) > 1e-6) {
        for (int i = 0; i < 3; i++) vec[2][i] -= d * vec[0][i];
        double nn = sqrt(dot3(vec[2], vec[2]));
        if (nn < 1e-12) {
            double t[3] = {1.0, 0.0, 0.0};
            if (fabs(vec[0][0]) > 0.9) { t[0] = 0.0; t[1] = 1.0; }
            cross3(vec[0], t, vec[2]);
            nn = sqrt(dot3(vec[2], vec[2]));
        }
        for (int i = 0; i < 3; i++) vec[2][i] /= nn;
    }
    cross3(vec[2], vec[0], vec[1]);
    for (int i = 0; i < 3; i++) for (int e = 0; e < 3; e++) V[i][e] = vec[e][i];
}

/* rotation matrix (columns = axes, det +1) -> unit quaternion with w >= 0 */
static void rot_to_quat(double R[3][3], double q[4])
{
    double tr = R[0][0] + R[1][1] + R[2][2];
    if (tr > 0.0) {
        double s = sqrt(tr + 1.0) * 2.0;
        q[0] = 0.25 * s;
        q[1] = (R[2][1] - R[1][2]) / s;
        q[2] = (R[0][2] - R[2][0]) / s;
        q[3] = (R[1][0] - R[0][1]) / s;
    } else if (R[0][0] > R[1][1] && R[0][0] > R[2][2]) {
        double s = sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]) * 2.0;
        q[0] = (R[2][1] - R[1][2]) / s;
        q[1] = 0.25 * s;
        q[2] = (R[0][1] + R[1][0]) / s;
        q[3] = (R[0][2] + R[2][0]) / s;
    } else if (R[1][1] > R[2][2]) {
        double s = sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]) * 2.0;
        q[0] = (R[0][2] - R[2][0]) / s;
        q[1] = (R[0][1] + R[1][0]) / s;
        q[2] = 0.25 * s;
        q[3] = (R[1][2] + R[2][1]) / s;
    } else {
        double s = sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]) * 2.0;
        q[0] = (R[1][0] - R[0][1]) / s;
        q[1] = (R[0][2] + R[2][0]) / s;
        q[2] = (R[1][2] + R[2][1]) / s;
        q[3] = 0.25 * s;
    }
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; i++) q[i] /= n;
    if (q[0] < 0.0) for (int i = 0; i < 4; i++) q[i] = -q[i];
}

/* Parent of k children (records c[0..k-1]) by opacity-weighted moment
 * matching (the parent construction read for Sec. 3 "Level of Detail"):
 * mu = sum w mu_i / W, Sigma = sum w (Sigma_i + d d^T) / W (the law of total
 * covariance of the opacity-weighted mixture), opacity = min(1, sum o_i),
 * SH = sum w SH_i / W, w_i = o_i.  Sigma is written back as scale = sqrt of
 * its eigenvalues (descending) and the rotation of its eigenvectors as a
 * unit quaternion with w >= 0.  The section then scales the merged Gaussian
 * up by a fixed factor, because a merged Gaussian covers less than the
 * children it replaces: the scales are multiplied by scale_up (so Sigma by
 * scale_up^2).  The record is produced in double (or_merge_children_d) and
 * stored rounded to float (or_merge_children).  All-zero opacities give the
 * all-zero padding parent. */
void or_merge_children_d(const float* c, int k, double scale_up, double* out)
{
    double W = 0.0, osum = 0.0;
    for (int i = 0; i < k; i++) { W += c[i * OR_REC + 10]; osum += c[i * OR_REC + 10]; }
    for (int a = 0; a < OR_REC; a++) out[a] = 0.0;
    if (!(W > 0.0)) return;                       /* padding parent */
    double mu[3] = {0, 0, 0};
    for (int i = 0; i < k; i++) {
        double w = c[i * OR_REC + 10];
        for (int a = 0; a < 3; a++) mu[a] += w * c[i * OR_REC + a];
    }
    for (int a = 0; a < 3; a++) mu[a] /= W;
    double S[3][3] = {{0}};
    for (int i = 0; i < k; i++) {
        const float* g = c + i * OR_REC;
        double w = g[10];
        if (w == 0.0) continue;
        double R[3][3];
        quat_rot_d(g + 6, R);
        double M[3][3];
        for (int a = 0; a < 3; a++) for (int j = 0; j < 3; j++) M[a][j] = R[a][j] * g[3 + j];
        double d[3] = {g[0] - mu[0], g[1] - mu[1], g[2] - mu[2]};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double sab = M[a][0] * M[b][0] + M[a][1] * M[b][1] + M[a][2] * M[b][2];
                S[a][b] += w * (sab + d[a] * d[b]);
            }
    }
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) S[a][b] /= W;
    double lam[3], V[3][3];
    eig_sym3(S, lam, V);
    double qd[4];
    rot_to_quat(V, qd);
    for (int a = 0; a < 3; a++) out[a] = mu[a];
    for (int e = 0; e < 3; e++) out[3 + e] = scale_up * sqrt(lam[e] > 0.0 ? lam[e] : 0.0);
    for (int i = 0; i < 4; i++) out[6 + i] = qd[i];
    out[10] = osum < 1.0 ? osum : 1.0;
    for (int j = 0; j < 48; j++) {
        double acc = 0.0;
        for (int i = 0; i < k; i++) acc += (double)c[i * OR_REC + 10] * c[i * OR_REC + 11 + j];
        out[11 + j] = acc / W;
    }
}

void or_merge_children(const float* c, int k, double scale_up, float* out)
{
    double d[OR_REC];
    or_merge_children_d(c, k, scale_up, d);
    for (int a = 0; a < OR_REC; a++) out[a] = (float)d[a];
}

/* ---- k-means parents (Sec. 3 "Level of Detail", the paper's builder) -----
 * The section clusters the Gaussians of a page by their attributes with
 * k-means, attributes scaled so that position dominates, and merges each
 * cluster by the arithmetic mean of position, rotation, opacity and SH, the
 * merged scale raised by a fixed factor.  Readings taken here:
 *  - members: the records of the level below with opacity > 0, in their
 *    (Morton) order; k = the level's Gaussians per page;
 *  - features (double): position minus the members' mean, divided by their
 *    RMS distance from it (1 when 0); and, times KM_W = 1/4, the quaternion
 *    in its w >= 0 form, the base colour (C0 times the DC coefficients) and
 *    the opacity;
 *  - seeds: the members at positions floor((2i + 1) m / (2k)), i < k; with
 *    m <= k members every member is a cluster of its own;
 *  - Lloyd iterations: each member to its nearest centroid (squared
 *    Euclidean distance, ties to the lower cluster), centroids to the mean
 *    of their members (an empty cluster keeps its centroid), until no
 *    assignment changes, at most KM_ITERS;
 *  - merge: the means of position, opacity and SH; the mean of the
 *    quaternions, each signed to agree with the cluster's first member,
 *    normalised ((1, 0, 0, 0) if it vanishes) and put in w >= 0 form; the
 *    mean of the scales times scale_up.  An empty cluster gives an all-zero
 *    (padding) parent. */
#define KM_ITERS 16
#define KM_DIM 11
static const double KM_W = 0.25;
static const double KM_C0 = 0.28209479177387814;   /* 1 / (2 sqrt(pi)) */

static double km_dist(const double* f, const double* c)
{
    double d = 0.0;
    for (int a = 0; a < KM_DIM; a++) { double e = f[a] - c[a]; d += e * e; }
    return d;
}

int or_kmeans_page(const float* c, int n, int k, double scale_up, float* out, int32_t* assign)
{
    memset(out, 0, sizeof(float) * OR_REC * (size_t)k);
    if (assign) for (int j = 0; j < n; j++) assign[j] = -1;
    int32_t* idx = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int m = 0;
    for (int j = 0; j < n; j++) if (c[j * OR_REC + 10] > 0.0f) idx[m++] = j;
    int32_t* as = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int iters = 0;
    if (m <= k) {
        for (int j = 0; j < m; j++) as[j] = j;
    } else {
        double c0[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < m; j++) for (int a = 0; a < 3; a++) c0[a] += c[idx[j] * OR_REC + a];
        for (int a = 0; a < 3; a++) c0[a] /= m;
        double ss = 0.0;
        for (int j = 0; j < m; j++)
            for (int a = 0; a < 3; a++) { double d = c[idx[j] * OR_REC + a] - c0[a]; ss += d * d; }
        double rms = sqrt(ss / m);
        double inv = rms > 0.0 ? 1.0 / rms : 1.0;
        double* F = malloc(sizeof(double) * KM_DIM * (size_t)m);
        for (int j = 0; j < m; j++) {
            const float* g = c + idx[j] * OR_REC;
            double* f = F + (size_t)j * KM_DIM;
            double sg = g[6] < 0.0f ? -1.0 : 1.0;
            for (int a = 0; a < 3; a++) f[a] = ((double)g[a] - c0[a]) * inv;
            for (int a = 0; a < 4; a++) f[3 + a] = KM_W * (sg * (double)g[6 + a]);
            for (int a = 0; a < 3; a++) f[7 + a] = KM_W * (KM_C0 * (double)g[11 + a]);
            f[10] = KM_W * (double)g[10];
        }
        double* C = malloc(sizeof(double) * KM_DIM * (size_t)k);
        double* S = malloc(sizeof(double) * KM_DIM * (size_t)k);
        int64_t* cnt = malloc(sizeof(int64_t) * (size_t)k);
        for (int i = 0; i < k; i++) {
            int sd = (int)(((int64_t)(2 * i + 1) * m) / (2 * (int64_t)k));
            memcpy(C + (size_t)i * KM_DIM, F + (size_t)sd * KM_DIM, sizeof(double) * KM_DIM);
        }
        for (int j = 0; j < m; j++) as[j] = -1;
        for (int it = 0; it < KM_ITERS; it++) {
            int changed = 0;
            for (int j = 0; j < m; j++) {
                const double* f = F + (size_t)j * KM_DIM;
                int best = 0;
                double bd = km_dist(f, C);
                for (int i = 1; i < k; i++) {
                    double d = km_dist(f, C + (size_t)i * KM_DIM);
                    if (d < bd) { bd = d; best = i; }
                }
                if (as[j] != best) { as[j] = best; changed = 1; }
            }
            iters = it + 1;
            if (!changed) break;
            memset(S, 0, sizeof(double) * KM_DIM * (size_t)k);
            memset(cnt, 0, sizeof(int64_t) * (size_t)k);
            for (int j = 0; j < m; j++) {
                cnt[as[j]]++;
                for (int a = 0; a < KM_DIM; a++) S[(size_t)as[j] * KM_DIM + a] += F[(size_t)j * KM_DIM + a];
            }
            for (int i = 0; i < k; i++)
                if (cnt[i] > 0)
                    for (int a = 0; a < KM_DIM; a++) C[(size_t)i * KM_DIM + a] = S[(size_t)i * KM_DIM + a] / cnt[i];
        }
        free(F); free(C); free(S); free(cnt);
    }
    /* merge every cluster (members in their order) */
    for (int i = 0; i < k; i++) {
        double acc[OR_REC];
        for (int a = 0; a < OR_REC; a++) acc[a] = 0.0;
        int cn = 0, first = -1;
        for (int j = 0; j < m; j++) {
            if (as[j] != i) continue;
            const float* g = c + idx[j] * OR_REC;
            if (first < 0) first = idx[j];
            const float* q0 = c + first * OR_REC + 6;
            double dot = (double)g[6] * q0[0] + (double)g[7] * q0[1] + (double)g[8] * q0[2] + (double)g[9] * q0[3];
            double sg = dot < 0.0 ? -1.0 : 1.0;
            for (int a = 0; a < 6; a++) acc[a] += g[a];
            for (int a = 6; a < 10; a++) acc[a] += sg * (double)g[a];
            for (int a = 10; a < OR_REC; a++) acc[a] += g[a];
            cn++;
        }
        if (cn == 0) continue;
        float* o = out + (size_t)i * OR_REC;
        for (int a = 0; a < 3; a++) o[a] = (float)(acc[a] / cn);
        for (int a = 3; a < 6; a++) o[a] = (float)(scale_up * (acc[a] / cn));
        double qn = sqrt(((acc[6] * acc[6] + acc[7] * acc[7]) + acc[8] * acc[8]) + acc[9] * acc[9]);
        double q[4] = {1.0, 0.0, 0.0, 0.0};
        if (qn > 0.0) for (int a = 0; a < 4; a++) q[a] = acc[6 + a] / qn;
        if (q[0] < 0.0) for (int a = 0; a < 4; a++) q[a] = -q[a];
        for (int a = 0; a < 4; a++) o[6 + a] = (float)q[a];
        for (int a = 10; a < OR_REC; a++) o[a] = (float)(acc[a] / cn);
    }
    if (assign) for (int j = 0; j < m; j++) assign[idx[j]] = as[j];
    free(as);
    free(idx);
    return iters;
}

static void round_half_form(float* rec)
{
    for (int a = 3; a < 11; a++) rec[a] = or_round_f16(rec[a]);
    for (int a = 11; a < OR_REC; a++) rec[a] = or_round_bf16(rec[a]);
}

/* ------------------------------------------------------------------------ */
or_scene* or_scene_build(const or_scene_in* in, int P, int L, double cell_m, double link_sigma, int attr_format,
                         float lod_scale_up, int lod_builder)
{
    if (!in || in->n <= 0 || P <= 0 || L < 1 || L > 3 || cell_m <= 0.0 || lod_builder < 0 || lod_builder > 1)
        return NULL;
    for (int l = 1; l < L; l++) if ((P >> (3 * l)) << (3 * l) != P || (P >> (3 * l)) == 0) return NULL;
    or_scene* s = calloc(1, sizeof(or_scene));
    int64_t n = in->n;
    s->n_in = n; s->P = P; s->L = L; s->cell = cell_m; s->link_sigma = link_sigma;
    s->attr_format = attr_format;
    s->n_pg = (int)((n + P - 1) / P);

    /* storage transform: 59-float records with unit quaternions */
    float* rec = malloc(sizeof(float) * OR_REC * (size_t)n);
    for (int64_t i = 0; i < n; i++) {
        float* r = rec + i * OR_REC;
        for (int a = 0; a < 3; a++) r[a] = in->means[i * 3 + a];
        for (int a = 0; a < 3; a++) r[3 + a] = in->scales[i * 3 + a];
        double qw = in->quats[i * 4], qx = in->quats[i * 4 + 1], qy = in->quats[i * 4 + 2], qz = in->quats[i * 4 + 3];
        double nq = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
        if (nq > 0.0) {
            r[6] = (float)(qw / nq); r[7] = (float)(qx / nq); r[8] = (float)(qy / nq); r[9] = (float)(qz / nq);
        } else {
            r[6] = 1.0f; r[7] = r[8] = r[9] = 0.0f;
        }
        r[10] = in->opacity[i];
        for (int j = 0; j < 48; j++) r[11 + j] = in->sh[i * 48 + j];
    }

    /* Morton order over the cube-ified box of the means */
    double lo[3], hi[3];
    for (int a = 0; a < 3; a++) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            double v = rec[i * OR_REC + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double side = 0.0;
    for (int a = 0; a < 3; a++) if (hi[a] - lo[a] > side) side = hi[a] - lo[a];
    if (!(side > 0.0)) side = 1.0;
    for (int a = 0; a < 3; a++) s->lo[a] = lo[a];
    mkey* mk = malloc(sizeof(mkey) * (size_t)n);
    for (int64_t i = 0; i < n; i++) {
        const float* r = rec + i * OR_REC;
        mk[i].code = morton3(morton_q(r[0], lo[0], side), morton_q(r[1], lo[1], side), morton_q(r[2], lo[2], side));
        mk[i].idx = i;
    }
    qsort(mk, (size_t)n, sizeof(mkey), cmp_mkey);

    /* pages of P, last one padded with zero Gaussians */
    int64_t np = (int64_t)s->n_pg * P;
    s->perm = malloc(sizeof(int64_t) * (size_t)np);
    s->attr[0] = calloc((size_t)np * OR_REC, sizeof(float));
    for (int64_t k = 0; k < np; k++) {
        if (k < n) {
            s->perm[k] = mk[k].idx;
            memcpy(s->attr[0] + k * OR_REC, rec + mk[k].idx * OR_REC, sizeof(float) * OR_REC);
        } else {
            s->perm[k] = -1;
        }
    }
    free(mk);
    free(rec);

    /* LOD levels from the full-precision level below */
    for (int l = 1; l < L; l++) {
        int64_t cnt = (int64_t)s->n_pg * (P >> (3 * l));
        s->attr[l] = calloc((size_t)cnt * OR_REC, sizeof(float));
        if (lod_builder == 1) {
            int pl = P >> (3 * l), pb = P >> (3 * (l - 1));
            /* pages are independent: OpenMP over them changes no record */
            #pragma omp parallel for schedule(dynamic, 16)
            for (int p = 0; p < s->n_pg; p++)
                or_kmeans_page(s->attr[l - 1] + (int64_t)p * pb * OR_REC, pb, pl, lod_scale_up,
                               s->attr[l] + (int64_t)p * pl * OR_REC, NULL);
        } else {
            for (int64_t i = 0; i < cnt; i++)
                or_merge_children(s->attr[l - 1] + (8 * i) * OR_REC, 8, lod_scale_up, s->attr[l] + i * OR_REC);
        }
    }

    /* proxy boxes: occupied cells of the means */
    cellrec* cr = malloc(sizeof(cellrec) * (size_t)n);
    for (int64_t k = 0; k < n; k++) {
        const float* r = s->attr[0] + k * OR_REC;
        int64_t ix = (int64_t)floor(((double)r[0] - lo[0]) / cell_m);
        int64_t iy = (int64_t)floor(((double)r[1] - lo[1]) / cell_m);
        int64_t iz = (int64_t)floor(((double)r[2] - lo[2]) / cell_m);
        cr[k].key = cell_key_of(ix, iy, iz);
        cr[k].page = (int32_t)(k / P);
        cr[k].m[0] = r[0]; cr[k].m[1] = r[1]; cr[k].m[2] = r[2];
    }
    qsort(cr, (size_t)n, sizeof(cellrec), cmp_cellrec);
    int64_t nc = 0;
    for (int64_t k = 0; k < n; k++) if (k == 0 || cr[k].key != cr[k - 1].key) nc++;
    int64_t* keys = malloc(sizeof(int64_t) * (size_t)nc);
    float* box = malloc(sizeof(float) * 6 * (size_t)nc);
    int32_t* tag = malloc(sizeof(int32_t) * (size_t)nc);
    {
        int64_t c = -1;
        int64_t k = 0;
        while (k < n) {
            int64_t e = k;
            while (e < n && cr[e].key == cr[k].key) e++;
            c++;
            keys[c] = cr[k].key;
            float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
            int32_t best = -1; int64_t bestn = 0;
            int64_t run = 0;
            for (int64_t t = k; t < e; t++) {
                for (int a = 0; a < 3; a++) {
                    if (cr[t].m[a] < b[a]) b[a] = cr[t].m[a];
                    if (cr[t].m[a] > b[3 + a]) b[3 + a] = cr[t].m[a];
                }
                run++;
                if (t + 1 == e || cr[t + 1].page != cr[t].page) {
                    if (run > bestn) { bestn = run; best = cr[t].page; }   /* pages ascend: ties keep the lower */
                    run = 0;
                }
            }
            memcpy(box + 6 * c, b, sizeof b);
            tag[c] = best;
            k = e;
        }
    }
    free(cr);
    /* cells grouped by tag page (ascending cell key inside) */
    cellsort* cs = malloc(sizeof(cellsort) * (size_t)nc);
    for (int64_t c = 0; c < nc; c++) { cs[c].page = tag[c]; cs[c].key = keys[c]; cs[c].src = c; }
    qsort(cs, (size_t)nc, sizeof(cellsort), cmp_cellsort);
    s->n_cells = nc;
    s->cell_box = malloc(sizeof(float) * 6 * (size_t)nc);
    s->cell_page = malloc(sizeof(int32_t) * (size_t)nc);
    s->cell_key = malloc(sizeof(int64_t) * (size_t)nc);
    s->cell_start = calloc((size_t)s->n_pg + 1, sizeof(int32_t));
    for (int64_t c = 0; c < nc; c++) {
        memcpy(s->cell_box + 6 * c, box + 6 * cs[c].src, sizeof(float) * 6);
        s->cell_page[c] = cs[c].page;
        s->cell_key[c] = cs[c].key;
        s->cell_start[cs[c].page + 1]++;
    }
    for (int p = 0; p < s->n_pg; p++) s->cell_start[p + 1] += s->cell_start[p];
    free(cs);

    /* page spheres: mu +- 3 sigma over the page's Gaussians, joined with its boxes */
    s->spheres = malloc(sizeof(float) * 4 * (size_t)s->n_pg);
    for (int p = 0; p < s->n_pg; p++) {
        double b0[3] = {INFINITY, INFINITY, INFINITY}, b1[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = 0; i < P; i++) {
            int64_t k = (int64_t)p * P + i;
            if (s->perm[k] < 0) continue;
            const float* r = s->attr[0] + k * OR_REC;
            double sig[3];
            axis_sigma(r, sig);
            for (int a = 0; a < 3; a++) {
                double e0 = (double)r[a] - 3.0 * sig[a], e1 = (double)r[a] + 3.0 * sig[a];
                if (e0 < b0[a]) b0[a] = e0;
                if (e1 > b1[a]) b1[a] = e1;
            }
        }
        for (int32_t c = s->cell_start[p]; c < s->cell_start[p + 1]; c++)
            for (int a = 0; a < 3; a++) {
                if (s->cell_box[6 * c + a] < b0[a]) b0[a] = s->cell_box[6 * c + a];
                if (s->cell_box[6 * c + 3 + a] > b1[a]) b1[a] = s->cell_box[6 * c + 3 + a];
            }
        double cen[3], rr = 0.0, shift = 0.0;
        for (int a = 0; a < 3; a++) {
            cen[a] = 0.5 * (b0[a] + b1[a]);
            rr += (b1[a] - b0[a]) * (b1[a] - b0[a]);
        }
        rr = 0.5 * sqrt(rr);
        float cf[3];
        for (int a = 0; a < 3; a++) {
            cf[a] = (float)cen[a];
            shift += ((double)cf[a] - cen[a]) * ((double)cf[a] - cen[a]);
        }
        double rad = rr + sqrt(shift);
        float rf = (float)rad;
        if ((double)rf < rad) rf = nextafterf(rf, INFINITY);
        s->spheres[4 * p] = cf[0]; s->spheres[4 * p + 1] = cf[1]; s->spheres[4 * p + 2] = cf[2];
        s->spheres[4 * p + 3] = rf;
    }

    /* links q -> p */
    int64_t lcap = 1024, ln = 0;
    linkrec* lk = malloc(sizeof(linkrec) * (size_t)lcap);
    double ls2 = link_sigma * link_sigma;
    for (int64_t k = 0; k < n; k++) {
        const float* r = s->attr[0] + k * OR_REC;
        int32_t p = (int32_t)(k / P);
        double mu[3] = {r[0], r[1], r[2]};
        double R[3][3];
        quat_rot_d(r + 6, R);
        double sig[3];
        axis_sigma(r, sig);
        int64_t i0[3], i1[3], im[3];
        for (int a = 0; a < 3; a++) {
            im[a] = (int64_t)floor((mu[a] - lo[a]) / cell_m);
            i0[a] = (int64_t)floor((mu[a] - link_sigma * sig[a] - lo[a]) / cell_m);
            i1[a] = (int64_t)floor((mu[a] + link_sigma * sig[a] - lo[a]) / cell_m);
        }
        for (int64_t ix = i0[0]; ix <= i1[0]; ix++)
            for (int64_t iy = i0[1]; iy <= i1[1]; iy++)
                for (int64_t iz = i0[2]; iz <= i1[2]; iz++) {
                    int64_t c = find_cell(keys, nc, cell_key_of(ix, iy, iz));
                    if (c < 0) continue;
                    int32_t q = tag[c];
                    if (q == p) continue;
                    int inside = (ix == im[0] && iy == im[1] && iz == im[2]);
                    if (!inside) {
                        double d[3], m = 0.0;
                        for (int a = 0; a < 3; a++)
                            d[a] = 0.5 * ((double)box[6 * c + a] + (double)box[6 * c + 3 + a]) - mu[a];
                        for (int j = 0; j < 3; j++) {
                            double dj = R[0][j] * d[0] + R[1][j] * d[1] + R[2][j] * d[2];
                            double t = dj / (double)r[3 + j];
                            m += t * t;
                        }
                        inside = (m <= ls2);
                    }
                    if (!inside) continue;
                    if (ln == lcap) { lcap *= 2; lk = realloc(lk, sizeof(linkrec) * (size_t)lcap); }
                    lk[ln].q = q; lk[ln].p = p; ln++;
                }
    }
    qsort(lk, (size_t)ln, sizeof(linkrec), cmp_link);
    s->link_start = calloc((size_t)s->n_pg + 1, sizeof(int32_t));
    s->link_dst = malloc(sizeof(int32_t) * (size_t)(ln > 0 ? ln : 1));
    int64_t u = 0;
    for (int64_t i = 0; i < ln; i++) {
        if (i > 0 && lk[i].q == lk[i - 1].q && lk[i].p == lk[i - 1].p) continue;
        s->link_dst[u++] = lk[i].p;
        s->link_start[lk[i].q + 1]++;
    }
    for (int p = 0; p < s->n_pg; p++) s->link_start[p + 1] += s->link_start[p];
    s->n_links = u;
    free(lk);
    free(keys); free(box); free(tag);

    /* reduced-precision page form: SH bf16, scale/quat/opacity fp16, means fp32 */
    if (attr_format == 1)
        for (int l = 0; l < L; l++) {
            int64_t cnt = (int64_t)s->n_pg * (P >> (3 * l));
            for (int64_t i = 0; i < cnt; i++) round_half_form(s->attr[l] + i * OR_REC);
        }
    return s;
}

void or_scene_free(or_scene* s)
{
    if (!s) return;
    free(s->perm);
    for (int l = 0; l < 3; l++) free(s->attr[l]);
    free(s->spheres); free(s->cell_box); free(s->cell_page); free(s->cell_key); free(s->cell_start);
    free(s->link_start); free(s->link_dst);
    free(s);
}

/* accessors used by or_frame.c */
int or_scene_P(const or_scene* s) { return s->P; }
int or_scene_L(const or_scene* s) { return s->L; }
int or_scene_npg(const or_scene* s) { return s->n_pg; }
int or_scene_format(const or_scene* s) { return s->attr_format; }
const float* or_scene_attr(const or_scene* s, int l) { return s->attr[l]; }
const float* or_scene_spheres(const or_scene* s) { return s->spheres; }
int64_t or_scene_ncells(const or_scene* s) { return s->n_cells; }
const float* or_scene_cellbox(const or_scene* s) { return s->cell_box; }
const int32_t* or_scene_cellpage(const or_scene* s) { return s->cell_page; }
const int32_t* or_scene_cellstart(const or_scene* s) { return s->cell_start; }
const int32_t* or_scene_linkstart(const or_scene* s) { return s->link_start; }
const int32_t* or_scene_linkdst(const or_scene* s) { return s->link_dst; }
const int64_t* or_scene_perm(const or_scene* s) { return s->perm; }

static int64_t put(void* dst, int64_t cap, const void* src, int64_t bytes)
{
    if (dst && cap >= bytes && bytes > 0) memcpy(dst, src, (size_t)bytes);
    return bytes;
}

int64_t or_scene_get(const or_scene* s, const char* name, void* dst, int64_t cap)
{
    int64_t np = (int64_t)s->n_pg * s->P;
    if (!strcmp(name, "n_pages")) { int64_t v = s->n_pg; return put(dst, cap, &v, 8); }
    if (!strcmp(name, "perm")) return put(dst, cap, s->perm, 8 * np);
    if (!strcmp(name, "attr0")) return put(dst, cap, s->attr[0], 4 * OR_REC * np);
    if (!strcmp(name, "attr1") && s->L > 1) return put(dst, cap, s->attr[1], 4 * OR_REC * (np >> 3));
    if (!strcmp(name, "attr2") && s->L > 2) return put(dst, cap, s->attr[2], 4 * OR_REC * (np >> 6));
    if (!strcmp(name, "spheres")) return put(dst, cap, s->spheres, 16 * (int64_t)s->n_pg);
    if (!strcmp(name, "n_cells")) { int64_t v = s->n_cells; return put(dst, cap, &v, 8); }
    if (!strcmp(name, "cell_box")) return put(dst, cap, s->cell_box, 24 * s->n_cells);
    if (!strcmp(name, "cell_page")) return put(dst, cap, s->cell_page, 4 * s->n_cells);
    if (!strcmp(name, "cell_start")) return put(dst, cap, s->cell_start, 4 * ((int64_t)s->n_pg + 1));
    if (!strcmp(name, "n_links")) { int64_t v = s->n_links; return put(dst, cap, &v, 8); }
    if (!strcmp(name, "link_start")) return put(dst, cap, s->link_start, 4 * ((int64_t)s->n_pg + 1));
    if (!strcmp(name, "link_dst")) return put(dst, cap, s->link_dst, 4 * s->n_links);
    if (!strcmp(name, "lo")) return put(dst, cap, s->lo, 24);
    return -1;
}
