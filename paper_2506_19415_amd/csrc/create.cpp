// create.cpp -- create-time paging of the scene (Sec. 3 of the paper), host C++.
//
//  storage transform   unit quaternions (normalised in double), activated
//                      scale and opacity, 59 floats per Gaussian
//  page assignment     Morton order of the means (21 bits per axis over the
//                      cube around their bounding box, ties by input index),
//                      consecutive pages of P, last page padded with zeros
//  proxy               occupied cells of a uniform grid (edge cell_m): box of
//                      the means inside, tagged with the page owning most of
//                      them (ties to the lower page), grouped by tag page
//  links               q -> p when a Gaussian of page p has its mean in, or the
//                      centre of, a box tagged q != p inside its link_sigma
//                      ellipsoid
//  spheres             per page: box of mu +- 3 sigma joined with its proxy
//                      boxes; centre and half diagonal, rounded outward
//  LOD                 parent = opacity-weighted moment match of 8 children
//  store               page-major, SoA inside each page block; the half form
//                      keeps means in fp32, scale/quat/opacity in fp16 and
//                      SH in bf16 (both round to nearest even)
#include <math.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <unordered_map>

#include "vm3dgs_impl.h"

namespace vm {

namespace {

template <class F>
void parallel_for(int64_t n, F f, int64_t serial_below = 65536) {
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 16) nt = 16;
    if (n < serial_below || nt == 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t a = (int64_t)t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([=] { f(a, b); });
    }
    for (auto& x : th) x.join();
}

struct Rot {
    double r[3][3];
};

// rotation of a unit quaternion w,x,y,z (double)
inline Rot rot_of(const float* q) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    Rot R;
    R.r[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R.r[0][1] = 2.0 * (x * y - w * z);
    R.r[0][2] = 2.0 * (x * z + w * y);
    R.r[1][0] = 2.0 * (x * y + w * z);
    R.r[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R.r[1][2] = 2.0 * (y * z - w * x);
    R.r[2][0] = 2.0 * (x * z - w * y);
    R.r[2][1] = 2.0 * (y * z + w * x);
    R.r[2][2] = 1.0 - 2.0 * (x * x + y * y);
    return R;
}

inline void axis_sd(const float* g, double sd[3]) {
    const Rot R = rot_of(g + 6);
    for (int a = 0; a < 3; ++a) {
        const double v0 = R.r[a][0] * g[3], v1 = R.r[a][1] * g[4], v2 = R.r[a][2] * g[5];
        sd[a] = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    }
}

inline uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

inline uint32_t quant21(double x, double lo, double side) {
    double t = floor((x - lo) / side * 2097152.0);
    t = t < 0.0 ? 0.0 : (t > 2097151.0 ? 2097151.0 : t);
    return (uint32_t)t;
}

inline int64_t cell_key(int64_t ix, int64_t iy, int64_t iz) {
    return ((ix + 1048576) << 42) | ((iy + 1048576) << 21) | (iz + 1048576);
}

// ---- symmetric 3x3 eigen-decomposition, closed form (Smith 1961) --------
inline void cross(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

void eigen_sym3(const double A[3][3], double lam[3], double V[3][3]) {
    const double pi = 3.14159265358979323846;
    const double p1 = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double q = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    const double d0 = A[0][0] - q, d1 = A[1][1] - q, d2 = A[2][2] - q;
    const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    if (p == 0.0) {
        lam[0] = lam[1] = lam[2] = q;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
        return;
    }
    double B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = (A[i][j] - (i == j ? q : 0.0)) / p;
    const double detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                        B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                        B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    double r = detB / 2.0;
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    lam[0] = q + 2.0 * p * cos(phi);
    lam[2] = q + 2.0 * p * cos(phi + 2.0 * pi / 3.0);
    lam[1] = 3.0 * q - lam[0] - lam[2];
    double vec[3][3];
    for (int e = 0; e < 3; e += 2) {
        double M[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = A[i][j] - (i == j ? lam[e] : 0.0);
        double c[3][3];
        cross(M[0], M[1], c[0]);
        cross(M[0], M[2], c[1]);
        cross(M[1], M[2], c[2]);
        int best = 0;
        double bn = dot(c[0], c[0]);
        for (int k = 1; k < 3; ++k) {
            const double nk = dot(c[k], c[k]);
            if (nk > bn) { bn = nk; best = k; }
        }
        if (bn <= 0.0) {
            vec[e][0] = (e == 0); vec[e][1] = 0.0; vec[e][2] = (e == 2);
            continue;
        }
        const double inv = 1.0 / sqrt(bn);
        for (int i = 0; i < 3; ++i) vec[e][i] = c[best][i] * inv;
    }
    const double d = dot(vec[0], vec[2]);
    if (fabs(d) > 1e-6) {
        for (int i = 0; i < 3; ++i) vec[2][i] -= d * vec[0][i];
        double nn = sqrt(dot(vec[2], vec[2]));
        if (nn < 1e-12) {
            double t[3] = {1.0, 0.0, 0.0};
            if (fabs(vec[0][0]) > 0.9) { t[0] = 0.0; t[1] = 1.0; }
            cross(vec[0], t, vec[2]);
            nn = sqrt(dot(vec[2], vec[2]));
        }
        for (int i = 0; i < 3; ++i) vec[2][i] /= nn;
    }
    cross(vec[2], vec[0], vec[1]);
    for (int i = 0; i < 3; ++i)
        for (int e = 0; e < 3; ++e) V[i][e] = vec[e][i];
}

void quat_of(const double R[3][3], double q[4]) {
    const double tr = R[0][0] + R[1][1] + R[2][2];
    if (tr > 0.0) {
        const double s = sqrt(tr + 1.0) * 2.0;
        q[0] = 0.25 * s;
        q[1] = (R[2][1] - R[1][2]) / s;
        q[2] = (R[0][2] - R[2][0]) / s;
        q[3] = (R[1][0] - R[0][1]) / s;
    } else if (R[0][0] > R[1][1] && R[0][0] > R[2][2]) {
        const double s = sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]) * 2.0;
        q[0] = (R[2][1] - R[1][2]) / s;
        q[1] = 0.25 * s;
        q[2] = (R[0][1] + R[1][0]) / s;
        q[3] = (R[0][2] + R[2][0]) / s;
    } else if (R[1][1] > R[2][2]) {
        const double s = sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]) * 2.0;
        q[0] = (R[0][2] - R[2][0]) / s;
        q[1] = (R[0][1] + R[1][0]) / s;
        q[2] = 0.25 * s;
        q[3] = (R[1][2] + R[2][1]) / s;
    } else {
        const double s = sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]) * 2.0;
        q[0] = (R[1][0] - R[0][1]) / s;
        q[1] = (R[0][2] + R[2][0]) / s;
        q[2] = (R[1][2] + R[2][1]) / s;
        q[3] = 0.25 * s;
    }
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; ++i) q[i] /= n;
    if (q[0] < 0.0)
        for (int i = 0; i < 4; ++i) q[i] = -q[i];
}

// moment matching of k children into one parent (all-zero when no opacity);
// the parent's scales are then multiplied by scale_up
void merge(const float* ch, int k, double scale_up, float* out) {
    double W = 0.0, osum = 0.0;
    for (int i = 0; i < k; ++i) { W += ch[i * REC + 10]; osum += ch[i * REC + 10]; }
    memset(out, 0, sizeof(float) * REC);
    if (!(W > 0.0)) return;
    double mu[3] = {0, 0, 0};
    for (int i = 0; i < k; ++i) {
        const double w = ch[i * REC + 10];
        for (int a = 0; a < 3; ++a) mu[a] += w * ch[i * REC + a];
    }
    for (int a = 0; a < 3; ++a) mu[a] /= W;
    double S[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < k; ++i) {
        const float* g = ch + i * REC;
        const double w = g[10];
        if (w == 0.0) continue;
        const Rot R = rot_of(g + 6);
        double M[3][3];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 3; ++j) M[a][j] = R.r[a][j] * g[3 + j];
        const double d[3] = {g[0] - mu[0], g[1] - mu[1], g[2] - mu[2]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double sab = M[a][0] * M[b][0] + M[a][1] * M[b][1] + M[a][2] * M[b][2];
                S[a][b] += w * (sab + d[a] * d[b]);
            }
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] /= W;
    double lam[3], V[3][3], q[4];
    eigen_sym3(S, lam, V);
    quat_of(V, q);
    for (int a = 0; a < 3; ++a) out[a] = (float)mu[a];
    for (int e = 0; e < 3; ++e) out[3 + e] = (float)(scale_up * sqrt(lam[e] > 0.0 ? lam[e] : 0.0));
    for (int i = 0; i < 4; ++i) out[6 + i] = (float)q[i];
    out[10] = (float)(osum < 1.0 ? osum : 1.0);
    for (int j = 0; j < 48; ++j) {
        double acc = 0.0;
        for (int i = 0; i < k; ++i) acc += (double)ch[i * REC + 10] * ch[i * REC + 11 + j];
        out[11 + j] = (float)(acc / W);
    }
}

// k-means parents of one page's level (Sec. 3 Level of Detail): the n
// records c of the level below go into k clusters, found by Lloyd's
// algorithm on scaled attributes, and each cluster becomes one parent.
//  - members: records with opacity > 0, in order; m <= k: one cluster each;
//  - features (double): position minus the members' mean over their RMS
//    distance from it (1 when 0); times 1/4 each: the quaternion in w >= 0
//    form, the base colour C0 * DC, the opacity;
//  - seeds: members floor((2i + 1) m / (2k)); at most 16 iterations of
//    nearest centroid (squared distance, ties to the lower cluster) and
//    centroid = mean of its members (empty clusters keep theirs), stopping
//    when no member moves;
//  - parent: means of position, opacity and SH; the quaternions' mean, each
//    signed to agree with the cluster's first member, normalised
//    ((1, 0, 0, 0) if it vanishes), w >= 0; the scales' mean times scale_up.
//    An empty cluster gives an all-zero parent.
constexpr int KM_ITERS = 16, KM_DIM = 11;
constexpr double KM_W = 0.25, KM_C0 = 0.28209479177387814;

void kmeans_page(const float* c, int n, int k, double scale_up, float* out) {
    std::fill(out, out + (size_t)k * REC, 0.0f);
    std::vector<int> mem;
    mem.reserve((size_t)n);
    for (int j = 0; j < n; ++j)
        if (c[(size_t)j * REC + 10] > 0.0f) mem.push_back(j);
    const int m = (int)mem.size();
    std::vector<int> cl((size_t)m, -1);
    if (m <= k) {
        for (int j = 0; j < m; ++j) cl[(size_t)j] = j;
    } else {
        double mean[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < m; ++j)
            for (int a = 0; a < 3; ++a) mean[a] += c[(size_t)mem[(size_t)j] * REC + a];
        for (int a = 0; a < 3; ++a) mean[a] /= m;
        double ss = 0.0;
        for (int j = 0; j < m; ++j)
            for (int a = 0; a < 3; ++a) {
                const double d = c[(size_t)mem[(size_t)j] * REC + a] - mean[a];
                ss += d * d;
            }
        const double rms = sqrt(ss / m);
        const double inv = rms > 0.0 ? 1.0 / rms : 1.0;
        std::vector<double> F((size_t)m * KM_DIM), C((size_t)k * KM_DIM), S((size_t)k * KM_DIM);
        std::vector<int64_t> cnt((size_t)k);
        for (int j = 0; j < m; ++j) {
            const float* g = c + (size_t)mem[(size_t)j] * REC;
            double* f = &F[(size_t)j * KM_DIM];
            const double sg = g[6] < 0.0f ? -1.0 : 1.0;
            for (int a = 0; a < 3; ++a) f[a] = ((double)g[a] - mean[a]) * inv;
            for (int a = 0; a < 4; ++a) f[3 + a] = KM_W * (sg * (double)g[6 + a]);
            for (int a = 0; a < 3; ++a) f[7 + a] = KM_W * (KM_C0 * (double)g[11 + a]);
            f[10] = KM_W * (double)g[10];
        }
        for (int i = 0; i < k; ++i) {
            const int seed = (int)(((int64_t)(2 * i + 1) * m) / (2 * (int64_t)k));
            std::copy(&F[(size_t)seed * KM_DIM], &F[(size_t)seed * KM_DIM] + KM_DIM, &C[(size_t)i * KM_DIM]);
        }
        auto dist = [&](const double* f, const double* ctr) {
            double d = 0.0;
            for (int a = 0; a < KM_DIM; ++a) {
                const double e = f[a] - ctr[a];
                d += e * e;
            }
            return d;
        };
        for (int it = 0; it < KM_ITERS; ++it) {
            bool moved = false;
            for (int j = 0; j < m; ++j) {
                const double* f = &F[(size_t)j * KM_DIM];
                int best = 0;
                double bd = dist(f, &C[0]);
                for (int i = 1; i < k; ++i) {
                    const double d = dist(f, &C[(size_t)i * KM_DIM]);
                    if (d < bd) { bd = d; best = i; }
                }
                if (cl[(size_t)j] != best) { cl[(size_t)j] = best; moved = true; }
            }
            if (!moved) break;
            std::fill(S.begin(), S.end(), 0.0);
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int j = 0; j < m; ++j) {
                const int i = cl[(size_t)j];
                ++cnt[(size_t)i];
                for (int a = 0; a < KM_DIM; ++a) S[(size_t)i * KM_DIM + a] += F[(size_t)j * KM_DIM + a];
            }
            for (int i = 0; i < k; ++i)
                if (cnt[(size_t)i] > 0)
                    for (int a = 0; a < KM_DIM; ++a)
                        C[(size_t)i * KM_DIM + a] = S[(size_t)i * KM_DIM + a] / cnt[(size_t)i];
        }
    }
    // members of each cluster in order; accumulate in double
    std::vector<double> acc((size_t)k * REC, 0.0);
    std::vector<int> n_in((size_t)k, 0), first((size_t)k, -1);
    for (int j = 0; j < m; ++j) {
        const int i = cl[(size_t)j];
        const float* g = c + (size_t)mem[(size_t)j] * REC;
        if (first[(size_t)i] < 0) first[(size_t)i] = mem[(size_t)j];
        const float* q0 = c + (size_t)first[(size_t)i] * REC + 6;
        const double dot = (double)g[6] * q0[0] + (double)g[7] * q0[1] + (double)g[8] * q0[2] + (double)g[9] * q0[3];
        const double sg = dot < 0.0 ? -1.0 : 1.0;
        double* A = &acc[(size_t)i * REC];
        for (int a = 0; a < 6; ++a) A[a] += g[a];
        for (int a = 6; a < 10; ++a) A[a] += sg * (double)g[a];
        for (int a = 10; a < REC; ++a) A[a] += g[a];
        ++n_in[(size_t)i];
    }
    for (int i = 0; i < k; ++i) {
        const int cn = n_in[(size_t)i];
        if (cn == 0) continue;
        const double* A = &acc[(size_t)i * REC];
        float* o = out + (size_t)i * REC;
        for (int a = 0; a < 3; ++a) o[a] = (float)(A[a] / cn);
        for (int a = 3; a < 6; ++a) o[a] = (float)(scale_up * (A[a] / cn));
        const double qn = sqrt(((A[6] * A[6] + A[7] * A[7]) + A[8] * A[8]) + A[9] * A[9]);
        double q[4] = {1.0, 0.0, 0.0, 0.0};
        if (qn > 0.0)
            for (int a = 0; a < 4; ++a) q[a] = A[6 + a] / qn;
        if (q[0] < 0.0)
            for (int a = 0; a < 4; ++a) q[a] = -q[a];
        for (int a = 0; a < 4; ++a) o[6 + a] = (float)q[a];
        for (int a = 10; a < REC; ++a) o[a] = (float)(A[a] / cn);
    }
}

// IEEE round to nearest even, bit-level: float -> binary16 / bfloat16
inline uint16_t f32_to_f16(float f) {
    uint32_t x;
    memcpy(&x, &f, 4);
    const uint32_t sign = (x >> 16) & 0x8000u;
    const uint32_t ax = x & 0x7fffffffu;
    if (ax > 0x7f800000u) return (uint16_t)(sign | 0x7e00u);          // NaN
    if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);         // >= 65520 rounds to inf
    if (ax < 0x38800000u) {                                           // below 2^-14: subnormal half
        if (ax < 0x33000000u) return (uint16_t)sign;                  // below 2^-25: zero (ties to even)
        const uint32_t e = ax >> 23;
        const uint32_t m = (ax & 0x7fffffu) | 0x800000u;
        const uint32_t shift = 126u - e;                              // 14 + 1 + (112 - e) ... exponent gap
        uint32_t h = m >> (shift + 0u);
        const uint32_t rem = m & ((1u << shift) - 1u);
        const uint32_t half = 1u << (shift - 1u);
        if (rem > half || (rem == half && (h & 1u))) ++h;
        return (uint16_t)(sign | h);
    }
    uint32_t h = ((ax >> 13) - (112u << 10));
    const uint32_t rem = ax & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;
    return (uint16_t)(sign | h);
}

inline uint16_t f32_to_bf16(float f) {
    uint32_t x;
    memcpy(&x, &f, 4);
    if ((x & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((x >> 16) | 0x40u);
    const uint32_t lsb = (x >> 16) & 1u;
    x += 0x7fffu + lsb;
    return (uint16_t)(x >> 16);
}

inline float f16_to_f32(uint16_t h) {
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    uint32_t x;
    if (e == 0) {
        if (m == 0) x = sign;
        else {
            e = 113;
            while (!(m & 0x400u)) { m <<= 1; --e; }
            m &= 0x3ffu;
            x = sign | (e << 23) | (m << 13);
        }
    } else if (e == 31) {
        x = sign | 0x7f800000u | (m << 13);
    } else {
        x = sign | ((e + 112u) << 23) | (m << 13);
    }
    float f;
    memcpy(&f, &x, 4);
    return f;
}

inline float bf16_to_f32(uint16_t b) {
    const uint32_t x = (uint32_t)b << 16;
    float f;
    memcpy(&f, &x, 4);
    return f;
}

}  // namespace

std::string build_paged_scene(const vm3dgs_scene& sc, int P, int L, int fmt, double cell_m, double link_sigma,
                              double lod_scale_up, int lod_builder, PagedScene& ps) {
    const int64_t n = (int64_t)sc.n;
    ps = PagedScene();
    ps.n_in = n; ps.P = P; ps.L = L; ps.fmt = fmt;
    ps.bytes_g = fmt == 1 ? 124 : 236;
    ps.n_pg = (int)((n + P - 1) / P);
    const int64_t np = (int64_t)ps.n_pg * P;

    // storage transform
    std::vector<float> rec((size_t)n * REC);
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            float* r = &rec[(size_t)i * REC];
            for (int k = 0; k < 3; ++k) r[k] = sc.means[i * 3 + k];
            for (int k = 0; k < 3; ++k) r[3 + k] = sc.scales[i * 3 + k];
            const double qw = sc.quats[i * 4], qx = sc.quats[i * 4 + 1], qy = sc.quats[i * 4 + 2],
                         qz = sc.quats[i * 4 + 3];
            const double nq = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
            if (nq > 0.0) {
                r[6] = (float)(qw / nq); r[7] = (float)(qx / nq); r[8] = (float)(qy / nq); r[9] = (float)(qz / nq);
            } else {
                r[6] = 1.0f; r[7] = r[8] = r[9] = 0.0f;
            }
            r[10] = sc.opacity[i];
            memcpy(r + 11, sc.sh + i * 48, sizeof(float) * 48);
        }
    });

    // Morton order
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            const double v = rec[(size_t)i * REC + a];
            lo[a] = std::min(lo[a], v);
            hi[a] = std::max(hi[a], v);
        }
    double side = 0.0;
    for (int a = 0; a < 3; ++a) side = std::max(side, hi[a] - lo[a]);
    if (!(side > 0.0)) side = 1.0;
    for (int a = 0; a < 3; ++a) ps.lo[a] = lo[a];
    std::vector<std::pair<uint64_t, int64_t>> mk((size_t)n);
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            const float* r = &rec[(size_t)i * REC];
            const uint64_t c = spread21(quant21(r[0], lo[0], side)) | (spread21(quant21(r[1], lo[1], side)) << 1) |
                               (spread21(quant21(r[2], lo[2], side)) << 2);
            mk[(size_t)i] = {c, i};
        }
    });
    std::sort(mk.begin(), mk.end());

    ps.perm.assign((size_t)np, -1);
    ps.rec[0].assign((size_t)np * REC, 0.0f);
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            ps.perm[(size_t)k] = mk[(size_t)k].second;
            memcpy(&ps.rec[0][(size_t)k * REC], &rec[(size_t)mk[(size_t)k].second * REC], sizeof(float) * REC);
        }
    });
    std::vector<std::pair<uint64_t, int64_t>>().swap(mk);
    std::vector<float>().swap(rec);

    // LOD levels from the full-precision level below
    for (int l = 1; l < L; ++l) {
        const int64_t cnt = (int64_t)ps.n_pg * ps.P_l(l);
        ps.rec[l].assign((size_t)cnt * REC, 0.0f);
        const float* src = ps.rec[l - 1].data();
        float* dst = ps.rec[l].data();
        if (lod_builder == 1) {
            const int pl = ps.P_l(l), pb = ps.P_l(l - 1);
            parallel_for(
                ps.n_pg,
                [&](int64_t a, int64_t b) {
                    for (int64_t p = a; p < b; ++p)
                        kmeans_page(src + (size_t)(p * pb) * REC, pb, pl, lod_scale_up, dst + (size_t)(p * pl) * REC);
                },
                64);
        } else {
            parallel_for(cnt, [&](int64_t a, int64_t b) {
                for (int64_t i = a; i < b; ++i)
                    merge(src + (size_t)(8 * i) * REC, 8, lod_scale_up, dst + (size_t)i * REC);
            });
        }
    }

    // proxy: occupied cells of the means
    struct CellRec {
        int64_t key;
        int32_t page;
        int32_t k;
    };
    std::vector<CellRec> cr((size_t)n);
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            const float* r = &ps.rec[0][(size_t)k * REC];
            const int64_t ix = (int64_t)floor(((double)r[0] - lo[0]) / cell_m);
            const int64_t iy = (int64_t)floor(((double)r[1] - lo[1]) / cell_m);
            const int64_t iz = (int64_t)floor(((double)r[2] - lo[2]) / cell_m);
            cr[(size_t)k] = {cell_key(ix, iy, iz), (int32_t)(k / P), (int32_t)k};
        }
    });
    std::sort(cr.begin(), cr.end(), [](const CellRec& x, const CellRec& y) {
        return x.key != y.key ? x.key < y.key : x.k < y.k;
    });
    std::vector<int64_t> ckeys;
    std::vector<float> cbox;
    std::vector<int32_t> ctag;
    for (size_t s = 0; s < cr.size();) {
        size_t e = s;
        while (e < cr.size() && cr[e].key == cr[s].key) ++e;
        float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        // pages ascend with k inside a cell (k sorted): majority by runs, ties to the lower page
        int32_t best = -1;
        int64_t bestn = 0, run = 0;
        for (size_t t = s; t < e; ++t) {
            const float* r = &ps.rec[0][(size_t)cr[t].k * REC];
            for (int a = 0; a < 3; ++a) {
                b[a] = std::min(b[a], r[a]);
                b[3 + a] = std::max(b[3 + a], r[a]);
            }
            ++run;
            if (t + 1 == e || cr[t + 1].page != cr[t].page) {
                if (run > bestn) { bestn = run; best = cr[t].page; }
                run = 0;
            }
        }
        ckeys.push_back(cr[s].key);
        for (int a = 0; a < 6; ++a) cbox.push_back(b[a]);
        ctag.push_back(best);
        s = e;
    }
    std::vector<CellRec>().swap(cr);
    const int64_t nc = (int64_t)ckeys.size();
    std::vector<int64_t> corder((size_t)nc);
    for (int64_t c = 0; c < nc; ++c) corder[(size_t)c] = c;
    std::sort(corder.begin(), corder.end(), [&](int64_t x, int64_t y) {
        return ctag[(size_t)x] != ctag[(size_t)y] ? ctag[(size_t)x] < ctag[(size_t)y] : ckeys[(size_t)x] < ckeys[(size_t)y];
    });
    ps.cell_lo.resize((size_t)nc * 4);
    ps.cell_hi.resize((size_t)nc * 4);
    ps.cell_page.resize((size_t)nc);
    ps.cell_start.assign((size_t)ps.n_pg + 1, 0);
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t s = corder[(size_t)c];
        const int32_t pg = ctag[(size_t)s];
        float* l4 = &ps.cell_lo[(size_t)c * 4];
        float* h4 = &ps.cell_hi[(size_t)c * 4];
        l4[0] = cbox[(size_t)s * 6]; l4[1] = cbox[(size_t)s * 6 + 1]; l4[2] = cbox[(size_t)s * 6 + 2];
        uint32_t pb = (uint32_t)pg;
        memcpy(&l4[3], &pb, 4);
        h4[0] = cbox[(size_t)s * 6 + 3]; h4[1] = cbox[(size_t)s * 6 + 4]; h4[2] = cbox[(size_t)s * 6 + 5]; h4[3] = 0.0f;
        ps.cell_page[(size_t)c] = pg;
        ps.cell_start[(size_t)pg + 1]++;
    }
    for (int p = 0; p < ps.n_pg; ++p) ps.cell_start[(size_t)p + 1] += ps.cell_start[(size_t)p];

    // page spheres
    ps.spheres.resize((size_t)ps.n_pg * 4);
    parallel_for(ps.n_pg, [&](int64_t a, int64_t b) {
        for (int64_t p = a; p < b; ++p) {
            double b0[3] = {INFINITY, INFINITY, INFINITY}, b1[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int i = 0; i < P; ++i) {
                const int64_t k = p * P + i;
                if (ps.perm[(size_t)k] < 0) continue;
                const float* r = &ps.rec[0][(size_t)k * REC];
                double sd[3];
                axis_sd(r, sd);
                for (int ax = 0; ax < 3; ++ax) {
                    b0[ax] = std::min(b0[ax], (double)r[ax] - 3.0 * sd[ax]);
                    b1[ax] = std::max(b1[ax], (double)r[ax] + 3.0 * sd[ax]);
                }
            }
            for (int32_t c = ps.cell_start[(size_t)p]; c < ps.cell_start[(size_t)p + 1]; ++c)
                for (int ax = 0; ax < 3; ++ax) {
                    b0[ax] = std::min(b0[ax], (double)ps.cell_lo[(size_t)c * 4 + ax]);
                    b1[ax] = std::max(b1[ax], (double)ps.cell_hi[(size_t)c * 4 + ax]);
                }
            double cen[3], rr = 0.0, shift = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
                cen[ax] = 0.5 * (b0[ax] + b1[ax]);
                rr += (b1[ax] - b0[ax]) * (b1[ax] - b0[ax]);
            }
            rr = 0.5 * sqrt(rr);
            float cf[3];
            for (int ax = 0; ax < 3; ++ax) {
                cf[ax] = (float)cen[ax];
                shift += ((double)cf[ax] - cen[ax]) * ((double)cf[ax] - cen[ax]);
            }
            const double rad = rr + sqrt(shift);
            float rf = (float)rad;
            if ((double)rf < rad) rf = nextafterf(rf, INFINITY);
            float* o = &ps.spheres[(size_t)p * 4];
            o[0] = cf[0]; o[1] = cf[1]; o[2] = cf[2]; o[3] = rf;
        }
    });

    // links: a map from cell key to its index (in key order), then per-thread lists
    std::unordered_map<int64_t, int32_t> cidx;
    cidx.reserve((size_t)nc * 2);
    for (int64_t c = 0; c < nc; ++c) cidx.emplace(ckeys[(size_t)c], (int32_t)c);
    const double ls2 = link_sigma * link_sigma;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::vector<uint64_t>> part(nth);
    {
        std::vector<std::thread> th;
        const int64_t chunk = (n + nth - 1) / nth;
        for (unsigned t = 0; t < nth; ++t) {
            th.emplace_back([&, t] {
                const int64_t a = (int64_t)t * chunk, b = std::min(n, a + chunk);
                auto& out = part[t];
                for (int64_t k = a; k < b; ++k) {
                    const float* r = &ps.rec[0][(size_t)k * REC];
                    const int32_t p = (int32_t)(k / P);
                    const double mu[3] = {r[0], r[1], r[2]};
                    const Rot R = rot_of(r + 6);
                    double sd[3];
                    axis_sd(r, sd);
                    int64_t i0[3], i1[3], im[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        im[ax] = (int64_t)floor((mu[ax] - lo[ax]) / cell_m);
                        i0[ax] = (int64_t)floor((mu[ax] - link_sigma * sd[ax] - lo[ax]) / cell_m);
                        i1[ax] = (int64_t)floor((mu[ax] + link_sigma * sd[ax] - lo[ax]) / cell_m);
                    }
                    for (int64_t ix = i0[0]; ix <= i1[0]; ++ix)
                        for (int64_t iy = i0[1]; iy <= i1[1]; ++iy)
                            for (int64_t iz = i0[2]; iz <= i1[2]; ++iz) {
                                auto it = cidx.find(cell_key(ix, iy, iz));
                                if (it == cidx.end()) continue;
                                const int32_t c = it->second;
                                const int32_t q = ctag[(size_t)c];
                                if (q == p) continue;
                                bool inside = ix == im[0] && iy == im[1] && iz == im[2];
                                if (!inside) {
                                    double d[3], m = 0.0;
                                    for (int ax = 0; ax < 3; ++ax)
                                        d[ax] = 0.5 * ((double)cbox[(size_t)c * 6 + ax] +
                                                       (double)cbox[(size_t)c * 6 + 3 + ax]) - mu[ax];
                                    for (int j = 0; j < 3; ++j) {
                                        const double dj = R.r[0][j] * d[0] + R.r[1][j] * d[1] + R.r[2][j] * d[2];
                                        const double tt = dj / (double)r[3 + j];
                                        m += tt * tt;
                                    }
                                    inside = m <= ls2;
                                }
                                if (inside) out.push_back(((uint64_t)(uint32_t)q << 32) | (uint32_t)p);
                            }
                }
            });
        }
        for (auto& x : th) x.join();
    }
    std::vector<uint64_t> links;
    for (auto& v : part) links.insert(links.end(), v.begin(), v.end());
    std::sort(links.begin(), links.end());
    links.erase(std::unique(links.begin(), links.end()), links.end());
    ps.link_start.assign((size_t)ps.n_pg + 1, 0);
    ps.link_dst.resize(links.size());
    for (size_t i = 0; i < links.size(); ++i) {
        ps.link_dst[i] = (int32_t)(links[i] & 0xffffffffu);
        ps.link_start[(size_t)(links[i] >> 32) + 1]++;
    }
    for (int p = 0; p < ps.n_pg; ++p) ps.link_start[(size_t)p + 1] += ps.link_start[(size_t)p];

    // half form: keep the decoded values the device will see
    if (fmt == 1)
        for (int l = 0; l < L; ++l) {
            float* r = ps.rec[l].data();
            const int64_t cnt = (int64_t)ps.n_pg * ps.P_l(l);
            parallel_for(cnt, [&](int64_t a, int64_t b) {
                for (int64_t i = a; i < b; ++i) {
                    float* g = r + (size_t)i * REC;
                    for (int k = 3; k < 11; ++k) g[k] = f16_to_f32(f32_to_f16(g[k]));
                    for (int k = 11; k < REC; ++k) g[k] = bf16_to_f32(f32_to_bf16(g[k]));
                }
            });
        }

    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        ps.level_base[l] = off;
        off += (int64_t)ps.n_pg * ps.P_l(l) * ps.bytes_g;
    }
    ps.store_bytes = off;
    return "";
}

void encode_store(const PagedScene& ps, uint8_t* dst) {
    for (int l = 0; l < ps.L; ++l) {
        const int C = ps.P_l(l);
        const float* rec = ps.rec[l].data();
        uint8_t* base = dst + ps.level_base[l];
        parallel_for(ps.n_pg, [&](int64_t a, int64_t b) {
            for (int64_t p = a; p < b; ++p) {
                uint8_t* blk = base + (size_t)p * C * ps.bytes_g;
                const float* g0 = rec + (size_t)p * C * REC;
                if (ps.fmt == 0) {
                    float* f = (float*)blk;
                    for (int i = 0; i < C; ++i)
                        for (int k = 0; k < REC; ++k) f[(size_t)k * C + i] = g0[(size_t)i * REC + k];
                } else {
                    float* f = (float*)blk;
                    uint32_t* u = (uint32_t*)blk;
                    for (int i = 0; i < C; ++i) {
                        const float* g = g0 + (size_t)i * REC;
                        for (int k = 0; k < 3; ++k) f[(size_t)k * C + i] = g[k];
                        for (int k = 0; k < 4; ++k) {
                            const uint32_t lo16 = f32_to_f16(g[3 + 2 * k]), hi16 = f32_to_f16(g[4 + 2 * k]);
                            u[(size_t)(3 + k) * C + i] = lo16 | (hi16 << 16);
                        }
                        for (int m = 0; m < 24; ++m) {
                            const uint32_t lo16 = f32_to_bf16(g[11 + 2 * m]), hi16 = f32_to_bf16(g[12 + 2 * m]);
                            u[(size_t)(7 + m) * C + i] = lo16 | (hi16 << 16);
                        }
                    }
                }
            }
        });
    }
}

}  // namespace vm
