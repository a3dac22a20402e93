// Shared device / host helpers of the registration library: counter-based
// random numbers, the rigid transform and its FP32 coordinate recipe, and the
// score / likelihood finalisation from exact integer sums.
//
// Every routine here runs with floating-point contraction disabled
// (-ffp-contract=off for the whole library); fused multiply-adds appear only
// where written explicitly, so the results are reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#define SMC_HD __host__ __device__ __forceinline__

namespace smc {

constexpr int kTagInit = 0;
constexpr int kTagPerturb = 1;
constexpr int kTagResample = 2;
constexpr int kTagProposal = 3;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products whose halves are xor-ed with the other two words and the
// round key; the key advances by the Weyl constants between rounds.
SMC_HD void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                          uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Counter (index, iteration, pair, tag * 256 + block) under key = seed.
SMC_HD void draw4(uint64_t seed, uint32_t index, uint32_t iter, uint32_t pair, uint32_t tag, uint32_t block,
                  uint32_t out[4]) {
    philox4x32_10(index, iter, pair, tag * 256u + block, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

// Uniform in (0, 1]: 27 bits of a over 26 bits of b, centred in its cell.
SMC_HD double uniform53(uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * 0x1p-53;
}

// ---------------------------------------------------------------- transform

struct Geom {
    int32_t tn[3];     // target voxels
    double ts[3];      // target spacing (mm)
    double ss[3];      // source spacing (mm)
};

SMC_HD void mat3_mul(const double a[9], const double b[9], double c[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = acc;
        }
}

// Euler 3D rotation, R = (Rz Rx) Ry, right-handed elementary rotations.
SMC_HD void euler_rotation(const double p[6], double R[9]) {
    const double cx = cos(p[0]), sx = sin(p[0]);
    const double cy = cos(p[1]), sy = sin(p[1]);
    const double cz = cos(p[2]), sz = sin(p[2]);
    const double rx[9] = {1.0, 0.0, 0.0, 0.0, cx, -sx, 0.0, sx, cx};
    const double ry[9] = {cy, 0.0, sy, 0.0, 1.0, 0.0, -sy, 0.0, cy};
    const double rz[9] = {cz, -sz, 0.0, sz, cz, 0.0, 0.0, 0.0, 1.0};
    double zx[9];
    mat3_mul(rz, rx, zx);
    mat3_mul(zx, ry, R);
}

// 3x4 target-mm -> source-mm map q = R p + (c + t - R c), c the target centre.
SMC_HD void rigid_matrix(const double p[6], const Geom &g, double M[12]) {
    double R[9];
    euler_rotation(p, R);
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = (0.5 * g.ts[d]) * (double)(g.tn[d] - 1);
    for (int d = 0; d < 3; ++d) {
        double rc = 0.0;
        for (int e = 0; e < 3; ++e) rc += R[3 * d + e] * c[e];
        for (int e = 0; e < 3; ++e) M[4 * d + e] = R[3 * d + e];
        M[4 * d + 3] = (c[d] + p[3 + d]) - rc;
    }
}

// The twelve FP32 recipe words of a physical map: the voxel-unit affine
// A = diag(1/s_S) M diag(s_T), o = m / s_S (+0.5 for nearest neighbour),
// computed in FP64 and rounded once.  Row d holds (A_d0, A_d1, A_d2, o_d).
SMC_HD void words_from_matrix(const double M[12], const double ts[3], const double ss[3], bool nearest,
                              float w[12]) {
    for (int d = 0; d < 3; ++d) {
        for (int e = 0; e < 3; ++e) w[4 * d + e] = (float)((M[4 * d + e] * ts[e]) / ss[d]);
        double o = M[4 * d + 3] / ss[d];
        if (nearest) o = o + 0.5;
        // + 0.0f turns a -0 offset into +0: the sign of a zero coordinate
        // changes no result, and the score kernels test "inside" on the bit
        // patterns of non-negative coordinates
        w[4 * d + 3] = (float)o + 0.0f;
    }
}

SMC_HD void particle_words(const double p[6], const Geom &g, bool nearest, float w[12]) {
    double M[12];
    rigid_matrix(p, g, M);
    words_from_matrix(M, g.ts, g.ss, nearest, w);
}

// ---------------------------------------------------------------- scores

enum ScoreKind : int32_t { kDice = 0, kNcc = 1, kSsd = 2, kMi = 3 };

// Mutual information: joint-histogram bins per axis (source bin s_fx >> 11,
// target bin t >> 3).  The finalised sums of an MI particle are
// (overlap count, bits of the score as a double, 0, 0, 0, 0).
constexpr int kMiBins = 32;

struct ScoreConst {
    int32_t kind;
    uint64_t t_on;      // |T| inside the target FOV (Dice)
    uint64_t min_n;     // minimum overlap count (NCC / SSD)
    double mu_s, sd_s;  // global source statistics (SSD)
    double mu_t, sd_t;  // global target statistics (SSD)
    double sigma;       // likelihood width
};

// Similarity z (higher is better) of one particle from its exact sums;
// -inf when an NCC / SSD overlap is below the minimum.
SMC_HD double score_from_sums(const int64_t m[6], const ScoreConst &sc) {
    if (sc.kind == kMi) {
        if ((uint64_t)m[0] < sc.min_n) return -INFINITY;
        double z;
        memcpy(&z, &m[1], sizeof z);
        return z;
    }
    if (sc.kind == kDice) {
        const uint64_t a = (uint64_t)m[1], c = (uint64_t)m[2];
        const uint64_t den = a + sc.t_on;
        if (den == 0) return 0.0;
        return (double)(2u * c) / (double)den;
    }
    if ((uint64_t)m[0] < sc.min_n) return -INFINITY;
    const double n = (double)m[0];
    const double ss = (double)m[1] / 256.0;
    const double st = (double)m[2];
    const double sss = (double)m[3] / 65536.0;
    const double stt = (double)m[4];
    const double sst = (double)m[5] / 256.0;
    if (sc.kind == kNcc) {
        if (n < 2.0) return 0.0;
        const double cov = sst - (ss * st) / n;
        const double vs = sss - (ss * ss) / n;
        const double vt = stt - (st * st) / n;
        if (!(vs > 0.0) || !(vt > 0.0)) return 0.0;
        return (cov * cov) / (vs * vt);
    }
    // SSD of mean-0 / std-1 normalised images over the overlap, negated
    if (n < 1.0) return -INFINITY;
    const double as = 1.0 / sc.sd_s, at = 1.0 / sc.sd_t;
    const double mu_s = sc.mu_s, mu_t = sc.mu_t;
    const double css = sss - 2.0 * mu_s * ss + n * mu_s * mu_s;
    const double ctt = stt - 2.0 * mu_t * st + n * mu_t * mu_t;
    const double cst = sst - mu_t * ss - mu_s * st + n * mu_s * mu_t;
    const double tot = as * as * css + at * at * ctt - 2.0 * as * at * cst;
    return -(tot / n);
}

// Natural logarithm used by the MI score, identical on host and device: with
// x = m 2^e, m in [sqrt(1/2), sqrt(2)), ln x = e ln 2 + 2 atanh(s) for
// s = (m - 1) / (m + 1), the atanh series summed to the s^25 term (|s| <=
// 0.172, error below 1e-20).  Library logarithms differ between platforms in
// the last bit, which could move an integer resampling step.
SMC_HD double mi_log(double x) {
    int e;
    double m = frexp(x, &e);
    if (m < 0.7071067811865476) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
    double t = s, acc = s;
    for (int k = 3; k <= 25; k += 2) {
        t = t * s2;
        acc = acc + t / (double)k;
    }
    return (double)e * 0.6931471805599453 + 2.0 * acc;
}

// Measurement update: Gaussian in the deficit from the ideal score.
SMC_HD double log_likelihood(double z, const ScoreConst &sc) {
    if (z == -INFINITY) return -INFINITY;
    const double zmax = sc.kind == kSsd ? 0.0 : 1.0;
    const double d = zmax - z;
    return -(d * d) * (0.5 / (sc.sigma * sc.sigma));
}

// ---- wide rotations: unit quaternions (w, x, y, z)

// Quaternion of R = Rz(p2) Rx(p0) Ry(p1): the product of the half-angle
// quaternions qz qx qy, written out (qz qx has no zero component).
SMC_HD void rotation_quaternion(const double p[6], double q[4]) {
    const double ca = cos(0.5 * p[0]), sa = sin(0.5 * p[0]);
    const double cb = cos(0.5 * p[1]), sb = sin(0.5 * p[1]);
    const double cc = cos(0.5 * p[2]), sc = sin(0.5 * p[2]);
    const double zx[4] = {cc * ca, cc * sa, sc * sa, sc * ca};
    q[0] = zx[0] * cb - zx[2] * sb;
    q[1] = zx[1] * cb - zx[3] * sb;
    q[2] = zx[0] * sb + zx[2] * cb;
    q[3] = zx[1] * sb + zx[3] * cb;
}

// Euler angles (p0, p1, p2) of the rotation of a unit quaternion, for
// R = Rz(p2) Rx(p0) Ry(p1): p0 = asin(R21), p1 = atan2(-R20, R22),
// p2 = atan2(-R01, R11), from the entries of the quaternion's matrix.
SMC_HD void quaternion_euler(const double q[4], double e[3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double r01 = 2.0 * (x * y - w * z), r11 = 1.0 - 2.0 * (x * x + z * z);
    const double r20 = 2.0 * (x * z - w * y), r21 = 2.0 * (y * z + w * x), r22 = 1.0 - 2.0 * (x * x + y * y);
    e[0] = asin(fmin(1.0, fmax(-1.0, r21)));
    e[1] = atan2(-r20, r22);
    e[2] = atan2(-r01, r11);
}

// a moved by whole turns into [c - pi, c + pi)
SMC_HD double wrap_near(double a, double c) {
    const double pi = 3.141592653589793, turn = 6.283185307179586;
    const double t = a - c + pi;
    return c + (t - turn * floor(t / turn)) - pi;
}

SMC_HD double reflect_into(double v, double lo, double hi) {
    if (v < lo) v = lo + (lo - v);
    if (v > hi) v = hi - (v - hi);
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

}  // namespace smc
