/*
 * CPU oracle for the particle-filter (sequential Monte Carlo) rigid
 * registration of 3D echo volumes (Uruththirakodeeswaran et al.,
 * arXiv 2504.19930).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code with the
 * HIP implementation; both follow the same written recipe.
 *
 * Plain, slow and direct: triple loops over voxels, one particle per OpenMP
 * iteration, FP64 everywhere except where the recipe fixes FP32 coordinates.
 * Compiled with -O2 -ffp-contract=off and no fast-math, so every floating
 * point operation below happens exactly as written.
 *
 * What each part follows:
 *   transform      Methods, Implementation Details: Euler 3D transform with
 *                  parameters (rx, ry, rz, tx, ty, tz) and the homogeneous
 *                  rigid matrix of Eq. 3.  Reading: R = Rz Rx Ry (ITK's Euler
 *                  3D default order), rotation about the target centre, the
 *                  map sends target points to source points (Eq. 1 compares
 *                  the target with the warped source).
 *   warp           Implementation Details: trilinear interpolation at
 *                  non-grid positions (images); nearest neighbour for masks.
 *   NCC            Eq. 2 (a squared correlation, range 0..1 as stated in the
 *                  Baseline and Evaluation Metrics subsection), summed over the
 *                  overlap.
 *   DSC            Eq. 4, over the full target grid (outside the source = 0).
 *   SSD            normalised mean squared difference over the overlap, using
 *                  the mean-0 / std-1 image normalisation of Implementation
 *                  Details (global statistics per volume).
 *   filter         Fig. 1 caption and Related Work: particles x^i, weights
 *                  w^i and measurements z^i; prediction, update, resampling and
 *                  estimation steps.  Readings: Gaussian likelihood of the score
 *                  deficit, systematic resampling every iteration, weighted-mean
 *                  estimate, annealed Gaussian random-walk prediction reflected
 *                  into the rotation / translation limits (Abstract).
 *   random numbers Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written
 *                  from the published round function and key schedule.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MI_BINS 32 /* joint-histogram bins per axis of the MI score */

/* Largest particle count.  Resampling sums q_i = floor(w_i 2^48) with
 * w_i <= 1 (the largest weight is exactly 1) in a uint64: the total stays
 * below 2^64 only for n < 2^16. */
#define OR_MAX_PARTICLES 65535u

/* ------------------------------------------------------------------ Philox */

/* Philox4x32-10: ten rounds of (two 32x32->64 multiplies, xor with the other
 * two words and the round key); the key is bumped by the Weyl constants
 * between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter layout: (index, iteration, pair, tag * 256 + block), key = seed. */
enum { OR_TAG_INIT = 0, OR_TAG_PERTURB = 1, OR_TAG_RESAMPLE = 2, OR_TAG_PROPOSAL = 3 };

static void draw(uint64_t seed, uint32_t index, uint32_t iter, uint32_t pair,
                 uint32_t tag, uint32_t block, uint32_t out[4])
{
    uint32_t ctr[4] = {index, iter, pair, tag * 256u + block};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in (0, 1] from two words: (27 high bits of a, 26 of b). */
double or_u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * 0x1p-53;
}

/* ------------------------------------------------------------------ volumes */

typedef struct {
    int32_t nx, ny, nz;
    double sx, sy, sz;
    const uint8_t *data; /* nz*ny*nx, x fastest */
    const uint8_t *fov;  /* same shape, nonzero = imaged; may be NULL */
} or_vol;

static inline size_t vidx(const or_vol *v, int i, int j, int k)
{
    return (size_t)i + (size_t)v->nx * ((size_t)j + (size_t)v->ny * (size_t)k);
}

/* ------------------------------------------------------------------ transform */

/* Elementary rotations about x, y, z (right-handed), row-major 3x3. */
static void rot_x(double a, double m[9])
{
    double c = cos(a), s = sin(a);
    double r[9] = {1, 0, 0, 0, c, -s, 0, s, c};
    memcpy(m, r, sizeof r);
}
static void rot_y(double a, double m[9])
{
    double c = cos(a), s = sin(a);
    double r[9] = {c, 0, s, 0, 1, 0, -s, 0, c};
    memcpy(m, r, sizeof r);
}
static void rot_z(double a, double m[9])
{
    double c = cos(a), s = sin(a);
    double r[9] = {c, -s, 0, s, c, 0, 0, 0, 1};
    memcpy(m, r, sizeof r);
}
/* C = A B, inner sums accumulated in index order from 0.0. */
static void matmul3(const double a[9], const double b[9], double c[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = acc;
        }
}

/* R = (Rz Rx) Ry for p = (rx, ry, rz, ...). */
void or_euler_R(const double p[6], double R[9])
{
    double rx[9], ry[9], rz[9], zx[9];
    rot_x(p[0], rx);
    rot_y(p[1], ry);
    rot_z(p[2], rz);
    matmul3(rz, rx, zx);
    matmul3(zx, ry, R);
}

/* ---- rotations as unit quaternions (w, x, y, z), for the wide-rotation mode */

/* Hamilton product a * b. */
static void quat_mul(const double a[4], const double b[4], double out[4])
{
    out[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    out[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    out[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    out[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* Quaternion of R = Rz(rz) Rx(rx) Ry(ry): qz * qx * qy, each elementary
 * rotation by angle a about axis e being (cos a/2, sin a/2 e). */
void or_euler_quat(const double p[6], double q[4])
{
    double qx[4] = {cos(0.5 * p[0]), sin(0.5 * p[0]), 0.0, 0.0};
    double qy[4] = {cos(0.5 * p[1]), 0.0, sin(0.5 * p[1]), 0.0};
    double qz[4] = {cos(0.5 * p[2]), 0.0, 0.0, sin(0.5 * p[2])};
    double zx[4];
    quat_mul(qz, qx, zx);
    quat_mul(zx, qy, q);
}

/* Rotation matrix (row major) of a unit quaternion. */
void or_quat_R(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Euler angles of R = Rz(rz) Rx(rx) Ry(ry).  Its bottom row is
 * (-cos rx sin ry, sin rx, cos rx cos ry) and its middle column
 * (-sin rz cos rx, cos rz cos rx, sin rx), so rx = asin(R21) in
 * [-pi/2, pi/2], ry = atan2(-R20, R22), rz = atan2(-R01, R11). */
void or_R_euler(const double R[9], double e[3])
{
    double s = R[7];
    if (s > 1.0) s = 1.0;
    if (s < -1.0) s = -1.0;
    e[0] = asin(s);
    e[1] = atan2(-R[6], R[8]);
    e[2] = atan2(-R[1], R[4]);
}

/* The angle equal to a modulo 2 pi in [c - pi, c + pi). */
static double wrap_near(double a, double c)
{
    const double two_pi = 6.283185307179586;
    double t = a - c + 3.141592653589793;
    return c + (t - two_pi * floor(t / two_pi)) - 3.141592653589793;
}

/* Target centre in mm: c_d = (0.5 * s_d) * (n_d - 1). */
static void centre(const int32_t n[3], const double s[3], double c[3])
{
    for (int d = 0; d < 3; ++d) c[d] = (0.5 * s[d]) * (double)(n[d] - 1);
}

/* Physical 3x4 map target mm -> source mm (Eq. 3 form): q = R p + (c + t - R c). */
void or_phys_matrix(const double p[6], const int32_t tn[3], const double ts[3], double M[12])
{
    double R[9], c[3];
    or_euler_R(p, R);
    centre(tn, ts, c);
    for (int d = 0; d < 3; ++d) {
        double rc = 0.0;
        for (int e = 0; e < 3; ++e) rc += R[3 * d + e] * c[e];
        for (int e = 0; e < 3; ++e) M[4 * d + e] = R[3 * d + e];
        M[4 * d + 3] = (c[d] + p[3 + d]) - rc;
    }
}

/* Voxel-unit affine u = A (i,j,k) + o, source voxel coordinates of target
 * voxel (i,j,k): A = diag(1/s_S) M3 diag(s_T), o = m / s_S; for nearest
 * neighbour o is shifted by +0.5 (round half up).  FP64. */
static void voxel_affine(const double M[12], const double ts[3], const double ss[3], int nn,
                         double A[9], double o[3])
{
    for (int d = 0; d < 3; ++d) {
        for (int e = 0; e < 3; ++e) A[3 * d + e] = (M[4 * d + e] * ts[e]) / ss[d];
        o[d] = M[4 * d + 3] / ss[d];
        if (nn) o[d] = o[d] + 0.5;
    }
}

/* The twelve FP32 "recipe words" (A row d, then o_d), rounded once. */
void or_recipe_words_from_matrix(const double M[12], const double ts[3], const double ss[3], int nn,
                                 float w[12])
{
    double A[9], o[3];
    voxel_affine(M, ts, ss, nn, A, o);
    for (int d = 0; d < 3; ++d) {
        for (int e = 0; e < 3; ++e) w[4 * d + e] = (float)A[3 * d + e];
        w[4 * d + 3] = (float)o[d];
    }
}

void or_recipe_words(const double p[6], const or_vol *src, const or_vol *tgt, int nn, float w[12])
{
    int32_t tn[3] = {tgt->nx, tgt->ny, tgt->nz};
    double ts[3] = {tgt->sx, tgt->sy, tgt->sz}, ss[3] = {src->sx, src->sy, src->sz};
    double M[12];
    or_phys_matrix(p, tn, ts, M);
    or_recipe_words_from_matrix(M, ts, ss, nn, w);
}

/* Recipe coordinate of target voxel (i,j,k), axis d:
 * u_d = fma(A_d2, k, fma(A_d1, j, fma(A_d0, i, o_d))) in FP32. */
static inline float recipe_u(const float w[12], int d, float fi, float fj, float fk)
{
    return fmaf(w[4 * d + 2], fk, fmaf(w[4 * d + 1], fj, fmaf(w[4 * d + 0], fi, w[4 * d + 3])));
}

/* ------------------------------------------------------------------ scoring */

/* Mask counts under nearest neighbour (recipe mode).  Over target voxels x in
 * the target FOV:
 *   n    = #{x : m(x) inside the source grid and its FOV}
 *   a    = #{x : ... and S[m] != 0}        (|warped S|)
 *   c    = #{x : ... and S[m] != 0 and T[x] != 0}   (|S n T|)
 *   b_ov = #{x : inside and T[x] != 0}
 * where m_d = floor(u_d) with u from the NN recipe words (o shifted by 0.5),
 * inside iff 0 <= u_d < n_d. */
void or_mask_counts(const or_vol *src, const or_vol *tgt, const float w[12], uint64_t out[4])
{
    uint64_t n = 0, a = 0, c = 0, b = 0;
    for (int k = 0; k < tgt->nz; ++k)
        for (int j = 0; j < tgt->ny; ++j)
            for (int i = 0; i < tgt->nx; ++i) {
                size_t ti = vidx(tgt, i, j, k);
                if (tgt->fov && tgt->fov[ti] == 0) continue;
                float u[3];
                for (int d = 0; d < 3; ++d) u[d] = recipe_u(w, d, (float)i, (float)j, (float)k);
                if (!(u[0] >= 0.0f && u[0] < (float)src->nx && u[1] >= 0.0f && u[1] < (float)src->ny &&
                      u[2] >= 0.0f && u[2] < (float)src->nz))
                    continue;
                int mi = (int)floorf(u[0]), mj = (int)floorf(u[1]), mk = (int)floorf(u[2]);
                size_t si = vidx(src, mi, mj, mk);
                if (src->fov && src->fov[si] == 0) continue;
                int s_on = src->data[si] != 0;
                int t_on = tgt->data[ti] != 0;
                n += 1;
                a += (uint64_t)s_on;
                c += (uint64_t)(s_on & t_on);
                b += (uint64_t)t_on;
            }
    out[0] = n; out[1] = a; out[2] = c; out[3] = b;
}

/* Linear interpolation as the recipe writes it: a + f (b - a) with one fused
 * multiply-add. */
static inline float lerpf_r(float a, float b, float f) { return fmaf(f, b - a, a); }

/* Image moments (recipe mode).  Over target voxels x in the target FOV whose
 * source position is inside, sums of n, s, t, s^2, t^2, s t with s the
 * interpolated source value in fixed point (8 fractional bits,
 * s_fx = floor(256 s + 0.5)) and t the target byte.  Trilinear: inside iff
 * 0 <= u_d <= n_d - 1 and all eight corners in the source FOV; corners
 * i0 = floor(u), i1 = min(i0 + 1, n - 1), f = u - i0, lerps along x, then y,
 * then z.  Nearest: as the mask rule, s_fx = 256 S[m]. */
/* The sampled source value at target voxel (i, j, k) in fixed point,
 * s_fx = floor(256 s + 0.5), and whether the sample is in the overlap:
 * trilinear inside iff 0 <= u <= n - 1 on every axis and the eight corners
 * in the source FOV; nearest (the words carry the +0.5 shift) inside iff
 * 0 <= u < n and the voxel in the source FOV. */
static int sample_fx(const or_vol *src, const float w[12], int trilinear, int i, int j, int k, uint64_t *sfx)
{
    float u[3];
    for (int d = 0; d < 3; ++d) u[d] = recipe_u(w, d, (float)i, (float)j, (float)k);
    if (trilinear) {
        if (!(u[0] >= 0.0f && u[0] <= (float)(src->nx - 1) && u[1] >= 0.0f &&
              u[1] <= (float)(src->ny - 1) && u[2] >= 0.0f && u[2] <= (float)(src->nz - 1)))
            return 0;
        int i0 = (int)floorf(u[0]), j0 = (int)floorf(u[1]), k0 = (int)floorf(u[2]);
        float fx = u[0] - (float)i0, fy = u[1] - (float)j0, fz = u[2] - (float)k0;
        int i1 = i0 + 1 < src->nx ? i0 + 1 : src->nx - 1;
        int j1 = j0 + 1 < src->ny ? j0 + 1 : src->ny - 1;
        int k1 = k0 + 1 < src->nz ? k0 + 1 : src->nz - 1;
        size_t c000 = vidx(src, i0, j0, k0), c100 = vidx(src, i1, j0, k0);
        size_t c010 = vidx(src, i0, j1, k0), c110 = vidx(src, i1, j1, k0);
        size_t c001 = vidx(src, i0, j0, k1), c101 = vidx(src, i1, j0, k1);
        size_t c011 = vidx(src, i0, j1, k1), c111 = vidx(src, i1, j1, k1);
        if (src->fov && !(src->fov[c000] && src->fov[c100] && src->fov[c010] && src->fov[c110] &&
                          src->fov[c001] && src->fov[c101] && src->fov[c011] && src->fov[c111]))
            return 0;
        const uint8_t *S = src->data;
        float x00 = lerpf_r((float)S[c000], (float)S[c100], fx);
        float x10 = lerpf_r((float)S[c010], (float)S[c110], fx);
        float x01 = lerpf_r((float)S[c001], (float)S[c101], fx);
        float x11 = lerpf_r((float)S[c011], (float)S[c111], fx);
        float y0 = lerpf_r(x00, x10, fy);
        float y1 = lerpf_r(x01, x11, fy);
        float s = lerpf_r(y0, y1, fz);
        *sfx = (uint64_t)floorf(s * 256.0f + 0.5f);
        return 1;
    }
    if (!(u[0] >= 0.0f && u[0] < (float)src->nx && u[1] >= 0.0f && u[1] < (float)src->ny && u[2] >= 0.0f &&
          u[2] < (float)src->nz))
        return 0;
    size_t si = vidx(src, (int)floorf(u[0]), (int)floorf(u[1]), (int)floorf(u[2]));
    if (src->fov && src->fov[si] == 0) return 0;
    *sfx = (uint64_t)src->data[si] * 256u;
    return 1;
}

void or_image_moments(const or_vol *src, const or_vol *tgt, const float w[12], int trilinear,
                      int64_t out[6])
{
    uint64_t n = 0, ss = 0, st = 0, sss = 0, stt = 0, sst = 0;
    for (int k = 0; k < tgt->nz; ++k)
        for (int j = 0; j < tgt->ny; ++j)
            for (int i = 0; i < tgt->nx; ++i) {
                size_t ti = vidx(tgt, i, j, k);
                if (tgt->fov && tgt->fov[ti] == 0) continue;
                uint64_t sfx;
                if (!sample_fx(src, w, trilinear, i, j, k, &sfx)) continue;
                uint64_t t = tgt->data[ti];
                n += 1;
                ss += sfx;
                st += t;
                sss += sfx * sfx;
                stt += t * t;
                sst += sfx * t;
            }
    out[0] = (int64_t)n; out[1] = (int64_t)ss; out[2] = (int64_t)st;
    out[3] = (int64_t)sss; out[4] = (int64_t)stt; out[5] = (int64_t)sst;
}

/* ---- mutual information (Related Work: the MI metric of landmark-free
 * echo registration).  Joint histogram of (source bin, target bin) over the
 * same overlap as the moments, OR_MI_BINS per axis: source bin s_fx >> 11
 * (s_fx <= 65280), target bin t >> 3.  Score: the symmetric uncertainty
 * 2 I(S;T) / (H(S) + H(T)) from the histogram's joint and marginal
 * frequencies, in [0, 1] and 1 for images equal up to a bijection of bins;
 * 0 when both marginal entropies vanish. ---- */

void or_joint_histogram(const or_vol *src, const or_vol *tgt, const float w[12], uint64_t *hist)
{
    memset(hist, 0, sizeof(uint64_t) * OR_MI_BINS * OR_MI_BINS);
    for (int k = 0; k < tgt->nz; ++k)
        for (int j = 0; j < tgt->ny; ++j)
            for (int i = 0; i < tgt->nx; ++i) {
                size_t ti = vidx(tgt, i, j, k);
                if (tgt->fov && tgt->fov[ti] == 0) continue;
                uint64_t sfx;
                if (!sample_fx(src, w, 1, i, j, k, &sfx)) continue;
                hist[(sfx >> 11) * OR_MI_BINS + (tgt->data[ti] >> 3)] += 1;
            }
}

/* Natural logarithm for the MI score, the same on every platform: x = m 2^e
 * with m in [sqrt(1/2), sqrt(2)), ln x = e ln 2 + 2 atanh(s), s = (m-1)/(m+1),
 * |s| <= 0.172, by the series 2 (s + s^3/3 + ... + s^25/25) (error below
 * 1e-20).  Written out so the score does not depend on the C library's log. */
double or_mi_log(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.7071067811865476) {
        m = m * 2.0;
        e = e - 1;
    }
    double s = (m - 1.0) / (m + 1.0), s2 = s * s, t = s, sum = s;
    for (int k = 3; k <= 25; k += 2) {
        t = t * s2;
        sum = sum + t / (double)k;
    }
    return (double)e * 0.6931471805599453 + 2.0 * sum;
}

double or_mi_score(const uint64_t *hist)
{
    uint64_t n = 0, ms[OR_MI_BINS] = {0}, mt[OR_MI_BINS] = {0};
    for (int a = 0; a < OR_MI_BINS; ++a)
        for (int b = 0; b < OR_MI_BINS; ++b) {
            uint64_t c = hist[a * OR_MI_BINS + b];
            n += c;
            ms[a] += c;
            mt[b] += c;
        }
    if (n == 0) return 0.0;
    double N = (double)n, hs = 0.0, ht = 0.0, hst = 0.0;
    for (int a = 0; a < OR_MI_BINS; ++a) {
        if (ms[a]) {
            double f = (double)ms[a] / N;
            hs = hs - f * or_mi_log(f);
        }
        if (mt[a]) {
            double f = (double)mt[a] / N;
            ht = ht - f * or_mi_log(f);
        }
    }
    for (int q = 0; q < OR_MI_BINS * OR_MI_BINS; ++q)
        if (hist[q]) {
            double f = (double)hist[q] / N;
            hst = hst - f * or_mi_log(f);
        }
    if (hs + ht <= 0.0) return 0.0;
    return 2.0 * (hs + ht - hst) / (hs + ht);
}

/* ---- FP64 mode: the same definitions with FP64 coordinates and values. ---- */

static void fp64_affine(const double p[6], const or_vol *src, const or_vol *tgt, double A[9], double o[3])
{
    int32_t tn[3] = {tgt->nx, tgt->ny, tgt->nz};
    double ts[3] = {tgt->sx, tgt->sy, tgt->sz}, ss[3] = {src->sx, src->sy, src->sz};
    double M[12];
    or_phys_matrix(p, tn, ts, M);
    voxel_affine(M, ts, ss, 0, A, o);
}

void or_mask_counts_fp64(const or_vol *src, const or_vol *tgt, const double p[6], uint64_t out[4])
{
    double A[9], o[3];
    fp64_affine(p, src, tgt, A, o);
    uint64_t n = 0, a = 0, c = 0, b = 0;
    for (int k = 0; k < tgt->nz; ++k)
        for (int j = 0; j < tgt->ny; ++j)
            for (int i = 0; i < tgt->nx; ++i) {
                size_t ti = vidx(tgt, i, j, k);
                if (tgt->fov && tgt->fov[ti] == 0) continue;
                double u[3];
                for (int d = 0; d < 3; ++d) u[d] = A[3 * d] * i + A[3 * d + 1] * j + A[3 * d + 2] * k + o[d];
                int m[3], inside = 1, nn[3] = {src->nx, src->ny, src->nz};
                for (int d = 0; d < 3; ++d) {
                    double r = floor(u[d] + 0.5);
                    if (!(r >= 0.0 && r < (double)nn[d])) inside = 0;
                    m[d] = inside ? (int)r : 0;
                }
                if (!inside) continue;
                size_t si = vidx(src, m[0], m[1], m[2]);
                if (src->fov && src->fov[si] == 0) continue;
                int s_on = src->data[si] != 0, t_on = tgt->data[ti] != 0;
                n += 1; a += (uint64_t)s_on; c += (uint64_t)(s_on & t_on); b += (uint64_t)t_on;
            }
    out[0] = n; out[1] = a; out[2] = c; out[3] = b;
}

/* Moments in intensity units (s not quantised), FP64 sums. */
void or_image_moments_fp64(const or_vol *src, const or_vol *tgt, const double p[6], int trilinear,
                           double out[6])
{
    double A[9], o[3];
    fp64_affine(p, src, tgt, A, o);
    double n = 0, ss = 0, st = 0, sss = 0, stt = 0, sst = 0;
    int nn[3] = {src->nx, src->ny, src->nz};
    for (int k = 0; k < tgt->nz; ++k)
        for (int j = 0; j < tgt->ny; ++j)
            for (int i = 0; i < tgt->nx; ++i) {
                size_t ti = vidx(tgt, i, j, k);
                if (tgt->fov && tgt->fov[ti] == 0) continue;
                double u[3];
                for (int d = 0; d < 3; ++d) u[d] = A[3 * d] * i + A[3 * d + 1] * j + A[3 * d + 2] * k + o[d];
                double s;
                if (trilinear) {
                    int ok = 1;
                    for (int d = 0; d < 3; ++d)
                        if (!(u[d] >= 0.0 && u[d] <= (double)(nn[d] - 1))) ok = 0;
                    if (!ok) continue;
                    int i0[3], i1[3];
                    double f[3];
                    for (int d = 0; d < 3; ++d) {
                        i0[d] = (int)floor(u[d]);
                        f[d] = u[d] - i0[d];
                        i1[d] = i0[d] + 1 < nn[d] ? i0[d] + 1 : nn[d] - 1;
                    }
                    double acc = 0.0;
                    int valid = 1;
                    for (int cz = 0; cz < 2; ++cz)
                        for (int cy = 0; cy < 2; ++cy)
                            for (int cx = 0; cx < 2; ++cx) {
                                size_t si = vidx(src, cx ? i1[0] : i0[0], cy ? i1[1] : i0[1], cz ? i1[2] : i0[2]);
                                if (src->fov && src->fov[si] == 0) valid = 0;
                                double wgt = (cx ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) *
                                             (cz ? f[2] : 1.0 - f[2]);
                                acc += wgt * (double)src->data[si];
                            }
                    if (!valid) continue;
                    s = acc;
                } else {
                    int m[3], inside = 1;
                    for (int d = 0; d < 3; ++d) {
                        double r = floor(u[d] + 0.5);
                        if (!(r >= 0.0 && r < (double)nn[d])) inside = 0;
                        m[d] = inside ? (int)r : 0;
                    }
                    if (!inside) continue;
                    size_t si = vidx(src, m[0], m[1], m[2]);
                    if (src->fov && src->fov[si] == 0) continue;
                    s = (double)src->data[si];
                }
                double t = (double)tgt->data[ti];
                n += 1; ss += s; st += t; sss += s * s; stt += t * t; sst += s * t;
            }
    out[0] = n; out[1] = ss; out[2] = st; out[3] = sss; out[4] = stt; out[5] = sst;
}

/* ------------------------------------------------------------------ scores */

/* Eq. 4: DSC = 2 |S n T| / (|S| + |T|); |T| = b over the whole target FOV.
 * An empty pair scores 0. */
double or_dice(uint64_t a, uint64_t c, uint64_t b_total)
{
    uint64_t den = a + b_total;
    if (den == 0) return 0.0;
    return (double)(2u * c) / (double)den;
}

/* Eq. 2 from moments (sums of s, t, s^2, t^2, s t over n voxels), any common
 * scale of s.  cov = Sst - Ss St / n, var_s = Sss - Ss^2 / n,
 * var_t = Stt - St^2 / n, NCC = cov^2 / (var_s var_t); fewer than two voxels or a
 * zero variance scores 0. */
double or_ncc_from_moments(const double m[6])
{
    double n = m[0], ss = m[1], st = m[2], sss = m[3], stt = m[4], sst = m[5];
    if (n < 2.0) return 0.0;
    double cov = sst - (ss * st) / n;
    double vs = sss - (ss * ss) / n;
    double vt = stt - (st * st) / n;
    if (!(vs > 0.0) || !(vt > 0.0)) return 0.0;
    return (cov * cov) / (vs * vt);
}

/* Normalised mean squared difference over the overlap, the images first
 * brought to mean 0 / std 1 with their global statistics (mu_s, sd_s),
 * (mu_t, sd_t).  Moments in intensity units.  Expanded:
 * sum((s - mu_s)/sd_s - (t - mu_t)/sd_t)^2
 *   = as^2 Sum(s - mu_s)^2 + at^2 Sum(t - mu_t)^2 - 2 as at Sum(s - mu_s)(t - mu_t). */
double or_msd_from_moments(const double m[6], double mu_s, double sd_s, double mu_t, double sd_t)
{
    double n = m[0], ss = m[1], st = m[2], sss = m[3], stt = m[4], sst = m[5];
    if (n < 1.0) return INFINITY;
    double as = 1.0 / sd_s, at = 1.0 / sd_t;
    double css = sss - 2.0 * mu_s * ss + n * mu_s * mu_s;
    double ctt = stt - 2.0 * mu_t * st + n * mu_t * mu_t;
    double cst = sst - mu_t * ss - mu_s * st + n * mu_s * mu_t;
    double tot = as * as * css + at * at * ctt - 2.0 * as * at * cst;
    return tot / n;
}

/* Fixed-point recipe moments to intensity-unit doubles: s = s_fx / 256. */
void or_moments_to_double(const int64_t mi[6], double m[6])
{
    m[0] = (double)mi[0];
    m[1] = (double)mi[1] / 256.0;
    m[2] = (double)mi[2];
    m[3] = (double)mi[3] / 65536.0;
    m[4] = (double)mi[4];
    m[5] = (double)mi[5] / 256.0;
}

/* ------------------------------------------------------------------ problem */

enum { OR_SCORE_DICE = 0, OR_SCORE_NCC = 1, OR_SCORE_SSD = 2, OR_SCORE_MI = 3 };

typedef struct {
    uint32_t n_particles, n_iters;
    uint64_t seed;
    uint32_t pair_id;
    int32_t score;      /* OR_SCORE_* */
    int32_t trilinear;  /* 1 trilinear, 0 nearest */
    int32_t fp64_mode;  /* 0 recipe (FP32 coordinates, exact integer moments), 1 FP64 */
    double x0[6], limit[6];
    double sigma_score;
    double sigma0[6];
    double anneal;
    double min_overlap_frac;
    /* learned proposal: prior from N(prop_mu, prop_sigma^2) truncated to the box */
    int32_t has_proposal;
    double prop_mu[6], prop_sigma[6];
    /* 1: wide rotations -- quaternion-mean estimate, and rotation axes whose
     * limit reaches pi wrap around the circle in the prediction */
    int32_t wide_rotation;
} or_params;

typedef struct {
    or_vol src, tgt;
    uint64_t t_on;       /* |T| over the target FOV */
    uint64_t t_fov;      /* number of target voxels in the FOV */
    double mu_s, sd_s, mu_t, sd_t;
} or_problem;

static void vol_stats(const or_vol *v, uint64_t *cnt, uint64_t *on, double *mu, double *sd)
{
    uint64_t n = 0, o = 0, s1 = 0, s2 = 0;
    size_t tot = (size_t)v->nx * v->ny * v->nz;
    for (size_t q = 0; q < tot; ++q) {
        if (v->fov && v->fov[q] == 0) continue;
        uint64_t x = v->data[q];
        n += 1; o += x != 0; s1 += x; s2 += x * x;
    }
    *cnt = n; *on = o;
    double dn = (double)n;
    double m = (double)s1 / dn;
    double var = (double)s2 / dn - m * m;
    *mu = m;
    *sd = var > 0.0 ? sqrt(var) : 1.0;
}

void or_problem_init(or_problem *pb, const or_vol *src, const or_vol *tgt)
{
    uint64_t c, o;
    pb->src = *src;
    pb->tgt = *tgt;
    vol_stats(tgt, &pb->t_fov, &pb->t_on, &pb->mu_t, &pb->sd_t);
    vol_stats(src, &c, &o, &pb->mu_s, &pb->sd_s);
}

/* Minimum overlap count for NCC / SSD: ceil(frac * |target FOV|). */
static uint64_t min_overlap(const or_problem *pb, const or_params *pr)
{
    return (uint64_t)ceil(pr->min_overlap_frac * (double)pb->t_fov);
}

/* Similarity z of one particle (higher is better): Dice, NCC, or -MSD.
 * Returns -inf where the overlap is below the minimum (NCC / SSD). */
double or_score_particle(const or_problem *pb, const or_params *pr, const double p[6])
{
    int nn = pr->score == OR_SCORE_DICE ? 1 : !pr->trilinear;
    if (pr->score == OR_SCORE_MI) {
        if (pr->fp64_mode || !pr->trilinear) return NAN;
        float w[12];
        uint64_t h[OR_MI_BINS * OR_MI_BINS], n = 0;
        or_recipe_words(p, &pb->src, &pb->tgt, 0, w);
        or_joint_histogram(&pb->src, &pb->tgt, w, h);
        for (int q = 0; q < OR_MI_BINS * OR_MI_BINS; ++q) n += h[q];
        if (n < min_overlap(pb, pr)) return -INFINITY;
        return or_mi_score(h);
    }
    if (pr->score == OR_SCORE_DICE) {
        uint64_t cnt[4];
        if (pr->fp64_mode) {
            or_mask_counts_fp64(&pb->src, &pb->tgt, p, cnt);
        } else {
            float w[12];
            or_recipe_words(p, &pb->src, &pb->tgt, 1, w);
            or_mask_counts(&pb->src, &pb->tgt, w, cnt);
        }
        return or_dice(cnt[1], cnt[2], pb->t_on);
    }
    double m[6];
    if (pr->fp64_mode) {
        or_image_moments_fp64(&pb->src, &pb->tgt, p, pr->trilinear, m);
    } else {
        float w[12];
        int64_t mi[6];
        or_recipe_words(p, &pb->src, &pb->tgt, nn, w);
        or_image_moments(&pb->src, &pb->tgt, w, pr->trilinear, mi);
        if ((uint64_t)mi[0] < min_overlap(pb, pr)) return -INFINITY;
        or_moments_to_double(mi, m);
        if (pr->score == OR_SCORE_NCC) return or_ncc_from_moments(m);
        return -or_msd_from_moments(m, pb->mu_s, pb->sd_s, pb->mu_t, pb->sd_t);
    }
    if ((uint64_t)m[0] < min_overlap(pb, pr)) return -INFINITY;
    if (pr->score == OR_SCORE_NCC) return or_ncc_from_moments(m);
    return -or_msd_from_moments(m, pb->mu_s, pb->sd_s, pb->mu_t, pb->sd_t);
}

/* ---- several frame pairs under one transform (multi-frame score): the
 * integer sums of every frame pair are added before the score is formed, so
 * Dice is 2 sum(a) / (sum(b) + sum(|T|)) and NCC is Eq. 2 over the union of
 * the overlaps.  Recipe mode; Dice and NCC (the normalised SSD keeps a
 * per-volume normalisation and is not pooled). */

/* Pooled sums of particle p over nf frame pairs: masks (n, a, c, b_overlap,
 * 0, 0), images the six moments. */
void or_frame_sums(const or_problem *pbs, uint32_t nf, const or_params *pr, const double p[6], int64_t out[6])
{
    for (int q = 0; q < 6; ++q) out[q] = 0;
    for (uint32_t f = 0; f < nf; ++f) {
        float w[12];
        if (pr->score == OR_SCORE_DICE) {
            uint64_t cnt[4];
            or_recipe_words(p, &pbs[f].src, &pbs[f].tgt, 1, w);
            or_mask_counts(&pbs[f].src, &pbs[f].tgt, w, cnt);
            for (int q = 0; q < 4; ++q) out[q] += (int64_t)cnt[q];
        } else {
            int64_t mi[6];
            or_recipe_words(p, &pbs[f].src, &pbs[f].tgt, !pr->trilinear, w);
            or_image_moments(&pbs[f].src, &pbs[f].tgt, w, pr->trilinear, mi);
            for (int q = 0; q < 6; ++q) out[q] += mi[q];
        }
    }
}

double or_score_particle_frames(const or_problem *pbs, uint32_t nf, const or_params *pr, const double p[6])
{
    if (nf == 1) return or_score_particle(pbs, pr, p);
    if (pr->score == OR_SCORE_SSD || pr->fp64_mode) return NAN;
    if (pr->score == OR_SCORE_MI) {
        uint64_t h[OR_MI_BINS * OR_MI_BINS], hf[OR_MI_BINS * OR_MI_BINS], n = 0, t_fov = 0;
        memset(h, 0, sizeof h);
        for (uint32_t f = 0; f < nf; ++f) {
            float w[12];
            or_recipe_words(p, &pbs[f].src, &pbs[f].tgt, 0, w);
            or_joint_histogram(&pbs[f].src, &pbs[f].tgt, w, hf);
            for (int q = 0; q < OR_MI_BINS * OR_MI_BINS; ++q) h[q] += hf[q];
            t_fov += pbs[f].t_fov;
        }
        for (int q = 0; q < OR_MI_BINS * OR_MI_BINS; ++q) n += h[q];
        if (n < (uint64_t)ceil(pr->min_overlap_frac * (double)t_fov)) return -INFINITY;
        return or_mi_score(h);
    }
    int64_t m[6];
    or_frame_sums(pbs, nf, pr, p, m);
    if (pr->score == OR_SCORE_DICE) {
        uint64_t t_on = 0;
        for (uint32_t f = 0; f < nf; ++f) t_on += pbs[f].t_on;
        return or_dice((uint64_t)m[1], (uint64_t)m[2], t_on);
    }
    uint64_t t_fov = 0;
    for (uint32_t f = 0; f < nf; ++f) t_fov += pbs[f].t_fov;
    if ((uint64_t)m[0] < (uint64_t)ceil(pr->min_overlap_frac * (double)t_fov)) return -INFINITY;
    double md[6];
    or_moments_to_double(m, md);
    return or_ncc_from_moments(md);
}

/* ------------------------------------------------------------------ filter */

/* Measurement update: log-likelihood of score z, a Gaussian in the deficit
 * from the ideal score (1 for Dice and NCC, 0 for -MSD). */
double or_loglik(double z, int score, double sigma)
{
    if (z == -INFINITY) return -INFINITY;
    double zmax = score == OR_SCORE_SSD ? 0.0 : 1.0;
    double d = zmax - z;
    return -(d * d) * (0.5 / (sigma * sigma));
}

/* Normalisation and estimate: w_i = exp(lw_i - max lw); ESS = (sum w)^2 / sum w^2;
 * estimate = sum w_i x_i / sum w_i.  All weights -inf: uniform, flagged. */
int or_normalise(uint32_t n, const double *lw, const double *x, double *w, double est[6], double *ess)
{
    double mx = -INFINITY;
    for (uint32_t i = 0; i < n; ++i)
        if (lw[i] > mx) mx = lw[i];
    int degenerate = mx == -INFINITY;
    for (uint32_t i = 0; i < n; ++i) w[i] = degenerate ? 1.0 : exp(lw[i] - mx);
    double s = 0.0, s2 = 0.0, acc[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t i = 0; i < n; ++i) {
        s += w[i];
        s2 += w[i] * w[i];
        for (int d = 0; d < 6; ++d) acc[d] += w[i] * x[6 * (size_t)i + d];
    }
    for (int d = 0; d < 6; ++d) est[d] = acc[d] / s;
    *ess = (s * s) / s2;
    return degenerate;
}

/* Label of the learned proposal (the target's addition, no paper passage):
 * the weighted particle cloud summarised by its weighted mean and per-axis
 * weighted variance, with the normalised weights of or_normalise, written in
 * units of the limits about x0 -- mean (xbar - x0) / L, variance Var / L^2,
 * floored at var_floor. */
void or_cloud_moments(uint32_t n, const double *lw, const double *x, const double x0[6], const double limit[6],
                      double var_floor, double mean[6], double var[6])
{
    double mx = -INFINITY;
    for (uint32_t i = 0; i < n; ++i)
        if (lw[i] > mx) mx = lw[i];
    int flat = mx == -INFINITY;
    double s = 0.0, xbar[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t i = 0; i < n; ++i) {
        double w = flat ? 1.0 : exp(lw[i] - mx);
        s += w;
        for (int d = 0; d < 6; ++d) xbar[d] += w * x[6 * (size_t)i + d];
    }
    for (int d = 0; d < 6; ++d) xbar[d] = xbar[d] / s;
    double dev[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t i = 0; i < n; ++i) {
        double w = flat ? 1.0 : exp(lw[i] - mx);
        for (int d = 0; d < 6; ++d) {
            double e = x[6 * (size_t)i + d] - xbar[d];
            dev[d] += w * e * e;
        }
    }
    for (int d = 0; d < 6; ++d) {
        mean[d] = (xbar[d] - x0[d]) / limit[d];
        double v = dev[d] / s / (limit[d] * limit[d]);
        var[d] = v > var_floor ? v : var_floor;
    }
}

/* The proposal the network's outputs stand for (the target's addition): the
 * outputs are a Gaussian in units of the limits about x0; the mean is clipped
 * to the box, the log-variance to [-20, 2], and the variance widened by
 * var_scale before it is turned back into radians / mm. */
void or_proposal_from_network(const float out[12], const double x0[6], const double limit[6], double var_scale,
                              double mean[6], double logvar[6])
{
    for (int d = 0; d < 6; ++d) {
        double u = (double)out[d], l = (double)out[6 + d];
        if (u < -1.0) u = -1.0;
        if (u > 1.0) u = 1.0;
        if (l < -20.0) l = -20.0;
        if (l > 2.0) l = 2.0;
        mean[d] = x0[d] + u * limit[d];
        logvar[d] = l + 2.0 * log(limit[d]) + log(var_scale);
    }
}

/* Normalisation as or_normalise, with the rotation of the estimate taken
 * from unit quaternions (wide-rotation mode): the particle quaternions are
 * put on the hemisphere of the first particle of largest log-weight, summed
 * with their weights and normalised (the weighted chordal mean to first order
 * in the spread, independent of how angles wrap); the Euler angles of that
 * rotation are then moved by whole turns to lie within pi of x0. */
int or_normalise_wide(uint32_t n, const double *lw, const double *x, const double x0[6], double *w, double est[6],
                      double *ess)
{
    int degenerate = or_normalise(n, lw, x, w, est, ess);
    double mx = -INFINITY;
    uint32_t ref = 0;
    for (uint32_t i = 0; i < n; ++i)
        if (lw[i] > mx) {
            mx = lw[i];
            ref = i;
        }
    double qr[4], acc[4] = {0.0, 0.0, 0.0, 0.0};
    or_euler_quat(x + 6 * (size_t)ref, qr);
    for (uint32_t i = 0; i < n; ++i) {
        double q[4];
        or_euler_quat(x + 6 * (size_t)i, q);
        double dot = q[0] * qr[0] + q[1] * qr[1] + q[2] * qr[2] + q[3] * qr[3];
        double sgn = dot < 0.0 ? -1.0 : 1.0;
        for (int c = 0; c < 4; ++c) acc[c] += (w[i] * sgn) * q[c];
    }
    double nrm = sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2] + acc[3] * acc[3]);
    double q[4], R[9], e[3];
    for (int c = 0; c < 4; ++c) q[c] = acc[c] / nrm;
    or_quat_R(q, R);
    or_R_euler(R, e);
    for (int d = 0; d < 3; ++d) est[d] = wrap_near(e[d], x0[d]);
    return degenerate;
}

/* Systematic resampling on an exact integer CDF.  q_i = floor(w_i 2^48),
 * Q = sum q_i, C_i the inclusive prefix sums; with one uniform word U the
 * j-th pointer is (j + U / 2^32) Q / N and the ancestor of j is the first i
 * whose C_i exceeds it, i.e. C_i N 2^32 > (j 2^32 + U) Q (128-bit exact). */
int or_resample(uint32_t n, const double *w, uint32_t u32, int32_t *anc)
{
    if (n < 1 || n > OR_MAX_PARTICLES) return -1;
    uint64_t *cdf = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t run = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t q = (uint64_t)floor(w[i] * 0x1p48);
        run += q;
        cdf[i] = run;
    }
    unsigned __int128 Q = run;
    unsigned __int128 scale = (unsigned __int128)n << 32;
    uint32_t i = 0;
    for (uint32_t j = 0; j < n; ++j) {
        unsigned __int128 rhs = ((((unsigned __int128)j) << 32) + u32) * Q;
        while (!((unsigned __int128)cdf[i] * scale > rhs)) ++i;
        anc[j] = (int32_t)i;
    }
    free(cdf);
    return 0;
}

/* Reflect once at the limits box, then clamp. */
static double reflect(double v, double lo, double hi)
{
    if (v < lo) v = lo + (lo - v);
    if (v > hi) v = hi - (v - hi);
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* Six standard normals for particle j at iteration k (Box-Muller on three
 * Philox blocks, two 53-bit uniforms each). */
void or_gauss6(uint64_t seed, uint32_t pair, uint32_t j, uint32_t k, double g[6])
{
    for (uint32_t b = 0; b < 3; ++b) {
        uint32_t r[4];
        draw(seed, j, k, pair, OR_TAG_PERTURB, b, r);
        double u1 = or_u53(r[0], r[1]), u2 = or_u53(r[2], r[3]);
        double rad = sqrt(-2.0 * log(u1));
        double th = 6.283185307179586 * u2;
        g[2 * b] = rad * cos(th);
        g[2 * b + 1] = rad * sin(th);
    }
}

/* Random-walk width after evaluation k (k >= 1): sigma0 * anneal^(k-1),
 * by repeated multiplication. */
static double sigma_k(const or_params *pr, int d, uint32_t k)
{
    double s = pr->sigma0[d];
    for (uint32_t m = 1; m < k; ++m) s = s * pr->anneal;
    return s;
}

/* Prediction: x_j = reflect(x_{a_j} + sigma_k g_j); in the wide-rotation mode
 * a rotation axis whose limit reaches pi wraps into [x0 - pi, x0 + pi)
 * instead (the box is then the whole circle). */
void or_perturb(const or_params *pr, uint32_t k, const double *x_old, const int32_t *anc, double *x_new)
{
    double lo[6], hi[6], sg[6];
    for (int d = 0; d < 6; ++d) {
        lo[d] = pr->x0[d] - pr->limit[d];
        hi[d] = pr->x0[d] + pr->limit[d];
        sg[d] = sigma_k(pr, d, k);
    }
    for (uint32_t j = 0; j < pr->n_particles; ++j) {
        double g[6];
        or_gauss6(pr->seed, pr->pair_id, j, k, g);
        for (int d = 0; d < 6; ++d) {
            double v = x_old[6 * (size_t)anc[j] + d] + sg[d] * g[d];
            if (pr->wide_rotation && d < 3 && pr->limit[d] >= 3.141592653589793)
                x_new[6 * (size_t)j + d] = wrap_near(v, pr->x0[d]);
            else
                x_new[6 * (size_t)j + d] = reflect(v, lo[d], hi[d]);
        }
    }
}

/* Proposal draw: per axis, the first of 16 tries mu + sigma g (g from
 * Box-Muller on Philox tag 3, counter word 1 = try) that lands in the box, or
 * mu clamped to the box; lq_i = sum_d ((x_d - mu_d) / sigma_d)^2 / 2, i.e.
 * -log q(x_i) up to a constant (the truncated Gaussian's normaliser). */
static void init_proposal(const or_params *pr, double *x, double *lq)
{
    for (uint32_t i = 0; i < pr->n_particles; ++i) {
        double p[6];
        int done[6] = {0, 0, 0, 0, 0, 0};
        for (int d = 0; d < 6; ++d) {
            double lo = pr->x0[d] - pr->limit[d], hi = pr->x0[d] + pr->limit[d];
            p[d] = fmin(fmax(pr->prop_mu[d], lo), hi);
        }
        for (uint32_t t = 0; t < 16; ++t) {
            double g[6];
            for (uint32_t b = 0; b < 3; ++b) {
                uint32_t r[4];
                draw(pr->seed, i, t, pr->pair_id, OR_TAG_PROPOSAL, b, r);
                double u1 = or_u53(r[0], r[1]), u2 = or_u53(r[2], r[3]);
                double rad = sqrt(-2.0 * log(u1));
                double th = 6.283185307179586 * u2;
                g[2 * b] = rad * cos(th);
                g[2 * b + 1] = rad * sin(th);
            }
            for (int d = 0; d < 6; ++d) {
                double lo = pr->x0[d] - pr->limit[d], hi = pr->x0[d] + pr->limit[d];
                double v = pr->prop_mu[d] + pr->prop_sigma[d] * g[d];
                if (!done[d] && v >= lo && v <= hi) {
                    p[d] = v;
                    done[d] = 1;
                }
            }
        }
        double q = 0.0;
        for (int d = 0; d < 6; ++d) {
            double z = (p[d] - pr->prop_mu[d]) / pr->prop_sigma[d];
            q += 0.5 * (z * z);
        }
        lq[i] = q;
        memcpy(x + 6 * (size_t)i, p, sizeof p);
    }
}

/* Prior draw: x_i = x0 + L (2u - 1), u from Philox tag 0. */
void or_init_particles(const or_params *pr, double *x)
{
    for (uint32_t i = 0; i < pr->n_particles; ++i)
        for (uint32_t b = 0; b < 3; ++b) {
            uint32_t r[4];
            draw(pr->seed, i, 0, pr->pair_id, OR_TAG_INIT, b, r);
            double ua = or_u53(r[0], r[1]), ub = or_u53(r[2], r[3]);
            int d0 = 2 * b, d1 = 2 * b + 1;
            x[6 * (size_t)i + d0] = pr->x0[d0] + pr->limit[d0] * (2.0 * ua - 1.0);
            x[6 * (size_t)i + d1] = pr->x0[d1] + pr->limit[d1] * (2.0 * ub - 1.0);
        }
}

void or_init_proposal(const or_params *pr, double *x, double *lq) { init_proposal(pr, x, lq); }

uint32_t or_resample_word(const or_params *pr, uint32_t k)
{
    uint32_t r[4];
    draw(pr->seed, 0, k, pr->pair_id, OR_TAG_RESAMPLE, 0, r);
    return r[0];
}

/* Score a set of particles (one OpenMP iteration per particle). */
void or_score_particles(const or_problem *pb, const or_params *pr, uint32_t n, const double *x, double *z)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < (int64_t)n; ++i) z[i] = or_score_particle(pb, pr, x + 6 * i);
}

/* One filter update after the scores of iteration k are known:
 * weights -> normalise / estimate -> (k < K) resample and predict. */
int or_filter_update(const or_params *pr, uint32_t k, const double *x, const double *z, const double *lq,
                     double *lw, double *w, double est[6], double *ess, int32_t *anc, double *x_next)
{
    uint32_t n = pr->n_particles;
    if (n < 1 || n > OR_MAX_PARTICLES) return -1;
    for (uint32_t i = 0; i < n; ++i) {
        lw[i] = or_loglik(z[i], pr->score, pr->sigma_score);
        /* importance correction of the proposal draw: log p - log q, p uniform */
        if (k == 1 && pr->has_proposal && lq) lw[i] = lw[i] + lq[i];
    }
    int degen = pr->wide_rotation ? or_normalise_wide(n, lw, x, pr->x0, w, est, ess)
                                  : or_normalise(n, lw, x, w, est, ess);
    if (k < pr->n_iters) {
        or_resample(n, w, or_resample_word(pr, k), anc);
        or_perturb(pr, k, x, anc, x_next);
    }
    return degen;
}

/* Whole registration over nf frame pairs scored together (nf = 1: one pair).
 * trace_score has K + 1 entries: the score of the estimate before iteration 1
 * (x0) and after each iteration; trace_ess and trace_est (6 per iteration)
 * have K.  x_out receives the final particle set, lw_out its log-weights,
 * anc_out the last ancestors (or -1). */
int or_smc_run_frames(const or_vol *srcs, const or_vol *tgts, uint32_t nf, const or_params *pr,
                      double est_out[6], double *trace_score, double *trace_ess, double *trace_est, double *x_out,
                      double *lw_out, int32_t *anc_out)
{
    uint32_t n = pr->n_particles;
    if (n < 1 || n > OR_MAX_PARTICLES) return -1;
    or_problem *pbs = (or_problem *)malloc(sizeof(or_problem) * nf);
    for (uint32_t f = 0; f < nf; ++f) or_problem_init(&pbs[f], &srcs[f], &tgts[f]);
    double *x = (double *)malloc(sizeof(double) * 6 * n);
    double *xn = (double *)malloc(sizeof(double) * 6 * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *lw = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * n);
    double *lq = (double *)calloc(n, sizeof(double));
    for (uint32_t i = 0; i < n; ++i) anc[i] = -1;
    double est[6];
    memcpy(est, pr->x0, sizeof est);
    int degen_any = 0;
    if (pr->has_proposal) init_proposal(pr, x, lq);
    else or_init_particles(pr, x);
    for (uint32_t k = 1; k <= pr->n_iters; ++k) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < (int64_t)n; ++i) z[i] = or_score_particle_frames(pbs, nf, pr, x + 6 * i);
        if (trace_score) trace_score[k - 1] = or_score_particle_frames(pbs, nf, pr, est);
        double ess;
        degen_any |= or_filter_update(pr, k, x, z, lq, lw, w, est, &ess, anc, xn);
        if (trace_ess) trace_ess[k - 1] = ess;
        if (trace_est) memcpy(trace_est + 6 * (k - 1), est, sizeof est);
        if (k < pr->n_iters) {
            double *t = x; x = xn; xn = t;
        }
    }
    if (trace_score) trace_score[pr->n_iters] = or_score_particle_frames(pbs, nf, pr, est);
    memcpy(est_out, est, sizeof est);
    if (x_out) memcpy(x_out, x, sizeof(double) * 6 * n);
    if (lw_out) memcpy(lw_out, lw, sizeof(double) * n);
    if (anc_out) memcpy(anc_out, anc, sizeof(int32_t) * n);
    free(x); free(xn); free(z); free(lw); free(w); free(anc); free(lq); free(pbs);
    return degen_any;
}

int or_smc_run(const or_vol *src, const or_vol *tgt, const or_params *pr, double est_out[6],
               double *trace_score, double *trace_ess, double *trace_est, double *x_out, double *lw_out,
               int32_t *anc_out)
{
    return or_smc_run_frames(src, tgt, 1, pr, est_out, trace_score, trace_ess, trace_est, x_out, lw_out, anc_out);
}

/* ------------------------------------------------------------------ warp apply */

/* Apply a physical 3x4 map (target mm -> source mm) to a source volume,
 * producing a volume on the target grid: nearest (the source byte) or
 * trilinear (floor(s + 0.5) clamped to 0..255); outside -> 0. */
void or_warp_apply(const or_vol *src, const double M[12], int trilinear, uint8_t *dst, int32_t nx, int32_t ny,
                   int32_t nz, double sx, double sy, double sz)
{
    double ts[3] = {sx, sy, sz}, ss[3] = {src->sx, src->sy, src->sz};
    float w[12];
    or_recipe_words_from_matrix(M, ts, ss, !trilinear, w);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t di = (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * (size_t)k);
                float u[3];
                for (int d = 0; d < 3; ++d) u[d] = recipe_u(w, d, (float)i, (float)j, (float)k);
                uint8_t val = 0;
                if (!trilinear) {
                    if (u[0] >= 0.0f && u[0] < (float)src->nx && u[1] >= 0.0f && u[1] < (float)src->ny &&
                        u[2] >= 0.0f && u[2] < (float)src->nz)
                        val = src->data[vidx(src, (int)floorf(u[0]), (int)floorf(u[1]), (int)floorf(u[2]))];
                } else if (u[0] >= 0.0f && u[0] <= (float)(src->nx - 1) && u[1] >= 0.0f &&
                           u[1] <= (float)(src->ny - 1) && u[2] >= 0.0f && u[2] <= (float)(src->nz - 1)) {
                    int i0 = (int)floorf(u[0]), j0 = (int)floorf(u[1]), k0 = (int)floorf(u[2]);
                    float fx = u[0] - (float)i0, fy = u[1] - (float)j0, fz = u[2] - (float)k0;
                    int i1 = i0 + 1 < src->nx ? i0 + 1 : src->nx - 1;
                    int j1 = j0 + 1 < src->ny ? j0 + 1 : src->ny - 1;
                    int k1 = k0 + 1 < src->nz ? k0 + 1 : src->nz - 1;
                    const uint8_t *S = src->data;
                    float x00 = lerpf_r((float)S[vidx(src, i0, j0, k0)], (float)S[vidx(src, i1, j0, k0)], fx);
                    float x10 = lerpf_r((float)S[vidx(src, i0, j1, k0)], (float)S[vidx(src, i1, j1, k0)], fx);
                    float x01 = lerpf_r((float)S[vidx(src, i0, j0, k1)], (float)S[vidx(src, i1, j0, k1)], fx);
                    float x11 = lerpf_r((float)S[vidx(src, i0, j1, k1)], (float)S[vidx(src, i1, j1, k1)], fx);
                    float s = lerpf_r(lerpf_r(x00, x10, fy), lerpf_r(x01, x11, fy), fz);
                    float r = floorf(s + 0.5f);
                    val = (uint8_t)(r > 255.0f ? 255.0f : r);
                }
                dst[di] = val;
            }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel loops (n < 1: all processors). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}
