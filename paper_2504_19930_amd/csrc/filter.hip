// Particle-filter kernels (Fig. 1): prior draw, and the per-iteration update
// -> normalise / estimate -> systematic resampling -> prediction, fused into
// one 1024-thread workgroup per registration pair.
//
// Determinism: log-weights come from exact integer sums; the resampling CDF
// is an exact 64-bit integer prefix sum of q_i = floor(w_i 2^48) and every
// pointer comparison is an exact 128-bit product, so the ancestors do not
// depend on reduction order.  Only the estimate and the ESS use FP64 tree
// sums.
#include "internal.h"

namespace smc {
namespace {

constexpr int kFT = 1024;  // filter workgroup
constexpr int kFW = kFT / 64;
// Particles whose resampling CDF the filter workgroup keeps in LDS (32 KB);
// larger sets search the CDF in global memory.
constexpr uint32_t kCdfLds = 4096;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

__device__ __forceinline__ double wave_add(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long *p, uint64_t n) {
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n; q += (uint64_t)gridDim.x * blockDim.x)
        p[q] = 0ull;
}

__global__ __launch_bounds__(256) void k_words(const double *x, uint32_t n, Geom g, bool nearest, float *words) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p[6];
    for (int d = 0; d < 6; ++d) p[d] = x[6 * (size_t)i + d];
    particle_words(p, g, nearest, words + 12 * (size_t)i);
}

// Prior: x_i = x0 + L (2u - 1), u from Philox (tag 0, three blocks).
constexpr uint32_t kProposalTries = 16;

// Six standard normals of try t for particle i from the proposal stream.
__device__ __forceinline__ void proposal_normals(const FilterState &f, uint32_t i, uint32_t t, double g[6]) {
    for (uint32_t b = 0; b < 3; ++b) {
        uint32_t r[4];
        draw4(f.seed, i, t, f.pair, kTagProposal, b, r);
        const double u1 = uniform53(r[0], r[1]), u2 = uniform53(r[2], r[3]);
        const double rad = sqrt(-2.0 * log(u1));
        const double th = 6.283185307179586 * u2;
        g[2 * b] = rad * cos(th);
        g[2 * b + 1] = rad * sin(th);
    }
}

__device__ __forceinline__ void init_body(const FilterState &f, uint32_t i, uint32_t stride) {
    if (i < f.n) {
        double p[6];
        if (f.has_proposal) {
            // per-axis rejection into the box (a product region), clamp after 16 tries
            bool done[6] = {false, false, false, false, false, false};
            for (int d = 0; d < 6; ++d) p[d] = fmin(fmax(f.prop_mu[d], f.lo[d]), f.hi[d]);
            for (uint32_t t = 0; t < kProposalTries; ++t) {
                double g[6];
                proposal_normals(f, i, t, g);
                for (int d = 0; d < 6; ++d) {
                    const double v = f.prop_mu[d] + f.prop_sigma[d] * g[d];
                    if (!done[d] && v >= f.lo[d] && v <= f.hi[d]) {
                        p[d] = v;
                        done[d] = true;
                    }
                }
            }
            double lq = 0.0;
            for (int d = 0; d < 6; ++d) {
                const double z = (p[d] - f.prop_mu[d]) / f.prop_sigma[d];
                lq += 0.5 * (z * z);
            }
            f.lq[i] = lq;
        } else {
            for (uint32_t b = 0; b < 3; ++b) {
                uint32_t r[4];
                draw4(f.seed, i, 0u, f.pair, kTagInit, b, r);
                const double ua = uniform53(r[0], r[1]), ub = uniform53(r[2], r[3]);
                const int d0 = 2 * b, d1 = 2 * b + 1;
                p[d0] = f.x0[d0] + f.limit[d0] * (2.0 * ua - 1.0);
                p[d1] = f.x0[d1] + f.limit[d1] * (2.0 * ub - 1.0);
            }
        }
        for (int d = 0; d < 6; ++d) f.x[6 * (size_t)i + d] = p[d];
        particle_words(p, f.geom, f.nearest, f.words + 12 * (size_t)i);
        f.lw[i] = 0.0;
        f.anc[i] = -1;
    }
    if (i == 0) {
        for (int d = 0; d < 6; ++d) f.est[d] = f.x0[d];
        particle_words(f.x0, f.geom, f.nearest, f.words + 12 * (size_t)f.n);
        f.flags[0] = 0;
        f.flags[1] = 0;
        f.flags[2] = f.has_proposal ? 1 : 0;
    }
    const uint32_t nt = f.n_iters + 1;
    for (uint32_t q = i; q < nt; q += stride) {
        f.trace_score[q] = __builtin_nan("");
        if (q < f.n_iters) {
            f.trace_ess[q] = __builtin_nan("");
            for (int d = 0; d < 6; ++d) f.trace_est[6 * q + d] = __builtin_nan("");
        }
    }
}

__global__ __launch_bounds__(256) void k_init(const FilterState f) {
    init_body(f, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ __launch_bounds__(256) void k_init_batch(const FilterState *fs) {
    const FilterState &f = fs[blockIdx.y];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < f.n || i < f.n_iters + 1) init_body(f, i, gridDim.x * blockDim.x);
}

__device__ __forceinline__ bool pointer_passed(unsigned long long c, unsigned __int128 scale,
                                               unsigned __int128 rhs) {
    return (unsigned __int128)c * scale > rhs;
}

__device__ __forceinline__ void filter_body(const FilterState &f, const uint32_t k) {
    __shared__ double red[kFW][12];
    __shared__ double bcast[12];
    __shared__ uint32_t ref_idx[kFW];
    __shared__ unsigned long long scan[kFT];
    __shared__ unsigned long long cdf_lds[kCdfLds];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const uint32_t n = f.n;
    // the binary searches of the resampling step read this CDF: each search is
    // a chain of dependent loads, far shorter from LDS than from L2
    unsigned long long *const cdf = n <= kCdfLds ? cdf_lds : f.cdf;

    // update: log-weights of the scores, and their maximum; a set drawn from
    // the proposal carries the importance correction in its first update
    const bool from_proposal = f.flags[2] != 0;
    double mx = -INFINITY;
    for (uint32_t i = tid; i < n; i += kFT) {
        int64_t m[6];
        for (int q = 0; q < 6; ++q) m[q] = (int64_t)f.sums[6 * (size_t)i + q];
        double l = log_likelihood(score_from_sums(m, f.sc), f.sc);
        if (k == 1 && from_proposal) l = l + f.lq[i];
        f.lw[i] = l;
        mx = fmax(mx, l);
    }
    if (tid == 0) {
        int64_t m[6];
        for (int q = 0; q < 6; ++q) m[q] = (int64_t)f.sums[6 * (size_t)n + q];
        f.trace_score[k - 1] = score_from_sums(m, f.sc);
    }
    mx = wave_max(mx);
    if (lane == 0) red[wave][0] = mx;
    __syncthreads();
    if (tid == 0) {
        double v = red[0][0];
        for (int w = 1; w < kFW; ++w) v = fmax(v, red[w][0]);
        bcast[0] = v;
    }
    __syncthreads();
    const double M = bcast[0];
    const bool degenerate = M == -INFINITY;

    // wide rotations: the reference hemisphere is that of the first particle
    // of largest log-weight (all of them when every weight is -inf)
    double qref[4] = {1.0, 0.0, 0.0, 0.0};
    if (f.wide) {
        uint32_t first = n;
        for (uint32_t i = tid; i < n; i += kFT)
            if (f.lw[i] == M) {
                first = i;
                break;
            }
        first = wave_min_u32(first);
        if (lane == 0) ref_idx[wave] = first;
        __syncthreads();
        uint32_t r = ref_idx[0];
        for (int w = 1; w < kFW; ++w) r = min(r, ref_idx[w]);
        rotation_quaternion(f.x + 6 * (size_t)(r < n ? r : 0u), qref);
    }

    // normalise and estimate: w_i = exp(lw_i - M), weighted mean, ESS, and
    // for wide rotations the weighted sum of hemisphere-aligned quaternions
    double s = 0.0, s2 = 0.0, sx[6] = {0, 0, 0, 0, 0, 0}, sq[4] = {0, 0, 0, 0};
    for (uint32_t i = tid; i < n; i += kFT) {
        const double w = degenerate ? 1.0 : exp(f.lw[i] - M);
        f.w[i] = w;
        s += w;
        s2 += w * w;
        for (int d = 0; d < 6; ++d) sx[d] += w * f.x[6 * (size_t)i + d];
        if (f.wide) {
            double q[4];
            rotation_quaternion(f.x + 6 * (size_t)i, q);
            const double dot = q[0] * qref[0] + q[1] * qref[1] + q[2] * qref[2] + q[3] * qref[3];
            const double ws = dot < 0.0 ? -w : w;
            for (int c = 0; c < 4; ++c) sq[c] += ws * q[c];
        }
    }
    s = wave_add(s);
    s2 = wave_add(s2);
    for (int d = 0; d < 6; ++d) sx[d] = wave_add(sx[d]);
    for (int c = 0; c < 4; ++c) sq[c] = wave_add(sq[c]);
    __syncthreads();
    if (lane == 0) {
        red[wave][0] = s;
        red[wave][1] = s2;
        for (int d = 0; d < 6; ++d) red[wave][2 + d] = sx[d];
        for (int c = 0; c < 4; ++c) red[wave][8 + c] = sq[c];
    }
    __syncthreads();
    if (tid < 12) {
        double v = 0.0;
        for (int w = 0; w < kFW; ++w) v += red[w][tid];
        bcast[tid] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double est[6];
        for (int d = 0; d < 6; ++d) est[d] = bcast[2 + d] / bcast[0];
        if (f.wide) {
            const double nq = sqrt(bcast[8] * bcast[8] + bcast[9] * bcast[9] + bcast[10] * bcast[10] +
                                   bcast[11] * bcast[11]);
            const double q[4] = {bcast[8] / nq, bcast[9] / nq, bcast[10] / nq, bcast[11] / nq};
            double e[3];
            quaternion_euler(q, e);
            for (int d = 0; d < 3; ++d) est[d] = wrap_near(e[d], f.x0[d]);
        }
        for (int d = 0; d < 6; ++d) {
            f.est[d] = est[d];
            f.trace_est[6 * (size_t)(k - 1) + d] = est[d];
        }
        f.trace_ess[k - 1] = (bcast[0] * bcast[0]) / bcast[1];
        if (degenerate) f.flags[0] = 1;
        f.flags[1] = degenerate ? 1 : 0;  // the latest iteration's weights were all -inf
        particle_words(est, f.geom, f.nearest, f.words + 12 * (size_t)n);
    }

    if (k < f.n_iters) {
        // exact integer CDF: contiguous chunk per thread, block scan of chunk sums
        const uint32_t per = (n + kFT - 1) / kFT;
        const uint32_t b0 = min(n, tid * per), b1 = min(n, b0 + per);
        unsigned long long local = 0;
        for (uint32_t i = b0; i < b1; ++i) local += (unsigned long long)floor(f.w[i] * 0x1p48);
        scan[tid] = local;
        __syncthreads();
        for (int off = 1; off < kFT; off <<= 1) {
            const unsigned long long v = tid >= off ? scan[tid - off] : 0ull;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        unsigned long long run = scan[tid] - local;
        for (uint32_t i = b0; i < b1; ++i) {
            run += (unsigned long long)floor(f.w[i] * 0x1p48);
            cdf[i] = run;
        }
        const unsigned long long Q = scan[kFT - 1];
        __syncthreads();

        uint32_t rw[4];
        draw4(f.seed, 0u, k, f.pair, kTagResample, 0u, rw);
        const unsigned __int128 scale = (unsigned __int128)n << 32;
        double sg[6];
        for (int d = 0; d < 6; ++d) {
            double v = f.sigma0[d];
            for (uint32_t m = 1; m < k; ++m) v = v * f.anneal;
            sg[d] = v;
        }
        for (uint32_t j = tid; j < n; j += kFT) {
            const unsigned __int128 rhs = ((((unsigned __int128)j) << 32) + rw[0]) * (unsigned __int128)Q;
            uint32_t lo = 0, hi = n - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (pointer_passed(cdf[mid], scale, rhs)) hi = mid;
                else lo = mid + 1;
            }
            f.anc[j] = (int32_t)lo;
            // prediction: reflected annealed Gaussian random walk (Box-Muller)
            double g[6];
            for (uint32_t b = 0; b < 3; ++b) {
                uint32_t r[4];
                draw4(f.seed, j, k, f.pair, kTagPerturb, b, r);
                const double u1 = uniform53(r[0], r[1]), u2 = uniform53(r[2], r[3]);
                const double rad = sqrt(-2.0 * log(u1));
                const double th = 6.283185307179586 * u2;
                g[2 * b] = rad * cos(th);
                g[2 * b + 1] = rad * sin(th);
            }
            for (int d = 0; d < 6; ++d) {
                const double v = f.x[6 * (size_t)lo + d] + sg[d] * g[d];
                // wide rotations: an axis whose limit covers the circle wraps
                f.x_next[6 * (size_t)j + d] = f.wide && d < 3 && f.limit[d] >= 3.141592653589793
                                                  ? wrap_near(v, f.x0[d])
                                                  : reflect_into(v, f.lo[d], f.hi[d]);
            }
        }
        __syncthreads();
        for (uint32_t j = tid; j < n; j += kFT) {
            double p[6];
            for (int d = 0; d < 6; ++d) {
                p[d] = f.x_next[6 * (size_t)j + d];
                f.x[6 * (size_t)j + d] = p[d];
            }
            particle_words(p, f.geom, f.nearest, f.words + 12 * (size_t)j);
        }
    }
    // clear the sums for the next evaluation
    for (uint32_t q = tid; q < 6 * (n + 1); q += kFT) f.sums[q] = 0ull;
}

__global__ __launch_bounds__(kFT) void k_filter(const FilterState f, const uint32_t k) { filter_body(f, k); }

__global__ __launch_bounds__(kFT) void k_filter_batch(const FilterState *fs, const uint32_t k) {
    const FilterState &f = fs[blockIdx.x];
    if (k <= f.n_iters) filter_body(f, k);
}

// Weighted mean and per-axis weighted variance of the particle set under the
// normalised weights exp(lw_i - max lw) of the last evaluation (uniform when
// every log-weight is -inf): out[0..5] the mean, out[6..11] the variance,
// in the filter's units.  One workgroup; FP64 tree sums.
__global__ __launch_bounds__(kFT) void k_cloud_moments(const FilterState f, double *out) {
    __shared__ double red[kFW][7];
    __shared__ double bc[7];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const uint32_t n = f.n;
    double mx = -INFINITY;
    for (uint32_t i = tid; i < n; i += kFT) mx = fmax(mx, f.lw[i]);
    mx = wave_max(mx);
    if (lane == 0) red[wave][0] = mx;
    __syncthreads();
    if (tid == 0) {
        double v = red[0][0];
        for (int w = 1; w < kFW; ++w) v = fmax(v, red[w][0]);
        bc[0] = v;
    }
    __syncthreads();
    const double M = bc[0];
    const bool flat = M == -INFINITY;
    // pass 1: total weight and weighted sums of the states
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (uint32_t i = tid; i < n; i += kFT) {
        const double w = flat ? 1.0 : exp(f.lw[i] - M);
        acc[0] += w;
        for (int d = 0; d < 6; ++d) acc[1 + d] += w * f.x[6 * (size_t)i + d];
    }
    for (int q = 0; q < 7; ++q) acc[q] = wave_add(acc[q]);
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < 7; ++q) red[wave][q] = acc[q];
    __syncthreads();
    if (tid < 7) {
        double v = 0.0;
        for (int w = 0; w < kFW; ++w) v += red[w][tid];
        bc[tid] = v;
    }
    __syncthreads();
    const double total = bc[0];
    double mean[6];
    for (int d = 0; d < 6; ++d) mean[d] = bc[1 + d] / total;
    // pass 2: weighted squared deviations from the mean
    double dv[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t i = tid; i < n; i += kFT) {
        const double w = flat ? 1.0 : exp(f.lw[i] - M);
        for (int d = 0; d < 6; ++d) {
            const double e = f.x[6 * (size_t)i + d] - mean[d];
            dv[d] += w * (e * e);
        }
    }
    for (int d = 0; d < 6; ++d) dv[d] = wave_add(dv[d]);
    __syncthreads();
    if (lane == 0)
        for (int d = 0; d < 6; ++d) red[wave][d] = dv[d];
    __syncthreads();
    if (tid < 6) {
        double v = 0.0;
        for (int w = 0; w < kFW; ++w) v += red[w][tid];
        out[tid] = mean[tid];
        out[6 + tid] = v / total;
    }
}

__global__ void k_ghost_final(const FilterState f) {
    int64_t m[6];
    for (int q = 0; q < 6; ++q) m[q] = (int64_t)f.sums[6 * (size_t)f.n + q];
    f.trace_score[f.n_iters] = score_from_sums(m, f.sc);
    for (int q = 0; q < 6; ++q) f.sums[6 * (size_t)f.n + q] = 0ull;
}

// One workgroup per particle: the histogram and its marginals (exact
// integer counts) in LDS, then one thread forms the entropies in bin order
// with mi_log, so the score is the same on every platform; 2 I / (H_s + H_t).
__global__ __launch_bounds__(256) void k_mi_finalize(uint32_t *hist, uint32_t p0, unsigned long long *sums) {
    constexpr int kHB = kMiBins * kMiBins;
    __shared__ uint32_t h[kHB];
    __shared__ unsigned long long marg[2 * kMiBins];
    __shared__ unsigned long long total;
    const uint32_t i = p0 + blockIdx.x;
    uint32_t *hp = hist + (size_t)kHB * i;
    const int tid = threadIdx.x;
    if (tid < 2 * kMiBins) marg[tid] = 0ull;
    if (tid == 0) total = 0ull;
    __syncthreads();
    unsigned long long mine = 0;
    for (int q = tid; q < kHB; q += 256) {
        const uint32_t v = hp[q];
        h[q] = v;
        hp[q] = 0u;  // ready for the next evaluation
        mine += v;
        if (v) {
            atomicAdd(&marg[q / kMiBins], (unsigned long long)v);
            atomicAdd(&marg[kMiBins + q % kMiBins], (unsigned long long)v);
        }
    }
    atomicAdd(&total, mine);
    __syncthreads();
    if (tid != 0) return;
    const unsigned long long n = total;
    double z = 0.0;
    if (n) {
        const double N = (double)n;
        double hs = 0.0, ht = 0.0, hst = 0.0;
        for (int a = 0; a < kMiBins; ++a) {
            if (marg[a]) {
                const double f = (double)marg[a] / N;
                hs = hs - f * mi_log(f);
            }
            if (marg[kMiBins + a]) {
                const double f = (double)marg[kMiBins + a] / N;
                ht = ht - f * mi_log(f);
            }
        }
        for (int q = 0; q < kHB; ++q)
            if (h[q]) {
                const double f = (double)h[q] / N;
                hst = hst - f * mi_log(f);
            }
        if (hs + ht > 0.0) z = 2.0 * (hs + ht - hst) / (hs + ht);
    }
    unsigned long long bits;
    memcpy(&bits, &z, sizeof bits);
    unsigned long long *o = sums + 6 * (size_t)i;
    o[0] = n;
    o[1] = bits;
    o[2] = o[3] = o[4] = o[5] = 0ull;
}

__global__ __launch_bounds__(256) void k_scores_from_sums(const unsigned long long *sums, uint32_t n,
                                                          const ScoreConst sc, double *z) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t m[6];
    for (int q = 0; q < 6; ++q) m[q] = (int64_t)sums[6 * (size_t)i + q];
    z[i] = score_from_sums(m, sc);
}

}  // namespace

hipError_t launch_mi_finalize(uint32_t *hist, uint32_t p0, uint32_t np, unsigned long long *sums, hipStream_t s) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mi_finalize, dim3(np), dim3(256), 0, s, hist, p0, sums);
    return hipGetLastError();
}

hipError_t launch_scores_from_sums(const unsigned long long *sums, uint32_t n, const ScoreConst &sc, double *z,
                                   hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scores_from_sums, dim3((n + 255) / 256), dim3(256), 0, s, sums, n, sc, z);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)(b < 2048 ? b : 2048)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_words(const double *x, uint32_t n, const Geom &g, bool nearest, float *words, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_words, dim3((n + 255) / 256), dim3(256), 0, s, x, n, g, nearest, words);
    return hipGetLastError();
}

hipError_t launch_init_particles(const FilterState &f, hipStream_t s) {
    const uint32_t n = f.n > f.n_iters + 1 ? f.n : f.n_iters + 1;
    hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_filter(const FilterState &f, uint32_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_filter, dim3(1), dim3(kFT), 0, s, f, k);
    return hipGetLastError();
}

hipError_t launch_init_batch(const FilterState *fs, uint32_t n_pairs, uint32_t max_threads, hipStream_t s) {
    hipLaunchKernelGGL(k_init_batch, dim3((max_threads + 255) / 256, n_pairs), dim3(256), 0, s, fs);
    return hipGetLastError();
}

hipError_t launch_filter_batch(const FilterState *fs, uint32_t n_pairs, uint32_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_filter_batch, dim3(n_pairs), dim3(kFT), 0, s, fs, k);
    return hipGetLastError();
}

hipError_t launch_cloud_moments(const FilterState &f, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_cloud_moments, dim3(1), dim3(kFT), 0, s, f, out);
    return hipGetLastError();
}

hipError_t launch_ghost_final(const FilterState &f, hipStream_t s) {
    hipLaunchKernelGGL(k_ghost_final, dim3(1), dim3(1), 0, s, f);
    return hipGetLastError();
}

}  // namespace smc
