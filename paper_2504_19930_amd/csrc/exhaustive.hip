// Exhaustive search over a regular grid of rigid transforms -- the paper's
// EX baseline (Baseline and Evaluation Metrics), an exhaustive optimizer over
// a fixed grid -- on the same warp-and-score kernels as the filter: grid
// points are scored in chunks as if they were particles, and each chunk's
// best point (ties to the lower index) is kept.
#include "internal.h"

namespace smc {
namespace {

struct GridArgs {
    double lo[6], step[6];
    uint32_t count[6];
    uint64_t first;   // global index of the chunk's first point
    uint32_t n;       // points in the chunk
};

// Grid point g -> parameters, axis 0 varying fastest.
__device__ __forceinline__ void grid_point(const GridArgs &a, uint64_t g, double p[6]) {
    for (int d = 0; d < 6; ++d) {
        const uint64_t c = g % a.count[d];
        g /= a.count[d];
        p[d] = a.lo[d] + a.step[d] * (double)c;
    }
}

__global__ __launch_bounds__(256) void k_grid_words(const GridArgs a, Geom geom, bool nearest, double *x,
                                                    float *words) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double p[6];
    grid_point(a, a.first + i, p);
    for (int d = 0; d < 6; ++d) x[6 * (size_t)i + d] = p[d];
    particle_words(p, geom, nearest, words + 12 * (size_t)i);
}

// Scores of the chunk (optional output) and its best point.
__global__ __launch_bounds__(256) void k_chunk_best(const unsigned long long *sums, uint32_t n, uint64_t first,
                                                    ScoreConst sc, double *scores, double *best_z,
                                                    unsigned long long *best_i) {
    double bz = -INFINITY;
    unsigned long long bi = ~0ull;
    for (uint32_t i = threadIdx.x; i < n; i += 256) {
        int64_t m[6];
        for (int q = 0; q < 6; ++q) m[q] = (int64_t)sums[6 * (size_t)i + q];
        const double z = score_from_sums(m, sc);
        if (scores) scores[i] = z;
        if (z > bz || (z == bz && first + i < bi)) {
            bz = z;
            bi = first + i;
        }
    }
    __shared__ double rz[256];
    __shared__ unsigned long long ri[256];
    rz[threadIdx.x] = bz;
    ri[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double z2 = rz[threadIdx.x + o];
            const unsigned long long i2 = ri[threadIdx.x + o];
            if (z2 > rz[threadIdx.x] || (z2 == rz[threadIdx.x] && i2 < ri[threadIdx.x])) {
                rz[threadIdx.x] = z2;
                ri[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *best_z = rz[0];
        *best_i = ri[0];
    }
}

}  // namespace

hipError_t launch_grid_words(const double lo[6], const double step[6], const uint32_t count[6], uint64_t first,
                             uint32_t n, const Geom &g, bool nearest, double *x, float *words, hipStream_t s) {
    GridArgs a;
    for (int d = 0; d < 6; ++d) {
        a.lo[d] = lo[d];
        a.step[d] = step[d];
        a.count[d] = count[d];
    }
    a.first = first;
    a.n = n;
    hipLaunchKernelGGL(k_grid_words, dim3((n + 255) / 256), dim3(256), 0, s, a, g, nearest, x, words);
    return hipGetLastError();
}

hipError_t launch_chunk_best(const unsigned long long *sums, uint32_t n, uint64_t first, const ScoreConst &sc,
                             double *scores, double *best_z, unsigned long long *best_i, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_best, dim3(1), dim3(256), 0, s, sums, n, first, sc, scores, best_z, best_i);
    return hipGetLastError();
}

}  // namespace smc
