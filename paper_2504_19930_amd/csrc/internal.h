// Internal launch interface between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace smc {

// Warp-and-score launch: particle range [p0, p0 + np) of `words`, sums
// accumulated (atomically, exactly) into sums[6 * p].
enum ScoreMode : int { kModeMask = 0, kModeImageTrilinear = 1, kModeImageNearest = 2 };

struct ScoreLaunch {
    int mode;
    const uint8_t *src;       // mask: prepared bits; image: intensities
    const uint8_t *src_ok;    // image: corner-valid bytes (source FOV) or nullptr
    const uint8_t *tgt;       // mask: prepared bits; image: intensities
    const uint8_t *tgt_fov;   // image: target FOV or nullptr
    const float *words;       // 12 per particle
    unsigned long long *sums; // 6 per particle
    int32_t sn[3], tn[3];
    uint32_t p0, np;
};

hipError_t launch_score(const ScoreLaunch &L, hipStream_t s);
void score_grid(const ScoreLaunch &L, dim3 *grid, dim3 *block);

// Preparation of inputs.
hipError_t launch_prep_mask(const uint8_t *vol, const uint8_t *fov, uint8_t *out, int64_t n, hipStream_t s);
hipError_t launch_corner_valid(const uint8_t *fov, uint8_t *out, const int32_t n[3], hipStream_t s);
// out[0..3] += (fov count, nonzero count, sum v, sum v^2) over the FOV
hipError_t launch_volume_sums(const uint8_t *vol, const uint8_t *fov, int64_t n, unsigned long long *out,
                              hipStream_t s);

// Filter state of one registration pair.
struct FilterState {
    uint32_t n;               // particles
    uint32_t n_iters;         // K
    uint64_t seed;
    uint32_t pair;
    Geom geom;
    bool nearest;             // recipe words with the +0.5 shift
    ScoreConst sc;
    double x0[6], limit[6], lo[6], hi[6], sigma0[6], anneal;
    double *x;                // n x 6 current particles
    double *x_next;           // n x 6 scratch
    float *words;             // (n + 1) x 12, the last row is the ghost (estimate)
    unsigned long long *sums; // (n + 1) x 6
    double *lw;               // n log-weights of the last evaluation
    double *w;                // n scratch weights
    unsigned long long *cdf;  // n
    int32_t *anc;             // n
    double *est;              // 6 current estimate
    double *trace_score;      // K + 1
    double *trace_ess;        // K
    double *trace_est;        // 6 K
    int32_t *flags;           // [0] degenerate weights seen
};

hipError_t launch_init_particles(const FilterState &f, hipStream_t s);
hipError_t launch_filter(const FilterState &f, uint32_t k, hipStream_t s);
hipError_t launch_ghost_final(const FilterState &f, hipStream_t s);
hipError_t launch_words(const double *x, uint32_t n, const Geom &g, bool nearest, float *words, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, hipStream_t s);

// warp_apply
hipError_t launch_warp_apply(const uint8_t *src, const int32_t sn[3], const float w[12], bool trilinear,
                             uint8_t *dst, const int32_t tn[3], uint32_t frames, int64_t src_stride,
                             int64_t dst_stride, hipStream_t s);

}  // namespace smc
