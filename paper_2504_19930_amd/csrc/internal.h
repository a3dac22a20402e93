// Internal launch interface between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace smc {

// floor and convert in one instruction (exact for the non-negative
// coordinates whose results are used)
__device__ __forceinline__ uint32_t floor_u32(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return (uint32_t)r;
}

// a * b + c on the low 24 bits of a and b, as one instruction (the compiler
// otherwise forms two multiplies and a three-way add); b is uniform across
// the wave (a stride) and is passed as a scalar operand.
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// Warp-and-score launch: particle range [p0, p0 + np) of `words`, sums
// accumulated (atomically, exactly) into sums[6 * p].
enum ScoreMode : int { kModeMask = 0, kModeImageTrilinear = 1, kModeImageNearest = 2 };

// Source layouts for trilinear sampling (see score.hip): bytes per voxel
// 1, 2, 4, 8, 8, 16; eight, four, two or one gathers per sample.
enum SourceLayout : int {
    kLayoutRaw = 0,
    kLayoutPairX = 1,
    kLayoutQuadXY = 2,
    kLayoutOct = 3,
    kLayoutOctTile = 4,
    kLayoutLerp = 5
};
constexpr int kLayouts = 6;
// The lerp layout marks elements that touch a voxel outside the source FOV
// with a pair of half-precision NaNs in the first word; no valid element
// holds a NaN, so this sentinel always exists.
constexpr uint32_t kLerpSentinel = 0x7E007E00u;

struct ScoreLaunch {
    int mode;
    const uint8_t *src;       // mask: prepared bits; image: intensities
    const void *src_packed;   // trilinear: source in `layout` (nullptr = raw bytes)
    bool has_sentinel;        // packed elements equal to `sentinel` mark samples outside the source FOV
    uint64_t sentinel;
    int layout;               // SourceLayout
    int pt;                   // particles per workgroup: 4, 8 or 16
    int zchunk;               // target z-extent of a tile (0 = up to 256)
    // masks: cull to the source mask's bounding box (exact for a and c only;
    // n and b_ov then count only the tiles that reach it)
    bool cull_box;
    int32_t box_lo[3], box_hi[3];
    const uint32_t *src_bits = nullptr;  // mask: bitmap of the source's on bits (the filter's launches)
    // mask, culled launches: summed-area table of the source's occupied cells
    // (or nullptr: the bounding box alone)
    const uint32_t *occ = nullptr;
    // mask, culled item-list launches (or nullptr): kWorkSlots counter pairs,
    // kWorkSlotWords apart; summed over the slots, word 0 counts the particle x
    // voxel pairs evaluated, word 1 the pairs covered (the culled ones included)
    unsigned long long *work = nullptr;
    const uint8_t *src_ok;    // image: corner-valid bytes (source FOV) or nullptr
    const uint8_t *tgt;       // mask: prepared bits; image: intensities
    const uint8_t *tgt_fov;   // image: target FOV or nullptr
    const float *words;       // 12 per particle
    unsigned long long *sums; // 6 per particle
    int32_t sn[3], tn[3];
    uint32_t p0, np;
    // mutual information: the launch adds into kMiBins^2 counts per particle
    // (indexed like words) instead of the moments
    uint32_t *hist = nullptr;
    // masks, the filter's launches: the culled item lists (capacity item_cap
    // items of 8 bytes) and their counters (kItemCounterWords 32-bit words);
    // launches with more items than item_cap use a grid of one workgroup per item
    void *items = nullptr;
    uint32_t *item_counters = nullptr;
    uint64_t item_cap = 0;
};
constexpr uint32_t kItemCounterWords = 512;
// Most work items (tiles x particle groups) one scoring launch takes: a grid
// dimension of signed 32-bit size.
constexpr uint64_t kMaxScoreItems = 0x7FFFFFFFull;
// Items (tiles x particle groups) of a launch of L's shape with np particles.
uint64_t score_items_for(const ScoreLaunch &L);

hipError_t launch_score(const ScoreLaunch &L, hipStream_t s);
// Gather probe (measurement): the launch's grid, culling, coordinates and
// source loads without the rest of the kernel's work; see score.hip.
bool gather_probe_supported(const ScoreLaunch &L);
hipError_t launch_gather_probe(const ScoreLaunch &L, uint32_t key, uint32_t *out, hipStream_t s);
void score_grid(const ScoreLaunch &L, dim3 *grid, dim3 *block);
bool score_pt_supported(int pt);
// whether a packed trilinear layout can address a source of this shape
bool layout_fits(int layout, const int32_t sn[3]);
// Pack a source volume into `layout` (edge corners repeat the last voxel).
// With fov, elements touching a voxel outside it hold `sentinel` instead.
hipError_t launch_pack_source(const uint8_t *vol, const uint8_t *fov, const int32_t n[3], int layout,
                              uint64_t sentinel, void *out, hipStream_t s);
// Over the elements of `layout` that lie inside the fov, count those equal to
// each candidate (truncated to the element width) -- or, for x-pairs with
// n_cand == 0, a 65536-bin histogram of all element values.
hipError_t launch_count_elements(const uint8_t *vol, const uint8_t *fov, const int32_t n[3], int layout,
                                 const uint64_t *cand, int n_cand, unsigned long long *counts, hipStream_t s);
size_t packed_bytes_per_voxel(int layout);
// bytes of a packed source of shape n (the tiled layout pads x and y to 4)
uint64_t packed_bytes(int layout, const int32_t n[3]);

// Batched warp-and-score: one persistent launch over the work items of many
// pairs of one class (masks, or trilinear images in one layout).
struct BatchPlan {
    int mode, layout, pt, vmode;  // vmode: source FOV validity (0 none, 1 gathered, 2 sentinel)
    const void *pairs;        // device array of per-pair kernel arguments (score_args)
    const uint32_t *offs;     // n_pairs + 1 item offsets
    const uint32_t *kmax;     // iterations per pair
    const uint32_t *lists;    // item ids grouped by XCD
    uint32_t list_off[9];
    uint32_t n_pairs;
    uint32_t grid;            // persistent workgroups
    // item queues: 8 counters (one per XCD list) per iteration, zero before
    // the run; iteration k uses counters[8 (k - 1) .. 8 k)
    uint32_t *counters;
    // masks: per iteration a cull pre-pass appends the live items (item id,
    // particle mask) of list x to live[list_off[x] ..), counted in
    // live_counts[kItemCounterWords / 2 (k - 1) + 32 x] (zero before the run)
    void *live = nullptr;
    uint32_t *live_counts = nullptr;
};
size_t score_args_bytes();
uint32_t score_items(const ScoreLaunch &L);
void score_args(const ScoreLaunch &L, void *out);
hipError_t launch_batch_score(const BatchPlan &P, uint32_t k, hipStream_t s);
const void *batch_kernel(const BatchPlan &P);
// resident workgroups per CU of the plan's kernel (the persistent grid size)
int batch_blocks_per_cu(const BatchPlan &P);
// source FOV validity mode of a launch: 0 none, 1 gathered mask, 2 sentinel
int score_vmode(const ScoreLaunch &L);

// Preparation of inputs.
hipError_t launch_prep_mask(const uint8_t *vol, const uint8_t *fov, uint8_t *out, int64_t n, hipStream_t s);
// Bounding box of the voxels with bit 1 set (mask on): out = {min x, y, z, max x, y, z};
// initialise out to {INT_MAX x3, -1 x3}.
hipError_t launch_mask_bbox(const uint8_t *prep, const int32_t n[3], int32_t *out, hipStream_t s);
// Bitmap of the prepared source mask's "on" bits (rows padded to 32 bits):
// bytes of the bitmap of a volume of shape n, and the packing launch.
uint64_t mask_bits_bytes(const int32_t n[3]);
hipError_t launch_pack_mask_bits(const uint8_t *prep, const int32_t n[3], uint32_t *out, hipStream_t s);
// Occupancy of the prepared source mask's "on" bits over cells of
// 2^kOccShift voxels a side, as a summed-area table with a zero first row,
// column and slice: words of the table, and the building launches.
constexpr int kOccShift = 1;
constexpr uint64_t kOccMaxWords = 16ull << 20;  // 64 MB
constexpr uint32_t kWorkSlots = 64, kWorkSlotWords = 16;
uint64_t mask_occ_words(const int32_t n[3]);
hipError_t launch_mask_occupancy(const uint8_t *prep, const int32_t n[3], uint32_t *sat, hipStream_t s);
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
    // [0] degenerate weights seen, [1] at the latest iteration, [2] the current
    // particle set is a draw from the proposal (its first update adds lq)
    int32_t *flags;
    // learned proposal: the next prior draw comes from a Gaussian truncated to
    // the limits box; the draw records itself in flags[2], and the first update
    // of such a set adds log p - log q (p uniform)
    int32_t has_proposal;
    double prop_mu[6], prop_sigma[6];
    double *lq;               // n: -log q(x_i) + const of the proposal draw
    // wide rotations: quaternion-mean estimate; rotation axes with limit >= pi wrap
    int32_t wide;
};

hipError_t launch_init_particles(const FilterState &f, hipStream_t s);
// Batched filter: one workgroup per pair, states in device memory.
hipError_t launch_init_batch(const FilterState *states_dev, uint32_t n_pairs, uint32_t max_threads, hipStream_t s);
hipError_t launch_filter_batch(const FilterState *states_dev, uint32_t n_pairs, uint32_t k, hipStream_t s);
hipError_t launch_filter(const FilterState &f, uint32_t k, hipStream_t s);
hipError_t launch_ghost_final(const FilterState &f, hipStream_t s);
// Weighted mean (out[0..5]) and per-axis weighted variance (out[6..11]) of the
// particle set under the normalised weights of the last evaluation.
hipError_t launch_cloud_moments(const FilterState &f, double *out, hipStream_t s);
hipError_t launch_words(const double *x, uint32_t n, const Geom &g, bool nearest, float *words, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, hipStream_t s);
// Mutual information: scores of particles p0 .. p0 + np - 1 from their joint
// histograms into their sums (overlap count, score bits), clearing the
// histograms for the next evaluation.
hipError_t launch_mi_finalize(uint32_t *hist, uint32_t p0, uint32_t np, unsigned long long *sums, hipStream_t s);
// Final scores of n particles from their sums.
hipError_t launch_scores_from_sums(const unsigned long long *sums, uint32_t n, const ScoreConst &sc, double *z,
                                   hipStream_t s);

// Learned proposal network (cnn.hip).
extern const int kCnnChannels[5];
extern const int kCnnSide;
extern const int kCnnFlat;
struct CnnBuffers {
    float *params;       // FP32 master weights (flat; layout in smc.h)
    uint16_t *wbf16;     // bfloat16 copy of the convolution part
    float *grads, *adam_m, *adam_v;
    int64_t n_params;
    uint16_t *act[4];    // layer outputs after ReLU, bfloat16
    float *dact[4];      // gradients w.r.t. layer pre-activations
    float *dout;         // B x 12
    float *partial;      // split-K partial tiles of the forward convolutions
    int64_t partial_cap; // floats in partial
};
// Floats of the forward split-K buffer a network of max_batch pairs needs.
int64_t cnn_partial_floats(int max_batch);
int64_t cnn_param_offset(int part);
hipError_t cnn_downsample(const uint8_t *vol, const int32_t n[3], float scale, uint16_t *out, hipStream_t s);
hipError_t cnn_forward(const CnnBuffers &c, const uint16_t *input, int B, float *out, hipStream_t s);
hipError_t cnn_backward(const CnnBuffers &c, const uint16_t *input, int B, const float *out, const float *target,
                        float *loss_dev, hipStream_t s);
hipError_t cnn_adam(const CnnBuffers &c, float lr, int t, hipStream_t s);
hipError_t cnn_refresh_bf16(const CnnBuffers &c, hipStream_t s);

// Exhaustive search (exhaustive.hip).
hipError_t launch_grid_words(const double lo[6], const double step[6], const uint32_t count[6], uint64_t first,
                             uint32_t n, const Geom &g, bool nearest, double *x, float *words, hipStream_t s);
hipError_t launch_chunk_best(const unsigned long long *sums, uint32_t n, uint64_t first, const ScoreConst &sc,
                             double *scores, double *best_z, unsigned long long *best_i, hipStream_t s);

// warp_apply
hipError_t launch_warp_apply(const uint8_t *src, const int32_t sn[3], const float w[12], bool trilinear,
                             uint8_t *dst, const int32_t tn[3], uint32_t frames, int64_t src_stride,
                             int64_t dst_stride, hipStream_t s);

}  // namespace smc
