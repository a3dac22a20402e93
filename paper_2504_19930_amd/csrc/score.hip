// Warp-and-score kernels: for every particle, map every target voxel into
// the source with the FP32 coordinate recipe, sample the source (nearest
// neighbour for masks, trilinear for images) and accumulate the exact integer
// sums the similarity needs (Eq. 4 for masks; Eq. 2 / normalised SSD for
// images).  This is the N x V inner loop of every filter iteration.
//
// Work decomposition: a 256-thread workgroup owns a 32 x 8 column of target
// voxels over a z-chunk and PT particles.  Each thread walks its column in
// z, so the particle-dependent part of the recipe,
//   mid_d = fma(A_d1, j, fma(A_d0, i, o_d)),
// is formed once and every voxel costs three FMAs (u_d = fma(A_d2, k, mid_d))
// per particle; the target byte is read once and reused by all PT particles.
// Sums stay in registers (32-bit where they provably fit, 64-bit otherwise),
// are reduced across the wave with shuffles, across the four waves in LDS,
// and land with one 64-bit atomic add per (workgroup, particle, sum).  Integer
// addition is associative, so the result does not depend on scheduling.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace smc {
namespace {

constexpr int kTX = 32;
constexpr int kTY = 8;
constexpr int kThreads = kTX * kTY;
constexpr int kWX = 16;  // wave patch width (x); 64 / kWX rows
static_assert(kTX % kWX == 0 && 64 % kWX == 0 && kTY % (64 / kWX) == 0, "waves must tile the 32 x 8 column");
static_assert(kWX == 16, "a wave's four quarters are 4 x 4 squares side by side in x");
constexpr int kWaves = kThreads / 64;
constexpr int kZChunkMax = 256;  // keeps every per-thread 32-bit sum below 2^32
constexpr int kSlab = 32;        // target slices staged in LDS at a time
constexpr uint32_t kItemChunk = 4;  // items a persistent workgroup takes at a time
// An item's second word: bit p for each live particle p (PT <= 16), and bit
// kInteriorBit when every live particle's image of the tile lies inside the
// source, so the scoring kernel can skip the per-sample inside test.
constexpr uint32_t kInteriorBit = 16;
// Bits 17..21 and 22..26: slices at the bottom and at the top of the item's
// tile that no live particle's image can sample an occupied source cell
// from (the pre-pass tests the tile's runs of kSpanSlices slices); the
// scoring kernel skips them.  Zero: the whole tile.  Only tiles of at most
// kSpanMaxDepth slices are trimmed.
constexpr uint32_t kSpanLoBit = 17, kSpanHiBit = 22, kSpanMask = 31;
constexpr int kSpanSlices = 4, kSpanMaxDepth = 32;

struct KArgs {
    const uint8_t *src, *src_ok, *tgt, *tgt_fov;
    const void *src_packed;
    const float *words;
    unsigned long long *sums;
    int32_t sn0, sn1, sn2, tn0, tn1, tn2;
    uint32_t p0, np;
    int32_t tiles_x, tiles_y, zchunk;
    // exact culling: a particle can add to the sums of a tile only if the
    // tile's image reaches the source-coordinate box [cull_lo, cull_hi]
    float cull_lo[3], cull_hi[3];
    // masks, culled launches: and only if a source voxel the image can sample
    // is on: summed-area table of occupied cells (nullptr: not used), its row
    // and slice strides, and the largest voxel index per axis
    const uint32_t *occ;
    uint32_t ocx, ocxy;
    float occ_hi[3];
    // source FOV validity of a trilinear sample: 0 none, 1 gather src_ok,
    // 2 packed elements equal to `sentinel` mark samples outside the FOV
    int32_t vmode;
    uint64_t sentinel;
    // packed layouts: byte size of the packed source and byte strides of its
    // rows and slices (32-bit buffer offsets; the host checks they fit)
    uint32_t src_bytes, ysb, zsb;
    // mutual information: per-particle joint histograms, kMiBins^2 counts each
    uint32_t *hist;
};

// Word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format,
// untyped loads; out-of-range offsets read zero).
constexpr int kBufferWord3 = 0x00020000;

// Culling margin (voxels): far above the FP32 rounding of the coordinate
// recipe for any coordinate below 2^16.
constexpr float kCullMargin = 0.0625f;

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Data that no kernel of a launch writes (recipe words, batch arguments,
// lists and offsets) is read through the constant address space, so the
// compiler can use scalar loads and scalar registers for uniform reads.
// (the address space exists only in the device compilation)
#if defined(__HIP_DEVICE_COMPILE__)
#define SMC_CONSTANT_AS __attribute__((address_space(4)))
#else
#define SMC_CONSTANT_AS
#endif
template <typename T>
__device__ __forceinline__ const SMC_CONSTANT_AS T *as_const(const T *p) {
    return (const SMC_CONSTANT_AS T *)p;
}

struct Tile {
    int i, j, k0, k1;
    int x0, y0;  // tile origin (column of the workgroup's first thread)
    bool ok;
    uint32_t pbase;
    int npg;
};

template <int PT>
__device__ __forceinline__ Tile tile_of(const KArgs &a, uint32_t bx, uint32_t by) {
    Tile t;
    const int tiles = a.tiles_x * a.tiles_y;
    int b = (int)bx;
    const int zc = b / tiles;
    b -= zc * tiles;
    const int ty = b / a.tiles_x;
    const int tx = b - ty * a.tiles_x;
    // each wave covers a kWX x (64 / kWX) patch of the tile, and each quarter
    // of the wave (16 lanes, which the texture path serves together) a 4 x 4
    // square of it: a gather costs about one cycle per cache line that a
    // quarter touches, and a square's rotated image spans fewer source rows
    // and slices than a 16-voxel row's
    const int lane = (int)(threadIdx.x % 64), wave = (int)(threadIdx.x / 64);
    t.x0 = tx * kTX;
    t.y0 = ty * kTY;
    t.i = t.x0 + (wave % (kTX / kWX)) * kWX + (lane / 16) * 4 + lane % 4;
    t.j = t.y0 + (wave / (kTX / kWX)) * (64 / kWX) + (lane % 16) / 4;
    t.ok = t.i < a.tn0 && t.j < a.tn1;
    t.k0 = zc * a.zchunk;
    t.k1 = min(t.k0 + a.zchunk, a.tn2);
    t.pbase = a.p0 + by * PT;
    t.npg = min(PT, (int)(a.p0 + a.np - t.pbase));
    return t;
}

// Particle-dependent row terms of the recipe for this thread's column.
// Slots past the end of the range repeat the last particle (their sums are
// never stored), which keeps this prologue free of branches.
template <int PT>
__device__ __forceinline__ void column_terms(const KArgs &a, const Tile &t, float mx[PT], float my[PT],
                                             float mz[PT], float ax[PT], float ay[PT], float az[PT]) {
    const float fi = (float)t.i, fj = (float)t.j;
    const uint32_t last = a.p0 + a.np - 1;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const uint32_t q = min(t.pbase + (uint32_t)p, last);
        const auto *w = as_const(a.words) + 12 * (size_t)q;
        mx[p] = fmaf(w[1], fj, fmaf(w[0], fi, w[3]));
        my[p] = fmaf(w[5], fj, fmaf(w[4], fi, w[7]));
        mz[p] = fmaf(w[9], fj, fmaf(w[8], fi, w[11]));
        ax[p] = w[2];
        ay[p] = w[6];
        az[p] = w[10];
    }
}

// Culling.  live_mask: bit p set iff particle p's image of this tile (the box of target voxels
// [i0, i1] x [j0, j1] x [k0, k1 - 1], mapped by the affine recipe) meets the
// cull box.  The image of a box under an affine map is bounded per axis by
// the image of its centre plus or minus sum_e |A_de| h_e (h the box's half
// extents); both are formed in FP32, whose rounding (a few ulps of values
// below 2^16) stays far inside the margin, so a tile is skipped only if no
// sample of it can land in the box.  Uniform across the workgroup.
//
// Centre and half extents of the box of target voxels [lo, hi] (inclusive).
__device__ __forceinline__ void box_centre(const int lo[3], const int hi[3], float c[3], float h[3]) {
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        c[e] = 0.5f * (float)(lo[e] + hi[e]);
        h[e] = 0.5f * (float)(hi[e] - lo[e]);
    }
}

// Whether the image of the box (centre c, half extents h) under the recipe
// words w can meet the cull box and, for masks with an occupancy table, can
// sample an occupied cell: the image's voxel indices (the nearest-neighbour
// words carry the +0.5, so a sample's index is the floor of its coordinate)
// lie in [floor(uc - r), floor(uc + r)] per axis; clipped to the source and
// taken to cells, the table's inclusion-exclusion count over that cell box is
// the number of occupied cells it holds.  None occupied: every sample reads an
// off bit and adds nothing to a or c.
template <typename P>
__device__ __forceinline__ bool box_reaches(P w, const float c[3], const float h[3], const KArgs &a) {
    bool ok = true;
    int32_t lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float uc = fmaf(w[4 * d + 2], c[2], fmaf(w[4 * d + 1], c[1], fmaf(w[4 * d], c[0], w[4 * d + 3])));
        const float r = fmaf(fabsf(w[4 * d + 2]), h[2], fmaf(fabsf(w[4 * d + 1]), h[1], fabsf(w[4 * d]) * h[0])) +
                        kCullMargin;
        ok = ok && uc + r >= a.cull_lo[d] && uc - r <= a.cull_hi[d];
        lo[d] = (int32_t)floorf(fmaxf(uc - r, 0.0f));
        hi[d] = (int32_t)floorf(fminf(uc + r, a.occ_hi[d]));
    }
    if (ok && a.occ) {
        if (lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]) return false;
        const uint32_t x0 = (uint32_t)lo[0] >> kOccShift, x1 = ((uint32_t)hi[0] >> kOccShift) + 1u;
        const uint32_t y0 = ((uint32_t)lo[1] >> kOccShift) * a.ocx, y1 = (((uint32_t)hi[1] >> kOccShift) + 1u) * a.ocx;
        const uint32_t z0 = ((uint32_t)lo[2] >> kOccShift) * a.ocxy,
                       z1 = (((uint32_t)hi[2] >> kOccShift) + 1u) * a.ocxy;
        const uint32_t *S = a.occ;
        const uint32_t n = S[z1 + y1 + x1] - S[z0 + y1 + x1] - S[z1 + y0 + x1] - S[z1 + y1 + x0] +
                           S[z0 + y0 + x1] + S[z0 + y1 + x0] + S[z1 + y0 + x0] - S[z0 + y0 + x0];
        ok = n != 0u;
    }
    return ok;
}

// Whether every sample of the box's image under the nearest-neighbour words w
// lies inside the source (0 <= u < n per axis), by the same bound.
template <typename P>
__device__ __forceinline__ bool box_inside(P w, const float c[3], const float h[3], const KArgs &a) {
    const float n[3] = {(float)a.sn0, (float)a.sn1, (float)a.sn2};
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float uc = fmaf(w[4 * d + 2], c[2], fmaf(w[4 * d + 1], c[1], fmaf(w[4 * d], c[0], w[4 * d + 3])));
        const float r = fmaf(fabsf(w[4 * d + 2]), h[2], fmaf(fabsf(w[4 * d + 1]), h[1], fabsf(w[4 * d]) * h[0])) +
                        kCullMargin;
        in = in && uc - r >= 0.0f && uc + r < n[d];
    }
    return in;
}

// The slices of the bottom and top runs (kSpanSlices each) of the tile box
// [lo, hi] that no live particle (bits of live; words w of particles 0 ..
// npg - 1) can sample an occupied cell from, by box_reaches on each run's
// box.  When no run is reached, live becomes 0.  Tiles deeper than
// kSpanMaxDepth are left whole.
template <typename P>
__device__ __forceinline__ void trim_span(const KArgs &a, P w, uint32_t npg, const int lo[3], const int hi[3],
                                          uint32_t &live, int &skip_lo, int &skip_hi) {
    const int depth = hi[2] - lo[2] + 1;
    skip_lo = skip_hi = 0;
    if (!live || depth <= kSpanSlices || depth > kSpanMaxDepth) return;
    const auto run_reaches = [&](int r0, int r1) {
        const int rl[3] = {lo[0], lo[1], lo[2] + r0}, rh[3] = {hi[0], hi[1], lo[2] + r1};
        float rc[3], rhh[3];
        box_centre(rl, rh, rc, rhh);
        bool any = false;
        for (uint32_t p = 0; p < npg && !any; ++p) any = ((live >> p) & 1u) && box_reaches(w + 12 * p, rc, rhh, a);
        return any;
    };
    while (skip_lo < depth && !run_reaches(skip_lo, min(skip_lo + kSpanSlices, depth) - 1)) skip_lo += kSpanSlices;
    if (skip_lo >= depth) {
        live = 0u;  // no run reaches an occupied cell: nothing of the tile can count
        skip_lo = 0;
        return;
    }
    int top = depth;  // runs from the top: [top - kSpanSlices, top)
    while (top - kSpanSlices > skip_lo && !run_reaches(top - kSpanSlices, top - 1)) top -= kSpanSlices;
    skip_hi = depth - top;
}

template <int PT>
__device__ __forceinline__ uint32_t live_mask(const KArgs &a, const Tile &t, uint32_t bx) {
    const int tiles = a.tiles_x * a.tiles_y;
    const int b = (int)bx % tiles;
    const int ty = b / a.tiles_x, tx = b - ty * a.tiles_x;
    const int lo[3] = {tx * kTX, ty * kTY, t.k0};
    const int hi[3] = {min(tx * kTX + kTX - 1, a.tn0 - 1), min(ty * kTY + kTY - 1, a.tn1 - 1), t.k1 - 1};
    float c[3], h[3];
    box_centre(lo, hi, c, h);
    const uint32_t last = a.p0 + a.np - 1;
    uint32_t live = 0;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const auto *w = as_const(a.words) + 12 * (size_t)min(t.pbase + (uint32_t)p, last);
        live |= (p < t.npg && box_reaches(w, c, h, a)) ? (1u << p) : 0u;
    }
    return live;
}

// ---------------------------------------------------------------- target slabs

// Stage target slices [kb, ke) of the workgroup's 32 x 8 column block (and
// its FOV when given) in LDS: slot z * 256 + row * 32 + column.  Coalesced
// 4-byte loads where rows are 4-byte aligned, bytes otherwise.  A gather
// costs about the same whatever its width, so this replaces one byte gather
// per thread and slice by a quarter of a coalesced load.  Loads past the
// volume's end read zero (bounds-checked buffer loads) and fill only slots
// of threads outside the target.
__device__ __forceinline__ void stage_target(const KArgs &a, const Tile &t, int kb, int ke,
                                             __amdgpu_buffer_rsrc_t rs_t, __amdgpu_buffer_rsrc_t rs_tf, bool tfov,
                                             uint32_t *tslab, uint32_t *fslab) {
    const uint32_t plane = (uint32_t)a.tn0 * (uint32_t)a.tn1;
    const uint32_t base = plane * (uint32_t)kb + (uint32_t)a.tn0 * (uint32_t)t.y0 + (uint32_t)t.x0;
    if ((a.tn0 & 3) == 0) {
        const uint32_t words = (uint32_t)(ke - kb) * (kThreads / 4);
        for (uint32_t d = threadIdx.x; d < words; d += kThreads) {
            const uint32_t z = d / (kThreads / 4), r = (d / (kTX / 4)) % kTY, c = d % (kTX / 4);
            const uint32_t o = base + plane * z + (uint32_t)a.tn0 * r + 4u * c;
            tslab[d] = __builtin_amdgcn_raw_buffer_load_b32(rs_t, o, 0, 0);
            if (tfov) fslab[d] = __builtin_amdgcn_raw_buffer_load_b32(rs_tf, o, 0, 0);
        }
    } else {
        const uint32_t bytes = (uint32_t)(ke - kb) * kThreads;
        for (uint32_t b = threadIdx.x; b < bytes; b += kThreads) {
            const uint32_t z = b / kThreads, r = (b / kTX) % kTY, c = b % kTX;
            const uint32_t o = base + plane * z + (uint32_t)a.tn0 * r + c;
            ((uint8_t *)tslab)[b] = (uint8_t)__builtin_amdgcn_raw_buffer_load_b8(rs_t, o, 0, 0);
            if (tfov) ((uint8_t *)fslab)[b] = (uint8_t)__builtin_amdgcn_raw_buffer_load_b8(rs_tf, o, 0, 0);
        }
    }
}

// The same with a constant b.
__device__ __forceinline__ uint32_t mad_u24v(uint32_t a, uint32_t b, uint32_t c) { return __umul24(a, b) + c; }

// ---------------------------------------------------------------- masks

// Source byte: bit 0 = inside the source FOV, bit 1 = mask on (and in FOV).
// Target byte: bit 0 = inside the target FOV, bit 1 = mask on (and in FOV).
// Per particle two packed counters: acc1 = n | a << 16, acc2 = b_ov | c << 16
// (each half counts at most one voxel per z step, and a z-chunk < 2^16).
// AC: only a and c (what Dice uses; the filter's launches), from the source
// bitmap (one bit per voxel, the "on" bit; rows of ceil(nx / 32) dwords):
// the sample is bit x % 32 of a dword, and one packed counter per particle
// takes a + 2^16 c as bit * (in-FOV + 2^16 on) of the target voxel.  The
// bitmap puts the rows of a slice 4 ceil(nx / 32) bytes apart, so the rotated
// footprint of a wave's samples spans a few cache lines instead of one or two
// per source row and slice as with a byte per voxel.
// staged (or nullptr): the key of the tile whose target slab the LDS holds,
// kept by a persistent workgroup across its items; an item whose tile has
// that key (tile_key: unique per tile among the workgroup's items) and fits
// one slab reuses the slab instead of staging it again.
template <int PT, bool AC = false, bool GIVEN = false>
__device__ __forceinline__ void mask_body(const KArgs &a, uint32_t bx, uint32_t by, uint32_t live_in = 0u,
                                          uint32_t *staged = nullptr, uint32_t tile_key = 0u) {
    const Tile t = tile_of<PT>(a, bx, by);
    // GIVEN: the cull pre-pass already tested this item (live_in != 0)
    const uint32_t live = GIVEN ? live_in : live_mask<PT>(a, t, bx);
    if (live == 0u) return;  // nothing of this tile can reach the source region
    float mx[PT], my[PT], mz[PT], ax[PT], ay[PT], az[PT];
    column_terms<PT>(a, t, mx, my, mz, ax, ay, az);
    // interior (bit kInteriorBit of a pre-pass item): every sample of the
    // live particles lies inside the source, so the inside test is dropped;
    // the other particle slots are pointed at slice n_z, whose offset
    // (n_z times the slice stride) is the bitmap's end, where loads read zero
    const bool interior = GIVEN && AC && ((live_in >> kInteriorBit) & 1u) != 0u;
    if (interior) {
#pragma unroll
        for (int p = 0; p < PT; ++p)
            if (!((live >> p) & 1u)) {
                ax[p] = ay[p] = az[p] = mx[p] = my[p] = 0.0f;
                mz[p] = (float)a.sn2;
            }
    }
    if constexpr (PT > 4) {
        // the per-particle slopes are uniform; with many particles they would
        // crowd the scalar registers out (and be spilled to vector lanes)
#pragma unroll
        for (int p = 0; p < PT; ++p) asm("" : "+v"(ax[p]), "+v"(ay[p]), "+v"(az[p]));
    }
    uint32_t acc1[PT], acc2[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) acc1[p] = acc2[p] = 0u;
    {
        // prepared source bytes through a bounds-checked buffer with 32-bit
        // offsets: an outside sample may form any offset, its result is masked
        const uint32_t sn0 = AC ? a.ysb : (uint32_t)a.sn0, sn01 = AC ? a.zsb : (uint32_t)a.sn0 * (uint32_t)a.sn1;
        const int nbytes = AC ? (int)a.src_bytes : a.sn0 * a.sn1 * a.sn2;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            AC ? const_cast<void *>(a.src_packed) : (void *)const_cast<uint8_t *>(a.src), (short)0, nbytes,
            kBufferWord3);
        // nearest (the words carry +0.5): inside iff 0 <= u < n, one unsigned
        // compare of bit patterns per axis (coordinates are never -0)
        const uint32_t nxb = __float_as_uint((float)a.sn0), nyb = __float_as_uint((float)a.sn1),
                       nzb = __float_as_uint((float)a.sn2);
        const __amdgpu_buffer_rsrc_t rs_t = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t *>(a.tgt), (short)0, a.tn0 * a.tn1 * a.tn2, kBufferWord3);
        __shared__ uint32_t tslab[kSlab * kThreads / 4];
        const uint8_t *tslab8 = (const uint8_t *)tslab;
        const uint32_t col = (uint32_t)(t.j - t.y0) * kTX + (uint32_t)(t.i - t.x0);
        const bool one_slab = t.k1 - t.k0 <= kSlab;
        // a pre-pass item's span: the slices of the tile some live particle
        // can sample an occupied cell from (the whole tile otherwise)
        const int kbeg = GIVEN ? t.k0 + (int)((live_in >> kSpanLoBit) & kSpanMask) : t.k0;
        const int kend = GIVEN ? t.k1 - (int)((live_in >> kSpanHiBit) & kSpanMask) : t.k1;
        for (int kb = t.k0; kb < t.k1; kb += kSlab) {
            const int ke = min(kb + kSlab, t.k1);
            if (!(staged && one_slab && *staged == tile_key)) {
                __syncthreads();  // every thread is done with the previous slab
                stage_target(a, t, kb, ke, rs_t, rs_t, false, tslab, tslab);
                __syncthreads();
                if (staged) *staged = one_slab ? tile_key : 0xFFFFFFFFu;
            } else {
                __syncthreads();  // the previous item's reduction slots are read
            }
            if (!t.ok) continue;
            const auto slices = [&](auto interior_tag) {
            constexpr bool INTERIOR = decltype(interior_tag)::value;
            for (int k = max(kb, kbeg); k < min(ke, kend); ++k) {
                const uint32_t tb = tslab8[(uint32_t)(k - kb) * kThreads + col];
                const uint32_t keep = (tb & 1u) ? 3u : 0u;
                const bool ton = (tb & 2u) != 0u;
                // AC: a source bit adds 1 to a where the target voxel is in its
                // FOV and 2^16 to c where it is on (bit 1 implies bit 0)
                const uint32_t tmul = (tb & 1u) + ((tb & 2u) << 15);
                const float fk = (float)k;
                // offsets of all PT samples first, then every load, then the sums
                uint32_t off[PT], ix[PT];
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    const float ux = fmaf(ax[p], fk, mx[p]);
                    const float uy = fmaf(ay[p], fk, my[p]);
                    const float uz = fmaf(az[p], fk, mz[p]);
                    // 24-bit multiply-adds: exact inside (offsets below 2^32);
                    // outside samples (and particles culled for this tile) load
                    // from the buffer's end: zero, no cache lines touched, so they
                    // count nothing
                    if constexpr (AC) {
                        // byte offset of dword x / 32 of the row; the bit index is
                        // x % 32 (the low five bits of the offset operand)
                        ix[p] = floor_u32(ux);
                        off[p] = mad_u24(floor_u32(uz), sn01, mad_u24(floor_u32(uy), sn0, (ix[p] >> 3) & ~3u));
                    } else {
                        off[p] = mad_u24(floor_u32(uz), sn01, mad_u24(floor_u32(uy), sn0, floor_u32(ux)));
                    }
                    if constexpr (!INTERIOR) {
                        const bool in = ((live >> p) & 1u) & (__float_as_uint(ux) < nxb) &
                                        (__float_as_uint(uy) < nyb) & (__float_as_uint(uz) < nzb);
                        off[p] = in ? off[p] : nbytes;
                    }
                }
                uint32_t val[PT];
#pragma unroll
                for (int p = 0; p < PT; ++p)
                    val[p] = AC ? __builtin_amdgcn_raw_buffer_load_b32(rs, off[p], 0, 0)
                                : __builtin_amdgcn_raw_buffer_load_b8(rs, off[p], 0, 0);
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    if constexpr (AC) {
                        acc1[p] = mad_u24v(__builtin_amdgcn_ubfe(val[p], ix[p], 1u), tmul, acc1[p]);
                    } else {
                        // v in 0..3 (bit 0 in both FOVs, bit 1 also on); inc = (v & 1) +
                        // (v >> 1) 2^16 = v + (v >> 1) (2^16 - 2)
                        const uint32_t v = val[p] & keep;
                        const uint32_t inc = mad_u24v(v >> 1, 65534u, v);
                        acc1[p] += inc;
                        acc2[p] += ton ? inc : 0u;
                    }
                }
            }
            };
            if (interior) slices(std::true_type{});
            else slices(std::false_type{});
        }
    }
    __shared__ unsigned long long red[kWaves][PT][4];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        // AC: a wave's halves stay below 64 x 256 < 2^16, so one sum serves both
        const uint32_t ac = AC ? wave_sum(acc1[p]) : 0u;
        const uint32_t n = AC ? 0u : wave_sum(acc1[p] & 0xFFFFu);
        const uint32_t aa = AC ? ac & 0xFFFFu : wave_sum(acc1[p] >> 16);
        const uint32_t b = AC ? 0u : wave_sum(acc2[p] & 0xFFFFu);
        const uint32_t c = AC ? ac >> 16 : wave_sum(acc2[p] >> 16);
        if (lane == 0) {
            red[wave][p][0] = n;
            red[wave][p][1] = aa;
            red[wave][p][2] = c;
            red[wave][p][3] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)(PT * 4)) {
        const int p = threadIdx.x / 4, m = threadIdx.x % 4;
        if (p < t.npg) {
            unsigned long long s = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s += red[w][p][m];
            if (s) atomicAdd(a.sums + 6 * (size_t)(t.pbase + p) + m, s);
        }
    }
}

// ---------------------------------------------------------------- images


typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Packed corners through a buffer resource with 32-bit byte offsets:
// off = the base element, dy / dz the byte steps to the element one row /
// one slice up (zero on the last row / slice, where the weight is zero).
template <int LAYOUT>
__device__ __forceinline__ void corners_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t dy, uint32_t dz,
                                            float v[8], uint64_t sentinel, bool &sent_ok) {
    if (LAYOUT == kLayoutPairX) {
        const uint32_t a = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
        const uint32_t b = __builtin_amdgcn_raw_buffer_load_b16(rs, off + dy, 0, 0);
        const uint32_t c = __builtin_amdgcn_raw_buffer_load_b16(rs, off + dz, 0, 0);
        const uint32_t d = __builtin_amdgcn_raw_buffer_load_b16(rs, off + dz + dy, 0, 0);
        const uint32_t st = (uint32_t)(sentinel & 0xFFFFu);
        sent_ok = (a != st) & (b != st) & (c != st) & (d != st);
        v[0] = (float)(a & 0xFFu);
        v[1] = (float)(a >> 8);
        v[2] = (float)(b & 0xFFu);
        v[3] = (float)(b >> 8);
        v[4] = (float)(c & 0xFFu);
        v[5] = (float)(c >> 8);
        v[6] = (float)(d & 0xFFu);
        v[7] = (float)(d >> 8);
    } else {
        uint32_t lo, hi;
        if (LAYOUT == kLayoutQuadXY) {
            lo = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
            hi = __builtin_amdgcn_raw_buffer_load_b32(rs, off + dz, 0, 0);
            const uint32_t st = (uint32_t)sentinel;
            sent_ok = (lo != st) & (hi != st);
        } else {
            const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
            lo = w.x;
            hi = w.y;
            sent_ok = (lo != (uint32_t)sentinel) | (hi != (uint32_t)(sentinel >> 32));
        }
        v[0] = (float)(lo & 0xFFu);
        v[1] = (float)((lo >> 8) & 0xFFu);
        v[2] = (float)((lo >> 16) & 0xFFu);
        v[3] = (float)(lo >> 24);
        v[4] = (float)(hi & 0xFFu);
        v[5] = (float)((hi >> 8) & 0xFFu);
        v[6] = (float)((hi >> 16) & 0xFFu);
        v[7] = (float)(hi >> 24);
    }
}

// The four x-lerps fma(fx, b - a, a) of a packed 2x2x2 neighbourhood (lo:
// bytes v0..v3 of slice z, hi: v4..v7 of slice z + 1).  Each byte b becomes
// the half 1024 + b with one byte permute (high byte 0x64); packed half
// subtractions give b - a and a exactly (integers below 2048), and the mixed-
// precision FMA forms f * (b - a) + a in FP32 with one rounding -- the same
// value as the FP32 formula, in 3 operations per lerp instead of 4.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ half2v as_half2(uint32_t u) {
    half2v h;
    __builtin_memcpy(&h, &u, sizeof h);
    return h;
}

__device__ __forceinline__ void x_lerps(uint32_t lo, uint32_t hi, float f, float &x00, float &x10, float &x01,
                                        float &x11) {
    constexpr uint32_t kMagic = 0x64646464u;
    const half2v a0 = as_half2(__builtin_amdgcn_perm(kMagic, lo, 0x04020400u));  // (v0, v2)
    const half2v b0 = as_half2(__builtin_amdgcn_perm(kMagic, lo, 0x04030401u));  // (v1, v3)
    const half2v a1 = as_half2(__builtin_amdgcn_perm(kMagic, hi, 0x04020400u));  // (v4, v6)
    const half2v b1 = as_half2(__builtin_amdgcn_perm(kMagic, hi, 0x04030401u));  // (v5, v7)
    const half2v k1024 = {(_Float16)1024.0f, (_Float16)1024.0f};
    const half2v d0 = b0 - a0, d1 = b1 - a1;
    const half2v v0 = a0 - k1024, v1 = a1 - k1024;
    x00 = fmaf(f, (float)d0.x, (float)v0.x);
    x10 = fmaf(f, (float)d0.y, (float)v0.y);
    x01 = fmaf(f, (float)d1.x, (float)v1.x);
    x11 = fmaf(f, (float)d1.y, (float)v1.y);
}

// The four x-lerps from a lerp-layout element: w0, w1 hold the starts a and
// w2, w3 the steps d (times 256, in half precision) of the rows (y, z),
// (y + 1, z), (y, z + 1), (y + 1, z + 1).  One mixed-precision FMA per lerp
// forms f * 256 d + 256 a in FP32 with one rounding; scaling by a power of
// two commutes with the rounding, so this is exactly 256 fma(f, d, a).
__device__ __forceinline__ void x_lerps_scaled(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, float f,
                                               float &x00, float &x10, float &x01, float &x11) {
    const half2v a0 = as_half2(w0), a1 = as_half2(w1), d0 = as_half2(w2), d1 = as_half2(w3);
    x00 = fmaf(f, (float)d0.x, (float)a0.x);
    x10 = fmaf(f, (float)d0.y, (float)a0.y);
    x01 = fmaf(f, (float)d1.x, (float)a1.x);
    x11 = fmaf(f, (float)d1.y, (float)a1.y);
}

// Raw packed corner words (quads and octets): lo = slice z, hi = slice z + 1.
template <int LAYOUT>
__device__ __forceinline__ void corner_words(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t dz, uint32_t &lo,
                                             uint32_t &hi, uint64_t sentinel, bool &sent_ok) {
    if (LAYOUT == kLayoutQuadXY) {
        lo = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        hi = __builtin_amdgcn_raw_buffer_load_b32(rs, off + dz, 0, 0);
        const uint32_t st = (uint32_t)sentinel;
        sent_ok = (lo != st) & (hi != st);
    } else {
        const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        lo = w.x;
        hi = w.y;
        sent_ok = (lo != (uint32_t)sentinel) | (hi != (uint32_t)(sentinel >> 32));
    }
}

// The eight trilinear corners of base voxel (ix, iy, iz) as floats, read from
// one of the source layouts (corners beyond the last voxel repeat it; their
// weight is zero there):
//   raw    uint8 per voxel, eight byte gathers
//   pairx  uint16 (v[x], v[x+1]), four gathers
//   quadxy uint32 (v[x,y], v[x+1,y], v[x,y+1], v[x+1,y+1]), two gathers
//   oct    uint64 (quad of slice z, quad of slice z+1), one gather
//   lerp   the oct cell as four x-lerp starts and steps times 256 in half
//          precision (16 bytes), one gather; see x_lerps_scaled
template <int LAYOUT>
__device__ __forceinline__ void corners(const void *src, uint32_t base, uint32_t dx, uint32_t dy, uint32_t dz,
                                        float v[8], uint64_t sentinel, bool &sent_ok) {
    if (LAYOUT == kLayoutRaw) {
        const uint8_t *S = (const uint8_t *)src + base;
        v[0] = (float)S[0];
        v[1] = (float)S[dx];
        v[2] = (float)S[dy];
        v[3] = (float)S[dy + dx];
        v[4] = (float)S[dz];
        v[5] = (float)S[dz + dx];
        v[6] = (float)S[dz + dy];
        v[7] = (float)S[dz + dy + dx];
        sent_ok = true;
    } else if (LAYOUT == kLayoutPairX) {
        const uint16_t *S = (const uint16_t *)src + base;
        const uint32_t a = S[0], b = S[dy], c = S[dz], d = S[dz + dy];
        const uint32_t st = (uint32_t)(sentinel & 0xFFFFu);
        sent_ok = a != st && b != st && c != st && d != st;
        v[0] = (float)(a & 0xFFu);
        v[1] = (float)(a >> 8);
        v[2] = (float)(b & 0xFFu);
        v[3] = (float)(b >> 8);
        v[4] = (float)(c & 0xFFu);
        v[5] = (float)(c >> 8);
        v[6] = (float)(d & 0xFFu);
        v[7] = (float)(d >> 8);
    } else {
        uint32_t lo, hi;
        if (LAYOUT == kLayoutQuadXY) {
            const uint32_t *S = (const uint32_t *)src + base;
            lo = S[0];
            hi = S[dz];
            const uint32_t st = (uint32_t)sentinel;
            sent_ok = lo != st && hi != st;
        } else {
            const uint2 w = ((const uint2 *)src)[base];
            lo = w.x;
            hi = w.y;
            sent_ok = lo != (uint32_t)sentinel || hi != (uint32_t)(sentinel >> 32);
        }
        v[0] = (float)(lo & 0xFFu);
        v[1] = (float)((lo >> 8) & 0xFFu);
        v[2] = (float)((lo >> 16) & 0xFFu);
        v[3] = (float)(lo >> 24);
        v[4] = (float)(hi & 0xFFu);
        v[5] = (float)((hi >> 8) & 0xFFu);
        v[6] = (float)((hi >> 16) & 0xFFu);
        v[7] = (float)(hi >> 24);
    }
}

struct Sums6 {
    uint32_t n, s, t, tt, st;
    unsigned long long ss;
};

// Sums per particle over the overlap: n, s, t, s^2, t^2, s t with s the
// sampled source value in units of 1/256 (exact: s_fx = floor(256 s + 0.5)).
// TRI: trilinear (inside iff 0 <= u <= n - 1 and the eight corners in the
// source FOV); otherwise nearest (the words carry the +0.5 shift).
// ACC 0: the six moments (NCC / SSD); ACC 1 (trilinear only): the joint
// histogram of the mutual-information score, counted in LDS per workgroup and
// added to the particle's histogram in global memory (bins left at zero are
// skipped).
template <int PT, int LAYOUT, bool TRI, int VMODE, int ACC = 0>
__device__ __forceinline__ void image_body(const KArgs &a, uint32_t bx, uint32_t by) {
    constexpr bool SOK = VMODE == 1;
    constexpr bool HIST = ACC == 1;
    constexpr int kHB = kMiBins * kMiBins;
    __shared__ uint32_t lhist[HIST ? PT : 1][HIST ? kHB : 1];
    const Tile t = tile_of<PT>(a, bx, by);
    const uint32_t live = live_mask<PT>(a, t, bx);
    if (live == 0u) return;  // every sample of this tile falls outside the source
    if constexpr (HIST) {
        for (uint32_t q = threadIdx.x; q < (uint32_t)(PT * kHB); q += kThreads) lhist[q / kHB][q % kHB] = 0u;
        __syncthreads();
    }
    float mx[PT], my[PT], mz[PT], ax[PT], ay[PT], az[PT];
    column_terms<PT>(a, t, mx, my, mz, ax, ay, az);
    Sums6 acc[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        acc[p].n = acc[p].s = acc[p].t = acc[p].tt = acc[p].st = 0u;
        acc[p].ss = 0ull;
    }
    {
        const uint32_t plane = (uint32_t)a.tn0 * (uint32_t)a.tn1;
        const uint32_t sn0 = (uint32_t)a.sn0, sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
        const float ex = (float)(a.sn0 - 1), ey = (float)(a.sn1 - 1), ez = (float)(a.sn2 - 1);
        const bool tfov = a.tgt_fov != nullptr;
        constexpr uint32_t kElemShift =
            LAYOUT == kLayoutLerp ? 4u
                                  : (LAYOUT == kLayoutOct || LAYOUT == kLayoutOctTile
                                         ? 3u
                                         : (LAYOUT == kLayoutQuadXY ? 2u : 1u));
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(a.src_packed), (short)0, (int)a.src_bytes,
                                              kBufferWord3);
        const __amdgpu_buffer_rsrc_t rs_ok = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t *>(a.src_ok), (short)0, a.sn0 * a.sn1 * a.sn2, kBufferWord3);
        const uint32_t exb = __float_as_uint(ex), eyb = __float_as_uint(ey), ezb = __float_as_uint(ez);
        // n and t of the overlap packed in one register: n < 2^9 and t < 2^16
        // for a z-chunk of at most 256 slices
        uint32_t nt[PT];
#pragma unroll
        for (int p = 0; p < PT; ++p) nt[p] = 0u;
        // mutual information: each thread holds its current run of samples
        // falling into one bin (neighbouring slices often share a bin) and
        // adds the run to the LDS histogram when the bin changes, so fewer
        // lanes contend for the same LDS words
        uint32_t rbin[HIST ? PT : 1], rcnt[HIST ? PT : 1];
#pragma unroll
        for (int p = 0; p < (HIST ? PT : 1); ++p) rbin[p] = rcnt[p] = 0u;
        // The target column block is staged in LDS a slab of kSlab slices at a
        // time with coalesced loads (four bytes per lane where rows are 4-byte
        // aligned): a gather costs the same whatever its width, and the
        // per-slice target byte would otherwise be a fifth of the gathers.
        // Loads past the volume's end read zero (bounds-checked buffer loads)
        // and land only in slots of threads outside the target.
        const int tbytes = a.tn0 * a.tn1 * a.tn2;
        const __amdgpu_buffer_rsrc_t rs_t =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(a.tgt), (short)0, tbytes, kBufferWord3);
        const __amdgpu_buffer_rsrc_t rs_tf = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t *>(a.tgt_fov), (short)0, tfov ? tbytes : 0, kBufferWord3);
        __shared__ uint32_t tslab[kSlab * kThreads / 4], fslab[kSlab * kThreads / 4];
        const uint8_t *tslab8 = (const uint8_t *)tslab, *fslab8 = (const uint8_t *)fslab;
        const uint32_t col = (uint32_t)(t.j - t.y0) * kTX + (uint32_t)(t.i - t.x0);
        for (int kb = t.k0; kb < t.k1; kb += kSlab) {
            const int ke = min(kb + kSlab, t.k1);
            __syncthreads();  // every thread is done with the previous slab
            stage_target(a, t, kb, ke, rs_t, rs_tf, tfov, tslab, fslab);
            __syncthreads();
            if (!t.ok) continue;
        for (int k = kb; k < ke; ++k) {
            const uint32_t sidx = (uint32_t)(k - kb) * kThreads + col;
            const uint32_t tv = tslab8[sidx];
            if (tfov && fslab8[sidx] == 0) continue;
            const uint32_t tv2 = tv * tv;
            const uint32_t nt1 = 1u + (tv << 9);
            const float fk = (float)k;
            if (TRI && LAYOUT != kLayoutRaw) {
                // all PT samples: coordinates and offsets, all loads issued before
                // any use, then sums predicated on inside && FOV-valid && particle
                // live for this tile
                float fxa[PT], fya[PT], fza[PT];
                uint32_t off[PT], ddy[PT], ddz[PT], vidx[PT];
                bool in[PT];
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    const float ux = fmaf(ax[p], fk, mx[p]);
                    const float uy = fmaf(ay[p], fk, my[p]);
                    const float uz = fmaf(az[p], fk, mz[p]);
                    // 0 <= u <= n - 1 as one unsigned compare of bit patterns: the
                    // coordinates are never -0 (the offset words are normalised to
                    // +0) and negative ones have the sign bit set
                    in[p] = ((live >> p) & 1u) & (__float_as_uint(ux) <= exb) & (__float_as_uint(uy) <= eyb) &
                            (__float_as_uint(uz) <= ezb);
                    // samples outside produce arbitrary offsets: the buffer loads
                    // are bounds-checked (zero beyond the end) and the sums ignore them
                    const uint32_t ix = floor_u32(ux), iy = floor_u32(uy), iz = floor_u32(uz);
                    fxa[p] = __builtin_amdgcn_fractf(ux);
                    fya[p] = __builtin_amdgcn_fractf(uy);
                    fza[p] = __builtin_amdgcn_fractf(uz);
                    if (LAYOUT == kLayoutOctTile) {
                        // (ix / 4) * 128 + (ix % 4) * 8 + (iy / 4) * 4 ysb + (iy % 4) * 32
                        // + iz * zsb, with ysb = 32 ceil(nx / 4) (signed 24-bit
                        // multiplies; arbitrary but in-buffer-checked for outside samples)
                        uint32_t o = __mul24((int)(ix & 3u), -24) + (ix << 5);
                        o += __mul24((int)(iy & 3u), 32 - (int)a.ysb);
                        off[p] = o + __umul24(iy, a.ysb) + __umul24(iz, a.zsb);
                        if (SOK) vidx[p] = ix + sn0 * iy + sn01 * iz;
                    } else {
                        off[p] = mad_u24(iz, a.zsb, mad_u24(iy, a.ysb, ix << kElemShift));
                        if (SOK) vidx[p] = off[p] >> kElemShift;
                    }
                    // samples outside the source box would gather from wrapped
                    // offsets near the volume (extra cache lines); send them to
                    // the buffer's end, where the load reads zero unfetched
                    if (LAYOUT == kLayoutOct || LAYOUT == kLayoutOctTile || LAYOUT == kLayoutLerp)
                        off[p] = in[p] ? off[p] : a.src_bytes;
                    if (LAYOUT == kLayoutPairX) ddy[p] = iy < (uint32_t)(a.sn1 - 1) ? a.ysb : 0u;
                    if (LAYOUT == kLayoutPairX || LAYOUT == kLayoutQuadXY)
                        ddz[p] = iz < (uint32_t)(a.sn2 - 1) ? a.zsb : 0u;
                }
                uint32_t okv[PT];
                float v[PT][8];
                uint32_t wlo[PT], whi[PT], wd0[PT], wd1[PT];
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    bool sent_ok;
                    if constexpr (LAYOUT == kLayoutPairX) {
                        corners_buf<LAYOUT>(rs, off[p], ddy[p], ddz[p], v[p], a.sentinel, sent_ok);
                    } else if constexpr (LAYOUT == kLayoutLerp) {
                        const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rs, off[p], 0, 0);
                        wlo[p] = w.x;
                        whi[p] = w.y;
                        wd0[p] = w.z;
                        wd1[p] = w.w;
                        sent_ok = w.x != kLerpSentinel;
                    } else {
                        corner_words<LAYOUT>(rs, off[p], LAYOUT == kLayoutQuadXY ? ddz[p] : 0u, wlo[p], whi[p],
                                             a.sentinel, sent_ok);
                    }
                    okv[p] = SOK ? __builtin_amdgcn_raw_buffer_load_b8(rs_ok, vidx[p], 0, 0)
                                 : (VMODE == 2 ? (sent_ok ? 1u : 0u) : 1u);
                }
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    float x00, x10, x01, x11;
                    if constexpr (LAYOUT == kLayoutPairX) {
                        x00 = fmaf(fxa[p], v[p][1] - v[p][0], v[p][0]);
                        x10 = fmaf(fxa[p], v[p][3] - v[p][2], v[p][2]);
                        x01 = fmaf(fxa[p], v[p][5] - v[p][4], v[p][4]);
                        x11 = fmaf(fxa[p], v[p][7] - v[p][6], v[p][6]);
                    } else if constexpr (LAYOUT == kLayoutLerp) {
                        x_lerps_scaled(wlo[p], whi[p], wd0[p], wd1[p], fxa[p], x00, x10, x01, x11);
                    } else {
                        x_lerps(wlo[p], whi[p], fxa[p], x00, x10, x01, x11);
                    }
                    const float y0 = fmaf(fya[p], x10 - x00, x00);
                    const float y1 = fmaf(fya[p], x11 - x01, x01);
                    const float sv = fmaf(fza[p], y1 - y0, y0);
                    // s_fx = floor(fl(256 s + 0.5)): 256 s is exact, so one fused
                    // step equals the multiply-add; the lerp layout's samples
                    // already carry the factor 256 and take a separate FP32 add
                    // (a rounding instruction that forms floor(x + 0.5) exactly
                    // would differ where x + 0.5 rounds up to an integer)
                    const uint32_t sfx0 =
                        LAYOUT == kLayoutLerp ? (uint32_t)(sv + 0.5f) : (uint32_t)fmaf(sv, 256.0f, 0.5f);
                    const bool valid = in[p] & (okv[p] != 0u);
                    if constexpr (HIST) {
                        if (valid) {
                            const uint32_t bin = (sfx0 >> 11) * kMiBins + (tv >> 3);
                            if (bin != rbin[p]) {
                                if (rcnt[p]) atomicAdd(&lhist[p][rbin[p]], rcnt[p]);
                                rbin[p] = bin;
                                rcnt[p] = 0u;
                            }
                            rcnt[p] += 1u;
                        }
                    } else if (valid) {
                        // under the lane mask: no selects on the five updates
                        nt[p] += nt1;
                        acc[p].s += sfx0;
                        acc[p].ss += (unsigned long long)sfx0 * sfx0;
                        acc[p].tt += tv2;
                        acc[p].st += __umul24(sfx0, tv);  // s_fx < 2^16, t < 2^8
                    }
                }
            } else if (TRI) {
                // raw bytes: eight gathers per sample through 64-bit addresses
                float fxa[PT], fya[PT], fza[PT];
                uint32_t base[PT], ddx[PT], ddy[PT], ddz[PT];
                bool in[PT];
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    const float ux = fmaf(ax[p], fk, mx[p]);
                    const float uy = fmaf(ay[p], fk, my[p]);
                    const float uz = fmaf(az[p], fk, mz[p]);
                    const float cx = __builtin_amdgcn_fmed3f(ux, 0.0f, ex);
                    const float cy = __builtin_amdgcn_fmed3f(uy, 0.0f, ey);
                    const float cz = __builtin_amdgcn_fmed3f(uz, 0.0f, ez);
                    in[p] = ((live >> p) & 1u) & (cx == ux) & (cy == uy) & (cz == uz);
                    const uint32_t ix = floor_u32(cx), iy = floor_u32(cy), iz = floor_u32(cz);
                    fxa[p] = __builtin_amdgcn_fractf(cx);
                    fya[p] = __builtin_amdgcn_fractf(cy);
                    fza[p] = __builtin_amdgcn_fractf(cz);
                    base[p] = ix + sn0 * iy + sn01 * iz;
                    ddx[p] = ix < (uint32_t)(a.sn0 - 1) ? 1u : 0u;
                    ddy[p] = iy < (uint32_t)(a.sn1 - 1) ? sn0 : 0u;
                    ddz[p] = iz < (uint32_t)(a.sn2 - 1) ? sn01 : 0u;
                }
                uint32_t okv[PT];
                float v[PT][8];
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    bool sent_ok;
                    corners<kLayoutRaw>(a.src_packed, base[p], ddx[p], ddy[p], ddz[p], v[p], a.sentinel, sent_ok);
                    okv[p] = SOK ? (uint32_t)a.src_ok[base[p]] : 1u;
                }
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    const float x00 = fmaf(fxa[p], v[p][1] - v[p][0], v[p][0]);
                    const float x10 = fmaf(fxa[p], v[p][3] - v[p][2], v[p][2]);
                    const float x01 = fmaf(fxa[p], v[p][5] - v[p][4], v[p][4]);
                    const float x11 = fmaf(fxa[p], v[p][7] - v[p][6], v[p][6]);
                    const float y0 = fmaf(fya[p], x10 - x00, x00);
                    const float y1 = fmaf(fya[p], x11 - x01, x01);
                    const float sv = fmaf(fza[p], y1 - y0, y0);
                    const uint32_t sfx0 = (uint32_t)fmaf(sv, 256.0f, 0.5f);
                    const bool valid = in[p] & (okv[p] != 0u);
                    const uint32_t sfx = valid ? sfx0 : 0u;
                    if constexpr (HIST) {
                        if (valid) atomicAdd(&lhist[p][(sfx0 >> 11) * kMiBins + (tv >> 3)], 1u);
                    } else {
                        nt[p] += valid ? nt1 : 0u;
                        acc[p].s += sfx;
                        acc[p].ss += (unsigned long long)sfx * sfx;
                        acc[p].tt += valid ? tv2 : 0u;
                        acc[p].st += sfx * tv;
                    }
                }
            } else {
#pragma unroll
                for (int p = 0; p < PT; ++p) {
                    if ((live >> p) & 1u) {
                        const float ux = fmaf(ax[p], fk, mx[p]);
                        const float uy = fmaf(ay[p], fk, my[p]);
                        const float uz = fmaf(az[p], fk, mz[p]);
                        const int ix = (int)floorf(ux), iy = (int)floorf(uy), iz = (int)floorf(uz);
                        if (!((uint32_t)ix < (uint32_t)a.sn0 && (uint32_t)iy < (uint32_t)a.sn1 &&
                              (uint32_t)iz < (uint32_t)a.sn2))
                            continue;
                        const uint32_t m = (uint32_t)ix + sn0 * (uint32_t)iy + sn01 * (uint32_t)iz;
                        if (SOK && a.src_ok[m] == 0) continue;
                        const uint32_t sfx = (uint32_t)a.src[m] << 8;
                        acc[p].n += 1u;
                        acc[p].s += sfx;
                        acc[p].t += tv;
                        acc[p].ss += (unsigned long long)sfx * sfx;
                        acc[p].tt += tv2;
                        acc[p].st += sfx * tv;
                    }
                }
            }
        }
        }  // slabs
        if constexpr (HIST) {
#pragma unroll
            for (int p = 0; p < PT; ++p)
                if (rcnt[p]) atomicAdd(&lhist[p][rbin[p]], rcnt[p]);
        }
#pragma unroll
        for (int p = 0; p < PT; ++p) {
            acc[p].n += nt[p] & 511u;
            acc[p].t += nt[p] >> 9;
        }
    }
    if constexpr (HIST) {
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < (uint32_t)(PT * kHB); q += kThreads) {
            const uint32_t p = q / kHB, b = q % kHB, v = lhist[p][b];
            if (v != 0u && (int)p < t.npg) atomicAdd(a.hist + (size_t)kHB * (t.pbase + p) + b, v);
        }
        return;
    }
    __shared__ unsigned long long red[kWaves][PT][6];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const uint32_t n = wave_sum(acc[p].n);
        const uint32_t s1 = wave_sum(acc[p].s);
        const uint32_t t1 = wave_sum(acc[p].t);
        const unsigned long long s2 = wave_sum(acc[p].ss);
        const uint32_t t2 = wave_sum(acc[p].tt);
        const unsigned long long st = wave_sum((unsigned long long)acc[p].st);
        if (lane == 0) {
            red[wave][p][0] = n;
            red[wave][p][1] = s1;
            red[wave][p][2] = t1;
            red[wave][p][3] = s2;
            red[wave][p][4] = t2;
            red[wave][p][5] = st;
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)(PT * 6)) {
        const int p = threadIdx.x / 6, m = threadIdx.x % 6;
        if (p < t.npg) {
            unsigned long long s = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s += red[w][p][m];
            if (s) atomicAdd(a.sums + 6 * (size_t)(t.pbase + p) + m, s);
        }
    }
}

// XCD-aware order of a one-dimensional grid of tiles x particle groups.
// The dispatcher hands workgroup b to XCD b % 8; XCD x is given the x-th
// contiguous eighth of the work sequence w = tile * groups + group, so it
// sweeps a few tiles at a time across all particle groups.  The particles
// of one filter are clustered, so the source footprint of the tiles in
// flight on an XCD stays within its L2 instead of every XCD streaming the
// whole source once per particle group.
__device__ __forceinline__ void xcd_order(uint32_t b, uint32_t total, uint32_t groups, uint32_t *bx,
                                          uint32_t *by) {
    const uint32_t x = b % 8u, r = b / 8u;
    const uint32_t q = total / 8u, rem = total % 8u;
    const uint32_t w = x * q + min(x, rem) + r;
    *bx = w / groups;
    *by = w - *bx * groups;
}

template <int PT, bool AC>
__global__ __launch_bounds__(kThreads) void k_score_mask(const KArgs a) {
    uint32_t bx, by;
    xcd_order(blockIdx.x, gridDim.x, (a.np + PT - 1) / PT, &bx, &by);
    mask_body<PT, AC>(a, bx, by);
}

// The octet variants with four particles per workgroup fit 72 VGPRs without
// spilling: ask for the seven waves per SIMD that allows.
template <int PT, int LAYOUT, int VMODE, int ACC>
constexpr int kImageWaves =
    PT == 4 && (LAYOUT == kLayoutOct || LAYOUT == kLayoutOctTile) && VMODE != 1 && ACC == 0
        ? 7
        : (PT == 4 && LAYOUT == kLayoutLerp && VMODE != 1 && ACC == 0 ? 6 : 1);

template <int PT, int LAYOUT, bool TRI, int VMODE, int ACC = 0>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kImageWaves<PT, LAYOUT, VMODE, ACC>)))
void k_score_image(const KArgs a) {
    uint32_t bx, by;
    xcd_order(blockIdx.x, gridDim.x, (a.np + PT - 1) / PT, &bx, &by);
    image_body<PT, LAYOUT, TRI, VMODE, ACC>(a, bx, by);
}

// ---------------------------------------------------------------- culled item lists

// Most (tile, particle group) items of a filter's mask launch cannot reach
// the source mask's bounding box (a concentrated cloud maps most tiles
// outside it).  Instead of a grid of one workgroup per item, most of which
// would only run the cull test and leave, a pre-pass tests every item on its
// own lane and appends the live ones, with their masks, to eight lists --
// list x holds the live items of the x-th contiguous eighth of the item
// sequence, the part the XCD-aware grid gives XCD x -- and a persistent grid
// takes items from its XCD's list through an atomic counter, then helps the
// other lists.  Sums are integer additions, so the result does not depend on
// which workgroup takes which item.  An item whose live particles all map the
// tile inside the source (by the cull's bound) is marked interior, and its
// samples skip the inside test: three compares and a select per sample.  The
// pre-pass also tests the tile's bottom and top runs of kSpanSlices slices
// with the same bound and trims those no live particle reaches.
constexpr uint32_t kListStride = 32;  // counter words 128 bytes apart

__device__ __forceinline__ uint32_t list_begin(uint32_t total, uint32_t x) {
    const uint32_t q = total / 8u, rem = total % 8u;
    return x * q + min(x, rem);
}

// work (or nullptr): adds the particle x voxel pairs of the live particles of
// the items (evaluated), of all their particles (covered) and of the live
// particles of interior items (interior), one atomic per count and wave into
// one of kWorkSlots counter triples (each on its own cache line, so the waves'
// atomics do not queue on one address).
template <int PT>
__global__ __launch_bounds__(256) void k_cull_items(const KArgs a, uint32_t total, uint2 *items, uint32_t *counts,
                                                    unsigned long long *work) {
    static_assert(PT <= (int)kInteriorBit, "particle bits below the interior bit");
    const uint32_t w = blockIdx.x * 256u + threadIdx.x;
    const uint32_t groups = (a.np + PT - 1) / PT;
    uint32_t live = 0u, x = 0u;
    unsigned long long evaluated = 0ull, covered = 0ull, interior = 0ull;
    if (w < total) {
        const uint32_t bx = w / groups, by = w - bx * groups;
        const int tiles = a.tiles_x * a.tiles_y;
        const int zc = (int)bx / tiles, b = (int)bx - zc * tiles;
        const int ty = b / a.tiles_x, tx = b - ty * a.tiles_x;
        const int k0 = zc * a.zchunk;
        const int lo[3] = {tx * kTX, ty * kTY, k0};
        const int hi[3] = {min(tx * kTX + kTX - 1, a.tn0 - 1), min(ty * kTY + kTY - 1, a.tn1 - 1),
                           min(k0 + a.zchunk, a.tn2) - 1};
        float c[3], h[3];
        box_centre(lo, hi, c, h);
        const uint32_t pbase = a.p0 + by * PT, npg = min((uint32_t)PT, a.p0 + a.np - pbase);
        bool inside = true;
        for (uint32_t p = 0; p < npg; ++p)
            if (box_reaches(a.words + 12 * (size_t)(pbase + p), c, h, a)) {
                live |= 1u << p;
                inside = inside && box_inside(a.words + 12 * (size_t)(pbase + p), c, h, a);
            }
        while (x < 7u && w >= list_begin(total, x + 1u)) ++x;
        const int depth = hi[2] - lo[2] + 1;
        const unsigned long long area = (unsigned long long)(hi[0] - lo[0] + 1) * (unsigned long long)(hi[1] - lo[1] + 1);
        covered = (unsigned long long)npg * area * depth;
        int skip_lo = 0, skip_hi = 0;
        trim_span(a, a.words + 12 * (size_t)pbase, npg, lo, hi, live, skip_lo, skip_hi);
        evaluated = (unsigned long long)__popc(live) * area * (unsigned long long)(depth - skip_lo - skip_hi);
        if (live && inside) {
            live |= 1u << kInteriorBit;
            interior = evaluated;
        }
        if (live) live |= ((uint32_t)skip_lo << kSpanLoBit) | ((uint32_t)skip_hi << kSpanHiBit);
    }
    const uint32_t lane = threadIdx.x % 64u;
    if (work) {
        evaluated = wave_sum(evaluated);
        covered = wave_sum(covered);
        interior = wave_sum(interior);
        if (lane == 0u) {
            unsigned long long *slot = work + kWorkSlotWords * ((blockIdx.x * 4u + threadIdx.x / 64u) % kWorkSlots);
            atomicAdd(slot, evaluated);
            atomicAdd(slot + 1, covered);
            atomicAdd(slot + 2, interior);
        }
    }
    // one atomic per wave when all its lanes fall in one list (the usual case)
    const uint32_t x0 = __shfl(x, 0);
    const bool one_list = __all(x == x0);
    const uint64_t m = __ballot(live != 0u);
    if (one_list) {
        if (m == 0ull) return;
        uint32_t base = 0u;
        if (lane == 0u) base = atomicAdd(counts + x0 * kListStride, (uint32_t)__popcll(m));
        base = __shfl(base, 0);
        if (live) {
            const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            items[list_begin(total, x0) + base + rank] = make_uint2(w, live);
        }
    } else if (live) {
        const uint32_t pos = atomicAdd(counts + x * kListStride, 1u);
        items[list_begin(total, x) + pos] = make_uint2(w, live);
    }
}

template <int PT>
__global__ __launch_bounds__(kThreads) void k_score_mask_items(const KArgs a, const uint2 *items,
                                                               const uint32_t *counts, uint32_t *take,
                                                               uint32_t total) {
    __shared__ uint32_t next_item;
    const uint32_t groups = (a.np + PT - 1) / PT;
    uint32_t staged = 0xFFFFFFFFu;  // tile whose target slab the LDS holds (none yet)
    for (uint32_t s = 0; s < 8; ++s) {
        const uint32_t x = (blockIdx.x + s) % 8u;
        const uint32_t begin = list_begin(total, x), n_items = counts[x * kListStride];
        for (;;) {
            // kItemChunk consecutive items at a time: the pre-pass appends a
            // wave's items (mostly of one tile) together
            if (threadIdx.x == 0) next_item = atomicAdd(take + x * kListStride, kItemChunk);
            __syncthreads();
            const uint32_t r0 = next_item;
            if (r0 >= n_items) break;
            const uint32_t r1 = min(r0 + kItemChunk, n_items);
            for (uint32_t r = r0; r < r1; ++r) {
                const uint2 it = items[begin + r];
                const uint32_t bx = it.x / groups, by = it.x - bx * groups;
                mask_body<PT, true, true>(a, bx, by, it.y, &staged, bx);
            }
            __syncthreads();  // next_item is read by all before thread 0 takes the next
        }
        __syncthreads();  // the same before the next list's first take
    }
}

// ---------------------------------------------------------------- batches

// Persistent warp-and-score over the work items of many pairs.  Item g of
// pair d (offs[d] <= g < offs[d + 1]) is particle group (g - offs[d]) mod
// ngroups(d) of tile (g - offs[d]) / ngroups(d).  Work lists are partitioned by
// XCD: workgroup b serves list b % 8 (the dispatcher hands workgroups to the
// eight XCDs round robin), so each pair's items stay on one XCD's L2.  The
// workgroups of an XCD take the items of its list in order from a shared
// counter, so the items in flight stay a narrow window of neighbouring tiles
// (a fixed stride per workgroup lets fast and slow workgroups drift apart
// until the window spans many pairs and the L2 hit rate collapses).
struct BatchArgs {
    const KArgs *pairs;
    const uint32_t *offs;      // n_pairs + 1 item offsets
    const uint32_t *kmax;      // iterations of each pair
    const uint32_t *lists;     // items, grouped by XCD
    uint32_t list_off[9];      // list x = lists[list_off[x] .. list_off[x + 1])
    uint32_t n_pairs;
    uint32_t k;                // iteration being scored (pairs with kmax < k are done)
    uint32_t *counters;        // 8 item counters of this launch, zero at launch
};

__device__ __forceinline__ uint32_t pair_of(const uint32_t *offs_g, uint32_t n, uint32_t g) {
    const auto *offs = as_const(offs_g);
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int PT, int MODE, int LAYOUT, int VMODE>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(MODE == kModeMask ? 1 : kImageWaves<PT, LAYOUT, VMODE, 0>)))
void k_batch_score(const BatchArgs b) {
    const auto *lists = as_const(b.lists);
    const auto *kmax = as_const(b.kmax);
    const auto *pairs = as_const(b.pairs);
    __shared__ uint32_t next_item;
    // the XCD's own list first, then the other lists' remaining items (the
    // tails hold the smallest pairs), so no XCD idles while another has work;
    // every workgroup leaves once all eight counters have passed their ends
    for (uint32_t s = 0; s < 8; ++s) {
        const uint32_t x = (blockIdx.x + s) % 8;
        const uint32_t begin = b.list_off[x], n_items = b.list_off[x + 1] - begin;
        for (;;) {
            if (threadIdx.x == 0) next_item = atomicAdd(b.counters + x, 1u);
            __syncthreads();
            const uint32_t r = next_item;
            if (r >= n_items) break;
            const uint32_t g = lists[begin + r];
            const uint32_t d = pair_of(b.offs, b.n_pairs, g);
            if (kmax[d] >= b.k) {  // pairs with fewer iterations are done
                const KArgs a = pairs[d];
                const uint32_t local = g - b.offs[d];
                const uint32_t ng = (a.np + PT - 1) / PT;
                const uint32_t bx = local / ng, by = local - bx * ng;
                if (MODE == kModeMask) mask_body<PT, true>(a, bx, by);  // the filter's launches
                else image_body<PT, LAYOUT, true, VMODE>(a, bx, by);
            }
            __syncthreads();  // next_item is read by all before thread 0 takes the next
        }
        __syncthreads();  // the same before the next list's first take
    }
}

// Mask classes: the live items of an iteration.  One thread per entry of the
// class's XCD lists tests its (tile, particle group) item against its pair's
// source mask box and appends live items, with their particle masks, interior
// bits and slice spans, to the same list's part of `live` (one atomic per wave where
// all its lanes are in one list); pairs past their last iteration add nothing.
template <int PT>
__global__ __launch_bounds__(256) void k_batch_cull(const BatchArgs b, uint2 *live, uint32_t *counts) {
    static_assert(PT <= (int)kInteriorBit, "particle bits below the interior bit");
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    const uint32_t total = b.list_off[8];
    uint32_t lm = 0u, x = 0u, g = 0u;
    if (e < total) {
        while (x < 7u && e >= b.list_off[x + 1]) ++x;
        g = b.lists[e];
        const uint32_t d = pair_of(b.offs, b.n_pairs, g);
        if (b.kmax[d] >= b.k) {
            const KArgs &a = b.pairs[d];
            const uint32_t local = g - b.offs[d];
            const uint32_t groups = (a.np + PT - 1) / PT;
            const uint32_t bx = local / groups, by = local - bx * groups;
            const int tiles = a.tiles_x * a.tiles_y;
            const int zc = (int)bx / tiles, tb = (int)bx - zc * tiles;
            const int ty = tb / a.tiles_x, tx = tb - ty * a.tiles_x;
            const int k0 = zc * a.zchunk;
            const int lo[3] = {tx * kTX, ty * kTY, k0};
            const int hi[3] = {min(tx * kTX + kTX - 1, a.tn0 - 1), min(ty * kTY + kTY - 1, a.tn1 - 1),
                               min(k0 + a.zchunk, a.tn2) - 1};
            float c[3], h[3];
            box_centre(lo, hi, c, h);
            const uint32_t pbase = a.p0 + by * PT, npg = min((uint32_t)PT, a.p0 + a.np - pbase);
            bool inside = true;
            for (uint32_t p = 0; p < npg; ++p)
                if (box_reaches(a.words + 12 * (size_t)(pbase + p), c, h, a)) {
                    lm |= 1u << p;
                    inside = inside && box_inside(a.words + 12 * (size_t)(pbase + p), c, h, a);
                }
            int skip_lo = 0, skip_hi = 0;
            trim_span(a, a.words + 12 * (size_t)pbase, npg, lo, hi, lm, skip_lo, skip_hi);
            if (lm && inside) lm |= 1u << kInteriorBit;
            if (lm) lm |= ((uint32_t)skip_lo << kSpanLoBit) | ((uint32_t)skip_hi << kSpanHiBit);
        }
    }
    const uint32_t lane = threadIdx.x % 64u;
    const uint32_t x0 = __shfl(x, 0);
    const bool one_list = __all(x == x0);
    const uint64_t m = __ballot(lm != 0u);
    if (one_list) {
        if (m == 0ull) return;
        uint32_t base = 0u;
        if (lane == 0u) base = atomicAdd(counts + x0 * kListStride, (uint32_t)__popcll(m));
        base = __shfl(base, 0);
        if (lm) {
            const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            live[b.list_off[x0] + base + rank] = make_uint2(g, lm);
        }
    } else if (lm) {
        const uint32_t pos = atomicAdd(counts + x * kListStride, 1u);
        live[b.list_off[x] + pos] = make_uint2(g, lm);
    }
}

// The mask class's persistent warp-and-score over the live items of one
// iteration: list x first (its XCD's), then the others, as k_batch_score.
template <int PT>
__global__ __launch_bounds__(kThreads) void k_batch_mask_items(const BatchArgs b, const uint2 *live,
                                                               const uint32_t *counts) {
    const auto *pairs = as_const(b.pairs);
    __shared__ uint32_t next_item;
    // key of the tile whose target slab the LDS holds: the batch-wide index of
    // the tile's first item (none yet)
    uint32_t staged = 0xFFFFFFFFu;
    for (uint32_t s = 0; s < 8; ++s) {
        const uint32_t x = (blockIdx.x + s) % 8;
        const uint32_t begin = b.list_off[x], n_items = counts[x * kListStride];
        for (;;) {
            if (threadIdx.x == 0) next_item = atomicAdd(b.counters + x, kItemChunk);
            __syncthreads();
            const uint32_t r0 = next_item;
            if (r0 >= n_items) break;
            for (uint32_t r = r0; r < min(r0 + kItemChunk, n_items); ++r) {
                const uint2 it = live[begin + r];
                const uint32_t d = pair_of(b.offs, b.n_pairs, it.x);
                const KArgs a = pairs[d];
                const uint32_t local = it.x - b.offs[d];
                const uint32_t ng = (a.np + PT - 1) / PT;
                const uint32_t bx = local / ng, by = local - bx * ng;
                mask_body<PT, true, true>(a, bx, by, it.y, &staged, it.x - by);
            }
            __syncthreads();  // next_item is read by all before thread 0 takes the next
        }
        __syncthreads();  // the same before the next list's first take
    }
}

KArgs make_args(const ScoreLaunch &L, int pt, int *nz_chunks) {
    KArgs a;
    a.src = L.src;
    a.src_packed = L.src_packed ? L.src_packed : (const void *)L.src;
    a.src_ok = L.src_ok;
    a.vmode = L.src_ok == nullptr ? 0 : (L.has_sentinel && L.layout != kLayoutRaw ? 2 : 1);
    a.sentinel = L.sentinel;
    a.tgt = L.tgt;
    a.tgt_fov = L.tgt_fov;
    a.words = L.words;
    a.sums = L.sums;
    a.hist = L.hist;
    a.sn0 = L.sn[0];
    a.sn1 = L.sn[1];
    a.sn2 = L.sn[2];
    a.tn0 = L.tn[0];
    a.tn1 = L.tn[1];
    a.tn2 = L.tn[2];
    a.p0 = L.p0;
    a.np = L.np;
    // occupancy culling: masks' culled launches with a table
    const bool occ = L.mode == kModeMask && L.cull_box && L.occ;
    a.occ = occ ? L.occ : nullptr;
    a.ocx = (uint32_t)((L.sn[0] + (1 << kOccShift) - 1) >> kOccShift) + 1u;
    a.ocxy = a.ocx * ((uint32_t)((L.sn[1] + (1 << kOccShift) - 1) >> kOccShift) + 1u);
    for (int d = 0; d < 3; ++d) a.occ_hi[d] = (float)(L.sn[d] - 1);
    a.tiles_x = (L.tn[0] + kTX - 1) / kTX;
    a.tiles_y = (L.tn[1] + kTY - 1) / kTY;
    const int zc = L.zchunk > 0 ? std::min(L.zchunk, kZChunkMax) : kZChunkMax;
    const int chunks = (L.tn[2] + zc - 1) / zc;
    a.zchunk = (L.tn[2] + chunks - 1) / chunks;
    for (int d = 0; d < 3; ++d) {
        if (L.mode == kModeImageTrilinear) {
            // inside iff 0 <= u <= n - 1
            a.cull_lo[d] = 0.0f;
            a.cull_hi[d] = (float)(L.sn[d] - 1);
        } else if (L.mode == kModeMask && L.cull_box) {
            // only samples landing in the source mask's bounding box add to a, c
            a.cull_lo[d] = (float)L.box_lo[d];
            a.cull_hi[d] = (float)(L.box_hi[d] + 1);
        } else {
            // nearest (words carry +0.5): inside iff 0 <= u < n
            a.cull_lo[d] = 0.0f;
            a.cull_hi[d] = (float)L.sn[d];
        }
    }
    if (L.mode == kModeMask) {
        // the filter's launches read the source bitmap: byte strides of its
        // rows and slices (zero without a bitmap; those launches use bytes)
        const uint32_t row = 4u * (uint32_t)((L.sn[0] + 31) / 32);
        a.src_packed = L.src_bits;
        a.src_bytes = L.src_bits ? (uint32_t)mask_bits_bytes(L.sn) : 0u;
        a.ysb = row;
        a.zsb = row * (uint32_t)L.sn[1];
        *nz_chunks = chunks;
        return a;
    }
    const uint32_t eb = (uint32_t)packed_bytes_per_voxel(L.layout);
    a.src_bytes = (uint32_t)std::min<uint64_t>(packed_bytes(L.layout, L.sn), 0xFFFFFFFFull);
    if (L.layout == kLayoutOctTile) {
        a.ysb = 32u * (uint32_t)((L.sn[0] + 3) / 4);  // a quarter of a row of tiles
        a.zsb = (uint32_t)(128ull * (uint64_t)((L.sn[0] + 3) / 4) * (uint64_t)((L.sn[1] + 3) / 4));
    } else {
        a.ysb = (uint32_t)L.sn[0] * eb;
        a.zsb = (uint32_t)((uint64_t)L.sn[0] * L.sn[1] * eb);
    }
    *nz_chunks = chunks;
    (void)pt;
    return a;
}

typedef void (*ScoreKernel)(const KArgs);

template <int PT, int LAYOUT, int ACC>
ScoreKernel pick_tri(int vmode) {
    if constexpr (LAYOUT != kLayoutRaw) {
        if (vmode == 2) return k_score_image<PT, LAYOUT, true, 2, ACC>;
    }
    return vmode ? k_score_image<PT, LAYOUT, true, 1, ACC> : k_score_image<PT, LAYOUT, true, 0, ACC>;
}

template <int PT, int ACC>
ScoreKernel pick_tri_layout(int layout, int vmode) {
    switch (layout) {
    case kLayoutPairX: return pick_tri<PT, kLayoutPairX, ACC>(vmode);
    case kLayoutQuadXY: return pick_tri<PT, kLayoutQuadXY, ACC>(vmode);
    case kLayoutOct: return pick_tri<PT, kLayoutOct, ACC>(vmode);
    case kLayoutOctTile: return pick_tri<PT, kLayoutOctTile, ACC>(vmode);
    case kLayoutLerp: return pick_tri<PT, kLayoutLerp, ACC>(vmode);
    default: return pick_tri<PT, kLayoutRaw, ACC>(vmode);
    }
}

template <int PT>
ScoreKernel pick(const ScoreLaunch &L) {
    if (L.mode == kModeMask) return L.cull_box && L.src_bits ? k_score_mask<PT, true> : k_score_mask<PT, false>;
    const bool sok = L.src_ok != nullptr;
    if (L.mode == kModeImageNearest)
        return sok ? k_score_image<PT, kLayoutRaw, false, 1> : k_score_image<PT, kLayoutRaw, false, 0>;
    const int vmode = !sok ? 0 : (L.has_sentinel ? 2 : 1);
    return L.hist ? pick_tri_layout<PT, 1>(L.layout, vmode) : pick_tri_layout<PT, 0>(L.layout, vmode);
}

}  // namespace

bool score_pt_supported(int pt) { return pt == 4 || pt == 8 || pt == 16; }

bool layout_fits(int layout, const int32_t sn[3]) {
    if (layout == kLayoutRaw) return true;
    // 32-bit buffer offsets; slice strides within the 24-bit multiplier
    const int32_t one[3] = {sn[0], sn[1], 1};
    // (below 4 GiB by a margin, so a load at the end offset cannot wrap)
    return packed_bytes(layout, sn) <= 0xFFFFFF00ull && packed_bytes(layout, one) < (1ull << 24);
}

size_t score_args_bytes() { return sizeof(KArgs); }

uint32_t score_items(const ScoreLaunch &L) {
    dim3 grid, block;
    score_grid(L, &grid, &block);
    return grid.x * grid.y;
}

void score_args(const ScoreLaunch &L, void *out) {
    int chunks;
    const KArgs a = make_args(L, score_pt_supported(L.pt) ? L.pt : 8, &chunks);
    memcpy(out, &a, sizeof a);
}

namespace {
template <int PT, int LAYOUT>
ScoreKernel pick_batch_image(int vmode) {
    typedef void (*BK)(const BatchArgs);
    BK k;
    if constexpr (LAYOUT != kLayoutRaw) {
        if (vmode == 2) return reinterpret_cast<ScoreKernel>(k_batch_score<PT, kModeImageTrilinear, LAYOUT, 2>);
    }
    if (vmode != 0) k = k_batch_score<PT, kModeImageTrilinear, LAYOUT, 1>;
    else k = k_batch_score<PT, kModeImageTrilinear, LAYOUT, 0>;
    return reinterpret_cast<ScoreKernel>(k);
}

template <int PT>
ScoreKernel pick_batch(int mode, int layout, int vmode) {
    if (mode == kModeMask) return reinterpret_cast<ScoreKernel>(k_batch_score<PT, kModeMask, kLayoutRaw, 0>);
    switch (layout) {
    case kLayoutPairX: return pick_batch_image<PT, kLayoutPairX>(vmode);
    case kLayoutQuadXY: return pick_batch_image<PT, kLayoutQuadXY>(vmode);
    case kLayoutOct: return pick_batch_image<PT, kLayoutOct>(vmode);
    case kLayoutOctTile: return pick_batch_image<PT, kLayoutOctTile>(vmode);
    case kLayoutLerp: return pick_batch_image<PT, kLayoutLerp>(vmode);
    default: return pick_batch_image<PT, kLayoutRaw>(vmode);
    }
}

template <int PT>
ScoreKernel pick_batch_pt(const BatchPlan &P) {
    return pick_batch<PT>(P.mode, P.layout, P.vmode);
}
}  // namespace

hipError_t launch_batch_score(const BatchPlan &P, uint32_t k, hipStream_t s) {
    if (P.n_pairs == 0) return hipSuccess;
    BatchArgs b;
    b.pairs = (const KArgs *)P.pairs;
    b.offs = P.offs;
    b.kmax = P.kmax;
    b.lists = P.lists;
    for (int x = 0; x < 9; ++x) b.list_off[x] = P.list_off[x];
    b.n_pairs = P.n_pairs;
    b.k = k;
    b.counters = P.counters + 8ull * (k - 1);
    if (P.mode == kModeMask && P.live && P.live_counts) {
        const int pt = score_pt_supported(P.pt) ? P.pt : 8;
        uint32_t *counts = P.live_counts + (uint64_t)(kItemCounterWords / 2) * (k - 1);
        const uint32_t total = P.list_off[8];
        const dim3 cg((total + 255u) / 256u);
        if (total == 0) return hipSuccess;
        if (pt == 4) hipLaunchKernelGGL(k_batch_cull<4>, cg, dim3(256), 0, s, b, (uint2 *)P.live, counts);
        else if (pt == 16) hipLaunchKernelGGL(k_batch_cull<16>, cg, dim3(256), 0, s, b, (uint2 *)P.live, counts);
        else hipLaunchKernelGGL(k_batch_cull<8>, cg, dim3(256), 0, s, b, (uint2 *)P.live, counts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (pt == 4)
            hipLaunchKernelGGL(k_batch_mask_items<4>, dim3(P.grid), dim3(kThreads), 0, s, b, (const uint2 *)P.live,
                               (const uint32_t *)counts);
        else if (pt == 16)
            hipLaunchKernelGGL(k_batch_mask_items<16>, dim3(P.grid), dim3(kThreads), 0, s, b, (const uint2 *)P.live,
                               (const uint32_t *)counts);
        else
            hipLaunchKernelGGL(k_batch_mask_items<8>, dim3(P.grid), dim3(kThreads), 0, s, b, (const uint2 *)P.live,
                               (const uint32_t *)counts);
        return hipGetLastError();
    }
    typedef void (*BK)(const BatchArgs);
    BK kern = reinterpret_cast<BK>(const_cast<void *>(batch_kernel(P)));
    hipLaunchKernelGGL(kern, dim3(P.grid), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

const void *batch_kernel(const BatchPlan &P) {
    const int pt = score_pt_supported(P.pt) ? P.pt : 8;
    if (P.mode == kModeMask && P.live) {
        if (pt == 4) return reinterpret_cast<const void *>(k_batch_mask_items<4>);
        if (pt == 16) return reinterpret_cast<const void *>(k_batch_mask_items<16>);
        return reinterpret_cast<const void *>(k_batch_mask_items<8>);
    }
    if (pt == 4) return reinterpret_cast<const void *>(pick_batch_pt<4>(P));
    if (pt == 16) return reinterpret_cast<const void *>(pick_batch_pt<16>(P));
    return reinterpret_cast<const void *>(pick_batch_pt<8>(P));
}

int batch_blocks_per_cu(const BatchPlan &P) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_kernel(P), kThreads, 0) != hipSuccess ||
        blocks < 1)
        blocks = 4;
    return blocks;
}

int score_vmode(const ScoreLaunch &L) {
    int chunks;
    return make_args(L, 8, &chunks).vmode;
}

// Work items (tiles x particle groups) of a launch, in 64 bits.
uint64_t score_items64(const ScoreLaunch &L) {
    int chunks;
    const int pt = score_pt_supported(L.pt) ? L.pt : 8;
    const KArgs a = make_args(L, pt, &chunks);
    return (uint64_t)a.tiles_x * (uint64_t)a.tiles_y * (uint64_t)chunks * (uint64_t)((L.np + pt - 1) / pt);
}

// A one-dimensional grid of one workgroup per item; grid.x = 0 (no launch
// possible) when the items exceed a grid dimension.
void score_grid(const ScoreLaunch &L, dim3 *grid, dim3 *block) {
    const uint64_t items = score_items64(L);
    *grid = dim3(items <= kMaxScoreItems ? (unsigned)items : 0u, 1, 1);
    *block = dim3(kThreads, 1, 1);
}

namespace {

template <int PT>
__global__ __launch_bounds__(kThreads) void k_probe_mask_items(const KArgs a, const uint2 *items,
                                                               const uint32_t *counts, uint32_t *take,
                                                               uint32_t total, uint32_t key, uint32_t *out);

// Resident workgroups of a persistent kernel on the current device (cached
// per device and kernel; the occupancy query is made once).
int persistent_blocks(const void *kernel) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(dev, kernel);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int cus = 0, per_cu = 0;
    if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 4;
    return cache[key] = cus * per_cu;
}

template <int PT>
hipError_t launch_mask_items_pt(const KArgs &a, uint32_t total, const ScoreLaunch &L, bool probe, uint32_t key,
                                uint32_t *out, hipStream_t s) {
    static_assert(kItemCounterWords == 16 * kListStride, "counts and takes, eight each");
    uint32_t *counts = L.item_counters, *take = L.item_counters + 8 * kListStride;
    hipError_t e = launch_fill_u64((unsigned long long *)L.item_counters, kItemCounterWords / 2, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cull_items<PT>, dim3((total + 255u) / 256u), dim3(256), 0, s, a, total, (uint2 *)L.items,
                       counts, probe ? nullptr : L.work);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (probe) {
        const int blocks = persistent_blocks(reinterpret_cast<const void *>(k_probe_mask_items<PT>));
        hipLaunchKernelGGL(k_probe_mask_items<PT>, dim3(blocks), dim3(kThreads), 0, s, a, (const uint2 *)L.items,
                           (const uint32_t *)counts, take, total, key, out);
    } else {
        const int blocks = persistent_blocks(reinterpret_cast<const void *>(k_score_mask_items<PT>));
        hipLaunchKernelGGL(k_score_mask_items<PT>, dim3(blocks), dim3(kThreads), 0, s, a, (const uint2 *)L.items,
                           (const uint32_t *)counts, take, total);
    }
    return hipGetLastError();
}

// The filter's mask launches through the culled item lists, when the
// context provides lists large enough for this launch.
bool uses_item_lists(const ScoreLaunch &L, uint64_t total) {
    return L.mode == kModeMask && L.cull_box && L.src_bits && L.items && L.item_counters && total <= L.item_cap;
}

hipError_t launch_mask_items(const ScoreLaunch &L, int pt, const KArgs &a, uint32_t total, bool probe, uint32_t key,
                             uint32_t *out, hipStream_t s) {
    if (pt == 4) return launch_mask_items_pt<4>(a, total, L, probe, key, out, s);
    if (pt == 16) return launch_mask_items_pt<16>(a, total, L, probe, key, out, s);
    return launch_mask_items_pt<8>(a, total, L, probe, key, out, s);
}

}  // namespace

uint64_t score_items_for(const ScoreLaunch &L) { return score_items64(L); }

hipError_t launch_score(const ScoreLaunch &L, hipStream_t s) {
    if (L.np == 0) return hipSuccess;
    int chunks;
    const int pt = score_pt_supported(L.pt) ? L.pt : 8;
    const KArgs a = make_args(L, pt, &chunks);
    dim3 grid, block;
    score_grid(L, &grid, &block);
    if (grid.x == 0) return hipErrorInvalidConfiguration;
    if (uses_item_lists(L, grid.x)) return launch_mask_items(L, pt, a, grid.x, false, 0u, nullptr, s);
    ScoreKernel k = pt == 4 ? pick<4>(L) : (pt == 16 ? pick<16>(L) : pick<8>(L));
    hipLaunchKernelGGL(k, grid, block, 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- gather probe

// Measurement kernels behind smc_gather_probe.  They run the grid, XCD order,
// tile culling, coordinates, offsets and source loads of the warp-and-score
// kernels exactly as those do, and replace everything else (target staging,
// interpolation, fixed-point rounding, sums and their reduction) by an XOR of
// the loaded words, so their time on a particle set is what the source
// gathers alone cost on that set.  The checksum is stored only if it equals a
// key the host never passes, which keeps every load live.
namespace {

template <int PT, bool AC, bool GIVEN = false>
__device__ __forceinline__ uint32_t probe_mask_body(const KArgs &a, uint32_t bx, uint32_t by, uint32_t live_in = 0u) {
    const Tile t = tile_of<PT>(a, bx, by);
    const uint32_t live = GIVEN ? live_in : live_mask<PT>(a, t, bx);
    uint32_t chk = 0u;
    if (live == 0u || !t.ok) return chk;
    float mx[PT], my[PT], mz[PT], ax[PT], ay[PT], az[PT];
    column_terms<PT>(a, t, mx, my, mz, ax, ay, az);
    const uint32_t sn0 = AC ? a.ysb : (uint32_t)a.sn0, sn01 = AC ? a.zsb : (uint32_t)a.sn0 * (uint32_t)a.sn1;
    const int nbytes = AC ? (int)a.src_bytes : a.sn0 * a.sn1 * a.sn2;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        AC ? const_cast<void *>(a.src_packed) : (void *)const_cast<uint8_t *>(a.src), (short)0, nbytes,
        kBufferWord3);
    const uint32_t nxb = __float_as_uint((float)a.sn0), nyb = __float_as_uint((float)a.sn1),
                   nzb = __float_as_uint((float)a.sn2);
    // the scoring kernel's interior items, as there
    const bool interior = GIVEN && AC && ((live_in >> kInteriorBit) & 1u) != 0u;
    if (interior) {
#pragma unroll
        for (int p = 0; p < PT; ++p)
            if (!((live >> p) & 1u)) {
                ax[p] = ay[p] = az[p] = mx[p] = my[p] = 0.0f;
                mz[p] = (float)a.sn2;
            }
    }
    // the scoring kernel's item spans, as there
    const int kbeg = GIVEN ? t.k0 + (int)((live_in >> kSpanLoBit) & kSpanMask) : t.k0;
    const int kend = GIVEN ? t.k1 - (int)((live_in >> kSpanHiBit) & kSpanMask) : t.k1;
    const auto slices = [&](auto interior_tag) {
        constexpr bool INTERIOR = decltype(interior_tag)::value;
        for (int k = kbeg; k < kend; ++k) {
            const float fk = (float)k;
            uint32_t off[PT];
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                const float ux = fmaf(ax[p], fk, mx[p]);
                const float uy = fmaf(ay[p], fk, my[p]);
                const float uz = fmaf(az[p], fk, mz[p]);
                const uint32_t xo = AC ? (floor_u32(ux) >> 3) & ~3u : floor_u32(ux);
                off[p] = mad_u24(floor_u32(uz), sn01, mad_u24(floor_u32(uy), sn0, xo));
                if constexpr (!INTERIOR) {
                    const bool in = ((live >> p) & 1u) & (__float_as_uint(ux) < nxb) &
                                    (__float_as_uint(uy) < nyb) & (__float_as_uint(uz) < nzb);
                    off[p] = in ? off[p] : (uint32_t)nbytes;
                }
            }
#pragma unroll
            for (int p = 0; p < PT; ++p)
                chk ^= AC ? __builtin_amdgcn_raw_buffer_load_b32(rs, off[p], 0, 0)
                          : __builtin_amdgcn_raw_buffer_load_b8(rs, off[p], 0, 0);
        }
    };
    if (interior) slices(std::true_type{});
    else slices(std::false_type{});
    return chk;
}

// Trilinear images in the one-gather layouts (octets, tiled octets, lerp
// elements), the layouts the filter's launches use.
template <int PT, int LAYOUT>
__device__ __forceinline__ uint32_t probe_image_body(const KArgs &a, uint32_t bx, uint32_t by) {
    const Tile t = tile_of<PT>(a, bx, by);
    const uint32_t live = live_mask<PT>(a, t, bx);
    uint32_t chk = 0u;
    if (live == 0u || !t.ok) return chk;
    float mx[PT], my[PT], mz[PT], ax[PT], ay[PT], az[PT];
    column_terms<PT>(a, t, mx, my, mz, ax, ay, az);
    constexpr uint32_t kElemShift = LAYOUT == kLayoutLerp ? 4u : 3u;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(a.src_packed), (short)0,
                                                                        (int)a.src_bytes, kBufferWord3);
    const uint32_t exb = __float_as_uint((float)(a.sn0 - 1)), eyb = __float_as_uint((float)(a.sn1 - 1)),
                   ezb = __float_as_uint((float)(a.sn2 - 1));
    for (int k = t.k0; k < t.k1; ++k) {
        const float fk = (float)k;
        uint32_t off[PT];
#pragma unroll
        for (int p = 0; p < PT; ++p) {
            const float ux = fmaf(ax[p], fk, mx[p]);
            const float uy = fmaf(ay[p], fk, my[p]);
            const float uz = fmaf(az[p], fk, mz[p]);
            const bool in = ((live >> p) & 1u) & (__float_as_uint(ux) <= exb) & (__float_as_uint(uy) <= eyb) &
                            (__float_as_uint(uz) <= ezb);
            const uint32_t ix = floor_u32(ux), iy = floor_u32(uy), iz = floor_u32(uz);
            if (LAYOUT == kLayoutOctTile) {
                uint32_t o = __mul24((int)(ix & 3u), -24) + (ix << 5);
                o += __mul24((int)(iy & 3u), 32 - (int)a.ysb);
                off[p] = o + __umul24(iy, a.ysb) + __umul24(iz, a.zsb);
            } else {
                off[p] = mad_u24(iz, a.zsb, mad_u24(iy, a.ysb, ix << kElemShift));
            }
            off[p] = in ? off[p] : a.src_bytes;
        }
#pragma unroll
        for (int p = 0; p < PT; ++p) {
            if constexpr (LAYOUT == kLayoutLerp) {
                const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rs, off[p], 0, 0);
                chk ^= w.x ^ w.y ^ w.z ^ w.w;
            } else {
                const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, off[p], 0, 0);
                chk ^= w.x ^ w.y;
            }
        }
    }
    return chk;
}

template <int PT, int MODE, int LAYOUT, bool AC = false>
__global__ __launch_bounds__(kThreads) void k_gather_probe(const KArgs a, uint32_t key, uint32_t *out) {
    uint32_t bx, by;
    xcd_order(blockIdx.x, gridDim.x, (a.np + PT - 1) / PT, &bx, &by);
    const uint32_t chk =
        MODE == kModeMask ? probe_mask_body<PT, AC>(a, bx, by) : probe_image_body<PT, LAYOUT>(a, bx, by);
    if (chk == key) out[0] = chk;
}

template <int PT>
__global__ __launch_bounds__(kThreads) void k_probe_mask_items(const KArgs a, const uint2 *items,
                                                               const uint32_t *counts, uint32_t *take,
                                                               uint32_t total, uint32_t key, uint32_t *out) {
    __shared__ uint32_t next_item;
    const uint32_t groups = (a.np + PT - 1) / PT;
    uint32_t chk = 0u;
    for (uint32_t s = 0; s < 8; ++s) {
        const uint32_t x = (blockIdx.x + s) % 8u;
        const uint32_t begin = list_begin(total, x), n_items = counts[x * kListStride];
        for (;;) {
            if (threadIdx.x == 0) next_item = atomicAdd(take + x * kListStride, kItemChunk);
            __syncthreads();
            const uint32_t r0 = next_item;
            if (r0 >= n_items) break;
            for (uint32_t r = r0; r < min(r0 + kItemChunk, n_items); ++r) {
                const uint2 it = items[begin + r];
                const uint32_t bx = it.x / groups, by = it.x - bx * groups;
                chk ^= probe_mask_body<PT, true, true>(a, bx, by, it.y);
            }
            __syncthreads();
        }
        __syncthreads();
    }
    if (chk == key) out[0] = chk;
}

template <int PT>
ScoreKernel probe_kernel(const ScoreLaunch &L) {
    typedef void (*PK)(const KArgs, uint32_t, uint32_t *);
    PK k = nullptr;
    if (L.mode == kModeMask)
        k = L.cull_box && L.src_bits ? k_gather_probe<PT, kModeMask, kLayoutRaw, true>
                                     : k_gather_probe<PT, kModeMask, kLayoutRaw, false>;
    else if (L.mode == kModeImageTrilinear && L.layout == kLayoutOct)
        k = k_gather_probe<PT, kModeImageTrilinear, kLayoutOct>;
    else if (L.mode == kModeImageTrilinear && L.layout == kLayoutOctTile)
        k = k_gather_probe<PT, kModeImageTrilinear, kLayoutOctTile>;
    else if (L.mode == kModeImageTrilinear && L.layout == kLayoutLerp)
        k = k_gather_probe<PT, kModeImageTrilinear, kLayoutLerp>;
    return reinterpret_cast<ScoreKernel>(k);
}

}  // namespace

bool gather_probe_supported(const ScoreLaunch &L) {
    if (L.tgt_fov != nullptr || L.hist != nullptr) return false;
    if (L.mode == kModeMask) return true;
    return L.mode == kModeImageTrilinear &&
           (L.layout == kLayoutOct || L.layout == kLayoutOctTile || L.layout == kLayoutLerp);
}

hipError_t launch_gather_probe(const ScoreLaunch &L, uint32_t key, uint32_t *out, hipStream_t s) {
    if (!gather_probe_supported(L)) return hipErrorInvalidValue;
    if (L.np == 0) return hipSuccess;
    int chunks;
    const int pt = score_pt_supported(L.pt) ? L.pt : 8;
    const KArgs a = make_args(L, pt, &chunks);
    dim3 grid, block;
    score_grid(L, &grid, &block);
    if (grid.x == 0) return hipErrorInvalidConfiguration;
    // the same schedule as the production launch (culled item lists or grid)
    if (uses_item_lists(L, grid.x)) return launch_mask_items(L, pt, a, grid.x, true, key, out, s);
    ScoreKernel k = pt == 4 ? probe_kernel<4>(L) : (pt == 16 ? probe_kernel<16>(L) : probe_kernel<8>(L));
    typedef void (*PK)(const KArgs, uint32_t, uint32_t *);
    hipLaunchKernelGGL(reinterpret_cast<PK>(k), grid, block, 0, s, a, key, out);
    return hipGetLastError();
}

}  // namespace smc
