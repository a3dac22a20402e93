// Whole-cycle application of the estimated transform (Methods: the transform
// found on the ED frame is applied to every frame): nearest neighbour copies
// the source byte, trilinear writes floor(v + 0.5); outside the source -> 0.
// Same FP32 coordinate recipe and interpolation order as the scoring kernels.
//
// Tiles of 32 x 8 x zc target voxels; each wave covers a 16 x 4 patch of a
// tile whose quarters are 4 x 4 squares, one thread per column.  Workgroups
// are ordered so that each XCD (the hardware hands workgroup b to XCD b % 8)
// runs a contiguous run of tiles: neighbouring tiles share source and
// destination cache lines, and one L2 then fetches each line once.
//
// The frames share the transform, so the nearest and the staged trilinear
// kernels take one workgroup per tile and loop over the frames: each voxel's
// source offset (and fractions) are computed once and reused for every frame.
//
// Nearest: per frame one byte gather per voxel from the kept offsets (samples
// outside the source read the buffer's end: zero, no cache line touched).
// Trilinear, staged (the usual case): the source points a tile samples lie in
// a box given by the affine map's extremes over the tile's corners plus a
// one-voxel margin; the workgroup copies that box of each frame into LDS with
// 16-byte loads, and the eight taps are LDS reads instead of byte gathers
// through the texture path (a cycle per distinct cache line a quarter-wave
// touches, four to eight lines under rotation).  Trilinear, direct: one
// workgroup per tile and frame, every tap a byte gather; the host takes it
// when the box would not fit the LDS budget, source rows are not 4-byte
// aligned, or coordinates reach 2^20 (where the margin would no longer cover
// FP32 rounding).
#include "internal.h"

namespace smc {
namespace {

constexpr int kWX = 32, kWY = 8;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format,
// untyped loads; out-of-range offsets read zero and writes are dropped).
constexpr int kBufferWord3 = 0x00020000;
// LDS bytes of a staged workgroup's source box: with its output tile (4 or 2
// KB) three workgroups per CU for 16-slice tiles (whose registers allow
// three), four for 8-slice tiles.
constexpr uint32_t kStageBudget16 = 48u * 1024u, kStageBudget8 = 36u * 1024u;
// Source-box rows of at most four 16-byte chunks; row passes a thread keeps
// in flight while staging.
constexpr uint32_t kChunks = 4;
constexpr int kStagePasses = 8;
// Frames per workgroup of the frame-looping kernels.
constexpr uint32_t kFrameGroup = 4;
// Zero bytes at the start of the staged LDS.
constexpr uint32_t kZeroBytes = 16;
// Bound on every partial sum of the coordinate recipe for the staged kernel:
// below 2^20 each FP32 rounding is at most 1/16 voxel, so a voxel's computed
// coordinate and its tile's computed extremes stay within the margin.
constexpr double kStageCoordLimit = 1048576.0;

struct WArgs {
    const uint8_t *src;
    uint8_t *dst;
    float w[12];
    int32_t sn0, sn1, sn2, tn0, tn1, tn2;
    int64_t src_stride, dst_stride;
    int32_t xblocks, bxy, zchunks, zc;  // tiles per row and per slab, slabs per frame, slices per tile
    uint32_t total;                     // workgroups
    uint32_t frames, fg;                // frames; frames per workgroup (groups of fg)
    // staged kernel: per source axis sum_e |w_de| (T_e - 1) over a tile's
    // extents T; LDS row pitch, rows per LDS slice, slice pitch
    float span[3];
    uint32_t P, rows, Pz;
};

struct WTile {
    int x0, y0, k0, k1, frame;  // frame: the group of frames fg * frame .. fg * frame + fg - 1
};

// Tile of this workgroup: the (x-block, row block, slab, frame group) order
// split into eight contiguous runs, run r on XCD r.
__device__ __forceinline__ WTile warp_tile(const WArgs &a) {
    const uint32_t T = a.total, b = blockIdx.x, xcd = b % 8u, kk = b / 8u, q = T / 8u, r = T % 8u;
    const uint32_t lin = (xcd < r ? xcd * (q + 1u) : r * (q + 1u) + (xcd - r) * q) + kk;
    const uint32_t per_frame = (uint32_t)a.bxy * (uint32_t)a.zchunks;
    WTile t;
    t.frame = (int)(lin / per_frame);
    const uint32_t rem = lin - (uint32_t)t.frame * per_frame;
    const int zc = (int)(rem / (uint32_t)a.bxy), bx = (int)(rem - (uint32_t)zc * (uint32_t)a.bxy);
    const int yb = bx / a.xblocks;
    t.x0 = (bx - yb * a.xblocks) * kWX;
    t.y0 = yb * kWY;
    t.k0 = zc * a.zc;
    t.k1 = min(t.k0 + a.zc, a.tn2);
    return t;
}

// The thread's column in its tile: waves are 16 x 4 patches, quarters 4 x 4.
__device__ __forceinline__ void warp_column(const WTile &t, int &i, int &j) {
    const int lane = (int)(threadIdx.x % 64), wave = (int)(threadIdx.x / 64);
    i = t.x0 + (wave % 2) * 16 + (lane / 16) * 4 + lane % 4;
    j = t.y0 + (wave / 2) * 4 + (lane % 16) / 4;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const uint8_t *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(p), (short)0, (int)bytes, kBufferWord3);
}

// Write one frame's output tile, assembled in LDS as ZC slices x kWY rows x
// kWX bytes, with 16-byte stores: thread t takes half t % 2 of row t / 2
// (rows past the target, and the tail of a row past its end, are skipped; a
// row whose 16 bytes do not all lie inside, or outputs whose rows are not
// 4-byte aligned, are written byte by byte).
template <int ZC>
__device__ __forceinline__ void store_tile(const uint8_t *tile, const WArgs &a, const WTile &t, int f) {
    static_assert(kWX == 32, "two 16-byte halves per tile row");
    const uint32_t plane = (uint32_t)a.tn0 * (uint32_t)a.tn1;
    const __amdgpu_buffer_rsrc_t rd = buffer_of(a.dst + a.dst_stride * f, plane * (uint32_t)a.tn2);
    const int x = t.x0 + 16 * (int)(threadIdx.x % 2u);
    const bool vec = a.tn0 % 4 == 0;
#pragma unroll
    for (int r = (int)(threadIdx.x / 2u); r < ZC * kWY; r += 128) {
        const int k = t.k0 + r / kWY, j = t.y0 + r % kWY;
        if (k >= t.k1 || j >= a.tn1 || x >= a.tn0) continue;
        const u32x4 v = *(const u32x4 *)(tile + r * kWX + (x - t.x0));
        const uint32_t o = (uint32_t)x + (uint32_t)a.tn0 * (uint32_t)j + plane * (uint32_t)k;
        if (vec && x + 16 <= a.tn0) {
            __builtin_amdgcn_raw_buffer_store_b128(v, rd, o, 0, 0);
        } else {
            for (int b = 0; b < 16 && x + b < a.tn0; ++b)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(v[b / 4] >> (8 * (b % 4))), rd, o + (uint32_t)b, 0, 0);
        }
    }
}

// Staged trilinear kernel.  LDS layout: 16 zero bytes (samples outside the
// source read them, with fractions 0), then the box: rows of P bytes, slices
// of Pz bytes, one more row and slice for the +1 taps.  The box of frame f + 1
// is loaded into registers while frame f is computed.
template <int ZC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ZC == 16 ? 3 : 4)))
void k_warp_trilinear_lds(const WArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ __attribute__((aligned(16))) uint8_t tile[ZC * kWY * kWX];
    const WTile t = warp_tile(a);
    const uint32_t sn0 = (uint32_t)a.sn0, sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
    const uint32_t nbytes = sn01 * (uint32_t)a.sn2;

    // source box: per axis the minimum of the affine map over the tile's
    // corners (unclipped extents), less one voxel, to the maximum plus two
    // (the second covers the trilinear +1 tap), clipped to the source
    const int c0[3] = {t.x0, t.y0, t.k0};
    const int ext[3] = {kWX - 1, kWY - 1, ZC - 1};
    const int sn[3] = {a.sn0, a.sn1, a.sn2};
    int lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float m = a.w[4 * d + 3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const float we = a.w[4 * d + e];
            m = fmaf(we, (float)(we < 0.0f ? c0[e] + ext[e] : c0[e]), m);
        }
        lo[d] = max((int)floorf(m) - 1, 0);
        hi[d] = min((int)floorf(m + a.span[d]) + 2, sn[d] - 1);
    }
    const bool any = lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2];
    const uint32_t xa = (uint32_t)lo[0] & ~15u;

    // staging list: thread -> (row slot t / 4 + 64 u, 16-byte chunk t % 4);
    // source offset and LDS index per pass (LDS index 0 = nothing to copy)
    uint32_t go[kStagePasses], gl[kStagePasses], tail = 0u;
    {
        const uint32_t nq = any ? ((uint32_t)hi[0] - xa) / 16u + 1u : 0u;
        const uint32_t ny = any ? (uint32_t)(hi[1] - lo[1] + 1) : 1u;
        const uint32_t nrows = any ? ny * (uint32_t)(hi[2] - lo[2] + 1) : 0u;
        const uint32_t c = threadIdx.x % 4u, dz = 64u / ny, dy = 64u - dz * ny;
        uint32_t r = threadIdx.x / 4u, zz = r / ny, yy = r - zz * ny;
#pragma unroll
        for (int u = 0; u < kStagePasses; ++u) {
            const bool ok = r < nrows && c < nq;
            go[u] = mad_u24((uint32_t)lo[2] + zz, sn01, mad_u24((uint32_t)lo[1] + yy, sn0, xa)) + 16u * c;
            gl[u] = ok ? kZeroBytes + mad_u24(zz, a.Pz, mad_u24(yy, a.P, 16u * c)) : 0u;
            // chunks that run past the source's end (handled by a shifted load)
            tail |= (ok && go[u] + 16u > nbytes) ? (1u << u) : 0u;
            r += 64u;
            zz += dy + yy >= ny ? dz + 1u : dz;
            yy = dy + yy >= ny ? dy + yy - ny : dy + yy;
        }
    }

    // the thread's column and, per slice, its LDS index and fractions
    int i, j;
    warp_column(t, i, j);
    const float fi = (float)i, fj = (float)j;
    const float mx = fmaf(a.w[1], fj, fmaf(a.w[0], fi, a.w[3]));
    const float my = fmaf(a.w[5], fj, fmaf(a.w[4], fi, a.w[7]));
    const float mz = fmaf(a.w[9], fj, fmaf(a.w[8], fi, a.w[11]));
    // LDS index of source voxel (x, y, z): z Pz + y P + x - base (mod 2^32)
    const uint32_t base = (uint32_t)lo[2] * a.Pz + (uint32_t)lo[1] * a.P + xa - kZeroBytes;
    const uint32_t P = a.P, Pz = a.Pz;
    uint32_t li[ZC];
    float fx[ZC], fy[ZC], fz[ZC];
    {
        // inside: 0 <= u <= n - 1 per axis, as unsigned compares of bit
        // patterns (the coordinates are never -0: the offset words are +0)
        const uint32_t bx = __float_as_uint((float)(a.sn0 - 1)), by = __float_as_uint((float)(a.sn1 - 1)),
                       bz = __float_as_uint((float)(a.sn2 - 1));
#pragma unroll
        for (int q = 0; q < ZC; ++q) {
            const float fk = (float)(t.k0 + q);
            const float ux = fmaf(a.w[2], fk, mx), uy = fmaf(a.w[6], fk, my), uz = fmaf(a.w[10], fk, mz);
            const bool in = (t.k0 + q < t.k1) & (__float_as_uint(ux) <= bx) & (__float_as_uint(uy) <= by) &
                            (__float_as_uint(uz) <= bz);
            li[q] = in ? mad_u24(floor_u32(uz), Pz, mad_u24(floor_u32(uy), P, floor_u32(ux) - base)) : 0u;
            // the +1 taps need no edge test: at u = n - 1 the fraction is
            // exactly 0 and the tap, whatever finite byte it reads, adds 0
            fx[q] = in ? __builtin_amdgcn_fractf(ux) : 0.0f;
            fy[q] = in ? __builtin_amdgcn_fractf(uy) : 0.0f;
            fz[q] = in ? __builtin_amdgcn_fractf(uz) : 0.0f;
        }
    }
    if (threadIdx.x == 0) *(u32x4 *)lds = u32x4{0u, 0u, 0u, 0u};
    // the thread's byte of the output tile in slice 0
    const uint32_t tl = (uint32_t)(j - t.y0) * kWX + (uint32_t)(i - t.x0);

    u32x4 v[kStagePasses];
    auto load_box = [&](int f) {
        const __amdgpu_buffer_rsrc_t rs = buffer_of(a.src + a.src_stride * f, nbytes);
#pragma unroll
        for (int u = 0; u < kStagePasses; ++u) {
            v[u] = u32x4{0u, 0u, 0u, 0u};
            if (gl[u] != 0u) {
                if (!((tail >> u) & 1u)) {
                    v[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, go[u], 0, 0);
                } else if (go[u] < nbytes) {
                    // k dwords past the end: load the last 16 bytes and shift
                    // them down (bytes past the end are never used: left 0)
                    const uint32_t k = (go[u] + 16u - nbytes) / 4u;
                    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rs, nbytes - 16u, 0, 0);
                    v[u].x = w[k];
                    v[u].y = k < 3u ? w[k + 1u] : 0u;
                    v[u].z = k < 2u ? w[k + 2u] : 0u;
                }
            }
        }
    };
    const int f0 = t.frame * (int)a.fg, f1 = min(f0 + (int)a.fg, (int)a.frames);
    load_box(f0);
    for (int f = f0; f < f1; ++f) {
        __syncthreads();  // every thread is done with frame f - 1's box and tile
#pragma unroll
        for (int u = 0; u < kStagePasses; ++u)
            if (gl[u] != 0u) *(u32x4 *)(lds + gl[u]) = v[u];
        __syncthreads();
        if (f + 1 < f1) load_box(f + 1);
#pragma unroll
        for (int q = 0; q < ZC; ++q) {
            // byte taps (2-byte LDS reads at odd addresses are far slower)
            const uint8_t *b0 = lds + li[q], *b1 = b0 + P, *b2 = b0 + Pz, *b3 = b2 + P;
            const float v0 = (float)b0[0], v1 = (float)b0[1], v2 = (float)b1[0], v3 = (float)b1[1],
                        v4 = (float)b2[0], v5 = (float)b2[1], v6 = (float)b3[0], v7 = (float)b3[1];
            const float x00 = fmaf(fx[q], v1 - v0, v0), x10 = fmaf(fx[q], v3 - v2, v2);
            const float x01 = fmaf(fx[q], v5 - v4, v4), x11 = fmaf(fx[q], v7 - v6, v6);
            const float y0 = fmaf(fy[q], x10 - x00, x00), y1 = fmaf(fy[q], x11 - x01, x01);
            // lerps of bytes stay within [0, 255]: no upper clamp needed
            tile[q * kWY * kWX + tl] = (uint8_t)floor_u32(fmaf(fz[q], y1 - y0, y0) + 0.5f);
        }
        __syncthreads();
        store_tile<ZC>(tile, a, t, f);
    }
}

// Nearest neighbour: one workgroup per tile and group of frames, looping over
// them two at a time: every gather of both frames issued, the bytes placed in
// two LDS output tiles, then the tiles written with 16-byte stores.
template <int ZC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_warp_nearest(const WArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t tile[2][ZC * kWY * kWX];
    const WTile t = warp_tile(a);
    int i, j;
    warp_column(t, i, j);
    const uint32_t sn0 = (uint32_t)a.sn0, sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
    const uint32_t nbytes = sn01 * (uint32_t)a.sn2;
    const float fi = (float)i, fj = (float)j;
    const float mx = fmaf(a.w[1], fj, fmaf(a.w[0], fi, a.w[3]));
    const float my = fmaf(a.w[5], fj, fmaf(a.w[4], fi, a.w[7]));
    const float mz = fmaf(a.w[9], fj, fmaf(a.w[8], fi, a.w[11]));
    // inside iff 0 <= u < n per axis, as unsigned compares of bit patterns
    // (the coordinates are never -0: the offset words are +0); samples
    // outside (or past the tile) read the buffer's end: zero
    const uint32_t nxb = __float_as_uint((float)a.sn0), nyb = __float_as_uint((float)a.sn1),
                   nzb = __float_as_uint((float)a.sn2);
    uint32_t off[ZC];
#pragma unroll
    for (int q = 0; q < ZC; ++q) {
        const float fk = (float)(t.k0 + q);
        const float ux = fmaf(a.w[2], fk, mx), uy = fmaf(a.w[6], fk, my), uz = fmaf(a.w[10], fk, mz);
        const bool in = (t.k0 + q < t.k1) & (__float_as_uint(ux) < nxb) & (__float_as_uint(uy) < nyb) &
                        (__float_as_uint(uz) < nzb);
        off[q] = in ? mad_u24(floor_u32(uz), sn01, mad_u24(floor_u32(uy), sn0, floor_u32(ux))) : nbytes;
    }
    // the thread's byte of an output tile in slice 0
    const uint32_t tl = (uint32_t)(j - t.y0) * kWX + (uint32_t)(i - t.x0);
    const int f0 = t.frame * (int)a.fg, f1 = min(f0 + (int)a.fg, (int)a.frames);
    for (int f = f0; f < f1; f += 2) {
        const bool two = f + 1 < f1;
        const __amdgpu_buffer_rsrc_t r0 = buffer_of(a.src + a.src_stride * f, nbytes);
        const __amdgpu_buffer_rsrc_t r1 = buffer_of(a.src + a.src_stride * (two ? f + 1 : f), nbytes);
        uint32_t v0[ZC], v1[ZC];
#pragma unroll
        for (int q = 0; q < ZC; ++q) {
            v0[q] = __builtin_amdgcn_raw_buffer_load_b8(r0, off[q], 0, 0);
            v1[q] = __builtin_amdgcn_raw_buffer_load_b8(r1, off[q], 0, 0);
        }
        __syncthreads();  // the tiles of the previous pair are written out
#pragma unroll
        for (int q = 0; q < ZC; ++q) {
            tile[0][q * kWY * kWX + tl] = (uint8_t)v0[q];
            tile[1][q * kWY * kWX + tl] = (uint8_t)v1[q];
        }
        __syncthreads();
        store_tile<ZC>(tile[0], a, t, f);
        if (two) store_tile<ZC>(tile[1], a, t, f + 1);
    }
}

// Direct trilinear kernel: one workgroup per tile and frame, every tap a byte
// gather from the source frame.
__global__ __launch_bounds__(256) void k_warp_trilinear(const WArgs a) {
    constexpr int kZU = 4;  // slices per batch of loads (eight taps each)
    const WTile t = warp_tile(a);
    int i, j;
    warp_column(t, i, j);
    if (i >= a.tn0 || j >= a.tn1) return;
    const uint8_t *S = a.src + a.src_stride * t.frame;
    uint8_t *D = a.dst + a.dst_stride * t.frame;
    const __amdgpu_buffer_rsrc_t rs = buffer_of(S, (uint32_t)a.sn0 * (uint32_t)a.sn1 * (uint32_t)a.sn2);
    const float fi = (float)i, fj = (float)j;
    const float mx = fmaf(a.w[1], fj, fmaf(a.w[0], fi, a.w[3]));
    const float my = fmaf(a.w[5], fj, fmaf(a.w[4], fi, a.w[7]));
    const float mz = fmaf(a.w[9], fj, fmaf(a.w[8], fi, a.w[11]));
    const uint32_t sn0 = (uint32_t)a.sn0, sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
    const size_t plane = (size_t)a.tn0 * (size_t)a.tn1;
    const size_t o0 = (size_t)i + (size_t)a.tn0 * (size_t)j;
    const int k0 = t.k0, k1 = t.k1;
    for (int kb = k0; kb < k1; kb += kZU) {
        uint32_t base[kZU], dx[kZU], dy[kZU], dz[kZU];
        float fx[kZU], fy[kZU], fz[kZU];
        bool in[kZU];
#pragma unroll
        for (int q = 0; q < kZU; ++q) {
            const float fk = (float)(kb + q);
            const float ux = fmaf(a.w[2], fk, mx), uy = fmaf(a.w[6], fk, my), uz = fmaf(a.w[10], fk, mz);
            in[q] = kb + q < k1 && ux >= 0.0f && ux <= (float)(a.sn0 - 1) && uy >= 0.0f &&
                    uy <= (float)(a.sn1 - 1) && uz >= 0.0f && uz <= (float)(a.sn2 - 1);
            const float flx = floorf(ux), fly = floorf(uy), flz = floorf(uz);
            const uint32_t ix = in[q] ? (uint32_t)flx : 0u, iy = in[q] ? (uint32_t)fly : 0u,
                           iz = in[q] ? (uint32_t)flz : 0u;
            fx[q] = ux - flx;
            fy[q] = uy - fly;
            fz[q] = uz - flz;
            dx[q] = ix < (uint32_t)(a.sn0 - 1) ? 1u : 0u;
            dy[q] = iy < (uint32_t)(a.sn1 - 1) ? sn0 : 0u;
            dz[q] = iz < (uint32_t)(a.sn2 - 1) ? sn01 : 0u;
            base[q] = ix + sn0 * iy + sn01 * iz;
        }
        float v[kZU][8];
#pragma unroll
        for (int q = 0; q < kZU; ++q) {
            const uint32_t b = base[q], ex = dx[q], ey = dy[q], ez = dz[q];
            v[q][0] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b, 0, 0);
            v[q][1] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b + ex, 0, 0);
            v[q][2] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b + ey, 0, 0);
            v[q][3] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b + ey + ex, 0, 0);
            v[q][4] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b + ez, 0, 0);
            v[q][5] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b + ez + ex, 0, 0);
            v[q][6] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b + ez + ey, 0, 0);
            v[q][7] = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, b + ez + ey + ex, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < kZU; ++q) {
            const float x00 = fmaf(fx[q], v[q][1] - v[q][0], v[q][0]);
            const float x10 = fmaf(fx[q], v[q][3] - v[q][2], v[q][2]);
            const float x01 = fmaf(fx[q], v[q][5] - v[q][4], v[q][4]);
            const float x11 = fmaf(fx[q], v[q][7] - v[q][6], v[q][6]);
            const float y0 = fmaf(fy[q], x10 - x00, x00), y1 = fmaf(fy[q], x11 - x01, x01);
            const float sv = fmaf(fz[q], y1 - y0, y0);
            const float r = floorf(sv + 0.5f);
            if (kb + q < k1) D[o0 + plane * (size_t)(kb + q)] = in[q] ? (uint8_t)(r > 255.0f ? 255.0f : r) : (uint8_t)0;
        }
    }
}

// Staged-box geometry for tiles of depth zc; false when it does not fit.
bool stage_geometry(WArgs &a, int zc, uint32_t &bytes) {
    const int T[3] = {kWX, kWY, zc};
    uint32_t ext[3];
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int e = 0; e < 3; ++e) s += fabs((double)a.w[4 * d + e]) * (double)(T[e] - 1);
        a.span[d] = (float)s;
        // a tile's box spans at most floor(min + span) + 2 - (floor(min) - 1) + 1
        // <= span + 5 voxels (plus rounding well below 0.1)
        ext[d] = (uint32_t)floor(s + 0.5) + 6u;
    }
    // rows hold the 16-byte chunks from the box's x-start rounded down to 16;
    // at most kChunks chunks a row and 64 rows per staging pass
    const uint32_t nq = (ext[0] + 14u) / 16u + 1u;
    if (nq > kChunks || (uint64_t)ext[1] * ext[2] > 64u * (uint64_t)kStagePasses) return false;
    // row and slice pitches odd multiples of 16 bytes, so the rows and slices
    // a wave's taps span fall on different LDS banks; one more row and slice
    // hold the +1 taps of the box's last ones
    a.P = 16u * (nq | 1u);
    a.rows = (ext[1] + 1u) | 1u;
    a.Pz = a.P * a.rows;
    // zero bytes, the box with its extra slice, 16 bytes of slack
    const uint64_t b = kZeroBytes + (uint64_t)a.Pz * (uint64_t)(ext[2] + 1u) + 16u;
    bytes = (uint32_t)(b > 0xFFFFFFFFull ? 0xFFFFFFFFull : b);
    return b <= (zc == 16 ? kStageBudget16 : kStageBudget8);
}

}  // namespace

hipError_t launch_warp_apply(const uint8_t *src, const int32_t sn[3], const float w[12], bool trilinear,
                             uint8_t *dst, const int32_t tn[3], uint32_t frames, int64_t src_stride,
                             int64_t dst_stride, hipStream_t s) {
    WArgs a = {};
    a.src = src;
    a.dst = dst;
    for (int q = 0; q < 12; ++q) a.w[q] = w[q];
    a.sn0 = sn[0];
    a.sn1 = sn[1];
    a.sn2 = sn[2];
    a.tn0 = tn[0];
    a.tn1 = tn[1];
    a.tn2 = tn[2];
    a.src_stride = src_stride;
    a.dst_stride = dst_stride;
    a.frames = frames;
    a.xblocks = (tn[0] + kWX - 1) / kWX;
    a.bxy = a.xblocks * ((tn[1] + kWY - 1) / kWY);
    const dim3 block(256);

    // frame-looping kernels: groups of kFrameGroup frames per workgroup (enough
    // workgroups to fill the GPU evenly; the per-tile work shared by four)
    const uint32_t groups = (frames + kFrameGroup - 1) / kFrameGroup;
    if (!trilinear) {
        a.zc = 16;
        a.fg = kFrameGroup;
        a.zchunks = (tn[2] + a.zc - 1) / a.zc;
        const uint64_t total = (uint64_t)a.bxy * (uint64_t)a.zchunks * groups;
        if (total > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
        a.total = (uint32_t)total;
        hipLaunchKernelGGL(k_warp_nearest<16>, dim3(a.total), block, 0, s, a);
        return hipGetLastError();
    }

    // staged trilinear: source rows 4-byte aligned (16-byte chunks at dword
    // offsets) and at least 16 bytes of source, every partial sum of the
    // recipe below 2^20, box within budget
    bool staged = sn[0] % 4 == 0 && (int64_t)sn[0] * sn[1] * sn[2] >= 16;
    for (int d = 0; d < 3 && staged; ++d) {
        double b = fabs((double)w[4 * d + 3]);
        for (int e = 0; e < 3; ++e) b += fabs((double)w[4 * d + e]) * (double)(tn[e] + 64);
        staged = b < kStageCoordLimit;
    }
    uint32_t bytes = 0;
    if (staged) {
        // four registers a slice (index, fractions): tiles of 16 or 8 slices
        staged = false;
        for (int z : {16, 8})
            if (stage_geometry(a, z, bytes)) {
                a.zc = z;
                staged = true;
                break;
            }
    }
    if (!staged) a.zc = 16;
    a.zchunks = (tn[2] + a.zc - 1) / a.zc;
    // staged: one workgroup per tile and group of frames; direct: one per tile
    // and frame
    a.fg = staged ? kFrameGroup : 1u;
    const uint64_t total = (uint64_t)a.bxy * (uint64_t)a.zchunks * (staged ? groups : frames);
    if (total > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
    a.total = (uint32_t)total;
    if (!staged) hipLaunchKernelGGL(k_warp_trilinear, dim3(a.total), block, 0, s, a);
    else if (a.zc == 16) hipLaunchKernelGGL(k_warp_trilinear_lds<16>, dim3(a.total), block, bytes, s, a);
    else hipLaunchKernelGGL(k_warp_trilinear_lds<8>, dim3(a.total), block, bytes, s, a);
    return hipGetLastError();
}

}  // namespace smc
