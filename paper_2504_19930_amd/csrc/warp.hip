// Whole-cycle application of the estimated transform (Methods: the transform
// found on the ED frame is applied to every frame): nearest neighbour copies
// the source byte, trilinear writes floor(v + 0.5); outside the source -> 0.
// Same FP32 coordinate recipe and interpolation order as the scoring kernels.
//
// A workgroup covers a 32 x 8 block of a chunk of kZC slices of one frame;
// each wave a 16 x 4 patch whose quarters (the 16 lanes the texture path
// serves together) are 4 x 4 squares, whose rotated images touch few source
// cache lines per gather.  A thread takes a few slices at a time: every offset first, then
// every load, then the stores, so many independent gathers are in flight.
// Sources are read through buffer loads with 32-bit offsets (a frame is
// below 2^31 bytes).
#include "internal.h"

namespace smc {
namespace {

constexpr int kWX = 32, kWY = 8, kZC = 16;
// Word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format,
// untyped loads; out-of-range offsets read zero).
constexpr int kBufferWord3 = 0x00020000;

struct WArgs {
    const uint8_t *src;
    uint8_t *dst;
    float w[12];
    int32_t sn0, sn1, sn2, tn0, tn1, tn2;
    int64_t src_stride, dst_stride;
    int32_t xblocks;
};

template <bool TRI>
__global__ __launch_bounds__(256) void k_warp_apply(const WArgs a) {
    // slices per batch of loads (fewer for trilinear: eight taps each)
    constexpr int kZU = TRI ? 4 : 8;
    // grid: x = row block * x-blocks + x-block, y = z-chunk, z = frame, so the
    // workgroups in flight share a slab of slices (contiguous memory)
    const int yb = (int)blockIdx.x / a.xblocks;
    // waves are 16 x 4 patches, each quarter-wave a 4 x 4 square
    const int lane = (int)(threadIdx.x % 64), wave = (int)(threadIdx.x / 64);
    const int i = ((int)blockIdx.x - yb * a.xblocks) * kWX + (wave % 2) * 16 + (lane / 16) * 4 + lane % 4;
    const int j = yb * kWY + (wave / 2) * 4 + (lane % 16) / 4;
    const int frame = (int)blockIdx.z;
    const int k0 = (int)blockIdx.y * kZC;
    if (i >= a.tn0 || j >= a.tn1) return;
    const uint8_t *S = a.src + a.src_stride * frame;
    uint8_t *D = a.dst + a.dst_stride * frame;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(S), (short)0,
                                                                        a.sn0 * a.sn1 * a.sn2, kBufferWord3);
    const float fi = (float)i, fj = (float)j;
    const float mx = fmaf(a.w[1], fj, fmaf(a.w[0], fi, a.w[3]));
    const float my = fmaf(a.w[5], fj, fmaf(a.w[4], fi, a.w[7]));
    const float mz = fmaf(a.w[9], fj, fmaf(a.w[8], fi, a.w[11]));
    const uint32_t sn0 = (uint32_t)a.sn0, sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
    const size_t plane = (size_t)a.tn0 * (size_t)a.tn1;
    const size_t o0 = (size_t)i + (size_t)a.tn0 * (size_t)j;
    const int k1 = min(k0 + kZC, a.tn2);
    for (int kb = k0; kb < k1; kb += kZU) {
        uint8_t val[kZU];
        if (!TRI) {
            uint32_t off[kZU];
            bool in[kZU];
#pragma unroll
            for (int q = 0; q < kZU; ++q) {
                const float fk = (float)(kb + q);
                const float ux = fmaf(a.w[2], fk, mx), uy = fmaf(a.w[6], fk, my), uz = fmaf(a.w[10], fk, mz);
                const int ix = (int)floorf(ux), iy = (int)floorf(uy), iz = (int)floorf(uz);
                in[q] = kb + q < k1 && (uint32_t)ix < (uint32_t)a.sn0 && (uint32_t)iy < (uint32_t)a.sn1 &&
                        (uint32_t)iz < (uint32_t)a.sn2;
                off[q] = in[q] ? (uint32_t)ix + sn0 * (uint32_t)iy + sn01 * (uint32_t)iz : 0u;
            }
#pragma unroll
            for (int q = 0; q < kZU; ++q) val[q] = in[q] ? (uint8_t)__builtin_amdgcn_raw_buffer_load_b8(rs, off[q], 0, 0) : (uint8_t)0;
        } else {
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
                val[q] = in[q] ? (uint8_t)(r > 255.0f ? 255.0f : r) : (uint8_t)0;
            }
        }
#pragma unroll
        for (int q = 0; q < kZU; ++q)
            if (kb + q < k1) D[o0 + plane * (size_t)(kb + q)] = val[q];
    }
}

}  // namespace

hipError_t launch_warp_apply(const uint8_t *src, const int32_t sn[3], const float w[12], bool trilinear,
                             uint8_t *dst, const int32_t tn[3], uint32_t frames, int64_t src_stride,
                             int64_t dst_stride, hipStream_t s) {
    WArgs a;
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
    a.xblocks = (tn[0] + kWX - 1) / kWX;
    dim3 grid((uint32_t)a.xblocks * (uint32_t)((tn[1] + kWY - 1) / kWY), (tn[2] + kZC - 1) / kZC, frames);
    if (trilinear) hipLaunchKernelGGL(k_warp_apply<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_warp_apply<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace smc
