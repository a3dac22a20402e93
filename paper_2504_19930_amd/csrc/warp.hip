// Whole-cycle application of the estimated transform (Methods: the transform
// found on the ED frame is applied to every frame): nearest neighbour copies
// the source byte, trilinear writes floor(v + 0.5); outside the source -> 0.
// Same FP32 coordinate recipe and interpolation order as the scoring kernels.
// One thread per output voxel of a 32 x 8 column, walking z; frames on grid.z.
#include "internal.h"

namespace smc {
namespace {

struct WArgs {
    const uint8_t *src;
    uint8_t *dst;
    float w[12];
    int32_t sn0, sn1, sn2, tn0, tn1, tn2;
    int64_t src_stride, dst_stride;
};

template <bool TRI>
__global__ __launch_bounds__(256) void k_warp_apply(const WArgs a) {
    const int i = blockIdx.x * 32 + (threadIdx.x % 32);
    const int j = blockIdx.y * 8 + (threadIdx.x / 32);
    if (i >= a.tn0 || j >= a.tn1) return;
    const uint8_t *S = a.src + a.src_stride * blockIdx.z;
    uint8_t *D = a.dst + a.dst_stride * blockIdx.z;
    const float fi = (float)i, fj = (float)j;
    const float mx = fmaf(a.w[1], fj, fmaf(a.w[0], fi, a.w[3]));
    const float my = fmaf(a.w[5], fj, fmaf(a.w[4], fi, a.w[7]));
    const float mz = fmaf(a.w[9], fj, fmaf(a.w[8], fi, a.w[11]));
    const uint32_t sn0 = (uint32_t)a.sn0, sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
    const size_t plane = (size_t)a.tn0 * (size_t)a.tn1;
    size_t o = (size_t)i + (size_t)a.tn0 * (size_t)j;
    for (int k = 0; k < a.tn2; ++k, o += plane) {
        const float fk = (float)k;
        const float ux = fmaf(a.w[2], fk, mx), uy = fmaf(a.w[6], fk, my), uz = fmaf(a.w[10], fk, mz);
        uint8_t val = 0;
        if (!TRI) {
            const int ix = (int)floorf(ux), iy = (int)floorf(uy), iz = (int)floorf(uz);
            if ((uint32_t)ix < (uint32_t)a.sn0 && (uint32_t)iy < (uint32_t)a.sn1 && (uint32_t)iz < (uint32_t)a.sn2)
                val = S[(uint32_t)ix + sn0 * (uint32_t)iy + sn01 * (uint32_t)iz];
        } else if (ux >= 0.0f && ux <= (float)(a.sn0 - 1) && uy >= 0.0f && uy <= (float)(a.sn1 - 1) &&
                   uz >= 0.0f && uz <= (float)(a.sn2 - 1)) {
            const float flx = floorf(ux), fly = floorf(uy), flz = floorf(uz);
            const uint32_t ix = (uint32_t)flx, iy = (uint32_t)fly, iz = (uint32_t)flz;
            const float fx = ux - flx, fy = uy - fly, fz = uz - flz;
            const uint32_t dx = ix < (uint32_t)(a.sn0 - 1) ? 1u : 0u;
            const uint32_t dy = iy < (uint32_t)(a.sn1 - 1) ? sn0 : 0u;
            const uint32_t dz = iz < (uint32_t)(a.sn2 - 1) ? sn01 : 0u;
            const uint8_t *P = S + ix + sn0 * iy + sn01 * iz;
            const float v000 = (float)P[0], v100 = (float)P[dx], v010 = (float)P[dy], v110 = (float)P[dy + dx];
            const float v001 = (float)P[dz], v101 = (float)P[dz + dx], v011 = (float)P[dz + dy];
            const float v111 = (float)P[dz + dy + dx];
            const float x00 = fmaf(fx, v100 - v000, v000), x10 = fmaf(fx, v110 - v010, v010);
            const float x01 = fmaf(fx, v101 - v001, v001), x11 = fmaf(fx, v111 - v011, v011);
            const float y0 = fmaf(fy, x10 - x00, x00), y1 = fmaf(fy, x11 - x01, x01);
            const float s = fmaf(fz, y1 - y0, y0);
            const float r = floorf(s + 0.5f);
            val = (uint8_t)(r > 255.0f ? 255.0f : r);
        }
        D[o] = val;
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
    dim3 grid((tn[0] + 31) / 32, (tn[1] + 7) / 8, frames);
    if (trilinear) hipLaunchKernelGGL(k_warp_apply<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_warp_apply<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace smc
