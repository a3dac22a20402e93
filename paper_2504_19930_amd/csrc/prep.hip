// Once-per-pair preparation: packed mask / FOV bytes, the trilinear
// corner-validity mask of the source FOV, and exact per-volume sums
// (FOV voxel count, nonzero count, sum and sum of squares) from which the
// host derives |T| for Dice, the minimum overlap and the mean-0 / std-1
// normalisation statistics of Implementation Details.
#include <stdint.h>

#include "internal.h"

namespace smc {
namespace {

// bit 0: inside the FOV (no FOV = everywhere); bit 1: nonzero and inside.
__global__ void k_prep_mask(const uint8_t *vol, const uint8_t *fov, uint8_t *out, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t in = fov ? (fov[q] != 0) : 1u;
        out[q] = (uint8_t)(in | ((in && vol[q] != 0) ? 2u : 0u));
    }
}

// Source mask as a bitmap for the filter's mask launches: bit x % 32 of
// dword (x / 32) + W (y + ny z), W = ceil(nx / 32), is set iff the prepared
// byte has its "on" bit (on and inside the source FOV); pad bits are zero.
__global__ void k_pack_mask_bits(const uint8_t *prep, int32_t nx, int32_t ny, int32_t nz, uint32_t W,
                                 uint32_t *out) {
    const int64_t n = (int64_t)W * ny * nz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = q / W;
        const int32_t x0 = (int32_t)(q - row * W) * 32;
        const uint8_t *r = prep + row * (int64_t)nx;
        uint32_t w = 0u;
        for (int b = 0; b < 32 && x0 + b < nx; ++b) w |= ((uint32_t)(r[x0 + b] >> 1) & 1u) << b;
        out[q] = w;
    }
}

// A trilinear sample with base corner (i, j, k) is valid iff all eight
// (edge-clamped) corners are inside the FOV.
__global__ void k_corner_valid(const uint8_t *fov, uint8_t *out, int32_t nx, int32_t ny, int32_t nz) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(q % nx);
        const int32_t j = (int32_t)((q / nx) % ny);
        const int32_t k = (int32_t)(q / ((int64_t)nx * ny));
        const int64_t dx = i + 1 < nx ? 1 : 0;
        const int64_t dy = j + 1 < ny ? nx : 0;
        const int64_t dz = k + 1 < nz ? (int64_t)nx * ny : 0;
        const bool ok = fov[q] && fov[q + dx] && fov[q + dy] && fov[q + dx + dy] && fov[q + dz] &&
                        fov[q + dz + dx] && fov[q + dz + dy] && fov[q + dz + dy + dx];
        out[q] = ok ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_volume_sums(const uint8_t *vol, const uint8_t *fov, int64_t n,
                                                     unsigned long long *out) {
    unsigned long long c = 0, o = 0, s1 = 0, s2 = 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        if (fov && fov[q] == 0) continue;
        const unsigned long long v = vol[q];
        c += 1;
        o += v != 0;
        s1 += v;
        s2 += v * v;
    }
    __shared__ unsigned long long red[4][4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_xor(c, off);
        o += __shfl_xor(o, off);
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
    }
    const int wave = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
        red[wave][0] = c;
        red[wave][1] = o;
        red[wave][2] = s1;
        red[wave][3] = s2;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        atomicAdd(out + threadIdx.x, s);
    }
}

// Trilinear source layouts: per base voxel the corner bytes the kernel needs,
// with corners past the last voxel repeating it (see score.hip).  The
// element of voxel q and its FOV validity (all voxels it covers inside):
//   pairx  (v[x], v[x+1]) of one row;  quadxy  the 2x2 of one slice;
//   oct    the 2x2x2 of the trilinear cell (lerp stores the same cell ready
//          for the x-lerps).
// A trilinear sample is inside the FOV iff every element it reads is, so an
// invalid element may hold a sentinel value that no valid element takes.
struct Elem {
    uint64_t value;
    bool valid;
};

__device__ __forceinline__ Elem element(const uint8_t *vol, const uint8_t *fov, int32_t nx, int32_t ny, int32_t nz,
                                        int layout, int64_t q) {
    const int32_t i = (int32_t)(q % nx);
    const int32_t j = (int32_t)((q / nx) % ny);
    const int32_t k = (int32_t)(q / ((int64_t)nx * ny));
    const int64_t dx = i + 1 < nx ? 1 : 0;
    const int64_t dy = j + 1 < ny ? nx : 0;
    const int64_t dz = k + 1 < nz ? (int64_t)nx * ny : 0;
    Elem e;
    if (layout == kLayoutPairX) {
        e.value = (uint64_t)vol[q] | ((uint64_t)vol[q + dx] << 8);
        e.valid = !fov || (fov[q] && fov[q + dx]);
        return e;
    }
    const uint32_t q0 = (uint32_t)vol[q] | ((uint32_t)vol[q + dx] << 8) | ((uint32_t)vol[q + dy] << 16) |
                        ((uint32_t)vol[q + dy + dx] << 24);
    const bool v0 = !fov || (fov[q] && fov[q + dx] && fov[q + dy] && fov[q + dy + dx]);
    if (layout == kLayoutQuadXY) {
        e.value = q0;
        e.valid = v0;
        return e;
    }
    const int64_t r = q + dz;
    const uint32_t q1 = (uint32_t)vol[r] | ((uint32_t)vol[r + dx] << 8) | ((uint32_t)vol[r + dy] << 16) |
                        ((uint32_t)vol[r + dy + dx] << 24);
    const bool v1 = !fov || (fov[r] && fov[r + dx] && fov[r + dy] && fov[r + dy + dx]);
    e.value = (uint64_t)q0 | ((uint64_t)q1 << 32);
    e.valid = v0 && v1;
    return e;
}

__global__ void k_pack_source(const uint8_t *vol, const uint8_t *fov, int32_t nx, int32_t ny, int32_t nz,
                              int layout, uint64_t sentinel, void *out) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const Elem e = element(vol, fov, nx, ny, nz, layout, q);
        const uint64_t v = e.valid ? e.value : sentinel;
        if (layout == kLayoutPairX) {
            ((uint16_t *)out)[q] = (uint16_t)v;
        } else if (layout == kLayoutQuadXY) {
            ((uint32_t *)out)[q] = (uint32_t)v;
        } else if (layout == kLayoutLerp) {
            // the four x-lerp starts a = v(x, .) and steps d = v(x + 1, .) - v(x, .)
            // of the rows (y, z), (y + 1, z), (y, z + 1), (y + 1, z + 1), each times
            // 256 in half precision (exact: |256 v| <= 65280 with at most eight
            // significant bits); elements outside the FOV carry the NaN sentinel
            uint32_t w[4];
            if (e.valid) {
                uint32_t h[8];
                for (int r = 0; r < 4; ++r) {
                    const int lo = (int)((e.value >> (16 * r)) & 0xFFu), hi = (int)((e.value >> (16 * r + 8)) & 0xFFu);
                    const _Float16 a = (_Float16)(256.0f * (float)lo), d = (_Float16)(256.0f * (float)(hi - lo));
                    h[r] = __builtin_bit_cast(uint16_t, a);
                    h[4 + r] = __builtin_bit_cast(uint16_t, d);
                }
                w[0] = h[0] | (h[1] << 16);
                w[1] = h[2] | (h[3] << 16);
                w[2] = h[4] | (h[5] << 16);
                w[3] = h[6] | (h[7] << 16);
            } else {
                w[0] = kLerpSentinel;
                w[1] = w[2] = w[3] = 0u;
            }
            ((uint4 *)out)[q] = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
            int64_t o = q;
            if (layout == kLayoutOctTile) {
                // 4 x 4 tiles of one slice, 16 octets (128 bytes) each, x fastest
                // inside a tile, tiles x fastest, then y, then slices
                const int64_t i = q % nx, j = (q / nx) % ny, k = q / ((int64_t)nx * ny);
                const int64_t tx = (nx + 3) / 4, ty = (ny + 3) / 4;
                o = ((k * ty + j / 4) * tx + i / 4) * 16 + (j % 4) * 4 + (i % 4);
            }
            ((uint2 *)out)[o] = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
        }
    }
}

__global__ void k_count_elements(const uint8_t *vol, const uint8_t *fov, int32_t nx, int32_t ny, int32_t nz,
                                 int layout, const uint64_t *cand, int n_cand, unsigned long long *counts) {
    const int64_t n = (int64_t)nx * ny * nz;
    const uint64_t mask = layout == kLayoutPairX ? 0xFFFFull : (layout == kLayoutQuadXY ? 0xFFFFFFFFull : ~0ull);
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const Elem e = element(vol, fov, nx, ny, nz, layout, q);
        if (!e.valid) continue;
        if (n_cand == 0) {
            atomicAdd(counts + e.value, 1ull);
        } else {
            for (int c = 0; c < n_cand; ++c)
                if (e.value == (cand[c] & mask)) atomicAdd(counts + c, 1ull);
        }
    }
}

__global__ void k_mask_bbox(const uint8_t *prep, int32_t nx, int32_t ny, int32_t nz, int32_t *out) {
    const int64_t n = (int64_t)nx * ny * nz;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {-1, -1, -1};
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        if (!(prep[q] & 2u)) continue;
        const int32_t c[3] = {(int32_t)(q % nx), (int32_t)((q / nx) % ny), (int32_t)(q / ((int64_t)nx * ny))};
        for (int d = 0; d < 3; ++d) {
            lo[d] = min(lo[d], c[d]);
            hi[d] = max(hi[d], c[d]);
        }
    }
    for (int d = 0; d < 3; ++d) {
        if (hi[d] < 0) continue;
        atomicMin(out + d, lo[d]);
        atomicMax(out + 3 + d, hi[d]);
    }
}

// Occupancy of the source mask's on bits over cells of 2^kOccShift voxels a
// side, as a summed-area table S[(z (cy + 1) + y) (cx + 1) + x] = number of
// occupied cells with cell coordinates below (x, y, z) (a zero first row,
// column and slice).  First the cells (one thread per table entry), then
// prefix sums along x, y and z (one thread per line).
__global__ void k_occ_cells(const uint8_t *prep, int32_t nx, int32_t ny, int32_t nz, int32_t cx, int32_t cy,
                            int32_t cz, uint32_t *S) {
    const int64_t X = cx + 1, XY = X * (cy + 1), n = XY * (cz + 1);
    constexpr int kc = 1 << kOccShift;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = (int32_t)(q % X), y = (int32_t)((q / X) % (cy + 1)), z = (int32_t)(q / XY);
        uint32_t on = 0u;
        if (x > 0 && y > 0 && z > 0) {
            const int32_t x0 = (x - 1) * kc, y0 = (y - 1) * kc, z0 = (z - 1) * kc;
            for (int32_t k = z0; k < min(z0 + kc, nz) && !on; ++k)
                for (int32_t j = y0; j < min(y0 + kc, ny) && !on; ++j)
                    for (int32_t i = x0; i < min(x0 + kc, nx); ++i)
                        if (prep[(int64_t)i + (int64_t)nx * (j + (int64_t)ny * k)] & 2u) {
                            on = 1u;
                            break;
                        }
        }
        S[q] = on;
    }
}

// Prefix sums of the table along one axis (0 = x, 1 = y, 2 = z).
__global__ void k_occ_prefix(uint32_t *S, int32_t cx, int32_t cy, int32_t cz, int32_t axis) {
    const int64_t X = cx + 1, Y = cy + 1, Z = cz + 1;
    const int64_t len = axis == 0 ? X : axis == 1 ? Y : Z;
    const int64_t step = axis == 0 ? 1 : axis == 1 ? X : X * Y;
    const int64_t lines = X * Y * Z / len;
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < lines; l += (int64_t)gridDim.x * blockDim.x) {
        // start of line l: the index with coordinate 0 along the axis
        int64_t base;
        if (axis == 0) base = l * X;
        else if (axis == 1) base = (l / X) * X * Y + l % X;
        else base = l;
        uint32_t run = 0u;
        for (int64_t t = 0; t < len; ++t) {
            run += S[base + t * step];
            S[base + t * step] = run;
        }
    }
}

unsigned blocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_prep_mask(const uint8_t *vol, const uint8_t *fov, uint8_t *out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_prep_mask, dim3(blocks_for(n)), dim3(256), 0, s, vol, fov, out, n);
    return hipGetLastError();
}

uint64_t mask_bits_bytes(const int32_t n[3]) {
    return 4ull * (uint64_t)((n[0] + 31) / 32) * (uint64_t)n[1] * (uint64_t)n[2];
}

hipError_t launch_pack_mask_bits(const uint8_t *prep, const int32_t n[3], uint32_t *out, hipStream_t s) {
    const uint32_t W = (uint32_t)((n[0] + 31) / 32);
    const int64_t tot = (int64_t)W * n[1] * n[2];
    hipLaunchKernelGGL(k_pack_mask_bits, dim3(blocks_for(tot)), dim3(256), 0, s, prep, n[0], n[1], n[2], W, out);
    return hipGetLastError();
}

hipError_t launch_mask_bbox(const uint8_t *prep, const int32_t n[3], int32_t *out, hipStream_t s) {
    const int64_t tot = (int64_t)n[0] * n[1] * n[2];
    hipLaunchKernelGGL(k_mask_bbox, dim3(blocks_for(tot)), dim3(256), 0, s, prep, n[0], n[1], n[2], out);
    return hipGetLastError();
}

uint64_t mask_occ_words(const int32_t n[3]) {
    const uint64_t cx = ((uint64_t)n[0] + (1u << kOccShift) - 1) >> kOccShift;
    const uint64_t cy = ((uint64_t)n[1] + (1u << kOccShift) - 1) >> kOccShift;
    const uint64_t cz = ((uint64_t)n[2] + (1u << kOccShift) - 1) >> kOccShift;
    return (cx + 1) * (cy + 1) * (cz + 1);
}

hipError_t launch_mask_occupancy(const uint8_t *prep, const int32_t n[3], uint32_t *sat, hipStream_t s) {
    const int32_t c = 1 << kOccShift;
    const int32_t cx = (n[0] + c - 1) / c, cy = (n[1] + c - 1) / c, cz = (n[2] + c - 1) / c;
    hipLaunchKernelGGL(k_occ_cells, dim3(blocks_for((int64_t)mask_occ_words(n))), dim3(256), 0, s, prep, n[0], n[1],
                       n[2], cx, cy, cz, sat);
    const int64_t X = cx + 1, Y = cy + 1, Z = cz + 1;
    const int64_t lines[3] = {Y * Z, X * Z, X * Y};
    for (int32_t axis = 0; axis < 3; ++axis)
        hipLaunchKernelGGL(k_occ_prefix, dim3(blocks_for(lines[axis])), dim3(256), 0, s, sat, cx, cy, cz, axis);
    return hipGetLastError();
}

hipError_t launch_corner_valid(const uint8_t *fov, uint8_t *out, const int32_t n[3], hipStream_t s) {
    const int64_t tot = (int64_t)n[0] * n[1] * n[2];
    hipLaunchKernelGGL(k_corner_valid, dim3(blocks_for(tot)), dim3(256), 0, s, fov, out, n[0], n[1], n[2]);
    return hipGetLastError();
}

size_t packed_bytes_per_voxel(int layout) {
    switch (layout) {
    case kLayoutPairX: return 2;
    case kLayoutQuadXY: return 4;
    case kLayoutOct: case kLayoutOctTile: return 8;
    case kLayoutLerp: return 16;
    default: return 1;
    }
}

uint64_t packed_bytes(int layout, const int32_t n[3]) {
    if (layout == kLayoutOctTile)
        return (uint64_t)((n[0] + 3) / 4) * (uint64_t)((n[1] + 3) / 4) * 128ull * (uint64_t)n[2];
    return (uint64_t)n[0] * n[1] * n[2] * packed_bytes_per_voxel(layout);
}

hipError_t launch_pack_source(const uint8_t *vol, const uint8_t *fov, const int32_t n[3], int layout,
                              uint64_t sentinel, void *out, hipStream_t s) {
    if (layout == kLayoutRaw) return hipSuccess;
    const int64_t tot = (int64_t)n[0] * n[1] * n[2];
    hipLaunchKernelGGL(k_pack_source, dim3(blocks_for(tot)), dim3(256), 0, s, vol, fov, n[0], n[1], n[2], layout,
                       sentinel, out);
    return hipGetLastError();
}

hipError_t launch_count_elements(const uint8_t *vol, const uint8_t *fov, const int32_t n[3], int layout,
                                 const uint64_t *cand, int n_cand, unsigned long long *counts, hipStream_t s) {
    const int64_t tot = (int64_t)n[0] * n[1] * n[2];
    hipLaunchKernelGGL(k_count_elements, dim3(blocks_for(tot)), dim3(256), 0, s, vol, fov, n[0], n[1], n[2], layout,
                       cand, n_cand, counts);
    return hipGetLastError();
}

hipError_t launch_volume_sums(const uint8_t *vol, const uint8_t *fov, int64_t n, unsigned long long *out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_volume_sums, dim3(blocks_for(n)), dim3(256), 0, s, vol, fov, n, out);
    return hipGetLastError();
}

}  // namespace smc
