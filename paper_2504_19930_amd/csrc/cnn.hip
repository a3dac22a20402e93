// Learned proposal network: downsampling to 64^3, four 3x3x3 stride-2
// convolutions (2 -> 16 -> 32 -> 64 -> 64 channels, zero padding 1, bias,
// ReLU), a linear head to 6 means and 6 log-variances, the Gaussian NLL of
// the filter's final weighted cloud, its backward pass and Adam.
//
// Convolutions are implicit GEMMs on the matrix cores, their operands
// gathered straight from the activations (no im2col buffer).  The forward
// pass (k_conv_fwd) gives each workgroup one 16x16 output tile and a range of
// K: its four waves take alternate 32-wide steps of v_mfma_f32_16x16x32_bf16
// (gfx950's BF16 matrix instruction, eight K values per lane), with the
// im2col offsets of the range precomputed in LDS, and their accumulators are
// added in LDS.  The deep layers have few output tiles, so K is also split
// across workgroups, whose partial tiles a second kernel adds in a fixed
// order with the bias and ReLU (no floating-point atomics: a forward pass is
// reproducible bit for bit).  The backward operators use one wave per 16x16
// tile and the same instruction.
//   forward  C[m = output voxel][n = c_out]  = sum_k X(m, k = (c_in, kz, ky, kx)) W(k, n)
//   dgrad    C[m = input voxel][n = c_in]    = sum_k dY(m, k = (c_out, kz, ky, kx)) W(k, n)
//   wgrad    C[m = c_out][n = (c_in, kz, ky, kx)] = sum_k dY(k = output voxel, m) X(k, n)   (split-K)
// Weights and stored activations are bfloat16 (round to nearest even),
// accumulation FP32, gradients FP32.
#include <hip/hip_fp16.h>

#include "internal.h"

namespace smc {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t b = __float_as_uint(f);
    b = b + 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct ConvShape {
    int B, ci, co, di;  // batch, channels in / out, input side (cubic); output side di / 2
};

// ---- operand gathers -------------------------------------------------------

// Input activation of layer L at (b, c, z, y, x), zero outside.  Layer 0 reads
// the FP16 network input, later layers bfloat16 activations.
template <bool HALF_IN>
__device__ __forceinline__ uint16_t act_bf16(const uint16_t *X, const ConvShape &s, int b, int c, int z, int y,
                                             int x) {
    if ((unsigned)z >= (unsigned)s.di || (unsigned)y >= (unsigned)s.di || (unsigned)x >= (unsigned)s.di) return 0;
    const uint16_t v = X[(((size_t)b * s.ci + c) * s.di + z) * s.di * s.di + (size_t)y * s.di + x];
    if (HALF_IN) return to_bf16(__half2float(__ushort_as_half(v)));
    return v;
}

// dL/dX of a convolution (X = relu output of the previous layer, so the
// stored gradient is masked by X > 0: the gradient of the previous
// pre-activation).  dY is FP32; W is read transposed: W[co][ci][t].
struct DgradOp {
    const float *dY;
    const uint16_t *W, *Xprev;  // Xprev: the layer input (bf16), for the ReLU mask
    float *dX;
    ConvShape s;
    int M, N, K;
    __device__ uint16_t a(int m, int k) const {
        const int di = s.di, dout = di / 2, vin = di * di * di;
        const int b = m / vin, r = m - b * vin;
        const int iz = r / (di * di), iy = (r / di) % di, ix = r % di;
        const int co = k / 27, t = k - 27 * co;
        const int kz = t / 9, ky = (t / 3) % 3, kx = t % 3;
        const int z2 = iz + 1 - kz, y2 = iy + 1 - ky, x2 = ix + 1 - kx;
        if ((z2 | y2 | x2) & 1) return 0;
        const int oz = z2 >> 1, oy = y2 >> 1, ox = x2 >> 1;
        if ((unsigned)oz >= (unsigned)dout || (unsigned)oy >= (unsigned)dout || (unsigned)ox >= (unsigned)dout) return 0;
        return to_bf16(dY[(((size_t)b * s.co + co) * dout + oz) * dout * dout + (size_t)oy * dout + ox]);
    }
    __device__ uint16_t b(int k, int n) const {
        const int co = k / 27, t = k - 27 * co;
        return W[((size_t)co * s.ci + n) * 27 + t];
    }
    __device__ void store(int m, int n, float acc) const {
        const int vin = s.di * s.di * s.di;
        const int b = m / vin, r = m - b * vin;
        const size_t o = ((size_t)b * s.ci + n) * vin + r;
        dX[o] = Xprev[o] != 0 ? acc : 0.0f;
    }
};

template <bool HALF_IN>
struct WgradOp {
    const float *dY;
    const uint16_t *X;
    float *dW;  // [co][ci*27], accumulated atomically (split-K)
    ConvShape s;
    int M, N, K;
    __device__ uint16_t a(int m, int k) const {  // m = c_out, k = output voxel (with batch)
        const int dout = s.di / 2, vox = dout * dout * dout;
        const int b = k / vox, r = k - b * vox;
        return to_bf16(dY[((size_t)b * s.co + m) * vox + r]);
    }
    __device__ uint16_t b(int k, int n) const {  // k = output voxel, n = (c_in, t)
        const int dout = s.di / 2, vox = dout * dout * dout;
        const int b = k / vox, r = k - b * vox;
        const int oz = r / (dout * dout), oy = (r / dout) % dout, ox = r % dout;
        const int c = n / 27, t = n - 27 * c;
        const int kz = t / 9, ky = (t / 3) % 3, kx = t % 3;
        return act_bf16<HALF_IN>(X, s, b, c, 2 * oz + kz - 1, 2 * oy + ky - 1, 2 * ox + kx - 1);
    }
    __device__ void store(int m, int n, float acc) const { atomicAdd(dW + (size_t)m * N + n, acc); }
};

// One wave per 16x16 tile of C; four waves per workgroup along M; split-K on
// grid.z.  Lane l holds A[row l % 16][k0 + 8 (l / 16) + i], B[k0 + 8 (l / 16) + i]
// [col l % 16], i = 0..7, for v_mfma_f32_16x16x32_bf16 and, after the MFMAs,
// C[4 (l / 16) + i][col l % 16], i = 0..3.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <class Op>
__global__ __launch_bounds__(256) void k_mfma_gemm(const Op op, int k_per_split) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int m0 = (blockIdx.x * 4 + wave) * 16, n0 = blockIdx.y * 16;
    if (m0 >= op.M) return;
    const int r = lane % 16, g = lane / 16;
    const int kb = blockIdx.z * k_per_split, ke = min(op.K, kb + k_per_split);
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const bool mrow = m0 + r < op.M, ncol = n0 + r < op.N;
    for (int k0 = kb; k0 < ke; k0 += 32) {
        bf16x8 av, bv;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + 8 * g + i;
            const bool kin = k < ke;
            av[i] = __builtin_bit_cast(__bf16, (uint16_t)(kin && mrow ? op.a(m0 + r, k) : 0));
            bv[i] = __builtin_bit_cast(__bf16, (uint16_t)(kin && ncol ? op.b(k, n0 + r) : 0));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + 4 * g + i;
        if (m < op.M && ncol) op.store(m, n0 + r, acc[i]);
    }
}

template <class Op>
hipError_t run_gemm(const Op &op, int splits, hipStream_t s) {
    const int kps = ((op.K + splits - 1) / splits + 31) / 32 * 32;
    const int nsplit = (op.K + kps - 1) / kps;
    dim3 grid((op.M + 63) / 64, (op.N + 15) / 16, nsplit);
    hipLaunchKernelGGL(k_mfma_gemm<Op>, grid, dim3(256), 0, s, op, kps);
    return hipGetLastError();
}

// ---- forward convolution --------------------------------------------------------

constexpr int kFwdMaxK = 64 * 27;  // largest K = c_in * 27 of the network

// One workgroup: output rows m0 .. m0 + 15 (output voxels, with batch),
// channels n0 .. n0 + 15, K steps [s0, s1) of 32.  Wave w takes steps
// s0 + w, s0 + w + 4, ...; lane l gathers A[m0 + l % 16][k0 + 8 (l / 16) + j]
// and B[k0 + 8 (l / 16) + j][n0 + l % 16], j = 0..7, and holds
// C[m0 + 4 (l / 16) + i][n0 + l % 16], i = 0..3.  splits == 1: bias, ReLU and
// BF16 rounding here; otherwise the FP32 partial tile goes to
// partial[split][m][n] for k_conv_fwd_finish.
template <bool HALF_IN>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t *X, const uint16_t *W, const float *bias,
                                                  uint16_t *Y, float *partial, ConvShape sh, int M, int N, int K,
                                                  int steps_per_split) {
    __shared__ int32_t koff[kFwdMaxK];  // (c, kz, ky, kx) -> input offset, low 3 bits: kz/ky/kx == 0
    __shared__ v4f red[3][64];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int m0 = blockIdx.x * 16, n0 = blockIdx.y * 16, split = blockIdx.z;
    const int di = sh.di, dout = di / 2, vin = di * di * di, vox = dout * dout * dout;
    const int k_begin = split * steps_per_split * 32, k_end = min(K, k_begin + steps_per_split * 32);
    for (int k = k_begin + (int)threadIdx.x; k < k_end; k += 256) {
        const int c = k / 27, t = k - 27 * c, kz = t / 9, ky = (t / 3) % 3, kx = t % 3;
        const int off = c * vin + (kz - 1) * di * di + (ky - 1) * di + (kx - 1);
        koff[k - k_begin] = off * 8 + (kz == 0 ? 4 : 0) + (ky == 0 ? 2 : 0) + (kx == 0 ? 1 : 0);
    }
    __syncthreads();
    // this lane's output voxel (row of A)
    const int r = lane % 16, g = lane / 16;
    const int m = m0 + r;
    const bool mrow = m < M;
    const int b = mrow ? m / vox : 0, rr = mrow ? m - b * vox : 0;
    const int oz = rr / (dout * dout), oy = (rr / dout) % dout, ox = rr % dout;
    const int base = b * sh.ci * vin + 2 * oz * di * di + 2 * oy * di + 2 * ox;
    // kz == 0 reads z = 2 oz - 1, outside only on the first output slice (likewise y, x)
    const int edge = (oz == 0 ? 4 : 0) | (oy == 0 ? 2 : 0) | (ox == 0 ? 1 : 0);
    const int n = n0 + r;
    const bool ncol = n < N;
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const int nsteps = (k_end - k_begin + 31) / 32;
    for (int st = wave; st < nsteps; st += 4) {
        const int kl = st * 32 + 8 * g;  // local K index of this lane's first value
        bf16x8 av, bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k_begin + kl + j;
            uint16_t a = 0, w = 0;
            if (k < k_end) {
                const int e = koff[kl + j];
                if (mrow && (e & edge) == 0) {
                    const uint16_t v = X[base + (e >> 3)];
                    a = HALF_IN ? to_bf16(__half2float(__ushort_as_half(v))) : v;
                }
                if (ncol) w = W[(size_t)n * K + k];
            }
            av[j] = __builtin_bit_cast(__bf16, a);
            bv[j] = __builtin_bit_cast(__bf16, w);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
    if (wave > 0) red[wave - 1][lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    acc += red[0][lane];
    acc += red[1][lane];
    acc += red[2][lane];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mo = m0 + 4 * g + i;
        if (mo >= M || !ncol) continue;
        if (gridDim.z == 1) {
            const int bo = mo / vox, ro = mo - bo * vox;
            Y[((size_t)bo * N + n) * vox + ro] = to_bf16(fmaxf(acc[i] + bias[n], 0.0f));
        } else {
            partial[((size_t)split * M + mo) * N + n] = acc[i];
        }
    }
}

// Sum of the split-K partial tiles in split order, bias, ReLU, BF16.
__global__ __launch_bounds__(256) void k_conv_fwd_finish(const float *partial, const float *bias, uint16_t *Y,
                                                         int M, int N, int vox, int splits) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= M * N) return;
    const int mo = q / N, n = q - mo * N;
    float v = 0.0f;
    for (int sp = 0; sp < splits; ++sp) v += partial[((size_t)sp * M + mo) * N + n];
    const int bo = mo / vox, ro = mo - bo * vox;
    Y[((size_t)bo * N + n) * vox + ro] = to_bf16(fmaxf(v + bias[n], 0.0f));
}

// K splits of a forward layer: enough workgroups to spread over the chip
// (about 512), at least one 32-step per wave, within the partial buffer.
int fwd_splits(int M, int N, int K, int64_t cap) {
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    const int steps = (K + 31) / 32;
    int sp = std::max(1, std::min((512 + tiles - 1) / tiles, steps / 4));
    while (sp > 1 && (int64_t)sp * M * N > cap) --sp;
    return sp;
}

template <bool HALF_IN>
hipError_t conv_fwd(const uint16_t *X, const uint16_t *W, const float *bias, uint16_t *Y, float *partial,
                    int64_t cap, const ConvShape &sh, hipStream_t s) {
    const int dout = sh.di / 2, vox = dout * dout * dout;
    const int M = sh.B * vox, N = sh.co, K = sh.ci * 27;
    const int steps = (K + 31) / 32;
    const int sp = fwd_splits(M, N, K, cap);
    const int sps = (steps + sp - 1) / sp;
    const int nsplit = (steps + sps - 1) / sps;
    dim3 grid((M + 15) / 16, (N + 15) / 16, nsplit);
    hipLaunchKernelGGL(k_conv_fwd<HALF_IN>, grid, dim3(256), 0, s, X, W, bias, Y, partial, sh, M, N, K, sps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit == 1) return e;
    hipLaunchKernelGGL(k_conv_fwd_finish, dim3((M * N + 255) / 256), dim3(256), 0, s, (const float *)partial, bias, Y,
                       M, N, vox, nsplit);
    return hipGetLastError();
}

// ---- small kernels -----------------------------------------------------------

// Trilinear resampling to side^3 at half-pixel centres, FP16 output.
__global__ void k_downsample(const uint8_t *vol, int nx, int ny, int nz, float scale, int side, uint16_t *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= side * side * side) return;
    const int a = q % side, bq = (q / side) % side, c = q / (side * side);
    const float px = fminf(fmaxf((a + 0.5f) * ((float)nx / side) - 0.5f, 0.0f), (float)(nx - 1));
    const float py = fminf(fmaxf((bq + 0.5f) * ((float)ny / side) - 0.5f, 0.0f), (float)(ny - 1));
    const float pz = fminf(fmaxf((c + 0.5f) * ((float)nz / side) - 0.5f, 0.0f), (float)(nz - 1));
    const int x0 = (int)floorf(px), y0 = (int)floorf(py), z0 = (int)floorf(pz);
    const int x1 = min(x0 + 1, nx - 1), y1 = min(y0 + 1, ny - 1), z1 = min(z0 + 1, nz - 1);
    const float fx = px - x0, fy = py - y0, fz = pz - z0;
    auto V = [&](int x, int y, int z) { return (float)vol[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z)]; };
    const float c00 = V(x0, y0, z0) * (1 - fx) + V(x1, y0, z0) * fx;
    const float c10 = V(x0, y1, z0) * (1 - fx) + V(x1, y1, z0) * fx;
    const float c01 = V(x0, y0, z1) * (1 - fx) + V(x1, y0, z1) * fx;
    const float c11 = V(x0, y1, z1) * (1 - fx) + V(x1, y1, z1) * fx;
    const float v = ((c00 * (1 - fy) + c10 * fy) * (1 - fz) + (c01 * (1 - fy) + c11 * fy) * fz) * scale;
    out[q] = __half_as_ushort(__float2half(v));
}

// Head: out[b][j] = sum_f h[b][f] Wh[j][f] + bh[j] (FP32), one workgroup per (b, j).
__global__ __launch_bounds__(256) void k_head_fwd(const uint16_t *h, const float *Wh, const float *bh, float *out,
                                                  int F) {
    const int b = blockIdx.y, j = blockIdx.x;
    float s = 0.0f;
    for (int f = threadIdx.x; f < F; f += 256) s += from_bf16(h[(size_t)b * F + f]) * Wh[(size_t)j * F + f];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)b * 12 + j] = red[0] + bh[j];
}

// Gaussian NLL (batch mean) and its gradient w.r.t. the 12 outputs.
__global__ void k_nll(const float *out, const float *target, int B, float *dout, float *loss) {
    const int b = threadIdx.x;
    __shared__ float red[1024];
    float l = 0.0f;
    if (b < B) {
        for (int d = 0; d < 6; ++d) {
            const float mu = out[b * 12 + d], lv = out[b * 12 + 6 + d];
            const float xb = target[b * 12 + d], var = target[b * 12 + 6 + d];
            const float e = expf(-lv), dm = xb - mu;
            l += 0.5f * ((var + dm * dm) * e + lv);
            dout[b * 12 + d] = -dm * e / B;
            dout[b * 12 + 6 + d] = 0.5f * (1.0f - (var + dm * dm) * e) / B;
        }
    }
    red[b] = l;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (b < o) red[b] += red[b + o];
        __syncthreads();
    }
    if (b == 0) *loss = red[0] / B;
}

// Head backward: dWh[j][f] = sum_b dout[b][j] h[b][f]; dbh[j] = sum_b dout[b][j];
// dh[b][f] = (sum_j dout[b][j] Wh[j][f]) masked by h > 0.
__global__ void k_head_bwd(const uint16_t *h, const float *Wh, const float *dout, int B, int F, float *dWh,
                           float *dbh, float *dh) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < F) {
        for (int j = 0; j < 12; ++j) {
            float s = 0.0f;
            for (int b = 0; b < B; ++b) s += dout[b * 12 + j] * from_bf16(h[(size_t)b * F + f]);
            dWh[(size_t)j * F + f] = s;
        }
        for (int b = 0; b < B; ++b) {
            float s = 0.0f;
            for (int j = 0; j < 12; ++j) s += dout[b * 12 + j] * Wh[(size_t)j * F + f];
            dh[(size_t)b * F + f] = h[(size_t)b * F + f] != 0 ? s : 0.0f;
        }
    }
    if (f < 12) {
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += dout[b * 12 + f];
        dbh[f] = s;
    }
}

// db[c] = sum over batch and voxels of dY[b][c][...]; one workgroup per channel.
__global__ __launch_bounds__(256) void k_bias_grad(const float *dY, int B, int C, int vox, float *db) {
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int b = 0; b < B; ++b)
        for (int r = threadIdx.x; r < vox; r += 256) s += dY[((size_t)b * C + c) * vox + r];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = red[0];
}

// Adam on FP32 master weights; refresh the bfloat16 copies of the
// convolution weights ([0, n_bf16) of the flat parameter vector).
// One Adam step (Kingma & Ba): m and v are the decayed first and second
// moments of the gradient, c1 = 1 - b1^t and c2 = 1 - b2^t their bias
// corrections.  The coefficients come from the host rounded once from FP64
// (1 - b and 1 - b^t lose digits if formed from FP32 b).
__global__ void k_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, int64_t n_bf16,
                       float lr, float b1, float omb1, float b2, float omb2, float c1, float c2, float eps) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const float gq = g[q];
        const float mq = b1 * m[q] + omb1 * gq;
        const float vq = b2 * v[q] + omb2 * (gq * gq);
        m[q] = mq;
        v[q] = vq;
        const float w = p[q] - lr * (mq / c1) / (sqrtf(vq / c2) + eps);
        p[q] = w;
        if (q < n_bf16) pb[q] = to_bf16(w);
    }
}

__global__ void k_to_bf16(const float *src, uint16_t *dst, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = to_bf16(src[q]);
}

__global__ void k_zero_f32(float *p, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0.0f;
}

unsigned blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65535); }

}  // namespace

// ---- host side ----------------------------------------------------------------

const int kCnnChannels[5] = {2, 16, 32, 64, 64};
const int kCnnSide = 64;
const int kCnnFlat = 64 * 4 * 4 * 4;

int64_t cnn_param_offset(int part) {
    // parts: W1 b1 W2 b2 W3 b3 W4 b4 Wh bh
    int64_t o = 0;
    for (int q = 0; q < part; ++q) {
        const int L = q / 2;
        if (q < 8) o += (q % 2 == 0) ? (int64_t)kCnnChannels[L + 1] * kCnnChannels[L] * 27 : kCnnChannels[L + 1];
        else o += (q == 8) ? 12 * kCnnFlat : 12;
    }
    return o;
}

int64_t cnn_partial_floats(int max_batch) {
    int64_t most = 1;
    for (int L = 0; L < 4; ++L) {
        const int d = (kCnnSide >> L) / 2;
        for (int B = 1; B <= max_batch; ++B) {
            const int M = B * d * d * d, N = kCnnChannels[L + 1], K = kCnnChannels[L] * 27;
            most = std::max(most, (int64_t)fwd_splits(M, N, K, INT64_MAX) * M * N);
        }
    }
    return std::min<int64_t>(most, (int64_t)1 << 22);
}

hipError_t cnn_downsample(const uint8_t *vol, const int32_t n[3], float scale, uint16_t *out, hipStream_t s) {
    const int tot = kCnnSide * kCnnSide * kCnnSide;
    hipLaunchKernelGGL(k_downsample, dim3((tot + 255) / 256), dim3(256), 0, s, vol, n[0], n[1], n[2], scale, kCnnSide,
                       out);
    return hipGetLastError();
}

hipError_t cnn_forward(const CnnBuffers &c, const uint16_t *input, int B, float *out, hipStream_t s) {
    const uint16_t *x = input;
    for (int L = 0; L < 4; ++L) {
        ConvShape sh{B, kCnnChannels[L], kCnnChannels[L + 1], kCnnSide >> L};
        const int dout = sh.di / 2;
        const uint16_t *W = c.wbf16 + cnn_param_offset(2 * L);
        const float *bias = c.params + cnn_param_offset(2 * L + 1);
        (void)dout;
        hipError_t e;
        if (L == 0) e = conv_fwd<true>(x, W, bias, c.act[0], c.partial, c.partial_cap, sh, s);
        else e = conv_fwd<false>(x, W, bias, c.act[L], c.partial, c.partial_cap, sh, s);
        if (e != hipSuccess) return e;
        x = c.act[L];
    }
    hipLaunchKernelGGL(k_head_fwd, dim3(12, B), dim3(256), 0, s, c.act[3], c.params + cnn_param_offset(8),
                       c.params + cnn_param_offset(9), out, kCnnFlat);
    return hipGetLastError();
}

hipError_t cnn_backward(const CnnBuffers &c, const uint16_t *input, int B, const float *out, const float *target,
                        float *loss_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_nll, dim3(1), dim3(1024), 0, s, out, target, B, c.dout, loss_dev);
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks(c.n_params)), dim3(256), 0, s, c.grads, (int64_t)c.n_params);
    // head
    hipLaunchKernelGGL(k_head_bwd, dim3((kCnnFlat + 255) / 256), dim3(256), 0, s, c.act[3],
                       c.params + cnn_param_offset(8), c.dout, B, kCnnFlat, c.grads + cnn_param_offset(8),
                       c.grads + cnn_param_offset(9), c.dact[3]);
    for (int L = 3; L >= 0; --L) {
        ConvShape sh{B, kCnnChannels[L], kCnnChannels[L + 1], kCnnSide >> L};
        const int dout = sh.di / 2, vox = dout * dout * dout;
        const float *dY = c.dact[L];
        hipLaunchKernelGGL(k_bias_grad, dim3(sh.co), dim3(256), 0, s, dY, B, sh.co, vox,
                           c.grads + cnn_param_offset(2 * L + 1));
        const int Mw = sh.co, Nw = sh.ci * 27, Kw = B * vox;
        const int splits = std::max(1, std::min(512, Kw / 256));
        hipError_t e;
        if (L == 0)
            e = run_gemm(WgradOp<true>{dY, input, c.grads + cnn_param_offset(0), sh, Mw, Nw, Kw}, splits, s);
        else
            e = run_gemm(WgradOp<false>{dY, c.act[L - 1], c.grads + cnn_param_offset(2 * L), sh, Mw, Nw, Kw}, splits,
                         s);
        if (e != hipSuccess) return e;
        if (L > 0) {
            const int vin = sh.di * sh.di * sh.di;
            e = run_gemm(DgradOp{dY, c.wbf16 + cnn_param_offset(2 * L), c.act[L - 1], c.dact[L - 1], sh, B * vin,
                                 sh.ci, sh.co * 27},
                         1, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

hipError_t cnn_adam(const CnnBuffers &c, float lr, int t, hipStream_t s) {
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, (double)t)), c2 = (float)(1.0 - pow(b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(c.n_params)), dim3(256), 0, s, c.params, c.grads, c.adam_m, c.adam_v,
                       c.wbf16, (int64_t)c.n_params, (int64_t)cnn_param_offset(8), lr, (float)b1, (float)(1.0 - b1),
                       (float)b2, (float)(1.0 - b2), c1, c2, 1e-8f);
    return hipGetLastError();
}

hipError_t cnn_refresh_bf16(const CnnBuffers &c, hipStream_t s) {
    const int64_t n = cnn_param_offset(8);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n)), dim3(256), 0, s, c.params, c.wbf16, n);
    return hipGetLastError();
}

}  // namespace smc
