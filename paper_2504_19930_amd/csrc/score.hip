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
#include "internal.h"

namespace smc {
namespace {

constexpr int kTX = 32;
constexpr int kTY = 8;
constexpr int kThreads = kTX * kTY;
constexpr int kWaves = kThreads / 64;
constexpr int kZChunkMax = 256;  // keeps every per-thread 32-bit sum below 2^32

struct KArgs {
    const uint8_t *src, *src_ok, *tgt, *tgt_fov;
    const float *words;
    unsigned long long *sums;
    int32_t sn0, sn1, sn2, tn0, tn1, tn2;
    uint32_t p0, np;
    int32_t tiles_x, tiles_y, zchunk;
};

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

struct Tile {
    int i, j, k0, k1;
    bool ok;
    uint32_t pbase;
    int npg;
};

template <int PT>
__device__ __forceinline__ Tile tile_of(const KArgs &a) {
    Tile t;
    const int tiles = a.tiles_x * a.tiles_y;
    int b = blockIdx.x;
    const int zc = b / tiles;
    b -= zc * tiles;
    const int ty = b / a.tiles_x;
    const int tx = b - ty * a.tiles_x;
    t.i = tx * kTX + (int)(threadIdx.x % kTX);
    t.j = ty * kTY + (int)(threadIdx.x / kTX);
    t.ok = t.i < a.tn0 && t.j < a.tn1;
    t.k0 = zc * a.zchunk;
    t.k1 = min(t.k0 + a.zchunk, a.tn2);
    t.pbase = a.p0 + blockIdx.y * PT;
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
        const float *w = a.words + 12 * (size_t)q;
        mx[p] = fmaf(w[1], fj, fmaf(w[0], fi, w[3]));
        my[p] = fmaf(w[5], fj, fmaf(w[4], fi, w[7]));
        mz[p] = fmaf(w[9], fj, fmaf(w[8], fi, w[11]));
        ax[p] = w[2];
        ay[p] = w[6];
        az[p] = w[10];
    }
}

// ---------------------------------------------------------------- masks

// Source byte: bit 0 = inside the source FOV, bit 1 = mask on (and in FOV).
// Target byte: bit 0 = inside the target FOV, bit 1 = mask on (and in FOV).
// Per particle two packed counters: acc1 = n | a << 16, acc2 = b_ov | c << 16
// (each half counts at most one voxel per z step, and a z-chunk < 2^16).
template <int PT>
__global__ __launch_bounds__(kThreads) void k_score_mask(const KArgs a) {
    const Tile t = tile_of<PT>(a);
    float mx[PT], my[PT], mz[PT], ax[PT], ay[PT], az[PT];
    column_terms<PT>(a, t, mx, my, mz, ax, ay, az);
    uint32_t acc1[PT], acc2[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) acc1[p] = acc2[p] = 0u;
    if (t.ok) {
        const size_t plane = (size_t)a.tn0 * (size_t)a.tn1;
        const uint8_t *tp = a.tgt + (size_t)t.i + (size_t)a.tn0 * (size_t)t.j + plane * (size_t)t.k0;
        const uint32_t sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
        for (int k = t.k0; k < t.k1; ++k, tp += plane) {
            const uint32_t tb = *tp;
            const uint32_t keep = (tb & 1u) ? 3u : 0u;
            const bool ton = (tb & 2u) != 0u;
            const float fk = (float)k;
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                if (p < t.npg) {
                    const int ix = (int)floorf(fmaf(ax[p], fk, mx[p]));
                    const int iy = (int)floorf(fmaf(ay[p], fk, my[p]));
                    const int iz = (int)floorf(fmaf(az[p], fk, mz[p]));
                    uint32_t v = 0u;
                    if ((uint32_t)ix < (uint32_t)a.sn0 && (uint32_t)iy < (uint32_t)a.sn1 &&
                        (uint32_t)iz < (uint32_t)a.sn2)
                        v = a.src[(uint32_t)ix + (uint32_t)a.sn0 * (uint32_t)iy + sn01 * (uint32_t)iz];
                    v &= keep;
                    const uint32_t inc = (v & 1u) | ((v & 2u) << 15);
                    acc1[p] += inc;
                    acc2[p] += ton ? inc : 0u;
                }
            }
        }
    }
    __shared__ unsigned long long red[kWaves][PT][4];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const uint32_t n = wave_sum(acc1[p] & 0xFFFFu);
        const uint32_t aa = wave_sum(acc1[p] >> 16);
        const uint32_t b = wave_sum(acc2[p] & 0xFFFFu);
        const uint32_t c = wave_sum(acc2[p] >> 16);
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

// Sums per particle over the overlap: n, s, t, s^2, t^2, s t with s the
// sampled source value in units of 1/256 (exact: s_fx = floor(256 s + 0.5)).
template <int PT, bool TRI, bool SOK, bool TFOV>
__global__ __launch_bounds__(kThreads) void k_score_image(const KArgs a) {
    const Tile t = tile_of<PT>(a);
    float mx[PT], my[PT], mz[PT], ax[PT], ay[PT], az[PT];
    column_terms<PT>(a, t, mx, my, mz, ax, ay, az);
    uint32_t cn[PT], cs[PT], ct[PT], ctt[PT], cst[PT];
    unsigned long long css[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        cn[p] = cs[p] = ct[p] = ctt[p] = cst[p] = 0u;
        css[p] = 0ull;
    }
    if (t.ok) {
        const size_t plane = (size_t)a.tn0 * (size_t)a.tn1;
        const size_t tofs0 = (size_t)t.i + (size_t)a.tn0 * (size_t)t.j;
        const uint32_t sn0 = (uint32_t)a.sn0, sn01 = (uint32_t)a.sn0 * (uint32_t)a.sn1;
        const float ex = (float)(a.sn0 - 1), ey = (float)(a.sn1 - 1), ez = (float)(a.sn2 - 1);
        for (int k = t.k0; k < t.k1; ++k) {
            const size_t tofs = tofs0 + plane * (size_t)k;
            if (TFOV && a.tgt_fov[tofs] == 0) continue;
            const uint32_t tv = a.tgt[tofs];
            const uint32_t tv2 = tv * tv;
            const float fk = (float)k;
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                if (p < t.npg) {
                    const float ux = fmaf(ax[p], fk, mx[p]);
                    const float uy = fmaf(ay[p], fk, my[p]);
                    const float uz = fmaf(az[p], fk, mz[p]);
                    uint32_t sfx;
                    if (TRI) {
                        if (!(ux >= 0.0f && ux <= ex && uy >= 0.0f && uy <= ey && uz >= 0.0f && uz <= ez))
                            continue;
                        const float flx = floorf(ux), fly = floorf(uy), flz = floorf(uz);
                        const uint32_t ix = (uint32_t)flx, iy = (uint32_t)fly, iz = (uint32_t)flz;
                        const float fx = ux - flx, fy = uy - fly, fz = uz - flz;
                        const uint32_t base = ix + sn0 * iy + sn01 * iz;
                        if (SOK && a.src_ok[base] == 0) continue;
                        const uint32_t dx = ix < (uint32_t)(a.sn0 - 1) ? 1u : 0u;
                        const uint32_t dy = iy < (uint32_t)(a.sn1 - 1) ? sn0 : 0u;
                        const uint32_t dz = iz < (uint32_t)(a.sn2 - 1) ? sn01 : 0u;
                        const uint8_t *S = a.src + base;
                        const float v000 = (float)S[0], v100 = (float)S[dx];
                        const float v010 = (float)S[dy], v110 = (float)S[dy + dx];
                        const float v001 = (float)S[dz], v101 = (float)S[dz + dx];
                        const float v011 = (float)S[dz + dy], v111 = (float)S[dz + dy + dx];
                        const float x00 = fmaf(fx, v100 - v000, v000);
                        const float x10 = fmaf(fx, v110 - v010, v010);
                        const float x01 = fmaf(fx, v101 - v001, v001);
                        const float x11 = fmaf(fx, v111 - v011, v011);
                        const float y0 = fmaf(fy, x10 - x00, x00);
                        const float y1 = fmaf(fy, x11 - x01, x01);
                        const float s = fmaf(fz, y1 - y0, y0);
                        sfx = (uint32_t)(s * 256.0f + 0.5f);
                    } else {
                        const int ix = (int)floorf(ux), iy = (int)floorf(uy), iz = (int)floorf(uz);
                        if (!((uint32_t)ix < (uint32_t)a.sn0 && (uint32_t)iy < (uint32_t)a.sn1 &&
                              (uint32_t)iz < (uint32_t)a.sn2))
                            continue;
                        const uint32_t m = (uint32_t)ix + sn0 * (uint32_t)iy + sn01 * (uint32_t)iz;
                        if (SOK && a.src_ok[m] == 0) continue;
                        sfx = (uint32_t)a.src[m] << 8;
                    }
                    cn[p] += 1u;
                    cs[p] += sfx;
                    ct[p] += tv;
                    css[p] += (unsigned long long)sfx * sfx;
                    ctt[p] += tv2;
                    cst[p] += sfx * tv;
                }
            }
        }
    }
    __shared__ unsigned long long red[kWaves][PT][6];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const uint32_t n = wave_sum(cn[p]);
        const uint32_t s1 = wave_sum(cs[p]);
        const uint32_t t1 = wave_sum(ct[p]);
        const unsigned long long s2 = wave_sum(css[p]);
        const uint32_t t2 = wave_sum(ctt[p]);
        const unsigned long long st = wave_sum((unsigned long long)cst[p]);
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

constexpr int kPT = 8;

KArgs make_args(const ScoreLaunch &L, int *nz_chunks) {
    KArgs a;
    a.src = L.src;
    a.src_ok = L.src_ok;
    a.tgt = L.tgt;
    a.tgt_fov = L.tgt_fov;
    a.words = L.words;
    a.sums = L.sums;
    a.sn0 = L.sn[0];
    a.sn1 = L.sn[1];
    a.sn2 = L.sn[2];
    a.tn0 = L.tn[0];
    a.tn1 = L.tn[1];
    a.tn2 = L.tn[2];
    a.p0 = L.p0;
    a.np = L.np;
    a.tiles_x = (L.tn[0] + kTX - 1) / kTX;
    a.tiles_y = (L.tn[1] + kTY - 1) / kTY;
    const int chunks = (L.tn[2] + kZChunkMax - 1) / kZChunkMax;
    a.zchunk = (L.tn[2] + chunks - 1) / chunks;
    *nz_chunks = chunks;
    return a;
}

}  // namespace

void score_grid(const ScoreLaunch &L, dim3 *grid, dim3 *block) {
    int chunks;
    const KArgs a = make_args(L, &chunks);
    *grid = dim3((unsigned)(a.tiles_x * a.tiles_y * chunks), (L.np + kPT - 1) / kPT, 1);
    *block = dim3(kThreads, 1, 1);
}

hipError_t launch_score(const ScoreLaunch &L, hipStream_t s) {
    if (L.np == 0) return hipSuccess;
    int chunks;
    const KArgs a = make_args(L, &chunks);
    dim3 grid, block;
    score_grid(L, &grid, &block);
    if (L.mode == kModeMask) {
        hipLaunchKernelGGL(k_score_mask<kPT>, grid, block, 0, s, a);
    } else {
        const bool tri = L.mode == kModeImageTrilinear;
        const bool sok = L.src_ok != nullptr, tfov = L.tgt_fov != nullptr;
#define SMC_IMG(T, A, B) hipLaunchKernelGGL((k_score_image<kPT, T, A, B>), grid, block, 0, s, a)
        if (tri) {
            if (sok) { if (tfov) SMC_IMG(true, true, true); else SMC_IMG(true, true, false); }
            else { if (tfov) SMC_IMG(true, false, true); else SMC_IMG(true, false, false); }
        } else {
            if (sok) { if (tfov) SMC_IMG(false, true, true); else SMC_IMG(false, true, false); }
            else { if (tfov) SMC_IMG(false, false, true); else SMC_IMG(false, false, false); }
        }
#undef SMC_IMG
    }
    return hipGetLastError();
}

}  // namespace smc
