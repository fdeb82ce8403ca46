// Learned pressure predictor: a 4-level 3D U-Net (16/32/48/64 channels, 3x3x3
// convolutions) in BF16 with FP32 accumulation on the gfx950 matrix cores, its
// backward pass and an Adam optimiser, all hand-written.
//
// Activations are channel-last BF16 ([z][y][x][c], c fastest) on cubic grids
// of n^3 cells (n divisible by 8).  Convolutions are implicit GEMMs on the
// matrix cores (v_mfma_f32_16x16x32_bf16 for grids of at least 16 cells per
// axis, see k_conv): the K dimension runs over (tap, input channel) and the
// input tile with its 1-voxel halo is staged in LDS.  Architecture (layer: level, in ->
// out channels):
//   encoder  e0a 0 16->16, e0b 0 16->16 (s0), pool
//            e1a 1 16->32, e1b 1 32->32 (s1), pool
//            e2a 2 32->48, e2b 2 48->48 (s2), pool
//            e3a 3 48->64, e3b 3 64->64 (d3)
//   decoder  d2c 2 64->48 (+s2), d2d 2 48->48 (d2)    after nearest upsampling
//            d1c 1 48->32 (+s1), d1d 1 32->32 (d1)
//            d0c 0 32->16 (+s0), d0d 0 16->16 (d0)
//   output   out 0 16->16, no activation; channel 0 is the prediction.
// Every convolution but the last is followed by ReLU; the skip connections are
// added before the ReLU.  The input has 3 feature channels padded to 16.
#include "../../include/stokes.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace {

typedef uint16_t bf16;
typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kLayers = 15;
constexpr int kBiasBlocks = 1024;      // blocks (partial sums) of the bias-gradient launch
constexpr int kLevels = 4;
constexpr int kCh[kLevels] = {16, 32, 48, 64};

struct LayerSpec {
    int level, cin, cout, relu;
};
constexpr LayerSpec kSpec[kLayers] = {
    {0, 16, 16, 1}, {0, 16, 16, 1}, {1, 16, 32, 1}, {1, 32, 32, 1}, {2, 32, 48, 1}, {2, 48, 48, 1},
    {3, 48, 64, 1}, {3, 64, 64, 1}, {2, 64, 48, 1}, {2, 48, 48, 1}, {1, 48, 32, 1}, {1, 32, 32, 1},
    {0, 32, 16, 1}, {0, 16, 16, 1}, {0, 16, 16, 0}};

__host__ __device__ inline float bf2f(bf16 h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}
__host__ __device__ inline bf16 f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)(u >> 16);   // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);                                  // round to nearest even
    return (bf16)(u >> 16);
}

// ------------------------------------------------------------------ convolution
// out[v][co] = act( sum_{tap, ci} W[co][tap][ci] * in[v + off(tap)][ci] + bias[co] + skip[v][co] )
// in:  n^3 x CIN, W: COUT x 27 x CIN (bf16), out: n^3 x COUT.  Zero padding.
// mask != nullptr (backward-data use): the result is multiplied by (mask[v][co] > 0).
//
// Implicit GEMM on v_mfma_f32_16x16x32_bf16 with K = (tap, ci) flattened (27 CIN,
// in chunks of 32; a lane's 8 consecutive k never straddle a tap since CIN is a
// multiple of 16).  A block owns 16 (x) x 4 (y) voxels and marches over zc
// z-planes; wavefront w computes y row w, all COUT channels at once (one
// accumulator per 16 channels, so each B operand read from LDS feeds COUT/16
// MFMAs).  LDS holds a ring of three input planes with the 1-voxel x-y halo
// (voxel stride CIN + 8 to spread the banks) and, when they fit in 32 KiB (the
// 16 -> 16, 16 -> 32 and 32 -> 16 layers, which run on the two finest levels),
// the layer's weights, staged once per block; larger layers read their weights
// through the caches (staging 55 KiB and more would leave one block per CU).
constexpr int kConvWLds = 32 * 1024;

template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_conv(int n, int zc, const bf16 *__restrict__ in, const bf16 *__restrict__ W,
        const float *__restrict__ bias, const bf16 *__restrict__ skip, const bf16 *__restrict__ mask, int relu,
        bf16 *__restrict__ out, float *__restrict__ out32) {
    constexpr int K = 27 * CIN, NCH = (K + 31) / 32, NCO = COUT / 16;
    constexpr int VS = CIN + 8, HP = 6 * 18 * VS;          // halo voxel stride, plane size (elements)
    constexpr int WS = K + 8;                              // LDS weight row stride (elements)
    constexpr bool WL = COUT * WS * 2 <= kConvWLds;
    __shared__ __attribute__((aligned(16))) bf16 ring[3 * HP];
    __shared__ __attribute__((aligned(16))) bf16 wsh[WL ? COUT * WS : 8];
    const int x0 = blockIdx.x * 16, y0 = blockIdx.y * 4, z0 = blockIdx.z * zc;
    const int z1 = min(z0 + zc, n);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int j = lane & 15, g = lane >> 4;
    constexpr int Q = CIN / 8;                             // 16-byte quads per voxel
    auto load_plane = [&](int p) {                         // input plane p -> ring slot p mod 3
        bf16 *dst = ring + ((p + 3) % 3) * HP;
        for (int t = tid; t < 108 * Q; t += 256) {
            const int vq = t / Q, cq = t % Q;
            const int hx = vq % 18, hy = vq / 18;
            const int gx = x0 + hx - 1, gy = y0 + hy - 1;
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (gx >= 0 && gx < n && gy >= 0 && gy < n && p >= 0 && p < n)
                val = *reinterpret_cast<const uint4 *>(in + ((size_t)((p * n + gy) * n + gx)) * CIN + cq * 8);
            *reinterpret_cast<uint4 *>(dst + (hy * 18 + hx) * VS + cq * 8) = val;
        }
    };
    if (WL) {
        for (int t = tid; t < COUT * (K / 8); t += 256) {
            const int co = t / (K / 8), q = t % (K / 8);
            *reinterpret_cast<uint4 *>(wsh + co * WS + q * 8) =
                *reinterpret_cast<const uint4 *>(W + (size_t)co * K + q * 8);
        }
    }
    load_plane(z0 - 1);
    load_plane(z0);
    const int x = x0 + j, y = y0 + w;
    for (int z = z0; z < z1; ++z) {
        load_plane(z + 1);
        __syncthreads();
        f4v acc[NCO];
#pragma unroll
        for (int c = 0; c < NCO; ++c) acc[c] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
        for (int ch = 0; ch < NCH; ++ch) {
            const int k0 = ch * 32 + g * 8;
            uint4 bq = make_uint4(0u, 0u, 0u, 0u);
            const bool kin = k0 < K;
            if (kin) {
                const int tap = k0 / CIN, ci = k0 % CIN;
                const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                bq = *reinterpret_cast<const uint4 *>(ring + ((z - 1 + dz + 3) % 3) * HP + ((w + dy) * 18 + j + dx) * VS + ci);
            }
            const bf8v bv = __builtin_bit_cast(bf8v, bq);
#pragma unroll
            for (int c = 0; c < NCO; ++c) {
                uint4 aq = make_uint4(0u, 0u, 0u, 0u);
                if (kin) {
                    if (WL) aq = *reinterpret_cast<const uint4 *>(wsh + (c * 16 + j) * WS + k0);
                    else aq = *reinterpret_cast<const uint4 *>(W + (size_t)(c * 16 + j) * K + k0);
                }
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, aq), bv, acc[c], 0, 0, 0);
            }
        }
        // lane holds voxel x and output channels 16 c + 4 g + e
        const size_t v = (size_t)((z * n + y) * n + x);
#pragma unroll
        for (int c = 0; c < NCO; ++c) {
            const int cb = c * 16 + g * 4;
            float r[4] = {acc[c][0], acc[c][1], acc[c][2], acc[c][3]};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = cb + e;
                float val = r[e];
                if (bias) val += bias[co];
                if (skip) val += bf2f(skip[v * COUT + co]);
                if (relu) val = fmaxf(val, 0.f);
                if (mask && !(bf2f(mask[v * COUT + co]) > 0.f)) val = 0.f;
                r[e] = val;
            }
            if (out) {
                ushort4 o;
                o.x = f2bf(r[0]); o.y = f2bf(r[1]); o.z = f2bf(r[2]); o.w = f2bf(r[3]);
                *reinterpret_cast<ushort4 *>(out + v * COUT + cb) = o;
            }
            if (out32) *reinterpret_cast<float4 *>(out32 + v * COUT + cb) = make_float4(r[0], r[1], r[2], r[3]);
        }
        __syncthreads();                                   // ring slot of z - 1 is loaded next
    }
}

// Weight gradient: dW[co][tap][ci] = sum_v dy[v][co] * in[v + off(tap)][ci], as
// one partial copy of dW per block along x (part[blockIdx.x][co][tap][ci]),
// summed in block order by k_sum_partials so that training is deterministic.
// Grid: x = voxel-tile groups (each block walks `tiles` tiles of 16x4x1 voxels),
// y = (co tile, ci tile) pair.  Wave w accumulates the taps w, w+4, ... .
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_conv_wgrad(int n, int tiles, const bf16 *__restrict__ in,
        const bf16 *__restrict__ dy, float *__restrict__ part) {
    float *dW = part + (size_t)blockIdx.x * COUT * 27 * CIN;
    __shared__ bf16 hx_s[3 * 6 * 18 * 16];   // input halo, 16 channels of this ci tile
    __shared__ bf16 dy_s[64 * 16];           // gradient tile, 16 channels of this co tile
    constexpr int NCI = CIN / 16;
    const int co0 = (blockIdx.y / NCI) * 16, ci0 = (blockIdx.y % NCI) * 16;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int j = lane & 15, kq = lane >> 4;
    const int tx_n = n / 16, ty_n = n / 4;
    const long long ntiles = (long long)tx_n * ty_n * n;
    f4v acc[7];
#pragma unroll
    for (int t = 0; t < 7; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < tiles; ++it) {
        const long long tile = (long long)blockIdx.x * tiles + it;
        if (tile >= ntiles) break;
        const int bxi = (int)(tile % tx_n), byi = (int)((tile / tx_n) % ty_n), z = (int)(tile / ((long long)tx_n * ty_n));
        const int x0 = bxi * 16, y0 = byi * 4;
        __syncthreads();
        for (int t = tid; t < 324 * 4; t += 256) {
            const int vq = t >> 2, cq = t & 3;
            const int hxx = vq % 18, hy = (vq / 18) % 6, hz = vq / 108;
            const int gx = x0 + hxx - 1, gy = y0 + hy - 1, gz = z + hz - 1;
            uint2 val = make_uint2(0u, 0u);
            if (gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n)
                val = *reinterpret_cast<const uint2 *>(in + ((size_t)((gz * n + gy) * n + gx)) * CIN + ci0 + cq * 4);
            *reinterpret_cast<uint2 *>(hx_s + vq * 16 + cq * 4) = val;
        }
        {
            const int vq = tid >> 2, cq = tid & 3;        // 64 voxels x 4 quads
            const int vx = x0 + (vq & 15), vy = y0 + (vq >> 4);
            *reinterpret_cast<uint2 *>(dy_s + vq * 16 + cq * 4) =
                *reinterpret_cast<const uint2 *>(dy + ((size_t)((z * n + vy) * n + vx)) * COUT + co0 + cq * 4);
        }
        __syncthreads();
        // K = 64 voxels of the tile, 16 per MFMA: chunk r is the y row r of the tile
#pragma unroll
        for (int t = 0; t < 7; ++t) {
            const int tap = w + 4 * t;
            if (tap < 27) {
                const int dz = tap / 9, dyy = (tap / 3) % 3, dx = tap % 3;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    s4v a, bb;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int vx = kq * 4 + e;                       // voxel x in the chunk
                        a[e] = (short)dy_s[(rr * 16 + vx) * 16 + j];    // A[co=j][k=voxel]
                        bb[e] = (short)hx_s[((dz * 6 + (rr + dyy)) * 18 + (vx + dx)) * 16 + j];  // B[k=voxel][ci=j]
                    }
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[t], 0, 0, 0);
                }
            }
        }
    }
    // D[co][ci]: lane holds ci = j and co = 4*kq + e
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        const int tap = w + 4 * t;
        if (tap < 27) {
#pragma unroll
            for (int e = 0; e < 4; ++e) dW[((size_t)(co0 + kq * 4 + e) * 27 + tap) * CIN + ci0 + j] = acc[t][e];
        }
    }
}

// Small grids (n < 16, or not a multiple of 16): the same convolution without LDS staging.  A wavefront
// takes 16 consecutive voxels of the flattened grid and gathers its operands
// from global memory (zero outside the grid).
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_conv_small(int n, const bf16 *__restrict__ in, const bf16 *__restrict__ W,
        const float *__restrict__ bias, const bf16 *__restrict__ skip, const bf16 *__restrict__ mask, int relu,
        bf16 *__restrict__ out, float *__restrict__ out32) {
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int j = lane & 15, kq = lane >> 4;
    const long long nv = (long long)n * n * n;
    const long long v = ((long long)blockIdx.x * 4 + w) * 16 + j;
    if (((long long)blockIdx.x * 4 + w) * 16 >= nv) return;      // whole wavefront out of range
    const bool valid = v < nv;
    const int x = (int)(v % n), y = (int)((v / n) % n), z = (int)(v / ((long long)n * n));
#pragma unroll 1
    for (int co0 = 0; co0 < COUT; co0 += 16) {
        f4v acc = {0.f, 0.f, 0.f, 0.f};
        const bf16 *wrow = W + (size_t)(co0 + j) * 27 * CIN + kq * 4;
#pragma unroll 1
        for (int tap = 0; tap < 27; ++tap) {
            const int gx = x + tap % 3 - 1, gy = y + (tap / 3) % 3 - 1, gz = z + tap / 9 - 1;
            const bool ok = valid && gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
            const bf16 *src = in + ((size_t)((gz * n + gy) * n + gx)) * CIN + kq * 4;
            for (int ci0 = 0; ci0 < CIN; ci0 += 16) {
                s4v a = *reinterpret_cast<const s4v *>(wrow + tap * CIN + ci0);
                s4v bb = {0, 0, 0, 0};
                if (ok) bb = *reinterpret_cast<const s4v *>(src + ci0);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc, 0, 0, 0);
            }
        }
        if (!valid) continue;
        float r[4] = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = co0 + kq * 4 + e;
            float val = r[e];
            if (bias) val += bias[co];
            if (skip) val += bf2f(skip[v * COUT + co]);
            if (relu) val = fmaxf(val, 0.f);
            if (mask && !(bf2f(mask[v * COUT + co]) > 0.f)) val = 0.f;
            r[e] = val;
        }
        if (out) {
            ushort4 o;
            o.x = f2bf(r[0]); o.y = f2bf(r[1]); o.z = f2bf(r[2]); o.w = f2bf(r[3]);
            *reinterpret_cast<ushort4 *>(out + v * COUT + co0 + kq * 4) = o;
        }
        if (out32) *reinterpret_cast<float4 *>(out32 + v * COUT + co0 + kq * 4) = make_float4(r[0], r[1], r[2], r[3]);
    }
}

// Small-grid weight gradient: one wavefront per (tap, co tile, ci tile) and
// voxel chunk; operands gathered from global memory; one partial copy of dW
// per chunk (as k_conv_wgrad).
template <int CIN, int COUT>
__global__ void __launch_bounds__(64) k_conv_wgrad_small(int n, int chunk, const bf16 *__restrict__ in,
        const bf16 *__restrict__ dy, float *__restrict__ part) {
    float *dW = part + (size_t)blockIdx.x * COUT * 27 * CIN;
    constexpr int NCI = CIN / 16;
    const int tap = blockIdx.y % 27, pair = blockIdx.y / 27;
    const int co0 = (pair / NCI) * 16, ci0 = (pair % NCI) * 16;
    const int lane = threadIdx.x, j = lane & 15, kq = lane >> 4;
    const long long nv = (long long)n * n * n;
    const int ox = tap % 3 - 1, oy = (tap / 3) % 3 - 1, oz = tap / 9 - 1;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    for (long long v0 = (long long)blockIdx.x * chunk; v0 < min(nv, (long long)(blockIdx.x + 1) * chunk); v0 += 16) {
        s4v a, bb;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const long long v = v0 + kq * 4 + e;
            short av = 0, bv = 0;
            if (v < nv) {
                av = (short)dy[v * COUT + co0 + j];
                const int x = (int)(v % n) + ox, y = (int)((v / n) % n) + oy, z = (int)(v / ((long long)n * n)) + oz;
                if (x >= 0 && x < n && y >= 0 && y < n && z >= 0 && z < n)
                    bv = (short)in[((size_t)((z * n + y) * n + x)) * CIN + ci0 + j];
            }
            a[e] = av;
            bb[e] = bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) dW[((size_t)(co0 + kq * 4 + e) * 27 + tap) * CIN + ci0 + j] = acc[e];
}

// Backward-data weights: Wt[ci][26 - tap][co] = W[co][tap][ci]
__global__ void k_flip_weights(int cin, int cout, const bf16 *__restrict__ W, bf16 *__restrict__ Wt) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int total = cin * cout * 27;
    if (t >= total) return;
    int ci = t % cin, tap = (t / cin) % 27, co = t / (cin * 27);
    Wt[((size_t)ci * 27 + (26 - tap)) * cout + co] = W[t];
}

// out[i] += sum_b part[b][i] over b = 0 .. nb-1 in order (i < m)
__global__ void k_sum_partials(long long m, int nb, const float *__restrict__ part, float *__restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int b = 0; b < nb; ++b) acc += part[(size_t)b * m + i];
        out[i] += acc;
    }
}

// bias gradient, one partial per block: part[block][c] = sum over the block's
// voxels of dy[v][c] (block-strided; the block's lane groups summed in order)
__global__ void __launch_bounds__(256) k_bias_grad(long long nv, int C, const bf16 *__restrict__ dy,
                                                   float *__restrict__ part) {
    __shared__ float sh[256];
    const int c = threadIdx.x % C;
    const int lanes = blockDim.x / C;
    float s = 0.f;
    if (threadIdx.x / C < lanes)
        for (long long v = (long long)blockIdx.x * lanes + threadIdx.x / C; v < nv; v += (long long)gridDim.x * lanes)
            s += bf2f(dy[v * C + c]);
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        float acc = 0.f;
        for (int gq = 0; gq < lanes; ++gq) acc += sh[gq * C + threadIdx.x];
        part[(size_t)blockIdx.x * C + threadIdx.x] = acc;
    }
}

// g = (g1 + g2) * (act > 0)   (g2 optional), elementwise over n
__global__ void k_mask_grad(long long n, const bf16 *__restrict__ g1, const bf16 *__restrict__ g2,
                            const bf16 *__restrict__ act, bf16 *__restrict__ g) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; t < n; t += (long long)gridDim.x * blockDim.x) {
        float v = bf2f(g1[t]) + (g2 ? bf2f(g2[t]) : 0.f);
        g[t] = f2bf(bf2f(act[t]) > 0.f ? v : 0.f);
    }
}

// average pooling 2x2x2 (channel-last), fine n -> coarse n/2
__global__ void k_pool(int nc, int C, const bf16 *__restrict__ f, bf16 *__restrict__ c) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)nc * nc * nc * C;
    if (t >= total) return;
    int ch = (int)(t % C);
    long long vc = t / C;
    int X = (int)(vc % nc), Y = (int)((vc / nc) % nc), Z = (int)(vc / ((long long)nc * nc));
    int nf = 2 * nc;
    float s = 0.f;
    for (int d = 0; d < 8; ++d) {
        int x = 2 * X + (d & 1), y = 2 * Y + ((d >> 1) & 1), z = 2 * Z + (d >> 2);
        s += bf2f(f[((size_t)((z * nf + y) * nf + x)) * C + ch]);
    }
    c[t] = f2bf(0.125f * s);
}

// pooling backward, accumulated: gf[child] += gc[parent] / 8
__global__ void k_pool_bwd_add(int nf, int C, const bf16 *__restrict__ gc, bf16 *__restrict__ gf) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)nf * nf * nf * C;
    if (t >= total) return;
    int ch = (int)(t % C);
    long long v = t / C;
    int x = (int)(v % nf), y = (int)((v / nf) % nf), z = (int)(v / ((long long)nf * nf));
    int nc = nf / 2;
    float add = 0.125f * bf2f(gc[((size_t)(((z >> 1) * nc + (y >> 1)) * nc + (x >> 1))) * C + ch]);
    gf[t] = f2bf(bf2f(gf[t]) + add);
}

// nearest upsampling coarse n/2 -> fine n
__global__ void k_upsample(int nf, int C, const bf16 *__restrict__ c, bf16 *__restrict__ f) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)nf * nf * nf * C;
    if (t >= total) return;
    int ch = (int)(t % C);
    long long v = t / C;
    int x = (int)(v % nf), y = (int)((v / nf) % nf), z = (int)(v / ((long long)nf * nf));
    int nc = nf / 2;
    f[t] = c[((size_t)(((z >> 1) * nc + (y >> 1)) * nc + (x >> 1))) * C + ch];
}

// upsampling backward: gc[parent] = sum of the 8 children
__global__ void k_upsample_bwd(int nc, int C, const bf16 *__restrict__ gf, bf16 *__restrict__ gc) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)nc * nc * nc * C;
    if (t >= total) return;
    int ch = (int)(t % C);
    long long vc = t / C;
    int X = (int)(vc % nc), Y = (int)((vc / nc) % nc), Z = (int)(vc / ((long long)nc * nc));
    int nf = 2 * nc;
    float s = 0.f;
    for (int d = 0; d < 8; ++d) {
        int x = 2 * X + (d & 1), y = 2 * Y + ((d >> 1) & 1), z = 2 * Z + (d >> 2);
        s += bf2f(gf[((size_t)((z * nf + y) * nf + x)) * C + ch]);
    }
    gc[t] = f2bf(s);
}

// planar FP32 features (3 x n^3) -> channel-last BF16 input with 16 channels (13 zero)
__global__ void k_pack_input(long long nv, const float *__restrict__ f0, const float *__restrict__ f1,
                             const float *__restrict__ f2, bf16 *__restrict__ x) {
    long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    bf16 *p = x + v * 16;
    p[0] = f2bf(f0[v]);
    p[1] = f2bf(f1[v]);
    p[2] = f2bf(f2[v]);
    for (int c = 3; c < 16; ++c) p[c] = 0;
}

// prediction = channel 0 of the FP32 output (planar)
__global__ void k_unpack_output(long long nv, const float *__restrict__ y, float *__restrict__ out) {
    long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    out[v] = y[v * 16];
}

// mean-square loss on channel 0 and its gradient (BF16, channel-last, 16 channels)
__global__ void __launch_bounds__(256) k_mse(long long nv, const float *__restrict__ y, const float *__restrict__ target,
                      bf16 *__restrict__ dy, float *__restrict__ part) {
    long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (v < nv) {
        float d = y[v * 16] - target[v];
        l = d * d;
        dy[v * 16] = f2bf(2.f * d / (float)nv);
        for (int c = 1; c < 16; ++c) dy[v * 16 + c] = 0;
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_down(l, o, 64);
    __shared__ float sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l / (float)nv;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Adam on FP32 master parameters; refreshes the BF16 weight copy
__global__ void k_adam(long long n, long long nw, float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, bf16 *__restrict__ pw, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float gg = g[t];
    float mm = b1 * m[t] + (1.f - b1) * gg;
    float vv = b2 * v[t] + (1.f - b2) * gg * gg;
    m[t] = mm;
    v[t] = vv;
    float pp = p[t] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    p[t] = pp;
    if (t < nw) pw[t] = f2bf(pp);
}

__global__ void k_cast_f2bf(long long n, const float *__restrict__ a, bf16 *__restrict__ b) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = f2bf(a[t]);
}

// counter-based uniform numbers (splitmix64 of seed + index), scaled to +-a
__global__ void k_init_uniform(long long n, unsigned long long seed, float a, float *__restrict__ p) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(t + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    float u = (float)((z >> 40) * (1.0 / 16777216.0));   // [0, 1)
    p[t] = a * (2.f * u - 1.f);
}

// ------------------------------------------------------------------ dispatch
template <int CIN, int COUT>
void conv_launch(hipStream_t s, int n, const bf16 *in, const bf16 *W, const float *bias, const bf16 *skip,
                 const bf16 *mask, int relu, bf16 *out, float *out32) {
    if (n < 16 || n % 16 != 0) {
        long long nv = (long long)n * n * n;
        k_conv_small<CIN, COUT><<<(unsigned)((nv + 63) / 64), 256, 0, s>>>(n, in, W, bias, skip, mask, relu, out, out32);
        return;
    }
    // z planes per block: enough blocks to fill the chip, at most 16 planes
    const long long tiles = (long long)(n / 16) * (n / 4);
    int zc = 1;
    while (zc < 16 && tiles * (n / (2 * zc)) >= 2048 && n % (2 * zc) == 0) zc *= 2;
    dim3 g(n / 16, n / 4, n / zc);
    k_conv<CIN, COUT><<<g, 256, 0, s>>>(n, zc, in, W, bias, skip, mask, relu, out, out32);
}

// Voxels per block of the small-grid weight gradient (a multiple of 16, at most
// 512 blocks) and the number of partial copies of dW either launch writes.
inline long long wgrad_chunk(long long nv) {
    long long c = (nv + 511) / 512;
    return std::max<long long>(64, ((c + 15) / 16) * 16);
}
inline bool wgrad_small(int n) { return n < 16 || n % 16 != 0; }
inline int wgrad_parts(int n) {
    if (wgrad_small(n)) {
        const long long nv = (long long)n * n * n;
        return (int)((nv + wgrad_chunk(nv) - 1) / wgrad_chunk(nv));
    }
    const long long ntiles = (long long)(n / 16) * (n / 4) * n;
    const long long tiles = std::max<long long>(1, (ntiles + 511) / 512);
    return (int)((ntiles + tiles - 1) / tiles);
}

// dW += the weight gradient, through `part` (wgrad_parts(n) copies of dW)
template <int CIN, int COUT>
void wgrad_launch(hipStream_t s, int n, const bf16 *in, const bf16 *dy, float *part, float *dW) {
    const long long wn = (long long)COUT * 27 * CIN;
    const int parts = wgrad_parts(n);
    if (wgrad_small(n)) {
        const long long nv = (long long)n * n * n;
        const int chunk = (int)wgrad_chunk(nv);
        dim3 g((unsigned)parts, 27 * (COUT / 16) * (CIN / 16));
        k_conv_wgrad_small<CIN, COUT><<<g, 64, 0, s>>>(n, chunk, in, dy, part);
    } else {
        const long long ntiles = (long long)(n / 16) * (n / 4) * n;
        const int tiles = (int)std::max<long long>(1, (ntiles + 511) / 512);
        dim3 g(parts, (COUT / 16) * (CIN / 16));
        k_conv_wgrad<CIN, COUT><<<g, 256, 0, s>>>(n, tiles, in, dy, part);
    }
    k_sum_partials<<<(unsigned)std::min<long long>((wn + 255) / 256, 1024), 256, 0, s>>>(wn, parts, part, dW);
}

#define CONV_CASES(X)                                                                       \
    X(16, 16) X(16, 32) X(32, 16) X(32, 32) X(32, 48) X(48, 32) X(48, 48) X(48, 64) X(64, 48) X(64, 64)

bool conv_any(hipStream_t s, int cin, int cout, int n, const bf16 *in, const bf16 *W, const float *bias,
              const bf16 *skip, const bf16 *mask, int relu, bf16 *out, float *out32) {
#define X(a, b)                                                                   \
    if (cin == a && cout == b) {                                                  \
        conv_launch<a, b>(s, n, in, W, bias, skip, mask, relu, out, out32);       \
        return true;                                                              \
    }
    CONV_CASES(X)
#undef X
    return false;
}

bool wgrad_any(hipStream_t s, int cin, int cout, int n, const bf16 *in, const bf16 *dy, float *part, float *dW) {
#define X(a, b)                                        \
    if (cin == a && cout == b) {                       \
        wgrad_launch<a, b>(s, n, in, dy, part, dW);    \
        return true;                                   \
    }
    CONV_CASES(X)
#undef X
    return false;
}

inline unsigned gridfor(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ====================================================================== the network
struct stokes_unet {
    int n = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t need = 0;
    // parameters
    long long nw = 0, np = 0;            // weights, weights + biases
    long long woff[kLayers], boff[kLayers];
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // FP32 master, grad, Adam
    bf16 *wb = nullptr, *wt = nullptr;   // BF16 weights, flipped weights (backward)
    long long step = 0;
    // activations and their gradients (BF16, channel-last)
    bf16 *act[24] = {}, *grad[24] = {};
    float *y = nullptr, *loss = nullptr;
    float *part = nullptr;               // per-block partial sums of the gradients and the loss
    bf16 *dy = nullptr;
    std::string err;
};

namespace {

// activation slots
enum { X_IN, A0, S0, P1, A1, S1, P2, A2, S2, P3, A3, D3, U2, X2, D2, U1, X1, D1, U0, X0, D0, Y16, NSLOT };
struct Slot {
    int level, ch;
};
constexpr Slot kSlot[NSLOT] = {{0, 16}, {0, 16}, {0, 16}, {1, 16}, {1, 32}, {1, 32}, {2, 32}, {2, 48},
                               {2, 48}, {3, 48}, {3, 64}, {3, 64}, {2, 64}, {2, 48}, {2, 48}, {1, 48},
                               {1, 32}, {1, 32}, {0, 32}, {0, 16}, {0, 16}, {0, 16}};

size_t carve(stokes_unet &u, char *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~size_t(255);
        char *ptr = base ? base + off : nullptr;
        off += bytes;
        return ptr;
    };
    long long w = 0;
    for (int l = 0; l < kLayers; ++l) {
        u.woff[l] = w;
        w += (long long)kSpec[l].cout * 27 * kSpec[l].cin;
    }
    u.nw = w;
    for (int l = 0; l < kLayers; ++l) {
        u.boff[l] = w;
        w += kSpec[l].cout;
    }
    u.np = w;
    u.p = (float *)take(sizeof(float) * u.np);
    u.g = (float *)take(sizeof(float) * u.np);
    u.m = (float *)take(sizeof(float) * u.np);
    u.v = (float *)take(sizeof(float) * u.np);
    u.wb = (bf16 *)take(sizeof(bf16) * u.nw);
    u.wt = (bf16 *)take(sizeof(bf16) * u.nw);
    for (int s = 0; s < NSLOT; ++s) {
        long long nl = u.n >> kSlot[s].level;
        size_t bytes = sizeof(bf16) * (size_t)(nl * nl * nl) * kSlot[s].ch;
        u.act[s] = (bf16 *)take(bytes);
        u.grad[s] = (bf16 *)take(bytes);
    }
    long long nv = (long long)u.n * u.n * u.n;
    u.y = (float *)take(sizeof(float) * nv * 16);
    u.dy = (bf16 *)take(sizeof(bf16) * nv * 16);
    u.loss = (float *)take(sizeof(float) * 64);
    long long parts = std::max<long long>((long long)kBiasBlocks * 64, (nv + 255) / 256);
    for (int l = 0; l < kLayers; ++l)
        parts = std::max<long long>(parts, (long long)wgrad_parts(u.n >> kSpec[l].level) * kSpec[l].cout * 27 * kSpec[l].cin);
    u.part = (float *)take(sizeof(float) * parts);
    return off + 256;
}

struct HipErr {
    hipError_t e;
};
#define UCHK(x)                                  \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) throw HipErr{e_};  \
    } while (0)

void forward(stokes_unet &u) {
    hipStream_t s = u.stream;
    auto W = [&](int l) { return u.wb + u.woff[l]; };
    auto B = [&](int l) { return u.p + u.boff[l]; };
    auto nl = [&](int lev) { return u.n >> lev; };
    auto conv = [&](int l, int in, const bf16 *skip, int out, float *out32) {
        const LayerSpec &L = kSpec[l];
        conv_any(s, L.cin, L.cout, nl(L.level), u.act[in], W(l), B(l), skip, nullptr, L.relu,
                 out >= 0 ? u.act[out] : nullptr, out32);
    };
    auto pool = [&](int lev_c, int C, int from, int to) {
        long long tot = (long long)nl(lev_c) * nl(lev_c) * nl(lev_c) * C;
        k_pool<<<gridfor(tot), 256, 0, s>>>(nl(lev_c), C, u.act[from], u.act[to]);
    };
    auto up = [&](int lev_f, int C, int from, int to) {
        long long tot = (long long)nl(lev_f) * nl(lev_f) * nl(lev_f) * C;
        k_upsample<<<gridfor(tot), 256, 0, s>>>(nl(lev_f), C, u.act[from], u.act[to]);
    };
    conv(0, X_IN, nullptr, A0, nullptr);
    conv(1, A0, nullptr, S0, nullptr);
    pool(1, 16, S0, P1);
    conv(2, P1, nullptr, A1, nullptr);
    conv(3, A1, nullptr, S1, nullptr);
    pool(2, 32, S1, P2);
    conv(4, P2, nullptr, A2, nullptr);
    conv(5, A2, nullptr, S2, nullptr);
    pool(3, 48, S2, P3);
    conv(6, P3, nullptr, A3, nullptr);
    conv(7, A3, nullptr, D3, nullptr);
    up(2, 64, D3, U2);
    conv(8, U2, u.act[S2], X2, nullptr);
    conv(9, X2, nullptr, D2, nullptr);
    up(1, 48, D2, U1);
    conv(10, U1, u.act[S1], X1, nullptr);
    conv(11, X1, nullptr, D1, nullptr);
    up(0, 32, D1, U0);
    conv(12, U0, u.act[S0], X0, nullptr);
    conv(13, X0, nullptr, D0, nullptr);
    conv(14, D0, nullptr, -1, u.y);
}

// backward of one convolution layer l: gpre = d(pre-activation) of its output,
// input slot `in`; accumulates dW, db; writes d(input) into grad[in] masked by
// the input activation (> 0) when `mask_in`, or skips it when `need_din` is false.
void conv_backward(stokes_unet &u, int l, int in, const bf16 *gpre, bool need_din, bool mask_in) {
    hipStream_t s = u.stream;
    const LayerSpec &L = kSpec[l];
    const int n = u.n >> L.level;
    const long long nv = (long long)n * n * n;
    wgrad_any(s, L.cin, L.cout, n, u.act[in], gpre, u.part, u.g + u.woff[l]);
    int tpb = 256 - 256 % L.cout;
    k_bias_grad<<<kBiasBlocks, tpb, 0, s>>>(nv, L.cout, gpre, u.part);
    k_sum_partials<<<1, 256, 0, s>>>(L.cout, kBiasBlocks, u.part, u.g + u.boff[l]);
    if (need_din) {
        long long wn = (long long)L.cout * 27 * L.cin;
        k_flip_weights<<<gridfor(wn), 256, 0, s>>>(L.cin, L.cout, u.wb + u.woff[l], u.wt + u.woff[l]);
        conv_any(s, L.cout, L.cin, n, gpre, u.wt + u.woff[l], nullptr, nullptr, mask_in ? u.act[in] : nullptr, 0,
                 u.grad[in], nullptr);
    }
}

void backward(stokes_unet &u) {
    hipStream_t s = u.stream;
    auto nl = [&](int lev) { return u.n >> lev; };
    auto numel = [&](int slot) {
        long long m = nl(kSlot[slot].level);
        return m * m * m * kSlot[slot].ch;
    };
    auto mask = [&](int slot, const bf16 *g2) {   // grad[slot] = (grad[slot] + g2) * (act[slot] > 0)
        long long t = numel(slot);
        k_mask_grad<<<std::min<long long>(gridfor(t), 8192), 256, 0, s>>>(t, u.grad[slot], g2, u.act[slot], u.grad[slot]);
    };
    auto up_bwd = [&](int lev_c, int C, int from, int to) {
        long long tot = (long long)nl(lev_c) * nl(lev_c) * nl(lev_c) * C;
        k_upsample_bwd<<<gridfor(tot), 256, 0, s>>>(nl(lev_c), C, u.grad[from], u.grad[to]);
    };
    auto pool_bwd_add = [&](int lev_f, int C, int from, int to) {
        long long tot = (long long)nl(lev_f) * nl(lev_f) * nl(lev_f) * C;
        k_pool_bwd_add<<<gridfor(tot), 256, 0, s>>>(nl(lev_f), C, u.grad[from], u.grad[to]);
    };
    // output layer (no activation): gpre = dy; grad[D0] = d(d0) masked by d0 > 0
    conv_backward(u, 14, D0, u.dy, true, true);
    // d0 = relu(conv13(x0)): grad[D0] is already d(pre13)
    conv_backward(u, 13, X0, u.grad[D0], true, true);
    // x0 = relu(conv12(u0) + s0): grad[X0] is d(pre12); s0 receives it too
    conv_backward(u, 12, U0, u.grad[X0], true, false);
    up_bwd(1, 32, U0, D1);
    mask(D1, nullptr);
    conv_backward(u, 11, X1, u.grad[D1], true, true);
    conv_backward(u, 10, U1, u.grad[X1], true, false);
    up_bwd(2, 48, U1, D2);
    mask(D2, nullptr);
    conv_backward(u, 9, X2, u.grad[D2], true, true);
    conv_backward(u, 8, U2, u.grad[X2], true, false);
    up_bwd(3, 64, U2, D3);
    mask(D3, nullptr);
    conv_backward(u, 7, A3, u.grad[D3], true, true);
    conv_backward(u, 6, P3, u.grad[A3], true, false);
    // s2 gets the decoder skip gradient plus the pooled path
    {
        long long t = numel(S2);
        (void)hipMemcpyAsync(u.grad[S2], u.grad[X2], sizeof(bf16) * t, hipMemcpyDeviceToDevice, s);
    }
    pool_bwd_add(2, 48, P3, S2);
    mask(S2, nullptr);
    conv_backward(u, 5, A2, u.grad[S2], true, true);
    conv_backward(u, 4, P2, u.grad[A2], true, false);
    {
        long long t = numel(S1);
        (void)hipMemcpyAsync(u.grad[S1], u.grad[X1], sizeof(bf16) * t, hipMemcpyDeviceToDevice, s);
    }
    pool_bwd_add(1, 32, P2, S1);
    mask(S1, nullptr);
    conv_backward(u, 3, A1, u.grad[S1], true, true);
    conv_backward(u, 2, P1, u.grad[A1], true, false);
    {
        long long t = numel(S0);
        (void)hipMemcpyAsync(u.grad[S0], u.grad[X0], sizeof(bf16) * t, hipMemcpyDeviceToDevice, s);
    }
    pool_bwd_add(0, 16, P1, S0);
    mask(S0, nullptr);
    conv_backward(u, 1, A0, u.grad[S0], true, true);
    conv_backward(u, 0, X_IN, u.grad[A0], false, false);
}

}  // namespace

// ====================================================================== C-ABI
extern "C" {

long long stokes_unet_param_count(void) {
    stokes_unet u;
    u.n = 8;
    carve(u, nullptr);
    return u.np;
}

double stokes_unet_forward_flops(int n) {
    if (n < 8 || n % 8 != 0) return 0.0;
    double f = 0.0;
    for (int l = 0; l < kLayers; ++l) {
        const double m = (double)(n >> kSpec[l].level);
        f += 2.0 * 27.0 * kSpec[l].cin * kSpec[l].cout * m * m * m;
    }
    return f;
}

size_t stokes_unet_workspace_size(int n) {
    if (n < 8 || n % 8 != 0) return 0;
    stokes_unet u;
    u.n = n;
    return carve(u, nullptr);
}

stokes_status stokes_unet_create(int n, void *workspace, size_t ws_bytes, void *stream, stokes_unet **out) {
    if (!out) return STOKES_EINVAL;
    *out = nullptr;
    if (n < 8 || n % 8 != 0 || !workspace) return STOKES_EINVAL;
    stokes_unet *u = new stokes_unet();
    u->n = n;
    u->stream = reinterpret_cast<hipStream_t>(stream);
    u->need = carve(*u, nullptr);
    if (ws_bytes < u->need) {
        delete u;
        return STOKES_ENOMEM;
    }
    u->ws = reinterpret_cast<char *>(workspace);
    carve(*u, u->ws);
    if (hipMemsetAsync(u->ws, 0, u->need, u->stream) != hipSuccess) {
        delete u;
        return STOKES_EHIP;
    }
    *out = u;
    return STOKES_OK;
}

// He-uniform initialisation from a counter-based generator (splitmix64), zero biases
stokes_status stokes_unet_init(stokes_unet *u, unsigned long long seed) {
    if (!u) return STOKES_EINVAL;
    try {
        for (int l = 0; l < kLayers; ++l) {
            long long cnt = (long long)kSpec[l].cout * 27 * kSpec[l].cin;
            float fan_in = 27.f * (l == 0 ? 3.f : (float)kSpec[l].cin);
            float a = std::sqrt(6.f / fan_in) * (l == kLayers - 1 ? 0.1f : 1.f);
            k_init_uniform<<<gridfor(cnt), 256, 0, u->stream>>>(cnt, seed + 1000003ull * l, a, u->p + u->woff[l]);
        }
        UCHK(hipMemsetAsync(u->p + u->nw, 0, sizeof(float) * (u->np - u->nw), u->stream));
        UCHK(hipMemsetAsync(u->m, 0, sizeof(float) * u->np, u->stream));
        UCHK(hipMemsetAsync(u->v, 0, sizeof(float) * u->np, u->stream));
        k_cast_f2bf<<<gridfor(u->nw), 256, 0, u->stream>>>(u->nw, u->p, u->wb);
        UCHK(hipStreamSynchronize(u->stream));
        u->step = 0;
    } catch (const HipErr &) {
        return STOKES_EHIP;
    }
    return STOKES_OK;
}

// Parameters as FP32 (host <-> device copies of the master weights and biases)
stokes_status stokes_unet_get_params(stokes_unet *u, float *host, long long count) {
    if (!u || !host || count != u->np) return STOKES_EINVAL;
    if (hipMemcpyAsync(host, u->p, sizeof(float) * count, hipMemcpyDeviceToHost, u->stream) != hipSuccess) return STOKES_EHIP;
    return hipStreamSynchronize(u->stream) == hipSuccess ? STOKES_OK : STOKES_EHIP;
}

stokes_status stokes_unet_set_params(stokes_unet *u, const float *host, long long count) {
    if (!u || !host || count != u->np) return STOKES_EINVAL;
    if (hipMemcpyAsync(u->p, host, sizeof(float) * count, hipMemcpyHostToDevice, u->stream) != hipSuccess) return STOKES_EHIP;
    k_cast_f2bf<<<gridfor(u->nw), 256, 0, u->stream>>>(u->nw, u->p, u->wb);
    return hipStreamSynchronize(u->stream) == hipSuccess ? STOKES_OK : STOKES_EHIP;
}

// prediction = net(features) on n^3: f0, f1, f2 and out are planar FP32 device arrays
stokes_status stokes_unet_forward(stokes_unet *u, const float *f0, const float *f1, const float *f2, float *out) {
    if (!u || !f0 || !f1 || !f2 || !out) return STOKES_EINVAL;
    long long nv = (long long)u->n * u->n * u->n;
    k_pack_input<<<gridfor(nv), 256, 0, u->stream>>>(nv, f0, f1, f2, u->act[X_IN]);
    forward(*u);
    k_unpack_output<<<gridfor(nv), 256, 0, u->stream>>>(nv, u->y, out);
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EHIP;
}

// one Adam step on the mean-square error between the prediction and `target`;
// *loss_out (host) receives the loss before the step.  Blocks until done.
stokes_status stokes_unet_train_step(stokes_unet *u, const float *f0, const float *f1, const float *f2,
                                     const float *target, float lr, float *loss_out) {
    if (!u || !f0 || !f1 || !f2 || !target) return STOKES_EINVAL;
    try {
        long long nv = (long long)u->n * u->n * u->n;
        hipStream_t s = u->stream;
        k_pack_input<<<gridfor(nv), 256, 0, s>>>(nv, f0, f1, f2, u->act[X_IN]);
        forward(*u);
        UCHK(hipMemsetAsync(u->loss, 0, sizeof(float), s));
        k_mse<<<gridfor(nv), 256, 0, s>>>(nv, u->y, target, u->dy, u->part);
        k_sum_partials<<<1, 256, 0, s>>>(1, (int)gridfor(nv), u->part, u->loss);
        UCHK(hipMemsetAsync(u->g, 0, sizeof(float) * u->np, s));
        backward(*u);
        u->step++;
        const float b1 = 0.9f, b2 = 0.999f;
        float c1 = 1.f - std::pow(b1, (float)u->step), c2 = 1.f - std::pow(b2, (float)u->step);
        k_adam<<<gridfor(u->np), 256, 0, s>>>(u->np, u->nw, u->p, u->g, u->m, u->v, u->wb, lr, b1, b2, 1e-8f, c1, c2);
        float l = 0.f;
        UCHK(hipMemcpyAsync(&l, u->loss, sizeof(float), hipMemcpyDeviceToHost, s));
        UCHK(hipStreamSynchronize(s));
        UCHK(hipGetLastError());
        if (loss_out) *loss_out = l;
    } catch (const HipErr &) {
        return STOKES_EHIP;
    }
    return STOKES_OK;
}

// Gradient of the last train step's loss (FP32, count = param count), for tests.
stokes_status stokes_unet_get_grads(stokes_unet *u, float *host, long long count) {
    if (!u || !host || count != u->np) return STOKES_EINVAL;
    if (hipMemcpyAsync(host, u->g, sizeof(float) * count, hipMemcpyDeviceToHost, u->stream) != hipSuccess) return STOKES_EHIP;
    return hipStreamSynchronize(u->stream) == hipSuccess ? STOKES_OK : STOKES_EHIP;
}

int stokes_unet_size(const stokes_unet *u) { return u ? u->n : 0; }

// library-internal: the stream a network launches on (not part of the public header)
void *stokes_unet_stream_internal(const stokes_unet *u) { return u ? reinterpret_cast<void *>(u->stream) : nullptr; }

void stokes_unet_destroy(stokes_unet *u) { delete u; }

}  // extern "C"
